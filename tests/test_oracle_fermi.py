"""Pins for the oracle's Fermi-like distribution and steric potential
(Sec. 2, Eq. (1)), CPU only."""
import math

import numpy as np
import pytest
from scipy.optimize import brentq
from scipy.special import logsumexp

import oracle
from paper_1711_04060_amd import inputs

MS = inputs.MEMBRANE_SPECIES


def _sp(steric=True):
    return oracle.species_from_molar(MS["valence"], MS["radius_A"], MS["bath_M"], steric=steric)


def test_table1_constants_give_lambda_and_bulk_void():
    """lambda = e^2/(eps0 kB T) from Table 1 is ~7048 A (Bjerrum length
    lambda/(4 pi eps_s) ~ 7.15 A in water); the membrane bath leaves a bulk
    void fraction Gamma_B ~ 0.614."""
    sp = _sp()
    assert sp.lam == pytest.approx(7048.03, abs=0.01)
    assert sp.lam / (4 * math.pi * 78.45) == pytest.approx(7.149, abs=1e-3)
    assert 1 - (sp.volume * sp.conc).sum() == pytest.approx(0.6141, abs=1e-4)


def test_zero_potential_gives_bath():
    """phi = 0 gives Gamma = Gamma_B, S = 0 and C = C_B (text after Eq. (1))."""
    sp = _sp()
    rho, sig, conc, S = oracle.fermi(np.zeros(5), sp)
    np.testing.assert_allclose(conc, np.repeat(sp.conc[:, None], 5, 1), rtol=2e-15)
    assert np.all(np.abs(S) <= 1e-15)
    # neutral bath: Cl = Na + 2 Ca, so rho_hat vanishes
    assert np.all(np.abs(rho) <= 1e-12 * sig)


def test_steric_off_is_boltzmann():
    sp = _sp(steric=False)
    phi = np.linspace(-30, 30, 61)
    rho, sig, conc, S = oracle.fermi(phi, sp)
    ref = sp.conc[:, None] * np.exp(-np.asarray(sp.valence)[:, None] * phi[None, :])
    np.testing.assert_allclose(conc, ref, rtol=1e-13)
    assert np.all(S == 0)


def test_sigma_is_minus_drho_dphi_without_sterics():
    """rho' of Eq. (11) is -sigma; without the steric term it is the exact
    derivative of rho_hat (central difference check)."""
    sp = _sp(steric=False)
    phi = np.linspace(-5, 5, 21)
    d = 1e-5
    rp = oracle.fermi(phi + d, sp)[0]
    rm = oracle.fermi(phi - d, sp)[0]
    sig = oracle.fermi(phi, sp)[1]
    np.testing.assert_allclose(-(rp - rm) / (2 * d), sig, rtol=1e-7)


def test_saturation_and_void_identity():
    """v_i C_i < 1 for every species and any phi (the saturation property
    after Eq. (1)), Gamma in (0, 1), and the void identity
    Gamma_B e^S + sum_i v_i C_i = 1 that defines S.  At |phi| of order 10^3
    the void fraction is below the smallest double and the exponent
    ln(v_i C_i) is a difference of terms of size |z_i phi|, so there the bound
    holds to that rounding (v_i C_i <= 1 + 8 eps |z_i phi|) and ln Gamma stays
    finite."""
    sp = _sp()
    phi = np.concatenate([np.linspace(-2000, 2000, 401), [-1e4, 1e4]])
    rho, sig, conc, S = oracle.fermi(phi, sp)
    occ = sp.volume[:, None] * conc
    slack = 8 * np.finfo(float).eps * (1 + np.abs(np.asarray(sp.valence))[:, None] * np.abs(phi))
    assert np.all(occ <= 1.0 + slack) and np.all(np.isfinite(S))
    moderate = np.abs(phi) <= 20
    assert np.all(occ[:, moderate] < 1.0)
    GB = 1 - (sp.volume * sp.conc).sum()
    ln_gamma = np.log(GB) + S
    assert np.all(ln_gamma < 0)
    assert np.all(np.exp(ln_gamma[moderate]) > 0)
    resid = np.abs(np.exp(ln_gamma) + occ.sum(0) - 1.0)
    assert np.all(resid <= 8 * np.finfo(float).eps * (1 + 2 * np.abs(phi)))


def test_charge_density_decreases_with_potential():
    """The ionic charge density rho_hat falls as phi rises and the anion rises.
    With Ca2+ present, Na+ itself is not monotone: at strongly negative phi the
    divalent ion fills the space and crowds Na+ out (a steric effect the
    Boltzmann limit lacks), so monotonicity of a single cation is checked on a
    NaCl-only bath."""
    sp = _sp()
    phi = np.linspace(-15, 15, 601)
    rho, _, conc, _ = oracle.fermi(phi, sp)
    assert np.all(np.diff(rho) < 0)
    assert np.all(np.diff(conc[2]) > 0)
    far = oracle.fermi(np.linspace(-50, -15, 101), sp)
    assert np.all(np.diff(far[0]) <= 1e-12 * np.abs(far[0][1:]))
    assert np.any(np.diff(far[2][0]) > 0)        # Na+ crowded out by Ca2+
    nacl = oracle.species_from_molar((1.0, -1.0, 0.0), (0.95, 1.81, 1.4), (0.1, 0.1, 55.5))
    c = oracle.fermi(np.linspace(-8, 8, 161), nacl)[2]
    assert np.all(np.diff(c[0]) < 0) and np.all(np.diff(c[1]) > 0)


def test_root_matches_library_brent():
    """The bisection root agrees with scipy's Brent method on the same
    void-fraction equation written in the log domain."""
    sp = _sp()
    v, cb, z = sp.volume, sp.conc, np.asarray(sp.valence)
    v0 = v.mean()
    GB = 1 - (v * cb).sum()

    def L(S, phi):
        return logsumexp(np.concatenate([[math.log(GB) + S], np.log(v * cb) - z * phi + v / v0 * S]))

    for phi in (-800.0, -40.0, -3.0, -0.2, 0.0, 0.7, 5.0, 60.0, 1500.0):
        hi = -math.log(GB)
        lo = hi - 1.0
        while L(lo, phi) >= 0:
            lo = hi - 2 * (hi - lo)
        ref = brentq(L, lo, hi, xtol=1e-15, rtol=4 * np.finfo(float).eps, maxiter=500, args=(phi,))
        got = oracle.steric_root(phi, sp)
        assert got == pytest.approx(ref, rel=1e-13, abs=1e-14)


def test_non_solvent_nodes_are_empty():
    sp = _sp()
    typ = np.array([0, 1, 2, 0], np.uint8)
    rho, sig, conc, S = oracle.fermi(np.array([1.0, 1.0, 1.0, -2.0]), sp, node_type=typ)
    assert rho[1] == rho[2] == sig[1] == sig[2] == 0
    assert np.all(conc[:, 1:3] == 0)
    assert sig[0] > 0 and sig[3] > 0


def test_pb_limit_of_fermi():
    """Vanishing ion and water volumes remove the steric term: the steric
    result tends to the Boltzmann one (the PF -> PB reduction)."""
    phi = np.linspace(-8, 8, 33)
    ref = oracle.fermi(phi, _sp(steric=False))[2]
    sp = oracle.species_from_molar(MS["valence"], np.array(MS["radius_A"]) * 1e-3, MS["bath_M"])
    got = oracle.fermi(phi, sp)[2]
    np.testing.assert_allclose(got, ref, rtol=1e-6)
