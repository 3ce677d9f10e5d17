"""Pins of the oracle's filter-region atomic model (Sec. 2, Eqs. (19)-(20))
and of the filter-region fill that turns its values into Dirichlet data of
the continuum model.

phi_b is checked against closed forms of the six-point surface average (an
atom or an occupied site on an axis of the site), the self term of an
occupied site, and the mean-value property of harmonic functions (the
six-point average of 1/r approaches 1/d as (a/d)^4); S_b against the void
fraction of Eq. (20); the fill against a brute-force numpy scan."""
import numpy as np
import pytest

import oracle
from paper_1711_04060_amd import inputs

PI = np.pi
MS = inputs.MEMBRANE_SPECIES


def _sp(steric=True):
    return oracle.species_from_molar(MS["valence"], MS["radius_A"], MS["bath_M"], steric=steric)


def _sites(xyz, radius, valence, occupied, atoms=None, eps_p=20.0, eps_b=10.0, V=1000.0):
    return dict(xyz=np.asarray(xyz, float), radius=np.asarray(radius, float), valence=np.asarray(valence, float),
                occupied=np.asarray(occupied, np.int32),
                atoms=np.zeros((0, 4)) if atoms is None else np.asarray(atoms, float),
                eps_p=eps_p, eps_b=eps_b, V_sites=V)


def _six_point_axis(d, a):
    """Mean of 1/|d e - A_k| over the six points +-a along each axis (e an axis)."""
    return (1.0 / (d - a) + 1.0 / (d + a) + 4.0 / np.sqrt(d * d + a * a)) / 6.0


def test_lone_occupied_site_is_its_self_term():
    sp = _sp()
    s = _sites([[1.0, 2.0, 3.0]], [0.99], [2.0], [1])
    phi, S, psi, conc = oracle.site_model(s, sp)
    assert phi[0] == pytest.approx(sp.lam / (4 * PI) * 2.0 / (10.0 * 0.99), rel=1e-14)


@pytest.mark.parametrize("axis", [0, 1, 2])
def test_atom_on_an_axis_gives_the_six_point_closed_form(axis):
    sp = _sp()
    c = np.array([0.5, -0.25, 2.0])
    d, a, z = 3.7, 0.95, -0.6
    atom = c.copy()
    atom[axis] += d
    s = _sites([c], [a], [1.0], [0], atoms=[[*atom, z]])
    phi, _, _, _ = oracle.site_model(s, sp)
    assert phi[0] == pytest.approx(sp.lam / (4 * PI) * z / 20.0 * _six_point_axis(d, a), rel=1e-13)


def test_other_occupied_site_enters_with_eps_b_and_empty_ones_do_not():
    sp = _sp()
    D, a = 2.5, 0.95
    s = _sites([[0, 0, 0], [0, 0, D], [0, D, 0]], [a, 0.99, 0.99], [1.0, 2.0, 2.0], [0, 1, 0])
    phi, _, _, _ = oracle.site_model(s, sp)
    assert phi[0] == pytest.approx(sp.lam / (4 * PI) * 2.0 / 10.0 * _six_point_axis(D, a), rel=1e-13)


def test_six_point_average_approaches_the_centre_value():
    """1/r is harmonic, so its six-point average over an octahedron of radius a
    around the centre differs from the centre value by O((a/d)^4)."""
    sp = _sp()
    rng = np.random.default_rng(9)
    dirs = rng.normal(size=(5, 3))
    dirs /= np.linalg.norm(dirs, axis=1)[:, None]
    for d in (5.0, 10.0, 20.0):
        atoms = np.column_stack([d * dirs, np.ones(5)])
        s = _sites([[0, 0, 0]], [1.0], [1.0], [0], atoms=atoms)
        phi, _, _, _ = oracle.site_model(s, sp)
        centre = sp.lam / (4 * PI) / 20.0 * 5 / d
        assert abs(phi[0] / centre - 1.0) <= 0.5 / d ** 4


def test_steric_term_is_the_void_fraction_of_the_pocket():
    sp = _sp()
    GB = oracle.bulk_void(sp)
    # bulk void fraction from the bath concentrations, independently
    v = 4 * PI * np.asarray(MS["radius_A"]) ** 3 / 3
    c = np.asarray(MS["bath_M"]) * 6.02214076e23 * 1e3 * 1e-30
    assert GB == pytest.approx(1.0 - (v * c).sum(), rel=1e-14)
    r = [0.95, 0.99, 0.95]
    V = 40.0
    for occ in ([0, 0, 0], [1, 0, 0], [1, 1, 1]):
        s = _sites([[0, 0, 0], [0, 0, 3], [0, 0, 6]], r, [1, 2, 1], occ, V=V)
        phi, S, psi, conc = oracle.site_model(s, sp)
        filled = sum(4 * PI * ri ** 3 / 3 for ri, o in zip(r, occ) if o)
        assert np.allclose(S, np.log((1 - filled / V) / GB), rtol=0, atol=1e-14)
        assert np.allclose(psi, phi - S / np.array([1, 2, 1]), rtol=0, atol=1e-14)
        # Eq. (1) at the site with the given potential and steric value
        p = v / v.mean()
        want = c[None, :] * np.exp(-np.asarray(MS["valence"])[None, :] * phi[:, None] + p[None, :] * S[:, None])
        np.testing.assert_allclose(conc, want, rtol=1e-13)
    # steric off: S = 0; a pocket filled beyond its volume is rejected
    s = _sites([[0, 0, 0]], [0.99], [2.0], [1], V=1.0)
    _, S, _, _ = oracle.site_model(s, _sp(steric=False))
    assert S[0] == 0.0
    with pytest.raises(oracle.OracleError):
        oracle.site_model(s, sp)


def test_fill_matches_brute_force():
    n, h = 21, 0.4
    rng = np.random.default_rng(4)
    typ = rng.choice([oracle.SOLVENT, oracle.SOLUTE], size=n ** 3, p=[0.8, 0.2]).astype(np.uint8)
    xyz = rng.uniform(1.0, (n - 1) * h - 1.0, size=(6, 3))
    xyz[1] = xyz[0] + [0.5, 0.0, 0.0]               # overlapping spheres: nearest centre wins
    rad = rng.uniform(0.6, 1.2, size=6)
    phi = rng.normal(size=6)
    s = _sites(xyz, rad, np.ones(6), np.zeros(6, np.int32))
    t2, fv, marked = oracle.site_fill(n, n, n, h, s, phi, typ)
    k, j, i = [a.ravel() for a in np.meshgrid(np.arange(n), np.arange(n), np.arange(n), indexing="ij")]
    pts = np.column_stack([i, j, k]) * h
    d2 = ((pts[:, None, :] - xyz[None, :, :]) ** 2).sum(axis=2)
    inside = d2 <= rad[None, :] ** 2
    d2m = np.where(inside, d2, np.inf)
    best = np.argmin(d2m, axis=1)
    hit = inside.any(axis=1) & (typ == oracle.SOLVENT)
    want_t = np.where(hit, oracle.FIXED, typ)
    np.testing.assert_array_equal(t2, want_t)
    np.testing.assert_array_equal(fv[hit], phi[best[hit]])
    assert np.all(fv[~hit] == 0.0)
    assert marked == hit.sum() and marked > 0
