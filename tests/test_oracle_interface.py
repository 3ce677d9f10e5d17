"""Pins of the oracle's interface treatment (Sec. 3): the singular-charge
decomposition of Eq. (5), the Laplace problem of Eqs. (9)-(10), the flux jump
of Eq. (8) and the SMIB right-hand-side terms of Eqs. (17)-(18).

Each check compares with something the oracle does not compute itself:
finite differences and Gauss's law for phi*, the exact piecewise-linear
solution of a layered 1D problem, the method of images for a uniform
dielectric, and the Born solution of a charged dielectric sphere."""
import numpy as np
import pytest

import oracle

PI = np.pi


def _charges(rng, m, lo, hi):
    pos = rng.uniform(lo, hi, size=(m, 3))
    q = rng.uniform(-1.0, 1.0, size=m)
    return np.column_stack([pos, q])


def test_coulomb_derivatives_match_central_differences():
    rng = np.random.default_rng(11)
    ch = _charges(rng, 7, -0.5, 0.5)
    pts = rng.uniform(1.0, 1.5, size=(20, 3)) * rng.choice([-1.0, 1.0], size=(20, 3))
    d = 1e-5
    for f in range(6):
        unit = np.zeros(3)
        unit[f // 2] = 1.0 if f % 2 else -1.0
        fd = (oracle.coulomb(pts + d * unit, ch, 0.7) - oracle.coulomb(pts - d * unit, ch, 0.7)) / (2 * d)
        an = oracle.coulomb(pts, ch, 0.7, dirs=np.full(len(pts), f))
        np.testing.assert_allclose(an, fd, rtol=1e-7, atol=1e-9)
    # dirs == 6 is the potential itself
    np.testing.assert_array_equal(oracle.coulomb(pts, ch, 0.7, dirs=np.full(len(pts), 6)),
                                  oracle.coulomb(pts, ch, 0.7))


def test_coulomb_gauss_law_on_a_cube():
    """The outward flux of grad(phi*) through the unit cube is
    -4 pi scale (sum of the charges inside); charges outside add nothing."""
    rng = np.random.default_rng(3)
    inner = _charges(rng, 5, 0.3, 0.7)
    outer = _charges(rng, 4, 1.3, 1.6)
    ch = np.vstack([inner, outer])
    scale = 1.0 / (4 * PI * 2.0)
    x, w = np.polynomial.legendre.leggauss(64)
    x, w = 0.5 * (x + 1.0), 0.5 * w
    U, V = np.meshgrid(x, x, indexing="ij")
    W = np.outer(w, w).ravel()
    flux = 0.0
    for f in range(6):
        ax, side = f // 2, f % 2
        pts = np.zeros((U.size, 3))
        others = [a for a in range(3) if a != ax]
        pts[:, others[0]] = U.ravel()
        pts[:, others[1]] = V.ravel()
        pts[:, ax] = float(side)
        flux += np.dot(W, oracle.coulomb(pts, ch, scale, dirs=np.full(U.size, f)))
    assert flux == pytest.approx(-4 * PI * scale * inner[:, 3].sum(), rel=1e-9, abs=1e-12)


@pytest.mark.parametrize("m_below", [True, False])
@pytest.mark.parametrize("eps_m,eps_s", [(2.0, 80.0), (78.45, 2.0), (3.0, 3.0)])
def test_smib_terms_give_exact_layered_solution(m_below, eps_m, eps_s):
    """Two layers along z, interface midway between node planes K0-1 and K0,
    Dirichlet a and b on the z faces, a prescribed flux jump J on every edge
    across the interface and no source: the exact solution is linear on each
    side (continuous, eps_s phi'_s - eps_m phi'_m = J along the normal that
    points out of Omega_m), and the FD solution reproduces it at the nodes."""
    nx = ny = 3
    nz, K0 = 21, 8
    h = 1.0 / (nz - 1)
    L = (nz - 1) * h
    xi = (K0 - 0.5) * h
    a, b, J = 0.7, -1.3, 2.5
    k = np.repeat(np.arange(nz), nx * ny)
    lower = k < K0
    solute = lower if m_below else ~lower
    typ = np.where(solute, oracle.SOLUTE, oracle.SOLVENT).astype(np.uint8)
    eps = np.where(solute, eps_m, eps_s)
    e_lo, e_hi = (eps_m, eps_s) if m_below else (eps_s, eps_m)
    # phi = a + g_lo z below xi, b - g_hi (L - z) above.  Continuity, and the
    # jump along the normal out of Omega_m: +z when Omega_m is below,
    # eps_s g_hi - eps_m g_lo = J; -z when it is above,
    # eps_s (-g_lo) - eps_m (-g_hi) = J.  Both read e_hi g_hi - e_lo g_lo = J.
    A = np.array([[xi, L - xi], [-e_lo, e_hi]])
    g_lo, g_hi = np.linalg.solve(A, [b - a, J])
    z = k * h
    exact = np.where(z < xi, a + g_lo * z, b - g_hi * (L - z))
    g = oracle.Grid(nx, ny, nz, h, eps, typ,
                    bc_phi=(oracle.NEUMANN,) * 4 + (oracle.DIRICHLET,) * 2, bc_value=(0, 0, 0, 0, a, b))
    N = nx * ny * nz
    jump = np.zeros((6, N))
    d = 5 if m_below else 4
    plane = K0 - 1 if m_below else K0
    jump[d, k == plane] = J
    rhs = oracle.smib_rhs(g, eps_m, eps_s, jump)
    x, info = oracle.linear_solve(g, None, rhs, tol=1e-14)
    np.testing.assert_allclose(x, exact, rtol=0, atol=1e-10)


def _images_problem(n, eps=2.0, lam=1.0):
    """Uniform dielectric in the unit cube; Omega_m = the block i <= n/2,
    k <= n/2 (touching the x = 0 and z = 0 faces); x = 0 Neumann, z = 0
    Dirichlet 0, the other faces FIXED.  Mirror charges across x = 0 (same
    sign) and z = 0 (opposite sign) make the Coulomb sum of charges plus
    images the exact potential; the decomposition is given the real charges
    only."""
    h = 1.0 / (n - 1)
    k, j, i = [a.ravel() for a in np.meshgrid(np.arange(n), np.arange(n), np.arange(n), indexing="ij")]
    half = (n - 1) // 2
    inside = (i <= half) & (k <= half) & (j >= 1) & (j <= n - 2)
    fixed = (i == n - 1) | (j == 0) | (j == n - 1) | (k == n - 1)
    typ = np.where(fixed, oracle.FIXED, np.where(inside, oracle.SOLUTE, oracle.SOLVENT)).astype(np.uint8)
    rng = np.random.default_rng(5)
    m = 6
    pos = np.stack([rng.uniform(0.1, 0.4, m), rng.uniform(0.25, 0.75, m), rng.uniform(0.1, 0.4, m)], 1)
    real = np.column_stack([pos, np.where(np.arange(m) % 2 == 0, 1.0, -1.0)])
    images = [real]
    for sx, sz, sq in ((-1, 1, 1), (1, -1, -1), (-1, -1, -1)):
        c = real.copy()
        c[:, 0] *= sx
        c[:, 2] *= sz
        c[:, 3] *= sq
        images.append(c)
    pts = np.column_stack([i * h, j * h, k * h])
    exact = oracle.coulomb(pts, np.vstack(images), lam / (4 * PI * eps))
    g = oracle.Grid(n, n, n, h, np.full(n ** 3, eps), typ, np.where(fixed, exact, 0.0),
                    bc_phi=(oracle.NEUMANN,) + (oracle.DIRICHLET,) * 5)
    near = np.min(np.linalg.norm(pts[:, None, :] - pos[None, :, :], axis=2), axis=1) <= 2.5 * h
    return g, real, exact, near


def test_decomposition_reproduces_image_solution():
    """Uniform dielectric: the total potential phi-tilde + phi* + phi^L must
    converge to the exact image solution; the Omega_m block meets a Dirichlet
    and a Neumann face, so both face rules of the Laplace problem count."""
    errs = []
    for n in (17, 33):
        g, real, exact, near = _images_problem(n)
        b_if, reg, lap, info = oracle.interface(g, real, 1.0, 2.0, 2.0)
        x, _ = oracle.linear_solve(g, None, b_if)
        tot = x + reg
        errs.append(np.abs(tot - exact)[~near].max() / np.abs(exact[~near]).max())
    assert errs[0] < 0.03 and errs[1] < 0.015
    assert errs[1] < 0.6 * errs[0]


def _born(n, R_cells, eps_m=2.0, eps_s=80.0):
    c = (n - 1) / 2.0
    k, j, i = [a.ravel() for a in np.meshgrid(np.arange(n), np.arange(n), np.arange(n), indexing="ij")]
    r = np.sqrt((i - c) ** 2 + (j - c) ** 2 + (k - c) ** 2)
    inside = r < R_cells
    face = (i == 0) | (i == n - 1) | (j == 0) | (j == n - 1) | (k == 0) | (k == n - 1)
    typ = np.where(inside, oracle.SOLUTE, np.where(face, oracle.FIXED, oracle.SOLVENT)).astype(np.uint8)
    out_exact = 1.0 / (4 * PI * eps_s * r)
    in_exact = 1.0 / (4 * PI * eps_m * r) + (1.0 / eps_s - 1.0 / eps_m) / (4 * PI * R_cells)
    g = oracle.Grid(n, n, n, 1.0, np.where(inside, eps_m, eps_s), typ, np.where(face, out_exact, 0.0))
    return g, np.array([[c, c, c, 1.0]]), r, inside, face, out_exact, in_exact


def test_decomposition_born_sphere():
    """Unit charge at the centre of a sphere (eps_m = 2) in eps_s = 80, exact
    exterior values on the box faces: inside, the total potential is
    1/(4 pi eps_m r) + (1/eps_s - 1/eps_m)/(4 pi R); outside, 1/(4 pi eps_s r).
    The staircase sphere limits the accuracy next to the interface."""
    g, ch, r, inside, face, out_exact, in_exact = _born(24, 6)
    b_if, reg, lap, info = oracle.interface(g, ch, 1.0, 2.0, 80.0)
    x, _ = oracle.linear_solve(g, None, b_if)
    tot = x + reg
    deep = inside & (r < 4)
    far = ~inside & ~face & (r > 9)
    e_in = np.abs(tot - in_exact)[deep].max() / np.abs(in_exact[inside]).max()
    e_far = np.abs(tot - out_exact)[far].max() / out_exact[far].max()
    e_out = np.abs(tot - out_exact)[~inside & ~face].max() / out_exact[~inside].max()
    assert e_in < 0.004
    assert e_far < 0.01
    assert e_out < 0.07
    # phi_reg is phi* + phi^L on Omega_m and zero elsewhere
    assert np.all(reg[~inside] == 0.0)


def test_interface_argument_checks_and_empty_charge_set():
    g, ch, r, inside, face, _, _ = _born(16, 4)
    with pytest.raises(oracle.OracleError):
        oracle.interface(g, ch, 1.0, 3.0, 80.0)       # eps on Omega_m is 2, not 3
    b_if, reg, lap, info = oracle.interface(g, np.zeros((0, 4)), 1.0, 2.0, 80.0)
    assert not b_if.any() and not reg.any() and not lap.any()
