"""Pins for the oracle's 7-point operator and its Jacobi-BiCGSTAB (CPU only).

Each test checks the oracle against something other than itself: closed-form
eigenpairs of the discrete Laplacian, an exact continuum solution that the
harmonic-mean faces reproduce node for node, the discrete Debye-Hueckel
solution, second-order convergence to a manufactured solution, and a dense
LAPACK solve of the same matrix.
"""
import math

import numpy as np
import pytest

import oracle
from oracle import DIRICHLET as D, NEUMANN as NM


def _grid(nx, ny, nz, h, eps, bc=(D,) * 6, bcv=(0.0,) * 6, node_type=None, fixed_value=None):
    return oracle.Grid(nx, ny, nz, h, np.broadcast_to(eps, (nx * ny * nz,)).astype(float).copy(),
                       node_type, fixed_value, tuple(bc), tuple(bcv))


def _ijk(nx, ny, nz):
    k, j, i = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    return i.ravel(), j.ravel(), k.ravel()


def _dense(nx, ny, nz, A):
    """Dense matrix from the seven diagonals (column offsets per the paper's
    A0..A6 convention)."""
    N = nx * ny * nz
    M = np.zeros((N, N))
    i, j, k = _ijk(nx, ny, nz)
    n = np.arange(N)
    M[n, n] = A[0]
    for d, off, ok in ((1, 1, i < nx - 1), (2, -1, i > 0), (3, -nx, j > 0), (4, nx, j < ny - 1),
                       (5, -nx * ny, k > 0), (6, nx * ny, k < nz - 1)):
        M[n[ok], n[ok] + off] = A[d][ok]
    return M


def _apply(g, sigma=None):
    isd, val = oracle.dirichlet(g)
    A = oracle.assemble(g.nx, g.ny, g.nz, g.h, g.eps, sigma, isd, g.bc_phi)
    return A, isd, val


# ------------------------------------------------------------- eigenpairs

@pytest.mark.parametrize("neumann_axes", [(), (0,), (1,), (2,), (0, 1)])
@pytest.mark.parametrize("modes", [(1, 1, 1), (2, 3, 1), (3, 1, 4)])
def test_laplacian_eigenpairs(neumann_axes, modes):
    """Constant eps: sin modes (Dirichlet axes) and cos modes (Neumann axes,
    node-centred mirror ghost) are exact eigenvectors with eigenvalue
    (4 eps / h^2) sum_d sin^2(m_d pi / (2 (n_d - 1)))."""
    nx, ny, nz, h, eps = 7, 9, 11, 0.3, 3.7
    bc = [D] * 6
    for a in neumann_axes:
        bc[2 * a] = bc[2 * a + 1] = NM
    g = _grid(nx, ny, nz, h, eps, bc)
    A, isd, _ = _apply(g)
    i, j, k = _ijk(nx, ny, nz)
    u = np.ones(nx * ny * nz)
    lam = 0.0
    for a, (idx, n, m) in enumerate(zip((i, j, k), (nx, ny, nz), modes)):
        arg = m * math.pi * idx / (n - 1)
        u *= np.cos(arg) if a in neumann_axes else np.sin(arg)
        lam += math.sin(m * math.pi / (2 * (n - 1))) ** 2
    lam *= 4.0 * eps / h ** 2
    Au = oracle.dia_matvec(nx, ny, nz, A, u)
    free = isd == 0
    np.testing.assert_allclose(Au[free], lam * u[free], rtol=0, atol=1e-12 * lam)
    np.testing.assert_allclose(Au[~free], u[~free], atol=1e-15)   # identity rows


def test_symmetric_with_dirichlet_only():
    """Dirichlet-only boundaries and harmonic faces give a symmetric matrix on
    the free unknowns (the symmetric case named before Table 2)."""
    rng = np.random.default_rng(0)
    nx, ny, nz = 6, 7, 8
    N = nx * ny * nz
    eps = np.exp(rng.uniform(0, math.log(80), N))
    typ = np.zeros(N, np.uint8)
    typ[rng.choice(N, 10, replace=False)] = oracle.FIXED
    g = _grid(nx, ny, nz, 0.7, eps, node_type=typ, fixed_value=rng.normal(size=N))
    A, isd, _ = _apply(g, sigma=rng.uniform(0, 3, N))
    x, y = rng.normal(size=N), rng.normal(size=N)
    x[isd == 1] = 0
    y[isd == 1] = 0
    a = x @ oracle.dia_matvec(nx, ny, nz, A, y)
    b = y @ oracle.dia_matvec(nx, ny, nz, A, x)
    assert abs(a - b) <= 1e-12 * abs(a)
    M = _dense(nx, ny, nz, A)
    f = np.flatnonzero(isd == 0)
    Mff = M[np.ix_(f, f)]
    np.testing.assert_allclose(Mff, Mff.T, rtol=0, atol=1e-13 * np.abs(Mff).max())


def test_dia_matvec_matches_dense():
    rng = np.random.default_rng(1)
    nx, ny, nz = 5, 6, 7
    N = nx * ny * nz
    g = _grid(nx, ny, nz, 0.4, rng.uniform(1, 5, N), bc=(NM, D, NM, NM, D, NM))
    A, _, _ = _apply(g, sigma=rng.uniform(0, 1, N))
    x = rng.normal(size=N)
    np.testing.assert_allclose(oracle.dia_matvec(nx, ny, nz, A, x), _dense(nx, ny, nz, A) @ x,
                               rtol=1e-14, atol=1e-12)


# -------------------------------------------------- exact discrete solutions

@pytest.mark.parametrize("eps1,eps2,K0", [(2.0, 80.0, 8), (78.45, 2.0, 5), (1.0, 1.0, 3)])
def test_layered_dielectric_is_exact(eps1, eps2, K0):
    """Two dielectric layers meeting midway between node planes K0-1 and K0.
    The continuum solution of -(eps phi')' = 0 (flux continuity at the
    interface, Eq. (4) third line) is piecewise linear; with harmonic-mean
    faces the discrete solution equals it at every node."""
    nx, ny, nz, h = 4, 5, 21, 0.5
    i, j, k = _ijk(nx, ny, nz)
    eps = np.where(k < K0, eps1, eps2).astype(float)
    g = _grid(nx, ny, nz, h, eps, bc=(NM, NM, NM, NM, D, D), bcv=(0, 0, 0, 0, 0.0, 1.0))
    x, info = oracle.linear_solve(g, None, np.zeros(nx * ny * nz), tol=1e-14)
    L, xi = (nz - 1) * h, (K0 - 0.5) * h
    F = 1.0 / (xi / eps1 + (L - xi) / eps2)
    z = k * h
    exact = np.where(z <= xi, F * z / eps1, 1.0 - F * (L - z) / eps2)
    np.testing.assert_allclose(x, exact, rtol=0, atol=1e-12)


def test_debye_hueckel_discrete_exact():
    """Uniform eps, sigma = eps kappa^2, Neumann x/y, phi = V at z = 0 and 0 at
    z = L: the discrete solution is V sinh((n-1-k) theta) / sinh((n-1) theta)
    with cosh(theta) = 1 + h^2 kappa^2 / 2 (linearised PB, 1D profile)."""
    nx, ny, nz, h, eps, kappa, V = 3, 4, 41, 0.5, 78.45, 0.3, 2.0
    N = nx * ny * nz
    g = _grid(nx, ny, nz, h, eps, bc=(NM, NM, NM, NM, D, D), bcv=(0, 0, 0, 0, V, 0.0))
    x, _ = oracle.linear_solve(g, np.full(N, eps * kappa ** 2), np.zeros(N), tol=1e-14)
    theta = math.acosh(1.0 + 0.5 * (h * kappa) ** 2)
    k = _ijk(nx, ny, nz)[2]
    exact = V * np.sinh((nz - 1 - k) * theta) / math.sinh((nz - 1) * theta)
    np.testing.assert_allclose(x, exact, rtol=0, atol=1e-13 * V)


def _manufactured(n):
    """u = sin(pi x) sin(pi y) sin(pi z) on [-1,1]^3, eps = 2 + |r|^2,
    f = -div(eps grad u) analytically."""
    h = 2.0 / (n - 1)
    i, j, k = _ijk(n, n, n)
    x, y, z = -1 + i * h, -1 + j * h, -1 + k * h
    sx, sy, sz = np.sin(np.pi * x), np.sin(np.pi * y), np.sin(np.pi * z)
    cx, cy, cz = np.cos(np.pi * x), np.cos(np.pi * y), np.cos(np.pi * z)
    eps = 2.0 + x * x + y * y + z * z
    u = sx * sy * sz
    f = 3 * np.pi ** 2 * eps * u - 2 * np.pi * (x * cx * sy * sz + y * sx * cy * sz + z * sx * sy * cz)
    return h, eps, u, f


def test_manufactured_second_order():
    errs = []
    for n in (17, 33, 65):
        h, eps, u, f = _manufactured(n)
        g = _grid(n, n, n, h, eps)
        x, info = oracle.linear_solve(g, None, f, tol=1e-12)
        errs.append(np.abs(x - u).max())
    orders = [math.log2(errs[m] / errs[m + 1]) for m in range(2)]
    assert all(1.9 <= o <= 2.1 for o in orders), (errs, orders)


# ----------------------------------------------------- BiCGSTAB vs dense LU

@pytest.mark.parametrize("seed", [0, 1, 2])
def test_bicgstab_matches_dense_lu(seed):
    rng = np.random.default_rng(seed)
    nx, ny, nz = 7, 8, 9
    N = nx * ny * nz
    eps = np.exp(rng.uniform(0, math.log(80), N))
    typ = np.zeros(N, np.uint8)
    typ[rng.choice(N, 12, replace=False)] = oracle.FIXED
    g = _grid(nx, ny, nz, 0.37, eps, bc=(NM, NM, D, D, D, NM), bcv=(0, 0, 0.3, -1.2, 0.7, 0),
              node_type=typ, fixed_value=rng.normal(size=N))
    sigma = np.where(rng.uniform(size=N) < 0.5, rng.uniform(0, 20, N), 0.0)
    b = rng.normal(size=N) * 50
    A, isd, val = _apply(g, sigma)
    M = _dense(nx, ny, nz, A)
    bfull = np.where(isd == 1, val, b)
    ref = np.linalg.solve(M, bfull)
    x, info = oracle.linear_solve(g, sigma, b, tol=1e-13)
    assert info["rel_res"] <= 1e-13
    assert np.linalg.norm(x - ref) <= 1e-11 * np.linalg.norm(ref)
    # the returned relative residual is measured against the lifted RHS
    r = bfull - M @ x
    xd = np.where(isd == 1, val, 0.0)
    assert np.linalg.norm(r) / np.linalg.norm(bfull - M @ xd) == pytest.approx(info["rel_res"], rel=1e-6, abs=1e-15)


def test_bicgstab_small_hand_system():
    """3x3 grid interior of a 3x3x3 box: one free node.  BiCGSTAB must return
    x = (b + sum of Dirichlet neighbour couplings) / diag after one step."""
    g = _grid(3, 3, 3, 1.0, 2.0, bcv=(1.0, 2.0, 3.0, 4.0, 5.0, 6.0))
    b = np.zeros(27)
    b[13] = 7.0
    x, info = oracle.linear_solve(g, None, b, tol=1e-14)
    # interior node: 6 faces of coefficient 2; neighbours carry face values
    assert x[13] == pytest.approx((7.0 + 2.0 * (1 + 2 + 3 + 4 + 5 + 6)) / 12.0, rel=1e-15)
    assert info["iters"] == 1


# ------------------------------------------------------------- edge cases

def test_zero_rhs_gives_dirichlet_lift_only():
    g = _grid(5, 5, 5, 0.5, 3.0)
    x, info = oracle.linear_solve(g, None, np.zeros(125), x0=np.ones(125), tol=1e-10)
    assert info["iters"] == 0 and np.all(x == 0)


def test_max_iter_reports_noconv():
    p = _grid(9, 9, 9, 0.25, 3.0)
    x, info = oracle.linear_solve(p, None, np.ones(729), tol=1e-12, maxit=1, check=False)
    assert info["status"] == oracle.ENOCONV and info["iters"] == 1


def test_singular_neumann_terminates():
    """All-Neumann, sigma = 0: singular.  An inconsistent RHS must end in a
    reported failure, not a hang."""
    g = _grid(5, 5, 5, 0.5, 2.0, bc=(NM,) * 6)
    b = np.random.default_rng(3).normal(size=125)
    x, info = oracle.linear_solve(g, None, b, tol=1e-12, maxit=500, check=False)
    assert info["status"] in (oracle.ENOCONV, oracle.EBREAKDOWN, oracle.ENONFINITE)


@pytest.mark.parametrize("bad", ["small", "eps0", "epsnan", "h0"])
def test_bad_arguments(bad):
    n = 2 if bad == "small" else 5
    eps = np.full(n ** 3, 2.0)
    if bad == "eps0":
        eps[7] = 0.0
    if bad == "epsnan":
        eps[3] = np.nan
    g = _grid(n, n, n, 0.0 if bad == "h0" else 0.5, eps)
    with pytest.raises(oracle.OracleError) as e:
        oracle.linear_solve(g, None, np.ones(n ** 3))
    assert e.value.code == oracle.EARG


def test_dirichlet_precedence():
    """Later faces (order -x,+x,-y,+y,-z,+z) win on edges; FIXED nodes keep
    their own value; Neumann faces never override Dirichlet ones."""
    n = 4
    typ = np.zeros(n ** 3, np.uint8)
    typ[0] = oracle.FIXED
    fv = np.zeros(n ** 3)
    fv[0] = 9.0
    g = _grid(n, n, n, 1.0, 1.0, bc=(D, NM, D, NM, D, NM), bcv=(1.0, 0, 2.0, 0, 3.0, 0),
              node_type=typ, fixed_value=fv)
    isd, val = oracle.dirichlet(g)
    idx = lambda i, j, k: i + n * (j + n * k)
    assert val[idx(0, 0, 0)] == 9.0
    assert val[idx(0, 2, 2)] == 1.0
    assert val[idx(0, 0, 2)] == 2.0
    assert val[idx(0, 2, 0)] == 3.0 and val[idx(2, 0, 0)] == 3.0
    assert isd[idx(3, 2, 2)] == 0 and isd[idx(3, 3, 3)] == 0
    assert isd.sum() == n ** 3 - (n - 1) ** 3


def test_max_norm_stop_rule():
    """Table 3's absolute max-norm test: the returned x meets ||b - A x||_inf <=
    tol, recomputed here with a sparse matrix of the same diagonals."""
    import scipy.sparse as sps
    g, sigma, b = _stop_rule_problem()
    N = g.nx * g.ny * g.nz
    isd, val = oracle.dirichlet(g)
    A = oracle.assemble(g.nx, g.ny, g.nz, g.h, g.eps, sigma, isd, g.bc_phi)
    offs = [0, 1, -1, -g.nx, g.nx, -g.nx * g.ny, g.nx * g.ny]
    # row n of diagonal d holds a[n, n + off_d]
    M = sps.lil_matrix((N, N))
    for d, off in enumerate(offs):
        for n in range(N):
            m = n + off
            if 0 <= m < N and A[d, n] != 0.0:
                M[n, m] += A[d, n]
    M = M.tocsr()
    for tol in (1e-3, 1e-7):
        x, info = oracle.linear_solve(g, sigma, b, tol=tol, rule=1)
        r = np.where(isd.astype(bool), val - x, b - M @ x)
        assert np.abs(r).max() <= tol
        assert info["max_res"] == pytest.approx(np.abs(r).max(), rel=1e-6, abs=1e-15)
    # the relative rule at a loose tolerance leaves a larger max norm than the strict absolute one
    x0, i0 = oracle.linear_solve(g, sigma, b, tol=1e-3)
    x1, i1 = oracle.linear_solve(g, sigma, b, tol=1e-9, rule=1)
    assert i1["iters"] > i0["iters"]


def _stop_rule_problem():
    rng = np.random.default_rng(12)
    nx, ny, nz = 9, 8, 7
    N = nx * ny * nz
    eps = rng.uniform(1.0, 40.0, N)
    g = oracle.Grid(nx, ny, nz, 0.3, eps, bc_phi=(D, NM, D, D, NM, D), bc_value=(0.5, 0, -0.25, 0.0, 0, 1.0))
    return g, rng.uniform(0.0, 2.0, N), rng.normal(size=N)


def test_pf1_operator_sine_modes():
    """PF1's operator eps_s (1 - lc^2 Lap_h) (Eq. (12), constant coefficient
    eps_s lc^2 on every face, eps_s on the diagonal): the Dirichlet sine modes
    are eigenvectors with eigenvalue eps_s (1 + lc^2 lambda_m)."""
    nx, ny, nz, h, eps_s, lc = 9, 8, 7, 0.4, 78.45, 1.9
    N = nx * ny * nz
    g = _grid(nx, ny, nz, h, eps_s * lc * lc, [D] * 6)
    isd, _ = oracle.dirichlet(g)
    A = oracle.assemble(nx, ny, nz, h, np.full(N, eps_s * lc * lc), np.full(N, eps_s), isd)
    i, j, k = _ijk(nx, ny, nz)
    for modes in ((1, 1, 1), (2, 3, 4)):
        u = np.ones(N)
        lam = 0.0
        for idx, n, m in zip((i, j, k), (nx, ny, nz), modes):
            u *= np.sin(m * math.pi * idx / (n - 1))
            lam += math.sin(m * math.pi / (2 * (n - 1))) ** 2
        lam *= 4.0 / h ** 2
        Au = oracle.dia_matvec(nx, ny, nz, A, u)
        free = isd == 0
        want = eps_s * (1.0 + lc * lc * lam)
        np.testing.assert_allclose(Au[free], want * u[free], rtol=0, atol=1e-12 * want)
