"""GPU parity: the HIP path (through the C-ABI) against the CPU oracle.

Bars (stated per test):
  * stencil operator, FP64: |y_gpu - y_oracle| <= 16 eps * sum_j |A_ij x_j|
    (a few roundings in a 7-term sum; reduction orders differ);
  * FP32 operator: same with the FP32 unit roundoff, against the FP64 oracle;
  * linear solves, FP64: relative L2 <= 1e-9 against the oracle solved to 1e-13
    (the GPU stops at rel. res. 1e-12 here so that the kappa amplification of
    the residual cannot exceed the bar; the 1e-10 benchmark stop is checked
    separately through its true residual);
  * mixed precision: true FP64 rel. res. <= 1e-10 and relative L2 <= 1e-8;
  * Fermi update: relative difference of C_i <= 1e-12 (1 + |z_i phi|): the root
    is only defined to the rounding of exponents of size |z_i phi|;
  * nonlinear loop: relative L2 <= 1e-9 at outer_tol 1e-11.
"""
import math
import os

import numpy as np
import pytest

import oracle
from paper_1711_04060_amd import inputs

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

D, NM = oracle.DIRICHLET, oracle.NEUMANN
EPS64 = np.finfo(np.float64).eps
EPS32 = np.finfo(np.float32).eps


def _pf():
    from paper_1711_04060_amd import pf
    pf.load()
    return pf


def dev(a, dt=None):
    dt = dt or torch.float64
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dt, device="cuda")


def host(t):
    return t.detach().cpu().numpy()


def _rand_problem(nx, ny, nz, seed, bc=(D,) * 6, bcv=(0.0,) * 6, nfixed=0, h=0.37):
    rng = np.random.default_rng(seed)
    N = nx * ny * nz
    eps = np.exp(rng.uniform(0, math.log(80), N))
    typ = np.zeros(N, np.uint8)
    typ[rng.uniform(size=N) < 0.3] = oracle.SOLUTE
    if nfixed:
        typ[rng.choice(N, nfixed, replace=False)] = oracle.FIXED
    fv = rng.normal(size=N)
    return inputs.Problem(name="rand", nx=nx, ny=ny, nz=nz, h=h, origin=(0, 0, 0), eps=eps, node_type=typ,
                          fixed_charge=np.zeros(N), bc_phi=tuple(bc), bc_value=tuple(bcv), fixed_value=fv)


def _oracle_A(p, sigma=None):
    isd, val = oracle.dirichlet(p)
    A = oracle.assemble(p.nx, p.ny, p.nz, p.h, p.eps, sigma, isd, p.bc_phi)
    return A, isd, val


def _abs_terms(p, A, x):
    return oracle.dia_matvec(p.nx, p.ny, p.nz, np.abs(A), np.abs(x))


SHAPES = [
    (5, 4, 3, (D,) * 6),
    (37, 23, 19, (D,) * 6),                      # several strips, ragged tail
    (33, 33, 33, (NM, NM, NM, NM, D, D)),
    (19, 41, 9, (NM, D, NM, NM, NM, D)),
    (70, 9, 12, (NM,) * 4 + (D, NM)),
]


@pytest.mark.parametrize("shape", SHAPES, ids=lambda s: f"{s[0]}x{s[1]}x{s[2]}")
@pytest.mark.parametrize("with_sigma", [False, True])
def test_spmv_fp64_matches_dia(shape, with_sigma):
    pf = _pf()
    nx, ny, nz, bc = shape
    p = _rand_problem(nx, ny, nz, seed=nx * 7 + ny, bc=bc, bcv=(0.5, -1, 2, 0, 1.5, -0.25), nfixed=3)
    rng = np.random.default_rng(1)
    sigma = rng.uniform(0, 50, p.N) if with_sigma else None
    x = rng.normal(size=p.N)
    A, isd, val = _oracle_A(p, sigma)
    g = pf.grid_from_problem(p)
    y = torch.empty(p.N, dtype=torch.float64, device="cuda")
    # plain operator
    pf.pf_spmv(g, None if sigma is None else dev(sigma), dev(x), y, 0)
    ref = oracle.dia_matvec(nx, ny, nz, A, x)
    bound = 16 * EPS64 * _abs_terms(p, A, x)
    assert np.all(np.abs(host(y) - ref) <= bound)
    # Jacobi-scaled operator M^-1 A x, M = diag(A)
    pf.pf_spmv(g, None if sigma is None else dev(sigma), dev(x), y, 1)
    ref = oracle.dia_matvec(nx, ny, nz, A, x) / A[0]
    bound = 16 * EPS64 * _abs_terms(p, A, x) / np.abs(A[0])
    assert np.all(np.abs(host(y) - ref) <= bound)


@pytest.mark.parametrize("shape", SHAPES[1:3], ids=lambda s: f"{s[0]}x{s[1]}x{s[2]}")
def test_spmv_fp32_matches_dia(shape):
    pf = _pf()
    nx, ny, nz, bc = shape
    p = _rand_problem(nx, ny, nz, seed=3, bc=bc)
    rng = np.random.default_rng(2)
    x = rng.normal(size=p.N).astype(np.float32)
    sigma = rng.uniform(0, 5, p.N)
    A, isd, val = _oracle_A(p, sigma)
    g = pf.grid_from_problem(p)
    y = torch.empty(p.N, dtype=torch.float32, device="cuda")
    pf.pf_spmv_f32(g, dev(sigma), dev(x, torch.float32), y, 1)
    x64 = x.astype(np.float64)
    ref = oracle.dia_matvec(nx, ny, nz, A, x64) / A[0]
    bound = 24 * EPS32 * _abs_terms(p, A, x64) / np.abs(A[0])
    assert np.all(np.abs(host(y).astype(np.float64) - ref) <= bound)


def test_residual_matches_oracle():
    pf = _pf()
    p = _rand_problem(37, 23, 19, seed=5, bc=(NM, NM, D, D, D, NM), bcv=(0, 0, 1, -1, 2, 0), nfixed=5)
    rng = np.random.default_rng(3)
    sigma = rng.uniform(0, 10, p.N)
    b = rng.normal(size=p.N) * 100
    x = rng.normal(size=p.N)
    A, isd, val = _oracle_A(p, sigma)
    x[isd == 1] = val[isd == 1]
    g = pf.grid_from_problem(p)
    r = torch.empty(p.N, dtype=torch.float64, device="cuda")
    rel = pf.pf_residual(g, dev(sigma), dev(b), dev(x), r)
    ref = np.where(isd == 1, 0.0, b - oracle.dia_matvec(p.nx, p.ny, p.nz, A, x))
    assert np.all(np.abs(host(r) - ref) <= 16 * EPS64 * (np.abs(b) + _abs_terms(p, A, x)))
    xd = np.where(isd == 1, val, 0.0)
    bl = np.where(isd == 1, 0.0, b - oracle.dia_matvec(p.nx, p.ny, p.nz, A, xd))
    assert rel == pytest.approx(np.linalg.norm(ref) / np.linalg.norm(bl), rel=1e-12)


def _rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


@pytest.mark.parametrize("name", ["sphere33", "rand_mixed_bc"])
def test_linear_solve_fp64_parity(name):
    pf = _pf()
    if name == "sphere33":
        p = inputs.sphere_poisson(33)
        sigma, b = None, p.b
    else:
        p = _rand_problem(37, 23, 19, seed=11, bc=(NM, NM, D, D, D, NM), bcv=(0, 0, 0.3, -1.2, 0.7, 0), nfixed=7)
        rng = np.random.default_rng(4)
        sigma = np.where(rng.uniform(size=p.N) < 0.5, rng.uniform(0, 20, p.N), 0.0)
        b = rng.normal(size=p.N) * 50
    ref, oinfo = oracle.linear_solve(p, sigma, b, tol=1e-13)
    g = pf.grid_from_problem(p)
    x = torch.zeros(p.N, dtype=torch.float64, device="cuda")
    info = pf.pf_linear_solve(g, None if sigma is None else dev(sigma), dev(b), x,
                              pf.pf_lin_opts_default(rel_tol=1e-12))
    assert info["status"] == 0 and info["rel_res"] <= 1e-12
    assert _rel(host(x), ref) <= 1e-9
    # the benchmark stop (1e-10) meets its residual bound and is within 1e-7 of the solution
    x2 = torch.zeros_like(x)
    info2 = pf.pf_linear_solve(g, None if sigma is None else dev(sigma), dev(b), x2)
    assert info2["rel_res"] <= 1e-10
    assert _rel(host(x2), ref) <= 1e-7


# (threads, nodes per thread, z-planes per workgroup, load pipeline depth):
# odd plane counts run a step past the tile's last plane; every shape and
# depth the autotuner may pick must give the same answers
LAUNCHES = [(256, 1, 3, 1), (256, 2, 2, 2), (512, 1, 5, 2), (512, 2, 4, 1), (1024, 1, 3, 2), (1024, 1, 7, 1)]


@pytest.mark.parametrize("launch", LAUNCHES, ids=lambda l: "t%d_p%d_kz%d_d%d" % l)
def test_launch_shapes_and_pipeline_depths(launch):
    pf = _pf()
    nt, ppt, kz, depth = launch
    p = _rand_problem(37, 23, 19, seed=11, bc=(NM, NM, D, D, D, NM), bcv=(0, 0, 0.3, -1.2, 0.7, 0), nfixed=7)
    rng = np.random.default_rng(4)
    sigma = np.where(rng.uniform(size=p.N) < 0.5, rng.uniform(0, 20, p.N), 0.0)
    b = rng.normal(size=p.N) * 50
    ref, _ = oracle.linear_solve(p, sigma, b, tol=1e-13)
    A, isd, val = _oracle_A(p, sigma)
    pf.pf_set_launch(nt * ppt, kz, nt, depth)
    try:
        g = pf.grid_from_problem(p)
    finally:
        pf.pf_set_launch(0, 0, 0, 0)
    x = rng.normal(size=p.N)
    y = torch.empty(p.N, dtype=torch.float64, device="cuda")
    pf.pf_spmv(g, dev(sigma), dev(x), y, 1)
    ref_y = oracle.dia_matvec(p.nx, p.ny, p.nz, A, x) / A[0]
    assert np.all(np.abs(host(y) - ref_y) <= 16 * EPS64 * _abs_terms(p, A, x) / np.abs(A[0]))
    xs = torch.zeros(p.N, dtype=torch.float64, device="cuda")
    info = pf.pf_linear_solve(g, dev(sigma), dev(b), xs, pf.pf_lin_opts_default(rel_tol=1e-12))
    assert info["status"] == 0 and _rel(host(xs), ref) <= 1e-9
    xs.zero_()
    info = pf.pf_linear_solve(g, dev(sigma), dev(b), xs, pf.pf_lin_opts_default(precision=pf.PF_MIXED))
    assert info["status"] == 0 and info["rel_res"] <= 1e-10 and _rel(host(xs), ref) <= 1e-8


def test_wide_planes():
    """Planes wider than the register halo (2 nx > threads): the WIDE form."""
    pf = _pf()
    p = _rand_problem(521, 5, 6, seed=21, bc=(D, NM, NM, D, D, NM), bcv=(0.4, 0, 0, -0.3, 1.0, 0))
    rng = np.random.default_rng(8)
    b = rng.normal(size=p.N) * 20
    A, isd, val = _oracle_A(p)
    ref, _ = oracle.linear_solve(p, None, b, tol=1e-13)
    g = pf.grid_from_problem(p)
    x = rng.normal(size=p.N)
    y = torch.empty(p.N, dtype=torch.float64, device="cuda")
    pf.pf_spmv(g, None, dev(x), y, 1)
    ref_y = oracle.dia_matvec(p.nx, p.ny, p.nz, A, x) / A[0]
    assert np.all(np.abs(host(y) - ref_y) <= 16 * EPS64 * _abs_terms(p, A, x) / np.abs(A[0]))
    xs = torch.zeros(p.N, dtype=torch.float64, device="cuda")
    info = pf.pf_linear_solve(g, None, dev(b), xs, pf.pf_lin_opts_default(rel_tol=1e-12))
    assert info["status"] == 0 and _rel(host(xs), ref) <= 1e-9


def test_linear_solve_mixed_parity():
    pf = _pf()
    p = inputs.sphere_poisson(65)
    ref, _ = oracle.linear_solve(p, None, p.b, tol=1e-13)
    g = pf.grid_from_problem(p)
    x = torch.zeros(p.N, dtype=torch.float64, device="cuda")
    info = pf.pf_linear_solve(g, None, dev(p.b), x, pf.pf_lin_opts_default(precision=pf.PF_MIXED))
    assert info["status"] == 0 and info["rel_res"] <= 1e-10 and info["refinements"] >= 1
    rel = pf.pf_residual(g, None, dev(p.b), x)
    assert rel <= 1e-10
    assert _rel(host(x), ref) <= 1e-8


def test_linear_solve_is_deterministic():
    pf = _pf()
    p = inputs.sphere_poisson(33)
    g = pf.grid_from_problem(p)
    xs = []
    for _ in range(2):
        x = torch.zeros(p.N, dtype=torch.float64, device="cuda")
        pf.pf_linear_solve(g, None, dev(p.b), x)
        xs.append(host(x))
    assert np.array_equal(xs[0], xs[1])


def test_zero_rhs_and_noconv_and_bad_args():
    pf = _pf()
    p = inputs.sphere_poisson(33)
    g = pf.grid_from_problem(p)
    x = torch.ones(p.N, dtype=torch.float64, device="cuda")
    info = pf.pf_linear_solve(g, None, torch.zeros_like(x), x)
    assert info["iters"] == 0 and float(x.abs().max()) == 0.0
    x = torch.zeros_like(x)
    info = pf.pf_linear_solve(g, None, dev(p.b), x, pf.pf_lin_opts_default(max_iter=1), check=False)
    assert info["status"] == pf.PF_ERR_NOCONV
    with pytest.raises(pf.PfError) as e:
        pf.pf_linear_solve(g, None, dev(p.b), x, pf.pf_lin_opts_default(rel_tol=-1.0))
    assert e.value.code == pf.PF_ERR_ARG
    bad = p.eps.copy()
    bad[100] = -1.0
    with pytest.raises(pf.PfError) as e:
        pf.pf_grid_create(p.nx, p.ny, p.nz, p.h, dev(bad))
    assert e.value.code == pf.PF_ERR_ARG
    bad[100] = np.nan
    with pytest.raises(pf.PfError) as e:
        pf.pf_grid_create(p.nx, p.ny, p.nz, p.h, dev(bad))
    assert e.value.code == pf.PF_ERR_ARG
    with pytest.raises(pf.PfError) as e:
        pf.pf_grid_create(2, 5, 5, 0.1, dev(np.ones(50)))
    assert e.value.code == pf.PF_ERR_ARG


@pytest.mark.parametrize("prec", [0, 1], ids=["fp64", "mixed"])
def test_nan_in_sigma_or_b_is_reported(prec):
    """A NaN injected into sigma (on a free row) or into b ends the solve
    with PF_ERR_NONFINITE, in both precisions, instead of iterating."""
    pf = _pf()
    p = inputs.sphere_poisson(17)
    g = pf.grid_from_problem(p)
    x = torch.zeros(p.N, dtype=torch.float64, device="cuda")
    free = 3 + 17 * (4 + 17 * 5)           # interior solvent node (a free row)
    assert p.node_type[free] == inputs.SOLVENT
    sigma = np.zeros(p.N)
    sigma[free] = np.nan
    opts = pf.pf_lin_opts_default(precision=prec)
    info = pf.pf_linear_solve(g, dev(sigma), dev(p.b), x, opts, check=False)
    assert info["status"] == pf.PF_ERR_NONFINITE
    b = p.b.copy()
    b[free] = np.nan
    x.zero_()
    info = pf.pf_linear_solve(g, None, dev(b), x, opts, check=False)
    assert info["status"] == pf.PF_ERR_NONFINITE
    # the grid still solves a good system afterwards
    x.zero_()
    info = pf.pf_linear_solve(g, None, dev(p.b), x, opts)
    assert info["status"] == 0


@pytest.mark.parametrize("prec", [0, 1], ids=["fp64", "mixed"])
def test_negative_sigma_is_rejected(prec):
    """sigma < 0 on a free row breaks the operator's precondition (a
    nonnegative diagonal shift, so that D > 0 and the Jacobi scaling is
    defined): the solve returns PF_ERR_ARG before iterating, single and
    batched.  A negative value on a Dirichlet row is not read and passes."""
    pf = _pf()
    p = inputs.sphere_poisson(17)
    g = pf.grid_from_problem(p)
    x = torch.zeros(p.N, dtype=torch.float64, device="cuda")
    free = 3 + 17 * (4 + 17 * 5)
    opts = pf.pf_lin_opts_default(precision=prec)
    sigma = np.full(p.N, 0.5)
    sigma[free] = -1e-3
    info = pf.pf_linear_solve(g, dev(sigma), dev(p.b), x, opts, check=False)
    assert info["status"] == pf.PF_ERR_ARG
    g2 = pf.grid_from_problem(p)
    x2 = torch.zeros(p.N, dtype=torch.float64, device="cuda")
    infos = pf.pf_linear_solve_batch([g, g2], [dev(sigma), None], [dev(p.b), dev(p.b)], [x, x2], opts,
                                     check=False)
    assert infos[0]["status"] == pf.PF_ERR_ARG and infos[1]["status"] == 0
    sigma[free] = 0.5
    sigma[0] = -5.0                        # corner: a Dirichlet row
    x.zero_()
    info = pf.pf_linear_solve(g, dev(sigma), dev(p.b), x, opts)
    assert info["status"] == 0


def test_singular_neumann_terminates():
    pf = _pf()
    n = 9
    g = pf.pf_grid_create(n, n, n, 0.5, dev(np.full(n ** 3, 2.0)), bc_phi=(NM,) * 6)
    b = dev(np.random.default_rng(0).normal(size=n ** 3))
    x = torch.zeros(n ** 3, dtype=torch.float64, device="cuda")
    info = pf.pf_linear_solve(g, None, b, x, pf.pf_lin_opts_default(max_iter=400), check=False)
    assert info["status"] in (pf.PF_ERR_NOCONV, pf.PF_ERR_BREAKDOWN, pf.PF_ERR_NONFINITE)


@pytest.mark.parametrize("batched", [False, True])
def test_mixed_falls_back_to_fp64_when_fp32_fails(batched):
    """Coefficients whose FP32 face terms overflow (eps ~ 1e38 with 1/h^2 =
    100; FP64 represents them without trouble) leave the FP32 Krylov run
    without a usable correction: the refinement step is undone, the solve
    finishes in FP64 and reports it, and the result meets the FP64 bar
    against the oracle.  In a batch, only that member falls back; a member
    with ordinary coefficients keeps refining in FP32."""
    pf = _pf()
    rng = np.random.default_rng(21)
    n = 17
    p = _rand_problem(n, n, n, seed=21, h=0.1)
    p = inputs.Problem(name="big_eps", nx=n, ny=n, nz=n, h=0.1, origin=(0, 0, 0), eps=p.eps * 1e36,
                       node_type=p.node_type, fixed_charge=np.zeros(p.N), bc_phi=(D,) * 6,
                       bc_value=(0.0,) * 6, fixed_value=p.fixed_value)
    b = rng.normal(size=p.N)
    ref, _ = oracle.linear_solve(p, None, b, tol=1e-13)
    opts = pf.pf_lin_opts_default(precision=pf.PF_MIXED, rel_tol=1e-12)
    g = pf.grid_from_problem(p)
    x = torch.zeros(p.N, dtype=torch.float64, device="cuda")
    if not batched:
        info = pf.pf_linear_solve(g, None, dev(b), x, opts)
    else:
        q = inputs.sphere_poisson(n)
        gq = pf.grid_from_problem(q)
        xq = torch.zeros(q.N, dtype=torch.float64, device="cuda")
        infos = pf.pf_linear_solve_batch([g, gq], [None, None], [dev(b), dev(q.b)], [x, xq], opts)
        info, iq = infos
        assert iq["status"] == 0 and iq["fp64_fallback"] == 0 and iq["refinements"] >= 1
        assert pf.pf_residual(gq, None, dev(q.b), xq) <= 1e-12
    assert info["status"] == 0 and info["fp64_fallback"] == 1 and info["refinements"] >= 1
    assert pf.pf_residual(g, None, dev(b), x) <= 1e-12
    assert _rel(host(x), ref) <= 1e-9


# ------------------------------------------------------------------- Fermi

def _membrane_params(pf, **kw):
    ms = inputs.MEMBRANE_SPECIES
    return pf.Params(ms["valence"], ms["radius_A"], ms["bath_M"], **kw)


@pytest.mark.parametrize("steric", [1, 0])
def test_fermi_matches_oracle(steric):
    pf = _pf()
    ms = inputs.MEMBRANE_SPECIES
    n = 13
    N = n ** 3
    rng = np.random.default_rng(7)
    span = 2000.0 if steric else 30.0
    phi = np.concatenate([rng.uniform(-span, span, N - 5), [0.0, 1e-3, -1e-3, span, -span]])
    typ = np.where(rng.uniform(size=N) < 0.2, oracle.SOLUTE, oracle.SOLVENT).astype(np.uint8)
    p = inputs.Problem("f", n, n, n, 1.0, (0, 0, 0), np.full(N, 2.0), typ, np.zeros(N))
    g = pf.grid_from_problem(p)
    prm = _membrane_params(pf, steric=steric)
    rho, sig, S = (torch.empty(N, dtype=torch.float64, device="cuda") for _ in range(3))
    conc = torch.empty(4 * N, dtype=torch.float64, device="cuda")
    pf.pf_fermi(g, prm, dev(phi), rho, sig, conc, S)
    sp = oracle.species_from_molar(ms["valence"], ms["radius_A"], ms["bath_M"], steric=bool(steric))
    orho, osig, oconc, oS = oracle.fermi(phi, sp, typ)
    z = np.abs(np.asarray(ms["valence"]))[:, None]
    tolc = 1e-12 * (1 + z * np.abs(phi)[None, :])
    c = host(conc).reshape(4, N)
    assert np.all(np.abs(c - oconc) <= tolc * np.abs(oconc) + 1e-300)
    np.testing.assert_allclose(host(S), oS, rtol=1e-12, atol=1e-12)
    scale = np.abs(osig) + 1e-300
    assert np.all(np.abs(host(sig) - osig) <= 4e-12 * (1 + 2 * np.abs(phi)) * scale)
    assert np.all(np.abs(host(rho) - orho) <= 4e-12 * (1 + 2 * np.abs(phi)) * scale)


# --------------------------------------------------------------- nonlinear

@pytest.mark.parametrize("n,nc", [(17, 40), (25, 200)])
def test_nonlinear_matches_oracle(n, nc):
    pf = _pf()
    prob = inputs.membrane_pore(n, n_charges=nc)
    ms = prob.meta["species"]
    sp = oracle.species_from_molar(ms["valence"], ms["radius_A"], ms["bath_M"])
    ref, oinfo, oconc, oS = oracle.nonlinear_solve(prob, prob.fixed_charge, sp, 78.45, 1.9, outer_tol=1e-11,
                                                  lin_tol=1e-13, want_conc=True)
    g = pf.grid_from_problem(prob)
    prm = pf.params_for(prob, outer_tol=1e-11, lin={"rel_tol": 1e-13})
    phi = torch.zeros(prob.N, dtype=torch.float64, device="cuda")
    conc = torch.empty(4 * prob.N, dtype=torch.float64, device="cuda")
    S = torch.empty(prob.N, dtype=torch.float64, device="cuda")
    info = pf.pf_nonlinear_solve(g, prm, phi, conc, S)
    assert info["status"] == 0
    assert _rel(host(phi), ref) <= 1e-9
    assert abs(info["outer_iters"] - oinfo["outer_iters"]) <= 3
    assert _rel(host(conc).reshape(4, -1), oconc) <= 1e-8


def test_nonlinear_bias_and_warm_start():
    pf = _pf()
    prob = inputs.membrane_pore(17, n_charges=40, bias_phi=150.0 / inputs.thermal_voltage_mV())
    ms = prob.meta["species"]
    sp = oracle.species_from_molar(ms["valence"], ms["radius_A"], ms["bath_M"])
    ref, _, _, _ = oracle.nonlinear_solve(prob, prob.fixed_charge, sp, 78.45, 1.9, outer_tol=1e-11, lin_tol=1e-13)
    g = pf.grid_from_problem(prob)
    prm = pf.params_for(prob, outer_tol=1e-11, lin={"rel_tol": 1e-13})
    phi = torch.zeros(prob.N, dtype=torch.float64, device="cuda")
    pf.pf_nonlinear_solve(g, prm, phi)
    assert _rel(host(phi), ref) <= 1e-9
    prm2 = pf.params_for(prob, outer_tol=1e-8, warm_start=1, lin={"rel_tol": 1e-13})
    info = pf.pf_nonlinear_solve(g, prm2, phi)
    assert info["outer_iters"] == 1


# ------------------------------------------------------------------- batch

def test_linear_batch_matches_single_solves():
    """Batched launches (one kernel launch per BiCGSTAB step for all members)
    give each member the answer of its standalone solve (FP64: 1e-9 against
    the oracle; mixed: residual 1e-10 and 1e-8)."""
    pf = _pf()
    probs = inputs.batch_systems(n_sys=6, seed_base=4000)
    probs = [p for p in probs if p.nx <= 65][:3] + [inputs.sphere_poisson(33)]
    grids = [pf.grid_from_problem(p) for p in probs]
    bs = [dev(p.b) for p in probs]
    sg = [None if p.sigma is None else dev(p.sigma) for p in probs]
    refs = [oracle.linear_solve(p, p.sigma, p.b, tol=1e-13)[0] for p in probs]
    for prec, tol, bar in ((0, 1e-12, 1e-9), (1, 1e-10, 1e-8)):
        xs = [torch.zeros(p.N, dtype=torch.float64, device="cuda") for p in probs]
        infos = pf.pf_linear_solve_batch(grids, sg, bs, xs, pf.pf_lin_opts_default(rel_tol=tol, precision=prec))
        for p, g, s, b, x, ref, info in zip(probs, grids, sg, bs, xs, refs, infos):
            assert info["status"] == 0 and info["rel_res"] <= tol
            assert pf.pf_residual(g, s, b, x) <= tol
            assert _rel(host(x), ref) <= bar, (p.name, prec)


def _small_linearised(count):
    """Linearised systems of the 64-system workload with at most 57^3 nodes."""
    return [p for p in inputs.batch_systems(n_sys=16) if p.nx <= 57][:count]


def _solve_with(pf, g, s, b, prec, shift_class, batched=False):
    """Solve(s) with the shift-per-class table allowed or not; returns the
    solutions and the step-A bytes per launch the library accounted."""
    os.environ["PF_SHIFT_CLASS"] = "1" if shift_class else "0"
    pf.pf_timing_enable(1, 1)
    try:
        opts = pf.pf_lin_opts_default(rel_tol=1e-12 if prec == 0 else 1e-10, precision=prec)
        if batched:
            xs = [torch.zeros_like(bb) for bb in b]
            infos = pf.pf_linear_solve_batch(g, s, b, xs, opts)
            kind = pf.TIMING_BATCH_FP64 if prec == 0 else pf.TIMING_BATCH_FP32
        else:
            xs = [torch.zeros_like(b)]
            infos = [pf.pf_linear_solve(g, s, b, xs[0], opts)]
            kind = prec
        t = pf.pf_timing_read(kind)
    finally:
        pf.pf_timing_enable(0, 1)
        os.environ.pop("PF_SHIFT_CLASS", None)
    return xs, infos, t


@pytest.mark.parametrize("prec", [0, 1], ids=["fp64", "mixed"])
def test_shift_per_class_table_matches_per_node_shift(prec):
    """A linearised system's shift is one value per coefficient class (zero in
    the solute, uniform in the solvent): the step kernels then take it from a
    per-class table instead of reading it per node.  The diagonal is summed
    in the same order, so both forms give the same iterates bit for bit; the
    table form reads 8 (FP64) or 4 (FP32) bytes per node less in step A.  A
    shift that differs at one free node keeps the per-node form and still
    matches the oracle."""
    pf = _pf()
    if os.environ.get("PF_PALETTE") == "0":
        pytest.skip("the class table needs the palette form")
    p = _small_linearised(1)[0]
    g = pf.grid_from_problem(p)
    s, b = dev(p.sigma), dev(p.b)
    elem = 8 if prec == 0 else 4
    xt, it, tt = _solve_with(pf, g, s, b, prec, True)
    xn, inn, tn = _solve_with(pf, g, s, b, prec, False)
    assert it[0]["status"] == 0 and inn[0]["status"] == 0
    assert it[0]["iters"] == inn[0]["iters"]
    assert torch.equal(xt[0], xn[0])
    per_t, per_n = tt["bytes"] / tt["launches"], tn["bytes"] / tn["launches"]
    assert per_n - per_t == elem * p.N
    ref = oracle.linear_solve(p, p.sigma, p.b, tol=1e-13)[0]
    assert _rel(host(xt[0]), ref) <= (1e-9 if prec == 0 else 1e-8)
    # one free solvent node with a different shift: per-node form, same bar
    sig2 = p.sigma.copy()
    isd, _ = oracle.dirichlet(p)
    free_solvent = np.flatnonzero((isd == 0) & (sig2 > 0))
    k = int(free_solvent[len(free_solvent) // 2])
    sig2[k] *= 1.5
    x2, i2, t2 = _solve_with(pf, g, dev(sig2), b, prec, True)
    assert i2[0]["status"] == 0 and t2["bytes"] / t2["launches"] == per_n
    ref2 = oracle.linear_solve(p, sig2, p.b, tol=1e-13)[0]
    assert _rel(host(x2[0]), ref2) <= (1e-9 if prec == 0 else 1e-8)
    assert _rel(ref2, ref) > 1e-12   # the perturbation is visible in the solution


def test_batch_shift_per_class_table_matches_oracle():
    """A batch whose members all have a shift per class runs the table form
    (step-A bytes counted without the shift); each member matches the oracle."""
    pf = _pf()
    if os.environ.get("PF_PALETTE") == "0":
        pytest.skip("the class table needs the palette form")
    probs = _small_linearised(3)
    grids = [pf.grid_from_problem(p) for p in probs]
    sg, bs = [dev(p.sigma) for p in probs], [dev(p.b) for p in probs]
    refs = [oracle.linear_solve(p, p.sigma, p.b, tol=1e-13)[0] for p in probs]
    for prec, bar in ((0, 1e-9), (1, 1e-8)):
        elem = 8 if prec == 0 else 4
        xs, infos, t = _solve_with(pf, grids, sg, bs, prec, True, batched=True)
        for p, x, ref, info in zip(probs, xs, refs, infos):
            assert info["status"] == 0
            assert _rel(host(x), ref) <= bar, (p.name, prec)
        # every launch counted moved at most the members' table-form bytes
        full = sum((9 * elem + 1 + 4) * p.N for p in probs)
        assert 0 < t["bytes"] / t["launches"] <= full


@pytest.fixture(scope="module")
def small_batch_refs():
    probs = _small_linearised(4)
    return probs, [oracle.linear_solve(p, p.sigma, p.b, tol=1e-13)[0] for p in probs]


@pytest.mark.parametrize("policy", range(9))
def test_every_batch_launch_policy_matches_oracle(policy, small_batch_refs):
    """Each of the batched launch policies (kernel instance, z-chunk length,
    step-B strip) the library may keep, pinned through PF_BATCH_POLICY, gives
    every member the oracle's solution (FP64 1e-9, mixed 1e-8)."""
    pf = _pf()
    probs, refs = small_batch_refs
    grids = [pf.grid_from_problem(p) for p in probs]
    sg, bs = [dev(p.sigma) for p in probs], [dev(p.b) for p in probs]
    os.environ["PF_BATCH_POLICY"] = str(policy)
    try:
        for prec, tol, bar in ((0, 1e-12, 1e-9), (1, 1e-10, 1e-8)):
            xs = [torch.zeros(p.N, dtype=torch.float64, device="cuda") for p in probs]
            infos = pf.pf_linear_solve_batch(grids, sg, bs, xs, pf.pf_lin_opts_default(rel_tol=tol, precision=prec))
            for p, x, ref, info in zip(probs, xs, refs, infos):
                assert info["status"] == 0 and info["rel_res"] <= tol
                assert _rel(host(x), ref) <= bar, (p.name, prec, policy)
    finally:
        os.environ.pop("PF_BATCH_POLICY", None)


def test_linear_batch_rejects_shared_grid():
    pf = _pf()
    p = inputs.sphere_poisson(33)
    g = pf.grid_from_problem(p)
    b = dev(p.b)
    xs = [torch.zeros(p.N, dtype=torch.float64, device="cuda") for _ in range(2)]
    with pytest.raises(pf.PfError) as e:
        pf.pf_linear_solve_batch([g, g], None, [b, b], xs)
    assert e.value.code == pf.PF_ERR_ARG
    # empty batches are valid calls that do nothing
    assert pf.pf_linear_solve_batch([], None, [], []) == []
    assert pf.pf_nonlinear_solve_batch([], [], []) == []
    # a batch of one solves like the single call (the batched kernel's
    # launch shape may differ, so to the FP64 bar rather than bit for bit)
    x1 = torch.zeros(p.N, dtype=torch.float64, device="cuda")
    (info,) = pf.pf_linear_solve_batch([g], None, [b], [x1])
    x0 = torch.zeros(p.N, dtype=torch.float64, device="cuda")
    pf.pf_linear_solve(g, None, b, x0)
    assert info["status"] == 0 and info["rel_res"] <= 1e-10
    assert _rel(host(x1), host(x0)) <= 1e-7


def test_nonlinear_batch_bias_sweep_matches_oracle():
    """Three bias voltages solved as one batch match their oracle solves."""
    pf = _pf()
    vt = inputs.thermal_voltage_mV()
    probs = [inputs.membrane_pore(17, n_charges=40, bias_phi=v / vt) for v in (-150.0, 0.0, 150.0)]
    grids = [pf.grid_from_problem(p) for p in probs]
    prms = [pf.params_for(p, outer_tol=1e-11, lin={"rel_tol": 1e-13}) for p in probs]
    phis = [torch.zeros(p.N, dtype=torch.float64, device="cuda") for p in probs]
    infos = pf.pf_nonlinear_solve_batch(grids, prms, phis)
    ms = probs[0].meta["species"]
    sp = oracle.species_from_molar(ms["valence"], ms["radius_A"], ms["bath_M"])
    for p, phi, info in zip(probs, phis, infos):
        ref, _, _, _ = oracle.nonlinear_solve(p, p.fixed_charge, sp, 78.45, 1.9, outer_tol=1e-11, lin_tol=1e-13)
        assert info["status"] == 0
        assert _rel(host(phi), ref) <= 1e-9


def test_timing_of_products_and_bad_kind():
    """pf_timing_read kinds 2 and 3 count the Jacobi-scaled products."""
    pf = _pf()
    p = inputs.sphere_poisson(33)
    g = pf.grid_from_problem(p)
    x = torch.ones(p.N, dtype=torch.float64, device="cuda")
    y = torch.empty_like(x)
    pf.pf_timing_enable(1, 1)
    try:
        pf.pf_spmv(g, None, x, y, 1)
        pf.pf_spmv(g, None, x, y, 0)          # the plain product is not timed
        pf.pf_spmv_f32(g, None, x.float(), y.float(), 1)
        t64 = pf.pf_timing_read(pf.TIMING_SPMV_FP64)
        t32 = pf.pf_timing_read(pf.TIMING_SPMV_FP32)
        # x and y in the working precision and the coefficient field: one
        # palette byte per node (the sphere's field has two values) or a full
        # value when the palette form is switched off
        coef = (lambda e: 1) if os.environ.get("PF_PALETTE") != "0" else (lambda e: e)
        assert t64["launches"] == 1 and t64["bytes"] == (16 + coef(8)) * p.N and t64["mean_ms"] >= 0
        assert t32["launches"] == 1 and t32["bytes"] == (8 + coef(4)) * p.N
        with pytest.raises(pf.PfError):
            pf.pf_timing_read(6)
    finally:
        pf.pf_timing_enable(0, 1)


# ------------------------------------------------------------- stop rules

@pytest.mark.parametrize("prec", [0, 1], ids=["fp64", "mixed"])
def test_max_norm_stop_rule(prec):
    """Table 3's absolute max-norm stop test: the GPU result meets
    ||b - A x||_inf <= tol with the residual recomputed by the oracle's
    diagonals, reports that max norm, and the oracle under the same rule
    agrees on the solution to the accuracy the rule allows."""
    pf = _pf()
    rng = np.random.default_rng(12)
    nx, ny, nz = 41, 37, 29
    N = nx * ny * nz
    eps = rng.uniform(1.0, 40.0, N)
    g = oracle.Grid(nx, ny, nz, 0.3, eps, bc_phi=(D, NM, D, D, NM, D), bc_value=(0.5, 0, -0.25, 0.0, 0, 1.0))
    sigma = rng.uniform(0.0, 2.0, N)
    b = rng.normal(size=N)
    isd, val = oracle.dirichlet(g)
    A = oracle.assemble(nx, ny, nz, g.h, eps, sigma, isd, g.bc_phi)
    G = pf.pf_grid_create(nx, ny, nz, g.h, dev(eps), None, None, None, g.bc_phi, g.bc_value)
    for tol in (1e-4, 1e-8):
        x = torch.zeros(N, dtype=torch.float64, device="cuda")
        info = pf.pf_linear_solve(G, dev(sigma), dev(b), x, pf.pf_lin_opts_default(rel_tol=tol, precision=prec,
                                                                               stop_rule=pf.PF_STOP_ABS_INF))
        xg = host(x)
        r = np.where(isd.astype(bool), 0.0, b - oracle.dia_matvec(nx, ny, nz, A, xg))
        rmax = np.abs(r).max()
        assert rmax <= tol
        # the residual itself is only defined to the rounding of its terms
        terms = (np.abs(b) + oracle.dia_matvec(nx, ny, nz, np.abs(A), np.abs(xg))).max()
        assert abs(info["max_res"] - rmax) <= 1e-6 * rmax + 64 * EPS64 * terms
        ref, rinfo = oracle.linear_solve(g, sigma, b, tol=tol, rule=1)
        # both residuals are within tol; the solutions differ by at most about kappa tol
        assert np.abs(xg - ref).max() <= 1e3 * tol
    # the default rule reports no max norm
    x = torch.zeros(N, dtype=torch.float64, device="cuda")
    info = pf.pf_linear_solve(G, dev(sigma), dev(b), x, pf.pf_lin_opts_default())
    assert info["max_res"] == -1.0


def test_batch_with_max_norm_stop_rule():
    """The absolute max-norm stop rule inside a batched solve: every member
    meets ||b - A x||_inf <= tol (residual recomputed from the oracle's
    diagonals)."""
    pf = _pf()
    probs = [p for p in inputs.batch_systems(n_sys=16, seed_base=4100) if p.nx <= 57][:4]
    grids = [pf.grid_from_problem(p) for p in probs]
    tol = 1e-6
    xs = [torch.zeros(p.N, dtype=torch.float64, device="cuda") for p in probs]
    infos = pf.pf_linear_solve_batch(grids, [dev(p.sigma) for p in probs], [dev(p.b) for p in probs], xs,
                                     pf.pf_lin_opts_default(rel_tol=tol, stop_rule=pf.PF_STOP_ABS_INF))
    for p, x, info in zip(probs, xs, infos):
        isd, val = oracle.dirichlet(p)
        A = oracle.assemble(p.nx, p.ny, p.nz, p.h, p.eps, p.sigma, isd, p.bc_phi)
        r = np.where(isd.astype(bool), 0.0, p.b - oracle.dia_matvec(p.nx, p.ny, p.nz, A, host(x)))
        assert info["status"] == 0
        assert np.abs(r).max() <= tol
