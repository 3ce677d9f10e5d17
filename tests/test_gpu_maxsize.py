"""The largest grid the library accepts (N < 2^29 nodes, so that the byte
offset of every FP64 element fits the stencil kernels' 32-bit offsets):
256 x 1024 x 2047 = 536,608,768 nodes, 262,144 short of the limit, with the
last element at byte offset 4,292,870,136 of each vector.

  * stencil operator on random eps: 64 random interior rows and the interior
    rows at the far corner (the last one included), each against the
    oracle's seven-diagonal assembly of the 3 x 3 x 3 window around it (the
    row of the window's centre node only involves those 27 nodes); every
    row of the first and last plane is a Dirichlet identity row (y = x,
    compared whole, up to the last element of the arrays);
  * FP64 and mixed-precision solves of A x = lambda u for the lowest sine
    mode u of the constant-coefficient operator with zero Dirichlet faces (an
    exact eigenvector, so FP64 BiCGSTAB with the constant Jacobi diagonal
    ends after one iteration; one mixed solve adds sigma = 1, the other
    solves the pure Poisson system without any FP64 fallback): the solution
    equals u (closed form, any size) to the FP64 and mixed-precision parity
    bars (1e-9, 1e-8).

The launch shape is pinned (512 threads, 512-node strips, 32 z-planes,
pipeline depth 1) so that the autotuner does not time its candidates at this
size.
"""
import gc
import math

import numpy as np
import pytest

import oracle

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu
EPS64 = np.finfo(np.float64).eps

NX, NY, NZ = 256, 1024, 2047
N = NX * NY * NZ
H = 0.5


def _pf():
    from paper_1711_04060_amd import pf
    pf.load()
    return pf


@pytest.fixture
def pinned_shape():
    pf = _pf()
    pf.pf_set_launch(512, 32, 512, 1)
    try:
        yield pf
    finally:
        pf.pf_set_launch(0, 0, 0, 0)
        gc.collect()
        torch.cuda.empty_cache()


def test_max_grid_size_limits():
    assert N < 1 << 29 and (N - 1) * 8 < 1 << 32
    assert (1 << 29) - N == 262144


def _node(i, j, k):
    return i + NX * (j + NY * k)


def test_spmv_at_max_size(pinned_shape):
    pf = pinned_shape
    gen = torch.Generator(device="cuda").manual_seed(11)
    eps = torch.exp(torch.rand(N, dtype=torch.float64, device="cuda", generator=gen) * math.log(80.0))
    x = torch.randn(N, dtype=torch.float64, device="cuda", generator=gen)
    g = pf.pf_grid_create(NX, NY, NZ, H, eps)
    y = torch.empty_like(x)
    pf.pf_spmv(g, None, x, y, 0)
    torch.cuda.synchronize()

    rng = np.random.default_rng(5)
    rows = [tuple(int(v) for v in rng.integers(1, (NX - 1, NY - 1, NZ - 1))) for _ in range(64)]
    rows += [(i, j, NZ - 2) for i in (1, NX - 2) for j in (1, NY - 2)]     # far corner of the interior
    rows += [(NX - 2, NY - 2, NZ - 2)]                                       # last interior node
    for (i, j, k) in rows:
        idx = torch.tensor([_node(i + di, j + dj, k + dk) for dk in (-1, 0, 1) for dj in (-1, 0, 1)
                            for di in (-1, 0, 1)], device="cuda")
        we, wx = eps[idx].cpu().numpy(), x[idx].cpu().numpy()
        isd = np.ones(27, np.uint8)
        isd[13] = 0
        A = oracle.assemble(3, 3, 3, H, we, None, isd)
        ref = oracle.dia_matvec(3, 3, 3, A, wx)[13]
        bound = 16 * EPS64 * oracle.dia_matvec(3, 3, 3, np.abs(A), np.abs(wx))[13]
        got = float(y[_node(i, j, k)])
        assert abs(got - ref) <= bound, (i, j, k, got, ref)
    # identity rows of the Dirichlet faces, including the last element of every array
    P = NX * NY
    assert torch.equal(y[N - P:], x[N - P:])
    assert torch.equal(y[:P], x[:P])
    del g
    gc.collect()


def _sine_mode():
    axes = []
    for n in (NX, NY, NZ):
        s = torch.sin(math.pi * torch.arange(n, dtype=torch.float64, device="cuda") / (n - 1))
        s[0] = 0.0
        s[-1] = 0.0
        axes.append(s)
    sx, sy, sz = axes
    u = (sz[:, None, None] * sy[None, :, None]) * sx[None, None, :]
    lam = sum(2.0 * (1.0 - math.cos(math.pi / (n - 1))) for n in (NX, NY, NZ)) / (H * H)
    return u.reshape(-1), lam


@pytest.mark.parametrize("precision", ["fp64", "mixed", "mixed_poisson"])
def test_eigenvector_solve_at_max_size(pinned_shape, precision):
    pf = pinned_shape
    eps = torch.ones(N, dtype=torch.float64, device="cuda")
    g = pf.pf_grid_create(NX, NY, NZ, H, eps)
    del eps
    u, lam = _sine_mode()
    b = u * lam
    x = torch.zeros(N, dtype=torch.float64, device="cuda")
    sigma = None
    if precision == "fp64":
        # b = lambda u carries only its own rounding: one iteration reaches 1e-10
        opts = pf.pf_lin_opts_default(rel_tol=1e-10, precision=pf.PF_FP64)
        tol, max_iters, bar = 1e-10, 4, 1e-9
    elif precision == "mixed_poisson":
        # pure Poisson (no reaction term): M^-1 A has a condition number near
        # 7.5e4 here and the FP32 copy of every residual after the first
        # refinement is rounding noise in every mode; each FP32 run is only
        # asked for two digits (the default inner tolerance), which FP32
        # BiCGSTAB reaches on this operator, so no refinement step fails
        # (1e-10: the FP64 residual itself cannot go much below
        # eps * 7.5e4 ~ 2e-11 on this operator)
        opts = pf.pf_lin_opts_default(rel_tol=1e-10, precision=pf.PF_MIXED, max_iter=10000)
        tol, max_iters, bar = 1e-10, 10000, 1e-8
    else:
        # the FP32 copy of b is u plus rounding noise in every mode; without a
        # reaction term the lowest mode of this grid gives M^-1 A a condition
        # number near 7e4, where FP32 BiCGSTAB needs thousands of iterations for
        # that noise, so the PF2 form with sigma = 1 (same eigenvector, shifted
        # eigenvalue) is solved, to 1e-12 so that the error bar holds
        sigma = torch.ones(N, dtype=torch.float64, device="cuda")
        b = u * (lam + 1.0)
        opts = pf.pf_lin_opts_default(rel_tol=1e-12, precision=pf.PF_MIXED, max_iter=3000)
        tol, max_iters, bar = 1e-12, 200, 1e-8
    info = pf.pf_linear_solve(g, sigma, b, x, opts)
    print(precision, {k: info[k] for k in ("iters", "refinements", "restarts", "rel_res", "fp64_fallback")})
    assert info["fp64_fallback"] == 0
    assert info["rel_res"] <= tol
    assert info["iters"] <= max_iters, info
    err = float(torch.linalg.vector_norm(x - u) / torch.linalg.vector_norm(u))
    assert err <= bar, err
    del g, x, b, u, sigma
    gc.collect()
