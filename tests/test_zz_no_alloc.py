"""pf_residual_noalloc against pf_residual, through the C-ABI.

The allocation-free variant runs the same residual kernels with its
partials and sums in the library's static device scratch.  With the grid's
usual launch shape the reduction order is the same, so the residual vector
and the relative residual must equal pf_residual's bit for bit.  Two calls
in a row, the second on a smaller grid, so that the second call finds the
scratch holding the first call's larger partials.  On a grid that never
solved (no workspace allocated, launch shape untuned) the residual vector is
still bit-identical (per-node arithmetic does not depend on the tiling) and
the relative residual agrees to rounding.
"""
import numpy as np
import pytest

from paper_1711_04060_amd import inputs

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _pf():
    from paper_1711_04060_amd import pf
    pf.load()
    return pf


def dev(a):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")


def _case(pf, p, sigma, seed):
    rng = np.random.default_rng(seed)
    x = dev(rng.normal(size=p.N))
    b = dev(p.b if p.b is not None else rng.normal(size=p.N))
    s = None if sigma is None else dev(sigma)
    g = pf.grid_from_problem(p)
    r_ref = torch.full((p.N,), np.nan, dtype=torch.float64, device="cuda")
    r_na = torch.full((p.N,), np.nan, dtype=torch.float64, device="cuda")
    rel_ref = pf.pf_residual(g, s, b, x, r_ref)
    rel_na = pf.pf_residual_noalloc(g, s, b, x, r_na)
    torch.cuda.synchronize()
    assert rel_na == rel_ref, (rel_na, rel_ref)          # same launch shape: same reduction order
    assert torch.equal(r_na, r_ref)
    # a fresh grid (workspace never allocated, launch shape not tuned): the
    # same residual vector; the sum in another order, to rounding
    g2 = pf.grid_from_problem(p)
    r2 = torch.full((p.N,), np.nan, dtype=torch.float64, device="cuda")
    rel2 = pf.pf_residual_noalloc(g2, s, b, x, r2)
    torch.cuda.synchronize()
    assert torch.equal(r2, r_ref)
    assert rel2 == pytest.approx(rel_ref, rel=1e-12)
    return rel_na


def test_noalloc_residual_matches_pf_residual_twice_shrinking():
    pf = _pf()
    big = inputs.batch_systems(n_sys=1, seed_base=4003)[0]     # linearised PB system with sigma
    small = inputs.sphere_poisson(33)
    rel1 = _case(pf, big, big.sigma, 1)
    rel2 = _case(pf, small, None, 2)
    assert np.isfinite(rel1) and np.isfinite(rel2) and rel1 > 0 and rel2 > 0


def test_noalloc_residual_of_a_solution_is_small():
    pf = _pf()
    p = inputs.sphere_poisson(33)
    g = pf.grid_from_problem(p)
    b = dev(p.b)
    x = torch.zeros(p.N, dtype=torch.float64, device="cuda")
    info = pf.pf_linear_solve(g, None, b, x)
    r = torch.empty_like(x)
    assert pf.pf_residual_noalloc(g, None, b, x, r) == pytest.approx(info["rel_res"], rel=1e-12)
    with pytest.raises(pf.PfError) as e:
        pf.pf_residual_noalloc(g, None, b, x, None)
    assert e.value.code == pf.PF_ERR_ARG
