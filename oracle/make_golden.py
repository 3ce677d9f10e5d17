"""Write the oracle's solutions of the benchmark workloads to tests/golden/.

TEST INFRASTRUCTURE ONLY.  Calls nothing but the oracle (``oracle/``) and the
seeded input generators (``paper_1711_04060_amd/inputs.py``, which hold none
of the method's arithmetic).  The GPU parity tests compare the library's
results with these files where the oracle cannot afford a whole solve at test
time.

Cases (each one file ``tests/golden/oracle_<case>.npz``):

  membrane97   Sec. 4, Table 2 loop on the 97^3 membrane workload (the PF
               nonlinear solve: Fermi update of Eq. (1), PF1 of Eq. (12),
               PF2 of Eq. (13), relaxation), outer max-norm 1e-11, BiCGSTAB
               (Table 3) 1e-13.  Stored: phi on every second node per axis.
  sphere193    The 193^3 dielectric-sphere Poisson system, Jacobi-BiCGSTAB
               (Table 3) to relative residual 1e-13.  Stored: x on every
               fourth node per axis.
  bias33_<m>   The 33^3 membrane with bias m of the 16-point sweep
               (-150..+150 mV on the -z face), Table 2 loop to 1e-11,
               BiCGSTAB 1e-13.  Stored: phi on every second node per axis.
  batch64      The 64 linearised Poisson-Boltzmann systems (33^3..129^3),
               each Jacobi-BiCGSTAB (Table 3) to relative residual 1e-13.
               Stored: each x on every (n-1)/8-th node per axis (9^3 nodes).

Every file also holds the whole vector's L2 norm, the iteration counts, the
oracle's wall time and the host it ran on.

    python -m oracle.make_golden membrane97
    python -m oracle.make_golden sphere193
    python -m oracle.make_golden bias33 [first last]
    python -m oracle.make_golden batch64
"""
from __future__ import annotations

import os
import platform
import subprocess
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_1711_04060_amd import inputs  # noqa: E402

GOLDEN = os.path.join(ROOT, "tests", "golden")

# tolerances of the stored solutions
OUTER_TOL = 1e-11
LIN_TOL = 1e-13
STRIDE = {"membrane97": 2, "sphere193": 4, "bias33": 2}


def subsample(v: np.ndarray, shape: tuple, stride: int) -> np.ndarray:
    """Every stride-th node along each axis; shape is (nz, ny, nx)."""
    return np.ascontiguousarray(v.reshape(shape)[::stride, ::stride, ::stride]).ravel()


def host_name() -> str:
    try:
        out = subprocess.run(["lscpu"], capture_output=True, text=True).stdout
        for line in out.splitlines():
            if line.startswith("Model name:"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor() or "unknown"


def _save(name: str, **arrays) -> str:
    os.makedirs(GOLDEN, exist_ok=True)
    path = os.path.join(GOLDEN, f"oracle_{name}.npz")
    tmp = path + ".tmp.npz"
    np.savez(tmp, **arrays)
    os.replace(tmp, path)
    return path


def _nonlinear(prob, tag: str, stride: int) -> str:
    ms = prob.meta["species"]
    sp = oracle.species_from_molar(ms["valence"], ms["radius_A"], ms["bath_M"])
    t0 = time.perf_counter()
    phi, info, _, _ = oracle.nonlinear_solve(prob, prob.fixed_charge, sp, prob.meta["eps_s"], prob.meta["lc_A"],
                                             omega=0.3, outer_tol=OUTER_TOL, max_outer=100000, lin_tol=LIN_TOL)
    secs = time.perf_counter() - t0
    print(f"[golden] {tag}: outer {info['outer_iters']} lin {info['total_lin_iters']} "
          f"delta {info['last_delta']:.3e} {secs:.1f} s", flush=True)
    return _save(tag, x_sub=subsample(phi, prob.shape, stride), shape=np.array(prob.shape, np.int64),
                 stride=np.int64(stride), norm2=np.float64(np.linalg.norm(phi)),
                 outer_tol=np.float64(OUTER_TOL), lin_tol=np.float64(LIN_TOL),
                 outer_iters=np.int64(info["outer_iters"]), lin_iters=np.int64(info["total_lin_iters"]),
                 bias_phi=np.float64(prob.bc_value[4]), seconds=np.float64(secs), host=np.str_(host_name()),
                 command=np.str_(" ".join(["python -m oracle.make_golden"] + sys.argv[1:])))


def membrane97() -> str:
    return _nonlinear(inputs.membrane_pore(97), "membrane97", STRIDE["membrane97"])


def sphere193() -> str:
    p = inputs.sphere_poisson(193)
    t0 = time.perf_counter()
    x, info = oracle.linear_solve(p, None, p.b, tol=LIN_TOL)
    secs = time.perf_counter() - t0
    print(f"[golden] sphere193: iters {info['iters']} rel_res {info['rel_res']:.3e} {secs:.1f} s", flush=True)
    return _save("sphere193", x_sub=subsample(x, p.shape, STRIDE["sphere193"]), shape=np.array(p.shape, np.int64),
                 stride=np.int64(STRIDE["sphere193"]), norm2=np.float64(np.linalg.norm(x)),
                 lin_tol=np.float64(LIN_TOL), lin_iters=np.int64(info["iters"]),
                 rel_res=np.float64(info["rel_res"]), seconds=np.float64(secs), host=np.str_(host_name()),
                 command=np.str_("python -m oracle.make_golden sphere193"))


def bias33(first: int = 0, last: int = 15) -> list:
    vt = inputs.thermal_voltage_mV()
    out = []
    for m, v in enumerate(inputs.bias_sweep_mV()):
        if first <= m <= last:
            prob = inputs.membrane_pore(33, bias_phi=v / vt)
            out.append(_nonlinear(prob, f"bias33_{m:02d}", STRIDE["bias33"]))
    return out


def batch64() -> str:
    probs = inputs.batch_systems()
    arrays = {}
    t0 = time.perf_counter()
    iters = []
    for b, p in enumerate(probs):
        x, info = oracle.linear_solve(p, p.sigma, p.b, tol=LIN_TOL)
        s = (p.nx - 1) // 8
        arrays[f"x_sub_{b:02d}"] = subsample(x, p.shape, s)
        arrays[f"stride_{b:02d}"] = np.int64(s)
        arrays[f"shape_{b:02d}"] = np.array(p.shape, np.int64)
        iters.append(info["iters"])
        print(f"[golden] batch64 member {b}: n {p.nx} iters {info['iters']} rel_res {info['rel_res']:.3e}", flush=True)
    secs = time.perf_counter() - t0
    return _save("batch64", **arrays, members=np.int64(len(probs)), lin_tol=np.float64(LIN_TOL),
                 lin_iters=np.array(iters, np.int64), seconds=np.float64(secs), host=np.str_(host_name()),
                 command=np.str_("python -m oracle.make_golden batch64"))


def main(argv) -> None:
    case = argv[0] if argv else ""
    # the OpenMP build of the same source (identical bits, independent loops
    # in parallel); OMP_NUM_THREADS sets the thread count
    oracle.use_openmp()
    if case == "membrane97":
        print(membrane97())
    elif case == "sphere193":
        print(sphere193())
    elif case == "batch64":
        print(batch64())
    elif case == "bias33":
        lo = int(argv[1]) if len(argv) > 1 else 0
        hi = int(argv[2]) if len(argv) > 2 else 15
        print("\n".join(bias33(lo, hi)))
    else:
        raise SystemExit(__doc__)


if __name__ == "__main__":
    main(sys.argv[1:])
