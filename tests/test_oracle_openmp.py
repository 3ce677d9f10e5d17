"""The OpenMP build of the oracle (used only to write the large golden files)
returns the same bits as the serial build: its parallel loops have
independent iterations and every sum stays sequential."""
import os
import subprocess
import sys

import numpy as np

import oracle
from paper_1711_04060_amd import inputs

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

_CHILD = r"""
import sys, numpy as np
sys.path.insert(0, {root!r})
import oracle
from paper_1711_04060_amd import inputs
oracle.use_openmp()
p = inputs.membrane_pore(17, n_charges=40)
ms = p.meta["species"]
sp = oracle.species_from_molar(ms["valence"], ms["radius_A"], ms["bath_M"])
phi, info, _, _ = oracle.nonlinear_solve(p, p.fixed_charge, sp, 78.45, 1.9, outer_tol=1e-6, lin_tol=1e-11)
x, _ = oracle.linear_solve(inputs.sphere_poisson(17), None, inputs.sphere_poisson(17).b, tol=1e-12)
np.save({out!r}, np.concatenate([phi, x, [info["outer_iters"], info["total_lin_iters"]]]))
"""


def test_openmp_build_gives_identical_bits(tmp_path):
    oracle.build(force=False, openmp=True)
    out = str(tmp_path / "omp.npy")
    env = dict(os.environ, OMP_NUM_THREADS="4")
    subprocess.run([sys.executable, "-c", _CHILD.format(root=ROOT, out=out)], check=True, env=env, timeout=600)
    got = np.load(out)
    p = inputs.membrane_pore(17, n_charges=40)
    ms = p.meta["species"]
    sp = oracle.species_from_molar(ms["valence"], ms["radius_A"], ms["bath_M"])
    phi, info, _, _ = oracle.nonlinear_solve(p, p.fixed_charge, sp, 78.45, 1.9, outer_tol=1e-6, lin_tol=1e-11)
    q = inputs.sphere_poisson(17)
    x, _ = oracle.linear_solve(q, None, q.b, tol=1e-12)
    ref = np.concatenate([phi, x, [info["outer_iters"], info["total_lin_iters"]]])
    assert np.array_equal(got, ref)
