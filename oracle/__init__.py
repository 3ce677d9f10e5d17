"""Serial FP64 CPU oracle for the Poisson-Fermi hot path (arXiv:1711.04060).

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` may import this package.  The product library
(``paper_1711_04060_amd``) never imports, links or calls it, and the two share
no code: the arithmetic lives in ``pfo.c`` (plain loops, sequential sums), and
this module only marshals numpy arrays and converts the physical constants of
Table 1 into the dimensionless parameters the C code takes.

Functions follow the paper:
  * ``assemble`` / ``dia_matvec``: the 7-point FD operator stored as the seven
    diagonals A0..A6 (Sec. 4, the diagonal format described before Table 2).
  * ``bicgstab`` / ``linear_solve``: Jacobi-BiCGSTAB (Sec. 4, Table 3).
  * ``fermi`` / ``steric_root``: Fermi-like distribution and steric potential
    (Sec. 2, Eq. (1)), by bisection.
  * ``nonlinear_solve``: the sequential PF solver (Sec. 4, Table 2) with the
    PF1/PF2 split of Eqs. (12)-(14) and the inexact-Newton linearisation of
    Eq. (11); ``rhs_extra`` adds the interface terms to every PF2 solve.
  * ``coulomb`` / ``smib_rhs`` / ``interface``: the singular-charge
    decomposition of Sec. 3 -- phi* of Eq. (5), the Laplace problem of
    Eqs. (9)-(10), the flux jump of Eq. (8) and the right-hand-side terms of
    the SMIB rows, Eqs. (17)-(18).
"""
from __future__ import annotations

import ctypes as C
import math
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "pfo.c")
_LIB = os.path.join(_HERE, "liboracle.so")

DIRICHLET, NEUMANN = 0, 1
SOLVENT, SOLUTE, FIXED = 0, 1, 2

OK, EARG, ENOMEM, ENOCONV, EBREAKDOWN, ENONFINITE = 0, -1, -2, -4, -5, -6


_LIB_OMP = os.path.join(_HERE, "liboracle_omp.so")
_use_omp = False

_CFLAGS = ["-O2", "-ffp-contract=off", "-fno-fast-math", "-std=c11", "-fPIC", "-shared", "-Wall",
           "-Wno-unused-function", "-Wno-maybe-uninitialized"]


def build(force: bool = True, openmp: bool = False) -> str:
    """Compile the oracle with gcc (plain FP64, no contraction, no fast-math).

    openmp=True builds liboracle_omp.so from the same source with -fopenmp:
    only loops with independent iterations run in parallel and every sum
    stays sequential, so it returns the same bits as the serial library
    (checked by a CPU test).  It serves the golden-file script only."""
    lib = _LIB_OMP if openmp else _LIB
    if force or not os.path.exists(lib) or os.path.getmtime(lib) < os.path.getmtime(_SRC):
        extra = ["-fopenmp"] if openmp else ["-Wno-unknown-pragmas"]
        cmd = ["gcc", *_CFLAGS, *extra, "-o", lib, _SRC, "-lm"]
        subprocess.run(cmd, check=True)
    return lib


def use_openmp() -> None:
    """Load the OpenMP build (before the first oracle call of the process)."""
    global _use_omp
    if _lib is not None and not _use_omp:
        raise RuntimeError("the serial oracle library is already loaded")
    _use_omp = True


class _Grid(C.Structure):
    _fields_ = [("nx", C.c_int), ("ny", C.c_int), ("nz", C.c_int), ("h", C.c_double),
                ("eps", C.c_void_p), ("type", C.c_void_p), ("fixed_value", C.c_void_p),
                ("bc", C.c_int * 6), ("bc_value", C.c_double * 6)]


class _LinInfo(C.Structure):
    _fields_ = [("iters", C.c_int), ("restarts", C.c_int), ("rel_res", C.c_double),
                ("bnorm", C.c_double), ("max_res", C.c_double)]


class _Species(C.Structure):
    _fields_ = [("nsp", C.c_int), ("z", C.c_void_p), ("v", C.c_void_p), ("cb", C.c_void_p),
                ("steric", C.c_int), ("lam", C.c_double)]


class _NlOpts(C.Structure):
    _fields_ = [("eps_s", C.c_double), ("lc", C.c_double), ("omega", C.c_double),
                ("outer_tol", C.c_double), ("max_outer", C.c_int), ("lin_tol", C.c_double),
                ("lin_maxit", C.c_int), ("warm_start", C.c_int), ("bc_psi", C.c_int * 6),
                ("rhs_extra", C.c_void_p)]


class _Sites(C.Structure):
    _fields_ = [("n_sites", C.c_int), ("xyz", C.c_void_p), ("radius", C.c_void_p), ("valence", C.c_void_p),
                ("occupied", C.c_void_p), ("n_atoms", C.c_int), ("atoms", C.c_void_p), ("eps_p", C.c_double),
                ("eps_b", C.c_double), ("V_sites", C.c_double)]


class _NlInfo(C.Structure):
    _fields_ = [("outer_iters", C.c_int), ("total_lin_iters", C.c_int),
                ("last_delta", C.c_double)]


_lib = None


def _L():
    global _lib
    if _lib is None:
        path = _LIB_OMP if _use_omp else _LIB
        if not os.path.exists(path) or os.path.getmtime(path) < os.path.getmtime(_SRC):
            build(force=False, openmp=_use_omp)
        lib = C.CDLL(path)
        P, I, D, S = C.c_void_p, C.c_int, C.c_double, C.c_size_t
        lib.pfo_dirichlet.argtypes = [C.POINTER(_Grid), I, P, P, P]
        lib.pfo_assemble.argtypes = [I, I, I, D, P, P, P, P, P]
        lib.pfo_dia_matvec.argtypes = [I, I, I, P, P, P]
        lib.pfo_dia_matvec.restype = None
        lib.pfo_bicgstab.argtypes = [I, I, I, P, P, P, P, P, D, I, C.POINTER(_LinInfo)]
        lib.pfo_linear_solve.argtypes = [C.POINTER(_Grid), P, P, P, D, I, C.POINTER(_LinInfo)]
        lib.pfo_linear_solve_rule.argtypes = [C.POINTER(_Grid), P, P, P, D, I, I, C.POINTER(_LinInfo)]
        lib.pfo_fermi.argtypes = [S, P, P, C.POINTER(_Species), P, P, P, P]
        lib.pfo_steric_root.argtypes = [D, C.POINTER(_Species)]
        lib.pfo_steric_root.restype = D
        lib.pfo_nonlinear_solve.argtypes = [C.POINTER(_Grid), P, C.POINTER(_Species),
                                            C.POINTER(_NlOpts), P, P, P, C.POINTER(_NlInfo)]
        lib.pfo_coulomb.argtypes = [S, P, P, I, P, D, P]
        lib.pfo_coulomb.restype = None
        lib.pfo_smib_rhs.argtypes = [C.POINTER(_Grid), D, D, P, P]
        lib.pfo_interface.argtypes = [C.POINTER(_Grid), I, P, D, D, D, D, I, P, P, P, C.POINTER(_LinInfo)]
        lib.pfo_bulk_void.argtypes = [C.POINTER(_Species)]
        lib.pfo_bulk_void.restype = D
        lib.pfo_site_model.argtypes = [C.POINTER(_Sites), C.POINTER(_Species), P, P, P, P]
        lib.pfo_site_fill.argtypes = [I, I, I, D, C.POINTER(_Sites), P, P, P]
        lib.pfo_site_fill.restype = C.c_long
        _lib = lib
    return _lib


def _p(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


class OracleError(RuntimeError):
    def __init__(self, code, what):
        super().__init__(f"{what}: oracle status {code}")
        self.code = code


# ------------------------------------------------------------------ problem

@dataclass
class Grid:
    """Host-side description of a grid problem (duck-typed: any object with
    these attributes works)."""
    nx: int
    ny: int
    nz: int
    h: float
    eps: np.ndarray
    node_type: np.ndarray | None = None
    fixed_value: np.ndarray | None = None
    bc_phi: tuple = (DIRICHLET,) * 6
    bc_value: tuple = (0.0,) * 6


def _grid(g, keep):
    eps = _f64(g.eps).ravel()
    typ = None if getattr(g, "node_type", None) is None else np.ascontiguousarray(g.node_type, dtype=np.uint8).ravel()
    fv = None if getattr(g, "fixed_value", None) is None else _f64(g.fixed_value).ravel()
    keep.extend([eps, typ, fv])
    s = _Grid()
    s.nx, s.ny, s.nz, s.h = int(g.nx), int(g.ny), int(g.nz), float(g.h)
    s.eps, s.type, s.fixed_value = _p(eps), _p(typ), _p(fv)
    for f in range(6):
        s.bc[f] = int(g.bc_phi[f])
        s.bc_value[f] = float(g.bc_value[f])
    return s


def dirichlet(g, system=0, bc_psi=(DIRICHLET,) * 6):
    """Dirichlet mask and values: system 0 = potential, 1 = PF1 density (Eq. (14))."""
    keep = []
    s = _grid(g, keep)
    N = g.nx * g.ny * g.nz
    isd = np.zeros(N, np.uint8)
    val = np.zeros(N)
    bp = (C.c_int * 6)(*[int(b) for b in bc_psi])
    st = _L().pfo_dirichlet(C.byref(s), system, C.cast(bp, C.c_void_p), _p(isd), _p(val))
    if st:
        raise OracleError(st, "dirichlet")
    return isd, val


def assemble(nx, ny, nz, h, coef, sigma, is_dir, bc=(DIRICHLET,) * 6):
    """Seven diagonals A[7, N] of (-div coef grad + sigma); identity on Dirichlet rows."""
    N = nx * ny * nz
    coef = _f64(coef).ravel()
    sig = None if sigma is None else _f64(sigma).ravel()
    isd = np.ascontiguousarray(is_dir, dtype=np.uint8).ravel()
    A = np.zeros((7, N))
    bcs = (C.c_int * 6)(*[int(b) for b in bc])
    st = _L().pfo_assemble(nx, ny, nz, float(h), _p(coef), _p(sig), C.cast(bcs, C.c_void_p), _p(isd), _p(A))
    if st:
        raise OracleError(st, "assemble")
    return A


def dia_matvec(nx, ny, nz, A, x):
    A = _f64(A)
    x = _f64(x).ravel()
    y = np.empty_like(x)
    _L().pfo_dia_matvec(nx, ny, nz, _p(A), _p(x), _p(y))
    return y


def bicgstab(nx, ny, nz, A, is_dir, value, b, x0=None, tol=1e-12, maxit=100000, check=True):
    """Right-Jacobi BiCGSTAB (Table 3).  Returns (x, info dict)."""
    N = nx * ny * nz
    A = _f64(A)
    isd = np.ascontiguousarray(is_dir, dtype=np.uint8).ravel()
    val = _f64(value).ravel()
    b = _f64(b).ravel()
    x = np.zeros(N) if x0 is None else _f64(x0).ravel().copy()
    info = _LinInfo()
    st = _L().pfo_bicgstab(nx, ny, nz, _p(A), _p(isd), _p(val), _p(b), _p(x), float(tol), int(maxit), C.byref(info))
    d = dict(status=st, iters=info.iters, restarts=info.restarts, rel_res=info.rel_res, bnorm=info.bnorm)
    if check and st:
        raise OracleError(st, "bicgstab")
    return x, d


def linear_solve(g, sigma, b, x0=None, tol=1e-12, maxit=100000, check=True, rule=0):
    """Assemble + BiCGSTAB for (-div eps grad + sigma) x = b on grid g.
    rule 0: stop on the relative L2 residual; 1: on the absolute max norm (Table 3)."""
    keep = []
    s = _grid(g, keep)
    N = g.nx * g.ny * g.nz
    sig = None if sigma is None else _f64(sigma).ravel()
    b = _f64(b).ravel()
    x = np.zeros(N) if x0 is None else _f64(x0).ravel().copy()
    info = _LinInfo()
    st = _L().pfo_linear_solve_rule(C.byref(s), _p(sig), _p(b), _p(x), float(tol), int(maxit), int(rule),
                                    C.byref(info))
    d = dict(status=st, iters=info.iters, restarts=info.restarts, rel_res=info.rel_res, bnorm=info.bnorm,
             max_res=info.max_res)
    if check and st:
        raise OracleError(st, "linear_solve")
    return x, d


# ------------------------------------------------------------ physics params

# Table 1 constants (SI, eps0 in F/cm as printed) and Avogadro's number,
# which Table 1 does not list.
KB, TEMP, QE, EPS0_F_PER_CM, NA = 1.38e-23, 298.15, 1.602e-19, 8.85e-14, 6.02214076e23


def lambda_length(length_unit_A=1.0, kB=KB, T=TEMP, e=QE, eps0_F_per_cm=EPS0_F_PER_CM):
    """e^2 / (eps0 kB T) in grid length units (Angstrom * length_unit_A)."""
    eps0 = eps0_F_per_cm * 100.0            # F/m
    lam_m = e * e / (eps0 * kB * T)         # metres
    return lam_m * 1e10 / length_unit_A


def molar_to_grid(length_unit_A=1.0, NA_=NA):
    """Multiplier from mol/L to particles per cubed grid length unit."""
    return NA_ * 1e3 * 1e-30 * length_unit_A ** 3


@dataclass
class Species:
    valence: np.ndarray
    radius: np.ndarray     # grid length units
    conc: np.ndarray       # particles per cubed grid length unit
    steric: bool = True
    lam: float = lambda_length()

    @property
    def volume(self):
        return 4.0 * math.pi * np.asarray(self.radius, float) ** 3 / 3.0


def species_from_molar(valence, radius_A, bath_M, steric=True, length_unit_A=1.0):
    return Species(np.asarray(valence, float), np.asarray(radius_A, float) / length_unit_A,
                   np.asarray(bath_M, float) * molar_to_grid(length_unit_A), steric,
                   lambda_length(length_unit_A))


def _species(sp, keep):
    z = _f64(sp.valence)
    v = _f64(sp.volume)
    cb = _f64(sp.conc)
    keep.extend([z, v, cb])
    s = _Species()
    s.nsp, s.z, s.v, s.cb, s.steric, s.lam = len(z), _p(z), _p(v), _p(cb), int(bool(sp.steric)), float(sp.lam)
    return s


def steric_root(phi, sp):
    keep = []
    s = _species(sp, keep)
    return _L().pfo_steric_root(float(phi), C.byref(s))


def fermi(phi, sp, node_type=None, want_conc=True):
    """Eq. (1) at every solvent node.  Returns rho_hat, sigma, conc[nsp, N], S."""
    phi = _f64(phi).ravel()
    N = phi.size
    typ = None if node_type is None else np.ascontiguousarray(node_type, dtype=np.uint8).ravel()
    keep = []
    s = _species(sp, keep)
    rho = np.empty(N)
    sig = np.empty(N)
    conc = np.empty((len(sp.valence), N)) if want_conc else None
    S = np.empty(N)
    st = _L().pfo_fermi(N, _p(phi), _p(typ), C.byref(s), _p(rho), _p(sig), _p(conc), _p(S))
    if st:
        raise OracleError(st, "fermi")
    return rho, sig, conc, S


def nonlinear_solve(g, fixed_charge, sp, eps_s, lc, omega=0.3, outer_tol=1e-8, max_outer=1000,
                    lin_tol=1e-12, lin_maxit=100000, phi0=None, bc_psi=(DIRICHLET,) * 6,
                    want_conc=False, check=True, rhs_extra=None):
    """Table 2: initial PF2 solve, then {Fermi, PF1, PF2, relax} to outer_tol."""
    keep = []
    s = _grid(g, keep)
    N = g.nx * g.ny * g.nz
    spc = _species(sp, keep)
    o = _NlOpts()
    o.eps_s, o.lc, o.omega, o.outer_tol = float(eps_s), float(lc), float(omega), float(outer_tol)
    o.max_outer, o.lin_tol, o.lin_maxit = int(max_outer), float(lin_tol), int(lin_maxit)
    o.warm_start = 0 if phi0 is None else 1
    for f in range(6):
        o.bc_psi[f] = int(bc_psi[f])
    extra = None if rhs_extra is None else _f64(rhs_extra).ravel()
    keep.append(extra)
    o.rhs_extra = _p(extra)
    q = None if fixed_charge is None else _f64(fixed_charge).ravel()
    phi = np.zeros(N) if phi0 is None else _f64(phi0).ravel().copy()
    conc = np.empty((len(sp.valence), N)) if want_conc else None
    S = np.empty(N) if want_conc else None
    info = _NlInfo()
    st = _L().pfo_nonlinear_solve(C.byref(s), _p(q), C.byref(spc), C.byref(o), _p(phi), _p(conc), _p(S), C.byref(info))
    d = dict(status=st, outer_iters=info.outer_iters, total_lin_iters=info.total_lin_iters,
             last_delta=info.last_delta)
    if check and st:
        raise OracleError(st, "nonlinear_solve")
    return phi, d, conc, S


# ------------------------------------------- interface treatment (Sec. 3)

def coulomb(points, charges, scale, dirs=None):
    """phi* of Eq. (5) (``scale`` = lambda / (4 pi eps_m)) or its derivative
    along face direction dirs[p] (0..5 = -x,+x,-y,+y,-z,+z; 6 = potential)
    at points [n, 3]; charges [M, 4] = x, y, z, valence."""
    pts = _f64(points).reshape(-1, 3)
    ch = _f64(charges).reshape(-1, 4)
    d = None if dirs is None else np.ascontiguousarray(dirs, dtype=np.int32).ravel()
    out = np.empty(len(pts))
    _L().pfo_coulomb(len(pts), _p(pts), _p(d), len(ch), _p(ch), float(scale), _p(out))
    return out


def smib_rhs(g, eps_m, eps_s, jump):
    """Right-hand-side terms of the SMIB rows (Eqs. (17)-(18)) for flux jumps
    jump[6, N] on the edges leaving Omega_m (SOLUTE nodes)."""
    keep = []
    s = _grid(g, keep)
    N = g.nx * g.ny * g.nz
    j = _f64(jump).reshape(6, N)
    b = np.zeros(N)
    st = _L().pfo_smib_rhs(C.byref(s), float(eps_m), float(eps_s), _p(j), _p(b))
    if st:
        raise OracleError(st, "smib_rhs")
    return b


def interface(g, charges, lam, eps_m, eps_s, tol=1e-12, maxit=100000):
    """Decomposition of Eq. (5): returns (b_if, phi_reg, phi_lap, info) --
    SMIB right-hand-side terms, phi* + phi^L on Omega_m, the Laplace solution."""
    keep = []
    s = _grid(g, keep)
    N = g.nx * g.ny * g.nz
    ch = _f64(charges).reshape(-1, 4)
    b = np.zeros(N)
    reg = np.zeros(N)
    lap = np.zeros(N)
    info = _LinInfo()
    st = _L().pfo_interface(C.byref(s), len(ch), _p(ch), float(lam), float(eps_m), float(eps_s),
                            float(tol), int(maxit), _p(b), _p(reg), _p(lap), C.byref(info))
    if st:
        raise OracleError(st, "interface")
    return b, reg, lap, dict(iters=info.iters, rel_res=info.rel_res)


# ------------------------------ filter-region atomic model, Eqs. (19)-(20)

def _sites(sites, keep):
    xyz = _f64(sites["xyz"]).reshape(-1, 3)
    rad = _f64(sites["radius"]).ravel()
    val = _f64(sites["valence"]).ravel()
    occ = np.ascontiguousarray(sites["occupied"], dtype=np.int32).ravel()
    atoms = _f64(sites["atoms"]).reshape(-1, 4)
    keep.extend([xyz, rad, val, occ, atoms])
    s = _Sites()
    s.n_sites = len(xyz)
    s.xyz, s.radius, s.valence, s.occupied = _p(xyz), _p(rad), _p(val), _p(occ)
    s.n_atoms, s.atoms = len(atoms), _p(atoms)
    s.eps_p, s.eps_b, s.V_sites = float(sites["eps_p"]), float(sites["eps_b"]), float(sites["V_sites"])
    return s


def bulk_void(sp):
    keep = []
    return _L().pfo_bulk_void(C.byref(_species(sp, keep)))


def site_model(sites, sp):
    """Eqs. (19)-(20) at every site: (phi_b, S_b, psi_b, conc_b[n_sites, nsp])."""
    keep = []
    s = _sites(sites, keep)
    spc = _species(sp, keep)
    n = s.n_sites
    phi, S, psi = np.empty(n), np.empty(n), np.empty(n)
    conc = np.empty((n, len(sp.valence)))
    st = _L().pfo_site_model(C.byref(s), C.byref(spc), _p(phi), _p(S), _p(psi), _p(conc))
    if st:
        raise OracleError(st, "site_model")
    return phi, S, psi, conc


def site_fill(nx, ny, nz, h, sites, phi_b, node_type, fixed_value=None):
    """Filter region: SOLVENT nodes inside a site sphere become FIXED with the
    nearest site's phi_b.  Returns (node_type, fixed_value, marked)."""
    keep = []
    s = _sites(sites, keep)
    typ = np.ascontiguousarray(node_type, dtype=np.uint8).ravel().copy()
    fv = np.zeros(nx * ny * nz) if fixed_value is None else _f64(fixed_value).ravel().copy()
    ph = _f64(phi_b).ravel()
    marked = _L().pfo_site_fill(int(nx), int(ny), int(nz), float(h), C.byref(s), _p(ph), _p(typ), _p(fv))
    if marked < 0:
        raise OracleError(marked, "site_fill")
    return typ, fv, marked
