"""Python binding of the C-ABI in include/pf.h (ctypes; argument marshalling only).

Every function has the name of the C entry point it calls.  Arrays are torch
tensors on the ROCm device (PyTorch provides device memory and streams); all
arithmetic of the hot path runs in the HIP kernels of ``libpf.so``.  There is
no fallback: if the library is missing or cannot be loaded, every call raises.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libpf.so")

PF_OK, PF_ERR_ARG, PF_ERR_ALLOC, PF_ERR_DEVICE = 0, -1, -2, -3
PF_ERR_NOCONV, PF_ERR_BREAKDOWN, PF_ERR_NONFINITE = -4, -5, -6
PF_BC_DIRICHLET, PF_BC_NEUMANN = 0, 1
PF_NODE_SOLVENT, PF_NODE_SOLUTE, PF_NODE_FIXED = 0, 1, 2
PF_FP64, PF_MIXED = 0, 1
PF_STOP_REL2, PF_STOP_ABS_INF = 0, 1

EXPORTS = ("pf_grid_create", "pf_grid_destroy", "pf_lin_opts_default", "pf_linear_solve",
           "pf_residual", "pf_residual_noalloc", "pf_spmv", "pf_spmv_f32", "pf_pf_params_default", "pf_nonlinear_solve",
           "pf_fermi", "pf_linear_solve_batch", "pf_nonlinear_solve_batch", "pf_last_error",
           "pf_set_launch", "pf_timing_enable", "pf_timing_read", "pf_coulomb",
           "pf_iface_params_default", "pf_interface_setup", "pf_site_model", "pf_site_fill",
           "pf_stream_probe")


class pf_grid_desc(C.Structure):
    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32), ("h", C.c_double),
                ("eps", C.c_void_p), ("node_type", C.c_void_p), ("fixed_charge", C.c_void_p),
                ("fixed_value", C.c_void_p), ("bc_phi", C.c_int32 * 6), ("bc_value", C.c_double * 6),
                ("bc_psi", C.c_int32 * 6), ("stream", C.c_void_p)]


class pf_lin_opts(C.Structure):
    _fields_ = [("rel_tol", C.c_double), ("max_iter", C.c_int32), ("precision", C.c_int32),
                ("inner_tol", C.c_double), ("max_refine", C.c_int32), ("check_every", C.c_int32),
                ("stop_rule", C.c_int32)]


class pf_lin_info(C.Structure):
    _fields_ = [("iters", C.c_int32), ("refinements", C.c_int32), ("restarts", C.c_int32),
                ("rel_res", C.c_double), ("seconds", C.c_double), ("status", C.c_int32),
                ("max_res", C.c_double), ("fp64_fallback", C.c_int32)]


class pf_pf_params(C.Structure):
    _fields_ = [("n_species", C.c_int32), ("valence", C.c_void_p), ("radius", C.c_void_p),
                ("bath_molar", C.c_void_p), ("steric", C.c_int32), ("lc", C.c_double),
                ("eps_s", C.c_double), ("kB", C.c_double), ("T", C.c_double), ("e", C.c_double),
                ("eps0", C.c_double), ("NA", C.c_double), ("length_unit_A", C.c_double),
                ("omega", C.c_double), ("outer_tol", C.c_double), ("max_outer", C.c_int32),
                ("warm_start", C.c_int32), ("lin", pf_lin_opts), ("rhs_extra", C.c_void_p)]


class pf_iface_params(C.Structure):
    _fields_ = [("n_charges", C.c_int32), ("charges", C.c_void_p), ("lambda_", C.c_double),
                ("eps_m", C.c_double), ("eps_s", C.c_double), ("lin", pf_lin_opts)]


class pf_site_params(C.Structure):
    _fields_ = [("n_sites", C.c_int32), ("site_xyz", C.c_void_p), ("site_radius", C.c_void_p),
                ("site_valence", C.c_void_p), ("occupied", C.c_void_p), ("n_atoms", C.c_int32),
                ("atoms", C.c_void_p), ("eps_p", C.c_double), ("eps_b", C.c_double), ("V_sites", C.c_double)]


class pf_nl_info(C.Structure):
    _fields_ = [("outer_iters", C.c_int32), ("total_lin_iters", C.c_int32),
                ("last_delta", C.c_double), ("seconds", C.c_double), ("status", C.c_int32)]


class PfError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{msg} (pf_status {code})")
        self.code = code


_lib = None


def load():
    """Load libpf.so (built in-tree by ``paper_1711_04060_amd.build``)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_1711_04060_amd.build`")
        lib = C.CDLL(LIB_PATH)
        P, I32, D = C.c_void_p, C.c_int32, C.c_double
        lib.pf_grid_create.argtypes = [C.POINTER(pf_grid_desc), C.POINTER(C.c_void_p)]
        lib.pf_grid_destroy.argtypes = [P]
        lib.pf_grid_destroy.restype = None
        lib.pf_lin_opts_default.argtypes = [C.POINTER(pf_lin_opts)]
        lib.pf_lin_opts_default.restype = None
        lib.pf_linear_solve.argtypes = [P, P, P, P, C.POINTER(pf_lin_opts), C.POINTER(pf_lin_info)]
        lib.pf_residual.argtypes = [P, P, P, P, C.POINTER(D), P]
        lib.pf_residual_noalloc.argtypes = [P, P, P, P, C.POINTER(D), P]
        lib.pf_stream_probe.argtypes = [I32, I32, C.c_int64, C.POINTER(P), I32, I32, P, C.POINTER(D)]
        lib.pf_spmv.argtypes = [P, P, P, P, I32]
        lib.pf_spmv_f32.argtypes = [P, P, P, P, I32]
        lib.pf_pf_params_default.argtypes = [C.POINTER(pf_pf_params)]
        lib.pf_pf_params_default.restype = None
        lib.pf_nonlinear_solve.argtypes = [P, C.POINTER(pf_pf_params), P, P, P, C.POINTER(pf_nl_info)]
        lib.pf_fermi.argtypes = [P, C.POINTER(pf_pf_params), P, P, P, P, P]
        lib.pf_linear_solve_batch.argtypes = [I32, P, P, P, P, C.POINTER(pf_lin_opts), P]
        lib.pf_nonlinear_solve_batch.argtypes = [I32, P, P, P, P]
        lib.pf_last_error.argtypes = []
        lib.pf_last_error.restype = C.c_char_p
        lib.pf_set_launch.argtypes = [I32, I32, I32, I32]
        lib.pf_timing_enable.argtypes = [I32, I32]
        lib.pf_timing_read.argtypes = [I32, C.POINTER(C.c_int64), C.POINTER(D), C.POINTER(D)]
        lib.pf_coulomb.argtypes = [P, P, C.c_int64, P, I32, D, P, P]
        lib.pf_iface_params_default.argtypes = [C.POINTER(pf_iface_params)]
        lib.pf_iface_params_default.restype = None
        lib.pf_interface_setup.argtypes = [P, C.POINTER(pf_iface_params), P, P, P, C.POINTER(pf_lin_info)]
        lib.pf_site_model.argtypes = [C.POINTER(pf_pf_params), C.POINTER(pf_site_params), P, P, P, P, P]
        lib.pf_site_fill.argtypes = [I32, I32, I32, D, C.POINTER(pf_site_params), P, P, P,
                                     C.POINTER(C.c_int64), P]
        for name in EXPORTS:
            if name not in ("pf_grid_destroy", "pf_lin_opts_default", "pf_pf_params_default", "pf_last_error",
                            "pf_iface_params_default"):
                getattr(lib, name).restype = C.c_int32
        _lib = lib
    return _lib


def pf_last_error() -> str:
    return load().pf_last_error().decode()


def _check(code, what, allow=()):
    if code != PF_OK and code not in allow:
        raise PfError(code, f"{what}: {pf_last_error()}")
    return code


def _ptr(t, dtype=None, n=None):
    """Device pointer of a contiguous CUDA/ROCm tensor (None -> NULL)."""
    if t is None:
        return None
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError("expected a device tensor")
    if not t.is_contiguous():
        raise ValueError("tensor must be contiguous")
    if dtype is not None and t.dtype != dtype:
        raise TypeError(f"expected {dtype}, got {t.dtype}")
    if n is not None and t.numel() != n:
        raise ValueError(f"expected {n} elements, got {t.numel()}")
    return C.c_void_p(t.data_ptr())


class Grid:
    """Owns one pf_grid handle."""

    def __init__(self, handle, nx, ny, nz, h):
        self.handle, self.nx, self.ny, self.nz, self.h = handle, nx, ny, nz, h
        self.N = nx * ny * nz

    def __del__(self):
        try:
            pf_grid_destroy(self)
        except Exception:
            pass


def pf_grid_create(nx, ny, nz, h, eps, node_type=None, fixed_charge=None, fixed_value=None,
                   bc_phi=(0,) * 6, bc_value=(0.0,) * 6, bc_psi=(0,) * 6, stream=None) -> Grid:
    import torch
    N = nx * ny * nz
    d = pf_grid_desc()
    d.nx, d.ny, d.nz, d.h = int(nx), int(ny), int(nz), float(h)
    d.eps = _ptr(eps, torch.float64, N)
    d.node_type = _ptr(node_type, torch.uint8, N)
    d.fixed_charge = _ptr(fixed_charge, torch.float64, N)
    d.fixed_value = _ptr(fixed_value, torch.float64, N)
    for f in range(6):
        d.bc_phi[f], d.bc_value[f], d.bc_psi[f] = int(bc_phi[f]), float(bc_value[f]), int(bc_psi[f])
    d.stream = None if stream is None else C.c_void_p(stream)
    h_out = C.c_void_p()
    _check(load().pf_grid_create(C.byref(d), C.byref(h_out)), "pf_grid_create")
    return Grid(h_out, nx, ny, nz, h)


def pf_grid_destroy(g: Grid):
    if g is not None and g.handle:
        load().pf_grid_destroy(g.handle)
        g.handle = None


def pf_lin_opts_default(**kw) -> pf_lin_opts:
    o = pf_lin_opts()
    load().pf_lin_opts_default(C.byref(o))
    for k, v in kw.items():
        setattr(o, k, v)
    return o


def _info(s):
    return {name: getattr(s, name) for name, _ in s._fields_}


def pf_linear_solve(g: Grid, sigma, b, x, opts: pf_lin_opts | None = None, check=True) -> dict:
    import torch
    info = pf_lin_info()
    code = load().pf_linear_solve(g.handle, _ptr(sigma, torch.float64, g.N), _ptr(b, torch.float64, g.N),
                                  _ptr(x, torch.float64, g.N), None if opts is None else C.byref(opts),
                                  C.byref(info))
    if check:
        _check(code, "pf_linear_solve")
    return _info(info)


def pf_residual(g: Grid, sigma, b, x, r=None) -> float:
    import torch
    rel = C.c_double()
    _check(load().pf_residual(g.handle, _ptr(sigma, torch.float64, g.N), _ptr(b, torch.float64, g.N),
                              _ptr(x, torch.float64, g.N), C.byref(rel), _ptr(r, torch.float64, g.N)),
           "pf_residual")
    return rel.value


def pf_residual_noalloc(g: Grid, sigma, b, x, r) -> float:
    """pf_residual without any allocation (scratch in a static device array); r is required."""
    import torch
    rel = C.c_double()
    _check(load().pf_residual_noalloc(g.handle, _ptr(sigma, torch.float64, g.N), _ptr(b, torch.float64, g.N),
                                      _ptr(x, torch.float64, g.N), C.byref(rel), _ptr(r, torch.float64, g.N)),
           "pf_residual_noalloc")
    return rel.value


STREAM_MIX = {0: (1, 1), 1: (3, 1), 2: (7, 4)}   # pf_stream_probe kinds: (inputs, outputs)


def pf_stream_probe(kind, width, sets, reps=30, stream=None):
    """Mean launch time (us) of the streaming probe over `sets` lists of
    device FP64 tensors (inputs first, then outputs), all of one length."""
    import torch
    r, w = STREAM_MIX[kind]
    flat = [t for st in sets for t in st]
    n = flat[0].numel()
    if any(len(st) != r + w for st in sets) or any(t.numel() != n or t.dtype != torch.float64 for t in flat):
        raise ValueError("each set needs %d inputs and %d outputs of equal length" % (r, w))
    arr = (C.c_void_p * len(flat))(*[t.data_ptr() for t in flat])
    us = C.c_double()
    st = None if stream is None else C.c_void_p(stream.cuda_stream)
    _check(load().pf_stream_probe(int(kind), int(width), n, arr, len(sets), int(reps), st, C.byref(us)),
           "pf_stream_probe")
    return us.value


def pf_spmv(g: Grid, sigma, x, y, jacobi: int = 0):
    import torch
    _check(load().pf_spmv(g.handle, _ptr(sigma, torch.float64, g.N), _ptr(x, torch.float64, g.N),
                          _ptr(y, torch.float64, g.N), int(jacobi)), "pf_spmv")


def pf_spmv_f32(g: Grid, sigma, x, y, jacobi: int = 1):
    import torch
    _check(load().pf_spmv_f32(g.handle, _ptr(sigma, torch.float64, g.N), _ptr(x, torch.float32, g.N),
                              _ptr(y, torch.float32, g.N), int(jacobi)), "pf_spmv_f32")


class Params:
    """pf_pf_params plus the host species arrays it points to."""

    def __init__(self, valence, radius_A, bath_molar, **kw):
        self.valence = np.ascontiguousarray(valence, np.float64)
        self.radius = np.ascontiguousarray(radius_A, np.float64)
        self.bath = np.ascontiguousarray(bath_molar, np.float64)
        p = pf_pf_params()
        load().pf_pf_params_default(C.byref(p))
        p.n_species = len(self.valence)
        p.valence = self.valence.ctypes.data_as(C.c_void_p)
        p.radius = self.radius.ctypes.data_as(C.c_void_p)
        p.bath_molar = self.bath.ctypes.data_as(C.c_void_p)
        lin = kw.pop("lin", None)
        self.rhs_extra = kw.pop("rhs_extra", None)   # device tensor kept alive with the params
        if self.rhs_extra is not None:
            p.rhs_extra = _ptr(self.rhs_extra)
        for k, v in kw.items():
            setattr(p, k, v)
        if lin:
            for k, v in lin.items():
                setattr(p.lin, k, v)
        self.c = p


def pf_pf_params_default(valence, radius_A, bath_molar, **kw) -> Params:
    return Params(valence, radius_A, bath_molar, **kw)


def pf_nonlinear_solve(g: Grid, p: Params, phi, conc=None, steric=None, check=True) -> dict:
    import torch
    info = pf_nl_info()
    nsp = p.c.n_species
    code = load().pf_nonlinear_solve(g.handle, C.byref(p.c), _ptr(phi, torch.float64, g.N),
                                     _ptr(conc, torch.float64, nsp * g.N), _ptr(steric, torch.float64, g.N),
                                     C.byref(info))
    if check:
        _check(code, "pf_nonlinear_solve")
    return _info(info)


def pf_fermi(g: Grid, p: Params, phi, rho_hat=None, sigma=None, conc=None, steric=None):
    import torch
    nsp = p.c.n_species
    _check(load().pf_fermi(g.handle, C.byref(p.c), _ptr(phi, torch.float64, g.N),
                           _ptr(rho_hat, torch.float64, g.N), _ptr(sigma, torch.float64, g.N),
                           _ptr(conc, torch.float64, nsp * g.N), _ptr(steric, torch.float64, g.N)),
           "pf_fermi")


def _ptr_array(items, fn):
    arr = (C.c_void_p * len(items))()
    for i, t in enumerate(items):
        v = fn(i, t)
        arr[i] = None if v is None else (v.value if isinstance(v, C.c_void_p) else v)
    return arr


def pf_linear_solve_batch(grids, sigmas, bs, xs, opts: pf_lin_opts | None = None, check=True):
    import torch
    n = len(grids)
    G = _ptr_array(grids, lambda i, g: g.handle)
    Sg = _ptr_array(sigmas if sigmas is not None else [None] * n,
                    lambda i, s: _ptr(s, torch.float64, grids[i].N))
    Bv = _ptr_array(bs, lambda i, b: _ptr(b, torch.float64, grids[i].N))
    Xv = _ptr_array(xs, lambda i, x: _ptr(x, torch.float64, grids[i].N))
    infos = (pf_lin_info * n)()
    code = load().pf_linear_solve_batch(n, G, Sg, Bv, Xv, None if opts is None else C.byref(opts), infos)
    if check:
        _check(code, "pf_linear_solve_batch")
    return [_info(infos[i]) for i in range(n)]


def pf_nonlinear_solve_batch(grids, params, phis, check=True):
    import torch
    n = len(grids)
    G = _ptr_array(grids, lambda i, g: g.handle)
    Pv = _ptr_array(params, lambda i, p: C.cast(C.pointer(p.c), C.c_void_p))
    Xv = _ptr_array(phis, lambda i, x: _ptr(x, torch.float64, grids[i].N))
    infos = (pf_nl_info * n)()
    code = load().pf_nonlinear_solve_batch(n, G, Pv, Xv, infos)
    if check:
        _check(code, "pf_nonlinear_solve_batch")
    return [_info(infos[i]) for i in range(n)]


def pf_set_launch(strip=0, zdepth=0, threads=0, pipeline=0):
    _check(load().pf_set_launch(int(strip), int(zdepth), int(threads), int(pipeline)), "pf_set_launch")


def pf_timing_enable(enable=1, sample=8):
    _check(load().pf_timing_enable(int(enable), int(sample)), "pf_timing_enable")


TIMING_SPMV_FP64, TIMING_SPMV_FP32 = 2, 3   # pf_timing_read kinds of the isolated products
TIMING_BATCH_FP64, TIMING_BATCH_FP32 = 4, 5  # batched BiCGSTAB step A


def pf_timing_read(kind=PF_FP64):
    """kind: PF_FP64 / PF_MIXED (BiCGSTAB step A), TIMING_SPMV_FP64 / TIMING_SPMV_FP32,
    TIMING_BATCH_FP64 / TIMING_BATCH_FP32."""
    n, ms, by = C.c_int64(), C.c_double(), C.c_double()
    _check(load().pf_timing_read(int(kind), C.byref(n), C.byref(ms), C.byref(by)), "pf_timing_read")
    return dict(launches=n.value, mean_ms=ms.value, bytes=by.value)


def grid_from_problem(prob, device="cuda", stream=None) -> Grid:
    """Upload an inputs.Problem's fields and create its grid."""
    import torch
    t = lambda a, dt: None if a is None else torch.as_tensor(np.ascontiguousarray(a), dtype=dt, device=device)
    return pf_grid_create(prob.nx, prob.ny, prob.nz, prob.h, t(prob.eps, torch.float64),
                          t(prob.node_type, torch.uint8), t(prob.fixed_charge, torch.float64),
                          t(prob.fixed_value, torch.float64), prob.bc_phi, prob.bc_value, prob.bc_psi,
                          stream)


def params_for(prob, lc=None, eps_s=None, **kw) -> Params:
    """Parameters of the membrane workload (species in prob.meta)."""
    sp = prob.meta["species"]
    return Params(sp["valence"], sp["radius_A"], sp["bath_M"],
                  lc=prob.meta.get("lc_A", 0.0) if lc is None else lc,
                  eps_s=prob.meta.get("eps_s", 78.45) if eps_s is None else eps_s, **kw)


# ------------------------------------------- singular-charge decomposition

def pf_coulomb(pts, charges, scale, out, dirs=None, stream=None):
    """phi* of Eq. (5) (scale = lambda / (4 pi eps_m)) or its derivative along
    face direction dirs[p] (int8, 0..5; 6 = potential) at points pts [n, 3];
    charges [M, 4] = x, y, z, valence.  All device tensors; `stream` is a
    torch stream (None = the default stream)."""
    import torch
    n = out.numel()
    M = charges.numel() // 4
    if pts.numel() != 3 * n or charges.numel() != 4 * M:
        raise ValueError("pts must be [n, 3] and charges [M, 4]")
    st = None if stream is None else C.c_void_p(stream.cuda_stream)
    _check(load().pf_coulomb(_ptr(pts, torch.float64), _ptr(dirs, torch.int8, n), n,
                             _ptr(charges, torch.float64) if M else None, M, float(scale),
                             _ptr(out, torch.float64), st), "pf_coulomb")


def pf_iface_params_default(**kw) -> pf_iface_params:
    p = pf_iface_params()
    load().pf_iface_params_default(C.byref(p))
    lin = kw.pop("lin", None)
    for k, v in kw.items():
        setattr(p, "lambda_" if k == "lam" else k, v)
    if lin:
        for k, v in lin.items():
            setattr(p.lin, k, v)
    return p


def pf_interface_setup(g: Grid, charges, lam, eps_m, eps_s, b_if, phi_reg=None, phi_lap=None,
                       lin=None, check=True) -> dict:
    """Interface terms of the decomposition (Sec. 3): fills b_if (and phi_reg
    = phi* + phi^L on Omega_m, phi_lap = the Laplace solution if given).
    charges: device [M, 4] in grid length units from node (0, 0, 0)."""
    import torch
    M = 0 if charges is None else charges.numel() // 4
    p = pf_iface_params_default(lam=float(lam), eps_m=float(eps_m), eps_s=float(eps_s), lin=lin)
    p.n_charges = M
    p.charges = _ptr(charges, torch.float64) if M else None
    info = pf_lin_info()
    code = load().pf_interface_setup(g.handle, C.byref(p), _ptr(b_if, torch.float64, g.N),
                                     _ptr(phi_reg, torch.float64, g.N), _ptr(phi_lap, torch.float64, g.N),
                                     C.byref(info))
    if check:
        _check(code, "pf_interface_setup")
    return _info(info)


# ------------------------------------------- filter-region atomic model

class Sites:
    """pf_site_params plus the arrays it points to.  atoms: device tensor
    [M, 4]; the site arrays are host arrays."""

    def __init__(self, xyz, radius, valence, occupied, atoms, eps_p=20.0, eps_b=10.0, V_sites=1.0):
        import torch
        self.xyz = np.ascontiguousarray(xyz, np.float64).reshape(-1, 3)
        self.radius = np.ascontiguousarray(radius, np.float64).ravel()
        self.valence = np.ascontiguousarray(valence, np.float64).ravel()
        self.occupied = np.ascontiguousarray(occupied, np.int32).ravel()
        self.atoms = atoms
        c = pf_site_params()
        c.n_sites = len(self.xyz)
        c.site_xyz = self.xyz.ctypes.data_as(C.c_void_p)
        c.site_radius = self.radius.ctypes.data_as(C.c_void_p)
        c.site_valence = self.valence.ctypes.data_as(C.c_void_p)
        c.occupied = self.occupied.ctypes.data_as(C.c_void_p)
        c.n_atoms = 0 if atoms is None else atoms.numel() // 4
        c.atoms = _ptr(atoms, torch.float64) if c.n_atoms else None
        c.eps_p, c.eps_b, c.V_sites = float(eps_p), float(eps_b), float(V_sites)
        self.c = c

    @property
    def n(self):
        return self.c.n_sites


def pf_site_model(p: Params, sites: Sites, stream=None):
    """Eqs. (19)-(20) at every site: numpy (phi_b, S_b, psi_b, conc_b[n_sites, n_species])."""
    n, nsp = sites.n, p.c.n_species
    phi, S, psi = np.empty(n), np.empty(n), np.empty(n)
    conc = np.empty((n, nsp))
    st = None if stream is None else C.c_void_p(stream.cuda_stream)
    P = lambda a: a.ctypes.data_as(C.c_void_p)
    _check(load().pf_site_model(C.byref(p.c), C.byref(sites.c), P(phi), P(S), P(psi), P(conc), st),
           "pf_site_model")
    return phi, S, psi, conc


def pf_site_fill(nx, ny, nz, h, sites: Sites, phi_b, node_type, fixed_value, stream=None) -> int:
    """Mark the filter region: SOLVENT nodes inside a site sphere become FIXED
    with that site's phi_b (device node_type uint8 and fixed_value float64,
    both updated in place).  Returns the number of nodes marked."""
    import torch
    N = nx * ny * nz
    ph = np.ascontiguousarray(phi_b, np.float64)
    marked = C.c_int64()
    st = None if stream is None else C.c_void_p(stream.cuda_stream)
    _check(load().pf_site_fill(int(nx), int(ny), int(nz), float(h), C.byref(sites.c), ph.ctypes.data_as(C.c_void_p),
                               _ptr(node_type, torch.uint8, N), _ptr(fixed_value, torch.float64, N),
                               C.byref(marked), st), "pf_site_fill")
    return marked.value
