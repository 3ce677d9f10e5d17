"""Seeded synthetic inputs for the Poisson-Fermi workloads.

This module only builds input fields (geometry, dielectric, node types,
charges spread to nodes, boundary data).  It contains none of the solver's
arithmetic, and both the GPU path and the CPU oracle consume its arrays.

Random numbers come from SplitMix64 (Steele, Lea and Flood, "Fast splittable
pseudorandom number generators", OOPSLA 2014): state advances by the golden
gamma 0x9E3779B97F4A7C15 and each output is the published three-step mix.
A uniform double in [0, 1) is the top 53 bits of an output times 2^-53.

Workloads (the paper's NCX protein structure is not available, so these
stand in for it at the same lateral scale, a 40 A box as in Eq. (4)):

  * ``sphere_poisson(n)``      dielectric sphere (eps 2 in 80) in [-1,1]^3,
                               +-1 point charges in the sphere, Dirichlet 0.
  * ``membrane_pore(n)``       40 A cube, membrane slab |z| <= 10 A (eps 2)
                               with a solvent pore r < 5 A and a charged
                               protein-like shell 5 <= r <= 10 A, four species
                               (Na+, Ca2+, Cl-, water), Dirichlet z faces,
                               Neumann x/y faces (Eq. (4)).
  * ``batch_systems()``        64 linearised-PB systems of seeded sizes.
"""
from __future__ import annotations

import dataclasses
import math
from dataclasses import dataclass, field

import numpy as np

DIRICHLET, NEUMANN = 0, 1
SOLVENT, SOLUTE, FIXED = 0, 1, 2

_GAMMA = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)


def splitmix64(seed: int, n: int, offset: int = 0) -> np.ndarray:
    """Outputs offset..offset+n-1 of the SplitMix64 stream seeded with `seed`."""
    k = np.arange(offset + 1, offset + n + 1, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = np.uint64(seed) + k * _GAMMA
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
        z = z ^ (z >> np.uint64(31))
    return z


def uniform(seed: int, n: int, offset: int = 0) -> np.ndarray:
    """Uniform doubles in [0, 1): top 53 bits of each output times 2^-53."""
    return (splitmix64(seed, n, offset) >> np.uint64(11)).astype(np.float64) * (2.0 ** -53)


class Stream:
    """Sequential reader over one SplitMix64 stream."""

    def __init__(self, seed: int):
        self.seed, self.pos = int(seed), 0

    def take(self, n: int) -> np.ndarray:
        u = uniform(self.seed, n, self.pos)
        self.pos += n
        return u


# Table 1 of the paper (kB, T, e, eps0 in F/cm) plus Avogadro's number, used
# only to turn bath concentrations into the linearised-PB shift of the
# batched workload.
TABLE1 = dict(kB=1.38e-23, T=298.15, e=1.602e-19, eps0_F_per_cm=8.85e-14, NA=6.02214076e23,
              eps_b=10.0, eps_p=20.0, eps_s=78.45, eps_m=2.0)

# Species of the membrane workload: Table 1 radii; bath 100 mM NaCl + 1 mM
# CaCl2 with Cl- for neutrality; water 55.5 M (not in the paper).
MEMBRANE_SPECIES = dict(name=("Na+", "Ca2+", "Cl-", "H2O"),
                        valence=(1.0, 2.0, -1.0, 0.0),
                        radius_A=(0.95, 0.99, 1.81, 1.4),
                        bath_M=(0.100, 0.001, 0.102, 55.5))


@dataclass
class Problem:
    """A grid problem.  Arrays are flat, x-fastest: idx = i + nx*(j + ny*k)."""
    name: str
    nx: int
    ny: int
    nz: int
    h: float
    origin: tuple
    eps: np.ndarray                       # [N] nodal dielectric
    node_type: np.ndarray                 # [N] uint8 SOLVENT/SOLUTE/FIXED
    fixed_charge: np.ndarray              # [N] charge (e) spread to nodes
    bc_phi: tuple = (DIRICHLET,) * 6      # faces -x,+x,-y,+y,-z,+z
    bc_value: tuple = (0.0,) * 6          # phi-hat on Dirichlet faces
    bc_psi: tuple = (DIRICHLET,) * 6      # PF1 density: Psi = 0 (Eq. (14))
    fixed_value: np.ndarray | None = None
    b: np.ndarray | None = None           # RHS for linear workloads
    sigma: np.ndarray | None = None       # diagonal shift for linear workloads
    meta: dict = field(default_factory=dict)

    @property
    def N(self) -> int:
        return self.nx * self.ny * self.nz

    @property
    def shape(self):
        return (self.nz, self.ny, self.nx)


def _index_grid(n):
    k, j, i = np.meshgrid(np.arange(n), np.arange(n), np.arange(n), indexing="ij")
    return i, j, k


def _spread(nodes_ijk, q, n):
    """Add each charge to its nearest node (coincident charges add)."""
    out = np.zeros(n * n * n)
    i, j, k = nodes_ijk
    np.add.at(out, i + n * (j + n * k), q)
    return out


def _ball_points(stream: Stream, m: int, radius: float):
    """m points uniform in the ball |x| < radius by rejection from the cube."""
    pts = []
    while len(pts) < m:
        u = stream.take(3 * 4 * m).reshape(-1, 3)
        cand = (2.0 * u - 1.0) * radius
        ok = (cand * cand).sum(axis=1) < radius * radius
        for c in cand[ok]:
            pts.append(c)
            if len(pts) == m:
                break
    return np.array(pts)


def sphere_poisson(n: int = 33, seed: int = 1, n_charges: int = 20, eps_in: float = 2.0,
                   eps_out: float = 80.0, radius: float = 0.5) -> Problem:
    """Dielectric sphere in [-1,1]^3 with +-1 charges, zero Dirichlet faces.

    n-1 must be a multiple of 4 so the sphere radius is a whole number of
    cells; a node is inside iff its squared index distance from the centre is
    strictly below (radius/h)^2.  Signs alternate +1 (even draw), -1 (odd).
    The right-hand side is the charge density q/h^3 (dimensionless)."""
    if (n - 1) % 4:
        raise ValueError("n-1 must be a multiple of 4")
    h = 2.0 / (n - 1)
    c = (n - 1) // 2
    rc = int(round(radius / h))
    i, j, k = _index_grid(n)
    inside = ((i - c) ** 2 + (j - c) ** 2 + (k - c) ** 2) < rc * rc
    eps = np.where(inside, eps_in, eps_out).astype(np.float64).ravel()
    node_type = np.where(inside, SOLUTE, SOLVENT).astype(np.uint8).ravel()
    pos = _ball_points(Stream(seed), n_charges, radius)
    q = np.where(np.arange(n_charges) % 2 == 0, 1.0, -1.0)
    ijk = np.rint((pos + 1.0) / h).astype(np.int64).T
    fixed = _spread(ijk, q, n)
    return Problem(name=f"sphere_poisson_{n}", nx=n, ny=n, nz=n, h=h, origin=(-1.0,) * 3,
                   eps=eps, node_type=node_type, fixed_charge=fixed, b=fixed / h ** 3,
                   meta=dict(positions=pos, charges=q, seed=seed))


def membrane_pore(n: int = 97, seed: int = 2, n_charges: int = 2000, bias_phi: float = 0.0,
                  box_A: float = 40.0, slab_half_A: float = 10.0, pore_A: float = 5.0,
                  shell_A: float = 10.0, q_max: float = 0.8) -> Problem:
    """Membrane slab with a pore and a charged shell in a 40 A cube.

    Solvent (eps_s = 78.45) outside the slab and inside the pore; solute
    (eps_m = 2) elsewhere in the slab.  Membership uses exact index tests:
    slab |k-c| <= slab/h, pore d_xy^2 < (pore/h)^2.  Charges U[-q_max, q_max]
    are uniform in the shell pore <= r_xy <= shell, |z| <= slab; a draw whose
    nearest node is solvent is rejected.  z faces are Dirichlet (bias_phi on
    -z, 0 on +z, phi-hat units), x/y faces Neumann (Eq. (4))."""
    h = box_A / (n - 1)
    c = (n - 1) // 2
    half = box_A / 2.0
    s_slab, s_pore = slab_half_A / h, pore_A / h
    if abs(s_slab - round(s_slab)) > 1e-9 or abs(s_pore - round(s_pore)) > 1e-9:
        raise ValueError("slab and pore radii must fall on grid lines")
    s_slab, s_pore = int(round(s_slab)), int(round(s_pore))
    i, j, k = _index_grid(n)
    d2 = (i - c) ** 2 + (j - c) ** 2
    in_slab = np.abs(k - c) <= s_slab
    pore = d2 < s_pore * s_pore
    solute = in_slab & ~pore
    eps = np.where(solute, TABLE1["eps_m"], TABLE1["eps_s"]).astype(np.float64).ravel()
    node_type = np.where(solute, SOLUTE, SOLVENT).astype(np.uint8).ravel()

    st = Stream(seed)
    pos, qs = [], []
    while len(pos) < n_charges:
        u = st.take(4 * 4096).reshape(-1, 4)
        xyz = np.stack([(2 * u[:, 0] - 1) * shell_A, (2 * u[:, 1] - 1) * shell_A,
                        (2 * u[:, 2] - 1) * slab_half_A], axis=1)
        q = -q_max + 2.0 * q_max * u[:, 3]
        r2 = xyz[:, 0] ** 2 + xyz[:, 1] ** 2
        ok = (r2 >= pore_A ** 2) & (r2 <= shell_A ** 2)
        for p, qq in zip(xyz[ok], q[ok]):
            ii, jj, kk = np.rint((p + half) / h).astype(np.int64)
            if node_type[ii + n * (jj + n * kk)] != SOLUTE:
                continue
            pos.append(p)
            qs.append(qq)
            if len(pos) == n_charges:
                break
    pos, qs = np.array(pos), np.array(qs)
    ijk = np.rint((pos + half) / h).astype(np.int64).T
    fixed = _spread(ijk, qs, n)
    return Problem(name=f"membrane_pore_{n}", nx=n, ny=n, nz=n, h=h, origin=(-half,) * 3,
                   eps=eps, node_type=node_type, fixed_charge=fixed,
                   bc_phi=(NEUMANN, NEUMANN, NEUMANN, NEUMANN, DIRICHLET, DIRICHLET),
                   bc_value=(0.0, 0.0, 0.0, 0.0, float(bias_phi), 0.0),
                   meta=dict(positions=pos, charges=qs, seed=seed, species=MEMBRANE_SPECIES,
                             lc_A=2 * 0.95, eps_s=TABLE1["eps_s"]))


def point_charges(prob: Problem) -> np.ndarray:
    """The problem's point charges as rows (x, y, z, valence), positions
    measured from node (0, 0, 0) in grid length units (the charges before
    they are spread to nodes)."""
    pos = np.asarray(prob.meta["positions"], dtype=np.float64).reshape(-1, 3)
    q = np.asarray(prob.meta["charges"], dtype=np.float64).ravel()
    return np.column_stack([pos - np.asarray(prob.origin, dtype=np.float64), q])


def lambda_length_A(unit_A: float = 1.0) -> float:
    """e^2 / (eps0 kB T) from the Table 1 constants, in units of unit_A Angstrom."""
    t = TABLE1
    return t["e"] ** 2 / (t["eps0_F_per_cm"] * 100.0 * t["kB"] * t["T"]) * 1e10 / unit_A


# Synthetic access / binding sites of the filter region (Sec. 2, Fig. 3): a
# Na+ pathway of five sites and a Ca2+ pathway of three, on two lines parallel
# to the pore axis, 2 A either side of it.  Positions in A from the box centre.
SITE_NAMES = ("aS1", "bS2", "bS3", "bS4", "aS5", "aS6", "bS7", "aS8")
SITE_XYZ_A = ((-2.0, 0.0, 6.0), (-2.0, 0.0, 3.0), (-2.0, 0.0, 0.0), (-2.0, 0.0, -3.0), (-2.0, 0.0, -6.0),
              (2.0, 0.0, -5.0), (2.0, 0.0, 0.0), (2.0, 0.0, 5.0))
SITE_ION = ("Na+",) * 5 + ("Ca2+",) * 3
# The five total-potential states of the exchange cycle (Sec. 2): occupied
# sites and whether the structure faces inward (z reversed) or outward.
TPS = (("TPS1", ("bS3", "bS7"), "inward"),
       ("TPS2", ("aS1", "bS3", "bS7"), "outward"),
       ("TPS3", ("aS1", "bS2", "bS4", "bS7"), "outward"),
       ("TPS4", ("bS2", "bS3", "bS4"), "outward"),
       ("TPS5", ("bS2", "bS3", "bS4"), "inward"))


def tps_states(n: int = 97, seed: int = 2, n_charges: int = 2000):
    """The five states of the exchange cycle on the n^3 membrane.

    The protein atoms are the membrane's shell charges plus twelve chelating
    oxygens of -0.53 e (together -6.36 e, as Sec. 2 reports for NCX), three
    around each binding site at 2.4 A from its centre in the plane normal to
    the pore axis.  They are spread to nodes for the continuum model and kept
    as point charges for the atomic model of the sites.  Inward-facing states
    reverse the z coordinate of every atom and site about the box centre.
    Site centres are moved to their nearest node (so that every site sphere
    holds at least its centre node), radii are the ion radii (Na+ 0.95 A,
    Ca2+ 0.99 A), valences 1 and 2, eps_p = 20, eps_b = 10 (Table 1), and the
    pocket volume of Eq. (20) is twice the volume of the eight site spheres."""
    base = membrane_pore(n, seed=seed, n_charges=n_charges)
    h, c = base.h, (n - 1) // 2
    half = 20.0
    ion_r = dict(zip(MEMBRANE_SPECIES["name"], MEMBRANE_SPECIES["radius_A"]))
    radius = np.array([ion_r[x] for x in SITE_ION])
    valence = np.array([1.0 if x == "Na+" else 2.0 for x in SITE_ION])
    v_sites = 2.0 * float((4.0 * np.pi * radius ** 3 / 3.0).sum())
    ox = []
    for name, xyz in zip(SITE_NAMES, SITE_XYZ_A):
        if name.startswith("b"):
            for t in range(3):
                ang = 2.0 * np.pi * t / 3.0
                ox.append((xyz[0] + 2.4 * np.cos(ang), xyz[1] + 2.4 * np.sin(ang), xyz[2]))
    pos = np.vstack([np.asarray(base.meta["positions"], float), np.array(ox)])
    q = np.concatenate([np.asarray(base.meta["charges"], float), np.full(len(ox), -0.53)])
    out = []
    for name, occ_names, facing in TPS:
        sgn = -1.0 if facing == "inward" else 1.0
        p = pos * np.array([1.0, 1.0, sgn])
        ijk = np.rint((p + half) / h).astype(np.int64).T
        prob = dataclasses.replace(base, name=f"{name}_{n}", fixed_charge=_spread(ijk, q, n),
                                   fixed_value=np.zeros(base.N),
                                   meta=dict(base.meta, positions=p, charges=q))
        sxyz = np.array(SITE_XYZ_A) * np.array([1.0, 1.0, sgn])
        snode = np.rint((sxyz + half) / h) * h          # nearest node, grid frame
        occupied = np.array([1 if s in occ_names else 0 for s in SITE_NAMES], np.int32)
        atoms = np.column_stack([p + half, q])
        out.append(dict(name=name, facing=facing, problem=prob, atoms=atoms,
                        sites=dict(xyz=snode, radius=radius, valence=valence, occupied=occupied,
                                   eps_p=20.0, eps_b=10.0, V_sites=v_sites)))
    return out


def thermal_voltage_mV() -> float:
    """kB T / e in mV with Table 1 constants (for converting bias voltages)."""
    return TABLE1["kB"] * TABLE1["T"] / TABLE1["e"] * 1e3


def bias_sweep_mV():
    """The 16 bias voltages -150..+150 mV in 20 mV steps."""
    return [-150.0 + 20.0 * m for m in range(16)]


def batch_systems(n_sys: int = 64, seed_base: int = 4000, unit_A: float = 10.0):
    """Linearised-PB systems of seeded sizes n = 33 + 8*U{0..12}.

    Box [-1,1]^3 in units of `unit_A` Angstrom, sphere R = 0.5 with eps 2
    inside and 80 outside, U{500..4000} charges +-1 alternating in the sphere,
    NaCl bath log-uniform in [10, 500] mM.  Each system is PF2 at phi_0 = 0:
    sigma = lambda * sum_i z_i^2 c_i on the eps-80 nodes (0 inside), RHS
    lambda q / h^3, zero Dirichlet faces."""
    t = TABLE1
    lam = lambda_length_A(unit_A)
    per_M = t["NA"] * 1e3 * 1e-30 * unit_A ** 3
    out = []
    for b in range(n_sys):
        st = Stream(seed_base + b)
        u = st.take(3)
        n = 33 + 8 * int(math.floor(13 * u[0]))
        m = 500 + int(math.floor(3501 * u[1]))
        c_mM = 10.0 * (500.0 / 10.0) ** u[2]
        h = 2.0 / (n - 1)
        cidx = (n - 1) // 2
        rc = int(round(0.5 / h))
        i, j, k = _index_grid(n)
        inside = ((i - cidx) ** 2 + (j - cidx) ** 2 + (k - cidx) ** 2) < rc * rc
        eps = np.where(inside, 2.0, 80.0).astype(np.float64).ravel()
        pos = _ball_points(st, m, 0.5)
        q = np.where(np.arange(m) % 2 == 0, 1.0, -1.0)
        ijk = np.rint((pos + 1.0) / h).astype(np.int64).T
        fixed = _spread(ijk, q, n)
        cb = c_mM * 1e-3 * per_M
        sigma = np.where(inside.ravel(), 0.0, lam * (1.0 + 1.0) * cb)
        out.append(Problem(name=f"batch_{b}", nx=n, ny=n, nz=n, h=h, origin=(-1.0,) * 3, eps=eps,
                           node_type=np.where(inside, SOLUTE, SOLVENT).astype(np.uint8).ravel(),
                           fixed_charge=fixed, b=lam * fixed / h ** 3, sigma=sigma,
                           meta=dict(n_charges=m, nacl_mM=c_mM, seed=seed_base + b, lam=lam)))
    return out
