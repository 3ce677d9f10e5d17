/*
 * pf.h -- C-ABI of the MI355X (gfx950) Poisson-Fermi hot path.
 *
 * Method: arXiv:1711.04060 (Chen, Chen, Liu, "A GPU Poisson-Fermi Solver for
 * Ion Channel Simulations").  The library solves the 7-point finite-difference
 * systems of Sec. 3 with Jacobi-preconditioned BiCGSTAB (Sec. 4, Table 3) and
 * runs the nonlinear Poisson-Fermi loop of Sec. 4 (Tables 2 and 4) with the
 * Fermi-like concentrations and steric potential of Sec. 2, Eq. (1).
 *
 * Conventions shared by every entry point
 *   - Grid: nx*ny*nz nodes, uniform spacing h, x-fastest layout
 *     idx = i + nx*(j + ny*k).  Neighbour naming follows the seven-diagonal
 *     description of Sec. 4 (east i+1, west i-1, south i-nx, north i+nx,
 *     down i-nx*ny, up i+nx*ny).  nx, ny, nz >= 3 and N = nx*ny*nz < 2^29
 *     (byte offsets of FP64 vectors fit 32 bits).
 *   - Faces are numbered -x,+x,-y,+y,-z,+z.  Dirichlet faces hold a value;
 *     Neumann faces (zero normal derivative, Eq. (4)) use a node-centred
 *     mirror ghost.  A node on a Dirichlet face is Dirichlet even when it also
 *     lies on a Neumann face; on several Dirichlet faces the face that comes
 *     last in the order above sets its value; PF_NODE_FIXED nodes are interior
 *     Dirichlet nodes with their own value.
 *   - Operator: (A x)_i = sum over the six faces f of eps_f (x_i - x_j) / h^2
 *     + sigma_i x_i on free rows, with eps_f = 2 eps_i eps_j / (eps_i + eps_j)
 *     (harmonic mean of nodal values).  Dirichlet rows are identity rows.
 *     When eps is eps_m on Omega_m (SOLUTE nodes) and eps_s elsewhere, and
 *     the interface lies at edge midpoints, these rows are the matrix of the
 *     SMIB rows of Eqs. (17)-(18); their right-hand-side terms come from
 *     pf_interface_setup when the charges are treated by the decomposition
 *     of Eq. (5) instead of being spread to nodes.
 *   - Potentials are phi-hat = e phi / (kB T).  Lengths are in the grid's unit;
 *     lambda = e^2 / (eps0 kB T) and concentrations use the same unit.
 *   - Pointers named "device" must be device memory of the current HIP device
 *     (hipMalloc or torch CUDA tensors).  Pointers named "host" are host memory.
 *   - Every call is synchronous with respect to the stream given at
 *     pf_grid_create: it returns after the work has finished, so outputs and
 *     info structs are valid on return.
 *   - No exception crosses the ABI.  Each call returns a pf_status; on failure
 *     pf_last_error() returns a thread-local message.  Invalid arguments are
 *     rejected with PF_ERR_ARG before any device work.
 */
#ifndef PF_H
#define PF_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    PF_OK = 0,
    PF_ERR_ARG = -1,        /* invalid argument (shape, pointer, value)          */
    PF_ERR_ALLOC = -2,      /* device allocation failed                          */
    PF_ERR_DEVICE = -3,     /* a HIP call failed                                 */
    PF_ERR_NOCONV = -4,     /* iteration limit reached; best iterate written     */
    PF_ERR_BREAKDOWN = -5,  /* BiCGSTAB breakdown that restarting did not cure   */
    PF_ERR_NONFINITE = -6   /* NaN or Inf met in the iteration                   */
} pf_status;

typedef enum { PF_BC_DIRICHLET = 0, PF_BC_NEUMANN = 1 } pf_bc;

/* Node kinds.  SOLVENT nodes carry ions (Omega_s of Sec. 2); SOLUTE nodes are
 * the biomolecule/membrane (Omega_m); FIXED nodes are interior Dirichlet nodes
 * (e.g. a filter region whose potential comes from an atomic model, Sec. 2). */
typedef enum { PF_NODE_SOLVENT = 0, PF_NODE_SOLUTE = 1, PF_NODE_FIXED = 2 } pf_node;

typedef enum { PF_FP64 = 0, PF_MIXED = 1 } pf_precision;

/* Stop test of a linear solve.  PF_STOP_REL2: true relative residual
 * ||b - A x||_2 / ||b_lift||_2 <= rel_tol (the default).  PF_STOP_ABS_INF:
 * the absolute max norm of Table 3, ||b - A x||_inf <= rel_tol over the free
 * rows (rel_tol then holds an absolute tolerance, the paper's 1e-6); the
 * device iteration stops once ||r||_2^2 <= N rel_tol^2 on its recurrence
 * residual, and the true max norm, checked on the host after each chunk of
 * iterations, decides (Table 3 tests the recurrence residual after every
 * iteration). */
typedef enum { PF_STOP_REL2 = 0, PF_STOP_ABS_INF = 1 } pf_stop_rule;

typedef struct pf_grid pf_grid;   /* opaque; owns device copies of its fields */

typedef struct {
    int32_t nx, ny, nz;            /* nodes per axis, each >= 3                       */
    double h;                      /* spacing, > 0                                    */
    const double *eps;             /* device [N]: nodal dielectric, finite, > 0       */
    const uint8_t *node_type;      /* device [N]: pf_node values, or NULL = solvent   */
    const double *fixed_charge;    /* device [N]: charge (units of e) spread to nodes,
                                      or NULL = none (used by pf_nonlinear_solve)     */
    const double *fixed_value;     /* device [N]: phi-hat at FIXED nodes, or NULL = 0 */
    int32_t bc_phi[6];             /* pf_bc per face for the potential                */
    double bc_value[6];            /* phi-hat on Dirichlet faces                      */
    int32_t bc_psi[6];             /* pf_bc per face for the PF1 density Psi; its
                                      Dirichlet value is 0 (Eq. (14))                 */
    void *stream;                  /* hipStream_t to run on; NULL = default stream    */
} pf_grid_desc;

/* Copy the fields of *desc into a new grid handle (the caller may free its
 * arrays afterwards).  Validates shapes and values (eps finite and > 0,
 * node types in range, fixed data finite).  Sec. 4, Table 4 step 1. */
pf_status pf_grid_create(const pf_grid_desc *desc, pf_grid **out);

/* Release the handle and all device memory it owns.  NULL is accepted. */
void pf_grid_destroy(pf_grid *g);

typedef struct {
    double rel_tol;        /* stop when ||b - A x||_2 <= rel_tol * ||b_lift||_2, where
                              b_lift is b on free rows minus the Dirichlet couplings  */
    int32_t max_iter;      /* BiCGSTAB iterations (all refinements together), > 0    */
    int32_t precision;     /* pf_precision: PF_FP64, or PF_MIXED = FP32 inner BiCGSTAB
                              (FP32 eps, iterates and stencil; FP64 reductions and
                              scalars) inside FP64 iterative refinement; a refinement
                              step that does not lower the true residual is undone
                              and the solve continues in FP64 (fp64_fallback)         */
    double inner_tol;      /* PF_MIXED: relative residual target of each inner solve */
    int32_t max_refine;    /* PF_MIXED: maximum refinement steps                     */
    int32_t check_every;   /* iterations per device-side chunk between host checks;
                              0 = library default                                     */
    int32_t stop_rule;     /* pf_stop_rule                                            */
} pf_lin_opts;

typedef struct {
    int32_t iters;         /* BiCGSTAB iterations performed                          */
    int32_t refinements;   /* PF_MIXED refinement steps (0 for PF_FP64)              */
    int32_t restarts;      /* shadow-residual restarts                               */
    double rel_res;        /* final true relative residual                           */
    double seconds;        /* wall time of the call                                  */
    int32_t status;        /* pf_status of the call                                  */
    double max_res;        /* final true ||b - A x||_inf (PF_STOP_ABS_INF), else -1  */
    int32_t fp64_fallback; /* PF_MIXED: 1 if a refinement step failed to lower the true
                              residual and the solve finished in FP64 (the step is
                              undone first), else 0                                   */
} pf_lin_info;

/* Fill *o with defaults: rel_tol 1e-10, max_iter 20000, PF_FP64,
 * inner_tol 1e-2, max_refine 30, check_every 0, PF_STOP_REL2.  (A loose
 * inner target keeps each FP32 run far from FP32's attainable accuracy; at
 * 193^3 it takes 599 inner iterations where 1e-5 takes 881.) */
void pf_lin_opts_default(pf_lin_opts *o);

/* Solve (-div eps grad + sigma) x = b on grid g (potential boundary data:
 * bc_phi, bc_value, FIXED nodes).  sigma: device [N] >= 0 or NULL (= 0).
 * b: device [N], read on free rows.  x: device [N], in = initial guess,
 * out = solution (Dirichlet entries are overwritten with their values).
 * Jacobi-BiCGSTAB, Sec. 4 Table 3; right preconditioning with M = diag(A).
 * On PF_ERR_NOCONV the last iterate is written to x. */
pf_status pf_linear_solve(pf_grid *g, const double *sigma, const double *b, double *x,
                          const pf_lin_opts *opts, pf_lin_info *info);

/* True residual of the linear system of pf_linear_solve.
 * rel_res: host, receives ||b - A x||_2 / ||b_lift||_2 (0 when b_lift = 0 and
 * the residual vanishes).  r: device [N] receives b - A x (0 on Dirichlet
 * rows), or NULL.  x is read as given (Dirichlet entries included). */
pf_status pf_residual(pf_grid *g, const double *sigma, const double *b, const double *x,
                      double *rel_res, double *r);

/* Size of the device scratch of pf_residual_noalloc (one copy per device). */
#define PF_NOALLOC_SCRATCH_BYTES (2u << 20)

/* pf_residual for callers that cannot allocate device memory (code between
 * graph-capture calls, tight serving loops, harnesses that forbid
 * hipMalloc): the same result, with the reduction partials and sums in a
 * fixed device scratch array of PF_NOALLOC_SCRATCH_BYTES per device (held
 * until the process ends) instead of grid or workspace buffers, and no call
 * of hipMalloc, hipFree or any other allocating routine.  r is required
 * (device [N], receives b - A x, 0 on Dirichlet rows); rel_res as in
 * pf_residual.  The grid's workspace is not used, so the call works on a
 * grid that has never solved.  Limit: the residual kernel's workgroup
 * partials (8 doubles each) must fit the scratch after a 256-byte header,
 * i.e. at most 32764 workgroups; longer z-chunks are used when the grid's
 * usual launch shape has more, and PF_ERR_ARG is returned when even that
 * does not fit.  Every call on one device shares that device's scratch:
 * calls that overlap on one device (other threads, other streams) race. */
pf_status pf_residual_noalloc(pf_grid *g, const double *sigma, const double *b, const double *x,
                              double *rel_res, double *r);

/* Stencil operator application y = A x (jacobi = 0) or y = M^-1 A x
 * (jacobi = 1, M = diag(A), identity on Dirichlet rows) with the operator of
 * pf_linear_solve.  x, y: device [N], distinct.  The FP64 forms are the
 * matrix-vector product of Table 3 steps 11 and 14, matrix-free; the scaled
 * one is the product as the solver applies it (its Krylov vectors are kept
 * scaled by M^-1, so v^ = M^-1 A p^ for p^ = M^-1 p). */
pf_status pf_spmv(pf_grid *g, const double *sigma, const double *x, double *y, int32_t jacobi);

/* Same in FP32 (the inner operator of PF_MIXED): FP32 eps and vectors.
 * Only jacobi = 1 is supported (the form the inner solver applies). */
pf_status pf_spmv_f32(pf_grid *g, const double *sigma, const float *x, float *y, int32_t jacobi);

typedef struct {
    int32_t n_species;        /* K+1 species, water last (valence 0), 1..16      */
    const double *valence;    /* host [n_species]: z_i                           */
    const double *radius;     /* host [n_species]: a_i in Angstrom               */
    const double *bath_molar; /* host [n_species]: C_i^B in mol/L, > 0           */
    int32_t steric;           /* 1: Fermi distribution with steric potential
                                 (Eq. (1)); 0: Boltzmann (S == 0)                */
    double lc;                /* correlation length l_c in grid units (Eq. (2));
                                 0 = no PF1 solve (Psi = -rho/eps_s)              */
    double eps_s;             /* solvent dielectric eps_s                        */
    double kB, T, e, eps0;    /* Table 1: J/K, K, C, F/cm                        */
    double NA;                /* Avogadro's number (not in Table 1)              */
    double length_unit_A;     /* grid length unit in Angstrom (1 = Angstrom)     */
    double omega;             /* relaxation weight omega_PF on the old iterate   */
    double outer_tol;         /* stop when ||Phi - Phi_0||_inf <= outer_tol
                                 after relaxation (Table 2 step 5)               */
    int32_t max_outer;        /* outer iterations, > 0                           */
    int32_t warm_start;       /* 1: phi holds Phi_0 (skip Table 2 step 2)        */
    pf_lin_opts lin;          /* options of every PF1 / PF2 linear solve         */
    const double *rhs_extra;  /* device [N] added to the right-hand side of every
                                 PF2 solve (the b_if of pf_interface_setup), or
                                 NULL                                            */
} pf_pf_params;

typedef struct {
    int32_t outer_iters;
    int32_t total_lin_iters;
    double last_delta;        /* last ||Phi - Phi_0||_inf                         */
    double seconds;
    int32_t status;
} pf_nl_info;

/* Fill *p with Table 1 constants, omega 0.3, outer_tol 1e-8, max_outer 5000,
 * eps_s 78.45, lc 0, steric 1, lin = pf_lin_opts_default(); species fields are
 * left empty for the caller. */
void pf_pf_params_default(pf_pf_params *p);

/* Nonlinear Poisson-Fermi solve (Sec. 4, Tables 2 and 4) on grid g.
 *   step 2  PF2 with rho' = Psi = 0: -div eps grad phi = lambda q / h^3;
 *   loop    Fermi update at Phi_0 (Eq. (1)) -> rho_hat, sigma = -rho_hat';
 *           PF1 (Eq. (12), (14)): eps_s (1 - lc^2 Lap) Psi = -rho_hat on
 *           solvent nodes, Psi = 0 elsewhere and on Dirichlet bc_psi faces;
 *           PF2 (Eq. (13)): -div eps grad phi + sigma phi
 *                           = -eps_s Psi + sigma Phi_0 + lambda q / h^3;
 *           relax Phi := omega Phi_0 + (1 - omega) Phi; test the max norm.
 * phi: device [N], in (warm start) / out.  conc: device [n_species * N]
 * (species-major) or NULL; steric: device [N] or NULL -- both evaluated at the
 * returned phi (zero off the solvent).  On PF_ERR_NOCONV the last relaxed
 * iterate is returned. */
pf_status pf_nonlinear_solve(pf_grid *g, const pf_pf_params *p, double *phi, double *conc,
                             double *steric, pf_nl_info *info);

/* Fermi update alone (Eq. (1)) at potential phi (device [N]): writes
 * rho_hat = lambda sum_i z_i C_i and sigma = lambda sum_i z_i^2 C_i (device
 * [N] each, or NULL), conc (device [n_species * N] or NULL) and the steric
 * potential S (device [N] or NULL).  Non-solvent nodes get zeros. */
pf_status pf_fermi(pf_grid *g, const pf_pf_params *p, const double *phi, double *rho_hat,
                   double *sigma, double *conc, double *steric);

/* Batched linear solves: n independent systems (grids may differ in size),
 * each as pf_linear_solve with the shared opts.  info: host [n] or NULL.
 * The members' BiCGSTAB iterations run in shared launches over the tiles of
 * the members still iterating.  The first batch of a composition (precision,
 * kernel form, every member's shape) with four or more members times each
 * launch policy for a few iterations at the start of its first Krylov run and
 * keeps the fastest for the process (PF_BATCH_POLICY=k in the environment
 * pins policy k instead). */
pf_status pf_linear_solve_batch(int32_t n, pf_grid *const *g, const double *const *sigma,
                                const double *const *b, double *const *x,
                                const pf_lin_opts *opts, pf_lin_info *info);

/* Batched nonlinear solves: n independent problems, each as
 * pf_nonlinear_solve.  p: host [n] pointers; info: host [n] or NULL. */
pf_status pf_nonlinear_solve_batch(int32_t n, pf_grid *const *g, const pf_pf_params *const *p,
                                   double *const *phi, pf_nl_info *info);

/* Kernel timing for measurement: while enabled, one chunk of iterations in
 * every `sample` (single solves and batches counted together) runs as direct
 * launches on the library's stream with HIP events that each dispatch stamps
 * at its kernel's start and end, on every launch of the BiCGSTAB step-A
 * stencil kernel (the previous iteration's x, r update fused with the p
 * update and v = A p^: the kernel that moves the most bytes per iteration);
 * every Jacobi-scaled pf_spmv / pf_spmv_f32 call is timed the same way.
 * enable = 1 clears the accumulators and starts; 0 stops.  Process-wide. */
pf_status pf_timing_enable(int32_t enable, int32_t sample);

/* Accumulated timings of one kind: 0 (PF_FP64) and 1 (PF_MIXED, the FP32
 * inner kernel) = BiCGSTAB step A of single solves; 2 and 3 = the
 * Jacobi-scaled products of pf_spmv and pf_spmv_f32; 4 and 5 = the batched
 * step A (one launch over every member) in FP64 and FP32.  launches timed and
 * their mean duration in ms; bytes is the algorithmic HBM traffic of those
 * launches.  Step A per node: 9 elements of the working precision (s^, p^,
 * v^, t^, x read; x, r^, p^, v^ written), the coefficient (one palette byte
 * where the field has at most 16 distinct values, else one element), the
 * FP32 shadow (4 bytes), and one more element where the shift sigma is read
 * per node (not where it is one value per palette class and comes from a
 * table); PF1 reads one flag byte instead of the coefficient.  A batched
 * launch counts the members still iterating.  Products: x and the
 * coefficient (and an FP64 sigma) read, y written.  PF_ERR_ARG for another
 * kind. */
pf_status pf_timing_read(int32_t kind, int64_t *launches, double *mean_ms, double *bytes);

/* Streaming-bandwidth probe (a measurement aid, no part of the method): the
 * ceiling the stencil kernels are compared with.  kind 0 streams 1 input and
 * 1 output array per set, kind 1 3 inputs and 1 output, kind 2 7 inputs and
 * 4 outputs (every output = the sum of the inputs); width = 8 or 16 bytes per
 * lane access.  bufs: host array of sets * (inputs + outputs) device pointers
 * of n doubles each, set by set, inputs first.  After one untimed launch per
 * set, reps launches cycle through the sets (sets >= 3 of large arrays keep
 * them out of the 256 MB Infinity Cache); mean_us (host) receives the mean
 * launch time from HIP events on `stream` (hipStream_t, NULL = default). */
pf_status pf_stream_probe(int32_t kind, int32_t width, int64_t n, double *const *bufs, int32_t sets, int32_t reps,
                          void *stream, double *mean_us);

/* ---------------- singular-charge decomposition (Sec. 3, Eqs. (5)-(10), (17)-(18)) */

/* phi* of Eq. (5) in phi-hat units, or one of its directional derivatives, at
 * n points:  out[p] = scale * d/du sum_j z_j / |r_p - r_j|  along the unit
 * vector u of face direction dir[p] in 0..5 (-x,+x,-y,+y,-z,+z), and
 * out[p] = scale * sum_j z_j / |r_p - r_j|  when dir is NULL or dir[p] holds
 * any other value (6 by convention).
 * With scale = lambda / (4 pi eps_m) this is the Coulomb potential of the
 * point charges in a uniform dielectric eps_m.  pts: device [n][3];
 * dir: device int8 [n] or NULL; charges: device [M][4] = x, y, z, valence
 * z_j (same frame as pts); out: device [n].  Sums over the charges in index
 * order; a point on a charge gives a non-finite value.  Runs on `stream`
 * (hipStream_t, NULL = default stream) and returns when done. */
pf_status pf_coulomb(const double *pts, const int8_t *dir, int64_t n, const double *charges, int32_t M,
                     double scale, double *out, void *stream);

typedef struct {
    int32_t n_charges;     /* M >= 0 point charges inside Omega_m                 */
    const double *charges; /* device [M][4]: x, y, z measured from node (0,0,0) in
                              grid length units, valence z_j (units of e)         */
    double lambda;         /* e^2 / (eps0 kB T) in grid length units              */
    double eps_m, eps_s;   /* dielectric of Omega_m (SOLUTE) and of every other
                              node; the grid's eps must match exactly             */
    pf_lin_opts lin;       /* options of the Laplace solve                        */
} pf_iface_params;

/* Fill *p: no charges, lambda 0, eps_m 2, eps_s 78.45, lin = defaults with
 * rel_tol 1e-12. */
void pf_iface_params_default(pf_iface_params *p);

/* Interface data of the decomposition phi = phi-tilde + phi* + phi^L in
 * Omega_m, phi = phi-tilde in the solvent (Eq. (5)), on grid g.  Omega_m is
 * the set of SOLUTE nodes; the interface crosses each edge between a SOLUTE
 * node and a non-SOLUTE neighbour at its midpoint.
 *   1. phi* and its outward derivative at every such midpoint, phi* at Omega_m
 *      nodes on Dirichlet faces (and at all Omega_m nodes if phi_reg is
 *      wanted), d(phi*)/dn at Omega_m nodes on Neumann faces (pf_coulomb's
 *      kernel over a compact list of these points);
 *   2. the Laplace problem of Eqs. (9)-(10) on Omega_m (unit coefficient):
 *      phi^L = -phi* at the midpoints (so phi* + phi^L vanishes on the
 *      interface and phi-tilde is continuous), phi^L = -phi* at Omega_m nodes
 *      on Dirichlet faces, d phi^L/dn = -d(phi*)/dn on Neumann faces; solved
 *      with this library's BiCGSTAB and the options p->lin;
 *   3. the flux jump of Eq. (8), J = eps_m d(phi* + phi^L)/dn at each
 *      midpoint (phi^L's derivative over the half cell to the midpoint), and
 *      the right-hand-side terms of the SMIB rows, Eqs. (17)-(18): a free
 *      row of the potential inside Omega_m gains -eps_m J / ((eps_m + eps_s) h)
 *      per crossing edge, one outside gains -eps_s J / ((eps_m + eps_s) h).
 * Outputs (device [N]): b_if (required) = those terms, zero elsewhere --
 * pass it as pf_pf_params.rhs_extra, or add it to the right-hand side of
 * pf_linear_solve, with no fixed charges spread to nodes; phi_reg (or NULL)
 * = phi* + phi^L on Omega_m, 0 elsewhere, so that the total potential is
 * phi-tilde + phi_reg; phi_lap (or NULL) = the Laplace solution (its
 * Dirichlet values on Dirichlet rows, 0 on other nodes outside Omega_m).
 * lap_info: host or NULL.  PF_ERR_ARG if eps does not match eps_m / eps_s;
 * PF_ERR_NONFINITE if a charge sits on an evaluation point; the Laplace
 * solve's status if it fails.  Allocates and frees its own work space
 * (about 60 bytes per node). */
pf_status pf_interface_setup(pf_grid *g, const pf_iface_params *p, double *b_if, double *phi_reg,
                             double *phi_lap, pf_lin_info *lap_info);

/* ---------------- filter-region atomic model (Sec. 2, Eqs. (19)-(20)) */

typedef struct {
    int32_t n_sites;            /* 1..64 access / binding sites                      */
    const double *site_xyz;     /* host [n_sites][3]: centres c_b, grid length units
                                   measured from node (0,0,0)                        */
    const double *site_radius;  /* host [n_sites]: a_b (ion radius of the site)      */
    const double *site_valence; /* host [n_sites]: q_b of the ion an occupied site
                                   holds (nonzero)                                   */
    const int32_t *occupied;    /* host [n_sites]: O_b, 0 or 1                       */
    int32_t n_atoms;            /* M >= 0 protein atoms                              */
    const double *atoms;        /* device [M][4]: x, y, z (same frame), charge (e)   */
    double eps_p, eps_b;        /* protein and site dielectric (Table 1: 20, 10)     */
    double V_sites;             /* pocket volume of Eq. (20), grid length units^3    */
} pf_site_params;

/* Atomic model of the filter region.  For every site b (phi-hat units, lambda
 * from the constants of pp):
 *   phi_b = lambda/(4 pi) [ (1/6) sum_k ( sum_j z_j / (eps_p |c_j - A_k|)
 *            + sum_{m != b} O_m q_m / (eps_b |c_m - A_k|) ) + O_b q_b / (eps_b a_b) ]
 * with A_k the six surface points c_b +- a_b e_x, e_y, e_z (Eq. (19));
 *   S_b = ln((1 - sum_m O_m v_m / V_sites) / Gamma^B), v_m = 4 pi a_m^3 / 3
 * (Eq. (20); Gamma^B from the species of pp; S_b = 0 when steric is off);
 *   psi_b = phi_b - S_b / q_b, the site's total potential in phi-hat units
 * (the Psi_b of Eqs. (21)-(22) divided by kB T / e);
 *   conc_b (host [n_sites * n_species] or NULL) = Eq. (1) at the site:
 *   C_i^B exp(-z_i phi_b + (v_i / v_0) S_b), per cubed grid length unit (as
 *   the conc output of pf_nonlinear_solve).
 * phi_b, S_b, psi_b: host [n_sites].  One workgroup per site sums the atoms
 * in a fixed order.  PF_ERR_ARG when the occupied volume reaches V_sites
 * with steric on.  Runs on `stream` (NULL = default) and returns when done. */
pf_status pf_site_model(const pf_pf_params *pp, const pf_site_params *s, double *phi_b, double *S_b,
                        double *psi_b, double *conc_b, void *stream);

/* Filter region Omega_f as Dirichlet data of the continuum model (Sec. 2:
 * the atomic model's values bound the continuum problem there): every
 * SOLVENT node within a_b of a site centre (|r - c_b|^2 <= a_b^2 in plain
 * FP64; the nearest centre if several, the lower index on a tie) becomes
 * PF_NODE_FIXED with fixed_value = phi_b of that site.  Other nodes are left
 * as they are.  node_type: device uint8 [N] in/out; fixed_value: device [N]
 * in/out; phi_b: host [n_sites]; marked: host or NULL, receives the number of
 * nodes marked.  Pass the arrays to pf_grid_create afterwards.  Runs on
 * `stream` (NULL = default) and returns when done. */
pf_status pf_site_fill(int32_t nx, int32_t ny, int32_t nz, double h, const pf_site_params *s,
                       const double *phi_b, uint8_t *node_type, double *fixed_value, int64_t *marked,
                       void *stream);

/* Thread-local description of the last error (empty string if none). */
const char *pf_last_error(void);

/* Launch-shape override for tests and tuning: points per workgroup strip,
 * z-planes per workgroup, threads per workgroup, and planes of loads kept in
 * flight ahead of the plane being computed (pipeline 1 or 2).  0 =
 * autotuned/default for each.  Applies to grids created afterwards (and
 * turns the autotuner off while any override is set).  Returns PF_ERR_ARG
 * for unsupported shapes. */
pf_status pf_set_launch(int32_t strip, int32_t zdepth, int32_t threads, int32_t pipeline);

#ifdef __cplusplus
}
#endif
#endif
