/*
 * pfo.h -- serial FP64 CPU oracle for the Poisson-Fermi hot path.
 *
 * TEST INFRASTRUCTURE ONLY.  This library exists so that tests, the smoke
 * check and the CPU-baseline leg of the benchmark can compare the GPU
 * library against a plain, slow, obviously correct implementation.  The
 * product path never links, loads or calls it.  It shares no code, header,
 * table or constant with the GPU library.
 *
 * What it computes (citations are to the paper, arXiv:1711.04060):
 *   - the 7-point finite-difference operator  -div(eps grad) + sigma
 *     (Sec. 3, the FD discretisation of Eqs. (7), (12), (13)), assembled
 *     explicitly as the seven diagonals A0..A6 of Sec. 4 (diagonal storage
 *     without offset arrays: A0 centre, A1 east i+1, A2 west i-1, A3 south
 *     i-nx, A4 north i+nx, A5 down i-nx*ny, A6 up i+nx*ny);
 *   - Jacobi-preconditioned BiCGSTAB (Sec. 4, Table 3), right-preconditioned
 *     with M = diag(A);
 *   - the Fermi-like concentrations and steric potential (Sec. 2, Eq. (1))
 *     by bisection on the void-fraction equation;
 *   - the sequential nonlinear solver of Sec. 4, Table 2 (initial PF2 solve,
 *     then PF1 / PF2 / relaxation until the max-norm update is small);
 *   - the singular-charge decomposition of Sec. 3 (Eqs. (5), (8)-(10)) with
 *     the right-hand-side terms of the SMIB rows (Eqs. (17)-(18)).
 *
 * Units: potentials are phi-hat = e*phi/(kB*T); lengths in the grid's unit;
 * concentrations per cubed length unit; lambda = e^2/(eps0*kB*T) in the
 * same length unit.  All arrays are host memory, x-fastest layout
 * idx = i + nx*(j + ny*k).
 */
#ifndef PFO_H
#define PFO_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { PFO_DIRICHLET = 0, PFO_NEUMANN = 1 };
enum { PFO_SOLVENT = 0, PFO_SOLUTE = 1, PFO_FIXED = 2 };

/* return codes */
enum { PFO_OK = 0, PFO_EARG = -1, PFO_ENOMEM = -2, PFO_ENOCONV = -4,
       PFO_EBREAKDOWN = -5, PFO_ENONFINITE = -6 };

typedef struct {
    int nx, ny, nz;               /* >= 3 each */
    double h;                     /* uniform spacing, > 0 */
    const double *eps;            /* [N] nodal dielectric, > 0 */
    const unsigned char *type;    /* [N] PFO_SOLVENT/SOLUTE/FIXED, or NULL = all solvent */
    const double *fixed_value;    /* [N] phi-hat at FIXED nodes, or NULL = 0 */
    int bc[6];                    /* faces -x,+x,-y,+y,-z,+z: PFO_DIRICHLET / PFO_NEUMANN */
    double bc_value[6];           /* Dirichlet value per face */
} pfo_grid;

/* Which rows are Dirichlet (identity rows) and their values.
 * system 0: the potential (bc, bc_value, FIXED nodes take fixed_value);
 * system 1: the PF1 density Psi (bc given in bc_psi, value 0, every
 *           non-solvent node is Dirichlet 0 -- Eq. (14)). */
int pfo_dirichlet(const pfo_grid *g, int system, const int *bc_psi,
                  unsigned char *is_dir, double *value);

/* Assemble the seven diagonals A[0..6][N] (A must hold 7*N doubles) of
 *   (-div_h coef grad_h + sigma) on free rows, identity on Dirichlet rows.
 * coef: nodal coefficient field (eps, or a constant for PF1); sigma may be NULL. */
int pfo_assemble(int nx, int ny, int nz, double h, const double *coef,
                 const double *sigma, const int *bc, const unsigned char *is_dir,
                 double *A);

/* y = A x with the seven diagonals. */
void pfo_dia_matvec(int nx, int ny, int nz, const double *A, const double *x, double *y);

typedef struct {
    int iters;          /* BiCGSTAB iterations */
    int restarts;       /* shadow-residual restarts */
    double rel_res;     /* final true ||b - A x||_2 / ||b_lifted||_2 */
    double bnorm;       /* ||b_lifted||_2 */
    double max_res;     /* final true ||b - A x||_inf (free rows; Dirichlet rows are 0) */
} pfo_lin_info;

/* Right-Jacobi BiCGSTAB on A x = b.  x: in = initial guess, out = solution;
 * Dirichlet rows of x are set to `value` before iterating.  b is read on
 * free rows only.  Stops when the true relative residual <= tol. */
int pfo_bicgstab(int nx, int ny, int nz, const double *A, const unsigned char *is_dir,
                 const double *value, const double *b, double *x, double tol,
                 int maxit, pfo_lin_info *info);

/* The same with a choice of stop test: rule 0 as above; rule 1 the absolute
 * max norm of Table 3, ||r||_inf <= tol, on the recurrence residual and then
 * confirmed on the true residual. */
int pfo_bicgstab_rule(int nx, int ny, int nz, const double *A, const unsigned char *is_dir,
                      const double *value, const double *b, double *x, double tol,
                      int maxit, int rule, pfo_lin_info *info);

/* Assemble + solve for system 0 of g: (-div eps grad + sigma) x = b. */
int pfo_linear_solve(const pfo_grid *g, const double *sigma, const double *b,
                     double *x, double tol, int maxit, pfo_lin_info *info);
int pfo_linear_solve_rule(const pfo_grid *g, const double *sigma, const double *b,
                          double *x, double tol, int maxit, int rule, pfo_lin_info *info);

typedef struct {
    int nsp;                  /* K+1 species, water last */
    const double *z;          /* [nsp] valences */
    const double *v;          /* [nsp] volumes 4*pi*a^3/3 */
    const double *cb;         /* [nsp] bath concentrations (> 0) */
    int steric;               /* 0: S == 0 (Boltzmann), 1: Fermi with steric potential */
    double lambda;            /* e^2/(eps0 kB T) in grid length units */
} pfo_species;

/* Eq. (1) at every node of type SOLVENT (or every node if type == NULL).
 * Outputs (each may be NULL): rho_hat = lambda*sum z_i C_i,
 * sigma = lambda*sum z_i^2 C_i, conc[nsp*N] (species-major), S[N]. */
int pfo_fermi(size_t N, const double *phi, const unsigned char *type,
              const pfo_species *sp, double *rho_hat, double *sigma,
              double *conc, double *S);

/* Root S of Gamma_B e^S + sum v_i c_i^B exp(-z_i phi + p_i S) = 1 at a single node. */
double pfo_steric_root(double phi, const pfo_species *sp);

typedef struct {
    double eps_s;             /* solvent dielectric */
    double lc;                /* correlation length (grid units); 0 = no PF1 solve */
    double omega;             /* relaxation weight on the old iterate */
    double outer_tol;         /* max-norm stop on the relaxed update */
    int max_outer;
    double lin_tol;           /* relative residual for every linear solve */
    int lin_maxit;
    int warm_start;           /* 1: phi holds the initial phi_0, skip the initial PF2 solve */
    int bc_psi[6];            /* Psi boundary kinds (Dirichlet value 0) */
    const double *rhs_extra;  /* [N] added to every PF2 right-hand side (the interface
                                 terms of pfo_interface), or NULL */
} pfo_nl_opts;

typedef struct {
    int outer_iters;
    int total_lin_iters;
    double last_delta;
} pfo_nl_info;

/* Table 2 of the paper.  fixed_charge: [N] charge (units of e) per node or
 * NULL.  phi: in (warm start) / out.  conc/S optional outputs at the final phi. */
int pfo_nonlinear_solve(const pfo_grid *g, const double *fixed_charge,
                        const pfo_species *sp, const pfo_nl_opts *o, double *phi,
                        double *conc, double *S, pfo_nl_info *info);

/* ---------------------------- interface treatment, Sec. 3 Eqs. (5)-(10), (17)-(18) */

/* phi* of Eq. (5) in phi-hat units, sum_j scale * z_j / |r - r_j| with
 * scale = lambda / (4 pi eps_m), or a directional derivative of it, at n
 * points.  pts [n][3] and charges [M][4] (x, y, z, valence z_j) share one
 * frame (grid length units).  dir NULL or dir[p] == 6: the potential;
 * dir[p] in 0..5: the derivative along the unit vector of face direction
 * dir[p] (-x,+x,-y,+y,-z,+z).  Sums over the charges in index order. */
void pfo_coulomb(size_t n, const double *pts, const int *dir, int M, const double *charges,
                 double scale, double *out);

/* Right-hand-side terms of the SMIB rows, Eqs. (17)-(18), added to b.
 * Omega_m = SOLUTE nodes.  jump[d*N + n] is the flux jump [eps dphi/dn]
 * (outside minus inside, n pointing out of Omega_m) at the midpoint of the
 * edge from Omega_m node n to its neighbour in direction d (read only where
 * that neighbour exists and lies outside Omega_m).  A free row of the
 * potential system (pfo_dirichlet system 0) inside Omega_m gains
 * -eps_m J / ((eps_m + eps_s) h) per such edge (c0 / h^2), one outside gains
 * -eps_s J / ((eps_m + eps_s) h) (d0 / h^2).  The matrix part of the SMIB
 * rows is the harmonic-mean operator of pfo_assemble when eps is eps_m on
 * Omega_m and eps_s elsewhere. */
int pfo_smib_rhs(const pfo_grid *g, double eps_m, double eps_s, const double *jump, double *b);

/* Interface data of the singular-charge decomposition (Eq. (5)):
 *   phi_star at the Dirichlet nodes of the Laplace problem: nodes outside Omega_m
 *   next to it, and Omega_m nodes on a domain face;
 *   phi^L: unit-coefficient Laplace problem (Eq. (9)) on the other Omega_m
 *   nodes, phi^L = -phi_star at those Dirichlet nodes (Eq. (10), signed so that
 *   phi_star + phi^L vanishes on the boundary of Omega_m and the total potential
 *   is continuous);
 *   J = eps_m (d phi_star / dn + (phi^L_out - phi^L_in) / h) at every edge midpoint
 *   (Eq. (8)), then pfo_smib_rhs.
 * eps must equal eps_m on SOLUTE nodes and eps_s on all others.
 * Outputs [N] (NULL allowed except b_if): b_if = SMIB right-hand-side terms;
 * phi_reg = phi_star + phi^L on Omega_m nodes, 0 elsewhere (total potential =
 * phi-tilde + phi_reg); phi_lap = the Laplace solution (its Dirichlet values
 * at the Dirichlet nodes, 0 on other nodes outside Omega_m). */
int pfo_interface(const pfo_grid *g, int M, const double *charges, double lambda, double eps_m,
                  double eps_s, double lap_tol, int lap_maxit, double *b_if, double *phi_reg,
                  double *phi_lap, pfo_lin_info *lap_info);

/* ------------------------------- filter-region atomic model, Eqs. (19)-(20) */

typedef struct {
    int n_sites;
    const double *xyz;        /* [n_sites][3] site centres c_b (grid length units) */
    const double *radius;     /* [n_sites] a_b */
    const double *valence;    /* [n_sites] q_b of the ion an occupied site holds (nonzero) */
    const int *occupied;      /* [n_sites] O_b: 0 or 1 */
    int n_atoms;
    const double *atoms;      /* [M][4] x, y, z, partial charge (e) */
    double eps_p, eps_b;      /* protein and site dielectric */
    double V_sites;           /* pocket volume of Eq. (20), > 0 */
} pfo_sites;

/* Bulk void fraction Gamma^B = 1 - sum_i v_i C_i^B of the species (1 when
 * steric is off, NAN for invalid species). */
double pfo_bulk_void(const pfo_species *sp);

/* Eq. (19): phi_b (phi-hat units, lambda from sp), the mean over the six
 * surface points c_b +- a_b e_x, e_y, e_z of the Coulomb sums of the atoms
 * (eps_p) and of the other occupied sites (eps_b), plus the self term
 * O_b q_b / (eps_b a_b), all times lambda / (4 pi).  Eq. (20): S_b =
 * ln((1 - sum_m O_m v_m / V_sites) / Gamma^B) with v_m = 4 pi a_m^3 / 3
 * (0 when steric is off).  psi_b = phi_b - S_b / q_b (the site's total
 * potential in phi-hat units).  conc_b [n_sites][nsp] or NULL: Eq. (1) at the
 * site, C_i^B exp(-z_i phi_b + (v_i / v_0) S_b).  PFO_EARG when the occupied
 * volume reaches V_sites. */
int pfo_site_model(const pfo_sites *s, const pfo_species *sp, double *phi_b, double *S_b,
                   double *psi_b, double *conc_b);

/* Filter region Omega_f: every SOLVENT node within a_b of a site centre
 * (|r - c_b|^2 <= a_b^2, the nearest centre if several, the lower index on a
 * tie) becomes FIXED with value phi_b of that site.  Other nodes are left
 * alone.  Returns the number of nodes marked, or a negative status. */
long pfo_site_fill(int nx, int ny, int nz, double h, const pfo_sites *s, const double *phi_b,
                   unsigned char *type, double *fixed_value);

#ifdef __cplusplus
}
#endif
#endif
