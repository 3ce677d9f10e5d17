/*
 * pfo.c -- serial FP64 CPU oracle for the Poisson-Fermi hot path.
 *
 * TEST INFRASTRUCTURE ONLY: called by tests, the smoke check and the
 * benchmark's CPU-baseline leg; never by the product library.  Plain loops,
 * sequential sums in index order, no blocking, no fusion.  Built with
 * -O2 -ffp-contract=off and without fast-math.  The OpenMP pragmas mark
 * loops whose iterations are independent (the mat-vec rows, pointwise vector
 * updates, the pointwise Fermi update); every sum stays a sequential loop,
 * so a build with -fopenmp (used to write the large golden files) gives the
 * same bits as the serial build, which ignores them.
 *
 * Readings of the paper that the code depends on (each is also listed in
 * the design notes):
 *   - Jacobi preconditioning is applied on the right, M = diag(A), so the
 *     residual is that of A x = b (Sec. 4 says "pointwise Jacobi"; Table 3
 *     shows no preconditioner step).
 *   - Stopping rule: true relative residual ||b - A x||_2 / ||b_lifted||_2
 *     (Table 3 uses an absolute max-norm; the tolerance is a parameter here).
 *   - Interface faces use the harmonic mean of nodal eps.  With eps_m on
 *     Omega_m, eps_s elsewhere and the interface at edge midpoints this is
 *     the matrix of the SMIB rows, Eqs. (17)-(18); their right-hand-side
 *     terms come from pfo_smib_rhs when the singular charges are treated by
 *     the decomposition of Eq. (5) (pfo_interface), and are absent when the
 *     charges are spread to nodes instead.
 *   - Neumann faces (Eq. (4)) use a node-centred mirror ghost; a node on a
 *     Dirichlet face is Dirichlet even if it also lies on a Neumann face.
 *   - A node on several Dirichlet faces takes the value of the face that
 *     comes last in the order -x,+x,-y,+y,-z,+z; a FIXED node takes its own
 *     fixed value.
 */
#include "pfo.h"

#include <float.h>
#include <math.h>
#include <stdlib.h>
#include <string.h>

#define IDX(i, j, k) ((size_t)(i) + (size_t)nx * ((size_t)(j) + (size_t)ny * (size_t)(k)))

/* ---------------------------------------------------------------- grid */

static int grid_ok(int nx, int ny, int nz, double h)
{
    return nx >= 3 && ny >= 3 && nz >= 3 && h > 0.0 && isfinite(h);
}

/* 1 if node (i,j,k) lies on face f (0:-x 1:+x 2:-y 3:+y 4:-z 5:+z). */
static int on_face(int i, int j, int k, int nx, int ny, int nz, int f)
{
    switch (f) {
    case 0: return i == 0;
    case 1: return i == nx - 1;
    case 2: return j == 0;
    case 3: return j == ny - 1;
    case 4: return k == 0;
    default: return k == nz - 1;
    }
}

int pfo_dirichlet(const pfo_grid *g, int system, const int *bc_psi,
                  unsigned char *is_dir, double *value)
{
    int nx = g->nx, ny = g->ny, nz = g->nz;
    if (!grid_ok(nx, ny, nz, g->h)) return PFO_EARG;
    const int *bc = (system == 0) ? g->bc : bc_psi;
    for (int k = 0; k < nz; ++k)
        for (int j = 0; j < ny; ++j)
            for (int i = 0; i < nx; ++i) {
                size_t n = IDX(i, j, k);
                unsigned char d = 0;
                double val = 0.0;
                for (int f = 0; f < 6; ++f) {
                    if (bc[f] == PFO_DIRICHLET && on_face(i, j, k, nx, ny, nz, f)) {
                        d = 1;
                        val = (system == 0) ? g->bc_value[f] : 0.0;
                    }
                }
                unsigned char t = g->type ? g->type[n] : PFO_SOLVENT;
                if (system == 0 && t == PFO_FIXED) {
                    d = 1;
                    val = g->fixed_value ? g->fixed_value[n] : 0.0;
                }
                if (system == 1 && t != PFO_SOLVENT) {
                    d = 1;
                    val = 0.0;   /* Eq. (14): Psi = 0 outside the solvent */
                }
                is_dir[n] = d;
                value[n] = d ? val : 0.0;
            }
    return PFO_OK;
}

/* --------------------------------------------------------- assembly (D1) */

/* Face coefficient between two nodes: harmonic mean of the nodal values. */
static double face_coef(double a, double b)
{
    return 2.0 * a * b / (a + b);
}

int pfo_assemble(int nx, int ny, int nz, double h, const double *coef,
                 const double *sigma, const int *bc, const unsigned char *is_dir,
                 double *A)
{
    if (!grid_ok(nx, ny, nz, h)) return PFO_EARG;
    size_t N = (size_t)nx * ny * nz;
    double *A0 = A, *A1 = A + N, *A2 = A + 2 * N, *A3 = A + 3 * N;
    double *A4 = A + 4 * N, *A5 = A + 5 * N, *A6 = A + 6 * N;
    memset(A, 0, 7 * N * sizeof(double));
    const double ih2 = 1.0 / (h * h);
    (void)bc; /* faces are Neumann wherever the node is not Dirichlet */

    for (int k = 0; k < nz; ++k)
        for (int j = 0; j < ny; ++j)
            for (int i = 0; i < nx; ++i) {
                size_t n = IDX(i, j, k);
                if (is_dir[n]) {
                    A0[n] = 1.0;
                    continue;
                }
                /* six directions: W,E,S,N,D,U.  An absent neighbour means the
                 * node sits on a Neumann face: its mirror image across the face
                 * is the neighbour on the other side, so that coefficient is
                 * added to the opposite diagonal. */
                double cW, cE, cS, cN, cD, cU;
                /* west / east */
                if (i > 0) { cW = face_coef(coef[n], coef[IDX(i - 1, j, k)]) * ih2; A2[n] -= cW; }
                else       { cW = face_coef(coef[n], coef[IDX(i + 1, j, k)]) * ih2; A1[n] -= cW; }
                if (i < nx - 1) { cE = face_coef(coef[n], coef[IDX(i + 1, j, k)]) * ih2; A1[n] -= cE; }
                else            { cE = face_coef(coef[n], coef[IDX(i - 1, j, k)]) * ih2; A2[n] -= cE; }
                /* south / north */
                if (j > 0) { cS = face_coef(coef[n], coef[IDX(i, j - 1, k)]) * ih2; A3[n] -= cS; }
                else       { cS = face_coef(coef[n], coef[IDX(i, j + 1, k)]) * ih2; A4[n] -= cS; }
                if (j < ny - 1) { cN = face_coef(coef[n], coef[IDX(i, j + 1, k)]) * ih2; A4[n] -= cN; }
                else            { cN = face_coef(coef[n], coef[IDX(i, j - 1, k)]) * ih2; A3[n] -= cN; }
                /* down / up */
                if (k > 0) { cD = face_coef(coef[n], coef[IDX(i, j, k - 1)]) * ih2; A5[n] -= cD; }
                else       { cD = face_coef(coef[n], coef[IDX(i, j, k + 1)]) * ih2; A6[n] -= cD; }
                if (k < nz - 1) { cU = face_coef(coef[n], coef[IDX(i, j, k + 1)]) * ih2; A6[n] -= cU; }
                else            { cU = face_coef(coef[n], coef[IDX(i, j, k - 1)]) * ih2; A5[n] -= cU; }
                A0[n] = cW + cE + cS + cN + cD + cU + (sigma ? sigma[n] : 0.0);
            }
    return PFO_OK;
}

void pfo_dia_matvec(int nx, int ny, int nz, const double *A, const double *x, double *y)
{
    size_t N = (size_t)nx * ny * nz;
    const double *A0 = A, *A1 = A + N, *A2 = A + 2 * N, *A3 = A + 3 * N;
    const double *A4 = A + 4 * N, *A5 = A + 5 * N, *A6 = A + 6 * N;
    size_t sx = 1, sy = (size_t)nx, sz = (size_t)nx * ny;
#pragma omp parallel for
    for (int k = 0; k < nz; ++k)
        for (int j = 0; j < ny; ++j)
            for (int i = 0; i < nx; ++i) {
                size_t n = IDX(i, j, k);
                double acc = A0[n] * x[n];
                if (i < nx - 1) acc += A1[n] * x[n + sx];
                if (i > 0)      acc += A2[n] * x[n - sx];
                if (j > 0)      acc += A3[n] * x[n - sy];
                if (j < ny - 1) acc += A4[n] * x[n + sy];
                if (k > 0)      acc += A5[n] * x[n - sz];
                if (k < nz - 1) acc += A6[n] * x[n + sz];
                y[n] = acc;
            }
}

/* ----------------------------------------------------- BiCGSTAB (Table 3) */

static double dot(size_t N, const double *a, const double *b)
{
    double s = 0.0;
    for (size_t n = 0; n < N; ++n) s += a[n] * b[n];
    return s;
}

/* r = bfull - A x, where bfull is b on free rows and the Dirichlet value on
 * Dirichlet rows. */
static void residual(int nx, int ny, int nz, const double *A, const unsigned char *is_dir,
                     const double *value, const double *b, const double *x, double *r)
{
    size_t N = (size_t)nx * ny * nz;
    pfo_dia_matvec(nx, ny, nz, A, x, r);
#pragma omp parallel for
    for (size_t n = 0; n < N; ++n) r[n] = (is_dir[n] ? value[n] : b[n]) - r[n];
}

static double maxabs(size_t N, const double *a)
{
    double m = 0.0;
    for (size_t n = 0; n < N; ++n) {
        double v = fabs(a[n]);
        if (v > m || isnan(v)) m = v;
    }
    return m;
}

/* The stop test: rule 0, ||r||_2 / ||b_lift||_2 <= tol; rule 1, the absolute
 * max norm of Table 3, ||r||_inf <= tol. */
static int small_res(size_t N, const double *r, double bnorm, double tol, int rule)
{
    return rule ? maxabs(N, r) <= tol : sqrt(dot(N, r, r)) / bnorm <= tol;
}

int pfo_bicgstab(int nx, int ny, int nz, const double *A, const unsigned char *is_dir,
                 const double *value, const double *b, double *x, double tol,
                 int maxit, pfo_lin_info *info)
{
    return pfo_bicgstab_rule(nx, ny, nz, A, is_dir, value, b, x, tol, maxit, 0, info);
}

int pfo_bicgstab_rule(int nx, int ny, int nz, const double *A, const unsigned char *is_dir,
                      const double *value, const double *b, double *x, double tol,
                      int maxit, int rule, pfo_lin_info *info)
{
    if (!(tol > 0.0) || maxit < 0 || (rule != 0 && rule != 1)) return PFO_EARG;
    size_t N = (size_t)nx * ny * nz;
    const double *A0 = A;
    double *w = (double *)malloc(10 * N * sizeof(double));
    if (!w) return PFO_ENOMEM;
    double *r = w, *rt = w + N, *p = w + 2 * N, *v = w + 3 * N, *s = w + 4 * N;
    double *t = w + 5 * N, *ph = w + 6 * N, *sh = w + 7 * N, *minv = w + 8 * N, *xd = w + 9 * N;
    int status = PFO_OK, iters = 0, restarts = 0;

    for (size_t n = 0; n < N; ++n) {
        minv[n] = 1.0 / A0[n];
        xd[n] = is_dir[n] ? value[n] : 0.0;
        if (is_dir[n]) x[n] = value[n];
    }
    /* ||b_lifted|| = ||bfull - A x_D|| with x_D holding only the Dirichlet values */
    residual(nx, ny, nz, A, is_dir, value, b, xd, r);
    const double bnorm = sqrt(dot(N, r, r));
    if (!isfinite(bnorm)) { status = PFO_ENONFINITE; goto done_nores; }
    if (bnorm == 0.0) {
        /* homogeneous problem: the solution is x_D */
        memcpy(x, xd, N * sizeof(double));
        if (info) { info->iters = 0; info->restarts = 0; info->rel_res = 0.0; info->bnorm = 0.0; info->max_res = 0.0; }
        free(w);
        return PFO_OK;
    }
    residual(nx, ny, nz, A, is_dir, value, b, x, r);
    double rnorm;
    if (small_res(N, r, bnorm, tol, rule)) goto done;

    double rho_old, alpha, omega, rho;
restart:
    memcpy(rt, r, N * sizeof(double));
    memset(p, 0, N * sizeof(double));
    memset(v, 0, N * sizeof(double));
    rho_old = 1.0; alpha = 1.0; omega = 1.0;
    int fresh = 1;
    while (iters < maxit) {
        rho = dot(N, rt, r);
        if (fabs(rho) < 1e-300 || fabs(rho) < 1e-14 * sqrt(dot(N, rt, rt)) * sqrt(dot(N, r, r))) {
            if (fresh) { status = PFO_EBREAKDOWN; goto done; }
            ++restarts;
            goto restart;
        }
        fresh = 0;
        ++iters;
        double beta = (rho / rho_old) * (alpha / omega);
        #pragma omp parallel for
        for (size_t n = 0; n < N; ++n) p[n] = r[n] + beta * (p[n] - omega * v[n]);
        #pragma omp parallel for
        for (size_t n = 0; n < N; ++n) ph[n] = minv[n] * p[n];
        pfo_dia_matvec(nx, ny, nz, A, ph, v);
        double rtv = dot(N, rt, v);
        if (rtv == 0.0) { ++restarts; goto restart; }
        alpha = rho / rtv;
        #pragma omp parallel for
        for (size_t n = 0; n < N; ++n) s[n] = r[n] - alpha * v[n];
        if (small_res(N, s, bnorm, tol, rule)) {
            /* early exit on the half-step residual (Templates form) */
            #pragma omp parallel for
            for (size_t n = 0; n < N; ++n) x[n] += alpha * ph[n];
            residual(nx, ny, nz, A, is_dir, value, b, x, r);
            if (small_res(N, r, bnorm, tol, rule)) goto done;
            ++restarts;
            goto restart;
        }
        #pragma omp parallel for
        for (size_t n = 0; n < N; ++n) sh[n] = minv[n] * s[n];
        pfo_dia_matvec(nx, ny, nz, A, sh, t);
        double tt = dot(N, t, t);
        if (tt == 0.0) { ++restarts; goto restart; }
        omega = dot(N, t, s) / tt;
        #pragma omp parallel for
        for (size_t n = 0; n < N; ++n) x[n] += alpha * ph[n] + omega * sh[n];
        #pragma omp parallel for
        for (size_t n = 0; n < N; ++n) r[n] = s[n] - omega * t[n];
        rho_old = rho;
        double rn = sqrt(dot(N, r, r));
        if (!isfinite(rn)) { status = PFO_ENONFINITE; goto done; }
        if (small_res(N, r, bnorm, tol, rule)) {
            /* confirm with the true residual; continue from it if it fails */
            residual(nx, ny, nz, A, is_dir, value, b, x, r);
            if (small_res(N, r, bnorm, tol, rule)) goto done;
            ++restarts;
            goto restart;
        }
        if (omega == 0.0) { ++restarts; goto restart; }
    }
    status = PFO_ENOCONV;
done:
    residual(nx, ny, nz, A, is_dir, value, b, x, r);
    rnorm = sqrt(dot(N, r, r));
    if (info) {
        info->iters = iters; info->restarts = restarts; info->rel_res = rnorm / bnorm; info->bnorm = bnorm;
        info->max_res = maxabs(N, r);
    }
    free(w);
    return status;
done_nores:
    if (info) { info->iters = 0; info->restarts = 0; info->rel_res = NAN; info->bnorm = bnorm; info->max_res = NAN; }
    free(w);
    return status;
}

int pfo_linear_solve(const pfo_grid *g, const double *sigma, const double *b,
                     double *x, double tol, int maxit, pfo_lin_info *info)
{
    return pfo_linear_solve_rule(g, sigma, b, x, tol, maxit, 0, info);
}

int pfo_linear_solve_rule(const pfo_grid *g, const double *sigma, const double *b,
                          double *x, double tol, int maxit, int rule, pfo_lin_info *info)
{
    int nx = g->nx, ny = g->ny, nz = g->nz;
    if (!grid_ok(nx, ny, nz, g->h) || !g->eps || !b || !x) return PFO_EARG;
    size_t N = (size_t)nx * ny * nz;
    for (size_t n = 0; n < N; ++n)
        if (!(g->eps[n] > 0.0) || !isfinite(g->eps[n])) return PFO_EARG;
    double *A = (double *)malloc(7 * N * sizeof(double));
    unsigned char *isd = (unsigned char *)malloc(N);
    double *val = (double *)malloc(N * sizeof(double));
    if (!A || !isd || !val) { free(A); free(isd); free(val); return PFO_ENOMEM; }
    int st = pfo_dirichlet(g, 0, NULL, isd, val);
    if (st == PFO_OK) st = pfo_assemble(nx, ny, nz, g->h, g->eps, sigma, g->bc, isd, A);
    if (st == PFO_OK) st = pfo_bicgstab_rule(nx, ny, nz, A, isd, val, b, x, tol, maxit, rule, info);
    free(A); free(isd); free(val);
    return st;
}

/* ------------------------------------------------------- Fermi, Eq. (1) */

/* log(sum_i exp(t_i)) with the maximum factored out. */
static double logsumexp(int n, const double *t)
{
    double m = t[0];
    for (int i = 1; i < n; ++i) if (t[i] > m) m = t[i];
    if (m == -INFINITY) return -INFINITY;
    double s = 0.0;
    for (int i = 0; i < n; ++i) s += exp(t[i] - m);
    return m + log(s);
}

#define PFO_MAXSP 16

/* L(S) = log( Gamma_B e^S + sum_i v_i c_i^B e^{-z_i phi + p_i S} ):
 * Eq. (1) with Gamma = Gamma_B e^S substituted into Gamma = 1 - sum v_i C_i
 * gives L(S) = 0.  L is strictly increasing in S. */
static double steric_L(double S, double phi, const pfo_species *sp, double lnGB, double v0)
{
    double t[PFO_MAXSP + 1];
    t[0] = lnGB + S;
    for (int i = 0; i < sp->nsp; ++i)
        t[i + 1] = log(sp->v[i]) + log(sp->cb[i]) - sp->z[i] * phi + (sp->v[i] / v0) * S;
    return logsumexp(sp->nsp + 1, t);
}

static int species_ok(const pfo_species *sp, double *lnGB, double *v0)
{
    if (sp->nsp < 1 || sp->nsp > PFO_MAXSP) return 0;
    double vs = 0.0, occ = 0.0;
    for (int i = 0; i < sp->nsp; ++i) {
        if (!(sp->v[i] > 0.0) || !(sp->cb[i] > 0.0)) return 0;
        vs += sp->v[i];
        occ += sp->v[i] * sp->cb[i];
    }
    *v0 = vs / sp->nsp;            /* mean volume over the K+1 species */
    double GB = 1.0 - occ;         /* bulk void fraction */
    if (sp->steric && !(GB > 0.0)) return 0;
    *lnGB = sp->steric ? log(GB) : 0.0;
    return 1;
}

/* Bisection for the unique root of L: start from the bracket
 * [S_hi - step, S_hi] with S_hi = -ln Gamma_B (where L >= 0), double the
 * step until L < 0 at the lower end, then halve the bracket until the two
 * ends are adjacent doubles. */
static double steric_root_impl(double phi, const pfo_species *sp, double lnGB, double v0)
{
    double hi = -lnGB;
    double step = 1.0, lo = hi - step;
    while (steric_L(lo, phi, sp, lnGB, v0) >= 0.0) {
        step *= 2.0;
        lo = hi - step;
        if (step > 1e300) return NAN;
    }
    for (int it = 0; it < 4000; ++it) {
        double mid = 0.5 * (lo + hi);
        if (mid <= lo || mid >= hi) break;
        if (steric_L(mid, phi, sp, lnGB, v0) >= 0.0) hi = mid; else lo = mid;
    }
    double Llo = steric_L(lo, phi, sp, lnGB, v0), Lhi = steric_L(hi, phi, sp, lnGB, v0);
    return (fabs(Llo) < fabs(Lhi)) ? lo : hi;
}

double pfo_steric_root(double phi, const pfo_species *sp)
{
    double lnGB, v0;
    if (!species_ok(sp, &lnGB, &v0)) return NAN;
    if (!sp->steric) return 0.0;
    return steric_root_impl(phi, sp, lnGB, v0);
}

int pfo_fermi(size_t N, const double *phi, const unsigned char *type,
              const pfo_species *sp, double *rho_hat, double *sigma,
              double *conc, double *S)
{
    double lnGB, v0;
    if (!species_ok(sp, &lnGB, &v0)) return PFO_EARG;
    int bad = 0;
#pragma omp parallel for reduction(| : bad)
    for (size_t n = 0; n < N; ++n) {
        int solvent = !type || type[n] == PFO_SOLVENT;
        double rh = 0.0, sg = 0.0, Sn = 0.0;
        if (solvent) {
            if (!isfinite(phi[n])) { bad = 1; }
            Sn = sp->steric ? steric_root_impl(phi[n], sp, lnGB, v0) : 0.0;
            for (int i = 0; i < sp->nsp; ++i) {
                double Ci = exp(log(sp->cb[i]) - sp->z[i] * phi[n] + (sp->v[i] / v0) * Sn);
                rh += sp->z[i] * Ci;
                sg += sp->z[i] * sp->z[i] * Ci;
                if (conc) conc[(size_t)i * N + n] = Ci;
            }
            rh *= sp->lambda;
            sg *= sp->lambda;
            if (!isfinite(rh) || !isfinite(sg)) bad = 1;
        } else if (conc) {
            for (int i = 0; i < sp->nsp; ++i) conc[(size_t)i * N + n] = 0.0;
        }
        if (rho_hat) rho_hat[n] = rh;
        if (sigma) sigma[n] = sg;
        if (S) S[n] = Sn;
    }
    return bad ? PFO_ENONFINITE : PFO_OK;
}

/* ------------------------------------------ nonlinear solver (Table 2) */

int pfo_nonlinear_solve(const pfo_grid *g, const double *fixed_charge,
                        const pfo_species *sp, const pfo_nl_opts *o, double *phi,
                        double *conc, double *S, pfo_nl_info *info)
{
    int nx = g->nx, ny = g->ny, nz = g->nz;
    if (!grid_ok(nx, ny, nz, g->h) || !g->eps || !phi || !o) return PFO_EARG;
    if (!(o->omega >= 0.0 && o->omega < 1.0) || !(o->outer_tol > 0.0) || o->lc < 0.0 ||
        !(o->eps_s > 0.0))
        return PFO_EARG;
    size_t N = (size_t)nx * ny * nz;
    const double h = g->h, h3 = h * h * h;
    int st = PFO_OK;

    double *A = (double *)malloc(7 * N * sizeof(double));
    double *work = (double *)malloc(8 * N * sizeof(double));
    unsigned char *dphi = (unsigned char *)malloc(N), *dpsi = (unsigned char *)malloc(N);
    if (!A || !work || !dphi || !dpsi) { st = PFO_ENOMEM; goto out; }
    double *vphi = work, *vpsi = work + N, *src = work + 2 * N, *rho = work + 3 * N;
    double *sig = work + 4 * N, *psi = work + 5 * N, *b = work + 6 * N, *phi0 = work + 7 * N;

    if ((st = pfo_dirichlet(g, 0, NULL, dphi, vphi)) != PFO_OK) goto out;
    if ((st = pfo_dirichlet(g, 1, o->bc_psi, dpsi, vpsi)) != PFO_OK) goto out;

    /* fixed charges spread to nodes enter as lambda q / h^3 (Eq. (3) scaled) */
    for (size_t n = 0; n < N; ++n) {
        src[n] = fixed_charge ? sp->lambda * fixed_charge[n] / h3 : 0.0;
        if (o->rhs_extra) src[n] += o->rhs_extra[n];
    }

    pfo_lin_info li;
    int total_lin = 0;
    if (!o->warm_start) {
        /* Table 2 step 2: PF2 with rho' = Psi = 0, i.e. the dielectric
         * Poisson problem with the fixed charges only. */
        if ((st = pfo_assemble(nx, ny, nz, h, g->eps, NULL, g->bc, dphi, A)) != PFO_OK) goto out;
        memset(phi0, 0, N * sizeof(double));
        st = pfo_bicgstab(nx, ny, nz, A, dphi, vphi, src, phi0, o->lin_tol, o->lin_maxit, &li);
        total_lin += li.iters;
        if (st != PFO_OK) goto out;
    } else {
        memcpy(phi0, phi, N * sizeof(double));
        for (size_t n = 0; n < N; ++n) if (dphi[n]) phi0[n] = vphi[n];
    }

    /* PF1 operator eps_s (1 - lc^2 Lap_h): coefficient eps_s lc^2 on every
     * face and eps_s on the diagonal.  Constant, so assembled once. */
    double *Apsi = NULL;
    if (o->lc > 0.0) {
        Apsi = (double *)malloc(7 * N * sizeof(double));
        double *cpsi = (double *)malloc(2 * N * sizeof(double));
        if (!Apsi || !cpsi) { free(Apsi); free(cpsi); st = PFO_ENOMEM; goto out; }
        for (size_t n = 0; n < N; ++n) { cpsi[n] = o->eps_s * o->lc * o->lc; cpsi[N + n] = o->eps_s; }
        st = pfo_assemble(nx, ny, nz, h, cpsi, cpsi + N, o->bc_psi, dpsi, Apsi);
        free(cpsi);
        if (st != PFO_OK) { free(Apsi); goto out; }
    }
    memset(psi, 0, N * sizeof(double));

    int it = 0;
    double delta = INFINITY;
    while (it < o->max_outer) {
        ++it;
        /* Table 2 step 3 input: C_k^0, rho(phi_0) and rho'(phi_0) = -sigma */
        if ((st = pfo_fermi(N, phi0, g->type, sp, rho, sig, NULL, NULL)) != PFO_OK) break;
        /* step 3: PF1, eps_s (lc^2 Lap - 1) Psi = rho  <=>  eps_s (1 - lc^2 Lap) Psi = -rho */
        if (o->lc > 0.0) {
            for (size_t n = 0; n < N; ++n) b[n] = -rho[n];
            st = pfo_bicgstab(nx, ny, nz, Apsi, dpsi, vpsi, b, psi, o->lin_tol, o->lin_maxit, &li);
            total_lin += li.iters;
            if (st != PFO_OK) break;
        } else {
            for (size_t n = 0; n < N; ++n) psi[n] = dpsi[n] ? 0.0 : -rho[n] / o->eps_s;
        }
        /* step 4: PF2, -div eps grad phi + sigma phi = -eps_s Psi + sigma phi_0 (+ fixed) */
        if ((st = pfo_assemble(nx, ny, nz, h, g->eps, sig, g->bc, dphi, A)) != PFO_OK) break;
        for (size_t n = 0; n < N; ++n) b[n] = -o->eps_s * psi[n] + sig[n] * phi0[n] + src[n];
        memcpy(phi, phi0, N * sizeof(double));
        st = pfo_bicgstab(nx, ny, nz, A, dphi, vphi, b, phi, o->lin_tol, o->lin_maxit, &li);
        total_lin += li.iters;
        if (st != PFO_OK) break;
        /* step 5: relax towards the old iterate, test the max-norm change */
        delta = 0.0;
        for (size_t n = 0; n < N; ++n) {
            double nv = o->omega * phi0[n] + (1.0 - o->omega) * phi[n];
            double d = fabs(nv - phi0[n]);
            if (d > delta || isnan(d)) delta = d;
            phi0[n] = nv;
        }
        if (!isfinite(delta)) { st = PFO_ENONFINITE; break; }
        if (delta <= o->outer_tol) break;
    }
    free(Apsi);
    memcpy(phi, phi0, N * sizeof(double));
    if (st == PFO_OK && delta > o->outer_tol) st = PFO_ENOCONV;
    if (st == PFO_OK && (conc || S)) st = pfo_fermi(N, phi, g->type, sp, NULL, NULL, conc, S);
    if (info) { info->outer_iters = it; info->total_lin_iters = total_lin; info->last_delta = delta; }
out:
    free(A); free(work); free(dphi); free(dpsi);
    return st;
}

/* ------------------------- interface treatment, Sec. 3 Eqs. (5)-(10), (17)-(18) */

static const int DI[6] = {-1, 1, 0, 0, 0, 0};
static const int DJ[6] = {0, 0, -1, 1, 0, 0};
static const int DK[6] = {0, 0, 0, 0, -1, 1};

void pfo_coulomb(size_t n, const double *pts, const int *dir, int M, const double *charges,
                 double scale, double *out)
{
    for (size_t p = 0; p < n; ++p) {
        const double *r = pts + 3 * p;
        int d = dir ? dir[p] : 6;
        double acc = 0.0;
        for (int j = 0; j < M; ++j) {
            const double *c = charges + 4 * (size_t)j;
            double dx = r[0] - c[0], dy = r[1] - c[1], dz = r[2] - c[2];
            double dist = sqrt(dx * dx + dy * dy + dz * dz);
            if (d == 6) {
                acc += c[3] / dist;
            } else {
                /* d/du (1/|r - c|) = -(r - c).u / |r - c|^3 along the unit vector u */
                double comp = (d < 2) ? dx : (d < 4) ? dy : dz;
                double sgn = (d & 1) ? 1.0 : -1.0;
                acc += -c[3] * sgn * comp / (dist * dist * dist);
            }
        }
        out[p] = scale * acc;
    }
}

int pfo_smib_rhs(const pfo_grid *g, double eps_m, double eps_s, const double *jump, double *b)
{
    int nx = g->nx, ny = g->ny, nz = g->nz;
    if (!grid_ok(nx, ny, nz, g->h) || !jump || !b || !g->type || !(eps_m > 0.0) || !(eps_s > 0.0))
        return PFO_EARG;
    size_t N = (size_t)nx * ny * nz;
    unsigned char *isd = (unsigned char *)malloc(N);
    double *val = (double *)malloc(N * sizeof(double));
    if (!isd || !val) { free(isd); free(val); return PFO_ENOMEM; }
    int st = pfo_dirichlet(g, 0, NULL, isd, val);
    const double cin = -eps_m / ((eps_m + eps_s) * g->h);   /* c0 / h^2 per unit jump */
    const double cout = -eps_s / ((eps_m + eps_s) * g->h);  /* d0 / h^2 per unit jump */
    for (int k = 0; k < nz && st == PFO_OK; ++k)
        for (int j = 0; j < ny; ++j)
            for (int i = 0; i < nx; ++i) {
                size_t n = IDX(i, j, k);
                if (isd[n]) continue;
                int inside = g->type[n] == PFO_SOLUTE;
                for (int d = 0; d < 6; ++d) {
                    int a = i + DI[d], bb = j + DJ[d], c = k + DK[d];
                    if (a < 0 || a >= nx || bb < 0 || bb >= ny || c < 0 || c >= nz) continue;
                    size_t m = IDX(a, bb, c);
                    int nb_inside = g->type[m] == PFO_SOLUTE;
                    if (inside && !nb_inside) b[n] += cin * jump[(size_t)d * N + n];
                    if (!inside && nb_inside) b[n] += cout * jump[(size_t)(d ^ 1) * N + m];
                }
            }
    free(isd); free(val);
    return st;
}

int pfo_interface(const pfo_grid *g, int M, const double *charges, double lambda, double eps_m,
                  double eps_s, double lap_tol, int lap_maxit, double *b_if, double *phi_reg,
                  double *phi_lap, pfo_lin_info *lap_info)
{
    int nx = g->nx, ny = g->ny, nz = g->nz;
    if (!grid_ok(nx, ny, nz, g->h) || !g->eps || !g->type || !b_if || M < 0 || (M > 0 && !charges) ||
        !(eps_m > 0.0) || !(eps_s > 0.0) || !isfinite(lambda))
        return PFO_EARG;
    const double h = g->h, ih2 = 1.0 / (h * h);
    size_t N = (size_t)nx * ny * nz;
    for (size_t n = 0; n < N; ++n) {
        double want = g->type[n] == PFO_SOLUTE ? eps_m : eps_s;
        if (g->eps[n] != want) return PFO_EARG;
    }
    const double scale = lambda / (4.0 * 3.14159265358979323846 * eps_m);
    int st = PFO_OK;
    double *eps1 = (double *)malloc(N * sizeof(double));
    unsigned char *tl = (unsigned char *)malloc(N);
    double *fv = (double *)calloc(N, sizeof(double));
    double *sig = (double *)calloc(N, sizeof(double));
    double *rhs = (double *)calloc(N, sizeof(double));
    double *xl = (double *)calloc(N, sizeof(double));
    double *pmid = (double *)calloc(6 * N, sizeof(double));   /* phi* at edge midpoints */
    double *gmid = (double *)calloc(6 * N, sizeof(double));   /* outward derivative of phi* there */
    double *jump = (double *)calloc(6 * N, sizeof(double));
    if (!eps1 || !tl || !fv || !sig || !rhs || !xl || !pmid || !gmid || !jump) { st = PFO_ENOMEM; goto out; }

    /* phi* and its outward derivative at the midpoint of every edge leaving Omega_m */
    for (int k = 0; k < nz; ++k)
        for (int j = 0; j < ny; ++j)
            for (int i = 0; i < nx; ++i) {
                size_t n = IDX(i, j, k);
                if (g->type[n] != PFO_SOLUTE) continue;
                for (int d = 0; d < 6; ++d) {
                    int a = i + DI[d], bb = j + DJ[d], c = k + DK[d];
                    if (a < 0 || a >= nx || bb < 0 || bb >= ny || c < 0 || c >= nz) continue;
                    if (g->type[IDX(a, bb, c)] == PFO_SOLUTE) continue;
                    double mid[3] = {(i + 0.5 * DI[d]) * h, (j + 0.5 * DJ[d]) * h, (k + 0.5 * DK[d]) * h};
                    pfo_coulomb(1, mid, NULL, M, charges, scale, &pmid[(size_t)d * N + n]);
                    pfo_coulomb(1, mid, &d, M, charges, scale, &gmid[(size_t)d * N + n]);
                }
            }

    /* Laplace problem, Eqs. (9)-(10), unit coefficient, unknowns on Omega_m.
     * - Across an edge leaving Omega_m the boundary sits at the midpoint: the
     *   outside value is the ghost -2 phi*(mid) - phi^L_in (their mean is
     *   -phi*(mid)); eliminating it adds 1/h^2 to the diagonal and
     *   -2 phi*(mid)/h^2 to the right-hand side, and the outside node itself
     *   is decoupled (Dirichlet 0).
     * - An Omega_m node on a Dirichlet face of the potential takes
     *   phi^L = -phi* there, so phi-tilde carries the face value.
     * - On a Neumann face the outward derivative of phi^L is -dphi_star/dn, so
     *   phi-tilde inherits the zero flux: the mirror ghost gains 2 h g, i.e.
     *   2 g / h on the right-hand side with g = -dphi_star/dn. */
    int st_d = PFO_OK;
    unsigned char *isd = (unsigned char *)malloc(N);
    double *dval = (double *)malloc(N * sizeof(double));
    if (!isd || !dval) { free(isd); free(dval); st = PFO_ENOMEM; goto out; }
    st_d = pfo_dirichlet(g, 0, NULL, isd, dval);
    for (int k = 0; k < nz && st_d == PFO_OK; ++k)
        for (int j = 0; j < ny; ++j)
            for (int i = 0; i < nx; ++i) {
                size_t n = IDX(i, j, k);
                eps1[n] = 1.0;
                int inside = g->type[n] == PFO_SOLUTE;
                tl[n] = (inside && !isd[n]) ? PFO_SOLVENT : PFO_FIXED;
                double r[3] = {i * h, j * h, k * h};
                if (inside && isd[n]) {
                    pfo_coulomb(1, r, NULL, M, charges, scale, &fv[n]);
                    fv[n] = -fv[n];
                }
                if (!inside || isd[n]) continue;
                for (int d = 0; d < 6; ++d) {
                    int a = i + DI[d], bb = j + DJ[d], c = k + DK[d];
                    if (a < 0 || a >= nx || bb < 0 || bb >= ny || c < 0 || c >= nz) {
                        /* node on the face in direction d, Neumann (not Dirichlet) */
                        double dn;
                        pfo_coulomb(1, r, &d, M, charges, scale, &dn);
                        rhs[n] += 2.0 * (-dn) / h;
                        continue;
                    }
                    if (g->type[IDX(a, bb, c)] == PFO_SOLUTE) continue;
                    sig[n] += ih2;
                    rhs[n] += -2.0 * ih2 * pmid[(size_t)d * N + n];
                }
            }
    free(isd);
    free(dval);
    if (st_d != PFO_OK) { st = st_d; goto out; }
    pfo_grid gl = *g;   /* same face kinds; Dirichlet face nodes inside Omega_m are FIXED */
    gl.eps = eps1;
    gl.type = tl;
    gl.fixed_value = fv;
    for (int f = 0; f < 6; ++f) gl.bc_value[f] = 0.0;
    st = pfo_linear_solve(&gl, sig, rhs, xl, lap_tol, lap_maxit, lap_info);
    if (st != PFO_OK) goto out;

    /* flux jumps, Eq. (8): J = eps_m d(phi* + phi^L)/dn at the midpoint, the
     * phi^L derivative over the half cell from the inside node to the
     * midpoint, where phi^L = -phi* */
    for (int k = 0; k < nz; ++k)
        for (int j = 0; j < ny; ++j)
            for (int i = 0; i < nx; ++i) {
                size_t n = IDX(i, j, k);
                if (g->type[n] != PFO_SOLUTE) continue;
                for (int d = 0; d < 6; ++d) {
                    int a = i + DI[d], bb = j + DJ[d], c = k + DK[d];
                    if (a < 0 || a >= nx || bb < 0 || bb >= ny || c < 0 || c >= nz) continue;
                    if (g->type[IDX(a, bb, c)] == PFO_SOLUTE) continue;
                    size_t e = (size_t)d * N + n;
                    jump[e] = eps_m * (gmid[e] + (-pmid[e] - xl[n]) / (0.5 * h));
                }
            }
    memset(b_if, 0, N * sizeof(double));
    st = pfo_smib_rhs(g, eps_m, eps_s, jump, b_if);
    if (st != PFO_OK) goto out;

    if (phi_reg) {
        for (int k = 0; k < nz; ++k)
            for (int j = 0; j < ny; ++j)
                for (int i = 0; i < nx; ++i) {
                    size_t n = IDX(i, j, k);
                    if (g->type[n] != PFO_SOLUTE) { phi_reg[n] = 0.0; continue; }
                    double r[3] = {i * h, j * h, k * h}, ps;
                    pfo_coulomb(1, r, NULL, M, charges, scale, &ps);
                    phi_reg[n] = ps + xl[n];
                }
    }
    if (phi_lap) memcpy(phi_lap, xl, N * sizeof(double));
out:
    free(eps1); free(tl); free(fv); free(sig); free(rhs); free(xl); free(pmid); free(gmid); free(jump);
    return st;
}

/* ------------------------------- filter-region atomic model, Eqs. (19)-(20) */

double pfo_bulk_void(const pfo_species *sp)
{
    double lnGB, v0;
    if (!species_ok(sp, &lnGB, &v0)) return NAN;
    return sp->steric ? exp(lnGB) : 1.0;
}

static int sites_ok(const pfo_sites *s)
{
    if (s->n_sites < 1 || !s->xyz || !s->radius || !s->valence || !s->occupied) return 0;
    if (s->n_atoms < 0 || (s->n_atoms > 0 && !s->atoms)) return 0;
    if (!(s->eps_p > 0.0) || !(s->eps_b > 0.0) || !(s->V_sites > 0.0)) return 0;
    for (int b = 0; b < s->n_sites; ++b)
        if (!(s->radius[b] > 0.0) || s->valence[b] == 0.0 || (s->occupied[b] != 0 && s->occupied[b] != 1))
            return 0;
    return 1;
}

int pfo_site_model(const pfo_sites *s, const pfo_species *sp, double *phi_b, double *S_b,
                   double *psi_b, double *conc_b)
{
    const double pi = 3.14159265358979323846;
    double lnGB, v0;
    if (!sites_ok(s) || !species_ok(sp, &lnGB, &v0) || !phi_b || !S_b || !psi_b) return PFO_EARG;
    /* Eq. (20): the same value at every site */
    double occ = 0.0;
    for (int m = 0; m < s->n_sites; ++m)
        if (s->occupied[m]) occ += 4.0 * pi * s->radius[m] * s->radius[m] * s->radius[m] / 3.0;
    double void_frac = 1.0 - occ / s->V_sites;
    if (sp->steric && !(void_frac > 0.0)) return PFO_EARG;
    double S = sp->steric ? log(void_frac) - lnGB : 0.0;
    for (int b = 0; b < s->n_sites; ++b) {
        const double *c = s->xyz + 3 * (size_t)b;
        double a = s->radius[b], acc = 0.0;
        for (int k = 0; k < 6; ++k) {
            double A[3] = {c[0], c[1], c[2]};
            A[k / 2] += (k & 1) ? a : -a;
            double sa = 0.0, ss = 0.0;
            for (int j = 0; j < s->n_atoms; ++j) {
                const double *t = s->atoms + 4 * (size_t)j;
                double dx = t[0] - A[0], dy = t[1] - A[1], dz = t[2] - A[2];
                sa += t[3] / sqrt(dx * dx + dy * dy + dz * dz);
            }
            for (int m = 0; m < s->n_sites; ++m) {
                if (m == b || !s->occupied[m]) continue;
                const double *cm = s->xyz + 3 * (size_t)m;
                double dx = cm[0] - A[0], dy = cm[1] - A[1], dz = cm[2] - A[2];
                ss += s->valence[m] / sqrt(dx * dx + dy * dy + dz * dz);
            }
            acc += sa / s->eps_p + ss / s->eps_b;
        }
        double self = s->occupied[b] ? s->valence[b] / (s->eps_b * a) : 0.0;
        phi_b[b] = sp->lambda / (4.0 * pi) * (acc / 6.0 + self);
        S_b[b] = S;
        psi_b[b] = phi_b[b] - S / s->valence[b];
        if (conc_b)
            for (int i = 0; i < sp->nsp; ++i)
                conc_b[(size_t)b * sp->nsp + i] = sp->cb[i] * exp(-sp->z[i] * phi_b[b] + (sp->v[i] / v0) * S);
    }
    return PFO_OK;
}

long pfo_site_fill(int nx, int ny, int nz, double h, const pfo_sites *s, const double *phi_b,
                   unsigned char *type, double *fixed_value)
{
    if (!grid_ok(nx, ny, nz, h) || !sites_ok(s) || !phi_b || !type || !fixed_value) return PFO_EARG;
    long marked = 0;
    for (int k = 0; k < nz; ++k)
        for (int j = 0; j < ny; ++j)
            for (int i = 0; i < nx; ++i) {
                size_t n = IDX(i, j, k);
                if (type[n] != PFO_SOLVENT) continue;
                int best = -1;
                double bd = 0.0;
                for (int b = 0; b < s->n_sites; ++b) {
                    const double *c = s->xyz + 3 * (size_t)b;
                    double dx = i * h - c[0], dy = j * h - c[1], dz = k * h - c[2];
                    double d2 = dx * dx + dy * dy + dz * dz;
                    if (d2 <= s->radius[b] * s->radius[b] && (best < 0 || d2 < bd)) { best = b; bd = d2; }
                }
                if (best >= 0) {
                    type[n] = PFO_FIXED;
                    fixed_value[n] = phi_b[best];
                    ++marked;
                }
            }
    return marked;
}
