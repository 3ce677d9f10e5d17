/*
 * oracle_sanitize.c -- drives every entry point of the oracle (oracle/pfo.c)
 * on small inputs for a build with AddressSanitizer and UndefinedBehavior-
 * Sanitizer (tests/test_oracle_sanitize.py compiles and runs it on the CPU).
 * It checks return codes only; the numbers themselves are pinned by the
 * other oracle tests.  Exit status 0 when every call returned what it should.
 */
#include "../oracle/pfo.h"

#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

static unsigned long long state = 0x2545F4914F6CDD1DULL;
static double urand(void)
{
    state ^= state << 13;
    state ^= state >> 7;
    state ^= state << 17;
    return (double)(state >> 11) * (1.0 / 9007199254740992.0);
}

static int fails = 0;
#define EXPECT(cond, what)                                                   \
    do {                                                                     \
        if (!(cond)) {                                                       \
            fprintf(stderr, "FAILED: %s (line %d)\n", what, __LINE__);       \
            ++fails;                                                         \
        }                                                                    \
    } while (0)

int main(void)
{
    const int nx = 9, ny = 7, nz = 8;
    const size_t N = (size_t)nx * ny * nz;
    const double h = 0.5;
    double *eps = malloc(N * sizeof(double)), *fv = malloc(N * sizeof(double));
    double *b = malloc(N * sizeof(double)), *x = malloc(N * sizeof(double));
    double *sig = malloc(N * sizeof(double)), *q = malloc(N * sizeof(double));
    double *A = malloc(7 * N * sizeof(double)), *y = malloc(N * sizeof(double));
    double *val = malloc(N * sizeof(double)), *rho = malloc(N * sizeof(double));
    double *conc = malloc(4 * N * sizeof(double)), *S = malloc(N * sizeof(double));
    double *phi = malloc(N * sizeof(double)), *bif = malloc(N * sizeof(double));
    double *preg = malloc(N * sizeof(double)), *plap = malloc(N * sizeof(double));
    unsigned char *type = malloc(N), *isd = malloc(N);
    for (size_t n = 0; n < N; ++n) {
        int k = (int)(n / (nx * ny));
        type[n] = (k >= 3 && k <= 4) ? PFO_SOLUTE : PFO_SOLVENT;
        if (n == N / 2 + 1) type[n] = PFO_FIXED;
        eps[n] = type[n] == PFO_SOLUTE ? 2.0 : 78.45;
        fv[n] = 0.25;
        b[n] = urand() - 0.5;
        sig[n] = urand();
        q[n] = type[n] == PFO_SOLUTE ? 0.01 * (urand() - 0.5) : 0.0;
        x[n] = 0.0;
    }
    pfo_grid g = {nx, ny, nz, h, eps, type, fv, {PFO_NEUMANN, PFO_NEUMANN, PFO_DIRICHLET, PFO_NEUMANN,
                                                  PFO_DIRICHLET, PFO_DIRICHLET},
                  {0, 0, 0.5, 0, 1.0, 0}};

    /* operator */
    EXPECT(pfo_dirichlet(&g, 0, NULL, isd, val) == PFO_OK, "dirichlet");
    EXPECT(pfo_assemble(nx, ny, nz, h, eps, sig, g.bc, isd, A) == PFO_OK, "assemble");
    pfo_dia_matvec(nx, ny, nz, A, b, y);

    /* linear solves, both stop rules, and the invalid-argument path */
    pfo_lin_info li;
    EXPECT(pfo_linear_solve(&g, sig, b, x, 1e-12, 1000, &li) == PFO_OK, "linear_solve");
    memset(x, 0, N * sizeof(double));
    EXPECT(pfo_linear_solve_rule(&g, NULL, b, x, 1e-9, 1000, 1, &li) == PFO_OK, "linear_solve_rule");
    EXPECT(pfo_linear_solve(&g, sig, b, x, -1.0, 1000, &li) == PFO_EARG, "bad tolerance");

    /* Fermi update and the steric root */
    const double zv[4] = {1, 2, -1, 0}, rad[4] = {0.95, 0.99, 1.81, 1.4};
    const double cbm[4] = {0.1, 0.001, 0.102, 55.5};
    double v[4], cb[4];
    for (int i = 0; i < 4; ++i) {
        v[i] = 4.0 * 3.14159265358979323846 * rad[i] * rad[i] * rad[i] / 3.0;
        cb[i] = cbm[i] * 6.02214076e-4;
    }
    pfo_species sp = {4, zv, v, cb, 1, 7048.03};
    for (size_t n = 0; n < N; ++n) phi[n] = 40.0 * (urand() - 0.5);
    EXPECT(pfo_fermi(N, phi, type, &sp, rho, sig, conc, S) == PFO_OK, "fermi");
    EXPECT(isfinite(pfo_steric_root(3.0, &sp)), "steric_root");
    EXPECT(pfo_bulk_void(&sp) > 0.0 && pfo_bulk_void(&sp) < 1.0, "bulk_void");

    /* nonlinear loop: local Psi (l_c = 0) and a PF1 solve (l_c > 0) with an
       extra right-hand side, and the iteration limit */
    pfo_nl_opts o = {78.45, 0.0, 0.3, 1e-9, 2000, 1e-12, 5000, 0,
                     {PFO_DIRICHLET, PFO_DIRICHLET, PFO_DIRICHLET, PFO_DIRICHLET, PFO_DIRICHLET, PFO_DIRICHLET},
                     NULL};
    pfo_nl_info ni;
    memset(phi, 0, N * sizeof(double));
    EXPECT(pfo_nonlinear_solve(&g, q, &sp, &o, phi, conc, S, &ni) == PFO_OK, "nonlinear l_c = 0");
    for (size_t n = 0; n < N; ++n) y[n] = 1e-3 * (urand() - 0.5);
    o.lc = 1.9;
    o.rhs_extra = y;
    memset(phi, 0, N * sizeof(double));
    EXPECT(pfo_nonlinear_solve(&g, q, &sp, &o, phi, NULL, NULL, &ni) == PFO_OK, "nonlinear l_c > 0");
    o.max_outer = 2;
    o.rhs_extra = NULL;
    memset(phi, 0, N * sizeof(double));
    EXPECT(pfo_nonlinear_solve(&g, q, &sp, &o, phi, NULL, NULL, &ni) == PFO_ENOCONV, "nonlinear limit");

    /* decomposition: Coulomb sums, SMIB terms, interface setup */
    const double charges[8] = {4.1, 3.2, 1.7, 1.0, 3.3, 2.9, 1.9, -0.5};
    double pts[6] = {0.3, 0.4, 0.5, 2.0, 2.0, 2.0}, out[2];
    const int dir[2] = {6, 1};
    pfo_coulomb(2, pts, dir, 2, charges, 1.0, out);
    EXPECT(isfinite(out[0]) && isfinite(out[1]), "coulomb");
    for (size_t n = 0; n < N; ++n) {
        eps[n] = type[n] == PFO_SOLUTE ? 2.0 : 78.45;
        if (type[n] == PFO_FIXED) type[n] = PFO_SOLVENT;
        y[n] = 0.0;
    }
    double *jump = calloc(6 * N, sizeof(double));
    memset(bif, 0, N * sizeof(double));
    EXPECT(pfo_smib_rhs(&g, 2.0, 78.45, jump, bif) == PFO_OK, "smib_rhs");
    EXPECT(pfo_interface(&g, 2, charges, 7048.03, 2.0, 78.45, 1e-12, 5000, bif, preg, plap, &li) == PFO_OK,
           "interface");

    /* filter-region atomic model and fill */
    const double sxyz[6] = {2.0, 1.5, 1.0, 2.5, 1.5, 2.2}, srad[2] = {0.95, 0.99}, sval[2] = {1, 2};
    const int occ[2] = {1, 0};
    const double atoms[8] = {0.5, 0.5, 0.5, -0.5, 3.0, 2.0, 1.5, 0.3};
    pfo_sites s = {2, sxyz, srad, sval, occ, 2, atoms, 20.0, 10.0, 50.0};
    double pb[2], Sb[2], psib[2], cbs[8];
    EXPECT(pfo_site_model(&s, &sp, pb, Sb, psib, cbs) == PFO_OK, "site_model");
    for (size_t n = 0; n < N; ++n) fv[n] = 0.0;
    EXPECT(pfo_site_fill(nx, ny, nz, h, &s, pb, type, fv) >= 0, "site_fill");

    free(jump);
    free(eps); free(fv); free(b); free(x); free(sig); free(q); free(A); free(y); free(val); free(rho);
    free(conc); free(S); free(phi); free(bif); free(preg); free(plap); free(type); free(isd);
    if (fails) return 1;
    printf("oracle sanitizer driver: all calls ok\n");
    return 0;
}
