// Device code of the filter-region atomic model (Sec. 2, Eqs. (19)-(20)) and
// of the fill that turns its site potentials into Dirichlet data of the
// continuum model (the filter region Omega_f).
#pragma once

#include "pf_kernels.h"

namespace pfk {

constexpr int SITE_NT = 256;    // threads per workgroup (one workgroup per site)
constexpr int MAX_SITES = 64;

// Site record in device memory: centre x, y, z, radius a, valence q, occupancy O.
struct SiteRec { double x, y, z, a, q, occ; };

struct SiteArgs {
    const SiteRec *site;
    int n_sites;
    const double *atoms;    // [M][4] x, y, z, charge
    int n_atoms;
    double eps_p, eps_b;
    double V_sites;         // pocket volume of Eq. (20)
    double scale;           // lambda / (4 pi)
    SpeciesDev sp;          // lnGB, z_i, ln C_i^B, p_i = v_i / v_0
    double *out;            // per site: phi_b, S_b, psi_b, C_1..C_nsp
};

// One workgroup per site b.  Each thread sums its atoms (strided) for the six
// surface points c_b +- a_b e_x, e_y, e_z; the six sums are reduced over the
// workgroup in a fixed tree order; thread 0 adds the occupied other sites,
// the self term, and evaluates Eq. (20) and Eq. (1) at the site.
__global__ __launch_bounds__(SITE_NT) void k_site_model(SiteArgs a)
{
    __shared__ double red[6][SITE_NT];
    const int b = blockIdx.x, t = threadIdx.x;
    const SiteRec s = a.site[b];
    double acc[6] = {0, 0, 0, 0, 0, 0};
    for (int j = t; j < a.n_atoms; j += SITE_NT) {
        const double *at = a.atoms + 4 * (size_t)j;
        const double x = at[0], y = at[1], z = at[2], q = at[3];
        for (int k = 0; k < 6; ++k) {
            const double ax = s.x + (k == 0 ? -s.a : k == 1 ? s.a : 0.0);
            const double ay = s.y + (k == 2 ? -s.a : k == 3 ? s.a : 0.0);
            const double az = s.z + (k == 4 ? -s.a : k == 5 ? s.a : 0.0);
            const double dx = x - ax, dy = y - ay, dz = z - az;
            acc[k] += q / sqrt(dx * dx + dy * dy + dz * dz);
        }
    }
    for (int k = 0; k < 6; ++k) red[k][t] = acc[k];
    __syncthreads();
    for (int w = SITE_NT / 2; w > 0; w >>= 1) {
        if (t < w)
            for (int k = 0; k < 6; ++k) red[k][t] += red[k][t + w];
        __syncthreads();
    }
    if (t != 0) return;
    const double pi = 3.14159265358979323846;
    double total = 0.0;
    for (int k = 0; k < 6; ++k) {
        const double ax = s.x + (k == 0 ? -s.a : k == 1 ? s.a : 0.0);
        const double ay = s.y + (k == 2 ? -s.a : k == 3 ? s.a : 0.0);
        const double az = s.z + (k == 4 ? -s.a : k == 5 ? s.a : 0.0);
        double ss = 0.0;
        for (int m = 0; m < a.n_sites; ++m) {
            const SiteRec o = a.site[m];
            if (m == b || o.occ == 0.0) continue;
            const double dx = o.x - ax, dy = o.y - ay, dz = o.z - az;
            ss += o.q / sqrt(dx * dx + dy * dy + dz * dz);
        }
        total += red[k][0] / a.eps_p + ss / a.eps_b;
    }
    const double self = s.occ != 0.0 ? s.q / (a.eps_b * s.a) : 0.0;
    const double phi = a.scale * (total / 6.0 + self);
    double filled = 0.0;
    for (int m = 0; m < a.n_sites; ++m) {
        const SiteRec o = a.site[m];
        if (o.occ != 0.0) filled += 4.0 * pi * o.a * o.a * o.a / 3.0;
    }
    const double S = a.sp.steric ? log(1.0 - filled / a.V_sites) - a.sp.lnGB : 0.0;
    double *out = a.out + (size_t)b * (3 + a.sp.nsp);
    out[0] = phi;
    out[1] = S;
    out[2] = phi - S / s.q;
    for (int i = 0; i < a.sp.nsp; ++i) out[3 + i] = exp(a.sp.lncb[i] - a.sp.z[i] * phi + a.sp.p[i] * S);
}

// Filter region: every SOLVENT node (type 0) with |r - c_b|^2 <= a_b^2 for
// some site (the nearest centre; the lower index on a tie) becomes FIXED
// (type 2) with the value phi_b of that site.  The distance test is evaluated
// without contraction, in the order x, y, z, so that the decision is the
// same as in any plain FP64 evaluation.  count receives the marked nodes.
__global__ __launch_bounds__(256) void k_site_fill(int nx, int ny, int nz, double h, const SiteRec *site,
                                                   const double *phi_b, int n_sites, uint8_t *type,
                                                   double *fixed_value, unsigned long long *count)
{
#pragma clang fp contract(off)
    __shared__ unsigned part[4];
    const size_t N = (size_t)nx * ny * nz;
    unsigned c = 0;
    for (size_t n = (size_t)blockIdx.x * blockDim.x + threadIdx.x; n < N;
         n += (size_t)gridDim.x * blockDim.x) {
        if (type[n] != 0) continue;
        const int i = (int)(n % nx), j = (int)((n / nx) % ny), k = (int)(n / ((size_t)nx * ny));
        int best = -1;
        double bd = 0.0;
        for (int b = 0; b < n_sites; ++b) {
            const SiteRec s = site[b];
            const double dx = (double)i * h - s.x, dy = (double)j * h - s.y, dz = (double)k * h - s.z;
            const double d2 = dx * dx + dy * dy + dz * dz;
            if (d2 <= s.a * s.a && (best < 0 || d2 < bd)) {
                best = b;
                bd = d2;
            }
        }
        if (best >= 0) {
            type[n] = 2;
            fixed_value[n] = phi_b[best];
            ++c;
        }
    }
    for (int o = 32; o > 0; o >>= 1) c += __shfl_xor(c, o, 64);
    if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = c;
    __syncthreads();
    if (threadIdx.x == 0) {
        const unsigned long long tot = (unsigned long long)part[0] + part[1] + part[2] + part[3];
        if (tot) atomicAdd(count, tot);
    }
}

}  // namespace pfk
