// Device code of the singular-charge decomposition (Sec. 3): the Coulomb
// potential phi* of Eq. (5) and its directional derivatives, the list of
// evaluation points the interface needs, the Laplace problem of
// Eqs. (9)-(10) and the right-hand-side terms of the SMIB rows,
// Eqs. (17)-(18), from the flux jump of Eq. (8).
//
// Omega_m is the set of SOLUTE nodes (flag F_SOLUTE).  The interface crosses
// every edge between an Omega_m node and a neighbour outside it, at the
// edge's midpoint.
#pragma once

#include "pf_kernels.h"

namespace pfk {

constexpr int IF_NT = 256;   // threads per workgroup of the interface kernels
constexpr int IF_CT = 256;   // charges per LDS tile of the Coulomb kernels

// Evaluation kinds per node (bit positions of the node's mask):
//   0..5   midpoint of the edge towards face direction d (-x,+x,-y,+y,-z,+z),
//          the neighbour being outside Omega_m: phi* and d phi*/du there;
//   6      the node itself: phi*;
//   8..13  the node, on a Neumann face f = kind - 8: d phi*/du along f.
constexpr int IF_NODE = 6, IF_FACE0 = 8;

__device__ __forceinline__ int face_di(int d) { return d == 0 ? -1 : d == 1 ? 1 : 0; }
__device__ __forceinline__ int face_dj(int d) { return d == 2 ? -1 : d == 3 ? 1 : 0; }
__device__ __forceinline__ int face_dk(int d) { return d == 4 ? -1 : d == 5 ? 1 : 0; }

struct IfGrid {
    int nx, ny, nz;
    double h;
    const uint8_t *flags;
    int want_reg;   // 1: every Omega_m node also needs phi* (for phi* + phi^L)
};

// Mask of the evaluations node n needs (0 outside Omega_m).
__device__ unsigned if_mask(const IfGrid &g, size_t n)
{
    const uint8_t f = g.flags[n];
    if (!(f & F_SOLUTE)) return 0u;
    const int i = (int)(n % g.nx), j = (int)((n / g.nx) % g.ny), k = (int)(n / ((size_t)g.nx * g.ny));
    const bool dir = f & F_DIR_PHI;
    unsigned m = (dir || g.want_reg) ? (1u << IF_NODE) : 0u;
    for (int d = 0; d < 6; ++d) {
        const int a = i + face_di(d), b = j + face_dj(d), c = k + face_dk(d);
        if (a < 0 || a >= g.nx || b < 0 || b >= g.ny || c < 0 || c >= g.nz) {
            // on face d; not Dirichlet, so that face is Neumann for the potential
            if (!dir) m |= 1u << (IF_FACE0 + d);
            continue;
        }
        const size_t nb = (size_t)a + (size_t)g.nx * ((size_t)b + (size_t)g.ny * (size_t)c);
        if (!(g.flags[nb] & F_SOLUTE)) m |= 1u << d;
    }
    return m;
}

// Index of evaluation `kind` of node n in the compact list.
__device__ __forceinline__ unsigned if_entry(const unsigned *off, const uint16_t *mask, size_t n, int kind)
{
    return off[n] + (unsigned)__popc((unsigned)mask[n] & ((1u << kind) - 1u));
}

// Pass 1: per-node masks and per-workgroup entry counts.  Workgroup b covers
// nodes [b IF_NT, (b + 1) IF_NT).
__global__ __launch_bounds__(IF_NT) void k_if_mask(IfGrid g, size_t N, uint16_t *mask, unsigned *blk)
{
    __shared__ unsigned part[IF_NT / 64];
    const size_t n = (size_t)blockIdx.x * IF_NT + threadIdx.x;
    unsigned c = 0;
    if (n < N) {
        const unsigned m = if_mask(g, n);
        mask[n] = (uint16_t)m;
        c = (unsigned)__popc(m);
    }
    for (int o = 32; o > 0; o >>= 1) c += __shfl_xor(c, o, 64);
    if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = c;
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned t = 0;
        for (int w = 0; w < IF_NT / 64; ++w) t += part[w];
        blk[blockIdx.x] = t;
    }
}

// Pass 2 (one workgroup of 1024 threads): exclusive prefix sums of the
// workgroup counts in place; blk[nb] receives the total.
__global__ __launch_bounds__(1024) void k_if_scan(unsigned *blk, int nb)
{
    __shared__ unsigned s[1024];
    const int t = threadIdx.x;
    const int per = (nb + 1023) / 1024;
    const int lo = min(nb, t * per), hi = min(nb, lo + per);
    unsigned sum = 0;
    for (int b = lo; b < hi; ++b) sum += blk[b];
    s[t] = sum;
    __syncthreads();
    for (int o = 1; o < 1024; o <<= 1) {   // inclusive Hillis-Steele scan
        const unsigned v = t >= o ? s[t - o] : 0u;
        __syncthreads();
        s[t] += v;
        __syncthreads();
    }
    unsigned run = s[t] - sum;   // exclusive start of this thread's range
    for (int b = lo; b < hi; ++b) {
        const unsigned c = blk[b];
        blk[b] = run;
        run += c;
    }
    if (t == 1023) blk[nb] = s[1023];
}

// Pass 3: per-node offsets and the compact list of (node << 4 | kind).
__global__ __launch_bounds__(IF_NT) void k_if_list(size_t N, const uint16_t *mask, const unsigned *blk,
                                                   unsigned *off, unsigned long long *code)
{
    __shared__ unsigned s[IF_NT];
    const int t = threadIdx.x;
    const size_t n = (size_t)blockIdx.x * IF_NT + t;
    const unsigned m = n < N ? (unsigned)mask[n] : 0u;
    const unsigned c = (unsigned)__popc(m);
    s[t] = c;
    __syncthreads();
    for (int o = 1; o < IF_NT; o <<= 1) {
        const unsigned v = t >= o ? s[t - o] : 0u;
        __syncthreads();
        s[t] += v;
        __syncthreads();
    }
    if (n >= N) return;
    unsigned e = blk[blockIdx.x] + s[t] - c;
    off[n] = e;
    for (int kind = 0; kind < 16; ++kind)
        if (m & (1u << kind)) code[e++] = ((unsigned long long)n << 4) | (unsigned)kind;
}

// 1/sqrt(x) for x > 0: the hardware estimate refined by one third-order
// step of the series (1 - e)^(-1/2) = 1 + e/2 + 3e^2/8 + ..., e = 1 - x y^2
// (Householder's method of order 3 for y^-2 = x), which takes the estimate's
// relative error e to about e^3.  x = 0 gives a non-finite value.
__device__ __forceinline__ double rsqrt_refined(double x)
{
    const double y = __builtin_amdgcn_rsq(x);
    const double e = fma(-x * y, y, 1.0);
    return fma(y * e, fma(e, 0.375, 0.5), y);
}

// Accumulate sum_j z_j / |r - r_j| and sum_j z_j d/da (1 / |r - r_j|) along
// the thread's axis a over one LDS tile of charges (x, y, z, z_j), in charge
// order.  The point's coordinates come in rotated so that the axis is the
// first one (pa), and each charge's coordinates are read in the same
// rotation (per-lane LDS offsets: lanes of one wave read words of the same
// record, so the reads broadcast without bank conflicts).
__device__ __forceinline__ void coulomb_tile(const double4 *ch, int cnt, double pa, double pb, double pc, int oa,
                                             int ob, int oc, double &phi, double &der)
{
    const char *base = reinterpret_cast<const char *>(ch);
    for (int j = 0; j < cnt; ++j) {
        const char *rec = base + 32 * j;
        const double ca = *reinterpret_cast<const double *>(rec + oa);
        const double cb = *reinterpret_cast<const double *>(rec + ob);
        const double cc = *reinterpret_cast<const double *>(rec + oc);
        const double q = *reinterpret_cast<const double *>(rec + 24);
        const double da = pa - ca, db = pb - cb, dc = pc - cc;
        const double r2 = da * da + db * db + dc * dc;
        const double inv = rsqrt_refined(r2);
        const double qi = q * inv;
        phi += qi;
        der -= qi * (inv * inv) * da;
    }
}

// Byte offsets of the rotated coordinates for axis a (x, y, z = 0, 1, 2).
__device__ __forceinline__ void axis_offsets(int a, int &oa, int &ob, int &oc)
{
    oa = 8 * a;
    ob = 8 * (a == 0 ? 1 : a == 1 ? 2 : 0);
    oc = 8 * (a == 0 ? 2 : a == 1 ? 0 : 1);
}

// Stage charges [t0, t0 + IF_CT) into LDS (every thread of the workgroup takes part).
__device__ __forceinline__ int stage_charges(double4 *tile, const double *charges, int M, int t0)
{
    const int cnt = min(IF_CT, M - t0);
    __syncthreads();
    for (int j = threadIdx.x; j < cnt; j += blockDim.x) {
        const double *c = charges + 4 * (size_t)(t0 + j);
        tile[j] = make_double4(c[0], c[1], c[2], c[3]);
    }
    __syncthreads();
    return cnt;
}

// phi* (V) and its derivative along the entry's direction (D) at every
// entry of the compact list; positions in grid length units from node 0.
__global__ __launch_bounds__(IF_NT) void k_coulomb_entries(size_t E, const unsigned long long *code, int nx, int ny,
                                                           double h, const double *charges, int M, double scale,
                                                           double *V, double *D)
{
    __shared__ double4 tile[IF_CT];
    const size_t e = (size_t)blockIdx.x * IF_NT + threadIdx.x;
    double p[3] = {0, 0, 0}, sgn = 1.0;
    int axis = 0;
    if (e < E) {
        const unsigned long long cd = code[e];
        const size_t n = (size_t)(cd >> 4);
        const int kind = (int)(cd & 15u);
        const int i = (int)(n % nx), j = (int)((n / nx) % ny), k = (int)(n / ((size_t)nx * ny));
        double fi = i, fj = j, fk = k;
        int d = -1;
        if (kind < 6) {
            d = kind;
            fi += 0.5 * face_di(d);
            fj += 0.5 * face_dj(d);
            fk += 0.5 * face_dk(d);
        } else if (kind >= IF_FACE0) {
            d = kind - IF_FACE0;
        }
        p[0] = fi * h;
        p[1] = fj * h;
        p[2] = fk * h;
        if (d >= 0) {
            axis = d >> 1;
            sgn = (d & 1) ? 1.0 : -1.0;
        }
    }
    int oa, ob, oc;
    axis_offsets(axis, oa, ob, oc);
    const double pa = p[axis], pb = p[(axis + 1) % 3], pc = p[(axis + 2) % 3];
    double phi = 0.0, der = 0.0;
    for (int t0 = 0; t0 < M; t0 += IF_CT) {
        const int cnt = stage_charges(tile, charges, M, t0);
        coulomb_tile(tile, cnt, pa, pb, pc, oa, ob, oc, phi, der);
    }
    if (e < E) {
        V[e] = scale * phi;
        D[e] = scale * sgn * der;
    }
}

// phi* or a directional derivative at explicit points: out[p] = potential if
// dir is null or dir[p] == 6, else the derivative along face direction dir[p].
__global__ __launch_bounds__(IF_NT) void k_coulomb_points(size_t n, const double *pts, const int8_t *dir,
                                                          const double *charges, int M, double scale, double *out)
{
    __shared__ double4 tile[IF_CT];
    const size_t p = (size_t)blockIdx.x * IF_NT + threadIdx.x;
    double c[3] = {0, 0, 0};
    int d = 6;
    if (p < n) {
        c[0] = pts[3 * p];
        c[1] = pts[3 * p + 1];
        c[2] = pts[3 * p + 2];
        d = dir ? (int)dir[p] : 6;
    }
    const bool deriv = d >= 0 && d < 6;
    const int axis = deriv ? d >> 1 : 0;
    int oa, ob, oc;
    axis_offsets(axis, oa, ob, oc);
    const double pa = c[axis], pb = c[(axis + 1) % 3], pc = c[(axis + 2) % 3];
    double phi = 0.0, der = 0.0;
    for (int t0 = 0; t0 < M; t0 += IF_CT) {
        const int cnt = stage_charges(tile, charges, M, t0);
        coulomb_tile(tile, cnt, pa, pb, pc, oa, ob, oc, phi, der);
    }
    if (p < n) out[p] = scale * (deriv ? ((d & 1) ? der : -der) : phi);
}

// Laplace problem of Eqs. (9)-(10), unit coefficient, unknowns on the
// Omega_m nodes that are free rows of the potential:
//   - Omega_m nodes on a Dirichlet face: phi^L = -phi* (FIXED, value fv);
//   - an edge leaving Omega_m has its boundary at the midpoint, where the
//     ghost -2 phi*(mid) - phi^L_in closes the row: +1/h^2 on the diagonal
//     (sig), -2 phi*(mid)/h^2 on the right-hand side; the outside node is
//     decoupled (Dirichlet 0);
//   - on a Neumann face, d phi^L/dn = -d phi*/dn: +2 (-d phi*/dn)/h.
__global__ void k_if_laplace(IfGrid g, size_t N, const uint16_t *mask, const unsigned *off, const double *V,
                             const double *D, double *eps1, uint8_t *type, double *fv, double *sig, double *rhs)
{
    const double h = g.h, ih2 = 1.0 / (h * h);
    for (size_t n = (size_t)blockIdx.x * blockDim.x + threadIdx.x; n < N;
         n += (size_t)gridDim.x * blockDim.x) {
        const uint8_t f = g.flags[n];
        const bool inside = f & F_SOLUTE, dir = f & F_DIR_PHI;
        eps1[n] = 1.0;
        type[n] = (inside && !dir) ? 0 : 2;
        fv[n] = (inside && dir) ? -V[if_entry(off, mask, n, IF_NODE)] : 0.0;
        double s = 0.0, r = 0.0;
        if (inside && !dir) {
            const unsigned m = mask[n];
            for (int d = 0; d < 6; ++d) {
                if (m & (1u << (IF_FACE0 + d))) r += 2.0 * (-D[if_entry(off, mask, n, IF_FACE0 + d)]) / h;
                if (m & (1u << d)) {
                    s += ih2;
                    r += -2.0 * ih2 * V[if_entry(off, mask, n, d)];
                }
            }
        }
        sig[n] = s;
        rhs[n] = r;
    }
}

// Flux jump of Eq. (8) on the edge (n, d) leaving Omega_m:
// J = eps_m (d phi*/dn + (phi^L(mid) - phi^L_n) / (h/2)) with phi^L(mid) = -phi*(mid).
__device__ __forceinline__ double if_jump(const unsigned *off, const uint16_t *mask, const double *V,
                                          const double *D, const double *xl, size_t n, int d, double eps_m,
                                          double h)
{
    const unsigned e = if_entry(off, mask, n, d);
    return eps_m * (D[e] + (-V[e] - xl[n]) / (0.5 * h));
}

// Right-hand-side terms of the SMIB rows (Eqs. (17)-(18)) on the free rows
// of the potential: c0/h^2 = -eps_m J / ((eps_m + eps_s) h) inside Omega_m,
// d0/h^2 = -eps_s J / ((eps_m + eps_s) h) outside, per crossing edge in face
// order; and phi_reg = phi* + phi^L on Omega_m (0 elsewhere) when asked.
__global__ void k_if_rhs(IfGrid g, size_t N, const uint16_t *mask, const unsigned *off, const double *V,
                         const double *D, const double *xl, double eps_m, double eps_s, double *b_if,
                         double *phi_reg)
{
    const double h = g.h;
    const double cin = -eps_m / ((eps_m + eps_s) * h), cout = -eps_s / ((eps_m + eps_s) * h);
    for (size_t n = (size_t)blockIdx.x * blockDim.x + threadIdx.x; n < N;
         n += (size_t)gridDim.x * blockDim.x) {
        const uint8_t f = g.flags[n];
        const bool inside = f & F_SOLUTE;
        double b = 0.0;
        if (!(f & F_DIR_PHI)) {
            const int i = (int)(n % g.nx), j = (int)((n / g.nx) % g.ny), k = (int)(n / ((size_t)g.nx * g.ny));
            for (int d = 0; d < 6; ++d) {
                const int a = i + face_di(d), bb = j + face_dj(d), c = k + face_dk(d);
                if (a < 0 || a >= g.nx || bb < 0 || bb >= g.ny || c < 0 || c >= g.nz) continue;
                const size_t nb = (size_t)a + (size_t)g.nx * ((size_t)bb + (size_t)g.ny * (size_t)c);
                const bool nb_inside = g.flags[nb] & F_SOLUTE;
                if (inside && !nb_inside) b += cin * if_jump(off, mask, V, D, xl, n, d, eps_m, h);
                if (!inside && nb_inside) b += cout * if_jump(off, mask, V, D, xl, nb, d ^ 1, eps_m, h);
            }
        }
        b_if[n] = b;
        if (phi_reg) phi_reg[n] = inside ? V[if_entry(off, mask, n, IF_NODE)] + xl[n] : 0.0;
    }
}

// Every node of Omega_m must carry eps_m and every other node eps_s (the
// harmonic-mean faces are then the SMIB matrix).  bad |= 1 on a mismatch.
// eps is the grid's coefficient field, whose sign marks Dirichlet rows.
__global__ void k_if_check(size_t N, const uint8_t *flags, const double *eps, double eps_m, double eps_s,
                           unsigned *bad)
{
    unsigned b = 0;
    for (size_t n = (size_t)blockIdx.x * blockDim.x + threadIdx.x; n < N;
         n += (size_t)gridDim.x * blockDim.x)
        if (fabs(eps[n]) != ((flags[n] & F_SOLUTE) ? eps_m : eps_s)) b = 1u;
    if (b) atomicOr(bad, b);
}

// bad |= 1 where b or (if given) r holds a value that is not finite.
__global__ void k_if_finite(size_t N, const double *b, const double *r, unsigned *bad)
{
    unsigned f = 0;
    for (size_t n = (size_t)blockIdx.x * blockDim.x + threadIdx.x; n < N;
         n += (size_t)gridDim.x * blockDim.x) {
        if (!isfinite(b[n])) f = 1u;
        if (r && !isfinite(r[n])) f = 1u;
    }
    if (f) atomicOr(bad, f);
}

}  // namespace pfk
