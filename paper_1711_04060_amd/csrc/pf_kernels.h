// pf_kernels.h -- gfx950 device kernels of the Poisson-Fermi hot path.
//
// Operator (Sec. 3: 7-point FD of Eqs. (7), (12), (13)):
//   (A x)_i = sum_f c_f (x_i - x_j) + sigma_i x_i,  c_f = 2 e_i e_j / (e_i + e_j) / h^2
// evaluated matrix-free from the nodal coefficient field e (or a constant for
// the PF1 operator), never stored as the seven diagonals of Sec. 4.
//
// Jacobi preconditioning (Sec. 4, Table 3, right-preconditioned with
// M = diag(A) = D) is carried by the storage of the Krylov vectors: every
// vector the stencil reads at a neighbour is kept scaled by D^-1 (p^ = D^-1 p,
// v^, r^, s^, t^ likewise).  Table 3's updates are linear, so they keep their
// form in the scaled vectors (p^ = r^ + beta (p^ - omega v^), s^ = r^ - alpha
// v^, x += alpha p^ + omega s^, r^ = s^ - omega t^), and the products the
// iteration needs become
//   v^ = D^-1 A p^ = p^ - D^-1 sum_f c_f p^_j,
// which use D only at the node itself.  D_i = sum_f c_f + sigma_i is formed
// there from the coefficient field the stencil stages anyway, so no inverse
// diagonal is stored or read.  The inner products use the unscaled values,
// D times the stored one (v = D v^, r = D r^), and are the ones of Table 3.
// Dirichlet rows (identity rows; every Krylov vector is 0 there) are marked
// by the sign bit of the stored coefficient (e < 0), or by a flag byte for the
// constant-coefficient PF1 operator, which reads no coefficient field.

// Stencil kernels march along z.  A workgroup owns a strip of S consecutive
// nodes of the flattened xy plane (m = i + nx*j) and a chunk of z planes.
// For each plane it stages the strip plus one row of halo on each side
// ([m0 - nx, m0 + S + nx)) in LDS; x and y neighbours are read from LDS, the
// z neighbours of the thread's own nodes stay in registers.  Node loads are
// coalesced along x.  Values that depend only on a node (the BiCGSTAB vector
// updates) are computed once per staged node, so the update and the stencil
// fuse into one pass.
//
// BiCGSTAB (Table 3, right Jacobi preconditioning) runs as two fused stencil
// kernels per iteration i:
//   step A: finishes iteration i-1 (x += alpha p^ + omega s^,
//           r^ = s^ - omega t^), forms p^ = r^ + beta (p^ - omega v^) and
//           v^ = D^-1 A p^, and sums shadow . v and r . r;
//   step B: s^ = r^ - alpha v^, t^ = D^-1 A s^, and sums t.s, t.t, s.s,
//           shadow . s and shadow . t.
// beta needs rho_i = shadow . r_i before step A forms p; with r_i = s - omega t
// it is shadow . s - omega shadow . t, known from step B's sums.
//
// Reductions: each workgroup reduces its products in FP64 (wave shuffles,
// then LDS) and stores one partial per quantity.  The next kernel sums the
// partials in every workgroup, in one fixed order (identical bits
// everywhere), and derives the BiCGSTAB scalars on the device before its own
// loads are needed: deterministic, no floating-point atomics, no host round
// trip inside an iteration.  (Taking a completion ticket inside the producer
// instead would need an agent-scope release per workgroup, which writes back
// the XCD's L2 each time; the kernel boundary provides that visibility once.)
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace pfk {

// node flag bits (one byte per node)
enum : uint8_t { F_DIR_PHI = 1, F_DIR_PSI = 2, F_SOLVENT = 4, F_SOLUTE = 8 };

// Device-side BiCGSTAB state (FP64 even when the vectors are FP32).  Values
// produced inside an iteration are kept per iteration parity q = i & 1: a
// kernel of iteration i reads the slots of iteration i-1 (or of its own
// iteration written by an earlier kernel) and its leading workgroup writes
// slot q, so no workgroup reads a slot that its own kernel writes.
struct Scalars {
    double rho[2];     // shadow . r at the start of iteration i
    double alpha[2];   // alpha_i
    double omega[2];   // omega_i
    double rr;         // ||r||^2 of the recurrence, last completed iteration
    double tol2;       // (rel_tol * ||b_lift||)^2
    double rt2;        // ||r_shadow||^2 at the last (re)start
    double red[4];     // sums of the last standalone reduction (residual, relaxation)
    int iter[2];       // iterations completed when iteration i starts
    int iter_done;     // iterations completed (host view)
    int maxit;
    int stop;          // ST_RUN while iterating, else the terminal state
    int stop_a;        // state decided by the last step A, published by the step B after it
    int fresh;         // 1 from a (re)start until step B of the first iteration
    int neg_shift;     // set when a free row of the operator has sigma < 0
    int shift_class;   // set when sigma is one value per palette class on the free rows
};
enum { ST_RUN = 0, ST_CONV = 1, ST_RESTART = 3, ST_NONFINITE = 4, ST_MAXIT = 5 };

// stencil operation selector
enum { OP_SPMV = 0, OP_SPMV_JAC = 1, OP_RESID = 2, OP_BA = 3, OP_BB = 4 };

// how the BiCGSTAB steps get the diagonal shift sigma of the own node: none,
// read from a per-node array, or (palette form) from a table by the node's
// palette class, where sigma is one value per class on the free rows (the
// linearised systems, whose shift is uniform in the solvent and zero in the
// solute)
enum { SIG_NONE = 0, SIG_NODE = 1, SIG_CLASS = 2 };

template <typename T>
struct ZArgs {
    int nx, ny, nz, P;          // P = nx*ny
    int S, KZ, nstrips, G;      // strip length, z planes per workgroup, strips, workgroups
    int lmax;                   // LDS elements per array (>= S + 2*nx)
    T ih2;                      // 1/h^2
    T ceps;                     // CEPS form: constant face coefficient (already / h^2)
    T cdiag, cidiag;            // CEPS form: constant diagonal 6 ceps + sigma and its inverse
    const T *eps;               // coefficient field, sign bit set on Dirichlet rows (non-CEPS)
    const uint8_t *epsi;        // PAL form: palette index of each node's coefficient, bit 7 = Dirichlet row
    const T *ftab;              // PAL form: face coefficients of every palette pair (PAL_MAX^2, / h^2)
    const uint8_t *flags;       // CEPS form: node flags, Dirichlet rows have bit dirbit
    uint8_t dirbit;
    const T *sig;               // SIG_NODE form (BA, BB): diagonal shift sigma
    const T *stab;              // SIG_CLASS form (BA, BB): sigma of each palette class (PAL_MAX)
    const T *x;                 // SPMV*/RESID operand; BA: s^; BB: r^
    const T *y0;                // BA: p^ (previous); BB: v^
    const T *y1;                // BA: v^ (previous)
    const T *y2;                // BA: t^
    const float *rt;            // BA, BB: shadow residual (unscaled, FP32 in both precisions)
    T *xio;                     // BA: iterate x (read and updated in place)
    T *out;                     // SPMV*: y; RESID: r; BA: v^ (new); BB: t^
    T *out_aux;                 // BA: p^ (new); BB: s^
    T *out_r;                   // BA: r^ (new)
    T *sink;                    // SINK_ELEMS doubles: target of masked stores (BA, BB)
    // product and residual extras (FP64 data)
    const double *b;            // RESID: right-hand side
    const double *sigma;        // SPMV*, RESID: diagonal shift or null
    double sig_const;           // used when sigma is null
    const double *dval;         // RESID lift form: Dirichlet values (0 on free rows) or null
    int lift;                   // RESID: use x = Dirichlet values on Dirichlet rows, 0 elsewhere
    float *rt32;                // RESID: optional shadow r, rounded to FP32
    double *rs64;               // RESID: optional Krylov start D^-1 r (FP64)
    float *rs32;                // RESID: optional Krylov start D^-1 r (FP32)
    // reduction and scalars
    Scalars *sc;
    double *partials;           // [G][PSTRIDE] partials written by this kernel
    const double *pin;          // partials of the previous phase (BA: step B, BB: step A)
    int Gin;                    // their count
    int parity;                 // iteration parity q
};

// ------------------------------------------------------------- helpers

// Workgroups are dispatched round-robin over the 8 XCDs (block b runs on XCD
// b % 8).  Remap so that each XCD receives a contiguous range of logical
// tiles: neighbouring strips then share that XCD's L2 for their halos.
__device__ __forceinline__ int xcd_remap(int b, int G)
{
    const int X = 8;
    const int per = G / X, rem = G % X;
    const int xcd = b % X, idx = b / X;
    return (xcd < rem) ? xcd * (per + 1) + idx : rem * (per + 1) + (xcd - rem) * per + idx;
}

// 1/d for d > 0: the hardware reciprocal estimate refined by two Newton steps
// (FP64; within an ulp or so of the correctly rounded quotient) or the
// hardware FP32 reciprocal (1 ulp).
__device__ __forceinline__ double rcp_pos(double d)
{
    double r = __builtin_amdgcn_rcp(d);
    double e = __builtin_fma(-d, r, 1.0);
    r = __builtin_fma(r, e, r);
    e = __builtin_fma(-d, r, 1.0);
    return __builtin_fma(r, e, r);
}
__device__ __forceinline__ float rcp_pos(float d) { return __builtin_amdgcn_rcpf(d); }

// Face coefficient: harmonic mean of the two nodal values, divided by h^2.
template <typename T>
__device__ __forceinline__ T face(T a, T b, T ih2)
{
    return (T(2) * a * b * ih2) * rcp_pos(a + b);
}

__device__ __forceinline__ double wave_sum(double v)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
    return v;
}

__device__ __forceinline__ double wave_max(double v)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_down(v, off, 64));
    return v;
}

// Partials: PSTRIDE doubles per workgroup (up to PSTRIDE quantities).
constexpr int PSTRIDE = 8;

// The BiCGSTAB stencil steps issue every store unconditionally: a store whose
// node is outside the tile (or a step past its last plane) goes to a sink
// slot of the thread instead.  Stores count in the same wait counter as
// loads, and a store under a branch would make the compiler assume the
// shorter path and wait for loads still meant to be in flight.
constexpr int SINK_ELEMS = 2048;   // >= threads * nodes per thread

// Reduce NQ per-thread values over the workgroup; thread 0 gets the result.
template <int NQ, int NT, bool MAX = false>
__device__ __forceinline__ void block_reduce(double (&v)[NQ])
{
    __shared__ double red[NT / 64][NQ];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
        double s = MAX ? wave_max(v[q]) : wave_sum(v[q]);
        if (lane == 0) red[w][q] = s;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
#pragma unroll
        for (int q = 0; q < NQ; ++q) {
            double s = red[0][q];
            for (int i = 1; i < NT / 64; ++i) s = MAX ? fmax(s, red[i][q]) : s + red[i][q];
            v[q] = s;
        }
    }
}

// Store the workgroup partials (thread 0 holds the reduced values).
template <int NQ>
__device__ __forceinline__ void store_partials(const double (&v)[NQ], double *partials, int slot)
{
    if (threadIdx.x == 0) {
#pragma unroll
        for (int q = 0; q < NQ; ++q) partials[slot * PSTRIDE + q] = v[q];
    }
}

// Fixed-order sum (or max) of the G partials, run by a finalize workgroup.
template <int NQ, int NT, bool MAX = false>
__device__ __forceinline__ void final_reduce(double (&v)[NQ], const double *partials, int G)
{
#pragma unroll
    for (int q = 0; q < NQ; ++q) v[q] = 0.0;
    for (int i = threadIdx.x; i < G; i += NT) {
#pragma unroll
        for (int q = 0; q < NQ; ++q) {
            const double p = partials[i * PSTRIDE + q];
            v[q] = MAX ? fmax(v[q], p) : v[q] + p;
        }
    }
    __syncthreads();
    block_reduce<NQ, NT, MAX>(v);
}

__device__ __forceinline__ bool finite(double x) { return __builtin_isfinite(x); }

// Sum of NQ quantities over G partials in one fixed order whatever the
// workgroup size (lanes 0..255 each add the partials lane, lane + 256, ...
// in increasing order, then a fixed tree), so every workgroup of a consumer
// kernel and the one-workgroup finalize kernel obtain identical bits.  The
// loads are split from the sum so that a kernel can issue them together with
// its first data loads: the first PJ*256 partials are loaded without a loop
// (indices past G load slot 0 and are not added).
constexpr int PJ = 4;

template <int NQ>
struct PartLoad {
    double l[PJ][NQ];
};

template <int NQ>
__device__ __forceinline__ void load_partials(PartLoad<NQ> &pl, const double *partials, int G)
{
    const int lane = threadIdx.x & 255;
#pragma unroll
    for (int j = 0; j < PJ; ++j) {
        const int i = lane + 256 * j;
        const int ic = i < G ? i : 0;
#pragma unroll
        for (int q = 0; q < NQ; ++q) pl.l[j][q] = partials[ic * PSTRIDE + q];
    }
}

// Every thread receives the result.
template <int NQ>
__device__ __forceinline__ void sum_loaded_partials(double (&tot)[NQ], const PartLoad<NQ> &pl,
                                                    const double *partials, int G)
{
    __shared__ double sred[4][NQ];
    __shared__ double sout[NQ];
    double v[NQ];
#pragma unroll
    for (int q = 0; q < NQ; ++q) v[q] = 0.0;
    if (threadIdx.x < 256) {
        const int lane = threadIdx.x;
#pragma unroll
        for (int j = 0; j < PJ; ++j) {
            if (lane + 256 * j < G) {
#pragma unroll
                for (int q = 0; q < NQ; ++q) v[q] += pl.l[j][q];
            }
        }
        for (int i = lane + 256 * PJ; i < G; i += 256) {
#pragma unroll
            for (int q = 0; q < NQ; ++q) v[q] += partials[i * PSTRIDE + q];
        }
    }
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
        const double sw = wave_sum(v[q]);
        if (lane == 0 && w < 4) sred[w][q] = sw;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
#pragma unroll
        for (int q = 0; q < NQ; ++q) sout[q] = ((sred[0][q] + sred[1][q]) + sred[2][q]) + sred[3][q];
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < NQ; ++q) tot[q] = sout[q];
}

template <int NQ>
__device__ __forceinline__ void sum_partials(double (&tot)[NQ], const double *partials, int G)
{
    PartLoad<NQ> pl;
    load_partials<NQ>(pl, partials, G);
    sum_loaded_partials<NQ>(tot, pl, partials, G);
}

// Start of step A of iteration i (parity q).  Step A also finishes iteration
// i-1: its x, r update (Table 3 steps 16, 17) needs omega_{i-1} = t.s / t.t
// (step 15), and the p update needs beta_i (step 8), i.e. rho_i = shadow . r_i
// (step 4).  Since r_i = s - omega t, rho_i = shadow . s - omega shadow . t
// from step B's sums, so no pass over r_i has to finish first; ||r_i||^2 for
// the stop test is summed from r_i itself in this step and tested by step B.
// tot: t.s, t.t, s.s, shadow . s, shadow . t of iteration i-1.
struct FinB {
    double alpha, omega, beta, rho, rr;
    int iter, stop;
    bool update;   // apply the x, r update of iteration i-1
};

__device__ __forceinline__ FinB fin_b(const Scalars *sc, const double (&tot)[5], int q)
{
    const int qp = q ^ 1;
    const double ts = tot[0], tt = tot[1], ss = tot[2], rs = tot[3], rtt = tot[4];
    FinB f{};
    f.alpha = sc->alpha[qp];
    f.iter = sc->iter[qp] + 1;
    f.stop = ST_RUN;
    f.update = true;
    if (!finite(ts) || !finite(tt) || !finite(ss) || !finite(rs) || !finite(rtt)) {
        f.stop = ST_NONFINITE;
        f.update = false;
        return f;
    }
    if (ss <= sc->tol2) {
        // ||s|| already meets the tolerance: x += alpha M^-1 p, r = s
        f.omega = 0.0;
        f.rho = rs;
        f.rr = ss;
        f.stop = ST_CONV;
        return f;
    }
    if (tt == 0.0) {
        f.stop = ST_RESTART;
        f.update = false;
        return f;
    }
    f.omega = ts / tt;
    f.rho = rs - f.omega * rtt;
    f.rr = fmax(0.0, ss - 2.0 * f.omega * ts + f.omega * f.omega * tt);
    if (f.rr > sc->tol2) {   // otherwise step B decides on the summed ||r_i||^2
        if (f.iter >= sc->maxit) {
            f.stop = ST_MAXIT;
            return f;
        }
        if (f.omega == 0.0 || fabs(f.rho) < 1e-300 || f.rho * f.rho < 1e-28 * sc->rt2 * f.rr) {
            f.stop = ST_RESTART;   // shadow residual nearly orthogonal to r
            return f;
        }
    }
    if (f.omega != 0.0 && sc->rho[qp] != 0.0) f.beta = (f.rho / sc->rho[qp]) * (f.alpha / f.omega);
    return f;
}

// Written by the leading workgroup.  The stop state goes to stop_a, not stop:
// the other workgroups of this step A test stop on entry and must still apply
// the x, r update when the state ends the run.
__device__ __forceinline__ void fin_b_store(Scalars *sc, const FinB &f, int q)
{
    sc->stop_a = f.stop;
    if (!f.update) return;
    sc->omega[q ^ 1] = f.omega;
    sc->rho[q] = f.rho;
    sc->iter[q] = f.iter;
    sc->iter_done = f.iter;
    sc->rr = f.rr;
}

// --------------------------------------------------- z-marching stencil

// |x| (a source modifier of the instruction that consumes it)
__device__ __forceinline__ double absT(double x) { return __builtin_fabs(x); }
__device__ __forceinline__ float absT(float x) { return __builtin_fabsf(x); }

// Loading (raw) and staging are split so that the loads of a plane can be
// issued two march steps before their values are needed.  OWN loads add what
// only the node's own outputs read (the shadow residual; BA: x; the shift
// sigma in the SIG form; the flag byte in the CEPS form).
template <typename T>
struct Raw {
    T e, x0, x1, x2, x3, x4, sg;
    float t;
    uint8_t f, ei;
};

// Palette form of the coefficient field: fields with at most PAL_MAX
// distinct values (the piecewise-constant dielectric of Eq. (7): eps_m in the
// solute region, eps_s in the solvent) are stored as one byte per node, the
// value's palette index with the Dirichlet mark in bit 7, and the face
// coefficient of each pair of palette values is precomputed (a table staged
// in LDS).  The stencil then stages a code per node instead of the value:
// +-(index + 1), negative on Dirichlet rows.
constexpr int PAL_MAX = 16;
constexpr int FTAB = PAL_MAX * PAL_MAX;

template <bool PAL, typename T>
__device__ __forceinline__ T coef(const Raw<T> &w)
{
    if constexpr (PAL) {
        const T c = (T)((w.ei & (PAL_MAX - 1)) + 1);
        return (w.ei & 128) ? -c : c;
    } else {
        return w.e;
    }
}

// Load of element g (g < 2^29 nodes, so the byte offset fits 32 bits): the
// array base stays in scalar registers and one 32-bit vector offset serves
// every array of the node.
template <typename U>
__device__ __forceinline__ U ldx(const U *base, unsigned g)
{
    return *reinterpret_cast<const U *>(reinterpret_cast<const char *>(base) + g * (unsigned)sizeof(U));
}

template <int OP, typename T, bool CEPS, int SIG, bool PAL, bool OWN>
__device__ __forceinline__ void load_raw(const ZArgs<T> &a, unsigned g, Raw<T> &w)
{
    if constexpr (PAL) w.ei = ldx(a.epsi, g);
    else if constexpr (!CEPS) w.e = ldx(a.eps, g);
    if constexpr (CEPS && OWN) w.f = a.flags[g];
    if constexpr (SIG == SIG_NODE && OWN) w.sg = ldx(a.sig, g);
    if constexpr (OP == OP_SPMV || OP == OP_SPMV_JAC) {
        w.x0 = ldx(a.x, g);
    } else if constexpr (OP == OP_RESID) {
        if (a.lift) w.x0 = a.dval ? (T)ldx(a.dval, g) : T(0);
        else w.x0 = ldx(a.x, g);
    } else if constexpr (OP == OP_BA) {
        w.x0 = ldx(a.x, g);    // s^
        w.x1 = ldx(a.y0, g);   // p^ (previous)
        w.x2 = ldx(a.y1, g);   // v^ (previous)
        w.x3 = ldx(a.y2, g);   // t^
        if constexpr (OWN) {
            w.x4 = ldx((const T *)a.xio, g);
            w.t = ldx(a.rt, g);
        }
    } else {
        w.x0 = ldx(a.x, g);    // r^
        w.x1 = ldx(a.y0, g);   // v^
        if constexpr (OWN) w.t = ldx(a.rt, g);
    }
}

// The value the stencil reads at a staged node (also the node's own stored
// output where the step has one).
template <int OP, typename T>
__device__ __forceinline__ T stage_raw(const Raw<T> &w, double alpha, double omega, double beta)
{
    if constexpr (OP == OP_BA) {
        // r^ = s^ - omega t^ (Table 3 step 17 of the previous iteration), then
        // p^ = r^ + beta (p^ - omega v^)   (step 9)
        const T r = w.x0 - (T)omega * w.x3;
        return r + (T)beta * (w.x1 - (T)omega * w.x2);
    } else if constexpr (OP == OP_BB) {
        // s^ = r^ - alpha v^   (Table 3 step 13)
        return w.x0 - (T)alpha * w.x1;
    } else {
        return w.x0;
    }
}

// Store target chosen without a branch: the target is `real` plus a byte
// offset (0, or the distance to the sink slot) that an empty asm hides from
// the compiler, which would otherwise turn the choice back into two
// conditional stores.  The base stays the global pointer, so the store stays
// a global (not flat) store.
template <typename T>
__device__ __forceinline__ T *pick(bool keep, T *real, T *sink)
{
    long d = keep ? 0L : (long)(reinterpret_cast<char *>(sink) - reinterpret_cast<char *>(real));
    asm volatile("" : "+v"(d));
    return reinterpret_cast<T *>(reinterpret_cast<char *>(real) + d);
}

// A workgroup-uniform double moved into scalar registers (it then takes no
// vector registers in the march loop and carries no pending vector load).
__device__ __forceinline__ double uniform(double x)
{
    const unsigned long long b = __builtin_bit_cast(unsigned long long, x);
    const unsigned lo = __builtin_amdgcn_readfirstlane((unsigned)b);
    const unsigned hi = __builtin_amdgcn_readfirstlane((unsigned)(b >> 32));
    return __builtin_bit_cast(double, ((unsigned long long)hi << 32) | lo);
}

// A store to the thread's sink slot that the compiler can neither drop nor
// merge with another (its address carries a hidden zero offset).
template <typename T>
__device__ __forceinline__ void sink_store(T *slot)
{
    long d = 0;
    asm volatile("" : "+v"(d));
    *reinterpret_cast<T *>(reinterpret_cast<char *>(slot) + d) = T(0);
}

// Step A's own-node update of the previous iteration (Table 3 steps 16, 17)
// in the scaled vectors: x += alpha p^ + omega s^, r^ = s^ - omega t^.
template <typename T>
__device__ __forceinline__ void stage_xr(const Raw<T> &w, T &xn, T &rn, double alpha, double omega)
{
    rn = w.x0 - (T)omega * w.x3;
    xn = w.x4 + (T)alpha * w.x1 + (T)omega * w.x0;
}

// A staged value materialised in a register of its own at this point of the
// step.  Without it the compiler keeps a staged value in the register its
// load wrote, or sinks its arithmetic to the value's first use (after the
// next loads were issued); either way the load register set stays live
// across the refill, the refill needs other registers, and the loop latch
// then waits for every load in flight to move them back.  The volatile asm
// is kept in program order with the scheduling barrier that follows it.
template <typename T>
__device__ __forceinline__ T own_reg(T x)
{
    T y;
    if constexpr (sizeof(T) == 8) asm volatile("v_mov_b64 %0, %1" : "=v"(y) : "v"(x));
    else asm volatile("v_mov_b32 %0, %1" : "=v"(y) : "v"(x));
    return y;
}
__device__ __forceinline__ uint8_t own_reg(uint8_t x)
{
    unsigned y;
    asm volatile("v_mov_b32 %0, %1" : "=v"(y) : "v"((unsigned)x));
    return (uint8_t)y;
}

// One workgroup's tile: logical tile index lb (strip, z-chunk) and partial
// slot `slot` of the system described by a.
//
// Memory pipeline: the raw loads of the next DEPTH planes are in flight
// while plane k is computed, in DEPTH register sets used in turn (for
// DEPTH = 2 the march is unrolled by two so that each set keeps fixed
// registers; DEPTH = 1 needs half the registers).  Every load is
// issued unconditionally with its plane clamped into the tile's range and
// its node clamped into the strip, so the number of loads per step is fixed
// and the wait before staging a plane covers only that plane's loads.
template <int OP, typename T, bool CEPS, int SIG, bool PAL, int NT, int PPT, bool WIDE, int DEPTH>
__device__ __forceinline__ void zmarch_tile(const ZArgs<T> &a, const int lb, const int slot)
{
    static_assert(!SIG || OP == OP_BA || OP == OP_BB, "the SIG form is a BiCGSTAB step form");
    static_assert(!(SIG && CEPS), "the CEPS form has a constant shift");
    static_assert(!(PAL && CEPS), "the CEPS form reads no coefficient field");
    static_assert(SIG != SIG_CLASS || PAL, "the class shift is indexed by the palette");
    // halo nodes per thread kept in registers (both halo rows fit when
    // 2 nx <= HMAX*NT); the WIDE form stages the rest in a slower
    // synchronous loop, for planes wider than that
    constexpr int HMAX = (NT >= 512) ? 1 : 2;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    // quantities this kernel sums (BA: shadow . v, r . r; BB: t.s, t.t, s.s,
    // shadow . s, shadow . t) and those of the previous phase's partials
    constexpr int NQ = (OP == OP_BB) ? 5 : (OP == OP_BA) ? 2 : 1;
    constexpr int NQP = (OP == OP_BB) ? 2 : 5;
    constexpr bool SCAL = (OP == OP_BA || OP == OP_BB);

    Scalars *sc = a.sc;
    int fresh = 0;
    if constexpr (SCAL) {
        // One read of the stop state for the whole workgroup: step B's
        // leading workgroup may set it while another workgroup of the same
        // system starts, and waves that read different values would leave
        // the tile apart (in the persistent batched walk the next barrier
        // they meet belongs to another tile).
        __shared__ int stop_seen;
        __syncthreads();   // the previous tile of this workgroup is done with stop_seen
        if (threadIdx.x == 0) stop_seen = sc->stop;
        __syncthreads();
        if (stop_seen != ST_RUN) return;
        if constexpr (OP == OP_BA) fresh = sc->fresh;
    }

    const int strip = lb % a.nstrips, zc = lb / a.nstrips;
    const int nx = a.nx, ny = a.ny, nz = a.nz, P = a.P;
    const int m0 = strip * a.S;
    const int k0 = zc * a.KZ, k1 = min(nz, k0 + a.KZ);
    const int lo = max(0, m0 - nx), hi = min(P, m0 + a.S + nx);
    const int mend = min(P, m0 + a.S);
    const int nhl = m0 - lo, nhalo = nhl + (hi - mend);
    const int kown_hi = min(k1, nz - 1);   // own planes loaded: k0-1 .. k1 (within the grid)
    const int khal_hi = k1 - 1;            // halo planes loaded: k0 .. k1-1
    const T ih2 = a.ih2;
    const size_t Ps = (size_t)P;

    // own nodes and their LDS neighbour offsets (mirror ghosts at the faces;
    // rows on Dirichlet faces are masked, so the mirror only matters on
    // Neumann faces); nodes past the strip end stand in for node m0
    int om[PPT], ox[PPT], oxm[PPT], oxp[PPT], oym[PPT], oyp[PPT];
    bool ok[PPT];
#pragma unroll
    for (int q = 0; q < PPT; ++q) {
        const int m = m0 + threadIdx.x + q * NT;
        ok[q] = m < mend;
        const int mm = ok[q] ? m : m0;
        const int j = mm / nx, i = mm - j * nx;
        om[q] = mm;
        ox[q] = mm - lo;
        oxm[q] = ((i > 0) ? mm - 1 : mm + 1) - lo;
        oxp[q] = ((i < nx - 1) ? mm + 1 : mm - 1) - lo;
        oym[q] = ((j > 0) ? mm - nx : mm + nx) - lo;
        oyp[q] = ((j < ny - 1) ? mm + nx : mm - nx) - lo;
    }
    // halo nodes of this thread (plane-local index; unused slots repeat lo)
    int hm[HMAX];
    bool hok[HMAX];
#pragma unroll
    for (int u = 0; u < HMAX; ++u) {
        const int hI = threadIdx.x + u * NT;
        hok[u] = hI < nhalo;
        hm[u] = !hok[u] ? lo : (hI < nhl) ? lo + hI : mend + (hI - nhl);
    }
    const unsigned Pu = (unsigned)P;
    auto gown = [&](int q, int k) { return (unsigned)om[q] + Pu * (unsigned)min(k, kown_hi); };
    auto ghal = [&](int u, int k) { return (unsigned)hm[u] + Pu * (unsigned)min(k, khal_hi); };

    // the face table: loaded first, stored behind the two LDS planes once
    // the plane loads are out, read after the barrier before the first output
    T *lftab = reinterpret_cast<T *>(smem_raw) + 4 * a.lmax;
    T *lstab = lftab + FTAB;   // SIG_CLASS: the shift of each palette class
    T ftv = T(0), stv = T(0);
    if constexpr (PAL) ftv = a.ftab[threadIdx.x & (FTAB - 1)];
    if constexpr (SIG == SIG_CLASS) stv = a.stab[threadIdx.x & (PAL_MAX - 1)];

    // ---- prologue loads: the previous phase's partials, then planes k0-1,
    //      k0 (own), k0 (halo), and the raw sets of planes k0+1 and k0+2
    PartLoad<NQP> pl;
    if constexpr (SCAL) load_partials<NQP>(pl, a.pin, a.Gin);
    __builtin_amdgcn_sched_barrier(0);
    Raw<T> rp[PPT], rc[PPT], hc[HMAX];
    Raw<T> rA[PPT], hA[HMAX], rB[PPT], hB[HMAX];
#pragma unroll
    for (int q = 0; q < PPT; ++q) {
        load_raw<OP, T, CEPS, SIG, PAL, true>(a, gown(q, k0), rc[q]);
        load_raw<OP, T, CEPS, SIG, PAL, false>(a, gown(q, max(k0 - 1, 0)), rp[q]);
    }
#pragma unroll
    for (int u = 0; u < HMAX; ++u) load_raw<OP, T, CEPS, SIG, PAL, false>(a, ghal(u, k0), hc[u]);
    // The sets go out in the order of the march steps (own, halo, then as
    // many stores as a step makes, here to the sink), so that at the loop's
    // first wait the loads of each set are as far from the newest event as in
    // every later step: the compiler takes the nearer of the two, and a
    // nearer distance here would make every step wait for loads meant to
    // stay in flight.
    constexpr int NST = PPT * ((OP == OP_BA) ? 4 : (OP == OP_BB) ? 2 : (OP == OP_SPMV_JAC) ? 1 : 0);
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int q = 0; q < PPT; ++q) load_raw<OP, T, CEPS, SIG, PAL, true>(a, gown(q, k0 + 1), rA[q]);
#pragma unroll
    for (int u = 0; u < HMAX; ++u) load_raw<OP, T, CEPS, SIG, PAL, false>(a, ghal(u, k0 + 1), hA[u]);
#pragma unroll
    for (int j = 0; j < NST; ++j) sink_store(a.sink + threadIdx.x);
    __builtin_amdgcn_sched_barrier(0);
    if constexpr (DEPTH == 2) {
#pragma unroll
        for (int q = 0; q < PPT; ++q) load_raw<OP, T, CEPS, SIG, PAL, true>(a, gown(q, k0 + 2), rB[q]);
#pragma unroll
        for (int u = 0; u < HMAX; ++u) load_raw<OP, T, CEPS, SIG, PAL, false>(a, ghal(u, k0 + 2), hB[u]);
#pragma unroll
        for (int j = 0; j < NST; ++j) sink_store(a.sink + threadIdx.x);
        __builtin_amdgcn_sched_barrier(0);
    }

    // ---- scalars of this step (while the plane loads are in flight)
    // alpha, omega: of the previous iteration in BA (its x, r update), of
    // this iteration in BB
    double alpha = 0, omega = 0, beta = 0;
    if constexpr (OP == OP_BA) {
        // finish step B of the previous iteration (a fresh start has r^ in s^,
        // t^ = 0, p^ = v^ = 0: with alpha = omega = beta = 0 the update keeps x
        // and sets p^ = r^)
        if (!fresh) {
            double tot[5];
            sum_loaded_partials<5>(tot, pl, a.pin, a.Gin);
            const FinB f = fin_b(sc, tot, a.parity);
            if (lb == 0 && threadIdx.x == 0) fin_b_store(sc, f, a.parity);
            if (!f.update) return;
            alpha = f.alpha;
            omega = f.omega;
            beta = (f.stop == ST_RUN) ? f.beta : 0.0;
        } else if (lb == 0 && threadIdx.x == 0) {
            sc->stop_a = ST_RUN;
        }
    } else if constexpr (OP == OP_BB) {
        // finish step A: the stop test on ||r_i||^2, then
        // alpha_i = rho_i / (shadow . v)   (Table 3 step 12)
        double tot[2];
        sum_loaded_partials<2>(tot, pl, a.pin, a.Gin);
        const double rtv = tot[0], rr = tot[1];
        int st = sc->stop_a;
        if (st == ST_RUN) {
            if (!finite(rtv) || !finite(rr)) st = ST_NONFINITE;
            else if (rr <= sc->tol2) st = ST_CONV;
            else if (sc->iter[a.parity] >= sc->maxit) st = ST_MAXIT;
            else if (rtv == 0.0) st = ST_RESTART;
            else alpha = sc->rho[a.parity] / rtv;
        }
        if (lb == 0 && threadIdx.x == 0) {
            sc->alpha[a.parity] = alpha;
            sc->rr = rr;
            sc->fresh = 0;
            if (st != ST_RUN) sc->stop = st;
        }
        if (st != ST_RUN) return;
    }
    alpha = uniform(alpha);
    omega = uniform(omega);
    beta = uniform(beta);
    if constexpr (PAL) {
        if (threadIdx.x < FTAB) lftab[threadIdx.x] = ftv;
        if constexpr (SIG == SIG_CLASS) {
            if (threadIdx.x < PAL_MAX) lstab[threadIdx.x] = stv;
        }
        __syncthreads();   // table visible before the first output
    }

    // two LDS planes (double buffer) of staged values and coefficients
    T *lval0 = reinterpret_cast<T *>(smem_raw);
    T *leps0 = lval0 + a.lmax;
    T *lval1 = leps0 + a.lmax;
    T *leps1 = lval1 + a.lmax;

    T vp[PPT], vc[PPT], vn[PPT];   // staged value, planes k-1, k, k+1
    T ep[PPT], ec[PPT], en[PPT];   // coefficient field (signed), planes k-1, k, k+1
    float tc[PPT], tn[PPT];        // shadow residual (BA, BB), planes k, k+1
    T rc_[PPT], rn_[PPT];          // BA: r^ of planes k, k+1
    T sc_[PPT], sn_[PPT];          // SIG_NODE: sigma of planes k, k+1
    uint8_t fc[PPT], fn[PPT];      // CEPS: flag bytes of planes k, k+1
    double acc[NQ];
#pragma unroll
    for (int q = 0; q < NQ; ++q) acc[q] = 0.0;

    // ---- stage plane k0 (registers + LDS buffer 0) and plane k0-1 (registers)
#pragma unroll
    for (int q = 0; q < PPT; ++q) {
        vc[q] = stage_raw<OP, T>(rc[q], alpha, omega, beta);
        ec[q] = CEPS ? T(0) : coef<PAL>(rc[q]);
        tc[q] = SCAL ? rc[q].t : 0.0f;
        sc_[q] = SIG == SIG_NODE ? rc[q].sg : T(0);
        fc[q] = CEPS ? rc[q].f : (uint8_t)0;
        vp[q] = stage_raw<OP, T>(rp[q], alpha, omega, beta);
        ep[q] = CEPS ? T(0) : coef<PAL>(rp[q]);
        vn[q] = en[q] = rn_[q] = sn_[q] = T(0);
        tn[q] = 0.0f;
        fn[q] = 0;
        rc_[q] = T(0);
        if constexpr (OP == OP_BA) {
            T xn;
            stage_xr<T>(rc[q], xn, rc_[q], alpha, omega);
            if (ok[q]) {
                const unsigned g0 = gown(q, k0);
                a.xio[g0] = xn;
                a.out_r[g0] = rc_[q];
            }
        }
        if (ok[q]) {
            if constexpr (SCAL) a.out_aux[gown(q, k0)] = vc[q];
            lval0[ox[q]] = vc[q];
            if constexpr (!CEPS) leps0[ox[q]] = ec[q];
        }
    }
#pragma unroll
    for (int u = 0; u < HMAX; ++u) {
        if (hok[u]) {
            lval0[hm[u] - lo] = stage_raw<OP, T>(hc[u], alpha, omega, beta);
            if constexpr (!CEPS) leps0[hm[u] - lo] = coef<PAL>(hc[u]);
        }
    }
    if (WIDE && nhalo > HMAX * NT) {
        for (int hI = threadIdx.x + HMAX * NT; hI < nhalo; hI += NT) {
            const int m = (hI < nhl) ? lo + hI : mend + (hI - nhl);
            Raw<T> w;
            load_raw<OP, T, CEPS, false, PAL, false>(a, (unsigned)m + Pu * (unsigned)k0, w);
            lval0[m - lo] = stage_raw<OP, T>(w, alpha, omega, beta);
            if constexpr (!CEPS) leps0[m - lo] = coef<PAL>(w);
        }
    }
    __syncthreads();

    int cur = 0;
    T hv[HMAX], he[HMAX];
    // One march step: output plane k from LDS buffer `cur`; ro / rh hold the
    // raw loads of plane k+1 and are refilled with plane k+1+DEPTH.  The march runs
    // in pairs of steps; a step past the tile's last plane (odd plane count)
    // computes but stores nothing.
    auto step = [&](const int k, Raw<T>(&ro)[PPT], Raw<T>(&rh)[HMAX]) {
        const bool live = k < k1;
        const bool has_up = (k + 1) < nz;
        const bool stage_next = (k + 1) < k1;
        // (1) stage plane k+1 from the raw loads issued DEPTH steps ago
        T xn[PPT];   // BA: updated x of plane k+1
#pragma unroll
        for (int q = 0; q < PPT; ++q) {
            vn[q] = own_reg(stage_raw<OP, T>(ro[q], alpha, omega, beta));
            if constexpr (!CEPS) en[q] = own_reg(coef<PAL>(ro[q]));
            if constexpr (CEPS) fn[q] = own_reg(ro[q].f);
            if constexpr (SIG == SIG_NODE) sn_[q] = own_reg(ro[q].sg);
            if constexpr (SCAL) tn[q] = own_reg(ro[q].t);
            if constexpr (OP == OP_BA) {
                stage_xr<T>(ro[q], xn[q], rn_[q], alpha, omega);
                xn[q] = own_reg(xn[q]);
                rn_[q] = own_reg(rn_[q]);
            }
        }
#pragma unroll
        for (int u = 0; u < HMAX; ++u) {
            hv[u] = own_reg(stage_raw<OP, T>(rh[u], alpha, omega, beta));
            if constexpr (!CEPS) he[u] = own_reg(coef<PAL>(rh[u]));
        }
        // (2) refill the set with plane k+1+DEPTH (clamped: re-reads of a plane
        //     already loaded near the tile's end hit the cache).  The
        //     scheduling barrier keeps the refill after the reads of the set
        //     above, so the loads can reuse its registers.
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int q = 0; q < PPT; ++q) load_raw<OP, T, CEPS, SIG, PAL, true>(a, gown(q, k + 1 + DEPTH), ro[q]);
#pragma unroll
        for (int u = 0; u < HMAX; ++u) load_raw<OP, T, CEPS, SIG, PAL, false>(a, ghal(u, k + 1 + DEPTH), rh[u]);
        if constexpr (SCAL) {
            // own outputs of plane k+1 when the tile owns it (else the sink)
#pragma unroll
            for (int q = 0; q < PPT; ++q) {
                const bool keep = stage_next && ok[q];
                const unsigned g1 = gown(q, k + 1);
                T *sk = a.sink + threadIdx.x + q * NT;
                *pick(keep, a.out_aux + g1, sk) = vn[q];
                if constexpr (OP == OP_BA) {
                    *pick(keep, a.xio + g1, sk) = xn[q];
                    *pick(keep, a.out_r + g1, sk) = rn_[q];
                }
            }
        }
        // mirror ghosts across the z faces, written into the register planes
        // (uniform branches, static indices)
        T vu[PPT], eu[PPT];
#pragma unroll
        for (int q = 0; q < PPT; ++q) { vu[q] = has_up ? vn[q] : vp[q]; eu[q] = has_up ? en[q] : ep[q]; }
        if (k == 0) {
#pragma unroll
            for (int q = 0; q < PPT; ++q) { vp[q] = vu[q]; ep[q] = eu[q]; }
        }
        // (3) output for plane k (live: uniform)
        const T *lv = cur ? lval1 : lval0;
        const T *le = cur ? leps1 : leps0;
#pragma unroll
        for (int q = 0; q < PPT; ++q) {
            const size_t g = (size_t)om[q] + Ps * k;
            T sum, D;
            bool dir;
            if constexpr (CEPS) {
                const T c = a.ceps;
                sum = c * (lv[oxm[q]] + lv[oxp[q]] + lv[oym[q]] + lv[oyp[q]] + vu[q] + vp[q]);
                D = a.cdiag;
                dir = (fc[q] & a.dirbit) != 0;
            } else if constexpr (PAL) {
                const int own = (int)absT(ec[q]) - 1;
                const T *row = lftab + own * PAL_MAX;
                const T c0 = row[(int)absT(le[oxm[q]]) - 1], c1 = row[(int)absT(le[oxp[q]]) - 1];
                const T c2 = row[(int)absT(le[oym[q]]) - 1], c3 = row[(int)absT(le[oyp[q]]) - 1];
                const T c4 = row[(int)absT(ep[q]) - 1], c5 = row[(int)absT(eu[q]) - 1];
                sum = c0 * lv[oxm[q]] + c1 * lv[oxp[q]] + c2 * lv[oym[q]] + c3 * lv[oyp[q]] + c4 * vp[q] +
                      c5 * vu[q];
                D = ((c0 + c1) + (c2 + c3)) + (c4 + c5);
                if constexpr (SIG == SIG_NODE) D += sc_[q];
                if constexpr (SIG == SIG_CLASS) D += lstab[own];
                dir = ec[q] < T(0);
            } else {
                const T e = absT(ec[q]);
                const T c0 = face(e, absT(le[oxm[q]]), ih2), c1 = face(e, absT(le[oxp[q]]), ih2);
                const T c2 = face(e, absT(le[oym[q]]), ih2), c3 = face(e, absT(le[oyp[q]]), ih2);
                const T c4 = face(e, absT(ep[q]), ih2), c5 = face(e, absT(eu[q]), ih2);
                sum = c0 * lv[oxm[q]] + c1 * lv[oxp[q]] + c2 * lv[oym[q]] + c3 * lv[oyp[q]] + c4 * vp[q] +
                      c5 * vu[q];
                D = ((c0 + c1) + (c2 + c3)) + (c4 + c5);
                if constexpr (SIG == SIG_NODE) D += sc_[q];
                dir = ec[q] < T(0);
            }
            if constexpr (OP == OP_SPMV) {
                if (live && ok[q]) {
                    const T Dt = CEPS ? D : D + (T)(a.sigma ? a.sigma[g] : a.sig_const);
                    a.out[g] = dir ? vc[q] : Dt * vc[q] - sum;
                }
            } else if constexpr (OP == OP_SPMV_JAC) {
                // y = D^-1 A x (the scaled product of the iteration)
                T y = vc[q];
                if (!CEPS && a.sigma && live) D += (T)a.sigma[g];
                if (!dir) y = vc[q] - sum * (CEPS ? a.cidiag : rcp_pos(D));
                *pick(live && ok[q], a.out + g, a.sink + threadIdx.x + q * NT) = y;
            } else if constexpr (OP == OP_RESID) {
                if (live && ok[q]) {
                    const double Dd = CEPS ? (double)D : (double)D + (a.sigma ? a.sigma[g] : a.sig_const);
                    const double Ax = Dd * (double)vc[q] - (double)sum;
                    const double r = dir ? 0.0 : a.b[g] - Ax;
                    a.out[g] = (T)r;
                    if (a.rt32) a.rt32[g] = (float)r;
                    if (a.rs64 || a.rs32) {
                        const double rs = r * rcp_pos(Dd);
                        if (a.rs64) a.rs64[g] = rs;
                        if (a.rs32) a.rs32[g] = (float)rs;
                    }
                    acc[0] += r * r;
                }
            } else if constexpr (OP == OP_BA) {
                // v = A p^ (Table 3 step 11, with the scaled p), stored as
                // v^ = D^-1 v; shadow . v (step 12) and ||r||^2 of the
                // previous iteration's r = D r^
                const T iD = CEPS ? a.cidiag : rcp_pos(D);
                const T v = dir ? T(0) : D * vc[q] - sum;
                const bool keep = live && ok[q];
                *pick(keep, a.out + g, a.sink + threadIdx.x + q * NT) = v * iD;
                const double r = dir ? 0.0 : (double)D * (double)rc_[q];
                acc[0] += keep ? (double)tc[q] * (double)v : 0.0;
                acc[1] += keep ? r * r : 0.0;
            } else {
                // t = A s^ (step 14), stored as t^ = D^-1 t; t.s, t.t
                // (step 15), s.s (half-step test), shadow . s and shadow . t
                // (rho of the next iteration), with s = D s^
                const T iD = CEPS ? a.cidiag : rcp_pos(D);
                const T t = dir ? T(0) : D * vc[q] - sum;
                const double s = dir ? 0.0 : (double)D * (double)vc[q];
                const bool keep = live && ok[q];
                *pick(keep, a.out + g, a.sink + threadIdx.x + q * NT) = t * iD;
                const double m = keep ? 1.0 : 0.0;
                acc[0] += m * ((double)t * s);
                acc[1] += m * ((double)t * (double)t);
                acc[2] += m * (s * s);
                acc[3] += m * ((double)tc[q] * s);
                acc[4] += m * ((double)tc[q] * (double)t);
            }
        }
        // (4) stage plane k+1 in the other LDS buffer (unused after the last
        //     plane of the tile)
        T *nv = cur ? lval0 : lval1;
        T *ne = cur ? leps0 : leps1;
#pragma unroll
        for (int q = 0; q < PPT; ++q) {
            if (ok[q]) {
                nv[ox[q]] = vn[q];
                if constexpr (!CEPS) ne[ox[q]] = en[q];
            }
        }
#pragma unroll
        for (int u = 0; u < HMAX; ++u) {
            if (hok[u]) {
                nv[hm[u] - lo] = hv[u];
                if constexpr (!CEPS) ne[hm[u] - lo] = he[u];
            }
        }
        // (plane k+1 exists only when the tile stages it: k + 1 < k1 <= nz)
        if (WIDE && stage_next && nhalo > HMAX * NT) {
            for (int hI = threadIdx.x + HMAX * NT; hI < nhalo; hI += NT) {
                const int m = (hI < nhl) ? lo + hI : mend + (hI - nhl);
                Raw<T> w;
                load_raw<OP, T, CEPS, false, PAL, false>(a, (unsigned)m + Pu * (unsigned)(k + 1), w);
                nv[m - lo] = stage_raw<OP, T>(w, alpha, omega, beta);
                if constexpr (!CEPS) ne[m - lo] = coef<PAL>(w);
            }
        }
        // one barrier per plane: the buffer written next step was last read
        // before this barrier
        __syncthreads();
        cur ^= 1;
        // (5) rotate
#pragma unroll
        for (int q = 0; q < PPT; ++q) {
            vp[q] = vc[q]; vc[q] = vn[q];
            ep[q] = ec[q]; ec[q] = en[q];
            tc[q] = tn[q]; rc_[q] = rn_[q]; sc_[q] = sn_[q]; fc[q] = fn[q];
        }
    };
    if constexpr (DEPTH == 2) {
        for (int k = k0; k < k1; k += 2) {
            step(k, rA, hA);
            step(k + 1, rB, hB);
        }
    } else {
        for (int k = k0; k < k1; ++k) step(k, rA, hA);
    }

    if constexpr (OP == OP_RESID || OP == OP_BA || OP == OP_BB) {
        block_reduce<NQ, NT>(acc);
        store_partials<NQ>(acc, a.partials, slot);
    }
}

template <int OP, typename T, bool CEPS, int SIG, bool PAL, int NT, int PPT, bool WIDE, int DEPTH>
__global__ __launch_bounds__(NT) void k_zmarch(ZArgs<T> a)
{
    zmarch_tile<OP, T, CEPS, SIG, PAL, NT, PPT, WIDE, DEPTH>(a, xcd_remap(blockIdx.x, a.G), blockIdx.x);
}

// System owning global block b: start[s] <= b < start[s+1].
__device__ __forceinline__ int batch_system(const int *start, int nsys, int b)
{
    int lo = 0, hi = nsys;   // invariant: start[lo] <= b < start[hi]
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (start[mid] <= b) lo = mid; else hi = mid;
    }
    return lo;
}

// Batched form: one launch covers the tiles of nsys systems (grids of any
// size); each system keeps its own scalars, partials and status.
// Batched launches hold tiles of very different cost (members of other
// sizes take other z-chunk lengths), so contiguous per-XCD ranges would load
// the XCDs unevenly.  Instead runs of C consecutive tiles go to one XCD and
// the runs are dealt to the XCDs in turn: neighbouring strips of a run share
// that XCD's L2 for their halo rows, and every XCD gets a slice of every
// part of the batch.  Indices past the last whole round of runs keep their
// order.  (A permutation of [0, G).)
template <int C>
__device__ __forceinline__ int xcd_runs(int b, int G)
{
    const int X = 8;
    const int full = (G / (X * C)) * (X * C);
    if (b >= full) return b;
    const int x = b % X, i = b / X;
    return ((i / C) * X + x) * C + i % C;
}

// Active members of a batched Krylov run: before each iteration one
// workgroup lists the members still iterating (stop == RUN) and the prefix
// sums of their tile counts for steps A and B, so that the step kernels
// walk only those members' tiles.  act[0..na) = member indices, pa/pb
// [0..na] = tile prefixes (pa[na] = step A's tile total), *na_out = na.
constexpr int ACT_NT = 256;

__global__ __launch_bounds__(ACT_NT) void k_batch_active(const Scalars *const *sc, const int *startA,
                                                         const int *startB, int n, int *act, int *pa, int *pb,
                                                         int *na_out)
{
    __shared__ int sa[ACT_NT], sb[ACT_NT], sf[ACT_NT];
    __shared__ int base[3];   // running member count and tile totals
    if (threadIdx.x == 0) base[0] = base[1] = base[2] = 0;
    __syncthreads();
    for (int c0 = 0; c0 < n; c0 += ACT_NT) {
        const int i = c0 + threadIdx.x;
        const bool on = i < n && sc[i]->stop == ST_RUN;
        sf[threadIdx.x] = on ? 1 : 0;
        sa[threadIdx.x] = on ? startA[i + 1] - startA[i] : 0;
        sb[threadIdx.x] = on ? startB[i + 1] - startB[i] : 0;
        __syncthreads();
        // inclusive scans of the three counts (Hillis-Steele)
        for (int off = 1; off < ACT_NT; off <<= 1) {
            const int f = threadIdx.x >= off ? sf[threadIdx.x - off] : 0;
            const int a = threadIdx.x >= off ? sa[threadIdx.x - off] : 0;
            const int b = threadIdx.x >= off ? sb[threadIdx.x - off] : 0;
            __syncthreads();
            sf[threadIdx.x] += f;
            sa[threadIdx.x] += a;
            sb[threadIdx.x] += b;
            __syncthreads();
        }
        if (on) {
            const int k = base[0] + sf[threadIdx.x] - 1;   // this member's slot
            act[k] = i;
            pa[k + 1] = base[1] + sa[threadIdx.x];
            pb[k + 1] = base[2] + sb[threadIdx.x];
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            base[0] += sf[ACT_NT - 1];
            base[1] += sa[ACT_NT - 1];
            base[2] += sb[ACT_NT - 1];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        pa[0] = 0;
        pb[0] = 0;
        *na_out = base[0];
    }
}

// Batched form: one launch over the tiles of the members still iterating,
// listed by k_batch_active and numbered densely from 0 (the tiles of members
// that stopped are not in the list).  The grid is sized for every member's
// tiles when the launch is captured; workgroups past the active total leave
// after reading it.  Tiles go to the XCDs in runs (xcd_runs), and the
// hardware hands each workgroup slot the next tile as one finishes.  Each
// member keeps its own scalars, partials and status.
template <int OP, typename T, bool CEPS, int SIG, bool PAL, int NT, int PPT, bool WIDE, int DEPTH>
__global__ __launch_bounds__(NT) void k_zmarch_batch(const ZArgs<T> *__restrict__ args,
                                                     const int *__restrict__ act,
                                                     const int *__restrict__ pref,
                                                     const int *__restrict__ na_ptr)
{
    const int na = *na_ptr;
    const int total = pref[na];
    const int v = blockIdx.x;
    if (v >= total) return;
    const int t = xcd_runs<16>(v, total);
    const int k = batch_system(pref, na, t);
    const int lb = t - pref[k];
    const ZArgs<T> a = args[act[k]];   // private copy: stores cannot alias it
    zmarch_tile<OP, T, CEPS, SIG, PAL, NT, PPT, WIDE, DEPTH>(a, lb, lb);
}

// Palette of a coefficient field: *miss receives the smallest index n whose
// |eps[n]| is not among the npal palette values (unchanged when every node's
// value is there).  Run repeatedly, adding the missed value each time.
__global__ void k_palette_scan(size_t N, const double *eps, const double *pal, int npal,
                               unsigned long long *miss)
{
    unsigned long long first = ~0ull;
    for (size_t n = (size_t)blockIdx.x * blockDim.x + threadIdx.x; n < N;
         n += (size_t)gridDim.x * blockDim.x) {
        const double v = fabs(eps[n]);
        bool hit = false;
        for (int i = 0; i < npal && !hit; ++i) hit = (v == pal[i]);
        if (!hit) { first = n; break; }
    }
    if (first != ~0ull) atomicMin(miss, first);
}

// Palette indices: byte = index of |eps| in the palette, bit 7 = Dirichlet
// row (eps < 0).
__global__ void k_palette_index(size_t N, const double *eps, const double *pal, int npal, uint8_t *idx)
{
    for (size_t n = (size_t)blockIdx.x * blockDim.x + threadIdx.x; n < N;
         n += (size_t)gridDim.x * blockDim.x) {
        const double e = eps[n], v = fabs(e);
        int k = 0;
        while (k < npal - 1 && pal[k] != v) ++k;
        idx[n] = (uint8_t)(k | (e < 0.0 ? 128 : 0));
    }
}

// Shift per palette class: the smallest and largest bit pattern of sigma on
// the free rows of each class (sigma >= 0 there, so the patterns order as the
// values; a negative zero or a NaN reads as a second value).  mm holds
// PAL_MAX minima, then PAL_MAX maxima, preset to ~0 and 0.  Each wave takes
// the classes of its lanes one at a time.
__global__ __launch_bounds__(256) void k_shift_classes(size_t N, const double *sigma, const uint8_t *epsi,
                                                       unsigned long long *mm)
{
    __shared__ unsigned long long smin[PAL_MAX], smax[PAL_MAX];
    if (threadIdx.x < PAL_MAX) {
        smin[threadIdx.x] = ~0ull;
        smax[threadIdx.x] = 0ull;
    }
    __syncthreads();
    const int lane = threadIdx.x & 63;
    for (size_t base = (size_t)blockIdx.x * blockDim.x; base < N; base += (size_t)gridDim.x * blockDim.x) {
        const size_t n = base + threadIdx.x;
        int c = PAL_MAX;   // none
        unsigned long long u = 0;
        if (n < N) {
            const uint8_t e = epsi[n];
            if (!(e & 128)) {
                c = e & (PAL_MAX - 1);
                u = (unsigned long long)__double_as_longlong(sigma[n]);
            }
        }
        for (;;) {
            const unsigned long long pending = __ballot(c < PAL_MAX);
            if (pending == 0ull) break;
            const int lead = __ffsll((long long)pending) - 1;
            const int cl = __shfl(c, lead);
            unsigned long long lo = (c == cl) ? u : ~0ull, hi = (c == cl) ? u : 0ull;
            for (int o = 32; o > 0; o >>= 1) {
                lo = min(lo, (unsigned long long)__shfl_xor(lo, o));
                hi = max(hi, (unsigned long long)__shfl_xor(hi, o));
            }
            if (lane == lead) {
                atomicMin(&smin[cl], lo);
                atomicMax(&smax[cl], hi);
            }
            if (c == cl) c = PAL_MAX;
        }
    }
    __syncthreads();
    if (threadIdx.x < PAL_MAX && smin[threadIdx.x] != ~0ull) {
        atomicMin(&mm[threadIdx.x], smin[threadIdx.x]);
        atomicMax(&mm[PAL_MAX + threadIdx.x], smax[threadIdx.x]);
    }
}

// The class table (FP64 and its FP32 rounding; 0 for classes without free
// rows) and the verdict: 1 when every class holds a single value.
__global__ void k_shift_table(const unsigned long long *mm, double *t64, float *t32, int *one_per_class)
{
    if (threadIdx.x != 0) return;
    int ok = 1;
    for (int c = 0; c < PAL_MAX; ++c) {
        const unsigned long long lo = mm[c], hi = mm[PAL_MAX + c];
        double v = 0.0;
        if (lo != ~0ull) {
            ok &= lo == hi;
            v = __longlong_as_double((long long)lo);
        }
        t64[c] = v;
        t32[c] = (float)v;
    }
    *one_per_class = ok;
}

// ------------------------------------------------------------ finalize

enum { FIN_SUM = 3, FIN_MAX = 4 };

struct FinArgs {
    Scalars *sc;
    const double *partials;
    int G;
    int slot;   // result goes to red[slot]
};

// FIN_SUM / FIN_MAX finish the standalone residual and relaxation reductions
// into red[slot] (the BiCGSTAB steps finish each other's sums themselves).
template <int KIND>
__device__ __forceinline__ void finalize_block(const FinArgs &f)
{
    double tot[1];
    final_reduce<1, 256, KIND == FIN_MAX>(tot, f.partials, f.G);
    if (threadIdx.x == 0) f.sc->red[f.slot] = tot[0];
}

template <int KIND>
__global__ __launch_bounds__(256) void k_finalize(FinArgs f)
{
    finalize_block<KIND>(f);
}

// One finalize per member of a batch (member = blockIdx.x).
template <int KIND>
__global__ __launch_bounds__(256) void k_finalize_batch(const FinArgs *f)
{
    finalize_block<KIND>(f[blockIdx.x]);
}

// Copy the scalar blocks of n systems into one array (one host read per chunk).
__global__ void k_gather_scalars(const Scalars *const *src, Scalars *dst, int n)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) dst[i] = *src[i];
}

// ------------------------------------------------------- small kernels

struct Faces { double v[6]; };

// Classify nodes: flag bits and Dirichlet values of the potential system.
// bcphi/bcpsi: bit f set = face f is Neumann.
__global__ void k_classify(int nx, int ny, int nz, const uint8_t *type, const double *fixed_value,
                           int bcphi, Faces bcval, int bcpsi, uint8_t *flags, double *dval)
{
    const size_t N = (size_t)nx * ny * nz;
    for (size_t n = (size_t)blockIdx.x * blockDim.x + threadIdx.x; n < N;
         n += (size_t)gridDim.x * blockDim.x) {
        const int i = (int)(n % nx), j = (int)((n / nx) % ny), k = (int)(n / ((size_t)nx * ny));
        const int on[6] = {i == 0, i == nx - 1, j == 0, j == ny - 1, k == 0, k == nz - 1};
        bool dphi = false, dpsi = false;
        double v = 0.0;
        for (int f = 0; f < 6; ++f) {
            if (on[f] && !((bcphi >> f) & 1)) { dphi = true; v = bcval.v[f]; }
            if (on[f] && !((bcpsi >> f) & 1)) dpsi = true;
        }
        const uint8_t t = type ? type[n] : 0;
        if (t == 2) { dphi = true; v = fixed_value ? fixed_value[n] : 0.0; }
        if (t != 0) dpsi = true;
        flags[n] = (dphi ? F_DIR_PHI : 0) | (dpsi ? F_DIR_PSI : 0) | (t == 0 ? F_SOLVENT : 0) |
                   (t == 1 ? F_SOLUTE : 0);
        dval[n] = dphi ? v : 0.0;
    }
}

// Count invalid inputs: eps not finite or <= 0, type > 2, fixed data not finite.
__global__ void k_validate(size_t N, const double *eps, const uint8_t *type, const double *q,
                           const double *fv, unsigned *bad)
{
    unsigned b = 0;
    for (size_t n = (size_t)blockIdx.x * blockDim.x + threadIdx.x; n < N;
         n += (size_t)gridDim.x * blockDim.x) {
        const double e = eps[n];
        if (!(e > 0.0) || !finite(e)) b |= 1u;
        if (type && type[n] > 2) b |= 2u;
        if (q && !finite(q[n])) b |= 4u;
        if (fv && !finite(fv[n])) b |= 8u;
    }
    if (b) atomicOr(bad, b);
}

template <typename T>
__global__ void k_convert(size_t N, const double *src, T *dst)
{
    for (size_t n = (size_t)blockIdx.x * blockDim.x + threadIdx.x; n < N;
         n += (size_t)gridDim.x * blockDim.x)
        dst[n] = (T)src[n];
}

template <typename T>
__global__ void k_fill(size_t N, T *dst, T v)
{
    for (size_t n = (size_t)blockIdx.x * blockDim.x + threadIdx.x; n < N;
         n += (size_t)gridDim.x * blockDim.x)
        dst[n] = v;
}

// A fixed non-constant pattern in [0.5, 1.5) (synthetic operands of the
// launch-shape tuner: constant vectors make the stencil products vanish).
template <typename T>
__global__ void k_fill_pattern(size_t N, T *dst, double off)
{
    for (size_t n = (size_t)blockIdx.x * blockDim.x + threadIdx.x; n < N;
         n += (size_t)gridDim.x * blockDim.x) {
        const double u = ((double)n + off) * 0.6180339887498949;
        dst[n] = (T)(0.5 + (u - floor(u)));
    }
}

// Two copies of N doubles in one launch: d0 = s0, d1 = s1.
__global__ void k_copy2(size_t N, double *d0, const double *s0, double *d1, const double *s1)
{
    for (size_t n = (size_t)blockIdx.x * blockDim.x + threadIdx.x; n < N;
         n += (size_t)gridDim.x * blockDim.x) {
        d0[n] = s0[n];
        d1[n] = s1[n];
    }
}

// Start (or restart) of a BiCGSTAB run in one launch: p^ = v^ = t^ = 0, x = 0
// when xz is given (the correction of a refinement step), and the scalar
// block set to `init` (threads of the first workgroup copy it word by word).
// The residual kernel has already written s^ = D^-1 r and the shadow r.  The
// next step kernels read all of it after this launch.
template <typename T>
__global__ void k_krylov_start(size_t N, T *p, T *v, T *t, T *xz, Scalars init, Scalars *sc)
{
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    for (size_t n = (size_t)blockIdx.x * blockDim.x + threadIdx.x; n < N; n += stride) {
        p[n] = T(0);
        v[n] = T(0);
        t[n] = T(0);
        if (xz) xz[n] = T(0);
    }
    static_assert(sizeof(Scalars) % 4 == 0, "scalar block is copied in 32-bit words");
    constexpr unsigned W = sizeof(Scalars) / 4;
    static_assert(W <= 256, "one word per thread of the first workgroup");
    if (blockIdx.x == 0 && threadIdx.x < W)
        reinterpret_cast<unsigned *>(sc)[threadIdx.x] = reinterpret_cast<const unsigned *>(&init)[threadIdx.x];
}

// Mark the Dirichlet rows of the potential system in the coefficient field:
// e := -e where the flags carry F_DIR_PHI (the stencil kernels take |e| for
// the face coefficients and read the row kind from the sign).
__global__ void k_mark_dirichlet(size_t N, const uint8_t *flags, double *eps)
{
    for (size_t n = (size_t)blockIdx.x * blockDim.x + threadIdx.x; n < N;
         n += (size_t)gridDim.x * blockDim.x)
        if (flags[n] & F_DIR_PHI) eps[n] = -eps[n];
}

// Flag a negative diagonal shift on a free row (sigma must be >= 0; a NaN is
// left to the solver's non-finite checks).  *neg must be zero on entry.
__global__ void k_check_shift(size_t N, const double *sigma, const uint8_t *flags, uint8_t dirbit, int *neg)
{
    int b = 0;
    for (size_t n = (size_t)blockIdx.x * blockDim.x + threadIdx.x; n < N;
         n += (size_t)gridDim.x * blockDim.x)
        if (!(flags[n] & dirbit) && sigma[n] < 0.0) b = 1;
    if (b) atomicOr(neg, 1);
}

// x_i := Dirichlet value on Dirichlet rows (potential system) or 0 (PF1).
__global__ void k_set_dirichlet(size_t N, double *x, const uint8_t *flags, uint8_t dirbit,
                                const double *dval)
{
    for (size_t n = (size_t)blockIdx.x * blockDim.x + threadIdx.x; n < N;
         n += (size_t)gridDim.x * blockDim.x)
        if (flags[n] & dirbit) x[n] = dval ? dval[n] : 0.0;
}

// x64 += d32 on free rows (iterative-refinement correction).
__global__ void k_correct(size_t N, double *x, const float *d, const uint8_t *flags, uint8_t dirbit)
{
    for (size_t n = (size_t)blockIdx.x * blockDim.x + threadIdx.x; n < N;
         n += (size_t)gridDim.x * blockDim.x)
        if (!(flags[n] & dirbit)) x[n] += (double)d[n];
}

// ---------------------------------------------- batched solve bookkeeping
// One launch for every member of a batch between its Krylov runs (member =
// blockIdx.y); each does what the single-system kernels above do.

// After an FP32 run: keep x (copy into s), then x += d on free rows unless
// the run ended non-finite (apply = 0).
struct CorrectMember {
    size_t N;
    double *x, *s;
    const float *d;
    const uint8_t *flags;
    int dirbit, apply;
};

__global__ void k_correct_batch(const CorrectMember *m)
{
    const CorrectMember c = m[blockIdx.y];
    for (size_t n = (size_t)blockIdx.x * blockDim.x + threadIdx.x; n < c.N; n += (size_t)gridDim.x * blockDim.x) {
        const double x = c.x[n];
        c.s[n] = x;
        if (c.apply && !(c.flags[n] & c.dirbit)) c.x[n] = x + (double)c.d[n];
    }
}

// Start of a Krylov run (k_krylov_start) for every member.
template <typename T>
struct StartMember {
    size_t N;
    T *p, *v, *t, *xz;
    Scalars *sc;
    Scalars init;
};

template <typename T>
__global__ void k_krylov_start_batch(const StartMember<T> *m)
{
    const StartMember<T> &c = m[blockIdx.y];
    const size_t N = c.N;
    T *p = c.p, *v = c.v, *t = c.t, *xz = c.xz;
    for (size_t n = (size_t)blockIdx.x * blockDim.x + threadIdx.x; n < N; n += (size_t)gridDim.x * blockDim.x) {
        p[n] = T(0);
        v[n] = T(0);
        t[n] = T(0);
        if (xz) xz[n] = T(0);
    }
    constexpr unsigned W = sizeof(Scalars) / 4;
    if (blockIdx.x == 0 && threadIdx.x < W)
        reinterpret_cast<unsigned *>(c.sc)[threadIdx.x] = reinterpret_cast<const unsigned *>(&c.init)[threadIdx.x];
}

}  // namespace pfk

namespace pfk {

// ------------------------------------------------------------ Fermi, Eq. (1)

constexpr int MAXSP = 16;
struct SpeciesDev {
    int nsp, steric;
    double lam;              // e^2/(eps0 kB T) in grid units
    double lnGB;             // ln(bulk void fraction), 0 when steric is off
    double z[MAXSP];         // valences
    double lncb[MAXSP];      // ln C_i^B
    double lnvcb[MAXSP];     // ln(v_i C_i^B)
    double p[MAXSP];         // v_i / v_0
};

// Steric potential S at potential phi: root of
//   L(S) = ln( Gamma_B e^S + sum_i v_i C_i^B e^{-z_i phi + p_i S} ) = 0,
// the void-fraction identity Gamma = Gamma_B e^S = 1 - sum_i v_i C_i.
// L is convex and increasing in S; Newton's method started at the upper
// bracket S = -ln Gamma_B (where L >= 0) descends monotonically to the root.
// Everything stays in the log domain: |z_i phi| reaches 10^3 at charged nodes.
__device__ __forceinline__ double steric_root(double phi, const SpeciesDev &sp)
{
    double S = -sp.lnGB;
    for (int it = 0; it < 200; ++it) {
        double m = sp.lnGB + S;
        for (int i = 0; i < sp.nsp; ++i) m = fmax(m, sp.lnvcb[i] - sp.z[i] * phi + sp.p[i] * S);
        double w0 = exp(sp.lnGB + S - m);
        double sum = w0, dsum = w0;
        for (int i = 0; i < sp.nsp; ++i) {
            const double w = exp(sp.lnvcb[i] - sp.z[i] * phi + sp.p[i] * S - m);
            sum += w;
            dsum += sp.p[i] * w;
        }
        const double L = m + log(sum);
        const double step = L * sum / dsum;
        const double Sn = S - step;
        if (!(fabs(Sn - S) > 4.0 * 2.220446049250313e-16 * fmax(1.0, fabs(S)))) return Sn;
        S = Sn;
    }
    return S;
}

// Fermi update at one solvent node of potential ph: rho_hat into rh,
// lambda sum z_i^2 C_i (= -rho_hat' of Eq. (11)) into sg, the steric
// potential into S, and C_i into conc[i*N + n] when conc is given.
__device__ __forceinline__ void fermi_at(double ph, const SpeciesDev &sp, double &rh, double &sg, double &S,
                                         double *conc, size_t n, size_t N)
{
    rh = 0.0;
    sg = 0.0;
    S = sp.steric ? steric_root(ph, sp) : 0.0;
    for (int i = 0; i < sp.nsp; ++i) {
        const double C = exp(sp.lncb[i] - sp.z[i] * ph + sp.p[i] * S);
        rh += sp.z[i] * C;
        sg += sp.z[i] * sp.z[i] * C;
        if (conc) conc[(size_t)i * N + n] = C;
    }
    rh *= sp.lam;
    sg *= sp.lam;
}

// Fermi update at every node; zeros off the solvent.  Writes any of:
// rhs1 = -rho_hat (the PF1 right-hand side), rho = rho_hat,
// sigma = lambda sum z_i^2 C_i (= -rho_hat' of Eq. (11)), conc[i*N + n], S.
__global__ void k_fermi(size_t N, const double *phi, const uint8_t *flags, SpeciesDev sp,
                        double *rhs1, double *rho, double *sigma, double *conc, double *Sout)
{
    for (size_t n = (size_t)blockIdx.x * blockDim.x + threadIdx.x; n < N;
         n += (size_t)gridDim.x * blockDim.x) {
        double rh = 0.0, sg = 0.0, S = 0.0;
        const bool solvent = flags[n] & F_SOLVENT;
        if (solvent) {
            fermi_at(phi[n], sp, rh, sg, S, conc, n, N);
        } else if (conc) {
            for (int i = 0; i < sp.nsp; ++i) conc[(size_t)i * N + n] = 0.0;
        }
        if (rhs1) rhs1[n] = -rh;
        if (rho) rho[n] = rh;
        if (sigma) sigma[n] = sg;
        if (Sout) Sout[n] = S;
    }
}

// Fixed-charge source lambda q / h^3, plus an extra right-hand side (the
// interface terms of the singular-charge decomposition) when given.
__global__ void k_source(size_t N, const double *q, double scale, const double *extra, double *src)
{
    for (size_t n = (size_t)blockIdx.x * blockDim.x + threadIdx.x; n < N;
         n += (size_t)gridDim.x * blockDim.x) {
        double v = q ? scale * q[n] : 0.0;
        if (extra) v += extra[n];
        src[n] = v;
    }
}

// PF1 with l_c = 0: Psi = -rho_hat / eps_s on free Psi rows, 0 elsewhere.
__global__ void k_psi_local(size_t N, const double *rhs1, const uint8_t *flags, double inv_eps_s,
                            double *psi)
{
    for (size_t n = (size_t)blockIdx.x * blockDim.x + threadIdx.x; n < N;
         n += (size_t)gridDim.x * blockDim.x)
        psi[n] = (flags[n] & F_DIR_PSI) ? 0.0 : rhs1[n] * inv_eps_s;
}

// PF2 right-hand side (Eq. (13) scaled): -eps_s Psi + sigma Phi_0 + lambda q / h^3.
__global__ void k_rhs_pf2(size_t N, const double *psi, const double *sigma, const double *phi0,
                          const double *src, double eps_s, double *b)
{
    for (size_t n = (size_t)blockIdx.x * blockDim.x + threadIdx.x; n < N;
         n += (size_t)gridDim.x * blockDim.x)
        b[n] = -eps_s * psi[n] + sigma[n] * phi0[n] + src[n];
}

// Relaxation (Table 2 step 5): Phi := omega Phi_0 + (1 - omega) Phi; the max
// norm of the change; Phi_0 := Phi.  Result in sc->red[0].
// Max norm of r over the free rows (flags without dirbit); NaN shows as +inf.
template <int NT>
__global__ __launch_bounds__(NT) void k_maxabs_free(size_t N, const double *r, const uint8_t *flags, uint8_t dirbit,
                                                    double *partials)
{
    double acc[1] = {0.0};
    const size_t stride = (size_t)gridDim.x * NT;
    for (size_t n = (size_t)blockIdx.x * NT + threadIdx.x; n < N; n += stride) {
        if (flags[n] & dirbit) continue;
        double d = fabs(r[n]);
        if (d != d) d = __builtin_inf();
        acc[0] = fmax(acc[0], d);
    }
    block_reduce<1, NT, true>(acc);
    store_partials<1>(acc, partials, blockIdx.x);
}

// Relaxation (Table 2 step 5) fused with the point-wise steps that open the
// next outer iteration: Phi_0 := omega Phi_0 + (1 - omega) Phi (also into
// Phi; max |change| into the partials), then at the new Phi_0 the Fermi
// update (Eq. (1)): sig = -rho_hat', and
//   rhs2 == null (a PF1 solve follows): rhs1 = -rho_hat;
//   rhs2 != null (local PF1, lc = 0): Psi = -rho_hat / eps_s (0 on PF1
//   Dirichlet rows) and the PF2 right-hand side of Eq. (13),
//   rhs2 = -eps_s Psi + sig Phi_0 + src, neither Psi nor rhs1 stored.
// Each value is the one the separate kernels compute, in the same order.
template <int NT>
__global__ __launch_bounds__(NT) void k_relax_fermi(size_t N, double *phi0, double *phi, double omega,
                                                    double *partials, const uint8_t *flags, SpeciesDev sp,
                                                    double *rhs1, double *sig, const double *src, double eps_s,
                                                    double inv_eps_s, double *rhs2)
{
    double acc[1] = {0.0};
    const size_t stride = (size_t)gridDim.x * NT;
    for (size_t n = (size_t)blockIdx.x * NT + threadIdx.x; n < N; n += stride) {
        const double old = phi0[n];
        const double nv = omega * old + (1.0 - omega) * phi[n];
        double d = fabs(nv - old);
        if (d != d) d = __builtin_inf();   // keep a NaN visible through fmax
        acc[0] = fmax(acc[0], d);
        phi0[n] = nv;
        phi[n] = nv;
        const uint8_t f = flags[n];
        double rh = 0.0, sg = 0.0, S = 0.0;
        if (f & F_SOLVENT) fermi_at(nv, sp, rh, sg, S, nullptr, n, N);
        sig[n] = sg;
        if (rhs2) {
            const double ps = (f & F_DIR_PSI) ? 0.0 : -rh * inv_eps_s;
            rhs2[n] = -eps_s * ps + sg * nv + src[n];
        } else {
            rhs1[n] = -rh;
        }
    }
    block_reduce<1, NT, true>(acc);
    store_partials<1>(acc, partials, blockIdx.x);
}

}  // namespace pfk
