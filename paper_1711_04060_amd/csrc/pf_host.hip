// pf_host.hip -- host side of the C-ABI in include/pf.h.
//
// Grid handles own device copies of the fields and the solver workspace.
// Linear solves run the Jacobi-BiCGSTAB of Sec. 4, Table 3 with three fused
// kernels per iteration (pf_kernels.h); the scalar recurrences stay on the
// device and the host reads one small status block per chunk of iterations.
// Each chunk is a captured hipGraph, so a chunk costs one launch.  The
// nonlinear loop of Tables 2 and 4 runs entirely on the device apart from one
// status read per outer iteration (the max-norm test of Table 2 step 5).
#include "pf_kernels.h"
#include <hip/hip_ext.h>
#include "pf_iface.h"
#include "pf_sites.h"
#include "pf_stream.h"
#include "../../include/pf.h"

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <functional>
#include <map>
#include <mutex>
#include <string>
#include <tuple>
#include <type_traits>
#include <vector>

using pfk::Scalars;

namespace {

thread_local std::string g_err;

pf_status fail(pf_status st, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return st;
}

#define HIPCHK(call)                                                                     \
    do {                                                                                 \
        hipError_t e_ = (call);                                                          \
        if (e_ != hipSuccess)                                                            \
            return fail(PF_ERR_DEVICE, "%s failed: %s", #call, hipGetErrorString(e_));   \
    } while (0)

#define PFCHK(call)                      \
    do {                                 \
        pf_status s_ = (call);           \
        if (s_ != PF_OK) return s_;      \
    } while (0)

constexpr int NT = 256;          // threads per workgroup of every kernel
constexpr int PW_MAX_G = 1024;   // workgroups of the pointwise kernels

// launch override (pf_set_launch): threads, points per thread, z-planes
int g_nt_override = 0, g_ppt_override = 0, g_kz_override = 0, g_depth_override = 0;

// kernel timing (pf_timing_enable / pf_timing_read): slots 0, 1 = BiCGSTAB
// step A in FP64 / FP32; 2, 3 = Jacobi-scaled products of pf_spmv /
// pf_spmv_f32; 4, 5 = batched step A in FP64 / FP32
constexpr int TIMING_SLOTS = 6;
struct Timing {
    bool enabled = false;
    int sample = 8;
    long chunk = 0;
    long long launches[TIMING_SLOTS] = {};
    double ms[TIMING_SLOTS] = {}, bytes[TIMING_SLOTS] = {};
    hipEvent_t p0 = nullptr, p1 = nullptr;   // around product launches
} g_timing;

constexpr size_t LDS_MAX = 152 * 1024;   // dynamic LDS per workgroup (gfx950 has 160 KB; static arrays use the rest)

// Launch shape of the z-marching stencil kernels: NTZ threads per
// workgroup, PPT nodes per thread (strip S = NTZ*PPT), KZ planes per
// workgroup.
struct ZCfg {
    int NTZ = 256, PPT = 2, S = 512, KZ = 8, nstrips = 1, nzc = 1, G = 1, lmax = 0;
    bool wide = false;   // halo rows exceed the registers' halo slots (WIDE kernel form)
    int depth = 1;       // planes of loads in flight ahead of the plane computed
    size_t lds = 0;
};

// Halo slots per thread of the z-march kernels (both halo rows, 2 nx nodes,
// fit in registers when 2 nx <= halo_slots(NT) * NT).
constexpr int halo_slots(int ntz) { return ntz >= 512 ? 1 : 2; }

// Load pipeline depth when none is given: two planes where the two register
// sets still leave four waves per SIMD (FP32, one node per thread).
int default_depth(size_t elem, int ppt) { return (elem == 4 && ppt == 1) ? 2 : 1; }

ZCfg make_cfg(int nx, int ny, int nz, size_t elem, int ntz, int ppt, int kz, int depth = 0)
{
    ZCfg c;
    const int P = nx * ny;
    c.NTZ = ntz;
    c.PPT = ppt;
    c.S = ntz * ppt;
    c.nstrips = (P + c.S - 1) / c.S;
    c.KZ = std::max(1, std::min(kz, nz));
    c.nzc = (nz + c.KZ - 1) / c.KZ;
    c.G = c.nstrips * c.nzc;
    c.lmax = std::min(P, c.S + 2 * nx);
    // two planes of (value, coefficient), the face table, the class shifts
    c.lds = (4 * (size_t)c.lmax + pfk::FTAB + pfk::PAL_MAX) * elem;
    c.wide = 2 * nx > halo_slots(ntz) * ntz;
    c.depth = c.wide ? 1 : (depth ? depth : (g_depth_override ? g_depth_override : default_depth(elem, ppt)));
    return c;
}

// Shape used before (or without) tuning: long strips for wide planes,
// z-chunks sized for several workgroups per CU.
ZCfg default_cfg(int nx, int ny, int nz, size_t elem)
{
    const int P = nx * ny;
    int ntz = g_nt_override ? g_nt_override : (P >= 16384 ? 1024 : 512);
    int ppt = g_ppt_override ? g_ppt_override : (P >= 16384 ? 2 : 1);
    int kz = g_kz_override;
    if (!kz) {
        const long strips = (P + (long)ntz * ppt - 1) / ((long)ntz * ppt);
        kz = (int)std::max<long>(4, std::min<long>(16, strips * nz / 1024));
    }
    ZCfg c = make_cfg(nx, ny, nz, elem, ntz, ppt, kz);
    while (c.lds > LDS_MAX && c.PPT > 1) c = make_cfg(nx, ny, nz, elem, c.NTZ, c.PPT - 1, c.KZ);
    while (c.lds > LDS_MAX && c.NTZ > 256) c = make_cfg(nx, ny, nz, elem, c.NTZ / 2, c.PPT, c.KZ);
    // very wide planes: only the 1024-thread, one-node-per-thread shape has a WIDE form
    if (c.wide && (c.NTZ != 1024 || c.PPT != 1)) c = make_cfg(nx, ny, nz, elem, 1024, 1, c.KZ);
    return c;
}

int pw_blocks(size_t N) { return (int)std::min<size_t>(PW_MAX_G, (N + NT - 1) / NT); }

// Captured iteration chunks of a grid: chunk length, element size, kernel
// form and the shift array the SIG form reads (grid-owned).
struct GraphKey {
    int m, elem, form;
    const void *sig;
    bool operator<(const GraphKey &o) const
    {
        return std::tie(m, elem, form, sig) < std::tie(o.m, o.elem, o.form, o.sig);
    }
};

// Krylov vectors of one precision; the shadow residual is kept in FP32 in
// both (the shadow vector of Table 3 is r0 rounded to FP32).
template <typename T>
struct Work {
    T *x = nullptr, *r = nullptr, *p[2] = {nullptr, nullptr}, *v[2] = {nullptr, nullptr}, *s = nullptr,
      *t = nullptr;
    float *rt = nullptr;
};

}  // namespace

struct pf_grid {
    int device = 0;                    // device current at creation (owner of every buffer and the stream)
    int nx = 0, ny = 0, nz = 0;
    size_t N = 0;
    double h = 0;
    hipStream_t stream = nullptr;      // internal blocking stream
    hipStream_t ustream = nullptr;     // caller's stream (ordering only)
    hipEvent_t ev = nullptr;
    int bcphi_mask = 0, bcpsi_mask = 0;
    double bcval[6] = {0, 0, 0, 0, 0, 0};
    std::vector<void *> allocs;

    double *eps64 = nullptr;           // coefficient field; sign bit set on Dirichlet rows (F_DIR_PHI)
    float *eps32 = nullptr;
    int npal = 0;                      // palette form: number of distinct |eps| (0: no palette)
    uint8_t *epsi = nullptr;           // palette index per node, bit 7 = Dirichlet row
    double *ftab64 = nullptr;          // face coefficients of palette pairs (FTAB values, / h^2)
    float *ftab32 = nullptr;
    double *stab64 = nullptr;          // shift of each palette class (SIG_CLASS form, per solve)
    float *stab32 = nullptr;
    unsigned long long *smm = nullptr; // per-class extremes of the shift (2 PAL_MAX)
    uint8_t *flags = nullptr;
    double *dval = nullptr;
    double *q = nullptr;               // fixed charge (may stay null)

    ZCfg c64, c32;     // step A of BiCGSTAB, residual and plain products
    ZCfg cb64, cb32;   // step B of BiCGSTAB (tuned on its own: lighter kernel)
    ZCfg cp64, cp32;   // standalone Jacobi-scaled product (tuned on first use)
    bool tunedp64 = false, tunedp32 = false;
    int Gmax = 1;

    // linear solver state
    float *sig32 = nullptr;            // FP32 copy of the shift of the current PF_MIXED solve
    double *b64 = nullptr;
    Work<double> w64;
    Work<float> w32;
    bool have64 = false, have32 = false;
    Scalars *sc = nullptr, *hsc = nullptr;
    double *partials = nullptr;                                // standalone reductions
    double *partA = nullptr, *partB = nullptr;   // BiCGSTAB steps A, B
    double *sink = nullptr;            // target of the stencil kernels' masked stores
    std::map<GraphKey, hipGraphExec_t> graphs;
    double *sig64 = nullptr;           // copy of a caller's shift array for the solve (allocated on use)
    std::vector<hipEvent_t> tev;       // timing events (2 per iteration of a chunk)
    bool last_timed_first = false;   // the first chunk of the last batch ran timed
    int last_run[4] = {0, 0, 0, 0};    // iterations of the last Krylov run per (precision, system)

    // nonlinear state
    double *phi0 = nullptr, *phi = nullptr, *psi = nullptr, *rhs1 = nullptr, *sig = nullptr,
           *rhs2 = nullptr, *src = nullptr;
};

namespace {

template <typename T>
pf_status dalloc(pf_grid *g, T **p, size_t n)
{
    void *q = nullptr;
    if (hipMalloc(&q, std::max<size_t>(n, 1) * sizeof(T)) != hipSuccess) {
        (void)hipGetLastError();
        return fail(PF_ERR_ALLOC, "hipMalloc of %zu bytes failed", n * sizeof(T));
    }
    g->allocs.push_back(q);
    *p = static_cast<T *>(q);
    return PF_OK;
}

template <typename T>
pf_status fill(pf_grid *g, T *p, T v, size_t n)
{
    hipLaunchKernelGGL((pfk::k_fill<T>), dim3(pw_blocks(n)), dim3(NT), 0, g->stream, n, p, v);
    HIPCHK(hipGetLastError());
    return PF_OK;
}

pf_status begin(pf_grid *g)
{
    g_err.clear();
    if (g->ustream) {
        HIPCHK(hipEventRecord(g->ev, g->ustream));
        HIPCHK(hipStreamWaitEvent(g->stream, g->ev, 0));
    }
    return PF_OK;
}

pf_status sync(pf_grid *g)
{
    HIPCHK(hipStreamSynchronize(g->stream));
    return PF_OK;
}

template <typename T>
pf_status tune(pf_grid *g);

template <typename T>
pf_status ensure_work(pf_grid *g)
{
    if constexpr (sizeof(T) == 8) {
        if (g->have64) return PF_OK;
        Work<double> &w = g->w64;
        PFCHK(dalloc(g, &g->b64, g->N));
        for (double **p : {&w.x, &w.r, &w.p[0], &w.p[1], &w.v[0], &w.v[1], &w.s, &w.t})
            PFCHK(dalloc(g, p, g->N));
        PFCHK(dalloc(g, &w.rt, g->N));
        g->have64 = true;
        PFCHK(tune<double>(g));
    } else {
        if (g->have32) return PF_OK;
        PFCHK(ensure_work<double>(g));
        Work<float> &w = g->w32;
        PFCHK(dalloc(g, &g->eps32, g->N));
        PFCHK(dalloc(g, &g->sig32, g->N));
        for (float **p : {&w.x, &w.r, &w.rt, &w.p[0], &w.p[1], &w.v[0], &w.v[1], &w.s, &w.t})
            PFCHK(dalloc(g, p, g->N));
        hipLaunchKernelGGL((pfk::k_convert<float>), dim3(pw_blocks(g->N)), dim3(NT), 0, g->stream,
                           g->N, (const double *)g->eps64, g->eps32);
        HIPCHK(hipGetLastError());
        g->have32 = true;
        PFCHK(tune<float>(g));
    }
    return PF_OK;
}

// --------------------------------------------------------------- launches

// e0, e1 (optional): events that the dispatch itself stamps at the kernel's
// start and end (hipExtLaunchKernel), so their interval is the kernel's own
// duration, without the marker packets of separate event records.
template <int OP, typename T, bool CEPS, int SIG, bool PAL, int NTZ, int PPT, bool WIDE = false, int DEPTH = 1>
hipError_t launch_zk(const ZCfg &c, const pfk::ZArgs<T> &a, hipStream_t s, hipEvent_t e0 = nullptr,
                     hipEvent_t e1 = nullptr)
{
    auto kern = pfk::k_zmarch<OP, T, CEPS, SIG, PAL, NTZ, PPT, WIDE, DEPTH>;
    if (c.lds > 64 * 1024) {
        static size_t granted = 0;   // per instantiation
        if (c.lds > granted) {
            hipError_t e = hipFuncSetAttribute((const void *)kern, hipFuncAttributeMaxDynamicSharedMemorySize,
                                               (int)c.lds);
            if (e != hipSuccess) return e;
            granted = c.lds;
        }
    }
    if (e0 || e1) hipExtLaunchKernelGGL(kern, dim3(c.G), dim3(NTZ), (std::uint32_t)c.lds, s, e0, e1, 0u, a);
    else hipLaunchKernelGGL(kern, dim3(c.G), dim3(NTZ), c.lds, s, a);
    return hipGetLastError();
}

template <int OP, typename T, bool CEPS, int SIG, bool PAL>
hipError_t launch_z(const ZCfg &c, const pfk::ZArgs<T> &a, hipStream_t s, hipEvent_t e0 = nullptr,
                    hipEvent_t e1 = nullptr)
{
    if (c.wide) {
        if (c.NTZ == 1024 && c.PPT == 1) return launch_zk<OP, T, CEPS, SIG, PAL, 1024, 1, true>(c, a, s, e0, e1);
        return hipErrorInvalidValue;
    }
    // the BiCGSTAB steps and the Jacobi-scaled product come in both pipeline
    // depths; the residual and plain products (a few launches per solve) in one
    constexpr bool PIPE = (OP == pfk::OP_BA || OP == pfk::OP_BB || OP == pfk::OP_SPMV_JAC);
    if (PIPE && c.depth == 2) {
        switch (c.NTZ * 10 + c.PPT) {
        case 2561: return launch_zk<OP, T, CEPS, SIG, PAL, 256, 1, false, 2>(c, a, s, e0, e1);
        case 2562: return launch_zk<OP, T, CEPS, SIG, PAL, 256, 2, false, 2>(c, a, s, e0, e1);
        case 5121: return launch_zk<OP, T, CEPS, SIG, PAL, 512, 1, false, 2>(c, a, s, e0, e1);
        case 5122: return launch_zk<OP, T, CEPS, SIG, PAL, 512, 2, false, 2>(c, a, s, e0, e1);
        case 10241: return launch_zk<OP, T, CEPS, SIG, PAL, 1024, 1, false, 2>(c, a, s, e0, e1);
        case 10242: return launch_zk<OP, T, CEPS, SIG, PAL, 1024, 2, false, 2>(c, a, s, e0, e1);
        default: return hipErrorInvalidValue;
        }
    }
    switch (c.NTZ * 10 + c.PPT) {
    case 2561: return launch_zk<OP, T, CEPS, SIG, PAL, 256, 1>(c, a, s, e0, e1);
    case 2562: return launch_zk<OP, T, CEPS, SIG, PAL, 256, 2>(c, a, s, e0, e1);
    case 5121: return launch_zk<OP, T, CEPS, SIG, PAL, 512, 1>(c, a, s, e0, e1);
    case 5122: return launch_zk<OP, T, CEPS, SIG, PAL, 512, 2>(c, a, s, e0, e1);
    case 10241: return launch_zk<OP, T, CEPS, SIG, PAL, 1024, 1>(c, a, s, e0, e1);
    case 10242: return launch_zk<OP, T, CEPS, SIG, PAL, 1024, 2>(c, a, s, e0, e1);
    default: return hipErrorInvalidValue;
    }
}

// Batched step over the active members' tiles: the grid covers every
// member's tiles (c.G); the kernel maps the first workgroups to the active
// ones.
template <int OP, typename T, bool CEPS, int SIG, bool PAL, int NTZ, int PPT, bool WIDE, int DEPTH>
hipError_t launch_batch_k(const ZCfg &c, const pfk::ZArgs<T> *args, const int *act, const int *pref, const int *na,
                          hipStream_t s, hipEvent_t e0, hipEvent_t e1)
{
    auto kern = pfk::k_zmarch_batch<OP, T, CEPS, SIG, PAL, NTZ, PPT, WIDE, DEPTH>;
    static size_t granted = 0;
    if (c.lds > 64 * 1024 && c.lds > granted) {
        hipError_t e = hipFuncSetAttribute((const void *)kern, hipFuncAttributeMaxDynamicSharedMemorySize,
                                           (int)c.lds);
        if (e != hipSuccess) return e;
        granted = c.lds;
    }
    if (e0 || e1)
        hipExtLaunchKernelGGL(kern, dim3(c.G), dim3(NTZ), (std::uint32_t)c.lds, s, e0, e1, 0u, args, act, pref, na);
    else hipLaunchKernelGGL(kern, dim3(c.G), dim3(NTZ), c.lds, s, args, act, pref, na);
    return hipGetLastError();
}

// c: the batch's combined launch (its NTZ, PPT, depth shared by every member;
// G = all members' tiles, lds and wide = the maxima)
template <int OP, typename T, bool CEPS, int SIG, bool PAL>
hipError_t launch_batch(const ZCfg &c, const pfk::ZArgs<T> *args, const int *act, const int *pref, const int *na,
                        hipStream_t s, hipEvent_t e0 = nullptr, hipEvent_t e1 = nullptr)
{
    if (c.wide) {
        if (c.NTZ == 1024 && c.PPT == 1)
            return launch_batch_k<OP, T, CEPS, SIG, PAL, 1024, 1, true, 1>(c, args, act, pref, na, s, e0, e1);
        return hipErrorInvalidValue;
    }
    if (c.depth == 2) {
        switch (c.NTZ * 10 + c.PPT) {
        case 2561: return launch_batch_k<OP, T, CEPS, SIG, PAL, 256, 1, false, 2>(c, args, act, pref, na, s, e0, e1);
        case 2562: return launch_batch_k<OP, T, CEPS, SIG, PAL, 256, 2, false, 2>(c, args, act, pref, na, s, e0, e1);
        case 5121: return launch_batch_k<OP, T, CEPS, SIG, PAL, 512, 1, false, 2>(c, args, act, pref, na, s, e0, e1);
        case 5122: return launch_batch_k<OP, T, CEPS, SIG, PAL, 512, 2, false, 2>(c, args, act, pref, na, s, e0, e1);
        case 10241: return launch_batch_k<OP, T, CEPS, SIG, PAL, 1024, 1, false, 2>(c, args, act, pref, na, s, e0, e1);
        case 10242: return launch_batch_k<OP, T, CEPS, SIG, PAL, 1024, 2, false, 2>(c, args, act, pref, na, s, e0, e1);
        default: return hipErrorInvalidValue;
        }
    }
    switch (c.NTZ * 10 + c.PPT) {
    case 2561: return launch_batch_k<OP, T, CEPS, SIG, PAL, 256, 1, false, 1>(c, args, act, pref, na, s, e0, e1);
    case 2562: return launch_batch_k<OP, T, CEPS, SIG, PAL, 256, 2, false, 1>(c, args, act, pref, na, s, e0, e1);
    case 5121: return launch_batch_k<OP, T, CEPS, SIG, PAL, 512, 1, false, 1>(c, args, act, pref, na, s, e0, e1);
    case 5122: return launch_batch_k<OP, T, CEPS, SIG, PAL, 512, 2, false, 1>(c, args, act, pref, na, s, e0, e1);
    case 10241: return launch_batch_k<OP, T, CEPS, SIG, PAL, 1024, 1, false, 1>(c, args, act, pref, na, s, e0, e1);
    case 10242: return launch_batch_k<OP, T, CEPS, SIG, PAL, 1024, 2, false, 1>(c, args, act, pref, na, s, e0, e1);
    default: return hipErrorInvalidValue;
    }
}

// Kernel forms of an operator: PF1 (constant coefficient), the potential
// system with a shift array (sigma read at every own node) or without one,
// each with the coefficient field read in full or as palette indices, and
// the palette form whose shift is one value per palette class (a table).
// Only the BiCGSTAB steps have the shift forms (the other kernels read sigma
// at their outputs), and only they and the Jacobi-scaled product have the
// palette forms.
enum { FORM_PLAIN = 0, FORM_SIG = 1, FORM_CEPS = 2, FORM_PAL = 3, FORM_PALSIG = 4, FORM_PALTAB = 5 };

template <int OP, typename T>
hipError_t launch_batch_form(int form, const ZCfg &c, const pfk::ZArgs<T> *args, const int *act, const int *pref,
                             const int *na, hipStream_t s, hipEvent_t e0 = nullptr, hipEvent_t e1 = nullptr)
{
    switch (form) {
    case FORM_CEPS: return launch_batch<OP, T, true, pfk::SIG_NONE, false>(c, args, act, pref, na, s, e0, e1);
    case FORM_SIG: return launch_batch<OP, T, false, pfk::SIG_NODE, false>(c, args, act, pref, na, s, e0, e1);
    case FORM_PAL: return launch_batch<OP, T, false, pfk::SIG_NONE, true>(c, args, act, pref, na, s, e0, e1);
    case FORM_PALSIG: return launch_batch<OP, T, false, pfk::SIG_NODE, true>(c, args, act, pref, na, s, e0, e1);
    case FORM_PALTAB: return launch_batch<OP, T, false, pfk::SIG_CLASS, true>(c, args, act, pref, na, s, e0, e1);
    default: return launch_batch<OP, T, false, pfk::SIG_NONE, false>(c, args, act, pref, na, s, e0, e1);
    }
}

template <typename T>
const ZCfg &cfg_of(const pf_grid *g)
{
    if constexpr (sizeof(T) == 8) return g->c64;
    else return g->c32;
}

template <typename T>
ZCfg &cfg_ref(pf_grid *g)
{
    if constexpr (sizeof(T) == 8) return g->c64;
    else return g->c32;
}

template <typename T>
ZCfg &cfgb_ref(pf_grid *g)
{
    if constexpr (sizeof(T) == 8) return g->cb64;
    else return g->cb32;
}

template <typename T>
ZCfg &cfgp_ref(pf_grid *g)
{
    if constexpr (sizeof(T) == 8) return g->cp64;
    else return g->cp32;
}

// Operator description: which system (potential or PF1 density), constant
// coefficient or not, diagonal shift.
struct OpDesc {
    bool psi = false;          // PF1 system (flags bit F_DIR_PSI), constant coefficient
    double ceps = 0;           // PF1 face coefficient eps_s lc^2 (before / h^2)
    const double *sigma = nullptr;
    double sig_const = 0;
    bool sig_class = false;    // sigma is one value per palette class on the free rows (table in the grid)
};

uint8_t dirbit(const OpDesc &op) { return op.psi ? pfk::F_DIR_PSI : pfk::F_DIR_PHI; }

// The palette form is used where the grid has one (PF_PALETTE=0 turns it off,
// for comparisons).
// The shift-per-class table replaces a per-node shift where it holds
// (PF_SHIFT_CLASS=0 turns it off, read at each solve, for comparisons).
bool shift_class_enabled()
{
    const char *e = getenv("PF_SHIFT_CLASS");
    return !(e && e[0] == '0');
}

bool use_palette(const pf_grid *g)
{
    static const bool on = [] {
        const char *e = getenv("PF_PALETTE");
        return !(e && e[0] == '0');
    }();
    return on && g->npal > 0;
}

// Kernel form of the BiCGSTAB steps for this operator on grid g.
int step_form(const OpDesc &op, const pf_grid *g)
{
    if (op.psi) return FORM_CEPS;
    if (use_palette(g)) return op.sigma ? (op.sig_class ? FORM_PALTAB : FORM_PALSIG) : FORM_PAL;
    return op.sigma ? FORM_SIG : FORM_PLAIN;
}

// Bytes per node of the coefficient read: the full field, a palette index,
// or (PF1) a flag byte.
double coef_bytes(int form, size_t elem)
{
    return (form == FORM_CEPS || form == FORM_PAL || form == FORM_PALSIG || form == FORM_PALTAB) ? 1.0 : (double)elem;
}

// Algorithmic bytes of one step-A launch on N nodes: s^, p^, v^, t^ and the
// coefficient read at every staged node, x, the FP32 shadow (and a per-node
// sigma) at own nodes; x, r^, p^, v^ written.
double step_a_bytes(const OpDesc &op, const pf_grid *g, size_t elem)
{
    const int form = step_form(op, g);
    const bool sig = form == FORM_SIG || form == FORM_PALSIG;
    const double per = 4.0 * elem + coef_bytes(form, elem) + elem + 4.0 + (sig ? (double)elem : 0.0) + 4.0 * elem;
    return per * (double)g->N;
}

template <typename T>
pfk::ZArgs<T> zbase_cfg(pf_grid *g, const OpDesc &op, const ZCfg &c)
{
    pfk::ZArgs<T> a{};
    a.nx = g->nx; a.ny = g->ny; a.nz = g->nz; a.P = g->nx * g->ny;
    a.S = c.S; a.KZ = c.KZ; a.nstrips = c.nstrips; a.G = c.G; a.lmax = c.lmax;
    const double ih2 = 1.0 / (g->h * g->h);
    a.ih2 = (T)ih2;
    a.ceps = (T)(op.ceps * ih2);
    a.cdiag = (T)(6.0 * op.ceps * ih2 + op.sig_const);
    a.cidiag = (T)(1.0 / (6.0 * op.ceps * ih2 + op.sig_const));
    a.flags = g->flags;
    a.dirbit = dirbit(op);
    a.epsi = g->epsi;
    if constexpr (sizeof(T) == 8) {
        a.eps = g->eps64;
        a.ftab = g->ftab64;
        a.sig = op.sigma;
        a.stab = g->stab64;
    } else {
        a.eps = g->eps32;
        a.ftab = g->ftab32;
        a.sig = op.sigma ? g->sig32 : nullptr;   // converted by the mixed solve's set-up
        a.stab = g->stab32;
    }
    a.sigma = op.sigma;
    a.sig_const = op.sig_const;
    a.dval = g->dval;
    a.sc = g->sc;
    a.partials = g->partials;
    a.sink = reinterpret_cast<T *>(g->sink);
    return a;
}

template <typename T>
pfk::ZArgs<T> zbase(pf_grid *g, const OpDesc &op)
{
    return zbase_cfg<T>(g, op, cfg_of<T>(g));
}

// Launch with the shape c (the one a was built for).  The BiCGSTAB steps
// pick their kernel form from the operator; the other kernels have the plain
// and the PF1 form.
template <int OP, typename T>
pf_status zlaunch(pf_grid *g, const OpDesc &op, const pfk::ZArgs<T> &a, const ZCfg &c, hipEvent_t e0 = nullptr,
                  hipEvent_t e1 = nullptr)
{
    constexpr bool STEP = (OP == pfk::OP_BA || OP == pfk::OP_BB);
    constexpr bool PALOK = STEP || OP == pfk::OP_SPMV_JAC;
    const bool pal = PALOK && use_palette(g);
    constexpr int SN = STEP ? pfk::SIG_NODE : pfk::SIG_NONE, SC = STEP ? pfk::SIG_CLASS : pfk::SIG_NONE;
    hipError_t e;
    if (op.psi) e = launch_z<OP, T, true, pfk::SIG_NONE, false>(c, a, g->stream, e0, e1);
    else if (STEP && op.sigma)
        e = pal ? (op.sig_class ? launch_z<OP, T, false, SC, PALOK>(c, a, g->stream, e0, e1)
                                : launch_z<OP, T, false, SN, PALOK>(c, a, g->stream, e0, e1))
                : launch_z<OP, T, false, SN, false>(c, a, g->stream, e0, e1);
    else
        e = pal ? launch_z<OP, T, false, pfk::SIG_NONE, PALOK>(c, a, g->stream, e0, e1)
                : launch_z<OP, T, false, pfk::SIG_NONE, false>(c, a, g->stream, e0, e1);
    if (e != hipSuccess) return fail(PF_ERR_DEVICE, "stencil kernel launch failed: %s", hipGetErrorString(e));
    return PF_OK;
}

template <int KIND>
pf_status finalize(pf_grid *g, int G, int slot = 0)
{
    pfk::FinArgs f{g->sc, g->partials, G, slot};
    hipLaunchKernelGGL((pfk::k_finalize<KIND>), dim3(1), dim3(256), 0, g->stream, f);
    HIPCHK(hipGetLastError());
    return PF_OK;
}

// Set-up of an operator for FP32 kernels: the FP32 copy of its shift array.
pf_status prepare_f32(pf_grid *g, const OpDesc &op)
{
    if (!op.sigma) return PF_OK;
    hipLaunchKernelGGL((pfk::k_convert<float>), dim3(pw_blocks(g->N)), dim3(NT), 0, g->stream, g->N, op.sigma,
                       g->sig32);
    HIPCHK(hipGetLastError());
    return PF_OK;
}

// True FP64 residual r = b - A x (and ||r||^2 into sc->red[slot]); optional
// shadow copy (r rounded to FP32) and Krylov start vector (s^ = D^-1 r, FP64
// or FP32).  lift: use the Dirichlet values as x (b_lift).  The launch shape
// c, the partials buffer and the scalar block are the grid's unless given.
pf_status residual64(pf_grid *g, const OpDesc &op, const double *b, const double *x, double *r, bool lift,
                     float *rt32, double *rs64, float *rs32, int slot = 0, const ZCfg *cshape = nullptr,
                     double *partials = nullptr, Scalars *sc = nullptr)
{
    const ZCfg &c = cshape ? *cshape : cfg_of<double>(g);
    pfk::ZArgs<double> a = zbase_cfg<double>(g, op, c);
    if (partials) a.partials = partials;
    if (sc) a.sc = sc;
    a.x = x;
    a.out = r;
    a.b = b;
    a.lift = lift ? 1 : 0;
    a.dval = op.psi ? nullptr : g->dval;
    a.rt32 = rt32;
    a.rs64 = rs64;
    a.rs32 = rs32;
    if (lift && op.psi) {
        // PF1: Dirichlet value 0 everywhere, so b_lift = b on free rows
        a.lift = 0;
        a.x = nullptr;
    }
    if (a.x == nullptr && !a.lift) {
        // x == 0: reuse the lift path with a zero Dirichlet field
        a.lift = 1;
        a.dval = nullptr;
    }
    PFCHK((zlaunch<pfk::OP_RESID, double>(g, op, a, c)));
    // the partials buffer is reused by the next standalone reduction, which
    // follows in stream order
    pfk::FinArgs f{a.sc, a.partials, a.G, slot};
    hipLaunchKernelGGL((pfk::k_finalize<pfk::FIN_SUM>), dim3(1), dim3(256), 0, g->stream, f);
    HIPCHK(hipGetLastError());
    return PF_OK;
}

pf_status read_scalars(pf_grid *g)
{
    HIPCHK(hipMemcpyAsync(g->hsc, g->sc, sizeof(Scalars), hipMemcpyDeviceToHost, g->stream));
    return sync(g);
}

pf_status write_scalars(pf_grid *g)
{
    HIPCHK(hipMemcpyAsync(g->sc, g->hsc, sizeof(Scalars), hipMemcpyHostToDevice, g->stream));
    return PF_OK;
}

// Arguments of the two kernels of one BiCGSTAB iteration.  parity selects
// the p/v ping-pong buffers: step A reads p[parity], v[parity] and writes
// p[parity^1], v[parity^1].
template <typename T>
pfk::ZArgs<T> args_a(pf_grid *g, const OpDesc &op, Work<T> &w, int parity, const ZCfg &c, int Gb)
{
    pfk::ZArgs<T> a = zbase_cfg<T>(g, op, c);
    a.x = w.s;
    a.y0 = w.p[parity];
    a.y1 = w.v[parity];
    a.y2 = w.t;
    a.rt = w.rt;
    a.xio = w.x;
    a.out = w.v[parity ^ 1];
    a.out_aux = w.p[parity ^ 1];
    a.out_r = w.r;
    a.partials = g->partA;
    a.pin = g->partB;
    a.Gin = Gb;
    a.parity = parity;
    return a;
}

template <typename T>
pfk::ZArgs<T> args_b(pf_grid *g, const OpDesc &op, Work<T> &w, int parity, const ZCfg &c, int Ga)
{
    pfk::ZArgs<T> b = zbase_cfg<T>(g, op, c);
    b.x = w.r;
    b.y0 = w.v[parity ^ 1];
    b.rt = w.rt;
    b.out = w.t;
    b.out_aux = w.s;
    b.partials = g->partB;
    b.pin = g->partA;
    b.Gin = Ga;
    b.parity = parity;
    return b;
}

// One BiCGSTAB iteration: stencil step A (x, r of the previous iteration;
// p, v), stencil step B (s, t).
template <typename T>
pf_status iteration(pf_grid *g, const OpDesc &op, Work<T> &w, int parity, hipEvent_t e0 = nullptr,
                    hipEvent_t e1 = nullptr)
{
    const ZCfg &ca = cfg_ref<T>(g), &cb = cfgb_ref<T>(g);
    PFCHK((zlaunch<pfk::OP_BA, T>(g, op, args_a<T>(g, op, w, parity, ca, cb.G), ca, e0, e1)));
    PFCHK((zlaunch<pfk::OP_BB, T>(g, op, args_b<T>(g, op, w, parity, cb, ca.G), cb)));
    return PF_OK;
}

// Chunk of m iterations (m even) captured once per (precision, operator
// form, system) and replayed.  The graph references only grid-owned buffers
// and the operator's shift array, which is part of the key.
template <typename T>
pf_status run_chunk(pf_grid *g, const OpDesc &op, Work<T> &w, int m, bool may_time = true)
{
    const bool timed = may_time && g_timing.enabled && (g_timing.chunk++ % g_timing.sample) == 0;
    if (may_time) g->last_timed_first = timed;
    if (timed && (int)g->tev.size() < 2 * m) {
        while ((int)g->tev.size() < 2 * m) {
            hipEvent_t e;
            HIPCHK(hipEventCreate(&e));
            g->tev.push_back(e);
        }
    }
    if (timed) {
        // sampled chunk: direct launches with HIP events around step A
        for (int i = 0; i < m; ++i) PFCHK(iteration<T>(g, op, w, i & 1, g->tev[2 * i], g->tev[2 * i + 1]));
        return PF_OK;
    }
    const GraphKey key{m, (int)sizeof(T), step_form(op, g), op.sigma};
    auto it = g->graphs.find(key);
    if (it == g->graphs.end()) {
        hipGraph_t graph;
        HIPCHK(hipStreamBeginCapture(g->stream, hipStreamCaptureModeRelaxed));
        pf_status st = PF_OK;
        for (int i = 0; i < m && st == PF_OK; ++i) st = iteration<T>(g, op, w, i & 1);
        hipError_t e = hipStreamEndCapture(g->stream, &graph);
        if (st != PF_OK) return st;
        if (e != hipSuccess) return fail(PF_ERR_DEVICE, "graph capture failed: %s", hipGetErrorString(e));
        hipGraphExec_t exec;
        e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
        (void)hipGraphDestroy(graph);
        if (e != hipSuccess) return fail(PF_ERR_DEVICE, "graph instantiate failed: %s", hipGetErrorString(e));
        it = g->graphs.emplace(key, exec).first;
    }
    HIPCHK(hipGraphLaunch(it->second, g->stream));
    return PF_OK;
}

// ---------------------------------------------------------------- tuner

// Launch shapes chosen per (grid shape, precision) for this process: step A
// (also used by the residual and product kernels) and step B.
std::map<std::tuple<int, int, int, int>, std::pair<ZCfg, ZCfg>> g_tuned;

bool tuning_enabled()
{
    const char *e = getenv("PF_TUNE");
    if (e && e[0] == '0') return false;
    return !g_nt_override && !g_ppt_override && !g_kz_override && !g_depth_override;
}

// Candidate shapes of the z-march kernels on this grid.
template <typename T>
std::vector<ZCfg> tune_candidates(const pf_grid *g)
{
    std::vector<ZCfg> out;
    const int shapes[6][2] = {{256, 1}, {256, 2}, {512, 1}, {512, 2}, {1024, 1}, {1024, 2}};
    for (auto &sh : shapes)
        for (int kz : {2, 4, 8, 16, 32})
            for (int depth : {1, 2}) {
                ZCfg c = make_cfg(g->nx, g->ny, g->nz, sizeof(T), sh[0], sh[1], kz, depth);
                if (c.lds > LDS_MAX || c.G > g->Gmax || kz > g->nz) continue;
                if ((c.wide && (c.NTZ != 1024 || c.PPT != 1)) || c.depth != depth) continue;
                out.push_back(c);
            }
    return out;
}

// Time steps A and B of BiCGSTAB separately over the candidate shapes on this
// grid (A from a fresh start, then B after one run of the best A) and keep
// the fastest of each.  Runs once per grid shape and precision; the grid's
// workspace holds synthetic vectors meanwhile (every solve reinitialises it).
template <typename T>
pf_status tune(pf_grid *g)
{
    if (!tuning_enabled()) return PF_OK;
    const auto key = std::make_tuple(g->nx, g->ny, g->nz, (int)sizeof(T));
    auto found = g_tuned.find(key);
    if (found != g_tuned.end()) {
        cfg_ref<T>(g) = found->second.first;
        cfgb_ref<T>(g) = found->second.second;
        return PF_OK;
    }
    Work<T> &w = [&]() -> Work<T> & {
        if constexpr (sizeof(T) == 8) return g->w64;
        else return g->w32;
    }();
    // non-constant operands, so that no step finds a vanishing product (a
    // restart or stop decision would make the timed launches exit early)
    hipLaunchKernelGGL((pfk::k_fill_pattern<T>), dim3(pw_blocks(g->N)), dim3(NT), 0, g->stream, g->N, w.r, 0.0);
    hipLaunchKernelGGL((pfk::k_fill_pattern<T>), dim3(pw_blocks(g->N)), dim3(NT), 0, g->stream, g->N, w.s, 0.37);
    hipLaunchKernelGGL((pfk::k_fill_pattern<float>), dim3(pw_blocks(g->N)), dim3(NT), 0, g->stream, g->N, w.rt,
                       0.71);
    HIPCHK(hipGetLastError());
    PFCHK(fill<T>(g, w.t, T(0), g->N));
    PFCHK(fill<T>(g, w.p[0], T(0), g->N));
    PFCHK(fill<T>(g, w.v[0], T(0), g->N));
    Scalars &h = *g->hsc;
    h = Scalars{};
    h.rho[0] = h.rho[1] = 1.0; h.alpha[1] = 1.0; h.omega[1] = 1.0;
    h.stop = pfk::ST_RUN; h.stop_a = pfk::ST_RUN; h.fresh = 1;
    h.maxit = 1 << 30;
    hipEvent_t e0, e1;
    HIPCHK(hipEventCreate(&e0));
    HIPCHK(hipEventCreate(&e1));
    const std::vector<ZCfg> cand = tune_candidates<T>(g);
    OpDesc op;
    pf_status st = PF_OK;
    // mean time per launch of step OP with shape c over 8 back-to-back
    // launches (after one untimed launch), the best of two such runs; 1e30 if
    // the shape cannot be launched here
    auto time_step = [&](auto opc, const pfk::ZArgs<T> &a, const ZCfg &c) -> float {
        constexpr int OPV = decltype(opc)::value;
        constexpr int K = 8;
        float best = 1e30f;
        if ((st = write_scalars(g)) != PF_OK) return 1e30f;
        if (zlaunch<OPV, T>(g, op, a, c) != PF_OK) {
            (void)hipGetLastError();
            g_err.clear();
            return 1e30f;
        }
        for (int run = 0; run < 2; ++run) {
            if ((st = write_scalars(g)) != PF_OK) return 1e30f;
            if (hipEventRecord(e0, g->stream) != hipSuccess) {
                st = fail(PF_ERR_DEVICE, "event record failed");
                return 1e30f;
            }
            for (int k = 0; k < K; ++k)
                if ((st = zlaunch<OPV, T>(g, op, a, c)) != PF_OK) return 1e30f;
            if (hipEventRecord(e1, g->stream) != hipSuccess || hipEventSynchronize(e1) != hipSuccess) {
                st = fail(PF_ERR_DEVICE, "event timing failed");
                return 1e30f;
            }
            float ms = 0;
            (void)hipEventElapsedTime(&ms, e0, e1);
            best = std::min(best, ms / K);
        }
        return best;
    };
    using OpA = std::integral_constant<int, pfk::OP_BA>;
    using OpB = std::integral_constant<int, pfk::OP_BB>;
    ZCfg bestA = cfg_ref<T>(g), bestB = cfgb_ref<T>(g);
    float msA = 1e30f, msB = 1e30f;
    for (const ZCfg &c : cand) {
        pfk::ZArgs<T> a = args_a<T>(g, op, w, 0, c, c.G);
        a.xio = w.r;   // keep the caller's iterate: the timed launches update r in its place
        const float ms = time_step(OpA{}, a, c);
        if (st != PF_OK) break;
        if (ms < msA) { msA = ms; bestA = c; }
    }
    if (st == PF_OK) {
        // one step A with the chosen shape provides step B's input partials
        pfk::ZArgs<T> a = args_a<T>(g, op, w, 0, bestA, bestA.G);
        a.xio = w.r;
        st = write_scalars(g);
        if (st == PF_OK) st = zlaunch<pfk::OP_BA, T>(g, op, a, bestA);
        for (const ZCfg &c : cand) {
            if (st != PF_OK) break;
            const pfk::ZArgs<T> b = args_b<T>(g, op, w, 0, c, bestA.G);
            const float ms = time_step(OpB{}, b, c);
            if (st != PF_OK) break;
            if (ms < msB) { msB = ms; bestB = c; }
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (st != PF_OK) return st;
    cfg_ref<T>(g) = bestA;
    cfgb_ref<T>(g) = bestB;
    g_tuned[key] = {bestA, bestB};
    if (getenv("PF_LOG"))
        fprintf(stderr,
                "[pf] tuned %dx%dx%d %s: step A threads %d strip %d z-planes %d depth %d (%.1f us); "
                "step B threads %d strip %d z-planes %d depth %d (%.1f us)\n",
                g->nx, g->ny, g->nz, sizeof(T) == 8 ? "fp64" : "fp32", bestA.NTZ, bestA.S, bestA.KZ, bestA.depth,
                msA * 1e3, bestB.NTZ, bestB.S, bestB.KZ, bestB.depth, msB * 1e3);
    return PF_OK;
}

// Shapes of the standalone Jacobi-scaled product, per (grid shape, precision).
std::map<std::tuple<int, int, int, int>, ZCfg> g_tuned_p;

// Time the Jacobi-scaled product D^-1 A x over the candidate shapes on this
// grid and keep the fastest.  Its three streams (x, eps in; y out) favour
// other shapes than the eleven of step A.  Timed launches cycle through four
// (x, y) pairs of the grid's workspace so that consecutive launches do not
// find their vectors in the Infinity Cache.
template <typename T>
pf_status tune_product(pf_grid *g, const OpDesc &op)
{
    bool &done = sizeof(T) == 8 ? g->tunedp64 : g->tunedp32;
    if (done || !tuning_enabled()) return PF_OK;
    const auto key = std::make_tuple(g->nx, g->ny, g->nz, (int)sizeof(T));
    auto found = g_tuned_p.find(key);
    if (found != g_tuned_p.end()) {
        cfgp_ref<T>(g) = found->second;
        done = true;
        return PF_OK;
    }
    Work<T> &w = [&]() -> Work<T> & {
        if constexpr (sizeof(T) == 8) return g->w64;
        else return g->w32;
    }();
    T *xs[4] = {w.r, w.s, w.t, w.x};
    T *ys[4] = {w.p[0], w.p[1], w.v[0], w.v[1]};
    for (T *x : xs) PFCHK(fill<T>(g, x, T(1), g->N));
    hipEvent_t e0, e1;
    HIPCHK(hipEventCreate(&e0));
    HIPCHK(hipEventCreate(&e1));
    pf_status st = PF_OK;
    ZCfg best = cfgp_ref<T>(g);
    float best_ms = 1e30f;
    for (const ZCfg &c : tune_candidates<T>(g)) {
        pfk::ZArgs<T> a = zbase_cfg<T>(g, op, c);
        a.x = xs[0];
        a.out = ys[0];
        if (zlaunch<pfk::OP_SPMV_JAC, T>(g, op, a, c) != PF_OK) {   // shape not launchable here
            (void)hipGetLastError();
            g_err.clear();
            continue;
        }
        constexpr int K = 8;
        float ms_c = 1e30f;
        for (int run = 0; run < 2 && st == PF_OK; ++run) {
            if (hipEventRecord(e0, g->stream) != hipSuccess) { st = fail(PF_ERR_DEVICE, "event record failed"); break; }
            for (int k = 0; k < K && st == PF_OK; ++k) {
                a.x = xs[k & 3];
                a.out = ys[k & 3];
                st = zlaunch<pfk::OP_SPMV_JAC, T>(g, op, a, c);
            }
            if (st != PF_OK) break;
            if (hipEventRecord(e1, g->stream) != hipSuccess || hipEventSynchronize(e1) != hipSuccess) {
                st = fail(PF_ERR_DEVICE, "event timing failed");
                break;
            }
            float ms = 0;
            (void)hipEventElapsedTime(&ms, e0, e1);
            ms_c = std::min(ms_c, ms / K);
        }
        if (st != PF_OK) break;
        if (ms_c < best_ms) { best_ms = ms_c; best = c; }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (st != PF_OK) return st;
    cfgp_ref<T>(g) = best;
    g_tuned_p[key] = best;
    done = true;
    if (getenv("PF_LOG"))
        fprintf(stderr, "[pf] tuned %dx%dx%d %s product: threads %d strip %d z-planes %d depth %d (%.1f us)\n",
                g->nx, g->ny, g->nz, sizeof(T) == 8 ? "fp64" : "fp32", best.NTZ, best.S, best.KZ, best.depth,
                best_ms * 1e3);
    return PF_OK;
}

int chunk_len(const pf_grid *g, const pf_lin_opts *o)
{
    int m = o->check_every > 0 ? o->check_every : (g->N < 200000 ? 32 : 16);
    m = std::max(2, m + (m & 1));
    return m;
}

// Reset the Krylov state from a residual already in w.s (s^ = D^-1 r) and
// w.rt (the shadow r) with ||r||^2 = rr.  Keeps the cumulative iteration
// count.  Asynchronous: one kernel zeroes p^, v^, t^ (and x when zero_x) and
// writes the scalar block, whose host copy is set to the same values.  The
// first step A reads r^ from s^ (r^ = s^ - omega t^ with t^ = 0) and
// p^ = v^ = 0.
// A Krylov start recorded instead of launched (batched solves launch every
// member's start together, in one kernel on the batch's stream).
struct StartRec {
    pf_grid *g;
    int elem;
    void *p, *v, *t, *xz;
    Scalars init;
};
std::vector<StartRec> *g_defer_start = nullptr;   // set while a batch decides its next runs

template <typename T>
pf_status krylov_start(pf_grid *g, Work<T> &w, double rr, double tol2, int iter, int maxit, bool zero_x = false)
{
    Scalars &h = *g->hsc;
    h = Scalars{};
    h.rho[0] = rr;            // shadow = r, so rho_0 = ||r||^2
    h.alpha[1] = 1.0;
    h.omega[1] = 1.0;
    h.rr = rr;
    h.tol2 = tol2;
    h.rt2 = rr;
    h.iter[0] = iter;
    h.iter_done = iter;
    h.maxit = maxit;
    h.stop = pfk::ST_RUN;
    h.stop_a = pfk::ST_RUN;
    h.fresh = 1;
    if (g_defer_start) {
        g_defer_start->push_back(StartRec{g, (int)sizeof(T), w.p[0], w.v[0], w.t, zero_x ? (void *)w.x : nullptr, h});
        return PF_OK;
    }
    hipLaunchKernelGGL((pfk::k_krylov_start<T>), dim3(pw_blocks(g->N)), dim3(NT), 0, g->stream, g->N, w.p[0],
                       w.v[0], w.t, zero_x ? w.x : (T *)nullptr, h, g->sc);
    HIPCHK(hipGetLastError());
    return PF_OK;
}

// Iterate until the device reports a state other than RUN.  The first batch
// of iterations is sized from the previous run on the same grid and operator
// (the outer loop repeats similar warm-started solves): 90% of that count,
// launched as back-to-back graph chunks of power-of-two lengths with one host
// read at the end.  Later chunks are short, so few iterations run past
// convergence as no-ops.  A fixed check_every overrides this.
template <typename T>
pf_status krylov_run(pf_grid *g, const OpDesc &op, Work<T> &w, int m_fixed, int *status, bool adaptive)
{
    const int slot = (sizeof(T) == 8 ? 0 : 2) + (op.psi ? 1 : 0);
    const int start_iter = g->hsc->iter_done;
    for (int batch = 0;; ++batch) {
        int parts[16];
        int np = 0;
        const int expect = g->last_run[slot];
        if (adaptive && batch == 0 && expect >= 8) {
            int total = std::max(2, (expect * 9 / 10) & ~1);
            for (int m = 256; m >= 2 && np < 16; m >>= 1)
                while (total >= m && np < 16) { parts[np++] = m; total -= m; }
        } else {
            parts[np++] = !adaptive ? m_fixed : (batch == 0 ? m_fixed : 8);
        }
        const int before = g->hsc->iter_done;
        // only the batch's first chunk may be the timed sample: its events are
        // read after the batch, and its iterations are the first ones run
        for (int k = 0; k < np; ++k) PFCHK(run_chunk<T>(g, op, w, parts[k], k == 0));
        const bool timed = np > 0 && g->last_timed_first;
        PFCHK(read_scalars(g));
        if (timed && !op.psi) {
            // iterations whose step A ran in full (later ones exit at once)
            const int ran = std::min(parts[0], g->hsc->iter_done - before);
            const int pi = sizeof(T) == 8 ? 0 : 1;
            for (int i = 0; i < ran; ++i) {
                float ms = 0;
                HIPCHK(hipEventElapsedTime(&ms, g->tev[2 * i], g->tev[2 * i + 1]));
                g_timing.ms[pi] += ms;
                g_timing.launches[pi] += 1;
                g_timing.bytes[pi] += step_a_bytes(op, g, sizeof(T));
            }
        }
        if (g->hsc->stop != pfk::ST_RUN) {
            *status = g->hsc->stop;
            g->last_run[slot] = g->hsc->iter_done - start_iter;
            return PF_OK;
        }
    }
}

pf_status check_opts(const pf_lin_opts *o)
{
    if (!o) return fail(PF_ERR_ARG, "null options");
    if (!(o->rel_tol > 0.0) || !std::isfinite(o->rel_tol)) return fail(PF_ERR_ARG, "rel_tol must be > 0");
    if (o->max_iter <= 0) return fail(PF_ERR_ARG, "max_iter must be > 0");
    if (o->precision != PF_FP64 && o->precision != PF_MIXED) return fail(PF_ERR_ARG, "unknown precision");
    if (o->precision == PF_MIXED && (!(o->inner_tol > 0.0) || o->inner_tol >= 1.0 || o->max_refine <= 0))
        return fail(PF_ERR_ARG, "mixed precision needs 0 < inner_tol < 1 and max_refine > 0");
    if (o->check_every < 0) return fail(PF_ERR_ARG, "check_every must be >= 0");
    if (o->stop_rule != PF_STOP_REL2 && o->stop_rule != PF_STOP_ABS_INF) return fail(PF_ERR_ARG, "unknown stop_rule");
    return PF_OK;
}

// State of one linear solve on grid-owned buffers (g->b64 holds b, g->w64.x
// the initial guess and, at the end, the solution).  The same steps drive a
// single solve and every member of a batch:
//   ls_init        dinv, Dirichlet values, ||b_lift|| (read back);
//   ls_round_*     true FP64 residual (read back), then either finish or
//                  start a Krylov run (FP64 restart, or FP32 correction);
//   ls_after       account for the run (FP32: x += d, the previous x kept in
//                  the idle FP64 vector s).
// A refinement step whose correction does not lower the true residual (an
// FP32 Krylov run that lost its accuracy on a badly conditioned system) is
// undone, and the solve continues with FP64 Krylov runs (ls_fallback).
struct LinSolve {
    pf_grid *g = nullptr;
    OpDesc op;
    const pf_lin_opts *o = nullptr;
    bool mixed = false;
    double bnorm = 0, tol2 = 0, rr = 0, rinf = 0;   // rinf: true ||r||_inf (PF_STOP_ABS_INF)
    double rr_start = 0;                             // ||r||^2 when the last refinement step began
    double rr_best = INFINITY;                       // FP64 Krylov runs: smallest true ||r||^2 so far
    int stall = 0;                                   // consecutive runs that did not halve ||r||
    int iter = 0, restarts = 0, refinements = 0;
    bool started = false, done = false, fallback = false;
    bool class_probe = false;   // the shift-per-class test ran in the set-up
    pf_status result = PF_OK;
};

// True residual of the current x into red[0] (and the shadow / FP32 copies
// the next Krylov run starts from).  Asynchronous.
pf_status ls_round_residual(LinSolve &L)
{
    pf_grid *g = L.g;
    if (L.mixed)
        PFCHK(residual64(g, L.op, g->b64, g->w64.x, g->w64.r, false, g->w32.rt, nullptr, g->w32.s));
    else
        PFCHK(residual64(g, L.op, g->b64, g->w64.x, g->w64.r, false, g->w64.rt, g->w64.s, nullptr));
    if (L.o->stop_rule == PF_STOP_ABS_INF) {   // ||r||_inf of the free rows into red[2]
        const int B = pw_blocks(g->N);
        hipLaunchKernelGGL(pfk::k_maxabs_free<NT>, dim3(B), dim3(NT), 0, g->stream, g->N, (const double *)g->w64.r,
                           (const uint8_t *)g->flags, dirbit(L.op), g->partials);
        HIPCHK(hipGetLastError());
        PFCHK(finalize<pfk::FIN_MAX>(g, B, 2));
    }
    return PF_OK;
}

// dinv, Dirichlet values, ||b_lift||^2 into red[1] and the first true
// residual into red[0]: one host read for both.
pf_status ls_init_launch(LinSolve &L)
{
    pf_grid *g = L.g;
    PFCHK(check_opts(L.o));
    PFCHK(ensure_work<double>(g));
    L.mixed = L.o->precision == PF_MIXED;
    if (L.mixed) PFCHK(ensure_work<float>(g));
    if (L.op.sigma) {   // sigma >= 0 on free rows, read back with ||b_lift||
        PFCHK(fill<int>(g, &g->sc->neg_shift, 0, 1));
        hipLaunchKernelGGL(pfk::k_check_shift, dim3(pw_blocks(g->N)), dim3(NT), 0, g->stream, g->N, L.op.sigma,
                           (const uint8_t *)g->flags, dirbit(L.op), &g->sc->neg_shift);
        HIPCHK(hipGetLastError());
    }
    if (L.op.sigma && L.op.sigma != g->sig) {
        // the iteration's kernels (and their captured graphs) read a
        // grid-owned copy of a caller's shift array
        if (!g->sig64) PFCHK(dalloc(g, &g->sig64, g->N));
        HIPCHK(hipMemcpyAsync(g->sig64, L.op.sigma, g->N * sizeof(double), hipMemcpyDeviceToDevice, g->stream));
        L.op.sigma = g->sig64;
    }
    if (L.mixed) PFCHK(prepare_f32(g, L.op));
    L.op.sig_class = false;
    // (not for the outer loop's own shift, the Fermi derivative, which
    // varies over the solvent)
    L.class_probe = L.op.sigma && L.op.sigma != g->sig && !L.op.psi && use_palette(g) && shift_class_enabled();
    if (L.class_probe) {   // is sigma one value per palette class?  read back with ||b_lift||
        if (!g->smm) {
            PFCHK(dalloc(g, &g->smm, 2 * pfk::PAL_MAX));
            PFCHK(dalloc(g, &g->stab64, pfk::PAL_MAX));
            PFCHK(dalloc(g, &g->stab32, pfk::PAL_MAX));
        }
        PFCHK(fill<unsigned long long>(g, g->smm, ~0ull, pfk::PAL_MAX));
        PFCHK(fill<unsigned long long>(g, g->smm + pfk::PAL_MAX, 0ull, pfk::PAL_MAX));
        hipLaunchKernelGGL(pfk::k_shift_classes, dim3(pw_blocks(g->N)), dim3(NT), 0, g->stream, g->N, L.op.sigma,
                           (const uint8_t *)g->epsi, g->smm);
        HIPCHK(hipGetLastError());
        hipLaunchKernelGGL(pfk::k_shift_table, dim3(1), dim3(64), 0, g->stream, (const unsigned long long *)g->smm,
                           g->stab64, g->stab32, &g->sc->shift_class);
        HIPCHK(hipGetLastError());
    }
    hipLaunchKernelGGL(pfk::k_set_dirichlet, dim3(pw_blocks(g->N)), dim3(NT), 0, g->stream, g->N, g->w64.x,
                       (const uint8_t *)g->flags, dirbit(L.op), L.op.psi ? nullptr : (const double *)g->dval);
    HIPCHK(hipGetLastError());
    PFCHK(residual64(g, L.op, g->b64, nullptr, g->w64.r, true, nullptr, nullptr, nullptr, 1));
    PFCHK(ls_round_residual(L));
    HIPCHK(hipMemcpyAsync(g->hsc, g->sc, sizeof(Scalars), hipMemcpyDeviceToHost, g->stream));
    return PF_OK;
}

// After the stream has synchronised.
pf_status ls_init_decide(LinSolve &L)
{
    pf_grid *g = L.g;
    if (L.op.sigma && g->hsc->neg_shift) {
        L.done = true;
        L.result = PF_ERR_ARG;
        return PF_OK;
    }
    L.op.sig_class = L.class_probe && g->hsc->shift_class;
    L.bnorm = std::sqrt(g->hsc->red[1]);
    if (!std::isfinite(L.bnorm)) {
        L.done = true;
        L.result = PF_ERR_NONFINITE;
        return PF_OK;
    }
    if (L.bnorm == 0.0) {
        // homogeneous problem: x = Dirichlet values, 0 on free rows
        PFCHK(fill<double>(g, g->w64.x, 0.0, g->N));
        hipLaunchKernelGGL(pfk::k_set_dirichlet, dim3(pw_blocks(g->N)), dim3(NT), 0, g->stream, g->N, g->w64.x,
                           (const uint8_t *)g->flags, dirbit(L.op), L.op.psi ? nullptr : (const double *)g->dval);
        HIPCHK(hipGetLastError());
        L.done = true;
        return PF_OK;
    }
    // the device-side trigger: ||r||_2^2 <= tol2.  For the max-norm rule,
    // ||r||_inf <= tol implies ||r||_2^2 <= N tol^2, so the trigger fires no
    // later than the rule can hold; the true max norm then decides.
    if (L.o->stop_rule == PF_STOP_ABS_INF) L.tol2 = (double)g->N * L.o->rel_tol * L.o->rel_tol;
    else L.tol2 = L.o->rel_tol * L.o->rel_tol * L.bnorm * L.bnorm;
    return PF_OK;
}

pf_status ls_round_launch(LinSolve &L)
{
    PFCHK(ls_round_residual(L));
    HIPCHK(hipMemcpyAsync(L.g->hsc, L.g->sc, sizeof(Scalars), hipMemcpyDeviceToHost, L.g->stream));
    return PF_OK;
}

// Undo the last FP32 correction (x from before it is in w64.s) and continue
// the solve in FP64: the true residual and the FP64 shadow are computed again
// and read back.
pf_status ls_fallback(LinSolve &L)
{
    pf_grid *g = L.g;
    HIPCHK(hipMemcpyAsync(g->w64.x, g->w64.s, g->N * sizeof(double), hipMemcpyDeviceToDevice, g->stream));
    L.mixed = false;
    L.fallback = true;
    PFCHK(ls_round_residual(L));
    HIPCHK(hipMemcpyAsync(g->hsc, g->sc, sizeof(Scalars), hipMemcpyDeviceToHost, g->stream));
    PFCHK(sync(g));
    L.rr = g->hsc->red[0];
    return PF_OK;
}

// After the stream has synchronised: finish, or start a Krylov run (*run).
pf_status ls_round_decide(LinSolve &L, bool *run)
{
    pf_grid *g = L.g;
    *run = false;
    L.rr = g->hsc->red[0];
    if (L.mixed && L.refinements > 0 && !(L.rr < L.rr_start)) PFCHK(ls_fallback(L));
    if (!std::isfinite(L.rr)) { L.result = PF_ERR_NONFINITE; L.done = true; return PF_OK; }
    if (L.o->stop_rule == PF_STOP_ABS_INF) {
        L.rinf = g->hsc->red[2];
        if (L.rinf <= L.o->rel_tol) { L.done = true; return PF_OK; }
        // the max norm still misses: aim the device trigger at the L2 norm
        // the max norm should reach if both shrink together (with a margin);
        // never below tol^2, where ||r||_2 <= tol already implies the rule
        const double tol = L.o->rel_tol, q = tol / L.rinf;
        L.tol2 = std::max(tol * tol, std::min(L.tol2, 0.25 * q * q * L.rr));
    } else if (L.rr <= L.tol2) {
        L.done = true;
        return PF_OK;
    }
    if (!L.mixed) {
        if (L.iter >= L.o->max_iter) { L.result = PF_ERR_NOCONV; L.done = true; return PF_OK; }
        // a tolerance below the attainable accuracy (rounding of A x at the
        // operator's condition number) shows as runs that end by the
        // recurrence while the true residual stays put: stop after three
        if (L.started) {
            L.stall = (L.rr > 0.25 * L.rr_best) ? L.stall + 1 : 0;
            if (L.stall >= 3) { L.result = PF_ERR_NOCONV; L.done = true; return PF_OK; }
        }
        L.rr_best = std::min(L.rr_best, L.rr);
        if (L.started) ++L.restarts;
        if (L.restarts > 1000) { L.result = PF_ERR_BREAKDOWN; L.done = true; return PF_OK; }
        L.started = true;
        PFCHK(krylov_start<double>(g, g->w64, L.rr, L.tol2, L.iter, L.o->max_iter));
    } else {
        if (L.refinements >= L.o->max_refine || L.iter >= L.o->max_iter) {
            L.result = PF_ERR_NOCONV;
            L.done = true;
            return PF_OK;
        }
        ++L.refinements;
        L.rr_start = L.rr;
        const double itol2 = L.o->inner_tol * L.o->inner_tol;
        PFCHK(krylov_start<float>(g, g->w32, L.rr, std::max(itol2 * L.rr, L.tol2), L.iter, L.o->max_iter, true));
    }
    *run = true;
    return PF_OK;
}

// After a Krylov run that ended with device status st (g->hsc is current).
// gpu = false: the caller does the copy and correction of every member in
// one batched launch.
pf_status ls_after(LinSolve &L, int st, bool gpu = true)
{
    pf_grid *g = L.g;
    L.iter = g->hsc->iter_done;
    if (L.mixed) {
        // keep x from before the correction; a non-finite FP32 run adds
        // nothing, so the next true residual equals the last one and the
        // solve falls back to FP64 (ls_round_decide)
        if (st == pfk::ST_RESTART) ++L.restarts;
        if (!gpu) return PF_OK;
        HIPCHK(hipMemcpyAsync(g->w64.s, g->w64.x, g->N * sizeof(double), hipMemcpyDeviceToDevice, g->stream));
        if (st != pfk::ST_NONFINITE) {
            hipLaunchKernelGGL(pfk::k_correct, dim3(pw_blocks(g->N)), dim3(NT), 0, g->stream, g->N, g->w64.x,
                               (const float *)g->w32.x, (const uint8_t *)g->flags, dirbit(L.op));
            HIPCHK(hipGetLastError());
        }
        return PF_OK;
    }
    if (st == pfk::ST_NONFINITE) { L.result = PF_ERR_NONFINITE; L.done = true; return PF_OK; }
    // FP64: CONV, MAXIT and RESTART all return to the true residual
    return PF_OK;
}

pf_status ls_finish(const LinSolve &L, pf_lin_info *info)
{
    pf_lin_info li{};
    li.iters = L.iter;
    li.refinements = L.refinements;
    li.restarts = L.restarts;
    li.rel_res = L.bnorm > 0 ? std::sqrt(L.rr) / L.bnorm : 0.0;
    li.max_res = L.o->stop_rule == PF_STOP_ABS_INF ? L.rinf : -1.0;
    li.status = L.result;
    li.fp64_fallback = L.fallback ? 1 : 0;
    if (info) *info = li;
    if (L.result == PF_ERR_NOCONV && L.o->stop_rule == PF_STOP_ABS_INF)
        return fail(L.result, "no convergence: max residual %.3e after %d iterations", L.rinf, L.iter);
    if (L.result == PF_ERR_NOCONV)
        return fail(L.result, "no convergence: rel_res %.3e after %d iterations", li.rel_res, L.iter);
    if (L.result == PF_ERR_NONFINITE) return fail(L.result, "non-finite value in the iteration");
    if (L.result == PF_ERR_BREAKDOWN) return fail(L.result, "repeated BiCGSTAB breakdown");
    if (L.result == PF_ERR_ARG) return fail(L.result, "sigma must be >= 0 on every free row");
    return PF_OK;
}

pf_status solve_internal(pf_grid *g, const OpDesc &op, const pf_lin_opts *o, pf_lin_info *info)
{
    LinSolve L;
    L.g = g;
    L.op = op;
    L.o = o;
    PFCHK(ls_init_launch(L));
    PFCHK(sync(g));
    PFCHK(ls_init_decide(L));
    const int m = chunk_len(g, o);
    bool first = true;   // the first true residual came with the init read
    while (!L.done) {
        if (!first) {
            PFCHK(ls_round_launch(L));
            PFCHK(sync(g));
        }
        first = false;
        bool run = false;
        PFCHK(ls_round_decide(L, &run));
        if (!run) break;
        int st = 0;
        const bool adaptive = o->check_every == 0;
        if (L.mixed) PFCHK(krylov_run<float>(g, L.op, g->w32, m, &st, adaptive));
        else PFCHK(krylov_run<double>(g, L.op, g->w64, m, &st, adaptive));
        PFCHK(ls_after(L, st));
    }
    return ls_finish(L, info);
}

// ------------------------------------------------------------------ batch

// Device tables of a batched Krylov run: kernel arguments per system, block
// offsets, scalar pointers and a gather buffer.  Grows on demand; one batch
// runs at a time per process.
struct BatchBuf {
    void *dev = nullptr;
    size_t bytes = 0;
    Scalars *hsc = nullptr;
    int hcap = 0;
    std::vector<hipEvent_t> ev;   // kernel timing of sampled chunks
} g_batch;

// Launch of one batched BiCGSTAB step: every member shares the kernel
// instance (threads, nodes per thread, pipeline depth).  Policies:
//   0: the instance most of the work was tuned to on its own (weighted by N),
//      each member with the z-chunk length of its own tuned shape;
//   1: 512 threads, one node per thread, the default depth, z-chunks of
//      clamp(strips nz / 256, 2, 16) planes (a batch has more tiles than one
//      system, so longer chunks lose less to the planes above and below);
//   2: 512 threads, one node per thread, depth 1, the members' z-chunks;
//   3: 256 threads, one node per thread, depth 1, long z-chunks as in 1;
//   4, 5: 512 threads, one node per thread, the default depth, z-chunks of
//      32 and 16 planes for every member (fewer planes re-read above and
//      below a chunk on the small members, fewer tiles once few members are
//      left);
//   6: as 5 for step A; step B with 512 threads x two nodes (its lighter
//      work per node favours longer strips);
//   7: as 5 for step A; step B with z-chunks of 32 planes;
//   8: as 5 for step A; step B as 6 with z-chunks of 32 planes.
// Step B with z-chunks of 64 planes was slower than 7 and dropped.
// step: 0 = A, 1 = B.
constexpr int NPOLICY = 9;

template <typename T>
std::vector<ZCfg> batch_shapes(const std::vector<LinSolve *> &act, int step, int policy, ZCfg &combined)
{
    int ntz = 512, ppt = 1, depth = default_depth(sizeof(T), 1);
    const bool own_kz = policy == 0 || policy == 2;
    if (policy == 2) depth = 1;
    if (policy == 3) { ntz = 256; depth = 1; }
    if ((policy == 6 || policy == 8) && step == 1) { ppt = 2; depth = default_depth(sizeof(T), 2); }
    if (policy == 0) {
        std::map<std::tuple<int, int, int>, double> weight;
        for (const LinSolve *L : act) {
            const ZCfg &t = step == 0 ? cfg_ref<T>(L->g) : cfgb_ref<T>(L->g);
            weight[std::make_tuple(t.NTZ, t.PPT, t.depth)] += (double)L->g->N;
        }
        auto best = std::max_element(weight.begin(), weight.end(),
                                     [](const auto &x, const auto &y) { return x.second < y.second; });
        ntz = std::get<0>(best->first);
        ppt = std::get<1>(best->first);
        depth = std::get<2>(best->first);
    }
    std::vector<ZCfg> cs;
    combined = ZCfg{};
    combined.NTZ = ntz;
    combined.PPT = ppt;
    combined.depth = depth;
    combined.G = 0;
    for (const LinSolve *L : act) {
        const pf_grid *g = L->g;
        int kz;
        if (own_kz) {
            kz = (step == 0 ? cfg_ref<T>(L->g) : cfgb_ref<T>(L->g)).KZ;
        } else if (policy >= 4) {
            kz = 16;   // 5, 6, and step A of 7 and 8
            if (policy == 4 || ((policy == 7 || policy == 8) && step == 1)) kz = 32;
        } else {
            const long S = (long)ntz * ppt;
            const long strips = ((long)g->nx * g->ny + S - 1) / S;
            kz = (int)std::max<long>(2, std::min<long>(16, strips * g->nz / 256));
        }
        ZCfg c = make_cfg(g->nx, g->ny, g->nz, sizeof(T), ntz, ppt, kz, depth);
        cs.push_back(c);
        combined.G += c.G;
        combined.lds = std::max(combined.lds, c.lds);
        combined.wide = combined.wide || c.wide;
    }
    if (combined.wide) {   // only the 1024-thread, one-node-per-thread instance has the WIDE form
        combined.NTZ = 1024; combined.PPT = 1; combined.depth = 1; combined.G = 0; combined.lds = 0;
        for (size_t i = 0; i < act.size(); ++i) {
            const pf_grid *g = act[i]->g;
            cs[i] = make_cfg(g->nx, g->ny, g->nz, sizeof(T), 1024, 1, cs[i].KZ, 1);
            combined.G += cs[i].G;
            combined.lds = std::max(combined.lds, cs[i].lds);
        }
    }
    return cs;
}

// Policy chosen per batch composition (precision, kernel form, member
// shapes) from one chunk per policy (its first chunks, over as many runs as
// that takes): the one with the most node-iterations per second is kept.
std::map<std::vector<long>, int> g_batch_policy;
std::map<std::vector<long>, std::vector<double>> g_batch_trials;   // per policy, -1 = not yet timed

// One instantiated graph chunk of a batched Krylov run under one policy, and
// the launches it holds (for the sampled chunks of kernel timing, which run
// as direct launches with events around step A).
struct BatchPlan {
    hipGraphExec_t exec = nullptr;
    std::function<pf_status(int, hipEvent_t, hipEvent_t)> launch_iter;
    // the first iteration after another plan's: step A from a table (device)
    // whose partial counts are that plan's step B tile counts
    std::function<pf_status(int, const void *)> launch_switch;
    std::function<void()> gather;
    std::vector<int> gB;   // step B tile count per member
    ~BatchPlan()
    {
        if (exec) (void)hipGraphExecDestroy(exec);
    }
};

// Run the Krylov iterations of all listed systems (same precision, same
// operator kind) together: one launch per kernel per iteration covers every
// system, captured as a graph chunk and replayed until no system is RUN.
// members: shapes of the whole batch (the policy is chosen for the batch
// and kept for every subset of its members that still iterates).
template <typename T>
pf_status batch_krylov_run(std::vector<LinSolve *> &act, const std::vector<long> &members, hipStream_t stream, int m,
                           std::vector<int> &status)
{
    const int n = (int)act.size();
    const bool psi = act[0]->op.psi;
    // one kernel form for every member: the SIG form if any member has a
    // shift array (members without one read zeros)
    int form = psi ? FORM_CEPS : FORM_PLAIN;
    if (!psi) {
        bool sig = false, pal = true, cls = true;
        for (const LinSolve *L : act) {
            sig = sig || L->op.sigma;
            pal = pal && use_palette(L->g);
            cls = cls && L->op.sigma && L->op.sig_class;
        }
        form = pal ? (sig ? (cls ? FORM_PALTAB : FORM_PALSIG) : FORM_PAL) : (sig ? FORM_SIG : FORM_PLAIN);
    }
    std::vector<long> key = {(long)sizeof(T), (long)form};
    key.insert(key.end(), members.begin(), members.end());
    const auto known = g_batch_policy.find(key);
    // PF_BATCH_POLICY=k forces policy k (profiler runs, whose serialised
    // launches would distort the comparison)
    const char *forced_env = getenv("PF_BATCH_POLICY");
    const int forced = forced_env ? std::min(NPOLICY - 1, std::max(0, atoi(forced_env))) : -1;
    // only batches of several members are compared (small ones keep policy 0)
    const int npol = (forced >= 0 || known != g_batch_policy.end() || !tuning_enabled() || members.size() < 4)
                         ? 1 : NPOLICY;
    const int pol0 = forced >= 0 ? forced : (known != g_batch_policy.end() ? known->second : 0);
    std::vector<double> *trials = nullptr;
    if (npol > 1) {
        trials = &g_batch_trials[key];
        if (trials->empty()) trials->assign(NPOLICY, -1.0);
    }
    auto next_untried = [&]() {
        for (int k = 0; k < NPOLICY; ++k)
            if ((*trials)[k] < 0) return k;
        return -1;
    };

    // device tables: per policy the step A / B arguments (two parities) and
    // tile start tables; shared scalar pointers and gather buffer
    const size_t szZ = sizeof(pfk::ZArgs<T>) * n;
    const size_t szI = sizeof(int) * (n + 1), szP = sizeof(void *) * n, szS = sizeof(Scalars) * n;
    auto al = [](size_t x) { return (x + 255) & ~(size_t)255; };
    const size_t per_pol = 4 * al(szZ) + 4 * al(szI) + al(sizeof(int) * n) + al(sizeof(int));
    const size_t need = npol * per_pol + al(szP) + al(szS) + al(szZ);
    if (need > g_batch.bytes) {
        if (g_batch.dev) (void)hipFree(g_batch.dev);
        g_batch.dev = nullptr;
        g_batch.bytes = 0;
        if (hipMalloc(&g_batch.dev, need) != hipSuccess) return fail(PF_ERR_ALLOC, "batch table allocation failed");
        g_batch.bytes = need;
    }
    if (n > g_batch.hcap) {
        if (g_batch.hsc) (void)hipHostFree(g_batch.hsc);
        g_batch.hsc = nullptr;
        g_batch.hcap = 0;
        if (hipHostMalloc((void **)&g_batch.hsc, szS, hipHostMallocDefault) != hipSuccess)
            return fail(PF_ERR_ALLOC, "batch pinned allocation failed");
        g_batch.hcap = n;
    }
    char *base = (char *)g_batch.dev;
    size_t off = 0;
    auto take = [&](size_t sz) { char *p = base + off; off += al(sz); return p; };
    std::vector<const Scalars *> scp(n);
    for (int i = 0; i < n; ++i) scp[i] = act[i]->g->sc;
    const Scalars **dscp = (const Scalars **)take(szP);
    Scalars *dgather = (Scalars *)take(szS);
    pfk::ZArgs<T> *dsw = (pfk::ZArgs<T> *)take(szZ);   // step-A table of a policy switch
    std::vector<pfk::ZArgs<T>> zas[NPOLICY][2];         // host copies of the step-A tables
    HIPCHK(hipMemcpyAsync(dscp, scp.data(), szP, hipMemcpyHostToDevice, stream));

    BatchPlan plans[NPOLICY];
    for (int k = 0; k < npol; ++k) {
        const int pol = npol == 1 ? pol0 : k;
        std::vector<pfk::ZArgs<T>> za[2], zb[2];
        std::vector<int> astart(n + 1, 0), bstart(n + 1, 0);
        ZCfg ca, cb;   // combined launches of steps A and B
        const std::vector<ZCfg> csa = batch_shapes<T>(act, 0, pol, ca), csb = batch_shapes<T>(act, 1, pol, cb);
        for (int par = 0; par < 2; ++par) { za[par].resize(n); zb[par].resize(n); }
        for (int i = 0; i < n; ++i) {
            LinSolve &L = *act[i];
            pf_grid *g = L.g;
            Work<T> *w;
            if constexpr (sizeof(T) == 8) w = &g->w64;
            else w = &g->w32;
            const T *zero_sig = nullptr;
            if ((form == FORM_SIG || form == FORM_PALSIG) && !L.op.sigma) {
                if constexpr (sizeof(T) == 8) {
                    if (!g->sig64) PFCHK(dalloc(g, &g->sig64, g->N));
                    zero_sig = g->sig64;
                } else {
                    zero_sig = g->sig32;
                }
                PFCHK(fill<T>(g, const_cast<T *>(zero_sig), T(0), g->N));
            }
            for (int par = 0; par < 2; ++par) {
                za[par][i] = args_a<T>(g, L.op, *w, par, csa[i], csb[i].G);
                zb[par][i] = args_b<T>(g, L.op, *w, par, csb[i], csa[i].G);
                if (zero_sig) za[par][i].sig = zb[par][i].sig = zero_sig;
            }
            astart[i + 1] = astart[i] + csa[i].G;
            bstart[i + 1] = bstart[i] + csb[i].G;
        }
        if (ca.lds > LDS_MAX || cb.lds > LDS_MAX) return fail(PF_ERR_ARG, "batch member too wide for the LDS strip");
        pfk::ZArgs<T> *dA[2] = {(pfk::ZArgs<T> *)take(szZ), (pfk::ZArgs<T> *)take(szZ)};
        pfk::ZArgs<T> *dB[2] = {(pfk::ZArgs<T> *)take(szZ), (pfk::ZArgs<T> *)take(szZ)};
        int *das = (int *)take(szI), *dbs = (int *)take(szI);
        // the active members' list and tile prefixes (k_batch_active)
        int *dpa = (int *)take(szI), *dpb = (int *)take(szI), *dact = (int *)take(sizeof(int) * n);
        int *dna = (int *)take(sizeof(int));
        for (int par = 0; par < 2; ++par) {
            HIPCHK(hipMemcpyAsync(dA[par], za[par].data(), szZ, hipMemcpyHostToDevice, stream));
            HIPCHK(hipMemcpyAsync(dB[par], zb[par].data(), szZ, hipMemcpyHostToDevice, stream));
        }
        HIPCHK(hipMemcpyAsync(das, astart.data(), szI, hipMemcpyHostToDevice, stream));
        HIPCHK(hipMemcpyAsync(dbs, bstart.data(), szI, hipMemcpyHostToDevice, stream));
        HIPCHK(hipStreamSynchronize(stream));   // the host vectors above go out of scope
        zas[k][0] = za[0];
        zas[k][1] = za[1];
        plans[k].gB.resize(n);
        for (int i = 0; i < n; ++i) plans[k].gB[i] = csb[i].G;

        // iteration i of a run of launches (parity i & 1); the active-member
        // list is refreshed every LIST_EVERY iterations: a member that stops
        // in between keeps its tiles in the launches until the next refresh,
        // where they leave at their first test of the stop state
        plans[k].launch_iter = [=](int i, hipEvent_t e0, hipEvent_t e1) -> pf_status {
            constexpr int LIST_EVERY = 8;
            const int par = i & 1;
            hipError_t e = hipSuccess;
            if (i % LIST_EVERY == 0) {
                hipLaunchKernelGGL(pfk::k_batch_active, dim3(1), dim3(pfk::ACT_NT), 0, stream, dscp,
                                   (const int *)das, (const int *)dbs, n, dact, dpa, dpb, dna);
                e = hipGetLastError();
                if (e != hipSuccess)
                    return fail(PF_ERR_DEVICE, "active-member list launch failed: %s", hipGetErrorString(e));
            }
            e = launch_batch_form<pfk::OP_BA, T>(form, ca, dA[par], dact, dpa, dna, stream, e0, e1);
            if (e != hipSuccess) return fail(PF_ERR_DEVICE, "batched step A launch failed: %s", hipGetErrorString(e));
            e = launch_batch_form<pfk::OP_BB, T>(form, cb, dB[par], dact, dpb, dna, stream);
            if (e != hipSuccess) return fail(PF_ERR_DEVICE, "batched step B launch failed: %s", hipGetErrorString(e));
            return PF_OK;
        };
        plans[k].launch_switch = [=](int i, const void *dAs) -> pf_status {
            const int par = i & 1;
            hipLaunchKernelGGL(pfk::k_batch_active, dim3(1), dim3(pfk::ACT_NT), 0, stream, dscp, (const int *)das,
                               (const int *)dbs, n, dact, dpa, dpb, dna);
            hipError_t e = hipGetLastError();
            if (e != hipSuccess) return fail(PF_ERR_DEVICE, "active-member list launch failed: %s", hipGetErrorString(e));
            e = launch_batch_form<pfk::OP_BA, T>(form, ca, (const pfk::ZArgs<T> *)dAs, dact, dpa, dna, stream);
            if (e != hipSuccess) return fail(PF_ERR_DEVICE, "batched step A launch failed: %s", hipGetErrorString(e));
            e = launch_batch_form<pfk::OP_BB, T>(form, cb, dB[par], dact, dpb, dna, stream);
            if (e != hipSuccess) return fail(PF_ERR_DEVICE, "batched step B launch failed: %s", hipGetErrorString(e));
            return PF_OK;
        };
        plans[k].gather = [=]() {
            hipLaunchKernelGGL(pfk::k_gather_scalars, dim3((n + 63) / 64), dim3(64), 0, stream, dscp, dgather, n);
        };
    }
    // Step A of iteration i sums the partials that step B of iteration i - 1
    // wrote, one per step-B tile of each member: the first iteration of plan
    // q after iterations of plan p reads plan p's counts (the policies tile
    // the members differently).
    std::vector<pfk::ZArgs<T>> zsw;
    auto switch_iter = [&](int q, int p, int i) -> pf_status {
        zsw = zas[q][i & 1];
        for (int j = 0; j < n; ++j) zsw[j].Gin = plans[p].gB[j];
        HIPCHK(hipMemcpyAsync(dsw, zsw.data(), szZ, hipMemcpyHostToDevice, stream));
        return plans[q].launch_switch(i, dsw);
    };
    // the chunk graph of plan k, captured on first use
    auto capture = [&](int k) -> pf_status {
        if (plans[k].exec) return PF_OK;
        hipGraph_t graph;
        HIPCHK(hipStreamBeginCapture(stream, hipStreamCaptureModeRelaxed));
        pf_status st = PF_OK;
        for (int i = 0; i < m && st == PF_OK; ++i) st = plans[k].launch_iter(i, nullptr, nullptr);
        plans[k].gather();
        hipError_t e = hipStreamEndCapture(stream, &graph);
        if (st != PF_OK) return st;
        if (e != hipSuccess) return fail(PF_ERR_DEVICE, "batch graph capture failed: %s", hipGetErrorString(e));
        e = hipGraphInstantiate(&plans[k].exec, graph, nullptr, nullptr, 0);
        (void)hipGraphDestroy(graph);
        if (e != hipSuccess) {
            plans[k].exec = nullptr;
            return fail(PF_ERR_DEVICE, "batch graph instantiate failed: %s", hipGetErrorString(e));
        }
        return PF_OK;
    };

    status.assign(n, pfk::ST_RUN);
    int use = 0;   // plan index of the chunks
    // kernel timing: iterations done per member before the chunk, step-A bytes per member
    std::vector<int> before(n);
    std::vector<double> abytes(n);
    for (int i = 0; i < n; ++i) {
        before[i] = act[i]->g->hsc->iter_done;
        abytes[i] = step_a_bytes(act[i]->op, act[i]->g, sizeof(T));
    }
    const int tslot = sizeof(T) == 8 ? 4 : 5;
    // one status read: members' scalars to the host, status updated; false
    // once no member iterates
    auto read_status = [&]() -> pf_status {
        HIPCHK(hipMemcpyAsync(g_batch.hsc, dgather, szS, hipMemcpyDeviceToHost, stream));
        HIPCHK(hipStreamSynchronize(stream));
        for (int i = 0; i < n; ++i) status[i] = g_batch.hsc[i].stop;
        return PF_OK;
    };
    auto running = [&]() {
        for (int i = 0; i < n; ++i)
            if (status[i] == pfk::ST_RUN) return true;
        return false;
    };
    if (npol > 1) {
        // every policy runs the same few iterations at the start of the run,
        // while (nearly) every member still iterates: two untimed (first
        // launches of a kernel instance), then TRIAL timed, each policy in
        // turn; the node-iterations per second decide
        constexpr int WARM = 2, TRIAL = 4;
        std::vector<double> &t = *trials;
        for (int k = 0; k < NPOLICY && running(); ++k) {
            for (int i = 0; i < WARM; ++i) {
                if (i == 0 && k > 0) PFCHK(switch_iter(k, k - 1, i));
                else PFCHK(plans[k].launch_iter(i, nullptr, nullptr));
            }
            plans[k].gather();
            PFCHK(read_status());
            for (int i = 0; i < n; ++i) before[i] = g_batch.hsc[i].iter_done;
            const auto t0 = std::chrono::steady_clock::now();
            for (int i = 0; i < TRIAL; ++i) PFCHK(plans[k].launch_iter(i, nullptr, nullptr));
            plans[k].gather();
            PFCHK(read_status());
            const double secs = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
            double work = 0;
            for (int i = 0; i < n; ++i) work += (double)(g_batch.hsc[i].iter_done - before[i]) * (double)act[i]->g->N;
            t[k] = secs > 0 ? work / secs : 0.0;
            for (int i = 0; i < n; ++i) before[i] = g_batch.hsc[i].iter_done;
        }
        if (next_untried() < 0) {
            // The trial iterations run with every member active, where
            // several policies come within a few percent of each other;
            // whole runs also have phases with few members left, which
            // favour short step-A z-chunks.  Within 1% of the best trial
            // rate (about the trials' noise), the first policy in this
            // order is kept (whole 64-system runs: 7 beats 5 by 3% and 4
            // by 5% in FP64, 8 and 6 lead in mixed precision).
            const int best = (int)(std::max_element(t.begin(), t.end()) - t.begin());
            static const int order[NPOLICY] = {7, 8, 6, 5, 4, 1, 3, 0, 2};
            use = best;
            for (int p : order)
                if (t[p] >= 0.99 * t[best]) { use = p; break; }
            g_batch_policy[key] = use;
            if (getenv("PF_LOG"))
                fprintf(stderr, "[pf] batch of %d: policies 0..8 at %.3g %.3g %.3g %.3g %.3g %.3g %.3g %.3g %.3g "
                                "node-iterations/s over %d iterations each; keeping policy %d\n", n, t[0], t[1], t[2],
                        t[3], t[4], t[5], t[6], t[7], t[8], TRIAL, use);
        } else {   // the run ended before every policy was timed: compare again next time
            trials->clear();
        }
    }
    if (npol > 1 && next_untried() < 0 && use != NPOLICY - 1 && running()) {
        // from the last policy timed to the one kept: two iterations (keeping
        // the chunks' parity), the first with the last policy's counts
        PFCHK(switch_iter(use, NPOLICY - 1, 0));
        PFCHK(plans[use].launch_iter(1, nullptr, nullptr));
        plans[use].gather();
        PFCHK(read_status());
        for (int i = 0; i < n; ++i) before[i] = g_batch.hsc[i].iter_done;
    }
    if (running()) PFCHK(capture(use));
    while (running()) {
        const bool timed = g_timing.enabled && (g_timing.chunk++ % g_timing.sample) == 0;
        hipError_t e = hipSuccess;
        if (timed) {
            while ((int)g_batch.ev.size() < 2 * m) {
                hipEvent_t ev;
                HIPCHK(hipEventCreate(&ev));
                g_batch.ev.push_back(ev);
            }
            for (int i = 0; i < m; ++i)
                PFCHK(plans[use].launch_iter(i, g_batch.ev[2 * i], g_batch.ev[2 * i + 1]));
            plans[use].gather();
            e = hipGetLastError();
        } else {
            e = hipGraphLaunch(plans[use].exec, stream);
        }
        if (e == hipSuccess) e = hipMemcpyAsync(g_batch.hsc, dgather, szS, hipMemcpyDeviceToHost, stream);
        if (e == hipSuccess) e = hipStreamSynchronize(stream);
        if (e != hipSuccess) return fail(PF_ERR_DEVICE, "batched chunk failed: %s", hipGetErrorString(e));
        if (timed) {
            // launch j of the chunk did a member's whole step A while the
            // member still iterated: j <= the iterations it completed here.
            // Every launch of the chunk counts (those after the last member
            // stopped exit at once and add time but no bytes), as in a
            // profiler's mean over all launches of the kernel.
            for (int j = 0; j < m; ++j) {
                double bytes = 0;
                for (int i = 0; i < n; ++i)
                    if (status[i] == pfk::ST_RUN && j <= g_batch.hsc[i].iter_done - before[i]) bytes += abytes[i];
                float ms = 0;
                HIPCHK(hipEventElapsedTime(&ms, g_batch.ev[2 * j], g_batch.ev[2 * j + 1]));
                g_timing.ms[tslot] += ms;
                g_timing.launches[tslot] += 1;
                g_timing.bytes[tslot] += bytes;
            }
        }
        for (int i = 0; i < n; ++i) {
            status[i] = g_batch.hsc[i].stop;
            before[i] = g_batch.hsc[i].iter_done;
        }
    }
    for (int i = 0; i < n; ++i) *act[i]->g->hsc = g_batch.hsc[i];
    return PF_OK;
}

// ------------------------------------------------ batched bookkeeping

// Device tables for the work between a batch's Krylov runs (corrections,
// true residuals, starts), grown on demand; pinned copies of the gathered
// scalar blocks.  Each table is reused only after a stream synchronisation.
struct RoundBuf {
    void *dev = nullptr;
    size_t bytes = 0;
    Scalars *hsc = nullptr;
    int hcap = 0;
} g_round;

struct RoundLayout {
    size_t corr, s64, s32, args, act, pref, na, fin, scp, gather, total;
};

RoundLayout round_layout(int n)
{
    auto al = [](size_t x) { return (x + 255) & ~(size_t)255; };
    RoundLayout L{};
    size_t o = 0;
    L.corr = o; o += al(sizeof(pfk::CorrectMember) * n);
    L.s64 = o; o += al(sizeof(pfk::StartMember<double>) * n);
    L.s32 = o; o += al(sizeof(pfk::StartMember<float>) * n);
    L.args = o; o += al(sizeof(pfk::ZArgs<double>) * n);
    L.act = o; o += al(sizeof(int) * n);
    L.pref = o; o += al(sizeof(int) * (n + 1));
    L.na = o; o += al(sizeof(int));
    L.fin = o; o += al(sizeof(pfk::FinArgs) * n);
    L.scp = o; o += al(sizeof(void *) * n);
    L.gather = o; o += al(sizeof(Scalars) * n);
    L.total = o;
    return L;
}

pf_status round_reserve(int n)
{
    const size_t need = round_layout(n).total;
    if (need > g_round.bytes) {
        if (g_round.dev) (void)hipFree(g_round.dev);
        g_round.dev = nullptr;
        g_round.bytes = 0;
        if (hipMalloc(&g_round.dev, need) != hipSuccess) return fail(PF_ERR_ALLOC, "batch table allocation failed");
        g_round.bytes = need;
    }
    if (n > g_round.hcap) {
        if (g_round.hsc) (void)hipHostFree(g_round.hsc);
        g_round.hsc = nullptr;
        g_round.hcap = 0;
        if (hipHostMalloc((void **)&g_round.hsc, sizeof(Scalars) * n, hipHostMallocDefault) != hipSuccess)
            return fail(PF_ERR_ALLOC, "batch pinned allocation failed");
        g_round.hcap = n;
    }
    return PF_OK;
}

// Launch shape of a member's true residual in a batched launch: 512 threads,
// one node per thread, z-chunks of 16 planes, shared by every member.
ZCfg round_resid_cfg(const pf_grid *g) { return make_cfg(g->nx, g->ny, g->nz, sizeof(double), 512, 1, 16, 1); }

// The batched bookkeeping serves batches whose members all fit that shape
// without the WIDE form and stop on the relative L2 residual (the max-norm
// rule adds a reduction per member).
bool rounds_batchable(const std::vector<LinSolve> &Ls)
{
    const char *e = getenv("PF_BATCH_ROUNDS");   // 0: member by member (for comparisons)
    if (e && e[0] == '0') return false;
    for (const LinSolve &L : Ls) {
        if (L.o->stop_rule == PF_STOP_ABS_INF) return false;
        const ZCfg c = round_resid_cfg(L.g);
        if (c.wide || c.G > L.g->Gmax || c.lds > LDS_MAX) return false;
    }
    return true;
}

// True FP64 residuals of the members in R (as ls_round_residual), their
// reductions into red[0], and every member's scalar block read back into
// its host copy: one launch each and one synchronisation.
pf_status batch_round_residuals(std::vector<LinSolve *> &R, hipStream_t stream)
{
    const int n = (int)R.size();
    PFCHK(round_reserve(n));
    const RoundLayout lay = round_layout(n);
    char *base = (char *)g_round.dev;
    static std::vector<pfk::ZArgs<double>> za;
    static std::vector<int> act, pref;
    static std::vector<pfk::FinArgs> fin;
    static std::vector<const Scalars *> scp;
    za.resize(n);
    act.resize(n);
    pref.assign(n + 1, 0);
    fin.resize(n);
    scp.resize(n);
    ZCfg comb{};
    comb.NTZ = 512; comb.PPT = 1; comb.depth = 1; comb.G = 0; comb.lds = 0; comb.wide = false;
    const bool psi = R[0]->op.psi;
    for (int i = 0; i < n; ++i) {
        const LinSolve &L = *R[i];
        pf_grid *g = L.g;
        const ZCfg c = round_resid_cfg(g);
        pfk::ZArgs<double> a = zbase_cfg<double>(g, L.op, c);
        a.x = g->w64.x;
        a.out = g->w64.r;
        a.b = g->b64;
        a.lift = 0;
        a.dval = L.op.psi ? nullptr : g->dval;
        if (L.mixed) {
            a.rt32 = g->w32.rt;
            a.rs64 = nullptr;
            a.rs32 = g->w32.s;
        } else {
            a.rt32 = g->w64.rt;
            a.rs64 = g->w64.s;
            a.rs32 = nullptr;
        }
        za[i] = a;
        act[i] = i;
        pref[i + 1] = pref[i] + c.G;
        fin[i] = pfk::FinArgs{g->sc, g->partials, c.G, 0};
        scp[i] = g->sc;
        comb.lds = std::max(comb.lds, c.lds);
    }
    comb.G = pref[n];
    const int na = n;
    auto *dargs = (pfk::ZArgs<double> *)(base + lay.args);
    int *dact = (int *)(base + lay.act), *dpref = (int *)(base + lay.pref), *dna = (int *)(base + lay.na);
    auto *dfin = (pfk::FinArgs *)(base + lay.fin);
    const Scalars **dscp = (const Scalars **)(base + lay.scp);
    Scalars *dgather = (Scalars *)(base + lay.gather);
    HIPCHK(hipMemcpyAsync(dargs, za.data(), sizeof(pfk::ZArgs<double>) * n, hipMemcpyHostToDevice, stream));
    HIPCHK(hipMemcpyAsync(dact, act.data(), sizeof(int) * n, hipMemcpyHostToDevice, stream));
    HIPCHK(hipMemcpyAsync(dpref, pref.data(), sizeof(int) * (n + 1), hipMemcpyHostToDevice, stream));
    HIPCHK(hipMemcpyAsync(dna, &na, sizeof(int), hipMemcpyHostToDevice, stream));
    HIPCHK(hipMemcpyAsync(dfin, fin.data(), sizeof(pfk::FinArgs) * n, hipMemcpyHostToDevice, stream));
    HIPCHK(hipMemcpyAsync(dscp, scp.data(), sizeof(void *) * n, hipMemcpyHostToDevice, stream));
    hipError_t e = psi ? launch_batch_k<pfk::OP_RESID, double, true, pfk::SIG_NONE, false, 512, 1, false, 1>(
                             comb, dargs, dact, dpref, dna, stream, nullptr, nullptr)
                       : launch_batch_k<pfk::OP_RESID, double, false, pfk::SIG_NONE, false, 512, 1, false, 1>(
                             comb, dargs, dact, dpref, dna, stream, nullptr, nullptr);
    if (e != hipSuccess) return fail(PF_ERR_DEVICE, "batched residual launch failed: %s", hipGetErrorString(e));
    hipLaunchKernelGGL((pfk::k_finalize_batch<pfk::FIN_SUM>), dim3(n), dim3(256), 0, stream, (const pfk::FinArgs *)dfin);
    HIPCHK(hipGetLastError());
    hipLaunchKernelGGL(pfk::k_gather_scalars, dim3((n + 63) / 64), dim3(64), 0, stream, dscp, dgather, n);
    HIPCHK(hipGetLastError());
    HIPCHK(hipMemcpyAsync(g_round.hsc, dgather, sizeof(Scalars) * n, hipMemcpyDeviceToHost, stream));
    HIPCHK(hipStreamSynchronize(stream));
    for (int i = 0; i < n; ++i) *R[i]->g->hsc = g_round.hsc[i];
    return PF_OK;
}

// After the FP32 runs of the members in M (statuses st): x kept in w64.s and
// the correction added (as ls_after), one launch for all.
pf_status batch_round_correct(const std::vector<LinSolve *> &M, const std::vector<int> &st, hipStream_t stream)
{
    const int n = (int)M.size();
    PFCHK(round_reserve(n));
    const RoundLayout lay = round_layout(n);
    static std::vector<pfk::CorrectMember> cm;
    cm.resize(n);
    size_t nmax = 0;
    for (int i = 0; i < n; ++i) {
        pf_grid *g = M[i]->g;
        cm[i] = pfk::CorrectMember{g->N, g->w64.x, g->w64.s, g->w32.x, g->flags, (int)dirbit(M[i]->op),
                                   st[i] != pfk::ST_NONFINITE ? 1 : 0};
        nmax = std::max(nmax, g->N);
    }
    auto *dcm = (pfk::CorrectMember *)((char *)g_round.dev + lay.corr);
    HIPCHK(hipMemcpyAsync(dcm, cm.data(), sizeof(pfk::CorrectMember) * n, hipMemcpyHostToDevice, stream));
    const int bx = (int)std::min<size_t>(256, (nmax + NT - 1) / NT);
    hipLaunchKernelGGL(pfk::k_correct_batch, dim3(bx, n), dim3(NT), 0, stream, (const pfk::CorrectMember *)dcm);
    HIPCHK(hipGetLastError());
    return PF_OK;
}

// The recorded Krylov starts, one launch per precision.
template <typename T>
pf_status launch_starts(const std::vector<StartRec> &recs, hipStream_t stream, size_t off)
{
    static std::vector<pfk::StartMember<T>> sm;
    sm.clear();
    size_t nmax = 0;
    for (const StartRec &r : recs) {
        if (r.elem != (int)sizeof(T)) continue;
        sm.push_back(pfk::StartMember<T>{r.g->N, (T *)r.p, (T *)r.v, (T *)r.t, (T *)r.xz, r.g->sc, r.init});
        nmax = std::max(nmax, r.g->N);
    }
    if (sm.empty()) return PF_OK;
    auto *dsm = (pfk::StartMember<T> *)((char *)g_round.dev + off);
    HIPCHK(hipMemcpyAsync(dsm, sm.data(), sizeof(pfk::StartMember<T>) * sm.size(), hipMemcpyHostToDevice, stream));
    const int bx = (int)std::min<size_t>(256, (nmax + NT - 1) / NT);
    hipLaunchKernelGGL((pfk::k_krylov_start_batch<T>), dim3(bx, (unsigned)sm.size()), dim3(NT), 0, stream,
                       (const pfk::StartMember<T> *)dsm);
    HIPCHK(hipGetLastError());
    return PF_OK;
}

// Solve several systems (same operator kind and options) as one batch.
// Between Krylov runs, the members' corrections, true residuals and restarts
// run as batched launches on the batch's stream with one status read per
// round (rounds_batchable), else member by member.
pf_status solve_batch(std::vector<LinSolve> &Ls)
{
    const int n = (int)Ls.size();
    if (n == 0) return PF_OK;
    for (auto &L : Ls) PFCHK(ls_init_launch(L));
    for (auto &L : Ls) PFCHK(sync(L.g));
    for (auto &L : Ls) PFCHK(ls_init_decide(L));
    hipStream_t bs = Ls[0].g->stream;
    const bool batched = rounds_batchable(Ls);
    if (batched) PFCHK(round_reserve(n));
    int m = 16;
    for (auto &L : Ls) m = std::max(m, chunk_len(L.g, L.o));
    std::vector<long> members;
    for (auto &L : Ls) members.push_back(((long)L.g->nx * 4096 + L.g->ny) * 4096 + L.g->nz);
    std::sort(members.begin(), members.end());
    std::vector<StartRec> starts;
    for (bool first = true;; first = false) {
        if (!first) {   // the first true residuals came with the init read
            if (batched) {
                std::vector<LinSolve *> R;
                for (auto &L : Ls)
                    if (!L.done) R.push_back(&L);
                if (!R.empty()) PFCHK(batch_round_residuals(R, bs));
            } else {
                for (auto &L : Ls)
                    if (!L.done) PFCHK(ls_round_launch(L));
                for (auto &L : Ls) PFCHK(sync(L.g));
            }
        }
        std::vector<LinSolve *> act;
        starts.clear();
        if (batched) g_defer_start = &starts;
        pf_status dst = PF_OK;
        for (auto &L : Ls) {
            if (L.done) continue;
            bool run = false;
            dst = ls_round_decide(L, &run);
            if (dst != PF_OK) break;
            if (run) act.push_back(&L);
        }
        g_defer_start = nullptr;
        if (dst != PF_OK) return dst;
        if (batched) {
            const RoundLayout lay = round_layout(n);
            PFCHK(launch_starts<double>(starts, bs, lay.s64));
            PFCHK(launch_starts<float>(starts, bs, lay.s32));
        }
        if (act.empty()) break;
        if (!batched)
            for (LinSolve *L : act) PFCHK(sync(L->g));   // Krylov starts written
        // members that fell back to FP64 run apart from those still refining in FP32
        std::vector<LinSolve *> a32, a64;
        for (LinSolve *L : act) (L->mixed ? a32 : a64).push_back(L);
        std::vector<int> st;
        if (!a32.empty()) {
            PFCHK(batch_krylov_run<float>(a32, members, bs, m, st));
            for (size_t i = 0; i < a32.size(); ++i) PFCHK(ls_after(*a32[i], st[i], !batched));
            if (batched) PFCHK(batch_round_correct(a32, st, bs));
        }
        if (!a64.empty()) {
            PFCHK(batch_krylov_run<double>(a64, members, bs, m, st));
            for (size_t i = 0; i < a64.size(); ++i) PFCHK(ls_after(*a64[i], st[i], !batched));
        }
    }
    for (auto &L : Ls) PFCHK(sync(L.g));
    return PF_OK;
}

// Algorithmic bytes of the Jacobi-scaled product: x and the coefficient (full
// or palette index) read, y written, and the FP64 sigma read when given.
double product_bytes(const pf_grid *g, const double *sigma, size_t elem)
{
    const double coef = use_palette(g) ? 1.0 : (double)elem;
    return (2.0 * elem + coef + (sigma ? 8.0 : 0.0)) * (double)g->N;
}

// Account one timed product launch (events p0, p1 already complete).
pf_status timing_add_product(int slot, double bytes)
{
    float ms = 0;
    HIPCHK(hipEventElapsedTime(&ms, g_timing.p0, g_timing.p1));
    g_timing.ms[slot] += ms;
    g_timing.launches[slot] += 1;
    g_timing.bytes[slot] += bytes;
    return PF_OK;
}

// Palette form of the grid's coefficient field: the distinct values of
// |eps| are found one at a time (each pass over the field reports the first
// node whose value is not yet in the palette); with at most PAL_MAX of them
// the field is also stored as one byte per node, and the face coefficient
// 2 e_a e_b / (e_a + e_b) / h^2 of every pair of palette values is tabulated
// (FP64, rounded to FP32 for the FP32 table).  Otherwise npal stays 0 and the
// kernels read the full field.
pf_status build_palette(pf_grid *g)
{
    const size_t N = g->N;
    double *dpal = nullptr;
    unsigned long long *dmiss = nullptr;
    PFCHK(dalloc(g, &dpal, pfk::PAL_MAX));
    PFCHK(dalloc(g, &dmiss, 1));
    std::vector<double> pal(pfk::PAL_MAX, 0.0);
    int npal = 0;
    PFCHK(sync(g));
    for (;;) {
        const unsigned long long none = ~0ull;
        unsigned long long miss = 0;
        HIPCHK(hipMemcpy(dpal, pal.data(), pfk::PAL_MAX * sizeof(double), hipMemcpyHostToDevice));
        HIPCHK(hipMemcpy(dmiss, &none, sizeof none, hipMemcpyHostToDevice));
        hipLaunchKernelGGL(pfk::k_palette_scan, dim3(pw_blocks(N)), dim3(NT), 0, g->stream, N,
                           (const double *)g->eps64, (const double *)dpal, npal, dmiss);
        HIPCHK(hipGetLastError());
        PFCHK(sync(g));
        HIPCHK(hipMemcpy(&miss, dmiss, sizeof miss, hipMemcpyDeviceToHost));
        if (miss == none) break;
        if (npal == pfk::PAL_MAX) return PF_OK;   // too many distinct values: no palette
        double v = 0;
        HIPCHK(hipMemcpy(&v, g->eps64 + miss, sizeof v, hipMemcpyDeviceToHost));
        pal[npal++] = std::fabs(v);
    }
    PFCHK(dalloc(g, &g->epsi, N));
    PFCHK(dalloc(g, &g->ftab64, pfk::FTAB));
    PFCHK(dalloc(g, &g->ftab32, pfk::FTAB));
    std::vector<double> ft(pfk::FTAB, 0.0);
    std::vector<float> ft32(pfk::FTAB, 0.0f);
    const double ih2 = 1.0 / (g->h * g->h);
    for (int a = 0; a < npal; ++a)
        for (int b = 0; b < npal; ++b) {
            ft[a * pfk::PAL_MAX + b] = (2.0 * pal[a] * pal[b]) / (pal[a] + pal[b]) * ih2;
            ft32[a * pfk::PAL_MAX + b] = (float)ft[a * pfk::PAL_MAX + b];
        }
    HIPCHK(hipMemcpy(g->ftab64, ft.data(), pfk::FTAB * sizeof(double), hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(g->ftab32, ft32.data(), pfk::FTAB * sizeof(float), hipMemcpyHostToDevice));
    hipLaunchKernelGGL(pfk::k_palette_index, dim3(pw_blocks(N)), dim3(NT), 0, g->stream, N,
                       (const double *)g->eps64, (const double *)dpal, npal, g->epsi);
    HIPCHK(hipGetLastError());
    PFCHK(sync(g));
    g->npal = npal;
    return PF_OK;
}

pf_status check_grid(const pf_grid *g)
{
    if (!g) return fail(PF_ERR_ARG, "null grid");
    return PF_OK;
}

double secs_since(std::chrono::steady_clock::time_point t0)
{
    return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
}

}  // namespace

// ====================================================================== ABI

extern "C" {

const char *pf_last_error(void) { return g_err.c_str(); }

void pf_lin_opts_default(pf_lin_opts *o)
{
    if (!o) return;
    o->rel_tol = 1e-10;
    o->max_iter = 20000;
    o->precision = PF_FP64;
    o->inner_tol = 1e-2;
    o->max_refine = 30;
    o->check_every = 0;
    o->stop_rule = PF_STOP_REL2;
}

pf_status pf_timing_enable(int32_t enable, int32_t sample)
{
    if (sample <= 0) return fail(PF_ERR_ARG, "sample must be > 0");
    const hipEvent_t p0 = g_timing.p0, p1 = g_timing.p1;
    g_timing = Timing{};
    g_timing.p0 = p0;
    g_timing.p1 = p1;
    g_timing.enabled = enable != 0;
    g_timing.sample = sample;
    if (!g_timing.enabled) return PF_OK;
    if (!g_timing.p0) HIPCHK(hipEventCreate(&g_timing.p0));
    if (!g_timing.p1) HIPCHK(hipEventCreate(&g_timing.p1));
    return PF_OK;
}

pf_status pf_timing_read(int32_t kind, int64_t *launches, double *mean_ms, double *bytes)
{
    if (kind < 0 || kind >= TIMING_SLOTS) return fail(PF_ERR_ARG, "kind must be 0..%d", TIMING_SLOTS - 1);
    const int i = kind;
    if (launches) *launches = g_timing.launches[i];
    if (mean_ms)
        *mean_ms = g_timing.launches[i] ? g_timing.ms[i] / g_timing.launches[i] : 0.0;
    if (bytes) *bytes = g_timing.bytes[i];
    return PF_OK;
}

pf_status pf_set_launch(int32_t strip, int32_t zdepth, int32_t threads, int32_t pipeline)
{
    if (pipeline < 0 || pipeline > 2) return fail(PF_ERR_ARG, "pipeline must be 0, 1 or 2");
    if (threads != 0 && threads != 256 && threads != 512 && threads != 1024)
        return fail(PF_ERR_ARG, "threads must be 0, 256, 512 or 1024");
    const int nt = threads ? threads : 256;
    if (strip != 0 && strip != nt && strip != 2 * nt)
        return fail(PF_ERR_ARG, "strip must be 0, threads or 2*threads");
    if (zdepth < 0) return fail(PF_ERR_ARG, "zdepth must be >= 0");
    g_nt_override = threads ? threads : (strip ? 256 : 0);
    g_ppt_override = strip ? strip / nt : 0;
    g_kz_override = zdepth;
    g_depth_override = pipeline;
    return PF_OK;
}

pf_status pf_grid_create(const pf_grid_desc *d, pf_grid **out)
{
    g_err.clear();
    if (!d || !out) return fail(PF_ERR_ARG, "null descriptor or output");
    *out = nullptr;
    if (d->nx < 3 || d->ny < 3 || d->nz < 3) return fail(PF_ERR_ARG, "nx, ny, nz must be >= 3");
    if (!(d->h > 0.0) || !std::isfinite(d->h)) return fail(PF_ERR_ARG, "h must be finite and > 0");
    if (!d->eps) return fail(PF_ERR_ARG, "eps is required");
    const size_t N = (size_t)d->nx * d->ny * d->nz;
    if (N >= (size_t)1 << 29) return fail(PF_ERR_ARG, "grid too large (N >= 2^29 nodes)");
    int bp = 0, bs = 0;
    for (int f = 0; f < 6; ++f) {
        if (d->bc_phi[f] != PF_BC_DIRICHLET && d->bc_phi[f] != PF_BC_NEUMANN) return fail(PF_ERR_ARG, "bad bc_phi");
        if (d->bc_psi[f] != PF_BC_DIRICHLET && d->bc_psi[f] != PF_BC_NEUMANN) return fail(PF_ERR_ARG, "bad bc_psi");
        if (!std::isfinite(d->bc_value[f])) return fail(PF_ERR_ARG, "bc_value must be finite");
        bp |= (d->bc_phi[f] == PF_BC_NEUMANN) << f;
        bs |= (d->bc_psi[f] == PF_BC_NEUMANN) << f;
    }
    pf_grid *g = new pf_grid();
    if (hipGetDevice(&g->device) != hipSuccess) { delete g; return fail(PF_ERR_DEVICE, "hipGetDevice failed"); }
    g->nx = d->nx; g->ny = d->ny; g->nz = d->nz; g->N = N; g->h = d->h;
    g->bcphi_mask = bp; g->bcpsi_mask = bs;
    for (int f = 0; f < 6; ++f) g->bcval[f] = d->bc_value[f];
    g->ustream = (hipStream_t)d->stream;
    g->c64 = g->cb64 = g->cp64 = default_cfg(d->nx, d->ny, d->nz, 8);
    g->c32 = g->cb32 = g->cp32 = default_cfg(d->nx, d->ny, d->nz, 4);
    if (g->c64.lds > LDS_MAX || g->c32.lds > LDS_MAX) {
        delete g;
        return fail(PF_ERR_ARG, "nx too large for the LDS strip (nx <= ~4800)");
    }
    // partials must cover every launch shape the tuner may pick (KZ >= 1)
    g->Gmax = std::max({(int)(((size_t)d->nx * d->ny + 255) / 256) * d->nz, g->c64.G, g->c32.G, PW_MAX_G});
    auto cleanup = [&](pf_status st) {
        pf_grid_destroy(g);
        return st;
    };
    if (hipStreamCreate(&g->stream) != hipSuccess) { delete g; return fail(PF_ERR_DEVICE, "hipStreamCreate failed"); }
    if (hipEventCreateWithFlags(&g->ev, hipEventDisableTiming) != hipSuccess) return cleanup(fail(PF_ERR_DEVICE, "hipEventCreate failed"));
    pf_status st;
    if ((st = begin(g)) != PF_OK) return cleanup(st);
    if ((st = dalloc(g, &g->eps64, N)) != PF_OK) return cleanup(st);
    if ((st = dalloc(g, &g->flags, N)) != PF_OK) return cleanup(st);
    if ((st = dalloc(g, &g->dval, N)) != PF_OK) return cleanup(st);
    if ((st = dalloc(g, &g->sc, 1)) != PF_OK) return cleanup(st);
    if ((st = dalloc(g, &g->partials, (size_t)g->Gmax * pfk::PSTRIDE)) != PF_OK) return cleanup(st);
    if ((st = dalloc(g, &g->partA, (size_t)g->Gmax * pfk::PSTRIDE)) != PF_OK) return cleanup(st);
    if ((st = dalloc(g, &g->partB, (size_t)g->Gmax * pfk::PSTRIDE)) != PF_OK) return cleanup(st);
    if ((st = dalloc(g, &g->sink, (size_t)pfk::SINK_ELEMS)) != PF_OK) return cleanup(st);
    if (hipHostMalloc((void **)&g->hsc, sizeof(Scalars), hipHostMallocDefault) != hipSuccess)
        return cleanup(fail(PF_ERR_ALLOC, "pinned host allocation failed"));
    if (d->fixed_charge && (st = dalloc(g, &g->q, N)) != PF_OK) return cleanup(st);
    unsigned *bad = nullptr;
    if ((st = dalloc(g, &bad, 1)) != PF_OK) return cleanup(st);
    if (hipMemsetAsync(bad, 0, sizeof(unsigned), g->stream) != hipSuccess ||
        hipMemsetAsync(g->sc, 0, sizeof(Scalars), g->stream) != hipSuccess)
        return cleanup(fail(PF_ERR_DEVICE, "hipMemsetAsync failed"));
    hipLaunchKernelGGL(pfk::k_validate, dim3(pw_blocks(N)), dim3(NT), 0, g->stream, N, d->eps, d->node_type,
                       d->fixed_charge, d->fixed_value, bad);
    if (hipGetLastError() != hipSuccess) return cleanup(fail(PF_ERR_DEVICE, "validate launch failed"));
    unsigned hbad = 0;
    if (hipMemcpyAsync(&hbad, bad, sizeof hbad, hipMemcpyDeviceToHost, g->stream) != hipSuccess ||
        hipStreamSynchronize(g->stream) != hipSuccess)
        return cleanup(fail(PF_ERR_DEVICE, "validation failed (are the field pointers device memory?)"));
    if (hbad & 1u) return cleanup(fail(PF_ERR_ARG, "eps must be finite and > 0 everywhere"));
    if (hbad & 2u) return cleanup(fail(PF_ERR_ARG, "node_type values must be 0, 1 or 2"));
    if (hbad & 4u) return cleanup(fail(PF_ERR_ARG, "fixed_charge must be finite"));
    if (hbad & 8u) return cleanup(fail(PF_ERR_ARG, "fixed_value must be finite"));
    if (hipMemcpyAsync(g->eps64, d->eps, N * sizeof(double), hipMemcpyDefault, g->stream) != hipSuccess)
        return cleanup(fail(PF_ERR_DEVICE, "copy of eps failed"));
    if (g->q && hipMemcpyAsync(g->q, d->fixed_charge, N * sizeof(double), hipMemcpyDefault, g->stream) != hipSuccess)
        return cleanup(fail(PF_ERR_DEVICE, "copy of fixed_charge failed"));
    pfk::Faces fv;
    for (int f = 0; f < 6; ++f) fv.v[f] = d->bc_value[f];
    hipLaunchKernelGGL(pfk::k_classify, dim3(pw_blocks(N)), dim3(NT), 0, g->stream, d->nx, d->ny, d->nz,
                       d->node_type, d->fixed_value, bp, fv, bs, g->flags, g->dval);
    if (hipGetLastError() != hipSuccess) return cleanup(fail(PF_ERR_DEVICE, "classify launch failed"));
    hipLaunchKernelGGL(pfk::k_mark_dirichlet, dim3(pw_blocks(N)), dim3(NT), 0, g->stream, N,
                       (const uint8_t *)g->flags, g->eps64);
    if (hipGetLastError() != hipSuccess) return cleanup(fail(PF_ERR_DEVICE, "Dirichlet mark launch failed"));
    if ((st = build_palette(g)) != PF_OK) return cleanup(st);
    if ((st = sync(g)) != PF_OK) return cleanup(st);
    *out = g;
    return PF_OK;
}

void pf_grid_destroy(pf_grid *g)
{
    if (!g) return;
    if (g->stream) (void)hipStreamSynchronize(g->stream);
    for (auto &kv : g->graphs) (void)hipGraphExecDestroy(kv.second);
    for (hipEvent_t e : g->tev) (void)hipEventDestroy(e);
    for (void *p : g->allocs) (void)hipFree(p);
    if (g->hsc) (void)hipHostFree(g->hsc);
    if (g->ev) (void)hipEventDestroy(g->ev);
    if (g->stream) (void)hipStreamDestroy(g->stream);
    delete g;
}

pf_status pf_linear_solve(pf_grid *g, const double *sigma, const double *b, double *x,
                          const pf_lin_opts *opts, pf_lin_info *info)
{
    auto t0 = std::chrono::steady_clock::now();
    PFCHK(check_grid(g));
    if (!b || !x) return fail(PF_ERR_ARG, "b and x are required");
    pf_lin_opts o;
    if (opts) o = *opts; else pf_lin_opts_default(&o);
    PFCHK(check_opts(&o));
    PFCHK(begin(g));
    PFCHK(ensure_work<double>(g));
    HIPCHK(hipMemcpyAsync(g->b64, b, g->N * sizeof(double), hipMemcpyDefault, g->stream));
    HIPCHK(hipMemcpyAsync(g->w64.x, x, g->N * sizeof(double), hipMemcpyDefault, g->stream));
    OpDesc op;
    op.sigma = sigma;
    pf_lin_info li{};
    pf_status st = solve_internal(g, op, &o, &li);
    if (st == PF_OK || st == PF_ERR_NOCONV) {
        HIPCHK(hipMemcpyAsync(x, g->w64.x, g->N * sizeof(double), hipMemcpyDefault, g->stream));
        PFCHK(sync(g));
    }
    li.seconds = secs_since(t0);
    li.status = st;
    if (info) *info = li;
    return st;
}

pf_status pf_residual(pf_grid *g, const double *sigma, const double *b, const double *x,
                      double *rel_res, double *r)
{
    PFCHK(check_grid(g));
    if (!b || !x || !rel_res) return fail(PF_ERR_ARG, "b, x and rel_res are required");
    PFCHK(begin(g));
    PFCHK(ensure_work<double>(g));
    OpDesc op;
    op.sigma = sigma;
    double *rbuf = r ? r : g->w64.r;
    PFCHK(residual64(g, op, b, nullptr, rbuf, true, nullptr, nullptr, nullptr, 1));
    PFCHK(residual64(g, op, b, x, rbuf, false, nullptr, nullptr, nullptr, 0));
    PFCHK(read_scalars(g));
    const double bn2 = g->hsc->red[1];
    const double rr = g->hsc->red[0];
    *rel_res = bn2 > 0 ? std::sqrt(rr / bn2) : (rr == 0 ? 0.0 : INFINITY);
    return PF_OK;
}

}  // extern "C"

// ------------------------------------------- residual without allocation

// Device scratch of pf_residual_noalloc: a scalar block (its red[] slots
// receive the two sums) followed by the workgroup partials.  One copy per
// device, held until the process ends.  In host code the name stands for a
// host-side symbol, never a device address: host code uses the per-device
// pointer from hipGetSymbolAddress.
static __device__ __align__(256) unsigned char scratch[PF_NOALLOC_SCRATCH_BYTES];

namespace {

constexpr int MAX_DEVICES = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[MAX_DEVICES] = {};

// Device address of `scratch` on device dev, looked up once per device with
// that device current.
pf_status scratch_for(int dev, void **out)
{
    if (dev < 0 || dev >= MAX_DEVICES) return fail(PF_ERR_DEVICE, "device %d out of range", dev);
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        int cur = 0;
        HIPCHK(hipGetDevice(&cur));
        if (cur != dev) HIPCHK(hipSetDevice(dev));
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (cur != dev) (void)hipSetDevice(cur);
        if (e != hipSuccess || !p)
            return fail(PF_ERR_DEVICE, "hipGetSymbolAddress(scratch) failed: %s", hipGetErrorString(e));
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return PF_OK;
}

}  // namespace

extern "C" {

pf_status pf_residual_noalloc(pf_grid *g, const double *sigma, const double *b, const double *x,
                              double *rel_res, double *r)
{
    PFCHK(check_grid(g));
    if (!b || !x || !rel_res || !r) return fail(PF_ERR_ARG, "b, x, rel_res and r are required");
    void *base = nullptr;
    PFCHK(scratch_for(g->device, &base));
    const size_t head = (sizeof(Scalars) + 255) & ~(size_t)255;
    const size_t cap = (PF_NOALLOC_SCRATCH_BYTES - head) / (pfk::PSTRIDE * sizeof(double));
    // pf_residual's launch shape; longer z-chunks only if its partials do not fit
    ZCfg c = cfg_of<double>(g);
    while ((size_t)c.G > cap && c.KZ < g->nz) c = make_cfg(g->nx, g->ny, g->nz, 8, c.NTZ, c.PPT, 2 * c.KZ, 1);
    if ((size_t)c.G > cap)
        return fail(PF_ERR_ARG, "grid needs %d workgroup partials; the scratch holds %zu", c.G, cap);
    Scalars *sc = static_cast<Scalars *>(base);
    double *part = reinterpret_cast<double *>(static_cast<char *>(base) + head);
    PFCHK(begin(g));
    OpDesc op;
    op.sigma = sigma;
    PFCHK(residual64(g, op, b, nullptr, r, true, nullptr, nullptr, nullptr, 1, &c, part, sc));
    PFCHK(residual64(g, op, b, x, r, false, nullptr, nullptr, nullptr, 0, &c, part, sc));
    double red[2] = {0, 0};
    HIPCHK(hipMemcpyAsync(red, sc->red, sizeof red, hipMemcpyDeviceToHost, g->stream));
    PFCHK(sync(g));
    const double rr = red[0], bn2 = red[1];
    *rel_res = bn2 > 0 ? std::sqrt(rr / bn2) : (rr == 0 ? 0.0 : INFINITY);
    return PF_OK;
}

pf_status pf_stream_probe(int32_t kind, int32_t width, int64_t n, double *const *bufs, int32_t sets, int32_t reps,
                          void *stream, double *mean_us)
{
    g_err.clear();
    static const int RW[3][2] = {{1, 1}, {3, 1}, {7, 4}};
    if (kind < 0 || kind > 2) return fail(PF_ERR_ARG, "kind must be 0, 1 or 2");
    if (width != 8 && width != 16) return fail(PF_ERR_ARG, "width must be 8 or 16 bytes");
    if (n <= 0 || sets <= 0 || reps <= 0 || !bufs || !mean_us) return fail(PF_ERR_ARG, "bad probe arguments");
    const int R = RW[kind][0], W = RW[kind][1], V = width / 8;
    if (n % V) return fail(PF_ERR_ARG, "n must be a multiple of %d", V);
    std::vector<pfk::StreamArgs> args(sets);
    for (int s = 0; s < sets; ++s) {
        for (int r = 0; r < R; ++r) args[s].in[r] = bufs[(size_t)s * (R + W) + r];
        for (int w = 0; w < W; ++w) args[s].out[w] = bufs[(size_t)s * (R + W) + R + w];
        args[s].n = (size_t)n;
        for (int j = 0; j < R + W; ++j)
            if (!bufs[(size_t)s * (R + W) + j]) return fail(PF_ERR_ARG, "null buffer");
    }
    const hipStream_t st = (hipStream_t)stream;
    const int G = (int)std::min<int64_t>(16384, std::max<int64_t>(1, (n / V + 255) / 256));
    auto launch = [&](const pfk::StreamArgs &a) {
        switch (kind * 2 + (V - 1)) {
        case 0: hipLaunchKernelGGL((pfk::k_stream<1, 1, 1>), dim3(G), dim3(256), 0, st, a); break;
        case 1: hipLaunchKernelGGL((pfk::k_stream<1, 1, 2>), dim3(G), dim3(256), 0, st, a); break;
        case 2: hipLaunchKernelGGL((pfk::k_stream<3, 1, 1>), dim3(G), dim3(256), 0, st, a); break;
        case 3: hipLaunchKernelGGL((pfk::k_stream<3, 1, 2>), dim3(G), dim3(256), 0, st, a); break;
        case 4: hipLaunchKernelGGL((pfk::k_stream<7, 4, 1>), dim3(G), dim3(256), 0, st, a); break;
        default: hipLaunchKernelGGL((pfk::k_stream<7, 4, 2>), dim3(G), dim3(256), 0, st, a); break;
        }
    };
    hipEvent_t e0, e1;
    HIPCHK(hipEventCreate(&e0));
    HIPCHK(hipEventCreate(&e1));
    for (int s = 0; s < sets; ++s) launch(args[s]);   // untimed first pass
    hipError_t e = hipEventRecord(e0, st);
    for (int k = 0; k < reps && e == hipSuccess; ++k) launch(args[k % sets]);
    if (e == hipSuccess) e = hipGetLastError();
    if (e == hipSuccess) e = hipEventRecord(e1, st);
    if (e == hipSuccess) e = hipEventSynchronize(e1);
    float ms = 0;
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (e != hipSuccess) return fail(PF_ERR_DEVICE, "stream probe failed: %s", hipGetErrorString(e));
    *mean_us = ms * 1e3 / reps;
    return PF_OK;
}

pf_status pf_spmv(pf_grid *g, const double *sigma, const double *x, double *y, int32_t jacobi)
{
    PFCHK(check_grid(g));
    if (!x || !y || x == y) return fail(PF_ERR_ARG, "x and y must be distinct device arrays");
    PFCHK(begin(g));
    PFCHK(ensure_work<double>(g));
    OpDesc op;
    op.sigma = sigma;
    if (jacobi) PFCHK(tune_product<double>(g, op));
    const ZCfg &c = jacobi ? cfgp_ref<double>(g) : cfg_of<double>(g);
    pfk::ZArgs<double> a = zbase_cfg<double>(g, op, c);
    a.x = x;
    a.out = y;
    const bool timed = jacobi && g_timing.enabled;
    hipEvent_t t0 = timed ? g_timing.p0 : nullptr, t1 = timed ? g_timing.p1 : nullptr;
    if (jacobi) PFCHK((zlaunch<pfk::OP_SPMV_JAC, double>(g, op, a, c, t0, t1)));
    else PFCHK((zlaunch<pfk::OP_SPMV, double>(g, op, a, c)));
    PFCHK(sync(g));
    if (timed) PFCHK(timing_add_product(2, product_bytes(g, sigma, sizeof(double))));
    return PF_OK;
}

pf_status pf_spmv_f32(pf_grid *g, const double *sigma, const float *x, float *y, int32_t jacobi)
{
    PFCHK(check_grid(g));
    if (!x || !y || x == y) return fail(PF_ERR_ARG, "x and y must be distinct device arrays");
    if (!jacobi) return fail(PF_ERR_ARG, "pf_spmv_f32 supports jacobi = 1 only");
    PFCHK(begin(g));
    PFCHK(ensure_work<float>(g));
    OpDesc op;
    op.sigma = sigma;
    PFCHK(tune_product<float>(g, op));
    const ZCfg &c = cfgp_ref<float>(g);
    pfk::ZArgs<float> a = zbase_cfg<float>(g, op, c);
    a.x = x;
    a.out = y;
    const bool timed = g_timing.enabled;
    PFCHK((zlaunch<pfk::OP_SPMV_JAC, float>(g, op, a, c, timed ? g_timing.p0 : nullptr,
                                             timed ? g_timing.p1 : nullptr)));
    PFCHK(sync(g));
    if (timed) PFCHK(timing_add_product(3, product_bytes(g, sigma, sizeof(float))));
    return PF_OK;
}

// ------------------------------------------------------------ nonlinear

void pf_pf_params_default(pf_pf_params *p)
{
    if (!p) return;
    std::memset(p, 0, sizeof *p);
    p->steric = 1;
    p->lc = 0.0;
    p->eps_s = 78.45;
    p->kB = 1.38e-23;
    p->T = 298.15;
    p->e = 1.602e-19;
    p->eps0 = 8.85e-14;
    p->NA = 6.02214076e23;
    p->length_unit_A = 1.0;
    p->omega = 0.3;
    p->outer_tol = 1e-8;
    p->max_outer = 5000;
    p->warm_start = 0;
    pf_lin_opts_default(&p->lin);
}

namespace {

// Species table in the units of the grid: lambda = e^2/(eps0 kB T),
// concentrations per cubed length unit, v_i = 4 pi a_i^3 / 3.
pf_status species_dev(const pf_pf_params *p, pfk::SpeciesDev *sp)
{
    if (p->n_species < 1 || p->n_species > pfk::MAXSP) return fail(PF_ERR_ARG, "n_species must be in 1..%d", pfk::MAXSP);
    if (!p->valence || !p->radius || !p->bath_molar) return fail(PF_ERR_ARG, "species arrays are required");
    if (!(p->kB > 0) || !(p->T > 0) || !(p->e > 0) || !(p->eps0 > 0) || !(p->NA > 0) || !(p->length_unit_A > 0))
        return fail(PF_ERR_ARG, "physical constants must be > 0");
    const double L = p->length_unit_A;
    const double lam = p->e * p->e / (p->eps0 * 100.0 * p->kB * p->T) * 1e10 / L;
    const double per_molar = p->NA * 1e3 * 1e-30 * L * L * L;
    std::memset(sp, 0, sizeof *sp);
    sp->nsp = p->n_species;
    sp->steric = p->steric ? 1 : 0;
    sp->lam = lam;
    double vsum = 0, occ = 0;
    double v[pfk::MAXSP];
    for (int i = 0; i < p->n_species; ++i) {
        const double a = p->radius[i] / L, c = p->bath_molar[i] * per_molar;
        if (!(a > 0) || !(c > 0) || !std::isfinite(p->valence[i])) return fail(PF_ERR_ARG, "species %d: radius and bath must be > 0", i);
        v[i] = 4.0 * M_PI * a * a * a / 3.0;
        vsum += v[i];
        occ += v[i] * c;
        sp->z[i] = p->valence[i];
        sp->lncb[i] = std::log(c);
        sp->lnvcb[i] = std::log(v[i] * c);
    }
    const double v0 = vsum / p->n_species;
    for (int i = 0; i < p->n_species; ++i) sp->p[i] = v[i] / v0;
    if (sp->steric) {
        if (!(occ < 1.0)) return fail(PF_ERR_ARG, "bath volume fraction must be < 1 (Gamma_B > 0)");
        sp->lnGB = std::log(1.0 - occ);
    }
    return PF_OK;
}

pf_status check_pf(const pf_pf_params *p)
{
    if (!p) return fail(PF_ERR_ARG, "null parameters");
    if (!(p->omega >= 0.0 && p->omega < 1.0)) return fail(PF_ERR_ARG, "omega must be in [0, 1)");
    if (!(p->outer_tol > 0)) return fail(PF_ERR_ARG, "outer_tol must be > 0");
    if (p->max_outer <= 0) return fail(PF_ERR_ARG, "max_outer must be > 0");
    if (!(p->lc >= 0) || !std::isfinite(p->lc)) return fail(PF_ERR_ARG, "lc must be >= 0");
    if (!(p->eps_s > 0)) return fail(PF_ERR_ARG, "eps_s must be > 0");
    return check_opts(&p->lin);
}

pf_status ensure_nl(pf_grid *g)
{
    if (g->phi0) return PF_OK;
    for (double **p : {&g->phi0, &g->phi, &g->psi, &g->rhs1, &g->sig, &g->rhs2, &g->src})
        PFCHK(dalloc(g, p, g->N));
    return PF_OK;
}

}  // namespace

pf_status pf_fermi(pf_grid *g, const pf_pf_params *p, const double *phi, double *rho_hat, double *sigma,
                   double *conc, double *steric)
{
    PFCHK(check_grid(g));
    if (!p || !phi) return fail(PF_ERR_ARG, "params and phi are required");
    pfk::SpeciesDev sp;
    PFCHK(species_dev(p, &sp));
    PFCHK(begin(g));
    hipLaunchKernelGGL(pfk::k_fermi, dim3(pw_blocks(g->N)), dim3(NT), 0, g->stream, g->N, phi,
                       (const uint8_t *)g->flags, sp, nullptr, rho_hat, sigma, conc, steric);
    HIPCHK(hipGetLastError());
    return sync(g);
}

}  // extern "C"

namespace {

// One nonlinear problem of a (possibly batched) Table 2 / Table 4 run.
struct NlSys {
    pf_grid *g = nullptr;
    const pf_pf_params *p = nullptr;
    pfk::SpeciesDev sp{};
    double *phi_out = nullptr, *conc = nullptr, *steric = nullptr;
    int it = 0, lin_iters = 0;
    double delta = INFINITY;
    pf_status st = PF_OK;
    bool done = false;
    bool pre = false;   // the last relaxation launch already did the next iteration's point-wise steps
    std::chrono::steady_clock::time_point t0;
};

// Linear solves of one phase of the outer loop: system i solves ops[i] with
// right-hand side bs[i] and initial guess / result xs[i] (grid buffers).
// Batched phases run every member's Krylov iterations in shared launches.
pf_status nl_linear_phase(std::vector<NlSys *> &sys, const std::vector<OpDesc> &ops,
                          const std::vector<const double *> &bs, const std::vector<const double *> &x0s,
                          const std::vector<double *> &xs, bool batched)
{
    const size_t n = sys.size();
    for (size_t i = 0; i < n; ++i) {   // right-hand side and initial guess into the grid's solve buffers
        pf_grid *g = sys[i]->g;
        hipLaunchKernelGGL(pfk::k_copy2, dim3(pw_blocks(g->N)), dim3(NT), 0, g->stream, g->N, g->b64, bs[i], g->w64.x,
                           x0s[i]);
        HIPCHK(hipGetLastError());
    }
    bool same_prec = true;
    for (size_t i = 1; i < n; ++i) same_prec &= sys[i]->p->lin.precision == sys[0]->p->lin.precision;
    std::vector<pf_lin_info> li(n);
    std::vector<pf_status> st(n, PF_OK);
    if (batched && n > 1 && same_prec) {
        std::vector<LinSolve> Ls(n);
        for (size_t i = 0; i < n; ++i) {
            Ls[i].g = sys[i]->g;
            Ls[i].op = ops[i];
            Ls[i].o = &sys[i]->p->lin;
        }
        PFCHK(solve_batch(Ls));
        for (size_t i = 0; i < n; ++i) st[i] = ls_finish(Ls[i], &li[i]);
    } else {
        for (size_t i = 0; i < n; ++i) {
            st[i] = solve_internal(sys[i]->g, ops[i], &sys[i]->p->lin, &li[i]);
            if (st[i] == PF_ERR_DEVICE || st[i] == PF_ERR_ALLOC || st[i] == PF_ERR_ARG) return st[i];
        }
    }
    for (size_t i = 0; i < n; ++i) {
        pf_grid *g = sys[i]->g;
        sys[i]->lin_iters += li[i].iters;
        if (st[i] != PF_OK) {
            sys[i]->st = st[i];
            sys[i]->done = true;
            continue;
        }
        HIPCHK(hipMemcpyAsync(xs[i], g->w64.x, g->N * sizeof(double), hipMemcpyDeviceToDevice, g->stream));
    }
    return PF_OK;
}

// Table 2 (sequential algorithm) with the device-resident steps of Table 4:
//   step 2   PF2 with rho' = Psi = 0 (fixed charges only), unless warm-started;
//   step 3   Fermi update at Phi_0 (Eq. (1)) and PF1 (Eq. (12), (14));
//   step 4   PF2 (Eq. (13)) warm-started from Phi_0;
//   step 5   Phi := omega Phi_0 + (1 - omega) Phi, stop on the max norm.
// From the second outer iteration on, step 5's kernel also does step 3's
// Fermi update (and, for the local PF1, Psi and the PF2 right-hand side) at
// the relaxed Phi_0, so the point-wise work of an outer iteration is one pass.
pf_status nl_drive(std::vector<NlSys> &S, bool batched)
{
    for (auto &s : S) {
        pf_grid *g = s.g;
        PFCHK(begin(g));
        PFCHK(ensure_work<double>(g));
        PFCHK(ensure_nl(g));
        const int B = pw_blocks(g->N);
        const double h3 = g->h * g->h * g->h;
        hipLaunchKernelGGL(pfk::k_source, dim3(B), dim3(NT), 0, g->stream, g->N, (const double *)g->q,
                           s.sp.lam / h3, s.p->rhs_extra, g->src);
        HIPCHK(hipGetLastError());
        if (!s.p->warm_start) {
            PFCHK(fill<double>(g, g->phi0, 0.0, g->N));
        } else {
            HIPCHK(hipMemcpyAsync(g->phi0, s.phi_out, g->N * sizeof(double), hipMemcpyDefault, g->stream));
            hipLaunchKernelGGL(pfk::k_set_dirichlet, dim3(B), dim3(NT), 0, g->stream, g->N, g->phi0,
                               (const uint8_t *)g->flags, (uint8_t)pfk::F_DIR_PHI, (const double *)g->dval);
            HIPCHK(hipGetLastError());
        }
        PFCHK(fill<double>(g, g->psi, 0.0, g->N));
    }
    {   // step 2
        std::vector<NlSys *> cold;
        std::vector<OpDesc> ops;
        std::vector<const double *> bs, x0s;
        std::vector<double *> xs;
        for (auto &s : S) {
            if (s.p->warm_start) continue;
            cold.push_back(&s);
            ops.push_back(OpDesc{});
            bs.push_back(s.g->src);
            x0s.push_back(s.g->phi0);
            xs.push_back(s.g->phi0);
        }
        if (!cold.empty()) PFCHK(nl_linear_phase(cold, ops, bs, x0s, xs, batched));
    }
    for (;;) {
        std::vector<NlSys *> act;
        for (auto &s : S)
            if (!s.done && s.it < s.p->max_outer) act.push_back(&s);
        if (act.empty()) break;
        // Fermi update at Phi_0: rhs1 = -rho_hat, sig = -rho_hat'  (Eq. (1), (11))
        for (NlSys *s : act) {
            pf_grid *g = s->g;
            ++s->it;
            if (s->pre) continue;
            hipLaunchKernelGGL(pfk::k_fermi, dim3(pw_blocks(g->N)), dim3(NT), 0, g->stream, g->N,
                               (const double *)g->phi0, (const uint8_t *)g->flags, s->sp, g->rhs1, (double *)nullptr,
                               g->sig, (double *)nullptr, (double *)nullptr);
            HIPCHK(hipGetLastError());
        }
        // PF1
        {
            std::vector<NlSys *> pf1;
            std::vector<OpDesc> ops;
            std::vector<const double *> bs, x0s;
            std::vector<double *> xs;
            for (NlSys *s : act) {
                pf_grid *g = s->g;
                if (s->p->lc > 0) {
                    OpDesc op;
                    op.psi = true;
                    op.ceps = s->p->eps_s * s->p->lc * s->p->lc;
                    op.sig_const = s->p->eps_s;
                    pf1.push_back(s);
                    ops.push_back(op);
                    bs.push_back(g->rhs1);
                    x0s.push_back(g->psi);
                    xs.push_back(g->psi);
                } else if (!s->pre) {
                    hipLaunchKernelGGL(pfk::k_psi_local, dim3(pw_blocks(g->N)), dim3(NT), 0, g->stream, g->N,
                                       (const double *)g->rhs1, (const uint8_t *)g->flags, 1.0 / s->p->eps_s, g->psi);
                    HIPCHK(hipGetLastError());
                }
            }
            if (!pf1.empty()) PFCHK(nl_linear_phase(pf1, ops, bs, x0s, xs, batched));
        }
        // PF2
        {
            std::vector<NlSys *> pf2;
            std::vector<OpDesc> ops;
            std::vector<const double *> bs, x0s;
            std::vector<double *> xs;
            for (NlSys *s : act) {
                if (s->done) continue;
                pf_grid *g = s->g;
                if (!s->pre || s->p->lc > 0) {   // else written by the relaxation kernel
                    hipLaunchKernelGGL(pfk::k_rhs_pf2, dim3(pw_blocks(g->N)), dim3(NT), 0, g->stream, g->N,
                                       (const double *)g->psi, (const double *)g->sig, (const double *)g->phi0,
                                       (const double *)g->src, s->p->eps_s, g->rhs2);
                    HIPCHK(hipGetLastError());
                }
                OpDesc op;
                op.sigma = g->sig;
                pf2.push_back(s);
                ops.push_back(op);
                bs.push_back(g->rhs2);
                x0s.push_back(g->phi0);   // warm start from Phi_0; the solution goes to phi
                xs.push_back(g->phi);
            }
            if (!pf2.empty()) PFCHK(nl_linear_phase(pf2, ops, bs, x0s, xs, batched));
        }
        // relaxation and max-norm test (Table 2 step 5)
        for (NlSys *s : act) {
            if (s->done) continue;
            pf_grid *g = s->g;
            const int B = pw_blocks(g->N);
            const bool local = !(s->p->lc > 0);
            hipLaunchKernelGGL((pfk::k_relax_fermi<NT>), dim3(B), dim3(NT), 0, g->stream, g->N, g->phi0, g->phi,
                               s->p->omega, g->partials, (const uint8_t *)g->flags, s->sp,
                               local ? nullptr : g->rhs1, g->sig, (const double *)g->src, s->p->eps_s,
                               1.0 / s->p->eps_s, local ? g->rhs2 : nullptr);
            HIPCHK(hipGetLastError());
            s->pre = true;
            PFCHK(finalize<pfk::FIN_MAX>(g, B));
            HIPCHK(hipMemcpyAsync(g->hsc, g->sc, sizeof(Scalars), hipMemcpyDeviceToHost, g->stream));
        }
        for (NlSys *s : act) {
            if (s->done) continue;
            PFCHK(sync(s->g));
            s->delta = s->g->hsc->red[0];
            if (!std::isfinite(s->delta)) { s->st = PF_ERR_NONFINITE; s->done = true; }
            else if (s->delta <= s->p->outer_tol) s->done = true;
        }
    }
    for (auto &s : S) {
        pf_grid *g = s.g;
        if (s.st == PF_OK && !(s.delta <= s.p->outer_tol)) s.st = PF_ERR_NOCONV;
        HIPCHK(hipMemcpyAsync(s.phi_out, g->phi0, g->N * sizeof(double), hipMemcpyDefault, g->stream));
        if (s.conc || s.steric) {
            hipLaunchKernelGGL(pfk::k_fermi, dim3(pw_blocks(g->N)), dim3(NT), 0, g->stream, g->N,
                               (const double *)g->phi0, (const uint8_t *)g->flags, s.sp, (double *)nullptr,
                               (double *)nullptr, (double *)nullptr, s.conc, s.steric);
            HIPCHK(hipGetLastError());
        }
    }
    for (auto &s : S) PFCHK(sync(s.g));
    return PF_OK;
}

void nl_info(const NlSys &s, pf_nl_info *info)
{
    if (!info) return;
    info->outer_iters = s.it;
    info->total_lin_iters = s.lin_iters;
    info->last_delta = s.delta;
    info->seconds = secs_since(s.t0);
    info->status = s.st;
}

pf_status nl_status_message(const NlSys &s)
{
    if (s.st == PF_ERR_NOCONV)
        return fail(s.st, "outer loop: delta %.3e after %d iterations", s.delta, s.it);
    if (s.st == PF_ERR_NONFINITE) return fail(s.st, "non-finite value in the outer loop");
    return s.st;
}

}  // namespace

extern "C" {

pf_status pf_nonlinear_solve(pf_grid *g, const pf_pf_params *p, double *phi, double *conc, double *steric,
                             pf_nl_info *info)
{
    g_err.clear();
    PFCHK(check_grid(g));
    if (!phi) return fail(PF_ERR_ARG, "phi is required");
    PFCHK(check_pf(p));
    std::vector<NlSys> S(1);
    S[0].t0 = std::chrono::steady_clock::now();
    S[0].g = g;
    S[0].p = p;
    S[0].phi_out = phi;
    S[0].conc = conc;
    S[0].steric = steric;
    PFCHK(species_dev(p, &S[0].sp));
    PFCHK(nl_drive(S, false));
    nl_info(S[0], info);
    return nl_status_message(S[0]);
}

pf_status pf_linear_solve_batch(int32_t n, pf_grid *const *g, const double *const *sigma,
                                const double *const *b, double *const *x, const pf_lin_opts *opts,
                                pf_lin_info *info)
{
    auto t0 = std::chrono::steady_clock::now();
    g_err.clear();
    if (n < 0 || (n > 0 && (!g || !b || !x))) return fail(PF_ERR_ARG, "bad batch arguments");
    pf_lin_opts o;
    if (opts) o = *opts; else pf_lin_opts_default(&o);
    PFCHK(check_opts(&o));
    for (int i = 0; i < n; ++i) {
        if (!g[i] || !b[i] || !x[i]) return fail(PF_ERR_ARG, "batch member %d: null grid, b or x", i);
        for (int j = 0; j < i; ++j)
            if (g[j] == g[i]) return fail(PF_ERR_ARG, "batch members %d and %d share a grid", j, i);
    }
    std::vector<LinSolve> Ls(n);
    for (int i = 0; i < n; ++i) {
        PFCHK(begin(g[i]));
        PFCHK(ensure_work<double>(g[i]));
        HIPCHK(hipMemcpyAsync(g[i]->b64, b[i], g[i]->N * sizeof(double), hipMemcpyDefault, g[i]->stream));
        HIPCHK(hipMemcpyAsync(g[i]->w64.x, x[i], g[i]->N * sizeof(double), hipMemcpyDefault, g[i]->stream));
        Ls[i].g = g[i];
        Ls[i].op.sigma = sigma ? sigma[i] : nullptr;
        Ls[i].o = &o;
    }
    PFCHK(solve_batch(Ls));
    pf_status worst = PF_OK;
    std::string first_err;
    for (int i = 0; i < n; ++i) {
        pf_lin_info li{};
        pf_status st = ls_finish(Ls[i], &li);
        if (st != PF_OK && worst == PF_OK) { worst = st; first_err = g_err; }
        if (st == PF_OK || st == PF_ERR_NOCONV)
            HIPCHK(hipMemcpyAsync(x[i], g[i]->w64.x, g[i]->N * sizeof(double), hipMemcpyDefault, g[i]->stream));
        li.status = st;
        if (info) info[i] = li;
    }
    for (int i = 0; i < n; ++i) PFCHK(sync(g[i]));
    const double secs = secs_since(t0);
    if (info)
        for (int i = 0; i < n; ++i) info[i].seconds = secs;
    g_err = first_err;
    return worst;
}

pf_status pf_nonlinear_solve_batch(int32_t n, pf_grid *const *g, const pf_pf_params *const *p,
                                   double *const *phi, pf_nl_info *info)
{
    g_err.clear();
    if (n < 0 || (n > 0 && (!g || !p || !phi))) return fail(PF_ERR_ARG, "bad batch arguments");
    std::vector<NlSys> S(n);
    for (int i = 0; i < n; ++i) {
        if (!g[i] || !phi[i]) return fail(PF_ERR_ARG, "batch member %d: null grid or phi", i);
        for (int j = 0; j < i; ++j)
            if (g[j] == g[i]) return fail(PF_ERR_ARG, "batch members %d and %d share a grid", j, i);
        PFCHK(check_pf(p[i]));
        S[i].t0 = std::chrono::steady_clock::now();
        S[i].g = g[i];
        S[i].p = p[i];
        S[i].phi_out = phi[i];
        PFCHK(species_dev(p[i], &S[i].sp));
    }
    PFCHK(nl_drive(S, true));
    pf_status worst = PF_OK;
    std::string first_err;
    for (int i = 0; i < n; ++i) {
        nl_info(S[i], info ? &info[i] : nullptr);
        pf_status st = nl_status_message(S[i]);
        if (st != PF_OK && worst == PF_OK) { worst = st; first_err = g_err; }
    }
    g_err = first_err;
    return worst;
}

}  // extern "C"

// ------------------------------------------- singular-charge decomposition

namespace {

// Device buffers of one interface setup, released on every exit path.
struct IfTemp {
    std::vector<void *> ptrs;
    ~IfTemp()
    {
        for (void *q : ptrs) (void)hipFree(q);
    }
    template <typename T>
    pf_status alloc(T **p, size_t n)
    {
        void *q = nullptr;
        if (hipMalloc(&q, std::max<size_t>(n, 1) * sizeof(T)) != hipSuccess) {
            (void)hipGetLastError();
            return fail(PF_ERR_ALLOC, "hipMalloc of %zu bytes failed", n * sizeof(T));
        }
        ptrs.push_back(q);
        *p = static_cast<T *>(q);
        return PF_OK;
    }
};

struct GridGuard {
    pf_grid *g = nullptr;
    ~GridGuard() { pf_grid_destroy(g); }
};

pf_status check_iface(const pf_iface_params *p)
{
    if (!p) return fail(PF_ERR_ARG, "null interface parameters");
    if (p->n_charges < 0 || (p->n_charges > 0 && !p->charges))
        return fail(PF_ERR_ARG, "n_charges must be >= 0 with a charge array");
    if (!(p->eps_m > 0) || !(p->eps_s > 0) || !std::isfinite(p->eps_m) || !std::isfinite(p->eps_s))
        return fail(PF_ERR_ARG, "eps_m and eps_s must be finite and > 0");
    if (!std::isfinite(p->lambda)) return fail(PF_ERR_ARG, "lambda must be finite");
    return PF_OK;
}

}  // namespace

extern "C" {

void pf_iface_params_default(pf_iface_params *p)
{
    if (!p) return;
    std::memset(p, 0, sizeof *p);
    p->eps_m = 2.0;
    p->eps_s = 78.45;
    pf_lin_opts_default(&p->lin);
    p->lin.rel_tol = 1e-12;
}

pf_status pf_coulomb(const double *pts, const int8_t *dir, int64_t n, const double *charges, int32_t M,
                     double scale, double *out, void *stream)
{
    g_err.clear();
    if (n < 0 || M < 0 || (n > 0 && (!pts || !out)) || (M > 0 && !charges))
        return fail(PF_ERR_ARG, "pf_coulomb: bad sizes or null arrays");
    if (n == 0) return PF_OK;
    hipStream_t s = static_cast<hipStream_t>(stream);
    const size_t blocks = ((size_t)n + pfk::IF_NT - 1) / pfk::IF_NT;
    if (blocks > 0x7fffffffu) return fail(PF_ERR_ARG, "pf_coulomb: too many points");
    hipLaunchKernelGGL(pfk::k_coulomb_points, dim3((unsigned)blocks), dim3(pfk::IF_NT), 0, s, (size_t)n, pts, dir,
                       charges, (int)M, scale, out);
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(s));
    return PF_OK;
}

pf_status pf_interface_setup(pf_grid *g, const pf_iface_params *p, double *b_if, double *phi_reg, double *phi_lap,
                             pf_lin_info *lap_info)
{
    PFCHK(check_grid(g));
    PFCHK(check_iface(p));
    if (!b_if) return fail(PF_ERR_ARG, "b_if must be a device array of N doubles");
    PFCHK(begin(g));
    const size_t N = g->N;
    const double h = g->h;
    const double scale = p->lambda / (4.0 * 3.14159265358979323846 * p->eps_m);
    IfTemp tmp;
    unsigned *bad = nullptr;
    PFCHK(tmp.alloc(&bad, 1));
    // hipMemsetAsync is fine here: this sequence is never captured in a graph
    HIPCHK(hipMemsetAsync(bad, 0, sizeof(unsigned), g->stream));
    hipLaunchKernelGGL(pfk::k_if_check, dim3(pw_blocks(N)), dim3(NT), 0, g->stream, N, (const uint8_t *)g->flags,
                       (const double *)g->eps64, p->eps_m, p->eps_s, bad);
    HIPCHK(hipGetLastError());
    unsigned hbad = 0;
    HIPCHK(hipMemcpyAsync(&hbad, bad, sizeof hbad, hipMemcpyDeviceToHost, g->stream));
    PFCHK(sync(g));
    if (hbad) return fail(PF_ERR_ARG, "eps must equal eps_m on SOLUTE nodes and eps_s on all other nodes");

    // evaluation list: masks, workgroup counts, prefix sums, entries
    pfk::IfGrid ig{g->nx, g->ny, g->nz, h, g->flags, phi_reg ? 1 : 0};
    const size_t nb = (N + pfk::IF_NT - 1) / pfk::IF_NT;
    uint16_t *mask = nullptr;
    unsigned *blk = nullptr, *off = nullptr;
    PFCHK(tmp.alloc(&mask, N));
    PFCHK(tmp.alloc(&blk, nb + 1));
    PFCHK(tmp.alloc(&off, N));
    hipLaunchKernelGGL(pfk::k_if_mask, dim3((unsigned)nb), dim3(pfk::IF_NT), 0, g->stream, ig, N, mask, blk);
    HIPCHK(hipGetLastError());
    hipLaunchKernelGGL(pfk::k_if_scan, dim3(1), dim3(1024), 0, g->stream, blk, (int)nb);
    HIPCHK(hipGetLastError());
    unsigned E = 0;   // at most 7 per node (six directions, one node value), below 2^32 for N < 2^29
    HIPCHK(hipMemcpyAsync(&E, blk + nb, sizeof E, hipMemcpyDeviceToHost, g->stream));
    PFCHK(sync(g));
    unsigned long long *code = nullptr;
    double *V = nullptr, *D = nullptr;
    PFCHK(tmp.alloc(&code, E));
    PFCHK(tmp.alloc(&V, E));
    PFCHK(tmp.alloc(&D, E));
    hipLaunchKernelGGL(pfk::k_if_list, dim3((unsigned)nb), dim3(pfk::IF_NT), 0, g->stream, N,
                       (const uint16_t *)mask, (const unsigned *)blk, off, code);
    HIPCHK(hipGetLastError());
    if (E > 0) {
        hipLaunchKernelGGL(pfk::k_coulomb_entries, dim3((E + pfk::IF_NT - 1) / pfk::IF_NT), dim3(pfk::IF_NT), 0,
                           g->stream, (size_t)E, (const unsigned long long *)code, g->nx, g->ny, h, p->charges,
                           (int)p->n_charges, scale, V, D);
        HIPCHK(hipGetLastError());
    }

    // Laplace problem (its own grid: unit coefficient, the potential's face kinds)
    double *eps1 = nullptr, *fv = nullptr, *sig = nullptr, *rhs = nullptr, *xl = nullptr;
    uint8_t *type = nullptr;
    PFCHK(tmp.alloc(&eps1, N));
    PFCHK(tmp.alloc(&type, N));
    PFCHK(tmp.alloc(&fv, N));
    PFCHK(tmp.alloc(&sig, N));
    PFCHK(tmp.alloc(&rhs, N));
    PFCHK(tmp.alloc(&xl, N));
    hipLaunchKernelGGL(pfk::k_if_laplace, dim3(pw_blocks(N)), dim3(NT), 0, g->stream, ig, N, (const uint16_t *)mask,
                       (const unsigned *)off, (const double *)V, (const double *)D, eps1, type, fv, sig, rhs);
    HIPCHK(hipGetLastError());
    PFCHK(fill<double>(g, xl, 0.0, N));
    PFCHK(sync(g));
    pf_grid_desc ld{};
    ld.nx = g->nx;
    ld.ny = g->ny;
    ld.nz = g->nz;
    ld.h = h;
    ld.eps = eps1;
    ld.node_type = type;
    ld.fixed_value = fv;
    for (int f = 0; f < 6; ++f) {
        ld.bc_phi[f] = ((g->bcphi_mask >> f) & 1) ? PF_BC_NEUMANN : PF_BC_DIRICHLET;
        ld.bc_value[f] = 0.0;
        ld.bc_psi[f] = PF_BC_DIRICHLET;
    }
    GridGuard gl;
    PFCHK(pf_grid_create(&ld, &gl.g));
    pf_lin_info li{};
    const pf_status lst = pf_linear_solve(gl.g, sig, rhs, xl, &p->lin, &li);
    if (lap_info) *lap_info = li;
    if (lst != PF_OK) return lst;
    g_err.clear();

    // flux jumps and SMIB terms; phi* + phi^L on Omega_m
    hipLaunchKernelGGL(pfk::k_if_rhs, dim3(pw_blocks(N)), dim3(NT), 0, g->stream, ig, N, (const uint16_t *)mask,
                       (const unsigned *)off, (const double *)V, (const double *)D, (const double *)xl, p->eps_m,
                       p->eps_s, b_if, phi_reg);
    HIPCHK(hipGetLastError());
    if (phi_lap) HIPCHK(hipMemcpyAsync(phi_lap, xl, N * sizeof(double), hipMemcpyDeviceToDevice, g->stream));
    HIPCHK(hipMemsetAsync(bad, 0, sizeof(unsigned), g->stream));
    hipLaunchKernelGGL(pfk::k_if_finite, dim3(pw_blocks(N)), dim3(NT), 0, g->stream, N, (const double *)b_if,
                       (const double *)phi_reg, bad);
    HIPCHK(hipGetLastError());
    HIPCHK(hipMemcpyAsync(&hbad, bad, sizeof hbad, hipMemcpyDeviceToHost, g->stream));
    PFCHK(sync(g));
    if (hbad) return fail(PF_ERR_NONFINITE, "interface terms are not finite (a charge on an evaluation point?)");
    return PF_OK;
}

}  // extern "C"

// ------------------------------------------- filter-region atomic model

namespace {

pf_status check_sites(const pf_site_params *s, std::vector<pfk::SiteRec> &rec)
{
    if (!s) return fail(PF_ERR_ARG, "null site parameters");
    if (s->n_sites < 1 || s->n_sites > pfk::MAX_SITES) return fail(PF_ERR_ARG, "n_sites must be in 1..%d", pfk::MAX_SITES);
    if (!s->site_xyz || !s->site_radius || !s->site_valence || !s->occupied)
        return fail(PF_ERR_ARG, "site arrays are required");
    if (s->n_atoms < 0 || (s->n_atoms > 0 && !s->atoms)) return fail(PF_ERR_ARG, "n_atoms must be >= 0 with an atom array");
    if (!(s->eps_p > 0) || !(s->eps_b > 0) || !(s->V_sites > 0)) return fail(PF_ERR_ARG, "eps_p, eps_b and V_sites must be > 0");
    rec.resize(s->n_sites);
    for (int b = 0; b < s->n_sites; ++b) {
        const double *c = s->site_xyz + 3 * b;
        if (!(s->site_radius[b] > 0) || !(s->site_valence[b] != 0) || !std::isfinite(s->site_valence[b]) ||
            (s->occupied[b] != 0 && s->occupied[b] != 1) || !std::isfinite(c[0] + c[1] + c[2]))
            return fail(PF_ERR_ARG, "site %d: radius > 0, valence != 0, occupancy 0/1 and a finite centre required", b);
        rec[b] = pfk::SiteRec{c[0], c[1], c[2], s->site_radius[b], s->site_valence[b], (double)s->occupied[b]};
    }
    return PF_OK;
}

}  // namespace

extern "C" {

pf_status pf_site_model(const pf_pf_params *pp, const pf_site_params *s, double *phi_b, double *S_b, double *psi_b,
                        double *conc_b, void *stream)
{
    g_err.clear();
    std::vector<pfk::SiteRec> rec;
    PFCHK(check_sites(s, rec));
    if (!pp) return fail(PF_ERR_ARG, "null species parameters");
    if (!phi_b || !S_b || !psi_b) return fail(PF_ERR_ARG, "phi_b, S_b and psi_b are required");
    pfk::SpeciesDev sp;
    PFCHK(species_dev(pp, &sp));
    double filled = 0;
    for (const auto &r : rec)
        if (r.occ != 0) filled += 4.0 * M_PI * r.a * r.a * r.a / 3.0;
    if (sp.steric && !(filled < s->V_sites))
        return fail(PF_ERR_ARG, "occupied site volume %.6g must stay below V_sites %.6g", filled, s->V_sites);
    hipStream_t st = static_cast<hipStream_t>(stream);
    const int n = s->n_sites, w = 3 + sp.nsp;
    IfTemp tmp;
    pfk::SiteRec *dsite = nullptr;
    double *dout = nullptr;
    PFCHK(tmp.alloc(&dsite, (size_t)n));
    PFCHK(tmp.alloc(&dout, (size_t)n * w));
    HIPCHK(hipMemcpyAsync(dsite, rec.data(), n * sizeof(pfk::SiteRec), hipMemcpyHostToDevice, st));
    pfk::SiteArgs a{dsite, n, s->atoms, s->n_atoms, s->eps_p, s->eps_b, s->V_sites, sp.lam / (4.0 * M_PI), sp, dout};
    hipLaunchKernelGGL(pfk::k_site_model, dim3(n), dim3(pfk::SITE_NT), 0, st, a);
    HIPCHK(hipGetLastError());
    std::vector<double> h((size_t)n * w);
    HIPCHK(hipMemcpyAsync(h.data(), dout, h.size() * sizeof(double), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    for (int b = 0; b < n; ++b) {
        phi_b[b] = h[(size_t)b * w];
        S_b[b] = h[(size_t)b * w + 1];
        psi_b[b] = h[(size_t)b * w + 2];
        if (conc_b)
            for (int i = 0; i < sp.nsp; ++i) conc_b[(size_t)b * sp.nsp + i] = h[(size_t)b * w + 3 + i];
    }
    return PF_OK;
}

pf_status pf_site_fill(int32_t nx, int32_t ny, int32_t nz, double h, const pf_site_params *s, const double *phi_b,
                       uint8_t *node_type, double *fixed_value, int64_t *marked, void *stream)
{
    g_err.clear();
    std::vector<pfk::SiteRec> rec;
    PFCHK(check_sites(s, rec));
    if (nx < 3 || ny < 3 || nz < 3 || !(h > 0) || !std::isfinite(h)) return fail(PF_ERR_ARG, "bad grid shape or spacing");
    if ((double)nx * ny * nz >= (double)(1u << 29)) return fail(PF_ERR_ARG, "grid too large (N must be < 2^29)");
    if (!phi_b || !node_type || !fixed_value) return fail(PF_ERR_ARG, "phi_b, node_type and fixed_value are required");
    for (int b = 0; b < s->n_sites; ++b)
        if (!std::isfinite(phi_b[b])) return fail(PF_ERR_ARG, "phi_b[%d] is not finite", b);
    hipStream_t st = static_cast<hipStream_t>(stream);
    const size_t N = (size_t)nx * ny * nz;
    IfTemp tmp;
    pfk::SiteRec *dsite = nullptr;
    double *dphi = nullptr;
    unsigned long long *dcount = nullptr;
    PFCHK(tmp.alloc(&dsite, (size_t)s->n_sites));
    PFCHK(tmp.alloc(&dphi, (size_t)s->n_sites));
    PFCHK(tmp.alloc(&dcount, 1));
    HIPCHK(hipMemcpyAsync(dsite, rec.data(), s->n_sites * sizeof(pfk::SiteRec), hipMemcpyHostToDevice, st));
    HIPCHK(hipMemcpyAsync(dphi, phi_b, s->n_sites * sizeof(double), hipMemcpyHostToDevice, st));
    HIPCHK(hipMemsetAsync(dcount, 0, sizeof(unsigned long long), st));
    hipLaunchKernelGGL(pfk::k_site_fill, dim3(pw_blocks(N)), dim3(256), 0, st, nx, ny, nz, h,
                       (const pfk::SiteRec *)dsite, (const double *)dphi, (int)s->n_sites, node_type, fixed_value,
                       dcount);
    HIPCHK(hipGetLastError());
    unsigned long long c = 0;
    HIPCHK(hipMemcpyAsync(&c, dcount, sizeof c, hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    if (marked) *marked = (int64_t)c;
    return PF_OK;
}

}  // extern "C"
