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
#include "../../include/pf.h"

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <string>
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
int g_nt_override = 0, g_ppt_override = 0, g_kz_override = 0;

// step-A kernel timing (pf_timing_enable / pf_timing_read)
struct Timing {
    bool enabled = false;
    int sample = 8;
    long chunk = 0;
    long long launches[2] = {0, 0};
    double ms[2] = {0, 0}, bytes[2] = {0, 0};
} g_timing;

constexpr size_t LDS_MAX = 152 * 1024;   // dynamic LDS per workgroup (gfx950 has 160 KB; static arrays use the rest)

// Launch shape of the z-marching stencil kernels: NTZ threads per
// workgroup, PPT nodes per thread (strip S = NTZ*PPT), KZ planes per
// workgroup.
struct ZCfg {
    int NTZ = 256, PPT = 2, S = 512, KZ = 8, nstrips = 1, nzc = 1, G = 1, lmax = 0;
    size_t lds = 0;
};

ZCfg make_cfg(int nx, int ny, int nz, size_t elem, int ntz, int ppt, int kz)
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
    c.lds = 4 * (size_t)c.lmax * elem;   // two planes of (value, coefficient)
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
    return c;
}

int pw_blocks(size_t N) { return (int)std::min<size_t>(PW_MAX_G, (N + NT - 1) / NT); }

template <typename T>
struct Work {
    T *x = nullptr, *r = nullptr, *rt = nullptr, *p[2] = {nullptr, nullptr},
      *v[2] = {nullptr, nullptr}, *s = nullptr, *t = nullptr;
};

}  // namespace

struct pf_grid {
    int nx = 0, ny = 0, nz = 0;
    size_t N = 0;
    double h = 0;
    hipStream_t stream = nullptr;      // internal blocking stream
    hipStream_t ustream = nullptr;     // caller's stream (ordering only)
    hipEvent_t ev = nullptr;
    int bcphi_mask = 0, bcpsi_mask = 0;
    double bcval[6] = {0, 0, 0, 0, 0, 0};
    std::vector<void *> allocs;

    double *eps64 = nullptr;
    float *eps32 = nullptr;
    uint8_t *flags = nullptr;
    double *dval = nullptr;
    double *q = nullptr;               // fixed charge (may stay null)

    ZCfg c64, c32;
    int Gmax = 1;

    // linear solver state
    double *dinv64 = nullptr, *dinv64_psi = nullptr;
    float *dinv32 = nullptr, *dinv32_psi = nullptr;
    double *b64 = nullptr;
    Work<double> w64;
    Work<float> w32;
    bool have64 = false, have32 = false;
    Scalars *sc = nullptr, *hsc = nullptr;
    double *partials = nullptr;
    unsigned *ticket = nullptr;
    std::map<long, hipGraphExec_t> graphs;
    std::vector<hipEvent_t> tev;       // timing events (2 per iteration of a chunk)
    bool last_timed = false;

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
        PFCHK(dalloc(g, &g->dinv64, g->N));
        PFCHK(dalloc(g, &g->dinv64_psi, g->N));
        PFCHK(dalloc(g, &g->b64, g->N));
        for (double **p : {&w.x, &w.r, &w.rt, &w.p[0], &w.p[1], &w.v[0], &w.v[1], &w.s, &w.t})
            PFCHK(dalloc(g, p, g->N));
        g->have64 = true;
        PFCHK(tune<double>(g));
    } else {
        if (g->have32) return PF_OK;
        PFCHK(ensure_work<double>(g));
        Work<float> &w = g->w32;
        PFCHK(dalloc(g, &g->eps32, g->N));
        PFCHK(dalloc(g, &g->dinv32, g->N));
        PFCHK(dalloc(g, &g->dinv32_psi, g->N));
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

template <int OP, typename T, bool CEPS, int NTZ, int PPT>
hipError_t launch_zk(const ZCfg &c, const pfk::ZArgs<T> &a, hipStream_t s)
{
    auto kern = pfk::k_zmarch<OP, T, CEPS, NTZ, PPT>;
    if (c.lds > 64 * 1024) {
        static size_t granted = 0;   // per instantiation
        if (c.lds > granted) {
            hipError_t e = hipFuncSetAttribute((const void *)kern, hipFuncAttributeMaxDynamicSharedMemorySize,
                                               (int)c.lds);
            if (e != hipSuccess) return e;
            granted = c.lds;
        }
    }
    hipLaunchKernelGGL(kern, dim3(c.G), dim3(NTZ), c.lds, s, a);
    return hipGetLastError();
}

template <int OP, typename T, bool CEPS>
hipError_t launch_z(const ZCfg &c, const pfk::ZArgs<T> &a, hipStream_t s)
{
    const int key = c.NTZ * 10 + c.PPT;
    switch (key) {
    case 2561: return launch_zk<OP, T, CEPS, 256, 1>(c, a, s);
    case 2562: return launch_zk<OP, T, CEPS, 256, 2>(c, a, s);
    case 5121: return launch_zk<OP, T, CEPS, 512, 1>(c, a, s);
    case 5122: return launch_zk<OP, T, CEPS, 512, 2>(c, a, s);
    case 10241: return launch_zk<OP, T, CEPS, 1024, 1>(c, a, s);
    case 10242: return launch_zk<OP, T, CEPS, 1024, 2>(c, a, s);
    default: return hipErrorInvalidValue;
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

// Operator description: which system (potential or PF1 density), constant
// coefficient or not, diagonal shift.
struct OpDesc {
    bool psi = false;          // PF1 system (flags bit F_DIR_PSI), constant coefficient
    double ceps = 0;           // PF1 face coefficient eps_s lc^2 (before / h^2)
    const double *sigma = nullptr;
    double sig_const = 0;
};

uint8_t dirbit(const OpDesc &op) { return op.psi ? pfk::F_DIR_PSI : pfk::F_DIR_PHI; }

template <typename T>
pfk::ZArgs<T> zbase(pf_grid *g, const OpDesc &op, const T *dinv)
{
    const ZCfg &c = cfg_of<T>(g);
    pfk::ZArgs<T> a{};
    a.nx = g->nx; a.ny = g->ny; a.nz = g->nz; a.P = g->nx * g->ny;
    a.S = c.S; a.KZ = c.KZ; a.nstrips = c.nstrips; a.G = c.G; a.lmax = c.lmax;
    const double ih2 = 1.0 / (g->h * g->h);
    a.ih2 = (T)ih2;
    a.ceps = (T)(op.ceps * ih2);
    if constexpr (sizeof(T) == 8) a.eps = g->eps64;
    else a.eps = g->eps32;
    a.dinv = dinv;
    a.sigma = op.sigma;
    a.sig_const = op.sig_const;
    a.dval = g->dval;
    a.sc = g->sc;
    a.partials = g->partials;
    a.ticket = g->ticket;
    return a;
}

template <int OP, typename T>
pf_status zlaunch(pf_grid *g, const OpDesc &op, const pfk::ZArgs<T> &a)
{
    const ZCfg &c = cfg_of<T>(g);
    hipError_t e = op.psi ? launch_z<OP, T, true>(c, a, g->stream) : launch_z<OP, T, false>(c, a, g->stream);
    if (e != hipSuccess) return fail(PF_ERR_DEVICE, "stencil kernel launch failed: %s", hipGetErrorString(e));
    return PF_OK;
}

template <typename T>
pf_status compute_dinv(pf_grid *g, const OpDesc &op, T *dinv)
{
    const double ih2 = 1.0 / (g->h * g->h);
    if (op.psi)
        hipLaunchKernelGGL((pfk::k_dinv<T, true>), dim3(pw_blocks(g->N)), dim3(NT), 0, g->stream, g->nx,
                           g->ny, g->nz, ih2, op.ceps * ih2, (const double *)g->eps64, op.sigma,
                           op.sig_const, (const uint8_t *)g->flags, dirbit(op), dinv);
    else
        hipLaunchKernelGGL((pfk::k_dinv<T, false>), dim3(pw_blocks(g->N)), dim3(NT), 0, g->stream, g->nx,
                           g->ny, g->nz, ih2, op.ceps * ih2, (const double *)g->eps64, op.sigma,
                           op.sig_const, (const uint8_t *)g->flags, dirbit(op), dinv);
    HIPCHK(hipGetLastError());
    return PF_OK;
}

// True FP64 residual r = b - A x (and ||r||^2 into sc->red[0]); optional
// shadow / FP32 copies.  lift: use the Dirichlet values as x (b_lift).
pf_status residual64(pf_grid *g, const OpDesc &op, const double *dinv, const double *b,
                     const double *x, double *r, bool lift, double *rt64, float *r32, float *rt32)
{
    pfk::ZArgs<double> a = zbase<double>(g, op, dinv);
    a.x = x;
    a.out = r;
    a.b = b;
    a.lift = lift ? 1 : 0;
    a.dval = op.psi ? nullptr : g->dval;
    a.rt64 = rt64;
    a.r32 = r32;
    a.rt32 = rt32;
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
    return zlaunch<pfk::OP_RESID, double>(g, op, a);
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

// One BiCGSTAB iteration: stencil step A (p, v), stencil step B (s, t),
// pointwise step C (x, r).  parity selects the p/v ping-pong buffers.
template <typename T>
pf_status iteration(pf_grid *g, const OpDesc &op, const T *dinv, Work<T> &w, int parity,
                    hipEvent_t e0 = nullptr, hipEvent_t e1 = nullptr)
{
    pfk::ZArgs<T> a = zbase<T>(g, op, dinv);
    a.x = w.r;
    a.y0 = w.p[parity];
    a.y1 = w.v[parity];
    a.rt = w.rt;
    a.out = w.v[parity ^ 1];
    a.out_aux = w.p[parity ^ 1];
    if (e0) HIPCHK(hipEventRecord(e0, g->stream));
    PFCHK((zlaunch<pfk::OP_BA, T>(g, op, a)));
    if (e1) HIPCHK(hipEventRecord(e1, g->stream));
    pfk::ZArgs<T> b = zbase<T>(g, op, dinv);
    b.x = w.r;
    b.y0 = w.v[parity ^ 1];
    b.out = w.t;
    b.out_aux = w.s;
    PFCHK((zlaunch<pfk::OP_BB, T>(g, op, b)));
    const int G = pw_blocks(g->N);
    hipLaunchKernelGGL((pfk::k_bicg_c<T, NT>), dim3(G), dim3(NT), 0, g->stream, g->N, w.x, w.r,
                       (const T *)w.p[parity ^ 1], (const T *)w.s, (const T *)w.t, dinv,
                       (const T *)w.rt, g->sc, g->partials, g->ticket, G);
    HIPCHK(hipGetLastError());
    return PF_OK;
}

// Chunk of m iterations (m even) captured once per (precision, system) and
// replayed.  The graph references only grid-owned buffers.
template <typename T>
pf_status run_chunk(pf_grid *g, const OpDesc &op, const T *dinv, Work<T> &w, int m)
{
    const bool timed = g_timing.enabled && (g_timing.chunk++ % g_timing.sample) == 0;
    g->last_timed = timed;
    if (timed && (int)g->tev.size() < 2 * m) {
        while ((int)g->tev.size() < 2 * m) {
            hipEvent_t e;
            HIPCHK(hipEventCreate(&e));
            g->tev.push_back(e);
        }
    }
    if (timed) {
        // sampled chunk: direct launches with HIP events around step A
        for (int i = 0; i < m; ++i) PFCHK(iteration<T>(g, op, dinv, w, i & 1, g->tev[2 * i], g->tev[2 * i + 1]));
        return PF_OK;
    }
    const long key = (long)m * 16 + (sizeof(T) == 8 ? 0 : 2) + (op.psi ? 1 : 0);
    auto it = g->graphs.find(key);
    if (it == g->graphs.end()) {
        hipGraph_t graph;
        HIPCHK(hipStreamBeginCapture(g->stream, hipStreamCaptureModeRelaxed));
        pf_status st = PF_OK;
        for (int i = 0; i < m && st == PF_OK; ++i) st = iteration<T>(g, op, dinv, w, i & 1);
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

// Launch shapes chosen per (grid shape, precision) for this process.
std::map<std::tuple<int, int, int, int>, ZCfg> g_tuned;

bool tuning_enabled()
{
    const char *e = getenv("PF_TUNE");
    if (e && e[0] == '0') return false;
    return !g_nt_override && !g_ppt_override && !g_kz_override;
}

// Time the BiCGSTAB step-A kernel (the kernel with the most traffic per
// iteration) for each candidate shape on this grid and keep the fastest.
// Runs once per grid shape and precision; the grid's workspace holds
// synthetic vectors meanwhile (every solve reinitialises it).
template <typename T>
pf_status tune(pf_grid *g)
{
    if (!tuning_enabled()) return PF_OK;
    const auto key = std::make_tuple(g->nx, g->ny, g->nz, (int)sizeof(T));
    auto found = g_tuned.find(key);
    if (found != g_tuned.end()) {
        cfg_ref<T>(g) = found->second;
        return PF_OK;
    }
    Work<T> &w = [&]() -> Work<T> & {
        if constexpr (sizeof(T) == 8) return g->w64;
        else return g->w32;
    }();
    T *dinv = nullptr;
    if constexpr (sizeof(T) == 8) dinv = g->dinv64;
    else dinv = g->dinv32;
    PFCHK(fill<T>(g, w.r, T(1), g->N));
    PFCHK(fill<T>(g, w.rt, T(1), g->N));
    PFCHK(fill<T>(g, w.p[0], T(0), g->N));
    PFCHK(fill<T>(g, w.v[0], T(0), g->N));
    PFCHK(fill<T>(g, dinv, T(0.1), g->N));
    Scalars &h = *g->hsc;
    h = Scalars{};
    h.rho = 1.0; h.alpha = 1.0; h.omega = 1.0; h.beta = 0.5; h.status = pfk::ST_RUN;
    hipEvent_t e0, e1;
    HIPCHK(hipEventCreate(&e0));
    HIPCHK(hipEventCreate(&e1));
    const ZCfg saved = cfg_ref<T>(g);
    ZCfg best = saved;
    float best_ms = 1e30f;
    const int shapes[6][2] = {{256, 1}, {256, 2}, {512, 1}, {512, 2}, {1024, 1}, {1024, 2}};
    OpDesc op;
    pf_status st = PF_OK;
    for (auto &sh : shapes) {
        for (int kz : {2, 4, 8, 16, 32}) {
            ZCfg c = make_cfg(g->nx, g->ny, g->nz, sizeof(T), sh[0], sh[1], kz);
            if (c.lds > LDS_MAX || c.G > g->Gmax || kz > g->nz) continue;
            cfg_ref<T>(g) = c;
            pfk::ZArgs<T> a = zbase<T>(g, op, dinv);
            a.x = w.r; a.y0 = w.p[0]; a.y1 = w.v[0]; a.rt = w.rt;
            a.out = w.v[1]; a.out_aux = w.p[1];
            float tot = 0;
            for (int rep = 0; rep < 4 && st == PF_OK; ++rep) {
                if ((st = write_scalars(g)) != PF_OK) break;
                if (hipEventRecord(e0, g->stream) != hipSuccess) { st = fail(PF_ERR_DEVICE, "event record failed"); break; }
                if (zlaunch<pfk::OP_BA, T>(g, op, a) != PF_OK) {
                    // shape not launchable here: skip it
                    (void)hipGetLastError();
                    g_err.clear();
                    tot = 1e30f;
                    break;
                }
                if (hipEventRecord(e1, g->stream) != hipSuccess || hipEventSynchronize(e1) != hipSuccess) {
                    st = fail(PF_ERR_DEVICE, "event timing failed");
                    break;
                }
                float ms = 0;
                (void)hipEventElapsedTime(&ms, e0, e1);
                if (rep > 0) tot += ms;
            }
            if (st != PF_OK) break;
            if (tot < best_ms) { best_ms = tot; best = c; }
        }
        if (st != PF_OK) break;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    cfg_ref<T>(g) = (st == PF_OK) ? best : saved;
    if (st != PF_OK) return st;
    g_tuned[key] = best;
    if (getenv("PF_LOG"))
        fprintf(stderr, "[pf] tuned %dx%dx%d %s: threads %d, strip %d, z-planes %d, step A %.1f us\n", g->nx, g->ny,
                g->nz, sizeof(T) == 8 ? "fp64" : "fp32", best.NTZ, best.S, best.KZ, best_ms / 3 * 1e3);
    return PF_OK;
}

int chunk_len(const pf_grid *g, const pf_lin_opts *o)
{
    int m = o->check_every > 0 ? o->check_every : (g->N < 200000 ? 32 : 16);
    m = std::max(2, m + (m & 1));
    return m;
}

// Reset the Krylov state from a residual already in w.r / w.rt with
// ||r||^2 = rr.  Keeps the cumulative iteration count.
template <typename T>
pf_status krylov_start(pf_grid *g, Work<T> &w, double rr, double tol2, int iter, int maxit)
{
    PFCHK(fill<T>(g, w.p[0], T(0), g->N));
    PFCHK(fill<T>(g, w.v[0], T(0), g->N));
    Scalars &h = *g->hsc;
    h = Scalars{};
    h.rho = rr;
    h.alpha = 1.0;
    h.omega = 1.0;
    h.beta = 0.0;
    h.rr = rr;
    h.tol2 = tol2;
    h.rt2 = rr;
    h.iter = iter;
    h.maxit = maxit;
    h.status = pfk::ST_RUN;
    return write_scalars(g);
}

// Iterate until the device reports a state other than RUN.
template <typename T>
pf_status krylov_run(pf_grid *g, const OpDesc &op, const T *dinv, Work<T> &w, int m, int *status)
{
    for (;;) {
        const int before = g->hsc->iter;
        PFCHK(run_chunk<T>(g, op, dinv, w, m));
        PFCHK(read_scalars(g));
        if (g->last_timed && !op.psi) {
            // iterations whose step A ran in full (later ones exit at once)
            const int ran = std::min(m, g->hsc->iter - before);
            const int pi = sizeof(T) == 8 ? 0 : 1;
            for (int i = 0; i < ran; ++i) {
                float ms = 0;
                HIPCHK(hipEventElapsedTime(&ms, g->tev[2 * i], g->tev[2 * i + 1]));
                g_timing.ms[pi] += ms;
                g_timing.launches[pi] += 1;
                g_timing.bytes[pi] += 8.0 * (double)g->N * sizeof(T);
            }
        }
        if (g->hsc->status != pfk::ST_RUN) {
            *status = g->hsc->status;
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
    return PF_OK;
}

// The linear solve on grid-owned buffers: g->b64 holds b, g->w64.x the
// initial guess; on return g->w64.x holds the solution.
pf_status solve_internal(pf_grid *g, const OpDesc &op, const pf_lin_opts *o, pf_lin_info *info)
{
    PFCHK(check_opts(o));
    PFCHK(ensure_work<double>(g));
    if (o->precision == PF_MIXED) PFCHK(ensure_work<float>(g));
    const uint8_t db = dirbit(op);
    Work<double> &w = g->w64;
    double *dinv = op.psi ? g->dinv64_psi : g->dinv64;
    PFCHK(compute_dinv<double>(g, op, dinv));
    hipLaunchKernelGGL(pfk::k_set_dirichlet, dim3(pw_blocks(g->N)), dim3(NT), 0, g->stream, g->N, w.x,
                       (const uint8_t *)g->flags, db, op.psi ? nullptr : (const double *)g->dval);
    HIPCHK(hipGetLastError());
    // ||b_lift||
    PFCHK(residual64(g, op, dinv, g->b64, nullptr, w.r, true, nullptr, nullptr, nullptr));
    PFCHK(read_scalars(g));
    const double bnorm = std::sqrt(g->hsc->red[0]);
    pf_lin_info li{};
    li.status = PF_OK;
    if (!std::isfinite(bnorm)) {
        li.status = PF_ERR_NONFINITE;
        if (info) *info = li;
        return fail(PF_ERR_NONFINITE, "right-hand side is not finite");
    }
    if (bnorm == 0.0) {
        // homogeneous problem: x = Dirichlet values, 0 on free rows
        PFCHK(fill<double>(g, w.x, 0.0, g->N));
        hipLaunchKernelGGL(pfk::k_set_dirichlet, dim3(pw_blocks(g->N)), dim3(NT), 0, g->stream, g->N, w.x,
                           (const uint8_t *)g->flags, db, op.psi ? nullptr : (const double *)g->dval);
        HIPCHK(hipGetLastError());
        if (info) *info = li;
        return PF_OK;
    }
    const double tol2 = o->rel_tol * o->rel_tol * bnorm * bnorm;
    const int m = chunk_len(g, o);
    int iter = 0, restarts = 0, refinements = 0;
    pf_status result = PF_OK;
    double rr = 0;

    if (o->precision == PF_FP64) {
        bool started = false;
        for (;;) {
            // true residual; also the shadow residual of a (re)start
            PFCHK(residual64(g, op, dinv, g->b64, w.x, w.r, false, w.rt, nullptr, nullptr));
            PFCHK(read_scalars(g));
            rr = g->hsc->red[0];
            if (!std::isfinite(rr)) { result = PF_ERR_NONFINITE; break; }
            if (rr <= tol2) break;
            if (iter >= o->max_iter) { result = PF_ERR_NOCONV; break; }
            if (started) ++restarts;
            if (restarts > 1000) { result = PF_ERR_BREAKDOWN; break; }
            started = true;
            PFCHK(krylov_start<double>(g, w, rr, tol2, iter, o->max_iter));
            int st = 0;
            PFCHK(krylov_run<double>(g, op, dinv, w, m, &st));
            iter = g->hsc->iter;
            if (st == pfk::ST_NONFINITE) { result = PF_ERR_NONFINITE; break; }
            // ST_CONV, ST_MAXIT and ST_RESTART all go back to the true residual
        }
    } else {
        // Mixed precision: FP64 residual -> FP32 BiCGSTAB correction -> FP64 update.
        Work<float> &v = g->w32;
        float *dinv32 = op.psi ? g->dinv32_psi : g->dinv32;
        PFCHK(compute_dinv<float>(g, op, dinv32));
        const double itol2 = o->inner_tol * o->inner_tol;
        for (;;) {
            PFCHK(residual64(g, op, dinv, g->b64, w.x, w.r, false, nullptr, v.r, v.rt));
            PFCHK(read_scalars(g));
            rr = g->hsc->red[0];
            if (!std::isfinite(rr)) { result = PF_ERR_NONFINITE; break; }
            if (rr <= tol2) break;
            if (refinements >= o->max_refine || iter >= o->max_iter) { result = PF_ERR_NOCONV; break; }
            ++refinements;
            PFCHK(fill<float>(g, v.x, 0.0f, g->N));
            PFCHK(krylov_start<float>(g, v, rr, std::max(itol2 * rr, tol2), iter, o->max_iter));
            int st = 0;
            PFCHK(krylov_run<float>(g, op, dinv32, v, m, &st));
            iter = g->hsc->iter;
            if (st == pfk::ST_NONFINITE) { result = PF_ERR_NONFINITE; break; }
            if (st == pfk::ST_RESTART) ++restarts;
            hipLaunchKernelGGL(pfk::k_correct, dim3(pw_blocks(g->N)), dim3(NT), 0, g->stream, g->N, w.x,
                               (const float *)v.x, (const uint8_t *)g->flags, db);
            HIPCHK(hipGetLastError());
        }
    }
    li.iters = iter;
    li.refinements = refinements;
    li.restarts = restarts;
    li.rel_res = std::sqrt(rr) / bnorm;
    li.status = result;
    if (info) *info = li;
    if (result == PF_ERR_NOCONV) return fail(result, "no convergence: rel_res %.3e after %d iterations", li.rel_res, iter);
    if (result == PF_ERR_NONFINITE) return fail(result, "non-finite value in the iteration");
    if (result == PF_ERR_BREAKDOWN) return fail(result, "repeated BiCGSTAB breakdown");
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
    o->inner_tol = 1e-5;
    o->max_refine = 30;
    o->check_every = 0;
}

pf_status pf_timing_enable(int32_t enable, int32_t sample)
{
    if (sample <= 0) return fail(PF_ERR_ARG, "sample must be > 0");
    g_timing = Timing{};
    g_timing.enabled = enable != 0;
    g_timing.sample = sample;
    return PF_OK;
}

pf_status pf_timing_read(int32_t precision, int64_t *launches, double *mean_ms, double *bytes)
{
    if (precision != PF_FP64 && precision != PF_MIXED) return fail(PF_ERR_ARG, "unknown precision");
    const int i = precision == PF_FP64 ? 0 : 1;
    if (launches) *launches = g_timing.launches[i];
    if (mean_ms) *mean_ms = g_timing.launches[i] ? g_timing.ms[i] / g_timing.launches[i] : 0.0;
    if (bytes) *bytes = g_timing.bytes[i];
    return PF_OK;
}

pf_status pf_set_launch(int32_t strip, int32_t zdepth, int32_t threads)
{
    if (threads != 0 && threads != 256 && threads != 512 && threads != 1024)
        return fail(PF_ERR_ARG, "threads must be 0, 256, 512 or 1024");
    const int nt = threads ? threads : 256;
    if (strip != 0 && strip != nt && strip != 2 * nt)
        return fail(PF_ERR_ARG, "strip must be 0, threads or 2*threads");
    if (zdepth < 0) return fail(PF_ERR_ARG, "zdepth must be >= 0");
    g_nt_override = threads ? threads : (strip ? 256 : 0);
    g_ppt_override = strip ? strip / nt : 0;
    g_kz_override = zdepth;
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
    if (N > (size_t)1 << 31) return fail(PF_ERR_ARG, "grid too large (N > 2^31)");
    int bp = 0, bs = 0;
    for (int f = 0; f < 6; ++f) {
        if (d->bc_phi[f] != PF_BC_DIRICHLET && d->bc_phi[f] != PF_BC_NEUMANN) return fail(PF_ERR_ARG, "bad bc_phi");
        if (d->bc_psi[f] != PF_BC_DIRICHLET && d->bc_psi[f] != PF_BC_NEUMANN) return fail(PF_ERR_ARG, "bad bc_psi");
        if (!std::isfinite(d->bc_value[f])) return fail(PF_ERR_ARG, "bc_value must be finite");
        bp |= (d->bc_phi[f] == PF_BC_NEUMANN) << f;
        bs |= (d->bc_psi[f] == PF_BC_NEUMANN) << f;
    }
    pf_grid *g = new pf_grid();
    g->nx = d->nx; g->ny = d->ny; g->nz = d->nz; g->N = N; g->h = d->h;
    g->bcphi_mask = bp; g->bcpsi_mask = bs;
    for (int f = 0; f < 6; ++f) g->bcval[f] = d->bc_value[f];
    g->ustream = (hipStream_t)d->stream;
    g->c64 = default_cfg(d->nx, d->ny, d->nz, 8);
    g->c32 = default_cfg(d->nx, d->ny, d->nz, 4);
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
    if ((st = dalloc(g, &g->partials, (size_t)g->Gmax * 4)) != PF_OK) return cleanup(st);
    if ((st = dalloc(g, &g->ticket, 1)) != PF_OK) return cleanup(st);
    if (hipHostMalloc((void **)&g->hsc, sizeof(Scalars), hipHostMallocDefault) != hipSuccess)
        return cleanup(fail(PF_ERR_ALLOC, "pinned host allocation failed"));
    if (d->fixed_charge && (st = dalloc(g, &g->q, N)) != PF_OK) return cleanup(st);
    unsigned *bad = nullptr;
    if ((st = dalloc(g, &bad, 1)) != PF_OK) return cleanup(st);
    if (hipMemsetAsync(bad, 0, sizeof(unsigned), g->stream) != hipSuccess ||
        hipMemsetAsync(g->ticket, 0, sizeof(unsigned), g->stream) != hipSuccess ||
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
    PFCHK(compute_dinv<double>(g, op, g->dinv64));
    double *rbuf = r ? r : g->w64.r;
    PFCHK(residual64(g, op, g->dinv64, b, nullptr, rbuf, true, nullptr, nullptr, nullptr));
    PFCHK(read_scalars(g));
    const double bn2 = g->hsc->red[0];
    PFCHK(residual64(g, op, g->dinv64, b, x, rbuf, false, nullptr, nullptr, nullptr));
    PFCHK(read_scalars(g));
    const double rr = g->hsc->red[0];
    *rel_res = bn2 > 0 ? std::sqrt(rr / bn2) : (rr == 0 ? 0.0 : INFINITY);
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
    PFCHK(compute_dinv<double>(g, op, g->dinv64));
    pfk::ZArgs<double> a = zbase<double>(g, op, g->dinv64);
    a.x = x;
    a.out = y;
    if (jacobi) PFCHK((zlaunch<pfk::OP_SPMV_JAC, double>(g, op, a)));
    else PFCHK((zlaunch<pfk::OP_SPMV, double>(g, op, a)));
    return sync(g);
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
    PFCHK(compute_dinv<float>(g, op, g->dinv32));
    pfk::ZArgs<float> a = zbase<float>(g, op, g->dinv32);
    a.x = x;
    a.out = y;
    PFCHK((zlaunch<pfk::OP_SPMV_JAC, float>(g, op, a)));
    return sync(g);
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

// Linear solve on grid buffers: b in src_b, initial guess / result in xio.
pf_status nl_solve(pf_grid *g, const OpDesc &op, const double *src_b, double *xio, const pf_lin_opts *o,
                   int *iters)
{
    HIPCHK(hipMemcpyAsync(g->b64, src_b, g->N * sizeof(double), hipMemcpyDeviceToDevice, g->stream));
    HIPCHK(hipMemcpyAsync(g->w64.x, xio, g->N * sizeof(double), hipMemcpyDeviceToDevice, g->stream));
    pf_lin_info li{};
    pf_status st = solve_internal(g, op, o, &li);
    *iters += li.iters;
    if (st != PF_OK) return st;
    HIPCHK(hipMemcpyAsync(xio, g->w64.x, g->N * sizeof(double), hipMemcpyDeviceToDevice, g->stream));
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

pf_status pf_nonlinear_solve(pf_grid *g, const pf_pf_params *p, double *phi, double *conc, double *steric,
                             pf_nl_info *info)
{
    auto t0 = std::chrono::steady_clock::now();
    PFCHK(check_grid(g));
    if (!phi) return fail(PF_ERR_ARG, "phi is required");
    PFCHK(check_pf(p));
    pfk::SpeciesDev sp;
    PFCHK(species_dev(p, &sp));
    PFCHK(begin(g));
    PFCHK(ensure_work<double>(g));
    PFCHK(ensure_nl(g));
    const size_t N = g->N;
    const int B = pw_blocks(N);
    const double h3 = g->h * g->h * g->h;
    pf_nl_info ni{};
    int lin_iters = 0;
    pf_status st = PF_OK;

    hipLaunchKernelGGL(pfk::k_source, dim3(B), dim3(NT), 0, g->stream, N, (const double *)g->q, sp.lam / h3, g->src);
    HIPCHK(hipGetLastError());

    OpDesc phi_op;                      // potential system, sigma set per iteration
    OpDesc psi_op;                      // PF1: eps_s (1 - lc^2 Lap)
    psi_op.psi = true;
    psi_op.ceps = p->eps_s * p->lc * p->lc;
    psi_op.sig_const = p->eps_s;

    if (!p->warm_start) {
        // Table 2 step 2: PF2 with rho' = Psi = 0 (fixed charges only)
        PFCHK(fill<double>(g, g->phi0, 0.0, N));
        st = nl_solve(g, phi_op, g->src, g->phi0, &p->lin, &lin_iters);
    } else {
        HIPCHK(hipMemcpyAsync(g->phi0, phi, N * sizeof(double), hipMemcpyDefault, g->stream));
        hipLaunchKernelGGL(pfk::k_set_dirichlet, dim3(B), dim3(NT), 0, g->stream, N, g->phi0,
                           (const uint8_t *)g->flags, (uint8_t)pfk::F_DIR_PHI, (const double *)g->dval);
        HIPCHK(hipGetLastError());
    }
    PFCHK(fill<double>(g, g->psi, 0.0, N));
    double delta = INFINITY;
    int it = 0;
    while (st == PF_OK && it < p->max_outer) {
        ++it;
        // Fermi update at Phi_0: rhs1 = -rho_hat, sig = -rho_hat'  (Eq. (1), (11))
        hipLaunchKernelGGL(pfk::k_fermi, dim3(B), dim3(NT), 0, g->stream, N, (const double *)g->phi0,
                           (const uint8_t *)g->flags, sp, g->rhs1, (double *)nullptr, g->sig,
                           (double *)nullptr, (double *)nullptr);
        HIPCHK(hipGetLastError());
        // PF1 (Eq. (12), (14))
        if (p->lc > 0) {
            st = nl_solve(g, psi_op, g->rhs1, g->psi, &p->lin, &lin_iters);
            if (st != PF_OK) break;
        } else {
            hipLaunchKernelGGL(pfk::k_psi_local, dim3(B), dim3(NT), 0, g->stream, N, (const double *)g->rhs1,
                               (const uint8_t *)g->flags, 1.0 / p->eps_s, g->psi);
            HIPCHK(hipGetLastError());
        }
        // PF2 (Eq. (13)), warm-started from Phi_0
        hipLaunchKernelGGL(pfk::k_rhs_pf2, dim3(B), dim3(NT), 0, g->stream, N, (const double *)g->psi,
                           (const double *)g->sig, (const double *)g->phi0, (const double *)g->src, p->eps_s,
                           g->rhs2);
        HIPCHK(hipGetLastError());
        HIPCHK(hipMemcpyAsync(g->phi, g->phi0, N * sizeof(double), hipMemcpyDeviceToDevice, g->stream));
        phi_op.sigma = g->sig;
        st = nl_solve(g, phi_op, g->rhs2, g->phi, &p->lin, &lin_iters);
        if (st != PF_OK) break;
        // relaxation and max-norm test (Table 2 step 5)
        hipLaunchKernelGGL((pfk::k_relax<NT>), dim3(B), dim3(NT), 0, g->stream, N, g->phi0, g->phi, p->omega,
                           g->sc, g->partials, g->ticket, B);
        HIPCHK(hipGetLastError());
        PFCHK(read_scalars(g));
        delta = g->hsc->red[0];
        if (!std::isfinite(delta)) { st = PF_ERR_NONFINITE; break; }
        if (delta <= p->outer_tol) break;
    }
    if (st == PF_OK && !(delta <= p->outer_tol)) st = PF_ERR_NOCONV;
    HIPCHK(hipMemcpyAsync(phi, g->phi0, N * sizeof(double), hipMemcpyDefault, g->stream));
    if (conc || steric) {
        hipLaunchKernelGGL(pfk::k_fermi, dim3(B), dim3(NT), 0, g->stream, N, (const double *)g->phi0,
                           (const uint8_t *)g->flags, sp, (double *)nullptr, (double *)nullptr,
                           (double *)nullptr, conc, steric);
        HIPCHK(hipGetLastError());
    }
    PFCHK(sync(g));
    ni.outer_iters = it;
    ni.total_lin_iters = lin_iters;
    ni.last_delta = delta;
    ni.seconds = secs_since(t0);
    ni.status = st;
    if (info) *info = ni;
    if (st == PF_ERR_NOCONV && g_err.empty()) return fail(st, "outer loop: delta %.3e after %d iterations", delta, it);
    return st;
}

pf_status pf_linear_solve_batch(int32_t n, pf_grid *const *g, const double *const *sigma,
                                const double *const *b, double *const *x, const pf_lin_opts *opts,
                                pf_lin_info *info)
{
    if (n < 0 || (n > 0 && (!g || !b || !x))) return fail(PF_ERR_ARG, "bad batch arguments");
    pf_status worst = PF_OK;
    for (int i = 0; i < n; ++i) {
        pf_status st = pf_linear_solve(g[i], sigma ? sigma[i] : nullptr, b[i], x[i], opts, info ? &info[i] : nullptr);
        if (st != PF_OK && worst == PF_OK) worst = st;
        if (st == PF_ERR_ARG || st == PF_ERR_DEVICE || st == PF_ERR_ALLOC) return st;
    }
    return worst;
}

pf_status pf_nonlinear_solve_batch(int32_t n, pf_grid *const *g, const pf_pf_params *const *p,
                                   double *const *phi, pf_nl_info *info)
{
    if (n < 0 || (n > 0 && (!g || !p || !phi))) return fail(PF_ERR_ARG, "bad batch arguments");
    pf_status worst = PF_OK;
    for (int i = 0; i < n; ++i) {
        pf_status st = pf_nonlinear_solve(g[i], p[i], phi[i], nullptr, nullptr, info ? &info[i] : nullptr);
        if (st != PF_OK && worst == PF_OK) worst = st;
        if (st == PF_ERR_ARG || st == PF_ERR_DEVICE || st == PF_ERR_ALLOC) return st;
    }
    return worst;
}

}  // extern "C"
