// pf_stream.h -- streaming-bandwidth probe: the ceiling the stencil kernels
// are measured against (a measurement aid; no part of the method).
//
// Each lane streams R input arrays and W output arrays of doubles with
// accesses of V doubles (V = 1: 64-bit, V = 2: 128-bit), grid-stride; every
// output receives the sum of the inputs so that no load can be dropped.
#pragma once

#include <hip/hip_runtime.h>

namespace pfk {

struct StreamArgs {
    const double *in[8];
    double *out[4];
    size_t n;   // doubles per array (a multiple of V)
};

template <int R, int W, int V>
__global__ __launch_bounds__(256) void k_stream(StreamArgs a)
{
    using Vec = typename std::conditional<V == 2, double2, double>::type;
    const size_t nv = a.n / V;
    for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < nv; i += (size_t)gridDim.x * 256) {
        Vec s;
        if constexpr (V == 2) { s.x = 0.0; s.y = 0.0; } else { s = 0.0; }
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const Vec v = reinterpret_cast<const Vec *>(a.in[r])[i];
            if constexpr (V == 2) { s.x += v.x; s.y += v.y; } else { s += v; }
        }
#pragma unroll
        for (int w = 0; w < W; ++w) reinterpret_cast<Vec *>(a.out[w])[i] = s;
    }
}

}  // namespace pfk
