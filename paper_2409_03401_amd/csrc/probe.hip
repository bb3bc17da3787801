// HBM streaming probe: the measured ceiling that the step's roofline is read against.
//
// A step reads every population once and writes every population once, so its
// ceiling on this GPU is that of a 1:1 read/write stream, not the vendor peak.  This
// kernel streams `bytes` with 16-byte non-temporal loads and stores in a grid-stride
// loop (four independent accesses in flight per thread), in one of three patterns:
// copy (read src, write dst), read only (src, folded into a value that is stored only
// when it is negative, which all-positive input never is), write only (dst).
#include <hip/hip_runtime.h>

#include <cstdint>

#include "lbm.h"

namespace {

// a native 16-byte vector (the non-temporal builtins take clang vector types)
typedef float v4f __attribute__((ext_vector_type(4)));

template <int MODE>
__global__ void __launch_bounds__(256) k_stream(const v4f* __restrict__ src, v4f* __restrict__ dst,
                                                unsigned long long n, float* __restrict__ sink) {
    const unsigned long long stride = (unsigned long long)gridDim.x * 256u;
    unsigned long long i = (unsigned long long)blockIdx.x * 256u + threadIdx.x;
    float acc = 0.0f;
    for (; i + 3 * stride < n; i += 4 * stride) {
        if constexpr (MODE == 0) {
            const v4f a = __builtin_nontemporal_load(src + i);
            const v4f b = __builtin_nontemporal_load(src + i + stride);
            const v4f c = __builtin_nontemporal_load(src + i + 2 * stride);
            const v4f d = __builtin_nontemporal_load(src + i + 3 * stride);
            __builtin_nontemporal_store(a, dst + i);
            __builtin_nontemporal_store(b, dst + i + stride);
            __builtin_nontemporal_store(c, dst + i + 2 * stride);
            __builtin_nontemporal_store(d, dst + i + 3 * stride);
        } else if constexpr (MODE == 1) {
            const v4f a = __builtin_nontemporal_load(src + i);
            const v4f b = __builtin_nontemporal_load(src + i + stride);
            const v4f c = __builtin_nontemporal_load(src + i + 2 * stride);
            const v4f d = __builtin_nontemporal_load(src + i + 3 * stride);
            acc += (a.x + b.x) + (c.x + d.x) + (a.w + b.w) + (c.w + d.w);
        } else {
            const float v = float(i & 1023u);
            __builtin_nontemporal_store(v4f(v), dst + i);
            __builtin_nontemporal_store(v4f(v), dst + i + stride);
            __builtin_nontemporal_store(v4f(v), dst + i + 2 * stride);
            __builtin_nontemporal_store(v4f(v), dst + i + 3 * stride);
        }
    }
    for (; i < n; i += stride) {
        if constexpr (MODE == 0) __builtin_nontemporal_store(__builtin_nontemporal_load(src + i), dst + i);
        else if constexpr (MODE == 1) acc += __builtin_nontemporal_load(src + i).x;
        else __builtin_nontemporal_store(v4f(1.0f), dst + i);
    }
    if constexpr (MODE == 1) {
        if (acc < 0.0f) sink[blockIdx.x & 255u] = acc;
    }
}

}  // namespace

extern "C" int lbm_probe_stream(const void* src, void* dst, size_t bytes, int32_t mode, int32_t grid,
                                void* stream) {
    if (bytes == 0 || bytes % 16 != 0) return LBM_EINVAL;
    if (grid < 1 || mode < 0 || mode > 2) return LBM_EINVAL;
    if ((mode != 2 && (!src || reinterpret_cast<uintptr_t>(src) % 16 != 0)) ||
        (!dst || reinterpret_cast<uintptr_t>(dst) % 16 != 0))
        return LBM_EINVAL;
    const unsigned long long n = bytes / 16;
    hipStream_t s = static_cast<hipStream_t>(stream);
    const v4f* in = static_cast<const v4f*>(src);
    v4f* out = static_cast<v4f*>(dst);
    float* sink = static_cast<float*>(dst);
    switch (mode) {
        case 0: hipLaunchKernelGGL(k_stream<0>, dim3(grid), dim3(256), 0, s, in, out, n, sink); break;
        case 1: hipLaunchKernelGGL(k_stream<1>, dim3(grid), dim3(256), 0, s, in, out, n, sink); break;
        default: hipLaunchKernelGGL(k_stream<2>, dim3(grid), dim3(256), 0, s, in, out, n, sink); break;
    }
    return hipGetLastError() == hipSuccess ? LBM_OK : LBM_EHIP;
}
