// Helpers shared by the device translation units of libpgcp: error checks,
// device buffers, launch sizes and fixed-order reductions.
#pragma once

#include <hip/hip_runtime.h>

#include <string>
#include <vector>

#include "pgcp_internal.h"

namespace pgcp {

#define HIPCHK(x)                                                                   \
    do {                                                                           \
        hipError_t _e = (x);                                                       \
        if (_e != hipSuccess)                                                      \
            return Error{PGCP_E_HIP, std::string(#x) + ": " + hipGetErrorString(_e)}; \
    } while (0)

constexpr int BLOCK = 256;
constexpr int WAVES = BLOCK / 64;
constexpr long long SPIN_MAX = 1ll << 24;

// ----------------------------------------------------------------- buffers

inline Error dev_alloc(DevBuf& b, size_t bytes) {
    if (b.bytes >= bytes && b.p) return Error{PGCP_OK, ""};
    if (b.p) (void)hipFree(b.p);
    b.p = nullptr;
    b.bytes = 0;
    if (bytes == 0) bytes = 16;
    HIPCHK(hipMalloc(&b.p, bytes));
    b.bytes = bytes;
    return Error{PGCP_OK, ""};
}

inline void dev_free(DevBuf& b) {
    if (b.p) (void)hipFree(b.p);
    b.p = nullptr;
    b.bytes = 0;
}

template <typename T>
inline Error upload(DevBuf& b, const std::vector<T>& v, hipStream_t s) {
    Error e = dev_alloc(b, v.size() * sizeof(T));
    if (e.code != PGCP_OK) return e;
    if (!v.empty()) HIPCHK(hipMemcpyAsync(b.p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice, s));
    return Error{PGCP_OK, ""};
}

inline unsigned grid_for(int64_t n) { return (unsigned)((n + BLOCK - 1) / BLOCK); }

// ----------------------------------------------------------------- small vector helpers

template <typename T> struct Vec2;
template <> struct Vec2<float> { using type = float2; };
template <> struct Vec2<double> { using type = double2; };

template <typename V, typename S>
__device__ __forceinline__ V axpy2(V x, S ax, S ay, V y) {   // y + a*x per component
    V o;
    o.x = y.x + ax * x.x;
    o.y = y.y + ay * x.y;
    return o;
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// Fixed-order block sum of NV values per thread; result valid in thread 0.
template <int NV>
__device__ __forceinline__ void block_sum(double (&v)[NV], double* lds) {
#pragma unroll
    for (int i = 0; i < NV; ++i) v[i] = wave_sum(v[i]);
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    if (lane == 0) {
#pragma unroll
        for (int i = 0; i < NV; ++i) lds[wave * NV + i] = v[i];
    }
    __syncthreads();
    if (threadIdx.x == 0) {
#pragma unroll
        for (int i = 0; i < NV; ++i) {
            double s = 0.0;
            for (int w = 0; w < WAVES; ++w) s += lds[w * NV + i];
            v[i] = s;
        }
    }
    __syncthreads();
}

}  // namespace pgcp
