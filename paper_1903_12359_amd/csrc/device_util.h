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

// Releases a buffer: pooled ones in the order of the calling scope's stream
// (else the stream they were made on), others with hipFree.
inline void dev_free(DevBuf& b) {
    if (b.p) {
        if (b.pooled) (void)hipFreeAsync(b.p, tls_alloc_set ? tls_alloc_stream : b.s);
        else (void)hipFree(b.p);
    }
    b = DevBuf{};
}

inline Error dev_alloc(DevBuf& b, size_t bytes) {
    if (b.bytes >= bytes && b.p) return Error{PGCP_OK, ""};
    dev_free(b);
    if (bytes == 0) bytes = 16;
    if (tls_alloc_set) {
        HIPCHK(hipMallocAsync(&b.p, bytes, tls_alloc_stream));
        b.s = tls_alloc_stream;
        b.pooled = true;
    } else {
        HIPCHK(hipMalloc(&b.p, bytes));
    }
    b.bytes = bytes;
    return Error{PGCP_OK, ""};
}

template <typename T, typename A>
inline Error upload(DevBuf& b, const std::vector<T, A>& v, hipStream_t s) {
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

// One DPP move of a double (both 32-bit halves) with a compile-time control.
template <int CTRL>
__device__ __forceinline__ double dpp_mov(double v) {
    int lo, hi;
    __builtin_memcpy(&lo, &v, 4);
    __builtin_memcpy(&hi, reinterpret_cast<const char*>(&v) + 4, 4);
    lo = __builtin_amdgcn_update_dpp(lo, lo, CTRL, 0xF, 0xF, false);
    hi = __builtin_amdgcn_update_dpp(hi, hi, CTRL, 0xF, 0xF, false);
    double r;
    __builtin_memcpy(&r, &lo, 4);
    __builtin_memcpy(reinterpret_cast<char*>(&r) + 4, &hi, 4);
    return r;
}

__device__ __forceinline__ double read_lane(double v, int l) {
    int lo, hi;
    __builtin_memcpy(&lo, &v, 4);
    __builtin_memcpy(&hi, reinterpret_cast<const char*>(&v) + 4, 4);
    lo = __builtin_amdgcn_readlane(lo, l);
    hi = __builtin_amdgcn_readlane(hi, l);
    double r;
    __builtin_memcpy(&r, &lo, 4);
    __builtin_memcpy(reinterpret_cast<char*>(&r) + 4, &hi, 4);
    return r;
}

// Sum over the 64 lanes of a wave, the same bits in every lane: DPP exchanges
// inside each row of 16 lanes (swap neighbours, swap pairs, mirror the
// half-rows, mirror the row), after which every lane holds its row's sum, then
// the four row sums in a fixed order.  All lanes must be active.
__device__ __forceinline__ double wave_sum(double v) {
    v += dpp_mov<0xB1>(v);    // quad_perm [1,0,3,2]
    v += dpp_mov<0x4E>(v);    // quad_perm [2,3,0,1]
    v += dpp_mov<0x141>(v);   // row_half_mirror
    v += dpp_mov<0x140>(v);   // row_mirror
    return (read_lane(v, 0) + read_lane(v, 16)) + (read_lane(v, 32) + read_lane(v, 48));
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
