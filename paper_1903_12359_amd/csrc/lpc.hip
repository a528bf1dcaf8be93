// Learned sparse-approximate-inverse preconditioner: the message-passing
// network that maps every piece's cotangent Laplacian to an SPD matrix with
// the Laplacian's sparsity, its inference, and its training (loss, hand-written
// backward pass, Adam).  Dense layers run on the bf16 matrix cores (MFMA
// 16x16x32, fp32 accumulation); everything else is plain vector code.
//
// Graph.  The directed edges are the off-diagonal SELL slots of the plan
// (slot el of slice s, width index k, lane i: edge p -> q with p = 64 s + i,
// q = sl_col[el]); padding slots (q == p) are not edges.  sl_rev[el] is the
// slot of the reverse edge.  Node states live per packed row, edge states per
// slot, both 64 wide in bf16.
//
// Network (width 64; weights W_* in bf16, biases and heads in fp32):
//   h_p  = relu(x_p W_x + b_x),   x_p  = (1, mask_p, valence_p / 6)
//   e_pq = relu(y_pq W_y + b_y),  y_pq = (a, a^2, mask_q), a = -L_pq / sqrt(L_pp L_qq)
//   three rounds r:  m_pq = relu([h_p, h_q, e_pq] W_e^r + b_e^r);  e_pq = m_pq
//                    g_p  = mean_q m_pq;   h_p = relu([h_p, g_p] W_v^r + b_v^r)
//   o_pq = (e_pq + e_qp)/2 . u_e + c_e,   o_p = h_p . u_v + c_v
// Preconditioner on the free rows (d = diag L):
//   M = D^-1/2 (diag(exp(o_p) + sum_q |o_pq|) + O) D^-1/2,  O_pq = o_pq
// symmetric, strictly diagonally dominant inside the bracket, hence SPD; zero
// outputs give M = D^-1 (Jacobi).
//
// Flat parameter vector (fp32 master copy, this order): W_x[3][64], b_x[64],
// W_y[3][64], b_y[64], then per round W_e[192][64], b_e[64], W_v[128][64],
// b_v[64], then u_e[64], c_e, u_v[64], c_v.  Weight matrices are [in][out].

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstring>
#include <vector>

#include "device_util.h"
#include "pgcp_internal.h"

namespace pgcp {

// ------------------------------------------------------------------ layout of the parameters

constexpr int F = 64;                        // width
constexpr int ROUNDS = 3;
constexpr int OFF_WX = 0, OFF_BX = 192, OFF_WY = 256, OFF_BY = 448, OFF_R0 = 512;
constexpr int R_WE = 0, R_BE = 12288, R_WV = 12352, R_BV = 20544, R_SIZE = 20608;
constexpr int OFF_HEAD = OFF_R0 + ROUNDS * R_SIZE;   // 62336
constexpr int OFF_UE = OFF_HEAD, OFF_CE = OFF_HEAD + 64, OFF_UV = OFF_HEAD + 65, OFF_CV = OFF_HEAD + 129;
constexpr int N_PARAMS = OFF_HEAD + 130;             // 62466

// bf16 weight blocks (element offsets into one buffer).  "T" blocks are
// [out][in] (the B operand of X W), "N" blocks [in][out] (the B operand of
// dZ W^T); rows are padded so that LDS rows start on different banks.
constexpr int XS = 200;   // row stride of a 192-wide tile
constexpr int VS = 136;   // row stride of a 128-wide tile
constexpr int MS = 72;    // row stride of a 64-wide tile
constexpr int BLK_WET = 64 * XS, BLK_WVT = 64 * VS, BLK_WEN = 192 * MS, BLK_WVN = 128 * MS;
constexpr int W_ROUND = BLK_WET + BLK_WVT + BLK_WEN + BLK_WVN;
constexpr int W_XY = 2 * 3 * 64;                      // W_x, W_y rounded, [3][64] each
constexpr int W_TOTAL = ROUNDS * W_ROUND + W_XY;

typedef short bf16_t;
typedef __bf16 v8bf __attribute__((ext_vector_type(8)));
typedef float v4f __attribute__((ext_vector_type(4)));

__host__ __device__ __forceinline__ bf16_t f2bf(float f) {
    // round to nearest even (the values here are finite)
    uint32_t u;
    memcpy(&u, &f, 4);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (bf16_t)(u >> 16);
}
__host__ __device__ __forceinline__ float bf2f(bf16_t b) {
    uint32_t u = ((uint32_t)(uint16_t)b) << 16;
    float f;
    memcpy(&f, &u, 4);
    return f;
}

__device__ __forceinline__ v4f mfma(const v8bf& a, const v8bf& b, const v4f& c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ v8bf ld8(const bf16_t* p) {   // 16 bytes, 16-byte aligned
    v8bf v;
    __builtin_memcpy(&v, p, 16);
    return v;
}
__device__ __forceinline__ v8bf ld8_strided(const bf16_t* p, int stride) {
    v8bf v;
#pragma unroll
    for (int t = 0; t < 8; ++t) {
        bf16_t x = p[t * stride];
        __builtin_memcpy(reinterpret_cast<char*>(&v) + 2 * t, &x, 2);
    }
    return v;
}

// ------------------------------------------------------------------ weights

// theta (fp32) -> bf16 blocks per round: W_e^T, W_v^T, W_e, W_v; then W_x, W_y.
__global__ void k_lpc_pack(const float* __restrict__ th, bf16_t* __restrict__ wb) {
    const int64_t total = (int64_t)W_TOTAL;
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < total; t += (int64_t)gridDim.x * blockDim.x) {
        float v = 0.f;
        if (t < ROUNDS * W_ROUND) {
            const int r = (int)(t / W_ROUND);
            int o = (int)(t % W_ROUND);
            const float* We = th + OFF_R0 + r * R_SIZE + R_WE;
            const float* Wv = th + OFF_R0 + r * R_SIZE + R_WV;
            if (o < BLK_WET) {
                const int j = o / XS, k = o % XS;
                v = k < 192 ? We[k * 64 + j] : 0.f;
            } else if ((o -= BLK_WET) < BLK_WVT) {
                const int j = o / VS, k = o % VS;
                v = k < 128 ? Wv[k * 64 + j] : 0.f;
            } else if ((o -= BLK_WVT) < BLK_WEN) {
                const int k = o / MS, j = o % MS;
                v = j < 64 ? We[k * 64 + j] : 0.f;
            } else {
                o -= BLK_WEN;
                const int k = o / MS, j = o % MS;
                v = j < 64 ? Wv[k * 64 + j] : 0.f;
            }
        } else {
            const int o = (int)(t - ROUNDS * W_ROUND);
            v = o < 192 ? th[OFF_WX + o] : th[OFF_WY + (o - 192)];
        }
        wb[t] = f2bf(v);
    }
}

// ------------------------------------------------------------------ inputs

__device__ __forceinline__ bool slot_valid(const int32_t* __restrict__ sl_col, int64_t el, int64_t p) {
    return sl_col[el] != (int32_t)p;
}

// One thread per packed row: valence, h_0.  One thread per slot: e_0.
__global__ void __launch_bounds__(BLOCK) k_lpc_input_h(int64_t N, const int32_t* __restrict__ sl_w,
                                                        const int64_t* __restrict__ sl_ptr,
                                                        const int32_t* __restrict__ sl_col,
                                                        const uint8_t* __restrict__ mask,
                                                        const bf16_t* __restrict__ wxy,
                                                        const float* __restrict__ th, float* __restrict__ val,
                                                        bf16_t* __restrict__ h0) {
    const int64_t p = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
    if (p >= N) return;
    const int64_t s = p >> 6;
    const int w = sl_w[s];
    const int64_t base = sl_ptr[s] + (p & 63);
    int cnt = 0;
    for (int k = 0; k < w; ++k) cnt += slot_valid(sl_col, base + (int64_t)k * 64, p) ? 1 : 0;
    val[p] = (float)cnt;
    const float x1 = mask[p] ? 1.f : 0.f, x2 = (float)cnt / 6.f;
    bf16_t out[F];
#pragma unroll
    for (int j = 0; j < F; ++j) {
        float z = bf2f(wxy[j]) + x1 * bf2f(wxy[64 + j]) + x2 * bf2f(wxy[128 + j]) + th[OFF_BX + j];
        out[j] = f2bf(fmaxf(z, 0.f));
    }
    __builtin_memcpy(h0 + p * F, out, sizeof(out));
}

// One wavefront per slice: e_0 of its slots, looping over the width.
__global__ void __launch_bounds__(64) k_lpc_input_e(const int64_t* __restrict__ sl_ptr,
                                                     const int32_t* __restrict__ sl_w,
                                                     const int32_t* __restrict__ sl_col,
                                                     const double* __restrict__ val64,
                                                     const double* __restrict__ diag64,
                                                     const uint8_t* __restrict__ mask,
                                                     const bf16_t* __restrict__ wxy,
                                                     const float* __restrict__ th, bf16_t* __restrict__ e0) {
    const int64_t s = blockIdx.x;
    const int lane = threadIdx.x;
    const int64_t p = s * 64 + lane;
    const int w = sl_w[s];
    const bf16_t* wy = wxy + 192;
    for (int k = 0; k < w; ++k) {
        const int64_t el = sl_ptr[s] + (int64_t)k * 64 + lane;
        const int32_t q = sl_col[el];
        bf16_t out[F];
        if (q == (int32_t)p) {
#pragma unroll
            for (int j = 0; j < F; ++j) out[j] = 0;
        } else {
            const float a = (float)(-val64[el] / sqrt(diag64[p] * diag64[q]));
            const float y0 = a, y1 = a * a, y2 = mask[q] ? 1.f : 0.f;
#pragma unroll
            for (int j = 0; j < F; ++j) {
                float z = y0 * bf2f(wy[j]) + y1 * bf2f(wy[64 + j]) + y2 * bf2f(wy[128 + j]) + th[OFF_BY + j];
                out[j] = f2bf(fmaxf(z, 0.f));
            }
        }
        __builtin_memcpy(e0 + el * F, out, sizeof(out));
    }
}

// ------------------------------------------------------------------ one round (forward)

// Persistent over slices.  Per slice and width index k, the 64 edges of the
// slice's lanes form a 64 x 192 input tile [h_p, h_q, e_pq] (staged in LDS);
// four waves compute 16 rows x 64 outputs each with MFMA; the ReLU output is
// the new edge state and is summed per row for the mean aggregation.  Then
// the vertex MLP on [h_p, g_p] (64 x 128) gives the new node states.
__global__ void __launch_bounds__(256) k_lpc_round(int64_t nslices, const int64_t* __restrict__ sl_ptr,
                                                    const int32_t* __restrict__ sl_w,
                                                    const int32_t* __restrict__ sl_col,
                                                    const float* __restrict__ val,
                                                    const bf16_t* __restrict__ h_in, const bf16_t* __restrict__ e_in,
                                                    bf16_t* __restrict__ h_out, bf16_t* __restrict__ e_out,
                                                    const bf16_t* __restrict__ wr, const float* __restrict__ thr) {
    __shared__ __attribute__((aligned(16))) bf16_t sWe[64 * XS];
    __shared__ __attribute__((aligned(16))) bf16_t sWv[64 * VS];
    __shared__ __attribute__((aligned(16))) bf16_t sX[64 * XS];
    __shared__ __attribute__((aligned(16))) bf16_t sM[64 * MS];
    __shared__ float sBe[64], sBv[64];
    __shared__ int sValid[64];
    const int tid = threadIdx.x, wave = tid >> 6, l = tid & 63;
    for (int t = tid; t < BLK_WET / 8; t += 256) __builtin_memcpy(sWe + 8 * t, wr + 8 * t, 16);
    for (int t = tid; t < BLK_WVT / 8; t += 256) __builtin_memcpy(sWv + 8 * t, wr + BLK_WET + 8 * t, 16);
    if (tid < 64) {
        sBe[tid] = thr[R_BE + tid];
        sBv[tid] = thr[R_BV + tid];
    }
    const int ar = 16 * wave + (l & 15);      // A-operand row of this lane
    const int ak = 8 * (l >> 4);              // A/B-operand k offset of this lane
    const int dr = 16 * wave + 4 * (l >> 4);  // first output row of this lane (D layout)
    const int dc = l & 15;                    // output column inside a 16-wide tile
    for (int64_t s = blockIdx.x; s < nslices; s += gridDim.x) {
        const int w = sl_w[s];
        const int64_t base = sl_ptr[s];
        float g[4][4];
#pragma unroll
        for (int ct = 0; ct < 4; ++ct)
#pragma unroll
            for (int v = 0; v < 4; ++v) g[ct][v] = 0.f;
        for (int k = 0; k < w; ++k) {
            __syncthreads();
            for (int idx = tid; idx < 64 * 24; idx += 256) {
                const int i = idx / 24, c = idx % 24, seg = c >> 3, off = (c & 7) * 8;
                const int64_t el = base + (int64_t)k * 64 + i, p = s * 64 + i;
                const int32_t q = sl_col[el];
                const bool ok = q != (int32_t)p;
                if (c == 0) sValid[i] = ok ? 1 : 0;
                const bf16_t* src = seg == 0 ? h_in + p * F : (seg == 1 ? h_in + (int64_t)q * F : e_in + el * F);
                uint4 v = make_uint4(0, 0, 0, 0);
                if (ok) __builtin_memcpy(&v, src + off, 16);
                __builtin_memcpy(sX + i * XS + c * 8, &v, 16);
            }
            __syncthreads();
            v4f acc[4];
#pragma unroll
            for (int ct = 0; ct < 4; ++ct) acc[ct] = v4f{0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int kk = 0; kk < 6; ++kk) {
                const v8bf a = ld8(sX + ar * XS + 32 * kk + ak);
#pragma unroll
                for (int ct = 0; ct < 4; ++ct) acc[ct] = mfma(a, ld8(sWe + (16 * ct + dc) * XS + 32 * kk + ak), acc[ct]);
            }
#pragma unroll
            for (int ct = 0; ct < 4; ++ct)
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int i = dr + v, j = 16 * ct + dc;
                    float m = fmaxf(acc[ct][v] + sBe[j], 0.f);
                    m = sValid[i] ? m : 0.f;
                    const bf16_t mb = f2bf(m);
                    g[ct][v] += bf2f(mb);
                    sM[i * MS + j] = mb;
                }
            __syncthreads();
            for (int idx = tid; idx < 64 * 8; idx += 256) {
                const int i = idx >> 3, c = idx & 7;
                const int64_t el = base + (int64_t)k * 64 + i;
                __builtin_memcpy(e_out + el * F + 8 * c, sM + i * MS + 8 * c, 16);
            }
        }
        // vertex MLP on [h_p, mean_q m_pq]
        __syncthreads();
        for (int idx = tid; idx < 64 * 8; idx += 256) {
            const int i = idx >> 3, c = idx & 7;
            __builtin_memcpy(sX + i * VS + 8 * c, h_in + (s * 64 + i) * F + 8 * c, 16);
        }
#pragma unroll
        for (int ct = 0; ct < 4; ++ct)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int i = dr + v;
                const float vl = fmaxf(val[s * 64 + i], 1.f);
                sX[i * VS + 64 + 16 * ct + dc] = f2bf(g[ct][v] / vl);
            }
        __syncthreads();
        v4f acc[4];
#pragma unroll
        for (int ct = 0; ct < 4; ++ct) acc[ct] = v4f{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int kk = 0; kk < 4; ++kk) {
            const v8bf a = ld8(sX + ar * VS + 32 * kk + ak);
#pragma unroll
            for (int ct = 0; ct < 4; ++ct) acc[ct] = mfma(a, ld8(sWv + (16 * ct + dc) * VS + 32 * kk + ak), acc[ct]);
        }
#pragma unroll
        for (int ct = 0; ct < 4; ++ct)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int i = dr + v, j = 16 * ct + dc;
                sM[i * MS + j] = f2bf(fmaxf(acc[ct][v] + sBv[j], 0.f));
            }
        __syncthreads();
        for (int idx = tid; idx < 64 * 8; idx += 256) {
            const int i = idx >> 3, c = idx & 7;
            __builtin_memcpy(h_out + (s * 64 + i) * F + 8 * c, sM + i * MS + 8 * c, 16);
        }
    }
}

// ------------------------------------------------------------------ heads and the SPAI values

__device__ __forceinline__ float dot64(const bf16_t* __restrict__ x, const float* __restrict__ u) {
    float acc = 0.f;
#pragma unroll
    for (int c = 0; c < 8; ++c) {
        bf16_t t[8];
        __builtin_memcpy(t, x + 8 * c, 16);
#pragma unroll
        for (int j = 0; j < 8; ++j) acc += bf2f(t[j]) * u[8 * c + j];
    }
    return acc;
}

__global__ void __launch_bounds__(BLOCK) k_lpc_head_e(int64_t nslot, const int32_t* __restrict__ sl_rev,
                                                       const bf16_t* __restrict__ e3, const float* __restrict__ th,
                                                       float* __restrict__ o_e) {
    const int64_t el = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
    if (el >= nslot) return;
    const int32_t rv = sl_rev[el];
    if (rv < 0) {
        o_e[el] = 0.f;
        return;
    }
    const float* u = th + OFF_UE;
    o_e[el] = 0.5f * (dot64(e3 + el * F, u) + dot64(e3 + (int64_t)rv * F, u)) + th[OFF_CE];
}

__global__ void __launch_bounds__(BLOCK) k_lpc_head_v(int64_t N, const bf16_t* __restrict__ h3,
                                                       const float* __restrict__ th, float* __restrict__ o_v) {
    const int64_t p = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
    if (p >= N) return;
    o_v[p] = dot64(h3 + p * F, th + OFF_UV) + th[OFF_CV];
}

// One thread per row: M's diagonal and off-diagonal values (FP32 and FP64)
// for the free rows; masked rows get an all-zero row.
__global__ void __launch_bounds__(BLOCK) k_lpc_spai(int64_t N, const int64_t* __restrict__ sl_ptr,
                                                     const int32_t* __restrict__ sl_w,
                                                     const int32_t* __restrict__ sl_col,
                                                     const double* __restrict__ diag64,
                                                     const uint8_t* __restrict__ mask,
                                                     const float* __restrict__ o_e, const float* __restrict__ o_v,
                                                     float* __restrict__ mval32, float* __restrict__ mdiag32,
                                                     double* __restrict__ mval64, double* __restrict__ mdiag64) {
    const int64_t p = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
    if (p >= N) return;
    const int64_t s = p >> 6;
    const int w = sl_w[s];
    const int64_t base = sl_ptr[s] + (p & 63);
    const bool free_p = !mask[p];
    const double dp = diag64[p];
    double sum = 0.0;
    for (int k = 0; k < w; ++k) {
        const int64_t el = base + (int64_t)k * 64;
        const int32_t q = sl_col[el];
        double m = 0.0;
        if (free_p && q != (int32_t)p && !mask[q]) {
            const double o = (double)o_e[el];
            sum += fabs(o);
            m = o / sqrt(dp * diag64[q]);
        }
        mval64[el] = m;
        mval32[el] = (float)m;
    }
    const double d = free_p ? (exp((double)o_v[p]) + sum) / dp : 0.0;
    mdiag64[p] = d;
    mdiag32[p] = (float)d;
}


// ================================================================== training

// AV[k][p] = (A v_k)_p on the free rows (A = L with masked rows and columns
// removed); 0 on masked rows.  One thread per row, P probes.
__global__ void __launch_bounds__(BLOCK) k_lpc_av(int64_t N, int P, const int64_t* __restrict__ sl_ptr,
                                                   const int32_t* __restrict__ sl_w,
                                                   const int32_t* __restrict__ sl_col,
                                                   const double* __restrict__ val64,
                                                   const double* __restrict__ diag64,
                                                   const uint8_t* __restrict__ mask, const float* __restrict__ V,
                                                   float* __restrict__ AV) {
    const int64_t p = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
    if (p >= N) return;
    const int64_t s = p >> 6;
    const int w = sl_w[s];
    const int64_t base = sl_ptr[s] + (p & 63);
    const bool fr = !mask[p];
    for (int k = 0; k < P; ++k) {
        const float* v = V + (int64_t)k * N;
        double acc = 0.0;
        if (fr) {
            acc = diag64[p] * (double)v[p];
            for (int t = 0; t < w; ++t) {
                const int64_t el = base + (int64_t)t * 64;
                const int32_t q = sl_col[el];
                if (q != (int32_t)p && !mask[q]) acc += val64[el] * (double)v[q];
            }
        }
        AV[(int64_t)k * N + p] = (float)acc;
    }
}

// R[k][p] = (M AV_k)_p - v_k,p on the free rows; per-slice partial sums of
// R^2 and v^2 per probe (one wavefront per slice).
__global__ void __launch_bounds__(64) k_lpc_resid(int64_t N, int P, const int64_t* __restrict__ sl_ptr,
                                                   const int32_t* __restrict__ sl_w,
                                                   const int32_t* __restrict__ sl_col,
                                                   const float* __restrict__ mval, const float* __restrict__ mdiag,
                                                   const uint8_t* __restrict__ mask, const float* __restrict__ V,
                                                   const float* __restrict__ AV, float* __restrict__ R,
                                                   double* __restrict__ slicepart) {
    const int64_t s = blockIdx.x;
    const int lane = threadIdx.x;
    const int64_t p = s * 64 + lane;
    const int w = sl_w[s];
    const int64_t base = sl_ptr[s] + lane;
    const bool fr = !mask[p];
    for (int k = 0; k < P; ++k) {
        const float* av = AV + (int64_t)k * N;
        double r = 0.0, vv = 0.0;
        if (fr) {
            double acc = (double)mdiag[p] * av[p];
            for (int t = 0; t < w; ++t) {
                const int64_t el = base + (int64_t)t * 64;
                const int32_t q = sl_col[el];
                if (q != (int32_t)p) acc += (double)mval[el] * av[q];
            }
            const double v = V[(int64_t)k * N + p];
            r = acc - v;
            vv = v * v;
        }
        R[(int64_t)k * N + p] = (float)r;
        const double r2 = wave_sum(r * r), v2 = wave_sum(vv);
        if (lane == 0) {
            slicepart[(s * P + k) * 2] = r2;
            slicepart[(s * P + k) * 2 + 1] = v2;
        }
    }
}

// Per piece: fixed-order sum of its slices' partials (2P values).
__global__ void __launch_bounds__(64) k_lpc_piece_sum(int P, const int32_t* __restrict__ row0,
                                                       const double* __restrict__ slicepart,
                                                       double* __restrict__ piece) {
    const int i = blockIdx.x;
    const int64_t s0 = row0[i] >> 6, s1 = row0[i + 1] >> 6;
    for (int t = threadIdx.x; t < 2 * P; t += 64) {
        double acc = 0.0;
        for (int64_t s = s0; s < s1; ++s) acc += slicepart[s * 2 * P + t];
        piece[(int64_t)i * 2 * P + t] = acc;
    }
}

// d loss / d o.  c[i*P + k] = 2 / (K P |v_k|^2 of piece i).
__global__ void __launch_bounds__(BLOCK) k_lpc_outgrad(int64_t N, int P, const int32_t* __restrict__ slice_sub,
                                                        const int64_t* __restrict__ sl_ptr,
                                                        const int32_t* __restrict__ sl_w,
                                                        const int32_t* __restrict__ sl_col,
                                                        const double* __restrict__ diag64,
                                                        const uint8_t* __restrict__ mask,
                                                        const float* __restrict__ AV, const float* __restrict__ R,
                                                        const double* __restrict__ c, const float* __restrict__ o_e,
                                                        const float* __restrict__ o_v, float* __restrict__ go_e,
                                                        float* __restrict__ go_v) {
    const int64_t p = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
    if (p >= N) return;
    const int64_t s = p >> 6;
    const int w = sl_w[s];
    const int64_t base = sl_ptr[s] + (p & 63);
    const int sub = slice_sub[s];
    if (mask[p]) {
        go_v[p] = 0.f;
        for (int t = 0; t < w; ++t) go_e[base + (int64_t)t * 64] = 0.f;
        return;
    }
    double G[16];
    double dMd = 0.0;
    for (int k = 0; k < P; ++k) {
        G[k] = c[(int64_t)sub * P + k] * (double)R[(int64_t)k * N + p];
        dMd += G[k] * (double)AV[(int64_t)k * N + p];
    }
    const double dp = diag64[p];
    go_v[p] = (float)(dMd * exp((double)o_v[p]) / dp);
    for (int t = 0; t < w; ++t) {
        const int64_t el = base + (int64_t)t * 64;
        const int32_t q = sl_col[el];
        double g = 0.0;
        if (q != (int32_t)p && !mask[q]) {
            double dMe = 0.0;
            for (int k = 0; k < P; ++k) dMe += G[k] * (double)AV[(int64_t)k * N + q];
            const double o = o_e[el];
            const double sg = o > 0.0 ? 1.0 : (o < 0.0 ? -1.0 : 0.0);
            g = dMe / sqrt(dp * diag64[q]) + sg * dMd / dp;
        }
        go_e[el] = (float)g;
    }
}

// Feature-parallel reductions: thread (j = tid % 64) of wave (tid / 64)
// accumulates one feature over a strided set of items; the four waves are
// combined in a fixed order.  gp is this workgroup's row of partial gradients.
__device__ __forceinline__ void wg_feature_sum(float acc, int off, float* __restrict__ gpw, float* lds) {
    const int j = threadIdx.x & 63, wv = threadIdx.x >> 6;
    lds[wv * 64 + j] = acc;
    __syncthreads();
    if (wv == 0) gpw[off + j] += lds[j] + lds[64 + j] + lds[128 + j] + lds[192 + j];
    __syncthreads();
}
__device__ __forceinline__ void wg_scalar_sum(float acc, int off, float* __restrict__ gpw, float* lds) {
    const int t = threadIdx.x;
    lds[t] = acc;
    __syncthreads();
    if (t == 0) {
        float s = 0.f;
        for (int u = 0; u < 256; ++u) s += lds[u];
        gpw[off] += s;
    }
    __syncthreads();
}

// Heads: du_e, dc_e, du_v, dc_v; the gradients of the last edge and node
// states: de3 = (go_e[el] + go_e[rev]) / 2 * u_e, dh3 = go_v * u_v.
__global__ void __launch_bounds__(256) k_lpc_head_bwd(int64_t N, int64_t nslot, const int32_t* __restrict__ sl_rev,
                                                       const bf16_t* __restrict__ e3, const bf16_t* __restrict__ h3,
                                                       const float* __restrict__ go_e, const float* __restrict__ go_v,
                                                       const float* __restrict__ th, float* __restrict__ de3,
                                                       float* __restrict__ dh3, float* __restrict__ gp) {
    __shared__ float lds[256];
    float* gpw = gp + (int64_t)blockIdx.x * N_PARAMS;
    const int j = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int64_t stride = (int64_t)gridDim.x * 4;
    float due = 0.f, dce = 0.f;
    const float ue = th[OFF_UE + j];
    for (int64_t el = (int64_t)blockIdx.x * 4 + wv; el < nslot; el += stride) {
        const int32_t rv = sl_rev[el];
        float d = 0.f;
        if (rv >= 0) {
            const float g = go_e[el];
            const float sj = 0.5f * (bf2f(e3[el * F + j]) + bf2f(e3[(int64_t)rv * F + j]));
            due += g * sj;
            if (j == 0) dce += g;
            d = 0.5f * (g + go_e[rv]) * ue;
        }
        de3[el * F + j] = d;
    }
    wg_feature_sum(due, OFF_UE, gpw, lds);
    wg_scalar_sum(dce, OFF_CE, gpw, lds);
    float duv = 0.f, dcv = 0.f;
    const float uv = th[OFF_UV + j];
    for (int64_t p = (int64_t)blockIdx.x * 4 + wv; p < N; p += stride) {
        const float g = go_v[p];
        duv += g * bf2f(h3[p * F + j]);
        if (j == 0) dcv += g;
        dh3[p * F + j] = g * uv;
    }
    wg_feature_sum(duv, OFF_UV, gpw, lds);
    wg_scalar_sum(dcv, OFF_CV, gpw, lds);
}

// Backward of one round, persistent over slices (see the forward kernel for
// the tiles).  Per slice: dzv = dh' * [h' > 0]; dW_v += [h, g]^T dzv;
// [dh, dg] = dzv W_v^T; then per width index k: dze = (de' + dg/val) * [e' > 0];
// dW_e += [h_p, h_q, e]^T dze; [dh_p, dh_q, de] = dze W_e^T.  dh_p of the own
// rows accumulates in registers (written to dh_own); dh_q goes to dxdst[slot]
// and is gathered by row q afterwards; de goes to de_out[slot].  Weight and
// bias gradients accumulate per workgroup across its slices and are written
// to its row of gp.
__global__ void __launch_bounds__(256) k_lpc_round_bwd(int64_t nslices, const int64_t* __restrict__ sl_ptr,
                                                        const int32_t* __restrict__ sl_w,
                                                        const int32_t* __restrict__ sl_col,
                                                        const float* __restrict__ val,
                                                        const bf16_t* __restrict__ h_in,
                                                        const bf16_t* __restrict__ e_in,
                                                        const bf16_t* __restrict__ h_out,
                                                        const bf16_t* __restrict__ e_out,
                                                        const float* __restrict__ dh_out,
                                                        const float* __restrict__ de_out_grad,
                                                        const bf16_t* __restrict__ wr, int round,
                                                        float* __restrict__ dh_own, float* __restrict__ dxdst,
                                                        float* __restrict__ de_in_grad, float* __restrict__ gp) {
    __shared__ __attribute__((aligned(16))) bf16_t sWeN[192 * MS];
    __shared__ __attribute__((aligned(16))) bf16_t sWvN[128 * MS];
    __shared__ __attribute__((aligned(16))) bf16_t sXT[192 * MS];
    __shared__ __attribute__((aligned(16))) bf16_t sDZ[64 * MS];
    __shared__ __attribute__((aligned(16))) bf16_t sDZT[64 * MS];
    __shared__ float sDG[64 * 65];
    __shared__ float sDBe[64], sDBv[64];
    __shared__ int sValid[64];
    const int tid = threadIdx.x, wave = tid >> 6, l = tid & 63;
    const bf16_t* gWeN = wr + BLK_WET + BLK_WVT;
    const bf16_t* gWvN = gWeN + BLK_WEN;
    for (int t = tid; t < BLK_WEN / 8; t += 256) __builtin_memcpy(sWeN + 8 * t, gWeN + 8 * t, 16);
    for (int t = tid; t < BLK_WVN / 8; t += 256) __builtin_memcpy(sWvN + 8 * t, gWvN + 8 * t, 16);
    if (tid < 64) {
        sDBe[tid] = 0.f;
        sDBv[tid] = 0.f;
    }
    const int ar = 16 * wave + (l & 15);
    const int ak = 8 * (l >> 4);
    const int dr = 16 * wave + 4 * (l >> 4);
    const int dc = l & 15;
    v4f accWe[3][4], accWv[2][4];
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) accWe[a][b] = v4f{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) accWv[a][b] = v4f{0.f, 0.f, 0.f, 0.f};

    for (int64_t s = blockIdx.x; s < nslices; s += gridDim.x) {
        const int w = sl_w[s];
        const int64_t base = sl_ptr[s];
        __syncthreads();
        // ---- vertex part: stage dzv (both layouts) and [h, g]^T
        for (int idx = tid; idx < 64 * 64; idx += 256) {
            const int i = idx >> 6, j = idx & 63;
            const int64_t p = s * 64 + i;
            const float d = (bf2f(h_out[p * F + j]) > 0.f) ? dh_out[p * F + j] : 0.f;
            const bf16_t db = f2bf(d);
            sDZ[i * MS + j] = db;
            sDZT[j * MS + i] = db;
            sXT[j * MS + i] = h_in[p * F + j];
            float gs = 0.f;
            for (int k = 0; k < w; ++k) {
                const int64_t el = base + (int64_t)k * 64 + i;
                if (sl_col[el] != (int32_t)p) gs += bf2f(e_out[el * F + j]);
            }
            sXT[(64 + j) * MS + i] = f2bf(gs / fmaxf(val[p], 1.f));
        }
        __syncthreads();
        if (tid < 64) {
            float a = 0.f;
            for (int i = 0; i < 64; ++i) a += bf2f(sDZ[i * MS + tid]);
            sDBv[tid] += a;
        }
        // dW_v += [h, g]^T dzv   (wave: feature rows 32 wave .. +31)
#pragma unroll
        for (int kk = 0; kk < 2; ++kk) {
#pragma unroll
            for (int rt = 0; rt < 2; ++rt) {
                const v8bf a = ld8(sXT + (32 * wave + 16 * rt + (l & 15)) * MS + 32 * kk + ak);
#pragma unroll
                for (int ct = 0; ct < 4; ++ct)
                    accWv[rt][ct] = mfma(a, ld8(sDZT + (16 * ct + dc) * MS + 32 * kk + ak), accWv[rt][ct]);
            }
        }
        // [dh, dg] = dzv W_v^T
        v4f dh[4];
#pragma unroll
        for (int ct = 0; ct < 4; ++ct) dh[ct] = v4f{0.f, 0.f, 0.f, 0.f};
        {
            v4f dg[4];
#pragma unroll
            for (int ct = 0; ct < 4; ++ct) dg[ct] = v4f{0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int kk = 0; kk < 2; ++kk) {
                const v8bf a = ld8(sDZ + ar * MS + 32 * kk + ak);
#pragma unroll
                for (int ct = 0; ct < 4; ++ct) {
                    dh[ct] = mfma(a, ld8(sWvN + (16 * ct + dc) * MS + 32 * kk + ak), dh[ct]);
                    dg[ct] = mfma(a, ld8(sWvN + (64 + 16 * ct + dc) * MS + 32 * kk + ak), dg[ct]);
                }
            }
#pragma unroll
            for (int ct = 0; ct < 4; ++ct)
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int i = dr + v;
                    sDG[i * 65 + 16 * ct + dc] = dg[ct][v] / fmaxf(val[s * 64 + i], 1.f);
                }
        }
        // ---- edge part
        for (int k = 0; k < w; ++k) {
            __syncthreads();
            for (int idx = tid; idx < 64 * 64; idx += 256) {
                const int i = idx >> 6, j = idx & 63;
                const int64_t p = s * 64 + i, el = base + (int64_t)k * 64 + i;
                const int32_t q = sl_col[el];
                const bool ok = q != (int32_t)p;
                if (j == 0) sValid[i] = ok ? 1 : 0;
                float d = 0.f;
                bf16_t hp = 0, hq = 0, ee = 0;
                if (ok) {
                    if (bf2f(e_out[el * F + j]) > 0.f) d = de_out_grad[el * F + j] + sDG[i * 65 + j];
                    hp = h_in[p * F + j];
                    hq = h_in[(int64_t)q * F + j];
                    ee = e_in[el * F + j];
                }
                const bf16_t db = f2bf(d);
                sDZ[i * MS + j] = db;
                sDZT[j * MS + i] = db;
                sXT[j * MS + i] = hp;
                sXT[(64 + j) * MS + i] = hq;
                sXT[(128 + j) * MS + i] = ee;
            }
            __syncthreads();
            if (tid < 64) {
                float a = 0.f;
                for (int i = 0; i < 64; ++i) a += bf2f(sDZ[i * MS + tid]);
                sDBe[tid] += a;
            }
            // dW_e += X^T dze   (wave: feature rows 48 wave .. +47)
#pragma unroll
            for (int kk = 0; kk < 2; ++kk) {
#pragma unroll
                for (int rt = 0; rt < 3; ++rt) {
                    const v8bf a = ld8(sXT + (48 * wave + 16 * rt + (l & 15)) * MS + 32 * kk + ak);
#pragma unroll
                    for (int ct = 0; ct < 4; ++ct)
                        accWe[rt][ct] = mfma(a, ld8(sDZT + (16 * ct + dc) * MS + 32 * kk + ak), accWe[rt][ct]);
                }
            }
            // [dh_p, dh_q, de] = dze W_e^T
            v4f dq[4], de[4];
#pragma unroll
            for (int ct = 0; ct < 4; ++ct) {
                dq[ct] = v4f{0.f, 0.f, 0.f, 0.f};
                de[ct] = v4f{0.f, 0.f, 0.f, 0.f};
            }
#pragma unroll
            for (int kk = 0; kk < 2; ++kk) {
                const v8bf a = ld8(sDZ + ar * MS + 32 * kk + ak);
#pragma unroll
                for (int ct = 0; ct < 4; ++ct) {
                    dh[ct] = mfma(a, ld8(sWeN + (16 * ct + dc) * MS + 32 * kk + ak), dh[ct]);
                    dq[ct] = mfma(a, ld8(sWeN + (64 + 16 * ct + dc) * MS + 32 * kk + ak), dq[ct]);
                    de[ct] = mfma(a, ld8(sWeN + (128 + 16 * ct + dc) * MS + 32 * kk + ak), de[ct]);
                }
            }
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int i = dr + v;
                if (!sValid[i]) continue;
                const int64_t el = base + (int64_t)k * 64 + i;
#pragma unroll
                for (int ct = 0; ct < 4; ++ct) {
                    dxdst[el * F + 16 * ct + dc] = dq[ct][v];
                    de_in_grad[el * F + 16 * ct + dc] = de[ct][v];
                }
            }
        }
#pragma unroll
        for (int ct = 0; ct < 4; ++ct)
#pragma unroll
            for (int v = 0; v < 4; ++v) dh_own[(s * 64 + dr + v) * F + 16 * ct + dc] = dh[ct][v];
    }
    // ---- this workgroup's weight and bias gradients
    __syncthreads();
    float* gpw = gp + (int64_t)blockIdx.x * N_PARAMS + OFF_R0 + round * R_SIZE;
#pragma unroll
    for (int rt = 0; rt < 3; ++rt)
#pragma unroll
        for (int ct = 0; ct < 4; ++ct)
#pragma unroll
            for (int v = 0; v < 4; ++v)
                gpw[R_WE + (48 * wave + 16 * rt + 4 * (l >> 4) + v) * 64 + 16 * ct + dc] = accWe[rt][ct][v];
#pragma unroll
    for (int rt = 0; rt < 2; ++rt)
#pragma unroll
        for (int ct = 0; ct < 4; ++ct)
#pragma unroll
            for (int v = 0; v < 4; ++v)
                gpw[R_WV + (32 * wave + 16 * rt + 4 * (l >> 4) + v) * 64 + 16 * ct + dc] = accWv[rt][ct][v];
    if (tid < 64) {
        gpw[R_BE + tid] = sDBe[tid];
        gpw[R_BV + tid] = sDBv[tid];
    }
}

// dh[q] = dh_own[q] + sum over the slots el' of row q of dxdst[rev(el')].
__global__ void __launch_bounds__(BLOCK) k_lpc_gather(int64_t N, const int64_t* __restrict__ sl_ptr,
                                                       const int32_t* __restrict__ sl_w,
                                                       const int32_t* __restrict__ sl_rev,
                                                       const float* __restrict__ dh_own,
                                                       const float* __restrict__ dxdst, float* __restrict__ dh) {
    const int64_t t = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
    if (t >= N * F) return;
    const int64_t q = t >> 6;
    const int j = (int)(t & 63);
    const int64_t s = q >> 6;
    const int w = sl_w[s];
    const int64_t base = sl_ptr[s] + (q & 63);
    float acc = dh_own[t];
    for (int k = 0; k < w; ++k) {
        const int32_t rv = sl_rev[base + (int64_t)k * 64];
        if (rv >= 0) acc += dxdst[(int64_t)rv * F + j];
    }
    dh[t] = acc;
}

// Input encoders: dW_x, db_x from dh_0; dW_y, db_y from de_0.
__global__ void __launch_bounds__(256) k_lpc_input_bwd(int64_t N, int64_t nslices, const int64_t* __restrict__ sl_ptr,
                                                        const int32_t* __restrict__ sl_w,
                                                        const int32_t* __restrict__ sl_col,
                                                        const double* __restrict__ val64,
                                                        const double* __restrict__ diag64,
                                                        const uint8_t* __restrict__ mask,
                                                        const float* __restrict__ val,
                                                        const bf16_t* __restrict__ h0, const bf16_t* __restrict__ e0,
                                                        const float* __restrict__ dh0, const float* __restrict__ de0,
                                                        float* __restrict__ gp) {
    __shared__ float lds[256];
    float* gpw = gp + (int64_t)blockIdx.x * N_PARAMS;
    const int j = threadIdx.x & 63, wv = threadIdx.x >> 6;
    float wx[3] = {0.f, 0.f, 0.f}, bx = 0.f;
    for (int64_t p = (int64_t)blockIdx.x * 4 + wv; p < N; p += (int64_t)gridDim.x * 4) {
        if (!(bf2f(h0[p * F + j]) > 0.f)) continue;
        const float d = dh0[p * F + j];
        wx[0] += d;
        wx[1] += mask[p] ? d : 0.f;
        wx[2] += d * val[p] / 6.f;
        bx += d;
    }
    for (int c = 0; c < 3; ++c) wg_feature_sum(wx[c], OFF_WX + 64 * c, gpw, lds);
    wg_feature_sum(bx, OFF_BX, gpw, lds);
    float wy[3] = {0.f, 0.f, 0.f}, by = 0.f;
    for (int64_t s = blockIdx.x; s < nslices; s += gridDim.x) {
        const int w = sl_w[s];
        for (int i = wv; i < 64; i += 4) {
            const int64_t p = s * 64 + i;
            for (int k = 0; k < w; ++k) {
                const int64_t el = sl_ptr[s] + (int64_t)k * 64 + i;
                const int32_t q = sl_col[el];
                if (q == (int32_t)p || !(bf2f(e0[el * F + j]) > 0.f)) continue;
                const float d = de0[el * F + j];
                const float a = (float)(-val64[el] / sqrt(diag64[p] * diag64[q]));
                wy[0] += d * a;
                wy[1] += d * a * a;
                wy[2] += mask[q] ? d : 0.f;
                by += d;
            }
        }
    }
    for (int c = 0; c < 3; ++c) wg_feature_sum(wy[c], OFF_WY + 64 * c, gpw, lds);
    wg_feature_sum(by, OFF_BY, gpw, lds);
}

__global__ void __launch_bounds__(BLOCK) k_lpc_fill(int64_t n, float* __restrict__ x) {
    for (int64_t t = (int64_t)blockIdx.x * BLOCK + threadIdx.x; t < n; t += (int64_t)gridDim.x * BLOCK) x[t] = 0.f;
}

// grad[t] = sum over workgroup rows of gp, in row order.
__global__ void __launch_bounds__(BLOCK) k_lpc_grad_reduce(int G, const float* __restrict__ gp,
                                                            float* __restrict__ grad) {
    const int t = blockIdx.x * BLOCK + threadIdx.x;
    if (t >= N_PARAMS) return;
    double acc = 0.0;
    for (int w = 0; w < G; ++w) acc += gp[(int64_t)w * N_PARAMS + t];
    grad[t] = (float)acc;
}

// Adam (Kingma and Ba), bias-corrected, on the fp32 master parameters.
__global__ void __launch_bounds__(BLOCK) k_lpc_adam(const float* __restrict__ grad, float* __restrict__ th,
                                                     float* __restrict__ m, float* __restrict__ v, float lr,
                                                     float bc1, float bc2) {
    const int t = blockIdx.x * BLOCK + threadIdx.x;
    if (t >= N_PARAMS) return;
    const float g = grad[t];
    const float mt = 0.9f * m[t] + 0.1f * g;
    const float vt = 0.999f * v[t] + 0.001f * g * g;
    m[t] = mt;
    v[t] = vt;
    th[t] -= lr * (mt / bc1) / (sqrtf(vt / bc2) + 1e-8f);
}


// ================================================================== host side

int64_t lpc_num_params() { return N_PARAMS; }

void lpc_free_part(pgcp_part* P) {
    DevBuf* all[] = {&P->d_lpc_val, &P->d_lpc_h, &P->d_lpc_e, &P->d_lpc_oe, &P->d_lpc_ov, &P->d_mval32,
                     &P->d_mdiag32, &P->d_mval64, &P->d_mdiag64, &P->d_lpc_av, &P->d_lpc_R, &P->d_lpc_sp,
                     &P->d_lpc_piece, &P->d_lpc_c, &P->d_lpc_goe, &P->d_lpc_gov, &P->d_lpc_dh, &P->d_lpc_dhown,
                     &P->d_lpc_de0, &P->d_lpc_de1, &P->d_lpc_dx, &P->d_pc};
    for (DevBuf* b : all) dev_free(*b);
    P->spai_sys = -1;
}

static constexpr int GP_ROWS = 512;   // workgroups of the gradient kernels = rows of partial gradients

static Error lpc_pack(pgcp_lpc* L, hipStream_t s) {
    k_lpc_pack<<<256, BLOCK, 0, s>>>((const float*)L->theta.p, (bf16_t*)L->wb.p);
    HIPCHK(hipGetLastError());
    return Error{PGCP_OK, ""};
}

Error lpc_create(pgcp_ctx* ctx, const float* params, pgcp_lpc** out) {
    pgcp_lpc* L = new pgcp_lpc();
    L->device = ctx->device;
    hipStream_t s = ctx->stream;
    Error e{PGCP_OK, ""};
    auto fail = [&](Error er) {
        lpc_destroy(L);
        return er;
    };
    if ((e = dev_alloc(L->theta, N_PARAMS * 4)).code) return fail(e);
    if ((e = dev_alloc(L->adam_m, N_PARAMS * 4)).code) return fail(e);
    if ((e = dev_alloc(L->adam_v, N_PARAMS * 4)).code) return fail(e);
    if ((e = dev_alloc(L->grad, N_PARAMS * 4)).code) return fail(e);
    if ((e = dev_alloc(L->wb, (size_t)W_TOTAL * 2)).code) return fail(e);
    std::vector<float> th(N_PARAMS, 0.f);
    if (params) std::memcpy(th.data(), params, N_PARAMS * 4);
    if (hipMemcpyAsync(L->theta.p, th.data(), N_PARAMS * 4, hipMemcpyHostToDevice, s) != hipSuccess)
        return fail(Error{PGCP_E_HIP, "parameter upload failed"});
    k_lpc_fill<<<64, BLOCK, 0, s>>>(N_PARAMS, (float*)L->adam_m.p);
    k_lpc_fill<<<64, BLOCK, 0, s>>>(N_PARAMS, (float*)L->adam_v.p);
    if ((e = lpc_pack(L, s)).code) return fail(e);
    if (hipStreamSynchronize(s) != hipSuccess) return fail(Error{PGCP_E_HIP, "stream synchronise failed"});
    *out = L;
    return Error{PGCP_OK, ""};
}

// Training-state file: the magic "PGCPLPC1", int64 parameter count, int64
// Adam step, then the fp32 master parameters and Adam's first and second
// moments (each [count]), then a 64-bit FNV-1a hash of everything before it.
// Little-endian, as the device and host are.
static constexpr char kLpcMagic[8] = {'P', 'G', 'C', 'P', 'L', 'P', 'C', '1'};

static uint64_t fnv1a(const unsigned char* p, size_t n, uint64_t h = 1469598103934665603ull) {
    for (size_t i = 0; i < n; ++i) {
        h ^= p[i];
        h *= 1099511628211ull;
    }
    return h;
}

Error lpc_save(pgcp_ctx* ctx, const pgcp_lpc* L, const char* path) {
    std::vector<float> th(N_PARAMS), m(N_PARAMS), v(N_PARAMS);
    hipStream_t s = ctx->stream;
    HIPCHK(hipMemcpyAsync(th.data(), L->theta.p, N_PARAMS * 4, hipMemcpyDeviceToHost, s));
    HIPCHK(hipMemcpyAsync(m.data(), L->adam_m.p, N_PARAMS * 4, hipMemcpyDeviceToHost, s));
    HIPCHK(hipMemcpyAsync(v.data(), L->adam_v.p, N_PARAMS * 4, hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    std::vector<unsigned char> buf;
    auto put = [&](const void* p, size_t n) {
        const unsigned char* c = (const unsigned char*)p;
        buf.insert(buf.end(), c, c + n);
    };
    const int64_t n = N_PARAMS, step = L->step;
    put(kLpcMagic, 8);
    put(&n, 8);
    put(&step, 8);
    put(th.data(), N_PARAMS * 4);
    put(m.data(), N_PARAMS * 4);
    put(v.data(), N_PARAMS * 4);
    const uint64_t h = fnv1a(buf.data(), buf.size());
    put(&h, 8);
    const std::string tmp = std::string(path) + ".tmp";
    FILE* f = std::fopen(tmp.c_str(), "wb");
    if (!f) return Error{PGCP_E_INVALID, std::string("cannot open ") + tmp + " for writing"};
    const bool ok = std::fwrite(buf.data(), 1, buf.size(), f) == buf.size();
    const bool closed = std::fclose(f) == 0;
    if (!ok || !closed || std::rename(tmp.c_str(), path) != 0) {
        std::remove(tmp.c_str());
        return Error{PGCP_E_INVALID, std::string("cannot write ") + path};
    }
    return Error{PGCP_OK, ""};
}

Error lpc_load(pgcp_ctx* ctx, const char* path, pgcp_lpc** out) {
    FILE* f = std::fopen(path, "rb");
    if (!f) return Error{PGCP_E_INVALID, std::string("cannot open ") + path};
    std::vector<unsigned char> buf;
    unsigned char tmp[1 << 16];
    size_t got;
    while ((got = std::fread(tmp, 1, sizeof(tmp), f)) > 0) buf.insert(buf.end(), tmp, tmp + got);
    std::fclose(f);
    const size_t want = 24 + 3 * (size_t)N_PARAMS * 4 + 8;
    if (buf.size() != want || std::memcmp(buf.data(), kLpcMagic, 8) != 0)
        return Error{PGCP_E_INVALID, std::string(path) + " is not a training-state file of this network"};
    int64_t n = 0, step = 0;
    uint64_t h = 0;
    std::memcpy(&n, buf.data() + 8, 8);
    std::memcpy(&step, buf.data() + 16, 8);
    std::memcpy(&h, buf.data() + want - 8, 8);
    if (n != N_PARAMS || step < 0) return Error{PGCP_E_INVALID, std::string(path) + ": wrong parameter count"};
    if (fnv1a(buf.data(), want - 8) != h) return Error{PGCP_E_INVALID, std::string(path) + ": checksum mismatch"};
    const float* th = reinterpret_cast<const float*>(buf.data() + 24);
    Error e = lpc_create(ctx, th, out);
    if (e.code) return e;
    pgcp_lpc* L = *out;
    hipStream_t s = ctx->stream;
    const bool ok = hipMemcpyAsync(L->adam_m.p, th + N_PARAMS, N_PARAMS * 4, hipMemcpyHostToDevice, s) == hipSuccess &&
                    hipMemcpyAsync(L->adam_v.p, th + 2 * N_PARAMS, N_PARAMS * 4, hipMemcpyHostToDevice, s) ==
                        hipSuccess &&
                    hipStreamSynchronize(s) == hipSuccess;
    if (!ok) {
        lpc_destroy(L);
        *out = nullptr;
        return Error{PGCP_E_HIP, "optimizer state upload failed"};
    }
    L->step = step;
    return Error{PGCP_OK, ""};
}

void lpc_destroy(pgcp_lpc* L) {
    if (!L) return;
    for (DevBuf* b : {&L->theta, &L->adam_m, &L->adam_v, &L->wb, &L->grad, &L->gp}) dev_free(*b);
    delete L;
}

Error lpc_get_params(pgcp_ctx* ctx, const pgcp_lpc* L, float* out) {
    HIPCHK(hipMemcpyAsync(out, L->theta.p, N_PARAMS * 4, hipMemcpyDeviceToHost, ctx->stream));
    HIPCHK(hipStreamSynchronize(ctx->stream));
    return Error{PGCP_OK, ""};
}

static const uint8_t* system_mask(const pgcp_part* P, int system) {
    return (const uint8_t*)(system == 0 ? P->d_mask_dncp.p : P->d_mask_harm.p);
}

// Forward pass on every piece of the plan, keeping the states of all rounds
// (h_0..h_3, e_0..e_3), then the heads and the SPAI values.
static Error lpc_forward(pgcp_ctx* ctx, pgcp_part* P, const pgcp_lpc* L, int system) {
    hipStream_t s = ctx->stream;
    const int64_t N = P->N, ns = P->sell_elems;
    Error e{PGCP_OK, ""};
    if ((e = dev_alloc(P->d_lpc_val, N * 4)).code) return e;
    if ((e = dev_alloc(P->d_lpc_h, (size_t)(ROUNDS + 1) * N * F * 2)).code) return e;
    if ((e = dev_alloc(P->d_lpc_e, (size_t)(ROUNDS + 1) * ns * F * 2)).code) return e;
    if ((e = dev_alloc(P->d_lpc_oe, ns * 4)).code) return e;
    if ((e = dev_alloc(P->d_lpc_ov, N * 4)).code) return e;
    if ((e = dev_alloc(P->d_mval32, ns * 4)).code) return e;
    if ((e = dev_alloc(P->d_mval64, ns * 8)).code) return e;
    if ((e = dev_alloc(P->d_mdiag32, N * 4)).code) return e;
    if ((e = dev_alloc(P->d_mdiag64, N * 8)).code) return e;
    const uint8_t* mask = system_mask(P, system);
    const float* th = (const float*)L->theta.p;
    const bf16_t* wb = (const bf16_t*)L->wb.p;
    const bf16_t* wxy = wb + ROUNDS * W_ROUND;
    bf16_t* H = (bf16_t*)P->d_lpc_h.p;
    bf16_t* E = (bf16_t*)P->d_lpc_e.p;
    const int64_t* sl_ptr = (const int64_t*)P->d_sl_ptr.p;
    const int32_t* sl_w = (const int32_t*)P->d_sl_w.p;
    const int32_t* sl_col = (const int32_t*)P->d_sl_col.p;
    k_lpc_input_h<<<grid_for(N), BLOCK, 0, s>>>(N, sl_w, sl_ptr, sl_col, mask, wxy, th, (float*)P->d_lpc_val.p, H);
    k_lpc_input_e<<<(unsigned)P->nslices, 64, 0, s>>>(sl_ptr, sl_w, sl_col, (const double*)P->d_val64.p,
                                                       (const double*)P->d_diag64.p, mask, wxy, th, E);
    HIPCHK(hipGetLastError());
    const unsigned grid = (unsigned)std::min<int64_t>(P->nslices, 2048);
    for (int r = 0; r < ROUNDS; ++r) {
        k_lpc_round<<<grid, 256, 0, s>>>(P->nslices, sl_ptr, sl_w, sl_col, (const float*)P->d_lpc_val.p,
                                         H + (size_t)r * N * F, E + (size_t)r * ns * F, H + (size_t)(r + 1) * N * F,
                                         E + (size_t)(r + 1) * ns * F, wb + (size_t)r * W_ROUND,
                                         th + OFF_R0 + r * R_SIZE);
        HIPCHK(hipGetLastError());
    }
    k_lpc_head_e<<<grid_for(ns), BLOCK, 0, s>>>(ns, (const int32_t*)P->d_sl_rev.p, E + (size_t)ROUNDS * ns * F, th,
                                                (float*)P->d_lpc_oe.p);
    k_lpc_head_v<<<grid_for(N), BLOCK, 0, s>>>(N, H + (size_t)ROUNDS * N * F, th, (float*)P->d_lpc_ov.p);
    k_lpc_spai<<<grid_for(N), BLOCK, 0, s>>>(N, sl_ptr, sl_w, sl_col, (const double*)P->d_diag64.p, mask,
                                             (const float*)P->d_lpc_oe.p, (const float*)P->d_lpc_ov.p,
                                             (float*)P->d_mval32.p, (float*)P->d_mdiag32.p, (double*)P->d_mval64.p,
                                             (double*)P->d_mdiag64.p);
    HIPCHK(hipGetLastError());
    P->spai_sys = system;
    return Error{PGCP_OK, ""};
}

Error lpc_infer(pgcp_ctx* ctx, pgcp_part* P, const pgcp_lpc* L, int system) {
    if (!P->assembled) return Error{PGCP_E_INVALID, "pgcp_assemble_cotan has not run"};
    if (system != 0 && system != 1) return Error{PGCP_E_INVALID, "system must be 0 (DNCP) or 1 (harmonic)"};
    return lpc_forward(ctx, P, L, system);
}

Error lpc_export(pgcp_ctx* ctx, const pgcp_part* P, int piece, double* o_off, double* o_diag, double* m_off,
                 double* m_diag) {
    if (P->spai_sys < 0) return Error{PGCP_E_INVALID, "pgcp_lpc_infer has not run"};
    const int32_t r0 = P->row0[piece];
    const int32_t n = P->sub_nv[piece];
    const int64_t s0 = r0 / 64, s1 = (r0 + (int64_t)n + 63) / 64;
    const int64_t e0 = P->sl_ptr[s0], e1 = P->sl_ptr[s1];
    std::vector<float> oe(e1 - e0), ov(n);
    std::vector<double> mv(e1 - e0), md(n);
    hipStream_t s = ctx->stream;
    HIPCHK(hipMemcpyAsync(oe.data(), (const float*)P->d_lpc_oe.p + e0, (e1 - e0) * 4, hipMemcpyDeviceToHost, s));
    HIPCHK(hipMemcpyAsync(ov.data(), (const float*)P->d_lpc_ov.p + r0, (size_t)n * 4, hipMemcpyDeviceToHost, s));
    HIPCHK(hipMemcpyAsync(mv.data(), (const double*)P->d_mval64.p + e0, (e1 - e0) * 8, hipMemcpyDeviceToHost, s));
    HIPCHK(hipMemcpyAsync(md.data(), (const double*)P->d_mdiag64.p + r0, (size_t)n * 8, hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    // rows and, within a row, columns by ascending global vertex
    std::vector<int32_t> by_rank, rank_of;
    piece_global_order(P, piece, by_rank, rank_of);
    std::vector<std::pair<int32_t, int64_t>> ent;
    int64_t o = 0;
    for (int32_t t = 0; t < n; ++t) {
        const int32_t l = by_rank[t];
        const int64_t r = r0 + l, sl = r / 64;
        const int lane = (int)(r & 63);
        if (o_diag) o_diag[t] = ov[l];
        if (m_diag) m_diag[t] = md[l];
        ent.clear();
        for (int k = 0; k < P->sl_w[sl]; ++k) {
            const int64_t el = P->sl_ptr[sl] + (int64_t)k * 64 + lane;
            if (P->sl_col[el] == r) continue;
            ent.emplace_back(rank_of[P->sl_col[el] - r0], el);
        }
        std::sort(ent.begin(), ent.end());
        for (const auto& q : ent) {
            if (o_off) o_off[o] = oe[q.second - e0];
            if (m_off) m_off[o] = mv[q.second - e0];
            ++o;
        }
    }
    return Error{PGCP_OK, ""};
}

// Loss and gradient over every piece of the plan (the batch), for the given
// system's mask and probe vectors (probes [n_probes][N], zero on masked rows
// is not required: they are ignored there); optionally one Adam step.
Error lpc_grad(pgcp_ctx* ctx, pgcp_part* P, pgcp_lpc* L, int system, const float* probes, int n_probes,
               double* loss, float* grad_host, int adam, float lr) {
    if (!P->assembled) return Error{PGCP_E_INVALID, "pgcp_assemble_cotan has not run"};
    if (system != 0 && system != 1) return Error{PGCP_E_INVALID, "system must be 0 (DNCP) or 1 (harmonic)"};
    if (n_probes < 1 || n_probes > 16) return Error{PGCP_E_INVALID, "1..16 probe vectors"};
    hipStream_t s = ctx->stream;
    const int64_t N = P->N, ns = P->sell_elems;
    const int K = P->K, Pn = n_probes;
    Error e{PGCP_OK, ""};
    if ((e = lpc_forward(ctx, P, L, system)).code) return e;
    if ((e = dev_alloc(P->d_lpc_av, (size_t)Pn * N * 4)).code) return e;
    if ((e = dev_alloc(P->d_lpc_R, (size_t)Pn * N * 4)).code) return e;
    if ((e = dev_alloc(P->d_lpc_sp, (size_t)P->nslices * 2 * Pn * 8)).code) return e;
    if ((e = dev_alloc(P->d_lpc_piece, (size_t)K * 2 * Pn * 8)).code) return e;
    if ((e = dev_alloc(P->d_lpc_c, (size_t)K * Pn * 8)).code) return e;
    if ((e = dev_alloc(P->d_lpc_goe, ns * 4)).code) return e;
    if ((e = dev_alloc(P->d_lpc_gov, N * 4)).code) return e;
    if ((e = dev_alloc(P->d_lpc_dh, (size_t)N * F * 4)).code) return e;
    if ((e = dev_alloc(P->d_lpc_dhown, (size_t)N * F * 4)).code) return e;
    if ((e = dev_alloc(P->d_lpc_de0, (size_t)ns * F * 4)).code) return e;
    if ((e = dev_alloc(P->d_lpc_de1, (size_t)ns * F * 4)).code) return e;
    if ((e = dev_alloc(P->d_lpc_dx, (size_t)ns * F * 4)).code) return e;
    if ((e = dev_alloc(L->gp, (size_t)GP_ROWS * N_PARAMS * 4)).code) return e;
    const uint8_t* mask = system_mask(P, system);
    const int64_t* sl_ptr = (const int64_t*)P->d_sl_ptr.p;
    const int32_t* sl_w = (const int32_t*)P->d_sl_w.p;
    const int32_t* sl_col = (const int32_t*)P->d_sl_col.p;
    const int32_t* sl_rev = (const int32_t*)P->d_sl_rev.p;
    const double* val64 = (const double*)P->d_val64.p;
    const double* diag64 = (const double*)P->d_diag64.p;
    float* AV = (float*)P->d_lpc_av.p;
    float* R = (float*)P->d_lpc_R.p;
    // ---- loss
    k_lpc_av<<<grid_for(N), BLOCK, 0, s>>>(N, Pn, sl_ptr, sl_w, sl_col, val64, diag64, mask, probes, AV);
    k_lpc_resid<<<(unsigned)P->nslices, 64, 0, s>>>(N, Pn, sl_ptr, sl_w, sl_col, (const float*)P->d_mval32.p,
                                                     (const float*)P->d_mdiag32.p, mask, probes, AV, R,
                                                     (double*)P->d_lpc_sp.p);
    k_lpc_piece_sum<<<K, 64, 0, s>>>(Pn, (const int32_t*)P->d_row0.p, (const double*)P->d_lpc_sp.p,
                                     (double*)P->d_lpc_piece.p);
    HIPCHK(hipGetLastError());
    std::vector<double> piece((size_t)K * 2 * Pn), c((size_t)K * Pn, 0.0);
    HIPCHK(hipMemcpyAsync(piece.data(), P->d_lpc_piece.p, piece.size() * 8, hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    double total = 0.0;
    int kb = 0;
    for (int i = 0; i < K; ++i) {
        bool any = false;
        for (int k = 0; k < Pn; ++k) any |= piece[((size_t)i * Pn + k) * 2 + 1] > 0.0;
        kb += any ? 1 : 0;
    }
    if (kb == 0) return Error{PGCP_E_INVALID, "probe vectors vanish on every free row"};
    for (int i = 0; i < K; ++i)
        for (int k = 0; k < Pn; ++k) {
            const double r2 = piece[((size_t)i * Pn + k) * 2], v2 = piece[((size_t)i * Pn + k) * 2 + 1];
            if (v2 > 0.0) {
                total += r2 / v2 / Pn;
                c[(size_t)i * Pn + k] = 2.0 / ((double)kb * Pn * v2);
            }
        }
    if (loss) *loss = total / kb;
    if (!grad_host && !adam) return Error{PGCP_OK, ""};
    HIPCHK(hipMemcpyAsync(P->d_lpc_c.p, c.data(), c.size() * 8, hipMemcpyHostToDevice, s));
    // ---- output gradients and heads
    k_lpc_outgrad<<<grid_for(N), BLOCK, 0, s>>>(N, Pn, (const int32_t*)P->d_slice_sub.p, sl_ptr, sl_w, sl_col, diag64,
                                                mask, AV, R, (const double*)P->d_lpc_c.p,
                                                (const float*)P->d_lpc_oe.p, (const float*)P->d_lpc_ov.p,
                                                (float*)P->d_lpc_goe.p, (float*)P->d_lpc_gov.p);
    k_lpc_fill<<<1024, BLOCK, 0, s>>>((int64_t)GP_ROWS * N_PARAMS, (float*)L->gp.p);
    HIPCHK(hipGetLastError());
    const bf16_t* H = (const bf16_t*)P->d_lpc_h.p;
    const bf16_t* E = (const bf16_t*)P->d_lpc_e.p;
    const float* th = (const float*)L->theta.p;
    const bf16_t* wb = (const bf16_t*)L->wb.p;
    float* dh = (float*)P->d_lpc_dh.p;
    float* dhown = (float*)P->d_lpc_dhown.p;
    float* de_cur = (float*)P->d_lpc_de0.p;
    float* de_next = (float*)P->d_lpc_de1.p;
    float* dx = (float*)P->d_lpc_dx.p;
    float* gp = (float*)L->gp.p;
    k_lpc_head_bwd<<<GP_ROWS, 256, 0, s>>>(N, ns, sl_rev, E + (size_t)ROUNDS * ns * F, H + (size_t)ROUNDS * N * F,
                                           (const float*)P->d_lpc_goe.p, (const float*)P->d_lpc_gov.p, th, de_cur, dh,
                                           gp);
    HIPCHK(hipGetLastError());
    // ---- rounds, last to first
    const unsigned grid = (unsigned)std::min<int64_t>(P->nslices, GP_ROWS);
    for (int r = ROUNDS - 1; r >= 0; --r) {
        k_lpc_round_bwd<<<grid, 256, 0, s>>>(P->nslices, sl_ptr, sl_w, sl_col, (const float*)P->d_lpc_val.p,
                                             H + (size_t)r * N * F, E + (size_t)r * ns * F, H + (size_t)(r + 1) * N * F,
                                             E + (size_t)(r + 1) * ns * F, dh, de_cur, wb + (size_t)r * W_ROUND, r,
                                             dhown, dx, de_next, gp);
        HIPCHK(hipGetLastError());
        k_lpc_gather<<<grid_for(N * F), BLOCK, 0, s>>>(N, sl_ptr, sl_w, sl_rev, dhown, dx, dh);
        HIPCHK(hipGetLastError());
        std::swap(de_cur, de_next);
    }
    k_lpc_input_bwd<<<GP_ROWS, 256, 0, s>>>(N, P->nslices, sl_ptr, sl_w, sl_col, val64, diag64, mask,
                                            (const float*)P->d_lpc_val.p, H, E, dh, de_cur, gp);
    k_lpc_grad_reduce<<<grid_for(N_PARAMS), BLOCK, 0, s>>>(GP_ROWS, gp, (float*)L->grad.p);
    HIPCHK(hipGetLastError());
    if (adam) {
        L->step++;
        const float bc1 = 1.f - std::pow(0.9f, (float)L->step), bc2 = 1.f - std::pow(0.999f, (float)L->step);
        k_lpc_adam<<<grid_for(N_PARAMS), BLOCK, 0, s>>>((const float*)L->grad.p, (float*)L->theta.p,
                                                         (float*)L->adam_m.p, (float*)L->adam_v.p, lr, bc1, bc2);
        HIPCHK(hipGetLastError());
        if ((e = lpc_pack(L, s)).code) return e;
        P->spai_sys = -1;   // the plan's SPAI values belong to the old parameters
    }
    if (grad_host) {
        HIPCHK(hipMemcpyAsync(grad_host, L->grad.p, N_PARAMS * 4, hipMemcpyDeviceToHost, s));
    }
    HIPCHK(hipStreamSynchronize(s));
    return Error{PGCP_OK, ""};
}

}  // namespace pgcp
