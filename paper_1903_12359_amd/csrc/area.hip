// Area distortion of a parameterization and its reduction by a Moebius map
// (Section 6, area distortion).
//
// d_area(T) = log A(f(T)) - log A(T) - (log sum A(f) - log sum A), with A the
// area of the flat triangle through the face's three points.  One evaluation
// of the objective (mean |d_area| of X composed with a Moebius map) is two
// passes over the faces: the image areas with the map applied to each corner
// on the fly (their logs kept, block sums of the areas), then the block sums
// of |d_area| against the device-side totals.  Block sums are added in a fixed
// order by one workgroup, so an evaluation is bitwise reproducible.  The
// search over the map's parameters (Nelder-Mead) runs on the host, one
// objective evaluation on the device per step.
#include <algorithm>
#include <cmath>
#include <limits>
#include <numeric>
#include <vector>

#include "device_util.h"
#include "pgcp_internal.h"

#define HIPTHROW(x)                                                                     \
    do {                                                                               \
        hipError_t _e = (x);                                                           \
        if (_e != hipSuccess) throw Error{PGCP_E_HIP, std::string(#x) + ": " + hipGetErrorString(_e)}; \
    } while (0)

namespace pgcp {
namespace {

// (a z + b) / (c z + d); the disk automorphism (z - alpha)/(1 - conj(alpha) z)
// is a = d = 1, b = -alpha, c = -conj(alpha).
struct Mob {
    double ar, ai, br, bi, cr, ci, dr, di;
};

// Image of parameter point v under the mode's map.  Sphere: stereographic
// projection sigma(p) = (x - i y)/(1 - z) = (1 + z)/(x + i y), taken as a
// homogeneous pair P:Q (the first form on the southern half, the second on the
// northern, so one member of the pair is at least 1 in size), mapped to
// P':Q' = (a P + b Q):(c P + d Q) and back by
// sigma^-1 = (2 Re(P' conj Q'), -2 Im(P' conj Q'), |P'|^2 - |Q'|^2)/(|P'|^2 + |Q'|^2),
// so the north pole (infinity) needs no special case.
__device__ __forceinline__ void image(const double* __restrict__ X, int64_t v, int sphere, const Mob& m, double& x,
                                      double& y, double& z) {
    if (sphere) {
        const double px = X[3 * v], py = X[3 * v + 1], pz = X[3 * v + 2];
        double Pr, Pi, Qr, Qi;
        if (pz <= 0.0) {
            Pr = px; Pi = -py; Qr = 1.0 - pz; Qi = 0.0;
        } else {
            Pr = 1.0 + pz; Pi = 0.0; Qr = px; Qi = py;
        }
        const double p2r = m.ar * Pr - m.ai * Pi + m.br * Qr - m.bi * Qi;
        const double p2i = m.ar * Pi + m.ai * Pr + m.br * Qi + m.bi * Qr;
        const double q2r = m.cr * Pr - m.ci * Pi + m.dr * Qr - m.di * Qi;
        const double q2i = m.cr * Pi + m.ci * Pr + m.dr * Qi + m.di * Qr;
        const double re = p2r * q2r + p2i * q2i, im = p2i * q2r - p2r * q2i;
        const double np2 = p2r * p2r + p2i * p2i, nq2 = q2r * q2r + q2i * q2i;
        const double s = 1.0 / (np2 + nq2);
        x = 2.0 * re * s;
        y = -2.0 * im * s;
        z = (np2 - nq2) * s;
    } else {
        const double zr = X[2 * v], zi = X[2 * v + 1];
        const double nr = m.ar * zr - m.ai * zi + m.br, ni = m.ar * zi + m.ai * zr + m.bi;
        const double er = m.cr * zr - m.ci * zi + m.dr, ei = m.cr * zi + m.ci * zr + m.di;
        const double den = er * er + ei * ei;
        x = (nr * er + ni * ei) / den;
        y = (ni * er - nr * ei) / den;
        z = 0.0;
    }
}

__device__ __forceinline__ double tri_area(double ax, double ay, double az, double bx, double by, double bz,
                                           double cx, double cy, double cz) {
    const double ux = bx - ax, uy = by - ay, uz = bz - az, vx = cx - ax, vy = cy - ay, vz = cz - az;
    const double wx = uy * vz - uz * vy, wy = uz * vx - ux * vz, wz = ux * vy - uy * vx;
    return 0.5 * sqrt(wx * wx + wy * wy + wz * wz);
}

// Sum of one value per thread over the workgroup (fixed tree), written by thread 0.
__device__ __forceinline__ void block_sum(double v, double* out) {
    __shared__ double sh[BLOCK];
    sh[threadIdx.x] = v;
    __syncthreads();
    for (int w = BLOCK / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) *out = sh[0];
}

__global__ void __launch_bounds__(BLOCK) k_area_src(int64_t nf, const double* __restrict__ V,
                                                    const int32_t* __restrict__ F, double* __restrict__ logA,
                                                    double* __restrict__ part, int* __restrict__ bad) {
    const int64_t t = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
    double a = 0.0;
    if (t < nf) {
        const int64_t i = F[3 * t], j = F[3 * t + 1], k = F[3 * t + 2];
        a = tri_area(V[3 * i], V[3 * i + 1], V[3 * i + 2], V[3 * j], V[3 * j + 1], V[3 * j + 2], V[3 * k],
                     V[3 * k + 1], V[3 * k + 2]);
        if (!(a > 0.0) || !isfinite(a)) atomicOr(bad, 1);
        logA[t] = log(a);
    }
    block_sum(a, part + blockIdx.x);
}

// Orientation of a face's three points: the signed area (times 2) in the
// plane, det[a, b, c] for points on the sphere (positive for a face seen
// counter-clockwise from outside).
__device__ __forceinline__ double orient(const double* p, int sphere) {
    if (sphere)
        return p[0] * (p[4] * p[8] - p[5] * p[7]) - p[1] * (p[3] * p[8] - p[5] * p[6]) +
               p[2] * (p[3] * p[7] - p[4] * p[6]);
    return (p[3] - p[0]) * (p[7] - p[1]) - (p[4] - p[1]) * (p[6] - p[0]);
}

// A face is inadmissible when its image area is zero or not finite, or when
// the map reverses its orientation (a Moebius map preserves orientation where
// it is finite, so a reversal means its pole lies inside the face).
__global__ void __launch_bounds__(BLOCK) k_area_img(int64_t nf, const double* __restrict__ X, int sphere, Mob m,
                                                    const int32_t* __restrict__ F, double* __restrict__ logAf,
                                                    double* __restrict__ part, int* __restrict__ bad) {
    const int64_t t = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
    double a = 0.0;
    if (t < nf) {
        double p[9], q[9];
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const int64_t v = F[3 * t + c];
            image(X, v, sphere, m, p[3 * c], p[3 * c + 1], p[3 * c + 2]);
            q[3 * c] = X[(sphere ? 3 : 2) * v];
            q[3 * c + 1] = X[(sphere ? 3 : 2) * v + 1];
            q[3 * c + 2] = sphere ? X[3 * v + 2] : 0.0;
        }
        a = tri_area(p[0], p[1], p[2], p[3], p[4], p[5], p[6], p[7], p[8]);
        const double turn = orient(p, sphere) * orient(q, sphere);
        if (!(a > 0.0) || !isfinite(a) || !(turn > 0.0)) {
            atomicOr(bad, 1);
            a = 0.0;
        }
        logAf[t] = log(a);
    }
    block_sum(a, part + blockIdx.x);
}

// tot[0] = sum A, tot[1] = sum A(f)
__global__ void __launch_bounds__(BLOCK) k_area_abs(int64_t nf, const double* __restrict__ logAf,
                                                    const double* __restrict__ logA, const double* __restrict__ tot,
                                                    double* __restrict__ d, double* __restrict__ part) {
    const int64_t t = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
    const double c = log(tot[1]) - log(tot[0]);
    double v = 0.0;
    if (t < nf) {
        const double dt = logAf[t] - logA[t] - c;
        if (d) d[t] = dt;
        v = fabs(dt);
    }
    block_sum(v, part + blockIdx.x);
}

// out[0] = sum of part[0..n) in a fixed order (one workgroup); clears *clear
// (the flag the next evaluation will set) when given
__global__ void __launch_bounds__(BLOCK) k_area_sum(int64_t n, const double* __restrict__ part,
                                                    double* __restrict__ out, int* __restrict__ clear) {
    double v = 0.0;
    for (int64_t i = threadIdx.x; i < n; i += BLOCK) v += part[i];
    block_sum(v, out);
    if (clear && threadIdx.x == 0) *clear = 0;
}

__global__ void __launch_bounds__(BLOCK) k_area_apply(int64_t nv, const double* __restrict__ X, int sphere, Mob m,
                                                      double* __restrict__ Y) {
    const int64_t v = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
    if (v >= nv) return;
    double x, y, z;
    image(X, v, sphere, m, x, y, z);
    if (sphere) {
        Y[3 * v] = x; Y[3 * v + 1] = y; Y[3 * v + 2] = z;
    } else {
        Y[2 * v] = x; Y[2 * v + 1] = y;
    }
}

Mob make_mob(int mode, const double* p) {
    if (mode == PGCP_DISK) return Mob{1.0, 0.0, -p[0], -p[1], -p[0], p[1], 1.0, 0.0};
    return Mob{p[0], p[1], p[2], p[3], p[4], p[5], p[6], p[7]};
}

bool admissible(int mode, const double* p) {
    if (mode == PGCP_DISK) return p[0] * p[0] + p[1] * p[1] < 1.0;
    const double dr = p[0] * p[6] - p[1] * p[7] - (p[2] * p[4] - p[3] * p[5]);
    const double di = p[0] * p[7] + p[1] * p[6] - (p[2] * p[5] + p[3] * p[4]);
    return dr != 0.0 || di != 0.0;
}

// Device state of one area computation on one mesh.  stat holds the totals
// (sum A, sum A(f), sum |d_area|) and two bad-area flags: evaluation k sets
// flag k % 2 and its last kernel clears the other, so no evaluation needs a
// separate clear, and one copy brings totals and flag back.
struct Stat {
    double tot[3];
    int bad[2];
};

struct AreaWork {
    pgcp_ctx* ctx;
    int64_t nf, nblk, k = 0;
    const double* X;
    const int32_t* F;
    int sphere;
    DevBuf logA, logAf, part, statb;
    Error init(pgcp_ctx* c, const double* V, const int32_t* Fd, int64_t n, const double* Xd, int sph) {
        ctx = c; nf = n; F = Fd; X = Xd; sphere = sph;
        nblk = (nf + BLOCK - 1) / BLOCK;
        Error e{PGCP_OK, ""};
        if ((e = dev_alloc(logA, nf * 8)).code) return e;
        if ((e = dev_alloc(logAf, nf * 8)).code) return e;
        if ((e = dev_alloc(part, nblk * 8)).code) return e;
        if ((e = dev_alloc(statb, sizeof(Stat))).code) return e;
        hipStream_t s = ctx->stream;
        Stat* st = (Stat*)statb.p;
        HIPCHK(hipMemsetAsync(statb.p, 0, sizeof(Stat), s));
        k_area_src<<<(unsigned)nblk, BLOCK, 0, s>>>(nf, V, F, (double*)logA.p, (double*)part.p, &st->bad[0]);
        k_area_sum<<<1, BLOCK, 0, s>>>(nblk, (const double*)part.p, &st->tot[0], &st->bad[1]);
        HIPCHK(hipGetLastError());
        Stat h;
        HIPCHK(hipMemcpyAsync(&h, statb.p, sizeof(Stat), hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
        k = 1;
        if (h.bad[0]) return Error{PGCP_E_DEGENERATE, "zero-area or non-finite triangle in the original mesh"};
        return e;
    }
    // mean |d_area| of X composed with m (+inf when an image area is zero or not
    // finite, or a face's orientation is reversed); d [nf] optional
    Error eval(const Mob& m, double* d, double* value) {
        hipStream_t s = ctx->stream;
        Stat* st = (Stat*)statb.p;
        const int slot = (int)(k & 1);
        k_area_img<<<(unsigned)nblk, BLOCK, 0, s>>>(nf, X, sphere, m, F, (double*)logAf.p, (double*)part.p,
                                                    &st->bad[slot]);
        k_area_sum<<<1, BLOCK, 0, s>>>(nblk, (const double*)part.p, &st->tot[1], nullptr);
        k_area_abs<<<(unsigned)nblk, BLOCK, 0, s>>>(nf, (const double*)logAf.p, (const double*)logA.p,
                                                    st->tot, d, (double*)part.p);
        k_area_sum<<<1, BLOCK, 0, s>>>(nblk, (const double*)part.p, &st->tot[2], &st->bad[slot ^ 1]);
        HIPCHK(hipGetLastError());
        Stat h;
        HIPCHK(hipMemcpyAsync(&h, statb.p, sizeof(Stat), hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
        ++k;
        const double v = h.tot[2] / (double)nf;
        *value = (h.bad[slot] || !std::isfinite(v)) ? std::numeric_limits<double>::infinity() : v;
        return Error{PGCP_OK, ""};
    }
    void release() {
        for (DevBuf* b : {&logA, &logAf, &part, &statb}) dev_free(*b);
    }
};

}  // namespace

Error run_area_distortion(pgcp_ctx* ctx, const double* V, const int32_t* F, int64_t nf, const double* X, int dim,
                          double* d, double* mean_abs) {
    AreaWork W;
    Error e = W.init(ctx, V, F, nf, X, dim == 3);
    const double id[8] = {1, 0, 0, 0, 0, 0, 1, 0};
    if (!e.code) e = W.eval(make_mob(PGCP_FREE, id), d, mean_abs);
    W.release();
    return e;
}

Error run_area_objective(pgcp_ctx* ctx, const double* V, const int32_t* F, int64_t nf, const double* X, int mode,
                         const double* params, double* value) {
    AreaWork W;
    Error e = W.init(ctx, V, F, nf, X, mode == PGCP_SPHERE);
    if (!e.code) {
        if (admissible(mode, params)) e = W.eval(make_mob(mode, params), nullptr, value);
        else *value = std::numeric_limits<double>::infinity();
    }
    W.release();
    return e;
}

// Nelder-Mead from the identity map (Nelder and Mead 1965; reflection 1,
// expansion 2, contraction 1/2, shrink 1/2), initial simplex of step 0.1
// along each parameter, stopped when the simplex's values lie within fatol
// and its points within xatol (max norm) of the best, or after max_evals
// evaluations.
Error run_area_mobius_opt(pgcp_ctx* ctx, const double* V, int64_t nv, const int32_t* F, int64_t nf, const double* X,
                          int mode, int max_evals, double* params, double* before, double* after, int32_t* n_evals,
                          double* Y) {
    const int n = mode == PGCP_DISK ? 2 : 8;
    const double fatol = 1e-12, xatol = 1e-10;
    AreaWork W;
    Error e = W.init(ctx, V, F, nf, X, mode == PGCP_SPHERE);
    int evals = 0;
    auto f = [&](const std::vector<double>& p) -> double {
        ++evals;
        if (!admissible(mode, p.data())) return std::numeric_limits<double>::infinity();
        double v = 0.0;
        Error r = W.eval(make_mob(mode, p.data()), nullptr, &v);
        if (r.code) throw r;
        return v;
    };
    try {
        if (e.code) throw e;
        std::vector<std::vector<double>> x(n + 1, std::vector<double>(n, 0.0));
        if (mode != PGCP_DISK) x[0][0] = x[0][6] = 1.0;
        for (int i = 1; i <= n; ++i) {
            x[i] = x[0];
            x[i][i - 1] += 0.1;
        }
        std::vector<double> fx(n + 1);
        for (int i = 0; i <= n; ++i) fx[i] = f(x[i]);
        *before = fx[0];
        std::vector<int> ord(n + 1);
        std::vector<double> xc(n), xr(n), xe(n), xk(n);
        while (evals < max_evals) {
            std::iota(ord.begin(), ord.end(), 0);
            std::stable_sort(ord.begin(), ord.end(), [&](int a, int b) { return fx[a] < fx[b]; });
            std::vector<std::vector<double>> xs(n + 1);
            std::vector<double> fs(n + 1);
            for (int i = 0; i <= n; ++i) {
                xs[i] = x[ord[i]];
                fs[i] = fx[ord[i]];
            }
            x.swap(xs);
            fx.swap(fs);
            double df = 0.0, dx = 0.0;
            for (int i = 1; i <= n; ++i) {
                df = std::max(df, std::fabs(fx[i] - fx[0]));
                for (int j = 0; j < n; ++j) dx = std::max(dx, std::fabs(x[i][j] - x[0][j]));
            }
            if (std::isfinite(fx[n]) && df <= fatol && dx <= xatol) break;
            for (int j = 0; j < n; ++j) {
                xc[j] = 0.0;
                for (int i = 0; i < n; ++i) xc[j] += x[i][j];
                xc[j] /= n;
                xr[j] = 2.0 * xc[j] - x[n][j];
            }
            const double fr = f(xr);
            if (fr < fx[0]) {
                for (int j = 0; j < n; ++j) xe[j] = 3.0 * xc[j] - 2.0 * x[n][j];
                const double fe = f(xe);
                if (fe < fr) { x[n] = xe; fx[n] = fe; }
                else { x[n] = xr; fx[n] = fr; }
                continue;
            }
            if (fr < fx[n - 1]) {
                x[n] = xr;
                fx[n] = fr;
                continue;
            }
            bool shrink;
            if (fr < fx[n]) {   // outside contraction
                for (int j = 0; j < n; ++j) xk[j] = 1.5 * xc[j] - 0.5 * x[n][j];
                const double fk = f(xk);
                shrink = !(fk <= fr);
                if (!shrink) { x[n] = xk; fx[n] = fk; }
            } else {            // inside contraction
                for (int j = 0; j < n; ++j) xk[j] = 0.5 * xc[j] + 0.5 * x[n][j];
                const double fk = f(xk);
                shrink = !(fk < fx[n]);
                if (!shrink) { x[n] = xk; fx[n] = fk; }
            }
            if (shrink)
                for (int i = 1; i <= n; ++i) {
                    for (int j = 0; j < n; ++j) x[i][j] = x[0][j] + 0.5 * (x[i][j] - x[0][j]);
                    fx[i] = f(x[i]);
                }
        }
        int best = (int)(std::min_element(fx.begin(), fx.end()) - fx.begin());
        for (int j = 0; j < n; ++j) params[j] = x[best][j];
        *after = fx[best];
        if (n_evals) *n_evals = evals;
        if (Y) {
            k_area_apply<<<grid_for(nv), BLOCK, 0, ctx->stream>>>(nv, X, mode == PGCP_SPHERE,
                                                                  make_mob(mode, params), Y);
            HIPTHROW(hipGetLastError());
            HIPTHROW(hipStreamSynchronize(ctx->stream));
        }
    } catch (const Error& err) {
        W.release();
        return err;
    }
    W.release();
    return Error{PGCP_OK, ""};
}

}  // namespace pgcp
