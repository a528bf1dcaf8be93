// Partial welding with the point replay on the GPU (Sections 3.4, 4.3, 4.4).
//
// Every map of a weld is fixed by its shared arc (see weld_maps.h): the host
// runs the zipper on the arcs of every pair of a round (O(k^2) per pair, pairs
// in parallel), records the map parameters, and then one kernel sends every
// other point of the round through its pair's recorded chain
//     z -> Moebius(close(zip_side(z)))
// one thread per point.  Points inside a welded union ("tracked": earlier
// seams) have one coordinate each and stay on the device, indexed by seam
// slot, for the whole weld.  Loop points keep one coordinate per component
// until they are glued (a vertex on the boundary between two components has a
// coordinate in each plane), so the non-arc loop points of a round are
// uploaded, replayed by the same kernel and read back for the next round's
// arcs.  The disk step replays tracked points through the geodesic chain of
// the outer loop and the Cayley map.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <cmath>
#include <limits>
#include <vector>

#include "device_util.h"
#include "pgcp_internal.h"
#include "weld_maps.h"

namespace pgcp {

using namespace weldmaps;

namespace {

#define HIPTHROW(x)                                                                     \
    do {                                                                               \
        hipError_t _e = (x);                                                           \
        if (_e != hipSuccess) throw Error{PGCP_E_HIP, std::string(#x) + ": " + hipGetErrorString(_e)}; \
    } while (0)

// ------------------------------------------------------------------ device maps (same branches as the host replay)

struct DZ {
    double x, y;
    bool inf;
};

__device__ __forceinline__ DZ dz(double x, double y, bool inf = false) { return DZ{x, y, inf}; }
__device__ __forceinline__ void cmul(double ax, double ay, double bx, double by, double& rx, double& ry) {
    rx = ax * bx - ay * by;
    ry = ax * by + ay * bx;
}
__device__ __forceinline__ void cdiv(double ax, double ay, double bx, double by, double& rx, double& ry) {
    const double den = bx * bx + by * by;
    rx = (ax * bx + ay * by) / den;
    ry = (ay * bx - ax * by) / den;
}
__device__ __forceinline__ void csqrtp(double x, double y, double& rx, double& ry) {
    const double r = sqrt(x * x + y * y);
    if (r == 0.0) {
        rx = 0.0;
        ry = y;
        return;
    }
    if (x >= 0.0) {
        const double t = sqrt(0.5 * (r + x));
        rx = t;
        ry = y / (2.0 * t);
    } else {
        const double t = sqrt(0.5 * (r - x));
        rx = fabs(y) / (2.0 * t);
        ry = copysign(t, y);
    }
}

// zip record: k, z0, z1, zeta, zeta_inf, squared, c[k-1], d[k-1]
__device__ DZ d_zip(const double* __restrict__ R, DZ p) {
    const int k = (int)R[0];
    const double z0x = R[1], z0y = R[2], z1x = R[3], z1y = R[4], zex = R[5], zey = R[6];
    const bool zeta_inf = R[7] != 0.0, squared = R[8] != 0.0;
    const double* c = R + 9;
    const double* d = R + 9 + (k - 1);
    if (p.inf) {
        p = dz(1.0, 0.0);
    } else {
        const double dx = p.x - z0x, dy = p.y - z0y;
        if (dx == 0.0 && dy == 0.0) {
            p = dz(0.0, 0.0, true);
        } else {
            double qx, qy;
            cdiv(p.x - z1x, p.y - z1y, dx, dy, qx, qy);
            csqrtp(qx, qy, p.x, p.y);
        }
    }
    for (int j = 0; j + 2 <= k; ++j) {
        const double cj = c[j], dj = d[j];
        if (p.inf) {
            if (dj != 0.0) p = dz(0.0, -cj / dj);
            else continue;
        } else {
            // L = c z / (1 + i d z)
            const double denx = 1.0 - dj * p.y, deny = dj * p.x;
            if (denx == 0.0 && deny == 0.0) {
                p = dz(0.0, 0.0, true);
                continue;
            }
            double lx, ly;
            cdiv(cj * p.x, cj * p.y, denx, deny, lx, ly);
            p.x = lx;
            p.y = ly;
        }
        double sx, sy;
        cmul(p.x, p.y, p.x, p.y, sx, sy);
        csqrtp(sx - 1.0, sy, p.x, p.y);
    }
    if (p.inf) {
        if (zeta_inf) return p;
        p = dz(-zex, -zey);
    } else if (!zeta_inf) {
        double qx, qy;
        cdiv(p.x, p.y, zex, zey, qx, qy);
        const double denx = 1.0 - qx, deny = -qy;
        if (denx == 0.0 && deny == 0.0) return dz(0.0, 0.0, true);
        double rx, ry;
        cdiv(p.x, p.y, denx, deny, rx, ry);
        p.x = rx;
        p.y = ry;
    }
    if (squared) {
        double sx, sy;
        cmul(p.x, p.y, p.x, p.y, sx, sy);
        p.x = sx;
        p.y = sy;
    }
    return p;
}

// close record: n, eta, eta_inf, c0[n], c1[n]
__device__ DZ d_close(const double* __restrict__ R, DZ p) {
    const int n = (int)R[0];
    const double etx = R[1], ety = R[2];
    const bool eta_inf = R[3] != 0.0;
    const double* c0 = R + 4;
    const double* c1 = R + 4 + n;
    for (int t = 0; t < n; ++t) {
        // T(z) = z / (c0 - i c1 z); T(inf) = i / c1
        if (p.inf) {
            if (c1[t] != 0.0) p = dz(0.0, 1.0 / c1[t]);
            else continue;
        } else {
            const double denx = c0[t] + c1[t] * p.y, deny = -c1[t] * p.x;
            if (denx == 0.0 && deny == 0.0) {
                p = dz(0.0, 0.0, true);
                continue;
            }
            double tx, ty;
            cdiv(p.x, p.y, denx, deny, tx, ty);
            p.x = tx;
            p.y = ty;
        }
        double sx, sy;
        cmul(p.x, p.y, p.x, p.y, sx, sy);
        csqrtp(sx + 1.0, sy, p.x, p.y);
    }
    // h_0
    if (eta_inf) {
        if (p.inf) return p;
        double sx, sy;
        cmul(p.x, p.y, p.x, p.y, sx, sy);
        return dz(sx, sy);
    }
    if (p.inf) {
        double sx, sy;
        cmul(etx, ety, etx, ety, sx, sy);
        return dz(sx, sy);
    }
    double qx, qy;
    cdiv(p.x, p.y, etx, ety, qx, qy);
    const double denx = 1.0 - qx, deny = -qy;
    if (denx == 0.0 && deny == 0.0) return dz(0.0, 0.0, true);
    double wx, wy;
    cdiv(p.x, p.y, denx, deny, wx, wy);
    double sx, sy;
    cmul(wx, wy, wx, wy, sx, sy);
    return dz(sx, sy);
}

// Moebius record: a, b, c, d
__device__ DZ d_mobius(const double* __restrict__ M, DZ p) {
    if (p.inf) {
        double rx, ry;
        cdiv(M[0], M[1], M[4], M[5], rx, ry);
        return dz(rx, ry);
    }
    double nx, ny, dx, dy;
    cmul(M[0], M[1], p.x, p.y, nx, ny);
    nx += M[2];
    ny += M[3];
    cmul(M[4], M[5], p.x, p.y, dx, dy);
    dx += M[6];
    dy += M[7];
    if (dx == 0.0 && dy == 0.0) return dz(0.0, 0.0, true);
    double rx, ry;
    cdiv(nx, ny, dx, dy, rx, ry);
    return dz(rx, ry);
}

__device__ DZ d_cayley(DZ p) {
    if (p.inf) return dz(1.0, 0.0);
    double rx, ry;
    cdiv(p.x, p.y - 1.0, p.x, p.y + 1.0, rx, ry);
    return dz(rx, ry);
}

// Per pair: offsets of the side-A and side-B zip records, of the close record
// and of the Moebius record (-1: absent), and 1 for the Cayley map at the end.
struct PairDesc {
    int64_t zip[2], close, mob;
    int64_t cayley;
};

// Points: uidx < n_seam addresses the tracked array, otherwise the round's
// uploaded loop points; pair; side (0 = A, 1 = B).
__global__ void __launch_bounds__(BLOCK) k_weld_replay(int64_t npts, const int32_t* __restrict__ pts,
                                                        const PairDesc* __restrict__ desc,
                                                        const double* __restrict__ rec, int64_t n_seam,
                                                        double2* __restrict__ zt, double2* __restrict__ ztmp) {
    const int64_t t = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
    if (t >= npts) return;
    const int64_t u = pts[3 * t];
    const PairDesc D = desc[pts[3 * t + 1]];
    const int side = pts[3 * t + 2];
    double2* slot = u < n_seam ? zt + u : ztmp + (u - n_seam);
    const double2 v = *slot;
    DZ p = isinf(v.x) ? dz(0.0, 0.0, true) : dz(v.x, v.y);
    p = d_zip(rec + D.zip[side], p);
    if (D.close >= 0) p = d_close(rec + D.close, p);
    if (D.mob >= 0) p = d_mobius(rec + D.mob, p);
    if (D.cayley) p = d_cayley(p);
    const double inf = __builtin_inf();
    *slot = p.inf ? make_double2(inf, inf) : make_double2(p.x, p.y);
}

__global__ void __launch_bounds__(BLOCK) k_weld_scatter(int64_t n, const int32_t* __restrict__ slot,
                                                         const double2* __restrict__ val, double2* __restrict__ zt) {
    const int64_t t = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
    if (t < n) zt[slot[t]] = val[t];
}

// ------------------------------------------------------------------ zipper and closing on the device
//
// Algorithms 1 and 2 on the arcs themselves.  One workgroup per job: the two
// arcs of a pair (A with branch +1, B with branch -1) are zipped and then
// closed; or, for the disk step, one arc is zipped with the squared final map.
// Every thread keeps PPT arc points in registers (in LDS for arcs of more than
// 4096 points).  Step j of either algorithm
// needs the current value of one arc point per arc: the thread that holds it
// publishes it in LDS (two alternating slots, so one barrier per step), and
// every thread then derives the same step parameters and updates its points.
// The branches are those of the host zip_arc / close_arcs (weld_maps.h); the
// records are written in the layout the replay kernel reads.

struct ZipJob {
    int64_t pt;    // first arc point (pair: A[0..k], then B[0..k])
    int64_t rec;   // first double of the job's records (zip A[, zip B, close])
    int32_t k;
    int32_t pair;
};

enum : int { ZE_OK = 0, ZE_ARC_INF, ZE_HALFPLANE, ZE_POST, ZE_GLUE_INF, ZE_GLUE_DEG, ZE_GLUE_ORDER };

__device__ __forceinline__ void axis_point(double s, double& x, double& y) {   // glued pair image: sqrt(s^2 - 1) branch
    if (fabs(s) <= 1.0) {
        x = sqrt(1.0 - s * s);
        y = 0.0;
    } else {
        x = 0.0;
        y = (s > 0.0 ? 1.0 : -1.0) * sqrt(s * s - 1.0);
    }
}

template <int BLK, int PPT, bool LDS>
__global__ void __launch_bounds__(BLK) k_zip_arcs(const ZipJob* __restrict__ jobs, double2* __restrict__ pts,
                                                   double* __restrict__ rec, int* __restrict__ err) {
    const ZipJob J = jobs[blockIdx.x];
    const int k = J.k;
    const int ns = J.pair ? 2 : 1;
    const int np = ns * (k + 1);
    const bool squared = !J.pair;
    double2* __restrict__ P = pts + J.pt;
    double* __restrict__ R = rec + J.rec;
    const int nzr = 9 + 2 * (k - 1);   // doubles of one zip record
    __shared__ double bx[2][2], by[2][2];
    __shared__ int binf[2][2];
    __shared__ double gy[2][2];
    __shared__ int ginf[2][2];
    __shared__ double ex, ey;
    __shared__ int einf;
    __shared__ int s_err;
    const int tid = threadIdx.x;
    if (tid == 0) s_err = 0;

    // g_1 of each arc: z -> sqrt((z - z1) / (z - z0))
    double z0x[2] = {0.0, 0.0}, z0y[2] = {0.0, 0.0}, z1x[2] = {0.0, 0.0}, z1y[2] = {0.0, 0.0};
    for (int s = 0; s < ns; ++s) {
        const double2 a = P[s * (k + 1)], b = P[s * (k + 1) + 1];
        if (isinf(a.x) || isinf(b.x)) {
            if (tid == 0) err[blockIdx.x] = ZE_ARC_INF;
            return;   // uniform: every thread read the same points
        }
        z0x[s] = a.x;
        z0y[s] = a.y;
        z1x[s] = b.x;
        z1y[s] = b.y;
    }
    if (tid == 0) {
        for (int s = 0; s < ns; ++s) {
            double* Z = R + s * nzr;
            Z[0] = (double)k;
            Z[1] = z0x[s];
            Z[2] = z0y[s];
            Z[3] = z1x[s];
            Z[4] = z1y[s];
            Z[8] = squared ? 1.0 : 0.0;
        }
    }
    // the thread's points: registers, or (long arcs) LDS
    double rx[PPT], ry[PPT];
    unsigned char rinf[PPT];
    __shared__ double lx[LDS ? BLK * PPT : 1], ly[LDS ? BLK * PPT : 1];
    __shared__ unsigned char linf[LDS ? BLK * PPT : 1];
    auto X = [&](int i) -> double& {
        if constexpr (LDS) return lx[tid + i * BLK];
        else return rx[i];
    };
    auto Y = [&](int i) -> double& {
        if constexpr (LDS) return ly[tid + i * BLK];
        else return ry[i];
    };
    auto INF = [&](int i) -> unsigned char& {
        if constexpr (LDS) return linf[tid + i * BLK];
        else return rinf[i];
    };
#pragma unroll
    for (int i = 0; i < PPT; ++i) {
        const int m = tid + i * BLK;
        X(i) = Y(i) = 0.0;
        INF(i) = 0;
        if (m >= np) continue;
        const int s = m > k ? 1 : 0;
        const int l = m - s * (k + 1);
        if (l == 0) {
            INF(i) = 1;
        } else if (l >= 2) {
            const double2 v = P[m];
            if (isinf(v.x)) {
                X(i) = 1.0;
            } else {
                double qx, qy;
                cdiv(v.x - (s ? z1x[1] : z1x[0]), v.y - (s ? z1y[1] : z1y[0]), v.x - (s ? z0x[1] : z0x[0]),
                     v.y - (s ? z0y[1] : z0y[0]), qx, qy);
                csqrtp(qx, qy, X(i), Y(i));
            }
        }
    }
    // Algorithm 1, steps j = 2..k
    for (int j = 2; j <= k; ++j) {
        const int par = j & 1;
#pragma unroll
        for (int i = 0; i < PPT; ++i) {
            const int m = tid + i * BLK;
            const int s = m > k ? 1 : 0;
            if (m < np && m - s * (k + 1) == j) {
                bx[s][par] = X(i);
                by[s][par] = Y(i);
                binf[s][par] = INF(i);
            }
        }
        __syncthreads();
        double cs[2], ds[2];
        bool bad = false;
        for (int s = 0; s < ns; ++s) {
            const double xr = bx[s][par], xq = by[s][par];
            if (binf[s][par] || !(xr > 0.0)) bad = true;
            const double r2 = xr * xr + xq * xq;
            cs[s] = xr / r2;
            ds[s] = xq / r2;
        }
        if (bad) {
            if (tid == 0) err[blockIdx.x] = ZE_HALFPLANE;
            return;   // uniform
        }
        if (tid == 0) {
            for (int s = 0; s < ns; ++s) {
                R[s * nzr + 9 + (j - 2)] = cs[s];
                R[s * nzr + 9 + (k - 1) + (j - 2)] = ds[s];
            }
        }
#pragma unroll
        for (int i = 0; i < PPT; ++i) {
            const int m = tid + i * BLK;
            if (m >= np) continue;
            const int s = m > k ? 1 : 0;
            const int l = m - s * (k + 1);
            const double c = s ? cs[1] : cs[0], d = s ? ds[1] : ds[0];
            if (l == j - 1) {
                X(i) = 0.0;
                Y(i) = s ? -1.0 : 1.0;
                INF(i) = 0;
            } else if (l == j) {
                X(i) = Y(i) = 0.0;
                INF(i) = 0;
            } else if (l < j - 1) {
                // zipped: z = i t, L = i c t / (1 - d t)
                if (INF(i)) {
                    if (d == 0.0) continue;
                    const double q = -c / d;
                    X(i) = 0.0;
                    Y(i) = (q > 0 ? 1.0 : -1.0) * sqrt(q * q + 1.0);
                    INF(i) = 0;
                    continue;
                }
                const double t = Y(i), den = 1.0 - d * t;
                if (den == 0.0) {
                    X(i) = Y(i) = 0.0;
                    INF(i) = 1;
                    continue;
                }
                const double q = c * t / den;
                const double sg = (q > 0.0) ? 1.0 : (q < 0.0 ? -1.0 : 0.0);
                X(i) = 0.0;
                Y(i) = sg * sqrt(q * q + 1.0);
            } else {
                // not yet zipped: L = c z / (1 + i d z), then sqrt(L^2 - 1)
                double lx, ly;
                if (INF(i)) {
                    if (d == 0.0) continue;
                    lx = 0.0;
                    ly = -c / d;
                } else {
                    const double denx = 1.0 - d * Y(i), deny = d * X(i);
                    if (denx == 0.0 && deny == 0.0) {
                        X(i) = Y(i) = 0.0;
                        INF(i) = 1;
                        continue;
                    }
                    cdiv(c * X(i), c * Y(i), denx, deny, lx, ly);
                }
                double sx, sy;
                cmul(lx, ly, lx, ly, sx, sy);
                csqrtp(sx - 1.0, sy, X(i), Y(i));
                INF(i) = 0;
            }
        }
    }
    // final map z / (1 - z / zeta), imaginary part (squared for the disk step)
    const int pz = (k + 1) & 1;
#pragma unroll
    for (int i = 0; i < PPT; ++i) {
        const int m = tid + i * BLK;
        const int s = m > k ? 1 : 0;
        if (m < np && m - s * (k + 1) == 0) {
            bx[s][pz] = X(i);
            by[s][pz] = Y(i);
            binf[s][pz] = INF(i);
        }
    }
    __syncthreads();
    double zx[2], zy[2];
    bool zinf[2];
    for (int s = 0; s < ns; ++s) {
        zx[s] = bx[s][pz];
        zy[s] = by[s][pz];
        zinf[s] = binf[s][pz] != 0;
    }
    if (tid == 0) {
        for (int s = 0; s < ns; ++s) {
            R[s * nzr + 5] = zx[s];
            R[s * nzr + 6] = zy[s];
            R[s * nzr + 7] = zinf[s] ? 1.0 : 0.0;
        }
    }
    bool post_bad = false;
#pragma unroll
    for (int i = 0; i < PPT; ++i) {
        const int m = tid + i * BLK;
        if (m >= np) continue;
        const int s = m > k ? 1 : 0;
        const int l = m - s * (k + 1);
        if (l == 0) {
            X(i) = Y(i) = 0.0;
            INF(i) = 1;
            continue;
        }
        INF(i) = 0;
        if (l == k) {
            X(i) = Y(i) = 0.0;
            continue;
        }
        double wx = X(i), wy = Y(i);
        if (!(s ? zinf[1] : zinf[0])) {
            double qx, qy;
            cdiv(X(i), Y(i), s ? zx[1] : zx[0], s ? zy[1] : zy[0], qx, qy);
            cdiv(X(i), Y(i), 1.0 - qx, -qy, wx, wy);
        }
        X(i) = 0.0;
        Y(i) = wy;
        if (squared) {
            double sx, sy;
            cmul(0.0, wy, 0.0, wy, sx, sy);
            X(i) = sx;
            Y(i) = sy;
        } else if (!((s ? -1.0 : 1.0) * wy > 0.0)) {
            post_bad = true;
        }
    }
    if (post_bad) atomicOr(&s_err, 1);
    __syncthreads();
    if (s_err) {
        if (tid == 0) err[blockIdx.x] = ZE_POST;
        return;   // uniform
    }
    if (J.pair) {
        // Algorithm 2: glue the pairs (A[j], B[j]) for j = k-1..1, then h_0
        double* RC = R + 2 * nzr;   // n, eta, eta_inf, c0[n], c1[n] with n = k - 1
        if (tid == 0) RC[0] = (double)(k - 1);
        for (int j = k - 1; j >= 1; --j) {
            const int par = j & 1;
#pragma unroll
            for (int i = 0; i < PPT; ++i) {
                const int m = tid + i * BLK;
                const int s = m > k ? 1 : 0;
                if (m < np && m - s * (k + 1) == j) {
                    gy[s][par] = Y(i);
                    ginf[s][par] = INF(i);
                }
            }
            __syncthreads();
            int code = ZE_OK;
            const double a = gy[0][par], b = gy[1][par];
            if (ginf[0][par] || ginf[1][par]) code = ZE_GLUE_INF;
            else if (a == 0.0 || b == 0.0 || a == b) code = ZE_GLUE_DEG;
            const double c0 = -2.0 * a * b / (a - b), c1 = (a + b) / (a - b);
            if (code == ZE_OK && !(c0 > 0.0)) code = ZE_GLUE_ORDER;
            if (code != ZE_OK) {
                if (tid == 0) err[blockIdx.x] = code;
                return;   // uniform
            }
            if (tid == 0) {
                RC[4 + (k - 1 - j)] = c0;
                RC[4 + (k - 1) + (k - 1 - j)] = c1;
            }
#pragma unroll
            for (int i = 0; i < PPT; ++i) {
                const int m = tid + i * BLK;
                if (m >= np) continue;
                const int s = m > k ? 1 : 0;
                const int l = m - s * (k + 1);
                if (l == j) {
                    X(i) = Y(i) = 0.0;
                    INF(i) = 0;
                    continue;
                }
                if (l < j && !INF(i)) {
                    // unglued arc point on the imaginary axis: T(i u) = i u / (c0 + c1 u)
                    const double u = Y(i), den = c0 + c1 * u;
                    if (den == 0.0) {
                        X(i) = Y(i) = 0.0;
                        INF(i) = 1;
                        continue;
                    }
                    axis_point(u / den, X(i), Y(i));
                    continue;
                }
                // T(z) = z / (c0 - i c1 z); T(inf) = i / c1
                double tx, ty;
                if (INF(i)) {
                    if (c1 == 0.0) continue;
                    tx = 0.0;
                    ty = 1.0 / c1;
                } else {
                    const double denx = c0 + c1 * Y(i), deny = -c1 * X(i);
                    if (denx == 0.0 && deny == 0.0) {
                        X(i) = Y(i) = 0.0;
                        INF(i) = 1;
                        continue;
                    }
                    cdiv(X(i), Y(i), denx, deny, tx, ty);
                }
                INF(i) = 0;
                if (l < j) {
                    axis_point(ty, X(i), Y(i));
                } else {
                    double sx, sy;
                    cmul(tx, ty, tx, ty, sx, sy);
                    csqrtp(sx + 1.0, sy, X(i), Y(i));
                }
            }
        }
        // h_0(z) = (z / (1 - z / eta))^2 with eta the image of A[0]
#pragma unroll
        for (int i = 0; i < PPT; ++i) {
            if (tid + i * BLK == 0) {
                ex = X(i);
                ey = Y(i);
                einf = INF(i);
            }
        }
        __syncthreads();
        const double etx = ex, ety = ey;
        const bool eta_inf = einf != 0;
        if (tid == 0) {
            RC[1] = etx;
            RC[2] = ety;
            RC[3] = eta_inf ? 1.0 : 0.0;
        }
#pragma unroll
        for (int i = 0; i < PPT; ++i) {
            const int m = tid + i * BLK;
            if (m >= np) continue;
            const int s = m > k ? 1 : 0;
            const int l = m - s * (k + 1);
            if (l == 0) {
                X(i) = Y(i) = 0.0;
                INF(i) = 1;
                continue;
            }
            double sx, sy;
            if (eta_inf) {
                if (INF(i)) continue;
                cmul(X(i), Y(i), X(i), Y(i), sx, sy);
            } else if (INF(i)) {
                cmul(etx, ety, etx, ety, sx, sy);
            } else {
                double qx, qy, wx, wy;
                cdiv(X(i), Y(i), etx, ety, qx, qy);
                const double denx = 1.0 - qx, deny = -qy;
                if (denx == 0.0 && deny == 0.0) {
                    X(i) = Y(i) = 0.0;
                    INF(i) = 1;
                    continue;
                }
                cdiv(X(i), Y(i), denx, deny, wx, wy);
                cmul(wx, wy, wx, wy, sx, sy);
            }
            X(i) = sx;
            Y(i) = sy;
            INF(i) = 0;
        }
    }
    const double dinf = __builtin_inf();
#pragma unroll
    for (int i = 0; i < PPT; ++i) {
        const int m = tid + i * BLK;
        if (m < np) P[m] = INF(i) ? make_double2(dinf, dinf) : make_double2(X(i), Y(i));
    }
    if (tid == 0) err[blockIdx.x] = ZE_OK;
}

// ------------------------------------------------------------------ host side

struct DComp {
    std::vector<int> outer;
    std::vector<EP> zo;
    std::vector<int32_t> tslot;   // seam slots of the tracked points
};

void put_zip(std::vector<double>& r, const ZipRecord& Z) {
    r.push_back((double)Z.k);
    r.push_back(Z.z0.real());
    r.push_back(Z.z0.imag());
    r.push_back(Z.z1.real());
    r.push_back(Z.z1.imag());
    r.push_back(Z.zeta.real());
    r.push_back(Z.zeta.imag());
    r.push_back(Z.zeta_inf ? 1.0 : 0.0);
    r.push_back(Z.squared ? 1.0 : 0.0);
    r.insert(r.end(), Z.c.begin(), Z.c.end());
    r.insert(r.end(), Z.d.begin(), Z.d.end());
}
void put_close(std::vector<double>& r, const CloseRecord& C) {
    r.push_back((double)C.c0.size());
    r.push_back(C.eta.real());
    r.push_back(C.eta.imag());
    r.push_back(C.eta_inf ? 1.0 : 0.0);
    r.insert(r.end(), C.c0.begin(), C.c0.end());
    r.insert(r.end(), C.c1.begin(), C.c1.end());
}
void put_mobius(std::vector<double>& r, const Mobius& M) {
    for (const cplx& v : {M.a, M.b, M.c, M.d}) {
        r.push_back(v.real());
        r.push_back(v.imag());
    }
}
inline double2 to_d2(const EP& p) {
    const double inf = std::numeric_limits<double>::infinity();
    return p.inf ? make_double2(inf, inf) : make_double2(p.z.real(), p.z.imag());
}
inline EP from_d2(const double2& v) { return std::isinf(v.x) ? EP{0.0, true} : EP{cplx(v.x, v.y), false}; }

// One weld: its arcs, records and the new component's structure.
struct Job {
    ZipRecord ZA, ZB;
    CloseRecord CR;
    Mobius M;
    DComp C;
    std::vector<EP> restA, restB;   // non-arc loop points (replayed on the device)
    std::vector<int32_t> arc_slot;  // arc points that become tracked, and their values
    std::vector<EP> arc_val;
    int na_rest = 0, nb_rest = 0;
    EP a_k, a_0;
    bool closed = false;
    int k = 0;
    std::vector<int> Aid, Bid;       // loops of A and B from the arc's start
    std::vector<EP> arcA, arcB;      // arc points; after the zipper and closing, their images
    bool on_device = false;
};

// Arcs of one weld and the loop points around them (O(loop length)).
Job weld_prep(const DComp& A, const DComp& B, bool closed) {
    Job J;
    J.closed = closed;
    int start, k;
    const int La = (int)A.outer.size(), Lb = (int)B.outer.size();
    if (closed) {
        if (La != Lb) throw Error{PGCP_E_WELD, "closed weld of loops of different length"};
        start = (int)(std::min_element(A.outer.begin(), A.outer.end()) - A.outer.begin());
        k = La - 1;
    } else {
        k = shared_arc(A.outer, B.outer, &start);
        if (k < 2) throw Error{PGCP_E_WELD, "components do not share one contiguous arc"};
    }
    J.k = k;
    std::vector<int>& Aid = J.Aid;
    std::vector<int>& Bid = J.Bid;
    Aid.resize(La);
    Bid.resize(Lb);
    std::vector<EP> Az(La), Bz(Lb);
    for (int s = 0; s < La; ++s) {
        Aid[s] = A.outer[(start + s) % La];
        Az[s] = A.zo[(start + s) % La];
    }
    const int i0 = (int)(std::find(B.outer.begin(), B.outer.end(), Aid[0]) - B.outer.begin());
    if (i0 >= Lb) throw Error{PGCP_E_WELD, "arc correspondence broken"};
    for (int s = 0; s < Lb; ++s) {
        const int t = ((i0 - s) % Lb + Lb) % Lb;
        Bid[s] = B.outer[t];
        Bz[s] = B.zo[t];
    }
    for (int s = 0; s <= k; ++s)
        if (Aid[s] != Bid[s]) throw Error{PGCP_E_WELD, "arc correspondence broken"};
    J.arcA.assign(Az.begin(), Az.begin() + k + 1);
    J.arcB.assign(Bz.begin(), Bz.begin() + k + 1);
    J.na_rest = La - k - 1;
    J.nb_rest = Lb - k - 1;
    J.restA.assign(Az.begin() + k + 1, Az.end());
    J.restB.assign(Bz.begin() + k + 1, Bz.end());
    return J;
}

// Algorithms 1 and 2 on the host, for a weld the device does not take.
void weld_arcs_host(Job& J) {
    J.ZA = zip_arc(J.arcA, J.k, +1, false);
    J.ZB = zip_arc(J.arcB, J.k, -1, false);
    J.CR = close_arcs(J.arcA, J.arcB, J.k);
}

// Normalisation and the new component, from the records and the arc images.
void weld_finish(Job& J, const DComp& A, const DComp& B, const std::vector<int32_t>& slot_of) {
    const int k = J.k;
    // auxiliary points 0 and infinity of both sides fix the normalisation
    const EP a0 = close_point(J.CR, zip_point(J.ZA, EP{0.0, false}));
    const EP ai = close_point(J.CR, zip_point(J.ZA, EP{0.0, true}));
    const EP b0 = close_point(J.CR, zip_point(J.ZB, EP{0.0, false}));
    const EP bi = close_point(J.CR, zip_point(J.ZB, EP{0.0, true}));
    if (a0.inf || b0.inf || ai.inf || bi.inf) throw Error{PGCP_E_WELD, "auxiliary point sent to infinity"};
    J.M = mobius3(a0.z, b0.z, 0.5 * (ai.z + bi.z));
    for (auto& p : J.arcA) p = mobius_apply(J.M, p);
    if (!J.closed) {
        J.C.outer.reserve(J.na_rest + J.nb_rest + 2);
        J.C.outer.push_back(J.Aid[k]);
        for (int s = 0; s < J.na_rest; ++s) J.C.outer.push_back(J.Aid[k + 1 + s]);
        J.C.outer.push_back(J.Aid[0]);
        for (int s = J.nb_rest - 1; s >= 0; --s) J.C.outer.push_back(J.Bid[k + 1 + s]);
        J.a_k = J.arcA[k];
        J.a_0 = J.arcA[0];
        for (int s = 1; s < k; ++s) {
            J.arc_slot.push_back(slot_of[J.Aid[s]]);
            J.arc_val.push_back(J.arcA[s]);
        }
    } else {
        for (int s = 0; s <= k; ++s) {
            J.arc_slot.push_back(slot_of[J.Aid[s]]);
            J.arc_val.push_back(J.arcA[s]);
        }
    }
    J.C.tslot = A.tslot;
    J.C.tslot.insert(J.C.tslot.end(), B.tslot.begin(), B.tslot.end());
    J.C.tslot.insert(J.C.tslot.end(), J.arc_slot.begin(), J.arc_slot.end());
}

ZipRecord get_zip(const double* r) {
    ZipRecord Z;
    Z.k = (int)r[0];
    Z.z0 = cplx(r[1], r[2]);
    Z.z1 = cplx(r[3], r[4]);
    Z.zeta = cplx(r[5], r[6]);
    Z.zeta_inf = r[7] != 0.0;
    Z.squared = r[8] != 0.0;
    Z.c.assign(r + 9, r + 9 + (Z.k - 1));
    Z.d.assign(r + 9 + (Z.k - 1), r + 9 + 2 * (Z.k - 1));
    return Z;
}

CloseRecord get_close(const double* r, int k) {
    CloseRecord C;
    C.k = k;
    const int n = (int)r[0];
    C.eta = cplx(r[1], r[2]);
    C.eta_inf = r[3] != 0.0;
    C.c0.assign(r + 4, r + 4 + n);
    C.c1.assign(r + 4 + n, r + 4 + 2 * n);
    return C;
}

// Largest job (arc points of both sides) the device zipper takes; longer arcs
// run on the host.
constexpr int ZIP_DEVICE_MAX = 8192;

// One arc job for the device: a pair (b != nullptr: zipped, then closed) or a
// single arc (zipped with the squared final map).
struct ArcTask {
    std::vector<EP>* a;
    std::vector<EP>* b;
    int k;
    ZipRecord* za;
    ZipRecord* zb;
    CloseRecord* cr;
};

// PGCP_ZIP=host runs every zipper on the host, PGCP_ZIP=lds every device zipper
// with the LDS-resident points (both for tests of each path on small meshes).
int zip_mode() {
    const char* v = getenv("PGCP_ZIP");
    if (v && !strcmp(v, "host")) return 1;
    if (v && !strcmp(v, "lds")) return 2;
    return 0;
}

bool device_takes(int k, bool pair) {
    return zip_mode() != 1 && k >= 2 && (pair ? 2 : 1) * (k + 1) <= ZIP_DEVICE_MAX;
}

const char* zip_error(int code) {
    switch (code) {
    case ZE_ARC_INF: return "arc point at infinity";
    case ZE_HALFPLANE: return "zipper point left the right half-plane";
    case ZE_POST: return "Algorithm 1 postcondition failed";
    case ZE_GLUE_INF: return "glued pair at infinity";
    case ZE_GLUE_DEG: return "degenerate glued pair";
    case ZE_GLUE_ORDER: return "glued pair out of cyclic order";
    default: return "device zipper did not finish";
    }
}

// Runs the tasks on the device (one workgroup each), replaces their arc points
// by the images and fills their records.
void device_arcs(hipStream_t s, const std::vector<ArcTask>& tasks, DevBuf& bj, DevBuf& bp, DevBuf& br,
                 DevBuf& be) {
    if (tasks.empty()) return;
    std::vector<ZipJob> zj(tasks.size());
    std::vector<double2> pts;
    int64_t nrec = 0;
    int maxnp = 0;
    for (size_t t = 0; t < tasks.size(); ++t) {
        const ArcTask& T = tasks[t];
        const bool pair = T.b != nullptr;
        if (!device_takes(T.k, pair)) throw Error{PGCP_E_WELD, "arc job too long for the device zipper"};
        zj[t] = ZipJob{(int64_t)pts.size(), nrec, T.k, pair ? 1 : 0};
        for (int l = 0; l <= T.k; ++l) pts.push_back(to_d2((*T.a)[l]));
        if (pair)
            for (int l = 0; l <= T.k; ++l) pts.push_back(to_d2((*T.b)[l]));
        const int64_t nz = 9 + 2 * (int64_t)(T.k - 1);
        nrec += pair ? 2 * nz + 4 + 2 * (int64_t)(T.k - 1) : nz;
        maxnp = std::max(maxnp, (pair ? 2 : 1) * (T.k + 1));
    }
    Error e{PGCP_OK, ""};
    if ((e = upload(bj, zj, s)).code) throw e;
    if ((e = upload(bp, pts, s)).code) throw e;
    if ((e = dev_alloc(br, (size_t)nrec * 8)).code) throw e;
    if ((e = dev_alloc(be, tasks.size() * 4)).code) throw e;
    // -1 marks a job whose workgroup did not report
    HIPTHROW(hipMemsetAsync(be.p, 0xff, tasks.size() * 4, s));
    const unsigned g = (unsigned)tasks.size();
    const ZipJob* J = (const ZipJob*)bj.p;
    double2* P = (double2*)bp.p;
    double* R = (double*)br.p;
    int* E = (int*)be.p;
    // 256-thread workgroups up to 2048 points: four waves of at most 256
    // registers fit beside a batched-CG workgroup of another context's solve
    // (1024-thread ones were ~20% faster per step alone but waited for it)
    if (zip_mode() == 2) k_zip_arcs<1024, 8, true><<<g, 1024, 0, s>>>(J, P, R, E);
    else if (maxnp <= 256) k_zip_arcs<256, 1, false><<<g, 256, 0, s>>>(J, P, R, E);
    else if (maxnp <= 512) k_zip_arcs<256, 2, false><<<g, 256, 0, s>>>(J, P, R, E);
    else if (maxnp <= 1024) k_zip_arcs<256, 4, false><<<g, 256, 0, s>>>(J, P, R, E);
    else if (maxnp <= 2048) k_zip_arcs<256, 8, false><<<g, 256, 0, s>>>(J, P, R, E);
    else if (maxnp <= 4096) k_zip_arcs<1024, 4, false><<<g, 1024, 0, s>>>(J, P, R, E);
    else k_zip_arcs<1024, 8, true><<<g, 1024, 0, s>>>(J, P, R, E);
    HIPTHROW(hipGetLastError());
    std::vector<double> rec(nrec);
    std::vector<int> err(tasks.size());
    HIPTHROW(hipMemcpyAsync(pts.data(), bp.p, pts.size() * 16, hipMemcpyDeviceToHost, s));
    HIPTHROW(hipMemcpyAsync(rec.data(), br.p, (size_t)nrec * 8, hipMemcpyDeviceToHost, s));
    HIPTHROW(hipMemcpyAsync(err.data(), be.p, tasks.size() * 4, hipMemcpyDeviceToHost, s));
    HIPTHROW(hipStreamSynchronize(s));
    for (size_t t = 0; t < tasks.size(); ++t) {
        const ArcTask& T = tasks[t];
        if (err[t] != ZE_OK) throw Error{PGCP_E_WELD, zip_error(err[t])};
        const int64_t p0 = zj[t].pt, r0 = zj[t].rec;
        for (int l = 0; l <= T.k; ++l) (*T.a)[l] = from_d2(pts[p0 + l]);
        *T.za = get_zip(rec.data() + r0);
        if (T.b) {
            for (int l = 0; l <= T.k; ++l) (*T.b)[l] = from_d2(pts[p0 + T.k + 1 + l]);
            const int64_t nz = 9 + 2 * (int64_t)(T.k - 1);
            *T.zb = get_zip(rec.data() + r0 + nz);
            *T.cr = get_close(rec.data() + r0 + 2 * nz, T.k);
        }
    }
}

}  // namespace

Error weld_all_device(pgcp_ctx* ctx, pgcp_part* P, const double* bdy_uv, double* welded_uv) {
    hipStream_t s = ctx->stream;
    const int K = P->K;
    const int64_t ns = P->n_seam;
    DevBuf zt, ztmp, recb, descb, ptsb, sslot, sval, zjob, zpts, zrec, zerr;
    auto release = [&]() {
        for (DevBuf* b : {&zt, &ztmp, &recb, &descb, &ptsb, &sslot, &sval, &zjob, &zpts, &zrec, &zerr}) dev_free(*b);
    };
    const char* vb = getenv("PGCP_VERBOSE");
    const bool verbose = vb && vb[0] == '1';
    auto now = [] { return std::chrono::steady_clock::now(); };
    auto ms = [](std::chrono::steady_clock::time_point a, std::chrono::steady_clock::time_point b) {
        return std::chrono::duration<double, std::milli>(b - a).count();
    };
    const auto t_start = now();
    double t_arcs = 0.0;
    try {
        std::vector<int32_t> slot_of(P->nv, -1);
        for (int64_t t = 0; t < ns; ++t) slot_of[P->seam_gv[t]] = (int32_t)t;
        Error e{PGCP_OK, ""};
        if ((e = dev_alloc(zt, (size_t)std::max<int64_t>(ns, 1) * 16)).code) throw e;
        std::vector<DComp> comps(K);
        std::vector<char> alive(K, 1);
        for (int i = 0; i < K; ++i) {
            const int e0 = P->loop_ptr[i], e1 = P->loop_ptr[i + 1];
            comps[i].outer.assign(P->loop_gv.begin() + e0, P->loop_gv.begin() + e1);
            comps[i].zo.resize(e1 - e0);
            for (int t = e0; t < e1; ++t) comps[i].zo[t - e0] = EP{cplx(bdy_uv[2 * t], bdy_uv[2 * t + 1]), false};
        }
        const int nrounds = (int)P->weld_rounds.size();
        // upload (slot, value) pairs and scatter them into the tracked array
        auto scatter = [&](const std::vector<int32_t>& sl, const std::vector<double2>& v) -> Error {
            if (sl.empty()) return Error{PGCP_OK, ""};
            Error er{PGCP_OK, ""};
            if ((er = upload(sslot, sl, s)).code) return er;
            if ((er = upload(sval, v, s)).code) return er;
            k_weld_scatter<<<grid_for((int64_t)sl.size()), BLOCK, 0, s>>>((int64_t)sl.size(),
                                                                          (const int32_t*)sslot.p,
                                                                          (const double2*)sval.p, (double2*)zt.p);
            HIPTHROW(hipGetLastError());
            return Error{PGCP_OK, ""};
        };
        for (int r = 0; r < nrounds; ++r) {
            const auto& rnd = P->weld_rounds[r];
            const bool closed = P->mode == PGCP_SPHERE && r == nrounds - 1;
            std::vector<Job> jobs(rnd.size());
            const auto t_r0 = now();
            // arcs of every pair; pairs whose arcs fit go to the device zipper
            std::vector<ArcTask> tasks;
            bool any_host = false;
            for (size_t t = 0; t < rnd.size(); ++t) {
                Job& J = jobs[t];
                J = weld_prep(comps[rnd[t].first], comps[rnd[t].second], closed);
                J.on_device = device_takes(J.k, true);
                if (J.on_device) tasks.push_back(ArcTask{&J.arcA, &J.arcB, J.k, &J.ZA, &J.ZB, &J.CR});
                else any_host = true;
            }
            device_arcs(s, tasks, zjob, zpts, zrec, zerr);
            std::vector<Error> errs(rnd.size(), Error{PGCP_OK, ""});
#pragma omp parallel for schedule(dynamic) if (any_host && rnd.size() > 1)
            for (size_t t = 0; t < rnd.size(); ++t) {
                try {
                    if (!jobs[t].on_device) weld_arcs_host(jobs[t]);
                    weld_finish(jobs[t], comps[rnd[t].first], comps[rnd[t].second], slot_of);
                } catch (const Error& er) {
                    errs[t] = er;
                }
            }
            for (auto& er : errs)
                if (er.code != PGCP_OK) throw er;
            t_arcs += ms(t_r0, now());
            if (verbose) {
                int kmax = 0;
                for (const Job& J : jobs) kmax = std::max(kmax, J.k);
                fprintf(stderr, "[pgcp] weld round %d: %zu pairs (%zu on the device), longest arc %d, arcs %.2f ms\n",
                        r, rnd.size(), tasks.size(), kmax, ms(t_r0, now()));
            }
            // pack the records and the point list of the round
            std::vector<double> rec;
            std::vector<PairDesc> desc(rnd.size());
            std::vector<int32_t> pts;
            std::vector<double2> tmp;
            for (size_t t = 0; t < rnd.size(); ++t) {
                Job& J = jobs[t];
                desc[t].zip[0] = (int64_t)rec.size();
                put_zip(rec, J.ZA);
                desc[t].zip[1] = (int64_t)rec.size();
                put_zip(rec, J.ZB);
                desc[t].close = (int64_t)rec.size();
                put_close(rec, J.CR);
                desc[t].mob = (int64_t)rec.size();
                put_mobius(rec, J.M);
                desc[t].cayley = 0;
                const DComp& A = comps[rnd[t].first];
                const DComp& B = comps[rnd[t].second];
                for (int32_t sl : A.tslot) pts.insert(pts.end(), {sl, (int32_t)t, 0});
                for (int32_t sl : B.tslot) pts.insert(pts.end(), {sl, (int32_t)t, 1});
                for (const EP& p : J.restA) {
                    pts.insert(pts.end(), {(int32_t)(ns + (int64_t)tmp.size()), (int32_t)t, 0});
                    tmp.push_back(to_d2(p));
                }
                for (const EP& p : J.restB) {
                    pts.insert(pts.end(), {(int32_t)(ns + (int64_t)tmp.size()), (int32_t)t, 1});
                    tmp.push_back(to_d2(p));
                }
            }
            if (ns + (int64_t)tmp.size() > INT32_MAX) throw Error{PGCP_E_INVALID, "weld point index overflow"};
            const int64_t npts = (int64_t)pts.size() / 3;
            if ((e = upload(recb, rec, s)).code) throw e;
            if ((e = upload(descb, desc, s)).code) throw e;
            if ((e = upload(ptsb, pts, s)).code) throw e;
            if ((e = upload(ztmp, tmp, s)).code) throw e;
            if (npts > 0) {
                k_weld_replay<<<grid_for(npts), BLOCK, 0, s>>>(npts, (const int32_t*)ptsb.p,
                                                               (const PairDesc*)descb.p, (const double*)recb.p, ns,
                                                               (double2*)zt.p, (double2*)ztmp.p);
                HIPTHROW(hipGetLastError());
            }
            // arc points of this round become tracked points with their final values
            std::vector<int32_t> asl;
            std::vector<double2> aval;
            for (const Job& J : jobs)
                for (size_t u = 0; u < J.arc_slot.size(); ++u) {
                    asl.push_back(J.arc_slot[u]);
                    aval.push_back(to_d2(J.arc_val[u]));
                }
            if ((e = scatter(asl, aval)).code) throw e;
            if (!tmp.empty())
                HIPTHROW(hipMemcpyAsync(tmp.data(), ztmp.p, tmp.size() * 16, hipMemcpyDeviceToHost, s));
            HIPTHROW(hipStreamSynchronize(s));
            // new components: loop coordinates from the replayed points
            size_t off = 0;
            for (size_t t = 0; t < rnd.size(); ++t) {
                Job& J = jobs[t];
                std::vector<EP> ra(J.na_rest), rb(J.nb_rest);
                for (int u = 0; u < J.na_rest; ++u) ra[u] = from_d2(tmp[off++]);
                for (int u = 0; u < J.nb_rest; ++u) rb[u] = from_d2(tmp[off++]);
                if (!J.closed) {
                    J.C.zo.reserve(J.C.outer.size());
                    J.C.zo.push_back(J.a_k);
                    for (int u = 0; u < J.na_rest; ++u) J.C.zo.push_back(ra[u]);
                    J.C.zo.push_back(J.a_0);
                    for (int u = J.nb_rest - 1; u >= 0; --u) J.C.zo.push_back(rb[u]);
                }
                comps[rnd[t].first] = std::move(J.C);
                comps[rnd[t].second] = DComp();
                alive[rnd[t].second] = 0;
            }
        }
        int last = -1, nlive = 0;
        for (int i = 0; i < K; ++i)
            if (alive[i]) {
                last = i;
                nlive++;
            }
        if (nlive != 1) throw Error{PGCP_E_WELD, "weld plan did not finish"};
        DComp& C = comps[last];
        if (P->mode == PGCP_DISK) {
            // geodesic algorithm on the outer loop (squared final map), then Cayley
            const int L = (int)C.outer.size();
            const int st = (int)(std::min_element(C.outer.begin(), C.outer.end()) - C.outer.begin());
            std::vector<int> id(L);
            std::vector<EP> arc(L);
            for (int u = 0; u < L; ++u) {
                id[u] = C.outer[(st + u) % L];
                arc[u] = C.zo[(st + u) % L];
            }
            ZipRecord Z;
            const auto t_d0 = now();
            if (device_takes(L - 1, false)) {
                device_arcs(s, {ArcTask{&arc, nullptr, L - 1, &Z, nullptr, nullptr}}, zjob, zpts, zrec, zerr);
            } else {
                Z = zip_arc(arc, L - 1, +1, true);
            }
            t_arcs += ms(t_d0, now());
            std::vector<double> rec;
            put_zip(rec, Z);
            std::vector<PairDesc> desc(1);
            desc[0].zip[0] = desc[0].zip[1] = 0;
            desc[0].close = -1;
            desc[0].mob = -1;
            desc[0].cayley = 1;
            std::vector<int32_t> pts;
            for (int32_t sl : C.tslot) pts.insert(pts.end(), {sl, 0, 0});
            const int64_t npts = (int64_t)pts.size() / 3;
            if (npts > 0) {
                if ((e = upload(recb, rec, s)).code) throw e;
                if ((e = upload(descb, desc, s)).code) throw e;
                if ((e = upload(ptsb, pts, s)).code) throw e;
                k_weld_replay<<<grid_for(npts), BLOCK, 0, s>>>(npts, (const int32_t*)ptsb.p,
                                                               (const PairDesc*)descb.p, (const double*)recb.p, ns,
                                                               (double2*)zt.p, (double2*)zt.p);
                HIPTHROW(hipGetLastError());
            }
            for (int u = 0; u < L; ++u) {
                const EP& p = arc[u];
                arc[u] = p.inf ? EP{1.0, false}
                               : EP{(p.z - cplx(0.0, 1.0)) / (p.z + cplx(0.0, 1.0)), false};
            }
            C.outer = id;
            C.zo = arc;
            HIPTHROW(hipStreamSynchronize(s));
        }
        std::vector<int32_t> osl;
        std::vector<double2> oval;
        for (size_t u = 0; u < C.outer.size(); ++u) {
            osl.push_back(slot_of[C.outer[u]]);
            oval.push_back(to_d2(C.zo[u]));
        }
        if ((e = scatter(osl, oval)).code) throw e;
        // every seam vertex must have been written exactly once: tracked + outer
        if ((int64_t)(C.tslot.size() + C.outer.size()) != ns)
            throw Error{PGCP_E_WELD, "seam vertex without a welded coordinate"};
        HIPTHROW(hipMemcpyAsync(welded_uv, zt.p, (size_t)ns * 16, hipMemcpyDeviceToHost, s));
        HIPTHROW(hipStreamSynchronize(s));
        P->welded = true;
        const auto t_rel = now();
        release();
        if (verbose)
            fprintf(stderr, "[pgcp] weld total %.2f ms (host arcs %.2f ms, buffer release %.2f ms)\n",
                    ms(t_start, now()), t_arcs, ms(t_rel, now()));
        return Error{PGCP_OK, ""};
    } catch (const Error& er) {
        release();
        return er;
    } catch (const std::exception& ex) {
        release();
        return Error{PGCP_E_WELD, ex.what()};
    }
}

}  // namespace pgcp
