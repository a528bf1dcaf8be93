// The maps of partial welding (Sections 3.4, 4.3.2; Algorithms 1 and 2) on the
// host: the zipper over a shared arc with its recorded parameters, the replay
// of that record for any other point, and the Moebius normalisation.  Shared
// by the host-only weld and the weld that replays tracked points on the GPU.
// Compiled with plain complex multiply and divide (-fcx-limited-range): every
// point at infinity is an explicit flag, so no operation meets inf or NaN.
#pragma once

#include <algorithm>
#include <cmath>
#include <vector>

#include "pgcp_internal.h"

namespace pgcp {
namespace weldmaps {

// A point of the extended plane.
struct EP {
    cplx z;
    bool inf;
};

// Principal square root (Re >= 0; on the negative real axis the sign of the
// imaginary zero picks the half, as for the C library's csqrt).  Plain
// formula: the weld's values stay far from overflow.
inline cplx csqrt_principal(cplx w) {
    const double x = w.real(), y = w.imag();
    const double r = std::sqrt(x * x + y * y);
    if (r == 0.0) return cplx(0.0, y);
    if (x >= 0.0) {
        const double t = std::sqrt(0.5 * (r + x));
        return cplx(t, y / (2.0 * t));
    }
    const double t = std::sqrt(0.5 * (r - x));
    return cplx(std::fabs(y) / (2.0 * t), std::copysign(t, y));
}

struct Component {
    std::vector<int> outer;       // CCW loop, global ids
    std::vector<EP> zo;           // coordinates aligned with outer
    std::vector<int> tracked;     // other boundary vertices of the welded pieces
    std::vector<EP> zt;
};

// ---------------------------------------------------------------- Algorithm 1

struct ZipRecord {
    int k = 0;
    cplx z0, z1;                  // g_1 parameters
    std::vector<double> c, d;     // L_xi_j for j = 2..k (index j-2)
    bool zeta_inf = false;
    cplx zeta;
    bool squared = false;
};

// Runs g_1..g_k and the final map on the arc points arc[0..k] (in place) and
// records the parameters.  Throws Error on a broken precondition.
inline ZipRecord zip_arc(std::vector<EP>& arc, int k, int branch, bool squared) {
    ZipRecord R;
    R.k = k;
    R.squared = squared;
    if (arc[0].inf || arc[1].inf) throw Error{PGCP_E_WELD, "arc point at infinity"};
    R.z0 = arc[0].z;
    R.z1 = arc[1].z;
    for (int l = 2; l <= k; ++l) {
        if (arc[l].inf) {
            arc[l].z = 1.0;
            arc[l].inf = false;
        } else {
            arc[l].z = csqrt_principal((arc[l].z - R.z1) / (arc[l].z - R.z0));
        }
    }
    arc[0] = EP{0.0, true};
    arc[1] = EP{0.0, false};
    R.c.resize(std::max(0, k - 1));
    R.d.resize(std::max(0, k - 1));
    for (int j = 2; j <= k; ++j) {
        cplx xi = arc[j].z;
        if (arc[j].inf || !(xi.real() > 0.0))
            throw Error{PGCP_E_WELD, "zipper point left the right half-plane"};
        double r2 = xi.real() * xi.real() + xi.imag() * xi.imag();
        double c = xi.real() / r2, d = xi.imag() / r2;
        R.c[j - 2] = c;
        R.d[j - 2] = d;
#pragma omp parallel for schedule(static) if (k >= 384)
        for (int l = 0; l <= k; ++l) {
            if (l == j - 1) {
                arc[l] = EP{cplx(0.0, (double)branch), false};
                continue;
            }
            if (l == j) {
                arc[l] = EP{0.0, false};
                continue;
            }
            if (l < j - 1) {
                // zipped: z = i t on the imaginary axis, L = i c t / (1 - d t)
                if (arc[l].inf) {
                    if (d == 0.0) continue;   // L(inf) = inf stays inf
                    const double s = -c / d;
                    arc[l] = EP{cplx(0.0, (s > 0 ? 1.0 : -1.0) * std::sqrt(s * s + 1.0)), false};
                    continue;
                }
                const double t = arc[l].z.imag(), den = 1.0 - d * t;
                if (den == 0.0) {
                    arc[l] = EP{0.0, true};
                    continue;
                }
                const double s = c * t / den;
                const double sg = (s > 0.0) ? 1.0 : (s < 0.0 ? -1.0 : 0.0);
                arc[l] = EP{cplx(0.0, sg * std::sqrt(s * s + 1.0)), false};
                continue;
            }
            // not yet zipped: L_xi(z) = c z / (1 + i d z), principal sqrt(L^2 - 1)
            if (arc[l].inf) {
                if (d == 0.0) continue;
                const cplx L = cplx(0.0, -c / d);
                arc[l] = EP{csqrt_principal(L * L - 1.0), false};
                continue;
            }
            const cplx den = 1.0 + cplx(0.0, d) * arc[l].z;
            if (den == cplx(0.0, 0.0)) {
                arc[l] = EP{0.0, true};
                continue;
            }
            const cplx L = c * arc[l].z / den;
            arc[l] = EP{csqrt_principal(L * L - 1.0), false};
        }
    }
    // final map z / (1 - z / zeta)
    R.zeta_inf = arc[0].inf;
    R.zeta = arc[0].z;
    for (int l = 1; l <= k; ++l) {
        if (l == k) {
            arc[l] = EP{0.0, false};
            continue;
        }
        cplx w;
        if (R.zeta_inf) w = arc[l].z;
        else w = arc[l].z / (1.0 - arc[l].z / R.zeta);
        w = cplx(0.0, w.imag());
        if (squared) w = w * w;
        arc[l] = EP{w, false};
    }
    arc[0] = EP{0.0, true};
    if (!squared) {
        for (int l = 1; l < k; ++l)
            if (!(branch * arc[l].z.imag() > 0.0))
                throw Error{PGCP_E_WELD, "Algorithm 1 postcondition failed"};
    }
    return R;
}

// Sends one non-arc point through the recorded Algorithm 1 chain.
inline EP zip_point(const ZipRecord& R, EP p) {
    if (p.inf) {
        p = EP{1.0, false};
    } else {
        cplx den = p.z - R.z0;
        if (den == cplx(0.0, 0.0)) p = EP{0.0, true};
        else p.z = csqrt_principal((p.z - R.z1) / den);
    }
    for (int j = 0; j + 2 <= R.k; ++j) {
        double c = R.c[j], d = R.d[j];
        if (p.inf) {
            if (d != 0.0) p = EP{cplx(0.0, -c / d), false};
            else continue;   // L(inf) = inf, sqrt(inf) = inf
        } else {
            cplx den = 1.0 + cplx(0.0, d) * p.z;
            if (den == cplx(0.0, 0.0)) {
                p = EP{0.0, true};
                continue;
            }
            p.z = c * p.z / den;
        }
        p.z = csqrt_principal(p.z * p.z - 1.0);
    }
    if (p.inf) {
        if (R.zeta_inf) return p;
        p = EP{-R.zeta, false};
    } else if (!R.zeta_inf) {
        cplx den = 1.0 - p.z / R.zeta;
        if (den == cplx(0.0, 0.0)) return EP{0.0, true};
        p.z = p.z / den;
    }
    if (R.squared) p.z = p.z * p.z;
    return p;
}

// ---------------------------------------------------------------- Algorithm 2

struct CloseRecord {
    int k = 0;
    std::vector<double> c0, c1;   // h_j for j = k-1..1 (index k-1-j)
    bool eta_inf = false;
    cplx eta;
};

// T(z) = z / (c0 - i c1 z); T(inf) = i / c1
inline EP T_apply(double c0, double c1, const EP& p) {
    if (p.inf) {
        if (c1 != 0.0) return EP{cplx(0.0, 1.0 / c1), false};
        return p;
    }
    cplx den = cplx(c0, 0.0) - cplx(0.0, c1) * p.z;
    if (den == cplx(0.0, 0.0)) return EP{0.0, true};
    return EP{p.z / den, false};
}

inline EP h0_apply(const CloseRecord& R, EP p) {
    if (R.eta_inf) {
        if (p.inf) return p;
        return EP{p.z * p.z, false};
    }
    if (p.inf) return EP{R.eta * R.eta, false};
    cplx den = 1.0 - p.z / R.eta;
    if (den == cplx(0.0, 0.0)) return EP{0.0, true};
    cplx w = p.z / den;
    return EP{w * w, false};
}

inline CloseRecord close_arcs(std::vector<EP>& A, std::vector<EP>& B, int k) {
    CloseRecord R;
    R.k = k;
    for (int j = k - 1; j >= 1; --j) {
        if (A[j].inf || B[j].inf) throw Error{PGCP_E_WELD, "glued pair at infinity"};
        double a = A[j].z.imag(), b = B[j].z.imag();
        if (a == 0.0 || b == 0.0 || a == b) throw Error{PGCP_E_WELD, "degenerate glued pair"};
        double c0 = -2.0 * a * b / (a - b), c1 = (a + b) / (a - b);
        if (!(c0 > 0.0)) throw Error{PGCP_E_WELD, "glued pair out of cyclic order"};
        R.c0.push_back(c0);
        R.c1.push_back(c1);
#pragma omp parallel for schedule(static) if (k >= 384)
        for (int m = 0; m < 2 * (k + 1); ++m) {
            auto& X = m <= k ? A : B;
            const int l = m <= k ? m : m - (k + 1);
            if (l == j) {
                X[l] = EP{0.0, false};
                continue;
            }
            if (l < j && !X[l].inf) {
                // unglued arc point on the imaginary axis: T(i u) = i u / (c0 + c1 u)
                const double u = X[l].z.imag(), den = c0 + c1 * u;
                if (den == 0.0) {
                    X[l] = EP{0.0, true};
                    continue;
                }
                const double s = u / den;
                if (std::fabs(s) <= 1.0) {
                    X[l] = EP{cplx(std::sqrt(1.0 - s * s), 0.0), false};
                } else {
                    const double sg = s > 0.0 ? 1.0 : -1.0;
                    X[l] = EP{cplx(0.0, sg * std::sqrt(s * s - 1.0)), false};
                }
                continue;
            }
            EP t = T_apply(c0, c1, X[l]);
            if (t.inf) {
                X[l] = t;
            } else if (l < j) {
                const double s = t.z.imag();
                if (std::fabs(s) <= 1.0) {
                    X[l] = EP{cplx(std::sqrt(1.0 - s * s), 0.0), false};
                } else {
                    const double sg = s > 0.0 ? 1.0 : -1.0;
                    X[l] = EP{cplx(0.0, sg * std::sqrt(s * s - 1.0)), false};
                }
            } else {
                X[l] = EP{csqrt_principal(t.z * t.z + 1.0), false};
            }
        }
    }
    R.eta_inf = A[0].inf;
    R.eta = A[0].z;
    for (auto* S : {&A, &B}) {
        auto& X = *S;
        for (int l = 1; l <= k; ++l) X[l] = h0_apply(R, X[l]);
        X[0] = EP{0.0, true};
    }
    return R;
}

inline EP close_point(const CloseRecord& R, EP p) {
    for (size_t t = 0; t < R.c0.size(); ++t) {
        p = T_apply(R.c0[t], R.c1[t], p);
        if (p.inf) continue;
        p.z = csqrt_principal(p.z * p.z + 1.0);
    }
    return h0_apply(R, p);
}

// ---------------------------------------------------------------- Mobius

struct Mobius {
    cplx a, b, c, d;
};

// {z1, z2, z3} -> {-1, 1, inf}
inline Mobius mobius3(cplx z1, cplx z2, cplx z3) {
    cplx p = 2.0 * (z2 - z3), q = z2 - z1;
    return Mobius{p - q, -p * z1 + q * z3, q, -q * z3};
}

inline EP mobius_apply(const Mobius& M, EP p) {
    if (p.inf) return EP{M.a / M.c, false};
    cplx den = M.c * p.z + M.d;
    if (den == cplx(0.0, 0.0)) return EP{0.0, true};
    return EP{(M.a * p.z + M.b) / den, false};
}

}  // namespace weldmaps
}  // namespace pgcp
