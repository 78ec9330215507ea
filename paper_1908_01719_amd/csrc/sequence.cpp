// Gradient profiles: f on pieces, F in closed form per piece, int F^2 by
// composite Gauss-Legendre quadrature between the breakpoints.
//
// Profiles (t in us; a lobe of sign s):
//   PGSE (Sec. 2, eq. pgse): f = +1 on [0, delta], -1 on (Delta, Delta+delta],
//     echo T = Delta + delta.
//   cos-OGSE (Sec. 3): f = cos(w t) on [0, delta], -cos(w (t - tau)) on
//     (tau, tau + delta], w = 2 n pi / delta, tau = (delta + Delta) / 2,
//     T = delta + Delta. sin-OGSE: the same with sin.
//   trapezoidal PGSE: each pulse of length delta ramps linearly over `ramp`
//     up to 1 and down again; second pulse (sign -1) from Delta; T = Delta + delta.
//   double profiles: the profile, a mixing time t_mix, the profile again;
//     T = 2 (Delta + delta) + t_mix.
#include "sequence.hpp"

#include <algorithm>
#include <cmath>
#include <string>

#include "assembly.hpp"

namespace dmri {
namespace {

enum Shape { CONST = 0, COS = 1, SIN = 2, RAMP = 3 };

struct Piece {
    double a, b;   // support [a, b]
    Shape shape;
    double s;      // sign / level
    double t0;     // phase origin (COS/SIN) or ramp zero (RAMP)
    double w;      // angular frequency (COS/SIN) or ramp length (RAMP)
};

double piece_f(const Piece& p, double t) {
    switch (p.shape) {
        case CONST: return p.s;
        case COS: return p.s * std::cos(p.w * (t - p.t0));
        case SIN: return p.s * std::sin(p.w * (t - p.t0));
        default: return p.s * (t - p.t0) / p.w;
    }
}

// int_a^t f over the piece (a <= t <= b).
double piece_int(const Piece& p, double t) {
    switch (p.shape) {
        case CONST: return p.s * (t - p.a);
        case COS: return p.s * (std::sin(p.w * (t - p.t0)) - std::sin(p.w * (p.a - p.t0))) / p.w;
        case SIN: return p.s * (std::cos(p.w * (p.a - p.t0)) - std::cos(p.w * (t - p.t0))) / p.w;
        default: {
            const double u = t - p.t0, v = p.a - p.t0;
            return p.s * (u * u - v * v) / (2.0 * p.w);
        }
    }
}

struct Profile {
    std::vector<Piece> pieces;   // sorted, disjoint interiors
    std::vector<double> F0;      // F at the start of each piece
    double T = 0;

    void finish() {
        std::sort(pieces.begin(), pieces.end(), [](const Piece& x, const Piece& y) { return x.a < y.a; });
        F0.assign(pieces.size(), 0.0);
        double acc = 0.0;
        for (size_t i = 0; i < pieces.size(); ++i) {
            F0[i] = acc;
            acc += piece_int(pieces[i], pieces[i].b);
        }
    }
    double F(double t) const {
        double acc = 0.0;
        for (size_t i = 0; i < pieces.size(); ++i) {
            const Piece& p = pieces[i];
            if (t <= p.a) return F0[i];
            if (t <= p.b) return F0[i] + piece_int(p, t);
            acc = F0[i] + piece_int(p, p.b);
        }
        return acc;
    }
    // (f(t0+), f(t1-)) for an interval inside one piece or between pieces.
    void limits(double t0, double t1, double& lo, double& hi) const {
        for (const Piece& p : pieces) {
            if (p.a <= t0 + 1e-9 * (1.0 + std::fabs(t0)) && t1 <= p.b + 1e-9 * (1.0 + std::fabs(t1))) {
                lo = piece_f(p, t0);
                hi = piece_f(p, t1);
                return;
            }
        }
        lo = hi = 0.0;
    }
    std::vector<double> breaks() const {
        std::vector<double> v{0.0, T};
        for (const Piece& p : pieces) {
            v.push_back(p.a);
            v.push_back(p.b);
        }
        std::sort(v.begin(), v.end());
        v.erase(std::unique(v.begin(), v.end()), v.end());
        return v;
    }
};

void add_single(Profile& P, int32_t kind, double d, double D, double extra, double shift) {
    if (kind == 0) {
        P.pieces.push_back({shift, shift + d, CONST, 1.0, 0.0, 0.0});
        P.pieces.push_back({shift + D, shift + D + d, CONST, -1.0, 0.0, 0.0});
    } else if (kind == 2 || kind == 3) {
        const double w = 2.0 * extra * M_PI / d;
        const double tau = 0.5 * (d + D);
        const Shape sh = kind == 2 ? COS : SIN;
        P.pieces.push_back({shift, shift + d, sh, 1.0, shift, w});
        P.pieces.push_back({shift + tau, shift + tau + d, sh, -1.0, shift + tau, w});
    } else {  // trapezoid
        const double e = extra;
        for (int lobe = 0; lobe < 2; ++lobe) {
            const double st = shift + (lobe ? D : 0.0), s = lobe ? -1.0 : 1.0;
            P.pieces.push_back({st, st + e, RAMP, s, st, e});
            if (d - 2.0 * e > 0) P.pieces.push_back({st + e, st + d - e, CONST, s, 0.0, 0.0});
            P.pieces.push_back({st + d - e, st + d, RAMP, -s, st + d, e});
        }
    }
}

// Gauss-Legendre nodes and weights on [-1, 1] (Newton on P_n).
void gauss_legendre(int n, std::vector<double>& x, std::vector<double>& w) {
    x.assign(n, 0.0);
    w.assign(n, 0.0);
    for (int i = 0; i < n; ++i) {
        double z = std::cos(M_PI * (i + 0.75) / (n + 0.5));
        for (int it = 0; it < 100; ++it) {
            double p0 = 1.0, p1 = z;
            for (int k = 2; k <= n; ++k) {
                const double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
                p0 = p1;
                p1 = p2;
            }
            const double dp = n * (z * p1 - p0) / (z * z - 1.0);
            const double dz = p1 / dp;
            z -= dz;
            if (std::fabs(dz) < 1e-16) {
                double q0 = 1.0, q1 = z;
                for (int k = 2; k <= n; ++k) {
                    const double q2 = ((2.0 * k - 1.0) * z * q1 - (k - 1.0) * q0) / k;
                    q0 = q1;
                    q1 = q2;
                }
                const double dq = n * (z * q1 - q0) / (z * z - 1.0);
                x[i] = z;
                w[i] = 2.0 / ((1.0 - z * z) * dq * dq);
                break;
            }
        }
    }
}

double int_F2(const Profile& P) {
    std::vector<double> gx, gw;
    gauss_legendre(12, gx, gw);
    const std::vector<double> br = P.breaks();
    double tot = 0.0;
    for (size_t i = 0; i + 1 < br.size(); ++i) {
        const double a = br[i], b = std::min(br[i + 1], P.T);
        if (!(b > a)) continue;
        const int m = 64;  // sub-intervals per smooth segment
        const double h = (b - a) / m;
        for (int j = 0; j < m; ++j) {
            const double c = a + (j + 0.5) * h;
            for (size_t k = 0; k < gx.size(); ++k) {
                const double F = P.F(c + 0.5 * h * gx[k]);
                tot += 0.5 * h * gw[k] * F * F;
            }
        }
    }
    return tot;
}

bool on_grid(double v, double dt) {
    const double r = v / dt;
    return std::fabs(r - std::round(r)) <= 1e-9 * std::max(1.0, std::fabs(r));
}

}  // namespace

SequenceTables make_sequence(int32_t kind, const double* params, int32_t n_params, double dt,
                             double theta) {
    static const int need[6] = {2, 3, 3, 3, 3, 4};
    if (kind < 0 || kind > 5) throw Error(DMRI_E_INVALID, "unknown sequence kind");
    if (!params || n_params != need[kind])
        throw Error(DMRI_E_INVALID, "sequence kind " + std::to_string(kind) + " takes " +
                                        std::to_string(need[kind]) + " parameters");
    for (int i = 0; i < n_params; ++i)
        if (!std::isfinite(params[i])) throw Error(DMRI_E_INVALID, "sequence parameters must be finite");
    if (!std::isfinite(dt) || !(dt > 0)) throw Error(DMRI_E_INVALID, "need dt > 0");
    if (!std::isfinite(theta) || theta < 0.5 || theta > 1.0)
        throw Error(DMRI_E_INVALID, "theta must be in [1/2, 1]");
    const double d = params[0], D = params[1];
    if (!(d > 0) || !(D >= d)) throw Error(DMRI_E_INVALID, "need 0 < delta <= Delta");
    const bool dbl = kind == 1 || kind == 5;
    const int32_t base = kind == 1 ? 0 : kind == 5 ? 4 : kind;
    double extra = 0.0;
    if (base == 2 || base == 3) {
        extra = params[2];
        if (!(extra >= 1) || extra != std::floor(extra))
            throw Error(DMRI_E_INVALID, "OGSE needs a whole number of periods >= 1");
    } else if (base == 4) {
        extra = params[2];
        if (!(extra > 0) || !(2.0 * extra <= d))
            throw Error(DMRI_E_INVALID, "trapezoid ramp must be in (0, delta/2]");
    }
    const double tmix = dbl ? params[n_params - 1] : 0.0;
    if (dbl && !(tmix >= 0)) throw Error(DMRI_E_INVALID, "mixing time must be >= 0");
    Profile P;
    add_single(P, base, d, D, extra, 0.0);
    const double T1 = D + d;
    P.T = T1;
    if (dbl) {
        add_single(P, base, d, D, extra, T1 + tmix);
        P.T = 2.0 * T1 + tmix;
    }
    P.finish();
    for (double v : P.breaks())
        if (!on_grid(v, dt))
            throw Error(DMRI_E_INVALID,
                        "every edge of the profile and the echo time must be a multiple of dt");
    const double steps = std::round(P.T / dt);
    if (steps > 1e7) throw Error(DMRI_E_INVALID, "too many time steps");
    SequenceTables S;
    S.dt = dt;
    S.theta = theta;
    S.n_steps = static_cast<int>(steps);
    S.F.assign(S.n_steps + 1, 0.0);
    S.f_start.assign(S.n_steps + 1, 0.0);
    S.f_end.assign(S.n_steps + 1, 0.0);
    for (int n = 0; n <= S.n_steps; ++n) S.F[n] = P.F(n * dt);
    S.F[S.n_steps] = P.F(P.T);
    for (int n = 1; n <= S.n_steps; ++n) P.limits((n - 1) * dt, n * dt, S.f_start[n], S.f_end[n]);
    S.has_f = true;
    // PGSE in closed form (Sec. 2: delta^2 (Delta - delta/3) per block).
    if (base == 0)
        S.int_F2 = (dbl ? 2.0 : 1.0) * d * d * (D - d / 3.0);
    else
        S.int_F2 = int_F2(P);
    return S;
}

}  // namespace dmri
