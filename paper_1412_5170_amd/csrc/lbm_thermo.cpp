// Coexistence densities of a flat interface (include/pplbm.h, lbm_coexistence): the Maxwell
// rule (Eq. 19) or the mechanical stability condition (Eq. 18), for the rescaled
// Carnahan-Starling EOS with psi from Eq. 7 or for the effective density of Eq. 33 with the
// pressure Eq. 7 implies.  Both rules have one form:
//     p0(rho_g) = p0(rho_l) = p_c,   integral_{rho_g}^{rho_l} (p_c - p0(rho)) w(rho) drho = 0,
// with w = 1/rho^2 (Eq. 19) or w = psi' / psi^(1+eps) (Eq. 18).  The spinodals come from a
// scan of dp0/drho and bisection; each p_c gives rho_g and rho_l by bisection on the rising
// branches; the integral is composite 8-point Gauss-Legendre in ln(rho); p_c is bisected.

#include <cmath>
#include <functional>

#include "../../include/pplbm.h"
#include "lbm_internal.h"

namespace {

struct Model {
    int kind;                   // LBM_EOS_*
    double a, bq, RT, K;        // C-S: a, b/4, R T, K
    double G;                   // interaction strength (< 0)
    double eps_psi;             // Eq. 33 exponent
    double rho_max;             // upper end of the density axis

    double p0(double r) const {
        if (kind == LBM_EOS_CARNAHAN_STARLING) {
            const double e = bq * r;
            const double Z = (1 + e + e * e - e * e * e) / ((1 - e) * (1 - e) * (1 - e));
            return K * (r * RT * Z - a * r * r);
        }
        const double s = psi(r);
        return r / 3 + G * s * s / 2;
    }
    double dp0(double r) const {
        if (kind == LBM_EOS_CARNAHAN_STARLING) {
            const double e = bq * r, om = 1 - e;
            const double Z = (1 + e + e * e - e * e * e) / (om * om * om);
            const double dZ = (4 + 4 * e - 2 * e * e) / (om * om * om * om);
            return K * (RT * (Z + e * dZ) - 2 * a * r);
        }
        return 1.0 / 3 + G * psi(r) * dpsi(r);
    }
    double psi(double r) const {
        if (kind == LBM_EOS_CARNAHAN_STARLING) return std::sqrt(2 * (p0(r) - r / 3) / G);
        if (eps_psi == 0) return std::exp(-1 / r);
        return std::pow(r / (1 + r), 1 / eps_psi);
    }
    double dpsi(double r) const {
        if (kind == LBM_EOS_CARNAHAN_STARLING) return (dp0(r) - 1.0 / 3) / (G * psi(r));
        if (eps_psi == 0) return psi(r) / (r * r);
        return psi(r) / (eps_psi * r * (1 + r));
    }
    // Eq. 18's weight psi' / psi^(1+e) = (ln psi)' exp(-e ln psi), written through ln psi so
    // that it stays finite where psi of Eq. 33 underflows.
    double mech_weight(double r, double e) const {
        if (kind == LBM_EOS_CARNAHAN_STARLING) return dpsi(r) / std::pow(psi(r), 1 + e);
        const double lp = eps_psi == 0 ? -1 / r : std::log(r / (1 + r)) / eps_psi;
        const double dlp = eps_psi == 0 ? 1 / (r * r) : 1 / (eps_psi * r * (1 + r));
        return dlp * std::exp(-e * lp);
    }
};

// Root of an increasing function on [lo, hi].
double bisect_up(const std::function<double(double)> &f, double lo, double hi) {
    for (int i = 0; i < 200 && hi - lo > 1e-17 * hi; ++i) {
        const double mid = 0.5 * (lo + hi);
        if (f(mid) < 0) lo = mid;
        else hi = mid;
    }
    return 0.5 * (lo + hi);
}

// 8-point Gauss-Legendre nodes and weights on [-1, 1] (positive half).
constexpr double kGx[4] = {0.1834346424956498, 0.5255324099163290, 0.7966664774136267,
                           0.9602898564975363};
constexpr double kGw[4] = {0.3626837833783620, 0.3137066458778873, 0.2223810344533745,
                           0.1012285362903763};

double integrate_log(const std::function<double(double)> &g, double r0, double r1, int panels) {
    const double t0 = std::log(r0), t1 = std::log(r1), h = (t1 - t0) / panels;
    double sum = 0;
    for (int k = 0; k < panels; ++k) {
        const double c = t0 + (k + 0.5) * h, half = 0.5 * h;
        double part = 0;
        for (int j = 0; j < 4; ++j) {
            const double ra = std::exp(c - half * kGx[j]), rb = std::exp(c + half * kGx[j]);
            part += kGw[j] * (g(ra) * ra + g(rb) * rb);
        }
        sum += half * part;
    }
    return sum;
}

int solve(const Model &m, const std::function<double(double)> &w, double *rho_g, double *rho_l) {
    // spinodals: dp0/drho changes sign + to - (gas side), then - to + (liquid side)
    const int N = 6000;
    const double lo = 1e-9, span = std::log(m.rho_max / lo);
    double s1 = -1, s2 = -1, prev_r = lo, prev = m.dp0(lo);
    for (int k = 1; k <= N && s2 < 0; ++k) {
        const double r = lo * std::exp(span * k / N);
        const double d = m.dp0(r);
        if (!std::isfinite(d)) break;
        if (s1 < 0 && prev > 0 && d < 0) s1 = bisect_up([&](double x) { return -m.dp0(x); }, prev_r, r);
        else if (s1 > 0 && prev < 0 && d > 0) s2 = bisect_up([&](double x) { return m.dp0(x); }, prev_r, r);
        prev = d;
        prev_r = r;
    }
    if (s1 < 0 || s2 < 0) return LBM_EINVAL;  // no van der Waals loop
    // p_c between the spinodal pressures, and above the pressure of a gas 1e-8 times as dense
    // as the gas spinodal (no coexistence this dilute is sought)
    const double top = m.p0(s1) * (1 - 1e-12);
    double bot = std::fmax(m.p0(s2), m.p0(1e-8 * s1)) * (1 + 1e-12) + 1e-300;
    if (!(top > bot)) return LBM_EINVAL;
    auto branches = [&](double pc, double *g, double *l) {
        *g = bisect_up([&](double x) { return m.p0(x) - pc; }, 0.0, s1);
        double hi = s2 + 0.5 * (m.rho_max - s2);
        for (int k = 2; m.p0(hi) < pc && k < 60; ++k) hi = s2 + (m.rho_max - s2) * (1 - std::ldexp(1.0, -k));
        *l = bisect_up([&](double x) { return m.p0(x) - pc; }, s2, hi);
    };
    auto I = [&](double pc, double *g, double *l) {
        branches(pc, g, l);
        return integrate_log([&](double r) { return (pc - m.p0(r)) * w(r); }, *g, *l, 256);
    };
    double g = 0, l = 0;
    double Ilo = I(bot, &g, &l), Ihi = I(top, &g, &l);
    if (!(Ilo * Ihi < 0)) return LBM_EINVAL;
    double a = bot, b = top;
    for (int it = 0; it < 200 && b - a > 1e-16 * b; ++it) {
        const double mid = 0.5 * (a + b);
        const double Im = I(mid, &g, &l);
        if ((Im > 0) == (Ihi > 0)) {
            b = mid;
            Ihi = Im;
        } else {
            a = mid;
        }
    }
    I(0.5 * (a + b), &g, &l);
    *rho_g = g;
    *rho_l = l;
    return std::isfinite(g) && std::isfinite(l) ? LBM_OK : LBM_EINVAL;
}

}  // namespace

extern "C" int lbm_coexistence(const lbm_eos *eos, const lbm_force *force, int rule, double eps_mech,
                               double *rho_g, double *rho_l) {
    if (!eos || !force || !rho_g || !rho_l || !(force->G < 0)) return LBM_EINVAL;
    if (rule != LBM_COEX_MAXWELL && rule != LBM_COEX_MECHANICAL) return LBM_EINVAL;
    if (rule == LBM_COEX_MECHANICAL && !(eps_mech >= 0 && std::isfinite(eps_mech))) return LBM_EINVAL;
    Model m{};
    m.kind = eos->kind;
    m.G = force->G;
    if (eos->kind == LBM_EOS_CARNAHAN_STARLING) {
        if (!(eos->a > 0) || !(eos->b > 0) || !(eos->R > 0) || !(eos->K > 0)) return LBM_EINVAL;
        if (!(eos->T_over_Tc > 0 && eos->T_over_Tc < 1)) return LBM_EINVAL;
        double rc, Tc, pc;
        pplbm::critical_point(eos->a, eos->b, eos->R, &rc, &Tc, &pc);
        m.a = eos->a;
        m.bq = eos->b / 4;
        m.RT = eos->R * eos->T_over_Tc * Tc;
        m.K = eos->K;
        m.rho_max = 4 / eos->b * (1 - 1e-9);
        if (rule == LBM_COEX_MECHANICAL) {
            // psi of Eq. 7 needs rho/3 - p0 > 0: stop the liquid axis where it vanishes
            double lo = 2 / eos->b, hi = m.rho_max;
            if (m.p0(hi) - hi / 3 > 0) {
                for (int i = 0; i < 200; ++i) {
                    const double mid = 0.5 * (lo + hi);
                    if (m.p0(mid) - mid / 3 < 0) lo = mid;
                    else hi = mid;
                }
                m.rho_max = lo;
            }
        }
    } else if (eos->kind == LBM_EOS_SBRAGAGLIA_SHAN) {
        if (!(eos->eps >= 0 && std::isfinite(eos->eps))) return LBM_EINVAL;
        m.eps_psi = eos->eps;
        m.rho_max = -6 * force->G + 4;  // psi -> 1, p0 -> rho/3 + G/2: the loop lies below
    } else {
        return LBM_EINVAL;
    }
    if (rule == LBM_COEX_MAXWELL)
        return solve(m, [](double r) { return 1 / (r * r); }, rho_g, rho_l);
    return solve(m, [&](double r) { return m.mech_weight(r, eps_mech); }, rho_g, rho_l);
}

extern "C" int lbm_eos_pressure(const lbm_eos *eos, const lbm_force *force, double rho, double *p) {
    if (!eos || !force || !p || !(rho > 0) || !(force->G < 0)) return LBM_EINVAL;
    Model m{};
    m.kind = eos->kind;
    m.G = force->G;
    if (eos->kind == LBM_EOS_CARNAHAN_STARLING) {
        if (!(eos->a > 0) || !(eos->b > 0) || !(eos->R > 0) || !(eos->K > 0) || !(eos->T_over_Tc > 0))
            return LBM_EINVAL;
        if (!(eos->b * rho / 4 < 1)) return LBM_EINVAL;
        double rc, Tc, pc;
        pplbm::critical_point(eos->a, eos->b, eos->R, &rc, &Tc, &pc);
        m.a = eos->a;
        m.bq = eos->b / 4;
        m.RT = eos->R * eos->T_over_Tc * Tc;
        m.K = eos->K;
    } else if (eos->kind == LBM_EOS_SBRAGAGLIA_SHAN) {
        if (!(eos->eps >= 0)) return LBM_EINVAL;
        m.eps_psi = eos->eps;
    } else {
        return LBM_EINVAL;
    }
    *p = m.p0(rho);
    return LBM_OK;
}
