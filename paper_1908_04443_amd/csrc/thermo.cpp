// thermo.cpp -- host equation-of-state helpers of the library: pressure,
// psi (Eq. 6), critical point and Maxwell coexistence densities, used to set
// temperatures and the limiter bounds rho_g, rho_l of the improved
// virtual-density scheme.
//
// Coexistence is found by Newton's method on the two conditions
//   p(rho_g) = p(rho_l),   integral_{rho_g}^{rho_l} (p(r) - p_s)/r^2 dr = 0
// (equal areas in the p-v plane), with the integral done by 64-point
// Gauss-Legendre panels in ln(rho), and started from the spinodal bracket.
#include <cmath>
#include <cstring>

#include "lbm_host.hpp"

namespace lbm {

double eos_pressure(const lbm_params& p, double rho) {
    const double a = p.eos_a, b = p.eos_b, RT = p.eos_R * p.eos_T;
    if (p.eos == LBM_EOS_CS) {
        const double h = 0.25 * b * rho, om = 1.0 - h;
        return rho * RT * (1.0 + h + h * h - h * h * h) / (om * om * om) - a * rho * rho;
    }
    const double br = b * rho;
    return rho * RT / (1.0 - br) - pr_aphi(p) * rho * rho / (1.0 + 2.0 * br - br * br);
}

double pr_Tc(double a, double b, double R) { return 0.0778 * a / (0.45724 * b * R); }

double pr_aphi(const lbm_params& p) {
    const double Tc = pr_Tc(p.eos_a, p.eos_b, p.eos_R);
    const double w = p.eos_omega;
    const double kap = 0.37464 + 1.54226 * w - 0.26992 * w * w;
    const double s = 1.0 + kap * (1.0 - std::sqrt(p.eos_T / Tc));
    return p.eos_a * s * s;
}

double psi_argument(const lbm_params& p, double rho) {
    return 2.0 * (eos_pressure(p, rho) - rho / 3.0) / p.G;
}

// dp/drho by a 4th-order central difference (step relative to rho)
static double slope(const lbm_params& p, double r) {
    const double h = 1e-4 * r;
    return (8.0 * (eos_pressure(p, r + h) - eos_pressure(p, r - h)) -
            (eos_pressure(p, r + 2 * h) - eos_pressure(p, r - 2 * h))) /
           (12.0 * h);
}

static double upper_density(const lbm_params& p) {
    return (p.eos == LBM_EOS_CS ? 4.0 : 1.0) / p.eos_b;
}

// sample the slope on a log grid and refine its minimum by parabolic steps
static double min_slope(const lbm_params& p, double* where) {
    const double hi = 0.95 * upper_density(p), lo = 1e-8 * hi;
    const int n = 4000;
    double best = 1e300, bx = lo;
    for (int i = 0; i <= n; ++i) {
        const double r = lo * std::pow(hi / lo, double(i) / n);
        const double s = slope(p, r);
        if (s < best) {
            best = s;
            bx = r;
        }
    }
    double step = bx * (std::pow(hi / lo, 1.0 / n) - 1.0);
    for (int it = 0; it < 100 && step > 1e-14 * bx; ++it) {
        const double sm = slope(p, bx - step), s0 = slope(p, bx), sp = slope(p, bx + step);
        const double den = sm - 2 * s0 + sp;
        double x = bx;
        if (den > 0) x = bx - 0.5 * step * (sp - sm) / den;
        if (x < bx - step) x = bx - step;
        if (x > bx + step) x = bx + step;
        bx = x;
        step *= 0.5;
    }
    if (where) *where = bx;
    return slope(p, bx);
}

int eos_critical(int eos, double a, double b, double R, double omega, double* Tc,
                 double* rhoc) {
    lbm_params p;
    std::memset(&p, 0, sizeof p);
    p.eos = eos;
    p.eos_a = a;
    p.eos_b = b;
    p.eos_R = R;
    p.eos_omega = omega;
    p.G = -1.0;
    double T;
    if (eos == LBM_EOS_PR) {
        T = pr_Tc(a, b, R);
    } else {
        // secant iteration on T for a zero minimum slope, after bracketing
        double lo = 1e-4 * a / (b * R), hi = 4.0 * a / (b * R);
        p.eos_T = lo;
        double flo = min_slope(p, nullptr);
        p.eos_T = hi;
        double fhi = min_slope(p, nullptr);
        if (!(flo < 0 && fhi > 0)) return LBM_EINVAL;
        for (int it = 0; it < 200 && (hi - lo) > 1e-15 * hi; ++it) {
            double mid = hi - fhi * (hi - lo) / (fhi - flo);
            if (!(mid > lo && mid < hi)) mid = 0.5 * (lo + hi);
            p.eos_T = mid;
            const double fm = min_slope(p, nullptr);
            if (fm < 0) {
                lo = mid;
                flo = fm;
            } else {
                hi = mid;
                fhi = fm;
            }
            // guard against one-sided secant stalls
            if (it % 3 == 2) {
                const double m2 = 0.5 * (lo + hi);
                p.eos_T = m2;
                const double f2 = min_slope(p, nullptr);
                if (f2 < 0) {
                    lo = m2;
                    flo = f2;
                } else {
                    hi = m2;
                    fhi = f2;
                }
            }
        }
        T = 0.5 * (lo + hi);
    }
    p.eos_T = T;
    double where = 0;
    min_slope(p, &where);
    if (Tc) *Tc = T;
    if (rhoc) *rhoc = where;
    return LBM_OK;
}

// 64-point Gauss-Legendre nodes on [-1, 1] (computed once by Newton on P_64)
static void gauss_legendre(double* x, double* w, int n) {
    for (int i = 0; i < n; ++i) {
        double z = std::cos(M_PI * (i + 0.75) / (n + 0.5)), dp = 0;
        for (int it = 0; it < 100; ++it) {
            double p0 = 1.0, p1 = z;
            for (int k = 2; k <= n; ++k) {
                const double pk = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
                p0 = p1;
                p1 = pk;
            }
            dp = n * (z * p1 - p0) / (z * z - 1.0);
            const double dz = p1 / dp;
            z -= dz;
            if (std::fabs(dz) < 1e-16) break;
        }
        x[i] = z;
        w[i] = 2.0 / ((1.0 - z * z) * dp * dp);
    }
}

// integral of (p - ps)/rho^2 over [rg, rl] = integral of (p - ps)/rho ds, s = ln rho
static double equal_area(const lbm_params& p, double rg, double rl, double ps) {
    static double gx[64], gw[64];
    static bool init = false;
    if (!init) {
        gauss_legendre(gx, gw, 64);
        init = true;
    }
    const int panels = 64;
    const double s0 = std::log(rg), s1 = std::log(rl), h = (s1 - s0) / panels;
    double acc = 0;
    for (int k = 0; k < panels; ++k) {
        const double c = s0 + (k + 0.5) * h;
        for (int i = 0; i < 64; ++i) {
            const double r = std::exp(c + 0.5 * h * gx[i]);
            acc += gw[i] * 0.5 * h * (eos_pressure(p, r) - ps) / r;
        }
    }
    return acc;
}

// root of p(rho) = ps on a bracket where p is monotone (Newton with bisection)
static double solve_p(const lbm_params& p, double ps, double lo, double hi) {
    double flo = eos_pressure(p, lo) - ps;
    double x = 0.5 * (lo + hi);
    for (int it = 0; it < 200; ++it) {
        const double fx = eos_pressure(p, x) - ps;
        if ((fx < 0) == (flo < 0)) {
            lo = x;
            flo = fx;
        } else {
            hi = x;
        }
        const double d = slope(p, x);
        double xn = (d != 0) ? x - fx / d : 0.5 * (lo + hi);
        if (!(xn > lo && xn < hi)) xn = 0.5 * (lo + hi);
        if (std::fabs(xn - x) <= 1e-16 * x) {
            x = xn;
            break;
        }
        x = xn;
    }
    return x;
}

int eos_coexistence(const lbm_params& p, double* rho_g, double* rho_l) {
    double rm = 0;
    if (min_slope(p, &rm) >= 0) return LBM_EINVAL;  // no two-phase region
    // spinodals: zeros of the slope on each side of its minimum
    auto slope_root = [&](double lo, double hi) {
        for (int it = 0; it < 200; ++it) {
            const double mid = 0.5 * (lo + hi);
            if ((slope(p, mid) > 0) == (slope(p, lo) > 0)) lo = mid;
            else hi = mid;
        }
        return 0.5 * (lo + hi);
    };
    const double cap = 0.999 * upper_density(p);
    const double ra = slope_root(1e-12, rm);
    double rb_hi = rm;
    while (slope(p, rb_hi) < 0 && rb_hi < cap) rb_hi = 0.5 * (rb_hi + cap);
    const double rb = slope_root(rm, rb_hi);
    const double pmax = eos_pressure(p, ra);
    double top = rb;
    while (eos_pressure(p, top) < pmax && top < cap) top = 0.5 * (top + cap);
    // bisection on the saturation pressure (the area decreases with ps)
    double plo = std::fmax(eos_pressure(p, rb), 0.0), phi = pmax, rg = 0, rl = 0;
    for (int it = 0; it < 120; ++it) {
        const double ps = 0.5 * (plo + phi);
        rg = solve_p(p, ps, 1e-14, ra);
        rl = solve_p(p, ps, rb, top);
        if (equal_area(p, rg, rl, ps) > 0) plo = ps;
        else phi = ps;
        if (phi - plo <= 1e-16 * phi) break;
    }
    *rho_g = rg;
    *rho_l = rl;
    return LBM_OK;
}

}  // namespace lbm
