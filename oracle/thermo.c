/*
 * thermo.c -- critical point and Maxwell coexistence densities of the
 * equation of state used by the oracle.
 *
 * TEST INFRASTRUCTURE ONLY (part of the CPU oracle; shares no code with the
 * GPU library).
 *
 * Plain bracketing methods only: golden-section search for extrema,
 * bisection for roots, composite Simpson quadrature for the equal-area
 * integral.  The limiter bounds rho_g, rho_l of the improved virtual-density
 * scheme are the coexisting gas and liquid densities of the system, which the
 * Maxwell construction gives for the equation of state (Sec. II A discusses
 * thermodynamic consistency with respect to that construction).
 */
#include <math.h>
#include <string.h>
#include "oracle.h"

static double pr_Tc(double a, double b, double R) {
    /* a = 0.45724 R^2 Tc^2 / pc and b = 0.0778 R Tc / pc (with Eq. 18) */
    return (0.0778 / 0.45724) * (a / b) / R;
}

/* analytic derivative dp/drho of the equation of state */
static double dpdrho(const orc_params* p, double rho) {
    double a = p->eos_a, b = p->eos_b, R = p->eos_R, T = p->eos_T;
    if (p->eos == ORC_EOS_CS) {
        /* d(rho Z_CS)/drho = (1 + 4e + 4e^2 - 4e^3 + e^4) / (1 - e)^4 */
        double e = b * rho / 4.0, om = 1.0 - e;
        return R * T * (1.0 + 4.0 * e + 4.0 * e * e - 4.0 * e * e * e + e * e * e * e) /
                   (om * om * om * om) -
               2.0 * a * rho;
    } else {
        double Tc = pr_Tc(a, b, R);
        double kap = 0.37464 + 1.54226 * p->eos_omega -
                     0.26992 * p->eos_omega * p->eos_omega;
        double s = 1.0 + kap * (1.0 - sqrt(T / Tc));
        double phiT = s * s;
        double D = 1.0 + 2.0 * b * rho - b * b * rho * rho;
        double Dp = 2.0 * b - 2.0 * b * b * rho;
        double om = 1.0 - b * rho;
        return R * T / (om * om) - a * phiT * (2.0 * rho * D - rho * rho * Dp) / (D * D);
    }
}

/* upper end of the physical density range */
static double rho_cap(const orc_params* p) {
    return (p->eos == ORC_EOS_CS) ? 4.0 / p->eos_b : 1.0 / p->eos_b;
}

typedef double (*fn_t)(const orc_params*, double);

static double neg_p(const orc_params* p, double r) { return -orc_eos_p(p, r); }
static double pos_p(const orc_params* p, double r) { return orc_eos_p(p, r); }

/* golden-section minimiser of a unimodal function on [lo, hi] */
static double golden_min(const orc_params* p, fn_t fn, double lo, double hi) {
    const double g = 0.5 * (sqrt(5.0) - 1.0);
    double x1 = hi - g * (hi - lo), x2 = lo + g * (hi - lo);
    double f1 = fn(p, x1), f2 = fn(p, x2);
    for (int it = 0; it < 200 && (hi - lo) > 1e-15 * (1.0 + fabs(hi)); ++it) {
        if (f1 < f2) {
            hi = x2;
            x2 = x1;
            f2 = f1;
            x1 = hi - g * (hi - lo);
            f1 = fn(p, x1);
        } else {
            lo = x1;
            x1 = x2;
            f1 = f2;
            x2 = lo + g * (hi - lo);
            f2 = fn(p, x2);
        }
    }
    return 0.5 * (lo + hi);
}

/* bisection for fn(x) = target on [lo, hi] with a sign change */
static double bisect(const orc_params* p, fn_t fn, double target, double lo,
                     double hi) {
    double flo = fn(p, lo) - target;
    for (int it = 0; it < 300; ++it) {
        double mid = 0.5 * (lo + hi);
        double fm = fn(p, mid) - target;
        if ((fm < 0.0) == (flo < 0.0)) {
            lo = mid;
            flo = fm;
        } else {
            hi = mid;
        }
        if (hi - lo <= 1e-16 * fabs(hi)) break;
    }
    return 0.5 * (lo + hi);
}

/* minimum over rho of dp/drho, and where it sits */
static double min_slope(const orc_params* p, double* where) {
    double r = golden_min(p, dpdrho, 1e-9, 0.9 * rho_cap(p));
    if (where) *where = r;
    return dpdrho(p, r);
}

int orc_critical(int32_t eos, double a, double b, double R, double omega,
                 double* Tc, double* rhoc) {
    orc_params p;
    memset(&p, 0, sizeof p);
    p.eos = eos;
    p.eos_a = a;
    p.eos_b = b;
    p.eos_R = R;
    p.eos_omega = omega;
    if (!(a > 0.0 && b > 0.0 && R > 0.0)) return ORC_EINVAL;
    double T;
    if (eos == ORC_EOS_PR) {
        T = pr_Tc(a, b, R);
    } else if (eos == ORC_EOS_CS) {
        /* the critical isotherm is the one whose smallest slope is zero */
        double lo = 1e-6 * a / (b * R), hi = 10.0 * a / (b * R);
        for (int it = 0; it < 200; ++it) {
            double mid = 0.5 * (lo + hi);
            p.eos_T = mid;
            if (min_slope(&p, NULL) < 0.0) lo = mid;
            else hi = mid;
        }
        T = 0.5 * (lo + hi);
    } else {
        return ORC_EINVAL;
    }
    p.eos_T = T;
    double where;
    min_slope(&p, &where);
    if (Tc) *Tc = T;
    if (rhoc) *rhoc = where;
    return ORC_OK;
}

/* equal-area residual: integral over [rg, rl] of (p - ps)/rho^2 drho,
 * written in s = ln(rho) (so drho/rho^2 = ds/rho), composite Simpson */
static double area(const orc_params* p, double rg, double rl, double ps) {
    const int n = 200000;
    double s0 = log(rg), s1 = log(rl), h = (s1 - s0) / n, acc = 0.0;
    for (int i = 0; i <= n; ++i) {
        double r = exp(s0 + i * h);
        double v = (orc_eos_p(p, r) - ps) / r;
        double c = (i == 0 || i == n) ? 1.0 : (i % 2 ? 4.0 : 2.0);
        acc += c * v;
    }
    return acc * h / 3.0;
}

int orc_coexistence(const orc_params* p, double* rho_g, double* rho_l) {
    double ra, rb, rm;
    if (min_slope(p, &rm) >= 0.0) return ORC_EINVAL; /* supercritical */
    /* spinodals: local maximum of p below rm, local minimum above it */
    ra = golden_min(p, neg_p, 1e-12, rm);
    double cap = rho_cap(p);
    double top = rm;
    /* upper search bound where the pressure rises again beyond the loop */
    while (top < cap && orc_eos_p(p, top) <= orc_eos_p(p, ra)) top = 0.5 * (top + cap);
    rb = golden_min(p, pos_p, rm, top);
    double plo = orc_eos_p(p, rb), phi = orc_eos_p(p, ra);
    if (plo < 0.0) plo = 0.0;
    double rg = 0.0, rl = 0.0;
    for (int it = 0; it < 200; ++it) {
        double ps = 0.5 * (plo + phi);
        rg = bisect(p, pos_p, ps, 1e-14, ra);
        rl = bisect(p, pos_p, ps, rb, top);
        double A = area(p, rg, rl, ps);
        if (A > 0.0) plo = ps; /* pressure too low */
        else phi = ps;
        if (phi - plo <= 1e-17 * fabs(phi)) break;
    }
    *rho_g = rg;
    *rho_l = rl;
    return ORC_OK;
}
