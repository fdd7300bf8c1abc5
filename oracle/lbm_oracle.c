/*
 * lbm_oracle.c -- plain FP64 CPU oracle of one pseudopotential MRT lattice
 * Boltzmann time step with the contact-angle wall schemes of Li, Yu & Luo.
 *
 * TEST INFRASTRUCTURE ONLY: used by the tests, the package smoke check and
 * the CPU-baseline leg of the benchmark to check the GPU library.  It shares
 * no code with the GPU library.
 *
 * The file is compiled twice: once with real = double, and once with
 * ORC_COMPLEX defined, where real = double complex, for complex-step
 * derivatives (a perturbation i*h carried through the same arithmetic gives
 * d/dparam = Im/h without cancellation).  Comparisons (limiter, domain
 * checks) act on real parts; the square root is the principal branch.
 *
 * Every phase of the step is its own plain loop over nodes, in the order
 *   density (Eq. 4) -> psi (Eq. 6) -> wall virtual density (Eqs. 16-17 and
 *   the limiter; or the constant virtual density; or psi = 0 for the
 *   solid-fluid interaction) -> force (Eq. 5, Eq. 8) -> velocity (Eq. 4)
 *   -> MRT collision with the forcing of Eq. 7 (Eq. 2) -> streaming with
 *   halfway bounce-back (Eq. 3, Fig. 3).
 * No fusion, no blocking.  Build with -ffp-contract=off.
 */
#include <math.h>
#include <complex.h>
#include <stdlib.h>
#include <string.h>
#include "oracle.h"

#ifdef ORC_COMPLEX
typedef double complex real;
#define RE(x) creal(x)
#define SQRT(x) csqrt(x)
#else
typedef double real;
#define RE(x) (x)
#define SQRT(x) sqrt(x)
#endif

typedef struct {
    int Q, D;
    int32_t e[19 * 3];
    double t[19], w[19];
    double M[19 * 19], Minv[19 * 19];
    int32_t opp[19];
} lat_t;

#ifndef ORC_COMPLEX
/* ------------------------------------------------------------------------
 * Lattice tables.  Velocity order (D2Q9): rest, +x, +y, -x, -y, (1,1),
 * (-1,1), (-1,-1), (1,-1).  D3Q19: rest, +-x, +-y, +-z, then the twelve
 * face diagonals in opposite pairs.  Lattice weights t are the standard
 * second-order ones; the force-stencil weights w of Eq. 5 are 1/3 and 1/12
 * in 2-D (stated with Eq. 5), and 1/6 and 1/12 in 3-D (sum w e e = I).
 * The moment rows of M are the orthogonal polynomial rows of Lallemand-Luo
 * (2-D) and d'Humieres et al. (3-D), in the order that matches the
 * relaxation matrix of Eq. 2 and the rows of Eq. 7.  M^-1 = M^T diag(M M^T)^-1.
 * ------------------------------------------------------------------------ */
static const int32_t E9[9][3] = {
    {0, 0, 0}, {1, 0, 0}, {0, 1, 0}, {-1, 0, 0}, {0, -1, 0},
    {1, 1, 0}, {-1, 1, 0}, {-1, -1, 0}, {1, -1, 0}};
static const int32_t E19[19][3] = {
    {0, 0, 0},  {1, 0, 0},  {-1, 0, 0}, {0, 1, 0},   {0, -1, 0},
    {0, 0, 1},  {0, 0, -1}, {1, 1, 0},  {-1, -1, 0}, {1, -1, 0},
    {-1, 1, 0}, {1, 0, 1},  {-1, 0, -1}, {1, 0, -1}, {-1, 0, 1},
    {0, 1, 1},  {0, -1, -1}, {0, 1, -1}, {0, -1, 1}};

static double row2d(int k, double cx, double cy) {
    double c2 = cx * cx + cy * cy;
    switch (k) {
    case 0: return 1.0;
    case 1: return -4.0 + 3.0 * c2;
    case 2: return 4.0 - 10.5 * c2 + 4.5 * c2 * c2;
    case 3: return cx;
    case 4: return (-5.0 + 3.0 * c2) * cx;
    case 5: return cy;
    case 6: return (-5.0 + 3.0 * c2) * cy;
    case 7: return cx * cx - cy * cy;
    default: return cx * cy;
    }
}

static double row3d(int k, double cx, double cy, double cz) {
    double c2 = cx * cx + cy * cy + cz * cz;
    switch (k) {
    case 0: return 1.0;
    case 1: return 19.0 * c2 - 30.0;
    case 2: return (21.0 * c2 * c2 - 53.0 * c2 + 24.0) / 2.0;
    case 3: return cx;
    case 4: return (5.0 * c2 - 9.0) * cx;
    case 5: return cy;
    case 6: return (5.0 * c2 - 9.0) * cy;
    case 7: return cz;
    case 8: return (5.0 * c2 - 9.0) * cz;
    case 9: return 3.0 * cx * cx - c2;
    case 10: return (3.0 * c2 - 5.0) * (3.0 * cx * cx - c2);
    case 11: return cy * cy - cz * cz;
    case 12: return (3.0 * c2 - 5.0) * (cy * cy - cz * cz);
    case 13: return cx * cy;
    case 14: return cy * cz;
    case 15: return cx * cz;
    case 16: return (cy * cy - cz * cz) * cx;
    case 17: return (cz * cz - cx * cx) * cy;
    default: return (cx * cx - cy * cy) * cz;
    }
}

int orc_lattice(int32_t lattice, int32_t* e, double* t, double* w, double* M,
                double* Minv, int32_t* opp) {
    int Q;
    if (lattice == 9) Q = 9;
    else if (lattice == 19) Q = 19;
    else return ORC_EINVAL;
    for (int a = 0; a < Q; ++a) {
        const int32_t* ea = (Q == 9) ? E9[a] : E19[a];
        e[3 * a + 0] = ea[0];
        e[3 * a + 1] = ea[1];
        e[3 * a + 2] = ea[2];
        int c2 = ea[0] * ea[0] + ea[1] * ea[1] + ea[2] * ea[2];
        if (Q == 9) {
            t[a] = (c2 == 0) ? 4.0 / 9.0 : (c2 == 1) ? 1.0 / 9.0 : 1.0 / 36.0;
            w[a] = (c2 == 0) ? 0.0 : (c2 == 1) ? 1.0 / 3.0 : 1.0 / 12.0;
        } else {
            t[a] = (c2 == 0) ? 1.0 / 3.0 : (c2 == 1) ? 1.0 / 18.0 : 1.0 / 36.0;
            w[a] = (c2 == 0) ? 0.0 : (c2 == 1) ? 1.0 / 6.0 : 1.0 / 12.0;
        }
    }
    for (int a = 0; a < Q; ++a) {
        opp[a] = -1;
        for (int b = 0; b < Q; ++b)
            if (e[3 * b] == -e[3 * a] && e[3 * b + 1] == -e[3 * a + 1] &&
                e[3 * b + 2] == -e[3 * a + 2])
                opp[a] = b;
    }
    for (int k = 0; k < Q; ++k)
        for (int a = 0; a < Q; ++a)
            M[k * Q + a] = (Q == 9) ? row2d(k, e[3 * a], e[3 * a + 1])
                                    : row3d(k, e[3 * a], e[3 * a + 1], e[3 * a + 2]);
    for (int k = 0; k < Q; ++k) {
        double d = 0.0;
        for (int a = 0; a < Q; ++a) d += M[k * Q + a] * M[k * Q + a];
        for (int a = 0; a < Q; ++a) Minv[a * Q + k] = M[k * Q + a] / d;
    }
    return ORC_OK;
}

void orc_set_threads(int n) {
#ifdef _OPENMP
    extern void omp_set_num_threads(int);
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}
#endif /* !ORC_COMPLEX */

static int get_lat(int32_t lattice, lat_t* L) {
    L->Q = (lattice == 9) ? 9 : 19;
    L->D = (lattice == 9) ? 2 : 3;
    return orc_lattice(lattice, L->e, L->t, L->w, L->M, L->Minv, L->opp);
}

static int check_params(const orc_params* p) {
    if (p->lattice != 9 && p->lattice != 19) return ORC_EINVAL;
    if (p->nx < 1 || p->ny < 1 || p->nz < 1) return ORC_EINVAL;
    if (p->lattice == 9 && p->nz != 1) return ORC_EINVAL;
    if (p->scheme < ORC_IVD || p->scheme > ORC_GF) return ORC_EINVAL;
    if (p->scheme == ORC_GF && p->lattice != 9) return ORC_EINVAL;  /* 2-D scheme */
    if (p->sfi_solid_psi < 0 || p->sfi_solid_psi > 4) return ORC_EINVAL;
    if (p->sfi_psi_presum != 0 && p->sfi_psi_presum != 1) return ORC_EINVAL;
    if (p->sfi_lattice_weights != 0 && p->sfi_lattice_weights != 1) return ORC_EINVAL;
    return ORC_OK;
}

/* neighbour of node n along velocity e, periodic in every axis */
static int64_t nbr(const orc_params* p, int64_t n, const int32_t* e) {
    int64_t nx = p->nx, ny = p->ny, nz = p->nz;
    int64_t x = n % nx, y = (n / nx) % ny, z = n / (nx * ny);
    x = ((x + e[0]) % nx + nx) % nx;
    y = ((y + e[1]) % ny + ny) % ny;
    z = ((z + e[2]) % nz + nz) % nz;
    return x + nx * (y + ny * z);
}

/* Non-ideal equation of state.  CS: Carnahan-Starling with the attraction
 * -a rho^2.  PR: Eq. 18 with phi(T) from the acentric factor omega and
 * Tc = (0.0778/0.45724) (a/b) / R, which follows from the definitions of a
 * and b given with Eq. 18. */
static real eos_p(const orc_params* p, real rho) {
    double a = p->eos_a, b = p->eos_b, R = p->eos_R, T = p->eos_T;
    if (p->eos == ORC_EOS_CS) {
        real eta = b * rho / 4.0;
        real one_m = 1.0 - eta;
        return rho * R * T * (1.0 + eta + eta * eta - eta * eta * eta) /
                   (one_m * one_m * one_m) -
               a * rho * rho;
    } else {
        double Tc = (0.0778 / 0.45724) * (a / b) / R;
        double kap = 0.37464 + 1.54226 * p->eos_omega -
                     0.26992 * p->eos_omega * p->eos_omega;
        double s = 1.0 + kap * (1.0 - sqrt(T / Tc));
        double phiT = s * s;
        return rho * R * T / (1.0 - b * rho) -
               a * phiT * rho * rho / (1.0 + 2.0 * b * rho - b * b * rho * rho);
    }
}

/* Eq. 6 with c = 1, cs^2 = 1/3: psi = sqrt(2 (p_EOS - rho/3) / G). */
static real psi_arg(const orc_params* p, real rho) {
    return 2.0 * (eos_p(p, rho) - rho / 3.0) / p->G;
}

#ifndef ORC_COMPLEX
double orc_eos_p(const orc_params* p, double rho) { return eos_p(p, rho); }
double orc_psi_arg(const orc_params* p, double rho) { return psi_arg(p, rho); }
#endif

static int psi_of(const orc_params* p, real rho, real* out) {
    real arg = psi_arg(p, rho);
    if (!(RE(arg) >= 0.0)) return ORC_EDOMAIN; /* negative or NaN */
    *out = SQRT(arg);
    return ORC_OK;
}

/* equilibrium of the standard second-order form */
static real feq(const lat_t* L, int a, real rho, const real* u) {
    real eu = 0.0, uu = 0.0;
    for (int d = 0; d < L->D; ++d) {
        eu += (double)L->e[3 * a + d] * u[d];
        uu += u[d] * u[d];
    }
    return L->t[a] * rho * (1.0 + 3.0 * eu + 4.5 * eu * eu - 1.5 * uu);
}

/* Moment-space source.  D2Q9: Eq. 7 as printed (the relaxation time in the
 * third row is tau_epsilon).  D3Q19: S = M G with the Guo discrete force
 * G_a = t_a [3 (e_a - u) + 9 (e_a.u) e_a] . F, plus the same
 * thermodynamic-consistency pressure shift 2 sigma |Fm|^2 / psi^2 carried by
 * the energy row, whose coefficient becomes 114 = 19 * 3 * 2. */
static void source(const orc_params* p, const lat_t* L, const real* u,
                   const real* F, const real* Fm, real psi, real* S) {
    int Q = L->Q, D = L->D;
    real uF = 0.0, Fm2 = 0.0;
    for (int d = 0; d < D; ++d) {
        uF += u[d] * F[d];
        Fm2 += Fm[d] * Fm[d];
    }
    real sig = p->sigma * Fm2 / (psi * psi);
    if (Q == 9) {
        S[0] = 0.0;
        S[1] = 6.0 * uF + 12.0 * sig / (p->tau[1] - 0.5);
        S[2] = -6.0 * uF - 12.0 * sig / (p->tau[2] - 0.5);
        S[3] = F[0];
        S[4] = -F[0];
        S[5] = F[1];
        S[6] = -F[1];
        S[7] = 2.0 * (u[0] * F[0] - u[1] * F[1]);
        S[8] = u[0] * F[1] + u[1] * F[0];
    } else {
        real G[19];
        for (int a = 0; a < Q; ++a) {
            real eu = 0.0, g = 0.0;
            for (int d = 0; d < D; ++d) eu += (double)L->e[3 * a + d] * u[d];
            for (int d = 0; d < D; ++d)
                g += (3.0 * ((double)L->e[3 * a + d] - u[d]) +
                      9.0 * eu * (double)L->e[3 * a + d]) * F[d];
            G[a] = L->t[a] * g;
        }
        for (int k = 0; k < Q; ++k) {
            real s = 0.0;
            for (int a = 0; a < Q; ++a) s += L->M[k * Q + a] * G[a];
            S[k] = s;
        }
        S[1] += 114.0 * sig / (p->tau[1] - 0.5);
    }
}

#ifndef ORC_COMPLEX
int orc_source(const orc_params* p, const double* u, const double* F,
               const double* Fm, double psi, double* S) {
    lat_t L;
    if (get_lat(p->lattice, &L) != ORC_OK) return ORC_EINVAL;
    source(p, &L, u, F, Fm, psi, S);
    return ORC_OK;
}
#endif

/* geometry: wall flag = solid node with at least one fluid neighbour among
 * the non-rest velocities (the solid nodes the force stencil of Eq. 5 reads),
 * and the position of each wall node in increasing node order */
typedef struct {
    int64_t N;
    uint8_t* wall;
    int64_t* widx;
    int64_t nwall;
} geom_t;

static int geom_build(const orc_params* p, const lat_t* L, const uint8_t* solid,
                      geom_t* g) {
    int64_t N = (int64_t)p->nx * p->ny * p->nz;
    g->N = N;
    g->wall = (uint8_t*)calloc((size_t)N, 1);
    g->widx = (int64_t*)malloc(sizeof(int64_t) * (size_t)N);
    if (!g->wall || !g->widx) return ORC_EINVAL;
    g->nwall = 0;
    for (int64_t n = 0; n < N; ++n) {
        g->widx[n] = -1;
        if (!solid[n]) continue;
        for (int a = 1; a < L->Q; ++a)
            if (!solid[nbr(p, n, &L->e[3 * a])]) g->wall[n] = 1;
        if (g->wall[n]) g->widx[n] = g->nwall++;
    }
    return ORC_OK;
}

static void geom_free(geom_t* g) {
    free(g->wall);
    free(g->widx);
}

typedef struct {
    real *rho, *psi, *F, *Fm, *u, *fpost;
} work_t;

static int work_alloc(const lat_t* L, int64_t N, work_t* w) {
    w->rho = (real*)calloc((size_t)N, sizeof(real));
    w->psi = (real*)calloc((size_t)N, sizeof(real));
    w->F = (real*)calloc((size_t)(3 * N), sizeof(real));
    w->Fm = (real*)calloc((size_t)(3 * N), sizeof(real));
    w->u = (real*)calloc((size_t)(3 * N), sizeof(real));
    w->fpost = (real*)calloc((size_t)(L->Q * N), sizeof(real));
    return (w->rho && w->psi && w->F && w->Fm && w->u && w->fpost) ? ORC_OK
                                                                   : ORC_EINVAL;
}

static void work_free(work_t* w) {
    free(w->rho);
    free(w->psi);
    free(w->F);
    free(w->Fm);
    free(w->u);
    free(w->fpost);
}

/* ------------------------------------------------------------------------
 * Curved geometric formulation (Sec. III A), 2-D.  For a wall node P:
 *   n_s  the unit solid normal of Eq. 13, -sum_e omega(|e|^2) s(P+e) e over
 *        the 5 x 5 block around P without P itself (|e|^2 = 1, 2, 4, 5, 8),
 *        with the 8th-order isotropic weights of Eq. 14 and s = 1 on solid
 *        nodes;
 *   n_1, n_2  n_s turned by +(pi/2 - theta_a) and -(pi/2 - theta_a), the
 *        two characteristic directions of Eq. 15;
 *   D_k  the point where the ray P + t n_k (t > 0) first meets one of the
 *        four mesh lines that bound the 3 x 3 block around P (x = x_P - 1,
 *        x_P + 1, y = y_P - 1, y_P + 1): every line is intersected and the
 *        smallest positive t is kept, so D_k = t n_k;
 *   rho(D_k)  interpolated from the position of D_k: the bilinear weights
 *        (1 - |D_x - i|)(1 - |D_y - j|) of the four lattice nodes around
 *        D_k, which on a mesh line reduce to the linear interpolation
 *        between the two nodes of that line.  Nodes whose weight is below
 *        GF_SNAP are not part of the stencil (D_k on a lattice node is that
 *        node alone, whatever the rounding of t n_k).  Only fluid nodes
 *        count: their weights are renormalised; no fluid node leaves D_k
 *        void;
 *   rho_P = max(rho(D_1), rho(D_2)) for theta_a <= 90 deg, else the min,
 *        Eq. 11; one void point gives the other; two void points, or no
 *        normal, give the w-weighted mean of the fluid neighbours (Eq. 17).
 * The paper leaves the location of D_1, D_2 to its Ref. [26]; this is the
 * reading taken here.  A ray that meets two lines at one t passes through
 * the corner node they share, so no choice between lines is ever made. */
#define GF_SNAP 1e-12

static int64_t node_at(const orc_params* p, int64_t n, int dx, int dy) {
    int32_t e[3] = {dx, dy, 0};
    return nbr(p, n, e);
}

/* Eq. 14: weight of an offset of squared length e2 in the normal of Eq. 13 */
static double gf_weight(int e2) {
    switch (e2) {
    case 1: return 4.0 / 21.0;
    case 2: return 4.0 / 45.0;
    case 4: return 1.0 / 60.0;
    case 5: return 2.0 / 315.0;
    case 8: return 1.0 / 5040.0;
    default: return 0.0;
    }
}

/* Unit solid normal at wall node b (pointing out of the solid); 0 if the
 * weighted sum vanishes. */
static int gf_normal(const orc_params* p, const uint8_t* solid, int64_t b, double* n) {
    double gx = 0.0, gy = 0.0;
    for (int dy = -2; dy <= 2; ++dy)
        for (int dx = -2; dx <= 2; ++dx) {
            double om = gf_weight(dx * dx + dy * dy);
            if (om == 0.0 || !solid[node_at(p, b, dx, dy)]) continue;
            gx += om * dx;
            gy += om * dy;
        }
    double len = hypot(gx, gy);
    if (len == 0.0) return 0;
    n[0] = -gx / len;
    n[1] = -gy / len;
    return 1;
}

/* D = t v at the smallest t > 0 where P + t v meets x = +-1 or y = +-1 */
static void gf_crossing(const double* v, double* D) {
    double best = INFINITY;
    for (int axis = 0; axis < 2; ++axis)
        for (int side = -1; side <= 1; side += 2) {
            if (v[axis] == 0.0) continue;
            double t = side / v[axis];
            if (t > 0.0 && t < best) best = t;
        }
    D[0] = best * v[0];
    D[1] = best * v[1];
}

/* rho at the point D (relative to wall node b): fluid nodes of its
 * interpolation stencil with renormalised weights; *ok = 0 if none. */
static real gf_rho_at(const orc_params* p, const uint8_t* solid, const real* rho, int64_t b,
                      const double* D, int* ok) {
    int i0 = (int)floor(D[0]), j0 = (int)floor(D[1]);
    real acc = 0.0;
    double wsum = 0.0;
    for (int j = j0; j <= j0 + 1; ++j)
        for (int i = i0; i <= i0 + 1; ++i) {
            double w = (1.0 - fabs(D[0] - i)) * (1.0 - fabs(D[1] - j));
            if (w < GF_SNAP) continue;
            int64_t m = node_at(p, b, i, j);
            if (solid[m]) continue;
            acc += w * rho[m];
            wsum += w;
        }
    *ok = wsum > 0.0;
    return *ok ? acc / wsum : 0.0;
}

/* The two characteristic directions of Eq. 15 */
static void gf_directions(const double* n, double theta_deg, double* v1, double* v2) {
    const double pi = 3.14159265358979323846;
    double turn = 0.5 * pi - theta_deg * (pi / 180.0);
    double c = cos(turn), s = sin(turn);
    v1[0] = c * n[0] - s * n[1];
    v1[1] = s * n[0] + c * n[1];
    v2[0] = c * n[0] + s * n[1];
    v2[1] = -s * n[0] + c * n[1];
}

static real gf_density(const orc_params* p, const lat_t* L, const uint8_t* solid,
                       const real* rho, int64_t b, double theta_deg) {
    double n[2], v[2][2], D[2];
    int have = gf_normal(p, solid, b, n);
    real r[2] = {0.0, 0.0};
    int ok[2] = {0, 0};
    if (have) {
        gf_directions(n, theta_deg, v[0], v[1]);
        for (int k = 0; k < 2; ++k) {
            gf_crossing(v[k], D);
            r[k] = gf_rho_at(p, solid, rho, b, D, &ok[k]);
        }
    }
    if (ok[0] && ok[1]) {
        int take_min = theta_deg > 90.0;
        int first = take_min ? RE(r[0]) <= RE(r[1]) : RE(r[0]) >= RE(r[1]);
        return first ? r[0] : r[1];
    }
    if (ok[0]) return r[0];
    if (ok[1]) return r[1];
    /* Eq. 17, the standard case */
    real num = 0.0;
    double den = 0.0;
    for (int a = 1; a < L->Q; ++a) {
        int64_t y = nbr(p, b, &L->e[3 * a]);
        if (!solid[y]) {
            num += L->w[a] * rho[y];
            den += L->w[a];
        }
    }
    return num / den;
}

#ifndef ORC_COMPLEX
/* For the pins: n_s, D_1 and D_2 of every wall node, relative to the node
 * (6 doubles per wall node, in wall-list order; NaN without a normal). */
int orc_gf_points(const orc_params* p, const uint8_t* solid, const double* theta_deg,
                  double* out) {
    if (check_params(p) != ORC_OK || p->lattice != 9) return ORC_EINVAL;
    int64_t nw = orc_wall_nodes(p, solid, NULL);
    int64_t* walls = malloc((size_t)(nw > 0 ? nw : 1) * sizeof(int64_t));
    if (!walls) return ORC_EINVAL;
    orc_wall_nodes(p, solid, walls);
    for (int64_t k = 0; k < nw; ++k) {
        double n[2], v[2][2];
        double* o = out + 6 * k;
        if (gf_normal(p, solid, walls[k], n)) {
            gf_directions(n, theta_deg[k], v[0], v[1]);
            o[0] = n[0];
            o[1] = n[1];
            gf_crossing(v[0], o + 2);
            gf_crossing(v[1], o + 4);
        } else {
            for (int i = 0; i < 6; ++i) o[i] = NAN;
        }
    }
    free(walls);
    return ORC_OK;
}
#endif

/* Phases 1-5 of the step: density, psi, wall virtual density, force and
 * velocity at time t from the post-streaming populations f. */
static int macro_phases(const orc_params* p, const lat_t* L, const geom_t* g,
                        const uint8_t* solid, const real* phi, const real* drho,
                        const real* f, work_t* w) {
    const int64_t N = g->N;
    const int Q = L->Q, D = L->D;
    int err = 0;

    /* 1. density, Eq. 4 */
#pragma omp parallel for schedule(static)
    for (int64_t n = 0; n < N; ++n) {
        real r = 0.0;
        if (!solid[n])
            for (int a = 0; a < Q; ++a) r += f[a * N + n];
        w->rho[n] = r;
    }
    /* 2. pseudopotential, Eq. 6 */
#pragma omp parallel for schedule(static) reduction(| : err)
    for (int64_t n = 0; n < N; ++n) {
        w->psi[n] = 0.0;
        if (!solid[n] && psi_of(p, w->rho[n], &w->psi[n]) != ORC_OK) err |= 1;
    }
    if (err) return ORC_EDOMAIN;

    /* 3. virtual density of the wall nodes */
    for (int64_t b = 0; b < N; ++b) {
        if (!g->wall[b]) continue;
        int64_t k = g->widx[b];
        if (p->scheme == ORC_IVD) {
            /* Eq. 17: weighted mean of the fluid neighbours' density */
            real num = 0.0;
            double den = 0.0;
            for (int a = 1; a < Q; ++a) {
                int64_t y = nbr(p, b, &L->e[3 * a]);
                if (!solid[y]) {
                    num += L->w[a] * w->rho[y];
                    den += L->w[a];
                }
            }
            real rave = num / den;
            /* Eq. 16, both branches in one form: phi >= 1 with drho = 0
             * lowers the angle, phi = 1 with drho >= 0 raises it */
            real rw = phi[k] * rave - drho[k];
            /* limiter: rho_g <= rho_w <= rho_l */
            if (RE(rw) > p->rho_l) rw = p->rho_l;
            if (RE(rw) < p->rho_g) rw = p->rho_g;
            w->rho[b] = rw;
            if (psi_of(p, rw, &w->psi[b]) != ORC_OK) return ORC_EDOMAIN;
        } else if (p->scheme == ORC_GF) {
            w->rho[b] = gf_density(p, L, solid, w->rho, b, RE(phi[k]));
            if (psi_of(p, w->rho[b], &w->psi[b]) != ORC_OK) return ORC_EDOMAIN;
        } else if (p->scheme == ORC_VD) {
            /* original scheme: one constant virtual density for the solid */
            w->rho[b] = p->rho_w;
            if (psi_of(p, p->rho_w, &w->psi[b]) != ORC_OK) return ORC_EDOMAIN;
        } else {
            /* solid-fluid interaction: the solid carries no pseudopotential
             * (the other values of sfi_solid_psi are alternative readings) */
            w->rho[b] = 0.0;
            w->psi[b] = 0.0;
            real rs = 0.0;
            if (p->sfi_solid_psi == 1) {
                real num = 0.0;
                double den = 0.0;
                for (int a = 1; a < Q; ++a) {
                    int64_t y = nbr(p, b, &L->e[3 * a]);
                    if (!solid[y]) {
                        num += L->w[a] * w->rho[y];
                        den += L->w[a];
                    }
                }
                rs = num / den;
            } else if (p->sfi_solid_psi == 2) {
                rs = p->rho_g;
            } else if (p->sfi_solid_psi == 3) {
                rs = p->rho_l;
            }
            if (RE(rs) > 0.0 && psi_of(p, rs, &w->psi[b]) != ORC_OK) return ORC_EDOMAIN;
        }
    }

    /* 4. force: cohesion Eq. 5, adhesion Eq. 8 (SFI only), body force */
#pragma omp parallel for schedule(static)
    for (int64_t n = 0; n < N; ++n) {
        for (int d = 0; d < 3; ++d) {
            w->F[d * N + n] = 0.0;
            w->Fm[d * N + n] = 0.0;
        }
        if (solid[n]) continue;
        real sm[3] = {0.0, 0.0, 0.0};
        double sa[3] = {0.0, 0.0, 0.0};
        const int own = p->scheme == ORC_SFI && p->sfi_solid_psi == 4;
        for (int a = 1; a < Q; ++a) {
            int64_t y = nbr(p, n, &L->e[3 * a]);
            real psy = (own && solid[y]) ? w->psi[n] : w->psi[y];
            for (int d = 0; d < D; ++d) {
                sm[d] += L->w[a] * psy * (double)L->e[3 * a + d];
                if (solid[y])
                    sa[d] += (p->sfi_lattice_weights ? L->t[a] : L->w[a]) * (double)L->e[3 * a + d];
            }
        }
        for (int d = 0; d < D; ++d) {
            real fm = -p->G * w->psi[n] * sm[d];
            real pre = p->sfi_psi_presum ? w->psi[n] : w->rho[n];
            real fa = (p->scheme == ORC_SFI) ? -p->G_w * pre * sa[d] : 0.0;
            w->Fm[d * N + n] = fm;
            w->F[d * N + n] = fm + fa + p->body_force[d];
        }
    }
    /* 5. velocity, Eq. 4 */
#pragma omp parallel for schedule(static)
    for (int64_t n = 0; n < N; ++n) {
        for (int d = 0; d < 3; ++d) w->u[d * N + n] = 0.0;
        if (solid[n]) continue;
        for (int d = 0; d < D; ++d) {
            real j = 0.0;
            for (int a = 0; a < Q; ++a) j += (double)L->e[3 * a + d] * f[a * N + n];
            w->u[d * N + n] = (j + 0.5 * w->F[d * N + n]) / w->rho[n];
        }
    }
    return ORC_OK;
}

/* Phases 6-7: MRT collision (Eq. 2 with m = M f, m_eq = M f_eq, S from
 * Eq. 7) and streaming (Eq. 3) with halfway bounce-back: a population that
 * would enter a solid node returns to its origin in the opposite direction
 * at the next time level. */
static void collide_stream(const orc_params* p, const lat_t* L, const geom_t* g,
                           const uint8_t* solid, const real* f, real* fnew,
                           work_t* w) {
    const int64_t N = g->N;
    const int Q = L->Q, D = L->D;

#pragma omp parallel for schedule(static)
    for (int64_t n = 0; n < N; ++n) {
        if (solid[n]) continue;
        real u[3], F[3], Fm[3], fe[19], m[19], meq[19], S[19], ms[19];
        for (int d = 0; d < 3; ++d) {
            u[d] = w->u[d * N + n];
            F[d] = w->F[d * N + n];
            Fm[d] = w->Fm[d * N + n];
        }
        real rho = w->rho[n];
        for (int a = 0; a < Q; ++a) fe[a] = feq(L, a, rho, u);
        for (int k = 0; k < Q; ++k) {
            real s = 0.0, se = 0.0;
            for (int a = 0; a < Q; ++a) {
                s += L->M[k * Q + a] * f[a * N + n];
                se += L->M[k * Q + a] * fe[a];
            }
            m[k] = s;
            meq[k] = se;
        }
        source(p, L, u, F, Fm, w->psi[n], S);
        for (int k = 0; k < Q; ++k) {
            double lam = 1.0 / p->tau[k];
            ms[k] = m[k] - lam * (m[k] - meq[k]) + (1.0 - 0.5 * lam) * S[k];
        }
        for (int a = 0; a < Q; ++a) {
            real s = 0.0;
            for (int k = 0; k < Q; ++k) s += L->Minv[a * Q + k] * ms[k];
            w->fpost[a * N + n] = s;
        }
        (void)D;
    }

    for (int64_t i = 0; i < (int64_t)Q * N; ++i) fnew[i] = 0.0;
#pragma omp parallel for schedule(static)
    for (int64_t n = 0; n < N; ++n) {
        if (solid[n]) continue;
        for (int a = 0; a < Q; ++a) {
            int64_t y = nbr(p, n, &L->e[3 * a]);
            if (!solid[y])
                fnew[a * N + y] = w->fpost[a * N + n];
            else
                fnew[L->opp[a] * N + n] = w->fpost[a * N + n];
        }
    }
}

/* advance f (in place) by nsteps */
static int run_steps(const orc_params* p, const lat_t* L, const geom_t* g,
                     const uint8_t* solid, const real* phi, const real* drho,
                     real* f, int64_t nsteps) {
    work_t w;
    int rc = work_alloc(L, g->N, &w);
    real* fnew = (real*)calloc((size_t)(L->Q * g->N), sizeof(real));
    if (rc != ORC_OK || !fnew) {
        work_free(&w);
        free(fnew);
        return ORC_EINVAL;
    }
    for (int64_t s = 0; s < nsteps && rc == ORC_OK; ++s) {
        rc = macro_phases(p, L, g, solid, phi, drho, f, &w);
        if (rc != ORC_OK) break;
        collide_stream(p, L, g, solid, f, fnew, &w);
        memcpy(f, fnew, sizeof(real) * (size_t)(L->Q * g->N));
    }
    free(fnew);
    work_free(&w);
    return rc;
}

#ifndef ORC_COMPLEX
int64_t orc_wall_nodes(const orc_params* p, const uint8_t* solid, int64_t* idx) {
    lat_t L;
    geom_t g;
    if (check_params(p) != ORC_OK || get_lat(p->lattice, &L) != ORC_OK) return -1;
    if (geom_build(p, &L, solid, &g) != ORC_OK) return -1;
    if (idx)
        for (int64_t n = 0; n < g.N; ++n)
            if (g.wall[n]) idx[g.widx[n]] = n;
    int64_t nw = g.nwall;
    geom_free(&g);
    return nw;
}

int orc_init_eq(const orc_params* p, const uint8_t* solid, const double* rho0,
                const double* u0, double* f) {
    lat_t L;
    if (check_params(p) != ORC_OK || get_lat(p->lattice, &L) != ORC_OK)
        return ORC_EINVAL;
    int64_t N = (int64_t)p->nx * p->ny * p->nz;
    for (int64_t n = 0; n < N; ++n) {
        double u[3] = {0.0, 0.0, 0.0};
        if (u0)
            for (int d = 0; d < L.D; ++d) u[d] = u0[d * N + n];
        for (int a = 0; a < L.Q; ++a)
            f[a * N + n] = solid[n] ? 0.0 : feq(&L, a, rho0[n], u);
    }
    return ORC_OK;
}

int orc_run(const orc_params* p, const uint8_t* solid, const double* phi,
            const double* drho, double* f, int64_t nsteps) {
    lat_t L;
    geom_t g;
    if (check_params(p) != ORC_OK || get_lat(p->lattice, &L) != ORC_OK)
        return ORC_EINVAL;
    if (geom_build(p, &L, solid, &g) != ORC_OK) return ORC_EINVAL;
    int rc = run_steps(p, &L, &g, solid, phi, drho, f, nsteps);
    geom_free(&g);
    return rc;
}

int orc_fields(const orc_params* p, const uint8_t* solid, const double* phi,
               const double* drho, const double* f, double* rho, double* u,
               double* force) {
    lat_t L;
    geom_t g;
    work_t w;
    if (check_params(p) != ORC_OK || get_lat(p->lattice, &L) != ORC_OK)
        return ORC_EINVAL;
    if (geom_build(p, &L, solid, &g) != ORC_OK) return ORC_EINVAL;
    int rc = work_alloc(&L, g.N, &w);
    if (rc == ORC_OK) rc = macro_phases(p, &L, &g, solid, phi, drho, f, &w);
    if (rc == ORC_OK) {
        int64_t N = g.N;
        for (int64_t n = 0; n < N; ++n) {
            if (rho) rho[n] = w.rho[n];
            for (int d = 0; d < L.D; ++d) {
                if (u) u[d * N + n] = w.u[d * N + n];
                if (force) force[d * N + n] = w.F[d * N + n];
            }
        }
    }
    work_free(&w);
    geom_free(&g);
    return rc;
}

int orc_loss(const orc_params* p, const uint8_t* solid, const double* phi,
             const double* drho, const double* f0, int64_t nsteps,
             const double* target, double* loss) {
    lat_t L;
    if (check_params(p) != ORC_OK || get_lat(p->lattice, &L) != ORC_OK)
        return ORC_EINVAL;
    int64_t N = (int64_t)p->nx * p->ny * p->nz;
    double* f = (double*)malloc(sizeof(double) * (size_t)(L.Q * N));
    if (!f) return ORC_EINVAL;
    memcpy(f, f0, sizeof(double) * (size_t)(L.Q * N));
    int rc = orc_run(p, solid, phi, drho, f, nsteps);
    if (rc == ORC_OK) {
        /* L = sum over fluid nodes of (rho_T - rho_target)^2 */
        double s = 0.0;
        for (int64_t n = 0; n < N; ++n) {
            if (solid[n]) continue;
            double r = 0.0;
            for (int a = 0; a < L.Q; ++a) r += f[a * N + n];
            s += (r - target[n]) * (r - target[n]);
        }
        *loss = s;
    }
    free(f);
    return rc;
}
#else  /* ORC_COMPLEX */
int orc_loss_grad_cs(const orc_params* p, const uint8_t* solid,
                     const double* phi, const double* drho, const double* f0,
                     int64_t nsteps, const double* target, int32_t which,
                     int64_t k, double h, double* loss, double* dloss) {
    lat_t L;
    geom_t g;
    if (check_params(p) != ORC_OK || get_lat(p->lattice, &L) != ORC_OK)
        return ORC_EINVAL;
    if (geom_build(p, &L, solid, &g) != ORC_OK) return ORC_EINVAL;
    int64_t N = g.N, nw = g.nwall;
    if (k < 0 || k >= nw || (which != 0 && which != 1)) {
        geom_free(&g);
        return ORC_EINVAL;
    }
    real* cphi = (real*)malloc(sizeof(real) * (size_t)(nw > 0 ? nw : 1));
    real* cdr = (real*)malloc(sizeof(real) * (size_t)(nw > 0 ? nw : 1));
    real* f = (real*)malloc(sizeof(real) * (size_t)(L.Q * N));
    int rc = (cphi && cdr && f) ? ORC_OK : ORC_EINVAL;
    if (rc == ORC_OK) {
        for (int64_t i = 0; i < nw; ++i) {
            cphi[i] = phi[i];
            cdr[i] = drho[i];
        }
        if (which == 0) cphi[k] += I * h;
        else cdr[k] += I * h;
        for (int64_t i = 0; i < (int64_t)L.Q * N; ++i) f[i] = f0[i];
        rc = run_steps(p, &L, &g, solid, cphi, cdr, f, nsteps);
    }
    if (rc == ORC_OK) {
        real s = 0.0;
        for (int64_t n = 0; n < N; ++n) {
            if (solid[n]) continue;
            real r = 0.0;
            for (int a = 0; a < L.Q; ++a) r += f[a * N + n];
            s += (r - target[n]) * (r - target[n]);
        }
        *loss = creal(s);
        *dloss = cimag(s) / h;
    }
    free(cphi);
    free(cdr);
    free(f);
    geom_free(&g);
    return rc;
}

int orc_state_tangent_cs(const orc_params* p, const uint8_t* solid,
                         const double* phi, const double* drho,
                         const double* f0, const double* df0, int64_t nsteps,
                         double h, double* f_out, double* df_out) {
    lat_t L;
    geom_t g;
    if (check_params(p) != ORC_OK || get_lat(p->lattice, &L) != ORC_OK)
        return ORC_EINVAL;
    if (geom_build(p, &L, solid, &g) != ORC_OK) return ORC_EINVAL;
    int64_t N = g.N, nw = g.nwall;
    real* cphi = (real*)malloc(sizeof(real) * (size_t)(nw > 0 ? nw : 1));
    real* cdr = (real*)malloc(sizeof(real) * (size_t)(nw > 0 ? nw : 1));
    real* f = (real*)malloc(sizeof(real) * (size_t)(L.Q * N));
    int rc = (cphi && cdr && f) ? ORC_OK : ORC_EINVAL;
    if (rc == ORC_OK) {
        for (int64_t i = 0; i < nw; ++i) {
            cphi[i] = phi[i];
            cdr[i] = drho[i];
        }
        for (int64_t i = 0; i < (int64_t)L.Q * N; ++i) f[i] = f0[i] + I * h * df0[i];
        rc = run_steps(p, &L, &g, solid, cphi, cdr, f, nsteps);
    }
    if (rc == ORC_OK)
        for (int64_t i = 0; i < (int64_t)L.Q * N; ++i) {
            f_out[i] = creal(f[i]);
            df_out[i] = cimag(f[i]) / h;
        }
    free(cphi);
    free(cdr);
    free(f);
    geom_free(&g);
    return rc;
}
#endif

#ifndef ORC_COMPLEX
int orc_get_threads(void) {
#ifdef _OPENMP
    extern int omp_get_max_threads(void);
    return omp_get_max_threads();
#else
    return 1;
#endif
}
#endif
