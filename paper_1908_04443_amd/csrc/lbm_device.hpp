// lbm_device.hpp -- device-side lattice tables, kernel argument block and
// per-node physics (equation of state, pseudopotential, MRT collision) shared
// by the step, field and adjoint kernels.
//
// Lattice units: dx = dt = 1, c = 1, cs^2 = 1/3.  Velocity order:
//   D2Q9  rest, +x, +y, -x, -y, (1,1), (-1,1), (-1,-1), (1,-1)
//   D3Q19 rest, +x, -x, +y, -y, +z, -z, then the face diagonals in opposite
//         pairs (1,1,0) (-1,-1,0) (1,-1,0) (-1,1,0) (1,0,1) (-1,0,-1)
//         (1,0,-1) (-1,0,1) (0,1,1) (0,-1,-1) (0,1,-1) (0,-1,1).
// Moment rows follow the orthogonal MRT bases (Lallemand-Luo in 2-D,
// d'Humieres et al. in 3-D) in the row order of the relaxation matrix of
// Eq. 2.  All moment coefficients are small integers, so the transforms are
// written as fully unrolled integer-coefficient sums: zero entries vanish at
// compile time and the cost is about a quarter of a dense product.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lbm {

// node classes stored per node (one byte)
enum : uint8_t { CLS_FLUID = 0, CLS_SOLID = 1, CLS_WALL = 3 };
enum { WET_IVD = 0, WET_VD = 1, WET_SFI = 2 };
enum { EOS_CS = 0, EOS_PR = 1 };

// ------------------------------------------------------------------ D2Q9
struct D2Q9 {
    static constexpr int Q = 9, D = 2;
    static constexpr int ex[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
    static constexpr int ey[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
    static constexpr int ez[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
    static constexpr int opp[9] = {0, 3, 4, 1, 2, 7, 8, 5, 6};
    // lattice weights t_a * 36 and force-stencil weights w_a * 12 (Eq. 5:
    // 1/3 for |e|^2 = 1, 1/12 for |e|^2 = 2)
    static constexpr int t36[9] = {16, 4, 4, 4, 4, 1, 1, 1, 1};
    static constexpr int w12[9] = {0, 4, 4, 4, 4, 1, 1, 1, 1};
    static constexpr int M[9][9] = {
        {1, 1, 1, 1, 1, 1, 1, 1, 1},
        {-4, -1, -1, -1, -1, 2, 2, 2, 2},
        {4, -2, -2, -2, -2, 1, 1, 1, 1},
        {0, 1, 0, -1, 0, 1, -1, -1, 1},
        {0, -2, 0, 2, 0, 1, -1, -1, 1},
        {0, 0, 1, 0, -1, 1, 1, -1, -1},
        {0, 0, -2, 0, 2, 1, 1, -1, -1},
        {0, 1, -1, 1, -1, 0, 0, 0, 0},
        {0, 0, 0, 0, 0, 1, -1, 1, -1}};
    // squared norms of the rows: M^-1 = M^T diag(1/norm)
    static constexpr int norm[9] = {9, 36, 36, 6, 12, 6, 12, 4, 4};
};

// ----------------------------------------------------------------- D3Q19
struct D3Q19 {
    static constexpr int Q = 19, D = 3;
    static constexpr int ex[19] = {0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1, 0, 0, 0, 0};
    static constexpr int ey[19] = {0, 0, 0, 1, -1, 0, 0, 1, -1, -1, 1, 0, 0, 0, 0, 1, -1, 1, -1};
    static constexpr int ez[19] = {0, 0, 0, 0, 0, 1, -1, 0, 0, 0, 0, 1, -1, -1, 1, 1, -1, -1, 1};
    static constexpr int opp[19] = {0, 2, 1, 4, 3, 6, 5, 8, 7, 10, 9, 12, 11, 14, 13, 16, 15, 18, 17};
    static constexpr int t36[19] = {12, 2, 2, 2, 2, 2, 2, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1};
    static constexpr int w12[19] = {0, 2, 2, 2, 2, 2, 2, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1};
    static constexpr int M[19][19] = {
        {1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1},
        {-30, -11, -11, -11, -11, -11, -11, 8, 8, 8, 8, 8, 8, 8, 8, 8, 8, 8, 8},
        {12, -4, -4, -4, -4, -4, -4, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1},
        {0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1, 0, 0, 0, 0},
        {0, -4, 4, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1, 0, 0, 0, 0},
        {0, 0, 0, 1, -1, 0, 0, 1, -1, -1, 1, 0, 0, 0, 0, 1, -1, 1, -1},
        {0, 0, 0, -4, 4, 0, 0, 1, -1, -1, 1, 0, 0, 0, 0, 1, -1, 1, -1},
        {0, 0, 0, 0, 0, 1, -1, 0, 0, 0, 0, 1, -1, -1, 1, 1, -1, -1, 1},
        {0, 0, 0, 0, 0, -4, 4, 0, 0, 0, 0, 1, -1, -1, 1, 1, -1, -1, 1},
        {0, 2, 2, -1, -1, -1, -1, 1, 1, 1, 1, 1, 1, 1, 1, -2, -2, -2, -2},
        {0, -4, -4, 2, 2, 2, 2, 1, 1, 1, 1, 1, 1, 1, 1, -2, -2, -2, -2},
        {0, 0, 0, 1, 1, -1, -1, 1, 1, 1, 1, -1, -1, -1, -1, 0, 0, 0, 0},
        {0, 0, 0, -2, -2, 2, 2, 1, 1, 1, 1, -1, -1, -1, -1, 0, 0, 0, 0},
        {0, 0, 0, 0, 0, 0, 0, 1, 1, -1, -1, 0, 0, 0, 0, 0, 0, 0, 0},
        {0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 1, 1, -1, -1},
        {0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 1, 1, -1, -1, 0, 0, 0, 0},
        {0, 0, 0, 0, 0, 0, 0, 1, -1, 1, -1, -1, 1, -1, 1, 0, 0, 0, 0},
        {0, 0, 0, 0, 0, 0, 0, -1, 1, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1},
        {0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 1, -1, -1, 1, -1, 1, 1, -1}};
    static constexpr int norm[19] = {19, 2394, 252, 10, 40, 10, 40, 10, 40, 36, 72, 12, 24, 4, 4, 4, 8, 8, 8};
};

// --------------------------------------------------------- argument block
// Everything a step needs besides the population buffers.  Built on the
// host from lbm_params; coefficients are pre-converted to the kernel type.
template <typename real>
struct Coef {
    int nx, ny, nz;
    int scheme, eos;
    real eos_a;     // attraction a (CS) ; unused for PR
    real eos_b;     // co-volume b
    real eos_RT;    // R*T
    real eos_aphi;  // a * phi(T) (PR)
    real two_over_G;  // psi^2 = 2 (p - rho/3) / G
    real G;         // interaction strength of Eq. 5
    real rho_w;     // VD constant virtual density
    real psi_w;     // psi(rho_w) for VD
    real G_w;       // SFI adhesion strength
    real rho_g, rho_l;
    real s[19];     // 1/tau per moment row
    real hs[19];    // 1 - s/2 per moment row
    real sig_e;     // 12 sigma / (tau_e - 1/2)  (3-D: 114 sigma / (tau_e - 1/2))
    real sig_eps;   // 12 sigma / (tau_eps - 1/2) (3-D: 0)
    real body[3];
};

template <typename real>
struct Fields {
    const real* fin;
    real* fout;
    const uint8_t* cls;
    const int32_t* widx;   // wall-list position of each wall node, -1 else
    const real* phi;       // per wall node (IVD)
    const real* drho;      // per wall node (IVD)
    int32_t* flag;         // set to 1 when a psi argument is < 0 or NaN
};

__device__ __forceinline__ int wrapi(int v, int n) {
    // any integer into [0, n); tiles may cover the lattice several times
    v %= n;
    return v < 0 ? v + n : v;
}

// ---------------------------------------------------- equation of state
template <typename real>
__device__ __forceinline__ real eos_p(const Coef<real>& C, real rho) {
    if (C.eos == EOS_CS) {
        real h = C.eos_b * real(0.25) * rho;
        real om = real(1) - h;
        real num = real(1) + h + h * h - h * h * h;
        return rho * C.eos_RT * num / (om * om * om) - C.eos_a * rho * rho;
    } else {
        real br = C.eos_b * rho;
        return rho * C.eos_RT / (real(1) - br) -
               C.eos_aphi * rho * rho / (real(1) + real(2) * br - br * br);
    }
}

// psi of Eq. 6; *bad set when the argument is negative or NaN
template <typename real>
__device__ __forceinline__ real psi_of(const Coef<real>& C, real rho, bool& bad) {
    real arg = C.two_over_G * (eos_p(C, rho) - rho * real(1.0 / 3.0));
    if (!(arg >= real(0))) {
        bad = true;
        return real(0);
    }
    return sqrt(arg);
}

// ---------------------------------------------------------- MRT collision
// Post-collision populations of one fluid node (Eq. 2, forcing of Eq. 7):
// m = M f, m* = m - S (m - m_eq) + (I - S/2) Src, f* = M^-1 m*.
// in: f (populations), rho, j = sum e f, F (total force), Fm (cohesive
// force of Eq. 5), psi (own pseudopotential).  out: fs.  Also returns u.
template <typename L, typename real>
__device__ __forceinline__ void collide(const Coef<real>& C, const real* f, real rho,
                                        const real* F, const real* Fm, real psi,
                                        real* fs, real* u_out) {
    constexpr int Q = L::Q;
    real m[Q];
#pragma unroll
    for (int k = 0; k < Q; ++k) {
        real s = real(0);
        bool first = true;
#pragma unroll
        for (int a = 0; a < Q; ++a) {
            if (L::M[k][a] == 0) continue;
            real term = (L::M[k][a] == 1) ? f[a] : (L::M[k][a] == -1) ? -f[a] : real(L::M[k][a]) * f[a];
            s = first ? term : s + term;
            first = false;
        }
        m[k] = s;
    }
    const real inv_rho = real(1) / rho;
    real u[3], Fv[3];
    Fv[0] = F[0];
    Fv[1] = F[1];
    Fv[2] = (L::D == 3) ? F[2] : real(0);
    u[0] = (m[3] + real(0.5) * Fv[0]) * inv_rho;
    u[1] = (m[5] + real(0.5) * Fv[1]) * inv_rho;
    u[2] = (L::D == 3) ? (m[7] + real(0.5) * Fv[2]) * inv_rho : real(0);
    u_out[0] = u[0];
    u_out[1] = u[1];
    if (L::D == 3) u_out[2] = u[2];
    const real uF = u[0] * Fv[0] + u[1] * Fv[1] + u[2] * Fv[2];
    real fm2 = Fm[0] * Fm[0] + Fm[1] * Fm[1];
    if (L::D == 3) fm2 += Fm[2] * Fm[2];
    const real sgm = (psi > real(0)) ? fm2 / (psi * psi) : real(0);
    real meq[Q], src[Q];
    if constexpr (L::Q == 9) {
        const real u2 = u[0] * u[0] + u[1] * u[1];
        meq[0] = rho;
        meq[1] = rho * (real(-2) + real(3) * u2);
        meq[2] = rho * (real(1) - real(3) * u2);
        meq[3] = rho * u[0];
        meq[4] = -rho * u[0];
        meq[5] = rho * u[1];
        meq[6] = -rho * u[1];
        meq[7] = rho * (u[0] * u[0] - u[1] * u[1]);
        meq[8] = rho * u[0] * u[1];
        src[0] = real(0);
        src[1] = real(6) * uF + C.sig_e * sgm;
        src[2] = real(-6) * uF - C.sig_eps * sgm;
        src[3] = Fv[0];
        src[4] = -Fv[0];
        src[5] = Fv[1];
        src[6] = -Fv[1];
        src[7] = real(2) * (u[0] * Fv[0] - u[1] * Fv[1]);
        src[8] = u[0] * Fv[1] + u[1] * Fv[0];
    } else {
        const real ux = u[0], uy = u[1], uz = u[2];
        const real u2 = ux * ux + uy * uy + uz * uz;
        const real pxx = real(2) * ux * ux - uy * uy - uz * uz;
        const real pww = uy * uy - uz * uz;
        meq[0] = rho;
        meq[1] = rho * (real(-11) + real(19) * u2);
        meq[2] = rho * (real(3) - real(5.5) * u2);
        meq[3] = rho * ux;
        meq[4] = real(-2.0 / 3.0) * rho * ux;
        meq[5] = rho * uy;
        meq[6] = real(-2.0 / 3.0) * rho * uy;
        meq[7] = rho * uz;
        meq[8] = real(-2.0 / 3.0) * rho * uz;
        meq[9] = rho * pxx;
        meq[10] = real(-0.5) * rho * pxx;
        meq[11] = rho * pww;
        meq[12] = real(-0.5) * rho * pww;
        meq[13] = rho * ux * uy;
        meq[14] = rho * uy * uz;
        meq[15] = rho * ux * uz;
        meq[16] = real(0);
        meq[17] = real(0);
        meq[18] = real(0);
        const real Fx = Fv[0], Fy = Fv[1], Fz = Fv[2];
        const real sxx = real(2) * ux * Fx - uy * Fy - uz * Fz;
        const real sww = uy * Fy - uz * Fz;
        src[0] = real(0);
        src[1] = real(38) * uF + C.sig_e * sgm;
        src[2] = real(-11) * uF;
        src[3] = Fx;
        src[4] = real(-2.0 / 3.0) * Fx;
        src[5] = Fy;
        src[6] = real(-2.0 / 3.0) * Fy;
        src[7] = Fz;
        src[8] = real(-2.0 / 3.0) * Fz;
        src[9] = real(2) * sxx;
        src[10] = -sxx;
        src[11] = real(2) * sww;
        src[12] = -sww;
        src[13] = ux * Fy + uy * Fx;
        src[14] = uy * Fz + uz * Fy;
        src[15] = ux * Fz + uz * Fx;
        src[16] = real(0);
        src[17] = real(0);
        src[18] = real(0);
    }
    // relax in moment space, scale by the inverse row norms
    real ms[Q];
#pragma unroll
    for (int k = 0; k < Q; ++k) {
        real mk = m[k] - C.s[k] * (m[k] - meq[k]) + C.hs[k] * src[k];
        ms[k] = mk * real(1.0 / L::norm[k]);
    }
#pragma unroll
    for (int a = 0; a < Q; ++a) {
        real s = real(0);
        bool first = true;
#pragma unroll
        for (int k = 0; k < Q; ++k) {
            if (L::M[k][a] == 0) continue;
            real term = (L::M[k][a] == 1) ? ms[k] : (L::M[k][a] == -1) ? -ms[k] : real(L::M[k][a]) * ms[k];
            s = first ? term : s + term;
            first = false;
        }
        fs[a] = s;
    }
}

template <typename L, typename real>
__device__ __forceinline__ real feq(int a, real rho, const real* u) {
    real eu = real(L::ex[a]) * u[0] + real(L::ey[a]) * u[1];
    real uu = u[0] * u[0] + u[1] * u[1];
    if (L::D == 3) {
        eu += real(L::ez[a]) * u[2];
        uu += u[2] * u[2];
    }
    return real(L::t36[a]) * real(1.0 / 36.0) * rho *
           (real(1) + real(3) * eu + real(4.5) * eu * eu - real(1.5) * uu);
}

}  // namespace lbm
