// adjoint2d.hip -- discrete adjoint of the fused D2Q9 step.
//
// The step f(t) -> f(t+1) is: density (Eq. 4), psi (Eq. 6), wall virtual
// density (Eqs. 16-17 with the limiter), force (Eq. 5 [+ Eq. 8]), MRT
// collision with the forcing of Eq. 7 (Eq. 2), push streaming with halfway
// bounce-back (Eq. 3).  Its transpose, applied to lam(t+1) = dL/df(t+1),
// gives lam(t) = dL/df(t) and adds the step's share of dL/dphi_b and
// dL/ddrho_b.  Two passes per step:
//
//  collide pass (per fluid node x, forward quantities recomputed from f(t)):
//    lam*_a(x) = lam_a(t+1) at x + e_a, or lam_opp(a)(t+1) at x when x + e_a
//                is solid (streaming transposed),
//    VJP of the collision -> dL/df(x) through the moments, dL/dF(x) and the
//    sigma term's dL/dF_m(x), dL/dpsi(x);
//    own-node part of the density path: dpsi/drho(x) * (dL/dpsi from the
//    sigma term and from psi(x) multiplying the Eq. 5 sum);
//    writes lam(t) partial = dL/df(x) + that density term, and the per-node
//    B(x) = dL/dF_m(x) (total), psi(x), rho(x) for the gather pass.
//  gather pass (per node):
//    dL/dpsi(y) += sum over fluid x = y - e_a of -G w_a psi(x) B(x).e_a
//    (Eq. 5 transposed: psi(y) enters the force of each fluid neighbour);
//    wall node b: r = phi_b rho_ave - drho_b, rho_w = clamp(r),
//    dL/dr = [rho_g <= r <= rho_l] dpsi/drho(rho_w) dL/dpsi(b);
//    dL/dphi_b += dL/dr rho_ave, dL/ddrho_b -= dL/dr, and each fluid
//    neighbour x = b + e_a gets w_a phi_b dL/dr / sum_fluid(w) (Eq. 17);
//    fluid y: ext(y) = dpsi/drho(y) * gathered dL/dpsi(y) + wall terms.
// lam(t) = partial + ext (ext broadcast to all directions).
// Built twice: LBM_PREC == 4 holds the FP32 instantiations (compiled with
// FMA contraction), LBM_PREC == 8 the FP64 ones (no contraction, so that
// FP64 follows the rounding steps of a plain scalar evaluation).  Without
// LBM_PREC both are instantiated.
#ifndef LBM_PREC
#define LBM_PREC 0
#endif
#include "tile2d.hpp"

namespace lbm {

template <typename real, int TX, int TY, int NT, bool BUF>
__global__ __launch_bounds__(NT) void k_adj_collide_d2q9(Coef<real> C, Fields<real> Fd,
                                                         AdjArgs<real> A) {
    using L = D2Q9;
    constexpr int LX = TX + 4, LY = TY + 4;
    constexpr int ROWS = NT / TX;
    constexpr int RPT = TY / ROWS;
    __shared__ TileLDS<real, TX, TY> S;
    __shared__ real s_ext[LX * LY];
    const int nx = C.nx, ny = C.ny;
    const uint32_t N = (uint32_t)nx * (uint32_t)ny;
    const int gxb = gridDim.x;
    const int bid = remap_xcd(blockIdx.x + gxb * blockIdx.y, gridDim.x * gridDim.y);
    const int x0 = (bid % gxb) * TX, y0 = (bid / gxb) * TY;
    const int tid = threadIdx.x, tx = tid % TX, ty = tid / TX;
    const PopIO<real, BUF> io(Fd.fin, Fd.fout, N, 9);
    const PopIO<real, BUF> lio(A.lam_in, A.lam_out, N, 9);
    bool bad = false;
    real f[RPT][9];
    d2q9_prologue<real, TX, TY, NT, BUF>(C, Fd, io, nx, nx, ny, x0, y0, 0, S, f, bad);

    // ext of lam(t+1) on the tile + 1 halo (pulled by the streaming transpose)
    for (int i = tid; i < (TX + 2) * (TY + 2); i += NT) {
        const int lx = 1 + i % (TX + 2), ly = 1 + i / (TX + 2);
        const int p = ly * LX + lx;
        s_ext[p] = (S.cls[p] == CLS_FLUID) ? A.ext_in[S.row[ly] + S.col[lx]] : real(0);
    }
    __syncthreads();

#pragma unroll
    for (int k = 0; k < RPT; ++k) {
        const int ly = ty + k * ROWS;
        const int gx = x0 + tx, gy = y0 + ly;
        if (gx >= nx || gy >= ny) continue;
        const int p = (ly + 2) * LX + tx + 2;
        const uint32_t n = S.row[ly + 2] + S.col[tx + 2];
        if (S.cls[p] != CLS_FLUID) {
            A.sb[n] = real(0);
            A.sb[(size_t)N + n] = real(0);
            A.sb[(size_t)2 * N + n] = real(0);
            A.sb[(size_t)3 * N + n] = real(0);
            continue;
        }
        const real rho = S.rho[p];
        const real psi_c = S.psi[p];
        real Fm[2], F[2];
        d2q9_force<real, LX>(C, S.cls, S.psi, p, rho, Fm, F);
        // V = sum_a w_a psi(x + e_a) e_a (the Eq. 5 sum) and the SFI vector
        real Vx = real(0), Vy = real(0), sx = real(0), sy = real(0);
#pragma unroll
        for (int a = 1; a < 9; ++a) {
            const int q = p + L::ex[a] + L::ey[a] * LX;
            const real w = real(L::w12[a]) * real(1.0 / 12.0);
            Vx += w * S.psi[q] * real(L::ex[a]);
            Vy += w * S.psi[q] * real(L::ey[a]);
            if (S.cls[q] != CLS_FLUID) {
                sx += w * real(L::ex[a]);
                sy += w * real(L::ey[a]);
            }
        }
        // streaming transposed: pull lam(t+1)
        real lam[9];
#pragma unroll
        for (int a = 0; a < 9; ++a) {
            const int q = p + L::ex[a] + L::ey[a] * LX;
            if (S.cls[q] == CLS_FLUID) {
                const uint32_t m = S.row[ly + 2 + L::ey[a]] + S.col[tx + 2 + L::ex[a]];
                lam[a] = lio.ld(a, m) + s_ext[q];
            } else {
                lam[a] = lio.ld(L::opp[a], n) + s_ext[p];
            }
        }
        real gf[9], rb, Fb[2], Fmb[2], psib;
        collide_vjp_d2q9<real>(C, f[k], rho, F, Fm, psi_c, lam, gf, rb, Fb, Fmb, psib);
        // the cohesive force enters F and the sigma term
        const real Bx = Fb[0] + Fmb[0], By = Fb[1] + Fmb[1];
        // psi(x) multiplies the Eq. 5 sum: F_m = -G psi(x) V
        psib += -C.G * (Bx * Vx + By * Vy);
        real dens = dpsi_drho(C, rho, psi_c) * psib;
        if (C.scheme == WET_SFI) dens += -C.G_w * (Fb[0] * sx + Fb[1] * sy);
#pragma unroll
        for (int a = 0; a < 9; ++a) lio.st(a, n, gf[a] + dens);
        A.sb[n] = Bx;
        A.sb[(size_t)N + n] = By;
        A.sb[(size_t)2 * N + n] = psi_c;
        A.sb[(size_t)3 * N + n] = rho;
    }
    (void)bad;
}

template <typename real, int TX, int TY, int NT>
__global__ __launch_bounds__(NT) void k_adj_gather_d2q9(Coef<real> C, Fields<real> Fd,
                                                        AdjArgs<real> A) {
    using L = D2Q9;
    constexpr int LX = TX + 4, LY = TY + 4;
    constexpr int ROWS = NT / TX;
    constexpr int RPT = TY / ROWS;
    __shared__ uint8_t s_cls[LX * LY];
    __shared__ real s_bx[LX * LY], s_by[LX * LY], s_psi[LX * LY], s_rho[LX * LY];
    __shared__ real s_q[LX * LY];  // w-normalised phi * dL/dr of wall nodes
    __shared__ uint32_t s_col[LX], s_row[LY];
    const int nx = C.nx, ny = C.ny;
    const uint32_t N = (uint32_t)nx * (uint32_t)ny;
    const int gxb = gridDim.x;
    const int bid = remap_xcd(blockIdx.x + gxb * blockIdx.y, gridDim.x * gridDim.y);
    const int x0 = (bid % gxb) * TX, y0 = (bid / gxb) * TY;
    const int tid = threadIdx.x, tx = tid % TX, ty = tid / TX;

    for (int i = tid; i < LX + LY; i += NT) {
        if (i < LX) s_col[i] = (uint32_t)wrapi(x0 - 2 + i, nx);
        else s_row[i - LX] = (uint32_t)wrapi(y0 - 2 + (i - LX), ny) * (uint32_t)nx;
    }
    __syncthreads();
    for (int i = tid; i < LX * LY; i += NT) {
        const int lx = i % LX, ly = i / LX;
        const uint32_t n = s_row[ly] + s_col[lx];
        const uint8_t c = Fd.cls[n];
        s_cls[i] = c;
        const bool fl = (c == CLS_FLUID);
        s_bx[i] = fl ? A.sb[n] : real(0);
        s_by[i] = fl ? A.sb[(size_t)N + n] : real(0);
        s_psi[i] = fl ? A.sb[(size_t)2 * N + n] : real(0);
        s_rho[i] = fl ? A.sb[(size_t)3 * N + n] : real(0);
        s_q[i] = real(0);
    }
    __syncthreads();

    // dL/dpsi at LDS position p gathered from the forces of its fluid
    // neighbours x = p - e_a
    auto psi_bar_gather = [&](int p) {
        real s = real(0);
#pragma unroll
        for (int a = 1; a < 9; ++a) {
            const int q = p - L::ex[a] - L::ey[a] * LX;
            if (s_cls[q] == CLS_FLUID) {
                const real w = real(L::w12[a]) * real(1.0 / 12.0);
                s += w * s_psi[q] * (s_bx[q] * real(L::ex[a]) + s_by[q] * real(L::ey[a]));
            }
        }
        return -C.G * s;
    };

    if (C.scheme == WET_IVD) {
        for (int i = tid; i < (TX + 2) * (TY + 2); i += NT) {
            const int lx = 1 + i % (TX + 2), ly = 1 + i / (TX + 2);
            const int p = ly * LX + lx;
            if (s_cls[p] != CLS_WALL) continue;
            real num = real(0), den = real(0);
#pragma unroll
            for (int a = 1; a < 9; ++a) {
                const int q = p + L::ex[a] + L::ey[a] * LX;
                if (s_cls[q] == CLS_FLUID) {
                    const real w = real(L::w12[a]) * real(1.0 / 12.0);
                    num += w * s_rho[q];
                    den += w;
                }
            }
            const real rave = num / den;
            const int kw = Fd.widx[s_row[ly] + s_col[lx]];
            const real ph = Fd.phi[kw];
            const real r = ph * rave - Fd.drho[kw];
            real rw = r > C.rho_l ? C.rho_l : r;
            rw = rw < C.rho_g ? C.rho_g : rw;
            const bool pass = (r <= C.rho_l) && (r >= C.rho_g);
            bool dummy = false;
            const real psw = psi_of(C, rw, dummy);
            const real rbar = pass ? dpsi_drho(C, rw, psw) * psi_bar_gather(p) : real(0);
            s_q[p] = ph * rbar / den;
            // the owning tile accumulates the parameter gradients
            const bool own = lx >= 2 && lx < TX + 2 && ly >= 2 && ly < TY + 2 &&
                             x0 + lx - 2 < nx && y0 + ly - 2 < ny;
            if (own) {
                A.grad_phi[kw] += rbar * rave;
                A.grad_drho[kw] -= rbar;
            }
        }
        __syncthreads();
    }

#pragma unroll
    for (int k = 0; k < RPT; ++k) {
        const int ly = ty + k * ROWS;
        const int gx = x0 + tx, gy = y0 + ly;
        if (gx >= nx || gy >= ny) continue;
        const int p = (ly + 2) * LX + tx + 2;
        const uint32_t n = s_row[ly + 2] + s_col[tx + 2];
        if (s_cls[p] != CLS_FLUID) {
            A.ext_out[n] = real(0);
            continue;
        }
        real e = dpsi_drho(C, s_rho[p], s_psi[p]) * psi_bar_gather(p);
        if (C.scheme == WET_IVD) {
#pragma unroll
            for (int a = 1; a < 9; ++a) {
                const int q = p - L::ex[a] - L::ey[a] * LX;
                if (s_cls[q] == CLS_WALL) e += real(L::w12[a]) * real(1.0 / 12.0) * s_q[q];
            }
        }
        A.ext_out[n] = e;
    }
}

// seed: kind 0 -> lam(T) = dL/drho(T) on every direction (partial 0, ext =
// seed on fluid nodes); kind 1 -> lam(T) = seed ([9][N]), ext 0.
template <typename real>
__global__ void k_adj_seed(int kind, const uint8_t* __restrict__ cls, const real* __restrict__ seed,
                           real* __restrict__ lam, real* __restrict__ ext, uint32_t N) {
    const uint32_t n = blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= N) return;
    const bool fl = cls[n] == CLS_FLUID;
    for (int a = 0; a < 9; ++a)
        lam[(size_t)a * N + n] = (kind == 1 && fl) ? seed[(size_t)a * N + n] : real(0);
    ext[n] = (kind == 0 && fl) ? seed[n] : real(0);
}

// lam = partial + ext, zero on solid nodes
template <typename real>
__global__ void k_adj_finish(const uint8_t* __restrict__ cls, const real* __restrict__ lam,
                             const real* __restrict__ ext, real* __restrict__ out, uint32_t N) {
    const uint32_t n = blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= N) return;
    const bool fl = cls[n] == CLS_FLUID;
    for (int a = 0; a < 9; ++a)
        out[(size_t)a * N + n] = fl ? lam[(size_t)a * N + n] + ext[n] : real(0);
}

// ----------------------------------------------------------------- launch
// FP32 uses 16 x 16 tiles.  Their halo share is that of 64 x 8 tiles, and on
// the small lattices the adjoint is run on they give twice the workgroups
// (256 on a 256^2 lattice instead of 128, for 256 CUs).  The adjoint step on
// that lattice went from 2.3x to 1.6x the forward step.
template <typename real>
struct AdjTile;
template <>
struct AdjTile<float> {
    static constexpr int TX = 16, TY = 16, NT = 256;
};
template <>
struct AdjTile<double> {
    static constexpr int TX = 64, TY = 4, NT = 256;
};

template <typename real>
hipError_t launch_adjoint2d(const Coef<real>& C, const Fields<real>& F, const AdjArgs<real>& A,
                            hipStream_t s) {
    using T = AdjTile<real>;
    dim3 grid((C.nx + T::TX - 1) / T::TX, (C.ny + T::TY - 1) / T::TY);
    const bool buf = (uint64_t)9 * C.nx * C.ny * sizeof(real) <= 0xFFFFFFFFull;
    if (buf)
        hipLaunchKernelGGL((k_adj_collide_d2q9<real, T::TX, T::TY, T::NT, true>), grid, dim3(T::NT),
                           0, s, C, F, A);
    else
        hipLaunchKernelGGL((k_adj_collide_d2q9<real, T::TX, T::TY, T::NT, false>), grid,
                           dim3(T::NT), 0, s, C, F, A);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((k_adj_gather_d2q9<real, T::TX, T::TY, T::NT>), grid, dim3(T::NT), 0, s, C,
                       F, A);
    return hipGetLastError();
}

template <typename real>
hipError_t launch_adj_seed(int kind, const uint8_t* cls, const real* seed, real* lam, real* ext,
                           uint32_t N, hipStream_t s) {
    hipLaunchKernelGGL(k_adj_seed<real>, dim3((N + 255) / 256), dim3(256), 0, s, kind, cls, seed,
                       lam, ext, N);
    return hipGetLastError();
}

template <typename real>
hipError_t launch_adj_finish(const uint8_t* cls, const real* lam, const real* ext, real* out,
                             uint32_t N, hipStream_t s) {
    hipLaunchKernelGGL(k_adj_finish<real>, dim3((N + 255) / 256), dim3(256), 0, s, cls, lam, ext,
                       out, N);
    return hipGetLastError();
}

#if LBM_PREC != 8
template hipError_t launch_adjoint2d<float>(const Coef<float>&, const Fields<float>&,
                                            const AdjArgs<float>&, hipStream_t);
#endif
#if LBM_PREC != 4
template hipError_t launch_adjoint2d<double>(const Coef<double>&, const Fields<double>&,
                                             const AdjArgs<double>&, hipStream_t);
#endif
#if LBM_PREC != 8
template hipError_t launch_adj_seed<float>(int, const uint8_t*, const float*, float*, float*,
                                           uint32_t, hipStream_t);
#endif
#if LBM_PREC != 4
template hipError_t launch_adj_seed<double>(int, const uint8_t*, const double*, double*, double*,
                                            uint32_t, hipStream_t);
#endif
#if LBM_PREC != 8
template hipError_t launch_adj_finish<float>(const uint8_t*, const float*, const float*, float*,
                                             uint32_t, hipStream_t);
#endif
#if LBM_PREC != 4
template hipError_t launch_adj_finish<double>(const uint8_t*, const double*, const double*, double*,
                                              uint32_t, hipStream_t);
#endif

}  // namespace lbm
