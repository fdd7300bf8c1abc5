// step2d.hip -- fused D2Q9 time step for gfx950.
//
// One launch advances the whole lattice by one time step (Sec. II A,
// Sec. III B): density (Eq. 4), pseudopotential (Eq. 6), wall virtual
// density (Eqs. 16-17 + limiter, or the constant / SFI variants), force
// (Eq. 5, Eq. 8), velocity (Eq. 4), MRT collision with the forcing of Eq. 7
// (Eq. 2) and push streaming with halfway bounce-back (Eq. 3, Fig. 3).
//
// The force at a node needs psi of its 8 neighbours at the same time level,
// and psi of a wall neighbour needs rho of that wall node's fluid
// neighbours.  Each workgroup therefore owns a TX x TY tile and rebuilds
// rho on the tile plus a 2-node halo and psi (with the wall virtual
// densities) on the tile plus a 1-node halo in LDS.  Halo populations are
// re-read (they are served by L2 / Infinity Cache, not HBM, when adjacent
// tiles run close in time); each owned node's populations are read once
// into registers, so the HBM traffic stays close to one read and one write
// of f per fluid node.
//
// State: post-streaming populations, SoA f[a*N + n]; fin -> fout ping-pong.
// Only fluid slots of fout are written; a population that would enter a
// solid node is written back to its origin in the opposite direction.
#include "lbm_device.hpp"
#include "lbm_kernels.hpp"

namespace lbm {

template <typename real, int TX, int TY, int NT, int MODE>
__global__ __launch_bounds__(NT) void k_step_d2q9(Coef<real> C, Fields<real> Fd,
                                                  FieldOut<real> Out) {
    using L = D2Q9;
    constexpr int LX = TX + 4, LY = TY + 4;  // tile + 2-node halo
    constexpr int ROWS = NT / TX;
    constexpr int RPT = TY / ROWS;  // owned nodes per thread
    static_assert(NT % TX == 0 && TY % ROWS == 0, "tile shape");
    constexpr int RING = 4 * LX + 4 * TY;

    __shared__ uint8_t s_cls[LX * LY];
    __shared__ real s_rho[LX * LY];
    __shared__ real s_psi[LX * LY];

    const int nx = C.nx, ny = C.ny;
    const size_t N = (size_t)nx * ny;
    const int x0 = blockIdx.x * TX, y0 = blockIdx.y * TY;
    const int tid = threadIdx.x, tx = tid % TX, ty = tid / TX;
    bool bad = false;

    // node classes of the tile + 2 halo
    for (int i = tid; i < LX * LY; i += NT) {
        int lx = i % LX, ly = i / LX;
        int gx = wrapi(x0 - 2 + lx, nx), gy = wrapi(y0 - 2 + ly, ny);
        s_cls[i] = Fd.cls[(size_t)gy * nx + gx];
    }
    __syncthreads();

    // owned tile nodes: populations into registers, density into LDS
    real f[RPT][9];
#pragma unroll
    for (int k = 0; k < RPT; ++k) {
        const int ly = ty + k * ROWS;
        const int p = (ly + 2) * LX + tx + 2;
        const size_t n = (size_t)wrapi(y0 + ly, ny) * nx + wrapi(x0 + tx, nx);
        real r = real(0);
        if (s_cls[p] == CLS_FLUID) {
#pragma unroll
            for (int a = 0; a < 9; ++a) f[k][a] = Fd.fin[a * N + n];
            r = f[k][0];
#pragma unroll
            for (int a = 1; a < 9; ++a) r += f[k][a];
        } else {
#pragma unroll
            for (int a = 0; a < 9; ++a) f[k][a] = real(0);
        }
        s_rho[p] = r;
    }
    // halo ring: density only
    for (int j = tid; j < RING; j += NT) {
        int lx, ly;
        if (j < 2 * LX) {
            ly = j / LX;
            lx = j % LX;
        } else if (j < 4 * LX) {
            const int jj = j - 2 * LX;
            ly = TY + 2 + jj / LX;
            lx = jj % LX;
        } else {
            const int jj = j - 4 * LX;
            ly = 2 + jj / 4;
            const int c = jj % 4;
            lx = c < 2 ? c : TX + c;
        }
        const int p = ly * LX + lx;
        real r = real(0);
        if (s_cls[p] == CLS_FLUID) {
            const size_t n = (size_t)wrapi(y0 - 2 + ly, ny) * nx + wrapi(x0 - 2 + lx, nx);
            r = Fd.fin[n];
#pragma unroll
            for (int a = 1; a < 9; ++a) r += Fd.fin[a * N + n];
        }
        s_rho[p] = r;
    }
    __syncthreads();

    // psi on tile + 1 halo; wall nodes first get their virtual density
    for (int i = tid; i < (TX + 2) * (TY + 2); i += NT) {
        const int lx = 1 + i % (TX + 2), ly = 1 + i / (TX + 2);
        const int p = ly * LX + lx;
        const uint8_t c = s_cls[p];
        real ps = real(0);
        if (c == CLS_FLUID) {
            ps = psi_of(C, s_rho[p], bad);
        } else if (c == CLS_WALL) {
            if (C.scheme == WET_IVD) {
                // Eq. 17: w-weighted mean over the fluid neighbours
                real num = real(0), den = real(0);
                bool first = true;
#pragma unroll
                for (int a = 1; a < 9; ++a) {
                    const int q = p + L::ex[a] + L::ey[a] * LX;
                    if (s_cls[q] == CLS_FLUID) {
                        const real w = real(L::w12[a]) * real(1.0 / 12.0);
                        num = first ? w * s_rho[q] : num + w * s_rho[q];
                        den = first ? w : den + w;
                        first = false;
                    }
                }
                const real rave = num / den;
                const size_t n = (size_t)wrapi(y0 - 2 + ly, ny) * nx + wrapi(x0 - 2 + lx, nx);
                const int kw = Fd.widx[n];
                // Eq. 16 (phi scales, drho shifts) and the limiter
                real rw = Fd.phi[kw] * rave - Fd.drho[kw];
                rw = rw > C.rho_l ? C.rho_l : rw;
                rw = rw < C.rho_g ? C.rho_g : rw;
                s_rho[p] = rw;
                ps = psi_of(C, rw, bad);
            } else if (C.scheme == WET_VD) {
                s_rho[p] = C.rho_w;
                ps = C.psi_w;
            } else {
                s_rho[p] = real(0);
            }
        }
        s_psi[p] = ps;
    }
    __syncthreads();

    double d_sum = 0.0;
    real d_umax = real(0), d_rmin = real(1e30), d_rmax = real(-1e30);
    int d_cnt = 0;

#pragma unroll
    for (int k = 0; k < RPT; ++k) {
        const int ly = ty + k * ROWS;
        const int gx = x0 + tx, gy = y0 + ly;
        if (gx >= nx || gy >= ny) continue;  // ragged tile: not owned
        const int p = (ly + 2) * LX + tx + 2;
        const size_t n = (size_t)gy * nx + gx;
        const uint8_t c = s_cls[p];
        if (c != CLS_FLUID) {
            if (MODE == MODE_FIELDS) {
                if (Out.rho) Out.rho[n] = (c == CLS_WALL) ? s_rho[p] : real(0);
                if (Out.u) {
                    Out.u[n] = real(0);
                    Out.u[N + n] = real(0);
                }
            }
            continue;
        }
        const real rho = s_rho[p];
        const real psi_c = s_psi[p];
        // Eq. 5 (and Eq. 8 for the solid-fluid interaction)
        real smx = real(0), smy = real(0), sax = real(0), say = real(0);
#pragma unroll
        for (int a = 1; a < 9; ++a) {
            const int q = p + L::ex[a] + L::ey[a] * LX;
            const real w = real(L::w12[a]) * real(1.0 / 12.0);
            const real wp = w * s_psi[q];
            if (L::ex[a] == 1) smx += wp;
            if (L::ex[a] == -1) smx -= wp;
            if (L::ey[a] == 1) smy += wp;
            if (L::ey[a] == -1) smy -= wp;
            if (C.scheme == WET_SFI && s_cls[q] != CLS_FLUID) {
                if (L::ex[a] == 1) sax += w;
                if (L::ex[a] == -1) sax -= w;
                if (L::ey[a] == 1) say += w;
                if (L::ey[a] == -1) say -= w;
            }
        }
        real Fm[2], F[2];
        Fm[0] = -C.G * psi_c * smx;
        Fm[1] = -C.G * psi_c * smy;
        const real fax = (C.scheme == WET_SFI) ? -C.G_w * rho * sax : real(0);
        const real fay = (C.scheme == WET_SFI) ? -C.G_w * rho * say : real(0);
        F[0] = Fm[0] + fax + C.body[0];
        F[1] = Fm[1] + fay + C.body[1];

        if (MODE == MODE_FIELDS) {
            const real jx = f[k][1] - f[k][3] + f[k][5] - f[k][6] - f[k][7] + f[k][8];
            const real jy = f[k][2] - f[k][4] + f[k][5] + f[k][6] - f[k][7] - f[k][8];
            const real ux = (jx + real(0.5) * F[0]) / rho;
            const real uy = (jy + real(0.5) * F[1]) / rho;
            if (Out.rho) Out.rho[n] = rho;
            if (Out.u) {
                Out.u[n] = ux;
                Out.u[N + n] = uy;
            }
            const real um = sqrt(ux * ux + uy * uy);
            d_sum += (double)rho;
            d_umax = um > d_umax ? um : d_umax;
            d_rmin = rho < d_rmin ? rho : d_rmin;
            d_rmax = rho > d_rmax ? rho : d_rmax;
            d_cnt += 1;
            continue;
        }

        real fs[9], u[2];
        collide<L, real>(C, f[k], rho, F, Fm, psi_c, fs, u);
        // push streaming with halfway bounce-back
#pragma unroll
        for (int a = 0; a < 9; ++a) {
            const int q = p + L::ex[a] + L::ey[a] * LX;
            if (s_cls[q] == CLS_FLUID) {
                int tx2 = gx + L::ex[a], ty2 = gy + L::ey[a];
                tx2 = tx2 < 0 ? tx2 + nx : (tx2 >= nx ? tx2 - nx : tx2);
                ty2 = ty2 < 0 ? ty2 + ny : (ty2 >= ny ? ty2 - ny : ty2);
                Fd.fout[a * N + (size_t)ty2 * nx + tx2] = fs[a];
            } else {
                Fd.fout[L::opp[a] * N + n] = fs[a];
            }
        }
    }

    if (MODE == MODE_FIELDS && Out.part) {
        block_reduce_diag<NT>(d_sum, d_umax, d_rmin, d_rmax, d_cnt,
                              Out.part + 5 * (blockIdx.y * gridDim.x + blockIdx.x));
    }
    if (bad) Fd.flag[0] = 1;
}

// ----------------------------------------------------------------- launch
template <typename real>
struct Tile2D;
template <>
struct Tile2D<float> {
    static constexpr int TX = 64, TY = 16, NT = 256;
};
template <>
struct Tile2D<double> {
    static constexpr int TX = 64, TY = 8, NT = 256;
};

template <typename real>
int grid2d_blocks(int nx, int ny) {
    using T = Tile2D<real>;
    return ((nx + T::TX - 1) / T::TX) * ((ny + T::TY - 1) / T::TY);
}

template <typename real>
hipError_t launch_step2d(const Coef<real>& C, const Fields<real>& F, const FieldOut<real>& O,
                         int mode, hipStream_t s) {
    using T = Tile2D<real>;
    dim3 grid((C.nx + T::TX - 1) / T::TX, (C.ny + T::TY - 1) / T::TY);
    if (mode == MODE_STEP)
        hipLaunchKernelGGL((k_step_d2q9<real, T::TX, T::TY, T::NT, MODE_STEP>), grid, dim3(T::NT),
                           0, s, C, F, O);
    else
        hipLaunchKernelGGL((k_step_d2q9<real, T::TX, T::TY, T::NT, MODE_FIELDS>), grid,
                           dim3(T::NT), 0, s, C, F, O);
    return hipGetLastError();
}

template int grid2d_blocks<float>(int, int);
template int grid2d_blocks<double>(int, int);
template hipError_t launch_step2d<float>(const Coef<float>&, const Fields<float>&,
                                         const FieldOut<float>&, int, hipStream_t);
template hipError_t launch_step2d<double>(const Coef<double>&, const Fields<double>&,
                                          const FieldOut<double>&, int, hipStream_t);

}  // namespace lbm
