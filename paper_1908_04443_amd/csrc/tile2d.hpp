// tile2d.hpp -- the first half of the fused D2Q9 tile step, shared by the
// step kernels and the adjoint's forward recompute: for a TX x TY tile at
// (x0, y0) it loads node classes of the tile plus a 2-node halo, the
// populations of the owned nodes into registers, the density of the tile
// plus 2-node halo, the wall virtual densities (Eqs. 16-17 with the
// limiter, the constant virtual density, the geometric formulation of
// Eq. 11, or none for Eq. 8) and psi (Eq. 6) on the tile plus a 1-node
// halo, all in LDS.
#pragma once
#include "lbm_device.hpp"
#include "lbm_kernels.hpp"

namespace lbm {

template <typename real, int TX, int TY>
struct TileLDS {
    static constexpr int LX = TX + 4, LY = TY + 4;
    uint8_t cls[LX * LY];
    real rho[LX * LY];
    real psi[LX * LY];
    uint32_t col[LX];  // wrapped x of each halo column
    uint32_t row[LY];  // wrapped y * pitch of each halo row
    int wl_count;      // wall-list length of the tile
};

// LDS position (lx, ly) of halo-ring entry j: two full rows below the tile,
// two full rows above, then two columns on each side of each tile row.
template <int TX, int TY>
__device__ __forceinline__ void ring_pos(int j, int& lx, int& ly) {
    constexpr int LX = TX + 4;
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
}

// w-weighted mean density of the fluid neighbours of LDS position p (Eq. 17)
template <typename real, int LX>
__device__ __forceinline__ real fluid_mean(const uint8_t* cls, const real* rho, int p) {
    using L = D2Q9;
    real num = real(0), den = real(0);
    bool first = true;
#pragma unroll
    for (int a = 1; a < 9; ++a) {
        const int q = p + L::ex[a] + L::ey[a] * LX;
        if (cls[q] == CLS_FLUID) {
            const real w = real(L::w12[a]) * real(1.0 / 12.0);
            num = first ? w * rho[q] : num + w * rho[q];
            den = first ? w : den + w;
            first = false;
        }
    }
    return fdiv(num, den);
}

// Geometric formulation (Eq. 11) at wall position p from its stencil code
// (see build_gf_stencils): the density at each characteristic point
// interpolates its two mesh-line nodes (weight t_k on the second), then the
// max or min of the two points; a void point drops out, two void points
// give the neighbour mean.
template <typename real, int LX>
__device__ __forceinline__ real gf_density(const uint8_t* cls, const real* rho, int p,
                                           int32_t code, real t0, real t1) {
    real r[2];
    bool ok[2];
#pragma unroll
    for (int k = 0; k < 2; ++k) {
        const int f = (code >> (10 * k)) & 0x3FF;
        const int ia = f & 15, ib = (f >> 4) & 15;
        const bool fa = (f >> 8) & 1, fb = (f >> 9) & 1;
        const int qa = p + (ia % 3 - 1) + (ia / 3 - 1) * LX;
        const int qb = p + (ib % 3 - 1) + (ib / 3 - 1) * LX;
        const real t = k == 0 ? t0 : t1;
        ok[k] = fa || fb;
        r[k] = (fa && fb) ? (real(1) - t) * rho[qa] + t * rho[qb]
               : fa       ? rho[qa]
               : fb       ? rho[qb]
                          : real(0);
    }
    if (!ok[0] && !ok[1]) return fluid_mean<real, LX>(cls, rho, p);
    if (!ok[0]) return r[1];
    if (!ok[1]) return r[0];
    const bool take_min = (code >> 20) & 1;
    if (take_min) return r[0] <= r[1] ? r[0] : r[1];
    return r[0] >= r[1] ? r[0] : r[1];
}

// Per-thread entry of the tile's wall list (see wall_list_head)
template <typename real>
struct WallEntry {
    bool on = false, gf = false;
    uint32_t e0 = 0;
    int pos = -1;
    int32_t code = 0;
    real phi = real(0), drho = real(0);
};

// The first wave loads the first 64 entries of the tile's wall list (if the
// context has lists for the scheme); the count goes to LDS.
template <typename real, bool GFW>
__device__ __forceinline__ void wall_list_head(const Coef<real>& C, const Fields<real>& Fd,
                                               int list_tile, int tid, int& lds_count,
                                               WallEntry<real>& we) {
    we.gf = GFW && C.scheme == WET_GF;
    we.on = (C.scheme == WET_IVD || we.gf) && Fd.tw_pack != nullptr;
    if (!we.on) return;
    we.e0 = (uint32_t)list_tile * (uint32_t)Fd.tw_stride;
    if (tid < 64) {
        const int w = Fd.tw_pack[we.e0 + tid];
        we.phi = Fd.tw_phi[we.e0 + tid];
        we.drho = Fd.tw_drho[we.e0 + tid];
        if (we.gf) we.code = Fd.tw_code[we.e0 + tid];
        if (tid < (w >> 16)) we.pos = w & 0xFFFF;
        if (tid == 0) lds_count = w >> 16;
    }
}

// Second phase of the prologue, after the barrier that follows the loads
// (LDS holds the classes and densities of the tile plus a 2-node halo):
// wall virtual densities (Eqs. 16-17 and the limiter, the constant virtual
// density, the geometric formulation of Eq. 11, or none for Eq. 8) and psi
// (Eq. 6) on the tile plus a 1-node halo; ends with a barrier.
template <typename real, int TX, int TY, int NT, bool GFW>
__device__ __forceinline__ void d2q9_psi_phase(const Coef<real>& C, const Fields<real>& Fd,
                                               TileLDS<real, TX, TY>& S, WallEntry<real>& we,
                                               bool& bad) {
    using L = D2Q9;
    constexpr int LX = TX + 4;
    const int tid = threadIdx.x;
    // wall-list entries beyond the first 64
    if (we.on && tid >= 64 && tid < S.wl_count) {
        we.pos = Fd.tw_pack[we.e0 + tid] & 0xFFFF;
        we.phi = Fd.tw_phi[we.e0 + tid];
        we.drho = Fd.tw_drho[we.e0 + tid];
        if (we.gf) we.code = Fd.tw_code[we.e0 + tid];
    }

    // psi on tile + 1 halo; wall nodes first get their virtual density
    // (with a wall list, the listed walls are done below by their entries)
    for (int i = tid; i < (TX + 2) * (TY + 2); i += NT) {
        const int lx = 1 + i % (TX + 2), ly = 1 + i / (TX + 2);
        const int p = ly * LX + lx;
        const uint8_t c = S.cls[p];
        real ps = real(0);
        if (c == CLS_WALL && we.on) continue;
        if (c == CLS_FLUID) {
            ps = psi_of(C, S.rho[p], bad);
        } else if (c == CLS_WALL) {
            if (C.scheme == WET_IVD) {
                // Eq. 17: w-weighted mean over the fluid neighbours
                real num = real(0), den = real(0);
                bool first = true;
#pragma unroll
                for (int a = 1; a < 9; ++a) {
                    const int q = p + L::ex[a] + L::ey[a] * LX;
                    if (S.cls[q] == CLS_FLUID) {
                        const real w = real(L::w12[a]) * real(1.0 / 12.0);
                        num = first ? w * S.rho[q] : num + w * S.rho[q];
                        den = first ? w : den + w;
                        first = false;
                    }
                }
                const real rave = fdiv(num, den);
                const int kw = Fd.widx[S.row[ly] + S.col[lx]];
                // Eq. 16 (phi scales, drho shifts) and the limiter
                real rw = Fd.phi[kw] * rave - Fd.drho[kw];
                rw = rw > C.rho_l ? C.rho_l : rw;
                rw = rw < C.rho_g ? C.rho_g : rw;
                S.rho[p] = rw;
                ps = psi_of(C, rw, bad);
            } else if (we.gf) {
                const int kw = Fd.widx[S.row[ly] + S.col[lx]];
                const real rw = gf_density<real, LX>(S.cls, S.rho, p, Fd.gfcode[kw], Fd.phi[kw],
                                                     Fd.drho[kw]);
                S.rho[p] = rw;
                ps = psi_of(C, rw, bad);
            } else if (C.scheme == WET_VD) {
                S.rho[p] = C.rho_w;
                ps = C.psi_w;
            } else {
                S.rho[p] = real(0);
            }
        }
        S.psi[p] = ps;
    }
    if (we.pos >= 0 && we.gf) {
        const real rw = gf_density<real, LX>(S.cls, S.rho, we.pos, we.code, we.phi, we.drho);
        S.rho[we.pos] = rw;
        S.psi[we.pos] = psi_of(C, rw, bad);
    } else if (we.pos >= 0) {
        // Eq. 17 over the fluid neighbours, Eq. 16 and the limiter
        const int p = we.pos;
        real num = real(0), den = real(0);
        bool first = true;
#pragma unroll
        for (int a = 1; a < 9; ++a) {
            const int q = p + L::ex[a] + L::ey[a] * LX;
            if (S.cls[q] == CLS_FLUID) {
                const real w = real(L::w12[a]) * real(1.0 / 12.0);
                num = first ? w * S.rho[q] : num + w * S.rho[q];
                den = first ? w : den + w;
                first = false;
            }
        }
        real rw = we.phi * fdiv(num, den) - we.drho;
        rw = rw > C.rho_l ? C.rho_l : rw;
        rw = rw < C.rho_g ? C.rho_g : rw;
        S.rho[p] = rw;
        S.psi[p] = psi_of(C, rw, bad);
    }
    __syncthreads();
}

// GFW: the geometric formulation is compiled in (a separate instantiation,
// so that the other schemes keep its registers out of their kernels).
// FLO: populations are loaded for fluid nodes only, once their classes have
// arrived (non-fluid slots are never used).  That saves the lines inside
// solids at the cost of a second dependent round trip per tile.
template <typename real, int TX, int TY, int NT, bool BUF, bool GFW = false, bool FLO = false>
__device__ __forceinline__ void d2q9_prologue(const Coef<real>& C, const Fields<real>& Fd,
                                              const PopIO<real, BUF>& io, const int nx,
                                              const int pitch, const int ny, const int x0,
                                              const int y0,
                                              const int list_tile, TileLDS<real, TX, TY>& S,
                                              real (&f)[TY / (NT / TX)][9], bool& bad) {
    constexpr int LX = TX + 4, LY = TY + 4;
    constexpr int ROWS = NT / TX;
    constexpr int RPT = TY / ROWS;
    static_assert(NT % TX == 0 && TY % ROWS == 0, "tile shape");
    constexpr int RING = 4 * LX + 4 * TY;
    const int tid = threadIdx.x, tx = tid % TX, ty = tid / TX;

    // One load phase: node classes, the populations of the owned nodes and
    // the populations of the halo ring are all issued before any of them is
    // needed, so a tile waits for one memory round trip instead of two.
    // Populations are loaded whatever the node class (solid slots are never
    // used: their density is replaced by 0 below); this costs the lines that
    // lie wholly inside solid regions and saves a dependent round trip.
    const bool inner2 = x0 >= 2 && y0 >= 2 && x0 + TX + 2 <= nx && y0 + TY + 2 <= ny;
    auto node = [&](int lx, int ly) -> uint32_t {
        if (inner2) return (uint32_t)(y0 - 2 + ly) * (uint32_t)pitch + (uint32_t)(x0 - 2 + lx);
        return (uint32_t)wrapi(y0 - 2 + ly, ny) * (uint32_t)pitch +
               (uint32_t)wrapi(x0 - 2 + lx, nx);
    };
    for (int i = tid; i < LX + LY; i += NT) {
        if (i < LX) S.col[i] = (uint32_t)wrapi(x0 - 2 + i, nx);
        else S.row[i - LX] = (uint32_t)wrapi(y0 - 2 + (i - LX), ny) * (uint32_t)pitch;
    }

    // Per-tile wall list (improved virtual density, geometric formulation):
    // the first wave loads the first 64 entries with the other loads of
    // this phase; entries beyond 64 (rare) follow after the barrier.
    WallEntry<real> we;
    wall_list_head<real, GFW>(C, Fd, list_tile, tid, S.wl_count, we);

    // owned tile nodes: populations into registers, density into LDS
    uint8_t oc[RPT];
    uint32_t on[RPT];
#pragma unroll
    for (int k = 0; k < RPT; ++k) {
        const int ly = ty + k * ROWS;
        on[k] = node(tx + 2, ly + 2);
        // FLO with a wall list: a position more than two nodes past the
        // lattice's last column or row (ragged tiles) is nobody's neighbour
        // and stays an empty solid cell.  (psi is needed up to one node past
        // the owned nodes; the list holds no wall beyond that, so no virtual
        // density is formed next to an empty cell.)
        oc[k] = (FLO && we.on && (x0 + tx >= nx + 2 || y0 + ly >= ny + 2))
                    ? (uint8_t)CLS_SOLID
                    : Fd.cls[on[k]];
    }
#pragma unroll
    for (int k = 0; k < RPT; ++k) {
#pragma unroll
        for (int a = 0; a < 9; ++a) f[k][a] = real(0);
        if (!FLO || oc[k] == CLS_FLUID) {
#pragma unroll
            for (int a = 0; a < 9; ++a) f[k][a] = io.ld(a, on[k]);
        }
    }
    // halo ring: density only
    constexpr int JR = (RING + NT - 1) / NT;
    uint8_t rc[JR];
    real rr[JR];
#pragma unroll
    for (int jj = 0; jj < JR; ++jj) {
        const int j = tid + jj * NT;
        rc[jj] = CLS_SOLID;
        rr[jj] = real(0);
        if (j < RING) {
            int lx, ly;
            ring_pos<TX, TY>(j, lx, ly);
            const uint32_t n = node(lx, ly);
            rc[jj] = (FLO && we.on && (x0 - 2 + lx >= nx + 2 || y0 - 2 + ly >= ny + 2))
                         ? (uint8_t)CLS_SOLID
                         : Fd.cls[n];
            if (!FLO || rc[jj] == CLS_FLUID) {
                real r = io.ld(0, n);
#pragma unroll
                for (int a = 1; a < 9; ++a) r += io.ld(a, n);
                rr[jj] = r;
            }
        }
    }
#pragma unroll
    for (int k = 0; k < RPT; ++k) {
        const int ly = ty + k * ROWS;
        const int p = (ly + 2) * LX + tx + 2;
        real r = f[k][0];
#pragma unroll
        for (int a = 1; a < 9; ++a) r += f[k][a];
        S.cls[p] = oc[k];
        S.rho[p] = (oc[k] == CLS_FLUID) ? r : real(0);
    }
#pragma unroll
    for (int jj = 0; jj < JR; ++jj) {
        const int j = tid + jj * NT;
        if (j < RING) {
            int lx, ly;
            ring_pos<TX, TY>(j, lx, ly);
            const int p = ly * LX + lx;
            S.cls[p] = rc[jj];
            S.rho[p] = (rc[jj] == CLS_FLUID) ? rr[jj] : real(0);
        }
    }
    __syncthreads();

    d2q9_psi_phase<real, TX, TY, NT, GFW>(C, Fd, S, we, bad);
}

// Eq. 5 cohesive force and Eq. 8 adhesion at LDS position p; returns the
// total force F (cohesion + adhesion + body force) and the cohesive part.
// FP64 sums the terms in the order of Eq. 5.
template <typename real, int LX>
__device__ __forceinline__ void d2q9_force(const Coef<real>& C, const uint8_t* cls, const real* psi,
                                           int p, real rho, real* Fm, real* F) {
    using L = D2Q9;
    const real psi_c = psi[p];
    real smx = real(0), smy = real(0), sax = real(0), say = real(0);
#pragma unroll
    for (int a = 1; a < 9; ++a) {
        const int q = p + L::ex[a] + L::ey[a] * LX;
        const real w = real(L::w12[a]) * real(1.0 / 12.0);
        // FP32 sums w (psi(x+e) - psi(x)) e, equal since sum w e = 0: the
        // rounding then scales with the psi gradient, not with psi, so the
        // force in a nearly uniform region keeps its digits
        const real wp = (sizeof(real) == 4) ? w * (psi[q] - psi_c) : w * psi[q];
        if (L::ex[a] == 1) smx += wp;
        if (L::ex[a] == -1) smx -= wp;
        if (L::ey[a] == 1) smy += wp;
        if (L::ey[a] == -1) smy -= wp;
        if (C.scheme == WET_SFI && cls[q] != CLS_FLUID) {
            if (L::ex[a] == 1) sax += w;
            if (L::ex[a] == -1) sax -= w;
            if (L::ey[a] == 1) say += w;
            if (L::ey[a] == -1) say -= w;
        }
    }
    Fm[0] = -C.G * psi_c * smx;
    Fm[1] = -C.G * psi_c * smy;
    const real fax = (C.scheme == WET_SFI) ? -C.G_w * rho * sax : real(0);
    const real fay = (C.scheme == WET_SFI) ? -C.G_w * rho * say : real(0);
    F[0] = Fm[0] + fax + C.body[0];
    F[1] = Fm[1] + fay + C.body[1];
}

}  // namespace lbm
