// tile2d_vec.hpp -- the fused D2Q9 tile step with 16-byte population
// accesses (FP32, lattices whose width is a multiple of 4).
//
// Same step, tile, LDS layout and state form as the scalar tile (tile2d.hpp
// and step2d.hip): density (Eq. 4), psi (Eq. 6), wall virtual densities
// (Eqs. 16-17, Eq. 11 or Eq. 8), force (Eq. 5), MRT collision with the
// forcing of Eq. 7 (Eq. 2), push streaming with halfway bounce-back (Eq. 3,
// Fig. 3).  What differs is how populations move:
//
//  * a lane owns a quad, 4 consecutive nodes of a tile row, and loads each
//    direction of it in one 16-byte access; the 2-node density halo is
//    loaded as whole quads too;
//  * each direction is stored as one aligned 16-byte quad: the destination
//    quad [x, x+4) of row y + e_y.  With e_x = 0 it holds the lane's own
//    post-collision values; with e_x = +1 its first element comes from the
//    previous lane (its node x - 1) and with e_x = -1 its last element from
//    the next lane (node x + 4), by a lane shift.  Destination slots on
//    non-fluid nodes receive 0 (they are never read as populations);
//  * the lanes at the ends of a tile row own the part of the quad they can
//    fill (a 12-byte store) plus the one value their shift pushes out of
//    the tile (a 4-byte store); quads that hold a non-fluid source node
//    fall back to one store per element;
//  * a population whose destination is not fluid bounces back into the
//    opposite slot of its own node (one 4-byte store each).
//
// Every output slot still has exactly one writer: the push from its fluid
// source, or the bounce-back of the node itself when the source is not
// fluid, as in the scalar tile.  The requests per node fall by four, which
// is what the scalar tile is limited by.
#pragma once
#include "tile2d.hpp"

namespace lbm {

// LDS column of the first element of ring quad j, and its LDS row: two full
// rows below the tile and two above (QX + 2 quads each, from the quad left
// of the tile to the quad right of it), then the quads left and right of
// each tile row.  Column 2 + 4 q for quad q (-1 <= q <= QX).
template <int QX, int TY>
__device__ __forceinline__ void ring_quad(int j, int& q, int& ly) {
    constexpr int W = QX + 2;
    if (j < 4 * W) {
        const int r = j / W;
        ly = r < 2 ? r : TY + r;
        q = j % W - 1;
    } else {
        const int jj = j - 4 * W;
        ly = 2 + jj / 2;
        q = (jj & 1) ? QX : -1;
    }
}

// lane shift of a wave: value of lane - 1 (up) or lane + 1 (down)
__device__ __forceinline__ float lane_prev(float v) { return __shfl_up(v, 1, 64); }
__device__ __forceinline__ float lane_next(float v) { return __shfl_down(v, 1, 64); }

template <int TX, int TY, int NT, bool GFW>
__device__ __forceinline__ void d2q9_tile_vec(const Coef<float>& C, const Fields<float>& Fd,
                                              const int nx, const int ny, const int x0,
                                              const int y0, const int list_tile) {
    using L = D2Q9;
    constexpr int LX = TX + 4, LY = TY + 4;
    constexpr int QX = TX / 4;       // quads per tile row
    constexpr int ROWS = NT / QX;    // tile rows per pass of the workgroup
    constexpr int RQ = TY / ROWS;    // quads per lane
    static_assert(TX % 4 == 0 && NT % QX == 0 && TY % ROWS == 0, "tile shape");
    static_assert(QX <= 64 && 64 % QX == 0, "a tile row must lie within one wave");
    constexpr int RINGQ = 4 * (QX + 2) + 2 * TY;
    constexpr int JR = (RINGQ + NT - 1) / NT;
    __shared__ TileLDS<float, TX, TY> S;
    const uint32_t N = (uint32_t)nx * (uint32_t)ny;
    const PopIO<float, true> io(Fd.fin, Fd.fout, N, 9);
    const int tid = threadIdx.x, qx = tid % QX, ty = tid / QX;
    bool bad = false;

    const bool inner = x0 >= 4 && y0 >= 2 && x0 + TX + 4 <= nx && y0 + TY + 2 <= ny;
    auto gx_of = [&](int x) { return inner ? x : wrapi(x, nx); };
    auto gy_of = [&](int y) { return inner ? y : wrapi(y, ny); };
    for (int i = tid; i < LX + LY; i += NT) {
        if (i < LX) S.col[i] = (uint32_t)wrapi(x0 - 2 + i, nx);
        else S.row[i - LX] = (uint32_t)wrapi(y0 - 2 + (i - LX), ny) * (uint32_t)nx;
    }
    WallEntry<float> we;
    wall_list_head<float, GFW>(C, Fd, list_tile, tid, S.wl_count, we);

    // one load phase: owned quads (populations kept), ring quads (summed)
    float f[RQ][4][9];
    uint32_t oc[RQ];
#pragma unroll
    for (int k = 0; k < RQ; ++k) {
        const int ly = ty + k * ROWS;
        const uint32_t n = (uint32_t)gy_of(y0 + ly) * (uint32_t)nx + (uint32_t)gx_of(x0 + 4 * qx);
        oc[k] = *reinterpret_cast<const uint32_t*>(Fd.cls + n);
#pragma unroll
        for (int a = 0; a < 9; ++a) ld_quad(io, a, n, f[k][0][a], f[k][1][a], f[k][2][a], f[k][3][a]);
    }
    float rr[JR][4];
    uint32_t rc[JR];
#pragma unroll
    for (int jj = 0; jj < JR; ++jj) {
        const int j = tid + jj * NT;
        rc[jj] = 0x01010101u;  // solid
        rr[jj][0] = rr[jj][1] = rr[jj][2] = rr[jj][3] = 0.0f;
        if (j < RINGQ) {
            int q, ly;
            ring_quad<QX, TY>(j, q, ly);
            const uint32_t n =
                (uint32_t)gy_of(y0 - 2 + ly) * (uint32_t)nx + (uint32_t)gx_of(x0 + 4 * q);
            rc[jj] = *reinterpret_cast<const uint32_t*>(Fd.cls + n);
            float t[9][4];
#pragma unroll
            for (int a = 0; a < 9; ++a) ld_quad(io, a, n, t[a][0], t[a][1], t[a][2], t[a][3]);
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                float r = t[0][e];
#pragma unroll
                for (int a = 1; a < 9; ++a) r += t[a][e];
                rr[jj][e] = r;
            }
        }
    }
#pragma unroll
    for (int k = 0; k < RQ; ++k) {
        const int p0 = (ty + k * ROWS + 2) * LX + 2 + 4 * qx;
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const uint8_t c = (uint8_t)(oc[k] >> (8 * e));
            float r = f[k][e][0];
#pragma unroll
            for (int a = 1; a < 9; ++a) r += f[k][e][a];
            S.cls[p0 + e] = c;
            S.rho[p0 + e] = (c == CLS_FLUID) ? r : 0.0f;
        }
    }
#pragma unroll
    for (int jj = 0; jj < JR; ++jj) {
        const int j = tid + jj * NT;
        if (j < RINGQ) {
            int q, ly;
            ring_quad<QX, TY>(j, q, ly);
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int lx = 2 + 4 * q + e;
                if (lx < 0 || lx >= LX) continue;
                const uint8_t c = (uint8_t)(rc[jj] >> (8 * e));
                S.cls[ly * LX + lx] = c;
                S.rho[ly * LX + lx] = (c == CLS_FLUID) ? rr[jj][e] : 0.0f;
            }
        }
    }
    __syncthreads();
    d2q9_psi_phase<float, TX, TY, NT, GFW>(C, Fd, S, we, bad);

    // rows of every direction start on 128-byte boundaries: the e_x = 0
    // directions then fill whole cache lines of this tile (non-temporal)
    const bool lines = ((reinterpret_cast<uintptr_t>(Fd.fout) | ((uintptr_t)nx * 4u) |
                         ((uintptr_t)x0 * 4u)) & 127) == 0;
#pragma unroll
    for (int k = 0; k < RQ; ++k) {
        const int ly = ty + k * ROWS;
        const int x = x0 + 4 * qx;
        const bool owned = x < nx && y0 + ly < ny;
        const int p0 = (ly + 2) * LX + 2 + 4 * qx;
        bool fl[4];
#pragma unroll
        for (int e = 0; e < 4; ++e) fl[e] = owned && S.cls[p0 + e] == CLS_FLUID;
        // collide the fluid nodes of the quad in place (f becomes f*)
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            if (!fl[e]) continue;
            float Fm[2], F[2], u[2];
            d2q9_force<float, LX>(C, S.cls, S.psi, p0 + e, S.rho[p0 + e], Fm, F);
            collide<L, float>(C, f[k][e], S.rho[p0 + e], F, Fm, S.psi[p0 + e], f[k][e], u);
        }
        // the neighbouring quads of the row are in this tile: lane -+ 1
        const bool has_prev = qx > 0;
        const bool has_next = qx < QX - 1 && x + 4 < nx;
        const uint32_t n_own = S.row[ly + 2] + (uint32_t)x;
#pragma unroll
        for (int a = 0; a < 9; ++a) {
            const int ex = L::ex[a], ey = L::ey[a];
            // shifted-in element (computed by every lane, used by the owner)
            const float in_prev = ex == 1 ? lane_prev(f[k][3][a]) : 0.0f;
            const float in_next = ex == -1 ? lane_next(f[k][0][a]) : 0.0f;
            if (!owned) continue;
            // destination quad [x, x+4) of LDS row ly + 2 + ey: its sources
            float v[4];
            bool mine[4], src[4];
            if (ex == 0) {
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    v[e] = f[k][e][a];
                    src[e] = fl[e];
                    mine[e] = true;
                }
            } else if (ex == 1) {
                v[0] = in_prev;
                src[0] = S.cls[p0 - 1] == CLS_FLUID;
                mine[0] = has_prev;
#pragma unroll
                for (int e = 1; e < 4; ++e) {
                    v[e] = f[k][e - 1][a];
                    src[e] = fl[e - 1];
                    mine[e] = true;
                }
            } else {
#pragma unroll
                for (int e = 0; e < 3; ++e) {
                    v[e] = f[k][e + 1][a];
                    src[e] = fl[e + 1];
                    mine[e] = true;
                }
                v[3] = in_next;
                src[3] = S.cls[p0 + 4] == CLS_FLUID;
                mine[3] = has_next;
            }
            const int pd = p0 + ey * LX;
            bool dst[4];
#pragma unroll
            for (int e = 0; e < 4; ++e) dst[e] = S.cls[pd + e] == CLS_FLUID;
            const uint32_t nd = S.row[ly + 2 + ey] + (uint32_t)x;
            const bool full = mine[0] && mine[1] && mine[2] && mine[3] && src[0] && src[1] &&
                              src[2] && src[3];
            const bool head3 = !mine[0] && mine[1] && mine[2] && mine[3] && src[1] && src[2] &&
                               src[3] && dst[1] && dst[2] && dst[3];
            const bool tail3 = mine[0] && mine[1] && mine[2] && !mine[3] && src[0] && src[1] &&
                               src[2] && dst[0] && dst[1] && dst[2];
            if (full) {
                const float w0 = dst[0] ? v[0] : 0.0f, w1 = dst[1] ? v[1] : 0.0f;
                const float w2 = dst[2] ? v[2] : 0.0f, w3 = dst[3] ? v[3] : 0.0f;
                if (ex == 0 && lines) st_quad<ST_NT>(io, a, nd, w0, w1, w2, w3);
                else st_quad(io, a, nd, w0, w1, w2, w3);
            } else if (head3) {
                st_triple(io, a, nd + 1, v[1], v[2], v[3]);
            } else if (tail3) {
                st_triple(io, a, nd, v[0], v[1], v[2]);
            } else {
#pragma unroll
                for (int e = 0; e < 4; ++e)
                    if (mine[e] && src[e] && dst[e]) io.st(a, nd + e, v[e]);
            }
            // the value this lane's shift pushes out of the tile row
            if (ex == 1 && !has_next && fl[3] && S.cls[pd + 4] == CLS_FLUID)
                io.st(a, S.row[ly + 2 + ey] + S.col[2 + 4 * qx + 4], f[k][3][a]);
            if (ex == -1 && !has_prev && fl[0] && S.cls[pd - 1] == CLS_FLUID)
                io.st(a, S.row[ly + 2 + ey] + S.col[2 + 4 * qx - 1], f[k][0][a]);
            // halfway bounce-back: into the opposite slot of the own node
            if (a > 0) {
#pragma unroll
                for (int e = 0; e < 4; ++e)
                    if (fl[e] && S.cls[p0 + e + ex + ey * LX] != CLS_FLUID)
                        io.st(L::opp[a], n_own + e, f[k][e][a]);
            }
        }
    }
    if (bad) Fd.flag[0] = 1;
}

}  // namespace lbm
