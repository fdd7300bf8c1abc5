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
// tiles run close in time on one XCD); each owned node's populations are
// read once into registers, so the HBM traffic stays close to one read and
// one write of f per fluid node.
//
// State: post-streaming populations, SoA f[a*N + n]; fin -> fout ping-pong.
// Only fluid slots of fout are written; a population that would enter a
// solid node is written back to its origin in the opposite direction.
// Built twice: LBM_PREC == 4 holds the FP32 instantiations (compiled with
// FMA contraction), LBM_PREC == 8 the FP64 ones (no contraction, so that
// FP64 follows the rounding steps of a plain scalar evaluation).  Without
// LBM_PREC both are instantiated.
#ifndef LBM_PREC
#define LBM_PREC 0
#endif
#include <array>
#include <type_traits>
#include <utility>

#include "tile2d.hpp"
#include "tile2d_vec.hpp"

namespace lbm {

// The work of one TX x TY tile at (x0, y0) of an nx x ny lattice; shared by
// the single-lattice kernel and the multi-case kernel.  The lattice's arrays
// keep row y at y * pitch (pitch >= nx; the columns past nx are never read,
// and a step writes 0 into those its tiles cover); the outputs of the field
// mode are dense (row y at y * nx).
// part: index of this tile's diagnostic partial; list_tile: its entry block
// in the wall lists.  MC: the multi-case kernel's two choices, each measured
// faster on the 96 uneven cases (where most tiles wrap) and slower on the
// 2048^2 lattice: tiles whose ring wraps also store the directions with
// ex = 0 non-temporally on line-aligned rows (1.7 % faster there, 0.5 %
// slower here), and populations are loaded for fluid nodes only (2.0 %
// faster there, 1.3 % slower here).
template <typename real, int TX, int TY, int NT, int MODE, bool BUF, bool GFW, bool MC = false>
__device__ __forceinline__ void d2q9_tile(const Coef<real>& C, const Fields<real>& Fd,
                                          const FieldOut<real>& Out, const int nx,
                                          const int pitch, const int ny, const int x0,
                                          const int y0, const int part, const int list_tile) {
    using L = D2Q9;
    constexpr int LX = TX + 4;
    constexpr int ROWS = NT / TX;
    constexpr int RPT = TY / ROWS;
    __shared__ TileLDS<real, TX, TY> S;
    const uint32_t N = (uint32_t)pitch * (uint32_t)ny;  // population plane stride
    const uint32_t Nd = (uint32_t)nx * (uint32_t)ny;    // plane stride of the dense outputs
    const PopIO<real, BUF> io(Fd.fin, Fd.fout, N, 9);
    const int tid = threadIdx.x, tx = tid % TX, ty = tid / TX;
    bool bad = false;
    real f[RPT][9];
    d2q9_prologue<real, TX, TY, NT, BUF, GFW, MC>(C, Fd, io, nx, pitch, ny, x0, y0, list_tile, S,
                                                  f, bad);

    double d_sum = 0.0;
    real d_umax = real(0), d_rmin = real(1e30), d_rmax = real(-1e30);
    int d_cnt = 0;
    // the tile and its 1-node ring lie inside the lattice without wrapping
    const bool interior = x0 >= 1 && y0 >= 1 && x0 + TX + 1 <= nx && y0 + TY + 1 <= ny;
    // rows of every direction start on 128-byte boundaries
    const bool lines = ((reinterpret_cast<uintptr_t>(Fd.fout) | ((uintptr_t)pitch * sizeof(real)) |
                         ((uintptr_t)x0 * sizeof(real))) & 127) == 0;

#pragma unroll
    for (int k = 0; k < RPT; ++k) {
        const int ly = ty + k * ROWS;
        const int gx = x0 + tx, gy = y0 + ly;
        if (gx >= nx || gy >= ny) {  // ragged tile: not owned
            // a position of the row's padding (pitch > nx) is never read; it
            // gets 0 so that the row's last cache line is written whole
            if (MODE == MODE_STEP && gx < pitch && gy < ny) {
                const uint32_t m = (uint32_t)gy * (uint32_t)pitch + (uint32_t)gx;
#pragma unroll
                for (int a = 0; a < 9; ++a) io.st(a, m, real(0));
            }
            continue;
        }
        const int p = (ly + 2) * LX + tx + 2;
        const uint32_t n = S.row[ly + 2] + S.col[tx + 2];
        const uint32_t od = (uint32_t)gy * (uint32_t)nx + (uint32_t)gx;  // dense output index
        const uint8_t c = S.cls[p];
        if (c != CLS_FLUID) {
            if (MODE == MODE_FIELDS) {
                if (Out.rho) Out.rho[od] = (c == CLS_WALL) ? S.rho[p] : real(0);
                if (Out.u) {
                    Out.u[od] = real(0);
                    Out.u[(size_t)Nd + od] = real(0);
                }
            }
            continue;
        }
        const real rho = S.rho[p];
        const real psi_c = S.psi[p];
        real Fm[2], F[2];
        d2q9_force<real, LX>(C, S.cls, S.psi, p, rho, Fm, F);

        if (MODE == MODE_FIELDS) {
            const real jx = f[k][1] - f[k][3] + f[k][5] - f[k][6] - f[k][7] + f[k][8];
            const real jy = f[k][2] - f[k][4] + f[k][5] + f[k][6] - f[k][7] - f[k][8];
            const real ux = (jx + real(0.5) * F[0]) / rho;
            const real uy = (jy + real(0.5) * F[1]) / rho;
            if (Out.rho) Out.rho[od] = rho;
            if (Out.u) {
                Out.u[od] = ux;
                Out.u[(size_t)Nd + od] = uy;
            }
            const real um = sqrt(ux * ux + uy * uy);
            // mass: the node's populations summed in FP64 (in FP32 the
            // density's own rounding repeats at every node of a uniform
            // region and would bias the total)
            double rs = (double)f[k][0];
#pragma unroll
            for (int a = 1; a < 9; ++a) rs += (double)f[k][a];
            d_sum += rs;
            d_umax = um > d_umax ? um : d_umax;
            d_rmin = rho < d_rmin ? rho : d_rmin;
            d_rmax = rho > d_rmax ? rho : d_rmax;
            d_cnt += 1;
            continue;
        }

        real fs[9], u[2];
        collide<L, real>(C, f[k], rho, F, Fm, psi_c, fs, u);
        // push streaming with halfway bounce-back
        if (interior) {
            // no neighbour wraps: the target is n + ex + ey pitch
            // With rows on 128-byte boundaries, the directions with ex = 0
            // fill whole cache lines of this tile (the rest population never
            // leaves its node; the y neighbours of a row segment lie in one
            // line segment), so those stores take the non-temporal policy.
            // Shifts in x split lines with the neighbouring tile: normal.
            auto push = [&](auto whole) {
                constexpr bool NT_OK = decltype(whole)::value;
#pragma unroll
                for (int a = 0; a < 9; ++a) {
                    const int q = p + L::ex[a] + L::ey[a] * LX;
                    if (NT_OK && L::ex[a] == 0)
                        io.template st_push<ST_NT>(S.cls[q] == CLS_FLUID, a, L::opp[a],
                                                   L::ey[a] * pitch, n, fs[a]);
                    else
                        io.st_push(S.cls[q] == CLS_FLUID, a, L::opp[a], L::ex[a] + L::ey[a] * pitch,
                                   n, fs[a]);
                }
            };
            if (lines) push(std::true_type{});
            else push(std::false_type{});
        } else {
            // a tile whose ring wraps: the neighbours' rows and columns come
            // from the tile's tables, and each direction is one store (to the
            // neighbour, or back to this node's opposite slot).  A wrap only
            // changes which row the directions with ex = 0 land in, so on
            // line-aligned rows they still fill whole lines of this tile.
            const uint32_t col[3] = {S.col[tx + 1], S.col[tx + 2], S.col[tx + 3]};
            const uint32_t row[3] = {S.row[ly + 1], S.row[ly + 2], S.row[ly + 3]};
            auto push = [&](auto whole) {
                constexpr bool NT_OK = decltype(whole)::value;
#pragma unroll
                for (int a = 0; a < 9; ++a) {
                    const int q = p + L::ex[a] + L::ey[a] * LX;
                    const uint32_t m = row[1 + L::ey[a]] + col[1 + L::ex[a]];
                    if (NT_OK && L::ex[a] == 0)
                        io.template st_sel<ST_NT>(S.cls[q] == CLS_FLUID, a, L::opp[a], m, n,
                                                  fs[a]);
                    else
                        io.st_sel(S.cls[q] == CLS_FLUID, a, L::opp[a], m, n, fs[a]);
                }
            };
            if (MC && lines) push(std::true_type{});
            else push(std::false_type{});
        }
    }

    if (MODE == MODE_FIELDS && Out.part) {
        block_reduce_diag<NT>(d_sum, d_umax, d_rmin, d_rmax, d_cnt, Out.part + 5 * part);
    }
    if (bad) Fd.flag[0] = 1;
}

// Workgroup -> tile order.  XCD: consecutive tiles go to one XCD (each XCD
// gets a contiguous range of the order, so neighbouring tiles share an L2).
// ORD > 0: the order runs through column groups ORD tiles wide, row by row
// inside a group, so the tile above a tile is only ORD places earlier.
template <typename real, int TX, int TY, int NT, int MODE, bool XCD, bool BUF, int ORD, int OCC,
          bool GFW>
__global__ __launch_bounds__(NT, OCC) void k_step_d2q9(Coef<real> C, Fields<real> Fd,
                                                       FieldOut<real> Out) {
    const int gxb = gridDim.x, gyb = gridDim.y, nblk = gxb * gyb;
    int bid = blockIdx.x + gxb * blockIdx.y;
    if (XCD) bid = remap_xcd(bid, nblk);
    int bx, by;
    if (ORD > 0) {
        const int g = bid / (ORD * gyb), r = bid - g * (ORD * gyb);
        const int w = (gxb - g * ORD) < ORD ? (gxb - g * ORD) : ORD;
        bx = g * ORD + r % w;
        by = r / w;
    } else {
        bx = bid % gxb;
        by = bid / gxb;
    }
    d2q9_tile<real, TX, TY, NT, MODE, BUF, GFW>(C, Fd, Out, C.nx, C.pitch > 0 ? C.pitch : C.nx,
                                                C.ny, bx * TX, by * TY, bid,
                                                by * gxb + bx);
}

// The same step with 16-byte population accesses (tile2d_vec.hpp): FP32,
// lattices whose width is a multiple of 4, arrays below 4 GiB.
template <int TX, int TY, int NT, bool XCD, int OCC, bool GFW>
__global__ __launch_bounds__(NT, OCC) void k_step_d2q9_vec(Coef<float> C, Fields<float> Fd) {
    const int gxb = gridDim.x, gyb = gridDim.y, nblk = gxb * gyb;
    int bid = blockIdx.x + gxb * blockIdx.y;
    if (XCD) bid = remap_xcd(bid, nblk);
    const int bx = bid % gxb, by = bid / gxb;
    d2q9_tile_vec<TX, TY, NT, GFW>(C, Fd, C.nx, C.ny, bx * TX, by * TY, by * gxb + bx);
}

// Many independent lattices in one launch: workgroup -> (case, tile) through
// a table; each case has its own size, node classes, wall list and wetting
// parameters inside packed arenas.  The physical parameters are shared.
template <typename real, int TX, int TY, int NT, bool BUF>
__global__ __launch_bounds__(NT) void k_step_d2q9_batch(Coef<real> C, BatchArgs<real> B) {
    const int bid = remap_xcd(blockIdx.x, gridDim.x);
    const TileRef t = B.tiles[bid];
    const CaseDesc cd = B.cases[t.c];
    Fields<real> Fd;
    Fd.fin = B.fin + cd.f_off;
    Fd.fout = B.fout + cd.f_off;
    Fd.cls = B.cls + cd.node_off;
    Fd.widx = B.widx + cd.node_off;
    Fd.phi = B.phi + cd.wall_off;
    Fd.drho = B.drho + cd.wall_off;
    Fd.flag = B.flag;
    Fd.tw_pack = B.tw_pack;
    Fd.tw_phi = B.tw_phi;
    Fd.tw_drho = B.tw_drho;
    Fd.tw_stride = B.tw_stride;
    Fd.tw_code = B.tw_code;
    FieldOut<real> none{nullptr, nullptr, nullptr};
    d2q9_tile<real, TX, TY, NT, MODE_STEP, BUF, false, true>(C, Fd, none, cd.nx, cd.pitch, cd.ny,
                                                          t.x0, t.y0, bid, bid);
}

// ----------------------------------------------------------------- launch
// Tile variants the autotuner chooses among (variant 0 is the default and
// the shape used by the field/diagnostic mode).
struct Shape2D {
    int TX, TY, NT;
    bool xcd;
    int ord;  // column-group width of the tile order (0: row-major)
    int occ;  // minimum waves per SIMD asked of the register allocator
    bool vec = false;  // 16-byte accesses (FP32 step, width a multiple of 4)
};

template <typename real>
struct Variants2D;
template <>
struct Variants2D<float> {
    static constexpr int count = 16;
    static constexpr int preferred = 10;  // 128 x 16 tiles, 512 threads
    static constexpr Shape2D shape[count] = {
        {64, 16, 256, true, 0, 1},  {64, 16, 256, false, 0, 1}, {128, 8, 256, true, 0, 1},
        {64, 32, 256, true, 0, 1},  {256, 4, 256, true, 0, 1},  {128, 16, 256, true, 0, 1},
        {64, 16, 256, true, 8, 1},  {128, 8, 256, true, 4, 1},  {64, 16, 256, true, 0, 8},
        {256, 8, 512, true, 0, 1},  {128, 16, 512, true, 0, 1}, {64, 32, 256, true, 8, 1},
        {128, 16, 512, true, 0, 1, true}, {64, 16, 256, true, 0, 1, true},
        {256, 8, 512, true, 0, 1, true},  {128, 32, 512, true, 0, 1, true}};
};
template <>
struct Variants2D<double> {
    static constexpr int count = 4;
    static constexpr int preferred = 0;
    static constexpr Shape2D shape[count] = {{64, 8, 256, true, 0, 1},
                                             {64, 8, 256, false, 0, 1},
                                             {128, 4, 256, true, 0, 1},
                                             {64, 8, 256, true, 8, 1}};
};

// variants beyond the tile shapes are the y-sweep kernel (step_march.hip)
template <typename real>
int step2d_variants() {
    return Variants2D<real>::count + step2d_march_variants<real>();
}

template <typename real>
int grid2d_blocks(int nx, int ny, int variant) {
    const Shape2D s = Variants2D<real>::shape[variant < Variants2D<real>::count ? variant : 0];
    return ((nx + s.TX - 1) / s.TX) * ((ny + s.TY - 1) / s.TY);
}

template <typename real, int V, int MODE, bool BUF = true, bool GFW = false>
static void launch_v(const Coef<real>& C, const Fields<real>& F, const FieldOut<real>& O,
                     hipStream_t s) {
    constexpr Shape2D sh = Variants2D<real>::shape[V];
    dim3 grid((C.nx + sh.TX - 1) / sh.TX, (C.ny + sh.TY - 1) / sh.TY);
    if constexpr (sh.vec && std::is_same<real, float>::value && MODE == MODE_STEP && BUF) {
        if (C.nx % 4 == 0 && (C.pitch == 0 || C.pitch == C.nx)) {
            hipLaunchKernelGGL((k_step_d2q9_vec<sh.TX, sh.TY, sh.NT, sh.xcd, sh.occ, GFW>), grid,
                               dim3(sh.NT), 0, s, C, F);
            return;
        }
    }
    // otherwise the scalar tile of the same shape (the wall lists match)
    hipLaunchKernelGGL(
        (k_step_d2q9<real, sh.TX, sh.TY, sh.NT, MODE, sh.xcd, BUF, sh.ord, sh.occ, GFW>), grid,
        dim3(sh.NT), 0, s, C, F, O);
}

template <typename real, int MODE, bool BUF, bool GFW, size_t... I>
static auto table_v(std::index_sequence<I...>) {
    using Fn = void (*)(const Coef<real>&, const Fields<real>&, const FieldOut<real>&,
                        hipStream_t);
    return std::array<Fn, sizeof...(I)>{&launch_v<real, (int)I, MODE, BUF, GFW>...};
}

// population arrays of 4 GiB or more cannot use 32-bit buffer offsets
template <typename real>
static bool fits_buffer(const Coef<real>& C, int Q) {
    return (uint64_t)Q * (uint64_t)C.nx * C.ny * C.nz * sizeof(real) <= 0xFFFFFFFFull;
}

template <typename real>
hipError_t launch_step2d(const Coef<real>& C, const Fields<real>& F, const FieldOut<real>& O,
                         int mode, int variant, hipStream_t s) {
    const bool gf = C.scheme == WET_GF;
    if (mode == MODE_FIELDS) variant = 0;
    if (!fits_buffer(C, 9)) {
        // one tile shape serves arrays past 4 GiB; the wall lists were built
        // for the context's shape, so the walls are looked up per node here
        Fields<real> G = F;
        G.tw_pack = nullptr;
        G.tw_code = nullptr;
        if (mode == MODE_STEP && gf) launch_v<real, 0, MODE_STEP, false, true>(C, G, O, s);
        else if (mode == MODE_STEP) launch_v<real, 0, MODE_STEP, false>(C, G, O, s);
        else if (gf) launch_v<real, 0, MODE_FIELDS, false, true>(C, G, O, s);
        else launch_v<real, 0, MODE_FIELDS, false>(C, G, O, s);
        return hipGetLastError();
    }
    // the sweep kernels have no geometric formulation: its steps run tiled
    if (variant >= Variants2D<real>::count && gf) variant = Variants2D<real>::preferred;
    if (variant >= Variants2D<real>::count)
        return launch_step2d_march<real>(C, F, O, variant - Variants2D<real>::count, s);
    if (variant < 0) return hipErrorInvalidValue;
    constexpr auto seq = std::make_index_sequence<Variants2D<real>::count>{};
    static const auto step = table_v<real, MODE_STEP, true, false>(seq);
    static const auto step_gf = table_v<real, MODE_STEP, true, true>(seq);
    if (mode == MODE_STEP) (gf ? step_gf : step)[variant](C, F, O, s);
    else if (gf) launch_v<real, 0, MODE_FIELDS, true, true>(C, F, O, s);
    else launch_v<real, 0, MODE_FIELDS, true>(C, F, O, s);
    return hipGetLastError();
}

template <typename real>
int tile2d_variants() {
    return Variants2D<real>::count;
}

// the variant a single-lattice context starts with (fastest on the 2048^2
// porous benchmark lattice); the autotuner may pick another
template <typename real>
int tile2d_preferred_variant() {
    return Variants2D<real>::preferred;
}

template <typename real>
void tile2d_shape(int variant, int* TX, int* TY) {
    const Shape2D sh = Variants2D<real>::shape[variant];
    *TX = sh.TX;
    *TY = sh.TY;
}

template <typename real, int V>
static void launch_b(const Coef<real>& C, const BatchArgs<real>& B, int ntiles, hipStream_t s) {
    constexpr Shape2D sh = Variants2D<real>::shape[V];
    hipLaunchKernelGGL((k_step_d2q9_batch<real, sh.TX, sh.TY, sh.NT, true>), dim3(ntiles),
                       dim3(sh.NT), 0, s, C, B);
}

template <typename real, size_t... I>
static auto table_b(std::index_sequence<I...>) {
    using Fn = void (*)(const Coef<real>&, const BatchArgs<real>&, int, hipStream_t);
    return std::array<Fn, sizeof...(I)>{&launch_b<real, (int)I>...};
}

template <typename real>
hipError_t launch_step2d_batch(const Coef<real>& C, const BatchArgs<real>& B, int ntiles,
                               int variant, hipStream_t s) {
    if (ntiles <= 0) return hipSuccess;
    if (variant < 0 || variant >= Variants2D<real>::count) return hipErrorInvalidValue;
    static const auto tab = table_b<real>(std::make_index_sequence<Variants2D<real>::count>{});
    tab[variant](C, B, ntiles, s);
    return hipGetLastError();
}

#if LBM_PREC != 8
template int tile2d_variants<float>();
template int tile2d_preferred_variant<float>();
#endif
#if LBM_PREC != 4
template int tile2d_variants<double>();
template int tile2d_preferred_variant<double>();
#endif
#if LBM_PREC != 8
template void tile2d_shape<float>(int, int*, int*);
#endif
#if LBM_PREC != 4
template void tile2d_shape<double>(int, int*, int*);
#endif
#if LBM_PREC != 8
template hipError_t launch_step2d_batch<float>(const Coef<float>&, const BatchArgs<float>&, int,
                                               int, hipStream_t);
#endif
#if LBM_PREC != 4
template hipError_t launch_step2d_batch<double>(const Coef<double>&, const BatchArgs<double>&,
                                                int, int, hipStream_t);
#endif
#if LBM_PREC != 8
template int step2d_variants<float>();
#endif
#if LBM_PREC != 4
template int step2d_variants<double>();
#endif
#if LBM_PREC != 8
template int grid2d_blocks<float>(int, int, int);
#endif
#if LBM_PREC != 4
template int grid2d_blocks<double>(int, int, int);
#endif
#if LBM_PREC != 8
template hipError_t launch_step2d<float>(const Coef<float>&, const Fields<float>&,
                                         const FieldOut<float>&, int, int, hipStream_t);
#endif
#if LBM_PREC != 4
template hipError_t launch_step2d<double>(const Coef<double>&, const Fields<double>&,
                                          const FieldOut<double>&, int, int, hipStream_t);
#endif

}  // namespace lbm
