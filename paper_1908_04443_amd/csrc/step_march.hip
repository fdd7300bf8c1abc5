// step_march.hip -- fused time step that sweeps a tile along the last axis
// (z for D3Q19, y for D2Q9).
//
// Same arithmetic as the tiled 2-D step (Sec. II A, Sec. III B: density,
// psi, wall virtual density, force, velocity, MRT collision with the Eq. 7
// forcing, streaming with halfway bounce-back; push for D2Q9, gather from a
// pull-form state for D3Q19, below).  A workgroup owns a
// TX x TY column of the cross-section (TY = 1 in 2-D) and a chunk of TZ
// slices along the sweep axis.  It walks the chunk plus two halo slices on
// each side; for each slice it
//   A  loads node classes and densities of the cross-section tile plus a
//      2-node halo into slot (it mod 5) of an LDS ring,
//   B  finishes the wall virtual densities and psi of the previous slice on
//      the tile plus a 1-node halo (ring of 4 psi slots),
//   C  collides and streams the slice two behind the load front, reading
//      its populations here rather than holding them in registers since
//      phase A, which keeps the register count low enough for several
//      waves per SIMD.
// The densities of phase A come from a separate density pass (k_density,
// launched just before): the halo then costs one value per node instead
// of Q populations, and each node's populations are read once, in phase C.
// (The FUSED variant below sums the densities in phase A instead.)
// With 19 populations and a 2-node halo around a 32 x 8 cross-section this
// removes most of the bytes of a 3-D step that sums the halo's
// populations inside the sweep.
// Built twice: LBM_PREC == 4 holds the FP32 instantiations (compiled with
// FMA contraction), LBM_PREC == 8 the FP64 ones (no contraction, so that
// FP64 follows the rounding steps of a plain scalar evaluation).  Without
// LBM_PREC both are instantiated.
#ifndef LBM_PREC
#define LBM_PREC 0
#endif
#include <array>
#include <utility>

#include "lbm_device.hpp"
#include "lbm_kernels.hpp"

namespace lbm {

// D3Q19 populations are kept in pull form: the step stores each node's
// post-collision populations in the node's own slots (whole cache lines per
// workgroup) and the next step gathers f_a(x) from slot a of x - e_a
// (Eq. 3).  Halfway bounce-back (Fig. 3) is folded into the store: a fluid
// node whose neighbour x + e_a is not fluid also writes its f*_a into slot
// opp(a) of that neighbour, which is exactly where the gather of direction
// opp(a) at x looks.  No non-fluid node gathers, so those slots are free.
// D2Q9 keeps the push form (the post-stream populations).

// node index of x - e_a for a node (x, y, z) inside the lattice, periodic
template <typename L>
__device__ __forceinline__ uint32_t up_node(int a, int x, int y, int z, int na, int nb, int nc,
                                            uint32_t nab) {
    int sx = x - L::ex[a], sy = y - L::ey[a], sz = z - L::ez[a];
    sx = sx < 0 ? sx + na : (sx >= na ? sx - na : sx);
    sy = sy < 0 ? sy + nb : (sy >= nb ? sy - nb : sy);
    sz = sz < 0 ? sz + nc : (sz >= nc ? sz - nc : sz);
    return (uint32_t)sz * nab + (uint32_t)sy * (uint32_t)na + (uint32_t)sx;
}

// Density of every node (Eq. 4), summed in velocity order; 0 off the fluid.
// D2Q9: from the post-stream populations of the node (a 1-D grid over the
// nodes).  D3Q19: gathered from the pull form; blockIdx.y and blockIdx.z
// give the row and the slice, so the gather needs no index division.
template <typename L, typename real>
__global__ __launch_bounds__(256) void k_density(const uint8_t* __restrict__ cls,
                                                 const real* __restrict__ f, real* __restrict__ rho,
                                                 int na, int nb, int nc) {
    constexpr int Q = L::Q;
    const uint32_t nab = (uint32_t)na * (uint32_t)nb, N = nab * (uint32_t)nc;
    if constexpr (L::D == 3) {
        const int x = blockIdx.x * 256 + threadIdx.x, y = blockIdx.y, z = blockIdx.z;
        if (x >= na) return;
        const uint32_t n = (uint32_t)z * nab + (uint32_t)y * (uint32_t)na + (uint32_t)x;
        real r = real(0);
        if (cls[n] == CLS_FLUID) {
            r = f[n];
#pragma unroll
            for (int a = 1; a < Q; ++a) r += f[(size_t)a * N + up_node<L>(a, x, y, z, na, nb, nc, nab)];
        }
        __builtin_nontemporal_store(r, &rho[n]);  // whole lines per row: 0.3 % faster step
    } else {
        const uint32_t n = blockIdx.x * 256u + threadIdx.x;
        if (n >= N) return;
        real r = real(0);
        if (cls[n] == CLS_FLUID) {
            r = f[n];
#pragma unroll
            for (int a = 1; a < Q; ++a) r += f[(size_t)a * N + n];
        }
        rho[n] = r;
    }
}

template <typename L, typename real>
static void launch_density(const Coef<real>& C, const Fields<real>& F, hipStream_t s) {
    const uint32_t N = (uint32_t)C.nx * (uint32_t)C.ny * (uint32_t)C.nz;
    // the 3-D grid fits: D3Q19 parameters are validated to ny, nz <= 65535
    const dim3 grid = (L::D == 3) ? dim3((C.nx + 255) / 256, C.ny, C.nz) : dim3((N + 255) / 256);
    hipLaunchKernelGGL((k_density<L, real>), grid, dim3(256), 0, s, F.cls, F.fin, F.rho, C.nx,
                       C.ny, C.nz);
}

// Where a block keeps what its sources send to the nodes around it (its
// part of Fd.ring, PsumFaces<TX, TY, TZ>::size values per block, block b at
// b * size), by the node's position (i, j, k) relative to the block's
// origin: the two faces below and above the block (k = -1, TZ) as
// (TY + 2) x (TX + 2) planes, then the rows j = -1 and j = TY of the slices
// 0 .. TZ - 1 (TX + 2 positions each), then the columns i = -1 and i = TX
// of those slices (TY positions each).  Each kind is contiguous, so a pass
// over one face reads neighbouring values.
template <int TX, int TY, int TZ>
struct PsumFaces {
    static constexpr int ZF = (TY + 2) * (TX + 2), YF = TZ * (TX + 2), XF = TZ * TY;
    static constexpr int size = 2 * ZF + 2 * YF + 2 * XF;
    __device__ __forceinline__ static int index(int i, int j, int k) {
        if (k < 0 || k >= TZ) return (k < 0 ? 0 : ZF) + (j + 1) * (TX + 2) + i + 1;
        if (j < 0 || j >= TY) return 2 * ZF + (j < 0 ? 0 : YF) + k * (TX + 2) + i + 1;
        return 2 * ZF + 2 * YF + (i < 0 ? 0 : XF) + k * TY + j;
    }
};

// Completes the densities a PSUM sweep formed: a fluid node on a face of
// its block adds the partial sums that the neighbouring blocks' sources
// sent to it.  The blocks that can send to it are those across the faces it
// lies on (f = -1 / +1 along an axis where it sits on the low / high face)
// and across the edges between two of those faces; D3Q19 has no velocity
// along a body diagonal, so the block across a corner sends nothing.  The
// six candidates are read unconditionally (a candidate that does not apply
// reads the first value of the face array and adds 0), so the loads of a wave are in
// flight together.  The offset of the neighbour (not its absolute position)
// locates the node in the neighbour's part, so a block that is its own
// periodic neighbour is handled too.
template <typename real, int TX, int TY, int TZ, int NPT>
__global__ __launch_bounds__(256) void k_psum_close(const uint8_t* __restrict__ cls,
                                                    real* __restrict__ rho,
                                                    const real* __restrict__ ring, int na, int nb,
                                                    int nc) {
    static_assert(TX > 2 && TY > 2 && TZ > 2, "a block has interior nodes along every axis");
    using PF = PsumFaces<TX, TY, TZ>;
    // NPT face nodes per thread, gridDim.x * 256 apart, all loads issued
    // before any sum.  Per block of the sweep: the two z faces (TX x TY),
    // the two y faces without their z edges (TX x (TZ - 2)), then the two x
    // faces without either ((TY - 2) x (TZ - 2)).
    constexpr int ZF = TX * TY, YF = TX * (TZ - 2), XF = (TY - 2) * (TZ - 2);
    constexpr uint32_t FPB = 2 * ZF + 2 * YF + 2 * XF;
    const int gx = na / TX, gy = nb / TY, gz = nc / TZ;
    const uint32_t total = (uint32_t)gx * (uint32_t)gy * (uint32_t)gz * FPB;
    auto wrap1 = [](int v, int m) { return v < 0 ? v + m : (v >= m ? v - m : v); };
    real v[NPT][6], r[NPT];
    uint8_t cl[NPT];
    uint32_t nn[NPT];
    bool ok[NPT];
#pragma unroll
    for (int p = 0; p < NPT; ++p) {
        const uint32_t t0 = (blockIdx.x + (uint32_t)p * gridDim.x) * 256u + threadIdx.x;
        ok[p] = t0 < total;
        const uint32_t t = ok[p] ? t0 : 0u;  // a thread past the end reads node 0 and stores nothing
        const uint32_t b = t / FPB;
        int q = (int)(t - b * FPB), i, j, k;
        if (q < 2 * ZF) {
            k = q < ZF ? 0 : TZ - 1;
            q = q < ZF ? q : q - ZF;
            i = q % TX;
            j = q / TX;
        } else if ((q -= 2 * ZF) < 2 * YF) {
            j = q < YF ? 0 : TY - 1;
            q = q < YF ? q : q - YF;
            i = q % TX;
            k = 1 + q / TX;
        } else {
            q -= 2 * YF;
            i = q < XF ? 0 : TX - 1;
            q = q < XF ? q : q - XF;
            j = 1 + q % (TY - 2);
            k = 1 + q / (TY - 2);
        }
        const int bx = (int)(b % (uint32_t)gx), by = (int)((b / (uint32_t)gx) % (uint32_t)gy);
        const int bz = (int)(b / ((uint32_t)gx * (uint32_t)gy));
        const int fx = i == 0 ? -1 : (i == TX - 1 ? 1 : 0);
        const int fy = j == 0 ? -1 : (j == TY - 1 ? 1 : 0);
        const int fz = k == 0 ? -1 : (k == TZ - 1 ? 1 : 0);
        nn[p] = ((uint32_t)(bz * TZ + k) * (uint32_t)nb + (uint32_t)(by * TY + j)) * (uint32_t)na +
                (uint32_t)(bx * TX + i);
        const int ox[6] = {fx, 0, 0, fx, fx, 0};
        const int oy[6] = {0, fy, 0, fy, 0, fy};
        const int oz[6] = {0, 0, fz, 0, fz, fz};
#pragma unroll
        for (int c = 0; c < 6; ++c) {
            const bool use = (c < 3) ? ((ox[c] | oy[c] | oz[c]) != 0)
                                     : (c == 3 ? (fx != 0 && fy != 0)
                                               : (c == 4 ? (fx != 0 && fz != 0) : (fy != 0 && fz != 0)));
            const int nbx = wrap1(bx + ox[c], gx), nby = wrap1(by + oy[c], gy),
                      nbz = wrap1(bz + oz[c], gz);
            const size_t at = (size_t)(nbx + gx * (nby + gy * nbz)) * PF::size +
                              PF::index(i - ox[c] * TX, j - oy[c] * TY, k - oz[c] * TZ);
            v[p][c] = ring[use ? at : (size_t)0];
            v[p][c] = use ? v[p][c] : real(0);
        }
        cl[p] = cls[nn[p]];
        r[p] = rho[nn[p]];
    }
#pragma unroll
    for (int p = 0; p < NPT; ++p) {
        real s = r[p];
#pragma unroll
        for (int c = 0; c < 6; ++c) s += v[p][c];
        if (ok[p] && cl[p] == CLS_FLUID) rho[nn[p]] = s;
    }
}

// FUSED: no density pass.  Phase A loads the populations of its slice,
// sums the density of every node of the slice (owned and halo) itself and
// keeps the owned node's populations in registers until phase C collides
// them two iterations later (a ring of three register sets, so the loop
// body is instantiated three times with the sets rotated).
// OCC: minimum waves per SIMD asked of the register allocator.
// PSUM (D3Q19, step mode): the sweep also forms the density of the next
// step.  After a slice collides, its post-collision populations are staged
// in LDS and every owned position, and every position of the 1-node ring
// around the cross-section, adds the ones that stream to it (from the
// slices below, at and above); the owned node's own bounce-backs add to
// its own density.  A node whose sources all lie in the block gets its
// whole density; the others get a partial sum, and the block writes what
// its sources send to the nodes around it into its part of Fd.ring (laid
// out as PsumFaces describes).  k_psum_close then adds those to the nodes
// on block faces.  Needs no ragged block.
template <typename L, typename real, int TX, int TY, int TZ, int MODE, bool XCD, bool BUF,
          bool FUSED = false, int OCC = 1, bool PSUM = false>
__global__ __launch_bounds__(TX* TY, OCC) void k_step_march(Coef<real> C, Fields<real> Fd,
                                                            FieldOut<real> Out) {
    constexpr bool D3 = (L::D == 3);
    constexpr bool PULL = D3;                // populations in pull form (D3Q19)
    constexpr int Q = L::Q;
    constexpr int NT = TX * TY;
    constexpr int HB = D3 ? 2 : 0;           // halo along the second tile axis
    constexpr int PA = TX + 4, PB = TY + 2 * HB, PS = PA * PB;
    constexpr int RING = PS - TX * TY;
    constexpr int JR = (RING + NT - 1) / NT;  // halo positions per thread
    static_assert(!FUSED || JR == 1, "the fused sweep keeps one halo position per thread");
    constexpr int NSLOT = 5, NPSI = 4;

    __shared__ uint8_t s_cls[NSLOT][PS];
    __shared__ real s_rho[NSLOT][PS];
    __shared__ real s_psi[NPSI][PS];
    static_assert(!PSUM || (D3 && !FUSED && MODE == MODE_STEP), "PSUM: D3Q19 step sweep");
    constexpr int NRING = 2 * (TX + 2) + 2 * TY;  // the 1-node ring around the cross-section
    static_assert(!PSUM || NRING <= NT, "one ring position per thread");
    using PF = PsumFaces<TX, TY, TZ>;
    // staged post-collision populations of the slice on the cross-section
    // with a zero border one node wide, slot after slot, and SPAD zeros
    // before the first slot and after the last.  A source two nodes outside
    // the cross-section (a ring position's) then falls on the border of the
    // row beside it or on the padding: every read is in the array and reads
    // 0 for a source outside the block.  Only the 16 velocities that move in
    // the cross-section are staged (slot SLOT[a]); the rest velocity and +-z
    // stay in their column and go straight into the owned node's sums.
    constexpr int SW = TX + 2, SS = (TX + 2) * (TY + 2), QS = 16, SPAD = SW + 1;
    constexpr int SLOT[19] = {-1, 0, 1, 2, 3, -1, -1, 4, 5, 6, 7, 8, 9, 10, 11, 12, 13, 14, 15};
    static_assert(!PSUM || (L::ex[5] == 0 && L::ey[5] == 0 && L::ez[5] == 1 && L::ex[6] == 0 &&
                            L::ey[6] == 0 && L::ez[6] == -1),
                  "velocities 5 and 6 are +z and -z");
    __shared__ real s_fs[PSUM ? QS * SS + 2 * SPAD : 1];

    const int na = C.nx;
    const int nb = D3 ? C.ny : 1;
    const int nc = D3 ? C.nz : C.ny;
    const uint32_t nab = (uint32_t)na * (uint32_t)nb;
    const uint32_t N = nab * (uint32_t)nc;
    const PopIO<real, BUF> io(Fd.fin, Fd.fout, N, Q);
    const int tid = threadIdx.x;
    const int nblk = gridDim.x * gridDim.y * gridDim.z;
    int bid = blockIdx.x + gridDim.x * (blockIdx.y + gridDim.y * blockIdx.z);
    if (XCD) bid = remap_xcd(bid, nblk);
    const int bx = bid % gridDim.x, by = (bid / gridDim.x) % gridDim.y;
    const int bz = bid / (gridDim.x * gridDim.y);
    const int a0 = bx * TX, b0 = by * TY, c0 = bz * TZ;

    // owned position of this thread
    const int own_la = 2 + tid % TX, own_lb = HB + tid / TX;
    const int own_a = a0 + own_la - 2, own_b = b0 + own_lb - HB;
    const bool own_in = own_a < na && own_b < nb;  // ragged tiles
    const uint32_t own_ab = (uint32_t)wrapi(own_b, nb) * na + wrapi(own_a, na);
    const int own_p = own_lb * PA + own_la;
    // halo positions j = tid, tid + NT, ... (j < RING) of the plane outside
    // the owned TX x TY block: in 3-D two full rows below and above, then two
    // columns on each side; in 2-D two nodes on each side
    const int own_aw = wrapi(own_a, na), own_bw = D3 ? wrapi(own_b, nb) : 0;
    int ring_p[JR], ring_x[JR], ring_y[JR];
    uint32_t ring_ab[JR];
#pragma unroll
    for (int jj = 0; jj < JR; ++jj) {
        const int j = tid + jj * NT;
        int la = 0, lb = 0;
        if (D3) {
            if (j < 2 * PA) {
                lb = j / PA;
                la = j % PA;
            } else if (j < 4 * PA) {
                lb = TY + 2 + (j - 2 * PA) / PA;
                la = (j - 2 * PA) % PA;
            } else {
                const int k = j - 4 * PA;
                lb = 2 + k / 4;
                const int c = k % 4;
                la = c < 2 ? c : TX + c;
            }
        } else {
            la = j < 2 ? j : TX + j;
        }
        const bool in = j < RING;
        ring_p[jj] = in ? lb * PA + la : 0;
        ring_x[jj] = in ? wrapi(a0 + la - 2, na) : 0;
        ring_y[jj] = in ? wrapi(b0 + lb - HB, nb) : 0;
        ring_ab[jj] = (uint32_t)ring_y[jj] * na + ring_x[jj];
    }

    // PSUM: this thread's ring position (i, j) around the cross-section
    // (rows below and above, then the columns left and right), and the
    // partial densities of the target slices cc - 1, cc, cc + 1 of the
    // owned position (acc) and of the ring position (racc)
    int ring_i = 0, ring_j = 0;
    if (PSUM && tid < NRING) {
        if (tid < TX + 2) {
            ring_i = tid - 1;
            ring_j = -1;
        } else if (tid < 2 * (TX + 2)) {
            ring_i = tid - (TX + 2) - 1;
            ring_j = TY;
        } else {
            const int k = tid - 2 * (TX + 2);
            ring_j = k / 2;
            ring_i = (k & 1) ? TX : -1;
        }
    }
    real acc[3] = {real(0), real(0), real(0)}, racc[3] = {real(0), real(0), real(0)};
    const size_t box0 = (size_t)(bx + gridDim.x * (by + gridDim.y * bz)) * PF::size;
    auto box_at = [&](int k, int j, int i) { return box0 + (size_t)PF::index(i, j, k); };
    // sum of the staged populations that stream to in-plane position q =
    // (j + 1) SW + i + 1 from the slice cc, split by the slice they reach
    // (non-fluid and outside positions hold 0)
    auto gather = [&](int q, real (&a3)[3]) __attribute__((always_inline)) {
#pragma unroll
        for (int b = 0; b < Q; ++b)
            if (SLOT[b] >= 0)
                a3[L::ez[b] + 1] += s_fs[SPAD + SLOT[b] * SS + q - L::ex[b] - L::ey[b] * SW];
    };
    if constexpr (PSUM) {
        for (int e = tid; e < QS * SS + 2 * SPAD; e += NT) s_fs[e] = real(0);
        // (the first barrier of the sweep orders these before any use)
    }

    // PSUM phase D for the slice cc_ collided last (staged in s_fs): its
    // contributions to the slices around it, then the slice below it is
    // complete for this block.  Runs after the barrier that follows the next
    // phase A, so it needs no barrier of its own; the classes of the slice
    // below are in ring slot sl_below.
    auto psum_phase = [&](int cc_, int sl_below) __attribute__((always_inline)) {
        const int oi = tid % TX, oj = tid / TX;
        gather((oj + 1) * SW + oi + 1, acc);
        if (tid < NRING) gather((ring_j + 1) * SW + ring_i + 1, racc);
        const int t = cc_ - 1;
        if (t >= c0) {
            Fd.rho_next[(uint32_t)t * nab + own_ab] =
                (s_cls[sl_below][own_p] == CLS_FLUID) ? acc[0] : real(0);
        } else {
            Fd.ring[box_at(-1, oj, oi)] = acc[0];  // the face below the block
        }
        if (tid < NRING) Fd.ring[box_at(t - c0, ring_j, ring_i)] = racc[0];
        acc[0] = acc[1];
        acc[1] = acc[2];
        acc[2] = real(0);
        racc[0] = racc[1];
        racc[1] = racc[2];
        racc[2] = real(0);
    };

    bool bad = false;
    double d_sum = 0.0;
    real d_umax = real(0), d_rmin = real(1e30), d_rmax = real(-1e30);
    int d_cnt = 0;

    // classes and densities of the next slice to enter the rings (not
    // fused): loaded one iteration before phase A writes them to LDS, so
    // the barrier after phase A does not wait for HBM
    uint8_t pc_own = CLS_SOLID, pc_ring[JR];
    real pr_own = real(0), pr_ring[JR];
    auto issue_slice = [&](int it) __attribute__((always_inline)) {
        const uint32_t base = (uint32_t)wrapi(c0 - 2 + it, nc) * nab;
        pc_own = Fd.cls[base + own_ab];
        pr_own = Fd.rho[base + own_ab];
#pragma unroll
        for (int jj = 0; jj < JR; ++jj) {
            pc_ring[jj] = CLS_SOLID;
            pr_ring[jj] = real(0);
            if (tid + jj * NT < RING) {
                pc_ring[jj] = Fd.cls[base + ring_ab[jj]];
                pr_ring[jj] = Fd.rho[base + ring_ab[jj]];
            }
        }
    };

    // Rl: populations of the owned node of slice c0 - 2 + it (fused only);
    // Rc: those of slice c0 - 4 + it, loaded two iterations earlier (fused)
    // or in phase A of this iteration
    auto body = [&](const int it, real (&Rl)[Q], real (&Rc)[Q]) __attribute__((always_inline)) {
        // ---------------- A: slice c0 - 2 + it
        {
            const int slot = it % NSLOT;
            const int cz = wrapi(c0 - 2 + it, nc);
            const uint32_t base = (uint32_t)cz * nab;
            if constexpr (FUSED) {
                // density of each node in velocity order, 0 off the fluid
                const uint8_t oc = Fd.cls[base + own_ab];
#pragma unroll
                for (int a = 0; a < Q; ++a)
                    Rl[a] = io.ld(a, PULL ? up_node<L>(a, own_aw, own_bw, cz, na, nb, nc, nab)
                                          : base + own_ab);
                uint8_t rc = CLS_SOLID;
                real rr = real(0);
                if (tid < RING) {
                    rc = Fd.cls[base + ring_ab[0]];
                    rr = io.ld(0, base + ring_ab[0]);
#pragma unroll
                    for (int a = 1; a < Q; ++a)
                        rr += io.ld(a, PULL ? up_node<L>(a, ring_x[0], ring_y[0], cz, na, nb, nc, nab)
                                            : base + ring_ab[0]);
                }
                real r = Rl[0];
#pragma unroll
                for (int a = 1; a < Q; ++a) r += Rl[a];
                s_cls[slot][own_p] = oc;
                s_rho[slot][own_p] = oc == CLS_FLUID ? r : real(0);
                if (tid < RING) {
                    s_cls[slot][ring_p[0]] = rc;
                    s_rho[slot][ring_p[0]] = rc == CLS_FLUID ? rr : real(0);
                }
            } else {
                // the owned node's populations of the slice phase C collides
                // in this iteration (its class arrived two iterations ago):
                // issued here, so that the barriers and phase B cover their
                // latency
                const int ccA = c0 - 4 + it;
                if (it >= 4 && ccA < nc && own_in &&
                    s_cls[(it - 2) % NSLOT][own_p] == CLS_FLUID) {
#pragma unroll
                    for (int a = 0; a < Q; ++a)
                        Rc[a] = io.ld(a, PULL ? up_node<L>(a, own_a, own_b, ccA, na, nb, nc, nab)
                                              : (uint32_t)ccA * nab + own_ab);
                }
                // densities come from the density pass: one value per node,
                // loaded in the previous iteration
                s_cls[slot][own_p] = pc_own;
                s_rho[slot][own_p] = pr_own;
#pragma unroll
                for (int jj = 0; jj < JR; ++jj) {
                    if (tid + jj * NT < RING) {
                        s_cls[slot][ring_p[jj]] = pc_ring[jj];
                        s_rho[slot][ring_p[jj]] = pr_ring[jj];
                    }
                }
                if (it + 1 < TZ + 4) issue_slice(it + 1);
            }
        }
        __syncthreads();
        // ---------------- D (PSUM) of the slice collided in the previous iteration
        if constexpr (PSUM) {
            if (it >= 5) psum_phase(c0 - 5 + it, (it - 4) % NSLOT);
        }
        // ---------------- B: psi (and wall densities) of slice c0 - 3 + it
        if (it >= 2) {
            const int sc = (it - 1) % NSLOT;
            const int sp = (it - 1) % NPSI;
            const int cz = wrapi(c0 - 3 + it, nc);
            constexpr int TA = TX + 2, TB = D3 ? TY + 2 : 1;
            for (int i = tid; i < TA * TB; i += NT) {
                const int la = 1 + i % TA;
                const int lb = D3 ? 1 + i / TA : 0;
                const int p = lb * PA + la;
                const uint8_t c = s_cls[sc][p];
                real ps = real(0);
                if (c == CLS_FLUID) {
                    ps = psi_of(C, s_rho[sc][p], bad);
                } else if (c == CLS_WALL) {
                    if (C.scheme == WET_IVD) {
                        real num = real(0), den = real(0);
                        bool first = true;
#pragma unroll
                        for (int a = 1; a < Q; ++a) {
                            const int ea = L::ex[a];
                            const int eb = D3 ? L::ey[a] : 0;
                            const int ec = D3 ? L::ez[a] : L::ey[a];
                            const int s2 = (it - 1 + ec + NSLOT) % NSLOT;
                            const int q = p + ea + eb * PA;
                            if (s_cls[s2][q] == CLS_FLUID) {
                                const real w = real(L::w12[a]) * real(1.0 / 12.0);
                                num = first ? w * s_rho[s2][q] : num + w * s_rho[s2][q];
                                den = first ? w : den + w;
                                first = false;
                            }
                        }
                        const real rave = num / den;
                        const uint32_t n = (uint32_t)cz * nab +
                                           (uint32_t)wrapi(b0 + lb - HB, nb) * na + wrapi(a0 + la - 2, na);
                        const int kw = Fd.widx[n];
                        real rw = Fd.phi[kw] * rave - Fd.drho[kw];
                        rw = rw > C.rho_l ? C.rho_l : rw;
                        rw = rw < C.rho_g ? C.rho_g : rw;
                        s_rho[sc][p] = rw;
                        ps = psi_of(C, rw, bad);
                    } else if (C.scheme == WET_VD) {
                        s_rho[sc][p] = C.rho_w;
                        ps = C.psi_w;
                    } else {
                        s_rho[sc][p] = real(0);
                    }
                }
                s_psi[sp][p] = ps;
            }
        }
        __syncthreads();
        // ---------------- C: collide and stream slice c0 - 4 + it
        const int cc = c0 - 4 + it;
        if (it >= 4 && cc < nc && own_in) {
            const int sc = (it - 2) % NSLOT;
            const int sp = (it - 2) % NPSI;
            const uint32_t n = (uint32_t)cc * nab + own_ab;
            const uint8_t c = s_cls[sc][own_p];
            if (c != CLS_FLUID) {
                if (MODE == MODE_FIELDS) {
                    if (Out.rho) Out.rho[n] = (c == CLS_WALL) ? s_rho[sc][own_p] : real(0);
                    if (Out.u)
                        for (int d = 0; d < L::D; ++d) Out.u[(size_t)d * N + n] = real(0);
                }
                if constexpr (PSUM) {
                    // a non-fluid position sends nothing
                    const int q = (tid / TX + 1) * SW + tid % TX + 1;
#pragma unroll
                    for (int a = 0; a < QS; ++a) s_fs[SPAD + a * SS + q] = real(0);
                }
            } else {
                const real rho = s_rho[sc][own_p];
                const real psi_c = s_psi[sp][own_p];
                real sm[3] = {real(0), real(0), real(0)}, sa[3] = {real(0), real(0), real(0)};
#pragma unroll
                for (int a = 1; a < Q; ++a) {
                    const int ea = L::ex[a];
                    const int eb = D3 ? L::ey[a] : 0;
                    const int ec = D3 ? L::ez[a] : L::ey[a];
                    const int q = own_p + ea + eb * PA;
                    const int s2 = (it - 2 + ec + NPSI) % NPSI;
                    const real w = real(L::w12[a]) * real(1.0 / 12.0);
                    // FP32: w (psi(x+e) - psi(x)), equal since sum w e = 0,
                    // with rounding that scales with the psi gradient
                    const real wp = (sizeof(real) == 4) ? w * (s_psi[s2][q] - psi_c)
                                                        : w * s_psi[s2][q];
                    const int e3[3] = {L::ex[a], L::ey[a], L::ez[a]};
#pragma unroll
                    for (int d = 0; d < L::D; ++d) {
                        if (e3[d] == 1) sm[d] += wp;
                        if (e3[d] == -1) sm[d] -= wp;
                    }
                    if (C.scheme == WET_SFI) {
                        const int s3 = (it - 2 + ec + NSLOT) % NSLOT;
                        if (s_cls[s3][q] != CLS_FLUID) {
#pragma unroll
                            for (int d = 0; d < L::D; ++d) {
                                if (e3[d] == 1) sa[d] += w;
                                if (e3[d] == -1) sa[d] -= w;
                            }
                        }
                    }
                }
                real Fm[3], F[3];
#pragma unroll
                for (int d = 0; d < 3; ++d) {
                    Fm[d] = (d < L::D) ? -C.G * psi_c * sm[d] : real(0);
                    const real fa = (C.scheme == WET_SFI) ? -C.G_w * rho * sa[d] : real(0);
                    F[d] = (d < L::D) ? Fm[d] + fa + C.body[d] : real(0);
                }
                real fl[Q];
#pragma unroll
                for (int a = 0; a < Q; ++a) fl[a] = Rc[a];
                if (MODE == MODE_FIELDS) {
                    real j[3] = {real(0), real(0), real(0)};
#pragma unroll
                    for (int a = 0; a < Q; ++a) {
                        const int e3[3] = {L::ex[a], L::ey[a], L::ez[a]};
#pragma unroll
                        for (int d = 0; d < L::D; ++d) {
                            if (e3[d] == 1) j[d] += fl[a];
                            if (e3[d] == -1) j[d] -= fl[a];
                        }
                    }
                    real uu = real(0);
#pragma unroll
                    for (int d = 0; d < L::D; ++d) {
                        const real ud = (j[d] + real(0.5) * F[d]) / rho;
                        if (Out.u) Out.u[(size_t)d * N + n] = ud;
                        uu += ud * ud;
                    }
                    if (Out.rho) Out.rho[n] = rho;
                    const real um = sqrt(uu);
                    // mass: the node's populations summed in FP64 (in FP32
                    // the density's own rounding repeats at every node of a
                    // uniform region and would bias the total)
                    double rs = (double)fl[0];
#pragma unroll
                    for (int a = 1; a < Q; ++a) rs += (double)fl[a];
                    d_sum += rs;
                    d_umax = um > d_umax ? um : d_umax;
                    d_rmin = rho < d_rmin ? rho : d_rmin;
                    d_rmax = rho > d_rmax ? rho : d_rmax;
                    d_cnt += 1;
                } else {
                    real fs[Q], u[3];
                    collide<L, real>(C, fl, rho, F, Fm, psi_c, fs, u);
                    const int ga = own_a, gb = D3 ? own_b : 0;
                    real bsum = real(0);  // PSUM: bounce-backs return to this node
                    uint32_t wmask = 0;   // pull form: directions whose neighbour is not fluid
#pragma unroll
                    for (int a = 0; a < Q; ++a) {
                        const int ea = L::ex[a];
                        const int eb = D3 ? L::ey[a] : 0;
                        const int ec = D3 ? L::ez[a] : L::ey[a];
                        const int s3 = (it - 2 + ec + NSLOT) % NSLOT;
                        const int q = own_p + ea + eb * PA;
                        const bool fluid_to = s_cls[s3][q] == CLS_FLUID;
                        if constexpr (PULL) {
                            // own slot; the bounce-backs follow, in one branch
                            // that waves away from walls skip
                            io.st_nt(a, n, fs[a]);
                            wmask |= fluid_to ? 0u : (1u << a);
                            if (PSUM) bsum += fluid_to ? real(0) : fs[a];
                        } else {
                            int ta = ga + ea, tb = gb + eb, tc = cc + ec;
                            ta = ta < 0 ? ta + na : (ta >= na ? ta - na : ta);
                            tb = tb < 0 ? tb + nb : (tb >= nb ? tb - nb : tb);
                            tc = tc < 0 ? tc + nc : (tc >= nc ? tc - nc : tc);
                            const uint32_t t = (uint32_t)tc * nab + (uint32_t)tb * na + ta;
                            if (fluid_to) io.st(a, t, fs[a]);
                            else io.st(L::opp[a], n, fs[a]);
                        }
                    }
                    if constexpr (PULL) {
                        if (wmask != 0u) {
                            // a wall neighbour's slot opp(a) gets f*_a, where the
                            // gather of direction opp(a) at this node looks
#pragma unroll
                            for (int a = 1; a < Q; ++a) {
                                if ((wmask >> a) & 1u) {
                                    int ta = ga + L::ex[a], tb = gb + L::ey[a], tc = cc + L::ez[a];
                                    ta = ta < 0 ? ta + na : (ta >= na ? ta - na : ta);
                                    tb = tb < 0 ? tb + nb : (tb >= nb ? tb - nb : tb);
                                    tc = tc < 0 ? tc + nc : (tc >= nc ? tc - nc : tc);
                                    io.st(L::opp[a], (uint32_t)tc * nab + (uint32_t)tb * na + ta,
                                          fs[a]);
                                }
                            }
                        }
                    }
                    if constexpr (PSUM) {
                        const int q = (tid / TX + 1) * SW + tid % TX + 1;
#pragma unroll
                        for (int a = 0; a < Q; ++a)
                            if (SLOT[a] >= 0) s_fs[SPAD + SLOT[a] * SS + q] = fs[a];
                        // what stays in the column: the rest population and
                        // +-z (slices cc, cc + 1, cc - 1), and the bounce-backs
                        acc[1] += fs[0] + bsum;
                        acc[2] += fs[5];
                        acc[0] += fs[6];
                    }
                }
            }
        }
        // no barrier here: the next phase A writes slot (it+1) mod 5, which
        // phase C of this iteration does not read (it reads it-3 .. it-1)
    };
    if constexpr (FUSED) {
        real R0[Q], R1[Q], R2[Q];
        for (int it = 0; it < TZ + 4; it += 3) {
            body(it, R0, R1);
            if (it + 1 < TZ + 4) body(it + 1, R1, R2);
            if (it + 2 < TZ + 4) body(it + 2, R2, R0);
        }
    } else {
        real R0[Q];
        issue_slice(0);
        for (int it = 0; it < TZ + 4; ++it) body(it, R0, R0);
    }
    if constexpr (PSUM) {
        // phase D of the last slice, then the top slice of the chunk (partial)
        // and the face above the block
        __syncthreads();
        psum_phase(c0 + TZ - 1, TZ % NSLOT);
        const int oi = tid % TX, oj = tid / TX;
        const int st = (TZ + 1) % NSLOT;  // classes of slice c0 + TZ - 1
        Fd.rho_next[(uint32_t)(c0 + TZ - 1) * nab + own_ab] =
            (s_cls[st][own_p] == CLS_FLUID) ? acc[0] : real(0);
        Fd.ring[box_at(TZ, oj, oi)] = acc[1];
        if (tid < NRING) {
            Fd.ring[box_at(TZ - 1, ring_j, ring_i)] = racc[0];
            Fd.ring[box_at(TZ, ring_j, ring_i)] = racc[1];
        }
    }

    if (MODE == MODE_FIELDS && Out.part) {
        block_reduce_diag<NT>(d_sum, d_umax, d_rmin, d_rmax, d_cnt, Out.part + 5 * bid);
    }
    if (bad) Fd.flag[0] = 1;
}


// D3Q19 step on a TX x TY x TZ brick with no march: after the density pass,
// one load phase brings the node classes and densities of the brick plus a
// 2-node halo in every direction (one value per node, mostly from L2) and
// each thread's TZ owned nodes' populations into registers; psi (with the
// wall virtual densities) follows on the brick plus a 1-node halo, then the
// owned nodes collide and store (pull form).  Two barriers per brick and no dependent
// chain along z, so many independent workgroups hide the memory latency.
// Step mode only (the field/diagnostic pass uses the sweep).
template <typename real, int TX, int TY, int TZ, bool XCD>
__global__ __launch_bounds__(TX* TY) void k_step_brick(Coef<real> C, Fields<real> Fd) {
    using L = D3Q19;
    constexpr int Q = 19, NT = TX * TY;
    constexpr int PX = TX + 4, PY = TY + 4, PZ = TZ + 4, PXY = PX * PY, PS = PXY * PZ;
    __shared__ uint8_t s_cls[PS];
    __shared__ real s_rho[PS];
    __shared__ real s_psi[PS];

    const int na = C.nx, nb = C.ny, nc = C.nz;
    const uint32_t nab = (uint32_t)na * (uint32_t)nb;
    const uint32_t N = nab * (uint32_t)nc;
    const PopIO<real, true> io(Fd.fin, Fd.fout, N, Q);
    const int tid = threadIdx.x;
    const int nblk = gridDim.x * gridDim.y * gridDim.z;
    int bid = blockIdx.x + gridDim.x * (blockIdx.y + gridDim.y * blockIdx.z);
    if (XCD) bid = remap_xcd(bid, nblk);
    const int bx = bid % gridDim.x, by = (bid / gridDim.x) % gridDim.y;
    const int bz = bid / (gridDim.x * gridDim.y);
    const int a0 = bx * TX, b0 = by * TY, c0 = bz * TZ;
    const int tx = tid % TX, ty = tid / TX;
    bool bad = false;

    // ---- one load phase: classes and densities of the halo box, owned populations
    const int ga = a0 + tx, gb = b0 + ty;
    const bool own_xy = ga < na && gb < nb;
    const uint32_t own_ab = (uint32_t)wrapi(gb, nb) * na + wrapi(ga, na);
    const int gaw = wrapi(ga, na), gbw = wrapi(gb, nb);
    real f[TZ][Q];
#pragma unroll
    for (int k = 0; k < TZ; ++k) {
        const int gcw = wrapi(c0 + k, nc);
#pragma unroll
        for (int a = 0; a < Q; ++a) f[k][a] = io.ld(a, up_node<L>(a, gaw, gbw, gcw, na, nb, nc, nab));
    }
    constexpr int JB = (PS + NT - 1) / NT;
    uint8_t hc[JB];
    real hr[JB];
#pragma unroll
    for (int j = 0; j < JB; ++j) {
        const int i = tid + j * NT;
        hc[j] = CLS_SOLID;
        hr[j] = real(0);
        if (i < PS) {
            const int lx = i % PX, ly = (i / PX) % PY, lz = i / PXY;
            const uint32_t n = (uint32_t)wrapi(c0 - 2 + lz, nc) * nab +
                               (uint32_t)wrapi(b0 - 2 + ly, nb) * na + wrapi(a0 - 2 + lx, na);
            hc[j] = Fd.cls[n];
            hr[j] = Fd.rho[n];
        }
    }
#pragma unroll
    for (int j = 0; j < JB; ++j) {
        const int i = tid + j * NT;
        if (i < PS) {
            s_cls[i] = hc[j];
            s_rho[i] = hr[j];
        }
    }
    __syncthreads();

    // ---- psi on the brick plus a 1-node halo; wall nodes get their virtual density
    constexpr int IX = TX + 2, IY = TY + 2, IZ = TZ + 2;
    for (int i = tid; i < IX * IY * IZ; i += NT) {
        const int lx = 1 + i % IX, ly = 1 + (i / IX) % IY, lz = 1 + i / (IX * IY);
        const int p = (lz * PY + ly) * PX + lx;
        const uint8_t c = s_cls[p];
        real ps = real(0);
        if (c == CLS_FLUID) {
            ps = psi_of(C, s_rho[p], bad);
        } else if (c == CLS_WALL) {
            if (C.scheme == WET_IVD) {
                // Eq. 17 over the fluid neighbours, Eq. 16 and the limiter
                real num = real(0), den = real(0);
                bool first = true;
#pragma unroll
                for (int a = 1; a < Q; ++a) {
                    const int q = p + L::ex[a] + L::ey[a] * PX + L::ez[a] * PXY;
                    if (s_cls[q] == CLS_FLUID) {
                        const real w = real(L::w12[a]) * real(1.0 / 12.0);
                        num = first ? w * s_rho[q] : num + w * s_rho[q];
                        den = first ? w : den + w;
                        first = false;
                    }
                }
                const real rave = num / den;
                const uint32_t n = (uint32_t)wrapi(c0 - 2 + lz, nc) * nab +
                                   (uint32_t)wrapi(b0 - 2 + ly, nb) * na + wrapi(a0 - 2 + lx, na);
                const int kw = Fd.widx[n];
                real rw = Fd.phi[kw] * rave - Fd.drho[kw];
                rw = rw > C.rho_l ? C.rho_l : rw;
                rw = rw < C.rho_g ? C.rho_g : rw;
                ps = psi_of(C, rw, bad);
            } else if (C.scheme == WET_VD) {
                ps = C.psi_w;
            }
        }
        s_psi[p] = ps;
    }
    __syncthreads();

    // ---- owned nodes: force (Eq. 5, Eq. 8), collision, pull-form store
#pragma unroll
    for (int k = 0; k < TZ; ++k) {
        const int gc = c0 + k;
        if (!own_xy || gc >= nc) continue;  // ragged brick: not owned
        const int p = ((k + 2) * PY + ty + 2) * PX + tx + 2;
        if (s_cls[p] != CLS_FLUID) continue;
        const uint32_t n = (uint32_t)gc * nab + own_ab;
        const real rho = s_rho[p];
        const real psi_c = s_psi[p];
        real sm[3] = {real(0), real(0), real(0)}, sa[3] = {real(0), real(0), real(0)};
#pragma unroll
        for (int a = 1; a < Q; ++a) {
            const int q = p + L::ex[a] + L::ey[a] * PX + L::ez[a] * PXY;
            const real w = real(L::w12[a]) * real(1.0 / 12.0);
            // FP32: w (psi(x+e) - psi(x)), equal since sum w e = 0
            const real wp = (sizeof(real) == 4) ? w * (s_psi[q] - psi_c) : w * s_psi[q];
            const int e3[3] = {L::ex[a], L::ey[a], L::ez[a]};
#pragma unroll
            for (int d = 0; d < 3; ++d) {
                if (e3[d] == 1) sm[d] += wp;
                if (e3[d] == -1) sm[d] -= wp;
            }
            if (C.scheme == WET_SFI && s_cls[q] != CLS_FLUID) {
#pragma unroll
                for (int d = 0; d < 3; ++d) {
                    if (e3[d] == 1) sa[d] += w;
                    if (e3[d] == -1) sa[d] -= w;
                }
            }
        }
        real Fm[3], F[3];
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            Fm[d] = -C.G * psi_c * sm[d];
            const real fa = (C.scheme == WET_SFI) ? -C.G_w * rho * sa[d] : real(0);
            F[d] = Fm[d] + fa + C.body[d];
        }
        real fs[Q], u[3];
        collide<L, real>(C, f[k], rho, F, Fm, psi_c, fs, u);
#pragma unroll
        for (int a = 0; a < Q; ++a) {
            // pull form: own slot; a wall neighbour also gets the bounce-back
            io.st_nt(a, n, fs[a]);
            const int q = p + L::ex[a] + L::ey[a] * PX + L::ez[a] * PXY;
            if (s_cls[q] != CLS_FLUID) {
                int ta = ga + L::ex[a], tb = gb + L::ey[a], tc = gc + L::ez[a];
                ta = ta < 0 ? ta + na : (ta >= na ? ta - na : ta);
                tb = tb < 0 ? tb + nb : (tb >= nb ? tb - nb : tb);
                tc = tc < 0 ? tc + nc : (tc >= nc ? tc - nc : tc);
                io.st(L::opp[a], (uint32_t)tc * nab + (uint32_t)tb * na + ta, fs[a]);
            }
        }
    }
    if (bad) Fd.flag[0] = 1;
}

// ----------------------------------------------------------------- launch
// Sweep-tile variants the autotuner chooses among (variant 0: default and
// the shape of the field/diagnostic mode).
struct Shape3D {
    int TX, TY, TZ;
    bool xcd;
    bool fused;  // densities summed in the sweep (no density pass)
    int occ;     // minimum waves per SIMD asked of the register allocator
    bool brick;  // k_step_brick: no march, TZ slices per thread
    bool psum = false;  // the sweep forms the next step's density (no density pass)
};

template <typename real>
struct Variants3D;
template <>
struct Variants3D<float> {
    static constexpr int count = 14;
    static constexpr int preferred = 2;  // 32 x 8 cross-section, chunks of 8 slices
    // on lattices their blocks tile, in this order: the sweeps that form the
    // next density (32 x 8 x 8: 0.662 ms against 0.805 ms for the best
    // plain sweep and its density pass, a step on the 256^3 sphere)
    static constexpr int npsum = 2;
    static constexpr int preferred_psum[npsum] = {10, 11};
    static constexpr Shape3D shape[count] = {
        {32, 8, 16, true, false, 1, false}, {32, 8, 16, false, false, 1, false},
        {32, 8, 8, true, false, 1, false},  {32, 8, 32, true, false, 1, false},
        {16, 16, 16, true, false, 1, false}, {32, 8, 16, true, true, 1, false},
        {32, 8, 32, true, true, 1, false},  {32, 8, 2, true, false, 1, true},
        {64, 4, 16, true, false, 1, false}, {256, 2, 16, true, false, 1, false},
        {32, 8, 8, true, false, 4, false, true}, {32, 8, 16, true, false, 4, false, true},
        {32, 8, 32, true, false, 4, false, true}, {32, 8, 32, true, false, 1, false, true}};
};
template <>
struct Variants3D<double> {
    static constexpr int count = 5;
    static constexpr int preferred = 3;  // the brick: 1.63 ms against 1.76 ms on the 256^3 sphere
    static constexpr int npsum = 0;
    static constexpr int preferred_psum[1] = {-1};
    static constexpr Shape3D shape[count] = {
        {32, 8, 16, true, false, 1, false}, {32, 8, 16, false, false, 1, false},
        {32, 8, 16, true, true, 1, false}, {32, 8, 2, true, false, 1, true},
        {32, 8, 16, true, false, 1, false, true}};
};

template <typename real>
int step3d_variants() {
    return Variants3D<real>::count;
}

template <typename real>
static bool psum_applies(const Coef<real>& C, const Shape3D& sh);

// the variant a D3Q19 context starts with (fastest on the 256^3 benchmark)
template <typename real>
int step3d_preferred_variant(int nx, int ny, int nz) {
    Coef<real> C{};
    C.nx = nx;
    C.ny = ny;
    C.nz = nz;
    for (int k = 0; k < Variants3D<real>::npsum; ++k) {
        const int v = Variants3D<real>::preferred_psum[k];
        if (psum_applies(C, Variants3D<real>::shape[v])) return v;
    }
    return Variants3D<real>::preferred;
}

template <typename real>
int grid3d_blocks(int nx, int ny, int nz, int variant) {
    const Shape3D s = Variants3D<real>::shape[variant];
    return ((nx + s.TX - 1) / s.TX) * ((ny + s.TY - 1) / s.TY) * ((nz + s.TZ - 1) / s.TZ);
}

// a PSUM variant forms the next density only on lattices its blocks tile
// exactly (otherwise it runs as the plain sweep of its shape)
template <typename real>
static bool psum_applies(const Coef<real>& C, const Shape3D& sh) {
    return sh.psum && C.nx % sh.TX == 0 && C.ny % sh.TY == 0 && C.nz % sh.TZ == 0 &&
           (uint64_t)19 * (uint64_t)C.nx * C.ny * C.nz * sizeof(real) <= 0xFFFFFFFFull;
}

template <typename real, int V, int MODE, bool BUF = true>
static void launch_v3(const Coef<real>& C, const Fields<real>& F, const FieldOut<real>& O,
                      hipStream_t s) {
    constexpr Shape3D sh = Variants3D<real>::shape[V];
    dim3 grid((C.nx + sh.TX - 1) / sh.TX, (C.ny + sh.TY - 1) / sh.TY, (C.nz + sh.TZ - 1) / sh.TZ);
    if constexpr (sh.brick && MODE == MODE_STEP && BUF) {
        hipLaunchKernelGGL((k_step_brick<real, sh.TX, sh.TY, sh.TZ, sh.xcd>), grid,
                           dim3(sh.TX * sh.TY), 0, s, C, F);
    } else if constexpr (sh.psum && MODE == MODE_STEP && BUF) {
        if (psum_applies(C, sh)) {
            hipLaunchKernelGGL(
                (k_step_march<D3Q19, real, sh.TX, sh.TY, sh.TZ, MODE_STEP, sh.xcd, true, false,
                              sh.occ, true>),
                grid, dim3(sh.TX * sh.TY), 0, s, C, F, O);
            constexpr uint32_t fpb = 2 * sh.TX * sh.TY + 2 * sh.TX * (sh.TZ - 2) +
                                     2 * (sh.TY - 2) * (sh.TZ - 2);
            const uint32_t faces = (uint32_t)(C.nx / sh.TX) * (uint32_t)(C.ny / sh.TY) *
                                   (uint32_t)(C.nz / sh.TZ) * fpb;
            constexpr int NPT = 2;  // face nodes per thread
            hipLaunchKernelGGL((k_psum_close<real, sh.TX, sh.TY, sh.TZ, NPT>),
                               dim3((faces + 256 * NPT - 1) / (256 * NPT)), dim3(256), 0, s, F.cls,
                               F.rho_next, F.ring, C.nx, C.ny, C.nz);
        } else {
            hipLaunchKernelGGL((k_step_march<D3Q19, real, sh.TX, sh.TY, sh.TZ, MODE_STEP, sh.xcd,
                                             true, false, sh.occ>),
                               grid, dim3(sh.TX * sh.TY), 0, s, C, F, O);
        }
    } else {
        hipLaunchKernelGGL(
            (k_step_march<D3Q19, real, sh.TX, sh.TY, sh.TZ, MODE, sh.xcd, BUF, sh.fused, sh.occ>),
            grid, dim3(sh.TX * sh.TY), 0, s, C, F, O);
    }
}

template <typename real, size_t... I>
static auto table_v3(std::index_sequence<I...>) {
    using Fn = void (*)(const Coef<real>&, const Fields<real>&, const FieldOut<real>&,
                        hipStream_t);
    return std::array<Fn, sizeof...(I)>{&launch_v3<real, (int)I, MODE_STEP>...};
}

// whether a step of this variant leaves the density of its output state in
// Fd.rho_next (a PSUM sweep on a lattice its blocks tile)
template <typename real>
bool step3d_forms_density(const Coef<real>& C, int variant) {
    if (variant < 0 || variant >= Variants3D<real>::count) return false;
    return psum_applies(C, Variants3D<real>::shape[variant]);
}

// elements of the per-block partial-sum boxes the PSUM variants need (the
// largest over those variants; 0 when none applies to the lattice)
template <typename real>
size_t step3d_ring_elems(int nx, int ny, int nz) {
    size_t m = 0;
    for (int v = 0; v < Variants3D<real>::count; ++v) {
        const Shape3D sh = Variants3D<real>::shape[v];
        if (!sh.psum || nx % sh.TX || ny % sh.TY || nz % sh.TZ) continue;
        const size_t e = (size_t)(nx / sh.TX) * (ny / sh.TY) * (nz / sh.TZ) *
                         (size_t)(2 * (sh.TY + 2) * (sh.TX + 2) + 2 * sh.TZ * (sh.TX + 2) +
                                  2 * sh.TZ * sh.TY);
        m = e > m ? e : m;
    }
    return m;
}

// the density pass alone, into Fd.rho (the density of Fd.fin)
template <typename real>
hipError_t launch_density3d(const Coef<real>& C, const Fields<real>& F, hipStream_t s) {
    launch_density<D3Q19, real>(C, F, s);
    return hipGetLastError();
}

// Fd.rho_valid: Fd.rho already holds the density of Fd.fin, so the density
// pass is skipped (the density a PSUM step formed, or one computed since)
template <typename real>
hipError_t launch_step3d(const Coef<real>& C, const Fields<real>& F, const FieldOut<real>& O,
                         int mode, int variant, hipStream_t s) {
    if (mode == MODE_FIELDS) variant = 0;
    if (variant < 0 || variant >= Variants3D<real>::count) return hipErrorInvalidValue;
    // population arrays of 4 GiB or more cannot use 32-bit buffer offsets
    if ((uint64_t)19 * (uint64_t)C.nx * C.ny * C.nz * sizeof(real) > 0xFFFFFFFFull) {
        if (!F.rho_valid) launch_density<D3Q19, real>(C, F, s);
        if (mode == MODE_STEP) launch_v3<real, 0, MODE_STEP, false>(C, F, O, s);
        else launch_v3<real, 0, MODE_FIELDS, false>(C, F, O, s);
        return hipGetLastError();
    }
    if (mode == MODE_FIELDS) {
        if (!F.rho_valid) launch_density<D3Q19, real>(C, F, s);
        launch_v3<real, 0, MODE_FIELDS>(C, F, O, s);
        return hipGetLastError();
    }
    if (!Variants3D<real>::shape[variant].fused && !F.rho_valid)
        launch_density<D3Q19, real>(C, F, s);
    static const auto tab = table_v3<real>(std::make_index_sequence<Variants3D<real>::count>{});
    tab[variant](C, F, O, s);
    return hipGetLastError();
}

// D2Q9 sweeping along y: a TX-wide strip (TY = 1) and chunks of TZ rows
struct Shape2M {
    int TX, TZ;
};
template <typename real>
struct Variants2M;
template <>
struct Variants2M<float> {
    static constexpr int count = 3;
    static constexpr Shape2M shape[count] = {{256, 32}, {256, 16}, {64, 16}};
};
template <>
struct Variants2M<double> {
    static constexpr int count = 1;
    static constexpr Shape2M shape[count] = {{128, 16}};
};

template <typename real>
int step2d_march_variants() {
    return Variants2M<real>::count;
}

template <typename real, int V, int MODE>
static void launch_v2m(const Coef<real>& C, const Fields<real>& F, const FieldOut<real>& O,
                       hipStream_t s) {
    constexpr Shape2M sh = Variants2M<real>::shape[V];
    dim3 grid((C.nx + sh.TX - 1) / sh.TX, 1, (C.ny + sh.TZ - 1) / sh.TZ);
    hipLaunchKernelGGL((k_step_march<D2Q9, real, sh.TX, 1, sh.TZ, MODE, true, true>), grid,
                       dim3(sh.TX), 0, s, C, F, O);
}

// (step mode only; the caller has checked that the populations fit a buffer)
template <typename real>
hipError_t launch_step2d_march(const Coef<real>& C, const Fields<real>& F, const FieldOut<real>& O,
                               int idx, hipStream_t s) {
    launch_density<D2Q9, real>(C, F, s);
    if (idx == 0) launch_v2m<real, 0, MODE_STEP>(C, F, O, s);
    else if constexpr (Variants2M<real>::count > 1) {
        if (idx == 1) launch_v2m<real, 1, MODE_STEP>(C, F, O, s);
        else if (idx == 2) launch_v2m<real, 2, MODE_STEP>(C, F, O, s);
        else return hipErrorInvalidValue;
    } else {
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

#if LBM_PREC != 8
template int step2d_march_variants<float>();
#endif
#if LBM_PREC != 4
template int step2d_march_variants<double>();
#endif
#if LBM_PREC != 8
template hipError_t launch_step2d_march<float>(const Coef<float>&, const Fields<float>&,
                                               const FieldOut<float>&, int, hipStream_t);
#endif
#if LBM_PREC != 4
template hipError_t launch_step2d_march<double>(const Coef<double>&, const Fields<double>&,
                                                const FieldOut<double>&, int, hipStream_t);
#endif
#if LBM_PREC != 8
template int step3d_variants<float>();
template int step3d_preferred_variant<float>(int, int, int);
#endif
#if LBM_PREC != 4
template int step3d_variants<double>();
template int step3d_preferred_variant<double>(int, int, int);
#endif
#if LBM_PREC != 8
template int grid3d_blocks<float>(int, int, int, int);
#endif
#if LBM_PREC != 4
template int grid3d_blocks<double>(int, int, int, int);
#endif
#if LBM_PREC != 8
template size_t step3d_ring_elems<float>(int, int, int);
#endif
#if LBM_PREC != 4
template size_t step3d_ring_elems<double>(int, int, int);
#endif
#if LBM_PREC != 8
template bool step3d_forms_density<float>(const Coef<float>&, int);
template hipError_t launch_density3d<float>(const Coef<float>&, const Fields<float>&, hipStream_t);
#endif
#if LBM_PREC != 4
template bool step3d_forms_density<double>(const Coef<double>&, int);
template hipError_t launch_density3d<double>(const Coef<double>&, const Fields<double>&,
                                             hipStream_t);
#endif
#if LBM_PREC != 8
template hipError_t launch_step3d<float>(const Coef<float>&, const Fields<float>&,
                                         const FieldOut<float>&, int, int, hipStream_t);
#endif
#if LBM_PREC != 4
template hipError_t launch_step3d<double>(const Coef<double>&, const Fields<double>&,
                                          const FieldOut<double>&, int, int, hipStream_t);
#endif

}  // namespace lbm
