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

// FUSED: no density pass.  Phase A loads the populations of its slice,
// sums the density of every node of the slice (owned and halo) itself and
// keeps the owned node's populations in registers until phase C collides
// them two iterations later (a ring of three register sets, so the loop
// body is instantiated three times with the sets rotated).
// OCC: minimum waves per SIMD asked of the register allocator.
template <typename L, typename real, int TX, int TY, int TZ, int MODE, bool XCD, bool BUF,
          bool FUSED = false, int OCC = 1>
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

    bool bad = false;
    double d_sum = 0.0;
    real d_umax = real(0), d_rmin = real(1e30), d_rmax = real(-1e30);
    int d_cnt = 0;

    // Rl: populations of the owned node of slice c0 - 2 + it (fused only);
    // Rc: those of slice c0 - 4 + it, loaded two iterations earlier
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
                // densities come from the density pass: one value per node
                s_cls[slot][own_p] = Fd.cls[base + own_ab];
                s_rho[slot][own_p] = Fd.rho[base + own_ab];
#pragma unroll
                for (int jj = 0; jj < JR; ++jj) {
                    if (tid + jj * NT < RING) {
                        s_cls[slot][ring_p[jj]] = Fd.cls[base + ring_ab[jj]];
                        s_rho[slot][ring_p[jj]] = Fd.rho[base + ring_ab[jj]];
                    }
                }
            }
        }
        __syncthreads();
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
                for (int a = 0; a < Q; ++a)
                    fl[a] = FUSED ? Rc[a]
                                  : io.ld(a, PULL ? up_node<L>(a, own_a, own_b, cc, na, nb, nc, nab) : n);
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
#pragma unroll
                    for (int a = 0; a < Q; ++a) {
                        const int ea = L::ex[a];
                        const int eb = D3 ? L::ey[a] : 0;
                        const int ec = D3 ? L::ez[a] : L::ey[a];
                        const int s3 = (it - 2 + ec + NSLOT) % NSLOT;
                        const int q = own_p + ea + eb * PA;
                        const bool fluid_to = s_cls[s3][q] == CLS_FLUID;
                        int ta = ga + ea, tb = gb + eb, tc = cc + ec;
                        ta = ta < 0 ? ta + na : (ta >= na ? ta - na : ta);
                        tb = tb < 0 ? tb + nb : (tb >= nb ? tb - nb : tb);
                        tc = tc < 0 ? tc + nc : (tc >= nc ? tc - nc : tc);
                        const uint32_t t = (uint32_t)tc * nab + (uint32_t)tb * na + ta;
                        if constexpr (PULL) {
                            // own slot; a wall neighbour also gets the bounce-back
                            io.st_nt(a, n, fs[a]);
                            if (!fluid_to) io.st(L::opp[a], t, fs[a]);
                        } else if (fluid_to) {
                            io.st(a, t, fs[a]);
                        } else {
                            io.st(L::opp[a], n, fs[a]);
                        }
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
        for (int it = 0; it < TZ + 4; ++it) body(it, R0, R0);
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
};

template <typename real>
struct Variants3D;
template <>
struct Variants3D<float> {
    static constexpr int count = 10;
    static constexpr int preferred = 2;  // 32 x 8 cross-section, chunks of 8 slices
    static constexpr Shape3D shape[count] = {
        {32, 8, 16, true, false, 1, false}, {32, 8, 16, false, false, 1, false},
        {32, 8, 8, true, false, 1, false},  {32, 8, 32, true, false, 1, false},
        {16, 16, 16, true, false, 1, false}, {32, 8, 16, true, true, 1, false},
        {32, 8, 32, true, true, 1, false},  {32, 8, 2, true, false, 1, true},
        {64, 4, 16, true, false, 1, false}, {256, 2, 16, true, false, 1, false}};
};
template <>
struct Variants3D<double> {
    static constexpr int count = 4;
    static constexpr int preferred = 3;  // the brick: 1.63 ms against 1.76 ms on the 256^3 sphere
    static constexpr Shape3D shape[count] = {
        {32, 8, 16, true, false, 1, false}, {32, 8, 16, false, false, 1, false},
        {32, 8, 16, true, true, 1, false}, {32, 8, 2, true, false, 1, true}};
};

template <typename real>
int step3d_variants() {
    return Variants3D<real>::count;
}

// the variant a D3Q19 context starts with (fastest on the 256^3 benchmark)
template <typename real>
int step3d_preferred_variant() {
    return Variants3D<real>::preferred;
}

template <typename real>
int grid3d_blocks(int nx, int ny, int nz, int variant) {
    const Shape3D s = Variants3D<real>::shape[variant];
    return ((nx + s.TX - 1) / s.TX) * ((ny + s.TY - 1) / s.TY) * ((nz + s.TZ - 1) / s.TZ);
}

template <typename real, int V, int MODE, bool BUF = true>
static void launch_v3(const Coef<real>& C, const Fields<real>& F, const FieldOut<real>& O,
                      hipStream_t s) {
    constexpr Shape3D sh = Variants3D<real>::shape[V];
    dim3 grid((C.nx + sh.TX - 1) / sh.TX, (C.ny + sh.TY - 1) / sh.TY, (C.nz + sh.TZ - 1) / sh.TZ);
    if constexpr (sh.brick && MODE == MODE_STEP && BUF)
        hipLaunchKernelGGL((k_step_brick<real, sh.TX, sh.TY, sh.TZ, sh.xcd>), grid,
                           dim3(sh.TX * sh.TY), 0, s, C, F);
    else
        hipLaunchKernelGGL(
            (k_step_march<D3Q19, real, sh.TX, sh.TY, sh.TZ, MODE, sh.xcd, BUF, sh.fused, sh.occ>),
            grid, dim3(sh.TX * sh.TY), 0, s, C, F, O);
}

template <typename real, size_t... I>
static auto table_v3(std::index_sequence<I...>) {
    using Fn = void (*)(const Coef<real>&, const Fields<real>&, const FieldOut<real>&,
                        hipStream_t);
    return std::array<Fn, sizeof...(I)>{&launch_v3<real, (int)I, MODE_STEP>...};
}

template <typename real>
hipError_t launch_step3d(const Coef<real>& C, const Fields<real>& F, const FieldOut<real>& O,
                         int mode, int variant, hipStream_t s) {
    if (mode == MODE_FIELDS) variant = 0;
    if (variant < 0 || variant >= Variants3D<real>::count) return hipErrorInvalidValue;
    // population arrays of 4 GiB or more cannot use 32-bit buffer offsets
    if ((uint64_t)19 * (uint64_t)C.nx * C.ny * C.nz * sizeof(real) > 0xFFFFFFFFull) {
        launch_density<D3Q19, real>(C, F, s);
        if (mode == MODE_STEP) launch_v3<real, 0, MODE_STEP, false>(C, F, O, s);
        else launch_v3<real, 0, MODE_FIELDS, false>(C, F, O, s);
        return hipGetLastError();
    }
    if (mode == MODE_FIELDS) {
        launch_density<D3Q19, real>(C, F, s);
        launch_v3<real, 0, MODE_FIELDS>(C, F, O, s);
        return hipGetLastError();
    }
    if (!Variants3D<real>::shape[variant].fused) launch_density<D3Q19, real>(C, F, s);
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
template int step3d_preferred_variant<float>();
#endif
#if LBM_PREC != 4
template int step3d_variants<double>();
template int step3d_preferred_variant<double>();
#endif
#if LBM_PREC != 8
template int grid3d_blocks<float>(int, int, int, int);
#endif
#if LBM_PREC != 4
template int grid3d_blocks<double>(int, int, int, int);
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
