// lbm_kernels.hpp -- launchers of the HIP kernels and the small device
// helpers the kernels share (wave64 / LDS reductions).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "lbm_device.hpp"

namespace lbm {

enum { MODE_STEP = 0, MODE_FIELDS = 1 };

// Outputs of the field mode of a step kernel: macroscopic fields and
// per-workgroup diagnostic partials (sum rho, max |u|, min rho, max rho,
// fluid count), each may be null.
template <typename real>
struct FieldOut {
    real* rho;
    real* u;
    double* part;
};

// Multi-case (batched) D2Q9 stepping: per-case descriptors and the
// workgroup -> (case, tile) table.  Offsets are element offsets into the
// packed arenas (populations: per ping-pong arena; node classes and wall
// indices: per-node arena; wetting parameters: per-wall arena).
struct CaseDesc {
    int32_t nx, ny;
    int32_t pitch, reserved;  // row pitch of the case's arrays (nodes), unused
    uint64_t f_off;
    uint64_t node_off;
    uint64_t wall_off;
};
struct TileRef {
    int32_t c, x0, y0, pad;
};
template <typename real>
struct BatchArgs {
    const real* fin;
    real* fout;
    const uint8_t* cls;
    const int32_t* widx;
    const real* phi;
    const real* drho;
    int32_t* flag;
    const CaseDesc* cases;
    const TileRef* tiles;
    // per-tile wall lists, indexed by tile-table position (see Fields)
    const int32_t* tw_pack = nullptr;
    const real* tw_phi = nullptr;
    const real* tw_drho = nullptr;
    int tw_stride = 0;
    const int32_t* tw_code = nullptr;
};

// wave64 butterfly reduction followed by a fixed-order pass over the waves of
// the workgroup: the result does not depend on scheduling.
template <int NT, typename real>
__device__ __forceinline__ void block_reduce_diag(double sum, real umax, real rmin, real rmax,
                                                  int cnt, double* out) {
    constexpr int NW = NT / 64;
    __shared__ double r_sum[NW], r_umax[NW], r_rmin[NW], r_rmax[NW];
    __shared__ int r_cnt[NW];
    double du = (double)umax, dmn = (double)rmin, dmx = (double)rmax;
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
        sum += __shfl_xor(sum, off, 64);
        double t = __shfl_xor(du, off, 64);
        du = t > du ? t : du;
        t = __shfl_xor(dmn, off, 64);
        dmn = t < dmn ? t : dmn;
        t = __shfl_xor(dmx, off, 64);
        dmx = t > dmx ? t : dmx;
        cnt += __shfl_xor(cnt, off, 64);
    }
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) {
        r_sum[wv] = sum;
        r_umax[wv] = du;
        r_rmin[wv] = dmn;
        r_rmax[wv] = dmx;
        r_cnt[wv] = cnt;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double s = r_sum[0], a = r_umax[0], b = r_rmin[0], c = r_rmax[0];
        int n = r_cnt[0];
        for (int i = 1; i < NW; ++i) {
            s += r_sum[i];
            a = r_umax[i] > a ? r_umax[i] : a;
            b = r_rmin[i] < b ? r_rmin[i] : b;
            c = r_rmax[i] > c ? r_rmax[i] : c;
            n += r_cnt[i];
        }
        out[0] = s;
        out[1] = a;
        out[2] = b;
        out[3] = c;
        out[4] = (double)n;
    }
}

// fused steps
// (variant: tile shape chosen by the autotuner; the field mode always uses
// variant 0)
template <typename real>
int step2d_variants();
template <typename real>
int grid2d_blocks(int nx, int ny, int variant);
template <typename real>
hipError_t launch_step2d(const Coef<real>& C, const Fields<real>& F, const FieldOut<real>& O,
                         int mode, int variant, hipStream_t s);
template <typename real>
int tile2d_variants();
template <typename real>
int tile2d_preferred_variant();
template <typename real>
void tile2d_shape(int variant, int* TX, int* TY);
template <typename real>
hipError_t launch_step2d_batch(const Coef<real>& C, const BatchArgs<real>& B, int ntiles,
                               int variant, hipStream_t s);
template <typename real>
int step2d_march_variants();
template <typename real>
hipError_t launch_step2d_march(const Coef<real>& C, const Fields<real>& F, const FieldOut<real>& O,
                               int idx, hipStream_t s);
template <typename real>
int step3d_variants();
template <typename real>
int step3d_preferred_variant(int nx, int ny, int nz);
template <typename real>
int grid3d_blocks(int nx, int ny, int nz, int variant);
template <typename real>
hipError_t launch_step3d(const Coef<real>& C, const Fields<real>& F, const FieldOut<real>& O,
                         int mode, int variant, hipStream_t s);
template <typename real>
bool step3d_forms_density(const Coef<real>& C, int variant);
template <typename real>
size_t step3d_ring_elems(int nx, int ny, int nz);
template <typename real>
hipError_t launch_density3d(const Coef<real>& C, const Fields<real>& F, hipStream_t s);

// discrete adjoint of the D2Q9 step (adjoint2d.hip)
template <typename real>
struct AdjArgs {
    const real* lam_in;  // partial lam(t+1) [9][N]
    const real* ext_in;  // density-path part of lam(t+1) [N]
    real* lam_out;       // partial lam(t) [9][N]
    real* ext_out;       // density-path part of lam(t) [N]
    real* sb;            // per node: dL/dF_m x, y, psi, rho ([4][N])
    real* grad_phi;      // per wall node (accumulated)
    real* grad_drho;
};
template <typename real>
hipError_t launch_adjoint2d(const Coef<real>& C, const Fields<real>& F, const AdjArgs<real>& A,
                            hipStream_t s);
template <typename real>
hipError_t launch_adj_seed(int kind, const uint8_t* cls, const real* seed, real* lam, real* ext,
                           uint32_t N, hipStream_t s);
template <typename real>
hipError_t launch_adj_finish(const uint8_t* cls, const real* lam, const real* ext, real* out,
                             uint32_t N, hipStream_t s);

// auxiliary kernels
// N storage nodes with rows `pitch` apart, of which the first nx of each row
// are the lattice's (rho and u dense, rows nx apart); nx = pitch = 1: plain
template <typename real>
hipError_t launch_init_eq(int lattice, const uint8_t* cls, const real* rho, const real* u,
                          real* f, int64_t N, hipStream_t s, int nx = 1, int pitch = 1);
template <typename real>
hipError_t launch_mask_solid(int Q, const uint8_t* cls, real* f, int64_t N, hipStream_t s);
// D3Q19 pull form: post-stream f -> pull form (dst cleared first), and back
template <typename real>
hipError_t launch_scatter3(const uint8_t* cls, const real* f, real* dst, int nx, int ny, int nz,
                           hipStream_t s);
template <typename real>
hipError_t launch_gather3(const uint8_t* cls, const real* src, real* f, int nx, int ny, int nz,
                          hipStream_t s);
template <typename real>
hipError_t launch_fill(real* p, real v, int64_t n, hipStream_t s);
hipError_t launch_fill_i32(int32_t* p, int32_t v, int64_t n, hipStream_t s);
hipError_t launch_gather_code(const int32_t* widx, const int32_t* code, int32_t* out, int64_t n,
                              hipStream_t s);
template <typename real>
hipError_t launch_gather_wall(const int32_t* widx, const real* phi, const real* drho, real* ophi,
                              real* odrho, int64_t n, hipStream_t s);
hipError_t launch_diag_final(const double* part, int nparts, double* out, hipStream_t s);

}  // namespace lbm
