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
enum { WET_IVD = 0, WET_VD = 1, WET_SFI = 2, WET_GF = 3 };
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
    // relaxation group of each row (GRP_* below)
    static constexpr int grp[9] = {0, 1, 2, 3, 4, 3, 4, 5, 5};
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
    static constexpr int grp[19] = {0, 1, 2, 3, 4, 3, 4, 3, 4, 5, 6, 5, 6, 5, 5, 5, 7, 7, 7};
};

// Moment groups that share one relaxation rate (isotropy): density, energy,
// energy square, momentum, energy flux, viscous stress, its 4th-order
// companion (3-D), and the 3rd-order moments m_x,y,z (3-D).
enum { GRP_RHO = 0, GRP_E, GRP_EPS, GRP_J, GRP_Q, GRP_NU, GRP_PI, GRP_M, NGRP };

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
    real s[NGRP];   // 1/tau per moment group
    real sig_e;     // 12 sigma / (tau_e - 1/2)  (3-D: 114 sigma / (tau_e - 1/2))
    real sig_eps;   // 12 sigma / (tau_eps - 1/2) (3-D: 0)
    real body[3];
    int pitch = 0;  // D2Q9: nodes from one row to the next in the arrays (0: nx)
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
    real* rho = nullptr;   // density of every node (0 off the fluid), written by
                           // the density pass that precedes a sweep step
    // D3Q19 sweeps that also form the next step's density: rho already holds
    // the density of fin (no density pass needed), rho_next receives that of
    // fout, ring the per-block partial sums for the nodes around each block
    bool rho_valid = false;
    real* rho_next = nullptr;
    real* ring = nullptr;
    // Per-tile wall lists of the D2Q9 tile step (improved virtual density):
    // tile t owns entries [t * tw_stride, (t + 1) * tw_stride); each entry
    // packs (wall count of the tile << 16) | LDS position of one wall node
    // of the tile plus its 1-node ring (0xFFFF past the count), with that
    // wall's phi and drho beside it.  tw_pack == nullptr: no lists.
    const int32_t* tw_pack = nullptr;
    const real* tw_phi = nullptr;
    const real* tw_drho = nullptr;
    int tw_stride = 0;
    // geometric formulation: stencil code per wall node (phi, drho then hold
    // the two interpolation weights) and per wall-list entry
    const int32_t* gfcode = nullptr;
    const int32_t* tw_code = nullptr;
};

// Workgroups are handed to the 8 XCDs of the chip round-robin by linear id.
// Remapping the id so that XCD x receives one contiguous range of tiles
// keeps the halo re-reads and the streaming writes that cross a tile edge
// inside one L2.  Bijective for any nb.
__device__ __forceinline__ int remap_xcd(int b, int nb) {
    constexpr int NXCD = 8;
    const int q = nb / NXCD, r = nb % NXCD;
    const int x = b % NXCD, k = b / NXCD;
    return (x < r) ? x * (q + 1) + k : r * (q + 1) + (x - r) * q + k;
}

// Population arrays are addressed through a buffer resource when the whole
// array is below 4 GiB: every direction of a node uses the same 32-bit
// per-lane byte offset (the node) and a scalar offset a*N*sizeof(real) (the
// direction), which is how CDNA addresses many arrays that share one index
// without a 64-bit address per access.  The resource's range check makes an
// out-of-range access read 0 and drop the write.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t make_rsrc(const void* p, uint32_t nbytes) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(p), (short)0, (int)nbytes,
                                             0x00020000);
}

template <typename real>
__device__ __forceinline__ real buf_ld(__amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff) {
    if constexpr (sizeof(real) == 4)
        return __builtin_bit_cast(real, __builtin_amdgcn_raw_buffer_load_b32(r, (int)voff, (int)soff, 0));
    else
        return __builtin_bit_cast(real, __builtin_amdgcn_raw_buffer_load_b64(r, (int)voff, (int)soff, 0));
}

// AUX is the cache policy of the store: 0 normal, ST_NT non-temporal (the
// gfx950 "nt" bit: the line is not kept in the caches for reuse).
constexpr int ST_NT = 2;
template <typename real, int AUX = 0>
__device__ __forceinline__ void buf_st(real v, __amdgpu_buffer_rsrc_t r, uint32_t voff,
                                       uint32_t soff) {
    if constexpr (sizeof(real) == 4)
        __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(uint32_t, v), r, (int)voff, (int)soff, AUX);
    else
    {
        typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));
        __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, v), r, (int)voff, (int)soff, AUX);
    }
}

// Read / write population a of node n (element index), through the buffer
// resource (BUF) or plain 64-bit addressing.
template <typename real, bool BUF>
struct PopIO {
    const real* fin;
    real* fout;
    uint32_t N;  // nodes
    __amdgpu_buffer_rsrc_t rin, rout;
    __device__ __forceinline__ PopIO(const real* i, real* o, uint32_t n, int Q) : fin(i), fout(o), N(n) {
        if constexpr (BUF) {
            const uint32_t bytes = (uint32_t)((uint64_t)Q * n * sizeof(real));
            rin = make_rsrc(i, bytes);
            rout = make_rsrc(o, bytes);
        }
    }
    __device__ __forceinline__ real ld(int a, uint32_t n) const {
        if constexpr (BUF) return buf_ld<real>(rin, n * (uint32_t)sizeof(real), (uint32_t)a * N * (uint32_t)sizeof(real));
        else return fin[(size_t)a * N + n];
    }
    __device__ __forceinline__ void st(int a, uint32_t n, real v) const {
        if constexpr (BUF) buf_st<real>(v, rout, n * (uint32_t)sizeof(real), (uint32_t)a * N * (uint32_t)sizeof(real));
        else fout[(size_t)a * N + n] = v;
    }
    // the same with a non-temporal store: for stores that fill whole cache
    // lines of one workgroup (the pull form's own slots).  Partly written
    // lines, as in a push, must merge in L2 and are slower this way.
    __device__ __forceinline__ void st_nt(int a, uint32_t n, real v) const {
        if constexpr (BUF)
            buf_st<real, ST_NT>(v, rout, n * (uint32_t)sizeof(real), (uint32_t)a * N * (uint32_t)sizeof(real));
        else __builtin_nontemporal_store(v, &fout[(size_t)a * N + n]);
    }
    // push with halfway bounce-back in one store: to slot a of node
    // n + delta if `stream`, else to slot b of node n (delta uniform across
    // the wavefront).  The smaller of the two slot offsets goes into the
    // scalar offset and the per-lane offset selects the rest, so a
    // wavefront with both kinds of lanes issues one store, not two.
    // Needs n + delta >= 0.
    template <int AUX = 0>
    __device__ __forceinline__ void st_push(bool stream, int a, int b, int delta, uint32_t n,
                                            real v) const {
        const int lo = a < b ? a : b;
        if constexpr (BUF) {
            const uint32_t ds = (uint32_t)((int)((a - lo) * N) + delta);
            const uint32_t db = (uint32_t)(b - lo) * N;
            buf_st<real, AUX>(v, rout, (n + (stream ? ds : db)) * (uint32_t)sizeof(real),
                              (uint32_t)lo * N * (uint32_t)sizeof(real));
        } else {
            fout[stream ? (int64_t)a * N + n + delta : (int64_t)b * N + n] = v;
        }
    }
    // the same with the streaming target given as a node (m), where it is
    // not at one offset across the wavefront (a tile whose neighbours wrap)
    template <int AUX = 0>
    __device__ __forceinline__ void st_sel(bool stream, int a, int b, uint32_t m, uint32_t n,
                                           real v) const {
        const int lo = a < b ? a : b;
        if constexpr (BUF) {
            const uint32_t e = stream ? (uint32_t)(a - lo) * N + m : (uint32_t)(b - lo) * N + n;
            buf_st<real, AUX>(v, rout, e * (uint32_t)sizeof(real),
                              (uint32_t)lo * N * (uint32_t)sizeof(real));
        } else {
            fout[stream ? (int64_t)a * N + m : (int64_t)b * N + n] = v;
        }
    }
    // store to node n + delta of direction a, delta uniform across the
    // wavefront: the shift goes into the scalar offset, so every direction
    // shares the per-lane offset of n.  Needs a * N + delta >= 0.
    __device__ __forceinline__ void st_shift(int a, int delta, uint32_t n, real v) const {
        if constexpr (BUF)
            buf_st<real>(v, rout, n * (uint32_t)sizeof(real),
                         (uint32_t)((int)(a * N) + delta) * (uint32_t)sizeof(real));
        else fout[(int64_t)a * N + n + delta] = v;
    }
};

// Four consecutive nodes n .. n+3 of FP32 direction a in one 16-byte
// buffer access (n a multiple of 4: the rows of a lattice whose width is a
// multiple of 4 start on 16-byte boundaries).  The partial store writes
// three consecutive nodes (12 bytes, 4-byte aligned).
// (The whole vector is bit-cast to floats before its elements are taken:
// a bit-cast of one element of an integer vector reads element 0.)
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
typedef unsigned int u32x3 __attribute__((ext_vector_type(3)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
__device__ __forceinline__ void ld_quad(const PopIO<float, true>& io, int a, uint32_t n,
                                        float& v0, float& v1, float& v2, float& v3) {
    const f32x4 r = __builtin_bit_cast(
        f32x4, __builtin_amdgcn_raw_buffer_load_b128(io.rin, (int)(n * 4u), (int)(a * io.N * 4u), 0));
    v0 = r.x;
    v1 = r.y;
    v2 = r.z;
    v3 = r.w;
}
template <int AUX = 0>
__device__ __forceinline__ void st_quad(const PopIO<float, true>& io, int a, uint32_t n, float v0,
                                        float v1, float v2, float v3) {
    const u32x4 w = {__builtin_bit_cast(unsigned, v0), __builtin_bit_cast(unsigned, v1),
                     __builtin_bit_cast(unsigned, v2), __builtin_bit_cast(unsigned, v3)};
    __builtin_amdgcn_raw_buffer_store_b128(w, io.rout, (int)(n * 4u), (int)(a * io.N * 4u), AUX);
}
__device__ __forceinline__ void st_triple(const PopIO<float, true>& io, int a, uint32_t n, float v0,
                                          float v1, float v2) {
    const u32x3 w = {__builtin_bit_cast(unsigned, v0), __builtin_bit_cast(unsigned, v1),
                     __builtin_bit_cast(unsigned, v2)};
    __builtin_amdgcn_raw_buffer_store_b96(w, io.rout, (int)(n * 4u), (int)(a * io.N * 4u), 0);
}

__device__ __forceinline__ int wrapi(int v, int n) {
    // any integer into [0, n); tiles may cover the lattice several times
    v %= n;
    return v < 0 ? v + n : v;
}

// a / b: IEEE division in FP64; in FP32 a times the hardware reciprocal
// (v_rcp_f32, 1 ulp), which is well inside the FP32 error budget of a step.
template <typename real>
__device__ __forceinline__ real fdiv(real a, real b) {
    if constexpr (sizeof(real) == 4) return a * __builtin_amdgcn_rcpf(b);
    else return a / b;
}

// ---------------------------------------------------- equation of state
template <typename real>
__device__ __forceinline__ real eos_p(const Coef<real>& C, real rho) {
    if (C.eos == EOS_CS) {
        real h = C.eos_b * real(0.25) * rho;
        real om = real(1) - h;
        real num = real(1) + h + h * h - h * h * h;
        return fdiv(rho * C.eos_RT * num, om * om * om) - C.eos_a * rho * rho;
    } else {
        real br = C.eos_b * rho;
        return fdiv(rho * C.eos_RT, real(1) - br) -
               fdiv(C.eos_aphi * rho * rho, real(1) + real(2) * br - br * br);
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
// Equilibrium moments m_eq = M f_eq of the second-order equilibrium, row k.
// D2Q9: rho (1, -2 + 3u^2, 1 - 3u^2, ux, -ux, uy, -uy, ux^2 - uy^2, ux uy).
// D3Q19: e_eq = rho(-11 + 19 u^2), eps_eq = rho(3 - 5.5 u^2), q_eq =
// -2/3 j, 3p_xx = rho(2ux^2 - uy^2 - uz^2), p_ww = rho(uy^2 - uz^2),
// pi rows = -1/2 of their p rows, 3rd-order rows 0.
template <typename L, typename real>
__device__ __forceinline__ real meq_row(int k, real rho, const real* u, real u2) {
    if constexpr (L::Q == 9) {
        switch (k) {
        case 1: return rho * (real(-2) + real(3) * u2);
        case 2: return rho * (real(1) - real(3) * u2);
        case 4: return -rho * u[0];
        case 6: return -rho * u[1];
        case 7: return rho * (u[0] * u[0] - u[1] * u[1]);
        default: return rho * u[0] * u[1];  // k == 8
        }
    } else {
        switch (k) {
        case 1: return rho * (real(-11) + real(19) * u2);
        case 2: return rho * (real(3) - real(5.5) * u2);
        case 4: return real(-2.0 / 3.0) * rho * u[0];
        case 6: return real(-2.0 / 3.0) * rho * u[1];
        case 8: return real(-2.0 / 3.0) * rho * u[2];
        case 9: return rho * (real(2) * u[0] * u[0] - u[1] * u[1] - u[2] * u[2]);
        case 10: return real(-0.5) * rho * (real(2) * u[0] * u[0] - u[1] * u[1] - u[2] * u[2]);
        case 11: return rho * (u[1] * u[1] - u[2] * u[2]);
        case 12: return real(-0.5) * rho * (u[1] * u[1] - u[2] * u[2]);
        case 13: return rho * u[0] * u[1];
        case 14: return rho * u[1] * u[2];
        case 15: return rho * u[0] * u[2];
        default: return real(0);  // 16, 17, 18
        }
    }
}

// Moment-space forcing, row k.  D2Q9: Eq. 7, with the thermodynamic-
// consistency term sig = |F_m|^2 / psi^2 on the e and eps rows.  D3Q19:
// M G of the Guo discrete force plus the same pressure shift on the e row.
template <typename L, typename real>
__device__ __forceinline__ real src_row(const Coef<real>& C, int k, const real* u, const real* F,
                                        real uF, real sgm) {
    if constexpr (L::Q == 9) {
        switch (k) {
        case 1: return real(6) * uF + C.sig_e * sgm;
        case 2: return real(-6) * uF - C.sig_eps * sgm;
        case 4: return -F[0];
        case 6: return -F[1];
        case 7: return real(2) * (u[0] * F[0] - u[1] * F[1]);
        default: return u[0] * F[1] + u[1] * F[0];  // k == 8
        }
    } else {
        switch (k) {
        case 1: return real(38) * uF + C.sig_e * sgm;
        case 2: return real(-11) * uF;
        case 4: return real(-2.0 / 3.0) * F[0];
        case 6: return real(-2.0 / 3.0) * F[1];
        case 8: return real(-2.0 / 3.0) * F[2];
        case 9: return real(2) * (real(2) * u[0] * F[0] - u[1] * F[1] - u[2] * F[2]);
        case 10: return -(real(2) * u[0] * F[0] - u[1] * F[1] - u[2] * F[2]);
        case 11: return real(2) * (u[1] * F[1] - u[2] * F[2]);
        case 12: return -(u[1] * F[1] - u[2] * F[2]);
        case 13: return u[0] * F[1] + u[1] * F[0];
        case 14: return u[1] * F[2] + u[2] * F[1];
        case 15: return u[0] * F[2] + u[2] * F[0];
        default: return real(0);
        }
    }
}

// FP32 D2Q9 collision.  Same m = M f, relaxation and M^-1 as the row-by-row
// form below, with two changes that matter in single precision:
//  * the Lallemand-Luo rows are factored into shared partial sums (axis
//    pairs, diagonal pairs), about a third of the arithmetic;
//  * the result is formed as an increment, f* = f + M^-1 (m* - m).  The
//    increment vanishes at equilibrium and its entries sum to zero up to
//    rounding of the (small) increment, so a resting bulk region does not
//    re-round its populations every step.  Re-forming f* from m* instead
//    repeats the same rounding error at every node of a uniform region each
//    step, which shows up as a steady FP32 mass drift.
// One reciprocal of rho serves both velocity components.
__device__ __forceinline__ void collide_d2q9_f32(const Coef<float>& C, const float* f, float rho,
                                                 const float* F, const float* Fm, float psi,
                                                 float* fs, float* u_out) {
    const float A = f[1] + f[3], B = f[2] + f[4];
    const float p57 = f[5] + f[7], p68 = f[6] + f[8];
    const float d13 = f[1] - f[3], d24 = f[2] - f[4];
    const float u57 = f[5] - f[7], v68 = f[6] - f[8];
    const float AB = A + B, Dg = p57 + p68;
    const float Ex = u57 - v68, Ey = u57 + v68;
    const float m_e = 2.0f * Dg - AB - 4.0f * f[0];
    const float m_eps = Dg - 2.0f * AB + 4.0f * f[0];
    const float jx = d13 + Ex, jy = d24 + Ey;
    const float m_qx = Ex - 2.0f * d13, m_qy = Ey - 2.0f * d24;
    const float m_pxx = A - B, m_pxy = p57 - p68;

    const float inv = __builtin_amdgcn_rcpf(rho);
    const float ux = (jx + 0.5f * F[0]) * inv, uy = (jy + 0.5f * F[1]) * inv;
    u_out[0] = ux;
    u_out[1] = uy;
    const float uF = ux * F[0] + uy * F[1];
    const float u2 = ux * ux + uy * uy;
    const float fm2 = Fm[0] * Fm[0] + Fm[1] * Fm[1];
    const float sgm = (psi > 0.0f) ? fdiv(fm2, psi * psi) : 0.0f;

    const float se = C.s[GRP_E], sp = C.s[GRP_EPS], sq = C.s[GRP_Q], sn = C.s[GRP_NU];
    // m* - m = s (m_eq - m) + (1 - s/2) Src per row (Eq. 2, Eq. 7); the
    // density row does not change and the momentum rows change by F
    const float de = se * (rho * (3.0f * u2 - 2.0f) - m_e) +
                     (1.0f - 0.5f * se) * (6.0f * uF + C.sig_e * sgm);
    const float dp = sp * (rho * (1.0f - 3.0f * u2) - m_eps) -
                     (1.0f - 0.5f * sp) * (6.0f * uF + C.sig_eps * sgm);
    const float dqx = -sq * (rho * ux + m_qx) - (1.0f - 0.5f * sq) * F[0];
    const float dqy = -sq * (rho * uy + m_qy) - (1.0f - 0.5f * sq) * F[1];
    const float dxx = sn * (rho * (ux * ux - uy * uy) - m_pxx) +
                      (1.0f - 0.5f * sn) * 2.0f * (ux * F[0] - uy * F[1]);
    const float dxy = sn * (rho * ux * uy - m_pxy) + (1.0f - 0.5f * sn) * (ux * F[1] + uy * F[0]);

    // f* - f = M^T diag(1/norm) (m* - m)
    const float e1 = de * (1.0f / 36.0f), p1 = dp * (1.0f / 36.0f);
    const float jx1 = F[0] * (1.0f / 6.0f), jy1 = F[1] * (1.0f / 6.0f);
    const float qx1 = dqx * (1.0f / 12.0f), qy1 = dqy * (1.0f / 12.0f);
    const float xx1 = dxx * 0.25f, xy1 = dxy * 0.25f;
    fs[0] = f[0] + (4.0f * (p1 - e1));
    const float ca = -e1 - 2.0f * p1;
    const float X = jx1 - 2.0f * qx1, Y = jy1 - 2.0f * qy1;
    fs[1] = f[1] + ((ca + xx1) + X);
    fs[3] = f[3] + ((ca + xx1) - X);
    fs[2] = f[2] + ((ca - xx1) + Y);
    fs[4] = f[4] + ((ca - xx1) - Y);
    const float cd = 2.0f * e1 + p1;
    const float Px = jx1 + qx1, Py = jy1 + qy1;
    fs[5] = f[5] + ((cd + xy1) + (Px + Py));
    fs[7] = f[7] + ((cd + xy1) - (Px + Py));
    fs[6] = f[6] + ((cd - xy1) + (Py - Px));
    fs[8] = f[8] + ((cd - xy1) - (Py - Px));
}

// FP32 D3Q19 collision: the d'Humieres rows factored into sums and
// differences of opposite-velocity pairs (axis pairs; xy, xz and yz
// face-diagonal pairs), the increment form f* = f + M^-1 (m* - m), and one
// reciprocal of rho; same m = M f, relaxation (grouped rates), forcing
// (M G of the Guo force plus the sigma term on the energy row) and
// M^-1 = M^T diag(1/norm) as the row-by-row form below.
__device__ __forceinline__ void collide_d3q19_f32(const Coef<float>& C, const float* f, float rho,
                                                  const float* F, const float* Fm, float psi,
                                                  float* fs, float* u_out) {
    const float sx = f[1] + f[2], dx = f[1] - f[2];
    const float sy = f[3] + f[4], dy = f[3] - f[4];
    const float sz = f[5] + f[6], dz = f[5] - f[6];
    const float s78 = f[7] + f[8], d78 = f[7] - f[8];
    const float s910 = f[9] + f[10], d910 = f[9] - f[10];
    const float s1112 = f[11] + f[12], d1112 = f[11] - f[12];
    const float s1314 = f[13] + f[14], d1314 = f[13] - f[14];
    const float s1516 = f[15] + f[16], d1516 = f[15] - f[16];
    const float s1718 = f[17] + f[18], d1718 = f[17] - f[18];
    const float Sxy = s78 + s910, Sxz = s1112 + s1314, Syz = s1516 + s1718;
    const float Sax = sx + sy + sz, Sdg = Sxy + Sxz + Syz;
    const float m_e = 8.0f * Sdg - 11.0f * Sax - 30.0f * f[0];
    const float m_eps = Sdg - 4.0f * Sax + 12.0f * f[0];
    const float Dx = (d78 + d910) + (d1112 + d1314);
    const float Dy = (d78 - d910) + (d1516 + d1718);
    const float Dz = (d1112 - d1314) + (d1516 - d1718);
    const float jx = dx + Dx, jy = dy + Dy, jz = dz + Dz;
    const float qx = Dx - 4.0f * dx, qy = Dy - 4.0f * dy, qz = Dz - 4.0f * dz;
    const float A9 = Sxy + Sxz - 2.0f * Syz;
    const float p9 = (2.0f * sx - sy - sz) + A9, p10 = (2.0f * (sy + sz) - 4.0f * sx) + A9;
    const float B11 = Sxy - Sxz;
    const float p11 = (sy - sz) + B11, p12 = 2.0f * (sz - sy) + B11;
    const float pxy = s78 - s910, pyz = s1516 - s1718, pxz = s1112 - s1314;
    const float mx = (d78 + d910) - (d1112 + d1314);
    const float my = (d910 - d78) + (d1516 + d1718);
    const float mz = (d1112 - d1314) - (d1516 - d1718);

    const float inv = __builtin_amdgcn_rcpf(rho);
    const float ux = (jx + 0.5f * F[0]) * inv, uy = (jy + 0.5f * F[1]) * inv;
    const float uz = (jz + 0.5f * F[2]) * inv;
    u_out[0] = ux;
    u_out[1] = uy;
    u_out[2] = uz;
    const float uF = ux * F[0] + uy * F[1] + uz * F[2];
    const float u2 = ux * ux + uy * uy + uz * uz;
    const float fm2 = Fm[0] * Fm[0] + Fm[1] * Fm[1] + Fm[2] * Fm[2];
    const float sgm = (psi > 0.0f) ? fdiv(fm2, psi * psi) : 0.0f;

    const float se = C.s[GRP_E], sp = C.s[GRP_EPS], sq = C.s[GRP_Q];
    const float sn = C.s[GRP_NU], spi = C.s[GRP_PI], sm = C.s[GRP_M];
    const float hq = 1.0f - 0.5f * sq, hn = 1.0f - 0.5f * sn, hp = 1.0f - 0.5f * spi;
    // m* - m = s (m_eq - m) + (1 - s/2) Src per row
    const float de = se * (rho * (19.0f * u2 - 11.0f) - m_e) +
                     (1.0f - 0.5f * se) * (38.0f * uF + C.sig_e * sgm);
    const float dp = sp * (rho * (3.0f - 5.5f * u2) - m_eps) - (1.0f - 0.5f * sp) * (11.0f * uF);
    const float t23 = 2.0f / 3.0f;
    const float dqx = -sq * (t23 * rho * ux + qx) - hq * (t23 * F[0]);
    const float dqy = -sq * (t23 * rho * uy + qy) - hq * (t23 * F[1]);
    const float dqz = -sq * (t23 * rho * uz + qz) - hq * (t23 * F[2]);
    const float T9 = 2.0f * ux * ux - uy * uy - uz * uz;
    const float G9 = 2.0f * ux * F[0] - uy * F[1] - uz * F[2];
    const float T11 = uy * uy - uz * uz, G11 = uy * F[1] - uz * F[2];
    const float d9 = sn * (rho * T9 - p9) + hn * 2.0f * G9;
    const float d10 = spi * (-0.5f * rho * T9 - p10) - hp * G9;
    const float d11 = sn * (rho * T11 - p11) + hn * 2.0f * G11;
    const float d12 = spi * (-0.5f * rho * T11 - p12) - hp * G11;
    const float dxy = sn * (rho * ux * uy - pxy) + hn * (ux * F[1] + uy * F[0]);
    const float dyz = sn * (rho * uy * uz - pyz) + hn * (uy * F[2] + uz * F[1]);
    const float dxz = sn * (rho * ux * uz - pxz) + hn * (ux * F[2] + uz * F[0]);

    // f* - f = M^T diag(1/norm) (m* - m)
    const float E = de * (1.0f / 2394.0f), P = dp * (1.0f / 252.0f);
    const float JX = F[0] * 0.1f, JY = F[1] * 0.1f, JZ = F[2] * 0.1f;
    const float QX = dqx * (1.0f / 40.0f), QY = dqy * (1.0f / 40.0f), QZ = dqz * (1.0f / 40.0f);
    const float X9 = d9 * (1.0f / 36.0f), X10 = d10 * (1.0f / 72.0f);
    const float W11 = d11 * (1.0f / 12.0f), W12 = d12 * (1.0f / 24.0f);
    const float Pxy = dxy * 0.25f, Pyz = dyz * 0.25f, Pxz = dxz * 0.25f;
    const float Mx = -sm * mx * 0.125f, My = -sm * my * 0.125f, Mz = -sm * mz * 0.125f;
    fs[0] = f[0] + (12.0f * P - 30.0f * E);
    const float ba = -11.0f * E - 4.0f * P;
    const float c9 = 2.0f * X9 - 4.0f * X10, c9h = 2.0f * X10 - X9;
    const float ax = JX - 4.0f * QX, ay = JY - 4.0f * QY, az = JZ - 4.0f * QZ;
    const float wyz = W11 - 2.0f * W12;
    fs[1] = f[1] + ((ba + c9) + ax);
    fs[2] = f[2] + ((ba + c9) - ax);
    fs[3] = f[3] + ((ba + c9h + wyz) + ay);
    fs[4] = f[4] + ((ba + c9h + wyz) - ay);
    fs[5] = f[5] + ((ba + c9h - wyz) + az);
    fs[6] = f[6] + ((ba + c9h - wyz) - az);
    const float bd = 8.0f * E + P, X = X9 + X10, Wt = W11 + W12;
    const float Lx = JX + QX, Ly = JY + QY, Lz = JZ + QZ;
    const float bxy = bd + X + Wt, bxz = bd + X - Wt, byz = bd - 2.0f * X;
    fs[7] = f[7] + ((bxy + Pxy) + ((Lx + Ly) + (Mx - My)));
    fs[8] = f[8] + ((bxy + Pxy) - ((Lx + Ly) + (Mx - My)));
    fs[9] = f[9] + ((bxy - Pxy) + ((Lx - Ly) + (Mx + My)));
    fs[10] = f[10] + ((bxy - Pxy) - ((Lx - Ly) + (Mx + My)));
    fs[11] = f[11] + ((bxz + Pxz) + ((Lx + Lz) + (Mz - Mx)));
    fs[12] = f[12] + ((bxz + Pxz) - ((Lx + Lz) + (Mz - Mx)));
    fs[13] = f[13] + ((bxz - Pxz) + ((Lx - Lz) - (Mx + Mz)));
    fs[14] = f[14] + ((bxz - Pxz) - ((Lx - Lz) - (Mx + Mz)));
    fs[15] = f[15] + ((byz + Pyz) + ((Ly + Lz) + (My - Mz)));
    fs[16] = f[16] + ((byz + Pyz) - ((Ly + Lz) + (My - Mz)));
    fs[17] = f[17] + ((byz - Pyz) + ((Ly - Lz) + (My + Mz)));
    fs[18] = f[18] + ((byz - Pyz) - ((Ly - Lz) + (My + Mz)));
}

// Post-collision populations of one fluid node (Eq. 2, forcing of Eq. 7):
// m = M f, m* = m - S (m - m_eq) + (I - S/2) Src, f* = M^-1 m*.
// in: f (populations), rho, F (total force), Fm (cohesive force of Eq. 5),
// psi (own pseudopotential).  out: fs and u.  Each row's m_eq and source
// are formed when the row is relaxed, which keeps few values live.
template <typename L, typename real>
__device__ __forceinline__ void collide(const Coef<real>& C, const real* f, real rho,
                                        const real* F, const real* Fm, real psi,
                                        real* fs, real* u_out) {
    if constexpr (L::Q == 9 && sizeof(real) == 4) {
        collide_d2q9_f32(C, f, rho, F, Fm, psi, fs, u_out);
        return;
    }
    if constexpr (L::Q == 19 && sizeof(real) == 4) {
        collide_d3q19_f32(C, f, rho, F, Fm, psi, fs, u_out);
        return;
    }
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
    real u[3], Fv[3];
    Fv[0] = F[0];
    Fv[1] = F[1];
    Fv[2] = (L::D == 3) ? F[2] : real(0);
    u[0] = (m[3] + real(0.5) * Fv[0]) / rho;
    u[1] = (m[5] + real(0.5) * Fv[1]) / rho;
    u[2] = (L::D == 3) ? (m[7] + real(0.5) * Fv[2]) / rho : real(0);
    u_out[0] = u[0];
    u_out[1] = u[1];
    if (L::D == 3) u_out[2] = u[2];
    const real uF = u[0] * Fv[0] + u[1] * Fv[1] + u[2] * Fv[2];
    const real u2 = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
    real fm2 = Fm[0] * Fm[0] + Fm[1] * Fm[1];
    if (L::D == 3) fm2 += Fm[2] * Fm[2];
    const real sgm = (psi > real(0)) ? fm2 / (psi * psi) : real(0);
    // Conserved rows: density keeps its value (S_0 = 0, m_eq = rho) and the
    // momentum rows give j + F for any relaxation rate, since
    // j - j_eq = -F/2.  All other rows relax with their group's rate.
    // FP32 forms the increment f* - f = M^-1 (m* - m) (it vanishes at
    // equilibrium, so a resting region does not re-round its populations
    // every step); FP64 forms f* = M^-1 m* in the order of Eq. 2.
    constexpr bool INC = sizeof(real) == 4;
#pragma unroll
    for (int k = 0; k < Q; ++k) {
        real mk;
        if (k == 0) mk = INC ? real(0) : m[0];
        else if (k == 3) mk = INC ? Fv[0] : m[3] + Fv[0];
        else if (k == 5) mk = INC ? Fv[1] : m[5] + Fv[1];
        else if (L::D == 3 && k == 7) mk = INC ? Fv[2] : m[7] + Fv[2];
        else {
            const real sk = C.s[L::grp[k]];
            const real me = meq_row<L, real>(k, rho, u, u2);
            const real sr = src_row<L, real>(C, k, u, Fv, uF, sgm);
            mk = INC ? sk * (me - m[k]) + (real(1) - real(0.5) * sk) * sr
                     : m[k] - sk * (m[k] - me) + (real(1) - real(0.5) * sk) * sr;
        }
        m[k] = mk * real(1.0 / L::norm[k]);
    }
#pragma unroll
    for (int a = 0; a < Q; ++a) {
        real s = real(0);
        bool first = true;
#pragma unroll
        for (int k = 0; k < Q; ++k) {
            if (L::M[k][a] == 0) continue;
            if (INC && k == 0) continue;  // the density row does not change
            real term = (L::M[k][a] == 1) ? m[k] : (L::M[k][a] == -1) ? -m[k] : real(L::M[k][a]) * m[k];
            s = first ? term : s + term;
            first = false;
        }
        fs[a] = INC ? f[a] + s : s;
    }
}

// dp/drho of the equation of state
template <typename real>
__device__ __forceinline__ real eos_dp(const Coef<real>& C, real rho) {
    if (C.eos == EOS_CS) {
        // d(rho Z)/drho of Carnahan-Starling = (1 + 4h + 4h^2 - 4h^3 + h^4) / (1 - h)^4
        const real h = C.eos_b * real(0.25) * rho;
        const real om = real(1) - h;
        const real om2 = om * om;
        const real num = real(1) + real(4) * h + real(4) * h * h - real(4) * h * h * h + h * h * h * h;
        return C.eos_RT * num / (om2 * om2) - real(2) * C.eos_a * rho;
    } else {
        const real br = C.eos_b * rho;
        const real om = real(1) - br;
        const real D = real(1) + real(2) * br - br * br;
        const real Dp = real(2) * C.eos_b - real(2) * C.eos_b * br;
        return C.eos_RT / (om * om) - C.eos_aphi * (real(2) * rho * D - rho * rho * Dp) / (D * D);
    }
}

// dpsi/drho for psi = sqrt(2 (p - rho/3) / G) (Eq. 6); 0 where psi = 0
template <typename real>
__device__ __forceinline__ real dpsi_drho(const Coef<real>& C, real rho, real psi) {
    if (!(psi > real(0))) return real(0);
    return C.two_over_G * (eos_dp(C, rho) - real(1.0 / 3.0)) / (real(2) * psi);
}

// Vector-Jacobian product of the collision of one fluid node (D2Q9), the
// transpose of collide(): given lam = d L / d f* (post-collision), returns
// gf = d L / d f through the moments, and the adjoints of the node's
// density (rho_bar, all explicit paths: m_eq, u), total force (F_bar) and
// of the cohesive force and own psi that enter Eq. 7's sigma term.
template <typename real>
__device__ __forceinline__ void collide_vjp_d2q9(const Coef<real>& C, const real* f, real rho,
                                                 const real* F, const real* Fm, real psi,
                                                 const real* lam, real* gf, real& rho_bar,
                                                 real* F_bar, real* Fm_bar, real& psi_bar) {
    using L = D2Q9;
    constexpr int Q = 9;
    // moments and velocity (forward)
    real m[Q];
#pragma unroll
    for (int k = 0; k < Q; ++k) {
        real s = real(0);
#pragma unroll
        for (int a = 0; a < Q; ++a)
            if (L::M[k][a] != 0) s += real(L::M[k][a]) * f[a];
        m[k] = s;
    }
    const real ux = (m[3] + real(0.5) * F[0]) / rho;
    const real uy = (m[5] + real(0.5) * F[1]) / rho;
    const real u2 = ux * ux + uy * uy;
    // mu_k = d L / d m*_k = (1/norm_k) sum_a M_ka lam_a
    real mu[Q];
#pragma unroll
    for (int k = 0; k < Q; ++k) {
        real s = real(0);
#pragma unroll
        for (int a = 0; a < Q; ++a)
            if (L::M[k][a] != 0) s += real(L::M[k][a]) * lam[a];
        mu[k] = s * real(1.0 / L::norm[k]);
    }
    real sk[Q], hk[Q];
#pragma unroll
    for (int k = 0; k < Q; ++k) {
        sk[k] = C.s[L::grp[k]];
        hk[k] = real(1) - real(0.5) * sk[k];
    }
    // m* = m - s (m - m_eq(rho, u)) + h S(u, F, Fm, psi)
    // d m_eq / d rho (at fixed u) and d m_eq / d u
    const real dmr[Q] = {real(1), real(-2) + real(3) * u2, real(1) - real(3) * u2, ux, -ux, uy, -uy,
                         ux * ux - uy * uy, ux * uy};
    real ubx = real(0), uby = real(0), rb = real(0);
#pragma unroll
    for (int k = 0; k < Q; ++k) rb += mu[k] * sk[k] * dmr[k];
    // d m_eq/du: k=1: 6 rho u, k=2: -6 rho u, k=3: (rho,0), k=4: (-rho,0), k=5: (0,rho),
    // k=6: (0,-rho), k=7: 2 rho (ux, -uy), k=8: rho (uy, ux)
    const real e1 = mu[1] * sk[1] * real(6) * rho - mu[2] * sk[2] * real(6) * rho;
    ubx += e1 * ux + (mu[3] * sk[3] - mu[4] * sk[4]) * rho + mu[7] * sk[7] * real(2) * rho * ux +
           mu[8] * sk[8] * rho * uy;
    uby += e1 * uy + (mu[5] * sk[5] - mu[6] * sk[6]) * rho - mu[7] * sk[7] * real(2) * rho * uy +
           mu[8] * sk[8] * rho * ux;
    // source rows (Eq. 7): S1 = 6 u.F + ce sig, S2 = -6 u.F - ceps sig, S3 = Fx, S4 = -Fx,
    // S5 = Fy, S6 = -Fy, S7 = 2 (ux Fx - uy Fy), S8 = ux Fy + uy Fx
    const real a1 = mu[1] * hk[1] * real(6) - mu[2] * hk[2] * real(6);
    ubx += a1 * F[0] + mu[7] * hk[7] * real(2) * F[0] + mu[8] * hk[8] * F[1];
    uby += a1 * F[1] - mu[7] * hk[7] * real(2) * F[1] + mu[8] * hk[8] * F[0];
    real Fbx = a1 * ux + mu[3] * hk[3] - mu[4] * hk[4] + mu[7] * hk[7] * real(2) * ux + mu[8] * hk[8] * uy;
    real Fby = a1 * uy + mu[5] * hk[5] - mu[6] * hk[6] - mu[7] * hk[7] * real(2) * uy + mu[8] * hk[8] * ux;
    // sigma term: sig = |Fm|^2 / psi^2
    const real sg = mu[1] * hk[1] * C.sig_e - mu[2] * hk[2] * C.sig_eps;
    if (psi > real(0)) {
        const real ip2 = real(1) / (psi * psi);
        Fm_bar[0] = sg * real(2) * Fm[0] * ip2;
        Fm_bar[1] = sg * real(2) * Fm[1] * ip2;
        psi_bar = -sg * real(2) * (Fm[0] * Fm[0] + Fm[1] * Fm[1]) * ip2 / psi;
    } else {
        Fm_bar[0] = Fm_bar[1] = real(0);
        psi_bar = real(0);
    }
    // u = (j + F/2) / rho
    const real jbx = ubx / rho, jby = uby / rho;
    Fbx += real(0.5) * jbx;
    Fby += real(0.5) * jby;
    rb -= (ubx * ux + uby * uy) / rho;
    // adjoint of m: direct (1 - s) part plus rho and j paths
    real mb[Q];
#pragma unroll
    for (int k = 0; k < Q; ++k) mb[k] = mu[k] * (real(1) - sk[k]);
    mb[0] += rb;
    mb[3] += jbx;
    mb[5] += jby;
#pragma unroll
    for (int a = 0; a < Q; ++a) {
        real s = real(0);
#pragma unroll
        for (int k = 0; k < Q; ++k)
            if (L::M[k][a] != 0) s += real(L::M[k][a]) * mb[k];
        gf[a] = s;
    }
    rho_bar = real(0);  // the density path is carried by mb[0] (rho = m_0 = sum f)
    F_bar[0] = Fbx;
    F_bar[1] = Fby;
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
