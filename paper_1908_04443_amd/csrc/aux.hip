// aux.hip -- small kernels around the step: equilibrium initialisation,
// clearing solid slots, fills, and the final pass of the diagnostics.
#include "lbm_kernels.hpp"

namespace lbm {

template <typename L, typename real>
__global__ void k_init_eq(const uint8_t* __restrict__ cls, const real* __restrict__ rho,
                          const real* __restrict__ u, real* __restrict__ f, int64_t N, int nx,
                          int pitch) {
    // storage index n (rows `pitch` apart; positions past nx in a row get 0);
    // rho and u are dense, rows nx apart
    const int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= N) return;
    const int64_t row = n / pitch, x = n - row * pitch;
    const int64_t nd = row * nx + x, Nd = N / pitch * nx;
    const bool fluid = x < nx && cls[n] == CLS_FLUID;
    real uu[3] = {real(0), real(0), real(0)};
    if (fluid && u) {
#pragma unroll
        for (int d = 0; d < L::D; ++d) uu[d] = u[d * Nd + nd];
    }
    const real r = fluid ? rho[nd] : real(0);
#pragma unroll
    for (int a = 0; a < L::Q; ++a) f[a * N + n] = fluid ? feq<L, real>(a, r, uu) : real(0);
}

template <typename real>
__global__ void k_mask_solid(int Q, const uint8_t* __restrict__ cls, real* __restrict__ f,
                             int64_t N) {
    const int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= N || cls[n] == CLS_FLUID) return;
    for (int a = 0; a < Q; ++a) f[a * N + n] = real(0);
}

// D3Q19 contexts keep their populations in pull form: slot a of node y holds
// the post-collision population that node y + e_a gathers in the next
// streaming (Eq. 3), and slot a of a non-fluid node y holds the bounce-back
// of its fluid neighbour y + e_a (halfway bounce-back, Fig. 3).  A
// post-stream field f then reads f_a(x) = slot_a(x - e_a) at every fluid x,
// with periodic wrap.
__device__ __forceinline__ int64_t src3(int x, int y, int z, int a, int nx, int ny, int nz) {
    int sx = x - D3Q19::ex[a], sy = y - D3Q19::ey[a], sz = z - D3Q19::ez[a];
    sx = sx < 0 ? sx + nx : (sx >= nx ? sx - nx : sx);
    sy = sy < 0 ? sy + ny : (sy >= ny ? sy - ny : sy);
    sz = sz < 0 ? sz + nz : (sz >= nz ? sz - nz : sz);
    return ((int64_t)sz * ny + sy) * nx + sx;
}

// post-stream f (Q x N) -> pull form; dst is cleared beforehand
template <typename real>
__global__ void k_scatter3(const uint8_t* __restrict__ cls, const real* __restrict__ f,
                           real* __restrict__ dst, int nx, int ny, int nz) {
    const int64_t N = (int64_t)nx * ny * nz;
    const int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= N || cls[n] != CLS_FLUID) return;
    const int x = (int)(n % nx), y = (int)((n / nx) % ny), z = (int)(n / ((int64_t)nx * ny));
#pragma unroll
    for (int a = 0; a < 19; ++a) dst[a * N + src3(x, y, z, a, nx, ny, nz)] = f[a * N + n];
}

// pull form -> post-stream f (Q x N), 0 off the fluid
template <typename real>
__global__ void k_gather3(const uint8_t* __restrict__ cls, const real* __restrict__ src,
                          real* __restrict__ f, int nx, int ny, int nz) {
    const int64_t N = (int64_t)nx * ny * nz;
    const int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= N) return;
    const bool fluid = cls[n] == CLS_FLUID;
    const int x = (int)(n % nx), y = (int)((n / nx) % ny), z = (int)(n / ((int64_t)nx * ny));
#pragma unroll
    for (int a = 0; a < 19; ++a)
        f[a * N + n] = fluid ? src[a * N + src3(x, y, z, a, nx, ny, nz)] : real(0);
}

template <typename T>
__global__ void k_fill(T* p, T v, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

// one workgroup: fixed-order reduction of the per-tile partials
__global__ void k_diag_final(const double* __restrict__ part, int nparts, double* out) {
    __shared__ double s_sum[256], s_umax[256], s_rmin[256], s_rmax[256], s_cnt[256];
    const int t = threadIdx.x;
    double sum = 0.0, umax = 0.0, rmin = 1e300, rmax = -1e300, cnt = 0.0;
    for (int i = t; i < nparts; i += 256) {
        const double* p = part + 5 * i;
        sum += p[0];
        umax = p[1] > umax ? p[1] : umax;
        rmin = p[2] < rmin ? p[2] : rmin;
        rmax = p[3] > rmax ? p[3] : rmax;
        cnt += p[4];
    }
    s_sum[t] = sum;
    s_umax[t] = umax;
    s_rmin[t] = rmin;
    s_rmax[t] = rmax;
    s_cnt[t] = cnt;
    __syncthreads();
    for (int off = 128; off >= 1; off >>= 1) {
        if (t < off) {
            s_sum[t] += s_sum[t + off];
            s_umax[t] = s_umax[t + off] > s_umax[t] ? s_umax[t + off] : s_umax[t];
            s_rmin[t] = s_rmin[t + off] < s_rmin[t] ? s_rmin[t + off] : s_rmin[t];
            s_rmax[t] = s_rmax[t + off] > s_rmax[t] ? s_rmax[t + off] : s_rmax[t];
            s_cnt[t] += s_cnt[t + off];
        }
        __syncthreads();
    }
    if (t == 0) {
        out[0] = s_sum[0];
        out[1] = s_umax[0];
        out[2] = s_rmin[0];
        out[3] = s_rmax[0];
        out[4] = s_cnt[0];
    }
}

// wall parameters of the per-tile wall lists: out[e] = in[widx[e]] (0 where
// the entry is empty)
template <typename real>
__global__ void k_gather_wall(const int32_t* __restrict__ widx, const real* __restrict__ phi,
                              const real* __restrict__ drho, real* __restrict__ ophi,
                              real* __restrict__ odrho, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int32_t k = widx[i];
    ophi[i] = k >= 0 ? phi[k] : real(0);
    odrho[i] = k >= 0 ? drho[k] : real(0);
}

__global__ void k_gather_code(const int32_t* __restrict__ widx, const int32_t* __restrict__ code,
                              int32_t* __restrict__ out, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int32_t k = widx[i];
    out[i] = k >= 0 ? code[k] : 0;
}

static inline unsigned nblk(int64_t n, int b) { return (unsigned)((n + b - 1) / b); }

hipError_t launch_gather_code(const int32_t* widx, const int32_t* code, int32_t* out, int64_t n,
                              hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_gather_code, dim3(nblk(n, 256)), dim3(256), 0, s, widx, code, out, n);
    return hipGetLastError();
}

template <typename real>
hipError_t launch_gather_wall(const int32_t* widx, const real* phi, const real* drho, real* ophi,
                              real* odrho, int64_t n, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL((k_gather_wall<real>), dim3(nblk(n, 256)), dim3(256), 0, s, widx, phi, drho,
                       ophi, odrho, n);
    return hipGetLastError();
}

template <typename real>
hipError_t launch_init_eq(int lattice, const uint8_t* cls, const real* rho, const real* u,
                          real* f, int64_t N, hipStream_t s, int nx, int pitch) {
    if (pitch < 1 || nx < 1 || nx > pitch || N % pitch) return hipErrorInvalidValue;
    if (lattice == 9)
        hipLaunchKernelGGL((k_init_eq<D2Q9, real>), dim3(nblk(N, 256)), dim3(256), 0, s, cls, rho,
                           u, f, N, nx, pitch);
    else
        hipLaunchKernelGGL((k_init_eq<D3Q19, real>), dim3(nblk(N, 256)), dim3(256), 0, s, cls,
                           rho, u, f, N, nx, pitch);
    return hipGetLastError();
}

template <typename real>
hipError_t launch_scatter3(const uint8_t* cls, const real* f, real* dst, int nx, int ny, int nz,
                           hipStream_t s) {
    const int64_t N = (int64_t)nx * ny * nz;
    hipLaunchKernelGGL((k_scatter3<real>), dim3(nblk(N, 256)), dim3(256), 0, s, cls, f, dst, nx,
                       ny, nz);
    return hipGetLastError();
}

template <typename real>
hipError_t launch_gather3(const uint8_t* cls, const real* src, real* f, int nx, int ny, int nz,
                          hipStream_t s) {
    const int64_t N = (int64_t)nx * ny * nz;
    hipLaunchKernelGGL((k_gather3<real>), dim3(nblk(N, 256)), dim3(256), 0, s, cls, src, f, nx,
                       ny, nz);
    return hipGetLastError();
}

template <typename real>
hipError_t launch_mask_solid(int Q, const uint8_t* cls, real* f, int64_t N, hipStream_t s) {
    hipLaunchKernelGGL((k_mask_solid<real>), dim3(nblk(N, 256)), dim3(256), 0, s, Q, cls, f, N);
    return hipGetLastError();
}

template <typename real>
hipError_t launch_fill(real* p, real v, int64_t n, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL((k_fill<real>), dim3(nblk(n, 256)), dim3(256), 0, s, p, v, n);
    return hipGetLastError();
}

hipError_t launch_fill_i32(int32_t* p, int32_t v, int64_t n, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL((k_fill<int32_t>), dim3(nblk(n, 256)), dim3(256), 0, s, p, v, n);
    return hipGetLastError();
}

hipError_t launch_diag_final(const double* part, int nparts, double* out, hipStream_t s) {
    hipLaunchKernelGGL(k_diag_final, dim3(1), dim3(256), 0, s, part, nparts, out);
    return hipGetLastError();
}

template hipError_t launch_init_eq<float>(int, const uint8_t*, const float*, const float*, float*,
                                          int64_t, hipStream_t, int, int);
template hipError_t launch_init_eq<double>(int, const uint8_t*, const double*, const double*,
                                           double*, int64_t, hipStream_t, int, int);
template hipError_t launch_scatter3<float>(const uint8_t*, const float*, float*, int, int, int,
                                           hipStream_t);
template hipError_t launch_scatter3<double>(const uint8_t*, const double*, double*, int, int, int,
                                            hipStream_t);
template hipError_t launch_gather3<float>(const uint8_t*, const float*, float*, int, int, int,
                                          hipStream_t);
template hipError_t launch_gather3<double>(const uint8_t*, const double*, double*, int, int, int,
                                           hipStream_t);
template hipError_t launch_mask_solid<float>(int, const uint8_t*, float*, int64_t, hipStream_t);
template hipError_t launch_mask_solid<double>(int, const uint8_t*, double*, int64_t, hipStream_t);
template hipError_t launch_fill<float>(float*, float, int64_t, hipStream_t);
template hipError_t launch_fill<double>(double*, double, int64_t, hipStream_t);
template hipError_t launch_gather_wall<float>(const int32_t*, const float*, const float*, float*,
                                              float*, int64_t, hipStream_t);
template hipError_t launch_gather_wall<double>(const int32_t*, const double*, const double*,
                                               double*, double*, int64_t, hipStream_t);

}  // namespace lbm
