// lbm_host.hpp -- host-side internals of the C-ABI library: the context
// object, status helpers, geometry preprocessing and EOS helpers.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/lbm.h"
#include "lbm_kernels.hpp"
#include "lbm_kernels.hpp"

namespace lbm {

// ---- status
int fail(int code, const std::string& msg);
int ok();
#define LBM_HIP(call)                                                              \
    do {                                                                           \
        hipError_t e_ = (call);                                                    \
        if (e_ != hipSuccess)                                                      \
            return ::lbm::fail(LBM_EDEVICE, std::string(#call) + ": " +            \
                                                hipGetErrorString(e_));            \
    } while (0)

// ---- equation of state (thermo.cpp)
double eos_pressure(const lbm_params& p, double rho);
double pr_Tc(double a, double b, double R);
double pr_aphi(const lbm_params& p);
double psi_argument(const lbm_params& p, double rho);
int eos_critical(int eos, double a, double b, double R, double omega, double* Tc, double* rhoc);
int eos_coexistence(const lbm_params& p, double* rho_g, double* rho_l);

// ---- validation
int validate(const lbm_params* p);

// ---- geometry (geometry.cpp)
// node class per node and the increasing list of wall nodes (solid nodes
// with a fluid neighbour along a non-rest lattice velocity)
struct Geometry {
    std::vector<uint8_t> cls;
    std::vector<int32_t> widx;
    std::vector<int64_t> walls;
    int64_t n_fluid = 0;
};
int build_geometry(const lbm_params& p, const uint8_t* solid, Geometry& g);
// Geometric-formulation stencils of every wall node (D2Q9): code packs, for
// the two characteristic points k = 0, 1, the 3x3 neighbour index (dx+1) +
// 3 (dy+1) of the two mesh-line nodes a, b (4 bits each, at bit 10 k) and
// whether each is fluid (bits 8, 9 of the k field); bit 20: take the min
// (theta_a > 90 deg) instead of the max; t[2 w + k] the weight of b.
void build_gf_stencils(const lbm_params& p, const Geometry& g, const double* theta_deg,
                       std::vector<int32_t>& code, std::vector<double>& t);

// ---- adjoint (api.cpp): checks and runs lbm_adjoint with work_dev as the
// call's scratch (the caller's workspace or the library's static array)
int adjoint_entry(lbm_ctx* c, int32_t seed_kind, const void* seed_dev, int64_t T, int64_t K,
                  const void* ckpt_dev, void* work_dev, size_t work_bytes, void* grad_phi_dev,
                  void* grad_drho_dev, void* lam0_dev);

// ---- workspace carving
struct Carver {
    char* base;
    size_t off = 0, cap;
    Carver(void* b, size_t c) : base((char*)b), cap(c) {}
    template <typename T>
    T* take(size_t count) {
        off = (off + 255) & ~size_t(255);
        T* p = base ? reinterpret_cast<T*>(base + off) : nullptr;
        off += count * sizeof(T);
        return p;
    }
};

}  // namespace lbm

// one lattice of a multi-case context
struct lbm_case {
    int nx = 0, ny = 0;
    int pitch = 0;    // nodes from one row to the next in the case's arrays
    int64_t N = 0;    // nx * ny lattice nodes
    int64_t NP = 0;   // pitch * ny stored nodes
    int64_t n_wall_max = 0;
    uint64_t f_off = 0, node_off = 0, wall_off = 0;
    lbm::Geometry geom;
    bool have_geom = false, have_fields = false;
};

// the context (opaque in the C ABI)
struct lbm_ctx {
    lbm_params p;
    int Q = 9, D = 2;
    int64_t N = 0;
    int prec = 4;
    hipStream_t stream = nullptr;
    void* ws = nullptr;
    size_t ws_bytes = 0;
    int64_t n_wall_max = 0;
    // carved device arrays
    void* f[2] = {nullptr, nullptr};
    int cur = 0;
    uint8_t* cls = nullptr;
    int32_t* widx = nullptr;
    int32_t* wall_list = nullptr;
    void* phi = nullptr;
    void* drho = nullptr;
    int32_t* flag = nullptr;
    double* part = nullptr;
    double* diag_out = nullptr;
    // node densities of the D3Q19 sweeps: rho_buf[rho_idx] is read by the
    // next step; rho_valid when it already holds the density of the current
    // state (formed by a step of a PSUM variant, or by a density pass since),
    // so that the next step needs no density pass; rho_buf[rho_idx ^ 1]
    // receives the density a PSUM step forms, with ring as its scratch
    void* rho_buf[2] = {nullptr, nullptr};
    int rho_idx = 0;
    bool rho_valid = false;
    void* ring = nullptr;
    int nparts = 0;
    int32_t* gfcode = nullptr;  // geometric-formulation stencil code per wall node
    // per-tile wall lists of the D2Q9 tile step (see Fields::tw_pack)
    int32_t* tw_pack = nullptr;
    int32_t* tw_code = nullptr;  // gfcode of each entry
    int32_t* tw_widx = nullptr;  // wall-list index of each entry, -1 when empty
    void* tw_phi = nullptr;
    void* tw_drho = nullptr;
    int64_t tw_cap = 0;     // entries available in the workspace
    int tw_stride = 0;      // entries per tile of the current lists (0: none)
    int tw_variant = -1;    // tile variant the lists were built for
    bool tw_dirty = true;   // geometry, wetting or variant changed since
    // host state
    lbm::Geometry geom;
    bool have_geom = false, have_fields = false, domain_error = false;
    int scheme = LBM_WET_IVD;
    int variant = 0;  // step-kernel tile variant (autotuner choice)
    double scalar = 0.0;
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    // multi-case contexts
    bool is_batch = false;
    size_t f_bytes = 0;  // bytes of one population arena
    std::vector<lbm_case> cases;
    lbm::CaseDesc* d_cases = nullptr;
    lbm::TileRef* d_tiles = nullptr;
    int64_t max_tiles = 0;
    int ntiles = 0;
    int tiles_variant = -1;  // variant the uploaded tile table was built for
    // graph replay of `graph_steps` steps (0: plain launches)
    int64_t graph_steps = 0;
    hipStream_t cap_stream = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t graph_exec = nullptr;
    int graph_parity = -1;
    bool graph_dirty = true;
};
