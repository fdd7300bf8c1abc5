// api.cpp -- the extern "C" entry points of include/lbm.h.
//
// Host code only: argument and call-order validation, workspace carving,
// geometry upload and stream-ordered kernel launches.  No device memory is
// allocated here; every device array is carved from the caller's workspace.
#include <cmath>
#include <cstdlib>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>

#include "lbm_host.hpp"

namespace lbm {

static thread_local std::string g_err;

// relaxation group of each moment row (same tables as the device side)
static const int kGroup9[9] = {0, 1, 2, 3, 4, 3, 4, 5, 5};
static const int kGroup19[19] = {0, 1, 2, 3, 4, 3, 4, 3, 4, 5, 6, 5, 6, 5, 5, 5, 7, 7, 7};

int fail(int code, const std::string& msg) {
    g_err = msg;
    return code;
}
int ok() { return LBM_OK; }

int validate(const lbm_params* p) {
    if (!p) return fail(LBM_EINVAL, "params is NULL");
    if (p->lattice != 9 && p->lattice != 19) return fail(LBM_EINVAL, "lattice must be 9 or 19");
    if (p->precision != 4 && p->precision != 8) return fail(LBM_EINVAL, "precision must be 4 or 8");
    if (p->nx < 1 || p->ny < 1 || p->nz < 1) return fail(LBM_EINVAL, "sizes must be positive");
    if (p->lattice == 9 && p->nz != 1) return fail(LBM_EINVAL, "D2Q9 needs nz == 1");
    if (p->lattice == 19 && (p->ny > 65535 || p->nz > 65535))
        return fail(LBM_EINVAL, "D3Q19 needs ny and nz of at most 65535 (launch grid rows)");
    const double N = (double)p->nx * p->ny * p->nz;
    if (N > 4.0e9) return fail(LBM_EINVAL, "lattice too large");
    for (int k = 0; k < p->lattice; ++k)
        if (!(p->tau[k] > 0.5)) return fail(LBM_EINVAL, "every tau must exceed 0.5");
    {
        // rows of one moment group (e.g. jx, jy; pxx, pxy) share one rate
        const int* grp = (p->lattice == 9) ? kGroup9 : kGroup19;
        for (int k = 0; k < p->lattice; ++k)
            for (int j = 0; j < k; ++j)
                if (grp[j] == grp[k] && p->tau[j] != p->tau[k])
                    return fail(LBM_EINVAL, "tau must be equal within a moment group (rows " +
                                                std::to_string(j) + " and " + std::to_string(k) + ")");
    }
    if (p->eos != LBM_EOS_CS && p->eos != LBM_EOS_PR) return fail(LBM_EINVAL, "unknown eos");
    if (!(p->eos_a > 0 && p->eos_b > 0 && p->eos_R > 0 && p->eos_T > 0))
        return fail(LBM_EINVAL, "EOS constants must be positive");
    if (!(p->G != 0.0) || !std::isfinite(p->G)) return fail(LBM_EINVAL, "G must be nonzero");
    if (!std::isfinite(p->sigma)) return fail(LBM_EINVAL, "sigma must be finite");
    if (!(p->rho_g > 0 && p->rho_g < p->rho_l)) return fail(LBM_EINVAL, "need 0 < rho_g < rho_l");
    return LBM_OK;
}

template <typename real>
static Coef<real> make_coef(const lbm_ctx* c) {
    const lbm_params& p = c->p;
    Coef<real> C;
    std::memset(&C, 0, sizeof C);
    C.nx = p.nx;
    C.ny = p.ny;
    C.nz = p.nz;
    C.scheme = c->scheme;
    C.eos = p.eos;
    C.eos_a = (real)p.eos_a;
    C.eos_b = (real)p.eos_b;
    C.eos_RT = (real)(p.eos_R * p.eos_T);
    C.eos_aphi = (real)(p.eos == LBM_EOS_PR ? pr_aphi(p) : 0.0);
    C.two_over_G = (real)(2.0 / p.G);
    C.G = (real)p.G;
    if (c->scheme == LBM_WET_VD) {
        C.rho_w = (real)c->scalar;
        C.psi_w = (real)std::sqrt(psi_argument(p, c->scalar));
    }
    if (c->scheme == LBM_WET_SFI) C.G_w = (real)c->scalar;
    C.rho_g = (real)p.rho_g;
    C.rho_l = (real)p.rho_l;
    const int* grp = (p.lattice == 9) ? kGroup9 : kGroup19;
    for (int g = 0; g < NGRP; ++g) C.s[g] = (real)1;
    for (int k = 0; k < p.lattice; ++k) C.s[grp[k]] = (real)(1.0 / p.tau[k]);
    if (p.lattice == 9) {
        C.sig_e = (real)(12.0 * p.sigma / (p.tau[1] - 0.5));
        C.sig_eps = (real)(12.0 * p.sigma / (p.tau[2] - 0.5));
    } else {
        C.sig_e = (real)(114.0 * p.sigma / (p.tau[1] - 0.5));
        C.sig_eps = (real)0;
    }
    for (int d = 0; d < 3; ++d) C.body[d] = (real)p.body_force[d];
    return C;
}

template <typename real>
static Fields<real> make_fields(const lbm_ctx* c, int src) {
    Fields<real> F;
    F.fin = (const real*)c->f[src];
    F.fout = (real*)c->f[src ^ 1];
    F.cls = c->cls;
    F.widx = c->widx;
    F.phi = (const real*)c->phi;
    F.drho = (const real*)c->drho;
    F.flag = c->flag;
    F.rho = (real*)c->rho_buf[c->rho_idx];
    F.rho_next = (real*)c->rho_buf[c->rho_idx ^ 1];
    F.ring = (real*)c->ring;
    F.rho_valid = c->rho_valid;
    F.gfcode = c->gfcode;
    return F;
}

// number of workgroups of the field/diagnostic launch (variant 0)
static int grid_blocks(const lbm_params& p) {
    if (p.lattice == 9)
        return p.precision == 4 ? grid2d_blocks<float>(p.nx, p.ny, 0)
                                : grid2d_blocks<double>(p.nx, p.ny, 0);
    return p.precision == 4 ? grid3d_blocks<float>(p.nx, p.ny, p.nz, 0)
                            : grid3d_blocks<double>(p.nx, p.ny, p.nz, 0);
}

static int variant_count(int lattice, int precision) {
    if (lattice == 9) return precision == 4 ? step2d_variants<float>() : step2d_variants<double>();
    return precision == 4 ? step3d_variants<float>() : step3d_variants<double>();
}

// lay out the workspace; with ctx == nullptr only the size is computed
static size_t layout(const lbm_params& p, int64_t nwm, lbm_ctx* c) {
    Carver cv(c ? c->ws : nullptr, c ? c->ws_bytes : 0);
    const int64_t N = (int64_t)p.nx * p.ny * p.nz;
    const size_t s = (size_t)p.precision;
    const int Q = p.lattice;
    const int64_t nw = nwm > 0 ? nwm : 1;
    const int nparts = grid_blocks(p);
    void* f0 = cv.take<char>((size_t)Q * N * s);
    void* f1 = cv.take<char>((size_t)Q * N * s);
    uint8_t* cls = cv.take<uint8_t>(N);
    int32_t* widx = cv.take<int32_t>(N);
    int32_t* wl = cv.take<int32_t>(nw);
    void* phi = cv.take<char>(nw * s);
    void* drho = cv.take<char>(nw * s);
    int32_t* flag = cv.take<int32_t>(4);
    double* part = cv.take<double>(5 * (size_t)nparts);
    double* dout = cv.take<double>(8);
    void* rho = cv.take<char>((size_t)N * s);  // density pass of the sweep kernels
    // D3Q19: the density a PSUM step forms, and its per-block partial sums
    void* rho2 = cv.take<char>(Q == 19 ? (size_t)N * s : 0);
    const size_t ring_el = Q != 19 ? 0
                           : (p.precision == 4 ? step3d_ring_elems<float>(p.nx, p.ny, p.nz)
                                               : step3d_ring_elems<double>(p.nx, p.ny, p.nz));
    void* ring = cv.take<char>(ring_el * s);
    // per-tile wall lists: up to 256 entries per tile of the tile variant
    // with the most tiles (D2Q9 only)
    int64_t twcap = 0;
    if (Q == 9) {
        const int nv = p.precision == 4 ? tile2d_variants<float>() : tile2d_variants<double>();
        for (int v = 0; v < nv; ++v) {
            const int64_t nt = p.precision == 4 ? grid2d_blocks<float>(p.nx, p.ny, v)
                                                : grid2d_blocks<double>(p.nx, p.ny, v);
            twcap = nt * 256 > twcap ? nt * 256 : twcap;
        }
    }
    int32_t* twp = cv.take<int32_t>(twcap);
    int32_t* tww = cv.take<int32_t>(twcap);
    void* twphi = cv.take<char>(twcap * s);
    void* twdrho = cv.take<char>(twcap * s);
    int32_t* twc = cv.take<int32_t>(twcap);
    int32_t* gfc = cv.take<int32_t>(nw);
    if (c) {
        c->rho_buf[0] = rho;
        c->rho_buf[1] = Q == 19 ? rho2 : rho;
        c->ring = ring;
        c->tw_code = twc;
        c->gfcode = gfc;
        c->tw_pack = twp;
        c->tw_widx = tww;
        c->tw_phi = twphi;
        c->tw_drho = twdrho;
        c->tw_cap = twcap;
        c->f[0] = f0;
        c->f[1] = f1;
        c->cls = cls;
        c->widx = widx;
        c->wall_list = wl;
        c->phi = phi;
        c->drho = drho;
        c->flag = flag;
        c->part = part;
        c->diag_out = dout;
        c->nparts = nparts;
    }
    return (cv.off + 255) & ~size_t(255);
}

template <typename real>
static int launch_mode(lbm_ctx* c, int mode, real* rho, real* u, double* part) {
    Coef<real> C = make_coef<real>(c);
    Fields<real> F = make_fields<real>(c, c->cur);
    FieldOut<real> O{rho, u, part};
    hipError_t e = (c->p.lattice == 9) ? launch_step2d<real>(C, F, O, mode, 0, c->stream)
                                       : launch_step3d<real>(C, F, O, mode, 0, c->stream);
    if (e != hipSuccess) return fail(LBM_EDEVICE, std::string("step launch: ") + hipGetErrorString(e));
    if (c->p.lattice == 19) c->rho_valid = true;  // the field pass used or formed it
    return LBM_OK;
}

// ---- multi-case tile table: (case, tile origin) for every tile of the
// chosen tile shape, case by case in row-major tile order
template <typename real>
static int ensure_tiles(lbm_ctx* c) {
    if (c->tiles_variant == c->variant) return LBM_OK;
    int TX = 0, TY = 0;
    tile2d_shape<real>(c->variant, &TX, &TY);
    std::vector<TileRef> t;
    for (size_t i = 0; i < c->cases.size(); ++i) {
        const lbm_case& k = c->cases[i];
        for (int y = 0; y < k.ny; y += TY)
            for (int x = 0; x < k.nx; x += TX) t.push_back(TileRef{(int32_t)i, x, y, 0});
    }
    if ((int64_t)t.size() > c->max_tiles) return fail(LBM_EINVAL, "tile table exceeds its space");
    LBM_HIP(hipMemcpyAsync(c->d_tiles, t.data(), t.size() * sizeof(TileRef),
                           hipMemcpyHostToDevice, c->stream));
    LBM_HIP(hipStreamSynchronize(c->stream));
    c->ntiles = (int)t.size();
    c->tiles_variant = c->variant;
    c->graph_dirty = true;
    return LBM_OK;
}

// one step from buffer `src` to `src ^ 1`, launched on stream s; D3Q19
// steps read the density buffer ridx (already the density of src when
// rvalid) and a PSUM step writes the next one into ridx ^ 1
template <typename real>
static hipError_t launch_one(lbm_ctx* c, const Coef<real>& C, int src, hipStream_t s,
                             int ridx = 0, bool rvalid = false) {
    if (c->is_batch) {
        BatchArgs<real> B;
        B.fin = (const real*)c->f[src];
        B.fout = (real*)c->f[src ^ 1];
        B.cls = c->cls;
        B.widx = c->widx;
        B.phi = (const real*)c->phi;
        B.drho = (const real*)c->drho;
        B.flag = c->flag;
        B.cases = c->d_cases;
        B.tiles = c->d_tiles;
        if (c->tw_stride > 0 && c->tw_variant == c->variant) {
            B.tw_pack = c->tw_pack;
            B.tw_phi = (const real*)c->tw_phi;
            B.tw_drho = (const real*)c->tw_drho;
            B.tw_stride = c->tw_stride;
            B.tw_code = c->tw_code;
        }
        return launch_step2d_batch<real>(C, B, c->ntiles, c->variant, s);
    }
    Fields<real> F = make_fields<real>(c, src);
    F.rho = (real*)c->rho_buf[ridx];
    F.rho_next = (real*)c->rho_buf[ridx ^ 1];
    F.rho_valid = rvalid;
    if (c->tw_stride > 0 && c->tw_variant == c->variant) {
        F.tw_pack = c->tw_pack;
        F.tw_phi = (const real*)c->tw_phi;
        F.tw_drho = (const real*)c->tw_drho;
        F.tw_stride = c->tw_stride;
        F.tw_code = c->tw_code;
    }
    FieldOut<real> O{nullptr, nullptr, nullptr};
    return (c->p.lattice == 9) ? launch_step2d<real>(C, F, O, MODE_STEP, c->variant, s)
                               : launch_step3d<real>(C, F, O, MODE_STEP, c->variant, s);
}

static void drop_graph(lbm_ctx* c) {
    if (c->graph_exec) (void)hipGraphExecDestroy(c->graph_exec);
    if (c->graph) (void)hipGraphDestroy(c->graph);
    c->graph_exec = nullptr;
    c->graph = nullptr;
    c->graph_parity = -1;
}

// Capture graph_steps (even) steps starting from buffer c->cur on the
// library's own capture stream; the graph is replayed on the context stream.
template <typename real>
static int capture_graph(lbm_ctx* c, const Coef<real>& C) {
    drop_graph(c);
    if (!c->cap_stream) LBM_HIP(hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking));
    // a PSUM variant's graph starts from a valid density (run_steps makes
    // it so before every replay) and keeps it valid; other variants run the
    // density pass in every captured step
    const bool forms = c->Q == 19 && step3d_forms_density<real>(C, c->variant);
    LBM_HIP(hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeRelaxed));
    int src = c->cur, ridx = c->rho_idx;
    hipError_t e = hipSuccess;
    for (int64_t i = 0; i < c->graph_steps && e == hipSuccess; ++i) {
        e = launch_one<real>(c, C, src, c->cap_stream, ridx, forms);
        src ^= 1;
        if (forms) ridx ^= 1;
    }
    hipGraph_t g = nullptr;
    hipError_t e2 = hipStreamEndCapture(c->cap_stream, &g);
    if (e != hipSuccess || e2 != hipSuccess) {
        if (g) (void)hipGraphDestroy(g);
        return fail(LBM_EDEVICE, std::string("graph capture: ") +
                                     hipGetErrorString(e != hipSuccess ? e : e2));
    }
    c->graph = g;
    LBM_HIP(hipGraphInstantiate(&c->graph_exec, g, nullptr, nullptr, 0));
    c->graph_parity = c->cur | (c->rho_idx << 1);
    c->graph_dirty = false;
    return LBM_OK;
}

// Per-tile wall lists of the D2Q9 tile step under the improved
// virtual-density scheme and the geometric formulation: for every tile, the
// wall nodes of the tile plus its 1-node ring (the ones whose virtual
// density the tile forms, Eqs. 16-17 or Eq. 11) with their LDS positions,
// so that the step kernel fetches their phi and drho (or stencil code and
// weights) with its first loads instead of through a dependent wall-index
// lookup.  Entry block t belongs to the t-th tile in the kernel's numbering
// (row-major for one lattice, table order for a multi-case context).  Lists
// are off (stride 0) when a tile would hold more than 256 entries or the
// workspace is too small.
struct ListTile {
    const Geometry* g;
    int nx, ny, x0, y0;
    int64_t woff;  // offset of the tile's case in the wall-parameter arena
};

template <typename real>
static int upload_wall_lists(lbm_ctx* c, const std::vector<ListTile>& tiles, int TX, int TY) {
    const int LX = TX + 4;
    const int64_t nt = (int64_t)tiles.size();
    auto wrap = [](int v, int n) { v %= n; return v < 0 ? v + n : v; };
    auto node = [&](const ListTile& t, int lx, int ly) {
        return (int64_t)wrap(t.y0 - 2 + ly, t.ny) * t.nx + wrap(t.x0 - 2 + lx, t.nx);
    };
    // in a ragged tile psi is needed up to one node past the lattice's last
    // column or row (the force of its owned nodes), so walls further out
    // carry no entry: none of them forms a virtual density next to the cells
    // the multi-case step leaves empty (two nodes past and beyond)
    auto listed = [&](const ListTile& t, int lx, int ly) {
        return t.x0 - 2 + lx <= t.nx && t.y0 - 2 + ly <= t.ny &&
               t.g->cls[node(t, lx, ly)] == CLS_WALL;
    };
    std::vector<int32_t> cnt(nt, 0);
    int maxc = 0;
    for (int64_t i = 0; i < nt; ++i) {
        int k = 0;
        for (int ly = 1; ly <= TY + 2; ++ly)
            for (int lx = 1; lx <= TX + 2; ++lx) k += listed(tiles[i], lx, ly);
        cnt[i] = k;
        maxc = k > maxc ? k : maxc;
    }
    const int stride = maxc <= 64 ? 64 : ((maxc + 63) / 64) * 64;
    c->tw_variant = c->variant;
    c->tw_dirty = false;
    c->graph_dirty = true;
    c->tw_stride = 0;
    if (stride > 256 || nt * stride > c->tw_cap) return LBM_OK;
    std::vector<int32_t> pack(nt * stride), widx(nt * stride, -1);
    for (int64_t i = 0; i < nt; ++i) {
        const int64_t e0 = i * stride;
        const int32_t hi = cnt[i] << 16;
        int k = 0;
        for (int ly = 1; ly <= TY + 2; ++ly)
            for (int lx = 1; lx <= TX + 2; ++lx) {
                if (!listed(tiles[i], lx, ly)) continue;
                const int64_t n = node(tiles[i], lx, ly);
                pack[e0 + k] = hi | (ly * LX + lx);
                widx[e0 + k] = (int32_t)(tiles[i].woff + tiles[i].g->widx[n]);
                ++k;
            }
        for (; k < stride; ++k) pack[e0 + k] = hi | 0xFFFF;
    }
    const size_t bytes = (size_t)nt * stride * 4;
    LBM_HIP(hipMemcpyAsync(c->tw_pack, pack.data(), bytes, hipMemcpyHostToDevice, c->stream));
    LBM_HIP(hipMemcpyAsync(c->tw_widx, widx.data(), bytes, hipMemcpyHostToDevice, c->stream));
    LBM_HIP(launch_gather_wall<real>(c->tw_widx, (const real*)c->phi, (const real*)c->drho,
                                     (real*)c->tw_phi, (real*)c->tw_drho, nt * stride,
                                     c->stream));
    if (c->scheme == LBM_WET_GF)
        LBM_HIP(launch_gather_code(c->tw_widx, c->gfcode, c->tw_code, nt * stride, c->stream));
    LBM_HIP(hipStreamSynchronize(c->stream));  // the host vectors go out of scope
    c->tw_stride = stride;
    return LBM_OK;
}

template <typename real>
static int ensure_wall_lists(lbm_ctx* c) {
    const bool want = c->p.lattice == 9 && (c->scheme == LBM_WET_IVD || c->scheme == LBM_WET_GF) &&
                      c->variant < tile2d_variants<real>() && (c->is_batch || c->have_geom);
    if (!want) {
        c->tw_stride = 0;
        return LBM_OK;
    }
    if (!c->tw_dirty && c->tw_variant == c->variant) return LBM_OK;
    int TX = 0, TY = 0;
    tile2d_shape<real>(c->variant, &TX, &TY);
    std::vector<ListTile> t;
    if (!c->is_batch) {
        for (int y = 0; y < c->p.ny; y += TY)
            for (int x = 0; x < c->p.nx; x += TX) t.push_back({&c->geom, c->p.nx, c->p.ny, x, y, 0});
    } else {
        // the order of ensure_tiles
        for (const lbm_case& k : c->cases) {
            if (!k.have_geom) {
                c->tw_stride = 0;
                return LBM_OK;
            }
            for (int y = 0; y < k.ny; y += TY)
                for (int x = 0; x < k.nx; x += TX)
                    t.push_back({&k.geom, k.nx, k.ny, x, y, (int64_t)k.wall_off});
        }
    }
    return upload_wall_lists<real>(c, t, TX, TY);
}

template <typename real>
static int run_steps(lbm_ctx* c, int64_t nsteps) {
    Coef<real> C = make_coef<real>(c);
    if (c->is_batch) {
        int rc = ensure_tiles<real>(c);
        if (rc != LBM_OK) return rc;
    }
    {
        int rc = ensure_wall_lists<real>(c);
        if (rc != LBM_OK) return rc;
    }
    int64_t done = 0;
    // D3Q19 sweeps that form the next step's density (PSUM variants)
    const bool forms = c->Q == 19 && !c->is_batch && step3d_forms_density<real>(C, c->variant);
    if (c->graph_steps > 0 && nsteps >= c->graph_steps) {
        if (forms && !c->rho_valid) {
            // the graph starts from a valid density: form it once here
            Fields<real> F = make_fields<real>(c, c->cur);
            LBM_HIP(launch_density3d<real>(C, F, c->stream));
            c->rho_valid = true;
        }
        if (c->graph_dirty || c->graph_parity != (c->cur | (c->rho_idx << 1)) || !c->graph_exec) {
            int rc = capture_graph<real>(c, C);
            if (rc != LBM_OK) return rc;
        }
        // an even number of steps per replay leaves the buffer parities as
        // they are
        for (; nsteps - done >= c->graph_steps; done += c->graph_steps)
            LBM_HIP(hipGraphLaunch(c->graph_exec, c->stream));
        if (done > 0 && c->Q == 19) c->rho_valid = forms;
    }
    for (; done < nsteps; ++done) {
        hipError_t e = launch_one<real>(c, C, c->cur, c->stream, c->rho_idx, c->rho_valid);
        if (e != hipSuccess)
            return fail(LBM_EDEVICE, std::string("step launch: ") + hipGetErrorString(e));
        c->cur ^= 1;
        if (c->Q == 19) {
            if (forms) c->rho_idx ^= 1;
            c->rho_valid = forms;
        }
    }
    return LBM_OK;
}

// ---- per-case views of a multi-case context (single-lattice launchers)
template <typename real>
static Coef<real> case_coef(const lbm_ctx* c, const lbm_case& k) {
    Coef<real> C = make_coef<real>(c);
    C.nx = k.nx;
    C.ny = k.ny;
    C.nz = 1;
    C.pitch = k.pitch;
    return C;
}

template <typename real>
static Fields<real> case_fields(const lbm_ctx* c, const lbm_case& k) {
    Fields<real> F;
    F.fin = (const real*)c->f[c->cur] + k.f_off;
    F.fout = (real*)c->f[c->cur ^ 1] + k.f_off;
    F.cls = c->cls + k.node_off;
    F.widx = c->widx + k.node_off;
    F.phi = (const real*)c->phi + k.wall_off;
    F.drho = (const real*)c->drho + k.wall_off;
    F.flag = c->flag;
    F.rho = (real*)c->rho_buf[0];
    F.gfcode = c->gfcode;
    return F;
}

template <typename real>
static int case_fields_launch(lbm_ctx* c, const lbm_case& k, real* rho, real* u, double* part) {
    FieldOut<real> O{rho, u, part};
    hipError_t e = launch_step2d<real>(case_coef<real>(c, k), case_fields<real>(c, k), O,
                                       MODE_FIELDS, 0, c->stream);
    if (e != hipSuccess) return fail(LBM_EDEVICE, std::string("field launch: ") + hipGetErrorString(e));
    return LBM_OK;
}

template <typename real>
static int fill_wetting(lbm_ctx* c, const void* phi_dev, const void* drho_dev, double phi0,
                        double drho0) {
    const int64_t nw = (int64_t)c->geom.walls.size();
    const size_t bytes = (size_t)nw * sizeof(real);
    if (nw == 0) return LBM_OK;
    if (phi_dev)
        LBM_HIP(hipMemcpyAsync(c->phi, phi_dev, bytes, hipMemcpyDeviceToDevice, c->stream));
    else
        LBM_HIP(launch_fill<real>((real*)c->phi, (real)phi0, nw, c->stream));
    if (drho_dev)
        LBM_HIP(hipMemcpyAsync(c->drho, drho_dev, bytes, hipMemcpyDeviceToDevice, c->stream));
    else
        LBM_HIP(launch_fill<real>((real*)c->drho, (real)drho0, nw, c->stream));
    if (phi_dev) {
        std::vector<real> h(nw);
        LBM_HIP(hipMemcpyAsync(h.data(), c->phi, bytes, hipMemcpyDeviceToHost, c->stream));
        LBM_HIP(hipStreamSynchronize(c->stream));
        for (int64_t i = 0; i < nw; ++i)
            if (!(h[i] > 0)) return fail(LBM_EINVAL, "phi must be positive on every wall node");
    }
    return LBM_OK;
}

// Geometric formulation: prescribed angles (per wall node from the device,
// or one value) -> stencil codes and interpolation weights (host), stored
// in gfcode and in the phi/drho arrays of the context.
template <typename real>
static int fill_gf(lbm_ctx* c, const void* theta_dev, double theta0) {
    const int64_t nw = (int64_t)c->geom.walls.size();
    std::vector<double> th(nw, theta0);
    if (theta_dev && nw > 0) {
        std::vector<real> h(nw);
        LBM_HIP(hipMemcpyAsync(h.data(), theta_dev, (size_t)nw * sizeof(real),
                               hipMemcpyDeviceToHost, c->stream));
        LBM_HIP(hipStreamSynchronize(c->stream));
        for (int64_t i = 0; i < nw; ++i) th[i] = (double)h[i];
    }
    for (int64_t i = 0; i < nw; ++i)
        if (!(th[i] > 0.0 && th[i] < 180.0))
            return fail(LBM_EINVAL, "geometric formulation: angles must lie in (0, 180) degrees");
    if (nw == 0) return LBM_OK;
    std::vector<int32_t> code;
    std::vector<double> t;
    build_gf_stencils(c->p, c->geom, th.data(), code, t);
    std::vector<real> t0(nw), t1(nw);
    for (int64_t i = 0; i < nw; ++i) {
        t0[i] = (real)t[2 * i];
        t1[i] = (real)t[2 * i + 1];
    }
    LBM_HIP(hipMemcpyAsync(c->gfcode, code.data(), (size_t)nw * 4, hipMemcpyHostToDevice, c->stream));
    LBM_HIP(hipMemcpyAsync(c->phi, t0.data(), (size_t)nw * sizeof(real), hipMemcpyHostToDevice,
                           c->stream));
    LBM_HIP(hipMemcpyAsync(c->drho, t1.data(), (size_t)nw * sizeof(real), hipMemcpyHostToDevice,
                           c->stream));
    LBM_HIP(hipStreamSynchronize(c->stream));  // the host vectors go out of scope
    return LBM_OK;
}

// geometry and fields set (on every case of a multi-case context)
static bool ready(const lbm_ctx* c) {
    if (!c->is_batch) return c->have_geom && c->have_fields;
    for (const lbm_case& k : c->cases)
        if (!k.have_geom || !k.have_fields) return false;
    return !c->cases.empty();
}

static int ctx_variants(const lbm_ctx* c) {
    if (c->is_batch) return c->prec == 4 ? tile2d_variants<float>() : tile2d_variants<double>();
    return variant_count(c->p.lattice, c->p.precision);
}

// bytes of one population buffer (one ping-pong side)
static size_t state_bytes(const lbm_ctx* c) {
    if (c->is_batch) return c->f_bytes;
    return (size_t)c->Q * c->N * c->prec;
}

// ---- multi-case layout: packed arenas for all cases
static uint64_t round_up(uint64_t v, uint64_t a) { return (v + a - 1) / a * a; }

// Row pitch of a case's arrays: the width rounded up to whole 128-byte lines,
// so that every row starts on a line (the arenas and each case's part start
// on one too).  A row that does not start on a line splits each tile row of
// the step into one more line at each end, partly written.
static uint64_t case_pitch(int nx, size_t elem_bytes) {
    return round_up((uint64_t)nx, 128 / elem_bytes);
}

static size_t layout_batch(const lbm_params& p, int ncases, const int32_t* nx, const int32_t* ny,
                           const int64_t* nwm, lbm_ctx* c) {
    Carver cv(c ? c->ws : nullptr, c ? c->ws_bytes : 0);
    const size_t s = (size_t)p.precision;
    uint64_t f_off = 0, node_off = 0, wall_off = 0;
    int64_t max_parts = 1;
    std::vector<lbm_case> cs(ncases);
    for (int i = 0; i < ncases; ++i) {
        lbm_case& k = cs[i];
        k.nx = nx[i];
        k.ny = ny[i];
        k.N = (int64_t)nx[i] * ny[i];
        k.pitch = (int)case_pitch(nx[i], s);
        k.NP = (int64_t)k.pitch * ny[i];
        k.n_wall_max = nwm[i];
        k.f_off = f_off;
        f_off += round_up(9 * (uint64_t)k.NP, 64);
        k.node_off = node_off;
        node_off += round_up((uint64_t)k.NP, 256);
        k.wall_off = wall_off;
        wall_off += round_up((uint64_t)(nwm[i] > 0 ? nwm[i] : 1), 64);
        const int parts = p.precision == 4 ? grid2d_blocks<float>(k.nx, k.ny, 0)
                                           : grid2d_blocks<double>(k.nx, k.ny, 0);
        max_parts = parts > max_parts ? parts : max_parts;
    }
    int64_t tiles_max = 0;
    const int nv = p.precision == 4 ? tile2d_variants<float>() : tile2d_variants<double>();
    for (int v = 0; v < nv; ++v) {
        int TX, TY;
        if (p.precision == 4) tile2d_shape<float>(v, &TX, &TY);
        else tile2d_shape<double>(v, &TX, &TY);
        int64_t t = 0;
        for (int i = 0; i < ncases; ++i)
            t += (int64_t)((nx[i] + TX - 1) / TX) * ((ny[i] + TY - 1) / TY);
        tiles_max = t > tiles_max ? t : tiles_max;
    }
    void* f0 = cv.take<char>(f_off * s);
    void* f1 = cv.take<char>(f_off * s);
    uint8_t* cls = cv.take<uint8_t>(node_off);
    int32_t* widx = cv.take<int32_t>(node_off);
    void* phi = cv.take<char>(wall_off * s);
    void* drho = cv.take<char>(wall_off * s);
    CaseDesc* dc = cv.take<CaseDesc>(ncases);
    TileRef* dt = cv.take<TileRef>(tiles_max);
    int32_t* twp = cv.take<int32_t>(tiles_max * 256);  // per-tile wall lists
    int32_t* tww = cv.take<int32_t>(tiles_max * 256);
    void* twphi = cv.take<char>(tiles_max * 256 * s);
    void* twdrho = cv.take<char>(tiles_max * 256 * s);
    int32_t* twc = cv.take<int32_t>(tiles_max * 256);
    int32_t* flag = cv.take<int32_t>(4);
    double* part = cv.take<double>(5 * (size_t)max_parts);
    double* dout = cv.take<double>(8);
    if (c) {
        c->f[0] = f0;
        c->f[1] = f1;
        c->cls = cls;
        c->widx = widx;
        c->phi = phi;
        c->drho = drho;
        c->d_cases = dc;
        c->d_tiles = dt;
        c->max_tiles = tiles_max;
        c->tw_pack = twp;
        c->tw_widx = tww;
        c->tw_phi = twphi;
        c->tw_drho = twdrho;
        c->tw_code = twc;
        c->tw_cap = tiles_max * 256;
        c->flag = flag;
        c->part = part;
        c->diag_out = dout;
        c->nparts = (int)max_parts;
        c->f_bytes = f_off * s;
        c->n_wall_max = (int64_t)wall_off;
        int64_t N = 0;
        for (auto& k : cs) N += k.N;
        c->N = N;
        c->cases = std::move(cs);
    }
    return (cv.off + 255) & ~size_t(255);
}

static int check_batch_args(const lbm_params* p, int32_t ncases, const int32_t* nx,
                            const int32_t* ny, const int64_t* nwm) {
    if (!p || !nx || !ny || !nwm) return fail(LBM_EINVAL, "NULL argument");
    if (p->lattice != 9) return fail(LBM_EINVAL, "multi-case contexts are D2Q9");
    if (ncases < 1) return fail(LBM_EINVAL, "ncases must be >= 1");
    lbm_params q = *p;
    q.nx = q.ny = q.nz = 1;
    int rc = validate(&q);
    if (rc != LBM_OK) return rc;
    for (int i = 0; i < ncases; ++i) {
        if (nx[i] < 1 || ny[i] < 1 || nwm[i] < 0) return fail(LBM_EINVAL, "bad case size");
        if ((uint64_t)9 * case_pitch(nx[i], (size_t)p->precision) * ny[i] * p->precision >
            0xFFFFFFFFull)
            return fail(LBM_EINVAL, "a case's populations must stay below 4 GiB");
    }
    return LBM_OK;
}

template <typename real>
static int upload_cases(lbm_ctx* c) {
    std::vector<CaseDesc> d(c->cases.size());
    for (size_t i = 0; i < d.size(); ++i) {
        const lbm_case& k = c->cases[i];
        d[i] = CaseDesc{k.nx, k.ny, k.pitch, 0, k.f_off, k.node_off, k.wall_off};
    }
    LBM_HIP(hipMemcpyAsync(c->d_cases, d.data(), d.size() * sizeof(CaseDesc),
                           hipMemcpyHostToDevice, c->stream));
    LBM_HIP(hipStreamSynchronize(c->stream));
    return LBM_OK;
}

// ---- adjoint workspace: K segment states, ping-pong lam (partial + ext),
// per-node gather inputs, gradient scratch
struct AdjLayout {
    size_t seg, lam0, lam1, ext0, ext1, sb, gphi, gdrho, total;
};
static AdjLayout adj_layout(const lbm_ctx* c, int64_t K) {
    AdjLayout L{};
    const size_t s = (size_t)c->prec, N = (size_t)c->N;
    size_t off = 0;
    auto take = [&](size_t bytes) {
        off = (off + 255) & ~size_t(255);
        size_t o = off;
        off += bytes;
        return o;
    };
    L.seg = take((size_t)K * 9 * N * s);
    L.lam0 = take(9 * N * s);
    L.lam1 = take(9 * N * s);
    L.ext0 = take(N * s);
    L.ext1 = take(N * s);
    L.sb = take(4 * N * s);
    const size_t nw = c->geom.walls.empty() ? 1 : c->geom.walls.size();
    L.gphi = take(nw * s);
    L.gdrho = take(nw * s);
    L.total = (off + 255) & ~size_t(255);
    return L;
}

// one forward step from fin to fout (same kernels as lbm_step)
template <typename real>
static hipError_t step_from(lbm_ctx* c, const Coef<real>& C, const void* fin, void* fout) {
    Fields<real> F = make_fields<real>(c, c->cur);
    F.fin = (const real*)fin;
    F.fout = (real*)fout;
    FieldOut<real> O{nullptr, nullptr, nullptr};
    return launch_step2d<real>(C, F, O, MODE_STEP, c->variant, c->stream);
}

template <typename real>
static int run_adjoint(lbm_ctx* c, int kind, const void* seed, int64_t T, int64_t K,
                       const void* ckpt, char* work, void* gphi, void* gdrho, void* lam0) {
    const AdjLayout Lw = adj_layout(c, K);
    const uint32_t N = (uint32_t)c->N;
    const size_t state = (size_t)9 * N * sizeof(real);
    const int64_t nw = (int64_t)c->geom.walls.size();
    real* gp = gphi ? (real*)gphi : (real*)(work + Lw.gphi);
    real* gd = gdrho ? (real*)gdrho : (real*)(work + Lw.gdrho);
    LBM_HIP(launch_fill<real>(gp, real(0), nw, c->stream));
    LBM_HIP(launch_fill<real>(gd, real(0), nw, c->stream));
    real* lam[2] = {(real*)(work + Lw.lam0), (real*)(work + Lw.lam1)};
    real* ext[2] = {(real*)(work + Lw.ext0), (real*)(work + Lw.ext1)};
    char* seg = work + Lw.seg;
    LBM_HIP(launch_adj_seed<real>(kind, c->cls, (const real*)seed, lam[0], ext[0], N, c->stream));
    int cur = 0;
    const Coef<real> C = make_coef<real>(c);
    const int64_t nseg = (T + K - 1) / K;
    for (int64_t sg = nseg - 1; sg >= 0; --sg) {
        const int64_t len = (T - sg * K) < K ? (T - sg * K) : K;
        // restore the checkpoint and recompute the segment's states
        LBM_HIP(hipMemcpyAsync(seg, (const char*)ckpt + (size_t)sg * state, state,
                               hipMemcpyDeviceToDevice, c->stream));
        for (int64_t i = 1; i < len; ++i)
            LBM_HIP(step_from<real>(c, C, seg + (size_t)(i - 1) * state, seg + (size_t)i * state));
        for (int64_t i = len - 1; i >= 0; --i) {
            Fields<real> F = make_fields<real>(c, c->cur);
            F.fin = (const real*)(seg + (size_t)i * state);
            F.fout = nullptr;
            AdjArgs<real> A;
            A.lam_in = lam[cur];
            A.ext_in = ext[cur];
            A.lam_out = lam[cur ^ 1];
            A.ext_out = ext[cur ^ 1];
            A.sb = (real*)(work + Lw.sb);
            A.grad_phi = gp;
            A.grad_drho = gd;
            LBM_HIP(launch_adjoint2d<real>(C, F, A, c->stream));
            cur ^= 1;
        }
    }
    if (lam0)
        LBM_HIP(launch_adj_finish<real>(c->cls, lam[cur], ext[cur], (real*)lam0, N, c->stream));
    return LBM_OK;
}
// argument checks and dispatch of lbm_adjoint; work_dev is the scratch of
// the call (the caller's workspace, or the library's own static array)
int adjoint_entry(lbm_ctx* c, int32_t seed_kind, const void* seed_dev, int64_t T, int64_t K,
                  const void* ckpt_dev, void* work_dev, size_t work_bytes, void* grad_phi_dev,
                  void* grad_drho_dev, void* lam0_dev) {
    if (!c || !seed_dev || !ckpt_dev || !work_dev) return fail(LBM_EINVAL, "NULL argument");
    if (c->is_batch || c->p.lattice != 9)
        return fail(LBM_EINVAL, "the adjoint is implemented for single D2Q9 lattices");
    if (seed_kind != 0 && seed_kind != 1) return fail(LBM_EINVAL, "seed_kind must be 0 or 1");
    if (c->scheme == LBM_WET_GF)
        return fail(LBM_EINVAL, "no adjoint of the geometric formulation (its max/min and "
                                "interpolation stencils have no parameters to differentiate)");
    if (T < 1 || K < 1) return fail(LBM_EINVAL, "need T >= 1 and K >= 1");
    if (!c->have_geom) return fail(LBM_ESTATE, "no geometry set");
    if (c->domain_error) return fail(LBM_EDOMAIN, "a previous step left the psi domain");
    const size_t need = adj_layout(c, K).total;
    if (work_bytes < need)
        return fail(LBM_ENOMEM, "adjoint workspace needs " + std::to_string(need) + " bytes");
    if (((uintptr_t)work_dev & 255) != 0) return fail(LBM_EINVAL, "workspace must be 256-byte aligned");
    return c->prec == 4 ? run_adjoint<float>(c, seed_kind, seed_dev, T, K, ckpt_dev, (char*)work_dev,
                                             grad_phi_dev, grad_drho_dev, lam0_dev)
                        : run_adjoint<double>(c, seed_kind, seed_dev, T, K, ckpt_dev,
                                              (char*)work_dev, grad_phi_dev, grad_drho_dev, lam0_dev);
}

}  // namespace lbm

using namespace lbm;

extern "C" {

const char* lbm_version(void) { return "lbm-gfx950 1.0"; }

const char* lbm_status_string(int code) {
    switch (code) {
    case LBM_OK: return "ok";
    case LBM_EINVAL: return "invalid argument";
    case LBM_ENOMEM: return "workspace too small";
    case LBM_EDOMAIN: return "psi argument negative or NaN";
    case LBM_ESTATE: return "call out of order";
    case LBM_EDEVICE: return "HIP runtime error";
    default: return "unknown status";
    }
}

const char* lbm_last_error(void) { return g_err.c_str(); }

int lbm_validate_params(const lbm_params* p) { return validate(p); }

int lbm_eos_critical(int32_t eos, double a, double b, double R, double omega, double* Tc,
                     double* rhoc) {
    if (eos != LBM_EOS_CS && eos != LBM_EOS_PR) return fail(LBM_EINVAL, "unknown eos");
    if (!(a > 0 && b > 0 && R > 0)) return fail(LBM_EINVAL, "EOS constants must be positive");
    int rc = eos_critical(eos, a, b, R, omega, Tc, rhoc);
    return rc == LBM_OK ? rc : fail(rc, "critical point not bracketed");
}

int lbm_eos_coexistence(const lbm_params* p, double* rho_g, double* rho_l) {
    if (!p || !rho_g || !rho_l) return fail(LBM_EINVAL, "NULL argument");
    if (!(p->eos_a > 0 && p->eos_b > 0 && p->eos_R > 0 && p->eos_T > 0))
        return fail(LBM_EINVAL, "EOS constants must be positive");
    int rc = eos_coexistence(*p, rho_g, rho_l);
    return rc == LBM_OK ? rc : fail(rc, "temperature is not below the critical point");
}

int lbm_eos_eval(const lbm_params* p, double rho, double* p_eos, double* psi) {
    if (!p) return fail(LBM_EINVAL, "NULL params");
    const double pe = eos_pressure(*p, rho);
    const double arg = psi_argument(*p, rho);
    if (p_eos) *p_eos = pe;
    if (psi) *psi = arg >= 0 ? std::sqrt(arg) : std::nan("");
    return arg >= 0 ? LBM_OK : fail(LBM_EDOMAIN, "psi argument negative");
}

size_t lbm_workspace_bytes(const lbm_params* p, int64_t n_wall_max) {
    if (validate(p) != LBM_OK || n_wall_max < 0) return 0;
    return layout(*p, n_wall_max, nullptr);
}

// The timing events of a context: they only measure time, so they are
// recorded without a system-scope fence (no cache writeback and
// invalidation around the timed launches)
static bool create_timing_events(lbm_ctx* c) {
    return hipEventCreateWithFlags(&c->ev0, hipEventDisableSystemFence) == hipSuccess &&
           hipEventCreateWithFlags(&c->ev1, hipEventDisableSystemFence) == hipSuccess;
}

int lbm_create(const lbm_params* p, void* stream, void* workspace, size_t ws_bytes,
               int64_t n_wall_max, lbm_ctx** out) {
    if (!out) return fail(LBM_EINVAL, "out is NULL");
    *out = nullptr;
    int rc = validate(p);
    if (rc != LBM_OK) return rc;
    if (n_wall_max < 0) return fail(LBM_EINVAL, "n_wall_max must be >= 0");
    const size_t need = layout(*p, n_wall_max, nullptr);
    if (!workspace || ws_bytes < need)
        return fail(LBM_ENOMEM, "workspace needs " + std::to_string(need) + " bytes");
    if (((uintptr_t)workspace & 255) != 0) return fail(LBM_EINVAL, "workspace must be 256-byte aligned");
    lbm_ctx* c = new (std::nothrow) lbm_ctx();
    if (!c) return fail(LBM_ENOMEM, "host allocation failed");
    c->p = *p;
    c->Q = p->lattice;
    c->D = p->lattice == 9 ? 2 : 3;
    c->N = (int64_t)p->nx * p->ny * p->nz;
    c->prec = p->precision;
    c->stream = (hipStream_t)stream;
    c->ws = workspace;
    c->ws_bytes = ws_bytes;
    c->n_wall_max = n_wall_max;
    layout(*p, n_wall_max, c);
    if (p->lattice == 9)
        c->variant = p->precision == 4 ? tile2d_preferred_variant<float>()
                                       : tile2d_preferred_variant<double>();
    else
        c->variant = p->precision == 4 ? step3d_preferred_variant<float>(p->nx, p->ny, p->nz)
                                       : step3d_preferred_variant<double>(p->nx, p->ny, p->nz);
    if (!create_timing_events(c)) {
        lbm_destroy(c);  // releases whichever event was created
        return fail(LBM_EDEVICE, "hipEventCreate failed");
    }
    *out = c;
    return LBM_OK;
}

int lbm_destroy(lbm_ctx* c) {
    if (!c) return LBM_OK;
    drop_graph(c);
    if (c->cap_stream) (void)hipStreamDestroy(c->cap_stream);
    if (c->ev0) (void)hipEventDestroy(c->ev0);
    if (c->ev1) (void)hipEventDestroy(c->ev1);
    delete c;
    return LBM_OK;
}

int lbm_set_geometry(lbm_ctx* c, const uint8_t* solid_host) {
    if (!c || !solid_host) return fail(LBM_EINVAL, "NULL argument");
    if (c->is_batch) return fail(LBM_EINVAL, "multi-case context: use the _case call");
    Geometry g;
    build_geometry(c->p, solid_host, g);
    if ((int64_t)g.walls.size() > c->n_wall_max)
        return fail(LBM_EINVAL, "geometry has " + std::to_string(g.walls.size()) +
                                    " wall nodes, more than n_wall_max = " +
                                    std::to_string(c->n_wall_max));
    if (g.n_fluid == 0) return fail(LBM_EINVAL, "geometry has no fluid node");
    std::vector<int32_t> wl(g.walls.size());
    for (size_t i = 0; i < wl.size(); ++i) wl[i] = (int32_t)g.walls[i];
    LBM_HIP(hipMemcpyAsync(c->cls, g.cls.data(), (size_t)c->N, hipMemcpyHostToDevice, c->stream));
    LBM_HIP(hipMemcpyAsync(c->widx, g.widx.data(), (size_t)c->N * 4, hipMemcpyHostToDevice,
                           c->stream));
    if (!wl.empty())
        LBM_HIP(hipMemcpyAsync(c->wall_list, wl.data(), wl.size() * 4, hipMemcpyHostToDevice,
                               c->stream));
    LBM_HIP(hipStreamSynchronize(c->stream));
    c->geom = std::move(g);
    c->have_geom = true;
    c->have_fields = false;
    c->rho_valid = false;
    c->tw_dirty = true;
    c->scheme = LBM_WET_IVD;
    c->scalar = 0.0;
    int rc = (c->prec == 4) ? fill_wetting<float>(c, nullptr, nullptr, 1.0, 0.0)
                            : fill_wetting<double>(c, nullptr, nullptr, 1.0, 0.0);
    if (rc != LBM_OK) return rc;
    LBM_HIP(launch_fill_i32(c->flag, 0, 4, c->stream));
    return LBM_OK;
}

int lbm_gf_stencils(const lbm_params* p, const uint8_t* solid_host, const double* theta_deg_host,
                    double theta0, int64_t cap, int64_t* count, int32_t* nodes_host,
                    double* weights_host) {
    const int rc = validate(p);
    if (rc != LBM_OK) return rc;
    if (!solid_host || !count) return fail(LBM_EINVAL, "NULL argument");
    if (p->lattice != 9) return fail(LBM_EINVAL, "the geometric formulation is two-dimensional");
    Geometry g;
    build_geometry(*p, solid_host, g);
    const int64_t nw = (int64_t)g.walls.size();
    *count = nw;
    if (!nodes_host && !weights_host) return LBM_OK;
    if (!nodes_host || !weights_host) return fail(LBM_EINVAL, "need both output arrays");
    if (cap < nw) return fail(LBM_EINVAL, "output arrays hold fewer entries than wall nodes");
    std::vector<double> th(nw, theta0);
    if (theta_deg_host)
        for (int64_t i = 0; i < nw; ++i) th[i] = theta_deg_host[i];
    for (int64_t i = 0; i < nw; ++i)
        if (!(th[i] > 0.0 && th[i] < 180.0))
            return fail(LBM_EINVAL, "geometric formulation: angles must lie in (0, 180) degrees");
    std::vector<int32_t> code;
    std::vector<double> t;
    build_gf_stencils(*p, g, th.data(), code, t);
    // decode: the weight of each fluid stencil node, as the step applies it
    for (int64_t w = 0; w < nw; ++w)
        for (int k = 0; k < 2; ++k) {
            const int f = (code[w] >> (10 * k)) & 0x3FF;
            const int ia = f & 15, ib = (f >> 4) & 15;
            const bool fa = (f >> 8) & 1, fb = (f >> 9) & 1;
            const double tt = t[2 * w + k];
            int32_t* nd = nodes_host + 8 * w + 4 * k;
            double* wt = weights_host + 4 * w + 2 * k;
            nd[0] = ia % 3 - 1;
            nd[1] = ia / 3 - 1;
            nd[2] = ib % 3 - 1;
            nd[3] = ib / 3 - 1;
            wt[0] = fa ? (fb ? 1.0 - tt : 1.0) : 0.0;
            wt[1] = fb ? (fa ? tt : 1.0) : 0.0;
        }
    return LBM_OK;
}

int lbm_wall_nodes(lbm_ctx* c, int64_t* idx_host, int64_t* count) {
    if (!c || !count) return fail(LBM_EINVAL, "NULL argument");
    if (c->is_batch) return fail(LBM_EINVAL, "multi-case context: use the _case call");
    if (!c->have_geom) return fail(LBM_ESTATE, "no geometry set");
    *count = (int64_t)c->geom.walls.size();
    if (idx_host)
        for (size_t i = 0; i < c->geom.walls.size(); ++i) idx_host[i] = c->geom.walls[i];
    return LBM_OK;
}

int lbm_set_wetting(lbm_ctx* c, int32_t scheme, double scalar, const void* phi_dev,
                    const void* drho_dev, double phi0, double drho0) {
    if (!c) return fail(LBM_EINVAL, "NULL context");
    if (!c->is_batch && !c->have_geom)
        return fail(LBM_ESTATE, "set the geometry before the wetting scheme");
    if (scheme == LBM_WET_IVD) {
        if (!phi_dev && !(phi0 > 0)) return fail(LBM_EINVAL, "phi must be positive");
        if (!std::isfinite(drho0)) return fail(LBM_EINVAL, "drho must be finite");
        if (c->is_batch) {
            // every case gets the uniform values; per-case arrays go through
            // lbm_set_wetting_case
            if (phi_dev || drho_dev)
                return fail(LBM_EINVAL, "multi-case context: per-node arrays need lbm_set_wetting_case");
            const int64_t nw = c->n_wall_max;
            if (c->prec == 4) {
                LBM_HIP(launch_fill<float>((float*)c->phi, (float)phi0, nw, c->stream));
                LBM_HIP(launch_fill<float>((float*)c->drho, (float)drho0, nw, c->stream));
            } else {
                LBM_HIP(launch_fill<double>((double*)c->phi, phi0, nw, c->stream));
                LBM_HIP(launch_fill<double>((double*)c->drho, drho0, nw, c->stream));
            }
        } else {
            int rc = (c->prec == 4) ? fill_wetting<float>(c, phi_dev, drho_dev, phi0, drho0)
                                    : fill_wetting<double>(c, phi_dev, drho_dev, phi0, drho0);
            if (rc != LBM_OK) return rc;
        }
    } else if (scheme == LBM_WET_VD) {
        if (!(scalar > 0) || !(psi_argument(c->p, scalar) >= 0))
            return fail(LBM_EINVAL, "virtual density outside the range where psi is real");
    } else if (scheme == LBM_WET_SFI) {
        if (!std::isfinite(scalar)) return fail(LBM_EINVAL, "G_w must be finite");
    } else if (scheme == LBM_WET_GF) {
        if (c->is_batch || c->p.lattice != 9)
            return fail(LBM_EINVAL, "the geometric formulation is for D2Q9 single-lattice contexts");
        int rc = c->prec == 4 ? fill_gf<float>(c, phi_dev, scalar) : fill_gf<double>(c, phi_dev, scalar);
        if (rc != LBM_OK) return rc;
    } else {
        return fail(LBM_EINVAL, "unknown wetting scheme");
    }
    c->scheme = scheme;
    c->scalar = scalar;
    c->tw_dirty = true;     // the wall lists carry phi and drho
    c->graph_dirty = true;  // the scheme is part of the captured launch arguments
    return LBM_OK;
}

// A new state has been written in post-stream form (solid slots zero): into
// f[cur] for D2Q9, into f[cur ^ 1] for D3Q19, which keeps its populations in
// pull form (each slot holds the population its downwind neighbour gathers;
// aux.hip).  Convert it and clear the other buffer.
static int finish_state(lbm_ctx* c) {
    const int64_t QN = (int64_t)c->Q * c->N;
    if (c->prec == 4) {
        if (c->Q == 19) {
            LBM_HIP(launch_fill<float>((float*)c->f[c->cur], 0.f, QN, c->stream));
            LBM_HIP(launch_scatter3<float>(c->cls, (const float*)c->f[c->cur ^ 1],
                                           (float*)c->f[c->cur], c->p.nx, c->p.ny, c->p.nz,
                                           c->stream));
        }
        LBM_HIP(launch_fill<float>((float*)c->f[c->cur ^ 1], 0.f, QN, c->stream));
    } else {
        if (c->Q == 19) {
            LBM_HIP(launch_fill<double>((double*)c->f[c->cur], 0.0, QN, c->stream));
            LBM_HIP(launch_scatter3<double>(c->cls, (const double*)c->f[c->cur ^ 1],
                                            (double*)c->f[c->cur], c->p.nx, c->p.ny, c->p.nz,
                                            c->stream));
        }
        LBM_HIP(launch_fill<double>((double*)c->f[c->cur ^ 1], 0.0, QN, c->stream));
    }
    return LBM_OK;
}

// The current state as post-stream populations (Q x N, 0 on solid) into dst.
static int read_state(lbm_ctx* c, void* dst) {
    if (c->Q == 19 && c->prec == 4)
        LBM_HIP(launch_gather3<float>(c->cls, (const float*)c->f[c->cur], (float*)dst, c->p.nx,
                                      c->p.ny, c->p.nz, c->stream));
    else if (c->Q == 19)
        LBM_HIP(launch_gather3<double>(c->cls, (const double*)c->f[c->cur], (double*)dst, c->p.nx,
                                       c->p.ny, c->p.nz, c->stream));
    else
        LBM_HIP(hipMemcpyAsync(dst, c->f[c->cur], (size_t)c->Q * c->N * c->prec,
                               hipMemcpyDeviceToDevice, c->stream));
    return LBM_OK;
}

int lbm_set_fields(lbm_ctx* c, const void* rho_dev, const void* u_dev) {
    if (!c || !rho_dev) return fail(LBM_EINVAL, "NULL argument");
    if (c->is_batch) return fail(LBM_EINVAL, "multi-case context: use the _case call");
    if (!c->have_geom) return fail(LBM_ESTATE, "set the geometry before the fields");
    // D3Q19: equilibrium into the spare buffer, then into the pull form
    const int dst = c->Q == 19 ? c->cur ^ 1 : c->cur;
    if (c->prec == 4) {
        LBM_HIP(launch_init_eq<float>(c->Q, c->cls, (const float*)rho_dev, (const float*)u_dev,
                                      (float*)c->f[dst], c->N, c->stream));
    } else {
        LBM_HIP(launch_init_eq<double>(c->Q, c->cls, (const double*)rho_dev,
                                       (const double*)u_dev, (double*)c->f[dst], c->N,
                                       c->stream));
    }
    int rc = finish_state(c);
    if (rc != LBM_OK) return rc;
    LBM_HIP(launch_fill_i32(c->flag, 0, 4, c->stream));
    c->have_fields = true;
    c->domain_error = false;
    c->rho_valid = false;
    return LBM_OK;
}

int lbm_set_state(lbm_ctx* c, const void* f_dev) {
    if (!c || !f_dev) return fail(LBM_EINVAL, "NULL argument");
    if (c->is_batch) return fail(LBM_EINVAL, "multi-case context: use the _case call");
    if (!c->have_geom) return fail(LBM_ESTATE, "set the geometry before the state");
    const int64_t QN = (int64_t)c->Q * c->N;
    const int dst = c->Q == 19 ? c->cur ^ 1 : c->cur;
    LBM_HIP(hipMemcpyAsync(c->f[dst], f_dev, (size_t)QN * c->prec, hipMemcpyDeviceToDevice,
                           c->stream));
    if (c->prec == 4)
        LBM_HIP(launch_mask_solid<float>(c->Q, c->cls, (float*)c->f[dst], c->N, c->stream));
    else
        LBM_HIP(launch_mask_solid<double>(c->Q, c->cls, (double*)c->f[dst], c->N, c->stream));
    int rc = finish_state(c);
    if (rc != LBM_OK) return rc;
    LBM_HIP(launch_fill_i32(c->flag, 0, 4, c->stream));
    c->have_fields = true;
    c->domain_error = false;
    c->rho_valid = false;
    return LBM_OK;
}

int lbm_step(lbm_ctx* c, int64_t nsteps) {
    if (!c) return fail(LBM_EINVAL, "NULL context");
    if (nsteps < 0) return fail(LBM_EINVAL, "nsteps must be >= 0");
    if (!ready(c)) return fail(LBM_ESTATE, "geometry and fields must be set");
    if (c->domain_error) return fail(LBM_EDOMAIN, "a previous step left the psi domain");
    return c->prec == 4 ? run_steps<float>(c, nsteps) : run_steps<double>(c, nsteps);
}

int lbm_step_timed(lbm_ctx* c, int64_t nsteps, double* ms_total) {
    if (!c || !ms_total) return fail(LBM_EINVAL, "NULL argument");
    if (!ready(c)) return fail(LBM_ESTATE, "geometry and fields must be set");
    if (c->domain_error) return fail(LBM_EDOMAIN, "a previous step left the psi domain");
    LBM_HIP(hipEventRecord(c->ev0, c->stream));
    int rc = c->prec == 4 ? run_steps<float>(c, nsteps) : run_steps<double>(c, nsteps);
    if (rc != LBM_OK) return rc;
    LBM_HIP(hipEventRecord(c->ev1, c->stream));
    LBM_HIP(hipEventSynchronize(c->ev1));
    float ms = 0.f;
    LBM_HIP(hipEventElapsedTime(&ms, c->ev0, c->ev1));
    *ms_total = ms;
    return LBM_OK;
}

int lbm_get_fields(lbm_ctx* c, void* rho_dev, void* u_dev, void* f_dev) {
    if (!c) return fail(LBM_EINVAL, "NULL context");
    if (c->is_batch) return fail(LBM_EINVAL, "multi-case context: use the _case call");
    if (!c->have_geom || !c->have_fields) return fail(LBM_ESTATE, "geometry and fields must be set");
    if (rho_dev || u_dev) {
        int rc = c->prec == 4 ? launch_mode<float>(c, MODE_FIELDS, (float*)rho_dev, (float*)u_dev, nullptr)
                              : launch_mode<double>(c, MODE_FIELDS, (double*)rho_dev,
                                                    (double*)u_dev, nullptr);
        if (rc != LBM_OK) return rc;
    }
    return f_dev ? read_state(c, f_dev) : LBM_OK;
}

int lbm_get_diagnostics(lbm_ctx* c, lbm_diag* out) {
    if (!c || !out) return fail(LBM_EINVAL, "NULL argument");
    if (!ready(c)) return fail(LBM_ESTATE, "geometry and fields must be set");
    if (c->is_batch) {
        // combine the per-case reductions (fixed case order)
        lbm_diag acc{0.0, 0.0, 1e300, -1e300, 0, 0};
        int worst = LBM_OK;
        for (int32_t i = 0; i < (int32_t)c->cases.size(); ++i) {
            lbm_diag d;
            int rc = lbm_get_diagnostics_case(c, i, &d);
            if (rc != LBM_OK && rc != LBM_EDOMAIN) return rc;
            if (rc == LBM_EDOMAIN) worst = rc;
            acc.mass += d.mass;
            acc.max_u = d.max_u > acc.max_u ? d.max_u : acc.max_u;
            acc.rho_min = d.rho_min < acc.rho_min ? d.rho_min : acc.rho_min;
            acc.rho_max = d.rho_max > acc.rho_max ? d.rho_max : acc.rho_max;
            acc.flag |= d.flag;
            acc.n_fluid += d.n_fluid;
        }
        *out = acc;
        return worst == LBM_OK ? LBM_OK : fail(worst, "psi argument became negative or NaN");
    }
    int rc = c->prec == 4 ? launch_mode<float>(c, MODE_FIELDS, nullptr, nullptr, c->part)
                          : launch_mode<double>(c, MODE_FIELDS, nullptr, nullptr, c->part);
    if (rc != LBM_OK) return rc;
    LBM_HIP(launch_diag_final(c->part, c->nparts, c->diag_out, c->stream));
    double h[5];
    int32_t flag[4];
    LBM_HIP(hipMemcpyAsync(h, c->diag_out, sizeof h, hipMemcpyDeviceToHost, c->stream));
    LBM_HIP(hipMemcpyAsync(flag, c->flag, sizeof flag, hipMemcpyDeviceToHost, c->stream));
    LBM_HIP(hipStreamSynchronize(c->stream));
    out->mass = h[0];
    out->max_u = h[1];
    out->rho_min = h[2];
    out->rho_max = h[3];
    out->n_fluid = (int32_t)h[4];
    out->flag = flag[0];
    if (flag[0]) {
        c->domain_error = true;
        return fail(LBM_EDOMAIN, "psi argument became negative or NaN");
    }
    return LBM_OK;
}

int lbm_variant_count(int32_t lattice, int32_t precision) {
    if ((lattice != 9 && lattice != 19) || (precision != 4 && precision != 8))
        return fail(LBM_EINVAL, "lattice must be 9/19 and precision 4/8");
    return variant_count(lattice, precision);
}

int lbm_set_variant(lbm_ctx* c, int32_t variant) {
    if (!c) return fail(LBM_EINVAL, "NULL context");
    if (variant < 0 || variant >= ctx_variants(c)) return fail(LBM_EINVAL, "variant out of range");
    c->variant = variant;
    c->graph_dirty = true;
    return LBM_OK;
}

int lbm_get_variant(lbm_ctx* c, int32_t* variant) {
    if (!c || !variant) return fail(LBM_EINVAL, "NULL argument");
    *variant = c->variant;
    return LBM_OK;
}

int lbm_autotune(lbm_ctx* c, int64_t steps, void* save_dev, int32_t* best_out,
                 double* ms_per_variant) {
    if (!c) return fail(LBM_EINVAL, "NULL context");
    if (steps < 1) return fail(LBM_EINVAL, "steps must be >= 1");
    if (!ready(c)) return fail(LBM_ESTATE, "geometry and fields must be set");
    if (c->domain_error) return fail(LBM_EDOMAIN, "a previous step left the psi domain");
    const int nv = ctx_variants(c);
    const size_t fbytes = state_bytes(c);
    const char* cache = std::getenv("LBM_AUTOTUNE_CACHE");
    // the problem a cached choice applies to: lattice, precision, size, and
    // for a multi-case context the count and sizes of its cases (FNV-1a)
    uint64_t sizes = 1469598103934665603ull;
    for (const lbm_case& k : c->cases) {
        for (const uint64_t v : {(uint64_t)k.nx, (uint64_t)k.ny}) {
            sizes ^= v;
            sizes *= 1099511628211ull;
        }
    }
    char key[192];
    std::snprintf(key, sizeof key, "lattice=%d precision=%d nx=%d ny=%d nz=%d cases=%d sizes=%016llx",
                  c->p.lattice, c->p.precision, c->p.nx, c->p.ny, c->p.nz,
                  c->is_batch ? (int)c->cases.size() : 1, (unsigned long long)sizes);
    const size_t klen = std::strlen(key);
    if (cache && !ms_per_variant) {
        if (FILE* fp = std::fopen(cache, "r")) {
            char line[256];
            int found = -1;
            while (std::fgets(line, sizeof line, fp)) {
                // the whole key, then the separator before "variant="
                if (std::strncmp(line, key, klen) == 0 && line[klen] == ' ') {
                    const char* v = std::strstr(line, "variant=");
                    if (v) found = std::atoi(v + 8);
                }
            }
            std::fclose(fp);
            if (found >= 0 && found < nv) {
                c->variant = found;
                c->graph_dirty = true;
                if (best_out) *best_out = found;
                return LBM_OK;
            }
        }
    }
    if (save_dev)
        LBM_HIP(hipMemcpyAsync(save_dev, c->f[c->cur], fbytes, hipMemcpyDeviceToDevice, c->stream));
    const int keep = c->variant;
    int best = 0;
    double best_ms = 1e300;
    for (int v = 0; v < nv; ++v) {
        c->variant = v;
        int rc = c->prec == 4 ? run_steps<float>(c, 2) : run_steps<double>(c, 2);
        if (rc != LBM_OK) {
            c->variant = keep;
            return rc;
        }
        LBM_HIP(hipEventRecord(c->ev0, c->stream));
        rc = c->prec == 4 ? run_steps<float>(c, steps) : run_steps<double>(c, steps);
        if (rc != LBM_OK) {
            c->variant = keep;
            return rc;
        }
        LBM_HIP(hipEventRecord(c->ev1, c->stream));
        LBM_HIP(hipEventSynchronize(c->ev1));
        float ms = 0.f;
        LBM_HIP(hipEventElapsedTime(&ms, c->ev0, c->ev1));
        const double per = ms / (double)steps;
        if (ms_per_variant) ms_per_variant[v] = per;
        if (per < best_ms) {
            best_ms = per;
            best = v;
        }
    }
    if (save_dev) {
        LBM_HIP(hipMemcpyAsync(c->f[c->cur], save_dev, fbytes, hipMemcpyDeviceToDevice, c->stream));
        LBM_HIP(hipStreamSynchronize(c->stream));
        c->rho_valid = false;
    }
    c->variant = best;
    c->graph_dirty = true;
    if (best_out) *best_out = best;
    if (cache) {
        if (FILE* fp = std::fopen(cache, "a")) {
            std::fprintf(fp, "%s variant=%d ms=%.6f\n", key, best, best_ms);
            std::fclose(fp);
        }
    }
    return LBM_OK;
}

size_t lbm_autotune_save_bytes(lbm_ctx* c) { return c ? state_bytes(c) : 0; }

size_t lbm_batch_workspace_bytes(const lbm_params* p, int32_t ncases, const int32_t* nx,
                                 const int32_t* ny, const int64_t* n_wall_max) {
    if (check_batch_args(p, ncases, nx, ny, n_wall_max) != LBM_OK) return 0;
    return layout_batch(*p, ncases, nx, ny, n_wall_max, nullptr);
}

int lbm_create_batch(const lbm_params* p, int32_t ncases, const int32_t* nx, const int32_t* ny,
                     const int64_t* n_wall_max, void* stream, void* workspace, size_t ws_bytes,
                     lbm_ctx** out) {
    if (!out) return fail(LBM_EINVAL, "out is NULL");
    *out = nullptr;
    int rc = check_batch_args(p, ncases, nx, ny, n_wall_max);
    if (rc != LBM_OK) return rc;
    const size_t need = layout_batch(*p, ncases, nx, ny, n_wall_max, nullptr);
    if (!workspace || ws_bytes < need)
        return fail(LBM_ENOMEM, "workspace needs " + std::to_string(need) + " bytes");
    if (((uintptr_t)workspace & 255) != 0) return fail(LBM_EINVAL, "workspace must be 256-byte aligned");
    lbm_ctx* c = new (std::nothrow) lbm_ctx();
    if (!c) return fail(LBM_ENOMEM, "host allocation failed");
    c->p = *p;
    c->p.nx = c->p.ny = c->p.nz = 0;
    c->Q = 9;
    c->D = 2;
    c->prec = p->precision;
    c->stream = (hipStream_t)stream;
    c->ws = workspace;
    c->ws_bytes = ws_bytes;
    c->is_batch = true;
    layout_batch(*p, ncases, nx, ny, n_wall_max, c);
    if (!create_timing_events(c)) {
        lbm_destroy(c);  // releases whichever event was created
        return fail(LBM_EDEVICE, "hipEventCreate failed");
    }
    rc = c->prec == 4 ? upload_cases<float>(c) : upload_cases<double>(c);
    if (rc != LBM_OK) {
        lbm_destroy(c);
        return rc;
    }
    *out = c;
    return LBM_OK;
}

int lbm_batch_cases(lbm_ctx* c, int32_t* ncases) {
    if (!c || !ncases) return fail(LBM_EINVAL, "NULL argument");
    *ncases = c->is_batch ? (int32_t)c->cases.size() : 1;
    return LBM_OK;
}

static int case_of(lbm_ctx* c, int32_t i, lbm_case** k) {
    if (!c) return fail(LBM_EINVAL, "NULL context");
    if (!c->is_batch) return fail(LBM_EINVAL, "not a multi-case context");
    if (i < 0 || i >= (int32_t)c->cases.size()) return fail(LBM_EINVAL, "case index out of range");
    *k = &c->cases[i];
    return LBM_OK;
}

int lbm_set_geometry_case(lbm_ctx* c, int32_t i, const uint8_t* solid_host) {
    lbm_case* k;
    int rc = case_of(c, i, &k);
    if (rc != LBM_OK) return rc;
    if (!solid_host) return fail(LBM_EINVAL, "NULL geometry");
    lbm_params q = c->p;
    q.nx = k->nx;
    q.ny = k->ny;
    q.nz = 1;
    Geometry g;
    build_geometry(q, solid_host, g);
    if ((int64_t)g.walls.size() > k->n_wall_max)
        return fail(LBM_EINVAL, "case geometry has more wall nodes than its n_wall_max");
    if (g.n_fluid == 0) return fail(LBM_EINVAL, "case geometry has no fluid node");
    // rows `pitch` apart; the columns past nx are solid with no wall entry
    LBM_HIP(hipMemsetAsync(c->cls + k->node_off, CLS_SOLID, (size_t)k->NP, c->stream));
    LBM_HIP(hipMemsetAsync(c->widx + k->node_off, 0xFF, (size_t)k->NP * 4, c->stream));
    LBM_HIP(hipMemcpy2DAsync(c->cls + k->node_off, (size_t)k->pitch, g.cls.data(), (size_t)k->nx,
                             (size_t)k->nx, (size_t)k->ny, hipMemcpyHostToDevice, c->stream));
    LBM_HIP(hipMemcpy2DAsync(c->widx + k->node_off, (size_t)k->pitch * 4, g.widx.data(),
                             (size_t)k->nx * 4, (size_t)k->nx * 4, (size_t)k->ny,
                             hipMemcpyHostToDevice, c->stream));
    LBM_HIP(hipStreamSynchronize(c->stream));
    const int64_t nw = (int64_t)g.walls.size();
    if (c->prec == 4) {
        LBM_HIP(launch_fill<float>((float*)c->phi + k->wall_off, 1.f, nw, c->stream));
        LBM_HIP(launch_fill<float>((float*)c->drho + k->wall_off, 0.f, nw, c->stream));
    } else {
        LBM_HIP(launch_fill<double>((double*)c->phi + k->wall_off, 1.0, nw, c->stream));
        LBM_HIP(launch_fill<double>((double*)c->drho + k->wall_off, 0.0, nw, c->stream));
    }
    k->geom = std::move(g);
    k->have_geom = true;
    k->have_fields = false;
    c->tw_dirty = true;
    return LBM_OK;
}

int lbm_wall_nodes_case(lbm_ctx* c, int32_t i, int64_t* idx_host, int64_t* count) {
    lbm_case* k;
    int rc = case_of(c, i, &k);
    if (rc != LBM_OK) return rc;
    if (!count) return fail(LBM_EINVAL, "NULL count");
    if (!k->have_geom) return fail(LBM_ESTATE, "no geometry set for this case");
    *count = (int64_t)k->geom.walls.size();
    if (idx_host)
        for (size_t j = 0; j < k->geom.walls.size(); ++j) idx_host[j] = k->geom.walls[j];
    return LBM_OK;
}

int lbm_set_wetting_case(lbm_ctx* c, int32_t i, const void* phi_dev, const void* drho_dev,
                         double phi0, double drho0) {
    lbm_case* k;
    int rc = case_of(c, i, &k);
    if (rc != LBM_OK) return rc;
    if (!k->have_geom) return fail(LBM_ESTATE, "no geometry set for this case");
    if (!phi_dev && !(phi0 > 0)) return fail(LBM_EINVAL, "phi must be positive");
    const int64_t nw = (int64_t)k->geom.walls.size();
    if (nw == 0) return LBM_OK;
    const size_t bytes = (size_t)nw * c->prec;
    char* ph = (char*)c->phi + k->wall_off * c->prec;
    char* dr = (char*)c->drho + k->wall_off * c->prec;
    if (phi_dev) LBM_HIP(hipMemcpyAsync(ph, phi_dev, bytes, hipMemcpyDeviceToDevice, c->stream));
    else if (c->prec == 4) LBM_HIP(launch_fill<float>((float*)ph, (float)phi0, nw, c->stream));
    else LBM_HIP(launch_fill<double>((double*)ph, phi0, nw, c->stream));
    if (drho_dev) LBM_HIP(hipMemcpyAsync(dr, drho_dev, bytes, hipMemcpyDeviceToDevice, c->stream));
    else if (c->prec == 4) LBM_HIP(launch_fill<float>((float*)dr, (float)drho0, nw, c->stream));
    else LBM_HIP(launch_fill<double>((double*)dr, drho0, nw, c->stream));
    c->tw_dirty = true;  // the wall lists carry copies of phi and drho
    return LBM_OK;
}

int lbm_set_fields_case(lbm_ctx* c, int32_t i, const void* rho_dev, const void* u_dev) {
    lbm_case* k;
    int rc = case_of(c, i, &k);
    if (rc != LBM_OK) return rc;
    if (!rho_dev) return fail(LBM_EINVAL, "NULL rho");
    if (!k->have_geom) return fail(LBM_ESTATE, "set the case geometry before its fields");
    const int64_t QN = 9 * k->NP;
    if (c->prec == 4) {
        LBM_HIP(launch_init_eq<float>(9, c->cls + k->node_off, (const float*)rho_dev,
                                      (const float*)u_dev, (float*)c->f[c->cur] + k->f_off, k->NP,
                                      c->stream, k->nx, k->pitch));
        LBM_HIP(launch_fill<float>((float*)c->f[c->cur ^ 1] + k->f_off, 0.f, QN, c->stream));
    } else {
        LBM_HIP(launch_init_eq<double>(9, c->cls + k->node_off, (const double*)rho_dev,
                                       (const double*)u_dev, (double*)c->f[c->cur] + k->f_off,
                                       k->NP, c->stream, k->nx, k->pitch));
        LBM_HIP(launch_fill<double>((double*)c->f[c->cur ^ 1] + k->f_off, 0.0, QN, c->stream));
    }
    LBM_HIP(launch_fill_i32(c->flag, 0, 4, c->stream));
    k->have_fields = true;
    c->domain_error = false;
    return LBM_OK;
}

int lbm_get_fields_case(lbm_ctx* c, int32_t i, void* rho_dev, void* u_dev, void* f_dev) {
    lbm_case* k;
    int rc = case_of(c, i, &k);
    if (rc != LBM_OK) return rc;
    if (!k->have_geom || !k->have_fields) return fail(LBM_ESTATE, "case geometry and fields must be set");
    if (rho_dev || u_dev) {
        rc = c->prec == 4 ? case_fields_launch<float>(c, *k, (float*)rho_dev, (float*)u_dev, nullptr)
                          : case_fields_launch<double>(c, *k, (double*)rho_dev, (double*)u_dev, nullptr);
        if (rc != LBM_OK) return rc;
    }
    if (f_dev)  // the 9 planes' rows, dense
        LBM_HIP(hipMemcpy2DAsync(f_dev, (size_t)k->nx * c->prec,
                                 (char*)c->f[c->cur] + k->f_off * c->prec,
                                 (size_t)k->pitch * c->prec, (size_t)k->nx * c->prec,
                                 (size_t)9 * k->ny, hipMemcpyDeviceToDevice, c->stream));
    return LBM_OK;
}

int lbm_get_diagnostics_case(lbm_ctx* c, int32_t i, lbm_diag* out) {
    lbm_case* k;
    int rc = case_of(c, i, &k);
    if (rc != LBM_OK) return rc;
    if (!out) return fail(LBM_EINVAL, "NULL output");
    if (!k->have_geom || !k->have_fields) return fail(LBM_ESTATE, "case geometry and fields must be set");
    rc = c->prec == 4 ? case_fields_launch<float>(c, *k, nullptr, nullptr, c->part)
                      : case_fields_launch<double>(c, *k, nullptr, nullptr, c->part);
    if (rc != LBM_OK) return rc;
    const int parts = c->prec == 4 ? grid2d_blocks<float>(k->nx, k->ny, 0)
                                   : grid2d_blocks<double>(k->nx, k->ny, 0);
    LBM_HIP(launch_diag_final(c->part, parts, c->diag_out, c->stream));
    double h[5];
    int32_t flag[4];
    LBM_HIP(hipMemcpyAsync(h, c->diag_out, sizeof h, hipMemcpyDeviceToHost, c->stream));
    LBM_HIP(hipMemcpyAsync(flag, c->flag, sizeof flag, hipMemcpyDeviceToHost, c->stream));
    LBM_HIP(hipStreamSynchronize(c->stream));
    *out = lbm_diag{h[0], h[1], h[2], h[3], flag[0], (int32_t)h[4]};
    if (flag[0]) {
        c->domain_error = true;
        return fail(LBM_EDOMAIN, "psi argument became negative or NaN");
    }
    return LBM_OK;
}

int lbm_set_graph_steps(lbm_ctx* c, int64_t steps) {
    if (!c) return fail(LBM_EINVAL, "NULL context");
    if (steps < 0) return fail(LBM_EINVAL, "steps must be >= 0");
    drop_graph(c);
    c->graph_steps = (steps + 1) / 2 * 2;  // even: a replay keeps the buffer parity
    c->graph_dirty = true;
    return LBM_OK;
}

size_t lbm_adjoint_workspace_bytes(lbm_ctx* c, int64_t K) {
    if (!c || K < 1 || c->is_batch || c->p.lattice != 9) return 0;
    return adj_layout(c, K).total;
}

int lbm_step_ckpt(lbm_ctx* c, int64_t T, int64_t K, void* ckpt_dev) {
    if (!c || !ckpt_dev) return fail(LBM_EINVAL, "NULL argument");
    if (T < 0 || K < 1) return fail(LBM_EINVAL, "need T >= 0 and K >= 1");
    if (c->is_batch) return fail(LBM_EINVAL, "checkpointed stepping is for single lattices");
    if (!ready(c)) return fail(LBM_ESTATE, "geometry and fields must be set");
    if (c->domain_error) return fail(LBM_EDOMAIN, "a previous step left the psi domain");
    const size_t state = (size_t)c->Q * c->N * c->prec;
    for (int64_t t = 0, sg = 0; t < T; t += K, ++sg) {
        // checkpoints hold post-stream populations, as lbm_get_fields writes them
        int rc0 = read_state(c, (char*)ckpt_dev + (size_t)sg * state);
        if (rc0 != LBM_OK) return rc0;
        const int64_t n = (T - t) < K ? (T - t) : K;
        int rc = c->prec == 4 ? run_steps<float>(c, n) : run_steps<double>(c, n);
        if (rc != LBM_OK) return rc;
    }
    return LBM_OK;
}

int lbm_adjoint(lbm_ctx* c, int32_t seed_kind, const void* seed_dev, int64_t T, int64_t K,
                const void* ckpt_dev, void* work_dev, size_t work_bytes, void* grad_phi_dev,
                void* grad_drho_dev, void* lam0_dev) {
    return adjoint_entry(c, seed_kind, seed_dev, T, K, ckpt_dev, work_dev, work_bytes,
                         grad_phi_dev, grad_drho_dev, lam0_dev);
}

}  // extern "C"
