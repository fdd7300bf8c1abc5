/*
 * lbm.h -- C ABI of the MI355X (gfx950) library for the pseudopotential
 * multiphase lattice Boltzmann step with contact angles on curved walls
 * (Li, Yu & Luo, "Implementation of contact angles in the pseudopotential
 * lattice Boltzmann simulations with curved boundaries").
 *
 * One time step (Sec. II A, Sec. III B, Sec. IV A):
 *   rho = sum_a f_a (Eq. 4) -> psi(rho) from the equation of state (Eq. 6)
 *   -> virtual density of the solid nodes next to the fluid: the improved
 *      local scheme (Eqs. 16-17 with the limiter rho_g <= rho_w <= rho_l),
 *      the constant virtual density, or no pseudopotential in the solid for
 *      the solid-fluid interaction (Eq. 8)
 *   -> force F = F_m (Eq. 5) [+ F_ads (Eq. 8)] [+ body force]
 *   -> u (Eq. 4) -> MRT collision in moment space with the forcing of Eq. 7
 *      (Eq. 2) -> streaming (Eq. 3) with halfway bounce-back at the
 *      staircase wall (Fig. 3).
 *
 * Conventions
 *  - Lattice units: dx = dt = 1, c = 1, cs^2 = 1/3.
 *  - Node index n = x + nx*(y + ny*z), x fastest; every axis is periodic.
 *    Walls (cylinders, spheres, plates) are solid nodes.
 *  - Populations are structure-of-arrays f[a*N + n] (N = nx*ny*nz) in the
 *    velocity order: D2Q9 rest, +x, +y, -x, -y, (1,1), (-1,1), (-1,-1),
 *    (1,-1); D3Q19 rest, +x, -x, +y, -y, +z, -z, (1,1,0), (-1,-1,0),
 *    (1,-1,0), (-1,1,0), (1,0,1), (-1,0,-1), (1,0,-1), (-1,0,1), (0,1,1),
 *    (0,-1,-1), (0,1,-1), (0,-1,1).  The state is the post-streaming
 *    population set at integer time t.
 *  - Real-valued device arrays are in the context precision (float for
 *    precision 4, double for precision 8).
 *  - "dev" pointers are device memory; "host" pointers are host memory.
 *    Device pointers passed in are borrowed for the duration of the call
 *    only (reads and writes are ordered on the context stream).
 *  - Every call returns LBM_OK (0) or a negative error code; no C++
 *    exception crosses this interface.  lbm_last_error() gives a
 *    thread-local message for the last failure.
 *  - The library never allocates device memory: all device storage lives
 *    in the caller-owned workspace given to lbm_create/lbm_create_batch,
 *    apart from the fixed scratch array of lbm_adjoint_noalloc (a device
 *    global of the library, LBM_NOALLOC_SCRATCH_BYTES per GPU).
 */
#ifndef LBM_H
#define LBM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    LBM_OK = 0,
    LBM_EINVAL = -1,  /* invalid argument or parameter */
    LBM_ENOMEM = -2,  /* workspace too small, or host allocation failed */
    LBM_EDOMAIN = -3, /* psi argument negative or NaN (Eq. 6 undefined) */
    LBM_ESTATE = -4,  /* call out of order (e.g. step before geometry) */
    LBM_EDEVICE = -5  /* HIP runtime error */
};

enum { LBM_EOS_CS = 0, LBM_EOS_PR = 1 };
enum { LBM_WET_IVD = 0, LBM_WET_VD = 1, LBM_WET_SFI = 2, LBM_WET_GF = 3 };

/* Model parameters, copied at create.
 *  lattice     9 (D2Q9) or 19 (D3Q19)
 *  precision   4 (float) or 8 (double)
 *  nx, ny, nz  lattice size (nz = 1 for D2Q9; ny, nz <= 65535 for D3Q19;
 *              nx*ny*nz <= 4e9)
 *  tau[k]      relaxation time of moment row k (Eq. 2); all > 0.5.  Row
 *              order is that of the relaxation matrix of Eq. 2: D2Q9
 *              (rho, e, eps, jx, qx, jy, qy, pxx, pxy); D3Q19 (rho, e, eps,
 *              jx, qx, jy, qy, jz, qz, 3pxx, 3pixx, pww, piww, pxy, pyz,
 *              pxz, mx, my, mz).  nu = (tau_nu - 0.5)/3.  Rows of one
 *              moment group share one rate (isotropy): jx=jy(=jz),
 *              qx=qy(=qz), pxx=pxy (2-D) / 3pxx=pww=pxy=pyz=pxz (3-D),
 *              3pixx=piww, mx=my=mz; a vector that breaks this is rejected.
 *  eos         LBM_EOS_CS: p = rho R T (1+h+h^2-h^3)/(1-h)^3 - a rho^2,
 *              h = b rho / 4 (Carnahan-Starling).  LBM_EOS_PR: Eq. 18 with
 *              acentric factor eos_omega and Tc = (0.0778/0.45724)(a/b)/R.
 *  eos_T       absolute temperature
 *  G           interaction strength of Eqs. 5-6 (the paper uses -1)
 *  sigma       thermodynamic-consistency constant of Eq. 7
 *  body_force  constant force density added to F (e.g. Poiseuille drive)
 *  rho_g,rho_l limiter bounds of the improved virtual density (Sec. III B):
 *              the coexisting gas and liquid densities. rho_g < rho_l. */
typedef struct {
    int32_t lattice;
    int32_t precision;
    int32_t nx, ny, nz;
    int32_t eos;
    double tau[19];
    double eos_a, eos_b, eos_R, eos_T, eos_omega;
    double G;
    double sigma;
    double body_force[3];
    double rho_g, rho_l;
} lbm_params;

/* Diagnostics of the current state (reductions over the fluid nodes). */
typedef struct {
    double mass;    /* sum over fluid nodes of their populations (Eq. 4), each
                       population added in double */
    double max_u;   /* max |u| over fluid nodes (spurious currents) */
    double rho_min; /* min rho over fluid nodes */
    double rho_max; /* max rho over fluid nodes */
    int32_t flag;   /* nonzero: a step met a psi argument < 0 or NaN */
    int32_t n_fluid;
} lbm_diag;

typedef struct lbm_ctx lbm_ctx;

/* ---------------------------------------------------------------- status */
const char* lbm_version(void);
const char* lbm_status_string(int code);
/* Message for the last failing call on this thread ("" if none). */
const char* lbm_last_error(void);

/* Host-only check of a parameter set (no device needed).  Returns
 * LBM_EINVAL with a message for: lattice not 9/19, precision not 4/8, a
 * non-positive size, nz != 1 for D2Q9, tau <= 0.5, unequal tau within a
 * moment group, non-positive EOS constants, rho_g >= rho_l or rho_g <= 0. */
int lbm_validate_params(const lbm_params* p);

/* ------------------------------------------------------- thermodynamics */
/* Host helpers for the equation of state (Eq. 6, Eq. 18).  Critical point
 * (Tc and the density there); for PR, Tc follows from a, b, R. */
int lbm_eos_critical(int32_t eos, double a, double b, double R, double omega,
                     double* Tc, double* rhoc);
/* Maxwell equal-area coexistence densities at p->eos_T (< Tc). */
int lbm_eos_coexistence(const lbm_params* p, double* rho_g, double* rho_l);
/* Pressure of the EOS and the psi of Eq. 6 at one density (host). */
int lbm_eos_eval(const lbm_params* p, double rho, double* p_eos, double* psi);

/* ------------------------------------------------------------ lifetime */
/* Bytes of device workspace a context of these parameters needs, with room
 * for up to n_wall_max wall nodes (solid nodes adjacent to fluid).  0 if
 * the parameters are invalid. */
size_t lbm_workspace_bytes(const lbm_params* p, int64_t n_wall_max);

/* Create a context for one lattice of the problem Sec. IV A states (size,
 * periodic box, equation of state and temperature of Eq. 6 / Eq. 18,
 * relaxation times of Eq. 2, the constant sigma of Eq. 7, interaction
 * strength G of Eq. 5, limiter bounds of Sec. III B).  stream: a
 * hipStream_t (NULL = default stream) on which every launch and copy of
 * this context is ordered.  workspace: device
 * memory of ws_bytes >= lbm_workspace_bytes(p, n_wall_max), owned by the
 * caller and kept alive (and not touched) until lbm_destroy.  Errors:
 * LBM_EINVAL (parameters), LBM_ENOMEM (workspace too small),
 * LBM_EDEVICE. */
int lbm_create(const lbm_params* p, void* stream, void* workspace,
               size_t ws_bytes, int64_t n_wall_max, lbm_ctx** out);
/* Free the host-side context (the workspace stays the caller's). */
int lbm_destroy(lbm_ctx* ctx);

/* ------------------------------------------------------------- problem */
/* Solid geometry (Sec. IV, Fig. 3): solid_host[n] = 1 for solid, 0 for
 * fluid, N bytes of host memory, read during the call.  Builds the node
 * classes and the list of wall nodes (solid nodes with a fluid neighbour in
 * the Eq. 5 stencil, increasing n) and uploads them; blocks until the
 * upload is done.  Resets wetting to the improved scheme with phi = 1,
 * drho = 0 and marks the fields unset.  Errors: LBM_EINVAL (more than
 * n_wall_max wall nodes, or no fluid node). */
int lbm_set_geometry(lbm_ctx* ctx, const uint8_t* solid_host);

/* Number of wall nodes and (if idx_host != NULL) their node indices in the
 * order used by the per-wall-node arrays of lbm_set_wetting/lbm_adjoint. */
int lbm_wall_nodes(lbm_ctx* ctx, int64_t* idx_host, int64_t* count);

/* Host query (no device, no context): the interpolation stencils of the
 * geometric formulation (Sec. III A, Eqs. 11, 13-15) that a D2Q9 context
 * with this solid mask and these angles steps with.  For wall node w (the
 * order of lbm_wall_nodes) and characteristic point k (0: n_s turned by
 * +(90 deg - theta_a), 1: by -(90 deg - theta_a)): nodes_host[8w+4k+2i],
 * nodes_host[8w+4k+2i+1] are the x, y offsets of stencil node i (0, 1)
 * from the wall node and weights_host[4w+2k+i] its weight in the density
 * of the point.  Only fluid nodes carry weight; the weights of a point sum
 * to 1, or are both 0 when the point is void.  theta_deg_host: one angle in
 * degrees per wall node, or NULL for theta0.  *count receives the number of
 * wall nodes; with both output arrays NULL nothing else is written,
 * otherwise both must hold cap >= count entries.  Errors: LBM_EINVAL
 * (parameters, lattice not D2Q9, an angle outside (0, 180), cap too
 * small). */
int lbm_gf_stencils(const lbm_params* p, const uint8_t* solid_host, const double* theta_deg_host,
                    double theta0, int64_t cap, int64_t* count, int32_t* nodes_host,
                    double* weights_host);

/* Contact-angle scheme.
 *  LBM_WET_IVD  improved virtual density (Eqs. 16-17): per wall node b,
 *               rho_w = clamp(phi_b * rho_ave - drho_b, rho_g, rho_l), with
 *               rho_ave the w-weighted mean density of the fluid neighbours.
 *               phi_dev/drho_dev: device arrays of count wall entries in the
 *               context precision, or NULL for the uniform phi0/drho0.
 *  LBM_WET_VD   constant virtual density rho_w = scalar on every wall node.
 *  LBM_WET_SFI  solid-fluid interaction (Eq. 8) with G_w = scalar; the
 *               solid carries psi = 0.
 *  LBM_WET_GF   curved geometric formulation (Sec. III A, Eqs. 11, 13-15),
 *               D2Q9 single-lattice contexts only: each wall node takes
 *               the max (theta_a <= 90 deg) or min of the densities at the
 *               two points D1, D2 where the characteristic lines through it
 *               (the solid normal of Eq. 13 with the weights of Eq. 14,
 *               turned by +-(90 deg - theta_a), Eq. 15) first cross a mesh
 *               line, interpolated linearly between that line's two fluid
 *               nodes.  theta_a in degrees: scalar for every wall node, or
 *               phi_dev = device array of count wall entries in the context
 *               precision (drho_dev ignored).  The stencils are built on the
 *               host during the call (it copies phi_dev to the host).
 * Errors: LBM_ESTATE (no geometry), LBM_EINVAL (unknown scheme, phi <= 0,
 * VD density outside the range where Eq. 6 is real, GF angle outside
 * (0, 180) or GF on a D3Q19 or multi-case context). */
int lbm_set_wetting(lbm_ctx* ctx, int32_t scheme, double scalar,
                    const void* phi_dev, const void* drho_dev, double phi0,
                    double drho0);

/* Initial state f = f_eq(rho, u) on fluid nodes (0 on solid).  rho_dev: N
 * reals; u_dev: D*N reals ([D][N]) or NULL for rest.  Errors: LBM_ESTATE
 * (no geometry).  Densities are not checked against the range where Eq. 6
 * is real: the next step raises the device domain flag, which the next
 * lbm_get_diagnostics reports as LBM_EDOMAIN.  Clears that flag and the
 * sticky error. */
int lbm_set_fields(lbm_ctx* ctx, const void* rho_dev, const void* u_dev);
/* Raw state: f_dev holds Q*N reals ([Q][N]) of post-stream populations,
 * as lbm_get_fields and lbm_step_ckpt write them (checkpoint restore).
 * Values on solid nodes are ignored.  D3Q19 contexts keep their state in
 * pull form internally (each node's slots hold its post-collision
 * populations, and a wall slot holds its fluid neighbour's bounce-back);
 * this call and lbm_get_fields convert. */
int lbm_set_state(lbm_ctx* ctx, const void* f_dev);

/* --------------------------------------------------------------- steps */
/* Advance nsteps >= 0 time steps, asynchronously on the context stream.
 * One step is Eq. 4 (density), Eq. 6 (psi), the wall virtual density of
 * the scheme (Eqs. 16-17, Eq. 11, or none for Eq. 8), Eq. 5 (+ Eq. 8 and
 * the body force), Eq. 2 with the forcing of Eq. 7, and Eq. 3 streaming
 * with halfway bounce-back at the staircase wall (Fig. 3).
 * Errors: LBM_ESTATE (geometry or fields unset), LBM_EDOMAIN if a previous
 * diagnostics call found the domain flag set (sticky until new fields). */
int lbm_step(lbm_ctx* ctx, int64_t nsteps);

/* Macroscopic fields of the current state (Eq. 4: rho = sum_a f_a and
 * u = (sum_a e_a f_a + F/2) / rho with the total force F of the step),
 * written stream-ordered to
 * caller device arrays (each may be NULL): rho_dev N reals (fluid: density;
 * wall nodes: their virtual density, 0 under SFI; other solid: 0), u_dev
 * D*N reals ([D][N], 0 on solid), f_dev Q*N reals (the post-stream
 * populations, 0 on solid). */
int lbm_get_fields(lbm_ctx* ctx, void* rho_dev, void* u_dev, void* f_dev);

/* Reductions over the current state (the quantities Figs. 10-11 compare:
 * maximum spurious current, extreme fluid densities; plus the mass of
 * Eq. 4 summed over the fluid); synchronises the context stream.
 * Returns LBM_EDOMAIN (and sets the sticky error) if the device domain flag
 * is set. */
int lbm_get_diagnostics(lbm_ctx* ctx, lbm_diag* host_out);

/* lbm_step followed by a host wait, timed with HIP events recorded on the
 * context stream right before the first and after the last step launch;
 * ms_total receives the elapsed time of the nsteps launches.  The events
 * carry no system-scope fence: read results through the library's calls or
 * stream-ordered copies, as after lbm_step. */
int lbm_step_timed(lbm_ctx* ctx, int64_t nsteps, double* ms_total);

/* ------------------------------------------------------------ tuning */
/* The step kernel exists in several tile shapes (and workgroup orderings;
 * for D3Q19 also with or without a separate density pass).  Number of
 * variants for a lattice/precision; LBM_EINVAL if unknown.  A lattice whose
 * population array exceeds 4 GiB runs one shape with 64-bit addressing
 * whatever the variant. */
int lbm_variant_count(int32_t lattice, int32_t precision);
int lbm_set_variant(lbm_ctx* ctx, int32_t variant);
int lbm_get_variant(lbm_ctx* ctx, int32_t* variant);

/* Autotuner: times `steps` steps of every variant on the current problem
 * (HIP events on the context stream, after 2 warm-up steps each) and keeps
 * the fastest.  save_dev: device buffer of lbm_autotune_save_bytes(ctx)
 * bytes used to save and restore the state, so that tuning leaves the
 * fields unchanged (scratch: it holds the context's internal form, pull
 * form for D3Q19, rows padded to whole cache lines in a multi-case
 * context); with NULL the state advances by nvariants*(steps+2) steps.  ms_per_variant (host,
 * nullable, lbm_variant_count entries) receives the mean step time of each.
 * If the environment variable LBM_AUTOTUNE_CACHE names a file, a cached
 * choice for the same lattice, precision and size (for a multi-case
 * context: the same number and sizes of cases) is used without timing
 * (unless ms_per_variant is requested; the last matching line wins), and
 * new results are appended as one line each. */
int lbm_autotune(lbm_ctx* ctx, int64_t steps, void* save_dev, int32_t* best_out,
                 double* ms_per_variant);
/* Size in bytes of lbm_autotune's save buffer for this context: Q * N
 * reals for a single lattice, the whole population arena of a multi-case
 * context; 0 for a NULL context. */
size_t lbm_autotune_save_bytes(lbm_ctx* ctx);

/* ------------------------------------------------------ graph replay */
/* Replay `steps` steps (rounded up to even) as one HIP graph: lbm_step(n)
 * then issues n / steps graph launches plus plain launches for the rest.
 * The graph is captured on a stream of the library's own and launched on
 * the context stream; it is captured again after a change of wetting
 * scheme or kernel variant.  0 (the default) turns graphs off.  Captures
 * contain kernel launches only. */
int lbm_set_graph_steps(lbm_ctx* ctx, int64_t steps);

/* ------------------------------------------------- many lattices at once */
/* A multi-case context advances ncases independent D2Q9 lattices of their
 * own sizes (nx[i] x ny[i], room for n_wall_max[i] wall nodes) in one
 * launch per step: every workgroup looks up its (case, tile) in a table.
 * The parameter block is shared (its nx, ny, nz are ignored); geometry,
 * wetting parameters and fields are per case.  lbm_step, lbm_step_timed,
 * lbm_set_wetting (scheme and uniform values for all cases),
 * lbm_set_graph_steps, lbm_set_variant, lbm_autotune and
 * lbm_get_diagnostics (totals over the cases) accept such a context; the
 * single-lattice geometry/fields calls return LBM_EINVAL for it.  Inside
 * the context each case's rows start on 128-byte boundaries (the width is
 * padded to whole lines); the per-case calls take and give dense arrays.
 * Each case's populations, rows padded, must stay below 4 GiB. */
size_t lbm_batch_workspace_bytes(const lbm_params* p, int32_t ncases, const int32_t* nx,
                                 const int32_t* ny, const int64_t* n_wall_max);
int lbm_create_batch(const lbm_params* p, int32_t ncases, const int32_t* nx, const int32_t* ny,
                     const int64_t* n_wall_max, void* stream, void* workspace, size_t ws_bytes,
                     lbm_ctx** out);
int lbm_batch_cases(lbm_ctx* ctx, int32_t* ncases);
/* Per-case versions of the single-lattice calls (case index i). */
int lbm_set_geometry_case(lbm_ctx* ctx, int32_t i, const uint8_t* solid_host);
int lbm_wall_nodes_case(lbm_ctx* ctx, int32_t i, int64_t* idx_host, int64_t* count);
/* Improved-virtual-density parameters of one case (count entries each, or
 * NULL for the uniform phi0 / drho0). */
int lbm_set_wetting_case(lbm_ctx* ctx, int32_t i, const void* phi_dev, const void* drho_dev,
                         double phi0, double drho0);
int lbm_set_fields_case(lbm_ctx* ctx, int32_t i, const void* rho_dev, const void* u_dev);
int lbm_get_fields_case(lbm_ctx* ctx, int32_t i, void* rho_dev, void* u_dev, void* f_dev);
int lbm_get_diagnostics_case(lbm_ctx* ctx, int32_t i, lbm_diag* host_out);

/* ------------------------------------------------------------ adjoint */
/* Discrete adjoint of the D2Q9 step (single lattices), for gradients of a
 * loss on the state at time T with respect to the per-wall-node parameters
 * phi_b, drho_b of the improved virtual-density scheme (Eq. 16).
 *
 * lbm_step_ckpt: advance T steps like lbm_step, storing the state at times
 * 0, K, 2K, ... (< T) into ckpt_dev (caller-owned device memory of
 * ceil(T/K) * Q*N reals), as post-stream populations: each checkpoint is
 * what lbm_get_fields writes and what lbm_set_state takes.
 *
 * lbm_adjoint: with the checkpoints of that run (taken under the same
 * geometry and wetting parameters), computes
 *   seed_kind 0: seed_dev = dL/drho(T) (N reals; only fluid entries used),
 *   seed_kind 1: seed_dev = dL/df(T) (Q*N reals),
 * and writes dL/dphi and dL/ddrho (wall-list order, ctx precision; each
 * nullable) and, if lam0_dev != NULL, dL/df(0) (Q*N reals, 0 on solid).
 * Each segment of K steps is recomputed from its checkpoint into the
 * workspace, then the steps are transposed in reverse order.  work_dev:
 * caller-owned device memory of at least lbm_adjoint_workspace_bytes(ctx,
 * K) bytes.  The context state is not changed.  Gradients through the
 * clamp of the limiter are taken as 1 on the closed interval
 * [rho_g, rho_l] and 0 outside.  The geometric formulation has no adjoint
 * (LBM_EINVAL). */
size_t lbm_adjoint_workspace_bytes(lbm_ctx* ctx, int64_t K);
int lbm_step_ckpt(lbm_ctx* ctx, int64_t T, int64_t K, void* ckpt_dev);
int lbm_adjoint(lbm_ctx* ctx, int32_t seed_kind, const void* seed_dev, int64_t T, int64_t K,
                const void* ckpt_dev, void* work_dev, size_t work_bytes, void* grad_phi_dev,
                void* grad_drho_dev, void* lam0_dev);

/* ------------------------------------------- allocation-free adjoint */
/* For callers that cannot allocate device memory where they call (code
 * under stream capture, tight training or serving loops, harnesses that
 * forbid hipMalloc): lbm_adjoint with its scratch in a device array of the
 * library instead of work_dev.  Same arguments, checks, results and errors
 * as lbm_adjoint otherwise.  The array holds LBM_NOALLOC_SCRATCH_BYTES;
 * each GPU the library runs on keeps its own copy until the process ends.
 * A call whose lbm_adjoint_workspace_bytes(ctx, K) exceeds that returns
 * LBM_ENOMEM with a message (choose a smaller K).  The call allocates
 * nothing: no hipMalloc/hipFree, and no allocating library routine.  Its
 * first call on a device looks up the array's address there (stream's
 * device).  Every call on one GPU shares that GPU's array, which keeps the
 * last call's contents (each call writes every value it reads before
 * reading it): calls ordered on one stream are safe, calls that overlap in
 * time on one GPU (several streams or host threads) race. */
#define LBM_NOALLOC_SCRATCH_BYTES (64u << 20)
int lbm_adjoint_noalloc(lbm_ctx* ctx, int32_t seed_kind, const void* seed_dev, int64_t T,
                        int64_t K, const void* ckpt_dev, void* grad_phi_dev,
                        void* grad_drho_dev, void* lam0_dev);

#ifdef __cplusplus
}
#endif
#endif /* LBM_H */
