/*
 * oracle.h -- C interface of the CPU oracle for the pseudopotential MRT
 * lattice Boltzmann step with contact-angle wall schemes (Li, Yu & Luo,
 * "Implementation of contact angles in the pseudopotential lattice Boltzmann
 * simulations with curved boundaries").
 *
 * TEST INFRASTRUCTURE ONLY.  This is a plain, slow, FP64 reference written
 * from the paper, used to check the GPU library.  Only the test-suite, the
 * package smoke check and the CPU-baseline leg of the benchmark may load it.
 * It shares no code, header, table or helper with the GPU library.
 *
 * Conventions: lattice units (dx = dt = 1, c = 1, cs^2 = 1/3, Sec. II A).
 * Node index n = x + nx*(y + ny*z), x fastest.  Populations are stored
 * structure-of-arrays, f[a*N + n].  Every axis is periodic; walls are solid
 * nodes.  All arrays are host memory owned by the caller.
 */
#ifndef LBM_ORACLE_H
#define LBM_ORACLE_H

#include <stdint.h>
#include <complex.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { ORC_EOS_CS = 0, ORC_EOS_PR = 1 };
/* wetting schemes: improved virtual density (Eqs. 16-17), constant virtual
 * density, solid-fluid interaction (Eq. 8), curved geometric formulation
 * (Eqs. 11, 13-15; 2-D only; the per-wall prescribed angle theta_a in
 * degrees is passed in the phi array) */
enum { ORC_IVD = 0, ORC_VD = 1, ORC_SFI = 2, ORC_GF = 3 };
enum { ORC_OK = 0, ORC_EINVAL = -1, ORC_EDOMAIN = -3 };

typedef struct {
    int32_t lattice;        /* 9 (D2Q9) or 19 (D3Q19) */
    int32_t nx, ny, nz;     /* nz = 1 for D2Q9 */
    double tau[19];         /* relaxation time of each moment row (Eq. 2) */
    int32_t eos;            /* ORC_EOS_CS or ORC_EOS_PR */
    double eos_a, eos_b, eos_R, eos_T, eos_omega;
    double G;               /* interaction strength of Eq. 5 (-1 in the paper) */
    double sigma;           /* thermodynamic-consistency constant of Eq. 7 */
    double body_force[3];   /* constant body force added to F */
    int32_t scheme;         /* ORC_IVD, ORC_VD, ORC_SFI, ORC_GF */
    double rho_w;           /* VD constant virtual density */
    double G_w;             /* SFI adhesion strength (Eq. 8) */
    double rho_g, rho_l;    /* limiter bounds of the improved scheme */
    /* SFI only: the pseudopotential the solid nodes carry in Eq. 5, which
     * the paper does not state.  0: none (the reading the library takes);
     * 1: psi of the Eq. 17 mean of the node's fluid neighbours; 2: psi(rho_g);
     * 3: psi(rho_l); 4: each fluid node sees its solid neighbours at its own
     * psi.  Values 1-4 exist for the study of Fig. 6 only. */
    int32_t sfi_solid_psi;
    /* SFI only: pre-sum factor of Eq. 8; 0: rho(x) as printed, 1: psi(x)
     * (for the same study) */
    int32_t sfi_psi_presum;
    /* SFI only: weights of the sum in Eq. 8; 0: those of Eq. 5 (1/3, 1/12 in
     * D2Q9), 1: the lattice weights (1/9, 1/36) (for the same study) */
    int32_t sfi_lattice_weights;
} orc_params;

/* ---- thermodynamics (real arithmetic) ---- */
double orc_eos_p(const orc_params* p, double rho);
/* psi argument 2*(rho*cs^2 - p)/(-G) ... returns the value under the root */
double orc_psi_arg(const orc_params* p, double rho);
int orc_critical(int32_t eos, double a, double b, double R, double omega,
                 double* Tc, double* rhoc);
int orc_coexistence(const orc_params* p, double* rho_g, double* rho_l);

/* ---- geometry ---- */
/* Number of wall nodes (solid nodes with a fluid neighbour in the force
 * stencil); if idx != NULL also writes their node indices in increasing
 * order. */
int64_t orc_wall_nodes(const orc_params* p, const uint8_t* solid, int64_t* idx);

/* The construction of the geometric formulation (Sec. III A, Eqs. 13-15) at
 * every wall node, for the pins: theta_deg one angle per wall node (wall
 * order); out 6 doubles per wall node: the unit normal n_s and the points
 * D_1, D_2, relative to the node (NaN where no normal can be formed). */
int orc_gf_points(const orc_params* p, const uint8_t* solid, const double* theta_deg,
                  double* out);

/* ---- real-valued state ---- */
int orc_init_eq(const orc_params* p, const uint8_t* solid, const double* rho0,
                const double* u0 /* [D][N] or NULL */, double* f);
int orc_run(const orc_params* p, const uint8_t* solid, const double* phi,
            const double* drho, double* f, int64_t nsteps);
int orc_fields(const orc_params* p, const uint8_t* solid, const double* phi,
               const double* drho, const double* f, double* rho, double* u,
               double* force /* [D][N] or NULL */);
int orc_loss(const orc_params* p, const uint8_t* solid, const double* phi,
             const double* drho, const double* f0, int64_t nsteps,
             const double* target, double* loss);

/* ---- complex-step differentiation of the same step ----
 * Runs the step with phi[k] (which == 0) or drho[k] (which == 1) perturbed by
 * i*h and returns d loss / d parameter = Im(loss)/h. */
int orc_loss_grad_cs(const orc_params* p, const uint8_t* solid,
                     const double* phi, const double* drho, const double* f0,
                     int64_t nsteps, const double* target, int32_t which,
                     int64_t k, double h, double* loss, double* dloss);
/* Directional derivative of the state after nsteps along an initial-state
 * perturbation df0 (complex step).  df_out receives d f(T). */
int orc_state_tangent_cs(const orc_params* p, const uint8_t* solid,
                         const double* phi, const double* drho,
                         const double* f0, const double* df0, int64_t nsteps,
                         double h, double* f_out, double* df_out);

/* ---- lattice tables, exposed for tests ---- */
int orc_lattice(int32_t lattice, int32_t* e /* [Q][3] */, double* t, double* w,
                double* M /* [Q][Q] */, double* Minv, int32_t* opp);
/* moment-space source vector S of Eq. 7 (D2Q9) or its 3-D counterpart */
int orc_source(const orc_params* p, const double* u, const double* F,
               const double* Fm, double psi, double* S);
void orc_set_threads(int n);
int orc_get_threads(void);

#ifdef __cplusplus
}
#endif
#endif
