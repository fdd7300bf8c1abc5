/* cabi_demo.c -- a plain C11 program that drives liblbm.so through the C
 * ABI of include/lbm.h alone: device memory from the HIP runtime, no
 * Python, no torch.
 *
 * A D2Q9 FP64 lattice of 96 x 80 with a cylinder (R = 12) and a droplet
 * (r = 10) resting on it, Carnahan-Starling fluid at 0.75 Tc, improved
 * virtual density with phi = 1.2 (Eqs. 16-17): 400 steps, then checks that
 * mass is conserved (halfway bounce-back and the collision conserve it,
 * Sec. II), that the fluid densities stay between the limiter bounds'
 * neighbourhood, that the wall virtual densities respect the limiter, and
 * that out-of-order and NULL calls are refused.  Prints one line and exits
 * 0 on success, 1 on any failure.
 */
#include <hip/hip_runtime_api.h>
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "lbm.h"

#define NX 96
#define NY 80

#define CHECK(call)                                                                   \
    do {                                                                              \
        int rc_ = (call);                                                             \
        if (rc_ != LBM_OK) {                                                          \
            fprintf(stderr, "%s: %s (%s)\n", #call, lbm_status_string(rc_),           \
                    lbm_last_error());                                                \
            return 1;                                                                 \
        }                                                                             \
    } while (0)

#define HIPCHECK(call)                                                                \
    do {                                                                              \
        hipError_t e_ = (call);                                                       \
        if (e_ != hipSuccess) {                                                       \
            fprintf(stderr, "%s: %s\n", #call, hipGetErrorString(e_));                \
            return 1;                                                                 \
        }                                                                             \
    } while (0)

static double min_image(double d, double n) {
    d = fmod(d + 0.5 * n, n);
    if (d < 0) d += n;
    return d - 0.5 * n;
}

int main(void) {
    lbm_params p;
    memset(&p, 0, sizeof p);
    p.lattice = 9;
    p.precision = 8;
    p.nx = NX;
    p.ny = NY;
    p.nz = 1;
    p.eos = LBM_EOS_CS;
    for (int k = 0; k < 19; ++k) p.tau[k] = 1.0;
    p.eos_a = 1.0;
    p.eos_b = 4.0;
    p.eos_R = 1.0;
    p.eos_omega = 0.344;
    double Tc = 0.0, rhoc = 0.0;
    CHECK(lbm_eos_critical(p.eos, p.eos_a, p.eos_b, p.eos_R, p.eos_omega, &Tc, &rhoc));
    p.eos_T = 0.75 * Tc;
    p.G = -1.0;
    p.sigma = 0.1071;
    CHECK(lbm_eos_coexistence(&p, &p.rho_g, &p.rho_l));
    CHECK(lbm_validate_params(&p));

    /* geometry and initial density on the host */
    static uint8_t solid[NX * NY];
    static double rho0[NX * NY], rho[NX * NY];
    const double cx = 48.0, cy = 30.0, R = 12.0, r0 = 10.0, dy0 = cy + R + r0;
    int64_t nsolid = 0;
    for (int y = 0; y < NY; ++y) {
        for (int x = 0; x < NX; ++x) {
            const double dx = min_image(x - cx, NX), dy = min_image(y - cy, NY);
            const int s = dx * dx + dy * dy <= R * R;
            solid[y * NX + x] = (uint8_t)s;
            nsolid += s;
            const double ex = min_image(x - cx, NX), ey = min_image(y - dy0, NY);
            const double r = sqrt(ex * ex + ey * ey);
            rho0[y * NX + x] = s ? 0.0
                                 : 0.5 * (p.rho_l + p.rho_g) -
                                       0.5 * (p.rho_l - p.rho_g) * tanh(2.0 * (r - r0) / 3.0);
        }
    }

    /* caller-owned device memory and stream */
    const size_t ws_bytes = lbm_workspace_bytes(&p, nsolid);
    if (ws_bytes == 0) {
        fprintf(stderr, "lbm_workspace_bytes: %s\n", lbm_last_error());
        return 1;
    }
    void *ws = NULL, *rho_dev = NULL;
    hipStream_t stream;
    HIPCHECK(hipMalloc(&ws, ws_bytes));
    HIPCHECK(hipMalloc(&rho_dev, sizeof rho0));
    HIPCHECK(hipStreamCreate(&stream));

    lbm_ctx* ctx = NULL;
    CHECK(lbm_create(&p, stream, ws, ws_bytes, nsolid, &ctx));
    if (lbm_step(ctx, 1) != LBM_ESTATE) {  /* nothing set yet */
        fprintf(stderr, "a step before the geometry was not refused\n");
        return 1;
    }
    if (lbm_step(NULL, 1) != LBM_EINVAL) {
        fprintf(stderr, "a NULL context was not refused\n");
        return 1;
    }
    CHECK(lbm_set_geometry(ctx, solid));
    int64_t nwall = 0;
    CHECK(lbm_wall_nodes(ctx, NULL, &nwall));
    CHECK(lbm_set_wetting(ctx, LBM_WET_IVD, 0.0, NULL, NULL, 1.2, 0.0));
    HIPCHECK(hipMemcpy(rho_dev, rho0, sizeof rho0, hipMemcpyHostToDevice));
    CHECK(lbm_set_fields(ctx, rho_dev, NULL));

    lbm_diag d0, d1;
    CHECK(lbm_get_diagnostics(ctx, &d0));
    CHECK(lbm_step(ctx, 400));
    CHECK(lbm_get_diagnostics(ctx, &d1));
    CHECK(lbm_get_fields(ctx, rho_dev, NULL, NULL));
    HIPCHECK(hipStreamSynchronize(stream));
    HIPCHECK(hipMemcpy(rho, rho_dev, sizeof rho, hipMemcpyDeviceToHost));

    int fail = 0;
    const double drift = fabs(d1.mass - d0.mass) / d0.mass;
    if (!(drift < 1e-12)) {
        fprintf(stderr, "mass drift %.3e\n", drift);
        fail = 1;
    }
    if (!(d1.rho_min > 0.5 * p.rho_g && d1.rho_max < 1.1 * p.rho_l) || d1.flag != 0) {
        fprintf(stderr, "fluid densities %.5f .. %.5f, flag %d\n", d1.rho_min, d1.rho_max,
                d1.flag);
        fail = 1;
    }
    /* wall nodes report their virtual density: inside the limiter bounds */
    int64_t nw_seen = 0;
    for (int y = 0; y < NY; ++y) {
        for (int x = 0; x < NX; ++x) {
            const double v = rho[y * NX + x];
            if (solid[y * NX + x] && v != 0.0) {
                ++nw_seen;
                if (v < p.rho_g - 1e-15 || v > p.rho_l + 1e-15) {
                    fprintf(stderr, "wall density %.6f outside [%.6f, %.6f]\n", v, p.rho_g, p.rho_l);
                    fail = 1;
                }
            }
        }
    }
    if (nw_seen != nwall) {
        fprintf(stderr, "%lld wall densities for %lld wall nodes\n", (long long)nw_seen,
                (long long)nwall);
        fail = 1;
    }
    CHECK(lbm_destroy(ctx));
    HIPCHECK(hipStreamDestroy(stream));
    HIPCHECK(hipFree(rho_dev));
    HIPCHECK(hipFree(ws));
    if (fail) return 1;
    printf("C ABI demo ok: %s, %dx%d D2Q9 FP64, %lld wall nodes, 400 steps, mass drift %.2e, "
           "rho %.5f .. %.5f, max|u| %.3e\n",
           lbm_version(), NX, NY, (long long)nwall, drift, d1.rho_min, d1.rho_max, d1.max_u);
    return 0;
}
