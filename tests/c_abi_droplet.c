/* The C ABI used from plain C, with no Python or PyTorch: a periodic 32^3
 * droplet at 0.9 T_c (the stationary-droplet workload, Sec. III B), device
 * memory from the HIP runtime, 200 FP64 steps through lbfe_step, then the
 * invariants of the method checked on the reductions: total mass kept to
 * rounding (streaming and collision conserve it, Eq. (10)), total momentum
 * zero to rounding (the droplet is symmetric about the box centre and
 * starts at rest), and the flow of the relaxing tanh profile far below the
 * lattice speed of sound 1/sqrt(3) (max |u| < 0.1: a stable run).
 *
 * Built by the package build next to liblbfe.so; run by
 * tests/test_gpu_c_abi.py.  Prints one line and returns 0 on success. */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>

#include <hip/hip_runtime_api.h>

#include "lbfe.h"

#define HIP_OK(call)                                                        \
    do {                                                                    \
        hipError_t e_ = (call);                                             \
        if (e_ != hipSuccess) {                                             \
            fprintf(stderr, "%s: %s\n", #call, hipGetErrorString(e_));     \
            return 1;                                                       \
        }                                                                   \
    } while (0)
#define CHECK(ctx, call)                                                    \
    do {                                                                    \
        int r_ = (call);                                                    \
        if (r_ != LBFE_OK) {                                                \
            fprintf(stderr, "%s: %d %s\n", #call, r_,                      \
                    (ctx) ? lbfe_last_error(ctx) : "");                     \
            return 1;                                                       \
        }                                                                   \
    } while (0)

int main(void) {
    lbfe_params p;
    lbfe_ctx *ctx = NULL;
    CHECK(ctx, lbfe_params_default(&p));
    const int n = 32;
    p.nx = p.ny = p.nz = n;
    p.T = 0.9 * 8.0 * p.a / (27.0 * p.R * p.b); /* 0.9 T_c of the vdW EOS */
    CHECK(ctx, lbfe_create(&p, NULL, &ctx));

    size_t ws = 0;
    void *work = NULL;
    CHECK(ctx, lbfe_workspace_bytes(&p, &ws));
    HIP_OK(hipMalloc(&work, ws));
    CHECK(ctx, lbfe_bind_workspace(ctx, work, ws));

    /* the coexistence pair the context derived (Maxwell's rule) */
    lbfe_params q;
    CHECK(ctx, lbfe_get_params(ctx, &q));

    /* droplet of radius 8 at the centre, interface width 5 (Eq. (35)) */
    const size_t N = (size_t)n * n * n;
    double *rho = (double *)malloc(N * sizeof(double));
    if (!rho) return 1;
    for (int z = 0; z < n; ++z)
        for (int y = 0; y < n; ++y)
            for (int x = 0; x < n; ++x) {
                const double dx = x - 16.0, dy = y - 16.0, dz = z - 16.0;
                const double r = sqrt(dx * dx + dy * dy + dz * dz);
                rho[((size_t)z * n + y) * n + x] =
                    0.5 * (q.rho_l + q.rho_v) - 0.5 * (q.rho_l - q.rho_v) * tanh(2.0 * (r - 8.0) / 5.0);
            }
    double *rho_dev = NULL;
    HIP_OK(hipMalloc((void **)&rho_dev, N * sizeof(double)));
    HIP_OK(hipMemcpy(rho_dev, rho, N * sizeof(double), hipMemcpyHostToDevice));
    CHECK(ctx, lbfe_init_density(ctx, rho_dev, NULL));

    double r0[8], r1[8];
    CHECK(ctx, lbfe_reduce(ctx, r0));
    CHECK(ctx, lbfe_step(ctx, 200));
    CHECK(ctx, lbfe_reduce(ctx, r1));
    int64_t steps = 0;
    CHECK(ctx, lbfe_step_count(ctx, &steps));

    const double dmass = fabs(r1[0] - r0[0]) / r0[0];
    const double mom = sqrt(r1[1] * r1[1] + r1[2] * r1[2] + r1[3] * r1[3]) / r1[0];
    printf("c_abi_droplet: %lld steps, rho_l %.6f rho_v %.6f, mass drift %.2e, |sum j|/sum rho %.2e, max|u| %.2e\n",
           (long long)steps, q.rho_l, q.rho_v, dmass, mom, r1[7]);
    const int ok = steps == 200 && dmass < 1e-12 && mom < 1e-12 && r1[7] < 0.1 && r1[7] >= 0.0;

    CHECK(ctx, lbfe_destroy(ctx));
    HIP_OK(hipFree(rho_dev));
    HIP_OK(hipFree(work));
    free(rho);
    return ok ? 0 : 1;
}
