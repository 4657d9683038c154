/* A plain C consumer of the library (test infrastructure): no Python and no
 * torch; device memory comes from the HIP runtime.  It solves one periodic
 * lattice to a tolerance through include/lbm.h and writes the displacement.
 *
 * usage: capi_consumer nx ny lambda mu precision tol max_steps check_every
 *                      force.bin displacement.bin [inplace_steps]
 * inplace_steps (optional, default 0): 0 two buffers (lbm_create); 1 in place
 * with the minimal workspace (lbm_workspace_bytes_inplace); k in 2..8 in place
 * with room for launches of up to k steps (lbm_workspace_bytes_inplace_blocked).
 * force.bin: gx then gy, FP64, [ny][nx] each (x fastest); displacement.bin
 * receives ux then uy in the same layout.  Prints one JSON line (solve status,
 * the warning bits of lbm_set_body_force, steps, residual); exit status 0
 * on success (converged or not), 1 on a library or HIP error, 2 on bad usage. */
#include <stdio.h>
#include <stdlib.h>

#include <hip/hip_runtime_api.h>

#include "lbm.h"

static int hip_ok(hipError_t e, const char *what) {
    if (e != hipSuccess) {
        fprintf(stderr, "%s: %s\n", what, hipGetErrorString(e));
        return 0;
    }
    return 1;
}

int main(int argc, char **argv) {
    if (argc != 11 && argc != 12) {
        fprintf(stderr, "usage: %s nx ny lambda mu precision tol max_steps check_every "
                        "force.bin displacement.bin [inplace_steps]\n", argv[0]);
        return 2;
    }
    const int inplace_steps = argc == 12 ? atoi(argv[11]) : 0;
    const int nx = atoi(argv[1]), ny = atoi(argv[2]);
    const double lam = atof(argv[3]), mu = atof(argv[4]);
    const int precision = atoi(argv[5]);
    const double tol = atof(argv[6]);
    const long long max_steps = atoll(argv[7]);
    const int check_every = atoi(argv[8]);
    if (nx < 1 || ny < 1) return 2;
    const size_t n = (size_t)nx * (size_t)ny;

    double *host = (double *)malloc(2 * n * sizeof(double));
    FILE *fin = fopen(argv[9], "rb");
    if (!host || !fin || fread(host, sizeof(double), 2 * n, fin) != 2 * n) {
        fprintf(stderr, "cannot read %s\n", argv[9]);
        return 2;
    }
    fclose(fin);

    const size_t ws = inplace_steps >= 2
                          ? lbm_workspace_bytes_inplace_blocked(nx, ny, precision, inplace_steps, 0)
                      : inplace_steps == 1 ? lbm_workspace_bytes_inplace(nx, ny, precision)
                                           : lbm_workspace_bytes(nx, ny, precision, 0);
    void *d_ws = NULL;
    double *d_g = NULL, *d_u = NULL;
    if (ws == 0 || !hip_ok(hipMalloc(&d_ws, ws), "hipMalloc workspace") ||
        !hip_ok(hipMalloc((void **)&d_g, 2 * n * sizeof(double)), "hipMalloc force") ||
        !hip_ok(hipMalloc((void **)&d_u, 2 * n * sizeof(double)), "hipMalloc displacement") ||
        !hip_ok(hipMemcpy(d_g, host, 2 * n * sizeof(double), hipMemcpyHostToDevice), "upload"))
        return 1;

    lbm_solver *s = NULL;
    int rc = inplace_steps > 0 ? lbm_create_inplace(nx, ny, precision, d_ws, ws, NULL, &s)
                               : lbm_create(nx, ny, precision, 0, d_ws, ws, NULL, &s);
    if (rc != LBM_OK) {
        fprintf(stderr, "lbm_create: %s\n", lbm_last_error(NULL));
        return 1;
    }
    rc = lbm_set_material(s, lam, mu);
    int force_status = 0;
    if (rc == LBM_OK) {
        rc = lbm_set_body_force(s, d_g, d_g + n);
        /* informational bits: LBM_W_MEAN_REMOVED, LBM_W_STAGGERED_LOAD */
        if (rc > 0) {
            force_status = rc;
            rc = LBM_OK;
        }
    }
    long long steps = 0;
    double residual = 0.0;
    int status = LBM_OK;
    if (rc == LBM_OK) {
        status = lbm_solve_to_tol(s, tol, max_steps, check_every, &steps, &residual);
        if (status < 0) rc = status;
    }
    if (rc == LBM_OK) rc = lbm_get_displacement(s, d_u, d_u + n);
    if (rc != LBM_OK) {
        fprintf(stderr, "lbm: %s\n", lbm_last_error(s));
        lbm_destroy(s);
        return 1;
    }
    /* the library works on the null stream here, so this copy follows it */
    if (!hip_ok(hipMemcpy(host, d_u, 2 * n * sizeof(double), hipMemcpyDeviceToHost), "download"))
        return 1;
    FILE *fout = fopen(argv[10], "wb");
    if (!fout || fwrite(host, sizeof(double), 2 * n, fout) != 2 * n) {
        fprintf(stderr, "cannot write %s\n", argv[10]);
        return 1;
    }
    fclose(fout);
    int cfg[4] = {0, 0, 0, 0};
    lbm_get_launch_config(s, cfg);
    printf("{\"status\": %d, \"force_status\": %d, \"steps\": %lld, \"residual\": %.17g, "
           "\"steps_per_launch\": %d, \"kernel\": %d}\n",
           status, force_status, steps, residual, cfg[0], cfg[1]);
    lbm_destroy(s);
    hipFree(d_u);
    hipFree(d_g);
    hipFree(d_ws);
    free(host);
    return 0;
}
