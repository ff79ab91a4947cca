/* A plain C99 caller of libcj.so (include/cj.h), for the ABI tests.
 *
 *   c_abi_caller host
 *       host-only calls: plan, plan info, launch info, status strings, an
 *       argument error; takes the address of every declared entry point.
 *   c_abi_caller solve NX NY STENCIL TOL F_IN U_OUT
 *       reads f (NY x NX doubles, x fastest) from F_IN, solves A u = f from
 *       u = 0 in device buffers from hipMalloc on the default stream, and
 *       writes u to U_OUT.  Prints the status, cycles and relative residual. */
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <hip/hip_runtime_api.h>

#include "cj.h"

typedef void (*any_fn)(void);

static int host_calls(void) {
    /* every entry point the header declares, so that a missing export fails
       to link */
    any_fn fns[] = {
        (any_fn)cj_options_init, (any_fn)cj_plan, (any_fn)cj_plan_ex, (any_fn)cj_plan_info,
        (any_fn)cj_plan_launch_info, (any_fn)cj_solve, (any_fn)cj_solve_dd, (any_fn)cj_sweeps,
        (any_fn)cj_residual, (any_fn)cj_residual_noalloc, (any_fn)cj_apply, (any_fn)cj_batch_create,
        (any_fn)cj_batch_info, (any_fn)cj_batch_solve, (any_fn)cj_batch_destroy, (any_fn)cj_server_create,
        (any_fn)cj_server_submit, (any_fn)cj_server_step, (any_fn)cj_server_stats, (any_fn)cj_server_destroy,
        (any_fn)cj_plan_destroy, (any_fn)cj_status_string, (any_fn)cj_last_error};
    size_t k;
    for (k = 0; k < sizeof(fns) / sizeof(fns[0]); ++k)
        if (!fns[k]) return 1;

    cj_options opt;
    cj_options_init(&opt);
    cj_plan_t p = NULL;
    cj_status st = cj_plan(129, 100, 9, CJ_BC_DIRICHLET0, 1e-10, &p);
    if (st != CJ_OK || !p) {
        printf("plan failed: %s\n", cj_last_error());
        return 1;
    }
    double kmin = 0.0, kmax = 0.0;
    int M = 0, cycles = 0, K = 0, rows = 0, wg = 0;
    const double* w = NULL;
    size_t ws = 0;
    if (cj_plan_info(p, &kmin, &kmax, &M, &cycles, &w, &ws) != CJ_OK) return 1;
    if (cj_plan_launch_info(p, &K, &rows, &wg) != CJ_OK) return 1;
    printf("plan M %d cycles %d kmin %.17g kmax %.17g w0 %.17g w1 %.17g workspace %zu K %d\n", M, cycles, kmin,
           kmax, w[0], w[1], ws, K);
    cj_plan_destroy(p);

    /* an argument error crosses the ABI as a status, with a message */
    p = NULL;
    st = cj_plan(16, 16, 7, CJ_BC_DIRICHLET0, 1e-10, &p);
    printf("stencil 7: %s (%s), plan %s\n", cj_status_string(st), cj_last_error(), p ? "set" : "null");
    if (st != CJ_ERR_ARG || p) return 1;
    printf("host ok\n");
    return 0;
}

static int solve(int nx, int ny, int stencil, double tol, const char* fin, const char* uout) {
    const size_t n = (size_t)nx * (size_t)ny;
    double* h = (double*)malloc(n * sizeof(double));
    FILE* fh = fopen(fin, "rb");
    if (!h || !fh || fread(h, sizeof(double), n, fh) != n) {
        printf("cannot read %s\n", fin);
        return 1;
    }
    fclose(fh);
    double *df = NULL, *du = NULL;
    if (hipMalloc((void**)&df, n * sizeof(double)) != hipSuccess ||
        hipMalloc((void**)&du, n * sizeof(double)) != hipSuccess) {
        printf("hipMalloc failed\n");
        return 1;
    }
    if (hipMemcpy(df, h, n * sizeof(double), hipMemcpyHostToDevice) != hipSuccess ||
        hipMemset(du, 0, n * sizeof(double)) != hipSuccess) {
        printf("copy in failed\n");
        return 1;
    }
    cj_plan_t p = NULL;
    if (cj_plan(nx, ny, stencil, CJ_BC_DIRICHLET0, tol, &p) != CJ_OK) {
        printf("plan failed: %s\n", cj_last_error());
        return 1;
    }
    cj_result r;
    memset(&r, 0, sizeof(r));
    const cj_status st = cj_solve(p, df, du, NULL, &r);
    printf("solve: %s cycles %d sweeps %lld relres %.17g\n", cj_status_string(st), r.cycles, r.sweeps,
           r.rel_residual);
    if (hipMemcpy(h, du, n * sizeof(double), hipMemcpyDeviceToHost) != hipSuccess) {
        printf("copy out failed\n");
        return 1;
    }
    FILE* fo = fopen(uout, "wb");
    if (!fo || fwrite(h, sizeof(double), n, fo) != n) return 1;
    fclose(fo);
    cj_plan_destroy(p);
    (void)hipFree(df);
    (void)hipFree(du);
    free(h);
    return (st == CJ_OK || st == CJ_STAGNATED) ? 0 : 2;
}

int main(int argc, char** argv) {
    if (argc == 2 && strcmp(argv[1], "host") == 0) return host_calls();
    if (argc == 8 && strcmp(argv[1], "solve") == 0)
        return solve(atoi(argv[2]), atoi(argv[3]), atoi(argv[4]), atof(argv[5]), argv[6], argv[7]);
    fprintf(stderr, "usage: %s host | solve NX NY STENCIL TOL F_IN U_OUT\n", argv[0]);
    return 64;
}
