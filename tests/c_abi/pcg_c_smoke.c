/* The C ABI from plain C (no Python): one shifted pipelined CG solve of the
 * 3-D 7-point Poisson problem on a 32^3 grid with the Jacobi preconditioner,
 * b = A * 1 (so x = 1), x0 = 0, to 1e-10 with the binary64 explicit check.
 * Device memory comes from hipMalloc; the library allocates none.
 * Exit status 0 when the solve converges with ||b - A x|| / ||b|| <= 1e-10
 * and max |x - 1| <= 1e-8, and the library's argument checks reject a null
 * workspace and a mismatched grid; 1 otherwise. */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <hip/hip_runtime_api.h>

#include "pcg.h"

#define CHECK_HIP(call)                                                        \
    do {                                                                       \
        if ((call) != hipSuccess) {                                            \
            fprintf(stderr, "HIP call failed: %s\n", #call);                   \
            return 1;                                                          \
        }                                                                      \
    } while (0)

int main(void)
{
    const int N = 32;
    const int64_t n = (int64_t)N * N * N;
    pcg_operator op;
    memset(&op, 0, sizeof(op));
    op.kind = PCG_OP_STENCIL3D7;
    op.nx = op.ny = op.nz = N;
    op.n = n;
    op.diag = 6.0;
    op.offdiag = -1.0;

    pcg_options opt;
    if (pcg_default_options(&opt) != PCG_OK) return 1;
    opt.method = PCG_PIPE_SHIFT;
    opt.pc = PCG_PC_JACOBI;
    opt.prec = PCG_FP64;
    opt.sigma = 1.0;
    opt.rtol = 1e-10;
    opt.max_iter = 2000;
    opt.true_residual_check = 1;

    /* b = A * 1: 6 minus the number of existing neighbours */
    double *hb = (double *)malloc((size_t)n * sizeof(double));
    double *hx = (double *)malloc((size_t)n * sizeof(double));
    if (!hb || !hx) return 1;
    for (int k = 0; k < N; ++k)
        for (int j = 0; j < N; ++j)
            for (int i = 0; i < N; ++i) {
                const int nb = (i > 0) + (i < N - 1) + (j > 0) + (j < N - 1) + (k > 0) + (k < N - 1);
                hb[((int64_t)k * N + j) * N + i] = 6.0 - nb;
            }

    size_t bytes = 0;
    if (pcg_workspace_size(&op, &opt, &bytes) != PCG_OK) return 1;
    void *ws = NULL;
    double *b = NULL, *x = NULL;
    CHECK_HIP(hipMalloc(&ws, bytes));
    CHECK_HIP(hipMalloc((void **)&b, (size_t)n * sizeof(double)));
    CHECK_HIP(hipMalloc((void **)&x, (size_t)n * sizeof(double)));
    CHECK_HIP(hipMemcpy(b, hb, (size_t)n * sizeof(double), hipMemcpyHostToDevice));
    CHECK_HIP(hipMemset(x, 0, (size_t)n * sizeof(double)));

    /* argument checks: a null workspace and a grid that does not match n */
    pcg_solver bad = NULL;
    const int reject_ws = pcg_create(&bad, &op, &opt, NULL, bytes, NULL) == PCG_ERR_INVALID;
    pcg_operator wrong = op;
    wrong.nz = N - 1;
    const int reject_grid = pcg_create(&bad, &wrong, &opt, ws, bytes, NULL) == PCG_ERR_INVALID;

    pcg_solver s = NULL;
    pcg_status st = pcg_create(&s, &op, &opt, ws, bytes, NULL);
    if (st != PCG_OK) {
        fprintf(stderr, "pcg_create: %s (%s)\n", pcg_status_str(st), pcg_last_error());
        return 1;
    }
    pcg_result res;
    st = pcg_solve(s, b, x, &res);
    if (st != PCG_OK) {
        fprintf(stderr, "pcg_solve: %s (%s)\n", pcg_status_str(st), pcg_last_error());
        return 1;
    }
    if (pcg_destroy(s) != PCG_OK) return 1;
    CHECK_HIP(hipMemcpy(hx, x, (size_t)n * sizeof(double), hipMemcpyDeviceToHost));
    double err = 0.0;
    for (int64_t e = 0; e < n; ++e) err = fmax(err, fabs(hx[e] - 1.0));
    printf("C ABI solve: status %d, %d iterations, explicit residual %.3e, max |x - 1| %.3e, "
           "rejects null workspace %d, mismatched grid %d\n",
           res.status, res.iterations, res.rel_res_true, err, reject_ws, reject_grid);
    CHECK_HIP(hipFree(ws));
    CHECK_HIP(hipFree(b));
    CHECK_HIP(hipFree(x));
    free(hb);
    free(hx);
    const int ok = res.status == PCG_CONVERGED && res.rel_res_true <= 1e-10 && err <= 1e-8 && reject_ws &&
                   reject_grid;
    return ok ? 0 : 1;
}
