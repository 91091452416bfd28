/*
 * pcg_oracle.c -- the oracle for the shifted pipelined CG hot path.
 *
 * TEST INFRASTRUCTURE, NOT PRODUCT CODE.  Only the test suite, the smoke
 * check and the benchmark's CPU-baseline leg may load this library.  It shares
 * no source, header, helper or constant with the HIP path.
 *
 * A plain, slow, obviously-correct CPU implementation in IEEE double precision
 * (compiled without FMA contraction and without fast-math) of
 *   - classic preconditioned CG ............... Alg. 1 (Section 1)
 *   - preconditioned pipelined CG (p-CG) ....... Alg. 2 (Section 2.1)
 *   - shifted preconditioned pipelined CG ...... Alg. 3 (Section 2.2)
 *   - p-CG with a variable shift sigma_i ........ Alg. 4 (Section 4.1)
 *   - p-CG with automated residual replacement (p-CG-rr, Section 5.2): a
 *     design of this project, since the criterion's source is not available
 *     (see the conventions below)
 * on an SPD operator given as a 2-D 5-point stencil, a 3-D 7-point stencil
 * (homogeneous Dirichlet, interior unknowns, x fastest) or a CSR matrix, with
 * no preconditioner or the Jacobi (diagonal) preconditioner.
 *
 * Every vector operation is its own full-length loop, executed in the order
 * the algorithm lists its steps; nothing is fused or reordered.  Conventions
 * where the paper leaves a choice open (each one is a documented reading):
 *   - delta of Alg. 3 is formed elementwise as sum_k (w_k + sigma r_k) u_k;
 *   - the three-term r and u updates add the second and third terms first,
 *     r - (alpha s + (alpha sigma) t), as the rounding model of Section 3.1
 *     assumes, with alpha*sigma formed once;
 *   - the stop test is taken at the top of iteration i on the recursive
 *     residual: sqrt((r_i, r_i)) <= rtol ||b||;
 *   - breakdown: gamma <= 0, delta <= 0 (pipelined), (s,p) <= 0 (CG) or a
 *     non-finite / non-positive alpha stops the solve, unless the caller asks
 *     to run on to the iteration cap as the accuracy runs of Section 5.1 do;
 *   - Jacobi: m = dinv .* w with dinv = 1/diag(A) formed once;
 *   - a stencil row sums centre, -x, +x, -y, +y, -z, +z in that order;
 *     a CSR row sums its entries in storage order;
 *   - a dot product sums sequentially inside fixed 4096-element chunks and
 *     then sums the chunk results sequentially, so the result is the same at
 *     any thread count;
 *   - FP32-storage emulation: every stored vector other than x and b (and the
 *     Jacobi diagonal) is rounded to binary32 at its store and widened on
 *     load; arithmetic, dots and scalars stay binary64.  m and n are
 *     transient and are not rounded.
 *   - optional residual replacement (not part of Alg. 1-3): when the
 *     recursive test is met but the explicit residual b - A x is not, the
 *     method restarts from the current x -- the initialisation steps are run
 *     again with x_0 := x_i and the next iteration takes the i = 0 branch
 *     (beta = 0) -- while the iteration count continues.
 *   - Alg. 4: each recurrence that carries a shift-difference correction
 *     forms the two-term recurrence first and subtracts the correction last,
 *     (a + beta y) - (sigma_i - sigma_{i-1}) c, and w_{i+1} is formed
 *     before r_i is overwritten, as the derivation of Section 4.1 requires;
 *     the shift schedule holds sigma_{-1}, sigma_0, sigma_1, ... and its
 *     last entry repeats past its end.
 *   - p-CG-rr: at the top of iteration i (after the stop test and the cap,
 *     before the breakdown checks), when i > i_start and i is a multiple of
 *     the monitoring period m, the gap f_i = (b - A x_i) - r_i is measured;
 *     if ||f_i|| > tau ||r_i|| the residual and the auxiliary vectors are
 *     reset to their true values -- r := b - A x_i, u := M^{-1} r,
 *     w := A u, s := A p_{i-1}, q := M^{-1} s, z := A q -- and iteration i
 *     starts again from its dot products, its beta continuing the old
 *     recurrence (gamma_{i-1}, alpha_{i-1} are kept).
 * Diagnostics: the stored vectors (r, u, w, z, q, s, t, p and the Jacobi
 * diagonal) when the solve returns and as the body of a chosen iteration
 * finds them; the explicit residual ||b - A x_i|| per iteration and the gap
 * norms ||f||, ||g||, ||h||, ||j|| of Section 3.1 from their definitions; a
 * test hook adds a given vector to w_0, planting a known gap h_0 whose
 * propagation the tests follow through the propagation matrices.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_CHUNK 4096

enum { ORC_2D5 = 0, ORC_3D7 = 1, ORC_CSR = 2 };
enum { ORC_CG = 0, ORC_PIPE = 1, ORC_PIPE_SHIFT = 2, ORC_PIPE_VAR = 3, ORC_PIPE_RR = 4 };
enum { ORC_CONVERGED = 0, ORC_MAX_ITER = 1, ORC_BREAKDOWN = 2, ORC_NONFINITE = 3 };

typedef struct {
    int32_t kind;
    int32_t pad_;
    int64_t n;
    int64_t nx, ny, nz;
    double centre;          /* stencil diagonal (including any diagonal shift) */
    double off;             /* stencil off-diagonal coefficient */
    const int64_t *row_ptr; /* CSR */
    const int32_t *col;
    const double *val;
} orc_op;

typedef struct {
    int32_t method;
    int32_t max_iter;
    double sigma;
    double rtol;
    int32_t jacobi;        /* 1: M = diag(A) */
    int32_t fp32_storage;  /* 1: emulate binary32 storage of the Krylov vectors */
    int32_t record_true;   /* 1: record ||b - A x_i|| / ||b|| every iteration */
    int32_t record_gaps;   /* 1: record gap norms (p-CG, p-CG-sh) */
    int32_t threads;       /* OpenMP threads, <= 0: library default */
    int32_t replace_max;   /* max residual replacements (0: none) */
    int32_t ignore_breakdown; /* 1: run to max_iter as the paper's accuracy runs do */
    const double *sigma_sched; /* Alg. 4: sigma_{-1}, sigma_0, ... (last entry repeats) */
    int32_t sigma_sched_len;
    const double *w0_perturb;  /* test hook: added to w_0 after the initialisation (NULL: none) */
    double rr_tau;             /* p-CG-rr: replace when ||f_i|| > rr_tau ||r_i|| */
    int32_t rr_period;         /* p-CG-rr: measure the gap every rr_period iterations */
    double rr_floor;           /* p-CG-rr: ... and only when ||f_i|| > rr_floor * eps || |A||x| + |b| || */
    int32_t snap_iter;         /* record the stored vectors as the body of iteration snap_iter finds them
                                  (after any restart or replacement at its top); < 0: never */
} orc_opts;

typedef struct {
    int32_t status;
    int32_t iterations;
    int32_t replacements;
    int32_t pad_;
    double bnorm;
    double rel_res_recursive;
    double rel_res_true;
    /* optional histories, each max_iter + 1 long (NULL: not recorded) */
    double *h_res;   /* sqrt(rho_i) / ||b|| at the top of iteration i */
    double *h_true;  /* ||b - A x_i|| / ||b|| */
    double *h_alpha;
    double *h_beta;
    double *h_gamma;
    double *h_delta;
    double *h_f, *h_g, *h_h, *h_j; /* gap norms, index as in Section 3.1 */
    /* optional ORC_NVEC * n buffers of the stored vectors, slot order r, u, w,
     * z, q, s, t, p, dinv; a vector the method does not keep is written as NaN */
    double *snap;        /* at the top of iteration snap_iter's body (untouched if never reached) */
    double *final_vecs;  /* when the solve returns */
} orc_result;

/* ---------------------------------------------------------------- helpers */

static int g_fp32 = 0;

/* store rounding: identity in binary64 mode, round-to-nearest binary32 else */
static inline double st(double v) { return g_fp32 ? (double)(float)v : v; }

static double *vec(int64_t n) { return (double *)calloc((size_t)(n > 0 ? n : 1), sizeof(double)); }

/* The stored vectors of a method, in the slot order of orc_result.snap. */
enum { ORC_NVEC = 9 };

static void dump_vecs(double *out, int64_t n, const double *const v[ORC_NVEC])
{
    for (int k = 0; k < ORC_NVEC; ++k) {
        double *o = out + (size_t)k * (size_t)n;
        if (v[k])
            memcpy(o, v[k], (size_t)n * sizeof(double));
        else
            for (int64_t i = 0; i < n; ++i) o[i] = NAN;
    }
}

/* out = A v.  Dirichlet stencil rows take neighbours that exist only. */
static void apply_A(const orc_op *A, const double *v, double *out)
{
    const int64_t n = A->n;
    if (A->kind == ORC_CSR) {
#pragma omp parallel for schedule(static)
        for (int64_t i = 0; i < n; ++i) {
            double acc = 0.0;
            for (int64_t k = A->row_ptr[i]; k < A->row_ptr[i + 1]; ++k)
                acc = acc + A->val[k] * v[A->col[k]];
            out[i] = acc;
        }
        return;
    }
    const int64_t nx = A->nx, ny = A->ny, nz = (A->kind == ORC_3D7) ? A->nz : 1;
    const int64_t sxy = nx * ny;
#pragma omp parallel for schedule(static)
    for (int64_t idx = 0; idx < n; ++idx) {
        const int64_t i = idx % nx, j = (idx / nx) % ny, k = idx / sxy;
        double acc = A->centre * v[idx];
        if (i > 0) acc = acc + A->off * v[idx - 1];
        if (i < nx - 1) acc = acc + A->off * v[idx + 1];
        if (j > 0) acc = acc + A->off * v[idx - nx];
        if (j < ny - 1) acc = acc + A->off * v[idx + nx];
        if (A->kind == ORC_3D7) {
            if (k > 0) acc = acc + A->off * v[idx - sxy];
            if (k < nz - 1) acc = acc + A->off * v[idx + sxy];
        }
        out[idx] = acc;
    }
}

/* dinv_k = 1 / a_kk */
static void jacobi_diag(const orc_op *A, double *dinv)
{
    for (int64_t i = 0; i < A->n; ++i) {
        double d = 0.0;
        if (A->kind == ORC_CSR) {
            for (int64_t k = A->row_ptr[i]; k < A->row_ptr[i + 1]; ++k)
                if (A->col[k] == i) d = d + A->val[k];
        } else {
            d = A->centre;
        }
        dinv[i] = st(1.0 / d);
    }
}

/* out = M^{-1} v */
static void apply_Minv(int64_t n, const double *dinv, const double *v, double *out)
{
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) out[i] = dinv ? dinv[i] * v[i] : v[i];
}

/* sum_k a_k b_k, chunked as described in the header */
static double dot(int64_t n, const double *a, const double *b)
{
    const int64_t nc = (n + ORC_CHUNK - 1) / ORC_CHUNK;
    double *part = vec(nc);
#pragma omp parallel for schedule(static)
    for (int64_t c = 0; c < nc; ++c) {
        const int64_t lo = c * ORC_CHUNK, hi = lo + ORC_CHUNK < n ? lo + ORC_CHUNK : n;
        double s = 0.0;
        for (int64_t i = lo; i < hi; ++i) s = s + a[i] * b[i];
        part[c] = s;
    }
    double s = 0.0;
    for (int64_t c = 0; c < nc; ++c) s = s + part[c];
    free(part);
    return s;
}

/* sum_k (w_k + sigma r_k) u_k, chunked like dot() */
static double dot_shift(int64_t n, const double *w, double sigma, const double *r, const double *u)
{
    const int64_t nc = (n + ORC_CHUNK - 1) / ORC_CHUNK;
    double *part = vec(nc);
#pragma omp parallel for schedule(static)
    for (int64_t c = 0; c < nc; ++c) {
        const int64_t lo = c * ORC_CHUNK, hi = lo + ORC_CHUNK < n ? lo + ORC_CHUNK : n;
        double s = 0.0;
        for (int64_t i = lo; i < hi; ++i) s = s + (w[i] + sigma * r[i]) * u[i];
        part[c] = s;
    }
    double s = 0.0;
    for (int64_t c = 0; c < nc; ++c) s = s + part[c];
    free(part);
    return s;
}

static double norm2(int64_t n, const double *a) { return sqrt(dot(n, a, a)); }

/* y = a + beta * y   (stored) */
static void aypx(int64_t n, const double *a, double beta, double *y)
{
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) y[i] = st(a[i] + beta * y[i]);
}

/* y = y + alpha * a  (x update: never rounded to binary32) */
static void axpy_x(int64_t n, double alpha, const double *a, double *y)
{
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) y[i] = y[i] + alpha * a[i];
}

/* y = y - alpha * a   (stored) */
static void ymax(int64_t n, double alpha, const double *a, double *y)
{
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) y[i] = st(y[i] - alpha * a[i]);
}

/* y = y - (alpha * a + as * c)   (stored; second and third terms first) */
static void ymax3(int64_t n, double alpha, const double *a, double as, const double *c, double *y)
{
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) y[i] = st(y[i] - (alpha * a[i] + as * c[i]));
}

/* y = (a + beta * y) - d * c   (stored; Alg. 4 recurrences with a shift correction) */
static void aypx_corr(int64_t n, const double *a, double beta, double d, const double *c, double *y)
{
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) y[i] = st((a[i] + beta * y[i]) - d * c[i]);
}

/* z = (nn + beta z) - d (s + sig t)   (stored; the z recurrence of Alg. 4) */
static void z_var(int64_t n, const double *nn, double beta, double d, const double *s, double sig,
                  const double *t, double *z)
{
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) z[i] = st((nn[i] + beta * z[i]) - d * (s[i] + sig * t[i]));
}

/* y = (y - alpha a) - d c   (stored; the w recurrence of Alg. 4) */
static void ymax_corr(int64_t n, double alpha, const double *a, double d, const double *c, double *y)
{
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) y[i] = st((y[i] - alpha * a[i]) - d * c[i]);
}

/* out = |A| |v| + |c|  (rounding scale of computing c - A v; entrywise) */
static void abs_scale(const orc_op *A, const double *v, const double *c, double *out)
{
    const int64_t n = A->n;
    if (A->kind == ORC_CSR) {
#pragma omp parallel for schedule(static)
        for (int64_t i = 0; i < n; ++i) {
            double acc = 0.0;
            for (int64_t k = A->row_ptr[i]; k < A->row_ptr[i + 1]; ++k) acc = acc + fabs(A->val[k]) * fabs(v[A->col[k]]);
            out[i] = acc + fabs(c[i]);
        }
        return;
    }
    const int64_t nx = A->nx, ny = A->ny, nz = (A->kind == ORC_3D7) ? A->nz : 1;
    const int64_t sxy = nx * ny;
    const double ac = fabs(A->centre), ao = fabs(A->off);
#pragma omp parallel for schedule(static)
    for (int64_t idx = 0; idx < n; ++idx) {
        const int64_t i = idx % nx, j = (idx / nx) % ny, k = idx / sxy;
        double acc = ac * fabs(v[idx]);
        if (i > 0) acc = acc + ao * fabs(v[idx - 1]);
        if (i < nx - 1) acc = acc + ao * fabs(v[idx + 1]);
        if (j > 0) acc = acc + ao * fabs(v[idx - nx]);
        if (j < ny - 1) acc = acc + ao * fabs(v[idx + nx]);
        if (A->kind == ORC_3D7) {
            if (k > 0) acc = acc + ao * fabs(v[idx - sxy]);
            if (k < nz - 1) acc = acc + ao * fabs(v[idx + sxy]);
        }
        out[idx] = acc + fabs(c[idx]);
    }
}

/* out = b - A x  (explicit residual, binary64) */
static void true_residual(const orc_op *A, const double *b, const double *x, double *tmp, double *out)
{
    apply_A(A, x, tmp);
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < A->n; ++i) out[i] = b[i] - tmp[i];
}

static int finite_pos(double v) { return isfinite(v) && v > 0.0; }

/* ------------------------------------------------------------ Alg. 1: CG */

static int solve_cg(const orc_op *A, const double *dinv, const orc_opts *o, const double *b, double *x,
                    orc_result *res)
{
    const int64_t n = A->n;
    double *r = vec(n), *u = vec(n), *p = vec(n), *s = vec(n), *tmp = vec(n), *tr = vec(n);
    const double bnorm = norm2(n, b);
    res->bnorm = bnorm;
    int replacements = 0;

    /* r_0 := b - A x_0; u_0 := M^{-1} r_0; p_0 := u_0 */
    apply_A(A, x, tmp);
    for (int64_t k = 0; k < n; ++k) r[k] = st(b[k] - tmp[k]);
    apply_Minv(n, dinv, r, u);
    for (int64_t k = 0; k < n; ++k) u[k] = st(u[k]);
    for (int64_t k = 0; k < n; ++k) p[k] = u[k];

    double gamma = dot(n, r, u), rho = dot(n, r, r), beta = 0.0;
    int status = ORC_MAX_ITER, i = 0;
    for (i = 0;; ++i) {
        if (res->h_res) res->h_res[i] = sqrt(rho) / bnorm;
        if (res->h_gamma) res->h_gamma[i] = gamma;
        if (res->h_beta) res->h_beta[i] = beta;
        if (res->h_true) {
            true_residual(A, b, x, tmp, tr);
            res->h_true[i] = norm2(n, tr) / bnorm;
        }
        if (!isfinite(rho)) { status = ORC_NONFINITE; break; }
        if (sqrt(rho) <= o->rtol * bnorm) {
            if (replacements < o->replace_max) {
                true_residual(A, b, x, tmp, tr);
                if (norm2(n, tr) > o->rtol * bnorm) {
                    /* restart from x: r := b - A x; u := M^{-1} r; p := u */
                    ++replacements;
                    for (int64_t k = 0; k < n; ++k) r[k] = st(tr[k]);
                    apply_Minv(n, dinv, r, u);
                    for (int64_t k = 0; k < n; ++k) u[k] = st(u[k]);
                    for (int64_t k = 0; k < n; ++k) p[k] = u[k];
                    gamma = dot(n, r, u);
                    rho = dot(n, r, r);
                    beta = 0.0;
                    --i;  /* redo the top of iteration i */
                    continue;
                }
            }
            status = ORC_CONVERGED;
            break;
        }
        if (i >= o->max_iter) { status = ORC_MAX_ITER; break; }
        if (!o->ignore_breakdown && !(gamma > 0.0)) { status = ORC_BREAKDOWN; break; }
        if (res->snap && i == o->snap_iter) {
            const double *v[ORC_NVEC] = {r, u, NULL, NULL, NULL, s, NULL, p, dinv};
            dump_vecs(res->snap, n, v);
        }

        apply_A(A, p, s);                          /* s_i := A p_i           */
        for (int64_t k = 0; k < n; ++k) s[k] = st(s[k]);
        const double sp = dot(n, s, p);
        if (!o->ignore_breakdown && !(sp > 0.0)) { status = ORC_BREAKDOWN; break; }
        const double alpha = gamma / sp;           /* alpha_i                */
        if (res->h_alpha) res->h_alpha[i] = alpha;
        if (res->h_delta) res->h_delta[i] = sp;
        if (!o->ignore_breakdown && !finite_pos(alpha)) { status = ORC_BREAKDOWN; break; }
        axpy_x(n, alpha, p, x);                    /* x_{i+1}                */
        ymax(n, alpha, s, r);                      /* r_{i+1}                */
        apply_Minv(n, dinv, r, u);                 /* u_{i+1} := M^{-1} r    */
        for (int64_t k = 0; k < n; ++k) u[k] = st(u[k]);
        const double gamma_new = dot(n, r, u);
        rho = dot(n, r, r);
        beta = gamma_new / gamma;                  /* beta_{i+1}             */
        aypx(n, u, beta, p);                       /* p_{i+1} := u + beta p  */
        gamma = gamma_new;
    }
    res->status = status;
    res->iterations = i;
    res->replacements = replacements;
    res->rel_res_recursive = sqrt(rho) / bnorm;
    true_residual(A, b, x, tmp, tr);
    res->rel_res_true = norm2(n, tr) / bnorm;
    if (res->final_vecs) {
        const double *v[ORC_NVEC] = {r, u, NULL, NULL, NULL, s, NULL, p, dinv};
        dump_vecs(res->final_vecs, n, v);
    }
    free(r); free(u); free(p); free(s); free(tmp); free(tr);
    return 0;
}

/* ------------------------------------------ Alg. 2 (p-CG) and Alg. 3 (p-CG-sh) */

/*
 * shifted == 0 follows Alg. 2 literally (delta = (w, u), r -= alpha s,
 * u -= alpha q, w_0 = A u_0).  shifted == 1 follows Alg. 3 with the given
 * sigma.  The two are kept as separate code paths so that the bitwise
 * identity of Alg. 3 at sigma = 0 with Alg. 2 can be tested.
 */
static int solve_pipe(const orc_op *A, const double *dinv, const orc_opts *o, int shifted, const double *b,
                      double *x, orc_result *res)
{
    const int64_t n = A->n;
    const double sigma = shifted ? o->sigma : 0.0;
    double *r = vec(n), *u = vec(n), *w = vec(n), *m = vec(n), *nn = vec(n);
    double *z = vec(n), *q = vec(n), *s = vec(n), *t = vec(n), *p = vec(n);
    double *tmp = vec(n), *tr = vec(n), *gap = vec(n);
    const double bnorm = norm2(n, b);
    res->bnorm = bnorm;
    int replacements = 0;

    /* r_0 := b - A x_0; u_0 := M^{-1} r_0; w_0 := A u_0 (- sigma r_0) */
    apply_A(A, x, tmp);
    for (int64_t k = 0; k < n; ++k) r[k] = st(b[k] - tmp[k]);
    apply_Minv(n, dinv, r, u);
    for (int64_t k = 0; k < n; ++k) u[k] = st(u[k]);
    apply_A(A, u, w);
    if (shifted)
        for (int64_t k = 0; k < n; ++k) w[k] = st(w[k] - sigma * r[k]);
    else
        for (int64_t k = 0; k < n; ++k) w[k] = st(w[k]);
    if (o->w0_perturb)
        for (int64_t k = 0; k < n; ++k) w[k] = st(w[k] + o->w0_perturb[k]);
    /* z_{-1} = q_{-1} = s_{-1} = t_{-1} = p_{-1} = 0 (calloc) */

    const int rr = o->method == ORC_PIPE_RR;
    int rr_count = 0;
    double alpha_prev = 0.0, gamma_prev = 0.0, rho = 0.0;
    int status = ORC_MAX_ITER, i = 0, i_start = 0, last_check = -1;
    for (i = 0;; ++i) {
        const double gamma = dot(n, r, u);                              /* gamma_i := (r_i, u_i) */
        const double delta = shifted ? dot_shift(n, w, sigma, r, u)     /* (w_i + sigma r_i, u_i) */
                                     : dot(n, w, u);                    /* (w_i, u_i)             */
        rho = dot(n, r, r);
        if (res->h_res) res->h_res[i] = sqrt(rho) / bnorm;
        if (res->h_gamma) res->h_gamma[i] = gamma;
        if (res->h_delta) res->h_delta[i] = delta;
        if (res->h_true) {
            true_residual(A, b, x, tmp, tr);
            res->h_true[i] = norm2(n, tr) / bnorm;
        }
        if (!isfinite(rho) || !isfinite(gamma) || !isfinite(delta)) { status = ORC_NONFINITE; break; }
        if (sqrt(rho) <= o->rtol * bnorm) {
            /* optional residual replacement when the explicit residual disagrees */
            if (replacements < o->replace_max) {
                true_residual(A, b, x, tmp, tr);
                if (norm2(n, tr) > o->rtol * bnorm) {
                    /* restart from x: the initialisation steps with x_0 := x_i */
                    ++replacements;
                    for (int64_t k = 0; k < n; ++k) r[k] = st(tr[k]);           /* r := b - A x  */
                    apply_Minv(n, dinv, r, u);
                    for (int64_t k = 0; k < n; ++k) u[k] = st(u[k]);            /* u := M^{-1} r */
                    apply_A(A, u, w);                                           /* w := A u (- sigma r) */
                    if (shifted)
                        for (int64_t k = 0; k < n; ++k) w[k] = st(w[k] - sigma * r[k]);
                    else
                        for (int64_t k = 0; k < n; ++k) w[k] = st(w[k]);
                    memset(z, 0, (size_t)n * sizeof(double));
                    memset(q, 0, (size_t)n * sizeof(double));
                    memset(s, 0, (size_t)n * sizeof(double));
                    memset(t, 0, (size_t)n * sizeof(double));
                    memset(p, 0, (size_t)n * sizeof(double));
                    i_start = i;
                    --i;  /* redo the top of iteration i; it takes the first-iteration branch */
                    continue;
                }
            }
            status = ORC_CONVERGED;
            break;
        }
        if (i >= o->max_iter) { status = ORC_MAX_ITER; break; }
        if (rr && i > i_start && i % o->rr_period == 0 && i != last_check) {
            /* p-CG-rr: measure the residual gap; reset r, u, w, s, q, z to their
             * true values when it has grown past tau ||r_i|| */
            last_check = i;
            true_residual(A, b, x, tmp, tr);
            for (int64_t k = 0; k < n; ++k) gap[k] = tr[k] - r[k];
            const double gnorm = norm2(n, gap);
            abs_scale(A, x, b, tmp);
            const double floor = 0x1p-53 * norm2(n, tmp);   /* rounding scale of b - A x */
            if (gnorm > o->rr_tau * sqrt(rho) && gnorm > o->rr_floor * floor) {
                ++rr_count;
                for (int64_t k = 0; k < n; ++k) r[k] = st(tr[k]);     /* r := b - A x_i      */
                apply_Minv(n, dinv, r, u);
                for (int64_t k = 0; k < n; ++k) u[k] = st(u[k]);      /* u := M^{-1} r       */
                apply_A(A, p, tmp);
                for (int64_t k = 0; k < n; ++k) s[k] = st(tmp[k]);    /* s := A p_{i-1}      */
                apply_Minv(n, dinv, s, q);
                for (int64_t k = 0; k < n; ++k) q[k] = st(q[k]);      /* q := M^{-1} s       */
                apply_A(A, u, w);
                for (int64_t k = 0; k < n; ++k) w[k] = st(w[k]);      /* w := A u            */
                apply_A(A, q, z);
                for (int64_t k = 0; k < n; ++k) z[k] = st(z[k]);      /* z := A q            */
                --i;  /* redo the top of iteration i from its dot products */
                continue;
            }
        }
        if (!o->ignore_breakdown && (!(gamma > 0.0) || !(delta > 0.0))) { status = ORC_BREAKDOWN; break; }
        if (res->snap && i == o->snap_iter) {
            const double *v[ORC_NVEC] = {r, u, w, z, q, s, t, p, dinv};
            dump_vecs(res->snap, n, v);
        }

        apply_Minv(n, dinv, w, m);                 /* m_i := M^{-1} w_i   */
        apply_A(A, m, nn);                         /* n_i := A m_i        */
        double alpha, beta;
        if (i > i_start) {
            beta = gamma / gamma_prev;
            alpha = 1.0 / (delta / gamma - beta / alpha_prev);
        } else {
            beta = 0.0;
            alpha = gamma / delta;
        }
        if (res->h_alpha) res->h_alpha[i] = alpha;
        if (res->h_beta) res->h_beta[i] = beta;
        if (!o->ignore_breakdown && !finite_pos(alpha)) { status = ORC_BREAKDOWN; break; }

        aypx(n, nn, beta, z);                      /* z_i := n_i + beta z_{i-1} */
        aypx(n, m, beta, q);                       /* q_i := m_i + beta q_{i-1} */
        aypx(n, w, beta, s);                       /* s_i := w_i + beta s_{i-1} */
        aypx(n, r, beta, t);                       /* t_i := r_i + beta t_{i-1} */
        aypx(n, u, beta, p);                       /* p_i := u_i + beta p_{i-1} */
        axpy_x(n, alpha, p, x);                    /* x_{i+1} := x_i + alpha p_i */
        if (shifted) {
            const double as = alpha * sigma;
            ymax3(n, alpha, s, as, t, r);          /* r_{i+1} := r_i - alpha s_i - alpha sigma t_i */
            ymax3(n, alpha, q, as, p, u);          /* u_{i+1} := u_i - alpha q_i - alpha sigma p_i */
        } else {
            ymax(n, alpha, s, r);                  /* r_{i+1} := r_i - alpha s_i */
            ymax(n, alpha, q, u);                  /* u_{i+1} := u_i - alpha q_i */
        }
        ymax(n, alpha, z, w);                      /* w_{i+1} := w_i - alpha z_i */

        if (o->record_gaps) {
            /* f_{i+1} = (b - A x_{i+1}) - r_{i+1} */
            if (res->h_f) {
                true_residual(A, b, x, tmp, gap);
                for (int64_t k = 0; k < n; ++k) gap[k] = gap[k] - r[k];
                res->h_f[i + 1] = norm2(n, gap);
            }
            /* g_i = (A p_i - sigma t_i) - s_i */
            if (res->h_g) {
                apply_A(A, p, tmp);
                for (int64_t k = 0; k < n; ++k) gap[k] = (tmp[k] - sigma * t[k]) - s[k];
                res->h_g[i] = norm2(n, gap);
            }
            /* h_{i+1} = (A u_{i+1} - sigma r_{i+1}) - w_{i+1} */
            if (res->h_h) {
                apply_A(A, u, tmp);
                for (int64_t k = 0; k < n; ++k) gap[k] = (tmp[k] - sigma * r[k]) - w[k];
                res->h_h[i + 1] = norm2(n, gap);
            }
            /* j_i = A q_i - z_i */
            if (res->h_j) {
                apply_A(A, q, tmp);
                for (int64_t k = 0; k < n; ++k) gap[k] = tmp[k] - z[k];
                res->h_j[i] = norm2(n, gap);
            }
        }
        alpha_prev = alpha;
        gamma_prev = gamma;
    }
    res->status = status;
    res->iterations = i;
    res->replacements = replacements + rr_count;
    res->rel_res_recursive = sqrt(rho) / bnorm;
    true_residual(A, b, x, tmp, tr);
    res->rel_res_true = norm2(n, tr) / bnorm;
    if (res->final_vecs) {
        const double *v[ORC_NVEC] = {r, u, w, z, q, s, t, p, dinv};
        dump_vecs(res->final_vecs, n, v);
    }
    free(r); free(u); free(w); free(m); free(nn);
    free(z); free(q); free(s); free(t); free(p);
    free(tmp); free(tr); free(gap);
    return 0;
}

/* ------------------------------------------------------------ entry points */

/* Solve A x = b; x holds x_0 on entry and the final iterate on return.
 * Returns 0, or -1 on invalid arguments. */
/* sigma_k of the schedule, k >= -1 (entry k + 1; the last entry repeats) */
static double sched_at(const orc_opts *o, int k)
{
    int idx = k + 1;
    if (idx > o->sigma_sched_len - 1) idx = o->sigma_sched_len - 1;
    return o->sigma_sched[idx];
}

/* Alg. 4 (Section 4.1): pipelined CG with the shift sigma_i of iteration i
 * taken from a schedule.  w_i is kept equal to A u_i - sigma_{i-1} r_i and
 * s_i to A p_i - sigma_i t_i, the corrections (sigma_i - sigma_{i-1}) (.)
 * keeping the auxiliary recurrences consistent with the changing shift. */
static int solve_pipe_var(const orc_op *A, const double *dinv, const orc_opts *o, const double *b, double *x,
                          orc_result *res)
{
    const int64_t n = A->n;
    double *r = vec(n), *u = vec(n), *w = vec(n), *m = vec(n), *nn = vec(n);
    double *z = vec(n), *q = vec(n), *s = vec(n), *t = vec(n), *p = vec(n);
    double *tmp = vec(n), *tr = vec(n), *gap = vec(n);
    const double bnorm = norm2(n, b);
    res->bnorm = bnorm;
    int replacements = 0;

    /* r_0 := b - A x_0; u_0 := M^{-1} r_0; w_0 := A u_0 - sigma_{-1} r_0 */
    apply_A(A, x, tmp);
    for (int64_t k = 0; k < n; ++k) r[k] = st(b[k] - tmp[k]);
    apply_Minv(n, dinv, r, u);
    for (int64_t k = 0; k < n; ++k) u[k] = st(u[k]);
    apply_A(A, u, w);
    {
        const double s_m1 = sched_at(o, -1);
        for (int64_t k = 0; k < n; ++k) w[k] = st(w[k] - s_m1 * r[k]);
    }
    if (o->w0_perturb)
        for (int64_t k = 0; k < n; ++k) w[k] = st(w[k] + o->w0_perturb[k]);

    double alpha_prev = 0.0, gamma_prev = 0.0, rho = 0.0;
    int status = ORC_MAX_ITER, i = 0, i_start = 0;
    for (i = 0;; ++i) {
        const double sig_prev = sched_at(o, i - 1), sig = sched_at(o, i), d = sig - sig_prev;
        const double gamma = dot(n, r, u);                     /* gamma_i := (r_i, u_i)              */
        const double delta = dot_shift(n, w, sig_prev, r, u);  /* (w_i + sigma_{i-1} r_i, u_i)       */
        rho = dot(n, r, r);
        if (res->h_res) res->h_res[i] = sqrt(rho) / bnorm;
        if (res->h_gamma) res->h_gamma[i] = gamma;
        if (res->h_delta) res->h_delta[i] = delta;
        if (res->h_true) {
            true_residual(A, b, x, tmp, tr);
            res->h_true[i] = norm2(n, tr) / bnorm;
        }
        if (!isfinite(rho) || !isfinite(gamma) || !isfinite(delta)) { status = ORC_NONFINITE; break; }
        if (sqrt(rho) <= o->rtol * bnorm) {
            if (replacements < o->replace_max) {
                true_residual(A, b, x, tmp, tr);
                if (norm2(n, tr) > o->rtol * bnorm) {
                    /* restart from x: w := A u - sigma_{i-1} r keeps w's definition */
                    ++replacements;
                    for (int64_t k = 0; k < n; ++k) r[k] = st(tr[k]);
                    apply_Minv(n, dinv, r, u);
                    for (int64_t k = 0; k < n; ++k) u[k] = st(u[k]);
                    apply_A(A, u, w);
                    for (int64_t k = 0; k < n; ++k) w[k] = st(w[k] - sig_prev * r[k]);
                    memset(z, 0, (size_t)n * sizeof(double));
                    memset(q, 0, (size_t)n * sizeof(double));
                    memset(s, 0, (size_t)n * sizeof(double));
                    memset(t, 0, (size_t)n * sizeof(double));
                    memset(p, 0, (size_t)n * sizeof(double));
                    i_start = i;
                    --i;
                    continue;
                }
            }
            status = ORC_CONVERGED;
            break;
        }
        if (i >= o->max_iter) { status = ORC_MAX_ITER; break; }
        if (!o->ignore_breakdown && (!(gamma > 0.0) || !(delta > 0.0))) { status = ORC_BREAKDOWN; break; }
        if (res->snap && i == o->snap_iter) {
            const double *v[ORC_NVEC] = {r, u, w, z, q, s, t, p, dinv};
            dump_vecs(res->snap, n, v);
        }

        apply_Minv(n, dinv, w, m);                 /* m_i := M^{-1} w_i   */
        apply_A(A, m, nn);                         /* n_i := A m_i        */
        double alpha, beta;
        if (i > i_start) {
            beta = gamma / gamma_prev;
            alpha = 1.0 / (delta / gamma - beta / alpha_prev);
        } else {
            beta = 0.0;
            alpha = gamma / delta;
        }
        if (res->h_alpha) res->h_alpha[i] = alpha;
        if (res->h_beta) res->h_beta[i] = beta;
        if (!o->ignore_breakdown && !finite_pos(alpha)) { status = ORC_BREAKDOWN; break; }

        aypx(n, r, beta, t);                       /* t_i := r_i + beta t_{i-1} */
        aypx(n, u, beta, p);                       /* p_i := u_i + beta p_{i-1} */
        aypx_corr(n, w, beta, d, t, s);            /* s_i := w_i + beta s_{i-1} - d t_i */
        aypx_corr(n, m, beta, d, p, q);            /* q_i := m_i + beta q_{i-1} - d p_i */
        z_var(n, nn, beta, d, s, sig, t, z);       /* z_i := n_i + beta z_{i-1} - d (s_i + sigma_i t_i) */
        axpy_x(n, alpha, p, x);                    /* x_{i+1} := x_i + alpha p_i */
        ymax_corr(n, alpha, z, d, r, w);           /* w_{i+1} := w_i - alpha z_i - d r_i (old r_i) */
        {
            const double as = alpha * sig;
            ymax3(n, alpha, s, as, t, r);          /* r_{i+1} := r_i - alpha s_i - alpha sigma_i t_i */
            ymax3(n, alpha, q, as, p, u);          /* u_{i+1} := u_i - alpha q_i - alpha sigma_i p_i */
        }

        if (o->record_gaps) {
            if (res->h_f) {                        /* f_{i+1} = (b - A x_{i+1}) - r_{i+1} */
                true_residual(A, b, x, tmp, gap);
                for (int64_t k = 0; k < n; ++k) gap[k] = gap[k] - r[k];
                res->h_f[i + 1] = norm2(n, gap);
            }
            if (res->h_g) {                        /* g_i = (A p_i - sigma_i t_i) - s_i */
                apply_A(A, p, tmp);
                for (int64_t k = 0; k < n; ++k) gap[k] = (tmp[k] - sig * t[k]) - s[k];
                res->h_g[i] = norm2(n, gap);
            }
            if (res->h_h) {                        /* h_{i+1} = (A u_{i+1} - sigma_i r_{i+1}) - w_{i+1} */
                apply_A(A, u, tmp);
                for (int64_t k = 0; k < n; ++k) gap[k] = (tmp[k] - sig * r[k]) - w[k];
                res->h_h[i + 1] = norm2(n, gap);
            }
            if (res->h_j) {                        /* j_i = A q_i - z_i */
                apply_A(A, q, tmp);
                for (int64_t k = 0; k < n; ++k) gap[k] = tmp[k] - z[k];
                res->h_j[i] = norm2(n, gap);
            }
        }
        alpha_prev = alpha;
        gamma_prev = gamma;
    }
    res->status = status;
    res->iterations = i;
    res->replacements = replacements;
    res->rel_res_recursive = sqrt(rho) / bnorm;
    true_residual(A, b, x, tmp, tr);
    res->rel_res_true = norm2(n, tr) / bnorm;
    if (res->final_vecs) {
        const double *v[ORC_NVEC] = {r, u, w, z, q, s, t, p, dinv};
        dump_vecs(res->final_vecs, n, v);
    }
    free(r); free(u); free(w); free(m); free(nn);
    free(z); free(q); free(s); free(t); free(p);
    free(tmp); free(tr); free(gap);
    return 0;
}

int orc_solve(const orc_op *A, const orc_opts *o, const double *b, double *x, orc_result *res)
{
    if (!A || !o || !b || !x || !res || A->n <= 0) return -1;
    if (o->method < ORC_CG || o->method > ORC_PIPE_RR) return -1;
    if (o->method == ORC_PIPE_RR && (o->rr_period < 1 || !(o->rr_tau > 0.0))) return -1;
    if (o->method == ORC_PIPE_VAR && (!o->sigma_sched || o->sigma_sched_len < 1)) return -1;
#ifdef _OPENMP
    int saved = omp_get_max_threads();
    if (o->threads > 0) omp_set_num_threads(o->threads);
#endif
    g_fp32 = o->fp32_storage ? 1 : 0;
    double *dinv = NULL;
    if (o->jacobi) {
        dinv = vec(A->n);
        jacobi_diag(A, dinv);
    }
    int rc;
    if (o->method == ORC_CG)
        rc = solve_cg(A, dinv, o, b, x, res);
    else if (o->method == ORC_PIPE_VAR)
        rc = solve_pipe_var(A, dinv, o, b, x, res);
    else
        rc = solve_pipe(A, dinv, o, o->method == ORC_PIPE_SHIFT, b, x, res);
    free(dinv);
    g_fp32 = 0;
#ifdef _OPENMP
    omp_set_num_threads(saved);
#endif
    return rc;
}

/* out = A v (exposed so that tests can check the operator against its definition) */
int orc_apply_A(const orc_op *A, const double *v, double *out)
{
    if (!A || !v || !out || A->n <= 0) return -1;
    apply_A(A, v, out);
    return 0;
}

/* chunked dot product (exposed for the determinism pin) */
double orc_dot(int64_t n, const double *a, const double *b, int threads)
{
#ifdef _OPENMP
    int saved = omp_get_max_threads();
    if (threads > 0) omp_set_num_threads(threads);
#endif
    double d = dot(n, a, b);
#ifdef _OPENMP
    omp_set_num_threads(saved);
#endif
    return d;
}

/* number of OpenMP threads a solve with threads <= 0 would use */
int orc_max_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
