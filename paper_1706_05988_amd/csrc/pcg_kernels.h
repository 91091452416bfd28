// pcg_kernels.h -- the HIP kernels of one solve (single system).
//
// Storage type T is double (binary64 form) or float (FP32-stream form: the
// Krylov vectors, CSR values and Jacobi diagonal stream in binary32 while
// every operation, the dot products, the scalars and x stay binary64; each
// stored value is rounded once at its store and all later uses see the
// stored bits).
//
// Passes of shifted pipelined CG (Alg. 3; Alg. 2 is sigma = 0):
//   k_init0    r_0 := b - A x_0, u_0 := M^-1 r_0; block partials of (b, b)
//   k_init1    head: ||b||^2 (stage 2);  w_0 := A u_0 - sigma r_0;
//              partials of gamma_0, delta_0, rho_0
//   k_pipe     one whole iteration i (see the kernel)
// Passes of classic CG (Alg. 1, two fused passes per iteration):
//   k_init0    r_0 := b - A x_0; partials of (b, b)
//   k_cg_init1 head: ||b||^2; partials of gamma_0 = (r_0, u_0), rho_0
//   k_cg_a     head: gamma_i, rho_i -> stop test, beta_i; p_i := u_i + beta_i p_{i-1}
//              (recomputed at the stencil neighbours), s_i := A p_i; partial (s_i, p_i)
//   k_cg_b     head: (s_i, p_i) -> alpha_i; x, r updates, u := M^-1 r;
//              partials of gamma_{i+1}, rho_{i+1}
// Support:
//   k_resid    partials of ||b - A x||^2 (explicit residual, binary64)
//   k_reduce   one block: stage 2 of a partial array into the state
//   k_jacobi   dinv_k := 1 / a_kk for CSR operators
#pragma once

#include "pcg_device.h"

namespace pcg {

template <typename T>
struct PassArgs {
    OpDev<T> A;
    const T *dinv;        // CSR Jacobi diagonal inverse (nullptr otherwise)
    double dinv_s;        // stencil Jacobi: 1/(diag + shift); 1.0 without preconditioner
    const double *b;
    double *x;
    T *r, *u;             // u == r without preconditioner
    const T *w_in;        // w_i (or, in CG, p_{i-1})
    T *w_out;             // w_{i+1} (or, in CG, p_i)
    T *z, *q, *s, *t, *p; // q == s and p == t without preconditioner
    const double *part_in;
    double *part_out;
    int32_t nparts;       // partials in part_in (= grid size of the previous pass)
    int32_t ntiles;
    const DevState *st_in;
    DevState *st_out;
    double *hist;         // history rows (5 doubles) or nullptr
    int32_t hist_cap;
    int32_t max_iter;
    double sigma;
    double rtol;
    int32_t i0;           // init passes: iteration count at which the (re)start happens
    int32_t xcd_map;
};

// M^{-1} applied at index k to the stored value v (binary64 product of the
// stored diagonal inverse and v).
template <typename T, bool JAC, int OP>
__device__ __forceinline__ double minv(const PassArgs<T> &a, uint32_t k, double v)
{
    if constexpr (!JAC) {
        return v;
    } else if constexpr (OP == OP_CSR) {
        return (double)a.dinv[k] * v;
    } else {
        return a.dinv_s * v;
    }
}

__device__ __forceinline__ void write_hist(double *h, int cap, int i, double res, double alpha, double beta,
                                           double gamma, double delta)
{
    if (h && i >= 0 && i < cap) {
        double *row = h + (size_t)i * 5;
        row[0] = res;
        row[1] = alpha;
        row[2] = beta;
        row[3] = gamma;
        row[4] = delta;
    }
}

// ----------------------------------------------------------------- init 0

// r_0 := b - A x_0 (stored), and for the pipelined methods with a
// preconditioner u_0 := M^-1 r_0 (stored).  Partials of (b, b).
template <typename T, int OP, bool JAC, bool STORE_U, int EPT>
__global__ void __launch_bounds__(1024) k_init0(PassArgs<T> a)
{
    __shared__ double lds[kMaxWaves * kFields];
    double acc[1] = {0.0};
    const TileRange tr = tile_range(a.ntiles, a.xcd_map);
    const uint32_t tile_elems = blockDim.x * EPT;
    for (int tile = tr.first; tile < tr.end; tile += tr.step) {
#pragma unroll
        for (int j = 0; j < EPT; ++j) {
            const uint32_t e = (uint32_t)tile * tile_elems + j * blockDim.x + threadIdx.x;
            if (e < (uint32_t)a.A.n) {
                const double be = a.b[e];
                const double ax = apply_row<OP>(a.A, e, [&](uint32_t k) { return a.x[k]; });
                const double r = rnd<T>(be - ax);
                a.r[e] = (T)r;
                if constexpr (STORE_U) a.u[e] = (T)minv<T, JAC, OP>(a, e, r);
                acc[0] += be * be;
            }
        }
    }
    block_sum<1>(acc, lds);
    store_partial<1>(a.part_out, acc);
}

// ----------------------------------------------------------------- init 1 (pipelined)

// head: ||b||^2 from the init-0 partials; w_0 := A u_0 - sigma r_0 into
// w_out; partials of gamma_0 = (r, u), delta_0 = (w + sigma r, u), rho_0.
// Block 0 writes the state for iteration i0.
template <typename T, int OP, bool JAC, int EPT>
__global__ void __launch_bounds__(1024) k_init1(PassArgs<T> a)
{
    __shared__ double lds[kMaxWaves * kFields];
    double bb[1];
    stage2<1>(a.part_in, a.nparts, bb, lds);
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        DevState o{};
        o.bnorm2 = bb[0];
        o.iter = a.i0;
        o.i_start = a.i0;
        o.status = isfinite(bb[0]) ? RUNNING : ST_NONFINITE;
        o.true_res2 = __builtin_nan("");
        *a.st_out = o;
    }
    const T *u = JAC ? a.u : a.r;
    double acc[3] = {0.0, 0.0, 0.0};
    const TileRange tr = tile_range(a.ntiles, a.xcd_map);
    const uint32_t tile_elems = blockDim.x * EPT;
    for (int tile = tr.first; tile < tr.end; tile += tr.step) {
#pragma unroll
        for (int j = 0; j < EPT; ++j) {
            const uint32_t e = (uint32_t)tile * tile_elems + j * blockDim.x + threadIdx.x;
            if (e < (uint32_t)a.A.n) {
                const double au = apply_row<OP>(a.A, e, [&](uint32_t k) { return ld(u, k); });
                const double r = ld(a.r, e), ue = ld(u, e);
                const double w = rnd<T>(au - a.sigma * r);
                a.w_out[e] = (T)w;
                acc[0] += r * ue;
                acc[1] += (w + a.sigma * r) * ue;
                acc[2] += r * r;
            }
        }
    }
    block_sum<3>(acc, lds);
    store_partial<3>(a.part_out, acc);
}

// ----------------------------------------------------------------- p-CG(-sh) iteration

// One iteration i of Alg. 3 as one pass:
//   head (every block, identical bits): gamma_i, delta_i, rho_i from the
//     previous pass's partials; stop test sqrt(rho_i) <= rtol ||b||, cap,
//     breakdown; beta_i = gamma_i / gamma_{i-1},
//     alpha_i = (delta_i / gamma_i - beta_i / alpha_{i-1})^-1 (i = i_start:
//     beta = 0, alpha = gamma / delta)
//   body (per unknown):  m = M^-1 w_i, n = A m (stencil / CSR over m at the
//     neighbours), then
//     z := n + beta z   q := m + beta q   s := w + beta s   t := r + beta t
//     p := u + beta p   x := x + alpha p
//     r := r - (alpha s + (alpha sigma) t)   u := u - (alpha q + (alpha sigma) p)
//     w_{i+1} := w - alpha z  (into the other w buffer: neighbours read w_i)
//   tail: block partials of gamma_{i+1} = (r, u),
//     delta_{i+1} = (w_{i+1} + sigma r, u), rho_{i+1} = (r, r).
template <typename T, int OP, bool JAC, int EPT>
__global__ void __launch_bounds__(1024) k_pipe(PassArgs<T> a)
{
    __shared__ double lds[kMaxWaves * kFields];
    const DevState S = *a.st_in;
    if (S.status != RUNNING) {
        if (blockIdx.x == 0 && threadIdx.x == 0) *a.st_out = S;
        return;
    }
    double tot[3];
    stage2<3>(a.part_in, a.nparts, tot, lds);
    const double gamma = tot[0], delta = tot[1], rho = tot[2];
    const int i = S.iter;
    int status = RUNNING;
    double alpha = __builtin_nan(""), beta = __builtin_nan("");
    if (!isfinite(gamma) || !isfinite(delta) || !isfinite(rho)) {
        status = ST_NONFINITE;
    } else if (sqrt(rho) <= a.rtol * sqrt(S.bnorm2)) {
        status = ST_CONVERGED;
    } else if (i >= a.max_iter) {
        status = ST_MAX_ITER;
    } else if (!(gamma > 0.0) || !(delta > 0.0)) {
        status = ST_BREAKDOWN;
    } else {
        if (i > S.i_start) {
            beta = gamma / S.gamma_prev;
            alpha = 1.0 / (delta / gamma - beta / S.alpha_prev);
        } else {
            beta = 0.0;
            alpha = gamma / delta;
        }
        if (!(isfinite(alpha) && alpha > 0.0)) status = ST_BREAKDOWN;
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        DevState o = S;
        o.rho = rho;
        if (status != RUNNING) {
            o.status = status;
        } else {
            o.iter = i + 1;
            o.alpha_prev = alpha;
            o.gamma_prev = gamma;
        }
        write_hist(a.hist, a.hist_cap, i, sqrt(rho / S.bnorm2), alpha, beta, gamma, delta);
        *a.st_out = o;
    }
    if (status != RUNNING) return;

    const bool first = (i == S.i_start);
    const double sigma = a.sigma, as = alpha * sigma;
    T *const u = JAC ? a.u : a.r;
    T *const q = JAC ? a.q : a.s;
    T *const p = JAC ? a.p : a.t;
    double acc[3] = {0.0, 0.0, 0.0};
    const TileRange tr = tile_range(a.ntiles, a.xcd_map);
    const uint32_t tile_elems = blockDim.x * EPT;
    for (int tile = tr.first; tile < tr.end; tile += tr.step) {
#pragma unroll
        for (int j = 0; j < EPT; ++j) {
            const uint32_t e = (uint32_t)tile * tile_elems + j * blockDim.x + threadIdx.x;
            if (e >= (uint32_t)a.A.n) continue;
            // preconditioner and SPMV on the fly: m, n never stored
            const double we = ld(a.w_in, e);
            const double me = minv<T, JAC, OP>(a, e, we);
            const double ne = apply_row<OP>(a.A, e, [&](uint32_t k) { return minv<T, JAC, OP>(a, k, ld(a.w_in, k)); });
            const double re = ld(a.r, e);
            const double ue = JAC ? ld(u, e) : re;
            const double zo = first ? 0.0 : ld(a.z, e);
            const double so = first ? 0.0 : ld(a.s, e);
            const double to = first ? 0.0 : ld(a.t, e);
            // beta-recurrences
            const double z = rnd<T>(ne + beta * zo);
            const double s = rnd<T>(we + beta * so);
            const double t = rnd<T>(re + beta * to);
            a.z[e] = (T)z;
            a.s[e] = (T)s;
            a.t[e] = (T)t;
            double qv = s, pv = t;
            if constexpr (JAC) {
                const double qo = first ? 0.0 : ld(q, e);
                const double po = first ? 0.0 : ld(p, e);
                qv = rnd<T>(me + beta * qo);
                pv = rnd<T>(ue + beta * po);
                q[e] = (T)qv;
                p[e] = (T)pv;
            }
            // alpha-recurrences with the shift terms grouped first
            a.x[e] = a.x[e] + alpha * pv;
            const double rn = rnd<T>(re - (alpha * s + as * t));
            a.r[e] = (T)rn;
            double un = rn;
            if constexpr (JAC) {
                un = rnd<T>(ue - (alpha * qv + as * pv));
                u[e] = (T)un;
            }
            const double wn = rnd<T>(we - alpha * z);
            a.w_out[e] = (T)wn;
            // next iteration's dot products
            acc[0] += rn * un;
            acc[1] += (wn + sigma * rn) * un;
            acc[2] += rn * rn;
        }
    }
    block_sum<3>(acc, lds);
    store_partial<3>(a.part_out, acc);
}

// ----------------------------------------------------------------- classic CG

// head: ||b||^2; partials of gamma_0 = (r_0, M^-1 r_0) and rho_0.
template <typename T, int OP, bool JAC, int EPT>
__global__ void __launch_bounds__(1024) k_cg_init1(PassArgs<T> a)
{
    __shared__ double lds[kMaxWaves * kFields];
    double bb[1];
    stage2<1>(a.part_in, a.nparts, bb, lds);
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        DevState o{};
        o.bnorm2 = bb[0];
        o.iter = a.i0;
        o.i_start = a.i0;
        o.status = isfinite(bb[0]) ? RUNNING : ST_NONFINITE;
        o.true_res2 = __builtin_nan("");
        *a.st_out = o;
    }
    double acc[2] = {0.0, 0.0};
    const TileRange tr = tile_range(a.ntiles, a.xcd_map);
    const uint32_t tile_elems = blockDim.x * EPT;
    for (int tile = tr.first; tile < tr.end; tile += tr.step) {
#pragma unroll
        for (int j = 0; j < EPT; ++j) {
            const uint32_t e = (uint32_t)tile * tile_elems + j * blockDim.x + threadIdx.x;
            if (e < (uint32_t)a.A.n) {
                const double r = ld(a.r, e);
                const double u = rnd<T>(minv<T, JAC, OP>(a, e, r));
                acc[0] += r * u;
                acc[1] += r * r;
            }
        }
    }
    block_sum<2>(acc, lds);
    store_partial<2>(a.part_out, acc);
}

// Pass A of CG iteration i.  w_in = p_{i-1}, w_out = p_i.
template <typename T, int OP, bool JAC, int EPT>
__global__ void __launch_bounds__(1024) k_cg_a(PassArgs<T> a)
{
    __shared__ double lds[kMaxWaves * kFields];
    const DevState S = *a.st_in;
    if (S.status != RUNNING) {
        if (blockIdx.x == 0 && threadIdx.x == 0) *a.st_out = S;
        return;
    }
    double tot[2];
    stage2<2>(a.part_in, a.nparts, tot, lds);
    const double gamma = tot[0], rho = tot[1];
    const int i = S.iter;
    int status = RUNNING;
    double beta = 0.0;
    if (!isfinite(gamma) || !isfinite(rho)) {
        status = ST_NONFINITE;
    } else if (sqrt(rho) <= a.rtol * sqrt(S.bnorm2)) {
        status = ST_CONVERGED;
    } else if (i >= a.max_iter) {
        status = ST_MAX_ITER;
    } else if (!(gamma > 0.0)) {
        status = ST_BREAKDOWN;
    } else if (i > S.i_start) {
        beta = gamma / S.gamma_prev;  // beta_i = (r_i, u_i) / (r_{i-1}, u_{i-1})
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        DevState o = S;
        o.rho = rho;
        o.gamma = gamma;
        if (status != RUNNING) o.status = status;
        write_hist(a.hist, a.hist_cap, i, sqrt(rho / S.bnorm2), __builtin_nan(""),
                   status == RUNNING ? beta : __builtin_nan(""), gamma, __builtin_nan(""));
        *a.st_out = o;
    }
    if (status != RUNNING) return;

    const bool first = (i == S.i_start);
    // p_i at index k, recomputed identically wherever it is needed
    auto pnew = [&](uint32_t k) {
        const double uk = rnd<T>(minv<T, JAC, OP>(a, k, ld(a.r, k)));
        return rnd<T>(uk + beta * (first ? 0.0 : ld(a.w_in, k)));
    };
    double acc[1] = {0.0};
    const TileRange tr = tile_range(a.ntiles, a.xcd_map);
    const uint32_t tile_elems = blockDim.x * EPT;
    for (int tile = tr.first; tile < tr.end; tile += tr.step) {
#pragma unroll
        for (int j = 0; j < EPT; ++j) {
            const uint32_t e = (uint32_t)tile * tile_elems + j * blockDim.x + threadIdx.x;
            if (e >= (uint32_t)a.A.n) continue;
            const double pe = pnew(e);
            const double se = rnd<T>(apply_row<OP>(a.A, e, pnew));
            a.w_out[e] = (T)pe;
            a.s[e] = (T)se;
            acc[0] += se * pe;
        }
    }
    block_sum<1>(acc, lds);
    store_partial<1>(a.part_out, acc);
}

// Pass B of CG iteration i.  w_out = p_i (written by pass A).
template <typename T, int OP, bool JAC, int EPT>
__global__ void __launch_bounds__(1024) k_cg_b(PassArgs<T> a)
{
    __shared__ double lds[kMaxWaves * kFields];
    const DevState S = *a.st_in;
    if (S.status != RUNNING) {
        if (blockIdx.x == 0 && threadIdx.x == 0) *a.st_out = S;
        return;
    }
    double tot[1];
    stage2<1>(a.part_in, a.nparts, tot, lds);
    const double sp = tot[0];
    const int i = S.iter;
    int status = RUNNING;
    double alpha = __builtin_nan("");
    if (!isfinite(sp)) {
        status = ST_NONFINITE;
    } else if (!(sp > 0.0)) {
        status = ST_BREAKDOWN;
    } else {
        alpha = S.gamma / sp;  // alpha_i = (r_i, u_i) / (s_i, p_i)
        if (!(isfinite(alpha) && alpha > 0.0)) status = ST_BREAKDOWN;
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        DevState o = S;
        if (status != RUNNING) {
            o.status = status;
        } else {
            o.iter = i + 1;
            o.gamma_prev = S.gamma;
            o.alpha_prev = alpha;
        }
        if (a.hist && i < a.hist_cap) {
            a.hist[(size_t)i * 5 + 1] = alpha;
            a.hist[(size_t)i * 5 + 4] = sp;
        }
        *a.st_out = o;
    }
    if (status != RUNNING) return;

    double acc[2] = {0.0, 0.0};
    const TileRange tr = tile_range(a.ntiles, a.xcd_map);
    const uint32_t tile_elems = blockDim.x * EPT;
    for (int tile = tr.first; tile < tr.end; tile += tr.step) {
#pragma unroll
        for (int j = 0; j < EPT; ++j) {
            const uint32_t e = (uint32_t)tile * tile_elems + j * blockDim.x + threadIdx.x;
            if (e >= (uint32_t)a.A.n) continue;
            const double pe = ld(a.w_out, e);
            const double se = ld(a.s, e);
            a.x[e] = a.x[e] + alpha * pe;
            const double rn = rnd<T>(ld(a.r, e) - alpha * se);
            a.r[e] = (T)rn;
            const double un = rnd<T>(minv<T, JAC, OP>(a, e, rn));
            acc[0] += rn * un;
            acc[1] += rn * rn;
        }
    }
    block_sum<2>(acc, lds);
    store_partial<2>(a.part_out, acc);
}

// ----------------------------------------------------------------- support

// partials of ||b - A x||^2 and ||b||^2 in binary64 (A in its storage precision).
template <typename T, int OP, int EPT>
__global__ void __launch_bounds__(1024) k_resid(PassArgs<T> a)
{
    __shared__ double lds[kMaxWaves * kFields];
    double acc[2] = {0.0, 0.0};
    const TileRange tr = tile_range(a.ntiles, a.xcd_map);
    const uint32_t tile_elems = blockDim.x * EPT;
    for (int tile = tr.first; tile < tr.end; tile += tr.step) {
#pragma unroll
        for (int j = 0; j < EPT; ++j) {
            const uint32_t e = (uint32_t)tile * tile_elems + j * blockDim.x + threadIdx.x;
            if (e < (uint32_t)a.A.n) {
                const double be = a.b[e];
                const double d = be - apply_row<OP>(a.A, e, [&](uint32_t k) { return a.x[k]; });
                acc[0] += d * d;
                acc[1] += be * be;
            }
        }
    }
    block_sum<2>(acc, lds);
    store_partial<2>(a.part_out, acc);
}

// One block: stage 2 of `nparts` residual partials into out->true_res2 and
// out->spare[0] (= ||b||^2).
__global__ void __launch_bounds__(1024) k_reduce_true(const double *part, int nparts, DevState *out)
{
    __shared__ double lds[kMaxWaves * kFields];
    double tot[2];
    stage2<2>(part, nparts, tot, lds);
    if (threadIdx.x == 0) {
        out->true_res2 = tot[0];
        out->spare[0] = tot[1];
    }
}

// dinv_k := 1 / a_kk (sum of the row's diagonal entries), rounded to T.
template <typename T>
__global__ void k_jacobi(OpDev<T> A, T *dinv)
{
    const uint32_t e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= (uint32_t)A.n) return;
    double d = 0.0;
    for (int32_t k = A.row_ptr[e]; k < A.row_ptr[e + 1]; ++k)
        if ((uint32_t)A.col[k] == e) d += (double)A.val[k];
    dinv[e] = (T)(1.0 / d);
}

// Gershgorin bounds of spec(M^-1 A) for a CSR operator: per block
// min_k (a_kk - R_k)/a_kk' and max_k (a_kk + R_k)/a_kk' with R_k the
// off-diagonal absolute row sum and a_kk' = a_kk with Jacobi, 1 without.
template <typename T>
__global__ void __launch_bounds__(256) k_gershgorin(OpDev<T> A, int jac, double *out /* 2 per block */)
{
    __shared__ double lo_s[256], hi_s[256];
    double lo = __builtin_inf(), hi = -__builtin_inf();
    for (uint32_t e = blockIdx.x * blockDim.x + threadIdx.x; e < (uint32_t)A.n; e += gridDim.x * blockDim.x) {
        double d = 0.0, R = 0.0;
        for (int32_t k = A.row_ptr[e]; k < A.row_ptr[e + 1]; ++k) {
            const double v = (double)A.val[k];
            if ((uint32_t)A.col[k] == e) d += v; else R += fabs(v);
        }
        const double sc = jac ? d : 1.0;
        lo = fmin(lo, (d - R) / sc);
        hi = fmax(hi, (d + R) / sc);
    }
    lo_s[threadIdx.x] = lo;
    hi_s[threadIdx.x] = hi;
    __syncthreads();
    for (int o = blockDim.x / 2; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) {
            lo_s[threadIdx.x] = fmin(lo_s[threadIdx.x], lo_s[threadIdx.x + o]);
            hi_s[threadIdx.x] = fmax(hi_s[threadIdx.x], hi_s[threadIdx.x + o]);
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        out[2 * blockIdx.x] = lo_s[0];
        out[2 * blockIdx.x + 1] = hi_s[0];
    }
}

// Validate a CSR structure on the device: counts rows whose row_ptr is not
// monotone or whose columns fall outside [0, n), and (with Jacobi) rows
// without a positive diagonal.  out[0] += bad rows (atomic, integer).
template <typename T>
__global__ void __launch_bounds__(256) k_csr_check(OpDev<T> A, int need_diag, int64_t nnz, int *out)
{
    int bad = 0;
    for (uint32_t e = blockIdx.x * blockDim.x + threadIdx.x; e < (uint32_t)A.n; e += gridDim.x * blockDim.x) {
        const int32_t k0 = A.row_ptr[e], k1 = A.row_ptr[e + 1];
        if (k0 < 0 || k1 < k0 || (int64_t)k1 > nnz) { ++bad; continue; }
        double d = 0.0;
        bool col_ok = true;
        for (int32_t k = k0; k < k1; ++k) {
            const int32_t c = A.col[k];
            if (c < 0 || c >= A.n) col_ok = false;
            else if ((uint32_t)c == e) d += (double)A.val[k];
        }
        if (!col_ok || (need_diag && !(d > 0.0))) ++bad;
    }
    if (bad) atomicAdd(out, bad);
}

}  // namespace pcg
