// pcg_kernels.h -- the HIP kernels of one solve (single system).
//
// Storage type T is double (binary64 form) or float (FP32-stream form: the
// Krylov vectors, CSR values and Jacobi diagonal stream in binary32 while
// every operation, the dot products, the scalars and x stay binary64; each
// stored value is rounded once at its store and all later uses see the
// stored bits).
//
// The solver's vectors (an internal copy of x, and r, u, w, w', z, q, s, t,
// p) are blocked in the workspace (see slot_ptr in pcg_device.h); b and the
// caller's x are plain vectors.
//
// Passes of shifted pipelined CG (Alg. 3; Alg. 2 is sigma = 0):
//   k_copy_x   caller x -> internal x (solve start) and back (solve end)
//   k_init0    r_0 := b - A x_0, u_0 := M^-1 r_0; clears z, q, s, t, p;
//              block partials of (b, b)
//   k_init1    head: ||b||^2 (stage 2);  w_0 := A u_0 - sigma r_0;
//              partials of gamma_0, delta_0, rho_0
//   k_pipe     one whole iteration i (see the kernel); x is written every
//              other iteration, and k_x_fixup completes it when a solve
//              stops after a pass that skipped it
//   k_pipe_rr  the same with automated residual replacement (p-CG-rr)
// Passes of classic CG (Alg. 1, two fused passes per iteration):
//   k_init0    r_0 := b - A x_0; clears p_{-1}; partials of (b, b)
//   k_cg_init1 head: ||b||^2; partials of gamma_0 = (r_0, u_0), rho_0
//   k_cg_a     head: gamma_i, rho_i -> stop test, beta_i; p_i := u_i + beta_i p_{i-1}
//              (recomputed at the stencil neighbours), s_i := A p_i; partial (s_i, p_i)
//   k_cg_a_zm  the same on a 3-D grid, marching along z with the p_i planes in LDS
//   k_cg_b     head: (s_i, p_i) -> alpha_i; x, r updates, u := M^-1 r;
//              partials of gamma_{i+1}, rho_{i+1}
// Support:
//   k_resid    partials of ||b - A x||^2 and ||b||^2 (explicit residual, binary64)
//   k_reduce_true  one block: stage 2 of the residual partials into the state
//   k_jacobi   dinv_k := 1 / a_kk for CSR operators
//   k_gershgorin, k_csr_check   CSR set-up
#pragma once

#include "pcg_device.h"

namespace pcg {

// init-0 clear mask
enum ClearBits : uint32_t { CLR_Z = 1, CLR_Q = 2, CLR_S = 4, CLR_T = 8, CLR_P = 16, CLR_WIN = 32 };

// Work split of the z-marching CG pass A on a 3-D grid: a work item is
// `rows` consecutive grid rows (y) of a plane over `seg` consecutive planes
// (z); nchunks * nsegs items.  rows = 0: the plain pass A.
struct CgZm {
    int32_t rows, seg, nchunks, nsegs;
};

// Points of a plane window each thread of the z-marching pass loads at once:
// the launch keeps (rows + 2) * nx <= kZmBatch * threads per block, so one
// batch covers the window.
constexpr int kZmBatch = 8;

template <typename T>
struct PassArgs {
    OpDev<T> A;
    const T *dinv;        // CSR Jacobi diagonal inverse (plain vector, nullptr otherwise)
    double dinv_s;        // stencil Jacobi: 1/(diag + shift); 1.0 without preconditioner
    const double *b;      // caller's right-hand side (plain)
    double *x_user;       // caller's x (plain): copy in / out, or the explicit residual's x
    char *blk;            // blocked vectors
    uint32_t tile_bytes;  // bytes of one 512-unknown tile of all slots
    // byte offsets of the slots within a tile (kNoSlot: absent).  Without a
    // preconditioner u, q, p are r, s, t (the kernels never touch off_u..).
    uint32_t off_x, off_r, off_u, off_win, off_wout, off_z, off_q, off_s, off_t, off_p;
    uint32_t clear;       // init 0: ClearBits of the slots to set to zero
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
    int32_t copy_out;     // k_copy_x: 0 = caller -> internal, 1 = internal -> caller
    int32_t x_plain;      // k_resid: read the caller's x instead of the internal one
    const double *sched;  // variable shift: sigma_{-1}, sigma_0, ... (last entry repeats)
    int32_t sched_len;
    int32_t rr_period;    // residual replacement: gap check every rr_period iterations
    double rr_tau;        // ... replace when ||f|| > rr_tau ||r||
    double rr_floor;      // ... and ||f|| > rr_floor * 2^-53 || |A||x| + |b| ||
    CgZm zm;              // CG pass A on a 3-D grid: z-marching split (rows = 0: plain)
    // CSR operand of the fused pipelined pass in sliced-ELL form (nullptr:
    // the pass reads the CSR arrays): see sell_row
    const int32_t *sell_ptr;
    const int32_t *sell_col;
    const T *sell_val;
    // sorted form (nullptr: rows in place): per slice slot, (row length << 8)
    // | the row's position among its wave's rows; see sell_sorted_rows
    const int32_t *sell_perm;
    // sorted form: per tile, the first column its rows gather and the width
    // of that column window (-1: wider than kSellWindow, gathered directly)
    const int2 *sell_win;
    // 16-bit columns (nullptr: 32-bit columns in sell_col): in the sorted
    // form with every tile windowed, each entry's offset in its tile's
    // window; in the in-place form, its column minus its row plus 2^15
    const uint16_t *sell_c16;
    // binary64 form whose matrix values are all binary32 numbers: the copy's
    // values stored as binary32 (exactly the same values; nullptr: sell_val)
    const float *sell_v32;
    int32_t run_through;  // 1: no breakdown stop (PCG_FLAG_RUN_THROUGH_BREAKDOWN)
};

template <typename V, typename T>
__device__ __forceinline__ V *vp(const PassArgs<T> &a, uint32_t off, uint32_t e)
{
    return slot_ptr<V>(a.blk, a.tile_bytes, off, e);
}

// Streaming loads / stores.  With NT the accesses carry the non-temporal
// hint so the once-touched vectors do not evict the stencil operand (w, or p
// in CG) from the caches.
template <bool NT, typename V>
__device__ __forceinline__ double lds(const V *p)
{
    if constexpr (NT) return (double)__builtin_nontemporal_load(p);
    else return (double)*p;
}

template <bool NT, typename V>
__device__ __forceinline__ void sts(V *p, double v)
{
    if constexpr (NT) __builtin_nontemporal_store((V)v, p);
    else *p = (V)v;
}

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

// The unknowns of one tile handled by this thread: e_j = tile * (B * EPT) +
// j * B + threadIdx (each access of a wave is one contiguous run).  Lanes
// past n work on the clamped index n - 1 (loads stay in bounds) and skip
// their stores and partial sums.
template <int EPT>
struct TileIdx {
    uint32_t e[EPT];
    bool live[EPT];
};

template <int EPT>
__device__ __forceinline__ TileIdx<EPT> tile_idx(int tile, uint32_t n)
{
    TileIdx<EPT> t;
    const uint32_t base = (uint32_t)tile * blockDim.x * EPT + threadIdx.x;
#pragma unroll
    for (int j = 0; j < EPT; ++j) {
        const uint32_t e = base + j * blockDim.x;
        t.live[j] = e < n;
        t.e[j] = t.live[j] ? e : n - 1;
    }
    return t;
}

// How a pass treats x.  x is only read at the end of a solve, so the fused
// pass may update it every other iteration: the pass of iteration i skips x
// and the pass of i + 1 applies x_{i+2} = (x_i + alpha_i p_i) + alpha_{i+1}
// p_{i+1} -- the same operations in the same order, p_i being the p it loads
// for its own beta-recurrence -- which halves x's traffic.  A solve that
// stops after a skipping pass completes x with k_x_fixup.
enum XMode : int { X_EACH = 0, X_SKIP = 1, X_CATCHUP = 2 };

__device__ __forceinline__ int lag_mode(int i, int i_start) { return ((i - i_start) & 1) ? X_CATCHUP : X_SKIP; }

struct PipeScalars {
    double alpha, beta;
    double sigma;       // sigma_i
    double dsig;        // sigma_i - sigma_{i-1} (0 for a constant shift)
    double alpha_prev = 0.0;  // alpha_{i-1} (X_CATCHUP)
};

// The pass state is read field by field where it is used (uniform loads),
// and only the thread that writes the next state copies the whole record:
// a per-thread copy of the struct held across the pass would be placed in
// LDS or scratch by the compiler and cost every pass a round trip at its head.
__device__ __forceinline__ bool state_writer() { return blockIdx.x == 0 && threadIdx.x == 0; }

// dst := src field by field (one thread; no local copy of the record)
__device__ __forceinline__ void copy_state(DevState *dst, const DevState *src)
{
    const double *s = reinterpret_cast<const double *>(src);
    double *d = reinterpret_cast<double *>(dst);
#pragma unroll
    for (int k = 0; k < int(sizeof(DevState) / 8); ++k) d[k] = s[k];
}

// sigma_k of a shift schedule, k >= -1
__device__ __forceinline__ double sched_at(const double *sched, int len, int k)
{
    const int idx = k + 1 < len ? k + 1 : len - 1;
    return sched[idx];
}

// Head of an iteration pass of the pipelined methods: stage 2 of the
// previous pass's partials, the stop test and the scalar recurrences
// (identical bits in every block), and block 0's state / history record.
// Returns false when the iteration has ended (or had ended before).
template <typename T, bool VAR = false>
__device__ __forceinline__ bool pipe_head(const PassArgs<T> &a, double *lds_red, PipeScalars &sc)
{
    const DevState *S = a.st_in;
    if (S->status != RUNNING) {
        if (state_writer()) copy_state(a.st_out, S);
        return false;
    }
    double tot[3];
    stage2<3>(a.part_in, a.nparts, tot, lds_red);
    const double gamma = tot[0], delta = tot[1], rho = tot[2];
    const int i = S->iter;
    int status = RUNNING;
    double alpha = __builtin_nan(""), beta = __builtin_nan("");
    if (!isfinite(gamma) || !isfinite(delta) || !isfinite(rho)) {
        status = ST_NONFINITE;
    } else if (sqrt(rho) <= a.rtol * sqrt(S->bnorm2)) {
        status = ST_CONVERGED;
    } else if (i >= a.max_iter) {
        status = ST_MAX_ITER;
    } else if (!a.run_through && (!(gamma > 0.0) || !(delta > 0.0))) {
        status = ST_BREAKDOWN;
    } else {
        if (i > S->i_start) {
            beta = gamma / S->gamma_prev;                            // beta_i
            alpha = 1.0 / (delta / gamma - beta / S->alpha_prev);    // alpha_i
        } else {
            beta = 0.0;
            alpha = gamma / delta;
        }
        if (!a.run_through && !(isfinite(alpha) && alpha > 0.0)) status = ST_BREAKDOWN;
    }
    if (state_writer()) {
        DevState *o = a.st_out;
        copy_state(o, S);
        o->rho = rho;
        if (status != RUNNING) {
            o->status = status;
        } else {
            o->iter = i + 1;
            o->alpha_prev = alpha;
            o->gamma_prev = gamma;
        }
        write_hist(a.hist, a.hist_cap, i, sqrt(rho / S->bnorm2), alpha, beta, gamma, delta);
    }
    sc.alpha = alpha;
    sc.beta = beta;
    sc.alpha_prev = S->alpha_prev;
    if constexpr (VAR) {
        const double sp = sched_at(a.sched, a.sched_len, i - 1);
        sc.sigma = sched_at(a.sched, a.sched_len, i);
        sc.dsig = sc.sigma - sp;
    } else {
        sc.sigma = a.sigma;
        sc.dsig = 0.0;
    }
    return status == RUNNING;
}

// ----------------------------------------------------------------- copy x

template <typename T, int EPT>
__device__ __forceinline__ void tile_copy_x(const PassArgs<T> &a, int tile)
{
    const TileIdx<EPT> ti = tile_idx<EPT>(tile, (uint32_t)a.A.n);
#pragma unroll
    for (int j = 0; j < EPT; ++j) {
        if (!ti.live[j]) continue;
        double *xi = vp<double>(a, a.off_x, ti.e[j]);
        if (a.copy_out) a.x_user[ti.e[j]] = *xi;
        else *xi = a.x_user[ti.e[j]];
    }
}

template <typename T, int EPT>
__global__ void __launch_bounds__(kMaxBlock) k_copy_x(PassArgs<T> a)
{
    const TileRange tr = tile_range(a.ntiles, a.xcd_map);
    for (int tile = tr.first; tile < tr.end; tile += tr.step) tile_copy_x<T, EPT>(a, tile);
}

// (A v) at a tile's rows in the form SELL names, (|A| v) with ABS (defined
// with the sliced-ELL copies below).
template <typename T, int OP, int EPT, int SELL, bool ABS = false, typename F>
__device__ __forceinline__ void tile_apply(const PassArgs<T> &a, int tile, const TileIdx<EPT> &ti, double (&out)[EPT],
                                           F v);

// ----------------------------------------------------------------- init 0

// r_0 := b - A x_0 (stored), and for the pipelined methods with a
// preconditioner u_0 := M^-1 r_0 (stored).  Clears the slots in a.clear (so
// the first iteration's beta = 0 terms are exact zeros).  Partials of (b, b).
template <typename T, int OP, bool JAC, bool STORE_U, int EPT, bool NT, int SELL = 0>
__device__ __forceinline__ void tile_init0(const PassArgs<T> &a, int tile, double (&acc)[1])
{
    const TileIdx<EPT> ti = tile_idx<EPT>(tile, (uint32_t)a.A.n);
    double be[EPT], ax[EPT];
    tile_apply<T, OP, EPT, SELL>(a, tile, ti, ax, [&](uint32_t k) { return *vp<double>(a, a.off_x, k); });
#pragma unroll
    for (int j = 0; j < EPT; ++j) be[j] = lds<NT>(a.b + ti.e[j]);
#pragma unroll
    for (int j = 0; j < EPT; ++j) {
        if (!ti.live[j]) continue;
        const uint32_t e = ti.e[j];
        const double r = rnd<T>(be[j] - ax[j]);
        sts<NT>(vp<T>(a, a.off_r, e), r);
        if constexpr (STORE_U) sts<NT>(vp<T>(a, a.off_u, e), minv<T, JAC, OP>(a, e, r));
        if (a.clear & CLR_Z) sts<NT>(vp<T>(a, a.off_z, e), 0.0);
        if (a.clear & CLR_Q) sts<NT>(vp<T>(a, a.off_q, e), 0.0);
        if (a.clear & CLR_S) sts<NT>(vp<T>(a, a.off_s, e), 0.0);
        if (a.clear & CLR_T) sts<NT>(vp<T>(a, a.off_t, e), 0.0);
        if (a.clear & CLR_P) sts<NT>(vp<T>(a, a.off_p, e), 0.0);
        if (a.clear & CLR_WIN) sts<NT>(vp<T>(a, a.off_win, e), 0.0);
        acc[0] += be[j] * be[j];
    }
}

template <typename T, int OP, bool JAC, bool STORE_U, int EPT, bool NT, int SELL = 0>
__global__ void __launch_bounds__(kMaxBlock) k_init0(PassArgs<T> a)
{
    __shared__ double lds_red[kMaxWaves * kFields];
    double acc[1] = {0.0};
    const TileRange tr = tile_range(a.ntiles, a.xcd_map);
    for (int tile = tr.first; tile < tr.end; tile += tr.step)
        tile_init0<T, OP, JAC, STORE_U, EPT, NT, SELL>(a, tile, acc);
    block_sum<1>(acc, lds_red);
    store_partial<1>(a.part_out, acc);
}

// ----------------------------------------------------------------- init 1 (pipelined)

// w_0 := A u_0 - sigma r_0 into w_out; partials of gamma_0 = (r, u),
// delta_0 = (w + sigma r, u), rho_0.
template <typename T, int OP, bool JAC, int EPT, bool NT, int SELL = 0>
__device__ __forceinline__ void tile_init1(const PassArgs<T> &a, int tile, double (&acc)[3])
{
    const uint32_t off_u = JAC ? a.off_u : a.off_r;
    const TileIdx<EPT> ti = tile_idx<EPT>(tile, (uint32_t)a.A.n);
    double au[EPT], re[EPT], ue[EPT];
    tile_apply<T, OP, EPT, SELL>(a, tile, ti, au, [&](uint32_t k) { return ld(vp<T>(a, off_u, k), 0); });
#pragma unroll
    for (int j = 0; j < EPT; ++j) {
        re[j] = lds<NT>(vp<T>(a, a.off_r, ti.e[j]));
        ue[j] = JAC ? ld(vp<T>(a, off_u, ti.e[j]), 0) : re[j];
    }
#pragma unroll
    for (int j = 0; j < EPT; ++j) {
        if (!ti.live[j]) continue;
        const double w = rnd<T>(au[j] - a.sigma * re[j]);
        sts<NT>(vp<T>(a, a.off_wout, ti.e[j]), w);
        acc[0] += re[j] * ue[j];
        acc[1] += (w + a.sigma * re[j]) * ue[j];
        acc[2] += re[j] * re[j];
    }
}

// head: ||b||^2 from the init-0 partials; then tile_init1 over the grid.
// Block 0 writes the state for iteration i0.
template <typename T, int OP, bool JAC, int EPT, bool NT, int SELL = 0>
__global__ void __launch_bounds__(kMaxBlock) k_init1(PassArgs<T> a)
{
    __shared__ double lds_red[kMaxWaves * kFields];
    double bb[1];
    stage2<1>(a.part_in, a.nparts, bb, lds_red);
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        DevState o{};
        o.bnorm2 = bb[0];
        o.iter = a.i0;
        o.i_start = a.i0;
        o.status = isfinite(bb[0]) ? RUNNING : ST_NONFINITE;
        o.true_res2 = __builtin_nan("");
        *a.st_out = o;
    }
    double acc[3] = {0.0, 0.0, 0.0};
    const TileRange tr = tile_range(a.ntiles, a.xcd_map);
    for (int tile = tr.first; tile < tr.end; tile += tr.step) tile_init1<T, OP, JAC, EPT, NT, SELL>(a, tile, acc);
    block_sum<3>(acc, lds_red);
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
//     w_{i+1} := w - alpha z  (into the other w slot: neighbours read w_i)
//   tail: block partials of gamma_{i+1} = (r, u),
//     delta_{i+1} = (w_{i+1} + sigma r, u), rho_{i+1} = (r, r).
// All loads of a tile are issued before any of its stores.
// What a tile of the fused pass reads, and n = A M^-1 w on it: none of it
// depends on the iteration's scalars, so a pass can issue the loads of its
// first tile before it waits for the reduction at its head.
template <int EPT>
struct PipeTile {
    TileIdx<EPT> ti;
    double ne[EPT], we[EPT], re[EPT], ue[EPT], zo[EPT], so[EPT], to[EPT], qo[EPT], po[EPT], xo[EPT];
};

// The CSR operand in sliced-ELL form.  Rows are grouped in slices of 64
// consecutive rows (one wave's rows of a tile); slice s holds its rows'
// entries column-major, entry k of row r at sell_ptr[s] + 64 k + (r mod 64),
// with (sell_ptr[s + 1] - sell_ptr[s]) / 64 = the longest row of the slice
// (shorter rows padded with their own column and a zero value).  A wave's
// load of entry k of its 64 rows is one contiguous 256-byte access, and its
// address does not depend on the row pointers, so the gathers of a row wait
// for one load instead of two.  Entries are summed in the row's CSR storage
// order and padding is skipped by the row's length, so (A v)_e has the bits
// of apply_row.
//
// The columns and values of entries k .. k + kCsrChunk - 1 of the slice at
// p0 (width w) in lane `lane`; indices past the width repeat entry k.  C16:
// 16-bit columns (sell_c16); binary32-stored values widen exactly.
template <typename T, bool C16>
__device__ __forceinline__ void sell_load_chunk(const PassArgs<T> &a, int32_t p0, int32_t k, int32_t w, uint32_t lane,
                                                int32_t (&c)[kCsrChunk], T (&wv)[kCsrChunk])
{
    if constexpr (sizeof(T) == 8) {
        if (a.sell_v32) {
#pragma unroll
            for (int u = 0; u < kCsrChunk; ++u) {
                const int32_t kk = k + u < w ? k + u : k;
                const int32_t idx = p0 + (kk << 6) + (int32_t)lane;
                if constexpr (C16) c[u] = a.sell_c16[idx];
                else c[u] = a.sell_col[idx];
                wv[u] = (T)a.sell_v32[idx];
            }
            return;
        }
    }
#pragma unroll
    for (int u = 0; u < kCsrChunk; ++u) {
        const int32_t kk = k + u < w ? k + u : k;
        const int32_t idx = p0 + (kk << 6) + (int32_t)lane;
        if constexpr (C16) c[u] = a.sell_c16[idx];
        else c[u] = a.sell_col[idx];
        wv[u] = a.sell_val[idx];
    }
}

// One row's product from slice s of a sliced-ELL copy: the row sits in
// lane `lane` of the slice and has len entries (the rest of the slice's
// width is padding, skipped).  C16: the columns are 16-bit offsets
// (sell_c16), v takes those.  ABS: |a_ij| in place of a_ij (as apply_row).
template <typename T, typename F, bool C16 = false, bool ABS = false>
__device__ __forceinline__ double sell_slice(const PassArgs<T> &a, uint32_t s, uint32_t lane, int32_t len, F v)
{
    const int32_t p0 = a.sell_ptr[s], w = (a.sell_ptr[s + 1] - p0) >> 6;
    double acc = 0.0;
    for (int32_t k = 0; k < w; k += kCsrChunk) {
        int32_t c[kCsrChunk];
        T wv[kCsrChunk];
        double g[kCsrChunk];
        sell_load_chunk<T, C16>(a, p0, k, w, lane, c, wv);
#pragma unroll
        for (int u = 0; u < kCsrChunk; ++u) g[u] = v((uint32_t)c[u]);
#pragma unroll
        for (int u = 0; u < kCsrChunk; ++u)
            if (k + u < len) acc += (ABS ? fabs((double)wv[u]) : (double)wv[u]) * g[u];
    }
    return acc;
}

template <typename T, typename F, bool ABS = false>
__device__ __forceinline__ double sell_row(const PassArgs<T> &a, uint32_t e, F v)
{
    return sell_slice<T, F, false, ABS>(a, e >> 6, e & 63, a.A.row_ptr[e + 1] - a.A.row_ptr[e], v);
}

// The sorted sliced-ELL form (SELL-C-sigma of Kreutzer et al., SIAM J. Sci.
// Comput. 36 (2014), with C = 64 and the sorting window = one wave's rows of
// a tile).  A wave owns the EPT x 64 rows tile * B * EPT + j B + 64 w + l
// (j < EPT, l < 64; B = blockDim.x, w = the wave); they are ordered by
// length, longest first, and cut into EPT slices of 64 (slice g EPT + j' for
// the wave's group g = tile * B / 64 + w), so that each slice is as wide as
// its own longest row instead of the longest of 64 rows taken in place.  The
// thread at (j', l) forms the product of the row in slot l of slice j'; the
// products then return to their rows through the wave's own stretch of LDS
// (EPT x 64 doubles; no block barrier).  Each row is still summed alone in
// CSR storage order, so ne has the bits of apply_row.
template <int EPT>
__device__ __forceinline__ double *sell_exchange_lds()
{
    __shared__ double xch[kMaxBlock * EPT];
    return xch;
}

// Two slices of one wave at once (s0 the wider, as sorted): their chunks'
// loads go out together while both have entries left, the second slice's
// part skipped (a wave-uniform branch) once it has none.
template <typename T, typename F, bool C16 = false, bool ABS = false>
__device__ __forceinline__ void sell_slice_pair(const PassArgs<T> &a, uint32_t s0, uint32_t lane, int32_t len0,
                                                int32_t len1, F v, double &out0, double &out1)
{
    const int32_t p0 = a.sell_ptr[s0], q0 = a.sell_ptr[s0 + 1], q1 = a.sell_ptr[s0 + 2];
    const int32_t w0 = (q0 - p0) >> 6, w1 = (q1 - q0) >> 6;
    double acc0 = 0.0, acc1 = 0.0;
    for (int32_t k = 0; k < w0; k += kCsrChunk) {
        const bool two = k < w1;
        int32_t c0[kCsrChunk], c1[kCsrChunk];
        T v0[kCsrChunk], v1[kCsrChunk];
        double g0[kCsrChunk], g1[kCsrChunk];
        sell_load_chunk<T, C16>(a, p0, k, w0, lane, c0, v0);
        if (two) sell_load_chunk<T, C16>(a, q0, k, w1, lane, c1, v1);
#pragma unroll
        for (int u = 0; u < kCsrChunk; ++u) g0[u] = v((uint32_t)c0[u]);
        if (two) {
#pragma unroll
            for (int u = 0; u < kCsrChunk; ++u) g1[u] = v((uint32_t)c1[u]);
        }
#pragma unroll
        for (int u = 0; u < kCsrChunk; ++u)
            if (k + u < len0) acc0 += (ABS ? fabs((double)v0[u]) : (double)v0[u]) * g0[u];
        if (two) {
#pragma unroll
            for (int u = 0; u < kCsrChunk; ++u)
                if (k + u < len1) acc1 += (ABS ? fabs((double)v1[u]) : (double)v1[u]) * g1[u];
        }
    }
    out0 = acc0, out1 = acc1;
}

// Column window of a tile: the operand values of the columns a tile's rows
// gather, staged in LDS once per tile when they span at most kSellWindow
// columns (a banded operator), so that the gathers read LDS.
constexpr int kSellWindow = 2048;

__device__ __forceinline__ double *sell_window_lds()
{
    __shared__ double win[kSellWindow];
    return win;
}

// The products of a wave's sorted slices with the operand v (binary64 slices
// two at a time: measured on banded random operators of 1e6 / 4e6 rows,
// 94.5 / 382.9 against 99.3 / 402.6 us per pass; the FP32-stream form gained
// nothing, 75.5 / 251.6 against 73.5 / 253.8).
template <typename T, int EPT, bool C16 = false, bool ABS = false, typename F>
__device__ __forceinline__ void sell_sorted_products(const PassArgs<T> &a, uint32_t g, uint32_t lane,
                                                     const int32_t (&len)[EPT], F v, double (&pr)[EPT])
{
    if constexpr (sizeof(T) == 8 && EPT % 2 == 0) {
#pragma unroll
        for (int j = 0; j < EPT; j += 2)
            sell_slice_pair<T, F, C16, ABS>(a, g * EPT + j, lane, len[j], len[j + 1], v, pr[j], pr[j + 1]);
    } else {
#pragma unroll
        for (int j = 0; j < EPT; ++j) pr[j] = sell_slice<T, F, C16, ABS>(a, g * EPT + j, lane, len[j], v);
    }
}

template <typename T, int EPT, bool ABS = false, typename F>
__device__ __forceinline__ void sell_sorted_rows(const PassArgs<T> &a, int tile, double (&ne)[EPT], F v)
{
    static_assert(EPT * 64 <= 256, "a row's position in its wave's rows is kept in 8 bits");
    double *xch = sell_exchange_lds<EPT>();
    const uint32_t lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const uint32_t g = (uint32_t)tile * (blockDim.x >> 6) + wave;
    double pr[EPT];
    uint32_t at[EPT];
    int32_t len[EPT];
#pragma unroll
    for (int j = 0; j < EPT; ++j) {
        const int32_t info = a.sell_perm[(size_t)(g * EPT + j) * 64 + lane];
        at[j] = (uint32_t)info & 255;
        len[j] = info >> 8;
    }
    const int2 wd = a.sell_win ? a.sell_win[tile] : make_int2(0, -1);  // the same in the whole block
    if (wd.y >= 0) {
        // the tile's column window: v at columns wd.x .. wd.x + wd.y - 1,
        // formed once (the same values v gives) and gathered from LDS
        double *win = sell_window_lds();
        __syncthreads();  // the previous tile's gathers from the window are done
        for (int c = threadIdx.x; c < wd.y; c += blockDim.x) win[c] = v((uint32_t)(wd.x + c));
        __syncthreads();
        if (a.sell_c16) {
            // every tile windowed: the entries carry their window offsets
            sell_sorted_products<T, EPT, true, ABS>(a, g, lane, len, [&](uint32_t k) { return win[k]; }, pr);
        } else {
            const uint32_t c0 = (uint32_t)wd.x;
            sell_sorted_products<T, EPT, false, ABS>(a, g, lane, len, [&](uint32_t k) { return win[k - c0]; }, pr);
        }
    } else {
        sell_sorted_products<T, EPT, false, ABS>(a, g, lane, len, v, pr);
    }
    double *xw = xch + wave * (EPT * 64);
    // the previous tile's reads of xw are done before it is written again
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
#pragma unroll
    for (int j = 0; j < EPT; ++j) xw[at[j]] = pr[j];
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
#pragma unroll
    for (int j = 0; j < EPT; ++j) ne[j] = xw[j * 64 + lane];
}

// One row of the in-place copy, through its 16-bit row-relative columns when
// the copy has them (every entry within 2^15 of its row).
template <bool ABS = false, typename T, typename F>
__device__ __forceinline__ double sell_plain_row(const PassArgs<T> &a, uint32_t e, F v)
{
    if (a.sell_c16) {
        auto rel = [&](uint32_t c) { return v(e + c - 32768u); };
        return sell_slice<T, decltype(rel), true, ABS>(a, e >> 6, e & 63, a.A.row_ptr[e + 1] - a.A.row_ptr[e], rel);
    }
    return sell_row<T, F, ABS>(a, e, v);
}

// (A v) at a tile's rows (ABS: (|A| v)): from the sorted copy (SELL 2), the
// in-place copy (SELL 1) or the operator itself (SELL 0, and every operator
// that is not CSR).  All three give the bits of apply_row.  SELL 2
// synchronises the block when the tile has a column window, so every
// thread of the block calls it for the tile.
template <typename T, int OP, int EPT, int SELL, bool ABS, typename F>
__device__ __forceinline__ void tile_apply(const PassArgs<T> &a, int tile, const TileIdx<EPT> &ti, double (&out)[EPT],
                                           F v)
{
    if constexpr (OP == OP_CSR && SELL == 2) {
        sell_sorted_rows<T, EPT, ABS>(a, tile, out, v);
    } else {
#pragma unroll
        for (int j = 0; j < EPT; ++j) {
            if constexpr (OP == OP_CSR && SELL == 1) out[j] = sell_plain_row<ABS>(a, ti.e[j], v);
            else out[j] = apply_row<OP, ABS>(a.A, ti.e[j], v);
        }
    }
}

template <typename T, int OP, bool JAC, int EPT, bool NT, int XM = X_EACH, int SELL = 0>
__device__ __forceinline__ void tile_pipe_load(const PassArgs<T> &a, int tile, PipeTile<EPT> &d)
{
    const uint32_t off_u = JAC ? a.off_u : a.off_r;
    const uint32_t off_q = JAC ? a.off_q : a.off_s;
    const uint32_t off_p = JAC ? a.off_p : a.off_t;
    d.ti = tile_idx<EPT>(tile, (uint32_t)a.A.n);
    const TileIdx<EPT> &ti = d.ti;
    double *ne = d.ne, *we = d.we, *re = d.re, *ue = d.ue, *zo = d.zo, *so = d.so, *to = d.to, *qo = d.qo,
           *po = d.po, *xo = d.xo;
    // loads: the stencil / CSR operand w_i (cached), then the streams
    auto operand = [&](uint32_t k) { return minv<T, JAC, OP>(a, k, ld(vp<T>(a, a.off_win, k), 0)); };
    if constexpr (OP == OP_CSR && SELL == 2) sell_sorted_rows<T, EPT>(a, tile, d.ne, operand);
#pragma unroll
    for (int j = 0; j < EPT; ++j) {
        const uint32_t e = ti.e[j];
        we[j] = ld(vp<T>(a, a.off_win, e), 0);
        if constexpr (OP == OP_CSR && SELL == 1) ne[j] = sell_plain_row(a, e, operand);
        else if constexpr (OP != OP_CSR || SELL == 0) ne[j] = apply_row<OP>(a.A, e, operand);
        re[j] = lds<NT>(vp<T>(a, a.off_r, e));
        zo[j] = lds<NT>(vp<T>(a, a.off_z, e));
        so[j] = lds<NT>(vp<T>(a, a.off_s, e));
        to[j] = lds<NT>(vp<T>(a, a.off_t, e));
        if constexpr (XM != X_SKIP) xo[j] = lds<NT>(vp<double>(a, a.off_x, e));
        else xo[j] = 0.0;
        if constexpr (JAC) {
            ue[j] = lds<NT>(vp<T>(a, off_u, e));
            qo[j] = lds<NT>(vp<T>(a, off_q, e));
            po[j] = lds<NT>(vp<T>(a, off_p, e));
        } else {
            ue[j] = re[j];
            qo[j] = so[j];
            po[j] = to[j];
        }
    }
}

// The recurrences and stores of a loaded tile, and its partials.
template <typename T, int OP, bool JAC, int EPT, bool NT, bool VAR = false, int XM = X_EACH>
__device__ __forceinline__ void tile_pipe_update(const PassArgs<T> &a, const PipeTile<EPT> &d, const PipeScalars &sc,
                                                 double (&acc)[3])
{
    const double alpha = sc.alpha, beta = sc.beta;
    const double sigma = sc.sigma, as = alpha * sigma, ds = sc.dsig;
    const uint32_t off_u = JAC ? a.off_u : a.off_r;
    const uint32_t off_q = JAC ? a.off_q : a.off_s;
    const uint32_t off_p = JAC ? a.off_p : a.off_t;
    const TileIdx<EPT> &ti = d.ti;
    const double *ne = d.ne, *we = d.we, *re = d.re, *ue = d.ue, *zo = d.zo, *so = d.so, *to = d.to, *qo = d.qo,
                 *po = d.po, *xo = d.xo;
#pragma unroll
    for (int j = 0; j < EPT; ++j) {
        if (!ti.live[j]) continue;
        const uint32_t e = ti.e[j];
        const double me = minv<T, JAC, OP>(a, e, we[j]);
        double z, s, t, qv, pv, wn;
        if constexpr (!VAR) {
            // beta-recurrences
            z = rnd<T>(ne[j] + beta * zo[j]);
            s = rnd<T>(we[j] + beta * so[j]);
            t = rnd<T>(re[j] + beta * to[j]);
            qv = s, pv = t;
            if constexpr (JAC) {
                qv = rnd<T>(me + beta * qo[j]);
                pv = rnd<T>(ue[j] + beta * po[j]);
            }
            wn = rnd<T>(we[j] - alpha * z);
        } else {
            // Alg. 4: t, p first; s, q, z carry the shift-difference
            // correction, subtracted after the two-term recurrence
            t = rnd<T>(re[j] + beta * to[j]);
            pv = t;
            if constexpr (JAC) pv = rnd<T>(ue[j] + beta * po[j]);
            s = rnd<T>((we[j] + beta * so[j]) - ds * t);
            qv = s;
            if constexpr (JAC) qv = rnd<T>((me + beta * qo[j]) - ds * pv);
            z = rnd<T>((ne[j] + beta * zo[j]) - ds * (s + sigma * t));
            wn = rnd<T>((we[j] - alpha * z) - ds * re[j]);  // the old r_i
        }
        // alpha-recurrences, the shift terms grouped first
        double xn = 0.0;
        if constexpr (XM == X_EACH) xn = xo[j] + alpha * pv;
        else if constexpr (XM == X_CATCHUP) xn = (xo[j] + sc.alpha_prev * po[j]) + alpha * pv;
        const double rn = rnd<T>(re[j] - (alpha * s + as * t));
        double un = rn;
        if constexpr (JAC) un = rnd<T>(ue[j] - (alpha * qv + as * pv));
        sts<NT>(vp<T>(a, a.off_z, e), z);
        sts<NT>(vp<T>(a, a.off_s, e), s);
        sts<NT>(vp<T>(a, a.off_t, e), t);
        if constexpr (JAC) {
            sts<NT>(vp<T>(a, off_q, e), qv);
            sts<NT>(vp<T>(a, off_p, e), pv);
            sts<NT>(vp<T>(a, off_u, e), un);
        }
        if constexpr (XM != X_SKIP) sts<NT>(vp<double>(a, a.off_x, e), xn);
        sts<NT>(vp<T>(a, a.off_r, e), rn);
        sts<NT>(vp<T>(a, a.off_wout, e), wn);
        // next iteration's dot products
        acc[0] += rn * un;
        acc[1] += (wn + sigma * rn) * un;
        acc[2] += rn * rn;
    }
}

template <typename T, int OP, bool JAC, int EPT, bool NT, bool VAR = false, int XM = X_EACH, int SELL = 0>
__device__ __forceinline__ void tile_pipe(const PassArgs<T> &a, int tile, const PipeScalars &sc, double (&acc)[3])
{
    PipeTile<EPT> d;
    tile_pipe_load<T, OP, JAC, EPT, NT, XM, SELL>(a, tile, d);
    tile_pipe_update<T, OP, JAC, EPT, NT, VAR, XM>(a, d, sc, acc);
}

// One pass with x's update mode fixed at compile time, so that the skipping
// pass has no x loads or stores in its code at all.
template <typename T, int OP, bool JAC, int EPT, bool NT, bool VAR, int XM, int SELL>
__device__ __forceinline__ void pipe_pass(const PassArgs<T> &a, const TileRange &tr, double *lds_red)
{
    PipeTile<EPT> d;
    if (tr.first < tr.end) tile_pipe_load<T, OP, JAC, EPT, NT, XM, SELL>(a, tr.first, d);
    PipeScalars sc;
    if (!pipe_head<T, VAR>(a, lds_red, sc)) return;
    double acc[3] = {0.0, 0.0, 0.0};
    for (int tile = tr.first; tile < tr.end; tile += tr.step) {
        if (tile != tr.first) tile_pipe_load<T, OP, JAC, EPT, NT, XM, SELL>(a, tile, d);
        tile_pipe_update<T, OP, JAC, EPT, NT, VAR, XM>(a, d, sc, acc);
    }
    block_sum<3>(acc, lds_red);
    store_partial<3>(a.part_out, acc);
}

// SELL: a CSR operand read in sliced-ELL form, 1 with the rows in place
// (sell_row), 2 sorted (sell_sorted_rows).
template <typename T, int OP, bool JAC, int EPT, bool NT, bool VAR = false, int SELL = 0>
__global__ void __launch_bounds__(kMaxBlock) k_pipe(PassArgs<T> a)
{
    __shared__ double lds_red[kMaxWaves * kFields];
    // The first tile's loads and SPMV go out before the head waits for the
    // previous pass's partials: the global reduction overlaps the SPMV, the
    // point of the pipelined method (Section 1), inside one pass.
    const TileRange tr = tile_range(a.ntiles, a.xcd_map);
    if (lag_mode(a.st_in->iter, a.st_in->i_start) == X_SKIP)
        pipe_pass<T, OP, JAC, EPT, NT, VAR, X_SKIP, SELL>(a, tr, lds_red);
    else
        pipe_pass<T, OP, JAC, EPT, NT, VAR, X_CATCHUP, SELL>(a, tr, lds_red);
}

// x := x + alpha p on one tile: completes x after a solve that stopped after
// a pass that skipped x (alpha = alpha_i and p = p_i of that pass's iteration).
template <typename T, bool JAC, int EPT>
__device__ __forceinline__ void tile_x_fixup(const PassArgs<T> &a, int tile, double alpha)
{
    const uint32_t off_p = JAC ? a.off_p : a.off_t;
    const TileIdx<EPT> ti = tile_idx<EPT>(tile, (uint32_t)a.A.n);
#pragma unroll
    for (int j = 0; j < EPT; ++j) {
        if (!ti.live[j]) continue;
        double *xp = vp<double>(a, a.off_x, ti.e[j]);
        *xp = *xp + alpha * ld(vp<T>(a, off_p, ti.e[j]), 0);
    }
}

template <typename T, bool JAC, int EPT>
__global__ void __launch_bounds__(kMaxBlock) k_x_fixup(PassArgs<T> a, double alpha)
{
    const TileRange tr = tile_range(a.ntiles, a.xcd_map);
    for (int tile = tr.first; tile < tr.end; tile += tr.step) tile_x_fixup<T, JAC, EPT>(a, tile, alpha);
}

// ------------------------------------------------- p-CG with residual replacement

// Gap check: partials of ||(b - A x) - r||^2 and || |A||x| + |b| ||^2 (the
// rounding scale of the explicit residual), x the internal binary64 copy.
template <typename T, int OP, int EPT, int SELL = 0>
__device__ __forceinline__ void tile_gap(const PassArgs<T> &a, int tile, double (&acc)[3])
{
    const TileIdx<EPT> ti = tile_idx<EPT>(tile, (uint32_t)a.A.n);
    double be[EPT], ax[EPT], aax[EPT], re[EPT];
    tile_apply<T, OP, EPT, SELL>(a, tile, ti, ax, [&](uint32_t k) { return *vp<double>(a, a.off_x, k); });
    tile_apply<T, OP, EPT, SELL, true>(a, tile, ti, aax, [&](uint32_t k) { return fabs(*vp<double>(a, a.off_x, k)); });
#pragma unroll
    for (int j = 0; j < EPT; ++j) {
        const uint32_t e = ti.e[j];
        be[j] = a.b[e];
        re[j] = ld(vp<T>(a, a.off_r, e), 0);
    }
#pragma unroll
    for (int j = 0; j < EPT; ++j) {
        if (!ti.live[j]) continue;
        const double f = (be[j] - ax[j]) - re[j];
        const double fl = aax[j] + fabs(be[j]);
        acc[0] += f * f;
        acc[1] += fl * fl;
    }
}

// Replacement, first pass: r := b - A x, u := M^-1 r, s := A p, q := M^-1 s
// (p = p_{i-1}; the method runs without shift).
template <typename T, int OP, bool JAC, int EPT, int SELL = 0>
__device__ __forceinline__ void tile_rr1(const PassArgs<T> &a, int tile)
{
    const uint32_t off_p = JAC ? a.off_p : a.off_t;
    const TileIdx<EPT> ti = tile_idx<EPT>(tile, (uint32_t)a.A.n);
    double be[EPT], ax[EPT], ap[EPT];
    tile_apply<T, OP, EPT, SELL>(a, tile, ti, ax, [&](uint32_t k) { return *vp<double>(a, a.off_x, k); });
    tile_apply<T, OP, EPT, SELL>(a, tile, ti, ap, [&](uint32_t k) { return ld(vp<T>(a, off_p, k), 0); });
#pragma unroll
    for (int j = 0; j < EPT; ++j) be[j] = a.b[ti.e[j]];
#pragma unroll
    for (int j = 0; j < EPT; ++j) {
        if (!ti.live[j]) continue;
        const uint32_t e = ti.e[j];
        const double r = rnd<T>(be[j] - ax[j]);
        const double sv = rnd<T>(ap[j]);
        *vp<T>(a, a.off_r, e) = (T)r;
        *vp<T>(a, a.off_s, e) = (T)sv;
        if constexpr (JAC) {
            *vp<T>(a, a.off_u, e) = (T)minv<T, JAC, OP>(a, e, r);
            *vp<T>(a, a.off_q, e) = (T)minv<T, JAC, OP>(a, e, sv);
        }
    }
}

// Replacement, second pass: w := A u, z := A q (neighbours written by the
// first pass); partials of gamma_i, delta_i, rho_i from the reset vectors.
template <typename T, int OP, bool JAC, int EPT, int SELL = 0>
__device__ __forceinline__ void tile_rr2(const PassArgs<T> &a, uint32_t off_wout, int tile, double (&acc)[3])
{
    const uint32_t off_u = JAC ? a.off_u : a.off_r;
    const uint32_t off_q = JAC ? a.off_q : a.off_s;
    const TileIdx<EPT> ti = tile_idx<EPT>(tile, (uint32_t)a.A.n);
    double au[EPT], aq[EPT], re[EPT], ue[EPT];
    tile_apply<T, OP, EPT, SELL>(a, tile, ti, au, [&](uint32_t k) { return ld(vp<T>(a, off_u, k), 0); });
    tile_apply<T, OP, EPT, SELL>(a, tile, ti, aq, [&](uint32_t k) { return ld(vp<T>(a, off_q, k), 0); });
#pragma unroll
    for (int j = 0; j < EPT; ++j) {
        const uint32_t e = ti.e[j];
        re[j] = ld(vp<T>(a, a.off_r, e), 0);
        ue[j] = JAC ? ld(vp<T>(a, off_u, e), 0) : re[j];
    }
#pragma unroll
    for (int j = 0; j < EPT; ++j) {
        if (!ti.live[j]) continue;
        const uint32_t e = ti.e[j];
        const double w = rnd<T>(au[j]);
        *vp<T>(a, off_wout, e) = (T)w;
        *vp<T>(a, a.off_z, e) = (T)rnd<T>(aq[j]);
        acc[0] += re[j] * ue[j];
        acc[1] += w * ue[j];
        acc[2] += re[j] * re[j];
    }
}

// One pass of pipelined CG with automated residual replacement.  Its role is
// decided at the head from the state and the previous pass's partials (the
// same bits in every block):
//   ITER phase: stop test / cap; then every rr_period iterations a GAP pass
//     (partials of ||f||^2 and the rounding scale; gamma, delta, rho are kept
//     in the state), else an iteration exactly as k_pipe (sigma = 0);
//   CHECK phase (after a gap pass): if ||f|| > tau ||r|| and ||f|| > floor,
//     the pass does replacement step 1, else it iterates;
//   RR2 phase: replacement step 2, whose partials restart iteration i.
// Passes that leave w alone flip `wflip`, so w_i is always found.  A CSR
// operator is read in the form SELL names.
template <typename T, int OP, bool JAC, int EPT, bool NT, int SELL = 0>
__global__ void __launch_bounds__(kMaxBlock) k_pipe_rr(PassArgs<T> a)
{
    enum { ROLE_ITER, ROLE_GAP, ROLE_RR1, ROLE_RR2, ROLE_STOP };
    __shared__ double lds_red[kMaxWaves * kFields];
    const DevState *S = a.st_in;
    if (S->status != RUNNING) {
        if (state_writer()) copy_state(a.st_out, S);
        return;
    }
    double tot[4];
    stage2<4>(a.part_in, a.nparts, tot, lds_red);
    const int i = S->iter, phase = S->rr_phase;
    int role = ROLE_ITER, status = RUNNING;
    double gamma = 0.0, delta = 0.0, rho = S->rho;
    double alpha = __builtin_nan(""), beta = __builtin_nan("");
    if (phase == RR_RR2) {
        role = ROLE_RR2;
    } else {
        if (phase == RR_CHECK) {
            gamma = S->gamma, delta = S->spare[1], rho = S->rho;
            const double gap = sqrt(tot[0]), floor = 0x1p-53 * sqrt(tot[1]);
            if (gap > a.rr_tau * sqrt(rho) && gap > a.rr_floor * floor) role = ROLE_RR1;
        } else {
            gamma = tot[0], delta = tot[1], rho = tot[2];
            if (!isfinite(gamma) || !isfinite(delta) || !isfinite(rho)) status = ST_NONFINITE;
            else if (sqrt(rho) <= a.rtol * sqrt(S->bnorm2)) status = ST_CONVERGED;
            else if (i >= a.max_iter) status = ST_MAX_ITER;
            else if (i > S->i_start && i % a.rr_period == 0 && S->last_check != i) role = ROLE_GAP;
        }
        if (status != RUNNING) {
            role = ROLE_STOP;
        } else if (role == ROLE_ITER) {
            if (!a.run_through && (!(gamma > 0.0) || !(delta > 0.0))) {
                status = ST_BREAKDOWN;
            } else {
                if (i > S->i_start) {
                    beta = gamma / S->gamma_prev;
                    alpha = 1.0 / (delta / gamma - beta / S->alpha_prev);
                } else {
                    beta = 0.0;
                    alpha = gamma / delta;
                }
                if (!a.run_through && !(isfinite(alpha) && alpha > 0.0)) status = ST_BREAKDOWN;
            }
            if (status != RUNNING) role = ROLE_STOP;
        }
    }
    if (state_writer()) {
        DevState *o = a.st_out;
        copy_state(o, S);
        switch (role) {
        case ROLE_STOP:
            o->status = status;
            o->rho = rho;
            break;
        case ROLE_GAP:
            o->rr_phase = RR_CHECK;
            o->gamma = gamma;
            o->spare[1] = delta;
            o->rho = rho;
            o->last_check = i;
            o->wflip = S->wflip ^ 1;
            break;
        case ROLE_RR1:
            o->rr_phase = RR_RR2;
            o->rr_count = S->rr_count + 1;
            o->wflip = S->wflip ^ 1;
            break;
        case ROLE_RR2:
            o->rr_phase = RR_ITER;
            break;
        default:
            o->rr_phase = RR_ITER;
            o->iter = i + 1;
            o->alpha_prev = alpha;
            o->gamma_prev = gamma;
            o->rho = rho;
            break;
        }
        if (role == ROLE_ITER || role == ROLE_STOP)
            write_hist(a.hist, a.hist_cap, i, sqrt(rho / S->bnorm2), alpha, beta, gamma, delta);
    }
    if (role == ROLE_STOP) return;
    // the w slots of this pass, swapped while w_i sits in the other one
    PassArgs<T> w = a;
    if (S->wflip) {
        w.off_win = a.off_wout;
        w.off_wout = a.off_win;
    }
    double acc[3] = {0.0, 0.0, 0.0};
    const TileRange tr = tile_range(a.ntiles, a.xcd_map);
    if (role == ROLE_ITER) {
        PipeScalars sc;
        sc.alpha = alpha;
        sc.beta = beta;
        sc.sigma = 0.0;
        sc.dsig = 0.0;
        for (int tile = tr.first; tile < tr.end; tile += tr.step)
            tile_pipe<T, OP, JAC, EPT, NT, false, X_EACH, SELL>(w, tile, sc, acc);
    } else if (role == ROLE_GAP) {
        for (int tile = tr.first; tile < tr.end; tile += tr.step) tile_gap<T, OP, EPT, SELL>(a, tile, acc);
    } else if (role == ROLE_RR1) {
        for (int tile = tr.first; tile < tr.end; tile += tr.step) tile_rr1<T, OP, JAC, EPT, SELL>(a, tile);
    } else {
        for (int tile = tr.first; tile < tr.end; tile += tr.step)
            tile_rr2<T, OP, JAC, EPT, SELL>(a, w.off_wout, tile, acc);
    }
    block_sum<3>(acc, lds_red);
    store_partial<3>(a.part_out, acc);
}

// ----------------------------------------------------------------- classic CG

// head: ||b||^2; partials of gamma_0 = (r_0, M^-1 r_0) and rho_0.
template <typename T, int OP, bool JAC, int EPT, bool NT>
__global__ void __launch_bounds__(kMaxBlock) k_cg_init1(PassArgs<T> a)
{
    __shared__ double lds_red[kMaxWaves * kFields];
    double bb[1];
    stage2<1>(a.part_in, a.nparts, bb, lds_red);
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
    const uint32_t n = (uint32_t)a.A.n;
    const TileRange tr = tile_range(a.ntiles, a.xcd_map);
    for (int tile = tr.first; tile < tr.end; tile += tr.step) {
        const TileIdx<EPT> ti = tile_idx<EPT>(tile, n);
        double re[EPT];
#pragma unroll
        for (int j = 0; j < EPT; ++j) re[j] = lds<NT>(vp<T>(a, a.off_r, ti.e[j]));
#pragma unroll
        for (int j = 0; j < EPT; ++j) {
            if (!ti.live[j]) continue;
            const double u = rnd<T>(minv<T, JAC, OP>(a, ti.e[j], re[j]));
            acc[0] += re[j] * u;
            acc[1] += re[j] * re[j];
        }
    }
    block_sum<2>(acc, lds_red);
    store_partial<2>(a.part_out, acc);
}

// Head of CG pass A: stage 2 of (r_i, u_i) and (r_i, r_i), the stop test
// and beta_i; block 0's state and history record.  false when the
// iteration has ended.
template <typename T>
__device__ __forceinline__ bool cg_a_head(const PassArgs<T> &a, double *lds_red, double &beta)
{
    const DevState *S = a.st_in;
    if (S->status != RUNNING) {
        if (state_writer()) copy_state(a.st_out, S);
        return false;
    }
    double tot[2];
    stage2<2>(a.part_in, a.nparts, tot, lds_red);
    const double gamma = tot[0], rho = tot[1];
    const int i = S->iter;
    int status = RUNNING;
    beta = 0.0;
    if (!isfinite(gamma) || !isfinite(rho)) {
        status = ST_NONFINITE;
    } else if (sqrt(rho) <= a.rtol * sqrt(S->bnorm2)) {
        status = ST_CONVERGED;
    } else if (i >= a.max_iter) {
        status = ST_MAX_ITER;
    } else if (!a.run_through && !(gamma > 0.0)) {
        status = ST_BREAKDOWN;
    } else if (i > S->i_start) {
        beta = gamma / S->gamma_prev;  // beta_i = (r_i, u_i) / (r_{i-1}, u_{i-1})
    }
    if (state_writer()) {
        DevState *o = a.st_out;
        copy_state(o, S);
        o->rho = rho;
        o->gamma = gamma;
        if (status != RUNNING) o->status = status;
        write_hist(a.hist, a.hist_cap, i, sqrt(rho / S->bnorm2), __builtin_nan(""),
                   status == RUNNING ? beta : __builtin_nan(""), gamma, __builtin_nan(""));
    }
    return status == RUNNING;
}

// p_i = M^{-1} r_i + beta_i p_{i-1} at index k, as stored (p_{-1} = 0 after
// the init, so the first iteration needs no branch)
template <typename T, bool JAC, int OP>
__device__ __forceinline__ double cg_pnew_of(const PassArgs<T> &a, uint32_t k, double rk, double pk, double beta)
{
    const double uk = rnd<T>(minv<T, JAC, OP>(a, k, rk));
    return rnd<T>(uk + beta * pk);
}

template <typename T, bool JAC, int OP>
__device__ __forceinline__ double cg_pnew(const PassArgs<T> &a, uint32_t k, double beta)
{
    return cg_pnew_of<T, JAC, OP>(a, k, ld(vp<T>(a, a.off_r, k), 0), ld(vp<T>(a, a.off_win, k), 0), beta);
}

// Pass A of CG iteration i.  w_in = p_{i-1}, w_out = p_i; a CSR operator
// from the form SELL names (tile_apply).
template <typename T, int OP, bool JAC, int EPT, bool NT, int SELL = 0>
__global__ void __launch_bounds__(kMaxBlock) k_cg_a(PassArgs<T> a)
{
    __shared__ double lds_red[kMaxWaves * kFields];
    double beta;
    if (!cg_a_head<T>(a, lds_red, beta)) return;

    // p_i at index k, recomputed identically wherever it is needed
    auto pnew = [&](uint32_t k) { return cg_pnew<T, JAC, OP>(a, k, beta); };
    double acc[1] = {0.0};
    const uint32_t n = (uint32_t)a.A.n;
    const TileRange tr = tile_range(a.ntiles, a.xcd_map);
    for (int tile = tr.first; tile < tr.end; tile += tr.step) {
        const TileIdx<EPT> ti = tile_idx<EPT>(tile, n);
        double pe[EPT], se[EPT];
        tile_apply<T, OP, EPT, SELL>(a, tile, ti, se, pnew);
#pragma unroll
        for (int j = 0; j < EPT; ++j) pe[j] = pnew(ti.e[j]);
#pragma unroll
        for (int j = 0; j < EPT; ++j) {
            if (!ti.live[j]) continue;
            const double sv = rnd<T>(se[j]);
            sts<NT>(vp<T>(a, a.off_wout, ti.e[j]), pe[j]);
            sts<NT>(vp<T>(a, a.off_s, ti.e[j]), sv);
            acc[0] += sv * pe[j];
        }
    }
    block_sum<1>(acc, lds_red);
    store_partial<1>(a.part_out, acc);
}

// Pass A of CG iteration i on the 7-point stencil, marching along z.  For
// each plane of its item a block forms p_i once per point -- over its rows
// and one halo row on either side -- into one of four LDS plane slots
// (extern shared: 4 x (rows + 2) x nx doubles), writes its own rows' p_i,
// and after one barrier evaluates s = A p_i on the plane before it, from
// that plane and its two neighbours in LDS.  The plain pass forms p_i anew
// at each of the seven points of every row (14 loads per unknown); this
// one loads r and p_{i-1} about (rows + 2) / rows times per unknown.  Four
// slots need one barrier per plane: filling plane z + 2 never overwrites a
// plane that s of plane z still reads.  The loads of plane z + 2 are issued
// into registers before s of plane z is evaluated, so they are in flight
// during it.  The values and the order of every sum are those of k_cg_a
// (apply_row reads its operands through the LDS window); only the partial
// sums are grouped differently.
template <typename T, bool JAC, bool NT>
__global__ void __launch_bounds__(kMaxBlock) k_cg_a_zm(PassArgs<T> a, CgZm zm)
{
    __shared__ double lds_red[kMaxWaves * kFields];
    extern __shared__ double zlds[];
    double beta;
    if (!cg_a_head<T>(a, lds_red, beta)) return;
    const uint32_t nx = (uint32_t)a.A.nx, ny = (uint32_t)a.A.ny, nz = (uint32_t)a.A.nz, nxy = nx * ny;
    const uint32_t slot = (uint32_t)(zm.rows + 2) * nx;
    double acc[1] = {0.0};
    const int nitems = zm.nchunks * zm.nsegs;
    for (int item = blockIdx.x; item < nitems; item += gridDim.x) {
        const uint32_t r0 = (uint32_t)(item % zm.nchunks) * (uint32_t)zm.rows;
        const uint32_t r1 = min(r0 + (uint32_t)zm.rows, ny);
        const uint32_t z0 = (uint32_t)(item / zm.nchunks) * (uint32_t)zm.seg;
        const uint32_t z1 = min(z0 + (uint32_t)zm.seg, nz);
        // window row w holds grid row r0 - 1 + w; rows outside the grid stay unfilled
        const uint32_t wr0 = r0 > 0 ? r0 - 1 : 0, wr1 = min(r1 + 1, ny);
        const uint32_t own0 = (r0 - wr0) * nx, own1 = (r1 - wr0) * nx;  // own rows, relative to wr0
        const uint32_t cnt = (wr1 - wr0) * nx;  // points of a plane window, <= kZmBatch * blockDim.x
        // r and p_{i-1} of one plane window, kZmBatch points per thread
        double rv[kZmBatch], pv[kZmBatch];
        auto load = [&](uint32_t zz) {
            const uint32_t g0 = zz * nxy + wr0 * nx;
#pragma unroll
            for (int j = 0; j < kZmBatch; ++j) {
                const uint32_t k = g0 + min(threadIdx.x + j * blockDim.x, cnt - 1);  // in bounds
                rv[j] = ld(vp<T>(a, a.off_r, k), 0);
                pv[j] = ld(vp<T>(a, a.off_win, k), 0);
            }
        };
        // p_i of the loaded plane into its LDS slot (and, on own rows of own
        // planes, to w_out)
        auto commit = [&](uint32_t zz) {
            double *buf = zlds + (size_t)(zz & 3u) * slot + (size_t)(wr0 + 1 - r0) * nx;
            const uint32_t g0 = zz * nxy + wr0 * nx;
            const bool own = zz >= z0 && zz < z1;
#pragma unroll
            for (int j = 0; j < kZmBatch; ++j) {
                const uint32_t t = threadIdx.x + j * blockDim.x;
                if (t >= cnt) continue;
                const double p = cg_pnew_of<T, JAC, OP_3D7>(a, g0 + t, rv[j], pv[j], beta);
                buf[t] = p;
                if (own && t >= own0 && t < own1) sts<NT>(vp<T>(a, a.off_wout, g0 + t), p);
            }
        };
        if (z0 > 0) load(z0 - 1), commit(z0 - 1);
        load(z0);
        commit(z0);
        if (z0 + 1 < nz) load(z0 + 1);
        for (uint32_t z = z0; z < z1; ++z) {
            if (z + 1 < nz) commit(z + 1);
            __syncthreads();
            // plane z + 2 is needed while z + 1 < z1 (as the upper neighbour of z1 - 1 at most)
            if (z + 2 < nz && z + 2 <= z1) load(z + 2);
            const double *cur = zlds + (size_t)(z & 3u) * slot;
            const double *prv = zlds + (size_t)((z + 3u) & 3u) * slot;
            const double *nxt = zlds + (size_t)((z + 1u) & 3u) * slot;
            const uint32_t ocnt = (r1 - r0) * nx, g0 = z * nxy + r0 * nx;
            for (uint32_t t = threadIdx.x; t < ocnt; t += blockDim.x) {
                const uint32_t e = g0 + t, w = nx + t;  // grid row r0 sits in window row 1
                // apply_row asks for e (also in place of a missing
                // neighbour), e -+ 1, e -+ nx and e -+ nx*ny
                const double se = apply_row<OP_3D7>(a.A, e, [&](uint32_t k) {
                    const int32_t d = (int32_t)(k - e);
                    if (d == (int32_t)nxy) return nxt[w];
                    if (d == -(int32_t)nxy) return prv[w];
                    return cur[(int32_t)w + d];
                });
                const double sv = rnd<T>(se);
                sts<NT>(vp<T>(a, a.off_s, e), sv);
                acc[0] += sv * cur[w];
            }
        }
        __syncthreads();  // the next item's fills reuse every slot
    }
    block_sum<1>(acc, lds_red);
    store_partial<1>(a.part_out, acc);
}

// Pass B of CG iteration i.  w_out = p_i (written by pass A).
template <typename T, int OP, bool JAC, int EPT, bool NT>
__global__ void __launch_bounds__(kMaxBlock) k_cg_b(PassArgs<T> a)
{
    __shared__ double lds_red[kMaxWaves * kFields];
    const DevState *S = a.st_in;
    if (S->status != RUNNING) {
        if (state_writer()) copy_state(a.st_out, S);
        return;
    }
    double tot[1];
    stage2<1>(a.part_in, a.nparts, tot, lds_red);
    const double sp = tot[0];
    const int i = S->iter;
    const double gamma_i = S->gamma;
    int status = RUNNING;
    double alpha = __builtin_nan("");
    if (!isfinite(sp)) {
        status = ST_NONFINITE;
    } else if (!a.run_through && !(sp > 0.0)) {
        status = ST_BREAKDOWN;
    } else {
        alpha = gamma_i / sp;  // alpha_i = (r_i, u_i) / (s_i, p_i)
        if (!a.run_through && !(isfinite(alpha) && alpha > 0.0)) status = ST_BREAKDOWN;
    }
    if (state_writer()) {
        DevState *o = a.st_out;
        copy_state(o, S);
        if (status != RUNNING) {
            o->status = status;
        } else {
            o->iter = i + 1;
            o->gamma_prev = gamma_i;
            o->alpha_prev = alpha;
        }
        if (a.hist && i < a.hist_cap) {
            a.hist[(size_t)i * 5 + 1] = alpha;
            a.hist[(size_t)i * 5 + 4] = sp;
        }
    }
    if (status != RUNNING) return;

    double acc[2] = {0.0, 0.0};
    const uint32_t n = (uint32_t)a.A.n;
    const TileRange tr = tile_range(a.ntiles, a.xcd_map);
    for (int tile = tr.first; tile < tr.end; tile += tr.step) {
        const TileIdx<EPT> ti = tile_idx<EPT>(tile, n);
        double pe[EPT], se[EPT], re[EPT], xo[EPT];
#pragma unroll
        for (int j = 0; j < EPT; ++j) {
            pe[j] = lds<NT>(vp<T>(a, a.off_wout, ti.e[j]));
            se[j] = lds<NT>(vp<T>(a, a.off_s, ti.e[j]));
            re[j] = lds<NT>(vp<T>(a, a.off_r, ti.e[j]));
            xo[j] = lds<NT>(vp<double>(a, a.off_x, ti.e[j]));
        }
#pragma unroll
        for (int j = 0; j < EPT; ++j) {
            if (!ti.live[j]) continue;
            const uint32_t e = ti.e[j];
            sts<NT>(vp<double>(a, a.off_x, e), xo[j] + alpha * pe[j]);
            const double rn = rnd<T>(re[j] - alpha * se[j]);
            sts<NT>(vp<T>(a, a.off_r, e), rn);
            const double un = rnd<T>(minv<T, JAC, OP>(a, e, rn));
            acc[0] += rn * un;
            acc[1] += rn * rn;
        }
    }
    block_sum<2>(acc, lds_red);
    store_partial<2>(a.part_out, acc);
}

// ----------------------------------------------------------------- support

// partials of ||b - A x||^2 and ||b||^2 in binary64 (A in its storage
// precision); x is the internal copy, or the caller's when x_plain is set.
template <typename T, int OP, int EPT, int SELL = 0>
__device__ __forceinline__ void tile_resid(const PassArgs<T> &a, int tile, double (&acc)[2])
{
    const TileIdx<EPT> ti = tile_idx<EPT>(tile, (uint32_t)a.A.n);
    double be[EPT], ax[EPT];
    if (a.x_plain)
        tile_apply<T, OP, EPT, SELL>(a, tile, ti, ax, [&](uint32_t k) { return a.x_user[k]; });
    else
        tile_apply<T, OP, EPT, SELL>(a, tile, ti, ax, [&](uint32_t k) { return *vp<double>(a, a.off_x, k); });
#pragma unroll
    for (int j = 0; j < EPT; ++j) be[j] = a.b[ti.e[j]];
#pragma unroll
    for (int j = 0; j < EPT; ++j) {
        if (!ti.live[j]) continue;
        const double d = be[j] - ax[j];
        acc[0] += d * d;
        acc[1] += be[j] * be[j];
    }
}

template <typename T, int OP, int EPT, int SELL = 0>
__global__ void __launch_bounds__(kMaxBlock) k_resid(PassArgs<T> a)
{
    __shared__ double lds_red[kMaxWaves * kFields];
    double acc[2] = {0.0, 0.0};
    const TileRange tr = tile_range(a.ntiles, a.xcd_map);
    for (int tile = tr.first; tile < tr.end; tile += tr.step) tile_resid<T, OP, EPT, SELL>(a, tile, acc);
    block_sum<2>(acc, lds_red);
    store_partial<2>(a.part_out, acc);
}

// One block: stage 2 of `nparts` residual partials into out->true_res2 and
// out->spare[0] (= ||b||^2).
static __global__ void __launch_bounds__(1024) k_reduce_true(const double *part, int nparts, DevState *out)
{
    __shared__ double lds_red[kMaxWaves * kFields];
    double tot[2];
    stage2<2>(part, nparts, tot, lds_red);
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

// Sliced-ELL copy of a CSR operator (see sell_row), built once per solver.
// Step 1: the longest row of each 64-row slice, into sell_ptr[s].
static __global__ void __launch_bounds__(256) k_sell_width(const int32_t *row_ptr, int32_t n, int32_t *sell_ptr)
{
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;  // one wave per slice
    int32_t len = r < n ? row_ptr[r + 1] - row_ptr[r] : 0;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) len = max(len, __shfl_xor(len, o, 64));
    if ((threadIdx.x & 63) == 0 && r < n) sell_ptr[r >> 6] = len;
}

// Step 2 (one block): exclusive prefix sum of 64 x width over the slices,
// in place; sell_ptr[nslices] = the total, or -1 when it exceeds cap.
static __global__ void __launch_bounds__(1024) k_sell_scan(int32_t *sell_ptr, int32_t nslices, int64_t cap)
{
    __shared__ int64_t part[1024];
    const int per = (nslices + 1023) / 1024;
    const int s0 = min(nslices, (int)threadIdx.x * per), s1 = min(nslices, s0 + per);
    int64_t mine = 0;
    for (int s = s0; s < s1; ++s) mine += 64 * (int64_t)sell_ptr[s];
    part[threadIdx.x] = mine;
    __syncthreads();
    if (threadIdx.x == 0) {
        int64_t run = 0;
        for (int t = 0; t < 1024; ++t) {
            const int64_t v = part[t];
            part[t] = run;
            run += v;
        }
        sell_ptr[nslices] = run <= cap ? (int32_t)run : -1;
    }
    __syncthreads();
    int64_t run = part[threadIdx.x];
    for (int s = s0; s < s1; ++s) {
        const int64_t w = 64 * (int64_t)sell_ptr[s];
        sell_ptr[s] = (int32_t)min(run, cap);
        run += w;
    }
}

// Step 3: each row's entries into its slice column, padding with the row's
// own column and a zero value.  With c16 (every entry within 2^15 of its
// row) the columns go out as 16-bit column - row + 2^15 instead of into
// sell_col.
template <typename T>
__global__ void __launch_bounds__(256) k_sell_fill(OpDev<T> A, const int32_t *sell_ptr, int32_t *sell_col, T *sell_val,
                                                   uint16_t *c16, float *v32)
{
    const uint32_t r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= (uint32_t)A.n) return;
    const uint32_t s = r >> 6, lane = r & 63;
    const int32_t p0 = sell_ptr[s], w = (sell_ptr[s + 1] - p0) >> 6;
    const int32_t k0 = A.row_ptr[r], len = A.row_ptr[r + 1] - k0;
    for (int32_t k = 0; k < w; ++k) {
        const int32_t idx = p0 + (k << 6) + (int32_t)lane;
        const int32_t c = k < len ? A.col[k0 + k] : (int32_t)r;
        if (c16) c16[idx] = (uint16_t)(c - (int32_t)r + 32768);
        else sell_col[idx] = c;
        const T v = k < len ? A.val[k0 + k] : (T)0;
        if (v32) v32[idx] = (float)v;  // exact: checked at set-up
        else sell_val[idx] = v;
    }
}

// Whether some entry lies 2^15 or more columns from its row (*far = 1; the
// in-place copy then keeps 32-bit columns).
static __global__ void __launch_bounds__(256) k_sell_far(const int32_t *row_ptr, const int32_t *col, int32_t n, int *far)
{
    int f = 0;
    for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < n; r += (int64_t)gridDim.x * blockDim.x)
        for (int32_t k = row_ptr[r]; k < row_ptr[r + 1]; ++k) {
            const int64_t d = (int64_t)col[k] - r;
            f |= d < -32768 || d > 32767;
        }
    if (f) atomicOr(far, 1);
}

// The sorted form (see sell_sorted_rows), step 1: one wave per group of EPT
// x 64 rows (a wave's rows of a B-thread tile) ranks its rows by length,
// longest first, ties by position in the group; writes slot rank of the
// group as (length << 8) | position and each slice's width (the length of
// its first slot) into sell_ptr[slice].  A row of 2^23 entries or more
// gives its slice a width that no capacity admits, so the copy is not made.
template <int EPT>
static __global__ void __launch_bounds__(256) k_sell_sort(const int32_t *row_ptr, int32_t n, int32_t block,
                                                         int32_t ngroups, int32_t *sell_ptr, int32_t *perm)
{
    constexpr int R = EPT * 64;
    __shared__ int32_t len_s[4][R];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int64_t g = (int64_t)blockIdx.x * 4 + wave;
    if (g >= ngroups) return;  // the whole wave
    const int wpb = block >> 6;
    const int64_t first = (g / wpb) * (int64_t)block * EPT + (g % wpb) * 64 + lane;
    int32_t L[EPT];
#pragma unroll
    for (int j = 0; j < EPT; ++j) {
        const int64_t r = first + (int64_t)j * block;
        L[j] = r < n ? row_ptr[r + 1] - row_ptr[r] : 0;
        len_s[wave][j * 64 + lane] = L[j];
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
#pragma unroll
    for (int j = 0; j < EPT; ++j) {
        const int o = j * 64 + lane;
        int rank = 0;
        for (int q = 0; q < R; ++q) {
            const int32_t lq = len_s[wave][q];
            rank += (lq > L[j]) || (lq == L[j] && q < o);
        }
        const bool fits = L[j] < (1 << 23);
        perm[g * R + rank] = ((fits ? L[j] : 0) << 8) | o;
        if ((rank & 63) == 0) sell_ptr[g * EPT + (rank >> 6)] = fits ? L[j] : (INT32_MAX >> 6);
    }
}

// The sorted form, step 3 (after k_sell_scan over the slices): one thread
// per slot copies its row's entries into the slot's column of its slice,
// padding with the row's own column (the last row's for a slot past it) and
// a zero value.
// With c16 (every tile windowed) the columns go out as 16-bit offsets in
// the slot's tile window instead of into sell_col.
template <typename T, int EPT>
__global__ void __launch_bounds__(256) k_sell_fill_sorted(OpDev<T> A, int32_t block, int64_t slots,
                                                           const int32_t *sell_ptr, const int32_t *perm,
                                                           int32_t *sell_col, T *sell_val, const int2 *win,
                                                           uint16_t *c16, float *v32)
{
    const int64_t P = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (P >= slots) return;
    const int64_t s = P >> 6, g = s / EPT;
    const int32_t lane = (int32_t)(P & 63);
    const int32_t info = perm[P], len = info >> 8, o = info & 255;
    const int wpb = block >> 6;
    const int64_t r = (g / wpb) * (int64_t)block * EPT + (int64_t)(o >> 6) * block + (g % wpb) * 64 + (o & 63);
    const int32_t p0 = sell_ptr[s], w = (sell_ptr[s + 1] - p0) >> 6;
    const int32_t k0 = len > 0 ? A.row_ptr[r] : 0;  // len > 0 only for r < n
    // a slot past the last row (last tile only) pads with that row, inside
    // the tile's column window
    const int32_t pad = r < A.n ? (int32_t)r : A.n - 1;
    const int32_t base = c16 ? win[(g / wpb)].x : 0;  // the tile's window
    for (int32_t k = 0; k < w; ++k) {
        const int64_t idx = p0 + ((int64_t)k << 6) + lane;
        const int32_t c = k < len ? A.col[k0 + k] : pad;
        if (c16) c16[idx] = (uint16_t)(c - base);
        else sell_col[idx] = c;
        const T v = k < len ? A.val[k0 + k] : (T)0;
        if (v32) v32[idx] = (float)v;  // exact: checked at set-up
        else sell_val[idx] = v;
    }
}

// Whether some matrix value is not a binary32 number (*inexact = 1; the
// binary64 form's copy then keeps binary64 values).
template <typename T>
__global__ void __launch_bounds__(256) k_vals_binary32(const T *val, int64_t nnz, int *inexact)
{
    int f = 0;
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < nnz; k += (int64_t)gridDim.x * blockDim.x) {
        const double v = (double)val[k];
        f |= !((double)(float)v == v);
    }
    if (f) atomicOr(inexact, 1);
}

// The sorted form, step 4: one block per tile of `rows` rows finds the
// smallest and largest column its rows gather (their entries and, for the
// padding, their own indices) and writes (first column, width), or width
// -1 when the window is wider than kSellWindow.
static __global__ void __launch_bounds__(256) k_sell_window(const int32_t *row_ptr, const int32_t *col, int32_t n,
                                                           int32_t rows, int2 *win)
{
    __shared__ int32_t lo_s[256], hi_s[256];
    const int64_t r0 = (int64_t)blockIdx.x * rows, r1 = min((int64_t)n, r0 + rows);  // r0 < n: one block per tile
    int32_t lo = (int32_t)r0, hi = (int32_t)(r1 - 1);
    const int32_t e0 = row_ptr[r0], e1 = row_ptr[r1];
    for (int32_t k = e0 + (int32_t)threadIdx.x; k < e1; k += blockDim.x) {
        lo = min(lo, col[k]);
        hi = max(hi, col[k]);
    }
    lo_s[threadIdx.x] = lo;
    hi_s[threadIdx.x] = hi;
    __syncthreads();
    for (int o = blockDim.x / 2; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) {
            lo_s[threadIdx.x] = min(lo_s[threadIdx.x], lo_s[threadIdx.x + o]);
            hi_s[threadIdx.x] = max(hi_s[threadIdx.x], hi_s[threadIdx.x + o]);
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const int64_t w = (int64_t)hi_s[0] - lo_s[0] + 1;
        win[blockIdx.x] = w <= kSellWindow ? make_int2(lo_s[0], (int32_t)w) : make_int2(0, -1);
    }
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
