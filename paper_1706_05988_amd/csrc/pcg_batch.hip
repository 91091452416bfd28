// pcg_batch.hip -- the batched persistent pass (kernels), the batch engine
// shared with the server, and pcg_batch_workspace_size / pcg_batch_solve.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <vector>

#include "pcg.h"
#include "pcg_batch_engine.h"

namespace pcg {

// ----------------------------------------------------------------- kernels

template <typename T>
__device__ __forceinline__ PassArgs<T> batch_args(const BatchSys &D, const BatchState &S)
{
    PassArgs<T> a;
    a.A.n = D.n;
    a.A.nx = D.nx;
    a.A.ny = D.ny;
    a.A.nz = D.nz;
    a.A.dx = D.dx;
    a.A.dxy = D.dxy;
    a.A.centre = D.centre;
    a.A.off = D.off;
    a.A.row_ptr = D.row_ptr;
    a.A.col = D.col;
    a.A.val = (const T *)D.val;
    a.dinv = (const T *)D.dinv;
    a.dinv_s = D.dinv_s;
    a.b = D.b;
    a.x_user = D.x;
    a.blk = D.blk;
    a.tile_bytes = D.tile_bytes;
    a.off_x = D.off_slot[V_X];
    a.off_r = D.off_slot[V_R];
    a.off_u = D.off_slot[V_U];
    // ITER reads w[wcur] and writes w[1 - wcur]; INIT1 writes w_0 into the
    // slot the first ITER pass reads
    a.off_win = D.off_slot[S.wcur ? V_W1 : V_W0];
    a.off_wout = S.phase == PH_INIT1 ? a.off_win : D.off_slot[S.wcur ? V_W0 : V_W1];
    a.off_z = D.off_slot[V_Z];
    a.off_q = D.off_slot[V_Q];
    a.off_s = D.off_slot[V_S];
    a.off_t = D.off_slot[V_T];
    a.off_p = D.off_slot[V_P];
    a.clear = CLR_Z | CLR_S | CLR_T | (D.jac ? (CLR_Q | CLR_P) : 0u);
    a.sigma = D.sigma;
    a.copy_out = S.phase == PH_COPYOUT;
    a.x_plain = 0;
    a.sell_ptr = D.sell_ptr;
    a.sell_col = D.sell_col;
    a.sell_val = (const T *)D.sell_val;
    a.sell_perm = D.sell_perm;
    a.sell_win = D.sell_win;
    a.sell_c16 = D.sell_c16;
    a.sell_v32 = D.sell_v32;
    return a;
}

// One tile of one system in its current phase; NF partials into acc.
template <typename T, int OP, bool JAC, int SELL>
__device__ __forceinline__ void batch_tile_form(const PassArgs<T> &a, const BatchState &S, int tile, double (&acc)[3])
{
    constexpr int E = kBatchEPT;
    switch (S.phase) {
    case PH_COPYIN:
    case PH_COPYOUT: tile_copy_x<T, E>(a, tile); break;
    case PH_INIT0: {
        double b1[1] = {0.0};
        tile_init0<T, OP, JAC, JAC, E, true, SELL>(a, tile, b1);
        acc[0] = b1[0];
        break;
    }
    case PH_INIT1: tile_init1<T, OP, JAC, E, true, SELL>(a, tile, acc); break;
    case PH_ITER: {
        PipeScalars sc;
        sc.alpha = S.alpha;
        sc.beta = S.beta;
        sc.sigma = a.sigma;
        sc.dsig = 0.0;
        sc.alpha_prev = S.alpha_prev;
        // x every other iteration (the same two updates in the same order)
        if (lag_mode(S.iter, S.i_start) == X_SKIP) tile_pipe<T, OP, JAC, E, true, false, X_SKIP, SELL>(a, tile, sc, acc);
        else tile_pipe<T, OP, JAC, E, true, false, X_CATCHUP, SELL>(a, tile, sc, acc);
        break;
    }
    case PH_XFIX: tile_x_fixup<T, JAC, E>(a, tile, S.alpha); break;
    case PH_RESID: {
        double r2[2] = {0.0, 0.0};
        tile_resid<T, OP, E, SELL>(a, tile, r2);
        acc[0] = r2[0];
        acc[1] = r2[1];
        break;
    }
    default: break;
    }
}

// The CSR operand of a system: its sorted sliced-ELL copy, in-place copy, or
// rows; the same form in every phase.
template <typename T, int OP, bool JAC>
__device__ __forceinline__ void batch_tile(const PassArgs<T> &a, const BatchState &S, int tile, double (&acc)[3])
{
    if constexpr (OP == OP_CSR) {
        if (a.sell_perm) return batch_tile_form<T, OP, JAC, 2>(a, S, tile, acc);
        if (a.sell_ptr) return batch_tile_form<T, OP, JAC, 1>(a, S, tile, acc);
    }
    batch_tile_form<T, OP, JAC, 0>(a, S, tile, acc);
}

template <typename T, int OP>
__device__ __forceinline__ void batch_tile_op(const BatchSys &D, const BatchState &S, int tile, double (&acc)[3])
{
    const PassArgs<T> a = batch_args<T>(D, S);
    if (D.jac) batch_tile<T, OP, true>(a, S, tile, acc);
    else batch_tile<T, OP, false>(a, S, tile, acc);
}

// One item of a system.  SPEC = kind * 2 + jac fixes the operator and the
// preconditioner at compile time for a batch whose systems all share them
// (the kernel then holds one tile body instead of six, and needs far fewer
// registers); kSpecAny reads them per system.
template <typename T, int SPEC>
__device__ __forceinline__ void batch_item(const BatchSys &D, const BatchState &S, int tile, double (&acc)[3])
{
    if constexpr (SPEC == kSpecAny) {
        switch (D.kind) {
        case PCG_OP_STENCIL2D5: batch_tile_op<T, OP_2D5>(D, S, tile, acc); break;
        case PCG_OP_STENCIL3D7: batch_tile_op<T, OP_3D7>(D, S, tile, acc); break;
        default: batch_tile_op<T, OP_CSR>(D, S, tile, acc); break;
        }
    } else {
        constexpr int kind = SPEC >> 1;
        constexpr int OP = kind == PCG_OP_STENCIL2D5 ? OP_2D5 : kind == PCG_OP_STENCIL3D7 ? OP_3D7 : OP_CSR;
        batch_tile<T, OP, (SPEC & 1) != 0>(batch_args<T>(D, S), S, tile, acc);
    }
}

__device__ __forceinline__ void batch_hist(const BatchSys &D, int i, double res, double alpha, double beta,
                                           double gamma, double delta)
{
    if (D.hist && i >= 0 && i < D.hist_cap) {
        double *row = D.hist + (size_t)i * 5;
        row[0] = res;
        row[1] = alpha;
        row[2] = beta;
        row[3] = gamma;
        row[4] = delta;
    }
}

// Decision of the top of iteration i from gamma_i, delta_i, rho_i (the same
// rules as the single-system pass head).  Returns the new state; the writer
// block records the history row.
__device__ __forceinline__ BatchState batch_decide(const BatchSys &D, BatchState S, double gamma, double delta,
                                                   double rho, bool writer)
{
    const int i = S.iter;
    int status = RUNNING;
    double alpha = __builtin_nan(""), beta = __builtin_nan("");
    if (!isfinite(gamma) || !isfinite(delta) || !isfinite(rho)) {
        status = ST_NONFINITE;
    } else if (sqrt(rho) <= D.rtol * sqrt(S.bnorm2)) {
        status = ST_CONVERGED;
    } else if (i >= D.max_iter) {
        status = ST_MAX_ITER;
    } else if (!(gamma > 0.0) || !(delta > 0.0)) {
        status = ST_BREAKDOWN;
    } else {
        if (i > S.i_start) {
            beta = gamma / S.gamma;                          // gamma_{i-1}
            alpha = 1.0 / (delta / gamma - beta / S.alpha);  // alpha_{i-1}
        } else {
            beta = 0.0;
            alpha = gamma / delta;
        }
        if (!(isfinite(alpha) && alpha > 0.0)) status = ST_BREAKDOWN;
    }
    if (writer) batch_hist(D, i, sqrt(rho / S.bnorm2), alpha, beta, gamma, delta);
    S.rho = rho;
    if (status == RUNNING) {
        S.phase = PH_ITER;
        S.alpha_prev = S.alpha;
        S.alpha = alpha;
        S.beta = beta;
        S.gamma = gamma;
    } else {
        S.status = status;
        // the last iteration pass (i - 1) left x: complete it with
        // alpha_{i-1} p_{i-1} (S.alpha, p as that pass stored it) first
        S.phase = (i > S.i_start && ((i - 1 - S.i_start) & 1) == 0) ? PH_XFIX : PH_RESID;
    }
    return S;
}

// The phase after the one S records, from that pass's partial sums `tot`.
__device__ __forceinline__ BatchState batch_next(const BatchSys &D, BatchState S, const double (&tot)[3], bool writer)
{
    switch (S.phase) {
    case PH_ADMIT: S.phase = PH_COPYIN; break;
    case PH_COPYIN: S.phase = PH_INIT0; break;
    case PH_INIT0:
        S.bnorm2 = tot[0];
        if (!isfinite(tot[0])) {
            S.status = ST_NONFINITE;
            S.phase = PH_COPYOUT;
        } else {
            S.phase = PH_INIT1;
        }
        break;
    case PH_INIT1: S = batch_decide(D, S, tot[0], tot[1], tot[2], writer); break;
    case PH_ITER:
        S.iter += 1;
        S.wcur ^= 1;
        S = batch_decide(D, S, tot[0], tot[1], tot[2], writer);
        break;
    case PH_XFIX: S.phase = PH_RESID; break;
    case PH_RESID: {
        S.true_res2 = tot[0];
        const bool restart = S.status == ST_CONVERGED && D.true_check && S.restarts < D.replace_max &&
                             S.iter < D.max_iter && sqrt(tot[0]) > D.rtol * sqrt(S.bnorm2);
        if (restart) {
            S.restarts += 1;
            S.status = RUNNING;
            S.i_start = S.iter;
            S.wcur = 0;
            S.phase = PH_INIT0;
        } else {
            S.phase = PH_COPYOUT;
        }
        break;
    }
    case PH_COPYOUT: S.phase = PH_DONE; break;
    default: break;
    }
    if (S.phase < PH_DONE) ++S.passes;
    return S;
}

// One pass over every item (system, tile).  Pass parity `par`: states and
// partials are read from slot par and written to slot 1 - par.  HEAD: the
// item block takes its system's transition itself; otherwise k_batch_trans
// has already written the transitioned state into slot 1 - par.
template <typename T, bool HEAD, int SPEC>
__global__ void __launch_bounds__(kBatchBlock) k_batch_step(BatchTables tb, int par)
{
    __shared__ double lds_red[kMaxWaves * kFields];
    const int nitems = tb.counts[0];
    const int G = gridDim.x;
    uint2 next = (int)blockIdx.x < nitems ? tb.items[blockIdx.x] : make_uint2(0u, 0u);
    for (int it = blockIdx.x; it < nitems; it += G) {
        const uint2 si = next;
        // the next item's (system, tile) is fetched while this item streams
        if (it + G < nitems) next = tb.items[it + G];
        const uint32_t s = si.x, tile = si.y;
        const BatchState *Sin = tb.st + (size_t)par * tb.max_sys + s;
        BatchState *Sout = tb.st + (size_t)(1 - par) * tb.max_sys + s;
        const BatchSys &D = tb.sys[s];
        BatchState S;
        if constexpr (HEAD) {
            const bool writer = tile == 0 && threadIdx.x == 0;
            const int phase = Sin->phase;
            if (phase >= PH_DONE) {
                if (writer) *Sout = *Sin;
                continue;
            }
            double tot[3] = {0.0, 0.0, 0.0};
            if (phase != PH_ADMIT && phase != PH_COPYIN && phase != PH_COPYOUT && phase != PH_XFIX)
                stage2<3>(D.part + (size_t)par * D.ntiles * kBatchWaves * kFields, D.ntiles * kBatchWaves, tot, lds_red);
            S = batch_next(D, *Sin, tot, writer);
            if (writer) *Sout = S;
        } else {
            S = *Sout;
        }
        double acc[3] = {0.0, 0.0, 0.0};
        if (S.phase >= PH_DONE) continue;
        batch_item<T, SPEC>(D, S, tile, acc);
        // one partial per wave: no block barrier between items
#pragma unroll
        for (int f = 0; f < 3; ++f) acc[f] = wave_sum(acc[f]);
        if ((threadIdx.x & 63) == 0) {
            double *pp = D.part + (((size_t)(1 - par) * D.ntiles + tile) * kBatchWaves + (threadIdx.x >> 6)) * kFields;
            pp[0] = acc[0];
            pp[1] = acc[1];
            pp[2] = acc[2];
        }
    }
}

// Split mode without large systems: the transition of every listed system,
// one block per system.
__global__ void __launch_bounds__(kBatchBlock) k_batch_trans(BatchTables tb, int par)
{
    __shared__ double lds_red[kMaxWaves * kFields];
    const int nact = tb.counts[1];
    for (int k = blockIdx.x; k < nact; k += gridDim.x) {
        const uint32_t s = tb.active[k];
        const BatchState *Sin = tb.st + (size_t)par * tb.max_sys + s;
        BatchState *Sout = tb.st + (size_t)(1 - par) * tb.max_sys + s;
        const BatchSys &D = tb.sys[s];
        const int phase = Sin->phase;
        if (phase >= PH_DONE) {
            if (threadIdx.x == 0) *Sout = *Sin;
            continue;
        }
        double tot[3] = {0.0, 0.0, 0.0};
        if (phase != PH_ADMIT && phase != PH_COPYIN && phase != PH_COPYOUT && phase != PH_XFIX)
            stage2<3>(D.part + (size_t)par * D.ntiles * kBatchWaves * kFields, D.ntiles * kBatchWaves, tot, lds_red);
        const BatchState S = batch_next(D, *Sin, tot, threadIdx.x == 0);
        if (threadIdx.x == 0) *Sout = S;
    }
}

// Split mode with large systems, in place of k_batch_trans: the listed
// systems of one chunk are transitioned as there; each (system, chunk) entry
// of a large system sums its kChunkParts partials of slot par in the stage-2
// order into the system's chunk array, and the block that writes the last
// chunk sum of its system (an agent-scope counter; release before, acquire
// after) adds the chunk sums in chunk order and takes the transition.  The
// counter returns to zero there, for the next pass's kernel.
__global__ void __launch_bounds__(kBatchBlock) k_batch_trans_chunked(BatchTables tb, int par)
{
    constexpr int kStage = 1024;  // chunk sums staged in LDS at a time
    __shared__ double lds_red[kMaxWaves * kFields];
    __shared__ double staged[kStage * 3];
    __shared__ int last;
    const int ni = tb.counts[0], nact = tb.counts[1], nc = tb.counts[2];
    for (int k = blockIdx.x; k < nact + nc; k += gridDim.x) {
        uint32_t s;
        int c = 0;
        if (k < nact) {
            s = tb.active[k];
            if (tb.sys[s].nchunks > 1) continue;  // its chunk entries take it
        } else {
            const uint2 sc = tb.items[ni + (k - nact)];
            s = sc.x;
            c = (int)sc.y;
        }
        const BatchSys &D = tb.sys[s];
        const BatchState *Sin = tb.st + (size_t)par * tb.max_sys + s;
        BatchState *Sout = tb.st + (size_t)(1 - par) * tb.max_sys + s;
        const int phase = Sin->phase;
        if (phase >= PH_DONE) {
            if (c == 0 && threadIdx.x == 0) *Sout = *Sin;
            continue;
        }
        const bool sums = phase != PH_ADMIT && phase != PH_COPYIN && phase != PH_COPYOUT && phase != PH_XFIX;
        const int nparts = D.ntiles * kBatchWaves;
        double tot[3] = {0.0, 0.0, 0.0};
        if (D.nchunks <= 1) {
            if (sums) stage2<3>(D.part + (size_t)par * nparts * kFields, nparts, tot, lds_red);
        } else {
            double cs[3] = {0.0, 0.0, 0.0};
            const int p0 = c * kChunkParts, np = min(kChunkParts, nparts - p0);
            if (sums) stage2<3>(D.part + ((size_t)par * nparts + p0) * kFields, np, cs, lds_red);
            if (threadIdx.x == 0) {
                double *o = D.chunk + ((size_t)par * D.nchunks + c) * kFields;
                o[0] = cs[0];
                o[1] = cs[1];
                o[2] = cs[2];
                const int before =
                    __hip_atomic_fetch_add(D.chunks_done, 1, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
                last = before == D.nchunks - 1;
                if (last) *D.chunks_done = 0;
            }
            __syncthreads();
            const bool mine = last != 0;
            __syncthreads();  // `last` is read before the next entry writes it
            if (!mine) continue;
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
            // the chunk sums, added in chunk order (the same bits in every
            // thread); loaded into LDS together, so the ordered sum waits on
            // one memory latency per kStage chunks instead of one per chunk
            const double *all = D.chunk + (size_t)par * D.nchunks * kFields;
            for (int q0 = 0; q0 < D.nchunks; q0 += kStage) {
                const int cnt = min(kStage, D.nchunks - q0);
                for (int q = threadIdx.x; q < cnt; q += blockDim.x)
#pragma unroll
                    for (int f = 0; f < 3; ++f) staged[q * 3 + f] = all[(q0 + q) * kFields + f];
                __syncthreads();
                for (int q = 0; q < cnt; ++q)
#pragma unroll
                    for (int f = 0; f < 3; ++f) tot[f] += staged[q * 3 + f];
                __syncthreads();
            }
        }
        const BatchState S = batch_next(D, *Sin, tot, threadIdx.x == 0);
        if (threadIdx.x == 0) *Sout = S;
    }
}

template <typename T, bool HEAD>
static void launch_step(int spec, dim3 g, dim3 b, hipStream_t st, const BatchTables &tb, int par)
{
    switch (spec) {
    case 0: hipLaunchKernelGGL((k_batch_step<T, HEAD, 0>), g, b, 0, st, tb, par); break;
    case 1: hipLaunchKernelGGL((k_batch_step<T, HEAD, 1>), g, b, 0, st, tb, par); break;
    case 2: hipLaunchKernelGGL((k_batch_step<T, HEAD, 2>), g, b, 0, st, tb, par); break;
    case 3: hipLaunchKernelGGL((k_batch_step<T, HEAD, 3>), g, b, 0, st, tb, par); break;
    case 4: hipLaunchKernelGGL((k_batch_step<T, HEAD, 4>), g, b, 0, st, tb, par); break;
    case 5: hipLaunchKernelGGL((k_batch_step<T, HEAD, 5>), g, b, 0, st, tb, par); break;
    default: hipLaunchKernelGGL((k_batch_step<T, HEAD, kSpecAny>), g, b, 0, st, tb, par); break;
    }
}

// ----------------------------------------------------------------- engine

#define BCHK(call)                                        \
    do {                                                  \
        hipError_t e_ = (call);                           \
        if (e_ != hipSuccess) return hip_fail(e_, #call); \
    } while (0)

static size_t up256(size_t v) { return (v + 255) & ~size_t(255); }

// The work list, one block uploaded in one copy: the two counts (16 bytes),
// the listed systems (padded to 8 bytes), then the (system, tile) pairs.
static size_t list_items_off(int max_sys) { return 16 + 8 * (size_t)((max_sys + 1) / 2); }
// (system, chunk) entries: a system of t work tiles has ceil(4 t / 1024) <= t / 256 + 1 chunks
static int64_t max_chunks(int max_sys, int64_t max_items) { return max_items / 256 + max_sys + 1; }
static size_t list_bytes(int max_sys, int64_t max_items)
{
    return list_items_off(max_sys) + 8 * (size_t)(max_items + max_chunks(max_sys, max_items));
}

size_t BatchEngine::table_bytes(int max_sys, int64_t max_items)
{
    return up256(sizeof(BatchSys) * max_sys) + up256(sizeof(BatchState) * 2 * (size_t)max_sys) +
           up256(list_bytes(max_sys, max_items));
}

pcg_status BatchEngine::system_layout(const pcg_operator *op, const pcg_options *opt, SysLayout *L)
{
    const size_t n = (size_t)op->n;
    const uint32_t es = opt->prec == PCG_FP64 ? 8 : 4;
    const bool jac = opt->pc == PCG_PC_JACOBI;
    SysLayout l{};
    for (int k = 0; k < V_COUNT; ++k) l.off_slot[k] = kNoSlot;
    uint32_t tb = 0;
    auto slot = [&](int k, uint32_t bytes_per) {
        l.off_slot[k] = tb;
        tb += kBlk * bytes_per;
    };
    slot(V_X, 8);
    slot(V_R, es);
    slot(V_W0, es);
    slot(V_W1, es);
    slot(V_S, es);
    slot(V_Z, es);
    slot(V_T, es);
    if (jac) {
        slot(V_U, es);
        slot(V_Q, es);
        slot(V_P, es);
    }
    l.tile_bytes = tb;
    l.ntiles = (int32_t)((n + kBlk - 1) / kBlk);
    l.nwork = (int32_t)((n + kBatchBlock * kBatchEPT - 1) / (kBatchBlock * kBatchEPT));
    size_t off = 0;
    l.blk = off;
    off += up256((size_t)l.ntiles * tb);
    l.part = off;
    off += up256((size_t)2 * l.nwork * kBatchWaves * kFields * 8);  // two partial slots, one per wave
    l.nchunks = (int32_t)(((int64_t)l.nwork * kBatchWaves + kChunkParts - 1) / kChunkParts);
    l.chunk = l.chunks_done = SIZE_MAX;
    if (l.nchunks > 1) {
        l.chunk = off;
        off += up256((size_t)2 * l.nchunks * kFields * 8);
        l.chunks_done = off;
        off += 256;
    }
    l.dinv = SIZE_MAX;
    if (op->kind == PCG_OP_CSR && jac) {
        l.dinv = off;
        off += up256(n * es);
    }
    l.hist = SIZE_MAX;
    if (opt->history_cap > 0) {
        l.hist = off;
        off += up256((size_t)opt->history_cap * PCG_HISTORY_FIELDS * 8);
    }
    l.flag = off;
    off += 256;
    l.gersh = off;
    off += up256((size_t)kGershBlocks * 2 * 8);
    // the iteration pass of a CSR system reads a sliced-ELL copy where its
    // padding stays within a quarter of nnz: rows in place, or sorted within
    // each wave's rows of a work tile (whichever is smaller)
    l.sell_ptr = l.sort_ptr = l.sort_perm = l.sort_win = l.sell_col = l.sell_val = SIZE_MAX;
    l.nslices = l.sort_nslices = 0;
    l.sell_cap = 0;
    if (op->kind == PCG_OP_CSR) {
        const int64_t cap = op->nnz + op->nnz / 4 + 4096;
        const int64_t slots = (int64_t)l.nwork * kBatchBlock * kBatchEPT;
        if (cap < (int64_t(1) << 31) - 64 && slots < (int64_t(1) << 31) - 1) {
            l.sell_cap = cap;
            l.nslices = (int32_t)((n + 63) / 64);
            l.sell_ptr = off;
            off += up256((size_t)(l.nslices + 1) * 4);
            l.sort_nslices = (int32_t)(slots / 64);
            l.sort_ptr = off;
            off += up256((size_t)(l.sort_nslices + 1) * 4);
            l.sort_perm = off;
            off += up256((size_t)slots * 4);
            l.sort_win = off;
            off += up256((size_t)l.nwork * 8);
            l.sell_col = off;
            off += up256((size_t)cap * 4);
            l.sell_val = off;
            off += up256((size_t)cap * es);
        }
    }
    l.bytes = off;
    *L = l;
    return PCG_OK;
}

pcg_status BatchEngine::validate(const pcg_operator *op, const pcg_options *opt)
{
    pcg_status st = validate_options(opt);
    if (st) return st;
    if ((st = validate_operator(op, opt->prec))) return st;
    if (opt->method == PCG_CG || opt->method == PCG_PIPE_VAR_SHIFT || opt->method == PCG_PIPE_RR)
        return invalid("the batched pass runs the constant-shift pipelined methods (PCG_PIPE, PCG_PIPE_SHIFT)");
    if (opt->flags) return invalid("the batched pass takes no option flags");
    if (opt->prec != prec_) return invalid("every system of a batch must use the batch's precision");
    return PCG_OK;
}

pcg_status BatchEngine::init(char *tables, int max_sys, int64_t max_items, int prec, hipStream_t stream, int K)
{
    max_sys_ = max_sys;
    max_items_ = max_items;
    prec_ = prec;
    stream_ = stream;
    K_ = K > 0 ? K + (K & 1) : 32;  // even: a launch starts at state slot 0
    // one block per listed system in the transition kernel (its chain of
    // dependent loads and a block reduction per system is what it costs)
    trans_grid_ = std::max(256, std::min(max_sys, 2048));
    size_t off = 0;
    auto take = [&](size_t b) {
        char *p = tables + off;
        off += up256(b);
        return p;
    };
    d_sys_ = (BatchSys *)take(sizeof(BatchSys) * max_sys);
    d_st_ = (BatchState *)take(sizeof(BatchState) * 2 * (size_t)max_sys);
    d_list_ = take(list_bytes(max_sys, max_items));
    sys_.assign(max_sys, BatchSys{});
    in_use_.assign(max_sys, 0);
    listed_.assign(max_sys, 0);
    BCHK(hipHostMalloc((void **)&h_st_, sizeof(BatchState) * max_sys, hipHostMallocDefault));
    BCHK(hipHostMalloc((void **)&h_list_, list_bytes(max_sys, max_items), hipHostMallocDefault));
    BCHK(hipEventCreate(&ev0_));
    BCHK(hipEventCreate(&ev1_));
    BCHK(hipEventCreate(&ev_up_));
    for (int k = 0; k < max_sys; ++k) {
        h_st_[k] = BatchState{};
        h_st_[k].phase = PH_FREE;
    }
    BCHK(hipMemcpyAsync(d_st_, h_st_, sizeof(BatchState) * max_sys, hipMemcpyHostToDevice, stream_));
    BCHK(hipMemcpyAsync(d_st_ + max_sys, h_st_, sizeof(BatchState) * max_sys, hipMemcpyHostToDevice, stream_));
    int32_t zero[2] = {0, 0};
    BCHK(hipMemcpyAsync(d_list_, zero, sizeof(zero), hipMemcpyHostToDevice, stream_));
    BCHK(hipStreamSynchronize(stream_));
    return PCG_OK;
}

BatchEngine::~BatchEngine()
{
    for (int k = 0; k < 3; ++k) {
        if (gexec_[k]) (void)hipGraphExecDestroy(gexec_[k]);
        if (graph_[k]) (void)hipGraphDestroy(graph_[k]);
    }
    if (h_st_) (void)hipHostFree(h_st_);
    if (h_list_) (void)hipHostFree(h_list_);
    if (ev0_) (void)hipEventDestroy(ev0_);
    if (ev1_) (void)hipEventDestroy(ev1_);
    if (ev_up_) (void)hipEventDestroy(ev_up_);
}

pcg_status BatchEngine::admit(const pcg_operator *op, const pcg_options *opt, const double *b, double *x, char *region,
                              int *slot_out)
{
    pcg_status st = validate(op, opt);
    if (st) return st;
    if (!b || !x || b == x) return invalid("b and x must be non-null and distinct");
    if (((uintptr_t)b % 8) || ((uintptr_t)x % 8)) return invalid("b and x must be 8-byte aligned");
    if (!region || ((uintptr_t)region % 256)) return invalid("system region must be 256-byte aligned");
    int slot = -1;
    for (int k = 0; k < max_sys_; ++k)
        if (!in_use_[k]) {
            slot = k;
            break;
        }
    if (slot < 0) return PCG_ERR_BUDGET;
    SysLayout L;
    system_layout(op, opt, &L);
    const int jac = opt->pc == PCG_PC_JACOBI;
    double gersh[2] = {0.0, 0.0};
    if (op->kind == PCG_OP_CSR) {
        if ((st = csr_setup(op, opt->prec, jac, jac ? region + L.dinv : nullptr, (int *)(region + L.flag), stream_)))
            return st;
        if (opt->method == PCG_PIPE_SHIFT && std::isnan(opt->sigma) &&
            (st = csr_gershgorin(op, opt->prec, jac, (double *)(region + L.gersh), stream_, &gersh[0], &gersh[1])))
            return st;
    }
    int form = 0, col_bits = 0, val_bits = 0;
    int64_t entries = 0;
    if (op->kind == PCG_OP_CSR && L.sell_col != SIZE_MAX) {
        SellPlan p;
        p.sell_ptr = (int32_t *)(region + L.sell_ptr);
        p.nslices = L.nslices;
        p.sort_ptr = (int32_t *)(region + L.sort_ptr);
        p.sort_perm = (int32_t *)(region + L.sort_perm);
        p.sort_nslices = L.sort_nslices;
        p.sort_block = kBatchBlock;
        p.sort_ept = kBatchEPT;
        p.cap = L.sell_cap;
        p.col = (int32_t *)(region + L.sell_col);
        p.val = region + L.sell_val;
        p.win = (int2 *)(region + L.sort_win);
        p.scratch = (int *)(region + L.flag) + 1;  // after the CSR check's flag
        if ((st = sell_build(op, opt->prec, p, stream_, &form, &entries, &col_bits, &val_bits))) return st;
    }
    BatchSys D{};
    D.kind = op->kind;
    D.jac = jac;
    D.n = (int32_t)op->n;
    D.ntiles = L.nwork;
    D.nx = op->nx;
    D.ny = op->ny;
    D.nz = op->kind == PCG_OP_STENCIL3D7 ? op->nz : 1;
    D.max_iter = opt->max_iter;
    if (op->kind != PCG_OP_CSR) {
        D.dx = make_fastdiv((uint32_t)op->nx);
        D.dxy = make_fastdiv((uint32_t)op->nx * (uint32_t)op->ny);
    }
    D.centre = op->diag + op->shift;
    D.off = op->offdiag;
    D.dinv_s = 1.0;
    if (jac && op->kind != PCG_OP_CSR)
        D.dinv_s = opt->prec == PCG_FP64 ? 1.0 / D.centre : (double)(float)(1.0 / D.centre);
    D.sigma = default_sigma(op, opt, gersh);
    D.rtol = opt->rtol;
    D.row_ptr = op->row_ptr;
    D.col = op->col_idx;
    D.val = op->vals;
    D.dinv = L.dinv == SIZE_MAX ? nullptr : region + L.dinv;
    D.b = b;
    D.x = x;
    D.blk = region + L.blk;
    D.tile_bytes = L.tile_bytes;
    for (int k = 0; k < V_COUNT; ++k) D.off_slot[k] = L.off_slot[k];
    D.part = (double *)(region + L.part);
    D.nchunks = L.nchunks;
    D.chunk = L.chunk == SIZE_MAX ? nullptr : (double *)(region + L.chunk);
    D.chunks_done = L.chunks_done == SIZE_MAX ? nullptr : (int32_t *)(region + L.chunks_done);
    D.sell_ptr = form == 1 ? (const int32_t *)(region + L.sell_ptr)
                 : form == 2 ? (const int32_t *)(region + L.sort_ptr)
                             : nullptr;
    D.sell_col = form ? (const int32_t *)(region + L.sell_col) : nullptr;
    D.sell_perm = form == 2 ? (const int32_t *)(region + L.sort_perm) : nullptr;
    D.sell_win = form == 2 ? (const int2 *)(region + L.sort_win) : nullptr;
    D.sell_c16 = form && col_bits == 16 ? (const uint16_t *)(region + L.sell_col) : nullptr;
    D.sell_v32 = form && opt->prec == PCG_FP64 && val_bits == 32 ? (const float *)(region + L.sell_val) : nullptr;
    D.sell_val = form ? (const void *)(region + L.sell_val) : nullptr;
    // the counter of written chunk sums starts at zero (the transition that
    // completes it sets it back)
    if (D.chunks_done) BCHK(hipMemsetAsync(D.chunks_done, 0, sizeof(int32_t), stream_));
    D.hist = L.hist == SIZE_MAX ? nullptr : (double *)(region + L.hist);
    D.hist_cap = opt->history_cap;
    D.replace_max = opt->replace_max;
    D.true_check = opt->true_residual_check;
    sys_[slot] = D;
    in_use_[slot] = 1;
    BatchState S{};
    S.phase = PH_ADMIT;
    S.status = RUNNING;
    BCHK(hipEventSynchronize(ev_up_));  // h_st_ may still be the source of an upload
    h_st_[slot] = S;
    // descriptor and state go up with the next table upload, before the next launch
    if (D.hist) BCHK(hipMemsetAsync(D.hist, 0xff, (size_t)D.hist_cap * PCG_HISTORY_FIELDS * 8, stream_));
    tables_dirty_ = true;
    slots_dirty_ = true;
    *slot_out = slot;
    return PCG_OK;
}

void BatchEngine::release(int slot)
{
    in_use_[slot] = 0;
    (void)hipEventSynchronize(ev_up_);  // h_st_ may still be the source of an upload
    h_st_[slot].phase = PH_FREE;
    tables_dirty_ = true;
    slots_dirty_ = true;
}

pcg_status BatchEngine::upload_tables()
{
    // items of every system still working, in slot order; the list of those
    // systems the same
    // the previous upload from the staging buffers has been carried out
    BCHK(hipEventSynchronize(ev_up_));
    int32_t *cnt = reinterpret_cast<int32_t *>(h_list_);
    uint32_t *act = reinterpret_cast<uint32_t *>(h_list_ + 16);
    uint32_t *items = reinterpret_cast<uint32_t *>(h_list_ + list_items_off(max_sys_));
    int64_t ni = 0;
    int na = 0, most = 0;
    for (int s = 0; s < max_sys_; ++s) {
        listed_[s] = 0;
        if (!in_use_[s] || h_st_[s].phase >= PH_DONE) continue;
        listed_[s] = 1;
        act[na++] = (uint32_t)s;
        most = std::max(most, (int)sys_[s].ntiles);
        for (int t = 0; t < sys_[s].ntiles; ++t) {
            if (ni >= max_items_) return PCG_ERR_BUDGET;
            items[2 * ni] = (uint32_t)s;
            items[2 * ni + 1] = (uint32_t)t;
            ++ni;
        }
    }
    // the chunk entries of the large systems follow the items
    int64_t nc = 0;
    const int64_t cap = max_items_ + max_chunks(max_sys_, max_items_);
    for (int k = 0; k < na; ++k) {
        const int s = (int)act[k];
        if (sys_[s].nchunks <= 1) continue;
        for (int c = 0; c < sys_[s].nchunks; ++c) {
            if (ni + nc >= cap) return PCG_ERR_BUDGET;
            items[2 * (ni + nc)] = (uint32_t)s;
            items[2 * (ni + nc) + 1] = (uint32_t)c;
            ++nc;
        }
    }
    cnt[0] = (int32_t)ni;
    cnt[1] = na;
    cnt[2] = (int32_t)nc;
    // descriptors and states only when a slot was admitted or released:
    // between launches the host copy of a running system's state equals the
    // device one (it was just read back), and admitted or released slots
    // carry their new state
    if (slots_dirty_) {
        BCHK(hipMemcpyAsync(d_sys_, sys_.data(), sizeof(BatchSys) * max_sys_, hipMemcpyHostToDevice, stream_));
        BCHK(hipMemcpyAsync(d_st_, h_st_, sizeof(BatchState) * max_sys_, hipMemcpyHostToDevice, stream_));
        slots_dirty_ = false;
    }
    // the work list in one copy; stream order puts it before the next
    // launch, and the staging buffer is next written after the read-back
    // that follows that launch has been waited for
    BCHK(hipMemcpyAsync(d_list_, h_list_, list_items_off(max_sys_) + 8 * (size_t)(ni + nc), hipMemcpyHostToDevice,
                        stream_));
    BCHK(hipEventRecord(ev_up_, stream_));
    tables_dirty_ = false;
    items_ = ni;
    active_ = na;
    chunks_ = nc;
    max_sys_items_ = most;
    return PCG_OK;
}

template <typename T, bool HEAD>
static int step_occupancy(int spec)
{
    int nb = 0;
    hipError_t e = hipSuccess;
    switch (spec) {
    case 0: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_batch_step<T, HEAD, 0>, kBatchBlock, 0); break;
    case 1: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_batch_step<T, HEAD, 1>, kBatchBlock, 0); break;
    case 2: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_batch_step<T, HEAD, 2>, kBatchBlock, 0); break;
    case 3: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_batch_step<T, HEAD, 3>, kBatchBlock, 0); break;
    case 4: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_batch_step<T, HEAD, 4>, kBatchBlock, 0); break;
    case 5: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_batch_step<T, HEAD, 5>, kBatchBlock, 0); break;
    default:
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_batch_step<T, HEAD, kSpecAny>, kBatchBlock, 0);
        break;
    }
    return e == hipSuccess ? nb : 0;
}

// Blocks of the persistent pass when the caller gave none: as many as the
// mode's pass kernel keeps resident (at most four per CU), so that every
// block starts at once and the items are shared out evenly.  The kernel
// without the head needs fewer registers, so the split modes can run more
// blocks than the fused one.
int BatchEngine::default_pass_grid(int split) const
{
    const int a = split ? (prec_ == PCG_FP64 ? step_occupancy<double, false>(spec_) : step_occupancy<float, false>(spec_))
                        : (prec_ == PCG_FP64 ? step_occupancy<double, true>(spec_) : step_occupancy<float, true>(spec_));
    const int per_cu = std::min(4, std::max(1, a));
    return per_cu * kNumCU;
}

void BatchEngine::enqueue_passes(hipStream_t st, int split)
{
    BatchTables tb{d_sys_,
                   d_st_,
                   reinterpret_cast<const int32_t *>(d_list_),
                   reinterpret_cast<const uint32_t *>(d_list_ + 16),
                   reinterpret_cast<const uint2 *>(d_list_ + list_items_off(max_sys_)),
                   max_sys_,
                   0};
    const dim3 pg(pass_grid_ > 0 ? pass_grid_ : default_pass_grid(split)), bk(kBatchBlock);
    for (int k = 0; k < K_; ++k) {
        const int par = k & 1;
        if (split) {
            if (split == 2) hipLaunchKernelGGL(k_batch_trans_chunked, dim3(chunk_grid_), bk, 0, st, tb, par);
            else hipLaunchKernelGGL(k_batch_trans, dim3(trans_grid_), bk, 0, st, tb, par);
            if (prec_ == PCG_FP64) launch_step<double, false>(spec_, pg, bk, st, tb, par);
            else launch_step<float, false>(spec_, pg, bk, st, tb, par);
        } else {
            if (prec_ == PCG_FP64) launch_step<double, true>(spec_, pg, bk, st, tb, par);
            else launch_step<float, true>(spec_, pg, bk, st, tb, par);
        }
    }
}

pcg_status BatchEngine::ensure_graph(int split)
{
    if (gexec_[split]) return PCG_OK;
    hipStream_t cs;
    BCHK(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
    hipError_t e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) {
        (void)hipStreamDestroy(cs);
        return hip_fail(e, "hipStreamBeginCapture");
    }
    enqueue_passes(cs, split);
    e = hipStreamEndCapture(cs, &graph_[split]);
    (void)hipStreamDestroy(cs);
    if (e != hipSuccess) return hip_fail(e, "hipStreamEndCapture");
    BCHK(hipGraphInstantiate(&gexec_[split], graph_[split], nullptr, nullptr, 0));
    return PCG_OK;
}

pcg_status BatchEngine::step(double *gpu_ms)
{
    pcg_status st;
    if (tables_dirty_ && (st = upload_tables())) return st;
    if (active_ == 0) return PCG_OK;
    // split when the batch is large, or when one system is: in a fused pass
    // each of a system's items sums all of that system's partials; with
    // chunked systems the chunk pass runs first
    const int split = chunks_ > 0 ? 2 : (items_ > split_items_ || max_sys_items_ > fused_sys_items_) ? 1 : 0;
    if ((st = ensure_graph(split))) return st;
    BCHK(hipEventRecord(ev0_, stream_));
    BCHK(hipGraphLaunch(gexec_[split], stream_));
    BCHK(hipEventRecord(ev1_, stream_));
    BCHK(hipMemcpyAsync(h_st_, d_st_, sizeof(BatchState) * max_sys_, hipMemcpyDeviceToHost, stream_));
    BCHK(hipStreamSynchronize(stream_));
    float ms = 0.f;
    BCHK(hipEventElapsedTime(&ms, ev0_, ev1_));
    if (gpu_ms) *gpu_ms += ms;
    ++launches_;
    // drop finished systems from the tables before the next launch
    for (int s = 0; s < max_sys_; ++s)
        if (listed_[s] && h_st_[s].phase >= PH_DONE) tables_dirty_ = true;
    return PCG_OK;
}

void BatchEngine::result(int slot, pcg_result *r) const
{
    const BatchState &S = h_st_[slot];
    std::memset(r, 0, sizeof(*r));
    const double bn = std::sqrt(S.bnorm2);
    r->status = S.status == RUNNING ? PCG_MAX_ITER : S.status;
    r->iterations = S.iter;
    r->replacements = S.restarts;
    r->launches = launches_;
    r->rel_res_recursive = bn > 0 ? std::sqrt(S.rho) / bn : std::sqrt(S.rho);
    r->rel_res_true = bn > 0 ? std::sqrt(S.true_res2) / bn : std::sqrt(S.true_res2);
    r->iter_passes = S.passes;
    r->sigma = sys_[slot].sigma;
}

pcg_status BatchEngine::copy_history(int slot, double *host, int cap)
{
    const BatchSys &D = sys_[slot];
    if (!D.hist || !host || cap <= 0) return PCG_OK;
    BCHK(hipMemcpyAsync(host, D.hist, (size_t)std::min(cap, D.hist_cap) * PCG_HISTORY_FIELDS * 8,
                        hipMemcpyDeviceToHost, stream_));
    BCHK(hipStreamSynchronize(stream_));
    return PCG_OK;
}

}  // namespace pcg

using namespace pcg;

// ------------------------------------------------------------------ C ABI

static pcg_status batch_plan(int32_t count, const pcg_operator *ops, const pcg_options *opts, size_t *tables,
                             std::vector<size_t> *offsets, size_t *total, int64_t *items)
{
    if (count < 1) return invalid("count must be >= 1");
    if (!ops || !opts) return invalid("ops and opts must be non-null");
    size_t off = 0;
    int64_t ni = 0;
    std::vector<size_t> sys_off(count);
    for (int k = 0; k < count; ++k) {
        pcg_status st = validate_options(&opts[k]);
        if (st) return st;
        if ((st = validate_operator(&ops[k], opts[0].prec))) return st;
        if (opts[k].prec != opts[0].prec) return invalid("every system of a batch must use the same precision");
        if (opts[k].method == PCG_CG || opts[k].method == PCG_PIPE_VAR_SHIFT || opts[k].method == PCG_PIPE_RR)
            return invalid("the batched pass runs the constant-shift pipelined methods");
        if (opts[k].flags) return invalid("the batched pass takes no option flags");
        BatchEngine::SysLayout L;
        BatchEngine::system_layout(&ops[k], &opts[k], &L);
        sys_off[k] = off;
        off += L.bytes;
        ni += L.nwork;
    }
    const size_t tb = (BatchEngine::table_bytes(count, ni) + 255) & ~size_t(255);
    for (auto &o : sys_off) o += tb;
    *tables = tb;
    *total = tb + off;
    *items = ni;
    if (offsets) *offsets = sys_off;
    return PCG_OK;
}

extern "C" pcg_status pcg_batch_workspace_size(int32_t count, const pcg_operator *ops, const pcg_options *opts,
                                               size_t *bytes)
{
    if (!bytes) return invalid("bytes is null");
    size_t tables, total;
    int64_t items;
    pcg_status st = batch_plan(count, ops, opts, &tables, nullptr, &total, &items);
    if (st) return st;
    *bytes = total;
    return PCG_OK;
}

extern "C" pcg_status pcg_batch_solve(int32_t count, const pcg_operator *ops, const pcg_options *opts,
                                      const double *const *b, double *const *x, pcg_result *results, void *workspace,
                                      size_t bytes, void *hip_stream)
{
    const auto t0 = std::chrono::steady_clock::now();
    if (!b || !x || !results) return invalid("b, x and results must be non-null");
    if (!workspace || ((uintptr_t)workspace % 256)) return invalid("workspace must be non-null and 256-byte aligned");
    size_t tables, total;
    int64_t items;
    std::vector<size_t> offs;
    pcg_status st = batch_plan(count, ops, opts, &tables, &offs, &total, &items);
    if (st) return st;
    if (bytes < total) return invalid("workspace too small");
    char *ws = (char *)workspace;
    BatchEngine eng;
    const int K = opts[0].iters_per_launch;  // 0: the engine default
    if ((st = eng.init(ws, count, items, opts[0].prec, (hipStream_t)hip_stream, K))) return st;
    if (opts[0].grid_blocks) eng.set_pass_grid(opts[0].grid_blocks);
    int spec = ops[0].kind * 2 + (opts[0].pc == PCG_PC_JACOBI);
    for (int k = 1; k < count; ++k)
        if (ops[k].kind * 2 + (opts[k].pc == PCG_PC_JACOBI) != spec) spec = kSpecAny;
    eng.set_spec(spec);
    std::vector<int> slot(count);
    for (int k = 0; k < count; ++k)
        if ((st = eng.admit(&ops[k], &opts[k], b[k], x[k], ws + offs[k], &slot[k]))) return st;
    double gpu_ms = 0.0;
    for (;;) {
        if ((st = eng.step(&gpu_ms))) return st;
        bool all = true;
        for (int k = 0; k < count; ++k)
            if (!eng.done(slot[k])) {
                all = false;
                break;
            }
        if (all) break;
    }
    const double secs = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    for (int k = 0; k < count; ++k) {
        eng.result(slot[k], &results[k]);
        results[k].seconds = secs;
        results[k].iter_kernel_ms = gpu_ms;
        if (opts[k].history_cap > 0 && (st = eng.copy_history(slot[k], opts[k].history, opts[k].history_cap)))
            return st;
    }
    return PCG_OK;
}
