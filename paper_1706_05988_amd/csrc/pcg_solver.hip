// pcg_solver.hip -- host side of the single-system C ABI (pcg.h): argument
// validation, workspace layout, kernel dispatch, HIP-graph capture of K
// iteration passes, and the solve loop (init passes, graph launches with the
// device status polled one launch behind, explicit residual, restarts).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstddef>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <type_traits>
#include <vector>

#include "pcg.h"
#include "pcg_internal.h"
#include "pcg_kernels.h"

using namespace pcg;

// ----------------------------------------------------------------- errors

namespace pcg {
thread_local std::string g_last_error;

pcg_status hip_fail(hipError_t e, const char *what)
{
    g_last_error = std::string(what) + ": " + hipGetErrorString(e);
    return PCG_ERR_HIP;
}

pcg_status invalid(const char *why)
{
    g_last_error = std::string("invalid argument: ") + why;
    return PCG_ERR_INVALID;
}
}  // namespace pcg

#define HIPCHK(call)                                      \
    do {                                                  \
        hipError_t e_ = (call);                           \
        if (e_ != hipSuccess) return hip_fail(e_, #call); \
    } while (0)

extern "C" const char *pcg_last_error(void) { return g_last_error.c_str(); }

extern "C" const char *pcg_status_str(pcg_status s)
{
    switch (s) {
    case PCG_OK: return "ok";
    case PCG_PENDING: return "pending";
    case PCG_ERR_INVALID: return "invalid argument";
    case PCG_ERR_NONFINITE: return "right-hand side is not finite";
    case PCG_ERR_HIP: return "HIP runtime error";
    case PCG_ERR_BUDGET: return "request can never fit the memory budget";
    case PCG_ERR_STATE: return "unknown handle or wrong state";
    default: return "unknown status";
    }
}

extern "C" pcg_status pcg_default_options(pcg_options *o)
{
    if (!o) return invalid("options is null");
    std::memset(o, 0, sizeof(*o));
    o->method = PCG_PIPE_SHIFT;
    o->pc = PCG_PC_NONE;
    o->prec = PCG_FP64;
    o->max_iter = 1000;
    o->sigma = std::nan("");
    o->rtol = 1e-10;
    o->true_residual_check = 1;
    o->replace_max = 4;
    o->iters_per_launch = 0;
    o->use_graph = 1;
    return PCG_OK;
}

// ------------------------------------------------------------ validation

namespace pcg {

static bool aligned(const void *p, size_t a) { return ((uintptr_t)p % a) == 0; }

pcg_status validate_operator(const pcg_operator *op, int prec)
{
    if (!op) return invalid("operator is null");
    if (op->kind < PCG_OP_STENCIL2D5 || op->kind > PCG_OP_CSR) return invalid("unknown operator kind");
    if (op->n < 1 || op->n >= (int64_t(1) << 31)) return invalid("n must be in [1, 2^31)");
    if (op->kind == PCG_OP_CSR) {
        if (!op->row_ptr || !op->col_idx || !op->vals) return invalid("CSR arrays must be non-null");
        if (op->nnz < 0 || op->nnz >= (int64_t(1) << 31)) return invalid("nnz must be in [0, 2^31)");
        if (!aligned(op->row_ptr, 4) || !aligned(op->col_idx, 4)) return invalid("CSR index arrays misaligned");
        if (!aligned(op->vals, prec == PCG_FP64 ? 8 : 4)) return invalid("CSR values misaligned");
    } else {
        if (op->nx < 1 || op->ny < 1 || op->nz < 1) return invalid("grid extents must be >= 1");
        if (op->kind == PCG_OP_STENCIL2D5 && op->nz != 1) return invalid("2-D stencil needs nz = 1");
        const int64_t cells = int64_t(op->nx) * op->ny * op->nz;
        if (cells != op->n) return invalid("n does not match the grid");
        if (!std::isfinite(op->diag) || !std::isfinite(op->offdiag) || !std::isfinite(op->shift))
            return invalid("stencil coefficients must be finite");
        if (!(op->diag + op->shift > 0.0)) return invalid("stencil diagonal must be positive");
    }
    return PCG_OK;
}

pcg_status validate_options(const pcg_options *o)
{
    if (!o) return invalid("options is null");
    if (o->method < PCG_CG || o->method > PCG_PIPE_RR) return invalid("unknown method");
    if (o->method == PCG_PIPE_RR && (o->rr_period < 0 || o->rr_period > (1 << 20)))
        return invalid("rr_period must be in [0, 2^20] (0: default)");
    if (o->method == PCG_PIPE_VAR_SHIFT) {
        if (!o->sigma_schedule || o->sigma_schedule_len < 1 || o->sigma_schedule_len > (1 << 24))
            return invalid("PCG_PIPE_VAR_SHIFT needs sigma_schedule with 1 .. 2^24 entries");
        for (int k = 0; k < o->sigma_schedule_len; ++k)
            if (!(o->sigma_schedule[k] >= 0.0 && std::isfinite(o->sigma_schedule[k])))
                return invalid("every sigma_schedule entry must be finite and >= 0");
    }
    if (o->pc < PCG_PC_NONE || o->pc > PCG_PC_JACOBI) return invalid("unknown preconditioner");
    if (o->prec < PCG_FP64 || o->prec > PCG_FP32_STREAM) return invalid("unknown precision");
    if (o->max_iter < 0) return invalid("max_iter must be >= 0");
    if (!(o->rtol > 0.0) || !std::isfinite(o->rtol)) return invalid("rtol must be finite and > 0");
    if (!std::isnan(o->sigma) && !(o->sigma >= 0.0 && std::isfinite(o->sigma)))
        return invalid("sigma must be >= 0 (or NaN for the default)");
    if (o->iters_per_launch < 0 || (o->iters_per_launch % 2) != 0)
        return invalid("iters_per_launch must be 0 or an even number >= 2");
    if (o->block_size != 0 && (o->block_size < 64 || o->block_size > kMaxBlock || o->block_size % 64 != 0))
        return invalid("block_size must be a multiple of 64 in [64, 256]");
    if (o->grid_blocks < 0 || o->grid_blocks > kMaxGrid) return invalid("grid_blocks out of range");
    if (o->history_cap < 0) return invalid("history_cap must be >= 0");
    if (o->history_cap > 0 && !o->history) return invalid("history buffer is null");
    if (o->replace_max < 0) return invalid("replace_max must be >= 0");
    if (o->flags & ~PCG_FLAG_RUN_THROUGH_BREAKDOWN) return invalid("unknown option flags");
    return PCG_OK;
}

// ----------------------------------------------------------------- shape

// Launch shape.  Without PCG_VAR_SET the measured defaults for MI355X
// (256-cube sweeps of every method / precision) apply: the fused pipelined
// pass with Jacobi streams 18 vectors and runs best as ONE block per CU with
// several unknowns per thread (a compact window of tiles in flight keeps HBM
// pages open), the lighter passes as more, smaller blocks; the XCD slab map
// measured slower everywhere and is off unless asked for.
constexpr int kZmBlocksPerCU = 3;  // z-marching CG pass A: 48 KB of LDS per block

LaunchShape choose_shape(const pcg_operator *op, const pcg_options *o)
{
    LaunchShape s{};
    const int var = o->variant;
    const bool set = var & PCG_VAR_SET;
    int blocks_per_cu;
    if (set) {
        s.ept = (var & PCG_VAR_EPT1) ? 1 : (var & PCG_VAR_EPT4) ? 4 : 2;
        s.nt = (var & PCG_VAR_NT) ? 1 : 0;
        s.block = 256;
        blocks_per_cu = kDefaultBlocksPerCU;
    } else {
        s.nt = 1;
        const bool pipe = o->method != PCG_CG, jac = o->pc == PCG_PC_JACOBI, fp64 = o->prec == PCG_FP64;
        if (pipe && op->kind == PCG_OP_CSR) {
            // gathers need more waves in flight than the stencil streams:
            // four blocks of 256 per CU on the sliced-ELL copy (measured on
            // the anisotropic 1024^2 / 2048^2 operators: binary64 44.4 /
            // 172.7 us per pass against 47.3 / 185.9 for 128-thread blocks on
            // CSR rows); the FP32-stream form takes 4 rows per thread while
            // that leaves about one tile per block (28.5 against 30.4 us at
            // 1024^2), 2 beyond (88.9 against 91.6 us at 2048^2)
            if (fp64) s.ept = 1, s.block = 256, blocks_per_cu = 4;
            else s.ept = op->n <= int64_t(kNumCU) * 4 * 256 * 4 ? 4 : 2, s.block = 256, blocks_per_cu = 4;
        } else if (pipe && jac) {
            // 4 unknowns per thread keep ~70 independent loads in flight per
            // thread; binary64 runs best as one block per CU, the lighter
            // binary32 streams with four
            s.ept = 4, s.block = 256, blocks_per_cu = fp64 ? 1 : 4;
        } else if (pipe) {
            // without a preconditioner (measured: FP32-stream 256^3 153.5
            // against 224.4 us with 1 unknown per thread in 128-thread
            // blocks, 3300^2 101.5 against 144.0; binary64 256^3 273.6 against
            // 291.1, 3300^2 174.9 against 184.8; binary64 1000^2 keeps the
            // lighter shape, 24.8 against 25.8 us)
            if (!fp64) s.ept = 4, s.block = 256, blocks_per_cu = op->n <= (int64_t(1) << 21) ? 2 : 4;
            else if (op->n >= (int64_t(1) << 22)) s.ept = 4, s.block = 256, blocks_per_cu = 4;
            else s.ept = 1, s.block = 128, blocks_per_cu = 4;
        } else if (fp64) {
            s.ept = 1, s.block = 128, blocks_per_cu = 4;
        } else {
            s.ept = 4, s.block = 256, blocks_per_cu = 4;
        }
    }
    // sliced-ELL CSR copy: built in for both forms, in place or sorted,
    // whichever is smaller (where its padding fits)
    s.sell = set ? ((var & PCG_VAR_CSR_SELL) ? 1 : 0) | ((var & PCG_VAR_CSR_SELL_SORTED) ? 2 : 0) : 3;
    if (o->block_size) s.block = o->block_size;
    auto tiles_grid = [&](int block, int ept, int per_cu, int *ntiles, int *grid) {
        const int64_t tile = int64_t(block) * ept;
        *ntiles = (int)((op->n + tile - 1) / tile);
        int g = o->grid_blocks ? o->grid_blocks : per_cu * kNumCU;
        if (g > *ntiles) g = *ntiles;
        if (g >= 64) g &= ~7;  // a multiple of the XCD count
        if (g < 1) g = 1;
        *grid = g;
    };
    tiles_grid(s.block, s.ept, blocks_per_cu, &s.ntiles, &s.grid);
    // the sorted copy sorts within a wave's rows of a tile, so it takes 4
    // rows per thread unless the shape is given (measured with the column
    // windows and 16-bit window offsets on banded random operators of 1e6,
    // 2e6, 4e6 and 1e7 rows of 4 to 40 entries, us per pass): binary64 four
    // blocks of 128 per CU (binary64 values at 1e6 / 4e6: 67.7 / 249.7, two
    // of 256: 67.3 / 261.1, six of 128: 75.6 / 285.1), and six beyond 1.5e6
    // rows when the values are stored as binary32 (four: 61.0 / 105.6 /
    // 218.9 / 512.0, six: 65.4 / 97.3 / 197.8 / 475.6, eight: 117.6 at 2e6);
    // FP32-stream blocks of 256, two per CU up to 1.5e6 rows (48.5 against
    // 49.8 for three at 1e6), three beyond (72.4 / 154.3 / 369.5 against
    // 83.0 / 185.4 / 437.0 for two, 89.3 at 2e6 for four)
    s.sort_block = s.block, s.sort_ept = s.ept, s.sort_ntiles = s.ntiles, s.sort_grid = s.grid;
    s.sort_grid_v32 = s.grid;
    if (!set && op->kind == PCG_OP_CSR) {
        const bool fp64 = o->prec == PCG_FP64, large = op->n > 1500000;
        s.sort_block = o->block_size ? o->block_size : fp64 ? 128 : 256;
        s.sort_ept = 4;
        const int per_cu = fp64 ? 4 : large ? 3 : 2;
        tiles_grid(s.sort_block, s.sort_ept, per_cu, &s.sort_ntiles, &s.sort_grid);
        s.sort_grid_v32 = s.sort_grid;
        if (fp64 && large) tiles_grid(s.sort_block, s.sort_ept, 6, &s.sort_ntiles, &s.sort_grid_v32);
    }
    const bool want_xcd = set && (var & PCG_VAR_XCD_MAP) != 0;
    s.xcd_map = (want_xcd && s.grid >= 64 && (s.grid % 8) == 0) ? 1 : 0;
    s.K = o->iters_per_launch ? o->iters_per_launch : (op->n >= (1 << 20) ? 16 : 64);
    // classic CG on a 3-D grid: pass A marches along z with the p_i planes in
    // LDS when its window fits (4 planes of rows + 2 grid rows in 48 KB, and
    // one plane window in kZmBatch points per thread) and the grid is large
    // enough (or the variant asks for it); segments of at least 8 planes keep
    // the refill of the first two planes of a segment small
    s.zm_rows = 0;
    if (o->method == PCG_CG && op->kind == PCG_OP_STENCIL3D7) {
        const size_t budget = 48 * 1024;
        const int zblock = o->block_size ? o->block_size : 256;  // its block size wherever it runs
        int rows = (int)(budget / (4 * sizeof(double) * (size_t)op->nx)) - 2;
        rows = std::min(rows, (int)((int64_t)kZmBatch * zblock / op->nx) - 2);
        rows = std::min(std::min(rows, 8), (int)op->ny);
        if (rows >= 1) {
            const int nchunks = (op->ny + rows - 1) / rows;
            auto split = [&](int grid, int *seg, int *nsegs) {
                const int want = (grid + nchunks - 1) / nchunks;
                *seg = std::max(std::min(op->nz, 8), (op->nz + want - 1) / want);
                *nsegs = (op->nz + *seg - 1) / *seg;
            };
            const bool forced = set && (var & PCG_VAR_CG_ZMARCH) != 0;
            int seg, nsegs;
            split(kZmBlocksPerCU * kNumCU, &seg, &nsegs);
            // built in where it measured faster: at least 4 rows per item (the
            // two halo rows are formed again by the neighbouring items: 320^3
            // with 2 rows was slower, 693 vs 620 us per iteration) and at
            // least 1.5 items per CU (160^3 with 460 items: 82.7 vs 88.6 us;
            // 128^3 with 256 items: 56.6 vs 53.1 us)
            const bool pays = rows >= 4 && 2 * nchunks * nsegs >= 3 * kNumCU;
            if (!set && pays) {
                // the built-in shape of this case: 256 threads, as many
                // blocks as the 48 KB plane window lets reside (3 per CU)
                if (!o->block_size) s.block = 256;
                s.ntiles = (int)((op->n + int64_t(s.block) * s.ept - 1) / (int64_t(s.block) * s.ept));
                int g = o->grid_blocks ? o->grid_blocks : kZmBlocksPerCU * kNumCU;
                if (g > s.ntiles) g = s.ntiles;
                if (g >= 64) g &= ~7;
                s.grid = std::max(g, 1);
            }
            split(s.grid, &seg, &nsegs);
            if (forced || (!set && pays))
                s.zm_rows = rows, s.zm_seg = seg, s.zm_nchunks = nchunks, s.zm_nsegs = nsegs;
        }
    }
    return s;
}

static size_t up256(size_t v) { return (v + 255) & ~size_t(255); }

size_t layout(const pcg_operator *op, const pcg_options *o, const LaunchShape &sh, Layout *L)
{
    const size_t n = (size_t)op->n;
    const uint32_t es = o->prec == PCG_FP64 ? 8 : 4;
    const bool jac = o->pc == PCG_PC_JACOBI;
    size_t off = 0;
    auto take = [&](size_t bytes) {
        size_t at = off;
        off += up256(bytes);
        return at;
    };
    Layout l{};
    l.state = take(2 * sizeof(DevState) + 128);
    // partials for the largest grid the passes may take (a sorted
    // sliced-ELL copy brings its own shape)
    const size_t parts = size_t(std::max({sh.grid, sh.sort_grid, sh.sort_grid_v32})) * kFields * 8;
    l.part[0] = take(parts);
    l.part[1] = take(parts);
    l.gersh = take(size_t(kGershBlocks) * 2 * 8);
    l.flag = take(64);
    l.hist = take(size_t(o->history_cap) * PCG_HISTORY_FIELDS * 8);
    l.dinv = (op->kind == PCG_OP_CSR && jac) ? take(n * es) : SIZE_MAX;
    l.sched = o->method == PCG_PIPE_VAR_SHIFT ? take(size_t(o->sigma_schedule_len) * 8) : SIZE_MAX;
    // the passes read a CSR operator in sliced-ELL form when its padding
    // stays within a quarter of nnz (decided at set-up)
    l.sell_ptr = l.sell_col = l.sell_val = l.sort_ptr = l.sort_perm = l.sort_win = SIZE_MAX;
    l.sell_cap = 0;
    l.nslices = l.sort_nslices = 0;
    if (op->kind == PCG_OP_CSR && sh.sell) {
        const int64_t cap = op->nnz + op->nnz / 4 + 4096;
        const int64_t slots = int64_t(sh.sort_ntiles) * sh.sort_block * sh.sort_ept;
        if (cap < (int64_t(1) << 31) - 64) {
            l.sell_cap = cap;
            if (sh.sell & 1) {
                l.nslices = (int32_t)((n + 63) / 64);
                l.sell_ptr = take(size_t(l.nslices + 1) * 4);
            }
            if ((sh.sell & 2) && slots < (int64_t(1) << 31) - 1) {
                l.sort_nslices = (int32_t)(slots / 64);
                l.sort_ptr = take(size_t(l.sort_nslices + 1) * 4);
                l.sort_perm = take(size_t(slots) * 4);
                l.sort_win = take(size_t(sh.sort_ntiles) * 8);
            }
            if (l.sell_ptr != SIZE_MAX || l.sort_ptr != SIZE_MAX) {
                l.sell_col = take(size_t(cap) * 4);
                l.sell_val = take(size_t(cap) * es);
            }
        }
    }
    // slots of a 512-unknown tile: x (binary64) first, then the stored vectors
    for (int k = 0; k < V_COUNT; ++k) l.slot_off[k] = kNoSlot;
    uint32_t tb = 0;
    auto slot = [&](int k, uint32_t bytes_per) {
        l.slot_off[k] = tb;
        tb += kBlk * bytes_per;
    };
    slot(V_X, 8);
    slot(V_R, es);
    slot(V_W0, es);  // CG: p ping-pong
    slot(V_W1, es);
    slot(V_S, es);
    if (o->method != PCG_CG) {
        slot(V_Z, es);
        slot(V_T, es);
        if (jac) {
            slot(V_U, es);
            slot(V_Q, es);
            slot(V_P, es);
        }
    }
    l.tile_bytes = tb;
    l.blk = take(((n + kBlk - 1) / kBlk) * (size_t)tb);
    l.total = off;
    if (L) *L = l;
    return off;
}

}  // namespace pcg

// ------------------------------------------------------------- dispatch

static_assert(sizeof(PassArgs<double>) <= sizeof(PassArgsAny), "PassArgsAny too small");
static_assert(sizeof(PassArgs<float>) <= sizeof(PassArgsAny), "PassArgsAny too small");

namespace {

using LaunchFn = void (*)(PassArgsAny, int, int, hipStream_t);

// Kernel table for one (T, OP, JAC, EPT, NT) combination.
struct Kernels {
    LaunchFn copy_x, init0_pipe, init0_cg, init1, pipe, pipe_var, pipe_rr, cg_init1, cg_a, cg_b, resid;
    void (*x_fixup)(PassArgsAny, double, int, int, hipStream_t);
};

template <typename T, int OP, bool JAC, int EPT, bool NT>
struct KernelSet {
    static PassArgs<T> &A(PassArgsAny &a) { return *reinterpret_cast<PassArgs<T> *>(a.bytes); }
    static void copy_x(PassArgsAny a, int g, int b, hipStream_t s)
    { hipLaunchKernelGGL((k_copy_x<T, EPT>), dim3(g), dim3(b), 0, s, A(a)); }
    // Launches `launch` with the CSR operand form of the pass as a constant:
    // 2 the sorted sliced-ELL copy, 1 the in-place copy, 0 the rows (and
    // every operator that is not CSR).
    template <typename L>
    static void by_form(PassArgsAny &a, L launch)
    {
        if constexpr (OP == OP_CSR) {
            if (A(a).sell_perm) return launch(std::integral_constant<int, 2>{});
            if (A(a).sell_ptr) return launch(std::integral_constant<int, 1>{});
        }
        launch(std::integral_constant<int, 0>{});
    }
    static void init0_pipe(PassArgsAny a, int g, int b, hipStream_t s)
    {
        by_form(a, [&](auto f) {
            hipLaunchKernelGGL((k_init0<T, OP, JAC, JAC, EPT, NT, decltype(f)::value>), dim3(g), dim3(b), 0, s, A(a));
        });
    }
    static void init0_cg(PassArgsAny a, int g, int b, hipStream_t s)
    {
        by_form(a, [&](auto f) {
            hipLaunchKernelGGL((k_init0<T, OP, JAC, false, EPT, NT, decltype(f)::value>), dim3(g), dim3(b), 0, s, A(a));
        });
    }
    static void init1(PassArgsAny a, int g, int b, hipStream_t s)
    {
        by_form(a, [&](auto f) {
            hipLaunchKernelGGL((k_init1<T, OP, JAC, EPT, NT, decltype(f)::value>), dim3(g), dim3(b), 0, s, A(a));
        });
    }
    static void pipe(PassArgsAny a, int g, int b, hipStream_t s)
    {
        by_form(a, [&](auto f) {
            hipLaunchKernelGGL((k_pipe<T, OP, JAC, EPT, NT, false, decltype(f)::value>), dim3(g), dim3(b), 0, s, A(a));
        });
    }
    static void pipe_var(PassArgsAny a, int g, int b, hipStream_t s)
    {
        by_form(a, [&](auto f) {
            hipLaunchKernelGGL((k_pipe<T, OP, JAC, EPT, NT, true, decltype(f)::value>), dim3(g), dim3(b), 0, s, A(a));
        });
    }
    static void pipe_rr(PassArgsAny a, int g, int b, hipStream_t s)
    {
        by_form(a, [&](auto f) {
            hipLaunchKernelGGL((k_pipe_rr<T, OP, JAC, EPT, NT, decltype(f)::value>), dim3(g), dim3(b), 0, s, A(a));
        });
    }
    static void cg_init1(PassArgsAny a, int g, int b, hipStream_t s)
    { hipLaunchKernelGGL((k_cg_init1<T, OP, JAC, EPT, NT>), dim3(g), dim3(b), 0, s, A(a)); }
    static void cg_a(PassArgsAny a, int g, int b, hipStream_t s)
    {
        if constexpr (OP == OP_3D7) {
            const PassArgs<T> &p = A(a);
            if (p.zm.rows > 0) {
                const size_t lds = 4 * sizeof(double) * (size_t)(p.zm.rows + 2) * (size_t)p.A.nx;
                hipLaunchKernelGGL((k_cg_a_zm<T, JAC, NT>), dim3(g), dim3(b), lds, s, p, p.zm);
                return;
            }
        }
        by_form(a, [&](auto f) {
            hipLaunchKernelGGL((k_cg_a<T, OP, JAC, EPT, NT, decltype(f)::value>), dim3(g), dim3(b), 0, s, A(a));
        });
    }
    static void cg_b(PassArgsAny a, int g, int b, hipStream_t s)
    { hipLaunchKernelGGL((k_cg_b<T, OP, JAC, EPT, NT>), dim3(g), dim3(b), 0, s, A(a)); }
    static void resid(PassArgsAny a, int g, int b, hipStream_t s)
    {
        by_form(a, [&](auto f) {
            hipLaunchKernelGGL((k_resid<T, OP, EPT, decltype(f)::value>), dim3(g), dim3(b), 0, s, A(a));
        });
    }
    static void x_fixup(PassArgsAny a, double alpha, int g, int b, hipStream_t s)
    { hipLaunchKernelGGL((k_x_fixup<T, JAC, EPT>), dim3(g), dim3(b), 0, s, A(a), alpha); }
    static Kernels table()
    { return Kernels{copy_x, init0_pipe, init0_cg, init1, pipe, pipe_var, pipe_rr, cg_init1, cg_a, cg_b, resid, x_fixup}; }
};

template <typename T, int OP, bool JAC, int EPT>
Kernels pick_nt(bool nt)
{
    return nt ? KernelSet<T, OP, JAC, EPT, true>::table() : KernelSet<T, OP, JAC, EPT, false>::table();
}

template <typename T, int OP, bool JAC>
Kernels pick_ept(int ept, bool nt)
{
    switch (ept) {
    case 1: return pick_nt<T, OP, JAC, 1>(nt);
    case 4: return pick_nt<T, OP, JAC, 4>(nt);
    default: return pick_nt<T, OP, JAC, 2>(nt);
    }
}

template <typename T, int OP>
Kernels pick_jac(bool jac, int ept, bool nt)
{
    return jac ? pick_ept<T, OP, true>(ept, nt) : pick_ept<T, OP, false>(ept, nt);
}

template <typename T>
Kernels pick_op(int op, bool jac, int ept, bool nt)
{
    switch (op) {
    case PCG_OP_STENCIL2D5: return pick_jac<T, OP_2D5>(jac, ept, nt);
    case PCG_OP_STENCIL3D7: return pick_jac<T, OP_3D7>(jac, ept, nt);
    default: return pick_jac<T, OP_CSR>(jac, ept, nt);
    }
}

Kernels pick(int prec, int op, bool jac, int ept, bool nt)
{
    return prec == PCG_FP64 ? pick_op<double>(op, jac, ept, nt) : pick_op<float>(op, jac, ept, nt);
}

}  // namespace

// --------------------------------------------------------------- solver

struct pcg_solver_ {
    pcg_operator op;
    pcg_options opt;
    hipStream_t stream;      // the caller's stream: all work goes here
    char *ws;
    size_t ws_bytes;
    Layout L;
    LaunchShape sh;
    Kernels kern;
    double sigma;            // shift in use (0 for CG / p-CG)
    std::vector<double> sched;  // variable shift: sigma_{-1}, sigma_0, ... (host copy)
    double dinv_s;           // stencil Jacobi scalar
    int sell = 0;            // the fused pass reads the CSR operator's sliced-ELL copy: 1 rows
                             // in place, 2 sorted (0: the CSR arrays)
    int64_t sell_entries = 0;  // entries of that copy, padding included
    int sell_col_bits = 0;     // its column words: 32, or 16 (window or row offsets)
    int sell_val_bits = 0;     // its values: 64, or 32 (binary64 values that are binary32 numbers)
    hipGraph_t graph = nullptr;
    hipGraphExec_t gexec = nullptr;
    const double *graph_b = nullptr;  // b baked into the captured graph
    DevState *pinned = nullptr;       // 2 host slots for polled status
    bool no_alloc = false;            // static-scratch solve: no pinned memory, events or graphs
    DevState host_state[2] = {};      // its status slots (pageable host memory)
    hipEvent_t ev_begin[2] = {nullptr, nullptr};
    hipEvent_t ev_end[2] = {nullptr, nullptr};
    hipEvent_t ev_copy[2] = {nullptr, nullptr};

    DevState *state(int k) { return reinterpret_cast<DevState *>(ws + L.state) + k; }
    double *part(int k) { return reinterpret_cast<double *>(ws + L.part[k]); }

    // Arguments of the pass at parity `par` (reads state / partial slot par,
    // writes 1 - par; w / p buffers by w_par, default par).
    PassArgsAny args(int par, const double *b, double *x_user, int i0 = 0, int w_par = -1);
    pcg_status run_init(const double *b, int i0);
    pcg_status run_copy_x(double *x_user, int out);
    pcg_status run_true_residual(const double *b, const double *x_plain, double *res2, double *b2 = nullptr);
    pcg_status launch_iterations(const double *b);
};

PassArgsAny pcg_solver_::args(int par, const double *b, double *x_user, int i0, int w_par)
{
    PassArgsAny any{};
    auto fill = [&](auto *tag) {
        using T = std::remove_pointer_t<decltype(tag)>;
        PassArgs<T> &a = *reinterpret_cast<PassArgs<T> *>(any.bytes);
        a.A = make_opdev<T>(&op);
        a.dinv = L.dinv == SIZE_MAX ? nullptr : reinterpret_cast<const T *>(ws + L.dinv);
        a.dinv_s = dinv_s;
        a.b = b;
        a.x_user = x_user;
        a.blk = ws + L.blk;
        a.tile_bytes = L.tile_bytes;
        const int wp = w_par < 0 ? par : w_par;
        a.off_x = L.slot_off[V_X];
        a.off_r = L.slot_off[V_R];
        a.off_u = L.slot_off[V_U];
        a.off_win = L.slot_off[wp ? V_W1 : V_W0];
        a.off_wout = L.slot_off[wp ? V_W0 : V_W1];
        a.off_z = L.slot_off[V_Z];
        a.off_q = L.slot_off[V_Q];
        a.off_s = L.slot_off[V_S];
        a.off_t = L.slot_off[V_T];
        a.off_p = L.slot_off[V_P];
        a.clear = 0;
        a.part_in = part(par);
        a.part_out = part(1 - par);
        a.nparts = sh.grid;
        a.ntiles = sh.ntiles;
        a.st_in = state(par);
        a.st_out = state(1 - par);
        a.hist = opt.history_cap > 0 ? reinterpret_cast<double *>(ws + L.hist) : nullptr;
        a.hist_cap = opt.history_cap;
        a.max_iter = opt.max_iter;
        a.sigma = sigma;
        a.rtol = opt.rtol;
        a.i0 = i0;
        a.xcd_map = sh.xcd_map;
        a.copy_out = 0;
        a.x_plain = 0;
        a.sched = L.sched == SIZE_MAX ? nullptr : reinterpret_cast<const double *>(ws + L.sched);
        a.sched_len = (int32_t)sched.size();
        a.rr_period = opt.rr_period > 0 ? opt.rr_period : 8;
        a.rr_tau = opt.rr_tau > 0.0 ? opt.rr_tau : std::cbrt(opt.prec == PCG_FP64 ? 0x1p-53 : 0x1p-24);
        a.rr_floor = opt.rr_floor > 0.0 ? opt.rr_floor : 100.0;
        a.zm = CgZm{sh.zm_rows, sh.zm_seg, sh.zm_nchunks, sh.zm_nsegs};
        a.sell_ptr = sell ? reinterpret_cast<const int32_t *>(ws + (sell == 2 ? L.sort_ptr : L.sell_ptr)) : nullptr;
        a.sell_col = sell ? reinterpret_cast<const int32_t *>(ws + L.sell_col) : nullptr;
        a.sell_val = sell ? reinterpret_cast<const T *>(ws + L.sell_val) : nullptr;
        a.sell_perm = sell == 2 ? reinterpret_cast<const int32_t *>(ws + L.sort_perm) : nullptr;
        a.sell_win = sell == 2 ? reinterpret_cast<const int2 *>(ws + L.sort_win) : nullptr;
        a.sell_c16 = sell && sell_col_bits == 16 ? reinterpret_cast<const uint16_t *>(ws + L.sell_col) : nullptr;
        a.sell_v32 = sell && opt.prec == PCG_FP64 && sell_val_bits == 32
                         ? reinterpret_cast<const float *>(ws + L.sell_val) : nullptr;
        a.run_through = (opt.flags & PCG_FLAG_RUN_THROUGH_BREAKDOWN) ? 1 : 0;
    };
    if (opt.prec == PCG_FP64) fill((double *)nullptr);
    else fill((float *)nullptr);
    return any;
}

// Members of PassArgs set after args(); every T-dependent member is a
// pointer, so PassArgs<double> and PassArgs<float> share this layout.
static_assert(offsetof(PassArgs<double>, clear) == offsetof(PassArgs<float>, clear), "PassArgs layout");
static_assert(offsetof(PassArgs<double>, copy_out) == offsetof(PassArgs<float>, copy_out), "PassArgs layout");
static_assert(offsetof(PassArgs<double>, x_plain) == offsetof(PassArgs<float>, x_plain), "PassArgs layout");
static_assert(offsetof(PassArgs<double>, sigma) == offsetof(PassArgs<float>, sigma), "PassArgs layout");
static PassArgs<double> &head(PassArgsAny &a) { return *reinterpret_cast<PassArgs<double> *>(a.bytes); }

// K iterations: pipelined = K passes, CG = 2K passes.  Pass k reads slot
// k % 2.  The w (pipelined) or p (CG) buffers flip once per iteration.
static void enqueue_iterations(pcg_solver_ *s, hipStream_t st, const double *b)
{
    const int K = s->sh.K;
    if (s->opt.method == PCG_CG) {
        for (int it = 0; it < K; ++it) {
            // pass A: state slot 0 -> 1, p[it%2] -> p[1-it%2]; pass B: slot 1 -> 0
            s->kern.cg_a(s->args(0, b, nullptr, 0, it & 1), s->sh.grid, s->sh.block, st);
            s->kern.cg_b(s->args(1, b, nullptr, 0, it & 1), s->sh.grid, s->sh.block, st);
        }
    } else {
        const LaunchFn pass = s->opt.method == PCG_PIPE_VAR_SHIFT ? s->kern.pipe_var
                              : s->opt.method == PCG_PIPE_RR      ? s->kern.pipe_rr
                                                                  : s->kern.pipe;
        for (int k = 0; k < K; ++k) pass(s->args(k & 1, b, nullptr), s->sh.grid, s->sh.block, st);
    }
}

pcg_status pcg_solver_::run_copy_x(double *x_user, int out)
{
    PassArgsAny a = args(0, nullptr, x_user);
    head(a).copy_out = out;
    kern.copy_x(a, sh.grid, sh.block, stream);
    HIPCHK(hipGetLastError());
    return PCG_OK;
}

pcg_status pcg_solver_::run_init(const double *b, int i0)
{
    // init0 writes partials to slot 1; init1 reads slot 1 and writes state 0,
    // partials 0 and (pipelined) w[0].
    if (opt.method == PCG_CG) {
        PassArgsAny a0 = args(0, b, nullptr, i0);
        head(a0).clear = CLR_WIN;  // the first pass A of a launch reads p_{-1} from p[0]
        kern.init0_cg(a0, sh.grid, sh.block, stream);
        kern.cg_init1(args(1, b, nullptr, i0), sh.grid, sh.block, stream);
    } else {
        PassArgsAny a0 = args(0, b, nullptr, i0);
        uint32_t clr = CLR_Z | CLR_S | CLR_T;
        if (opt.pc == PCG_PC_JACOBI) clr |= CLR_Q | CLR_P;
        head(a0).clear = clr;
        kern.init0_pipe(a0, sh.grid, sh.block, stream);
        PassArgsAny a1 = args(1, b, nullptr, i0, 1);  // w_par 1: w_out = w[0]
        if (opt.method == PCG_PIPE_VAR_SHIFT) {
            // w_{i0} := A u - sigma_{i0 - 1} r keeps the definition of w under a (re)start
            const size_t k = std::min(size_t(i0), sched.size() - 1);
            head(a1).sigma = sched[k];
        }
        kern.init1(a1, sh.grid, sh.block, stream);
    }
    HIPCHK(hipGetLastError());
    return PCG_OK;
}

// ||b - A x||^2 and ||b||^2 (binary64): partials into slot 1 (free between
// iteration launches), summed into the true_res2 / spare[0] fields of state 0.
// x_plain: the caller's x, or nullptr for the internal copy.
pcg_status pcg_solver_::run_true_residual(const double *b, const double *x_plain, double *res2, double *b2)
{
    PassArgsAny a = args(0, b, const_cast<double *>(x_plain));
    head(a).x_plain = x_plain != nullptr;
    kern.resid(a, sh.grid, sh.block, stream);
    hipLaunchKernelGGL(k_reduce_true, dim3(1), dim3(1024), 0, stream, part(1), sh.grid, state(0));
    HIPCHK(hipGetLastError());
    HIPCHK(hipMemcpyAsync(&pinned[0], state(0), sizeof(DevState), hipMemcpyDeviceToHost, stream));
    HIPCHK(hipStreamSynchronize(stream));
    *res2 = pinned[0].true_res2;
    if (b2) *b2 = pinned[0].spare[0];
    return PCG_OK;
}

// ------------------------------------------------------------- CSR set-up

namespace pcg {

pcg_status csr_setup(const pcg_operator *op, int prec, int jac, void *dinv, int *flag, hipStream_t stream)
{
    // validate the structure on the device before any pass reads it
    HIPCHK(hipMemsetAsync(flag, 0, sizeof(int), stream));
    if (prec == PCG_FP64)
        hipLaunchKernelGGL(k_csr_check<double>, dim3(kGershBlocks), dim3(256), 0, stream, make_opdev<double>(op), jac,
                           op->nnz, flag);
    else
        hipLaunchKernelGGL(k_csr_check<float>, dim3(kGershBlocks), dim3(256), 0, stream, make_opdev<float>(op), jac,
                           op->nnz, flag);
    int bad = 0;
    HIPCHK(hipMemcpyAsync(&bad, flag, sizeof(int), hipMemcpyDeviceToHost, stream));
    HIPCHK(hipStreamSynchronize(stream));
    if (bad) return invalid("CSR structure invalid (row_ptr, col_idx or missing diagonal)");
    if (jac) {
        const int g = (int)((op->n + 255) / 256);
        if (prec == PCG_FP64)
            hipLaunchKernelGGL(k_jacobi<double>, dim3(g), dim3(256), 0, stream, make_opdev<double>(op), (double *)dinv);
        else
            hipLaunchKernelGGL(k_jacobi<float>, dim3(g), dim3(256), 0, stream, make_opdev<float>(op), (float *)dinv);
    }
    HIPCHK(hipGetLastError());
    return PCG_OK;
}

// Sliced-ELL copies of a CSR operator (synchronous): the rows in place
// and / or sorted within each wave's rows, as reserved; the smaller of the
// two is kept (the sorted one only when at least 1/32 smaller, since it
// also routes the products through LDS).
pcg_status sell_build(const pcg_operator *op, int prec, const SellPlan &p, hipStream_t stream, int *form,
                      int64_t *entries, int *col_bits, int *val_bits)
{
    *form = 0;
    *entries = 0;
    *col_bits = 0;
    *val_bits = 0;
    if (!p.col || (!p.sell_ptr && !p.sort_ptr)) return PCG_OK;
    const int32_t n = (int32_t)op->n;
    int32_t total[2] = {-1, -1};
    int32_t *sp = p.sell_ptr, *tp = p.sort_ptr, *perm = p.sort_perm;
    if (sp) {
        const int g = (int)((op->n + 255) / 256);
        hipLaunchKernelGGL(k_sell_width, dim3(g), dim3(256), 0, stream, op->row_ptr, n, sp);
        hipLaunchKernelGGL(k_sell_scan, dim3(1), dim3(1024), 0, stream, sp, p.nslices, p.cap);
        HIPCHK(hipGetLastError());
        HIPCHK(hipMemcpyAsync(&total[0], sp + p.nslices, sizeof(int32_t), hipMemcpyDeviceToHost, stream));
    }
    if (tp) {
        const int32_t ngroups = p.sort_nslices / p.sort_ept;
        const int g = (ngroups + 3) / 4;
        if (p.sort_ept == 1)
            hipLaunchKernelGGL(k_sell_sort<1>, dim3(g), dim3(256), 0, stream, op->row_ptr, n, p.sort_block, ngroups, tp, perm);
        else if (p.sort_ept == 2)
            hipLaunchKernelGGL(k_sell_sort<2>, dim3(g), dim3(256), 0, stream, op->row_ptr, n, p.sort_block, ngroups, tp, perm);
        else
            hipLaunchKernelGGL(k_sell_sort<4>, dim3(g), dim3(256), 0, stream, op->row_ptr, n, p.sort_block, ngroups, tp, perm);
        hipLaunchKernelGGL(k_sell_scan, dim3(1), dim3(1024), 0, stream, tp, p.sort_nslices, p.cap);
        HIPCHK(hipGetLastError());
        HIPCHK(hipMemcpyAsync(&total[1], tp + p.sort_nslices, sizeof(int32_t), hipMemcpyDeviceToHost, stream));
    }
    HIPCHK(hipStreamSynchronize(stream));
    int f = total[0] >= 0 ? 1 : 0;
    if (total[1] >= 0 && (f == 0 || int64_t(total[1]) + total[1] / 32 < int64_t(total[0]))) f = 2;
    if (f == 0) return PCG_OK;
    // the sorted copy's tile windows; when every tile has one, the columns
    // are stored as 16-bit offsets in their tile's window (in the first half
    // of the column array)
    uint16_t *c16 = nullptr;
    if (f == 1 && p.scratch) {
        HIPCHK(hipMemsetAsync(p.scratch, 0, sizeof(int), stream));
        hipLaunchKernelGGL(k_sell_far, dim3(std::min<int64_t>((op->n + 255) / 256, 4096)), dim3(256), 0, stream,
                           op->row_ptr, op->col_idx, n, p.scratch);
        HIPCHK(hipGetLastError());
        int far = 1;
        HIPCHK(hipMemcpyAsync(&far, p.scratch, sizeof(int), hipMemcpyDeviceToHost, stream));
        HIPCHK(hipStreamSynchronize(stream));
        if (!far) c16 = reinterpret_cast<uint16_t *>(p.col);
    }
    if (f == 2) {
        if (!p.win) return invalid("sorted sliced-ELL copy without its window table");
        const int rows = p.sort_block * p.sort_ept;
        const int ntiles = (int)(int64_t(p.sort_nslices) * 64 / rows);
        hipLaunchKernelGGL(k_sell_window, dim3(ntiles), dim3(256), 0, stream, op->row_ptr, op->col_idx, n, rows, p.win);
        HIPCHK(hipGetLastError());
        std::vector<int2> w(ntiles);
        HIPCHK(hipMemcpyAsync(w.data(), p.win, sizeof(int2) * ntiles, hipMemcpyDeviceToHost, stream));
        HIPCHK(hipStreamSynchronize(stream));
        bool all = true;
        for (const int2 &t : w) all = all && t.y >= 0;
        if (all) c16 = reinterpret_cast<uint16_t *>(p.col);
    }
    // binary64 values that are all binary32 numbers are stored as binary32
    // (the same values; half the bytes), in the first half of the value array
    float *v32 = nullptr;
    if (prec == PCG_FP64 && p.scratch) {
        HIPCHK(hipMemsetAsync(p.scratch, 0, sizeof(int), stream));
        hipLaunchKernelGGL(k_vals_binary32<double>, dim3((int)std::min<int64_t>((op->nnz + 255) / 256, 4096)), dim3(256),
                           0, stream, reinterpret_cast<const double *>(op->vals), op->nnz, p.scratch);
        HIPCHK(hipGetLastError());
        int inexact = 1;
        HIPCHK(hipMemcpyAsync(&inexact, p.scratch, sizeof(int), hipMemcpyDeviceToHost, stream));
        HIPCHK(hipStreamSynchronize(stream));
        if (!inexact) v32 = reinterpret_cast<float *>(p.val);
    }
    auto fill = [&](auto *tag) {
        using T = std::remove_pointer_t<decltype(tag)>;
        T *sv = reinterpret_cast<T *>(p.val);
        if (f == 1) {
            const int g = (int)((op->n + 255) / 256);
            hipLaunchKernelGGL(k_sell_fill<T>, dim3(g), dim3(256), 0, stream, make_opdev<T>(op), sp, p.col, sv, c16, v32);
            return;
        }
        const int64_t slots = int64_t(p.sort_nslices) * 64;
        const int g = (int)((slots + 255) / 256);
        if (p.sort_ept == 1)
            hipLaunchKernelGGL((k_sell_fill_sorted<T, 1>), dim3(g), dim3(256), 0, stream, make_opdev<T>(op), p.sort_block,
                               slots, tp, perm, p.col, sv, p.win, c16, v32);
        else if (p.sort_ept == 2)
            hipLaunchKernelGGL((k_sell_fill_sorted<T, 2>), dim3(g), dim3(256), 0, stream, make_opdev<T>(op), p.sort_block,
                               slots, tp, perm, p.col, sv, p.win, c16, v32);
        else
            hipLaunchKernelGGL((k_sell_fill_sorted<T, 4>), dim3(g), dim3(256), 0, stream, make_opdev<T>(op), p.sort_block,
                               slots, tp, perm, p.col, sv, p.win, c16, v32);
    };
    if (prec == PCG_FP64) fill((double *)nullptr);
    else fill((float *)nullptr);
    HIPCHK(hipGetLastError());
    *form = f;
    *entries = total[f - 1];
    *col_bits = c16 ? 16 : 32;
    *val_bits = prec == PCG_FP64 && !v32 ? 64 : 32;
    return PCG_OK;
}

// The solver's copies, as its layout reserved them.
static pcg_status sell_setup(const pcg_operator *op, int prec, const LaunchShape &sh, const Layout &L, char *ws,
                             hipStream_t stream, int *form, int64_t *entries, int *col_bits, int *val_bits)
{
    SellPlan p;
    if (L.sell_col != SIZE_MAX) {
        p.sell_ptr = L.sell_ptr == SIZE_MAX ? nullptr : reinterpret_cast<int32_t *>(ws + L.sell_ptr);
        p.nslices = L.nslices;
        p.sort_ptr = L.sort_ptr == SIZE_MAX ? nullptr : reinterpret_cast<int32_t *>(ws + L.sort_ptr);
        p.sort_perm = L.sort_perm == SIZE_MAX ? nullptr : reinterpret_cast<int32_t *>(ws + L.sort_perm);
        p.sort_nslices = L.sort_nslices;
        p.sort_block = sh.sort_block;
        p.sort_ept = sh.sort_ept;
        p.cap = L.sell_cap;
        p.col = reinterpret_cast<int32_t *>(ws + L.sell_col);
        p.val = ws + L.sell_val;
        p.win = L.sort_win == SIZE_MAX ? nullptr : reinterpret_cast<int2 *>(ws + L.sort_win);
        p.scratch = reinterpret_cast<int *>(ws + L.flag) + 1;  // after the CSR check's flag
    }
    return sell_build(op, prec, p, stream, form, entries, col_bits, val_bits);
}

pcg_status csr_gershgorin(const pcg_operator *op, int prec, int jac, double *gb, hipStream_t stream, double *lo,
                          double *hi)
{
    if (prec == PCG_FP64)
        hipLaunchKernelGGL(k_gershgorin<double>, dim3(kGershBlocks), dim3(256), 0, stream, make_opdev<double>(op), jac,
                           gb);
    else
        hipLaunchKernelGGL(k_gershgorin<float>, dim3(kGershBlocks), dim3(256), 0, stream, make_opdev<float>(op), jac,
                           gb);
    HIPCHK(hipGetLastError());
    std::vector<double> h(2 * kGershBlocks);
    HIPCHK(hipMemcpyAsync(h.data(), gb, h.size() * 8, hipMemcpyDeviceToHost, stream));
    HIPCHK(hipStreamSynchronize(stream));
    double l = INFINITY, u = -INFINITY;
    for (int k = 0; k < kGershBlocks; ++k) {
        l = std::fmin(l, h[2 * k]);
        u = std::fmax(u, h[2 * k + 1]);
    }
    *lo = std::fmax(l, 0.0);  // SPD: the spectrum is positive
    *hi = u;
    return PCG_OK;
}

}  // namespace pcg

// ------------------------------------------------------------- C ABI

extern "C" pcg_status pcg_workspace_size(const pcg_operator *op, const pcg_options *opt, size_t *bytes)
{
    if (!bytes) return invalid("bytes is null");
    pcg_status st = validate_options(opt);
    if (st) return st;
    if ((st = validate_operator(op, opt->prec))) return st;
    *bytes = layout(op, opt, choose_shape(op, opt), nullptr);
    return PCG_OK;
}

double pcg::default_sigma(const pcg_operator *op, const pcg_options *opt, const double *gersh_host)
{
    if (opt->method != PCG_PIPE_SHIFT) return 0.0;
    if (!std::isnan(opt->sigma)) return opt->sigma;
    if (op->kind != PCG_OP_CSR) {
        // Dirichlet grid Laplacian: lambda_min + lambda_max = 2 (diag + shift)
        // (cos(j pi/(N+1)) runs symmetrically about 0), so the spectrum
        // midpoint of A is diag + shift and that of A M^-1 with the constant
        // Jacobi diagonal is 1.
        return opt->pc == PCG_PC_JACOBI ? 1.0 : op->diag + op->shift;
    }
    return 0.5 * (gersh_host[0] + gersh_host[1]);
}

// Bind a solver object to (op, opt), a workspace and a stream: validation,
// launch shape, workspace layout, kernel table, CSR set-up and the shift.
// Allocates nothing; the caller has set s->pinned (status slots).
static pcg_status init_solver(pcg_solver_ *s, const pcg_operator *op, const pcg_options *opt, void *workspace,
                              size_t bytes, void *hip_stream)
{
    pcg_status st = validate_options(opt);
    if (st) return st;
    if ((st = validate_operator(op, opt->prec))) return st;
    if (!workspace || !aligned(workspace, 256)) return invalid("workspace must be non-null and 256-byte aligned");
    const LaunchShape sh = choose_shape(op, opt);
    if (sh.zm_rows > 0 && (int64_t)(sh.zm_rows + 2) * op->nx > (int64_t)kZmBatch * sh.block)
        return invalid("z-marching pass: plane window larger than one load batch per thread");
    Layout L;
    const size_t need = layout(op, opt, sh, &L);
    if (bytes < need) return invalid("workspace too small");

    s->op = *op;
    if (s->op.kind != PCG_OP_STENCIL3D7) s->op.nz = 1;
    s->opt = *opt;
    s->stream = (hipStream_t)hip_stream;
    s->ws = (char *)workspace;
    s->ws_bytes = bytes;
    s->L = L;
    s->sh = sh;
    s->kern = pick(opt->prec, op->kind, opt->pc == PCG_PC_JACOBI, sh.ept, sh.nt != 0);
    const double centre = op->diag + op->shift;
    s->dinv_s = 1.0;
    if (opt->pc == PCG_PC_JACOBI && op->kind != PCG_OP_CSR)
        s->dinv_s = opt->prec == PCG_FP64 ? 1.0 / centre : (double)(float)(1.0 / centre);

    double gersh[2] = {0.0, 0.0};
    if (op->kind == PCG_OP_CSR) {
        const int jac = opt->pc == PCG_PC_JACOBI;
        if ((st = csr_setup(op, opt->prec, jac, jac ? s->ws + L.dinv : nullptr, reinterpret_cast<int *>(s->ws + L.flag),
                            s->stream)))
            return st;
        if (opt->method == PCG_PIPE_SHIFT && std::isnan(opt->sigma) &&
            (st = csr_gershgorin(op, opt->prec, jac, reinterpret_cast<double *>(s->ws + L.gersh), s->stream, &gersh[0],
                                 &gersh[1])))
            return st;
        if ((st = sell_setup(op, opt->prec, sh, L, s->ws, s->stream, &s->sell, &s->sell_entries, &s->sell_col_bits,
                             &s->sell_val_bits)))
            return st;
        // the sorted copy is laid out for its own shape: the passes take it,
        // and its grid
        const int sort_grid = opt->prec == PCG_FP64 && s->sell_val_bits == 32 ? sh.sort_grid_v32 : sh.sort_grid;
        if (s->sell == 2 && (sh.sort_ept != sh.ept || sh.sort_block != sh.block || sort_grid != sh.grid)) {
            s->sh.ept = sh.sort_ept, s->sh.block = sh.sort_block;
            s->sh.ntiles = sh.sort_ntiles, s->sh.grid = sort_grid;
            s->kern = pick(opt->prec, op->kind, opt->pc == PCG_PC_JACOBI, s->sh.ept, s->sh.nt != 0);
        }
    }
    s->sigma = default_sigma(op, opt, gersh);
    if (opt->method == PCG_PIPE_VAR_SHIFT) {
        s->sched.assign(opt->sigma_schedule, opt->sigma_schedule + opt->sigma_schedule_len);
        s->opt.sigma_schedule = nullptr;  // the caller's array is not kept
        HIPCHK(hipMemcpyAsync(s->ws + L.sched, s->sched.data(), s->sched.size() * 8, hipMemcpyHostToDevice, s->stream));
        HIPCHK(hipStreamSynchronize(s->stream));
    }
    return PCG_OK;
}

extern "C" pcg_status pcg_create(pcg_solver *out, const pcg_operator *op, const pcg_options *opt, void *workspace,
                                 size_t bytes, void *hip_stream)
{
    if (!out) return invalid("solver out-pointer is null");
    *out = nullptr;
    pcg_status st = validate_options(opt);
    if (st) return st;
    if ((st = validate_operator(op, opt->prec))) return st;
    if (!workspace || !aligned(workspace, 256)) return invalid("workspace must be non-null and 256-byte aligned");
    if (bytes < layout(op, opt, choose_shape(op, opt), nullptr)) return invalid("workspace too small");

    pcg_solver_ *s = new pcg_solver_();
    auto fail = [&](pcg_status e) {
        pcg_destroy(s);
        return e;
    };
    hipError_t he;
    if ((he = hipHostMalloc((void **)&s->pinned, 2 * sizeof(DevState), hipHostMallocDefault)) != hipSuccess)
        return fail(hip_fail(he, "hipHostMalloc"));
    for (int k = 0; k < 2; ++k) {
        if ((he = hipEventCreate(&s->ev_begin[k])) != hipSuccess) return fail(hip_fail(he, "hipEventCreate"));
        if ((he = hipEventCreate(&s->ev_end[k])) != hipSuccess) return fail(hip_fail(he, "hipEventCreate"));
        if ((he = hipEventCreateWithFlags(&s->ev_copy[k], hipEventDisableTiming)) != hipSuccess)
            return fail(hip_fail(he, "hipEventCreate"));
    }
    if ((st = init_solver(s, op, opt, workspace, bytes, hip_stream))) return fail(st);
    *out = s;
    return PCG_OK;
}

extern "C" pcg_status pcg_solver_info(pcg_solver s, pcg_solver_shape *out)
{
    if (!s || !out) return invalid("null argument");
    out->block = s->sh.block;
    out->ept = s->sh.ept;
    out->grid = s->sh.grid;
    out->ntiles = s->sh.ntiles;
    out->iters_per_launch = s->sh.K;
    out->csr_form = s->sell;
    out->csr_col_bits = s->sell_col_bits;
    out->csr_val_bits = s->sell_val_bits;
    out->csr_entries = s->sell_entries;
    return PCG_OK;
}

extern "C" pcg_status pcg_destroy(pcg_solver s)
{
    if (!s) return PCG_OK;
    if (s->gexec) (void)hipGraphExecDestroy(s->gexec);
    if (s->graph) (void)hipGraphDestroy(s->graph);
    for (int k = 0; k < 2; ++k) {
        if (s->ev_begin[k]) (void)hipEventDestroy(s->ev_begin[k]);
        if (s->ev_end[k]) (void)hipEventDestroy(s->ev_end[k]);
        if (s->ev_copy[k]) (void)hipEventDestroy(s->ev_copy[k]);
    }
    if (s->pinned && !s->no_alloc) (void)hipHostFree(s->pinned);
    delete s;
    return PCG_OK;
}

// Build (once per b) the graph of K iteration passes.  The passes read only
// the workspace and b, so the graph is reused by every solve with that b.
static pcg_status ensure_graph(pcg_solver_ *s, const double *b)
{
    if (s->gexec && s->graph_b == b) return PCG_OK;
    if (s->gexec) {
        (void)hipGraphExecDestroy(s->gexec);
        s->gexec = nullptr;
    }
    if (s->graph) {
        (void)hipGraphDestroy(s->graph);
        s->graph = nullptr;
    }
    hipStream_t cs;
    HIPCHK(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
    hipError_t e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) {
        (void)hipStreamDestroy(cs);
        return hip_fail(e, "hipStreamBeginCapture");
    }
    enqueue_iterations(s, cs, b);
    e = hipStreamEndCapture(cs, &s->graph);
    (void)hipStreamDestroy(cs);
    if (e != hipSuccess) return hip_fail(e, "hipStreamEndCapture");
    HIPCHK(hipGraphInstantiate(&s->gexec, s->graph, nullptr, nullptr, 0));
    s->graph_b = b;
    return PCG_OK;
}

pcg_status pcg_solver_::launch_iterations(const double *b)
{
    if (opt.use_graph) {
        pcg_status st = ensure_graph(this, b);
        if (st) return st;
        HIPCHK(hipGraphLaunch(gexec, stream));
    } else {
        enqueue_iterations(this, stream, b);
        HIPCHK(hipGetLastError());
    }
    return PCG_OK;
}

extern "C" pcg_status pcg_solve(pcg_solver s, const double *b, double *x, pcg_result *res)
{
    if (!s) return PCG_ERR_STATE;
    if (!b || !x || !res) return invalid("b, x and result must be non-null");
    if (!aligned(b, 8) || !aligned(x, 8)) return invalid("b and x must be 8-byte aligned");
    if (b == x) return invalid("x must not alias b");
    const auto t0 = std::chrono::steady_clock::now();
    std::memset(res, 0, sizeof(*res));
    res->sigma = s->sigma;
    res->rel_res_true = std::nan("");
    const pcg_options &o = s->opt;
    if (o.history_cap > 0)
        HIPCHK(hipMemsetAsync(s->ws + s->L.hist, 0xff, size_t(o.history_cap) * PCG_HISTORY_FIELDS * 8, s->stream));

    pcg_status st = s->run_copy_x(x, 0);
    if (st) return st;
    if ((st = s->run_init(b, 0))) return st;

    DevState S{};
    int launches = 0;
    double kernel_ms = 0.0;
    int replacements = 0, rr_before = 0;
    auto add_time = [&](int slot) -> pcg_status {
        if (o.timing) {
            float ms = 0.f;
            HIPCHK(hipEventElapsedTime(&ms, s->ev_begin[slot], s->ev_end[slot]));
            kernel_ms += ms;
        }
        return PCG_OK;
    };
    for (;;) {
        // Two launches in flight: issue launch g, then wait for the status
        // copied after launch g - 1, so the host round trip overlaps work.
        bool done = false;
        for (int g = 0; !done; ++g) {
            const int slot = g & 1;
            if (s->no_alloc) {
                // one launch at a time, its status read back into pageable memory
                if ((st = s->launch_iterations(b))) return st;
                HIPCHK(hipMemcpyAsync(&s->pinned[slot], s->state(0), sizeof(DevState), hipMemcpyDeviceToHost,
                                      s->stream));
                HIPCHK(hipStreamSynchronize(s->stream));
                ++launches;
                done = s->pinned[slot].status != RUNNING;
                if (done) S = s->pinned[slot];
                continue;
            }
            if (o.timing) HIPCHK(hipEventRecord(s->ev_begin[slot], s->stream));
            if ((st = s->launch_iterations(b))) return st;
            if (o.timing) HIPCHK(hipEventRecord(s->ev_end[slot], s->stream));
            HIPCHK(hipMemcpyAsync(&s->pinned[slot], s->state(0), sizeof(DevState), hipMemcpyDeviceToHost, s->stream));
            HIPCHK(hipEventRecord(s->ev_copy[slot], s->stream));
            ++launches;
            if (g > 0) {
                const int prev = slot ^ 1;
                HIPCHK(hipEventSynchronize(s->ev_copy[prev]));
                if ((st = add_time(prev))) return st;
                done = s->pinned[prev].status != RUNNING;
            }
            if (done) {
                HIPCHK(hipEventSynchronize(s->ev_copy[slot]));
                if ((st = add_time(slot))) return st;
                S = s->pinned[slot];
            }
        }
        // the fused pass updates x every other iteration (k_pipe); complete x
        // when the last pass that ran skipped it
        const bool lagged = o.method == PCG_PIPE || o.method == PCG_PIPE_SHIFT || o.method == PCG_PIPE_VAR_SHIFT;
        if (lagged && S.iter > S.i_start && ((S.iter - 1 - S.i_start) & 1) == 0) {
            s->kern.x_fixup(s->args(0, b, nullptr), S.alpha_prev, s->sh.grid, s->sh.block, s->stream);
            HIPCHK(hipGetLastError());
        }
        if (S.status == ST_NONFINITE && !(std::isfinite(S.bnorm2))) {
            res->status = PCG_NONFINITE;
            res->iterations = 0;
            HIPCHK(hipStreamSynchronize(s->stream));
            return PCG_ERR_NONFINITE;
        }
        if (S.status == ST_CONVERGED && o.true_residual_check && replacements < o.replace_max &&
            S.iter < o.max_iter) {
            double tr2 = 0.0;
            if ((st = s->run_true_residual(b, nullptr, &tr2))) return st;
            // restart from x when the explicit residual misses the tolerance
            if (std::sqrt(tr2) > o.rtol * std::sqrt(S.bnorm2)) {
                ++replacements;
                rr_before += S.rr_count;  // the restart starts a fresh device state
                if ((st = s->run_init(b, S.iter))) return st;
                continue;
            }
        }
        break;
    }
    double tr2 = 0.0;
    if ((st = s->run_true_residual(b, nullptr, &tr2))) return st;
    if ((st = s->run_copy_x(x, 1))) return st;
    const double bn = std::sqrt(S.bnorm2);
    res->status = S.status;
    res->iterations = S.iter;
    res->replacements = replacements + rr_before + S.rr_count;
    res->launches = launches;
    res->rel_res_recursive = bn > 0 ? std::sqrt(S.rho) / bn : std::sqrt(S.rho);
    res->rel_res_true = bn > 0 ? std::sqrt(tr2) / bn : std::sqrt(tr2);
    res->iter_kernel_ms = kernel_ms;
    res->iter_passes = (o.method == PCG_CG ? 2 : 1) * S.iter;
    if (o.method == PCG_PIPE_VAR_SHIFT)  // sigma_{i-1}: the shift of the final w_i
        res->sigma = s->sched[std::min(size_t(S.iter), s->sched.size() - 1)];
    if (o.history_cap > 0)
        HIPCHK(hipMemcpyAsync(o.history, s->ws + s->L.hist, size_t(o.history_cap) * PCG_HISTORY_FIELDS * 8,
                              hipMemcpyDeviceToHost, s->stream));
    HIPCHK(hipStreamSynchronize(s->stream));
    res->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    return PCG_OK;
}

extern "C" pcg_status pcg_true_residual(pcg_solver s, const double *b, const double *x, double *rel)
{
    if (!s) return PCG_ERR_STATE;
    if (!b || !x || !rel) return invalid("b, x and rel must be non-null");
    double tr2 = 0.0, b2 = 0.0;
    pcg_status st = s->run_true_residual(b, x, &tr2, &b2);
    if (st) return st;
    *rel = b2 > 0 ? std::sqrt(tr2) / std::sqrt(b2) : std::sqrt(tr2);
    return PCG_OK;
}

// ------------------------------------------------- static-scratch solve

// Device scratch of pcg_solve_static: the workspace of one solver (state,
// partials, Krylov vectors) lives here instead of in caller memory.  Each
// device that runs the library holds its own copy until the process ends.
// Host code never passes this array's name to a kernel or a copy: the name
// is a host-side stand-in, and the device address comes from
// hipGetSymbolAddress, per device.
static __device__ __align__(256) char scratch[PCG_STATIC_SCRATCH_BYTES];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_static_mu[kMaxDevices];       // one static solve per device at a time
char *g_static_ptr[kMaxDevices] = {};      // device address of `scratch`, per device
}  // namespace

extern "C" pcg_status pcg_solve_static(const pcg_operator *op, const pcg_options *opt, const double *b, double *x,
                                       pcg_result *result, void *hip_stream)
{
    if (!result) return invalid("result must be non-null");
    pcg_status st = validate_options(opt);
    if (st) return st;
    if ((st = validate_operator(op, opt->prec))) return st;
    if (!b || !x) return invalid("b and x must be non-null");
    const size_t need = layout(op, opt, choose_shape(op, opt), nullptr);
    if (need > PCG_STATIC_SCRATCH_BYTES) {
        g_last_error = "invalid argument: the solve needs " + std::to_string(need) +
                       " bytes of scratch; the static scratch holds " + std::to_string((size_t)PCG_STATIC_SCRATCH_BYTES);
        return PCG_ERR_INVALID;
    }
    int dev = 0;
    HIPCHK(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) return invalid("device index beyond the static scratch table");
    std::lock_guard<std::mutex> lk(g_static_mu[dev]);
    if (!g_static_ptr[dev]) {
        // once per device, with that device current
        void *p = nullptr;
        HIPCHK(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        g_static_ptr[dev] = static_cast<char *>(p);
    }
    pcg_solver_ s;
    s.no_alloc = true;
    s.pinned = s.host_state;
    pcg_options o = *opt;
    o.use_graph = 0;  // passes are launched one by one: no graph instantiation
    o.timing = 0;     // no events
    if ((st = init_solver(&s, op, &o, g_static_ptr[dev], PCG_STATIC_SCRATCH_BYTES, hip_stream))) return st;
    return pcg_solve(&s, b, x, result);
}
