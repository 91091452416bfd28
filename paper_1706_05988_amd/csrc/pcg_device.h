// pcg_device.h -- device-side building blocks of the fused p-CG(-sh) passes.
//
// Everything here is gfx950 code written for 64-wide wavefronts:
//   * FastDiv: division by a runtime constant (grid extents) with one
//     multiply-high, used to recover stencil coordinates from a flat index.
//   * wave64 butterfly reductions and a fixed-order block reduction, which
//     give the same bits in every lane and every block -- the basis of the
//     deterministic two-stage FP64 grid reduction of the dot products.
//   * the operator: Dirichlet 5-/7-point stencils (matrix-free, neighbours
//     summed centre, -x, +x, -y, +y, -z, +z) and CSR rows (storage order).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace pcg {

// ------------------------------------------------------------------ enums

enum OpKind : int { OP_2D5 = 0, OP_3D7 = 1, OP_CSR = 2 };

// run status kept in the device state (PCG_CONVERGED.. values of pcg.h, or
// RUNNING while the iteration goes on)
enum RunStatus : int { RUNNING = -1, ST_CONVERGED = 0, ST_MAX_ITER = 1, ST_BREAKDOWN = 2, ST_NONFINITE = 3 };

constexpr int kFields = 4;      // doubles per block partial (32 bytes)
#ifndef PCG_CSR_CHUNK
#define PCG_CSR_CHUNK 8
#endif
constexpr int kCsrChunk = PCG_CSR_CHUNK;  // CSR entries whose loads are issued together
constexpr int kMaxWaves = 16;   // up to 1024 threads per block (reduction scratch)
constexpr int kMaxBlock = 256;  // threads per block of the solver passes: a bound of
                                // 256 lets a pass keep all of a tile's loads in
                                // registers (a 1024 bound caps it at 128 VGPRs and spills)

// ------------------------------------------------------------------ state

// Scalars carried from one pass to the next.  Pass k reads slot k%2 and
// block 0 writes slot (k+1)%2, so no block ever reads what another block of
// the same pass writes.
struct DevState {
    double bnorm2;      // ||b||^2
    double alpha_prev;  // alpha_{i-1}
    double gamma_prev;  // gamma_{i-1}
    double rho;         // rho_i = (r_i, r_i) of the last head reduction
    double gamma;       // CG: gamma_i handed from pass A to pass B
    double true_res2;   // ||b - A x||^2 of the last explicit-residual pass
    int32_t iter;       // i at the top of the next pass
    int32_t i_start;    // iteration of the last (re)start: takes the i = 0 branch
    int32_t status;     // RunStatus
    int32_t rr_phase;   // residual replacement: RrPhase of the next pass
    double spare[2];    // [0]: ||b||^2 of an explicit-residual pass; [1]: delta_i held across a gap check
    int32_t wflip;      // residual replacement: w_i sits in the slot the pass would write
    int32_t last_check; // residual replacement: iteration of the last gap check
    int32_t rr_count;   // residual replacements performed
    int32_t pad;
};
static_assert(sizeof(DevState) == 96, "DevState layout");

// Residual-replacement pass sequence (pipelined CG with replacement):
// ITER passes iterate or, every rr_period iterations, measure the gap
// (b - A x) - r instead; the CHECK pass that follows either iterates or
// starts a replacement, which takes two passes (the second is RR2).
enum RrPhase : int32_t { RR_ITER = 0, RR_CHECK = 1, RR_RR2 = 2 };

// ------------------------------------------------------------ fast division

// q = x / d for 0 <= x < 2^31, d >= 1:  q = (umulhi(x, m) + x) >> s with
// s = ceil(log2 d) and m = floor(2^32 (2^s - d) / d) + 1 (round-up method of
// Granlund & Montgomery; exact for 31-bit numerators).
struct FastDiv {
    uint32_t d, m, s, pad;
};

inline FastDiv make_fastdiv(uint32_t d)
{
    FastDiv f{};
    f.d = d;
    uint32_t s = 0;
    while ((1ull << s) < d) ++s;
    f.s = s;
    f.m = (uint32_t)(((1ull << 32) * ((1ull << s) - d)) / d + 1);
    return f;
}

__host__ __device__ inline uint32_t fdiv(uint32_t x, const FastDiv &f)
{
#if defined(__HIP_DEVICE_COMPILE__)
    uint32_t hi = __umulhi(x, f.m);
#else
    uint32_t hi = (uint32_t)(((uint64_t)x * f.m) >> 32);
#endif
    return (hi + x) >> f.s;
}

// --------------------------------------------------------------- operator

template <typename T>
struct OpDev {
    int32_t n;           // unknowns
    int32_t nx, ny, nz;  // stencil grid
    FastDiv dx;          // / nx
    FastDiv dxy;         // / (nx * ny)
    double centre;       // diag + shift
    double off;          // off-diagonal coefficient
    const int32_t *row_ptr;
    const int32_t *col;
    const T *val;
};

template <typename T>
__device__ __forceinline__ double ld(const T *p, uint32_t i) { return (double)p[i]; }

// Round a value to the storage type and back, so that every later use of a
// stored quantity sees exactly the stored bits.
template <typename T>
__device__ __forceinline__ double rnd(double v) { return (double)(T)v; }

// Stencil neighbourhood of row e: the neighbour indices in the fixed order
// -x, +x, -y, +y, -z, +z and whether each exists (Dirichlet boundary).  A
// missing neighbour's index is clamped to e itself, so that every operand
// load is unconditional (all loads of a row issue back to back) and the
// missing terms are dropped by a select, never by a branch around a load.
template <int OP>
struct Nbhd {
    static constexpr int ND = OP == OP_3D7 ? 6 : 4;
    uint32_t idx[ND];
    bool ok[ND];
};

template <int OP, typename T>
__device__ __forceinline__ Nbhd<OP> neighbours(const OpDev<T> &A, uint32_t e)
{
    Nbhd<OP> h;
    const uint32_t q = fdiv(e, A.dx);  // e / nx
    const uint32_t i = e - q * (uint32_t)A.nx;
    uint32_t j, k = 0;
    if constexpr (OP == OP_3D7) {
        k = fdiv(e, A.dxy);
        j = q - k * (uint32_t)A.ny;
    } else {
        j = q;
    }
    const uint32_t nx = (uint32_t)A.nx, sxy = (uint32_t)A.nx * (uint32_t)A.ny;
    h.ok[0] = i > 0;
    h.ok[1] = i + 1 < nx;
    h.ok[2] = j > 0;
    h.ok[3] = j + 1 < (uint32_t)A.ny;
    h.idx[0] = h.ok[0] ? e - 1 : e;
    h.idx[1] = h.ok[1] ? e + 1 : e;
    h.idx[2] = h.ok[2] ? e - nx : e;
    h.idx[3] = h.ok[3] ? e + nx : e;
    if constexpr (OP == OP_3D7) {
        h.ok[4] = k > 0;
        h.ok[5] = k + 1 < (uint32_t)A.nz;
        h.idx[4] = h.ok[4] ? e - sxy : e;
        h.idx[5] = h.ok[5] ? e + sxy : e;
    }
    return h;
}

// (A v)_e.  v(k) returns the k-th entry of the operand.  Stencil rows sum
// centre, -x, +x, -y, +y, -z, +z in that order (missing neighbours skipped);
// CSR rows sum their entries in storage order.
template <int OP, bool ABS = false, typename T, typename F>
__device__ __forceinline__ double apply_row(const OpDev<T> &A, uint32_t e, F v)
{
    if constexpr (OP == OP_CSR) {
        // Chunks of kCsrChunk entries: all index / value loads of a chunk are
        // issued together (positions past the row end re-read the row's
        // first entry, which is in bounds and cached), then all gathers, then
        // the products are added in storage order.  A row costs three memory
        // latencies per chunk instead of two per entry.
        const int32_t k0 = A.row_ptr[e], k1 = A.row_ptr[e + 1];
        double acc = 0.0;
        for (int32_t k = k0; k < k1; k += kCsrChunk) {
            int32_t c[kCsrChunk];
            T w[kCsrChunk];
            double g[kCsrChunk];
#pragma unroll
            for (int j = 0; j < kCsrChunk; ++j) {
                const int32_t kk = k + j < k1 ? k + j : k0;
                c[j] = A.col[kk];
                w[j] = A.val[kk];
            }
#pragma unroll
            for (int j = 0; j < kCsrChunk; ++j) g[j] = v((uint32_t)c[j]);
#pragma unroll
            for (int j = 0; j < kCsrChunk; ++j)
                if (k + j < k1) acc += (ABS ? fabs((double)w[j]) : (double)w[j]) * g[j];
        }
        return acc;
    } else {
        const Nbhd<OP> h = neighbours<OP>(A, e);
        double nv[Nbhd<OP>::ND];
        const double c = v(e);
#pragma unroll
        for (int d = 0; d < Nbhd<OP>::ND; ++d) nv[d] = v(h.idx[d]);
        const double cc = ABS ? fabs(A.centre) : A.centre, oo = ABS ? fabs(A.off) : A.off;
        double acc = cc * c;
#pragma unroll
        for (int d = 0; d < Nbhd<OP>::ND; ++d) acc = h.ok[d] ? acc + oo * nv[d] : acc;
        return acc;
    }
}

// ---------------------------------------------------------------- reductions

__device__ __forceinline__ double wave_sum(double v)
{
    // xor butterfly: every lane ends with the same bits (each step adds the
    // same two operands in every lane, and IEEE addition is commutative)
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// Sum NF values over the block in a fixed order; the result is returned in
// every thread.  lds: kMaxWaves * kFields doubles.  Ends with a barrier so
// the LDS can be reused.
template <int NF>
__device__ __forceinline__ void block_sum(double (&v)[NF], double *lds)
{
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
#pragma unroll
    for (int f = 0; f < NF; ++f) v[f] = wave_sum(v[f]);
    if (lane == 0) {
#pragma unroll
        for (int f = 0; f < NF; ++f) lds[wave * kFields + f] = v[f];
    }
    __syncthreads();
#pragma unroll
    for (int f = 0; f < NF; ++f) {
        double s = 0.0;
        for (int w = 0; w < nw; ++w) s += lds[w * kFields + f];
        v[f] = s;
    }
    __syncthreads();
}

// Stage 2 of the grid reduction: sum the P block partials (kFields doubles
// each) in a fixed order -- thread t takes partials t, t + B, t + 2B, ...
// sequentially, then the fixed block order above.  Every block computes the
// same bits.
template <int NF>
__device__ __forceinline__ void stage2(const double *part, int P, double (&tot)[NF], double *lds)
{
#pragma unroll
    for (int f = 0; f < NF; ++f) tot[f] = 0.0;
    // thread t sums partials t, t + B, t + 2B, ... in that order; the loads of
    // four of them are issued before the first is added, so a grid of P
    // blocks costs ceil(P / 4B) memory latencies here, not ceil(P / B)
    const int B = blockDim.x;
    for (int k0 = threadIdx.x; k0 < P; k0 += 4 * B) {
        double v[4][NF];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int k = k0 + u * B < P ? k0 + u * B : P - 1;
#pragma unroll
            for (int f = 0; f < NF; ++f) v[u][f] = part[k * kFields + f];
        }
#pragma unroll
        for (int u = 0; u < 4; ++u)
            if (k0 + u * B < P) {
#pragma unroll
                for (int f = 0; f < NF; ++f) tot[f] += v[u][f];
            }
    }
    block_sum<NF>(tot, lds);
}

// Write the block's NF partial sums (already block-summed, so equal in every
// thread) to part[blockIdx]; unused fields are written as zero.
template <int NF>
__device__ __forceinline__ void store_partial(double *part, const double (&v)[NF])
{
    if (threadIdx.x == 0) {
#pragma unroll
        for (int f = 0; f < kFields; ++f) part[blockIdx.x * kFields + f] = f < NF ? v[f] : 0.0;
    }
}

// ------------------------------------------------------- blocked vectors

// The solver's vectors live in the workspace interleaved per tile of
// kBlk = 512 unknowns: tile t holds slot 0 (512 values), slot 1, ... one
// after another, so the ~10 vectors one pass streams through are read and
// written in one contiguous region per tile instead of ~10 regions spread
// over HBM (measured ~10% more bandwidth for this access pattern on MI355X).
// The address of unknown e of a slot at byte offset `off` within a tile is
//     base + (e / kBlk) * tile_bytes + off + (e % kBlk) * sizeof(value).
constexpr uint32_t kBlkShift = 9;
constexpr uint32_t kBlk = 1u << kBlkShift;
constexpr uint32_t kNoSlot = 0xffffffffu;

template <typename V>
__host__ __device__ __forceinline__ V *slot_ptr(char *base, uint32_t tile_bytes, uint32_t off, uint32_t e)
{
    return reinterpret_cast<V *>(base + (size_t)(e >> kBlkShift) * tile_bytes + off +
                                 (size_t)(e & (kBlk - 1)) * sizeof(V));
}

// ------------------------------------------------------- persistent tiling

// Tiles are contiguous runs of blockDim * EPT unknowns.  With the XCD map on,
// the tiles are split into 8 contiguous slabs and the blocks that the
// hardware places on XCD x (blockIdx % 8 == x) sweep slab x in order, so a
// stencil's neighbouring rows and planes are fetched through the same L2.
struct TileRange {
    int first, step, end;
};

__device__ __forceinline__ TileRange tile_range(int ntiles, int xcd_map)
{
    TileRange t;
    if (xcd_map) {
        const int per = (ntiles + 7) >> 3;
        const int x = blockIdx.x & 7;
        t.first = x * per + (int)(blockIdx.x >> 3);
        t.step = (int)(gridDim.x >> 3);
        t.end = min(ntiles, (x + 1) * per);
    } else {
        t.first = blockIdx.x;
        t.step = gridDim.x;
        t.end = ntiles;
    }
    return t;
}

}  // namespace pcg
