// pcg_internal.h -- host-side declarations shared by the library's sources.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <string>

#include "pcg.h"
#include "pcg_device.h"

namespace pcg {

constexpr int kNumCU = 256;              // MI355X compute units (8 XCDs x 32)
constexpr int kDefaultBlocksPerCU = 4;   // persistent grid: 4 blocks of 256 threads per CU
constexpr int kMaxGrid = 16384;
constexpr int kGershBlocks = 256;

// vector slots of the blocked workspace region
enum VecSlot { V_X = 0, V_R, V_U, V_W0, V_W1, V_Z, V_Q, V_S, V_T, V_P, V_COUNT };

struct LaunchShape {
    int block;    // threads per block
    int ept;      // unknowns per thread per tile
    int ntiles;   // tiles of block * ept unknowns
    int grid;     // persistent blocks
    int xcd_map;  // XCD-slab tile order on/off
    int nt;       // non-temporal streams on/off
    int K;        // iterations per graph launch
    int zm_rows, zm_seg, zm_nchunks, zm_nsegs;  // CG pass A z-marching split (zm_rows = 0: plain)
    // CSR operand of the fused pipelined pass in sliced-ELL form (where it
    // fits): bit 0 rows in place, bit 1 rows sorted by length within each
    // wave's rows; with both, set-up keeps the smaller copy.  The sorted copy
    // is laid out for the shape sort_*, which replaces the shape above when
    // that copy is the one kept.  sort_grid_v32 is the sorted copy's grid
    // when it stores binary64 values as binary32 (known after set-up).
    int sell;
    int sort_block, sort_ept, sort_ntiles, sort_grid, sort_grid_v32;
};

// byte offsets into the caller's workspace (SIZE_MAX: absent)
struct Layout {
    size_t state, part[2], gersh, flag, hist, dinv;
    size_t sched;                // variable-shift schedule (SIZE_MAX: none)
    size_t blk;                  // blocked vectors: ceil(n / 512) tiles of tile_bytes
    // sliced-ELL copy of a CSR operator for the fused pipelined pass
    // (SIZE_MAX: none): slice offsets, columns and values of up to sell_cap entries
    size_t sell_ptr, sell_col, sell_val;
    int64_t sell_cap;
    int32_t nslices;
    // its sorted form: slice offsets, per-slot (length << 8) | position and
    // per-tile column windows
    size_t sort_ptr, sort_perm, sort_win;
    int32_t sort_nslices;
    uint32_t tile_bytes;
    uint32_t slot_off[V_COUNT];  // byte offset of each slot in a tile (kNoSlot: absent)
    size_t total;
};

// Type-erased kernel arguments (PassArgs<double> or PassArgs<float>).
struct PassArgsAny {
    alignas(16) unsigned char bytes[384];
};

template <typename T>
inline OpDev<T> make_opdev(const pcg_operator *op)
{
    OpDev<T> A{};
    A.n = (int32_t)op->n;
    A.nx = op->nx;
    A.ny = op->ny;
    A.nz = op->kind == PCG_OP_STENCIL3D7 ? op->nz : 1;
    if (op->kind != PCG_OP_CSR) {
        A.dx = make_fastdiv((uint32_t)op->nx);
        A.dxy = make_fastdiv((uint32_t)op->nx * (uint32_t)op->ny);
    }
    A.centre = op->diag + op->shift;
    A.off = op->offdiag;
    A.row_ptr = op->row_ptr;
    A.col = op->col_idx;
    A.val = (const T *)op->vals;
    return A;
}

extern thread_local std::string g_last_error;
pcg_status hip_fail(hipError_t e, const char *what);
pcg_status invalid(const char *why);
pcg_status validate_operator(const pcg_operator *op, int prec);
pcg_status validate_options(const pcg_options *o);
// Validate a CSR operator's structure on the device (synchronous on stream);
// with jac, also fill dinv (n values of the storage type) with 1 / a_kk.
pcg_status csr_setup(const pcg_operator *op, int prec, int jac, void *dinv, int *flag_dev, hipStream_t stream);
// The shift in use: 0 for CG / p-CG, the caller's sigma, or (NaN) the
// midpoint of the spectrum bounds of A M^-1 -- closed form for stencils,
// gersh_host[0..1] (Gershgorin) for CSR.
double default_sigma(const pcg_operator *op, const pcg_options *opt, const double *gersh_host);
// Gershgorin bounds of spec(M^-1 A) of a CSR operator (synchronous).
pcg_status csr_gershgorin(const pcg_operator *op, int prec, int jac, double *scratch_dev, hipStream_t stream,
                          double *lo, double *hi);

// Where the sliced-ELL copies of a CSR operator go (device memory; nullptr /
// 0 for a form not reserved): the in-place form's nslices + 1 slice offsets,
// the sorted form's sort_nslices + 1 offsets and per-slot words (laid out for
// tiles of sort_block x sort_ept rows), and the shared entry arrays of cap
// entries.
struct SellPlan {
    int32_t *sell_ptr = nullptr;
    int32_t nslices = 0;
    int32_t *sort_ptr = nullptr, *sort_perm = nullptr;
    int32_t sort_nslices = 0;
    int sort_block = 0, sort_ept = 0;
    int64_t cap = 0;
    int32_t *col = nullptr;
    void *val = nullptr;  // cap values of the storage type
    int2 *win = nullptr;  // sorted form: per tile, its column window (see k_sell_window)
    int *scratch = nullptr;  // one device int for the set-up's checks
};
// Build the smaller of the reserved copies that fits cap (synchronous):
// *form 0 (none fits), 1 (in place; slice offsets at sell_ptr) or 2 (sorted;
// at sort_ptr / sort_perm, tile windows at win); *entries its entries;
// *col_bits 32, or 16 when every tile of a sorted copy has a window (the
// columns are then 16-bit window offsets in the first half of col) or every
// entry of an in-place copy lies within 2^15 of its row (16-bit offsets from
// the row); *val_bits 32 or 64 (binary64 values that are all binary32
// numbers are stored as binary32, in the first half of val).
pcg_status sell_build(const pcg_operator *op, int prec, const SellPlan &p, hipStream_t stream, int *form,
                      int64_t *entries, int *col_bits, int *val_bits);

}  // namespace pcg
