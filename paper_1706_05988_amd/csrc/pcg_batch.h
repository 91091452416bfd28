// pcg_batch.h -- many independent solves advanced by one persistent pass.
//
// Every active system moves one phase or one iteration per pass:
//   ADMIT   (admitted, nothing done yet)
//   COPYIN  caller x -> internal (blocked) x
//   INIT0   r_0 := b - A x_0, u_0 := M^-1 r_0, z = q = s = t = p := 0; (b, b)
//   INIT1   w_0 := A u_0 - sigma r_0; gamma_0, delta_0, rho_0
//   ITER    one iteration of shifted pipelined CG (Alg. 3); x is written
//           every other iteration (the pass of iteration i leaves it, that
//           of i + 1 applies both updates in order)
//   XFIX    x := x + alpha p when the last iteration pass left x
//   RESID   ||b - A x|| in binary64 (after the iteration ends)
//   COPYOUT internal x -> caller x
// The pass kernel works on a table of (system, tile) items; each tile is
// 256 * kBatchEPT unknowns and writes one partial per wave into its
// system's partial array (no block barrier between items).  At its head,
// every item block sums its system's partials of the previous pass in
// tile and wave order (so a system's results depend
// only on that system, never on the rest of the batch), takes the stop /
// breakdown / restart decisions and the scalar recurrences -- the same bits
// in every block of the system -- and performs the next phase on its tile;
// the block of tile 0 writes the system's new state.  State and partials
// ping-pong between two slots (pass k reads slot k%2), so one kernel per
// iteration suffices and the passes need no atomics or fences across the
// XCDs (only the transition of a chunked system counts its chunk sums).
// With many items that head (a chain of dependent loads and a block
// reduction before the tile's own loads) costs more than a kernel launch,
// so large batches run split: a transition kernel (one block per system,
// or per chunk of a large system's partials) followed by the pass without
// the head.  Both compute the same transition with the same reduction, so
// the results do not depend on the mode.
#pragma once

#include "pcg_internal.h"
#include "pcg_kernels.h"

namespace pcg {

// A state's phase is the one its system performed in the pass that wrote it.
enum Phase : int32_t {
    PH_ADMIT = 0, PH_COPYIN, PH_INIT0, PH_INIT1, PH_ITER, PH_XFIX, PH_RESID, PH_COPYOUT, PH_DONE, PH_FREE
};

constexpr int kBatchBlock = 256;      // threads of a pass block
constexpr int kSpecAny = -1;          // pass kernels read operator kind and preconditioner per system
constexpr int kBatchWaves = kBatchBlock / 64;  // partials per work tile (one per wave)
#ifndef PCG_BATCH_EPT
#define PCG_BATCH_EPT 4
#endif
constexpr int kBatchEPT = PCG_BATCH_EPT;  // unknowns per thread: a work tile is 256 * kBatchEPT unknowns
// A system with more partials than this has them summed in fixed chunks of
// this many (one block per chunk, the stage-2 order within a chunk), and its
// transition adds the chunk sums in chunk order: the sum of a large system
// does not wait on one block reading all its partials.  The block that
// writes a system's last chunk sum (counted with an atomic) takes the
// transition, in the same kernel.
constexpr int kChunkParts = 1024;

// Per-system descriptor, written once at admission.
struct BatchSys {
    int32_t kind, jac, n, ntiles;  // ntiles: work tiles of the pass
    int32_t nx, ny, nz, max_iter;
    FastDiv dx, dxy;
    double centre, off, dinv_s, sigma, rtol;
    const int32_t *row_ptr;
    const int32_t *col;
    const void *val;
    const void *dinv;
    const double *b;
    double *x;
    char *blk;
    uint32_t tile_bytes;
    uint32_t off_slot[V_COUNT];
    uint32_t pad0;
    double *part;       // 2 slots of ntiles * kBatchWaves * kFields (one partial per wave)
    double *hist;       // history rows or nullptr
    double *chunk;      // nchunks > 1: 2 slots of nchunks * kFields chunk sums
    int32_t *chunks_done;  // nchunks > 1: chunk sums of the current transition written so far
    // CSR: the iteration pass's sliced-ELL copy (in place, or sorted for the
    // pass's 256 x kBatchEPT-row tiles when sell_perm is set; nullptr: CSR rows)
    const int32_t *sell_ptr;
    const int32_t *sell_col;
    const int32_t *sell_perm;
    const int2 *sell_win;   // sorted copy: per work tile, its column window
    const uint16_t *sell_c16;  // 16-bit columns (see PassArgs::sell_c16), or nullptr
    const float *sell_v32;     // binary32-stored values of a binary64 system (see PassArgs::sell_v32)
    const void *sell_val;
    int32_t hist_cap, replace_max, true_check, nchunks;
};

// Per-system scalars, advanced by the finalize kernel.
struct BatchState {
    int32_t phase, status, iter, i_start;
    int32_t wcur, restarts, passes, pad;
    double alpha, beta, gamma;  // alpha_i, beta_i, gamma_i of the iteration i the next ITER pass performs;
                                // after it, alpha and gamma serve as alpha_{i-1}, gamma_{i-1}
    double bnorm2, rho, true_res2;
    double alpha_prev;          // alpha_{i-1} while iterating (the catching-up pass's first x update)
    double pad2;
};

struct BatchTables {
    const BatchSys *sys;
    BatchState *st;          // 2 slots of max_sys states
    const int32_t *counts;   // [0] = items, [1] = listed systems, [2] = chunks
    const uint32_t *active;  // listed systems (split mode)
    const uint2 *items;      // (system, work tile) of each item, then (system, chunk) of each chunk
    int32_t max_sys;
    int32_t pad;
};

}  // namespace pcg
