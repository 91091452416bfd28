// pcg_batch.h -- many independent solves advanced by one persistent pass.
//
// Every active system moves one phase or one iteration per pass:
//   COPYIN  caller x -> internal (blocked) x
//   INIT0   r_0 := b - A x_0, u_0 := M^-1 r_0, z = q = s = t = p := 0; (b, b)
//   INIT1   w_0 := A u_0 - sigma r_0; gamma_0, delta_0, rho_0
//   ITER    one iteration of shifted pipelined CG (Alg. 3)
//   RESID   ||b - A x|| in binary64 (after the iteration ends)
//   COPYOUT internal x -> caller x
// The pass kernel works on a table of (system, tile) items; each tile is
// 512 unknowns (256 threads x 2) and writes one block partial into its
// system's partial array.  The finalize kernel that follows each pass sums
// each system's partials in tile order (so a system's results depend only on
// that system, never on the rest of the batch), takes the stop / breakdown /
// restart decisions and the scalar recurrences, and moves the system to its
// next phase.  Kernel boundaries order the two, so no atomics or fences are
// needed across the XCDs.
#pragma once

#include "pcg_internal.h"
#include "pcg_kernels.h"

namespace pcg {

enum Phase : int32_t {
    PH_COPYIN = 0, PH_INIT0, PH_INIT1, PH_ITER, PH_RESID, PH_COPYOUT, PH_DONE, PH_FREE
};

constexpr int kBatchBlock = 256;      // threads of a pass block: one 512-unknown tile
constexpr int kBatchEPT = 2;

// Per-system descriptor, written once at admission.
struct BatchSys {
    int32_t kind, jac, n, ntiles;
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
    double *part;       // ntiles * kFields
    double *hist;       // history rows or nullptr
    int32_t hist_cap, replace_max, true_check, pad1;
};

// Per-system scalars, advanced by the finalize kernel.
struct BatchState {
    int32_t phase, status, iter, i_start;
    int32_t wcur, restarts, passes, pad;
    double alpha, beta, gamma;  // alpha_i, beta_i, gamma_i of the iteration i the next ITER pass performs;
                                // after it, alpha and gamma serve as alpha_{i-1}, gamma_{i-1}
    double bnorm2, rho, true_res2;
};

struct BatchTables {
    const BatchSys *sys;
    BatchState *st;
    const uint32_t *item_sys;
    const uint32_t *item_tile;
    const uint32_t *active;
    const int32_t *counts;  // [0] = items, [1] = active systems
};

}  // namespace pcg
