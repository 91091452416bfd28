/*
 * pcg.h -- C ABI of libpcg, a shifted pipelined Conjugate Gradients library
 * for one AMD Instinct MI355X (gfx950).
 *
 * The library solves A x = b for a real symmetric positive definite n-by-n
 * operator A (Section 2.1 of Cools & Vanroose, "Numerically stable variants
 * of the communication-hiding pipelined Conjugate Gradients algorithm") with
 *   - classic preconditioned CG ........................ Alg. 1  (PCG_CG)
 *   - preconditioned pipelined CG ...................... Alg. 2  (PCG_PIPE)
 *   - shifted preconditioned pipelined CG .............. Alg. 3  (PCG_PIPE_SHIFT)
 *   - the same with an iteration-dependent shift ........ Alg. 4  (PCG_PIPE_VAR_SHIFT,
 *     Section 4.1: sigma_i from a caller-given schedule; the corrections
 *     (sigma_i - sigma_{i-1}) t_i, p_i, (s_i + sigma_i t_i), r_i of s, q, z
 *     and w ride in the same fused pass with no extra vector traffic)
 *   - Alg. 2 with automated residual replacement ....... p-CG-rr (PCG_PIPE_RR,
 *     Section 5.2): every rr_period iterations one pass measures the gap
 *     f_i = (b - A x_i) - r_i in binary64; when ||f_i|| exceeds rr_tau ||r_i||
 *     and rr_floor times the rounding scale 2^-53 || |A||x_i| + |b| || of that
 *     explicit residual, two passes reset r, u, w, s, q, z to their true
 *     values (r = b - A x_i, u = M^-1 r, w = A u, s = A p_{i-1},
 *     q = M^-1 s, z = A q) and iteration i restarts from the reset vectors'
 *     dot products while beta continues the old recurrence.  The criterion
 *     is this library's own (the paper cites it from elsewhere); all of it
 *     runs inside the K-pass graph, with no host round trip.
 * Alg. 3 with sigma = 0 is Alg. 2 (end of Section 2.2); both run the same
 * fused kernel.  Each pipelined iteration is ONE device pass: the
 * preconditioner apply and SPMV (m_i = M^-1 w_i, n_i = A m_i), the five
 * beta-recurrences (z, q, s, t, p), the four alpha-recurrences including the
 * shift terms (x, r, u, w), and the local parts of the next iteration's dot
 * products gamma = (r, u), delta = (w + sigma r, u) and rho = (r, r).  The
 * global part of the reduction is summed in a fixed order at the head of the
 * next pass, overlapping that pass's SPMV loads -- the single-GPU form of the
 * paper's overlap of the global reduction with the SPMV (Section 1).
 *
 * Conventions for every entry point
 *   - All calls return a pcg_status: PCG_OK (0), PCG_PENDING (1, polling
 *     only) or a negative error.  No C++ exception crosses the ABI.
 *   - Device pointers are HIP device addresses (e.g. torch tensors' data_ptr).
 *     The library never allocates device memory: the caller provides a
 *     workspace of at least pcg_workspace_size() bytes (256-byte aligned).
 *     The one exception is the fixed static scratch of pcg_solve_static.
 *   - All device work is issued on the caller's HIP stream (hipStream_t passed
 *     as void*, NULL = the legacy default stream), stream-ordered with the
 *     caller's own work.  pcg_solve() returns after the solve has completed.
 *   - x and b are always binary64 vectors of length n.  In PCG_FP32_STREAM
 *     form the Krylov vectors (r, u, w, z, q, s, t, p), the CSR values and the
 *     Jacobi diagonal are stored in binary32; all arithmetic, dot products,
 *     scalar recurrences, the explicit residual and x stay binary64.
 *   - Handles are not thread-safe: one thread at a time per pcg_solver.
 */
#ifndef PCG_H
#define PCG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ------------------------------------------------------------------ status */

typedef int32_t pcg_status;

#define PCG_OK              0
#define PCG_PENDING         1   /* pcg_poll(): the ticket has not finished       */
#define PCG_ERR_INVALID   (-1)  /* bad argument (null, size, layout, alignment)  */
#define PCG_ERR_NONFINITE (-2)  /* b holds NaN or Inf                             */
#define PCG_ERR_HIP       (-3)  /* a HIP runtime call failed (see pcg_last_error) */
#define PCG_ERR_BUDGET    (-4)  /* a request can never fit the server's memory    */
#define PCG_ERR_STATE     (-5)  /* unknown ticket / handle used in a wrong state  */

/* outcome of a solve, in pcg_result.status */
#define PCG_CONVERGED  0   /* recursive (and, if checked, explicit) residual <= rtol */
#define PCG_MAX_ITER   1   /* iteration cap reached                                 */
#define PCG_BREAKDOWN  2   /* gamma <= 0, delta <= 0, (s,p) <= 0 or alpha not > 0     */
#define PCG_NONFINITE  3   /* a reduction produced NaN / Inf                         */

typedef enum { PCG_CG = 0, PCG_PIPE = 1, PCG_PIPE_SHIFT = 2, PCG_PIPE_VAR_SHIFT = 3, PCG_PIPE_RR = 4 } pcg_method;
typedef enum { PCG_OP_STENCIL2D5 = 0, PCG_OP_STENCIL3D7 = 1, PCG_OP_CSR = 2 } pcg_op_kind;
typedef enum { PCG_PC_NONE = 0, PCG_PC_JACOBI = 1 } pcg_pc_kind;
typedef enum { PCG_FP64 = 0, PCG_FP32_STREAM = 1 } pcg_precision;

/* ---------------------------------------------------------------- operator */

/*
 * The SPD operator A (Section 2.1: a real SPD n-by-n matrix).
 *
 * Stencils (matrix-free): the second-order finite-difference Laplacian on the
 * interior points of an nx-by-ny(-by-nz) grid with homogeneous Dirichlet
 * boundaries, lexicographic order with x fastest: row k holds (diag + shift)
 * on the diagonal and `offdiag` for each existing grid neighbour (4 in 2-D,
 * 6 in 3-D).  The unscaled Laplacian is diag = 4 (2-D) / 6 (3-D),
 * offdiag = -1; shift adds c I.  n must equal nx*ny (2-D) or nx*ny*nz (3-D).
 *
 * CSR: n rows; row_ptr (n + 1 int32, row_ptr[0] = 0, row_ptr[n] = nnz),
 * col_idx (nnz int32 in [0, n)), vals (nnz values: double in PCG_FP64 form,
 * float in PCG_FP32_STREAM form); all device memory, borrowed until
 * pcg_destroy().  Each row must hold its diagonal entry when the Jacobi
 * preconditioner is used.  n and nnz must be < 2^31.
 */
typedef struct {
    int32_t kind;               /* pcg_op_kind                                    */
    int32_t nx, ny, nz;         /* stencil grid (nz = 1 for 2-D)                  */
    int64_t n;                  /* number of unknowns                             */
    double diag, offdiag, shift;/* stencil coefficients                           */
    const int32_t *row_ptr;     /* CSR, device                                    */
    const int32_t *col_idx;     /* CSR, device                                    */
    const void *vals;           /* CSR, device, double or float per precision     */
    int64_t nnz;                /* CSR                                            */
} pcg_operator;

/* ----------------------------------------------------------------- options */

#define PCG_HISTORY_FIELDS 5    /* per iteration: sqrt(rho_i)/||b||, alpha_i, beta_i, gamma_i, delta_i */

typedef struct {
    int32_t method;             /* pcg_method                                              */
    int32_t pc;                 /* pcg_pc_kind; Jacobi: M = diag(A), m = (1/a_kk) w         */
    int32_t prec;               /* pcg_precision                                           */
    int32_t max_iter;           /* iteration cap (>= 0)                                    */
    double sigma;               /* shift of Alg. 3 (>= 0); NaN: midpoint of the spectrum
                                   bounds of A M^-1 (closed form for stencils, Gershgorin
                                   for CSR); ignored by PCG_CG and PCG_PIPE                 */
    double rtol;                /* stop at the top of iteration i when
                                   sqrt((r_i, r_i)) <= rtol ||b||  (> 0)                  */
    int32_t true_residual_check;/* 1: at a claim of convergence also compute
                                   ||b - A x|| / ||b|| in binary64 and, if it exceeds rtol,
                                   restart from x (below)                                   */
    int32_t replace_max;        /* max restarts from x ("residual replacement": the
                                   initialisation is re-run with x_0 := x_i while the
                                   iteration count continues); 0 = none                     */
    int32_t iters_per_launch;   /* K: iteration passes per HIP graph launch (even, >= 2);
                                   0 = library default                                       */
    int32_t history_cap;        /* rows of `history` (0 = no history)                       */
    double *history;            /* HOST buffer of history_cap * PCG_HISTORY_FIELDS doubles,
                                   row i = iteration i (NaN for alpha.. when not computed);
                                   filled when pcg_solve returns                            */
    int32_t block_size;         /* threads per block (64..256, multiple of 64); 0 = tuned    */
    int32_t grid_blocks;        /* blocks of the persistent grid; 0 = tuned                 */
    int32_t timing;             /* 1: time the iteration graph launches with HIP events     */
    int32_t use_graph;          /* 1: capture the K passes of a launch in a HIP graph
                                   (pcg_default_options' choice); 0: launch them one by one  */
    int32_t variant;            /* 0: the tuned kernel variant; else PCG_VAR_SET | bits below */
    int32_t sigma_schedule_len; /* PCG_PIPE_VAR_SHIFT: entries of sigma_schedule, 1 .. 2^24    */
    int32_t rr_period;          /* PCG_PIPE_RR: gap check every rr_period iterations (0: 8)  */
    int32_t flags;              /* PCG_FLAG_* bits below (0: none)                          */
    const double *sigma_schedule; /* PCG_PIPE_VAR_SHIFT: HOST array sigma_{-1}, sigma_0,
                                   sigma_1, ... (each finite, >= 0); entry k + 1 is the shift
                                   of iteration k and the last entry repeats past the end.
                                   w_i is kept equal to A u_i - sigma_{i-1} r_i (w_0 uses
                                   sigma_{-1}).  Copied at pcg_create; ignored by the other
                                   methods.  The batch and server entry points reject this
                                   method.                                                   */
    double rr_tau;              /* PCG_PIPE_RR: relative gap threshold; NaN or <= 0: the cube
                                   root of the storage unit roundoff (binary64 4.8e-6,
                                   binary32 3.9e-3)                                          */
    double rr_floor;            /* PCG_PIPE_RR: gap must also exceed rr_floor times the
                                   rounding scale of b - A x; NaN or <= 0: 100               */
} pcg_options;

/* Option flags (pcg_options.flags).
 * PCG_FLAG_RUN_THROUGH_BREAKDOWN: pcg_solve and pcg_solve_static do not stop
 * at a breakdown (gamma <= 0, delta <= 0, (s, p) <= 0, or an alpha that is
 * not finite and positive) but run on to the stop test or the iteration
 * cap, as the accuracy runs of Section 5.1 do (Table 1 reports p-CG after a
 * fixed number of iterations); non-finite dot products still end the solve.
 * The batch and server entry points reject the flag. */
#define PCG_FLAG_RUN_THROUGH_BREAKDOWN 0x01

/* Kernel variant bits (pcg_options.variant).  Every variant performs the same
 * per-unknown arithmetic; they differ in how unknowns map to threads, so the
 * order in which dot-product partials are accumulated (and hence the last
 * bits of gamma, delta, rho) may differ between variants.  Each variant is
 * deterministic run to run. */
#define PCG_VAR_SET      0x01   /* use the bits below instead of the tuned default      */
#define PCG_VAR_XCD_MAP  0x02   /* tiles in 8 contiguous slabs, one per XCD             */
#define PCG_VAR_NT       0x04   /* non-temporal hint on the once-touched streams        */
#define PCG_VAR_EPT1     0x10   /* 1 unknown per thread per tile (default 2)            */
#define PCG_VAR_EPT4     0x20   /* 4 unknowns per thread per tile                       */
#define PCG_VAR_CG_ZMARCH 0x40  /* PCG_CG, 3-D stencil: pass A marches along z through
                                   LDS also where the built-in rule would not (grids
                                   with fewer work items than CUs)                      */
#define PCG_VAR_CSR_SELL 0x80   /* CSR: the passes of every method (iteration, set-up,
                                   explicit residual, PCG_PIPE_RR's gap check and
                                   replacement) read a sliced-ELL copy of the operator
                                   (64-row slices, built at pcg_create when its padding
                                   stays within a quarter of nnz; the same sums in the
                                   same order)                                          */
#define PCG_VAR_CSR_SELL_SORTED 0x100 /* as PCG_VAR_CSR_SELL, with the rows sorted by
                                   length (longest first) within each wave's rows of a
                                   tile (SELL-C-sigma, C = 64) so that rows of mixed
                                   lengths pad little; each row's sum is unchanged.  With
                                   both bits the smaller copy is kept.  Without
                                   PCG_VAR_SET both are tried, the sorted copy with 4
                                   unknowns per thread (the passes then take that shape) */

typedef struct {
    int32_t status;             /* PCG_CONVERGED .. PCG_NONFINITE                         */
    int32_t iterations;         /* i at exit (x = x_i)                                    */
    int32_t replacements;       /* restarts from x                                        */
    int32_t launches;           /* graph (or single-pass) launches issued                 */
    double rel_res_recursive;   /* sqrt((r_i, r_i)) / ||b||                              */
    double rel_res_true;        /* ||b - A x_i|| / ||b|| in binary64 (NaN if not computed) */
    double seconds;             /* host wall time of pcg_solve                            */
    double iter_kernel_ms;      /* HIP-event time of the iteration launches (timing = 1)  */
    int32_t iter_passes;        /* iteration passes that did work (iterations of all methods;
                                   CG counts 2 passes per iteration)                       */
    int32_t admitted_at;        /* server: launches the server had issued when the request
                                   joined the batch (it was resident for `launches`
                                   launches from there); 0 for the other entry points      */
    double sigma;               /* the shift actually used                                */
} pcg_result;

/* Fill *opt with defaults: PCG_PIPE_SHIFT, no PC, FP64, max_iter 1000,
 * sigma NaN (midpoint), rtol 1e-10, true-residual check on, 4 restarts,
 * library-chosen launch shape, HIP graphs on. */
pcg_status pcg_default_options(pcg_options *opt);

/* -------------------------------------------------------------- one solver */

typedef struct pcg_solver_ *pcg_solver;

/* Bytes of device workspace a solver for (op, opt) needs. */
pcg_status pcg_workspace_size(const pcg_operator *op, const pcg_options *opt, size_t *bytes);

/*
 * Create a solver bound to op, opt, a device workspace (>= the size above,
 * 256-byte aligned, owned by the caller, borrowed until pcg_destroy) and a
 * HIP stream.  Validates all arguments (PCG_ERR_INVALID), sets up the Jacobi
 * diagonal for CSR operators on the stream, and captures the iteration graph.
 */
pcg_status pcg_create(pcg_solver *solver, const pcg_operator *op, const pcg_options *opt,
                      void *workspace, size_t bytes, void *hip_stream);

/*
 * Solve A x = b.  b: device, n binary64 (read only).  x: device, n binary64,
 * x_0 on entry and the final iterate on return (overwritten in place; it must
 * not alias b).  Blocks the calling host thread until done.  Returns
 * PCG_ERR_NONFINITE (x untouched beyond x_0) when ||b|| is not finite.
 */
pcg_status pcg_solve(pcg_solver solver, const double *b, double *x, pcg_result *result);

/* ||b - A x|| / ||b|| in binary64 for the solver's operator (Section 3.1's
 * explicit residual); device b, x; host *rel. */
pcg_status pcg_true_residual(pcg_solver solver, const double *b, const double *x, double *rel);

pcg_status pcg_destroy(pcg_solver solver);

/* What a solver runs: its passes' launch shape and the form in which the
 * fused pass reads a CSR operator (decided at pcg_create; a sorted
 * sliced-ELL copy brings its own shape).  Errors: PCG_ERR_INVALID for a
 * null argument. */
typedef struct {
    int32_t block;              /* threads per block                                      */
    int32_t ept;                /* unknowns per thread per tile                            */
    int32_t grid;               /* persistent blocks                                       */
    int32_t ntiles;             /* tiles of block x ept unknowns                           */
    int32_t iters_per_launch;   /* iterations per graph launch                            */
    int32_t csr_form;           /* 0: CSR arrays (or a stencil), 1: sliced-ELL copy with
                                   the rows in place, 2: sorted sliced-ELL copy           */
    int32_t csr_col_bits;       /* the copy's column words: 32, or 16 when every tile of
                                   a sorted copy gathers from an LDS window of at most
                                   2048 columns (offsets in that window) or every entry
                                   of an in-place copy lies within 2^15 of its row
                                   (offsets from the row); 0 if no copy                   */
    int32_t csr_val_bits;       /* the copy's values: 64, or 32 (FP32-stream form, or a
                                   binary64 operator whose values are all binary32 numbers:
                                   stored as binary32, exactly); 0 if no copy            */
    int64_t csr_entries;        /* entries of that copy, padding included (0 if none)     */
} pcg_solver_shape;
pcg_status pcg_solver_info(pcg_solver solver, pcg_solver_shape *shape);

/* ------------------------------------------------- solve without allocation */

/* Size of the device scratch behind pcg_solve_static, per device. */
#define PCG_STATIC_SCRATCH_BYTES ((size_t)64 << 20)

/*
 * For callers that cannot allocate memory (code under HIP graph capture,
 * tight serving loops, harnesses that forbid hipMalloc): the same solve as
 * pcg_create + pcg_solve + pcg_destroy, with the workspace taken from a
 * static device array of PCG_STATIC_SCRATCH_BYTES inside the library instead
 * of caller memory.  It calls no hipMalloc, hipFree, hipHostMalloc, event or
 * graph creation: the iteration passes are launched one by one on the
 * caller's stream and the status is read back into ordinary host memory
 * after each launch of K passes.  Same kernels, launch shape and results as
 * pcg_solve with opt->use_graph = 0; opt->timing is ignored (iter_kernel_ms
 * is 0).  op, opt, b, x, result: as for pcg_create and pcg_solve.  Blocks
 * the calling thread until the solve is done.
 * Limit: a solve whose pcg_workspace_size() exceeds PCG_STATIC_SCRATCH_BYTES
 * is rejected with PCG_ERR_INVALID (pcg_last_error states both sizes); e.g.
 * binary64 Jacobi p-CG-sh holds about 80 bytes per unknown, so n up to
 * about 800,000.
 * Sharing: each device has ONE scratch array, which keeps the contents of
 * the last call.  Calls from threads of one process on the same device are
 * serialised by a lock inside the library; anything else that overlapped
 * two solves on one device's scratch would race.
 */
pcg_status pcg_solve_static(const pcg_operator *op, const pcg_options *opt, const double *b, double *x,
                            pcg_result *result, void *hip_stream);

/* -------------------------------------------------------------- autotuner */

/*
 * Launch-shape autotuner.  The fused pass is bound by memory latency and
 * bandwidth, and how many unknowns each thread handles (1, 2 or 4), the
 * block size (128 or 256) and the number of resident blocks per CU (1, 2 or
 * 4; 8 for 128-thread blocks) decide how many independent loads are in
 * flight; for a CSR operator each shape is also tried on the sliced-ELL
 * copies (PCG_VAR_CSR_SELL, and with 2 or 4
 * unknowns per thread PCG_VAR_CSR_SELL_SORTED).  The best choice
 * depends on the operator, the method, the preconditioner and the storage
 * form.  pcg_tune measures every candidate (and the library's built-in
 * choice) on the caller's operator -- a solver is created on `workspace`
 * for each; an 8-pass probe sizes a run of about 3 ms of passes (24 to
 * 4096) from a zero initial guess, timed with HIP events -- and writes the
 * fastest (the built-in choice unless another shape is 1% faster) into
 * opt->variant (PCG_VAR_SET | unknowns-per-thread bits | PCG_VAR_NT
 * [| PCG_VAR_CSR_SELL | PCG_VAR_CSR_SELL_SORTED]),
 * opt->block_size and opt->grid_blocks; *best_us (host, may be NULL)
 * receives its time per pass.  b: device right-hand side (n binary64);
 * x: device scratch of n binary64, overwritten.  workspace: at least
 * pcg_tune_workspace_size() bytes, 256-byte aligned.
 * When the environment variable PCG_TUNE_CACHE names a file, results are
 * looked up there first (key: operator kind and sizes, nnz, method,
 * preconditioner, precision) and new ones appended, one line per key, so a
 * later process skips the measurement.  Errors: PCG_ERR_INVALID as for
 * pcg_create; PCG_ERR_HIP from the device.  opt is changed only on success.
 */
pcg_status pcg_tune_workspace_size(const pcg_operator *op, const pcg_options *opt, size_t *bytes);
pcg_status pcg_tune(const pcg_operator *op, pcg_options *opt, void *workspace, size_t bytes, const double *b,
                    double *x, void *hip_stream, double *best_us);

/* ------------------------------------------------------------ batched solve */

/*
 * Solve `count` independent systems A_k x_k = b_k in ONE persistent pass per
 * iteration (every active system advances one phase or iteration per pass).
 * ops[k], opts[k]: per-system operator and options.  All systems must share
 * the precision and use PCG_PIPE or PCG_PIPE_SHIFT; operator kind and
 * preconditioner may differ (a batch whose systems all share them runs pass
 * kernels compiled for that pair).  The launch shape comes from opts[0]:
 * grid_blocks (0: as many blocks as the pass kernels keep resident, at most
 * 4 per CU) and iters_per_launch (0: 32).  b[k], x[k]: host arrays of device
 * pointers.  Per-system results in results[k].  Each system's arithmetic --
 * tiling, reduction order -- depends only on that system, so its result does
 * not depend on what else is in the batch nor on the launch shape.
 */
pcg_status pcg_batch_workspace_size(int32_t count, const pcg_operator *ops, const pcg_options *opts,
                                    size_t *bytes);
pcg_status pcg_batch_solve(int32_t count, const pcg_operator *ops, const pcg_options *opts,
                           const double *const *b, double *const *x, pcg_result *results,
                           void *workspace, size_t bytes, void *hip_stream);

/*
 * Launch-shape autotuner of the batched pass.  Times complete pcg_batch_solve
 * calls on the caller's batch for the library's default shape (grid_blocks
 * and iters_per_launch 0) and for every persistent grid of 1, 2, 3 or 4
 * blocks per CU with every graph length K of 16, 32 or 64 passes (each
 * candidate twice, its faster host wall time counting; a shape other than
 * the default must beat it by 1%), and writes the winner into
 * opts[0].grid_blocks and opts[0].iters_per_launch; *best_ms
 * (host, may be NULL) receives its solve time.  x0[k]: device initial guesses
 * (n_k binary64, read only), copied into x[k] before every candidate solve;
 * x[k]: device scratch, overwritten (it holds a solution on return).
 * workspace, bytes, hip_stream: as for pcg_batch_solve.  With PCG_TUNE_CACHE
 * naming a file, the result is looked up there first (key: precision, count
 * and a hash of every system's operator kind, sizes, nnz, preconditioner and
 * method) and a new one appended.  Errors: PCG_ERR_INVALID for null or
 * aliased pointers and a short workspace, otherwise as pcg_batch_solve.
 * opts is changed only on success.
 */
pcg_status pcg_batch_tune(int32_t count, const pcg_operator *ops, pcg_options *opts, const double *const *b,
                          const double *const *x0, double *const *x, void *workspace, size_t bytes,
                          void *hip_stream, double *best_ms);

/* ---------------------------------------------------------------- serving */

typedef struct pcg_server_ *pcg_server;

/*
 * A continuously batching solve server.  `arena` (device, `arena_bytes`,
 * owned by the caller) is the HBM budget from which the server sub-allocates
 * each admitted request's Krylov vectors; requests wait until their footprint
 * and a slot (max_slots) are free, and join the running batch at the next
 * launch boundary.  A scheduler thread owned by the server drives the device.
 * Every request must use the precision of the first one, whose options also
 * fix the launch shape of the whole run: grid_blocks (0: the pass kernels'
 * resident blocks, at most 4 per CU) and iters_per_launch (0: 32), e.g. as
 * pcg_batch_tune chose them on a sample of the expected requests.
 */
pcg_status pcg_server_create(pcg_server *server, void *arena, size_t arena_bytes, int32_t max_slots,
                             void *hip_stream);
/* Enqueue a solve; op, b, x device data stay borrowed until the ticket is
 * done.  opt->prec must be the first request's; opt->method must be PCG_PIPE
 * or PCG_PIPE_SHIFT; operator kind and preconditioner may differ between
 * requests.  Errors: PCG_ERR_INVALID (bad arguments, another precision or
 * method), PCG_ERR_BUDGET (the request alone exceeds the arena),
 * PCG_ERR_STATE (null or closing server).  A request that fails while it
 * runs (non-finite right-hand side, breakdown) reports that in its result's
 * status and pcg_wait / pcg_poll return PCG_OK; the other requests are
 * unaffected.  A HIP error during a launch fails every running request:
 * their pcg_wait / pcg_poll return that error; the server drains its stream,
 * takes back their slots and arena ranges and goes on with the queue. */
pcg_status pcg_submit(pcg_server server, const pcg_operator *op, const pcg_options *opt,
                      const double *b, double *x, uint64_t *ticket);
pcg_status pcg_poll(pcg_server server, uint64_t ticket, pcg_result *result);   /* PCG_PENDING until done */
pcg_status pcg_wait(pcg_server server, uint64_t ticket, pcg_result *result);

/* Counters of a server (a snapshot under the server's lock). */
typedef struct {
    int64_t submitted;          /* tickets issued                                          */
    int64_t completed;          /* requests finished (PCG_OK from pcg_wait / pcg_poll)      */
    int64_t failed;             /* requests that failed (admission or launch errors)        */
    int32_t queued;             /* waiting for a slot or arena space                        */
    int32_t running;            /* resident on the device now                               */
    int32_t max_running;        /* most requests resident in one launch so far              */
    int32_t launches;           /* launches of K passes issued                              */
    size_t arena_bytes;         /* arena bytes available to requests (after the tables)     */
    size_t arena_free;          /* of which free now                                        */
    size_t arena_largest_free;  /* largest free contiguous range                            */
} pcg_server_stats;

pcg_status pcg_server_info(pcg_server server, pcg_server_stats *stats);

/* A server whose process environment sets PCG_SERVER_FAIL_AT_LAUNCH=k at
 * pcg_server_create fails its k-th launch (counted from 0) without issuing
 * any device work, as a HIP error would: a test hook for the failure path,
 * whose requests get PCG_ERR_HIP while their slots and arena ranges return
 * to the server. */
pcg_status pcg_server_destroy(pcg_server server);

/* ------------------------------------------------------- shift selection */

/*
 * Rounding-error amplification of pipelined CG (Section 3.2) and the
 * a-posteriori choice of the shift (Section 5.1).  Host functions: every
 * pointer is a HOST array; nothing touches the device.
 *
 * alpha[k], beta[k] (k = 0 .. i) are iteration k's coefficients, as a solve
 * records them in columns 1 and 2 of pcg_options.history (a p-CG run,
 * PCG_PIPE, is the one Section 5.1 analyses).  The local rounding errors of
 * iteration j reach iteration i through P_i ... P_j, with the 4x4 local
 * propagation matrix
 *     P_k = [ 1   -a b        -a        0   ]
 *           [ 0    b           1        0   ]   a = alpha_k, b = beta_k,
 *           [ 0   -a b s'      1 - a s' -a b]   s' = sigma_{k-1}, s = sigma_k,
 *           [ 0   -b (s - s') -(s - s')  b  ]
 * of Section 4.2 (with s' = s it is P_k(sigma) of Section 3.2), and
 *     psi_i = max over 1 <= j <= i of || P_i ... P_j ||_2 .
 * Errors: PCG_ERR_INVALID for null pointers, i < 1, a non-finite alpha_k or
 * beta_k (1 <= k <= i), or a non-finite shift.
 */
/* psi_i(sigma) for a constant shift. */
pcg_status pcg_psi(const double *alpha, const double *beta, int32_t i, double sigma, double *psi);
/* psi_i for a shift schedule sigma_{-1}, sigma_0, ... (the layout of
 * pcg_options.sigma_schedule; the last entry repeats). */
pcg_status pcg_psi_variable(const double *alpha, const double *beta, int32_t i, const double *sigma_schedule,
                            int32_t sigma_schedule_len, double *psi);
/* psi_i on a grid of grid_len shifts (written to psi_out unless NULL) and the
 * chosen shift: the smallest grid shift whose psi_i is at most `slack` (>= 1)
 * times the grid minimum.  psi_i falls slowly towards the top of the
 * spectrum and explodes there, and Section 5.1 warns that a too large shift
 * may destroy convergence, so the smallest near-minimal shift is taken;
 * slack = 1 is the plain argmin (ties to the smaller shift). */
pcg_status pcg_select_shift(const double *alpha, const double *beta, int32_t i, const double *grid,
                            int32_t grid_len, double slack, double *psi_out, double *sigma_best);

/* --------------------------------------------------------- measurement */

/*
 * Streaming-bandwidth probe: the ceiling the fused iteration passes, whose
 * bound is HBM bandwidth, are compared with.  One launch streams nin input
 * and nout output vectors of n binary64 values with the fused passes'
 * tiling (a persistent grid of four 256-thread blocks per CU, 4 values per
 * thread per tile, every load of a tile issued before its stores); output j
 * receives in_j + c_j * (sum of the inputs).  flags: PCG_PROBE_NT puts the
 * non-temporal hint on every access; PCG_PROBE_BLOCKED lays the streams out
 * as the solver's workspace does (512-value tiles of every stream one after
 * another) instead of one vector after another; PCG_PROBE_FP32 streams
 * binary32 values instead of binary64 (bytes moved per launch then
 * (nin + nout) * 4 n); PCG_PROBE_WIDE gives each lane 16-byte accesses
 * (4 binary32 or 2 binary64 consecutive values; plain vectors only, n a
 * multiple of that count); PCG_PROBE_BLOCKS_PER_CU(k), k in 1..15, sets the
 * persistent grid to k blocks per CU instead of 4.
 * Supported mixes: nout = 0 with nin in {1, 2, 4, 8, 9, 16} (read only; each
 * block writes one sum to a sink), and (nin, nout) in {(1, 1), (2, 1),
 * (4, 4), (5, 4), (8, 8), (9, 8), (9, 9)}.
 * buffer: device, 256-byte aligned, at least (nin + nout) * round_up(8 n,
 * 4096) + 65536 bytes (the streams, then the sink); its contents are read
 * and overwritten.  One warm-up launch, then `reps` launches between two HIP
 * events on hip_stream; *us_per_launch (host) receives their average
 * duration.  Bytes moved per launch: (nin + nout) * 8 n (binary64).  Errors:
 * PCG_ERR_INVALID (sizes, mix, flags, buffer), PCG_ERR_HIP.
 */
#define PCG_PROBE_NT      1
#define PCG_PROBE_BLOCKED 2
#define PCG_PROBE_FP32    4
#define PCG_PROBE_WIDE    8
#define PCG_PROBE_BLOCKS_PER_CU(k) ((int32_t)(k) << 8)
pcg_status pcg_stream_probe(int32_t nin, int32_t nout, int32_t flags, int64_t n, void *buffer, size_t bytes,
                            int32_t reps, void *hip_stream, double *us_per_launch);

/* ------------------------------------------------------------------ misc */

const char *pcg_status_str(pcg_status status);
/* Text of the last HIP error seen by this thread (empty if none). */
const char *pcg_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* PCG_H */
