// pcg_tune.hip -- launch-shape autotuner with an on-disk cache (pcg_tune*).
//
// Host code on top of the public entry points: every candidate shape runs a
// short probe (8 passes) that sizes its timed run to about 3 ms of passes
// (24 .. 4096), each a pcg_create + warm-up and timed pcg_solve on the
// caller's workspace; the timed solve's HIP-event time per iteration pass
// ranks the candidates.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <vector>

#include "pcg.h"

namespace pcg {
pcg_status invalid(const char *why);  // records the message for pcg_last_error
}
using pcg::invalid;

namespace {

struct Shape {
    int32_t variant, block, grid;
};

constexpr int kNumCU = 256;       // MI355X compute units
constexpr int kWarm = 8;               // passes of the probe that sizes the timed run
constexpr int kMinTimed = 24, kMaxTimed = 4096;
constexpr double kTimedUs = 3000.0;     // ~3 ms of timed passes per candidate

std::vector<Shape> candidates()
{
    std::vector<Shape> c;
    c.push_back({0, 0, 0});  // the library's built-in choice
    const int ept_bits[3] = {PCG_VAR_EPT1, 0, PCG_VAR_EPT4};
    for (int eb : ept_bits)
        for (int block : {128, 256})
            for (int per_cu : {1, 2, 4}) c.push_back({PCG_VAR_SET | PCG_VAR_NT | eb, block, per_cu * kNumCU});
    return c;
}

pcg_options shaped(const pcg_options &o, const Shape &s, int iters)
{
    pcg_options t = o;
    t.variant = s.variant;
    t.block_size = s.block;
    t.grid_blocks = s.grid;
    t.max_iter = iters;
    t.rtol = 1e-300;  // run the passes; convergence is not the point
    t.true_residual_check = 0;
    t.replace_max = 0;
    t.history_cap = 0;
    t.history = nullptr;
    t.timing = 1;
    t.use_graph = 1;
    t.iters_per_launch = iters + (iters & 1);
    return t;
}

std::string cache_key(const pcg_operator *op, const pcg_options *o)
{
    char buf[256];
    std::snprintf(buf, sizeof(buf), "k%d_n%lld_%dx%dx%d_nnz%lld_m%d_pc%d_p%d", op->kind, (long long)op->n,
                  op->kind == PCG_OP_CSR ? 0 : op->nx, op->kind == PCG_OP_CSR ? 0 : op->ny,
                  op->kind == PCG_OP_STENCIL3D7 ? op->nz : 1, op->kind == PCG_OP_CSR ? (long long)op->nnz : 0LL,
                  o->method, o->pc, o->prec);
    return buf;
}

bool cache_lookup(const std::string &key, Shape *s, double *us)
{
    const char *path = std::getenv("PCG_TUNE_CACHE");
    if (!path || !*path) return false;
    FILE *f = std::fopen(path, "r");
    if (!f) return false;
    char k[256];
    Shape t{};
    double u = 0.0;
    bool found = false;
    while (std::fscanf(f, "%255s %d %d %d %lf", k, &t.variant, &t.block, &t.grid, &u) == 5)
        if (key == k) {  // the last line for a key wins
            *s = t;
            *us = u;
            found = true;
        }
    std::fclose(f);
    return found;
}

void cache_store(const std::string &key, const Shape &s, double us)
{
    const char *path = std::getenv("PCG_TUNE_CACHE");
    if (!path || !*path) return;
    FILE *f = std::fopen(path, "a");
    if (!f) return;
    std::fprintf(f, "%s %d %d %d %.4f\n", key.c_str(), s.variant, s.block, s.grid, us);
    std::fclose(f);
}

}  // namespace

extern "C" pcg_status pcg_tune_workspace_size(const pcg_operator *op, const pcg_options *opt, size_t *bytes)
{
    if (!op || !opt || !bytes) return invalid("operator, options and bytes must be non-null");
    size_t most = 0;
    for (const Shape &s : candidates()) {
        const pcg_options t = shaped(*opt, s, kMaxTimed);
        size_t b = 0;
        const pcg_status st = pcg_workspace_size(op, &t, &b);
        if (st) return st;
        if (b > most) most = b;
    }
    *bytes = most;
    return PCG_OK;
}

extern "C" pcg_status pcg_tune(const pcg_operator *op, pcg_options *opt, void *workspace, size_t bytes,
                               const double *b, double *x, void *hip_stream, double *best_us)
{
    if (!op || !opt) return invalid("operator and options must be non-null");
    if (!b || !x || b == x) return invalid("b and scratch x must be non-null and distinct");
    size_t need = 0;
    pcg_status st = pcg_tune_workspace_size(op, opt, &need);
    if (st) return st;
    if (!workspace || ((uintptr_t)workspace % 256)) return invalid("workspace must be non-null and 256-byte aligned");
    if (bytes < need) return invalid("workspace smaller than pcg_tune_workspace_size");
    const std::string key = cache_key(op, opt);
    Shape best{};
    double best_t = 0.0;
    if (!cache_lookup(key, &best, &best_t)) {
        // one solve of `iters` passes from x = 0 after a warm-up solve (graph
        // capture, first touch); *us = time per working pass
        auto run = [&](const Shape &sh, int iters, double *us) -> pcg_status {
            const pcg_options t = shaped(*opt, sh, iters);
            pcg_solver sv = nullptr;
            pcg_status e = pcg_create(&sv, op, &t, workspace, bytes, hip_stream);
            if (e) return e;
            pcg_result r{};
            for (int rep = 0; rep < 2 && !e; ++rep) {
                if (hipMemsetAsync(x, 0, sizeof(double) * (size_t)op->n, (hipStream_t)hip_stream) != hipSuccess)
                    e = PCG_ERR_HIP;
                if (!e) e = pcg_solve(sv, b, x, &r);
            }
            pcg_destroy(sv);
            *us = r.iter_passes > 0 ? r.iter_kernel_ms * 1e3 / r.iter_passes : INFINITY;
            return e;
        };
        best_t = INFINITY;
        for (const Shape &sh : candidates()) {
            double probe = 0.0, us = 0.0;
            if ((st = run(sh, kWarm, &probe))) return st;
            if (!std::isfinite(probe)) continue;
            const int timed = (int)std::fmin(kMaxTimed, std::fmax(kMinTimed, std::ceil(kTimedUs / probe)));
            if ((st = run(sh, timed, &us))) return st;
            if (us < best_t) {
                best_t = us;
                best = sh;
            }
        }
        if (!std::isfinite(best_t)) return invalid("no candidate shape ran an iteration pass");
        cache_store(key, best, best_t);
    }
    opt->variant = best.variant;
    opt->block_size = best.block;
    opt->grid_blocks = best.grid;
    if (best_us) *best_us = best_t;
    return PCG_OK;
}
