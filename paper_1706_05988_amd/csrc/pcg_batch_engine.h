// pcg_batch_engine.h -- host side of the batched persistent pass: system
// slots, device tables, the captured graph of K passes and
// the step / poll cycle.  Used by pcg_batch_solve and by the server.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <vector>

#include "pcg_batch.h"

namespace pcg {

class BatchEngine {
public:
    // Byte layout of one system's device region (offsets from its start).
    struct SysLayout {
        size_t blk, part, chunk, chunks_done, dinv, hist, flag, gersh, bytes;
        // CSR: sliced-ELL copies (SIZE_MAX: none), see SellPlan
        size_t sell_ptr, sort_ptr, sort_perm, sort_win, sell_col, sell_val;
        int32_t nslices, sort_nslices;
        int64_t sell_cap;
        int32_t nchunks;  // chunks of kChunkParts partials (1: summed whole)
        uint32_t tile_bytes;
        int32_t ntiles;   // layout tiles (kBlk unknowns)
        int32_t nwork;    // work tiles of the pass (kBatchBlock * kBatchEPT unknowns)
        uint32_t off_slot[V_COUNT];
    };

    BatchEngine() = default;
    ~BatchEngine();
    BatchEngine(const BatchEngine &) = delete;
    BatchEngine &operator=(const BatchEngine &) = delete;

    static size_t table_bytes(int max_sys, int64_t max_items);
    static pcg_status system_layout(const pcg_operator *op, const pcg_options *opt, SysLayout *L);

    // tables: device memory of table_bytes(max_sys, max_items), 256-aligned.
    pcg_status init(char *tables, int max_sys, int64_t max_items, int prec, hipStream_t stream, int K);
    void set_pass_grid(int g) { pass_grid_ = g; }
    // Compile-time operator / preconditioner of the pass kernels (kind * 2 +
    // jac) when every system that will ever be admitted shares them, else
    // kSpecAny.  Set before the first step.
    void set_spec(int spec) { spec_ = spec; }
    pcg_status validate(const pcg_operator *op, const pcg_options *opt);
    // Admit a system whose device region (system_layout bytes) starts at
    // `region`; it joins the batch at the next step.  PCG_ERR_BUDGET when
    // every slot is taken.
    pcg_status admit(const pcg_operator *op, const pcg_options *opt, const double *b, double *x, char *region,
                     int *slot);
    void release(int slot);
    // One graph launch (K passes), then the per-system states are read back.
    pcg_status step(double *gpu_ms);
    bool done(int slot) const { return h_st_[slot].phase == PH_DONE; }
    void result(int slot, pcg_result *r) const;
    pcg_status copy_history(int slot, double *host, int cap);
    int active() const { return active_; }
    int64_t items() const { return items_; }
    int launches() const { return launches_; }

private:
    pcg_status upload_tables();
    pcg_status ensure_graph(int split);
    void enqueue_passes(hipStream_t st, int split);
    int default_pass_grid(int split) const;

    int max_sys_ = 0;
    int64_t max_items_ = 0;
    int prec_ = 0;
    int K_ = 8;
    int pass_grid_ = 0;      // persistent blocks of the pass; 0: default_pass_grid()
    int trans_grid_ = 256;   // blocks of the transition kernel (set by init)
    int chunk_grid_ = 256;
    int spec_ = kSpecAny;
    // above this many items a launch runs split (measured: the fused head
    // costs ~100 us per pass on a full 512-system batch, the extra kernel ~5 us)
    int64_t split_items_ = 4096;
    // ... and when a listed system has more items than this: in a fused pass
    // every item block of a system runs stage 2 over all of that system's
    // partials, so that head's reads grow with the square of its item count
    // (a 4M-unknown system: ~3900 items, ~1.5 GB of partial reads per pass)
    int fused_sys_items_ = 64;
    int max_sys_items_ = 0;  // most items of one listed system
    hipStream_t stream_ = nullptr;
    BatchSys *d_sys_ = nullptr;
    BatchState *d_st_ = nullptr;
    char *d_list_ = nullptr;      // counts, listed systems, (system, tile) items
    std::vector<BatchSys> sys_;
    std::vector<char> in_use_;
    std::vector<char> listed_;   // the system's items are in the device tables
    BatchState *h_st_ = nullptr;  // pinned: admission staging and read-back
    char *h_list_ = nullptr;      // pinned: staging of the work list
    bool tables_dirty_ = true;
    bool slots_dirty_ = true;     // a slot was admitted or released since the last upload
    int64_t items_ = 0;
    int64_t chunks_ = 0;          // (system, chunk) entries of the large systems
    int active_ = 0;
    int launches_ = 0;
    // [0]: fused passes (few items), [1]: transition + pass (many items),
    // [2]: chunk sums with the transition + pass (a system above kChunkParts
    // partials)
    hipGraph_t graph_[3] = {nullptr, nullptr, nullptr};
    hipGraphExec_t gexec_[3] = {nullptr, nullptr, nullptr};
    hipEvent_t ev0_ = nullptr, ev1_ = nullptr;
    hipEvent_t ev_up_ = nullptr;  // after the last upload from the staging buffers
};

}  // namespace pcg
