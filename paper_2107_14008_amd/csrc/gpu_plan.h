// Device buffers of a context and the on-GPU planner (ORB tree, dual walk,
// TaskGroup CSR and work items built from particles already in HBM).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <functional>
#include <string>
#include <utility>
#include <vector>

#include "device.h"
#include "plan.h"

namespace pmfmm {

struct DevBuf {
    void* p = nullptr;
    size_t bytes = 0;
    hipError_t ensure(size_t want) {
        if (want <= bytes && p != nullptr) return hipSuccess;
        if (p) (void)hipFree(p);
        p = nullptr;
        bytes = 0;
        if (want == 0) want = 16;
        hipError_t e = hipMalloc(&p, want);
        if (e == hipSuccess) bytes = want;
        return e;
    }
    // Grow keeping the first `keep` bytes.
    hipError_t grow(size_t want, size_t keep, hipStream_t s) {
        if (want <= bytes && p != nullptr) return hipSuccess;
        void* q = nullptr;
        hipError_t e = hipMalloc(&q, want);
        if (e != hipSuccess) return e;
        if (p && keep) {
            e = hipMemcpyAsync(q, p, keep, hipMemcpyDeviceToDevice, s);
            if (e != hipSuccess) { (void)hipFree(q); return e; }
            e = hipStreamSynchronize(s);
            if (e != hipSuccess) { (void)hipFree(q); return e; }
        }
        if (p) (void)hipFree(p);
        p = q;
        bytes = want;
        return hipSuccess;
    }
    void release() {
        if (p) (void)hipFree(p);
        p = nullptr;
        bytes = 0;
    }
    template <class T>
    T* as() const { return static_cast<T*>(p); }
};

// Everything the kernels of one context read or write.
struct DevPlan {
    // used by the forward / adjoint passes
    DevBuf perm, leaf, leafc, js, items, queue, leaf_slot, partial, counter, boxes, table,
        adj_table;
    DevBuf x64, x32, stage_pos, stage_mass, far;
    DevBuf cell, cell_aux, cellc, M, Lc, Lt, m2l_row, m2l_src, m2l_shift, level_cells;
    DevBuf w64, w32, fargrad;
    // on-GPU planner scratch
    DevBuf p2p_row, wpos, keys, keys_tmp, plist, plist_tmp, hist, flag, lv_first, tile_sums;
    bool force64 = false;   // sort by the full 64-bit keys (a long run of equal short keys)
    DevBuf pc, pc_tmp, clo, chi, wcell, box_first, walkbox, front, front_next, p2p_keys,
        p2p_keys_tmp, m2l_keys, m2l_keys_tmp, wcount, cost, cost_keys, cost_keys_tmp, queue_tmp,
        item_count, cell_axis, farflag, walk_ctl, froots, loop_cells, m2l_vals, rowcnt,
        longrows;
    // scratch of the M2L rows, which may be built on another stream beside
    // the P2P rows
    DevBuf rowcnt_m2l, tile_sums_m2l, longrows_m2l;
    hipEvent_t fork_ev = nullptr, m2l_done = nullptr;
    // the particle records gathered on the side stream
    hipEvent_t geom_ev = nullptr, gather_ev = nullptr;
    // cells the level loop partitions, by depth (loop_cells holds them);
    // n_froots subtrees finished in one launch (0: the loop does every level)
    std::vector<int32_t> loop_depth_begin;
    int n_froots = 0;
    // walk sizes seen on the last level-by-level build of this tree shape
    uint32_t walk_cap_front = 0, walk_cap_p2p = 0, walk_cap_m2l = 0;
    int walk_levels = 0;
    std::vector<uint32_t> walk_sizes;   // frontier size per level, last build

    // pinned host words for the planner's read-backs (a copy into pageable
    // memory goes through a staging buffer and costs tens of microseconds)
    uint32_t* host_rb = nullptr;
    static constexpr int kHostRbWords = 4096;
    hipError_t ensure_host_rb() {
        if (host_rb) return hipSuccess;
        return hipHostMalloc(reinterpret_cast<void**>(&host_rb), kHostRbWords * 4, hipHostMallocDefault);
    }
    void release_all() {
        if (host_rb) (void)hipHostFree(host_rb);
        host_rb = nullptr;
        for (hipEvent_t* e : {&fork_ev, &m2l_done, &geom_ev, &gather_ev})
            if (*e) (void)hipEventDestroy(*e);
        fork_ev = m2l_done = geom_ev = gather_ev = nullptr;
        for (DevBuf* b : {&rowcnt_m2l, &tile_sums_m2l, &longrows_m2l}) b->release();
        for (DevBuf* b : {&perm, &leaf, &leafc, &js, &items, &queue, &leaf_slot, &partial, &counter,
                          &boxes, &table, &x64, &x32, &stage_pos, &stage_mass, &far, &cell,
                          &cell_aux, &cellc, &M, &Lc, &Lt, &m2l_row, &m2l_src, &m2l_shift, &level_cells,
                          &w64, &w32, &fargrad, &p2p_row, &wpos, &keys, &keys_tmp, &plist, &plist_tmp, &hist,
                          &flag, &lv_first, &tile_sums, &pc, &pc_tmp, &clo, &chi, &wcell,
                          &box_first, &walkbox, &front, &front_next, &p2p_keys, &p2p_keys_tmp,
                          &m2l_keys, &m2l_keys_tmp, &wcount, &cost, &cost_keys, &cost_keys_tmp,
                          &queue_tmp, &item_count, &cell_axis, &farflag, &walk_ctl, &froots,
                          &loop_cells, &m2l_vals, &rowcnt, &longrows})
            b->release();
    }
};

// Counts the host needs after a device plan.
struct PlanCounts {
    int64_t n_p2p = 0, n_m2l = 0, n_items = 0, candidate_pairs = 0;
    // smallest depth of an M2L source / target cell (the pass-up and
    // pass-down need no level above it); INT32_MAX without M2L tasks
    int32_t m2l_min_depth_src = 0x7fffffff, m2l_min_depth_tgt = 0x7fffffff;
};

// Sort / scan primitives (gpu_sort.hip).
int64_t sort_tiles(int64_t n);
// 32-bit words of the `hist` scratch radix_sort_u64 needs for nseg
// segments of n keys.
int64_t sort_hist_words(int64_t n, int nseg = 1);
// Stable sort of keys[seg n .. (seg + 1) n) (and vals alongside) for each of
// the nseg segments, by bits [bit_begin, bit_end) in 8-bit passes; the
// result ends in the tmp buffers when the pass count is odd.
hipError_t radix_sort_u64(uint64_t* keys, uint32_t* vals, uint64_t* tmp_keys, uint32_t* tmp_vals,
                          uint32_t* hist, int64_t n, int bit_begin, int bit_end, hipStream_t s,
                          bool* result_in_tmp, int nseg = 1);
// The same for 32-bit keys (bits beyond 32 ignored).
hipError_t radix_sort_u32(uint32_t* keys, uint32_t* vals, uint32_t* tmp_keys, uint32_t* tmp_vals,
                          uint32_t* hist, int64_t n, int bit_begin, int bit_end, hipStream_t s,
                          bool* result_in_tmp, int nseg = 1);
hipError_t exclusive_scan_i32(const int32_t* in, int32_t* out, int64_t n, uint32_t* tile_sums,
                              hipStream_t s);

// Enqueues the checks of device particles (finite positions, finite
// non-negative masses); gpu_build_plan reads their result.
hipError_t gpu_enqueue_checks(DevPlan& d, const double* pos, const double* mass, int64_t n,
                              hipStream_t s);

// Uploads the tree shape of `topo` (cells, leaves, depth levels) and the
// per-box constants.
hipError_t upload_topology(DevPlan& d, const Plan& topo, const BoxDev* boxdev, hipStream_t s);

// Called by gpu_build_plan as soon as the M2L lists are enqueued (on the
// `side` stream given to gpu_build_plan when there is one and M2L tasks
// exist, else on `s`), before the P2P rows and the work items are done on
// `s`, with the M2L task count and the smallest source / target depth, so
// that the far field can start on the side stream while the rows and items
// are built.  Returns an error message ("" on success).
using M2LReady = std::function<std::string(int64_t n_m2l, int32_t dmin_src, int32_t dmin_tgt)>;

// Builds the plan on the device from caller-order particles `pos` (n, 3) and
// `mass` (n) in device memory, for the shape uploaded by upload_topology.
// Fills perm, cell bounds and centres, x64 / x32, the P2P and M2L CSR, the
// work items and queue.  Synchronises `s` (the list sizes come back to the
// host).  Returns an error message ("" on success); when the checks of
// gpu_enqueue_checks (which must precede it on `s`) fail, stops early and
// sets *input_error to a message naming the first offending particle.
std::string gpu_build_plan(DevPlan& d, const Plan& topo, const double* pos, const double* mass,
                           int chunk, hipStream_t s, PlanCounts& out, std::string* input_error,
                           const M2LReady& on_m2l = M2LReady(), hipStream_t side = nullptr);

// Re-cuts the work items for a new chunk size from the device CSR.
std::string gpu_make_items(DevPlan& d, const Plan& topo, int64_t n_p2p, int chunk, hipStream_t s,
                           PlanCounts& out);

}  // namespace pmfmm
