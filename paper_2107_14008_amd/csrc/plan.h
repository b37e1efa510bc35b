// Host-side plan: ORB tree, dual-walk task lists and P2P work items.
//
// Built on the CPU (the paper builds the tree and both task lists on the
// host as well, Sec. 3) and uploaded once per build.  All geometry decisions
// use correctly rounded float64 +, -, *, sqrt, fabs, max and comparisons in
// a fixed order; this file must be compiled without floating-point
// contraction.
#pragma once

#include <cstdint>
#include <string>
#include <vector>

namespace pmfmm {

// Work queue of the persistent P2P and adjoint launches, cut into
// kQueueSegs segments of consecutive item slots (slots follow the ORB leaf
// order, so a segment is a compact region of the box): slot s is in segment
// floor(s kQueueSegs / n_items), and the queue lists the segments in order,
// each longest first.  Workgroups are dispatched round robin over the 8 XCDs
// of an MI355X, each with its own L2: workgroup b starts on segment
// b % kQueueSegs, so the sources one XCD reads stay near one region, and
// moves on to the other segments when its own is exhausted.  Each segment
// has its own counter, kCounterStride ints apart (one 128-byte line each).
constexpr int kQueueSegs = 8;
constexpr int kCounterStride = 32;

struct BoxParams {
    double box, r_s, r_cut, G, theta;
    int32_t max_leaf, order;
    int32_t m2l_cut;   // 0: M2L only for pairs wholly inside r_cut; 1: by centre distance
};

struct Cell {
    double lo[3], hi[3];
    int32_t first, count;   // leaf-order particle range (global)
    int32_t child[2];       // global cell ids, -1 for a leaf
    int32_t parent;         // global cell id, -1 for a root
    int32_t depth;          // 0 at the box root
    int32_t leaf;           // global leaf id, -1 for an internal cell
    int32_t box;
};

// Work item of the persistent P2P launch: the tasks [t0, t1) of one i leaf.
struct WorkItem {
    int32_t leaf, t0, t1, slot;
};

struct Plan {
    int64_t n = 0;
    std::vector<BoxParams> boxes;
    std::vector<int32_t> box_first_particle;  // nbox + 1
    std::vector<int32_t> box_first_leaf;      // nbox + 1
    std::vector<int32_t> box_first_cell;      // nbox + 1
    std::vector<double> pos;                  // (n, 3) wrapped, caller order
    std::vector<double> mass;                 // (n)
    std::vector<int32_t> perm;                // leaf order -> caller index
    std::vector<Cell> cells;
    std::vector<int32_t> leaf_cell;           // leaf -> cell
    std::vector<int32_t> leaf_first, leaf_count, leaf_box;
    std::vector<int32_t> p2p_row, p2p_j, p2p_shift;
    std::vector<int32_t> m2l_row, m2l_src, m2l_shift;
    std::vector<int32_t> cell_first, cell_count, cell_child;  // views for the ABI
    std::vector<double> cell_lo, cell_hi;
    std::vector<WorkItem> items;              // natural (slot) order
    std::vector<int32_t> queue;               // slots: kQueueSegs segments, each longest first
    std::vector<int32_t> leaf_slot_begin;     // n_leaves + 1
    std::vector<int32_t> cells_by_depth;      // cells grouped by depth
    std::vector<int32_t> depth_begin;         // max_depth + 2
    int64_t candidate_pairs = 0;
    bool far_field = false;                   // any box with M2L tasks
    int max_order = -1;
};

// Builds tree + lists for every box.  Returns an empty string on success,
// otherwise a message (invalid input).
std::string make_plan(Plan& plan, const std::vector<BoxParams>& boxes,
                      const std::vector<int64_t>& counts, const double* pos,
                      const double* mass, int threads);

// Tree shape only (no particles): cells with first / count / children /
// parent / depth / leaf / box, the leaf table, cells grouped by depth.  The
// ORB shape depends on the particle counts and MAXLEAF alone.
void make_topology(Plan& plan, const std::vector<BoxParams>& boxes,
                   const std::vector<int64_t>& counts);

// Tasks per work item when the caller leaves the choice to the library: an
// item then holds at most 32 x 64 x 64 pair evaluations, a small part of a
// wavefront's share of a large launch, so the longest-first queue ends with
// little idle time, while the per-item partial sums (1.5 KB each, read by
// the ordered reduction) stay few (measured at 128^3 and 256^3: 16 to 48
// tasks give the same P2P time within 1 %, 8 is 20 % slower, whole rows
// leave a tail).
constexpr int kAutoChunk = 32;

// (Re)cuts the P2P rows into work items of at most `chunk` tasks
// (0 = automatic) and orders the queue by decreasing pair count.
void make_items(Plan& plan, int chunk);

}  // namespace pmfmm
