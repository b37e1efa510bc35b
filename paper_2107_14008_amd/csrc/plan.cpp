// Host plan: ORB tree (Sec. 2), dual walk into P2P and M2L task lists
// (Sec. 3), TaskGroup / GroupIdx ordering (Sec. 3.2) and P2P work items.
//
// Tree reading: a cell with more than MAXLEAF particles splits along the
// axis of largest extent (first axis on ties); the left child takes the
// floor(n/2) particles smallest by (coordinate, caller index); leaf
// particles are kept in ascending caller index; cells are numbered in
// pre-order.  Walk reading: for a cell pair (t, u) with source image shift
// s, R = (c_u - c_t) + s L, gap = max(|R| - (h_t + h_u), 0) per axis; the
// pair is dropped when |gap|^2 >= r_cut^2 (1 + 2^-40), sent to M2L when the
// far field is on, |(|R| + h_t + h_u)|^2 < r_cut^2 (1 - 2^-40) and
// (rad_t + rad_u)^2 < theta^2 |R|^2, recorded as P2P when both cells are
// leaves, and refined otherwise by splitting the cell of larger radius
// (both on a tie).  The guards keep every rounding error on the safe side
// of the per-pair cutoff test done in the kernels.  With the centre-distance
// cut (m2l_cut = 1) a pair passing the opening-angle test goes to M2L when
// |R|^2 < r_cut^2 and is dropped otherwise.
#include "plan.h"

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <future>
#include <thread>
#include <unordered_map>

namespace pmfmm {
namespace {

constexpr double kGuard = 0x1p-40;

struct Rec {
    double x[3];
    int32_t idx;
    int32_t pad;
};

// Number of cells and leaves of the subtree over n particles; the tree's
// shape depends on n alone, which lets subtrees be built in parallel with
// their pre-order ids known in advance.
struct Shape {
    int64_t ml;
    std::unordered_map<int64_t, std::pair<int64_t, int64_t>> memo;
    std::pair<int64_t, int64_t> fill(int64_t n) {
        if (n <= ml) return {1, 1};
        auto it = memo.find(n);
        if (it != memo.end()) return it->second;
        auto a = fill(n / 2);
        auto b = fill(n - n / 2);
        std::pair<int64_t, int64_t> r{1 + a.first + b.first, a.second + b.second};
        memo.emplace(n, r);
        return r;
    }
    std::pair<int64_t, int64_t> get(int64_t n) const {
        if (n <= ml) return {1, 1};
        return memo.at(n);
    }
};

struct TreeBuilder {
    const Shape* shape;
    int64_t ml;
    Cell* cells;
    int32_t* leaf_cell;
    int32_t* perm;
    int32_t box;
    int32_t particle_base;  // global caller index of the box's first particle
    int spawn_depth;

    void build(Rec* a, int64_t n, int32_t cell, int32_t leaf, int32_t first,
               int32_t parent, int depth) {
        double lo[3] = {a[0].x[0], a[0].x[1], a[0].x[2]};
        double hi[3] = {lo[0], lo[1], lo[2]};
        for (int64_t k = 1; k < n; ++k)
            for (int d = 0; d < 3; ++d) {
                lo[d] = std::min(lo[d], a[k].x[d]);
                hi[d] = std::max(hi[d], a[k].x[d]);
            }
        Cell& c = cells[cell];
        for (int d = 0; d < 3; ++d) { c.lo[d] = lo[d]; c.hi[d] = hi[d]; }
        c.first = first;
        c.count = (int32_t)n;
        c.child[0] = c.child[1] = -1;
        c.parent = parent;
        c.depth = depth;
        c.leaf = -1;
        c.box = box;
        if (n <= ml) {
            std::sort(a, a + n, [](const Rec& p, const Rec& q) { return p.idx < q.idx; });
            for (int64_t k = 0; k < n; ++k) perm[first + k] = particle_base + a[k].idx;
            c.leaf = leaf;
            leaf_cell[leaf] = cell;
            return;
        }
        const double e0 = hi[0] - lo[0], e1 = hi[1] - lo[1], e2 = hi[2] - lo[2];
        int axis = 0;
        double best = e0;
        if (e1 > best) { axis = 1; best = e1; }
        if (e2 > best) { axis = 2; }
        const int64_t nl = n / 2;
        std::nth_element(a, a + nl, a + n, [axis](const Rec& p, const Rec& q) {
            if (p.x[axis] < q.x[axis]) return true;
            if (q.x[axis] < p.x[axis]) return false;
            return p.idx < q.idx;
        });
        const auto left_shape = shape->get(nl);
        const int32_t lc = cell + 1;
        const int32_t rc = cell + 1 + (int32_t)left_shape.first;
        const int32_t rl = leaf + (int32_t)left_shape.second;
        c.child[0] = lc;
        c.child[1] = rc;
        if (depth < spawn_depth && n > 32768) {
            auto fut = std::async(std::launch::async, [&] {
                build(a, nl, lc, leaf, first, cell, depth + 1);
            });
            build(a + nl, n - nl, rc, rl, first + (int32_t)nl, cell, depth + 1);
            fut.get();
        } else {
            build(a, nl, lc, leaf, first, cell, depth + 1);
            build(a + nl, n - nl, rc, rl, first + (int32_t)nl, cell, depth + 1);
        }
    }
};

double wrap_coord(double x, double box) {
    if (x >= 0.0 && x < box) return x;
    double y = x - box * std::floor(x / box);
    if (y >= box) y -= box;
    if (y < 0.0) y += box;
    if (!(y >= 0.0 && y < box)) y = 0.0;
    return y;
}

struct PairT {
    int32_t t, u;
    int32_t s, box;
};

struct WalkGeom {
    std::vector<double> c, hs, rad;   // per cell
    const Cell* cells;
    struct BoxW {
        double sv[27][3];
        double rc2_drop, rc2_m2l, th2, rc2;
        bool use_m2l, centre_cut;
    };
    std::vector<BoxW> bw;
};

// One classification step of the dual walk.  Emits into p2p / m2l or pushes
// children onto `next`.
inline void walk_step(const WalkGeom& g, const PairT& p, std::vector<uint64_t>& p2p,
                      std::vector<uint64_t>& m2l, std::vector<PairT>& next) {
    const WalkGeom::BoxW& b = g.bw[p.box];
    const double* ct = &g.c[3 * (size_t)p.t];
    const double* cu = &g.c[3 * (size_t)p.u];
    const double* ht = &g.hs[3 * (size_t)p.t];
    const double* hu = &g.hs[3 * (size_t)p.u];
    double R[3], A[3], H[3], gp[3];
    for (int a = 0; a < 3; ++a) {
        R[a] = (cu[a] - ct[a]) + b.sv[p.s][a];
        A[a] = std::fabs(R[a]);
        H[a] = ht[a] + hu[a];
        gp[a] = std::max(A[a] - H[a], 0.0);
    }
    const double gap2 = (gp[0] * gp[0] + gp[1] * gp[1]) + gp[2] * gp[2];
    if (!(gap2 < b.rc2_drop)) return;
    const double rt = g.rad[p.t], ru = g.rad[p.u];
    if (b.use_m2l) {
        double dm[3] = {A[0] + H[0], A[1] + H[1], A[2] + H[2]};
        const double dmax2 = (dm[0] * dm[0] + dm[1] * dm[1]) + dm[2] * dm[2];
        const double R2 = (R[0] * R[0] + R[1] * R[1]) + R[2] * R[2];
        const double lhs = rt + ru;
        const bool mac = lhs * lhs < b.th2 * R2;
        if (b.centre_cut ? mac : (mac && dmax2 < b.rc2_m2l)) {
            // the centre-distance reading drops an accepted pair at or
            // beyond r_cut (its kernel derivatives are zero there)
            if (b.centre_cut && !(R2 < b.rc2)) return;
            m2l.push_back(((uint64_t)(uint32_t)p.t << 32) |
                          ((uint64_t)(uint32_t)p.u << 5) | (uint64_t)p.s);
            return;
        }
    }
    const Cell& Ct = g.cells[p.t];
    const Cell& Cu = g.cells[p.u];
    const bool lt = Ct.leaf >= 0, lu = Cu.leaf >= 0;
    if (lt && lu) {
        p2p.push_back(((uint64_t)(uint32_t)Ct.leaf << 32) |
                      ((uint64_t)(uint32_t)Cu.leaf << 5) | (uint64_t)p.s);
        return;
    }
    if (!lt && (lu || rt > ru)) {
        next.push_back({Ct.child[0], p.u, p.s, p.box});
        next.push_back({Ct.child[1], p.u, p.s, p.box});
    } else if (!lu && (lt || ru > rt)) {
        next.push_back({p.t, Cu.child[0], p.s, p.box});
        next.push_back({p.t, Cu.child[1], p.s, p.box});
    } else {
        for (int k = 0; k < 2; ++k)
            for (int k2 = 0; k2 < 2; ++k2)
                next.push_back({Ct.child[k], Cu.child[k2], p.s, p.box});
    }
}

// Rows by the high 32 bits of the keys (counting sort), each row sorted by
// the low 32 bits; col = low bits >> 5, shift = low bits & 31.
void keys_to_csr(std::vector<uint64_t>& keys, int64_t n_rows, int threads,
                 std::vector<int32_t>& row, std::vector<int32_t>& col,
                 std::vector<int32_t>& shift) {
    row.assign(n_rows + 1, 0);
    for (uint64_t k : keys) row[(k >> 32) + 1]++;
    for (int64_t r = 0; r < n_rows; ++r) row[r + 1] += row[r];
    std::vector<uint32_t> low(keys.size());
    {
        std::vector<int32_t> fill(row.begin(), row.end() - 1);
        for (uint64_t k : keys) low[fill[k >> 32]++] = (uint32_t)(k & 0xffffffffu);
    }
    std::vector<uint64_t>().swap(keys);
    std::atomic<int64_t> next{0};
    auto work = [&] {
        for (;;) {
            int64_t r0 = next.fetch_add(1024);
            if (r0 >= n_rows) break;
            int64_t r1 = std::min<int64_t>(n_rows, r0 + 1024);
            for (int64_t r = r0; r < r1; ++r) std::sort(low.begin() + row[r], low.begin() + row[r + 1]);
        }
    };
    std::vector<std::thread> th;
    for (int t = 1; t < threads; ++t) th.emplace_back(work);
    work();
    for (auto& t : th) t.join();
    col.resize(low.size());
    shift.resize(low.size());
    for (size_t k = 0; k < low.size(); ++k) {
        col[k] = (int32_t)(low[k] >> 5);
        shift[k] = (int32_t)(low[k] & 31u);
    }
}

struct PhaseClock {
    bool on = std::getenv("PMFMM_PLAN_TIMING") != nullptr;
    std::chrono::steady_clock::time_point t = std::chrono::steady_clock::now();
    void lap(const char* what) {
        if (!on) return;
        auto now = std::chrono::steady_clock::now();
        std::fprintf(stderr, "[pmfmm plan] %-10s %8.2f ms\n", what,
                     std::chrono::duration<double, std::milli>(now - t).count());
        t = now;
    }
};

}  // namespace

std::string make_plan(Plan& plan, const std::vector<BoxParams>& boxes,
                      const std::vector<int64_t>& counts, const double* pos,
                      const double* mass, int threads) {
    if (threads <= 0) threads = (int)std::max(1u, std::thread::hardware_concurrency());
    PhaseClock clk;
    const int nbox = (int)boxes.size();
    plan = Plan();
    plan.boxes = boxes;
    int64_t n = 0;
    for (int b = 0; b < nbox; ++b) {
        if (counts[b] < 1) return "box " + std::to_string(b) + ": needs at least one particle";
        n += counts[b];
    }
    if (n > (int64_t)INT32_MAX) return "too many particles (limit 2^31 - 1)";
    plan.n = n;
    plan.pos.resize(3 * (size_t)n);
    plan.mass.assign(mass, mass + n);
    plan.box_first_particle.assign(nbox + 1, 0);
    for (int b = 0; b < nbox; ++b) plan.box_first_particle[b + 1] = plan.box_first_particle[b] + (int32_t)counts[b];
    for (int b = 0; b < nbox; ++b) {
        const double L = boxes[b].box;
        for (int64_t i = plan.box_first_particle[b]; i < plan.box_first_particle[b + 1]; ++i) {
            for (int d = 0; d < 3; ++d) {
                const double x = pos[3 * i + d];
                if (!std::isfinite(x))
                    return "box " + std::to_string(b) + ": non-finite position at particle " + std::to_string(i);
                plan.pos[3 * i + d] = wrap_coord(x, L);
            }
            const double m = mass[i];
            if (!std::isfinite(m) || m < 0.0)
                return "box " + std::to_string(b) + ": negative or non-finite mass at particle " + std::to_string(i);
        }
    }

    clk.lap("wrap");
    // ---- tree shapes and global numbering
    std::vector<Shape> shapes(nbox);
    plan.box_first_leaf.assign(nbox + 1, 0);
    plan.box_first_cell.assign(nbox + 1, 0);
    for (int b = 0; b < nbox; ++b) {
        shapes[b].ml = boxes[b].max_leaf;
        auto s = shapes[b].fill(counts[b]);
        plan.box_first_cell[b + 1] = plan.box_first_cell[b] + (int32_t)s.first;
        plan.box_first_leaf[b + 1] = plan.box_first_leaf[b] + (int32_t)s.second;
    }
    const int64_t n_cells = plan.box_first_cell[nbox];
    const int64_t n_leaves = plan.box_first_leaf[nbox];
    if (n_cells >= (int64_t)1 << 27) return "too many tree cells (limit 2^27)";
    plan.cells.resize(n_cells);
    plan.leaf_cell.resize(n_leaves);
    plan.perm.resize(n);
    int spawn_depth = 0;
    while ((1 << spawn_depth) < threads) ++spawn_depth;
    spawn_depth += 1;
    {
        std::vector<Rec> recs(n);
        for (int64_t i = 0; i < n; ++i) {
            for (int d = 0; d < 3; ++d) recs[i].x[d] = plan.pos[3 * i + d];
            recs[i].pad = 0;
        }
        std::vector<std::future<void>> futs;
        for (int b = 0; b < nbox; ++b) {
            const int32_t p0 = plan.box_first_particle[b];
            for (int64_t k = 0; k < counts[b]; ++k) recs[p0 + k].idx = (int32_t)k;
            TreeBuilder tb{&shapes[b], boxes[b].max_leaf, plan.cells.data(), plan.leaf_cell.data(),
                           plan.perm.data(), b, p0, nbox == 1 ? spawn_depth : 0};
            Rec* base = recs.data() + p0;
            const int64_t nb = counts[b];
            const int32_t c0 = plan.box_first_cell[b], l0 = plan.box_first_leaf[b];
            if (nbox == 1) {
                tb.build(base, nb, c0, l0, p0, -1, 0);
            } else {
                futs.push_back(std::async(std::launch::deferred, [tb, base, nb, c0, l0, p0]() mutable {
                    tb.build(base, nb, c0, l0, p0, -1, 0);
                }));
            }
        }
        if (!futs.empty()) {
            std::atomic<size_t> next{0};
            auto work = [&] {
                for (;;) {
                    size_t k = next.fetch_add(1);
                    if (k >= futs.size()) break;
                    futs[k].get();
                }
            };
            std::vector<std::thread> th;
            for (int t = 1; t < threads; ++t) th.emplace_back(work);
            work();
            for (auto& t : th) t.join();
        }
    }
    clk.lap("orb");
    plan.leaf_first.resize(n_leaves);
    plan.leaf_count.resize(n_leaves);
    plan.leaf_box.resize(n_leaves);
    for (int64_t l = 0; l < n_leaves; ++l) {
        const Cell& c = plan.cells[plan.leaf_cell[l]];
        plan.leaf_first[l] = c.first;
        plan.leaf_count[l] = c.count;
        plan.leaf_box[l] = c.box;
    }

    // ---- dual walk
    WalkGeom g;
    g.cells = plan.cells.data();
    g.c.resize(3 * n_cells);
    g.hs.resize(3 * n_cells);
    g.rad.resize(n_cells);
    for (int64_t k = 0; k < n_cells; ++k) {
        const Cell& c = plan.cells[k];
        for (int a = 0; a < 3; ++a) {
            g.c[3 * k + a] = 0.5 * (c.lo[a] + c.hi[a]);
            g.hs[3 * k + a] = 0.5 * (c.hi[a] - c.lo[a]);
        }
        const double* h = &g.hs[3 * k];
        g.rad[k] = std::sqrt((h[0] * h[0] + h[1] * h[1]) + h[2] * h[2]);
    }
    g.bw.resize(nbox);
    std::vector<PairT> frontier;
    for (int b = 0; b < nbox; ++b) {
        auto& w = g.bw[b];
        const BoxParams& bp = boxes[b];
        for (int s = 0; s < 27; ++s) {
            const double sx = (double)(s % 3 - 1), sy = (double)((s / 3) % 3 - 1), sz = (double)(s / 9 - 1);
            w.sv[s][0] = sx * bp.box;
            w.sv[s][1] = sy * bp.box;
            w.sv[s][2] = sz * bp.box;
        }
        const double rc2 = bp.r_cut * bp.r_cut;
        w.rc2_drop = rc2 * (1.0 + kGuard);
        w.rc2_m2l = rc2 * (1.0 - kGuard);
        w.th2 = bp.theta * bp.theta;
        w.rc2 = rc2;
        w.use_m2l = bp.order >= 0 && bp.theta > 0.0;
        w.centre_cut = bp.m2l_cut == 1;
        if (w.use_m2l) plan.max_order = std::max<int>(plan.max_order, bp.order);
        const int32_t root = plan.box_first_cell[b];
        for (int s = 0; s < 27; ++s) frontier.push_back({root, root, s, b});
    }
    std::vector<uint64_t> p2p_keys, m2l_keys;
    // breadth-first until there is enough independent work for the threads
    while (!frontier.empty() && frontier.size() < (size_t)threads * 512) {
        std::vector<PairT> next;
        next.reserve(frontier.size() * 2);
        for (const PairT& p : frontier) walk_step(g, p, p2p_keys, m2l_keys, next);
        frontier.swap(next);
    }
    {
        std::vector<std::vector<uint64_t>> tp(threads), tm(threads);
        std::atomic<size_t> next_idx{0};
        auto work = [&](int tid) {
            std::vector<PairT> stack;
            for (;;) {
                size_t k0 = next_idx.fetch_add(64);
                if (k0 >= frontier.size()) break;
                size_t k1 = std::min(frontier.size(), k0 + 64);
                for (size_t k = k0; k < k1; ++k) {
                    stack.push_back(frontier[k]);
                    while (!stack.empty()) {
                        PairT p = stack.back();
                        stack.pop_back();
                        walk_step(g, p, tp[tid], tm[tid], stack);
                    }
                }
            }
        };
        std::vector<std::thread> th;
        for (int t = 1; t < threads; ++t) th.emplace_back(work, t);
        work(0);
        for (auto& t : th) t.join();
        for (int t = 0; t < threads; ++t) {
            p2p_keys.insert(p2p_keys.end(), tp[t].begin(), tp[t].end());
            std::vector<uint64_t>().swap(tp[t]);
            m2l_keys.insert(m2l_keys.end(), tm[t].begin(), tm[t].end());
            std::vector<uint64_t>().swap(tm[t]);
        }
    }
    clk.lap("walk");
    plan.far_field = !m2l_keys.empty();
    keys_to_csr(p2p_keys, n_leaves, threads, plan.p2p_row, plan.p2p_j, plan.p2p_shift);
    keys_to_csr(m2l_keys, n_cells, threads, plan.m2l_row, plan.m2l_src, plan.m2l_shift);

    clk.lap("csr");
    int64_t cand = 0;
    for (int64_t i = 0; i < n_leaves; ++i)
        for (int32_t t = plan.p2p_row[i]; t < plan.p2p_row[i + 1]; ++t)
            cand += (int64_t)plan.leaf_count[i] * plan.leaf_count[plan.p2p_j[t]];
    plan.candidate_pairs = cand;

    // ---- flat views and depth levels
    plan.cell_first.resize(n_cells);
    plan.cell_count.resize(n_cells);
    plan.cell_child.resize(2 * n_cells);
    plan.cell_lo.resize(3 * n_cells);
    plan.cell_hi.resize(3 * n_cells);
    int max_depth = 0;
    for (int64_t k = 0; k < n_cells; ++k) {
        const Cell& c = plan.cells[k];
        plan.cell_first[k] = c.first;
        plan.cell_count[k] = c.count;
        plan.cell_child[2 * k] = c.child[0];
        plan.cell_child[2 * k + 1] = c.child[1];
        for (int a = 0; a < 3; ++a) { plan.cell_lo[3 * k + a] = c.lo[a]; plan.cell_hi[3 * k + a] = c.hi[a]; }
        max_depth = std::max(max_depth, c.depth);
    }
    plan.depth_begin.assign(max_depth + 2, 0);
    for (int64_t k = 0; k < n_cells; ++k) plan.depth_begin[plan.cells[k].depth + 1]++;
    for (int d = 0; d <= max_depth; ++d) plan.depth_begin[d + 1] += plan.depth_begin[d];
    plan.cells_by_depth.resize(n_cells);
    {
        std::vector<int32_t> fill(plan.depth_begin.begin(), plan.depth_begin.end() - 1);
        for (int64_t k = 0; k < n_cells; ++k) plan.cells_by_depth[fill[plan.cells[k].depth]++] = (int32_t)k;
    }
    clk.lap("views");
    return std::string();
}

namespace {

struct TopoBuilder {
    const Shape* shape;
    int64_t ml;
    Cell* cells;
    int32_t* leaf_cell;
    int32_t box;
    void build(int64_t n, int32_t cell, int32_t leaf, int32_t first, int32_t parent, int depth) {
        Cell& c = cells[cell];
        for (int d = 0; d < 3; ++d) c.lo[d] = c.hi[d] = 0.0;
        c.first = first;
        c.count = (int32_t)n;
        c.child[0] = c.child[1] = -1;
        c.parent = parent;
        c.depth = depth;
        c.leaf = -1;
        c.box = box;
        if (n <= ml) {
            c.leaf = leaf;
            leaf_cell[leaf] = cell;
            return;
        }
        const int64_t nl = n / 2;
        const auto ls = shape->get(nl);
        const int32_t lc = cell + 1, rc = cell + 1 + (int32_t)ls.first;
        c.child[0] = lc;
        c.child[1] = rc;
        build(nl, lc, leaf, first, cell, depth + 1);
        build(n - nl, rc, leaf + (int32_t)ls.second, first + (int32_t)nl, cell, depth + 1);
    }
};

}  // namespace

void make_topology(Plan& plan, const std::vector<BoxParams>& boxes,
                   const std::vector<int64_t>& counts) {
    const int nbox = (int)boxes.size();
    plan.boxes = boxes;
    plan.box_first_particle.assign(nbox + 1, 0);
    plan.box_first_leaf.assign(nbox + 1, 0);
    plan.box_first_cell.assign(nbox + 1, 0);
    std::vector<Shape> shapes(nbox);
    for (int b = 0; b < nbox; ++b) {
        shapes[b].ml = boxes[b].max_leaf;
        auto s = shapes[b].fill(counts[b]);
        plan.box_first_particle[b + 1] = plan.box_first_particle[b] + (int32_t)counts[b];
        plan.box_first_cell[b + 1] = plan.box_first_cell[b] + (int32_t)s.first;
        plan.box_first_leaf[b + 1] = plan.box_first_leaf[b] + (int32_t)s.second;
    }
    plan.n = plan.box_first_particle[nbox];
    const int64_t nc = plan.box_first_cell[nbox], nl = plan.box_first_leaf[nbox];
    plan.cells.assign(nc, Cell{});
    plan.leaf_cell.assign(nl, 0);
    for (int b = 0; b < nbox; ++b) {
        TopoBuilder tb{&shapes[b], boxes[b].max_leaf, plan.cells.data(), plan.leaf_cell.data(), b};
        tb.build(counts[b], plan.box_first_cell[b], plan.box_first_leaf[b], plan.box_first_particle[b], -1, 0);
    }
    plan.leaf_first.resize(nl);
    plan.leaf_count.resize(nl);
    plan.leaf_box.resize(nl);
    for (int64_t l = 0; l < nl; ++l) {
        const Cell& c = plan.cells[plan.leaf_cell[l]];
        plan.leaf_first[l] = c.first;
        plan.leaf_count[l] = c.count;
        plan.leaf_box[l] = c.box;
    }
    int max_depth = 0;
    for (const Cell& c : plan.cells) max_depth = std::max(max_depth, c.depth);
    plan.depth_begin.assign(max_depth + 2, 0);
    for (const Cell& c : plan.cells) plan.depth_begin[c.depth + 1]++;
    for (int d = 0; d <= max_depth; ++d) plan.depth_begin[d + 1] += plan.depth_begin[d];
    plan.cells_by_depth.resize(nc);
    std::vector<int32_t> fill(plan.depth_begin.begin(), plan.depth_begin.end() - 1);
    for (int64_t k = 0; k < nc; ++k) plan.cells_by_depth[fill[plan.cells[k].depth]++] = (int32_t)k;
    plan.max_order = -1;
    for (const auto& b : boxes)
        if (b.order >= 0 && b.theta > 0.0) plan.max_order = std::max<int>(plan.max_order, b.order);
}

void make_items(Plan& plan, int chunk) {
    const int64_t n_leaves = (int64_t)plan.leaf_count.size();
    const int64_t n_tasks = (int64_t)plan.p2p_j.size();
    if (chunk <= 0) chunk = kAutoChunk;
    plan.items.clear();
    plan.leaf_slot_begin.assign(n_leaves + 1, 0);
    std::vector<int64_t> cost;
    for (int64_t i = 0; i < n_leaves; ++i) {
        const int32_t r0 = plan.p2p_row[i], r1 = plan.p2p_row[i + 1];
        const int32_t len = r1 - r0;
        plan.leaf_slot_begin[i] = (int32_t)plan.items.size();
        if (len == 0) continue;
        const int32_t parts = (len + chunk - 1) / chunk;
        const int32_t base = len / parts, extra = len % parts;
        int32_t t = r0;
        for (int32_t k = 0; k < parts; ++k) {
            const int32_t sz = base + (k < extra ? 1 : 0);
            int64_t c = 0;
            for (int32_t q = t; q < t + sz; ++q) c += plan.leaf_count[plan.p2p_j[q]];
            c *= plan.leaf_count[i];
            plan.items.push_back({(int32_t)i, t, t + sz, (int32_t)plan.items.size()});
            cost.push_back(c);
            t += sz;
        }
    }
    plan.leaf_slot_begin[n_leaves] = (int32_t)plan.items.size();
    // queue: the kQueueSegs segments of consecutive slots in order, each
    // longest first (the GPU kernels start each XCD on its own segment)
    plan.queue.resize(plan.items.size());
    for (size_t k = 0; k < plan.queue.size(); ++k) plan.queue[k] = (int32_t)k;
    const int64_t n_items = (int64_t)plan.items.size();
    auto seg = [&](int32_t a) { return (int64_t)a * kQueueSegs / n_items; };
    std::stable_sort(plan.queue.begin(), plan.queue.end(), [&](int32_t a, int32_t b) {
        const int64_t sa = seg(a), sb = seg(b);
        return sa != sb ? sa < sb : cost[a] > cost[b];
    });
}

}  // namespace pmfmm
