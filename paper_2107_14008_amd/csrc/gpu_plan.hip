// On-GPU planner: the ORB tree (Sec. 2), the dual walk into P2P and M2L
// task lists (Sec. 3) and the TaskGroup / GroupIdx CSR with its work items
// (Sec. 3.2), built from particles already in HBM.  Same readings as the
// host planner (plan.cpp), and the same results bit for bit: every geometry
// decision is the same rounded float64 operation in the same order.
//
// ORB without per-cell sorting: the particles are sorted once per axis by
// (coordinate, caller index) with a stable radix sort; the shape of the tree
// (which cell holds which range of positions) depends on the particle count
// alone and comes from the host.  Level by level, each splitting cell reads
// its bounds from the ends of its three sorted ranges, marks the floor(n/2)
// first particles of its split axis as "left", and every axis list is
// partitioned stably (prefix sums of the left marks), which keeps each child
// range sorted on every axis.  Once a subtree holds at most 8192 particles
// and 1024 cells, one workgroup finishes it in LDS (k_orb_fused), so the
// launches per level are paid only for the top levels.
//
// Dual walk: level-synchronous over a frontier of cell pairs (the canonical
// half of the symmetric walk); one thread per pair classifies it and appends
// P2P keys, M2L keys (each with its mirror) or child pairs with one atomic
// per wavefront.  The keys (i << 32 | j << 5 | shift) are then sorted,
// which yields the canonical (i, j, shift) order and the CSR rows.
#include <algorithm>
#include <chrono>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <vector>

#include "gpu_plan.h"

namespace pmfmm {
namespace {

constexpr double kGuard = 0x1p-40;

struct WalkBox {
    double L, rc2_drop, rc2_m2l, th2;
    int32_t use_m2l, centre_cut;   // centre_cut: M2L by centre distance, else drop
    double rc2;
};

__device__ __forceinline__ double wrap_coord(double x, double L) {
#pragma clang fp contract(off)
    if (x >= 0.0 && x < L) return x;
    double y = x - L * floor(x / L);
    if (y >= L) y -= L;
    if (y < 0.0) y += L;
    if (!(y >= 0.0 && y < L)) y = 0.0;
    return y;
}

__device__ __forceinline__ int box_of(const int32_t* __restrict__ bf, int nbox, int i) {
    int lo = 0, hi = nbox - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (bf[mid] <= i) lo = mid; else hi = mid - 1;
    }
    return lo;
}

// Order-preserving key of a non-negative double (+0 and -0 equal).
__device__ __forceinline__ uint64_t coord_key(double x) {
    return x == 0.0 ? 0ull : (uint64_t)__double_as_longlong(x);
}

// Sort key of a wrapped coordinate x in [0, L): floor(x 2^bits / L) with
// 24 or 32 bits, a non-decreasing function of x (a rounded product and a
// floor), so that sorting by it and then ordering each run of equal keys by
// x is the order by x.  24 bits (three 8-bit radix passes) up to
// kKey24Max particles, where a bin of L / 2^24 rarely holds two of them;
// beyond, the runs of equal keys would cost k_run_fix more than the fourth
// pass (measured at 256^3), and the key has 32 bits.
constexpr int64_t kKey24Max = int64_t(1) << 22;
__device__ __forceinline__ uint32_t coord_key(double x, double scale, double kmax) {
    const double t = x * scale;
    return t >= kmax ? (uint32_t)kmax : (uint32_t)t;
}

__global__ void k_wrap_keys(const double* __restrict__ pos, int64_t n, const int32_t* __restrict__ bf,
                            int nbox, const BoxDev* __restrict__ boxes, double* __restrict__ wpos,
                            uint32_t* __restrict__ keys, uint32_t* __restrict__ vals, int key_bits) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double L = boxes[box_of(bf, nbox, (int)i)].L;
    const double range = key_bits == 24 ? 16777216.0 : 4294967296.0;
    const double scale = range / L;
    for (int a = 0; a < 3; ++a) {
        const double x = wrap_coord(pos[3 * i + a], L);
        wpos[3 * i + a] = x;
        keys[a * n + i] = coord_key(x, scale, range - 1.0);
        vals[a * n + i] = (uint32_t)i;
    }
}

// Full 64-bit keys of the wrapped coordinates (the fallback sort).
__global__ void k_keys64(const double* __restrict__ wpos, int64_t n, uint64_t* __restrict__ keys,
                         uint32_t* __restrict__ vals) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    for (int a = 0; a < 3; ++a) {
        keys[a * n + i] = coord_key(wpos[3 * i + a]);
        vals[a * n + i] = (uint32_t)i;
    }
}

// After the stable sort by the key, each run of equal keys of one axis
// list is in caller order; this puts it in coordinate order (stable, so
// equal coordinates stay in caller order).  The first position of a run of
// at most kRunMax elements sorts it in place (insertion sort).  A longer
// run is only checked: its start checks its first kRunMax - 1 neighbour
// pairs and every later position the pair it ends; any pair out of order
// sets *longrun, and the caller then sorts by the full 64-bit keys.
constexpr int kRunMax = 64;

__global__ void k_run_fix(const uint32_t* __restrict__ keys, uint32_t* __restrict__ vals, int64_t n,
                          const double* __restrict__ wpos, int* __restrict__ longrun) {
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= 3 * n) return;
    const int a = q >= n ? (q >= 2 * n ? 2 : 1) : 0;
    const int64_t s0 = (int64_t)a * n, s1 = s0 + n;
    const uint32_t h = keys[q];
    auto x_of = [&](int64_t p) { return wpos[3 * (size_t)vals[p] + a]; };
    if (q == s0 || keys[q - 1] != h) {
        if (q + 1 >= s1 || keys[q + 1] != h) return;   // a run of one
        if (q + kRunMax < s1 && keys[q + kRunMax] == h) {
            double prev = x_of(q);
            for (int64_t p = q + 1; p < q + kRunMax; ++p) {
                const double x = x_of(p);
                if (x < prev) {
                    atomicOr(longrun, 1);
                    return;
                }
                prev = x;
            }
            return;
        }
        int64_t e = q + 2;
        while (e < s1 && keys[e] == h) ++e;
        for (int64_t i = q + 1; i < e; ++i) {
            const uint32_t vi = vals[i];
            const double xi = wpos[3 * (size_t)vi + a];
            int64_t j = i - 1;
            while (j >= q) {
                const uint32_t vj = vals[j];
                if (!(xi < wpos[3 * (size_t)vj + a])) break;
                vals[j + 1] = vj;
                --j;
            }
            vals[j + 1] = vi;
        }
    } else if (q - kRunMax >= s0 && keys[q - kRunMax] == h) {
        // kRunMax or more positions into a long run (keys are sorted)
        if (x_of(q) < x_of(q - 1)) atomicOr(longrun, 1);
    }
}

__global__ void k_box_keys(const uint32_t* __restrict__ vals, int64_t n, const int32_t* __restrict__ bf,
                           int nbox, uint32_t* __restrict__ keys) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    keys[i] = (uint32_t)box_of(bf, nbox, (int)vals[i]);
}

__global__ void k_init_pc(int64_t n, const int32_t* __restrict__ bf, const int32_t* __restrict__ bfc,
                          int nbox, int32_t* __restrict__ pc) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    pc[i] = bfc[box_of(bf, nbox, (int)i)];
}

// Bounds of every cell of one depth from the ends of its sorted ranges,
// the split axis of those that split, and pfirst[c]: the left marks before
// cell c's first position, the same in each of the three lists.  A
// splitting cell marks the first floor(count / 2) positions of its range in
// every list and nothing else is marked, so with the level's cells in
// position order (the pre-order within one depth) pfirst[c] = the marks of
// the level's cells before c: a scan over the level's cells, no marks read.
// One workgroup.
constexpr int kCellsT = 1024;

__global__ void __launch_bounds__(kCellsT)
k_cells_level(const int32_t* __restrict__ level, int nd, const int4* __restrict__ cell,
              const int4* __restrict__ aux, const uint32_t* __restrict__ plist, int64_t n,
              const double* __restrict__ wpos, double* __restrict__ clo, double* __restrict__ chi,
              int32_t* __restrict__ axis_out, int32_t* __restrict__ pfirst) {
    __shared__ uint32_t wsum[kCellsT / 64];
    __shared__ uint32_t carry;
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    if (t == 0) carry = 0u;
    __syncthreads();
    for (int k0 = 0; k0 < nd; k0 += kCellsT) {
        const int k = k0 + t;
        uint32_t half = 0u;
        int c = -1;
        if (k < nd) {
            c = level[k];
            const int4 ci = cell[c];
            double lo[3], hi[3];
            for (int a = 0; a < 3; ++a) {
                lo[a] = wpos[3 * (size_t)plist[a * n + ci.x] + a];
                hi[a] = wpos[3 * (size_t)plist[a * n + ci.x + ci.y - 1] + a];
                clo[3 * (size_t)c + a] = lo[a];
                chi[3 * (size_t)c + a] = hi[a];
            }
            if (aux[c].x >= 0) {
#pragma clang fp contract(off)
                const double e0 = hi[0] - lo[0], e1 = hi[1] - lo[1], e2 = hi[2] - lo[2];
                int axis = 0;
                double best = e0;
                if (e1 > best) { axis = 1; best = e1; }
                if (e2 > best) axis = 2;
                axis_out[c] = axis;
                half = (uint32_t)(ci.y / 2);
            }
        }
        uint32_t x = half;
        for (int off = 1; off < 64; off <<= 1) {
            const uint32_t y = __shfl_up(x, off);
            if (lane >= off) x += y;
        }
        if (lane == 63) wsum[wave] = x;
        __syncthreads();
        uint32_t before = 0u, tot = 0u;
        for (int w = 0; w < kCellsT / 64; ++w) {
            const uint32_t v = wsum[w];
            if (w < wave) before += v;
            tot += v;
        }
        if (k < nd) pfirst[c] = (int32_t)(carry + before + x - half);
        __syncthreads();
        if (t == 0) carry += tot;
        __syncthreads();
    }
}

// Left marks of the particles of the cells splitting at this level (sax[c]
// >= 0), from their positions in the split axis's list, as bytes indexed by
// particle (a byte store needs no atomic); k_pack_marks then packs them
// into bits for the level's random reads.
__global__ void k_flag(int64_t n, const int32_t* __restrict__ pc, const int4* __restrict__ cell,
                       const int32_t* __restrict__ sax, const uint32_t* __restrict__ plist,
                       uint8_t* __restrict__ flag) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int c = pc[i];
    const int ax = sax[c];
    if (ax < 0) return;
    const int4 ci = cell[c];
    flag[plist[ax * n + i]] = (i - ci.x < ci.y / 2) ? 1 : 0;
}

// The stable partition of one level, with the left marks of the three lists
// (list a at [a n, (a + 1) n) of plist) computed where they are used instead
// of stored: a position's mark is its particle's left mark if its cell
// splits at this level, else 0.  A tile is the list positions [b T, (b + 1)
// T), T = 1024, of all three lists, whose cells are the same (one pc / sax /
// cell read serves the three).  k_level_sums counts each tile's marks per
// list; k_cells_level has given the count of marks before each splitting
// cell's first position (the same in the three lists), and k_level_move
// counts them before every position (the tiles before its own, summed
// where they are needed, + the in-tile scan) and from the difference places
// the position.
constexpr int kLvThreads = 256;
constexpr int kLvRounds = 4;
constexpr int kLvTile = kLvThreads * kLvRounds;   // 1024 positions of each list

// The particles' left marks as bits: k_flag writes one byte per particle of
// a splitting cell (scattered by particle), and this packs the bytes of
// particles [64 w, 64 w + 64) into word w (one wavefront per word).  The
// level's random reads by particle then fall on n / 8 bytes, which stay in
// an XCD's 4 MB L2 up to tens of millions of particles; the bytes outgrow
// it from about four million.
__global__ void k_pack_marks(int64_t n, const uint8_t* __restrict__ flag,
                             uint64_t* __restrict__ bits) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const uint64_t b = __ballot(i < n && flag[i] != 0);
    if ((threadIdx.x & 63) == 0 && i < n) bits[i >> 6] = b;
}

__device__ __forceinline__ uint32_t mark_bit(const uint64_t* __restrict__ bits, uint32_t p) {
    return (uint32_t)(bits[p >> 6] >> (p & 63u)) & 1u;
}

// sax[c]: the split axis of a cell that splits at this level, else -1.  On
// the split axis's own list the mark follows from the position alone, so
// only the two other lists read the particle's bit.
// tile_sums[a ntiles + b]: the marks of list a in tile b.
__global__ void __launch_bounds__(kLvThreads)
k_level_sums(int64_t n, const int32_t* __restrict__ pc, const int32_t* __restrict__ sax,
             const int4* __restrict__ cell, const uint32_t* __restrict__ plist,
             const uint64_t* __restrict__ bits, uint32_t* __restrict__ tile_sums, int ntiles) {
    __shared__ uint64_t wsum[kLvThreads / 64];
    const int64_t base = (int64_t)blockIdx.x * kLvTile;
    // the three counts packed 21 bits apart (each at most kLvTile)
    uint64_t cnt = 0;
    for (int r = 0; r < kLvRounds; ++r) {
        const int64_t i = base + r * kLvThreads + threadIdx.x;
        if (i >= n) continue;
        const int c = pc[i];
        const int ax = sax[c];
        if (ax < 0) continue;
        const int4 ci = cell[c];
        const uint32_t own = (i - ci.x < ci.y / 2) ? 1u : 0u;
        for (int a = 0; a < 3; ++a) {
            const uint32_t m = a == ax ? own : mark_bit(bits, plist[(int64_t)a * n + i]);
            cnt += (uint64_t)m << (21 * a);
        }
    }
    for (int off = 32; off > 0; off >>= 1) cnt += __shfl_down(cnt, off);
    if ((threadIdx.x & 63) == 0) wsum[threadIdx.x >> 6] = cnt;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint64_t t = 0;
        for (int w = 0; w < kLvThreads / 64; ++w) t += wsum[w];
        for (int a = 0; a < 3; ++a)
            tile_sums[(size_t)a * ntiles + blockIdx.x] = (uint32_t)(t >> (21 * a)) & 0x1fffffu;
    }
}

// SCANNED: `offs` holds the exclusive scan of tile_sums over all 3 ntiles
// entries, so the tiles before tile b of list a hold offs[a ntiles + b] -
// offs[a ntiles] marks; otherwise each workgroup adds up tile_sums itself
// (no scan launch; quadratic in the tiles, so for up to kLvSumMax of them).
constexpr int kLvSumMax = 2048;

template <bool SCANNED>
__global__ void __launch_bounds__(kLvThreads)
k_level_move(int64_t n, const int32_t* __restrict__ pc, int32_t* __restrict__ pc_out,
             const int4* __restrict__ cell, const int4* __restrict__ aux,
             const int32_t* __restrict__ sax, const uint32_t* __restrict__ plist,
             uint32_t* __restrict__ pout, const uint64_t* __restrict__ bits,
             const uint32_t* __restrict__ tile_sums, const uint32_t* __restrict__ offs,
             int ntiles, const int32_t* __restrict__ pfirst) {
    __shared__ uint8_t mk[3][kLvTile];
    __shared__ uint16_t pre[3][kLvTile];
    __shared__ uint64_t wsum[kLvThreads / 64];
    __shared__ uint32_t woff[3][kLvThreads / 64];
    const int t = threadIdx.x;
    const int lane = t & 63, wave = t >> 6;
    if (!SCANNED) {
        // this tile's offsets: the counts of the tiles before it, per list
        for (int a = 0; a < 3; ++a) {
            uint32_t c = 0;
            for (int k = t; k < (int)blockIdx.x; k += kLvThreads) c += tile_sums[(size_t)a * ntiles + k];
            for (int off = 32; off > 0; off >>= 1) c += __shfl_down(c, off);
            if (lane == 0) woff[a][wave] = c;
        }
    }
    const int64_t base = (int64_t)blockIdx.x * kLvTile;
    uint32_t pv[kLvRounds][3];
    int32_t cv[kLvRounds];
    for (int r = 0; r < kLvRounds; ++r) {
        const int64_t i = base + r * kLvThreads + t;
        uint32_t m[3] = {0u, 0u, 0u};
        cv[r] = -1;
        pv[r][0] = pv[r][1] = pv[r][2] = 0u;
        if (i < n) {
            const int c = pc[i];
            cv[r] = c;
            for (int a = 0; a < 3; ++a) pv[r][a] = plist[(int64_t)a * n + i];
            const int ax = sax[c];
            if (ax >= 0) {
                const int4 ci = cell[c];
                const uint32_t own = (i - ci.x < ci.y / 2) ? 1u : 0u;
                for (int a = 0; a < 3; ++a) m[a] = a == ax ? own : mark_bit(bits, pv[r][a]);
            }
        }
        for (int a = 0; a < 3; ++a) mk[a][r * kLvThreads + t] = (uint8_t)m[a];
    }
    __syncthreads();
    // in-tile exclusive prefix per list: thread t owns positions
    // [kLvRounds t, kLvRounds (t + 1)); the three counts packed 21 bits apart
    uint64_t own = 0;
    for (int j = 0; j < kLvRounds; ++j)
        for (int a = 0; a < 3; ++a) own += (uint64_t)mk[a][kLvRounds * t + j] << (21 * a);
    uint64_t x = own;
    for (int off = 1; off < 64; off <<= 1) {
        const uint64_t y = __shfl_up(x, off);
        if (lane >= off) x += y;
    }
    if (lane == 63) wsum[wave] = x;
    __syncthreads();
    uint64_t run = x - own;
    for (int w = 0; w < wave; ++w) run += wsum[w];
    for (int j = 0; j < kLvRounds; ++j) {
        for (int a = 0; a < 3; ++a) {
            pre[a][kLvRounds * t + j] = (uint16_t)((run >> (21 * a)) & 0x1fffffu);
            run += (uint64_t)mk[a][kLvRounds * t + j] << (21 * a);
        }
    }
    __syncthreads();
    uint32_t toff[3];
    for (int a = 0; a < 3; ++a) {
        toff[a] = 0;
        if (SCANNED) {
            toff[a] = offs[(size_t)a * ntiles + blockIdx.x] - offs[(size_t)a * ntiles];
        } else {
            for (int w = 0; w < kLvThreads / 64; ++w) toff[a] += woff[a][w];
        }
    }
    for (int r = 0; r < kLvRounds; ++r) {
        const int64_t i = base + r * kLvThreads + t;
        if (i >= n) continue;
        const int c = cv[r];
        if (sax[c] < 0) {
            for (int a = 0; a < 3; ++a) pout[(int64_t)a * n + i] = pv[r][a];
            pc_out[i] = c;
            continue;
        }
        const int4 ci = cell[c];
        const int64_t first = ci.x, nl = ci.y / 2;
        const int64_t pf = pfirst[c];
        for (int a = 0; a < 3; ++a) {
            const int j = r * kLvThreads + t;
            const int64_t lr = (int64_t)(toff[a] + pre[a][j]) - pf;
            const int64_t pos = mk[a][j] ? first + lr : first + nl + (i - first - lr);
            pout[(int64_t)a * n + pos] = pv[r][a];
        }
        pc_out[i] = (i - first < nl) ? aux[c].x : aux[c].y;
    }
}

// The bottom levels of the tree in one launch: one workgroup per subtree of
// at most kFuseM particles and kFuseC cells.  The three sorted lists of the
// subtree's range are held in LDS as 16-bit local ids (a particle's local id
// is its rank in the x list) and partitioned level by level exactly as the
// level loop does (first floor(n/2) of the split axis left, stable), then
// each leaf's particles are written to perm in ascending caller index.
// Bounds of every cell of the subtree are written to clo / chi.
constexpr int kFuseM = 8192;
constexpr int kFuseC = 1024;
constexpr int kFuseT = 1024;
constexpr int kFuseRounds = (3 * kFuseM + kFuseT - 1) / kFuseT;   // 24
constexpr uint16_t kNoChild = 0xffffu;


// roots[b] = (subtree root cell, cells in the subtree, root depth, deepest depth)
__global__ void __launch_bounds__(kFuseT)
k_orb_fused(const int4* __restrict__ roots, const int4* __restrict__ cell,
            const int4* __restrict__ aux, const uint32_t* __restrict__ plist, int64_t n,
            const double* __restrict__ wpos, int32_t* __restrict__ loc, double* __restrict__ clo,
            double* __restrict__ chi, int32_t* __restrict__ perm) {
    __shared__ __align__(16) uint16_t lst[2 * 3 * kFuseM];
    __shared__ uint8_t flag[kFuseM];
    __shared__ uint16_t pcl[kFuseM];
    // per local cell: first | count << 16 | child0 << 32 | depth << 48 | axis << 56
    __shared__ uint64_t cinfo[kFuseC];
    __shared__ uint16_t cch1[kFuseC];
    __shared__ uint32_t sfirst[3 * kFuseC];
    __shared__ uint32_t wsum[kFuseT / 64];
    __shared__ uint64_t wmask[(kFuseT / 64) * kFuseRounds];
    __shared__ uint32_t wpre[(kFuseT / 64) * kFuseRounds];
    const int4 r = roots[blockIdx.x];
    const int root = r.x, nsub = r.y, depth_span = r.w - r.z;
    const int4 rc = cell[root];
    const int base = rc.x, m = rc.y;
    const int t = threadIdx.x;
    const int lane = t & 63, wave = t >> 6;
    const uint64_t below = lane ? (~0ull >> (64 - lane)) : 0ull;
    const uint32_t* __restrict__ l0 = plist + base;
    auto L = [&](int buf, int a, int k) -> uint16_t& { return lst[(buf * 3 + a) * kFuseM + k]; };
    auto c_first = [](uint64_t ci) { return (int)(ci & 0xffffu); };
    auto c_count = [](uint64_t ci) { return (int)((ci >> 16) & 0xffffu); };
    auto c_child0 = [](uint64_t ci) { return (int)((ci >> 32) & 0xffffu); };
    auto c_dep = [](uint64_t ci) { return (int)((ci >> 48) & 0xffu); };
    auto c_axis = [](uint64_t ci) { return (int)(ci >> 56); };

    for (int k = t; k < m; k += kFuseT) {
        L(0, 0, k) = (uint16_t)k;
        loc[l0[k]] = k;
        pcl[k] = 0;
    }
    for (int c = t; c < nsub; c += kFuseT) {
        const int4 ci = cell[root + c], ai = aux[root + c];
        const uint64_t ch0 = ai.x >= 0 ? (uint64_t)(ai.x - root) : (uint64_t)kNoChild;
        cinfo[c] = (uint64_t)(ci.x - base) | ((uint64_t)ci.y << 16) | (ch0 << 32) |
                   ((uint64_t)(ai.w - r.z) << 48);
        cch1[c] = ai.y >= 0 ? (uint16_t)(ai.y - root) : kNoChild;
    }
    // loc[] is written and read through global memory by this workgroup
    // only, so the barrier's workgroup-scope ordering suffices (an
    // agent-scope fence here writes back the whole L2, per workgroup)
    __syncthreads();
    for (int k = t; k < m; k += kFuseT) {
        L(0, 1, k) = (uint16_t)loc[plist[n + base + k]];
        L(0, 2, k) = (uint16_t)loc[plist[2 * n + base + k]];
    }
    __syncthreads();

    const int R = (3 * m + kFuseT - 1) / kFuseT;   // rounds of 64 positions per wave
    int cur = 0;
    for (int dep = 0;; ++dep) {
        // bounds of the cells of this depth, split axis of those that split
        for (int c = t; c < nsub; c += kFuseT) {
            const uint64_t ci = cinfo[c];
            if (c_dep(ci) != dep) continue;
            const int f = c_first(ci), e = f + c_count(ci) - 1;
            double lo[3], hi[3];
            for (int a = 0; a < 3; ++a) {
                lo[a] = wpos[3 * (size_t)l0[L(cur, a, f)] + a];
                hi[a] = wpos[3 * (size_t)l0[L(cur, a, e)] + a];
                clo[3 * (size_t)(root + c) + a] = lo[a];
                chi[3 * (size_t)(root + c) + a] = hi[a];
            }
            if (c_child0(ci) != kNoChild) {
#pragma clang fp contract(off)
                const double e0 = hi[0] - lo[0], e1 = hi[1] - lo[1], e2 = hi[2] - lo[2];
                int axis = 0;
                double best = e0;
                if (e1 > best) { axis = 1; best = e1; }
                if (e2 > best) axis = 2;
                cinfo[c] = (ci & 0x00ffffffffffffffull) | ((uint64_t)axis << 56);
            }
        }
        if (dep == depth_span) break;
        __syncthreads();
        auto splits = [&](uint64_t ci) { return c_dep(ci) == dep && c_child0(ci) != kNoChild; };
        for (int k = t; k < m; k += kFuseT) {
            const uint64_t ci = cinfo[pcl[k]];
            if (!splits(ci)) continue;
            flag[L(cur, c_axis(ci), k)] = (k - c_first(ci) < c_count(ci) / 2) ? 1 : 0;
        }
        __syncthreads();
        // Stable partition of the three lists by one exclusive scan over the
        // left marks of all 3m positions (each cell's range is contiguous in
        // every list, so differences inside a range count that range only).
        // Wave w owns the positions [w R 64, (w + 1) R 64), 64 consecutive
        // ones per round; a round's marks are one ballot, and a position's
        // prefix is wave base + round prefix + popcount of the lanes below.
        uint64_t* __restrict__ mymask = &wmask[wave * kFuseRounds];
        uint32_t* __restrict__ mypre = &wpre[wave * kFuseRounds];
#pragma unroll 4
        for (int rr = 0; rr < R; ++rr) {
            const int q = (wave * R + rr) * 64 + lane;
            bool f = false;
            if (q < 3 * m) {
                const int a = q >= m ? (q >= 2 * m ? 2 : 1) : 0;
                const int k = q - a * m;
                f = splits(cinfo[pcl[k]]) && flag[L(cur, a, k)];
            }
            const uint64_t mk = __ballot(f);
            if (lane == 0) mymask[rr] = mk;
        }
        {
            // lane rr scans the round counts of its wave
            const uint32_t cnt = lane < R ? (uint32_t)__popcll(mymask[lane]) : 0u;
            uint32_t x = cnt;
            for (int off = 1; off < 64; off <<= 1) {
                const uint32_t y = __shfl_up(x, off);
                if (lane >= off) x += y;
            }
            if (lane < R) mypre[lane] = x - cnt;
            if (lane == 63) wsum[wave] = x;
        }
        __syncthreads();
        if (t < kFuseT / 64) {
            uint32_t acc = 0;
            for (int w = 0; w < t; ++w) acc += wsum[w];
            for (int rr = 0; rr < R; ++rr) wpre[t * kFuseRounds + rr] += acc;
        }
        __syncthreads();
        auto prefix = [&](int q) {
            const int w = q / (R * 64), rr = (q >> 6) - w * R, l = q & 63;
            const uint64_t mk = wmask[w * kFuseRounds + rr];
            const uint64_t bl = l ? (~0ull >> (64 - l)) : 0ull;
            return wpre[w * kFuseRounds + rr] + (uint32_t)__popcll(mk & bl);
        };
        for (int x = t; x < 3 * nsub; x += kFuseT) {
            const int c = x / 3, a = x - 3 * c;
            const uint64_t ci = cinfo[c];
            if (splits(ci)) sfirst[a * kFuseC + c] = prefix(a * m + c_first(ci));
        }
        __syncthreads();
#pragma unroll 4
        for (int rr = 0; rr < R; ++rr) {
            const int q = (wave * R + rr) * 64 + lane;
            if (q < 3 * m) {
                const int a = q >= m ? (q >= 2 * m ? 2 : 1) : 0;
                const int k = q - a * m;
                const int c = pcl[k];
                const uint64_t ci = cinfo[c];
                int pos = k;
                if (splits(ci)) {
                    const uint64_t mk = mymask[rr];
                    const int f = c_first(ci), nl = c_count(ci) / 2;
                    const int lr = (int)(mypre[rr] + (uint32_t)__popcll(mk & below) -
                                         sfirst[a * kFuseC + c]);
                    pos = ((mk >> lane) & 1ull) ? f + lr : f + nl + (k - f - lr);
                }
                L(cur ^ 1, a, pos) = L(cur, a, k);
            }
        }
        __syncthreads();
        for (int k = t; k < m; k += kFuseT) {
            const int c = pcl[k];
            const uint64_t ci = cinfo[c];
            if (splits(ci)) pcl[k] = (k - c_first(ci) < c_count(ci) / 2) ? c_child0(ci) : cch1[c];
        }
        cur ^= 1;
        __syncthreads();
    }
    // leaves: particles in ascending caller index
    uint32_t* gid = reinterpret_cast<uint32_t*>(&lst[(cur ^ 1) * 3 * kFuseM]);
    __syncthreads();
    for (int k = t; k < m; k += kFuseT) gid[k] = l0[L(cur, 0, k)];
    __syncthreads();
    for (int k = t; k < m; k += kFuseT) {
        const uint64_t ci = cinfo[pcl[k]];
        const int f = c_first(ci), e = f + c_count(ci);
        const uint32_t id = gid[k];
        int rank = 0;
        for (int q = f; q < e; ++q) rank += gid[q] < id ? 1 : 0;
        perm[base + f + rank] = (int32_t)id;
    }
}

// Centre, half size and radius of every cell (the host planner's formulas).
// What the dual walk reads of a cell, in one 80-byte record: centre and
// radius, half sizes, and (leaf id, child 0, child 1, box).
struct WalkCell {
    double4 c;
    double4 h;
    int4 info;
};

__global__ void k_geom(int nc, const double* __restrict__ clo, const double* __restrict__ chi,
                       const int4* __restrict__ cell, const int4* __restrict__ aux,
                       double4* __restrict__ cellc, WalkCell* __restrict__ wcell,
                       double4* __restrict__ leafc) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= nc) return;
    double cc[3], h[3];
    double rad;
    {
#pragma clang fp contract(off)
        for (int a = 0; a < 3; ++a) {
            const double lo = clo[3 * (size_t)c + a], hi = chi[3 * (size_t)c + a];
            cc[a] = 0.5 * (lo + hi);
            h[a] = 0.5 * (hi - lo);
        }
        rad = sqrt((h[0] * h[0] + h[1] * h[1]) + h[2] * h[2]);
    }
    cellc[c] = make_double4(cc[0], cc[1], cc[2], rad);
    const int lf = cell[c].w;
    const int4 ax = aux[c];
    WalkCell w;
    w.c = make_double4(cc[0], cc[1], cc[2], rad);
    w.h = make_double4(h[0], h[1], h[2], 0.0);
    w.info = make_int4(lf, ax.x, ax.y, ax.z);
    wcell[c] = w;
    if (lf >= 0) leafc[lf] = make_double4(cc[0], cc[1], cc[2], 0.0);
}

__device__ __forceinline__ uint32_t wave_excl_scan(uint32_t v, uint32_t* total) {
    const int lane = threadIdx.x & 63;
    uint32_t x = v;
    for (int off = 1; off < 64; off <<= 1) {
        const uint32_t y = __shfl_up(x, off);
        if (lane >= off) x += y;
    }
    *total = __shfl(x, 63);
    return x - v;
}

// Appends `cnt` items per lane at one atomic per wavefront; returns the
// lane's first slot.
__device__ __forceinline__ uint32_t wave_append(uint32_t cnt, uint32_t* counter) {
    uint32_t total;
    const uint32_t off = wave_excl_scan(cnt, &total);
    uint32_t base = 0;
    if (total != 0) {
        if ((threadIdx.x & 63) == 0) base = atomicAdd(counter, total);
        base = __shfl(base, 0);
    }
    return base + off;
}

// Classification of one cell pair (the dual-walk rules of the host planner).
//
// Only half of the walk is visited: every rule is symmetric under
// (t, u, s) -> (u, t, s') with s' = 26 - s the opposite image (R changes
// sign exactly, |R| and the half sizes do not change, and a tie splits both
// cells), so the pairs with s > 13, or s = 13 and t <= u, are walked and
// each result is also emitted mirrored.  Cells are in pre-order, so two
// different cells of a walked pair have disjoint subtrees and the order of
// t and u carries over to all their descendants; only a self pair (t, t, 13)
// drops its child pair (c1, c0), the mirror of (c0, c1).
struct WalkOut {
    uint32_t n_child, n_p2p, n_m2l;
    int2 child[4];
    uint64_t key[2];
};

// Task key (a << ks) | (b << 5) | s with ks = 5 + bits of the largest id:
// sorting it gives the canonical (a, b, s) order with as few radix passes
// as the ids need.
__device__ __forceinline__ uint64_t walk_key(int a, int b, int s, int ks) {
    return ((uint64_t)(uint32_t)a << ks) | ((uint64_t)(uint32_t)b << 5) | (uint64_t)s;
}

__device__ __forceinline__ void walk_classify(const int2 pr, const WalkBox* __restrict__ wbox,
                                              const WalkCell* __restrict__ wcell, int2 ks,
                                              WalkOut& o) {
    const int t = pr.x, u = pr.y >> 5, s = pr.y & 31;
    const WalkCell wt = wcell[t], wu = wcell[u];
    const int4 at = make_int4(wt.info.y, wt.info.z, wt.info.w, 0);
    const int4 au = make_int4(wu.info.y, wu.info.z, wu.info.w, 0);
    const WalkBox wb = wbox[wt.info.w];
    const double4 ct = wt.c, cu = wu.c, ht = wt.h, hu = wu.h;
    const double sL[3] = {(double)(s % 3 - 1) * wb.L, (double)((s / 3) % 3 - 1) * wb.L,
                          (double)(s / 9 - 1) * wb.L};
    const double cta[3] = {ct.x, ct.y, ct.z}, cua[3] = {cu.x, cu.y, cu.z};
    const double hta[3] = {ht.x, ht.y, ht.z}, hua[3] = {hu.x, hu.y, hu.z};
    double R[3], A[3], H[3], gp[3], gap2, dmax2 = 0.0, R2 = 0.0, lhs = 0.0;
    {
#pragma clang fp contract(off)
        for (int a = 0; a < 3; ++a) {
            R[a] = (cua[a] - cta[a]) + sL[a];
            A[a] = fabs(R[a]);
            H[a] = hta[a] + hua[a];
            const double g = A[a] - H[a];
            gp[a] = g > 0.0 ? g : 0.0;
        }
        gap2 = (gp[0] * gp[0] + gp[1] * gp[1]) + gp[2] * gp[2];
        if (wb.use_m2l) {
            const double d0 = A[0] + H[0], d1 = A[1] + H[1], d2 = A[2] + H[2];
            dmax2 = (d0 * d0 + d1 * d1) + d2 * d2;
            R2 = (R[0] * R[0] + R[1] * R[1]) + R[2] * R[2];
            lhs = ct.w + cu.w;
            lhs = lhs * lhs;
            R2 = wb.th2 * R2;
        }
    }
    if (!(gap2 < wb.rc2_drop)) return;
    const bool self = (t == u) && (s == 13);
    if (wb.use_m2l && wb.centre_cut && lhs < R2) {
        // centre-distance cut: R2 holds theta^2 |R|^2, so recompute |R|^2
        double Rc2;
        {
#pragma clang fp contract(off)
            Rc2 = (R[0] * R[0] + R[1] * R[1]) + R[2] * R[2];
        }
        if (!(Rc2 < wb.rc2)) return;
        o.n_m2l = self ? 1 : 2;
        o.key[0] = walk_key(t, u, s, ks.y);
        o.key[1] = walk_key(u, t, 26 - s, ks.y);
        return;
    }
    if (wb.use_m2l && !wb.centre_cut && dmax2 < wb.rc2_m2l && lhs < R2) {
        o.n_m2l = self ? 1 : 2;
        o.key[0] = walk_key(t, u, s, ks.y);
        o.key[1] = walk_key(u, t, 26 - s, ks.y);
        return;
    }
    const int lt = wt.info.x, lu = wu.info.x;
    const double rt = ct.w, ru = cu.w;
    if (lt >= 0 && lu >= 0) {
        o.n_p2p = self ? 1 : 2;
        o.key[0] = walk_key(lt, lu, s, ks.x);
        o.key[1] = walk_key(lu, lt, 26 - s, ks.x);
    } else if (self) {
        o.child[0] = make_int2(at.x, (at.x << 5) | s);
        o.child[1] = make_int2(at.x, (at.y << 5) | s);
        o.child[2] = make_int2(at.y, (at.y << 5) | s);
        o.n_child = 3;
    } else if (lt < 0 && (lu >= 0 || rt > ru)) {
        o.child[0] = make_int2(at.x, pr.y);
        o.child[1] = make_int2(at.y, pr.y);
        o.n_child = 2;
    } else if (lu < 0 && (lt >= 0 || ru > rt)) {
        o.child[0] = make_int2(t, (au.x << 5) | s);
        o.child[1] = make_int2(t, (au.y << 5) | s);
        o.n_child = 2;
    } else {
        o.child[0] = make_int2(at.x, (au.x << 5) | s);
        o.child[1] = make_int2(at.x, (au.y << 5) | s);
        o.child[2] = make_int2(at.y, (au.x << 5) | s);
        o.child[3] = make_int2(at.y, (au.y << 5) | s);
        o.n_child = 4;
    }
}

// One level of the walk, frontier size known on the host.
__global__ void __launch_bounds__(256)
k_walk(const int2* __restrict__ front, int nf, int2* __restrict__ next,
       const WalkBox* __restrict__ wbox, const WalkCell* __restrict__ wcell, int2 ks,
       uint32_t* __restrict__ counters, uint64_t* __restrict__ p2p_keys,
       uint64_t* __restrict__ m2l_keys) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    WalkOut o{0u, 0u, 0u, {}, {0ull, 0ull}};
    if (k < nf) walk_classify(front[k], wbox, wcell, ks, o);
    const uint32_t cslot = wave_append(o.n_child, &counters[0]);
    for (uint32_t q = 0; q < o.n_child; ++q) next[cslot + q] = o.child[q];
    const uint32_t pslot = wave_append(o.n_p2p, &counters[1]);
    for (uint32_t q = 0; q < o.n_p2p; ++q) p2p_keys[pslot + q] = o.key[q];
    const uint32_t mslot = wave_append(o.n_m2l, &counters[2]);
    for (uint32_t q = 0; q < o.n_m2l; ++q) m2l_keys[mslot + q] = o.key[q];
}

// One level of the walk with the frontier size read on the device (no host
// round trip between levels).  Capacities are checked; an overflow is
// reported and the host then redoes the walk level by level.  The appends
// are aggregated per workgroup (one atomic per counter per 1024 pairs):
// all workgroups add to the same three counters, and at one atomic per
// wavefront those additions, serialised at one address, took most of a
// level's time.
// ctl: [0] p2p total, [1] m2l total, [2] overflow flag, [3] largest frontier;
// sizes[it] = frontier size of level it.
constexpr int kWalkT = 1024;
// frontiers up to this size go to the one-workgroup top of the walk
constexpr uint32_t kWalkTopMax = 4 * kWalkT;

// Appends one group's outputs (a WalkOut per thread of the workgroup): the
// keys to the key arrays and the child pairs to `next` at slots reserved
// from *next_count, or, with `lch`, to that workgroup-local array from 0.
// One atomic per counter per group.  Returns the group's child count.
__device__ __forceinline__ uint32_t walk_emit(const WalkOut& o, int2* __restrict__ next,
                                              uint32_t* __restrict__ next_count,
                                              uint32_t cap_front, int2* lch,
                                              uint32_t* __restrict__ ctl, uint32_t cap_p2p,
                                              uint32_t cap_m2l, uint64_t* __restrict__ p2p_keys,
                                              uint64_t* __restrict__ m2l_keys, uint64_t* wtot,
                                              uint32_t* bbase) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    // packed counts: children (<= 4096 per group) | p2p << 16 | m2l << 32
    const uint64_t v = (uint64_t)o.n_child | ((uint64_t)o.n_p2p << 16) |
                       ((uint64_t)o.n_m2l << 32);
    uint64_t x = v;
    for (int off = 1; off < 64; off <<= 1) {
        const uint64_t y = __shfl_up(x, off);
        if (lane >= off) x += y;
    }
    if (lane == 63) wtot[wave] = x;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint64_t run = 0;
        for (int w = 0; w < kWalkT / 64; ++w) {
            const uint64_t tw = wtot[w];
            wtot[w] = run;
            run += tw;
        }
        const uint32_t tc = (uint32_t)(run & 0xffffu), tp = (uint32_t)((run >> 16) & 0xffffu),
                       tm = (uint32_t)(run >> 32);
        bbase[0] = (tc != 0 && lch == nullptr) ? atomicAdd(next_count, tc) : 0u;
        bbase[1] = tp ? atomicAdd(&ctl[0], tp) : 0u;
        bbase[2] = tm ? atomicAdd(&ctl[1], tm) : 0u;
        bbase[3] = tc;
    }
    __syncthreads();
    const uint64_t off = wtot[wave] + x - v;
    const uint32_t cslot = bbase[0] + (uint32_t)(off & 0xffffu);
    const uint32_t pslot = bbase[1] + (uint32_t)((off >> 16) & 0xffffu);
    const uint32_t mslot = bbase[2] + (uint32_t)(off >> 32);
    // (fixed trip counts: the WalkOut arrays stay in registers)
    if (lch != nullptr) {
#pragma unroll
        for (uint32_t q = 0; q < 4; ++q)
            if (q < o.n_child) lch[cslot + q] = o.child[q];
    } else if (cslot + o.n_child <= cap_front) {
#pragma unroll
        for (uint32_t q = 0; q < 4; ++q)
            if (q < o.n_child) next[cslot + q] = o.child[q];
    } else if (o.n_child) {
        ctl[2] = 1u;
    }
#pragma unroll
    for (uint32_t q = 0; q < 2; ++q) {
        if (q < o.n_p2p) {
            if (pslot + q < cap_p2p) p2p_keys[pslot + q] = o.key[q]; else ctl[2] = 1u;
        }
        if (q < o.n_m2l) {
            if (mslot + q < cap_m2l) m2l_keys[mslot + q] = o.key[q]; else ctl[2] = 1u;
        }
    }
    const uint32_t tc = bbase[3];
    __syncthreads();   // wtot, bbase (and lch, for its readers) are reused next
    return tc;
}

// One level's share of workgroup `blk` of `nblk` (nf pairs in front).
// Returns false when the frontier is beyond its capacity.
__device__ __forceinline__ bool walk_level(const int2* __restrict__ front, int2* __restrict__ next,
                                           int it, uint32_t nf, uint32_t blk, uint32_t nblk,
                                           uint32_t* __restrict__ sizes, uint32_t* __restrict__ ctl,
                                           uint32_t cap_front, uint32_t cap_p2p, uint32_t cap_m2l,
                                           const WalkBox* __restrict__ wbox,
                                           const WalkCell* __restrict__ wcell, int2 ks,
                                           uint64_t* __restrict__ p2p_keys,
                                           uint64_t* __restrict__ m2l_keys, uint64_t* wtot,
                                           uint32_t* bbase) {
    if (nf > cap_front) return false;
    const uint32_t stride = nblk * blockDim.x;
    for (uint32_t base = blk * blockDim.x; base < nf; base += stride) {
        const uint32_t k = base + threadIdx.x;
        WalkOut o{0u, 0u, 0u, {}, {0ull, 0ull}};
        if (k < nf) walk_classify(front[k], wbox, wcell, ks, o);
        (void)walk_emit(o, next, &sizes[it + 1], cap_front, nullptr, ctl, cap_p2p, cap_m2l,
                        p2p_keys, m2l_keys, wtot, bbase);
    }
    if (blk == 0 && threadIdx.x == 0) atomicMax(&ctl[3], nf);
    return true;
}

// Levels it and it + 1 of the walk in workgroup `blk` of `nblk`: each
// workgroup classifies a group of level it, keeps the group's child pairs
// (at most four per pair) in LDS (`lch`) and classifies them in turn; only
// their children (level it + 2) go to `next`.  The descendants of a pair
// depend on that pair alone, so the middle level needs no other
// workgroup's results and its pairs never go through global memory.
// sizes[it + 1] counts the middle level (for the next build's sizing).
// Two levels per launch took the 128^3 walk from 0.55 to 0.33 ms; three
// took 0.37 ms (the deeper a workgroup's subtree, the more the workgroups'
// shares differ).
__device__ __forceinline__ void walk_two(const int2* __restrict__ front, int2* __restrict__ next,
                                         int it, uint32_t nf, uint32_t blk, uint32_t nblk,
                                         uint32_t* __restrict__ sizes, uint32_t* __restrict__ ctl,
                                         uint32_t cap_front, uint32_t cap_p2p, uint32_t cap_m2l,
                                         const WalkBox* __restrict__ wbox,
                                         const WalkCell* __restrict__ wcell, int2 ks,
                                         uint64_t* __restrict__ p2p_keys,
                                         uint64_t* __restrict__ m2l_keys, uint64_t* wtot,
                                         uint32_t* bbase, int2* lch) {
    const uint32_t stride = nblk * blockDim.x;
    for (uint32_t base = blk * blockDim.x; base < nf; base += stride) {
        const uint32_t k = base + threadIdx.x;
        WalkOut o{0u, 0u, 0u, {}, {0ull, 0ull}};
        if (k < nf) walk_classify(front[k], wbox, wcell, ks, o);
        const uint32_t n1 = walk_emit(o, nullptr, nullptr, 0u, lch, ctl, cap_p2p, cap_m2l,
                                      p2p_keys, m2l_keys, wtot, bbase);
        if (threadIdx.x == 0 && n1 != 0) atomicAdd(&sizes[it + 1], n1);
        for (uint32_t r = 0; r < n1; r += blockDim.x) {
            const uint32_t j = r + threadIdx.x;
            WalkOut o2{0u, 0u, 0u, {}, {0ull, 0ull}};
            if (j < n1) walk_classify(lch[j], wbox, wcell, ks, o2);
            (void)walk_emit(o2, next, &sizes[it + 2], cap_front, nullptr, ctl, cap_p2p, cap_m2l,
                            p2p_keys, m2l_keys, wtot, bbase);
        }
    }
    if (blk == 0 && threadIdx.x == 0) atomicMax(&ctl[3], nf);
}

// Levels it and it + 1, the frontier size read on the device.
__global__ void __launch_bounds__(kWalkT)
k_walk_multi(const int2* __restrict__ front, int2* __restrict__ next, int it,
             uint32_t* __restrict__ sizes, uint32_t* __restrict__ ctl, uint32_t cap_front,
             uint32_t cap_p2p, uint32_t cap_m2l, const WalkBox* __restrict__ wbox,
             const WalkCell* __restrict__ wcell, int2 ks, uint64_t* __restrict__ p2p_keys,
             uint64_t* __restrict__ m2l_keys) {
    __shared__ uint64_t wtot[kWalkT / 64];
    __shared__ uint32_t bbase[4];
    __shared__ int2 lch[4 * kWalkT];
    const uint32_t nf = sizes[it];
    if (nf > cap_front) return;
    walk_two(front, next, it, nf, blockIdx.x, gridDim.x, sizes, ctl, cap_front, cap_p2p, cap_m2l,
             wbox, wcell, ks, p2p_keys, m2l_keys, wtot, bbase, lch);
}

// Launches of k_walk_top's steps: two levels per step, one for an odd last
// level; step q reads buffer q & 1 and writes the other, so the frontier of
// level `levels` ends in buffer walk_top_steps(levels) & 1.
constexpr int walk_top_steps(int levels) { return levels / 2 + (levels & 1); }

// The first frontier (each box's root against itself with the zero shift and
// the 13 shifts of code > 13, the canonical half) and the walk's first
// `levels` levels in one workgroup, two at a time: the top of the walk has
// frontiers of a few hundred pairs, where a launch per level costs more than
// the level.  The frontier sizes, which thread 0 adds to with atomics, are
// read back with atomic loads.
__global__ void __launch_bounds__(kWalkT)
k_walk_top(int nbox, const int32_t* __restrict__ box_root, int2* __restrict__ buf0,
           int2* __restrict__ buf1, int levels, uint32_t* __restrict__ sizes,
           uint32_t* __restrict__ ctl, uint32_t cap_front, uint32_t cap_p2p, uint32_t cap_m2l,
           const WalkBox* __restrict__ wbox, const WalkCell* __restrict__ wcell, int2 ks,
           uint64_t* __restrict__ p2p_keys, uint64_t* __restrict__ m2l_keys) {
    __shared__ uint64_t wtot[kWalkT / 64];
    __shared__ uint32_t bbase[4];
    __shared__ int2 lch[4 * kWalkT];
    const uint32_t nf0 = (uint32_t)(14 * nbox);
    for (uint32_t q = threadIdx.x; q < nf0; q += blockDim.x) {
        const int b = (int)(q / 14), j = (int)(q - 14 * (uint32_t)b);
        const int root = box_root[b];
        buf0[q] = make_int2(root, (root << 5) | (13 + j));
    }
    if (threadIdx.x == 0) sizes[0] = nf0;
    __syncthreads();
    int step = 0;
    for (int it = 0; it < levels; ++step) {
        const uint32_t nf = it == 0 ? nf0
                                    : __hip_atomic_load(&sizes[it], __ATOMIC_RELAXED,
                                                        __HIP_MEMORY_SCOPE_AGENT);
        if (nf > cap_front) return;
        const int2* front = (step & 1) ? buf1 : buf0;
        int2* next = (step & 1) ? buf0 : buf1;
        if (it + 2 <= levels) {
            walk_two(front, next, it, nf, 0u, 1u, sizes, ctl, cap_front, cap_p2p, cap_m2l, wbox,
                     wcell, ks, p2p_keys, m2l_keys, wtot, bbase, lch);
            it += 2;
        } else {
            (void)walk_level(front, next, it, nf, 0u, 1u, sizes, ctl, cap_front, cap_p2p,
                             cap_m2l, wbox, wcell, ks, p2p_keys, m2l_keys, wtot, bbase);
            it += 1;
        }
        __syncthreads();
    }
}

// Smallest target / source depth of the walk's M2L keys (key = t << ks |
// u << 5 | s), kept as 0x7fffffff - depth by atomicMax into zeroed words
// out[0] (targets) and out[1] (sources); the key count is *count.
__global__ void k_m2l_depths(const uint64_t* __restrict__ keys, const uint32_t* __restrict__ count,
                             uint32_t cap, int ks, const int4* __restrict__ aux,
                             uint32_t* __restrict__ out) {
    const uint32_t n = min(*count, cap);
    uint32_t bt = 0u, bs = 0u;
    for (uint32_t k = blockIdx.x * blockDim.x + threadIdx.x; k < n; k += gridDim.x * blockDim.x) {
        const uint64_t key = keys[k];
        const int t = (int)(key >> ks), u = (int)((key & ((1ull << ks) - 1ull)) >> 5);
        bt = max(bt, 0x7fffffffu - (uint32_t)aux[t].w);
        bs = max(bs, 0x7fffffffu - (uint32_t)aux[u].w);
    }
    if (bt) atomicMax(&out[0], bt);
    if (bs) atomicMax(&out[1], bs);
}

__global__ void k_zero_u32(uint32_t* p, int n) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0u;
}

// CSR rows from the walk's unsorted keys (row << ks | value): each key takes
// a slot in its row with an atomic count, the counts are scanned into the
// row starts, the values are placed, and each row's values are sorted
// (bitonic, in LDS), which gives the canonical (i, j, shift) order since the
// values of one row are distinct.
__global__ void k_row_count(const uint64_t* __restrict__ keys, int64_t nk, int ks,
                            int32_t* __restrict__ cnt, int32_t* __restrict__ slot) {
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k < nk) slot[k] = atomicAdd(&cnt[keys[k] >> ks], 1);
}

__global__ void k_row_place(const uint64_t* __restrict__ keys, int64_t nk, int ks,
                            const int32_t* __restrict__ row, const int32_t* __restrict__ slot,
                            int32_t* __restrict__ vals) {
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= nk) return;
    const uint64_t key = keys[k];
    vals[row[key >> ks] + slot[k]] = (int32_t)(key & ((1ull << ks) - 1));
}

// Ascending bitonic sort of b[0, P) (P a power of two) by the T threads of
// the workgroup; t is the caller's thread index.
__device__ void bitonic_sort(int32_t* b, int P, int t, int T) {
    for (int size = 2; size <= P; size <<= 1) {
        for (int stride = size >> 1; stride > 0; stride >>= 1) {
            for (int p = t; p < P / 2; p += T) {
                const int lo = 2 * p - (p & (stride - 1)), hi = lo + stride;
                const bool up = (lo & size) == 0;
                const int32_t x = b[lo], y = b[hi];
                if ((x > y) == up) {
                    b[lo] = y;
                    b[hi] = x;
                }
            }
            __syncthreads();
        }
    }
}

__device__ __forceinline__ int pow2_at_least(int n) {
    int P = 1;
    while (P < n) P <<= 1;
    return P;
}

// One wavefront per row of at most kRowShort values; longer rows are listed
// for k_row_sort_long.
constexpr int kRowShort = 256;
constexpr int kRowLds = 8192;

__global__ void __launch_bounds__(64)
k_row_sort_short(const int32_t* __restrict__ row, int32_t* __restrict__ vals,
                 int32_t* __restrict__ longs, int32_t* __restrict__ nlong) {
    __shared__ int32_t b[kRowShort];
    const int r = blockIdx.x, t = threadIdx.x;
    const int r0 = row[r], len = row[r + 1] - r0;
    if (len <= 1) return;
    if (len > kRowShort) {
        if (t == 0) longs[atomicAdd(nlong, 1)] = r;
        return;
    }
    const int P = pow2_at_least(len);
    for (int k = t; k < P; k += 64) b[k] = k < len ? vals[r0 + k] : INT32_MAX;
    __syncthreads();
    bitonic_sort(b, P, t, 64);
    for (int k = t; k < len; k += 64) vals[r0 + k] = b[k];
}

// The listed long rows, one workgroup at a time each: in LDS up to lds_cap
// (<= kRowLds) values, else in scratch[2 r0, 2 r0 + P) (P < 2 len, so rows
// never share scratch; the caller provides twice the value count).
__global__ void __launch_bounds__(256)
k_row_sort_long(const int32_t* __restrict__ row, int32_t* __restrict__ vals,
                const int32_t* __restrict__ longs, const int32_t* __restrict__ nlong,
                int32_t* __restrict__ scratch, int lds_cap) {
    __shared__ int32_t lds[kRowLds];
    const int t = threadIdx.x;
    const int count = *nlong;
    for (int q = blockIdx.x; q < count; q += gridDim.x) {
        const int r = longs[q];
        const int r0 = row[r], len = row[r + 1] - r0;
        const int P = pow2_at_least(len);
        int32_t* b = P <= lds_cap ? lds : scratch + 2 * (size_t)r0;
        for (int k = t; k < P; k += 256) b[k] = k < len ? vals[r0 + k] : INT32_MAX;
        __syncthreads();
        bitonic_sort(b, P, t, 256);
        for (int k = t; k < len; k += 256) vals[r0 + k] = b[k];
        __syncthreads();
    }
}

// M2L sources and shifts from the sorted row values, and the smallest
// depth of the tasks' source and target cells (mindep[0] / mindep[1],
// preset to INT32_MAX).
__global__ void k_m2l_split(const int32_t* __restrict__ row, int nrows, const int32_t* __restrict__ vals,
                            const int4* __restrict__ aux, int32_t* __restrict__ src,
                            int32_t* __restrict__ shift, int32_t* __restrict__ mindep) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= nrows) return;
    const int r0 = row[c], r1 = row[c + 1];
    if (r0 == r1) return;
    int dmin = INT32_MAX;
    for (int k = r0; k < r1; ++k) {
        const int u = vals[k] >> 5;
        src[k] = u;
        shift[k] = vals[k] & 31;
        dmin = min(dmin, aux[u].w);
    }
    atomicMin(&mindep[0], dmin);
    atomicMin(&mindep[1], aux[c].w);
}

__global__ void k_item_count(int nl, const int32_t* __restrict__ row, int chunk,
                             int32_t* __restrict__ cnt) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i > nl) return;
    if (i == nl) { cnt[i] = 0; return; }
    const int len = row[i + 1] - row[i];
    cnt[i] = (len + chunk - 1) / chunk;
}

// Work items of each TaskGroup row, one wavefront per row and one lane per
// item; the queue key is (segment of the slot) * 256 + 255 - (pair count >>
// cshift), so the sorted queue holds the kQueueSegs segments in order, each
// longest first up to 1/256 of the largest item.  Slots from the item count
// to `cap` get segment kQueueSegs (after every item in the stable sort).
// rowcand[i]: candidate pairs of row i; ctl[2]: the item count.
__global__ void k_items(int nl, const int32_t* __restrict__ row, const int32_t* __restrict__ js,
                        const int4* __restrict__ leaf, int chunk, int cshift,
                        const int32_t* __restrict__ slot0, int cap, int4* __restrict__ items,
                        uint64_t* __restrict__ cost_keys, uint32_t* __restrict__ slots,
                        unsigned long long* __restrict__ rowcand, uint32_t* __restrict__ ctl) {
    const int64_t gt = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int i = (int)(gt >> 6), lane = (int)(gt & 63);
    unsigned long long total = 0;
    if (i < nl) {
        const int r0 = row[i], len = row[i + 1] - r0;
        if (len > 0) {
            const int parts = (len + chunk - 1) / chunk;
            const int base = len / parts, extra = len % parts;
            const int ni = leaf[i].y;
            for (int k = lane; k < parts; k += 64) {
                const int t = r0 + k * base + min(k, extra);
                const int sz = base + (k < extra ? 1 : 0);
                // the tasks' source counts, eight loads in flight at a time
                unsigned long long c = 0;
                int q = t;
                for (; q + 8 <= t + sz; q += 8) {
                    int jv[8];
#pragma unroll
                    for (int u = 0; u < 8; ++u) jv[u] = js[q + u] >> 5;
#pragma unroll
                    for (int u = 0; u < 8; ++u) c += (unsigned long long)leaf[jv[u]].y;
                }
                for (; q < t + sz; ++q) c += (unsigned long long)leaf[js[q] >> 5].y;
                c *= (unsigned long long)ni;
                total += c;
                const int s = slot0[i] + k;
                items[s] = make_int4(i, t, t + sz, s);
                const unsigned long long b = c >> cshift;
                const uint64_t seg = (uint64_t)((int64_t)s * kQueueSegs / slot0[nl]);
                cost_keys[s] = (seg << 8) | (uint64_t)(255u - (b > 255ull ? 255u : (uint32_t)b));
                slots[s] = (uint32_t)s;
            }
        }
    }
    {
        // padding slots, spread over all threads of the grid
        const int n_items = slot0[nl];
        if (gt == 0) ctl[2] = (uint32_t)n_items;
        const int64_t stride = (int64_t)gridDim.x * blockDim.x;
        for (int64_t s = n_items + gt; s < cap; s += stride) {
            cost_keys[s] = ((uint64_t)kQueueSegs << 8) | 255u;
            slots[s] = (uint32_t)s;
        }
    }
    // the row's candidate pairs (summed by k_sum_rows: one atomic per row
    // on a single counter would serialise)
    for (int off = 32; off > 0; off >>= 1) total += __shfl_down(total, off);
    if (lane == 0 && i < nl) rowcand[i] = total;
}

// out = sum of v[0, n), by one workgroup of 1024 threads.
__global__ void __launch_bounds__(1024)
k_sum_rows(const unsigned long long* __restrict__ v, int n, unsigned long long* __restrict__ out) {
    __shared__ unsigned long long part[1024 / 64];
    unsigned long long x = 0;
    for (int i = threadIdx.x; i < n; i += 1024) x += v[i];
    for (int off = 32; off > 0; off >>= 1) x += __shfl_down(x, off);
    if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = x;
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long t = 0;
        for (int w = 0; w < 1024 / 64; ++w) t += part[w];
        *out = t;
    }
}

__global__ void k_check(const double* __restrict__ pos, const double* __restrict__ mass, int64_t n,
                        int* __restrict__ bad) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double x = pos[3 * i], y = pos[3 * i + 1], z = pos[3 * i + 2], m = mass[i];
    if (!(isfinite(x) && isfinite(y) && isfinite(z))) atomicMin(&bad[0], (int)i);
    if (!(isfinite(m) && m >= 0.0)) atomicMin(&bad[1], (int)i);
}

__global__ void k_fill_i32(int* p, int n, int v) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

inline unsigned grid_of(int64_t n, int b = 256) { return (unsigned)((n + b - 1) / b); }

int bits_for(uint64_t maxv) {
    int b = 0;
    while (b < 64 && (maxv >> b) != 0) ++b;
    return b;
}

#define TRY(expr)                                                                   \
    do {                                                                            \
        hipError_t e_ = (expr);                                                     \
        if (e_ != hipSuccess) return std::string(#expr) + ": " + hipGetErrorString(e_); \
    } while (0)

template <class T>
hipError_t up(DevBuf& b, const std::vector<T>& v, hipStream_t s) {
    hipError_t e = b.ensure(std::max<size_t>(16, v.size() * sizeof(T)));
    if (e != hipSuccess || v.empty()) return e;
    return hipMemcpyAsync(b.p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice, s);
}

// Sorts keys (and values) in place; swaps in the scratch buffers when the
// number of passes leaves the result there.
std::string sort_in_place(DevBuf& keys, DevBuf* vals, DevBuf& ktmp, DevBuf* vtmp, DevBuf& hist,
                          int64_t n, int bit_end, hipStream_t s) {
    if (n <= 1) return std::string();
    bit_end = std::min(64, (bit_end + 7) / 8 * 8);
    TRY(ktmp.ensure(n * 8));
    if (vals) TRY(vtmp->ensure(n * 4));
    TRY(hist.ensure((size_t)sort_hist_words(n) * 4));
    bool in_tmp = false;
    TRY(radix_sort_u64(keys.as<uint64_t>(), vals ? vals->as<uint32_t>() : nullptr, ktmp.as<uint64_t>(),
                       vtmp ? vtmp->as<uint32_t>() : nullptr, hist.as<uint32_t>(), n, 0, bit_end, s,
                       &in_tmp));
    if (in_tmp) {
        std::swap(keys, ktmp);
        if (vals) std::swap(*vals, *vtmp);
    }
    return std::string();
}

// LDS capacity of the long-row sort; PMFMM_ROW_LDS lowers it (tests use it
// to send rows through the scratch path).
int row_lds_cap() {
    const char* v = std::getenv("PMFMM_ROW_LDS");
    if (!v) return kRowLds;
    const int c = std::atoi(v);
    return c < 0 ? 0 : std::min(c, kRowLds);
}

// Wall-clock phases of the device planner, printed to stderr when the
// environment variable PMFMM_PLAN_TIMING is set (synchronises each phase).
struct PhaseTimer {
    bool on = std::getenv("PMFMM_PLAN_TIMING") != nullptr;
    hipStream_t s;
    std::chrono::steady_clock::time_point t = std::chrono::steady_clock::now();
    explicit PhaseTimer(hipStream_t st) : s(st) {}
    void lap(const char* what) {
        if (!on) return;
        (void)hipStreamSynchronize(s);
        auto now = std::chrono::steady_clock::now();
        std::fprintf(stderr, "[pmfmm gpu plan] %-10s %8.3f ms\n", what,
                     std::chrono::duration<double, std::milli>(now - t).count());
        t = now;
    }
};

}  // namespace

hipError_t gpu_enqueue_checks(DevPlan& d, const double* pos, const double* mass, int64_t n,
                              hipStream_t s) {
    hipError_t e = d.wcount.ensure(128);
    if (e != hipSuccess) return e;
    // wcount[0..1]: first bad position / mass (INT_MAX: none); wcount[2]:
    // the long-run flag of the coordinate sort
    hipLaunchKernelGGL(k_fill_i32, dim3(1), dim3(64), 0, s, reinterpret_cast<int*>(d.wcount.p), 2,
                       0x7fffffff);
    hipLaunchKernelGGL(k_fill_i32, dim3(1), dim3(64), 0, s, reinterpret_cast<int*>(d.wcount.p) + 2,
                       1, 0);
    hipLaunchKernelGGL(k_check, dim3(grid_of(n)), dim3(256), 0, s, pos, mass, n,
                       reinterpret_cast<int*>(d.wcount.p));
    return hipGetLastError();
}

hipError_t upload_topology(DevPlan& d, const Plan& topo, const BoxDev* boxdev, hipStream_t s) {
    const int64_t nc = (int64_t)topo.cells.size(), nl = (int64_t)topo.leaf_cell.size();
    std::vector<int32_t> cell(4 * nc), aux(4 * nc), leaf(4 * nl);
    for (int64_t k = 0; k < nc; ++k) {
        const Cell& c = topo.cells[k];
        cell[4 * k] = c.first;
        cell[4 * k + 1] = c.count;
        cell[4 * k + 2] = c.parent;
        cell[4 * k + 3] = c.leaf;
        aux[4 * k] = c.child[0];
        aux[4 * k + 1] = c.child[1];
        aux[4 * k + 2] = c.box;
        aux[4 * k + 3] = c.depth;
    }
    for (int64_t l = 0; l < nl; ++l) {
        const Cell& c = topo.cells[topo.leaf_cell[l]];
        leaf[4 * l] = c.first;
        leaf[4 * l + 1] = c.count;
        leaf[4 * l + 2] = c.box;
        leaf[4 * l + 3] = topo.leaf_cell[l];
    }
    const int nbox = (int)topo.boxes.size();
    std::vector<WalkBox> wb(nbox);
    std::vector<BoxDev> bd(boxdev, boxdev + nbox);
    for (int b = 0; b < nbox; ++b) {
        const BoxParams& p = topo.boxes[b];
        const double rc2 = p.r_cut * p.r_cut;
        wb[b].L = p.box;
        wb[b].rc2_drop = rc2 * (1.0 + kGuard);
        wb[b].rc2_m2l = rc2 * (1.0 - kGuard);
        wb[b].th2 = p.theta * p.theta;
        wb[b].use_m2l = (p.order >= 0 && p.theta > 0.0) ? 1 : 0;
        wb[b].centre_cut = p.m2l_cut == 1 ? 1 : 0;
        wb[b].rc2 = rc2;
    }
    std::vector<int32_t> bfc(topo.box_first_cell.begin(), topo.box_first_cell.end());
    d.walk_levels = 0;      // a new shape: size the walk level by level once

    // Subtrees finished by k_orb_fused: the highest cells with at most kFuseM
    // particles and kFuseC cells (cells are in pre-order, so a subtree is the
    // contiguous id range [c, c + sub[c])).  A leaf (<= 64 particles) always
    // qualifies, so the subtrees cover every leaf; the level loop partitions
    // the cells above them, all of which split.
    std::vector<int32_t> sub(nc, 1), deep(nc, 0);
    for (int64_t k = nc - 1; k >= 0; --k) {
        const Cell& c = topo.cells[k];
        deep[k] = c.depth;
        if (c.child[0] >= 0) {
            sub[k] = 1 + sub[c.child[0]] + sub[c.child[1]];
            deep[k] = std::max(deep[c.child[0]], deep[c.child[1]]);
        }
    }
    auto fusable = [&](int64_t k) {
        return topo.cells[k].count <= kFuseM && sub[k] <= kFuseC;
    };
    std::vector<int32_t> roots, split(nc, 0), loop_cells;
    std::vector<int32_t> loop_begin(1, 0);
    for (int64_t k = 0; k < nc; ++k) {
        const Cell& c = topo.cells[k];
        if (!fusable(k)) {
            if (c.child[0] < 0) return hipErrorInvalidValue;   // a leaf above kFuseM
            split[k] = 1;
        } else if (c.parent < 0 || !fusable(c.parent)) {
            roots.push_back((int32_t)k);
            roots.push_back(sub[k]);
            roots.push_back(c.depth);
            roots.push_back(deep[k]);
        }
    }
    for (int dep = 0; dep + 1 < (int)topo.depth_begin.size(); ++dep) {
        const size_t before = loop_cells.size();
        for (int q = topo.depth_begin[dep]; q < topo.depth_begin[dep + 1]; ++q)
            if (split[topo.cells_by_depth[q]]) loop_cells.push_back(topo.cells_by_depth[q]);
        if (loop_cells.size() == before) break;
        loop_begin.push_back((int32_t)loop_cells.size());
    }
    d.n_froots = (int)(roots.size() / 4);
    const std::vector<int32_t> sax0(nc, -1);
    d.loop_depth_begin = loop_begin;
    hipError_t e;
    if ((e = up(d.cell, cell, s)) != hipSuccess) return e;
    if ((e = up(d.cell_aux, aux, s)) != hipSuccess) return e;
    if ((e = up(d.leaf, leaf, s)) != hipSuccess) return e;
    if ((e = up(d.level_cells, topo.cells_by_depth, s)) != hipSuccess) return e;
    if ((e = up(d.loop_cells, loop_cells, s)) != hipSuccess) return e;
    // split axis per cell: -1 except for the level loop's cells, whose axis
    // k_cells_level writes at their level of every build
    if ((e = up(d.cell_axis, sax0, s)) != hipSuccess) return e;
    if ((e = up(d.froots, roots, s)) != hipSuccess) return e;
    if ((e = up(d.box_first, topo.box_first_particle, s)) != hipSuccess) return e;
    if ((e = up(d.walkbox, wb, s)) != hipSuccess) return e;
    if ((e = up(d.boxes, bd, s)) != hipSuccess) return e;
    if ((e = up(d.item_count, bfc, s)) != hipSuccess) return e;   // box -> root cell (scratch reuse)
    return hipStreamSynchronize(s);
}

std::string gpu_build_plan(DevPlan& d, const Plan& topo, const double* pos, const double* mass,
                           int chunk, hipStream_t s, PlanCounts& out, std::string* input_error,
                           const M2LReady& on_m2l, hipStream_t side) {
    input_error->clear();
    const int64_t n = topo.n;
    const int nbox = (int)topo.boxes.size();
    const int64_t nc = (int64_t)topo.cells.size(), nl = (int64_t)topo.leaf_cell.size();
    PhaseTimer clk(s);

    // ---- wrap, sort each axis by (coordinate, caller index)
    TRY(d.wpos.ensure(n * 24));
    TRY(d.keys.ensure(n * 24));
    TRY(d.plist.ensure(n * 12));
    TRY(d.plist_tmp.ensure(n * 12));
    TRY(d.keys_tmp.ensure(n * 24));
    const int key_bits = n <= kKey24Max ? 24 : 32;
    hipLaunchKernelGGL(k_wrap_keys, dim3(grid_of(n)), dim3(256), 0, s, pos, n,
                       d.box_first.as<int32_t>(), nbox, d.boxes.as<BoxDev>(), d.wpos.as<double>(),
                       d.keys.as<uint32_t>(), d.plist.as<uint32_t>(), key_bits);
    TRY(hipGetLastError());
    // the three axis lists are three segments of one sort: by the key,
    // then each run of equal keys by coordinate
    TRY(d.hist.ensure((size_t)sort_hist_words(n, 3) * 4));
    uint32_t* v = d.plist.as<uint32_t>();
    uint32_t* vt = d.plist_tmp.as<uint32_t>();
    bool in_tmp = false;
    if (n > 1) {
        TRY(radix_sort_u32(d.keys.as<uint32_t>(), v, d.keys_tmp.as<uint32_t>(), vt,
                           d.hist.as<uint32_t>(), n, 0, key_bits, s, &in_tmp, 3));
        if (in_tmp) {
            // the sorted keys and lists are the scratch buffers now
            std::swap(d.keys, d.keys_tmp);
            std::swap(d.plist, d.plist_tmp);
            v = d.plist.as<uint32_t>();
            vt = d.plist_tmp.as<uint32_t>();
        }
        hipLaunchKernelGGL(k_run_fix, dim3(grid_of(3 * n)), dim3(256), 0, s, d.keys.as<uint32_t>(), v,
                           n, d.wpos.as<double>(), reinterpret_cast<int*>(d.wcount.p) + 2);
        TRY(hipGetLastError());
    }
    // The input checks (wcount[0..1]) and the long-run flag (wcount[2]) come
    // back with the walk's counts, in the same round trip: with bad input
    // the tree is built on wrapped (finite) coordinates and then dropped;
    // with a long run the build is redone with the 64-bit sort (force64).
    {
        if (d.force64) {
            // coordinates closer than the key resolves, out of order
            // in a long run: sort by the full keys
            uint64_t* k = d.keys.as<uint64_t>();
            uint64_t* kt = d.keys_tmp.as<uint64_t>();
            hipLaunchKernelGGL(k_keys64, dim3(grid_of(n)), dim3(256), 0, s, d.wpos.as<double>(), n, k,
                               v);
            TRY(hipGetLastError());
            TRY(radix_sort_u64(k, v, kt, vt, d.hist.as<uint32_t>(), n, 0, 64, s, &in_tmp, 3));
            if (in_tmp) TRY(hipMemcpyAsync(v, vt, n * 12, hipMemcpyDeviceToDevice, s));
        }
    }
    if (n > 1 && nbox > 1) {
        // then stably by box: each box's particles in coordinate order
        uint32_t* k = d.keys.as<uint32_t>();
        hipLaunchKernelGGL(k_box_keys, dim3(grid_of(3 * n)), dim3(256), 0, s, v, 3 * n,
                           d.box_first.as<int32_t>(), nbox, k);
        TRY(hipGetLastError());
        TRY(radix_sort_u32(k, v, d.keys_tmp.as<uint32_t>(), vt, d.hist.as<uint32_t>(), n, 0,
                           bits_for(nbox - 1) + 1, s, &in_tmp, 3));
        if (in_tmp) TRY(hipMemcpyAsync(v, vt, n * 12, hipMemcpyDeviceToDevice, s));
    }

    clk.lap("sort");
    // ---- ORB levels
    TRY(d.pc.ensure(n * 4));
    TRY(d.pc_tmp.ensure(n * 4));
    // mark bytes at 0, mark bits at bits_off; k_orb_fused reuses the buffer
    // for n int32
    const int64_t bits_off = (n + 255) / 256 * 256;
    TRY(d.flag.ensure(std::max<int64_t>(n * 4, bits_off + (n + 63) / 64 * 8)));
    uint64_t* bits = reinterpret_cast<uint64_t*>(d.flag.as<uint8_t>() + bits_off);
    const int64_t lv_tiles = (n + kLvTile - 1) / kLvTile;
    TRY(d.lv_first.ensure(nc * 4));
    // per-list tile sums, their scan (large n) and the scan's scratch
    TRY(d.tile_sums.ensure((6 * lv_tiles + sort_tiles(3 * lv_tiles)) * 4 + 16));
    TRY(d.clo.ensure(nc * 24));
    TRY(d.chi.ensure(nc * 24));
    TRY(d.cell_axis.ensure(nc * 4));
    hipLaunchKernelGGL(k_init_pc, dim3(grid_of(n)), dim3(256), 0, s, n, d.box_first.as<int32_t>(),
                       d.item_count.as<int32_t>(), nbox, d.pc.as<int32_t>());
    TRY(hipGetLastError());
    // the level loop partitions the cells above the fused subtrees
    const int nloop = (int)d.loop_depth_begin.size() - 1;
    for (int dep = 0; dep < nloop; ++dep) {
        const int c0 = d.loop_depth_begin[dep], ncd = d.loop_depth_begin[dep + 1] - c0;
        hipLaunchKernelGGL(k_cells_level, dim3(1), dim3(kCellsT), 0, s,
                           d.loop_cells.as<int32_t>() + c0, ncd, d.cell.as<int4>(),
                           d.cell_aux.as<int4>(), d.plist.as<uint32_t>(), n, d.wpos.as<double>(),
                           d.clo.as<double>(), d.chi.as<double>(), d.cell_axis.as<int32_t>(),
                           d.lv_first.as<int32_t>());
        TRY(hipGetLastError());
        hipLaunchKernelGGL(k_flag, dim3(grid_of(n)), dim3(256), 0, s, n, d.pc.as<int32_t>(),
                           d.cell.as<int4>(), d.cell_axis.as<int32_t>(), d.plist.as<uint32_t>(),
                           d.flag.as<uint8_t>());
        hipLaunchKernelGGL(k_pack_marks, dim3(grid_of(n)), dim3(256), 0, s, n,
                           d.flag.as<uint8_t>(), bits);
        hipLaunchKernelGGL(k_level_sums, dim3(lv_tiles), dim3(kLvThreads), 0, s, n,
                           d.pc.as<int32_t>(), d.cell_axis.as<int32_t>(), d.cell.as<int4>(),
                           d.plist.as<uint32_t>(), bits, d.tile_sums.as<uint32_t>(), (int)lv_tiles);
        TRY(hipGetLastError());
        if (lv_tiles <= kLvSumMax) {
            hipLaunchKernelGGL(k_level_move<false>, dim3(lv_tiles), dim3(kLvThreads), 0, s, n,
                               d.pc.as<int32_t>(), d.pc_tmp.as<int32_t>(), d.cell.as<int4>(),
                               d.cell_aux.as<int4>(), d.cell_axis.as<int32_t>(),
                               d.plist.as<uint32_t>(), d.plist_tmp.as<uint32_t>(), bits,
                               d.tile_sums.as<uint32_t>(), nullptr, (int)lv_tiles,
                               d.lv_first.as<int32_t>());
        } else {
            uint32_t* offs = d.tile_sums.as<uint32_t>() + 3 * lv_tiles;
            TRY(exclusive_scan_i32(d.tile_sums.as<int32_t>(), reinterpret_cast<int32_t*>(offs),
                                   3 * lv_tiles, offs + 3 * lv_tiles, s));
            hipLaunchKernelGGL(k_level_move<true>, dim3(lv_tiles), dim3(kLvThreads), 0, s, n,
                               d.pc.as<int32_t>(), d.pc_tmp.as<int32_t>(), d.cell.as<int4>(),
                               d.cell_aux.as<int4>(), d.cell_axis.as<int32_t>(),
                               d.plist.as<uint32_t>(), d.plist_tmp.as<uint32_t>(), bits,
                               d.tile_sums.as<uint32_t>(), offs, (int)lv_tiles,
                               d.lv_first.as<int32_t>());
        }
        TRY(hipGetLastError());
        std::swap(d.plist, d.plist_tmp);
        std::swap(d.pc, d.pc_tmp);
    }
    // the subtrees below, each in one workgroup; leaves into perm
    TRY(d.perm.ensure(n * 4));
    hipLaunchKernelGGL(k_orb_fused, dim3(d.n_froots), dim3(kFuseT), 0, s, d.froots.as<int4>(),
                       d.cell.as<int4>(), d.cell_aux.as<int4>(), d.plist.as<uint32_t>(), n,
                       d.wpos.as<double>(), d.flag.as<int32_t>(), d.clo.as<double>(),
                       d.chi.as<double>(), d.perm.as<int32_t>());
    TRY(hipGetLastError());

    clk.lap("levels");
    // ---- leaf order, geometry, particle records
    TRY(d.leafc.ensure(nl * 32));
    TRY(d.cellc.ensure(nc * 32));
    TRY(d.wcell.ensure(nc * sizeof(WalkCell)));
    hipLaunchKernelGGL(k_geom, dim3(grid_of(nc)), dim3(256), 0, s, (int)nc, d.clo.as<double>(),
                       d.chi.as<double>(), d.cell.as<int4>(), d.cell_aux.as<int4>(),
                       d.cellc.as<double4>(), d.wcell.as<WalkCell>(), d.leafc.as<double4>());
    TRY(hipGetLastError());
    TRY(d.x64.ensure(n * 32));
    TRY(d.x32.ensure(n * 16));
    GatherArgs g{pos, mass, d.perm.as<int32_t>(), d.leaf.as<int4>(), d.leafc.as<double4>(),
                 d.boxes.as<BoxDev>(), d.x64.as<double4>(), d.x32.as<float4>(), (int32_t)nl};
    // With a side stream the particle records are gathered there, beside the
    // walk (which reads only the cells); s waits for them before the build
    // returns (and before any early return).
    const bool side_gather = side != nullptr && side != s;
    if (side_gather) {
        for (hipEvent_t* e : {&d.geom_ev, &d.gather_ev})
            if (!*e) TRY(hipEventCreateWithFlags(e, hipEventDisableTiming));
        TRY(hipEventRecord(d.geom_ev, s));
        TRY(hipStreamWaitEvent(side, d.geom_ev, 0));
        TRY(launch_gather(g, nullptr, side));
        TRY(hipEventRecord(d.gather_ev, side));
    } else {
        TRY(launch_gather(g, nullptr, s));
    }
    auto join_gather = [&]() -> hipError_t {
        return side_gather ? hipStreamWaitEvent(s, d.gather_ev, 0) : hipSuccess;
    };

    clk.lap("records");
    // ---- dual walk
    TRY(d.wcount.ensure(128));
    // the canonical half of (root, root, s): the zero shift and the 13
    // shifts with code > 13
    const int64_t nf0 = 14 * (int64_t)nbox;
    std::vector<int32_t> f0(2 * nf0);
    for (int b = 0; b < nbox; ++b)
        for (int q = 0; q < 14; ++q) {
            const int root = topo.box_first_cell[b];
            f0[2 * (14 * b + q)] = root;
            f0[2 * (14 * b + q) + 1] = (root << 5) | (13 + q);
        }
    int64_t n_p2p = 0, n_m2l = 0;
    int32_t dmin_src = 0x7fffffff, dmin_tgt = 0x7fffffff;
    bool done = false;
    int flags[3] = {0, 0, 0};
    bool have_flags = false;
    const int2 ks = make_int2(5 + bits_for((uint64_t)std::max<int64_t>(1, nl - 1)),
                              5 + bits_for((uint64_t)std::max<int64_t>(1, nc - 1)));
    // Level-by-level walk without host round trips, sized from the previous
    // build of the same tree shape; falls back to the host-driven loop.
    if (d.walk_cap_front > 0 && d.walk_levels > 0) {
        const uint32_t capf = d.walk_cap_front, capp = d.walk_cap_p2p, capm = d.walk_cap_m2l;
        const int L = d.walk_levels;
        TRY(d.front.ensure((size_t)std::max<int64_t>(capf, nf0) * 8));
        TRY(d.front_next.ensure((size_t)capf * 8));
        TRY(d.p2p_keys.ensure((size_t)capp * 8));
        TRY(d.m2l_keys.ensure((size_t)std::max<uint32_t>(capm, 1) * 8));
        DevBuf* bufs[2] = {&d.front, &d.front_next};
        // the top levels in one workgroup while the last build's frontiers
        // were small (any size is handled; this only chooses the split),
        // then two levels per launch up to level Le >= L
        int top = 0;
        while (top < L && top < (int)d.walk_sizes.size() && d.walk_sizes[top] <= kWalkTopMax) ++top;
        const int Le = top + 2 * ((L - top + 1) / 2);
        TRY(d.walk_ctl.ensure((size_t)(Le + 8) * 4));
        hipLaunchKernelGGL(k_zero_u32, dim3((Le + 8 + 255) / 256), dim3(256), 0, s,
                           d.walk_ctl.as<uint32_t>(), Le + 8);
        uint32_t* ctl = d.walk_ctl.as<uint32_t>();
        uint32_t* sizes = ctl + 4;
        hipLaunchKernelGGL(k_walk_top, dim3(1), dim3(kWalkT), 0, s, nbox, d.item_count.as<int32_t>(),
                           d.front.as<int2>(), d.front_next.as<int2>(), top, sizes, ctl, capf,
                           capp, capm, d.walkbox.as<WalkBox>(), d.wcell.as<WalkCell>(), ks,
                           d.p2p_keys.as<uint64_t>(), d.m2l_keys.as<uint64_t>());
        int cur = walk_top_steps(top) & 1;   // the buffer that holds level `top`
        for (int it = top; it < L; it += 2) {
            // workgroups for the frontier the last build had at this level
            // (the kernel strides over any size; this only trims launches)
            const int64_t prev = it < (int)d.walk_sizes.size() ? d.walk_sizes[it] : capf;
            const unsigned g = (unsigned)std::min<int64_t>(512, (prev + prev / 4 + 2 * kWalkT) / kWalkT);
            hipLaunchKernelGGL(k_walk_multi, dim3(g), dim3(kWalkT), 0, s, bufs[cur]->as<int2>(),
                               bufs[cur ^ 1]->as<int2>(), it, sizes, ctl, capf, capp, capm,
                               d.walkbox.as<WalkBox>(), d.wcell.as<WalkCell>(), ks,
                               d.p2p_keys.as<uint64_t>(), d.m2l_keys.as<uint64_t>());
            cur ^= 1;
        }
        hipLaunchKernelGGL(k_m2l_depths, dim3(8), dim3(256), 0, s, d.m2l_keys.as<uint64_t>(),
                           ctl + 1, capm, ks.y, d.cell_aux.as<int4>(), ctl + 5 + Le);
        TRY(hipGetLastError());
        // the walk's counts and the input checks in one round trip, into
        // pinned memory
        TRY(d.ensure_host_rb());
        if (Le + 7 + 3 > DevPlan::kHostRbWords) return "walk has too many levels for the read-back buffer";
        TRY(hipMemcpyAsync(d.host_rb, ctl, (Le + 7) * 4, hipMemcpyDeviceToHost, s));
        TRY(hipMemcpyAsync(d.host_rb + Le + 7, d.wcount.p, 12, hipMemcpyDeviceToHost, s));
        TRY(hipStreamSynchronize(s));
        std::vector<uint32_t> hc(d.host_rb, d.host_rb + Le + 7);
        std::memcpy(flags, d.host_rb + Le + 7, 12);
        have_flags = true;
        if (clk.on) {
            std::fprintf(stderr, "[pmfmm gpu plan] walk frontier per level:");
            for (int it = 0; it <= Le; ++it) std::fprintf(stderr, " %u", hc[4 + it]);
            std::fprintf(stderr, "\n");
        }
        if (hc[2] == 0 && hc[4 + Le] == 0 && hc[0] <= capp && hc[1] <= capm) {
            n_p2p = hc[0];
            n_m2l = hc[1];
            dmin_tgt = (int32_t)(0x7fffffffu - hc[5 + Le]);
            dmin_src = (int32_t)(0x7fffffffu - hc[6 + Le]);
            d.walk_sizes.assign(hc.begin() + 4, hc.begin() + 4 + L);
            done = true;
        }
    }
    if (!done) {
        int64_t nf = nf0;
        TRY(d.front.ensure(std::max<size_t>(f0.size() * 4, 4096)));
        TRY(hipMemcpyAsync(d.front.p, f0.data(), f0.size() * 4, hipMemcpyHostToDevice, s));
        // this loop's counters: wcount[20..23] (words 0..2 hold the checks)
        uint32_t* wc = d.wcount.as<uint32_t>() + 20;
        hipLaunchKernelGGL(k_zero_u32, dim3(1), dim3(64), 0, s, wc, 4);
        if (d.p2p_keys.bytes < 16) TRY(d.p2p_keys.ensure(1 << 20));
        if (d.m2l_keys.bytes < 16) TRY(d.m2l_keys.ensure(1 << 16));
        uint32_t hc[4] = {0, 0, 0, 0};
        int levels = 0;
        int64_t max_front = nf;
        d.walk_sizes.clear();
        while (nf > 0) {
            d.walk_sizes.push_back((uint32_t)nf);
            TRY(d.front_next.grow((size_t)4 * nf * 8, 0, s));
            // each pair adds at most 4 children and 2 keys (itself and mirror)
            if ((size_t)(n_p2p + 2 * nf) * 8 > d.p2p_keys.bytes)
                TRY(d.p2p_keys.grow((size_t)(n_p2p + 2 * nf) * 8 * 2, (size_t)n_p2p * 8, s));
            if ((size_t)(n_m2l + 2 * nf) * 8 > d.m2l_keys.bytes)
                TRY(d.m2l_keys.grow((size_t)(n_m2l + 2 * nf) * 8 * 2, (size_t)n_m2l * 8, s));
            hipLaunchKernelGGL(k_zero_u32, dim3(1), dim3(64), 0, s, wc, 1);
            hipLaunchKernelGGL(k_walk, dim3(grid_of(nf)), dim3(256), 0, s, d.front.as<int2>(), (int)nf,
                               d.front_next.as<int2>(), d.walkbox.as<WalkBox>(), d.wcell.as<WalkCell>(),
                               ks, wc, d.p2p_keys.as<uint64_t>(), d.m2l_keys.as<uint64_t>());
            TRY(hipGetLastError());
            TRY(hipMemcpyAsync(hc, wc, 16, hipMemcpyDeviceToHost, s));
            TRY(hipStreamSynchronize(s));
            nf = hc[0];
            n_p2p = hc[1];
            n_m2l = hc[2];
            max_front = std::max<int64_t>(max_front, nf);
            ++levels;
            std::swap(d.front, d.front_next);
        }
        if (n_m2l > 0) {
            // smallest M2L depths (words 4, 5 of wcount, zeroed here)
            uint32_t cnt32 = (uint32_t)n_m2l;
            TRY(hipMemcpyAsync(d.wcount.as<uint32_t>() + 6, &cnt32, 4, hipMemcpyHostToDevice, s));
            hipLaunchKernelGGL(k_zero_u32, dim3(1), dim3(64), 0, s, d.wcount.as<uint32_t>() + 4, 2);
            hipLaunchKernelGGL(k_m2l_depths, dim3(8), dim3(256), 0, s, d.m2l_keys.as<uint64_t>(),
                               d.wcount.as<uint32_t>() + 6, (uint32_t)n_m2l, ks.y,
                               d.cell_aux.as<int4>(), d.wcount.as<uint32_t>() + 4);
            TRY(hipGetLastError());
            uint32_t dd[2] = {0u, 0u};
            TRY(hipMemcpyAsync(dd, d.wcount.as<uint32_t>() + 4, 8, hipMemcpyDeviceToHost, s));
            TRY(hipStreamSynchronize(s));
            dmin_tgt = (int32_t)(0x7fffffffu - dd[0]);
            dmin_src = (int32_t)(0x7fffffffu - dd[1]);
        }
        // sizes for the next build of this shape (with some room to move)
        d.walk_levels = levels + 2;
        d.walk_cap_front = (uint32_t)std::min<int64_t>(0x7fffffff, max_front + max_front / 2 + 4096);
        d.walk_cap_p2p = (uint32_t)std::min<int64_t>(0x7fffffff, n_p2p + n_p2p / 4 + 4096);
        d.walk_cap_m2l = (uint32_t)std::min<int64_t>(0x7fffffff, n_m2l + n_m2l / 4 + 4096);
    }

    if (!have_flags) {
        TRY(hipMemcpyAsync(flags, d.wcount.p, 12, hipMemcpyDeviceToHost, s));
        TRY(hipStreamSynchronize(s));
    }
    if (flags[0] != 0x7fffffff || flags[1] != 0x7fffffff || (flags[2] != 0 && !d.force64))
        TRY(join_gather());
    if (flags[0] != 0x7fffffff) {
        *input_error = "non-finite position at particle " + std::to_string(flags[0]);
        return std::string();
    }
    if (flags[1] != 0x7fffffff) {
        *input_error = "negative or non-finite mass at particle " + std::to_string(flags[1]);
        return std::string();
    }
    if (flags[2] != 0 && !d.force64) {
        // a run of equal keys too long for k_run_fix: build again
        // with the full 64-bit sort
        d.force64 = true;
        std::string e = gpu_build_plan(d, topo, pos, mass, chunk, s, out, input_error, on_m2l, side);
        d.force64 = false;
        return e;
    }
    clk.lap("walk");
    // ---- canonical order and CSR
    TRY(d.p2p_row.ensure((nl + 1) * 4));
    TRY(d.js.ensure(std::max<int64_t>(1, n_p2p) * 4));
    TRY(d.m2l_row.ensure((nc + 1) * 4));
    TRY(d.m2l_src.ensure(std::max<int64_t>(1, n_m2l) * 4));
    TRY(d.m2l_shift.ensure(std::max<int64_t>(1, n_m2l) * 4));
    TRY(d.m2l_vals.ensure(std::max<int64_t>(1, n_m2l) * 4));
    // slots, then long-row scratch: two int32 per key
    TRY(d.p2p_keys_tmp.ensure(std::max<int64_t>(1, n_p2p) * 8));
    TRY(d.m2l_keys_tmp.ensure(std::max<int64_t>(1, n_m2l) * 8));
    TRY(d.rowcnt.ensure((nl + 2) * 4));
    TRY(d.longrows.ensure((nl + 1) * 4));
    TRY(d.tile_sums.ensure(sort_tiles(nl + 1) * 4 + 16));
    TRY(d.rowcnt_m2l.ensure((nc + 2) * 4));
    TRY(d.longrows_m2l.ensure((nc + 1) * 4));
    TRY(d.tile_sums_m2l.ensure(sort_tiles(nc + 1) * 4 + 16));
    struct RowList {
        const DevBuf& keys;
        int64_t nk;
        int nrows;
        int ks;
        DevBuf& row;
        DevBuf& vals;
        DevBuf& tmp;       // per-key slots, then long-row scratch
        DevBuf& cnt;       // nrows + 2 counts
        DevBuf& longs;     // nrows + 1
        DevBuf& tsums;     // scan scratch
    };
    const RowList p2p_rows{d.p2p_keys, n_p2p, (int)nl, ks.x, d.p2p_row, d.js,
                           d.p2p_keys_tmp, d.rowcnt, d.longrows, d.tile_sums};
    const RowList m2l_rows{d.m2l_keys, n_m2l, (int)nc, ks.y, d.m2l_row, d.m2l_vals,
                           d.m2l_keys_tmp, d.rowcnt_m2l, d.longrows_m2l, d.tile_sums_m2l};
    // the rows in two parts: the atomic row counts, then the rest
    auto count_rows = [&](const RowList& rl, hipStream_t st) -> hipError_t {
        hipLaunchKernelGGL(k_zero_u32, dim3(grid_of(rl.nrows + 2)), dim3(256), 0, st,
                           rl.cnt.as<uint32_t>(), rl.nrows + 2);
        if (rl.nk > 0)
            hipLaunchKernelGGL(k_row_count, dim3(grid_of(rl.nk)), dim3(256), 0, st,
                               rl.keys.as<uint64_t>(), rl.nk, rl.ks, rl.cnt.as<int32_t>(),
                               rl.tmp.as<int32_t>());
        return hipGetLastError();
    };
    auto finish_rows = [&](const RowList& rl, hipStream_t st) -> hipError_t {
        int32_t* cnt = rl.cnt.as<int32_t>();
        int32_t* slot = rl.tmp.as<int32_t>();
        hipError_t e = exclusive_scan_i32(cnt, rl.row.as<int32_t>(), rl.nrows + 1,
                                          rl.tsums.as<uint32_t>(), st);
        if (e != hipSuccess) return e;
        if (rl.nk > 0) {
            hipLaunchKernelGGL(k_row_place, dim3(grid_of(rl.nk)), dim3(256), 0, st,
                               rl.keys.as<uint64_t>(), rl.nk, rl.ks, rl.row.as<int32_t>(), slot,
                               rl.vals.as<int32_t>());
            // the count of long rows goes in cnt[nrows + 1] (zeroed above)
            int32_t* nlong = cnt + rl.nrows + 1;
            hipLaunchKernelGGL(k_row_sort_short, dim3(rl.nrows), dim3(64), 0, st,
                               rl.row.as<int32_t>(), rl.vals.as<int32_t>(),
                               rl.longs.as<int32_t>(), nlong);
            hipLaunchKernelGGL(k_row_sort_long, dim3(64), dim3(256), 0, st, rl.row.as<int32_t>(),
                               rl.vals.as<int32_t>(), rl.longs.as<int32_t>(), nlong, slot,
                               row_lds_cap());
        }
        return hipGetLastError();
    };
    // With M2L tasks and a side stream, the M2L rows and then the far field
    // (on_m2l) run on the side stream while the P2P rows and the work items
    // are built on s; the side stream starts after everything before it on
    // s (the walk), and s waits for the M2L rows (not the far field) before
    // the build ends.
    const bool fork = side != nullptr && side != s && n_m2l > 0;
    hipStream_t ms = s;
    if (fork) {
        for (hipEvent_t* e : {&d.fork_ev, &d.m2l_done})
            if (!*e) TRY(hipEventCreateWithFlags(e, hipEventDisableTiming));
        TRY(hipEventRecord(d.fork_ev, s));
        TRY(hipStreamWaitEvent(side, d.fork_ev, 0));
        ms = side;
        // the P2P row counts (a long kernel) first, so the device has work
        // on s while the host enqueues the side stream's launches
        TRY(count_rows(p2p_rows, s));
    }
    TRY(count_rows(m2l_rows, ms));
    TRY(finish_rows(m2l_rows, ms));
    // M2L sources and shifts; the smallest depths go to wcount words 16, 17
    // (the walk's k_m2l_depths gave the same values to the host already)
    hipLaunchKernelGGL(k_fill_i32, dim3(1), dim3(64), 0, ms, reinterpret_cast<int*>(d.wcount.p) + 16,
                       2, 0x7fffffff);
    if (n_m2l > 0)
        hipLaunchKernelGGL(k_m2l_split, dim3(grid_of(nc)), dim3(256), 0, ms, d.m2l_row.as<int32_t>(),
                           (int)nc, d.m2l_vals.as<int32_t>(), d.cell_aux.as<int4>(),
                           d.m2l_src.as<int32_t>(), d.m2l_shift.as<int32_t>(),
                           reinterpret_cast<int32_t*>(d.wcount.p) + 16);
    TRY(hipGetLastError());
    if (fork) TRY(hipEventRecord(d.m2l_done, side));
    if (!fork) TRY(count_rows(p2p_rows, s));
    if (on_m2l) {
        std::string e = on_m2l(n_m2l, dmin_src, dmin_tgt);
        if (!e.empty()) return e;
    }
    TRY(finish_rows(p2p_rows, s));
    if (fork) TRY(hipStreamWaitEvent(s, d.m2l_done, 0));
    TRY(join_gather());
    out.n_p2p = n_p2p;
    out.n_m2l = n_m2l;
    clk.lap("csr");
    std::string e2 = gpu_make_items(d, topo, n_p2p, chunk, s, out);
    clk.lap("items");
    return e2;
}

std::string gpu_make_items(DevPlan& d, const Plan& topo, int64_t n_p2p, int chunk, hipStream_t s,
                           PlanCounts& out) {
    const int64_t nl = (int64_t)topo.leaf_cell.size();
    if (chunk <= 0) chunk = kAutoChunk;
    TRY(d.cost.ensure((nl + 1) * 4));
    TRY(d.leaf_slot.ensure((nl + 1) * 4));
    TRY(d.tile_sums.ensure(sort_tiles(nl + 1) * 4 + 16));
    hipLaunchKernelGGL(k_item_count, dim3(grid_of(nl + 1)), dim3(256), 0, s, (int)nl,
                       d.p2p_row.as<int32_t>(), chunk, d.cost.as<int32_t>());
    TRY(hipGetLastError());
    TRY(exclusive_scan_i32(d.cost.as<int32_t>(), d.leaf_slot.as<int32_t>(), nl + 1,
                           d.tile_sums.as<uint32_t>(), s));
    // buffers sized for the most items the rows can give (sum over rows of
    // ceil(len / chunk) <= n_p2p / chunk + rows), so the count is read back
    // only at the end
    const int64_t cap = std::max<int64_t>(1, (n_p2p + chunk - 1) / chunk + nl);
    TRY(d.items.ensure(cap * 16));
    TRY(d.cost_keys.ensure(cap * 8));
    // per-row candidate pairs in the sort's scratch (free until the sort)
    TRY(d.cost_keys_tmp.ensure(std::max<int64_t>(cap, nl) * 8));
    TRY(d.queue.ensure(cap * 4));
    TRY(d.wcount.ensure(128));
    hipLaunchKernelGGL(k_zero_u32, dim3(1), dim3(64), 0, s, d.wcount.as<uint32_t>(), 16);
    // largest item: chunk tasks of at most 64 x 64 pairs
    const int cshift = std::max(0, bits_for((uint64_t)chunk * 64 * 64) - 8);
    hipLaunchKernelGGL(k_items, dim3(grid_of((nl + 1) * 64)), dim3(256), 0, s, (int)nl,
                       d.p2p_row.as<int32_t>(), d.js.as<int32_t>(), d.leaf.as<int4>(), chunk, cshift,
                       d.leaf_slot.as<int32_t>(), (int)cap, d.items.as<int4>(),
                       d.cost_keys.as<uint64_t>(), d.queue.as<uint32_t>(),
                       d.cost_keys_tmp.as<unsigned long long>(), d.wcount.as<uint32_t>() + 8);
    hipLaunchKernelGGL(k_sum_rows, dim3(1), dim3(1024), 0, s, d.cost_keys_tmp.as<unsigned long long>(),
                       (int)nl, reinterpret_cast<unsigned long long*>(d.wcount.as<uint32_t>() + 8));
    TRY(hipGetLastError());
    std::string err = sort_in_place(d.cost_keys, &d.queue, d.cost_keys_tmp, &d.queue_tmp, d.hist,
                                    cap, 12, s);
    if (!err.empty()) return err;
    // words 8, 9: candidate pairs; 10: items; 16, 17: M2L depths (set by the build)
    uint32_t w[10];
    TRY(d.ensure_host_rb());
    TRY(hipMemcpyAsync(d.host_rb, d.wcount.as<uint32_t>() + 8, sizeof(w), hipMemcpyDeviceToHost, s));
    TRY(hipStreamSynchronize(s));
    std::memcpy(w, d.host_rb, sizeof(w));
    unsigned long long cand = 0;
    std::memcpy(&cand, w, 8);
    const int64_t n_items = (int64_t)w[2];
    TRY(d.partial.ensure(std::max<int64_t>(1, n_items) * 4 * 64 * 8));
    out.n_items = n_items;
    out.candidate_pairs = (int64_t)cand;
    out.m2l_min_depth_src = (int32_t)w[8];
    out.m2l_min_depth_tgt = (int32_t)w[9];
    return std::string();
}

}  // namespace pmfmm
