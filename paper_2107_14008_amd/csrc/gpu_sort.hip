// Device primitives of the on-GPU planner: a stable LSD radix sort of 64-bit
// or 32-bit keys (optionally carrying 32-bit values), also of several
// equal-length segments at once, and an exclusive prefix sum of 32-bit
// integers.
//
// Radix sort: 8-bit digits, tiles of 4096 elements (256 threads x 16
// rounds; 1024 for segments under kSmallSortN elements, whose few tiles
// would otherwise leave most CUs idle); a tile never straddles two segments.  Per pass: (1) per-tile
// digit histogram in LDS, (2) one exclusive scan over the
// [segment][digit][tile] table (segment-major, so segment s lands in
// [s n, (s + 1) n)), (3) scatter: inside a tile the 256 elements of a round
// are ranked per digit with wavefront ballots (eight ballots give each lane
// the mask of lanes holding its digit) and a running per-digit count in
// LDS, so the order of equal digits is kept (stable), which makes the sort
// stable across passes; the tile is ordered in LDS and written out in runs.
#include <algorithm>

#include "gpu_plan.h"

namespace pmfmm {
namespace {

constexpr int kThreads = 256;
constexpr int kRounds = 16;
constexpr int kTile = kThreads * kRounds;  // 4096
constexpr int kRoundsSmall = 4;
constexpr int64_t kSmallSortN = int64_t(1) << 20;

int radix_rounds(int64_t n) { return n < kSmallSortN ? kRoundsSmall : kRounds; }

int64_t radix_tiles(int64_t n) {
    const int64_t t = (int64_t)kThreads * radix_rounds(n);
    return (n + t - 1) / t;
}

// Block b handles tile (b % tiles) of segment (b / tiles); its elements are
// [seg n + tile T, min(seg n + (tile + 1) T, (seg + 1) n)), T = 256 R.
struct TileRange {
    int64_t begin, end;
    size_t col;   // (seg * 256) * tiles + tile: add digit * tiles
};

template <int R>
__device__ __forceinline__ TileRange tile_range(int64_t n, int tiles) {
    const int seg = blockIdx.x / tiles, tile = blockIdx.x - seg * tiles;
    TileRange t;
    t.begin = (int64_t)seg * n + (int64_t)tile * (kThreads * R);
    t.end = min((int64_t)seg * n + n, t.begin + kThreads * R);
    t.col = (size_t)seg * 256 * tiles + tile;
    return t;
}

template <class K, int R>
__global__ void __launch_bounds__(kThreads)
rs_hist(const K* __restrict__ keys, int64_t n, int shift, uint32_t* __restrict__ hist,
        int tiles) {
    __shared__ uint32_t h[256];
    h[threadIdx.x] = 0;
    __syncthreads();
    const TileRange tr = tile_range<R>(n, tiles);
    for (int r = 0; r < R; ++r) {
        const int64_t i = tr.begin + r * kThreads + threadIdx.x;
        if (i < tr.end) atomicAdd(&h[(keys[i] >> shift) & 255u], 1u);
    }
    __syncthreads();
    hist[tr.col + (size_t)threadIdx.x * tiles] = h[threadIdx.x];
}

// Exclusive scan of m 32-bit values by one workgroup of 1024 threads.
__global__ void __launch_bounds__(1024) scan_single(uint32_t* __restrict__ a, int64_t m) {
    __shared__ uint32_t part[1024];
    const int t = threadIdx.x;
    const int64_t per = (m + 1023) / 1024;
    const int64_t b = t * per, e = min(m, b + per);
    uint32_t s = 0;
    for (int64_t i = b; i < e; ++i) s += a[i];
    part[t] = s;
    __syncthreads();
    for (int off = 1; off < 1024; off <<= 1) {
        uint32_t v = t >= off ? part[t - off] : 0u;
        __syncthreads();
        part[t] += v;
        __syncthreads();
    }
    uint32_t run = t == 0 ? 0u : part[t - 1];
    for (int64_t i = b; i < e; ++i) {
        const uint32_t v = a[i];
        a[i] = run;
        run += v;
    }
}

// Scatter of one pass.  The tile is first put in digit order in LDS (local
// position = the digit's start in the tile + the element's stable rank among
// the tile's elements of that digit), then written out position by
// position: consecutive positions of one digit go to consecutive addresses,
// so the global writes come in runs instead of one element per line.
template <class K, bool VALS, int R>
__global__ void __launch_bounds__(kThreads)
rs_scatter(const K* __restrict__ kin, const uint32_t* __restrict__ vin,
           K* __restrict__ kout, uint32_t* __restrict__ vout, int64_t n, int shift,
           const uint32_t* __restrict__ hist, const uint32_t* __restrict__ offs, int tiles) {
    __shared__ K ks[kThreads * R];
    __shared__ uint32_t vs[VALS ? kThreads * R : 1];
    __shared__ uint32_t start[256];     // digit start inside the tile
    __shared__ uint32_t goff[256];      // digit start in the output
    __shared__ uint32_t run[256];       // elements of each digit placed so far
    __shared__ uint32_t wc[kThreads / 64][256];
    const int t = threadIdx.x;
    const int lane = t & 63, wave = t >> 6;
    const TileRange tr = tile_range<R>(n, tiles);
    // exclusive scan of the tile's digit counts (one wave scans 4 per lane)
    {
        const uint32_t c = hist[tr.col + (size_t)t * tiles];
        goff[t] = offs[tr.col + (size_t)t * tiles];
        run[t] = 0;
        start[t] = c;
        for (int w = 0; w < kThreads / 64; ++w) wc[w][t] = 0;
    }
    __syncthreads();
    if (wave == 0) {
        uint32_t v[4], tot = 0;
        for (int j = 0; j < 4; ++j) {
            v[j] = start[4 * lane + j];
            tot += v[j];
        }
        uint32_t x = tot;
        for (int off = 1; off < 64; off <<= 1) {
            const uint32_t y = __shfl_up(x, off);
            if (lane >= off) x += y;
        }
        uint32_t e = x - tot;
        for (int j = 0; j < 4; ++j) {
            start[4 * lane + j] = e;
            e += v[j];
        }
    }
    __syncthreads();
    const uint64_t below = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    for (int r = 0; r < R; ++r) {
        const int64_t i = tr.begin + r * kThreads + t;
        const bool valid = i < tr.end;
        K key = 0;
        uint32_t val = 0;
        uint32_t d = 0;
        if (valid) {
            key = kin[i];
            if (VALS) val = vin[i];
            d = (uint32_t)(key >> shift) & 255u;
        }
        uint64_t m = __ballot(valid);
        for (int b = 0; b < 8; ++b) {
            const bool bit = (d >> b) & 1u;
            const uint64_t bb = __ballot(bit);
            m &= bit ? bb : ~bb;
        }
        const uint32_t rank = (uint32_t)__popcll(m & below);
        if (valid && rank == 0) wc[wave][d] = (uint32_t)__popcll(m);
        __syncthreads();
        if (valid) {
            uint32_t pos = start[d] + run[d] + rank;
            for (int w = 0; w < wave; ++w) pos += wc[w][d];
            ks[pos] = key;
            if (VALS) vs[pos] = val;
        }
        __syncthreads();
        uint32_t add = 0;
        for (int w = 0; w < kThreads / 64; ++w) {
            add += wc[w][t];
            wc[w][t] = 0;
        }
        run[t] += add;
        __syncthreads();
    }
    const int len = (int)(tr.end - tr.begin);
    for (int p = t; p < len; p += kThreads) {
        const K key = ks[p];
        const uint32_t d = (uint32_t)(key >> shift) & 255u;
        const uint32_t o = goff[d] + (uint32_t)p - start[d];
        kout[o] = key;
        if (VALS) vout[o] = vs[p];
    }
}

// ---- exclusive scan of int32 (tiles of 4096)
__global__ void __launch_bounds__(kThreads)
scan_tile_sums(const int32_t* __restrict__ in, int64_t n, uint32_t* __restrict__ sums) {
    __shared__ int32_t red[kThreads];
    const int64_t base = (int64_t)blockIdx.x * kTile + (int64_t)threadIdx.x * kRounds;
    int32_t s = 0;
    for (int r = 0; r < kRounds; ++r)
        if (base + r < n) s += in[base + r];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int off = kThreads / 2; off > 0; off >>= 1) {
        if ((int)threadIdx.x < off) red[threadIdx.x] += red[threadIdx.x + off];
        __syncthreads();
    }
    if (threadIdx.x == 0) sums[blockIdx.x] = (uint32_t)red[0];
}

// SCANNED: sums holds each tile's offset (scan_single ran); otherwise the
// tile sums themselves, and each workgroup adds up those before its tile
// (one launch fewer; for up to kApplySumMax tiles).
constexpr int kApplySumMax = 4096;

template <bool SCANNED>
__global__ void __launch_bounds__(kThreads)
scan_tile_apply(const int32_t* __restrict__ in, int32_t* __restrict__ out, int64_t n,
                const uint32_t* __restrict__ sums) {
    __shared__ int32_t part[kThreads];
    __shared__ uint32_t toff;
    const int t = threadIdx.x;
    if (!SCANNED) {
        uint32_t c = 0;
        for (int k = t; k < (int)blockIdx.x; k += kThreads) c += sums[k];
        for (int off = 32; off > 0; off >>= 1) c += __shfl_down(c, off);
        if ((t & 63) == 0) part[t >> 6] = (int32_t)c;
        __syncthreads();
        if (t == 0) {
            uint32_t a = 0;
            for (int w = 0; w < kThreads / 64; ++w) a += (uint32_t)part[w];
            toff = a;
        }
        __syncthreads();
    }
    const int64_t base = (int64_t)blockIdx.x * kTile + (int64_t)t * kRounds;
    int32_t v[kRounds];
    int32_t s = 0;
    for (int r = 0; r < kRounds; ++r) {
        v[r] = base + r < n ? in[base + r] : 0;
        s += v[r];
    }
    part[t] = s;
    __syncthreads();
    for (int off = 1; off < kThreads; off <<= 1) {
        int32_t x = t >= off ? part[t - off] : 0;
        __syncthreads();
        part[t] += x;
        __syncthreads();
    }
    int32_t run = (int32_t)(SCANNED ? sums[blockIdx.x] : toff) + (t == 0 ? 0 : part[t - 1]);
    for (int r = 0; r < kRounds; ++r) {
        if (base + r < n) out[base + r] = run;
        run += v[r];
    }
}

}  // namespace

hipError_t exclusive_scan_i32(const int32_t* in, int32_t* out, int64_t n, uint32_t* tile_sums,
                              hipStream_t s);

int64_t sort_tiles(int64_t n) { return (n + kTile - 1) / kTile; }

int64_t sort_hist_words(int64_t n, int nseg) {
    const int64_t m = (int64_t)nseg * 256 * radix_tiles(n);
    return 2 * m + sort_tiles(m) + 16;
}

template <class K, int R>
hipError_t radix_sort_r(K* keys, uint32_t* vals, K* tmp_keys, uint32_t* tmp_vals, uint32_t* hist,
                        int64_t n, int bit_begin, int bit_end, hipStream_t s, bool* result_in_tmp,
                        int nseg) {
    const int tiles = (int)radix_tiles(n);
    const int blocks = nseg * tiles;
    K* ka = keys;
    K* kb = tmp_keys;
    uint32_t* va = vals;
    uint32_t* vb = tmp_vals;
    // scratch layout: counts [m], their exclusive scan [m], tile sums
    const int64_t m = (int64_t)nseg * 256 * tiles;
    uint32_t* offs = hist + m;
    uint32_t* scan_scratch = hist + 2 * m;
    for (int shift = bit_begin; shift < bit_end; shift += 8) {
        hipLaunchKernelGGL((rs_hist<K, R>), dim3(blocks), dim3(kThreads), 0, s, ka, n, shift, hist,
                           tiles);
        const hipError_t e = exclusive_scan_i32(reinterpret_cast<const int32_t*>(hist),
                                                reinterpret_cast<int32_t*>(offs), m, scan_scratch, s);
        if (e != hipSuccess) return e;
        if (vals)
            hipLaunchKernelGGL((rs_scatter<K, true, R>), dim3(blocks), dim3(kThreads), 0, s, ka, va,
                               kb, vb, n, shift, hist, offs, tiles);
        else
            hipLaunchKernelGGL((rs_scatter<K, false, R>), dim3(blocks), dim3(kThreads), 0, s, ka, va,
                               kb, vb, n, shift, hist, offs, tiles);
        std::swap(ka, kb);
        std::swap(va, vb);
        *result_in_tmp = !*result_in_tmp;
    }
    return hipGetLastError();
}

template <class K>
hipError_t radix_sort(K* keys, uint32_t* vals, K* tmp_keys, uint32_t* tmp_vals, uint32_t* hist,
                      int64_t n, int bit_begin, int bit_end, hipStream_t s, bool* result_in_tmp,
                      int nseg) {
    *result_in_tmp = false;
    if (n <= 1 || nseg < 1) return hipSuccess;
    if (radix_rounds(n) == kRoundsSmall)
        return radix_sort_r<K, kRoundsSmall>(keys, vals, tmp_keys, tmp_vals, hist, n, bit_begin,
                                             bit_end, s, result_in_tmp, nseg);
    return radix_sort_r<K, kRounds>(keys, vals, tmp_keys, tmp_vals, hist, n, bit_begin, bit_end, s,
                                    result_in_tmp, nseg);
}

hipError_t radix_sort_u64(uint64_t* keys, uint32_t* vals, uint64_t* tmp_keys, uint32_t* tmp_vals,
                          uint32_t* hist, int64_t n, int bit_begin, int bit_end, hipStream_t s,
                          bool* result_in_tmp, int nseg) {
    return radix_sort<uint64_t>(keys, vals, tmp_keys, tmp_vals, hist, n, bit_begin, bit_end, s,
                                result_in_tmp, nseg);
}

hipError_t radix_sort_u32(uint32_t* keys, uint32_t* vals, uint32_t* tmp_keys, uint32_t* tmp_vals,
                          uint32_t* hist, int64_t n, int bit_begin, int bit_end, hipStream_t s,
                          bool* result_in_tmp, int nseg) {
    return radix_sort<uint32_t>(keys, vals, tmp_keys, tmp_vals, hist, n, std::min(bit_begin, 32),
                                std::min(bit_end, 32), s, result_in_tmp, nseg);
}

hipError_t exclusive_scan_i32(const int32_t* in, int32_t* out, int64_t n, uint32_t* tile_sums,
                              hipStream_t s) {
    if (n <= 0) return hipSuccess;
    const int tiles = (int)sort_tiles(n);
    hipLaunchKernelGGL(scan_tile_sums, dim3(tiles), dim3(kThreads), 0, s, in, n, tile_sums);
    if (tiles <= kApplySumMax) {
        hipLaunchKernelGGL(scan_tile_apply<false>, dim3(tiles), dim3(kThreads), 0, s, in, out, n,
                           tile_sums);
    } else {
        hipLaunchKernelGGL(scan_single, dim3(1), dim3(1024), 0, s, tile_sums, (int64_t)tiles);
        hipLaunchKernelGGL(scan_tile_apply<true>, dim3(tiles), dim3(kThreads), 0, s, in, out, n,
                           tile_sums);
    }
    return hipGetLastError();
}

}  // namespace pmfmm
