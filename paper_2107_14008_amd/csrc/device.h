// Device-side data layout and kernel launchers of the short-range library.
//
// Layout in HBM (all arrays global over a batch of boxes):
//   x64[k]  double4 (x, y, z, m)            particle k in leaf order
//   x32[k]  float4  ((x - c_leaf) sigma, m) single-precision cell-relative form,
//                                           in units of 1 / sigma of its box
//   leaf[l] int4    (first, count, box, cell)
//   leafc[l] double4 (centre x, y, z, 0)    expansion / offset centre
//   p2p_row[l] .. p2p_row[l+1]              TaskGroup rows of i leaf l
//   p2p_js[t] = (j leaf << 5) | shift code  TaskGroup entries
//   items[q] int4 (leaf, t0, t1, slot)      work items; queue: per segment
//                                           (kQueueSegs), longest first
//   partial[(slot * 3 + axis) * 64 + lane]  per-item float64 partial sums
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "plan.h"
#include "truncation_poly.h"

namespace pmfmm {

enum Mode : int {
    kFP64Exact = 0,
    kFP64Table = 1,
    kFP32Exact = 2,
    kFP32Table = 3,
    kFP32R2 = 4,    // float32, segment table over r^2 (cutoff at the last row)
    kFP64R2 = 5     // float64, segment table over r^2 (closest pairs evaluated exactly)
};

constexpr bool is_fp32(int mode) {
    return mode == kFP32Exact || mode == kFP32Table || mode == kFP32R2;
}

// Largest workgroup of the P2P kernel: 16 waves share one LDS copy of a
// table; the float64 exact form keeps its polynomial's coefficients and
// a source record in registers and is compiled for 4-wave workgroups
// (up to 512 VGPRs per lane instead of 128).
constexpr int p2p_max_threads(int mode) { return mode == kFP64Exact ? 256 : 1024; }
// Waves per SIMD the float32 forms must leave room for: two 16-wave
// workgroups per CU (their tables fit twice in LDS), so at most 64 VGPRs and
// the matching scalar registers per wave.
constexpr int p2p_min_waves_per_simd(int mode) { return is_fp32(mode) ? 8 : 1; }
// The same for the adjoint: every float64 form evaluates g and h exactly.
constexpr int adjoint_max_threads(int mode) { return is_fp32(mode) ? 1024 : 256; }

// r^2 table form: scaled r^2 covers [2^kR2Emin, 2^kR2Emax) (r_cut^2 = 2^kR2Emax).
constexpr int kR2Emin = -35;
constexpr int kR2Emax = 11;
// float64 r^2 table: scaled r^2 in [2^kR2Emin64, 2^kR2Emax); closer pairs
// (r < 2^-8 r_cut) take the exact erfc / exp path.
constexpr int kR2Emin64 = kR2Emax - 16;
// float32 r^2 table at 2^bits segments per octave: rows r2_rows(bits) (the
// last, at s = 2^kR2Emax, zero); row k holds (c0, c1) at 8 k and (c2, 0) at
// r2_plane_c2(bits) + 8 k, so a lookup is one 8-byte and one 4-byte LDS read
// from the same address.
constexpr int kR2Plane = 5952;   // rows the fit scratch holds (128 per octave)
constexpr int r2_rows(int bits) { return ((kR2Emax - kR2Emin) << bits) + 1; }
constexpr int r2_plane_c2(int bits) { return (r2_rows(bits) * 8 + 255) / 256 * 256; }
constexpr int r2_table_bytes(int bits) { return (r2_plane_c2(bits) + r2_rows(bits) * 8 + 15) / 16 * 16; }
static_assert(r2_rows(7) <= kR2Plane, "r^2 table rows");
static_assert(r2_plane_c2(7) < 65536, "the c2 plane offset is an LDS read's immediate");
// Linear (degree 1) float32 r^2 tables: rows of (c0, c1) only, over
// [2^kR2EminLin, 2^kR2Emax) at up to 512 segments per octave, with a zero
// row below the floor (the clamp maps every s under it there) and a zero
// row at s = 2^kR2Emax; pairs closer than the floor (r < 2^-9.5 r_cut, a
// few per million) are added by an exact pass instead.  Two 16-wave
// workgroups per CU still fit their tables at 512 per octave.
constexpr int kR2EminLin = kR2Emax - 19;
constexpr int r2_rows_lin(int bits) { return ((kR2Emax - kR2EminLin) << bits) + 2; }
constexpr int r2_table_bytes_lin(int bits) { return (r2_rows_lin(bits) * 8 + 15) / 16 * 16; }
static_assert(2 * r2_table_bytes_lin(9) <= 160 * 1024, "two linear r^2 tables per CU");
// Adjoint of the float32 r^2 form: g(s) and h(s) over s in
// [2^kAdjEmin, 2^kR2Emax) at 2^kAdjBits segments per octave, as three
// arrays of kAdjPlane float pairs by row: (g c0, g c1), (h c0, h c1),
// (g c2, h c2).  The floor sits above
// kR2Emin because h's quadratic coefficient grows as s^(-9/2) and must stay
// a finite float.
constexpr int kAdjBits = 5;
constexpr int kAdjEmin = -26;
constexpr int kAdjPlane = 1216;
static_assert(((kR2Emax - kAdjEmin) << kAdjBits) + 1 <= kAdjPlane, "adjoint table rows");
constexpr int kAdjTableBytes = 6 * kAdjPlane * 4;

// ------------------------------------------------------ truncation factor
//
// T(x) = erfc(x) + (2x / sqrt(pi)) exp(-x^2) of Eq. (tr) in float64 with a
// single exponential: T = exp(-x^2) U(x), where U(x) = exp(x^2) erfc(x) +
// 2x / sqrt(pi) is smooth on [0, 3] and comes from the generated
// polynomial of truncation_poly.h (degree 24 in t = (x - 3/2) / (3/2),
// within 2 ulp of U), evaluated as an even and an odd half in t^2 (two
// independent chains).  exp(-x^2) follows the Cody-Waite reduction of the
// same header: x^2 = s + ds exactly (ds from a fused multiply-add),
// n = rint(s / ln 2), r = (n ln2_hi - s) + n ln2_lo - ds, exp(-x^2) =
// 2^-n p(r) with p the header's degree-11 polynomial.  x > 3 (cutoffs
// beyond 6 r_s) takes the library erfc and exp.  *ex receives exp(-x^2)
// (the adjoint needs it).

// a b + c as one three-operand fused multiply-add, c a uniform constant
// held in a scalar register pair.  Written out because the compiler
// otherwise keeps each polynomial coefficient in vector registers and
// copies it into the accumulator of the two-operand form before every step
// (one extra 64-bit move per coefficient).
__device__ __forceinline__ double fma_sc(double a, double b, double c) {
    double r;
    asm("v_fma_f64 %0, %1, %2, %3" : "=v"(r) : "v"(a), "v"(b), "s"(c));
    return r;
}

__device__ inline double truncation_T_f64(double x, double* ex) {
    if (x <= kTPolyXMax) {
        const double s = x * x;
        const double ds = fma(x, x, -s);
        const double n = rint(s * kInvLn2);
        double r = fma(n, kLn2Hi, -s);
        r = fma(n, kLn2Lo, r) - ds;
        double p = kExpPoly[kExpDegree];
#pragma unroll
        for (int k = kExpDegree - 1; k >= 0; --k) p = fma_sc(p, r, kExpPoly[k]);
        const double e = ldexp(p, -(int)n);
        const double t = fma(x, kTPolyInvHalfWidth, -1.0);
        const double t2 = t * t;
        constexpr int kE = kTPolyDegree - (kTPolyDegree & 1);       // top even power
        constexpr int kO = kTPolyDegree - 1 + (kTPolyDegree & 1);   // top odd power
        double ev = kTPoly[kE], od = kTPoly[kO];
#pragma unroll
        for (int k = kE - 2; k >= 0; k -= 2) ev = fma_sc(ev, t2, kTPoly[k]);
#pragma unroll
        for (int k = kO - 2; k >= 1; k -= 2) od = fma_sc(od, t2, kTPoly[k]);
        *ex = e;
        return e * fma(od, t, ev);
    }
    const double e = exp(-x * x);
    *ex = e;
    return erfc(x) + 1.12837916709551257390 * x * e;
}

// ------------------------------------------------------ source culling
//
// Before the pairs of a j leaf, lane k tests source k against the box of the
// wave's targets and the ballot of the results leaves out the sources that
// reach no target inside r_cut: the loops skip them with a scalar branch
// (at 128^3 about half of the candidate sources, the pair set unchanged).
// The box distance takes, per axis, the displacement of the box edge that
// the pair loop itself would form (same operations, so each target's
// |d_a| is at least that component: rounding is monotonic), and adds the
// squares the way r^2 is added: it never exceeds a target's r^2, so a
// source with a pair inside r_cut always survives.

// float32, in the j leaf's frame: targets p = pv - off in [plo, phi].
__device__ inline uint64_t live_f32(const float4* __restrict__ src, int nj, int lane,
                                             float3 plo, float3 phi, float rc2) {
    const float4 q = src[lane < nj ? lane : 0];
    const float bx = fmaxf(fmaxf(plo.x - q.x, q.x - phi.x), 0.f);
    const float by = fmaxf(fmaxf(plo.y - q.y, q.y - phi.y), 0.f);
    const float bz = fmaxf(fmaxf(plo.z - q.z, q.z - phi.z), 0.f);
    const float d2 = fmaf(bz, bz, fmaf(by, by, bx * bx));
    return __ballot((lane < nj) & (d2 < rc2));
}

// float64: targets x in [lo, hi]; d = (q - x) + s as in the pair forms.
template <bool SHIFTED>
__device__ inline uint64_t live_f64(const double4* __restrict__ src, int nj, int lane,
                                             const double3& lo, const double3& hi, double sx,
                                             double sy, double sz, double rc2) {
    const double4 q = src[lane < nj ? lane : 0];
    double d2;
    {
#pragma clang fp contract(off)
        double hx = q.x - hi.x, lx = q.x - lo.x;
        double hy = q.y - hi.y, ly = q.y - lo.y;
        double hz = q.z - hi.z, lz = q.z - lo.z;
        if (SHIFTED) {
            hx = hx + sx;
            lx = lx + sx;
            hy = hy + sy;
            ly = ly + sy;
            hz = hz + sz;
            lz = lz + sz;
        }
        const double bx = fmax(fmax(hx, -lx), 0.0);
        const double by = fmax(fmax(hy, -ly), 0.0);
        const double bz = fmax(fmax(hz, -lz), 0.0);
        d2 = (bx * bx + by * by) + bz * bz;
    }
    return __ballot((lane < nj) & (d2 < rc2));
}

template <class T3>
__device__ inline void wave_box(T3& lo, T3& hi) {
    for (int o = 32; o > 0; o >>= 1) {
        lo.x = min(lo.x, __shfl_xor(lo.x, o));
        lo.y = min(lo.y, __shfl_xor(lo.y, o));
        lo.z = min(lo.z, __shfl_xor(lo.z, o));
        hi.x = max(hi.x, __shfl_xor(hi.x, o));
        hi.y = max(hi.y, __shfl_xor(hi.y, o));
        hi.z = max(hi.z, __shfl_xor(hi.z, o));
    }
}

// First queue position of segment x of a queue of n items (segments and
// counters: kQueueSegs in plan.h).
__device__ inline int32_t queue_seg_begin(int x, int32_t n) {
    return (int32_t)(((int64_t)x * n + kQueueSegs - 1) / kQueueSegs);
}

// Per-box constants.  The float32 forms work on offsets scaled by sigma
// (x32 and the per-task centre offsets): sigma = 1, except for the r^2
// table, where sigma^2 = 2^kR2Emax / r_cut^2 puts the cutoff at
// r'^2 = 2^kR2Emax.  The float constants below are in those units; results
// are scaled back by sigma^2 (forces) or sigma^3 / sigma^2 (adjoint).
struct BoxDev {
    double L;        // box side
    double alpha;    // 1 / (2 r_s)
    double rc2;      // r_cut * r_cut
    double G;
    float alpha_f;   // alpha / sigma
    float rc2_f;     // r_cut^2 sigma^2 (exactly 2^kR2Emax for the r^2 table)
    float tab_scale_f;  // tab_scale / sigma
    float tiny_f;    // float32 r^2 clamp below (coincident pairs): rc2_f * 1e-14,
                     // 2^kR2Emin for the r^2 table
    double tab_scale;  // n_tab / 3 / (2 r_s): x-table units per unit distance
    int32_t order;     // expansion order p of this box (< 0: no far field)
    int32_t pad;
    double sigma;      // scale of the float32 offsets
};

struct P2PArgs {
    const double4* x64;
    const float4* x32;
    const int4* leaf;
    const double4* leafc;
    const int32_t* p2p_js;
    const int4* items;
    const int32_t* queue;
    int32_t n_items;
    int32_t* counter;
    double* partial;
    const BoxDev* boxes;
    const void* table;   // coefficient table, layout per mode (see p2p.hip)
    int32_t n_tab;
    int32_t level;
    int32_t round_floor;
    int32_t accum32;     // float32 forms: item sums in float32 with TwoSum compensation
};

struct ReduceArgs {
    const int4* leaf;
    const int32_t* leaf_slot;   // n_leaves + 1
    const double* partial;
    const double* far;          // (n, 3) leaf order or nullptr
    const int32_t* needL;       // per cell: far holds the leaf's particles (with far)
    const int32_t* perm;
    const BoxDev* boxes;
    double* out;                // (n, 3) caller order
    int32_t n_leaves;
};

struct GatherArgs {
    const double* pos_in;       // (n, 3) caller order
    const double* mass_in;      // (n)
    const int32_t* perm;
    const int4* leaf;
    double4* leafc;             // .w set to the leaf's common mass (0: none)
    const BoxDev* boxes;
    double4* x64;
    float4* x32;
    int32_t n_leaves;
};

struct FarArgs {
    const double4* x64;
    const int4* leaf;
    const double4* leafc;
    const int4* cell;           // (first, count, parent, leaf) per cell
    const int4* cell_aux;       // (child0, child1, box, depth) per cell
    const double4* cellc;       // centre per cell
    const int32_t* m2l_row;
    const int32_t* m2l_src;
    const int32_t* m2l_shift;
    const int32_t* level_cells; // cells of one depth
    int32_t n_level;
    const BoxDev* boxes;
    double* M;                  // (n_cells, ncoef)
    double* Lc;                 // (n_cells, ncoef)
    double* Lt;                 // (n_m2l, ncoef): each M2L task's contribution
    int32_t n_m2l;
    double* far;                // (n, 3) leaf order
    int32_t* needM;             // per cell: multipole needed (M2L source subtree)
    int32_t* needL;             // per cell: local expansion needed (M2L target subtree)
    int32_t n_cells, n_leaves, order, ncoef;
};

struct AdjArgs {
    const double4* x64;
    const float4* x32;
    const double4* w64;         // (w, 0) per particle, leaf order
    const float4* w32;          // the same in float32
    const int4* leaf;
    const double4* leafc;
    const int32_t* p2p_js;
    const int4* items;
    const int32_t* queue;
    int32_t n_items;
    int32_t* counter;
    double* partial;            // (slot, 4, 64): grad x, y, z, m
    const BoxDev* boxes;
    const void* table;          // float32 r^2 adjoint tables in device memory, or null
};

struct AdjReduceArgs {
    const int4* leaf;
    const int32_t* leaf_slot;
    const double* partial;
    const double4* far;         // (gx, gy, gz, gm) per particle, leaf order, or null
    const int32_t* perm;
    const BoxDev* boxes;
    double* grad_pos;           // (n, 3) caller order
    double* grad_mass;          // (n)
    int32_t n_leaves;
};

// Static scratch of the forward that allocates nothing (pmfmm_forward_static):
// the queue counters in the first kStaticCounterBytes, then the partial sums
// of up to kStaticMaxItems work items (3 x 64 doubles each).
constexpr size_t kStaticScratchBytes = (size_t)64 << 20;
constexpr size_t kStaticCounterBytes = 4096;
constexpr size_t kStaticPartialBytes = 3 * 64 * sizeof(double);
constexpr int64_t kStaticMaxItems =
    (int64_t)((kStaticScratchBytes - kStaticCounterBytes) / kStaticPartialBytes);
static_assert((size_t)kQueueSegs * kCounterStride * 4 <= kStaticCounterBytes, "counters");
// Device address of that scratch on the current device (resolved with
// hipGetSymbolAddress on the first call per device, then cached).
hipError_t static_scratch(void** out);

// Launchers (return the hipError_t of the launch).
hipError_t launch_gather(const GatherArgs& a, const double* pos_dev_unwrapped,
                         hipStream_t s);
hipError_t launch_zero_i32(int32_t* p, int32_t n, hipStream_t s);
hipError_t launch_p2p(int mode, const P2PArgs& a, int wg_waves, int grid_wgs,
                      size_t lds_bytes, hipStream_t s);
hipError_t launch_reduce(const ReduceArgs& a, hipStream_t s);
// Recomputes x32 from x64 and the leaf centres with the boxes' current sigma.
hipError_t launch_rescale_x32(const int4* leaf, const double4* leafc, const BoxDev* boxes,
                              const double4* x64, float4* x32, int32_t n_leaves, hipStream_t s);
hipError_t launch_gather_w(const double* w, const int32_t* perm, double4* w64,
                           float4* w32, int32_t n, hipStream_t s);
// a.table: the float32 r^2 adjoint tables (float32 modes), or null for
// the exact erfc / exp form.
hipError_t launch_adjoint(int mode, const AdjArgs& a, int wg_waves, int grid_wgs, hipStream_t s);
hipError_t launch_adj_reduce(const AdjReduceArgs& a, hipStream_t s);

// Kick (vel += acc dt) and drift (pos += vel dt, wrapped into [0, L)) of
// n particles, (n, 3) float64 device arrays (step.hip).
hipError_t launch_kick(int64_t n, double* vel, const double* acc, double dt, hipStream_t s);
hipError_t launch_drift(int64_t n, double* pos, const double* vel, double dt, double L, hipStream_t s);

// Far field (far.hip).
hipError_t launch_p2m(const FarArgs& a, hipStream_t s);
hipError_t launch_m2m_level(const FarArgs& a, hipStream_t s);
hipError_t launch_m2l(const FarArgs& a, hipStream_t s);
hipError_t launch_l2l_level(const FarArgs& a, hipStream_t s);
hipError_t launch_l2p(const FarArgs& a, hipStream_t s);
// Far-field adjoint (sign-flipped transposes): leaf Lt from the cotangent
// w into M; the L2P Hessian term into fg from the forward locals in Lc; the
// P2M terms added to fg from the adjoint locals in Lc.
hipError_t launch_w2m(const FarArgs& a, const double4* w64, hipStream_t s);
hipError_t launch_far_hess(const FarArgs& a, const double4* w64, double4* fg, hipStream_t s);
hipError_t launch_far_adj(const FarArgs& a, double4* fg, hipStream_t s);
hipError_t launch_zero_f64(double* p, int64_t n, hipStream_t s);
// Marks the cells whose expansions the far field needs (sources and targets
// of M2L tasks and their subtrees).
hipError_t launch_far_flags(const FarArgs& a, hipStream_t s);

// Occupancy helpers: max resident workgroups per CU of the P2P kernel.
int p2p_blocks_per_cu(int mode, int wg_waves, size_t lds_bytes);
int adjoint_blocks_per_cu(int mode, int wg_waves, bool table);
int n_coef(int order);

}  // namespace pmfmm
