// P2P kernels: the truncated pair force over TaskGroup rows (Sec. 3.2,
// Alg. 1 and Alg. 2), the ordered reduction of work-item partials, and the
// particle gather into leaf order (Sec. 3.1).
//
// Mapping on CDNA4: one wavefront (64 lanes) per work item; lane l holds
// target particle l of the i leaf (Alg. 1: one thread per i particle).
// Sources are read with wave-uniform addresses, so the compiler turns them
// into scalar loads broadcast from SGPRs instead of staging each j leaf
// through LDS; LDS holds the interpolation table of Eq. (int) instead (the
// paper keeps T_i and E_i in shared memory, Sec. 3.3).  Before the pairs
// of a j leaf the wave culls the sources that reach none of its targets
// (device.h).  Work items (i leaf, a range of its j leaves) are pulled by a
// persistent grid from per-XCD segments of the queue (plan.h), longest
// first within a segment, and every item writes its own partial sums,
// which a second kernel adds in a fixed order: results do not depend on
// scheduling.
#include "device.h"

#include <mutex>

// Scratch of pmfmm_forward_static: the queue counters, then the work items'
// partial sums (kStaticCounterBytes + 1536 bytes per item).  Each GPU the
// library runs on holds its own copy until the process ends.  In host code
// `scratch` names a host-side stand-in, never device memory: the device
// address comes from hipGetSymbolAddress (static_scratch below).
static __device__ __align__(256) unsigned char scratch[pmfmm::kStaticScratchBytes];

namespace pmfmm {
namespace {

constexpr float kTwoOverSqrtPiF = 1.12837916709551257390f;

__device__ __forceinline__ int uni(int v) { return __builtin_amdgcn_readfirstlane(v); }

__device__ __forceinline__ void shift_of(int s, double L, double& sx, double& sy, double& sz) {
    sx = (double)(s % 3 - 1) * L;
    sy = (double)((s / 3) % 3 - 1) * L;
    sz = (double)(s / 9 - 1) * L;
}

// Wrap into [0, L); identical steps to the host plan (no contraction).
__device__ __forceinline__ double wrap_coord(double x, double L) {
#pragma clang fp contract(off)
    if (x >= 0.0 && x < L) return x;
    double y = x - L * floor(x / L);
    if (y >= L) y -= L;
    if (y < 0.0) y += L;
    if (!(y >= 0.0 && y < L)) y = 0.0;
    return y;
}

// ------------------------------------------------------------ pair forms

// float64, exact T (truncation_T_f64: one exponential and a polynomial).
// The displacement and r^2 follow the exact steps of the definition
// (d = (x_j - x_i) + s L; r2 = (dx dx + dy dy) + dz dz, no fused
// multiply-add) so the cutoff decision is bit-identical to a plain float64
// evaluation.  Lanes beyond the cutoff skip T (a wave with none inside
// skips it altogether).
template <bool SHIFTED>
__device__ __forceinline__ void pair_f64_exact(const double4 q, double xi, double yi, double zi,
                                               double sx, double sy, double sz, double rc2,
                                               double alpha, double& ax, double& ay, double& az) {
    double dx, dy, dz, r2;
    {
#pragma clang fp contract(off)
        dx = q.x - xi;
        dy = q.y - yi;
        dz = q.z - zi;
        if (SHIFTED) {
            dx = dx + sx;
            dy = dy + sy;
            dz = dz + sz;
        }
        r2 = (dx * dx + dy * dy) + dz * dz;
    }
    if ((r2 > 0.0) & (r2 < rc2)) {
        const double idr = rsqrt(r2);
        const double x = r2 * idr * alpha;
        double ex;
        const double T = truncation_T_f64(x, &ex);
        const double g = q.w * T * (idr * idr * idr);
        ax = fma(g, dx, ax);
        ay = fma(g, dy, ay);
        az = fma(g, dz, az);
    }
}

// float64, Taylor table of Eq. (int) with coefficients pre-scaled to table
// units: T = c0 + e (c1 + e (c2 + e (c3 + e c4))), e = u - d, u = x n_tab / 3.
template <int LEVEL, bool SHIFTED>
__device__ __forceinline__ void pair_f64_table(const double4 q, double xi, double yi, double zi,
                                               double sx, double sy, double sz, double rc2,
                                               double scale, double rnd, int dmax,
                                               const double2* __restrict__ t01,
                                               const double2* __restrict__ t23,
                                               const double* __restrict__ t4, double& ax,
                                               double& ay, double& az) {
    double dx, dy, dz, r2;
    {
#pragma clang fp contract(off)
        dx = q.x - xi;
        dy = q.y - yi;
        dz = q.z - zi;
        if (SHIFTED) {
            dx = dx + sx;
            dy = dy + sy;
            dz = dz + sz;
        }
        r2 = (dx * dx + dy * dy) + dz * dz;
    }
    const bool ok = (r2 > 0.0) & (r2 < rc2);
    const double r2s = ok ? r2 : 1.0;
    const double idr = rsqrt(r2s);
    const double u = r2s * idr * scale;
    int d = (int)(u + rnd);
    d = min(d, dmax);
    const double e = u - (double)d;
    const double2 c01 = t01[d];
    double T;
    if constexpr (LEVEL == 0) {
        T = c01.x;
    } else if constexpr (LEVEL == 1) {
        T = fma(c01.y, e, c01.x);
    } else {
        const double2 c23 = t23[d];
        if constexpr (LEVEL == 2) {
            T = fma(fma(c23.x, e, c01.y), e, c01.x);
        } else if constexpr (LEVEL == 3) {
            T = fma(fma(fma(c23.y, e, c23.x), e, c01.y), e, c01.x);
        } else {
            T = fma(fma(fma(fma(t4[d], e, c23.y), e, c23.x), e, c01.y), e, c01.x);
        }
    }
    const double g = ok ? q.w * T * (idr * idr * idr) : 0.0;
    ax = fma(g, dx, ax);
    ay = fma(g, dy, ay);
    az = fma(g, dz, az);
}

// float32 on cell-relative offsets: (px, py, pz) = target offset minus the
// source leaf's offset, so d = q.xyz - p.  r^2 is clamped into
// [tiny, r_cut^2] before 1/r (tiny = 1e-14 r_cut^2, below float32
// resolution of the offsets): pairs outside the cutoff are masked out
// anyway, the clamp keeps the table index in range, and a coincident pair
// (d = 0) then contributes g * 0 = 0 with a finite g, which is what the
// r^2 > 0 test of the definition gives.
__device__ __forceinline__ void pair_f32_exact(const float4 q, float px, float py, float pz,
                                               float rc2, float tiny, float alpha, float& ax,
                                               float& ay, float& az) {
    const float dx = q.x - px, dy = q.y - py, dz = q.z - pz;
    const float r2 = fmaf(dz, dz, fmaf(dy, dy, dx * dx));
    const bool ok = r2 < rc2;
    const float r2c = __builtin_amdgcn_fmed3f(r2, tiny, rc2);
    const float idr = __builtin_amdgcn_rsqf(r2c);
    const float x = r2c * idr * alpha;
    const float T = erfcf(x) + kTwoOverSqrtPiF * x * expf(-x * x);
    const float g = ok ? q.w * T * (idr * idr * idr) : 0.f;
    ax = fmaf(g, dx, ax);
    ay = fmaf(g, dy, ay);
    az = fmaf(g, dz, az);
}

// Table form: u = x n_tab / 3 + rnd with rnd = 1/2 (nearest node) or 0
// (node below); node d = floor(u), offset e = frac(u) in [0, 1).  The host
// stores each node's Eq. (int) polynomial re-expanded in e (for the nearest
// node it is centred at u = d + 1/2), so no clamp or float conversion of d
// is needed; the table carries one node past x = 3.
template <int LEVEL>
__device__ __forceinline__ void pair_f32_table(const float4 q, float px, float py, float pz,
                                               float rc2, float tiny, float scale, float rnd,
                                               const float4* __restrict__ t03,
                                               const float* __restrict__ t4, float& ax, float& ay,
                                               float& az) {
    const float dx = q.x - px, dy = q.y - py, dz = q.z - pz;
    const float r2 = fmaf(dz, dz, fmaf(dy, dy, dx * dx));
    const bool ok = r2 < rc2;
    const float r2c = __builtin_amdgcn_fmed3f(r2, tiny, rc2);
    const float idr = __builtin_amdgcn_rsqf(r2c);
    const float u = fmaf(r2c * idr, scale, rnd);
    const int d = (int)u;
    const float e = __builtin_amdgcn_fractf(u);
    const float4 c = t03[d];
    float T;
    if constexpr (LEVEL == 0) {
        T = c.x;
    } else if constexpr (LEVEL == 1) {
        T = fmaf(c.y, e, c.x);
    } else if constexpr (LEVEL == 2) {
        T = fmaf(fmaf(c.z, e, c.y), e, c.x);
    } else if constexpr (LEVEL == 3) {
        T = fmaf(fmaf(fmaf(c.w, e, c.z), e, c.y), e, c.x);
    } else {
        T = fmaf(fmaf(fmaf(fmaf(t4[d], e, c.w), e, c.z), e, c.y), e, c.x);
    }
    const float g = ok ? q.w * T * (idr * idr * idr) : 0.f;
    ax = fmaf(g, dx, ax);
    ay = fmaf(g, dy, ay);
    az = fmaf(g, dz, az);
}

// s + c += x with Knuth's TwoSum: the rounding error of s + x, recovered
// exactly in float32 arithmetic, is added into the compensation c.
__device__ __forceinline__ void two_sum(float& s, float& c, float x) {
#pragma clang fp contract(off)
    const float t = s + x;
    const float xv = t - s;
    const float sv = t - xv;
    c += (s - sv) + (x - xv);
    s = t;
}

// Four consecutive sources, read by one wave-uniform load.  pin() is an
// empty statement that takes all sixteen values in scalar registers: it keeps
// the compiler from sinking each source's load into the masked region of its
// pair, which would leave one load and one wait per pair.
template <class V>
struct Src4 {
    V v[4];
};

template <class V>
__device__ __forceinline__ void pin(const Src4<V>& b) {
    asm volatile("" ::"s"(b.v[0].x), "s"(b.v[0].y), "s"(b.v[0].z), "s"(b.v[0].w),
                 "s"(b.v[1].x), "s"(b.v[1].y), "s"(b.v[1].z), "s"(b.v[1].w),
                 "s"(b.v[2].x), "s"(b.v[2].y), "s"(b.v[2].z), "s"(b.v[2].w),
                 "s"(b.v[3].x), "s"(b.v[3].y), "s"(b.v[3].z), "s"(b.v[3].w));
}

// r^2 table (not the paper's table; see the host builder in abi.cpp): the
// whole radial factor F = T(r) / r^3 as a function of s = r'^2, with
// offsets scaled so that r_cut^2 = 2^kR2Emax.  s is clamped below at
// 2^kR2Emin; its float bits (exponent and top `bits` mantissa bits) index
// the segment directly (2^bits segments per octave), and each row holds F's
// polynomial in s itself; no 1/r is evaluated at all.  A coincident pair
// (d = 0) gets a finite F times d = 0.  Only lanes inside the cutoff read
// the table and add: most candidate pairs lie beyond r_cut (about three in
// four in clustered boxes), and an LDS read costs its issue slot whatever
// its active lanes, so a wave whose lanes are all beyond r_cut for a source
// skips the read altogether.
template <int LEVEL, bool UNI, int BITS>
__device__ __forceinline__ void pair_f32_r2(const float4 q, float px, float py, float pz,
                                            float smax, float smin, uint32_t shift,
                                            uint32_t boff, const unsigned char* __restrict__ tab,
                                            float& ax, float& ay, float& az) {
    // row k of the table: (c0, c1) at 8 k, (c2, 0) at kC2 + 8 k (an
    // immediate offset of the same address)
    constexpr int kC2 = r2_plane_c2(BITS);
    const float dx = q.x - px, dy = q.y - py, dz = q.z - pz;
    const float r2 = fmaf(dz, dz, fmaf(dy, dy, dx * dx));
    if (r2 < smax) {
        // r2 >= +0, so the clamp below smin is an unsigned max of the bits
        const uint32_t sb = max(__float_as_uint(r2), __float_as_uint(smin));
        const float sc = __uint_as_float(sb);
        // boff = -(row of 2^kR2Emin) * 8 mod 2^32: one shift-add per address
        const unsigned char* c = tab + (((sb >> shift) << 3) + boff);
        const float2 c01 = *reinterpret_cast<const float2*>(c);
        float F;
        if constexpr (LEVEL == 1) {
            F = fmaf(c01.y, sc, c01.x);
        } else {
            F = fmaf(fmaf(*reinterpret_cast<const float*>(c + kC2), sc, c01.y), sc, c01.x);
        }
        // UNI: the j leaf's sources share one mass, applied once per leaf
        const float g = UNI ? F : q.w * F;
        ax = fmaf(g, dx, ax);
        ay = fmaf(g, dy, ay);
        az = fmaf(g, dz, az);
    }
}

// A pair of the linear r^2 form closer than its table's floor (0 < s <
// sfloor; the main pass read the zero row for it): F from erfcf / expf, s
// clamped below at tiny as in the quadratic form.  Coincident pairs (s = 0)
// contribute nothing either way.
template <bool UNI>
__device__ __forceinline__ void pair_f32_close(const float4 q, float px, float py, float pz,
                                               float sfloor, float tiny, float alpha, float& ax,
                                               float& ay, float& az) {
    const float dx = q.x - px, dy = q.y - py, dz = q.z - pz;
    const float r2 = fmaf(dz, dz, fmaf(dy, dy, dx * dx));
    if (r2 < sfloor && r2 > 0.f) {
        const float r2c = fmaxf(r2, tiny);
        const float idr = __builtin_amdgcn_rsqf(r2c);
        const float x = r2c * idr * alpha;
        const float T = erfcf(x) + kTwoOverSqrtPiF * x * expf(-x * x);
        const float g = (UNI ? 1.f : q.w) * T * (idr * idr * idr);
        ax = fmaf(g, dx, ax);
        ay = fmaf(g, dy, ay);
        az = fmaf(g, dz, az);
    }
}

// The pairs of one j leaf in the float32 r^2 form: four sources per 64-byte
// scalar load, ahead of the masked table reads.  With a linear table
// (LEVEL 1), the sources in `near` (those that may come closer than the
// table's floor to a target) then go through pair_f32_close.
template <int LEVEL, bool UNI, int BITS>
__device__ __forceinline__ void leaf_f32_r2(const float4* __restrict__ src, int nj, uint64_t live,
                                            float px, float py, float pz, float smax,
                                            float smin, uint32_t shift, uint32_t boff,
                                            const unsigned char* __restrict__ tab, float& ax,
                                            float& ay, float& az, uint64_t near = 0,
                                            float sfloor = 0.f, float tiny = 0.f,
                                            float alpha = 0.f) {
    int k = 0;
    for (; k + 4 <= nj; k += 4) {
        const uint32_t g4 = (uint32_t)(live >> k) & 0xFu;
        if (g4 == 0) continue;
        const Src4<float4> b = *reinterpret_cast<const Src4<float4>*>(src + k);
        pin(b);
#pragma unroll
        for (int u = 0; u < 4; ++u)
            if (g4 & (1u << u))
                pair_f32_r2<LEVEL, UNI, BITS>(b.v[u], px, py, pz, smax, smin, shift, boff, tab, ax,
                                              ay, az);
    }
    for (; k < nj; ++k)
        if ((live >> k) & 1u)
            pair_f32_r2<LEVEL, UNI, BITS>(src[k], px, py, pz, smax, smin, shift, boff, tab, ax, ay,
                                          az);
    if constexpr (LEVEL == 1) {
        for (uint64_t m = near; m != 0; m &= m - 1)
            pair_f32_close<UNI>(src[__builtin_ctzll(m)], px, py, pz, sfloor, tiny, alpha, ax, ay,
                                az);
    }
}

// live_f32's cull, plus the sources whose squared distance to the targets'
// box is below near2 (in `near`).
__device__ __forceinline__ uint64_t live_near_f32(const float4* __restrict__ src, int nj, int lane,
                                                  float3 plo, float3 phi, float rc2, float near2,
                                                  uint64_t& near) {
    const float4 q = src[lane < nj ? lane : 0];
    const float bx = fmaxf(fmaxf(plo.x - q.x, q.x - phi.x), 0.f);
    const float by = fmaxf(fmaxf(plo.y - q.y, q.y - phi.y), 0.f);
    const float bz = fmaxf(fmaxf(plo.z - q.z, q.z - phi.z), 0.f);
    const float d2 = fmaf(bz, bz, fmaf(by, by, bx * bx));
    near = __ballot((lane < nj) & (d2 < near2));
    return __ballot((lane < nj) & (d2 < rc2));
}

// float64 r^2 table (not the paper's table; host builder in abi.cpp): the
// scaled radial factor F = T(r) / r^3 / sigma^3 of s = r^2 sigma^2, with
// sigma^2 = 2^kR2Emax / r_cut^2, on segments of [2^kR2Emin64, 2^kR2Emax)
// indexed by the high 32 bits of s (exponent and top `bits` mantissa bits);
// each row holds the NC coefficients of the segment's polynomial in
// t = s - s_k (s_k the segment start: the same high bits, zero below).  The
// cutoff test is the definition's, on r^2 itself; a pair inside it has
// s <= 2^11, and the row after the last segment holds F(2^11) for a pair
// whose scaled s rounds up to 2^11.  As in the float32 form, only lanes
// inside the cutoff read the table.  A pair closer than 2^(kR2Emin64 / 2)
// r_cut (r < r_cut / 256, rare) or at r = 0 contributes nothing here and
// raises the lane's `near` flag; pair_f64_r2_close then adds the close pairs
// of that j leaf with the library erfc / exp (rare: no need for the faster
// truncation_T_f64, whose registers would crowd the main loop's).  The item's sums are
// multiplied by sigma^3 at the end.
struct R2Tab64 {
    const unsigned char* tab;  // LDS rows of NC doubles
    double rc2, sig2, alpha;
    uint32_t hlo;              // high word of 2^kR2Emin64
    uint32_t hshift, hmask;    // segment = hi >> hshift; start = hi & hmask
    uint32_t hoff;             // -(row of hlo) * row bytes, mod 2^32
};

template <bool SHIFTED>
__device__ __forceinline__ double disp_r2(const double4 q, double xi, double yi, double zi,
                                          double sx, double sy, double sz, double& dx,
                                          double& dy, double& dz) {
#pragma clang fp contract(off)
    dx = q.x - xi;
    dy = q.y - yi;
    dz = q.z - zi;
    if (SHIFTED) {
        dx = dx + sx;
        dy = dy + sy;
        dz = dz + sz;
    }
    return (dx * dx + dy * dy) + dz * dz;
}

template <int NC, bool SHIFTED>
__device__ __forceinline__ void pair_f64_r2(const double4 q, double xi, double yi, double zi,
                                            double sx, double sy, double sz, const R2Tab64& T,
                                            double& ax, double& ay, double& az, bool& near) {
    double dx, dy, dz;
    const double r2 = disp_r2<SHIFTED>(q, xi, yi, zi, sx, sy, sz, dx, dy, dz);
    const double s = r2 * T.sig2;
    const uint32_t hi = (uint32_t)__double2hiint(s);
    const bool low = hi < T.hlo;
    near |= low;
    if (!low & (r2 < T.rc2)) {
        const double* __restrict__ c =
            reinterpret_cast<const double*>(T.tab + (__umul24(hi >> T.hshift, NC * 8) + T.hoff));
        const double t = s - __hiloint2double((int)(hi & T.hmask), 0);
        double F = c[NC - 1];
#pragma unroll
        for (int k = NC - 2; k >= 0; --k) F = fma(F, t, c[k]);
        const double g = q.w * F;
        ax = fma(g, dx, ax);
        ay = fma(g, dy, ay);
        az = fma(g, dz, az);
    }
}

template <bool SHIFTED>
__device__ __forceinline__ void pair_f64_r2_close(const double4 q, double xi, double yi, double zi,
                                                  double sx, double sy, double sz,
                                                  const R2Tab64& T, double& ax, double& ay,
                                                  double& az) {
    double dx, dy, dz;
    const double r2 = disp_r2<SHIFTED>(q, xi, yi, zi, sx, sy, sz, dx, dy, dz);
    const double s = r2 * T.sig2;
    if (r2 > 0.0 && (uint32_t)__double2hiint(s) < T.hlo) {
        const double r = sqrt(r2);
        const double x = r * T.alpha;
        const double Tx = erfc(x) + 1.12837916709551257390 * x * exp(-x * x);
        const double g = q.w * (Tx / (s * sqrt(s)));
        ax = fma(g, dx, ax);
        ay = fma(g, dy, ay);
        az = fma(g, dz, az);
    }
}

template <int NC, bool SHIFTED>
__device__ __forceinline__ void leaf_f64_r2(const double4* __restrict__ src, int nj,
                                            uint64_t live, double xi,
                                            double yi, double zi, double sx, double sy, double sz,
                                            const R2Tab64& T, double& ax, double& ay, double& az) {
    bool near = false;
    int k = 0;
    for (; k + 4 <= nj; k += 4) {
        const uint32_t g4 = (uint32_t)(live >> k) & 0xFu;
        if (g4 == 0) continue;
        const Src4<double4> b = *reinterpret_cast<const Src4<double4>*>(src + k);
        pin(b);
#pragma unroll
        for (int u = 0; u < 4; ++u)
            if (g4 & (1u << u))
                pair_f64_r2<NC, SHIFTED>(b.v[u], xi, yi, zi, sx, sy, sz, T, ax, ay, az, near);
    }
    for (; k < nj; ++k)
        if ((live >> k) & 1u)
            pair_f64_r2<NC, SHIFTED>(src[k], xi, yi, zi, sx, sy, sz, T, ax, ay, az, near);
    if (near)
        for (int k = 0; k < nj; ++k)
            if ((live >> k) & 1u)
                pair_f64_r2_close<SHIFTED>(src[k], xi, yi, zi, sx, sy, sz, T, ax, ay, az);
}

// LDS table layouts (bytes), matching the host builder in abi.cpp:
//   float64 r^2 table: double c0 .. c(NC-1) per row [16 2^bits rows]
//   float32 r^2 table: float2 (c0, c1) [r2_rows(bits)] at 0, then
//                      float2 (c2, 0) [r2_rows(bits)] at r2_plane_c2(bits)
//   linear float32 r^2 table: float2 (c0, c1) [r2_rows_lin(bits)], the
//                      first and the last row zero
//   float32: float4 c0..c3 [n_tab + 1], then float c4 [n_tab + 1]
//   float64: double2 (c0, c1) [n_tab], double2 (c2, c3) [n_tab], double c4 [n_tab]
__device__ __forceinline__ void load_table(unsigned char* lds, const void* __restrict__ table,
                                           int bytes) {
    const uint4* src = reinterpret_cast<const uint4*>(table);
    uint4* dst = reinterpret_cast<uint4*>(lds);
    for (int i = threadIdx.x; i < bytes / 16; i += blockDim.x) dst[i] = src[i];
    __syncthreads();
}

template <int MODE, int LEVEL, bool ACC32, int BITS>
__global__ void __launch_bounds__(p2p_max_threads(MODE), p2p_min_waves_per_simd(MODE))
p2p_kernel(const double4* __restrict__ x64, const float4* __restrict__ x32,
           const int4* __restrict__ leaf, const double4* __restrict__ leafc,
           const int32_t* __restrict__ p2p_js, const int4* __restrict__ items,
           const int32_t* __restrict__ queue, int32_t n_items, int32_t* __restrict__ counter,
           double* __restrict__ partial, const BoxDev* __restrict__ boxes,
           const void* __restrict__ table, int32_t n_tab, int32_t table_bytes,
           int32_t round_floor) {
    extern __shared__ __align__(16) unsigned char lds[];
    constexpr bool kTable = (MODE == kFP64Table) || (MODE == kFP32Table) || (MODE == kFP32R2) ||
                            (MODE == kFP64R2);
    if constexpr (kTable) load_table(lds, table, table_bytes);
    const int lane = threadIdx.x & 63;
    const int dmax = n_tab - 1;

    int seg = (int)(blockIdx.x % kQueueSegs), done = 0;
    for (;;) {
        const int beg = queue_seg_begin(seg, n_items);
        int q = 0;
        if (lane == 0) q = atomicAdd(counter + seg * kCounterStride, 1);
        q = uni(q);
        if (q >= queue_seg_begin(seg + 1, n_items) - beg) {
            // this segment is exhausted (for good: its counter only grows)
            if (++done == kQueueSegs) break;
            seg = seg + 1 == kQueueSegs ? 0 : seg + 1;
            continue;
        }
        const int slot = uni(queue[beg + q]);
        const int4 it = items[slot];
        const int il = uni(it.x), t0 = uni(it.y), t1 = uni(it.z);
        const int4 li = leaf[il];
        const int ni = uni(li.y);
        const int pi = uni(li.x) + (lane < ni ? lane : 0);
        const BoxDev bx = boxes[uni(li.z)];
        const double4 ci = leafc[il];
        double ax = 0.0, ay = 0.0, az = 0.0;

        if constexpr (is_fp32(MODE)) {
            const float4 pv = x32[pi];
            const float rc2 = bx.rc2_f, tiny = bx.tiny_f;
            const double sig = bx.sigma;
            const float rnd = round_floor ? 0.f : 0.5f;
            const float4* t03 = reinterpret_cast<const float4*>(lds);
            const float* t4 = reinterpret_cast<const float*>(lds + 16 * (n_tab + 1));
            // r^2 table: n_tab = segments per octave = 2^bits (runtime values,
            // so that the address is one shift and one shift-add)
            const uint32_t r2bits = 31u - (uint32_t)__builtin_clz((uint32_t)n_tab);
            const uint32_t r2shift = 23u - r2bits;
            // the quadratic tables start at 2^kR2Emin; the linear ones have
            // their zero row at the segment just below 2^kR2EminLin, which
            // is where the clamp at smin (the float below the floor) puts
            // every closer pair
            constexpr bool kLin = MODE == kFP32R2 && LEVEL == 1;
            const uint32_t r2boff =
                kLin ? 0u - ((((uint32_t)(127 + kR2EminLin) << r2bits) - 1u) << 3)
                     : 0u - (((uint32_t)(127 + kR2Emin) << r2bits) << 3);
            const float sfloor = kLin ? __uint_as_float((uint32_t)(127 + kR2EminLin) << 23) : 0.f;
            const float smin = kLin ? __uint_as_float(__float_as_uint(sfloor) - 1u) : tiny;
            // a target closer than the floor to a source is within 2 sqrt(floor)
            // of the targets' box (float32 rounding moves distances by ~1e-5
            // of the floor's 2^-4)
            const float near2 = 4.f * sfloor;
            // box of the wave's targets in their leaf's frame (lanes past
            // the leaf repeat target 0)
            float3 lo = make_float3(pv.x, pv.y, pv.z), hi = lo;
            wave_box(lo, hi);
            // compensated float32 item sums (accum32): s + c
            float3 s32 = make_float3(0.f, 0.f, 0.f), c32 = s32;
            for (int t = t0; t < t1; ++t) {
                const int js = uni(p2p_js[t]);
                const int jl = js >> 5;
                const int4 lj = leaf[jl];
                const double4 cj = leafc[jl];
                double sx, sy, sz;
                shift_of(js & 31, bx.L, sx, sy, sz);
                const float offx = (float)(((cj.x - ci.x) + sx) * sig);
                const float offy = (float)(((cj.y - ci.y) + sy) * sig);
                const float offz = (float)(((cj.z - ci.z) + sz) * sig);
                const float px = pv.x - offx;
                const float py = pv.y - offy;
                const float pz = pv.z - offz;
                const float4* __restrict__ src = x32 + uni(lj.x);
                const int nj = uni(lj.y);
                float fx = 0.f, fy = 0.f, fz = 0.f;
                // targets in this frame: [lo - off, hi - off] per axis
                // (exact: the shift is monotonic)
                uint64_t near = 0;
                const float3 blo = make_float3(lo.x - offx, lo.y - offy, lo.z - offz);
                const float3 bhi = make_float3(hi.x - offx, hi.y - offy, hi.z - offz);
                const uint64_t live = kLin ? live_near_f32(src, nj, lane, blo, bhi, rc2, near2, near)
                                           : live_f32(src, nj, lane, blo, bhi, rc2);
                if constexpr (MODE == kFP32Exact) {
                    for (int k = 0; k < nj; ++k)
                        if ((live >> k) & 1u)
                            pair_f32_exact(src[k], px, py, pz, rc2, tiny, bx.alpha_f, fx, fy, fz);
                } else if constexpr (MODE == kFP32Table) {
#pragma unroll 4
                    for (int k = 0; k < nj; ++k)
                        if ((live >> k) & 1u)
                            pair_f32_table<LEVEL>(src[k], px, py, pz, rc2, tiny, bx.tab_scale_f,
                                                  rnd, t03, t4, fx, fy, fz);
                } else if (cj.w != 0.0) {
                    // every source of the j leaf has mass cj.w (the gather
                    // marks such leaves): one multiplication per leaf
                    // instead of one per pair
                    leaf_f32_r2<LEVEL, true, BITS>(src, nj, live, px, py, pz, rc2, smin, r2shift,
                                                   r2boff, lds, fx, fy, fz, near, sfloor, tiny,
                                                   bx.alpha_f);
                    const float mu = (float)cj.w;
                    fx *= mu;
                    fy *= mu;
                    fz *= mu;
                } else {
                    leaf_f32_r2<LEVEL, false, BITS>(src, nj, live, px, py, pz, rc2, smin, r2shift,
                                                    r2boff, lds, fx, fy, fz, near, sfloor, tiny,
                                                    bx.alpha_f);
                }
                if constexpr (ACC32) {
                    two_sum(s32.x, c32.x, fx);
                    two_sum(s32.y, c32.y, fy);
                    two_sum(s32.z, c32.z, fz);
                } else {
                    ax += (double)fx;
                    ay += (double)fy;
                    az += (double)fz;
                }
            }
            if constexpr (ACC32) {
                ax = (double)s32.x + (double)c32.x;
                ay = (double)s32.y + (double)c32.y;
                az = (double)s32.z + (double)c32.z;
            }
            const double s2 = sig * sig;
            ax *= s2;
            ay *= s2;
            az *= s2;
        } else {
            const double4 pv = x64[pi];
            const double rc2 = bx.rc2;
            const double rnd = round_floor ? 0.0 : 0.5;
            const double2* t01 = reinterpret_cast<const double2*>(lds);
            const double2* t23 = reinterpret_cast<const double2*>(lds + 16 * n_tab);
            const double* t4 = reinterpret_cast<const double*>(lds + 32 * n_tab);
            // float64 r^2 table: n_tab = segments per octave = 2^bits
            R2Tab64 r2t;
            if constexpr (MODE == kFP64R2) {
                const uint32_t hbits =
                    31u - (uint32_t)__builtin_clz((uint32_t)(n_tab > 0 ? n_tab : 1));
                r2t.tab = lds;
                r2t.rc2 = rc2;
                r2t.sig2 = (double)(1 << kR2Emax) / rc2;
                r2t.alpha = bx.alpha;
                r2t.hshift = 20u - hbits;
                r2t.hmask = ~((1u << r2t.hshift) - 1u);
                r2t.hlo = (uint32_t)(1023 + kR2Emin64) << 20;
                r2t.hoff = 0u - (r2t.hlo >> r2t.hshift) * (uint32_t)((LEVEL + 1) * 8);
            }
            double3 lo = make_double3(pv.x, pv.y, pv.z), hi = lo;
            wave_box(lo, hi);
            for (int t = t0; t < t1; ++t) {
                const int js = uni(p2p_js[t]);
                const int jl = js >> 5;
                const int s = js & 31;
                const int4 lj = leaf[jl];
                double sx, sy, sz;
                shift_of(s, bx.L, sx, sy, sz);
                const double4* __restrict__ src = x64 + uni(lj.x);
                const int nj = uni(lj.y);
                const uint64_t live =
                    s == 13 ? live_f64<false>(src, nj, lane, lo, hi, 0.0, 0.0, 0.0, rc2)
                            : live_f64<true>(src, nj, lane, lo, hi, sx, sy, sz, rc2);
                if constexpr (MODE == kFP64R2) {
                    if (s == 13)
                        leaf_f64_r2<LEVEL + 1, false>(src, nj, live, pv.x, pv.y, pv.z, 0.0, 0.0,
                                                      0.0, r2t, ax, ay, az);
                    else
                        leaf_f64_r2<LEVEL + 1, true>(src, nj, live, pv.x, pv.y, pv.z, sx, sy, sz,
                                                     r2t, ax, ay, az);
                } else if (s == 13) {
                    for (int k = 0; k < nj; ++k) {
                        if (!((live >> k) & 1u)) continue;
                        if constexpr (MODE == kFP64Exact)
                            pair_f64_exact<false>(src[k], pv.x, pv.y, pv.z, 0.0, 0.0, 0.0, rc2,
                                                  bx.alpha, ax, ay, az);
                        else
                            pair_f64_table<LEVEL, false>(src[k], pv.x, pv.y, pv.z, 0.0, 0.0, 0.0,
                                                         rc2, bx.tab_scale, rnd, dmax, t01, t23,
                                                         t4, ax, ay, az);
                    }
                } else {
                    for (int k = 0; k < nj; ++k) {
                        if (!((live >> k) & 1u)) continue;
                        if constexpr (MODE == kFP64Exact)
                            pair_f64_exact<true>(src[k], pv.x, pv.y, pv.z, sx, sy, sz, rc2,
                                                 bx.alpha, ax, ay, az);
                        else
                            pair_f64_table<LEVEL, true>(src[k], pv.x, pv.y, pv.z, sx, sy, sz, rc2,
                                                        bx.tab_scale, rnd, dmax, t01, t23, t4, ax,
                                                        ay, az);
                    }
                }
            }
            if constexpr (MODE == kFP64R2) {
                const double sig3 = r2t.sig2 * sqrt(r2t.sig2);
                ax *= sig3;
                ay *= sig3;
                az *= sig3;
            }
        }
        double* dst = partial + (size_t)slot * 192;
        dst[lane] = ax;
        dst[64 + lane] = ay;
        dst[128 + lane] = az;
    }
}

// One wavefront per leaf: sum the leaf's item partials in slot order, add
// the far-field part (leaves with a local expansion), scale by G and
// scatter to the caller's order.
__global__ void __launch_bounds__(256)
reduce_kernel(const int4* __restrict__ leaf, const int32_t* __restrict__ leaf_slot,
              const double* __restrict__ partial, const double* __restrict__ far,
              const int32_t* __restrict__ needL, const int32_t* __restrict__ perm,
              const BoxDev* __restrict__ boxes, double* __restrict__ out, int32_t n_leaves) {
    const int l = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (l >= n_leaves) return;
    const int4 li = leaf[l];
    if (lane >= li.y) return;
    const int s0 = leaf_slot[l], s1 = leaf_slot[l + 1];
    double ax = 0.0, ay = 0.0, az = 0.0;
    for (int s = s0; s < s1; ++s) {
        const double* p = partial + (size_t)s * 192;
        ax += p[lane];
        ay += p[64 + lane];
        az += p[128 + lane];
    }
    const int k = li.x + lane;
    if (far != nullptr && needL[li.w]) {   // L2P wrote only these leaves
        ax += far[3 * (size_t)k];
        ay += far[3 * (size_t)k + 1];
        az += far[3 * (size_t)k + 2];
    }
    const double G = boxes[li.z].G;
    const int o = perm[k];
    out[3 * (size_t)o] = G * ax;
    out[3 * (size_t)o + 1] = G * ay;
    out[3 * (size_t)o + 2] = G * az;
}

// One wavefront per leaf: particles into leaf order, wrapped, as float64
// records and as float32 offsets from the leaf centre.
__global__ void __launch_bounds__(256)
gather_kernel(const double* __restrict__ pos_in, const double* __restrict__ mass_in,
              const int32_t* __restrict__ perm, const int4* __restrict__ leaf,
              double4* __restrict__ leafc, const BoxDev* __restrict__ boxes,
              double4* __restrict__ x64, float4* __restrict__ x32, int32_t n_leaves) {
    const int l = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (l >= n_leaves) return;
    const int4 li = leaf[l];
    if (lane >= li.y) return;
    const int k = li.x + lane;
    const int o = perm[k];
    const double L = boxes[li.z].L;
    const double x = wrap_coord(pos_in[3 * (size_t)o], L);
    const double y = wrap_coord(pos_in[3 * (size_t)o + 1], L);
    const double z = wrap_coord(pos_in[3 * (size_t)o + 2], L);
    const double m = mass_in[o];
    x64[k] = make_double4(x, y, z, m);
    // leafc[l].w: the mass every particle of the leaf has, or 0 when they
    // differ (the float32 r^2 P2P applies it once per leaf)
    {
        const double m0 = __shfl(m, 0);
        const uint64_t act = __ballot(1);
        const bool same = m == m0;
        if (lane == 0) leafc[l].w = (__ballot(same) == act) ? m0 : 0.0;
    }
    const double4 c = leafc[l];
    const double sig = boxes[li.z].sigma;
    x32[k] = make_float4((float)((x - c.x) * sig), (float)((y - c.y) * sig),
                         (float)((z - c.z) * sig), (float)m);
}

// x32 again from x64 after the boxes' sigma changed.
__global__ void __launch_bounds__(256)
rescale_x32_kernel(const int4* __restrict__ leaf, const double4* __restrict__ leafc,
                   const BoxDev* __restrict__ boxes, const double4* __restrict__ x64,
                   float4* __restrict__ x32, int32_t n_leaves) {
    const int l = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (l >= n_leaves) return;
    const int4 li = leaf[l];
    if (lane >= li.y) return;
    const int k = li.x + lane;
    const double4 p = x64[k];
    const double4 c = leafc[l];
    const double sig = boxes[li.z].sigma;
    x32[k] = make_float4((float)((p.x - c.x) * sig), (float)((p.y - c.y) * sig),
                         (float)((p.z - c.z) * sig), (float)p.w);
}

__global__ void zero_i32_kernel(int32_t* p, int32_t n) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0;
}

template <int MODE, int LEVEL, int BITS = 0>
hipError_t launch_one(const P2PArgs& a, int wg_waves, int grid_wgs, size_t lds, hipStream_t s) {
    const int tb = (int)lds;
    // the compensated float32 sums are a variant of the float32 kernels only
    if (is_fp32(MODE) && a.accum32)
        hipLaunchKernelGGL((p2p_kernel<MODE, LEVEL, is_fp32(MODE), BITS>), dim3(grid_wgs),
                           dim3(64 * wg_waves), lds, s, a.x64, a.x32, a.leaf, a.leafc, a.p2p_js,
                           a.items, a.queue, a.n_items, a.counter, a.partial, a.boxes, a.table,
                           a.n_tab, tb, a.round_floor);
    else
        hipLaunchKernelGGL((p2p_kernel<MODE, LEVEL, false, BITS>), dim3(grid_wgs),
                           dim3(64 * wg_waves), lds, s, a.x64, a.x32, a.leaf, a.leafc, a.p2p_js,
                           a.items, a.queue, a.n_items, a.counter, a.partial, a.boxes, a.table,
                           a.n_tab, tb, a.round_floor);
    return hipGetLastError();
}

// The float32 r^2 form at its segments per octave (n_tab = 2^BITS): 16 to
// 128 for the quadratic tables, 64 to 512 for the linear ones.
template <int LEVEL>
hipError_t launch_r2(const P2PArgs& a, int wg_waves, int grid_wgs, size_t lds, hipStream_t s) {
    if constexpr (LEVEL == 1) {
        switch (a.n_tab) {
            case 64: return launch_one<kFP32R2, 1, 6>(a, wg_waves, grid_wgs, lds, s);
            case 128: return launch_one<kFP32R2, 1, 7>(a, wg_waves, grid_wgs, lds, s);
            case 256: return launch_one<kFP32R2, 1, 8>(a, wg_waves, grid_wgs, lds, s);
            case 512: return launch_one<kFP32R2, 1, 9>(a, wg_waves, grid_wgs, lds, s);
        }
    } else {
        switch (a.n_tab) {
            case 16: return launch_one<kFP32R2, LEVEL, 4>(a, wg_waves, grid_wgs, lds, s);
            case 32: return launch_one<kFP32R2, LEVEL, 5>(a, wg_waves, grid_wgs, lds, s);
            case 64: return launch_one<kFP32R2, LEVEL, 6>(a, wg_waves, grid_wgs, lds, s);
            case 128: return launch_one<kFP32R2, LEVEL, 7>(a, wg_waves, grid_wgs, lds, s);
        }
    }
    return hipErrorInvalidValue;
}

template <int MODE, int LEVEL>
int occ_one(int wg_waves, size_t lds) {
    int blocks = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, p2p_kernel<MODE, LEVEL, false, MODE == kFP32R2 ? 6 : 0>,
                                                     64 * wg_waves, lds) != hipSuccess)
        return 1;
    return blocks > 0 ? blocks : 1;
}

}  // namespace

hipError_t launch_p2p(int mode, const P2PArgs& a, int wg_waves, int grid_wgs, size_t lds,
                      hipStream_t s) {
    if (a.n_items == 0) return hipSuccess;
    switch (mode) {
        case kFP64Exact: return launch_one<kFP64Exact, 0>(a, wg_waves, grid_wgs, 0, s);
        case kFP32Exact: return launch_one<kFP32Exact, 0>(a, wg_waves, grid_wgs, 0, s);
        case kFP32Table:
            switch (a.level) {
                case 0: return launch_one<kFP32Table, 0>(a, wg_waves, grid_wgs, lds, s);
                case 1: return launch_one<kFP32Table, 1>(a, wg_waves, grid_wgs, lds, s);
                case 2: return launch_one<kFP32Table, 2>(a, wg_waves, grid_wgs, lds, s);
                case 3: return launch_one<kFP32Table, 3>(a, wg_waves, grid_wgs, lds, s);
                default: return launch_one<kFP32Table, 4>(a, wg_waves, grid_wgs, lds, s);
            }
        case kFP32R2:
            if (a.level == 1) return launch_r2<1>(a, wg_waves, grid_wgs, lds, s);
            return launch_r2<2>(a, wg_waves, grid_wgs, lds, s);
        case kFP64R2:
            switch (a.level) {
                case 4: return launch_one<kFP64R2, 4>(a, wg_waves, grid_wgs, lds, s);
                case 5: return launch_one<kFP64R2, 5>(a, wg_waves, grid_wgs, lds, s);
                default: return launch_one<kFP64R2, 6>(a, wg_waves, grid_wgs, lds, s);
            }
        case kFP64Table:
            switch (a.level) {
                case 0: return launch_one<kFP64Table, 0>(a, wg_waves, grid_wgs, lds, s);
                case 1: return launch_one<kFP64Table, 1>(a, wg_waves, grid_wgs, lds, s);
                case 2: return launch_one<kFP64Table, 2>(a, wg_waves, grid_wgs, lds, s);
                case 3: return launch_one<kFP64Table, 3>(a, wg_waves, grid_wgs, lds, s);
                default: return launch_one<kFP64Table, 4>(a, wg_waves, grid_wgs, lds, s);
            }
    }
    return hipErrorInvalidValue;
}

int p2p_blocks_per_cu(int mode, int wg_waves, size_t lds) {
    switch (mode) {
        case kFP64Exact: return occ_one<kFP64Exact, 0>(wg_waves, 0);
        case kFP32Exact: return occ_one<kFP32Exact, 0>(wg_waves, 0);
        case kFP32Table: return occ_one<kFP32Table, 2>(wg_waves, lds);
        case kFP32R2: return occ_one<kFP32R2, 2>(wg_waves, lds);
        case kFP64R2: return occ_one<kFP64R2, 6>(wg_waves, lds);
        default: return occ_one<kFP64Table, 4>(wg_waves, lds);
    }
}

hipError_t launch_reduce(const ReduceArgs& a, hipStream_t s) {
    if (a.n_leaves == 0) return hipSuccess;
    const int wgs = (a.n_leaves + 3) / 4;
    hipLaunchKernelGGL(reduce_kernel, dim3(wgs), dim3(256), 0, s, a.leaf, a.leaf_slot, a.partial,
                       a.far, a.needL, a.perm, a.boxes, a.out, a.n_leaves);
    return hipGetLastError();
}

hipError_t launch_gather(const GatherArgs& a, const double* /*unused*/, hipStream_t s) {
    if (a.n_leaves == 0) return hipSuccess;
    const int wgs = (a.n_leaves + 3) / 4;
    hipLaunchKernelGGL(gather_kernel, dim3(wgs), dim3(256), 0, s, a.pos_in, a.mass_in, a.perm,
                       a.leaf, a.leafc, a.boxes, a.x64, a.x32, a.n_leaves);
    return hipGetLastError();
}

hipError_t launch_rescale_x32(const int4* leaf, const double4* leafc, const BoxDev* boxes,
                              const double4* x64, float4* x32, int32_t n_leaves, hipStream_t s) {
    if (n_leaves == 0) return hipSuccess;
    hipLaunchKernelGGL(rescale_x32_kernel, dim3((n_leaves + 3) / 4), dim3(256), 0, s, leaf, leafc,
                       boxes, x64, x32, n_leaves);
    return hipGetLastError();
}

hipError_t static_scratch(void** out) {
    // one address per device, resolved on the first call with that device
    // current (each GPU holds its own copy of the array)
    constexpr int kMaxDevices = 64;
    static std::mutex mu;
    static void* addr[kMaxDevices] = {};
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(mu);
    if (addr[dev] == nullptr) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (p == nullptr) return hipErrorInvalidSymbol;
        addr[dev] = p;
    }
    *out = addr[dev];
    return hipSuccess;
}

hipError_t launch_zero_i32(int32_t* p, int32_t n, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(zero_i32_kernel, dim3((n + 255) / 256), dim3(256), 0, s, p, n);
    return hipGetLastError();
}

}  // namespace pmfmm
