// Adjoint of the P2P short-range force (not in the paper; derived from the
// pair sum of Sec. 2, Eq. (tr)).
//
// For the loss L = sum_i w_i . a_i with a_i = G sum_l m_l g(r) d_il,
// d = x_l + s L - x_i, g = T / r^3, and h = g'(r) / r =
// -(3 T + (4 / sqrt(pi)) x^3 exp(-x^2)) / r^5 (x = r / 2 r_s), the gradient
// gathered over particle k's own neighbours (the P2P lists are symmetric) is
//   dL/dx_k = G [ m_k sum_l (g w_l + h (d.w_l) d) - sum_l m_l (g w_k + h (d.w_k) d) ]
//   dL/dm_k = -G sum_l g (w_l . d),                            d = d_kl,
// the delta function of the hard cutoff being left out.  Same wavefront
// mapping and work queue as the forward P2P kernel; the source records are
// (x, m) and (w, 0), both read with wave-uniform addresses.  g and h are
// evaluated exactly (float64: truncation_T_f64, one exponential; float32:
// erfcf and expf), or, in the float32 r^2 form, read from quadratic tables
// in r^2 (adj_pair_f32_r2).
#include "device.h"

namespace pmfmm {
namespace {

constexpr double kFourOverSqrtPi = 2.25675833419102514780;
constexpr float kTwoOverSqrtPiF = 1.12837916709551257390f;
constexpr float kFourOverSqrtPiF = 2.25675833419102514780f;

__device__ __forceinline__ int uni(int v) { return __builtin_amdgcn_readfirstlane(v); }

template <bool SHIFTED>
__device__ __forceinline__ void adj_pair_f64(const double4 q, const double4 wl, double xk,
                                             double yk, double zk, double4 wk, double sx,
                                             double sy, double sz, double rc2, double alpha,
                                             double* A, double* Bv, double& gm) {
    double dx, dy, dz, r2;
    {
#pragma clang fp contract(off)
        dx = q.x - xk;
        dy = q.y - yk;
        dz = q.z - zk;
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
        const double idr2 = idr * idr;
        const double g = T * idr * idr2;
        const double h = -(3.0 * T + kFourOverSqrtPi * x * x * x * ex) * idr2 * idr2 * idr;
        const double dwl = dx * wl.x + dy * wl.y + dz * wl.z;
        const double dwk = dx * wk.x + dy * wk.y + dz * wk.z;
        const double hl = h * dwl, hk = q.w * h * dwk, gl = q.w * g;
        A[0] += g * wl.x + hl * dx;
        A[1] += g * wl.y + hl * dy;
        A[2] += g * wl.z + hl * dz;
        Bv[0] += gl * wk.x + hk * dx;
        Bv[1] += gl * wk.y + hk * dy;
        Bv[2] += gl * wk.z + hk * dz;
        gm -= g * dwl;
    }
}

// Offsets in units of 1 / sigma (see BoxDev): g and h come out as
// sigma^-3 g and sigma^-5 h, d as sigma d, so A and B carry a factor
// sigma^-3 and gm sigma^-2, which the caller takes back out.
__device__ __forceinline__ void adj_pair_f32(const float4 q, const float4 wl, float px, float py,
                                             float pz, float4 wk, float rc2, float alpha,
                                             float* A, float* Bv, float& gm) {
    const float dx = q.x - px, dy = q.y - py, dz = q.z - pz;
    const float r2 = fmaf(dz, dz, fmaf(dy, dy, dx * dx));
    const bool ok = (r2 > 0.f) & (r2 < rc2);
    const float r2s = ok ? r2 : 1.f;
    const float idr = rsqrtf(r2s);
    const float x = r2s * idr * alpha;
    const float ex = expf(-x * x);
    const float T = erfcf(x) + kTwoOverSqrtPiF * x * ex;
    const float idr2 = idr * idr;
    const float g = ok ? T * idr * idr2 : 0.f;
    const float h = ok ? -(3.f * T + kFourOverSqrtPiF * x * x * x * ex) * idr2 * idr2 * idr : 0.f;
    const float dwl = dx * wl.x + dy * wl.y + dz * wl.z;
    const float dwk = dx * wk.x + dy * wk.y + dz * wk.z;
    const float hl = h * dwl, hk = q.w * h * dwk, gl = q.w * g;
    A[0] += g * wl.x + hl * dx;
    A[1] += g * wl.y + hl * dy;
    A[2] += g * wl.z + hl * dz;
    Bv[0] += gl * wk.x + hk * dx;
    Bv[1] += gl * wk.y + hk * dy;
    Bv[2] += gl * wk.z + hk * dz;
    gm -= g * dwl;
}

// Float32 r^2 tables (host builder in abi.cpp): g and h as quadratics in
// s = r'^2 on segments indexed by the float bits of s, in the units of the
// forward r^2 form (r_cut^2 = 2^kR2Emax), for s >= 2^kAdjEmin (the floor
// keeps h's quadratic coefficient, which grows as s^(-9/2), a finite
// float).  A pair closer than that (r < 2^-18.5 r_cut, rare) takes g and h
// from erfcf / expf instead, at s no smaller than `tiny` = 2^kR2Emin, the
// forward's floor (float32 offsets resolve no closer pairs).  Coincident
// pairs (d = 0, the particle itself included) are left out as in the
// exact form.  Only lanes inside the cutoff read the six coefficients from
// LDS.
__device__ __forceinline__ void adj_pair_f32_r2(const float4 q, const float4 wl, float px,
                                                float py, float pz, float4 wk, float smax,
                                                float smin, uint32_t boff, float alpha, float tiny,
                                                const unsigned char* __restrict__ tab, float* A,
                                                float* Bv, float& gm) {
    const float dx = q.x - px, dy = q.y - py, dz = q.z - pz;
    const float r2 = fmaf(dz, dz, fmaf(dy, dy, dx * dx));
    if ((r2 > 0.f) & (r2 < smax)) {
        float g, h;
        if (r2 >= smin) {
            const uint32_t sb = __float_as_uint(r2);
            // (g c0, g c1), (h c0, h c1), (g c2, h c2) pairs of the row
            const unsigned char* c = tab + (((sb >> (23 - kAdjBits)) << 3) + boff);
            const float2 g01 = *reinterpret_cast<const float2*>(c);
            const float2 h01 = *reinterpret_cast<const float2*>(c + 8 * kAdjPlane);
            const float2 c2 = *reinterpret_cast<const float2*>(c + 16 * kAdjPlane);
            g = fmaf(fmaf(c2.x, r2, g01.y), r2, g01.x);
            h = fmaf(fmaf(c2.y, r2, h01.y), r2, h01.x);
        } else {
            const float rr = fmaxf(r2, tiny);
            const float idr = rsqrtf(rr);
            const float x = rr * idr * alpha;
            const float ex = expf(-x * x);
            const float T = erfcf(x) + kTwoOverSqrtPiF * x * ex;
            const float idr2 = idr * idr;
            g = T * idr * idr2;
            h = -(3.f * T + kFourOverSqrtPiF * x * x * x * ex) * idr2 * idr2 * idr;
        }
        const float dwl = dx * wl.x + dy * wl.y + dz * wl.z;
        const float dwk = dx * wk.x + dy * wk.y + dz * wk.z;
        const float hl = h * dwl, hk = q.w * h * dwk, gl = q.w * g;
        A[0] += g * wl.x + hl * dx;
        A[1] += g * wl.y + hl * dy;
        A[2] += g * wl.z + hl * dz;
        Bv[0] += gl * wk.x + hk * dx;
        Bv[1] += gl * wk.y + hk * dy;
        Bv[2] += gl * wk.z + hk * dz;
        gm -= g * dwl;
    }
}

// F32: float32 offsets; TAB (float32 only): g and h from the r^2 tables,
// staged in LDS (6 kAdjPlane floats), instead of erfc and exp.
template <bool F32, bool TAB>
__global__ void __launch_bounds__(adjoint_max_threads(F32 ? kFP32Exact : kFP64Exact))
adjoint_kernel(const double4* __restrict__ x64, const float4* __restrict__ x32,
               const double4* __restrict__ w64, const float4* __restrict__ w32,
               const int4* __restrict__ leaf, const double4* __restrict__ leafc,
               const int32_t* __restrict__ p2p_js, const int4* __restrict__ items,
               const int32_t* __restrict__ queue, int32_t n_items, int32_t* __restrict__ counter,
               double* __restrict__ partial, const BoxDev* __restrict__ boxes,
               const float* __restrict__ table) {
    extern __shared__ __align__(16) unsigned char adj_lds[];
    if constexpr (TAB) {
        const uint4* src = reinterpret_cast<const uint4*>(table);
        uint4* dst = reinterpret_cast<uint4*>(adj_lds);
        for (int i = threadIdx.x; i < 6 * kAdjPlane / 4; i += blockDim.x) dst[i] = src[i];
        __syncthreads();
    }
    const int lane = threadIdx.x & 63;
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
        const int pk = uni(li.x) + (lane < ni ? lane : 0);
        const BoxDev bx = boxes[uni(li.z)];
        double A[3] = {0.0, 0.0, 0.0}, Bv[3] = {0.0, 0.0, 0.0}, gm = 0.0;
        double mk;
        if constexpr (F32) {
            const float4 pv = x32[pk];
            const float4 wk = w32[pk];
            mk = x64[pk].w;
            const double4 ci = leafc[il];
            float3 lo = make_float3(pv.x, pv.y, pv.z), hi = lo;
            wave_box(lo, hi);
            for (int t = t0; t < t1; ++t) {
                const int js = uni(p2p_js[t]);
                const int jl = js >> 5, s = js & 31;
                const int4 lj = leaf[jl];
                const double4 cj = leafc[jl];
                const double sx = (double)(s % 3 - 1) * bx.L, sy = (double)((s / 3) % 3 - 1) * bx.L,
                             sz = (double)(s / 9 - 1) * bx.L;
                const float offx = (float)(((cj.x - ci.x) + sx) * bx.sigma);
                const float offy = (float)(((cj.y - ci.y) + sy) * bx.sigma);
                const float offz = (float)(((cj.z - ci.z) + sz) * bx.sigma);
                const float px = pv.x - offx, py = pv.y - offy, pz = pv.z - offz;
                const float4* __restrict__ src = x32 + uni(lj.x);
                const float4* __restrict__ wsrc = w32 + uni(lj.x);
                const int nj = uni(lj.y);
                float a[3] = {0.f, 0.f, 0.f}, b[3] = {0.f, 0.f, 0.f}, g = 0.f;
                const uint64_t live =
                    live_f32(src, nj, lane, make_float3(lo.x - offx, lo.y - offy, lo.z - offz),
                             make_float3(hi.x - offx, hi.y - offy, hi.z - offz), bx.rc2_f);
                if constexpr (TAB) {
                    // boff = -(row of 2^kAdjEmin) * 8 mod 2^32, kept opaque (an
                    // empty asm on its scalar register) so that the address is one
                    // shift and one shift-add and the three reads take their
                    // plane offsets as immediates
                    uint32_t boff = 0u - (((uint32_t)(127 + kAdjEmin) << kAdjBits) << 3);
                    asm volatile("" : "+s"(boff));
                    const float smin = __uint_as_float((uint32_t)(127 + kAdjEmin) << 23);
                    for (int k = 0; k < nj; ++k)
                        if ((live >> k) & 1u)
                            adj_pair_f32_r2(src[k], wsrc[k], px, py, pz, wk, bx.rc2_f, smin, boff,
                                            bx.alpha_f, bx.tiny_f, adj_lds, a, b, g);
                } else {
                    for (int k = 0; k < nj; ++k)
                        if ((live >> k) & 1u)
                            adj_pair_f32(src[k], wsrc[k], px, py, pz, wk, bx.rc2_f, bx.alpha_f, a,
                                         b, g);
                }
                for (int c = 0; c < 3; ++c) {
                    A[c] += (double)a[c];
                    Bv[c] += (double)b[c];
                }
                gm += (double)g;
            }
            const double s2 = bx.sigma * bx.sigma, s3 = s2 * bx.sigma;
            for (int c = 0; c < 3; ++c) {
                A[c] *= s3;
                Bv[c] *= s3;
            }
            gm *= s2;
        } else {
            const double4 pv = x64[pk];
            const double4 wk = w64[pk];
            mk = pv.w;
            double3 lo = make_double3(pv.x, pv.y, pv.z), hi = lo;
            wave_box(lo, hi);
            for (int t = t0; t < t1; ++t) {
                const int js = uni(p2p_js[t]);
                const int jl = js >> 5, s = js & 31;
                const int4 lj = leaf[jl];
                const double sx = (double)(s % 3 - 1) * bx.L, sy = (double)((s / 3) % 3 - 1) * bx.L,
                             sz = (double)(s / 9 - 1) * bx.L;
                const double4* __restrict__ src = x64 + uni(lj.x);
                const double4* __restrict__ wsrc = w64 + uni(lj.x);
                const int nj = uni(lj.y);
                const uint64_t live =
                    s == 13 ? live_f64<false>(src, nj, lane, lo, hi, 0.0, 0.0, 0.0, bx.rc2)
                            : live_f64<true>(src, nj, lane, lo, hi, sx, sy, sz, bx.rc2);
                if (s == 13) {
                    for (int k = 0; k < nj; ++k)
                        if ((live >> k) & 1u)
                            adj_pair_f64<false>(src[k], wsrc[k], pv.x, pv.y, pv.z, wk, 0.0, 0.0,
                                                0.0, bx.rc2, bx.alpha, A, Bv, gm);
                } else {
                    for (int k = 0; k < nj; ++k)
                        if ((live >> k) & 1u)
                            adj_pair_f64<true>(src[k], wsrc[k], pv.x, pv.y, pv.z, wk, sx, sy, sz,
                                               bx.rc2, bx.alpha, A, Bv, gm);
                }
            }
        }
        double* dst = partial + (size_t)slot * 256;
        dst[lane] = mk * A[0] - Bv[0];
        dst[64 + lane] = mk * A[1] - Bv[1];
        dst[128 + lane] = mk * A[2] - Bv[2];
        dst[192 + lane] = gm;
    }
}

__global__ void __launch_bounds__(256)
adj_reduce_kernel(const int4* __restrict__ leaf, const int32_t* __restrict__ leaf_slot,
                  const double* __restrict__ partial, const double4* __restrict__ far,
                  const int32_t* __restrict__ perm,
                  const BoxDev* __restrict__ boxes, double* __restrict__ gpos,
                  double* __restrict__ gmass, int32_t n_leaves) {
    const int l = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (l >= n_leaves) return;
    const int4 li = leaf[l];
    if (lane >= li.y) return;
    double g[4] = {0.0, 0.0, 0.0, 0.0};
    for (int s = leaf_slot[l]; s < leaf_slot[l + 1]; ++s) {
        const double* p = partial + (size_t)s * 256;
        for (int c = 0; c < 4; ++c) g[c] += p[64 * c + lane];
    }
    if (far != nullptr) {
        const double4 f = far[li.x + lane];
        g[0] += f.x;
        g[1] += f.y;
        g[2] += f.z;
        g[3] += f.w;
    }
    const double G = boxes[li.z].G;
    const int o = perm[li.x + lane];
    gpos[3 * (size_t)o] = G * g[0];
    gpos[3 * (size_t)o + 1] = G * g[1];
    gpos[3 * (size_t)o + 2] = G * g[2];
    gmass[o] = G * g[3];
}

// w (caller order) -> leaf order, float64 and float32 records.
__global__ void gather_w_kernel(const double* __restrict__ w, const int32_t* __restrict__ perm,
                                double4* __restrict__ w64, float4* __restrict__ w32, int32_t n) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    const int o = perm[k];
    const double x = w[3 * (size_t)o], y = w[3 * (size_t)o + 1], z = w[3 * (size_t)o + 2];
    w64[k] = make_double4(x, y, z, 0.0);
    w32[k] = make_float4((float)x, (float)y, (float)z, 0.f);
}

template <bool F32, bool TAB>
int occ_adj(int wg_waves) {
    int blocks = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, adjoint_kernel<F32, TAB>, 64 * wg_waves,
                                                     TAB ? kAdjTableBytes : 0) != hipSuccess)
        return 1;
    return blocks > 0 ? blocks : 1;
}

}  // namespace

hipError_t launch_gather_w(const double* w, const int32_t* perm, double4* w64, float4* w32,
                           int32_t n, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(gather_w_kernel, dim3((n + 255) / 256), dim3(256), 0, s, w, perm, w64, w32,
                       n);
    return hipGetLastError();
}

hipError_t launch_adjoint(int mode, const AdjArgs& a, int wg_waves, int grid_wgs, hipStream_t s) {
    if (a.n_items == 0) return hipSuccess;
    const dim3 grid(grid_wgs), block(64 * wg_waves);
    const float* tab = static_cast<const float*>(a.table);
    if (is_fp32(mode) && tab != nullptr)
        hipLaunchKernelGGL((adjoint_kernel<true, true>), grid, block, kAdjTableBytes, s, a.x64, a.x32,
                           a.w64, a.w32, a.leaf, a.leafc, a.p2p_js, a.items, a.queue, a.n_items,
                           a.counter, a.partial, a.boxes, tab);
    else if (is_fp32(mode))
        hipLaunchKernelGGL((adjoint_kernel<true, false>), grid, block, 0, s, a.x64, a.x32, a.w64,
                           a.w32, a.leaf, a.leafc, a.p2p_js, a.items, a.queue, a.n_items,
                           a.counter, a.partial, a.boxes, nullptr);
    else
        hipLaunchKernelGGL((adjoint_kernel<false, false>), grid, block, 0, s, a.x64, a.x32, a.w64,
                           a.w32, a.leaf, a.leafc, a.p2p_js, a.items, a.queue, a.n_items,
                           a.counter, a.partial, a.boxes, nullptr);
    return hipGetLastError();
}

hipError_t launch_adj_reduce(const AdjReduceArgs& a, hipStream_t s) {
    if (a.n_leaves == 0) return hipSuccess;
    hipLaunchKernelGGL(adj_reduce_kernel, dim3((a.n_leaves + 3) / 4), dim3(256), 0, s, a.leaf,
                       a.leaf_slot, a.partial, a.far, a.perm, a.boxes, a.grad_pos, a.grad_mass,
                       a.n_leaves);
    return hipGetLastError();
}

int adjoint_blocks_per_cu(int mode, int wg_waves, bool table) {
    if (!is_fp32(mode)) return occ_adj<false, false>(wg_waves);
    return table ? occ_adj<true, true>(wg_waves) : occ_adj<true, false>(wg_waves);
}

}  // namespace pmfmm
