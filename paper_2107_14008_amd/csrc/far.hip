// Truncated far field of the short-range tree (Sec. 2): P2M, M2M (pass-up),
// M2L over the M2L task list, L2L (pass-down) and L2P, in float64.
//
// Expansion (centres z = cell AABB centres; R = z_B - (z_A + s L)):
//   M_m(z_A) = sum_j m_j (z_A - y_j)^m / m!
//   M_m(z_P) = sum_{k <= m} M_k(z_C) (z_P - z_C)^(m-k) / (m-k)!
//   L_n(z_B) = sum_{|m| <= p-|n|} M_m(z_A) D_{n+m}(R)      (Sec. 2, M2L equation)
//   L_n(z_c) = sum_{k >= n} L_k(z_P) (z_c - z_P)^(k-n) / (k-n)!
//   a(x)     = grad_u sum_n L_n u^n / n!,  u = x - z_B   (G applied later)
// D_k = d^k psi for psi = erfc(r / 2 r_s) / r, as the full Cartesian tensor
// of a radial function (the truncated kernel is not harmonic, so the
// traceless shortcut of the plain 1/r kernel does not apply):
//   D_k = sum_{2m <= k} prod_a k_a! / (2^m_a m_a! (k_a - 2 m_a)!) R_a^(k_a - 2 m_a) f_(|k|-|m|)(r)
// with f_(j) = ((1/r) d/dr)^j psi obtained by the upward recursion
//   B_0 = erfc(a r) / r,  B_j = ((2j - 1) B_(j-1) + (2 a^2)^j exp(-a^2 r^2) / (a sqrt(pi))) / r^2,
//   f_(j) = (-1)^j B_j,  a = 1 / (2 r_s),
// which adds only positive terms (stable at small r / r_s).
//
// Mapping: one wavefront per cell (or per leaf); lanes own coefficients
// (P2M, M2M, M2L, L2L) or particles (L2P).  These operators are a small
// share of the step (the paper measures P2P as the dominant cost, Sec. 3);
// they run as plain vector-ALU kernels, one launch per tree level for the
// pass-up and pass-down.
#include "device.h"

namespace pmfmm {
namespace {

constexpr int kMaxP = 6;
constexpr int kMaxNC = 84;

struct MITable {
    signed char a[kMaxNC], b[kMaxNC], c[kMaxNC];
    short idx[kMaxP + 1][kMaxP + 1][kMaxP + 1];
};

constexpr MITable make_mi() {
    MITable t{};
    int k = 0;
    for (int deg = 0; deg <= kMaxP; ++deg)
        for (int a = deg; a >= 0; --a)
            for (int b = deg - a; b >= 0; --b) {
                const int c = deg - a - b;
                t.a[k] = (signed char)a;
                t.b[k] = (signed char)b;
                t.c[k] = (signed char)c;
                t.idx[a][b][c] = (short)k;
                ++k;
            }
    return t;
}

__constant__ MITable c_mi = make_mi();
__constant__ double c_fact[kMaxP + 1] = {1.0, 1.0, 2.0, 6.0, 24.0, 120.0, 720.0};
__constant__ double c_ifact[kMaxP + 1] = {1.0, 1.0, 0.5, 1.0 / 6.0, 1.0 / 24.0, 1.0 / 120.0,
                                          1.0 / 720.0};

constexpr double kInvSqrtPi = 0.56418958354775628695;

__device__ __forceinline__ double ipow(double x, int n) {
    double r = 1.0;
    for (int i = 0; i < n; ++i) r *= x;
    return r;
}

__device__ __forceinline__ int ncoef_of(int p) { return (p + 1) * (p + 2) * (p + 3) / 6; }

// Radial derivatives f_(0..p) of the truncated kernel at distance r.
__device__ void radial_f(double r, double alpha, int p, double* f) {
    const double r2 = r * r;
    const double g = exp(-alpha * alpha * r2) / (alpha) * kInvSqrtPi;
    double B = erfc(alpha * r) / r;
    double two_a2_pow = 1.0;
    f[0] = B;
    for (int j = 1; j <= p; ++j) {
        two_a2_pow *= 2.0 * alpha * alpha;
        B = ((2.0 * j - 1.0) * B + two_a2_pow * g) / r2;
        f[j] = (j & 1) ? -B : B;
    }
}

__device__ double d_entry(int a, int b, int c, const double R[3], const double* f) {
    double sum = 0.0;
    for (int ma = 0; 2 * ma <= a; ++ma) {
        const double ca = c_fact[a] / (ipow(2.0, ma) * c_fact[ma] * c_fact[a - 2 * ma]);
        const double pa = ipow(R[0], a - 2 * ma);
        for (int mb = 0; 2 * mb <= b; ++mb) {
            const double cb = c_fact[b] / (ipow(2.0, mb) * c_fact[mb] * c_fact[b - 2 * mb]);
            const double pb = ipow(R[1], b - 2 * mb);
            for (int mc = 0; 2 * mc <= c; ++mc) {
                const double cc = c_fact[c] / (ipow(2.0, mc) * c_fact[mc] * c_fact[c - 2 * mc]);
                const double pc = ipow(R[2], c - 2 * mc);
                sum += ca * cb * cc * pa * pb * pc * f[a + b + c - ma - mb - mc];
            }
        }
    }
    return sum;
}

// ---- P2M: one wavefront per leaf, lanes own coefficients.
__global__ void __launch_bounds__(256)
p2m_kernel(const double4* __restrict__ x64, const int4* __restrict__ leaf,
           const double4* __restrict__ cellc, const BoxDev* __restrict__ boxes,
           const int32_t* __restrict__ needM, double* __restrict__ M, int n_leaves, int ncoef) {
    // four leaves per workgroup, one wavefront each: most leaves need no
    // multipole and their wavefront returns at once
    const int l = blockIdx.x * 4 + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (l >= n_leaves) return;
    const int4 li = leaf[l];
    if (!needM[li.w]) return;
    const int p = boxes[li.z].order;
    if (p < 0) return;
    const int nc = ncoef_of(p);
    const double4 c = cellc[li.w];
    for (int k = lane; k < nc; k += 64) {
        const int a = c_mi.a[k], b = c_mi.b[k], cc = c_mi.c[k];
        const double inv = c_ifact[a] * c_ifact[b] * c_ifact[cc];
        double acc = 0.0;
        for (int j = 0; j < li.y; ++j) {
            const double4 q = x64[li.x + j];
            acc += q.w * ipow(c.x - q.x, a) * ipow(c.y - q.y, b) * ipow(c.z - q.z, cc);
        }
        M[(size_t)li.w * ncoef + k] = acc * inv;
    }
}

// ---- M2M for the internal cells of one depth.
__global__ void __launch_bounds__(64)
m2m_kernel(const int32_t* __restrict__ level_cells, int n_level, const int4* __restrict__ cell,
           const int4* __restrict__ aux, const double4* __restrict__ cellc,
           const BoxDev* __restrict__ boxes, const int32_t* __restrict__ needM,
           double* __restrict__ M, int ncoef) {
    if ((int)blockIdx.x >= n_level) return;
    const int P = level_cells[blockIdx.x];
    if (cell[P].w >= 0 || !needM[P]) return;          // leaf: P2M already did it
    const int4 ax = aux[P];
    const int p = boxes[ax.z].order;
    if (p < 0) return;
    const int nc = ncoef_of(p);
    const double4 cp = cellc[P];
    for (int m = threadIdx.x; m < nc; m += 64) {
        const int m0 = c_mi.a[m], m1 = c_mi.b[m], m2 = c_mi.c[m];
        double acc = 0.0;
        for (int ch = 0; ch < 2; ++ch) {
            const int C = ch == 0 ? ax.x : ax.y;
            const double4 cc = cellc[C];
            const double dz[3] = {cp.x - cc.x, cp.y - cc.y, cp.z - cc.z};
            const double* MC = M + (size_t)C * ncoef;
            for (int k0 = 0; k0 <= m0; ++k0)
                for (int k1 = 0; k1 <= m1; ++k1)
                    for (int k2 = 0; k2 <= m2; ++k2) {
                        const double w = ipow(dz[0], m0 - k0) * c_ifact[m0 - k0] *
                                         ipow(dz[1], m1 - k1) * c_ifact[m1 - k1] *
                                         ipow(dz[2], m2 - k2) * c_ifact[m2 - k2];
                        acc += MC[c_mi.idx[k0][k1][k2]] * w;
                    }
        }
        M[(size_t)P * ncoef + m] = acc;
    }
}

// ---- M2L: one wavefront per task (t, u, s) of the M2L list; the D tensor
// of the task is built in LDS by the lanes, lane n then computes the task's
// contribution to L_n(z_t) into its own row of Lt (no ordering between
// tasks is needed); m2l_sum_kernel adds each target's rows in list order.
__global__ void __launch_bounds__(64)
m2l_task_kernel(const int32_t* __restrict__ row, const int32_t* __restrict__ src,
                const int32_t* __restrict__ shift, const int4* __restrict__ aux,
                const double4* __restrict__ cellc, const BoxDev* __restrict__ boxes,
                const double* __restrict__ M, double* __restrict__ Lt, int n_cells, int ncoef) {
    __shared__ double Dsh[kMaxNC];
    const int q = blockIdx.x;
    const int lane = threadIdx.x;
    // target cell of task q: the row holding it
    int lo = 0, hi = n_cells - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (row[mid] <= q) lo = mid; else hi = mid - 1;
    }
    const int t = lo;
    const BoxDev bx = boxes[aux[t].z];
    const int p = bx.order;
    const int nc = ncoef_of(p);
    const double4 ct = cellc[t];
    const int u = src[q];
    const int s = shift[q];
    const double4 cu = cellc[u];
    const double R[3] = {ct.x - (cu.x + (double)(s % 3 - 1) * bx.L),
                         ct.y - (cu.y + (double)((s / 3) % 3 - 1) * bx.L),
                         ct.z - (cu.z + (double)(s / 9 - 1) * bx.L)};
    const double r = sqrt(R[0] * R[0] + R[1] * R[1] + R[2] * R[2]);
    double f[kMaxP + 1];
    radial_f(r, bx.alpha, p, f);
    for (int k = lane; k < nc; k += 64) Dsh[k] = d_entry(c_mi.a[k], c_mi.b[k], c_mi.c[k], R, f);
    __syncthreads();
    const double* Mu = M + (size_t)u * ncoef;
    double* out = Lt + (size_t)q * ncoef;
    for (int n = lane; n < ncoef; n += 64) {
        double acc = 0.0;
        if (n < nc) {
            const int n0 = c_mi.a[n], n1 = c_mi.b[n], n2 = c_mi.c[n];
            const int mend = ncoef_of(p - (n0 + n1 + n2));
            for (int m = 0; m < mend; ++m)
                acc += Mu[m] * Dsh[c_mi.idx[n0 + c_mi.a[m]][n1 + c_mi.b[m]][n2 + c_mi.c[m]]];
        }
        out[n] = acc;
    }
}

// L of every cell that needs one: the sum of its tasks' rows in list order
// (zero without tasks).
__global__ void __launch_bounds__(64)
m2l_sum_kernel(const int32_t* __restrict__ row, const int32_t* __restrict__ needL,
               const double* __restrict__ Lt, double* __restrict__ Lc, int n_cells, int ncoef) {
    const int t = blockIdx.x;
    if (t >= n_cells || !needL[t]) return;
    const int r0 = row[t], r1 = row[t + 1];
    for (int n = threadIdx.x; n < ncoef; n += 64) {
        double acc = 0.0;
        for (int q = r0; q < r1; ++q) acc += Lt[(size_t)q * ncoef + n];
        Lc[(size_t)t * ncoef + n] = acc;
    }
}

// ---- L2L for the cells of one depth (>= 1): add the parent's shifted local.
__global__ void __launch_bounds__(64)
l2l_kernel(const int32_t* __restrict__ level_cells, int n_level, const int4* __restrict__ cell,
           const int4* __restrict__ aux, const double4* __restrict__ cellc,
           const BoxDev* __restrict__ boxes, const int32_t* __restrict__ needL,
           double* __restrict__ Lc, int ncoef) {
    if ((int)blockIdx.x >= n_level) return;
    const int C = level_cells[blockIdx.x];
    const int P = cell[C].z;
    if (P < 0 || !needL[C] || !needL[P]) return;
    const int p = boxes[aux[C].z].order;
    if (p < 0) return;
    const int nc = ncoef_of(p);
    const double4 cc = cellc[C], cp = cellc[P];
    const double dz[3] = {cc.x - cp.x, cc.y - cp.y, cc.z - cp.z};
    const double* LP = Lc + (size_t)P * ncoef;
    for (int n = threadIdx.x; n < nc; n += 64) {
        const int n0 = c_mi.a[n], n1 = c_mi.b[n], n2 = c_mi.c[n];
        const int deg = n0 + n1 + n2;
        double acc = 0.0;
        for (int k0 = n0; k0 <= p; ++k0)
            for (int k1 = n1; k0 + k1 <= p; ++k1)
                for (int k2 = n2; k0 + k1 + k2 <= p; ++k2) {
                    const double w = ipow(dz[0], k0 - n0) * c_ifact[k0 - n0] *
                                     ipow(dz[1], k1 - n1) * c_ifact[k1 - n1] *
                                     ipow(dz[2], k2 - n2) * c_ifact[k2 - n2];
                    acc += LP[c_mi.idx[k0][k1][k2]] * w;
                }
        (void)deg;
        Lc[(size_t)C * ncoef + n] += acc;
    }
}

// ---- L2P: one wavefront per leaf (four per workgroup), lane = particle.
// Only leaves with a local expansion are written; the reduction reads the
// far part of exactly those (the same needL flag).
__global__ void __launch_bounds__(256)
l2p_kernel(const double4* __restrict__ x64, const int4* __restrict__ leaf,
           const double4* __restrict__ cellc, const BoxDev* __restrict__ boxes,
           const int32_t* __restrict__ needL, const double* __restrict__ Lc,
           double* __restrict__ far, int n_leaves, int ncoef) {
    const int l = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (l >= n_leaves) return;
    const int4 li = leaf[l];
    const int lane = threadIdx.x & 63;
    if (lane >= li.y) return;
    const int k = li.x + lane;
    const int p = boxes[li.z].order;
    if (p < 0 || !needL[li.w]) return;
    double ax = 0.0, ay = 0.0, az = 0.0;
    {
        const int nc = ncoef_of(p);
        const double4 c = cellc[li.w];
        const double4 q = x64[k];
        const double u[3] = {q.x - c.x, q.y - c.y, q.z - c.z};
        double pw[3][kMaxP + 1];
        for (int a = 0; a < 3; ++a) {
            pw[a][0] = 1.0;
            for (int i = 1; i <= kMaxP; ++i) pw[a][i] = pw[a][i - 1] * u[a] / (double)i;
        }
        const double* L = Lc + (size_t)li.w * ncoef;
        for (int n = 1; n < nc; ++n) {
            const int n0 = c_mi.a[n], n1 = c_mi.b[n], n2 = c_mi.c[n];
            const double Ln = L[n];
            if (n0 > 0) ax += Ln * pw[0][n0 - 1] * pw[1][n1] * pw[2][n2];
            if (n1 > 0) ay += Ln * pw[0][n0] * pw[1][n1 - 1] * pw[2][n2];
            if (n2 > 0) az += Ln * pw[0][n0] * pw[1][n1] * pw[2][n2 - 1];
        }
    }
    far[3 * (size_t)k] = ax;
    far[3 * (size_t)k + 1] = ay;
    far[3 * (size_t)k + 2] = az;
}

// ---- Adjoint of the far field (not in the paper).  For L = sum_i w_i . a_i
// with the tree, the lists and the centres fixed, the transposed operators
// become the forward ones on sign-flipped coefficients: with
// Lt_n = (-1)^|n| dL/dL_n and Mt_m = (-1)^|m| dL/dM_m, the transpose of
// L2L is M2M on Lt, that of M2L is M2L on Lt (the M2L list is symmetric:
// (t, u, s) holds with (u, t, 26 - s), and D_k(-R) = (-1)^|k| D_k(R)), and
// that of M2M is L2L on Mt.  At the leaves (no G):
//   Lt_n(B) = -sum_{i in B} sum_a w_ia (z_B - x_i)^(n - e_a) / (n - e_a)!   (from L2P)
//   dL/dx_k = Hess phi_B(u) w_k + m_k grad psi_B(u),  dL/dm_k = psi_B(u)
// with u = x_k - z_B, phi_B the forward local polynomial and
// psi_B(u) = sum_m Mt_m(B) u^m / m! (from P2M).

// Lt of every leaf that needs one (into M, the pass-up's input).
__global__ void __launch_bounds__(64)
w2m_kernel(const double4* __restrict__ x64, const double4* __restrict__ w64,
           const int4* __restrict__ leaf, const double4* __restrict__ cellc,
           const BoxDev* __restrict__ boxes, const int32_t* __restrict__ needM,
           double* __restrict__ M, int n_leaves, int ncoef) {
    const int l = blockIdx.x;
    if (l >= n_leaves) return;
    const int4 li = leaf[l];
    if (!needM[li.w]) return;
    const int p = boxes[li.z].order;
    if (p < 0) return;
    const int nc = ncoef_of(p);
    const double4 c = cellc[li.w];
    for (int k = threadIdx.x; k < nc; k += 64) {
        const int e[3] = {c_mi.a[k], c_mi.b[k], c_mi.c[k]};
        double acc = 0.0;
        for (int j = 0; j < li.y; ++j) {
            const double4 q = x64[li.x + j];
            const double4 wq = w64[li.x + j];
            const double v[3] = {c.x - q.x, c.y - q.y, c.z - q.z};
            const double wa[3] = {wq.x, wq.y, wq.z};
            for (int a = 0; a < 3; ++a) {
                if (e[a] == 0) continue;
                double t = wa[a];
                for (int b = 0; b < 3; ++b) {
                    const int eb = e[b] - (a == b ? 1 : 0);
                    t *= ipow(v[b], eb) * c_ifact[eb];
                }
                acc -= t;
            }
        }
        M[(size_t)li.w * ncoef + k] = acc;
    }
}

// u_a^i / i! for i <= p.
__device__ __forceinline__ void scaled_powers(const double u[3], double pw[3][kMaxP + 1]) {
    for (int a = 0; a < 3; ++a) {
        pw[a][0] = 1.0;
        for (int i = 1; i <= kMaxP; ++i) pw[a][i] = pw[a][i - 1] * u[a] / (double)i;
    }
}

// The L2P term Hess phi_B(u) w_k from the forward locals, one wavefront per
// leaf, lane = particle: fg[k] = (gx, gy, gz, 0).
__global__ void __launch_bounds__(64)
far_hess_kernel(const double4* __restrict__ x64, const double4* __restrict__ w64,
                const int4* __restrict__ leaf, const double4* __restrict__ cellc,
                const BoxDev* __restrict__ boxes, const int32_t* __restrict__ needL,
                const double* __restrict__ Lc, double4* __restrict__ fg, int n_leaves,
                int ncoef) {
    const int l = blockIdx.x;
    if (l >= n_leaves) return;
    const int4 li = leaf[l];
    const int lane = threadIdx.x;
    if (lane >= li.y) return;
    const int k = li.x + lane;
    const int p = boxes[li.z].order;
    double g[3] = {0.0, 0.0, 0.0};
    if (p >= 0 && needL[li.w]) {
        const int nc = ncoef_of(p);
        const double4 c = cellc[li.w];
        const double4 q = x64[k];
        const double4 wq = w64[k];
        const double u[3] = {q.x - c.x, q.y - c.y, q.z - c.z};
        const double w[3] = {wq.x, wq.y, wq.z};
        double pw[3][kMaxP + 1];
        scaled_powers(u, pw);
        const double* L = Lc + (size_t)li.w * ncoef;
        for (int n = 4; n < nc; ++n) {
            const int e[3] = {c_mi.a[n], c_mi.b[n], c_mi.c[n]};
            const double Ln = L[n];
            for (int a = 0; a < 3; ++a) {
                if (e[a] == 0) continue;
                for (int b = 0; b < 3; ++b) {
                    const int f0 = e[0] - (a == 0) - (b == 0), f1 = e[1] - (a == 1) - (b == 1),
                              f2 = e[2] - (a == 2) - (b == 2);
                    if (f0 < 0 || f1 < 0 || f2 < 0) continue;
                    g[a] += Ln * pw[0][f0] * pw[1][f1] * pw[2][f2] * w[b];
                }
            }
        }
    }
    fg[k] = make_double4(g[0], g[1], g[2], 0.0);
}

// The P2M terms from the adjoint locals Mt (in Lc after the adjoint pass):
// fg[k] += (m_k grad psi(u), psi(u)).
__global__ void __launch_bounds__(64)
far_adj_kernel(const double4* __restrict__ x64, const int4* __restrict__ leaf,
               const double4* __restrict__ cellc, const BoxDev* __restrict__ boxes,
               const int32_t* __restrict__ needL, const double* __restrict__ Lc,
               double4* __restrict__ fg, int n_leaves, int ncoef) {
    const int l = blockIdx.x;
    if (l >= n_leaves) return;
    const int4 li = leaf[l];
    const int lane = threadIdx.x;
    if (lane >= li.y) return;
    const int k = li.x + lane;
    const int p = boxes[li.z].order;
    if (p < 0 || !needL[li.w]) return;
    const int nc = ncoef_of(p);
    const double4 c = cellc[li.w];
    const double4 q = x64[k];
    const double u[3] = {q.x - c.x, q.y - c.y, q.z - c.z};
    double pw[3][kMaxP + 1];
    scaled_powers(u, pw);
    const double* Mt = Lc + (size_t)li.w * ncoef;
    double psi = 0.0, gx = 0.0, gy = 0.0, gz = 0.0;
    for (int n = 0; n < nc; ++n) {
        const int n0 = c_mi.a[n], n1 = c_mi.b[n], n2 = c_mi.c[n];
        const double Mn = Mt[n];
        psi += Mn * pw[0][n0] * pw[1][n1] * pw[2][n2];
        if (n0 > 0) gx += Mn * pw[0][n0 - 1] * pw[1][n1] * pw[2][n2];
        if (n1 > 0) gy += Mn * pw[0][n0] * pw[1][n1 - 1] * pw[2][n2];
        if (n2 > 0) gz += Mn * pw[0][n0] * pw[1][n1] * pw[2][n2 - 1];
    }
    double4 o = fg[k];
    o.x += q.w * gx;
    o.y += q.w * gy;
    o.z += q.w * gz;
    o.w = psi;
    fg[k] = o;
}

// Sources and targets of M2L rows.
__global__ void far_mark_kernel(const int32_t* __restrict__ row, const int32_t* __restrict__ src,
                                int n_cells, int32_t* __restrict__ needM,
                                int32_t* __restrict__ needL) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= n_cells) return;
    const int r0 = row[c], r1 = row[c + 1];
    if (r0 == r1) return;
    needL[c] = 1;
    for (int q = r0; q < r1; ++q) needM[src[q]] = 1;
}

// A cell needs an expansion when it or an ancestor was marked.
__global__ void far_spread_kernel(const int4* __restrict__ cell, int n_cells,
                                  const int32_t* __restrict__ markM,
                                  const int32_t* __restrict__ markL, int32_t* __restrict__ needM,
                                  int32_t* __restrict__ needL) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= n_cells) return;
    int m = 0, l = 0;
    for (int a = c; a >= 0; a = cell[a].z) {
        m |= markM[a];
        l |= markL[a];
    }
    needM[c] = m;
    needL[c] = l;
}

__global__ void zero_i32_n(int32_t* p, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0;
}

__global__ void zero_f64_kernel(double* p, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0.0;
}

}  // namespace

int n_coef(int order) { return order < 0 ? 1 : (order + 1) * (order + 2) * (order + 3) / 6; }

hipError_t launch_zero_f64(double* p, int64_t n, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(zero_f64_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, p, n);
    return hipGetLastError();
}

// needM / needL hold 2 n_cells ints each: marks first, then the spread flags.
hipError_t launch_far_flags(const FarArgs& a, hipStream_t s) {
    const int64_t nc = a.n_cells;
    int32_t* markM = a.needM + nc;
    int32_t* markL = a.needL + nc;
    const unsigned g = (unsigned)((nc + 255) / 256);
    hipLaunchKernelGGL(zero_i32_n, dim3(g), dim3(256), 0, s, markM, nc);
    hipLaunchKernelGGL(zero_i32_n, dim3(g), dim3(256), 0, s, markL, nc);
    hipLaunchKernelGGL(far_mark_kernel, dim3(g), dim3(256), 0, s, a.m2l_row, a.m2l_src, (int)nc, markM,
                       markL);
    hipLaunchKernelGGL(far_spread_kernel, dim3(g), dim3(256), 0, s, a.cell, (int)nc, markM, markL,
                       a.needM, a.needL);
    return hipGetLastError();
}

hipError_t launch_p2m(const FarArgs& a, hipStream_t s) {
    if (a.n_leaves == 0) return hipSuccess;
    hipLaunchKernelGGL(p2m_kernel, dim3((a.n_leaves + 3) / 4), dim3(256), 0, s, a.x64, a.leaf,
                       a.cellc, a.boxes, a.needM, a.M, a.n_leaves, a.ncoef);
    return hipGetLastError();
}

hipError_t launch_m2m_level(const FarArgs& a, hipStream_t s) {
    if (a.n_level == 0) return hipSuccess;
    hipLaunchKernelGGL(m2m_kernel, dim3(a.n_level), dim3(64), 0, s, a.level_cells, a.n_level,
                       a.cell, a.cell_aux, a.cellc, a.boxes, a.needM, a.M, a.ncoef);
    return hipGetLastError();
}

hipError_t launch_m2l(const FarArgs& a, hipStream_t s) {
    if (a.n_cells == 0) return hipSuccess;
    if (a.n_m2l > 0)
        hipLaunchKernelGGL(m2l_task_kernel, dim3(a.n_m2l), dim3(64), 0, s, a.m2l_row, a.m2l_src,
                           a.m2l_shift, a.cell_aux, a.cellc, a.boxes, a.M, a.Lt, a.n_cells,
                           a.ncoef);
    hipLaunchKernelGGL(m2l_sum_kernel, dim3(a.n_cells), dim3(64), 0, s, a.m2l_row, a.needL, a.Lt,
                       a.Lc, a.n_cells, a.ncoef);
    return hipGetLastError();
}

hipError_t launch_l2l_level(const FarArgs& a, hipStream_t s) {
    if (a.n_level == 0) return hipSuccess;
    hipLaunchKernelGGL(l2l_kernel, dim3(a.n_level), dim3(64), 0, s, a.level_cells, a.n_level,
                       a.cell, a.cell_aux, a.cellc, a.boxes, a.needL, a.Lc, a.ncoef);
    return hipGetLastError();
}

hipError_t launch_w2m(const FarArgs& a, const double4* w64, hipStream_t s) {
    if (a.n_leaves == 0) return hipSuccess;
    hipLaunchKernelGGL(w2m_kernel, dim3(a.n_leaves), dim3(64), 0, s, a.x64, w64, a.leaf, a.cellc,
                       a.boxes, a.needM, a.M, a.n_leaves, a.ncoef);
    return hipGetLastError();
}

hipError_t launch_far_hess(const FarArgs& a, const double4* w64, double4* fg, hipStream_t s) {
    if (a.n_leaves == 0) return hipSuccess;
    hipLaunchKernelGGL(far_hess_kernel, dim3(a.n_leaves), dim3(64), 0, s, a.x64, w64, a.leaf,
                       a.cellc, a.boxes, a.needL, a.Lc, fg, a.n_leaves, a.ncoef);
    return hipGetLastError();
}

hipError_t launch_far_adj(const FarArgs& a, double4* fg, hipStream_t s) {
    if (a.n_leaves == 0) return hipSuccess;
    hipLaunchKernelGGL(far_adj_kernel, dim3(a.n_leaves), dim3(64), 0, s, a.x64, a.leaf, a.cellc,
                       a.boxes, a.needL, a.Lc, fg, a.n_leaves, a.ncoef);
    return hipGetLastError();
}

hipError_t launch_l2p(const FarArgs& a, hipStream_t s) {
    if (a.n_leaves == 0) return hipSuccess;
    hipLaunchKernelGGL(l2p_kernel, dim3((a.n_leaves + 3) / 4), dim3(256), 0, s, a.x64, a.leaf,
                       a.cellc, a.boxes, a.needL, a.Lc, a.far, a.n_leaves, a.ncoef);
    return hipGetLastError();
}

}  // namespace pmfmm
