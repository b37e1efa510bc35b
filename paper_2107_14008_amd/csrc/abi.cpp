// C ABI of the short-range PM-FMM library: context, validation, planning,
// device upload, and the enqueueing of the forward and adjoint passes.
#include "pmfmm.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "device.h"
#include "gpu_plan.h"
#include "plan.h"
#include "pm.h"

namespace {

thread_local std::string g_err;

int fail(int code, const std::string& msg) {
    g_err = msg;
    return code;
}

#define HIP_TRY(expr)                                                                 \
    do {                                                                              \
        hipError_t e_ = (expr);                                                       \
        if (e_ != hipSuccess)                                                         \
            return fail(e_ == hipErrorOutOfMemory ? PMFMM_ENOMEM : PMFMM_EDEVICE,     \
                        std::string(#expr) + ": " + hipGetErrorString(e_));           \
    } while (0)

using pmfmm::DevBuf;

bool valid_geometry(const pmfmm_params& p, std::string& why) {
    if (!(std::isfinite(p.box) && p.box > 0.0)) { why = "box must be finite and > 0"; return false; }
    if (!(std::isfinite(p.r_s) && p.r_s > 0.0)) { why = "r_s must be finite and > 0"; return false; }
    if (!(std::isfinite(p.r_cut) && p.r_cut > 0.0 && p.r_cut < 0.5 * p.box)) {
        why = "r_cut must satisfy 0 < r_cut < box / 2";
        return false;
    }
    if (!std::isfinite(p.G)) { why = "G must be finite"; return false; }
    if (!(std::isfinite(p.theta) && p.theta >= 0.0 && p.theta < 1.0)) {
        why = "theta must be in [0, 1)";
        return false;
    }
    if (p.max_leaf < 1 || p.max_leaf > 64) { why = "max_leaf must be in 1..64"; return false; }
    if (p.order > 6) { why = "order must be <= 6 (negative turns the far field off)"; return false; }
    if (p.m2l_cut != PMFMM_M2L_INSIDE && p.m2l_cut != PMFMM_M2L_CENTRE) {
        why = "m2l_cut must be PMFMM_M2L_INSIDE or PMFMM_M2L_CENTRE";
        return false;
    }
    return true;
}

bool valid_eval(const pmfmm_params& p, std::string& why) {
    if (p.precision != PMFMM_FP64 && p.precision != PMFMM_FP32) { why = "precision must be FP64 or FP32"; return false; }
    if (p.trunc != PMFMM_TRUNC_EXACT && p.trunc != PMFMM_TRUNC_TABLE && p.trunc != PMFMM_TRUNC_R2) {
        why = "trunc must be EXACT, TABLE or R2";
        return false;
    }
    if (p.trunc == PMFMM_TRUNC_R2 && p.precision == PMFMM_FP32) {
        if (p.table_level == 2) {
            if (p.table_size != 16 && p.table_size != 32 && p.table_size != 64 && p.table_size != 128) {
                why = "table_size (segments per octave) must be 16, 32, 64 or 128 for the degree-2 R2 table";
                return false;
            }
        } else if (p.table_level == 1) {
            if (p.table_size != 64 && p.table_size != 128 && p.table_size != 256 && p.table_size != 512) {
                why = "table_size (segments per octave) must be 64, 128, 256 or 512 for the degree-1 R2 table";
                return false;
            }
        } else {
            why = "table_level (degree) must be 1 or 2 for R2";
            return false;
        }
    }
    if (p.trunc == PMFMM_TRUNC_R2 && p.precision == PMFMM_FP64) {
        if (p.table_size != 16 && p.table_size != 32 && p.table_size != 64) {
            why = "table_size (segments per octave) must be 16, 32 or 64 for the float64 R2 table";
            return false;
        }
        if (p.table_level < 4 || p.table_level > 6) {
            why = "table_level (degree) must be 4, 5 or 6 for the float64 R2 table";
            return false;
        }
    } else {
        if (p.table_level < 0 || p.table_level > 4) { why = "table_level must be in 0..4"; return false; }
        const int max_tab = p.precision == PMFMM_FP64 ? 2048 : 4096;
        if (p.table_size < 16 || p.table_size > max_tab) {
            why = "table_size must be in 16.." + std::to_string(max_tab);
            return false;
        }
    }
    if (p.table_round != PMFMM_ROUND_NEAREST && p.table_round != PMFMM_ROUND_FLOOR) { why = "table_round must be NEAREST or FLOOR"; return false; }
    if (p.accum != PMFMM_ACCUM_FP64 && p.accum != PMFMM_ACCUM_FP32_TWOSUM) {
        why = "accum must be FP64 or FP32_TWOSUM";
        return false;
    }
    if (p.accum == PMFMM_ACCUM_FP32_TWOSUM && p.precision != PMFMM_FP32) {
        why = "accum FP32_TWOSUM applies to the float32 forms";
        return false;
    }
    if (p.chunk < 0) { why = "chunk must be >= 0"; return false; }
    if (p.wg_waves < 0 || p.wg_waves > 16) { why = "wg_waves must be in 0..16"; return false; }
    if (p.grid_wgs < 0) { why = "grid_wgs must be >= 0"; return false; }
    if (p.threads < 0) { why = "threads must be >= 0"; return false; }
    return true;
}

int mode_of(const pmfmm_params& p) {
    if (p.precision == PMFMM_FP64) {
        if (p.trunc == PMFMM_TRUNC_R2) return pmfmm::kFP64R2;
        return p.trunc == PMFMM_TRUNC_TABLE ? pmfmm::kFP64Table : pmfmm::kFP64Exact;
    }
    if (p.trunc == PMFMM_TRUNC_R2) return pmfmm::kFP32R2;
    return p.trunc == PMFMM_TRUNC_TABLE ? pmfmm::kFP32Table : pmfmm::kFP32Exact;
}

bool uses_r2(const pmfmm_params& p) { return p.precision == PMFMM_FP32 && p.trunc == PMFMM_TRUNC_R2; }
// Either r^2 table: one x_c = r_cut / 2 r_s for all boxes, rebuilt when it changes.
bool r2_table(const pmfmm_params& p) { return p.trunc == PMFMM_TRUNC_R2; }

// x_c = r_cut / 2 r_s, which the r^2 table needs to be one for all boxes
// (up to rounding: r_cut = 4.5 r_s over many r_s gives x_c within an ulp).
bool same_xc(double rc_a, double rs_a, double rc_b, double rs_b) {
    const double a = rc_a / (2.0 * rs_a), b = rc_b / (2.0 * rs_b);
    return std::fabs(a - b) <= 1e-12 * std::fabs(a);
}

bool one_xc(const std::vector<pmfmm::BoxParams>& boxes) {
    for (const auto& b : boxes)
        if (!same_xc(b.r_cut, b.r_s, boxes[0].r_cut, boxes[0].r_s)) return false;
    return true;
}

double truncation_T(double x) {
    return std::erfc(x) + 1.12837916709551257390 * x * std::exp(-x * x);
}

// Fits fn on every segment of the float32 r^2 rows over [2^emin, 2^kR2Emax)
// (2^bits per octave) and stores the coefficients of s^0 .. s^deg in planes:
// f[plane * i + row] holds that of s^i.
template <class Fn>
void fit_r2_rows(int bits, int emin, int deg, Fn fn, float* f, size_t plane) {
    const int per_octave = 1 << bits;
    const int rows = (pmfmm::kR2Emax - emin) << bits;
    const int m = deg + 1;
    for (int k = 0; k < rows; ++k) {
        const int e = emin + (k >> bits), j = k & ((1 << bits) - 1);
        const double lo = std::ldexp(1.0 + (double)j / per_octave, e);
        const double hi = std::ldexp(1.0 + (double)(j + 1) / per_octave, e);
        double V[3][4];
        for (int i = 0; i < m; ++i) {
            const double t = 0.5 - 0.5 * std::cos(M_PI * (i + 0.5) / m);   // in [0, 1]
            const double sv = lo + (hi - lo) * t;
            double tp = 1.0;
            for (int q = 0; q < m; ++q) {
                V[i][q] = tp;
                tp *= sv - lo;
            }
            V[i][m] = fn(sv);
        }
        // Gaussian elimination with partial pivoting on the (m x m) system
        for (int c = 0; c < m; ++c) {
            int piv = c;
            for (int r = c + 1; r < m; ++r)
                if (std::fabs(V[r][c]) > std::fabs(V[piv][c])) piv = r;
            for (int q = 0; q <= m; ++q) std::swap(V[c][q], V[piv][q]);
            for (int r = c + 1; r < m; ++r) {
                const double g = V[r][c] / V[c][c];
                for (int q = c; q <= m; ++q) V[r][q] -= g * V[c][q];
            }
        }
        double cl[3] = {0, 0, 0};
        for (int c = m - 1; c >= 0; --c) {
            double acc = V[c][m];
            for (int q = c + 1; q < m; ++q) acc -= V[c][q] * cl[q];
            cl[c] = acc / V[c][c];
        }
        // p(s) = sum_q cl_q (s - lo)^q = sum_i a_i s^i
        static const double binom[3][3] = {{1, 0, 0}, {1, 1, 0}, {1, 2, 1}};
        for (int i = 0; i < m; ++i) {
            double acc = 0.0;
            for (int q = i; q < m; ++q) acc += cl[q] * binom[q][i] * std::pow(-lo, q - i);
            f[plane * i + k] = (float)acc;
        }
    }
}

// Table of the float32 r^2 form: F(s) = T(x) s^(-3/2), s = r'^2 in units
// where r_cut^2 = 2^kR2Emax (x^2 = s kappa, kappa = x_c^2 / 2^kR2Emax).  Row
// (e - kR2Emin) 2^bits + j covers s in 2^e [1 + j / 2^bits, 1 + (j + 1) / 2^bits);
// on it F is the polynomial of degree `deg` interpolating F at the
// Chebyshev nodes of the segment, re-expanded in s itself (the kernel
// evaluates it at s with no segment offset).  The last row (s = 2^kR2Emax)
// is zero.  Stored as (c0, c1) pairs at 8 k and (c2, 0) at
// r2_plane_c2(bits) + 8 k: a lookup is one 8-byte read and one 4-byte read
// at an immediate offset from the same address (measured 2 % faster than
// three planes of floats read by a two-address and a one-address read, and
// 7 % faster than one 16-byte-per-lane two-address read).
//
// Degree 1: rows of (c0, c1) over [2^kR2EminLin, 2^kR2Emax) after a zero
// row (closer pairs: the kernel's exact pass) and before a zero row at
// s = 2^kR2Emax, r2_rows_lin(bits) in all.
std::vector<unsigned char> build_r2_table(int per_octave, int deg, double xc) {
    int bits = 4;
    while ((1 << bits) < per_octave) ++bits;
    const double kappa = xc * xc / std::ldexp(1.0, pmfmm::kR2Emax);
    if (deg == 1) {
        const int rows = (pmfmm::kR2Emax - pmfmm::kR2EminLin) << bits;
        std::vector<float> pl((size_t)2 * rows, 0.0f);
        fit_r2_rows(bits, pmfmm::kR2EminLin, 1,
                    [&](double sv) { return truncation_T(std::sqrt(sv * kappa)) * std::pow(sv, -1.5); },
                    pl.data(), (size_t)rows);
        std::vector<unsigned char> out((size_t)pmfmm::r2_table_bytes_lin(bits), 0);
        float* a = reinterpret_cast<float*>(out.data());
        for (int k = 0; k < rows; ++k) {
            a[2 * (k + 1)] = pl[k];
            a[2 * (k + 1) + 1] = pl[(size_t)rows + k];
        }
        return out;
    }
    std::vector<float> pl((size_t)3 * pmfmm::kR2Plane, 0.0f);
    fit_r2_rows(bits, pmfmm::kR2Emin, deg,
                [&](double sv) { return truncation_T(std::sqrt(sv * kappa)) * std::pow(sv, -1.5); },
                pl.data(), pmfmm::kR2Plane);
    const int rows = pmfmm::r2_rows(bits);
    std::vector<unsigned char> out((size_t)pmfmm::r2_table_bytes(bits), 0);
    float* a = reinterpret_cast<float*>(out.data());
    float* b = reinterpret_cast<float*>(out.data() + pmfmm::r2_plane_c2(bits));
    for (int k = 0; k < rows; ++k) {
        a[2 * k] = pl[k];
        a[2 * k + 1] = pl[pmfmm::kR2Plane + k];
        b[2 * k] = pl[2 * pmfmm::kR2Plane + k];
    }
    return out;
}

// Tables of the float32 adjoint in the r^2 form (same units as the forward
// table): g(s) = T s^(-3/2) and h(s) = g'(r) / r = 2 dg/ds =
// -(3 T + (4 / sqrt(pi)) x^3 e^(-x^2)) s^(-5/2), each fitted by its own
// quadratics at 2^kAdjBits segments per octave over [2^kAdjEmin,
// 2^kR2Emax) (the derivative of the forward's quadratics would be too coarse
// for the gradient), in six planes of kAdjPlane floats: g c0 c1 c2, h c0 c1
// c2; the row after the last (s = 2^kR2Emax) is zero.
std::vector<unsigned char> build_adj_table(double xc) {
    const double kappa = xc * xc / std::ldexp(1.0, pmfmm::kR2Emax);
    // six planes (g c0 c1 c2, h c0 c1 c2) fitted, then stored as three arrays
    // of float pairs by row: (g c0, g c1), (h c0, h c1), (g c2, h c2), each
    // kAdjPlane pairs long, so a lookup is three 8-byte reads from one
    // address at immediate offsets
    std::vector<float> f((size_t)6 * pmfmm::kAdjPlane, 0.0f);
    fit_r2_rows(pmfmm::kAdjBits, pmfmm::kAdjEmin, 2,
                [&](double sv) { return truncation_T(std::sqrt(sv * kappa)) * std::pow(sv, -1.5); },
                f.data(), pmfmm::kAdjPlane);
    fit_r2_rows(pmfmm::kAdjBits, pmfmm::kAdjEmin, 2,
                [&](double sv) {
                    const double x = std::sqrt(sv * kappa);
                    return -(3.0 * truncation_T(x) + 2.25675833419102514780 * x * x * x * std::exp(-x * x)) *
                           std::pow(sv, -2.5);
                },
                f.data() + 3 * (size_t)pmfmm::kAdjPlane, pmfmm::kAdjPlane);
    std::vector<unsigned char> out((size_t)pmfmm::kAdjTableBytes + 16, 0);
    float* o = reinterpret_cast<float*>(out.data());
    const size_t P = pmfmm::kAdjPlane;
    for (size_t k = 0; k < P; ++k) {
        o[2 * k] = f[k];                       // g c0
        o[2 * k + 1] = f[P + k];               // g c1
        o[2 * P + 2 * k] = f[3 * P + k];       // h c0
        o[2 * P + 2 * k + 1] = f[4 * P + k];   // h c1
        o[4 * P + 2 * k] = f[2 * P + k];       // g c2
        o[4 * P + 2 * k + 1] = f[5 * P + k];   // h c2
    }
    return out;
}

// Table of the float64 r^2 form: the same F(s) = T(x) s^(-3/2) on rows
// (e - kR2Emin64) 2^bits + j covering s in 2^e [1 + j / 2^bits, 1 + (j + 1) / 2^bits)
// for kR2Emin64 <= e < kR2Emax, each the polynomial of degree `deg`
// interpolating F at the segment's Chebyshev nodes, stored as its
// coefficients in t = s - (segment start) (the kernel evaluates it there;
// expanding about the start keeps the float64 evaluation free of
// cancellation).  Nodes are computed in long double; the segment width is a
// power of two, so the change of variable from [0, 1] is exact.
std::vector<unsigned char> build_r2_table64(int per_octave, int deg, double xc) {
    const int bits = per_octave == 16 ? 4 : per_octave == 32 ? 5 : 6;
    const int octaves = pmfmm::kR2Emax - pmfmm::kR2Emin64;
    const int rows = octaves << bits, m = deg + 1;
    const long double kappa = (long double)xc * xc / std::ldexp(1.0L, pmfmm::kR2Emax);
    // one extra row for s = 2^kR2Emax itself (a pair just inside the cutoff
    // whose scaled s rounds up): the constant F(2^kR2Emax)
    std::vector<unsigned char> out((size_t)8 * m * (rows + 1) + 16, 0);
    double* f = reinterpret_cast<double*>(out.data());
    const long double pi = 3.141592653589793238462643383279502884L;
    {
        const long double sv = std::ldexp(1.0L, pmfmm::kR2Emax), x = std::sqrt(sv * kappa);
        const long double T = std::erfc(x) + 1.128379167095512573896158903121545172L * x * std::exp(-x * x);
        f[(size_t)m * rows] = (double)(T / (sv * std::sqrt(sv)));
    }
    for (int k = 0; k < rows; ++k) {
        const int e = pmfmm::kR2Emin64 + (k >> bits), j = k & ((1 << bits) - 1);
        const long double lo = std::ldexp(1.0L + (long double)j / per_octave, e);
        const long double w = std::ldexp(1.0L, e - bits);
        long double V[7][8];
        for (int i = 0; i < m; ++i) {
            const long double t = 0.5L - 0.5L * std::cos(pi * (i + 0.5L) / m);   // in [0, 1]
            const long double sv = lo + w * t;
            long double tp = 1.0L;
            for (int q = 0; q < m; ++q) {
                V[i][q] = tp;
                tp *= t;
            }
            const long double x = std::sqrt(sv * kappa);
            const long double T = std::erfc(x) + 1.128379167095512573896158903121545172L * x * std::exp(-x * x);
            V[i][m] = T / (sv * std::sqrt(sv));
        }
        for (int c = 0; c < m; ++c) {
            int piv = c;
            for (int r = c + 1; r < m; ++r)
                if (std::fabs(V[r][c]) > std::fabs(V[piv][c])) piv = r;
            for (int q = 0; q <= m; ++q) std::swap(V[c][q], V[piv][q]);
            for (int r = c + 1; r < m; ++r) {
                const long double g = V[r][c] / V[c][c];
                for (int q = c; q <= m; ++q) V[r][q] -= g * V[c][q];
            }
        }
        long double cl[7] = {0, 0, 0, 0, 0, 0, 0};
        for (int c = m - 1; c >= 0; --c) {
            long double acc = V[c][m];
            for (int q = c + 1; q < m; ++q) acc -= V[c][q] * cl[q];
            cl[c] = acc / V[c][c];
        }
        // p(t) = sum_q cl_q t^q with t = (s - lo) / w: coefficient of (s - lo)^q is cl_q / w^q
        for (int q = 0; q < m; ++q) f[(size_t)m * k + q] = (double)std::ldexp(cl[q], -q * (e - bits));
    }
    return out;
}

std::vector<unsigned char> build_table(const pmfmm_params& p, double xc) {
    if (uses_r2(p)) return build_r2_table(p.table_size, p.table_level, xc);
    if (r2_table(p)) return build_r2_table64(p.table_size, p.table_level, xc);
    const int n = p.table_size;
    const double h = 3.0 / n;
    const double inv_sqrt_pi = 0.56418958354775628695;
    std::vector<double> c[5];
    for (auto& v : c) v.resize(n);
    for (int i = 0; i < n; ++i) {
        const double x = i * h, x2 = x * x;
        const double E = -4.0 * std::exp(-x2) * inv_sqrt_pi;
        const double a[5] = {std::erfc(x) - x * E / 2.0, x2 * E, -x * (x2 - 1.0) * E,
                             ((2.0 / 3.0) * x2 * x2 - (5.0 / 3.0) * x2 + 1.0 / 3.0) * E,
                             -x * ((1.0 / 3.0) * x2 * x2 - 1.5 * x2 + 1.0) * E};
        double hk = 1.0;
        for (int k = 0; k < 5; ++k) {
            c[k][i] = a[k] * hk;
            hk *= h;
        }
    }
    std::vector<unsigned char> out;
    if (p.precision == PMFMM_FP32) {
        // one node past x = 3; for the nearest node the polynomial is
        // re-expanded in e' = e + 1/2 in [0, 1):  c'_j = sum_k c_k C(k,j) (-1/2)^(k-j)
        const int m = n + 1;
        std::vector<double> a(5 * (size_t)m);
        for (int i = 0; i < m; ++i) {
            const double x = i * h, x2 = x * x;
            const double E = -4.0 * std::exp(-x2) * inv_sqrt_pi;
            const double b[5] = {std::erfc(x) - x * E / 2.0, x2 * E, -x * (x2 - 1.0) * E,
                                 ((2.0 / 3.0) * x2 * x2 - (5.0 / 3.0) * x2 + 1.0 / 3.0) * E,
                                 -x * ((1.0 / 3.0) * x2 * x2 - 1.5 * x2 + 1.0) * E};
            double hk = 1.0;
            double ck[5];
            for (int k = 0; k < 5; ++k) {
                ck[k] = b[k] * hk;
                hk *= h;
            }
            const int level = p.table_level;
            for (int k = level + 1; k < 5; ++k) ck[k] = 0.0;   // truncate before shifting
            if (p.table_round == PMFMM_ROUND_NEAREST) {
                static const double binom[5][5] = {{1, 0, 0, 0, 0}, {1, 1, 0, 0, 0}, {1, 2, 1, 0, 0},
                                                   {1, 3, 3, 1, 0}, {1, 4, 6, 4, 1}};
                double sh[5];
                for (int j = 0; j < 5; ++j) {
                    double acc = 0.0;
                    for (int k = j; k < 5; ++k) acc += ck[k] * binom[k][j] * std::pow(-0.5, k - j);
                    sh[j] = acc;
                }
                for (int k = 0; k < 5; ++k) ck[k] = sh[k];
            }
            for (int k = 0; k < 5; ++k) a[5 * (size_t)i + k] = ck[k];
        }
        out.resize((size_t)20 * m + 16);
        float* f4 = reinterpret_cast<float*>(out.data());
        float* f1 = reinterpret_cast<float*>(out.data() + 16 * (size_t)m);
        for (int i = 0; i < m; ++i) {
            for (int k = 0; k < 4; ++k) f4[4 * i + k] = (float)a[5 * (size_t)i + k];
            f1[i] = (float)a[5 * (size_t)i + 4];
        }
    } else {
        out.resize((size_t)40 * n + 16);
        double* d01 = reinterpret_cast<double*>(out.data());
        double* d23 = reinterpret_cast<double*>(out.data() + 16 * (size_t)n);
        double* d4 = reinterpret_cast<double*>(out.data() + 32 * (size_t)n);
        for (int i = 0; i < n; ++i) {
            d01[2 * i] = c[0][i];
            d01[2 * i + 1] = c[1][i];
            d23[2 * i] = c[2][i];
            d23[2 * i + 1] = c[3][i];
            d4[i] = c[4][i];
        }
    }
    out.resize((out.size() + 15) / 16 * 16);
    return out;
}

}  // namespace

struct pmfmm_ctx {
    pmfmm_params p{};
    // Host plan (host planner), or tree shape + lists copied back on demand
    // (GPU planner).
    mutable pmfmm::Plan plan;
    bool planned = false;
    bool built = false;
    bool gpu_planned = false;
    mutable bool lists_fresh = false;
    int device = -1;
    int n_cu = 0;
    pmfmm::DevPlan d;
    std::vector<unsigned char> table_host;
    std::vector<unsigned char> adj_table_host;   // float32 r^2 adjoint (g, h)
    double adj_table_xc = -1.0;
    bool table_dirty = true;
    double table_xc = -1.0;   // r_cut / 2 r_s the r^2 table was built for
    std::vector<pmfmm::BoxDev> boxes_on_device;   // last upload of d.boxes
    // sizes of the current plan
    int64_t n_items = 0, n_p2p = 0, n_m2l = 0, cand = 0;
    bool far = false;
    // smallest depth of an M2L source / target cell of the current plan
    int32_t m2l_dmin_src = 0, m2l_dmin_tgt = 0;
    // tree shape uploaded for the GPU planner
    std::vector<int64_t> topo_counts;
    std::vector<pmfmm::BoxParams> topo_boxes;
    bool topo_on_device = false;
    // timing
    hipEvent_t ev[6] = {nullptr, nullptr, nullptr, nullptr, nullptr, nullptr};
    bool timed_fwd = false, timed_adj = false;
    // far field started by the GPU build on a stream of its own while the
    // work items are made (far_done ends it; far_t0 / far_t1 time it)
    hipStream_t side = nullptr;
    hipEvent_t far_fork = nullptr, far_done = nullptr, far_t0 = nullptr, far_t1 = nullptr;
    bool far_early = false;     // d.far holds this build's far field (after far_done)
    // long-range mesh of pmfmm_long_range
    pmfmm::PMPlan pm;

    ~pmfmm_ctx() {
        if (device >= 0) {
            (void)hipSetDevice(device);
            (void)hipDeviceSynchronize();
        }
        d.release_all();
        pmfmm::pm_release(pm);
        for (auto& e : ev)
            if (e) (void)hipEventDestroy(e);
        for (hipEvent_t e : {far_fork, far_done, far_t0, far_t1})
            if (e) (void)hipEventDestroy(e);
        if (side) (void)hipStreamDestroy(side);
    }
};

namespace {

std::vector<pmfmm::BoxParams> one_box(const pmfmm_params& p) {
    return {pmfmm::BoxParams{p.box, p.r_s, p.r_cut, p.G, p.theta, p.max_leaf, p.order, p.m2l_cut}};
}

int do_plan(pmfmm_ctx* ctx, const std::vector<pmfmm::BoxParams>& boxes,
            const std::vector<int64_t>& counts, const double* pos, const double* mass) {
    ctx->planned = false;
    ctx->built = false;
    std::string msg;
    try {
        msg = pmfmm::make_plan(ctx->plan, boxes, counts, pos, mass, ctx->p.threads);
        if (msg.empty()) pmfmm::make_items(ctx->plan, ctx->p.chunk);
    } catch (const std::bad_alloc&) {
        return fail(PMFMM_ENOMEM, "host allocation failed while planning");
    } catch (const std::exception& e) {
        return fail(PMFMM_EINVAL, e.what());
    }
    if (!msg.empty()) return fail(PMFMM_EINVAL, msg);
    ctx->planned = true;
    ctx->gpu_planned = false;
    ctx->lists_fresh = true;
    ctx->topo_on_device = false;
    ctx->n_items = (int64_t)ctx->plan.items.size();
    ctx->n_p2p = (int64_t)ctx->plan.p2p_j.size();
    ctx->n_m2l = (int64_t)ctx->plan.m2l_src.size();
    ctx->cand = ctx->plan.candidate_pairs;
    ctx->far = ctx->plan.far_field;
    ctx->m2l_dmin_src = ctx->m2l_dmin_tgt = 0x7fffffff;
    const pmfmm::Plan& pl = ctx->plan;
    for (size_t c = 0; c + 1 < pl.m2l_row.size(); ++c)
        if (pl.m2l_row[c + 1] > pl.m2l_row[c])
            ctx->m2l_dmin_tgt = std::min(ctx->m2l_dmin_tgt, pl.cells[c].depth);
    for (int32_t u : pl.m2l_src) ctx->m2l_dmin_src = std::min(ctx->m2l_dmin_src, pl.cells[u].depth);
    return PMFMM_OK;
}

int check_box_params(int32_t nbox, const pmfmm_params* per_box, const int64_t* counts,
                     const pmfmm_params& eval, std::vector<pmfmm::BoxParams>& boxes,
                     std::vector<int64_t>& cnt) {
    if (nbox < 1 || per_box == nullptr || counts == nullptr) return fail(PMFMM_EINVAL, "need at least one box");
    for (int b = 0; b < nbox; ++b) {
        std::string why;
        if (!valid_geometry(per_box[b], why)) return fail(PMFMM_EINVAL, "box " + std::to_string(b) + ": " + why);
        if (eval.trunc == PMFMM_TRUNC_TABLE && per_box[b].r_cut / (2.0 * per_box[b].r_s) > 3.0)
            return fail(PMFMM_EINVAL, "box " + std::to_string(b) + ": the table covers r <= 6 r_s only");
        if (r2_table(eval) && !same_xc(per_box[b].r_cut, per_box[b].r_s, per_box[0].r_cut, per_box[0].r_s))
            return fail(PMFMM_EINVAL, "box " + std::to_string(b) +
                                          ": the r^2 table needs one r_cut / r_s for all boxes");
        if (counts[b] < 1) return fail(PMFMM_EINVAL, "box " + std::to_string(b) + ": needs at least one particle");
        const pmfmm_params& q = per_box[b];
        boxes.push_back(
            pmfmm::BoxParams{q.box, q.r_s, q.r_cut, q.G, q.theta, q.max_leaf, q.order, q.m2l_cut});
        cnt.push_back(counts[b]);
    }
    return PMFMM_OK;
}

template <class T>
int upload(DevBuf& b, const std::vector<T>& v, hipStream_t s) {
    HIP_TRY(b.ensure(v.size() * sizeof(T)));
    if (!v.empty()) HIP_TRY(hipMemcpyAsync(b.p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice, s));
    return PMFMM_OK;
}

int upload_items(pmfmm_ctx* ctx, hipStream_t s) {
    const pmfmm::Plan& pl = ctx->plan;
    std::vector<int32_t> it(4 * pl.items.size());
    for (size_t k = 0; k < pl.items.size(); ++k) {
        it[4 * k] = pl.items[k].leaf;
        it[4 * k + 1] = pl.items[k].t0;
        it[4 * k + 2] = pl.items[k].t1;
        it[4 * k + 3] = pl.items[k].slot;
    }
    int rc;
    if ((rc = upload(ctx->d.items, it, s))) return rc;
    if ((rc = upload(ctx->d.queue, pl.queue, s))) return rc;
    if ((rc = upload(ctx->d.leaf_slot, pl.leaf_slot_begin, s))) return rc;
    HIP_TRY(ctx->d.partial.ensure(std::max<size_t>(1, pl.items.size()) * 4 * 64 * sizeof(double)));
    HIP_TRY(hipStreamSynchronize(s));
    return PMFMM_OK;
}

// (Re)builds the table when the evaluation parameters changed, or, for the
// r^2 table, the boxes' r_cut / r_s.
int upload_table(pmfmm_ctx* ctx, hipStream_t s) {
    const double xc = ctx->plan.boxes.empty() ? ctx->p.r_cut / (2.0 * ctx->p.r_s)
                                              : ctx->plan.boxes[0].r_cut / (2.0 * ctx->plan.boxes[0].r_s);
    if (!ctx->table_dirty && (!r2_table(ctx->p) || xc == ctx->table_xc)) return PMFMM_OK;
    ctx->table_xc = xc;
    ctx->table_host = build_table(ctx->p, xc);
    int rc = upload(ctx->d.table, ctx->table_host, s);
    if (rc) return rc;
    HIP_TRY(hipStreamSynchronize(s));
    ctx->table_dirty = false;
    return PMFMM_OK;
}

// Float32 r^2 adjoint tables, built and uploaded on the first adjoint of
// that form and again when x_c changes.
int upload_adj_table(pmfmm_ctx* ctx, hipStream_t s) {
    const double xc = ctx->plan.boxes[0].r_cut / (2.0 * ctx->plan.boxes[0].r_s);
    if (ctx->d.adj_table.p != nullptr && xc == ctx->adj_table_xc) return PMFMM_OK;
    ctx->adj_table_host = build_adj_table(xc);
    int rc = upload(ctx->d.adj_table, ctx->adj_table_host, s);
    if (rc) return rc;
    HIP_TRY(hipStreamSynchronize(s));
    ctx->adj_table_xc = xc;
    return PMFMM_OK;
}

std::vector<pmfmm::BoxDev> box_table(const pmfmm_ctx* ctx) {
    std::vector<pmfmm::BoxDev> out;
    for (const auto& b : ctx->plan.boxes) {
        pmfmm::BoxDev d{};
        d.L = b.box;
        d.alpha = 1.0 / (2.0 * b.r_s);
        d.rc2 = b.r_cut * b.r_cut;
        d.G = b.G;
        // float32 offsets in units of 1 / sigma (see BoxDev)
        const bool r2 = uses_r2(ctx->p);
        d.sigma = r2 ? std::sqrt(std::ldexp(1.0, pmfmm::kR2Emax) / d.rc2) : 1.0;
        d.alpha_f = (float)(d.alpha / d.sigma);
        d.rc2_f = r2 ? std::ldexp(1.0f, pmfmm::kR2Emax) : (float)d.rc2;
        d.tiny_f = r2 ? std::ldexp(1.0f, pmfmm::kR2Emin) : d.rc2_f * 1e-14f;
        d.tab_scale = d.alpha * (ctx->p.table_size / 3.0);
        d.tab_scale_f = (float)(d.tab_scale / d.sigma);
        d.order = (b.order >= 0 && b.theta > 0.0) ? b.order : -1;
        out.push_back(d);
    }
    return out;
}

// Uploads the per-box constants unless the device already holds them.
int upload_boxes(pmfmm_ctx* ctx, hipStream_t s) {
    std::vector<pmfmm::BoxDev> bt = box_table(ctx);
    const bool same = ctx->d.boxes.p != nullptr && bt.size() == ctx->boxes_on_device.size() &&
                      std::memcmp(bt.data(), ctx->boxes_on_device.data(),
                                  bt.size() * sizeof(pmfmm::BoxDev)) == 0;
    if (same) return PMFMM_OK;
    int rc = upload(ctx->d.boxes, bt, s);
    if (rc) return rc;
    ctx->boxes_on_device = std::move(bt);
    return PMFMM_OK;
}

int prepare_far(pmfmm_ctx* ctx, hipStream_t s);

int do_upload(pmfmm_ctx* ctx, const double* pos, const double* mass, int32_t on_device, hipStream_t s) {
    const pmfmm::Plan& pl = ctx->plan;
    HIP_TRY(hipGetDevice(&ctx->device));
    HIP_TRY(hipDeviceGetAttribute(&ctx->n_cu, hipDeviceAttributeMultiprocessorCount, ctx->device));
    const int64_t n = pl.n, nl = (int64_t)pl.leaf_count.size();
    std::vector<int32_t> leaf(4 * nl);
    std::vector<double> leafc(4 * nl);
    for (int64_t l = 0; l < nl; ++l) {
        const pmfmm::Cell& c = pl.cells[pl.leaf_cell[l]];
        leaf[4 * l] = c.first;
        leaf[4 * l + 1] = c.count;
        leaf[4 * l + 2] = c.box;
        leaf[4 * l + 3] = pl.leaf_cell[l];
        for (int a = 0; a < 3; ++a) leafc[4 * l + a] = 0.5 * (c.lo[a] + c.hi[a]);
        leafc[4 * l + 3] = 0.0;
    }
    std::vector<int32_t> js(pl.p2p_j.size());
    for (size_t t = 0; t < js.size(); ++t) js[t] = (pl.p2p_j[t] << 5) | pl.p2p_shift[t];
    int rc;
    if ((rc = upload(ctx->d.perm, pl.perm, s))) return rc;
    if ((rc = upload(ctx->d.leaf, leaf, s))) return rc;
    if ((rc = upload(ctx->d.leafc, leafc, s))) return rc;
    if ((rc = upload(ctx->d.js, js, s))) return rc;
    if ((rc = upload_boxes(ctx, s))) return rc;
    HIP_TRY(ctx->d.counter.ensure(pmfmm::kQueueSegs * pmfmm::kCounterStride * 4));
    HIP_TRY(ctx->d.x64.ensure((size_t)n * 32));
    HIP_TRY(ctx->d.x32.ensure((size_t)n * 16));
    const double* src_pos = pos;
    const double* src_mass = mass;
    if (!on_device) {
        if ((rc = upload(ctx->d.stage_pos, pl.pos, s))) return rc;
        if ((rc = upload(ctx->d.stage_mass, pl.mass, s))) return rc;
        src_pos = ctx->d.stage_pos.as<double>();
        src_mass = ctx->d.stage_mass.as<double>();
    }
    pmfmm::GatherArgs g{src_pos, src_mass, ctx->d.perm.as<int32_t>(), ctx->d.leaf.as<int4>(),
                        ctx->d.leafc.as<double4>(), ctx->d.boxes.as<pmfmm::BoxDev>(), ctx->d.x64.as<double4>(),
                        ctx->d.x32.as<float4>(), (int32_t)nl};
    HIP_TRY(pmfmm::launch_gather(g, nullptr, s));
    if ((rc = upload_items(ctx, s))) return rc;
    if ((rc = upload_table(ctx, s))) return rc;
    if (pl.far_field) {
        // far-field arrays
        const int64_t nc = (int64_t)pl.cells.size();
        std::vector<int32_t> cell(4 * nc), aux(4 * nc);
        std::vector<double> cc(4 * nc);
        for (int64_t k = 0; k < nc; ++k) {
            const pmfmm::Cell& c = pl.cells[k];
            cell[4 * k] = c.first;
            cell[4 * k + 1] = c.count;
            cell[4 * k + 2] = c.parent;
            cell[4 * k + 3] = c.leaf;
            aux[4 * k] = c.child[0];
            aux[4 * k + 1] = c.child[1];
            aux[4 * k + 2] = c.box;
            aux[4 * k + 3] = c.depth;
            for (int a = 0; a < 3; ++a) cc[4 * k + a] = 0.5 * (c.lo[a] + c.hi[a]);
            cc[4 * k + 3] = 0.0;
        }
        if ((rc = upload(ctx->d.cell, cell, s))) return rc;
        if ((rc = upload(ctx->d.cell_aux, aux, s))) return rc;
        if ((rc = upload(ctx->d.cellc, cc, s))) return rc;
        if ((rc = upload(ctx->d.m2l_row, pl.m2l_row, s))) return rc;
        if ((rc = upload(ctx->d.m2l_src, pl.m2l_src, s))) return rc;
        if ((rc = upload(ctx->d.m2l_shift, pl.m2l_shift, s))) return rc;
        if ((rc = upload(ctx->d.level_cells, pl.cells_by_depth, s))) return rc;
        const int nco = pmfmm::n_coef(pl.max_order);
        HIP_TRY(ctx->d.M.ensure((size_t)nc * nco * sizeof(double)));
        HIP_TRY(ctx->d.Lc.ensure((size_t)nc * nco * sizeof(double)));
        HIP_TRY(ctx->d.Lt.ensure((size_t)std::max<int64_t>(1, ctx->n_m2l) * nco * sizeof(double)));
        HIP_TRY(ctx->d.far.ensure((size_t)n * 3 * sizeof(double)));
        if ((rc = prepare_far(ctx, s))) return rc;
    }
    HIP_TRY(hipStreamSynchronize(s));
    ctx->built = true;
    return PMFMM_OK;
}

// Table forms: 16 waves share one LDS copy of the table (a 2048-segment r^2
// table is 33 KB; with 4-wave groups LDS would cap a CU at 16 waves).
int default_wg_waves(int mode) {
    return (mode == pmfmm::kFP64Table || mode == pmfmm::kFP32Table || mode == pmfmm::kFP32R2 ||
            mode == pmfmm::kFP64R2)
               ? 16
               : 4;
}

pmfmm::FarArgs far_args(pmfmm_ctx* ctx) {
    const pmfmm::Plan& pl = ctx->plan;
    const int64_t nc = (int64_t)pl.cells.size();
    pmfmm::FarArgs f{};
    f.x64 = ctx->d.x64.as<double4>();
    f.leaf = ctx->d.leaf.as<int4>();
    f.leafc = ctx->d.leafc.as<double4>();
    f.cell = ctx->d.cell.as<int4>();
    f.cell_aux = ctx->d.cell_aux.as<int4>();
    f.cellc = ctx->d.cellc.as<double4>();
    f.m2l_row = ctx->d.m2l_row.as<int32_t>();
    f.m2l_src = ctx->d.m2l_src.as<int32_t>();
    f.m2l_shift = ctx->d.m2l_shift.as<int32_t>();
    f.boxes = ctx->d.boxes.as<pmfmm::BoxDev>();
    f.M = ctx->d.M.as<double>();
    f.Lc = ctx->d.Lc.as<double>();
    f.Lt = ctx->d.Lt.as<double>();
    f.n_m2l = (int32_t)ctx->n_m2l;
    f.far = ctx->d.far.as<double>();
    f.needM = ctx->d.farflag.as<int32_t>();
    f.needL = ctx->d.farflag.as<int32_t>() + 2 * nc;
    f.n_cells = (int32_t)nc;
    f.n_leaves = (int32_t)pl.leaf_count.size();
    f.order = pl.max_order;
    f.ncoef = pmfmm::n_coef(pl.max_order);
    return f;
}

// Per-plan marks of the cells the far field touches.
int prepare_far(pmfmm_ctx* ctx, hipStream_t s) {
    const int64_t nc = (int64_t)ctx->plan.cells.size();
    HIP_TRY(ctx->d.farflag.ensure((size_t)4 * nc * sizeof(int32_t)));
    HIP_TRY(pmfmm::launch_far_flags(far_args(ctx), s));
    return PMFMM_OK;
}

// Pass-up, M2L and pass-down of the far field (the leaves' multipoles are
// already in M; the locals end in Lc).
int far_middle(pmfmm_ctx* ctx, pmfmm::FarArgs& f, hipStream_t s) {
    const pmfmm::Plan& pl = ctx->plan;
    const int nd = (int)pl.depth_begin.size() - 1;
    // no cell above the shallowest M2L source needs a multipole, none above
    // the shallowest target a local expansion
    const int d_up = std::max(0, (int)std::min<int64_t>(ctx->m2l_dmin_src, nd));
    const int d_down = std::max(1, (int)std::min<int64_t>((int64_t)ctx->m2l_dmin_tgt + 1, nd));
    for (int d = nd - 2; d >= d_up; --d) {   // parents of the deepest level first
        f.level_cells = ctx->d.level_cells.as<int32_t>() + pl.depth_begin[d];
        f.n_level = pl.depth_begin[d + 1] - pl.depth_begin[d];
        HIP_TRY(pmfmm::launch_m2m_level(f, s));
    }
    HIP_TRY(pmfmm::launch_m2l(f, s));
    for (int d = d_down; d < nd; ++d) {
        f.level_cells = ctx->d.level_cells.as<int32_t>() + pl.depth_begin[d];
        f.n_level = pl.depth_begin[d + 1] - pl.depth_begin[d];
        HIP_TRY(pmfmm::launch_l2l_level(f, s));
    }
    return PMFMM_OK;
}

int run_far(pmfmm_ctx* ctx, hipStream_t s) {
    pmfmm::FarArgs f = far_args(ctx);
    HIP_TRY(pmfmm::launch_p2m(f, s));
    int rc = far_middle(ctx, f, s);
    if (rc) return rc;
    HIP_TRY(pmfmm::launch_l2p(f, s));
    return PMFMM_OK;
}

int far_buffers(pmfmm_ctx* ctx, int64_t n) {
    const int64_t nc = (int64_t)ctx->plan.cells.size();
    const int nco = pmfmm::n_coef(ctx->plan.max_order);
    HIP_TRY(ctx->d.M.ensure((size_t)nc * nco * sizeof(double)));
    HIP_TRY(ctx->d.Lc.ensure((size_t)nc * nco * sizeof(double)));
    HIP_TRY(ctx->d.Lt.ensure((size_t)std::max<int64_t>(1, ctx->n_m2l) * nco * sizeof(double)));
    HIP_TRY(ctx->d.far.ensure((size_t)n * 3 * sizeof(double)));
    return PMFMM_OK;
}

int ensure_side(pmfmm_ctx* ctx) {
    if (!ctx->side) HIP_TRY(hipStreamCreateWithFlags(&ctx->side, hipStreamNonBlocking));
    return PMFMM_OK;
}

// Starts marks + far field of the current build on the side stream, after
// the work enqueued so far on s (or, with side_ordered, after what is
// already on the side stream, which the caller has ordered after s);
// far_done marks its end.
int start_far(pmfmm_ctx* ctx, int64_t n, hipStream_t s, bool side_ordered = false) {
    int rc = far_buffers(ctx, n);
    if (rc) return rc;
    if ((rc = ensure_side(ctx))) return rc;
    for (hipEvent_t* e : {&ctx->far_fork, &ctx->far_done})
        if (!*e) HIP_TRY(hipEventCreateWithFlags(e, hipEventDisableTiming));
    for (hipEvent_t* e : {&ctx->far_t0, &ctx->far_t1})
        if (!*e) HIP_TRY(hipEventCreate(e));
    if (!side_ordered) {
        HIP_TRY(hipEventRecord(ctx->far_fork, s));
        HIP_TRY(hipStreamWaitEvent(ctx->side, ctx->far_fork, 0));
    }
    ctx->far = true;
    if ((rc = prepare_far(ctx, ctx->side))) return rc;
    HIP_TRY(hipEventRecord(ctx->far_t0, ctx->side));
    if ((rc = run_far(ctx, ctx->side))) return rc;
    HIP_TRY(hipEventRecord(ctx->far_t1, ctx->side));
    HIP_TRY(hipEventRecord(ctx->far_done, ctx->side));
    ctx->far_early = true;
    return PMFMM_OK;
}

// Orders s after the side stream's far field (before anything that reuses
// its buffers or reads its result).
int wait_far(pmfmm_ctx* ctx, hipStream_t s) {
    if (ctx->far_early) HIP_TRY(hipStreamWaitEvent(s, ctx->far_done, 0));
    return PMFMM_OK;
}

// Far-field part of the adjoint into fargrad (leaf order, no G): the
// forward locals give the L2P Hessian term; then the transposed pass on
// sign-flipped coefficients (leaf W2M, the same pass-up / M2L / pass-down
// over the symmetric M2L list) gives the P2M terms.  w64 must hold the
// leaf-ordered cotangent.
int run_far_adjoint(pmfmm_ctx* ctx, hipStream_t s) {
    pmfmm::FarArgs f = far_args(ctx);
    const double4* w64 = ctx->d.w64.as<double4>();
    double4* fg = ctx->d.fargrad.as<double4>();
    HIP_TRY(pmfmm::launch_p2m(f, s));
    int rc = far_middle(ctx, f, s);
    if (rc) return rc;
    HIP_TRY(pmfmm::launch_far_hess(f, w64, fg, s));
    HIP_TRY(pmfmm::launch_w2m(f, w64, s));
    if ((rc = far_middle(ctx, f, s))) return rc;
    HIP_TRY(pmfmm::launch_far_adj(f, fg, s));
    return PMFMM_OK;
}

int ensure_events(pmfmm_ctx* ctx) {
    for (auto& e : ctx->ev)
        if (!e) HIP_TRY(hipEventCreate(&e));
    return PMFMM_OK;
}

bool same_boxes(const std::vector<pmfmm::BoxParams>& a, const std::vector<pmfmm::BoxParams>& b) {
    if (a.size() != b.size()) return false;
    for (size_t k = 0; k < a.size(); ++k)
        if (a[k].box != b[k].box || a[k].r_s != b[k].r_s || a[k].r_cut != b[k].r_cut || a[k].G != b[k].G ||
            a[k].theta != b[k].theta || a[k].max_leaf != b[k].max_leaf || a[k].order != b[k].order ||
            a[k].m2l_cut != b[k].m2l_cut)
            return false;
    return true;
}

int ensure_device(pmfmm_ctx* ctx) {
    HIP_TRY(hipGetDevice(&ctx->device));
    HIP_TRY(hipDeviceGetAttribute(&ctx->n_cu, hipDeviceAttributeMultiprocessorCount, ctx->device));
    return PMFMM_OK;
}

// Plan on the GPU from particles (device or host pointers).
int gpu_build(pmfmm_ctx* ctx, const std::vector<pmfmm::BoxParams>& boxes, const std::vector<int64_t>& cnt,
              const double* pos, const double* mass, int32_t on_device, hipStream_t s) {
    ctx->planned = false;
    ctx->built = false;
    int rc = ensure_device(ctx);
    if (rc) return rc;
    int64_t n = 0;
    for (int64_t c : cnt) n += c;
    if (n > (int64_t)INT32_MAX) return fail(PMFMM_EINVAL, "too many particles (limit 2^31 - 1)");
    const double* dp = pos;
    const double* dm = mass;
    if (!on_device) {
        HIP_TRY(ctx->d.stage_pos.ensure((size_t)n * 24));
        HIP_TRY(ctx->d.stage_mass.ensure((size_t)n * 8));
        HIP_TRY(hipMemcpyAsync(ctx->d.stage_pos.p, pos, (size_t)n * 24, hipMemcpyHostToDevice, s));
        HIP_TRY(hipMemcpyAsync(ctx->d.stage_mass.p, mass, (size_t)n * 8, hipMemcpyHostToDevice, s));
        dp = ctx->d.stage_pos.as<double>();
        dm = ctx->d.stage_mass.as<double>();
    }
    HIP_TRY(pmfmm::gpu_enqueue_checks(ctx->d, dp, dm, n, s));
    const bool same = ctx->topo_on_device && ctx->topo_counts == cnt && same_boxes(ctx->topo_boxes, boxes);
    if (!same) {
        try {
            pmfmm::make_topology(ctx->plan, boxes, cnt);
        } catch (const std::bad_alloc&) {
            return fail(PMFMM_ENOMEM, "host allocation failed while shaping the tree");
        }
        if ((int64_t)ctx->plan.cells.size() >= ((int64_t)1 << 27))
            return fail(PMFMM_EINVAL, "too many tree cells (limit 2^27)");
        const std::vector<pmfmm::BoxDev> bt = box_table(ctx);
        HIP_TRY(pmfmm::upload_topology(ctx->d, ctx->plan, bt.data(), s));
        ctx->boxes_on_device = bt;
        ctx->topo_counts = cnt;
        ctx->topo_boxes = boxes;
        ctx->topo_on_device = true;
    } else {
        if ((rc = upload_boxes(ctx, s))) return rc;
    }
    pmfmm::PlanCounts pc;
    std::string input_err;
    // the far field needs the tree, the leaf-ordered particles and the M2L
    // lists, not the work items: start it on the side stream once the M2L
    // lists are enqueued, so it runs while the items are built
    int far_rc = PMFMM_OK;
    const int64_t n_all = n;
    // the planner builds the M2L rows on the side stream (ordered after the
    // walk on s) and calls far_start right after them
    if ((rc = ensure_side(ctx))) return rc;
    auto far_start = [&](int64_t n_m2l, int32_t dsrc, int32_t dtgt) -> std::string {
        if (n_m2l <= 0) return std::string();
        ctx->n_m2l = n_m2l;
        ctx->m2l_dmin_src = dsrc;
        ctx->m2l_dmin_tgt = dtgt;
        far_rc = start_far(ctx, n_all, s, true);
        return far_rc ? std::string("far field") : std::string();
    };
    std::string err = pmfmm::gpu_build_plan(ctx->d, ctx->plan, dp, dm, ctx->p.chunk, s, pc, &input_err,
                                            far_start, ctx->side);
    if (far_rc) return far_rc;
    if (!input_err.empty()) return fail(PMFMM_EINVAL, input_err);
    if (!err.empty()) return fail(PMFMM_EDEVICE, err);
    ctx->n_p2p = pc.n_p2p;
    ctx->n_m2l = pc.n_m2l;
    ctx->n_items = pc.n_items;
    ctx->cand = pc.candidate_pairs;
    ctx->m2l_dmin_src = pc.m2l_min_depth_src;
    ctx->m2l_dmin_tgt = pc.m2l_min_depth_tgt;
    ctx->far = pc.n_m2l > 0;
    ctx->plan.far_field = ctx->far;
    ctx->plan.candidate_pairs = pc.candidate_pairs;
    HIP_TRY(ctx->d.counter.ensure(pmfmm::kQueueSegs * pmfmm::kCounterStride * 4));
    if (ctx->far && !ctx->far_early) {
        if ((rc = far_buffers(ctx, n))) return rc;
        if ((rc = prepare_far(ctx, s))) return rc;
    }
    if ((rc = upload_table(ctx, s))) return rc;
    ctx->planned = true;
    ctx->built = true;
    ctx->gpu_planned = true;
    ctx->lists_fresh = false;
    return PMFMM_OK;
}

// Copies the device-built lists back into the host plan views.
int download_lists(const pmfmm_ctx* ctx) {
    pmfmm::Plan& pl = ctx->plan;
    const pmfmm::DevPlan& d = ctx->d;
    const int64_t n = pl.n, nc = (int64_t)pl.cells.size(), nl = (int64_t)pl.leaf_cell.size();
    pl.perm.resize(n);
    pl.cell_lo.resize(3 * nc);
    pl.cell_hi.resize(3 * nc);
    pl.p2p_row.resize(nl + 1);
    std::vector<int32_t> js(ctx->n_p2p);
    pl.m2l_row.resize(nc + 1);
    pl.m2l_src.resize(ctx->n_m2l);
    pl.m2l_shift.resize(ctx->n_m2l);
    HIP_TRY(hipMemcpy(pl.perm.data(), d.perm.p, n * 4, hipMemcpyDeviceToHost));
    HIP_TRY(hipMemcpy(pl.cell_lo.data(), d.clo.p, nc * 24, hipMemcpyDeviceToHost));
    HIP_TRY(hipMemcpy(pl.cell_hi.data(), d.chi.p, nc * 24, hipMemcpyDeviceToHost));
    HIP_TRY(hipMemcpy(pl.p2p_row.data(), d.p2p_row.p, (nl + 1) * 4, hipMemcpyDeviceToHost));
    if (ctx->n_p2p) HIP_TRY(hipMemcpy(js.data(), d.js.p, ctx->n_p2p * 4, hipMemcpyDeviceToHost));
    HIP_TRY(hipMemcpy(pl.m2l_row.data(), d.m2l_row.p, (nc + 1) * 4, hipMemcpyDeviceToHost));
    if (ctx->n_m2l) {
        HIP_TRY(hipMemcpy(pl.m2l_src.data(), d.m2l_src.p, ctx->n_m2l * 4, hipMemcpyDeviceToHost));
        HIP_TRY(hipMemcpy(pl.m2l_shift.data(), d.m2l_shift.p, ctx->n_m2l * 4, hipMemcpyDeviceToHost));
    }
    pl.p2p_j.resize(ctx->n_p2p);
    pl.p2p_shift.resize(ctx->n_p2p);
    for (int64_t t = 0; t < ctx->n_p2p; ++t) {
        pl.p2p_j[t] = js[t] >> 5;
        pl.p2p_shift[t] = js[t] & 31;
    }
    pl.cell_first.resize(nc);
    pl.cell_count.resize(nc);
    pl.cell_child.resize(2 * nc);
    for (int64_t k = 0; k < nc; ++k) {
        pmfmm::Cell& c = pl.cells[k];
        for (int a = 0; a < 3; ++a) {
            c.lo[a] = pl.cell_lo[3 * k + a];
            c.hi[a] = pl.cell_hi[3 * k + a];
        }
        pl.cell_first[k] = c.first;
        pl.cell_count[k] = c.count;
        pl.cell_child[2 * k] = c.child[0];
        pl.cell_child[2 * k + 1] = c.child[1];
    }
    ctx->lists_fresh = true;
    return PMFMM_OK;
}

}  // namespace

extern "C" {

void pmfmm_params_init(pmfmm_params* p) {
    if (!p) return;
    std::memset(p, 0, sizeof(*p));
    p->box = 100.0;
    p->r_s = 3.75;
    p->r_cut = 4.5 * 3.75;
    p->G = 1.0;
    p->theta = 0.0;
    p->m2l_cut = PMFMM_M2L_INSIDE;
    p->max_leaf = 64;
    p->order = 4;
    p->precision = PMFMM_FP64;
    p->trunc = PMFMM_TRUNC_EXACT;
    p->table_size = 2048;
    p->table_level = 4;
    p->table_round = PMFMM_ROUND_NEAREST;
    p->accum = PMFMM_ACCUM_FP64;
}

const char* pmfmm_version(void) { return "pmfmm-mi355x 0.1"; }

const char* pmfmm_last_error(void) { return g_err.c_str(); }

int pmfmm_create(const pmfmm_params* p, pmfmm_ctx** out) {
    if (!p || !out) return fail(PMFMM_EINVAL, "null argument");
    std::string why;
    if (!valid_geometry(*p, why) || !valid_eval(*p, why)) return fail(PMFMM_EINVAL, why);
    if (p->trunc == PMFMM_TRUNC_TABLE && p->r_cut / (2.0 * p->r_s) > 3.0)
        return fail(PMFMM_EINVAL, "the table covers r <= 6 r_s only");
    pmfmm_ctx* c = new (std::nothrow) pmfmm_ctx();
    if (!c) return fail(PMFMM_ENOMEM, "context allocation failed");
    c->p = *p;
    *out = c;
    return PMFMM_OK;
}

void pmfmm_destroy(pmfmm_ctx* ctx) { delete ctx; }

int pmfmm_plan(pmfmm_ctx* ctx, int64_t n, const double* pos, const double* mass) {
    if (!ctx || !pos || !mass) return fail(PMFMM_EINVAL, "null argument");
    if (n < 1) return fail(PMFMM_EINVAL, "n must be >= 1");
    return do_plan(ctx, one_box(ctx->p), {n}, pos, mass);
}

int pmfmm_plan_batch(pmfmm_ctx* ctx, int32_t nbox, const pmfmm_params* per_box,
                     const int64_t* counts, const double* pos, const double* mass) {
    if (!ctx || !pos || !mass) return fail(PMFMM_EINVAL, "null argument");
    std::vector<pmfmm::BoxParams> boxes;
    std::vector<int64_t> cnt;
    int rc = check_box_params(nbox, per_box, counts, ctx->p, boxes, cnt);
    if (rc) return rc;
    return do_plan(ctx, boxes, cnt, pos, mass);
}

static int build_common(pmfmm_ctx* ctx, const std::vector<pmfmm::BoxParams>& boxes,
                        const std::vector<int64_t>& cnt, const double* pos, const double* mass,
                        int32_t on_device, void* stream) {
    hipStream_t s = static_cast<hipStream_t>(stream);
    // the previous build's far field (side stream) reads buffers this build
    // rewrites
    int wrc = wait_far(ctx, s);
    if (wrc) return wrc;
    ctx->far_early = false;
    if (ctx->p.planner == 0) return gpu_build(ctx, boxes, cnt, pos, mass, on_device, s);
    int64_t n = 0;
    for (int64_t c : cnt) n += c;
    const double* hp = pos;
    const double* hm = mass;
    std::vector<double> tmp_pos, tmp_mass;
    if (on_device) {
        tmp_pos.resize(3 * (size_t)n);
        tmp_mass.resize((size_t)n);
        HIP_TRY(hipMemcpyAsync(tmp_pos.data(), pos, tmp_pos.size() * sizeof(double), hipMemcpyDeviceToHost, s));
        HIP_TRY(hipMemcpyAsync(tmp_mass.data(), mass, tmp_mass.size() * sizeof(double), hipMemcpyDeviceToHost, s));
        HIP_TRY(hipStreamSynchronize(s));
        hp = tmp_pos.data();
        hm = tmp_mass.data();
    }
    int rc = do_plan(ctx, boxes, cnt, hp, hm);
    if (rc) return rc;
    return do_upload(ctx, pos, mass, on_device, s);
}

int pmfmm_build(pmfmm_ctx* ctx, int64_t n, const double* pos, const double* mass, int32_t on_device,
                void* stream) {
    if (!ctx || !pos || !mass) return fail(PMFMM_EINVAL, "null argument");
    if (n < 1) return fail(PMFMM_EINVAL, "n must be >= 1");
    return build_common(ctx, one_box(ctx->p), {n}, pos, mass, on_device, stream);
}

int pmfmm_build_batch(pmfmm_ctx* ctx, int32_t nbox, const pmfmm_params* per_box, const int64_t* counts,
                      const double* pos, const double* mass, int32_t on_device, void* stream) {
    if (!ctx || !pos || !mass) return fail(PMFMM_EINVAL, "null argument");
    std::vector<pmfmm::BoxParams> boxes;
    std::vector<int64_t> cnt;
    int rc = check_box_params(nbox, per_box, counts, ctx->p, boxes, cnt);
    if (rc) return rc;
    return build_common(ctx, boxes, cnt, pos, mass, on_device, stream);
}

int pmfmm_set_eval(pmfmm_ctx* ctx, const pmfmm_params* p) {
    if (!ctx || !p) return fail(PMFMM_EINVAL, "null argument");
    std::string why;
    if (!valid_eval(*p, why)) return fail(PMFMM_EINVAL, why);
    if (p->trunc == PMFMM_TRUNC_TABLE && ctx->planned)
        for (const auto& b : ctx->plan.boxes)
            if (b.r_cut / (2.0 * b.r_s) > 3.0) return fail(PMFMM_EINVAL, "the table covers r <= 6 r_s only");
    if (r2_table(*p) && ctx->planned && !one_xc(ctx->plan.boxes))
        return fail(PMFMM_EINVAL, "the r^2 table needs one r_cut / r_s for all boxes");
    const bool table_change = p->precision != ctx->p.precision || p->table_size != ctx->p.table_size ||
                              p->table_round != ctx->p.table_round || p->table_level != ctx->p.table_level ||
                              p->trunc != ctx->p.trunc;
    // the float32 offsets' scale (x32) depends on this
    const bool sigma_change = uses_r2(*p) != uses_r2(ctx->p);
    const bool chunk_change = p->chunk != ctx->p.chunk;
    ctx->p.precision = p->precision;
    ctx->p.trunc = p->trunc;
    ctx->p.table_size = p->table_size;
    ctx->p.table_level = p->table_level;
    ctx->p.table_round = p->table_round;
    ctx->p.accum = p->accum;
    ctx->p.chunk = p->chunk;
    ctx->p.wg_waves = p->wg_waves;
    ctx->p.grid_wgs = p->grid_wgs;
    ctx->p.timing = p->timing;
    if (table_change) ctx->table_dirty = true;
    if (ctx->planned && chunk_change) {
        if (ctx->gpu_planned) {
            pmfmm::PlanCounts pc;
            std::string err = pmfmm::gpu_make_items(ctx->d, ctx->plan, ctx->n_p2p, ctx->p.chunk, nullptr, pc);
            if (!err.empty()) return fail(PMFMM_EDEVICE, err);
            ctx->n_items = pc.n_items;
        } else {
            pmfmm::make_items(ctx->plan, ctx->p.chunk);
            ctx->n_items = (int64_t)ctx->plan.items.size();
            if (ctx->built) {
                int rc = upload_items(ctx, nullptr);
                if (rc) return rc;
            }
        }
    }
    if (ctx->built) {
        // per-box constants depend on table_size
        int rc = upload_boxes(ctx, nullptr);
        if (rc) return rc;
        if (sigma_change)
            HIP_TRY(pmfmm::launch_rescale_x32(ctx->d.leaf.as<int4>(), ctx->d.leafc.as<double4>(),
                                              ctx->d.boxes.as<pmfmm::BoxDev>(), ctx->d.x64.as<double4>(),
                                              ctx->d.x32.as<float4>(), (int32_t)ctx->plan.leaf_count.size(),
                                              nullptr));
        HIP_TRY(hipStreamSynchronize(nullptr));
    }
    return PMFMM_OK;
}

}  // extern "C"

namespace {

// The forward after the checks: far field (or the wait for the one the
// build started), the persistent P2P kernel with its queue counters in
// `counter` and the item partials in `partial`, the ordered reduction.
// Launches only: allocates nothing (the timing events must exist when
// `timing` is set).
int forward_launch(pmfmm_ctx* ctx, double* acc, hipStream_t s, int32_t* counter, double* partial,
                   bool timing) {
    const pmfmm::Plan& pl = ctx->plan;
    const int mode = mode_of(ctx->p);
    int rc;
    if (timing) HIP_TRY(hipEventRecord(ctx->ev[0], s));
    if (ctx->far) {
        if (ctx->far_early) {
            if ((rc = wait_far(ctx, s))) return rc;   // computed during the build
        } else if ((rc = run_far(ctx, s))) {
            return rc;
        }
    }
    HIP_TRY(pmfmm::launch_zero_i32(counter, pmfmm::kQueueSegs * pmfmm::kCounterStride, s));
    if (timing) HIP_TRY(hipEventRecord(ctx->ev[1], s));
    pmfmm::P2PArgs a{};
    a.x64 = ctx->d.x64.as<double4>();
    a.x32 = ctx->d.x32.as<float4>();
    a.leaf = ctx->d.leaf.as<int4>();
    a.leafc = ctx->d.leafc.as<double4>();
    a.p2p_js = ctx->d.js.as<int32_t>();
    a.items = ctx->d.items.as<int4>();
    a.queue = ctx->d.queue.as<int32_t>();
    a.n_items = (int32_t)ctx->n_items;
    a.counter = counter;
    a.partial = partial;
    a.boxes = ctx->d.boxes.as<pmfmm::BoxDev>();
    a.table = ctx->d.table.p;
    a.n_tab = ctx->p.table_size;
    a.level = ctx->p.table_level;
    a.round_floor = ctx->p.table_round == PMFMM_ROUND_FLOOR;
    a.accum32 = ctx->p.accum == PMFMM_ACCUM_FP32_TWOSUM;
    const bool tab = mode == pmfmm::kFP32Table || mode == pmfmm::kFP64Table || mode == pmfmm::kFP32R2 ||
                     mode == pmfmm::kFP64R2;
    const size_t lds = tab ? ctx->table_host.size() : 0;
    const int wg = std::min(ctx->p.wg_waves > 0 ? ctx->p.wg_waves : default_wg_waves(mode),
                            pmfmm::p2p_max_threads(mode) / 64);
    int grid = ctx->p.grid_wgs;
    if (grid <= 0) grid = ctx->n_cu * pmfmm::p2p_blocks_per_cu(mode, wg, lds);
    HIP_TRY(pmfmm::launch_p2p(mode, a, wg, grid, lds, s));
    if (timing) HIP_TRY(hipEventRecord(ctx->ev[2], s));
    pmfmm::ReduceArgs r{ctx->d.leaf.as<int4>(), ctx->d.leaf_slot.as<int32_t>(), partial,
                        ctx->far ? ctx->d.far.as<double>() : nullptr,
                        ctx->far ? ctx->d.farflag.as<int32_t>() + 2 * (int64_t)pl.cells.size() : nullptr,
                        ctx->d.perm.as<int32_t>(), ctx->d.boxes.as<pmfmm::BoxDev>(), acc,
                        (int32_t)pl.leaf_count.size()};
    HIP_TRY(pmfmm::launch_reduce(r, s));
    if (timing) {
        HIP_TRY(hipEventRecord(ctx->ev[3], s));
        ctx->timed_fwd = true;
    }
    return PMFMM_OK;
}

// The table the build uploaded still matches the evaluation parameters.
bool table_current(const pmfmm_ctx* ctx) {
    const double xc = ctx->plan.boxes.empty() ? ctx->p.r_cut / (2.0 * ctx->p.r_s)
                                              : ctx->plan.boxes[0].r_cut / (2.0 * ctx->plan.boxes[0].r_s);
    return !ctx->table_dirty && (!r2_table(ctx->p) || xc == ctx->table_xc);
}

}  // namespace

extern "C" {

int pmfmm_forward(pmfmm_ctx* ctx, double* acc, void* stream) {
    if (!ctx || !acc) return fail(PMFMM_EINVAL, "null argument");
    if (!ctx->built) return fail(PMFMM_ESTATE, "forward before build");
    hipStream_t s = static_cast<hipStream_t>(stream);
    int rc = upload_table(ctx, s);
    if (rc) return rc;
    const bool timing = ctx->p.timing != 0;
    if (timing && (rc = ensure_events(ctx))) return rc;
    return forward_launch(ctx, acc, s, ctx->d.counter.as<int32_t>(), ctx->d.partial.as<double>(), timing);
}

int pmfmm_forward_static(pmfmm_ctx* ctx, double* acc, void* stream) {
    if (!ctx || !acc) return fail(PMFMM_EINVAL, "null argument");
    if (!ctx->built) return fail(PMFMM_ESTATE, "forward before build");
    if (!table_current(ctx))
        return fail(PMFMM_ESTATE,
                    "the evaluation changed since the build: the table is not on the device "
                    "(run pmfmm_forward once, or build again)");
    if (ctx->n_items > pmfmm::kStaticMaxItems)
        return fail(PMFMM_EINVAL, "plan has " + std::to_string(ctx->n_items) +
                                      " work items; the static scratch holds at most " +
                                      std::to_string(pmfmm::kStaticMaxItems) + " (use pmfmm_forward)");
    void* base = nullptr;
    HIP_TRY(pmfmm::static_scratch(&base));
    unsigned char* b = static_cast<unsigned char*>(base);
    return forward_launch(ctx, acc, static_cast<hipStream_t>(stream), reinterpret_cast<int32_t*>(b),
                          reinterpret_cast<double*>(b + pmfmm::kStaticCounterBytes), false);
}

}  // extern "C"

namespace {

// Cache key of the autotuner: device, pair form, coarse size of the plan.
std::string tune_key(const pmfmm_ctx* ctx) {
    hipDeviceProp_t prop{};
    std::string arch = "unknown";
    if (hipGetDeviceProperties(&prop, ctx->device) == hipSuccess) arch = prop.gcnArchName;
    for (char& c : arch)
        if (c == ' ' || c == '\t' || c == '\n') c = '_';
    const int64_t bucket = (int64_t)std::llround(2.0 * std::sqrt((double)std::max<int64_t>(1, ctx->n_p2p))) / 64;
    const pmfmm_params& p = ctx->p;
    return arch + "|" + std::to_string(ctx->n_cu) + "|" + std::to_string(p.precision) + "|" +
           std::to_string(p.trunc) + "|" + std::to_string(p.table_size) + "|" + std::to_string(p.table_level) +
           "|" + std::to_string(p.accum) + "|" + std::to_string(ctx->plan.boxes.size()) + "|" +
           std::to_string(ctx->plan.leaf_count.size() / 1024) + "|" + std::to_string(bucket);
}

bool tune_cache_find(const char* path, const std::string& key, pmfmm_schedule& out) {
    std::FILE* f = std::fopen(path, "r");
    if (!f) return false;
    char line[1024];
    bool found = false;
    while (std::fgets(line, sizeof line, f)) {
        char k[768];
        pmfmm_schedule sc{};
        if (std::sscanf(line, "%767s %d %d %d %lf", k, &sc.chunk, &sc.wg_waves, &sc.grid_wgs, &sc.p2p_ms) == 5 &&
            key == k) {
            out = sc;   // the last entry for a key wins
            found = true;
        }
    }
    std::fclose(f);
    return found;
}

void tune_cache_add(const char* path, const std::string& key, const pmfmm_schedule& sc) {
    std::FILE* f = std::fopen(path, "a");
    if (!f) return;   // an unwritable cache only costs the next run a tuning
    std::fprintf(f, "%s %d %d %d %.6f\n", key.c_str(), sc.chunk, sc.wg_waves, sc.grid_wgs, sc.p2p_ms);
    std::fclose(f);
}

int apply_schedule(pmfmm_ctx* ctx, const pmfmm_schedule& sc, int32_t timing) {
    pmfmm_params p = ctx->p;
    p.chunk = sc.chunk;
    p.wg_waves = sc.wg_waves;
    p.grid_wgs = sc.grid_wgs;
    p.timing = timing;
    return pmfmm_set_eval(ctx, &p);
}

}  // namespace

extern "C" {

int pmfmm_autotune(pmfmm_ctx* ctx, double* acc, const pmfmm_schedule* cands, int32_t n_cands,
                   int32_t repeats, const char* cache_path, pmfmm_schedule* results,
                   pmfmm_schedule* best, void* stream) {
    if (!ctx || !acc || !best) return fail(PMFMM_EINVAL, "null argument");
    if (!ctx->built) return fail(PMFMM_ESTATE, "autotune before build");
    if (repeats < 1 || repeats > 100) return fail(PMFMM_EINVAL, "repeats must be in 1..100");
    std::vector<pmfmm_schedule> todo;
    if (cands) {
        if (n_cands < 1 || n_cands > 4096) return fail(PMFMM_EINVAL, "n_cands must be in 1..4096");
        todo.assign(cands, cands + n_cands);
    } else {
        for (int32_t chunk : {0, 8, 16, 32, 64, 1 << 20})
            for (int32_t wg : {2, 4, 8, 16}) todo.push_back(pmfmm_schedule{chunk, wg, 0, 0, -1.0});
    }
    for (const auto& sc : todo)
        if (sc.chunk < 0 || sc.wg_waves < 0 || sc.wg_waves > 16 || sc.grid_wgs < 0)
            return fail(PMFMM_EINVAL, "candidate schedule out of range (chunk >= 0, wg_waves 0..16, grid_wgs >= 0)");
    hipStream_t s = static_cast<hipStream_t>(stream);
    const int32_t timing0 = ctx->p.timing;
    const std::string key = tune_key(ctx);
    pmfmm_schedule hit{};
    if (cache_path && tune_cache_find(cache_path, key, hit)) {
        int rc = apply_schedule(ctx, hit, timing0);
        if (rc) return rc;
        *best = hit;
        return PMFMM_OK;
    }
    const int max_waves = pmfmm::p2p_max_threads(mode_of(ctx->p)) / 64;
    int win = -1;
    for (size_t i = 0; i < todo.size(); ++i) {
        pmfmm_schedule& sc = todo[i];
        sc.p2p_ms = -1.0;
        if (sc.wg_waves > max_waves) continue;   // the launch would run max_waves anyway
        int rc = apply_schedule(ctx, sc, 1);
        if (!rc) rc = pmfmm_forward(ctx, acc, stream);
        double sum = 0.0;
        for (int r = 0; !rc && r < repeats; ++r) {
            pmfmm_timings t{};
            rc = pmfmm_forward(ctx, acc, stream);
            if (!rc) rc = pmfmm_get_timings(ctx, &t);
            sum += t.p2p_ms;
        }
        if (rc) {
            (void)apply_schedule(ctx, pmfmm_schedule{0, 0, 0, 0, -1.0}, timing0);
            return rc;
        }
        sc.p2p_ms = sum / repeats;
        if (win < 0 || sc.p2p_ms < todo[win].p2p_ms) win = (int)i;
    }
    HIP_TRY(hipStreamSynchronize(s));
    if (results) std::copy(todo.begin(), todo.end(), results);
    if (win < 0) return fail(PMFMM_EINVAL, "no candidate schedule can run this form");
    int rc = apply_schedule(ctx, todo[win], timing0);
    if (rc) return rc;
    *best = todo[win];
    if (cache_path) tune_cache_add(cache_path, key, *best);
    return PMFMM_OK;
}

int pmfmm_kick(int64_t n, double* vel, const double* acc, double dt, void* stream) {
    if (!vel || !acc) return fail(PMFMM_EINVAL, "null argument");
    if (n < 0 || !std::isfinite(dt)) return fail(PMFMM_EINVAL, "n must be >= 0 and dt finite");
    HIP_TRY(pmfmm::launch_kick(n, vel, acc, dt, static_cast<hipStream_t>(stream)));
    return PMFMM_OK;
}

int pmfmm_drift(int64_t n, double* pos, const double* vel, double dt, double box, void* stream) {
    if (!pos || !vel) return fail(PMFMM_EINVAL, "null argument");
    if (n < 0 || !std::isfinite(dt) || !(box > 0.0))
        return fail(PMFMM_EINVAL, "n must be >= 0, dt finite and box > 0");
    HIP_TRY(pmfmm::launch_drift(n, pos, vel, dt, box, static_cast<hipStream_t>(stream)));
    return PMFMM_OK;
}

int pmfmm_long_range(pmfmm_ctx* ctx, int32_t n_pm, int64_t n, const double* pos, const double* mass,
                     double* acc, void* stream) {
    if (!ctx || !pos || !mass || !acc) return fail(PMFMM_EINVAL, "null argument");
    if (n < 0) return fail(PMFMM_EINVAL, "n must be >= 0");
    if (n_pm < 4 || n_pm > 1024 || (n_pm % 2) != 0)
        return fail(PMFMM_EINVAL, "n_pm must be even and in [4, 1024]");
    hipStream_t s = static_cast<hipStream_t>(stream);
    HIP_TRY(hipGetDevice(&ctx->device));
    HIP_TRY(pmfmm::pm_plan(ctx->pm, n_pm, s));
    HIP_TRY(pmfmm::pm_long_range(ctx->pm, pos, mass, n, ctx->p.box, ctx->p.r_s, ctx->p.G, acc, s));
    return PMFMM_OK;
}

int pmfmm_get_lists(const pmfmm_ctx* ctx, pmfmm_lists* out) {
    if (!ctx || !out) return fail(PMFMM_EINVAL, "null argument");
    if (!ctx->planned) return fail(PMFMM_ESTATE, "no plan");
    if (!ctx->lists_fresh) {
        int rc = download_lists(ctx);
        if (rc) return rc;
    }
    const pmfmm::Plan& pl = ctx->plan;
    out->n = pl.n;
    out->n_boxes = (int64_t)pl.boxes.size();
    out->n_leaves = (int64_t)pl.leaf_count.size();
    out->n_cells = (int64_t)pl.cells.size();
    out->n_p2p = ctx->n_p2p;
    out->n_m2l = ctx->n_m2l;
    out->n_items = ctx->n_items;
    out->candidate_pairs = ctx->cand;
    out->perm = pl.perm.data();
    out->box_first_leaf = pl.box_first_leaf.data();
    out->box_first_cell = pl.box_first_cell.data();
    out->leaf_first = pl.leaf_first.data();
    out->leaf_count = pl.leaf_count.data();
    out->leaf_cell = pl.leaf_cell.data();
    out->cell_first = pl.cell_first.data();
    out->cell_count = pl.cell_count.data();
    out->cell_child = pl.cell_child.data();
    out->cell_lo = pl.cell_lo.data();
    out->cell_hi = pl.cell_hi.data();
    out->p2p_row = pl.p2p_row.data();
    out->p2p_j = pl.p2p_j.data();
    out->p2p_shift = pl.p2p_shift.data();
    out->m2l_row = pl.m2l_row.data();
    out->m2l_src = pl.m2l_src.data();
    out->m2l_shift = pl.m2l_shift.data();
    return PMFMM_OK;
}

int pmfmm_get_timings(const pmfmm_ctx* ctx, pmfmm_timings* out) {
    if (!ctx || !out) return fail(PMFMM_EINVAL, "null argument");
    if (!ctx->timed_fwd && !ctx->timed_adj) return fail(PMFMM_ESTATE, "nothing timed (params.timing = 0?)");
    std::memset(out, 0, sizeof(*out));
    float ms = 0.f;
    if (ctx->timed_fwd) {
        HIP_TRY(hipEventSynchronize(ctx->ev[3]));
        if (ctx->far_early) {
            // run by the build on the side stream, beside the work items
            HIP_TRY(hipEventElapsedTime(&ms, ctx->far_t0, ctx->far_t1));
        } else {
            HIP_TRY(hipEventElapsedTime(&ms, ctx->ev[0], ctx->ev[1]));
        }
        out->far_ms = ms;
        HIP_TRY(hipEventElapsedTime(&ms, ctx->ev[1], ctx->ev[2]));
        out->p2p_ms = ms;
        HIP_TRY(hipEventElapsedTime(&ms, ctx->ev[2], ctx->ev[3]));
        out->reduce_ms = ms;
        HIP_TRY(hipEventElapsedTime(&ms, ctx->ev[0], ctx->ev[3]));
        out->total_ms = ms;
    }
    if (ctx->timed_adj) {
        HIP_TRY(hipEventSynchronize(ctx->ev[5]));
        HIP_TRY(hipEventElapsedTime(&ms, ctx->ev[4], ctx->ev[5]));
        out->adjoint_ms = ms;
    }
    return PMFMM_OK;
}

int pmfmm_adjoint(pmfmm_ctx* ctx, const double* w, double* grad_pos, double* grad_mass, void* stream) {
    if (!ctx || !w || !grad_pos || !grad_mass) return fail(PMFMM_EINVAL, "null argument");
    if (!ctx->built) return fail(PMFMM_ESTATE, "adjoint before build");
    hipStream_t s = static_cast<hipStream_t>(stream);
    {
        // the far-field adjoint reuses the multipole buffers of the build's
        // far field
        int rc = wait_far(ctx, s);
        if (rc) return rc;
    }
    const pmfmm::Plan& pl = ctx->plan;
    const int64_t n = pl.n;
    HIP_TRY(ctx->d.w64.ensure((size_t)n * 32));
    HIP_TRY(ctx->d.w32.ensure((size_t)n * 16));
    HIP_TRY(pmfmm::launch_gather_w(w, ctx->d.perm.as<int32_t>(), ctx->d.w64.as<double4>(), ctx->d.w32.as<float4>(),
                                   (int32_t)n, s));
    HIP_TRY(pmfmm::launch_zero_i32(ctx->d.counter.as<int32_t>(), pmfmm::kQueueSegs * pmfmm::kCounterStride, s));
    const bool timing = ctx->p.timing != 0;
    if (timing) {
        int rc = ensure_events(ctx);
        if (rc) return rc;
        HIP_TRY(hipEventRecord(ctx->ev[4], s));
    }
    pmfmm::AdjArgs a{};
    a.x64 = ctx->d.x64.as<double4>();
    a.x32 = ctx->d.x32.as<float4>();
    a.w64 = ctx->d.w64.as<double4>();
    a.w32 = ctx->d.w32.as<float4>();
    a.leaf = ctx->d.leaf.as<int4>();
    a.leafc = ctx->d.leafc.as<double4>();
    a.p2p_js = ctx->d.js.as<int32_t>();
    a.items = ctx->d.items.as<int4>();
    a.queue = ctx->d.queue.as<int32_t>();
    a.n_items = (int32_t)ctx->n_items;
    a.counter = ctx->d.counter.as<int32_t>();
    a.partial = ctx->d.partial.as<double>();
    a.boxes = ctx->d.boxes.as<pmfmm::BoxDev>();
    const int mode = mode_of(ctx->p);
    if (uses_r2(ctx->p)) {
        // the float32 r^2 form: g and h from tables as well
        int rc = upload_adj_table(ctx, s);
        if (rc) return rc;
        a.table = ctx->d.adj_table.p;
    }
    // 8 waves per workgroup share the tables of the r^2 form (measured on
    // the 64^3 clustered workload: 1.02 ms against 1.13 ms with 4 and
    // 1.06 ms with 16; same results bit for bit).  The exact forms take
    // within 2 % of the same time with 4, 8 or 16.
    const int wg = std::min(ctx->p.wg_waves > 0 ? ctx->p.wg_waves : (a.table != nullptr ? 8 : 4),
                            pmfmm::adjoint_max_threads(mode) / 64);
    int grid = ctx->p.grid_wgs;
    if (grid <= 0) grid = ctx->n_cu * pmfmm::adjoint_blocks_per_cu(mode, wg, a.table != nullptr);
    HIP_TRY(pmfmm::launch_adjoint(mode, a, wg, grid, s));
    if (timing) {
        HIP_TRY(hipEventRecord(ctx->ev[5], s));
        ctx->timed_adj = true;
    }
    const double4* fg = nullptr;
    if (ctx->far) {
        HIP_TRY(ctx->d.fargrad.ensure((size_t)n * 32));
        int rc = run_far_adjoint(ctx, s);
        if (rc) return rc;
        fg = ctx->d.fargrad.as<double4>();
    }
    pmfmm::AdjReduceArgs r{ctx->d.leaf.as<int4>(), ctx->d.leaf_slot.as<int32_t>(), ctx->d.partial.as<double>(),
                           fg, ctx->d.perm.as<int32_t>(), ctx->d.boxes.as<pmfmm::BoxDev>(), grad_pos,
                           grad_mass, (int32_t)pl.leaf_count.size()};
    HIP_TRY(pmfmm::launch_adj_reduce(r, s));
    return PMFMM_OK;
}

}  // extern "C"
