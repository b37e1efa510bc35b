// Long-range part of the force split (Sec. 2) on a periodic mesh: cloud in
// cell assignment, a 3D real FFT, the Gaussian-filtered Newtonian Green's
// function, the spectral gradient, three inverse FFTs and cloud in cell
// interpolation, in float64.
//
//   rho(g)  = (N / L)^3 sum_i m_i W(x_i - g L / N)        (CIC weights W)
//   phi(k)  = -4 pi G rho(k) exp(-k^2 r_s^2) / k^2 / C(k)^2,  phi(0) = 0,
//             C(k) = prod_a sinc^2(k_a L / 2N) (undoes the assignment and
//             the interpolation once each)
//   a_a(k)  = -i k_a phi(k), the Nyquist component of k_a set to zero
//   a(x_i)  = sum_g W(x_i - g L / N) a(g)
//
// exp(-k^2 r_s^2) is the transform of erf(r / 2 r_s) / r over that of 1 / r,
// so this force plus the short-range pair force of Eq. (tr) is Newton's.
// The FFTs are rocFFT's (through hipFFT), plain library transforms; the
// deposit uses float64 atomics, so sums agree run to run only to rounding.
#include "pm.h"

#include <cmath>

namespace pmfmm {
namespace {

constexpr double kPi = 3.14159265358979323846;

__device__ __forceinline__ double wrap_pm(double x, double L) {
#pragma clang fp contract(off)
    if (x >= 0.0 && x < L) return x;
    double y = x - L * floor(x / L);
    if (y >= L) y -= L;
    if (y < 0.0) y += L;
    if (!(y >= 0.0 && y < L)) y = 0.0;
    return y;
}

// Lower node and the two CIC weights along one axis.
__device__ __forceinline__ void cic_axis(double x, double L, int n, int& g, double& w0, double& w1) {
    const double u = wrap_pm(x, L) * ((double)n / L);
    const double fl = floor(u);
    const double f = u - fl;
    g = (int)fl;
    if (g >= n) g -= n;
    w0 = 1.0 - f;
    w1 = f;
}

__global__ void pm_zero(double* __restrict__ p, int64_t m) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < m) p[i] = 0.0;
}

__global__ void pm_deposit(const double* __restrict__ pos, const double* __restrict__ mass, int64_t np,
                           double L, int n, double* __restrict__ rho) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= np) return;
    int g[3];
    double w[3][2];
    for (int a = 0; a < 3; ++a) cic_axis(pos[3 * i + a], L, n, g[a], w[a][0], w[a][1]);
    const double inv_cell = (double)n / L;
    const double mi = mass[i] * inv_cell * inv_cell * inv_cell;
    for (int dx = 0; dx < 2; ++dx) {
        const int x = g[0] + dx < n ? g[0] + dx : 0;
        for (int dy = 0; dy < 2; ++dy) {
            const int y = g[1] + dy < n ? g[1] + dy : 0;
            for (int dz = 0; dz < 2; ++dz) {
                const int z = g[2] + dz < n ? g[2] + dz : 0;
                atomicAdd(&rho[((int64_t)x * n + y) * n + z], mi * w[0][dx] * w[1][dy] * w[2][dz]);
            }
        }
    }
}

__device__ __forceinline__ double sinc(double x) { return x == 0.0 ? 1.0 : sin(x) / x; }

// One thread per mode of the half spectrum (n, n, n / 2 + 1): the three
// gradient spectra, scaled by 1 / n^3 for the unnormalised inverse FFT.
__global__ void pm_green(const double2* __restrict__ rk, int n, double L, double r_s, double G,
                         double2* __restrict__ ax, double2* __restrict__ ay, double2* __restrict__ az) {
    const int nzh = n / 2 + 1;
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t total = (int64_t)n * n * nzh;
    if (q >= total) return;
    const int iz = (int)(q % nzh);
    const int iy = (int)((q / nzh) % n);
    const int ix = (int)(q / ((int64_t)nzh * n));
    const double dk = 2.0 * kPi / L;
    // numpy fftfreq order: index n / 2 is -n / 2 (the Nyquist mode)
    const int mx = ix < (n + 1) / 2 ? ix : ix - n;
    const int my = iy < (n + 1) / 2 ? iy : iy - n;
    const int mz = iz < (n + 1) / 2 ? iz : iz - n;
    const double kx = dk * mx, ky = dk * my, kz = dk * mz;
    const double k2 = kx * kx + ky * ky + kz * kz;
    double2 zero = make_double2(0.0, 0.0);
    if (k2 == 0.0) {
        ax[q] = zero;
        ay[q] = zero;
        az[q] = zero;
        return;
    }
    const double h2 = 0.5 * L / (double)n;
    const double c = sinc(kx * h2) * sinc(ky * h2) * sinc(kz * h2);
    const double C = c * c;
    const double inv_n3 = 1.0 / ((double)n * (double)n * (double)n);
    const double gk = -4.0 * kPi * G * exp(-k2 * r_s * r_s) / k2 / (C * C) * inv_n3;
    const double2 r = rk[q];
    const double pr = r.x * gk, pi = r.y * gk;   // phi(k)
    const bool even = (n % 2) == 0;
    const double kxx = (even && ix == n / 2) ? 0.0 : kx;
    const double kyy = (even && iy == n / 2) ? 0.0 : ky;
    const double kzz = (even && iz == n / 2) ? 0.0 : kz;
    // -i k phi = (k pi, -k pr)
    ax[q] = make_double2(kxx * pi, -kxx * pr);
    ay[q] = make_double2(kyy * pi, -kyy * pr);
    az[q] = make_double2(kzz * pi, -kzz * pr);
}

__global__ void pm_interp(const double* __restrict__ pos, int64_t np, double L, int n,
                          const double* __restrict__ fx, const double* __restrict__ fy,
                          const double* __restrict__ fz, double* __restrict__ acc) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= np) return;
    int g[3];
    double w[3][2];
    for (int a = 0; a < 3; ++a) cic_axis(pos[3 * i + a], L, n, g[a], w[a][0], w[a][1]);
    double s[3] = {0.0, 0.0, 0.0};
    for (int dx = 0; dx < 2; ++dx) {
        const int x = g[0] + dx < n ? g[0] + dx : 0;
        for (int dy = 0; dy < 2; ++dy) {
            const int y = g[1] + dy < n ? g[1] + dy : 0;
            for (int dz = 0; dz < 2; ++dz) {
                const int z = g[2] + dz < n ? g[2] + dz : 0;
                const int64_t node = ((int64_t)x * n + y) * n + z;
                const double wt = w[0][dx] * w[1][dy] * w[2][dz];
                s[0] += wt * fx[node];
                s[1] += wt * fy[node];
                s[2] += wt * fz[node];
            }
        }
    }
    acc[3 * i] = s[0];
    acc[3 * i + 1] = s[1];
    acc[3 * i + 2] = s[2];
}

inline unsigned blocks_of(int64_t m) { return (unsigned)((m + 255) / 256); }

}  // namespace

hipError_t pm_plan(PMPlan& p, int n, hipStream_t s) {
    if (p.n == n && p.fwd != 0) {
        if (hipfftSetStream(p.fwd, s) != HIPFFT_SUCCESS || hipfftSetStream(p.inv, s) != HIPFFT_SUCCESS)
            return hipErrorUnknown;
        return hipSuccess;
    }
    pm_release(p);
    const int64_t n3 = (int64_t)n * n * n, nh = (int64_t)n * n * (n / 2 + 1);
    hipError_t e;
    if ((e = hipMalloc(&p.rho, n3 * sizeof(double))) != hipSuccess) return e;
    if ((e = hipMalloc(&p.rk, nh * 2 * sizeof(double))) != hipSuccess) return e;
    for (int a = 0; a < 3; ++a) {
        if ((e = hipMalloc(&p.gk[a], nh * 2 * sizeof(double))) != hipSuccess) return e;
        if ((e = hipMalloc(&p.field[a], n3 * sizeof(double))) != hipSuccess) return e;
    }
    if (hipfftPlan3d(&p.fwd, n, n, n, HIPFFT_D2Z) != HIPFFT_SUCCESS) return hipErrorUnknown;
    if (hipfftPlan3d(&p.inv, n, n, n, HIPFFT_Z2D) != HIPFFT_SUCCESS) return hipErrorUnknown;
    if (hipfftSetStream(p.fwd, s) != HIPFFT_SUCCESS || hipfftSetStream(p.inv, s) != HIPFFT_SUCCESS)
        return hipErrorUnknown;
    p.n = n;
    return hipSuccess;
}

void pm_release(PMPlan& p) {
    if (p.fwd) (void)hipfftDestroy(p.fwd);
    if (p.inv) (void)hipfftDestroy(p.inv);
    p.fwd = p.inv = 0;
    if (p.rho) (void)hipFree(p.rho);
    if (p.rk) (void)hipFree(p.rk);
    p.rho = nullptr;
    p.rk = nullptr;
    for (int a = 0; a < 3; ++a) {
        if (p.gk[a]) (void)hipFree(p.gk[a]);
        if (p.field[a]) (void)hipFree(p.field[a]);
        p.gk[a] = nullptr;
        p.field[a] = nullptr;
    }
    p.n = 0;
}

hipError_t pm_long_range(PMPlan& p, const double* pos, const double* mass, int64_t np, double L,
                         double r_s, double G, double* acc, hipStream_t s) {
    const int n = p.n;
    const int64_t n3 = (int64_t)n * n * n, nh = (int64_t)n * n * (n / 2 + 1);
    hipLaunchKernelGGL(pm_zero, dim3(blocks_of(n3)), dim3(256), 0, s, p.rho, n3);
    if (np > 0)
        hipLaunchKernelGGL(pm_deposit, dim3(blocks_of(np)), dim3(256), 0, s, pos, mass, np, L, n, p.rho);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    if (hipfftExecD2Z(p.fwd, p.rho, reinterpret_cast<hipfftDoubleComplex*>(p.rk)) != HIPFFT_SUCCESS)
        return hipErrorUnknown;
    hipLaunchKernelGGL(pm_green, dim3(blocks_of(nh)), dim3(256), 0, s,
                       reinterpret_cast<const double2*>(p.rk), n, L, r_s, G,
                       reinterpret_cast<double2*>(p.gk[0]), reinterpret_cast<double2*>(p.gk[1]),
                       reinterpret_cast<double2*>(p.gk[2]));
    if ((e = hipGetLastError()) != hipSuccess) return e;
    for (int a = 0; a < 3; ++a)
        if (hipfftExecZ2D(p.inv, reinterpret_cast<hipfftDoubleComplex*>(p.gk[a]), p.field[a]) !=
            HIPFFT_SUCCESS)
            return hipErrorUnknown;
    if (np > 0)
        hipLaunchKernelGGL(pm_interp, dim3(blocks_of(np)), dim3(256), 0, s, pos, np, L, n, p.field[0],
                           p.field[1], p.field[2], acc);
    return hipGetLastError();
}

}  // namespace pmfmm
