// Time stepping of the particles (the simulation loop around the force
// split; the paper's runs of Sec. 4 take time steps without naming the
// integrator, read here as a kick-drift-kick leapfrog): a kick adds acc dt
// to the velocities, a drift adds vel dt to the positions and wraps them
// into [0, L).  Both are elementwise over the
// (n, 3) caller-order arrays, bound by HBM traffic.
#include "device.h"

namespace pmfmm {
namespace {

__global__ void kick_kernel(int64_t m, double* __restrict__ vel, const double* __restrict__ acc,
                            double dt) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < m) vel[i] += acc[i] * dt;
}

__global__ void drift_kernel(int64_t m, double* __restrict__ pos, const double* __restrict__ vel,
                             double dt, double L) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= m) return;
    double x = pos[i] + vel[i] * dt;
    if (!(x >= 0.0 && x < L)) {
        x -= L * floor(x / L);
        if (x >= L) x -= L;
        if (x < 0.0) x += L;
        if (!(x >= 0.0 && x < L)) x = 0.0;
    }
    pos[i] = x;
}

}  // namespace

hipError_t launch_kick(int64_t n, double* vel, const double* acc, double dt, hipStream_t s) {
    const int64_t m = 3 * n;
    if (m <= 0) return hipSuccess;
    hipLaunchKernelGGL(kick_kernel, dim3((unsigned)((m + 255) / 256)), dim3(256), 0, s, m, vel, acc, dt);
    return hipGetLastError();
}

hipError_t launch_drift(int64_t n, double* pos, const double* vel, double dt, double L, hipStream_t s) {
    const int64_t m = 3 * n;
    if (m <= 0) return hipSuccess;
    hipLaunchKernelGGL(drift_kernel, dim3((unsigned)((m + 255) / 256)), dim3(256), 0, s, m, pos, vel, dt,
                       L);
    return hipGetLastError();
}

}  // namespace pmfmm
