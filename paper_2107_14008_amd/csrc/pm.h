// Long-range mesh force of the split (pm.hip): mesh buffers and FFT plans
// of one mesh size, owned by a context.
#pragma once

#include <hip/hip_runtime.h>
#include <hipfft/hipfft.h>

#include <cstdint>

namespace pmfmm {

struct PMPlan {
    int n = 0;                    // nodes per axis (0: nothing allocated)
    hipfftHandle fwd = 0, inv = 0;
    double* rho = nullptr;        // (n, n, n) density
    double* rk = nullptr;         // (n, n, n / 2 + 1) complex spectrum
    double* gk[3] = {nullptr, nullptr, nullptr};     // gradient spectra
    double* field[3] = {nullptr, nullptr, nullptr};  // (n, n, n) accelerations
};

// (Re)allocates the mesh and plans for n nodes per axis (kept while n stays
// the same) and binds the plans to stream s.
hipError_t pm_plan(PMPlan& p, int n, hipStream_t s);
void pm_release(PMPlan& p);
// Long-range accelerations of np particles (pos (np, 3), mass (np), device,
// caller order) into acc (np, 3), on the mesh of p, enqueued on s.
hipError_t pm_long_range(PMPlan& p, const double* pos, const double* mass, int64_t np, double L,
                         double r_s, double G, double* acc, hipStream_t s);

}  // namespace pmfmm
