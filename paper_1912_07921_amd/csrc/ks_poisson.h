// Internal interface of the Hartree solver (ks_poisson.hip): the Poisson
// equation Lap v_H = -4 pi n as one product with a fixed real kernel in
// Fourier space, evaluated with hand-written FFTs.  Not part of the ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>

#include "ks_internal.h"

namespace ks {

constexpr int kFftMaxLen = 512;     // longest transform along one axis
constexpr int kFftMaxStages = 12;

// One axis of the transform: length M = product of the radices (16, 8, 4,
// 2, 3, 5, in this order), twiddles tw[m] = exp(-2 pi i m / M) on the
// device.
struct FftAxis {
    int M = 1;
    int nst = 0;
    int rad[kFftMaxStages] = {};
    const double2 *tw = nullptr;
};

// Per grid: transform lengths (on a finite grid the smallest product of 2,
// 3 and 5 that is >= 2 n_a - 1, so that the cyclic convolution equals the
// free-space one; n_a on a periodic grid), the
// twiddle tables and the kernel K in Fourier space.  K is real and even
// along every axis, so only the octant k_a <= M_a / 2 is stored:
// K[(kz * (My/2 + 1) + ky) * (Mx/2 + 1) + kx], scaled by 1 / (Mx My Mz)
// (and h^3 on a finite grid).
struct PoissonPlan {
    bool periodic = false;
    FftAxis ax[3];
    double2 *tw[3] = {nullptr, nullptr, nullptr};
    double *K = nullptr;
    // work array of one solve: [nz][My][Mx/2 + 1] complex
    size_t work_elems = 0;
};

// Transform lengths of a grid; false if a length exceeds kFftMaxLen or (on
// a periodic grid) is not a product of 2, 3 and 5: the grid's Hartree term
// is then unsupported.
bool poisson_lengths(const Geo &g, bool periodic, int M[3]);

// Build the plan: twiddles and K (for a finite grid K is the transform of
// the sampled 1/r, computed here with a temporary M^3 array).
// Synchronous on `st`.
hipError_t poisson_plan_create(const Geo &g, bool periodic, PoissonPlan *pp,
                               hipStream_t st);
void poisson_plan_destroy(PoissonPlan *pp);

// v = v_H[rho] (add = false) or v += v_H[rho] (add = true); work holds
// pp.work_elems complex values.  Five launches, no allocation and no
// memset (safe under stream capture).
hipError_t launch_hartree(const PoissonPlan &pp, const Geo &g,
                          const double *rho, double *v, bool add,
                          double2 *work, hipStream_t st);

// part[b] = sum over block b of a[i] * b[i] (blocks of the density kernel:
// density_blocks(N) of them).
hipError_t launch_real_dot_partial(const double *a, const double *b, long N,
                                   double *part, hipStream_t st);

}  // namespace ks
