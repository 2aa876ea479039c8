// Internal interface of the observables (ks_observe.hip): the macroscopic
// current from the commutator [H, r] and damped transforms of traces.  Not
// part of the ABI.
#pragma once

#include <hip/hip_runtime.h>

#include "ks_internal.h"

namespace ks {

struct CurArgs {
    Geo geo;
    const double2 *psi = nullptr;   // [ns][N] states of this launch
    const double2 *kph = nullptr;   // [nk][3] exp(i k_a L_a)
    int nstates = 1;                // states per k-point
    int sg0 = 0;                    // global index of launch state 0
    double A[3] = {0.0, 0.0, 0.0};  // vector potential at the time
    ProjDev pj;
    double *nl = nullptr;           // [ns][natoms][3] projector terms
};

// Projector part of the current (the stencil part is the H.psi kernel's
// mode kCurrent).
hipError_t launch_current_nl(const CurArgs &a, int ns, hipStream_t st);

// mode 0: strength function (scale = kick), mode 1: conductivity (scale =
// field, out holds nw complex values)
hipError_t launch_damped_ft(const double *f, int nt, int stride, double dt,
                            double scale, double gamma, const double *w,
                            int nw, int mode, double *out, hipStream_t st);

}  // namespace ks
