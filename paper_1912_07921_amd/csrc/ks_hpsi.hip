// H.psi pass: kernel instantiations and launch (single grid).
#ifndef KS_HPSI_PART
#define KS_HPSI_PART 0
#endif
// Planes the H.psi kernel's loads run ahead: the FP64 kernels (part 0)
// keep one register set (fewer registers; measured faster at 64^3, 48^3
// and 128^3), the mixed ones two alternating sets.
#ifndef KS_HPSI_PF
#define KS_HPSI_PF (KS_HPSI_PART == 0 ? 1 : 2)
#endif

#include "ks_device.h"

#include <algorithm>

namespace ks {

// Occupancy hint (waves per SIMD the register allocation must allow); 0
// leaves the choice to the compiler.
#ifndef KS_HPSI_MIN_WAVES
#define KS_HPSI_MIN_WAVES 0
#endif
#if KS_HPSI_MIN_WAVES > 0
#define KS_HPSI_ATTR __attribute__((amdgpu_waves_per_eu(KS_HPSI_MIN_WAVES)))
#else
#define KS_HPSI_ATTR
#endif

template <class R, class InT, class TT, int MODE, bool GRAD, int HM, int RPT>
__global__ __launch_bounds__(512) KS_HPSI_ATTR void k_hpsi(HArgs a)
{
    hpsi_item<R, InT, TT, MODE, GRAD, HM, RPT>(
        a, xcd_remap(blockIdx.x, gridDim.x),
        make_double4(a.A[0], a.A[1], a.A[2], a.a2half));
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
#if KS_HPSI_PART == 0
int hpsi_threads(int nx, int TY, int rpt)
{
    const int want = std::max(nx * ((TY + rpt - 1) / rpt), 64);
    return ((want + 63) / 64) * 64;
}

int hpsi_halo_per_thread(const Geo &g, int TY, int nthr)
{
    // dynamic halo entries (in-grid rows, and wrapped columns on a
    // periodic x axis) of a full tile
    const int dyn = 2 * kHalf * g.nx + (g.per[0] ? 2 * kHalf * (TY + 2 * kHalf)
                                                  : 0);
    const int hm = (dyn + nthr - 1) / nthr;
    return hm <= 2 ? 2 : (hm <= 4 ? 4 : (hm <= 8 ? 8 : 16));
}

size_t hpsi_lds_bytes(int nx, int TY, int zchunk, bool mixed)
{
    const size_t v = mixed ? 8 : 16;
    return 2 * (size_t)(TY + 2 * kHalf) * (nx + 2 * kHalf) * v + 90 * v +
           (size_t)zchunk * TY * sizeof(int4);
}

#endif

template <class R, class InT, class TT, int MODE, bool GRAD>
static hipError_t go_hpsi2(const HArgs &a, int ns, hipStream_t st)
{
    const int nthr = hpsi_threads(a.geo.nx, a.TY, a.rpt);
    const size_t lds = hpsi_lds_bytes(a.geo.nx, a.TY, a.zchunk,
                                      sizeof(R) == 4);
    dim3 grid((unsigned)(a.ntile_y * a.nzc * ns));
    const int hm = hpsi_halo_per_thread(a.geo, a.TY, nthr);
    if (a.rpt == 2) {
        if (hm <= 2)
            hipLaunchKernelGGL((k_hpsi<R, InT, TT, MODE, GRAD, 2, 2>), grid,
                               dim3(nthr), lds, st, a);
        else if (hm <= 4)
            hipLaunchKernelGGL((k_hpsi<R, InT, TT, MODE, GRAD, 4, 2>), grid,
                               dim3(nthr), lds, st, a);
        else
            hipLaunchKernelGGL((k_hpsi<R, InT, TT, MODE, GRAD, 8, 2>), grid,
                               dim3(nthr), lds, st, a);
        return hipGetLastError();
    }
    switch (hm) {
    case 2:
        hipLaunchKernelGGL((k_hpsi<R, InT, TT, MODE, GRAD, 2, 1>), grid,
                           dim3(nthr), lds, st, a);
        break;
    case 4:
        hipLaunchKernelGGL((k_hpsi<R, InT, TT, MODE, GRAD, 4, 1>), grid,
                           dim3(nthr), lds, st, a);
        break;
    case 8:
        hipLaunchKernelGGL((k_hpsi<R, InT, TT, MODE, GRAD, 8, 1>), grid,
                           dim3(nthr), lds, st, a);
        break;
    default:
        hipLaunchKernelGGL((k_hpsi<R, InT, TT, MODE, GRAD, 16, 1>), grid,
                           dim3(nthr), lds, st, a);
        break;
    }
    return hipGetLastError();
}

template <class R, class InT, class TT, int MODE>
static hipError_t go_hpsi(const HArgs &a, int ns, hipStream_t st)
{
    const bool grad = (a.A[0] != 0.0) || (a.A[1] != 0.0) || (a.A[2] != 0.0);
    return grad ? go_hpsi2<R, InT, TT, MODE, true>(a, ns, st)
                : go_hpsi2<R, InT, TT, MODE, false>(a, ns, st);
}

// The file is compiled twice: KS_HPSI_PART 0 holds the FP64 kernels and the
// dispatcher, KS_HPSI_PART 1 the mixed-precision kernels (two objects that
// compile in parallel).
hipError_t launch_hpsi_mixed(int mode, bool in_is_f64, const HArgs &a, int ns,
                             hipStream_t st);

#if KS_HPSI_PART == 0
hipError_t launch_hpsi(int mode, bool mixed, bool in_is_f64, const HArgs &a,
                       int ns, hipStream_t st)
{
    if (ns <= 0)
        return hipSuccess;
    if (mixed)
        return launch_hpsi_mixed(mode, in_is_f64, a, ns, st);
    switch (mode) {
    case kApply: return go_hpsi<double, double2, double2, kApply>(a, ns, st);
    case kTerm: return go_hpsi<double, double2, double2, kTerm>(a, ns, st);
    case kFinal: return go_hpsi<double, double2, double2, kFinal>(a, ns, st);
    case kFinalPred:
        return go_hpsi<double, double2, double2, kFinalPred>(a, ns, st);
    }
    return hipErrorInvalidValue;
}

hipError_t launch_hpsi_current(const HArgs &a, int ns, hipStream_t st)
{
    if (ns <= 0)
        return hipSuccess;
    if (a.rpt != 1)
        return hipErrorInvalidValue;
    const int nthr = hpsi_threads(a.geo.nx, a.TY, 1);
    const size_t lds = hpsi_lds_bytes(a.geo.nx, a.TY, a.zchunk, false);
    dim3 grid((unsigned)(a.ntile_y * a.nzc * ns));
    using D2 = double2;
    switch (hpsi_halo_per_thread(a.geo, a.TY, nthr)) {
    case 2:
        hipLaunchKernelGGL((k_hpsi<double, D2, D2, kCurrent, true, 2, 1>),
                           grid, dim3(nthr), lds, st, a);
        break;
    case 4:
        hipLaunchKernelGGL((k_hpsi<double, D2, D2, kCurrent, true, 4, 1>),
                           grid, dim3(nthr), lds, st, a);
        break;
    case 8:
        hipLaunchKernelGGL((k_hpsi<double, D2, D2, kCurrent, true, 8, 1>),
                           grid, dim3(nthr), lds, st, a);
        break;
    default:
        hipLaunchKernelGGL((k_hpsi<double, D2, D2, kCurrent, true, 16, 1>),
                           grid, dim3(nthr), lds, st, a);
        break;
    }
    return hipGetLastError();
}
#else
hipError_t launch_hpsi_mixed(int mode, bool in_is_f64, const HArgs &a, int ns,
                             hipStream_t st)
{
    if (in_is_f64) {
        switch (mode) {
        case kApply: return go_hpsi<float, double2, float2, kApply>(a, ns, st);
        case kTerm: return go_hpsi<float, double2, float2, kTerm>(a, ns, st);
        default: break;
        }
    } else {
        switch (mode) {
        case kTerm: return go_hpsi<float, float2, float2, kTerm>(a, ns, st);
        case kFinal: return go_hpsi<float, float2, float2, kFinal>(a, ns, st);
        case kFinalPred:
            return go_hpsi<float, float2, float2, kFinalPred>(a, ns, st);
        default: break;
        }
    }
    return hipErrorInvalidValue;
}
#endif

}  // namespace ks
