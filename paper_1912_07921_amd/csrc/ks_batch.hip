// Batched (multi-job) form: H.psi and projector launches over the work
// items of every job of a job table.
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

// ---------------------------------------------------------------------------
// Batched (multi-job) passes.  One launch covers the work items of every
// job of a batch: workgroup b takes launch indices b, b + G, b + 2G, ...
// (G, the grid size, a multiple of 8, so every index of one workgroup stays
// on its XCD; the host sizes G to the item count, so each workgroup
// usually takes one item) and decodes (job, item) from the job's item
// offset (the H.psi items remapped per XCD within each job, below).  The pointers of Taylor pass p (exponential
// e = (p-1)/4, term j = (p-1)%4 + 1) and the time of the pass come from the
// job table and the job's device step counter, so a captured step replays
// unchanged.
// ---------------------------------------------------------------------------
// The job table, item offsets, A(t) tables and step counters do not change
// while a batch kernel runs: read them through the constant address space
// (scalar loads into SGPRs, shared by the whole wavefront).
template <class T> using cptr_t = __attribute__((address_space(4))) const T *;
template <class T> __device__ __forceinline__ cptr_t<T> cp(const T *p)
{
    return (cptr_t<T>)p;
}

// a whole struct read through the constant address space
template <class T> __device__ __forceinline__ T cload(cptr_t<T> p)
{
    T v;
    __builtin_memcpy(&v, (const T *)p, sizeof(T));
    return v;
}

__device__ __forceinline__ int find_job(const int *off, int njobs, int item)
{
    int j = 0;
    while (j + 1 < njobs && item >= cp(off)[j + 1])
        ++j;
    return j;
}

// input of Taylor pass p: exponential 0 starts from psi, 1 from psi_half
__device__ __forceinline__ const void *pass_input(cptr_t<JobDev> J, int p)
{
    const int e = (p - 1) / 4, j = (p - 1) % 4 + 1;
    if (j == 1)
        return e == 0 ? (const void *)J->psi : (const void *)J->half;
    return J->t[j - 2];
}

// H.psi items: the launch-index range of every job starts at a multiple of
// 8 (its item count padded up), so launch index L of a job sits on XCD
// L % 8 = r % 8 with r = L - off[job]; each job's items are remapped within
// the job, giving every XCD a contiguous eighth of every job (neighbouring
// y-tiles share halo rows in that XCD's L2, and jobs of different cost load
// all XCDs alike).  Indices past the job's items are padding.
#ifndef KS_BATCH_REMAP
#define KS_BATCH_REMAP 1
#endif
template <class R, class InT, class TT, int MODE, bool GRAD, int HM, int RPT>
__global__ __launch_bounds__(512) void k_hpsi_batch(BArgs b)
{
    const int total = cp(b.off)[b.njobs];
    for (int L = blockIdx.x; L < total; L += gridDim.x) {
        const int jb = find_job(b.off, b.njobs, L);
        const cptr_t<JobDev> J = cp(b.jobs) + jb;
        // the pass's arguments stay in the constant address space (read by
        // scalar loads where used, like kernel arguments)
        const HArgs &a = *(const HArgs *)(cp(b.hargs) + 8 * jb + b.pass - 1);
        const int r = L - cp(b.off)[jb];
        const int n = a.ntile_y * a.nzc * J->stot;
        if (r >= n)
            continue;                      // padding (uniform per workgroup)
        const int item = KS_BATCH_REMAP ? xcd_remap(r, n) : r;
        const int e = (b.pass - 1) / 4;
        // A(t0 + (step + e) dt)
        const double4 Av = cload<double4>(cp(J->Atab) + 2 * *cp(J->step) + e);
        hpsi_item<R, InT, TT, MODE, GRAD, HM, RPT>(a, item, Av);
        __syncthreads();   // LDS is reused by the next item
    }
}

template <class R, class InT>
__global__ __launch_bounds__(256) void k_gather_batch(BArgs b)
{
    const int total = cp(b.off)[b.njobs];
    for (int L = blockIdx.x; L < total; L += gridDim.x) {
        const int jb = find_job(b.off, b.njobs, L);
        const cptr_t<JobDev> J = cp(b.jobs) + jb;
        GArgs a = cload<GArgs>(&J->g);
        a.in = pass_input(J, b.pass);
        int r = L - cp(b.off)[jb];
        const int ch = r % a.nchunk;
        r /= a.nchunk;
        const int ngrp = (a.ns + kGatherStates - 1) / kGatherStates;
        const int grp = r % ngrp;
        gather_item<R, InT>(a, r / ngrp, grp, ch);
    }
}

template <class R>
__global__ __launch_bounds__(256) void k_gather_finalize_batch(BArgs b)
{
    const int total = cp(b.off)[b.njobs];
    for (int L = blockIdx.x; L < total; L += gridDim.x) {
        const int jb = find_job(b.off, b.njobs, L);
        const GArgs g = cload<GArgs>(&(cp(b.jobs) + jb)->g);
        gather_finalize_item<R>(g,
                                (long)(L - cp(b.off)[jb]) * blockDim.x +
                                    threadIdx.x);
    }
}

template <class R>
__global__ __launch_bounds__(kApplyThreads) void k_kbapply_batch(BArgs b)
{
    const int total = cp(b.off)[b.njobs];
    for (int L = blockIdx.x; L < total; L += gridDim.x) {
        const int jb = find_job(b.off, b.njobs, L);
        const GArgs a = cload<GArgs>(&(cp(b.jobs) + jb)->g);
        const int r = L - cp(b.off)[jb];
        kbapply_item<R, KS_APPLY_SPW_SMALL>(a, r % a.pj.nhchunk,
                                            r / a.pj.nhchunk);
    }
}

#if KS_HPSI_PART == 0
__global__ void k_step_advance(int *const *steps, int njobs)
{
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j < njobs)
        *steps[j] += 1;
}

__global__ void k_step_set(int *const *steps, int njobs, const int *values)
{
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j < njobs)
        *steps[j] = values[j];
}

int batch_items(int kind, const JobDev &J)
{
    switch (kind) {
    case kItemHpsi:
        return J.h.ntile_y * J.h.nzc * J.stot;
    case kItemGather:
        return J.g.pj.natoms > 0
                   ? J.g.pj.natoms *
                         ((J.stot + kGatherStates - 1) / kGatherStates) *
                         J.g.nchunk
                   : 0;
    case kItemGatherFin:
        return J.g.pj.natoms > 0
                   ? (int)(((long)J.stot * J.g.pj.natoms * kMaxProj + 255) /
                           256)
                   : 0;
    case kItemApply:
        return (J.g.pj.natoms > 0 && J.g.pj.nhull > 0)
                   ? J.g.pj.nhchunk *
                         apply_groups(J.stot, KS_APPLY_SPW_SMALL)
                   : 0;
    }
    return 0;
}

#endif

template <class R, class InT, class TT, int MODE, bool GRAD>
static hipError_t go_hpsi_batch(const BArgs &b, int hm, int rpt, int nthr,
                                size_t lds, int grid, hipStream_t st)
{
    if (rpt == 2) {
        if (hm <= 2)
            hipLaunchKernelGGL((k_hpsi_batch<R, InT, TT, MODE, GRAD, 2, 2>),
                               dim3(grid), dim3(nthr), lds, st, b);
        else if (hm <= 4)
            hipLaunchKernelGGL((k_hpsi_batch<R, InT, TT, MODE, GRAD, 4, 2>),
                               dim3(grid), dim3(nthr), lds, st, b);
        else
            hipLaunchKernelGGL((k_hpsi_batch<R, InT, TT, MODE, GRAD, 8, 2>),
                               dim3(grid), dim3(nthr), lds, st, b);
        return hipGetLastError();
    }
    switch (hm) {
    case 2:
        hipLaunchKernelGGL((k_hpsi_batch<R, InT, TT, MODE, GRAD, 2, 1>),
                           dim3(grid), dim3(nthr), lds, st, b);
        break;
    case 4:
        hipLaunchKernelGGL((k_hpsi_batch<R, InT, TT, MODE, GRAD, 4, 1>),
                           dim3(grid), dim3(nthr), lds, st, b);
        break;
    case 8:
        hipLaunchKernelGGL((k_hpsi_batch<R, InT, TT, MODE, GRAD, 8, 1>),
                           dim3(grid), dim3(nthr), lds, st, b);
        break;
    default:
        hipLaunchKernelGGL((k_hpsi_batch<R, InT, TT, MODE, GRAD, 16, 1>),
                           dim3(grid), dim3(nthr), lds, st, b);
        break;
    }
    return hipGetLastError();
}

template <class R, class InT, class TT, int MODE>
static hipError_t go_hpsi_batch_g(const BArgs &b, bool grad, int hm, int rpt,
                                  int nthr, size_t lds, int grid,
                                  hipStream_t st)
{
    return grad ? go_hpsi_batch<R, InT, TT, MODE, true>(b, hm, rpt, nthr,
                                                        lds, grid, st)
                : go_hpsi_batch<R, InT, TT, MODE, false>(b, hm, rpt, nthr,
                                                         lds, grid, st);
}

// Compiled twice like the single-grid H.psi file: part 0 holds the FP64
// pass kernels and everything else, part 1 the mixed-precision pass kernels.
hipError_t launch_pass_batch_mixed(const BArgs &b, bool grad, int hm, int rpt,
                                   int nthr, size_t lds, int grid,
                                   hipStream_t st);

#if KS_HPSI_PART == 0
hipError_t launch_pass_batch(bool mixed, const BArgs &b, bool grad, int hm,
                             int rpt, int nthr, size_t lds, int grid,
                             hipStream_t st)
{
    if (mixed)
        return launch_pass_batch_mixed(b, grad, hm, rpt, nthr, lds, grid, st);
    const int j = (b.pass - 1) % 4 + 1, e = (b.pass - 1) / 4;
    using D2 = double2;
    if (j < 4)
        return go_hpsi_batch_g<double, D2, D2, kTerm>(b, grad, hm, rpt, nthr,
                                                      lds, grid, st);
    return e == 0 ? go_hpsi_batch_g<double, D2, D2, kFinalPred>(
                        b, grad, hm, rpt, nthr, lds, grid, st)
                  : go_hpsi_batch_g<double, D2, D2, kFinal>(
                        b, grad, hm, rpt, nthr, lds, grid, st);
}
#else
hipError_t launch_pass_batch_mixed(const BArgs &b, bool grad, int hm, int rpt,
                                   int nthr, size_t lds, int grid,
                                   hipStream_t st)
{
    const int j = (b.pass - 1) % 4 + 1, e = (b.pass - 1) / 4;
    if (j == 1)
        return go_hpsi_batch_g<float, double2, float2, kTerm>(
            b, grad, hm, rpt, nthr, lds, grid, st);
    if (j < 4)
        return go_hpsi_batch_g<float, float2, float2, kTerm>(
            b, grad, hm, rpt, nthr, lds, grid, st);
    return e == 0 ? go_hpsi_batch_g<float, float2, float2, kFinalPred>(
                        b, grad, hm, rpt, nthr, lds, grid, st)
                  : go_hpsi_batch_g<float, float2, float2, kFinal>(
                        b, grad, hm, rpt, nthr, lds, grid, st);
}
#endif

#if KS_HPSI_PART == 0
hipError_t launch_projectors_batch(bool mixed, const BArgs &bg,
                                   const BArgs &bf, const BArgs &ba,
                                   int grid, hipStream_t st)
{
    const int j = (bg.pass - 1) % 4 + 1;
    const bool f64 = !mixed || j == 1;
    if (bg.off_total > 0) {
        if (!mixed)
            hipLaunchKernelGGL((k_gather_batch<double, double2>), dim3(grid),
                               dim3(256), 0, st, bg);
        else if (f64)
            hipLaunchKernelGGL((k_gather_batch<float, double2>), dim3(grid),
                               dim3(256), 0, st, bg);
        else
            hipLaunchKernelGGL((k_gather_batch<float, float2>), dim3(grid),
                               dim3(256), 0, st, bg);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess)
            return e;
    }
    if (bf.off_total > 0) {
        if (!mixed)
            hipLaunchKernelGGL((k_gather_finalize_batch<double>), dim3(grid),
                               dim3(256), 0, st, bf);
        else
            hipLaunchKernelGGL((k_gather_finalize_batch<float>), dim3(grid),
                               dim3(256), 0, st, bf);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess)
            return e;
    }
    if (ba.off_total > 0) {
        if (!mixed)
            hipLaunchKernelGGL((k_kbapply_batch<double>), dim3(grid),
                               dim3(kApplyThreads), 0, st, ba);
        else
            hipLaunchKernelGGL((k_kbapply_batch<float>), dim3(grid),
                               dim3(kApplyThreads), 0, st, ba);
        return hipGetLastError();
    }
    return hipSuccess;
}

hipError_t launch_step_advance(int *const *steps, int njobs, hipStream_t st)
{
    hipLaunchKernelGGL(k_step_advance, dim3((njobs + 63) / 64), dim3(64), 0,
                       st, steps, njobs);
    return hipGetLastError();
}

hipError_t launch_step_set(int *const *steps, int njobs, const int *values,
                           hipStream_t st)
{
    hipLaunchKernelGGL(k_step_set, dim3((njobs + 63) / 64), dim3(64), 0, st,
                       steps, njobs, values);
    return hipGetLastError();
}

#endif

}  // namespace ks
