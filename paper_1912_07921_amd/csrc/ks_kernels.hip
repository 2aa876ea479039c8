// Projector, density, dipole, norm, kick, Gram and exchange kernels and
// their launchers.
#include "ks_device.h"

#include <algorithm>

namespace ks {

template <class R, class InT>
__global__ __launch_bounds__(256) void k_gather(GArgs a)
{
    gather_item<R, InT>(a, blockIdx.x, blockIdx.y, blockIdx.z);
}

// The same work in the plane order of the work items: workgroup -> (state
// group, work item), consecutive work items (the chunks of one range of
// planes) of one state group on one XCD.  Used for launches large enough
// that the chunks of overlapping spheres would otherwise miss the L2.
template <class R, class InT>
__global__ __launch_bounds__(256) void k_gather_planes(GArgs a)
{
    const int L = xcd_remap(blockIdx.x, gridDim.x);
    const int grp = L / a.pj.ngpairs;
    const int *it = reinterpret_cast<const int *>(a.pj.gpairs) +
                    2 * (L - grp * a.pj.ngpairs);
    gather_item<R, InT>(a, gp(it)[0], grp, gp(it)[1]);
}

template <class R>
__global__ __launch_bounds__(256) void k_gather_finalize(GArgs a)
{
    gather_finalize_item<R>(a, (long)blockIdx.x * blockDim.x + threadIdx.x);
}

template <class R, int SPW>
__global__ __launch_bounds__(kApplyThreads) void k_kbapply(GArgs a)
{
    kbapply_item<R, SPW>(a, blockIdx.x, blockIdx.y);
}

// ---------------------------------------------------------------------------
// density: rho(g) = sum over sources in fixed order (density partials or
// weighted |psi|^2); optional v = v_ion + v_x(rho); optional dipole partials
// ---------------------------------------------------------------------------
constexpr int kDensThreads = 256;
#ifndef KS_DENS_U
#define KS_DENS_U 8
#endif
#ifndef KS_DENS_NT
#define KS_DENS_NT 1
#endif

// block blk of the density launch of `a` (sbuf: 3 doubles per wavefront)
__device__ __forceinline__ void density_block(const DArgs &a, long blk,
                                              double *sbuf)
{
    const Geo G = a.geo;
    const long g = blk * kDensThreads + threadIdx.x;
    double rho = 0.0;
    if (g < G.N) {
        // sources in order; U loads issued before their adds (the
        // partials are read once: non-temporal)
        constexpr int U = KS_DENS_U;
        int s = 0;
        if (a.npart) {
            const double *p = a.npart + g;
            for (; s + U <= a.nsrc; s += U) {
                double v[U];
#pragma unroll
                for (int u = 0; u < U; ++u)
                    v[u] = KS_DENS_NT ? __builtin_nontemporal_load(
                                            gp(p + (size_t)(s + u) * G.N))
                                      : p[(size_t)(s + u) * G.N];
#pragma unroll
                for (int u = 0; u < U; ++u)
                    rho += v[u];
            }
            for (; s < a.nsrc; ++s)
                rho += p[(size_t)s * G.N];
        } else {
            const double2 *p = a.psi + g;
            for (; s + U <= a.nsrc; s += U) {
                double2 v[U];
#pragma unroll
                for (int u = 0; u < U; ++u)
                    v[u] = p[(size_t)(s + u) * G.N];
#pragma unroll
                for (int u = 0; u < U; ++u)
                    rho += a.wocc[s + u] * (v[u].x * v[u].x + v[u].y * v[u].y);
            }
            for (; s < a.nsrc; ++s) {
                const double2 v = p[(size_t)s * G.N];
                rho += a.wocc[s] * (v.x * v.x + v.y * v.y);
            }
        }
        if (a.rho)
            a.rho[g] = rho;
        if (a.vout) {
            double vx = a.xc ? -cbrt(3.0 * rho / M_PI) : 0.0;
            a.vout[g] = a.vion[g] + vx;
        }
    }
    if (a.dpart) {
        double d[3] = {0.0, 0.0, 0.0};
        if (g < G.N) {
            int x = (int)(g % G.nx);
            int y = (int)((g / G.nx) % G.ny);
            int z = (int)(g / ((long)G.nx * G.ny));
            d[0] = axis_coord(G.nx, G.h[0], G.per[0], x) * rho;
            d[1] = axis_coord(G.ny, G.h[1], G.per[1], y) * rho;
            d[2] = axis_coord(G.nz, G.h[2], G.per[2], z) * rho;
        }
        block_sum<double, 3>(d, sbuf);
        if (threadIdx.x == 0)
            for (int c = 0; c < 3; ++c)
                a.dpart[(size_t)blk * 3 + c] = d[c];
    }
}

__global__ __launch_bounds__(kDensThreads) void k_density(DArgs a)
{
    __shared__ double sbuf[(kDensThreads / 64) * 3];
    density_block(a, blockIdx.x, sbuf);
}

// The densities of several grids in one launch: launch block L is block
// L - off[j] of job j (off[j] <= L < off[j + 1]), each computed exactly as
// k_density computes it.
__global__ __launch_bounds__(kDensThreads) void k_density_batch(
    const DArgs *args, const int *off, int njobs, int total)
{
    __shared__ double sbuf[(kDensThreads / 64) * 3];
    for (int L = blockIdx.x; L < total; L += gridDim.x) {
        int j = 0;
        while (j + 1 < njobs && L >= off[j + 1])
            ++j;
        const DArgs a = args[j];
        density_block(a, L - off[j], sbuf);
        __syncthreads();   // sbuf is reused by the next block
    }
}

// sum of nblocks dipole partials in fixed order, times h^3; with a device
// step counter, into out[3 * (step + 1) ...]
__device__ __forceinline__ void dipole_finalize_job(const double *dpart,
                                                    int nblocks, double h3,
                                                    double *out,
                                                    const int *step,
                                                    double *sbuf)
{
    if (step)
        out += 3 * (*step + 1);
    double d[3] = {0.0, 0.0, 0.0};
    for (int b = threadIdx.x; b < nblocks; b += blockDim.x)
        for (int c = 0; c < 3; ++c)
            d[c] += dpart[(size_t)b * 3 + c];
    block_sum<double, 3>(d, sbuf);
    if (threadIdx.x == 0)
        for (int c = 0; c < 3; ++c)
            out[c] = h3 * d[c];
}

__global__ __launch_bounds__(256) void k_dipole_finalize(const double *dpart,
                                                         int nblocks,
                                                         double h3,
                                                         double *out,
                                                         const int *step)
{
    __shared__ double sbuf[4 * 3];
    dipole_finalize_job(dpart, nblocks, h3, out, step, sbuf);
}

// one workgroup per job
__global__ __launch_bounds__(256) void k_dipole_finalize_batch(
    const DipJob *jobs)
{
    __shared__ double sbuf[4 * 3];
    const DipJob J = jobs[blockIdx.x];
    dipole_finalize_job(J.dpart, J.nblocks, J.h3, J.out, J.step, sbuf);
}

// per-state partial sums of |psi|^2 over chunks of the grid
__global__ __launch_bounds__(256) void k_norm_partial(Geo G,
                                                      const double2 *psi,
                                                      int nchunks,
                                                      double *part)
{
    __shared__ double sbuf[4];
    const int s = blockIdx.y;
    const long chunk = (G.N + nchunks - 1) / nchunks;
    const long b = (long)blockIdx.x * chunk;
    const long e = min(G.N, b + chunk);
    const double2 *p = psi + (size_t)s * G.N;
    double acc[1] = {0.0};
    for (long g = b + threadIdx.x; g < e; g += blockDim.x) {
        double2 v = p[g];
        acc[0] += v.x * v.x + v.y * v.y;
    }
    block_sum<double, 1>(acc, sbuf);
    if (threadIdx.x == 0)
        part[(size_t)s * nchunks + blockIdx.x] = acc[0];
}

__device__ __forceinline__ void norm_finalize_state(const double *part,
                                                    int ns, int ntiles,
                                                    double h3, double *out,
                                                    const int *step, int s,
                                                    double *sbuf, int *flag)
{
    if (step)
        out += (size_t)ns * (*step + 1);
    double acc[1] = {0.0};
    for (int t = threadIdx.x; t < ntiles; t += blockDim.x)
        acc[0] += part[(size_t)s * ntiles + t];
    block_sum<double, 1>(acc, sbuf);
    if (threadIdx.x == 0) {
        const double v = h3 * acc[0];
        out[s] = v;
        // every writer stores the same value, so the order does not matter
        if (flag && !isfinite(v))
            *flag = 1;
    }
}

__global__ __launch_bounds__(64) void k_norm_finalize(const double *part,
                                                      int ntiles, double h3,
                                                      double *out,
                                                      const int *step)
{
    __shared__ double sbuf[1];
    norm_finalize_state(part, gridDim.x, ntiles, h3, out, step, blockIdx.x,
                        sbuf, nullptr);
}

// state blockIdx.x of job blockIdx.y
__global__ __launch_bounds__(64) void k_norm_finalize_batch(
    const NormJob *jobs)
{
    __shared__ double sbuf[1];
    const NormJob J = jobs[blockIdx.y];
    if ((int)blockIdx.x >= J.ns)
        return;
    norm_finalize_state(J.part, J.ns, J.ntiles, J.h3, J.out, J.step,
                        blockIdx.x, sbuf, J.flag);
}

// psi <- exp(i kappa z) psi
__global__ __launch_bounds__(256) void k_kick(Geo G, double2 *psi,
                                              double kappa)
{
    const long g = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= G.N)
        return;
    const int z = (int)(g / ((long)G.nx * G.ny));
    double s, c;
    sincos(kappa * axis_coord(G.nz, G.h[2], G.per[2], z), &s, &c);
    double2 *p = psi + (size_t)blockIdx.y * G.N + g;
    double2 v = *p;
    double2 o;
    o.x = v.x * c - v.y * s;
    o.y = v.x * s + v.y * c;
    *p = o;
}

// ---------------------------------------------------------------------------
// Gram matrix partials on the FP64 matrix cores: part[ks][k][i][j] = sum
// over the ks-th slice of the grid of conj(psi_ki) psi_kj.  A workgroup
// (four wavefronts) owns a T x T tile of (i, j) (T = 64, or 32 for few
// states), each wavefront a T/2 x T/2 quarter as blocks of 16 x 16
// accumulated by
// v_mfma_f64_16x16x4f64 (D[16][16] += A[16][4] B[4][16], four grid points
// per instruction): Re G = Ar^T Ar + Ai^T Ai and Im G = Ar^T Ai - Ai^T Ar,
// with A the states' values at the points.  32 points of the tile's T + T
// states are staged through LDS per round (coalesced rows of 512 bytes).
// Operand layout on gfx950: lane l holds A[l % 16][l / 16] and
// B[l / 16][l % 16]; D[4 r + l / 16][l % 16] is element r of lane l's
// accumulator.
// ---------------------------------------------------------------------------
constexpr int kGK = 32;          // points per LDS stage

template <int kGT>
__global__ __launch_bounds__(256) void k_gram_partial(Geo G,
                                                      const double2 *psi,
                                                      int ns, int ksplit,
                                                      double2 *part)
{
    constexpr int B = kGT / 32;      // 16 x 16 blocks per wavefront side
    __shared__ double2 sa[kGT][kGK + 1];
    __shared__ double2 sb[kGT][kGK + 1];
    const int ntile = (ns + kGT - 1) / kGT;
    const int ti = blockIdx.x % ntile, tj = blockIdx.x / ntile;
    const int kk = blockIdx.y;
    const int ks = blockIdx.z;
    const long slice = (G.N + ksplit - 1) / ksplit;
    const long gb = ks * slice, ge = min(G.N, gb + slice);
    const double2 *pk = psi + (size_t)kk * ns * G.N;
    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    const int r0 = (wave >> 1) * (kGT / 2), c0 = (wave & 1) * (kGT / 2);
    const int li = lane & 15, lk = lane >> 4;
    gd4_t re[B][B], im[B][B];
#pragma unroll
    for (int u = 0; u < B; ++u)
#pragma unroll
        for (int w = 0; w < B; ++w) {
            re[u][w] = gd4_t{0.0, 0.0, 0.0, 0.0};
            im[u][w] = gd4_t{0.0, 0.0, 0.0, 0.0};
        }
    for (long g0 = gb; g0 < ge; g0 += kGK) {
#pragma unroll
        for (int u = 0; u < kGT / 8; ++u) {
            const int r = (tid >> 5) + 8 * u, c = tid & 31;   // kGK = 32
            const long g = g0 + c;
            const int si = ti * kGT + r, sj = tj * kGT + r;
            sa[r][c] = (si < ns && g < ge) ? pk[(size_t)si * G.N + g]
                                           : make_double2(0.0, 0.0);
            sb[r][c] = (sj < ns && g < ge) ? pk[(size_t)sj * G.N + g]
                                           : make_double2(0.0, 0.0);
        }
        __syncthreads();
#pragma unroll
        for (int k4 = 0; k4 < kGK; k4 += 4) {
            double2 a[B], b[B];
#pragma unroll
            for (int u = 0; u < B; ++u) {
                a[u] = sa[r0 + 16 * u + li][k4 + lk];
                b[u] = sb[c0 + 16 * u + li][k4 + lk];
            }
#pragma unroll
            for (int u = 0; u < B; ++u)
#pragma unroll
                for (int w = 0; w < B; ++w) {
                    re[u][w] = __builtin_amdgcn_mfma_f64_16x16x4f64(
                        a[u].x, b[w].x, re[u][w], 0, 0, 0);
                    re[u][w] = __builtin_amdgcn_mfma_f64_16x16x4f64(
                        a[u].y, b[w].y, re[u][w], 0, 0, 0);
                    im[u][w] = __builtin_amdgcn_mfma_f64_16x16x4f64(
                        a[u].x, b[w].y, im[u][w], 0, 0, 0);
                    im[u][w] = __builtin_amdgcn_mfma_f64_16x16x4f64(
                        -a[u].y, b[w].x, im[u][w], 0, 0, 0);
                }
        }
        __syncthreads();
    }
#pragma unroll
    for (int u = 0; u < B; ++u)
#pragma unroll
        for (int w = 0; w < B; ++w)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int i = ti * kGT + r0 + 16 * u + 4 * r + lk;
                const int j = tj * kGT + c0 + 16 * w + li;
                if (i < ns && j < ns)
                    part[(((size_t)ks * gridDim.y + kk) * ns + i) * ns + j] =
                        make_double2(re[u][w][r], im[u][w][r]);
            }
}

__global__ __launch_bounds__(256) void k_gram_finalize(const double2 *part,
                                                       long count, int ksplit,
                                                       double h3,
                                                       double2 *out)
{
    const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= count)
        return;
    double2 s = make_double2(0.0, 0.0);
    for (int k = 0; k < ksplit; ++k) {
        double2 v = part[(size_t)k * count + i];
        s.x += v.x;
        s.y += v.y;
    }
    out[i] = make_double2(h3 * s.x, h3 * s.y);
}

// per-state partial sums of conj(a) b over chunks of the grid
__global__ __launch_bounds__(256) void k_dot_partial(Geo G, const double2 *a,
                                                     const double2 *b,
                                                     int nchunks,
                                                     double2 *part)
{
    __shared__ double sbuf[4 * 2];
    const int s = blockIdx.y;
    const long chunk = (G.N + nchunks - 1) / nchunks;
    const long gb = (long)blockIdx.x * chunk;
    const long ge = min(G.N, gb + chunk);
    const double2 *pa = a + (size_t)s * G.N, *pb = b + (size_t)s * G.N;
    double acc[2] = {0.0, 0.0};
    for (long g = gb + threadIdx.x; g < ge; g += blockDim.x) {
        double2 u = pa[g], v = pb[g];
        acc[0] += u.x * v.x + u.y * v.y;
        acc[1] += u.x * v.y - u.y * v.x;
    }
    block_sum<double, 2>(acc, sbuf);
    if (threadIdx.x == 0)
        part[(size_t)s * nchunks + blockIdx.x] = make_double2(acc[0], acc[1]);
}

// partial sums of rho^(4/3) (exchange energy)
__global__ __launch_bounds__(256) void k_exchange_partial(Geo G,
                                                          const double *rho,
                                                          double *part)
{
    __shared__ double sbuf[4];
    const long g = (long)blockIdx.x * blockDim.x + threadIdx.x;
    double acc[1] = {0.0};
    if (g < G.N)
        acc[0] = pow(rho[g], 4.0 / 3.0);
    block_sum<double, 1>(acc, sbuf);
    if (threadIdx.x == 0)
        part[blockIdx.x] = acc[0];
}

int gather_chunks(int max_npts)
{
    return std::max(1, (max_npts + kGatherChunk - 1) / kGatherChunk);
}

int gather_chunk_points() { return kGatherChunk; }

// Gather launches of at least this many workgroups run in plane order
// (128^3 x 256 states, 64 atoms: 45k workgroups, 0.91 -> 0.83 ms; at 2.5k
// and 96 workgroups the plain order is 2-10 % faster).
constexpr long kGatherPlaneOrderMin = 8192;

hipError_t launch_gather(bool mixed, bool in_is_f64, const GArgs &a, int ns,
                         hipStream_t st)
{
    if (ns <= 0 || a.pj.natoms <= 0)
        return hipSuccess;
    GArgs b = a;
    b.ns = ns;
    const int ngrp = (ns + kGatherStates - 1) / kGatherStates;
    const long nblk = (long)a.pj.ngpairs * ngrp;
    dim3 blk(256);
    if (nblk >= kGatherPlaneOrderMin && nblk <= 0x7fffffffL) {
        dim3 grid((unsigned)nblk);
        if (!mixed)
            hipLaunchKernelGGL((k_gather_planes<double, double2>), grid, blk,
                               0, st, b);
        else if (in_is_f64)
            hipLaunchKernelGGL((k_gather_planes<float, double2>), grid, blk,
                               0, st, b);
        else
            hipLaunchKernelGGL((k_gather_planes<float, float2>), grid, blk,
                               0, st, b);
    } else {
        dim3 grid(a.pj.natoms, ngrp, a.nchunk);
        if (!mixed)
            hipLaunchKernelGGL((k_gather<double, double2>), grid, blk, 0, st,
                               b);
        else if (in_is_f64)
            hipLaunchKernelGGL((k_gather<float, double2>), grid, blk, 0, st,
                               b);
        else
            hipLaunchKernelGGL((k_gather<float, float2>), grid, blk, 0, st,
                               b);
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess)
        return e;
    const long total = (long)ns * a.pj.natoms * kMaxProj;
    dim3 g2((unsigned)((total + 255) / 256));
    if (!mixed)
        hipLaunchKernelGGL((k_gather_finalize<double>), g2, dim3(256), 0, st,
                           b);
    else
        hipLaunchKernelGGL((k_gather_finalize<float>), g2, dim3(256), 0, st,
                           b);
    return hipGetLastError();
}

hipError_t launch_kbapply(bool mixed, const GArgs &a, int ns, hipStream_t st)
{
    if (ns <= 0 || a.pj.natoms <= 0 || a.pj.nhull <= 0)
        return hipSuccess;
    GArgs b = a;
    b.ns = ns;
    const int spw = apply_spw(ns, mixed);
    dim3 grid(a.pj.nhchunk, apply_groups(ns, spw));
    constexpr int SL = KS_APPLY_SPW_LARGE, SS = KS_APPLY_SPW_SMALL,
                  SL32 = KS_APPLY_SPW_LARGE32;
    if (!mixed && spw == SL)
        hipLaunchKernelGGL((k_kbapply<double, SL>), grid,
                           dim3(kApplyThreads), 0, st, b);
    else if (!mixed)
        hipLaunchKernelGGL((k_kbapply<double, SS>), grid,
                           dim3(kApplyThreads), 0, st, b);
    else if (spw == SL32)
        hipLaunchKernelGGL((k_kbapply<float, SL32>), grid,
                           dim3(kApplyThreads), 0, st, b);
    else
        hipLaunchKernelGGL((k_kbapply<float, SS>), grid, dim3(kApplyThreads),
                           0, st, b);
    return hipGetLastError();
}

// he_p[e][j] = p_j (without N_j) of entry e's atom at its sphere point, by
// the gather's own evaluation (the same point image, the same shapes).
__global__ __launch_bounds__(256) void k_hull_table(ProjDev pj, Geo G,
                                                    const int2 *ent,
                                                    long nent, double *he_p)
{
    const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= nent)
        return;
    const int2 ai = ent[e];
    const int at = ai.x;
    const long ip = gp(pj.ioff)[at] + ai.y;
    const int pk = gp(pj.sxyz)[ip];
    const int code = gp(pj.sshift)[ip];
    const int ix = pk & 0x3ff, iy = (pk >> 10) & 0x3ff, iz = pk >> 20;
    const int tx = (int)(signed char)(code & 0xff);
    const int ty = (int)(signed char)((code >> 8) & 0xff);
    const int tz = (int)(signed char)((code >> 16) & 0xff);
    const double4 ap = gld(pj.apos + at);
    const double2 ar = gld(pj.arad + at);
    const double dx = axis_coord(G.nx, G.h[0], G.per[0], ix) +
                      tx * (G.nx * G.h[0]) - ap.x;
    const double dy = axis_coord(G.ny, G.h[1], G.per[1], iy) +
                      ty * (G.ny * G.h[1]) - ap.y;
    const double dz = axis_coord(G.nz, G.h[2], G.per[2], iz) +
                      tz * (G.nz * G.h[2]) - ap.z;
    double p[kMaxProj];
    proj_shape<double>(dx, dy, dz, dx * dx + dy * dy + dz * dz, ar,
                       gp(pj.nproj)[at], p);
#pragma unroll
    for (int j = 0; j < kMaxProj; ++j)
        he_p[e * kMaxProj + j] = p[j];
}

hipError_t launch_hull_table(const ProjDev &pj, const Geo &g,
                             const int2 *ent, long nent, double *he_p,
                             hipStream_t st)
{
    if (nent <= 0)
        return hipSuccess;
    hipLaunchKernelGGL(k_hull_table, dim3((unsigned)((nent + 255) / 256)),
                       dim3(256), 0, st, pj, g, ent, nent, he_p);
    return hipGetLastError();
}

// out[g] = sum_j w[j] src[j][g], j = 0 .. h-1 in order (potential
// extrapolation of the CFM4 propagator).
struct VComb {
    const double *src[4];
    double w[4];
};

__global__ __launch_bounds__(256) void k_vcombine(long N, int h, VComb c,
                                                  double *out)
{
    const long g = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= N)
        return;
    double s = 0.0;
    for (int j = 0; j < h; ++j)
        s += c.w[j] * c.src[j][g];
    out[g] = s;
}

hipError_t launch_vcombine(long N, int h, const double *const src[4],
                           const double w[4], double *out, hipStream_t st)
{
    if (h < 1 || h > 4)
        return hipErrorInvalidValue;
    VComb c;
    for (int j = 0; j < 4; ++j) {
        c.src[j] = j < h ? src[j] : nullptr;
        c.w[j] = j < h ? w[j] : 0.0;
    }
    hipLaunchKernelGGL(k_vcombine, dim3((unsigned)((N + 255) / 256)),
                       dim3(256), 0, st, N, h, c, out);
    return hipGetLastError();
}

int density_blocks(long N)
{
    return (int)((N + kDensThreads - 1) / kDensThreads);
}

hipError_t launch_density(const DArgs &a, hipStream_t st)
{
    hipLaunchKernelGGL(k_density, dim3(density_blocks(a.geo.N)),
                       dim3(kDensThreads), 0, st, a);
    return hipGetLastError();
}

hipError_t launch_density_batch(const DArgs *args, const int *blk_off,
                                int njobs, int nblocks, hipStream_t st)
{
    if (njobs <= 0 || nblocks <= 0)
        return hipSuccess;
    const int grid = std::min(nblocks, 1 << 22);
    hipLaunchKernelGGL(k_density_batch, dim3(grid), dim3(kDensThreads), 0, st,
                       args, blk_off, njobs, nblocks);
    return hipGetLastError();
}

hipError_t launch_dipole_finalize_batch(const DipJob *jobs, int njobs,
                                        hipStream_t st)
{
    if (njobs <= 0)
        return hipSuccess;
    hipLaunchKernelGGL(k_dipole_finalize_batch, dim3(njobs), dim3(256), 0, st,
                       jobs);
    return hipGetLastError();
}

hipError_t launch_norm_finalize_batch(const NormJob *jobs, int njobs,
                                      int max_ns, hipStream_t st)
{
    if (njobs <= 0 || max_ns <= 0)
        return hipSuccess;
    hipLaunchKernelGGL(k_norm_finalize_batch, dim3(max_ns, njobs), dim3(64), 0,
                       st, jobs);
    return hipGetLastError();
}

hipError_t launch_dipole_finalize(const double *dpart, int nblocks,
                                  double h3, double *out, hipStream_t st,
                                  const int *step)
{
    hipLaunchKernelGGL(k_dipole_finalize, dim3(1), dim3(256), 0, st, dpart,
                       nblocks, h3, out, step);
    return hipGetLastError();
}

hipError_t launch_norm_partial(const Geo &g, const double2 *psi, int ns,
                               int nchunks, double *normpart, hipStream_t st)
{
    if (ns <= 0)
        return hipSuccess;
    hipLaunchKernelGGL(k_norm_partial, dim3(nchunks, ns), dim3(256), 0, st, g,
                       psi, nchunks, normpart);
    return hipGetLastError();
}

hipError_t launch_norm_finalize(const double *normpart, int ns, int ntiles,
                                double h3, double *out, hipStream_t st,
                                const int *step)
{
    if (ns <= 0)
        return hipSuccess;
    hipLaunchKernelGGL(k_norm_finalize, dim3(ns), dim3(64), 0, st, normpart,
                       ntiles, h3, out, step);
    return hipGetLastError();
}

__global__ __launch_bounds__(256) void k_to_f32(const double *in, float *out,
                                               long n)
{
    const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n)
        out[i] = (float)in[i];
}

hipError_t launch_to_f32(const double *in, float *out, long n,
                         hipStream_t st)
{
    if (n <= 0)
        return hipSuccess;
    hipLaunchKernelGGL(k_to_f32, dim3((unsigned)((n + 255) / 256)), dim3(256),
                       0, st, in, out, n);
    return hipGetLastError();
}

__global__ __launch_bounds__(256) void k_to_f32_batch(const F32Copy *copies,
                                                     const int *blk_off,
                                                     int ncopies)
{
    int j = 0;
    while (j + 1 < ncopies && (int)blockIdx.x >= blk_off[j + 1])
        ++j;
    const F32Copy c = copies[j];
    const long i = (long)(blockIdx.x - blk_off[j]) * blockDim.x + threadIdx.x;
    if (i < c.n)
        c.dst[i] = (float)c.src[i];
}

hipError_t launch_to_f32_batch(const F32Copy *copies, const int *blk_off,
                               int ncopies, int nblocks, hipStream_t st)
{
    if (ncopies <= 0 || nblocks <= 0)
        return hipSuccess;
    hipLaunchKernelGGL(k_to_f32_batch, dim3((unsigned)nblocks), dim3(256), 0,
                       st, copies, blk_off, ncopies);
    return hipGetLastError();
}

hipError_t launch_kick(const Geo &g, double2 *psi, int ns, double kappa,
                       hipStream_t st)
{
    if (ns <= 0)
        return hipSuccess;
    dim3 grid((unsigned)((g.N + 255) / 256), ns);
    hipLaunchKernelGGL(k_kick, grid, dim3(256), 0, st, g, psi, kappa);
    return hipGetLastError();
}

hipError_t launch_gram(const Geo &g, const double2 *psi, int nk, int ns,
                       double2 *part, int ksplit, double2 *out,
                       hipStream_t st)
{
    const int T = gram_tile(ns);
    const int ntile = (ns + T - 1) / T;
    dim3 grid(ntile * ntile, nk, ksplit);
    if (T == 64)
        hipLaunchKernelGGL((k_gram_partial<64>), grid, dim3(256), 0, st, g,
                           psi, ns, ksplit, part);
    else
        hipLaunchKernelGGL((k_gram_partial<32>), grid, dim3(256), 0, st, g,
                           psi, ns, ksplit, part);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess)
        return e;
    const long count = (long)nk * ns * ns;
    double h3 = g.h[0] * g.h[1] * g.h[2];
    hipLaunchKernelGGL(k_gram_finalize, dim3((unsigned)((count + 255) / 256)),
                       dim3(256), 0, st, part, count, ksplit, h3, out);
    return hipGetLastError();
}

hipError_t launch_dot_partial(const Geo &g, const double2 *a,
                              const double2 *b, int ns, int nchunks,
                              double2 *part, hipStream_t st)
{
    if (ns <= 0)
        return hipSuccess;
    hipLaunchKernelGGL(k_dot_partial, dim3(nchunks, ns), dim3(256), 0, st, g,
                       a, b, nchunks, part);
    return hipGetLastError();
}

hipError_t launch_exchange_partial(const Geo &g, const double *rho,
                                   double *part, hipStream_t st)
{
    hipLaunchKernelGGL(k_exchange_partial, dim3(density_blocks(g.N)),
                       dim3(256), 0, st, g, rho, part);
    return hipGetLastError();
}

}  // namespace ks
