// Hartree potential on gfx950: the Poisson equation Lap v_H = -4 pi n
// solved as one product with a fixed real kernel in Fourier space.
//
//  - Finite grid (free space): v_H(r_i) = h^3 sum_j n_j G(r_i - r_j),
//    G(r) = 1/|r|, G(0) = the mean of 1/|r| over one grid cell.  Zero
//    padding to M_a >= 2 n_a - 1 per axis (the smallest product of 2, 3
//    and 5) makes the cyclic convolution of the padded arrays equal to this
//    sum (offsets span -(n-1) .. n-1), so
//    K = h^3 DFT(G sampled at the wrapped offsets) / (Mx My Mz).
//  - Periodic grid: K = 4 pi / |G|^2 / (Mx My Mz), G = 2 pi k / L, K(0) = 0
//    (uniform compensating background).
//
// One solve is five launches over a work array of nz planes of My x
// (Mx/2 + 1) complex values (the density is real, so along x only the half
// spectrum k <= Mx/2 is kept): x forward (two density rows per complex
// line, zero padded, split into the rows' half spectra), y forward (only
// the nz planes that hold density), z forward + product with K + z inverse
// in one launch (lines of the z axis; only z < nz is read or written back),
// y inverse (keeping y < ny), x inverse (two rows per line rebuilt from
// their half spectra; the real and imaginary parts are the two rows of v,
// x < nx).  Lines that would transform zeros are never touched.
//
// Each 1D transform is a mixed-radix Stockham FFT (radices 16, 8, 4, 2, 3,
// 5; the 8- and 16-point butterflies are computed in registers from 2- and
// 4-point ones, so a length of 128 or 256 takes two stages) of NL whole
// lines held in LDS as [point][line] with a padded row (NL + 1 complex
// values: the 16-byte accesses of consecutive lines fall in distinct
// banks), ping-ponging between two buffers, one barrier per stage.
// Along y and z the NL lines are NL consecutive x positions, so every global
// access moves NL * 16 contiguous bytes; along x the lines are whole rows.
#include "ks_poisson.h"

#include "ks_device.h"

#include <algorithm>
#include <cmath>
#include <vector>

namespace ks {
namespace {

constexpr int kFftThreads = 256;

// Paired kinds work on two real rows per complex line (rows 2l and 2l + 1
// of the density / potential, the second one absent past the last row):
// kFromDensityPair loads rho_a + i rho_b; kToWorkUnpack splits the
// transform into the two rows' half spectra (k <= M/2, by Hermitian
// symmetry); kFromWorkPair rebuilds the full spectrum of X_a + i X_b from
// the two half spectra; kToPotentialPair writes Re to row a, Im to row b.
enum InKind : int { kFromWork = 0, kFromDensityPair = 1, kFromGreen = 2,
                    kFromWorkPair = 3 };
enum OutKind : int { kToWork = 0, kToPotentialPair = 1,
                     kToPotentialPairAdd = 2, kToWorkUnpack = 3 };
enum Op : int { kForward = 0, kInverse = 1, kConvolve = 2 };

// One launch: lines l = a + la * b (l < nlines) of the work array, line
// element i at a * sa + b * sb + i * sp.  In the paired x passes line l
// holds rows r = 2l and 2l + 1 (r < nrows) of the density / potential
// (length nrow each), whose work rows sit at (r % la) * sa + (r / la) * sb.
struct LinePass {
    FftAxis ax;
    int nlines = 0, la = 1, nrows = 0;
    long sa = 0, sb = 0, sp = 1;
    int nin = 0, nout = 0;          // points read (rest zero) / written
    int in_kind = kFromWork, out_kind = kToWork, op = kForward;
    double2 *work = nullptr;
    const double *rho = nullptr;
    double *v = nullptr;
    int nrow = 0;
    // kFromGreen: G at the wrapped offsets of an M[0] x M[1] x M[2] grid
    int Mg[3] = {1, 1, 1};
    double hg[3] = {1.0, 1.0, 1.0};
    double g0 = 0.0;
    // kConvolve: line a is kx, line b is ky; K octant of Mx x My x M
    const double *K = nullptr;
    int Kx = 1, Ky = 1;
};

__device__ __forceinline__ double2 conj_if(double2 w, bool c)
{
    if (c)
        w.y = -w.y;
    return w;
}

// 4-point DFT of (a0, a1, a2, a3) into y0..y3 (w_4 = -i forward, +i
// inverse).
__device__ __forceinline__ void dft4(double2 a0, double2 a1, double2 a2,
                                     double2 a3, double2 &y0, double2 &y1,
                                     double2 &y2, double2 &y3, bool inv)
{
    const double2 s02 = cadd(a0, a2), d02 = csub(a0, a2);
    const double2 s13 = cadd(a1, a3), d13 = csub(a1, a3);
    const double2 r = inv ? cmk<double2>(-d13.y, d13.x)
                          : cmk<double2>(d13.y, -d13.x);
    y0 = cadd(s02, s13);
    y2 = csub(s02, s13);
    y1 = cadd(d02, r);
    y3 = csub(d02, r);
}

// x * w_16^m (conjugated root for the inverse); m is a constant after
// unrolling.  cos and sin of 2 pi m / 16 from cos(pi/8), sin(pi/8), 1/sqrt2.
__device__ __forceinline__ double2 mul_w16(double2 x, int m, bool inv)
{
    constexpr double c1 = 0.92387953251128675613, s1 = 0.38268343236508977173;
    constexpr double r2 = 0.70710678118654752440;
    constexpr double C[16] = {1, c1, r2, s1, 0, -s1, -r2, -c1,
                              -1, -c1, -r2, -s1, 0, s1, r2, c1};
    constexpr double S[16] = {0, s1, r2, c1, 1, c1, r2, s1,
                              0, -s1, -r2, -c1, -1, -c1, -r2, -s1};
    const int mm = m & 15;
    if (mm == 0)
        return x;
    return cmul(x, cmk<double2>(C[mm], inv ? S[mm] : -S[mm]));
}

// y = DFT_P(c).  P = 8 and 16 are composed of 2- and 4-point DFTs with the
// inner roots of unity (q = 4 q1 + q2, u = u1 + (P/4) u2):
//   DFT_P(c)[u] = DFT_4 over q2 of ( w_P^{u1 q2} DFT_{P/4} over q1 of
//                 c[4 q1 + q2] )[u1].
// P = 3 and 5 take their roots from the twiddle table (w_P^m =
// tw[m * M / P]; conjugated for the inverse transform).
template <int P>
__device__ __forceinline__ void small_dft(const double2 (&c)[P],
                                          double2 (&y)[P],
                                          const double2 *__restrict__ tw,
                                          int M, bool inv)
{
    if constexpr (P == 2) {
        y[0] = cadd(c[0], c[1]);
        y[1] = csub(c[0], c[1]);
    } else if constexpr (P == 4) {
        dft4(c[0], c[1], c[2], c[3], y[0], y[1], y[2], y[3], inv);
    } else if constexpr (P == 8) {
        double2 z[4][2];
#pragma unroll
        for (int q2 = 0; q2 < 4; ++q2) {
            z[q2][0] = cadd(c[q2], c[4 + q2]);
            z[q2][1] = mul_w16(csub(c[q2], c[4 + q2]), 2 * q2, inv);
        }
#pragma unroll
        for (int u1 = 0; u1 < 2; ++u1)
            dft4(z[0][u1], z[1][u1], z[2][u1], z[3][u1], y[u1], y[u1 + 2],
                 y[u1 + 4], y[u1 + 6], inv);
    } else if constexpr (P == 16) {
        double2 z[4][4];
#pragma unroll
        for (int q2 = 0; q2 < 4; ++q2) {
            dft4(c[q2], c[4 + q2], c[8 + q2], c[12 + q2], z[q2][0], z[q2][1],
                 z[q2][2], z[q2][3], inv);
#pragma unroll
            for (int u1 = 1; u1 < 4; ++u1)
                z[q2][u1] = mul_w16(z[q2][u1], u1 * q2, inv);
        }
#pragma unroll
        for (int u1 = 0; u1 < 4; ++u1)
            dft4(z[0][u1], z[1][u1], z[2][u1], z[3][u1], y[u1], y[u1 + 4],
                 y[u1 + 8], y[u1 + 12], inv);
    } else {
        const int step = M / P;
#pragma unroll
        for (int u = 0; u < P; ++u) {
            double2 acc = c[0];
#pragma unroll
            for (int q = 1; q < P; ++q)
                acc = cadd(acc, cmul(c[q], conj_if(tw[((u * q) % P) * step],
                                                   inv)));
            y[u] = acc;
        }
    }
}

// One Stockham stage of radix P on NL lines: sub-transforms of length L
// (stored as X[j][k], j < L, k < r P, at j r P + k) combine into
// transforms of length L P (X'[j + L u][k'] at (j + L u) r + k', k' < r):
//   X'[j + L u][k'] = sum_q w_P^{u q} w_{L P}^{j q} X[j][k' + r q].
template <int P, int NL>
__device__ __forceinline__ void fft_stage(const double2 *__restrict__ A,
                                          double2 *__restrict__ B, int M,
                                          int L, int r,
                                          const double2 *__restrict__ tw,
                                          bool inv)
{
    constexpr int PS = NL + 1;
    constexpr int bstep = kFftThreads / NL;   // butterflies per sweep
    const int tstep = M / (L * P);
    const int nb = L * r;
    // each thread keeps one line and walks the butterflies b = j r + k of
    // that line with stride bstep (one division per stage, no division in
    // the loop)
    const int l = threadIdx.x % NL;
    int b = threadIdx.x / NL;
    int j = b / r, k = b - j * r;
    const int dj = bstep / r, dk = bstep - dj * r;
    for (; b < nb; b += bstep) {
        double2 c[P], y[P];
#pragma unroll
        for (int q = 0; q < P; ++q) {
            const double2 x = A[(j * r * P + k + r * q) * PS + l];
            c[q] = q == 0 ? x : cmul(x, conj_if(tw[j * q * tstep], inv));
        }
        small_dft<P>(c, y, tw, M, inv);
#pragma unroll
        for (int u = 0; u < P; ++u)
            B[((j + L * u) * r + k) * PS + l] = y[u];
        j += dj;
        k += dk;
        if (k >= r) {
            k -= r;
            ++j;
        }
    }
}

// Transform the NL lines in A (B is scratch); returns the buffer that holds
// the result.  Ends with a barrier.
template <int NL>
__device__ double2 *fft_lines(double2 *A, double2 *B, const FftAxis &ax,
                              const double2 *tw, bool inv)
{
    int L = 1, r = ax.M;
    for (int s = 0; s < ax.nst; ++s) {
        const int p = ax.rad[s];
        r /= p;
        switch (p) {
        case 16: fft_stage<16, NL>(A, B, ax.M, L, r, tw, inv); break;
        case 8: fft_stage<8, NL>(A, B, ax.M, L, r, tw, inv); break;
        case 4: fft_stage<4, NL>(A, B, ax.M, L, r, tw, inv); break;
        case 2: fft_stage<2, NL>(A, B, ax.M, L, r, tw, inv); break;
        case 3: fft_stage<3, NL>(A, B, ax.M, L, r, tw, inv); break;
        default: fft_stage<5, NL>(A, B, ax.M, L, r, tw, inv); break;
        }
        __syncthreads();
        double2 *t = A;
        A = B;
        B = t;
        L *= p;
    }
    return A;
}

__device__ __forceinline__ double green(const LinePass &p, int i, int a,
                                        int b)
{
    const int idx[3] = {i, a, b};
    double r2 = 0.0;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        const int M = p.Mg[d];
        const int off = 2 * idx[d] > M ? idx[d] - M : idx[d];
        const double x = off * p.hg[d];
        r2 += x * x;
    }
    return r2 > 0.0 ? 1.0 / sqrt(r2) : p.g0;
}

// Most (point, line) pairs one thread owns in a launch (NL M <= 256 x this).
constexpr int kMaxPts = 12;

// The (point i, line li) pairs of the NL lines that this thread owns, in
// the order that makes global accesses contiguous: along i for whole rows,
// along li (x positions) otherwise.  All of a thread's loads are issued
// before any of them is used.
struct Points {
    int i[kMaxPts], li[kMaxPts];
    bool ok[kMaxPts];
};

template <int NL>
__device__ __forceinline__ void own_points(int M, bool rows, Points &q)
{
    if (rows) {
        int i = threadIdx.x % M, li = threadIdx.x / M;
        const int di = kFftThreads % M, dli = kFftThreads / M;
#pragma unroll
        for (int n = 0; n < kMaxPts; ++n) {
            q.i[n] = i;
            q.li[n] = li;
            q.ok[n] = li < NL;
            i += di;
            li += dli;
            if (i >= M) {
                i -= M;
                ++li;
            }
        }
    } else {
        const int li = threadIdx.x % NL, i0 = threadIdx.x / NL;
#pragma unroll
        for (int n = 0; n < kMaxPts; ++n) {
            q.i[n] = i0 + n * (kFftThreads / NL);
            q.li[n] = li;
            q.ok[n] = q.i[n] < M;
        }
    }
}

template <int NL>
__global__ __launch_bounds__(kFftThreads) void k_fft_lines(LinePass p)
{
    extern __shared__ double2 lds[];
    __shared__ long lbase[NL];     // work-array offset of each line
    __shared__ long lbase1[NL];    // paired: offset of the second row
    __shared__ int lcoord[NL][2];  // its (a, b); a < 0: past the last line
    __shared__ int lpair[NL];      // paired: the second row exists
    constexpr int PS = NL + 1;
    const int M = p.ax.M;
    double2 *A = lds, *B = lds + (size_t)M * PS;
    double2 *tw = B + (size_t)M * PS;   // the twiddle table, M values
    const int l0 = blockIdx.x * NL;
    const bool rows = p.sp == 1;   // whole contiguous lines (x axis)
    for (int m = threadIdx.x; m < M; m += kFftThreads)
        tw[m] = p.ax.tw[m];
    const bool paired = p.in_kind == kFromDensityPair ||
                        p.in_kind == kFromWorkPair;
    if (threadIdx.x < NL) {
        const int l = l0 + threadIdx.x;
        if (paired) {
            const int r0 = 2 * l, r1 = 2 * l + 1;
            lbase[threadIdx.x] = (r0 % p.la) * p.sa + (r0 / p.la) * p.sb;
            lbase1[threadIdx.x] = (r1 % p.la) * p.sa + (r1 / p.la) * p.sb;
            lpair[threadIdx.x] = r1 < p.nrows;
            lcoord[threadIdx.x][0] = l < p.nlines ? 0 : -1;
            lcoord[threadIdx.x][1] = 0;
        } else {
            const int a = l % p.la, b = l / p.la;
            lbase[threadIdx.x] = a * p.sa + b * p.sb;
            lcoord[threadIdx.x][0] = l < p.nlines ? a : -1;
            lcoord[threadIdx.x][1] = b;
        }
    }
    __syncthreads();
    Points q;
    own_points<NL>(M, rows, q);
    {
        double2 val[kMaxPts];
#pragma unroll
        for (int n = 0; n < kMaxPts; ++n) {
            val[n] = cmk<double2>(0.0, 0.0);
            const int i = q.i[n], li = q.li[n];
            if (q.ok[n] && i < p.nin && lcoord[li][0] >= 0) {
                const long r0 = 2L * (l0 + li);
                if (p.in_kind == kFromWork) {
                    val[n] = p.work[lbase[li] + i * p.sp];
                } else if (p.in_kind == kFromDensityPair) {
                    val[n].x = p.rho[r0 * p.nrow + i];
                    if (lpair[li])
                        val[n].y = p.rho[(r0 + 1) * p.nrow + i];
                } else if (p.in_kind == kFromWorkPair) {
                    // Z_i = X_a,i + i X_b,i; past the half spectrum from
                    // X_{M-i} = conj(X_i) of each real row
                    const int h = M / 2 + 1;
                    const int m = i < h ? i : M - i;
                    const double2 xa = p.work[lbase[li] + m];
                    const double2 xb = lpair[li] ? p.work[lbase1[li] + m]
                                                 : cmk<double2>(0.0, 0.0);
                    val[n] = i < h ? cmk<double2>(xa.x - xb.y, xa.y + xb.x)
                                   : cmk<double2>(xa.x + xb.y, xb.x - xa.y);
                } else {
                    val[n].x = green(p, i, lcoord[li][0], lcoord[li][1]);
                }
            }
        }
#pragma unroll
        for (int n = 0; n < kMaxPts; ++n)
            if (q.ok[n])
                A[q.i[n] * PS + q.li[n]] = val[n];
    }
    __syncthreads();
    double2 *R = fft_lines<NL>(A, B, p.ax, tw, p.op == kInverse);
    if (p.op == kConvolve) {
        // lines of the z axis: the points are along li (x positions)
        const int hx = p.Kx / 2 + 1, hy = p.Ky / 2 + 1;
        const int li = threadIdx.x % NL;
        const int a = lcoord[li][0], b = lcoord[li][1];
        if (a >= 0) {
            const int kx = min(a, p.Kx - a), ky = min(b, p.Ky - b);
            const double *Kl = p.K + (long)ky * hx + kx;
            const long kstride = (long)hy * hx;
            for (int i = threadIdx.x / NL; i < M; i += kFftThreads / NL)
                R[i * PS + li] = cscale(R[i * PS + li],
                                        Kl[min(i, M - i) * kstride]);
        }
        __syncthreads();
        double2 *other = R == A ? B : A;
        R = fft_lines<NL>(R, other, p.ax, tw, true);
    }
#pragma unroll
    for (int n = 0; n < kMaxPts; ++n) {
        const int i = q.i[n], li = q.li[n];
        if (q.ok[n] && i < p.nout && lcoord[li][0] >= 0) {
            const double2 val = R[i * PS + li];
            const long r0 = 2L * (l0 + li);
            if (p.out_kind == kToWork) {
                p.work[lbase[li] + i * p.sp] = val;
            } else if (p.out_kind == kToWorkUnpack) {
                // the two real rows' spectra: (Z_i + conj Z_{M-i}) / 2 and
                // (Z_i - conj Z_{M-i}) / (2i)
                const double2 zm = R[((M - i) % M) * PS + li];
                p.work[lbase[li] + i] = cmk<double2>(0.5 * (val.x + zm.x),
                                                     0.5 * (val.y - zm.y));
                if (lpair[li])
                    p.work[lbase1[li] + i] =
                        cmk<double2>(0.5 * (val.y + zm.y),
                                     0.5 * (zm.x - val.x));
            } else if (p.out_kind == kToPotentialPair) {
                p.v[r0 * p.nrow + i] = val.x;
                if (lpair[li])
                    p.v[(r0 + 1) * p.nrow + i] = val.y;
            } else {
                p.v[r0 * p.nrow + i] += val.x;
                if (lpair[li])
                    p.v[(r0 + 1) * p.nrow + i] += val.y;
            }
        }
    }
}

// Lines per workgroup: both LDS buffers and the twiddles within 96 KiB, at
// most kMaxPts points per thread, and, down to 8 lines, at least one
// workgroup per CU.  (Groups of 4 lines leave most of the 256 threads idle
// in the 16-point stages; measured slower.)
int lines_per_group(int M, int nlines)
{
    int nl = 32;
    while (nl > 8 && (nlines + nl - 1) / nl < 256)
        nl /= 2;
    while (nl > 2 && ((2 * (size_t)M * (nl + 1) + M) * sizeof(double2) >
                          98304 ||
                      nl * M > kFftThreads * kMaxPts))
        nl /= 2;
    return nl;
}

hipError_t run_pass(const LinePass &p, hipStream_t st)
{
    if (p.nlines <= 0)
        return hipSuccess;
    const int nl = lines_per_group(p.ax.M, p.nlines);
    if (nl * p.ax.M > kFftThreads * kMaxPts)
        return hipErrorInvalidValue;   // more points than a thread holds
    // two line buffers and the twiddle table
    const size_t lds = (2 * (size_t)p.ax.M * (nl + 1) + p.ax.M) *
                       sizeof(double2);
    const dim3 grid((p.nlines + nl - 1) / nl), block(kFftThreads);
    switch (nl) {
    case 32: hipLaunchKernelGGL(k_fft_lines<32>, grid, block, lds, st, p);
        break;
    case 16: hipLaunchKernelGGL(k_fft_lines<16>, grid, block, lds, st, p);
        break;
    case 8: hipLaunchKernelGGL(k_fft_lines<8>, grid, block, lds, st, p);
        break;
    case 4: hipLaunchKernelGGL(k_fft_lines<4>, grid, block, lds, st, p);
        break;
    default: hipLaunchKernelGGL(k_fft_lines<2>, grid, block, lds, st, p);
        break;
    }
    return hipGetLastError();
}

// K octant from the transformed Green function T ([Mz][My][Mx]).
__global__ void k_kernel_extract(const double2 *T, int Mx, int My, int Mz,
                                 double scale, double *K)
{
    const int hx = Mx / 2 + 1, hy = My / 2 + 1, hz = Mz / 2 + 1;
    const long n = (long)hx * hy * hz;
    const long g = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= n)
        return;
    const int kx = (int)(g % hx), ky = (int)((g / hx) % hy);
    const int kz = (int)(g / ((long)hx * hy));
    K[g] = scale * T[((long)kz * My + ky) * Mx + kx].x;
}

// K octant of the periodic kernel 4 pi / |G|^2 (0 at G = 0).
__global__ void k_kernel_periodic(int Mx, int My, int Mz, double Lx,
                                  double Ly, double Lz, double scale,
                                  double *K)
{
    const int hx = Mx / 2 + 1, hy = My / 2 + 1, hz = Mz / 2 + 1;
    const long n = (long)hx * hy * hz;
    const long g = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= n)
        return;
    const int kx = (int)(g % hx), ky = (int)((g / hx) % hy);
    const int kz = (int)(g / ((long)hx * hy));
    const double gx = 2.0 * M_PI * kx / Lx, gy = 2.0 * M_PI * ky / Ly;
    const double gz = 2.0 * M_PI * kz / Lz;
    const double G2 = gx * gx + gy * gy + gz * gz;
    K[g] = G2 > 0.0 ? scale * 4.0 * M_PI / G2 : 0.0;
}

__global__ __launch_bounds__(256) void k_real_dot_partial(const double *a,
                                                          const double *b,
                                                          long N,
                                                          double *part)
{
    __shared__ double sbuf[4];
    const long g = (long)blockIdx.x * blockDim.x + threadIdx.x;
    double acc[1] = {g < N ? a[g] * b[g] : 0.0};
    block_sum<double, 1>(acc, sbuf);
    if (threadIdx.x == 0)
        part[blockIdx.x] = acc[0];
}

// Integral of 1/|r| over the box [0,a] x [0,b] x [0,c] (closed form).
double corner_box_integral(double a, double b, double c)
{
    const double R = std::sqrt(a * a + b * b + c * c);
    return b * c * std::log((a + R) / std::sqrt(b * b + c * c)) +
           c * a * std::log((b + R) / std::sqrt(c * c + a * a)) +
           a * b * std::log((c + R) / std::sqrt(a * a + b * b)) -
           0.5 * a * a * std::atan(b * c / (a * R)) -
           0.5 * b * b * std::atan(c * a / (b * R)) -
           0.5 * c * c * std::atan(a * b / (c * R));
}

bool factorize(int M, FftAxis *ax)
{
    if (M < 1 || M > kFftMaxLen)
        return false;
    int m = M, nst = 0;
    for (int p : {16, 8, 4, 2, 3, 5})
        while (m % p == 0) {
            if (nst == kFftMaxStages)
                return false;
            ax->rad[nst++] = p;
            m /= p;
        }
    if (m != 1)
        return false;
    ax->M = M;
    ax->nst = nst;
    return true;
}

}  // namespace

bool poisson_lengths(const Geo &g, bool periodic, int M[3])
{
    const int n[3] = {g.nx, g.ny, g.nz};
    for (int d = 0; d < 3; ++d) {
        if (periodic) {
            M[d] = n[d];
        } else {
            // smallest length >= 2 n - 1 with factors 2, 3, 5 only
            FftAxis ax;
            M[d] = std::max(1, 2 * n[d] - 1);
            while (M[d] <= kFftMaxLen && !factorize(M[d], &ax))
                ++M[d];
        }
    }
    for (int d = 0; d < 3; ++d) {
        FftAxis ax;
        if (!factorize(M[d], &ax))
            return false;
    }
    return true;
}

void poisson_plan_destroy(PoissonPlan *pp)
{
    for (int d = 0; d < 3; ++d) {
        if (pp->tw[d])
            (void)hipFree(pp->tw[d]);
        pp->tw[d] = nullptr;
    }
    if (pp->K)
        (void)hipFree(pp->K);
    pp->K = nullptr;
}

hipError_t poisson_plan_create(const Geo &g, bool periodic, PoissonPlan *pp,
                               hipStream_t st)
{
    int M[3];
    if (!poisson_lengths(g, periodic, M))
        return hipErrorInvalidValue;
    pp->periodic = periodic;
    hipError_t e;
    for (int d = 0; d < 3; ++d) {
        factorize(M[d], &pp->ax[d]);
        std::vector<double2> tw(M[d]);
        for (int m = 0; m < M[d]; ++m) {
            const double ang = 2.0 * M_PI * m / M[d];
            tw[m] = make_double2(std::cos(ang), -std::sin(ang));
        }
        e = hipMalloc(&pp->tw[d], sizeof(double2) * M[d]);
        if (e != hipSuccess)
            return e;
        e = hipMemcpyAsync(pp->tw[d], tw.data(), sizeof(double2) * M[d],
                           hipMemcpyHostToDevice, st);
        if (e != hipSuccess)
            return e;
        pp->ax[d].tw = pp->tw[d];
    }
    const int Mx = M[0], My = M[1], Mz = M[2];
    const long nK = (long)(Mx / 2 + 1) * (My / 2 + 1) * (Mz / 2 + 1);
    e = hipMalloc(&pp->K, sizeof(double) * nK);
    if (e != hipSuccess)
        return e;
    pp->work_elems = (size_t)g.nz * My * (Mx / 2 + 1);
    const double vol = (double)Mx * My * Mz;
    const int nb = (int)((nK + 255) / 256);
    if (periodic) {
        hipLaunchKernelGGL(k_kernel_periodic, dim3(nb), dim3(256), 0, st, Mx,
                           My, Mz, g.nx * g.h[0], g.ny * g.h[1],
                           g.nz * g.h[2], 1.0 / vol, pp->K);
        e = hipGetLastError();
        if (e != hipSuccess)
            return e;
        return hipStreamSynchronize(st);
    }
    // finite grid: transform G sampled on the full Mx x My x Mz grid
    double2 *T = nullptr;
    e = hipMalloc(&T, sizeof(double2) * (size_t)Mx * My * Mz);
    if (e != hipSuccess)
        return e;
    const double g0 = 8.0 * corner_box_integral(0.5 * g.h[0], 0.5 * g.h[1],
                                                0.5 * g.h[2]) /
                      (g.h[0] * g.h[1] * g.h[2]);
    LinePass p;
    p.work = T;
    // x: rows (y, z) of the full grid, G generated on the fly
    p.ax = pp->ax[0];
    p.nlines = My * Mz;
    p.la = My;
    p.sa = Mx;
    p.sb = (long)Mx * My;
    p.sp = 1;
    p.nin = p.nout = Mx;
    p.in_kind = kFromGreen;
    p.out_kind = kToWork;
    p.op = kForward;
    for (int d = 0; d < 3; ++d) {
        p.Mg[d] = M[d];
        p.hg[d] = g.h[d];
    }
    p.g0 = g0;
    e = run_pass(p, st);
    // y: lines (x, z)
    if (e == hipSuccess) {
        p.ax = pp->ax[1];
        p.nlines = Mx * Mz;
        p.la = Mx;
        p.sa = 1;
        p.sb = (long)Mx * My;
        p.sp = Mx;
        p.nin = p.nout = My;
        p.in_kind = kFromWork;
        e = run_pass(p, st);
    }
    // z: lines (x, y)
    if (e == hipSuccess) {
        p.ax = pp->ax[2];
        p.nlines = Mx * My;
        p.la = Mx;
        p.sa = 1;
        p.sb = Mx;
        p.sp = (long)Mx * My;
        p.nin = p.nout = Mz;
        e = run_pass(p, st);
    }
    if (e == hipSuccess) {
        const double h3 = g.h[0] * g.h[1] * g.h[2];
        hipLaunchKernelGGL(k_kernel_extract, dim3(nb), dim3(256), 0, st, T,
                           Mx, My, Mz, h3 / vol, pp->K);
        e = hipGetLastError();
    }
    const hipError_t es = hipStreamSynchronize(st);
    (void)hipFree(T);
    return e != hipSuccess ? e : es;
}

hipError_t launch_hartree(const PoissonPlan &pp, const Geo &g,
                          const double *rho, double *v, bool add,
                          double2 *work, hipStream_t st)
{
    const int Mx = pp.ax[0].M, My = pp.ax[1].M;
    const int Mh = Mx / 2 + 1;                 // half spectrum along x
    const long plane = (long)Mh * My;
    const int nrows = g.ny * g.nz;
    hipError_t e;
    LinePass p;
    p.work = work;
    p.rho = rho;
    p.v = v;
    p.nrow = g.nx;
    // x forward: density rows (y < ny, z < nz) two at a time, zero padded
    // to Mx, split into the two rows' half spectra
    p.ax = pp.ax[0];
    p.nlines = (nrows + 1) / 2;
    p.nrows = nrows;
    p.la = g.ny;
    p.sa = Mh;
    p.sb = plane;
    p.sp = 1;
    p.nin = g.nx;
    p.nout = Mh;
    p.in_kind = kFromDensityPair;
    p.out_kind = kToWorkUnpack;
    p.op = kForward;
    if ((e = run_pass(p, st)) != hipSuccess)
        return e;
    // y forward: lines (x < Mh, z < nz), rows y >= ny are zero
    p.ax = pp.ax[1];
    p.nlines = Mh * g.nz;
    p.la = Mh;
    p.sa = 1;
    p.sb = plane;
    p.sp = Mh;
    p.nin = g.ny;
    p.nout = My;
    p.in_kind = kFromWork;
    p.out_kind = kToWork;
    if ((e = run_pass(p, st)) != hipSuccess)
        return e;
    // z: forward, times K, inverse; planes z >= nz are zero on input and
    // not needed on output
    p.ax = pp.ax[2];
    p.nlines = Mh * My;
    p.la = Mh;
    p.sa = 1;
    p.sb = Mh;
    p.sp = plane;
    p.nin = p.nout = g.nz;
    p.op = kConvolve;
    p.K = pp.K;
    p.Kx = Mx;
    p.Ky = My;
    if ((e = run_pass(p, st)) != hipSuccess)
        return e;
    // y inverse, keeping y < ny
    p.ax = pp.ax[1];
    p.nlines = Mh * g.nz;
    p.la = Mh;
    p.sa = 1;
    p.sb = plane;
    p.sp = Mh;
    p.nin = My;
    p.nout = g.ny;
    p.op = kInverse;
    if ((e = run_pass(p, st)) != hipSuccess)
        return e;
    // x inverse, two rows at a time from their half spectra, keeping
    // x < nx: the real part is row a, the imaginary part row b
    p.ax = pp.ax[0];
    p.nlines = (nrows + 1) / 2;
    p.nrows = nrows;
    p.la = g.ny;
    p.sa = Mh;
    p.sb = plane;
    p.sp = 1;
    p.nin = Mx;
    p.nout = g.nx;
    p.in_kind = kFromWorkPair;
    p.out_kind = add ? kToPotentialPairAdd : kToPotentialPair;
    return run_pass(p, st);
}

hipError_t launch_real_dot_partial(const double *a, const double *b, long N,
                                   double *part, hipStream_t st)
{
    hipLaunchKernelGGL(k_real_dot_partial, dim3(density_blocks(N)),
                       dim3(256), 0, st, a, b, N, part);
    return hipGetLastError();
}

}  // namespace ks
