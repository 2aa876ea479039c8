// gfx950 kernels of the real-time TDDFT hot path.
//
// H.psi = -1/2 Lap psi + (v + |A|^2/2) psi - i A.grad psi + V_NL psi on a
// uniform grid (section "Periodic systems": finite-difference Laplacian and
// gradient; eq. Hamiltonian_dipole: one-body potential; section
// "Magneto-optics": non-local pseudopotentials; section "t-SURFF": uniform
// vector potential), applied to batches of resident states (sections "Memory
// layout" and "GPUs").
//
// Stencil design (HBM bound: 32 B moved per point and state in FP64):
//  - a workgroup owns a tile of full x-rows (nx x TY) of one state and marches
//    along z over a chunk of planes;
//  - each thread keeps the 9-deep z-column of its point in registers, so every
//    value is loaded from memory once per pass (plus the y-halo rows);
//  - the current xy plane (with 4 halo rows on each side) is staged in LDS for
//    the x and y neighbours; x-rows are read as consecutive 16-byte complex
//    values across the wavefront (coalesced);
//  - the KB scatter is fused into the single store of the output; the Taylor
//    recurrence scale, the final Taylor sum, the ETRS predictor and the
//    density/norm partial sums are fused into the epilogue.
#include "ks_internal.h"

#include <hip/hip_runtime.h>

namespace ks {

// Half-width-4 central weights: Laplacian (c0..c4) and gradient (d1..d4).
__constant__ double kLap[5] = {-205.0 / 72.0, 8.0 / 5.0, -1.0 / 5.0,
                               8.0 / 315.0, -1.0 / 560.0};
__constant__ double kGrad[5] = {0.0, 4.0 / 5.0, -1.0 / 5.0, 4.0 / 105.0,
                                -1.0 / 280.0};

template <class R> struct Cplx;
template <> struct Cplx<double> { using T = double2; };
template <> struct Cplx<float> { using T = float2; };

template <class V> __device__ __forceinline__ V czero()
{
    V r;
    r.x = 0;
    r.y = 0;
    return r;
}
template <class V> __device__ __forceinline__ V cmk(double a, double b)
{
    V r;
    r.x = a;
    r.y = b;
    return r;
}
template <class V> __device__ __forceinline__ V cadd(V a, V b)
{
    V r;
    r.x = a.x + b.x;
    r.y = a.y + b.y;
    return r;
}
template <class V> __device__ __forceinline__ V csub(V a, V b)
{
    V r;
    r.x = a.x - b.x;
    r.y = a.y - b.y;
    return r;
}
template <class V, class S> __device__ __forceinline__ V cscale(V a, S s)
{
    V r;
    r.x = a.x * s;
    r.y = a.y * s;
    return r;
}
template <class V> __device__ __forceinline__ V cmul(V a, V b)
{
    V r;
    r.x = a.x * b.x - a.y * b.y;
    r.y = a.x * b.y + a.y * b.x;
    return r;
}
// a * conj(b)
template <class V> __device__ __forceinline__ V cmulc(V a, V b)
{
    V r;
    r.x = a.x * b.x + a.y * b.y;
    r.y = a.y * b.x - a.x * b.y;
    return r;
}

template <class R, class T> __device__ __forceinline__ typename Cplx<R>::T
ldc(const T *p, long i)
{
    T v = p[i];
    typename Cplx<R>::T r;
    r.x = (R)v.x;
    r.y = (R)v.y;
    return r;
}

__device__ __forceinline__ int floordiv(int a, int n)
{
    return a >= 0 ? a / n : -((-a + n - 1) / n);
}

template <class R> __device__ __forceinline__ typename Cplx<R>::T
phase(double ang)
{
    double s, c;
    sincos(ang, &s, &c);
    return cmk<typename Cplx<R>::T>(c, s);
}

// Lattice shift packed as three signed bytes (x, y, z).
__device__ __forceinline__ double shift_angle(int code, const double *kL)
{
    int tx = (int)(signed char)(code & 0xff);
    int ty = (int)(signed char)((code >> 8) & 0xff);
    int tz = (int)(signed char)((code >> 16) & 0xff);
    return tx * kL[0] + ty * kL[1] + tz * kL[2];
}

// value at (x, y, z) with y in range, z possibly outside (boundary rule)
template <class R, class InT>
__device__ __forceinline__ typename Cplx<R>::T
load_z(const InT *st, const Geo &G, const double *kL, int x, int y, int z)
{
    using V = typename Cplx<R>::T;
    if ((unsigned)z < (unsigned)G.nz)
        return ldc<R>(st, ((long)z * G.ny + y) * G.nx + x);
    if (!G.per[2])
        return czero<V>();
    int w = floordiv(z, G.nz);
    int zz = z - w * G.nz;
    V v = ldc<R>(st, ((long)zz * G.ny + y) * G.nx + x);
    return cmul(v, phase<R>(w * kL[2]));
}

// value at (x, y, z) with z in range, y possibly outside
template <class R, class InT>
__device__ __forceinline__ typename Cplx<R>::T
load_y(const InT *st, const Geo &G, const double *kL, int x, int y, int z)
{
    using V = typename Cplx<R>::T;
    if ((unsigned)y < (unsigned)G.ny)
        return ldc<R>(st, ((long)z * G.ny + y) * G.nx + x);
    if (!G.per[1])
        return czero<V>();
    int w = floordiv(y, G.ny);
    int yy = y - w * G.ny;
    V v = ldc<R>(st, ((long)z * G.ny + yy) * G.nx + x);
    return cmul(v, phase<R>(w * kL[1]));
}

// neighbour along x within an LDS row (index possibly outside [0, nx))
template <class V, class R>
__device__ __forceinline__ V row_x(const V *row, int xi, int nx, int per,
                                   double kLx)
{
    if ((unsigned)xi < (unsigned)nx)
        return row[xi];
    if (!per)
        return czero<V>();
    int w = floordiv(xi, nx);
    return cmul(row[xi - w * nx], phase<R>(w * kLx));
}

template <class T> __device__ __forceinline__ T wave_sum(T v)
{
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1)
        v += __shfl_xor(v, off, 64);
    return v;
}

// Deterministic block reduction of NV values; result valid in thread 0.
template <class T, int NV>
__device__ __forceinline__ void block_sum(T (&v)[NV], T *sbuf)
{
    const int tid = threadIdx.x;
    const int nw = (blockDim.x + 63) >> 6;
#pragma unroll
    for (int i = 0; i < NV; ++i)
        v[i] = wave_sum(v[i]);
    if ((tid & 63) == 0)
#pragma unroll
        for (int i = 0; i < NV; ++i)
            sbuf[(tid >> 6) * NV + i] = v[i];
    __syncthreads();
    if (tid == 0)
        for (int i = 0; i < NV; ++i) {
            T s = 0;
            for (int w = 0; w < nw; ++w)
                s += sbuf[w * NV + i];
            v[i] = s;
        }
}

// ---------------------------------------------------------------------------
// H.psi with a fused epilogue.  R: arithmetic precision; InT: storage type of
// the input states; TT: storage type of t-terms (t1, t2, term outputs).
// ---------------------------------------------------------------------------
template <class R, class InT, class TT, int MODE>
__global__ __launch_bounds__(512) void k_hpsi(HArgs a)
{
    using V = typename Cplx<R>::T;
    extern __shared__ unsigned char smem_raw[];
    V *sp = reinterpret_cast<V *>(smem_raw);

    const Geo G = a.geo;
    const int nx = G.nx, ny = G.ny, nz = G.nz;
    const long N = G.N;
    const int tile = blockIdx.x;
    const int tile_y = tile % a.ntile_y;
    const int zc = tile / a.ntile_y;
    const int sl = blockIdx.y;
    const int sg = a.sg0 + sl;
    const int kk = sg / a.nstates;
    const double *kL = a.kL + 3 * kk;

    const int TY = a.TY;
    const int y0 = tile_y * TY;
    const int rows = min(TY, ny - y0);
    const int tid = threadIdx.x;
    const int x = tid % nx;
    const int yl = tid / nx;
    const bool act = yl < rows;
    const int y = y0 + (act ? yl : 0);
    const int z0 = zc * a.zchunk;
    const int z1 = min(nz, z0 + a.zchunk);

    const InT *in = reinterpret_cast<const InT *>(a.in) + (size_t)sl * N;
    const R ih2x = (R)(1.0 / (G.h[0] * G.h[0]));
    const R ih2y = (R)(1.0 / (G.h[1] * G.h[1]));
    const R ih2z = (R)(1.0 / (G.h[2] * G.h[2]));
    const R ihx = (R)(1.0 / G.h[0]), ihy = (R)(1.0 / G.h[1]),
            ihz = (R)(1.0 / G.h[2]);
    R LC[5], GD[5];
#pragma unroll
    for (int m = 0; m < 5; ++m) {
        LC[m] = (R)kLap[m];
        GD[m] = (R)kGrad[m];
    }
    const bool has_A = (a.A[0] != 0.0) || (a.A[1] != 0.0) || (a.A[2] != 0.0);
    const R Ax = (R)a.A[0], Ay = (R)a.A[1], Az = (R)a.A[2];
    const V cs = cmk<V>(a.cre, a.cim);
    const V *Dst = reinterpret_cast<const V *>(a.D) +
                   (size_t)sl * a.pj.natoms * kMaxProj;
    const double w_occ = (MODE == kFinal || MODE == kFinalPred)
                             ? a.wocc[sg] : 0.0;

    V q[2 * kHalf + 1];
#pragma unroll
    for (int m = 0; m < 2 * kHalf; ++m)
        q[m] = act ? load_z<R>(in, G, kL, x, y, z0 - kHalf + m)
                   : czero<V>();

    double nrm = 0.0;
    const int nthr = blockDim.x;
    const int row = yl + kHalf;

    for (int z = z0; z < z1; ++z) {
        q[2 * kHalf] = act ? load_z<R>(in, G, kL, x, y, z + kHalf)
                           : czero<V>();
        if (act)
            sp[row * nx + x] = q[kHalf];
        for (int e = tid; e < 2 * kHalf * nx; e += nthr) {
            int hr = e / nx, hx = e - hr * nx;
            int yy = hr < kHalf ? y0 - kHalf + hr : y0 + rows + (hr - kHalf);
            int lr = hr < kHalf ? hr : rows + hr;
            sp[lr * nx + hx] = load_y<R>(in, G, kL, hx, yy, z);
        }
        __syncthreads();
        if (act) {
            const V c = q[kHalf];
            const V *rp = sp + row * nx;
            V sx = czero<V>(), gx = czero<V>();
            if (x >= kHalf && x < nx - kHalf) {
#pragma unroll
                for (int m = 1; m <= kHalf; ++m) {
                    V p = rp[x + m], n = rp[x - m];
                    sx = cadd(sx, cscale(cadd(p, n), LC[m]));
                    gx = cadd(gx, cscale(csub(p, n), GD[m]));
                }
            } else {
#pragma unroll
                for (int m = 1; m <= kHalf; ++m) {
                    V p = row_x<V, R>(rp, x + m, nx, G.per[0], kL[0]);
                    V n = row_x<V, R>(rp, x - m, nx, G.per[0], kL[0]);
                    sx = cadd(sx, cscale(cadd(p, n), LC[m]));
                    gx = cadd(gx, cscale(csub(p, n), GD[m]));
                }
            }
            V sy = czero<V>(), gy = czero<V>();
#pragma unroll
            for (int m = 1; m <= kHalf; ++m) {
                V p = sp[(row + m) * nx + x], n = sp[(row - m) * nx + x];
                sy = cadd(sy, cscale(cadd(p, n), LC[m]));
                gy = cadd(gy, cscale(csub(p, n), GD[m]));
            }
            V sz = czero<V>(), gz = czero<V>();
#pragma unroll
            for (int m = 1; m <= kHalf; ++m) {
                V p = q[kHalf + m], n = q[kHalf - m];
                sz = cadd(sz, cscale(cadd(p, n), LC[m]));
                gz = cadd(gz, cscale(csub(p, n), GD[m]));
            }
            const long g = ((long)z * ny + y) * nx + x;
            // -1/2 Lap + (v + |A|^2/2)
            V lap = cadd(cadd(cscale(sx, ih2x), cscale(sy, ih2y)),
                         cscale(sz, ih2z));
            lap = cadd(lap, cscale(c, LC[0] * (ih2x + ih2y + ih2z)));
            const R vv = (R)(a.v[g] + a.a2half);
            V hp = cadd(cscale(lap, (R)-0.5), cscale(c, vv));
            if (has_A) {
                // -i A.grad
                V gr = cadd(cadd(cscale(gx, Ax * ihx), cscale(gy, Ay * ihy)),
                            cscale(gz, Az * ihz));
                hp.x += gr.y;
                hp.y -= gr.x;
            }
            if (a.pj.natoms > 0 && a.pj.rowhit[z * ny + y]) {
                const int e0 = a.pj.soff[g], e1 = a.pj.soff[g + 1];
                for (int e = e0; e < e1; ++e) {
                    const int2 en = a.pj.sent[e];
                    const int at = en.x, pt = en.y;
                    const int np = a.pj.nproj[at];
                    const int npt = a.pj.npts[at];
                    const long pb = a.pj.poff[at] + pt;
                    V acc = czero<V>();
                    const V *Da = Dst + at * kMaxProj;
                    for (int j = 0; j < np; ++j) {
                        R pv;
                        if constexpr (sizeof(R) == 8)
                            pv = a.pj.ptab[pb + (long)j * npt];
                        else
                            pv = a.pj.ptabf[pb + (long)j * npt];
                        acc = cadd(acc, cscale(Da[j], pv));
                    }
                    const int code = a.pj.sshift[a.pj.ioff[at] + pt];
                    if (code)
                        acc = cmulc(acc, phase<R>(shift_angle(code, kL)));
                    hp = cadd(hp, acc);
                }
            }
            if constexpr (MODE == kApply) {
                double2 o;
                o.x = hp.x;
                o.y = hp.y;
                reinterpret_cast<double2 *>(a.out)[(size_t)sl * N + g] = o;
            } else if constexpr (MODE == kTerm) {
                V t = cmul(cs, hp);
                TT o;
                o.x = t.x;
                o.y = t.y;
                reinterpret_cast<TT *>(a.out)[(size_t)sl * N + g] = o;
            } else {
                const V t4 = cmul(cs, hp);
                const size_t i = (size_t)sl * N + g;
                const double2 b = a.base[i];
                const TT u1 = reinterpret_cast<const TT *>(a.t1)[i];
                const TT u2 = reinterpret_cast<const TT *>(a.t2)[i];
                double re = b.x + (double)u1.x + (double)u2.x + (double)c.x +
                            (double)t4.x;
                double im = b.y + (double)u1.y + (double)u2.y + (double)c.y +
                            (double)t4.y;
                double2 o;
                o.x = re;
                o.y = im;
                reinterpret_cast<double2 *>(a.out)[i] = o;
                if constexpr (MODE == kFinalPred) {
                    double pr = b.x + 2.0 * u1.x + 4.0 * u2.x + 8.0 * c.x +
                                16.0 * (double)t4.x;
                    double pi = b.y + 2.0 * u1.y + 4.0 * u2.y + 8.0 * c.y +
                                16.0 * (double)t4.y;
                    if (a.npart)
                        a.npart[i] = w_occ * (pr * pr + pi * pi);
                } else {
                    const double sq = re * re + im * im;
                    if (a.npart)
                        a.npart[i] = w_occ * sq;
                    nrm += sq;
                }
            }
        }
        __syncthreads();
#pragma unroll
        for (int m = 0; m < 2 * kHalf; ++m)
            q[m] = q[m + 1];
    }
    if constexpr (MODE == kFinal) {
        if (!a.normpart)
            return;
        double vals[1] = {nrm};
        block_sum<double, 1>(vals, reinterpret_cast<double *>(smem_raw));
        if (tid == 0)
            a.normpart[(size_t)sl * (a.ntile_y * a.nzc) + tile] = vals[0];
    }
}

// ---------------------------------------------------------------------------
// KB projector gather: D[s][a][j] = h^3 E_{a,l(j)} sum_pt p~_j(pt) in_s(pt)
// One workgroup per (atom, state); fixed-order reduction (deterministic).
// ---------------------------------------------------------------------------
template <class R, class InT>
__global__ __launch_bounds__(256) void k_gather(GArgs a)
{
    using V = typename Cplx<R>::T;
    __shared__ R sbuf[(256 / 64) * 2 * kMaxProj];
    const int at = blockIdx.x;
    const int sl = blockIdx.y;
    const int sg = a.sg0 + sl;
    const int kk = sg / a.nstates;
    const double *kL = a.kL + 3 * kk;
    const InT *in = reinterpret_cast<const InT *>(a.in) + (size_t)sl * a.geo.N;
    const int np = a.pj.nproj[at];
    const int npt = a.pj.npts[at];
    const long io = a.pj.ioff[at];
    const long po = a.pj.poff[at];
    R acc[2 * kMaxProj];
#pragma unroll
    for (int j = 0; j < 2 * kMaxProj; ++j)
        acc[j] = 0;
    for (int pt = threadIdx.x; pt < npt; pt += blockDim.x) {
        V val = ldc<R>(in, a.pj.sidx[io + pt]);
        const int code = a.pj.sshift[io + pt];
        if (code)
            val = cmul(val, phase<R>(shift_angle(code, kL)));
#pragma unroll
        for (int j = 0; j < kMaxProj; ++j) {
            if (j < np) {
                R pv;
                if constexpr (sizeof(R) == 8)
                    pv = a.pj.ptab[po + (long)j * npt + pt];
                else
                    pv = a.pj.ptabf[po + (long)j * npt + pt];
                acc[2 * j] += pv * val.x;
                acc[2 * j + 1] += pv * val.y;
            }
        }
    }
    block_sum<R, 2 * kMaxProj>(acc, sbuf);
    if (threadIdx.x == 0) {
        V *D = reinterpret_cast<V *>(a.D) +
               ((size_t)sl * a.pj.natoms + at) * kMaxProj;
        for (int j = 0; j < kMaxProj; ++j) {
            R e = (j < np) ? (R)a.pj.Ej[at * kMaxProj + j] : (R)0;
            D[j] = cmk<V>(e * acc[2 * j], e * acc[2 * j + 1]);
        }
    }
}

// ---------------------------------------------------------------------------
// density: rho(g) = sum over sources in fixed order (density partials or
// weighted |psi|^2); optional v = v_ion + v_x(rho); optional dipole partials
// ---------------------------------------------------------------------------
constexpr int kDensThreads = 256;

__device__ __forceinline__ double axis_coord(int n, double h, int per, int i)
{
    return per ? i * h : (i - 0.5 * (n - 1)) * h;
}

__global__ __launch_bounds__(kDensThreads) void k_density(DArgs a)
{
    __shared__ double sbuf[(kDensThreads / 64) * 3];
    const Geo G = a.geo;
    const long g = (long)blockIdx.x * blockDim.x + threadIdx.x;
    double rho = 0.0;
    if (g < G.N) {
        if (a.npart) {
            for (int s = 0; s < a.nsrc; ++s)
                rho += a.npart[(size_t)s * G.N + g];
        } else {
            for (int s = 0; s < a.nsrc; ++s) {
                double2 v = a.psi[(size_t)s * G.N + g];
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
                a.dpart[(size_t)blockIdx.x * 3 + c] = d[c];
    }
}

// sum of nblocks dipole partials in fixed order, times h^3
__global__ __launch_bounds__(256) void k_dipole_finalize(const double *dpart,
                                                         int nblocks,
                                                         double h3,
                                                         double *out)
{
    __shared__ double sbuf[4 * 3];
    double d[3] = {0.0, 0.0, 0.0};
    for (int b = threadIdx.x; b < nblocks; b += blockDim.x)
        for (int c = 0; c < 3; ++c)
            d[c] += dpart[(size_t)b * 3 + c];
    block_sum<double, 3>(d, sbuf);
    if (threadIdx.x == 0)
        for (int c = 0; c < 3; ++c)
            out[c] = h3 * d[c];
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

__global__ __launch_bounds__(64) void k_norm_finalize(const double *part,
                                                      int ntiles, double h3,
                                                      double *out)
{
    __shared__ double sbuf[1];
    const int s = blockIdx.x;
    double acc[1] = {0.0};
    for (int t = threadIdx.x; t < ntiles; t += blockDim.x)
        acc[0] += part[(size_t)s * ntiles + t];
    block_sum<double, 1>(acc, sbuf);
    if (threadIdx.x == 0)
        out[s] = h3 * acc[0];
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
// Gram matrix partials: part[ks][k][i][j] = sum over the ks-th slice of the
// grid of conj(psi_ki) psi_kj; 32 x 32 state tiles staged through LDS.
// ---------------------------------------------------------------------------
constexpr int kGT = 32;   // state tile
constexpr int kGK = 32;   // points per LDS stage

__global__ __launch_bounds__(256) void k_gram_partial(Geo G,
                                                      const double2 *psi,
                                                      int ns, int ksplit,
                                                      double2 *part)
{
    __shared__ double2 sa[kGT][kGK + 1];
    __shared__ double2 sb[kGT][kGK + 1];
    const int ntile = (ns + kGT - 1) / kGT;
    const int ti = blockIdx.x % ntile, tj = blockIdx.x / ntile;
    const int kk = blockIdx.y;
    const int ks = blockIdx.z;
    const long slice = (G.N + ksplit - 1) / ksplit;
    const long gb = ks * slice, ge = min(G.N, gb + slice);
    const double2 *pk = psi + (size_t)kk * ns * G.N;
    const int tx = threadIdx.x % 16, ty = threadIdx.x / 16;
    double2 acc[2][2];
    for (int u = 0; u < 2; ++u)
        for (int w = 0; w < 2; ++w)
            acc[u][w] = make_double2(0.0, 0.0);
    for (long g0 = gb; g0 < ge; g0 += kGK) {
        for (int e = threadIdx.x; e < kGT * kGK; e += blockDim.x) {
            int r = e / kGK, c = e % kGK;
            long g = g0 + c;
            int si = ti * kGT + r, sj = tj * kGT + r;
            sa[r][c] = (si < ns && g < ge) ? pk[(size_t)si * G.N + g]
                                           : make_double2(0.0, 0.0);
            sb[r][c] = (sj < ns && g < ge) ? pk[(size_t)sj * G.N + g]
                                           : make_double2(0.0, 0.0);
        }
        __syncthreads();
        for (int c = 0; c < kGK; ++c)
            for (int u = 0; u < 2; ++u) {
                double2 av = sa[ty + 16 * u][c];
                for (int w = 0; w < 2; ++w) {
                    double2 bv = sb[tx + 16 * w][c];
                    // conj(a) * b
                    acc[u][w].x += av.x * bv.x + av.y * bv.y;
                    acc[u][w].y += av.x * bv.y - av.y * bv.x;
                }
            }
        __syncthreads();
    }
    for (int u = 0; u < 2; ++u)
        for (int w = 0; w < 2; ++w) {
            int i = ti * kGT + ty + 16 * u, j = tj * kGT + tx + 16 * w;
            if (i < ns && j < ns)
                part[(((size_t)ks * gridDim.y + kk) * ns + i) * ns + j] =
                    acc[u][w];
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

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
template <class R, class InT, class TT, int MODE>
static hipError_t go_hpsi(const HArgs &a, int ns, hipStream_t st)
{
    using V = typename Cplx<R>::T;
    const int nthr = ((a.geo.nx * a.TY + 63) / 64) * 64;
    size_t lds = (size_t)(a.TY + 2 * kHalf) * a.geo.nx * sizeof(V);
    if (lds < 64 * sizeof(double))
        lds = 64 * sizeof(double);
    dim3 grid(a.ntile_y * a.nzc, ns);
    hipLaunchKernelGGL((k_hpsi<R, InT, TT, MODE>), grid, dim3(nthr), lds, st,
                       a);
    return hipGetLastError();
}

hipError_t launch_hpsi(int mode, bool mixed, bool in_is_f64, const HArgs &a,
                       int ns, hipStream_t st)
{
    if (ns <= 0)
        return hipSuccess;
    if (!mixed) {
        switch (mode) {
        case kApply: return go_hpsi<double, double2, double2, kApply>(a, ns, st);
        case kTerm: return go_hpsi<double, double2, double2, kTerm>(a, ns, st);
        case kFinal: return go_hpsi<double, double2, double2, kFinal>(a, ns, st);
        case kFinalPred:
            return go_hpsi<double, double2, double2, kFinalPred>(a, ns, st);
        }
    } else if (in_is_f64) {
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

hipError_t launch_gather(bool mixed, bool in_is_f64, const GArgs &a, int ns,
                         hipStream_t st)
{
    if (ns <= 0 || a.pj.natoms <= 0)
        return hipSuccess;
    dim3 grid(a.pj.natoms, ns);
    if (!mixed)
        hipLaunchKernelGGL((k_gather<double, double2>), grid, dim3(256), 0, st,
                           a);
    else if (in_is_f64)
        hipLaunchKernelGGL((k_gather<float, double2>), grid, dim3(256), 0, st,
                           a);
    else
        hipLaunchKernelGGL((k_gather<float, float2>), grid, dim3(256), 0, st,
                           a);
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

hipError_t launch_dipole_finalize(const double *dpart, int nblocks,
                                  double h3, double *out, hipStream_t st)
{
    hipLaunchKernelGGL(k_dipole_finalize, dim3(1), dim3(256), 0, st, dpart,
                       nblocks, h3, out);
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
                                double h3, double *out, hipStream_t st)
{
    if (ns <= 0)
        return hipSuccess;
    hipLaunchKernelGGL(k_norm_finalize, dim3(ns), dim3(64), 0, st, normpart,
                       ntiles, h3, out);
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
    const int ntile = (ns + kGT - 1) / kGT;
    dim3 grid(ntile * ntile, nk, ksplit);
    hipLaunchKernelGGL(k_gram_partial, grid, dim3(256), 0, st, g, psi, ns,
                       ksplit, part);
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
