// Device-side building blocks shared by the gfx950 kernel files of the
// real-time TDDFT hot path: complex helpers, streaming loads and stores,
// reductions, Bloch phases, the H.psi work item and the projector gather /
// apply work items.
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
//  - the KB term V_NL psi, formed on the projector hull rows by the apply
//    work item, is read at hull points and added before the single store
//    of the output; the Taylor recurrence scale, the final Taylor sum, the
//    ETRS predictor and the density/norm partial sums are fused into the
//    epilogue.
#pragma once

#include "ks_internal.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <type_traits>

namespace ks {

// Planes of lead of the H.psi kernel's loads (1 or 2, see hpsi_item).
#ifndef KS_HPSI_PF
#define KS_HPSI_PF 2
#endif

// Half-width-4 central weights: Laplacian (c0..c4) and gradient (d1..d4).
static __constant__ double kLap[5] = {-205.0 / 72.0, 8.0 / 5.0, -1.0 / 5.0,
                                      8.0 / 315.0, -1.0 / 560.0};
static __constant__ double kGrad[5] = {0.0, 4.0 / 5.0, -1.0 / 5.0,
                                       4.0 / 105.0, -1.0 / 280.0};

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

// Every buffer the kernels touch is global memory.  Accesses go through an
// explicitly global pointer, so that pointers read from memory (the job
// table of the batched form) compile to global, not flat, instructions.
template <class T> using gptr_t = __attribute__((address_space(1))) T *;
template <class T> __device__ __forceinline__ gptr_t<T> gp(T *p)
{
    return (gptr_t<T>)p;
}

// Loads and stores of the HIP vector classes through global pointers go by
// the compiler's native vector types.
typedef double gd2_t __attribute__((ext_vector_type(2)));
typedef float gf2_t __attribute__((ext_vector_type(2)));
typedef double gd4_t __attribute__((ext_vector_type(4)));
typedef int gi4_t __attribute__((ext_vector_type(4)));

__device__ __forceinline__ double2 gld(const double2 *p)
{
    const gd2_t v = *gp(reinterpret_cast<const gd2_t *>(p));
    return make_double2(v.x, v.y);
}
__device__ __forceinline__ float2 gld(const float2 *p)
{
    const gf2_t v = *gp(reinterpret_cast<const gf2_t *>(p));
    return make_float2(v.x, v.y);
}
__device__ __forceinline__ double4 gld(const double4 *p)
{
    const gd4_t v = *gp(reinterpret_cast<const gd4_t *>(p));
    return make_double4(v.x, v.y, v.z, v.w);
}
__device__ __forceinline__ int4 gld(const int4 *p)
{
    const gi4_t v = *gp(reinterpret_cast<const gi4_t *>(p));
    return make_int4(v.x, v.y, v.z, v.w);
}
__device__ __forceinline__ void gst(double2 *p, double2 v)
{
    *gp(reinterpret_cast<gd2_t *>(p)) = gd2_t{v.x, v.y};
}
__device__ __forceinline__ void gst(float2 *p, float2 v)
{
    *gp(reinterpret_cast<gf2_t *>(p)) = gf2_t{v.x, v.y};
}

template <class R, class T> __device__ __forceinline__ typename Cplx<R>::T
ldc(const T *p, long i)
{
    T v = gld(p + i);
    typename Cplx<R>::T r;
    r.x = (R)v.x;
    r.y = (R)v.y;
    return r;
}

// Streaming stores and loads of data touched once per pass (the H.psi
// outputs, the Taylor terms read by the final pass): non-temporal, so they
// do not evict the plane and halo lines that neighbouring workgroups reuse
// from L2.
#ifndef KS_NT_STORE
#define KS_NT_STORE 1
#endif
#ifndef KS_NT_LOAD
#define KS_NT_LOAD 1
#endif
typedef double nd2_t __attribute__((ext_vector_type(2)));
typedef float nf2_t __attribute__((ext_vector_type(2)));

__device__ __forceinline__ void st_stream(double2 *p, double x, double y)
{
#if KS_NT_STORE
    nd2_t v = {x, y};
    __builtin_nontemporal_store(v, gp(reinterpret_cast<nd2_t *>(p)));
#else
    gst(p, make_double2(x, y));
#endif
}
__device__ __forceinline__ void st_stream(float2 *p, float x, float y)
{
#if KS_NT_STORE
    nf2_t v = {x, y};
    __builtin_nontemporal_store(v, gp(reinterpret_cast<nf2_t *>(p)));
#else
    gst(p, make_float2(x, y));
#endif
}
__device__ __forceinline__ void st_stream(double *p, double x)
{
#if KS_NT_STORE
    __builtin_nontemporal_store(x, gp(p));
#else
    *gp(p) = x;
#endif
}
__device__ __forceinline__ double2 ld_stream(const double2 *p)
{
#if KS_NT_LOAD
    const nd2_t v =
        __builtin_nontemporal_load(gp(reinterpret_cast<const nd2_t *>(p)));
    return make_double2(v.x, v.y);
#else
    return gld(p);
#endif
}
__device__ __forceinline__ float2 ld_stream(const float2 *p)
{
#if KS_NT_LOAD
    const nf2_t v =
        __builtin_nontemporal_load(gp(reinterpret_cast<const nf2_t *>(p)));
    return make_float2(v.x, v.y);
#else
    return gld(p);
#endif
}

// a state value at a sphere point for the gather (non-temporal with
// KS_GATHER_NT: the states are larger than the MALL and the next pass
// streams them again anyway, while the point tables are re-read by every
// state group)
#ifndef KS_GATHER_NT
#define KS_GATHER_NT 1
#endif
template <class R, class T>
__device__ __forceinline__ typename Cplx<R>::T ldc_g(const T *p, long i)
{
    const T v = KS_GATHER_NT ? ld_stream(p + i) : gld(p + i);
    typename Cplx<R>::T r;
    r.x = (R)v.x;
    r.y = (R)v.y;
    return r;
}

// Raw buffer accesses (gfx9 buffer descriptor, no stride): an offset at or
// beyond the buffer's size reads zero and drops a store, so an access with
// nothing to move needs no branch around it.
typedef __amdgpu_buffer_rsrc_t BufRes;
__device__ __forceinline__ BufRes buf_res(const void *p, size_t bytes)
{
    return __builtin_amdgcn_make_buffer_rsrc(
        const_cast<void *>(p), (short)0,
        (int)(bytes < 0x7fffffffUL ? bytes : 0x7fffffffUL), 0x00020000);
}
template <class T> __device__ __forceinline__ T bld_raw(BufRes r, unsigned off);
template <> __device__ __forceinline__ double2 bld_raw<double2>(BufRes r,
                                                                unsigned off)
{
    return __builtin_bit_cast(double2,
                              __builtin_amdgcn_raw_buffer_load_b128(r, off, 0,
                                                                    0));
}
template <> __device__ __forceinline__ float2 bld_raw<float2>(BufRes r,
                                                              unsigned off)
{
    return __builtin_bit_cast(float2,
                              __builtin_amdgcn_raw_buffer_load_b64(r, off, 0,
                                                                   0));
}
// the same with the non-temporal hint (streams read once)
#ifndef KS_NT_ONCE
#define KS_NT_ONCE 1
#endif
template <class T>
__device__ __forceinline__ T bld_raw_nt(BufRes r, unsigned off);
template <>
__device__ __forceinline__ double2 bld_raw_nt<double2>(BufRes r, unsigned off)
{
    return __builtin_bit_cast(
        double2, __builtin_amdgcn_raw_buffer_load_b128(r, off, 0,
                                                       KS_NT_ONCE ? 2 : 0));
}
template <>
__device__ __forceinline__ float2 bld_raw_nt<float2>(BufRes r, unsigned off)
{
    return __builtin_bit_cast(
        float2, __builtin_amdgcn_raw_buffer_load_b64(r, off, 0,
                                                     KS_NT_ONCE ? 2 : 0));
}
// complex value of storage type T at byte offset off, in precision R
template <class R, class T>
__device__ __forceinline__ typename Cplx<R>::T bld(BufRes r, unsigned off)
{
    const T v = bld_raw<T>(r, off);
    typename Cplx<R>::T o;
    o.x = (R)v.x;
    o.y = (R)v.y;
    return o;
}
template <class R, class T>
__device__ __forceinline__ typename Cplx<R>::T bld_nt(BufRes r, unsigned off)
{
    const T v = bld_raw_nt<T>(r, off);
    typename Cplx<R>::T o;
    o.x = (R)v.x;
    o.y = (R)v.y;
    return o;
}
__device__ __forceinline__ double bld_d(BufRes r, unsigned off)
{
    return __builtin_bit_cast(double,
                              __builtin_amdgcn_raw_buffer_load_b64(r, off, 0,
                                                                   0));
}
// non-temporal stores (the outputs are read by the next pass only)
template <class T>
__device__ __forceinline__ void bst(BufRes r, unsigned off, double x,
                                    double y);
template <>
__device__ __forceinline__ void bst<double2>(BufRes r, unsigned off,
                                             double x, double y)
{
    typedef int i4 __attribute__((ext_vector_type(4)));
    __builtin_amdgcn_raw_buffer_store_b128(
        __builtin_bit_cast(i4, make_double2(x, y)), r, off, 0, 2);
}
template <>
__device__ __forceinline__ void bst<float2>(BufRes r, unsigned off, double x,
                                            double y)
{
    typedef int i2 __attribute__((ext_vector_type(2)));
    __builtin_amdgcn_raw_buffer_store_b64(
        __builtin_bit_cast(i2, make_float2((float)x, (float)y)), r, off, 0,
        2);
}
__device__ __forceinline__ void bst_d(BufRes r, unsigned off, double v)
{
    typedef int i2 __attribute__((ext_vector_type(2)));
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(i2, v), r, off,
                                          0, 2);
}

__device__ __forceinline__ int floordiv(int a, int n)
{
    return a >= 0 ? a / n : -((-a + n - 1) / n);
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
// Bloch phases.  kph[k][a] = exp(i k_a L_a) is tabulated on the host; a wrap
// by w cells along axis a multiplies by kph[k][a]^w (|w| is 1 except on
// axes shorter than the stencil).
// ---------------------------------------------------------------------------
template <class V>
__device__ __forceinline__ V phase_pow(const double2 *kph, int axis, int w)
{
    const double2 kv = gld(kph + axis);
    V ph = cmk<V>(kv.x, kv.y);
    if (w < 0) {
        ph.y = -ph.y;
        w = -w;
    }
    V r = ph;
    for (int i = 1; i < w; ++i)
        r = cmul(r, ph);
    return r;
}

template <class V>
__device__ __forceinline__ V shift_phase(const double2 *kph, int code)
{
    // lattice shift packed as three signed bytes (x, y, z)
    V r = cmk<V>(1.0, 0.0);
#pragma unroll
    for (int ax = 0; ax < 3; ++ax) {
        const int t = (int)(signed char)((code >> (8 * ax)) & 0xff);
        if (t)
            r = cmul(r, phase_pow<V>(kph, ax, t));
    }
    return r;
}

__device__ __forceinline__ double axis_coord(int n, double h, int per, int i)
{
    return per ? i * h : (i - 0.5 * (n - 1)) * h;
}

// ---------------------------------------------------------------------------
// Workgroups are handed to the 8 XCDs round robin in launch order; remap the
// launch index so that each XCD receives a contiguous range of work items
// (neighbouring y-tiles of the same state, which share halo rows in that
// XCD's L2).
// ---------------------------------------------------------------------------
#ifndef KS_XCD_REMAP
#define KS_XCD_REMAP 1
#endif
__device__ __forceinline__ int xcd_remap(int L, int nblk)
{
    if (!KS_XCD_REMAP)
        return L;
    constexpr int X = 8;
    const int per = nblk / X, rem = nblk % X;
    const int x = L % X, i = L / X;
    return x * per + min(x, rem) + i;
}

// ---------------------------------------------------------------------------
// H.psi with a fused epilogue.  R: arithmetic precision; InT: storage type of
// the input states; TT: storage type of t-terms (t1, t2, term outputs);
// GRAD: the velocity-gauge term -i A.grad is present; HM: halo loads per
// thread and plane.
//
// LDS holds the current xy plane of the tile padded by 4 rows above and below
// and 4 columns left and right: the neighbours' values, zeros (zero
// boundary; written once) or Bloch-wrapped values.  The stencil reads its x
// and y neighbours there without branches; the z neighbours come from a
// per-thread register queue.  Per z-plane: one barrier, two plane buffers
// alternating.  Every stream is fetched PF planes ahead of its use (PF = 1
// in the FP64 kernels, 2 in the FP32 ones, whose registers allow a second
// set): the halo of plane z+PF, the own column of plane z+4+PF, the
// potential and the KB term of plane z+PF are in flight while plane z is
// computed.  The KB term V_NL in is precomputed on the hull rows
// (k_kbapply) and added with one coalesced read.
// ---------------------------------------------------------------------------
extern __shared__ double2 smem_d2[];

// One work item of the H.psi pass described by `a`: work item w is
// (launch state, z-chunk, y-tile).  The whole workgroup takes part.  Avec
// holds the vector potential (x, y, z) and |A|^2 / 2 of the pass.  Thread
// t owns column x = t % nx of rows yl + r * TYh (r < RPT, yl = t / nx,
// TYh = ceil(TY / RPT)): every row set is a contiguous run of the plane, so
// loads stay coalesced while a tile of TY rows needs only TY / RPT thread
// rows.
template <class R, class InT, class TT, int MODE, bool GRAD, int HM, int RPT>
__device__ __forceinline__ void hpsi_item(const HArgs &a, const int w,
                                          const double4 Avec)
{
    using V = typename Cplx<R>::T;
    unsigned char *smem_raw = reinterpret_cast<unsigned char *>(smem_d2);

    const int nx = a.geo.nx, ny = a.geo.ny, nz = a.geo.nz;
    const int P = nx * ny;
    const long N = a.geo.N;
    const int ntiles = a.ntile_y * a.nzc;
    const int sl = w / ntiles;
    const int tile = w - sl * ntiles;
    const int zc = tile / a.ntile_y;
    const int tile_y = tile - zc * a.ntile_y;
    const int sg = a.sg0 + sl;
    const int kk = sg / a.nstates;
    const double2 *kph = a.kph + 3 * kk;
    const int perx = a.geo.per[0], pery = a.geo.per[1], perz = a.geo.per[2];

    const int TY = a.TY;
    // rows per thread of this item's shape (the launch's RPT is the most
    // any item of it uses)
    const int rpt = RPT > 1 ? a.rpt : 1;
    const int TYh = (TY + rpt - 1) / rpt;
    const int y0 = tile_y * TY;
    const int rows = min(TY, ny - y0);
    const int tid = threadIdx.x;
    const int nthr = blockDim.x;
    const int x = tid % nx;
    const int yl = tid / nx;
    const int RS = nx + 2 * kHalf;                  // LDS row stride
    bool act[RPT];
    int ylr[RPT], own[RPT], po[RPT];
#pragma unroll
    for (int r = 0; r < RPT; ++r) {
        ylr[r] = yl + r * TYh;
        act[r] = r < rpt && yl < TYh && ylr[r] < rows;
        const int y = y0 + (act[r] ? ylr[r] : 0);
        own[r] = (ylr[r] + kHalf) * RS + x + kHalf; // LDS slot of the point
        po[r] = y * nx + x;                         // offset within a plane
    }
    const int z0 = zc * a.zchunk;
    const int z1 = min(nz, z0 + a.zchunk);

    const int plane = (TY + 2 * kHalf) * RS;
    V *buf0 = reinterpret_cast<V *>(smem_raw);
    V *buf1 = buf0 + plane;
    V *sPh = buf1 + plane;        // x/y wrap phases, 81 entries
    V *sPz = sPh + 81;            // z wrap phases, 9 entries
    int4 *sRow = reinterpret_cast<int4 *>(sPz + 9);   // hull rows of tile

    const InT *in = reinterpret_cast<const InT *>(a.in) + (size_t)sl * N;
    const bool proj = MODE != kCurrent && a.rowinfo != nullptr;
    const V *Wst = reinterpret_cast<const V *>(a.W) + (size_t)sl * a.nhull;

    // ---- Bloch phases of x/y wraps by -4..4 cells: sPh[(wy+4)*9 + wx+4],
    // of z wraps: sPz[wz+4]; hull rows of this tile: sRow[(z-z0)*TY + row] --
    for (int t = tid; t < 81 + 9; t += nthr) {
        V ph;
        if (t < 81) {
            const int wx = t % 9 - 4, wy = t / 9 - 4;
            ph = cmk<V>(1.0, 0.0);
            if (wx)
                ph = cmul(ph, phase_pow<V>(kph, 0, wx));
            if (wy)
                ph = cmul(ph, phase_pow<V>(kph, 1, wy));
        } else {
            const int wz = t - 81 - 4;
            ph = wz ? phase_pow<V>(kph, 2, wz) : cmk<V>(1.0, 0.0);
        }
        sPh[t] = ph;
    }
    if (proj)
        for (int t = tid; t < (z1 - z0) * TY; t += nthr) {
            const int zz = z0 + t / TY, r = t % TY;
            int4 ri = make_int4(1, 0, 0, 0);
            if (r < rows)
                ri = gld(a.rowinfo + zz * ny + y0 + r);
            sRow[t] = ri;
        }

    // ---- halo of the padded plane: 8 rows of nx and 8 columns of rows+8.
    // Both buffers start zeroed, which holds every entry outside a
    // zero-boundary axis for all planes.  The other ("dynamic") entries are
    // loaded per plane: the in-grid (or wrapped) halo rows, and on a
    // periodic x axis the wrapped columns of every row with content.
    // Dynamic entry d goes to this thread when d = tid + i * nthr, i < HM.
    // hoff: offset within a plane (-1: none); hpk: LDS slot | phase id << 20
    // (id 40: no wrap) ----
    for (int t = tid; t < 2 * plane; t += nthr)
        buf0[t] = czero<V>();
    const int u0 = pery ? 0 : max(0, kHalf - y0);   // first dynamic top row
    const int nup = kHalf - u0;
    const int nlow = pery ? kHalf : max(0, min(kHalf, ny - (y0 + rows)));
    const int ndy = (nup + nlow) * nx;
    const int r_lo = u0, r_hi = rows + kHalf + nlow;
    const int ndyn = ndy + (perx ? (r_hi - r_lo) * 2 * kHalf : 0);
    int hoff[HM], hpk[HM];
#pragma unroll
    for (int i = 0; i < HM; ++i) {
        const int d = tid + i * nthr;
        hoff[i] = -1;
        hpk[i] = 0;
        if (d >= ndyn)
            continue;
        int r, xs, slot;
        if (d < ndy) {
            int hx;
            if (d < nup * nx) {
                r = u0 + d / nx;
                hx = d - (d / nx) * nx;
            } else {
                const int d1 = d - nup * nx;
                r = rows + kHalf + d1 / nx;
                hx = d1 - (d1 / nx) * nx;
            }
            xs = hx;
            slot = r * RS + hx + kHalf;
        } else {
            const int d2 = d - ndy;
            const int cc = d2 % (2 * kHalf);
            r = r_lo + d2 / (2 * kHalf);
            xs = cc < kHalf ? cc - kHalf : nx + cc - kHalf;
            slot = r * RS + (cc < kHalf ? cc : nx + cc);
        }
        int ys = y0 - kHalf + r;
        int wy = 0, wx = 0;
        if (ys < 0 || ys >= ny) {
            wy = floordiv(ys, ny);
            ys -= wy * ny;
        }
        if (xs < 0 || xs >= nx) {
            wx = floordiv(xs, nx);
            xs -= wx * nx;
        }
        hoff[i] = ys * nx + xs;
        hpk[i] = slot | (((wy + 4) * 9 + wx + 4) << 20);
    }
    __syncthreads();   // zeroed buffers, phase tables and hull rows ready

    // ---- loads and stores.  Every per-plane access is a raw buffer access
    // whose offset is out of range where there is nothing to move (the
    // hardware then returns zero, or drops the store), so no memory
    // instruction sits behind a branch and the compiler knows exactly how
    // many are in flight; the loads of plane z+2 are issued at the start of
    // plane z into one of two register sets that alternate with the parity
    // of z, so no register that a load is still filling is ever moved.
    // Bloch phases are applied where a value is consumed. ----
    constexpr unsigned kOOB = 0x80000000u;
    const BufRes rin = buf_res(in, (size_t)N * sizeof(InT));
    // the potential: FP64, or its FP32 copy in the FP32 kernels (half the
    // bytes of the stream every state re-reads)
    constexpr bool V32 = sizeof(R) == 4;
    constexpr unsigned VB = V32 ? 4u : 8u;
    const BufRes rv = buf_res(MODE == kCurrent
                                  ? nullptr
                                  : (V32 ? (const void *)a.v32
                                         : (const void *)a.v),
                              MODE == kCurrent ? 0 : (size_t)N * VB);
    const BufRes rw = buf_res(Wst, proj ? (size_t)a.nhull * sizeof(V) : 0);
    constexpr bool FIN = MODE == kFinal || MODE == kFinalPred;
    const size_t sN = (size_t)sl * N;
    const BufRes rbase = buf_res(FIN ? a.base + sN : nullptr,
                                 FIN ? (size_t)N * 16 : 0);
    const BufRes rt1 = buf_res(FIN ? reinterpret_cast<const TT *>(a.t1) + sN
                                   : nullptr,
                               FIN ? (size_t)N * sizeof(TT) : 0);
    const BufRes rt2 = buf_res(FIN ? reinterpret_cast<const TT *>(a.t2) + sN
                                   : nullptr,
                               FIN ? (size_t)N * sizeof(TT) : 0);
    using OutT = typename std::conditional<MODE == kTerm, TT, double2>::type;
    const BufRes rout = buf_res(MODE == kCurrent
                                    ? nullptr
                                    : reinterpret_cast<OutT *>(a.out) + sN,
                                MODE == kCurrent ? 0
                                                 : (size_t)N * sizeof(OutT));
    const BufRes rnp = buf_res(FIN && a.npart ? a.npart + sN : nullptr,
                               FIN && a.npart ? (size_t)N * 8 : 0);

    // byte offsets of plane zq (any integer for the own column)
    auto col_off = [&](int r, int zq) -> unsigned {
        int zz = zq;
        if (zq < 0 || zq >= nz) {
            if (!perz)
                return kOOB;
            zz = zq - floordiv(zq, nz) * nz;
        }
        return act[r] ? (unsigned)(zz * P + po[r]) * (unsigned)sizeof(InT)
                      : kOOB;
    };
    // the own column of plane zq as loaded, with its Bloch phase
    auto col_fix = [&](V v, int zq) -> V {
        if (perz && (zq < 0 || zq >= nz))
            v = cmul(v, sPz[floordiv(zq, nz) + 4]);
        return v;
    };
    auto halo_off = [&](int i, int zq) -> unsigned {
        return (hoff[i] >= 0 && zq < nz)
                   ? (unsigned)(zq * P + hoff[i]) * (unsigned)sizeof(InT)
                   : kOOB;
    };
    auto halo_fix = [&](int i, V v) -> V {
        const int pid = hpk[i] >> 20;
        return pid != 40 ? cmul(v, sPh[pid]) : v;
    };
    auto v_off = [&](int r, int zq) -> unsigned {
        return (act[r] && zq < nz) ? (unsigned)(zq * P + po[r]) * VB : kOOB;
    };
    auto v_ld = [&](unsigned off) -> double {
        if constexpr (V32)
            return (double)__builtin_bit_cast(
                float, __builtin_amdgcn_raw_buffer_load_b32(rv, off, 0, 0));
        else
            return bld_d(rv, off);
    };
    auto kb_off = [&](int r, int zq) -> unsigned {
        if (!proj || !act[r] || zq >= z1)
            return kOOB;
        const int4 ri = sRow[(zq - z0) * TY + ylr[r]];
        return (x >= ri.x && x <= ri.y)
                   ? (unsigned)(ri.z + x - ri.x) * (unsigned)sizeof(V)
                   : kOOB;
    };

    // ---- prologue: the 9-deep columns around z0, plane z0 in LDS, and
    // the register sets: S[1] holds plane z0+1 (halo, potential, KB term)
    // and the own column of plane z0+1+kHalf, S[0] the potential and KB
    // term of plane z0 ----
    V q[RPT][2 * kHalf + 1];
#pragma unroll
    for (int r = 0; r < RPT; ++r) {
#pragma unroll
        for (int m = 0; m <= 2 * kHalf; ++m)
            q[r][m] = col_fix(bld<R, InT>(rin, col_off(r, z0 - kHalf + m)),
                              z0 - kHalf + m);
        if (act[r])
            buf0[own[r]] = q[r][kHalf];
    }
#pragma unroll
    for (int i = 0; i < HM; ++i) {
        const V hv0 = bld<R, InT>(rin, halo_off(i, z0));
        if (hoff[i] >= 0)
            buf0[hpk[i] & 0xfffff] = halo_fix(i, hv0);
    }
    V shv[2][HM], snq[2][RPT], skb[2][RPT];
    double sv[2][RPT];
#pragma unroll
    for (int i = 0; i < HM; ++i) {
        shv[1][i] = bld<R, InT>(rin, halo_off(i, z0 + 1));
        shv[0][i] = czero<V>();
    }
#pragma unroll
    for (int r = 0; r < RPT; ++r) {
        snq[1][r] = bld<R, InT>(rin, col_off(r, z0 + kHalf + 1));
        snq[0][r] = czero<V>();
        if (KS_HPSI_PF == 2) {
            sv[1][r] = v_ld(v_off(r, z0 + 1));
            sv[0][r] = v_ld(v_off(r, z0));
            skb[1][r] = bld_nt<R, V>(rw, kb_off(r, z0 + 1));
            skb[0][r] = bld_nt<R, V>(rw, kb_off(r, z0));
        } else {
            sv[1][r] = v_ld(v_off(r, z0));
            sv[0][r] = 0.0;
            skb[1][r] = bld_nt<R, V>(rw, kb_off(r, z0));
            skb[0][r] = czero<V>();
        }
    }

    R LC[5], GD[5];
#pragma unroll
    for (int m = 0; m < 5; ++m) {
        LC[m] = (R)kLap[m];
        GD[m] = (R)kGrad[m];
    }
    const R ih2x = (R)(1.0 / (a.geo.h[0] * a.geo.h[0]));
    const R ih2y = (R)(1.0 / (a.geo.h[1] * a.geo.h[1]));
    const R ih2z = (R)(1.0 / (a.geo.h[2] * a.geo.h[2]));
    const R c0sum = LC[0] * (ih2x + ih2y + ih2z);
    const R Ax = (R)(Avec.x / a.geo.h[0]), Ay = (R)(Avec.y / a.geo.h[1]),
            Az = (R)(Avec.z / a.geo.h[2]);
    const V cs = cmk<V>(a.cre, a.cim);
    const double w_occ = FIN ? gp(a.wocc)[sg] : 0.0;
    double nrm = 0.0;
    double jc[3] = {0.0, 0.0, 0.0};   // kCurrent: Im(conj psi [H, r_a] psi)

    // one plane; PH = (z - z0) & 1 selects the LDS buffer holding plane z
    // and, with two register sets (PF = 2), the set the loads of plane
    // z+2 go to (the other set holds plane z+1).  With one set (PF = 1)
    // the loads of plane z+1 are issued at the start of plane z and used
    // at its end, so no load is in flight across planes.
    constexpr int PF = KS_HPSI_PF;
    static_assert(PF == 1 || PF == 2, "pipeline depth of one or two planes");
    auto plane_step = [&](auto Pc, const int z) {
        constexpr int PH = decltype(Pc)::value;
        constexpr int LS = PF == 2 ? PH : 0;       // set loaded now
        constexpr int CS = PF == 2 ? 1 - PH : 0;   // set used at the end
        V *cur = PH == 0 ? buf0 : buf1;
        V *nxt = PH == 0 ? buf1 : buf0;
        // potential and KB term of plane z (loaded two planes ago into
        // this set) before the set is refilled
        double vc[RPT];
        V kbc[RPT];
#pragma unroll
        for (int r = 0; r < RPT; ++r) {
            vc[r] = sv[PF == 2 ? PH : 1][r];
            kbc[r] = skb[PF == 2 ? PH : 1][r];
        }
        // keep the refills below the reads of the set's previous values
        // (no load may be scheduled above them: its register would then
        // still hold a live value and need a copy, i.e. a wait)
        __builtin_amdgcn_sched_barrier(0);
        // the final pass's other inputs at plane z, then plane z+2 of
        // every stream (in flight during this plane and the next)
        double2 fb[RPT];
        TT f1[RPT], f2[RPT];
#pragma unroll
        for (int r = 0; r < RPT; ++r) {
            if constexpr (FIN) {
                const unsigned gi = (unsigned)(z * P + po[r]);
                fb[r] = bld_raw_nt<double2>(rbase,
                                            act[r] ? gi * 16u : kOOB);
                f1[r] = bld_raw_nt<TT>(
                    rt1, act[r] ? gi * (unsigned)sizeof(TT) : kOOB);
                f2[r] = bld_raw_nt<TT>(
                    rt2, act[r] ? gi * (unsigned)sizeof(TT) : kOOB);
            }
        }
#pragma unroll
        for (int i = 0; i < HM; ++i)
            shv[LS][i] = bld<R, InT>(rin, halo_off(i, z + PF));
#pragma unroll
        for (int r = 0; r < RPT; ++r) {
            snq[LS][r] = bld<R, InT>(rin, col_off(r, z + kHalf + PF));
            sv[LS][r] = v_ld(v_off(r, z + PF));
            skb[LS][r] = bld_nt<R, V>(rw, kb_off(r, z + PF));
        }
        __syncthreads();
#pragma unroll
        for (int r = 0; r < RPT; ++r) {
            const V c = q[r][kHalf];
            const V *rp = cur + own[r];
            V hp = czero<V>();
            if (act[r]) {
                V sx = czero<V>(), sy = czero<V>(), sz = czero<V>();
                V gx = czero<V>(), gy = czero<V>(), gz = czero<V>();
                V ux = czero<V>(), uy = czero<V>(), uz = czero<V>();
#pragma unroll
                for (int m = 1; m <= kHalf; ++m) {
                    const V xp = rp[m], xn = rp[-m];
                    const V yp = rp[m * RS], yn = rp[-m * RS];
                    const V zp = q[r][kHalf + m], zn = q[r][kHalf - m];
                    sx = cadd(sx, cscale(cadd(xp, xn), LC[m]));
                    sy = cadd(sy, cscale(cadd(yp, yn), LC[m]));
                    sz = cadd(sz, cscale(cadd(zp, zn), LC[m]));
                    if constexpr (GRAD) {
                        gx = cadd(gx, cscale(csub(xp, xn), GD[m]));
                        gy = cadd(gy, cscale(csub(yp, yn), GD[m]));
                        gz = cadd(gz, cscale(csub(zp, zn), GD[m]));
                    }
                    if constexpr (MODE == kCurrent) {
                        // taps of the gauge term weighted by their
                        // displacement: sum m d_m (psi_+m + psi_-m)
                        const R wm = (R)m * GD[m];
                        ux = cadd(ux, cscale(cadd(xp, xn), wm));
                        uy = cadd(uy, cscale(cadd(yp, yn), wm));
                        uz = cadd(uz, cscale(cadd(zp, zn), wm));
                    }
                }
                if constexpr (MODE == kCurrent) {
                    // [H, r_a] psi = -grad_a psi - i A_a sum m d_m (psi_+ +
                    // psi_-): the kinetic taps -c_m/(2h^2) at displacement
                    // m h give -d_m/h (m c_m = 2 d_m for these weights)
                    const V gg[3] = {gx, gy, gz}, uu[3] = {ux, uy, uz};
#pragma unroll
                    for (int ax = 0; ax < 3; ++ax) {
                        const double ih = 1.0 / a.geo.h[ax];
                        const double A = ax == 0 ? Avec.x
                                                 : (ax == 1 ? Avec.y : Avec.z);
                        const double tx = -gg[ax].x * ih + A * uu[ax].y;
                        const double ty = -gg[ax].y * ih - A * uu[ax].x;
                        jc[ax] += c.x * ty - c.y * tx;
                    }
                } else {
                    V lap = cadd(cadd(cscale(sx, ih2x), cscale(sy, ih2y)),
                                 cscale(sz, ih2z));
                    lap = cadd(lap, cscale(c, c0sum));
                    const R vv = (R)(vc[r] + Avec.w);
                    hp = cadd(cscale(lap, (R)-0.5), cscale(c, vv));
                    if constexpr (GRAD) {
                        // -i A.grad
                        const V gr = cadd(cadd(cscale(gx, Ax),
                                               cscale(gy, Ay)),
                                          cscale(gz, Az));
                        hp.x += gr.y;
                        hp.y -= gr.x;
                    }
                    hp = cadd(hp, kbc[r]);
                }
            }
            if constexpr (MODE != kCurrent) {
                const unsigned gi = (unsigned)(z * P + po[r]);
                if constexpr (MODE == kApply) {
                    bst<double2>(rout, act[r] ? gi * 16u : kOOB,
                                 (double)hp.x, (double)hp.y);
                } else if constexpr (MODE == kTerm) {
                    const V t = cmul(cs, hp);
                    bst<TT>(rout, act[r] ? gi * (unsigned)sizeof(TT) : kOOB,
                            t.x, t.y);
                } else {
                    const V t4 = cmul(cs, hp);
                    const double2 bb = fb[r];
                    const TT u1 = f1[r], u2 = f2[r];
                    const double re = bb.x + (double)u1.x + (double)u2.x +
                                      (double)c.x + (double)t4.x;
                    const double im = bb.y + (double)u1.y + (double)u2.y +
                                      (double)c.y + (double)t4.y;
                    bst<double2>(rout, act[r] ? gi * 16u : kOOB, re, im);
                    double part;
                    if constexpr (MODE == kFinalPred) {
                        const double pr = bb.x + 2.0 * u1.x + 4.0 * u2.x +
                                          8.0 * c.x + 16.0 * (double)t4.x;
                        const double pi = bb.y + 2.0 * u1.y + 4.0 * u2.y +
                                          8.0 * c.y + 16.0 * (double)t4.y;
                        part = w_occ * (pr * pr + pi * pi);
                    } else {
                        const double sq = re * re + im * im;
                        part = w_occ * sq;
                        if (act[r])
                            nrm += sq;
                    }
                    bst_d(rnp, act[r] ? gi * 8u : kOOB, part);
                }
            }
        }
        // plane z+1 into the other buffer (free: its last readers passed
        // this plane's barrier): own values from the columns, the halo from
        // the other register set (loaded during the previous plane)
        if (z + 1 < z1) {
#pragma unroll
            for (int r = 0; r < RPT; ++r)
                if (act[r])
                    nxt[own[r]] = q[r][kHalf + 1];
#pragma unroll
            for (int i = 0; i < HM; ++i)
                if (hoff[i] >= 0)
                    nxt[hpk[i] & 0xfffff] = halo_fix(i, shv[CS][i]);
        }
#pragma unroll
        for (int r = 0; r < RPT; ++r) {
#pragma unroll
            for (int m = 0; m < 2 * kHalf; ++m)
                q[r][m] = q[r][m + 1];
            q[r][2 * kHalf] = col_fix(snq[CS][r], z + kHalf + 1);
            if constexpr (PF == 1) {
                sv[1][r] = sv[0][r];     // potential and KB term of z + 1
                skb[1][r] = skb[0][r];
            }
        }
    };
    int z = z0;
    for (; z + 1 < z1; z += 2) {
        plane_step(std::integral_constant<int, 0>{}, z);
        plane_step(std::integral_constant<int, 1>{}, z + 1);
    }
    if (z < z1)
        plane_step(std::integral_constant<int, 0>{}, z);
    if constexpr (MODE == kFinal) {
        if (!a.normpart)
            return;
        __syncthreads();
        double vals[1] = {nrm};
        block_sum<double, 1>(vals, reinterpret_cast<double *>(smem_raw));
        if (tid == 0)
            gp(a.normpart)[(size_t)sl * ntiles + tile] = vals[0];
    }
    if constexpr (MODE == kCurrent) {
        __syncthreads();
        block_sum<double, 3>(jc, reinterpret_cast<double *>(smem_raw));
        if (tid == 0)
#pragma unroll
            for (int ax = 0; ax < 3; ++ax)
                gp(a.normpart)[((size_t)sl * ntiles + tile) * 3 + ax] =
                    jc[ax];
    }
}

// ---------------------------------------------------------------------------
// KB projectors.  p_j(r) = N_j P_j(r) rad(r) with the real solid harmonics
// P = (1; x, y, z; xy, yz, zx, x^2 - y^2, 3z^2 - r^2) and
// rad = exp(-r^2 / (2 sigma^2)) (1 - r^2 / rc^2)^2, evaluated here without
// N_j (which the coefficients carry).
// ---------------------------------------------------------------------------
template <class R>
__device__ __forceinline__ void proj_shape(double dx, double dy, double dz,
                                           double r2, double2 ar, int np,
                                           R p[kMaxProj])
{
    const double wv = 1.0 - r2 * ar.y;
    const R rad = (R)(exp(-r2 * ar.x) * wv * wv);
    const R X = (R)dx, Y = (R)dy, Z = (R)dz;
    p[0] = rad;
    p[1] = rad * X;
    p[2] = rad * Y;
    p[3] = rad * Z;
    p[4] = rad * X * Y;
    p[5] = rad * Y * Z;
    p[6] = rad * Z * X;
    p[7] = rad * (X * X - Y * Y);
    p[8] = rad * ((R)3 * Z * Z - (X * X + Y * Y + Z * Z));
    for (int j = np; j < kMaxProj; ++j)
        p[j] = 0;
}

// Stage 1 of the gather: S_j = sum_pt P_j(r) rad(r) exp(i k.T) in(pt) over
// chunks of kGatherChunk sphere points.  A workgroup takes one atom, one
// chunk and 4 * kGatherSPW states: wavefront w handles kGatherSPW states,
// each lane a point, so the projector shape is evaluated once per point and
// wavefront.
#ifndef KS_GATHER_CHUNK
#define KS_GATHER_CHUNK 512
#endif
#ifndef KS_GATHER_SPW
#define KS_GATHER_SPW 2
#endif
constexpr int kGatherChunk = KS_GATHER_CHUNK;
constexpr int kGatherSPW = KS_GATHER_SPW;   // states per wavefront
constexpr int kGatherStates = 4 * kGatherSPW;

template <class R, class InT>
__device__ __forceinline__ void gather_item(const GArgs &a, const int at,
                                            const int grp, const int ch)
{
    using V = typename Cplx<R>::T;
    constexpr int U = kGatherChunk / 64;      // points per lane
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int s0 = grp * kGatherStates + wave * kGatherSPW;
    const int np = gp(a.pj.nproj)[at];
    const int npt = gp(a.pj.npts)[at];
    const long io = gp(a.pj.ioff)[at];
    const double4 ap = gld(a.pj.apos + at);
    const double2 ar = gld(a.pj.arad + at);
    const int nx = a.geo.nx, ny = a.geo.ny, nz = a.geo.nz;
    const double Lx = nx * a.geo.h[0], Ly = ny * a.geo.h[1],
                 Lz = nz * a.geo.h[2];
    const int p0 = ch * kGatherChunk;
    const int p1 = min(npt, p0 + kGatherChunk);
    // all loads of the chunk are issued before any is used: the point
    // tables first, then the states at those points
    int gi[U], pk[U], code[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
        const int pt = p0 + lane + 64 * u;
        const bool ok = pt < p1;
        gi[u] = ok ? gp(a.pj.sidx)[io + pt] : -1;
        pk[u] = ok ? gp(a.pj.sxyz)[io + pt] : 0;
        code[u] = ok ? gp(a.pj.sshift)[io + pt] : 0;
    }
    V val[U][kGatherSPW];
#pragma unroll
    for (int u = 0; u < U; ++u)
#pragma unroll
        for (int q = 0; q < kGatherSPW; ++q) {
            const int sl = s0 + q;
            val[u][q] = (gi[u] >= 0 && sl < a.ns)
                            ? ldc_g<R>(reinterpret_cast<const InT *>(a.in) +
                                         (size_t)sl * a.geo.N, gi[u])
                            : czero<V>();
        }
    R acc[kGatherSPW][2 * kMaxProj];
#pragma unroll
    for (int q = 0; q < kGatherSPW; ++q)
#pragma unroll
        for (int j = 0; j < 2 * kMaxProj; ++j)
            acc[q][j] = 0;
#pragma unroll
    for (int u = 0; u < U; ++u) {
        if (gi[u] < 0)
            continue;
        const int ix = pk[u] & 0x3ff, iy = (pk[u] >> 10) & 0x3ff,
                  iz = pk[u] >> 20;
        const int tx = (int)(signed char)(code[u] & 0xff);
        const int ty = (int)(signed char)((code[u] >> 8) & 0xff);
        const int tz = (int)(signed char)((code[u] >> 16) & 0xff);
        const double dx = axis_coord(nx, a.geo.h[0], a.geo.per[0], ix) +
                          tx * Lx - ap.x;
        const double dy = axis_coord(ny, a.geo.h[1], a.geo.per[1], iy) +
                          ty * Ly - ap.y;
        const double dz = axis_coord(nz, a.geo.h[2], a.geo.per[2], iz) +
                          tz * Lz - ap.z;
        const double r2 = dx * dx + dy * dy + dz * dz;
        R p[kMaxProj];
        proj_shape<R>(dx, dy, dz, r2, ar, np, p);
#pragma unroll
        for (int q = 0; q < kGatherSPW; ++q) {
            const int sl = s0 + q;
            if (sl >= a.ns)
                break;
            V v = val[u][q];
            if (code[u]) {
                const int kk = (a.sg0 + sl) / a.nstates;
                v = cmul(v, shift_phase<V>(a.kph + 3 * kk, code[u]));
            }
#pragma unroll
            for (int j = 0; j < kMaxProj; ++j) {
                acc[q][2 * j] += p[j] * v.x;
                acc[q][2 * j + 1] += p[j] * v.y;
            }
        }
    }
    // sum over the 64 lanes by a transpose through LDS: column c of the
    // workgroup (wave, state, projector, re/im) gets the lanes' values as
    // rows; thread c then adds its column in lane order (deterministic)
    constexpr int kCols = 4 * kGatherSPW * 2 * kMaxProj;
    static_assert(kCols <= 256, "one thread of the workgroup per column");
    __shared__ R red[kCols][65];
    __syncthreads();               // the previous item's reads are done
#pragma unroll
    for (int q = 0; q < kGatherSPW; ++q)
#pragma unroll
        for (int j = 0; j < 2 * kMaxProj; ++j)
            red[(wave * kGatherSPW + q) * 2 * kMaxProj + j][lane] = acc[q][j];
    __syncthreads();
    const int c = threadIdx.x;
    if (c < kCols) {
        R sum = 0;
        for (int r = 0; r < 64; ++r)
            sum += red[c][r];
        const int w = c / (2 * kMaxProj * kGatherSPW);
        const int q = (c / (2 * kMaxProj)) % kGatherSPW;
        const int jj = c % (2 * kMaxProj);
        const int sl = grp * kGatherStates + w * kGatherSPW + q;
        if (sl < a.ns) {
            R *part = reinterpret_cast<R *>(a.Dpart) +
                      2 * ((((size_t)sl * a.pj.natoms + at) * a.nchunk + ch) *
                           kMaxProj);
            gp(part)[jj] = sum;    // (j, re/im) interleaved as in V
        }
    }
}

// Stage 2: D[s][a][j] = N_j^2 h^3 E_{a,l(j)} sum over chunks (in order).
template <class R>
__device__ __forceinline__ void gather_finalize_item(const GArgs &a,
                                                     const long i)
{
    using V = typename Cplx<R>::T;
    const long total = (long)a.ns * a.pj.natoms * kMaxProj;
    if (i >= total)
        return;
    const int j = (int)(i % kMaxProj);
    const long sa = i / kMaxProj;           // s * natoms + atom
    const int at = (int)(sa % a.pj.natoms);
    const int nch = (gp(a.pj.npts)[at] + kGatherChunk - 1) / kGatherChunk;
    const V *part = reinterpret_cast<const V *>(a.Dpart) +
                    (size_t)sa * a.nchunk * kMaxProj + j;
    R re = 0, im = 0;
    for (int c = 0; c < nch; ++c) {
        const V v = gld(part + (size_t)c * kMaxProj);
        re += v.x;
        im += v.y;
    }
    const R e = (j < gp(a.pj.nproj)[at]) ? (R)gp(a.pj.EjN2)[at * kMaxProj + j]
                                     : (R)0;
    gst(reinterpret_cast<V *>(a.D) + i, cmk<V>(e * re, e * im));
}

// V_NL in on the hull: W[s][h] = sum over atoms a whose sphere holds hull
// point h of sum_j P_j(r) rad(r) D[s][a][j] exp(-i k.T).  A workgroup takes
// a chunk of 64 hull points (one per lane) and kApplyWaves * SPW states
// (SPW per wavefront).  The wavefront walks the chunk's atoms in a uniform
// loop; for atom i every lane whose hull point lies in its sphere (the
// lane's next hull entry has slot i: entries are in atom order, so each
// lane still adds its terms in atom order, deterministically) adds the
// atom's term.  The projector values come from a per-grid table of the
// entries (evaluated once at creation), the coefficients of the atom and
// the wavefront's states through scalar loads (one address for the whole
// wavefront): no LDS staging, no barrier, no per-lane coefficient read.
// (Staging the coefficients in LDS and reading them per lane cost 23 %
// more at 128^3 x 256, 26 % more in the FP32 kernels.)
// States per wavefront: for launches of many states 8 in FP64 and 16 in
// FP32 (fewer hull-entry walks and table reads per state), 4 for few (more
// workgroups): 128^3 x 256 FP64 1.02 -> 0.92 ms with 8 (1.01 ms with 16),
// FP32 0.74 -> 0.68 ms with 16; 64^3 x 32 12.3 -> 16.6 us with 8.
#ifndef KS_APPLY_SPW_SMALL
#define KS_APPLY_SPW_SMALL 4
#endif
#ifndef KS_APPLY_SPW_LARGE
#define KS_APPLY_SPW_LARGE 8
#endif
#ifndef KS_APPLY_SPW_LARGE32
#define KS_APPLY_SPW_LARGE32 16
#endif
#ifndef KS_APPLY_LARGE_NS
#define KS_APPLY_LARGE_NS 128
#endif
#ifndef KS_APPLY_WAVES
#define KS_APPLY_WAVES 4
#endif
constexpr int kApplyWaves = KS_APPLY_WAVES;
constexpr int kApplyThreads = 64 * kApplyWaves;
// states per wavefront of a single-grid launch of ns states in FP64 or
// FP32 (the batched launch, whose jobs are small, takes the small count)
__host__ __device__ constexpr int apply_spw(int ns, bool fp32)
{
    return ns < KS_APPLY_LARGE_NS
               ? KS_APPLY_SPW_SMALL
               : (fp32 ? KS_APPLY_SPW_LARGE32 : KS_APPLY_SPW_LARGE);
}
// state groups of the apply for ns states at spw states per wavefront
__host__ __device__ constexpr int apply_groups(int ns, int spw)
{
    return (ns + kApplyWaves * spw - 1) / (kApplyWaves * spw);
}
template <class T> using kptr_t = __attribute__((address_space(4))) const T *;

template <class R, int SPW>
__device__ __forceinline__ void kbapply_item(const GArgs &a, const int chunk,
                                             const int grp)
{
    using V = typename Cplx<R>::T;
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int s0 = (grp * kApplyWaves + wave) * SPW;
    const int h = chunk * kHullChunk + lane;
    const bool valid = h < a.pj.nhull;
    int e = valid ? gp(a.pj.he_off)[h] : 0;
    const int e1 = valid ? gp(a.pj.he_off)[h + 1] : 0;
    const int c0 = __builtin_amdgcn_readfirstlane(gp(a.pj.hc_off)[chunk]);
    const int c1 =
        __builtin_amdgcn_readfirstlane(gp(a.pj.hc_off)[chunk + 1]);
    V acc[SPW];
#pragma unroll
    for (int q = 0; q < SPW; ++q)
        acc[q] = czero<V>();
    int slot = e < e1 ? gp(a.pj.he_slot)[e] : -1;
    const kptr_t<R> Dall = (kptr_t<R>)reinterpret_cast<const R *>(a.D);
    for (int i = 0; i < c1 - c0; ++i) {
        const int at =
            __builtin_amdgcn_readfirstlane(gp(a.pj.hc_atoms)[c0 + i]);
        if (slot != i)
            continue;
        const int code = gp(a.pj.he_code)[e];
        R p[kMaxProj];
#pragma unroll
        for (int j = 0; j < kMaxProj; ++j)
            p[j] = (R)gp(a.pj.he_p)[(size_t)e * kMaxProj + j];
        // all 9 projectors: past the atom's count both the coefficients
        // and the tabulated values are zero
#pragma unroll
        for (int q = 0; q < SPW; ++q) {
            const int sl = s0 + q;
            if (sl < a.ns) {
                const kptr_t<R> D =
                    Dall + 2 * ((size_t)sl * a.pj.natoms + at) * kMaxProj;
                R d[2 * kMaxProj];
#pragma unroll
                for (int j = 0; j < 2 * kMaxProj; ++j)
                    d[j] = D[j];
                V t = czero<V>();
#pragma unroll
                for (int j = 0; j < kMaxProj; ++j)
                    t = cadd(t, cscale(cmk<V>(d[2 * j], d[2 * j + 1]), p[j]));
                if (code) {
                    const int kk = (a.sg0 + sl) / a.nstates;
                    t = cmul(t, shift_phase<V>(a.kph + 3 * kk, code));
                }
                acc[q] = cadd(acc[q], t);
            }
        }
        ++e;
        slot = e < e1 ? gp(a.pj.he_slot)[e] : -1;
    }
    // W is read once, by the next H.psi pass, and is larger than the MALL:
    // non-temporal stores
    if (valid)
#pragma unroll
        for (int q = 0; q < SPW; ++q) {
            const int sl = s0 + q;
            if (sl < a.ns)
                st_stream(reinterpret_cast<V *>(a.W) +
                              (size_t)sl * a.pj.nhull + h,
                          acc[q].x, acc[q].y);
        }
}

}  // namespace ks
