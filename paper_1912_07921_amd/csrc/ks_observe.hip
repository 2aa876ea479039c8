// Observables after the propagator on gfx950: the macroscopic current
// J(t) = -(i/Omega) sum_k w_k sum_s f_s <psi|[H, r]|psi> (section "Electric
// and thermal conductivities", eq. current_density) and the damped Fourier
// transforms of sampled traces that give the strength function of a kicked
// run and the conductivity (eq. FT).
//
// The commutator is taken on the grid: [H, r_a] has the matrix elements
// H_ij (x_j - x_i) with x_j - x_i the displacement of the coupled point (m h
// for a stencil tap m, also across a periodic wrap; the difference of the
// two points' sphere images for the projector term).  Per state this gives
//   h^3 sum_g conj(psi) [H, r_a] psi =
//     h^3 sum_g conj(psi_g) sum_{m=1..4} [ -c_m m / (2 h_a) (psi_{g+m} -
//       psi_{g-m}) - i A_a m d_m (psi_{g+m} + psi_{g-m}) ]      (stencil)
//   + 2i h^3 sum_atoms sum_j N_j^2 h^3 E_j Im(conj(C_j) D_ja)   (projectors)
// with C_j = sum p_j e^{ik.T} psi and D_ja = sum p_j e^{ik.T} (r - R)_a psi
// over the atom's sphere (p_j without its grid normalisation N_j).  Both
// parts are imaginary, so J_a = (1/Omega) sum_s w_s Im(...).  The stencil
// part runs in the H.psi kernel (mode kCurrent: its LDS-staged planes give
// the neighbours, m c_m = 2 d_m turns the kinetic taps into -grad); this
// file holds the projector part and the transforms.
#include "ks_observe.h"

#include "ks_device.h"

namespace ks {
namespace {

constexpr int kCurThreads = 256;

// Projector part of atom blockIdx.x and state blockIdx.y, all three axes
// from one pass over the sphere (the state values and projector shapes are
// loaded and evaluated once for C_j and the three D_ja):
// nl[(sl * natoms + at) * 3 + a] = 2 h^3 sum_j N_j^2 h^3 E_j
// Im(conj(C_j) D_ja).
__global__ __launch_bounds__(kCurThreads) void k_current_nl(CurArgs a)
{
    // per projector: C_j, D_jx, D_jy, D_jz, re and im
    constexpr int NV = 8 * kMaxProj;
    __shared__ double sbuf[(kCurThreads / 64) * NV];
    const Geo G = a.geo;
    const ProjDev &pj = a.pj;
    const int at = blockIdx.x, sl = blockIdx.y;
    const int kk = (a.sg0 + sl) / a.nstates;
    const double2 *psi = a.psi + (size_t)sl * G.N;
    const int np = gp(pj.nproj)[at];
    const int npt = gp(pj.npts)[at];
    const long io = gp(pj.ioff)[at];
    const double4 ap = gld(pj.apos + at);
    const double2 ar = gld(pj.arad + at);
    const double Lx = G.nx * G.h[0], Ly = G.ny * G.h[1], Lz = G.nz * G.h[2];
    double acc[NV];
#pragma unroll
    for (int i = 0; i < NV; ++i)
        acc[i] = 0.0;
    for (int pt = threadIdx.x; pt < npt; pt += kCurThreads) {
        const int gi = gp(pj.sidx)[io + pt];
        const int pk = gp(pj.sxyz)[io + pt];
        const int code = gp(pj.sshift)[io + pt];
        const int ix = pk & 0x3ff, iy = (pk >> 10) & 0x3ff, iz = pk >> 20;
        const int tx = (int)(signed char)(code & 0xff);
        const int ty = (int)(signed char)((code >> 8) & 0xff);
        const int tz = (int)(signed char)((code >> 16) & 0xff);
        const double d[3] = {
            axis_coord(G.nx, G.h[0], G.per[0], ix) + tx * Lx - ap.x,
            axis_coord(G.ny, G.h[1], G.per[1], iy) + ty * Ly - ap.y,
            axis_coord(G.nz, G.h[2], G.per[2], iz) + tz * Lz - ap.z};
        const double r2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
        double p[kMaxProj];
        proj_shape<double>(d[0], d[1], d[2], r2, ar, np, p);
        double2 v = gld(psi + gi);
        if (code)
            v = cmul(v, shift_phase<double2>(a.kph + 3 * kk, code));
#pragma unroll
        for (int j = 0; j < kMaxProj; ++j) {
            const double px = p[j] * v.x, py = p[j] * v.y;
            acc[8 * j] += px;
            acc[8 * j + 1] += py;
#pragma unroll
            for (int ax = 0; ax < 3; ++ax) {
                acc[8 * j + 2 + 2 * ax] += d[ax] * px;
                acc[8 * j + 3 + 2 * ax] += d[ax] * py;
            }
        }
    }
    // sum over the workgroup: lanes by wave_sum, waves through LDS (fully
    // unrolled so the sums stay in registers)
    const int wave = threadIdx.x >> 6;
#pragma unroll
    for (int i = 0; i < NV; ++i) {
        const double v = wave_sum(acc[i]);
        if ((threadIdx.x & 63) == 0)
            sbuf[wave * NV + i] = v;
    }
    __syncthreads();
    if (threadIdx.x < 3) {
        const int ax = threadIdx.x;
        const double h3 = G.h[0] * G.h[1] * G.h[2];
        double out = 0.0;
        for (int j = 0; j < np; ++j) {
            double s[4] = {0.0, 0.0, 0.0, 0.0};
            const int c[4] = {8 * j, 8 * j + 1, 8 * j + 2 + 2 * ax,
                              8 * j + 3 + 2 * ax};
            for (int w = 0; w < kCurThreads / 64; ++w)
#pragma unroll
                for (int u = 0; u < 4; ++u)
                    s[u] += sbuf[w * NV + c[u]];
            out += gp(pj.EjN2)[at * kMaxProj + j] *
                   (s[0] * s[3] - s[1] * s[2]);
        }
        a.nl[((size_t)sl * pj.natoms + at) * 3 + ax] = 2.0 * h3 * out;
    }
}

// Damped transform of a trace f(t_n), t_n = n dt, trapezoid weights:
// F(w) = dt sum_n w_n (f_n - f0) e^{i s w t_n} e^{-gamma t_n}, with f0 =
// f(0) when subtract is set (else 0).  Mode 0 (strength function):
// out[i] = (2 w / (pi kappa)) Im F with s = +1; mode 1 (conductivity):
// out[2i], out[2i+1] = F / E0 with s = -1.
__global__ __launch_bounds__(256) void k_damped_ft(const double *f, int nt,
                                                   int stride, double dt,
                                                   double scale, double gamma,
                                                   const double *w, int nw,
                                                   int mode, double *out)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nw)
        return;
    const double om = w[i];
    const double f0 = mode == 0 ? f[0] : 0.0;
    const double s = mode == 0 ? 1.0 : -1.0;
    double re = 0.0, im = 0.0;
    for (int n = 0; n < nt; ++n) {
        const double wt = (n == 0 || n == nt - 1) ? 0.5 : 1.0;
        const double t = n * dt;
        const double amp = wt * (f[(long)n * stride] - f0) * exp(-gamma * t);
        double sn, cs;
        sincos(s * om * t, &sn, &cs);
        re += amp * cs;
        im += amp * sn;
    }
    re *= dt;
    im *= dt;
    if (mode == 0) {
        out[i] = 2.0 * om / M_PI * im / scale;
    } else {
        out[2 * i] = re / scale;
        out[2 * i + 1] = im / scale;
    }
}

}  // namespace

hipError_t launch_current_nl(const CurArgs &a, int ns, hipStream_t st)
{
    if (ns <= 0 || a.pj.natoms == 0)
        return hipSuccess;
    hipLaunchKernelGGL(k_current_nl, dim3(a.pj.natoms, ns),
                       dim3(kCurThreads), 0, st, a);
    return hipGetLastError();
}

hipError_t launch_damped_ft(const double *f, int nt, int stride, double dt,
                            double scale, double gamma, const double *w,
                            int nw, int mode, double *out, hipStream_t st)
{
    if (nw <= 0)
        return hipSuccess;
    hipLaunchKernelGGL(k_damped_ft, dim3((nw + 255) / 256), dim3(256), 0, st,
                       f, nt, stride, dt, scale, gamma, w, nw, mode, out);
    return hipGetLastError();
}

}  // namespace ks
