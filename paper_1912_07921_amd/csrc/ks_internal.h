// Internal interface between the C-ABI layer (ks_api.cpp) and the gfx950
// kernels (ks_kernels.hip).  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

namespace ks {

constexpr int kHalf = 4;      // stencil half-width (25-point star)
constexpr int kMaxProj = 9;   // s + p + d projectors per atom

// Epilogue of the H.psi kernel.
enum Mode : int {
    kApply = 0,      // out = H in                               (complex128)
    kTerm = 1,       // out = c * H in                           (t-term type)
    kFinal = 2,      // t4 = c * H t3; out = base + t1 + t2 + t3 + t4,
                     // density partials and norms of out        (complex128)
    kFinalPred = 3   // as kFinal, plus the predictor
                     // base + 2 t1 + 4 t2 + 8 t3 + 16 t4 feeds the density
};

struct Geo {
    int nx, ny, nz;
    long N;
    int per[3];
    double h[3];
};

// Projector tables on the device.  Sphere points of atom a occupy
// [ioff[a], ioff[a] + npts[a]) of sidx/sshift (sshift: the lattice shift
// T that brings the point into the sphere, three signed bytes); the
// normalised table is ptab[poff[a] + j * npts[a] + pt].  The scatter
// evaluates projectors from apos (x, y, z, rc^2) and arad
// (1 / (2 sigma^2), 1 / rc^2); EjN[a][j] = N_j h^3 E_{a,l(j)}.
struct ProjDev {
    int natoms = 0;
    const int *nproj = nullptr;
    const int *npts = nullptr;
    const long *ioff = nullptr;
    const long *poff = nullptr;
    const int *sidx = nullptr;
    const int *sshift = nullptr;
    const double *ptab = nullptr;
    const float *ptabf = nullptr;
    const double *EjN = nullptr;
    const double4 *apos = nullptr;
    const double2 *arad = nullptr;
};

struct HArgs {
    Geo geo;
    const void *in = nullptr;      // input states of this launch
    void *out = nullptr;
    const double2 *base = nullptr; // psi for the final modes
    const void *t1 = nullptr;
    const void *t2 = nullptr;
    const double *v = nullptr;     // local potential
    double a2half = 0.0;           // |A|^2 / 2
    double A[3] = {0.0, 0.0, 0.0};
    double cre = 1.0, cim = 0.0;   // complex scale of H.in
    const double2 *kph = nullptr;  // [nk][3] exp(i k_a L_a)
    int nstates = 1;               // states per k-point
    int sg0 = 0;                   // global state index of launch state 0
    const double *wocc = nullptr;  // [nk*nstates] w_k f_s
    double *npart = nullptr;       // [ns][N] density partials
    double *normpart = nullptr;    // [ns][ntiles]
    ProjDev pj;
    const void *D = nullptr;       // [ns][natoms][9] projector coefficients
    int TY = 1, zchunk = 1, ntile_y = 1, nzc = 1;
};

// LDS available to one workgroup of the H.psi kernel.
constexpr size_t kLdsBudget = 65536;

struct GArgs {
    Geo geo;
    const void *in = nullptr;
    void *D = nullptr;
    const double2 *kph = nullptr;
    int nstates = 1;
    int sg0 = 0;
    int ns = 0;                    // states in this launch
    void *Dpart = nullptr;         // [ns][natoms][nchunk][9] chunk sums
    int nchunk = 1;                // chunks of the largest sphere
    ProjDev pj;
};

struct DArgs {
    Geo geo;
    int nsrc = 0;                  // number of states summed
    const double *npart = nullptr; // [nsrc][N] partials, or
    const double2 *psi = nullptr;  // [nsrc][N] states (weights wocc)
    const double *wocc = nullptr;
    double *rho = nullptr;
    const double *vion = nullptr;  // optional: v_out = vion + v_x(rho)
    double *vout = nullptr;
    int xc = 0;
    double *dpart = nullptr;       // optional [nblocks][3] dipole partials
};

// Launch shape of the H.psi kernel.
int hpsi_threads(int nx, int TY);
size_t hpsi_lds_bytes(int nx, int TY, int natoms, bool mixed);

// Launchers (ks_kernels.hip).  All asynchronous on `st`.
hipError_t launch_hpsi(int mode, bool mixed, bool in_is_f64, const HArgs &a,
                       int ns, hipStream_t st);
hipError_t launch_gather(bool mixed, bool in_is_f64, const GArgs &a, int ns,
                         hipStream_t st);
int gather_chunks(int max_npts);
int density_blocks(long N);
hipError_t launch_density(const DArgs &a, hipStream_t st);
hipError_t launch_dipole_finalize(const double *dpart, int nblocks,
                                  double h3, double *out, hipStream_t st);
hipError_t launch_norm_partial(const Geo &g, const double2 *psi, int ns,
                               int nchunks, double *normpart, hipStream_t st);
hipError_t launch_norm_finalize(const double *normpart, int ns, int ntiles,
                                double h3, double *out, hipStream_t st);
hipError_t launch_kick(const Geo &g, double2 *psi, int ns, double kappa,
                       hipStream_t st);
hipError_t launch_gram(const Geo &g, const double2 *psi, int nk, int ns,
                       double2 *part, int ksplit, double2 *out,
                       hipStream_t st);
hipError_t launch_dot_partial(const Geo &g, const double2 *a,
                              const double2 *b, int ns, int nchunks,
                              double2 *part, hipStream_t st);
hipError_t launch_exchange_partial(const Geo &g, const double *rho,
                                   double *part, hipStream_t st);

}  // namespace ks
