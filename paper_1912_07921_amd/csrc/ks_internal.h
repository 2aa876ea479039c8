// Internal interface between the C-ABI layer (ks_api.cpp) and the gfx950
// kernels (ks_kernels.hip).  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

struct ks_grid;   // the C ABI's grid object (ks_api.cpp)

namespace ks {

constexpr int kHalf = 4;      // stencil half-width (25-point star)
constexpr int kMaxProj = 9;   // s + p + d projectors per atom

// Epilogue of the H.psi kernel.
enum Mode : int {
    kApply = 0,      // out = H in                               (complex128)
    kTerm = 1,       // out = c * H in                           (t-term type)
    kFinal = 2,      // t4 = c * H t3; out = base + t1 + t2 + t3 + t4,
                     // density partials and norms of out        (complex128)
    kFinalPred = 3,  // as kFinal, plus the predictor
                     // base + 2 t1 + 4 t2 + 8 t3 + 16 t4 feeds the density
    kCurrent = 4     // no output: per tile, sum over its points of
                     // Im(conj(psi) [H_stencil, r_a] psi), a = x, y, z,
                     // into normpart[tile][3] (FP64 only)
};

struct Geo {
    int nx, ny, nz;
    long N;
    int per[3];
    double h[3];
};

// Projector data on the device.
//  - Sphere points of atom a occupy [ioff[a], ioff[a] + npts[a]) of sidx
//    (grid index), sxyz (x | y << 10 | z << 20) and sshift (lattice shift T
//    that brings the point into the sphere, three signed bytes).
//  - apos[a] = (x, y, z, rc^2), arad[a] = (1 / (2 sigma^2), 1 / rc^2); the
//    projector values are evaluated from these (p_j = N_j P_j(r) rad(r)).
//  - EjN2[a][j] = N_j^2 h^3 E_{a,l(j)} (N_j: grid normalisation of p_j).
//  - Hull: for grid row (z, y), rowinfo = (x_lo, x_hi, base, 0) spans the x
//    range that spheres cover (x_lo > x_hi: none); hull point
//    h = base + x - x_lo.  hxyz[h] packs its coordinates.  Hull chunks of 64
//    points list the atoms whose sphere meets them in
//    hc_atoms[hc_off[c] .. hc_off[c+1]).
struct ProjDev {
    int natoms = 0;
    const int *nproj = nullptr;
    const int *npts = nullptr;
    const long *ioff = nullptr;
    const int *sidx = nullptr;
    const int *sxyz = nullptr;
    const int *sshift = nullptr;
    const double *EjN2 = nullptr;
    const double4 *apos = nullptr;
    const double2 *arad = nullptr;
    const int4 *rowinfo = nullptr;
    int nhull = 0;
    const int *hxyz = nullptr;
    int nhchunk = 0;
    const int *hc_off = nullptr;
    const int *hc_atoms = nullptr;
    // per hull point h, the spheres containing it: entries
    // [he_off[h], he_off[h+1]) in atom order, each with the atom's slot in
    // its hull chunk's atom list, the Bloch phase code of the apply
    // (lattice shift from the point to its image in the sphere, negated)
    // and the 9 projector values at the image (zero past nproj)
    const int *he_off = nullptr;
    const int *he_slot = nullptr;
    const int *he_code = nullptr;
    const double *he_p = nullptr;
    // the gather's (atom, chunk) work items in dispatch order: sorted by
    // the z plane of the chunk's first point (sphere points are stored z
    // major), so that chunks of overlapping spheres that cover the same
    // planes run together and share the L2
    int ngpairs = 0;
    const int2 *gpairs = nullptr;
};

constexpr int kHullChunk = 64;

// State tile of one Gram workgroup: 64 x 64 states, or 32 x 32 when there
// are at most 32 (a larger tile would be mostly empty).
inline int gram_tile(int ns) { return ns > 32 ? 64 : 32; }

struct HArgs {
    Geo geo;
    const void *in = nullptr;      // input states of this launch
    void *out = nullptr;
    const double2 *base = nullptr; // psi for the final modes
    const void *t1 = nullptr;
    const void *t2 = nullptr;
    const double *v = nullptr;     // local potential
    const float *v32 = nullptr;    // its FP32 copy (read by the FP32 kernels)
    double a2half = 0.0;           // |A|^2 / 2
    double A[3] = {0.0, 0.0, 0.0};
    double cre = 1.0, cim = 0.0;   // complex scale of H.in
    const double2 *kph = nullptr;  // [nk][3] exp(i k_a L_a)
    int nstates = 1;               // states per k-point
    int sg0 = 0;                   // global state index of launch state 0
    const double *wocc = nullptr;  // [nk*nstates] w_k f_s
    double *npart = nullptr;       // [ns][N] density partials
    double *normpart = nullptr;    // [ns][ntiles]
    const int4 *rowinfo = nullptr; // hull rows (null: no projectors)
    const void *W = nullptr;       // [ns][nhull] V_NL in on the hull
    int nhull = 0;
    int TY = 1, zchunk = 1, ntile_y = 1, nzc = 1;
    int rpt = 1;                   // rows marched per thread (1 or 2)
};

// LDS one workgroup may use (gfx950: 160 KiB per workgroup), and the most
// the default launch shape asks for.
constexpr size_t kLdsBudget = 163840;
constexpr size_t kLdsDefault = 98304;

// Most threads of one H.psi workgroup.
constexpr int kRowThreads = 512;

struct GArgs {
    Geo geo;
    const void *in = nullptr;
    void *D = nullptr;             // [ns][natoms][9] coefficients
    void *W = nullptr;             // [ns][nhull] (apply stage)
    const double2 *kph = nullptr;
    int nstates = 1;
    int sg0 = 0;
    int ns = 0;                    // states in this launch
    void *Dpart = nullptr;         // [ns][natoms][nchunk][9] chunk sums
    int nchunk = 1;                // gather chunks of the largest sphere
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

// ks_apply_h with the projector scratch at `base` (cap bytes of device
// memory on `device`) instead of the grid's workspace; KS_E_ARG when the
// call's states need more than cap bytes.  Defined in ks_api.cpp.
int apply_h_scratch(ks_grid *g, const void *d_psi, void *d_hpsi, int k,
                    int s0, int ns, double t, char *base, size_t cap,
                    int device);
// Record an error message for ks_last_error(); returns code.
int set_error(int code, const char *msg);

// Launch shape of the H.psi kernel.
int hpsi_threads(int nx, int TY, int rpt);
int hpsi_halo_per_thread(const Geo &g, int TY, int nthr);
size_t hpsi_lds_bytes(int nx, int TY, int zchunk, bool mixed);

// Launchers (ks_kernels.hip).  All asynchronous on `st`.
hipError_t launch_hpsi(int mode, bool mixed, bool in_is_f64, const HArgs &a,
                       int ns, hipStream_t st);
// The stencil part of the current (mode kCurrent, one row per thread).
hipError_t launch_hpsi_current(const HArgs &a, int ns, hipStream_t st);
// KB projectors: D = coefficients of `in` (gather), then W = V_NL in on
// the hull (apply).  Both no-ops without atoms.
hipError_t launch_gather(bool mixed, bool in_is_f64, const GArgs &a, int ns,
                         hipStream_t st);
hipError_t launch_kbapply(bool mixed, const GArgs &a, int ns, hipStream_t st);
// Projector values of the hull entries: he_p[e][j] for the atom and sphere
// point of entry e (ent[e] = (atom, index of the point in the atom's
// sphere list)), evaluated as the gather evaluates them.
hipError_t launch_hull_table(const ProjDev &pj, const Geo &g,
                             const int2 *ent, long nent, double *he_p,
                             hipStream_t st);
int gather_chunks(int max_npts);
int gather_chunk_points();          // sphere points per gather chunk
int density_blocks(long N);
hipError_t launch_density(const DArgs &a, hipStream_t st);
hipError_t launch_dipole_finalize(const double *dpart, int nblocks,
                                  double h3, double *out, hipStream_t st,
                                  const int *step = nullptr);
hipError_t launch_norm_partial(const Geo &g, const double2 *psi, int ns,
                               int nchunks, double *normpart, hipStream_t st);
hipError_t launch_norm_finalize(const double *normpart, int ns, int ntiles,
                                double h3, double *out, hipStream_t st,
                                const int *step = nullptr);
hipError_t launch_kick(const Geo &g, double2 *psi, int ns, double kappa,
                       hipStream_t st);
// out[i] = (float)in[i], i < n (the FP32 copy of a potential)
hipError_t launch_to_f32(const double *in, float *out, long n,
                         hipStream_t st);
// the same for several potentials in one launch: copy j converts
// src[j][0 .. n[j]) into dst[j]; blocks of 256 points, blk_off[j] the first
// block of copy j
struct F32Copy {
    const double *src = nullptr;
    float *dst = nullptr;
    long n = 0;
};
hipError_t launch_to_f32_batch(const F32Copy *copies, const int *blk_off,
                               int ncopies, int nblocks, hipStream_t st);

// Reductions of several grids in one launch each (the batched form).  The
// tables are device arrays; every entry is computed exactly as the
// single-grid launch computes it.
struct DipJob {
    const double *dpart = nullptr;   // density_blocks(N) x 3 partials
    int nblocks = 0;
    double h3 = 0.0;
    double *out = nullptr;           // trace; slot step + 1
    const int *step = nullptr;
};
struct NormJob {
    const double *part = nullptr;    // [ns][ntiles] partials
    int ns = 0, ntiles = 0;
    double h3 = 0.0;
    double *out = nullptr;           // [steps + 1][ns]; slot step + 1
    const int *step = nullptr;
    int *flag = nullptr;             // set to 1 (sticky) by a NaN / Inf norm
};
// blk_off[j] = first launch block of job j (blk_off[njobs] = nblocks)
hipError_t launch_density_batch(const DArgs *args, const int *blk_off,
                                int njobs, int nblocks, hipStream_t st);
hipError_t launch_dipole_finalize_batch(const DipJob *jobs, int njobs,
                                        hipStream_t st);
hipError_t launch_norm_finalize_batch(const NormJob *jobs, int njobs,
                                      int max_ns, hipStream_t st);
hipError_t launch_gram(const Geo &g, const double2 *psi, int nk, int ns,
                       double2 *part, int ksplit, double2 *out,
                       hipStream_t st);
hipError_t launch_dot_partial(const Geo &g, const double2 *a,
                              const double2 *b, int ns, int nchunks,
                              double2 *part, hipStream_t st);
hipError_t launch_vcombine(long N, int h, const double *const src[4],
                           const double w[4], double *out, hipStream_t st);
hipError_t launch_exchange_partial(const Geo &g, const double *rho,
                                   double *part, hipStream_t st);

// ---- batched (multi-job) form ----
// One job of a batch, in device memory: the static parts of its H.psi and
// projector arguments plus the buffers the Taylor passes rotate through.
struct JobDev {
    HArgs h;                       // geometry, launch shape, kph, wocc, hull
    GArgs g;                       // projector tables, D, Dpart, W, ns
    int stot = 0;
    double2 *psi = nullptr;        // caller's states (in/out)
    double2 *half = nullptr;       // psi_half
    void *t[3] = {nullptr, nullptr, nullptr};
    double *npart = nullptr;
    int npart_end = 0;             // final density needed (a density-
                                   // dependent potential or the dipole)
    double *normpart_end = nullptr;
    const double *vion = nullptr;
    double *vcur = nullptr, *vpred = nullptr;
    int nonlin = 0;                // the potential depends on the density
    double dt = 0.0;
    // [max_steps][2] (A, |A|^2 / 2) at the two ends of each step, tabulated
    // on the host exactly as the single-job propagator evaluates them
    const double4 *Atab = nullptr;
    const int *step = nullptr;     // device step counter of the job
};

enum ItemKind : int { kItemHpsi = 0, kItemGather = 1, kItemGatherFin = 2,
                      kItemApply = 3 };

struct BArgs {
    const JobDev *jobs = nullptr;
    // [njobs][8] H.psi arguments of each job's Taylor passes (vector
    // potential left to the kernel, from the job's A(t) table)
    const HArgs *hargs = nullptr;
    int njobs = 0;
    const int *off = nullptr;      // [njobs+1] item offsets (device)
    int off_total = 0;             // items over all jobs (host copy)
    int pass = 1;                  // Taylor pass 1..8 of the ETRS step
};

int batch_items(int kind, const JobDev &J);
hipError_t launch_pass_batch(bool mixed, const BArgs &b, bool grad, int hm,
                             int rpt, int nthr, size_t lds, int grid,
                             hipStream_t st);
hipError_t launch_projectors_batch(bool mixed, const BArgs &bg,
                                   const BArgs &bf, const BArgs &ba,
                                   int grid, hipStream_t st);
hipError_t launch_step_advance(int *const *steps, int njobs, hipStream_t st);
hipError_t launch_step_set(int *const *steps, int njobs, const int *values,
                           hipStream_t st);

}  // namespace ks
