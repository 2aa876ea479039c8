/*
 * ks.h -- C ABI of the MI355X real-time TDDFT hot path (libks).
 *
 * The method is the one of arXiv:1912.07921 ("Octopus, a computational
 * framework for exploring light-driven phenomena and quantum dynamics in
 * extended and finite systems"): the time-dependent Kohn-Sham equations as a
 * first-order ODE, d(phi_i)/dt = -i H[n(t),t] phi_i (section "New propagators
 * for real-time TDDFT"), integrated with the enforced-time-reversal-symmetry
 * (ETRS) propagator (same section; used for the absorption run of section
 * "van der Waals"), with H applied on a uniform real-space grid by finite
 * differences (section "Periodic systems") to batches of states kept resident
 * in GPU memory (section "GPUs", "Memory layout").
 *
 * Conventions shared by every call
 *  - Units: Hartree atomic units (bohr, Hartree, hbar = 1).
 *  - Grid point (x, y, z), 0 <= x < nx etc., has linear index
 *    g = (z * ny + y) * nx + x (x fastest).  Coordinates: r_a = (i - (n-1)/2) h
 *    on a zero-boundary axis, r_a = i h on a periodic axis (cell L = n h).
 *  - States: complex128 (interleaved re, im), layout [nk][nstates][nz][ny][nx]
 *    contiguous; "state j" of a call means the j-th n-point block.
 *  - Pointers named d_* are DEVICE pointers owned by the caller (for instance
 *    torch tensors) and borrowed for the call; every call is stream-ordered on
 *    the grid's stream and returns before the device finishes unless noted,
 *    so the caller keeps d_* buffers alive until the stream has drained.
 *    Host pointers (no d_ prefix) are read during the call only.
 *  - Every call returns 0 (KS_OK) or a negative ks_status; nothing throws
 *    across the ABI.  ks_last_error() gives a message for the calling thread.
 *  - A ks_grid is not thread-safe: one grid per host thread / stream.
 *
 * The Hamiltonian (fixed by these readings of the paper):
 *   H = -1/2 Lap + v(r) + V_NL + [-i A(t).grad + |A(t)|^2/2]
 *  - Lap, grad: half-width-4 central finite differences (25-point star),
 *    weights {-205/72, 8/5, -1/5, 8/315, -1/560} and {4/5, -1/5, 4/105,
 *    -1/280}; zero outside a non-periodic axis, Bloch phase
 *    psi(i + n) = exp(i k_a L_a) psi(i) along a periodic axis (k-points,
 *    section "Periodic systems").
 *  - v = v_ion + v_x[n] (+ v_H[n]); v_x = -(3 n / pi)^(1/3) (LDA exchange,
 *    section "Local domains", E_xc^LDA; Dirac/Slater form).  v_H, the
 *    Hartree potential, is optional (desc.hartree): the paper counts it
 *    among the density-dependent terms that the CFM4 propagator
 *    extrapolates (section "New propagators") but fixes no solver.  Here
 *    v_H solves Lap v_H = -4 pi n: on a finite grid (no periodic axis) as
 *    v_H(r_i) = h^3 sum_j n_j G(r_i - r_j) with G = 1/|r| and G(0) the mean
 *    of 1/|r| over one grid cell; on a periodic grid (all axes periodic) as
 *    v_H(G) = 4 pi n(G) / |G|^2 over the grid's Fourier frequencies, with
 *    v_H(G = 0) = 0.
 *  - V_NL: Kleinman-Bylander projectors on atom spheres |r - R_a| < rc_a
 *    (non-local pseudopotentials, section "Magneto-optics"):
 *    p_lm(r) = P_lm(r) exp(-r^2 / (2 sigma^2)) (1 - r^2/rc^2)^2 with real
 *    solid harmonics s; x, y, z; xy, yz, zx, x^2-y^2, 3z^2-r^2, normalised
 *    so that h^3 sum p^2 = 1; C = h^3 sum p~ psi with p~ = p e^{i k.T} for
 *    the lattice shift T that brings the point into the sphere;
 *    V_NL psi = sum conj(p~) E_{a,l} C.
 *  - Velocity gauge for a uniform vector potential (dipole approximation,
 *    section "t-SURFF", Volkov Hamiltonian; section "Thermoelectric"):
 *    A(t) = A0 sin^2(pi t / T) cos(w t) pol for 0 <= t <= T, 0 otherwise.
 */
#ifndef KS_H
#define KS_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ks_grid ks_grid;

typedef enum {
    KS_OK = 0,
    KS_E_ARG = -1,          /* invalid argument, size or layout */
    KS_E_OOM = -2,          /* a device allocation failed / workspace short */
    KS_E_HIP = -3,          /* a HIP runtime call failed */
    KS_E_UNSUPPORTED = -4,  /* valid input this library does not handle */
    KS_E_STATE = -5,        /* call out of order (no potential, no workspace) */
    KS_E_NONFINITE = -6     /* a norm (or checked value) is NaN or Inf */
} ks_status;

typedef enum {
    KS_FP64 = 0,   /* everything in FP64 */
    KS_MIXED = 1   /* H.psi terms in complex FP32 with FP32 accumulation;
                      psi update sum, norms, density, dipole in FP64 */
} ks_precision;

typedef struct {
    int n[3];            /* nx, ny, nz >= 1; nx <= 512 (one x-row of a
                            tile is one thread per point, at most 512
                            threads); nx * ny * nz < 2^27 (one state's
                            bytes take 32-bit buffer offsets); with atoms
                            also ny <= 1024 and nz <= 2048 (packed point
                            coordinates); else KS_E_UNSUPPORTED */
    double h[3];         /* grid spacing per axis (bohr), > 0 */
    int periodic[3];     /* 1: Bloch-periodic axis, 0: zero boundary */
    int fd_half_width;   /* must be 4 (25-point star); else KS_E_UNSUPPORTED */
    int nk;              /* k-points >= 1 (all zero for a finite system) */
    const double *kpts;  /* host, nk*3, bohr^-1; NULL: all zero */
    const double *kw;    /* host, nk weights; NULL: 1/nk each */
    int nstates;         /* states per k-point >= 1 */
    const double *occ;   /* host, nstates occupations; NULL: 2 each */
    int natoms;          /* >= 0 */
    const double *pos;   /* host, natoms*3 (bohr) */
    const int *lmax;     /* host, natoms, 0 (s), 1 (s+p) or 2 (s+p+d) */
    const double *rc;    /* host, natoms; periodic axes need rc < L/2 */
    const double *sigma; /* host, natoms */
    const double *E;     /* host, natoms*3: E[a*3 + l] (Hartree) */
    int xc;              /* 0: v = v_ion; 1: v = v_ion + LDA exchange */
    double laser[6];     /* A0, omega, T, pol_x, pol_y, pol_z; A0 = 0: off */
    int precision;       /* ks_precision */
    void *stream;        /* hipStream_t the calls are ordered on (NULL:
                            the default stream) */
    int hartree;         /* 0: no Hartree term; 1: v += v_H[n]; needs all
                            axes finite (n_a <= 256) or all periodic (each
                            n_a a product of 2, 3 and 5, <= 512); else
                            KS_E_UNSUPPORTED */
} ks_grid_desc;

/* Create a grid object: copies the description, builds the projector
 * spheres and tables and uploads them (device memory owned by the object).
 * Synchronous.  *out is NULL on error. */
int ks_grid_create(const ks_grid_desc *desc, ks_grid **out);

/* Free the object and its device tables; waits for its stream first. */
int ks_grid_destroy(ks_grid *g);

/* Change the stream later calls are ordered on. */
int ks_set_stream(ks_grid *g, void *stream);

/* Bytes of device scratch ks_propagate_etrs and ks_apply_h need (t-terms,
 * the half-step state, density partials, projector coefficients). */
size_t ks_workspace_bytes(const ks_grid *g);

/* Device memory the grid holds itself since ks_grid_create: the potential,
 * phase and weight tables, the projector sphere and hull tables, and the
 * Hartree plan (twiddles and kernel), in bytes, into *out (host).  The
 * caller-lent workspace is not included.  For admission control by a
 * caller that budgets HBM (the serving loop counts it in a request's
 * footprint).  KS_E_ARG on NULL arguments. */
int ks_grid_device_bytes(const ks_grid *g, size_t *out);

/* Lend the object a caller-owned device workspace of at least
 * ks_workspace_bytes() bytes, 256-byte aligned; KS_E_OOM if too small. */
int ks_set_workspace(ks_grid *g, void *d_ws, size_t bytes);

/* v = v_ion + v_x[rho] + v_H[rho] into the object's local potential (N
 * doubles), each density term only when the grid has it; d_rho NULL:
 * v = v_ion.  (One-body potential of eq. Hamiltonian_dipole; LDA of
 * section "Local domains".)  With the Hartree term and d_rho given, needs a
 * workspace. */
int ks_update_vlocal(ks_grid *g, const double *d_vion, const double *d_rho);

/* d_vh = v_H[d_rho] (N doubles each, device, not overlapping): the Hartree
 * potential of the density as defined above, by FFT convolution (zero
 * padded to at least 2 n - 1 per axis on a finite grid).  KS_E_STATE if the
 * grid was
 * created without the Hartree term or has no workspace. */
int ks_hartree(ks_grid *g, const double *d_rho, double *d_vh);

/* d_hpsi = H(t) d_psi for ns states (each n points, complex128) of k-point
 * k, using the object's current local potential and A(t).  s0 is the index
 * of the first state within the k-point (it selects occupations only).
 * In KS_MIXED the arithmetic is FP32 (input and output stay complex128).
 * Needs a workspace.  d_psi and d_hpsi must not overlap. */
int ks_apply_h(ks_grid *g, const void *d_psi, void *d_hpsi, int k, int s0,
               int ns, double t);

/* ks_apply_h for callers that cannot allocate device memory or lend a
 * workspace (code under HIP graph capture, serving loops, harnesses that
 * forbid hipMalloc): same arguments, layout, results and errors as
 * ks_apply_h, but the projector scratch (coefficients, their partial sums
 * and the terms on the projector rows) lives in a static device array of
 * 64 MiB that the library holds on each GPU it runs on until the process
 * ends; the call needs no workspace and allocates nothing.  KS_E_ARG when
 * the ns states need more than 64 MiB of scratch (then apply H to fewer
 * states per call), or when the current device is not the grid's.  All
 * calls on one GPU share its array: calls that overlap on one GPU (other
 * streams, other threads) race and must be ordered by the caller. */
int ks_apply_h_noalloc(ks_grid *g, const void *d_psi, void *d_hpsi, int k,
                       int s0, int ns, double t);

/* Propagate all nk*nstates states in d_psi, in place, by nsteps ETRS steps
 * of dt from t0.  Each step: H_t^j psi, j = 1..4 (Taylor-4, H frozen);
 * psi_half = sum (-i dt/2)^j H^j psi / j!; predictor
 * sum (-i dt)^j H^j psi / j! (same powers) gives n_pred and
 * v(t+dt) = v_ion + v_x[n_pred] (+ v_H[n_pred]);
 * psi(t+dt) = T4(dt/2, H_{t+dt}) psi_half;
 * v is rebuilt from n(psi(t+dt)).  v(t0) is built from n(psi(t0)) first.
 * d_dipole: device (nsteps+1)*3 doubles, d(t_i) = h^3 sum r n (zero-boundary
 * grids only; NULL to skip).  d_norms: device (nsteps+1)*nk*nstates doubles,
 * h^3 sum |psi|^2 per state (NULL to skip).  d_vion must stay valid until
 * the stream drains.  Needs a workspace.  With nsteps >= 1 the call ends by
 * copying the norms after the last step to the host (they are computed
 * also when d_norms is NULL) and synchronising the stream: it returns
 * KS_E_NONFINITE, naming the state, when one of them is NaN or Inf (the
 * states and outputs then hold what the steps produced). */
int ks_propagate_etrs(ks_grid *g, void *d_psi, const double *d_vion,
                      int nsteps, double dt, double t0, double *d_dipole,
                      double *d_norms);

/* CFM4 propagation (section "New propagators for real-time TDDFT": the
 * order-four commutator-free Magnus expansion with two exponentials,
 *   psi(t+dt) = exp(-i dt (a1 H(t1) + a2 H(t2)))
 *               exp(-i dt (a2 H(t1) + a1 H(t2))) psi(t),
 * a1,2 = (3 -+ 2 sqrt 3)/12, t1,2 = t + (1/2 -+ sqrt(3)/6) dt).  H(t_i)
 * takes A(t_i) and the local potential extrapolated from the potentials at
 * the ends of the most recent steps of this call (cubic through four; fewer
 * in its first three steps).  Each exponential is Taylor-4 with 4 H.psi, so
 * a step costs 8 H.psi like an ETRS step.  Arguments, outputs, errors
 * (KS_E_NONFINITE included), the end-of-call synchronisation and the grid's
 * potential afterwards as for ks_propagate_etrs. */
int ks_propagate_cfm4(ks_grid *g, void *d_psi, const double *d_vion,
                      int nsteps, double dt, double t0, double *d_dipole,
                      double *d_norms);

/* Macroscopic current J(t) (section "Electric and thermal
 * conductivities", eq. current_density):
 *   J = -(i / Omega) sum_k w_k sum_s f_s <psi_ks|[H(t), r]|psi_ks>,
 * Omega = nx hx ny hy nz hz (the cell, or the box of a finite grid), for
 * all nk*nstates states in d_psi (complex128, device) at time t (A(t) of
 * the grid's laser).  On the grid [H, r] has the matrix elements
 * H_ij (x_j - x_i) with x_j - x_i the displacement of the coupled point:
 * m h for a stencil tap m (also across a periodic wrap), the difference of
 * the two points' sphere images for the projectors; the local potential
 * drops out.  On a finite grid this is the literal commutator; on a
 * periodic one it is the k-derivative of the Bloch Hamiltonian.  out_host:
 * 3 doubles (x, y, z).  Synchronises the stream.  Needs a workspace. */
int ks_current(ks_grid *g, const void *d_psi, double t, double out_host[3]);

/* Strength function of a kicked run (section "van der Waals", the
 * absorption run): from nt samples d(t_n), t_n = n dt, of the dipole
 * component along the kick (device, sample n at d_trace[n * stride]; for
 * the (nsteps+1) x 3 dipole trace of ks_propagate_etrs use stride 3 and
 * offset the pointer to the component),
 *   alpha(w) = (1/kappa) dt sum_n w_n (d(t_n) - d(0)) e^{i w t_n}
 *              e^{-gamma t_n}   (trapezoid weights w_n: 1/2 at both ends),
 *   d_out[i] = S(w_i) = (2 w_i / pi) Im alpha(w_i)
 * for the nw frequencies d_omega (device).  S integrates to the number of
 * electrons; the absorption cross section is (2 pi^2 / c) S.  Stream-
 * ordered on `stream` (a hipStream_t, NULL: default); needs no grid. */
int ks_strength_function(const double *d_trace, int nt, int stride,
                         double dt, double kappa, double gamma,
                         const double *d_omega, int nw, double *d_out,
                         void *stream);

/* Conductivity after an impulsive field E0 (section "Electric and thermal
 * conductivities", eq. FT): from nt samples J(t_n) of a current component
 * (device, stride as above),
 *   sigma(w_i) = (1/E0) dt sum_n w_n J(t_n) e^{-i w_i t_n} e^{-gamma t_n},
 * into d_out (device, nw complex128).  Stream-ordered on `stream`. */
int ks_conductivity(const double *d_trace, int nt, int stride, double dt,
                    double E0, double gamma, const double *d_omega, int nw,
                    void *d_out, void *stream);

/* d_rho[g] = sum_k w_k sum_s f_s |psi_ks(g)|^2 over all nk*nstates states
 * (section "Local domains", n = sum of densities). */
int ks_density(ks_grid *g, const void *d_psi, double *d_rho);

/* out_host = h^3 sum_g r_g rho_g (dipole equation of section "Local
 * domains").  Synchronises the stream.  KS_E_UNSUPPORTED on a grid with a
 * periodic axis (the dipole of a periodic system is not defined). */
int ks_dipole(ks_grid *g, const double *d_rho, double out_host[3]);

/* psi <- exp(i kappa z) psi for all states (delta kick along z, the
 * perturbation of the absorption run in section "van der Waals"). */
int ks_kick(ks_grid *g, void *d_psi, double kappa);

/* d_norms[j] = h^3 sum_g |psi_j(g)|^2 for all nk*nstates states. */
int ks_norms(ks_grid *g, const void *d_psi, double *d_norms);

/* d_gram[k][i][j] = h^3 sum_g conj(psi_ki(g)) psi_kj(g), complex128,
 * nk*nstates*nstates entries (orthonormality check). */
int ks_gram(ks_grid *g, const void *d_psi, void *d_gram);

/* Total energy sum_k w_k sum_s f_s <psi|T + v_ion + V_NL + gauge(t)|psi>
 * + E_x[n], E_x = -(3/4)(3/pi)^(1/3) h^3 sum n^(4/3) when xc == 1,
 * + E_H[n] = 1/2 h^3 sum n v_H[n] when hartree == 1.
 * Synchronises the stream.  Needs a workspace. */
int ks_energy(ks_grid *g, const void *d_psi, const double *d_vion, double t,
              double *out_host);

/* Launch shape of the H.psi kernel: a workgroup owns tile_rows full x-rows
 * of one state and marches through zchunk z-planes; each thread marches
 * rows_per_thread (1 or 2) rows of the tile, ceil(tile_rows /
 * rows_per_thread) apart.  0 keeps the library's choice for that
 * parameter.  KS_E_ARG / KS_E_UNSUPPORTED if the shape does not fit (at
 * most 512 threads of nx * ceil(tile_rows / rows_per_thread), 160 KiB of
 * LDS, 16 halo loads per thread (8 with two rows)).  The workspace size does
 * not depend on the shape.  States, dipoles and densities do not depend on
 * the shape; the norm diagnostics sum per-tile partials, so their last bits
 * do. */
int ks_set_launch(ks_grid *g, int tile_rows, int zchunk, int rows_per_thread);

/* Propagation overlap: with halves = 2 and projectors present, each Taylor
 * exponential runs the first half of the states on the grid's stream and
 * the second half on a second stream of the grid, forked from and joined
 * back into it, so that one half's small projector kernels can run beside
 * the other half's stencil.  1 (the default) runs all states in one chain.
 * Results are the same either way; kernel profiling always runs one chain.
 * KS_E_ARG for other values. */
int ks_set_overlap(ks_grid *g, int halves);

/* out[0] = tile_rows, out[1] = zchunk, out[2] = workgroups per H.psi launch
 * over all states, out[3] = threads per workgroup, out[4] = rows per
 * thread. */
int ks_get_launch(const ks_grid *g, int out[5]);

/* Kernel timing with HIP events on the grid's stream.  After
 * ks_profile_begin(g, capacity, class_mask), every later launch of the
 * H.psi kernel (class 0), of the projector gather (class 1), of the density
 * / reduction kernels (class 2) and of the projector apply (class 3) whose
 * bit is set in class_mask (1 << class) is bracketed by a pair of events,
 * up to `capacity` pairs.  ks_profile_end() waits for the stream, stops
 * recording and returns per class the summed kernel time (ms) and the
 * number of launches timed, in out_ms[4] and out_count[4] (host arrays).
 * Events between launches cost time of their own: time throughput with
 * profiling off, or with only the class of interest on. */
int ks_profile_begin(ks_grid *g, int capacity, int class_mask);
int ks_profile_end(ks_grid *g, double out_ms[4], long out_count[4]);

/* Time only every `every`-th launch of each class (counted from
 * ks_profile_begin; default 1 = all), so that a long run is sampled with
 * few events.  Takes effect at the next ks_profile_begin. */
int ks_profile_every(ks_grid *g, int every);

/* Autotuner: time the four H.psi passes of one Taylor exponential (the
 * three term passes and the final sum, the mix a step runs; projector
 * terms included as they are) on the caller's states `d_psi`
 * ([nk][nstates][N] complex128, read only) over
 * candidate launch shapes (for one and for two rows per thread: the tallest
 * tile of 512 threads, the even split of ny into as many tiles, 3/4, 1/2
 * and 1/4 of it; z-chunks of nz, nz/2, ... down to 8 planes), `reps` timed
 * launches each, and keep the fastest.  Results of every call are the same
 * for every shape; only speed changes.  Synchronises the grid's stream.
 * Writes the chosen (tile rows, z-chunk, rows per thread) to out_shape and
 * its mean time per pass in microseconds to *out_us (either may be NULL).
 * Overwrites the workspace's Taylor buffers; needs a workspace. */
int ks_autotune(ks_grid *g, const void *d_psi, int reps, int out_shape[3],
                double *out_us);

/* ---- batched form ----
 * Several grid objects ("jobs") propagated together: every Taylor pass of
 * all jobs runs as one H.psi launch over the work items of a job table
 * (with one batched projector gather and apply), the density / potential /
 * dipole / norm reductions of all jobs as one launch each, and one ETRS
 * step (the same step as ks_propagate_etrs) is captured once as a HIP graph
 * and replayed.  Results
 * equal those of ks_propagate_etrs on each job alone, for the same launch
 * shapes.  Grids must share the precision, have a workspace, and not be used
 * on their own while the batch exists (the batch sets their stream). */
typedef struct ks_batch ks_batch;

typedef struct {
    ks_grid *grid;
    void *d_psi;           /* the job's states, propagated in place */
    const double *d_vion;  /* must stay valid while the batch exists */
    double dt, t0;
    double *d_dipole;      /* device (max_steps+1)*3 or NULL */
    double *d_norms;       /* device (max_steps+1)*nk*nstates or NULL */
    int max_steps;         /* steps the output buffers have room for */
    int first_step;        /* steps the job has already taken (0: fresh) */
} ks_job;

/* Bind the jobs, build the device job table, and compute the v(t0),
 * dipole(t0) and norms(t0) of every job with first_step 0 (stream-ordered on
 * `stream`).  A job with first_step = m > 0 resumes a trajectory that an
 * earlier batch (or ks_propagate_etrs) left after m steps: its states are
 * psi(t0 + m dt), its grid still holds the potential from the end of step m,
 * step s of the job uses t = t0 + s dt, and its outputs go to rows m+1, ...
 * of d_dipole / d_norms.  The result is bitwise that of one uninterrupted
 * run, so jobs may join and leave (continuous batching). */
int ks_batch_create(const ks_job *jobs, int njobs, void *stream,
                    ks_batch **out);

/* Advance every job by nsteps ETRS steps (KS_E_ARG if a job would pass its
 * max_steps).  The first call with graphs on captures one step.  Does not
 * wait for the device.  A job that records norms and whose norm becomes NaN
 * or Inf is reported as KS_E_NONFINITE (naming the job) by the first
 * ks_batch_step call after the step that produced it has completed, and at
 * the latest by ks_batch_destroy; the steps are not enqueued then. */
int ks_batch_step(ks_batch *b, int nsteps);

/* Graph replay (1, the default) or eager launches (0) for later steps. */
int ks_batch_set_graph(ks_batch *b, int use_graph);

/* Steps job `job` has taken so far. */
int ks_batch_steps_done(const ks_batch *b, int job, int *out);

/* Wait for the stream and free the batch (not the grids).  Returns
 * KS_E_NONFINITE (after freeing) if a job's recorded norm became NaN or Inf
 * and no earlier call has reported it. */
int ks_batch_destroy(ks_batch *b);

/* KS_OK if all n host values are finite, else KS_E_NONFINITE with the
 * index of the first NaN or Inf in ks_last_error() (KS_E_ARG for a NULL
 * pointer or n < 0).  The propagators apply it to the norms they copy back
 * at the end of a call; a caller may apply it to any trace it copies back
 * (dipoles, norms, energies).  Needs no GPU. */
int ks_check_finite(const double *values, long n);

/* Message of the last error on the calling thread ("" if none). */
const char *ks_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* KS_H */
