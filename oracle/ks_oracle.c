/*
 * ks_oracle.c -- plain, slow, FP64 reference of the real-time TDDFT hot path.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or
 * calls this file; only the test-suite, the smoke check and the CPU-baseline
 * leg of the benchmark do.  It shares no source, header or table with the HIP
 * path.
 *
 * What it computes (arXiv:1912.07921, "Octopus, a computational framework for
 * exploring light-driven phenomena ..."):
 *
 *   - the time-dependent Kohn-Sham equations written as a first-order ODE,
 *     d(phi_i)/dt = -i H[n(t),t] phi_i  (section "New propagators for
 *     real-time TDDFT", the ODE system and its right-hand side f_i);
 *   - H = -1/2 Laplacian + v(r,t) (one-body part of eq. Hamiltonian_dipole),
 *     plus non-local pseudopotential projectors (section "Magneto-optics",
 *     the non-local pseudopotential term), plus, for a uniform vector
 *     potential in the dipole approximation, the velocity-gauge kinetic term
 *     of the Volkov Hamiltonian (section "t-SURFF"; section "Thermoelectric
 *     ... currents": E induced by a vector potential A(t));
 *   - the Laplacian and gradient by high-order finite differences on a uniform
 *     real-space grid (section "Periodic systems": FD weights for gradient and
 *     Laplacian);
 *   - Bloch boundary conditions for k-points (section "Periodic systems");
 *   - the enforced-time-reversal-symmetry (ETRS) propagator (section "New
 *     propagators", the list of propagators in Octopus; its use in the
 *     "vdW / HF dimer" absorption run);
 *   - the electron density, the LDA exchange potential (section "Local
 *     domains", E_xc^LDA), the time-dependent dipole d(t) = int r n(r,t) dr
 *     (section "Local domains", the dipole equation) and the delta kick
 *     (section "van der Waals", the HF-dimer absorption run).
 *
 * Readings of what the paper leaves open (each stated once, here):
 *   R1  Laplacian: half-width-4 central stencil with the unique maximal-order
 *       weights {-205/72, 8/5, -1/5, 8/315, -1/560}; gradient weights
 *       {4/5, -1/5, 4/105, -1/280} (Fornberg 1988).  Values outside a
 *       non-periodic axis are zero; along a periodic axis
 *       psi(i + N) = exp(i k_a L_a) psi(i).
 *   R2  Grid coordinates: x_i = (i - (N-1)/2) h on a non-periodic axis,
 *       x_i = i h on a periodic axis (cell length L = N h).
 *   R3  Kleinman-Bylander projectors: sphere S_a = {g : |r_g - R_a|^2 < rc^2}
 *       (nearest image on periodic axes), p_{a,lm}(g) = P_lm(r) *
 *       exp(-r^2 / (2 sigma^2)) * (1 - r^2/rc^2)^2 with real solid harmonics
 *       s: 1; p: x, y, z; d: xy, yz, zx, x^2-y^2, 3z^2-r^2; each normalised
 *       so that h^3 sum_g p^2 = 1.  One energy E_{a,l} per (atom, l).  Under
 *       Bloch conditions the gathered projector is p~(g) = p(g) e^{i k.T_g},
 *       T_g the lattice shift bringing r_g into the sphere:
 *       C = h^3 sum_g p~(g) psi(g), (V_NL psi)(g) = sum conj(p~(g)) E C.
 *   R4  Velocity gauge: H = 1/2(-i grad + A)^2 + V = -1/2 Lap - i A.grad
 *       + |A|^2/2 + V for a uniform A(t) (A already divided by c);
 *       A(t) = A0 sin^2(pi t / T) cos(w t) pol for 0 <= t <= T, else 0.
 *   R5  Exponential: 4th-order Taylor series, exp(-i tau H) psi ~
 *       sum_{k=0..4} (-i tau H)^k psi / k!, H frozen during one exponential.
 *   R6  ETRS step: with u_k = H_t^k psi(t),
 *         psi_half = sum (-i dt/2)^k u_k / k!,
 *         psi_pred = sum (-i dt  )^k u_k / k!   (same powers),
 *         v(t+dt)  = v_ion + v_x[n(psi_pred)] (+ v_H, R11),
 *         psi(t+dt) = T4(dt/2, H_{t+dt}) psi_half;
 *       then v is rebuilt from n(psi(t+dt)) for the next step.
 *   R7  LDA exchange only (Dirac/Slater): v_x = -(3 n / pi)^(1/3),
 *       E_x = -(3/4)(3/pi)^(1/3) h^3 sum n^(4/3).  No correlation; no
 *       Hartree unless R11 is switched on.
 *   R8  Density n = sum_k w_k sum_s f_s |psi_ks|^2; dipole d = h^3 sum r n.
 *   R9  Kick: psi <- exp(i kappa z) psi.
 *   R10 CFM4 (the order-four commutator-free Magnus propagator): H(t1),
 *       H(t2) take A(t_i) exactly and the local potential extrapolated
 *       from the potentials at the ends of the most recent steps (cubic
 *       through four points; through the points available in the first
 *       three steps of a run, so the run starts at lower order).  Each
 *       exponential is Taylor-4 of a H(t1) + b H(t2) with step dt.
 *   R11 Hartree potential (optional; the paper names it as part of the
 *       density-dependent potential but prescribes no solver): v_H solves
 *       Lap v_H = -4 pi n.  Finite grid (no periodic axis): free space,
 *       v_H(r_i) = h^3 sum_j n_j G(r_i - r_j), G(r) = 1/|r| for r != 0 and
 *       G(0) = the mean of 1/|r| over the grid cell centred at the origin.
 *       Periodic grid (all axes periodic): v_H(G) = 4 pi n(G) / |G|^2 over
 *       the grid's discrete Fourier frequencies G_a = 2 pi m_a / L_a,
 *       m_a in (-n_a/2, n_a/2], with v_H(G = 0) = 0 (a compensating uniform
 *       background).  Mixed periodicity is not defined.  With R11 on,
 *       v = v_ion + v_H[n] (+ v_x[n]) and E gains E_H = 1/2 h^3 sum n v_H.
 *   R12 Macroscopic current (section "Electric and thermal conductivities",
 *       eq. current_density): J = -(i/Omega) sum_k w_k sum_s f_s
 *       <psi|[H, r]|psi>, Omega = the cell (box) volume n_a h_a.  On the
 *       grid the commutator has the matrix elements H_ij (x_j - x_i), with
 *       x_j - x_i the displacement of the coupled point: m h along the
 *       axis for a stencil tap m (so wrapped taps of a periodic axis count
 *       their true displacement), and the difference of the two points'
 *       images inside the atom's sphere for the projector term.  The local
 *       potential is diagonal and drops out.
 *   R13 Spectra from traces sampled at t_n = n dt, n = 0 .. nt-1 (section
 *       "van der Waals", the absorption run; section "Electric and thermal
 *       conductivities", eq. FT), with the trapezoid rule (weights 1/2 at
 *       both ends) and a damping window e^{-gamma t}:
 *       polarizability alpha(w) = (1/kappa) dt sum w_n (d(t_n) - d(0))
 *       e^{+i w t_n} e^{-gamma t_n} after a kick kappa, strength function
 *       S(w) = (2 w / pi) Im alpha(w) (integrates to the electron count);
 *       conductivity sigma(w) = (1/E0) dt sum w_n J(t_n) e^{-i w t_n}
 *       e^{-gamma t_n}.
 *
 * Layout: psi is complex double, [nk][nstates][nz][ny][nx], x fastest.
 */
#include <complex.h>
#include <math.h>
#include <stdlib.h>
#include <string.h>
#include <omp.h>

#ifndef M_PI
#define M_PI 3.14159265358979323846
#endif

typedef double complex cplx;

/* Input description; mirrors what a user of the method supplies. */
typedef struct {
    int n[3];            /* nx, ny, nz */
    double h[3];         /* spacing per axis, bohr */
    int periodic[3];     /* 1: Bloch-periodic axis, 0: zero boundary */
    int nk;              /* number of k-points */
    const double *kpts;  /* nk*3, bohr^-1 */
    const double *kw;    /* nk weights */
    int nstates;         /* states per k-point */
    const double *occ;   /* nstates occupations */
    int natoms;
    const double *pos;   /* natoms*3 */
    const int *lmax;     /* natoms, 0..2 */
    const double *rc;    /* natoms */
    const double *sigma; /* natoms */
    const double *E;     /* natoms*3, E[a*3 + l] in Hartree */
    int xc;              /* 0: none, 1: LDA exchange */
    double laser[6];     /* A0, omega, T, pol_x, pol_y, pol_z */
    int hartree;         /* 0: none, 1: + Hartree potential (R11) */
} orc_desc;

typedef struct {
    int npts;
    int nproj;
    int *idx;       /* grid index of each sphere point */
    int *lshift;    /* lattice shift (in cells) per point: 3 ints */
    double *p;      /* nproj * npts, normalised real projector values */
    int l[9];       /* angular momentum of each projector */
    double E[9];    /* KB energy of each projector */
} orc_atom;

typedef struct {
    orc_desc d;
    long N;
    double *kpts, *kw, *occ;
    orc_atom *atoms;
} orc_system;

void orc_destroy(orc_system *S);

/* FD weights (reading R1). */
static const double LAP_C[5] = {-205.0 / 72.0, 8.0 / 5.0, -1.0 / 5.0,
                                8.0 / 315.0, -1.0 / 560.0};
static const double GRAD_D[5] = {0.0, 4.0 / 5.0, -1.0 / 5.0, 4.0 / 105.0,
                                 -1.0 / 280.0};

static double coord(const orc_system *S, int axis, int i)
{
    if (S->d.periodic[axis])
        return i * S->d.h[axis];
    return (i - 0.5 * (S->d.n[axis] - 1)) * S->d.h[axis];
}

static double cell_len(const orc_system *S, int axis)
{
    return S->d.n[axis] * S->d.h[axis];
}

static double dvol(const orc_system *S)
{
    return S->d.h[0] * S->d.h[1] * S->d.h[2];
}

/* Real solid harmonics in the order s; px py pz; dxy dyz dzx dx2-y2 d3z2-r2. */
static double solid_harmonic(int j, double x, double y, double z)
{
    switch (j) {
    case 0: return 1.0;
    case 1: return x;
    case 2: return y;
    case 3: return z;
    case 4: return x * y;
    case 5: return y * z;
    case 6: return z * x;
    case 7: return x * x - y * y;
    case 8: return 3.0 * z * z - (x * x + y * y + z * z);
    }
    return 0.0;
}

static int proj_l(int j)
{
    return j == 0 ? 0 : (j < 4 ? 1 : 2);
}

/* Build the sphere and the normalised projector table of one atom (R3). */
static int build_atom(orc_system *S, int a, orc_atom *A)
{
    const orc_desc *d = &S->d;
    double X[3] = {d->pos[3 * a], d->pos[3 * a + 1], d->pos[3 * a + 2]};
    double rc = d->rc[a], sg = d->sigma[a];
    int lmax = d->lmax[a];
    A->nproj = (lmax + 1) * (lmax + 1);
    for (int ax = 0; ax < 3; ++ax)
        if (d->periodic[ax] && !(rc < 0.5 * cell_len(S, ax)))
            return -1;
    /* first pass: count */
    long cnt = 0;
    for (int z = 0; z < d->n[2]; ++z)
        for (int y = 0; y < d->n[1]; ++y)
            for (int x = 0; x < d->n[0]; ++x) {
                int ii[3] = {x, y, z};
                double r2 = 0.0;
                for (int ax = 0; ax < 3; ++ax) {
                    double dd = coord(S, ax, ii[ax]) - X[ax];
                    if (d->periodic[ax]) {
                        double L = cell_len(S, ax);
                        dd -= L * nearbyint(dd / L);
                    }
                    r2 += dd * dd;
                }
                if (r2 < rc * rc)
                    ++cnt;
            }
    A->npts = (int)cnt;
    A->idx = malloc(sizeof(int) * (cnt ? cnt : 1));
    A->lshift = malloc(sizeof(int) * 3 * (cnt ? cnt : 1));
    A->p = calloc((size_t)A->nproj * (cnt ? cnt : 1), sizeof(double));
    long q = 0;
    for (int z = 0; z < d->n[2]; ++z)
        for (int y = 0; y < d->n[1]; ++y)
            for (int x = 0; x < d->n[0]; ++x) {
                int ii[3] = {x, y, z};
                double r[3], r2 = 0.0;
                int sh[3] = {0, 0, 0};
                for (int ax = 0; ax < 3; ++ax) {
                    double dd = coord(S, ax, ii[ax]) - X[ax];
                    if (d->periodic[ax]) {
                        double L = cell_len(S, ax);
                        double m = nearbyint(dd / L);
                        dd -= L * m;
                        sh[ax] = -(int)m; /* r_g + T_g - R = dd, T_g = sh*L */
                    }
                    r[ax] = dd;
                    r2 += dd * dd;
                }
                if (!(r2 < rc * rc))
                    continue;
                A->idx[q] = (z * d->n[1] + y) * d->n[0] + x;
                for (int ax = 0; ax < 3; ++ax)
                    A->lshift[3 * q + ax] = sh[ax];
                double w = 1.0 - r2 / (rc * rc);
                double radial = exp(-r2 / (2.0 * sg * sg)) * w * w;
                for (int j = 0; j < A->nproj; ++j)
                    A->p[(size_t)j * cnt + q] =
                        solid_harmonic(j, r[0], r[1], r[2]) * radial;
                ++q;
            }
    for (int j = 0; j < A->nproj; ++j) {
        double s = 0.0;
        for (long i = 0; i < cnt; ++i)
            s += A->p[(size_t)j * cnt + i] * A->p[(size_t)j * cnt + i];
        s *= dvol(S);
        double nrm = s > 0.0 ? 1.0 / sqrt(s) : 0.0;
        for (long i = 0; i < cnt; ++i)
            A->p[(size_t)j * cnt + i] *= nrm;
        A->l[j] = proj_l(j);
        A->E[j] = d->E[3 * a + A->l[j]];
    }
    return 0;
}

orc_system *orc_create(const orc_desc *d)
{
    if (d->n[0] < 1 || d->n[1] < 1 || d->n[2] < 1 || d->nk < 1 ||
        d->nstates < 0 || d->natoms < 0)
        return NULL;
    {
        const int np = d->periodic[0] + d->periodic[1] + d->periodic[2];
        if (d->hartree && np != 0 && np != 3)
            return NULL;   /* R11 is defined for these two cases only */
    }
    orc_system *S = calloc(1, sizeof(orc_system));
    S->d = *d;
    S->N = (long)d->n[0] * d->n[1] * d->n[2];
    S->kpts = malloc(sizeof(double) * 3 * d->nk);
    S->kw = malloc(sizeof(double) * d->nk);
    S->occ = malloc(sizeof(double) * (d->nstates ? d->nstates : 1));
    for (int i = 0; i < 3 * d->nk; ++i)
        S->kpts[i] = d->kpts ? d->kpts[i] : 0.0;
    for (int i = 0; i < d->nk; ++i)
        S->kw[i] = d->kw ? d->kw[i] : 1.0 / d->nk;
    for (int i = 0; i < d->nstates; ++i)
        S->occ[i] = d->occ ? d->occ[i] : 2.0;
    S->d.kpts = S->kpts;
    S->d.kw = S->kw;
    S->d.occ = S->occ;
    S->atoms = calloc(d->natoms ? d->natoms : 1, sizeof(orc_atom));
    for (int a = 0; a < d->natoms; ++a) {
        if (build_atom(S, a, &S->atoms[a]) != 0) {
            S->d.natoms = a; /* free what exists */
            orc_destroy(S);
            return NULL;
        }
    }
    /* the caller's atom arrays are not kept */
    S->d.pos = NULL;
    S->d.lmax = NULL;
    S->d.rc = S->d.sigma = S->d.E = NULL;
    return S;
}

void orc_destroy(orc_system *S)
{
    if (!S)
        return;
    for (int a = 0; a < S->d.natoms; ++a) {
        free(S->atoms[a].idx);
        free(S->atoms[a].lshift);
        free(S->atoms[a].p);
    }
    free(S->atoms);
    free(S->kpts);
    free(S->kw);
    free(S->occ);
    free(S);
}

long orc_npoints(const orc_system *S) { return S->N; }

int orc_atom_npts(const orc_system *S, int a) { return S->atoms[a].npts; }

/* Copy atom a's grid indices and its nproj*npts projector table out. */
void orc_atom_table(const orc_system *S, int a, int *idx, double *p)
{
    const orc_atom *A = &S->atoms[a];
    memcpy(idx, A->idx, sizeof(int) * A->npts);
    memcpy(p, A->p, sizeof(double) * A->nproj * A->npts);
}

/* psi at integer position (x,y,z) under the boundary rule of R1. */
static cplx fetch(const orc_system *S, const cplx *psi, int k, int x, int y,
                  int z);
void orc_laser_A(const orc_system *S, double t, double A[3]);

/*
 * [H, r_axis] psi for one state on k-point k (R12): out_i =
 * sum_j H_ij (x_j - x_i) psi_j.
 */
static void comm_r_one(const orc_system *S, int k, const double A[3],
                       int axis, const cplx *psi, cplx *out)
{
    const orc_desc *d = &S->d;
    const double h = d->h[axis];
    for (int z = 0; z < d->n[2]; ++z)
        for (int y = 0; y < d->n[1]; ++y)
            for (int x = 0; x < d->n[0]; ++x) {
                long g = ((long)z * d->n[1] + y) * d->n[0] + x;
                cplx acc = 0.0;
                for (int m = 1; m <= 4; ++m) {
                    int p[3] = {x, y, z}, q[3] = {x, y, z};
                    p[axis] += m;
                    q[axis] -= m;
                    cplx fp = fetch(S, psi, k, p[0], p[1], p[2]);
                    cplx fm = fetch(S, psi, k, q[0], q[1], q[2]);
                    /* kinetic taps -1/2 c_m / h^2 at displacements +-m h */
                    acc += (-0.5 * LAP_C[m] / (h * h)) * (m * h) * (fp - fm);
                    /* gauge taps -i A d_m / h (+m) and +i A d_m / h (-m) */
                    acc += (-I * A[axis] * GRAD_D[m] / h) * (m * h) * fp +
                           (I * A[axis] * GRAD_D[m] / h) * (-m * h) * fm;
                }
                out[g] = acc;
            }
    /* projectors: sum_g V_ig (X_g - X_i) psi_g with X the coordinate of the
     * point's image inside the sphere */
    double h3 = dvol(S);
    for (int a = 0; a < d->natoms; ++a) {
        const orc_atom *At = &S->atoms[a];
        for (int j = 0; j < At->nproj; ++j) {
            const double *p = At->p + (size_t)j * At->npts;
            cplx C = 0.0, D = 0.0;
            for (int i = 0; i < At->npts; ++i) {
                const int *sh = At->lshift + 3 * i;
                double kT = 0.0;
                for (int ax = 0; ax < 3; ++ax)
                    kT += S->kpts[3 * k + ax] * sh[ax] * cell_len(S, ax);
                const long gi = At->idx[i];
                const int c[3] = {(int)(gi % d->n[0]),
                                  (int)((gi / d->n[0]) % d->n[1]),
                                  (int)(gi / ((long)d->n[0] * d->n[1]))};
                const double X = coord(S, axis, c[axis]) +
                                 sh[axis] * cell_len(S, axis);
                C += p[i] * cexp(I * kT) * psi[gi];
                D += p[i] * cexp(I * kT) * X * psi[gi];
            }
            C *= h3;
            D *= h3;
            for (int i = 0; i < At->npts; ++i) {
                const int *sh = At->lshift + 3 * i;
                double kT = 0.0;
                for (int ax = 0; ax < 3; ++ax)
                    kT += S->kpts[3 * k + ax] * sh[ax] * cell_len(S, ax);
                const long gi = At->idx[i];
                const int c[3] = {(int)(gi % d->n[0]),
                                  (int)((gi / d->n[0]) % d->n[1]),
                                  (int)(gi / ((long)d->n[0] * d->n[1]))};
                const double X = coord(S, axis, c[axis]) +
                                 sh[axis] * cell_len(S, axis);
                out[gi] += p[i] * cexp(-I * kT) * At->E[j] * (D - X * C);
            }
        }
    }
}

/* [H(t), r_axis] applied to ns states of k-point k (R12), for tests. */
void orc_comm_r(const orc_system *S, int k, double t, int axis, int ns,
                const cplx *in, cplx *out)
{
    double A[3];
    orc_laser_A(S, t, A);
#pragma omp parallel for
    for (int s = 0; s < ns; ++s)
        comm_r_one(S, k, A, axis, in + (size_t)s * S->N,
                   out + (size_t)s * S->N);
}

/*
 * Macroscopic current J(t) of all nk*ns states (R12): J_a = -(i/Omega)
 * sum_k w_k sum_s f_s h^3 sum_g conj(psi) [H, r_a] psi.  Jc receives the
 * complex values (the imaginary parts vanish up to rounding).
 */
void orc_current(const orc_system *S, const cplx *psi, double t, cplx Jc[3])
{
    const long N = S->N;
    const int ns = S->d.nstates;
    double A[3];
    orc_laser_A(S, t, A);
    const double omega = cell_len(S, 0) * cell_len(S, 1) * cell_len(S, 2);
    cplx *tmp = malloc(sizeof(cplx) * N);
    for (int ax = 0; ax < 3; ++ax) {
        cplx acc = 0.0;
        for (int k = 0; k < S->d.nk; ++k)
            for (int s = 0; s < ns; ++s) {
                const cplx *p = psi + ((size_t)k * ns + s) * N;
                comm_r_one(S, k, A, ax, p, tmp);
                cplx e = 0.0;
                for (long g = 0; g < N; ++g)
                    e += conj(p[g]) * tmp[g];
                acc += S->kw[k] * S->occ[s] * dvol(S) * e;
            }
        Jc[ax] = -I * acc / omega;
    }
    free(tmp);
}

/* Strength function S(w) of a kicked run from the dipole component d
 * (nt samples) along the kick (R13). */
void orc_strength_function(const double *d, int nt, double dt, double kappa,
                           double gamma, const double *w, int nw,
                           double *out)
{
    for (int i = 0; i < nw; ++i) {
        cplx alpha = 0.0;
        for (int n = 0; n < nt; ++n) {
            const double wt = (n == 0 || n == nt - 1) ? 0.5 : 1.0;
            const double t = n * dt;
            alpha += wt * (d[n] - d[0]) * cexp(I * w[i] * t) *
                     exp(-gamma * t);
        }
        alpha *= dt / kappa;
        out[i] = 2.0 * w[i] / M_PI * cimag(alpha);
    }
}

/* Conductivity sigma(w) from a current component J (nt samples) after an
 * impulsive field E0 (R13). */
void orc_conductivity(const double *J, int nt, double dt, double E0,
                      double gamma, const double *w, int nw, cplx *out)
{
    for (int i = 0; i < nw; ++i) {
        cplx acc = 0.0;
        for (int n = 0; n < nt; ++n) {
            const double wt = (n == 0 || n == nt - 1) ? 0.5 : 1.0;
            const double t = n * dt;
            acc += wt * J[n] * cexp(-I * w[i] * t) * exp(-gamma * t);
        }
        out[i] = acc * dt / E0;
    }
}

/* psi at integer position (x,y,z) under the boundary rule of R1. */
static cplx fetch(const orc_system *S, const cplx *psi, int k, int x, int y,
                  int z)
{
    int ii[3] = {x, y, z};
    cplx ph = 1.0;
    for (int ax = 0; ax < 3; ++ax) {
        int n = S->d.n[ax];
        if (ii[ax] >= 0 && ii[ax] < n)
            continue;
        if (!S->d.periodic[ax])
            return 0.0;
        int w = (int)floor((double)ii[ax] / n);
        ii[ax] -= w * n;
        ph *= cexp(I * S->kpts[3 * k + ax] * cell_len(S, ax) * w);
    }
    return ph * psi[((long)ii[2] * S->d.n[1] + ii[1]) * S->d.n[0] + ii[0]];
}

/* H psi for one state on one k-point (R1, R3, R4). */
static void apply_h_one(const orc_system *S, const double *v, int k,
                        const double A[3], const cplx *psi, cplx *hpsi)
{
    const orc_desc *d = &S->d;
    double a2 = 0.5 * (A[0] * A[0] + A[1] * A[1] + A[2] * A[2]);
    for (int z = 0; z < d->n[2]; ++z)
        for (int y = 0; y < d->n[1]; ++y)
            for (int x = 0; x < d->n[0]; ++x) {
                long g = ((long)z * d->n[1] + y) * d->n[0] + x;
                cplx lap = 0.0, grad[3] = {0.0, 0.0, 0.0};
                for (int ax = 0; ax < 3; ++ax) {
                    cplx s = LAP_C[0] * psi[g];
                    cplx t = 0.0;
                    for (int m = 1; m <= 4; ++m) {
                        int p[3] = {x, y, z}, q[3] = {x, y, z};
                        p[ax] += m;
                        q[ax] -= m;
                        cplx fp = fetch(S, psi, k, p[0], p[1], p[2]);
                        cplx fm = fetch(S, psi, k, q[0], q[1], q[2]);
                        s += LAP_C[m] * (fp + fm);
                        t += GRAD_D[m] * (fp - fm);
                    }
                    lap += s / (d->h[ax] * d->h[ax]);
                    grad[ax] = t / d->h[ax];
                }
                cplx out = -0.5 * lap + (v[g] + a2) * psi[g];
                out += -I * (A[0] * grad[0] + A[1] * grad[1] + A[2] * grad[2]);
                hpsi[g] = out;
            }
    /* non-local part */
    double h3 = dvol(S);
    for (int a = 0; a < d->natoms; ++a) {
        const orc_atom *At = &S->atoms[a];
        for (int j = 0; j < At->nproj; ++j) {
            const double *p = At->p + (size_t)j * At->npts;
            cplx C = 0.0;
            for (int i = 0; i < At->npts; ++i) {
                const int *sh = At->lshift + 3 * i;
                double kT = 0.0;
                for (int ax = 0; ax < 3; ++ax)
                    kT += S->kpts[3 * k + ax] * sh[ax] * cell_len(S, ax);
                C += p[i] * cexp(I * kT) * psi[At->idx[i]];
            }
            C *= h3;
            for (int i = 0; i < At->npts; ++i) {
                const int *sh = At->lshift + 3 * i;
                double kT = 0.0;
                for (int ax = 0; ax < 3; ++ax)
                    kT += S->kpts[3 * k + ax] * sh[ax] * cell_len(S, ax);
                hpsi[At->idx[i]] += p[i] * cexp(-I * kT) * At->E[j] * C;
            }
        }
    }
}

/* H psi for ns consecutive states of k-point k.  psi, hpsi: ns*N. */
void orc_apply_h(const orc_system *S, const double *v, int k,
                 const double A[3], int ns, const cplx *psi, cplx *hpsi)
{
    long N = S->N;
#pragma omp parallel for schedule(dynamic, 1)
    for (int s = 0; s < ns; ++s)
        apply_h_one(S, v, k, A, psi + (size_t)s * N, hpsi + (size_t)s * N);
}

/* Uniform vector potential of the laser pulse at time t (R4). */
void orc_laser_A(const orc_system *S, double t, double A[3])
{
    const double *L = S->d.laser;
    double a = 0.0;
    if (L[0] != 0.0 && t >= 0.0 && t <= L[2]) {
        double s = sin(M_PI * t / L[2]);
        a = L[0] * s * s * cos(L[1] * t);
    }
    A[0] = a * L[3];
    A[1] = a * L[4];
    A[2] = a * L[5];
}

/* n(g) = sum_k w_k sum_s f_s |psi_ks(g)|^2 (R8).  psi: nk*ns*N. */
void orc_density(const orc_system *S, const cplx *psi, double *rho)
{
    long N = S->N;
    int ns = S->d.nstates;
#pragma omp parallel for
    for (long g = 0; g < N; ++g) {
        double n = 0.0;
        for (int k = 0; k < S->d.nk; ++k)
            for (int s = 0; s < ns; ++s) {
                cplx c = psi[((size_t)k * ns + s) * N + g];
                n += S->kw[k] * S->occ[s] * (creal(c) * creal(c) +
                                             cimag(c) * cimag(c));
            }
        rho[g] = n;
    }
}

/*
 * Integral of 1/|r| over the box [0,a] x [0,b] x [0,c] (one corner at the
 * origin), in closed form: with R = |(a, b, c)|,
 *   bc ln((a+R)/|(b,c)|) + ca ln((b+R)/|(c,a)|) + ab ln((c+R)/|(a,b)|)
 *   - a^2/2 atan(bc/(aR)) - b^2/2 atan(ca/(bR)) - c^2/2 atan(ab/(cR)).
 */
static double corner_integral(double a, double b, double c)
{
    double R = sqrt(a * a + b * b + c * c);
    return b * c * log((a + R) / sqrt(b * b + c * c)) +
           c * a * log((b + R) / sqrt(c * c + a * a)) +
           a * b * log((c + R) / sqrt(a * a + b * b)) -
           0.5 * a * a * atan(b * c / (a * R)) -
           0.5 * b * b * atan(c * a / (b * R)) -
           0.5 * c * c * atan(a * b / (c * R));
}

/* G(0) of R11: the mean of 1/|r| over the cell of sides h centred at 0. */
double orc_coulomb_cell_mean(const double h[3])
{
    return 8.0 * corner_integral(0.5 * h[0], 0.5 * h[1], 0.5 * h[2]) /
           (h[0] * h[1] * h[2]);
}

/*
 * One-dimensional discrete Fourier transform along `axis` of the complex
 * array f (layout [nz][ny][nx]), in place: f(m) <- sum_j f(j) e^{sgn 2 pi i
 * j m / n}.  Written out term by term (O(n) per output).
 */
static void dft_axis(const int n[3], cplx *f, int axis, int sgn)
{
    const int na = n[axis];
    const long stride = axis == 0 ? 1 : axis == 1 ? n[0] : (long)n[0] * n[1];
    const long nlines = (long)n[0] * n[1] * n[2] / na;
#pragma omp parallel
    {
        cplx *in = malloc(sizeof(cplx) * na);
        cplx *tw = malloc(sizeof(cplx) * na);
        for (int j = 0; j < na; ++j)
            tw[j] = cexp(sgn * 2.0 * M_PI * I * j / na);
#pragma omp for
        for (long line = 0; line < nlines; ++line) {
            /* first element of the line: the index with coordinate 0 on
             * `axis` and the other two taken from `line` */
            long base;
            if (axis == 0)
                base = line * na;
            else if (axis == 1)
                base = (line / n[0]) * n[0] * n[1] + line % n[0];
            else
                base = line;
            for (int j = 0; j < na; ++j)
                in[j] = f[base + j * stride];
            for (int m = 0; m < na; ++m) {
                cplx acc = 0.0;
                for (int j = 0; j < na; ++j)
                    acc += in[j] * tw[(long)j * m % na];
                f[base + m * stride] = acc;
            }
        }
        free(in);
        free(tw);
    }
}

/* v_H at grid point i of a finite grid (R11): h^3 sum_j n_j G(r_i - r_j). */
static double free_space_point(const orc_system *S, const double *rho,
                               long i, double g0)
{
    const int *n = S->d.n;
    const double *h = S->d.h;
    const int xi = (int)(i % n[0]), yi = (int)((i / n[0]) % n[1]);
    const int zi = (int)(i / ((long)n[0] * n[1]));
    double acc = 0.0;
    for (long j = 0; j < S->N; ++j) {
        const int xj = (int)(j % n[0]), yj = (int)((j / n[0]) % n[1]);
        const int zj = (int)(j / ((long)n[0] * n[1]));
        const double dx = (xi - xj) * h[0], dy = (yi - yj) * h[1];
        const double dz = (zi - zj) * h[2];
        const double r2 = dx * dx + dy * dy + dz * dz;
        acc += rho[j] * (r2 > 0.0 ? 1.0 / sqrt(r2) : g0);
    }
    return dvol(S) * acc;
}

/* v_H of a finite grid at the listed grid points only (count of them);
 * returns -1 on a grid with a periodic axis. */
int orc_hartree_at(const orc_system *S, const double *rho, const long *idx,
                   int count, double *out)
{
    if (S->d.periodic[0] || S->d.periodic[1] || S->d.periodic[2])
        return -1;
    const double g0 = orc_coulomb_cell_mean(S->d.h);
#pragma omp parallel for schedule(dynamic)
    for (int c = 0; c < count; ++c)
        out[c] = free_space_point(S, rho, idx[c], g0);
    return 0;
}

/*
 * Hartree potential v_H[n] of R11 into vh.  Returns 0, or -1 when the grid
 * has mixed periodicity.
 */
int orc_hartree(const orc_system *S, const double *rho, double *vh)
{
    const int *n = S->d.n;
    const double *h = S->d.h;
    const long N = S->N;
    const int np = S->d.periodic[0] + S->d.periodic[1] + S->d.periodic[2];
    if (np == 0) {
        const double g0 = orc_coulomb_cell_mean(h);
#pragma omp parallel for schedule(static)
        for (long i = 0; i < N; ++i)
            vh[i] = free_space_point(S, rho, i, g0);
        return 0;
    }
    if (np != 3)
        return -1;
    cplx *f = malloc(sizeof(cplx) * N);
    for (long i = 0; i < N; ++i)
        f[i] = rho[i];
    for (int a = 0; a < 3; ++a)
        dft_axis(n, f, a, -1);
    for (long i = 0; i < N; ++i) {
        const int m[3] = {(int)(i % n[0]), (int)((i / n[0]) % n[1]),
                          (int)(i / ((long)n[0] * n[1]))};
        double G2 = 0.0;
        for (int a = 0; a < 3; ++a) {
            const int ma = 2 * m[a] > n[a] ? m[a] - n[a] : m[a];
            const double Ga = 2.0 * M_PI * ma / (n[a] * h[a]);
            G2 += Ga * Ga;
        }
        f[i] = G2 > 0.0 ? f[i] * (4.0 * M_PI / G2) : 0.0;
    }
    for (int a = 0; a < 3; ++a)
        dft_axis(n, f, a, +1);
    for (long i = 0; i < N; ++i)
        vh[i] = creal(f[i]) / N;
    free(f);
    return 0;
}

/* E_H = 1/2 h^3 sum n v_H (R11). */
double orc_hartree_energy(const orc_system *S, const double *rho)
{
    double *vh = malloc(sizeof(double) * S->N);
    orc_hartree(S, rho, vh);
    double s = 0.0;
    for (long g = 0; g < S->N; ++g)
        s += rho[g] * vh[g];
    free(vh);
    return 0.5 * dvol(S) * s;
}

/* v = v_ion + v_x[n] (R7) + v_H[n] (R11); rho may be NULL (neither
 * density term). */
void orc_vlocal(const orc_system *S, const double *vion, const double *rho,
                double *v)
{
    for (long g = 0; g < S->N; ++g) {
        double vx = 0.0;
        if (S->d.xc == 1 && rho)
            vx = -cbrt(3.0 * rho[g] / M_PI);
        v[g] = vion[g] + vx;
    }
    if (S->d.hartree && rho) {
        double *vh = malloc(sizeof(double) * S->N);
        orc_hartree(S, rho, vh);
        for (long g = 0; g < S->N; ++g)
            v[g] += vh[g];
        free(vh);
    }
}

/* E_x = -(3/4)(3/pi)^(1/3) h^3 sum n^(4/3) (R7). */
double orc_exchange_energy(const orc_system *S, const double *rho)
{
    double s = 0.0;
    for (long g = 0; g < S->N; ++g)
        s += pow(rho[g], 4.0 / 3.0);
    return -0.75 * cbrt(3.0 / M_PI) * dvol(S) * s;
}

/* d = h^3 sum_g r_g n_g (R8). */
void orc_dipole(const orc_system *S, const double *rho, double d[3])
{
    d[0] = d[1] = d[2] = 0.0;
    for (int z = 0; z < S->d.n[2]; ++z)
        for (int y = 0; y < S->d.n[1]; ++y)
            for (int x = 0; x < S->d.n[0]; ++x) {
                double n = rho[((long)z * S->d.n[1] + y) * S->d.n[0] + x];
                d[0] += coord(S, 0, x) * n;
                d[1] += coord(S, 1, y) * n;
                d[2] += coord(S, 2, z) * n;
            }
    for (int i = 0; i < 3; ++i)
        d[i] *= dvol(S);
}

/* psi <- exp(i kappa z) psi for all nk*ns states (R9). */
void orc_kick(const orc_system *S, cplx *psi, double kappa)
{
    long N = S->N;
    int tot = S->d.nk * S->d.nstates;
    for (int s = 0; s < tot; ++s)
        for (int z = 0; z < S->d.n[2]; ++z) {
            cplx ph = cexp(I * kappa * coord(S, 2, z));
            for (long i = 0; i < (long)S->d.n[0] * S->d.n[1]; ++i)
                psi[(size_t)s * N + (long)z * S->d.n[0] * S->d.n[1] + i] *= ph;
        }
}

/* ||psi_s||^2 = h^3 sum |psi|^2 for nk*ns states. */
void orc_norms(const orc_system *S, const cplx *psi, double *norms)
{
    long N = S->N;
    int tot = S->d.nk * S->d.nstates;
    for (int s = 0; s < tot; ++s) {
        double a = 0.0;
        for (long g = 0; g < N; ++g) {
            cplx c = psi[(size_t)s * N + g];
            a += creal(c) * creal(c) + cimag(c) * cimag(c);
        }
        norms[s] = a * dvol(S);
    }
}

/* G_ij = <psi_i|psi_j> = h^3 sum conj(psi_i) psi_j, per k: nk*ns*ns. */
void orc_gram(const orc_system *S, const cplx *psi, cplx *G)
{
    long N = S->N;
    int ns = S->d.nstates;
    for (int k = 0; k < S->d.nk; ++k)
#pragma omp parallel for collapse(2)
        for (int i = 0; i < ns; ++i)
            for (int j = 0; j < ns; ++j) {
                const cplx *a = psi + ((size_t)k * ns + i) * N;
                const cplx *b = psi + ((size_t)k * ns + j) * N;
                cplx s = 0.0;
                for (long g = 0; g < N; ++g)
                    s += conj(a[g]) * b[g];
                G[((size_t)k * ns + i) * ns + j] = s * dvol(S);
            }
}

/*
 * Total energy of R7: sum_k w_k sum_s f_s <psi|T + v_ion + V_NL + gauge|psi>
 * + E_x[n] + E_H[n].  Work space: ns*N complex.
 */
double orc_energy(const orc_system *S, const cplx *psi, const double *vion,
                  double t)
{
    long N = S->N;
    int ns = S->d.nstates;
    double A[3];
    orc_laser_A(S, t, A);
    cplx *hp = malloc(sizeof(cplx) * (size_t)ns * N);
    double e = 0.0;
    for (int k = 0; k < S->d.nk; ++k) {
        const cplx *pk = psi + (size_t)k * ns * N;
        orc_apply_h(S, vion, k, A, ns, pk, hp);
        for (int s = 0; s < ns; ++s) {
            cplx acc = 0.0;
            for (long g = 0; g < N; ++g)
                acc += conj(pk[(size_t)s * N + g]) * hp[(size_t)s * N + g];
            e += S->kw[k] * S->occ[s] * creal(acc) * dvol(S);
        }
    }
    free(hp);
    if (S->d.xc == 1 || S->d.hartree) {
        double *rho = malloc(sizeof(double) * N);
        orc_density(S, psi, rho);
        if (S->d.xc == 1)
            e += orc_exchange_energy(S, rho);
        if (S->d.hartree)
            e += orc_hartree_energy(S, rho);
        free(rho);
    }
    return e;
}

/*
 * One 4th-order Taylor exponential (R5): out = sum_{k=0..4} (-i tau H)^k in/k!
 * for ns states of k-point k.  out may alias in.
 */
void orc_taylor4(const orc_system *S, const double *v, int k,
                 const double A[3], double tau, int ns, const cplx *in,
                 cplx *out)
{
    size_t M = (size_t)ns * S->N;
    cplx *term = malloc(sizeof(cplx) * M);
    cplx *next = malloc(sizeof(cplx) * M);
    cplx *acc = malloc(sizeof(cplx) * M);
    memcpy(term, in, sizeof(cplx) * M);
    memcpy(acc, in, sizeof(cplx) * M);
    for (int p = 1; p <= 4; ++p) {
        orc_apply_h(S, v, k, A, ns, term, next);
        for (size_t i = 0; i < M; ++i) {
            term[i] = (-I * tau / p) * next[i];
            acc[i] += term[i];
        }
    }
    memcpy(out, acc, sizeof(cplx) * M);
    free(term);
    free(next);
    free(acc);
}

/*
 * ETRS propagation (R6) of all nk*ns states, in place, for nsteps steps of
 * dt from t0.  v is rebuilt from n(psi) at t0 first.  dipole: (nsteps+1)*3
 * or NULL; norms: (nsteps+1)*nk*ns or NULL.  Returns 0.
 */
int orc_propagate_etrs(const orc_system *S, cplx *psi, const double *vion,
                       int nsteps, double dt, double t0, double *dipole,
                       double *norms)
{
    long N = S->N;
    int ns = S->d.nstates, nk = S->d.nk;
    size_t M = (size_t)ns * N;
    double *rho = malloc(sizeof(double) * N);
    double *v = malloc(sizeof(double) * N);
    double *vnext = malloc(sizeof(double) * N);
    cplx *u = malloc(sizeof(cplx) * M * 5);         /* u_0 .. u_4 */
    cplx *half = malloc(sizeof(cplx) * M * nk);
    cplx *pred = malloc(sizeof(cplx) * M * nk);

    orc_density(S, psi, rho);
    orc_vlocal(S, vion, (S->d.xc || S->d.hartree) ? rho : NULL, v);
    if (dipole)
        orc_dipole(S, rho, dipole);
    if (norms)
        orc_norms(S, psi, norms);

    /* Taylor coefficients (-i dt/2)^p / p! and (-i dt)^p / p! */
    cplx ch[5], cp[5];
    {
        double fact = 1.0;
        for (int p = 0; p <= 4; ++p) {
            if (p > 0)
                fact *= p;
            ch[p] = cpow(-I * dt / 2, p) / fact;
            cp[p] = cpow(-I * dt, p) / fact;
        }
    }
    for (int step = 0; step < nsteps; ++step) {
        double t = t0 + step * dt;
        double At[3], An[3];
        orc_laser_A(S, t, At);
        orc_laser_A(S, t + dt, An);
        /* powers u_k = H_t^k psi(t); half and predictor sums */
        for (int k = 0; k < nk; ++k) {
            cplx *pk = psi + (size_t)k * M;
            memcpy(u, pk, sizeof(cplx) * M);
            for (int p = 1; p <= 4; ++p)
                orc_apply_h(S, v, k, At, ns, u + (p - 1) * M, u + p * M);
            for (size_t i = 0; i < M; ++i) {
                cplx sh = 0.0, sp = 0.0;
                for (int p = 0; p <= 4; ++p) {
                    sh += ch[p] * u[p * M + i];
                    sp += cp[p] * u[p * M + i];
                }
                half[(size_t)k * M + i] = sh;
                pred[(size_t)k * M + i] = sp;
            }
        }
        /* Hamiltonian at t+dt from the predicted density */
        orc_density(S, pred, rho);
        orc_vlocal(S, vion, (S->d.xc || S->d.hartree) ? rho : NULL, vnext);
        for (int k = 0; k < nk; ++k)
            orc_taylor4(S, vnext, k, An, dt / 2, ns, half + (size_t)k * M,
                        psi + (size_t)k * M);
        /* potential for the next step from the new density */
        orc_density(S, psi, rho);
        orc_vlocal(S, vion, (S->d.xc || S->d.hartree) ? rho : NULL, v);
        if (dipole)
            orc_dipole(S, rho, dipole + 3 * (step + 1));
        if (norms)
            orc_norms(S, psi, norms + (size_t)(step + 1) * nk * ns);
    }
    free(rho);
    free(v);
    free(vnext);
    free(u);
    free(half);
    free(pred);
    return 0;
}

/*
 * Lagrange weights for the value at x of the polynomial through the points
 * x_j = -j (j = 0 .. h-1), i.e. extrapolation from the h most recent steps
 * (unit step) to the offset x: L_j(x) = prod_{m != j} (x + m) / (m - j).
 */
static void lagrange_back(int h, double x, double *L)
{
    for (int j = 0; j < h; ++j) {
        double w = 1.0;
        for (int m = 0; m < h; ++m)
            if (m != j)
                w *= (x + m) / (double)(m - j);
        L[j] = w;
    }
}

/*
 * CFM4 propagation (section "New propagators for real-time TDDFT", the
 * order-four commutator-free Magnus expansion with two exponentials):
 *   psi(t+dt) = exp(-i dt (a1 H(t1) + a2 H(t2)))
 *               exp(-i dt (a2 H(t1) + a1 H(t2))) psi(t),
 *   a1,2 = (3 -+ 2 sqrt 3)/12, t1,2 = t + (1/2 -+ sqrt(3)/6) dt.
 * H(t_i) uses A(t_i) exactly and a local potential extrapolated from the
 * potentials v(t), v(t - dt), ... of the most recent steps (up to four
 * points: the cubic through them; fewer at the start of a run, R10-CFM).
 * Each exponential is a Taylor-4 series (R5) of the operator
 * a H(t1) + b H(t2) applied literally as a H(t1) psi + b H(t2) psi, with
 * the step dt.  v is rebuilt from n(psi) at the end of every step.
 * Arguments as for orc_propagate_etrs.
 */
int orc_propagate_cfm4(const orc_system *S, cplx *psi, const double *vion,
                       int nsteps, double dt, double t0, double *dipole,
                       double *norms)
{
    long N = S->N;
    int ns = S->d.nstates, nk = S->d.nk;
    size_t M = (size_t)ns * N;
    const double a1 = (3.0 - 2.0 * sqrt(3.0)) / 12.0;
    const double a2 = (3.0 + 2.0 * sqrt(3.0)) / 12.0;
    const double c1 = 0.5 - sqrt(3.0) / 6.0, c2 = 0.5 + sqrt(3.0) / 6.0;
    double *rho = malloc(sizeof(double) * N);
    double *hist = malloc(sizeof(double) * N * 4);   /* v(t - j dt) */
    double *v1 = malloc(sizeof(double) * N);
    double *v2 = malloc(sizeof(double) * N);
    cplx *term = malloc(sizeof(cplx) * M);
    cplx *h1 = malloc(sizeof(cplx) * M);
    cplx *h2 = malloc(sizeof(cplx) * M);
    cplx *acc = malloc(sizeof(cplx) * M);
    int nhist = 0;

    orc_density(S, psi, rho);
    orc_vlocal(S, vion, (S->d.xc || S->d.hartree) ? rho : NULL, hist);
    nhist = 1;
    if (dipole)
        orc_dipole(S, rho, dipole);
    if (norms)
        orc_norms(S, psi, norms);
    for (int step = 0; step < nsteps; ++step) {
        double t = t0 + step * dt;
        double A1[3], A2[3], L1[4], L2[4];
        orc_laser_A(S, t + c1 * dt, A1);
        orc_laser_A(S, t + c2 * dt, A2);
        lagrange_back(nhist, c1, L1);
        lagrange_back(nhist, c2, L2);
        for (long g = 0; g < N; ++g) {
            double s1 = 0.0, s2 = 0.0;
            for (int j = 0; j < nhist; ++j) {
                s1 += L1[j] * hist[(size_t)j * N + g];
                s2 += L2[j] * hist[(size_t)j * N + g];
            }
            v1[g] = s1;
            v2[g] = s2;
        }
        /* the right-hand exponential first: weights (a2, a1), then (a1, a2) */
        const double wa[2] = {a2, a1}, wb[2] = {a1, a2};
        for (int e = 0; e < 2; ++e) {
            for (int k = 0; k < nk; ++k) {
                cplx *pk = psi + (size_t)k * M;
                memcpy(term, pk, sizeof(cplx) * M);
                memcpy(acc, pk, sizeof(cplx) * M);
                for (int p = 1; p <= 4; ++p) {
                    orc_apply_h(S, v1, k, A1, ns, term, h1);
                    orc_apply_h(S, v2, k, A2, ns, term, h2);
                    for (size_t i = 0; i < M; ++i) {
                        term[i] = (-I * dt / p) * (wa[e] * h1[i] +
                                                   wb[e] * h2[i]);
                        acc[i] += term[i];
                    }
                }
                memcpy(pk, acc, sizeof(cplx) * M);
            }
        }
        /* v(t + dt) from the new density, newest first in the history */
        for (int j = (nhist < 4 ? nhist : 3); j > 0; --j)
            memcpy(hist + (size_t)j * N, hist + (size_t)(j - 1) * N,
                   sizeof(double) * N);
        if (nhist < 4)
            ++nhist;
        orc_density(S, psi, rho);
        orc_vlocal(S, vion, (S->d.xc || S->d.hartree) ? rho : NULL, hist);
        if (dipole)
            orc_dipole(S, rho, dipole + 3 * (step + 1));
        if (norms)
            orc_norms(S, psi, norms + (size_t)(step + 1) * nk * ns);
    }
    free(rho);
    free(hist);
    free(v1);
    free(v2);
    free(term);
    free(h1);
    free(h2);
    free(acc);
    return 0;
}

int orc_num_threads(void) { return omp_get_max_threads(); }
