// C ABI of libks: argument checks, projector set-up, workspace layout and the
// sequencing of the ETRS step (section "New propagators for real-time TDDFT")
// over the gfx950 kernels of ks_kernels.hip.
#include "../../include/ks.h"
#include "ks_internal.h"
#include "ks_observe.h"
#include "ks_poisson.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <map>
#include <mutex>
#include <tuple>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>
#include <array>
#include <vector>

using namespace ks;

namespace {

thread_local std::string g_err;

int fail(int code, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

#define KS_HIP(call)                                                         \
    do {                                                                     \
        hipError_t e_ = (call);                                              \
        if (e_ != hipSuccess)                                                \
            return fail(KS_E_HIP, "%s: %s", #call, hipGetErrorString(e_));   \
    } while (0)

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

}  // namespace

struct ks_grid {
    Geo geo;
    int nk = 1, ns = 1, stot = 1;
    std::vector<double> kpts, kw, occ, wocc;
    std::vector<double2> kph;   // [nk][3] exp(i k_a L_a)
    int xc = 0;
    int hartree = 0;
    bool nonlin = false;        // the potential depends on the density
    PoissonPlan pp;             // Hartree solver (hartree == 1)
    double laser[6] = {0, 0, 0, 0, 0, 0};
    bool mixed = false;
    hipStream_t stream = nullptr;
    int device = 0;

    // owned device memory
    std::vector<void *> owned;
    double *d_v = nullptr;       // current local potential
    double2 *d_kph = nullptr;
    double *d_wocc = nullptr;
    bool vloc_set = false;

    // projectors
    ProjDev pj;
    int natoms = 0;
    long total_pts = 0;
    long nhull = 0;
    std::vector<int> h_npts, h_nproj;

    // launch shape
    int TY = 1, zchunk = 1, ntile_y = 1, nzc = 1, rpt = 1;

    // device bytes of the tables allocated by dev_alloc
    size_t owned_bytes = 0;

    // workspace
    char *ws = nullptr;
    size_t ws_bytes = 0;
    struct {
        size_t t1, t2, t3, half, npart, normpart, D, W, Dpart, rho, vpred,
            dpart, gpart, dotpart, xpart, step, vhist, veff, pwork, vh, cpart,
            cnl, normchk, v32, total;
    } lay{};
    int ntiles_max = 64;
    int nchunk = 1;
    int gram_ksplit = 16;
    int norm_chunks = 64;

    // kernel timing
    std::vector<hipEvent_t> ev;   // 2 per record
    std::vector<int> ev_class;
    int ev_used = 0;
    bool profiling = false;
    int prof_mask = 0xf;
    int prof_every = 1;          // time one launch in prof_every per class
    long prof_seen[4] = {0, 0, 0, 0};
    // second stream: the states are propagated in two halves whose pass
    // chains overlap (one half's projector kernels beside the other half's
    // stencil)
    hipStream_t side = nullptr;
    hipEvent_t fork_ev = nullptr, join_ev = nullptr;
    int halves = 1;
    // end-of-call norms copied back by the propagators (pinned, stot)
    double *h_norms = nullptr;
};

namespace {

template <class T> int dev_alloc(ks_grid *g, T **p, size_t count)
{
    void *q = nullptr;
    size_t bytes = std::max<size_t>(count * sizeof(T), 16);
    hipError_t e = hipMalloc(&q, bytes);
    if (e != hipSuccess)
        return fail(KS_E_OOM, "hipMalloc(%zu): %s", bytes,
                    hipGetErrorString(e));
    g->owned.push_back(q);
    g->owned_bytes += bytes;
    *p = static_cast<T *>(q);
    return KS_OK;
}

template <class T>
int dev_upload(ks_grid *g, T **p, const std::vector<T> &host)
{
    int rc = dev_alloc(g, p, host.size());
    if (rc)
        return rc;
    if (!host.empty())
        KS_HIP(hipMemcpy(*p, host.data(), host.size() * sizeof(T),
                         hipMemcpyHostToDevice));
    return KS_OK;
}

double axis_coord(const Geo &G, int axis, int i)
{
    int n = axis == 0 ? G.nx : (axis == 1 ? G.ny : G.nz);
    return G.per[axis] ? i * G.h[axis] : (i - 0.5 * (n - 1)) * G.h[axis];
}

double solid_harm(int j, double x, double y, double z)
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
    default: return 3.0 * z * z - (x * x + y * y + z * z);
    }
}

// Build the sphere point lists of every atom (grid index, packed
// coordinates, lattice shift), the projector normalisations, the hull rows
// and the per-chunk atom lists of the hull, and upload them.
int build_projectors(ks_grid *g, const ks_grid_desc *d)
{
    const Geo &G = g->geo;
    const int na = d->natoms;
    g->natoms = na;
    g->pj.natoms = na;
    if (na == 0)
        return KS_OK;
    if (na > 65535)
        return fail(KS_E_UNSUPPORTED, "more than 65535 atoms");
    const int n3[3] = {G.nx, G.ny, G.nz};
    std::vector<int> nproj(na), npts(na);
    std::vector<long> ioff(na);
    std::vector<int> sidx, sxyz, sshift;
    std::vector<double> EjN2((size_t)na * kMaxProj, 0.0);
    std::vector<double4> apos(na);
    std::vector<double2> arad(na);
    const double h3 = G.h[0] * G.h[1] * G.h[2];
    for (int a = 0; a < na; ++a) {
        const int lmax = d->lmax[a];
        const double rc = d->rc[a], sg = d->sigma[a];
        const double X[3] = {d->pos[3 * a], d->pos[3 * a + 1],
                             d->pos[3 * a + 2]};
        if (lmax < 0 || lmax > 2)
            return fail(KS_E_ARG, "atom %d: lmax %d not in 0..2", a, lmax);
        if (!(rc > 0.0) || !(sg > 0.0))
            return fail(KS_E_ARG, "atom %d: rc and sigma must be > 0", a);
        for (int ax = 0; ax < 3; ++ax)
            if (G.per[ax] && !(rc < 0.5 * n3[ax] * G.h[ax]))
                return fail(KS_E_UNSUPPORTED,
                            "atom %d: rc must be below half the cell", a);
        nproj[a] = (lmax + 1) * (lmax + 1);
        apos[a] = make_double4(X[0], X[1], X[2], rc * rc);
        arad[a] = make_double2(1.0 / (2.0 * sg * sg), 1.0 / (rc * rc));
        // index ranges (unwrapped) of the bounding box of the sphere
        int lo[3], hi[3];
        for (int ax = 0; ax < 3; ++ax) {
            double o = axis_coord(G, ax, 0);
            lo[ax] = (int)std::floor((X[ax] - rc - o) / G.h[ax]) - 1;
            hi[ax] = (int)std::ceil((X[ax] + rc - o) / G.h[ax]) + 1;
            if (!G.per[ax]) {
                lo[ax] = std::max(lo[ax], 0);
                hi[ax] = std::min(hi[ax], n3[ax] - 1);
            }
        }
        ioff[a] = (long)sidx.size();
        double norm2[kMaxProj] = {0};
        for (int iz = lo[2]; iz <= hi[2]; ++iz)
            for (int iy = lo[1]; iy <= hi[1]; ++iy)
                for (int ix = lo[0]; ix <= hi[0]; ++ix) {
                    const int ii[3] = {ix, iy, iz};
                    int w[3], wr[3];
                    double r[3], r2 = 0.0;
                    for (int ax = 0; ax < 3; ++ax) {
                        int n = n3[ax];
                        int q = ii[ax];
                        int ww = q >= 0 ? q / n : -((-q + n - 1) / n);
                        w[ax] = ww;
                        wr[ax] = q - ww * n;
                        r[ax] = axis_coord(G, ax, wr[ax]) +
                                ww * n * G.h[ax] - X[ax];
                        r2 += r[ax] * r[ax];
                    }
                    if (!(r2 < rc * rc))
                        continue;
                    sidx.push_back((wr[2] * G.ny + wr[1]) * G.nx + wr[0]);
                    sxyz.push_back(wr[0] | (wr[1] << 10) | (wr[2] << 20));
                    sshift.push_back((w[0] & 0xff) | ((w[1] & 0xff) << 8) |
                                     ((w[2] & 0xff) << 16));
                    const double win = 1.0 - r2 / (rc * rc);
                    const double rad = std::exp(-r2 / (2.0 * sg * sg)) *
                                       win * win;
                    for (int j = 0; j < nproj[a]; ++j) {
                        const double pv = solid_harm(j, r[0], r[1], r[2]) *
                                          rad;
                        norm2[j] += pv * pv;
                    }
                }
        npts[a] = (int)(sidx.size() - ioff[a]);
        for (int j = 0; j < nproj[a]; ++j) {
            const double s2 = norm2[j] * h3;
            const double nj2 = s2 > 0.0 ? 1.0 / s2 : 0.0;   // N_j^2
            const int l = j == 0 ? 0 : (j < 4 ? 1 : 2);
            EjN2[(size_t)a * kMaxProj + j] = nj2 * h3 * d->E[3 * a + l];
        }
    }
    g->total_pts = (long)sidx.size();
    g->nchunk = gather_chunks(*std::max_element(npts.begin(), npts.end()));
    // gather work items (atom, chunk), ordered by the first point's plane
    std::vector<int2> gpairs;
    {
        const int cp = gather_chunk_points();
        std::vector<std::tuple<int, int, int>> key;   // (plane, atom, chunk)
        for (int a = 0; a < na; ++a)
            for (int c = 0; (long)c * cp < npts[a]; ++c)
                key.emplace_back(sxyz[ioff[a] + (long)c * cp] >> 20, a, c);
        std::sort(key.begin(), key.end());
        for (const auto &k : key)
            gpairs.push_back(make_int2(std::get<1>(k), std::get<2>(k)));
    }
    g->h_npts = npts;
    g->h_nproj = nproj;

    // hull rows: x range covered by spheres in each (z, y) row
    const long nrows = (long)G.nz * G.ny;
    std::vector<int> xlo(nrows, G.nx), xhi(nrows, -1);
    for (size_t i = 0; i < sidx.size(); ++i) {
        const long row = sidx[i] / G.nx;
        const int x = sidx[i] % G.nx;
        xlo[row] = std::min(xlo[row], x);
        xhi[row] = std::max(xhi[row], x);
    }
    std::vector<int4> rowinfo(nrows);
    std::vector<int> hxyz;
    long nhull = 0;
    for (long row = 0; row < nrows; ++row) {
        rowinfo[row] = make_int4(xlo[row], xhi[row], (int)nhull, 0);
        if (xhi[row] >= xlo[row]) {
            const int y = (int)(row % G.ny), z = (int)(row / G.ny);
            for (int x = xlo[row]; x <= xhi[row]; ++x)
                hxyz.push_back(x | (y << 10) | (z << 20));
            nhull += xhi[row] - xlo[row] + 1;
        }
    }
    if (nhull >= (1L << 31))
        return fail(KS_E_UNSUPPORTED, "projector hull too large");
    const int nhch = (int)((nhull + kHullChunk - 1) / kHullChunk);
    std::vector<std::vector<int>> chunk_atoms(nhch);
    for (int a = 0; a < na; ++a) {
        int last = -1;
        for (int i = 0; i < npts[a]; ++i) {
            const int gg = sidx[ioff[a] + i];
            const long row = gg / G.nx;
            const int x = gg % G.nx;
            const long hh = rowinfo[row].z + (x - rowinfo[row].x);
            const int c = (int)(hh / kHullChunk);
            if (c != last &&
                (chunk_atoms[c].empty() || chunk_atoms[c].back() != a))
                chunk_atoms[c].push_back(a);
            last = c;
        }
    }
    std::vector<int> hc_off(nhch + 1, 0), hc_atoms;
    for (int c = 0; c < nhch; ++c) {
        hc_off[c + 1] = hc_off[c] + (int)chunk_atoms[c].size();
        hc_atoms.insert(hc_atoms.end(), chunk_atoms[c].begin(),
                        chunk_atoms[c].end());
    }
    g->nhull = nhull;
    // hull entries: every sphere point as (hull point, atom), grouped by
    // hull point with atoms in index order; the apply's phase code is the
    // negated wrap of the point's image
    const long nent = (long)sidx.size();
    std::vector<int> he_off(nhull + 1, 0), he_slot(nent), he_code(nent);
    std::vector<int2> ent(nent);
    {
        std::vector<long> hof(nent);
        for (int a = 0; a < na; ++a)
            for (int i = 0; i < npts[a]; ++i) {
                const long k = ioff[a] + i;
                const int gg = sidx[k];
                const long row = gg / G.nx;
                hof[k] = rowinfo[row].z + (gg % G.nx - rowinfo[row].x);
                ++he_off[hof[k] + 1];
            }
        for (long h = 0; h < nhull; ++h)
            he_off[h + 1] += he_off[h];
        std::vector<int> fill(he_off.begin(), he_off.end() - 1);
        for (int a = 0; a < na; ++a)
            for (int i = 0; i < npts[a]; ++i) {
                const long k = ioff[a] + i;
                const long h = hof[k];
                const int e = fill[h]++;
                const int c = (int)(h / kHullChunk);
                const auto &ca = chunk_atoms[c];
                he_slot[e] = (int)(std::find(ca.begin(), ca.end(), a) -
                                   ca.begin());
                const int w = sshift[k];
                int code = 0;
                for (int ax = 0; ax < 3; ++ax) {
                    const int t = (int)(signed char)((w >> (8 * ax)) & 0xff);
                    code |= ((-t) & 0xff) << (8 * ax);
                }
                he_code[e] = code;
                ent[e] = make_int2(a, i);
            }
    }

    int *d_nproj, *d_npts, *d_sidx, *d_sxyz, *d_sshift, *d_hxyz, *d_hc_off,
        *d_hc_atoms, *d_he_off, *d_he_slot, *d_he_code;
    int2 *d_ent, *d_gpairs = nullptr;
    double *d_he_p;
    long *d_ioff;
    double *d_EjN2;
    double4 *d_apos;
    double2 *d_arad;
    int4 *d_rowinfo;
    int rc;
    if ((rc = dev_upload(g, &d_nproj, nproj)) ||
        (rc = dev_upload(g, &d_npts, npts)) ||
        (rc = dev_upload(g, &d_ioff, ioff)) ||
        (rc = dev_upload(g, &d_sidx, sidx)) ||
        (rc = dev_upload(g, &d_sxyz, sxyz)) ||
        (rc = dev_upload(g, &d_sshift, sshift)) ||
        (rc = dev_upload(g, &d_EjN2, EjN2)) ||
        (rc = dev_upload(g, &d_apos, apos)) ||
        (rc = dev_upload(g, &d_arad, arad)) ||
        (rc = dev_upload(g, &d_rowinfo, rowinfo)) ||
        (rc = dev_upload(g, &d_hxyz, hxyz)) ||
        (rc = dev_upload(g, &d_hc_off, hc_off)) ||
        (rc = dev_upload(g, &d_hc_atoms, hc_atoms)) ||
        (rc = dev_upload(g, &d_he_off, he_off)) ||
        (rc = dev_upload(g, &d_he_slot, he_slot)) ||
        (rc = dev_upload(g, &d_he_code, he_code)) ||
        (rc = dev_upload(g, &d_ent, ent)) ||
        (!gpairs.empty() && (rc = dev_upload(g, &d_gpairs, gpairs))) ||
        (rc = dev_alloc(g, &d_he_p, (size_t)nent * kMaxProj)))
        return rc;
    g->pj.nproj = d_nproj;
    g->pj.npts = d_npts;
    g->pj.ioff = d_ioff;
    g->pj.sidx = d_sidx;
    g->pj.ngpairs = (int)gpairs.size();
    g->pj.gpairs = d_gpairs;
    g->pj.sxyz = d_sxyz;
    g->pj.sshift = d_sshift;
    g->pj.EjN2 = d_EjN2;
    g->pj.apos = d_apos;
    g->pj.arad = d_arad;
    g->pj.rowinfo = d_rowinfo;
    g->pj.nhull = (int)nhull;
    g->pj.hxyz = d_hxyz;
    g->pj.nhchunk = nhch;
    g->pj.hc_off = d_hc_off;
    g->pj.hc_atoms = d_hc_atoms;
    g->pj.he_off = d_he_off;
    g->pj.he_slot = d_he_slot;
    g->pj.he_code = d_he_code;
    g->pj.he_p = d_he_p;
    // projector values of the entries, evaluated on the device as the
    // gather evaluates them (synchronous: creation is)
    KS_HIP(launch_hull_table(g->pj, G, d_ent, nent, d_he_p, g->stream));
    KS_HIP(hipStreamSynchronize(g->stream));
    return KS_OK;
}

// LDS bytes of one H.psi workgroup.
size_t lds_for(const ks_grid *g, int TY, int zchunk)
{
    return hpsi_lds_bytes(g->geo.nx, TY, g->natoms > 0 ? zchunk : 0,
                          g->mixed);
}

// Launch shape: rows per tile TY (up to 512 threads, one or two rows per
// thread) and planes per z-chunk (the full z extent unless that leaves fewer
// than ~4 workgroups per CU).  Either may be forced (> 0) by the caller.
bool tile_ok(const ks_grid *g, int TY, int rpt)
{
    const Geo &G = g->geo;
    if (TY < 1 || TY > G.ny || rpt < 1 || rpt > 2)
        return false;
    const int nthr = hpsi_threads(G.nx, TY, rpt);
    if (nthr > kRowThreads)
        return false;
    // the kernel holds at most 16 halo loads per thread and plane (8 when
    // it marches two rows per thread)
    const int dyn = 2 * kHalf * G.nx +
                    (G.per[0] ? 2 * kHalf * (TY + 2 * kHalf) : 0);
    const int hm = (dyn + nthr - 1) / nthr;
    return hm <= (rpt == 2 ? 8 : 16);
}

int set_tiles(ks_grid *g, int TY, int zchunk, int rpt)
{
    const Geo &G = g->geo;
    const bool auto_rpt = rpt <= 0, auto_ty = TY <= 0;
    if (auto_rpt)
        rpt = (TY > 0 && G.nx * TY <= kRowThreads) ? 1 : (g->mixed ? 1 : 2);
    for (;;) {
        if (auto_ty) {
            // the tallest tile that fits the threads and the default LDS
            // share: the 8 halo rows are then the smallest fraction of what
            // it loads
            TY = std::max(1, std::min(G.ny, rpt * kRowThreads / G.nx));
            while (TY > 1 &&
                   (!tile_ok(g, TY, rpt) ||
                    lds_for(g, TY, std::min(G.nz, 16)) > kLdsDefault))
                --TY;
        }
        // two rows per thread allow 8 halo loads per thread and plane:
        // the wrapped columns of a wide periodic row exceed that at any
        // height, and one row per thread then takes it
        if (auto_rpt && rpt == 2 && !tile_ok(g, TY, rpt)) {
            rpt = 1;
            continue;
        }
        break;
    }
    if (!tile_ok(g, TY, rpt))
        return fail(KS_E_ARG, "tile height %d with %d rows per thread "
                    "invalid for nx=%d ny=%d", TY, rpt, G.nx, G.ny);
    const int ntile_y = (G.ny + TY - 1) / TY;
    if (zchunk <= 0) {
        // about two workgroups per CU over the launch, chunks of at least
        // 32 planes (the z-halo of 8 planes stays a small fraction)
        const long per_state = ntile_y;
        int nzc = (int)std::max<long>(1, 512 / std::max<long>(1, per_state *
                                                                  g->stot));
        nzc = std::min(nzc, std::max(1, G.nz / 32));
        zchunk = (G.nz + nzc - 1) / nzc;
        // keep the default LDS share where a one-plane chunk would meet it;
        // wider rows (nx above ~300 in FP64) exceed it at any chunk, and
        // then only the LDS of the CU bounds the chunk (shorter chunks
        // would only re-read more z-halo planes)
        const size_t cap = lds_for(g, TY, 1) <= kLdsDefault ? kLdsDefault
                                                             : kLdsBudget;
        while (zchunk > 1 && lds_for(g, TY, zchunk) > cap)
            zchunk = (zchunk + 1) / 2;
    }
    zchunk = std::min(zchunk, G.nz);
    if (lds_for(g, TY, zchunk) > kLdsBudget)
        return fail(KS_E_UNSUPPORTED, "tile needs %zu bytes of LDS",
                    lds_for(g, TY, zchunk));
    const int nzc = (G.nz + zchunk - 1) / zchunk;
    if ((long)ntile_y * nzc * g->stot >= (1L << 31))
        return fail(KS_E_UNSUPPORTED, "too many workgroups");
    g->TY = TY;
    g->rpt = rpt;
    g->ntile_y = ntile_y;
    g->zchunk = zchunk;
    g->nzc = nzc;
    return KS_OK;
}

void layout(ks_grid *g)
{
    const size_t N = g->geo.N, S = g->stot;
    const size_t tb = S * N * (g->mixed ? 8 : 16);
    size_t off = 0;
    auto take = [&](size_t bytes) {
        size_t o = off;
        off += align256(std::max<size_t>(bytes, 16));
        return o;
    };
    // norm partials sized for the finest launch shape (one row, one plane
    // per tile), so that the workspace does not depend on the shape
    g->ntiles_max = std::max(g->geo.ny * g->geo.nz, g->norm_chunks);
    const size_t ndb = density_blocks((long)N);
    g->lay.t1 = take(tb);
    g->lay.t2 = take(tb);
    g->lay.t3 = take(tb);
    g->lay.half = take(S * N * 16);
    g->lay.npart = take(S * N * 8);
    g->lay.normpart = take(S * g->ntiles_max * 8);
    g->lay.D = take(S * std::max(1, g->natoms) * kMaxProj * 16);
    g->lay.W = take(S * std::max<size_t>(1, g->nhull) * 16);
    g->lay.Dpart = take(S * std::max(1, g->natoms) * g->nchunk * kMaxProj *
                        16);
    g->lay.rho = take(N * 8);
    g->lay.vpred = take(N * 8);
    g->lay.dpart = take(ndb * 3 * 8);
    // Gram: split the grid so that about 2048 workgroups share the work
    // (gram_tile x gram_tile state tiles per k-point), each slice at least
    // 512 points
    {
        const long nt = (g->ns + gram_tile(g->ns) - 1) / gram_tile(g->ns);
        const long tiles = nt * nt * g->nk;
        const long want = std::max<long>(1, (2048 + tiles - 1) / tiles);
        const long most = std::max<long>(1, (long)N / 512);
        g->gram_ksplit = (int)std::max<long>(1, std::min(want, most));
    }
    g->lay.gpart = take((size_t)g->gram_ksplit * g->nk * g->ns * g->ns * 16);
    g->lay.dotpart = take(S * g->norm_chunks * 16);
    g->lay.xpart = take(ndb * 8);
    g->lay.step = take(sizeof(int));
    g->lay.vhist = take(4 * N * 8);
    g->lay.veff = take(N * 8);
    g->lay.pwork = take(g->hartree ? g->pp.work_elems * 16 : 0);
    g->lay.vh = take(g->hartree ? N * 8 : 0);
    g->lay.cpart = take(S * (size_t)g->geo.ny * g->geo.nz * 3 * 8);
    g->lay.cnl = take(S * std::max(1, g->natoms) * 3 * 8);
    g->lay.normchk = take(S * 8);
    g->lay.v32 = take(g->mixed ? N * 4 : 0);
    g->lay.total = off;
}

template <class T> T *wsp(ks_grid *g, size_t off)
{
    return reinterpret_cast<T *>(g->ws + off);
}

// The density kernel (with a.vout: v_out = v_ion + v_x[n]) followed, on a
// grid with the Hartree term, by v_out += v_H[n].
int density_potential(ks_grid *g, DArgs a, hipStream_t st)
{
    const bool hart = g->hartree && a.vout && a.nsrc > 0;
    if (hart && !a.rho)
        a.rho = wsp<double>(g, g->lay.rho);
    KS_HIP(launch_density(a, st));
    if (hart)
        KS_HIP(launch_hartree(g->pp, g->geo, a.rho, a.vout, true,
                              wsp<double2>(g, g->lay.pwork), st));
    return KS_OK;
}

#define KS_TRY(call)                                                         \
    do {                                                                     \
        const int rc_ = (call);                                              \
        if (rc_)                                                             \
            return rc_;                                                      \
    } while (0)

// Event pair around one launch of class c (0 H.psi, 1 projector gather,
// 2 reductions, 3 projector apply).
struct Timed {
    ks_grid *g;
    int slot = -1;
    Timed(ks_grid *gg, int c) : g(gg)
    {
        if (g->profiling && ((g->prof_mask >> c) & 1) &&
            g->prof_seen[c]++ % g->prof_every == 0 &&
            g->ev_used < (int)g->ev_class.size()) {
            slot = g->ev_used++;
            g->ev_class[slot] = c;
            (void)hipEventRecord(g->ev[2 * slot], g->stream);
        }
    }
    ~Timed()
    {
        if (slot >= 0)
            (void)hipEventRecord(g->ev[2 * slot + 1], g->stream);
    }
};

void laser_A(const ks_grid *g, double t, double A[3])
{
    const double *L = g->laser;
    double a = 0.0;
    if (L[0] != 0.0 && t >= 0.0 && t <= L[2]) {
        double s = std::sin(M_PI * t / L[2]);
        a = L[0] * s * s * std::cos(L[1] * t);
    }
    A[0] = a * L[3];
    A[1] = a * L[4];
    A[2] = a * L[5];
}

HArgs base_hargs(ks_grid *g)
{
    HArgs a;
    a.geo = g->geo;
    a.kph = g->d_kph;
    a.nstates = g->ns;
    a.wocc = g->d_wocc;
    if (g->natoms > 0 && g->nhull > 0) {
        a.rowinfo = g->pj.rowinfo;
        a.nhull = (int)g->nhull;
        if (g->ws)
            a.W = g->ws + g->lay.W;
    }
    a.TY = g->TY;
    a.rpt = g->rpt;
    a.zchunk = g->zchunk;
    a.ntile_y = g->ntile_y;
    a.nzc = g->nzc;
    return a;
}

GArgs base_gargs(ks_grid *g)
{
    GArgs a;
    a.geo = g->geo;
    a.kph = g->d_kph;
    a.nstates = g->ns;
    a.pj = g->pj;
    a.nchunk = g->nchunk;
    if (g->ws) {
        a.Dpart = g->ws + g->lay.Dpart;
        a.W = g->ws + g->lay.W;
    }
    return a;
}

int need_ws(const ks_grid *g)
{
    if (!g->ws)
        return fail(KS_E_STATE, "no workspace set (ks_set_workspace)");
    return KS_OK;
}

// One Taylor-4 exponential of H (potential v, vector potential A) with
// step tau applied to all states in `in`: t_j = (-i tau / j) H t_{j-1};
// the last pass writes out = in + t1 + t2 + t3 + t4 (mode kFinal) or also the
// predictor density (kFinalPred).
// Weights of the polynomial through the values at x_j = -j (j < h, unit
// steps back from now) evaluated at x: extrapolation of the potential.
void lagrange_back(int h, double x, double L[4])
{
    for (int j = 0; j < h; ++j) {
        double w = 1.0;
        for (int m = 0; m < h; ++m)
            if (m != j)
                w *= (x + m) / (double)(m - j);
        L[j] = w;
    }
}

double half_a2(const double A[3])
{
    return 0.5 * (A[0] * A[0] + A[1] * A[1] + A[2] * A[2]);
}

// The four passes of one Taylor exponential for states [s0, s0 + ns) on
// stream st: every buffer is offset to the first of those states.
int exp_chain(ks_grid *g, hipStream_t st, int s0, int ns, const double2 *in,
              double2 *out, const double *v, const double A[3],
              double a2half, double tau, int final_mode, double *npart,
              double *normpart)
{
    const bool mx = g->mixed;
    const size_t N = g->geo.N;
    const size_t tsz = mx ? 8 : 16;     // Taylor terms and projector data
    const size_t na = std::max(1, g->natoms);
    auto off = [](void *p, size_t bytes) {
        return static_cast<void *>(static_cast<char *>(p) + bytes);
    };
    void *tb[3];
    for (int k = 0; k < 3; ++k)
        tb[k] = off(g->ws + (k == 0 ? g->lay.t1 : k == 1 ? g->lay.t2
                                                        : g->lay.t3),
                    (size_t)s0 * N * tsz);
    in += (size_t)s0 * N;
    out += (size_t)s0 * N;
    HArgs a = base_hargs(g);
    a.sg0 = s0;
    a.v = v;
    if (mx)
        a.v32 = wsp<float>(g, g->lay.v32);   // filled by taylor_exponential
    a.A[0] = A[0];
    a.A[1] = A[1];
    a.A[2] = A[2];
    a.a2half = a2half;
    if (a.W)
        a.W = off(const_cast<void *>(a.W), (size_t)s0 * g->nhull * tsz);
    GArgs ga = base_gargs(g);
    ga.sg0 = s0;
    ga.D = off(g->ws + g->lay.D, (size_t)s0 * na * kMaxProj * tsz);
    if (ga.W)
        ga.W = off(ga.W, (size_t)s0 * g->nhull * tsz);
    if (ga.Dpart)
        ga.Dpart = off(ga.Dpart,
                       (size_t)s0 * na * g->nchunk * kMaxProj * tsz);
    const void *cur = in;
    for (int j = 1; j <= 4; ++j) {
        const bool f64 = (j == 1) || !mx;
        ga.in = cur;
        if (g->natoms > 0) {
            {
                Timed tm(g, 1);
                KS_HIP(launch_gather(mx, f64, ga, ns, st));
            }
            Timed tm(g, 3);
            KS_HIP(launch_kbapply(mx, ga, ns, st));
        }
        a.in = cur;
        a.cre = 0.0;
        a.cim = -tau / j;
        if (j < 4) {
            a.out = tb[j - 1];
            {
                Timed tm(g, 0);
                KS_HIP(launch_hpsi(kTerm, mx, f64, a, ns, st));
            }
            cur = tb[j - 1];
        } else {
            a.out = out;
            a.base = in;
            a.t1 = tb[0];
            a.t2 = tb[1];
            a.npart = npart ? npart + (size_t)s0 * N : nullptr;
            a.normpart = normpart
                             ? normpart + (size_t)s0 * g->ntile_y * g->nzc
                             : nullptr;
            Timed tm(g, 0);
            KS_HIP(launch_hpsi(final_mode, mx, false, a, ns, st));
        }
    }
    return KS_OK;
}

// End of a propagation call: the norms after its last step (row nsteps of
// d_norms, or finalized from the last step's partials into the workspace)
// are copied back and checked; KS_E_NONFINITE names the first state whose
// norm is NaN or Inf.  Synchronises the stream.
int check_end_norms(ks_grid *g, int nsteps, const double *d_norms,
                    const double *normpart)
{
    if (nsteps < 1)
        return KS_OK;
    const int S = g->stot;
    const double *src = d_norms ? d_norms + (size_t)nsteps * S : nullptr;
    if (!src) {
        double *chk = wsp<double>(g, g->lay.normchk);
        const double h3 = g->geo.h[0] * g->geo.h[1] * g->geo.h[2];
        KS_HIP(launch_norm_finalize(normpart, S, g->ntile_y * g->nzc, h3,
                                    chk, g->stream));
        src = chk;
    }
    KS_HIP(hipMemcpyAsync(g->h_norms, src, sizeof(double) * S,
                          hipMemcpyDeviceToHost, g->stream));
    KS_HIP(hipStreamSynchronize(g->stream));
    return ks_check_finite(g->h_norms, S);
}

// One Taylor-4 exponential of H (potential v, vector potential A) for all
// states.  With two halves (and projectors, whose small kernels are what
// the overlap hides) the second half runs on the side stream, forked from
// and joined back into the grid's stream; kernel profiling runs whole.
int taylor_exponential(ks_grid *g, const double2 *in, double2 *out,
                       const double *v, const double A[3], double a2half,
                       double tau, int final_mode, double *npart,
                       double *normpart)
{
    const int S = g->stot;
    // the FP32 kernels read an FP32 copy of the potential
    if (g->mixed)
        KS_HIP(launch_to_f32(v, wsp<float>(g, g->lay.v32), g->geo.N,
                             g->stream));
    if (g->halves < 2 || S < 2 || g->natoms == 0 || g->profiling)
        return exp_chain(g, g->stream, 0, S, in, out, v, A, a2half, tau,
                         final_mode, npart, normpart);
    const int sa = S / 2;
    KS_HIP(hipEventRecord(g->fork_ev, g->stream));
    KS_HIP(hipStreamWaitEvent(g->side, g->fork_ev, 0));
    int rc = exp_chain(g, g->stream, 0, sa, in, out, v, A, a2half, tau,
                       final_mode, npart, normpart);
    if (rc)
        return rc;
    rc = exp_chain(g, g->side, sa, S - sa, in, out, v, A, a2half, tau,
                   final_mode, npart, normpart);
    if (rc)
        return rc;
    KS_HIP(hipEventRecord(g->join_ev, g->side));
    KS_HIP(hipStreamWaitEvent(g->stream, g->join_ev, 0));
    return KS_OK;
}

// Argument checks of ks_apply_h and its allocation-free variant.
int apply_h_check(const ks_grid *g, const void *d_psi, const void *d_hpsi,
                  int k, int s0, int ns)
{
    if (!g || !d_psi || !d_hpsi)
        return fail(KS_E_ARG, "NULL argument");
    if (k < 0 || k >= g->nk || s0 < 0 || ns < 0 || s0 + ns > g->ns)
        return fail(KS_E_ARG, "k=%d s0=%d ns=%d out of range", k, s0, ns);
    if (d_psi == d_hpsi)
        return fail(KS_E_ARG, "d_psi and d_hpsi must not overlap");
    if (!g->vloc_set)
        return fail(KS_E_STATE, "no local potential (ks_update_vlocal)");
    return KS_OK;
}

// d_hpsi = H(t) d_psi for ns states of k-point k, with the projector
// coefficients D, their chunk partials and the hull-row terms W at the
// given device addresses (each indexed from the call's first state).
int apply_h_core(ks_grid *g, const void *d_psi, void *d_hpsi, int k, int s0,
                 int ns, double t, void *D, void *Dpart, void *W, float *v32)
{
    if (g->mixed)
        KS_HIP(launch_to_f32(g->d_v, v32, g->geo.N, g->stream));
    double A[3];
    laser_A(g, t, A);
    GArgs ga = base_gargs(g);
    ga.in = d_psi;
    ga.D = D;
    ga.Dpart = Dpart;
    ga.W = W;
    ga.sg0 = k * g->ns + s0;
    if (g->natoms > 0) {
        Timed tm(g, 1);
        KS_HIP(launch_gather(g->mixed, true, ga, ns, g->stream));
        KS_HIP(launch_kbapply(g->mixed, ga, ns, g->stream));
    }
    HArgs a = base_hargs(g);
    a.in = d_psi;
    a.out = d_hpsi;
    a.v = g->d_v;
    a.v32 = v32;
    if (a.rowinfo)
        a.W = W;
    a.A[0] = A[0];
    a.A[1] = A[1];
    a.A[2] = A[2];
    a.a2half = 0.5 * (A[0] * A[0] + A[1] * A[1] + A[2] * A[2]);

    a.sg0 = k * g->ns + s0;
    {
        Timed tm(g, 0);
        KS_HIP(launch_hpsi(kApply, g->mixed, true, a, ns, g->stream));
    }
    return KS_OK;
}

}  // namespace

// ks_apply_h on the projector scratch at `base` (cap bytes of device
// memory) instead of the workspace: the allocation-free entry point.  The
// scratch holds, for the call's ns states, the coefficients, their chunk
// partials and the hull-row terms, each 256-byte aligned; every one of
// them is written by the call before it is read.
int ks::apply_h_scratch(ks_grid *g, const void *d_psi, void *d_hpsi, int k,
                        int s0, int ns, double t, char *base, size_t cap,
                        int device)
{
    int rc = apply_h_check(g, d_psi, d_hpsi, k, s0, ns);
    if (rc)
        return rc;
    if (device != g->device)
        return fail(KS_E_ARG, "the grid lives on device %d, the current "
                    "device is %d", g->device, device);
    const size_t vs = g->mixed ? 8 : 16;
    const size_t na = std::max(1, g->natoms);
    const size_t nD = align256((size_t)ns * na * kMaxProj * vs);
    const size_t nP = align256((size_t)ns * na * g->nchunk * kMaxProj * vs);
    const size_t nW = align256((size_t)ns * std::max<long>(1, g->nhull) * vs);
    const size_t nV = g->mixed ? align256((size_t)g->geo.N * 4) : 0;
    const size_t need = (g->natoms > 0 ? nD + nP + nW : 0) + nV;
    if (need > cap)
        return fail(KS_E_ARG, "%d states need %zu bytes of projector scratch "
                    "and the static scratch holds %zu: apply H to fewer "
                    "states per call", ns, need, cap);
    char *pv = base + (g->natoms > 0 ? nD + nP + nW : 0);
    return apply_h_core(g, d_psi, d_hpsi, k, s0, ns, t, base, base + nD,
                        base + nD + nP, reinterpret_cast<float *>(pv));
}

int ks::set_error(int code, const char *msg)
{
    return fail(code, "%s", msg);
}

// ---------------------------------------------------------------------------
// C ABI
// ---------------------------------------------------------------------------
extern "C" {

const char *ks_last_error(void) { return g_err.c_str(); }

int ks_check_finite(const double *values, long n)
{
    if (!values || n < 0)
        return fail(KS_E_ARG, "values is NULL or n < 0");
    for (long i = 0; i < n; ++i)
        if (!std::isfinite(values[i]))
            return fail(KS_E_NONFINITE, "value %ld is %s", i,
                        std::isnan(values[i]) ? "NaN" : "infinite");
    return KS_OK;
}

int ks_grid_create(const ks_grid_desc *d, ks_grid **out)
{
    if (!out)
        return fail(KS_E_ARG, "out is NULL");
    *out = nullptr;
    if (!d)
        return fail(KS_E_ARG, "desc is NULL");
    for (int a = 0; a < 3; ++a) {
        if (d->n[a] < 1)
            return fail(KS_E_ARG, "n[%d] = %d must be >= 1", a, d->n[a]);
        if (!(d->h[a] > 0.0))
            return fail(KS_E_ARG, "h[%d] must be > 0", a);
    }
    // a tile row of x points is one thread each, at most 512 threads
    if (d->n[0] > kRowThreads)
        return fail(KS_E_UNSUPPORTED, "nx = %d > %d", d->n[0], kRowThreads);
    if (d->fd_half_width != 4)
        return fail(KS_E_UNSUPPORTED, "fd_half_width %d (only 4)",
                    d->fd_half_width);
    const long N = (long)d->n[0] * d->n[1] * d->n[2];
    // one state's bytes are addressed by 32-bit buffer offsets
    if (N >= (1L << 27))
        return fail(KS_E_UNSUPPORTED, "grid of %ld points: at most 2^27 - 1 "
                    "points", N);
    if (d->nk < 1 || d->nstates < 1 || d->natoms < 0)
        return fail(KS_E_ARG, "nk, nstates must be >= 1, natoms >= 0");
    if ((long)d->nk * d->nstates > 65535)
        return fail(KS_E_UNSUPPORTED, "nk*nstates > 65535");
    if (d->natoms > 0 && (!d->pos || !d->lmax || !d->rc || !d->sigma || !d->E))
        return fail(KS_E_ARG, "atom arrays missing");
    // sphere and hull points carry their (x, y, z) packed in 10 + 10 + 11
    // bits of one int
    if (d->natoms > 0 && (d->n[1] > 1024 || d->n[2] > 2048))
        return fail(KS_E_UNSUPPORTED, "projectors need ny <= 1024 and "
                    "nz <= 2048 (ny = %d, nz = %d)", d->n[1], d->n[2]);
    if (d->xc != 0 && d->xc != 1)
        return fail(KS_E_ARG, "xc must be 0 or 1");
    if (d->hartree != 0 && d->hartree != 1)
        return fail(KS_E_ARG, "hartree must be 0 or 1");
    const int nper = (d->periodic[0] ? 1 : 0) + (d->periodic[1] ? 1 : 0) +
                     (d->periodic[2] ? 1 : 0);
    if (d->hartree && nper != 0 && nper != 3)
        return fail(KS_E_UNSUPPORTED,
                    "Hartree term needs all axes finite or all periodic");
    if (d->precision != KS_FP64 && d->precision != KS_MIXED)
        return fail(KS_E_ARG, "precision must be KS_FP64 or KS_MIXED");
    if (d->laser[0] != 0.0 && !(d->laser[2] > 0.0))
        return fail(KS_E_ARG, "laser duration must be > 0");

    ks_grid *g = new ks_grid;
    g->geo.nx = d->n[0];
    g->geo.ny = d->n[1];
    g->geo.nz = d->n[2];
    g->geo.N = N;
    for (int a = 0; a < 3; ++a) {
        g->geo.per[a] = d->periodic[a] ? 1 : 0;
        g->geo.h[a] = d->h[a];
    }
    g->nk = d->nk;
    g->ns = d->nstates;
    g->stot = d->nk * d->nstates;
    g->xc = d->xc;
    g->hartree = d->hartree;
    g->nonlin = d->xc || d->hartree;
    std::memcpy(g->laser, d->laser, sizeof g->laser);
    g->mixed = d->precision == KS_MIXED;
    g->stream = static_cast<hipStream_t>(d->stream);
    if (hipStreamCreateWithFlags(&g->side, hipStreamNonBlocking) !=
            hipSuccess ||
        hipEventCreateWithFlags(&g->fork_ev, hipEventDisableTiming) !=
            hipSuccess ||
        hipEventCreateWithFlags(&g->join_ev, hipEventDisableTiming) !=
            hipSuccess) {
        ks_grid_destroy(g);
        return fail(KS_E_HIP, "stream or event creation failed");
    }
    g->kpts.assign(3 * d->nk, 0.0);
    if (d->kpts)
        g->kpts.assign(d->kpts, d->kpts + 3 * d->nk);
    g->kw.assign(d->nk, 1.0 / d->nk);
    if (d->kw)
        g->kw.assign(d->kw, d->kw + d->nk);
    g->occ.assign(d->nstates, 2.0);
    if (d->occ)
        g->occ.assign(d->occ, d->occ + d->nstates);
    g->wocc.resize(g->stot);
    for (int k = 0; k < d->nk; ++k)
        for (int s = 0; s < d->nstates; ++s)
            g->wocc[k * d->nstates + s] = g->kw[k] * g->occ[s];
    g->kph.resize(3 * d->nk);
    for (int k = 0; k < d->nk; ++k)
        for (int a = 0; a < 3; ++a) {
            const double ang = g->kpts[3 * k + a] * d->n[a] * d->h[a];
            g->kph[3 * k + a] = make_double2(std::cos(ang), std::sin(ang));
        }
    (void)hipGetDevice(&g->device);
    if (hipHostMalloc(reinterpret_cast<void **>(&g->h_norms),
                      sizeof(double) * g->stot, hipHostMallocDefault) !=
        hipSuccess) {
        g->h_norms = nullptr;
        ks_grid_destroy(g);
        return fail(KS_E_OOM, "pinned host buffer of %d norms", g->stot);
    }
    int rc;
    if ((rc = dev_upload(g, &g->d_kph, g->kph)) ||
        (rc = dev_upload(g, &g->d_wocc, g->wocc)) ||
        (rc = dev_alloc(g, &g->d_v, (size_t)N)) ||
        (rc = build_projectors(g, d))) {
        ks_grid_destroy(g);
        return rc;
    }
    if ((rc = set_tiles(g, 0, 0, 0))) {
        ks_grid_destroy(g);
        return rc;
    }
    if (g->hartree) {
        int M[3];
        if (!poisson_lengths(g->geo, nper == 3, M)) {
            ks_grid_destroy(g);
            return fail(KS_E_UNSUPPORTED,
                        "Hartree transform lengths %d x %d x %d: each must "
                        "be a product of 2, 3 and 5 up to %d", M[0], M[1],
                        M[2], kFftMaxLen);
        }
        const hipError_t e =
            poisson_plan_create(g->geo, nper == 3, &g->pp, g->stream);
        if (e != hipSuccess) {
            ks_grid_destroy(g);
            return fail(e == hipErrorOutOfMemory ? KS_E_OOM : KS_E_HIP,
                        "Hartree plan: %s", hipGetErrorString(e));
        }
    }
    layout(g);
    *out = g;
    return KS_OK;
}

int ks_grid_destroy(ks_grid *g)
{
    if (!g)
        return KS_OK;
    (void)hipStreamSynchronize(g->stream);
    if (g->side) {
        (void)hipStreamSynchronize(g->side);
        (void)hipStreamDestroy(g->side);
    }
    if (g->fork_ev)
        (void)hipEventDestroy(g->fork_ev);
    if (g->join_ev)
        (void)hipEventDestroy(g->join_ev);
    for (hipEvent_t e : g->ev)
        (void)hipEventDestroy(e);
    for (void *p : g->owned)
        (void)hipFree(p);
    if (g->h_norms)
        (void)hipHostFree(g->h_norms);
    poisson_plan_destroy(&g->pp);
    delete g;
    return KS_OK;
}

int ks_grid_device_bytes(const ks_grid *g, size_t *out)
{
    if (!g || !out)
        return fail(KS_E_ARG, "grid or output is NULL");
    size_t b = g->owned_bytes;
    // the Hartree plan: twiddles per axis and the kernel's octant
    if (g->pp.K) {
        for (int d = 0; d < 3; ++d)
            b += sizeof(double2) * g->pp.ax[d].M;
        b += sizeof(double) * (size_t)(g->pp.ax[0].M / 2 + 1) *
             (g->pp.ax[1].M / 2 + 1) * (g->pp.ax[2].M / 2 + 1);
    }
    *out = b;
    return KS_OK;
}

int ks_set_overlap(ks_grid *g, int halves)
{
    if (!g || halves < 1 || halves > 2)
        return fail(KS_E_ARG, "grid is NULL or halves not 1 or 2");
    g->halves = halves;
    return KS_OK;
}

int ks_set_stream(ks_grid *g, void *stream)
{
    if (!g)
        return fail(KS_E_ARG, "grid is NULL");
    g->stream = static_cast<hipStream_t>(stream);
    return KS_OK;
}

size_t ks_workspace_bytes(const ks_grid *g) { return g ? g->lay.total : 0; }

int ks_set_workspace(ks_grid *g, void *d_ws, size_t bytes)
{
    if (!g)
        return fail(KS_E_ARG, "grid is NULL");
    if (!d_ws)
        return fail(KS_E_ARG, "workspace pointer is NULL");
    if (reinterpret_cast<uintptr_t>(d_ws) % 256)
        return fail(KS_E_ARG, "workspace must be 256-byte aligned");
    if (bytes < g->lay.total)
        return fail(KS_E_OOM, "workspace of %zu bytes < %zu needed", bytes,
                    g->lay.total);
    g->ws = static_cast<char *>(d_ws);
    g->ws_bytes = bytes;
    return KS_OK;
}

int ks_update_vlocal(ks_grid *g, const double *d_vion, const double *d_rho)
{
    if (!g || !d_vion)
        return fail(KS_E_ARG, "grid or v_ion is NULL");
    // v = v_ion + v_x(rho): the density kernel with rho itself as the one
    // source partial (no source at all when rho is not given)
    DArgs a;
    a.geo = g->geo;
    a.vion = d_vion;
    a.vout = g->d_v;
    a.xc = (d_rho && g->xc) ? 1 : 0;
    a.nsrc = d_rho ? 1 : 0;
    a.npart = d_rho ? d_rho : d_vion;  // not read when nsrc == 0
    if (d_rho && g->hartree) {
        const int rc = need_ws(g);
        if (rc)
            return rc;
    }
    KS_HIP(launch_density(a, g->stream));
    if (d_rho && g->hartree)
        KS_HIP(launch_hartree(g->pp, g->geo, d_rho, g->d_v, true,
                              wsp<double2>(g, g->lay.pwork), g->stream));
    g->vloc_set = true;
    return KS_OK;
}

int ks_apply_h(ks_grid *g, const void *d_psi, void *d_hpsi, int k, int s0,
               int ns, double t)
{
    int rc = apply_h_check(g, d_psi, d_hpsi, k, s0, ns);
    if (rc)
        return rc;
    if ((rc = need_ws(g)))
        return rc;
    return apply_h_core(g, d_psi, d_hpsi, k, s0, ns, t, g->ws + g->lay.D,
                        g->ws + g->lay.Dpart, g->ws + g->lay.W,
                        wsp<float>(g, g->lay.v32));
}

int ks_hartree(ks_grid *g, const double *d_rho, double *d_vh)
{
    if (!g || !d_rho || !d_vh)
        return fail(KS_E_ARG, "NULL argument");
    if (!g->hartree)
        return fail(KS_E_STATE, "grid created without the Hartree term");
    if (d_rho == d_vh)
        return fail(KS_E_ARG, "d_rho and d_vh must not overlap");
    int rc = need_ws(g);
    if (rc)
        return rc;
    Timed tm(g, 2);
    KS_HIP(launch_hartree(g->pp, g->geo, d_rho, d_vh, false,
                          wsp<double2>(g, g->lay.pwork), g->stream));
    return KS_OK;
}

int ks_current(ks_grid *g, const void *d_psi, double t, double out_host[3])
{
    if (!g || !d_psi || !out_host)
        return fail(KS_E_ARG, "NULL argument");
    if (!std::isfinite(t))
        return fail(KS_E_ARG, "t must be finite");
    int rc = need_ws(g);
    if (rc)
        return rc;
    // stencil part: the H.psi kernel's tiles (one row per thread, the
    // tallest tile within 512 threads and the default LDS share), each
    // writing its three partial sums
    const Geo &G = g->geo;
    int TY = std::max(1, std::min(G.ny, kRowThreads / G.nx));
    while (TY > 1 && (!tile_ok(g, TY, 1) ||
                      hpsi_lds_bytes(G.nx, TY, g->zchunk, false) >
                          kLdsDefault))
        --TY;
    if (!tile_ok(g, TY, 1) ||
        hpsi_lds_bytes(G.nx, TY, g->zchunk, false) > kLdsBudget)
        return fail(KS_E_UNSUPPORTED, "no tile shape for the current");
    HArgs h = base_hargs(g);
    h.rowinfo = nullptr;
    h.W = nullptr;
    h.in = d_psi;
    h.TY = TY;
    h.rpt = 1;
    h.ntile_y = (G.ny + TY - 1) / TY;
    h.nzc = (G.nz + g->zchunk - 1) / g->zchunk;
    h.sg0 = 0;
    double A[3];
    laser_A(g, t, A);
    for (int d = 0; d < 3; ++d)
        h.A[d] = A[d];
    h.normpart = wsp<double>(g, g->lay.cpart);
    // projector part
    CurArgs a;
    a.geo = g->geo;
    a.psi = static_cast<const double2 *>(d_psi);
    a.kph = g->d_kph;
    a.nstates = g->ns;
    a.sg0 = 0;
    for (int d = 0; d < 3; ++d)
        a.A[d] = A[d];
    a.pj = g->pj;
    a.nl = wsp<double>(g, g->lay.cnl);
    {
        Timed tm(g, 2);
        KS_HIP(launch_hpsi_current(h, g->stot, g->stream));
        KS_HIP(launch_current_nl(a, g->stot, g->stream));
    }
    const int nch = h.ntile_y * h.nzc;
    const int na = g->natoms;
    std::vector<double> hp((size_t)g->stot * nch * 3);
    std::vector<double> hn((size_t)g->stot * std::max(1, na) * 3, 0.0);
    KS_HIP(hipMemcpyAsync(hp.data(), h.normpart, hp.size() * sizeof(double),
                          hipMemcpyDeviceToHost, g->stream));
    if (na > 0)
        KS_HIP(hipMemcpyAsync(hn.data(), a.nl,
                              (size_t)g->stot * na * 3 * sizeof(double),
                              hipMemcpyDeviceToHost, g->stream));
    KS_HIP(hipStreamSynchronize(g->stream));
    const double h3 = g->geo.h[0] * g->geo.h[1] * g->geo.h[2];
    const double vol = g->geo.nx * g->geo.h[0] * g->geo.ny * g->geo.h[1] *
                       g->geo.nz * g->geo.h[2];
    for (int ax = 0; ax < 3; ++ax) {
        double J = 0.0;
        for (int s = 0; s < g->stot; ++s) {
            double loc = 0.0, nl = 0.0;
            for (int c = 0; c < nch; ++c)
                loc += hp[((size_t)s * nch + c) * 3 + ax];
            for (int at = 0; at < na; ++at)
                nl += hn[((size_t)s * na + at) * 3 + ax];
            J += g->wocc[s] * (h3 * loc + nl);
        }
        out_host[ax] = J / vol;
    }
    if (!std::isfinite(out_host[0]) || !std::isfinite(out_host[1]) ||
        !std::isfinite(out_host[2]))
        return fail(KS_E_NONFINITE, "current is not finite");
    return KS_OK;
}

int ks_strength_function(const double *d_trace, int nt, int stride,
                         double dt, double kappa, double gamma,
                         const double *d_omega, int nw, double *d_out,
                         void *stream)
{
    if (!d_trace || (nw > 0 && (!d_omega || !d_out)))
        return fail(KS_E_ARG, "NULL argument");
    if (nt < 2 || stride < 1 || nw < 0 || !(dt > 0.0) || kappa == 0.0 ||
        !std::isfinite(kappa) || !(gamma >= 0.0))
        return fail(KS_E_ARG, "need nt >= 2, stride >= 1, nw >= 0, dt > 0, "
                              "kappa != 0, gamma >= 0");
    KS_HIP(launch_damped_ft(d_trace, nt, stride, dt, kappa, gamma, d_omega,
                            nw, 0, d_out, static_cast<hipStream_t>(stream)));
    return KS_OK;
}

int ks_conductivity(const double *d_trace, int nt, int stride, double dt,
                    double E0, double gamma, const double *d_omega, int nw,
                    void *d_out, void *stream)
{
    if (!d_trace || (nw > 0 && (!d_omega || !d_out)))
        return fail(KS_E_ARG, "NULL argument");
    if (nt < 2 || stride < 1 || nw < 0 || !(dt > 0.0) || E0 == 0.0 ||
        !std::isfinite(E0) || !(gamma >= 0.0))
        return fail(KS_E_ARG, "need nt >= 2, stride >= 1, nw >= 0, dt > 0, "
                              "E0 != 0, gamma >= 0");
    KS_HIP(launch_damped_ft(d_trace, nt, stride, dt, E0, gamma, d_omega, nw,
                            1, static_cast<double *>(d_out),
                            static_cast<hipStream_t>(stream)));
    return KS_OK;
}

int ks_density(ks_grid *g, const void *d_psi, double *d_rho)
{
    if (!g || !d_psi || !d_rho)
        return fail(KS_E_ARG, "NULL argument");
    DArgs a;
    a.geo = g->geo;
    a.nsrc = g->stot;
    a.psi = static_cast<const double2 *>(d_psi);
    a.wocc = g->d_wocc;
    a.rho = d_rho;
    KS_TRY(density_potential(g, a, g->stream));
    return KS_OK;
}

int ks_dipole(ks_grid *g, const double *d_rho, double out_host[3])
{
    if (!g || !d_rho || !out_host)
        return fail(KS_E_ARG, "NULL argument");
    if (g->geo.per[0] || g->geo.per[1] || g->geo.per[2])
        return fail(KS_E_UNSUPPORTED, "dipole of a periodic grid");
    int rc = need_ws(g);
    if (rc)
        return rc;
    // rho -> rho (copy into the workspace) with dipole partials
    DArgs a;
    a.geo = g->geo;
    a.nsrc = 1;
    a.npart = d_rho;
    a.dpart = wsp<double>(g, g->lay.dpart);
    KS_TRY(density_potential(g, a, g->stream));
    double *dout = wsp<double>(g, g->lay.xpart);
    const double h3 = g->geo.h[0] * g->geo.h[1] * g->geo.h[2];
    KS_HIP(launch_dipole_finalize(a.dpart, density_blocks(g->geo.N), h3, dout,
                                  g->stream));
    KS_HIP(hipMemcpyAsync(out_host, dout, 3 * sizeof(double),
                          hipMemcpyDeviceToHost, g->stream));
    KS_HIP(hipStreamSynchronize(g->stream));
    for (int c = 0; c < 3; ++c)
        if (!std::isfinite(out_host[c]))
            return fail(KS_E_NONFINITE, "dipole is not finite");
    return KS_OK;
}

int ks_kick(ks_grid *g, void *d_psi, double kappa)
{
    if (!g || !d_psi)
        return fail(KS_E_ARG, "NULL argument");
    KS_HIP(launch_kick(g->geo, static_cast<double2 *>(d_psi), g->stot, kappa,
                       g->stream));
    return KS_OK;
}

int ks_norms(ks_grid *g, const void *d_psi, double *d_norms)
{
    if (!g || !d_psi || !d_norms)
        return fail(KS_E_ARG, "NULL argument");
    int rc = need_ws(g);
    if (rc)
        return rc;
    double *part = wsp<double>(g, g->lay.normpart);
    const double h3 = g->geo.h[0] * g->geo.h[1] * g->geo.h[2];
    KS_HIP(launch_norm_partial(g->geo, static_cast<const double2 *>(d_psi),
                               g->stot, g->norm_chunks, part, g->stream));
    KS_HIP(launch_norm_finalize(part, g->stot, g->norm_chunks, h3, d_norms,
                                g->stream));
    return KS_OK;
}

int ks_gram(ks_grid *g, const void *d_psi, void *d_gram)
{
    if (!g || !d_psi || !d_gram)
        return fail(KS_E_ARG, "NULL argument");
    int rc = need_ws(g);
    if (rc)
        return rc;
    KS_HIP(launch_gram(g->geo, static_cast<const double2 *>(d_psi), g->nk,
                       g->ns, wsp<double2>(g, g->lay.gpart), g->gram_ksplit,
                       static_cast<double2 *>(d_gram), g->stream));
    return KS_OK;
}

int ks_energy(ks_grid *g, const void *d_psi, const double *d_vion, double t,
              double *out_host)
{
    if (!g || !d_psi || !d_vion || !out_host)
        return fail(KS_E_ARG, "NULL argument");
    int rc = need_ws(g);
    if (rc)
        return rc;
    if (g->mixed)
        return fail(KS_E_UNSUPPORTED, "ks_energy runs on an FP64 grid");
    // H[v_ion] psi for every k into the half-step buffer
    double A[3];
    laser_A(g, t, A);
    double2 *hp = wsp<double2>(g, g->lay.half);
    const double2 *psi = static_cast<const double2 *>(d_psi);
    void *D = g->ws + g->lay.D;
    const long N = g->geo.N;
    for (int k = 0; k < g->nk; ++k) {
        GArgs ga = base_gargs(g);
        ga.in = psi + (size_t)k * g->ns * N;
        ga.D = D;
        ga.sg0 = k * g->ns;
        KS_HIP(launch_gather(false, true, ga, g->ns, g->stream));
        KS_HIP(launch_kbapply(false, ga, g->ns, g->stream));
        HArgs a = base_hargs(g);
        a.in = ga.in;
        a.out = hp + (size_t)k * g->ns * N;
        a.v = d_vion;
        a.A[0] = A[0];
        a.A[1] = A[1];
        a.A[2] = A[2];
        a.a2half = 0.5 * (A[0] * A[0] + A[1] * A[1] + A[2] * A[2]);

        a.sg0 = k * g->ns;
        KS_HIP(launch_hpsi(kApply, false, true, a, g->ns, g->stream));
    }
    double2 *dp = wsp<double2>(g, g->lay.dotpart);
    KS_HIP(launch_dot_partial(g->geo, psi, hp, g->stot, g->norm_chunks, dp,
                              g->stream));
    std::vector<double2> hdp((size_t)g->stot * g->norm_chunks);
    KS_HIP(hipMemcpyAsync(hdp.data(), dp, hdp.size() * sizeof(double2),
                          hipMemcpyDeviceToHost, g->stream));
    double ex = 0.0, eh = 0.0;
    const int nb = density_blocks(N);
    std::vector<double> hx, hh;
    if (g->nonlin) {
        DArgs a;
        a.geo = g->geo;
        a.nsrc = g->stot;
        a.psi = psi;
        a.wocc = g->d_wocc;
        a.rho = wsp<double>(g, g->lay.rho);
        KS_HIP(launch_density(a, g->stream));
        double *part = wsp<double>(g, g->lay.xpart);
        if (g->xc) {
            KS_HIP(launch_exchange_partial(g->geo, a.rho, part, g->stream));
            hx.resize(nb);
            KS_HIP(hipMemcpyAsync(hx.data(), part, nb * sizeof(double),
                                  hipMemcpyDeviceToHost, g->stream));
        }
        if (g->hartree) {
            // E_H = 1/2 h^3 sum n v_H; the partials buffer is reused after
            // the (stream-ordered) copy of the exchange partials
            double *vh = wsp<double>(g, g->lay.vh);
            KS_HIP(launch_hartree(g->pp, g->geo, a.rho, vh, false,
                                  wsp<double2>(g, g->lay.pwork), g->stream));
            KS_HIP(launch_real_dot_partial(a.rho, vh, N, part, g->stream));
            hh.resize(nb);
            KS_HIP(hipMemcpyAsync(hh.data(), part, nb * sizeof(double),
                                  hipMemcpyDeviceToHost, g->stream));
        }
    }
    KS_HIP(hipStreamSynchronize(g->stream));
    const double h3 = g->geo.h[0] * g->geo.h[1] * g->geo.h[2];
    double e = 0.0;
    for (int s = 0; s < g->stot; ++s) {
        double acc = 0.0;
        for (int c = 0; c < g->norm_chunks; ++c)
            acc += hdp[(size_t)s * g->norm_chunks + c].x;
        e += g->wocc[s] * acc * h3;
    }
    if (g->xc) {
        double sx = 0.0;
        for (int b = 0; b < nb; ++b)
            sx += hx[b];
        ex = -0.75 * std::cbrt(3.0 / M_PI) * h3 * sx;
    }
    if (g->hartree) {
        double sh = 0.0;
        for (int b = 0; b < nb; ++b)
            sh += hh[b];
        eh = 0.5 * h3 * sh;
    }
    *out_host = e + ex + eh;
    if (!std::isfinite(*out_host))
        return fail(KS_E_NONFINITE, "energy is not finite");
    return KS_OK;
}

int ks_set_launch(ks_grid *g, int tile_rows, int zchunk, int rows_per_thread)
{
    if (!g)
        return fail(KS_E_ARG, "grid is NULL");
    const int oldTY = g->TY, oldz = g->zchunk, oldr = g->rpt;
    int rc = set_tiles(g, tile_rows, zchunk, rows_per_thread);
    if (rc) {
        set_tiles(g, oldTY, oldz, oldr);
        return rc;
    }
    layout(g);
    if (g->ws && g->lay.total > g->ws_bytes) {
        g->ws = nullptr;   // the caller must lend a larger workspace
        return fail(KS_E_OOM, "workspace too small for this launch shape");
    }
    return KS_OK;
}

int ks_autotune(ks_grid *g, const void *d_psi, int reps, int out_shape[3],
                double *out_us)
{
    if (!g || !d_psi || reps < 1)
        return fail(KS_E_ARG, "NULL grid or psi, or reps < 1");
    int rc = need_ws(g);
    if (rc)
        return rc;
    const Geo &G = g->geo;
    const int S = g->stot;
    const bool mx = g->mixed;
    // candidate (tile rows, rows per thread): for one and two rows per
    // thread the tallest tile of 512 threads, the one that splits ny evenly
    // into as many tiles, 3/4, 1/2 and 1/4 of it, and the tallest tile (and
    // its half) whose thread rows fill whole wavefronts
    std::vector<std::pair<int, int>> shapes;
    for (int rpt = 1; rpt <= 2; ++rpt) {
        const int m = std::max(1, std::min(G.ny, rpt * kRowThreads / G.nx));
        const int nt = (G.ny + m - 1) / m;
        int full = 0;
        for (int ty = m; ty >= rpt && !full; --ty)
            if ((G.nx * ((ty + rpt - 1) / rpt)) % 64 == 0)
                full = ty;
        for (int ty : {m, m - 1, (m * 3) / 4, m / 2, m / 4,
                       (G.ny + nt - 1) / nt, full, full / 2})
            if (ty >= rpt)
                shapes.push_back({ty, rpt});
    }
    // candidate z-chunks: the whole axis, halves down to 8 planes
    std::vector<int> zcs;
    for (int z = G.nz; z >= 8; z = (z + 1) / 2) {
        zcs.push_back(z);
        if (z == 1)
            break;
    }
    if (zcs.empty())
        zcs.push_back(G.nz);
    const int oldTY = g->TY, oldz = g->zchunk, oldr = g->rpt;
    // valid W for the timed passes: projector coefficients of psi
    GArgs ga = base_gargs(g);
    ga.D = g->ws + g->lay.D;
    ga.in = d_psi;
    if (g->natoms > 0) {
        KS_HIP(launch_gather(mx, true, ga, S, g->stream));
        KS_HIP(launch_kbapply(mx, ga, S, g->stream));
    }
    if (mx)
        KS_HIP(launch_to_f32(g->d_v, wsp<float>(g, g->lay.v32), G.N,
                             g->stream));
    hipEvent_t e0, e1;
    KS_HIP(hipEventCreate(&e0));
    KS_HIP(hipEventCreate(&e1));
    int bestTY = oldTY, bestz = oldz, bestr = oldr;
    double best = 1e300;
    std::vector<std::array<int, 3>> tried;
    auto run = [&](int ty, int zc, int rpt) -> int {
        for (auto &p : tried)
            if (p[0] == ty && p[1] == zc && p[2] == rpt)
                return KS_OK;
        tried.push_back({ty, zc, rpt});
        if (set_tiles(g, ty, zc, rpt) != KS_OK)
            return KS_OK;            // shape not allowed here: skip it
        g_err.clear();
        // one Taylor-4 exponential's four passes (three terms and the
        // final sum into psi_half), the mix of passes a step runs
        HArgs a = base_hargs(g);
        a.v = g->d_v;
        a.v32 = wsp<float>(g, g->lay.v32);
        a.cre = 0.0;
        // a grid with a laser runs the passes with the gradient term: time
        // that kernel, at the pulse's amplitude
        if (g->laser[0] != 0.0) {
            for (int d = 0; d < 3; ++d)
                a.A[d] = g->laser[0] * g->laser[3 + d];
            a.a2half = half_a2(a.A);
        }
        auto expo = [&]() -> int {
            void *tb[3] = {g->ws + g->lay.t1, g->ws + g->lay.t2,
                           g->ws + g->lay.t3};
            const void *cur = d_psi;
            for (int j = 1; j <= 4; ++j) {
                a.in = cur;
                a.cim = -0.01 / j;
                if (j < 4) {
                    a.out = tb[j - 1];
                    KS_HIP(launch_hpsi(kTerm, mx, j == 1 || !mx, a, S,
                                       g->stream));
                    cur = tb[j - 1];
                } else {
                    a.out = g->ws + g->lay.half;
                    a.base = static_cast<const double2 *>(d_psi);
                    a.t1 = tb[0];
                    a.t2 = tb[1];
                    KS_HIP(launch_hpsi(kFinal, mx, false, a, S, g->stream));
                }
            }
            return KS_OK;
        };
        int e = expo();                                          // warm
        if (e)
            return e;
        KS_HIP(hipEventRecord(e0, g->stream));
        for (int r = 0; r < reps; ++r)
            if ((e = expo()))
                return e;
        KS_HIP(hipEventRecord(e1, g->stream));
        KS_HIP(hipEventSynchronize(e1));
        float ms = 0.f;
        KS_HIP(hipEventElapsedTime(&ms, e0, e1));
        const double us = 1e3 * ms / (4.0 * reps);
        if (us < best) {
            best = us;
            bestTY = g->TY;
            bestz = g->zchunk;
            bestr = g->rpt;
        }
        return KS_OK;
    };
    // the default shape first, then every candidate
    rc = run(oldTY, oldz, oldr);
    for (auto &sh : shapes)
        for (int zc : zcs)
            if (!rc)
                rc = run(sh.first, zc, sh.second);
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (rc)
        set_tiles(g, oldTY, oldz, oldr);
    else
        set_tiles(g, bestTY, bestz, bestr);
    layout(g);
    if (rc)
        return rc;
    g_err.clear();
    if (out_shape) {
        out_shape[0] = g->TY;
        out_shape[1] = g->zchunk;
        out_shape[2] = g->rpt;
    }
    if (out_us)
        *out_us = best;
    return KS_OK;
}

int ks_get_launch(const ks_grid *g, int out[5])
{
    if (!g || !out)
        return fail(KS_E_ARG, "NULL argument");
    out[0] = g->TY;
    out[1] = g->zchunk;
    out[2] = g->ntile_y * g->nzc * g->stot;
    out[3] = hpsi_threads(g->geo.nx, g->TY, g->rpt);
    out[4] = g->rpt;
    return KS_OK;
}

int ks_profile_begin(ks_grid *g, int capacity, int class_mask)
{
    if (!g || capacity < 1 || (class_mask & ~0xf) || !class_mask)
        return fail(KS_E_ARG, "grid is NULL, capacity < 1 or bad mask");
    g->prof_mask = class_mask;
    while ((int)g->ev_class.size() < capacity) {
        hipEvent_t a, b;
        KS_HIP(hipEventCreate(&a));
        KS_HIP(hipEventCreate(&b));
        g->ev.push_back(a);
        g->ev.push_back(b);
        g->ev_class.push_back(0);
    }
    g->ev_used = 0;
    for (int c = 0; c < 4; ++c)
        g->prof_seen[c] = 0;
    g->profiling = true;
    return KS_OK;
}

int ks_profile_every(ks_grid *g, int every)
{
    if (!g || every < 1)
        return fail(KS_E_ARG, "grid is NULL or every < 1");
    g->prof_every = every;
    return KS_OK;
}

int ks_profile_end(ks_grid *g, double out_ms[4], long out_count[4])
{
    if (!g || !out_ms || !out_count)
        return fail(KS_E_ARG, "NULL argument");
    g->profiling = false;
    KS_HIP(hipStreamSynchronize(g->stream));
    for (int c = 0; c < 4; ++c) {
        out_ms[c] = 0.0;
        out_count[c] = 0;
    }
    for (int i = 0; i < g->ev_used; ++i) {
        float ms = 0.0f;
        KS_HIP(hipEventElapsedTime(&ms, g->ev[2 * i], g->ev[2 * i + 1]));
        out_ms[g->ev_class[i]] += ms;
        out_count[g->ev_class[i]] += 1;
    }
    g->ev_used = 0;
    return KS_OK;
}

int ks_propagate_etrs(ks_grid *g, void *d_psi, const double *d_vion,
                      int nsteps, double dt, double t0, double *d_dipole,
                      double *d_norms)
{
    if (!g || !d_psi || !d_vion)
        return fail(KS_E_ARG, "NULL argument");
    if (nsteps < 0)
        return fail(KS_E_ARG, "nsteps < 0");
    if (!std::isfinite(dt) || !std::isfinite(t0))
        return fail(KS_E_ARG, "dt and t0 must be finite");
    if (d_dipole && (g->geo.per[0] || g->geo.per[1] || g->geo.per[2]))
        return fail(KS_E_UNSUPPORTED, "dipole of a periodic grid");
    int rc = need_ws(g);
    if (rc)
        return rc;
    double2 *psi = static_cast<double2 *>(d_psi);
    double2 *half = wsp<double2>(g, g->lay.half);
    double *npart = wsp<double>(g, g->lay.npart);
    double *normpart = wsp<double>(g, g->lay.normpart);
    double *rho = wsp<double>(g, g->lay.rho);
    double *vpred = wsp<double>(g, g->lay.vpred);
    double *dpart = wsp<double>(g, g->lay.dpart);
    const double h3 = g->geo.h[0] * g->geo.h[1] * g->geo.h[2];
    const int S = g->stot;
    const int ntiles = g->ntile_y * g->nzc;
    const int ndb = density_blocks(g->geo.N);

    // v(t0) from n(psi(t0)); d(t0); norms(t0)
    {
        DArgs a;
        a.geo = g->geo;
        a.nsrc = S;
        a.psi = psi;
        a.wocc = g->d_wocc;
        a.rho = rho;
        a.vion = d_vion;
        a.vout = g->d_v;
        a.xc = g->xc;
        a.dpart = d_dipole ? dpart : nullptr;
        KS_TRY(density_potential(g, a, g->stream));
        if (d_dipole)
            KS_HIP(launch_dipole_finalize(dpart, ndb, h3, d_dipole,
                                          g->stream));
        if (d_norms) {
            KS_HIP(launch_norm_partial(g->geo, psi, S, g->norm_chunks,
                                       normpart, g->stream));
            KS_HIP(launch_norm_finalize(normpart, S, g->norm_chunks, h3,
                                        d_norms, g->stream));
        }
        g->vloc_set = true;
    }
    const bool want_n_end = g->nonlin || d_dipole;
    for (int step = 0; step < nsteps; ++step) {
        const double t = t0 + step * dt;
        double At[3], An[3];
        laser_A(g, t, At);
        laser_A(g, t + dt, An);
        // exponential 1: H_t, tau = dt/2; predictor density when the
        // potential depends on the density
        rc = taylor_exponential(g, psi, half, g->d_v, At, half_a2(At),
                                0.5 * dt,
                                g->nonlin ? kFinalPred : kFinal,
                                g->nonlin ? npart : nullptr, nullptr);
        if (rc)
            return rc;
        const double *vnext = d_vion;
        if (g->nonlin) {
            DArgs a;
            a.geo = g->geo;
            a.nsrc = S;
            a.npart = npart;
            a.rho = rho;
            a.vion = d_vion;
            a.vout = vpred;
            a.xc = g->xc;
            Timed tm(g, 2);
            KS_TRY(density_potential(g, a, g->stream));
            vnext = vpred;
        }
        // exponential 2: H_{t+dt}, tau = dt/2, from psi_half into psi
        // (norm partials when recorded, and always on the last step)
        const bool norm_now = d_norms || step == nsteps - 1;
        rc = taylor_exponential(g, half, psi, vnext, An, half_a2(An),
                                0.5 * dt, kFinal,
                                want_n_end ? npart : nullptr,
                                norm_now ? normpart : nullptr);
        if (rc)
            return rc;
        if (want_n_end) {
            DArgs a;
            a.geo = g->geo;
            a.nsrc = S;
            a.npart = npart;
            a.rho = rho;
            a.vion = d_vion;
            a.vout = g->d_v;
            a.xc = g->xc;
            a.dpart = d_dipole ? dpart : nullptr;
            Timed tm(g, 2);
            KS_TRY(density_potential(g, a, g->stream));
            if (d_dipole)
                KS_HIP(launch_dipole_finalize(dpart, ndb, h3,
                                              d_dipole + 3 * (step + 1),
                                              g->stream));
        }
        if (d_norms) {
            Timed tm(g, 2);
            KS_HIP(launch_norm_finalize(normpart, S, ntiles, h3,
                                        d_norms + (size_t)(step + 1) * S,
                                        g->stream));
        }
    }
    return check_end_norms(g, nsteps, d_norms, normpart);
}

int ks_propagate_cfm4(ks_grid *g, void *d_psi, const double *d_vion,
                      int nsteps, double dt, double t0, double *d_dipole,
                      double *d_norms)
{
    if (!g || !d_psi || !d_vion)
        return fail(KS_E_ARG, "NULL argument");
    if (nsteps < 0)
        return fail(KS_E_ARG, "nsteps < 0");
    if (!std::isfinite(dt) || !std::isfinite(t0))
        return fail(KS_E_ARG, "dt and t0 must be finite");
    if (d_dipole && (g->geo.per[0] || g->geo.per[1] || g->geo.per[2]))
        return fail(KS_E_UNSUPPORTED, "dipole of a periodic grid");
    int rc = need_ws(g);
    if (rc)
        return rc;
    double2 *psi = static_cast<double2 *>(d_psi);
    double2 *half = wsp<double2>(g, g->lay.half);
    double *npart = wsp<double>(g, g->lay.npart);
    double *normpart = wsp<double>(g, g->lay.normpart);
    double *rho = wsp<double>(g, g->lay.rho);
    double *dpart = wsp<double>(g, g->lay.dpart);
    double *veff = wsp<double>(g, g->lay.veff);
    double *vh[4];
    for (int j = 0; j < 4; ++j)
        vh[j] = wsp<double>(g, g->lay.vhist) + (size_t)j * g->geo.N;
    const double h3 = g->geo.h[0] * g->geo.h[1] * g->geo.h[2];
    const int S = g->stot;
    const int ntiles = g->ntile_y * g->nzc;
    const int ndb = density_blocks(g->geo.N);
    const double a1 = (3.0 - 2.0 * std::sqrt(3.0)) / 12.0;
    const double a2 = (3.0 + 2.0 * std::sqrt(3.0)) / 12.0;
    const double c1 = 0.5 - std::sqrt(3.0) / 6.0;
    const double c2 = 0.5 + std::sqrt(3.0) / 6.0;
    // history ring: hist[0] is v at the current time, hist[j] j steps back
    int ring[4] = {0, 1, 2, 3};
    int nhist = 0;
    // v(t0) from n(psi(t0)); d(t0); norms(t0)
    {
        DArgs a;
        a.geo = g->geo;
        a.nsrc = S;
        a.psi = psi;
        a.wocc = g->d_wocc;
        a.rho = rho;
        a.vion = d_vion;
        a.vout = vh[ring[0]];
        a.xc = g->xc;
        a.dpart = d_dipole ? dpart : nullptr;
        KS_TRY(density_potential(g, a, g->stream));
        if (d_dipole)
            KS_HIP(launch_dipole_finalize(dpart, ndb, h3, d_dipole,
                                          g->stream));
        if (d_norms) {
            KS_HIP(launch_norm_partial(g->geo, psi, S, g->norm_chunks,
                                       normpart, g->stream));
            KS_HIP(launch_norm_finalize(normpart, S, g->norm_chunks, h3,
                                        d_norms, g->stream));
        }
        nhist = 1;
    }
    const bool want_n_end = true;   // v(t + dt) feeds the extrapolation
    for (int step = 0; step < nsteps; ++step) {
        const double t = t0 + step * dt;
        double A1[3], A2[3], L1[4], L2[4];
        laser_A(g, t + c1 * dt, A1);
        laser_A(g, t + c2 * dt, A2);
        lagrange_back(nhist, c1, L1);
        lagrange_back(nhist, c2, L2);
        // exp(-i dt (a H1 + b H2)) = exp(-i dt/2 H_w) with H_w the
        // combination of weights 2a, 2b (summing to one): potential, vector
        // potential and |A|^2/2 combine linearly
        const double wts[2][2] = {{2.0 * a2, 2.0 * a1}, {2.0 * a1, 2.0 * a2}};
        for (int e = 0; e < 2; ++e) {
            const double w1 = wts[e][0], w2 = wts[e][1];
            double W[4] = {0, 0, 0, 0};
            const double *src[4] = {nullptr, nullptr, nullptr, nullptr};
            for (int j = 0; j < nhist; ++j) {
                W[j] = w1 * L1[j] + w2 * L2[j];
                src[j] = vh[ring[j]];
            }
            {
                Timed tm(g, 2);
                KS_HIP(launch_vcombine(g->geo.N, nhist, src, W, veff,
                                       g->stream));
            }
            double Aw[3];
            for (int d = 0; d < 3; ++d)
                Aw[d] = w1 * A1[d] + w2 * A2[d];
            const double a2w = w1 * half_a2(A1) + w2 * half_a2(A2);
            rc = e == 0 ? taylor_exponential(g, psi, half, veff, Aw, a2w,
                                             0.5 * dt, kFinal, nullptr,
                                             nullptr)
                        : taylor_exponential(g, half, psi, veff, Aw, a2w,
                                             0.5 * dt, kFinal,
                                             want_n_end ? npart : nullptr,
                                             (d_norms || step == nsteps - 1)
                                                 ? normpart
                                                 : nullptr);
            if (rc)
                return rc;
        }
        // v(t + dt) from the new density becomes the newest history entry
        const int slot = ring[3];
        for (int j = 3; j > 0; --j)
            ring[j] = ring[j - 1];
        ring[0] = slot;
        if (nhist < 4)
            ++nhist;
        {
            DArgs a;
            a.geo = g->geo;
            a.nsrc = S;
            a.npart = npart;
            a.rho = rho;
            a.vion = d_vion;
            a.vout = vh[ring[0]];
            a.xc = g->xc;
            a.dpart = d_dipole ? dpart : nullptr;
            Timed tm(g, 2);
            KS_TRY(density_potential(g, a, g->stream));
            if (d_dipole)
                KS_HIP(launch_dipole_finalize(dpart, ndb, h3,
                                              d_dipole + 3 * (step + 1),
                                              g->stream));
        }
        if (d_norms) {
            Timed tm(g, 2);
            KS_HIP(launch_norm_finalize(normpart, S, ntiles, h3,
                                        d_norms + (size_t)(step + 1) * S,
                                        g->stream));
        }
    }
    // the grid's potential is v at the final time
    KS_HIP(hipMemcpyAsync(g->d_v, vh[ring[0]], sizeof(double) * g->geo.N,
                          hipMemcpyDeviceToDevice, g->stream));
    g->vloc_set = true;
    return check_end_norms(g, nsteps, d_norms, normpart);
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Batched form: several grid objects (jobs) propagated together.  Every
// Taylor pass of all jobs is one H.psi launch (plus one batched projector
// gather, finalize and apply launch); the density, potential, dipole and
// norm reductions are one launch each for all jobs (the Hartree term, where
// a job has it, one solve per job); one ETRS step is captured as a HIP
// graph once and replayed.  Time-dependent inputs (A(t), output slots) come
// from per-job device step counters, so the replayed graph needs no change.
// ---------------------------------------------------------------------------
// Device and pinned host blocks of the batch tables, kept for reuse by
// later batches: a serving loop rebuilds its batch whenever a job joins or
// leaves, and would otherwise allocate and free some 2 njobs + 20 blocks
// (and a pinned buffer) each time.  Blocks come in power-of-two sizes from
// 256 bytes, per device; the pool holds what the most tables resident at
// once needed until the process ends.
namespace {

struct PoolBlock {
    void *p;
    size_t bytes;     // size class
    int dev;
    int pinned;       // 1: pinned host memory
};

std::mutex g_pool_mu;
std::map<std::tuple<int, int, size_t>, std::vector<void *>> g_pool;

int pool_get(size_t bytes, bool pinned, PoolBlock *out)
{
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess)
        return fail(KS_E_HIP, "hipGetDevice failed");
    size_t c = 256;
    while (c < bytes)
        c <<= 1;
    *out = PoolBlock{nullptr, c, dev, pinned ? 1 : 0};
    {
        std::lock_guard<std::mutex> lk(g_pool_mu);
        auto &v = g_pool[std::make_tuple(out->pinned, dev, c)];
        if (!v.empty()) {
            out->p = v.back();
            v.pop_back();
            return KS_OK;
        }
    }
    hipError_t e = pinned ? hipHostMalloc(&out->p, c, hipHostMallocDefault)
                          : hipMalloc(&out->p, c);
    if (e != hipSuccess) {
        out->p = nullptr;
        return fail(KS_E_OOM, "%s(%zu): %s",
                    pinned ? "hipHostMalloc" : "hipMalloc", c,
                    hipGetErrorString(e));
    }
    return KS_OK;
}

void pool_put(const PoolBlock &b)
{
    if (!b.p)
        return;
    std::lock_guard<std::mutex> lk(g_pool_mu);
    g_pool[std::make_tuple(b.pinned, b.dev, b.bytes)].push_back(b.p);
}

}  // namespace

struct ks_batch {
    std::vector<ks_grid *> grids;
    std::vector<ks_job> jobs;
    std::vector<JobDev> hjobs;
    hipStream_t stream = nullptr;
    bool mixed = false, grad = false;
    int hm = 2, rpt = 1, nthr = 64;
    size_t lds = 0;
    int grid_hpsi = 0, grid_proj = 0;
    std::vector<PoolBlock> owned;   // from the block pool
    JobDev *d_jobs = nullptr;
    HArgs *d_hargs = nullptr;
    int *d_off[4] = {nullptr, nullptr, nullptr, nullptr};
    int off_total[4] = {0, 0, 0, 0};
    int **d_steps = nullptr;
    // reductions of a step, one launch each for all jobs: the predictor
    // densities (jobs whose potential depends on the density), the
    // end-of-step densities, the dipoles and the norms
    DArgs *d_dpred = nullptr, *d_dend = nullptr;
    int *d_dpred_off = nullptr, *d_dend_off = nullptr;
    int npred = 0, nend = 0, blk_pred = 0, blk_end = 0;
    DipJob *d_dip = nullptr;
    NormJob *d_norm = nullptr;
    int ndip = 0, nnorm = 0, max_ns = 0;
    std::vector<int> steps_done;
    bool use_graph = true;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    // FP32 copies of each job's potential before each exponential (mixed
    // batches): copy tables and block offsets for exponentials 0 and 1
    F32Copy *d_conv[2] = {nullptr, nullptr};
    int *d_conv_off = nullptr;
    int conv_blocks = 0;
    // per-job sticky flags of a NaN / Inf norm (device), their copy after
    // the latest ks_batch_step (pinned host) and its completion event
    int *d_flags = nullptr;
    int *h_flags = nullptr;
    hipEvent_t flag_ev = nullptr;
    bool flag_pending = false;
};

namespace {

template <class T> int batch_alloc(ks_batch *b, T **p, size_t count,
                                    bool pinned = false)
{
    PoolBlock blk;
    const int rc = pool_get(std::max<size_t>(count * sizeof(T), 16), pinned,
                            &blk);
    if (rc)
        return rc;
    b->owned.push_back(blk);
    *p = static_cast<T *>(blk.p);
    return KS_OK;
}

BArgs batch_args(const ks_batch *b, int kind, int pass)
{
    BArgs a;
    a.jobs = b->d_jobs;
    a.njobs = (int)b->hjobs.size();
    a.off = b->d_off[kind];
    a.off_total = b->off_total[kind];
    a.pass = pass;
    a.hargs = b->d_hargs;
    return a;
}

// Report a non-finite norm of any job from the flags copied back after an
// earlier ks_batch_step: only once that copy has completed, unless `wait`.
int batch_poll_flags(ks_batch *b, bool wait)
{
    if (!b->flag_pending)
        return KS_OK;
    if (wait) {
        KS_HIP(hipEventSynchronize(b->flag_ev));
    } else {
        const hipError_t e = hipEventQuery(b->flag_ev);
        if (e == hipErrorNotReady) {
            (void)hipGetLastError();   // not an error: leave none behind
            return KS_OK;
        }
        KS_HIP(e);
    }
    b->flag_pending = false;
    for (size_t i = 0; i < b->jobs.size(); ++i)
        if (b->h_flags[i])
            return fail(KS_E_NONFINITE, "job %zu: a norm became NaN or Inf",
                        i);
    return KS_OK;
}

// Enqueue one ETRS step of every job on the batch stream.
int batch_enqueue_step(ks_batch *b)
{
    const hipStream_t st = b->stream;
    for (int e = 0; e < 2; ++e) {
        // the FP32 kernels read an FP32 copy of the exponential's potential
        if (b->mixed)
            KS_HIP(launch_to_f32_batch(b->d_conv[e], b->d_conv_off,
                                       (int)b->grids.size(), b->conv_blocks,
                                       st));
        for (int j = 1; j <= 4; ++j) {
            const int p = 4 * e + j;
            KS_HIP(launch_projectors_batch(b->mixed,
                                           batch_args(b, kItemGather, p),
                                           batch_args(b, kItemGatherFin, p),
                                           batch_args(b, kItemApply, p),
                                           b->grid_proj, st));
            KS_HIP(launch_pass_batch(b->mixed, batch_args(b, kItemHpsi, p),
                                     b->grad, b->hm, b->rpt, b->nthr, b->lds,
                                     b->grid_hpsi, st));
        }
        if (e == 0) {
            // v(t + dt) from the predicted density: the exchange term in
            // the batched launch, the Hartree term per job
            KS_HIP(launch_density_batch(b->d_dpred, b->d_dpred_off, b->npred,
                                        b->blk_pred, st));
            for (ks_grid *g : b->grids)
                if (g->nonlin && g->hartree)
                    KS_HIP(launch_hartree(g->pp, g->geo,
                                          wsp<double>(g, g->lay.rho),
                                          wsp<double>(g, g->lay.vpred), true,
                                          wsp<double2>(g, g->lay.pwork), st));
        }
    }
    KS_HIP(launch_density_batch(b->d_dend, b->d_dend_off, b->nend, b->blk_end,
                                st));
    for (size_t i = 0; i < b->grids.size(); ++i) {
        ks_grid *g = b->grids[i];
        if (b->hjobs[i].npart_end && g->hartree)
            KS_HIP(launch_hartree(g->pp, g->geo, wsp<double>(g, g->lay.rho),
                                  g->d_v, true, wsp<double2>(g, g->lay.pwork),
                                  st));
    }
    KS_HIP(launch_dipole_finalize_batch(b->d_dip, b->ndip, st));
    KS_HIP(launch_norm_finalize_batch(b->d_norm, b->nnorm, b->max_ns, st));
    KS_HIP(launch_step_advance(b->d_steps, (int)b->grids.size(), st));
    return KS_OK;
}

}  // namespace

extern "C" {

int ks_batch_create(const ks_job *jobs, int njobs, void *stream,
                    ks_batch **out)
{
    if (!out)
        return fail(KS_E_ARG, "out is NULL");
    *out = nullptr;
    if (!jobs || njobs < 1)
        return fail(KS_E_ARG, "need at least one job");
    const bool mixed = jobs[0].grid ? jobs[0].grid->mixed : false;
    for (int i = 0; i < njobs; ++i) {
        const ks_job &jb = jobs[i];
        ks_grid *g = jb.grid;
        if (!g || !jb.d_psi || !jb.d_vion)
            return fail(KS_E_ARG, "job %d: NULL grid, psi or v_ion", i);
        if (!g->ws)
            return fail(KS_E_STATE, "job %d: grid has no workspace", i);
        if (g->mixed != mixed)
            return fail(KS_E_ARG, "jobs of one batch share the precision");
        if (!std::isfinite(jb.dt) || !std::isfinite(jb.t0) ||
            jb.max_steps < 0 || jb.first_step < 0 ||
            jb.first_step > jb.max_steps)
            return fail(KS_E_ARG, "job %d: bad dt, t0, first_step or "
                        "max_steps", i);
        if (jb.first_step > 0 && !g->vloc_set)
            return fail(KS_E_STATE, "job %d resumes at step %d but its grid "
                        "holds no potential", i, jb.first_step);
        if (jb.d_dipole && (g->geo.per[0] || g->geo.per[1] || g->geo.per[2]))
            return fail(KS_E_UNSUPPORTED, "job %d: dipole of a periodic "
                        "grid", i);
        for (int k = 0; k < i; ++k)
            if (jobs[k].grid == g)
                return fail(KS_E_ARG, "a grid object appears twice");
    }
    ks_batch *b = new ks_batch;
    b->stream = static_cast<hipStream_t>(stream);
    b->mixed = mixed;
    b->jobs.assign(jobs, jobs + njobs);
    b->hm = 2;
    for (int i = 0; i < njobs; ++i) {
        ks_grid *g = jobs[i].grid;
        g->stream = b->stream;
        b->grids.push_back(g);
        JobDev J;
        J.h = base_hargs(g);
        J.g = base_gargs(g);
        J.g.D = g->ws + g->lay.D;
        J.g.ns = g->stot;
        J.g.sg0 = 0;
        J.stot = g->stot;
        J.psi = static_cast<double2 *>(jobs[i].d_psi);
        J.half = wsp<double2>(g, g->lay.half);
        J.t[0] = g->ws + g->lay.t1;
        J.t[1] = g->ws + g->lay.t2;
        J.t[2] = g->ws + g->lay.t3;
        J.npart = wsp<double>(g, g->lay.npart);
        J.npart_end = (g->nonlin || jobs[i].d_dipole) ? 1 : 0;
        J.normpart_end = jobs[i].d_norms ? wsp<double>(g, g->lay.normpart)
                                         : nullptr;
        J.vion = jobs[i].d_vion;
        J.vcur = g->d_v;
        J.vpred = wsp<double>(g, g->lay.vpred);
        J.nonlin = g->nonlin ? 1 : 0;
        J.dt = jobs[i].dt;
        J.step = wsp<int>(g, g->lay.step);
        b->hjobs.push_back(J);
        if (g->laser[0] != 0.0)
            b->grad = true;
        b->rpt = std::max(b->rpt, g->rpt);
        b->nthr = std::max(b->nthr, hpsi_threads(g->geo.nx, g->TY, g->rpt));
        b->lds = std::max(b->lds, lds_for(g, g->TY, g->zchunk));
    }
    // halo loads per thread for the workgroup size of the batch (the
    // largest any job asks for)
    for (ks_grid *g : b->grids)
        b->hm = std::max(b->hm, hpsi_halo_per_thread(g->geo, g->TY, b->nthr));
    if (b->rpt == 2 && b->hm > 8) {
        ks_batch_destroy(b);
        return fail(KS_E_UNSUPPORTED, "batch halo too large for two-row "
                    "tiles");
    }
    int rc;
    std::vector<int *> steps(njobs);
    for (int i = 0; i < njobs; ++i)
        steps[i] = const_cast<int *>(b->hjobs[i].step);
    if ((rc = batch_alloc(b, &b->d_jobs, njobs)) ||
        (rc = batch_alloc(b, &b->d_steps, njobs))) {
        ks_batch_destroy(b);
        return rc;
    }
    for (int i = 0; i < njobs; ++i) {
        // A(t) at both ends of every step, with the same arithmetic as the
        // single-job propagator (t = t0 + s dt and t + dt)
        const ks_job &jb = jobs[i];
        std::vector<double4> tab(2 * (size_t)std::max(jb.max_steps, 1));
        for (int s = 0; s < jb.max_steps; ++s) {
            const double t = jb.t0 + s * jb.dt;
            double A[3];
            for (int e = 0; e < 2; ++e) {
                laser_A(jb.grid, e ? t + jb.dt : t, A);
                tab[2 * s + e] = make_double4(
                    A[0], A[1], A[2],
                    0.5 * (A[0] * A[0] + A[1] * A[1] + A[2] * A[2]));
            }
        }
        double4 *d = nullptr;
        if ((rc = batch_alloc(b, &d, tab.size()))) {
            ks_batch_destroy(b);
            return rc;
        }
        if (hipMemcpy(d, tab.data(), tab.size() * sizeof(double4),
                      hipMemcpyHostToDevice) != hipSuccess) {
            ks_batch_destroy(b);
            return fail(KS_E_HIP, "upload of the A(t) table failed");
        }
        b->hjobs[i].Atab = d;
    }
    for (int kind = 0; kind < 4; ++kind) {
        std::vector<int> off(njobs + 1, 0);
        long sum = 0;
        for (int i = 0; i < njobs; ++i) {
            const long n = batch_items(kind, b->hjobs[i]);
            // H.psi: every job's launch range starts at a multiple of 8
            // (the kernel's per-job XCD remap)
            sum += kind == kItemHpsi ? (n + 7) / 8 * 8 : n;
            if (sum >= (1L << 31)) {
                ks_batch_destroy(b);
                return fail(KS_E_UNSUPPORTED, "batch of %ld work items",
                            sum);
            }
            off[i + 1] = (int)sum;
        }
        b->off_total[kind] = off[njobs];
        if ((rc = batch_alloc(b, &b->d_off[kind], njobs + 1))) {
            ks_batch_destroy(b);
            return rc;
        }
        if (hipMemcpy(b->d_off[kind], off.data(), off.size() * sizeof(int),
                      hipMemcpyHostToDevice) != hipSuccess) {
            ks_batch_destroy(b);
            return fail(KS_E_HIP, "upload of item offsets failed");
        }
    }
    // the H.psi arguments of every job's eight Taylor passes: exponential
    // e = (p-1)/4 starts from psi (e = 0) or psi_half (e = 1); term j writes
    // t_j, the fourth pass the sum (psi_half, then psi); the potential is
    // v(t) in the first exponential and v(t+dt) (predicted when the
    // potential depends on the density) in the second
    std::vector<HArgs> hargs(8 * (size_t)njobs);
    for (int i = 0; i < njobs; ++i) {
        const JobDev &J = b->hjobs[i];
        for (int p = 1; p <= 8; ++p) {
            const int e = (p - 1) / 4, j = (p - 1) % 4 + 1;
            HArgs a = J.h;
            a.A[0] = a.A[1] = a.A[2] = 0.0;
            a.a2half = 0.0;
            a.in = j == 1 ? (e == 0 ? (const void *)J.psi
                                    : (const void *)J.half)
                          : J.t[j - 2];
            a.v = e == 0 ? J.vcur : (J.nonlin ? J.vpred : J.vion);
            a.v32 = mixed ? wsp<float>(b->grids[i], b->grids[i]->lay.v32)
                          : nullptr;
            a.cre = 0.0;
            a.cim = -0.5 * J.dt / j;
            if (j < 4) {
                a.out = J.t[j - 1];
            } else {
                a.out = e == 0 ? (void *)J.half : (void *)J.psi;
                a.base = e == 0 ? J.psi : J.half;
                a.t1 = J.t[0];
                a.t2 = J.t[1];
                a.npart = e == 0 ? (J.nonlin ? J.npart : nullptr)
                                 : (J.npart_end ? J.npart : nullptr);
                a.normpart = e == 1 ? J.normpart_end : nullptr;
            }
            hargs[8 * (size_t)i + p - 1] = a;
        }
    }
    if ((rc = batch_alloc(b, &b->d_hargs, hargs.size()))) {
        ks_batch_destroy(b);
        return rc;
    }
    if (hipMemcpy(b->d_hargs, hargs.data(), hargs.size() * sizeof(HArgs),
                  hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(b->d_jobs, b->hjobs.data(), njobs * sizeof(JobDev),
                  hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(b->d_steps, steps.data(), njobs * sizeof(int *),
                  hipMemcpyHostToDevice) != hipSuccess) {
        ks_batch_destroy(b);
        return fail(KS_E_HIP, "upload of the job table failed");
    }
    // non-finite norm flags, cleared once (they stay set once raised)
    if ((rc = batch_alloc(b, &b->d_flags, njobs)) ||
        hipMemset(b->d_flags, 0, njobs * sizeof(int)) != hipSuccess ||
        (rc = batch_alloc(b, &b->h_flags, njobs, true)) ||
        hipEventCreateWithFlags(&b->flag_ev, hipEventDisableTiming) !=
            hipSuccess) {
        ks_batch_destroy(b);
        return rc ? rc : fail(KS_E_HIP, "batch flag buffers");
    }
    std::memset(b->h_flags, 0, njobs * sizeof(int));   // a reused block
    // FP32 potential copies of the mixed jobs, per exponential
    if (mixed) {
        std::vector<F32Copy> c0(njobs), c1(njobs);
        std::vector<int> off(njobs + 1, 0);
        for (int i = 0; i < njobs; ++i) {
            ks_grid *g = b->grids[i];
            const JobDev &J = b->hjobs[i];
            float *dst = wsp<float>(g, g->lay.v32);
            c0[i] = F32Copy{J.vcur, dst, g->geo.N};
            c1[i] = F32Copy{J.nonlin ? J.vpred : J.vion, dst, g->geo.N};
            off[i + 1] = off[i] + (int)((g->geo.N + 255) / 256);
        }
        b->conv_blocks = off[njobs];
        if ((rc = batch_alloc(b, &b->d_conv[0], njobs)) ||
            (rc = batch_alloc(b, &b->d_conv[1], njobs)) ||
            (rc = batch_alloc(b, &b->d_conv_off, njobs + 1)) ||
            hipMemcpy(b->d_conv[0], c0.data(), njobs * sizeof(F32Copy),
                      hipMemcpyHostToDevice) != hipSuccess ||
            hipMemcpy(b->d_conv[1], c1.data(), njobs * sizeof(F32Copy),
                      hipMemcpyHostToDevice) != hipSuccess ||
            hipMemcpy(b->d_conv_off, off.data(), (njobs + 1) * sizeof(int),
                      hipMemcpyHostToDevice) != hipSuccess) {
            ks_batch_destroy(b);
            return rc ? rc : fail(KS_E_HIP, "upload of the FP32 copy tables");
        }
    }
    // tables of the batched reductions (the same arguments the single-job
    // propagator passes)
    {
        std::vector<DArgs> dpred, dend;
        std::vector<int> opred(1, 0), oend(1, 0);
        std::vector<DipJob> dip;
        std::vector<NormJob> nrm;
        for (int i = 0; i < njobs; ++i) {
            ks_grid *g = b->grids[i];
            const ks_job &jb = b->jobs[i];
            const double h3 = g->geo.h[0] * g->geo.h[1] * g->geo.h[2];
            const int *step = b->hjobs[i].step;
            const int nb = density_blocks(g->geo.N);
            DArgs a;
            a.geo = g->geo;
            a.nsrc = g->stot;
            a.npart = b->hjobs[i].npart;
            a.rho = wsp<double>(g, g->lay.rho);
            a.vion = jb.d_vion;
            a.xc = g->xc;
            if (g->nonlin) {
                a.vout = wsp<double>(g, g->lay.vpred);
                dpred.push_back(a);
                opred.push_back(opred.back() + nb);
            }
            if (b->hjobs[i].npart_end) {
                a.vout = g->d_v;
                a.dpart = jb.d_dipole ? wsp<double>(g, g->lay.dpart)
                                      : nullptr;
                dend.push_back(a);
                oend.push_back(oend.back() + nb);
                if (jb.d_dipole) {
                    DipJob d;
                    d.dpart = a.dpart;
                    d.nblocks = nb;
                    d.h3 = h3;
                    d.out = jb.d_dipole;
                    d.step = step;
                    dip.push_back(d);
                }
            }
            if (jb.d_norms) {
                NormJob n;
                n.part = wsp<double>(g, g->lay.normpart);
                n.ns = g->stot;
                n.ntiles = g->ntile_y * g->nzc;
                n.h3 = h3;
                n.out = jb.d_norms;
                n.step = step;
                n.flag = b->d_flags + i;
                nrm.push_back(n);
                b->max_ns = std::max(b->max_ns, g->stot);
            }
        }
        if ((long)opred.back() + oend.back() >= (1L << 31)) {
            ks_batch_destroy(b);
            return fail(KS_E_UNSUPPORTED, "batch densities too large");
        }
        b->npred = (int)dpred.size();
        b->nend = (int)dend.size();
        b->blk_pred = opred.back();
        b->blk_end = oend.back();
        b->ndip = (int)dip.size();
        b->nnorm = (int)nrm.size();
        auto put = [&](auto **dst, const auto &v) -> int {
            int r = batch_alloc(b, dst, v.size());
            if (r)
                return r;
            if (!v.empty() &&
                hipMemcpy(*dst, v.data(), v.size() * sizeof(v[0]),
                          hipMemcpyHostToDevice) != hipSuccess)
                return fail(KS_E_HIP, "upload of the reduction tables failed");
            return KS_OK;
        };
        if ((rc = put(&b->d_dpred, dpred)) ||
            (rc = put(&b->d_dpred_off, opred)) ||
            (rc = put(&b->d_dend, dend)) || (rc = put(&b->d_dend_off, oend)) ||
            (rc = put(&b->d_dip, dip)) || (rc = put(&b->d_norm, nrm))) {
            ks_batch_destroy(b);
            return rc;
        }
    }
    // grids of one work item per workgroup (a multiple of 8, XCD-aware
    // order): items of different jobs differ in cost, and the hardware
    // dispatcher hands the next item to whichever CU frees first, where a
    // fixed chain of items per workgroup would end with its longest chain
    // (measured on the serving mix: 6 % shorter steps than chains of ~6
    // items on 1024 workgroups).  At most 2^22 workgroups (2^31 threads of
    // 512); beyond that each takes every 2^22-th item.
    auto pgrid = [](int items) {
        const int g = std::min(std::max(items, 1), 1 << 22);
        return ((g + 7) / 8) * 8;
    };
    b->grid_hpsi = pgrid(b->off_total[kItemHpsi]);
    b->grid_proj = pgrid(std::max({b->off_total[kItemGather],
                                   b->off_total[kItemGatherFin],
                                   b->off_total[kItemApply]}));
    // initial potential, dipole and norms of every job that starts at step
    // 0; a resumed job keeps the potential its grid holds from the end of
    // its last step (eager)
    for (int i = 0; i < njobs; ++i) {
        ks_grid *g = b->grids[i];
        const ks_job &jb = b->jobs[i];
        if (jb.first_step > 0)
            continue;
        const double h3 = g->geo.h[0] * g->geo.h[1] * g->geo.h[2];
        DArgs a;
        a.geo = g->geo;
        a.nsrc = g->stot;
        a.psi = static_cast<const double2 *>(jb.d_psi);
        a.wocc = g->d_wocc;
        a.rho = wsp<double>(g, g->lay.rho);
        a.vion = jb.d_vion;
        a.vout = g->d_v;
        a.xc = g->xc;
        a.dpart = jb.d_dipole ? wsp<double>(g, g->lay.dpart) : nullptr;
        hipError_t e = launch_density(a, b->stream);
        if (e == hipSuccess && g->hartree)
            e = launch_hartree(g->pp, g->geo, a.rho, a.vout, true,
                               wsp<double2>(g, g->lay.pwork), b->stream);
        if (e == hipSuccess && jb.d_dipole)
            e = launch_dipole_finalize(a.dpart, density_blocks(g->geo.N), h3,
                                       jb.d_dipole, b->stream);
        if (e == hipSuccess && jb.d_norms) {
            double *part = wsp<double>(g, g->lay.normpart);
            e = launch_norm_partial(g->geo,
                                    static_cast<const double2 *>(jb.d_psi),
                                    g->stot, g->norm_chunks, part, b->stream);
            if (e == hipSuccess)
                e = launch_norm_finalize(part, g->stot, g->norm_chunks, h3,
                                         jb.d_norms, b->stream);
        }
        if (e != hipSuccess) {
            ks_batch_destroy(b);
            return fail(KS_E_HIP, "batch initialisation: %s",
                        hipGetErrorString(e));
        }
        g->vloc_set = true;
    }
    std::vector<int> first(njobs);
    for (int i = 0; i < njobs; ++i)
        first[i] = jobs[i].first_step;
    int *d_first = nullptr;
    if ((rc = batch_alloc(b, &d_first, njobs))) {
        ks_batch_destroy(b);
        return rc;
    }
    if (hipMemcpy(d_first, first.data(), njobs * sizeof(int),
                  hipMemcpyHostToDevice) != hipSuccess ||
        launch_step_set(b->d_steps, njobs, d_first, b->stream) !=
            hipSuccess) {
        ks_batch_destroy(b);
        return fail(KS_E_HIP, "batch initialisation failed");
    }
    b->steps_done = first;
    *out = b;
    return KS_OK;
}

int ks_batch_set_graph(ks_batch *b, int use_graph)
{
    if (!b)
        return fail(KS_E_ARG, "batch is NULL");
    b->use_graph = use_graph != 0;
    return KS_OK;
}

int ks_batch_step(ks_batch *b, int nsteps)
{
    if (!b || nsteps < 0)
        return fail(KS_E_ARG, "batch is NULL or nsteps < 0");
    for (size_t i = 0; i < b->jobs.size(); ++i)
        if (b->steps_done[i] + nsteps > b->jobs[i].max_steps)
            return fail(KS_E_ARG, "job %zu would exceed its %d steps", i,
                        b->jobs[i].max_steps);
    if (nsteps == 0)
        return KS_OK;
    int frc = batch_poll_flags(b, false);
    if (frc)
        return frc;
    if (b->use_graph) {
        if (!b->exec) {
            KS_HIP(hipStreamBeginCapture(b->stream,
                                         hipStreamCaptureModeThreadLocal));
            int rc = batch_enqueue_step(b);
            hipGraph_t graph = nullptr;
            hipError_t e = hipStreamEndCapture(b->stream, &graph);
            if (rc) {
                if (graph)
                    (void)hipGraphDestroy(graph);
                return rc;
            }
            if (e != hipSuccess)
                return fail(KS_E_HIP, "graph capture: %s",
                            hipGetErrorString(e));
            b->graph = graph;
            KS_HIP(hipGraphInstantiate(&b->exec, graph, nullptr, nullptr, 0));
        }
        for (int s = 0; s < nsteps; ++s)
            KS_HIP(hipGraphLaunch(b->exec, b->stream));
    } else {
        for (int s = 0; s < nsteps; ++s) {
            int rc = batch_enqueue_step(b);
            if (rc)
                return rc;
        }
    }
    for (auto &d : b->steps_done)
        d += nsteps;
    KS_HIP(hipMemcpyAsync(b->h_flags, b->d_flags,
                          b->jobs.size() * sizeof(int),
                          hipMemcpyDeviceToHost, b->stream));
    KS_HIP(hipEventRecord(b->flag_ev, b->stream));
    b->flag_pending = true;
    return KS_OK;
}

int ks_batch_steps_done(const ks_batch *b, int job, int *out)
{
    if (!b || !out || job < 0 || job >= (int)b->jobs.size())
        return fail(KS_E_ARG, "bad batch, job or output");
    *out = b->steps_done[job];
    return KS_OK;
}

int ks_batch_destroy(ks_batch *b)
{
    if (!b)
        return KS_OK;
    (void)hipStreamSynchronize(b->stream);
    const int rc = b->h_flags && b->flag_ev ? batch_poll_flags(b, true)
                                            : KS_OK;
    if (b->exec)
        (void)hipGraphExecDestroy(b->exec);
    if (b->graph)
        (void)hipGraphDestroy(b->graph);
    for (const PoolBlock &blk : b->owned)
        pool_put(blk);
    if (b->flag_ev)
        (void)hipEventDestroy(b->flag_ev);
    delete b;
    return rc;
}

}  // extern "C"
