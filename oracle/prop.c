/*
 * oracle/prop.c -- FP64 reference time loops for the constant-density
 * acoustic operator, forward and adjoint.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the plain, slow, obviously
 * correct CPU definition that the GPU path is checked against.  Only the
 * test suite, the smoke check and the CPU-baseline leg of the benchmark
 * load it.  It shares no code, header or constant with the GPU library.
 *
 * What is computed (paper: eq. (wave) of Sec. 2.1, the 2nd-order-in-time /
 * 8th-order-in-space scheme and absorbing boundary of Sec. 4.1, the
 * receiver projection R of Sec. 2.1 and the adjoint equation (FWI_lambda)):
 *
 *   padded grid = physical grid plus nb cells on every side; values outside
 *   the padded grid are zero, so the discrete Laplacian L is symmetric.
 *
 *   forward, n = 0 .. nt-1, u^{-1} = u^0 = 0:
 *     (1+k) u^{n+1} = 2 u^n - (1-k) u^{n-1} + c (L u^n + P q^n)
 *     d^n = R u^{n+1}
 *   adjoint, j = nt-1 .. 0, mu^{nt} = mu^{nt+1} = 0:
 *     (1+k) mu^j = 2 mu^{j+1} - (1-k) mu^{j+2} + c (L mu^{j+1} + R^T d^j)
 *     out^j = P^T mu^j
 *
 * c = v^2 dt^2 and k = eta dt / 2 are given per padded point by the caller
 * (oracle/core.py builds them).  The Laplacian weights w[0..4] are given by
 * the caller too (derived there from a Taylor/Vandermonde system).
 *
 * Everything is double precision.  The only parallelism is an OpenMP loop
 * over independent grid rows; every reduction is serial, so results do not
 * depend on the thread count.
 */
#include <stdlib.h>
#include <string.h>

typedef struct {
    int ndim;            /* 2 or 3 */
    int nz, ny, nx;      /* physical grid (ny = 1 in 2D) */
    int nb;              /* pad width on every side */
    int nt;              /* time steps */
    double w[5];         /* Laplacian weights a_0..a_4 (dimensionless) */
    double inv_dx2;      /* 1 / dx^2 */
    double inv_dt2;      /* 1 / dt^2 */
} or_grid;

static long pz(const or_grid* g) { return g->nz + 2L * g->nb; }
static long py(const or_grid* g) { return g->ndim == 3 ? g->ny + 2L * g->nb : 1; }
static long px(const or_grid* g) { return g->nx + 2L * g->nb; }

long or_padded_size(const or_grid* g) { return pz(g) * py(g) * px(g); }
long or_phys_size(const or_grid* g) { return (long)g->nz * g->ny * g->nx; }

/* value of u at padded (z,y,x), zero outside the padded grid */
static double at(const or_grid* g, const double* u, long z, long y, long x)
{
    if (z < 0 || z >= pz(g) || y < 0 || y >= py(g) || x < 0 || x >= px(g))
        return 0.0;
    return u[(z * py(g) + y) * px(g) + x];
}

/* (L u) at padded (z,y,x): sum over the active axes of the 9-point
 * centred second difference, divided by dx^2. */
static double lap(const or_grid* g, const double* u, long z, long y, long x)
{
    double s = 0.0;
    for (int d = 0; d < g->ndim; ++d) {
        long ez = 0, ey = 0, ex = 0;
        if (d == 0) ex = 1;
        else if (d == 1) ez = 1;
        else ey = 1;
        double t = g->w[0] * at(g, u, z, y, x);
        for (long k = 1; k <= 4; ++k)
            t += g->w[k] * (at(g, u, z + k * ez, y + k * ey, x + k * ex) +
                            at(g, u, z - k * ez, y - k * ey, x - k * ex));
        s += t;
    }
    return s * g->inv_dx2;
}

/* physical linear index of padded (z,y,x), or -1 outside the physical grid */
static long phys_index(const or_grid* g, long z, long y, long x)
{
    long jz = z - g->nb, jx = x - g->nb, jy = g->ndim == 3 ? y - g->nb : y;
    if (jz < 0 || jz >= g->nz || jx < 0 || jx >= g->nx || jy < 0 || jy >= g->ny)
        return -1;
    return (jz * g->ny + jy) * g->nx + jx;
}

/*
 * Forward modelling S = R A^{-1}.
 *   src_kind 0: point source, src[n] injected at padded index src_idx.
 *   src_kind 1: dense source, src[n*phys + p] on every physical cell.
 *   data[n*nrec + r] = u^{n+1} at padded index rec_idx[r].
 *   dtt (optional, may be NULL): dtt[n*phys + p] = v^2 (L u^n + P q^n) at
 *   physical cells, i.e. the discrete (d/dm) A(m) u used by the gradient.
 * Returns 0, or -1 if memory could not be allocated.
 */
int or_forward(const or_grid* g, const double* c, const double* kap,
               int src_kind, const double* src, long src_idx,
               int nrec, const long* rec_idx, double* data, double* dtt)
{
    const long N = or_padded_size(g), NP = or_phys_size(g);
    double* um = calloc(N, sizeof(double));   /* u^{n-1} */
    double* u0 = calloc(N, sizeof(double));   /* u^n     */
    double* up = calloc(N, sizeof(double));   /* u^{n+1} */
    if (!um || !u0 || !up) { free(um); free(u0); free(up); return -1; }

    for (int n = 0; n < g->nt; ++n) {
#pragma omp parallel for schedule(static)
        for (long z = 0; z < pz(g); ++z)
            for (long y = 0; y < py(g); ++y)
                for (long x = 0; x < px(g); ++x) {
                    long i = (z * py(g) + y) * px(g) + x;
                    long p = phys_index(g, z, y, x);
                    double q = 0.0;
                    if (src_kind == 0) {
                        if (i == src_idx) q = src[n];
                    } else if (p >= 0) {
                        q = src[(long)n * NP + p];
                    }
                    double lq = lap(g, u0, z, y, x) + q;
                    up[i] = (2.0 * u0[i] - (1.0 - kap[i]) * um[i] + c[i] * lq) /
                            (1.0 + kap[i]);
                    if (dtt && p >= 0)
                        dtt[(long)n * NP + p] = c[i] * g->inv_dt2 * lq;
                }
        for (int r = 0; r < nrec; ++r)
            data[(long)n * nrec + r] = up[rec_idx[r]];
        double* t = um; um = u0; u0 = up; up = t;
    }
    free(um); free(u0); free(up);
    return 0;
}

/*
 * Adjoint modelling S^T = A^{-T} R^T (same recurrence run backward in time).
 *   data[j*nrec + r] is injected at padded index rec_idx[r] at step j
 *   (receivers sharing a cell add up).
 *   out[j*phys + p] = mu^j at physical cells.
 */
int or_adjoint(const or_grid* g, const double* c, const double* kap,
               int nrec, const long* rec_idx, const double* data, double* out)
{
    const long N = or_padded_size(g), NP = or_phys_size(g);
    double* m2 = calloc(N, sizeof(double));   /* mu^{j+2} */
    double* m1 = calloc(N, sizeof(double));   /* mu^{j+1} */
    double* m0 = calloc(N, sizeof(double));   /* mu^j     */
    double* inj = calloc(N, sizeof(double));
    if (!m2 || !m1 || !m0 || !inj) {
        free(m2); free(m1); free(m0); free(inj); return -1;
    }
    for (int j = g->nt - 1; j >= 0; --j) {
        for (int r = 0; r < nrec; ++r)
            inj[rec_idx[r]] += data[(long)j * nrec + r];
#pragma omp parallel for schedule(static)
        for (long z = 0; z < pz(g); ++z)
            for (long y = 0; y < py(g); ++y)
                for (long x = 0; x < px(g); ++x) {
                    long i = (z * py(g) + y) * px(g) + x;
                    double lq = lap(g, m1, z, y, x) + inj[i];
                    m0[i] = (2.0 * m1[i] - (1.0 - kap[i]) * m2[i] + c[i] * lq) /
                            (1.0 + kap[i]);
                    long p = phys_index(g, z, y, x);
                    if (p >= 0) out[(long)j * NP + p] = m0[i];
                }
        for (int r = 0; r < nrec; ++r) inj[rec_idx[r]] = 0.0;
        double* t = m2; m2 = m1; m1 = m0; m0 = t;
    }
    free(m2); free(m1); free(m0); free(inj);
    return 0;
}
