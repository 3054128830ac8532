/*
 * nlse_oracle.c -- plain FP64 CPU oracle for the 2SHOC-RK4 integration of the NLSE
 *
 *     i Psi_t + a Lap(Psi) - V Psi + s |Psi|^2 Psi = 0          (Sec. 1, Eq. NLSE)
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the slow, obviously correct reference
 * the GPU library is checked against.  Only the test suite, the smoke check and
 * the CPU-baseline leg of the benchmark may load it.  It shares no code, header,
 * constant table or helper with the GPU library, and the GPU library never calls
 * it.
 *
 * Every step follows the paper in its own order and notation:
 *   - step 1 of 2SHOC, the second-order difference D (Sec. 2.1 Eq. 2shoc1d;
 *     Sec. 2.2 Eq. 2d2shocs1; Sec. 2.3 Eq. 3d2shocs);
 *   - the boundary closure of step 1 (Sec. 3.2: Dirichlet Eq. dbc_lap, MSD Eq. msdbc_lap,
 *     in 1D and, with the paper's remark that MSD carries over to several
 *     dimensions, in 2D/3D with b-1 the closest interior node);
 *   - step 2 of 2SHOC in the single-storage form (Eq. 2shoc1d2, 2d2shocs2, 3d2shocs2);
 *   - F(Psi) = i[a Lap + (s|Psi|^2 - V) Psi] on the interior, then the boundary
 *     time derivative (Eq. dbc_ut, Eq. msdbc_ut), interior first, boundary second;
 *   - classic RK4 as the ten array operations of Sec. 3.1 Eq. RK4.
 * Alternatives kept for the equivalence pins: the per-axis (multi-storage) forms
 * (Eq. 2d2shocMs1-2, 3d2shocMs1-2), the non-compact fourth-order stencils
 * (Sec. 2.1, Eq. 2dnonhoc, Sec. 2.3) and the second-order central difference
 * "CD" (Sec. 3.1).
 *
 * Build: gcc -O2 -ffp-contract=off -fno-fast-math -fopenmp -shared -fPIC.
 * No fused multiply-add, constants precomputed once (Sec. 5 counts operations
 * with divisions hoisted the same way).  OpenMP only splits independent
 * per-node loops; every reduction is a serial loop in node order.
 *
 * Storage: n[a] intervals per axis, n[a] + 1 nodes including both boundary
 * nodes, C order [z][y][x] with x fastest, complex values interleaved (re, im).
 */
#include <complex.h>
#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef double complex zd;

enum { ORC_DIRICHLET = 0, ORC_MSD = 1 };
enum { ORC_LAP_2SHOC = 0, ORC_LAP_2SHOC_AXIS = 1, ORC_LAP_NONCOMPACT = 2, ORC_LAP_CD = 3 };

typedef struct {
    int dim;          /* 1, 2 or 3 */
    long n[3];        /* intervals per axis (unused axes ignored) */
    double h, a, s;   /* grid step (same on every axis), a > 0, s */
    const double *V;  /* real potential on every node, or NULL for V = 0 */
    int bc;           /* ORC_DIRICHLET or ORC_MSD */
    int lap;          /* ORC_LAP_* */
} orc_problem;

/* ------------------------------------------------------------------ grid -- */

typedef struct {
    long m[3];    /* nodes per axis (1 for unused axes) */
    long st[3];   /* strides */
    long total;
} geom;

static geom make_geom(const orc_problem *P)
{
    geom g;
    for (int a = 0; a < 3; ++a) g.m[a] = (a < P->dim) ? P->n[a] + 1 : 1;
    g.st[0] = 1;
    g.st[1] = g.m[0];
    g.st[2] = g.m[0] * g.m[1];
    g.total = g.m[0] * g.m[1] * g.m[2];
    return g;
}

static int is_interior(const orc_problem *P, const long idx[3])
{
    for (int a = 0; a < P->dim; ++a)
        if (idx[a] == 0 || idx[a] == P->n[a]) return 0;
    return 1;
}

static void coords_of(const geom *g, long p, long idx[3])
{
    idx[0] = p % g->m[0];
    idx[1] = (p / g->m[0]) % g->m[1];
    idx[2] = p / (g->m[0] * g->m[1]);
}

static double pot(const orc_problem *P, long p) { return P->V ? P->V[p] : 0.0; }

static double abs2(zd z) { return creal(z) * creal(z) + cimag(z) * cimag(z); }

static zd times_i(zd z) { return CMPLX(-cimag(z), creal(z)); }

/* N = s|Psi|^2 - V  (Eq. nbnb1) */
static double nonlin(const orc_problem *P, const zd *psi, long p)
{
    return P->s * abs2(psi[p]) - pot(P, p);
}

static int validate(const orc_problem *P)
{
    if (P->dim < 1 || P->dim > 3) return -1;
    for (int a = 0; a < P->dim; ++a)
        if (P->n[a] < 2) return -1;
    if (!(P->h > 0.0) || !(P->a > 0.0)) return -1;
    if (P->bc != ORC_DIRICHLET && P->bc != ORC_MSD) return -1;
    if (P->lap < ORC_LAP_2SHOC || P->lap > ORC_LAP_CD) return -1;
    return 0;
}

/* ------------------------------------------- step 1: second differences -- */

/* D on interior nodes: the standard 3/5/7-point Laplacian divided by h^2
 * (Eq. 2shoc1d, Eq. 2d2shocs1, Eq. 3d2shocs). */
static void step1_interior(const orc_problem *P, const geom *g, const zd *psi, zd *D)
{
    const double ih2 = 1.0 / (P->h * P->h);
    const long s1 = g->st[1], s2 = g->st[2];
    long nz = g->m[2], ny = g->m[1], nx = g->m[0];
#pragma omp parallel for collapse(2) schedule(static)
    for (long k = 0; k < nz; ++k)
        for (long j = 0; j < ny; ++j)
            for (long i = 0; i < nx; ++i) {
                long idx[3] = {i, j, k};
                if (!is_interior(P, idx)) continue;
                long p = i + j * s1 + k * s2;
                if (P->dim == 1)
                    D[p] = ih2 * (psi[p + 1] - 2.0 * psi[p] + psi[p - 1]);
                else if (P->dim == 2)
                    D[p] = ih2 * (psi[p + 1] + psi[p - 1] + psi[p + s1] + psi[p - s1] - 4.0 * psi[p]);
                else
                    D[p] = ih2 * (psi[p + 1] + psi[p - 1] + psi[p + s1] + psi[p - s1]
                                  + psi[p + s2] + psi[p - s2] - 6.0 * psi[p]);
            }
}

/* Dirichlet closure of step 1: Lap Psi_b = -(s|Psi_b|^2 - V_b) Psi_b / a (Eq. dbc_lap). */
static zd dirichlet_lap_b(const orc_problem *P, const zd *psi, long b)
{
    return -(nonlin(P, psi, b) * psi[b]) / P->a;
}

/* The node b-1 of the MSD rule for boundary node p (Sec. 3.2): the closest
 * interior node, one step inward along every axis on which p is a boundary
 * node.  For a face node that is the inward neighbour in the normal direction,
 * as the paper defines it; for an edge or corner node (boundary in two or three
 * axes, where the normal is not defined) it is the diagonal interior neighbour. */
static long msd_inner(const orc_problem *P, const geom *g, long p)
{
    long idx[3];
    coords_of(g, p, idx);
    long q = p;
    for (int a = 0; a < P->dim; ++a) {
        if (idx[a] == 0) q += g->st[a];
        else if (idx[a] == P->n[a]) q -= g->st[a];
    }
    return q;
}

/* MSD closure of step 1 (Eq. msdbc_lap):
 *   Lap Psi_b = [ Im(i D_{b-1} / Psi_{b-1}) + (N_{b-1} - N_b) / a ] Psi_b,
 * with Im(i z) = Re(z).  D_{b-1} is the step-1 value at the inner node b-1.
 * A zero inner value leaves the ratio term out. */
static zd msd_lap_b(const orc_problem *P, const zd *psi, const zd *D, long b, long bm1)
{
    double ratio = 0.0;
    if (psi[bm1] != 0.0) ratio = creal(D[bm1] / psi[bm1]);
    double Nb = nonlin(P, psi, b), Nbm1 = nonlin(P, psi, bm1);
    return (ratio + (Nbm1 - Nb) / P->a) * psi[b];
}

static void step1_boundary(const orc_problem *P, const geom *g, const zd *psi, zd *D)
{
    /* interior first (already done), boundary second; b-1 is always interior */
    for (long p = 0; p < g->total; ++p) {
        long idx[3];
        coords_of(g, p, idx);
        if (is_interior(P, idx)) continue;
        D[p] = P->bc == ORC_MSD ? msd_lap_b(P, psi, D, p, msd_inner(P, g, p)) : dirichlet_lap_b(P, psi, p);
    }
}

/* ----------------------------------------------- step 2: the Laplacian -- */

/* Single-storage step 2 (Eq. 2shoc1d2, Eq. 2d2shocs2, Eq. 3d2shocs2) on interior nodes. */
static void step2_single(const orc_problem *P, const geom *g, const zd *psi, const zd *D, zd *lap)
{
    const double c76 = 7.0 / 6.0, c112 = 1.0 / 12.0, c6h2 = 1.0 / (6.0 * P->h * P->h);
    const long s1 = g->st[1], s2 = g->st[2];
    long nz = g->m[2], ny = g->m[1], nx = g->m[0];
#pragma omp parallel for collapse(2) schedule(static)
    for (long k = 0; k < nz; ++k)
        for (long j = 0; j < ny; ++j)
            for (long i = 0; i < nx; ++i) {
                long idx[3] = {i, j, k};
                if (!is_interior(P, idx)) continue;
                long p = i + j * s1 + k * s2;
                if (P->dim == 1) {
                    lap[p] = c76 * D[p] - c112 * (D[p + 1] + D[p - 1]);
                } else if (P->dim == 2) {
                    zd faces = D[p + 1] + D[p - 1] + D[p + s1] + D[p - s1];
                    zd corners = psi[p + 1 + s1] + psi[p - 1 + s1] + psi[p + 1 - s1] + psi[p - 1 - s1];
                    lap[p] = -c112 * (faces - 12.0 * D[p]) + c6h2 * (corners - 4.0 * psi[p]);
                } else {
                    zd faces = D[p + 1] + D[p - 1] + D[p + s1] + D[p - s1] + D[p + s2] + D[p - s2];
                    /* the 12 nodes at distance sqrt(2) h: the four in-plane corners of each
                     * of the xy, xz and yz planes through the node */
                    zd edges = psi[p + 1 + s1] + psi[p - 1 + s1] + psi[p + 1 - s1] + psi[p - 1 - s1]
                             + psi[p + 1 + s2] + psi[p - 1 + s2] + psi[p + 1 - s2] + psi[p - 1 - s2]
                             + psi[p + s1 + s2] + psi[p - s1 + s2] + psi[p + s1 - s2] + psi[p - s1 - s2];
                    lap[p] = -c112 * (faces - 10.0 * D[p]) + c6h2 * (edges - 12.0 * psi[p]);
                }
            }
}

/* Per-axis step-1 value on a face node q normal to axis a, the boundary closure of the
 * per-axis forms.  The paper gives no rule for D^a on the boundary.  This oracle takes the
 * step-1 boundary value of q (Eq. dbc_lap or Eq. msdbc_lap, held in Dfull) minus the
 * central differences along the face, so that the D^a of q sum to the single-storage
 * boundary value.  q must lie on exactly one boundary (its tangential neighbours exist). */
static zd face_value(const orc_problem *P, const geom *g, const zd *psi, const zd *Dfull, long q, int a)
{
    const double ih2 = 1.0 / (P->h * P->h);
    zd tang = 0.0;
    for (int b = 0; b < P->dim; ++b)
        if (b != a) tang += ih2 * (psi[q + g->st[b]] - 2.0 * psi[q] + psi[q - g->st[b]]);
    return Dfull[q] - tang;
}

/* The full step-1 array: interior differences and the boundary closure. */
static zd *step1_full(const orc_problem *P, const geom *g, const zd *psi)
{
    zd *Dfull = calloc((size_t)g->total, sizeof(zd));
    step1_interior(P, g, psi, Dfull);
    step1_boundary(P, g, psi, Dfull);
    return Dfull;
}

/* Per-axis (multi-storage) 2SHOC (Eq. 2d2shocMs1-2, Eq. 3d2shocMs1-2):
 *   D^a = delta_a^2 Psi,  Lap = sum_a [ (7/6) D^a - (1/12)(D^a_{+a} + D^a_{-a}) ],
 * with D^a on a face node normal to a from face_value.  Only D^a on faces normal to
 * a is ever read. */
static void lap_per_axis(const orc_problem *P, const geom *g, const zd *psi, zd *lap)
{
    const double ih2 = 1.0 / (P->h * P->h), c76 = 7.0 / 6.0, c112 = 1.0 / 12.0;
    zd *Da[3] = {NULL, NULL, NULL};
    for (int a = 0; a < P->dim; ++a) Da[a] = calloc((size_t)g->total, sizeof(zd));
    zd *Dfull = step1_full(P, g, psi);
    for (long p = 0; p < g->total; ++p) {
        long idx[3];
        coords_of(g, p, idx);
        int nb = 0, bax = -1;
        for (int a = 0; a < P->dim; ++a)
            if (idx[a] == 0 || idx[a] == P->n[a]) { ++nb; bax = a; }
        if (nb == 0) {
            for (int a = 0; a < P->dim; ++a)
                Da[a][p] = ih2 * (psi[p + g->st[a]] - 2.0 * psi[p] + psi[p - g->st[a]]);
        } else if (nb == 1) {
            Da[bax][p] = face_value(P, g, psi, Dfull, p, bax);
        }
    }
    for (long p = 0; p < g->total; ++p) {
        long idx[3];
        coords_of(g, p, idx);
        if (!is_interior(P, idx)) continue;
        zd acc = 0.0;
        for (int a = 0; a < P->dim; ++a) {
            long st = g->st[a];
            acc += c76 * Da[a][p] - c112 * (Da[a][p + st] + Da[a][p - st]);
        }
        lap[p] = acc;
    }
    for (int a = 0; a < P->dim; ++a) free(Da[a]);
    free(Dfull);
}

/* Value of Psi along axis a at offset off from the interior node p.  One node beyond a
 * boundary node b it is the ghost Psi_{b-+1} = 2 Psi_b - Psi_{b+-1} + h^2 D^a_b, the value
 * whose second difference at b is the step-1 boundary value D^a_b (face_value, from Eq.
 * dbc_lap): with it the five-point stencil next to the boundary is exactly the 2SHOC
 * combination (7/6) D^a - (1/12)(neighbouring D^a) that Sec. 2.1 shows it equals.  With zero
 * boundary values D^a_b = 0 and the ghost is the odd reflection. */
static zd along(const orc_problem *P, const geom *g, const zd *psi, const zd *Dfull, long p, const long idx[3],
                int a, int off)
{
    long t = idx[a] + off;
    long st = g->st[a];
    const double h2 = P->h * P->h;
    if (t < 0) {
        long pb = p - idx[a] * st;
        return 2.0 * psi[pb] - psi[pb + st] + h2 * face_value(P, g, psi, Dfull, pb, a);
    }
    if (t > P->n[a]) {
        long pb = p + (P->n[a] - idx[a]) * st;
        return 2.0 * psi[pb] - psi[pb - st] + h2 * face_value(P, g, psi, Dfull, pb, a);
    }
    return psi[p + off * st];
}

/* Non-compact fourth-order stencil per axis (Sec. 2.1, Eq. 2dnonhoc, Sec. 2.3):
 *   (-Psi_{+2} + 16 Psi_{+1} - 30 Psi + 16 Psi_{-1} - Psi_{-2}) / (12 h^2). */
static void lap_noncompact(const orc_problem *P, const geom *g, const zd *psi, zd *lap)
{
    const double i12h2 = 1.0 / (12.0 * P->h * P->h);
    zd *Dfull = step1_full(P, g, psi);
    for (long p = 0; p < g->total; ++p) {
        long idx[3];
        coords_of(g, p, idx);
        if (!is_interior(P, idx)) continue;
        zd acc = 0.0;
        for (int a = 0; a < P->dim; ++a) {
            zd m2 = along(P, g, psi, Dfull, p, idx, a, -2), p2 = along(P, g, psi, Dfull, p, idx, a, 2);
            acc += i12h2 * (-p2 + 16.0 * psi[p + g->st[a]] - 30.0 * psi[p]
                            + 16.0 * psi[p - g->st[a]] - m2);
        }
        lap[p] = acc;
    }
    free(Dfull);
}

/* Laplacian of the chosen form on every interior node (boundary entries untouched). */
static void laplacian(const orc_problem *P, const geom *g, const zd *psi, zd *lap, zd *D)
{
    switch (P->lap) {
    case ORC_LAP_2SHOC:
        step1_interior(P, g, psi, D);
        step1_boundary(P, g, psi, D);
        step2_single(P, g, psi, D, lap);
        break;
    case ORC_LAP_2SHOC_AXIS:
        lap_per_axis(P, g, psi, lap);
        break;
    case ORC_LAP_NONCOMPACT:
        lap_noncompact(P, g, psi, lap);
        break;
    default: /* CD: the step-1 value is the (second-order) Laplacian */
        step1_interior(P, g, psi, lap);
        break;
    }
}

/* ---------------------------------------------------------- F(Psi) -- */

/* F = i[a Lap + (s|Psi|^2 - V) Psi] on the interior (Sec. 3.1), then the boundary:
 * Dirichlet F_b = 0 (Eq. dbc_ut); MSD F_b = i Im(F_{b-1} / Psi_{b-1}) Psi_b (Eq. msdbc_ut). */
static void rhs(const orc_problem *P, const geom *g, const zd *psi, zd *F, zd *lap, zd *D)
{
    laplacian(P, g, psi, lap, D);
    const long s1 = g->st[1], s2 = g->st[2];
    long nz = g->m[2], ny = g->m[1], nx = g->m[0];
#pragma omp parallel for collapse(2) schedule(static)
    for (long k = 0; k < nz; ++k)
        for (long j = 0; j < ny; ++j)
            for (long i = 0; i < nx; ++i) {
                long idx[3] = {i, j, k};
                long p = i + j * s1 + k * s2;
                if (!is_interior(P, idx)) { F[p] = 0.0; continue; }
                F[p] = times_i(P->a * lap[p] + nonlin(P, psi, p) * psi[p]);
            }
    if (P->bc == ORC_MSD) {   /* every interior F first, then the boundary */
        for (long b = 0; b < g->total; ++b) {
            long idx[3];
            coords_of(g, b, idx);
            if (is_interior(P, idx)) continue;
            long bm1 = msd_inner(P, g, b);
            double im = 0.0;
            if (psi[bm1] != 0.0) im = cimag(F[bm1] / psi[bm1]);
            F[b] = CMPLX(0.0, im) * psi[b];
        }
    }
}

/* ------------------------------------------------------------ exports -- */

int orc_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

void orc_set_threads(int t)
{
#ifdef _OPENMP
    if (t > 0) omp_set_num_threads(t);
#else
    (void)t;
#endif
}

long orc_nodes(const orc_problem *P)
{
    if (validate(P)) return -1;
    return make_geom(P).total;
}

/* Laplacian of the chosen form; boundary entries of out are set to 0. */
int orc_laplacian(const orc_problem *P, const double *psi_in, double *out)
{
    int e = validate(P);
    if (e) return e;
    geom g = make_geom(P);
    zd *D = calloc((size_t)g.total, sizeof(zd));
    zd *lap = (zd *)out;
    memset(lap, 0, sizeof(zd) * (size_t)g.total);
    laplacian(P, &g, (const zd *)psi_in, lap, D);
    free(D);
    return 0;
}

/* Step-1 array D including its boundary closure (single-storage form). */
int orc_step1(const orc_problem *P, const double *psi_in, double *out)
{
    int e = validate(P);
    if (e) return e;
    geom g = make_geom(P);
    zd *D = (zd *)out;
    memset(D, 0, sizeof(zd) * (size_t)g.total);
    step1_interior(P, &g, (const zd *)psi_in, D);
    step1_boundary(P, &g, (const zd *)psi_in, D);
    return 0;
}

int orc_rhs(const orc_problem *P, const double *psi_in, double *out)
{
    int e = validate(P);
    if (e) return e;
    geom g = make_geom(P);
    zd *D = calloc((size_t)g.total, sizeof(zd));
    zd *lap = calloc((size_t)g.total, sizeof(zd));
    rhs(P, &g, (const zd *)psi_in, (zd *)out, lap, D);
    free(D);
    free(lap);
    return 0;
}

/* Classic RK4, the ten array operations of Sec. 3.1 Eq. RK4, nsteps steps of size k, in place. */
int orc_rk4(const orc_problem *P, double *psi_io, long nsteps, double k)
{
    int e = validate(P);
    if (e) return e;
    geom g = make_geom(P);
    const long N = g.total;
    zd *psi = (zd *)psi_io;
    zd *Ktot = calloc((size_t)N, sizeof(zd)), *Ktmp = calloc((size_t)N, sizeof(zd));
    zd *tmp = calloc((size_t)N, sizeof(zd));
    zd *lap = calloc((size_t)N, sizeof(zd)), *D = calloc((size_t)N, sizeof(zd));
    const double k2 = k / 2.0, k6 = k / 6.0;
    for (long step = 0; step < nsteps; ++step) {
        rhs(P, &g, psi, Ktot, lap, D);                                    /* 1  */
#pragma omp parallel for schedule(static)
        for (long p = 0; p < N; ++p) tmp[p] = psi[p] + k2 * Ktot[p];      /* 2  */
        rhs(P, &g, tmp, Ktmp, lap, D);                                    /* 3  */
#pragma omp parallel for schedule(static)
        for (long p = 0; p < N; ++p) {
            Ktot[p] = Ktot[p] + 2.0 * Ktmp[p];                            /* 4  */
            tmp[p] = psi[p] + k2 * Ktmp[p];                               /* 5  */
        }
        rhs(P, &g, tmp, Ktmp, lap, D);                                    /* 6  */
#pragma omp parallel for schedule(static)
        for (long p = 0; p < N; ++p) {
            Ktot[p] = Ktot[p] + 2.0 * Ktmp[p];                            /* 7  */
            tmp[p] = psi[p] + k * Ktmp[p];                                /* 8  */
        }
        rhs(P, &g, tmp, Ktmp, lap, D);                                    /* 9  */
#pragma omp parallel for schedule(static)
        for (long p = 0; p < N; ++p) psi[p] = psi[p] + k6 * (Ktot[p] + Ktmp[p]);  /* 10 */
    }
    free(Ktot); free(Ktmp); free(tmp); free(lap); free(D);
    return 0;
}

/* Mass M = h^d sum over all nodes |Psi|^2 (serial, node order). */
double orc_mass(const orc_problem *P, const double *psi_in)
{
    if (validate(P)) return NAN;
    geom g = make_geom(P);
    const zd *psi = (const zd *)psi_in;
    double acc = 0.0;
    for (long p = 0; p < g.total; ++p) acc += abs2(psi[p]);
    return pow(P->h, P->dim) * acc;
}

/* Energy E = h^d sum over interior nodes [ -a Re(conj(Psi) Lap Psi) + V |Psi|^2 - (s/2) |Psi|^4 ],
 * the discrete Hamiltonian of Eq. NLSE with the chosen Laplacian (serial, node order). */
double orc_energy(const orc_problem *P, const double *psi_in)
{
    if (validate(P)) return NAN;
    geom g = make_geom(P);
    const zd *psi = (const zd *)psi_in;
    zd *D = calloc((size_t)g.total, sizeof(zd)), *lap = calloc((size_t)g.total, sizeof(zd));
    laplacian(P, &g, psi, lap, D);
    double acc = 0.0;
    for (long p = 0; p < g.total; ++p) {
        long idx[3];
        coords_of(&g, p, idx);
        if (!is_interior(P, idx)) continue;
        double r2 = abs2(psi[p]);
        acc += -P->a * creal(conj(psi[p]) * lap[p]) + pot(P, p) * r2 - 0.5 * P->s * r2 * r2;
    }
    free(D); free(lap);
    return pow(P->h, P->dim) * acc;
}

/* Linearised stability bound (Sec. 3.3, Eq. kdfull with Tables t:bc2 and t:sumresults):
 *   k_max = sqrt(8) h^2 / (a max(|B|_inf, max_{i,j} |L_i - G_j|)),  L_i = (h^2/a)(s|Psi_i|^2 - V_i)
 * over interior nodes.  Only the extreme G values matter:
 *   max_{i,j} |L_i - G_j| = max(G_max - L_min, L_max - G_min).
 * B_b = 0 for Dirichlet; for MSD B_b = (h^2/(i a)) F_{b-1}/Psi_{b-1}, over every node b-1
 * that the MSD rule reads (the interior nodes next to the boundary).
 * Also returns L_min, L_max and |B|_inf through the optional out array (3 doubles). */
double orc_max_dt(const orc_problem *P, const double *psi_in, double *aux)
{
    static const double gmax[3] = {64.0 / 12.0, 128.0 / 12.0, 192.0 / 12.0};
    static const double gmin[3] = {-4.0 / 12.0, -8.0 / 12.0, -12.0 / 12.0};
    if (validate(P)) return NAN;
    geom g = make_geom(P);
    const zd *psi = (const zd *)psi_in;
    const double h2a = P->h * P->h / P->a;
    double lmin = INFINITY, lmax = -INFINITY, bmax = 0.0;
    for (long p = 0; p < g.total; ++p) {
        long idx[3];
        coords_of(&g, p, idx);
        if (!is_interior(P, idx)) continue;
        double L = h2a * nonlin(P, psi, p);
        if (L < lmin) lmin = L;
        if (L > lmax) lmax = L;
    }
    if (P->bc == ORC_MSD) {
        zd *F = calloc((size_t)g.total, sizeof(zd)), *D = calloc((size_t)g.total, sizeof(zd));
        zd *lap = calloc((size_t)g.total, sizeof(zd));
        rhs(P, &g, psi, F, lap, D);
        for (long b = 0; b < g.total; ++b) {
            long idx[3];
            coords_of(&g, b, idx);
            if (is_interior(P, idx)) continue;
            long q = msd_inner(P, &g, b);
            if (psi[q] != 0.0) {
                double B = h2a * cabs(F[q] / psi[q]);
                if (B > bmax) bmax = B;
            }
        }
        free(F); free(D); free(lap);
    }
    double m = gmax[P->dim - 1] - lmin;
    if (lmax - gmin[P->dim - 1] > m) m = lmax - gmin[P->dim - 1];
    if (bmax > m) m = bmax;
    if (aux) { aux[0] = lmin; aux[1] = lmax; aux[2] = bmax; }
    return sqrt(8.0) * P->h * P->h / (P->a * m);
}
