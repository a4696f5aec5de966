/*
 * CPU oracle of the particle time step of the non-hybrid PDF method
 * (Bakosi, Franzese & Boybeyi).  TEST INFRASTRUCTURE ONLY: a plain FP64 restatement
 * of the method that checks the GPU library.  It shares no source with it.
 *
 * One step n -> n+1 (Table 1 order with the two FEM solves removed; their fields
 * are frozen nodal inputs):
 *   1. particle loop (Table 2, right): for every particle, interpolate the nodal
 *      fields at its position (Eq. 37), advance velocity (Eq. 27 with the
 *      closure of Eqs. 11, 18), frequency (Eqs. 19-20) and position (Eq. 7),
 *      track it through the grid (Sec. 3.6) applying the particle boundary
 *      conditions (Sec. 3.8), and apply the scalar source (Sec. 4.1.2);
 *   2. group particles by host element; in every element build the velocity
 *      bins by the sort-and-divide procedure (Sec. 3.5, App. A) and apply IECM
 *      mixing (Eq. 24) with the timescale of Eq. (25);
 *   3. estimate nodal statistics (Sec. 3.3) from the particles of the elements
 *      around each node, weighted by the P1 shape functions (Eq. 37).
 * Number control (Sec. 3.7, App. B) is a separate call.
 *
 * Arithmetic is IEEE double throughout, written for readability, not speed.
 */
#include "orc.h"

#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* nodal field record: grad<P>(2), wp(6), <U>(3), lap<U>(3), <omega>(1), R(6) */
#define NF 24
/* nodal fields: grad<P> (2), wp_11, wp_22, wp_33, wp_12, wp_13, wp_23 (6), <U> (3),
   lap<U> (3), <omega>, R (6), wp_21, wp_31, wp_32 (3: wp is not symmetric, Eq. 13) */
enum { F_GP = 0, F_WP = 2, F_MU = 8, F_LAP = 11, F_OM = 14, F_RE = 15, F_WPT = 21 };
enum { TAG_INIT = 1, TAG_STEP = 2, TAG_WALL_GAMMA = 3, TAG_INIT_GAMMA = 4 };
enum { K_INTERIOR = 0, K_WALL = 1, K_SLIP = 2, K_PERIODIC = 3 };
#define MAX_WALK 64
#define MAX_REFL 4
#define GAMMA_ATTEMPTS 16
#define NSTAT 13

struct orc_grid {
    int64_t nn, ne;
    double period;
    double* xy;       /* [nn][2] */
    int32_t* tri;     /* [ne][3] */
    uint8_t* ukind;   /* [ne][3] user kinds */
    double* fx;       /* [ne][3] element-frame vertex x */
    double* fy;       /* [ne][3] */
    double* area;     /* [ne] */
    int32_t* nbr;     /* [ne][3] */
    uint8_t* kind;    /* [ne][3] classified */
    double* shift;    /* [ne][3] x shift applied when crossing a periodic edge */
    int64_t* n2e_ptr; /* [nn+1] */
    int32_t* n2e;     /* elements around each node, ascending */
    double* F;        /* [nn][NF] */
    double* gU;       /* [ne][6]: dU1/dx, dU1/dy, dU2/dx, dU2/dy, dU3/dx, dU3/dy */
    uint8_t* wall;    /* [ne] element has an edge or node on a no-slip wall */
    double* wline;    /* [ne][4] point and inward unit normal of its wall line */
    orc_model m;
};

typedef struct {
    double x, y, u[3], om, psi, w;
    uint64_t pid;
    int32_t e;
    int32_t alive;
} part;

struct orc_ens {
    orc_grid* g;
    orc_init_desc d;
    part* p;
    int64_t n, cap;
    int64_t step;
    uint64_t next_pid;
    double* tm;       /* [ne] micromixing timescale, Eq. (25) at the centroid */
    int64_t* seg;     /* [ne+1] element segments in order[] */
    int64_t* order;   /* particle indices grouped by element, canonical inside */
    int have_order;
    double* stats;    /* [nn][NSTAT] */
    int have_stats;
    int64_t cnt[8];
};

/* =====================================================================================
 * Counter-based random numbers (Sec. 3.9 asks for reproducible, race-free streams).
 * Philox4x32-10 as published by Salmon, Moraes, Dror & Shaw (SC'11): ten rounds of two
 * 32x32->64 multiplications with a Weyl-sequence key schedule.
 * Key = (low word of seed, high word of seed XOR problem id);
 * counter = (low word of pid, high word of pid, step, tag << 16 | index).
 * ===================================================================================== */
void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int r = 0; r < 10; ++r) {
        uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)c0;
        uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)c2;
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t n0 = hi1 ^ c1 ^ k0, n1 = lo1, n2 = hi0 ^ c3 ^ k1, n3 = lo0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

static void draw4(uint64_t seed, int32_t problem, uint64_t pid, uint32_t step, uint32_t tag,
                  uint32_t idx, uint32_t w[4])
{
    uint32_t key[2] = { (uint32_t)seed, (uint32_t)(seed >> 32) ^ (uint32_t)problem };
    uint32_t ctr[4] = { (uint32_t)pid, (uint32_t)(pid >> 32), step, (tag << 16) | idx };
    orc_philox4x32_10(ctr, key, w);
}

/* open-interval uniform: (w + 1/2) 2^-32 */
double orc_u01(uint32_t w) { return ((double)w + 0.5) * (1.0 / 4294967296.0); }

/* Box-Muller transform: two independent standard Gaussians from two uniforms */
void orc_box_muller(uint32_t a, uint32_t b, double out[2])
{
    double u1 = orc_u01(a), u2 = orc_u01(b);
    double r = sqrt(-2.0 * log(u1));
    double th = 6.283185307179586 * u2;
    out[0] = r * cos(th);
    out[1] = r * sin(th);
}

void orc_normals(uint64_t seed, int32_t problem, uint64_t pid, uint32_t step, uint32_t tag,
                 int64_t n, double* out)
{
    for (int64_t i = 0; i < n; i += 4) {
        uint32_t w[4];
        double z[2];
        draw4(seed, problem, pid, step, tag, (uint32_t)(i / 4), w);
        orc_box_muller(w[0], w[1], z);
        out[i] = z[0];
        if (i + 1 < n) out[i + 1] = z[1];
        orc_box_muller(w[2], w[3], z);
        if (i + 2 < n) out[i + 2] = z[0];
        if (i + 3 < n) out[i + 3] = z[1];
    }
}

/* Gamma(shape, mean) by Marsaglia & Tsang (2000), shape >= 1.  Attempt a uses the
   counter index a; if every attempt is rejected the mean is returned. */
double orc_gamma(double shape, double mean, uint64_t seed, int32_t problem, uint64_t pid,
                 uint32_t step, uint32_t tag)
{
    double d = shape - 1.0 / 3.0;
    double c = 1.0 / sqrt(9.0 * d);
    for (uint32_t a = 0; a < GAMMA_ATTEMPTS; ++a) {
        uint32_t w[4];
        double z[2];
        draw4(seed, problem, pid, step, tag, a, w);
        orc_box_muller(w[0], w[1], z);
        double x = z[0];
        double u = orc_u01(w[2]);
        double v = 1.0 + c * x;
        if (v <= 0.0) continue;
        v = v * v * v;
        if (u < 1.0 - 0.0331 * (x * x) * (x * x)) return d * v * (mean / shape);
        if (log(u) < 0.5 * x * x + d * (1.0 - v + log(v))) return d * v * (mean / shape);
    }
    return mean;
}

/* =====================================================================================
 * Grid (Secs. 3.3, 3.4, 3.6, 3.8)
 * ===================================================================================== */
static void seterr(char* err, int32_t len, const char* msg)
{
    if (err && len > 0) { strncpy(err, msg, (size_t)len - 1); err[len - 1] = 0; }
}

/* area coordinates N^A, N^B, N^C (not normalised) of point P in element e:
   N^A and N^C are the signed half cross products of Eqs. (44)-(45) (no absolute value:
   the text calls them signed), N^B = A_e - N^A - N^C (Sec. 3.6). */
static void area_coords(const orc_grid* g, int32_t e, double x, double y, double N[3])
{
    const double xA = g->fx[3 * e], xB = g->fx[3 * e + 1], xC = g->fx[3 * e + 2];
    const double yA = g->fy[3 * e], yB = g->fy[3 * e + 1], yC = g->fy[3 * e + 2];
    double NA = 0.5 * ((xC - xB) * (y - yB) - (yC - yB) * (x - xB));
    double NC = 0.5 * ((x - xB) * (yA - yB) - (y - yB) * (xA - xB));
    N[0] = NA;
    N[2] = NC;
    N[1] = g->area[e] - NA - NC;
}

/* shape-function values N^A, N^B, N^C at P (Eq. 38): area coordinates / A_e */
void orc_bary(const orc_grid* g, int32_t e, double x, double y, double lam[3])
{
    double N[3];
    area_coords(g, e, x, y, N);
    lam[0] = N[0] / g->area[e];
    lam[1] = N[1] / g->area[e];
    lam[2] = N[2] / g->area[e];
}

static int inside(const double N[3]) { return N[0] >= 0.0 && N[1] >= 0.0 && N[2] >= 0.0; }

/* P1 interpolation of all nodal fields (Eq. 37) */
static void interp(const orc_grid* g, int32_t e, const double lam[3], double f[NF])
{
    const int32_t* t = g->tri + 3 * e;
    for (int q = 0; q < NF; ++q)
        f[q] = lam[0] * g->F[(int64_t)t[0] * NF + q] + lam[1] * g->F[(int64_t)t[1] * NF + q] +
               lam[2] * g->F[(int64_t)t[2] * NF + q];
}

/* gradient of a nodal scalar field over element e (Eqs. 39-40) */
static void elem_grad(const orc_grid* g, int32_t e, double qA, double qB, double qC, double* dx,
                      double* dy)
{
    const double xA = g->fx[3 * e], xB = g->fx[3 * e + 1], xC = g->fx[3 * e + 2];
    const double yA = g->fy[3 * e], yB = g->fy[3 * e + 1], yC = g->fy[3 * e + 2];
    double xBA = xB - xA, xCA = xC - xA, yBA = yB - yA, yCA = yC - yA;
    double s = 1.0 / (2.0 * g->area[e]);
    *dx = s * ((-yCA + yBA) * qA + yCA * qB + (-yBA) * qC);
    *dy = s * ((xCA - xBA) * qA + (-xCA) * qB + xBA * qC);
}

int32_t orc_locate_brute(const orc_grid* g, double x, double y, double* xs)
{
    double shifts[3] = { 0.0, -g->period, g->period };
    int ns = g->period > 0 ? 3 : 1;
    for (int32_t e = 0; e < g->ne; ++e)
        for (int s = 0; s < ns; ++s) {
            double N[3];
            area_coords(g, e, x + shifts[s], y, N);
            if (inside(N)) { if (xs) *xs = x + shifts[s]; return e; }
        }
    return -1;
}

static int finite_all(const double* a, int64_t n)
{
    for (int64_t i = 0; i < n; ++i) if (!isfinite(a[i])) return 0;
    return 1;
}

/* Fields derived from the nodal mean velocity: element gradients (Eqs. 39-40) and the
   two-pass nodal Laplacian (Sec. 3.4). */
static void derive_fields(orc_grid* g)
{
    const int64_t nn = g->nn, ne = g->ne;
    const int32_t* tri = g->tri;
    /* element gradients of <U_i> (Eqs. 39-40), constant per element */
    for (int64_t e = 0; e < ne; ++e) {
        const int32_t* t = tri + 3 * e;
        for (int i = 0; i < 3; ++i)
            elem_grad(g, (int32_t)e, g->F[(int64_t)t[0] * NF + F_MU + i], g->F[(int64_t)t[1] * NF + F_MU + i],
                      g->F[(int64_t)t[2] * NF + F_MU + i], &g->gU[6 * e + 2 * i], &g->gU[6 * e + 2 * i + 1]);
    }

    /* second derivatives by the two-pass procedure of Sec. 3.4: element gradients are
       averaged to the nodes over the surrounding elements; the gradients of those nodal
       gradients are averaged to the nodes again.  lap<U_i> = d2/dx2 + d2/dy2. */
    {
        double* gn = (double*)calloc(6 * nn, sizeof(double));
        for (int64_t n = 0; n < nn; ++n) {
            int64_t cnt = g->n2e_ptr[n + 1] - g->n2e_ptr[n];
            for (int64_t j = g->n2e_ptr[n]; j < g->n2e_ptr[n + 1]; ++j)
                for (int q = 0; q < 6; ++q) gn[6 * n + q] += g->gU[6 * (int64_t)g->n2e[j] + q];
            if (cnt > 0) for (int q = 0; q < 6; ++q) gn[6 * n + q] /= (double)cnt;
        }
        /* per element: d/dx of (dU_i/dx) and d/dy of (dU_i/dy) */
        double* h = (double*)malloc(sizeof(double) * 6 * ne);
        for (int64_t e = 0; e < ne; ++e) {
            const int32_t* t = tri + 3 * e;
            for (int i = 0; i < 3; ++i) {
                double dxx, dxy, dyx, dyy;
                elem_grad(g, (int32_t)e, gn[6 * (int64_t)t[0] + 2 * i], gn[6 * (int64_t)t[1] + 2 * i], gn[6 * (int64_t)t[2] + 2 * i], &dxx, &dxy);
                elem_grad(g, (int32_t)e, gn[6 * (int64_t)t[0] + 2 * i + 1], gn[6 * (int64_t)t[1] + 2 * i + 1], gn[6 * (int64_t)t[2] + 2 * i + 1], &dyx, &dyy);
                h[6 * e + 2 * i] = dxx;
                h[6 * e + 2 * i + 1] = dyy;
            }
        }
        for (int64_t n = 0; n < nn; ++n) {
            int64_t cnt = g->n2e_ptr[n + 1] - g->n2e_ptr[n];
            for (int i = 0; i < 3; ++i) {
                double sxx = 0, syy = 0;
                for (int64_t j = g->n2e_ptr[n]; j < g->n2e_ptr[n + 1]; ++j) {
                    sxx += h[6 * (int64_t)g->n2e[j] + 2 * i];
                    syy += h[6 * (int64_t)g->n2e[j] + 2 * i + 1];
                }
                g->F[n * NF + F_LAP + i] = cnt > 0 ? sxx / (double)cnt + syy / (double)cnt : 0.0;
            }
        }
        free(h);
        free(gn);
    }

}

orc_grid* orc_grid_create(int64_t nn, const double* xy, int64_t ne, const int32_t* tri,
                          const uint8_t* edge_kind, double period_x,
                          const double* grad_p, const double* wp, const double* mean_u,
                          const double* mean_omega, const double* rey, const orc_model* m,
                          char* err, int32_t errlen)
{
    if (nn < 3 || ne < 1 || !xy || !tri || !edge_kind || !m) { seterr(err, errlen, "bad args"); return NULL; }
    orc_grid* g = (orc_grid*)calloc(1, sizeof(orc_grid));
    g->nn = nn; g->ne = ne; g->period = period_x; g->m = *m;
    g->xy = (double*)malloc(sizeof(double) * 2 * nn);
    memcpy(g->xy, xy, sizeof(double) * 2 * nn);
    g->tri = (int32_t*)malloc(sizeof(int32_t) * 3 * ne);
    memcpy(g->tri, tri, sizeof(int32_t) * 3 * ne);
    g->ukind = (uint8_t*)malloc(3 * ne);
    memcpy(g->ukind, edge_kind, 3 * ne);
    g->fx = (double*)malloc(sizeof(double) * 3 * ne);
    g->fy = (double*)malloc(sizeof(double) * 3 * ne);
    g->area = (double*)malloc(sizeof(double) * ne);
    g->nbr = (int32_t*)malloc(sizeof(int32_t) * 3 * ne);
    g->kind = (uint8_t*)malloc(3 * ne);
    g->shift = (double*)calloc(3 * ne, sizeof(double));
    g->n2e_ptr = (int64_t*)calloc(nn + 1, sizeof(int64_t));
    g->F = (double*)malloc(sizeof(double) * NF * nn);
    g->gU = (double*)malloc(sizeof(double) * 6 * ne);
    g->wall = (uint8_t*)calloc(ne, 1);
    g->wline = (double*)calloc(4 * ne, sizeof(double));

    for (int64_t i = 0; i < 3 * ne; ++i)
        if (tri[i] < 0 || tri[i] >= nn) { seterr(err, errlen, "node index out of range"); orc_grid_destroy(g); return NULL; }
    if (!finite_all(xy, 2 * nn)) { seterr(err, errlen, "non-finite node coordinate"); orc_grid_destroy(g); return NULL; }

    /* element frames: vertices of an element that straddles the periodic seam are
       unwrapped by +period so that every element is a proper triangle */
    for (int64_t e = 0; e < ne; ++e) {
        double vx[3], vy[3];
        for (int k = 0; k < 3; ++k) { vx[k] = xy[2 * (int64_t)tri[3 * e + k]]; vy[k] = xy[2 * (int64_t)tri[3 * e + k] + 1]; }
        if (period_x > 0) {
            double lo = fmin(vx[0], fmin(vx[1], vx[2])), hi = fmax(vx[0], fmax(vx[1], vx[2]));
            if (hi - lo > 0.5 * period_x)
                for (int k = 0; k < 3; ++k) if (vx[k] < 0.5 * period_x) vx[k] += period_x;
        }
        for (int k = 0; k < 3; ++k) { g->fx[3 * e + k] = vx[k]; g->fy[3 * e + k] = vy[k]; }
        g->area[e] = 0.5 * ((vx[1] - vx[0]) * (vy[2] - vy[0]) - (vy[1] - vy[0]) * (vx[2] - vx[0]));
        if (!(g->area[e] > 0.0)) { seterr(err, errlen, "element not counter-clockwise"); orc_grid_destroy(g); return NULL; }
    }

    /* elements surrounding points (Sec. 3.3 linked lists), ascending element id */
    for (int64_t i = 0; i < 3 * ne; ++i) g->n2e_ptr[tri[i] + 1]++;
    for (int64_t n = 0; n < nn; ++n) g->n2e_ptr[n + 1] += g->n2e_ptr[n];
    g->n2e = (int32_t*)malloc(sizeof(int32_t) * 3 * ne);
    {
        int64_t* fill = (int64_t*)calloc(nn, sizeof(int64_t));
        for (int64_t e = 0; e < ne; ++e)
            for (int k = 0; k < 3; ++k) {
                int32_t n = tri[3 * e + k];
                g->n2e[g->n2e_ptr[n] + fill[n]++] = (int32_t)e;
            }
        free(fill);
    }

    /* element neighbours across each edge (edge k is opposite vertex k) and edge kinds */
    for (int64_t e = 0; e < ne; ++e)
        for (int k = 0; k < 3; ++k) {
            int32_t a = tri[3 * e + (k + 1) % 3], b = tri[3 * e + (k + 2) % 3];
            int32_t other = -1, count = 0;
            for (int64_t j = g->n2e_ptr[a]; j < g->n2e_ptr[a + 1]; ++j) {
                int32_t f = g->n2e[j];
                if (f == e) continue;
                const int32_t* t = tri + 3 * (int64_t)f;
                if (t[0] == b || t[1] == b || t[2] == b) { other = f; ++count; }
            }
            if (count > 1) { seterr(err, errlen, "edge shared by more than two elements"); orc_grid_destroy(g); return NULL; }
            g->nbr[3 * e + k] = other;
            if (other < 0) {
                uint8_t uk = edge_kind[3 * e + k];
                if (uk != K_WALL && uk != K_SLIP) { seterr(err, errlen, "boundary edge must be wall or slip"); orc_grid_destroy(g); return NULL; }
                g->kind[3 * e + k] = uk;
            } else {
                /* a shared edge whose two sides sit in frames a period apart is periodic */
                double xa_e = 0, xa_f = 0;
                for (int q = 0; q < 3; ++q) {
                    if (tri[3 * e + q] == a) xa_e = g->fx[3 * e + q];
                    if (tri[3 * (int64_t)other + q] == a) xa_f = g->fx[3 * (int64_t)other + q];
                }
                if (period_x > 0 && fabs(xa_f - xa_e) > 0.5 * period_x) {
                    g->kind[3 * e + k] = K_PERIODIC;
                    g->shift[3 * e + k] = (xa_f > xa_e) ? period_x : -period_x;
                } else {
                    g->kind[3 * e + k] = K_INTERIOR;
                }
            }
        }

    /* nodal fields */
    for (int64_t n = 0; n < nn; ++n) {
        double* f = g->F + n * NF;
        f[F_GP] = grad_p[2 * n]; f[F_GP + 1] = grad_p[2 * n + 1];
        for (int q = 0; q < 6; ++q) f[F_WP + q] = wp[6 * n + q];
        for (int q = 0; q < 3; ++q) f[F_WPT + q] = wp[6 * n + 3 + q];     /* symmetric input */
        for (int q = 0; q < 3; ++q) f[F_MU + q] = mean_u[3 * n + q];
        f[F_OM] = mean_omega[n];
        for (int q = 0; q < 6; ++q) f[F_RE + q] = rey[6 * n + q];
        f[F_LAP] = f[F_LAP + 1] = f[F_LAP + 2] = 0.0;
        if (!finite_all(f, NF)) { seterr(err, errlen, "non-finite nodal field"); orc_grid_destroy(g); return NULL; }
        if (!(f[F_OM] > 0.0)) { seterr(err, errlen, "mean frequency must be positive"); orc_grid_destroy(g); return NULL; }
        if (!(f[F_RE] + f[F_RE + 1] + f[F_RE + 2] > 0.0)) { seterr(err, errlen, "kinetic energy must be positive"); orc_grid_destroy(g); return NULL; }
    }

    derive_fields(g);

    /* wall elements (Sec. 3.8: elements with an edge or a node on a no-slip wall) and
       the line of the wall edge, among the wall edges touching the element's nodes,
       whose midpoint is nearest to the element centroid (ties: lowest owner*3+edge) */
    {
        uint8_t* wnode = (uint8_t*)calloc(nn, 1);
        for (int64_t e = 0; e < ne; ++e)
            for (int k = 0; k < 3; ++k)
                if (g->kind[3 * e + k] == K_WALL) {
                    wnode[tri[3 * e + (k + 1) % 3]] = 1;
                    wnode[tri[3 * e + (k + 2) % 3]] = 1;
                }
        for (int64_t e = 0; e < ne; ++e) {
            const int32_t* t = tri + 3 * e;
            if (!(wnode[t[0]] || wnode[t[1]] || wnode[t[2]])) continue;
            g->wall[e] = 1;
            double cx = (g->fx[3 * e] + g->fx[3 * e + 1] + g->fx[3 * e + 2]) / 3.0;
            double cy = (g->fy[3 * e] + g->fy[3 * e + 1] + g->fy[3 * e + 2]) / 3.0;
            double best = INFINITY;
            int64_t bestkey = -1;
            for (int v = 0; v < 3; ++v) {
                int32_t node = t[v];
                if (!wnode[node]) continue;
                for (int64_t j = g->n2e_ptr[node]; j < g->n2e_ptr[node + 1]; ++j) {
                    int32_t f = g->n2e[j];
                    /* x offset from f's frame to e's frame through the shared node */
                    double off = 0.0;
                    for (int q = 0; q < 3; ++q)
                        if (tri[3 * (int64_t)f + q] == node) off = g->fx[3 * e + v] - g->fx[3 * (int64_t)f + q];
                    for (int k = 0; k < 3; ++k) {
                        if (g->kind[3 * (int64_t)f + k] != K_WALL) continue;
                        int pa = (k + 1) % 3, pb = (k + 2) % 3;
                        double ax = g->fx[3 * (int64_t)f + pa] + off, ay = g->fy[3 * (int64_t)f + pa];
                        double bx = g->fx[3 * (int64_t)f + pb] + off, by = g->fy[3 * (int64_t)f + pb];
                        double mx = 0.5 * (ax + bx) - cx, my = 0.5 * (ay + by) - cy;
                        double d2 = mx * mx + my * my;
                        int64_t key = 3 * (int64_t)f + k;
                        if (d2 < best || (d2 == best && key < bestkey)) {
                            double ex = bx - ax, ey = by - ay, len = sqrt(ex * ex + ey * ey);
                            best = d2; bestkey = key;
                            g->wline[4 * e] = ax; g->wline[4 * e + 1] = ay;
                            g->wline[4 * e + 2] = -ey / len; g->wline[4 * e + 3] = ex / len;
                        }
                    }
                }
            }
        }
        free(wnode);
    }
    return g;
}

void orc_grid_destroy(orc_grid* g)
{
    if (!g) return;
    free(g->xy); free(g->tri); free(g->ukind); free(g->fx); free(g->fy); free(g->area);
    free(g->nbr); free(g->kind); free(g->shift); free(g->n2e_ptr); free(g->n2e); free(g->F);
    free(g->gU); free(g->wall); free(g->wline);
    free(g);
}

void orc_grid_export(const orc_grid* g, double* frame, double* area, int32_t* nbr, uint8_t* kind,
                     double* gradu, double* lapu, uint8_t* wall, double* wline)
{
    for (int64_t e = 0; e < g->ne; ++e) {
        for (int k = 0; k < 3; ++k) {
            if (frame) { frame[6 * e + 2 * k] = g->fx[3 * e + k]; frame[6 * e + 2 * k + 1] = g->fy[3 * e + k]; }
            if (nbr) nbr[3 * e + k] = g->nbr[3 * e + k];
            if (kind) kind[3 * e + k] = g->kind[3 * e + k];
        }
        if (area) area[e] = g->area[e];
        if (gradu) for (int q = 0; q < 6; ++q) gradu[6 * e + q] = g->gU[6 * e + q];
        if (wall) wall[e] = g->wall[e];
        if (wline) for (int q = 0; q < 4; ++q) wline[4 * e + q] = g->wline[4 * e + q];
    }
    if (lapu) for (int64_t n = 0; n < g->nn; ++n) for (int i = 0; i < 3; ++i) lapu[3 * n + i] = g->F[n * NF + F_LAP + i];
}

/* =====================================================================================
 * Particle tracking (Sec. 3.6) and particle wall conditions (Sec. 3.8)
 * ===================================================================================== */

/* concave-boundary fall-back (Sec. 3.6, Fig. 2): search the elements surrounding the
   nodes of element c (nodes in vertex order, elements ascending).  Returns the first
   element that contains P, with the x shift that moves P into that element's frame. */
static int fallback(const orc_grid* g, int32_t c, double x, double y, int32_t* found, double* sh)
{
    for (int v = 0; v < 3; ++v) {
        int32_t node = g->tri[3 * (int64_t)c + v];
        for (int64_t j = g->n2e_ptr[node]; j < g->n2e_ptr[node + 1]; ++j) {
            int32_t f = g->n2e[j];
            if (f == c) continue;
            double off = 0.0;
            for (int q = 0; q < 3; ++q)
                if (g->tri[3 * (int64_t)f + q] == node) off = g->fx[3 * (int64_t)f + q] - g->fx[3 * (int64_t)c + v];
            double N[3];
            area_coords(g, f, x + off, y, N);
            if (inside(N)) { *found = f; *sh = off; return 1; }
        }
    }
    return 0;
}

typedef struct {
    int32_t wall_a;     /* crossed a no-slip wall: trajectory (a), Eq. (54) */
    int64_t steps, refl, fb;
} walk_info;

/* next-best-element walk: while P is outside the current element, step across the
   edge opposite the smallest area coordinate (ties: A, B, C order).  Periodic edges
   shift P by the period; a boundary edge first triggers the fall-back search and,
   when that finds nothing, a perfect reflection across the edge line.  No-slip walls
   mark the particle for U = 0 (Eq. 56) and a new frequency; free-slip walls reverse
   the normal velocity.  At most 4 reflections and 64 moves. */
static int walk(const orc_grid* g, int32_t* pe, double* px, double* py, double* shift_acc,
                double u[3], walk_info* wi)
{
    int32_t c = *pe;
    double x = *px, y = *py;
    int refl = 0;
    for (int it = 0; it < MAX_WALK; ++it) {
        double N[3];
        area_coords(g, c, x, y, N);
        if (inside(N)) { *pe = c; *px = x; *py = y; return 0; }
        int k = 0;
        if (N[1] < N[k]) k = 1;
        if (N[2] < N[k]) k = 2;
        uint8_t kd = g->kind[3 * (int64_t)c + k];
        if (kd == K_INTERIOR) { c = g->nbr[3 * (int64_t)c + k]; wi->steps++; continue; }
        if (kd == K_PERIODIC) {
            double s = g->shift[3 * (int64_t)c + k];
            x += s; *shift_acc += s;
            c = g->nbr[3 * (int64_t)c + k];
            wi->steps++;
            continue;
        }
        int32_t f;
        double s;
        if (fallback(g, c, x, y, &f, &s)) { c = f; x += s; *shift_acc += s; wi->fb++; continue; }
        if (refl == MAX_REFL) break;
        /* mirror across the line of edge k (from vertex k+1 to vertex k+2, interior on
           its left) */
        int pa = (k + 1) % 3, pb = (k + 2) % 3;
        double ax = g->fx[3 * (int64_t)c + pa], ay = g->fy[3 * (int64_t)c + pa];
        double ex = g->fx[3 * (int64_t)c + pb] - ax, ey = g->fy[3 * (int64_t)c + pb] - ay;
        double len = sqrt(ex * ex + ey * ey);
        double nx = -ey / len, ny = ex / len;
        double d = (x - ax) * nx + (y - ay) * ny;
        x = x - 2.0 * d * nx;
        y = y - 2.0 * d * ny;
        if (kd == K_WALL) {
            wi->wall_a = 1;
        } else {
            double un = u[0] * nx + u[1] * ny;
            u[0] = u[0] - 2.0 * un * nx;
            u[1] = u[1] - 2.0 * un * ny;
        }
        ++refl;
        wi->refl++;
    }
    *pe = c; *px = x; *py = y;
    return ORC_E_LOST;
}

/* =====================================================================================
 * Particle loop (Table 2, right column): Eqs. (7), (10)/(27), (11), (18), (19), (20)
 * ===================================================================================== */
typedef struct { int64_t c[8]; } counters;

/* Weights of the three nodal values that give a field at (x, y) in element e: the area
   coordinates (P1 interpolation, Eq. 37), or 1/3 each when the statistics are used as
   element averages of the nodal values (Sec. 3.3, second estimator). */
static void field_weights(const orc_ens* E, int32_t e, double x, double y, double lam[3])
{
    if (E->d.estimator == 1) {
        lam[0] = lam[1] = lam[2] = 1.0 / 3.0;
        return;
    }
    orc_bary(E->g, e, x, y, lam);
}

static int advance_one(const orc_ens* E, part* p, double dt, counters* cn)
{
    const orc_grid* g = E->g;
    const orc_model* m = &g->m;
    double lam[3], f[NF];
    field_weights(E, p->e, p->x, p->y, lam);
    interp(g, p->e, lam, f);
    const double* gu = g->gU + 6 * (int64_t)p->e;
    const double R11 = f[F_RE], R22 = f[F_RE + 1], R33 = f[F_RE + 2];
    const double R12 = f[F_RE + 3], R13 = f[F_RE + 4], R23 = f[F_RE + 5];
    const double W11 = f[F_WP], W22 = f[F_WP + 1], W33 = f[F_WP + 2];
    const double W12 = f[F_WP + 3], W13 = f[F_WP + 4], W23 = f[F_WP + 5];
    const double W21 = f[F_WPT], W31 = f[F_WPT + 1], W32 = f[F_WPT + 2];

    double k = 0.5 * (R11 + R22 + R33);                       /* k = <u_i u_i>/2 */
    double Om = f[F_OM];
    double eps = Om * (k + m->nu * m->CT * m->CT * Om);          /* Eq. (18) */
    double wpR = W11 * R11 + W22 * R22 + W33 * R33 + ((W12 + W21) * R12 + (W13 + W31) * R13 + (W23 + W32) * R23);
    double c0eps = -2.0 * wpR / (3.0 * k);                     /* C0*eps from Eq. (11) */
    if (c0eps < 0.0) { c0eps = 0.0; cn->c[5]++; }
    /* production P = -<u_i u_j> d<U_i>/dx_j, j over the two resolved directions */
    double prod = -(R11 * gu[0] + R12 * gu[1] + R12 * gu[2] + R22 * gu[3] + R13 * gu[4] + R23 * gu[5]);
    double Sw = m->Cw2 - m->Cw1 * prod / eps;                  /* Eq. (20) */
    double G[3][3] = { { (W11 - 0.5 * eps) / k, W12 / k, W13 / k },
                       { W21 / k, (W22 - 0.5 * eps) / k, W23 / k },
                       { W31 / k, W32 / k, (W33 - 0.5 * eps) / k } };   /* Eq. (11) */

    /* 6 Gaussians and one uniform per particle and step (Sec. 3.9) */
    uint32_t w[8];
    draw4(E->d.seed, E->d.problem, p->pid, (uint32_t)E->step, TAG_STEP, 0, w);
    draw4(E->d.seed, E->d.problem, p->pid, (uint32_t)E->step, TAG_STEP, 1, w + 4);
    double z01[2], z23[2], z45[2];
    orc_box_muller(w[0], w[1], z01);
    orc_box_muller(w[2], w[3], z23);
    orc_box_muller(w[4], w[5], z45);
    double sdt = sqrt(dt);
    double dW[2] = { sdt * z01[0], sdt * z01[1] };               /* shared by Eqs. (7), (10) */
    double dWp[3] = { sdt * z23[0], sdt * z23[1], sdt * z45[0] };
    double dWo = sdt * z45[1];
    double eta = orc_u01(w[6]);
    double s2nu = sqrt(2.0 * m->nu);

    /* velocity prediction, Eq. (27) */
    double du[3] = { p->u[0] - f[F_MU], p->u[1] - f[F_MU + 1], p->u[2] - f[F_MU + 2] };
    double gp[3] = { f[F_GP], f[F_GP + 1], 0.0 };
    double un[3];
    for (int i = 0; i < 3; ++i) {
        double drift = -gp[i] / m->rho + 2.0 * m->nu * f[F_LAP + i] + G[i][0] * du[0] + G[i][1] * du[1] + G[i][2] * du[2];
        un[i] = p->u[i] + drift * dt + s2nu * (gu[2 * i] * dW[0] + gu[2 * i + 1] * dW[1]) + sqrt(c0eps) * dWp[i];
    }
    /* turbulent frequency, Eq. (19); the diffusion uses |omega| and a negative result
       is reflected (omega stays non-negative) */
    double om = p->om;
    double omn = om - m->C3 * Om * (om - Om) * dt - Sw * Om * om * dt +
                 sqrt(2.0 * m->C3 * m->C4 * Om * Om * fabs(om)) * dWo;
    if (omn < 0.0) { omn = -omn; cn->c[4]++; }
    /* position, Eq. (7), with the velocity at the start of the step */
    double x0 = p->x, y0 = p->y;
    double xn = x0 + p->u[0] * dt + s2nu * dW[0];
    double yn = y0 + p->u[1] * dt + s2nu * dW[1];

    int32_t e = p->e;
    double shift = 0.0;
    walk_info wi = { 0, 0, 0, 0 };
    int rc = walk(g, &e, &xn, &yn, &shift, un, &wi);
    cn->c[2] += wi.refl;
    cn->c[3] += wi.fb;
    cn->c[6] += wi.steps;
    if (rc != 0) return rc;

    /* no-slip wall conditions (Sec. 3.8): trajectory (a) crossed the wall; trajectory
       (b) is tested with probability f_w of Eq. (53) in wall elements only.  Both set
       U = 0 (Eq. 56) and draw omega from a Gamma law with variance C4 <omega>^2
       (Eq. 58) around the nodal <omega> at the particle. */
    int hit = 0;
    if (wi.wall_a) { hit = 1; cn->c[0]++; }
    else if (g->wall[e] && m->nu * dt > 0.0) {
        const double* L = g->wline + 4 * (int64_t)e;
        double dn = (x0 + shift - L[0]) * L[2] + (y0 - L[1]) * L[3];
        double dn1 = (xn - L[0]) * L[2] + (yn - L[1]) * L[3];
        if (dn < 0.0) dn = 0.0;
        if (dn1 < 0.0) dn1 = 0.0;
        double fw = exp(-dn * dn1 / (m->nu * dt));
        if (eta < fw) { hit = 1; cn->c[1]++; }
    }
    if (hit) {
        double lam2[3], f2[NF];
        field_weights(E, e, xn, yn, lam2);
        interp(g, e, lam2, f2);
        un[0] = un[1] = un[2] = 0.0;
        omn = orc_gamma(1.0 / m->C4, f2[F_OM], E->d.seed, E->d.problem, p->pid, (uint32_t)E->step, TAG_WALL_GAMMA);
    }
    p->x = xn; p->y = yn; p->e = e;
    p->u[0] = un[0]; p->u[1] = un[1]; p->u[2] = un[2];
    p->om = omn;
    /* concentrated source (Sec. 4.1.2): particles inside the source disk get psi = 1 */
    if (E->d.src_continuous) {
        double dx = xn - E->d.src_x, dy = yn - E->d.src_y;
        if (g->period > 0) { if (dx > 0.5 * g->period) dx -= g->period; else if (dx < -0.5 * g->period) dx += g->period; }
        if (dx * dx + dy * dy < E->d.src_r * E->d.src_r) { p->psi = 1.0; cn->c[7]++; }
    }
    if (!(isfinite(p->x) && isfinite(p->y) && isfinite(p->u[0]) && isfinite(p->u[1]) && isfinite(p->u[2]) && isfinite(p->om)))
        return ORC_E_NONFINITE;
    return 0;
}

/* =====================================================================================
 * Velocity-conditioned scalar mean (Sec. 3.5, App. A) and IECM mixing (Eqs. 24-25)
 * ===================================================================================== */

/* number of groups at each level of the sort-and-divide procedure: a level divides
   every group into at most bins[l] parts while keeping at least min_per_bin particles
   per part, i.e. min(bins[l], max(1, floor(n / (m * groups so far)))).  Once a level is
   reduced the following levels have one group (the procedure stops, Sec. 3.5). */
static int32_t bin_structure(int32_t n, const int32_t bins[3], int32_t m, int32_t g[3])
{
    int64_t P = 1;
    int stopped = 0;
    for (int l = 0; l < 3; ++l) {
        int64_t q = (int64_t)n / ((int64_t)m * P);
        if (q < 1) q = 1;
        int64_t gl = bins[l] < q ? bins[l] : q;
        if (stopped) gl = 1;
        if (gl < bins[l]) stopped = 1;
        g[l] = (int32_t)gl;
        P *= gl;
    }
    return (int32_t)P;
}

/* insertion sort of idx[0..n) by (key[idx], pid[idx]) ascending */
static void sort_by(int64_t* idx, int32_t n, const part* P, int comp)
{
    for (int32_t i = 1; i < n; ++i) {
        int64_t t = idx[i];
        double kt = P[t].u[comp];
        uint64_t pt = P[t].pid;
        int32_t j = i - 1;
        while (j >= 0) {
            double kj = P[idx[j]].u[comp];
            uint64_t pj = P[idx[j]].pid;
            if (kj > kt || (kj == kt && pj > pt)) { idx[j + 1] = idx[j]; --j; }
            else break;
        }
        idx[j + 1] = t;
    }
}

/* canonical order of one element's particles (Sec. 3.5): sort by U1, divide into
   groups of equal count, sort each group by U2, divide again, sort by U3.  Group t of
   a level with C_l cumulative groups holds the positions n with floor(C_l n / N) = t,
   so the final bin of position n is floor(C' n / N) (App. A). Ties on a velocity
   component are broken by particle id. Returns C'. */
static int32_t canonical_order(int64_t* idx, int32_t n, const part* P, const int32_t bins[3], int32_t m)
{
    int32_t g[3];
    int32_t Cp = bin_structure(n, bins, m, g);
    if (n == 0) return Cp;
    sort_by(idx, n, P, 0);
    int64_t C = g[0];
    for (int l = 1; l < 3; ++l) {
        for (int64_t t = 0; t < C; ++t) {
            int64_t lo = (t * n + C - 1) / C, hi = ((t + 1) * n + C - 1) / C;   /* ceil */
            sort_by(idx + lo, (int32_t)(hi - lo), P, l);
        }
        C *= g[l];
    }
    return Cp;
}

/* Fox's projection conditioning (Eqs. 64-66).  Over the particles of one element, with
   weights w: means, then the central second moments <u_a u_b>, <u_a phi'>, <phi'^2>;
   rho_a and rho_ab of Eq. (66); the projection vector alpha solves rho_ab alpha_b = rho_a
   (Eq. 65); the projected velocity (Eq. 64) is taken of the normalised fluctuations,
   U_rho = sum_a alpha_a (U_a - <U_a>) / <u_a^2>^(1/2), the combination for which a joint
   Gaussian PDF makes <phi'|U> a function of U_rho alone.  Degenerate samples: a component
   without variance (standard deviation at most 1e-12 times its largest magnitude in the
   element, i.e. a spread made of rounding), and a component that is a linear combination
   of the earlier ones (taken in the order U1, U2, U3; remaining diagonal of the Cholesky
   factor of rho below 1e-12), get alpha = 0; without scalar variance (the same test on
   psi) alpha = 0 and every key is 0.
   The particles are then sorted by (U_rho, pid) and divided into
   min(nc, max(1, floor(n / min_per_bin))) equal-count intervals. */
static void projection_keys(int32_t n, const int64_t* idx, const part* P, double* key, double alpha[3])
{
    double W = 0.0, mu[3] = { 0, 0, 0 }, mp = 0.0, umax[3] = { 0, 0, 0 }, pmax = 0.0;
    for (int32_t r = 0; r < n; ++r) {
        const part* q = &P[idx[r]];
        W += q->w;
        for (int a = 0; a < 3; ++a) {
            mu[a] += q->w * q->u[a];
            umax[a] = fmax(umax[a], fabs(q->u[a]));
        }
        mp += q->w * q->psi;
        pmax = fmax(pmax, fabs(q->psi));
    }
    for (int a = 0; a < 3; ++a) mu[a] /= W;
    mp /= W;
    double Cuu[3][3] = { { 0 } }, Cup[3] = { 0, 0, 0 }, Cpp = 0.0;
    for (int32_t r = 0; r < n; ++r) {
        const part* q = &P[idx[r]];
        double d[3] = { q->u[0] - mu[0], q->u[1] - mu[1], q->u[2] - mu[2] };
        double dp = q->psi - mp;
        for (int a = 0; a < 3; ++a) {
            for (int b = 0; b < 3; ++b) Cuu[a][b] += q->w * d[a] * d[b];
            Cup[a] += q->w * d[a] * dp;
        }
        Cpp += q->w * dp * dp;
    }
    for (int a = 0; a < 3; ++a) {
        for (int b = 0; b < 3; ++b) Cuu[a][b] /= W;
        Cup[a] /= W;
    }
    Cpp /= W;
    double sd[3];
    for (int a = 0; a < 3; ++a) {
        sd[a] = sqrt(Cuu[a][a]);
        if (!(sd[a] > 1e-12 * umax[a])) sd[a] = 0.0;
        alpha[a] = 0.0;
    }
    if (sqrt(Cpp) > 1e-12 * pmax) {
        /* Eq. (66) */
        double rho[3][3], rv[3];
        for (int a = 0; a < 3; ++a) {
            rv[a] = sd[a] > 0.0 ? Cup[a] / (sd[a] * sqrt(Cpp)) : 0.0;
            for (int b = 0; b < 3; ++b) rho[a][b] = (sd[a] > 0.0 && sd[b] > 0.0) ? Cuu[a][b] / (sd[a] * sd[b]) : 0.0;
        }
        /* Eq. (65) on the independent components: Cholesky factor L of rho restricted to
           them, then forward and back substitution */
        int sel[3], k = 0;
        double L[3][3] = { { 0 } };
        for (int a = 0; a < 3; ++a) {
            if (!(sd[a] > 0.0)) continue;
            double l[3], dd = rho[a][a];
            for (int i = 0; i < k; ++i) {
                double s = rho[a][sel[i]];
                for (int j = 0; j < i; ++j) s -= L[i][j] * l[j];
                l[i] = s / L[i][i];
                dd -= l[i] * l[i];
            }
            if (!(dd > 1e-12)) continue;
            for (int i = 0; i < k; ++i) L[k][i] = l[i];
            L[k][k] = sqrt(dd);
            sel[k++] = a;
        }
        double z[3];
        for (int i = 0; i < k; ++i) {
            double s = rv[sel[i]];
            for (int j = 0; j < i; ++j) s -= L[i][j] * z[j];
            z[i] = s / L[i][i];
        }
        for (int i = k - 1; i >= 0; --i) {
            double s = z[i];
            for (int j = i + 1; j < k; ++j) s -= L[j][i] * alpha[sel[j]];
            alpha[sel[i]] = s / L[i][i];
        }
    }
    /* Eq. (64) on the normalised fluctuations */
    for (int32_t r = 0; r < n; ++r) {
        const part* q = &P[idx[r]];
        double v = 0.0;
        for (int a = 0; a < 3; ++a)
            if (alpha[a] != 0.0) v += alpha[a] * ((q->u[a] - mu[a]) / sd[a]);
        key[r] = v;
    }
}

/* sorts idx[0..n) by (U_rho, pid); returns the number of intervals */
static int32_t projection_order(int64_t* idx, int32_t n, const part* P, int32_t nc, int32_t m, double alpha[3])
{
    if (n == 0) return 1;
    double* key = (double*)malloc(sizeof(double) * n);
    projection_keys(n, idx, P, key, alpha);
    for (int32_t i = 1; i < n; ++i) {   /* insertion sort of (key, idx) pairs */
        int64_t t = idx[i];
        double kt = key[i];
        int32_t j = i - 1;
        while (j >= 0 && (key[j] > kt || (key[j] == kt && P[idx[j]].pid > P[t].pid))) {
            idx[j + 1] = idx[j];
            key[j + 1] = key[j];
            --j;
        }
        idx[j + 1] = t;
        key[j + 1] = kt;
    }
    free(key);
    int64_t q = n / m;
    if (q < 1) q = 1;
    return (int32_t)(nc < q ? nc : q);
}

int32_t orc_project_element(int32_t n, const double* u, const double* psi, const double* w, const uint64_t* pid,
                            int32_t nc, int32_t min_per_bin, double* key, int32_t* pos, int32_t* bin,
                            double alpha[3])
{
    part* P = (part*)calloc(n > 0 ? n : 1, sizeof(part));
    int64_t* idx = (int64_t*)malloc(sizeof(int64_t) * (n > 0 ? n : 1));
    for (int32_t i = 0; i < n; ++i) {
        P[i].u[0] = u[3 * i]; P[i].u[1] = u[3 * i + 1]; P[i].u[2] = u[3 * i + 2];
        P[i].psi = psi[i]; P[i].w = w[i]; P[i].pid = pid[i]; idx[i] = i;
    }
    projection_keys(n, idx, P, key, alpha);
    int32_t Cp = projection_order(idx, n, P, nc, min_per_bin, alpha);
    for (int32_t r = 0; r < n; ++r) {
        pos[idx[r]] = r;
        bin[idx[r]] = (int32_t)(((int64_t)Cp * r) / n);
    }
    free(P); free(idx);
    return Cp;
}

int32_t orc_bin_element(int32_t n, const double* u, const uint64_t* pid, const int32_t bins[3],
                        int32_t min_per_bin, int32_t* pos, int32_t* bin)
{
    part* P = (part*)calloc(n > 0 ? n : 1, sizeof(part));
    int64_t* idx = (int64_t*)malloc(sizeof(int64_t) * (n > 0 ? n : 1));
    for (int32_t i = 0; i < n; ++i) {
        P[i].u[0] = u[3 * i]; P[i].u[1] = u[3 * i + 1]; P[i].u[2] = u[3 * i + 2];
        P[i].pid = pid[i]; idx[i] = i;
    }
    int32_t Cp = canonical_order(idx, n, P, bins, min_per_bin);
    for (int32_t r = 0; r < n; ++r) {
        pos[idx[r]] = r;
        bin[idx[r]] = (int32_t)(((int64_t)Cp * r) / n);
    }
    free(P); free(idx);
    return Cp;
}

/* micromixing timescale, Eq. (25), at the element centroid */
static double tm_element(const orc_grid* g, const orc_init_desc* d, int64_t e)
{
    const orc_model* m = &g->m;
    double f[NF];
    const int32_t* t = g->tri + 3 * e;
    for (int q = 0; q < NF; ++q)
        f[q] = (g->F[(int64_t)t[0] * NF + q] + g->F[(int64_t)t[1] * NF + q] + g->F[(int64_t)t[2] * NF + q]) / 3.0;
    double k = 0.5 * (f[F_RE] + f[F_RE + 1] + f[F_RE + 2]);
    double Om = f[F_OM];
    double eps = Om * (k + m->nu * m->CT * m->CT * Om);
    double Uc = sqrt(f[F_MU] * f[F_MU] + f[F_MU + 1] * f[F_MU + 1] + f[F_MU + 2] * f[F_MU + 2]);
    double cx = (g->fx[3 * e] + g->fx[3 * e + 1] + g->fx[3 * e + 2]) / 3.0;
    double cy = (g->fy[3 * e] + g->fy[3 * e + 1] + g->fy[3 * e + 2]) / 3.0;
    double dx = cx - d->src_x, dy = cy - d->src_y;
    if (g->period > 0) { if (dx > 0.5 * g->period) dx -= g->period; else if (dx < -0.5 * g->period) dx += g->period; }
    double dist = sqrt(dx * dx + dy * dy);
    double first = Uc > 0.0 ? m->Cs * cbrt(d->src_r * d->src_r / eps) + m->Ct * dist / Uc : INFINITY;
    double second = fmax(k / eps, m->CT * sqrt(m->nu / eps));
    return fmin(first, second);
}

double orc_tm(const orc_ens* E, int32_t e) { return E->tm[e]; }

/* group live particles by host element (stable), then canonical order per element;
   with mix != 0 apply IECM: psi <- psi - f (psi - <phi|V>_bin), f = min(dt/t_m, 1),
   <phi|V>_bin = sum(w psi)/sum(w) over the bin (App. A, with particle weights) */
static void element_pass(orc_ens* E, double dt, int mix)
{
    const orc_grid* g = E->g;
    int64_t ne = g->ne;
    free(E->seg); free(E->order);
    E->seg = (int64_t*)calloc(ne + 1, sizeof(int64_t));
    int64_t nl = 0;
    for (int64_t i = 0; i < E->n; ++i) if (E->p[i].alive) { E->seg[E->p[i].e + 1]++; ++nl; }
    for (int64_t e = 0; e < ne; ++e) E->seg[e + 1] += E->seg[e];
    E->order = (int64_t*)malloc(sizeof(int64_t) * (nl > 0 ? nl : 1));
    {
        int64_t* fill = (int64_t*)calloc(ne, sizeof(int64_t));
        for (int64_t i = 0; i < E->n; ++i)
            if (E->p[i].alive) { int32_t e = E->p[i].e; E->order[E->seg[e] + fill[e]++] = i; }
        free(fill);
    }
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t e = 0; e < ne; ++e) {
        int32_t n = (int32_t)(E->seg[e + 1] - E->seg[e]);
        if (n == 0) continue;
        int64_t* idx = E->order + E->seg[e];
        double alpha[3];
        int32_t Cp = E->d.conditioning == 1 ? projection_order(idx, n, E->p, E->d.bins[0], E->d.min_per_bin, alpha)
                                            : canonical_order(idx, n, E->p, E->d.bins, E->d.min_per_bin);
        if (!mix) continue;
        double fmix = dt / E->tm[e];
        if (fmix > 1.0) fmix = 1.0;
        int32_t r = 0;
        for (int32_t b = 0; b < Cp; ++b) {
            int32_t lo = r;
            double sw = 0.0, swp = 0.0;
            while (r < n && ((int64_t)Cp * r) / n == b) { sw += E->p[idx[r]].w; swp += E->p[idx[r]].w * E->p[idx[r]].psi; ++r; }
            if (r == lo) continue;
            double mean = swp / sw;
            for (int32_t q = lo; q < r; ++q) {
                part* P = &E->p[idx[q]];
                P->psi = P->psi - fmix * (P->psi - mean);
            }
        }
    }
    E->have_order = 1;
}

/* =====================================================================================
 * Eulerian statistics at the nodes (Sec. 3.3): weighted by the P1 shape function of the
 * node (Eq. 37) over the particles of the elements around the node; second moments
 * about the node's own mean with the same weights (Eq. 36).
 * ===================================================================================== */
/* Second estimator of Sec. 3.3 (Eqs. 35-36): means and central second moments of the
   particles of every element (first pass), then at every node the plain average over the
   surrounding elements that hold particles (second pass).  W is the total weight of the
   surrounding elements; a node without such elements gets NaN. */
static void compute_stats_elements(orc_ens* E)
{
    const orc_grid* g = E->g;
    double* es = (double*)malloc(sizeof(double) * NSTAT * g->ne);
#pragma omp parallel for schedule(dynamic, 256)
    for (int64_t e = 0; e < g->ne; ++e) {
        double W = 0.0, M[5] = { 0, 0, 0, 0, 0 }, C[7] = { 0, 0, 0, 0, 0, 0, 0 };
        for (int64_t r = E->seg[e]; r < E->seg[e + 1]; ++r) {
            const part* P = &E->p[E->order[r]];
            W += P->w;
            M[0] += P->w * P->u[0]; M[1] += P->w * P->u[1]; M[2] += P->w * P->u[2];
            M[3] += P->w * P->om; M[4] += P->w * P->psi;
        }
        if (W > 0.0) for (int q = 0; q < 5; ++q) M[q] /= W;
        for (int64_t r = E->seg[e]; r < E->seg[e + 1]; ++r) {
            const part* P = &E->p[E->order[r]];
            double d[5] = { P->u[0] - M[0], P->u[1] - M[1], P->u[2] - M[2], P->om - M[3], P->psi - M[4] };
            C[0] += P->w * d[0] * d[0]; C[1] += P->w * d[1] * d[1]; C[2] += P->w * d[2] * d[2];
            C[3] += P->w * d[0] * d[1]; C[4] += P->w * d[0] * d[2]; C[5] += P->w * d[1] * d[2];
            C[6] += P->w * d[4] * d[4];
        }
        double* o = es + e * NSTAT;
        o[0] = W;
        for (int q = 0; q < 5; ++q) o[1 + q] = M[q];
        for (int q = 0; q < 7; ++q) o[6 + q] = W > 0.0 ? C[q] / W : 0.0;
    }
#pragma omp parallel for schedule(dynamic, 256)
    for (int64_t nd = 0; nd < g->nn; ++nd) {
        double* o = E->stats + nd * NSTAT;
        double W = 0.0, S[NSTAT] = { 0 };
        int K = 0;
        for (int64_t j = g->n2e_ptr[nd]; j < g->n2e_ptr[nd + 1]; ++j) {
            const double* x = es + (int64_t)g->n2e[j] * NSTAT;
            W += x[0];
            if (x[0] > 0.0) {
                ++K;
                for (int q = 1; q < NSTAT; ++q) S[q] += x[q];
            }
        }
        o[0] = W;
        for (int q = 1; q < NSTAT; ++q) o[q] = K > 0 ? S[q] / (double)K : NAN;
    }
    free(es);
    E->have_stats = 1;
}

static void compute_stats(orc_ens* E)
{
    const orc_grid* g = E->g;
    if (!E->stats) E->stats = (double*)malloc(sizeof(double) * NSTAT * g->nn);
    if (E->d.estimator == 1) {
        compute_stats_elements(E);
        return;
    }
#pragma omp parallel for schedule(dynamic, 256)
    for (int64_t nd = 0; nd < g->nn; ++nd) {
        double W = 0.0, S[5] = { 0, 0, 0, 0, 0 };
        for (int pass = 0; pass < 2; ++pass) {
            double M[5], C[7] = { 0, 0, 0, 0, 0, 0, 0 };
            if (pass == 1) for (int q = 0; q < 5; ++q) M[q] = S[q] / W;
            for (int64_t j = g->n2e_ptr[nd]; j < g->n2e_ptr[nd + 1]; ++j) {
                int32_t e = g->n2e[j];
                int slot = 0;
                for (int q = 0; q < 3; ++q) if (g->tri[3 * (int64_t)e + q] == (int32_t)nd) slot = q;
                for (int64_t r = E->seg[e]; r < E->seg[e + 1]; ++r) {
                    const part* P = &E->p[E->order[r]];
                    double lam[3];
                    orc_bary(g, e, P->x, P->y, lam);
                    double wl = P->w * lam[slot];
                    double q5[5] = { P->u[0], P->u[1], P->u[2], P->om, P->psi };
                    if (pass == 0) {
                        W += wl;
                        for (int q = 0; q < 5; ++q) S[q] += wl * q5[q];
                    } else {
                        double d[5];
                        for (int q = 0; q < 5; ++q) d[q] = q5[q] - M[q];
                        C[0] += wl * d[0] * d[0]; C[1] += wl * d[1] * d[1]; C[2] += wl * d[2] * d[2];
                        C[3] += wl * d[0] * d[1]; C[4] += wl * d[0] * d[2]; C[5] += wl * d[1] * d[2];
                        C[6] += wl * d[4] * d[4];
                    }
                }
            }
            if (pass == 1) {
                double* o = E->stats + nd * NSTAT;
                o[0] = W;
                if (W == 0.0) { for (int q = 1; q < NSTAT; ++q) o[q] = NAN; }
                else {
                    for (int q = 0; q < 5; ++q) o[1 + q] = M[q];
                    for (int q = 0; q < 7; ++q) o[6 + q] = C[q] / W;
                }
            }
        }
    }
    E->have_stats = 1;
}

/* =====================================================================================
 * Ensemble set-up (Sec. 3.7, first paragraph): an equal number of particles per
 * element, uniform in the element; velocity Gaussian around the nodal mean; frequency
 * Gamma-distributed around the nodal mean frequency; scalar 1 inside the source.
 * ===================================================================================== */
static int grow(orc_ens* E, int64_t need)
{
    if (need <= E->cap) return 0;
    int64_t nc = E->cap ? E->cap : 1024;
    while (nc < need) nc *= 2;
    part* q = (part*)realloc(E->p, sizeof(part) * nc);
    if (!q) return ORC_E_NOMEM;
    E->p = q; E->cap = nc;
    return 0;
}

orc_ens* orc_init(orc_grid* g, const orc_init_desc* d, char* err, int32_t errlen)
{
    if (!g || !d || d->ppe < 0 || d->min_per_bin < 1 || d->bins[0] < 1 || d->bins[1] < 1 || d->bins[2] < 1 ||
        !(d->omega_shape >= 1.0) || !(d->u_sigma >= 0.0) || !(d->src_r >= 0.0) || d->estimator < 0 ||
        d->estimator > 1 || d->conditioning < 0 || d->conditioning > 1) {
        seterr(err, errlen, "bad init descriptor");
        return NULL;
    }
    orc_ens* E = (orc_ens*)calloc(1, sizeof(orc_ens));
    E->g = g; E->d = *d;
    int64_t n = g->ne * (int64_t)d->ppe;
    if (grow(E, n > 0 ? n : 1)) { free(E); seterr(err, errlen, "out of memory"); return NULL; }
    E->n = n;
    E->next_pid = (uint64_t)n;
    E->tm = (double*)malloc(sizeof(double) * g->ne);
    for (int64_t e = 0; e < g->ne; ++e) E->tm[e] = tm_element(g, d, e);
#pragma omp parallel for schedule(static)
    for (int64_t e = 0; e < g->ne; ++e) {
        const double xA = g->fx[3 * e], xB = g->fx[3 * e + 1], xC = g->fx[3 * e + 2];
        const double yA = g->fy[3 * e], yB = g->fy[3 * e + 1], yC = g->fy[3 * e + 2];
        for (int32_t k = 0; k < d->ppe; ++k) {
            part* P = &E->p[e * d->ppe + k];
            uint64_t pid = (uint64_t)(e * d->ppe + k);
            uint32_t w[8];
            draw4(d->seed, d->problem, pid, 0, TAG_INIT, 0, w);
            draw4(d->seed, d->problem, pid, 0, TAG_INIT, 1, w + 4);
            /* uniform point in the triangle: fold the unit square onto the triangle */
            double a = orc_u01(w[0]), b = orc_u01(w[1]);
            if (a + b > 1.0) { a = 1.0 - a; b = 1.0 - b; }
            P->x = xA + a * (xB - xA) + b * (xC - xA);
            P->y = yA + a * (yB - yA) + b * (yC - yA);
            P->e = (int32_t)e;
            double lam[3], f[NF];
            field_weights(E, (int32_t)e, P->x, P->y, lam);
            interp(g, (int32_t)e, lam, f);
            double z01[2], z23[2];
            orc_box_muller(w[2], w[3], z01);
            orc_box_muller(w[4], w[5], z23);
            P->u[0] = f[F_MU] + d->u_sigma * z01[0];
            P->u[1] = f[F_MU + 1] + d->u_sigma * z01[1];
            P->u[2] = f[F_MU + 2] + d->u_sigma * z23[0];
            P->om = orc_gamma(d->omega_shape, f[F_OM], d->seed, d->problem, pid, 0, TAG_INIT_GAMMA);
            double dx = P->x - d->src_x, dy = P->y - d->src_y;
            if (g->period > 0) { if (dx > 0.5 * g->period) dx -= g->period; else if (dx < -0.5 * g->period) dx += g->period; }
            P->psi = (dx * dx + dy * dy < d->src_r * d->src_r) ? 1.0 : 0.0;
            P->w = 1.0;
            P->pid = pid;
            P->alive = 1;
        }
    }
    element_pass(E, 0.0, 0);
    compute_stats(E);
    return E;
}

void orc_ens_destroy(orc_ens* E)
{
    if (!E) return;
    free(E->p); free(E->tm); free(E->seg); free(E->order); free(E->stats);
    free(E);
}

int32_t orc_step(orc_ens* E, double dt)
{
    if (!E || !(dt > 0.0) || !isfinite(dt)) return ORC_E_INVAL;
    int rc = 0;
    int64_t c0 = 0, c1 = 0, c2 = 0, c3 = 0, c4 = 0, c5 = 0, c6 = 0, c7 = 0;
#pragma omp parallel for schedule(static) reduction(+ : c0, c1, c2, c3, c4, c5, c6, c7)
    for (int64_t i = 0; i < E->n; ++i) {
        if (!E->p[i].alive) continue;
        counters cn;
        memset(&cn, 0, sizeof(cn));
        int r = advance_one(E, &E->p[i], dt, &cn);
        c0 += cn.c[0]; c1 += cn.c[1]; c2 += cn.c[2]; c3 += cn.c[3];
        c4 += cn.c[4]; c5 += cn.c[5]; c6 += cn.c[6]; c7 += cn.c[7];
        if (r != 0) {
#pragma omp critical
            { if (rc == 0) rc = r; }
        }
    }
    E->cnt[0] += c0; E->cnt[1] += c1; E->cnt[2] += c2; E->cnt[3] += c3;
    E->cnt[4] += c4; E->cnt[5] += c5; E->cnt[6] += c6; E->cnt[7] += c7;
    E->step++;
    element_pass(E, dt, 1);
    compute_stats(E);
    return rc;
}

int64_t orc_count(const orc_ens* E)
{
    int64_t n = 0;
    for (int64_t i = 0; i < E->n; ++i) n += E->p[i].alive ? 1 : 0;
    return n;
}

int64_t orc_step_index(const orc_ens* E) { return E->step; }

void orc_export(const orc_ens* E, double* x, double* y, double* u, double* om, double* psi, double* w,
                uint64_t* pid, int32_t* elem)
{
    int64_t j = 0;
    for (int64_t i = 0; i < E->n; ++i) {
        const part* P = &E->p[i];
        if (!P->alive) continue;
        if (x) x[j] = P->x;
        if (y) y[j] = P->y;
        if (u) { u[3 * j] = P->u[0]; u[3 * j + 1] = P->u[1]; u[3 * j + 2] = P->u[2]; }
        if (om) om[j] = P->om;
        if (psi) psi[j] = P->psi;
        if (w) w[j] = P->w;
        if (pid) pid[j] = P->pid;
        if (elem) elem[j] = P->e;
        ++j;
    }
}

int32_t orc_import(orc_ens* E, int64_t n, const double* x, const double* y, const double* u,
                   const double* om, const double* psi, const double* w, const uint64_t* pid,
                   const int32_t* elem, int64_t step, uint64_t next_pid)
{
    if (n < 0 || step < 0) return ORC_E_INVAL;
    for (int64_t i = 0; i < n; ++i) if (elem[i] < 0 || elem[i] >= E->g->ne) return ORC_E_INVAL;
    if (grow(E, n > 0 ? n : 1)) return ORC_E_NOMEM;
    for (int64_t i = 0; i < n; ++i) {
        part* P = &E->p[i];
        P->x = x[i]; P->y = y[i];
        P->u[0] = u[3 * i]; P->u[1] = u[3 * i + 1]; P->u[2] = u[3 * i + 2];
        P->om = om[i]; P->psi = psi[i]; P->w = w[i]; P->pid = pid[i]; P->e = elem[i]; P->alive = 1;
    }
    E->n = n;
    E->step = step;
    E->next_pid = next_pid;
    element_pass(E, 0.0, 0);
    compute_stats(E);
    return 0;
}

int32_t orc_stats(const orc_ens* E, double* out)
{
    if (!E->have_stats) return ORC_E_STATE;
    memcpy(out, E->stats, sizeof(double) * NSTAT * E->g->nn);
    return 0;
}

int32_t orc_refresh_stats(orc_ens* E)
{
    element_pass(E, 0.0, 0);
    compute_stats(E);
    return 0;
}

void orc_counters(const orc_ens* E, int64_t out[8]) { for (int q = 0; q < 8; ++q) out[q] = E->cnt[q]; }

/* =====================================================================================
 * Particle-number control (Sec. 3.7, App. B), per element on the canonical order of the
 * last element pass.
 *  - 0 < n < n_min: c = min(n_min - n, n) donors at positions floor((2i+1) n / (2c));
 *    every donor is split into two particles of half weight with identical state; the
 *    new particle gets pid next_pid + (clones of lower elements) + i.
 *  - n > n_max: pairs of neighbouring particles of the same bin, (first+2j, first+2j+1),
 *    taken in order of j and then bin, are merged until n - n_max merges are done or
 *    the pairs run out; the first of a pair receives the weight sum and the
 *    weight-averaged velocity, frequency and scalar, keeping its position; the second
 *    is removed.  Total weight, weighted sums and every bin mean are conserved.
 * ===================================================================================== */
int32_t orc_control(orc_ens* E, int32_t n_min, int32_t n_max, int64_t* report)
{
    if (!E || n_min < 0 || n_max < 1 || n_max < n_min) return ORC_E_INVAL;
    if (!E->have_order) return ORC_E_STATE;
    const orc_grid* g = E->g;
    int64_t ne = g->ne;
    int64_t* nclone = (int64_t*)calloc(ne + 1, sizeof(int64_t));
    int64_t merged = 0, empty = 0, below = 0, above = 0;
    for (int64_t e = 0; e < ne; ++e) {
        int32_t n = (int32_t)(E->seg[e + 1] - E->seg[e]);
        int64_t* idx = E->order + E->seg[e];
        if (n == 0) { ++empty; continue; }
        if (n < n_min) {
            ++below;
            nclone[e + 1] = (n_min - n) < n ? (n_min - n) : n;
        } else if (n > n_max) {
            ++above;
            int32_t gl[3];
            int32_t Cp = bin_structure(n, E->d.bins, E->d.min_per_bin, gl);
            int64_t want = n - n_max, done = 0;
            for (int32_t j = 0; done < want; ++j) {
                int any = 0;
                for (int32_t b = 0; b < Cp && done < want; ++b) {
                    int64_t first = ((int64_t)b * n + Cp - 1) / Cp;
                    int64_t size = ((int64_t)(b + 1) * n + Cp - 1) / Cp - first;
                    if (size < 2 * (int64_t)j + 2) continue;
                    any = 1;
                    part* R = &E->p[idx[first + 2 * j]];
                    part* V = &E->p[idx[first + 2 * j + 1]];
                    double W = R->w + V->w;
                    for (int q = 0; q < 3; ++q) R->u[q] = (R->w * R->u[q] + V->w * V->u[q]) / W;
                    R->om = (R->w * R->om + V->w * V->om) / W;
                    R->psi = (R->w * R->psi + V->w * V->psi) / W;
                    R->w = W;
                    V->alive = 0;
                    ++done;
                }
                if (!any) break;
            }
            merged += done;
        }
    }
    for (int64_t e = 0; e < ne; ++e) nclone[e + 1] += nclone[e];
    int64_t total = nclone[ne];
    int rc = grow(E, E->n + total);
    if (rc) { free(nclone); return rc; }
    int64_t base = E->n;
    for (int64_t e = 0; e < ne; ++e) {
        int64_t c = nclone[e + 1] - nclone[e];
        if (c == 0) continue;
        int32_t n = (int32_t)(E->seg[e + 1] - E->seg[e]);
        int64_t* idx = E->order + E->seg[e];
        for (int64_t i = 0; i < c; ++i) {
            int64_t pos = ((2 * i + 1) * (int64_t)n) / (2 * c);
            part* D = &E->p[idx[pos]];
            D->w = 0.5 * D->w;
            part* Q = &E->p[base + nclone[e] + i];
            *Q = *D;
            Q->pid = E->next_pid + (uint64_t)(nclone[e] + i);
        }
    }
    E->n += total;
    E->next_pid += (uint64_t)total;
    /* drop merged particles */
    int64_t j = 0;
    for (int64_t i = 0; i < E->n; ++i) if (E->p[i].alive) E->p[j++] = E->p[i];
    E->n = j;
    E->have_order = 0;
    if (report) {
        report[0] = E->n; report[1] = total; report[2] = merged; report[3] = empty;
        report[4] = below; report[5] = above;
    }
    free(nclone);
    return 0;
}

/* Statistics feedback (Sec. 3.1, Table 1: a time step uses the Eulerian statistics of the
   step before).  The nodal mean velocity of the last statistics, scaled by alpha (the
   alpha of Eq. 47 in the redistribution test of Sec. 3.7), becomes the nodal <U> field;
   with bit 0 of feed the Reynolds stresses become the nodal R field where their trace is
   positive, with bit 1 the mean frequency becomes the nodal <omega> where it is
   positive.  Nodes without particles (W = 0) keep their fields.  Element gradients and
   Laplacians are derived again from the new <U>.  The micromixing time scale keeps its
   set-up value. */
int32_t orc_feedback(orc_ens* E, double alpha, int32_t feed_rey)
{
    if (!E->have_stats) return ORC_E_STATE;
    orc_grid* g = E->g;
    for (int64_t n = 0; n < g->nn; ++n) {
        const double* o = E->stats + n * NSTAT;
        double* f = g->F + n * NF;
        if (!(o[0] > 0.0)) continue;
        for (int q = 0; q < 3; ++q) f[F_MU + q] = alpha * o[1 + q];
        if ((feed_rey & 1) && o[6] + o[7] + o[8] > 0.0)
            for (int q = 0; q < 6; ++q) f[F_RE + q] = o[6 + q];
        if ((feed_rey & 2) && o[4] > 0.0) f[F_OM] = o[4];
    }
    derive_fields(g);
    return 0;
}

/* Mean velocity correction of Eq. (31): the particles of element e move by -de[e] in
   their two in-plane velocity components (the element gradient of the pressure increment
   is constant per element), and the nodal mean velocity of node n by -dn[n] where the
   node has statistics. */
int32_t orc_shift_velocities(orc_ens* E, const double* de, const double* dn)
{
    if (!E->have_stats) return ORC_E_STATE;
    for (int64_t i = 0; i < E->n; ++i) {
        part* P = &E->p[i];
        if (!P->alive) continue;
        P->u[0] -= de[2 * (int64_t)P->e];
        P->u[1] -= de[2 * (int64_t)P->e + 1];
    }
    for (int64_t n = 0; n < E->g->nn; ++n) {
        double* o = E->stats + n * NSTAT;
        if (!(o[0] > 0.0)) continue;
        o[1] -= dn[2 * n];
        o[2] -= dn[2 * n + 1];
    }
    return 0;
}

/* replaces the nodal elliptic-relaxation tensor by wp [nn][3][3] (row-major ij) */
void orc_set_wp(orc_grid* g, const double* wp)
{
    for (int64_t n = 0; n < g->nn; ++n) {
        const double* w = wp + 9 * n;
        double* f = g->F + n * NF;
        f[F_WP] = w[0]; f[F_WP + 1] = w[4]; f[F_WP + 2] = w[8];
        f[F_WP + 3] = w[1]; f[F_WP + 4] = w[2]; f[F_WP + 5] = w[5];
        f[F_WPT] = w[3]; f[F_WPT + 1] = w[6]; f[F_WPT + 2] = w[7];
    }
}

/* replaces the nodal mean pressure gradient [nn][2] */
void orc_set_grad_p(orc_grid* g, const double* gp)
{
    for (int64_t n = 0; n < g->nn; ++n) {
        g->F[n * NF + F_GP] = gp[2 * n];
        g->F[n * NF + F_GP + 1] = gp[2 * n + 1];
    }
}

/* Time step of Eq. (26): CFL * min_n sqrt(A_n) / max_n ||<Z>_n||_2, A_n the average area
   of the elements around node n, <Z>_n = (<U_1>, <U_2>, <U_3>, <omega>, <psi>) the nodal
   means of the last statistics (nodes without particles are skipped).  Returns 0 when no
   node has a positive mean norm. */
double orc_cfl_dt(const orc_ens* E, double cfl)
{
    if (!E->have_stats) return -1.0;
    const orc_grid* g = E->g;
    double lmin = INFINITY, zmax = 0.0;
    for (int64_t n = 0; n < g->nn; ++n) {
        const int64_t c = g->n2e_ptr[n + 1] - g->n2e_ptr[n];
        if (c > 0) {
            double a = 0.0;
            for (int64_t j = g->n2e_ptr[n]; j < g->n2e_ptr[n + 1]; ++j) a += g->area[g->n2e[j]];
            const double l = sqrt(a / (double)c);
            if (l < lmin) lmin = l;
        }
        const double* o = E->stats + n * NSTAT;
        if (o[0] > 0.0) {
            double z = 0.0;
            for (int q = 1; q <= 5; ++q) z += o[q] * o[q];
            z = sqrt(z);
            if (z > zmax) zmax = z;
        }
    }
    return zmax > 0.0 ? cfl * lmin / zmax : 0.0;
}

/* Particle redistribution (App. B): while the element holding the fewest particles (mine)
   has fewer than n_min, one particle of the element holding the most (maxe) moves to mine.
   Readings:
   - ties in the fewest / most counts go to the lowest element index;
   - the loop also stops once max - min <= 1 (a move would then only swap the two counts,
     so the printed condition min != max would never end when the total does not divide
     evenly);
   - the particle that moves is drawn uniformly among maxe's current particles (canonical
     order of the last pass, then later arrivals in arrival order); it keeps its pid and
     weight, so the particle count and the total weight are unchanged;
   - it takes position, velocity, frequency and scalar of a particle drawn uniformly among
     mine's current particles (the copy of App. B); when mine is empty it keeps its own
     properties and is placed at mine's centroid (in mine's frame, like every position
     held by an element);
   - move k draws one Philox block with key (seed, problem) and counter (k, step, tag 5):
     word 0 picks the moving particle, word 1 the particle copied.
   Returns the number of moves, or a negative status. */
enum { TAG_REDIST = 5 };

typedef struct { int64_t n, cap; int64_t* v; } ivec;
static void ivec_push(ivec* a, int64_t x)
{
    if (a->n == a->cap) { a->cap = a->cap ? 2 * a->cap : 8; a->v = (int64_t*)realloc(a->v, sizeof(int64_t) * a->cap); }
    a->v[a->n++] = x;
}

int64_t orc_redistribute(orc_ens* E, int32_t n_min)
{
    if (!E || n_min < 0) return ORC_E_INVAL;
    if (!E->have_order) return ORC_E_STATE;
    const orc_grid* g = E->g;
    const int64_t ne = g->ne;
    int64_t* cnt = (int64_t*)malloc(sizeof(int64_t) * ne);
    ivec* cur = (ivec*)calloc(ne, sizeof(ivec));   /* current particles of the touched elements */
    char* touched = (char*)calloc(ne, 1);
    for (int64_t e = 0; e < ne; ++e) cnt[e] = E->seg[e + 1] - E->seg[e];
    int64_t moves = 0;
    for (;;) {
        int64_t mine = 0, maxe = 0;
        for (int64_t e = 1; e < ne; ++e) {
            if (cnt[e] < cnt[mine]) mine = e;
            if (cnt[e] > cnt[maxe]) maxe = e;
        }
        if (cnt[mine] >= n_min || cnt[maxe] - cnt[mine] <= 1) break;
        for (int s = 0; s < 2; ++s) {
            int64_t e = s ? maxe : mine;
            if (!touched[e]) {
                touched[e] = 1;
                for (int64_t r = E->seg[e]; r < E->seg[e + 1]; ++r) ivec_push(&cur[e], E->order[r]);
            }
        }
        uint32_t w[4];
        draw4(E->d.seed, E->d.problem, (uint64_t)moves, (uint32_t)E->step, TAG_REDIST, 0, w);
        int64_t r = (int64_t)(orc_u01(w[0]) * (double)cur[maxe].n);
        part* P = &E->p[cur[maxe].v[r]];
        int64_t moving = cur[maxe].v[r];
        memmove(cur[maxe].v + r, cur[maxe].v + r + 1, sizeof(int64_t) * (cur[maxe].n - r - 1));
        cur[maxe].n--;
        if (cur[mine].n > 0) {
            int64_t d = (int64_t)(orc_u01(w[1]) * (double)cur[mine].n);
            const part* D = &E->p[cur[mine].v[d]];
            P->x = D->x;
            P->y = D->y;
            P->u[0] = D->u[0]; P->u[1] = D->u[1]; P->u[2] = D->u[2];
            P->om = D->om;
            P->psi = D->psi;
        } else {
            P->x = (g->fx[3 * mine] + g->fx[3 * mine + 1] + g->fx[3 * mine + 2]) / 3.0;
            P->y = (g->fy[3 * mine] + g->fy[3 * mine + 1] + g->fy[3 * mine + 2]) / 3.0;
        }
        P->e = (int32_t)mine;
        ivec_push(&cur[mine], moving);
        cnt[mine]++;
        cnt[maxe]--;
        ++moves;
    }
    if (moves > 0) E->have_order = 0;
    for (int64_t e = 0; e < ne; ++e) free(cur[e].v);
    free(cur); free(touched); free(cnt);
    return moves;
}
