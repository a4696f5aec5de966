/*
 * CPU oracle of the particle time step of the non-hybrid PDF method
 * (Bakosi, Franzese & Boybeyi, "A non-hybrid method for the PDF equations of
 * turbulent flows on unstructured grids").
 *
 * TEST INFRASTRUCTURE ONLY.  This is a plain, slow, FP64 restatement of the method,
 * used to check the GPU library.  It shares no source with the GPU library; only
 * tests, the smoke check and the benchmark's CPU-baseline leg may load it.
 *
 * Every function cites the passage of the paper it restates.  Where the paper is
 * silent the reading taken is stated next to the code.
 */
#ifndef ORC_H
#define ORC_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { ORC_OK = 0, ORC_E_INVAL = -1, ORC_E_NOMEM = -2, ORC_E_MESH = -4, ORC_E_CAPACITY = -5,
       ORC_E_LOST = -6, ORC_E_NONFINITE = -7, ORC_E_STATE = -8 };

typedef struct orc_grid orc_grid;
typedef struct orc_ens orc_ens;

/* model constants: nu, rho, C3, C4, CT, Cw1, Cw2, Cs, Ct (Table 4, Eq. 25) */
typedef struct { double nu, rho, C3, C4, CT, Cw1, Cw2, Cs, Ct; } orc_model;

typedef struct {
    int32_t ppe; double u_sigma, omega_shape;
    double src_x, src_y, src_r; int32_t src_continuous;
    int32_t bins[3]; int32_t min_per_bin;
    uint64_t seed; int32_t problem;
    int32_t estimator;   /* 0: P1-weighted nodal moments and P1 interpolation;
                            1: element means averaged to the nodes, element-averaged fields (Sec. 3.3) */
    int32_t conditioning; /* 0: sort-and-divide velocity bins (Sec. 3.5, App. A);
                             1: Fox's projection on one velocity direction, bins[0] intervals (Eqs. 64-66) */
} orc_init_desc;

/* --- units (used by the pins) --- */
void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);
double orc_u01(uint32_t w);
void orc_box_muller(uint32_t a, uint32_t b, double out[2]);
void orc_normals(uint64_t seed, int32_t problem, uint64_t pid, uint32_t step, uint32_t tag,
                 int64_t n, double* out); /* n Gaussians from idx = 0,1,... (4 words each) */
double orc_gamma(double shape, double mean, uint64_t seed, int32_t problem, uint64_t pid,
                 uint32_t step, uint32_t tag);

/* --- grid --- */
orc_grid* orc_grid_create(int64_t nn, const double* xy, int64_t ne, const int32_t* tri,
                          const uint8_t* edge_kind, double period_x,
                          const double* grad_p, const double* wp, const double* mean_u,
                          const double* mean_omega, const double* rey, const orc_model* m,
                          char* err, int32_t errlen);
void orc_grid_destroy(orc_grid*);
/* element frame vertex coordinates [ne][6] (xA,yA,xB,yB,xC,yC), area [ne], neighbours [ne][3],
   classified edge kinds [ne][3], grad<U> [ne][6], laplacian<U> [nn][3], wall flag [ne],
   wall line [ne][4] (px,py,nx,ny) */
void orc_grid_export(const orc_grid*, double* frame, double* area, int32_t* nbr, uint8_t* kind,
                     double* gradu, double* lapu, uint8_t* wall, double* wline);
/* barycentric area coordinates of (x,y) in element e (Eqs. 44-45) */
void orc_bary(const orc_grid*, int32_t e, double x, double y, double lam[3]);
/* brute-force point location over all elements: first element (ascending id) whose closed
   area coordinates are all >= 0, trying shifts 0, -period, +period; -1 if none */
int32_t orc_locate_brute(const orc_grid*, double x, double y, double* xs);

/* --- ensemble --- */
orc_ens* orc_init(orc_grid*, const orc_init_desc*, char* err, int32_t errlen);
void orc_ens_destroy(orc_ens*);
int32_t orc_step(orc_ens*, double dt);
int64_t orc_count(const orc_ens*);
int64_t orc_step_index(const orc_ens*);
/* arrays of orc_count() entries in the oracle's internal order */
void orc_export(const orc_ens*, double* x, double* y, double* u /*[n][3]*/, double* om,
                double* psi, double* w, uint64_t* pid, int32_t* elem);
/* replace the particle state; n entries; elem must be the host element of (x,y) */
int32_t orc_import(orc_ens*, int64_t n, const double* x, const double* y, const double* u,
                   const double* om, const double* psi, const double* w, const uint64_t* pid,
                   const int32_t* elem, int64_t step, uint64_t next_pid);
/* nodal statistics [nn][13]: W, <U1>,<U2>,<U3>,<w>,<psi>, R11,R22,R33,R12,R13,R23, var(psi) */
int32_t orc_stats(const orc_ens*, double* out);
/* recompute the statistics of the current state (no advance) */
int32_t orc_refresh_stats(orc_ens*);
/* statistics feedback into the grid's nodal fields (see orc.c) */
int32_t orc_feedback(orc_ens*, double alpha, int32_t feed_rey);
/* Eq. (31): particles of element e shift by -de[e][2], nodal mean velocities by -dn[n][2] */
int32_t orc_shift_velocities(orc_ens*, const double* de, const double* dn);
/* replaces the nodal mean pressure gradient [nn][2] */
void orc_set_grad_p(orc_grid*, const double* gp);
/* replaces the nodal elliptic-relaxation tensor, wp [nn][3][3] row-major */
void orc_set_wp(orc_grid*, const double* wp);
/* time step of Eq. (26) from the last statistics (see orc.c) */
double orc_cfl_dt(const orc_ens*, double cfl);
/* particle redistribution of App. B (see orc.c); returns the number of moves */
int64_t orc_redistribute(orc_ens*, int32_t n_min);
/* number control; report[0..5] = live, cloned, merged, empty elems, elems below, above */
int32_t orc_control(orc_ens*, int32_t n_min, int32_t n_max, int64_t* report);
/* counters: wall (a), wall (b), reflections, fallbacks, omega reflections, C0 clamps,
   walk steps, source hits */
void orc_counters(const orc_ens*, int64_t out[8]);
/* element pass on its own: canonical order (positions) and bin of each particle of one
   element given its velocities and pids; returns bins used (C') */
int32_t orc_bin_element(int32_t n, const double* u /*[n][3]*/, const uint64_t* pid,
                        const int32_t bins[3], int32_t min_per_bin, int32_t* pos, int32_t* bin);
/* Fox's projection of one element (Eqs. 64-66): projected velocity key[n], canonical
   positions and bins (nc intervals, at least min_per_bin particles each), and the
   projection vector alpha[3] of the normalised velocities; returns bins used */
int32_t orc_project_element(int32_t n, const double* u /*[n][3]*/, const double* psi, const double* w,
                            const uint64_t* pid, int32_t nc, int32_t min_per_bin, double* key, int32_t* pos,
                            int32_t* bin, double alpha[3]);
/* micromixing timescale of element e (Eq. 25 at the centroid) */
double orc_tm(const orc_ens*, int32_t e);

#ifdef __cplusplus
}
#endif
#endif
