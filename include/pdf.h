/*
 * pdf.h - C ABI of libpdfgpu.so: the particle time step of the non-hybrid PDF method
 * (Bakosi, Franzese & Boybeyi, "A non-hybrid method for the PDF equations of turbulent
 * flows on unstructured grids") on one AMD Instinct MI355X (gfx950).
 *
 * The method (Secs. 2-3 of the paper) represents a turbulent flow by Lagrangian
 * particles carrying position X, velocity U (3 components), turbulent frequency omega
 * and a passive scalar psi.  An unstructured triangular grid supplies Eulerian fields at
 * its nodes, locates particles and receives nodal statistics.  One explicit time step
 * (Sec. 3.1, Table 1 without the two FEM solves, whose fields are inputs here):
 *   1. interpolate the nodal fields to each particle with P1 shape functions (Eq. 37);
 *   2. advance U by the generalized Langevin model (Eqs. 10/27, closure Eqs. 11, 18) and
 *      omega by Eqs. (19)-(20), forward Euler;
 *   3. move X by Eq. (7) and track it by the next-best-element walk (Sec. 3.6) with the
 *      wall conditions of Sec. 3.8 and the scalar source of Sec. 4.1.2;
 *   4. group particles by host element, build velocity bins by the sort-and-divide
 *      procedure (Sec. 3.5, App. A) and mix psi by IECM (Eqs. 24-25);
 *   5. reduce shape-function-weighted means and central second moments to the nodes
 *      (Sec. 3.3).
 * Particle-number control (Sec. 3.7, App. B) is a separate call.
 *
 * Two forms beyond the plain FP64 step:
 *  - precision PDF_MIXED: velocity, frequency, scalar and weight are stored and advanced
 *    in FP32 (nodal fields used by the particles in FP32, FP32 random-number mapping,
 *    Kahan-compensated FP32 nodal sums); positions, the barycentric locate / reflect
 *    tests and the final division of nodal sums by nodal weights stay FP64.
 *  - several problems per ensemble: independent grids and particle sets (own seeds,
 *    time steps, model constants, sources and bins) advanced together by the same
 *    kernel launches; optionally every two steps replayed from a captured HIP graph
 *    (pdf_set_options) with launch parameters chosen by pdf_autotune.
 *
 * Conventions
 *  - Every call returns a pdf_status; 0 is success.  On failure pdf_last_error() returns
 *    a message for the calling thread.  No exception crosses the ABI.
 *  - Input arrays are host pointers owned by the caller; the library copies what it needs
 *    to the device during the call.  Handles own all device memory until destroyed.
 *  - hip_stream is a hipStream_t (NULL = the default stream).  Work is enqueued on it in
 *    order; calls that return host data synchronise that stream.
 *  - Device-side failures (a particle that cannot be tracked, non-finite state, capacity
 *    exhausted) are recorded in a sticky per-ensemble error word and returned by the next
 *    synchronising call (pdf_stats, pdf_control, pdf_count, pdf_particles_export,
 *    pdf_sync).  After such an error the ensemble must be destroyed.
 *  - A handle is not thread-safe; different handles are independent.
 *  - Symmetric tensors are stored as (11, 22, 33, 12, 13, 23).
 */
#ifndef PDF_H
#define PDF_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct pdf_grid_s* pdf_grid;
typedef struct pdf_ens_s* pdf_ens;
typedef int32_t pdf_status;

#define PDF_OK 0
#define PDF_E_INVAL (-1)     /* bad argument */
#define PDF_E_NOMEM (-2)     /* device or host allocation failed */
#define PDF_E_HIP (-3)       /* HIP runtime error */
#define PDF_E_MESH (-4)      /* invalid mesh (orientation, adjacency, boundary kinds) */
#define PDF_E_CAPACITY (-5)  /* particle capacity exhausted */
#define PDF_E_LOST (-6)      /* a particle could not be located after 64 moves */
#define PDF_E_NONFINITE (-7) /* non-finite input field or particle state */
#define PDF_E_STATE (-8)     /* call not valid in the current state */

/* state precision of an ensemble (pdf_init_desc.precision) */
enum { PDF_FP64 = 0, PDF_MIXED = 1 };

/* estimator of the Eulerian statistics (pdf_init_desc.estimator), Sec. 3.3:
 *  PDF_EST_P1       nodal moments weighted by the P1 shape functions of the particles'
 *                   positions; fields interpolated to the particles (Eq. 37);
 *  PDF_EST_ELEMENT  the paper's two passes: element means and central moments, averaged over
 *                   the surrounding elements with particles; a particle uses the average of
 *                   its element's three nodal values. */
enum { PDF_EST_P1 = 0, PDF_EST_ELEMENT = 1 };

/* conditioning of the scalar mean <phi|V> of the IECM model (pdf_init_desc.conditioning):
 *  PDF_COND_BINS        sort-and-divide velocity bins, bins[0] x bins[1] x bins[2] (Sec. 3.5,
 *                       App. A);
 *  PDF_COND_PROJECTION  Fox's projection (Eqs. 64-66): per element, alpha solves
 *                       rho_ab alpha_b = rho_a with the normalised velocity and velocity-scalar
 *                       correlations; the particles are ordered by the projected normalised
 *                       velocity sum_a alpha_a (U_a - <U_a>) / <u_a^2>^(1/2) (ties by pid) and
 *                       divided into min(bins[0], max(1, n / min_per_bin)) equal-count
 *                       intervals (bins[1], bins[2] unused).  Components without variance
 *                       (spread below 1e-12 of their largest magnitude) or linearly dependent
 *                       on earlier ones (order U1, U2, U3) get alpha = 0; a scalar without
 *                       variance gives alpha = 0, i.e. one key for all particles. */
enum { PDF_COND_BINS = 0, PDF_COND_PROJECTION = 1 };

/* boundary kinds of element edges; edge k of a triangle is the edge opposite vertex k */
enum { PDF_EDGE_INTERIOR = 0, PDF_EDGE_WALL = 1, PDF_EDGE_SLIP = 2, PDF_EDGE_PERIODIC = 3 };

#define PDF_NSTAT 13     /* statistics per node, see pdf_stats */
#define PDF_STATS_ALL 0x1FFFu  /* stat_mask selecting all PDF_NSTAT statistics */
#define PDF_NCOUNTERS 8  /* event counters, see pdf_counters */
#define PDF_NTIMERS 12   /* kernel timers, see pdf_timing */

/* Unstructured P1 triangular mesh (Secs. 3.3-3.4, 3.6).
 *  xy        [n_nodes][2] node coordinates.
 *  tri       [n_elems][3] node ids, counter-clockwise.
 *  edge_kind [n_elems][3] kind of the edge opposite vertex k.  Read only for edges that
 *            belong to a single element, which must be PDF_EDGE_WALL (no-slip) or
 *            PDF_EDGE_SLIP (free-slip).  Shared edges are classified by the library:
 *            periodic when the two sides lie a period apart, interior otherwise.
 *  period_x  > 0: x is periodic with this period; nodes lie in [0, period_x) and an
 *            element spanning the seam references the nodes near x = 0.  0: not periodic. */
typedef struct {
    int64_t n_nodes;
    const double* xy;
    int64_t n_elems;
    const int32_t* tri;
    const uint8_t* edge_kind;
    double period_x;
} pdf_mesh_desc;

/* Frozen Eulerian nodal fields (the outputs of the FEM solves of Sec. 3.2 and of the
 * statistics of Sec. 3.3), each [n_nodes][k]:
 *  grad_p [2]  mean pressure gradient d<P>/dx_i (divided by rho inside Eq. 27);
 *  wp     [6]  elliptic-relaxation tensor of Eq. (11);
 *  mean_u [3]  mean velocity <U_i>;
 *  mean_omega [1] mean turbulent frequency <omega> (> 0);
 *  rey    [6]  Reynolds stresses <u_i u_j> (trace > 0).
 * The library derives the element gradients of <U_i> (Eqs. 39-40) and their nodal
 * second derivatives by the two-pass averaging of Sec. 3.4. */
typedef struct {
    const double* grad_p;
    const double* wp;
    const double* mean_u;
    const double* mean_omega;
    const double* rey;
} pdf_fields_desc;

/* Model constants: viscosity nu, density rho, C3, C4, C_T, C_omega1, C_omega2 (Table 4)
 * and C_s, C_t of the micromixing timescale, Eq. (25). */
typedef struct {
    double nu, rho, C3, C4, CT, Cw1, Cw2, Cs, Ct;
} pdf_model;

/* Particle set-up (Sec. 3.7, first paragraph) and per-ensemble options.
 *  ppe            particles per element at set-up (uniform in each element);
 *  u_sigma        standard deviation of the Gaussian initial velocity about <U>(x);
 *  omega_shape    shape of the Gamma initial frequency about <omega>(x) (>= 1);
 *  src_x, src_y, src_r   scalar source disk (Sec. 4.1.2); psi = 1 inside at set-up;
 *  src_continuous 1: particles inside the disk after tracking get psi = 1 every step;
 *  bins[3]        requested velocity bins per direction (Sec. 3.5), each >= 1;
 *  min_per_bin    minimum particles per bin (>= 1; the paper uses 2);
 *  precision      PDF_FP64 or PDF_MIXED (the same for every problem of an ensemble);
 *  seed           seed of the counter-based generator (key: seed low word, seed high
 *                 word XOR the problem's index in the ensemble);
 *  capacity       particle slots for this problem (0: max(2 x ppe x n_elems, 1024));
 *                 the ensemble allocates the sum over its problems;
 *  estimator      PDF_EST_P1 or PDF_EST_ELEMENT (the same for every problem);
 *  conditioning   PDF_COND_BINS or PDF_COND_PROJECTION (may differ between problems). */
typedef struct {
    int32_t ppe;
    double u_sigma, omega_shape;
    double src_x, src_y, src_r;
    int32_t src_continuous;
    int32_t bins[3];
    int32_t min_per_bin;
    int32_t precision;
    uint64_t seed;
    int64_t capacity;
    int32_t estimator;
    int32_t conditioning;
} pdf_init_desc;

/* Result of pdf_control. */
typedef struct {
    int64_t live;    /* live particles after the call */
    int64_t cloned;  /* particles added by splitting */
    int64_t merged;  /* particles removed by merging */
    int64_t empty;   /* elements without particles */
    int64_t below;   /* elements that were below n_min */
    int64_t above;   /* elements that were above n_max */
} pdf_control_report;

/* Build the device grid: validates the mesh (counter-clockwise, manifold, boundary kinds)
 * and the fields (finite, <omega> > 0, k > 0), builds neighbours, element frames across the
 * periodic seam, the elements around each node, wall lines of wall elements (Sec. 3.8),
 * element gradients and nodal Laplacians of <U>, and uploads everything.
 * Errors: PDF_E_INVAL, PDF_E_MESH, PDF_E_NONFINITE, PDF_E_NOMEM, PDF_E_HIP. */
pdf_status pdf_grid_create(const pdf_mesh_desc* mesh, const pdf_fields_desc* fields,
                           const pdf_model* model, void* hip_stream, pdf_grid* out);
pdf_status pdf_grid_destroy(pdf_grid grid);

/* Create an ensemble of n_problems >= 1 independent problems, problem p on grids[p] with
 * descs[p], and seed ppe particles per element (Sec. 3.7): pid = e * ppe + k within each
 * problem; initial element-grouping, binning and statistics are computed.  The grids
 * must outlive the ensemble.  Errors: PDF_E_INVAL, PDF_E_NOMEM, PDF_E_CAPACITY,
 * PDF_E_HIP. */
pdf_status pdf_particles_init(const pdf_grid* grids, const pdf_init_desc* descs,
                              int32_t n_problems, void* hip_stream, pdf_ens* out);
pdf_status pdf_ens_destroy(pdf_ens ens);

/* Advance n_steps time steps; problem p uses the time step dt[p] (> 0, one entry per
 * problem).  Enqueues only; does not synchronise (a changed dt is uploaded first, with a
 * synchronisation).  With an unchanged dt the call can be captured into a HIP graph by the
 * caller (with pdf_control without a report); a replay advances the ensemble by the
 * captured steps with the captured dt.  A step moves the particle state from one of two
 * device buffers to the other, so a graph meant to be replayed must hold an even number of
 * steps. */
pdf_status pdf_step(pdf_ens ens, const double* dt, int32_t n_steps, void* hip_stream);

/* Nodal statistics of the last step (Sec. 3.3) of one problem.  Statistic j (0..12) is
 *   W = sum_p w_p N_n(x_p), <U1>, <U2>, <U3>, <omega>, <psi>,
 *   <u1u1>, <u2u2>, <u3u3>, <u1u2>, <u1u3>, <u2u3>, <psi'psi'>
 * over the particles of the elements around node n, weighted by w_p N_n(x_p); the
 * second moments are about the node's own means (NaN where W = 0).
 * stat_mask: bit j selects statistic j (PDF_STATS_ALL: all 13); out = [n_nodes][k] with the
 * k selected statistics in ascending j.  A mask that selects none or has bits above 12 is
 * PDF_E_INVAL.
 * out_is_device != 0: out is a device pointer and the copy is enqueued on hip_stream;
 * otherwise out is host memory and the call synchronises (a subset of the columns is
 * selected on the device, in a temporary allocated for the call: PDF_E_NOMEM if it fails). */
pdf_status pdf_stats(pdf_ens ens, int32_t problem, uint32_t stat_mask, double* out, int32_t out_is_device,
                     void* hip_stream);

/* Per-element particle-number control (Sec. 3.7, App. B) on the canonical order of the
 * last step: elements with 0 < n < n_min split min(n_min - n, n) particles into two
 * half-weight copies; elements with n > n_max merge pairs of particles of one velocity
 * bin into their weighted average, up to n - n_max merges.  Conserves the total weight and
 * the weighted sums of U, omega and psi in every element and bin.
 * report != NULL: synchronises, fills report and returns a capacity error (clones beyond
 * the capacity are not written; those written are counted).  report == NULL: only enqueues
 * (no synchronisation, no host copy), so that pdf_step and pdf_control can be captured
 * together into one HIP graph by the caller; the particle kernels of the following steps
 * then cover the whole capacity, whose unused slots return at once, and a capacity error
 * is returned by the next synchronising call.  Errors: PDF_E_INVAL (n_min > n_max,
 * n_max < 1), PDF_E_STATE (no step since the last control), PDF_E_CAPACITY, PDF_E_HIP. */
pdf_status pdf_control(pdf_ens ens, int32_t n_min, int32_t n_max, pdf_control_report* report,
                       void* hip_stream);

/* Live particles of one problem, or of the whole ensemble for problem = -1
 * (synchronises). */
pdf_status pdf_count(pdf_ens ens, int32_t problem, int64_t* live);

/* Copy the live particles of one problem to host arrays of at least cap entries (any
 * pointer may be NULL): x, y, u [n][3], omega, psi, weight, pid, host element (numbered
 * within the problem's grid).  *n_out = live count.  Order: element-grouped, canonical
 * within elements after a step.  Mixed-form values are widened to double.  Synchronises. */
pdf_status pdf_particles_export(pdf_ens ens, int32_t problem, int64_t cap, double* x, double* y,
                                double* u, double* omega, double* psi, double* w,
                                uint64_t* pid, int32_t* elem, int64_t* n_out, void* hip_stream);

/* Replace the particle state with n host-side particles (elem must be each particle's host
 * element); sets the step counter and the next pid, then recomputes grouping, bins and
 * statistics without mixing.  Single-problem ensembles only (problem 0); mixed-form
 * ensembles round the values to FP32.  Synchronises.  Errors: PDF_E_INVAL,
 * PDF_E_CAPACITY, PDF_E_NONFINITE. */
pdf_status pdf_particles_import(pdf_ens ens, int32_t problem, int64_t n, const double* x,
                                const double* y, const double* u, const double* omega,
                                const double* psi, const double* w, const uint64_t* pid,
                                const int32_t* elem, int64_t step, uint64_t next_pid,
                                void* hip_stream);

/* Event counters of one problem since set-up (synchronises): wall (a), wall (b),
 * reflections, fall-back searches, omega reflections, C0 clamps, walk moves, source hits. */
pdf_status pdf_counters(pdf_ens ens, int32_t problem, int64_t out[PDF_NCOUNTERS]);

/* Kernel timing with HIP events on the ensemble's stream.  enable = 1 starts (and resets)
 * recording, 0 stops.  ms_out[PDF_NTIMERS] (may be NULL) receives the summed durations and
 * launches_out[PDF_NTIMERS] the launch counts, in the order: init, advance, scan,
 * scatter, element pass, node finalize, control plan, control scan, control apply, fill,
 * count, other.  Synchronises when reading. */
pdf_status pdf_timing(pdf_ens ens, int32_t enable, double* ms_out, int64_t* launches_out);

/* Statistics feedback (Sec. 3.1, Table 1 order: a step uses the Eulerian statistics of the
 * step before).  enable != 0: the nodal mean velocity of the current statistics, scaled
 * by alpha (the alpha of Eq. 47 in the redistribution test of Sec. 3.7; 1 for plain
 * feedback), with bit 0 of feed the Reynolds stresses (where their trace is positive) and
 * with bit 1 the mean frequency (where positive) become the ensemble's nodal <U>, R and
 * <omega> fields, now and after every later step; element
 * gradients (Eq. 40) and nodal Laplacians (Sec. 3.4) of <U> are derived again.  Nodes
 * without particles keep their fields; the micromixing time scale keeps its set-up value.
 * The ensemble works on its own copy of the fields (the grid is not modified).
 * enable = 0 stops the feedback and keeps the current fields.  Synchronises. */
pdf_status pdf_set_feedback(pdf_ens ens, int32_t enable, double alpha, int32_t feed, void* hip_stream);

/* Particle redistribution (App. B) of one problem (problem = -1: every problem, in order)
 * on the canonical order of the last step: while the element with the fewest particles has
 * fewer than n_min and at least two fewer than the element with the most, one particle of
 * the fullest element moves to the emptiest (ties: lowest element index).  The moving
 * particle is drawn uniformly among the giving element's current particles, keeps its
 * pid and weight, and takes position, velocity, frequency and scalar of a particle drawn
 * uniformly among the receiving element's current particles, or, when that element is
 * empty, keeps its properties and sits at the element's centroid.  Move k of a problem
 * draws one Philox block with the problem's key and counter (k, step, tag 5).  Particle
 * count, pids and total weight do not change.  The moves are planned on the device (the
 * host reads two small per-problem summaries: the count extremes and the level histograms)
 * and applied by two device kernels; a later pdf_control needs another step first.
 * *moves_out (may be NULL) receives the number of moves.  Synchronises.
 * Errors: PDF_E_INVAL (n_min < 0, bad problem), PDF_E_STATE (no step since the last
 * control or redistribution), PDF_E_CAPACITY (a problem whose counts span more than 2^22
 * levels, or whose elements times the count levels one side visits exceed 2^31 - 1),
 * PDF_E_NOMEM, PDF_E_HIP. */
pdf_status pdf_redistribute(pdf_ens ens, int32_t problem, int32_t n_min, int64_t* moves_out,
                            void* hip_stream);

/* Constants of the elliptic relaxation model, Eqs. (12)-(17) (Table 4: C1 = 1.85,
 * C2 = 0.63, C_L = 0.134, C_eta = 72, C_v = 1.4, gamma_5 = 0.1). */
typedef struct {
    double C1, C2, CL, Ceta, Cv, gamma5;
} pdf_elliptic_model;

/* Elliptic relaxation, Eq. (12) (Sec. 3.2), from the ensemble's current nodal statistics
 * (single-problem ensembles): P1 finite elements on the grid's triangles, right-hand side
 * (1 - C1)/2 k <omega> delta_ij + k H_ijkl d<U_k>/dx_l (Eqs. 13-15; nodal velocity
 * gradients are the averages of the element gradients around the node), L of Eqs. (16)-(17)
 * per element from the averages of its vertices' k and epsilon (C_xi = 1 + 1.3 n_i^2 for
 * wp_ii, 1 for the off-diagonal components, n the outward normal of the nearest no-slip wall
 * edge), wp_ij = -4.5 eps n_i n_j at no-slip wall nodes (Eq. 59, n the normalised sum of
 * the adjacent wall edges' outward normals) and zero off-diagonal components at free-slip
 * nodes (Sec. 4.1.1).  The nine components are solved together by Jacobi-preconditioned
 * conjugate gradients from zero, until every component's residual norm falls below tol
 * times its initial one, or max_iter iterations.  store != 0: the solution becomes the
 * ensemble's nodal wp field (all nine components) for the following steps, closing the loop
 * of Table 1 (the ensemble then works on its own copy of the fields).  wp_out (may be NULL)
 * receives wp_ij at the nodes, [nn][9] row-major in (i, j), on the device when
 * out_is_device, else on the host; *iters_out (may be NULL) the iterations.  Synchronises.
 * Errors: PDF_E_INVAL (several problems, consts or tol invalid), PDF_E_STATE (a node
 * without statistics), PDF_E_NOMEM, PDF_E_HIP. */
pdf_status pdf_elliptic_relaxation(pdf_ens ens, const pdf_elliptic_model* consts, double tol, int32_t max_iter,
                                   int32_t store, double* wp_out, int32_t out_is_device, int32_t* iters_out,
                                   void* hip_stream);

/* Stabilised pressure projection, Eqs. (30)-(33) (Sec. 3.2), after a step of a single-problem
 * ensemble: with <U>* the nodal mean velocity of the current statistics, solves
 * (1/rho) lap dP = (div <U>* - C_p (1/rho) lap P) / dt for the increment dP (P1 finite
 * elements, natural condition at the walls, the solution with zero nodal sum), then applies
 * Eq. (31): every particle's in-plane velocity moves by -(dt/rho) times the gradient of dP
 * in its element, and the nodal mean velocity of the statistics by -(dt/rho) times the
 * average of those gradients around the node.  P (zero at the first call) accumulates dP;
 * the nodal mean-pressure gradient used by later steps becomes the set-up field plus the
 * nodal average of the element gradients of P; with statistics feedback on, the corrected
 * nodal mean velocity is fed back again.  CG from zero to tol relative residual or max_iter
 * iterations, preconditioned by a smoothed-aggregation multigrid V-cycle built once per
 * ensemble from the assembled matrix (Jacobi when its aggregation stalls); a grid of at
 * most 400 nodes is solved by its dense coarse inverse alone.  dp_out (may be NULL) receives dP [nn];
 * *iters_out (may be NULL) the iterations.  Synchronises.
 * Errors: PDF_E_INVAL, PDF_E_STATE (a node without statistics), PDF_E_NOMEM, PDF_E_HIP. */
pdf_status pdf_pressure_projection(pdf_ens ens, double dt, double cp, double tol, int32_t max_iter, double* dp_out,
                                   int32_t out_is_device, int32_t* iters_out, void* hip_stream);

/* Time step of Eq. (26) (Sec. 3.1) for one problem from its last statistics:
 * *dt_out = cfl * min_n sqrt(A_n) / max_n ||(<U_1>, <U_2>, <U_3>, <omega>, <psi>)_n||_2, A_n the
 * average area of the elements around node n (the paper uses cfl = 0.7); nodes without
 * particles do not enter the maximum; 0 when no node has a positive norm.  Synchronises. */
pdf_status pdf_cfl_dt(pdf_ens ens, int32_t problem, double cfl, double* dt_out, void* hip_stream);

/* pdf_cfl_dt without any allocation, for callers that cannot allocate device memory (code
 * under HIP graph capture, serving loops, harnesses that forbid hipMalloc).  Writes the same
 * time step as pdf_cfl_dt (bit for bit) into dt_out, one double in device memory owned by the
 * caller, as work enqueued on hip_stream: no synchronisation, no host copy.  The statistics
 * it reads must be complete in hip_stream's order (pass the stream of the pdf_step calls).
 * Its partial results live in a fixed array of the library, 1 MiB on every device it runs on
 * (looked up at pdf_particles_init), held until the process ends: calls that overlap on one
 * device race for it and must be ordered by the caller (one stream, or events).
 * Errors: PDF_E_INVAL, PDF_E_CAPACITY (the problem has more than 2^24 nodes), PDF_E_STATE
 * (the array of the device could not be set up), PDF_E_HIP. */
pdf_status pdf_cfl_dt_noalloc(pdf_ens ens, int32_t problem, double cfl, double* dt_out, void* hip_stream);

/* Launch options of an ensemble; none changes any result.
 *  use_graph  1: pdf_step replays every two steps from a captured HIP graph on a
 *             stream of the ensemble (ordered after and before hip_stream by events),
 *             captured again when the slot bound or a time step changes;
 *  adv_block  workgroup size of the particle loop: 64 (the default), 128 or 256;
 *  ppl        particles per lane of the wavefront element kernel (elements with more
 *             than 64 x ppl particles take the workgroup kernel): 1..6 or 8. */
typedef struct {
    int32_t use_graph;
    int32_t adv_block;
    int32_t ppl;
} pdf_options;

pdf_status pdf_get_options(pdf_ens ens, pdf_options* out);
/* Errors: PDF_E_INVAL for values outside the lists above.  Synchronises. */
pdf_status pdf_set_options(pdf_ens ens, const pdf_options* opt);

/* Autotuner: times candidate (adv_block, ppl) pairs on the live ensemble, each for one
 * warm-up step plus steps_per_trial steps, and keeps the fastest.  The ensemble really
 * advances by all these steps (results do not depend on the options).  trial_ms, when
 * not NULL, receives up to *n_trials timings; *n_trials returns the number of trials.
 * Synchronises. */
pdf_status pdf_autotune(pdf_ens ens, const double* dt, int32_t steps_per_trial, void* hip_stream,
                        pdf_options* chosen, int32_t* n_trials, double* trial_ms);

/* Wait for the ensemble's work and return its sticky device error, if any. */
pdf_status pdf_sync(pdf_ens ens);

/* Message of the last failure on the calling thread ("" if none). */
const char* pdf_last_error(void);

#ifdef __cplusplus
}
#endif
#endif
