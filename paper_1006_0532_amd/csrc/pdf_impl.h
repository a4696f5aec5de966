// Internal types of libpdfgpu: device data layout and host-side handles.
#pragma once
#include "amg.h"
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
#include <vector>

#include "pdf.h"

namespace pdfgpu {

// Per-node field record, 24 doubles (192 B, 16-B aligned):
// grad<P>(2), wp_11, wp_22, wp_33, wp_12, wp_13, wp_23 (6), <U>(3), lap<U>(3), <omega>(1),
// R(6), wp_21, wp_31, wp_32 (3; the elliptic-relaxation tensor is not symmetric, Eq. 13)
constexpr int NODE_STRIDE = 24;
enum { NF_GP = 0, NF_WP = 2, NF_MU = 8, NF_LAP = 11, NF_OM = 14, NF_RE = 15, NF_WPT = 21 };

// Edge kinds after classification.
enum : uint8_t { KIND_INTERIOR = 0, KIND_WALL = 1, KIND_SLIP = 2, KIND_PERIODIC = 3 };

// Per-element record used by the particle kernels (176 B).
struct __attribute__((aligned(16))) ElemGeo {
    double x[3], y[3];  // vertices in the element's own frame (seam elements unwrapped)
    double area;        // A_e > 0
    double inv_area;    // 1 / A_e
    double shift[3];    // x shift added when leaving through a periodic edge
    double gu[6];       // d<U1>/dx, d<U1>/dy, d<U2>/dx, d<U2>/dy, d<U3>/dx, d<U3>/dy
    double wl[4];       // wall line: point (x, y) and inward unit normal (x, y)
    int32_t node[3];
    int32_t nbr[3];     // -1 across a boundary edge
    uint8_t kind[3];
    uint8_t wall;       // element touches a no-slip wall by an edge or a node
    int32_t prob;       // problem of the ensemble the element belongs to
};
static_assert(sizeof(ElemGeo) % 16 == 0, "ElemGeo alignment");

constexpr int NSTAT = PDF_NSTAT;     // statistics per node
constexpr int NPART = 13;            // partial sums per element vertex
constexpr int NCOUNT = PDF_NCOUNTERS;
constexpr int CNT_SLOTS = 256;       // spread copies of every event counter

// device error bits (sticky)
enum : uint32_t { ERR_LOST = 1u, ERR_NONFINITE = 2u, ERR_CAPACITY = 4u, ERR_BADELEM = 8u };

// timers
enum { T_INIT = 0, T_ADVANCE, T_SCAN, T_SCATTER, T_ELEMENT, T_NODE, T_CPLAN, T_CSCAN, T_CAPPLY,
       T_FILL, T_COUNT, T_OTHER, T_N };

struct RngKey {
    uint32_t k0, k1;
};

struct ModelC {
    double nu, rho, C3, C4, CT, Cw1, Cw2, Cs, Ct;
};

// Structure-of-arrays particle state in HBM: positions always FP64, the rest in R
// (double: FP64 form, float: mixed form).
template <class R>
struct SoaT {
    double *x, *y;
    R *u0, *u1, *u2, *om, *psi, *w;
    uint64_t* pid;
    int32_t* elem;  // host element; -1 = dead slot
};

// the same arrays untyped, as the host holds them
struct SoaRaw {
    double *x = nullptr, *y = nullptr;
    void *u0 = nullptr, *u1 = nullptr, *u2 = nullptr, *om = nullptr, *psi = nullptr, *w = nullptr;
    uint64_t* pid = nullptr;
    int32_t* elem = nullptr;
    template <class R>
    SoaT<R> as() const
    {
        return SoaT<R>{x, y, (R*)u0, (R*)u1, (R*)u2, (R*)om, (R*)psi, (R*)w, pid, elem};
    }
};

// Per-problem parameters of an ensemble (one entry per independent problem).
struct ProbParams {
    ModelC m;
    double dt;                     // time step of the current pdf_step
    double period;                 // x period of the problem's grid (0: none)
    double src_x, src_y, src_r2;   // scalar source disk
    double u_sigma, omega_shape;   // set-up distributions
    RngKey key;                    // (seed lo, seed hi ^ problem)
    int32_t src_cont;
    int32_t bins0, bins1, bins2, minpb;
    int32_t ppe;
    int32_t estimator;             // 0: P1-weighted moments, P1 fields; 1: element means to nodes
    int32_t conditioning;          // 0: sort-and-divide bins; 1: Fox's projection (Eqs. 64-66)
    int64_t eoff, ne;              // element range in the ensemble
    int64_t noff, nn;              // node range
    int64_t soff;                  // first set-up slot
    uint64_t next_pid;             // next particle id of the problem
    double sdt, s2nu, irho;        // sqrt(dt), sqrt(2 nu), 1 / rho (kept with dt and m)
};

}  // namespace pdfgpu

struct pdf_grid_s {
    int device = 0;
    int64_t nn = 0, ne = 0;
    double period = 0.0;
    pdfgpu::ModelC model{};
    // host copies
    std::vector<pdfgpu::ElemGeo> h_geo;
    std::vector<double> h_node;       // [nn][NODE_STRIDE]
    std::vector<int64_t> h_n2e_ptr;   // [nn+1]
    std::vector<int32_t> h_n2e;       // element*3 + slot, ascending element
    // device
    pdfgpu::ElemGeo* d_geo = nullptr;
    double* d_node = nullptr;
    int64_t* d_n2e_ptr = nullptr;
    int32_t* d_n2e = nullptr;
};

// Device view of the grid an ensemble runs on: the grid's own arrays for one problem,
// concatenated copies (element, node and CSR indices offset) for several.
struct DevGrid {
    int64_t nn = 0, ne = 0;
    pdfgpu::ElemGeo* geo = nullptr;
    double* node = nullptr;          // FP64 node records
    float* node32 = nullptr;         // FP32 node records (mixed form)
    int64_t* n2e_ptr = nullptr;
    int32_t* n2e = nullptr;
    bool owned = false;              // arrays allocated by the ensemble
    bool own_fields = false;         // geo and node copied for statistics feedback (one problem)
};

// Work arrays of the Eulerian solves (allocated on first use, one problem).
struct FemState {
    bool geom = false;
    uint8_t* wkind = nullptr;     // [nn] 0 interior, 1 free-slip node, 2 no-slip node
    double* wnrm = nullptr;       // [nn][2] outward wall normal of no-slip nodes
    double* enrm = nullptr;       // [ne][2] normal of the nearest no-slip wall edge
    double* ke = nullptr;         // [ne][8] element matrices (see fem.h)
    double *f = nullptr, *xfix = nullptr, *b = nullptr, *x = nullptr;        // [nn][9]
    double *r = nullptr, *z = nullptr, *p = nullptr, *Ap = nullptr, *diag = nullptr;
    uint16_t* fixed = nullptr;    // [nn] Dirichlet bits of the nine components
    uint16_t* nofix = nullptr;    // [nn] all zero
    double* L2 = nullptr;         // [ne][4]
    double* sc = nullptr;         // CG scalars [6][9]
    double* partial = nullptr;    // reduction partials
    bool pressure = false;        // P and gp0 set up
    int32_t *csr_rp = nullptr, *csr_col = nullptr;   // assembled stiffness matrix of the grid
    double* csr_val = nullptr;
    double* partial2 = nullptr;   // block partials of the assembled-matrix CG
    int64_t csr_nnz = 0;
    pdfgpu::HostCsr hcsr;            // host copy of the assembled matrix (multigrid set-up)
    double* cval4 = nullptr;         // [4][csr_nnz] assembled elliptic-relaxation operator
    pdfgpu::AmgDev* amg = nullptr;   // multigrid preconditioner of the pressure CG (null: Jacobi)
    bool amg_tried = false;
    double *P = nullptr, *gp0 = nullptr, *gP = nullptr, *gdP = nullptr;       // [nn], [nn][2], [ne][2]
};

struct pdf_ens_s {
    pdf_grid grid = nullptr;         // grid of problem 0
    std::vector<pdf_grid> grids;     // grid of every problem
    std::vector<pdf_init_desc> descs;
    std::vector<pdfgpu::ProbParams> h_prm;
    pdfgpu::ProbParams* d_prm = nullptr;
    int32_t n_problems = 1;
    int32_t precision = 0;           // PDF_FP64 or PDF_MIXED
    DevGrid dg;
    pdf_init_desc d{};
    hipStream_t stream = nullptr;
    int64_t cap = 0;
    int64_t n_slots_ub = 0;   // host-side upper bound of the used slots
    int64_t step = 0;
    uint64_t next_pid = 0;
    int cur = 0;              // which SoA buffer is current
    pdfgpu::SoaRaw buf[2]{};
    int32_t* counts = nullptr;   // [ne] particles per element (zero between steps)
    int32_t* start = nullptr;    // [ne+1] segment starts of the current buffer
    int32_t* idx = nullptr;      // [cap] slot of each grouped particle
    int32_t* arrival = nullptr;  // [cap] arrival rank of each slot in its new host (particle loop)
    int32_t* scan_tmp = nullptr; // block sums
    int64_t* d_meta = nullptr;   // [0] used slots, [1] live, [2] clones of the last control, [4] step
    void* part = nullptr;        // [ne][3][NPART] per-vertex partial sums (state precision)
    double* stats = nullptr;     // [nn][NSTAT]
    void* shift = nullptr;       // [nn][5] reference values of the single-pass moments (state precision)
    double* tm = nullptr;        // [ne] micromixing timescale, Eq. (25)
    uint32_t* err = nullptr;     // sticky device error word
    unsigned long long* cnt = nullptr;  // [n_problems][NCOUNT][CNT_SLOTS]
    unsigned long long* d_scalar = nullptr;  // small reduction results
    // element-pass scratch for elements too large for on-chip memory, [cap] each
    double* gkey = nullptr;      // 2 doubles per particle (key, pid bits)
    int32_t* gord = nullptr;     // 2 ints per particle
    double* gu3 = nullptr;       // 3 velocity components + pid per particle (4 doubles)
    // number control
    int32_t* ctl_clone = nullptr;   // [ne]
    int32_t* ctl_off = nullptr;     // [ne+1]
    unsigned long long* ctl_rep = nullptr;  // merged, empty, below, above
    // timing
    bool timing = false;
    std::vector<std::pair<int, std::pair<hipEvent_t, hipEvent_t>>> events;
    double t_ms[pdfgpu::T_N] = {0};
    int64_t t_n[pdfgpu::T_N] = {0};
    int lds_max = 0;            // particles per element on chip in the workgroup kernel
    int ppl = 4;                // particles per lane in the wavefront kernel
    int adv_block = 64;         // threads per workgroup of the particle loop
    // statistics feedback after every step
    bool fb_on = false;
    double fb_alpha = 1.0;
    int32_t fb_rey = 0;
    double* fb_gn = nullptr;    // [nn][6]
    double* fb_h = nullptr;     // [ne][6]
    // graph-captured steps
    bool use_graph = false;
    bool capturing = false;    // a step is being captured into a graph
    hipStream_t gstream = nullptr;
    hipEvent_t gev[2] = {nullptr, nullptr};
    hipGraphExec_t gexec[2] = {nullptr, nullptr};   // two steps starting from buffer 0 / 1
    int64_t g_nub[2] = {-1, -1};
    std::vector<double> g_dt[2];
    int32_t* big_list = nullptr;    // [ne] elements left to the workgroup kernel
    int32_t* big_count = nullptr;   // [4] large elements, no-slip resamples, wavefronts of several problems,
                                    // particles for the full particle loop
    int32_t* wave_list = nullptr;   // [cap / 64 + 2] wavefronts of several problems (batched ensembles)
    int ppl_min = 1;                // wavefront capacity suggested by the smallest set-up count
    std::vector<int> tiers;         // particles per lane of the wavefront tiers, ascending
    bool ctl_valid = false;     // the current buffer holds the canonical order of a pass
    bool any_proj = false;      // some problem conditions by Fox's projection
    bool wp_full = false;       // the nodal wp field has nine components (stored by the solve)
    FemState fem;
    int32_t* redist_plan = nullptr;  // [redist_cap][4] moves of the last redistribution
    int64_t redist_cap = 0;
};
