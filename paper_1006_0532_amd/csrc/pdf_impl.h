// Internal types of libpdfgpu: device data layout and host-side handles.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
#include <vector>

#include "pdf.h"

namespace pdfgpu {

// Per-node field record, 22 doubles (176 B, 16-B aligned):
// grad<P>(2), wp(6), <U>(3), lap<U>(3), <omega>(1), R(6), pad(1)
constexpr int NODE_STRIDE = 22;
enum { NF_GP = 0, NF_WP = 2, NF_MU = 8, NF_LAP = 11, NF_OM = 14, NF_RE = 15 };

// Edge kinds after classification.
enum : uint8_t { KIND_INTERIOR = 0, KIND_WALL = 1, KIND_SLIP = 2, KIND_PERIODIC = 3 };

// Per-element record used by the particle kernels (176 B).
struct __attribute__((aligned(16))) ElemGeo {
    double x[3], y[3];  // vertices in the element's own frame (seam elements unwrapped)
    double area;        // A_e > 0
    double shift[3];    // x shift added when leaving through a periodic edge
    double gu[6];       // d<U1>/dx, d<U1>/dy, d<U2>/dx, d<U2>/dy, d<U3>/dx, d<U3>/dy
    double wl[4];       // wall line: point (x, y) and inward unit normal (x, y)
    int32_t node[3];
    int32_t nbr[3];     // -1 across a boundary edge
    uint8_t kind[3];
    uint8_t wall;       // element touches a no-slip wall by an edge or a node
    int32_t pad;
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

// Structure-of-arrays particle state in HBM (FP64 form).
struct Soa {
    double *x, *y, *u0, *u1, *u2, *om, *psi, *w;
    uint64_t* pid;
    int32_t* elem;  // host element; -1 = dead slot
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

struct pdf_ens_s {
    pdf_grid grid = nullptr;
    pdf_init_desc d{};
    int32_t problem = 0;
    hipStream_t stream = nullptr;
    int64_t cap = 0;
    int64_t n_slots_ub = 0;   // host-side upper bound of the used slots
    int64_t step = 0;
    uint64_t next_pid = 0;
    int cur = 0;              // which SoA buffer is current
    pdfgpu::Soa buf[2]{};
    int32_t* counts = nullptr;   // [ne] particles per element (zero between steps)
    int32_t* start = nullptr;    // [ne+1] segment starts of the current buffer
    int32_t* idx = nullptr;      // [cap] slot of each grouped particle
    int32_t* scan_tmp = nullptr; // block sums
    int64_t* d_meta = nullptr;   // [0] used slots, [1] report scratch...
    double* part = nullptr;      // [ne][3][NPART] per-vertex partial sums
    double* stats = nullptr;     // [nn][NSTAT]
    double* shift = nullptr;     // [nn][5] reference values of the single-pass moments
    double* tm = nullptr;        // [ne] micromixing timescale, Eq. (25)
    uint32_t* err = nullptr;     // sticky device error word
    unsigned long long* cnt = nullptr;  // [NCOUNT][CNT_SLOTS]
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
    int32_t* big_list = nullptr;
    int32_t* big_count = nullptr;
    bool ctl_valid = false;     // the current buffer holds the canonical order of a pass
};
