// Kernel argument blocks and launchers of libpdfgpu.
//
// Every particle kernel is instantiated for the two forms of the state:
//   R = double  FP64 form: everything in FP64;
//   R = float   mixed form: velocity, frequency, scalar and weight (and their updates,
//               the nodal fields they use and the nodal sums) in FP32; positions, the
//               barycentric locate / reflect tests and the final nodal division in FP64.
// An ensemble may hold several independent problems (the batched form): their grids are
// concatenated, every element record carries its problem index, and per-problem
// parameters sit in a small device table.
#pragma once
#include "pdf_impl.h"

namespace pdfgpu {

constexpr int EP_NT = 256;      // threads per element in the element pass
constexpr int MAXBINS = 1024;   // upper bound of bins[0]*bins[1]*bins[2]
constexpr int EP_BIG_BLOCKS = 512;  // workgroups of the large-element pass

template <class R>
struct AdvanceArgs {
    SoaT<R> s;
    const ElemGeo* geo;
    const R* node;              // [nn][NODE_STRIDE] in the state's precision
    const int64_t* n2e_ptr;
    const int32_t* n2e;
    int32_t* counts;
    uint32_t* err;
    unsigned long long* cnt;    // [problem][NCOUNT][CNT_SLOTS]
    const int64_t* meta;        // [0] used slots, [4] step counter
    int32_t* arrival;           // [cap] rank of each particle among its new host's arrivals
    int32_t* wall_list;         // [cap] slots that take a new frequency (no-slip events)
    int32_t* wall_count;
    int32_t* wave_list;         // [wave_cap] wavefronts whose lanes hold several problems
    int32_t* wave_count;
    int64_t wave_cap;
    int32_t* redo_list;         // [cap] slots for the full particle loop (walks that reach a wall)
    int32_t* redo_count;
    int64_t ne;
    ProbParams p0;              // parameters of problem 0 (single-problem ensembles)
    const ProbParams* prm;      // [n_problems] (batched ensembles)
};

template <class R>
struct ElementArgs {
    SoaT<R> in, out;
    const int32_t* start;
    const int32_t* idx;
    const ElemGeo* geo;
    const ProbParams* prm;
    const R* shift;
    R* part;
    const double* tm;
    int32_t mix;          // 0: binning and statistics only (set-up, import)
    int64_t ne;
    int64_t cap;
    int32_t lds_max;
    int32_t* big_list;    // [ne] elements left to the workgroup kernel
    int32_t* big_count;
    double* gkey;
    int32_t* gord;
    double* gu3;
    int32_t any_proj;     // some problem conditions by Fox's projection
};

template <class R>
struct NodeArgs {
    const R* part;
    const int64_t* n2e_ptr;
    const int32_t* n2e;
    R* shift;
    double* stats;
    int64_t nn;
    const int32_t* start;
    int64_t ne;
    int64_t* meta;
    int32_t* big_count;     // [2] large-element worklist, no-slip resample list
    int32_t advance_step;   // 1 after a time step: the device step counter moves on
    int32_t estimator;      // 1: element means and moments averaged over the elements around
                            //    the node (then part holds W, sums and shift per element)
};

template <class R>
struct InitArgs {
    SoaT<R> s;
    const ElemGeo* geo;
    const R* node;
    const ProbParams* prm;
    int32_t n_problems;
    int64_t n;
};

template <class R>
struct ControlArgs {
    SoaT<R> s;
    const int32_t* start;
    const ElemGeo* geo;
    ProbParams* prm;
    int32_t n_problems;
    int32_t* clone;
    const int32_t* off;
    unsigned long long* rep;
    uint32_t* err;
    const int64_t* nslots;
    int64_t ne, cap;
    int32_t n_min, n_max;
};

// wp_full: the nodal wp field has nine components (else symmetric: six are read)
template <class R>
void launch_advance(const AdvanceArgs<R>& a, int64_t n_ub, bool batched, bool wp_full, int block, hipStream_t s);
// wavefront tiers of increasing capacity 64 x tiers[t], then the workgroup kernel
template <class R>
void launch_element_pass(const ElementArgs<R>& a, const int* tiers, int n_tiers, hipStream_t s);
template <class R>
hipError_t prepare_element_pass(int lds_max);
template <class R>
size_t element_pass_smem(int lds_max);
template <class R>
void launch_node_finalize(const NodeArgs<R>& a, hipStream_t s);
template <class R>
void launch_init(const InitArgs<R>& a, hipStream_t s);
template <class R>
void launch_ctl_plan(const ControlArgs<R>& a, hipStream_t s);
template <class R>
void launch_ctl_apply(const ControlArgs<R>& a, hipStream_t s);
template <class R>
void launch_shift_init(const R* node, int64_t nn, R* shift, hipStream_t s);
// redistribution moves (App. B): plan [m][4] = destination slot, position source (slot or
// -(e + 1): centroid of element e), property source slot, new element; stage holds m
// entries of scratch state
template <class R>
void launch_redistribute(const SoaT<R>& st, const SoaT<R>& stage, const int32_t* plan, const ElemGeo* geo, int64_t m,
                         hipStream_t s);

void launch_count(const int32_t* elem, const int64_t* nslots, int64_t n_ub, int64_t ne, int32_t* counts,
                  uint32_t* err, hipStream_t s);
void launch_count_range(const int32_t* elem, const int64_t* nslots, int64_t n_ub, int32_t lo, int32_t hi,
                        unsigned long long* out, hipStream_t s);
int64_t scan_blocks(int64_t n);
int64_t scan_max_elems();
void launch_scan(const int32_t* in, int64_t n, int32_t* out, int32_t* tmp, hipStream_t s);
void launch_scatter(const int32_t* elem, const int64_t* nslots, int64_t n_ub, int64_t ne, int32_t* counts,
                    const int32_t* start, int32_t* idx, uint32_t* err, hipStream_t s);
// idx[start[elem[i]] + arrival[i]] = i for the used slots (arrival ranks from the particle loop)
void launch_place(const int32_t* elem, const int32_t* arrival, const int64_t* nslots, int64_t n_ub, int64_t ne,
                  const int32_t* start, int32_t* idx, uint32_t* err, hipStream_t s);
void launch_tm(const ElemGeo* geo, const double* node, int64_t ne, const ProbParams* prm, double* tm,
               hipStream_t s);
void launch_ctl_finish(int64_t* meta, const int32_t* off, int64_t ne, const unsigned long long* rep, int64_t cap,
                       ProbParams* prm, int32_t n_problems, hipStream_t s);
// statistics feedback: nodal <U> (scaled by alpha) and optionally R from the statistics,
// then element gradients and nodal Laplacians of <U>; gn [6 nn] and h [6 ne] are scratch
void launch_feedback(const double* stats, double* node, ElemGeo* geo, const int64_t* n2e_ptr, const int32_t* n2e,
                     int64_t nn, int64_t ne, double alpha, int32_t rey, double* gn, double* h, hipStream_t s);
// Eq. (26) ingredients over nodes [n0, n0 + nn): out[0] = min sqrt(A_n), out[1] = max |<Z>_n|
// as double bits; out must hold +inf and 0 on entry
void launch_cfl(const ElemGeo* geo, const int64_t* n2e_ptr, const int32_t* n2e, const double* stats, int64_t n0,
                int64_t nn, unsigned long long* out, hipStream_t s);
void launch_fill_i32(int32_t* p, int64_t n, int32_t v, hipStream_t s);
void launch_fill_u64(unsigned long long* p, int64_t n, unsigned long long v, hipStream_t s);
void launch_f64_to_f32(const double* in, float* out, int64_t n, hipStream_t s);
void launch_f32_to_f64(const float* in, double* out, int64_t n, hipStream_t s);

}  // namespace pdfgpu
