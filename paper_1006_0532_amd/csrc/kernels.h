// Kernel argument blocks and launchers of libpdfgpu.
#pragma once
#include "pdf_impl.h"

namespace pdfgpu {

constexpr int EP_NT = 256;      // threads per element in the element pass
constexpr int MAXBINS = 1024;   // upper bound of bins[0]*bins[1]*bins[2]
constexpr int EP_BIG_BLOCKS = 512;  // workgroups of the large-element pass

struct AdvanceArgs {
    Soa s;
    const ElemGeo* geo;
    const double* node;
    const int64_t* n2e_ptr;
    const int32_t* n2e;
    int32_t* counts;
    uint32_t* err;
    unsigned long long* cnt;
    const int64_t* nslots;
    int64_t ne;
    double period;
    ModelC m;
    double dt;
    RngKey key;
    uint32_t step;
    double src_x, src_y, src_r2;
    int32_t src_cont;
};

struct ElementArgs {
    Soa in, out;
    const int32_t* start;
    const int32_t* idx;
    const ElemGeo* geo;
    const double* shift;
    double* part;
    const double* tm;
    double dt;
    int64_t ne;
    int64_t cap;
    int32_t bins0, bins1, bins2, minpb;
    int32_t lds_max;
    int32_t ppl;          // particles per lane of the wavefront kernel (1..6, 8)
    int32_t* big_list;    // [ne] elements left to the workgroup kernel
    int32_t* big_count;
    double* gkey;
    int32_t* gord;
    double* gu3;
};

struct NodeArgs {
    const double* part;
    const int64_t* n2e_ptr;
    const int32_t* n2e;
    double* shift;
    double* stats;
    int64_t nn;
    const int32_t* start;
    int64_t ne;
    int64_t* meta;
    int32_t* big_count;
};

struct InitArgs {
    Soa s;
    const ElemGeo* geo;
    const double* node;
    int64_t n;
    int32_t ppe;
    RngKey key;
    double u_sigma, omega_shape;
    double src_x, src_y, src_r2;
    double period;
};

struct ControlArgs {
    Soa s;
    const int32_t* start;
    int32_t* clone;
    const int32_t* off;
    unsigned long long* rep;
    uint32_t* err;
    const int64_t* nslots;
    int64_t ne, cap;
    int32_t n_min, n_max;
    int32_t bins0, bins1, bins2, minpb;
    uint64_t next_pid;
};

void launch_advance(const AdvanceArgs& a, int64_t n_ub, hipStream_t s);
void launch_count(const int32_t* elem, const int64_t* nslots, int64_t n_ub, int64_t ne, int32_t* counts,
                  uint32_t* err, hipStream_t s);
int64_t scan_blocks(int64_t n);
int64_t scan_max_elems();
void launch_scan(const int32_t* in, int64_t n, int32_t* out, int32_t* tmp, hipStream_t s);
void launch_scatter(const int32_t* elem, const int64_t* nslots, int64_t n_ub, int64_t ne, int32_t* counts,
                    const int32_t* start, int32_t* idx, uint32_t* err, hipStream_t s);
hipError_t prepare_element_pass(int lds_max);
size_t element_pass_smem(int lds_max);
void launch_element_pass(const ElementArgs& a, hipStream_t s);
void launch_node_finalize(const NodeArgs& a, hipStream_t s);
void launch_init(const InitArgs& a, hipStream_t s);
void launch_tm(const ElemGeo* geo, const double* node, int64_t ne, ModelC m, double sx, double sy, double sr,
               double period, double* tm, hipStream_t s);
void launch_ctl_plan(const ControlArgs& a, hipStream_t s);
void launch_ctl_apply(const ControlArgs& a, hipStream_t s);
void launch_ctl_finish(int64_t* meta, const int32_t* off, int64_t ne, const unsigned long long* rep, int64_t cap,
                       hipStream_t s);
void launch_fill_i32(int32_t* p, int64_t n, int32_t v, hipStream_t s);
void launch_fill_u64(unsigned long long* p, int64_t n, unsigned long long v, hipStream_t s);
void launch_fill_f64(double* p, int64_t n, double v, hipStream_t s);
void launch_shift_init(const double* node, int64_t nn, double* shift, hipStream_t s);

}  // namespace pdfgpu
