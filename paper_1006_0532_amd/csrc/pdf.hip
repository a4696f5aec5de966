// C ABI of libpdfgpu (include/pdf.h): argument checks, device memory, and the order of the
// kernel launches of one time step.  All arithmetic of the method runs in kernels.hip.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "kernels.h"
#include "pdf_impl.h"

using namespace pdfgpu;

namespace pdfgpu {
pdf_status build_grid(pdf_grid_s& g, const pdf_mesh_desc& m, const pdf_fields_desc& f);

static thread_local std::string g_last_error;
void set_error(const std::string& msg) { g_last_error = msg; }
}  // namespace pdfgpu

#define HIP_TRY(expr)                                                                              \
    do {                                                                                           \
        hipError_t _e = (expr);                                                                    \
        if (_e != hipSuccess) {                                                                    \
            set_error(std::string("HIP error at ") + #expr + ": " + hipGetErrorString(_e));      \
            return PDF_E_HIP;                                                                      \
        }                                                                                          \
    } while (0)

namespace {

template <class T>
pdf_status dalloc(T** p, int64_t count)
{
    *p = nullptr;
    if (count <= 0) count = 1;
    hipError_t e = hipMalloc((void**)p, sizeof(T) * (size_t)count);
    if (e != hipSuccess) {
        *p = nullptr;
        (void)hipGetLastError();
        set_error(std::string("device allocation of ") + std::to_string(sizeof(T) * count) + " bytes failed");
        return PDF_E_NOMEM;
    }
    return PDF_OK;
}

template <class T>
void dfree(T*& p)
{
    if (p) (void)hipFree((void*)p);
    p = nullptr;
}

// kernel timing with HIP events on the launch stream
struct Timed {
    pdf_ens_s* E;
    int id;
    hipStream_t s;
    hipEvent_t a = nullptr;
    Timed(pdf_ens_s* e, int i, hipStream_t st) : E(e), id(i), s(st)
    {
        if (E->timing && hipEventCreate(&a) == hipSuccess) (void)hipEventRecord(a, s);
    }
    ~Timed()
    {
        if (!E->timing || !a) return;
        hipEvent_t b = nullptr;
        if (hipEventCreate(&b) == hipSuccess) {
            (void)hipEventRecord(b, s);
            E->events.push_back({id, {a, b}});
        } else {
            (void)hipEventDestroy(a);
        }
    }
};

void collect_timing(pdf_ens_s* E)
{
    for (auto& ev : E->events) {
        float ms = 0.f;
        if (hipEventSynchronize(ev.second.second) == hipSuccess &&
            hipEventElapsedTime(&ms, ev.second.first, ev.second.second) == hipSuccess) {
            E->t_ms[ev.first] += ms;
            E->t_n[ev.first] += 1;
        }
        (void)hipEventDestroy(ev.second.first);
        (void)hipEventDestroy(ev.second.second);
    }
    E->events.clear();
}

hipStream_t as_stream(void* s) { return reinterpret_cast<hipStream_t>(s); }

pdf_status check_device_error(pdf_ens_s* E)
{
    uint32_t err = 0;
    HIP_TRY(hipMemcpy(&err, E->err, sizeof(uint32_t), hipMemcpyDeviceToHost));
    if (err == 0) return PDF_OK;
    if (err & ERR_LOST) { set_error("a particle could not be located (walk and fall-back failed)"); return PDF_E_LOST; }
    if (err & ERR_NONFINITE) { set_error("non-finite particle state"); return PDF_E_NONFINITE; }
    if (err & ERR_CAPACITY) { set_error("particle capacity exhausted"); return PDF_E_CAPACITY; }
    set_error("inconsistent element index in the particle state");
    return PDF_E_STATE;
}

Soa& cur(pdf_ens_s* E) { return E->buf[E->cur]; }

// group the particles of the current buffer by element, bin them, mix (dt > 0), write
// canonical order into the other buffer and reduce the statistics
pdf_status regroup(pdf_ens_s* E, double dt, bool counts_ready, hipStream_t s)
{
    pdf_grid_s* g = E->grid;
    Soa& in = cur(E);
    if (!counts_ready) {
        Timed t(E, T_COUNT, s);
        launch_count(in.elem, E->d_meta, E->n_slots_ub, g->ne, E->counts, E->err, s);
    }
    {
        Timed t(E, T_SCAN, s);
        launch_scan(E->counts, g->ne, E->start, E->scan_tmp, s);
    }
    {
        Timed t(E, T_SCATTER, s);
        launch_scatter(in.elem, E->d_meta, E->n_slots_ub, g->ne, E->counts, E->start, E->idx, E->err, s);
    }
    ElementArgs ea{};
    ea.in = in;
    ea.out = E->buf[1 - E->cur];
    ea.start = E->start;
    ea.idx = E->idx;
    ea.geo = g->d_geo;
    ea.shift = E->shift;
    ea.part = E->part;
    ea.tm = E->tm;
    ea.dt = dt;
    ea.ne = g->ne;
    ea.cap = E->cap;
    ea.bins0 = E->d.bins[0];
    ea.bins1 = E->d.bins[1];
    ea.bins2 = E->d.bins[2];
    ea.minpb = E->d.min_per_bin;
    ea.lds_max = E->lds_max;
    ea.ppl = E->ppl;
    ea.big_list = E->big_list;
    ea.big_count = E->big_count;
    ea.gkey = E->gkey;
    ea.gord = E->gord;
    ea.gu3 = E->gu3;
    {
        Timed t(E, T_ELEMENT, s);
        launch_element_pass(ea, s);
    }
    NodeArgs na{};
    na.part = E->part;
    na.n2e_ptr = g->d_n2e_ptr;
    na.n2e = g->d_n2e;
    na.shift = E->shift;
    na.stats = E->stats;
    na.nn = g->nn;
    na.start = E->start;
    na.ne = g->ne;
    na.meta = E->d_meta;
    na.big_count = E->big_count;
    {
        Timed t(E, T_NODE, s);
        launch_node_finalize(na, s);
    }
    E->cur = 1 - E->cur;
    HIP_TRY(hipGetLastError());
    return PDF_OK;
}

}  // namespace

extern "C" {

const char* pdf_last_error(void) { return g_last_error.c_str(); }

pdf_status pdf_grid_create(const pdf_mesh_desc* mesh, const pdf_fields_desc* fields, const pdf_model* model,
                           void* hip_stream, pdf_grid* out)
{
    if (!mesh || !fields || !model || !out) {
        set_error("pdf_grid_create: null argument");
        return PDF_E_INVAL;
    }
    *out = nullptr;
    const pdf_model& m = *model;
    const double vals[9] = {m.nu, m.rho, m.C3, m.C4, m.CT, m.Cw1, m.Cw2, m.Cs, m.Ct};
    for (double v : vals)
        if (!std::isfinite(v)) { set_error("pdf_grid_create: non-finite model constant"); return PDF_E_INVAL; }
    if (!(m.nu >= 0.0) || !(m.rho > 0.0) || !(m.C4 > 0.0) || !(m.C4 <= 1.0) || !(m.C3 >= 0.0)) {
        set_error("pdf_grid_create: model constants out of range (nu >= 0, rho > 0, 0 < C4 <= 1)");
        return PDF_E_INVAL;
    }
    pdf_grid_s* g = new pdf_grid_s();
    g->model = ModelC{m.nu, m.rho, m.C3, m.C4, m.CT, m.Cw1, m.Cw2, m.Cs, m.Ct};
    pdf_status st = build_grid(*g, *mesh, *fields);
    if (st != PDF_OK) {
        delete g;
        return st;
    }
    hipStream_t s = as_stream(hip_stream);
    if (hipGetDevice(&g->device) != hipSuccess) {
        set_error("pdf_grid_create: no HIP device");
        delete g;
        return PDF_E_HIP;
    }
    st = dalloc(&g->d_geo, g->ne);
    if (st == PDF_OK) st = dalloc(&g->d_node, g->nn * NODE_STRIDE);
    if (st == PDF_OK) st = dalloc(&g->d_n2e_ptr, g->nn + 1);
    if (st == PDF_OK) st = dalloc(&g->d_n2e, 3 * g->ne);
    if (st != PDF_OK) {
        pdf_grid_destroy(g);
        return st;
    }
    hipError_t e = hipMemcpyAsync(g->d_geo, g->h_geo.data(), sizeof(ElemGeo) * g->ne, hipMemcpyHostToDevice, s);
    if (e == hipSuccess)
        e = hipMemcpyAsync(g->d_node, g->h_node.data(), sizeof(double) * g->nn * NODE_STRIDE, hipMemcpyHostToDevice, s);
    if (e == hipSuccess)
        e = hipMemcpyAsync(g->d_n2e_ptr, g->h_n2e_ptr.data(), sizeof(int64_t) * (g->nn + 1), hipMemcpyHostToDevice, s);
    if (e == hipSuccess)
        e = hipMemcpyAsync(g->d_n2e, g->h_n2e.data(), sizeof(int32_t) * 3 * g->ne, hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) {
        set_error(std::string("pdf_grid_create: ") + hipGetErrorString(e));
        pdf_grid_destroy(g);
        return PDF_E_HIP;
    }
    *out = g;
    return PDF_OK;
}

pdf_status pdf_grid_destroy(pdf_grid g)
{
    if (!g) return PDF_OK;
    dfree(g->d_geo);
    dfree(g->d_node);
    dfree(g->d_n2e_ptr);
    dfree(g->d_n2e);
    delete g;
    return PDF_OK;
}

pdf_status pdf_ens_destroy(pdf_ens E)
{
    if (!E) return PDF_OK;
    (void)hipDeviceSynchronize();
    for (auto& ev : E->events) {
        (void)hipEventDestroy(ev.second.first);
        (void)hipEventDestroy(ev.second.second);
    }
    for (int b = 0; b < 2; ++b) {
        Soa& S = E->buf[b];
        dfree(S.x); dfree(S.y); dfree(S.u0); dfree(S.u1); dfree(S.u2); dfree(S.om); dfree(S.psi); dfree(S.w);
        dfree(S.pid); dfree(S.elem);
    }
    dfree(E->counts); dfree(E->start); dfree(E->idx); dfree(E->scan_tmp); dfree(E->d_meta); dfree(E->part);
    dfree(E->stats); dfree(E->shift); dfree(E->tm); dfree(E->err); dfree(E->cnt); dfree(E->gkey); dfree(E->gord);
    dfree(E->gu3); dfree(E->ctl_clone); dfree(E->ctl_off); dfree(E->ctl_rep); dfree(E->big_list);
    dfree(E->big_count);
    delete E;
    return PDF_OK;
}

pdf_status pdf_particles_init(const pdf_grid* grids, const pdf_init_desc* descs, int32_t n_problems,
                              void* hip_stream, pdf_ens* out)
{
    if (!grids || !descs || !out || !grids[0]) {
        set_error("pdf_particles_init: null argument");
        return PDF_E_INVAL;
    }
    *out = nullptr;
    if (n_problems != 1) {
        set_error("pdf_particles_init: n_problems must be 1");
        return PDF_E_INVAL;
    }
    const pdf_init_desc& d = descs[0];
    pdf_grid_s* g = grids[0];
    const int64_t nb = (int64_t)d.bins[0] * d.bins[1] * d.bins[2];
    if (d.ppe < 0 || d.bins[0] < 1 || d.bins[1] < 1 || d.bins[2] < 1 || nb > MAXBINS || d.min_per_bin < 1 ||
        !(d.omega_shape >= 1.0) || !(d.u_sigma >= 0.0) || !(d.src_r >= 0.0) || !std::isfinite(d.u_sigma) ||
        !std::isfinite(d.omega_shape) || !std::isfinite(d.src_x) || !std::isfinite(d.src_y) ||
        !std::isfinite(d.src_r) || d.precision != 0 || d.capacity < 0) {
        set_error("pdf_particles_init: invalid descriptor (bins product <= 1024, omega_shape >= 1, precision 0)");
        return PDF_E_INVAL;
    }
    if (g->ne > scan_max_elems()) {
        set_error("pdf_particles_init: too many elements for the segment scan");
        return PDF_E_INVAL;
    }
    const int64_t n0 = g->ne * (int64_t)d.ppe;
    int64_t cap = d.capacity > 0 ? d.capacity : std::max<int64_t>(2 * n0, 1024);
    if (cap < n0) {
        set_error("pdf_particles_init: capacity below the initial particle count");
        return PDF_E_CAPACITY;
    }
    if (cap > (int64_t)INT32_MAX - 1) {
        set_error("pdf_particles_init: capacity above 2^31 - 2 slots");
        return PDF_E_INVAL;
    }
    HIP_TRY(hipSetDevice(g->device));
    hipStream_t s = as_stream(hip_stream);
    pdf_ens_s* E = new pdf_ens_s();
    E->grid = g;
    E->d = d;
    E->cap = cap;
    E->stream = s;
    E->next_pid = (uint64_t)n0;
    pdf_status st = PDF_OK;
    for (int b = 0; b < 2 && st == PDF_OK; ++b) {
        Soa& S = E->buf[b];
        st = dalloc(&S.x, cap);
        if (st == PDF_OK) st = dalloc(&S.y, cap);
        if (st == PDF_OK) st = dalloc(&S.u0, cap);
        if (st == PDF_OK) st = dalloc(&S.u1, cap);
        if (st == PDF_OK) st = dalloc(&S.u2, cap);
        if (st == PDF_OK) st = dalloc(&S.om, cap);
        if (st == PDF_OK) st = dalloc(&S.psi, cap);
        if (st == PDF_OK) st = dalloc(&S.w, cap);
        if (st == PDF_OK) st = dalloc(&S.pid, cap);
        if (st == PDF_OK) st = dalloc(&S.elem, cap);
    }
    if (st == PDF_OK) st = dalloc(&E->counts, g->ne);
    if (st == PDF_OK) st = dalloc(&E->start, g->ne + 1);
    if (st == PDF_OK) st = dalloc(&E->idx, cap);
    if (st == PDF_OK) st = dalloc(&E->scan_tmp, scan_blocks(g->ne) + 1);
    if (st == PDF_OK) st = dalloc(&E->d_meta, 8);
    if (st == PDF_OK) st = dalloc(&E->part, g->ne * 3 * NPART);
    if (st == PDF_OK) st = dalloc(&E->stats, g->nn * NSTAT);
    if (st == PDF_OK) st = dalloc(&E->shift, g->nn * 5);
    if (st == PDF_OK) st = dalloc(&E->tm, g->ne);
    if (st == PDF_OK) st = dalloc(&E->err, 1);
    if (st == PDF_OK) st = dalloc(&E->cnt, NCOUNT * CNT_SLOTS);
    if (st == PDF_OK) st = dalloc(&E->gkey, 2 * cap);
    if (st == PDF_OK) st = dalloc(&E->gord, 2 * cap);
    if (st == PDF_OK) st = dalloc(&E->gu3, 4 * cap);
    if (st == PDF_OK) st = dalloc(&E->ctl_clone, g->ne);
    if (st == PDF_OK) st = dalloc(&E->ctl_off, g->ne + 1);
    if (st == PDF_OK) st = dalloc(&E->ctl_rep, 4);
    if (st == PDF_OK) st = dalloc(&E->big_list, g->ne);
    if (st == PDF_OK) st = dalloc(&E->big_count, 1);
    if (st != PDF_OK) {
        pdf_ens_destroy(E);
        return st;
    }
    // element pass: a wavefront per element holds up to 64 * ppl particles (ppl from the
    // set-up count with 30 % headroom); larger elements go to the workgroup kernel, whose
    // on-chip path takes up to lds_max particles within 64 KiB of LDS
    E->ppl = (int)std::min<int64_t>(8, std::max<int64_t>(1, (13 * (int64_t)d.ppe + 639) / 640));
    if (E->ppl == 7) E->ppl = 8;
    {
        const int fixed = (int)element_pass_smem(0);
        const int per = (int)element_pass_smem(1) - fixed;
        E->lds_max = std::max(64, (65536 - fixed) / per);
        HIP_TRY(prepare_element_pass(E->lds_max));
    }
    launch_fill_i32(E->counts, g->ne, 0, s);
    launch_fill_i32(E->big_count, 1, 0, s);
    launch_fill_i32(E->idx, cap, 0, s);
    launch_fill_u64(E->cnt, NCOUNT * CNT_SLOTS, 0ull, s);
    launch_fill_i32(reinterpret_cast<int32_t*>(E->err), 1, 0, s);
    launch_fill_i32(E->buf[0].elem, cap, -1, s);
    launch_fill_i32(E->buf[1].elem, cap, -1, s);
    std::vector<int64_t> meta(8, 0);
    meta[0] = n0;
    meta[1] = n0;
    HIP_TRY(hipMemcpyAsync(E->d_meta, meta.data(), sizeof(int64_t) * 8, hipMemcpyHostToDevice, s));
    E->n_slots_ub = n0;
    launch_shift_init(g->d_node, g->nn, E->shift, s);
    launch_tm(g->d_geo, g->d_node, g->ne, g->model, d.src_x, d.src_y, d.src_r, g->period, E->tm, s);
    InitArgs ia{};
    ia.s = E->buf[0];
    ia.geo = g->d_geo;
    ia.node = g->d_node;
    ia.n = n0;
    ia.ppe = d.ppe;
    ia.key = RngKey{(uint32_t)d.seed, (uint32_t)(d.seed >> 32) ^ (uint32_t)E->problem};
    ia.u_sigma = d.u_sigma;
    ia.omega_shape = d.omega_shape;
    ia.src_x = d.src_x;
    ia.src_y = d.src_y;
    ia.src_r2 = d.src_r * d.src_r;
    ia.period = g->period;
    E->cur = 0;
    {
        Timed t(E, T_INIT, s);
        launch_init(ia, s);
    }
    HIP_TRY(hipGetLastError());
    st = regroup(E, 0.0, false, s);
    if (st != PDF_OK) {
        pdf_ens_destroy(E);
        return st;
    }
    E->n_slots_ub = n0;
    E->ctl_valid = true;
    HIP_TRY(hipStreamSynchronize(s));
    st = check_device_error(E);
    if (st != PDF_OK) {
        pdf_ens_destroy(E);
        return st;
    }
    *out = E;
    return PDF_OK;
}

pdf_status pdf_step(pdf_ens E, const double* dt, int32_t n_steps, void* hip_stream)
{
    if (!E || !dt || n_steps < 0) {
        set_error("pdf_step: invalid argument");
        return PDF_E_INVAL;
    }
    const double h = dt[0];
    if (!(h > 0.0) || !std::isfinite(h)) {
        set_error("pdf_step: dt must be positive and finite");
        return PDF_E_INVAL;
    }
    pdf_grid_s* g = E->grid;
    HIP_TRY(hipSetDevice(g->device));
    hipStream_t s = as_stream(hip_stream);
    E->stream = s;
    for (int32_t it = 0; it < n_steps; ++it) {
        AdvanceArgs a{};
        a.s = cur(E);
        a.geo = g->d_geo;
        a.node = g->d_node;
        a.n2e_ptr = g->d_n2e_ptr;
        a.n2e = g->d_n2e;
        a.counts = E->counts;
        a.err = E->err;
        a.cnt = E->cnt;
        a.nslots = E->d_meta;
        a.ne = g->ne;
        a.period = g->period;
        a.m = g->model;
        a.dt = h;
        a.key = RngKey{(uint32_t)E->d.seed, (uint32_t)(E->d.seed >> 32) ^ (uint32_t)E->problem};
        a.step = (uint32_t)E->step;
        a.src_x = E->d.src_x;
        a.src_y = E->d.src_y;
        a.src_r2 = E->d.src_r * E->d.src_r;
        a.src_cont = E->d.src_continuous;
        {
            Timed t(E, T_ADVANCE, s);
            launch_advance(a, E->n_slots_ub, s);
        }
        HIP_TRY(hipGetLastError());
        pdf_status st = regroup(E, h, true, s);
        if (st != PDF_OK) return st;
        E->step += 1;
    }
    E->ctl_valid = true;   // canonical order of the last element pass
    return PDF_OK;
}

pdf_status pdf_sync(pdf_ens E)
{
    if (!E) {
        set_error("pdf_sync: null ensemble");
        return PDF_E_INVAL;
    }
    HIP_TRY(hipSetDevice(E->grid->device));
    HIP_TRY(hipStreamSynchronize(E->stream));
    return check_device_error(E);
}

pdf_status pdf_stats(pdf_ens E, int32_t problem, double* out, int32_t out_is_device, void* hip_stream)
{
    if (!E || !out || problem != 0) {
        set_error("pdf_stats: invalid argument");
        return PDF_E_INVAL;
    }
    HIP_TRY(hipSetDevice(E->grid->device));
    hipStream_t s = as_stream(hip_stream);
    const size_t bytes = sizeof(double) * (size_t)E->grid->nn * NSTAT;
    if (out_is_device) {
        HIP_TRY(hipMemcpyAsync(out, E->stats, bytes, hipMemcpyDeviceToDevice, s));
        return PDF_OK;
    }
    HIP_TRY(hipMemcpyAsync(out, E->stats, bytes, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    return check_device_error(E);
}

pdf_status pdf_count(pdf_ens E, int32_t problem, int64_t* live)
{
    if (!E || !live || problem != 0) {
        set_error("pdf_count: invalid argument");
        return PDF_E_INVAL;
    }
    HIP_TRY(hipSetDevice(E->grid->device));
    HIP_TRY(hipStreamSynchronize(E->stream));
    int64_t meta[2];
    HIP_TRY(hipMemcpy(meta, E->d_meta, sizeof(meta), hipMemcpyDeviceToHost));
    *live = meta[1];
    return check_device_error(E);
}

pdf_status pdf_control(pdf_ens E, int32_t n_min, int32_t n_max, pdf_control_report* report, void* hip_stream)
{
    if (!E || n_min < 0 || n_max < 1 || n_max < n_min) {
        set_error("pdf_control: need 0 <= n_min <= n_max and n_max >= 1");
        return PDF_E_INVAL;
    }
    pdf_grid_s* g = E->grid;
    HIP_TRY(hipSetDevice(g->device));
    hipStream_t s = as_stream(hip_stream);
    E->stream = s;
    if (!E->ctl_valid) {
        set_error("pdf_control: no element pass since the last control");
        return PDF_E_STATE;
    }
    launch_fill_u64(E->ctl_rep, 4, 0ull, s);
    ControlArgs c{};
    c.s = cur(E);
    c.start = E->start;
    c.clone = E->ctl_clone;
    c.off = E->ctl_off;
    c.rep = E->ctl_rep;
    c.err = E->err;
    c.nslots = E->d_meta;
    c.ne = g->ne;
    c.cap = E->cap;
    c.n_min = n_min;
    c.n_max = n_max;
    c.bins0 = E->d.bins[0];
    c.bins1 = E->d.bins[1];
    c.bins2 = E->d.bins[2];
    c.minpb = E->d.min_per_bin;
    c.next_pid = E->next_pid;
    {
        Timed t(E, T_CPLAN, s);
        launch_ctl_plan(c, s);
    }
    {
        Timed t(E, T_CSCAN, s);
        launch_scan(E->ctl_clone, g->ne, E->ctl_off, E->scan_tmp, s);
    }
    {
        Timed t(E, T_CAPPLY, s);
        launch_ctl_apply(c, s);
        launch_ctl_finish(E->d_meta, E->ctl_off, g->ne, E->ctl_rep, E->cap, s);
    }
    HIP_TRY(hipGetLastError());
    int64_t meta[3];
    unsigned long long rep[4];
    HIP_TRY(hipMemcpyAsync(meta, E->d_meta, sizeof(meta), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipMemcpyAsync(rep, E->ctl_rep, sizeof(rep), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    E->n_slots_ub = meta[0];
    E->next_pid += (uint64_t)meta[2];
    E->ctl_valid = false;
    if (report) {
        report->live = meta[1];
        report->cloned = meta[2];
        report->merged = (int64_t)rep[0];
        report->empty = (int64_t)rep[1];
        report->below = (int64_t)rep[2];
        report->above = (int64_t)rep[3];
    }
    return check_device_error(E);
}

pdf_status pdf_particles_export(pdf_ens E, int32_t problem, int64_t cap, double* x, double* y, double* u,
                                double* omega, double* psi, double* w, uint64_t* pid, int32_t* elem, int64_t* n_out,
                                void* hip_stream)
{
    if (!E || problem != 0 || cap < 0) {
        set_error("pdf_particles_export: invalid argument");
        return PDF_E_INVAL;
    }
    HIP_TRY(hipSetDevice(E->grid->device));
    hipStream_t s = as_stream(hip_stream);
    HIP_TRY(hipStreamSynchronize(s));
    HIP_TRY(hipStreamSynchronize(E->stream));
    int64_t meta[2];
    HIP_TRY(hipMemcpy(meta, E->d_meta, sizeof(meta), hipMemcpyDeviceToHost));
    const int64_t ns = meta[0];
    Soa& S = cur(E);
    std::vector<int32_t> el(ns);
    HIP_TRY(hipMemcpy(el.data(), S.elem, sizeof(int32_t) * ns, hipMemcpyDeviceToHost));
    int64_t live = 0;
    for (int64_t i = 0; i < ns; ++i) live += el[i] >= 0 ? 1 : 0;
    if (n_out) *n_out = live;
    if (live > cap) {
        set_error("pdf_particles_export: output capacity too small");
        return PDF_E_CAPACITY;
    }
    std::vector<double> tmp(ns);
    auto pull = [&](const double* src, double* dst, int stride, int comp) -> pdf_status {
        if (!dst) return PDF_OK;
        HIP_TRY(hipMemcpy(tmp.data(), src, sizeof(double) * ns, hipMemcpyDeviceToHost));
        int64_t j = 0;
        for (int64_t i = 0; i < ns; ++i)
            if (el[i] >= 0) dst[stride * (j++) + comp] = tmp[i];
        return PDF_OK;
    };
    pdf_status st;
    if ((st = pull(S.x, x, 1, 0)) != PDF_OK) return st;
    if ((st = pull(S.y, y, 1, 0)) != PDF_OK) return st;
    if ((st = pull(S.u0, u, 3, 0)) != PDF_OK) return st;
    if ((st = pull(S.u1, u, 3, 1)) != PDF_OK) return st;
    if ((st = pull(S.u2, u, 3, 2)) != PDF_OK) return st;
    if ((st = pull(S.om, omega, 1, 0)) != PDF_OK) return st;
    if ((st = pull(S.psi, psi, 1, 0)) != PDF_OK) return st;
    if ((st = pull(S.w, w, 1, 0)) != PDF_OK) return st;
    if (pid) {
        std::vector<uint64_t> t(ns);
        HIP_TRY(hipMemcpy(t.data(), S.pid, sizeof(uint64_t) * ns, hipMemcpyDeviceToHost));
        int64_t j = 0;
        for (int64_t i = 0; i < ns; ++i)
            if (el[i] >= 0) pid[j++] = t[i];
    }
    if (elem) {
        int64_t j = 0;
        for (int64_t i = 0; i < ns; ++i)
            if (el[i] >= 0) elem[j++] = el[i];
    }
    return check_device_error(E);
}

pdf_status pdf_particles_import(pdf_ens E, int32_t problem, int64_t n, const double* x, const double* y,
                                const double* u, const double* omega, const double* psi, const double* w,
                                const uint64_t* pid, const int32_t* elem, int64_t step, uint64_t next_pid,
                                void* hip_stream)
{
    if (!E || problem != 0 || n < 0 || step < 0 || (n > 0 && (!x || !y || !u || !omega || !psi || !w || !pid || !elem))) {
        set_error("pdf_particles_import: invalid argument");
        return PDF_E_INVAL;
    }
    if (n > E->cap) {
        set_error("pdf_particles_import: more particles than capacity");
        return PDF_E_CAPACITY;
    }
    pdf_grid_s* g = E->grid;
    for (int64_t i = 0; i < n; ++i)
        if (elem[i] < 0 || elem[i] >= g->ne) {
            set_error("pdf_particles_import: element index out of range");
            return PDF_E_INVAL;
        }
    {
        std::vector<uint64_t> ids(pid, pid + n);
        std::sort(ids.begin(), ids.end());
        if (std::adjacent_find(ids.begin(), ids.end()) != ids.end()) {
            set_error("pdf_particles_import: particle ids must be unique");
            return PDF_E_INVAL;
        }
        if (n > 0 && next_pid <= ids.back()) {
            set_error("pdf_particles_import: next_pid must exceed every particle id");
            return PDF_E_INVAL;
        }
    }
    for (int64_t i = 0; i < n; ++i)
        if (!(std::isfinite(x[i]) && std::isfinite(y[i]) && std::isfinite(u[3 * i]) && std::isfinite(u[3 * i + 1]) &&
              std::isfinite(u[3 * i + 2]) && std::isfinite(omega[i]) && std::isfinite(psi[i]) && std::isfinite(w[i]))) {
            set_error("pdf_particles_import: non-finite particle state");
            return PDF_E_NONFINITE;
        }
    HIP_TRY(hipSetDevice(g->device));
    hipStream_t s = as_stream(hip_stream);
    E->stream = s;
    HIP_TRY(hipStreamSynchronize(s));
    Soa& S = cur(E);
    launch_fill_i32(S.elem, E->cap, -1, s);
    if (n > 0) {
        std::vector<double> c(n);
        for (int comp = 0; comp < 3; ++comp) {
            for (int64_t i = 0; i < n; ++i) c[i] = u[3 * i + comp];
            double* dst = comp == 0 ? S.u0 : (comp == 1 ? S.u1 : S.u2);
            HIP_TRY(hipMemcpyAsync(dst, c.data(), sizeof(double) * n, hipMemcpyHostToDevice, s));
            HIP_TRY(hipStreamSynchronize(s));
        }
        HIP_TRY(hipMemcpyAsync(S.x, x, sizeof(double) * n, hipMemcpyHostToDevice, s));
        HIP_TRY(hipMemcpyAsync(S.y, y, sizeof(double) * n, hipMemcpyHostToDevice, s));
        HIP_TRY(hipMemcpyAsync(S.om, omega, sizeof(double) * n, hipMemcpyHostToDevice, s));
        HIP_TRY(hipMemcpyAsync(S.psi, psi, sizeof(double) * n, hipMemcpyHostToDevice, s));
        HIP_TRY(hipMemcpyAsync(S.w, w, sizeof(double) * n, hipMemcpyHostToDevice, s));
        HIP_TRY(hipMemcpyAsync(S.pid, pid, sizeof(uint64_t) * n, hipMemcpyHostToDevice, s));
        HIP_TRY(hipMemcpyAsync(S.elem, elem, sizeof(int32_t) * n, hipMemcpyHostToDevice, s));
    }
    int64_t meta[2] = {n, n};
    HIP_TRY(hipMemcpyAsync(E->d_meta, meta, sizeof(meta), hipMemcpyHostToDevice, s));
    launch_fill_i32(E->counts, g->ne, 0, s);
    E->n_slots_ub = n;
    E->step = step;
    E->next_pid = next_pid;
    pdf_status st = regroup(E, 0.0, false, s);
    if (st != PDF_OK) return st;
    E->ctl_valid = true;
    HIP_TRY(hipStreamSynchronize(s));
    return check_device_error(E);
}

pdf_status pdf_counters(pdf_ens E, int32_t problem, int64_t out[PDF_NCOUNTERS])
{
    if (!E || !out || problem != 0) {
        set_error("pdf_counters: invalid argument");
        return PDF_E_INVAL;
    }
    HIP_TRY(hipSetDevice(E->grid->device));
    HIP_TRY(hipStreamSynchronize(E->stream));
    std::vector<unsigned long long> c(NCOUNT * CNT_SLOTS);
    HIP_TRY(hipMemcpy(c.data(), E->cnt, sizeof(unsigned long long) * c.size(), hipMemcpyDeviceToHost));
    for (int q = 0; q < NCOUNT; ++q) {
        unsigned long long t = 0;
        for (int k = 0; k < CNT_SLOTS; ++k) t += c[(size_t)q * CNT_SLOTS + k];
        out[q] = (int64_t)t;
    }
    return check_device_error(E);
}

pdf_status pdf_timing(pdf_ens E, int32_t enable, double* ms_out, int64_t* launches_out)
{
    if (!E) {
        set_error("pdf_timing: null ensemble");
        return PDF_E_INVAL;
    }
    HIP_TRY(hipSetDevice(E->grid->device));
    collect_timing(E);
    if (ms_out)
        for (int q = 0; q < T_N; ++q) ms_out[q] = E->t_ms[q];
    if (launches_out)
        for (int q = 0; q < T_N; ++q) launches_out[q] = E->t_n[q];
    if (enable) {
        for (int q = 0; q < T_N; ++q) {
            E->t_ms[q] = 0.0;
            E->t_n[q] = 0;
        }
    }
    E->timing = enable != 0;
    return PDF_OK;
}

}  // extern "C"
