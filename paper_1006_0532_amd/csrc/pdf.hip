// C ABI of libpdfgpu (include/pdf.h): argument checks, device memory, and the order of the
// kernel launches of one time step.  The arithmetic of the method runs in the kernels of
// kernels.hip (the step), redist.hip (App. B), fem.hip and amg.hip (the Eulerian solves) and
// noalloc.hip.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <limits>
#include <set>
#include <string>
#include <unordered_map>
#include <vector>

#include "device.h"
#include "fem.h"
#include "kernels.h"
#include "pdf_impl.h"

using namespace pdfgpu;

namespace pdfgpu {
pdf_status build_grid(pdf_grid_s& g, const pdf_mesh_desc& m, const pdf_fields_desc& f);
double* noalloc_scratch(int device);
pdf_status redistribution_plan(pdf_ens_s* E, const std::vector<int>& problems, int32_t n_min, uint32_t step,
                               int32_t** plan_buf, int64_t* plan_cap, int64_t* total, hipStream_t s);

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
        if (E->timing && !E->capturing && hipEventCreate(&a) == hipSuccess) (void)hipEventRecord(a, s);
    }
    ~Timed()
    {
        if (!a) return;
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


SoaRaw& cur(pdf_ens_s* E) { return E->buf[E->cur]; }

// group the particles of the current buffer by element, bin them, mix (mix != 0), write
// canonical order into the other buffer and reduce the statistics
template <class R>
pdf_status regroup(pdf_ens_s* E, bool mix, bool counts_ready, bool advance_step, hipStream_t s)
{
    DevGrid& g = E->dg;
    SoaRaw& in = cur(E);
    if (!counts_ready) {
        Timed t(E, T_COUNT, s);
        launch_count(in.elem, E->d_meta, E->n_slots_ub, g.ne, E->counts, E->err, s);
    }
    {
        Timed t(E, T_SCAN, s);
        launch_scan(E->counts, g.ne, E->start, E->scan_tmp, s);
    }
    if (counts_ready) {
        // the particle loop left every particle's arrival rank: place without atomics
        Timed t(E, T_SCATTER, s);
        launch_fill_i32(E->counts, g.ne, 0, s);
        launch_place(in.elem, E->arrival, E->d_meta, E->n_slots_ub, g.ne, E->start, E->idx, E->err, s);
    } else {
        Timed t(E, T_SCATTER, s);
        launch_scatter(in.elem, E->d_meta, E->n_slots_ub, g.ne, E->counts, E->start, E->idx, E->err, s);
    }
    ElementArgs<R> ea{};
    ea.in = in.as<R>();
    ea.out = E->buf[1 - E->cur].as<R>();
    ea.start = E->start;
    ea.idx = E->idx;
    ea.geo = g.geo;
    ea.prm = E->d_prm;
    ea.shift = static_cast<const R*>(E->shift);
    ea.part = static_cast<R*>(E->part);
    ea.tm = E->tm;
    ea.mix = mix ? 1 : 0;
    ea.ne = g.ne;
    ea.cap = E->cap;
    ea.lds_max = E->lds_max;
    ea.big_list = E->big_list;
    ea.big_count = E->big_count;
    ea.gkey = E->gkey;
    ea.gord = E->gord;
    ea.gu3 = E->gu3;
    ea.any_proj = E->any_proj ? 1 : 0;
    {
        Timed t(E, T_ELEMENT, s);
        launch_element_pass<R>(ea, E->tiers.data(), (int)E->tiers.size(), s);
    }
    NodeArgs<R> na{};
    na.part = static_cast<const R*>(E->part);
    na.n2e_ptr = g.n2e_ptr;
    na.n2e = g.n2e;
    na.shift = static_cast<R*>(E->shift);
    na.stats = E->stats;
    na.nn = g.nn;
    na.start = E->start;
    na.ne = g.ne;
    na.meta = E->d_meta;
    na.big_count = E->big_count;
    na.advance_step = advance_step ? 1 : 0;
    na.estimator = E->h_prm[0].estimator;
    {
        Timed t(E, T_NODE, s);
        launch_node_finalize<R>(na, s);
    }
    E->cur = 1 - E->cur;
    HIP_TRY(hipGetLastError());
    return PDF_OK;
}

pdf_status regroup_any(pdf_ens_s* E, bool mix, bool counts_ready, bool advance_step, hipStream_t s)
{
    return E->precision == PDF_MIXED ? regroup<float>(E, mix, counts_ready, advance_step, s)
                                     : regroup<double>(E, mix, counts_ready, advance_step, s);
}

// statistics of the last pass -> nodal fields and their derived fields (FP64 records; the
// FP32 copy of the mixed form follows)
void apply_feedback(pdf_ens_s* E, hipStream_t s)
{
    DevGrid& g = E->dg;
    launch_feedback(E->stats, g.node, g.geo, g.n2e_ptr, g.n2e, g.nn, g.ne, E->fb_alpha, E->fb_rey, E->fb_gn,
                    E->fb_h, s);
    if (g.node32) launch_f64_to_f32(g.node, g.node32, g.nn * NODE_STRIDE, s);
}

// one time step: particle loop, then grouping, binning, mixing and statistics
template <class R>
pdf_status step_once(pdf_ens_s* E, hipStream_t s)
{
    DevGrid& g = E->dg;
    AdvanceArgs<R> a{};
    a.s = cur(E).as<R>();
    a.geo = g.geo;
    a.node = E->precision == PDF_MIXED ? reinterpret_cast<const R*>(g.node32) : reinterpret_cast<const R*>(g.node);
    a.n2e_ptr = g.n2e_ptr;
    a.n2e = g.n2e;
    a.counts = E->counts;
    a.err = E->err;
    a.cnt = E->cnt;
    a.meta = E->d_meta;
    a.arrival = E->arrival;
    a.wall_list = E->idx;          // free between the particle loop and the scatter
    a.wall_count = E->big_count + 1;
    a.wave_list = E->wave_list;
    a.wave_count = E->big_count + 2;
    a.wave_cap = E->n_problems > 1 ? E->cap / 64 + 2 : 0;
    a.redo_list = E->gord;         // element-pass scratch, free during the particle loop
    a.redo_count = E->big_count + 3;
    a.ne = g.ne;
    a.p0 = E->h_prm[0];
    a.prm = E->d_prm;
    {
        Timed t(E, T_ADVANCE, s);
        launch_advance<R>(a, E->n_slots_ub, E->n_problems > 1, E->wp_full, E->adv_block, s);
    }
    HIP_TRY(hipGetLastError());
    pdf_status st = regroup<R>(E, true, true, true, s);
    if (st != PDF_OK) return st;
    if (E->fb_on) apply_feedback(E, s);
    E->step += 1;
    return PDF_OK;
}

pdf_status step_any(pdf_ens_s* E, hipStream_t s)
{
    return E->precision == PDF_MIXED ? step_once<float>(E, s) : step_once<double>(E, s);
}

// upload the per-problem time steps when they changed
pdf_status set_dt(pdf_ens_s* E, const double* dt, hipStream_t s)
{
    // only the time-step entries are uploaded: the device table's next pids move on with
    // number control, which need not report them to the host
    bool changed = false;
    for (int p = 0; p < E->n_problems; ++p)
        if (E->h_prm[p].dt != dt[p]) {
            E->h_prm[p].dt = dt[p];
            E->h_prm[p].sdt = std::sqrt(dt[p]);
            HIP_TRY(hipMemcpyAsync(&E->d_prm[p].dt, &E->h_prm[p].dt, sizeof(double), hipMemcpyHostToDevice, s));
            HIP_TRY(hipMemcpyAsync(&E->d_prm[p].sdt, &E->h_prm[p].sdt, sizeof(double), hipMemcpyHostToDevice, s));
            changed = true;
        }
    if (changed) HIP_TRY(hipStreamSynchronize(s));   // the host table may change again
    return PDF_OK;
}

void drop_graphs(pdf_ens_s* E)
{
    for (int c = 0; c < 2; ++c) {
        if (E->gexec[c]) (void)hipGraphExecDestroy(E->gexec[c]);
        E->gexec[c] = nullptr;
        E->g_nub[c] = -1;
        E->g_dt[c].clear();
    }
}

// Two steps from buffer c captured once into a HIP graph and replayed; captured again when
// the slot bound (after number control) or a time step changes.
pdf_status graph_steps(pdf_ens_s* E, int32_t n_steps, hipStream_t s)
{
    if (!E->gstream) {
        HIP_TRY(hipStreamCreateWithFlags(&E->gstream, hipStreamNonBlocking));
        HIP_TRY(hipEventCreateWithFlags(&E->gev[0], hipEventDisableTiming));
        HIP_TRY(hipEventCreateWithFlags(&E->gev[1], hipEventDisableTiming));
    }
    hipStream_t gs = E->gstream;
    HIP_TRY(hipEventRecord(E->gev[0], s));
    HIP_TRY(hipStreamWaitEvent(gs, E->gev[0], 0));
    std::vector<double> dts(E->n_problems);
    for (int p = 0; p < E->n_problems; ++p) dts[p] = E->h_prm[p].dt;
    int32_t left = n_steps;
    while (left >= 2) {
        const int c = E->cur;
        if (!E->gexec[c] || E->g_nub[c] != E->n_slots_ub || E->g_dt[c] != dts) {
            if (E->gexec[c]) (void)hipGraphExecDestroy(E->gexec[c]);
            E->gexec[c] = nullptr;
            const int64_t step0 = E->step;
            HIP_TRY(hipStreamBeginCapture(gs, hipStreamCaptureModeThreadLocal));
            E->capturing = true;
            pdf_status st = step_any(E, gs);
            if (st == PDF_OK) st = step_any(E, gs);
            E->capturing = false;
            hipGraph_t graph = nullptr;
            const hipError_t ce = hipStreamEndCapture(gs, &graph);
            E->step = step0;
            if (st != PDF_OK) {
                if (graph) (void)hipGraphDestroy(graph);
                return st;
            }
            HIP_TRY(ce);
            const hipError_t ie = hipGraphInstantiate(&E->gexec[c], graph, nullptr, nullptr, 0);
            (void)hipGraphDestroy(graph);
            HIP_TRY(ie);
            E->g_nub[c] = E->n_slots_ub;
            E->g_dt[c] = dts;
        }
        HIP_TRY(hipGraphLaunch(E->gexec[c], gs));
        E->step += 2;
        left -= 2;
    }
    if (left) {
        pdf_status st = step_any(E, gs);
        if (st != PDF_OK) return st;
    }
    HIP_TRY(hipEventRecord(E->gev[1], gs));
    HIP_TRY(hipStreamWaitEvent(s, E->gev[1], 0));
    return PDF_OK;
}

template <class R>
pdf_status control_impl(pdf_ens_s* E, int32_t n_min, int32_t n_max, pdf_control_report* report, hipStream_t s)
{
    DevGrid& g = E->dg;
    launch_fill_u64(E->ctl_rep, 4, 0ull, s);
    ControlArgs<R> c{};
    c.s = cur(E).as<R>();
    c.start = E->start;
    c.geo = g.geo;
    c.prm = E->d_prm;
    c.n_problems = E->n_problems;
    c.clone = E->ctl_clone;
    c.off = E->ctl_off;
    c.rep = E->ctl_rep;
    c.err = E->err;
    c.nslots = E->d_meta;
    c.ne = g.ne;
    c.cap = E->cap;
    c.n_min = n_min;
    c.n_max = n_max;
    {
        Timed t(E, T_CPLAN, s);
        launch_ctl_plan<R>(c, s);
    }
    {
        Timed t(E, T_CSCAN, s);
        launch_scan(E->ctl_clone, g.ne, E->ctl_off, E->scan_tmp, s);
    }
    {
        Timed t(E, T_CAPPLY, s);
        launch_ctl_apply<R>(c, s);
        launch_ctl_finish(E->d_meta, E->ctl_off, g.ne, E->ctl_rep, E->cap, E->d_prm, E->n_problems, s);
    }
    HIP_TRY(hipGetLastError());
    E->ctl_valid = false;
    if (!report) {
        // enqueued only: the slots now in use are known on the device alone, so later launches
        // cover the capacity (their threads beyond the used slots return at once); errors
        // surface at the next synchronising call
        E->n_slots_ub = E->cap;
        return PDF_OK;
    }
    int64_t meta[3];
    unsigned long long rep[4];
    HIP_TRY(hipMemcpyAsync(meta, E->d_meta, sizeof(meta), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipMemcpyAsync(rep, E->ctl_rep, sizeof(rep), hipMemcpyDeviceToHost, s));
    std::vector<ProbParams> prm(E->n_problems);
    HIP_TRY(hipMemcpyAsync(prm.data(), E->d_prm, sizeof(ProbParams) * E->n_problems, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    for (int p = 0; p < E->n_problems; ++p) E->h_prm[p].next_pid = prm[p].next_pid;
    E->n_slots_ub = meta[0];
    {
        report->live = meta[1];
        report->cloned = meta[2];
        report->merged = (int64_t)rep[0];
        report->empty = (int64_t)rep[1];
        report->below = (int64_t)rep[2];
        report->above = (int64_t)rep[3];
    }
    return check_device_error(E);
}

void free_devgrid(DevGrid& g)
{
    if (g.owned) {
        dfree(g.geo);
        dfree(g.node);
        dfree(g.n2e_ptr);
        dfree(g.n2e);
    } else if (g.own_fields) {
        dfree(g.geo);
        dfree(g.node);
    }
    dfree(g.node32);
    g = DevGrid{};
}

// device grid of the ensemble: the grid itself for one problem, concatenated copies with
// offset element, node and CSR indices for several
pdf_status build_devgrid(pdf_ens_s* E, hipStream_t s)
{
    DevGrid& d = E->dg;
    const int P = E->n_problems;
    if (P == 1) {
        pdf_grid_s* g = E->grids[0];
        d.nn = g->nn;
        d.ne = g->ne;
        d.geo = g->d_geo;
        d.node = g->d_node;
        d.n2e_ptr = g->d_n2e_ptr;
        d.n2e = g->d_n2e;
        d.owned = false;
    } else {
        int64_t nn = 0, ne = 0;
        for (auto* g : E->grids) {
            nn += g->nn;
            ne += g->ne;
        }
        std::vector<ElemGeo> geo;
        std::vector<double> node;
        std::vector<int64_t> ptr(1, 0);
        std::vector<int32_t> n2e;
        geo.reserve(ne);
        node.reserve(nn * NODE_STRIDE);
        n2e.reserve(3 * ne);
        int64_t eo = 0, no = 0;
        for (int p = 0; p < P; ++p) {
            const pdf_grid_s* g = E->grids[p];
            for (const ElemGeo& G0 : g->h_geo) {
                ElemGeo G = G0;
                for (int k = 0; k < 3; ++k) {
                    G.node[k] += (int32_t)no;
                    if (G.nbr[k] >= 0) G.nbr[k] += (int32_t)eo;
                }
                G.prob = p;
                geo.push_back(G);
            }
            node.insert(node.end(), g->h_node.begin(), g->h_node.end());
            const int64_t base = (int64_t)n2e.size();
            for (int64_t i = 0; i < g->nn; ++i) ptr.push_back(base + g->h_n2e_ptr[i + 1]);
            for (int32_t v : g->h_n2e) n2e.push_back(v + 3 * (int32_t)eo);
            eo += g->ne;
            no += g->nn;
        }
        d.nn = nn;
        d.ne = ne;
        d.owned = true;
        pdf_status st = dalloc(&d.geo, ne);
        if (st == PDF_OK) st = dalloc(&d.node, nn * NODE_STRIDE);
        if (st == PDF_OK) st = dalloc(&d.n2e_ptr, nn + 1);
        if (st == PDF_OK) st = dalloc(&d.n2e, 3 * ne);
        if (st != PDF_OK) return st;
        HIP_TRY(hipMemcpyAsync(d.geo, geo.data(), sizeof(ElemGeo) * ne, hipMemcpyHostToDevice, s));
        HIP_TRY(hipMemcpyAsync(d.node, node.data(), sizeof(double) * nn * NODE_STRIDE, hipMemcpyHostToDevice, s));
        HIP_TRY(hipMemcpyAsync(d.n2e_ptr, ptr.data(), sizeof(int64_t) * (nn + 1), hipMemcpyHostToDevice, s));
        HIP_TRY(hipMemcpyAsync(d.n2e, n2e.data(), sizeof(int32_t) * 3 * ne, hipMemcpyHostToDevice, s));
        HIP_TRY(hipStreamSynchronize(s));
    }
    if (E->precision == PDF_MIXED) {
        pdf_status st = dalloc(&d.node32, d.nn * NODE_STRIDE);
        if (st != PDF_OK) return st;
        launch_f64_to_f32(d.node, d.node32, d.nn * NODE_STRIDE, s);
    }
    return PDF_OK;
}

// particles per lane for a set-up count with 30 % headroom (7 is not instantiated)
int ppl_for(int64_t ppe)
{
    int p = (int)std::min<int64_t>(8, std::max<int64_t>(1, (13 * ppe + 639) / 640));
    return p == 7 ? 8 : p;
}

// wavefront tiers from the smallest suggested capacity up to ppl: doubling to 4 particles
// per lane, then 6 and 8 (an element is taken by the smallest tier that holds it; between 4
// and 8 a tier of 6 keeps three wavefronts per SIMD in FP64 where 8 allows two)
void set_tiers(pdf_ens_s* E)
{
    E->tiers.clear();
    int t = std::min(E->ppl_min, E->ppl);
    while (t < E->ppl) {
        E->tiers.push_back(t);
        t = t < 4 ? 2 * t : (t < 6 ? 6 : 8);
    }
    E->tiers.push_back(E->ppl);
}

// bytes of one state array entry other than x, y, pid, elem
size_t real_size(const pdf_ens_s* E) { return E->precision == PDF_MIXED ? sizeof(float) : sizeof(double); }

pdf_status alloc_raw(void** p, int64_t count, size_t elem)
{
    *p = nullptr;
    if (count <= 0) count = 1;
    hipError_t e = hipMalloc(p, elem * (size_t)count);
    if (e != hipSuccess) {
        *p = nullptr;
        (void)hipGetLastError();
        set_error(std::string("device allocation of ") + std::to_string(elem * count) + " bytes failed");
        return PDF_E_NOMEM;
    }
    return PDF_OK;
}

void free_raw(void*& p)
{
    if (p) (void)hipFree(p);
    p = nullptr;
}

template <class R>
void launch_init_any(pdf_ens_s* E, int64_t n0, hipStream_t s)
{
    InitArgs<R> ia{};
    ia.s = E->buf[0].as<R>();
    ia.geo = E->dg.geo;
    ia.node = E->precision == PDF_MIXED ? reinterpret_cast<const R*>(E->dg.node32)
                                        : reinterpret_cast<const R*>(E->dg.node);
    ia.prm = E->d_prm;
    ia.n_problems = E->n_problems;
    ia.n = n0;
    launch_init<R>(ia, s);
}

template <class R>
pdf_status setup_precision(pdf_ens_s* E, hipStream_t s)
{
    const int fixed = (int)element_pass_smem<R>(0);
    const int per = (int)element_pass_smem<R>(1) - fixed;
    E->lds_max = std::max(64, (65536 - fixed) / per);
    HIP_TRY(prepare_element_pass<R>(E->lds_max));
    const R* node = E->precision == PDF_MIXED ? reinterpret_cast<const R*>(E->dg.node32)
                                              : reinterpret_cast<const R*>(E->dg.node);
    launch_shift_init<R>(node, E->dg.nn, static_cast<R*>(E->shift), s);
    return PDF_OK;
}

// device-to-host copy of one state array of the current buffer, as doubles
pdf_status pull_real(pdf_ens_s* E, const void* src, int64_t ns, std::vector<double>& out)
{
    out.resize(ns);
    if (ns == 0) return PDF_OK;
    if (E->precision == PDF_MIXED) {
        std::vector<float> t(ns);
        HIP_TRY(hipMemcpy(t.data(), src, sizeof(float) * ns, hipMemcpyDeviceToHost));
        for (int64_t i = 0; i < ns; ++i) out[i] = (double)t[i];
    } else {
        HIP_TRY(hipMemcpy(out.data(), src, sizeof(double) * ns, hipMemcpyDeviceToHost));
    }
    return PDF_OK;
}

pdf_status push_real(pdf_ens_s* E, void* dst, const std::vector<double>& in, hipStream_t s)
{
    const int64_t n = (int64_t)in.size();
    if (n == 0) return PDF_OK;
    if (E->precision == PDF_MIXED) {
        std::vector<float> t(n);
        for (int64_t i = 0; i < n; ++i) t[i] = (float)in[i];
        HIP_TRY(hipMemcpyAsync(dst, t.data(), sizeof(float) * n, hipMemcpyHostToDevice, s));
        HIP_TRY(hipStreamSynchronize(s));
    } else {
        HIP_TRY(hipMemcpyAsync(dst, in.data(), sizeof(double) * n, hipMemcpyHostToDevice, s));
        HIP_TRY(hipStreamSynchronize(s));
    }
    return PDF_OK;
}

}  // namespace



namespace {

// the grid's element and node records are shared with other ensembles: an ensemble that
// changes its fields (statistics feedback, the Eulerian solves) works on copies
pdf_status ensure_own_fields(pdf_ens_s* E, hipStream_t s)
{
    DevGrid& g = E->dg;
    if (g.owned || g.own_fields) return PDF_OK;
    ElemGeo* geo = nullptr;
    double* node = nullptr;
    pdf_status st = dalloc(&geo, g.ne);
    if (st == PDF_OK) st = dalloc(&node, g.nn * NODE_STRIDE);
    if (st != PDF_OK) {
        dfree(geo);
        return st;
    }
    HIP_TRY(hipMemcpyAsync(geo, g.geo, sizeof(ElemGeo) * g.ne, hipMemcpyDeviceToDevice, s));
    HIP_TRY(hipMemcpyAsync(node, g.node, sizeof(double) * g.nn * NODE_STRIDE, hipMemcpyDeviceToDevice, s));
    g.geo = geo;
    g.node = node;
    g.own_fields = true;
    drop_graphs(E);   // captured steps read the old records
    return PDF_OK;
}

// ---------------------------------------------------------------------------------------
// Eulerian solves (Sec. 3.2)
// ---------------------------------------------------------------------------------------
template <class T>
pdf_status fem_alloc(T*& p, int64_t n)
{
    if (p) return PDF_OK;
    return dalloc(&p, n);
}

// boundary geometry of the grid: node kinds and normals, nearest-wall normals per element
pdf_status fem_geometry(pdf_ens_s* E, hipStream_t s)
{
    FemState& F = E->fem;
    if (F.geom) return PDF_OK;
    const pdf_grid_s* gr = E->grid;
    const int64_t nn = gr->nn, ne = gr->ne;
    std::vector<uint8_t> wk(nn, 0);
    std::vector<double> nrm(2 * nn, 0.0), edges;
    for (int64_t e = 0; e < ne; ++e) {
        const ElemGeo& G = gr->h_geo[e];
        for (int k = 0; k < 3; ++k) {
            if (G.kind[k] != KIND_WALL && G.kind[k] != KIND_SLIP) continue;
            const int a = (k + 1) % 3, b = (k + 2) % 3;
            const double dx = G.x[b] - G.x[a], dy = G.y[b] - G.y[a];
            const double len = std::sqrt(dx * dx + dy * dy);
            const double ox = dy / len, oy = -dx / len;     // right of a->b: outside a CCW element
            if (G.kind[k] == KIND_WALL) {
                for (int v : {a, b}) {
                    nrm[2 * G.node[v]] += len * ox;
                    nrm[2 * G.node[v] + 1] += len * oy;
                    wk[G.node[v]] = 2;
                }
                edges.insert(edges.end(), {0.5 * (G.x[a] + G.x[b]), 0.5 * (G.y[a] + G.y[b]), ox, oy});
            } else {
                for (int v : {a, b})
                    if (wk[G.node[v]] == 0) wk[G.node[v]] = 1;
            }
        }
    }
    // a node on both kinds counts as no-slip
    for (int64_t e = 0; e < ne; ++e) {
        const ElemGeo& G = gr->h_geo[e];
        for (int k = 0; k < 3; ++k)
            if (G.kind[k] == KIND_WALL) wk[G.node[(k + 1) % 3]] = wk[G.node[(k + 2) % 3]] = 2;
    }
    for (int64_t n = 0; n < nn; ++n)
        if (wk[n] == 2) {
            const double l = std::sqrt(nrm[2 * n] * nrm[2 * n] + nrm[2 * n + 1] * nrm[2 * n + 1]);
            nrm[2 * n] /= l;
            nrm[2 * n + 1] /= l;
        }
    pdf_status st = fem_alloc(F.wkind, nn);
    if (st == PDF_OK) st = fem_alloc(F.wnrm, 2 * nn);
    if (st == PDF_OK) st = fem_alloc(F.enrm, 2 * ne);
    if (st == PDF_OK) st = fem_alloc(F.ke, 8 * ne);
    if (st != PDF_OK) return st;
    fem_elem_matrices(E->dg.geo, ne, F.ke, s);
    const int32_t nw = (int32_t)(edges.size() / 4);
    double* d_edges = nullptr;
    st = dalloc(&d_edges, 4 * (int64_t)std::max<int32_t>(nw, 1));
    if (st != PDF_OK) return st;
    HIP_TRY(hipMemcpyAsync(F.wkind, wk.data(), nn, hipMemcpyHostToDevice, s));
    HIP_TRY(hipMemcpyAsync(F.wnrm, nrm.data(), sizeof(double) * 2 * nn, hipMemcpyHostToDevice, s));
    if (nw) HIP_TRY(hipMemcpyAsync(d_edges, edges.data(), sizeof(double) * edges.size(), hipMemcpyHostToDevice, s));
    fem_nearest_wall(E->dg.geo, ne, d_edges, nw, gr->period, F.enrm, s);
    HIP_TRY(hipGetLastError());
    HIP_TRY(hipStreamSynchronize(s));
    dfree(d_edges);
    F.geom = true;
    return PDF_OK;
}

pdf_status fem_work(pdf_ens_s* E)
{
    FemState& F = E->fem;
    const int64_t nn = E->dg.nn, ne = E->dg.ne;
    pdf_status st = PDF_OK;
    for (double** q : {&F.f, &F.xfix, &F.b, &F.x, &F.r, &F.z, &F.p, &F.Ap, &F.diag})
        if (st == PDF_OK) st = fem_alloc(*q, 9 * nn);
    if (st == PDF_OK) st = fem_alloc(F.fixed, nn + 1);
    if (st == PDF_OK && !F.nofix) {
        st = fem_alloc(F.nofix, nn + 1);
        if (st == PDF_OK) launch_fill_i32(reinterpret_cast<int32_t*>(F.nofix), (nn + 1) / 2, 0, E->stream);
    }
    if (st == PDF_OK) st = fem_alloc(F.L2, 4 * ne);
    if (st == PDF_OK) st = fem_alloc(F.sc, 6 * 9);
    if (st == PDF_OK) st = fem_alloc(F.partial, (int64_t)FEM_RED_BLOCKS * 18);
    return st;
}

// statistics must be defined at every node
pdf_status fem_check(pdf_ens_s* E, hipStream_t s, const char* who)
{
    launch_fill_u64(E->d_scalar, 1, 0ull, s);
    fem_check_stats(E->stats, E->dg.nn, E->d_scalar, s);
    unsigned long long bad = 0;
    HIP_TRY(hipMemcpyAsync(&bad, E->d_scalar, sizeof(bad), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    if (bad) {
        set_error(std::string(who) + ": " + std::to_string(bad) + " nodes without statistics");
        return PDF_E_STATE;
    }
    return PDF_OK;
}

// Jacobi-preconditioned CG on NC independent components: x holds the Dirichlet values
// (and zero elsewhere) on entry and the solution on return
template <int NC>
pdf_status fem_cg(pdf_ens_s* E, const FemOp& op, const double* b, double tol, int32_t max_iter, int32_t* iters,
                  hipStream_t s)
{
    FemState& F = E->fem;
    const int64_t nn = op.nn;
    launch_fill_u64(reinterpret_cast<unsigned long long*>(F.sc), 6 * NC, 0ull, s);
    fem_diag<NC>(op, F.diag, s);
    FemOp full = op;
    full.fixed = F.nofix;            // the initial residual includes the Dirichlet columns
    fem_apply<NC>(full, F.x, F.Ap, s);
    fem_cg_init<NC>(b, F.Ap, F.diag, op.fixed, nn, F.r, F.z, F.p, s);
    fem_dot<NC>(F.r, F.z, F.r, F.r, nn, F.partial, F.sc + 2 * NC, s);
    fem_cg_beta<NC>(F.sc, s);
    double rr0[NC], h[2 * NC];
    HIP_TRY(hipMemcpyAsync(rr0, F.sc + 3 * NC, sizeof(rr0), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    int32_t it = 0;
    auto done = [&](const double* rr) {
        for (int c = 0; c < NC; ++c)
            if (rr[c] > tol * tol * rr0[c]) return false;
        return true;
    };
    if (!done(rr0)) {
        while (it < max_iter) {
            fem_apply<NC>(op, F.p, F.Ap, s);
            fem_dot<NC>(F.p, F.Ap, nullptr, nullptr, nn, F.partial, F.sc + NC, s);
            fem_cg_alpha<NC>(F.sc, s);
            fem_cg_xr<NC>(F.sc, F.p, F.Ap, F.diag, op.fixed, nn, F.x, F.r, F.z, s);
            fem_dot<NC>(F.r, F.z, F.r, F.r, nn, F.partial, F.sc + 2 * NC, s);
            fem_cg_beta<NC>(F.sc, s);
            fem_cg_p<NC>(F.sc, F.z, nn, F.p, s);
            ++it;
            if (it % 8 == 0 || it == max_iter) {
                HIP_TRY(hipMemcpyAsync(h, F.sc + 2 * NC, sizeof(h), hipMemcpyDeviceToHost, s));
                HIP_TRY(hipStreamSynchronize(s));
                if (done(h + NC)) break;
            }
        }
    }
    HIP_TRY(hipGetLastError());
    if (iters) *iters = it;
    return PDF_OK;
}

// The pressure system's stiffness matrix does not change: assemble it once per ensemble
// into CSR (columns ascending; contributions summed in the node->element order), so that
// each CG iteration reads 12 bytes per nonzero instead of rebuilding element matrices.
pdf_status fem_pressure_matrix(pdf_ens_s* E, hipStream_t s)
{
    FemState& F = E->fem;
    if (F.csr_rp) return PDF_OK;
    const pdf_grid_s* gr = E->grid;
    const int64_t nn = gr->nn;
    std::vector<int32_t> rp(nn + 1, 0), col;
    std::vector<double> val;
    std::vector<int32_t> nb;
    for (int64_t n = 0; n < nn; ++n) {
        nb.clear();
        for (int64_t j = gr->h_n2e_ptr[n]; j < gr->h_n2e_ptr[n + 1]; ++j) {
            const ElemGeo& G = gr->h_geo[gr->h_n2e[j] / 3];
            for (int b = 0; b < 3; ++b) nb.push_back(G.node[b]);
        }
        std::sort(nb.begin(), nb.end());
        nb.erase(std::unique(nb.begin(), nb.end()), nb.end());
        std::vector<double> v(nb.size(), 0.0);
        for (int64_t j = gr->h_n2e_ptr[n]; j < gr->h_n2e_ptr[n + 1]; ++j) {
            const int32_t ea = gr->h_n2e[j];
            const ElemGeo& G = gr->h_geo[ea / 3];
            const int a = ea % 3;
            double bx[3], by[3];
            for (int q = 0; q < 3; ++q) {
                const int b = q == 2 ? 0 : q + 1, c = q == 0 ? 2 : q - 1;
                bx[q] = (G.y[b] - G.y[c]) / (2.0 * G.area);
                by[q] = (G.x[c] - G.x[b]) / (2.0 * G.area);
            }
            for (int b = 0; b < 3; ++b) {
                const size_t k = std::lower_bound(nb.begin(), nb.end(), G.node[b]) - nb.begin();
                v[k] += G.area * (bx[a] * bx[b] + by[a] * by[b]);
            }
        }
        col.insert(col.end(), nb.begin(), nb.end());
        val.insert(val.end(), v.begin(), v.end());
        rp[n + 1] = (int32_t)col.size();
    }
    pdf_status st = dalloc(&F.csr_rp, nn + 1);
    if (st == PDF_OK) st = dalloc(&F.csr_col, (int64_t)col.size());
    if (st == PDF_OK) st = dalloc(&F.csr_val, (int64_t)val.size());
    if (st == PDF_OK) st = dalloc(&F.partial2, 2 * (int64_t)fem_csr_blocks(nn));
    if (st != PDF_OK) return st;
    HIP_TRY(hipMemcpyAsync(F.csr_rp, rp.data(), sizeof(int32_t) * rp.size(), hipMemcpyHostToDevice, s));
    HIP_TRY(hipMemcpyAsync(F.csr_col, col.data(), sizeof(int32_t) * col.size(), hipMemcpyHostToDevice, s));
    HIP_TRY(hipMemcpyAsync(F.csr_val, val.data(), sizeof(double) * val.size(), hipMemcpyHostToDevice, s));
    HIP_TRY(hipStreamSynchronize(s));
    F.csr_nnz = (int64_t)col.size();
    F.hcsr.n = F.hcsr.m = nn;
    F.hcsr.rp = std::move(rp);
    F.hcsr.col = std::move(col);
    F.hcsr.val = std::move(val);
    return PDF_OK;
}

// multigrid preconditioner of the pressure matrix, built on first use (Jacobi when the
// hierarchy cannot be built or uploaded)
void fem_pressure_amg(pdf_ens_s* E, hipStream_t s)
{
    FemState& F = E->fem;
    if (F.amg_tried) return;
    F.amg_tried = true;
    AmgHost h;
    if (!amg_build(F.hcsr, h)) return;
    F.amg = new AmgDev();
    if (amg_upload(h, *F.amg, s) != hipSuccess) {
        (void)hipGetLastError();
        delete F.amg;
        F.amg = nullptr;
    }
}

// Jacobi-preconditioned CG on the assembled scalar matrix from x = 0, with fused reductions
pdf_status fem_cg_csr(pdf_ens_s* E, const double* b, double tol, int32_t max_iter, int32_t* iters, hipStream_t s)
{
    FemState& F = E->fem;
    const int64_t nn = E->dg.nn;
    const int nb = fem_csr_blocks(nn);
    // two p buffers (the vectors hold nine components' room), partials of r.z, r.r and
    // of p.Kp, and the two r.z slots
    double* pbuf[2] = {F.p, F.p + nn};
    static_assert(3 * CG2_BLOCKS <= FEM_RED_BLOCKS * 18, "CG partials fit the reduction buffer");
    double* part_rz = F.partial;
    double* part_py = F.partial + 2 * CG2_BLOCKS;
    launch_fill_u64(reinterpret_cast<unsigned long long*>(F.sc), 6, 0ull, s);
    launch_fill_u64(reinterpret_cast<unsigned long long*>(pbuf[1]), nn, 0ull, s);
    fem_csr_diag(F.csr_rp, F.csr_col, F.csr_val, nn, F.diag, s);
    fem_csr_apply_dot(F.csr_rp, F.csr_col, F.csr_val, F.x, nn, F.Ap, F.partial2, nb, s);
    fem_cg_init<1>(b, F.Ap, F.diag, F.nofix, nn, F.r, F.z, F.p, s);
    fem_cg2_dots(F.r, F.z, nn, part_rz, s);
    std::vector<double> h(2 * CG2_BLOCKS);
    // r.r from the partials, in the same fixed order on the host
    auto rr_sum = [&]() -> pdf_status {
        HIP_TRY(hipMemcpyAsync(h.data(), part_rz, sizeof(double) * h.size(), hipMemcpyDeviceToHost, s));
        HIP_TRY(hipStreamSynchronize(s));
        return PDF_OK;
    };
    auto rr_of = [&]() {
        double t = 0.0;
        for (int q = 0; q < CG2_BLOCKS; ++q) t += h[2 * q + 1];
        return t;
    };
    if (F.amg) {
        // preconditioned by the multigrid V-cycle: z = M^-1 r after every update
        amg_vcycle(*F.amg, F.r, F.z, s);
        fem_cg2_dots(F.r, F.z, nn, part_rz, s);
        pdf_status st = rr_sum();
        if (st != PDF_OK) return st;
        const double rr0 = rr_of();
        int32_t it = 0;
        if (rr0 > 0.0) {
            while (it < max_iter) {
                const int k = it;
                fem_cg2_apply(F.csr_rp, F.csr_col, F.csr_val, F.z, pbuf[(k + 1) & 1], pbuf[k & 1], nn, F.Ap, part_rz,
                              part_py, F.sc, k, s);
                fem_cg2_update_xr(F.sc, part_py, pbuf[k & 1], F.Ap, nn, F.x, F.r, k, s);
                amg_vcycle(*F.amg, F.r, F.z, s);
                fem_cg2_dots(F.r, F.z, nn, part_rz, s);
                ++it;
                if (it % 2 == 0 || it == max_iter) {
                    st = rr_sum();
                    if (st != PDF_OK) return st;
                    if (!(rr_of() > tol * tol * rr0)) break;
                }
            }
        }
        HIP_TRY(hipGetLastError());
        if (iters) *iters = it;
        return PDF_OK;
    }
    pdf_status st = rr_sum();
    if (st != PDF_OK) return st;
    const double rr0 = rr_of();
    int32_t it = 0;
    if (rr0 > 0.0) {
        while (it < max_iter) {
            const int k = it;
            fem_cg2_apply(F.csr_rp, F.csr_col, F.csr_val, F.z, pbuf[(k + 1) & 1], pbuf[k & 1], nn, F.Ap, part_rz,
                          part_py, F.sc, k, s);
            fem_cg2_update(F.sc, part_py, pbuf[k & 1], F.Ap, F.diag, nn, F.x, F.r, F.z, part_rz, k, s);
            ++it;
            if (it % 16 == 0 || it == max_iter) {
                st = rr_sum();
                if (st != PDF_OK) return st;
                if (!(rr_of() > tol * tol * rr0)) break;
            }
        }
    }
    HIP_TRY(hipGetLastError());
    if (iters) *iters = it;
    return PDF_OK;
}

FemOp fem_op(pdf_ens_s* E, double mass, double stiff, const double* L2, const uint16_t* fixed)
{
    FemOp op{};
    op.geo = E->dg.geo;
    op.ke = E->fem.ke;
    op.n2e_ptr = E->dg.n2e_ptr;
    op.n2e = E->dg.n2e;
    op.nn = E->dg.nn;
    op.mass = mass;
    op.stiff = stiff;
    op.L2 = L2;
    op.fixed = fixed;
    return op;
}

}  // namespace

// ---------------------------------------------------------------------------------------
// Particle redistribution (App. B): planned on the device (redist.hip), applied here from
// the state of the last step by gathering every move's sources into the idle state buffer,
// then writing them.
// ---------------------------------------------------------------------------------------
namespace {

template <class R>
pdf_status apply_redistribution(pdf_ens_s* E, int64_t m, hipStream_t s)
{
    if (m == 0) return PDF_OK;
    launch_redistribute<R>(cur(E).as<R>(), E->buf[1 - E->cur].as<R>(), E->redist_plan, E->dg.geo, m, s);
    HIP_TRY(hipGetLastError());
    HIP_TRY(hipStreamSynchronize(s));
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
    drop_graphs(E);
    if (E->gstream) (void)hipStreamDestroy(E->gstream);
    for (int k = 0; k < 2; ++k)
        if (E->gev[k]) (void)hipEventDestroy(E->gev[k]);
    for (int b = 0; b < 2; ++b) {
        SoaRaw& S = E->buf[b];
        dfree(S.x); dfree(S.y); free_raw(S.u0); free_raw(S.u1); free_raw(S.u2); free_raw(S.om); free_raw(S.psi);
        free_raw(S.w); dfree(S.pid); dfree(S.elem);
    }
    dfree(E->counts); dfree(E->start); dfree(E->idx); dfree(E->arrival); dfree(E->scan_tmp); dfree(E->d_meta); free_raw(E->part);
    dfree(E->stats); free_raw(E->shift); dfree(E->tm); dfree(E->err); dfree(E->cnt); dfree(E->gkey); dfree(E->gord);
    dfree(E->gu3); dfree(E->ctl_clone); dfree(E->ctl_off); dfree(E->ctl_rep); dfree(E->big_list);
    dfree(E->big_count); dfree(E->wave_list); dfree(E->d_prm); dfree(E->d_scalar);
    free_devgrid(E->dg);
    dfree(E->fb_gn);
    dfree(E->fb_h);
    dfree(E->redist_plan);
    FemState& F = E->fem;
    dfree(F.wkind); dfree(F.wnrm); dfree(F.enrm); dfree(F.ke); dfree(F.f); dfree(F.xfix); dfree(F.b); dfree(F.x); dfree(F.r);
    dfree(F.z); dfree(F.p); dfree(F.Ap); dfree(F.diag); dfree(F.fixed); dfree(F.nofix); dfree(F.L2); dfree(F.sc);
    dfree(F.partial);
    dfree(F.P); dfree(F.gp0); dfree(F.gP); dfree(F.gdP);
    dfree(F.csr_rp); dfree(F.csr_col); dfree(F.csr_val); dfree(F.partial2); dfree(F.cval4);
    if (F.amg) {
        amg_free(*F.amg);
        delete F.amg;
        F.amg = nullptr;
    }
    delete E;
    return PDF_OK;
}

pdf_status pdf_particles_init(const pdf_grid* grids, const pdf_init_desc* descs, int32_t n_problems,
                              void* hip_stream, pdf_ens* out)
{
    if (!grids || !descs || !out || n_problems < 1) {
        set_error("pdf_particles_init: null argument or n_problems < 1");
        return PDF_E_INVAL;
    }
    *out = nullptr;
    int64_t n0 = 0, ne = 0, cap = 0;
    for (int p = 0; p < n_problems; ++p) {
        const pdf_init_desc& d = descs[p];
        const pdf_grid_s* g = grids[p];
        if (!g) {
            set_error("pdf_particles_init: null grid");
            return PDF_E_INVAL;
        }
        const int64_t nb = (int64_t)d.bins[0] * d.bins[1] * d.bins[2];
        if (d.ppe < 0 || d.bins[0] < 1 || d.bins[1] < 1 || d.bins[2] < 1 || nb > MAXBINS || d.min_per_bin < 1 ||
            !(d.omega_shape >= 1.0) || !(d.u_sigma >= 0.0) || !(d.src_r >= 0.0) || !std::isfinite(d.u_sigma) ||
            !std::isfinite(d.omega_shape) || !std::isfinite(d.src_x) || !std::isfinite(d.src_y) ||
            !std::isfinite(d.src_r) || (d.precision != PDF_FP64 && d.precision != PDF_MIXED) ||
            d.precision != descs[0].precision || d.capacity < 0 || g->device != grids[0]->device ||
            (d.estimator != PDF_EST_P1 && d.estimator != PDF_EST_ELEMENT) || d.estimator != descs[0].estimator ||
            (d.conditioning != PDF_COND_BINS && d.conditioning != PDF_COND_PROJECTION)) {
            set_error("pdf_particles_init: invalid descriptor (bins product <= 1024, omega_shape >= 1, one "
                      "precision, estimator and device for all problems)");
            return PDF_E_INVAL;
        }
        const int64_t n0p = g->ne * (int64_t)d.ppe;
        n0 += n0p;
        ne += g->ne;
        cap += d.capacity > 0 ? d.capacity : std::max<int64_t>(2 * n0p, 1024);
        if (d.capacity > 0 && d.capacity < n0p) {
            set_error("pdf_particles_init: capacity below the initial particle count");
            return PDF_E_CAPACITY;
        }
    }
    if (ne > scan_max_elems() || ne > (int64_t)INT32_MAX / 3) {
        set_error("pdf_particles_init: too many elements for the segment scan");
        return PDF_E_INVAL;
    }
    if (cap > (int64_t)INT32_MAX - 1) {
        set_error("pdf_particles_init: capacity above 2^31 - 2 slots");
        return PDF_E_INVAL;
    }
    pdf_grid_s* g0 = grids[0];
    HIP_TRY(hipSetDevice(g0->device));
    // device address of the fixed scratch of pdf_cfl_dt_noalloc, looked up once per device
    // (a failure is reported by that call, not here)
    (void)noalloc_scratch(g0->device);
    hipStream_t s = as_stream(hip_stream);
    pdf_ens_s* E = new pdf_ens_s();
    E->grid = g0;
    E->grids.assign(grids, grids + n_problems);
    E->descs.assign(descs, descs + n_problems);
    E->n_problems = n_problems;
    E->precision = descs[0].precision;
    E->d = descs[0];
    E->cap = cap;
    E->stream = s;
    pdf_status st = build_devgrid(E, s);
    // per-problem parameter table
    {
        int64_t eo = 0, no = 0, so = 0;
        for (int p = 0; p < n_problems && st == PDF_OK; ++p) {
            const pdf_init_desc& d = descs[p];
            const pdf_grid_s* g = grids[p];
            ProbParams P{};
            P.m = g->model;
            P.dt = 0.0;
            P.sdt = 0.0;
            P.s2nu = std::sqrt(2.0 * P.m.nu);
            P.irho = 1.0 / P.m.rho;
            P.period = g->period;
            P.src_x = d.src_x;
            P.src_y = d.src_y;
            P.src_r2 = d.src_r * d.src_r;
            P.u_sigma = d.u_sigma;
            P.omega_shape = d.omega_shape;
            P.key = RngKey{(uint32_t)d.seed, (uint32_t)(d.seed >> 32) ^ (uint32_t)p};
            P.src_cont = d.src_continuous;
            P.bins0 = d.bins[0];
            P.bins1 = d.bins[1];
            P.bins2 = d.bins[2];
            P.minpb = d.min_per_bin;
            P.ppe = d.ppe > 0 ? d.ppe : 1;
            P.estimator = d.estimator;
            P.conditioning = d.conditioning;
            if (d.conditioning == PDF_COND_PROJECTION) E->any_proj = true;
            P.eoff = eo;
            P.ne = g->ne;
            P.noff = no;
            P.nn = g->nn;
            P.soff = so;
            P.next_pid = (uint64_t)(g->ne * (int64_t)d.ppe);
            E->h_prm.push_back(P);
            eo += g->ne;
            no += g->nn;
            so += g->ne * (int64_t)d.ppe;
        }
    }
    const size_t rs = real_size(E);
    for (int b = 0; b < 2 && st == PDF_OK; ++b) {
        SoaRaw& S = E->buf[b];
        st = dalloc(&S.x, cap);
        if (st == PDF_OK) st = dalloc(&S.y, cap);
        if (st == PDF_OK) st = alloc_raw(&S.u0, cap, rs);
        if (st == PDF_OK) st = alloc_raw(&S.u1, cap, rs);
        if (st == PDF_OK) st = alloc_raw(&S.u2, cap, rs);
        if (st == PDF_OK) st = alloc_raw(&S.om, cap, rs);
        if (st == PDF_OK) st = alloc_raw(&S.psi, cap, rs);
        if (st == PDF_OK) st = alloc_raw(&S.w, cap, rs);
        if (st == PDF_OK) st = dalloc(&S.pid, cap);
        if (st == PDF_OK) st = dalloc(&S.elem, cap);
    }
    const DevGrid& g = E->dg;
    if (st == PDF_OK) st = dalloc(&E->d_prm, n_problems);
    if (st == PDF_OK) st = dalloc(&E->counts, g.ne);
    if (st == PDF_OK) st = dalloc(&E->start, g.ne + 1);
    if (st == PDF_OK) st = dalloc(&E->idx, cap);
    if (st == PDF_OK) st = dalloc(&E->arrival, cap);
    if (st == PDF_OK) st = dalloc(&E->scan_tmp, scan_blocks(g.ne) + 1);
    if (st == PDF_OK) st = dalloc(&E->d_meta, 8);
    if (st == PDF_OK) st = alloc_raw(&E->part, g.ne * 3 * NPART, rs);
    if (st == PDF_OK) st = dalloc(&E->stats, g.nn * NSTAT);
    if (st == PDF_OK) st = alloc_raw(&E->shift, g.nn * 5, rs);
    if (st == PDF_OK) st = dalloc(&E->tm, g.ne);
    if (st == PDF_OK) st = dalloc(&E->err, 1);
    if (st == PDF_OK) st = dalloc(&E->cnt, (int64_t)n_problems * NCOUNT * CNT_SLOTS);
    if (st == PDF_OK) st = dalloc(&E->d_scalar, 8);
    if (st == PDF_OK) st = dalloc(&E->gkey, 2 * cap);
    if (st == PDF_OK) st = dalloc(&E->gord, 2 * cap);
    if (st == PDF_OK) st = dalloc(&E->gu3, 4 * cap);
    if (st == PDF_OK) st = dalloc(&E->ctl_clone, g.ne);
    if (st == PDF_OK) st = dalloc(&E->ctl_off, g.ne + 1);
    if (st == PDF_OK) st = dalloc(&E->ctl_rep, 4);
    if (st == PDF_OK) st = dalloc(&E->big_list, g.ne);
    if (st == PDF_OK) st = dalloc(&E->big_count, 4);
    if (st == PDF_OK && n_problems > 1) st = dalloc(&E->wave_list, cap / 64 + 2);
    if (st != PDF_OK) {
        pdf_ens_destroy(E);
        return st;
    }
    // element pass: a wavefront per element holds up to 64 * ppl particles (ppl from the
    // largest set-up count with 30 % headroom); larger elements go to the workgroup
    // kernel, whose on-chip path takes up to lds_max particles within 64 KiB of LDS.
    // Number control later sets the first tier to its upper bound.
    int64_t ppe_max = 1, ppe_min = INT32_MAX;
    for (auto& d : E->descs) {
        ppe_max = std::max<int64_t>(ppe_max, d.ppe);
        if (d.ppe > 0) ppe_min = std::min<int64_t>(ppe_min, d.ppe);
    }
    E->ppl = ppl_for(ppe_max);
    E->ppl_min = ppl_for(ppe_min == INT32_MAX ? ppe_max : ppe_min);
    set_tiers(E);
    HIP_TRY(hipMemcpyAsync(E->d_prm, E->h_prm.data(), sizeof(ProbParams) * n_problems, hipMemcpyHostToDevice, s));
    st = E->precision == PDF_MIXED ? setup_precision<float>(E, s) : setup_precision<double>(E, s);
    if (st != PDF_OK) {
        pdf_ens_destroy(E);
        return st;
    }
    launch_fill_i32(E->counts, g.ne, 0, s);
    launch_fill_i32(E->big_count, 4, 0, s);
    launch_fill_i32(E->idx, cap, 0, s);
    launch_fill_u64(E->cnt, (int64_t)n_problems * NCOUNT * CNT_SLOTS, 0ull, s);
    launch_fill_i32(reinterpret_cast<int32_t*>(E->err), 1, 0, s);
    launch_fill_i32(E->buf[0].elem, cap, -1, s);
    launch_fill_i32(E->buf[1].elem, cap, -1, s);
    std::vector<int64_t> meta(8, 0);
    meta[0] = n0;
    meta[1] = n0;
    HIP_TRY(hipMemcpyAsync(E->d_meta, meta.data(), sizeof(int64_t) * 8, hipMemcpyHostToDevice, s));
    E->n_slots_ub = n0;
    launch_tm(g.geo, g.node, g.ne, E->d_prm, E->tm, s);
    E->cur = 0;
    {
        Timed t(E, T_INIT, s);
        if (E->precision == PDF_MIXED) launch_init_any<float>(E, n0, s);
        else launch_init_any<double>(E, n0, s);
    }
    HIP_TRY(hipGetLastError());
    st = regroup_any(E, false, false, false, s);
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
    for (int p = 0; p < E->n_problems; ++p)
        if (!(dt[p] > 0.0) || !std::isfinite(dt[p])) {
            set_error("pdf_step: dt must be positive and finite");
            return PDF_E_INVAL;
        }
    HIP_TRY(hipSetDevice(E->grid->device));
    hipStream_t s = as_stream(hip_stream);
    E->stream = s;
    pdf_status st = set_dt(E, dt, s);
    if (st != PDF_OK) return st;
    if (E->use_graph && n_steps > 0) {
        st = graph_steps(E, n_steps, s);
        if (st != PDF_OK) return st;
    } else {
        for (int32_t it = 0; it < n_steps; ++it) {
            st = step_any(E, s);
            if (st != PDF_OK) return st;
        }
    }
    if (n_steps > 0) E->ctl_valid = true;   // canonical order of the last element pass
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

// the selected columns of the statistics of nodes [0, nn) into out[nn][k]
__global__ void __launch_bounds__(256) k_stats_select(const double* __restrict__ src, int64_t nn, uint32_t mask,
                                                     int k, double* __restrict__ out)
{
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= nn * k) return;
    const int64_t n = i / k;
    int c = (int)(i - n * k), j = 0;
    for (;; ++j)
        if (((mask >> j) & 1u) && c-- == 0) break;
    out[i] = src[n * NSTAT + j];
}

pdf_status pdf_stats(pdf_ens E, int32_t problem, uint32_t stat_mask, double* out, int32_t out_is_device,
                     void* hip_stream)
{
    if (!E || !out || problem < 0 || problem >= E->n_problems || stat_mask == 0u ||
        (stat_mask & ~(uint32_t)PDF_STATS_ALL) != 0u) {
        set_error("pdf_stats: invalid argument (problem, output or stat_mask)");
        return PDF_E_INVAL;
    }
    HIP_TRY(hipSetDevice(E->grid->device));
    hipStream_t s = as_stream(hip_stream);
    const ProbParams& P = E->h_prm[problem];
    const int k = __builtin_popcount(stat_mask);
    const double* src = E->stats + P.noff * NSTAT;
    if (out_is_device) {
        if (k == NSTAT) {
            HIP_TRY(hipMemcpyAsync(out, src, sizeof(double) * (size_t)P.nn * NSTAT, hipMemcpyDeviceToDevice, s));
        } else if (P.nn > 0) {
            hipLaunchKernelGGL(k_stats_select, dim3((unsigned)((P.nn * k + 255) / 256)), dim3(256), 0, s, src, P.nn,
                               stat_mask, k, out);
            HIP_TRY(hipGetLastError());
        }
        return PDF_OK;
    }
    if (k == NSTAT) {
        HIP_TRY(hipMemcpyAsync(out, src, sizeof(double) * (size_t)P.nn * NSTAT, hipMemcpyDeviceToHost, s));
        HIP_TRY(hipStreamSynchronize(s));
        return check_device_error(E);
    }
    // a subset of the columns: selected on the device into a temporary, then copied
    if (P.nn == 0) return check_device_error(E);
    struct Tmp {
        double* p = nullptr;
        ~Tmp()
        {
            if (p) (void)hipFree(p);
        }
    } tmp;
    if (hipMalloc((void**)&tmp.p, sizeof(double) * (size_t)P.nn * k) != hipSuccess) {
        (void)hipGetLastError();
        tmp.p = nullptr;
        set_error("pdf_stats: device allocation of the selected columns failed");
        return PDF_E_NOMEM;
    }
    hipLaunchKernelGGL(k_stats_select, dim3((unsigned)((P.nn * k + 255) / 256)), dim3(256), 0, s, src, P.nn, stat_mask,
                       k, tmp.p);
    HIP_TRY(hipGetLastError());
    HIP_TRY(hipMemcpyAsync(out, tmp.p, sizeof(double) * (size_t)P.nn * k, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    return check_device_error(E);
}

pdf_status pdf_redistribute(pdf_ens E, int32_t problem, int32_t n_min, int64_t* moves_out, void* hip_stream)
{
    if (moves_out) *moves_out = 0;
    if (!E || n_min < 0 || problem < -1 || problem >= E->n_problems) {
        set_error("pdf_redistribute: need n_min >= 0 and -1 <= problem < n_problems");
        return PDF_E_INVAL;
    }
    HIP_TRY(hipSetDevice(E->grid->device));
    hipStream_t s = as_stream(hip_stream);
    E->stream = s;
    if (!E->ctl_valid) {
        set_error("pdf_redistribute: no element pass since the last control or redistribution");
        return PDF_E_STATE;
    }
    int64_t meta[5];
    HIP_TRY(hipMemcpyAsync(meta, E->d_meta, sizeof(meta), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    E->step = meta[4];   // the device's step counter (steps replayed from a caller's graph included)
    pdf_status st = check_device_error(E);
    if (st != PDF_OK) return st;
    std::vector<int> probs;
    for (int p = 0; p < E->n_problems; ++p)
        if (problem < 0 || p == problem) probs.push_back(p);
    int64_t total = 0;
    st = redistribution_plan(E, probs, n_min, (uint32_t)E->step, &E->redist_plan, &E->redist_cap, &total, s);
    if (st != PDF_OK) return st;
    st = E->precision == PDF_MIXED ? apply_redistribution<float>(E, total, s)
                                   : apply_redistribution<double>(E, total, s);
    if (st != PDF_OK) return st;
    if (total > 0) E->ctl_valid = false;
    if (moves_out) *moves_out = total;
    return check_device_error(E);
}

pdf_status pdf_elliptic_relaxation(pdf_ens E, const pdf_elliptic_model* consts, double tol, int32_t max_iter,
                                   int32_t store, double* wp_out, int32_t out_is_device, int32_t* iters_out,
                                   void* hip_stream)
{
    if (iters_out) *iters_out = 0;
    if (!E || E->n_problems != 1 || !(tol > 0.0) || !(tol < 1.0) || max_iter < 0) {
        set_error("pdf_elliptic_relaxation: one problem, 0 < tol < 1, max_iter >= 0");
        return PDF_E_INVAL;
    }
    pdf_elliptic_model c = consts ? *consts : pdf_elliptic_model{1.85, 0.63, 0.134, 72.0, 1.4, 0.1};
    if (!std::isfinite(c.C1) || !std::isfinite(c.C2) || !(c.CL > 0.0) || !(c.Ceta >= 0.0) || !std::isfinite(c.Cv) ||
        !std::isfinite(c.gamma5) || !std::isfinite(c.CL) || !std::isfinite(c.Ceta)) {
        set_error("pdf_elliptic_relaxation: invalid constants");
        return PDF_E_INVAL;
    }
    HIP_TRY(hipSetDevice(E->grid->device));
    hipStream_t s = as_stream(hip_stream);
    HIP_TRY(hipStreamSynchronize(E->stream));
    E->stream = s;
    pdf_status st = fem_geometry(E, s);
    if (st == PDF_OK) st = fem_work(E);
    if (st == PDF_OK && store) st = ensure_own_fields(E, s);
    if (st == PDF_OK) st = fem_check(E, s, "pdf_elliptic_relaxation");
    if (st != PDF_OK) return st;
    FemState& F = E->fem;
    const DevGrid& g = E->dg;
    const ModelC& m = E->grid->model;
    EllipticConst ec{c.C1, c.C2, c.CL, c.Ceta, c.Cv, c.gamma5, m.nu, m.CT};
    fem_elliptic_inputs(g.geo, g.n2e_ptr, g.n2e, E->stats, g.nn, g.ne, ec, F.wkind, F.wnrm, F.enrm, F.f, F.xfix,
                        F.fixed, F.L2, E->err, s);
    FemOp op = fem_op(E, 1.0, 1.0, F.L2, F.fixed);
    fem_mass_rhs(op, F.f, F.b, s);
    // the operator on the grid's CSR pattern: assembled once per solve (L^2 changes with
    // the statistics), then applied a thread per row and component
    st = fem_pressure_matrix(E, s);
    if (st != PDF_OK) return st;
    if (!F.cval4) {
        st = dalloc(&F.cval4, 4 * F.csr_nnz);
        if (st != PDF_OK) return st;
    }
    op.crp = F.csr_rp;
    op.ccol = F.csr_col;
    op.nnz = F.csr_nnz;
    fem_assemble4(op, F.cval4, s);
    op.cval = F.cval4;
    launch_fill_u64(reinterpret_cast<unsigned long long*>(F.x), 9 * g.nn, 0ull, s);
    fem_set_fixed(F.xfix, F.fixed, g.nn, F.x, s);
    st = fem_cg<9>(E, op, F.b, tol, max_iter, iters_out, s);
    if (st != PDF_OK) return st;
    if (store) {
        if (!E->wp_full) drop_graphs(E);   // captured steps run the six-component particle loop
        E->wp_full = true;
        fem_store_wp(F.x, g.nn, E->dg.node, s);
        if (g.node32) launch_f64_to_f32(g.node, g.node32, g.nn * NODE_STRIDE, s);
        HIP_TRY(hipGetLastError());
    }
    if (wp_out) {
        const size_t bytes = sizeof(double) * 9 * g.nn;
        HIP_TRY(hipMemcpyAsync(wp_out, F.x, bytes, out_is_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost, s));
    }
    HIP_TRY(hipStreamSynchronize(s));
    return check_device_error(E);
}

pdf_status pdf_pressure_projection(pdf_ens E, double dt, double cp, double tol, int32_t max_iter, double* dp_out,
                                   int32_t out_is_device, int32_t* iters_out, void* hip_stream)
{
    if (iters_out) *iters_out = 0;
    if (!E || E->n_problems != 1 || !(dt > 0.0) || !std::isfinite(dt) || !(cp >= 0.0) || !std::isfinite(cp) ||
        !(tol > 0.0) || !(tol < 1.0) || max_iter < 0) {
        set_error("pdf_pressure_projection: one problem, dt > 0, cp >= 0, 0 < tol < 1, max_iter >= 0");
        return PDF_E_INVAL;
    }
    HIP_TRY(hipSetDevice(E->grid->device));
    hipStream_t s = as_stream(hip_stream);
    HIP_TRY(hipStreamSynchronize(E->stream));
    E->stream = s;
    pdf_status st = ensure_own_fields(E, s);
    if (st == PDF_OK) st = fem_work(E);
    FemState& F = E->fem;
    const DevGrid& g = E->dg;
    const int64_t nn = g.nn, ne = g.ne;
    if (st == PDF_OK) st = fem_alloc(F.P, nn);
    if (st == PDF_OK) st = fem_alloc(F.gp0, 2 * nn);
    if (st == PDF_OK) st = fem_alloc(F.gP, 2 * ne);
    if (st == PDF_OK) st = fem_alloc(F.gdP, 2 * ne);
    if (st == PDF_OK) st = fem_pressure_matrix(E, s);
    if (st == PDF_OK) fem_pressure_amg(E, s);
    if (st == PDF_OK) st = fem_check(E, s, "pdf_pressure_projection");
    if (st != PDF_OK) return st;
    if (!F.pressure) {
        // the set-up mean-pressure gradient is the imposed part; P starts at zero
        launch_fill_u64(reinterpret_cast<unsigned long long*>(F.P), nn, 0ull, s);
        HIP_TRY(hipMemcpy2DAsync(F.gp0, 2 * sizeof(double), g.node + NF_GP, NODE_STRIDE * sizeof(double),
                                 2 * sizeof(double), nn, hipMemcpyDeviceToDevice, s));
        F.pressure = true;
    }
    const double rho = E->grid->model.rho;
    FemOp op = fem_op(E, 0.0, 1.0, nullptr, F.nofix);
    fem_pressure_rhs(op, E->stats, F.P, rho, dt, cp, F.b, E->err, s);
    // compatibility with the constant null space: remove the mean of the right-hand side
    fem_dot<1>(F.b, nullptr, nullptr, nullptr, nn, F.partial, F.sc, s);
    fem_sub_mean(F.sc, nn, F.b, s);
    launch_fill_u64(reinterpret_cast<unsigned long long*>(F.x), nn, 0ull, s);
    st = fem_cg_csr(E, F.b, tol, max_iter, iters_out, s);
    if (st != PDF_OK) return st;
    // the solution with zero nodal sum
    fem_dot<1>(F.x, nullptr, nullptr, nullptr, nn, F.partial, F.sc, s);
    fem_sub_mean(F.sc, nn, F.x, s);
    fem_elem_grad(g.geo, F.x, ne, F.gdP, s);
    fem_add(F.x, nn, F.P, s);
    fem_elem_grad(g.geo, F.P, ne, F.gP, s);
    const double scale = dt / rho;
    fem_pressure_update(g.n2e_ptr, g.n2e, F.gP, F.gdP, F.gp0, nn, scale, E->dg.node, E->stats, s);
    if (E->precision == PDF_MIXED)
        fem_correct_particles<float>(cur(E).as<float>(), E->d_meta, E->n_slots_ub, F.gdP, scale, s);
    else
        fem_correct_particles<double>(cur(E).as<double>(), E->d_meta, E->n_slots_ub, F.gdP, scale, s);
    if (g.node32) launch_f64_to_f32(g.node, g.node32, nn * NODE_STRIDE, s);
    // with statistics feedback on, the corrected mean velocity is the one fed back
    if (E->fb_on) apply_feedback(E, s);
    HIP_TRY(hipGetLastError());
    if (dp_out)
        HIP_TRY(hipMemcpyAsync(dp_out, F.x, sizeof(double) * nn,
                               out_is_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    return check_device_error(E);
}

pdf_status pdf_control(pdf_ens E, int32_t n_min, int32_t n_max, pdf_control_report* report, void* hip_stream)
{
    if (!E || n_min < 0 || n_max < 1 || n_max < n_min) {
        set_error("pdf_control: need 0 <= n_min <= n_max and n_max >= 1");
        return PDF_E_INVAL;
    }
    HIP_TRY(hipSetDevice(E->grid->device));
    hipStream_t s = as_stream(hip_stream);
    E->stream = s;
    if (!E->ctl_valid) {
        set_error("pdf_control: no element pass since the last control");
        return PDF_E_STATE;
    }
    // the first wavefront tier of the element pass holds the upper bound: after control
    // nearly every element is at or below it, and the few that the next particle loop
    // pushes above take the next tier (fewer particles per lane: fewer live registers and
    // rows to rank; a tier that most elements fall past would cost a second sweep)
    const int hint = std::min(E->ppl, n_max > 64 * 6 ? 8 : (n_max + 63) / 64);
    if (hint != E->ppl_min) {
        E->ppl_min = hint;
        set_tiers(E);
        drop_graphs(E);   // captured steps launch the old tiers
    }
    return E->precision == PDF_MIXED ? control_impl<float>(E, n_min, n_max, report, s)
                                     : control_impl<double>(E, n_min, n_max, report, s);
}

pdf_status pdf_count(pdf_ens E, int32_t problem, int64_t* live)
{
    if (!E || !live || problem < -1 || problem >= E->n_problems) {
        set_error("pdf_count: invalid argument");
        return PDF_E_INVAL;
    }
    HIP_TRY(hipSetDevice(E->grid->device));
    HIP_TRY(hipStreamSynchronize(E->stream));
    if (problem == -1 || E->n_problems == 1) {
        int64_t meta[2];
        HIP_TRY(hipMemcpy(meta, E->d_meta, sizeof(meta), hipMemcpyDeviceToHost));
        *live = meta[1];
        return check_device_error(E);
    }
    const ProbParams& P = E->h_prm[problem];
    hipStream_t s = E->stream;
    launch_fill_u64(E->d_scalar, 1, 0ull, s);
    launch_count_range(cur(E).elem, E->d_meta, E->n_slots_ub, (int32_t)P.eoff, (int32_t)(P.eoff + P.ne),
                       E->d_scalar, s);
    unsigned long long c = 0;
    HIP_TRY(hipMemcpyAsync(&c, E->d_scalar, sizeof(c), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    *live = (int64_t)c;
    return check_device_error(E);
}

pdf_status pdf_particles_export(pdf_ens E, int32_t problem, int64_t cap, double* x, double* y, double* u,
                                double* omega, double* psi, double* w, uint64_t* pid, int32_t* elem, int64_t* n_out,
                                void* hip_stream)
{
    if (!E || problem < 0 || problem >= E->n_problems || cap < 0) {
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
    const ProbParams& P = E->h_prm[problem];
    const int32_t lo = (int32_t)P.eoff, hi = (int32_t)(P.eoff + P.ne);
    SoaRaw& S = cur(E);
    std::vector<int32_t> el(ns);
    if (ns) HIP_TRY(hipMemcpy(el.data(), S.elem, sizeof(int32_t) * ns, hipMemcpyDeviceToHost));
    int64_t live = 0;
    for (int64_t i = 0; i < ns; ++i) live += (el[i] >= lo && el[i] < hi) ? 1 : 0;
    if (n_out) *n_out = live;
    if (live > cap) {
        set_error("pdf_particles_export: output capacity too small");
        return PDF_E_CAPACITY;
    }
    std::vector<double> tmp;
    auto keep = [&](int64_t i) { return el[i] >= lo && el[i] < hi; };
    auto put = [&](const std::vector<double>& src, double* dst, int stride, int comp) {
        int64_t j = 0;
        for (int64_t i = 0; i < ns; ++i)
            if (keep(i)) dst[stride * (j++) + comp] = src[i];
    };
    pdf_status st;
    if (x) {
        tmp.resize(ns);
        if (ns) HIP_TRY(hipMemcpy(tmp.data(), S.x, sizeof(double) * ns, hipMemcpyDeviceToHost));
        put(tmp, x, 1, 0);
    }
    if (y) {
        tmp.resize(ns);
        if (ns) HIP_TRY(hipMemcpy(tmp.data(), S.y, sizeof(double) * ns, hipMemcpyDeviceToHost));
        put(tmp, y, 1, 0);
    }
    const void* comps[3] = {S.u0, S.u1, S.u2};
    for (int c = 0; c < 3 && u; ++c) {
        if ((st = pull_real(E, comps[c], ns, tmp)) != PDF_OK) return st;
        put(tmp, u, 3, c);
    }
    if (omega) {
        if ((st = pull_real(E, S.om, ns, tmp)) != PDF_OK) return st;
        put(tmp, omega, 1, 0);
    }
    if (psi) {
        if ((st = pull_real(E, S.psi, ns, tmp)) != PDF_OK) return st;
        put(tmp, psi, 1, 0);
    }
    if (w) {
        if ((st = pull_real(E, S.w, ns, tmp)) != PDF_OK) return st;
        put(tmp, w, 1, 0);
    }
    if (pid) {
        std::vector<uint64_t> t(ns);
        if (ns) HIP_TRY(hipMemcpy(t.data(), S.pid, sizeof(uint64_t) * ns, hipMemcpyDeviceToHost));
        int64_t j = 0;
        for (int64_t i = 0; i < ns; ++i)
            if (keep(i)) pid[j++] = t[i];
    }
    if (elem) {
        int64_t j = 0;
        for (int64_t i = 0; i < ns; ++i)
            if (keep(i)) elem[j++] = el[i] - lo;
    }
    return check_device_error(E);
}

pdf_status pdf_particles_import(pdf_ens E, int32_t problem, int64_t n, const double* x, const double* y,
                                const double* u, const double* omega, const double* psi, const double* w,
                                const uint64_t* pid, const int32_t* elem, int64_t step, uint64_t next_pid,
                                void* hip_stream)
{
    if (!E || problem != 0 || E->n_problems != 1 || n < 0 || step < 0 ||
        (n > 0 && (!x || !y || !u || !omega || !psi || !w || !pid || !elem))) {
        set_error("pdf_particles_import: invalid argument (single-problem ensembles only)");
        return PDF_E_INVAL;
    }
    if (n > E->cap) {
        set_error("pdf_particles_import: more particles than capacity");
        return PDF_E_CAPACITY;
    }
    const DevGrid& g = E->dg;
    for (int64_t i = 0; i < n; ++i)
        if (elem[i] < 0 || elem[i] >= g.ne) {
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
    HIP_TRY(hipSetDevice(E->grid->device));
    hipStream_t s = as_stream(hip_stream);
    E->stream = s;
    HIP_TRY(hipStreamSynchronize(s));
    drop_graphs(E);
    SoaRaw& S = cur(E);
    launch_fill_i32(S.elem, E->cap, -1, s);
    if (n > 0) {
        pdf_status st;
        std::vector<double> c(n);
        void* comps[3] = {S.u0, S.u1, S.u2};
        for (int comp = 0; comp < 3; ++comp) {
            for (int64_t i = 0; i < n; ++i) c[i] = u[3 * i + comp];
            if ((st = push_real(E, comps[comp], c, s)) != PDF_OK) return st;
        }
        if ((st = push_real(E, S.om, std::vector<double>(omega, omega + n), s)) != PDF_OK) return st;
        if ((st = push_real(E, S.psi, std::vector<double>(psi, psi + n), s)) != PDF_OK) return st;
        if ((st = push_real(E, S.w, std::vector<double>(w, w + n), s)) != PDF_OK) return st;
        HIP_TRY(hipMemcpyAsync(S.x, x, sizeof(double) * n, hipMemcpyHostToDevice, s));
        HIP_TRY(hipMemcpyAsync(S.y, y, sizeof(double) * n, hipMemcpyHostToDevice, s));
        HIP_TRY(hipMemcpyAsync(S.pid, pid, sizeof(uint64_t) * n, hipMemcpyHostToDevice, s));
        HIP_TRY(hipMemcpyAsync(S.elem, elem, sizeof(int32_t) * n, hipMemcpyHostToDevice, s));
    }
    int64_t meta[5] = {n, n, 0, 0, step};
    HIP_TRY(hipMemcpyAsync(E->d_meta, meta, sizeof(meta), hipMemcpyHostToDevice, s));
    launch_fill_i32(E->counts, g.ne, 0, s);
    E->n_slots_ub = n;
    E->step = step;
    E->h_prm[0].next_pid = next_pid;
    HIP_TRY(hipMemcpyAsync(E->d_prm, E->h_prm.data(), sizeof(ProbParams), hipMemcpyHostToDevice, s));
    pdf_status st = regroup_any(E, false, false, false, s);
    if (st != PDF_OK) return st;
    E->ctl_valid = true;
    HIP_TRY(hipStreamSynchronize(s));
    return check_device_error(E);
}

pdf_status pdf_counters(pdf_ens E, int32_t problem, int64_t out[PDF_NCOUNTERS])
{
    if (!E || !out || problem < 0 || problem >= E->n_problems) {
        set_error("pdf_counters: invalid argument");
        return PDF_E_INVAL;
    }
    HIP_TRY(hipSetDevice(E->grid->device));
    HIP_TRY(hipStreamSynchronize(E->stream));
    std::vector<unsigned long long> c(NCOUNT * CNT_SLOTS);
    HIP_TRY(hipMemcpy(c.data(), E->cnt + (size_t)problem * NCOUNT * CNT_SLOTS, sizeof(unsigned long long) * c.size(),
                      hipMemcpyDeviceToHost));
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

pdf_status pdf_set_feedback(pdf_ens E, int32_t enable, double alpha, int32_t feed_rey, void* hip_stream)
{
    if (!E || !std::isfinite(alpha)) {
        set_error("pdf_set_feedback: invalid argument");
        return PDF_E_INVAL;
    }
    HIP_TRY(hipSetDevice(E->grid->device));
    hipStream_t s = as_stream(hip_stream);
    HIP_TRY(hipStreamSynchronize(E->stream));
    drop_graphs(E);
    E->stream = s;
    E->fb_on = enable != 0;
    E->fb_alpha = alpha;
    E->fb_rey = feed_rey & 3;
    if (!enable) return PDF_OK;
    DevGrid& g = E->dg;
    {
        pdf_status st = ensure_own_fields(E, s);
        if (st != PDF_OK) return st;
    }
    if (!E->fb_gn) {
        pdf_status st = dalloc(&E->fb_gn, 6 * g.nn);
        if (st == PDF_OK) st = dalloc(&E->fb_h, 6 * g.ne);
        if (st != PDF_OK) return st;
    }
    apply_feedback(E, s);
    HIP_TRY(hipGetLastError());
    HIP_TRY(hipStreamSynchronize(s));
    return check_device_error(E);
}

pdf_status pdf_cfl_dt(pdf_ens E, int32_t problem, double cfl, double* dt_out, void* hip_stream)
{
    if (!E || !dt_out || problem < 0 || problem >= E->n_problems || !(cfl > 0.0) || !std::isfinite(cfl)) {
        set_error("pdf_cfl_dt: invalid argument");
        return PDF_E_INVAL;
    }
    HIP_TRY(hipSetDevice(E->grid->device));
    hipStream_t s = as_stream(hip_stream);
    HIP_TRY(hipStreamSynchronize(E->stream));
    const ProbParams& P = E->h_prm[problem];
    const DevGrid& g = E->dg;
    union { double d; unsigned long long u; } inf_bits;
    inf_bits.d = std::numeric_limits<double>::infinity();
    launch_fill_u64(E->d_scalar, 1, inf_bits.u, s);
    launch_fill_u64(E->d_scalar + 1, 1, 0ull, s);
    launch_cfl(g.geo, g.n2e_ptr, g.n2e, E->stats, P.noff, P.nn, E->d_scalar, s);
    unsigned long long r[2];
    HIP_TRY(hipMemcpyAsync(r, E->d_scalar, sizeof(r), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    double lmin, zmax;
    std::memcpy(&lmin, &r[0], sizeof(double));
    std::memcpy(&zmax, &r[1], sizeof(double));
    *dt_out = zmax > 0.0 ? cfl * lmin / zmax : 0.0;
    return check_device_error(E);
}

pdf_status pdf_get_options(pdf_ens E, pdf_options* out)
{
    if (!E || !out) {
        set_error("pdf_get_options: null argument");
        return PDF_E_INVAL;
    }
    out->use_graph = E->use_graph ? 1 : 0;
    out->adv_block = E->adv_block;
    out->ppl = E->ppl;
    return PDF_OK;
}

pdf_status pdf_set_options(pdf_ens E, const pdf_options* opt)
{
    if (!E || !opt || (opt->adv_block != 64 && opt->adv_block != 128 && opt->adv_block != 256) ||
        !(opt->ppl >= 1 && opt->ppl <= 8 && opt->ppl != 7)) {
        set_error("pdf_set_options: adv_block must be 64, 128 or 256 and ppl one of 1..6, 8");
        return PDF_E_INVAL;
    }
    HIP_TRY(hipSetDevice(E->grid->device));
    HIP_TRY(hipStreamSynchronize(E->stream));
    if (opt->adv_block != E->adv_block || opt->ppl != E->ppl || (opt->use_graph != 0) != E->use_graph)
        drop_graphs(E);
    E->use_graph = opt->use_graph != 0;
    E->adv_block = opt->adv_block;
    E->ppl = opt->ppl;
    set_tiers(E);
    return PDF_OK;
}

pdf_status pdf_autotune(pdf_ens E, const double* dt, int32_t steps_per_trial, void* hip_stream, pdf_options* chosen,
                        int32_t* n_trials, double* trial_ms)
{
    if (!E || !dt || steps_per_trial < 1) {
        set_error("pdf_autotune: invalid argument");
        return PDF_E_INVAL;
    }
    HIP_TRY(hipSetDevice(E->grid->device));
    hipStream_t s = as_stream(hip_stream);
    pdf_options base{};
    pdf_get_options(E, &base);
    // candidates: particle-loop workgroup size x wavefront capacity of the element pass
    std::vector<pdf_options> cand;
    const int p0 = base.ppl;
    const int ppls[3] = {p0 > 1 ? (p0 == 8 ? 6 : p0 - 1) : 1, p0, p0 >= 6 ? 8 : p0 + 1};
    for (int b : {64, 128, 256})
        for (int q = 0; q < 3; ++q) {
            if (q > 0 && ppls[q] == ppls[q - 1]) continue;
            cand.push_back(pdf_options{base.use_graph, b, ppls[q]});
        }
    hipEvent_t t0, t1;
    HIP_TRY(hipEventCreate(&t0));
    HIP_TRY(hipEventCreate(&t1));
    double best = 1e300;
    pdf_options pick = base;
    int k = 0;
    for (const pdf_options& o : cand) {
        pdf_status st = pdf_set_options(E, &o);
        if (st == PDF_OK) st = pdf_step(E, dt, 1, hip_stream);   // warm-up, captures graphs
        if (st != PDF_OK) {
            (void)hipEventDestroy(t0);
            (void)hipEventDestroy(t1);
            return st;
        }
        (void)hipEventRecord(t0, s);
        st = pdf_step(E, dt, steps_per_trial, hip_stream);
        (void)hipEventRecord(t1, s);
        if (st == PDF_OK && hipEventSynchronize(t1) != hipSuccess) st = PDF_E_HIP;
        float ms = 0.f;
        (void)hipEventElapsedTime(&ms, t0, t1);
        if (st != PDF_OK) {
            (void)hipEventDestroy(t0);
            (void)hipEventDestroy(t1);
            return st;
        }
        if (trial_ms && n_trials && k < *n_trials) trial_ms[k] = ms;
        ++k;
        if (ms < best) {
            best = ms;
            pick = o;
        }
    }
    (void)hipEventDestroy(t0);
    (void)hipEventDestroy(t1);
    if (n_trials) *n_trials = k;
    pdf_status st = pdf_set_options(E, &pick);
    if (st != PDF_OK) return st;
    if (chosen) *chosen = pick;
    return check_device_error(E);
}

}  // extern "C"
