// Kernels of libpdfgpu (gfx950).  One time step is
//   k_advance      per particle: P1 interpolation, GLM velocity and frequency SDEs, move,
//                  next-best-element walk with wall conditions, source; counts particles
//                  per new host element (wavefront-aggregated atomics)
//   k_scan_*       exclusive scan of the counts -> element segment starts
//   k_scatter      per particle: slot inside its element's segment (grouping by element)
//   k_element_pass per element: sort-and-divide velocity binning in LDS, bin means, IECM
//                  mixing, shape-weighted partial sums per vertex, write the element's
//                  particles in canonical order into the other state buffer
//   k_node_finalize per node: fixed-order sum of the vertex partials -> statistics
// and number control is k_ctl_plan (merges), a scan, and k_ctl_apply (splits).
// The particle kernels are templates on the state precision R (double: FP64 form, float:
// mixed form); the particle loop also on whether the ensemble holds several problems.
#include "device.h"
#include "kernels.h"

namespace pdfgpu {

// =====================================================================================
// advance + track (Eqs. 7, 10/27, 11, 18-20; Secs. 3.6, 3.8, 4.1.2)
// =====================================================================================

// fall-back search of Sec. 3.6 (Fig. 2): elements around the nodes of element c, nodes in
// vertex order, elements ascending; returns the first that contains P and the x offset
// into its frame
__device__ __noinline__ bool fallback_search(const ElemGeo* __restrict__ geo, const int64_t* __restrict__ n2e_ptr,
                                             const int32_t* __restrict__ n2e, int32_t c, double x, double y,
                                             int32_t& found, double& off)
{
    const ElemGeo* G = geo + c;
    for (int v = 0; v < 3; ++v) {
        const int32_t node = G->node[v];
        const int64_t j0 = n2e_ptr[node], j1 = n2e_ptr[node + 1];
        for (int64_t j = j0; j < j1; ++j) {
            const int32_t ent = n2e[j];
            const int32_t fe = ent / 3, slot = ent - 3 * fe;
            if (fe == c) continue;
            const double o = geo[fe].x[slot] - G->x[v];
            double na, nb, nc;
            area_coords(geo + fe, x + o, y, na, nb, nc);
            if (na >= 0.0 && nb >= 0.0 && nc >= 0.0) {
                found = fe;
                off = o;
                return true;
            }
        }
    }
    return false;
}

// Where the particle loop takes a particle's problem parameters from: the single problem's
// copy in the kernel arguments, the table entry of each lane's problem, or the table entry
// of the problem that all lanes of the wavefront share (a wave-uniform index, so the
// parameters are scalar loads)
enum { PM_ONE = 0, PM_LANE = 1, PM_WAVE = 2 };
// The table is read through the constant address space: it does not change during the
// loop, and through a generic pointer the compiler would have to assume that the loop's
// own stores may overwrite it, and load the parameters into vector registers.
typedef const __attribute__((address_space(4))) ProbParams ConstProb;

struct AdvEvents {
    int ev_a, ev_b, omrefl, clamp, src, steps, refl, fb;
    int resample;   // the frequency is drawn again after the loop (no-slip event)
};

// One particle of the particle loop with the parameters P of its problem.  Returns its new
// host element (its old one when it could not be tracked).  DEFER: a particle whose walk
// reaches a wall or free-slip edge is left untouched and -2 returned, for the full loop of
// k_advance_redo (the fall-back search and the reflections are rare, and their call and
// registers would set the budget of the whole loop).  R = double: FP64 throughout;
// R = float: velocity, frequency and their SDEs in FP32, positions and tracking in FP64.
// WPFULL: the nodal wp field has all nine components (stored by the elliptic-relaxation
// solve); otherwise it is symmetric and the three lower components are not read
template <class R, bool WPFULL, bool DEFER, class PP>
__device__ __forceinline__ int32_t advance_one(const AdvanceArgs<R>& a, const int64_t i, const int32_t e,
                                               const uint32_t step, AdvEvents& ev, const PP& P)
{
    using M = RMath<R>;
    const R nu = (R)P.m.nu, rho = (R)P.m.rho, C3 = (R)P.m.C3, C4 = (R)P.m.C4, CT = (R)P.m.CT,
            Cw1 = (R)P.m.Cw1, Cw2 = (R)P.m.Cw2;
    const R dt = (R)P.dt;
    const double x0 = a.s.x[i], y0 = a.s.y[i];
    const R u0 = a.s.u0[i], u1 = a.s.u1[i], u2 = a.s.u2[i];
    const R om = a.s.om[i];
    const uint64_t pid = a.s.pid[i];

    // (a1) P1 interpolation of the nodal fields (Eq. 37); area coordinates in FP64.
    // The lanes of a wavefront mostly share one or two elements (particles are in
    // canonical order): loop over the distinct elements, so that element and node records
    // are wave-uniform scalar loads instead of per-lane vector loads.
    R f[NODE_STRIDE], gu[6];
    {
        unsigned long long todo = __ballot(true);
        while (todo) {
            const int src = __ffsll((long long)todo) - 1;
            const int32_t eu = __builtin_amdgcn_readfirstlane(__shfl(e, src));
            todo &= ~__ballot(e == eu);
            if (e == eu) {
                const ElemGeo* Gu = a.geo + eu;
                double na, nb, nc;
                area_coords(Gu, x0, y0, na, nb, nc);
                const double ia = Gu->inv_area;
                // statistics as element averages of the nodal values (second estimator of
                // Sec. 3.3) or P1 interpolation (Eq. 37)
                const bool avg = P.estimator == 1;
                const R la = avg ? R(1) / R(3) : (R)(na * ia), lb = avg ? R(1) / R(3) : (R)(nb * ia),
                        lc = avg ? R(1) / R(3) : (R)(nc * ia);
                const R* __restrict__ FA = a.node + (int64_t)Gu->node[0] * NODE_STRIDE;
                const R* __restrict__ FB = a.node + (int64_t)Gu->node[1] * NODE_STRIDE;
                const R* __restrict__ FC = a.node + (int64_t)Gu->node[2] * NODE_STRIDE;
                // fields in groups of eight (the last one shorter with the six-component wp);
                // the empty asm statements keep the compiler from loading all node values
                // into scalar registers at once (groups of 8 measured faster than 7 or 11).
                // Explicit fused multiply-adds fix the rounding whatever the operands'
                // registers.
                auto ip = [&](int q) { return fma(lc, FC[q], fma(lb, FB[q], la * FA[q])); };
#pragma unroll
                for (int q = 0; q < 8; ++q) f[q] = ip(q);
                asm volatile("" ::: "memory");
#pragma unroll
                for (int q = 8; q < 16; ++q) f[q] = ip(q);
                asm volatile("" ::: "memory");
#pragma unroll
                for (int q = 16; q < (WPFULL ? 24 : 21); ++q) f[q] = ip(q);
#pragma unroll
                for (int q = 0; q < 6; ++q) gu[q] = (R)Gu->gu[q];
            }
        }
    }
    const R gu0 = gu[0], gu1 = gu[1], gu2 = gu[2], gu3 = gu[3], gu4 = gu[4], gu5 = gu[5];

    // (a2) closure (Eqs. 11, 18, 20)
    const R R11 = f[NF_RE], R22 = f[NF_RE + 1], R33 = f[NF_RE + 2];
    const R R12 = f[NF_RE + 3], R13 = f[NF_RE + 4], R23 = f[NF_RE + 5];
    const R Om = f[NF_OM];
    const R k = R(0.5) * (R11 + R22 + R33);
    const R eps = Om * (k + nu * CT * CT * Om);
    const R prod = -(R11 * gu0 + R12 * gu1 + R12 * gu2 + R22 * gu3 + R13 * gu4 + R23 * gu5);
    const R W11 = f[NF_WP], W22 = f[NF_WP + 1], W33 = f[NF_WP + 2];
    const R W12 = f[NF_WP + 3], W13 = f[NF_WP + 4], W23 = f[NF_WP + 5];
    const R W21 = WPFULL ? f[NF_WPT] : W12, W31 = WPFULL ? f[NF_WPT + 1] : W13, W32 = WPFULL ? f[NF_WPT + 2] : W23;
    const R wpR = W11 * R11 + W22 * R22 + W33 * R33 + ((W12 + W21) * R12 + (W13 + W31) * R13 + (W23 + W32) * R23);
    R c0eps = -R(2) * wpR / (R(3) * k);
    if (c0eps < R(0)) {
        c0eps = R(0);
        ev.clamp = 1;
    }
    const R Sw = Cw2 - Cw1 * prod / eps;
    const R ik = R(1) / k;
    const R G11 = (W11 - R(0.5) * eps) * ik, G22 = (W22 - R(0.5) * eps) * ik, G33 = (W33 - R(0.5) * eps) * ik;
    const R G12 = W12 * ik, G13 = W13 * ik, G23 = W23 * ik;
    const R G21 = W21 * ik, G31 = W31 * ik, G32 = W32 * ik;

    // random numbers: 6 Gaussians and one uniform (Sec. 3.9)
    const RngKey key{P.key.k0, P.key.k1};
    const Words4 wA = rng_draw(key, pid, step, TAG_STEP, 0);
    const Words4 wB = rng_draw(key, pid, step, TAG_STEP, 1);
    R z0, z1, z2, z3, z4, z5;
    M::normal2(wA.w0, wA.w1, z0, z1);
    M::normal2(wA.w2, wA.w3, z2, z3);
    M::normal2(wB.w0, wB.w1, z4, z5);
    // FP64: the host's correctly rounded values (the same as computing them here)
    const R sdt = sizeof(R) == sizeof(double) ? (R)P.sdt : M::sqrt_(dt);
    const R dWx = sdt * z0, dWy = sdt * z1;
    const R dWp0 = sdt * z2, dWp1 = sdt * z3, dWp2 = sdt * z4, dWo = sdt * z5;
    const R s2nu = sizeof(R) == sizeof(double) ? (R)P.s2nu : M::sqrt_(R(2) * nu);
    const R sc0 = M::sqrt_(c0eps);

    // velocity, Eq. (27)
    const R d0 = u0 - f[NF_MU], d1 = u1 - f[NF_MU + 1], d2 = u2 - f[NF_MU + 2];
    const R irho = sizeof(R) == sizeof(double) ? (R)P.irho : R(1) / rho;
    const R dr0 = -f[NF_GP] * irho + R(2) * nu * f[NF_LAP] + G11 * d0 + G12 * d1 + G13 * d2;
    const R dr1 = -f[NF_GP + 1] * irho + R(2) * nu * f[NF_LAP + 1] + G21 * d0 + G22 * d1 + G23 * d2;
    const R dr2 = R(2) * nu * f[NF_LAP + 2] + G31 * d0 + G32 * d1 + G33 * d2;
    R v0 = u0 + dr0 * dt + s2nu * (gu0 * dWx + gu1 * dWy) + sc0 * dWp0;
    R v1 = u1 + dr1 * dt + s2nu * (gu2 * dWx + gu3 * dWy) + sc0 * dWp1;
    R v2 = u2 + dr2 * dt + s2nu * (gu4 * dWx + gu5 * dWy) + sc0 * dWp2;
    // frequency, Eq. (19): |omega| in the diffusion, reflected at zero
    const R aom = om < R(0) ? -om : om;
    R omn = om - C3 * Om * (om - Om) * dt - Sw * Om * om * dt + M::sqrt_(R(2) * C3 * C4 * Om * Om * aom) * dWo;
    if (omn < R(0)) {
        omn = -omn;
        ev.omrefl = 1;
    }
    // position, Eq. (7), with the start-of-step velocity, in FP64 in both forms (the mixed
    // form widens its FP32 velocity and Gaussian and scales them by the FP64 dt, sqrt(dt)
    // and sqrt(2 nu), so the displacement carries no FP32 rounding of its own)
    double x, y;
    if constexpr (sizeof(R) == sizeof(double)) {
        x = x0 + u0 * P.dt + s2nu * dWx;
        y = y0 + u1 * P.dt + s2nu * dWy;
    } else {
        x = x0 + (double)u0 * P.dt + P.s2nu * (P.sdt * (double)z0);
        y = y0 + (double)u1 * P.dt + P.s2nu * (P.sdt * (double)z1);
    }

    // (a3) next-best-element walk (Sec. 3.6) with particle wall conditions (Sec. 3.8)
    int32_t c = e;
    double shift = 0.0;
    bool found = false;
    int wall_a = 0;
    for (int it = 0; it < 64; ++it) {
        const ElemGeo* C = a.geo + c;
        double ma, mb, mc;
        area_coords(C, x, y, ma, mb, mc);
        if (ma >= 0.0 && mb >= 0.0 && mc >= 0.0) {
            found = true;
            break;
        }
        int kk = 0;
        double mn = ma;
        if (mb < mn) {
            kk = 1;
            mn = mb;
        }
        if (mc < mn) kk = 2;
        const uint8_t kd = C->kind[kk];
        if (kd == KIND_INTERIOR) {
            c = C->nbr[kk];
            ++ev.steps;
            continue;
        }
        if (kd == KIND_PERIODIC) {
            x += C->shift[kk];
            shift += C->shift[kk];
            c = C->nbr[kk];
            ++ev.steps;
            continue;
        }
        if constexpr (DEFER) return -2;
        int32_t fe;
        double off;
        if (fallback_search(a.geo, a.n2e_ptr, a.n2e, c, x, y, fe, off)) {
            c = fe;
            x += off;
            shift += off;
            ++ev.fb;
            continue;
        }
        if (ev.refl == 4) break;
        // mirror across the line of edge kk (vertex kk+1 -> kk+2, interior on the left)
        const int pa = (kk + 1) % 3, pb = (kk + 2) % 3;
        const double ax = C->x[pa], ay = C->y[pa];
        const double ex = C->x[pb] - ax, ey = C->y[pb] - ay;
        const double len = sqrt(ex * ex + ey * ey);
        const double nx = -ey / len, ny = ex / len;
        const double dd = (x - ax) * nx + (y - ay) * ny;
        x = x - 2.0 * dd * nx;
        y = y - 2.0 * dd * ny;
        if (kd == KIND_WALL) {
            wall_a = 1;
        } else {
            const R rnx = (R)nx, rny = (R)ny;
            const R un = v0 * rnx + v1 * rny;
            v0 = v0 - R(2) * un * rnx;
            v1 = v1 - R(2) * un * rny;
        }
        ++ev.refl;
    }
    if (!found) {
        atomicOr(a.err, ERR_LOST);
        return e;   // the particle keeps its start-of-step state
    }
    // no-slip events: (a) crossed the wall; (b) Eq. (53) in wall elements.  The test is a
    // discrete decision on positions: FP64 in both forms.
    bool hit = wall_a != 0;
    const ElemGeo* C = a.geo + c;
    if (!hit && C->wall && P.m.nu * P.dt > 0.0) {
        double dn = (x0 + shift - C->wl[0]) * C->wl[2] + (y0 - C->wl[1]) * C->wl[3];
        double dn1 = (x - C->wl[0]) * C->wl[2] + (y - C->wl[1]) * C->wl[3];
        dn = dn < 0.0 ? 0.0 : dn;
        dn1 = dn1 < 0.0 ? 0.0 : dn1;
        const double fw = exp(-dn * dn1 / (P.m.nu * P.dt));
        if (u01(wB.w2) < fw) {
            hit = true;
            ev.ev_b = 1;
        }
    }
    if (hit) {
        ev.ev_a = wall_a;
        double pa_, pb_, pc_;
        area_coords(C, x, y, pa_, pb_, pc_);
        const R* __restrict__ HA = a.node + (int64_t)C->node[0] * NODE_STRIDE;
        const R* __restrict__ HB = a.node + (int64_t)C->node[1] * NODE_STRIDE;
        const R* __restrict__ HC = a.node + (int64_t)C->node[2] * NODE_STRIDE;
        const bool avg = P.estimator == 1;
        const R omw = avg ? (HA[NF_OM] + HB[NF_OM] + HC[NF_OM]) / R(3)
                          : (R)(pa_ / C->area) * HA[NF_OM] + (R)(pb_ / C->area) * HB[NF_OM] +
                                (R)(pc_ / C->area) * HC[NF_OM];
        v0 = v1 = v2 = R(0);
        // Eq. (58): omega ~ Gamma with this mean, drawn by k_wall_resample (the sampler is
        // kept out of the particle loop, whose register budget it would set)
        omn = omw;
        ev.resample = 1;
    }
    // the slot index passes through an empty asm statement, so that the store addresses are
    // formed here instead of being kept in registers from the loads at the start
    int64_t io = i;
    asm volatile("" : "+v"(io));
    a.s.x[io] = x;
    a.s.y[io] = y;
    a.s.u0[io] = v0;
    a.s.u1[io] = v1;
    a.s.u2[io] = v2;
    a.s.om[io] = omn;
    a.s.elem[io] = c;
    if (P.src_cont) {
        double dx = x - P.src_x, dy = y - P.src_y;
        if (P.period > 0.0) {
            if (dx > 0.5 * P.period) dx -= P.period;
            else if (dx < -0.5 * P.period) dx += P.period;
        }
        if (dx * dx + dy * dy < P.src_r2) {
            a.s.psi[io] = R(1);
            ev.src = 1;
        }
    }
    if (!(isfinite(x) && isfinite(y) && isfinite(v0) && isfinite(v1) && isfinite(v2) && isfinite(omn)))
        atomicOr(a.err, ERR_NONFINITE);
    return c;
}

// event counters of one wavefront: counts of flagged lanes and sums of the walk counts
__device__ __forceinline__ void wave_events(const AdvEvents& ev, int v[NCOUNT])
{
    v[0] = __popcll(__ballot(ev.ev_a != 0));
    v[1] = __popcll(__ballot(ev.ev_b != 0));
    v[4] = __popcll(__ballot(ev.omrefl != 0));
    v[5] = __popcll(__ballot(ev.clamp != 0));
    v[7] = __popcll(__ballot(ev.src != 0));
    v[2] = v[3] = v[6] = 0;
    if (__ballot(ev.steps != 0 || ev.refl != 0 || ev.fb != 0)) {
        v[6] = wave_sum_int(ev.steps);
        v[2] = wave_sum_int(ev.refl);
        v[3] = wave_sum_int(ev.fb);
    }
}

// Event counters: added to one of CNT_SLOTS spread copies per counter (no single hot
// address).  One problem: one workgroup sum per counter.  Several problems: one sum per
// wavefront whose lanes share a problem, single lanes otherwise.
template <int PM>
__device__ __forceinline__ void flush_events(unsigned long long* __restrict__ cnt, const AdvEvents& ev, int prob,
                                             const int64_t wave)
{
    const int lane = lane_id(), wid = threadIdx.x >> 6, nw = blockDim.x >> 6;
    if (PM == PM_ONE) {
        __shared__ int wsum[4][NCOUNT];
        int v[NCOUNT];
        wave_events(ev, v);
        if (lane == 0)
            for (int q = 0; q < NCOUNT; ++q) wsum[wid][q] = v[q];
        __syncthreads();
        if (threadIdx.x < NCOUNT) {
            const int q = threadIdx.x;
            int tot = 0;
            for (int w = 0; w < nw; ++w) tot += wsum[w][q];
            if (tot) atomicAdd(cnt + q * CNT_SLOTS + (blockIdx.x & (CNT_SLOTS - 1)), (unsigned long long)tot);
        }
        return;
    }
    const unsigned long long act = __ballot(prob >= 0);
    if (!act) return;
    const int p0 = __shfl(prob, __ffsll((long long)act) - 1);
    const int slot = (int)(wave & (CNT_SLOTS - 1));
    if (PM == PM_WAVE || !__ballot(prob >= 0 && prob != p0)) {
        int v[NCOUNT];
        wave_events(ev, v);
        if (lane < NCOUNT && v[lane])
            atomicAdd(cnt + ((int64_t)p0 * NCOUNT + lane) * CNT_SLOTS + slot, (unsigned long long)v[lane]);
        return;
    }
    if (prob < 0) return;
    const int own[NCOUNT] = {ev.ev_a != 0, ev.ev_b != 0, ev.refl, ev.fb, ev.omrefl != 0, ev.clamp != 0,
                             ev.steps, ev.src != 0};
    for (int q = 0; q < NCOUNT; ++q)
        if (own[q]) atomicAdd(cnt + ((int64_t)prob * NCOUNT + q) * CNT_SLOTS + slot, (unsigned long long)own[q]);
}

// particles per new host element: runs of equal keys among the lanes share one atomic,
// whose return value plus the lane's place in its run is the particle's arrival rank in
// the element (its offset in the element's segment of the grouped order)
struct HostCount {
    int leader, rank, base;
};
__device__ __forceinline__ HostCount count_new_hosts(int32_t* __restrict__ counts, int32_t key)
{
    HostCount h;
    int len;
    wave_runs(key, h.leader, len, h.rank);
    h.base = 0;
    if (h.rank == 0 && key >= 0) h.base = atomicAdd(counts + key, len);
    return h;
}
__device__ __forceinline__ int arrival_rank(const HostCount& h) { return __shfl(h.base, h.leader) + h.rank; }

// One slot of the particle loop (merged particles are dead slots, elem < 0); i is the slot
// index of the lane, slots beyond the used ones are idle lanes.  PM_WAVE: a wavefront whose
// live lanes hold more than one problem does nothing here and is listed for
// k_advance_mixed_waves, which runs it with PM_LANE.
template <class R, int PM, bool WPFULL, bool DEFER>
__device__ __forceinline__ void particle_slot(const AdvanceArgs<R>& a, const int64_t i)
{
    const int64_t nslots = a.meta[0];
    const uint32_t step = (uint32_t)a.meta[4];
    int32_t key = -1;
    int prob = -1;
    AdvEvents ev = {0, 0, 0, 0, 0, 0, 0, 0, 0};
    int32_t e = -1;
    if (i < nslots) {
        e = a.s.elem[i];
        if (e >= a.ne) {
            atomicOr(a.err, ERR_BADELEM);
            e = -1;
        }
        if constexpr (PM == PM_ONE) {
            if (e >= 0) {
                key = advance_one<R, WPFULL, DEFER>(a, i, e, step, ev, a.p0);
                prob = 0;
            }
        } else if constexpr (PM == PM_LANE) {
            if (e >= 0) {
                prob = a.geo[e].prob;
                key = advance_one<R, WPFULL, DEFER>(a, i, e, step, ev, *(ConstProb*)(a.prm + prob));
            }
        }
    }
    if (PM == PM_WAVE) {
        const int pl = e >= 0 ? a.geo[e].prob : -1;
        const unsigned long long act = __ballot(pl >= 0);
        const int pu = act ? __builtin_amdgcn_readfirstlane(__shfl(pl, __ffsll((long long)act) - 1)) : 0;
        if (__ballot(pl >= 0 && pl != pu)) {
            if (lane_id() == 0) {
                const int k = atomicAdd(a.wave_count, 1);
                if (k < a.wave_cap) a.wave_list[k] = (int32_t)(i >> 6);
                else atomicOr(a.err, ERR_CAPACITY);
            }
            return;
        }
        if (e >= 0) {
            key = advance_one<R, WPFULL, DEFER>(a, i, e, step, ev, *(ConstProb*)(a.prm + pu));
            prob = pu;
        }
    }
    if constexpr (DEFER) {
        // particles left to k_advance_redo: listed (one atomic per wavefront), nothing counted
        const bool redo = key == -2;
        if (redo) {
            key = -1;
            prob = -1;
            ev = AdvEvents{0, 0, 0, 0, 0, 0, 0, 0, 0};
        }
        const unsigned long long rb = __ballot(redo);
        if (rb) {
            const int lane = lane_id();
            int base = 0;
            if (lane == 0) base = atomicAdd(a.redo_count, __popcll(rb));
            base = __shfl(base, 0);
            if (redo) a.redo_list[base + __popcll(rb & ((1ull << lane) - 1ull))] = (int32_t)i;
        }
    }
    // slots whose frequency is drawn again: one atomic per wavefront
    const unsigned long long rm = __ballot(ev.resample != 0);
    if (rm) {
        const int lane = lane_id();
        int base = 0;
        if (lane == 0) base = atomicAdd(a.wall_count, __popcll(rm));
        base = __shfl(base, 0);
        if (ev.resample) a.wall_list[base + __popcll(rm & ((1ull << lane) - 1ull))] = (int32_t)i;
    }
    // the counting atomic is in flight while the event counters are flushed
    const HostCount hc = count_new_hosts(a.counts, key);
    flush_events<PM>(a.cnt, ev, prob, i >> 6);
    const int arrival = arrival_rank(hc);
    if (key >= 0) a.arrival[i] = arrival;
}

// One problem: at least four wavefronts per SIMD (at most 128 registers).  With the fall-back
// search and the reflections left to k_advance_redo and the store addresses formed at the
// stores, the FP64 loop needs 114 registers (4.7 ms on the 8e7-particle channel; 5.17 ms at
// three wavefronts with that code in the loop, whose call took 158 registers and spilled 29
// at four, 8.0 ms) and the mixed loop 90, five wavefronts (3.35 ms; 3.86 ms at four with the
// code in the loop).
template <class R, bool WPFULL>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4)))
k_advance(AdvanceArgs<R> a)
{
    particle_slot<R, PM_ONE, WPFULL, true>(a, (int64_t)blockIdx.x * blockDim.x + threadIdx.x);
}

// Several problems: the wavefronts whose lanes share one problem (all but those across the
// ends of the problems' slot ranges, and some among the clones of number control) read its
// parameters as scalars, which keeps the register budget of the one-problem loop
template <class R>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4)))
k_advance_batched(AdvanceArgs<R> a)
{
    particle_slot<R, PM_WAVE, false, true>(a, (int64_t)blockIdx.x * blockDim.x + threadIdx.x);
}

// ... and the listed wavefronts with each lane's parameters from the table (one wavefront per
// workgroup, grid-stride over the list)
template <class R>
__global__ void __launch_bounds__(64) k_advance_mixed_waves(AdvanceArgs<R> a)
{
    const int n = (int)min((int64_t)*a.wave_count, a.wave_cap);
    for (int w = blockIdx.x; w < n; w += gridDim.x)
        particle_slot<R, PM_LANE, false, false>(a, (int64_t)a.wave_list[w] * 64 + threadIdx.x);
}

// The particles whose walk reached a wall or free-slip edge in k_advance or
// k_advance_batched, advanced again from their unchanged start-of-step state by the full
// loop (fall-back search of Sec. 3.6, reflections of Sec. 3.8): the same counter-based random
// numbers give the same step.  One wavefront per workgroup, grid-stride over the list.
template <class R, int PM, bool WPFULL>
__global__ void __launch_bounds__(64) k_advance_redo(AdvanceArgs<R> a)
{
    const int64_t n = *a.redo_count;
    for (int64_t b = (int64_t)blockIdx.x * 64; b < n; b += (int64_t)gridDim.x * 64) {
        const int64_t j = b + threadIdx.x;
        particle_slot<R, PM, WPFULL, false>(a, j < n ? (int64_t)a.redo_list[j] : INT64_MAX);
    }
}

// Eq. (58) for the particles of the last no-slip events: omega ~ Gamma(1/C4) with the mean
// the particle loop left in omega.  The sampler's accept / reject decisions are FP64 in
// both forms.
template <class R>
__global__ void __launch_bounds__(256) k_wall_resample(SoaT<R> s, const int32_t* __restrict__ list,
                                                       const int32_t* __restrict__ count, const ElemGeo* __restrict__ geo,
                                                       const ProbParams* __restrict__ prm, const int64_t* __restrict__ meta)
{
    const int n = *count;
    const uint32_t step = (uint32_t)meta[4];
    for (int j = blockIdx.x * 256 + threadIdx.x; j < n; j += gridDim.x * 256) {
        const int64_t i = list[j];
        const ProbParams& P = prm[geo[s.elem[i]].prob];
        s.om[i] = (R)gamma_draw<double>(1.0 / P.m.C4, (double)s.om[i], P.key, s.pid[i], step, TAG_WALL_GAMMA);
    }
}

// =====================================================================================
// grouping by element: count (for set-up/import), scan, scatter
// =====================================================================================
__global__ void __launch_bounds__(256) k_count(const int32_t* __restrict__ elem, const int64_t* __restrict__ nslots,
                                               int64_t ne, int32_t* __restrict__ counts, uint32_t* __restrict__ err)
{
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    int32_t key = -1;
    if (i < *nslots) {
        key = elem[i];
        if (key >= ne) {
            atomicOr(err, ERR_BADELEM);
            key = -1;
        }
    }
    int leader, len, rank;
    wave_runs(key, leader, len, rank);
    if (rank == 0 && key >= 0) atomicAdd(counts + key, len);
}

constexpr int SCAN_NT = 256, SCAN_IPT = 8, SCAN_TILE = SCAN_NT * SCAN_IPT;

// block-wide exclusive scan of one int per thread; returns the block total
__device__ __forceinline__ int block_exclusive_scan(int v, int& total)
{
    __shared__ int wsum[SCAN_NT / 64];
    const int lane = lane_id(), wid = threadIdx.x >> 6;
    int inc = v;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const int t = __shfl_up(inc, (unsigned)o);
        if (lane >= o) inc += t;
    }
    if (lane == 63) wsum[wid] = inc;
    __syncthreads();
    int base = 0, tot = 0;
#pragma unroll
    for (int w = 0; w < SCAN_NT / 64; ++w) {
        if (w < wid) base += wsum[w];
        tot += wsum[w];
    }
    __syncthreads();
    total = tot;
    return base + inc - v;
}

__global__ void __launch_bounds__(SCAN_NT) k_scan_reduce(const int32_t* __restrict__ in, int64_t n,
                                                         int32_t* __restrict__ bsum)
{
    const int64_t base = (int64_t)blockIdx.x * SCAN_TILE + (int64_t)threadIdx.x * SCAN_IPT;
    int s = 0;
#pragma unroll
    for (int q = 0; q < SCAN_IPT; ++q)
        if (base + q < n) s += in[base + q];
    int total;
    (void)block_exclusive_scan(s, total);
    if (threadIdx.x == 0) bsum[blockIdx.x] = total;
}

// exclusive scan of nb block sums in place (single block; nb <= SCAN_TILE)
__global__ void __launch_bounds__(SCAN_NT) k_scan_top(int32_t* __restrict__ bsum, int64_t nb)
{
    const int64_t base = (int64_t)threadIdx.x * SCAN_IPT;
    int v[SCAN_IPT];
    int s = 0;
#pragma unroll
    for (int q = 0; q < SCAN_IPT; ++q) {
        v[q] = (base + q < nb) ? bsum[base + q] : 0;
        s += v[q];
    }
    int total;
    int run = block_exclusive_scan(s, total);
#pragma unroll
    for (int q = 0; q < SCAN_IPT; ++q) {
        if (base + q < nb) bsum[base + q] = run;
        run += v[q];
    }
}

__global__ void __launch_bounds__(SCAN_NT) k_scan_apply(const int32_t* __restrict__ in, int64_t n,
                                                        const int32_t* __restrict__ bsum, int32_t* __restrict__ out,
                                                        int64_t nb)
{
    const int64_t base = (int64_t)blockIdx.x * SCAN_TILE + (int64_t)threadIdx.x * SCAN_IPT;
    int v[SCAN_IPT];
    int s = 0;
#pragma unroll
    for (int q = 0; q < SCAN_IPT; ++q) {
        v[q] = (base + q < n) ? in[base + q] : 0;
        s += v[q];
    }
    int total;
    int run = block_exclusive_scan(s, total) + bsum[blockIdx.x];
#pragma unroll
    for (int q = 0; q < SCAN_IPT; ++q) {
        if (base + q < n) out[base + q] = run;
        run += v[q];
    }
    if (blockIdx.x == nb - 1 && threadIdx.x == SCAN_NT - 1) out[n] = run;
}

// Slot of every live particle inside its element's segment; the counts return to zero.
// A workgroup covers SCAT_ROUNDS x 256 consecutive slots: every wavefront issues the
// returning atomics of all its rounds before it waits for the first result.
constexpr int SCAT_ROUNDS = 4;
__global__ void __launch_bounds__(256) k_scatter(const int32_t* __restrict__ elem, const int64_t* __restrict__ nslots,
                                                 int64_t ne, int32_t* __restrict__ counts,
                                                 const int32_t* __restrict__ start, int32_t* __restrict__ idx,
                                                 uint32_t* __restrict__ err)
{
    const int64_t ns = *nslots;
    const int lane = lane_id(), wid = threadIdx.x >> 6;
    const int64_t first = (int64_t)blockIdx.x * (256 * SCAT_ROUNDS) + (int64_t)wid * (64 * SCAT_ROUNDS) + lane;
    int32_t key[SCAT_ROUNDS];
    int leader[SCAT_ROUNDS], len[SCAT_ROUNDS], rank[SCAT_ROUNDS], base[SCAT_ROUNDS];
#pragma unroll
    for (int r = 0; r < SCAT_ROUNDS; ++r) {
        const int64_t i = first + 64 * r;
        key[r] = -1;
        if (i < ns) {
            key[r] = elem[i];
            if (key[r] >= ne) key[r] = -1;
        }
    }
#pragma unroll
    for (int r = 0; r < SCAT_ROUNDS; ++r) {
        wave_runs(key[r], leader[r], len[r], rank[r]);
        base[r] = 0;
        if (rank[r] == 0 && key[r] >= 0) base[r] = atomicSub(counts + key[r], len[r]) - len[r];
    }
#pragma unroll
    for (int r = 0; r < SCAT_ROUNDS; ++r) {
        const int b = __shfl(base[r], leader[r]);
        if (key[r] >= 0) {
            const int64_t lo = start[key[r]], hi = start[key[r] + 1];
            const int64_t slot = lo + (int64_t)b + rank[r];
            if (slot >= lo && slot < hi) idx[slot] = (int32_t)(first + 64 * r);
            else atomicOr(err, ERR_BADELEM);
        }
    }
}

// Slot of every live particle inside its element's segment from the arrival ranks of the
// particle loop (no atomics); the counts are cleared separately.
__device__ __forceinline__ void place_one(const int32_t* __restrict__ start, int32_t* __restrict__ idx,
                                          uint32_t* __restrict__ err, int64_t ne, int64_t i, int32_t e, int32_t r)
{
    if (e < 0 || e >= ne) return;
    const int64_t lo = start[e], hi = start[e + 1];
    const int64_t slot = lo + (int64_t)r;
    if (slot >= lo && slot < hi) idx[slot] = (int32_t)i;
    else atomicOr(err, ERR_BADELEM);
}

// four slots per thread, read as one 16-byte load of each array
__global__ void __launch_bounds__(256) k_place(const int32_t* __restrict__ elem, const int32_t* __restrict__ arrival,
                                               const int64_t* __restrict__ nslots, int64_t n_ub, int64_t ne,
                                               const int32_t* __restrict__ start, int32_t* __restrict__ idx,
                                               uint32_t* __restrict__ err)
{
    const int64_t i0 = ((int64_t)blockIdx.x * 256 + threadIdx.x) * 4;
    const int64_t n = min(n_ub, *nslots);
    if (i0 >= n) return;
    if (i0 + 4 <= n) {
        const int4 e4 = *reinterpret_cast<const int4*>(elem + i0);
        const int4 r4 = *reinterpret_cast<const int4*>(arrival + i0);
        place_one(start, idx, err, ne, i0, e4.x, r4.x);
        place_one(start, idx, err, ne, i0 + 1, e4.y, r4.y);
        place_one(start, idx, err, ne, i0 + 2, e4.z, r4.z);
        place_one(start, idx, err, ne, i0 + 3, e4.w, r4.w);
    } else {
        for (int64_t i = i0; i < n; ++i) place_one(start, idx, err, ne, i, elem[i], arrival[i]);
    }
}

// =====================================================================================
// element pass (Sec. 3.5, App. A, Eqs. 24-25; Sec. 3.3)
// =====================================================================================
// (velocity component, pid) as a pair of integers whose lexicographic order is the
// order of the reals (-0 is first folded onto +0); a strict total order for any bits
struct SortKey {
    uint64_t k;
    uint64_t p;
};
__device__ __forceinline__ uint64_t order_bits(double v)
{
    const uint64_t u = (uint64_t)__double_as_longlong(v + 0.0);
    return (u >> 63) ? ~u : (u | 0x8000000000000000ull);
}
__device__ __forceinline__ uint64_t order_bits(float v)
{
    const uint32_t u = (uint32_t)__float_as_uint(v + 0.0f);
    return (uint64_t)((u >> 31) ? ~u : (u | 0x80000000u));
}
__device__ __forceinline__ bool key_less(const SortKey& a, uint64_t bk, uint64_t bp)
{
    return a.k < bk || (a.k == bk && a.p < bp);
}

// groups per level of the sort-and-divide procedure (App. A; Sec. 3.5 asks for at least m
// particles per bin): level l splits each group into min(b_l, max(1, floor(n / (m P))))
// groups, P the product of the earlier levels' counts, and once a level gets fewer groups
// than requested the later levels take one; returns the number of bins
__device__ __forceinline__ int bin_structure(int n, int b0, int b1, int b2, int m, int& g0, int& g1, int& g2)
{
    const int bl[3] = {b0, b1, b2};
    int g[3];
    long long P = 1;
    bool stopped = false;
    for (int l = 0; l < 3; ++l) {
        long long q = (long long)n / ((long long)m * P);
        if (q < 1) q = 1;
        long long gl = bl[l] < q ? bl[l] : q;
        if (stopped) gl = 1;
        if (gl < bl[l]) stopped = true;
        g[l] = (int)gl;
        P *= gl;
    }
    g0 = g[0];
    g1 = g[1];
    g2 = g[2];
    return (int)P;
}

// floor(a / b) for 0 <= a, 0 < b, both below 2^24: single-precision reciprocal estimate,
// then exact integer correction
__device__ __forceinline__ int div_small(int a, int b)
{
    int q = (int)((float)a * __builtin_amdgcn_rcpf((float)b));
    while (q * b > a) --q;
    while ((q + 1) * b <= a) ++q;
    return q;
}

// keeps a load index inside [0, n): ranks are unique for unique pids, this only guards
// memory safety against corrupted input
__device__ __forceinline__ int clampi(int j, int n) { return j < 0 ? 0 : (j >= n ? n - 1 : j); }

// IECM mixing fraction of element e, Eq. (24): f = min(dt / t_m, 1); 0 when not mixing
__device__ __forceinline__ double mix_fraction(int32_t mix, double dt, double tm)
{
    double f = mix ? dt / tm : 0.0;
    return f > 1.0 ? 1.0 : f;
}

// Plain running sum (the few particles of one lane of the element pass; the lanes' sums are
// then added with the precision's Acc)
template <class R>
struct LaneSum {
    R s = R(0);
    __device__ void add(R v) { s += v; }
    __device__ R value() const { return s; }
};

// Per-vertex partial sums of one particle (Sec. 3.3): weight, shifted first moments and
// shifted products, accumulated with shape-function weight w * lambda_v.
template <class R, class A>
__device__ __forceinline__ void add_partials(A (&acc)[3][NPART], const R (&rs)[3][5], const R lam[3], R w,
                                             R u0, R u1, R u2, R om, R psi)
{
    const R q5[5] = {u0, u1, u2, om, psi};
#pragma unroll
    for (int v = 0; v < 3; ++v) {
        const R wl = w * lam[v];
        R d[5];
#pragma unroll
        for (int q = 0; q < 5; ++q) d[q] = q5[q] - rs[v][q];
        acc[v][0].add(wl);
#pragma unroll
        for (int q = 0; q < 5; ++q) acc[v][1 + q].add(wl * d[q]);
        acc[v][6].add(wl * d[0] * d[0]);
        acc[v][7].add(wl * d[1] * d[1]);
        acc[v][8].add(wl * d[2] * d[2]);
        acc[v][9].add(wl * d[0] * d[1]);
        acc[v][10].add(wl * d[0] * d[2]);
        acc[v][11].add(wl * d[1] * d[2]);
        acc[v][12].add(wl * d[4] * d[4]);
    }
}

// Fox's projection (Eqs. 64-66) from an element's central weighted sums
// cs = {uu 00, 11, 22, 01, 02, 12, u0 phi', u1 phi', u2 phi', phi'^2}, total weight W and the
// largest magnitudes of U_a (umax) and psi (pmax): the standard deviations sd (0 for a
// spread at rounding level) and the projection vector alpha solving rho_ab alpha_b = rho_a
// on the independent components (Cholesky of rho in the order U1, U2, U3, dropping a
// component whose remaining diagonal is at most 1e-12).  The same steps on every lane.
__device__ __noinline__ void fox_alpha(double W, const double (&cs)[10], const double (&umax)[3], double pmax,
                                       double (&alpha)[3], double (&sd)[3])
{
    const int ix[3][3] = {{0, 3, 4}, {3, 1, 5}, {4, 5, 2}};
    double Cuu[3][3], Cup[3];
    for (int a = 0; a < 3; ++a) {
        for (int b = 0; b < 3; ++b) Cuu[a][b] = cs[ix[a][b]] / W;
        Cup[a] = cs[6 + a] / W;
    }
    const double Cpp = cs[9] / W;
    for (int a = 0; a < 3; ++a) {
        sd[a] = sqrt(Cuu[a][a]);
        if (!(sd[a] > 1e-12 * umax[a])) sd[a] = 0.0;
        alpha[a] = 0.0;
    }
    if (!(sqrt(Cpp) > 1e-12 * pmax)) return;
    double rho[3][3], rv[3];
    for (int a = 0; a < 3; ++a) {
        rv[a] = sd[a] > 0.0 ? Cup[a] / (sd[a] * sqrt(Cpp)) : 0.0;
        for (int b = 0; b < 3; ++b) rho[a][b] = (sd[a] > 0.0 && sd[b] > 0.0) ? Cuu[a][b] / (sd[a] * sd[b]) : 0.0;
    }
    int sel[3] = {0, 0, 0}, k = 0;
    double L[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
    for (int a = 0; a < 3; ++a) {
        if (!(sd[a] > 0.0)) continue;
        double l[3] = {0, 0, 0}, dd = rho[a][a];
        for (int i = 0; i < k; ++i) {
            double t = rho[a][sel[i]];
            for (int j = 0; j < i; ++j) t -= L[i][j] * l[j];
            l[i] = t / L[i][i];
            dd -= l[i] * l[i];
        }
        if (!(dd > 1e-12)) continue;
        for (int i = 0; i < k; ++i) L[k][i] = l[i];
        L[k][k] = sqrt(dd);
        sel[k++] = a;
    }
    double z[3] = {0, 0, 0};
    for (int i = 0; i < k; ++i) {
        double t = rv[sel[i]];
        for (int j = 0; j < i; ++j) t -= L[i][j] * z[j];
        z[i] = t / L[i][i];
    }
    for (int i = k - 1; i >= 0; --i) {
        double t = z[i];
        for (int j = i + 1; j < k; ++j) t -= L[j][i] * alpha[sel[j]];
        alpha[sel[i]] = t / L[i][i];
    }
}

// projected velocity of Eq. (64) on the normalised fluctuations
__device__ __forceinline__ double fox_key(const double (&alpha)[3], const double (&sd)[3], const double (&mu)[3],
                                          double u0, double u1, double u2)
{
    const double u[3] = {u0, u1, u2};
    double v = 0.0;
#pragma unroll
    for (int a = 0; a < 3; ++a)
        if (alpha[a] != 0.0) v += alpha[a] * ((u[a] - mu[a]) / sd[a]);
    return v;
}

__device__ __forceinline__ double wave_max_double(double v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o));
    return v;
}

// sums (max != 0: maxima) of k <= 16 values over a workgroup; every thread gets the results
template <int NT>
__device__ __forceinline__ void block_reduce(double* v, int k, bool max, double* scratch)
{
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    for (int q = 0; q < k; ++q) {
        const double t = max ? wave_max_double(v[q]) : wave_sum_double(v[q]);
        if (lane == 0) scratch[wid * 16 + q] = t;
    }
    __syncthreads();
    for (int q = 0; q < k; ++q) {
        double t = 0.0;   // the maxima taken here are of magnitudes
        for (int w = 0; w < NT / 64; ++w) t = max ? fmax(t, scratch[w * 16 + q]) : t + scratch[w * 16 + q];
        v[q] = t;
    }
    __syncthreads();
}

template <int NT, class R>
__device__ __forceinline__ void element_body(const ElementArgs<R>& a, int32_t e, int64_t s0, int n, R* U0, R* U1,
                                             R* U2, uint64_t* PID, SortKey* kp, int32_t* ordA, int32_t* ordB,
                                             R* bmean, R* red)
{
    const int tid = threadIdx.x;
    const ElemGeo* G = a.geo + e;
    const ProbParams& P = a.prm[G->prob];
    // load velocities and pids of the element's particles (load order j)
    for (int j = tid; j < n; j += NT) {
        const int64_t gi = a.idx[s0 + j];
        U0[j] = a.in.u0[gi];
        U1[j] = a.in.u1[gi];
        U2[j] = a.in.u2[gi];
        PID[j] = a.in.pid[gi];
        ordA[j] = j;
    }
    __syncthreads();
    // Fox's projection: element moments, projection vector, projected velocities
    const bool proj = P.conditioning == 1;
    double fmu[3] = {0, 0, 0}, falpha[3] = {0, 0, 0}, fsd[3] = {0, 0, 0};
    if (proj) {
        double* scratch = reinterpret_cast<double*>(red);
        double m[5] = {0, 0, 0, 0, 0}, mx[4] = {0, 0, 0, 0};
        for (int j = tid; j < n; j += NT) {
            const int64_t gi = a.idx[s0 + j];
            const double w = a.in.w[gi], ps = a.in.psi[gi];
            const double u[3] = {U0[j], U1[j], U2[j]};
            m[0] += w;
            for (int c = 0; c < 3; ++c) {
                m[1 + c] += w * u[c];
                mx[c] = fmax(mx[c], fabs(u[c]));
            }
            m[4] += w * ps;
            mx[3] = fmax(mx[3], fabs(ps));
        }
        block_reduce<NT>(m, 5, false, scratch);
        block_reduce<NT>(mx, 4, true, scratch);
        for (int c = 0; c < 3; ++c) fmu[c] = m[1 + c] / m[0];
        const double mp = m[4] / m[0];
        double cs[10] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
        for (int j = tid; j < n; j += NT) {
            const int64_t gi = a.idx[s0 + j];
            const double w = a.in.w[gi];
            const double d0 = (double)U0[j] - fmu[0], d1 = (double)U1[j] - fmu[1], d2 = (double)U2[j] - fmu[2];
            const double dp = (double)a.in.psi[gi] - mp;
            cs[0] += w * d0 * d0;
            cs[1] += w * d1 * d1;
            cs[2] += w * d2 * d2;
            cs[3] += w * d0 * d1;
            cs[4] += w * d0 * d2;
            cs[5] += w * d1 * d2;
            cs[6] += w * d0 * dp;
            cs[7] += w * d1 * dp;
            cs[8] += w * d2 * dp;
            cs[9] += w * dp * dp;
        }
        block_reduce<NT>(cs, 10, false, scratch);
        const double umax[3] = {mx[0], mx[1], mx[2]};
        fox_alpha(m[0], cs, umax, mx[3], falpha, fsd);
    }
    int g0, g1, g2;
    const int Cp = bin_structure(n, P.bins0, proj ? 1 : P.bins1, proj ? 1 : P.bins2, P.minpb, g0, g1, g2);
    const int gl[3] = {g0, g1, g2};
    // three levels: sort every group of the previous level by (U_l, pid) (rank sort); one
    // level by the projected velocity with Fox's projection
    long long C = 1;
    for (int l = 0; l < (proj ? 1 : 3); ++l) {
        const R* Ul = l == 0 ? U0 : (l == 1 ? U1 : U2);
        for (int pos = tid; pos < n; pos += NT) {
            const int j = clampi(ordA[pos], n);
            kp[pos].k = proj ? order_bits(fox_key(falpha, fsd, fmu, U0[j], U1[j], U2[j])) : order_bits(Ul[j]);
            kp[pos].p = PID[j];
        }
        __syncthreads();
        for (int pos = tid; pos < n; pos += NT) {
            const long long t = C * pos / n;
            const int lo = (int)((t * n + C - 1) / C), hi = (int)(((t + 1) * n + C - 1) / C);
            const uint64_t mk = kp[pos].k;
            const uint64_t mp = kp[pos].p;
            int r = 0;
            for (int q = lo; q < hi; ++q) r += key_less(kp[q], mk, mp) ? 1 : 0;
            ordB[lo + (r < hi - lo ? r : hi - lo - 1)] = ordA[pos];
        }
        __syncthreads();
        int32_t* t = ordA;
        ordA = ordB;
        ordB = t;
        C *= gl[l];
    }
    // bin means of psi, weighted (App. A)
    R* wacc = reinterpret_cast<R*>(kp);
    for (int pos = tid; pos < n; pos += NT) {
        const int64_t gi = a.idx[s0 + clampi(ordA[pos], n)];
        const R w = a.in.w[gi];
        wacc[2 * pos] = w * a.in.psi[gi];
        wacc[2 * pos + 1] = w;
    }
    __syncthreads();
    for (int b = tid; b < Cp; b += NT) {
        const int lo = (int)(((long long)b * n + Cp - 1) / Cp), hi = (int)(((long long)(b + 1) * n + Cp - 1) / Cp);
        Acc<R> sw, swp;
        for (int q = lo; q < hi; ++q) {
            swp.add(wacc[2 * q]);
            sw.add(wacc[2 * q + 1]);
        }
        bmean[b] = swp.value() / sw.value();
    }
    __syncthreads();

    // IECM (Eq. 24); statistics partials; canonical write-out
    const R fmix = (R)mix_fraction(a.mix, P.dt, a.tm[e]);
    const double inv_area = G->inv_area;
    const bool est = P.estimator == 1;
    R rs[3][5];
#pragma unroll
    for (int v = 0; v < 3; ++v)
#pragma unroll
        for (int q = 0; q < 5; ++q) rs[v][q] = a.shift[(int64_t)G->node[v] * 5 + q];
    Acc<R> acc[3][NPART];
    for (int pos = tid; pos < n; pos += NT) {
        const int j = clampi(ordA[pos], n);
        const int64_t gi = a.idx[s0 + j];
        const double x = a.in.x[gi], y = a.in.y[gi];
        const R w = a.in.w[gi], om = a.in.om[gi];
        R psi = a.in.psi[gi];
        const R u0 = U0[j], u1 = U1[j], u2 = U2[j];
        const int b = (int)(((long long)Cp * pos) / n);
        psi = psi - fmix * (psi - bmean[b]);
        const int64_t o = s0 + pos;
        a.out.x[o] = x;
        a.out.y[o] = y;
        a.out.u0[o] = u0;
        a.out.u1[o] = u1;
        a.out.u2[o] = u2;
        a.out.om[o] = om;
        a.out.psi[o] = psi;
        a.out.w[o] = w;
        a.out.pid[o] = PID[j];
        a.out.elem[o] = e;
        double na, nb, nc;
        area_coords(G, x, y, na, nb, nc);
        // second estimator: the element's own sums (weight 1 on the first vertex slot)
        const R lam[3] = {est ? R(1) : (R)(na * inv_area), est ? R(0) : (R)(nb * inv_area),
                          est ? R(0) : (R)(nc * inv_area)};
        add_partials<R>(acc, rs, lam, w, u0, u1, u2, om, psi);
    }
    // fixed-order reduction: butterfly inside each wavefront, then waves in order
    const int lane = lane_id(), wid = tid >> 6;
#pragma unroll
    for (int v = 0; v < 3; ++v)
#pragma unroll
        for (int q = 0; q < NPART; ++q) {
            const R s = wave_sum_real<R>(acc[v][q].value());
            if (lane == 0) red[wid * 3 * NPART + v * NPART + q] = s;
        }
    __syncthreads();
    if (tid < 3 * NPART) {
        Acc<R> s;
        for (int w = 0; w < NT / 64; ++w) s.add(red[w * 3 * NPART + tid]);
        R v = s.value();
        // second estimator: the second slot carries the shift of the element's sums
        if (est && tid >= NPART && tid < NPART + 5) v = a.shift[(int64_t)G->node[0] * 5 + (tid - NPART)];
        a.part[(int64_t)e * 3 * NPART + tid] = v;
    }
}

// on-chip layout of the workgroup kernel: [reduction][bin means][keys][pids][U0 U1 U2][ordA ordB]
template <class R>
size_t element_pass_smem(int lds_max)
{
    return (size_t)(EP_NT / 64) * 3 * NPART * sizeof(double) + MAXBINS * sizeof(double) +
           (size_t)lds_max * (sizeof(SortKey) + sizeof(uint64_t) + 3 * sizeof(R) + 2 * sizeof(int32_t));
}

// Elements with more particles than the wavefront kernel holds: one workgroup per element,
// taken from the worklist the wavefront kernel fills (on-chip keys up to lds_max
// particles, global scratch at the element's segment offset above that).
template <int NT, class R>
__global__ void __launch_bounds__(NT) k_element_block(ElementArgs<R> a)
{
    extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
    R* red = reinterpret_cast<R*>(smem);                                   // [NT/64][39]
    R* bmean = reinterpret_cast<R*>(smem + (NT / 64) * 3 * NPART * sizeof(double));   // [MAXBINS]
    unsigned char* p = smem + (NT / 64) * 3 * NPART * sizeof(double) + MAXBINS * sizeof(double);
    const int nbig = *a.big_count;
    const int32_t* big = a.big_list;
    for (int k = blockIdx.x; k < nbig; k += gridDim.x) {
        const int32_t e = big[k];
        const int64_t s0 = a.start[e];
        const int n = a.start[e + 1] - a.start[e];
        if (n <= a.lds_max) {
            const int M = a.lds_max;
            SortKey* kp = reinterpret_cast<SortKey*>(p);
            uint64_t* PID = reinterpret_cast<uint64_t*>(kp + M);
            R* U0 = reinterpret_cast<R*>(PID + M);
            R* U1 = U0 + M;
            R* U2 = U1 + M;
            int32_t* ordA = reinterpret_cast<int32_t*>(U2 + M);
            int32_t* ordB = ordA + M;
            element_body<NT, R>(a, e, s0, n, U0, U1, U2, PID, kp, ordA, ordB, bmean, red);
        } else {
            const int64_t cap = a.cap;
            SortKey* kp = reinterpret_cast<SortKey*>(a.gkey) + s0;
            R* U0 = reinterpret_cast<R*>(a.gu3) + s0;
            R* U1 = reinterpret_cast<R*>(a.gu3) + cap + s0;
            R* U2 = reinterpret_cast<R*>(a.gu3) + 2 * cap + s0;
            uint64_t* PID = reinterpret_cast<uint64_t*>(a.gu3 + 3 * cap) + s0;
            int32_t* ordA = a.gord + s0;
            int32_t* ordB = a.gord + cap + s0;
            element_body<NT, R>(a, e, s0, n, U0, U1, U2, PID, kp, ordA, ordB, bmean, red);
        }
        __syncthreads();
    }
}

// orders LDS traffic between the lanes of one wavefront
__device__ __forceinline__ void wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// wavefronts per workgroup of the wavefront element kernel (two: small workgroups fill the
// CUs more evenly than four, and LDS stays within 64 KiB), and the wavefronts per SIMD the
// register budget is set for (up to five particles per lane fit 128 registers: four
// wavefronts per SIMD)
template <int PPL>
struct WaveBlock {
    static constexpr int waves = 2;
    static constexpr int per_simd = PPL <= 5 ? 4 : 1;
};
// Wavefronts per SIMD of a tier: FP32 state with at most four particles per lane fits 96
// registers, five wavefronts (3.55 -> 3.37 ms on the 8e7-particle channel; the LDS of a
// workgroup allows five); the projection's extra registers would spill there
template <int PPL, class R, bool PROJ>
constexpr int element_wave_occupancy()
{
    return sizeof(R) == sizeof(float) && PPL <= 4 && !PROJ ? 5 : WaveBlock<PPL>::per_simd;
}

// One wavefront per element (up to 64*PPL particles, PPL per lane).  Lanes own particles
// in load order while the three sort levels rank (U_l, pid) keys staged in LDS; then each
// lane takes the particles at canonical positions lane + 64 r, so bin sums, partial sums
// and the coalesced write-out follow the canonical order only.
// Tiers of increasing capacity: a launch takes the elements with n_below < n <= 64 PPL
// (n_below = -1 for the first tier, so empty elements are handled there); the last tier
// puts larger elements on the workgroup kernel's worklist (last != 0).
template <int PPL, class R, bool PROJ>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(element_wave_occupancy<PPL, R, PROJ>())))
k_element_wave(ElementArgs<R> a, int n_below, int last)
{
    constexpr int N = 64 * PPL;
    constexpr int RED = (13 * 65 * 8 + 15) & ~15;         // transposed reduction, padded rows
    // keys, pids, 31-bit keys, claims [24N] / then (w psi, w) pairs [16N] and bin means (at
    // most n bins) [8N] / then the transposed reduction
    constexpr int R1 = (24 * N > RED) ? 24 * N : RED;
    constexpr int WAVE_BYTES = R1 + 4 * N;
    static_assert(WAVE_BYTES % 16 == 0 && R1 % 16 == 0, "16-byte aligned LDS slices");
    constexpr int WPB = WaveBlock<PPL>::waves;
    __shared__ __attribute__((aligned(16))) unsigned char sm[WPB * WAVE_BYTES];
    // wave-uniform values go through readfirstlane so that they live in scalar registers
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
    const int64_t e = (int64_t)blockIdx.x * WPB + wave;
    if (e >= a.ne) return;
    unsigned char* base = sm + wave * WAVE_BYTES;
    uint64_t* kk = reinterpret_cast<uint64_t*>(base);          // [N] keys by position
    uint64_t* kpid = kk + N;                                     // [N] pids by position
    uint32_t* k32 = reinterpret_cast<uint32_t*>(kpid + N);       // [N] 31-bit keys by position
    uint32_t* claim = k32 + N;                                   // [N] rank collision check
    R* wacc = reinterpret_cast<R*>(base);
    R* red = reinterpret_cast<R*>(base);
    int32_t* ord = reinterpret_cast<int32_t*>(base + R1);
    R* bmean = reinterpret_cast<R*>(base + 16 * N);
    const int64_t s0 = __builtin_amdgcn_readfirstlane(a.start[e]);
    const int n = __builtin_amdgcn_readfirstlane(a.start[e + 1]) - (int)s0;
    if (n <= n_below) return;   // an earlier tier's element
    if (n == 0) {
        if (lane < 3 * NPART) a.part[e * 3 * NPART + lane] = R(0);
        return;
    }
    if (n > N) {
        if (last && lane == 0) {
            const int k = atomicAdd(a.big_count, 1);
            a.big_list[k] = (int32_t)e;
        }
        return;
    }
    const ElemGeo* G = a.geo + e;
    const ProbParams& P = a.prm[G->prob];
    // load order: particle j = lane + 64 r
    int gi[PPL], pos[PPL];
    R U0[PPL], U1[PPL], U2[PPL];
    uint64_t pd[PPL];
#pragma unroll
    for (int r = 0; r < PPL; ++r) {
        const int j = lane + 64 * r;
        pos[r] = j;
        gi[r] = 0;
        U0[r] = U1[r] = U2[r] = R(0);
        pd[r] = 0;
        if (j < n) {
            gi[r] = a.idx[s0 + j];
            U0[r] = a.in.u0[gi[r]];
            U1[r] = a.in.u1[gi[r]];
            U2[r] = a.in.u2[gi[r]];
            pd[r] = a.in.pid[gi[r]];
        }
    }
    // Fox's projection (instantiated only for ensembles that use it): element moments by
    // wavefront reductions, the projection vector, and the projected velocities as keys
    const bool proj = PROJ && P.conditioning == 1;
    double fk[PROJ ? PPL : 1];
    if constexpr (PROJ) {
        if (proj) {
            double m[5] = {0, 0, 0, 0, 0}, mx[4] = {0, 0, 0, 0};
            R wq[PPL], pq[PPL];
#pragma unroll
            for (int r = 0; r < PPL; ++r) {
                wq[r] = pq[r] = R(0);
                if (lane + 64 * r < n) {
                    wq[r] = a.in.w[gi[r]];
                    pq[r] = a.in.psi[gi[r]];
                    const double w = wq[r], u[3] = {U0[r], U1[r], U2[r]};
                    m[0] += w;
                    for (int c = 0; c < 3; ++c) {
                        m[1 + c] += w * u[c];
                        mx[c] = fmax(mx[c], fabs(u[c]));
                    }
                    m[4] += w * (double)pq[r];
                    mx[3] = fmax(mx[3], fabs((double)pq[r]));
                }
            }
            for (int q = 0; q < 5; ++q) m[q] = wave_sum_double(m[q]);
            for (int q = 0; q < 4; ++q) mx[q] = wave_max_double(mx[q]);
            const double mu[3] = {m[1] / m[0], m[2] / m[0], m[3] / m[0]};
            const double mp = m[4] / m[0];
            double cs[10] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
#pragma unroll
            for (int r = 0; r < PPL; ++r)
                if (lane + 64 * r < n) {
                    const double w = wq[r];
                    const double d0 = (double)U0[r] - mu[0], d1 = (double)U1[r] - mu[1], d2 = (double)U2[r] - mu[2];
                    const double dp = (double)pq[r] - mp;
                    cs[0] += w * d0 * d0;
                    cs[1] += w * d1 * d1;
                    cs[2] += w * d2 * d2;
                    cs[3] += w * d0 * d1;
                    cs[4] += w * d0 * d2;
                    cs[5] += w * d1 * d2;
                    cs[6] += w * d0 * dp;
                    cs[7] += w * d1 * dp;
                    cs[8] += w * d2 * dp;
                    cs[9] += w * dp * dp;
                }
            for (int q = 0; q < 10; ++q) cs[q] = wave_sum_double(cs[q]);
            double alpha[3], sd[3];
            const double umax[3] = {mx[0], mx[1], mx[2]};
            fox_alpha(m[0], cs, umax, mx[3], alpha, sd);
#pragma unroll
            for (int r = 0; r < PPL; ++r) fk[r] = fox_key(alpha, sd, mu, U0[r], U1[r], U2[r]);
        }
    }
    int g0, g1, g2;
    const int Cp = bin_structure(n, P.bins0, proj ? 1 : P.bins1, proj ? 1 : P.bins2, P.minpb, g0, g1, g2);
    const int gl[3] = {g0, g1, g2};
    long long C = 1;
#pragma unroll
    for (int l = 0; l < 3; ++l) {
        if (proj && l > 0) break;
        if (l == 0) {
            // first level, the whole element one group: exact ranks by a counting pass over
            // 64 buckets of equal width in the key's value (a monotone map: a lower bucket
            // holds only smaller keys), then (key, pid) comparisons inside the particle's
            // own bucket.  Keys in bucket order use kk / kpid; counts and starts use the
            // 31-bit key slice.
            int* hist = reinterpret_cast<int*>(k32);
            int* bst = hist + 64;
            double v[PPL];
            uint64_t mk[PPL];
            double vlo = __builtin_inf(), vhi = -__builtin_inf();
#pragma unroll
            for (int r = 0; r < PPL; ++r) {
                if constexpr (PROJ)
                    v[r] = proj ? fk[r] : (double)U0[r];
                else
                    v[r] = (double)U0[r];
                mk[r] = order_bits(v[r]);
                if (lane + 64 * r < n) {
                    vlo = fmin(vlo, v[r]);
                    vhi = fmax(vhi, v[r]);
                }
            }
            vlo = -wave_max_double(-vlo);
            vhi = wave_max_double(vhi);
            const double span = vhi - vlo;
            const double scale = span > 0.0 ? 64.0 / span : 0.0;
            hist[lane] = 0;
            wave_sync();
            int bk[PPL], off[PPL];
#pragma unroll
            for (int r = 0; r < PPL; ++r) {
                bk[r] = off[r] = 0;
                if (lane + 64 * r < n) {
                    // a product that is not a number (0 x inf when the span underflows)
                    // goes to bucket 0, like the smallest key
                    const double t = (v[r] - vlo) * scale;
                    bk[r] = t >= 63.0 ? 63 : (t > 0.0 ? (int)t : 0);
                    off[r] = atomicAdd(&hist[bk[r]], 1);
                }
            }
            wave_sync();
            const int cnt = hist[lane];
            int inc = cnt;
#pragma unroll
            for (int o = 1; o < 64; o <<= 1) {
                const int t = __shfl_up(inc, o);
                if (lane >= o) inc += t;
            }
            bst[lane] = inc - cnt;
            wave_sync();
#pragma unroll
            for (int r = 0; r < PPL; ++r)
                if (lane + 64 * r < n) {
                    const int q = bst[bk[r]] + off[r];
                    kk[q] = mk[r];
                    kpid[q] = pd[r];
                }
            wave_sync();
#pragma unroll
            for (int r = 0; r < PPL; ++r)
                if (lane + 64 * r < n) {
                    const int q0 = bst[bk[r]], q1 = q0 + hist[bk[r]];
                    int rank = q0;
                    for (int q = q0; q < q1; ++q) {
                        const uint64_t kq = kk[q];
                        rank += (kq < mk[r] || (kq == mk[r] && kpid[q] < pd[r])) ? 1 : 0;
                    }
                    pos[r] = rank;
                }
            wave_sync();
            C *= gl[0];
            continue;
        }
        // later levels: rank inside the groups the previous level formed (group t holds the
        // positions ceil(t n / C) .. ceil((t + 1) n / C) - 1); the groups' first positions in
        // a table, in the slot-order LDS that is free until the hand-over
        int* gb = ord;
        for (int t = lane; t < (int)C; t += 64) gb[t] = div_small(t * n + (int)C - 1, (int)C);
        wave_sync();
        uint64_t mk[PPL];
        int lo[PPL], hi[PPL];
        uint64_t kmin = ~0ull, kmax = 0ull;
#pragma unroll
        for (int r = 0; r < PPL; ++r) {
            mk[r] = order_bits(l == 1 ? U1[r] : U2[r]);
            const int t = div_small((int)C * pos[r], n);
            lo[r] = gb[t];
            hi[r] = t + 1 < (int)C ? gb[t + 1] : n;
            if (lane + 64 * r < n) {
                kmin = mk[r] < kmin ? mk[r] : kmin;
                kmax = mk[r] > kmax ? mk[r] : kmax;
            }
        }
        // 31-bit keys: (key - min) shifted right until the element's span fits; the map is
        // monotone, so ranks by these keys are exact unless two keys fall together, which
        // the slot claim below detects
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) {
            const uint64_t a = __shfl_xor(kmin, o), b = __shfl_xor(kmax, o);
            kmin = a < kmin ? a : kmin;
            kmax = b > kmax ? b : kmax;
        }
        const uint64_t span = kmax - kmin;
        const int sh = (span >> 31) ? 33 - __clzll(span) : 0;
        uint32_t m32[PPL];
#pragma unroll
        for (int r = 0; r < PPL; ++r) {
            m32[r] = (uint32_t)((mk[r] - kmin) >> sh);
            if (lane + 64 * r < n) {
                kk[pos[r]] = mk[r];
                kpid[pos[r]] = pd[r];
                k32[pos[r]] = m32[r];
            }
        }
        wave_sync();
        // rank inside the group by the 31-bit key: a < b is the sign of a - b (both below
        // 2^31), so the comparisons are independent integer operations
        auto lt = [](uint32_t a, uint32_t b) { return (int)((a - b) >> 31); };
        int rk[PPL];
#pragma unroll
        for (int r = 0; r < PPL; ++r) rk[r] = 0;
#pragma unroll
        for (int r = 0; r < PPL; ++r)
            if (lane + 64 * r < n) {
                int q = lo[r];
                for (; q + 4 <= hi[r]; q += 4)
                    rk[r] += lt(k32[q], m32[r]) + lt(k32[q + 1], m32[r]) + lt(k32[q + 2], m32[r]) +
                             lt(k32[q + 3], m32[r]);
                for (; q < hi[r]; ++q) rk[r] += lt(k32[q], m32[r]);
            }
        // equal keys give equal ranks: detect by claiming the slots, then rank exactly
        // by (key, pid) in that case
#pragma unroll
        for (int r = 0; r < PPL; ++r)
            if (lane + 64 * r < n)
                claim[lo[r] + (rk[r] < hi[r] - lo[r] ? rk[r] : hi[r] - lo[r] - 1)] = (uint32_t)(lane + 64 * r);
        wave_sync();
        bool clash = false;
#pragma unroll
        for (int r = 0; r < PPL; ++r)
            if (lane + 64 * r < n)
                clash |= claim[lo[r] + (rk[r] < hi[r] - lo[r] ? rk[r] : hi[r] - lo[r] - 1)] != (uint32_t)(lane + 64 * r);
        if (__ballot(clash)) {
#pragma unroll
            for (int r = 0; r < PPL; ++r) {
                rk[r] = 0;
                if (lane + 64 * r < n)
                    for (int q = lo[r]; q < hi[r]; ++q) {
                        const uint64_t kq = kk[q];
                        rk[r] += (kq < mk[r] || (kq == mk[r] && kpid[q] < pd[r])) ? 1 : 0;
                    }
            }
        }
        wave_sync();
#pragma unroll
        for (int r = 0; r < PPL; ++r) {
            const int np = lo[r] + (rk[r] < hi[r] - lo[r] ? rk[r] : hi[r] - lo[r] - 1);
            if (lane + 64 * r < n) pos[r] = np;
        }
        C *= gl[l];
    }
    // hand over to canonical order: slot of the particle at each position.  With FP32 state
    // and at least three particles per lane the velocities and pids also move to their
    // canonical lanes through the sort's LDS instead of a second global read (measured
    // 4.41 -> 4.08 ms on channel_large, 23.9 -> 19.6 ms on the large street canyon once the
    // lanes sum their particles plainly); with FP64 state the extra live registers spill
    // (4.69 -> 4.82 ms), so the global read is kept there, and so it is for three per lane
    // with the projection, whose registers would spill.
    constexpr bool PERM = sizeof(R) == sizeof(float) && (PPL >= 4 || (PPL == 3 && !PROJ));
#pragma unroll
    for (int r = 0; r < PPL; ++r)
        if (lane + 64 * r < n) ord[pos[r]] = gi[r];
    R cu0[PPL], cu1[PPL], cu2[PPL];
    uint64_t cpd[PPL];
    if constexpr (PERM) {
        R* lu = reinterpret_cast<R*>(base);
#pragma unroll
        for (int r = 0; r < PPL; ++r)
            if (lane + 64 * r < n) {
                lu[pos[r]] = U0[r];
                lu[N + pos[r]] = U1[r];
                lu[2 * N + pos[r]] = U2[r];
            }
        wave_sync();
#pragma unroll
        for (int r = 0; r < PPL; ++r) {
            const int p = lane + 64 * r;
            cu0[r] = cu1[r] = cu2[r] = R(0);
            if (p < n) {
                cu0[r] = lu[p];
                cu1[r] = lu[N + p];
                cu2[r] = lu[2 * N + p];
            }
        }
        wave_sync();
        uint64_t* lp = reinterpret_cast<uint64_t*>(base);
#pragma unroll
        for (int r = 0; r < PPL; ++r)
            if (lane + 64 * r < n) lp[pos[r]] = pd[r];
        wave_sync();
#pragma unroll
        for (int r = 0; r < PPL; ++r) {
            const int p = lane + 64 * r;
            cpd[r] = p < n ? lp[p] : 0ull;
        }
    }
    wave_sync();
    int gp[PPL];
    R ws[PPL], ps[PPL];
#pragma unroll
    for (int r = 0; r < PPL; ++r) {
        const int p = lane + 64 * r;
        gp[r] = 0;
        ws[r] = ps[r] = R(0);
        if (p < n) {
            gp[r] = ord[p];
            ws[r] = a.in.w[gp[r]];
            ps[r] = a.in.psi[gp[r]];
            wacc[2 * p] = ws[r] * ps[r];
            wacc[2 * p + 1] = ws[r];
        }
    }
    wave_sync();
    // bin means of psi, weighted (App. A)
    for (int b = lane; b < Cp; b += 64) {
        const int lo = div_small(b * n + Cp - 1, Cp), hi = div_small((b + 1) * n + Cp - 1, Cp);
        Acc<R> sw, swp;
        for (int q = lo; q < hi; ++q) {
            swp.add(wacc[2 * q]);
            sw.add(wacc[2 * q + 1]);
        }
        bmean[b] = swp.value() / sw.value();
    }
    wave_sync();

    const R fmix = (R)mix_fraction(a.mix, P.dt, a.tm[e]);
    const double inv_area = G->inv_area;
    const bool est = P.estimator == 1;
    R rs[3][5];
#pragma unroll
    for (int v = 0; v < 3; ++v)
#pragma unroll
        for (int q = 0; q < 5; ++q) rs[v][q] = a.shift[(int64_t)G->node[v] * 5 + q];
    // each lane adds its (at most PPL) particles plainly; the 64 lane sums are added with Acc
    // below (Kahan-compensated in FP32)
    LaneSum<R> acc[3][NPART];
#pragma unroll
    for (int r = 0; r < PPL; ++r) {
        const int p = lane + 64 * r;
        if (p >= n) continue;
        const int64_t g = gp[r];
        const double x = a.in.x[g], y = a.in.y[g];
        const R om = a.in.om[g];
        const R u0 = PERM ? cu0[r] : a.in.u0[g], u1 = PERM ? cu1[r] : a.in.u1[g], u2 = PERM ? cu2[r] : a.in.u2[g];
        const uint64_t pid = PERM ? cpd[r] : a.in.pid[g];
        const int b = div_small(Cp * p, n);
        const R psi = ps[r] - fmix * (ps[r] - bmean[b]);
        const R w = ws[r];
        const int64_t o = s0 + p;
        a.out.x[o] = x;
        a.out.y[o] = y;
        a.out.u0[o] = u0;
        a.out.u1[o] = u1;
        a.out.u2[o] = u2;
        a.out.om[o] = om;
        a.out.psi[o] = psi;
        a.out.w[o] = w;
        a.out.pid[o] = pid;
        a.out.elem[o] = (int32_t)e;
        double na, nb, nc;
        area_coords(G, x, y, na, nb, nc);
        // second estimator: the element's own sums (weight 1 on the first vertex slot)
        const R lam[3] = {est ? R(1) : (R)(na * inv_area), est ? R(0) : (R)(nb * inv_area),
                          est ? R(0) : (R)(nc * inv_area)};
        add_partials<R>(acc, rs, lam, w, u0, u1, u2, om, psi);
    }
    // fixed-order wavefront reduction through LDS: row q holds the 64 lanes' values
#pragma unroll
    for (int v = 0; v < 3; ++v) {
#pragma unroll
        for (int q = 0; q < NPART; ++q) red[q * 65 + lane] = acc[v][q].value();
        wave_sync();
        if (lane < NPART) {
            Acc<R> s;
            for (int l = 0; l < 64; ++l) s.add(red[lane * 65 + l]);
            R val = s.value();
            // second estimator: the second slot carries the shift of the element's sums
            if (est && v == 1 && lane < 5) val = a.shift[(int64_t)G->node[0] * 5 + lane];
            a.part[e * 3 * NPART + v * NPART + lane] = val;
        }
        wave_sync();
    }
}

// =====================================================================================
// node finalize (Sec. 3.3): fixed-order sum over the elements around the node
// =====================================================================================
template <class R>
__global__ void __launch_bounds__(256) k_node_finalize(NodeArgs<R> a)
{
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i == 0) {
        a.meta[0] = a.start[a.ne];   // used slots after compaction
        a.meta[1] = a.start[a.ne];   // live particles
        if (a.advance_step) a.meta[4] += 1;   // step counter of the random streams
        a.big_count[0] = 0;          // worklist of large elements, empty for the next pass
        a.big_count[1] = 0;          // list of no-slip resamples, empty for the next step
        a.big_count[2] = 0;          // list of wavefronts with several problems, the same
        a.big_count[3] = 0;          // list of particles for the full particle loop, the same
    }
    if (i >= a.nn) return;
    if (a.estimator == 1) {
        // second estimator of Sec. 3.3: plain average over the surrounding elements with
        // particles of the element means (shift + sum / W) and central moments
        double W = 0.0, Sm[5] = {0, 0, 0, 0, 0}, Sc[7] = {0, 0, 0, 0, 0, 0, 0};
        int K = 0;
        for (int64_t j = a.n2e_ptr[i]; j < a.n2e_ptr[i + 1]; ++j) {
            const R* pp = a.part + (int64_t)(a.n2e[j] / 3) * 3 * NPART;
            const double We = (double)pp[0];
            W += We;
            if (!(We > 0.0)) continue;
            ++K;
            double d[5];
            for (int q = 0; q < 5; ++q) {
                d[q] = (double)pp[1 + q] / We;
                Sm[q] += (double)pp[NPART + q] + d[q];
            }
            Sc[0] += (double)pp[6] / We - d[0] * d[0];
            Sc[1] += (double)pp[7] / We - d[1] * d[1];
            Sc[2] += (double)pp[8] / We - d[2] * d[2];
            Sc[3] += (double)pp[9] / We - d[0] * d[1];
            Sc[4] += (double)pp[10] / We - d[0] * d[2];
            Sc[5] += (double)pp[11] / We - d[1] * d[2];
            Sc[6] += (double)pp[12] / We - d[4] * d[4];
        }
        double* o = a.stats + i * NSTAT;
        R* r = a.shift + i * 5;
        o[0] = W;
        if (K == 0) {
            const double nan = __builtin_nan("");
            for (int q = 1; q < NSTAT; ++q) o[q] = nan;
            return;
        }
        for (int q = 0; q < 5; ++q) {
            o[1 + q] = Sm[q] / (double)K;
            r[q] = (R)o[1 + q];
        }
        for (int q = 0; q < 7; ++q) o[6 + q] = Sc[q] / (double)K;
        return;
    }
    Acc<R> S[NPART];
    for (int64_t j = a.n2e_ptr[i]; j < a.n2e_ptr[i + 1]; ++j) {
        const R* pp = a.part + (int64_t)a.n2e[j] * NPART;
#pragma unroll
        for (int q = 0; q < NPART; ++q) S[q].add(pp[q]);
    }
    // the division by the nodal weight and the moments are FP64 in both forms
    double* o = a.stats + i * NSTAT;
    R* r = a.shift + i * 5;
    const double W = (double)S[0].value();
    o[0] = W;
    if (W == 0.0) {
        const double nan = __builtin_nan("");
        for (int q = 1; q < NSTAT; ++q) o[q] = nan;
        for (int q = 0; q < 5; ++q) r[q] = R(0);
        return;
    }
    double d[5];
#pragma unroll
    for (int q = 0; q < 5; ++q) d[q] = (double)S[1 + q].value() / W;
#pragma unroll
    for (int q = 0; q < 5; ++q) o[1 + q] = (double)r[q] + d[q];
    o[6] = (double)S[6].value() / W - d[0] * d[0];
    o[7] = (double)S[7].value() / W - d[1] * d[1];
    o[8] = (double)S[8].value() / W - d[2] * d[2];
    o[9] = (double)S[9].value() / W - d[0] * d[1];
    o[10] = (double)S[10].value() / W - d[0] * d[2];
    o[11] = (double)S[11].value() / W - d[1] * d[2];
    o[12] = (double)S[12].value() / W - d[4] * d[4];
#pragma unroll
    for (int q = 0; q < 5; ++q) r[q] = (R)o[1 + q];
}

// =====================================================================================
// set-up (Sec. 3.7): ppe particles per element of every problem
// =====================================================================================
template <class R>
__global__ void __launch_bounds__(256) k_init(InitArgs<R> a)
{
    using M = RMath<R>;
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= a.n) return;
    // problem of slot i: the last one whose first slot is <= i
    int lo = 0, hi = a.n_problems - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (a.prm[mid].soff <= i) lo = mid;
        else hi = mid - 1;
    }
    const ProbParams& P = a.prm[lo];
    const int64_t k = i - P.soff;
    const int32_t e = (int32_t)(P.eoff + k / P.ppe);
    const ElemGeo* G = a.geo + e;
    const uint64_t pid = (uint64_t)k;
    const Words4 wA = rng_draw(P.key, pid, 0, TAG_INIT, 0);
    const Words4 wB = rng_draw(P.key, pid, 0, TAG_INIT, 1);
    // uniform point in the element (positions are FP64 in both forms)
    double s = u01(wA.w0), t = u01(wA.w1);
    if (s + t > 1.0) {
        s = 1.0 - s;
        t = 1.0 - t;
    }
    const double x = G->x[0] + s * (G->x[1] - G->x[0]) + t * (G->x[2] - G->x[0]);
    const double y = G->y[0] + s * (G->y[1] - G->y[0]) + t * (G->y[2] - G->y[0]);
    double na, nb, nc;
    area_coords(G, x, y, na, nb, nc);
    const bool avg = P.estimator == 1;
    const R la = avg ? R(1) / R(3) : (R)(na * G->inv_area), lb = avg ? R(1) / R(3) : (R)(nb * G->inv_area),
            lc = avg ? R(1) / R(3) : (R)(nc * G->inv_area);
    const R* FA = a.node + (int64_t)G->node[0] * NODE_STRIDE;
    const R* FB = a.node + (int64_t)G->node[1] * NODE_STRIDE;
    const R* FC = a.node + (int64_t)G->node[2] * NODE_STRIDE;
    R z0, z1, z2, z3;
    M::normal2(wA.w2, wA.w3, z0, z1);
    M::normal2(wB.w0, wB.w1, z2, z3);
    const R mu0 = la * FA[NF_MU] + lb * FB[NF_MU] + lc * FC[NF_MU];
    const R mu1 = la * FA[NF_MU + 1] + lb * FB[NF_MU + 1] + lc * FC[NF_MU + 1];
    const R mu2 = la * FA[NF_MU + 2] + lb * FB[NF_MU + 2] + lc * FC[NF_MU + 2];
    const R omm = la * FA[NF_OM] + lb * FB[NF_OM] + lc * FC[NF_OM];
    const R sig = (R)P.u_sigma;
    a.s.x[i] = x;
    a.s.y[i] = y;
    a.s.u0[i] = mu0 + sig * z0;
    a.s.u1[i] = mu1 + sig * z1;
    a.s.u2[i] = mu2 + sig * z2;
    a.s.om[i] = (R)gamma_draw<double>(P.omega_shape, (double)omm, P.key, pid, 0, TAG_INIT_GAMMA);
    double dx = x - P.src_x, dy = y - P.src_y;
    if (P.period > 0.0) {
        if (dx > 0.5 * P.period) dx -= P.period;
        else if (dx < -0.5 * P.period) dx += P.period;
    }
    a.s.psi[i] = (dx * dx + dy * dy < P.src_r2) ? R(1) : R(0);
    a.s.w[i] = R(1);
    a.s.pid[i] = pid;
    a.s.elem[i] = e;
}

// micromixing timescale per element, Eq. (25) at the centroid (FP64 in both forms)
__global__ void __launch_bounds__(256) k_tm(const ElemGeo* __restrict__ geo, const double* __restrict__ node,
                                            int64_t ne, const ProbParams* __restrict__ prm, double* __restrict__ tm)
{
    const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (e >= ne) return;
    const ElemGeo* G = geo + e;
    const ProbParams& P = prm[G->prob];
    const ModelC& m = P.m;
    const double src_r = sqrt(P.src_r2);
    const double* A = node + (int64_t)G->node[0] * NODE_STRIDE;
    const double* B = node + (int64_t)G->node[1] * NODE_STRIDE;
    const double* C = node + (int64_t)G->node[2] * NODE_STRIDE;
    auto cen = [&](int q) { return (A[q] + B[q] + C[q]) / 3.0; };
    const double k = 0.5 * (cen(NF_RE) + cen(NF_RE + 1) + cen(NF_RE + 2));
    const double Om = cen(NF_OM);
    const double eps = Om * (k + m.nu * m.CT * m.CT * Om);
    const double m0 = cen(NF_MU), m1 = cen(NF_MU + 1), m2 = cen(NF_MU + 2);
    const double Uc = sqrt(m0 * m0 + m1 * m1 + m2 * m2);
    const double cx = (G->x[0] + G->x[1] + G->x[2]) / 3.0, cy = (G->y[0] + G->y[1] + G->y[2]) / 3.0;
    double dx = cx - P.src_x, dy = cy - P.src_y;
    if (P.period > 0.0) {
        if (dx > 0.5 * P.period) dx -= P.period;
        else if (dx < -0.5 * P.period) dx += P.period;
    }
    const double dist = sqrt(dx * dx + dy * dy);
    const double first = Uc > 0.0 ? m.Cs * cbrt(src_r * src_r / eps) + m.Ct * dist / Uc : __builtin_inf();
    const double second = fmax(k / eps, m.CT * sqrt(m.nu / eps));
    tm[e] = fmin(first, second);
}

// =====================================================================================
// number control (Sec. 3.7, App. B)
// =====================================================================================
template <class R>
__global__ void __launch_bounds__(256) k_ctl_plan(ControlArgs<R> a)
{
    const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
    int merged = 0, empty = 0, below = 0, above = 0;
    if (e < a.ne) {
        const int64_t s0 = a.start[e];
        const int n = a.start[e + 1] - a.start[e];
        int c = 0;
        if (n == 0) {
            empty = 1;
        } else if (n < a.n_min) {
            below = 1;
            c = (a.n_min - n) < n ? (a.n_min - n) : n;
        } else if (n > a.n_max) {
            above = 1;
            const ProbParams& P = a.prm[a.geo[e].prob];
            int g0, g1, g2;
            const int Cp = bin_structure(n, P.bins0, P.bins1, P.bins2, P.minpb, g0, g1, g2);
            const int want = n - a.n_max;
            for (int j = 0; merged < want; ++j) {
                bool any = false;
                for (int b = 0; b < Cp && merged < want; ++b) {
                    const long long first = ((long long)b * n + Cp - 1) / Cp;
                    const long long size = ((long long)(b + 1) * n + Cp - 1) / Cp - first;
                    if (size < 2LL * j + 2) continue;
                    any = true;
                    const int64_t r = s0 + first + 2 * j, v = r + 1;
                    const R wr = a.s.w[r], wv = a.s.w[v];
                    const R W = wr + wv;
                    a.s.u0[r] = (wr * a.s.u0[r] + wv * a.s.u0[v]) / W;
                    a.s.u1[r] = (wr * a.s.u1[r] + wv * a.s.u1[v]) / W;
                    a.s.u2[r] = (wr * a.s.u2[r] + wv * a.s.u2[v]) / W;
                    a.s.om[r] = (wr * a.s.om[r] + wv * a.s.om[v]) / W;
                    a.s.psi[r] = (wr * a.s.psi[r] + wv * a.s.psi[v]) / W;
                    a.s.w[r] = W;
                    a.s.elem[v] = -1;
                    ++merged;
                }
                if (!any) break;
            }
        }
        a.clone[e] = c;
    }
    const int sm = wave_sum_int(merged), se = wave_sum_int(empty), sb = wave_sum_int(below),
              sa = wave_sum_int(above);
    if (lane_id() == 0) {
        if (sm) atomicAdd(a.rep + 0, (unsigned long long)sm);
        if (se) atomicAdd(a.rep + 1, (unsigned long long)se);
        if (sb) atomicAdd(a.rep + 2, (unsigned long long)sb);
        if (sa) atomicAdd(a.rep + 3, (unsigned long long)sa);
    }
}

// splits: clones appended after the used slots; new pids continue the problem's numbering
// in element order
template <class R>
__global__ void __launch_bounds__(256) k_ctl_apply(ControlArgs<R> a)
{
    const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (e >= a.ne) return;
    const int c = a.clone[e];
    if (c == 0) return;
    const ProbParams& P = a.prm[a.geo[e].prob];
    const int64_t s0 = a.start[e];
    const int64_t n = a.start[e + 1] - a.start[e];
    const int64_t base = *a.nslots + a.off[e];
    const uint64_t pid0 = P.next_pid + (uint64_t)(a.off[e] - a.off[P.eoff]);
    for (int i = 0; i < c; ++i) {
        const int64_t src = s0 + ((2LL * i + 1) * n) / (2LL * c);
        const int64_t dst = base + i;
        if (dst >= a.cap) {
            atomicOr(a.err, ERR_CAPACITY);
            continue;
        }
        const R w = R(0.5) * a.s.w[src];
        a.s.w[src] = w;
        a.s.x[dst] = a.s.x[src];
        a.s.y[dst] = a.s.y[src];
        a.s.u0[dst] = a.s.u0[src];
        a.s.u1[dst] = a.s.u1[src];
        a.s.u2[dst] = a.s.u2[src];
        a.s.om[dst] = a.s.om[src];
        a.s.psi[dst] = a.s.psi[src];
        a.s.w[dst] = w;
        a.s.pid[dst] = pid0 + (uint64_t)i;
        a.s.elem[dst] = (int32_t)e;
    }
}

// slots and live count after control, the clone total, and every problem's next pid.
// Clones are written in the order of their offsets, so when the capacity cut them short
// the ones that exist are the first room = cap - slots of that order: a prefix of every
// problem's range, whose pids stay contiguous.
__global__ void k_ctl_finish(int64_t* __restrict__ meta, const int32_t* __restrict__ off, int64_t ne,
                             const unsigned long long* __restrict__ rep, int64_t cap, ProbParams* __restrict__ prm,
                             int32_t n_problems)
{
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    const int64_t total = off[ne];
    const int64_t room = cap - meta[0] > 0 ? cap - meta[0] : 0;
    const int64_t made = total < room ? total : room;
    meta[0] += made;
    meta[1] = meta[1] - (int64_t)rep[0] + made;
    meta[2] = made;
    for (int p = 0; p < n_problems; ++p) {
        const int64_t lo = off[prm[p].eoff], hi = off[prm[p].eoff + prm[p].ne];
        const int64_t fit = made - lo < 0 ? 0 : (made - lo > hi - lo ? hi - lo : made - lo);
        prm[p].next_pid += (uint64_t)fit;
    }
}

// Particle redistribution (App. B), applied in two passes so that a slot that serves as a
// copy source and also receives a new state is read before it is written.
// plan[4 i ..]: destination slot, position source (slot, or -(e + 1) for the centroid of
// element e), property source slot (velocity, frequency, scalar), new element.
template <class R>
__global__ void __launch_bounds__(256) k_redist_gather(SoaT<R> s, SoaT<R> stage, const int32_t* __restrict__ plan,
                                                       const ElemGeo* __restrict__ geo, int64_t m)
{
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= m) return;
    const int32_t xs = plan[4 * i + 1], ps = plan[4 * i + 2];
    double x, y;
    if (xs >= 0) {
        x = s.x[xs];
        y = s.y[xs];
    } else {
        const ElemGeo& G = geo[-(int64_t)xs - 1];
        x = (G.x[0] + G.x[1] + G.x[2]) / 3.0;
        y = (G.y[0] + G.y[1] + G.y[2]) / 3.0;
    }
    stage.x[i] = x;
    stage.y[i] = y;
    stage.u0[i] = s.u0[ps];
    stage.u1[i] = s.u1[ps];
    stage.u2[i] = s.u2[ps];
    stage.om[i] = s.om[ps];
    stage.psi[i] = s.psi[ps];
}

template <class R>
__global__ void __launch_bounds__(256) k_redist_write(SoaT<R> s, SoaT<R> stage, const int32_t* __restrict__ plan,
                                                      int64_t m)
{
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= m) return;
    const int32_t d = plan[4 * i];
    s.x[d] = stage.x[i];
    s.y[d] = stage.y[i];
    s.u0[d] = stage.u0[i];
    s.u1[d] = stage.u1[i];
    s.u2[d] = stage.u2[i];
    s.om[d] = stage.om[i];
    s.psi[d] = stage.psi[i];
    s.elem[d] = plan[4 * i + 3];
}

__global__ void __launch_bounds__(256) k_fill_i32(int32_t* __restrict__ p, int64_t n, int32_t v)
{
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i < n) p[i] = v;
}

__global__ void __launch_bounds__(256) k_fill_u64(unsigned long long* __restrict__ p, int64_t n,
                                                  unsigned long long v)
{
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i < n) p[i] = v;
}

__global__ void __launch_bounds__(256) k_f64_to_f32(const double* __restrict__ in, float* __restrict__ out, int64_t n)
{
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i < n) out[i] = (float)in[i];
}

__global__ void __launch_bounds__(256) k_f32_to_f64(const float* __restrict__ in, double* __restrict__ out, int64_t n)
{
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i < n) out[i] = (double)in[i];
}

// live particles whose element lies in [lo, hi) (the particles of one problem)
__global__ void __launch_bounds__(256) k_count_range(const int32_t* __restrict__ elem,
                                                     const int64_t* __restrict__ nslots, int32_t lo, int32_t hi,
                                                     unsigned long long* __restrict__ out)
{
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    int in = 0;
    if (i < *nslots) {
        const int32_t e = elem[i];
        in = (e >= lo && e < hi) ? 1 : 0;
    }
    const int c = __popcll(__ballot(in != 0));
    if (lane_id() == 0 && c) atomicAdd(out, (unsigned long long)c);
}

// initial shift of the single-pass moments: the frozen <U>, <omega> and psi = 0
template <class R>
__global__ void __launch_bounds__(256) k_shift_init(const R* __restrict__ node, int64_t nn, R* __restrict__ shift)
{
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= nn) return;
    const R* F = node + i * NODE_STRIDE;
    shift[i * 5 + 0] = F[NF_MU];
    shift[i * 5 + 1] = F[NF_MU + 1];
    shift[i * 5 + 2] = F[NF_MU + 2];
    shift[i * 5 + 3] = F[NF_OM];
    shift[i * 5 + 4] = R(0);
}

// =====================================================================================
// statistics feedback (Sec. 3.1, Table 1 order: a step uses the statistics of the step
// before): nodal fields from the last statistics, then the derived fields again
// =====================================================================================
// nodal <U> <- alpha * mean velocity; R <- Reynolds stresses (trace > 0); nodes without
// particles keep their fields
// rey: bit 0 feeds the Reynolds stresses (where their trace is positive), bit 1 the mean
// frequency (where positive)
__global__ void __launch_bounds__(256) k_fb_nodes(const double* __restrict__ stats, double* __restrict__ node,
                                                  int64_t nn, double alpha, int32_t rey)
{
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= nn) return;
    const double* o = stats + i * NSTAT;
    double* f = node + i * NODE_STRIDE;
    if (!(o[0] > 0.0)) return;
    for (int q = 0; q < 3; ++q) f[NF_MU + q] = alpha * o[1 + q];
    if ((rey & 1) && o[6] + o[7] + o[8] > 0.0)
        for (int q = 0; q < 6; ++q) f[NF_RE + q] = o[6 + q];
    if ((rey & 2) && o[4] > 0.0) f[NF_OM] = o[4];
}

// gradient of a P1 field from its vertex values (Eqs. 39-40), in the element's frame
__device__ __forceinline__ void p1_grad(const ElemGeo& G, double qa, double qb, double qc, double& gx, double& gy)
{
    const double xba = G.x[1] - G.x[0], xca = G.x[2] - G.x[0];
    const double yba = G.y[1] - G.y[0], yca = G.y[2] - G.y[0];
    const double inv2a = 1.0 / (2.0 * G.area);
    gx = inv2a * ((yba - yca) * qa + yca * qb - yba * qc);
    gy = inv2a * ((xca - xba) * qa - xca * qb + xba * qc);
}

__global__ void __launch_bounds__(256) k_fb_grad(ElemGeo* __restrict__ geo, const double* __restrict__ node, int64_t ne)
{
    const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (e >= ne) return;
    ElemGeo& G = geo[e];
    for (int i = 0; i < 3; ++i)
        p1_grad(G, node[(int64_t)G.node[0] * NODE_STRIDE + NF_MU + i], node[(int64_t)G.node[1] * NODE_STRIDE + NF_MU + i],
                node[(int64_t)G.node[2] * NODE_STRIDE + NF_MU + i], G.gu[2 * i], G.gu[2 * i + 1]);
}

// two-pass second derivatives (Sec. 3.4): element gradients averaged to the nodes ...
__global__ void __launch_bounds__(256) k_fb_gn(const ElemGeo* __restrict__ geo, const int64_t* __restrict__ n2e_ptr,
                                               const int32_t* __restrict__ n2e, int64_t nn, double* __restrict__ gn)
{
    const int64_t n = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (n >= nn) return;
    double s[6] = {0, 0, 0, 0, 0, 0};
    const int64_t j0 = n2e_ptr[n], j1 = n2e_ptr[n + 1];
    for (int64_t j = j0; j < j1; ++j)
        for (int q = 0; q < 6; ++q) s[q] += geo[n2e[j] / 3].gu[q];
    const double c = (double)(j1 - j0);
    for (int q = 0; q < 6; ++q) gn[6 * n + q] = j1 > j0 ? s[q] / c : 0.0;
}

// ... their element gradients (d/dx of the x-derivative, d/dy of the y-derivative) ...
__global__ void __launch_bounds__(256) k_fb_h(const ElemGeo* __restrict__ geo, const double* __restrict__ gn, int64_t ne,
                                              double* __restrict__ h)
{
    const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (e >= ne) return;
    const ElemGeo& G = geo[e];
    const int64_t a = G.node[0], b = G.node[1], c = G.node[2];
    for (int i = 0; i < 3; ++i) {
        double dxx, dxy, dyx, dyy;
        p1_grad(G, gn[6 * a + 2 * i], gn[6 * b + 2 * i], gn[6 * c + 2 * i], dxx, dxy);
        p1_grad(G, gn[6 * a + 2 * i + 1], gn[6 * b + 2 * i + 1], gn[6 * c + 2 * i + 1], dyx, dyy);
        h[6 * e + 2 * i] = dxx;
        h[6 * e + 2 * i + 1] = dyy;
    }
}

// ... averaged to the nodes again: lap<U_i> = d2/dx2 + d2/dy2
__global__ void __launch_bounds__(256) k_fb_lap(const int64_t* __restrict__ n2e_ptr, const int32_t* __restrict__ n2e,
                                                const double* __restrict__ h, int64_t nn, double* __restrict__ node)
{
    const int64_t n = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (n >= nn) return;
    const int64_t j0 = n2e_ptr[n], j1 = n2e_ptr[n + 1];
    const double c = (double)(j1 - j0);
    for (int i = 0; i < 3; ++i) {
        double sxx = 0.0, syy = 0.0;
        for (int64_t j = j0; j < j1; ++j) {
            sxx += h[6 * (int64_t)(n2e[j] / 3) + 2 * i];
            syy += h[6 * (int64_t)(n2e[j] / 3) + 2 * i + 1];
        }
        node[n * NODE_STRIDE + NF_LAP + i] = j1 > j0 ? sxx / c + syy / c : 0.0;
    }
}

// time step of Eq. (26): min over nodes of sqrt(average element area around the node) and
// max over nodes with particles of |(<U>, <omega>, <psi>)|, as the bits of non-negative
// doubles (their integer order is their numeric order)
__global__ void __launch_bounds__(256) k_cfl(const ElemGeo* __restrict__ geo, const int64_t* __restrict__ n2e_ptr,
                                             const int32_t* __restrict__ n2e, const double* __restrict__ stats,
                                             int64_t n0, int64_t nn, unsigned long long* __restrict__ out)
{
    const int64_t n = n0 + (int64_t)blockIdx.x * 256 + threadIdx.x;
    double l = __builtin_inf(), z = 0.0;
    if (n < n0 + nn) cfl_node(geo, n2e_ptr, n2e, stats, n, l, z);
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        l = fmin(l, __shfl_xor(l, o));
        z = fmax(z, __shfl_xor(z, o));
    }
    if (lane_id() == 0) {
        atomicMin(out, (unsigned long long)__double_as_longlong(l));
        atomicMax(out + 1, (unsigned long long)__double_as_longlong(z));
    }
}

// =====================================================================================
// launchers
// =====================================================================================
static inline unsigned blocks_for(int64_t n, int nt) { return (unsigned)((n + nt - 1) / nt); }

template <class R>
void launch_advance(const AdvanceArgs<R>& a, int64_t n_ub, bool batched, bool wp_full, int block, hipStream_t s)
{
    if (n_ub <= 0) return;
    if (block != 64 && block != 128) block = 256;
    const unsigned small = (unsigned)std::min<int64_t>((n_ub + 63) / 64, 1024);
    if (batched) {
        hipLaunchKernelGGL(k_advance_batched<R>, dim3(blocks_for(n_ub, block)), dim3(block), 0, s, a);
        hipLaunchKernelGGL(k_advance_mixed_waves<R>, dim3(small), dim3(64), 0, s, a);
        hipLaunchKernelGGL((k_advance_redo<R, PM_LANE, false>), dim3(small), dim3(64), 0, s, a);
    } else if (wp_full) {
        hipLaunchKernelGGL((k_advance<R, true>), dim3(blocks_for(n_ub, block)), dim3(block), 0, s, a);
        hipLaunchKernelGGL((k_advance_redo<R, PM_ONE, true>), dim3(small), dim3(64), 0, s, a);
    } else {
        hipLaunchKernelGGL((k_advance<R, false>), dim3(blocks_for(n_ub, block)), dim3(block), 0, s, a);
        hipLaunchKernelGGL((k_advance_redo<R, PM_ONE, false>), dim3(small), dim3(64), 0, s, a);
    }
    hipLaunchKernelGGL(k_wall_resample<R>, dim3(256), dim3(256), 0, s, a.s, (const int32_t*)a.wall_list,
                       (const int32_t*)a.wall_count, a.geo, a.prm, a.meta);
}
void launch_count(const int32_t* elem, const int64_t* nslots, int64_t n_ub, int64_t ne, int32_t* counts,
                  uint32_t* err, hipStream_t s)
{
    if (n_ub > 0) hipLaunchKernelGGL(k_count, dim3(blocks_for(n_ub, 256)), dim3(256), 0, s, elem, nslots, ne, counts, err);
}
void launch_count_range(const int32_t* elem, const int64_t* nslots, int64_t n_ub, int32_t lo, int32_t hi,
                        unsigned long long* out, hipStream_t s)
{
    if (n_ub > 0)
        hipLaunchKernelGGL(k_count_range, dim3(blocks_for(n_ub, 256)), dim3(256), 0, s, elem, nslots, lo, hi, out);
}
int64_t scan_blocks(int64_t n) { return (n + SCAN_TILE - 1) / SCAN_TILE; }
void launch_scan(const int32_t* in, int64_t n, int32_t* out, int32_t* tmp, hipStream_t s)
{
    const int64_t nb = scan_blocks(n);
    hipLaunchKernelGGL(k_scan_reduce, dim3((unsigned)nb), dim3(SCAN_NT), 0, s, in, n, tmp);
    hipLaunchKernelGGL(k_scan_top, dim3(1), dim3(SCAN_NT), 0, s, tmp, nb);
    hipLaunchKernelGGL(k_scan_apply, dim3((unsigned)nb), dim3(SCAN_NT), 0, s, in, n, tmp, out, nb);
}
int64_t scan_max_elems() { return (int64_t)SCAN_TILE * SCAN_TILE; }
void launch_scatter(const int32_t* elem, const int64_t* nslots, int64_t n_ub, int64_t ne, int32_t* counts,
                    const int32_t* start, int32_t* idx, uint32_t* err, hipStream_t s)
{
    if (n_ub > 0)
        hipLaunchKernelGGL(k_scatter, dim3(blocks_for(n_ub, 256 * SCAT_ROUNDS)), dim3(256), 0, s, elem, nslots, ne, counts,
                           start, idx, err);
}
void launch_place(const int32_t* elem, const int32_t* arrival, const int64_t* nslots, int64_t n_ub, int64_t ne,
                  const int32_t* start, int32_t* idx, uint32_t* err, hipStream_t s)
{
    if (n_ub > 0)
        hipLaunchKernelGGL(k_place, dim3(blocks_for((n_ub + 3) / 4, 256)), dim3(256), 0, s, elem, arrival, nslots, n_ub,
                           ne, start, idx, err);
}
template <class R>
hipError_t prepare_element_pass(int lds_max)
{
    return hipFuncSetAttribute((const void*)k_element_block<EP_NT, R>, hipFuncAttributeMaxDynamicSharedMemorySize,
                               (int)element_pass_smem<R>(lds_max));
}
template <int PPL, class R>
static void launch_wave_tier(const ElementArgs<R>& a, int n_below, int last, hipStream_t s)
{
    constexpr int WPB = WaveBlock<PPL>::waves;
    if (a.any_proj)
        hipLaunchKernelGGL((k_element_wave<PPL, R, true>), dim3((unsigned)((a.ne + WPB - 1) / WPB)), dim3(64 * WPB), 0,
                           s, a, n_below, last);
    else
        hipLaunchKernelGGL((k_element_wave<PPL, R, false>), dim3((unsigned)((a.ne + WPB - 1) / WPB)), dim3(64 * WPB), 0,
                           s, a, n_below, last);
}
template <class R>
void launch_element_pass(const ElementArgs<R>& a, const int* tiers, int n_tiers, hipStream_t s)
{
    for (int t = 0; t < n_tiers; ++t) {
        const int n_below = t == 0 ? -1 : 64 * tiers[t - 1], last = t == n_tiers - 1 ? 1 : 0;
        switch (tiers[t]) {
        case 1: launch_wave_tier<1, R>(a, n_below, last, s); break;
        case 2: launch_wave_tier<2, R>(a, n_below, last, s); break;
        case 3: launch_wave_tier<3, R>(a, n_below, last, s); break;
        case 4: launch_wave_tier<4, R>(a, n_below, last, s); break;
        case 5: launch_wave_tier<5, R>(a, n_below, last, s); break;
        case 6: launch_wave_tier<6, R>(a, n_below, last, s); break;
        default: launch_wave_tier<8, R>(a, n_below, last, s); break;
        }
    }
    hipLaunchKernelGGL((k_element_block<EP_NT, R>), dim3(EP_BIG_BLOCKS), dim3(EP_NT), element_pass_smem<R>(a.lds_max),
                       s, a);
}
template <class R>
void launch_node_finalize(const NodeArgs<R>& a, hipStream_t s)
{
    hipLaunchKernelGGL(k_node_finalize<R>, dim3(blocks_for(a.nn > 0 ? a.nn : 1, 256)), dim3(256), 0, s, a);
}
template <class R>
void launch_init(const InitArgs<R>& a, hipStream_t s)
{
    if (a.n > 0) hipLaunchKernelGGL(k_init<R>, dim3(blocks_for(a.n, 256)), dim3(256), 0, s, a);
}
void launch_tm(const ElemGeo* geo, const double* node, int64_t ne, const ProbParams* prm, double* tm,
               hipStream_t s)
{
    if (ne > 0) hipLaunchKernelGGL(k_tm, dim3(blocks_for(ne, 256)), dim3(256), 0, s, geo, node, ne, prm, tm);
}
template <class R>
void launch_ctl_plan(const ControlArgs<R>& a, hipStream_t s)
{
    hipLaunchKernelGGL(k_ctl_plan<R>, dim3(blocks_for(a.ne, 256)), dim3(256), 0, s, a);
}
template <class R>
void launch_ctl_apply(const ControlArgs<R>& a, hipStream_t s)
{
    hipLaunchKernelGGL(k_ctl_apply<R>, dim3(blocks_for(a.ne, 256)), dim3(256), 0, s, a);
}
void launch_ctl_finish(int64_t* meta, const int32_t* off, int64_t ne, const unsigned long long* rep, int64_t cap,
                       ProbParams* prm, int32_t n_problems, hipStream_t s)
{
    hipLaunchKernelGGL(k_ctl_finish, dim3(1), dim3(64), 0, s, meta, off, ne, rep, cap, prm, n_problems);
}
void launch_feedback(const double* stats, double* node, ElemGeo* geo, const int64_t* n2e_ptr, const int32_t* n2e,
                     int64_t nn, int64_t ne, double alpha, int32_t rey, double* gn, double* h, hipStream_t s)
{
    if (nn <= 0 || ne <= 0) return;
    hipLaunchKernelGGL(k_fb_nodes, dim3(blocks_for(nn, 256)), dim3(256), 0, s, stats, node, nn, alpha, rey);
    hipLaunchKernelGGL(k_fb_grad, dim3(blocks_for(ne, 256)), dim3(256), 0, s, geo, (const double*)node, ne);
    hipLaunchKernelGGL(k_fb_gn, dim3(blocks_for(nn, 256)), dim3(256), 0, s, (const ElemGeo*)geo, n2e_ptr, n2e, nn, gn);
    hipLaunchKernelGGL(k_fb_h, dim3(blocks_for(ne, 256)), dim3(256), 0, s, (const ElemGeo*)geo, (const double*)gn, ne, h);
    hipLaunchKernelGGL(k_fb_lap, dim3(blocks_for(nn, 256)), dim3(256), 0, s, n2e_ptr, n2e, (const double*)h, nn, node);
}
void launch_cfl(const ElemGeo* geo, const int64_t* n2e_ptr, const int32_t* n2e, const double* stats, int64_t n0,
                int64_t nn, unsigned long long* out, hipStream_t s)
{
    if (nn > 0) hipLaunchKernelGGL(k_cfl, dim3(blocks_for(nn, 256)), dim3(256), 0, s, geo, n2e_ptr, n2e, stats, n0, nn, out);
}
template <class R>
void launch_redistribute(const SoaT<R>& st, const SoaT<R>& stage, const int32_t* plan, const ElemGeo* geo, int64_t m,
                         hipStream_t s)
{
    if (m <= 0) return;
    hipLaunchKernelGGL(k_redist_gather<R>, dim3(blocks_for(m, 256)), dim3(256), 0, s, st, stage, plan, geo, m);
    hipLaunchKernelGGL(k_redist_write<R>, dim3(blocks_for(m, 256)), dim3(256), 0, s, st, stage, plan, m);
}

void launch_fill_i32(int32_t* p, int64_t n, int32_t v, hipStream_t s)
{
    if (n > 0) hipLaunchKernelGGL(k_fill_i32, dim3(blocks_for(n, 256)), dim3(256), 0, s, p, n, v);
}
void launch_fill_u64(unsigned long long* p, int64_t n, unsigned long long v, hipStream_t s)
{
    if (n > 0) hipLaunchKernelGGL(k_fill_u64, dim3(blocks_for(n, 256)), dim3(256), 0, s, p, n, v);
}
void launch_f64_to_f32(const double* in, float* out, int64_t n, hipStream_t s)
{
    if (n > 0) hipLaunchKernelGGL(k_f64_to_f32, dim3(blocks_for(n, 256)), dim3(256), 0, s, in, out, n);
}
void launch_f32_to_f64(const float* in, double* out, int64_t n, hipStream_t s)
{
    if (n > 0) hipLaunchKernelGGL(k_f32_to_f64, dim3(blocks_for(n, 256)), dim3(256), 0, s, in, out, n);
}
template <class R>
void launch_shift_init(const R* node, int64_t nn, R* shift, hipStream_t s)
{
    if (nn > 0) hipLaunchKernelGGL(k_shift_init<R>, dim3(blocks_for(nn, 256)), dim3(256), 0, s, node, nn, shift);
}

// both forms of the state
#define PDF_INSTANTIATE(R)                                                                               \
    template void launch_advance<R>(const AdvanceArgs<R>&, int64_t, bool, bool, int, hipStream_t);       \
    template hipError_t prepare_element_pass<R>(int);                                                    \
    template size_t element_pass_smem<R>(int);                                                           \
    template void launch_element_pass<R>(const ElementArgs<R>&, const int*, int, hipStream_t);          \
    template void launch_node_finalize<R>(const NodeArgs<R>&, hipStream_t);                              \
    template void launch_init<R>(const InitArgs<R>&, hipStream_t);                                       \
    template void launch_ctl_plan<R>(const ControlArgs<R>&, hipStream_t);                                \
    template void launch_ctl_apply<R>(const ControlArgs<R>&, hipStream_t);                               \
    template void launch_shift_init<R>(const R*, int64_t, R*, hipStream_t);                              \
    template void launch_redistribute<R>(const SoaT<R>&, const SoaT<R>&, const int32_t*, const ElemGeo*, int64_t, \
                                         hipStream_t);
PDF_INSTANTIATE(double)
PDF_INSTANTIATE(float)
#undef PDF_INSTANTIATE

}  // namespace pdfgpu
