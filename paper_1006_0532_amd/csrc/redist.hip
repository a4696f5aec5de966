// Particle redistribution of App. B on the device.
//
// App. B moves one particle at a time from the fullest element (ties to the lowest index) to
// the emptiest (ties to the lowest index) until the emptiest holds n_min particles or the
// two differ by at most one.  While the loop runs the fullest count exceeds the emptiest by
// two or more, so an element that gave a particle never becomes the emptiest and one that
// received never becomes the fullest: the receiving side visits the counts l = lmin,
// lmin + 1, ... and takes at level l every element with at most l particles in index order,
// and the giving side visits h = hmax, hmax - 1, ... and takes every element with at least h
// in index order.  Move m is therefore the m-th (level, element) pair of each side, and
// only the slot choices inside one element (which slot leaves, which resident a newcomer
// copies) depend on earlier moves of that same element.
//
// The device computes, per problem: the element counts and their extremes; histograms of
// the levels, from which the host finds the number of moves K and the levels each side
// reaches (a walk over levels, not over moves); for each side the move index of every
// (element, level) pair, as the level's start plus the element's rank among the elements
// already taken at that level (per-workgroup counts, their scan over workgroups, and a
// ballot inside the workgroup); then one thread per giving element draws its leaving slots
// in move order, and one thread per receiving element draws the particle each newcomer
// copies.  The moves are applied by the gather / write kernels of the library.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>
#include <string>
#include <vector>

#include "device.h"
#include "kernels.h"
#include "pdf_impl.h"

namespace pdfgpu {
void set_error(const std::string& msg);
}
using namespace pdfgpu;

namespace {

constexpr uint32_t TAG_REDIST = 5;
constexpr int RD_NT = 256;
// limit of the level histograms: count levels one side can visit
constexpr int64_t RD_MAX_LEVELS = 1 << 22;

unsigned rd_blocks(int64_t n) { return (unsigned)((n + RD_NT - 1) / RD_NT); }

__device__ __forceinline__ Words4 rd_draw(RngKey key, int32_t m, uint32_t step)
{
    return philox4x32_10((uint32_t)m, 0u, step, TAG_REDIST << 16, key.k0, key.k1);
}

// counts of the problem's elements and their minimum and maximum (mm = {INT_MAX, INT_MIN} on entry)
__global__ void __launch_bounds__(RD_NT) k_rd_counts(const int32_t* __restrict__ start, int64_t e0, int64_t ne,
                                                    int32_t* __restrict__ c0, int32_t* __restrict__ mm)
{
    const int64_t i = (int64_t)blockIdx.x * RD_NT + threadIdx.x;
    int lo = INT_MAX, hi = INT_MIN;
    if (i < ne) {
        const int c = start[e0 + i + 1] - start[e0 + i];
        c0[i] = c;
        lo = hi = c;
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        lo = min(lo, __shfl_xor(lo, o));
        hi = max(hi, __shfl_xor(hi, o));
    }
    if ((threadIdx.x & 63) == 0) {
        atomicMin(mm, lo);
        atomicMax(mm + 1, hi);
    }
}

// elements per level: receiving side t = c - lmin (t < nlo), giving side t = cmax - c (t < nhi)
__global__ void __launch_bounds__(RD_NT) k_rd_hist(const int32_t* __restrict__ c0, int64_t ne, int32_t lmin,
                                                  int32_t nlo, int32_t cmax, int32_t nhi, int32_t* __restrict__ hlo,
                                                  int32_t* __restrict__ hhi)
{
    const int64_t i = (int64_t)blockIdx.x * RD_NT + threadIdx.x;
    if (i >= ne) return;
    const int c = c0[i];
    if (c - lmin < nlo) atomicAdd(hlo + (c - lmin), 1);
    if (cmax - c < nhi) atomicAdd(hhi + (cmax - c), 1);
}

// first level of each element on one side (receiving: c - lmin; giving: cmax - c) and the
// number of levels it can take part in, L - key
__global__ void __launch_bounds__(RD_NT) k_rd_keys(const int32_t* __restrict__ c0, int64_t ne, int32_t base,
                                                  int32_t sgn, int32_t L, int32_t* __restrict__ key,
                                                  int32_t* __restrict__ len)
{
    const int64_t i = (int64_t)blockIdx.x * RD_NT + threadIdx.x;
    if (i >= ne) return;
    const int k = sgn > 0 ? c0[i] - base : base - c0[i];
    key[i] = k;
    len[i] = k < L ? L - k : 0;
}

// T[b][t] = number of elements of workgroup b taken at level t (key <= t)
__global__ void __launch_bounds__(RD_NT) k_rd_table(const int32_t* __restrict__ key, int64_t ne, int32_t L,
                                                   int32_t* __restrict__ T)
{
    const int64_t i = (int64_t)blockIdx.x * RD_NT + threadIdx.x;
    const int k = i < ne ? key[i] : INT_MAX;
    for (int t = 0; t < L; ++t) {
        const int c = __syncthreads_count(k <= t);
        if (threadIdx.x == 0) T[(int64_t)blockIdx.x * L + t] = c;
    }
}

// exclusive scan of T over the workgroups, one thread per level
__global__ void __launch_bounds__(RD_NT) k_rd_table_scan(int32_t* __restrict__ T, int64_t nb, int32_t L)
{
    const int64_t t = (int64_t)blockIdx.x * RD_NT + threadIdx.x;
    if (t >= L) return;
    int run = 0;
    for (int64_t b = 0; b < nb; ++b) {
        const int v = T[b * L + t];
        T[b * L + t] = run;
        run += v;
    }
}

// move index of every (element, level) pair of one side: the level's first move S[t] plus the
// element's rank among the elements taken at that level; list[off[i] + t - key[i]] holds it,
// or -1 from the first pair at or beyond the K moves
__global__ void __launch_bounds__(RD_NT) k_rd_enum(const int32_t* __restrict__ key, int64_t ne, int32_t L,
                                                  const int32_t* __restrict__ T, const int64_t* __restrict__ S,
                                                  int64_t K, const int32_t* __restrict__ off,
                                                  int32_t* __restrict__ list)
{
    __shared__ int wsum[RD_NT / 64];
    const int64_t i = (int64_t)blockIdx.x * RD_NT + threadIdx.x;
    const int k = i < ne ? key[i] : INT_MAX;
    const int lane = lane_id(), wid = threadIdx.x >> 6;
    for (int t = 0; t < L; ++t) {
        const bool in = k <= t;
        const unsigned long long b = __ballot(in);
        const int below = __popcll(b & ((1ull << lane) - 1ull));
        if (lane == 0) wsum[wid] = __popcll(b);
        __syncthreads();
        int pre = 0;
        for (int w = 0; w < wid; ++w) pre += wsum[w];
        __syncthreads();
        if (in) {
            const int64_t m = S[t] + T[(int64_t)blockIdx.x * L + t] + pre + below;
            list[off[i] + (t - k)] = m < K ? (int32_t)m : -1;
        }
    }
}

// giving side: in move order, the leaving slot is the r-th of the element's slots still
// present, r = floor(u * h) with h the element's count before the move (App. B)
__global__ void __launch_bounds__(RD_NT) k_rd_donors(const int32_t* __restrict__ start, int64_t e0, int64_t ne,
                                                    const int32_t* __restrict__ c0, const int32_t* __restrict__ key,
                                                    const int32_t* __restrict__ off, const int32_t* __restrict__ list,
                                                    int32_t L, int32_t cmax, uint32_t* __restrict__ gone, RngKey rk,
                                                    uint32_t step, int32_t* __restrict__ slot_of)
{
    const int64_t i = (int64_t)blockIdx.x * RD_NT + threadIdx.x;
    if (i >= ne || key[i] >= L) return;
    const int32_t s0 = start[e0 + i], n = c0[i];
    for (int j = 0; j < L - key[i]; ++j) {
        const int32_t m = list[off[i] + j];
        if (m < 0) break;
        const int h = cmax - (key[i] + j);
        const Words4 w = rd_draw(rk, m, step);
        int64_t left = (int64_t)(u01(w.w0) * (double)h);
        // walk the element's slots a 32-bit word of the departure mask at a time
        int32_t q = s0;
        const int32_t q1 = s0 + n;
        while (q < q1) {
            const int32_t wi = q >> 5, b0 = q & 31;
            const int32_t nb = min(32 - b0, q1 - q);
            const uint32_t span = (nb == 32 ? 0xffffffffu : ((1u << nb) - 1u)) << b0;
            const uint32_t present = ~gone[wi] & span;
            const int cnt = __popc(present);
            if (left < cnt) {
                uint32_t p = present;
                for (int64_t z = 0; z < left; ++z) p &= p - 1u;
                q = (wi << 5) + (__ffs(p) - 1);
                break;
            }
            left -= cnt;
            q += nb;
        }
        atomicOr(gone + (q >> 5), 1u << (q & 31));
        slot_of[m] = q;
    }
}

// receiving side: in move order, the newcomer takes the position, velocity, frequency and
// scalar of the d-th particle of the element's list (residents in slot order, then the
// earlier newcomers), d = floor(u * l) with l the element's count before the move; into an
// empty element it keeps its own properties and takes the centroid (App. B)
__global__ void __launch_bounds__(RD_NT) k_rd_receivers(const int32_t* __restrict__ start, int64_t e0, int64_t ne,
                                                       const int32_t* __restrict__ c0,
                                                       const int32_t* __restrict__ key,
                                                       const int32_t* __restrict__ off,
                                                       const int32_t* __restrict__ list, int32_t L, int32_t lmin,
                                                       RngKey rk, uint32_t step, const int32_t* __restrict__ slot_of,
                                                       int32_t* __restrict__ plan)
{
    const int64_t i = (int64_t)blockIdx.x * RD_NT + threadIdx.x;
    if (i >= ne || key[i] >= L) return;
    const int32_t s0 = start[e0 + i], n = c0[i], eg = (int32_t)(e0 + i);
    for (int j = 0; j < L - key[i]; ++j) {
        const int32_t m = list[off[i] + j];
        if (m < 0) break;
        const int l = lmin + key[i] + j;
        const int32_t slot = slot_of[m];
        int32_t pos, prop;
        if (l == 0) {
            pos = -eg - 1;
            prop = slot;
        } else {
            const Words4 w = rd_draw(rk, m, step);
            const int64_t d = (int64_t)(u01(w.w1) * (double)l);
            if (d < n) {
                pos = prop = s0 + (int32_t)d;
            } else {
                const int32_t mj = list[off[i] + (int32_t)(d - n)];
                pos = plan[4 * (int64_t)mj + 1];
                prop = plan[4 * (int64_t)mj + 2];
            }
        }
        plan[4 * (int64_t)m] = slot;
        plan[4 * (int64_t)m + 1] = pos;
        plan[4 * (int64_t)m + 2] = prop;
        plan[4 * (int64_t)m + 3] = eg;
    }
}

// device temporaries of one call, freed on every path
struct Scratch {
    std::vector<void*> ptrs;
    ~Scratch()
    {
        for (void* p : ptrs) (void)hipFree(p);
    }
    template <class T>
    pdf_status get(T** p, int64_t count)
    {
        *p = nullptr;
        if (count < 1) count = 1;
        if (hipMalloc((void**)p, sizeof(T) * (size_t)count) != hipSuccess) {
            (void)hipGetLastError();
            *p = nullptr;
            set_error("redistribution: device allocation of " + std::to_string(sizeof(T) * count) + " bytes failed");
            return PDF_E_NOMEM;
        }
        ptrs.push_back((void*)*p);
        return PDF_OK;
    }
};

#define RD_TRY(expr)                                                                               \
    do {                                                                                           \
        hipError_t _e = (expr);                                                                    \
        if (_e != hipSuccess) {                                                                    \
            set_error(std::string("redistribution: ") + hipGetErrorString(_e));                   \
            return PDF_E_HIP;                                                                      \
        }                                                                                          \
    } while (0)

// what the level walk of one problem found
struct RdProblem {
    int p = 0;
    int64_t ne = 0, e0 = 0;
    int32_t lmin = 0, cmax = 0;
    int64_t K = 0;
    int32_t Llo = 0, Lhi = 0;        // levels visited by the receiving and the giving side
    std::vector<int64_t> Slo, Shi;   // first move of each level
    int32_t* c0 = nullptr;
};

// move index of every (element, level) pair of one side into list (offsets in off)
pdf_status enumerate_side(Scratch& sc, const RdProblem& q, int sgn, int32_t L, const std::vector<int64_t>& S,
                          int32_t*& key, int32_t*& off, int32_t*& list, hipStream_t s)
{
    const int64_t ne = q.ne, nb = rd_blocks(ne);
    // the (element, level) pairs are listed with 32-bit offsets: ne x L bounds their number
    if (ne * (int64_t)L > INT32_MAX) {
        set_error("redistribution: one problem's elements times the levels one side visits exceed 2^31 - 1");
        return PDF_E_CAPACITY;
    }
    int32_t *len = nullptr, *tmp = nullptr, *T = nullptr;
    int64_t* dS = nullptr;
    pdf_status st = sc.get(&key, ne);
    if (st == PDF_OK) st = sc.get(&len, ne);
    if (st == PDF_OK) st = sc.get(&off, ne + 1);
    if (st == PDF_OK) st = sc.get(&tmp, scan_blocks(ne) + 1);
    if (st == PDF_OK) st = sc.get(&T, nb * L);
    if (st == PDF_OK) st = sc.get(&dS, L);
    if (st != PDF_OK) return st;
    hipLaunchKernelGGL(k_rd_keys, dim3(rd_blocks(ne)), dim3(RD_NT), 0, s, q.c0, ne, sgn > 0 ? q.lmin : q.cmax, sgn,
                       L, key, len);
    launch_scan(len, ne, off, tmp, s);
    int32_t total = 0;
    RD_TRY(hipMemcpyAsync(&total, off + ne, sizeof(int32_t), hipMemcpyDeviceToHost, s));
    RD_TRY(hipMemcpyAsync(dS, S.data(), sizeof(int64_t) * L, hipMemcpyHostToDevice, s));
    hipLaunchKernelGGL(k_rd_table, dim3((unsigned)nb), dim3(RD_NT), 0, s, key, ne, L, T);
    hipLaunchKernelGGL(k_rd_table_scan, dim3(rd_blocks(L)), dim3(RD_NT), 0, s, T, nb, L);
    RD_TRY(hipStreamSynchronize(s));
    st = sc.get(&list, total);
    if (st != PDF_OK) return st;
    hipLaunchKernelGGL(k_rd_enum, dim3((unsigned)nb), dim3(RD_NT), 0, s, key, ne, L, T, dS, q.K, off, list);
    RD_TRY(hipGetLastError());
    return PDF_OK;
}

}  // namespace

namespace pdfgpu {

// App. B for the listed problems of E on the canonical order of the last pass: the moves of
// all problems in plan (4 ints each: slot, position source or -(e + 1), property source,
// new element), their number in total.  plan_buf / plan_cap: the ensemble's plan storage,
// grown here.
pdf_status redistribution_plan(pdf_ens_s* E, const std::vector<int>& problems, int32_t n_min, uint32_t step,
                               int32_t** plan_buf, int64_t* plan_cap, int64_t* total, hipStream_t s)
{
    *total = 0;
    Scratch sc;
    std::vector<RdProblem> work;
    // counts, extremes and level histograms, then the walk over levels
    for (int p : problems) {
        const ProbParams& P = E->h_prm[p];
        RdProblem q;
        q.p = p;
        q.ne = P.ne;
        q.e0 = P.eoff;
        if (q.ne == 0) continue;
        int32_t* mm = nullptr;
        pdf_status st = sc.get(&q.c0, q.ne);
        if (st == PDF_OK) st = sc.get(&mm, 2);
        if (st != PDF_OK) return st;
        launch_fill_i32(mm, 1, INT_MAX, s);
        launch_fill_i32(mm + 1, 1, INT_MIN, s);
        hipLaunchKernelGGL(k_rd_counts, dim3(rd_blocks(q.ne)), dim3(RD_NT), 0, s, E->start, q.e0, q.ne, q.c0, mm);
        int32_t h_mm[2];
        RD_TRY(hipMemcpyAsync(h_mm, mm, sizeof(h_mm), hipMemcpyDeviceToHost, s));
        RD_TRY(hipStreamSynchronize(s));
        q.lmin = h_mm[0];
        q.cmax = h_mm[1];
        if (q.lmin >= n_min || q.cmax - q.lmin <= 1) continue;
        // the receiving side stays below n_min and below cmax - 1, the giving side above lmin + 1
        const int64_t nlo = std::min<int64_t>((int64_t)std::min(n_min, q.cmax) - q.lmin, RD_MAX_LEVELS);
        const int64_t nhi = std::min<int64_t>((int64_t)q.cmax - q.lmin + 1, RD_MAX_LEVELS);
        int32_t *hlo = nullptr, *hhi = nullptr;
        st = sc.get(&hlo, nlo);
        if (st == PDF_OK) st = sc.get(&hhi, nhi);
        if (st != PDF_OK) return st;
        launch_fill_i32(hlo, nlo, 0, s);
        launch_fill_i32(hhi, nhi, 0, s);
        hipLaunchKernelGGL(k_rd_hist, dim3(rd_blocks(q.ne)), dim3(RD_NT), 0, s, q.c0, q.ne, q.lmin, (int32_t)nlo,
                           q.cmax, (int32_t)nhi, hlo, hhi);
        std::vector<int32_t> Hlo(nlo), Hhi(nhi);
        RD_TRY(hipMemcpyAsync(Hlo.data(), hlo, sizeof(int32_t) * nlo, hipMemcpyDeviceToHost, s));
        RD_TRY(hipMemcpyAsync(Hhi.data(), hhi, sizeof(int32_t) * nhi, hipMemcpyDeviceToHost, s));
        RD_TRY(hipStreamSynchronize(s));
        // elements taken per level: receiving side P_t = #{c <= lmin + t}, giving Q_t = #{c >= cmax - t}
        for (int64_t t = 1; t < nlo; ++t) Hlo[t] += Hlo[t - 1];
        for (int64_t t = 1; t < nhi; ++t) Hhi[t] += Hhi[t - 1];
        int64_t l = q.lmin, h = q.cmax, r = 0, u = 0, K = 0;
        q.Slo.clear();
        q.Shi.clear();
        q.Slo.push_back(0);
        q.Shi.push_back(0);
        while (!(l >= n_min || h - l <= 1)) {
            if (q.cmax - h >= nhi || l - q.lmin >= nlo) {
                set_error("redistribution: one side would visit more count levels than its limit");
                return PDF_E_CAPACITY;
            }
            const int64_t Pt = Hlo[l - q.lmin], Qt = Hhi[q.cmax - h];
            const int64_t stp = std::min(Pt - r, Qt - u);
            K += stp;
            r += stp;
            u += stp;
            if (r == Pt) {
                ++l;
                r = 0;
                q.Slo.push_back(K);
            }
            if (u == Qt) {
                --h;
                u = 0;
                q.Shi.push_back(K);
            }
        }
        if (K == 0) continue;
        if (K > INT32_MAX / 4) {
            set_error("redistribution: too many moves for one call");
            return PDF_E_CAPACITY;
        }
        q.K = K;
        q.Llo = (int32_t)(l - q.lmin + (r > 0 ? 1 : 0));
        q.Lhi = (int32_t)(q.cmax - h + (u > 0 ? 1 : 0));
        q.Slo.resize(q.Llo);
        q.Shi.resize(q.Lhi);
        *total += K;
        work.push_back(std::move(q));
    }
    if (*total == 0) return PDF_OK;
    if (*total > *plan_cap) {
        if (*plan_buf) (void)hipFree(*plan_buf);
        *plan_buf = nullptr;
        *plan_cap = 0;
        if (hipMalloc((void**)plan_buf, sizeof(int32_t) * 4 * (size_t)*total) != hipSuccess) {
            (void)hipGetLastError();
            *plan_buf = nullptr;
            set_error("redistribution: device allocation of the plan failed");
            return PDF_E_NOMEM;
        }
        *plan_cap = *total;
    }
    // departures of every problem are marked in one bit per slot
    uint32_t* gone = nullptr;
    const int64_t words = E->cap / 32 + 1;
    pdf_status st = sc.get(&gone, words);
    if (st != PDF_OK) return st;
    launch_fill_i32(reinterpret_cast<int32_t*>(gone), words, 0, s);
    int64_t base = 0;
    for (const RdProblem& q : work) {
        const ProbParams& P = E->h_prm[q.p];
        int32_t *khi = nullptr, *ohi = nullptr, *lhi = nullptr, *klo = nullptr, *olo = nullptr, *llo = nullptr;
        int32_t* slot_of = nullptr;
        st = enumerate_side(sc, q, -1, q.Lhi, q.Shi, khi, ohi, lhi, s);
        if (st == PDF_OK) st = enumerate_side(sc, q, +1, q.Llo, q.Slo, klo, olo, llo, s);
        if (st == PDF_OK) st = sc.get(&slot_of, q.K);
        if (st != PDF_OK) return st;
        hipLaunchKernelGGL(k_rd_donors, dim3(rd_blocks(q.ne)), dim3(RD_NT), 0, s, E->start, q.e0, q.ne, q.c0, khi, ohi,
                           lhi, q.Lhi, q.cmax, gone, P.key, step, slot_of);
        hipLaunchKernelGGL(k_rd_receivers, dim3(rd_blocks(q.ne)), dim3(RD_NT), 0, s, E->start, q.e0, q.ne, q.c0, klo,
                           olo, llo, q.Llo, q.lmin, P.key, step, slot_of, *plan_buf + 4 * base);
        RD_TRY(hipGetLastError());
        base += q.K;
    }
    RD_TRY(hipStreamSynchronize(s));   // the kernels are done with the scratch before it is freed
    return PDF_OK;
}

}  // namespace pdfgpu
