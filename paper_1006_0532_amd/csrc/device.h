// Device building blocks of libpdfgpu: counter-based random numbers, P1 geometry,
// wavefront collectives.  Included by the kernel translation unit only.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "pdf_impl.h"

namespace pdfgpu {

// ------------------------------------------------------------------------------------
// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11): ten rounds; each round multiplies
// words 0 and 2 by fixed 32-bit constants, mixes the high halves with words 1, 3 and the
// key, and the key advances by the Weyl constants between rounds.
// Key (seed low word, seed high word XOR problem); counter (pid low, pid high, step,
// tag << 16 | index).
// ------------------------------------------------------------------------------------
struct Words4 {
    uint32_t w0, w1, w2, w3;
};
enum : uint32_t { TAG_INIT = 1, TAG_STEP = 2, TAG_WALL_GAMMA = 3, TAG_INIT_GAMMA = 4 };

__device__ __forceinline__ Words4 philox4x32_10(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                               uint32_t k0, uint32_t k1)
{
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint32_t m0 = 0xD2511F53u, m1 = 0xCD9E8D57u;
        const uint32_t lo0 = m0 * c0, hi0 = __umulhi(m0, c0);
        const uint32_t lo1 = m1 * c2, hi1 = __umulhi(m1, c2);
        const uint32_t n0 = hi1 ^ c1 ^ k0;
        const uint32_t n2 = hi0 ^ c3 ^ k1;
        c0 = n0;
        c1 = lo1;
        c2 = n2;
        c3 = lo0;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    return Words4{c0, c1, c2, c3};
}

__device__ __forceinline__ Words4 rng_draw(RngKey key, uint64_t pid, uint32_t step, uint32_t tag, uint32_t idx)
{
    return philox4x32_10((uint32_t)pid, (uint32_t)(pid >> 32), step, (tag << 16) | idx, key.k0, key.k1);
}

// uniform on the open interval (0, 1): (w + 1/2) * 2^-32, exact in double
__device__ __forceinline__ double u01(uint32_t w) { return ((double)w + 0.5) * 2.3283064365386962890625e-10; }

// Box-Muller: two independent standard normal variates from two uniform words
__device__ __forceinline__ void box_muller(uint32_t a, uint32_t b, double& z0, double& z1)
{
    const double r = sqrt(-2.0 * log(u01(a)));
    double s, c;
    sincos(6.283185307179586 * u01(b), &s, &c);
    z0 = r * c;
    z1 = r * s;
}

// Gamma(shape >= 1) with the given mean, Marsaglia & Tsang (ACM TOMS 2000): attempt a
// draws from counter index a; after 16 rejected attempts the mean is returned.
__device__ __noinline__ double gamma_draw(double shape, double mean, RngKey key, uint64_t pid, uint32_t step,
                                          uint32_t tag)
{
    const double d = shape - 1.0 / 3.0;
    const double c = 1.0 / sqrt(9.0 * d);
    for (uint32_t a = 0; a < 16u; ++a) {
        const Words4 w = rng_draw(key, pid, step, tag, a);
        double x, unused;
        box_muller(w.w0, w.w1, x, unused);
        const double u = u01(w.w2);
        double v = 1.0 + c * x;
        if (v <= 0.0) continue;
        v = v * v * v;
        if (u < 1.0 - 0.0331 * (x * x) * (x * x)) return d * v * (mean / shape);
        if (log(u) < 0.5 * x * x + d * (1.0 - v + log(v))) return d * v * (mean / shape);
    }
    return mean;
}

// ------------------------------------------------------------------------------------
// P1 triangle geometry (Eqs. 37-38, 44-45)
// ------------------------------------------------------------------------------------
// signed area coordinates: N^A = ((r_C - r_B) x (r_P - r_B))/2, N^C = ((r_P - r_B) x (r_A - r_B))/2,
// N^B = A_e - N^A - N^C
__device__ __forceinline__ void area_coords(const ElemGeo* __restrict__ G, double x, double y, double& na,
                                            double& nb, double& nc)
{
    const double xa = G->x[0], xb = G->x[1], xc = G->x[2];
    const double ya = G->y[0], yb = G->y[1], yc = G->y[2];
    na = 0.5 * ((xc - xb) * (y - yb) - (yc - yb) * (x - xb));
    nc = 0.5 * ((x - xb) * (ya - yb) - (y - yb) * (xa - xb));
    nb = G->area - na - nc;
}

// ------------------------------------------------------------------------------------
// wavefront helpers (64 lanes)
// ------------------------------------------------------------------------------------
__device__ __forceinline__ int lane_id() { return (int)__lane_id(); }

// Runs of equal keys among consecutive lanes: leader lane of my run, run length (valid
// at the leader), my rank inside the run.
__device__ __forceinline__ void wave_runs(int32_t key, int& leader, int& len, int& rank)
{
    const int lane = lane_id();
    const int32_t prev = __shfl_up(key, 1u);
    const bool head = (lane == 0) || (key != prev);
    const unsigned long long heads = __ballot(head);
    const unsigned long long le = (lane == 63) ? ~0ull : ((1ull << (lane + 1)) - 1ull);
    leader = 63 - __clzll(heads & le);
    const unsigned long long above = heads & ~le;
    const int next = above ? (__ffsll((long long)above) - 1) : 64;
    len = next - lane;   // meaningful at the leader only
    rank = lane - leader;
}

__device__ __forceinline__ int wave_sum_int(int v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    return v;
}

__device__ __forceinline__ double wave_sum_double(double v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    return v;
}

}  // namespace pdfgpu
