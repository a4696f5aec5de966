// Device building blocks of libpdfgpu: counter-based random numbers, P1 geometry,
// wavefront collectives.  Included by the translation units that hold kernels.
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

__host__ __device__ __forceinline__ Words4 philox4x32_10(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                                        uint32_t k0, uint32_t k1)
{
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        // 32 x 32 -> 64-bit products: one v_mad_u64_u32 each on gfx950
        const uint64_t p0 = (uint64_t)0xD2511F53u * c0;
        const uint64_t p2 = (uint64_t)0xCD9E8D57u * c2;
        const uint32_t n0 = (uint32_t)(p2 >> 32) ^ c1 ^ k0;
        const uint32_t n2 = (uint32_t)(p0 >> 32) ^ c3 ^ k1;
        c1 = (uint32_t)p2;
        c3 = (uint32_t)p0;
        c0 = n0;
        c2 = n2;
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
__host__ __device__ __forceinline__ double u01(uint32_t w) { return ((double)w + 0.5) * 2.3283064365386962890625e-10; }

// sin(2 pi u) and cos(2 pi u) for u in [0, 1).  4u is exact, so the quadrant q and the
// fraction f = 4u - q are exact; folding f > 1/2 onto 1 - f (exact) leaves the angle
// (pi/2) f <= pi/4, where the Taylor series of sin and cos in f (coefficients
// (pi/2)^n / n!, rounded from 60-digit arithmetic) converge below 1e-17.
__host__ __device__ __forceinline__ void sincos_2pi(double u, double& s, double& c)
{
    const double t = 4.0 * u;
    const int q = (int)t;
    double f = t - (double)q;
    const bool fold = f > 0.5;
    if (fold) f = 1.0 - f;
    const double f2 = f * f;
    double ps = -0x1.8a404211f9547p-45;
    ps = fma(ps, f2, 0x1.aaec32af93359p-38);
    ps = fma(ps, f2, -0x1.6fadb9f155744p-31);
    ps = fma(ps, f2, 0x1.e8f434d018d63p-25);
    ps = fma(ps, f2, -0x1.e3074fde8871fp-19);
    ps = fma(ps, f2, 0x1.50783487ee782p-13);
    ps = fma(ps, f2, -0x1.32d2cce62bd86p-8);
    ps = fma(ps, f2, 0x1.466bc6775aae2p-4);
    ps = fma(ps, f2, -0x1.4abbce625be53p-1);
    ps = fma(ps, f2, 0x1.921fb54442d18p+0);
    const double sf = ps * f;
    double pc = 0x1.ef6e308d6d1c4p-49;
    pc = fma(pc, f2, -0x1.2a0c591af8314p-41);
    pc = fma(pc, f2, 0x1.20c62c2f2d7f5p-34);
    pc = fma(pc, f2, -0x1.b6e24f44b128fp-28);
    pc = fma(pc, f2, 0x1.f9d38a3763cc3p-22);
    pc = fma(pc, f2, -0x1.a6d1f2a204a8cp-16);
    pc = fma(pc, f2, 0x1.e1f506891babbp-11);
    pc = fma(pc, f2, -0x1.55d3c7e3cbffap-6);
    pc = fma(pc, f2, 0x1.03c1f081b5ac4p-2);
    pc = fma(pc, f2, -0x1.3bd3cc9be45dep+0);
    const double cf = fma(pc, f2, 1.0);
    const double sp = fold ? cf : sf, cp = fold ? sf : cf;   // sin, cos of (pi/2) * (4u - q)
    const bool odd = (q & 1) != 0, neg_s = q >= 2, neg_c = q == 1 || q == 2;
    const double a = odd ? cp : sp, b = odd ? sp : cp;
    s = neg_s ? -a : a;
    c = neg_c ? -b : b;
}

// natural logarithm for u in (0, 1]: u = m 2^e with m in [sqrt(1/2), sqrt(2)); log m =
// 2 atanh(s), s = (m - 1)/(m + 1), |s| <= 0.172, summed to s^25; ln 2 split so that e ln2_hi
// is exact.
__host__ __device__ __forceinline__ double log_unit(double u)
{
    int e;
    double m = frexp(u, &e);
    if (m < 0.7071067811865476) {
        m *= 2.0;
        e -= 1;
    }
    const double s = (m - 1.0) / (m + 1.0);
    const double z = s * s;
    double p = 1.0 / 25.0;
    p = fma(p, z, 1.0 / 23.0);
    p = fma(p, z, 1.0 / 21.0);
    p = fma(p, z, 1.0 / 19.0);
    p = fma(p, z, 1.0 / 17.0);
    p = fma(p, z, 1.0 / 15.0);
    p = fma(p, z, 1.0 / 13.0);
    p = fma(p, z, 1.0 / 11.0);
    p = fma(p, z, 1.0 / 9.0);
    p = fma(p, z, 1.0 / 7.0);
    p = fma(p, z, 1.0 / 5.0);
    p = fma(p, z, 1.0 / 3.0);
    const double lm = fma(2.0 * s, z * p, 2.0 * s);
    const double de = (double)e;
    return fma(de, 0x1.62e42fee00000p-1, fma(de, 0x1.a39ef35793c76p-33, lm));
}

// Box-Muller: two independent standard normal variates from two uniform words
__host__ __device__ __forceinline__ void box_muller(uint32_t a, uint32_t b, double& z0, double& z1)
{
    const double r = sqrt(-2.0 * log_unit(u01(a)));
    double s, c;
    sincos_2pi(u01(b), s, c);
    z0 = r * c;
    z1 = r * s;
}

// ------------------------------------------------------------------------------------
// mixed form: the same Philox words mapped in FP32
// ------------------------------------------------------------------------------------
// uniform on (0, 1) from the top 24 bits: ((w >> 8) + 1/2) * 2^-24, exact in float
__device__ __forceinline__ float u01f(uint32_t w) { return ((float)(w >> 8) + 0.5f) * 5.9604644775390625e-8f; }

// uniform on (0, 1) from all 32 bits with the relative precision of a float at every
// magnitude: (w + 1/2) 2^-32, w rounded to 24 significant bits, kept below 1.  The radius
// of the Box-Muller map takes its logarithm, so small u (the tail of the Gaussian) must not
// lose the low bits that the 24-bit map above drops.
__device__ __forceinline__ float u01f_fine(uint32_t w)
{
    return fminf(fmaf((float)w, 0x1p-32f, 0x1p-33f), 0x1.fffffep-1f);
}

__device__ __forceinline__ void box_muller_f(uint32_t a, uint32_t b, float& z0, float& z1)
{
    const float r = sqrtf(-2.0f * logf(u01f_fine(a)));
    float s, c;
    sincospif(2.0f * u01f(b), &s, &c);   // sin, cos of 2 pi u; 2u is exact
    z0 = r * c;
    z1 = r * s;
}

// precision-generic wrappers: R = double (FP64 form) or float (mixed form)
template <class R> struct RMath;
template <> struct RMath<double> {
    __device__ static double uni(uint32_t w) { return u01(w); }
    __device__ static void normal2(uint32_t a, uint32_t b, double& z0, double& z1) { box_muller(a, b, z0, z1); }
    __device__ static double sqrt_(double v) { return sqrt(v); }
    __device__ static double log_(double v) { return log(v); }
    __device__ static double exp_(double v) { return exp(v); }
};
template <> struct RMath<float> {
    __device__ static float uni(uint32_t w) { return u01f(w); }
    __device__ static void normal2(uint32_t a, uint32_t b, float& z0, float& z1) { box_muller_f(a, b, z0, z1); }
    __device__ static float sqrt_(float v) { return sqrtf(v); }
    __device__ static float log_(float v) { return logf(v); }
    __device__ static float exp_(float v) { return expf(v); }
};

// Gamma(shape >= 1) with the given mean, Marsaglia & Tsang (ACM TOMS 2000): attempt a
// draws from counter index a; after 16 rejected attempts the mean is returned.
template <class R>
__device__ __noinline__ R gamma_draw(R shape, R mean, RngKey key, uint64_t pid, uint32_t step, uint32_t tag)
{
    using M = RMath<R>;
    const R d = shape - R(1) / R(3);
    const R c = R(1) / M::sqrt_(R(9) * d);
    for (uint32_t a = 0; a < 16u; ++a) {
        const Words4 w = rng_draw(key, pid, step, tag, a);
        R x, unused;
        M::normal2(w.w0, w.w1, x, unused);
        const R u = M::uni(w.w2);
        R v = R(1) + c * x;
        if (v <= R(0)) continue;
        v = v * v * v;
        if (u < R(1) - R(0.0331) * (x * x) * (x * x)) return d * v * (mean / shape);
        if (M::log_(u) < R(0.5) * x * x + d * (R(1) - v + M::log_(v))) return d * v * (mean / shape);
    }
    return mean;
}

// Running sum: plain in FP64; Kahan-compensated in FP32 (mixed form)
template <class R> struct Acc;
template <> struct Acc<double> {
    double s = 0.0;
    __device__ void add(double v) { s += v; }
    __device__ double value() const { return s; }
};
template <> struct Acc<float> {
    float s = 0.0f, c = 0.0f;
    __device__ void add(float v)
    {
        const float y = v - c;
        const float t = s + y;
        c = (t - s) - y;
        s = t;
    }
    __device__ float value() const { return s - c; }
};

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
    // explicit fused multiply-adds: the same rounding in every kernel, whatever registers
    // (scalar or vector) the vertex coordinates sit in
    na = 0.5 * fma(xc - xb, y - yb, -((yc - yb) * (x - xb)));
    nc = 0.5 * fma(x - xb, ya - yb, -((y - yb) * (xa - xb)));
    nb = G->area - na - nc;
}

// Eq. (26) ingredients of node n: l = sqrt of the average area of the elements around the
// node (inf without elements), z = |(<U1>, <U2>, <U3>, <omega>, <psi>)| where the node has
// statistics (W > 0), else 0
__device__ __forceinline__ void cfl_node(const ElemGeo* __restrict__ geo, const int64_t* __restrict__ n2e_ptr,
                                         const int32_t* __restrict__ n2e, const double* __restrict__ stats, int64_t n,
                                         double& l, double& z)
{
    const int64_t j0 = n2e_ptr[n], j1 = n2e_ptr[n + 1];
    if (j1 > j0) {
        double a = 0.0;
        for (int64_t j = j0; j < j1; ++j) a += geo[n2e[j] / 3].area;
        l = sqrt(a / (double)(j1 - j0));
    }
    const double* o = stats + n * NSTAT;
    if (o[0] > 0.0) {
        double s = 0.0;
        for (int q = 1; q <= 5; ++q) s += o[q] * o[q];
        z = sqrt(s);
    }
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

// FP32 butterfly sum carrying the rounding error of every addition (two-sum), so the
// result is as accurate as a sum in twice the precision
__device__ __forceinline__ float wave_sum_comp(float v)
{
    float c = 0.0f;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        const float w = __shfl_xor(v, o), cw = __shfl_xor(c, o);
        const float s = v + w;
        const float bb = s - v;
        const float e = (v - (s - bb)) + (w - bb);
        v = s;
        c = c + cw + e;
    }
    return v + c;
}

template <class R> __device__ __forceinline__ R wave_sum_real(R v);
template <> __device__ __forceinline__ double wave_sum_real<double>(double v) { return wave_sum_double(v); }
template <> __device__ __forceinline__ float wave_sum_real<float>(float v) { return wave_sum_comp(v); }

}  // namespace pdfgpu
