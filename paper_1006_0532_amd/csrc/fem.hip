// P1 finite-element kernels of the Eulerian solves (Sec. 3.2); see fem.h.
#include <hip/hip_runtime.h>

#include "device.h"
#include "fem.h"

namespace pdfgpu {

namespace {

inline unsigned blocks(int64_t n, int nt) { return (unsigned)((n + nt - 1) / nt); }

// dN_a/dx, dN_a/dy of the element's three vertices (Eqs. 39-40)
__device__ __forceinline__ void p1_grad(const ElemGeo& G, double (&bx)[3], double (&by)[3])
{
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const int b = a == 2 ? 0 : a + 1, c = a == 0 ? 2 : a - 1;
        bx[a] = (G.y[b] - G.y[c]) / (2.0 * G.area);
        by[a] = (G.x[c] - G.x[b]) / (2.0 * G.area);
    }
}

__global__ void __launch_bounds__(256) k_fem_elem_matrices(const ElemGeo* __restrict__ geo, int64_t ne,
                                                           double* __restrict__ ke)
{
    const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (e >= ne) return;
    const ElemGeo& G = geo[e];
    double bx[3], by[3];
    p1_grad(G, bx, by);
    double* k = ke + e * 8;
    k[0] = G.area * (bx[0] * bx[0] + by[0] * by[0]);
    k[1] = G.area * (bx[1] * bx[1] + by[1] * by[1]);
    k[2] = G.area * (bx[2] * bx[2] + by[2] * by[2]);
    k[3] = G.area * (bx[0] * bx[1] + by[0] * by[1]);
    k[4] = G.area * (bx[0] * bx[2] + by[0] * by[2]);
    k[5] = G.area * (bx[1] * bx[2] + by[1] * by[2]);
    k[6] = G.area / 12.0;
    k[7] = 0.0;
}

// row n of (mass M + stiff L^2 K) x, or its diagonal (x unused); Dirichlet rows give 0
// (diagonal: 1)
template <int NC>
__global__ void __launch_bounds__(256) k_fem_apply(FemOp op, const double* x, double* y, int diag_only)
{
    const int64_t n = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (n >= op.nn) return;
    double acc[NC];
#pragma unroll
    for (int c = 0; c < NC; ++c) acc[c] = 0.0;
    for (int64_t j = op.n2e_ptr[n]; j < op.n2e_ptr[n + 1]; ++j) {
        const int32_t v = op.n2e[j];
        const int64_t e = v / 3;
        const int a = v - 3 * (int)e;
        const ElemGeo& G = op.geo[e];
        const double* K = op.ke + e * 8;
        double l2[4] = {1.0, 1.0, 1.0, 1.0};
        if (op.L2)
#pragma unroll
            for (int q = 0; q < 4; ++q) l2[q] = op.L2[e * 4 + q];
        for (int b = 0; b < 3; ++b) {
            if (diag_only && b != a) continue;
            // (a, b) -> slot: diagonal a; (0, 1), (0, 2), (1, 2) -> 3, 4, 5
            const double kab = K[a == b ? a : a + b + 2];
            const double mab = K[6] * (a == b ? 2.0 : 1.0);
            const int64_t nb = G.node[b];
#pragma unroll
            for (int c = 0; c < NC; ++c) {
                const double l = NC == 9 ? ((c / 3 == c % 3) ? l2[c / 3] : l2[3]) : l2[0];
                const double coef = op.mass * mab + op.stiff * (l * kab);
                acc[c] += coef * (diag_only ? 1.0 : x[nb * NC + c]);
            }
        }
    }
    const uint32_t fm = op.fixed[n];
    const double fixed_value = diag_only ? 1.0 : 0.0;
#pragma unroll
    for (int c = 0; c < NC; ++c) y[n * NC + c] = ((fm >> c) & 1u) ? fixed_value : acc[c];
}

__global__ void __launch_bounds__(256) k_fem_assemble4(FemOp op, double* __restrict__ cval)
{
    const int64_t n = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (n >= op.nn) return;
    const int32_t k0 = op.crp[n], k1 = op.crp[n + 1];
    for (int32_t k = k0; k < k1; ++k)
#pragma unroll
        for (int g = 0; g < 4; ++g) cval[g * op.nnz + k] = 0.0;
    for (int64_t j = op.n2e_ptr[n]; j < op.n2e_ptr[n + 1]; ++j) {
        const int32_t v = op.n2e[j];
        const int64_t e = v / 3;
        const int a = v - 3 * (int)e;
        const double* K = op.ke + e * 8;
        double l2[4] = {1.0, 1.0, 1.0, 1.0};
        if (op.L2)
#pragma unroll
            for (int q = 0; q < 4; ++q) l2[q] = op.L2[e * 4 + q];
        for (int b = 0; b < 3; ++b) {
            const int32_t nb = op.geo[e].node[b];
            int32_t k = k0;
            while (k < k1 - 1 && op.ccol[k] != nb) ++k;     // the row holds every vertex of its elements
            const double kab = K[a == b ? a : a + b + 2];
            const double mab = K[6] * (a == b ? 2.0 : 1.0);
#pragma unroll
            for (int g = 0; g < 4; ++g) cval[g * op.nnz + k] += op.mass * mab + op.stiff * (l2[g] * kab);
        }
    }
}

// y = A x (diag_only: the diagonal) of the assembled nine-component operator, a thread per
// (row, component); Dirichlet rows give 0 (diagonal: 1)
__global__ void __launch_bounds__(256) k_fem_apply_csr9(FemOp op, const double* __restrict__ x,
                                                        double* __restrict__ y, int diag_only)
{
    const int64_t q = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (q >= op.nn * 9) return;
    const int64_t n = q / 9;
    const int c = (int)(q - 9 * n);
    const int g = c / 3 == c % 3 ? c / 3 : 3;
    const double* __restrict__ v = op.cval + g * op.nnz;
    double acc = 0.0;
    for (int32_t k = op.crp[n]; k < op.crp[n + 1]; ++k) {
        const int32_t j = op.ccol[k];
        if (diag_only) {
            if (j == n) acc = v[k];
        } else {
            acc += v[k] * x[(int64_t)j * 9 + c];
        }
    }
    const bool fx = (op.fixed[n] >> c) & 1u;
    y[q] = fx ? (diag_only ? 1.0 : 0.0) : acc;
}

template <int NC>
__global__ void __launch_bounds__(256) k_fem_dot(const double* __restrict__ a, const double* __restrict__ b,
                                                 const double* __restrict__ a2, const double* __restrict__ b2,
                                                 int64_t nn, double* __restrict__ partial)
{
    constexpr int NQ = 2 * NC;
    __shared__ double red[4][NQ];
    double s[NQ];
#pragma unroll
    for (int q = 0; q < NQ; ++q) s[q] = 0.0;
    for (int64_t n = (int64_t)blockIdx.x * 256 + threadIdx.x; n < nn; n += (int64_t)gridDim.x * 256) {
#pragma unroll
        for (int c = 0; c < NC; ++c) {
            s[c] += a[n * NC + c] * (b ? b[n * NC + c] : 1.0);
            if (a2) s[NC + c] += a2[n * NC + c] * b2[n * NC + c];
        }
    }
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
        const double t = wave_sum_double(s[q]);
        if (lane == 0) red[w][q] = t;
    }
    __syncthreads();
    if (threadIdx.x < NQ) {
        double t = 0.0;
        for (int k = 0; k < 4; ++k) t += red[k][threadIdx.x];
        partial[(int64_t)blockIdx.x * NQ + threadIdx.x] = t;
    }
}

// out[q] = sum over the nb partials of component q (q < nout <= 18): a workgroup of 256
// sums them in one fixed order (strided per thread, then the wavefronts, then the four
// wavefront sums), so the loads are in flight together
__global__ void __launch_bounds__(256) k_fem_dot_finish(const double* __restrict__ partial, int nb, int nq, int nout,
                                                        double* __restrict__ out)
{
    __shared__ double red[4][18];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    for (int q = 0; q < nout; ++q) {
        double t = 0.0;
        for (int k = threadIdx.x; k < nb; k += 256) t += partial[(int64_t)k * nq + q];
        t = wave_sum_double(t);
        if (lane == 0) red[w][q] = t;
    }
    __syncthreads();
    const int q = threadIdx.x;
    if (q < nout) out[q] = (red[0][q] + red[1][q]) + (red[2][q] + red[3][q]);
}

template <int NC>
__global__ void __launch_bounds__(256) k_cg_init(const double* __restrict__ b, const double* __restrict__ Ax,
                                                 const double* __restrict__ diag, const uint16_t* __restrict__ fixed,
                                                 int64_t n, double* __restrict__ r, double* __restrict__ z,
                                                 double* __restrict__ p)
{
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    const bool fx = (fixed[i / NC] >> (int)(i % NC)) & 1u;
    const double ri = fx ? 0.0 : b[i] - Ax[i];
    const double zi = fx ? 0.0 : ri / diag[i];
    r[i] = ri;
    z[i] = zi;
    p[i] = zi;
}

template <int NC>
__global__ void k_cg_alpha(double* sc)
{
    const int c = threadIdx.x;
    if (c >= NC) return;
    const double rz = sc[c], pap = sc[NC + c];
    sc[4 * NC + c] = pap > 0.0 ? rz / pap : 0.0;
}

template <int NC>
__global__ void __launch_bounds__(256) k_cg_xr(const double* __restrict__ sc, const double* __restrict__ p,
                                               const double* __restrict__ Ap, const double* __restrict__ diag,
                                               const uint16_t* __restrict__ fixed, int64_t nn, double* __restrict__ x,
                                               double* __restrict__ r, double* __restrict__ z)
{
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= nn * NC) return;
    const int c = (int)(i % NC);
    const double al = sc[4 * NC + c];
    x[i] += al * p[i];
    const double ri = r[i] - al * Ap[i];
    r[i] = ri;
    z[i] = ((fixed[i / NC] >> c) & 1u) ? 0.0 : ri / diag[i];
}

template <int NC>
__global__ void k_cg_beta(double* sc)
{
    const int c = threadIdx.x;
    if (c >= NC) return;
    const double rz = sc[c], rzn = sc[2 * NC + c];
    sc[5 * NC + c] = rz > 0.0 ? rzn / rz : 0.0;
    sc[c] = rzn;
}

template <int NC>
__global__ void __launch_bounds__(256) k_cg_p(const double* __restrict__ sc, const double* __restrict__ z,
                                              int64_t nn, double* __restrict__ p)
{
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= nn * NC) return;
    p[i] = z[i] + sc[5 * NC + (int)(i % NC)] * p[i];
}

// element gradient of the nodal mean velocity (components 0..2 of the statistics' means)
__device__ __forceinline__ void elem_grad_u(const ElemGeo& G, const double* __restrict__ stats, double (&g)[3][2])
{
    double bx[3], by[3];
    p1_grad(G, bx, by);
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        double gx = 0.0, gy = 0.0;
#pragma unroll
        for (int b = 0; b < 3; ++b) {
            const double u = stats[(int64_t)G.node[b] * NSTAT + 1 + c];
            gx += bx[b] * u;
            gy += by[b] * u;
        }
        g[c][0] = gx;
        g[c][1] = gy;
    }
}

// k, epsilon (Eq. 18) from nodal statistics
__device__ __forceinline__ void k_eps(const double* o, double nu, double CT, double& k, double& eps)
{
    k = 0.5 * (o[6] + o[7] + o[8]);
    const double om = o[4];
    eps = om * (k + nu * CT * CT * om);
}

__global__ void __launch_bounds__(256) k_fem_elliptic_nodes(const ElemGeo* __restrict__ geo,
                                                            const int64_t* __restrict__ n2e_ptr,
                                                            const int32_t* __restrict__ n2e,
                                                            const double* __restrict__ stats, int64_t nn,
                                                            EllipticConst cst, const uint8_t* __restrict__ wkind,
                                                            const double* __restrict__ wnrm, double* __restrict__ f,
                                                            double* __restrict__ xfix, uint16_t* __restrict__ fixed)
{
    const int64_t n = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (n >= nn) return;
    const double* o = stats + n * NSTAT;
    // nodal velocity gradient: plain average of the element gradients around the node
    double G[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
    const int64_t j0 = n2e_ptr[n], j1 = n2e_ptr[n + 1];
    for (int64_t j = j0; j < j1; ++j) {
        double g[3][2];
        elem_grad_u(geo[n2e[j] / 3], stats, g);
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            G[c][0] += g[c][0];
            G[c][1] += g[c][1];
        }
    }
    const double cnt = (double)(j1 - j0);
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        G[c][0] /= cnt;
        G[c][1] /= cnt;
    }
    double R[3][3];
    R[0][0] = o[6];
    R[1][1] = o[7];
    R[2][2] = o[8];
    R[0][1] = R[1][0] = o[9];
    R[0][2] = R[2][0] = o[10];
    R[1][2] = R[2][1] = o[11];
    double k, eps;
    k_eps(o, cst.nu, cst.CT, k, eps);
    const double om = o[4];
    const double det = R[0][0] * (R[1][1] * R[2][2] - R[1][2] * R[2][1]) -
                       R[0][1] * (R[1][0] * R[2][2] - R[1][2] * R[2][0]) +
                       R[0][2] * (R[1][0] * R[2][1] - R[1][1] * R[2][0]);
    const double k23 = 2.0 * k / 3.0;
    const double Av = fmin(1.0, cst.Cv * det / (k23 * k23 * k23));             // Eq. (14)
    double bt[3][3];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int jj = 0; jj < 3; ++jj) bt[i][jj] = R[i][jj] / (2.0 * k) - (i == jj ? 1.0 / 3.0 : 0.0);   // Eq. (15)
    const double g5 = cst.gamma5;
    const int wk = wkind[n];
    const double n3[3] = {wk == 2 ? wnrm[2 * n] : 0.0, wk == 2 ? wnrm[2 * n + 1] : 0.0, 0.0};
    uint32_t fm = 0;
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int jj = 0; jj < 3; ++jj) {
            // H_ijkl dU_k/dx_l with H of Eq. (13)
            double h = (cst.C2 * Av + g5 / 3.0) * G[i][jj] - g5 / 3.0 * G[jj][i];
            double t3 = 0.0, t4 = 0.0;
#pragma unroll
            for (int q = 0; q < 3; ++q) {
                t3 += bt[i][q] * G[q][jj];
                t4 += bt[i][q] * G[jj][q];
            }
            h = h + g5 * t3 - g5 * t4;
            const int c = 3 * i + jj;
            f[n * 9 + c] = k * h + (i == jj ? 0.5 * (1.0 - cst.C1) * k * om : 0.0);
            const bool fx = wk == 2 || (wk == 1 && i != jj);
            fm |= (fx ? 1u : 0u) << c;
            xfix[n * 9 + c] = wk == 2 ? -4.5 * eps * n3[i] * n3[jj] : 0.0;      // Eq. (59)
        }
    fixed[n] = (uint16_t)fm;
}

__global__ void __launch_bounds__(256) k_fem_elliptic_elems(const ElemGeo* __restrict__ geo,
                                                            const double* __restrict__ stats, int64_t ne,
                                                            EllipticConst cst, const double* __restrict__ enrm,
                                                            double* __restrict__ L2)
{
    const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (e >= ne) return;
    const ElemGeo& G = geo[e];
    double ks = 0.0, es = 0.0;
#pragma unroll
    for (int v = 0; v < 3; ++v) {
        double k, eps;
        k_eps(stats + (int64_t)G.node[v] * NSTAT, cst.nu, cst.CT, k, eps);
        ks += k;
        es += eps;
    }
    const double ke = ks / 3.0, ee = es / 3.0;
    const double kol = cst.Ceta * pow(cst.nu * cst.nu * cst.nu / ee, 0.25);
    const double turb = pow(ke, 1.5) / ee;
    const double n3[3] = {enrm[2 * e], enrm[2 * e + 1], 0.0};
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const double cxi = i < 3 ? 1.0 + 1.3 * n3[i] * n3[i] : 1.0;                 // Eq. (17)
        const double L = cst.CL * fmax(cxi * turb, kol);                             // Eq. (16)
        L2[e * 4 + i] = L * L;
    }
}

__global__ void __launch_bounds__(256) k_fem_set_fixed(const double* __restrict__ xfix,
                                                       const uint16_t* __restrict__ fixed, int64_t nn,
                                                       double* __restrict__ x)
{
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i < 9 * nn) x[i] = ((fixed[i / 9] >> (int)(i % 9)) & 1u) ? xfix[i] : x[i];
}

__global__ void __launch_bounds__(256) k_fem_pressure_rhs(FemOp op, const double* __restrict__ stats,
                                                          const double* __restrict__ P, double rho, double dt,
                                                          double cp, double* __restrict__ b)
{
    const int64_t n = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (n >= op.nn) return;
    double D = 0.0, KP = 0.0;
    for (int64_t j = op.n2e_ptr[n]; j < op.n2e_ptr[n + 1]; ++j) {
        const int32_t v = op.n2e[j];
        const int64_t e = v / 3;
        const int a = v - 3 * (int)e;
        const ElemGeo& G = op.geo[e];
        double bx[3], by[3];
        p1_grad(G, bx, by);
        double div = 0.0;
#pragma unroll
        for (int q = 0; q < 3; ++q) {
            const double* o = stats + (int64_t)G.node[q] * NSTAT;
            div += bx[q] * o[1];
        }
#pragma unroll
        for (int q = 0; q < 3; ++q) {
            const double* o = stats + (int64_t)G.node[q] * NSTAT;
            div += by[q] * o[2];
        }
        D += G.area * div / 3.0;
#pragma unroll
        for (int q = 0; q < 3; ++q) KP += G.area * (bx[a] * bx[q] + by[a] * by[q]) * P[G.node[q]];
    }
    b[n] = -(rho / dt) * D - (cp / dt) * KP;
}

__global__ void __launch_bounds__(256) k_fem_sub_mean(const double* __restrict__ sum, int64_t nn,
                                                      double* __restrict__ v)
{
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i < nn) v[i] = v[i] - sum[0] / (double)nn;
}

__global__ void __launch_bounds__(256) k_fem_add(const double* __restrict__ a, int64_t n, double* __restrict__ y)
{
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i < n) y[i] += a[i];
}

__global__ void __launch_bounds__(256) k_fem_check_stats(const double* __restrict__ stats, int64_t nn,
                                                         unsigned long long* __restrict__ count)
{
    const int64_t n = (int64_t)blockIdx.x * 256 + threadIdx.x;
    bool bad = false;
    if (n < nn)
        for (int q = 0; q < 12; ++q) bad |= !isfinite(stats[n * NSTAT + q]);
    const unsigned long long m = __ballot(bad);
    if ((threadIdx.x & 63) == 0 && m) atomicAdd(count, (unsigned long long)__popcll(m));
}

__global__ void __launch_bounds__(256) k_fem_elem_grad(const ElemGeo* __restrict__ geo, const double* __restrict__ q,
                                                       int64_t ne, double* __restrict__ g)
{
    const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (e >= ne) return;
    const ElemGeo& G = geo[e];
    double bx[3], by[3];
    p1_grad(G, bx, by);
    double gx = 0.0, gy = 0.0;
#pragma unroll
    for (int b = 0; b < 3; ++b) {
        gx += bx[b] * q[G.node[b]];
        gy += by[b] * q[G.node[b]];
    }
    g[2 * e] = gx;
    g[2 * e + 1] = gy;
}

__global__ void __launch_bounds__(256) k_fem_pressure_update(const int64_t* __restrict__ n2e_ptr,
                                                             const int32_t* __restrict__ n2e,
                                                             const double* __restrict__ gP,
                                                             const double* __restrict__ gdP,
                                                             const double* __restrict__ gp0, int64_t nn,
                                                             double scale, double* __restrict__ node,
                                                             double* __restrict__ stats)
{
    const int64_t n = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (n >= nn) return;
    double a0 = 0.0, a1 = 0.0, d0 = 0.0, d1 = 0.0;
    const int64_t j0 = n2e_ptr[n], j1 = n2e_ptr[n + 1];
    for (int64_t j = j0; j < j1; ++j) {
        const int64_t e = n2e[j] / 3;
        a0 += gP[2 * e];
        a1 += gP[2 * e + 1];
        d0 += gdP[2 * e];
        d1 += gdP[2 * e + 1];
    }
    const double cnt = (double)(j1 - j0);
    node[n * NODE_STRIDE + NF_GP] = gp0[2 * n] + a0 / cnt;
    node[n * NODE_STRIDE + NF_GP + 1] = gp0[2 * n + 1] + a1 / cnt;
    double* o = stats + n * NSTAT;
    if (o[0] > 0.0) {
        o[1] -= scale * (d0 / cnt);
        o[2] -= scale * (d1 / cnt);
    }
}

template <class R>
__global__ void __launch_bounds__(256) k_fem_correct_particles(SoaT<R> st, const int64_t* __restrict__ nslots,
                                                               int64_t n_ub, const double* __restrict__ gdP,
                                                               double scale)
{
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= n_ub || i >= nslots[0]) return;
    const int32_t e = st.elem[i];
    if (e < 0) return;
    const double d0 = scale * gdP[2 * (int64_t)e], d1 = scale * gdP[2 * (int64_t)e + 1];
    st.u0[i] = (R)((double)st.u0[i] - d0);
    st.u1[i] = (R)((double)st.u1[i] - d1);
}

// outward normal of the no-slip wall edge whose midpoint is nearest to the element centroid
// (minimum image across a periodic seam of length L; first minimum in edge order)
__global__ void __launch_bounds__(256) k_fem_nearest_wall(const ElemGeo* __restrict__ geo, int64_t ne,
                                                          const double* __restrict__ edges, int32_t nw, double L,
                                                          double* __restrict__ enrm)
{
    const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (e >= ne) return;
    const ElemGeo& G = geo[e];
    const double cx = (G.x[0] + G.x[1] + G.x[2]) / 3.0, cy = (G.y[0] + G.y[1] + G.y[2]) / 3.0;
    double best = __builtin_inf();
    int32_t jb = -1;
    for (int32_t j = 0; j < nw; ++j) {
        double dx = edges[4 * j] - cx;
        if (L > 0.0) dx = dx - L * rint(dx / L);
        const double dy = edges[4 * j + 1] - cy;
        const double d2 = dx * dx + dy * dy;
        if (d2 < best) {
            best = d2;
            jb = j;
        }
    }
    enrm[2 * e] = jb >= 0 ? edges[4 * jb + 2] : 0.0;
    enrm[2 * e + 1] = jb >= 0 ? edges[4 * jb + 3] : 0.0;
}

__global__ void __launch_bounds__(256) k_fem_store_wp(const double* __restrict__ x, int64_t nn,
                                                      double* __restrict__ node)
{
    const int64_t n = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (n >= nn) return;
    const double* w = x + 9 * n;
    double* f = node + n * NODE_STRIDE;
    f[NF_WP] = w[0];
    f[NF_WP + 1] = w[4];
    f[NF_WP + 2] = w[8];
    f[NF_WP + 3] = w[1];
    f[NF_WP + 4] = w[2];
    f[NF_WP + 5] = w[5];
    f[NF_WPT] = w[3];
    f[NF_WPT + 1] = w[6];
    f[NF_WPT + 2] = w[7];
}


// ---- assembled scalar operator (pressure) with fused reductions ----
__device__ __forceinline__ void block_partial(double v, double* red, double* out)
{
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    v = wave_sum_double(v);
    if (lane == 0) red[w] = v;
    __syncthreads();
    if (threadIdx.x == 0) *out = (red[0] + red[1]) + (red[2] + red[3]);
}

__global__ void __launch_bounds__(256) k_csr_apply_dot(const int32_t* __restrict__ row_ptr,
                                                       const int32_t* __restrict__ col,
                                                       const double* __restrict__ val, const double* __restrict__ x,
                                                       int64_t nn, double* __restrict__ y, double* __restrict__ partial)
{
    __shared__ double red[4];
    const int64_t n = (int64_t)blockIdx.x * 256 + threadIdx.x;
    double pq = 0.0;
    if (n < nn) {
        double acc = 0.0;
        for (int32_t j = row_ptr[n]; j < row_ptr[n + 1]; ++j) acc += val[j] * x[col[j]];
        y[n] = acc;
        pq = x[n] * acc;
    }
    block_partial(pq, red, partial + blockIdx.x);
}

__global__ void __launch_bounds__(256) k_csr_diag(const int32_t* __restrict__ row_ptr, const int32_t* __restrict__ col,
                                                  const double* __restrict__ val, int64_t nn, double* __restrict__ d)
{
    const int64_t n = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (n >= nn) return;
    double v = 1.0;
    for (int32_t j = row_ptr[n]; j < row_ptr[n + 1]; ++j)
        if (col[j] == n) v = val[j];
    d[n] = v;
}

// sum of nb partials (stride q apart, nq per block) by one workgroup in a fixed order
__device__ __forceinline__ double finish_sum(const double* partial, int nb, int nq, int q, double* red)
{
    double t = 0.0;
    for (int k = threadIdx.x; k < nb; k += 256) t += partial[(int64_t)k * nq + q];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    t = wave_sum_double(t);
    if (lane == 0) red[w] = t;
    __syncthreads();
    const double v = (red[0] + red[1]) + (red[2] + red[3]);
    __syncthreads();
    return v;
}

// CG in two launches per iteration on CG2_BLOCKS workgroups (grid-stride rows): each
// workgroup sums the CG2_BLOCKS partials of the launch before in the same fixed order, so
// the scalars need no launch of their own; p is updated on the fly inside the product.
// Scalars: sc[0], sc[1] hold r.z of alternate iterations.
__device__ __forceinline__ double finish_cg2(const double* __restrict__ partial, int stride, int o, double* red)
{
    double t = 0.0;
    for (int q = threadIdx.x; q < CG2_BLOCKS; q += 256) t += partial[q * stride + o];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    t = wave_sum_double(t);
    if (lane == 0) red[w] = t;
    __syncthreads();
    const double v = (red[0] + red[1]) + (red[2] + red[3]);
    __syncthreads();
    return v;
}

// iteration k: beta = (r.z now) / (r.z of iteration k - 1) (0 at k = 0), p_k = z + beta
// p_(k-1) read from pold and written to pnew for the own rows, y = K p_k and the
// partials of p_k . y
__global__ void __launch_bounds__(256) k_cg2_apply(const int32_t* __restrict__ row_ptr, const int32_t* __restrict__ col,
                                                   const double* __restrict__ val, const double* __restrict__ z,
                                                   const double* __restrict__ pold, double* __restrict__ pnew,
                                                   int64_t nn, double* __restrict__ y,
                                                   const double* __restrict__ part_rz, double* __restrict__ part_py,
                                                   double* __restrict__ sc, int k)
{
    __shared__ double red[4];
    const double rz = finish_cg2(part_rz, 2, 0, red);
    const double rz_prev = sc[(k + 1) & 1];
    const double beta = (k > 0 && rz_prev > 0.0) ? rz / rz_prev : 0.0;
    if (blockIdx.x == 0 && threadIdx.x == 0) sc[k & 1] = rz;
    double pq = 0.0;
    for (int64_t n = (int64_t)blockIdx.x * 256 + threadIdx.x; n < nn; n += (int64_t)gridDim.x * 256) {
        double acc = 0.0;
        for (int32_t j = row_ptr[n]; j < row_ptr[n + 1]; ++j) {
            const int32_t c = col[j];
            acc += val[j] * (z[c] + beta * pold[c]);
        }
        const double pn = z[n] + beta * pold[n];
        pnew[n] = pn;
        y[n] = acc;
        pq += pn * acc;
    }
    block_partial(pq, red, part_py + blockIdx.x);
}

// iteration k: alpha = (r.z) / (p . K p); x += alpha p, r -= alpha K p, z = r / diag, and
// the partials of r.z and r.r
__global__ void __launch_bounds__(256) k_cg2_update(const double* __restrict__ sc, const double* __restrict__ part_py,
                                                    const double* __restrict__ p, const double* __restrict__ y,
                                                    const double* __restrict__ diag, int64_t nn, double* __restrict__ x,
                                                    double* __restrict__ r, double* __restrict__ z,
                                                    double* __restrict__ part_rz, int k)
{
    __shared__ double red[4];
    const double pap = finish_cg2(part_py, 1, 0, red);
    const double rz = sc[k & 1];
    const double al = pap > 0.0 ? rz / pap : 0.0;
    double rzl = 0.0, rrl = 0.0;
    for (int64_t n = (int64_t)blockIdx.x * 256 + threadIdx.x; n < nn; n += (int64_t)gridDim.x * 256) {
        x[n] += al * p[n];
        const double ri = r[n] - al * y[n];
        const double zi = ri / diag[n];
        r[n] = ri;
        z[n] = zi;
        rzl += ri * zi;
        rrl += ri * ri;
    }
    block_partial(rzl, red, part_rz + 2 * blockIdx.x);
    __syncthreads();
    block_partial(rrl, red, part_rz + 2 * blockIdx.x + 1);
}

// iteration k with a preconditioner applied outside: alpha as in k_cg2_update; x += alpha p,
// r -= alpha K p only
__global__ void __launch_bounds__(256) k_cg2_update_xr(const double* __restrict__ sc,
                                                       const double* __restrict__ part_py, const double* __restrict__ p,
                                                       const double* __restrict__ y, int64_t nn,
                                                       double* __restrict__ x, double* __restrict__ r, int k)
{
    __shared__ double red[4];
    const double pap = finish_cg2(part_py, 1, 0, red);
    const double rz = sc[k & 1];
    const double al = pap > 0.0 ? rz / pap : 0.0;
    for (int64_t n = (int64_t)blockIdx.x * 256 + threadIdx.x; n < nn; n += (int64_t)gridDim.x * 256) {
        x[n] += al * p[n];
        r[n] -= al * y[n];
    }
}

// partials of r.z and r.r in the layout of k_cg2_update
__global__ void __launch_bounds__(256) k_cg2_dots(const double* __restrict__ r, const double* __restrict__ z, int64_t nn,
                                                  double* __restrict__ part_rz)
{
    __shared__ double red[4];
    double rzl = 0.0, rrl = 0.0;
    for (int64_t n = (int64_t)blockIdx.x * 256 + threadIdx.x; n < nn; n += (int64_t)gridDim.x * 256) {
        rzl += r[n] * z[n];
        rrl += r[n] * r[n];
    }
    block_partial(rzl, red, part_rz + 2 * blockIdx.x);
    __syncthreads();
    block_partial(rrl, red, part_rz + 2 * blockIdx.x + 1);
}

}  // namespace

int fem_csr_blocks(int64_t nn) { return (int)blocks(nn > 0 ? nn : 1, 256); }
void fem_csr_apply_dot(const int32_t* row_ptr, const int32_t* col, const double* val, const double* x, int64_t nn,
                       double* y, double* partial, int nblocks, hipStream_t s)
{
    hipLaunchKernelGGL(k_csr_apply_dot, dim3(nblocks), dim3(256), 0, s, row_ptr, col, val, x, nn, y, partial);
}
void fem_csr_diag(const int32_t* row_ptr, const int32_t* col, const double* val, int64_t nn, double* d, hipStream_t s)
{
    if (nn > 0) hipLaunchKernelGGL(k_csr_diag, dim3(blocks(nn, 256)), dim3(256), 0, s, row_ptr, col, val, nn, d);
}
void fem_cg2_apply(const int32_t* row_ptr, const int32_t* col, const double* val, const double* z, const double* pold,
                   double* pnew, int64_t nn, double* y, const double* part_rz, double* part_py, double* sc, int k,
                   hipStream_t s)
{
    hipLaunchKernelGGL(k_cg2_apply, dim3(CG2_BLOCKS), dim3(256), 0, s, row_ptr, col, val, z, pold, pnew, nn, y, part_rz,
                       part_py, sc, k);
}
void fem_cg2_update(const double* sc, const double* part_py, const double* p, const double* y, const double* diag,
                    int64_t nn, double* x, double* r, double* z, double* part_rz, int k, hipStream_t s)
{
    hipLaunchKernelGGL(k_cg2_update, dim3(CG2_BLOCKS), dim3(256), 0, s, sc, part_py, p, y, diag, nn, x, r, z, part_rz,
                       k);
}
void fem_cg2_update_xr(const double* sc, const double* part_py, const double* p, const double* y, int64_t nn,
                       double* x, double* r, int k, hipStream_t s)
{
    hipLaunchKernelGGL(k_cg2_update_xr, dim3(CG2_BLOCKS), dim3(256), 0, s, sc, part_py, p, y, nn, x, r, k);
}
void fem_cg2_dots(const double* r, const double* z, int64_t nn, double* part_rz, hipStream_t s)
{
    hipLaunchKernelGGL(k_cg2_dots, dim3(CG2_BLOCKS), dim3(256), 0, s, r, z, nn, part_rz);
}

void fem_store_wp(const double* wp9, int64_t nn, double* node, hipStream_t s)
{
    if (nn > 0) hipLaunchKernelGGL(k_fem_store_wp, dim3(blocks(nn, 256)), dim3(256), 0, s, wp9, nn, node);
}

void fem_nearest_wall(const ElemGeo* geo, int64_t ne, const double* edges, int32_t nw, double period, double* enrm,
                      hipStream_t s)
{
    if (ne > 0)
        hipLaunchKernelGGL(k_fem_nearest_wall, dim3(blocks(ne, 256)), dim3(256), 0, s, geo, ne, edges, nw, period,
                           enrm);
}

void fem_elem_matrices(const ElemGeo* geo, int64_t ne, double* ke, hipStream_t s)
{
    if (ne > 0) hipLaunchKernelGGL(k_fem_elem_matrices, dim3(blocks(ne, 256)), dim3(256), 0, s, geo, ne, ke);
}

void fem_assemble4(const FemOp& op, double* cval, hipStream_t s)
{
    if (op.nn > 0) hipLaunchKernelGGL(k_fem_assemble4, dim3(blocks(op.nn, 256)), dim3(256), 0, s, op, cval);
}

template <int NC>
void fem_apply(const FemOp& op, const double* x, double* y, hipStream_t s)
{
    if (op.nn <= 0) return;
    if (NC == 9 && op.cval)
        hipLaunchKernelGGL(k_fem_apply_csr9, dim3(blocks(op.nn * 9, 256)), dim3(256), 0, s, op, x, y, 0);
    else
        hipLaunchKernelGGL(k_fem_apply<NC>, dim3(blocks(op.nn, 256)), dim3(256), 0, s, op, x, y, 0);
}
template <int NC>
void fem_diag(const FemOp& op, double* d, hipStream_t s)
{
    if (op.nn <= 0) return;
    if (NC == 9 && op.cval)
        hipLaunchKernelGGL(k_fem_apply_csr9, dim3(blocks(op.nn * 9, 256)), dim3(256), 0, s, op, (const double*)d, d, 1);
    else
        hipLaunchKernelGGL(k_fem_apply<NC>, dim3(blocks(op.nn, 256)), dim3(256), 0, s, op, (const double*)d, d, 1);
}
template <int NC>
void fem_dot(const double* a, const double* b, const double* a2, const double* b2, int64_t nn, double* partial,
             double* out, hipStream_t s)
{
    hipLaunchKernelGGL(k_fem_dot<NC>, dim3(FEM_RED_BLOCKS), dim3(256), 0, s, a, b, a2, b2, nn, partial);
    static_assert(2 * NC <= 18, "at most 18 sums");
    hipLaunchKernelGGL(k_fem_dot_finish, dim3(1), dim3(256), 0, s, partial, FEM_RED_BLOCKS, 2 * NC,
                       a2 ? 2 * NC : NC, out);
}
template <int NC>
void fem_cg_init(const double* b, const double* Ax, const double* diag, const uint16_t* fixed, int64_t nn, double* r,
                 double* z, double* p, hipStream_t s)
{
    if (nn > 0)
        hipLaunchKernelGGL(k_cg_init<NC>, dim3(blocks(nn * NC, 256)), dim3(256), 0, s, b, Ax, diag, fixed, nn * NC, r,
                           z, p);
}
template <int NC>
void fem_cg_alpha(double* sc, hipStream_t s)
{
    hipLaunchKernelGGL(k_cg_alpha<NC>, dim3(1), dim3(64), 0, s, sc);
}
template <int NC>
void fem_cg_xr(const double* sc, const double* p, const double* Ap, const double* diag, const uint16_t* fixed,
               int64_t nn, double* x, double* r, double* z, hipStream_t s)
{
    if (nn > 0)
        hipLaunchKernelGGL(k_cg_xr<NC>, dim3(blocks(nn * NC, 256)), dim3(256), 0, s, sc, p, Ap, diag, fixed, nn, x, r,
                           z);
}
template <int NC>
void fem_cg_beta(double* sc, hipStream_t s)
{
    hipLaunchKernelGGL(k_cg_beta<NC>, dim3(1), dim3(64), 0, s, sc);
}
template <int NC>
void fem_cg_p(const double* sc, const double* z, int64_t nn, double* p, hipStream_t s)
{
    if (nn > 0) hipLaunchKernelGGL(k_cg_p<NC>, dim3(blocks(nn * NC, 256)), dim3(256), 0, s, sc, z, nn, p);
}

void fem_elliptic_inputs(const ElemGeo* geo, const int64_t* n2e_ptr, const int32_t* n2e, const double* stats,
                         int64_t nn, int64_t ne, const EllipticConst& c, const uint8_t* wkind, const double* wnrm,
                         const double* enrm, double* f, double* xfix, uint16_t* fixed, double* L2, uint32_t* err,
                         hipStream_t s)
{
    (void)err;
    if (nn > 0)
        hipLaunchKernelGGL(k_fem_elliptic_nodes, dim3(blocks(nn, 256)), dim3(256), 0, s, geo, n2e_ptr, n2e, stats, nn,
                           c, wkind, wnrm, f, xfix, fixed);
    if (ne > 0)
        hipLaunchKernelGGL(k_fem_elliptic_elems, dim3(blocks(ne, 256)), dim3(256), 0, s, geo, stats, ne, c, enrm, L2);
}
void fem_mass_rhs(const FemOp& op, const double* f, double* b, hipStream_t s)
{
    FemOp m = op;
    m.mass = 1.0;
    m.stiff = 0.0;
    m.cval = nullptr;
    fem_apply<9>(m, f, b, s);
}
void fem_set_fixed(const double* xfix, const uint16_t* fixed, int64_t nn, double* x, hipStream_t s)
{
    if (nn > 0) hipLaunchKernelGGL(k_fem_set_fixed, dim3(blocks(9 * nn, 256)), dim3(256), 0, s, xfix, fixed, nn, x);
}
void fem_pressure_rhs(const FemOp& op, const double* stats, const double* P, double rho, double dt, double cp,
                      double* b, uint32_t* err, hipStream_t s)
{
    (void)err;
    if (op.nn > 0)
        hipLaunchKernelGGL(k_fem_pressure_rhs, dim3(blocks(op.nn, 256)), dim3(256), 0, s, op, stats, P, rho, dt, cp,
                           b);
}
void fem_sub_mean(const double* sum, int64_t nn, double* v, hipStream_t s)
{
    if (nn > 0) hipLaunchKernelGGL(k_fem_sub_mean, dim3(blocks(nn, 256)), dim3(256), 0, s, sum, nn, v);
}
void fem_add(const double* a, int64_t n, double* y, hipStream_t s)
{
    if (n > 0) hipLaunchKernelGGL(k_fem_add, dim3(blocks(n, 256)), dim3(256), 0, s, a, n, y);
}
void fem_check_stats(const double* stats, int64_t nn, unsigned long long* count, hipStream_t s)
{
    if (nn > 0) hipLaunchKernelGGL(k_fem_check_stats, dim3(blocks(nn, 256)), dim3(256), 0, s, stats, nn, count);
}
void fem_elem_grad(const ElemGeo* geo, const double* q, int64_t ne, double* g, hipStream_t s)
{
    if (ne > 0) hipLaunchKernelGGL(k_fem_elem_grad, dim3(blocks(ne, 256)), dim3(256), 0, s, geo, q, ne, g);
}
void fem_pressure_update(const int64_t* n2e_ptr, const int32_t* n2e, const double* gP, const double* gdP,
                         const double* gp0, int64_t nn, double scale, double* node, double* stats, hipStream_t s)
{
    if (nn > 0)
        hipLaunchKernelGGL(k_fem_pressure_update, dim3(blocks(nn, 256)), dim3(256), 0, s, n2e_ptr, n2e, gP, gdP, gp0,
                           nn, scale, node, stats);
}
template <class R>
void fem_correct_particles(const SoaT<R>& st, const int64_t* nslots, int64_t n_ub, const double* gdP, double scale,
                           hipStream_t s)
{
    if (n_ub > 0)
        hipLaunchKernelGGL(k_fem_correct_particles<R>, dim3(blocks(n_ub, 256)), dim3(256), 0, s, st, nslots, n_ub, gdP,
                           scale);
}

#define FEM_NC(NC)                                                                                              \
    template void fem_apply<NC>(const FemOp&, const double*, double*, hipStream_t);                            \
    template void fem_diag<NC>(const FemOp&, double*, hipStream_t);                                            \
    template void fem_dot<NC>(const double*, const double*, const double*, const double*, int64_t, double*,   \
                              double*, hipStream_t);                                                           \
    template void fem_cg_init<NC>(const double*, const double*, const double*, const uint16_t*, int64_t,      \
                                  double*, double*, double*, hipStream_t);                                     \
    template void fem_cg_alpha<NC>(double*, hipStream_t);                                                      \
    template void fem_cg_xr<NC>(const double*, const double*, const double*, const double*, const uint16_t*,   \
                                int64_t, double*, double*, double*, hipStream_t);                              \
    template void fem_cg_beta<NC>(double*, hipStream_t);                                                       \
    template void fem_cg_p<NC>(const double*, const double*, int64_t, double*, hipStream_t);
FEM_NC(1)
FEM_NC(9)
#undef FEM_NC
template void fem_correct_particles<double>(const SoaT<double>&, const int64_t*, int64_t, const double*, double,
                                            hipStream_t);
template void fem_correct_particles<float>(const SoaT<float>&, const int64_t*, int64_t, const double*, double,
                                           hipStream_t);

}  // namespace pdfgpu
