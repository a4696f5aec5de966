// Smoothed-aggregation multigrid preconditioner of the pressure solve; see amg.h.
#include "amg.h"

#include <algorithm>
#include <cmath>

#include "device.h"

namespace pdfgpu {

namespace {

// ---- host setup ----

HostCsr transpose(const HostCsr& A)
{
    HostCsr T;
    T.n = A.m;
    T.m = A.n;
    T.rp.assign(T.n + 1, 0);
    for (int32_t c : A.col) ++T.rp[c + 1];
    for (int64_t i = 0; i < T.n; ++i) T.rp[i + 1] += T.rp[i];
    T.col.resize(A.col.size());
    T.val.resize(A.val.size());
    std::vector<int32_t> fill(T.rp.begin(), T.rp.end() - 1);
    for (int64_t i = 0; i < A.n; ++i)       // rows in order: the columns of T come out ascending
        for (int32_t k = A.rp[i]; k < A.rp[i + 1]; ++k) {
            const int32_t q = fill[A.col[k]]++;
            T.col[q] = (int32_t)i;
            T.val[q] = A.val[k];
        }
    return T;
}

// C = A B, rows of C with ascending columns; sums in the order of A's row, then B's
HostCsr multiply(const HostCsr& A, const HostCsr& B)
{
    HostCsr C;
    C.n = A.n;
    C.m = B.m;
    C.rp.assign(1, 0);
    std::vector<double> acc(B.m, 0.0);
    std::vector<int64_t> mark(B.m, -1);
    std::vector<int32_t> cols;
    for (int64_t i = 0; i < A.n; ++i) {
        cols.clear();
        for (int32_t k = A.rp[i]; k < A.rp[i + 1]; ++k) {
            const int32_t j = A.col[k];
            const double a = A.val[k];
            for (int32_t q = B.rp[j]; q < B.rp[j + 1]; ++q) {
                const int32_t c = B.col[q];
                if (mark[c] != i) {
                    mark[c] = i;
                    acc[c] = 0.0;
                    cols.push_back(c);
                }
                acc[c] += a * B.val[q];
            }
        }
        std::sort(cols.begin(), cols.end());
        for (int32_t c : cols) {
            C.col.push_back(c);
            C.val.push_back(acc[c]);
        }
        C.rp.push_back((int32_t)C.col.size());
    }
    return C;
}

// dense inverse of a symmetric positive definite matrix by Cholesky (false: not definite)
bool spd_inverse(std::vector<double>& a, int64_t n, std::vector<double>& inv)
{
    for (int64_t j = 0; j < n; ++j) {
        double d = a[j * n + j];
        for (int64_t k = 0; k < j; ++k) d -= a[j * n + k] * a[j * n + k];
        if (!(d > 0.0)) return false;
        const double l = std::sqrt(d);
        a[j * n + j] = l;
        for (int64_t i = j + 1; i < n; ++i) {
            double v = a[i * n + j];
            for (int64_t k = 0; k < j; ++k) v -= a[i * n + k] * a[j * n + k];
            a[i * n + j] = v / l;
        }
    }
    inv.assign(n * n, 0.0);
    std::vector<double> y(n);
    for (int64_t c = 0; c < n; ++c) {       // solve L L^T x = e_c
        for (int64_t i = 0; i < n; ++i) {
            double v = i == c ? 1.0 : 0.0;
            for (int64_t k = 0; k < i; ++k) v -= a[i * n + k] * y[k];
            y[i] = v / a[i * n + i];
        }
        for (int64_t i = n - 1; i >= 0; --i) {
            double v = y[i];
            for (int64_t k = i + 1; k < n; ++k) v -= a[k * n + i] * inv[k * n + c];
            inv[i * n + c] = v / a[i * n + i];
        }
    }
    return true;
}

}  // namespace

bool amg_build(const HostCsr& A0, AmgHost& out)
{
    const double theta = 0.08;
    out = AmgHost{};
    HostCsr A = A0;
    while (A.n > AMG_COARSE) {
        if ((int)out.lv.size() >= AMG_MAX_LEVELS) return false;
        const int64_t n = A.n;
        std::vector<double> d(n, 0.0);
        for (int64_t i = 0; i < n; ++i)
            for (int32_t k = A.rp[i]; k < A.rp[i + 1]; ++k)
                if (A.col[k] == i) d[i] = A.val[k];
        for (int64_t i = 0; i < n; ++i)
            if (!(d[i] > 0.0)) return false;
        auto strong = [&](int64_t i, int32_t k) {
            const int32_t j = A.col[k];
            return j != i && std::fabs(A.val[k]) >= theta * std::sqrt(d[i] * d[j]);
        };
        // greedy aggregation in node order
        std::vector<int32_t> agg(n, -1);
        int32_t na = 0;
        for (int64_t i = 0; i < n; ++i) {
            if (agg[i] >= 0) continue;
            bool free = true;
            for (int32_t k = A.rp[i]; k < A.rp[i + 1] && free; ++k)
                if (strong(i, k) && agg[A.col[k]] >= 0) free = false;
            if (!free) continue;
            agg[i] = na;
            for (int32_t k = A.rp[i]; k < A.rp[i + 1]; ++k)
                if (strong(i, k)) agg[A.col[k]] = na;
            ++na;
        }
        const std::vector<int32_t> first = agg;
        for (int64_t i = 0; i < n; ++i) {
            if (agg[i] >= 0) continue;
            double best = -1.0;
            for (int32_t k = A.rp[i]; k < A.rp[i + 1]; ++k)
                if (strong(i, k) && first[A.col[k]] >= 0 && std::fabs(A.val[k]) > best) {
                    best = std::fabs(A.val[k]);
                    agg[i] = first[A.col[k]];
                }
        }
        for (int64_t i = 0; i < n; ++i) {
            if (agg[i] >= 0) continue;
            agg[i] = na;
            for (int32_t k = A.rp[i]; k < A.rp[i + 1]; ++k)
                if (strong(i, k) && agg[A.col[k]] < 0) agg[A.col[k]] = na;
            ++na;
        }
        if (na == 0 || na > (n * 9) / 10) return false;
        // Gershgorin bound of D^-1 A and the damping of both the prolongator and smoother
        double lam = 0.0;
        for (int64_t i = 0; i < n; ++i) {
            double s = 0.0;
            for (int32_t k = A.rp[i]; k < A.rp[i + 1]; ++k) s += std::fabs(A.val[k]);
            lam = std::max(lam, s / d[i]);
        }
        const double om = 4.0 / (3.0 * lam);
        // P = T - om D^-1 A T, T the aggregates' constants
        HostCsr P;
        P.n = n;
        P.m = na;
        P.rp.assign(1, 0);
        std::vector<double> acc(na, 0.0);
        std::vector<int64_t> mark(na, -1);
        std::vector<int32_t> cols;
        for (int64_t i = 0; i < n; ++i) {
            cols.clear();
            auto add = [&](int32_t c, double v) {
                if (mark[c] != i) {
                    mark[c] = i;
                    acc[c] = 0.0;
                    cols.push_back(c);
                }
                acc[c] += v;
            };
            add(agg[i], 1.0);
            for (int32_t k = A.rp[i]; k < A.rp[i + 1]; ++k) add(agg[A.col[k]], -om / d[i] * A.val[k]);
            std::sort(cols.begin(), cols.end());
            for (int32_t c : cols)
                if (acc[c] != 0.0) {
                    P.col.push_back(c);
                    P.val.push_back(acc[c]);
                }
            P.rp.push_back((int32_t)P.col.size());
        }
        AmgHostLevel L;
        L.R = transpose(P);
        HostCsr Ac = multiply(L.R, multiply(A, P));
        L.dinv.resize(n);
        for (int64_t i = 0; i < n; ++i) L.dinv[i] = om / d[i];
        L.P = std::move(P);
        L.A = std::move(A);
        out.lv.push_back(std::move(L));
        A = std::move(Ac);
    }
    // coarsest level: (A + alpha 1 1^T)^-1, alpha the mean diagonal over n
    const int64_t nc = A.n;
    if (nc <= 0) return false;
    std::vector<double> dense(nc * nc, 0.0);
    double tr = 0.0;
    for (int64_t i = 0; i < nc; ++i)
        for (int32_t k = A.rp[i]; k < A.rp[i + 1]; ++k) {
            dense[i * nc + A.col[k]] += A.val[k];
            if (A.col[k] == i) tr += A.val[k];
        }
    const double alpha = tr / ((double)nc * (double)nc);
    for (int64_t q = 0; q < nc * nc; ++q) dense[q] += alpha;
    // the product P^T A P is symmetric up to rounding: use its symmetric part
    for (int64_t i = 0; i < nc; ++i)
        for (int64_t j = 0; j < i; ++j) {
            const double v = 0.5 * (dense[i * nc + j] + dense[j * nc + i]);
            dense[i * nc + j] = dense[j * nc + i] = v;
        }
    if (!spd_inverse(dense, nc, out.cinv)) return false;
    out.nc = nc;
    return true;
}

// ---- device ----

namespace {

inline unsigned nblk(int64_t n) { return (unsigned)((n + 255) / 256); }

// Row i of a CSR product, sum_k val_k g(col_k): one thread per row for the sparse fine
// matrices (WAVE = false), one wavefront per row with the lanes striding over the row
// and a fixed-order wavefront sum for the denser coarse (Galerkin) matrices and the
// restriction.  Returns the sum in every lane of the row's wavefront (or the thread);
// valid is false for a row beyond n.
template <bool WAVE>
struct RowMap {
    int64_t i;
    bool valid;
    __device__ RowMap(int64_t n)
    {
        i = WAVE ? (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6) : (int64_t)blockIdx.x * 256 + threadIdx.x;
        valid = i < n;
    }
    template <class G>
    __device__ double dot(const int32_t* __restrict__ rp, const int32_t* __restrict__ col,
                          const double* __restrict__ val, G g) const
    {
        double s = 0.0;
        if (WAVE) {
            for (int32_t k = rp[i] + (int32_t)(threadIdx.x & 63); k < rp[i + 1]; k += 64) s += val[k] * g(col[k]);
            return wave_sum_double(s);
        }
        for (int32_t k = rp[i]; k < rp[i + 1]; ++k) s += val[k] * g(col[k]);
        return s;
    }
    __device__ bool writer() const { return valid && (!WAVE || (threadIdx.x & 63) == 0); }
};

template <bool WAVE>
inline unsigned rows_grid(int64_t n)
{
    return WAVE ? (unsigned)((n + 3) / 4) : nblk(n);
}

// x = dinv b (one Jacobi sweep from zero), r = b - A x
template <bool WAVE>
__global__ void __launch_bounds__(256) k_amg_pre(const int32_t* __restrict__ rp, const int32_t* __restrict__ col,
                                                 const double* __restrict__ val, const double* __restrict__ dinv,
                                                 const double* __restrict__ b, int64_t n, double* __restrict__ x,
                                                 double* __restrict__ r)
{
    const RowMap<WAVE> m(n);
    if (!m.valid) return;
    const double ax = m.dot(rp, col, val, [&](int32_t j) { return dinv[j] * b[j]; });
    if (m.writer()) {
        x[m.i] = dinv[m.i] * b[m.i];
        r[m.i] = b[m.i] - ax;
    }
}

// y = A x
template <bool WAVE>
__global__ void __launch_bounds__(256) k_amg_spmv(const int32_t* __restrict__ rp, const int32_t* __restrict__ col,
                                                  const double* __restrict__ val, const double* __restrict__ x,
                                                  int64_t n, double* __restrict__ y)
{
    const RowMap<WAVE> m(n);
    if (!m.valid) return;
    const double s = m.dot(rp, col, val, [&](int32_t j) { return x[j]; });
    if (m.writer()) y[m.i] = s;
}

// t = x + P xc
template <bool WAVE>
__global__ void __launch_bounds__(256) k_amg_prolong(const int32_t* __restrict__ rp, const int32_t* __restrict__ col,
                                                     const double* __restrict__ val, const double* __restrict__ xc,
                                                     const double* __restrict__ x, int64_t n, double* __restrict__ t)
{
    const RowMap<WAVE> m(n);
    if (!m.valid) return;
    const double s = m.dot(rp, col, val, [&](int32_t j) { return xc[j]; });
    if (m.writer()) t[m.i] = x[m.i] + s;
}

// x = t + dinv (b - A t)
template <bool WAVE>
__global__ void __launch_bounds__(256) k_amg_post(const int32_t* __restrict__ rp, const int32_t* __restrict__ col,
                                                  const double* __restrict__ val, const double* __restrict__ dinv,
                                                  const double* __restrict__ b, const double* __restrict__ t, int64_t n,
                                                  double* __restrict__ x)
{
    const RowMap<WAVE> m(n);
    if (!m.valid) return;
    const double at = m.dot(rp, col, val, [&](int32_t j) { return t[j]; });
    if (m.writer()) x[m.i] = t[m.i] + dinv[m.i] * (b[m.i] - at);
}

// x = C b for the dense coarsest inverse: a wavefront per row, a fixed-order sum
__global__ void __launch_bounds__(256) k_amg_dense(const double* __restrict__ c, const double* __restrict__ b,
                                                   int64_t n, double* __restrict__ x)
{
    const int64_t row = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (row >= n) return;
    double s = 0.0;
    for (int64_t j = lane; j < n; j += 64) s += c[row * n + j] * b[j];
    s = wave_sum_double(s);
    if (lane == 0) x[row] = s;
}

template <class T>
hipError_t put(T*& d, const std::vector<T>& h, hipStream_t s)
{
    const size_t bytes = sizeof(T) * std::max<size_t>(h.size(), 1);
    hipError_t e = hipMalloc((void**)&d, bytes);
    if (e != hipSuccess) {
        d = nullptr;
        return e;
    }
    if (!h.empty()) e = hipMemcpyAsync(d, h.data(), sizeof(T) * h.size(), hipMemcpyHostToDevice, s);
    return e;
}

hipError_t put_csr(DevCsr& d, const HostCsr& h, hipStream_t s)
{
    d.n = h.n;
    d.nnz = (int64_t)h.col.size();
    hipError_t e = put(d.rp, h.rp, s);
    if (e == hipSuccess) e = put(d.col, h.col, s);
    if (e == hipSuccess) e = put(d.val, h.val, s);
    return e;
}

template <class T>
void drop(T*& p)
{
    if (p) (void)hipFree((void*)p);
    p = nullptr;
}

void drop_csr(DevCsr& c)
{
    drop(c.rp);
    drop(c.col);
    drop(c.val);
}

hipError_t work(double*& p, int64_t n)
{
    hipError_t e = hipMalloc((void**)&p, sizeof(double) * (size_t)std::max<int64_t>(n, 1));
    if (e != hipSuccess) p = nullptr;
    return e;
}

// a wavefront per row pays off above this many nonzeros per row on average
inline bool wide(const DevCsr& c) { return c.n > 0 && c.nnz > 12 * c.n; }

void vcycle(AmgDev& d, size_t l, const double* b, double* x, hipStream_t s)
{
    if (l == d.lv.size()) {
        hipLaunchKernelGGL(k_amg_dense, dim3((unsigned)((d.nc + 3) / 4)), dim3(256), 0, s, d.cinv, b, d.nc, x);
        return;
    }
    AmgDevLevel& L = d.lv[l];
    const int64_t n = L.A.n;
    const bool wa = wide(L.A);
    if (wa)
        hipLaunchKernelGGL(k_amg_pre<true>, dim3(rows_grid<true>(n)), dim3(256), 0, s, L.A.rp, L.A.col, L.A.val,
                           L.dinv, b, n, L.x, L.r);
    else
        hipLaunchKernelGGL(k_amg_pre<false>, dim3(rows_grid<false>(n)), dim3(256), 0, s, L.A.rp, L.A.col, L.A.val,
                           L.dinv, b, n, L.x, L.r);
    const bool last = l + 1 == d.lv.size();
    double* bc = last ? d.cb : d.lv[l + 1].b;
    double* xc = last ? d.cx : d.lv[l + 1].x;
    if (wide(L.R))
        hipLaunchKernelGGL(k_amg_spmv<true>, dim3(rows_grid<true>(L.R.n)), dim3(256), 0, s, L.R.rp, L.R.col, L.R.val,
                           L.r, L.R.n, bc);
    else
        hipLaunchKernelGGL(k_amg_spmv<false>, dim3(rows_grid<false>(L.R.n)), dim3(256), 0, s, L.R.rp, L.R.col,
                           L.R.val, L.r, L.R.n, bc);
    vcycle(d, l + 1, bc, xc, s);
    if (wide(L.P))
        hipLaunchKernelGGL(k_amg_prolong<true>, dim3(rows_grid<true>(n)), dim3(256), 0, s, L.P.rp, L.P.col, L.P.val,
                           xc, L.x, n, L.t);
    else
        hipLaunchKernelGGL(k_amg_prolong<false>, dim3(rows_grid<false>(n)), dim3(256), 0, s, L.P.rp, L.P.col,
                           L.P.val, xc, L.x, n, L.t);
    if (wa)
        hipLaunchKernelGGL(k_amg_post<true>, dim3(rows_grid<true>(n)), dim3(256), 0, s, L.A.rp, L.A.col, L.A.val,
                           L.dinv, b, L.t, n, x);
    else
        hipLaunchKernelGGL(k_amg_post<false>, dim3(rows_grid<false>(n)), dim3(256), 0, s, L.A.rp, L.A.col, L.A.val,
                           L.dinv, b, L.t, n, x);
}

}  // namespace

hipError_t amg_upload(const AmgHost& h, AmgDev& d, hipStream_t s)
{
    amg_free(d);
    hipError_t e = hipSuccess;
    d.lv.resize(h.lv.size());
    for (size_t l = 0; l < h.lv.size() && e == hipSuccess; ++l) {
        const AmgHostLevel& H = h.lv[l];
        AmgDevLevel& L = d.lv[l];
        e = put_csr(L.A, H.A, s);
        if (e == hipSuccess) e = put_csr(L.P, H.P, s);
        if (e == hipSuccess) e = put_csr(L.R, H.R, s);
        if (e == hipSuccess) e = put(L.dinv, H.dinv, s);
        if (e == hipSuccess) e = work(L.b, H.A.n);
        if (e == hipSuccess) e = work(L.x, H.A.n);
        if (e == hipSuccess) e = work(L.r, H.A.n);
        if (e == hipSuccess) e = work(L.t, H.A.n);
    }
    d.nc = h.nc;
    if (e == hipSuccess) e = put(d.cinv, h.cinv, s);
    if (e == hipSuccess) e = work(d.cb, h.nc);
    if (e == hipSuccess) e = work(d.cx, h.nc);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) amg_free(d);
    return e;
}

void amg_free(AmgDev& d)
{
    for (AmgDevLevel& L : d.lv) {
        drop_csr(L.A);
        drop_csr(L.P);
        drop_csr(L.R);
        drop(L.dinv);
        drop(L.b);
        drop(L.x);
        drop(L.r);
        drop(L.t);
    }
    d.lv.clear();
    drop(d.cinv);
    drop(d.cb);
    drop(d.cx);
    d.nc = 0;
}

void amg_vcycle(AmgDev& d, const double* r, double* z, hipStream_t s) { vcycle(d, 0, r, z, s); }

}  // namespace pdfgpu
