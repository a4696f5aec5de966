// Entry point of libpdfgpu that allocates nothing: the time step of Eq. (26) computed into
// caller-owned device memory, with its partial results in a fixed device array of this
// library instead of the ensemble's scratch.  For callers that cannot allocate device
// memory (HIP graph capture, tight serving loops).
#include <hip/hip_runtime.h>

#include <cmath>
#include <mutex>
#include <string>

#include "device.h"
#include "pdf_impl.h"

namespace pdfgpu {
void set_error(const std::string& msg);
}
using namespace pdfgpu;

namespace {

constexpr int NA_THREADS = 256;
constexpr int64_t NA_MAX_BLOCKS = 65536;    // partial (min, max) pairs: nodes up to 2^24
constexpr int NA_MAX_DEVICES = 64;

// Per-workgroup partial results of the reduction (1 MiB per device, held until the
// process ends).  In host code the name is only a handle for the symbol lookup: kernels
// receive the device address that hipGetSymbolAddress returned for the current device.
static __device__ __align__(256) double scratch[2 * NA_MAX_BLOCKS];

std::mutex g_mutex;
double* g_scratch[NA_MAX_DEVICES] = {};

// partial min of l and max of z over the nodes of one workgroup (Eq. 26 ingredients)
__global__ void __launch_bounds__(NA_THREADS) k_cfl_partials(const ElemGeo* __restrict__ geo,
                                                            const int64_t* __restrict__ n2e_ptr,
                                                            const int32_t* __restrict__ n2e,
                                                            const double* __restrict__ stats, int64_t n0, int64_t nn,
                                                            double* __restrict__ part)
{
    __shared__ double sl[NA_THREADS / 64], sz[NA_THREADS / 64];
    const int64_t n = n0 + (int64_t)blockIdx.x * NA_THREADS + threadIdx.x;
    double l = __builtin_inf(), z = 0.0;
    if (n < n0 + nn) cfl_node(geo, n2e_ptr, n2e, stats, n, l, z);
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        l = fmin(l, __shfl_xor(l, o));
        z = fmax(z, __shfl_xor(z, o));
    }
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) {
        sl[w] = l;
        sz[w] = z;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int k = 1; k < NA_THREADS / 64; ++k) {
            l = fmin(l, sl[k]);
            z = fmax(z, sz[k]);
        }
        part[2 * blockIdx.x] = l;
        part[2 * blockIdx.x + 1] = z;
    }
}

// dt = cfl * min l / max z (0 when no node has a positive norm), from nb partial pairs
__global__ void __launch_bounds__(NA_THREADS) k_cfl_finish(const double* __restrict__ part, int64_t nb, double cfl,
                                                          double* __restrict__ dt_out)
{
    __shared__ double sl[NA_THREADS / 64], sz[NA_THREADS / 64];
    double l = __builtin_inf(), z = 0.0;
    for (int64_t b = threadIdx.x; b < nb; b += NA_THREADS) {
        l = fmin(l, part[2 * b]);
        z = fmax(z, part[2 * b + 1]);
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        l = fmin(l, __shfl_xor(l, o));
        z = fmax(z, __shfl_xor(z, o));
    }
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) {
        sl[w] = l;
        sz[w] = z;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int k = 1; k < NA_THREADS / 64; ++k) {
            l = fmin(l, sl[k]);
            z = fmax(z, sz[k]);
        }
        *dt_out = z > 0.0 ? cfl * l / z : 0.0;
    }
}

}  // namespace

namespace pdfgpu {

// Device address of the scratch array on the current device, looked up once per device
// (at ensemble set-up, with that device current).  Null on failure, with the error set.
double* noalloc_scratch(int device)
{
    if (device < 0 || device >= NA_MAX_DEVICES) {
        set_error("no-allocation scratch: device index out of range");
        return nullptr;
    }
    std::lock_guard<std::mutex> lock(g_mutex);
    if (!g_scratch[device]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            (void)hipGetLastError();
            set_error(std::string("hipGetSymbolAddress of the no-allocation scratch: ") + hipGetErrorString(e));
            return nullptr;
        }
        g_scratch[device] = static_cast<double*>(p);
    }
    return g_scratch[device];
}

}  // namespace pdfgpu

extern "C" pdf_status pdf_cfl_dt_noalloc(pdf_ens E, int32_t problem, double cfl, double* dt_out, void* hip_stream)
{
    if (!E || !dt_out || problem < 0 || problem >= E->n_problems || !(cfl > 0.0) || !std::isfinite(cfl)) {
        set_error("pdf_cfl_dt_noalloc: invalid argument");
        return PDF_E_INVAL;
    }
    const ProbParams& P = E->h_prm[problem];
    const int64_t nb = (P.nn + NA_THREADS - 1) / NA_THREADS;
    if (nb > NA_MAX_BLOCKS) {
        set_error("pdf_cfl_dt_noalloc: the problem has more than 2^24 nodes, the limit of the fixed scratch");
        return PDF_E_CAPACITY;
    }
    const int dev = E->grid->device;
    double* part = (dev >= 0 && dev < NA_MAX_DEVICES) ? g_scratch[dev] : nullptr;
    if (!part) {
        set_error("pdf_cfl_dt_noalloc: the no-allocation scratch of this device was not set up");
        return PDF_E_STATE;
    }
    hipError_t e = hipSetDevice(dev);
    if (e != hipSuccess) {
        set_error(std::string("pdf_cfl_dt_noalloc: ") + hipGetErrorString(e));
        return PDF_E_HIP;
    }
    hipStream_t s = reinterpret_cast<hipStream_t>(hip_stream);
    const DevGrid& g = E->dg;
    if (nb > 0)
        hipLaunchKernelGGL(k_cfl_partials, dim3((unsigned)nb), dim3(NA_THREADS), 0, s, g.geo, g.n2e_ptr, g.n2e,
                           E->stats, P.noff, P.nn, part);
    hipLaunchKernelGGL(k_cfl_finish, dim3(1), dim3(NA_THREADS), 0, s, part, nb, cfl, dt_out);
    e = hipGetLastError();
    if (e != hipSuccess) {
        set_error(std::string("pdf_cfl_dt_noalloc: ") + hipGetErrorString(e));
        return PDF_E_HIP;
    }
    return PDF_OK;
}
