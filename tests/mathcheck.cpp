// Host build of the device random-number and math helpers of libpdfgpu, for CPU tests.
#include "device.h"

using namespace pdfgpu;

extern "C" {
void mc_philox(const uint32_t* ctr, const uint32_t* key, uint32_t* out)
{
    const Words4 w = philox4x32_10(ctr[0], ctr[1], ctr[2], ctr[3], key[0], key[1]);
    out[0] = w.w0; out[1] = w.w1; out[2] = w.w2; out[3] = w.w3;
}
void mc_sincos_2pi(const double* u, long n, double* s, double* c)
{
    for (long i = 0; i < n; ++i) sincos_2pi(u[i], s[i], c[i]);
}
void mc_log_unit(const double* u, long n, double* o)
{
    for (long i = 0; i < n; ++i) o[i] = log_unit(u[i]);
}
void mc_box_muller(const uint32_t* a, const uint32_t* b, long n, double* z)
{
    for (long i = 0; i < n; ++i) box_muller(a[i], b[i], z[2 * i], z[2 * i + 1]);
}
}
