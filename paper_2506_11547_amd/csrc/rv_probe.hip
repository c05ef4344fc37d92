// Test hooks for the device steps of the rule, one kernel per step, so the
// test suite can compare each step with the CPU oracle bit for bit and check
// the hardware's rounding of the primitive operations.  Not used by a solve.
#include "rv_device.h"
#include "rv_table.h"

#pragma GCC visibility push(default)
#include "rotvote_probe.h"
#pragma GCC visibility pop

#define RVP_API extern "C" __attribute__((visibility("default")))

namespace {

__global__ void k_recip(const float* in, float* out, int64_t n, int fast)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n)
        out[i] = fast ? rv::recip_1_2(in[i]) : 1.0f / in[i];
}

__global__ void k_div_sqrt(const float* a, const float* b, float* q, float* r, int64_t n)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) {
        q[i] = a[i] / b[i];
        r[i] = __builtin_sqrtf(a[i]);
    }
}

__global__ void k_basis(const float* x, const float* y, int64_t n, float* u, float* v, int* ok)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n)
        return;
    float a[3], b[3];
    const bool oka = rv::load_unit(x, n, i, a);
    const bool okb = rv::load_unit(y, n, i, b);
    rv::Quat qu, qv;
    rv::circle_basis(a, b, qu, qv);
    u[4 * i + 0] = qu.w; u[4 * i + 1] = qu.x; u[4 * i + 2] = qu.y; u[4 * i + 3] = qu.z;
    v[4 * i + 0] = qv.w; v[4 * i + 1] = qv.x; v[4 * i + 2] = qv.y; v[4 * i + 3] = qv.z;
    ok[i] = (oka && okb) ? 1 : 0;
}

template <bool kFast>
__global__ void k_cells(const float* q, int64_t n, int G, int* out)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n)
        out[i] = rv::cell_index<kFast>(q[4 * i], q[4 * i + 1], q[4 * i + 2], q[4 * i + 3],
                                       (float)G * 0.5f, (float)G - 0.5f, G);
}

__global__ void k_decode(const int* idx, int64_t n, int G, float* q)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) {
        const rv::Quat d = rv::decode_cell(idx[i], G);
        q[4 * i] = d.w; q[4 * i + 1] = d.x; q[4 * i + 2] = d.y; q[4 * i + 3] = d.z;
    }
}

__global__ void k_residual(const float* x, const float* y, int64_t n, const float* q, float* out)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n)
        return;
    float a[3], b[3];
    const bool oka = rv::load_unit(x, n, i, a);
    const bool okb = rv::load_unit(y, n, i, b);
    float D[3], P[3];
    for (int m = 0; m < 3; ++m) {
        D[m] = a[m] - b[m];
        P[m] = a[m] + b[m];
    }
    const rv::Quat qq{q[0], q[1], q[2], q[3]};
    out[i] = (oka && okb) ? rv::residual2(D, P, qq) : -1.0f;
}

__global__ void k_table(int J, float2* out)
{
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j < J)
        out[j] = rv::table_entry(j, J);
}

int blocks(int64_t n) { return (int)((n + 255) / 256); }

int finish()
{
    hipError_t e = hipGetLastError();
    if (e == hipSuccess)
        e = hipDeviceSynchronize();
    return e == hipSuccess ? 0 : (int)e;
}

}  // namespace

// All pointers are device memory; every call is synchronous on the null stream.
RVP_API int rvp_recip(const float* in, float* out, int64_t n, int fast)
{
    if (n <= 0) return 0;
    hipLaunchKernelGGL(k_recip, dim3(blocks(n)), dim3(256), 0, 0, in, out, n, fast);
    return finish();
}

RVP_API int rvp_div_sqrt(const float* a, const float* b, float* q, float* r, int64_t n)
{
    if (n <= 0) return 0;
    hipLaunchKernelGGL(k_div_sqrt, dim3(blocks(n)), dim3(256), 0, 0, a, b, q, r, n);
    return finish();
}

RVP_API int rvp_basis(const float* x, const float* y, int64_t n, float* u, float* v, int* ok)
{
    if (n <= 0) return 0;
    hipLaunchKernelGGL(k_basis, dim3(blocks(n)), dim3(256), 0, 0, x, y, n, u, v, ok);
    return finish();
}

RVP_API int rvp_cells(const float* q, int64_t n, int G, int* out, int fast)
{
    if (n <= 0) return 0;
    if (fast)
        hipLaunchKernelGGL(k_cells<true>, dim3(blocks(n)), dim3(256), 0, 0, q, n, G, out);
    else
        hipLaunchKernelGGL(k_cells<false>, dim3(blocks(n)), dim3(256), 0, 0, q, n, G, out);
    return finish();
}

RVP_API int rvp_decode(const int* idx, int64_t n, int G, float* q)
{
    if (n <= 0) return 0;
    hipLaunchKernelGGL(k_decode, dim3(blocks(n)), dim3(256), 0, 0, idx, n, G, q);
    return finish();
}

RVP_API int rvp_residual(const float* x, const float* y, int64_t n, const float* q, float* out)
{
    if (n <= 0) return 0;
    hipLaunchKernelGGL(k_residual, dim3(blocks(n)), dim3(256), 0, 0, x, y, n, q, out);
    return finish();
}

RVP_API int rvp_table(int J, float* out)
{
    if (J <= 0) return 0;
    hipLaunchKernelGGL(k_table, dim3(blocks(J)), dim3(256), 0, 0, J, reinterpret_cast<float2*>(out));
    return finish();
}
