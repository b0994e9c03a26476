// A measurement kernel: the streaming part of the CG step without its
// gathers.  Rows in chunks of 64 (one row per lane), `slots` FP64 values per
// row stored slot-major inside each chunk as in the SELL-64 matrix, one read
// each of the row's r, p and x, one write each of q, p and x; the persistent
// grid, the XCD-contiguous ranges and the one-chunk-ahead loads of the CG
// step.  What it reaches is the rate at which this device streams the step's
// bytes when nothing else limits it, the ceiling the CG step is compared with.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <string>

#include "device_common.h"
#include "host_common.h"
#include "kernels.h"
#include "ss_internal.h"

namespace ss {
namespace {

template <int S>
__global__ __launch_bounds__(kBS) __attribute__((amdgpu_waves_per_eu(1, 4))) void k_stream(
    int32_t nchunks, const double *__restrict__ val, const double *__restrict__ r, const double *__restrict__ p,
    const double *__restrict__ x, double *__restrict__ q, double *__restrict__ po, double *__restrict__ xo,
    double *__restrict__ sink)
{
    constexpr int W = kBS / 64;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int rb = dev::xcd_remap(blockIdx.x, gridDim.x);
    const int cpb = (nchunks + (int)gridDim.x - 1) / (int)gridDim.x;
    const int cend = min(rb * cpb + cpb, nchunks);
    double vv[S], rv, pv, xv;
    auto load = [&](int c) {
        const int cc = min(c, nchunks - 1);
        const size_t base = (size_t)cc * 64 * S;
#pragma unroll
        for (int u = 0; u < S; ++u) vv[u] = val[base + (size_t)u * 64 + lane];
        const size_t i = (size_t)cc * 64 + lane;
        rv = r[i];
        pv = p[i];
        xv = x[i];
    };
    int c = rb * cpb + w;
    load(c);
    double acc = 0.0;
    for (; c < cend; c += W) {
        double s = 0.0;
#pragma unroll
        for (int u = 0; u < S; ++u) s = s + vv[u] * pv;
        const size_t i = (size_t)c * 64 + lane;
        q[i] = s;
        po[i] = rv + 0.5 * pv;
        xo[i] = xv + 0.25 * pv;
        acc = acc + s;
        load(c + W);
    }
    // keeps the products live; the host never sets the values that would store
    if (acc == 1.0e300) sink[0] = acc;
}

template <int S>
void launch(hipStream_t s, int grid, int32_t nchunks, const double *val, const double *r, const double *p,
            const double *x, double *q, double *po, double *xo, double *sink)
{
    hipLaunchKernelGGL((k_stream<S>), dim3(grid), dim3(kBS), 0, s, nchunks, val, r, p, x, q, po, xo, sink);
}

}  // namespace
}  // namespace ss

using namespace ss;

extern "C" int ss_stream_rate(int64_t rows, int32_t slots, int32_t reps, void *hip_stream, double *ms_per_launch,
                              double *bytes_per_launch)
{
    if (rows < 64 || rows > (int64_t)INT32_MAX / 64 * 64 || reps < 1 || !ms_per_launch)
        return fail(SS_EINVAL, "need 64 <= rows < 2^31, reps >= 1 and an output");
    if (slots != 5 && slots != 7 && slots != 9 && slots != 27)
        return fail(SS_EINVAL, "slots must be 5, 7, 9 or 27");
    const int32_t nchunks = (int32_t)(rows / 64);
    const size_t n = (size_t)nchunks * 64;
    hipStream_t s = (hipStream_t)hip_stream;
    double *buf = nullptr;
    const size_t total = n * ((size_t)slots + 6) + 1;
    if (hipMalloc((void **)&buf, sizeof(double) * total) != hipSuccess) {
        (void)hipGetLastError();
        return fail(SS_ENOMEM, "device allocation failed");
    }
    double *val = buf, *r = val + n * slots, *p = r + n, *x = p + n, *q = x + n, *po = q + n, *xo = po + n,
           *sink = xo + n;
    hipEvent_t ev[2] = {nullptr, nullptr};
    auto done = [&](int code, const std::string &msg) {
        for (auto &e : ev)
            if (e) (void)hipEventDestroy(e);
        (void)hipFree(buf);
        return code == SS_OK ? SS_OK : fail(code, msg);
    };
    if (hipMemsetAsync(buf, 0, sizeof(double) * total, s) != hipSuccess) return done(SS_EDEVICE, "memset failed");
    const int grid = xcd_grid(std::min<int32_t>(1024, std::max<int32_t>(1, (nchunks + 3) / 4)));
    auto run = [&]() {
        switch (slots) {
        case 5: launch<5>(s, grid, nchunks, val, r, p, x, q, po, xo, sink); break;
        case 7: launch<7>(s, grid, nchunks, val, r, p, x, q, po, xo, sink); break;
        case 9: launch<9>(s, grid, nchunks, val, r, p, x, q, po, xo, sink); break;
        default: launch<27>(s, grid, nchunks, val, r, p, x, q, po, xo, sink); break;
        }
    };
    for (auto &e : ev)
        if (hipEventCreate(&e) != hipSuccess) return done(SS_EDEVICE, "event creation failed");
    for (int i = 0; i < 3; ++i) run();
    (void)hipEventRecord(ev[0], s);
    for (int32_t i = 0; i < reps; ++i) run();
    (void)hipEventRecord(ev[1], s);
    hipError_t err = hipGetLastError();
    if (err == hipSuccess) err = hipEventSynchronize(ev[1]);
    float t = 0.0f;
    if (err == hipSuccess) err = hipEventElapsedTime(&t, ev[0], ev[1]);
    if (err != hipSuccess) return done(SS_EDEVICE, std::string("stream probe: ") + hipGetErrorString(err));
    *ms_per_launch = t / reps;
    if (bytes_per_launch) *bytes_per_launch = (double)n * (8.0 * slots + 48.0);
    return done(SS_OK, "");
}
