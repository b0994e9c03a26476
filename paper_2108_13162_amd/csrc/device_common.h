// Device helpers shared by the kernel sources: workgroup-to-XCD mapping,
// fixed-order wavefront / workgroup sums and agent-scope atomic flags.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace ss {
namespace dev {

constexpr int kWG = 256;    // workgroup size of every kernel
constexpr int kNumXcd = 8;  // MI355X: workgroups are dealt round-robin to 8 XCDs

// Workgroup b of a grid of `grid` (a multiple of 8) runs on XCD b % 8; this
// index gives each XCD a contiguous range of work.
__device__ __forceinline__ int xcd_remap(int b, int grid)
{
    const int per = grid / kNumXcd;
    return (b % kNumXcd) * per + b / kNumXcd;
}

// Immediate of s_waitcnt in the gfx9-family layout that gfx950 uses:
// vmcnt in bits 3:0 (low part) and 15:14 (high part), expcnt in bits 6:4,
// lgkmcnt in bits 11:8.  A counter at its field maximum is not waited for.
constexpr unsigned waitcnt_imm(unsigned vmcnt, unsigned expcnt, unsigned lgkmcnt)
{
    return (vmcnt & 0xFu) | ((expcnt & 0x7u) << 4) | ((lgkmcnt & 0xFu) << 8) | (((vmcnt >> 4) & 0x3u) << 14);
}
// Wait until no vector memory operation (load or store) of the wave is
// outstanding; LDS, scalar and export counters are left alone.
constexpr unsigned kWaitVmcnt0 = waitcnt_imm(0, 7, 15);
static_assert(kWaitVmcnt0 == 0x0F70u, "s_waitcnt vmcnt(0) expcnt(7) lgkmcnt(15) on gfx9");
static_assert((kWaitVmcnt0 & 0xC00Fu) == 0, "both vmcnt fields are zero");
static_assert(((kWaitVmcnt0 >> 4) & 0x7u) == 7 && ((kWaitVmcnt0 >> 8) & 0xFu) == 15,
              "expcnt and lgkmcnt at their maxima");

__device__ __forceinline__ int32_t flag_load(const int32_t *p)
{
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ void flag_store(int32_t *p, int32_t v)
{
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Butterfly sum over the 64 lanes, every lane gets the total.
template <typename T>
__device__ __forceinline__ T wave_sum(T v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = v + __shfl_xor(v, o, 64);
    return v;
}

// Butterfly sum over the lanes of equal lane % S (S a power of two <= 64):
// lane l gets the sum of its residue class.
template <int S, typename T>
__device__ __forceinline__ T wave_sum_strided(T v)
{
#pragma unroll
    for (int o = 32; o >= S; o >>= 1) v = v + __shfl_xor(v, o, 64);
    return v;
}

// Fixed-order sum over the workgroup (kWG threads), returned to every
// thread.  ws: kWG/64 + 1 slots.
template <typename T>
__device__ __forceinline__ T block_sum_all(T v, T *ws)
{
    v = wave_sum(v);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    if (lane == 0) ws[w] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        T t = T(0);
#pragma unroll
        for (int i = 0; i < kWG / 64; ++i) t = t + ws[i];
        ws[kWG / 64] = t;
    }
    __syncthreads();
    const T t = ws[kWG / 64];
    __syncthreads();
    return t;
}

}  // namespace dev
}  // namespace ss
