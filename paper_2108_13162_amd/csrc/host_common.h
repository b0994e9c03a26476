// Host-side helpers shared by the solver drivers: the device allocator
// wrapper (caller-supplied allocator or hipMalloc) and HIP error checking.
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <string>
#include <vector>

#include "ss_internal.h"

namespace ss {

struct DeviceMem {
    ss_alloc_fn alloc = nullptr;
    ss_free_fn release = nullptr;
    void *ctx = nullptr;
    std::vector<void *> blocks;

    void *get(size_t bytes)
    {
        if (bytes == 0) bytes = 16;
        bytes = (bytes + 255) & ~size_t(255);
        void *p = nullptr;
        if (alloc) {
            p = alloc(ctx, bytes);
            // the kernels use 16-byte accesses: a caller's block must be
            // aligned like hipMalloc's
            if (p && (reinterpret_cast<uintptr_t>(p) & 255)) {
                if (release) release(ctx, p);
                p = nullptr;
            }
        } else if (hipMalloc(&p, bytes) != hipSuccess) {
            (void)hipGetLastError();
            p = nullptr;
        }
        if (p) blocks.push_back(p);
        return p;
    }
    void put(void *p)
    {
        auto it = std::find(blocks.begin(), blocks.end(), p);
        if (it == blocks.end()) return;
        blocks.erase(it);
        if (release)
            release(ctx, p);
        else
            (void)hipFree(p);
    }
    void clear()
    {
        for (void *p : blocks) {
            if (release)
                release(ctx, p);
            else
                (void)hipFree(p);
        }
        blocks.clear();
    }
};

}  // namespace ss

// Returns SS_EDEVICE (with the HIP error text) from the enclosing function.
#define SS_HIP(call)                                                                                         \
    do {                                                                                                     \
        hipError_t e_ = (call);                                                                              \
        if (e_ != hipSuccess) return fail(SS_EDEVICE, std::string(#call) + ": " + hipGetErrorString(e_)); \
    } while (0)
