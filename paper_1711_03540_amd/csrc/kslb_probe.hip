// kslb_probe.hip -- device-peak measurement kernels (see include/kslb_probe.h).
#include <hip/hip_runtime.h>

#include <cstdint>

#include "../../include/kslb_probe.h"

namespace {

typedef unsigned int u4v __attribute__((ext_vector_type(4)));

// Each workgroup copies kCopyPer x 256 consecutive 16-byte words: all of a
// lane's loads are issued before its stores, so kCopyPer loads per lane are in
// flight at once; streaming (non-temporal) stores, as the solver's one-step
// kernel uses.
constexpr int kCopyPer = 4;

__global__ __launch_bounds__(256) void k_probe_copy(u4v* __restrict__ dst, const u4v* __restrict__ src, int64_t n)
{
    const int64_t base = (int64_t)blockIdx.x * (256 * kCopyPer) + threadIdx.x;
    u4v v[kCopyPer];
#pragma unroll
    for (int k = 0; k < kCopyPer; k++) {
        const int64_t i = base + 256 * k;
        if (i < n) v[k] = src[i];
    }
#pragma unroll
    for (int k = 0; k < kCopyPer; k++) {
        const int64_t i = base + 256 * k;
        if (i < n) __builtin_nontemporal_store(v[k], dst + i);
    }
}

constexpr int kLdsLanes = 256;
constexpr int kLdsBytes = 32 * 1024;                 // five workgroups fit a 160 KiB CU
constexpr int kLdsVecs = kLdsBytes / 16;                 // 16-byte words in the area
constexpr int kLdsPerLane = kLdsVecs / kLdsLanes;        // 8 words per lane per sweep

__global__ __launch_bounds__(kLdsLanes) void k_probe_lds(uint64_t* __restrict__ out, int iters)
{
    __shared__ u4v area[kLdsVecs];
    const int t = threadIdx.x;
    for (int k = t; k < kLdsVecs; k += kLdsLanes) area[k] = u4v{(unsigned)k, (unsigned)(k * 3), (unsigned)(k ^ 77), 1u};
    __syncthreads();
    u4v acc = {0u, 0u, 0u, 0u};
    const uint64_t c0 = __builtin_readcyclecounter();
    const uint64_t r0 = __builtin_amdgcn_s_memrealtime();
    for (int it = 0; it < iters; it++) {
        // lane t reads words t, t + 256, ...: each wave's 64 lanes touch 64
        // consecutive 16-byte words per load
#pragma unroll
        for (int k = 0; k < kLdsPerLane; k++) acc ^= area[k * kLdsLanes + ((t + it) & (kLdsLanes - 1))];
    }
    __syncthreads();
    const uint64_t c1 = __builtin_readcyclecounter();
    const uint64_t r1 = __builtin_amdgcn_s_memrealtime();
    // fold the lanes' values so that every load is live
    unsigned v = acc.x ^ acc.y ^ acc.z ^ acc.w;
    v = __reduce_xor_sync(~0ull, v);
    __shared__ unsigned part[kLdsLanes / 64];
    if ((t & 63) == 0) part[t >> 6] = v;
    __syncthreads();
    if (t == 0) {
        unsigned f = 0;
        for (int w = 0; w < kLdsLanes / 64; w++) f ^= part[w];
        uint64_t* o = out + 4 * (int64_t)blockIdx.x;
        o[0] = (uint64_t)iters * kLdsBytes;
        o[1] = c1 - c0;
        o[2] = r1 - r0;
        o[3] = f;
    }
}

}  // namespace

extern "C" {

int kslb_probe_copy(void* dst, const void* src, size_t bytes, void* stream)
{
    if (!dst || !src || bytes % 16) return (int)hipErrorInvalidValue;
    const int64_t n = (int64_t)(bytes / 16);
    if (n == 0) return 0;
    const int64_t grid = (n + 256 * kCopyPer - 1) / (256 * kCopyPer);
    if (grid > 0x7fffffff) return (int)hipErrorInvalidValue;
    k_probe_copy<<<(unsigned)grid, 256, 0, (hipStream_t)stream>>>((u4v*)dst, (const u4v*)src, n);
    return (int)hipGetLastError();
}

int kslb_probe_lds(uint64_t* out, int blocks, int iters, void* stream)
{
    if (!out || blocks < 1 || iters < 1) return (int)hipErrorInvalidValue;
    k_probe_lds<<<(unsigned)blocks, kLdsLanes, 0, (hipStream_t)stream>>>(out, iters);
    return (int)hipGetLastError();
}

}  // extern "C"
