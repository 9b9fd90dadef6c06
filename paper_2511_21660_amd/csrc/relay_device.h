// relay_device.h -- device helpers shared by the one-shot-per-workgroup
// kernels (relay_block.hip, relay_large.hip): absolute LDS addressing and
// block-wide reductions.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace rb {
namespace {

template <typename T>
__device__ __forceinline__ __attribute__((address_space(3))) T &lds_b(uint32_t byte_addr) {
    return *(__attribute__((address_space(3))) T *)(size_t)byte_addr;
}

// Sum over the block (every thread gets the total); `red` is the byte address
// of TPB/64 doubles of LDS scratch.
template <int TPB>
__device__ __forceinline__ double block_sum(double x, uint32_t red) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off, 64);
    const int wave = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) lds_b<double>(red + 8u * wave) = x;
    __syncthreads();
    double tot = 0.0;
#pragma unroll
    for (int w = 0; w < TPB / 64; ++w) tot += lds_b<double>(red + 8u * w);
    __syncthreads();
    return tot;
}

// OR of a predicate over the block (every thread gets the result); `flags` is
// the 16-byte aligned byte address of TPB/64 bytes of LDS scratch (zeroed at
// kernel start), one byte per wave, read back as TPB/256 words.  One barrier:
// the caller guarantees another barrier before the next call, so no wave can
// overwrite a flag that another wave has still to read.  (The library's
// kernels address LDS absolutely from 0 and must not use static LDS, so the
// runtime's __syncthreads_or, which keeps its scratch in static LDS, is not
// used.)
template <int TPB>
__device__ __forceinline__ bool block_or(bool pred, uint32_t flags) {
    const bool any = __any(pred);
    const int wave = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) lds_b<uint8_t>(flags + (uint32_t)wave) = any ? 1 : 0;
    __syncthreads();
    uint32_t acc = 0;
#pragma unroll
    for (int q = 0; q < TPB / 256; ++q) acc |= lds_b<uint32_t>(flags + 4u * (uint32_t)q);
    return acc != 0u;
}

}  // namespace
}  // namespace rb
