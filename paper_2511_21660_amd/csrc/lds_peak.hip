// lds_peak.hip -- LDS read bandwidth of one MI355X (gfx950), measured.
//
// The LDS roofline of the decoding kernels needs the chip's LDS read
// bandwidth per CU per clock.  Each workgroup of 256 threads fills a 16 KiB
// LDS buffer, then every thread reads it in a loop: eight reads per trip at
// eight fixed, conflict-free addresses (lane t of a wave reads element
// u * stride + t, stride = 256 passed at run time, so a wave touches
// consecutive elements).  The addresses are made opaque once, so the compiler
// can neither fuse two reads into one two-address instruction nor compute an
// address per read, and a memory clobber at the top of every trip makes it
// read again.  The values are summed with three-input adds (half a VALU
// instruction per 4-byte read), so the reads, not the VALU, set the rate.
// Element width 4, 8 or 16 bytes selects ds_read_b32, _b64 or _b128.  Thread
// 0 of every workgroup records the shader clock (clock64) and the
// constant-rate wall clock (wall_clock64) around its loop, so the host can
// state the clock the reads ran at.

#include <hip/hip_runtime.h>

#include <cstdint>

namespace {

constexpr int kThreads = 256;
constexpr int kBufBytes = 16384;

template <typename T>
__global__ __launch_bounds__(kThreads) void lds_read_kernel(int iters, int stride, uint32_t *out,
                                                             unsigned long long *clk) {
    constexpr int NE = kBufBytes / (int)sizeof(T);  // elements, a power of two
    constexpr int NW = (int)(sizeof(T) / 4);        // 32-bit words per element
    __shared__ T buf[NE];
    const int t = threadIdx.x;
    uint32_t *w = reinterpret_cast<uint32_t *>(buf);
    for (int i = t; i < kBufBytes / 4; i += kThreads) w[i] = (uint32_t)i * 2654435761u;
    __syncthreads();
    int idx[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
        idx[u] = (u * stride + t) & (NE - 1);
        asm volatile("" : "+v"(idx[u]));
    }
    const unsigned long long c0 = clock64();
    const unsigned long long r0 = wall_clock64();
    uint32_t acc[2] = {0u, 0u};
    for (int k = 0; k < iters; k += 8) {
        asm volatile("" ::: "memory");
        T v[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) v[u] = buf[idx[u]];
#pragma unroll
        for (int u = 0; u < 8; u += (NW == 1 ? 2 : 1)) {
            const uint32_t *a = reinterpret_cast<const uint32_t *>(&v[u]);
            if (NW == 1) {
                const uint32_t *b = reinterpret_cast<const uint32_t *>(&v[u + 1]);
                acc[0] = acc[0] + a[0] + b[0];
            } else {
#pragma unroll
                for (int q = 0; q < NW; q += 2) acc[q / 2 % 2] = acc[q / 2 % 2] + a[q] + a[q + 1];
            }
        }
    }
    __syncthreads();
    const unsigned long long c1 = clock64();
    const unsigned long long r1 = wall_clock64();
    out[(size_t)blockIdx.x * kThreads + t] = acc[0] ^ acc[1];
    if (t == 0) {
        clk[(size_t)blockIdx.x * 2 + 0] = c1 - c0;
        clk[(size_t)blockIdx.x * 2 + 1] = r1 - r0;
    }
}

}  // namespace

extern "C" {

// Runs `reps` timed launches of the probe with element width `bytes` (4, 8
// or 16) over `blocks` workgroups of 256 threads, `iters` reads per thread
// (a multiple of 8).  Device buffers: out uint32 [blocks * 256], clk uint64
// [blocks * 2].  Returns 0 and the mean launch time in *ms, or a HIP error
// code; -1 for bad arguments.
int lds_peak_run(int bytes, int blocks, int iters, int reps, uint32_t *d_out, unsigned long long *d_clk,
                 float *ms) {
    if (blocks < 1 || iters < 8 || iters % 8 || reps < 1 || !d_out || !d_clk || !ms) return -1;
    const void *fn = bytes == 4    ? (const void *)lds_read_kernel<uint32_t>
                     : bytes == 8  ? (const void *)lds_read_kernel<uint2>
                     : bytes == 16 ? (const void *)lds_read_kernel<uint4>
                                   : nullptr;
    if (!fn) return -1;
    int stride = kThreads;
    void *args[] = {&iters, &stride, &d_out, &d_clk};
    hipError_t e = hipLaunchKernel(fn, dim3(blocks), dim3(kThreads), args, 0, nullptr);  // warm-up
    if (e != hipSuccess) return (int)e;
    hipEvent_t a, b;
    if ((e = hipEventCreate(&a)) != hipSuccess) return (int)e;
    if ((e = hipEventCreate(&b)) != hipSuccess) return (int)e;
    (void)hipEventRecord(a, nullptr);
    for (int r = 0; r < reps; ++r) (void)hipLaunchKernel(fn, dim3(blocks), dim3(kThreads), args, 0, nullptr);
    (void)hipEventRecord(b, nullptr);
    e = hipEventSynchronize(b);
    float t = 0.0f;
    if (e == hipSuccess) e = hipEventElapsedTime(&t, a, b);
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    if (e != hipSuccess) return (int)e;
    *ms = t / (float)reps;
    return (int)hipGetLastError();
}

// Rate of the constant clock read by wall_clock64 on `device`, in kHz (0 on error).
int lds_peak_wall_clock_khz(int device) {
    int khz = 0;
    if (hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, device) != hipSuccess) return 0;
    return khz;
}

}  // extern "C"
