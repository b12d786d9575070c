// LDS atomic throughput probe (measurement only; not part of the counting
// library).  The wedge kernel spends one LDS atomic add per wedge on a bucket
// counter; this probe measures how many such adds one MI355X retires per
// second, so that the kernel's achieved rate can be set against a measured
// ceiling.
//
// Each workgroup has the wedge kernel's shape (1024 threads, a 128 KiB LDS
// table) and issues non-returning ds_add on the table:
//   pattern 0: conflict-free, lane i of a wave adds to word i of its own
//              stripe (64 distinct consecutive words per wave);
//   pattern 1: scattered, every lane adds to a pseudo-random word of the whole
//              table, the way end vertices hit the dense bucket counters;
//   pattern 2: scattered over 64-bit words (the 64-bit bucket counters).
// The table is summed into global memory at the end so the adds stay live.
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace {

constexpr int kThreads = 1024;
constexpr uint32_t kWords = 32768;  // 128 KiB of u32
constexpr int kUnroll = 8;

template <int PATTERN>
__global__ __launch_bounds__(kThreads) void k_lds_add(uint32_t iters, unsigned long long* out) {
    __shared__ uint32_t tab[kWords];
    for (uint32_t i = threadIdx.x; i < kWords; i += kThreads) tab[i] = 0;
    __syncthreads();
    const uint32_t tid = threadIdx.x;
    // per-lane start and odd stride (xorshift of the thread and block index)
    uint32_t s = (tid + 1u) * 0x9E3779B1u ^ (blockIdx.x * 0x85EBCA77u);
    s ^= s << 13;
    s ^= s >> 17;
    s ^= s << 5;
    const uint32_t stride = (s >> 7) | 1u;
    uint32_t a = s;
    if (PATTERN == 0) {
        const uint32_t base = (tid & ~63u) + (tid & 63u);  // word tid: 64 consecutive words per wave
        for (uint32_t it = 0; it < iters; ++it) {
#pragma unroll
            for (int k = 0; k < kUnroll; ++k) atomicAdd(&tab[(base + k * kThreads) & (kWords - 1)], 1u);
        }
    } else if (PATTERN == 1) {
        for (uint32_t it = 0; it < iters; ++it) {
#pragma unroll
            for (int k = 0; k < kUnroll; ++k) {
                a += stride;
                atomicAdd(&tab[a & (kWords - 1)], 1u);
            }
        }
    } else {
        unsigned long long* t64 = reinterpret_cast<unsigned long long*>(tab);
        for (uint32_t it = 0; it < iters; ++it) {
#pragma unroll
            for (int k = 0; k < kUnroll; ++k) {
                a += stride;
                atomicAdd(&t64[a & (kWords / 2 - 1)], 1ull);
            }
        }
    }
    __syncthreads();
    unsigned long long sum = 0;
    for (uint32_t i = threadIdx.x; i < kWords; i += kThreads) sum += tab[i];
    atomicAdd(out, sum);
}

}  // namespace

extern "C" {

// Runs `pattern` (0, 1 or 2 above) with `blocks` workgroups of 1024 threads,
// each thread issuing iters * 8 adds, `repeats` times; *adds_per_s gets the
// best rate over the repeats (adds retired per second, whole device), *ms the
// best launch time, *check the number of adds the last launch recorded, which
// must equal blocks * 1024 * iters * 8 (for pattern 2 the table is summed as
// u32 halves; the high halves stay zero).  Returns 0 on success, else a
// hipError_t.
int bbc_probe_lds_atomics(int device, int pattern, int blocks, int iters, int repeats,
                          double* adds_per_s, double* ms, unsigned long long* check) {
    if (pattern < 0 || pattern > 2 || blocks < 1 || iters < 1 || repeats < 1 || !adds_per_s || !ms ||
        !check)
        return (int)hipErrorInvalidValue;
    hipError_t e = hipSetDevice(device);
    if (e != hipSuccess) return (int)e;
    unsigned long long* d_out = nullptr;
    e = hipMalloc(&d_out, sizeof(unsigned long long));
    if (e != hipSuccess) return (int)e;
    hipEvent_t e0, e1;
    hipEventCreate(&e0);
    hipEventCreate(&e1);
    float best = 1e30f;
    for (int r = 0; r < repeats + 1; ++r) {  // the first launch warms up
        hipMemset(d_out, 0, sizeof(unsigned long long));
        hipEventRecord(e0, 0);
        if (pattern == 0)
            hipLaunchKernelGGL(k_lds_add<0>, dim3(blocks), dim3(kThreads), 0, 0, (uint32_t)iters, d_out);
        else if (pattern == 1)
            hipLaunchKernelGGL(k_lds_add<1>, dim3(blocks), dim3(kThreads), 0, 0, (uint32_t)iters, d_out);
        else
            hipLaunchKernelGGL(k_lds_add<2>, dim3(blocks), dim3(kThreads), 0, 0, (uint32_t)iters, d_out);
        hipEventRecord(e1, 0);
        e = hipEventSynchronize(e1);
        if (e != hipSuccess) break;
        float t = 0;
        hipEventElapsedTime(&t, e0, e1);
        if (r > 0 && t < best) best = t;
    }
    if (e == hipSuccess) e = hipMemcpy(check, d_out, sizeof(unsigned long long), hipMemcpyDeviceToHost);
    hipEventDestroy(e0);
    hipEventDestroy(e1);
    hipFree(d_out);
    if (e != hipSuccess) return (int)e;
    const double adds = (double)blocks * kThreads * (double)iters * kUnroll;
    *ms = best;
    *adds_per_s = adds / (best * 1e-3);
    return 0;
}

}  // extern "C"
