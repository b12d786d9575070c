// Device-wide exclusive prefix sums (u32, u64) and fill/copy kernels.
//
// Per-tile sums, then the per-tile scan with its offset added.  With few tiles
// (at most kScanFewTiles) each tile adds up the sums of the tiles before it
// itself; with more, one workgroup scans the tile sums in between (three
// launches).  out has n + 1 entries;
// out[n] is the total.  Fills are plain kernels (no hipMemset) so that the
// whole pipeline stays capturable in a HIP graph.
#include "bbc_internal.h"

namespace bbc {

constexpr int kScanThreads = 256;
constexpr int kScanItems = 8;
constexpr uint32_t kScanTile = kScanThreads * kScanItems;

template <typename T>
__device__ inline T block_excl_scan(T v, T* s_wave, T* total) {
    // s_wave: kScanThreads / 64 entries
    const uint32_t lane = lane_id(), wave = threadIdx.x >> 6;
    T incl = wave_incl_scan(v);
    if (lane == 63) s_wave[wave] = incl;
    __syncthreads();
    T wave_off = 0, tot = 0;
    for (uint32_t w = 0; w < kScanThreads / 64; ++w) {
        T s = s_wave[w];
        if (w < wave) wave_off += s;
        tot += s;
    }
    __syncthreads();
    *total = tot;
    return wave_off + incl - v;
}

template <typename T>
__global__ __launch_bounds__(kScanThreads) void k_tile_sums(const T* in, uint32_t n, T* sums) {
    __shared__ T s_wave[kScanThreads / 64];
    const uint64_t base = (uint64_t)blockIdx.x * kScanTile;
    T acc = 0;
    for (int i = 0; i < kScanItems; ++i) {
        uint64_t idx = base + (uint64_t)i * kScanThreads + threadIdx.x;
        if (idx < n) acc += in[idx];
    }
    T tot;
    block_excl_scan(acc, s_wave, &tot);
    if (threadIdx.x == 0) sums[blockIdx.x] = tot;
}

template <typename T>
__global__ __launch_bounds__(1024) void k_scan_sums(T* sums, uint32_t nb, T* total_out) {
    // One workgroup: exclusive scan of nb tile sums in place, chunks of 1024.
    __shared__ T s_wave[16];
    __shared__ T s_carry;
    if (threadIdx.x == 0) s_carry = 0;
    __syncthreads();
    const uint32_t lane = lane_id(), wave = threadIdx.x >> 6;
    for (uint32_t c = 0; c < nb; c += 1024) {
        uint32_t i = c + threadIdx.x;
        T v = i < nb ? sums[i] : 0;
        T incl = wave_incl_scan(v);
        if (lane == 63) s_wave[wave] = incl;
        __syncthreads();
        T off = s_carry, tot = 0;
        for (uint32_t w = 0; w < 16; ++w) {
            T s = s_wave[w];
            if (w < wave) off += s;
            tot += s;
        }
        if (i < nb) sums[i] = off + incl - v;
        __syncthreads();
        if (threadIdx.x == 0) s_carry += tot;
        __syncthreads();
    }
    if (threadIdx.x == 0) *total_out = s_carry;
}

template <typename T>
__global__ __launch_bounds__(kScanThreads) void k_tile_scan(const T* in, T* out, uint32_t n,
                                                            const T* offs, const T* total) {
    __shared__ T s_wave[kScanThreads / 64];
    const uint64_t base = (uint64_t)blockIdx.x * kScanTile;
    // blocked layout: thread t owns items base + t*kScanItems .. +kScanItems
    T v[kScanItems];
    T acc = 0;
    const uint64_t my = base + (uint64_t)threadIdx.x * kScanItems;
    for (int i = 0; i < kScanItems; ++i) {
        v[i] = (my + i < n) ? in[my + i] : 0;
        acc += v[i];
    }
    T tot;
    T run = block_excl_scan(acc, s_wave, &tot) + offs[blockIdx.x];
    for (int i = 0; i < kScanItems; ++i) {
        if (my + i < n) out[my + i] = run;
        run += v[i];
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) out[n] = *total;
}

// the per-tile scan, taking its offset as the sum of the earlier tiles' sums;
// the last tile writes the total
constexpr uint32_t kScanFewTiles = 1024;

template <typename T>
__global__ __launch_bounds__(kScanThreads) void k_tile_scan_few(const T* in, T* out, uint32_t n,
                                                                const T* sums) {
    __shared__ T s_wave[kScanThreads / 64];
    const uint64_t base = (uint64_t)blockIdx.x * kScanTile;
    T pre = 0;
    for (uint32_t i = threadIdx.x; i < blockIdx.x; i += kScanThreads) pre += sums[i];
    T v[kScanItems];
    T acc = 0;
    const uint64_t my = base + (uint64_t)threadIdx.x * kScanItems;
    for (int i = 0; i < kScanItems; ++i) {
        v[i] = (my + i < n) ? in[my + i] : 0;
        acc += v[i];
    }
    T off, tot;
    block_excl_scan(pre, s_wave, &off);  // off: the sum of all earlier tiles
    T run = block_excl_scan(acc, s_wave, &tot) + off;
    for (int i = 0; i < kScanItems; ++i) {
        if (my + i < n) out[my + i] = run;
        run += v[i];
    }
    if (blockIdx.x == gridDim.x - 1 && threadIdx.x == 0) out[n] = off + tot;
}

size_t scan_tmp_bytes(uint32_t n) {
    size_t nb = (size_t)(n + kScanTile - 1) / kScanTile + 1;
    return (size_t)kMaxScanSet * (nb + 2) * sizeof(u64) + 256;
}

template <typename T>
static hipError_t scan_impl(const T* in, T* out, uint32_t n, void* tmp, size_t tmp_bytes,
                            hipStream_t st) {
    uint32_t nb = (n + kScanTile - 1) / kScanTile;
    if (nb == 0) nb = 1;
    if ((size_t)(nb + 2) * sizeof(T) > tmp_bytes) return hipErrorInvalidValue;
    T* sums = (T*)tmp;
    T* total = sums + nb;
    hipLaunchKernelGGL(k_tile_sums<T>, dim3(nb), dim3(kScanThreads), 0, st, in, n, sums);
    if (nb <= kScanFewTiles) {
        hipLaunchKernelGGL(k_tile_scan_few<T>, dim3(nb), dim3(kScanThreads), 0, st, in, out, n,
                           (const T*)sums);
        return hipGetLastError();
    }
    hipLaunchKernelGGL(k_scan_sums<T>, dim3(1), dim3(1024), 0, st, sums, nb, total);
    hipLaunchKernelGGL(k_tile_scan<T>, dim3(nb), dim3(kScanThreads), 0, st, in, out, n,
                       (const T*)sums, (const T*)total);
    return hipGetLastError();
}

// Several scans of the same length in one pair of launches (blockIdx.y picks
// the array), for the groups of per-vertex scans the pipeline runs together.
template <typename T>
struct ScanSet {
    const T* in[kMaxScanSet];
    T* out[kMaxScanSet];
};

template <typename T>
__global__ __launch_bounds__(kScanThreads) void k_tile_sums_set(ScanSet<T> set, uint32_t n,
                                                                T* sums) {
    __shared__ T s_wave[kScanThreads / 64];
    const T* in = set.in[blockIdx.y];
    const uint64_t base = (uint64_t)blockIdx.x * kScanTile;
    T acc = 0;
    for (int i = 0; i < kScanItems; ++i) {
        uint64_t idx = base + (uint64_t)i * kScanThreads + threadIdx.x;
        if (idx < n) acc += in[idx];
    }
    T tot;
    block_excl_scan(acc, s_wave, &tot);
    if (threadIdx.x == 0) sums[(size_t)blockIdx.y * gridDim.x + blockIdx.x] = tot;
}

template <typename T>
__global__ __launch_bounds__(kScanThreads) void k_tile_scan_few_set(ScanSet<T> set, uint32_t n,
                                                                    const T* sums_all) {
    __shared__ T s_wave[kScanThreads / 64];
    const T* in = set.in[blockIdx.y];
    T* out = set.out[blockIdx.y];
    const T* sums = sums_all + (size_t)blockIdx.y * gridDim.x;
    const uint64_t base = (uint64_t)blockIdx.x * kScanTile;
    T pre = 0;
    for (uint32_t i = threadIdx.x; i < blockIdx.x; i += kScanThreads) pre += sums[i];
    T v[kScanItems];
    T acc = 0;
    const uint64_t my = base + (uint64_t)threadIdx.x * kScanItems;
    for (int i = 0; i < kScanItems; ++i) {
        v[i] = (my + i < n) ? in[my + i] : 0;
        acc += v[i];
    }
    T off, tot;
    block_excl_scan(pre, s_wave, &off);
    T run = block_excl_scan(acc, s_wave, &tot) + off;
    for (int i = 0; i < kScanItems; ++i) {
        if (my + i < n) out[my + i] = run;
        run += v[i];
    }
    if (blockIdx.x == gridDim.x - 1 && threadIdx.x == 0) out[n] = off + tot;
}

template <typename T>
static hipError_t scan_set_impl(const T* const* ins, T* const* outs, uint32_t k, uint32_t n,
                                void* tmp, size_t tmp_bytes, hipStream_t st) {
    uint32_t nb = (n + kScanTile - 1) / kScanTile;
    if (nb == 0) nb = 1;
    if (k == 0 || k > kMaxScanSet || nb > kScanFewTiles || (size_t)k * nb * sizeof(T) > tmp_bytes) {
        for (uint32_t i = 0; i < k; ++i) {  // one scan at a time
            hipError_t e = scan_impl<T>(ins[i], outs[i], n, tmp, tmp_bytes, st);
            if (e != hipSuccess) return e;
        }
        return hipSuccess;
    }
    ScanSet<T> set;
    for (uint32_t i = 0; i < kMaxScanSet; ++i) {
        set.in[i] = i < k ? ins[i] : nullptr;
        set.out[i] = i < k ? outs[i] : nullptr;
    }
    hipLaunchKernelGGL(k_tile_sums_set<T>, dim3(nb, k), dim3(kScanThreads), 0, st, set, n, (T*)tmp);
    hipLaunchKernelGGL(k_tile_scan_few_set<T>, dim3(nb, k), dim3(kScanThreads), 0, st, set, n,
                       (const T*)tmp);
    return hipGetLastError();
}

hipError_t scan_excl_u32_set(const uint32_t* const* ins, uint32_t* const* outs, uint32_t k,
                             uint32_t n, void* tmp, size_t tmp_bytes, hipStream_t st) {
    return scan_set_impl<uint32_t>(ins, outs, k, n, tmp, tmp_bytes, st);
}

hipError_t scan_excl_u64_set(const u64* const* ins, u64* const* outs, uint32_t k, uint32_t n,
                             void* tmp, size_t tmp_bytes, hipStream_t st) {
    return scan_set_impl<u64>(ins, outs, k, n, tmp, tmp_bytes, st);
}

hipError_t scan_excl_u32(const uint32_t* in, uint32_t* out, uint32_t n, void* tmp,
                         size_t tmp_bytes, hipStream_t st) {
    return scan_impl<uint32_t>(in, out, n, tmp, tmp_bytes, st);
}

hipError_t scan_excl_u64(const u64* in, u64* out, uint32_t n, void* tmp, size_t tmp_bytes,
                         hipStream_t st) {
    return scan_impl<u64>(in, out, n, tmp, tmp_bytes, st);
}

template <typename T>
__global__ void k_fill(T* p, T v, size_t n) {
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (size_t)gridDim.x * blockDim.x)
        p[i] = v;
}

__global__ void k_copy_u32(const uint32_t* __restrict__ s, uint32_t* __restrict__ d, size_t n) {
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (size_t)gridDim.x * blockDim.x)
        d[i] = s[i];
}

static dim3 grid_for(size_t n) {
    size_t b = (n + 255) / 256;
    if (b > 8192) b = 8192;
    if (b == 0) b = 1;
    return dim3((unsigned)b);
}

hipError_t fill_u32(uint32_t* p, uint32_t v, size_t n, hipStream_t st) {
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_fill<uint32_t>, grid_for(n), dim3(256), 0, st, p, v, n);
    return hipGetLastError();
}

hipError_t fill_u64(u64* p, u64 v, size_t n, hipStream_t st) {
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_fill<u64>, grid_for(n), dim3(256), 0, st, p, v, n);
    return hipGetLastError();
}

hipError_t copy_u32(const uint32_t* src, uint32_t* dst, size_t n, hipStream_t st) {
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_copy_u32, grid_for(n), dim3(256), 0, st, src, dst, n);
    return hipGetLastError();
}

}  // namespace bbc
