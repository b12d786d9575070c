// Work planning for the wedge kernel.
//
// The counting of Algorithm 2 (Section 4.1) is independent per start vertex u
// (the outer loop; Algorithm 4 of Section 5.2 runs it in parallel).  Its cost
// is W_u, the number of wedges with start u.  The start's buckets (one pair of
// counters per end vertex w) must see every wedge (u, ., w) before C(.,2) is
// applied, so a start is split only along the end-vertex axis (disjoint w
// ranges each hold complete counts) or, when the end-vertex space is small,
// along the middle-vertex axis with an exact merge of partial counts
// (C(a+b,2) = C(a,2) + C(b,2) + ab).
//
// Per start with W_u > 0 (S = number of same-side vertices below u, so the
// end vertices have sidx in [0, S)):
//   * light   (W_u <= kLightMax): one hashed piece; many light starts share
//             one work item, each in its own region of the on-chip table;
//   * small S (S <= kDenseW): dense counters over [0, S); split into record
//             chunks of ~kRecordChunkWedges wedges merged through G;
//   * else:   the end-vertex space is cut into tiles of kTile.  The wedges of u
//             are estimated per tile in proportion to the tile's degree mass
//             (an end vertex is reached through its edges).  A tile expected to
//             hold more than kHashTarget wedges becomes one dense piece (its
//             counters always fit); runs of lighter tiles are packed greedily
//             into hashed pieces of at most kHashTarget expected wedges.  A
//             hashed piece that overflows anyway is redone by the wedge kernel
//             in halves.
#include "bbc_internal.h"

namespace bbc {

__device__ inline uint32_t next_pow2(uint32_t x) {
    uint32_t p = 1;
    while (p < x) p <<= 1;
    return p;
}

__device__ inline uint32_t log2_pow2(uint32_t x) { return 31u - __clz(x); }

// Sort key putting the most expensive pieces first (ascending key): a 16-bit
// log-scale of the estimated cost, 4 units per record visited plus the
// expected wedges.
__device__ inline uint32_t cost_key(double wedges, uint32_t nrec) {
    const double c = wedges + 4.0 * nrec;
    const double q = log2(1.0 + c) * 2048.0;
    return 65535u - (uint32_t)fmin(q, 65535.0);
}

// Tile runs of a start with end-vertex space [0, S) on the side whose rows start
// at `base`; calls emit(t0, t1, dense, expected wedges) per run and returns the
// number of runs.
template <typename F>
__device__ uint32_t plan_runs(const uint32_t* __restrict__ row_ptr, uint32_t base, uint32_t S,
                              u64 W, F emit) {
    const uint32_t T = (S + kTile - 1) / kTile;
    const double tot = (double)(row_ptr[base + S] - row_ptr[base]);
    const double scale = tot > 0 ? (double)W / tot : 0.0;
    uint32_t n = 0, rs = kNoTile;
    double re = 0;
    for (uint32_t t = 0; t < T; ++t) {
        const uint32_t lo = t * kTile, hi = min(S, lo + kTile);
        const double e = (double)(row_ptr[base + hi] - row_ptr[base + lo]) * scale;
        if (e > kHashTarget) {
            if (rs != kNoTile) {
                emit(rs, t, false, re);
                ++n;
                rs = kNoTile;
            }
            emit(t, t + 1, true, e);
            ++n;
        } else if (rs != kNoTile && re + e > kHashTarget) {
            emit(rs, t, false, re);
            ++n;
            rs = t;
            re = e;
        } else {
            if (rs == kNoTile) {
                rs = t;
                re = 0;
            }
            re += e;
        }
    }
    if (rs != kNoTile) {
        emit(rs, T, false, re);
        ++n;
    }
    return n;
}

__global__ void k_plan_count(const u64* __restrict__ wu, const uint32_t* __restrict__ lowcnt,
                             const uint32_t* __restrict__ row_ptr, Dims d, uint32_t* __restrict__ hp, u64* __restrict__ lr,
                             uint32_t* __restrict__ lf, uint32_t* __restrict__ gs) {
    for (uint32_t r = blockIdx.x * blockDim.x + threadIdx.x; r < d.n; r += gridDim.x * blockDim.x) {
        uint32_t side = r >= d.n_u ? 1u : 0u;
        uint32_t S = r - d.base[side];
        u64 W = wu[r];
        uint32_t k = lowcnt[r];
        uint32_t h = 0, l = 0, f = 0, g = 0;
        if (W == 0) {
        } else if (W <= kLightMax) {
            l = max(kMinRegion, next_pow2((uint32_t)(2 * W)));
            f = 1;
        } else if (S <= kDenseW) {
            u64 np = (W + kRecordChunkWedges - 1) / kRecordChunkWedges;
            if (np > k) np = k;
            h = (uint32_t)np;
            g = np > 1 ? S : 0;
        } else {
            h = plan_runs(row_ptr, d.base[side], S, W, [](uint32_t, uint32_t, bool, double) {});
        }
        hp[r] = h;
        lr[r] = l;
        lf[r] = f;
        gs[r] = g;
    }
}

__global__ void k_plan_write(const u64* __restrict__ wu, const uint32_t* __restrict__ lowcnt,
                             const uint32_t* __restrict__ row_ptr,
                             const uint32_t* __restrict__ mptr, const uint32_t* __restrict__ hp,
                             const uint32_t* __restrict__ hp_off, const u64* __restrict__ lr,
                             const u64* __restrict__ lr_off, const uint32_t* __restrict__ lf_off,
                             const uint32_t* __restrict__ gs_off, Dims d, uint32_t n_heavy,
                             Piece* __restrict__ pieces, u64* __restrict__ light_off,
                             uint32_t* __restrict__ hkey) {
    for (uint32_t r = blockIdx.x * blockDim.x + threadIdx.x; r < d.n; r += gridDim.x * blockDim.x) {
        u64 W = wu[r];
        if (W == 0) continue;
        uint32_t side = r >= d.n_u ? 1u : 0u;
        uint32_t S = r - d.base[side];
        uint32_t k = lowcnt[r], m0 = mptr[r];
        uint32_t sideflag = side ? kPieceSideV : 0u;
        uint32_t h = hp[r];
        if (h > 0) {
            Piece* out = pieces + hp_off[r];
            uint32_t* key = hkey + hp_off[r];
            if (S <= kDenseW) {
                for (uint32_t i = 0; i < h; ++i) {
                    uint32_t c0 = (uint32_t)((u64)k * i / h), c1 = (uint32_t)((u64)k * (i + 1) / h);
                    Piece p;
                    p.rec0 = m0 + c0;
                    p.nrec = c1 - c0;
                    p.lo = 0;
                    p.hi = S;
                    p.t0 = kNoTile;
                    p.t1 = kNoTile;
                    p.region = 0;
                    p.flags = kPieceDense | (h > 1 ? kPieceMerge : 0u) | sideflag;
                    p.gbase = gs_off[r];
                    p.start_row = r;
                    out[i] = p;
                    key[i] = cost_key((double)W * (c1 - c0) / k, c1 - c0);
                }
            } else {
                const uint32_t T = (S + kTile - 1) / kTile;
                uint32_t i = 0;
                plan_runs(row_ptr, d.base[side], S, W,
                          [&](uint32_t t0, uint32_t t1, bool dense, double est) {
                    Piece p;
                    p.rec0 = m0;
                    p.nrec = k;
                    p.lo = t0 * kTile;
                    p.hi = min(S, t1 * kTile);
                    p.t0 = t0;
                    p.t1 = t1;
                    p.region = log2_pow2(kHashSlots) << 16;
                    p.flags = ((t0 == 0 && t1 == T) ? 0u : kPiecePartial) |
                              (dense ? kPieceDense : 0u) | sideflag;
                    p.gbase = kEmpty;
                    p.start_row = r;
                    if (i < h) {
                        out[i] = p;
                        key[i] = cost_key(est, k);
                    }
                    ++i;
                });
            }
                } else if (lr[r] > 0) {
            uint32_t idx = lf_off[r];
            u64 off = lr_off[r];
            u64 item = off / kLightWindow;
            uint32_t base = (uint32_t)(off - item * kLightWindow);
            Piece p;
            p.rec0 = m0;
            p.nrec = k;
            p.lo = 0;
            p.hi = S;
            p.t0 = kNoTile;
            p.t1 = kNoTile;
            p.region = base | (log2_pow2((uint32_t)lr[r]) << 16);
            p.flags = sideflag;
            p.gbase = kEmpty;
            p.start_row = r;
            pieces[n_heavy + idx] = p;
            light_off[idx] = off;
        }
    }
}

// first light piece of each light item: item i holds the pieces whose region
// offset lies in [i H, (i+1) H)
__global__ void k_items_first(const u64* __restrict__ light_off, uint32_t n_light,
                              uint32_t n_items, uint32_t* __restrict__ first) {
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i <= n_items;
         i += gridDim.x * blockDim.x) {
        u64 key = (u64)i * kLightWindow;
        uint32_t lo = 0, hi = n_light;
        while (lo < hi) {
            uint32_t mid = (lo + hi) >> 1;
            if (light_off[mid] < key)
                lo = mid + 1;
            else
                hi = mid;
        }
        first[i] = lo;
    }
}

// W = sum of W_u, and the number of starts with W_u > 0
__global__ __launch_bounds__(256) void k_sum_u64(const u64* __restrict__ a, uint32_t n,
                                                 u64* __restrict__ out, u64* __restrict__ nonzero) {
    __shared__ u64 s_s[4], s_c[4];
    u64 s = 0, c = 0;
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        s += a[i];
        c += a[i] != 0;
    }
    s = wave_reduce_sum(s);
    c = wave_reduce_sum(c);
    if (lane_id() == 0) {
        s_s[threadIdx.x >> 6] = s;
        s_c[threadIdx.x >> 6] = c;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        s = s_s[0] + s_s[1] + s_s[2] + s_s[3];
        c = s_c[0] + s_c[1] + s_c[2] + s_c[3];
        if (s) atomicAdd(out, s);
        if (c) atomicAdd(nonzero, c);
    }
}

__global__ void k_gather_totals(const uint32_t* __restrict__ hp_off, const u64* __restrict__ lr_off,
                                const uint32_t* __restrict__ lf_off,
                                const uint32_t* __restrict__ gs_off, uint32_t n, Control* ctl) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        ctl->tot_heavy = hp_off[n];
        ctl->tot_light_region = lr_off[n];
        ctl->tot_light = lf_off[n];
        ctl->tot_g = gs_off[n];
    }
}

hipError_t launch_gather_totals(const uint32_t* hp_off, const u64* lr_off, const uint32_t* lf_off,
                                const uint32_t* gs_off, uint32_t n, Control* ctl, hipStream_t st) {
    hipLaunchKernelGGL(k_gather_totals, dim3(1), dim3(64), 0, st, hp_off, lr_off, lf_off, gs_off, n,
                       ctl);
    return hipGetLastError();
}

static dim3 grid_n(uint64_t n, uint32_t threads, uint32_t cap = 16384) {
    uint64_t b = (n + threads - 1) / threads;
    if (b > cap) b = cap;
    if (b == 0) b = 1;
    return dim3((unsigned)b);
}

hipError_t launch_plan_count(const u64* wu, const uint32_t* lowcnt, const uint32_t* row_ptr, Dims d,
                             uint32_t* hp,
                             u64* lr, uint32_t* lf, uint32_t* gs, u64* wsum, u64* nonzero,
                             hipStream_t st) {
    hipLaunchKernelGGL(k_plan_count, grid_n(d.n, 256), dim3(256), 0, st, wu, lowcnt, row_ptr, d, hp,
                       lr, lf, gs);
    hipLaunchKernelGGL(k_sum_u64, grid_n(d.n, 256, 512), dim3(256), 0, st, wu, d.n, wsum, nonzero);
    return hipGetLastError();
}

hipError_t launch_plan_write(const u64* wu, const uint32_t* lowcnt, const uint32_t* row_ptr,
                             const uint32_t* mptr,
                             const uint32_t* hp, const uint32_t* hp_off, const u64* lr,
                             const u64* lr_off, const uint32_t* lf_off, const uint32_t* gs_off,
                             Dims d, uint32_t n_heavy, Piece* pieces, u64* light_off,
                             uint32_t* hkey, uint32_t n_light, uint32_t n_light_items,
                             uint32_t* items_first, hipStream_t st) {
    hipLaunchKernelGGL(k_plan_write, grid_n(d.n, 256), dim3(256), 0, st, wu, lowcnt, row_ptr, mptr, hp,
                       hp_off, lr, lr_off, lf_off, gs_off, d, n_heavy, pieces, light_off, hkey);
    hipLaunchKernelGGL(k_items_first, grid_n((uint64_t)n_light_items + 1, 256), dim3(256), 0, st,
                       (const u64*)light_off, n_light, n_light_items, items_first);
    return hipGetLastError();
}

}  // namespace bbc
