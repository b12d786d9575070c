// Preprocessing of the bucket method (Section 4.1, Algorithm 2: the vertex
// priorities and the neighbour lists in priority order; Section 4.2 notes the
// O(n) binning sort of the vertices):
//   1. validate edges, count degrees and reserve each edge's slot in its rows;
//   2. order all vertices by priority (degree, id) with a stable LSD radix sort
//      on the degree (ids enter in ascending order, so ties keep id order);
//   3. per-side index (sidx) and cross counts from a scan of side flags;
//   4. signed CSR: row offsets by scan, entries placed at the reserved slots,
//      then a segmented sort of every row by neighbour priority (size classes:
//      registers, lane groups, LDS bitonic, LDS bitmaps);
//   5. per row the number k of lower-priority neighbours (middle vertices);
//   6. one record per edge, oriented from its higher-priority end, holding the
//      middle row and the prefix length pos; W_u = sum of pos over u's records;
//   7. tile boundary tables for long rows.
#include "bbc_internal.h"

namespace bbc {

// ---------------------------------------------------------------- degrees ----
// One pass over the edges counts the degrees and gives every edge its slot in
// both of its rows: the value a row's counter had when the endpoint was added
// (any order of the slots is fine, the rows are sorted afterwards).  Each
// workgroup takes chunks of kAggChunk edges; the endpoints of one vertex inside
// a chunk are ranked in an LDS table and reserve their slots with one global
// returning atomic, so a hub costs one global atomic per chunk instead of one
// per edge (device-wide atomics are the cost here: on MI355X they retire at a
// few G/s).  Chunks of 16K edges and a 16K-slot table let every vertex of a
// small graph of a batch (at most 8192) aggregate within a chunk.  Endpoints
// that find no table slot reserve theirs directly.
constexpr int kAggThreads = 1024;
constexpr int kAggPer = 16;  // edges per thread per chunk
constexpr uint32_t kAggChunk = kAggThreads * kAggPer;
constexpr uint32_t kAggLog2 = 14;
constexpr uint32_t kAggSlots = 1u << kAggLog2;

__device__ inline bool edge_ok(int32_t u, int32_t v, int8_t s, uint32_t n_u, uint32_t n_v) {
    return (u >= 0) & ((uint32_t)u < n_u) & (v >= 0) & ((uint32_t)v < n_v) & ((s == 1) | (s == -1));
}

// Per endpoint a thread keeps one word: its table slot with its rank among the
// slot's endpoints (slot | rank << kAggLog2; a chunk has at most 2 * kAggChunk
// endpoints, so the word stays below 2^29), or kAggDirect / kAggSkip; the rank
// of a direct reservation goes to a register of its own, so that its return is
// waited for once, after the chunk (the loops are unrolled to keep all of it in
// registers, and the flush issues its returning atomics before it waits).
constexpr uint32_t kAggDirect = 1u << 30;
constexpr uint32_t kAggSkip = 1u << 31;  // invalid edge or past the end
constexpr uint32_t kAggFlush = kAggSlots / kAggThreads;
static_assert(2 * kAggChunk <= (1u << (30 - kAggLog2)), "slot and rank share a word");

__global__ __launch_bounds__(kAggThreads) void k_degree(const int32_t* __restrict__ eu,
                                                        const int32_t* __restrict__ ev,
                                                        const int8_t* __restrict__ sg, uint64_t m,
                                                        uint32_t n_u, uint32_t n_v,
                                                        uint32_t* __restrict__ deg,
                                                        uint2* __restrict__ rank, Control* ctl) {
    __shared__ uint32_t keys[kAggSlots];
    __shared__ uint32_t cnt[kAggSlots];  // ranks handed out; after the flush, the reserved base
    const uint32_t tid = threadIdx.x;
    for (uint64_t c0 = (uint64_t)blockIdx.x * kAggChunk; c0 < m; c0 += (uint64_t)gridDim.x * kAggChunk) {
        for (uint32_t i = tid; i < kAggSlots; i += kAggThreads) {
            keys[i] = kEmpty;
            cnt[i] = 0;
        }
        __syncthreads();
        // the chunk's edges first: all loads in flight together, and none
        // pending once the first returning atomic is issued (a later wait for
        // a load would wait for that atomic too: they complete in order)
        int32_t eu_k[kAggPer], ev_k[kAggPer];
        int8_t sg_k[kAggPer];
#pragma unroll
        for (int k = 0; k < kAggPer; ++k) {
            const uint64_t e = c0 + (uint64_t)k * kAggThreads + tid;
            const uint64_t ec = e < m ? e : m - 1;  // (c0 < m)
            eu_k[k] = eu[ec];
            ev_k[k] = ev[ec];
            sg_k[k] = sg[ec];
        }
        uint32_t xk[kAggPer][2];
        uint32_t okm = 0;     // bit k: edge k of this thread is in range and valid
        u64 err = ~0ull;      // the first invalid edge of this thread, as edge_err keeps it
#pragma unroll
        for (int k = 0; k < kAggPer; ++k) {
            const uint64_t e = c0 + (uint64_t)k * kAggThreads + tid;
            const int32_t u = eu_k[k], v = ev_k[k];
            const bool ok = edge_ok(u, v, sg_k[k], n_u, n_v);
            const bool range = (u < 0) | ((uint32_t)u >= n_u) | (v < 0) | ((uint32_t)v >= n_v);
            const u64 code = (e << 4) | (range ? kErrRange : kErrSign);
            err = (e < m && !ok && code < err) ? code : err;
            okm |= (e < m && ok ? 1u : 0u) << k;
            xk[k][0] = (uint32_t)u;
            xk[k][1] = n_u + (uint32_t)v;
        }
        if (err != ~0ull) atomicMin(&ctl->edge_err, err);
        uint32_t code[kAggPer][2], rg[kAggPer][2];
#pragma unroll
        for (int k = 0; k < kAggPer; ++k) {
            code[k][0] = code[k][1] = kAggSkip;  // (rg is read only where code says direct)
            if (!((okm >> k) & 1u)) continue;
#pragma unroll
            for (int t = 0; t < 2; ++t) {
                const int sl = agg_slot<kAggLog2>(keys, xk[k][t]);
                if (sl >= 0) {
                    code[k][t] = (uint32_t)sl | (atomicAdd(&cnt[sl], 1u) << kAggLog2);
                } else {
                    code[k][t] = kAggDirect;
                    rg[k][t] = atomicAdd(&deg[xk[k][t]], 1u);  // slot reserved directly
                }
            }
        }
        __syncthreads();
        {
            uint32_t fk[kAggFlush], fr[kAggFlush];
#pragma unroll
            for (uint32_t j = 0; j < kAggFlush; ++j) {
                const uint32_t i = j * kAggThreads + tid;
                fk[j] = keys[i];
                fr[j] = 0;
                if (fk[j] != kEmpty) fr[j] = atomicAdd(&deg[fk[j]], cnt[i]);
            }
#pragma unroll
            for (uint32_t j = 0; j < kAggFlush; ++j)
                if (fk[j] != kEmpty) cnt[j * kAggThreads + tid] = fr[j];
        }
        __syncthreads();
#pragma unroll
        for (int k = 0; k < kAggPer; ++k) {
            if (code[k][0] == kAggSkip) continue;
            uint32_t r[2];
#pragma unroll
            for (int t = 0; t < 2; ++t)
                r[t] = code[k][t] == kAggDirect
                           ? rg[k][t]
                           : cnt[code[k][t] & (kAggSlots - 1u)] + (code[k][t] >> kAggLog2);
            rank[c0 + (uint64_t)k * kAggThreads + tid] = make_uint2(r[0], r[1]);
        }
        __syncthreads();
    }
}

// ------------------------------------------------------------- radix sort ----
// Stable LSD radix sort of (key, value) pairs, 8-bit digits.  Tiles of 2048
// elements per workgroup; per-tile digit histograms are scanned digit-major so
// that each tile writes its elements of digit d after all earlier tiles'.
constexpr int kRsThreads = 256;
constexpr int kRsItems = 8;
constexpr uint32_t kRsTile = kRsThreads * kRsItems;

__global__ __launch_bounds__(kRsThreads) void k_rs_hist(const uint32_t* __restrict__ keys,
                                                        uint32_t n, uint32_t shift,
                                                        uint32_t* __restrict__ hist) {
    __shared__ uint32_t h[256];
    h[threadIdx.x] = 0;
    __syncthreads();
    const uint64_t base = (uint64_t)blockIdx.x * kRsTile;
    for (int i = 0; i < kRsItems; ++i) {
        uint64_t idx = base + (uint64_t)i * kRsThreads + threadIdx.x;
        if (idx < n) atomicAdd(&h[(keys[idx] >> shift) & 255u], 1u);
    }
    __syncthreads();
    hist[(uint64_t)threadIdx.x * gridDim.x + blockIdx.x] = h[threadIdx.x];
}

// vals == nullptr means value = element index.  The tile is ranked by digit
// (stable: by round, wave and lane, i.e. by index), placed in digit order in
// LDS, and then written out so that consecutive threads write consecutive
// elements of one digit's run (coalesced).
__global__ __launch_bounds__(kRsThreads) void k_rs_scatter(
    const uint32_t* __restrict__ keys, const uint32_t* __restrict__ vals, uint32_t n,
    uint32_t shift, const uint32_t* __restrict__ offs, uint32_t* __restrict__ keys_out,
    uint32_t* __restrict__ vals_out) {
    __shared__ uint32_t sk[kRsTile], sv[kRsTile];
    __shared__ uint32_t gofs[256];  // where this tile's run of each digit starts in the output
    __shared__ uint32_t tofs[256];  // where it starts in the tile
    __shared__ uint32_t loc[256];   // elements of each digit ranked so far
    __shared__ uint32_t wh[kRsThreads / 64][256];
    __shared__ uint32_t wsum[kRsThreads / 64];
    const uint32_t tid = threadIdx.x, lane = lane_id(), wave = tid >> 6;
    gofs[tid] = offs[(uint64_t)tid * gridDim.x + blockIdx.x];
    loc[tid] = 0;
    for (int w = 0; w < kRsThreads / 64; ++w) wh[w][tid] = 0;
    __syncthreads();
    const uint64_t base = (uint64_t)blockIdx.x * kRsTile;
    const u64 lt_mask = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    uint32_t kk[kRsItems], vv[kRsItems], dd[kRsItems], rk[kRsItems];
    for (int r = 0; r < kRsItems; ++r) {
        uint64_t idx = base + (uint64_t)r * kRsThreads + tid;
        bool valid = idx < n;
        uint32_t key = valid ? keys[idx] : 0u;
        uint32_t val = valid ? (vals ? vals[idx] : (uint32_t)idx) : 0u;
        uint32_t d = (key >> shift) & 255u;
        u64 peers = __ballot(valid);
        for (int b = 0; b < 8; ++b) {
            u64 bb = __ballot((d >> b) & 1u);
            peers &= ((d >> b) & 1u) ? bb : ~bb;
        }
        uint32_t lrank = __popcll(peers & lt_mask);
        if (valid && lrank == 0) wh[wave][d] = (uint32_t)__popcll(peers);
        __syncthreads();
        {
            uint32_t run = loc[tid];
            for (int w = 0; w < kRsThreads / 64; ++w) {
                uint32_t c = wh[w][tid];
                wh[w][tid] = run;
                run += c;
            }
            loc[tid] = run;
        }
        __syncthreads();
        kk[r] = key;
        vv[r] = val;
        dd[r] = valid ? d : 256u;
        rk[r] = valid ? wh[wave][d] + lrank : 0u;
        __syncthreads();
        for (int w = 0; w < kRsThreads / 64; ++w) wh[w][tid] = 0;
        __syncthreads();
    }
    // tile-local start of each digit: exclusive scan of the counts
    {
        const uint32_t c = loc[tid];
        const uint32_t inc = wave_incl_scan(c);
        if (lane == 63) wsum[wave] = inc;
        __syncthreads();
        uint32_t add = 0;
        for (uint32_t w = 0; w < wave; ++w) add += wsum[w];
        tofs[tid] = add + inc - c;
    }
    __syncthreads();
    for (int r = 0; r < kRsItems; ++r)
        if (dd[r] < 256u) {
            const uint32_t pos = tofs[dd[r]] + rk[r];
            sk[pos] = kk[r];
            sv[pos] = vv[r];
        }
    __syncthreads();
    const uint32_t in_tile = (uint32_t)min<uint64_t>(kRsTile, n > base ? n - base : 0);
    for (uint32_t i = tid; i < in_tile; i += kRsThreads) {
        const uint32_t key = sk[i];
        const uint32_t d = (key >> shift) & 255u;
        const uint32_t dst = gofs[d] + (i - tofs[d]);
        keys_out[dst] = key;
        vals_out[dst] = sv[i];
    }
}

// ------------------------------------------------------ sides and rows -------
__global__ void k_side_flags(const uint32_t* __restrict__ inv, uint32_t n, uint32_t n_u,
                             uint32_t* __restrict__ flag) {
    for (uint32_t r = blockIdx.x * blockDim.x + threadIdx.x; r < n; r += gridDim.x * blockDim.x)
        flag[r] = inv[r] < n_u ? 1u : 0u;
}

// rank r -> sidx of its vertex, its row, the row's length and cross threshold
__global__ void k_assign(const uint32_t* __restrict__ inv, const uint32_t* __restrict__ cnt_u,
                         const uint32_t* __restrict__ deg, uint32_t n, uint32_t n_u,
                         uint32_t* __restrict__ sidx_of, uint32_t* __restrict__ rowdeg,
                         uint32_t* __restrict__ rowcross) {
    for (uint32_t r = blockIdx.x * blockDim.x + threadIdx.x; r < n; r += gridDim.x * blockDim.x) {
        uint32_t g = inv[r], cu = cnt_u[r];
        uint32_t sidx, cross, row;
        if (g < n_u) {
            sidx = cu;
            cross = r - cu;  // V vertices below r
            row = sidx;
        } else {
            sidx = r - cu;
            cross = cu;      // U vertices below r
            row = n_u + sidx;
        }
        sidx_of[g] = sidx;
        rowdeg[row] = deg[g];
        rowcross[row] = cross;
    }
}

// Per input vertex x: {sidx(x), start of its row}, so that the scatter reads
// one 8-byte entry per endpoint (a random read costs a whole memory sector).
__global__ void k_vertex_pack(const uint32_t* __restrict__ sidx_of,
                              const uint32_t* __restrict__ row_ptr, uint32_t n, uint32_t n_u,
                              uint2* __restrict__ vx) {
    for (uint32_t x = blockIdx.x * blockDim.x + threadIdx.x; x < n; x += gridDim.x * blockDim.x) {
        const uint32_t s = sidx_of[x];
        vx[x] = make_uint2(s, row_ptr[(x < n_u ? 0u : n_u) + s]);
    }
}

// Each edge lands in row u (entry sidx(v)) and row v (entry sidx(u)), at the
// slots the degree pass reserved for it.  A thread takes kScatterPer edges per
// round, each round's loads issued together (a batch's union gives a thread
// about a hundred edges).
constexpr int kScatterPer = 4;

__global__ __launch_bounds__(256) void k_scatter(const int32_t* __restrict__ eu,
                                                 const int32_t* __restrict__ ev,
                                                 const int8_t* __restrict__ sg, uint64_t m,
                                                 uint32_t n_u, uint32_t n_v,
                                                 const uint2* __restrict__ vx,
                                                 const uint2* __restrict__ rank,
                                                 uint32_t* __restrict__ col) {
    // XCD-aware: workgroup b runs on XCD b % 8 (round-robin dispatch); XCD x
    // takes the x-th eighth of the edges, so the rows a batched graph writes
    // are written through one L2
    if (n_u + n_v == 0) return;  // no edge can be valid (and vertex 0 does not exist)
    const uint32_t x = blockIdx.x & 7u, bx = blockIdx.x >> 3, nbx = gridDim.x >> 3;
    const uint64_t e_lo = m * x / 8, e_hi = m * (x + 1) / 8;
    const uint64_t span = (uint64_t)nbx * blockDim.x;
    for (uint64_t e0 = e_lo + (uint64_t)bx * blockDim.x + threadIdx.x; e0 < e_hi;
         e0 += kScatterPer * span) {
        int32_t u[kScatterPer], v[kScatterPer];
        int8_t s[kScatterPer];
        uint2 r[kScatterPer];
#pragma unroll
        for (int q = 0; q < kScatterPer; ++q) {
            const uint64_t e = e0 + q * span;
            const uint64_t ec = e < e_hi ? e : e0;  // (e0 < e_hi)
            u[q] = eu[ec];
            v[q] = ev[ec];
            s[q] = sg[ec];
            r[q] = rank[ec];
        }
        bool ok[kScatterPer];
        uint2 pu[kScatterPer], pv[kScatterPer];  // {sidx, row start}
#pragma unroll
        for (int q = 0; q < kScatterPer; ++q) {  // (an edge left out reads vertex 0)
            ok[q] = e0 + q * span < e_hi && edge_ok(u[q], v[q], s[q], n_u, n_v);
            pu[q] = vx[ok[q] ? (uint32_t)u[q] : 0u];
            pv[q] = vx[ok[q] ? n_u + (uint32_t)v[q] : 0u];
        }
#pragma unroll
        for (int q = 0; q < kScatterPer; ++q) {
            if (!ok[q]) continue;
            const uint32_t neg = s[q] < 0 ? 1u : 0u;
            col[pu[q].y + r[q].x] = (pv[q].x << 1) | neg;
            col[pv[q].y + r[q].y] = (pu[q].x << 1) | neg;
        }
    }
}

// Row lengths are non-decreasing inside each side in the (side, length)
// order of rows (the row order itself for one graph, whose sidx order is
// degree order; the list d.rlist for a batch), so each size class is a
// contiguous range of positions per side.
__global__ void k_classes(const uint32_t* __restrict__ rowdeg, Dims d, Control* ctl) {
    uint32_t t = threadIdx.x;
    if (t >= 2 * kNumClassBounds) return;
    uint32_t side = t / kNumClassBounds, c = t % kNumClassBounds;
    uint32_t lo = d.base[side], hi = d.base[side] + d.size[side];
    uint32_t th = class_hi((int)c);
    while (lo < hi) {
        uint32_t mid = (lo + hi) >> 1;
        if (rowdeg[row_at(d, mid)] <= th)
            lo = mid + 1;
        else
            hi = mid;
    }
    ctl->cls[side][c] = lo;
}

// ---------------------------------------------------------- row sorting ------
// Class ranges, per side: c0 [base, cls0): len <= 1, c1 [cls0, cls1): <= 8,
// c2 <= 16, c3 <= 32, c4 <= 64, c5 (64, 4096], c6 > 4096.
__device__ inline void class_range(const Control* ctl, const Dims& d, int side, int c0, int c1,
                                   uint32_t* lo, uint32_t* hi) {
    *lo = c0 == 0 ? d.base[side] : ctl->cls[side][c0 - 1];
    *hi = c1 >= kNumClassBounds ? d.base[side] + d.size[side] : ctl->cls[side][c1];
}

__device__ inline void cswap(uint32_t& a, uint32_t& b) {
    uint32_t x = min(a, b), y = max(a, b);
    a = x;
    b = y;
}

// rows with len <= 8: one thread per row, 8-input sorting network in registers
__global__ void k_sort_tiny(const uint32_t* __restrict__ row_ptr, const uint32_t* __restrict__ in,
                            uint32_t* __restrict__ out, Dims d, Control* ctl) {
    uint32_t lo0, hi0, lo1, hi1;
    class_range(ctl, d, 0, 0, 1, &lo0, &hi0);
    class_range(ctl, d, 1, 0, 1, &lo1, &hi1);
    uint32_t n0 = hi0 - lo0, tot = n0 + (hi1 - lo1);
    bool dup = false;
    for (uint32_t q = blockIdx.x * blockDim.x + threadIdx.x; q < tot; q += gridDim.x * blockDim.x) {
        uint32_t r = row_at(d, q < n0 ? lo0 + q : lo1 + (q - n0));
        uint32_t a = row_ptr[r], L = row_ptr[r + 1] - a;
        uint32_t x[8];
#pragma unroll
        for (int i = 0; i < 8; ++i) x[i] = (uint32_t)i < L ? in[a + i] : kEmpty;
        // Batcher odd-even merge sort network for 8 inputs (19 comparators)
        cswap(x[0], x[1]); cswap(x[2], x[3]); cswap(x[4], x[5]); cswap(x[6], x[7]);
        cswap(x[0], x[2]); cswap(x[1], x[3]); cswap(x[4], x[6]); cswap(x[5], x[7]);
        cswap(x[1], x[2]); cswap(x[5], x[6]);
        cswap(x[0], x[4]); cswap(x[1], x[5]); cswap(x[2], x[6]); cswap(x[3], x[7]);
        cswap(x[2], x[4]); cswap(x[3], x[5]);
        cswap(x[1], x[2]); cswap(x[3], x[4]); cswap(x[5], x[6]);
#pragma unroll
        for (int i = 0; i < 8; ++i) {
            if ((uint32_t)i < L) {
                out[a + i] = x[i];
                if (i > 0 && (x[i] >> 1) == (x[i - 1] >> 1)) dup = true;
            }
        }
    }
    if (dup) atomicOr(&ctl->dup, 1u);
}

// rows with G/2 < len <= G (G = 16, 32, 64): G lanes per row, bitonic sort
// across the lanes with shuffles.
template <int G>
__global__ __launch_bounds__(256) void k_sort_group(const uint32_t* __restrict__ row_ptr,
                                                    const uint32_t* __restrict__ in,
                                                    uint32_t* __restrict__ out, Dims d,
                                                    Control* ctl) {
    constexpr int cls = G == 16 ? 2 : (G == 32 ? 3 : 4);
    uint32_t lo0, hi0, lo1, hi1;
    class_range(ctl, d, 0, cls, cls, &lo0, &hi0);
    class_range(ctl, d, 1, cls, cls, &lo1, &hi1);
    uint32_t n0 = hi0 - lo0, tot = n0 + (hi1 - lo1);
    const uint32_t gl = threadIdx.x & (G - 1);
    const uint32_t groups_per_block = blockDim.x / G;
    const uint32_t gid = blockIdx.x * groups_per_block + threadIdx.x / G;
    const uint32_t gstride = gridDim.x * groups_per_block;
    bool dup = false;
    // every lane of a wave runs the same number of iterations (uniform bound)
    const uint32_t iters = (tot + gstride - 1) / gstride;
    for (uint32_t it = 0; it < iters; ++it) {
        uint32_t q = gid + it * gstride;
        bool act = q < tot;
        uint32_t r = act ? row_at(d, q < n0 ? lo0 + q : lo1 + (q - n0)) : 0;
        uint32_t a = act ? row_ptr[r] : 0, L = act ? row_ptr[r + 1] - a : 0;
        uint32_t v = gl < L ? in[a + gl] : kEmpty;
#pragma unroll
        for (int k = 2; k <= G; k <<= 1) {
#pragma unroll
            for (int j = k >> 1; j > 0; j >>= 1) {
                uint32_t o = __shfl_xor(v, j, 64);
                bool asc = (gl & k) == 0;
                bool low = (gl & j) == 0;
                v = (low == asc) ? min(v, o) : max(v, o);
            }
        }
        uint32_t prev = __shfl_up(v, 1, 64);
        if (gl < L) {
            out[a + gl] = v;
            if (gl > 0 && (prev >> 1) == (v >> 1)) dup = true;
        }
    }
    if (dup) atomicOr(&ctl->dup, 1u);
}

// Entries of a row are per-side indices of the other side; in a batch they lie
// in the row's graph's block of that side.
__device__ inline void entry_range(const Dims& d, uint32_t r, uint32_t* lo, uint32_t* hi) {
    const uint32_t side = r >= d.n_u ? 1u : 0u;
    if (d.blk[0]) {
        const uint32_t g = block_of(d.blk[side], d.n_graphs, r - d.base[side]);
        *lo = d.blk[side ^ 1u][g];
        *hi = d.blk[side ^ 1u][g + 1];
    } else {
        *lo = 0;
        *hi = d.size[side ^ 1u];
    }
}

// Emits the set bits of an LDS bitmap (bit y: entry (lo + y) << 1 | sign) in
// order to out[base ..), each thread owning `per` consecutive words, and fills
// [base + set bits, base + want) with copies of the last entry: fewer bits than
// entries means a repeated neighbour, and the copies keep every entry in range
// and the repetition visible to the per-graph duplicate check.  Returns after a
// barrier; s_scan needs blockDim / 64 words.
__device__ inline void bitmap_emit(const uint32_t* bm, const uint32_t* sg, uint32_t words,
                                   uint32_t per, uint32_t lo, uint32_t* __restrict__ out,
                                   uint64_t base, uint32_t want, uint32_t* s_scan,
                                   uint32_t* s_last) {
    const uint32_t tid = threadIdx.x, lane = lane_id(), wave = tid >> 6;
    const uint32_t nw = blockDim.x >> 6;
    const uint32_t w0 = tid * per, w1 = min(words, w0 + per);
    uint32_t cnt = 0, last = 0;  // last: 1 + highest set bit of this thread's words
    for (uint32_t i = w0; i < w1; ++i) {
        cnt += __popc(bm[i]);
        if (bm[i]) last = i * 32 + (32 - __clz(bm[i]));
    }
    const uint32_t incl = wave_incl_scan(cnt);
    for (uint32_t off = 32; off > 0; off >>= 1) last = max(last, __shfl_xor(last, off, 64));
    if (lane == 63) s_scan[wave] = incl;
    if (lane == 0) atomicMax(s_last, last);
    __syncthreads();
    uint32_t off = 0, total = 0;
    for (uint32_t w = 0; w < nw; ++w) {
        if (w < wave) off += s_scan[w];
        total += s_scan[w];
    }
    uint64_t pos = base + off + incl - cnt;
    for (uint32_t i = w0; i < w1; ++i) {
        uint32_t bits = bm[i];
        while (bits) {
            const uint32_t bt = __ffs(bits) - 1;
            if (pos < base + want) out[pos] = ((lo + i * 32 + bt) << 1) | ((sg[i] >> bt) & 1u);
            ++pos;
            bits &= bits - 1;
        }
    }
    if (total < want && *s_last > 0) {
        const uint32_t y = *s_last - 1;
        const uint32_t v = ((lo + y) << 1) | ((sg[y >> 5] >> (y & 31)) & 1u);
        for (uint32_t i = total + tid; i < want; i += blockDim.x) out[base + i] = v;
    }
    __syncthreads();
}

// rows with 64 < len <= 4096 whose entries span at most kMidBits indices
// (every row of a batch): one wave per row, an LDS bitmap (plus a sign bitmap)
// per wave, no workgroup barriers.  A repeated neighbour leaves fewer bits than
// entries; the row's remaining slots get copies of its last entry, as in
// bitmap_emit.
constexpr uint32_t kMidBits = 16384;
constexpr uint32_t kMidWords = kMidBits / 32;

__global__ __launch_bounds__(256) void k_sort_mid_bitmap(const uint32_t* __restrict__ row_ptr,
                                                        const uint32_t* __restrict__ in,
                                                        uint32_t* __restrict__ out, Dims d,
                                                        Control* ctl) {
    __shared__ uint32_t s_bm[4][kMidWords];
    __shared__ uint32_t s_sg[4][kMidWords];
    const uint32_t lane = lane_id(), wave = threadIdx.x >> 6;
    uint32_t* bm = s_bm[wave];
    uint32_t* sg = s_sg[wave];
    uint32_t lo0, hi0, lo1, hi1;
    class_range(ctl, d, 0, 5, 5, &lo0, &hi0);
    class_range(ctl, d, 1, 5, 5, &lo1, &hi1);
    const uint32_t n0 = hi0 - lo0, tot = n0 + (hi1 - lo1);
    bool dup = false;
    for (uint32_t q = blockIdx.x * 4 + wave; q < tot; q += gridDim.x * 4) {
        const uint32_t r = row_at(d, q < n0 ? lo0 + q : lo1 + (q - n0));
        uint32_t elo, ehi;
        entry_range(d, r, &elo, &ehi);
        const uint32_t R = ehi - elo;
        if (R > kMidBits) continue;  // k_sort_wave or k_sort_block sorts this row
        const uint32_t a = row_ptr[r], L = row_ptr[r + 1] - a;
        const uint32_t words = (R + 31) / 32;
        for (uint32_t i = lane; i < words; i += 64) {
            bm[i] = 0;
            sg[i] = 0;
        }
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        for (uint32_t i0 = 0; i0 < L; i0 += 4 * 64) {
            uint32_t xs[4];
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                const uint32_t i = i0 + k * 64 + lane;
                xs[k] = i < L ? in[a + i] : 0u;
            }
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                if (i0 + k * 64 + lane >= L) continue;
                const uint32_t x = xs[k];
                const uint32_t y = (x >> 1) - elo;
                if (y >= R) continue;  // cannot happen: entries lie in the block
                const uint32_t msk = 1u << (y & 31);
                if (atomicOr(&bm[y >> 5], msk) & msk) dup = true;
                if (x & 1u) atomicOr(&sg[y >> 5], msk);
            }
        }
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        // lane owns words [w0, w1); emit in order after a wave scan of counts
        const uint32_t per = (words + 63) / 64;
        const uint32_t w0 = lane * per, w1 = min(words, w0 + per);
        uint32_t cnt = 0, last = 0;  // last: 1 + highest set bit
        for (uint32_t i = w0; i < w1; ++i) {
            cnt += __popc(bm[i]);
            if (bm[i]) last = i * 32 + (32 - __clz(bm[i]));
        }
        const uint32_t incl = wave_incl_scan(cnt);
        const uint32_t total = __shfl(incl, 63, 64);
        for (uint32_t off = 32; off > 0; off >>= 1) last = max(last, __shfl_xor(last, off, 64));
        uint32_t pos = incl - cnt;
        for (uint32_t i = w0; i < w1; ++i) {
            uint32_t bits = bm[i];
            while (bits) {
                const uint32_t bt = __ffs(bits) - 1;
                if (pos < L) out[a + pos] = ((elo + i * 32 + bt) << 1) | ((sg[i] >> bt) & 1u);
                ++pos;
                bits &= bits - 1;
            }
        }
        if (total < L && last > 0) {
            const uint32_t y = last - 1;
            const uint32_t v = ((elo + y) << 1) | ((sg[y >> 5] >> (y & 31)) & 1u);
            for (uint32_t i = total + lane; i < L; i += 64) out[a + i] = v;
        }
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    }
    if (dup) atomicOr(&ctl->dup, 1u);
}

// rows with 64 < len <= kWaveRowMax whose entries span more than kMidBits
// indices: one wave per row, a bitonic sort in registers.  Lane l holds the
// row's entries l, 64 + l, ... (padded with kEmpty, above every entry); a
// compare-exchange at distance j >= 64 stays in the lane, one at j < 64 takes a
// shuffle.  No LDS and no barriers.
constexpr uint32_t kWaveRowMax = 1024;

// One compare-exchange step of a bitonic network (block size k, distance j)
// over the wave's 64 * E entries, which are entries gbase + r * 64 + lane of
// the whole sequence (so the direction follows the global index).
template <int E>
__device__ inline void wave_bitonic_step(uint32_t (&x)[E], uint32_t lane, uint32_t gbase,
                                         uint32_t k, uint32_t j) {
    if (j >= 64) {
#pragma unroll
        for (int r = 0; r < E; ++r) {
            const int r2 = r ^ (int)(j >> 6);
            if (r2 > r) {
                const bool asc = ((gbase + r * 64u + lane) & k) == 0;
                const uint32_t lo = min(x[r], x[r2]), hi = max(x[r], x[r2]);
                x[r] = asc ? lo : hi;
                x[r2] = asc ? hi : lo;
            }
        }
    } else {
#pragma unroll
        for (int r = 0; r < E; ++r) {
            const uint32_t o = __shfl_xor(x[r], (int)j, 64);
            const bool asc = ((gbase + r * 64u + lane) & k) == 0;
            const bool low = (lane & j) == 0;
            x[r] = (low == asc) ? min(x[r], o) : max(x[r], o);
        }
    }
}

// all blocks k <= 64 * E: sorts the wave's entries, ascending when gbase is
// an even multiple of 64 * E, descending when an odd one
template <int E>
__device__ inline void wave_bitonic(uint32_t (&x)[E], uint32_t lane, uint32_t gbase = 0) {
#pragma unroll
    for (uint32_t k = 2; k <= 64u * E; k <<= 1) {
#pragma unroll
        for (uint32_t j = k >> 1; j > 0; j >>= 1) wave_bitonic_step<E>(x, lane, gbase, k, j);
    }
}

// the steps of block size k (> 64 * E) with distance below 64 * E
template <int E>
__device__ inline void wave_bitonic_merge(uint32_t (&x)[E], uint32_t lane, uint32_t gbase,
                                          uint32_t k) {
#pragma unroll
    for (uint32_t j = 32u * E; j > 0; j >>= 1) wave_bitonic_step<E>(x, lane, gbase, k, j);
}

template <int E>
__device__ inline bool wave_sort_row(const uint32_t* __restrict__ in, uint32_t* __restrict__ out,
                                     uint32_t a, uint32_t L, uint32_t lane) {
    uint32_t x[E];
#pragma unroll
    for (int r = 0; r < E; ++r) {
        const uint32_t i = r * 64u + lane;
        x[r] = i < L ? in[a + i] : kEmpty;
    }
    wave_bitonic<E>(x, lane);
    bool dup = false;
#pragma unroll
    for (int r = 0; r < E; ++r) {
        const uint32_t i = r * 64u + lane;
        uint32_t prev = __shfl_up(x[r], 1, 64);
        if (r > 0) {
            const uint32_t last = __shfl(x[r > 0 ? r - 1 : 0], 63, 64);
            if (lane == 0) prev = last;
        }
        if (i < L) {
            out[a + i] = x[r];
            if (i > 0 && (prev >> 1) == (x[r] >> 1)) dup = true;
        }
    }
    return dup;
}

__global__ __launch_bounds__(256) void k_sort_wave(const uint32_t* __restrict__ row_ptr,
                                                  const uint32_t* __restrict__ in,
                                                  uint32_t* __restrict__ out, Dims d,
                                                  Control* ctl) {
    const uint32_t lane = lane_id(), wave = threadIdx.x >> 6;
    uint32_t lo0, hi0, lo1, hi1;
    class_range(ctl, d, 0, 5, 5, &lo0, &hi0);
    class_range(ctl, d, 1, 5, 5, &lo1, &hi1);
    const uint32_t n0 = hi0 - lo0, tot = n0 + (hi1 - lo1);
    bool dup = false;
    for (uint32_t q = blockIdx.x * 4 + wave; q < tot; q += gridDim.x * 4) {
        const uint32_t r = row_at(d, q < n0 ? lo0 + q : lo1 + (q - n0));
        const uint32_t a = row_ptr[r], L = row_ptr[r + 1] - a;
        if (L > kWaveRowMax) continue;  // k_sort_block sorts this row
        uint32_t elo, ehi;
        entry_range(d, r, &elo, &ehi);
        if (ehi - elo <= kMidBits) continue;  // k_sort_mid_bitmap sorts this row
        if (L <= 128)
            dup |= wave_sort_row<2>(in, out, a, L, lane);
        else if (L <= 256)
            dup |= wave_sort_row<4>(in, out, a, L, lane);
        else if (L <= 512)
            dup |= wave_sort_row<8>(in, out, a, L, lane);
        else
            dup |= wave_sort_row<16>(in, out, a, L, lane);
    }
    if (dup) atomicOr(&ctl->dup, 1u);
}

// rows with kWaveRowMax < len <= 4096 whose entries span more than kMidBits
// indices: one workgroup per row, a bitonic sort of P = 2^ceil(log2 len)
// entries (padded with kEmpty).  Each wave holds a chunk of 256 entries in
// registers for the steps of distance below 256 (first the whole chunk sort,
// then after each block size's larger-distance steps, which run in LDS with a
// barrier each): about 10 barriers per row instead of 78.
constexpr int kBlockSortThreads = 1024;
constexpr uint32_t kSortChunk = 256;  // 4 entries per lane

__global__ __launch_bounds__(kBlockSortThreads) void k_sort_block(const uint32_t* __restrict__ row_ptr,
                                                                  const uint32_t* __restrict__ in,
                                                                  uint32_t* __restrict__ out, Dims d,
                                                                  Control* ctl) {
    static_assert(kBlockSortThreads / 64 * kSortChunk >= 4096, "a chunk per wave covers a row");
    __shared__ uint32_t s[4096];
    const uint32_t tid = threadIdx.x, lane = lane_id(), wave = tid >> 6;
    uint32_t lo0, hi0, lo1, hi1;
    class_range(ctl, d, 0, 5, 5, &lo0, &hi0);
    class_range(ctl, d, 1, 5, 5, &lo1, &hi1);
    uint32_t n0 = hi0 - lo0, tot = n0 + (hi1 - lo1);
    bool dup = false;
    for (uint32_t q = blockIdx.x; q < tot; q += gridDim.x) {
        uint32_t r = row_at(d, q < n0 ? lo0 + q : lo1 + (q - n0));
        uint32_t a = row_ptr[r], L = row_ptr[r + 1] - a;
        if (L <= kWaveRowMax) continue;  // k_sort_wave or k_sort_mid_bitmap sorts this row
        uint32_t elo, ehi;
        entry_range(d, r, &elo, &ehi);
        if (ehi - elo <= kMidBits) continue;  // k_sort_mid_bitmap sorts this row
        uint32_t P = kSortChunk;
        while (P < L) P <<= 1;
        const bool mine = wave * kSortChunk < P;  // this wave holds a chunk
        const uint32_t gbase = wave * kSortChunk;
        uint32_t x[kSortChunk / 64];
        if (mine) {
#pragma unroll
            for (int k = 0; k < (int)(kSortChunk / 64); ++k) {
                const uint32_t i = gbase + k * 64u + lane;
                x[k] = i < L ? in[a + i] : kEmpty;
            }
            wave_bitonic<kSortChunk / 64>(x, lane, gbase);
#pragma unroll
            for (int k = 0; k < (int)(kSortChunk / 64); ++k) s[gbase + k * 64u + lane] = x[k];
        }
        __syncthreads();
        for (uint32_t k = 2 * kSortChunk; k <= P; k <<= 1) {
            for (uint32_t j = k >> 1; j >= kSortChunk; j >>= 1) {
                for (uint32_t i = tid; i < P; i += kBlockSortThreads) {
                    const uint32_t ij = i ^ j;
                    if (ij > i) {
                        const uint32_t xa = s[i], ya = s[ij];
                        const bool asc = (i & k) == 0;
                        if ((xa > ya) == asc) {
                            s[i] = ya;
                            s[ij] = xa;
                        }
                    }
                }
                __syncthreads();
            }
            if (mine) {
#pragma unroll
                for (int kk = 0; kk < (int)(kSortChunk / 64); ++kk) x[kk] = s[gbase + kk * 64u + lane];
                wave_bitonic_merge<kSortChunk / 64>(x, lane, gbase, k);
#pragma unroll
                for (int kk = 0; kk < (int)(kSortChunk / 64); ++kk) s[gbase + kk * 64u + lane] = x[kk];
            }
            __syncthreads();
        }
        for (uint32_t i = tid; i < L; i += kBlockSortThreads) {
            uint32_t v = s[i];
            out[a + i] = v;
            if (i > 0 && (s[i - 1] >> 1) == (v >> 1)) dup = true;
        }
        __syncthreads();
    }
    if (dup) atomicOr(&ctl->dup, 1u);
}

// rows with len > 4096: one workgroup per (row, sidx chunk of 2^18): mark the
// row's entries of the chunk in an LDS bitmap (plus a sign bitmap), then emit
// the set bits in order.  Entries are distinct unless an edge is repeated,
// which the bitmap detects.
constexpr int kBigThreads = 1024;
constexpr uint32_t kBigWords = kBitmapChunk / 32;

__device__ inline void big_pair(const Control* ctl, const Dims& d, uint32_t q, uint32_t* row,
                                uint32_t* chunk, uint32_t* ok) {
    // side 0 big rows (entries index side 1), then side 1 big rows
    uint32_t b0 = ctl->cls[0][5], e0 = d.base[0] + d.size[0];
    uint32_t b1 = ctl->cls[1][5], e1 = d.base[1] + d.size[1];
    uint32_t ch0 = (d.size[1] + kBitmapChunk - 1) / kBitmapChunk;
    uint32_t ch1 = (d.size[0] + kBitmapChunk - 1) / kBitmapChunk;
    uint32_t np0 = (e0 - b0) * ch0, np1 = (e1 - b1) * ch1;
    *ok = 1;
    if (q < np0) {
        *row = row_at(d, b0 + q / ch0);
        *chunk = q % ch0;
    } else if (q - np0 < np1) {
        q -= np0;
        *row = row_at(d, b1 + q / ch1);
        *chunk = q % ch1;
    } else {
        *ok = 0;
    }
}

__global__ __launch_bounds__(kBigThreads) void k_sort_big(const uint32_t* __restrict__ row_ptr,
                                                          const uint32_t* __restrict__ in,
                                                          uint32_t* __restrict__ out, Dims d,
                                                          Control* ctl) {
    __shared__ uint32_t bm[kBigWords];
    __shared__ uint32_t sgn[kBigWords];
    __shared__ uint32_t s_wave[kBigThreads / 64];
    __shared__ uint32_t s_before, s_inside, s_last;
    const uint32_t tid = threadIdx.x, lane = lane_id();
    bool dup = false;
    for (uint32_t q = blockIdx.x;; q += gridDim.x) {
        uint32_t r, c, ok;
        big_pair(ctl, d, q, &r, &c, &ok);
        if (!ok) break;
        for (uint32_t i = tid; i < kBigWords; i += kBigThreads) {
            bm[i] = 0;
            sgn[i] = 0;
        }
        if (tid == 0) {
            s_before = 0;
            s_inside = 0;
            s_last = 0;
        }
        __syncthreads();
        const uint32_t a = row_ptr[r], L = row_ptr[r + 1] - a;
        const uint32_t c0 = c * kBitmapChunk;
        uint32_t before = 0, inside = 0;  // entries below this chunk / in it (with repeats)
        constexpr int kLoads = 8;  // entries loaded together per thread
        for (uint32_t e0 = 0; e0 < L; e0 += kLoads * kBigThreads) {
            uint32_t xs[kLoads];
#pragma unroll
            for (int k = 0; k < kLoads; ++k) {
                const uint32_t e = e0 + k * kBigThreads + tid;
                xs[k] = e < L ? in[a + e] : 0u;
            }
#pragma unroll
            for (int k = 0; k < kLoads; ++k) {
                if (e0 + k * kBigThreads + tid >= L) continue;
                const uint32_t x = xs[k], y = x >> 1;
                if (y < c0) {
                    before++;
                } else if (y - c0 < kBitmapChunk) {
                    inside++;
                    const uint32_t bit = y - c0;
                    const uint32_t m = 1u << (bit & 31);
                    const uint32_t old = atomicOr(&bm[bit >> 5], m);
                    if (old & m) dup = true;
                    if (x & 1u) atomicOr(&sgn[bit >> 5], m);
                }
            }
        }
        before = wave_reduce_sum(before);
        inside = wave_reduce_sum(inside);
        if (lane == 0) {
            atomicAdd(&s_before, before);
            atomicAdd(&s_inside, inside);
        }
        __syncthreads();
        // this chunk's entries take [a + s_before, a + s_before + s_inside)
        bitmap_emit(bm, sgn, kBigWords, kBigWords / kBigThreads, c0, out, (uint64_t)a + s_before,
                    min(s_inside, L - min(L, s_before)), s_wave, &s_last);
    }
    if (dup) atomicOr(&ctl->dup, 1u);
}

// --------------------------------------------------- lower neighbour counts --
// k_r (entries below the row's own priority: its middles) and the rest (its
// upper entries, each the middle of a record of a higher start)
__global__ void k_lowcount(const uint32_t* __restrict__ row_ptr, const uint32_t* __restrict__ col,
                           const uint32_t* __restrict__ rowcross, uint32_t n,
                           uint32_t* __restrict__ lowcnt) {
    for (uint32_t r = blockIdx.x * blockDim.x + threadIdx.x; r < n; r += gridDim.x * blockDim.x) {
        uint32_t a = row_ptr[r], L = row_ptr[r + 1] - a;
        const uint32_t k = lower_bound_u32(col + a, L, rowcross[r] << 1);
        lowcnt[r] = k;
    }
}

// ------------------------------------------------------------- records ------
// One record per edge, at its start u (the end of higher priority).  The first
// k_u entries of u's sorted row are its neighbours v of lower priority, the
// middles, in ascending priority; entry j takes the slot mptr[u] + k_u - 1 - j,
// so u's records run from its highest-priority middle down.  Priority is
// (degree, id), so the middles with long rows (more than kLongDeg entries)
// come first and the short ones end the run; front[u] is u's first short
// record (preset to mptr[u+1]: none).  pos_v(u), the number of entries of v's
// sorted row before u (exactly v's neighbours of lower priority than u, the
// wedge ends of Algorithm 2 through v), comes from a binary search for u in
// v's row (a middle has lower priority, so mostly a short row).  W_u and Ws_u (the wedges
// through short middle rows) are sums of pos over u's records, aggregated per
// workgroup in an LDS table (a hub's records span many threads).
//   .x = first entry of row v, .y = pos << 1 | neg(u, v), .z = sidx(v), .w = row u
//
// A thread takes kRecPer consecutive CSR entries and a wave 64 * kRecPer; the
// rows of a wave's first and last entry bound those of the others.  The
// searches of a thread's records step together, so their loads overlap.
constexpr int kRecPer = 4;  // consecutive entries per thread
constexpr int kRecThreads = 256;
constexpr uint32_t kRecLog2 = 10;
constexpr uint32_t kRecSlots = 1u << kRecLog2;

__global__ __launch_bounds__(kRecThreads) void k_records(
    const uint32_t* __restrict__ row_ptr, const uint32_t* __restrict__ col,
    const uint32_t* __restrict__ lowcnt, const uint32_t* __restrict__ mptr, Dims d, uint64_t m,
    uint4* __restrict__ recs, u64* __restrict__ wu, u64* __restrict__ wsu,
    uint32_t* __restrict__ front) {
    __shared__ uint32_t keys[kRecSlots];
    __shared__ u64 sw[kRecSlots], ss[kRecSlots];
    __shared__ uint32_t sf[kRecSlots];
    const uint32_t tid = threadIdx.x, lane = lane_id();
    const uint32_t nnz = row_ptr[d.n];  // entries actually placed (invalid edges are not)
    // slots past the last start's records (invalid edges leave some) hold
    // harmless empty records
    for (uint64_t j = (uint64_t)mptr[d.n] + (uint64_t)blockIdx.x * kRecThreads + tid; j < m;
         j += (uint64_t)gridDim.x * kRecThreads)
        recs[j] = make_uint4(0, 0, 0, 0);
    constexpr uint32_t kSpan = 64 * kRecPer;
    const uint32_t nwaves = gridDim.x * (kRecThreads / 64);
    // (64-bit positions: nnz may come within a span of 2^32)
    for (uint64_t s0 = (uint64_t)(blockIdx.x * (kRecThreads / 64) + (tid >> 6)) * kSpan;;
         s0 += (uint64_t)nwaves * kSpan) {
        // (uniform over the workgroup: its waves' spans are adjacent)
        const uint64_t blk0 = s0 - (uint64_t)(tid >> 6) * kSpan;
        if (blk0 >= nnz) break;
        for (uint32_t i = tid; i < kRecSlots; i += kRecThreads) {
            keys[i] = kEmpty;
            sw[i] = 0;
            ss[i] = 0;
            sf[i] = kEmpty;
        }
        __syncthreads();
        if (s0 < nnz) {
            const uint32_t rlo = wave_block_of(row_ptr, d.n, (uint32_t)s0);
            const uint32_t rhi =
                wave_block_of(row_ptr, d.n, (uint32_t)(min<uint64_t>(s0 + kSpan, nnz) - 1));
            const uint64_t e0 = s0 + lane * kRecPer;
            // this thread's entries: row, middle, slot; then the searches
            uint32_t rs[kRecPer], len[kRecPer], key[kRecPer], slot[kRecPer], urow[kRecPer];
            uint32_t x[kRecPer], pos[kRecPer];
            bool rec[kRecPer];  // entry q is a record with its fields set
#pragma unroll
            for (int q = 0; q < kRecPer; ++q) rec[q] = false;
            if (e0 < nnz) {
                uint32_t r = rlo, hi = rhi + 1;  // row_ptr[r] <= e0 < row_ptr[hi]
                while (hi - r > 1) {
                    const uint32_t mid = (r + hi) >> 1;
                    if (row_ptr[mid] <= e0)
                        r = mid;
                    else
                        hi = mid;
                }
                uint32_t ra = row_ptr[r], rb = row_ptr[r + 1], k = lowcnt[r];
#pragma unroll
                for (int q = 0; q < kRecPer; ++q) {
                    const uint64_t e = e0 + q;
                    if (e >= nnz) continue;
                    while (rb <= e) {  // (rows without entries are passed over)
                        ++r;
                        ra = rb;
                        rb = row_ptr[r + 1];
                        k = lowcnt[r];
                    }
                    const uint32_t jj = (uint32_t)(e - ra);
                    if (jj >= k) continue;  // an upper entry: a record of the other end
                    const uint32_t side = r >= d.n_u ? 1u : 0u;
                    x[q] = col[e];
                    urow[q] = r;
                    slot[q] = mptr[r] + (k - 1u - jj);
                    key[q] = (r - d.base[side]) << 1;  // u's entry in v's row, sign cleared
                    const uint32_t sv = x[q] >> 1;
                    if (sv >= d.size[side ^ 1u] || slot[q] >= m) {  // only with invalid input
                        if (slot[q] < m) recs[slot[q]] = make_uint4(0, 0, 0, 0);
                        continue;
                    }
                    const uint32_t vrow = d.base[side ^ 1u] + sv;
                    rs[q] = row_ptr[vrow];
                    len[q] = row_ptr[vrow + 1] - rs[q];
                    rec[q] = true;
                }
            }
            // lower bounds of key in the rows of the middles, all at once
            {
                uint32_t lo[kRecPer], n[kRecPer];
                bool any = false;
#pragma unroll
                for (int q = 0; q < kRecPer; ++q) {
                    lo[q] = 0;
                    n[q] = rec[q] ? len[q] : 0u;
                    any |= n[q] > 0;
                }
                while (any) {
                    any = false;
#pragma unroll
                    for (int q = 0; q < kRecPer; ++q) {
                        if (n[q] == 0) continue;
                        const uint32_t h = n[q] >> 1;
                        if (col[rs[q] + lo[q] + h] < key[q]) {
                            lo[q] += h + 1;
                            n[q] -= h + 1;
                        } else {
                            n[q] = h;
                        }
                        any |= n[q] > 0;
                    }
                }
#pragma unroll
                for (int q = 0; q < kRecPer; ++q) pos[q] = lo[q];
            }
            // write the records; sums per start, flushed when the start changes
            uint32_t cur = kEmpty, f = kEmpty;
            u64 accW = 0, accS = 0;
            auto flush = [&]() {
                if (cur == kEmpty) return;
                const int sl = agg_slot<kRecLog2>(keys, cur);
                if (sl >= 0) {
                    if (accW) atomicAdd(&sw[sl], accW);
                    if (accS) atomicAdd(&ss[sl], accS);
                    if (f != kEmpty) atomicMin(&sf[sl], f);
                } else {
                    if (accW) atomicAdd(&wu[cur], accW);
                    if (accS) atomicAdd(&wsu[cur], accS);
                    if (f != kEmpty) atomicMin(&front[cur], f);
                }
            };
#pragma unroll
            for (int q = 0; q < kRecPer; ++q) {
                if (!rec[q]) continue;
                const uint32_t sv = x[q] >> 1;
                recs[slot[q]] = make_uint4(rs[q], (pos[q] << 1) | (x[q] & 1u), sv, urow[q]);
                if (urow[q] != cur) {
                    flush();
                    cur = urow[q];
                    accW = accS = 0;
                    f = kEmpty;
                }
                accW += pos[q];
                if (len[q] <= kLongDeg) {
                    accS += pos[q];
                    f = min(f, slot[q]);
                }
            }
            flush();
        }
        __syncthreads();
        for (uint32_t i = tid; i < kRecSlots; i += kRecThreads)
            if (keys[i] != kEmpty) {
                if (sw[i]) atomicAdd(&wu[keys[i]], sw[i]);
                if (ss[i]) atomicAdd(&wsu[keys[i]], ss[i]);
                if (sf[i] != kEmpty) atomicMin(&front[keys[i]], sf[i]);
            }
        __syncthreads();
    }
}

// ------------------------------------------------------- tile boundaries ----
// For a long row of side Y (entries: X-side sidx), tb[t] = number of entries
// with sidx < t * kTile, t = 0..ntile[X]; one wave per row.
__global__ __launch_bounds__(256) void k_tile_table(const uint32_t* __restrict__ row_ptr,
                                                    const uint32_t* __restrict__ col, Dims d,
                                                    const Control* ctl, uint32_t* __restrict__ tb) {
    uint32_t lo0 = ctl->cls[0][4], hi0 = d.base[0] + d.size[0];
    uint32_t lo1 = ctl->cls[1][4], hi1 = d.base[1] + d.size[1];
    uint32_t n0 = hi0 - lo0, tot = n0 + (hi1 - lo1);
    const uint32_t lane = lane_id();
    const uint32_t wid = (blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const uint32_t wstride = (gridDim.x * blockDim.x) >> 6;
    for (uint32_t q = wid; q < tot; q += wstride) {
        uint32_t side = q < n0 ? 0u : 1u;     // side Y of the row
        uint32_t r = side == 0 ? lo0 + q : lo1 + (q - n0);
        uint32_t rel = side == 0 ? q : q - n0;
        uint32_t nt = d.ntile[side ^ 1u];
        uint32_t a = row_ptr[r], L = row_ptr[r + 1] - a;
        uint32_t* out = tb + d.tb_off[side] + (uint64_t)rel * (nt + 1);
        for (uint32_t t = lane; t <= nt; t += 64) {
            uint64_t key = (uint64_t)t * kTile;
            out[t] = key >= d.size[side ^ 1u] ? L : lower_bound_u32(col + a, L, (uint32_t)key << 1);
        }
    }
}

// ------------------------------------------------------------- launchers -----
static dim3 grid_n(uint64_t n, uint32_t threads, uint32_t cap = 16384) {
    uint64_t b = (n + threads - 1) / threads;
    if (b > cap) b = cap;
    if (b == 0) b = 1;
    return dim3((unsigned)b);
}

hipError_t launch_degree(const int32_t* eu, const int32_t* ev, const int8_t* sg, uint64_t m,
                         uint32_t n_u, uint32_t n_v, uint32_t* deg, uint2* rank, Control* ctl,
                         hipStream_t st) {
    hipLaunchKernelGGL(k_degree, grid_n(m, kAggChunk, 2048), dim3(kAggThreads), 0, st, eu, ev, sg, m,
                       n_u, n_v, deg, rank, ctl);
    return hipGetLastError();
}

size_t radix_tmp_bytes(uint32_t n) {
    uint32_t nb = (n + kRsTile - 1) / kRsTile;
    if (nb == 0) nb = 1;
    size_t h = (size_t)256 * nb;
    return (2 * h + 1) * sizeof(uint32_t) + scan_tmp_bytes((uint32_t)h) + 1024;
}

// Sorts (keys, index) by key over the low `bits` bits.  Result values (the
// element indices in sorted order) end in *vals_result.
hipError_t radix_sort_by_key(const uint32_t* keys_in, uint32_t n, uint32_t bits, uint32_t* k0,
                             uint32_t* v0, uint32_t* k1, uint32_t* v1, void* tmp, size_t tmp_bytes,
                             uint32_t** vals_result, hipStream_t st, uint32_t** keys_result) {
    uint32_t nb = (n + kRsTile - 1) / kRsTile;
    if (nb == 0) nb = 1;
    uint32_t h = 256 * nb;
    uint32_t* hist = (uint32_t*)tmp;
    uint32_t* offs = hist + h;
    void* stmp = (void*)(offs + h + 1);
    size_t stmp_bytes = tmp_bytes - (2 * (size_t)h + 1) * sizeof(uint32_t);
    uint32_t passes = (bits + 7) / 8;
    if (passes == 0) passes = 1;
    const uint32_t* kin = keys_in;
    const uint32_t* vin = nullptr;
    uint32_t *ko = k0, *vo = v0;
    for (uint32_t p = 0; p < passes; ++p) {
        uint32_t shift = 8 * p;
        hipLaunchKernelGGL(k_rs_hist, dim3(nb), dim3(kRsThreads), 0, st, kin, n, shift, hist);
        hipError_t e = scan_excl_u32(hist, offs, h, stmp, stmp_bytes, st);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(k_rs_scatter, dim3(nb), dim3(kRsThreads), 0, st, kin, vin, n, shift,
                           (const uint32_t*)offs, ko, vo);
        kin = ko;
        vin = vo;
        *vals_result = vo;
        if (keys_result) *keys_result = ko;
        if (ko == k0) {
            ko = k1;
            vo = v1;
        } else {
            ko = k0;
            vo = v0;
        }
    }
    return hipGetLastError();
}

hipError_t launch_sides(const uint32_t* inv, uint32_t n, uint32_t n_u, uint32_t* flag,
                        hipStream_t st) {
    hipLaunchKernelGGL(k_side_flags, grid_n(n, 256), dim3(256), 0, st, inv, n, n_u, flag);
    return hipGetLastError();
}

hipError_t launch_assign(const uint32_t* inv, const uint32_t* cnt_u, const uint32_t* deg,
                         uint32_t n, uint32_t n_u, uint32_t* sidx_of, uint32_t* rowdeg,
                         uint32_t* rowcross, hipStream_t st) {
    hipLaunchKernelGGL(k_assign, grid_n(n, 256), dim3(256), 0, st, inv, cnt_u, deg, n, n_u, sidx_of,
                       rowdeg, rowcross);
    return hipGetLastError();
}

hipError_t launch_scatter(const int32_t* eu, const int32_t* ev, const int8_t* sg, uint64_t m,
                          uint32_t n_u, uint32_t n_v, const uint32_t* sidx_of,
                          const uint32_t* row_ptr, const uint2* rank, uint2* vx, uint32_t* col,
                          hipStream_t st) {
    const uint32_t n = n_u + n_v;
    hipLaunchKernelGGL(k_vertex_pack, grid_n(n, 256), dim3(256), 0, st, sidx_of, row_ptr, n, n_u,
                       vx);
    hipLaunchKernelGGL(k_scatter, dim3((grid_n(m, 256 * kScatterPer).x + 7) & ~7u), dim3(256), 0, st,
                       eu, ev, sg,
                       m, n_u, n_v,
                       (const uint2*)vx, rank, col);
    return hipGetLastError();
}

hipError_t launch_row_sort(const uint32_t* rowdeg, const uint32_t* row_ptr, const uint32_t* in,
                           uint32_t* out, Dims d, Control* ctl, uint32_t num_cus, hipStream_t st) {
    hipLaunchKernelGGL(k_classes, dim3(1), dim3(64), 0, st, rowdeg, d, ctl);
    hipLaunchKernelGGL(k_sort_tiny, grid_n(d.n, 256), dim3(256), 0, st, row_ptr, in, out, d, ctl);
    hipLaunchKernelGGL(k_sort_group<16>, grid_n((uint64_t)d.n * 16, 256), dim3(256), 0, st,
                       row_ptr, in, out, d, ctl);
    hipLaunchKernelGGL(k_sort_group<32>, grid_n((uint64_t)d.n * 32, 256, 8192), dim3(256), 0, st,
                       row_ptr, in, out, d, ctl);
    hipLaunchKernelGGL(k_sort_group<64>, grid_n((uint64_t)d.n * 64, 256, 8192), dim3(256), 0, st,
                       row_ptr, in, out, d, ctl);
    hipLaunchKernelGGL(k_sort_mid_bitmap, dim3(num_cus * 8), dim3(256), 0, st, row_ptr, in, out, d,
                       ctl);
    // a batch's graphs have at most kBatchSide <= kMidBits vertices per side, so
    // the bitmap sort takes every medium row of a batch
    static_assert(kBatchSide <= kMidBits, "batch rows are bitmap-sorted");
    if (!d.blk[0]) {
        hipLaunchKernelGGL(k_sort_wave, dim3(num_cus * 8), dim3(256), 0, st, row_ptr, in, out, d,
                           ctl);
        hipLaunchKernelGGL(k_sort_block, dim3(num_cus * 2), dim3(kBlockSortThreads), 0, st, row_ptr,
                           in, out, d, ctl);
    }
    hipLaunchKernelGGL(k_sort_big, dim3(num_cus * 2), dim3(kBigThreads), 0, st, row_ptr, in, out, d,
                       ctl);
    return hipGetLastError();
}

hipError_t launch_lowcount(const uint32_t* row_ptr, const uint32_t* col, const uint32_t* rowcross,
                           uint32_t n, uint32_t* lowcnt, hipStream_t st) {
    hipLaunchKernelGGL(k_lowcount, grid_n(n, 256), dim3(256), 0, st, row_ptr, col, rowcross, n,
                       lowcnt);
    return hipGetLastError();
}

hipError_t launch_records(const uint32_t* row_ptr, const uint32_t* col, const uint32_t* lowcnt,
                          const uint32_t* mptr, Dims d, uint64_t m, uint4* recs, u64* wu, u64* wsu,
                          uint32_t* front, hipStream_t st) {
    hipLaunchKernelGGL(k_records, grid_n(2 * m, kRecThreads * kRecPer, 8192), dim3(kRecThreads), 0,
                       st, row_ptr, col, lowcnt, mptr, d, m, recs, wu, wsu, front);
    return hipGetLastError();
}

hipError_t launch_tile_table(const uint32_t* row_ptr, const uint32_t* col, Dims d,
                             const Control* ctl, uint32_t* tb, uint32_t num_cus, hipStream_t st) {
    hipLaunchKernelGGL(k_tile_table, dim3(num_cus * 8), dim3(256), 0, st, row_ptr, col, d, ctl, tb);
    return hipGetLastError();
}

}  // namespace bbc
