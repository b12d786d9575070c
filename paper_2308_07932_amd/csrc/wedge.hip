// Wedge enumeration and bucket counting: the counting stage of Algorithm 2
// (Section 4.1), run as in Algorithm 4 (Section 5.2) with a parallel loop over
// start vertices and per-start buckets.
//
// For a start u and a middle v (p(v) < p(u)), the end vertices w with
// p(w) < p(u) are the first pos entries of row v.  A wedge u-v-w is symmetric
// when sign(u,v) == sign(v,w) and asymmetric otherwise (Definitions 5, 6); the
// start's bucket for w counts both kinds (l, m), packed as l + (m << 32) in one
// 64-bit word so that each wedge is one LDS atomic.  By Lemmas 1 and 2 the
// pair (u, w) contributes C(l,2) + C(m,2) balanced butterflies and l*m
// unbalanced ones, each butterfly being counted once, at its top-priority
// vertex (Theorem 1).
//
// One persistent workgroup per CU takes work items from a global counter.  An
// item is a list of pieces (see plan.hip); the workgroup keeps the item's
// buckets in LDS (dense counters addressed by w - lo, or a hash table), then
// sums C(.,2) over them and adds to the 64-bit totals.  Pieces that split a
// start along the middle vertices merge their partial counts exactly through a
// global array G with returning atomics: with old = counts already merged,
// C(old + c, 2) = C(old, 2) + C(c, 2) + old * c, so adding C(c,2) + old*c is
// exact in any arrival order.  A hashed piece of a heavy start whose table
// fills up is abandoned (its counts are never added) and redone as two halves
// of its tile run; a single tile is redone with dense counters, which always
// fit, so every piece ends exact.
#include <type_traits>

#include "bbc_internal.h"

namespace bbc {

struct WedgeArgs {
    const Piece* pieces;
    const uint32_t* order;  // heavy item i runs piece order[i] (largest first)
    const uint32_t* items_first;
    uint32_t n_heavy, n_items;
    const uint4* recs;
    const uint32_t* col;
    const uint32_t* tb;
    Dims d;
    uint32_t first_long[2];  // sidx of the first row longer than kLongDeg, per side
    u64* G;
    const uint32_t* sw_off;   // short-middle wedge list of heavy piece p: [sw_off[p], sw_off[p+1])
    const uint32_t* sw_list;  // packed w << 1 | asymmetric
    const uint32_t* sw_mid;   // per-vertex mode: the row of each listed wedge's middle
    Control* ctl;
    u64* gres;  // batches: per graph {balanced, unbalanced, wedges, -}; else NULL (totals in ctl)
    u64* pv;    // per-vertex mode: balanced butterflies per row (n entries, zeroed)
    uint32_t n_dense;  // heavy items 0..n_dense-1 are dense pieces, n_dense..n_heavy-n_wave-1
                       // hashed, the last n_wave one-wave pieces
    uint32_t n_wave;
    uint32_t item0;    // first item k_wedge runs (n_heavy, or 0 when it runs them all)
    Piece* redo;       // halves of hashed pieces k_wedge_pieces<true> gave up on (ctl->redo_n),
                       // run by k_wedge as items n_items, n_items + 1, ...
    uint32_t col_pad;  // index of col's first pad entry (kColPad entries of kColPadValue)
};

// Thread 0's running totals for one graph at a time; flushed to memory when
// the graph changes and at the end (a single graph flushes once).
struct GraphAcc {
    uint32_t g;
    u64 bal, unb;
    __device__ void reset() {
        g = 0;
        bal = unb = 0;
    }
    __device__ void flush(const WedgeArgs& a) {
        if (bal == 0 && unb == 0) return;
        u64* dst = a.gres ? a.gres + 4ull * g : &a.ctl->balanced;
        atomicAdd(dst, bal);
        atomicAdd(dst + 1, unb);
        bal = unb = 0;
    }
    __device__ void add(const WedgeArgs& a, uint32_t graph, u64 b, u64 u) {
        if (graph != g) {
            flush(a);
            g = graph;
        }
        bal += b;
        unb += u;
    }
};

constexpr uint32_t kScanMax = 16;     // short middle prefixes are read whole and filtered
constexpr uint32_t kUnroll = 4;       // independent CSR loads in flight per lane
constexpr uint32_t kWaves = kWedgeThreads / 64;
constexpr uint32_t kStack = 16;       // pending halves of an abandoned piece
constexpr uint32_t kChunk = 1024;     // longer sub-intervals are cut; the tail chunks are
constexpr uint32_t kQueue = 256;      // queued in LDS and shared by all waves afterwards

__device__ inline uint32_t hash32(uint32_t w) { return w * 0x9E3779B1u; }

// The 16-bit-half hash table: 2 x kHashSlots keys, then as many u32 counters
// (l | m << 16).  Returns false if w finds no slot within `lim` probes.
constexpr uint32_t kHash16Slots = 2 * kHashSlots;
static_assert(kLightWindow16 + 2 * kLightMax <= kHash16Slots, "a light item's regions fit its table");
constexpr uint32_t kHash16Log2 = 31u - __builtin_clz(kHash16Slots);
__device__ inline bool bucket_add16(uint32_t* s32, uint32_t lim, uint32_t w, uint32_t inc,
                                    uint32_t i0 = 0) {
    const uint32_t h = hash32(w) >> (32 - kHash16Log2);
    for (uint32_t i = i0; i < lim; ++i) {
        const uint32_t s = (h + i) & (kHash16Slots - 1u);
        uint32_t k = s32[s];
        if (k == kEmpty) {
            k = atomicCAS(&s32[s], kEmpty, w);
            if (k == kEmpty) k = w;
        }
        if (k == w) {
            atomicAdd(&s32[kHash16Slots + s], inc);
            return true;
        }
    }
    return false;
}

// The same table for the light starts of an item: w is hashed into its
// start's region, probed whole (a region holds more slots than the start has
// distinct ends, so it never fills).
__device__ inline bool bucket_add16r(uint32_t* s32, uint32_t region, uint32_t w, uint32_t inc,
                                     uint32_t i0 = 0) {
    const uint32_t rb = region & 0xFFFFu, lg = (region >> 16) & 31u;
    const uint32_t msk = (1u << lg) - 1u;
    const uint32_t h = hash32(w) >> (32 - lg);
    for (uint32_t i = i0; i <= msk; ++i) {
        const uint32_t s = rb + ((h + i) & msk);
        uint32_t k = s32[s];
        if (k == kEmpty) {
            k = atomicCAS(&s32[s], kEmpty, w);
            if (k == kEmpty) k = w;
        }
        if (k == w) {
            atomicAdd(&s32[kHash16Slots + s], inc);
            return true;
        }
    }
    return false;
}

// counters (l | m << 16) of w in a region of the 16-bit-half table (light
// starts of an item), as a 64-bit bucket value (l + (m << 32))
__device__ inline u64 bucket_get16r(const uint32_t* s32, uint32_t region, uint32_t w) {
    const uint32_t rb = region & 0xFFFFu, lg = (region >> 16) & 31u;
    const uint32_t msk = (1u << lg) - 1u;
    const uint32_t h = hash32(w) >> (32 - lg);
    for (uint32_t i = 0; i <= msk; ++i) {
        const uint32_t s = rb + ((h + i) & msk);
        if (s32[s] == w) {
            const uint32_t c = s32[kHash16Slots + s];
            return (c & 0xFFFFu) | ((u64)(c >> 16) << 32);
        }
        if (s32[s] == kEmpty) break;
    }
    return 0;
}

// counters (l | m << 16) of w in the 16-bit-half table, present after the
// counting pass, as a 64-bit bucket value (l + (m << 32))
__device__ inline u64 bucket_get16(const uint32_t* s32, uint32_t w) {
    constexpr uint32_t lg = 31u - __builtin_clz(kHash16Slots);
    const uint32_t h = hash32(w) >> (32 - lg);
    for (uint32_t i = 0; i < kHash16Slots; ++i) {
        const uint32_t s = (h + i) & (kHash16Slots - 1u);
        if (s32[s] == w) {
            const uint32_t c = s32[kHash16Slots + s];
            return (c & 0xFFFFu) | ((u64)(c >> 16) << 32);
        }
        if (s32[s] == kEmpty) break;
    }
    return 0;
}

// Add one wedge to the bucket of end vertex w.  Returns false if the hashed
// region has no room for w within `lim` probes.
__device__ inline bool bucket_add(u64* s_tab, uint32_t* keys, u64* hvals, bool dense,
                                  uint32_t dlo, uint32_t region, uint32_t lim, uint32_t w,
                                  u64 inc) {
    if (dense) {
        atomicAdd(&s_tab[w - dlo], inc);
        return true;
    }
    const uint32_t rb = region & 0xFFFFu, lg = (region >> 16) & 31u;
    const uint32_t msk = (1u << lg) - 1u;
    const uint32_t h = hash32(w) >> (32 - lg);
    for (uint32_t i = 0; i < lim; ++i) {
        const uint32_t s = rb + ((h + i) & msk);
        uint32_t k = keys[s];
        if (k == kEmpty) {
            k = atomicCAS(&keys[s], kEmpty, w);
            if (k == kEmpty) k = w;  // inserted here
        }
        if (k == w) {
            atomicAdd(&hvals[s], inc);
            return true;
        }
    }
    return false;
}

// Value of a bucket (l symmetric, m asymmetric wedges) in the per-vertex
// readback: a wedge through middle v lies in l - 1 (symmetric) or m - 1
// (asymmetric) balanced butterflies with start u and end w (Section 5.1).
__device__ inline u64 middle_share(u64 v, uint32_t asym) {
    const u64 l = v & 0xFFFFFFFFull, m = v >> 32;
    return asym ? m - 1 : l - 1;
}

// hashed bucket of w in a region (present: the counting pass inserted it)
__device__ inline u64 bucket_get(const uint32_t* keys, const u64* hvals, uint32_t region,
                                 uint32_t w) {
    const uint32_t rb = region & 0xFFFFu, lg = (region >> 16) & 31u;
    const uint32_t msk = (1u << lg) - 1u;
    const uint32_t h = hash32(w) >> (32 - lg);
    for (uint32_t i = 0; i <= msk; ++i) {
        const uint32_t s = rb + ((h + i) & msk);
        if (keys[s] == w) return hvals[s];
        if (keys[s] == kEmpty) break;
    }
    return 0;
}

// PV: per-vertex mode.  After a piece's buckets are complete, a second pass
// over the same wedges reads back each wedge's bucket and adds its share to
// the middle vertex; the finalize adds each bucket's C(l,2) + C(m,2) to the
// end vertex and the piece's total to the start (Section 5.1, Algorithm 3,
// with the end vertex distinct from the start).  Every wedge must keep its
// middle: pieces are then never split by record chunks, long sub-intervals are
// not queued, and the listed short-middle wedges carry their middle's row.
template <bool PV>
__global__ __launch_bounds__(kWedgeThreads) void k_wedge(WedgeArgs a) {
    // on-chip buckets: dense mode uses s_tab[0 .. kDenseW); hash mode uses
    // keys = (uint32_t*)s_tab [0 .. kHashSlots) and vals = s_tab + kHashSlots/2.
    __shared__ u64 s_tab[kDenseW];
    __shared__ Piece s_pc[kMaxItemPieces];
    __shared__ uint32_t s_pre[kMaxItemPieces + 1];
    __shared__ Piece s_stack[kStack];
    __shared__ uint32_t s_sp;
    __shared__ uint32_t s_item;
    __shared__ uint32_t s_abort;
    __shared__ uint32_t s_batch;
    __shared__ uint32_t s_wadj[kWaves][64];   // per wave: compacted sub-intervals' address - start,
    __shared__ uint32_t s_waux[kWaves][64];   // sign(u,v) | filter << 1 | piece << 2,
    // head flags of the current kUnroll windows (one byte per position).  The
    // plain count interleaves them: the flag of window position p is byte
    // (p % 64) * kUnroll + p / 64, so a lane reads its flags for all windows in
    // one 32-bit word.  Per-vertex mode, whose readback keeps more registers
    // live, reads them window by window (byte p), which measured faster there.
    __shared__ uint32_t s_head[kWaves][64];
    static_assert(kUnroll == 4, "one 32-bit word of head flags per lane");
    constexpr uint32_t kQ = PV ? 1 : kQueue;
    __shared__ uint32_t s_qadj[kQ], s_qlen[kQ], s_qaux[kQ];  // queued long chunks
    __shared__ uint32_t s_wvrow[PV ? kWaves : 1][64];  // PV: row of each interval's middle
    __shared__ uint32_t s_qn, s_qtake, s_swtake;
    __shared__ bool s_multi;
    __shared__ uint32_t s_next, s_nextok, s_done;
    __shared__ bool s_more;
    __shared__ u64 s_red[2][kWaves];
    __shared__ u64 s_pb[kMaxItemPieces], s_pu[kMaxItemPieces];  // per-piece totals (batches)
    uint32_t* keys = (uint32_t*)s_tab;
    u64* hvals = s_tab + kHashSlots / 2;
    uint32_t* s32 = (uint32_t*)s_tab;  // 16-bit-half dense counters

    const uint32_t tid = threadIdx.x, lane = lane_id(), wave = tid >> 6;
    const uint32_t* __restrict__ col = a.col;
    s_head[wave][lane] = 0;

    __shared__ GraphAcc s_acc;     // this workgroup's totals (thread 0)
    __shared__ Piece s_pf;         // the next heavy item's piece, fetched ahead
    __shared__ uint32_t s_pf_item, s_nredo;
    if (tid == 0) {
        s_acc.reset();
        s_pf_item = kEmpty;
        s_item = a.item0 + atomicAdd(&a.ctl->queue, 1u);
        // halves left by the hashed-piece kernel (it ran before this launch)
        s_nredo = a.redo ? a.ctl->redo_n : 0u;
    }
    // items: heavy pieces [0, n_heavy), light items [n_heavy, n_items), redo
    // halves [n_items, n_items + s_nredo)
    auto is_heavy = [&](uint32_t it) { return it < a.n_heavy || it >= a.n_items; };
    auto heavy_piece = [&](uint32_t it) {
        return it < a.n_heavy ? a.pieces[a.order[it]] : a.redo[it - a.n_items];
    };
    for (;;) {
        __syncthreads();  // every thread is done with the previous item; s_item is set
        const uint32_t item = s_item;
        if (item >= a.n_items + s_nredo) break;
        if (tid == 0) s_nextok = 0;  // the next item is taken during this one
        uint32_t np = 1;
        if (is_heavy(item)) {
            if (tid == 0) s_pc[0] = (s_pf_item == item) ? s_pf : heavy_piece(item);
        } else {
            const uint32_t li = item - a.n_heavy;
            const uint32_t p0 = a.n_heavy + a.items_first[li];
            np = a.n_heavy + a.items_first[li + 1] - p0;
            if (np == 0 || np > kMaxItemPieces) {  // never planned; uniform across the block
                if (tid == 0) s_item = a.item0 + atomicAdd(&a.ctl->queue, 1u);
                continue;
            }
            if (tid < np) s_pc[tid] = a.pieces[p0 + tid];
        }
        if (tid == 0) s_sp = 0;
        const bool heavy = is_heavy(item);

        for (;;) {  // the item's pieces, then any re-split halves (heavy items only)
            __syncthreads();
            // prefix of record counts over the pieces (wave 0)
            if (wave == 0) {
                uint32_t carry = 0;
                u64 multi = 0;  // pieces of more than one graph (batches)
                for (uint32_t c = 0; c < np; c += 64) {
                    uint32_t i = c + lane;
                    uint32_t v = i < np ? s_pc[i].nrec : 0u;
                    uint32_t incl = wave_incl_scan(v);
                    if (i < np) s_pre[i] = carry + incl - v;
                    carry += __shfl(incl, 63, 64);
                    multi |= __ballot(i < np && s_pc[i].graph != s_pc[0].graph);
                }
                if (lane == 0) {
                    s_pre[np] = carry;
                    s_multi = multi != 0;
                }
            }
            if (tid == 0) {
                s_abort = 0;
                s_batch = 0;
                s_qn = 0;
                s_qtake = 0;
                s_swtake = 0;
                s_done = 0;
            }
            const bool dense = (s_pc[0].flags & kPieceDense) != 0;
            const bool d16 = (s_pc[0].flags & kPieceDense16) != 0;  // u32 counters l | m << 16
            // packed counters run in k_wedge_pieces only (never planned in
            // per-vertex mode, and a redone piece is hashed or 32-bit dense)
            if (tid == 0 && (s_pc[0].flags & kDensePacked)) atomicOr(&a.ctl->internal_err, 8u);
            const bool h16 = !dense && (s_pc[0].flags & kPieceHash16) != 0;
            const uint32_t dlo = s_pc[0].lo;
            const uint32_t dwidth = s_pc[0].hi - s_pc[0].lo;
            // a split piece may give up early (it is halved and redone); an
            // unsplit one holds at most kHashSlots/2 distinct ends and probes on
            const uint32_t lim0 =
                (heavy && (s_pc[0].flags & kPiecePartial)) ? a.d.probe_limit : kHashSlots;
            const uint32_t plo0 = s_pc[0].lo, phi0 = s_pc[0].hi, region0 = s_pc[0].region;
            if (dense) {
                // up to a whole 16-byte unit past the width, which the finalize reads
                const uint32_t words = d16 ? (dwidth + 3) / 4 * 2 : (dwidth + 1) / 2 * 2;
                for (uint32_t i = tid; i < words; i += kWedgeThreads) s_tab[i] = 0;
            } else if (h16) {
                for (uint32_t i = tid; i < kHash16Slots; i += kWedgeThreads) {
                    s32[i] = kEmpty;
                    s32[kHash16Slots + i] = 0;
                }
            } else {
                for (uint32_t i = tid; i < kHashSlots; i += kWedgeThreads) {
                    keys[i] = kEmpty;
                    hvals[i] = 0;
                }
            }
            __syncthreads();
            const uint32_t total = s_pre[np];
            // records per grab.  Each grab is one chain of dependent loads (records,
            // tile offsets, entries), so fewer, larger grabs per wave are faster,
            // unless the sub-intervals vary widely: split starts and hashed whole
            // starts take up to 32 in grabs of total/32 (at least 4); dense whole
            // starts and light items up to 64 in grabs of total/16 (at least 8).
            const bool varied = (s_pc[0].flags & kPiecePartial) || (heavy && !dense);
            const uint32_t bsz = varied ? min(32u, max(4u, (total + 31) / 32))
                                        : min(64u, max(8u, (total + a.d.grab_div - 1) / a.d.grab_div));

            // pass over the piece's records: count (readback = false) or, in
            // per-vertex mode, read the complete buckets back (readback = true)
            auto records_pass = [&](const bool readback) {
            for (;;) {
                uint32_t base = 0;
                if (lane == 0) base = atomicAdd(&s_batch, bsz);  // this wave's next records
                base = __shfl(base, 0, 64);
                if (base >= total || s_abort) break;  // s_abort: the piece will be redone
                const uint32_t f = base + lane;
                const bool act = lane < bsz && f < total;
                uint32_t p = 0;
                if (np > 1 && act) {
                    uint32_t lo = 0, hi = np;  // last piece with s_pre[p] <= f
                    while (hi - lo > 1) {
                        uint32_t mid = (lo + hi) >> 1;
                        if (s_pre[mid] <= f)
                            lo = mid;
                        else
                            hi = mid;
                    }
                    p = lo;
                }
                // -- 1. this lane's record and its sub-interval [ia, ib) of row v
                uint32_t rs = 0, s1 = 0, ia = 0, ib = 0, filt = 0, vrow = 0;
                if (act) {
                    const Piece& P = s_pc[p];
                    const uint4 rc = a.recs[P.rec0 + (f - s_pre[p])];
                    rs = rc.x;
                    if (PV) vrow = a.d.base[(P.flags & kPieceSideV) ? 0u : 1u] + rc.z;
                    const uint32_t pos = rc.y >> 1;
                    s1 = rc.y & 1u;
                    ib = pos;
                    if (P.flags & kPiecePartial) {
                        const uint32_t ys = (P.flags & kPieceSideV) ? 0u : 1u;  // side of v
                        const uint32_t vs = rc.z;
                        if (vs >= a.first_long[ys]) {
                            const uint32_t* t = a.tb + a.d.tb_off[ys] +
                                                (uint64_t)(vs - a.first_long[ys]) *
                                                    (a.d.ntile[ys ^ 1u] + 1);
                            ia = min(t[P.t0], pos);
                            ib = min(t[P.t1], pos);
                        } else if (pos <= kScanMax) {
                            filt = 1;  // short prefix: read it all, keep entries in [lo, hi)
                        } else {
                            ia = lower_bound_u32(col + rs, pos, P.lo << 1);
                            ib = ia + lower_bound_u32(col + rs + ia, pos - ia, P.hi << 1);
                        }
                    }
                }
                // -- a long sub-interval of a one-piece item keeps its first kChunk
                // entries; the rest goes to the LDS queue in chunks of kChunk (as many
                // as fit).  The queue is drained with the first piece's buckets, so an
                // item of several pieces keeps its intervals whole.
                if (!PV && np == 1 && ib - ia > kChunk) {
                    const uint32_t want = (ib - ia - 1) / kChunk;  // chunks beyond the first
                    uint32_t old = s_qn, got = 0;
                    for (;;) {
                        got = min(want, kQueue - min(old, kQueue));
                        if (got == 0) break;
                        const uint32_t seen = atomicCAS(&s_qn, old, old + got);
                        if (seen == old) break;
                        old = seen;
                    }
                    if (got > 0) {
                        const uint32_t keep_end = max(ia + kChunk, ib - got * kChunk);
                        for (uint32_t c = 0; c < got; ++c) {
                            const uint32_t c0 = keep_end + c * kChunk;
                            s_qadj[old + c] = rs + c0;
                            s_qlen[old + c] = min(kChunk, ib - c0);
                            s_qaux[old + c] = s1 | (filt << 1) | (p << 2);
                        }
                        ib = keep_end;
                    }
                }
                const uint32_t len = ib - ia;
                // -- 2. compact the non-empty sub-intervals of the wave into LDS.  Entry
                // q of the concatenation (q in [excl, excl + len) of its interval) is
                // col[adj + q] with adj = rs + ia - excl.
                const u64 nz = __ballot(len > 0);
                const uint32_t excl = wave_incl_scan(len) - len;
                const uint32_t T = __shfl(excl + len, 63, 64);
                if (len > 0) {
                    const uint32_t ci = (uint32_t)__popcll(nz & ((lane == 0) ? 0ull : (~0ull >> (64 - lane))));
                    s_wadj[wave][ci] = rs + ia - excl;
                    s_waux[wave][ci] = s1 | (filt << 1) | (p << 2);
                    if (PV) s_wvrow[wave][ci] = vrow;
                }
                // -- 3. all lanes over the concatenated wedges, kUnroll windows of 64 at a
                // time.  The owner of position q is found from head flags: each interval
                // marks its first position, a ballot gives the window's heads, and the
                // owner index is (heads before the window) + (heads at or before q) - 1.
                bool ok = true;
                uint32_t before = 0;
                const u64 le_mask = ~0ull >> (63 - lane);  // lanes 0..lane
                for (uint32_t j = 0; j < T && ok; j += 64 * kUnroll) {
                    uint8_t* hb = (uint8_t*)s_head[wave];
                    if (len > 0 && excl >= j && excl < j + 64 * kUnroll) {
                        const uint32_t hp = excl - j;
                        hb[PV ? hp : (hp & 63u) * kUnroll + (hp >> 6)] = 1;
                    }
                    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
                    uint32_t x[kUnroll], aux[kUnroll], own[PV ? kUnroll : 1];
                    if constexpr (PV) {
#pragma unroll
                        for (uint32_t u = 0; u < kUnroll; ++u) {
                            const u64 M = __ballot(hb[u * 64 + lane] != 0);
                            const uint32_t idx = before + (uint32_t)__popcll(M & le_mask) - 1u;
                            before += (uint32_t)__popcll(M);
                            const uint32_t q = j + u * 64 + lane;
                            aux[u] = kEmpty;
                            x[u] = 0;
                            own[PV ? u : 0] = kEmpty;
                            if (q < T) {
                                aux[u] = s_waux[wave][idx];
                                x[u] = col[s_wadj[wave][idx] + q];
                                own[PV ? u : 0] = idx;
                            }
                        }
                    } else {
                        // owners and their interval entries for all windows first (the
                        // LDS reads are waited for together), then the CSR loads
                        const uint32_t hd4 = s_head[wave][lane];
                        uint32_t adj[kUnroll];
#pragma unroll
                        for (uint32_t u = 0; u < kUnroll; ++u) {
                            const u64 M = __ballot(((hd4 >> (8 * u)) & 0xFFu) != 0);
                            const uint32_t idx = before + (uint32_t)__popcll(M & le_mask) - 1u;
                            before += (uint32_t)__popcll(M);
                            const bool in = j + u * 64 + lane < T;
                            const uint32_t ii = in ? idx : 0u;  // a filled entry either way
                            aux[u] = in ? s_waux[wave][ii] : kEmpty;
                            adj[u] = s_wadj[wave][ii];
                        }
#pragma unroll
                        for (uint32_t u = 0; u < kUnroll; ++u) {
                            const uint32_t q = j + u * 64 + lane;
                            x[u] = q < T ? col[adj[u] + q] : 0u;
                        }
                    }
                    // the wave's flags are cleared (all 4 * 64 bytes, either layout)
                    s_head[wave][lane] = 0;
                    if (PV && readback) {
                        // each wedge's share, summed per interval over the lanes
                        // (owners are non-decreasing across lanes), then one
                        // atomic per interval and window into its middle's count
#pragma unroll
                        for (uint32_t u = 0; u < kUnroll; ++u) {
                            const uint32_t idx = own[PV ? u : 0];
                            u64 val = 0;
                            if (aux[u] != kEmpty) {
                                const uint32_t w = x[u] >> 1;
                                const bool keep = !((aux[u] & 2u) && (w < plo0 || w >= phi0));
                                if (keep) {
                                    const Piece& P = s_pc[aux[u] >> 2];
                                    u64 bv;
                                    if (dense && d16) {
                                        const uint32_t c = s32[w - dlo];
                                        bv = (c & 0xFFFFu) | ((u64)(c >> 16) << 32);
                                    } else if (h16) {  // light items of several pieces: regions
                                        bv = np > 1 ? bucket_get16r(s32, P.region, w)
                                                    : bucket_get16(s32, w);
                                    } else {
                                        bv = dense ? s_tab[w - dlo]
                                                   : bucket_get(keys, hvals, P.region, w);
                                    }
                                    val = middle_share(bv, (x[u] ^ aux[u]) & 1u);
                                }
                            }
                            for (uint32_t off = 1; off < 64; off <<= 1) {
                                const u64 o = __shfl_up(val, off, 64);
                                const uint32_t oi = __shfl_up(idx, off, 64);
                                if (lane >= off && oi == idx) val += o;
                            }
                            const uint32_t ni = __shfl_down(idx, 1, 64);
                            if ((lane == 63 || ni != idx) && idx != kEmpty && val != 0)
                                atomicAdd(&a.pv[s_wvrow[wave][idx]], val);
                        }
                    } else if (np == 1 && dense && !d16) {
                        // one dense piece: counters addressed by w - lo, never full
#pragma unroll
                        for (uint32_t u = 0; u < kUnroll; ++u) {
                            if (aux[u] == kEmpty) continue;
                            const uint32_t w = x[u] >> 1;
                            if ((aux[u] & 2u) && (w < plo0 || w >= phi0)) continue;
                            atomicAdd(&s_tab[w - dlo], ((x[u] ^ aux[u]) & 1u) ? (1ull << 32) : 1ull);
                        }
                    } else if (np == 1 && dense) {  // two tiles, 16-bit halves
#pragma unroll
                        for (uint32_t u = 0; u < kUnroll; ++u) {
                            if (aux[u] == kEmpty) continue;
                            const uint32_t w = x[u] >> 1;
                            if ((aux[u] & 2u) && (w < plo0 || w >= phi0)) continue;
                            atomicAdd(&s32[w - dlo], ((x[u] ^ aux[u]) & 1u) ? 0x10000u : 1u);
                        }
                    } else if (np == 1 && h16) {
                        bool lok = true;
#pragma unroll 1
                        for (uint32_t u = 0; u < kUnroll; ++u) {
                            if (aux[u] == kEmpty || !lok) continue;
                            const uint32_t w = x[u] >> 1;
                            if ((aux[u] & 2u) && (w < plo0 || w >= phi0)) continue;
                            lok = bucket_add16(s32, lim0, w, ((x[u] ^ aux[u]) & 1u) ? 0x10000u : 1u);
                        }
                        ok = __ballot(!lok) == 0;
                    } else if (np == 1) {
                        bool lok = true;
#pragma unroll 1
                        for (uint32_t u = 0; u < kUnroll; ++u) {
                            if (aux[u] == kEmpty || !lok) continue;
                            const uint32_t w = x[u] >> 1;
                            if ((aux[u] & 2u) && (w < plo0 || w >= phi0)) continue;
                            lok = bucket_add(s_tab, keys, hvals, false, 0, region0, lim0, w,
                                             ((x[u] ^ aux[u]) & 1u) ? (1ull << 32) : 1ull);
                        }
                        ok = __ballot(!lok) == 0;  // the whole wave leaves together
                    } else {  // light starts of an item: regions of the 16-bit-half table
                        // The first probes of the step's windows go together (their
                        // region, key and insert reads wait for LDS once each); an
                        // entry whose first slot holds another key probes on from
                        // the second slot.
                        uint32_t rg[kUnroll], sl[kUnroll], kk[kUnroll];
#pragma unroll
                        for (uint32_t u = 0; u < kUnroll; ++u)
                            rg[u] = s_pc[aux[u] == kEmpty ? 0u : aux[u] >> 2].region;
#pragma unroll
                        for (uint32_t u = 0; u < kUnroll; ++u) {
                            const uint32_t lg = (rg[u] >> 16) & 31u;
                            sl[u] = (rg[u] & 0xFFFFu) + (hash32(x[u] >> 1) >> (32 - lg));
                            kk[u] = s32[sl[u]];
                        }
#pragma unroll
                        for (uint32_t u = 0; u < kUnroll; ++u) {
                            if (aux[u] != kEmpty && kk[u] == kEmpty) {
                                const uint32_t o = atomicCAS(&s32[sl[u]], kEmpty, x[u] >> 1);
                                kk[u] = o == kEmpty ? x[u] >> 1 : o;
                            }
                        }
                        bool lok = true;
#pragma unroll
                        for (uint32_t u = 0; u < kUnroll; ++u) {
                            if (aux[u] == kEmpty) continue;
                            const uint32_t w = x[u] >> 1;
                            const uint32_t inc = ((x[u] ^ aux[u]) & 1u) ? 0x10000u : 1u;
                            if (kk[u] == w)
                                atomicAdd(&s32[kHash16Slots + sl[u]], inc);
                            else if (lok)
                                lok = bucket_add16r(s32, rg[u], w, inc, 1);
                        }
                        ok = __ballot(!lok) == 0;
                    }
                }
                __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
                if (!ok) s_abort = 1;
            }
            };
            records_pass(false);
            // -- the bucketed wedges through short middle rows (split starts) fill
            // the tail of the record sweep: waves take 64 * kUnroll at a time
            if (heavy && (s_pc[0].flags & kPiecePartial) && s_pc[0].list != kEmpty) {
                const uint32_t b0 = a.sw_off[s_pc[0].list];
                const uint32_t n_sw = a.sw_off[s_pc[0].list + 1] - b0;
                bool ok = true;
                for (;;) {
                    uint32_t c = 0;
                    if (lane == 0) c = atomicAdd(&s_swtake, 64 * kUnroll);
                    c = __shfl(c, 0, 64);
                    if (c >= n_sw || s_abort || !ok) break;
                    uint32_t x[kUnroll];
#pragma unroll
                    for (uint32_t u = 0; u < kUnroll; ++u) {
                        const uint32_t q = c + u * 64 + lane;
                        x[u] = q < n_sw ? a.sw_list[b0 + q] : kEmpty;
                    }
                    bool lok = true;
#pragma unroll
                    for (uint32_t u = 0; u < kUnroll; ++u) {
                        if (x[u] == kEmpty || !lok) continue;
                        const uint32_t w = x[u] >> 1;
                        if (w < plo0 || w >= phi0) continue;  // a re-split half keeps its share
                        if (dense && d16)
                            atomicAdd(&s32[w - dlo], (x[u] & 1u) ? 0x10000u : 1u);
                        else if (h16)
                            lok = bucket_add16(s32, lim0, w, (x[u] & 1u) ? 0x10000u : 1u);
                        else
                            lok = bucket_add(s_tab, keys, hvals, dense, dlo, region0, lim0, w,
                                             (x[u] & 1u) ? (1ull << 32) : 1ull);
                    }
                    ok = __ballot(!lok) == 0;  // wave-uniform: lane 0 keeps taking entries
                }
                if (!ok) s_abort = 1;
            }
            // the first wave done with the sweep takes the next item from the queue
            // and fetches its piece while the other waves finish
            {
                uint32_t f = 1;
                if (lane == 0) f = atomicAdd(&s_done, 1u);
                if (lane == 0 && f == 0 && !s_nextok) {
                    const uint32_t nx = a.item0 + atomicAdd(&a.ctl->queue, 1u);
                    if (nx < a.n_items + s_nredo && is_heavy(nx) && s_pf_item != nx) {
                        s_pf = heavy_piece(nx);
                        s_pf_item = nx;
                    }
                    s_next = nx;
                    s_nextok = 1;
                }
            }
            __syncthreads();
            // -- queued chunks of long sub-intervals: one wave per chunk, coalesced
            // (s_qn is final after the barrier above, so the branch is uniform)
            if (!PV && np == 1 && s_qn > 0) {
                bool ok = true;
                for (;;) {
                    uint32_t c = 0;
                    if (lane == 0) c = atomicAdd(&s_qtake, 1u);
                    c = __shfl(c, 0, 64);
                    if (c >= s_qn || s_abort || !ok) break;
                    const uint32_t adj = s_qadj[c], qlen = s_qlen[c], aux = s_qaux[c];
                    for (uint32_t e0 = 0; e0 < qlen && ok; e0 += 64 * kUnroll) {
                        uint32_t x[kUnroll];
#pragma unroll
                        for (uint32_t u = 0; u < kUnroll; ++u) {
                            const uint32_t e = e0 + u * 64 + lane;
                            x[u] = e < qlen ? col[adj + e] : kEmpty;
                        }
                        bool lok = true;
#pragma unroll
                        for (uint32_t u = 0; u < kUnroll; ++u) {
                            if (x[u] == kEmpty || !lok) continue;
                            const uint32_t w = x[u] >> 1;
                            if ((aux & 2u) && (w < plo0 || w >= phi0)) continue;
                            const u64 inc = ((x[u] ^ aux) & 1u) ? (1ull << 32) : 1ull;
                            if (dense && d16)
                                atomicAdd(&s32[w - dlo], ((x[u] ^ aux) & 1u) ? 0x10000u : 1u);
                            else if (dense)
                                atomicAdd(&s_tab[w - dlo], inc);
                            else if (h16)
                                lok = bucket_add16(s32, lim0, w, ((x[u] ^ aux) & 1u) ? 0x10000u : 1u);
                            else
                                lok = bucket_add(s_tab, keys, hvals, false, 0, region0, lim0, w, inc);
                        }
                        ok = __ballot(!lok) == 0;  // wave-uniform: lane 0 keeps taking chunks
                    }
                }
                if (!ok) s_abort = 1;
                __syncthreads();
            }

            if (s_abort) {
                // Abandon this piece's counts; redo it as two halves of its tile
                // run, or, for a single tile, with dense counters.
                if (tid == 0) {
                    atomicAdd(&a.ctl->resplits, 1ull);
                    Piece P = s_pc[0];
                    if (!heavy || np != 1 || !(P.flags & kPiecePartial) || s_sp + 1 >= kStack) {
                        atomicOr(&a.ctl->internal_err, 1u);  // cannot happen by construction
                        s_sp = kStack + 1;
                    } else if (P.t1 - P.t0 > 1) {
                        const uint32_t tm = (P.t0 + P.t1) >> 1;
                        Piece hi = P;
                        hi.t0 = tm;
                        hi.lo = tm * kTile;
                        s_stack[s_sp++] = hi;
                        P.t1 = tm;
                        P.hi = min(P.hi, tm * kTile);
                        s_pc[0] = P;
                    } else {
                        P.flags |= kPieceDense;
                        s_pc[0] = P;
                    }
                }
                __syncthreads();
                if (s_sp > kStack) break;
                continue;
            }

            if (PV) {  // second pass: the middles' shares from the complete buckets
                if (tid == 0) {
                    s_batch = 0;
                    s_swtake = 0;
                }
                __syncthreads();
                records_pass(true);
                // the listed short-middle wedges: each share goes to the wedge's
                // middle, summed over runs of one middle (consecutive lanes)
                if (heavy && (s_pc[0].flags & kPiecePartial) && s_pc[0].list != kEmpty) {
                    const uint32_t b0 = a.sw_off[s_pc[0].list];
                    const uint32_t n_sw = a.sw_off[s_pc[0].list + 1] - b0;
                    const u64 le = ~0ull >> (63 - lane);
                    for (;;) {
                        uint32_t c = 0;
                        if (lane == 0) c = atomicAdd(&s_swtake, 64u);
                        c = __shfl(c, 0, 64);
                        if (c >= n_sw) break;
                        const uint32_t q = c + lane;
                        uint32_t x = kEmpty, mid = kEmpty;
                        if (q < n_sw) {
                            x = a.sw_list[b0 + q];
                            mid = a.sw_mid[b0 + q];
                        }
                        u64 val = 0;
                        if (x != kEmpty) {
                            const uint32_t w = x >> 1;
                            if (w >= plo0 && w < phi0) {
                                u64 bv;
                                if (dense && d16) {
                                    const uint32_t c = s32[w - dlo];
                                    bv = (c & 0xFFFFu) | ((u64)(c >> 16) << 32);
                                } else if (h16) {
                                    bv = bucket_get16(s32, w);
                                } else {
                                    bv = dense ? s_tab[w - dlo] : bucket_get(keys, hvals, region0, w);
                                }
                                val = middle_share(bv, x & 1u);
                            }
                        }
                        const u64 heads = __ballot(lane == 0 || __shfl_up(mid, 1, 64) != mid);
                        const uint32_t seg = (uint32_t)__popcll(heads & le);
                        for (uint32_t off = 1; off < 64; off <<= 1) {
                            const u64 o = __shfl_up(val, off, 64);
                            const uint32_t os = __shfl_up(seg, off, 64);
                            if (lane >= off && os == seg) val += o;
                        }
                        const uint32_t ns = __shfl_down(seg, 1, 64);
                        if ((lane == 63 || ns != seg) && mid != kEmpty && val != 0)
                            atomicAdd(&a.pv[mid], val);
                    }
                }
                __syncthreads();
            }

            // -- finalize: C(l,2) + C(m,2) and l*m over the buckets
            u64 bal = 0, unb = 0;
            // a light item of a batch may hold starts of several graphs, and in
            // per-vertex mode every start needs its own total: then one wave
            // per piece sums the piece's own hash region
            const bool per_piece = np > 1 && (PV || (a.gres != nullptr && s_multi));
            const u64 ubase0 = a.d.base[(s_pc[0].flags & kPieceSideV) ? 1u : 0u];
            if (per_piece) {
                for (uint32_t p = wave; p < np; p += kWaves) {
                    const uint32_t region = s_pc[p].region;
                    const uint32_t rb = region & 0xFFFFu, sz = 1u << ((region >> 16) & 31u);
                    const u64 ubase = a.d.base[(s_pc[p].flags & kPieceSideV) ? 1u : 0u];
                    u64 pb = 0, pu = 0;
                    for (uint32_t i = lane; i < sz; i += 64) {  // light starts: 16-bit halves
                        const uint32_t c = s32[kHash16Slots + rb + i];
                        const uint32_t l = c & 0xFFFFu, mm = c >> 16;
                        const u64 b = ((l * (l - 1u)) >> 1) + ((mm * (mm - 1u)) >> 1);
                        pb += b;
                        pu += l * mm;
                        if (PV && b) atomicAdd(&a.pv[ubase + s32[rb + i]], b);
                    }
                    pb = wave_reduce_sum(pb);
                    pu = wave_reduce_sum(pu);
                    if (lane == 0) {
                        s_pb[p] = pb;
                        s_pu[p] = pu;
                    }
                }
            } else if (!PV && dense && d16 && !(s_pc[0].flags & kPieceMerge)) {
                // 16-bit halves: C(l,2) + C(m,2) and l*m fit 32 bits; entries past
                // the width are zero, and so are buckets no wedge reached
                const uint4* t4 = reinterpret_cast<const uint4*>(s32);
                for (uint32_t g = tid; g < (dwidth + 3) / 4; g += kWedgeThreads) {
                    const uint4 c = t4[g];
                    const uint32_t cc[4] = {c.x, c.y, c.z, c.w};
#pragma unroll
                    for (int k = 0; k < 4; ++k) {
                        const uint32_t l = cc[k] & 0xFFFFu, mm = cc[k] >> 16;
                        bal += ((l * (l - 1u)) >> 1) + ((mm * (mm - 1u)) >> 1);
                        unb += l * mm;
                    }
                }
            } else if (!PV && dense && !(s_pc[0].flags & kPieceMerge)) {
                const ulonglong2* t2 = reinterpret_cast<const ulonglong2*>(s_tab);
                for (uint32_t g = tid; g < (dwidth + 1) / 2; g += kWedgeThreads) {
                    const ulonglong2 c = t2[g];
                    const u64 cc[2] = {c.x, c.y};
#pragma unroll
                    for (int k = 0; k < 2; ++k) {
                        const u64 l = cc[k] & 0xFFFFFFFFull, mm = cc[k] >> 32;
                        bal += choose2(l) + choose2(mm);
                        unb += l * mm;
                    }
                }
            } else if (dense) {
                const bool merge = (s_pc[0].flags & kPieceMerge) != 0;
                const uint32_t gb = s_pc[0].gbase;
                for (uint32_t i = tid; i < dwidth; i += kWedgeThreads) {
                    u64 v;
                    if (d16) {
                        const uint32_t c = s32[i];
                        v = (c & 0xFFFFu) | ((u64)(c >> 16) << 32);
                    } else {
                        v = s_tab[i];
                    }
                    if (v == 0) continue;
                    const u64 l = v & 0xFFFFFFFFull, m = v >> 32;
                    bal += choose2(l) + choose2(m);
                    unb += l * m;
                    if (PV && choose2(l) + choose2(m))
                        atomicAdd(&a.pv[ubase0 + dlo + i], choose2(l) + choose2(m));
                    if (merge) {
                        const u64 old = atomicAdd(&a.G[(uint64_t)gb + i], v);
                        const u64 ol = old & 0xFFFFFFFFull, om = old >> 32;
                        bal += ol * l + om * m;
                        unb += ol * m + om * l;
                    }
                }
            } else if (PV && h16) {  // end vertices get their buckets' counts
                for (uint32_t i = tid; i < kHash16Slots; i += kWedgeThreads) {
                    if (s32[i] == kEmpty) continue;
                    const uint32_t c = s32[kHash16Slots + i];
                    const uint32_t l = c & 0xFFFFu, mm = c >> 16;
                    const u64 b = ((l * (l - 1u)) >> 1) + ((mm * (mm - 1u)) >> 1);
                    bal += b;
                    unb += l * mm;
                    if (b) atomicAdd(&a.pv[ubase0 + s32[i]], b);
                }
            } else if (h16) {
                // counters of empty slots are zero
                const uint4* c4 = reinterpret_cast<const uint4*>(s32 + kHash16Slots);
                for (uint32_t g = tid; g < kHash16Slots / 4; g += kWedgeThreads) {
                    const uint4 c = c4[g];
                    const uint32_t cc[4] = {c.x, c.y, c.z, c.w};
#pragma unroll
                    for (int k = 0; k < 4; ++k) {
                        const uint32_t l = cc[k] & 0xFFFFu, mm = cc[k] >> 16;
                        bal += ((l * (l - 1u)) >> 1) + ((mm * (mm - 1u)) >> 1);
                        unb += l * mm;
                    }
                }
            } else if (!PV) {
                const ulonglong2* v2 = reinterpret_cast<const ulonglong2*>(hvals);
                for (uint32_t g = tid; g < kHashSlots / 2; g += kWedgeThreads) {
                    const ulonglong2 c = v2[g];
                    const u64 cc[2] = {c.x, c.y};
#pragma unroll
                    for (int k = 0; k < 2; ++k) {
                        const u64 l = cc[k] & 0xFFFFFFFFull, mm = cc[k] >> 32;
                        bal += choose2(l) + choose2(mm);
                        unb += l * mm;
                    }
                }
            } else {
                for (uint32_t i = tid; i < kHashSlots; i += kWedgeThreads) {
                    if (keys[i] == kEmpty) continue;
                    const u64 v = hvals[i];
                    const u64 l = v & 0xFFFFFFFFull, m = v >> 32;
                    bal += choose2(l) + choose2(m);
                    unb += l * m;
                    if (PV && choose2(l) + choose2(m))
                        atomicAdd(&a.pv[ubase0 + keys[i]], choose2(l) + choose2(m));
                }
            }
            if (!per_piece) {
                bal = wave_reduce_sum(bal);
                unb = wave_reduce_sum(unb);
                if (lane == 0) {
                    s_red[0][wave] = bal;
                    s_red[1][wave] = unb;
                }
            }
            // whether re-split halves remain, decided before the barrier; thread 0
            // pops the next half after it, and the barrier at the top of the piece
            // loop (or of the item loop) orders that pop before any use
            if (tid == 0) s_more = s_sp > 0 && s_sp <= kStack;
            __syncthreads();
            const bool more = s_more;
            if (tid == 0) {
                if (per_piece) {
                    for (uint32_t p = 0; p < np; ++p) {
                        s_acc.add(a, s_pc[p].graph, s_pb[p], s_pu[p]);
                        if (PV && s_pb[p]) atomicAdd(&a.pv[s_pc[p].start_row], s_pb[p]);
                    }
                } else {
                    u64 sb = 0, su = 0;
                    for (uint32_t w = 0; w < kWaves; ++w) {
                        sb += s_red[0][w];
                        su += s_red[1][w];
                    }
                    s_acc.add(a, s_pc[0].graph, sb, su);
                    if (PV && sb) atomicAdd(&a.pv[s_pc[0].start_row], sb);
                }
                if (more) s_pc[0] = s_stack[--s_sp];
            }
            if (!more) break;
        }
        if (tid == 0) s_item = s_nextok ? s_next : a.item0 + atomicAdd(&a.ctl->queue, 1u);
    }
    if (tid == 0) s_acc.flush(a);
}

// ---------------------------------------------------------------------------
// Dense pieces (plain count): one start's records restricted to an end-vertex
// range [lo, hi) whose counters always fit the table, as u64 l + (m << 32)
// per end vertex (kDenseW of them) or, for a start with fewer than 2^16
// middles, u32 l | (m << 16) over two tiles.  The counting is the same as in
// k_wedge; what differs is how the work is scheduled, because a wave's time
// here goes to chains of dependent memory loads (record -> tile offsets ->
// CSR entries), each about a microsecond under load, more than to the adds:
//   * the CSR entries of the next sweep step (kUnroll windows of 64) are
//     loaded before the adds of the current step are issued;
//   * the record and tile offsets of a wave's next grab are loaded while its
//     current grab is swept, as long as enough records remain for every wave
//     (a grab claimed early by a busy wave would otherwise leave others idle
//     at the end of the piece);
//   * each wave's first grab is fixed (wave w takes records [w*b, (w+1)*b))
//     and loaded while the table is cleared.
// A dense piece never overflows, so there is no abandon-and-redo path; the
// long-interval queue, the bucketed short-middle wedges and the exact merge of
// record chunks through G work as in k_wedge.
namespace {

// this lane's record of a grab, and the sub-interval of its middle row
struct DenseGrab {
    uint32_t rs, pos, vs, s1;  // record: row start, prefix length, middle sidx, sign(u, v)
    uint32_t ta, tb;           // tile offsets of the piece's range (long middles of split starts)
};

// Where a piece's grabs come from: its records, the grab size, and for a split
// start the tile tables that give each record's sub-interval of the range
struct GrabSrc {
    uint32_t rec0, total, bsz, t0, t1, tstride, flong;
    bool partial;
    const uint32_t* tbl;
};

__device__ inline GrabSrc grab_src(const WedgeArgs& a, uint32_t rec0, uint32_t nrec,
                                   uint32_t flags, uint32_t t0, uint32_t t1) {
    GrabSrc g;
    g.rec0 = rec0;
    g.total = nrec;
    g.t0 = t0;
    g.t1 = t1;
    g.partial = (flags & kPiecePartial) != 0;
    const uint32_t ys = (flags & kPieceSideV) ? 0u : 1u;  // side of the middles
    g.bsz = g.partial ? min(32u, max(4u, (nrec + 15) / 16))
                      : min(64u, max(8u, (nrec + a.d.grab_div - 1) / a.d.grab_div));
    g.tbl = g.partial ? a.tb + a.d.tb_off[ys] : nullptr;
    g.tstride = a.d.ntile[ys ^ 1u] + 1;
    g.flong = a.first_long[ys];
    return g;
}

// Loads below are issued by every lane (inactive lanes read a valid address
// and drop the value): a load in a per-lane branch makes the compiler wait
// for all outstanding loads where the branches meet.
// -- this lane's record of the grab at `base` (total > 0)
__device__ inline void grab_records(const WedgeArgs& a, const GrabSrc& s, uint32_t base,
                                    uint32_t lane, DenseGrab& g) {
    const uint32_t f = base + lane;
    const bool act = lane < s.bsz && f < s.total;
    const uint4 rc = a.recs[s.rec0 + (act ? f : 0u)];
    g.rs = rc.x;
    g.pos = act ? rc.y >> 1 : 0u;
    g.s1 = rc.y & 1u;
    g.vs = rc.z;
}

// -- the tile offsets of the piece's range in the record's middle row (split
// starts; each long middle row has a tile table)
__device__ inline void grab_tiles(const GrabSrc& s, DenseGrab& g) {
    g.ta = 0;
    g.tb = g.pos;
    if (s.partial) {
        const bool lng = g.pos > 0 && g.vs >= s.flong;
        const uint32_t* t = s.tbl + (uint64_t)(lng ? g.vs - s.flong : 0u) * s.tstride;
        const uint32_t a0 = t[s.t0], a1 = t[s.t1];
        if (lng) {
            g.ta = a0;
            g.tb = a1;
        }
    }
}

// 2 (C(l,2) + C(m,2)) and 2 l m of one u32 bucket l | (m << 16), l + m < 2^16:
// dot products of the two 16-bit halves
__device__ inline void bucket16_sums(uint32_t c, u64& q2, u64& lm2) {
    typedef unsigned short h2 __attribute__((ext_vector_type(2)));
    const h2 a = __builtin_bit_cast(h2, c);
    const h2 d = a - (h2){1, 1};  // l - 1, m - 1 (an empty half gives 0 * 0xFFFF = 0)
    q2 += __builtin_amdgcn_udot2(a, d, 0u, false);
    lm2 += __builtin_amdgcn_udot2(a, __builtin_bit_cast(h2, __builtin_amdgcn_alignbit(c, c, 16)), 0u,
                                  false);
}

// Sums over a word of two 8-bit-half buckets (bytes l0, m0, l1, m1), kept in
// the instructions' accumulators: q += every byte squared, s += every byte,
// lm += l0 m0 + l1 m1; then 2 (C(l,2) + C(m,2)) = q - s over the words
__device__ inline void bucket8_acc(uint32_t c, uint32_t& q, uint32_t& s, uint32_t& lm) {
    q = __builtin_amdgcn_udot4(c, c, q, false);
    s = __builtin_amdgcn_sad_u8(c, 0u, s);
    lm = __builtin_amdgcn_udot4(c & 0x00FF00FFu, (c >> 8) & 0x00FF00FFu, lm, false);
}

// ... and over a word of four 4-bit-half buckets (byte i = l_i | m_i << 4,
// l_i + m_i <= 15): the l and m nibbles split into bytes first
__device__ inline void bucket4_acc(uint32_t c, uint32_t& q, uint32_t& s, uint32_t& lm) {
    const uint32_t l = c & 0x0F0F0F0Fu, m = (c >> 4) & 0x0F0F0F0Fu;
    q = __builtin_amdgcn_udot4(l, l, q, false);
    q = __builtin_amdgcn_udot4(m, m, q, false);
    s = __builtin_amdgcn_sad_u8(l + m, 0u, s);
    lm = __builtin_amdgcn_udot4(l, m, lm, false);
}

// dense counter layouts of k_wedge_pieces (log2 of end vertices per u32 word
// for the packed ones)
enum : int { kD32 = 0, kD16, kD8, kD4 };
static_assert(kTile % 4 == 0, "a packed piece's base keeps the field of w in its low bits");
static_assert(3 * 64 * kUnroll <= kColPad, "the sweep's loads past a grab stay in the pad");

}  // namespace

template <bool HASH>
__global__ __launch_bounds__(kWedgeThreads) void k_wedge_pieces(WedgeArgs a) {
    // the counters, then 64 junk words that the lanes past a grab's end add to
    // (one per lane, so that they do not contend)
    __shared__ u64 s_tab[kDenseW + 32];
    // per non-empty sub-interval of a grab (address - first position, sign),
    // then the sentinel that owns the positions from T on: (pad - T, 2)
    __shared__ uint2 s_wrec[kWaves][65];
    __shared__ uint32_t s_head[kWaves][64];  // head flags, interleaved as in k_wedge
    __shared__ uint32_t s_qadj[kQueue], s_qlen[kQueue], s_qaux[kQueue];
    __shared__ Piece s_p, s_pf;
    __shared__ uint32_t s_item, s_pf_item, s_next, s_nextok, s_done;
    __shared__ uint32_t s_batch, s_qn, s_qtake, s_swtake, s_abort;
    __shared__ u64 s_red[2][kWaves];
    __shared__ GraphAcc s_acc;
    uint32_t* s32 = (uint32_t*)s_tab;
    uint32_t* keys = (uint32_t*)s_tab;  // 64-bit hashed layout: keys, then counters
    u64* hvals = s_tab + kHashSlots / 2;
    const uint32_t tid = threadIdx.x, lane = lane_id();
    const uint32_t wave = __builtin_amdgcn_readfirstlane(tid >> 6);  // (uniform: LDS bases in SGPRs)
    // dense pieces are heavy items 0 .. n_dense-1, hashed ones n_dense .. n_heavy-1
    auto fetch = [&]() -> uint32_t {
        if (HASH) {
            const uint32_t i = a.n_dense + atomicAdd(&a.ctl->queue_hash, 1u);
            return i < a.n_heavy - a.n_wave ? i : kEmpty;
        }
        const uint32_t i = atomicAdd(&a.ctl->queue_dense, 1u);
        return i < a.n_dense ? i : kEmpty;
    };
    const uint32_t* __restrict__ col = a.col;
    const u64 le_mask = ~0ull >> (63 - lane);  // lanes 0..lane
    s_head[wave][lane] = 0;
    if (tid == 0) {
        s_acc.reset();
        s_pf_item = kEmpty;
        s_item = fetch();
        if (s_item != kEmpty) s_p = a.pieces[a.order[s_item]];
    }
    for (;;) {
        __syncthreads();  // s_item and s_p are set; the previous item is done
        const uint32_t item = s_item;
        if (item == kEmpty) break;
        Piece P;  // wave-uniform: the fields live in scalar registers
        P.rec0 = __builtin_amdgcn_readfirstlane(s_p.rec0);
        P.nrec = __builtin_amdgcn_readfirstlane(s_p.nrec);
        P.lo = __builtin_amdgcn_readfirstlane(s_p.lo);
        P.hi = __builtin_amdgcn_readfirstlane(s_p.hi);
        P.t0 = __builtin_amdgcn_readfirstlane(s_p.t0);
        P.t1 = __builtin_amdgcn_readfirstlane(s_p.t1);
        P.flags = __builtin_amdgcn_readfirstlane(s_p.flags);
        P.gbase = __builtin_amdgcn_readfirstlane(s_p.gbase);
        P.list = __builtin_amdgcn_readfirstlane(s_p.list);
        P.graph = __builtin_amdgcn_readfirstlane(s_p.graph);
        P.region = __builtin_amdgcn_readfirstlane(s_p.region);
        const int dk = HASH ? kD32
                            : (P.flags & kPieceDense4) ? kD4
                            : (P.flags & kPieceDense8) ? kD8
                            : (P.flags & kPieceDense16) ? kD16 : kD32;
        const bool d16 = dk != kD32;  // u32 words of l | m halves (16, 8 or 4 bits each)
        const uint32_t wlog = dk == kD4 ? 2u : dk == kD8 ? 1u : 0u;  // log2 ends per word
        const bool h16 = HASH && (P.flags & kPieceHash16) != 0;  // else u32 keys + u64 counters
        // a split piece's hash table may give up (the piece is then redone in
        // halves by k_wedge); an unsplit one holds at most kHashSlots/2 ends
        const uint32_t lim = (P.flags & kPiecePartial) ? a.d.probe_limit : kHashSlots;
        const bool partial = (P.flags & kPiecePartial) != 0;
        const uint32_t dlo = P.lo, plo = P.lo, phi = P.hi, dwidth = P.hi - P.lo;
        const GrabSrc src = grab_src(a, P.rec0, P.nrec, P.flags, P.t0, P.t1);
        const uint32_t total = src.total, bsz = src.bsz, flong = src.flong;
        const uint32_t junk32 = 2 * kDenseW + lane, junk64 = kDenseW + (lane >> 1);
        if (tid == 0) {
            s_batch = kWaves * bsz;  // grabs beyond every wave's first one
            s_qn = s_qtake = s_swtake = 0;
            s_nextok = 0;
            s_done = 0;
            s_abort = 0;
        }
        // a grab's records (issued now, used later), then its tile offsets
        auto load_rec = [&](uint32_t base, DenseGrab& g) { grab_records(a, src, base, lane, g); };
        auto load_tiles = [&](DenseGrab& g) { grab_tiles(src, g); };
        // one wedge into the bucket of end vertex w; false when a hashed table
        // has no room for w within the probe limit
        auto add_one = [&](uint32_t w, bool asym) -> bool {
            if (!HASH) {
                const uint32_t off = w - dlo;
                if (d16) {
                    // half width 16 >> wlog bits; this end's field at (off mod 2^wlog)
                    const uint32_t inc = (asym ? 1u << (16u >> wlog) : 1u)
                                         << ((off & ((1u << wlog) - 1u)) << (5u - wlog));
                    atomicAdd(&s32[off >> wlog], inc);
                } else {
                    atomicAdd(&s_tab[off], asym ? (1ull << 32) : 1ull);
                }
                return true;
            }
            if (h16) return bucket_add16(s32, lim, w, asym ? 0x10000u : 1u);
            return bucket_add(s_tab, keys, hvals, false, 0, P.region, lim, w,
                              asym ? (1ull << 32) : 1ull);
        };
        DenseGrab cur;
        uint32_t cur_base = wave * bsz;
        if (total > 0) load_rec(cur_base, cur);
        // -- clear the counters of the range (up to a whole 16-byte unit past
        // its end, which the finalize reads), while the records arrive
        if (!HASH) {
            const uint32_t words =
                d16 ? (((dwidth + (1u << wlog) - 1u) >> wlog) + 3) / 4 * 2 : (dwidth + 1) / 2 * 2;
            for (uint32_t i = tid; i < words; i += kWedgeThreads) s_tab[i] = 0;
        } else if (h16) {
            for (uint32_t i = tid; i < kHash16Slots; i += kWedgeThreads) {
                s32[i] = kEmpty;
                s32[kHash16Slots + i] = 0;
            }
        } else {
            for (uint32_t i = tid; i < kHashSlots; i += kWedgeThreads) {
                keys[i] = kEmpty;
                hvals[i] = 0;
            }
        }
        if (total > 0) load_tiles(cur);
        __syncthreads();  // table cleared, s_batch set

        // -- the records, grab by grab; the sweep is compiled once per dense
        // counter layout (DK), chosen per piece
        auto records = [&](auto dktag) {
        constexpr int DK = decltype(dktag)::value;
        bool have = cur_base < total;
        while (have) {
            // this lane's sub-interval [ia, ib) of its middle row.  A split
            // start's pieces hold its long-middle records only (the planner
            // gives them the records before its first short one), and every
            // long middle row has a tile table.
            uint32_t ia = 0, ib = cur.pos;
            if (partial && cur.pos > 0) {
                if (cur.vs >= flong) {
                    ia = min(cur.ta, cur.pos);
                    ib = min(cur.tb, cur.pos);
                } else {
                    ib = 0;
                    atomicOr(&a.ctl->internal_err, 4u);  // cannot happen by construction
                }
            }
            const uint32_t rs = cur.rs, s1 = cur.s1;
            // claim the next grab now when enough records remain for every
            // wave, and start loading it; otherwise claim it after this sweep
            DenseGrab nxt;
            uint32_t nxt_base = kEmpty;
            {
                uint32_t nb = 0;
                if (lane == 0) {
                    const uint32_t seen = __hip_atomic_load(&s_batch, __ATOMIC_RELAXED,
                                                            __HIP_MEMORY_SCOPE_WORKGROUP);
                    nb = (seen < total && total - seen > 2 * kWaves * bsz)
                             ? atomicAdd(&s_batch, bsz) : kEmpty;
                }
                nxt_base = __shfl(nb, 0, 64);
                if (nxt_base != kEmpty) load_rec(nxt_base, nxt);
            }
            // a long sub-interval keeps its first kChunk entries; the rest goes to
            // the LDS queue in chunks of kChunk (as many as fit)
            if (ib - ia > kChunk) {
                const uint32_t want = (ib - ia - 1) / kChunk;
                uint32_t old = s_qn, got = 0;
                for (;;) {
                    got = min(want, kQueue - min(old, kQueue));
                    if (got == 0) break;
                    const uint32_t seen = atomicCAS(&s_qn, old, old + got);
                    if (seen == old) break;
                    old = seen;
                }
                if (got > 0) {
                    const uint32_t keep_end = max(ia + kChunk, ib - got * kChunk);
                    for (uint32_t c = 0; c < got; ++c) {
                        const uint32_t c0 = keep_end + c * kChunk;
                        s_qadj[old + c] = rs + c0;
                        s_qlen[old + c] = min(kChunk, ib - c0);
                        s_qaux[old + c] = s1;
                    }
                    ib = keep_end;
                }
            }
            const uint32_t len = ib - ia;
            const u64 nz = __ballot(len > 0);
            const uint32_t excl = wave_incl_scan(len) - len;
            const uint32_t T = __builtin_amdgcn_readfirstlane(__shfl(excl + len, 63, 64));
            if (len > 0) {
                const uint32_t ci = (uint32_t)__popcll(nz & (le_mask >> 1));
                s_wrec[wave][ci] = make_uint2(rs + ia - excl, s1);
            }
            // the sentinel: positions q >= T read col[pad + q - T] (the steps
            // loaded past the last reach q < T + 3 * 64 * kUnroll <= T + kColPad)
            if (lane == 0) s_wrec[wave][__popcll(nz)] = make_uint2(a.col_pad - T, 2u);
            // -- sweep the T concatenated wedges, kUnroll windows of 64 per step;
            // the entries of step j + 1 are loaded before the adds of step j
            uint32_t before = 0;
            uint32_t xa[kUnroll], aa[kUnroll];
            // Every position has an owner (the sentinel from T on), so no
            // lane needs a bound check.
            auto step_load = [&](uint32_t j, uint32_t* x, uint32_t* aux) {
                uint8_t* hb = (uint8_t*)s_head[wave];
                if (len > 0 && excl >= j && excl < j + 64 * kUnroll) {
                    const uint32_t hp = excl - j;
                    hb[(hp & 63u) * kUnroll + (hp >> 6)] = 1;
                }
                if (lane == 0 && T >= j && T < j + 64 * kUnroll) {
                    const uint32_t hp = T - j;
                    hb[(hp & 63u) * kUnroll + (hp >> 6)] = 1;
                }
                __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
                const uint32_t hd4 = s_head[wave][lane];
                uint32_t adj[kUnroll];
#pragma unroll
                for (uint32_t u = 0; u < kUnroll; ++u) {
                    // owner = heads before the window + heads at or before this
                    // lane - 1; the heads of lanes 1..lane are the bits below
                    // this lane of M >> 1 (one mbcnt), lane 0's is scalar
                    const bool own = ((hd4 >> (8 * u)) & 0xFFu) != 0;
                    const u64 M = __ballot(own);
                    const u64 Ms = M >> 1;
                    const uint32_t upto = __builtin_amdgcn_mbcnt_hi(
                        (uint32_t)(Ms >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)Ms, 0u));
                    const uint32_t idx = (before + (uint32_t)(M & 1u) - 1u) + upto;
                    before += (uint32_t)__popcll(M);
                    const uint2 r = s_wrec[wave][idx];
                    adj[u] = r.x;
                    aux[u] = r.y;
                }
#pragma unroll
                for (uint32_t u = 0; u < kUnroll; ++u) x[u] = col[adj[u] + j + u * 64 + lane];
                __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
                s_head[wave][lane] = 0;
                // keep the previous step's adds below these loads: hoisted
                // above them they would wait for that step's entries first
                __builtin_amdgcn_sched_barrier(0);
            };
            // the adds of one step; false (for the whole wave) when a hashed
            // table found no room
            auto step_add = [&](const uint32_t* x, const uint32_t* aux) -> bool {
                if (!HASH) {
                    // No branches: the pad entries past a grab's end (end
                    // vertex 2^31 - 1) fall on the junk word behind the table.
                    // An entry x = w << 1 | sign(v, w) adds 1 to the l half of
                    // w's counter, or to the m half when sign(v, w) differs
                    // from the record's sign(u, v), s1.  With y = x ^ s1, bit 0
                    // of y selects the half, and the bits above it the end's
                    // slot in a packed word (dlo is a multiple of kTile, so
                    // w's low bits give the slot): the field is y's low
                    // 1 / 2 / 3 bits, each field 16 / 8 / 4 bits wide.
#pragma unroll
                    for (uint32_t u = 0; u < kUnroll; ++u) {
                        const uint32_t y = x[u] ^ aux[u];
                        if (DK == kD32) {
                            const uint32_t at = min((x[u] >> 1) - dlo, junk64);
                            atomicAdd(&s_tab[at], (u64)1 << ((y & 1u) << 5));
                        } else if (DK == kD16) {
                            const uint32_t at = min((x[u] >> 1) - dlo, junk32);
                            atomicAdd(&s32[at], 1u << ((y & 1u) << 4));
                        } else if (DK == kD8) {
                            const uint32_t at = min((x[u] >> 2) - (dlo >> 1), junk32);
                            atomicAdd(&s32[at], 1u << ((y & 3u) << 3));
                        } else {
                            const uint32_t at = min((x[u] >> 3) - (dlo >> 2), junk32);
                            atomicAdd(&s32[at], 1u << ((y & 7u) << 2));
                        }
                    }
                    return true;
                }
                bool lok = true;
                if (h16) {
                    // The first probes of the step's windows go together, so
                    // that their key reads, and then their inserts, wait for
                    // LDS once; an entry whose first slot holds another key
                    // probes on from the second slot.  (The sentinel's pad
                    // entries take no part.)
                    uint32_t sl[kUnroll], kk[kUnroll];
#pragma unroll
                    for (uint32_t u = 0; u < kUnroll; ++u) {
                        sl[u] = hash32(x[u] >> 1) >> (32 - kHash16Log2);
                        kk[u] = s32[sl[u]];
                    }
#pragma unroll
                    for (uint32_t u = 0; u < kUnroll; ++u) {
                        if ((aux[u] & 2u) == 0 && kk[u] == kEmpty) {
                            const uint32_t o = atomicCAS(&s32[sl[u]], kEmpty, x[u] >> 1);
                            kk[u] = o == kEmpty ? x[u] >> 1 : o;
                        }
                    }
#pragma unroll
                    for (uint32_t u = 0; u < kUnroll; ++u) {
                        if (aux[u] & 2u) continue;
                        const uint32_t w = x[u] >> 1;
                        const uint32_t inc = ((x[u] ^ aux[u]) & 1u) ? 0x10000u : 1u;
                        if (kk[u] == w)
                            atomicAdd(&s32[kHash16Slots + sl[u]], inc);
                        else if (lok)
                            lok = bucket_add16(s32, lim, w, inc, 1);
                    }
                    return __ballot(!lok) == 0;
                }
#pragma unroll
                for (uint32_t u = 0; u < kUnroll; ++u) {
                    if ((aux[u] & 2u) || !lok) continue;
                    lok = add_one(x[u] >> 1, ((x[u] ^ aux[u]) & 1u) != 0);
                }
                return __ballot(!lok) == 0;
            };
            // two register sets take turns (no copies: a copy of a value still
            // being loaded would wait for the load); the step after the last
            // is loaded too (pad entries), which keeps the loads out of branches
            uint32_t xb[kUnroll], ab[kUnroll];
            bool ok = true;
            bool tiles_pending = nxt_base != kEmpty;  // uniform
            if (T > 0) {
                // Steps go in pairs (a, then b) with one exit, after b: an
                // exit after a would leave b's loads pending on a path back
                // to the loop head as the wait-count analysis sees it, and
                // every step would then wait for the previous step's loads
                // before reusing their registers.  An odd number of steps
                // peels the first one.
                constexpr uint32_t S = 64 * kUnroll;
                const uint32_t nsteps = (T + S - 1) / S;
                uint32_t j = 0;
                if (nsteps & 1u) {
                    step_load(0, xb, ab);
                    step_load(S, xa, aa);  // (past T when nsteps == 1: pad entries)
                    if (tiles_pending) {
                        load_tiles(nxt);  // the next grab's records have arrived
                        tiles_pending = false;
                    }
                    ok = step_add(xb, ab);
                    j = S;
                } else {
                    step_load(0, xa, aa);
                }
                if (j < T && ok) {
                    for (;;) {
                        step_load(j + S, xb, ab);
                        if (tiles_pending) {
                            load_tiles(nxt);
                            tiles_pending = false;
                        }
                        ok = step_add(xa, aa) && ok;
                        step_load(j + 2 * S, xa, aa);
                        ok = step_add(xb, ab) && ok;
                        j += 2 * S;
                        if (j >= T || !ok) break;
                    }
                }
            }
            if (!ok) s_abort = 1;  // the piece is abandoned
            __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
            // the next grab: loaded above, or claimed now
            if (nxt_base != kEmpty) {
                if (tiles_pending) load_tiles(nxt);
                cur = nxt;
                cur_base = nxt_base;
            } else {
                uint32_t nb = 0;
                if (lane == 0) nb = atomicAdd(&s_batch, bsz);
                cur_base = __shfl(nb, 0, 64);
                if (cur_base < total) {
                    load_rec(cur_base, cur);
                    load_tiles(cur);
                }
            }
            have = cur_base < total && !(HASH && s_abort);
        }
        };
        if constexpr (!HASH) {
            if (dk == kD16)
                records(std::integral_constant<int, kD16>());
            else if (dk == kD8)
                records(std::integral_constant<int, kD8>());
            else if (dk == kD4)
                records(std::integral_constant<int, kD4>());
            else
                records(std::integral_constant<int, kD32>());
        } else {
            records(std::integral_constant<int, kD32>());
        }
        // -- the bucketed wedges through short middle rows (split starts);
        // the next chunk's entries are loaded before the current chunk's adds
        if (partial && P.list != kEmpty) {
            const uint32_t b0 = a.sw_off[P.list];
            const uint32_t n_sw = a.sw_off[P.list + 1] - b0;
            auto take = [&]() {
                uint32_t c = 0;
                if (lane == 0) c = atomicAdd(&s_swtake, 64 * kUnroll);
                return __shfl(c, 0, 64);
            };
            auto load = [&](uint32_t c, uint32_t* x) {
#pragma unroll
                for (uint32_t u = 0; u < kUnroll; ++u) {
                    const uint32_t q = c + u * 64 + lane;
                    const uint32_t v = a.sw_list[b0 + (q < n_sw ? q : 0u)];
                    x[u] = q < n_sw ? v : kEmpty;
                }
            };
            auto add = [&](const uint32_t* x) -> bool {
                bool lok = true;
#pragma unroll
                for (uint32_t u = 0; u < kUnroll; ++u) {
                    if (x[u] == kEmpty || !lok) continue;
                    const uint32_t w = x[u] >> 1;
                    if (w < plo || w >= phi) continue;
                    lok = add_one(w, (x[u] & 1u) != 0);
                }
                return !HASH || __ballot(!lok) == 0;
            };
            uint32_t xa[kUnroll], xb[kUnroll];
            uint32_t c = (n_sw > 0 && !(HASH && s_abort)) ? take() : n_sw;
            bool ok = true;
            if (c < n_sw) {
                load(c, xa);
                for (;;) {
                    c = take();
                    load(c, xb);  // past the end: all lanes marked empty
                    ok = add(xa);
                    if (c >= n_sw || !ok) break;
                    c = take();
                    load(c, xa);
                    ok = add(xb);
                    if (c >= n_sw || !ok) break;
                }
            }
            if (!ok) s_abort = 1;
        }
        // the first wave done takes the next item and fetches its piece
        {
            uint32_t f = 1;
            if (lane == 0) f = atomicAdd(&s_done, 1u);
            if (lane == 0 && f == 0) {
                const uint32_t nx = fetch();
                if (nx != kEmpty) {
                    s_pf = a.pieces[a.order[nx]];
                    s_pf_item = nx;
                }
                s_next = nx;
                s_nextok = 1;
            }
        }
        __syncthreads();
        // -- queued chunks of long sub-intervals: one wave per chunk
        if (s_qn > 0 && !(HASH && s_abort)) {
            for (;;) {
                uint32_t c = 0;
                if (lane == 0) c = atomicAdd(&s_qtake, 1u);
                c = __shfl(c, 0, 64);
                if (c >= s_qn || (HASH && s_abort)) break;
                const uint32_t adj = s_qadj[c], qlen = s_qlen[c], aux = s_qaux[c];
                auto load = [&](uint32_t e0, uint32_t* x) {
#pragma unroll
                    for (uint32_t u = 0; u < kUnroll; ++u) {
                        const uint32_t e = e0 + u * 64 + lane;
                        const uint32_t v = col[adj + (e < qlen ? e : 0u)];
                        x[u] = e < qlen ? v : kEmpty;
                    }
                };
                auto add = [&](const uint32_t* x) -> bool {
                    bool lok = true;
#pragma unroll
                    for (uint32_t u = 0; u < kUnroll; ++u) {
                        if (x[u] == kEmpty || !lok) continue;
                        const uint32_t w = x[u] >> 1;
                        lok = add_one(w, ((x[u] ^ aux) & 1u) != 0);
                    }
                    return !HASH || __ballot(!lok) == 0;
                };
                uint32_t xa[kUnroll], xb[kUnroll];
                bool ok = true;
                load(0, xa);
                for (uint32_t e0 = 0;;) {
                    e0 += 64 * kUnroll;
                    load(e0, xb);
                    ok = add(xa);
                    if (e0 >= qlen || !ok) break;
                    e0 += 64 * kUnroll;
                    load(e0, xa);
                    ok = add(xb);
                    if (e0 >= qlen || !ok) break;
                }
                if (!ok) s_abort = 1;
            }
        }
        __syncthreads();  // every wave is done with the piece's wedges; s_abort is final
        const bool aborted = HASH && s_abort;
        // -- finalize: C(l,2) + C(m,2) and l*m over the range
        u64 bal = 0, unb = 0;
        if (aborted) {
            // counts abandoned: the piece is redone in halves by k_wedge
        } else if (HASH && h16) {
            // counters of empty slots are zero; l + m < 2^16 (a start with
            // fewer than 2^16 middles)
            const uint4* c4 = reinterpret_cast<const uint4*>(s32 + kHash16Slots);
            u64 q2 = 0, lm2 = 0;
            for (uint32_t g = tid; g < kHash16Slots / 4; g += kWedgeThreads) {
                const uint4 c = c4[g];
                bucket16_sums(c.x, q2, lm2);
                bucket16_sums(c.y, q2, lm2);
                bucket16_sums(c.z, q2, lm2);
                bucket16_sums(c.w, q2, lm2);
            }
            bal = q2 >> 1;
            unb = lm2 >> 1;
        } else if (HASH) {
            const ulonglong2* v2 = reinterpret_cast<const ulonglong2*>(hvals);
            for (uint32_t g = tid; g < kHashSlots / 2; g += kWedgeThreads) {
                const ulonglong2 c = v2[g];
                const u64 cc[2] = {c.x, c.y};
#pragma unroll
                for (int k = 0; k < 2; ++k) {
                    const u64 l = cc[k] & 0xFFFFFFFFull, mm = cc[k] >> 32;
                    bal += choose2(l) + choose2(mm);
                    unb += l * mm;
                }
            }
        } else if (dk == kD8 || dk == kD4) {
            // packed halves: per-word sums stay far below 2^32 (at most
            // 4 * 255^2 per word), summed per group of four words into 64 bits
            const uint4* t4 = reinterpret_cast<const uint4*>(s32);
            const uint32_t groups = (((dwidth + (1u << wlog) - 1u) >> wlog) + 3) / 4;
            uint32_t q = 0, sl = 0, lm = 0;
            for (uint32_t g = tid; g < groups; g += kWedgeThreads) {
                const uint4 c = t4[g];
                if (dk == kD8) {
                    bucket8_acc(c.x, q, sl, lm);
                    bucket8_acc(c.y, q, sl, lm);
                    bucket8_acc(c.z, q, sl, lm);
                    bucket8_acc(c.w, q, sl, lm);
                } else {
                    bucket4_acc(c.x, q, sl, lm);
                    bucket4_acc(c.y, q, sl, lm);
                    bucket4_acc(c.z, q, sl, lm);
                    bucket4_acc(c.w, q, sl, lm);
                }
            }
            bal = (q - sl) >> 1;
            unb = lm;
        } else if (d16 && !(P.flags & kPieceMerge)) {
            // 2 (C(l,2) + C(m,2)) and 2 l m from dot products of the halves
            // (l + m < 2^16); entries past the range and unreached ones are zero
            const uint4* t4 = reinterpret_cast<const uint4*>(s32);
            u64 q2 = 0, lm2 = 0;
            for (uint32_t g = tid; g < (dwidth + 3) / 4; g += kWedgeThreads) {
                const uint4 c = t4[g];
                bucket16_sums(c.x, q2, lm2);
                bucket16_sums(c.y, q2, lm2);
                bucket16_sums(c.z, q2, lm2);
                bucket16_sums(c.w, q2, lm2);
            }
            bal = q2 >> 1;  // every term is even: l(l-1) + m(m-1) and 2lm
            unb = lm2 >> 1;
        } else if (!(P.flags & kPieceMerge)) {
            const ulonglong2* t2 = reinterpret_cast<const ulonglong2*>(s_tab);
            for (uint32_t g = tid; g < (dwidth + 1) / 2; g += kWedgeThreads) {
                const ulonglong2 c = t2[g];
                const u64 cc[2] = {c.x, c.y};
#pragma unroll
                for (int k = 0; k < 2; ++k) {
                    const u64 l = cc[k] & 0xFFFFFFFFull, mm = cc[k] >> 32;
                    bal += choose2(l) + choose2(mm);
                    unb += l * mm;
                }
            }
        } else {
            const uint32_t gb = P.gbase;
            for (uint32_t i = tid; i < dwidth; i += kWedgeThreads) {
                u64 v;
                if (d16) {
                    const uint32_t c = s32[i];
                    v = (c & 0xFFFFu) | ((u64)(c >> 16) << 32);
                } else {
                    v = s_tab[i];
                }
                if (v == 0) continue;
                const u64 l = v & 0xFFFFFFFFull, m = v >> 32;
                bal += choose2(l) + choose2(m);
                unb += l * m;
                const u64 old = atomicAdd(&a.G[(uint64_t)gb + i], v);
                const u64 ol = old & 0xFFFFFFFFull, om = old >> 32;
                bal += ol * l + om * m;
                unb += ol * m + om * l;
            }
        }
        bal = wave_reduce_sum(bal);
        unb = wave_reduce_sum(unb);
        if (lane == 0) {
            s_red[0][wave] = bal;
            s_red[1][wave] = unb;
        }
        __syncthreads();
        if (tid == 0) {
            u64 sb = 0, su = 0;
            for (uint32_t w = 0; w < kWaves; ++w) {
                sb += s_red[0][w];
                su += s_red[1][w];
            }
            if (!aborted) {
                s_acc.add(a, P.graph, sb, su);
            } else {
                // redo as the two halves of its tile run, or, for a single tile,
                // with dense counters (which always fit): k_wedge runs them
                atomicAdd(&a.ctl->resplits, 1ull);
                Piece Q = s_p;
                if (!(Q.flags & kPiecePartial)) {
                    atomicOr(&a.ctl->internal_err, 1u);  // cannot happen by construction
                } else if (Q.t1 - Q.t0 > 1) {
                    const uint32_t tm = (Q.t0 + Q.t1) >> 1;
                    Piece hi = Q;
                    hi.t0 = tm;
                    hi.lo = tm * kTile;
                    Q.t1 = tm;
                    Q.hi = min(Q.hi, tm * kTile);
                    const uint32_t r = atomicAdd(&a.ctl->redo_n, 2u);
                    a.redo[r] = Q;
                    a.redo[r + 1] = hi;
                } else {
                    Q.flags |= kPieceDense;
                    a.redo[atomicAdd(&a.ctl->redo_n, 1u)] = Q;
                }
            }
            const uint32_t nx = s_nextok ? s_next : fetch();
            s_item = nx;
            if (nx != kEmpty) s_p = (s_pf_item == nx) ? s_pf : a.pieces[a.order[nx]];
        }
    }
    if (tid == 0) s_acc.flush(a);
}


// ---------------------------------------------------------------------------
// One-wave pieces (k_wedge_wave): a start with at most kWaveMaxW wedges whose
// end vertices [lo, S) fit kWaveWords packed counters is counted by one wave
// alone, in a slice of the workgroup's LDS: the wave clears its slice, sweeps
// the start's records 64 at a time (each record's whole prefix, the same
// concatenated sweep as k_wedge_pieces: head flags, a sentinel past the end,
// steps in pairs), and sums C(l,2) + C(m,2) and l m over its slice.  Waves take
// pieces from a global counter and never wait for one another (Section 4.1's
// per-start buckets, one start per wavefront).
__global__ __launch_bounds__(kWedgeThreads) void k_wedge_wave(WedgeArgs a) {
    // per wave: kWaveWords counters, then 64 junk words for the lanes past a
    // grab's end (and, with invalid input, for ends outside the range)
    constexpr uint32_t kSlice = kWaveWords + 64;
    __shared__ __align__(16) uint32_t s_cnt[kWaves * kSlice];
    __shared__ uint2 s_rec[kWaves][65];
    __shared__ uint32_t s_hd[kWaves][64];
    const uint32_t lane = lane_id();
    const uint32_t wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    uint32_t* slice = s_cnt + wave * kSlice;
    const uint32_t junk = kWaveWords + lane;  // relative to slice
    const uint32_t* __restrict__ col = a.col;
    const u64 le_mask = ~0ull >> (63 - lane);
    const uint32_t first = a.n_heavy - a.n_wave;
    uint32_t g = 0;
    u64 bal = 0, unb = 0;  // this wave's totals for graph g
    auto flush = [&]() {
        if (lane == 0 && (bal | unb)) {
            u64* dst = a.gres ? a.gres + 4ull * g : &a.ctl->balanced;
            atomicAdd(dst, bal);
            atomicAdd(dst + 1, unb);
        }
        bal = unb = 0;
    };
    s_hd[wave][lane] = 0;
    // a wave takes runs of G consecutive pieces (most expensive first): one
    // atomic per run keeps the shared counter cold when there are millions of
    // small pieces, and runs of 1 balance the few large ones
    const uint32_t G = max(1u, a.n_wave / (gridDim.x * kWaves * 8u));
    uint32_t it = 0, it_end = 0;
    for (;;) {
        if (it == it_end) {
            uint32_t b = 0;
            if (lane == 0) b = atomicAdd(&a.ctl->queue_wave, G);
            it = __builtin_amdgcn_readfirstlane(__shfl(b, 0, 64));
            if (it >= a.n_wave) break;
            it_end = min(it + G, a.n_wave);
        }
        const Piece* pp = a.pieces + a.order[first + it];
        ++it;
        const uint32_t rec0 = __builtin_amdgcn_readfirstlane(pp->rec0);
        const uint32_t nrec = __builtin_amdgcn_readfirstlane(pp->nrec);
        const uint32_t dlo = __builtin_amdgcn_readfirstlane(pp->lo);
        const uint32_t dhi = __builtin_amdgcn_readfirstlane(pp->hi);
        const uint32_t flags = __builtin_amdgcn_readfirstlane(pp->flags);
        const uint32_t graph = __builtin_amdgcn_readfirstlane(pp->graph);
        const int dk = (flags & kPieceDense4) ? kD4 : (flags & kPieceDense8) ? kD8 : kD16;
        const uint32_t wlog = dk == kD4 ? 2u : dk == kD8 ? 1u : 0u;
        const uint32_t groups = (((dhi - dlo + (1u << wlog) - 1u) >> wlog) + 3u) / 4u;
        if (groups > kWaveWords / 4 || dhi <= dlo) {  // cannot happen by construction
            if (lane == 0) atomicOr(&a.ctl->internal_err, 16u);
            continue;
        }
        // the first 64 records load while the slice is cleared
        auto load_rec = [&](uint32_t base, uint32_t& rs, uint32_t& pos, uint32_t& s1) {
            const bool act = base + lane < nrec;
            const uint4 rc = a.recs[rec0 + (act ? base + lane : 0u)];
            rs = rc.x;
            pos = act ? rc.y >> 1 : 0u;
            s1 = rc.y & 1u;
        };
        uint32_t rs, pos, s1;
        load_rec(0, rs, pos, s1);
        uint4* s4 = reinterpret_cast<uint4*>(slice);
        for (uint32_t i = lane; i < groups; i += 64) s4[i] = make_uint4(0, 0, 0, 0);
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        auto sweep = [&](auto dktag) {
            constexpr int DK = decltype(dktag)::value;
            for (uint32_t base = 0; base < nrec; base += 64) {
                // next 64 records, loaded during this sweep
                uint32_t nrs = 0, npos = 0, ns1 = 0;
                if (base + 64 < nrec) load_rec(base + 64, nrs, npos, ns1);
                const uint32_t len = pos;
                const u64 nz = __ballot(len > 0);
                const uint32_t excl = wave_incl_scan(len) - len;
                const uint32_t T = __builtin_amdgcn_readfirstlane(__shfl(excl + len, 63, 64));
                if (len > 0) s_rec[wave][__popcll(nz & (le_mask >> 1))] = make_uint2(rs - excl, s1);
                if (lane == 0) s_rec[wave][__popcll(nz)] = make_uint2(a.col_pad - T, 2u);
                uint32_t before = 0;
                auto step_load = [&](uint32_t j, uint32_t* x, uint32_t* aux) {
                    uint8_t* hb = (uint8_t*)s_hd[wave];
                    if (len > 0 && excl >= j && excl < j + 64 * kUnroll) {
                        const uint32_t hp = excl - j;
                        hb[(hp & 63u) * kUnroll + (hp >> 6)] = 1;
                    }
                    if (lane == 0 && T >= j && T < j + 64 * kUnroll) {
                        const uint32_t hp = T - j;
                        hb[(hp & 63u) * kUnroll + (hp >> 6)] = 1;
                    }
                    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
                    const uint32_t hd4 = s_hd[wave][lane];
                    uint32_t adj[kUnroll];
#pragma unroll
                    for (uint32_t u = 0; u < kUnroll; ++u) {
                        const bool own = ((hd4 >> (8 * u)) & 0xFFu) != 0;
                        const u64 M = __ballot(own);
                        const u64 Ms = M >> 1;
                        const uint32_t upto = __builtin_amdgcn_mbcnt_hi(
                            (uint32_t)(Ms >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)Ms, 0u));
                        const uint32_t idx = (before + (uint32_t)(M & 1u) - 1u) + upto;
                        before += (uint32_t)__popcll(M);
                        const uint2 r = s_rec[wave][idx];
                        adj[u] = r.x;
                        aux[u] = r.y;
                    }
#pragma unroll
                    for (uint32_t u = 0; u < kUnroll; ++u) x[u] = col[adj[u] + j + u * 64 + lane];
                    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
                    s_hd[wave][lane] = 0;
                    __builtin_amdgcn_sched_barrier(0);
                };
                auto step_add = [&](const uint32_t* x, const uint32_t* aux) {
#pragma unroll
                    for (uint32_t u = 0; u < kUnroll; ++u) {
                        const uint32_t y = x[u] ^ aux[u];
                        if (DK == kD16) {
                            const uint32_t at = min((x[u] >> 1) - dlo, junk);
                            atomicAdd(&slice[at], 1u << ((y & 1u) << 4));
                        } else if (DK == kD8) {
                            const uint32_t at = min((x[u] >> 2) - (dlo >> 1), junk);
                            atomicAdd(&slice[at], 1u << ((y & 3u) << 3));
                        } else {
                            const uint32_t at = min((x[u] >> 3) - (dlo >> 2), junk);
                            atomicAdd(&slice[at], 1u << ((y & 7u) << 2));
                        }
                    }
                };
                if (T > 0) {
                    constexpr uint32_t S = 64 * kUnroll;
                    const uint32_t nsteps = (T + S - 1) / S;
                    uint32_t xa[kUnroll], aa[kUnroll], xb[kUnroll], ab[kUnroll];
                    uint32_t j = 0;
                    if (nsteps & 1u) {
                        step_load(0, xb, ab);
                        step_load(S, xa, aa);
                        step_add(xb, ab);
                        j = S;
                    } else {
                        step_load(0, xa, aa);
                    }
                    if (j < T) {
                        for (;;) {
                            step_load(j + S, xb, ab);
                            step_add(xa, aa);
                            step_load(j + 2 * S, xa, aa);
                            step_add(xb, ab);
                            j += 2 * S;
                            if (j >= T) break;
                        }
                    }
                }
                __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
                rs = nrs;
                pos = npos;
                s1 = ns1;
            }
        };
        if (dk == kD16)
            sweep(std::integral_constant<int, kD16>());
        else if (dk == kD8)
            sweep(std::integral_constant<int, kD8>());
        else
            sweep(std::integral_constant<int, kD4>());
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        // finalize over the slice: 2 (C(l,2) + C(m,2)) and 2 l m
        u64 q2 = 0, lm2 = 0;
        for (uint32_t i = lane; i < groups; i += 64) {
            const uint4 c = s4[i];
            if (dk == kD16) {
                bucket16_sums(c.x, q2, lm2);
                bucket16_sums(c.y, q2, lm2);
                bucket16_sums(c.z, q2, lm2);
                bucket16_sums(c.w, q2, lm2);
            } else {
                uint32_t q = 0, sl = 0, lm = 0;
                if (dk == kD8) {
                    bucket8_acc(c.x, q, sl, lm);
                    bucket8_acc(c.y, q, sl, lm);
                    bucket8_acc(c.z, q, sl, lm);
                    bucket8_acc(c.w, q, sl, lm);
                } else {
                    bucket4_acc(c.x, q, sl, lm);
                    bucket4_acc(c.y, q, sl, lm);
                    bucket4_acc(c.z, q, sl, lm);
                    bucket4_acc(c.w, q, sl, lm);
                }
                q2 += q - sl;
                lm2 += 2ull * lm;
            }
        }
        q2 = wave_reduce_sum(q2);
        lm2 = wave_reduce_sum(lm2);
        if (graph != g) {
            flush();
            g = graph;
        }
        bal += q2 >> 1;
        unb += lm2 >> 1;
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");  // the slice's reads before the next clear
    }
    flush();
}

// per-vertex output by input vertex id: out[x] = count of x's row
__global__ void k_pv_out(const u64* __restrict__ pv, const uint32_t* __restrict__ sidx_of, Dims d,
                         u64* __restrict__ out) {
    for (uint32_t x = blockIdx.x * blockDim.x + threadIdx.x; x < d.n; x += gridDim.x * blockDim.x)
        out[x] = pv[d.base[x >= d.n_u ? 1u : 0u] + sidx_of[x]];
}

hipError_t launch_pv_out(const u64* pv, const uint32_t* sidx_of, Dims d, u64* out, hipStream_t st) {
    uint32_t blocks = (d.n + 255) / 256;
    if (blocks > 16384) blocks = 16384;
    if (blocks == 0) blocks = 1;
    hipLaunchKernelGGL(k_pv_out, dim3(blocks), dim3(256), 0, st, pv, sidx_of, d, out);
    return hipGetLastError();
}

// Plain count: the dense heavy items (0..n_dense-1) run in k_wedge_pieces<false>,
// the hashed ones in k_wedge_pieces<true>, then the light items and the halves
// of hashed pieces redone in k_wedge; per-vertex mode runs every item in
// k_wedge<true>.
hipError_t launch_wedge(const Piece* pieces, const uint32_t* order, const uint32_t* items_first,
                        uint32_t n_heavy, uint32_t n_dense, uint32_t n_wave, Piece* redo,
                        uint32_t n_items, const uint4* recs, const uint32_t* col, const uint32_t* tb,
                        Dims d, const uint32_t first_long[2], u64* G, const uint32_t* sw_off,
                        const uint32_t* sw_list, const uint32_t* sw_mid, Control* ctl, u64* gres,
                        u64* pv, uint32_t col_pad,
                        uint32_t num_cus, hipStream_t st) {
    WedgeArgs a;
    a.col_pad = col_pad;
    a.pieces = pieces;
    a.order = order;
    a.items_first = items_first;
    a.n_heavy = n_heavy;
    a.n_items = n_items;
    a.recs = recs;
    a.col = col;
    a.tb = tb;
    a.d = d;
    a.first_long[0] = first_long[0];
    a.first_long[1] = first_long[1];
    a.G = G;
    a.sw_off = sw_off;
    a.sw_list = sw_list;
    a.sw_mid = sw_mid;
    a.ctl = ctl;
    a.gres = gres;
    a.pv = pv;
    a.n_dense = pv ? 0 : n_dense;
    a.n_wave = pv ? 0 : n_wave;
    a.item0 = pv ? 0 : n_heavy;
    a.redo = pv ? nullptr : redo;
    if (!pv && n_dense > 0) {
        const uint32_t grid = min(num_cus, n_dense);
        hipLaunchKernelGGL(k_wedge_pieces<false>, dim3(grid), dim3(kWedgeThreads), 0, st, a);
    }
    if (!pv && n_heavy - n_wave > n_dense) {
        const uint32_t grid = min(num_cus, n_heavy - n_wave - n_dense);
        hipLaunchKernelGGL(k_wedge_pieces<true>, dim3(grid), dim3(kWedgeThreads), 0, st, a);
    }
    if (!pv && n_wave > 0) {
        const uint32_t grid = min(num_cus, (n_wave + kWaves - 1) / kWaves);
        hipLaunchKernelGGL(k_wedge_wave, dim3(grid), dim3(kWedgeThreads), 0, st, a);
    }
    // light items, and any halves the hashed pieces left
    const uint32_t rest = n_items - a.item0;
    uint32_t grid = num_cus;
    if (grid > rest && (pv || n_heavy - n_wave == n_dense)) grid = rest;  // (no redo possible)
    if (grid == 0) return hipGetLastError();
    if (pv)
        hipLaunchKernelGGL(k_wedge<true>, dim3(grid), dim3(kWedgeThreads), 0, st, a);
    else
        hipLaunchKernelGGL(k_wedge<false>, dim3(grid), dim3(kWedgeThreads), 0, st, a);
    return hipGetLastError();
}

}  // namespace bbc
