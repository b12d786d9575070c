// Internal definitions shared by the HIP sources of libbbc (not installed).
//
// Vocabulary (paper: Sections 2-4):
//   * side 0 is U, side 1 is V; a vertex's "sidx" is its position among the
//     vertices of its own side in ascending priority order, the priority being
//     (degree, global id) with global ids U = 0..n_u-1, V = n_u..n-1
//     (Definition 4).  Within one side sidx order equals priority order.
//   * the CSR holds one row per vertex: rows 0..n_u-1 are U vertices by sidx,
//     rows n_u..n-1 are V vertices by sidx.  An entry is (sidx(nbr) << 1) | neg,
//     neg = 1 for a negative edge; every row is sorted ascending, i.e. by the
//     neighbour's priority (the sorted adjacency of Algorithm 2).
//   * cross(x) = number of vertices of the other side with lower priority than
//     x: a neighbour y of x is a valid middle vertex (p(y) < p(x)) iff
//     sidx(y) < cross(x).  A same-side end vertex w is valid (p(w) < p(x)) iff
//     sidx(w) < sidx(x).
//   * a "record" is an edge oriented from its higher-priority end u (the wedge
//     start) to its lower one v (the middle): it stores where row v starts and
//     pos = |{w in Gamma(v) : p(w) < p(u)}|, so the wedges (u, v, .) are the
//     first pos entries of row v.  A start's records with a long middle row
//     (more than kLongDeg entries) come first, those with a short one last.
//   * batches: many graphs are counted as one disjoint union.  The priority
//     sort key is (graph, degree, id), so each graph's vertices form one
//     contiguous sidx block per side (blk[side][g] .. blk[side][g+1]) and
//     priorities are only ever compared inside a graph, exactly as when the
//     graph is counted alone.  A start's end vertices are then the sidx range
//     [block start, sidx(u)), and every piece carries its graph's index.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace bbc {

typedef unsigned long long u64;

constexpr uint32_t kEmpty = 0xFFFFFFFFu;
constexpr u64 kEmpty64 = ~0ull;
constexpr uint32_t kNoTile = 0xFFFFFFFFu;

// ---- degree classes used by the row sort and the record builder ----------
// thresholds on row length; class c holds rows with kClassHi[c-1] < len <= kClassHi[c]
constexpr int kNumClassBounds = 6;
__host__ __device__ constexpr uint32_t class_hi(int c) {
    return c == 0 ? 1u : c == 1 ? 8u : c == 2 ? 16u : c == 3 ? 32u : c == 4 ? 64u : 4096u;
}
constexpr uint32_t kLongDeg = 64;            // rows longer than this carry a tile table
constexpr uint32_t kBitmapChunk = 1u << 18;  // sidx span handled per block by the big-row sort

// ---- wedge kernel geometry -------------------------------------------------
constexpr int kWedgeThreads = 1024;
constexpr uint32_t kDenseW = 16384;           // dense counters per item (u64 each, 128 KiB)
constexpr uint32_t kHashSlots = 8192;         // hash slots (u32 key + u64 counters)
constexpr uint32_t kLightMax = kHashSlots / 4;     // max wedges of a batched (light) start
constexpr uint32_t kMinRegion = 64;
// Light item i holds the light starts whose region offset lies in [iH, iH+H)
// with H = kLightWindow16; a region is at most 2 * kLightMax slots, so the
// item's regions end below H + 2 * kLightMax = 2 * kHashSlots, the size of the
// table of u32 keys and u32 counters (l | m << 16; a light start has at most
// kLightMax < 2^16 wedges, so no count can reach 2^16).
constexpr uint32_t kLightWindow16 = 2 * kHashSlots - 2 * kLightMax;
// offsets of one window lie at least kMinRegion apart
constexpr uint32_t kMaxItemPieces = kLightWindow16 / kMinRegion + 1;
constexpr uint32_t kTile = 16384;             // end-vertex tile width (sidx units)
// The CSR column array carries kColPad entries of kColPadValue past its 2m
// entries: the wedge sweep points the lanes past the end of a grab there, and
// that end vertex lies outside every counter table.
constexpr uint32_t kColPad = 1024;
constexpr uint32_t kColPadValue = 0xFFFFFFFEu;
constexpr u64 kRecordChunkWedges = 65536;     // min wedges per record chunk of a small-side start
constexpr uint32_t kChunkDiv = 2048;          // ... and at least W_total / kChunkDiv
constexpr uint32_t kBatchSide = kDenseW;          // batches: graphs up to this many vertices
constexpr uint64_t kBatchMaxEdges = 1ull << 30;   //   per side share one union of at most
constexpr uint64_t kBatchMaxVertices = 1ull << 29;  //   these many edges, vertices, graphs
constexpr uint32_t kBatchMaxGraphs = 1u << 17;
constexpr uint32_t kDefaultHashTarget = 4096;   // expected wedges per hashed run of tiles
constexpr uint32_t kDefaultProbeLimit = 256;    // probes before a split hashed piece gives up

// piece flags
constexpr uint32_t kPieceDense = 1u;    // counters addressed by w - lo (else hashed)
constexpr uint32_t kPieceMerge = 2u;    // partial counts: merge exactly through G
constexpr uint32_t kPiecePartial = 4u;  // w-range is a tile range: look up sub-intervals
constexpr uint32_t kPieceSideV = 8u;    // the start vertex lies on side V
constexpr uint32_t kPieceDense16 = 16u; // dense with 16-bit l | m halves (two tiles wide)
constexpr uint32_t kPieceHash16 = 32u;  // hashed with 16-bit l | m halves (2 x kHashSlots slots)
// Packed dense counters.  l + m <= |N(u) & N(w)| <= deg(w), so over end
// vertices of degree at most 2^b - 1 both counts fit in b bits: a u32 word
// then holds 32 / 2b end vertices and one 128 KiB table spans more tiles.
constexpr uint32_t kPieceDense8 = 64u;   // l | m << 8 per end vertex, two per word (four tiles)
constexpr uint32_t kPieceDense4 = 128u;  // l | m << 4 per end vertex, four per word (eight tiles)
constexpr uint32_t kDensePacked = kPieceDense8 | kPieceDense4;
constexpr uint32_t kPieceWave = 256u;  // counted by one wave alone (k_wedge_wave)
// One-wave pieces: each wave of a workgroup owns kWaveWords u32 counters
// (l | m halves of 16, 8 or 4 bits, so 1, 2 or 4 end vertices per word), and
// takes starts of at most kWaveMaxW wedges whose cost W_u + kWaveRecordCost
// k_u is at most W / wave_share of a count's W wedges (but at least kWaveMinW
// and at most kWaveMaxCost; default share kWaveShare): one wave alone counts a
// start, so a start much larger than a wave's share of the count would leave
// the wave working long after the others are done, and one above
// kWaveMaxCost is counted faster by a workgroup (measured on the batched
// workload: wedge step 34.3 -> 31.6 ms)
constexpr uint32_t kWaveWords = 2048;
constexpr u64 kWaveMaxW = 1u << 16;
constexpr u64 kWaveMinW = 1u << 12;
constexpr u64 kWaveMaxCost = 1u << 15;
constexpr u64 kWaveShare = 2048;
constexpr u64 kWaveRecordCost = 8;

// One unit of counting: records [rec0, rec0 + nrec) of one start vertex,
// restricted to end vertices with sidx in [lo, hi).
struct Piece {
    uint32_t rec0, nrec;
    uint32_t lo, hi;
    uint32_t t0, t1;      // tile range [t0, t1) when kPiecePartial
    uint32_t region;      // hash region: base | log2(size) << 16
    uint32_t flags;
    uint32_t gbase;       // merge array offset (kPieceMerge)
    uint32_t start_row;   // row of the start vertex
    uint32_t list;        // kPiecePartial: heavy piece owning the bucketed short wedges
    uint32_t graph;       // graph of the start (batches; 0 for a single graph)
};

// Error word bits (device -> host); edge errors keep the first offending edge.
constexpr u64 kErrRange = 1;
constexpr u64 kErrSign = 2;
constexpr u64 kErrDup = 3;

// Layout of the small device "control" block.
struct Control {
    u64 edge_err;        // min over bad edges of (index << 4 | code), ~0 if none
    u64 balanced;
    u64 unbalanced;
    u64 wedges;
    u64 resplits;        // hashed pieces abandoned and redone in halves
    uint32_t internal_err;
    uint32_t pad0;
    uint32_t dup;        // duplicate edge seen
    uint32_t queue;      // wedge-kernel work counter
    uint32_t cls[2][kNumClassBounds];  // first row (absolute) with len > class_hi(c), per side
    uint32_t nbig_pairs; // (big row, chunk) pairs for the bitmap sort
    uint32_t queue_dense;  // work counter of the dense-piece wedge kernel
    u64 tot_heavy, tot_light_region, tot_light, tot_g;  // planner totals
    u64 active_starts;   // vertices with W_u > 0
    u64 tot_tiles;       // tile-to-piece map entries of split starts
    u64 tot_sw;          // bucketed short-middle wedges of split starts
    u64 n_dense, n_dense16, n_hashed;  // tile pieces by kind
    u64 n_dense_pieces;  // heavy pieces with dense counters (small-side chunks and dense tiles)
    uint32_t queue_hash;  // work counter of the hashed-piece wedge kernel
    uint32_t redo_n;      // halves of hashed pieces to redo (in the redo list)
    u64 n_dense8, n_dense4;  // tile pieces with packed 8- and 4-bit counters
    u64 n_wave;              // one-wave pieces (the last n_wave heavy items)
    uint32_t queue_wave;     // work counter of the one-wave kernel
    uint32_t pad1;
};

struct Dims {
    uint32_t n_u, n_v, n;
    uint32_t base[2];   // first row of each side
    uint32_t size[2];   // vertices per side
    uint32_t ntile[2];  // ceil(size[s] / kTile): tiles over side s's sidx space
    uint64_t tb_off[2]; // tile-table offset for rows of side s (entries index the other side)
    uint32_t hash_target;  // planner: expected wedges per hashed tile run
    uint32_t probe_limit;  // wedge kernel: probes before a split hashed piece is halved
    u64 chunk_min;         // planner: min wedges per record chunk of a small-side start
    // batches (n_graphs > 1): per-side sidx block starts of the graphs (n_graphs
    // + 1 entries each) and a per-graph error word (min of index << 4 | code)
    uint32_t n_graphs;
    const uint32_t* blk[2];
    u64* gerr;
    // per-vertex mode: starts are not split by record chunks, and the listed
    // short-middle wedges carry their middles
    uint32_t per_vertex;
    uint32_t light_window;  // H of the light items (kLightWindow16)
    uint32_t light_max;     // light starts: W_u <= light_max (at most kLightMax)
    uint32_t grab_div;      // grabs of total / grab_div records (unsplit pieces, light items)
    uint32_t wave_share;    // one-wave starts: at most W / wave_share wedges (0: no such bound)
    // rows in ascending (side, length) order, or NULL when the row index order
    // already is (one graph: rows are sorted by degree within each side)
    const uint32_t* rlist;
};

// the row at position p of the (side, length) order
__device__ inline uint32_t row_at(const Dims& d, uint32_t p) { return d.rlist ? d.rlist[p] : p; }

// index g of the block [blk[g], blk[g+1]) holding x (blk[0] = 0 <= x)
__host__ __device__ inline uint32_t block_of(const uint32_t* blk, uint32_t nb, uint32_t x) {
    uint32_t lo = 0, hi = nb;  // last g with blk[g] <= x
    while (hi - lo > 1) {
        const uint32_t mid = (lo + hi) >> 1;
        if (blk[mid] <= x)
            lo = mid;
        else
            hi = mid;
    }
    return lo;
}

// ---- small device helpers ---------------------------------------------------
__device__ inline uint32_t lane_id() { return threadIdx.x & 63u; }

// block_of for x uniform over the wave (blk[0] <= x): 64 bounds per round
// (lane l reads the l-th of 64 evenly spaced candidates and a ballot keeps the
// last one at or below x), so 20,000 blocks take three dependent rounds
// instead of fifteen.
__device__ inline uint32_t wave_block_of(const uint32_t* blk, uint32_t nb, uint32_t x) {
    const uint32_t lane = lane_id();
    uint32_t lo = 0, n = nb;  // the answer lies in [lo, lo + n)
    while (n > 1) {
        const uint32_t step = (n + 63) / 64;
        const uint32_t c = lo + lane * step;
        const u64 le = __ballot(c < lo + n && blk[c] <= x);
        const uint32_t l = le ? 63u - (uint32_t)__clzll(le) : 0u;  // (lane 0 qualifies)
        const uint32_t end = lo + n;
        lo += l * step;
        n = min(step, end - lo);
    }
    return lo;
}

__device__ inline uint32_t lower_bound_u32(const uint32_t* a, uint32_t n, uint32_t key) {
    uint32_t lo = 0, hi = n;
    while (lo < hi) {
        uint32_t mid = (lo + hi) >> 1;
        if (a[mid] < key)
            lo = mid + 1;
        else
            hi = mid;
    }
    return lo;
}

template <typename T>
__device__ inline T wave_reduce_sum(T v) {
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

__device__ inline uint32_t wave_reduce_min(uint32_t v) {
    for (int off = 32; off > 0; off >>= 1) v = min(v, (uint32_t)__shfl_xor(v, off, 64));
    return v;
}

__device__ inline uint32_t wave_reduce_max(uint32_t v) {
    for (int off = 32; off > 0; off >>= 1) v = max(v, (uint32_t)__shfl_xor(v, off, 64));
    return v;
}

// inclusive scan across the 64 lanes of a wave
template <typename T>
__device__ inline T wave_incl_scan(T v) {
    const uint32_t lane = lane_id();
    for (int off = 1; off < 64; off <<= 1) {
        T o = __shfl_up(v, off, 64);
        if (lane >= (uint32_t)off) v += o;
    }
    return v;
}

__device__ inline u64 choose2(u64 k) { return k < 2 ? 0 : k * (k - 1) / 2; }

// Workgroup-local aggregation of global atomics on hot keys (hub vertices):
// the slot of `key` in an open-addressing LDS table of SLOTS keys, or -1 when
// no slot is found within a few probes (the caller then goes to global memory
// directly).  Keys are never removed, so a key that found no slot never finds
// one later in the same round.
template <uint32_t LOG2_SLOTS>
__device__ inline int agg_slot(uint32_t* keys, uint32_t key) {
    constexpr uint32_t kMask = (1u << LOG2_SLOTS) - 1u;
    const uint32_t h = (key * 0x9E3779B1u) >> (32 - LOG2_SLOTS);
    for (uint32_t i = 0; i < 8; ++i) {
        const uint32_t s = (h + i) & kMask;
        uint32_t k = keys[s];
        if (k == kEmpty) {
            k = atomicCAS(&keys[s], kEmpty, key);
            if (k == kEmpty) return (int)s;
        }
        if (k == key) return (int)s;
    }
    return -1;
}

// Edge ingestion of a batch into its union graph (batch.hip).
struct IngestArgs {
    const int32_t* src_u;   // caller's concatenated edges (local ids)
    const int32_t* src_v;
    const int8_t* src_s;
    const u64* src_off;     // per included graph: index of its first edge in src_*
    const uint32_t* dst_off;  // per included graph: first union edge (n_graphs + 1 entries)
    const uint32_t* gnu;    // per included graph: |U|, |V|
    const uint32_t* gnv;
    const uint32_t* uoff;   // per included graph: first union U id / V id (sidx block starts)
    const uint32_t* voff;
    uint32_t n_graphs;
    uint64_t m;             // union edges
    int32_t* eu;            // out: union edges
    int32_t* ev;
    int8_t* sg;
    u64* gerr;              // out: per graph min(local edge index << 4 | code)
    Control* ctl;           // edge_err gets any code (the batch then needs a redo)
};

}  // namespace bbc

// ---- context arenas, for the counting service (defined in api.hip) ----------
struct bbc_context;
namespace bbc {
size_t context_resident_bytes(const bbc_context* c);  // device bytes its arenas hold now
size_t context_last_need(const bbc_context* c);  // total arena bytes a refused growth wanted
void context_set_budget(bbc_context* c, size_t bytes);  // cap its arenas (0: no cap)
bool context_trim(bbc_context* c);  // free its arenas (after its stream is idle)
}  // namespace bbc

// ---- host-side launchers (defined in the .hip files) ------------------------
namespace bbc {
hipError_t scan_excl_u32(const uint32_t* in, uint32_t* out, uint32_t n, void* tmp, size_t tmp_bytes,
                         hipStream_t st);
hipError_t scan_excl_u64(const u64* in, u64* out, uint32_t n, void* tmp, size_t tmp_bytes,
                         hipStream_t st);
size_t scan_tmp_bytes(uint32_t n);
hipError_t fill_u32(uint32_t* p, uint32_t v, size_t n, hipStream_t st);
// k <= kMaxScanSet scans of length n in one pair of launches (else one by one)
constexpr uint32_t kMaxScanSet = 4;
hipError_t scan_excl_u32_set(const uint32_t* const* ins, uint32_t* const* outs, uint32_t k,
                             uint32_t n, void* tmp, size_t tmp_bytes, hipStream_t st);
hipError_t scan_excl_u64_set(const u64* const* ins, u64* const* outs, uint32_t k, uint32_t n,
                             void* tmp, size_t tmp_bytes, hipStream_t st);
hipError_t fill_u64(u64* p, u64 v, size_t n, hipStream_t st);
hipError_t copy_u32(const uint32_t* src, uint32_t* dst, size_t n, hipStream_t st);
}  // namespace bbc
