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
//   * light   (W_u <= light_max <= kLightMax): one hashed piece; many light starts share
//             one work item, each in its own region of the on-chip table;
//   * small S (S - lo <= kDenseW, lo = the start's graph block start, 0 for
//             a single graph): dense counters over [lo, S); split into record
//             chunks of at least kRecordChunkWedges and W_total / kChunkDiv
//             wedges, merged exactly through G;
//   * else:   the end-vertex space is cut into tiles of kTile.  The wedges of u
//             are estimated per tile in proportion to the tile's degree mass
//             (an end vertex is reached through its edges).  A tile expected to
//             hold more than the hash target (a tunable, default 4096) wedges
//             becomes one dense piece (its counters always fit); runs of
//             lighter tiles are packed greedily into hashed pieces of at most
//             that many expected wedges.  A hashed piece that overflows anyway
//             is redone by the wedge kernel in halves.  The decisions use exact
//             integer arithmetic so that the counting and the writing pass
//             plan identically.
//
// A start cut into tile pieces ("split start") visits its records once per
// piece.  Records through a long middle row find their sub-interval of a tile
// in O(1) from the row's tile table; the wedges through short middle rows are
// instead bucketed once, per piece, into a packed list (w << 1 | asymmetric)
// that the piece reads contiguously.
#include "bbc_internal.h"

namespace bbc {

__device__ inline uint32_t next_pow2(uint32_t x) {
    uint32_t p = 1;
    while (p < x) p <<= 1;
    return p;
}

__device__ inline uint32_t log2_pow2(uint32_t x) { return 31u - __clz(x); }

// Sort key of a heavy piece (ascending, 8 bits: one radix pass): by the
// kernel that runs it (workgroup pieces with dense counters, then hashed
// ones, then one-wave pieces), each group most expensive first by a 6-bit
// log-scale of the estimated cost (half doublings), 4 units per record
// visited plus the expected wedges.
enum : uint32_t { kGroupDense = 0, kGroupHashed = 1, kGroupWave = 2 };
__device__ inline uint32_t cost_key(double wedges, uint32_t nrec, uint32_t group) {
    const double c = wedges + 4.0 * nrec;
    const double q = log2(1.0 + c) * 2.0;
    return (group << 6) | (63u - (uint32_t)fmin(q, 63.0));
}

// Kinds of the pieces of a split start
enum : uint32_t { kRunHash = 0, kRunD32, kRunD16, kRunD8, kRunD4 };

// The planner's tile loops read two values at end-vertex tile boundaries h
// (h = S, or a multiple of kTile below S) of one side: the degree mass below
// h, row_ptr[base + h], and the degree of the vertex at sidx h - 1.  Both are
// the same for every start of the side except at h = S, so a workgroup keeps
// them per tile boundary in LDS (sides of at most kPlanTiles tiles); each
// step of a loop then waits for LDS rather than for a global load.
constexpr uint32_t kPlanTiles = 1024;
struct TileBounds {
    const uint32_t* mass[2];  // per side: row_ptr at sidx t * kTile, or nullptr
    const uint32_t* deg[2];   // per side: degree of sidx t * kTile - 1 (t >= 1)
};

// Fill the workgroup's table (single graphs only; a batch never splits a
// start into tiles) and wait for it.
__device__ inline TileBounds load_tile_bounds(const uint32_t* __restrict__ row_ptr, const Dims& d,
                                              uint32_t (*s_mass)[kPlanTiles],
                                              uint32_t (*s_deg)[kPlanTiles]) {
    TileBounds tb = {{nullptr, nullptr}, {nullptr, nullptr}};
    for (uint32_t side = 0; side < 2 && d.n_graphs == 1; ++side) {
        const uint32_t n_side = side ? d.n - d.n_u : d.n_u;
        const uint32_t nt = n_side / kTile + 1;  // boundaries 0, kTile, ... <= n_side
        if (nt > kPlanTiles) continue;
        for (uint32_t t = threadIdx.x; t < nt; t += blockDim.x) {
            const uint32_t h = d.base[side] + t * kTile;
            s_mass[side][t] = row_ptr[h];
            s_deg[side][t] = t > 0 ? row_ptr[h] - row_ptr[h - 1] : 0u;
        }
        tb.mass[side] = s_mass[side];
        tb.deg[side] = s_deg[side];
    }
    __syncthreads();
    return tb;
}

// The boundary values of one start's end-vertex space [0, S)
struct TileView {
    const uint32_t* row_ptr;
    const uint32_t* lmass;  // LDS table of the side, or nullptr
    const uint32_t* ldeg;
    uint32_t base, S, mass_S, deg_S;
    __device__ TileView(const uint32_t* __restrict__ rp, const TileBounds& tb, uint32_t side,
                        uint32_t b, uint32_t s)
        : row_ptr(rp), lmass(tb.mass[side]), ldeg(tb.deg[side]), base(b), S(s) {
        mass_S = rp[b + s];
        deg_S = s > 0 ? mass_S - rp[b + s - 1] : 0u;
    }
    __device__ uint32_t mass(uint32_t h) const {
        return h == S ? mass_S : lmass ? lmass[h / kTile] : row_ptr[base + h];
    }
    __device__ uint32_t deg_last(uint32_t h) const {
        return h == S ? deg_S : ldeg ? ldeg[h / kTile] : row_ptr[base + h] - row_ptr[base + h - 1];
    }
};

// First tile of a start's end-vertex space [0, S) holding an end vertex of
// degree at least 2: an end w of degree 1 has l + m <= 1, so it lies in no
// butterfly, and the tiles below (rows are sorted by degree) get no piece.
__device__ inline uint32_t first_live_tile(const TileView& tv) {
    const uint32_t S = tv.S, T = (S + kTile - 1) / kTile;
    uint32_t t = 0;
    while (t < T && tv.deg_last(min(S, (t + 1) * kTile)) <= 1) ++t;
    return t;
}

// Tile runs of a start with end-vertex space [0, S) on the side whose rows start
// at `base`; calls emit(t0, t1, kind, expected wedges) per run and returns the
// number of runs.  A range of degree mass x is expected to hold W * x / tot
// wedges; "more than target" is tested exactly as x * W > target * tot.
//
// From tile t the widest dense counters that fit are chosen: a bucket's counts
// satisfy l + m <= min(k, deg(w)) (k = the start's middles), and rows are
// sorted by degree, so the last end vertex of a range bounds them all.  With
// `pack`, counters of 4 bits (eight tiles per piece) or 8 bits (four tiles)
// per half are tried first; then 16 bits (two tiles), else 32 (one tile).
// When the range is expected to hold more than the target it becomes one
// dense piece; otherwise tile t joins the open hashed run, which holds up to
// the target (twice that with 16-bit table halves, k < 2^16).  Runs start at
// the first live tile.
template <typename F>
__device__ uint32_t plan_runs(const TileView& tv, uint32_t t_live, u64 W, uint32_t k,
                              uint32_t target, bool pack, F emit) {
    using u128 = unsigned __int128;
    const uint32_t S = tv.S, T = (S + kTile - 1) / kTile;
    const u64 tot = tv.mass(S) - tv.mass(0);
    const u128 lim = (u128)target * tot;
    const u128 lim_run = k < (1u << 16) ? 2 * lim : lim;
    auto est = [&](u64 x) { return tot > 0 ? (double)x * (double)W / (double)tot : 0.0; };
    // the largest possible count of a bucket whose end vertex is below sidx hi
    auto bound = [&](uint32_t hi) { return min(k, tv.deg_last(hi)); };
    uint32_t n = 0, rs = kNoTile;
    u64 rx = 0;  // degree mass of the open run
    for (uint32_t t = t_live; t < T;) {
        uint32_t span = 1, kind = kRunD32;
        if (pack && bound(min(S, (t + 8) * kTile)) <= 15u) {
            span = 8;
            kind = kRunD4;
        } else if (pack && bound(min(S, (t + 4) * kTile)) <= 255u) {
            span = 4;
            kind = kRunD8;
        } else if (bound(min(S, (t + 2) * kTile)) <= 65535u) {
            span = 2;
            kind = kRunD16;
        }
        const uint32_t t1 = min(T, t + span);
        const uint32_t lo = t * kTile;
        const u64 xs = tv.mass(min(S, t1 * kTile)) - tv.mass(lo);
        if ((u128)xs * W > lim) {
            if (rs != kNoTile) {
                emit(rs, t, kRunHash, est(rx));
                ++n;
                rs = kNoTile;
            }
            emit(t, t1, kind, est(xs));
            ++n;
            t = t1;
            continue;
        }
        const u64 x = tv.mass(min(S, lo + kTile)) - tv.mass(lo);
        if (rs != kNoTile && (u128)(rx + x) * W > lim_run) {
            emit(rs, t, kRunHash, est(rx));
            ++n;
            rs = t;
            rx = x;
        } else {
            if (rs == kNoTile) {
                rs = t;
                rx = 0;
            }
            rx += x;
        }
        ++t;
    }
    if (rs != kNoTile) {
        emit(rs, T, kRunHash, est(rx));
        ++n;
    }
    return n;
}

enum : uint32_t { kClassNone = 0, kClassLight, kClassSmallSide, kClassTiles, kClassWave };

struct StartPlan {
    uint32_t cls, pieces, region, tiles;  // tiles > 0: a split start with T tiles
    uint32_t graph, lo;                   // the start's graph and its sidx block start
    uint32_t wlog;                        // one-wave pieces: log2 of ends per counter word
};

// The layout of a one-wave piece over end vertices [lo & ~3, S): the widest
// packing the range's last end vertex allows (l + m <= min(k, deg(w))), if the
// range then fits one wave's counter slice; else kEmpty.
__device__ inline uint32_t wave_layout(const uint32_t* __restrict__ row_ptr, uint32_t base,
                                       uint32_t lo, uint32_t S, uint32_t k) {
    // an empty end range has no last vertex (W > 0 there only with invalid
    // input: a duplicate pair puts u into its own prefix)
    if (S <= lo) return kEmpty;
    const uint32_t dg = row_ptr[base + S] - row_ptr[base + S - 1];
    const uint32_t bound = min(k, dg);
    const uint32_t wl = bound <= 15u ? 2u : bound <= 255u ? 1u : bound <= 65535u ? 0u : kEmpty;
    if (wl == kEmpty || S - (lo & ~3u) > (kWaveWords << wl)) return kEmpty;
    return wl;
}

// wedges per record chunk of a small-side start
__device__ inline u64 chunk_wedges(const Dims& d, const Control* ctl) {
    const u64 c = ctl->wedges / kChunkDiv;
    return c > d.chunk_min ? c : d.chunk_min;
}

// a one-wave start's share of the count: its cost W_u + kWaveRecordCost k_u
// (a wave reads its records 64 at a time, each round a chain of loads) is at
// most W / wave_share, at least kWaveMinW and at most kWaveMaxCost, above
// which a workgroup counts the start faster (no bound for wave_share 0)
__device__ inline u64 wave_max_cost(const Dims& d, const Control* ctl) {
    if (d.wave_share == 0) return ~0ull;
    const u64 c = ctl->wedges / d.wave_share;
    return c < kWaveMinW ? kWaveMinW : c > kWaveMaxCost ? kWaveMaxCost : c;
}

// The plan of start r.  With TILES, a split start's tile runs are planned
// here (and tallied by kind in nk); without, a split start only gets its class
// (the writing pass takes its piece and tile counts from the counting pass).
template <bool TILES>
__device__ inline StartPlan plan_start(const uint32_t* __restrict__ row_ptr, const TileBounds& tb,
                                       const Dims& d, uint32_t r, u64 W, uint32_t k, u64 chunk,
                                       u64 wave_max, u64* nk = nullptr) {
    StartPlan sp = {kClassNone, 0, 0, 0, 0, 0, 0};
    const uint32_t side = r >= d.n_u ? 1u : 0u;
    const uint32_t S = r - d.base[side];
    if (d.n_graphs > 1) {
        sp.graph = block_of(d.blk[side], d.n_graphs, S);
        sp.lo = d.blk[side][sp.graph];
    }
    if (W == 0) return sp;
    // a small start whose end range fits one wave's packed counters: one wave
    // counts it alone (no workgroup barriers, no hashing)
    if (!d.per_vertex && W <= kWaveMaxW && W + kWaveRecordCost * k <= wave_max) {
        const uint32_t wl = wave_layout(row_ptr, d.base[side], sp.lo, S, k);
        if (wl != kEmpty) {
            sp.cls = kClassWave;
            sp.pieces = 1;
            sp.wlog = wl;
            return sp;
        }
    }
    if (W <= d.light_max) {
        sp.cls = kClassLight;
        sp.region = max(kMinRegion, next_pow2((uint32_t)(2 * W)));
        return sp;
    }
    if (S - sp.lo <= kDenseW) {
        u64 np = d.per_vertex ? 1 : (W + chunk - 1) / chunk;
        if (np > k) np = k;
        sp.cls = kClassSmallSide;
        sp.pieces = (uint32_t)np;
        return sp;
    }
    // (tile pieces index end vertices from sidx 0: a batch never gets here, as
    // its graphs have at most kDenseW vertices per side)
    const uint32_t T = (S + kTile - 1) / kTile;
    bool whole = false;
    sp.cls = kClassTiles;
    if (!TILES) return sp;
    const TileView tv(row_ptr, tb, side, d.base[side], S);
    const uint32_t t_live = first_live_tile(tv);
    sp.pieces = plan_runs(tv, t_live, W, k, d.hash_target, !d.per_vertex,
                          [&](uint32_t t0, uint32_t t1, uint32_t kind, double) {
                              whole = whole || (t0 == t_live && t1 == T && kind == kRunHash);
                              if (nk) ++nk[kind];
                          });
    // One hashed run over everything is left unsplit only when its W wedges
    // cannot fill the table (at most W distinct ends); otherwise it keeps its
    // tiles so that an overflowing run can be halved.
    whole = whole && W <= kHashSlots / 2;
    sp.tiles = whole ? 0u : T;
    return sp;
}

__global__ void k_plan_count(const u64* __restrict__ wu, const u64* __restrict__ wsu,
                             const uint32_t* __restrict__ lowcnt,
                             const uint32_t* __restrict__ row_ptr, Dims d,
                             uint32_t* __restrict__ hp, u64* __restrict__ lr,
                             uint32_t* __restrict__ lf, uint32_t* __restrict__ gs,
                             uint32_t* __restrict__ tc, u64* __restrict__ swc, Control* ctl) {
    __shared__ uint32_t s_mass[2][kPlanTiles], s_deg[2][kPlanTiles];
    const TileBounds tb = load_tile_bounds(row_ptr, d, s_mass, s_deg);
    const u64 chunk = chunk_wedges(d, ctl), wave_max = wave_max_cost(d, ctl);
    u64 n_wave = 0;
    for (uint32_t r = blockIdx.x * blockDim.x + threadIdx.x; r < d.n; r += gridDim.x * blockDim.x) {
        const u64 W = wu[r];
        u64 nk[5] = {0, 0, 0, 0, 0};  // tile pieces by kind
        const StartPlan sp = plan_start<true>(row_ptr, tb, d, r, W, lowcnt[r], chunk, wave_max, nk);
        n_wave += sp.cls == kClassWave ? 1u : 0u;
        const uint32_t side = r >= d.n_u ? 1u : 0u;
        if (sp.cls == kClassTiles && d.n_graphs > 1) atomicOr(&ctl->internal_err, 2u);
        if (sp.cls == kClassTiles) {
            if (nk[kRunD32]) atomicAdd(&ctl->n_dense, nk[kRunD32]);
            if (nk[kRunD16]) atomicAdd(&ctl->n_dense16, nk[kRunD16]);
            if (nk[kRunD8]) atomicAdd(&ctl->n_dense8, nk[kRunD8]);
            if (nk[kRunD4]) atomicAdd(&ctl->n_dense4, nk[kRunD4]);
            if (nk[kRunHash]) atomicAdd(&ctl->n_hashed, nk[kRunHash]);
            const u64 ndense = nk[kRunD32] + nk[kRunD16] + nk[kRunD8] + nk[kRunD4];
            if (ndense) atomicAdd(&ctl->n_dense_pieces, ndense);
        } else if (sp.cls == kClassSmallSide) {
            atomicAdd(&ctl->n_dense_pieces, (u64)sp.pieces);
        }
        hp[r] = sp.pieces;
        lr[r] = sp.cls == kClassLight ? sp.region : 0u;
        lf[r] = sp.cls == kClassLight ? 1u : 0u;
        gs[r] = (sp.cls == kClassSmallSide && sp.pieces > 1) ? r - d.base[side] - sp.lo : 0u;
        tc[r] = sp.tiles;
        swc[r] = sp.tiles ? wsu[r] : 0ull;
    }
    n_wave = wave_reduce_sum(n_wave);
    if (lane_id() == 0 && n_wave) atomicAdd(&ctl->n_wave, n_wave);
}

__global__ void k_plan_write(const u64* __restrict__ wu, const uint32_t* __restrict__ lowcnt,
                             const uint32_t* __restrict__ row_ptr,
                             const uint32_t* __restrict__ mptr, const uint32_t* __restrict__ front,
                             const uint32_t* __restrict__ hp_off, const u64* __restrict__ lr_off,
                             const uint32_t* __restrict__ lf_off,
                             const uint32_t* __restrict__ gs_off,
                             const uint32_t* __restrict__ tc_off, Dims d, uint32_t n_heavy,
                             Piece* __restrict__ pieces, u64* __restrict__ light_off,
                             uint32_t* __restrict__ hkey, uint32_t* __restrict__ tile_piece,
                             const Control* ctl) {
    __shared__ uint32_t s_mass[2][kPlanTiles], s_deg[2][kPlanTiles];
    const TileBounds tb = load_tile_bounds(row_ptr, d, s_mass, s_deg);
    const u64 chunk = chunk_wedges(d, ctl), wave_max = wave_max_cost(d, ctl);
    for (uint32_t r = blockIdx.x * blockDim.x + threadIdx.x; r < d.n; r += gridDim.x * blockDim.x) {
        const u64 W = wu[r];
        if (W == 0) continue;
        const uint32_t k = lowcnt[r], m0 = mptr[r];
        StartPlan sp = plan_start<false>(row_ptr, tb, d, r, W, k, chunk, wave_max);
        if (sp.cls == kClassTiles) {  // as planned by the counting pass
            sp.pieces = hp_off[r + 1] - hp_off[r];
            sp.tiles = tc_off[r + 1] - tc_off[r];
        }
        const uint32_t side = r >= d.n_u ? 1u : 0u;
        const uint32_t S = r - d.base[side];
        const uint32_t sideflag = side ? kPieceSideV : 0u;
        if (sp.cls == kClassLight) {
            const uint32_t idx = lf_off[r];
            const u64 off = lr_off[r];
            const u64 item = off / d.light_window;
            Piece p;
            p.rec0 = m0;
            p.nrec = k;
            p.lo = sp.lo;
            p.hi = S;
            p.t0 = kNoTile;
            p.t1 = kNoTile;
            p.region = (uint32_t)(off - item * d.light_window) | (log2_pow2(sp.region) << 16);
            // the 16-bit-half table (a light start has at most kLightMax < 2^16 wedges)
            p.flags = sideflag | kPieceHash16;
            p.gbase = kEmpty;
            p.start_row = r;
            p.list = kEmpty;
            p.graph = sp.graph;
            pieces[n_heavy + idx] = p;
            light_off[idx] = off;
            continue;
        }
        const uint32_t h = sp.pieces;
        const uint32_t b = hp_off[r];
        if (sp.cls == kClassWave) {
            Piece p;
            p.rec0 = m0;
            p.nrec = k;
            p.lo = sp.lo & ~3u;  // (so that w's low bits give its slot in a packed word)
            p.hi = S;
            p.t0 = kNoTile;
            p.t1 = kNoTile;
            p.region = 0;
            p.flags = kPieceDense | kPieceWave | sideflag |
                      (sp.wlog == 2 ? kPieceDense4 : sp.wlog == 1 ? kPieceDense8 : kPieceDense16);
            p.gbase = kEmpty;
            p.start_row = r;
            p.list = kEmpty;
            p.graph = sp.graph;
            pieces[b] = p;
            hkey[b] = cost_key((double)W, k, kGroupWave);
            continue;
        }
        if (sp.cls == kClassSmallSide) {
            for (uint32_t i = 0; i < h; ++i) {
                const uint32_t c0 = (uint32_t)((u64)k * i / h), c1 = (uint32_t)((u64)k * (i + 1) / h);
                Piece p;
                p.rec0 = m0 + c0;
                p.nrec = c1 - c0;
                p.lo = sp.lo;
                p.hi = S;
                p.t0 = kNoTile;
                p.t1 = kNoTile;
                p.region = 0;
                p.flags = kPieceDense | (h > 1 ? kPieceMerge : 0u) | sideflag;
                p.gbase = gs_off[r];
                p.start_row = r;
                p.list = kEmpty;
                p.graph = sp.graph;
                pieces[b + i] = p;
                hkey[b + i] = cost_key((double)W * (c1 - c0) / k, c1 - c0, kGroupDense);
            }
            continue;
        }
        // tile runs; a split start keeps only its long-middle records, the
        // short-middle wedges come from the bucketed list of each piece (with
        // their middles in per-vertex mode)
        const uint32_t T = (S + kTile - 1) / kTile;
        const bool split = sp.tiles > 0;
        const bool bucketed = split;
        const uint32_t nlong = front[r] - m0;
        const TileView tv(row_ptr, tb, side, d.base[side], S);
        const uint32_t t_live = first_live_tile(tv);
        if (split)  // tiles of ends of degree <= 1: no piece
            for (uint32_t t = 0; t < t_live; ++t) tile_piece[tc_off[r] + t] = kEmpty;
        uint32_t i = 0;
        plan_runs(tv, t_live, W, k, d.hash_target, !d.per_vertex,
                  [&](uint32_t t0, uint32_t t1, uint32_t kind, double est) {
            if (i >= h) return;
            const bool dense = kind != kRunHash;
            Piece p;
            p.rec0 = m0;
            p.nrec = bucketed ? nlong : k;
            p.lo = split ? t0 * kTile : 0u;  // an unsplit run takes every end
            p.hi = min(S, t1 * kTile);
            p.t0 = t0;
            p.t1 = t1;
            p.region = log2_pow2(kHashSlots) << 16;
            const bool pair = k < (1u << 16);
            p.flags = (split ? kPiecePartial : 0u) | (dense ? kPieceDense : 0u) |
                      (kind == kRunD16 ? kPieceDense16 : 0u) | (kind == kRunD8 ? kPieceDense8 : 0u) |
                      (kind == kRunD4 ? kPieceDense4 : 0u) |
                      ((!dense && split && pair) ? kPieceHash16 : 0u) | sideflag;
            p.gbase = kEmpty;
            p.start_row = r;
            p.list = bucketed ? b + i : kEmpty;
            p.graph = 0;
            pieces[b + i] = p;
            hkey[b + i] = cost_key(est, p.nrec, dense ? kGroupDense : kGroupHashed);
            if (split)
                for (uint32_t t = t0; t < t1; ++t) tile_piece[tc_off[r] + t] = i;
            ++i;
        });
    }
}

// -- bucketing of the short-middle wedges of split starts, two passes over
// their short records: count per piece, then place.  A workgroup takes 256
// records, 64 per wave; a wave reads the concatenation of the prefixes of its
// short records of split starts 64 entries at a time (coalesced), finding each
// entry's owner from head flags that mark where each prefix begins; four such
// windows are loaded together, so the two dependent reads of an entry (the
// entry, then its tile's piece) are waited for once per four windows.  A prefix
// is sorted by end vertex, so its tiles, and the pieces they belong to, do not
// decrease: a window splits into runs of one piece.  Runs are counted in an LDS
// table keyed by piece and reach global memory once per (workgroup, piece).
// The fill pass reserves each piece's slots then and walks the prefixes again,
// each run taking consecutive slots.  A piece that finds no table slot goes to
// global memory directly, run by run.  In per-vertex mode `mids` receives, for
// every list entry, the row of the wedge's middle vertex.
constexpr int kSwThreads = 256;
constexpr uint32_t kSwWaves = kSwThreads / 64;
// 512 table slots: a chunk of 256 records meets a few hundred pieces at most,
// and the small table (14.6 KiB of LDS per workgroup) keeps 7-8 waves per SIMD
constexpr uint32_t kSwLog2 = 9;
constexpr uint32_t kSwSlots = 1u << kSwLog2;
constexpr uint32_t kSwUnroll = 4;  // windows of 64 entries loaded together
// per-piece counts a chunk keeps between the passes (a chunk holds at most
// 256 records of at most kLongDeg entries each, so a count fits 16 bits)
constexpr uint32_t kSwKept = 64;
static_assert(kSwThreads * kLongDeg < (1u << 16), "chunk counts fit 16 bits");

size_t short_wedge_chunk_slots(uint64_t m) { return (size_t)((m + kSwThreads - 1) / kSwThreads) * kSwKept; }

// Slot of `key` in the chunk's LDS table (inserting it), or -1 after 8 probes;
// a newly taken slot is appended to `used`, so that the flush and the reset
// touch only the slots in use.
__device__ inline int sw_slot(uint32_t* keys, uint32_t key, uint32_t* used, uint32_t* n_used) {
    constexpr uint32_t kMask = kSwSlots - 1u;
    const uint32_t h = (key * 0x9E3779B1u) >> (32 - kSwLog2);
    for (uint32_t i = 0; i < 8; ++i) {
        const uint32_t s = (h + i) & kMask;
        uint32_t k = keys[s];
        if (k == kEmpty) {
            k = atomicCAS(&keys[s], kEmpty, key);
            if (k == kEmpty) {
                used[atomicAdd(n_used, 1u)] = s;
                return (int)s;
            }
        }
        if (k == key) return (int)s;
    }
    return -1;
}

template <bool kFill>
__global__ __launch_bounds__(kSwThreads) void k_short_wedges(
    const uint4* __restrict__ recs, uint32_t m, const uint32_t* __restrict__ col,
    const uint32_t* __restrict__ front, const uint32_t* __restrict__ tc,
    const uint32_t* __restrict__ tc_off, const uint32_t* __restrict__ hp_off,
    const uint32_t* __restrict__ tile_piece, uint32_t n_u, uint32_t* __restrict__ counts,
    uint32_t* __restrict__ cursor, uint32_t* __restrict__ list, uint32_t* __restrict__ mids,
    uint16_t* __restrict__ chunk_cnt) {
    __shared__ uint32_t keys[kSwSlots];
    __shared__ uint32_t cnt[kSwSlots];
    __shared__ uint32_t base[kSwSlots];
    __shared__ uint32_t s_adj[kSwWaves][64];  // per non-empty prefix: address - its first position
    __shared__ uint32_t s_tb[kSwWaves][64];   // its start's tile-to-piece table
    __shared__ uint32_t s_pb[kSwWaves][64];   // its start's first heavy piece
    __shared__ uint32_t s_s1[kSwWaves][64];   // sign(u, v) of its record
    __shared__ uint32_t s_mid[kSwWaves][64];  // the row of its middle v (per-vertex mode)
    __shared__ uint8_t s_head[kSwWaves][64 * kSwUnroll];
    __shared__ uint32_t s_used[kSwSlots];  // table slots taken in this chunk
    __shared__ uint32_t s_nused;
    // a chunk whose short records all belong to one start with at most
    // kSwSlots tiles maps tiles to that start's pieces from LDS, and counts
    // per piece directly (index = piece - the start's first piece)
    __shared__ uint32_t s_tp[kSwSlots];
    __shared__ uint32_t s_umin[kSwWaves], s_umax[kSwWaves];
    const uint32_t tid = threadIdx.x, lane = lane_id(), wave = tid >> 6;
    const u64 le_mask = ~0ull >> (63 - lane);  // lanes 0..lane
    for (uint32_t u = 0; u < kSwUnroll; ++u) s_head[wave][u * 64 + lane] = 0;
    for (uint32_t i = tid; i < kSwSlots; i += kSwThreads) {
        keys[i] = kEmpty;
        cnt[i] = 0;
    }
    if (tid == 0) s_nused = 0;
    __syncthreads();
    for (uint32_t c0 = blockIdx.x * kSwThreads; c0 < m; c0 += gridDim.x * kSwThreads) {
        const uint32_t j = c0 + tid;
        uint4 rc = make_uint4(0, 0, 0, 0);
        bool mine = false;
        if (j < m) {
            rc = recs[j];
            const uint32_t u = rc.w;
            mine = tc[u] > 0 && j >= front[u];  // short record of a split start
        }
        const uint32_t len = mine ? rc.y >> 1 : 0u;
        // chunks without a short record of a split start are skipped whole (the
        // table is clean: every chunk resets the slots it used)
        if (!__syncthreads_or(len > 0)) continue;
        const u64 nz = __ballot(len > 0);
        const uint32_t excl = wave_incl_scan(len) - len;
        const uint32_t T = __shfl(excl + len, 63, 64);
        if (len > 0) {
            const uint32_t ci = (uint32_t)__popcll(nz & (le_mask >> 1));
            s_adj[wave][ci] = rc.x - excl;
            s_tb[wave][ci] = tc_off[rc.w];
            s_pb[wave][ci] = hp_off[rc.w];
            s_s1[wave][ci] = rc.y & 1u;
            s_mid[wave][ci] = (rc.w < n_u ? n_u : 0u) + rc.z;  // v lies on the other side
        }
        {
            const uint32_t umin = wave_reduce_min(len > 0 ? rc.w : kEmpty);
            const uint32_t umax = wave_reduce_max(len > 0 ? rc.w : 0u);
            if (lane == 0) {
                s_umin[wave] = umin;
                s_umax[wave] = umax;
            }
        }
        __syncthreads();
        uint32_t u0 = kEmpty, u1 = 0;
        for (uint32_t w = 0; w < kSwWaves; ++w) {
            u0 = min(u0, s_umin[w]);
            u1 = max(u1, s_umax[w]);
        }
        const bool fast = u0 == u1 && tc[u0] <= kSwSlots;  // uniform over the workgroup
        uint32_t pb0 = 0, h0 = 0;
        if (fast) {
            pb0 = hp_off[u0];
            h0 = hp_off[u0 + 1] - pb0;
            const uint32_t tb0 = tc_off[u0], nt = tc[u0];
            for (uint32_t t = tid; t < nt; t += kSwThreads) s_tp[t] = tile_piece[tb0 + t];
            __syncthreads();
        }
        // place = false: count runs per piece; place = true (fill pass): each
        // run takes consecutive slots from its piece's reserved range
        auto walk = [&](const bool place) {
            uint32_t before = 0;
            for (uint32_t w0 = 0; w0 < T; w0 += 64 * kSwUnroll) {
                if (len > 0 && excl >= w0 && excl < w0 + 64 * kSwUnroll) s_head[wave][excl - w0] = 1;
                __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
                uint32_t idx[kSwUnroll], x[kSwUnroll], gp[kSwUnroll];
#pragma unroll
                for (uint32_t u = 0; u < kSwUnroll; ++u) {
                    const u64 M = __ballot(s_head[wave][u * 64 + lane] != 0);
                    idx[u] = before + (uint32_t)__popcll(M & le_mask) - 1u;
                    before += (uint32_t)__popcll(M);
                    const uint32_t q = w0 + u * 64 + lane;
                    x[u] = q < T ? col[s_adj[wave][idx[u]] + q] : 0u;
                }
#pragma unroll
                for (uint32_t u = 0; u < kSwUnroll; ++u) {
                    const uint32_t q = w0 + u * 64 + lane;
                    if (fast) {  // gp: the piece's index among the start's pieces
                        gp[u] = q < T ? s_tp[(x[u] >> 1) / kTile] : kEmpty;
                    } else {
                        const uint32_t tp =
                            q < T ? tile_piece[s_tb[wave][idx[u]] + (x[u] >> 1) / kTile] : kEmpty;
                        gp[u] = tp != kEmpty ? s_pb[wave][idx[u]] + tp : kEmpty;
                    }
                    s_head[wave][u * 64 + lane] = 0;
                }
#pragma unroll
                for (uint32_t u = 0; u < kSwUnroll; ++u) {
                    const uint32_t wu = w0 + u * 64;
                    if (wu >= T) continue;  // uniform over the wave
                    const bool valid = wu + lane < T;
                    const uint32_t val =
                        valid ? (x[u] & ~1u) | ((x[u] ^ s_s1[wave][idx[u]]) & 1u) : 0u;
                    // runs of equal piece among the valid lanes (a prefix of the window)
                    const uint32_t prev = __shfl_up(gp[u], 1, 64);
                    const u64 H = __ballot(valid && (lane == 0 || prev != gp[u]));
                    const uint32_t nvalid = min(64u, T - wu);
                    const uint32_t head = 63u - (uint32_t)__clzll(H & le_mask);  // this lane's run
                    uint32_t rlen = 0;
                    if ((H >> lane) & 1ull) {
                        const u64 later = lane < 63 ? H >> (lane + 1) : 0ull;
                        rlen = later ? (uint32_t)__builtin_ctzll(later) + 1u : nvalid - lane;
                    }
                    uint32_t at = kEmpty;  // the run's first slot, if this pass writes it
                    if (rlen && gp[u] != kEmpty) {  // (a run of ends in no piece is dropped)
                        const int sl = fast ? (int)gp[u] : sw_slot(keys, gp[u], s_used, &s_nused);
                        if (!place) {
                            if (sl >= 0)
                                atomicAdd(&cnt[sl], rlen);
                            else if (!kFill)
                                atomicAdd(&counts[gp[u]], rlen);
                            else
                                at = atomicAdd(&cursor[gp[u]], rlen);  // no slot: placed now
                        } else if (sl >= 0) {
                            at = base[sl] + atomicAdd(&cnt[sl], rlen);
                        }
                    }
                    if (kFill) {
                        at = __shfl(at, (int)head, 64);
                        if (valid && at != kEmpty) {
                            list[at + (lane - head)] = val;
                            if (mids) mids[at + (lane - head)] = s_mid[wave][idx[u]];
                        }
                    }
                }
                __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
            }
        };
        // a single-start chunk of at most kSwKept pieces keeps its per-piece
        // counts from the count pass, so the fill pass walks its entries once
        const bool kept = fast && h0 <= kSwKept;
        uint16_t* kc = chunk_cnt + (size_t)(c0 / kSwThreads) * kSwKept;
        if (!(kFill && kept)) {
            walk(false);
            __syncthreads();
        }
        if (fast) {
            for (uint32_t i = tid; i < h0; i += kSwThreads) {
                const uint32_t c = (kFill && kept) ? kc[i] : cnt[i];
                if (!kFill && kept) kc[i] = (uint16_t)c;
                if (c == 0) continue;
                if (!kFill)
                    atomicAdd(&counts[pb0 + i], c);
                else
                    base[i] = atomicAdd(&cursor[pb0 + i], c);
                cnt[i] = 0;
            }
            __syncthreads();
            if (kFill) {
                walk(true);
                __syncthreads();
                for (uint32_t i = tid; i < h0; i += kSwThreads) cnt[i] = 0;
                __syncthreads();
            }
            continue;
        }
        const uint32_t nused = s_nused;
        for (uint32_t k = tid; k < nused; k += kSwThreads) {
            const uint32_t i = s_used[k];
            if (!kFill)
                atomicAdd(&counts[keys[i]], cnt[i]);
            else
                base[i] = atomicAdd(&cursor[keys[i]], cnt[i]);
            cnt[i] = 0;
        }
        __syncthreads();
        if (kFill) walk(true);
        __syncthreads();
        for (uint32_t k = tid; k < nused; k += kSwThreads) {
            const uint32_t i = s_used[k];
            keys[i] = kEmpty;
            cnt[i] = 0;
        }
        __syncthreads();
        if (tid == 0) s_nused = 0;  // ordered before the next chunk's inserts by its barrier
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
                                const uint32_t* __restrict__ gs_off,
                                const uint32_t* __restrict__ tc_off, const u64* __restrict__ sw_off,
                                uint32_t n, Control* ctl) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        ctl->tot_heavy = hp_off[n];
        ctl->tot_light_region = lr_off[n];
        ctl->tot_light = lf_off[n];
        ctl->tot_g = gs_off[n];
        ctl->tot_tiles = tc_off[n];
        ctl->tot_sw = sw_off[n];
    }
}

// first light piece of each light item: item i holds the pieces whose region
// offset lies in [i H, (i+1) H)
__global__ void k_items_first(const u64* __restrict__ light_off, uint32_t n_light,
                              uint32_t n_items, u64 H, uint32_t* __restrict__ first) {
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i <= n_items;
         i += gridDim.x * blockDim.x) {
        u64 key = (u64)i * H;
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

static dim3 grid_n(uint64_t n, uint32_t threads, uint32_t cap = 16384) {
    uint64_t b = (n + threads - 1) / threads;
    if (b > cap) b = cap;
    if (b == 0) b = 1;
    return dim3((unsigned)b);
}

hipError_t launch_plan_count(const u64* wu, const u64* wsu, const uint32_t* lowcnt,
                             const uint32_t* row_ptr, Dims d, uint32_t* hp, u64* lr, uint32_t* lf,
                             uint32_t* gs, uint32_t* tc, u64* swc, u64* wsum, u64* nonzero,
                             Control* ctl, hipStream_t st) {
    // W first: the record-chunk size of small-side starts depends on it
    hipLaunchKernelGGL(k_sum_u64, grid_n(d.n, 256, 512), dim3(256), 0, st, wu, d.n, wsum, nonzero);
    hipLaunchKernelGGL(k_plan_count, grid_n(d.n, 256), dim3(256), 0, st, wu, wsu, lowcnt, row_ptr, d,
                       hp, lr, lf, gs, tc, swc, ctl);
    return hipGetLastError();
}

hipError_t launch_gather_totals(const uint32_t* hp_off, const u64* lr_off, const uint32_t* lf_off,
                                const uint32_t* gs_off, const uint32_t* tc_off, const u64* sw_off,
                                uint32_t n, Control* ctl, hipStream_t st) {
    hipLaunchKernelGGL(k_gather_totals, dim3(1), dim3(64), 0, st, hp_off, lr_off, lf_off, gs_off,
                       tc_off, sw_off, n, ctl);
    return hipGetLastError();
}

hipError_t launch_plan_write(const u64* wu, const uint32_t* lowcnt, const uint32_t* row_ptr,
                             const uint32_t* mptr, const uint32_t* front, const uint32_t* hp_off,
                             const u64* lr_off, const uint32_t* lf_off, const uint32_t* gs_off,
                             const uint32_t* tc_off, Dims d, uint32_t n_heavy, Piece* pieces,
                             u64* light_off, uint32_t* hkey, uint32_t* tile_piece, uint32_t n_light,
                             uint32_t n_light_items, uint32_t* items_first, const Control* ctl,
                             hipStream_t st) {
    hipLaunchKernelGGL(k_plan_write, grid_n(d.n, 256), dim3(256), 0, st, wu, lowcnt, row_ptr, mptr,
                       front, hp_off, lr_off, lf_off, gs_off, tc_off, d, n_heavy, pieces, light_off,
                       hkey, tile_piece, ctl);
    hipLaunchKernelGGL(k_items_first, grid_n((uint64_t)n_light_items + 1, 256), dim3(256), 0, st,
                       (const u64*)light_off, n_light, n_light_items, (u64)d.light_window,
                       items_first);
    return hipGetLastError();
}

hipError_t launch_short_wedges(const uint4* recs, uint32_t m, const uint32_t* col,
                               const uint32_t* front, const uint32_t* tc, const uint32_t* tc_off,
                               const uint32_t* hp_off, const uint32_t* tile_piece, uint32_t n_u,
                               uint32_t* counts, uint32_t* cursor, uint32_t* list, uint32_t* mids,
                               uint16_t* chunk_cnt, bool fill, hipStream_t st) {
    if (fill)
        hipLaunchKernelGGL(k_short_wedges<true>, grid_n(m, kSwThreads, 8192), dim3(kSwThreads), 0, st,
                           recs, m, col, front, tc, tc_off, hp_off, tile_piece, n_u, counts, cursor,
                           list, mids, chunk_cnt);
    else
        hipLaunchKernelGGL(k_short_wedges<false>, grid_n(m, kSwThreads, 8192), dim3(kSwThreads), 0,
                           st, recs, m, col, front, tc, tc_off, hp_off, tile_piece, n_u, counts,
                           cursor, list, mids, chunk_cnt);
    return hipGetLastError();
}

}  // namespace bbc
