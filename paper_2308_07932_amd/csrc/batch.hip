// Many graphs in one pass: the batch is counted as one disjoint union.
//
// The method of Section 4 counts each butterfly once, at its vertex of highest
// priority (Theorem 1), and the butterflies of a disjoint union are exactly
// those of its parts.  So a batch is relabelled into one union graph whose
// graph g owns the U ids [uoff[g], uoff[g+1]) and the V ids [voff[g],
// voff[g+1]); the priority sort key becomes (graph, degree, id), which keeps
// every graph's vertices in one sidx block per side and orders them inside the
// block exactly as a count of that graph alone would (Definition 4).  The
// planner and the wedge kernel then only need the block start of a start
// vertex and the graph index that its totals go to.
//
// Kernels here: copying and checking the edges of the included graphs into the
// union (with the per-graph first bad edge), the sort keys, the per-graph
// duplicate check (run only when the row sort saw a duplicate), and the
// per-graph wedge totals.
#include "bbc_internal.h"

namespace bbc {


// An edge whose ids are out of range is written with u = -1, so that the
// degree and scatter passes drop it (their own range check fails) instead of
// placing it in another graph's id block (a graph with no vertex on a side
// shares its block start with the next graph); an edge with a bad sign keeps
// its in-range ids with sign +1.  Either way its graph is reported and left
// out of the redo, and the other graphs' rows never see the edge.
//
// A wave takes spans of kIngestSpan consecutive union edges; the graphs of a
// span's first and last edge bound those of the others, so an edge searches
// only that range (usually a single graph).
constexpr uint32_t kIngestPer = 8;
constexpr uint32_t kIngestSpan = 64 * kIngestPer;

__global__ __launch_bounds__(256) void k_ingest(IngestArgs a) {
    const uint32_t lane = lane_id();
    const uint64_t nw = (uint64_t)gridDim.x * (blockDim.x >> 6);
    for (uint64_t s0 = ((uint64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6)) * kIngestSpan;
         s0 < a.m; s0 += nw * kIngestSpan) {
        const uint64_t s1 = min<uint64_t>(s0 + kIngestSpan, a.m);
        const uint32_t jlo = wave_block_of(a.dst_off, a.n_graphs, (uint32_t)s0);
        const uint32_t jhi = wave_block_of(a.dst_off, a.n_graphs, (uint32_t)(s1 - 1));
        for (uint32_t k = 0; k < kIngestPer; ++k) {
            const uint64_t i = s0 + (uint64_t)k * 64 + lane;
            if (i >= s1) break;
            uint32_t j = jlo, hi = jhi + 1;  // dst_off[j] <= i < dst_off[hi]
            while (hi - j > 1) {
                const uint32_t mid = (j + hi) >> 1;
                if (a.dst_off[mid] <= (uint32_t)i)
                    j = mid;
                else
                    hi = mid;
            }
            const uint64_t e = i - a.dst_off[j];
            const uint64_t src = a.src_off[j] + e;
            int32_t u = a.src_u[src], v = a.src_v[src];
            int8_t s = a.src_s[src];
            u64 code = 0;
            bool drop = false;
            if (u < 0 || v < 0 || (uint32_t)u >= a.gnu[j] || (uint32_t)v >= a.gnv[j]) {
                code = kErrRange;
                drop = true;
            } else if (s != 1 && s != -1) {
                code = kErrSign;
                s = 1;
            }
            if (code) {
                atomicMin(&a.gerr[j], (e << 4) | code);
                atomicMin(&a.ctl->edge_err, code);
            }
            a.eu[i] = drop ? -1 : (int32_t)(a.uoff[j] + (uint32_t)u);
            a.ev[i] = drop ? 0 : (int32_t)(a.voff[j] + (uint32_t)v);
            a.sg[i] = s;
        }
    }
}

// priority sort key of union vertex x: graph << deg_bits | degree
__global__ void k_batch_keys(const uint32_t* __restrict__ deg, Dims d, uint32_t deg_bits,
                             uint32_t* __restrict__ key) {
    for (uint32_t x = blockIdx.x * blockDim.x + threadIdx.x; x < d.n; x += gridDim.x * blockDim.x) {
        const uint32_t side = x >= d.n_u ? 1u : 0u;
        const uint32_t g = block_of(d.blk[side], d.n_graphs, x - d.base[side]);
        // a graph with repeated pairs may exceed the bound; its counts are
        // discarded, so clamping only keeps its key in range
        key[x] = (g << deg_bits) | min(deg[x], (1u << deg_bits) - 1u);
    }
}

// (side, length) key of every row, for the row list of a batch
__global__ void k_row_keys(const uint32_t* __restrict__ rowdeg, Dims d, uint32_t deg_bits,
                           uint32_t* __restrict__ key) {
    for (uint32_t r = blockIdx.x * blockDim.x + threadIdx.x; r < d.n; r += gridDim.x * blockDim.x)
        key[r] = ((r >= d.n_u ? 1u : 0u) << deg_bits) | min(rowdeg[r], (1u << deg_bits) - 1u);
}

// Graphs whose sorted rows hold two entries with the same neighbour (only
// when the row sort flagged a duplicate somewhere).
__global__ void k_dup_graphs(const uint32_t* __restrict__ row_ptr, const uint32_t* __restrict__ col,
                             Dims d, const Control* ctl) {
    if (!ctl->dup) return;
    for (uint32_t r = blockIdx.x * blockDim.x + threadIdx.x; r < d.n; r += gridDim.x * blockDim.x) {
        const uint32_t a = row_ptr[r], b = row_ptr[r + 1];
        for (uint32_t i = a + 1; i < b; ++i)
            if ((col[i] >> 1) == (col[i - 1] >> 1)) {
                const uint32_t side = r >= d.n_u ? 1u : 0u;
                const uint32_t g = block_of(d.blk[side], d.n_graphs, r - d.base[side]);
                // a graph with a bad edge (written as a placeholder) keeps that error
                if (d.gerr[g] == kEmpty64) atomicMin(&d.gerr[g], kErrDup);
                break;
            }
    }
}

// W of every graph: one wave sums W_u over the graph's U rows and V rows
__global__ __launch_bounds__(256) void k_graph_wedges(const u64* __restrict__ wu, Dims d,
                                                      u64* __restrict__ gres) {
    const uint32_t lane = lane_id();
    const uint32_t wid = (blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const uint32_t wstride = (gridDim.x * blockDim.x) >> 6;
    for (uint32_t g = wid; g < d.n_graphs; g += wstride) {
        u64 s = 0;
        for (uint32_t side = 0; side < 2; ++side) {
            const uint32_t r0 = d.base[side] + d.blk[side][g], r1 = d.base[side] + d.blk[side][g + 1];
            for (uint32_t r = r0 + lane; r < r1; r += 64) s += wu[r];
        }
        s = wave_reduce_sum(s);
        if (lane == 0) gres[4ull * g + 2] = s;
    }
}

static dim3 grid_n(uint64_t n, uint32_t threads, uint32_t cap = 16384) {
    uint64_t b = (n + threads - 1) / threads;
    if (b > cap) b = cap;
    if (b == 0) b = 1;
    return dim3((unsigned)b);
}

hipError_t launch_ingest(const IngestArgs& a, hipStream_t st) {
    hipLaunchKernelGGL(k_ingest, grid_n(a.m, 256), dim3(256), 0, st, a);
    return hipGetLastError();
}

hipError_t launch_batch_keys(const uint32_t* deg, Dims d, uint32_t deg_bits, uint32_t* key,
                             hipStream_t st) {
    hipLaunchKernelGGL(k_batch_keys, grid_n(d.n, 256), dim3(256), 0, st, deg, d, deg_bits, key);
    return hipGetLastError();
}

hipError_t launch_row_keys(const uint32_t* rowdeg, Dims d, uint32_t deg_bits, uint32_t* key,
                           hipStream_t st) {
    hipLaunchKernelGGL(k_row_keys, grid_n(d.n, 256), dim3(256), 0, st, rowdeg, d, deg_bits, key);
    return hipGetLastError();
}

hipError_t launch_dup_graphs(const uint32_t* row_ptr, const uint32_t* col, Dims d,
                             const Control* ctl, hipStream_t st) {
    hipLaunchKernelGGL(k_dup_graphs, grid_n(d.n, 256), dim3(256), 0, st, row_ptr, col, d, ctl);
    return hipGetLastError();
}

hipError_t launch_graph_wedges(const u64* wu, Dims d, u64* gres, hipStream_t st) {
    hipLaunchKernelGGL(k_graph_wedges, grid_n((uint64_t)d.n_graphs * 64, 256), dim3(256), 0, st, wu,
                       d, gres);
    return hipGetLastError();
}

}  // namespace bbc
