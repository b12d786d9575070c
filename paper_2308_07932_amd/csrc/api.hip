// Host side of the C ABI declared in include/bbc.h: argument checks, the
// device workspace, and the launch sequence of the counting pipeline.
#include <stdarg.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <chrono>
#include <mutex>
#include <vector>

#include "bbc.h"
#include "bbc_internal.h"

namespace bbc {
// edges of one graph: its CSR holds 2m entries and the kColPad pad entries the
// wedge sweeps read past a grab, all at 32-bit positions
constexpr uint64_t kMaxEdges = (1ull << 31) - kColPad;
// launchers defined in prep.hip / plan.hip / wedge.hip
hipError_t launch_degree(const int32_t*, const int32_t*, const int8_t*, uint64_t, uint32_t, uint32_t,
                         uint32_t*, uint2*, Control*, hipStream_t);
size_t radix_tmp_bytes(uint32_t n);
hipError_t radix_sort_by_key(const uint32_t*, uint32_t, uint32_t, uint32_t*, uint32_t*, uint32_t*,
                             uint32_t*, void*, size_t, uint32_t**, hipStream_t,
                             uint32_t** keys_result = nullptr);
hipError_t launch_sides(const uint32_t*, uint32_t, uint32_t, uint32_t*, hipStream_t);
hipError_t launch_assign(const uint32_t*, const uint32_t*, const uint32_t*, uint32_t, uint32_t,
                         uint32_t*, uint32_t*, uint32_t*, hipStream_t);
hipError_t launch_scatter(const int32_t*, const int32_t*, const int8_t*, uint64_t, uint32_t,
                          uint32_t, const uint32_t*, const uint32_t*, const uint2*, uint2*,
                          uint32_t*, hipStream_t);
hipError_t launch_row_sort(const uint32_t*, const uint32_t*, const uint32_t*, uint32_t*, Dims,
                           Control*, uint32_t, hipStream_t);
hipError_t launch_lowcount(const uint32_t*, const uint32_t*, const uint32_t*, uint32_t, uint32_t*,
                           hipStream_t);
hipError_t launch_records(const uint32_t*, const uint32_t*, const uint32_t*, const uint32_t*, Dims,
                          uint64_t, uint4*, u64*, u64*, uint32_t*, hipStream_t);
hipError_t launch_tile_table(const uint32_t*, const uint32_t*, Dims, const Control*, uint32_t*,
                             uint32_t, hipStream_t);
hipError_t launch_plan_count(const u64*, const u64*, const uint32_t*, const uint32_t*, Dims,
                             uint32_t*, u64*, uint32_t*, uint32_t*, uint32_t*, u64*, u64*, u64*,
                             Control*, hipStream_t);
hipError_t launch_gather_totals(const uint32_t*, const u64*, const uint32_t*, const uint32_t*,
                                const uint32_t*, const u64*, uint32_t, Control*, hipStream_t);
hipError_t launch_plan_write(const u64*, const uint32_t*, const uint32_t*, const uint32_t*,
                             const uint32_t*, const uint32_t*, const u64*, const uint32_t*,
                             const uint32_t*, const uint32_t*, Dims, uint32_t, Piece*, u64*,
                             uint32_t*, uint32_t*, uint32_t, uint32_t, uint32_t*, const Control*,
                             hipStream_t);
hipError_t launch_short_wedges(const uint4*, uint32_t, const uint32_t*, const uint32_t*,
                               const uint32_t*, const uint32_t*, const uint32_t*, const uint32_t*,
                               uint32_t, uint32_t*, uint32_t*, uint32_t*, uint32_t*, uint16_t*,
                               bool, hipStream_t);
size_t short_wedge_chunk_slots(uint64_t m);
hipError_t launch_wedge(const Piece*, const uint32_t*, const uint32_t*, uint32_t, uint32_t, uint32_t, Piece*,
                        uint32_t, const uint4*, const uint32_t*, const uint32_t*, Dims, const uint32_t[2], u64*,
                        const uint32_t*, const uint32_t*, const uint32_t*, Control*, u64*, u64*,
                        uint32_t, uint32_t, hipStream_t);
hipError_t launch_pv_out(const u64*, const uint32_t*, Dims, u64*, hipStream_t);
hipError_t launch_ingest(const IngestArgs&, hipStream_t);
hipError_t launch_batch_keys(const uint32_t*, Dims, uint32_t, uint32_t*, hipStream_t);
hipError_t launch_dup_graphs(const uint32_t*, const uint32_t*, Dims, const Control*, hipStream_t);
hipError_t launch_row_keys(const uint32_t*, Dims, uint32_t, uint32_t*, hipStream_t);
hipError_t launch_graph_wedges(const u64*, Dims, u64*, hipStream_t);
}  // namespace bbc

using namespace bbc;

// ---------------------------------------------------------------------------
// Device workspace: one growing buffer carved into 256-byte aligned slices.
struct Arena {
    char* base = nullptr;
    size_t cap = 0;
    size_t used = 0;
};

enum { kEvStart, kEvPrepEnd, kEvPlanA, kEvPlanB, kEvPlanC, kEvWedgeA, kEvWedgeB, kEvEnd,
       kEvSwA, kEvSwB, kNumEv };
constexpr int kNumPhases = 5;  // see bbc_last_phase_ms

struct bbc_context {
    int device = 0;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    uint32_t num_cus = 0;
    size_t budget = 0;  // 0 = unlimited
    Arena prep, plan, batch;
    Control* host_ctl = nullptr;  // pinned
    hipEvent_t ev[kNumEv] = {};
    bool timing = false;
    bool timing_valid = false;
    double phase_ms[kNumPhases] = {0, 0, 0, 0, 0};
    int64_t stats[14] = {0};
    uint32_t hash_target = bbc::kDefaultHashTarget;
    uint32_t probe_limit = bbc::kDefaultProbeLimit;
    uint64_t chunk_min = bbc::kRecordChunkWedges;
    uint32_t light_max = bbc::kLightMax;
    uint32_t grab_div = 16;
    uint32_t wave_share = (uint32_t)bbc::kWaveShare;
    uint64_t union_edges = bbc::kBatchMaxEdges;
    int64_t* pv_host = nullptr;  // pinned staging of per-vertex counts
    size_t pv_host_cap = 0;
    bool use_graphs = false;     // capture the two device segments and replay them
    struct GraphSlot {
        std::vector<uint64_t> key;
        hipGraphExec_t exec = nullptr;
    } seg[2];
    int64_t graph_captures = 0, graph_replays = 0;
    // an allocation-free call carves its workspace from this device's static
    // scratch array instead of the arenas (NULL: arenas)
    char* fixed_base = nullptr;
    size_t fixed_cap = 0, fixed_used = 0;
    size_t last_need = 0;  // arena bytes the last refused growth asked for in total
    char err[512] = {0};
};

static bbc_status fail(bbc_context* c, bbc_status s, const char* fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(c->err, sizeof(c->err), fmt, ap);
    va_end(ap);
    return s;
}

#define HIPCHECK(ctx, call)                                                                     \
    do {                                                                                        \
        hipError_t e_ = (call);                                                                 \
        if (e_ != hipSuccess)                                                                   \
            return fail((ctx), BBC_ERR_DEVICE, "%s failed: %s", #call, hipGetErrorString(e_));  \
    } while (0)

static size_t align_up(size_t x) { return (x + 255) & ~(size_t)255; }

static size_t total_reserved(const bbc_context* c) {
    return c->prep.cap + c->plan.cap + c->batch.cap;
}

static bbc_status arena_reserve(bbc_context* c, Arena& a, size_t bytes) {
    if (bytes <= a.cap) return BBC_OK;
    size_t want = bytes + bytes / 4;
    if (c->budget && total_reserved(c) - a.cap + want > c->budget) {
        want = bytes;
        c->last_need = total_reserved(c) - a.cap + bytes;
        if (total_reserved(c) - a.cap + want > c->budget)
            return fail(c, BBC_ERR_OUT_OF_MEMORY,
                        "device workspace of %zu bytes exceeds BBC_MAX_DEVICE_BYTES=%zu", bytes,
                        c->budget);
    }
    if (a.base) {
        hipError_t e = hipStreamSynchronize(c->stream);
        if (e != hipSuccess) return fail(c, BBC_ERR_DEVICE, "hipStreamSynchronize: %s", hipGetErrorString(e));
        (void)hipFree(a.base);
        a.base = nullptr;
        a.cap = 0;
    }
    void* p = nullptr;
    hipError_t e = hipMalloc(&p, want);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        e = hipMalloc(&p, bytes);
        want = bytes;
    }
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return fail(c, BBC_ERR_OUT_OF_MEMORY, "hipMalloc(%zu) failed", bytes);
    }
    a.base = (char*)p;
    a.cap = want;
    return BBC_OK;
}

// ---- for the counting service (server.hip): a context's resident arenas,
// releasing them, and capping their total
namespace bbc {
size_t context_resident_bytes(const bbc_context* c) { return total_reserved(c); }
size_t context_last_need(const bbc_context* c) { return c->last_need; }
void context_set_budget(bbc_context* c, size_t bytes) {
    c->budget = bytes;
    c->last_need = 0;
}
bool context_trim(bbc_context* c) {
    if (hipSetDevice(c->device) != hipSuccess || hipStreamSynchronize(c->stream) != hipSuccess) {
        (void)hipGetLastError();
        return false;
    }
    for (Arena* a : {&c->prep, &c->plan, &c->batch}) {
        if (a->base) (void)hipFree(a->base);
        a->base = nullptr;
        a->cap = a->used = 0;
    }
    for (auto& g : c->seg)  // replay graphs point into the freed arenas
        if (g.exec) {
            (void)hipGraphExecDestroy(g.exec);
            g.exec = nullptr;
            g.key.clear();
        }
    (void)hipGetLastError();
    return true;
}
}  // namespace bbc

// Workspace for one pipeline stage: the arena `a` grown to `bytes`, or, in an
// allocation-free call, the next `bytes` of the fixed scratch (an error, never
// an allocation, when it does not fit).
static bbc_status workspace(bbc_context* c, Arena& a, size_t bytes, char** base) {
    if (!c->fixed_base) {
        bbc_status s = arena_reserve(c, a, bytes);
        *base = a.base;
        return s;
    }
    if (bytes > c->fixed_cap - c->fixed_used)
        return fail(c, BBC_ERR_TOO_LARGE,
                    "workspace of %zu bytes exceeds the %zu bytes of allocation-free scratch left",
                    bytes, c->fixed_cap - c->fixed_used);
    *base = c->fixed_base + c->fixed_used;
    c->fixed_used += (bytes + 255) & ~(size_t)255;
    return BBC_OK;
}

// The scratch of bbc_count_noalloc: one array per device, held for the life of
// the process and shared by every allocation-free call on that device.  Host
// code never uses the symbol itself as an address; it uses the device address
// that hipGetSymbolAddress returns for the device (resolved once per device in
// bbc_create, with the device current).
static __device__ __align__(256) char scratch[BBC_NOALLOC_SCRATCH_BYTES];
constexpr int kMaxDevices = 64;
static char* g_scratch_ptr[kMaxDevices];
static bool g_scratch_done[kMaxDevices];
static std::mutex g_scratch_mu;

static void resolve_scratch(int device) {
    if (device < 0 || device >= kMaxDevices) return;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (g_scratch_done[device]) return;
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) == hipSuccess)
        g_scratch_ptr[device] = (char*)p;
    else
        (void)hipGetLastError();  // left NULL: bbc_count_noalloc reports BBC_ERR_DEVICE
    g_scratch_done[device] = true;
}

static char* scratch_ptr(int device) {
    if (device < 0 || device >= kMaxDevices) return nullptr;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    return g_scratch_ptr[device];
}

// Two-pass layout helper: first pass measures, second pass hands out pointers.
struct Carver {
    char* base;
    size_t off = 0;
    explicit Carver(char* b) : base(b) {}
    template <typename T>
    T* take(size_t count) {
        T* p = base ? (T*)(base + off) : nullptr;
        off += align_up(count * sizeof(T) + 1);
        return p;
    }
};

struct PrepBufs {
    int32_t* eu;
    int32_t* ev;
    int8_t* sg;
    uint32_t *deg, *k0, *v0, *k1, *v1, *flag, *cnt_u, *sidx_of, *rowdeg, *rowcross, *row_ptr,
        *cursor, *col_in, *col, *lowcnt, *mptr, *tb, *hp, *hp_off, *lf, *lf_off, *gs, *gs_off,
        *tc, *tc_off;
    uint2* vx;  // per input vertex: {sidx, row start} (the scatter's lookups)
    u64 *lr, *lr_off, *wu, *wsu, *swc, *swc_off;
    uint4* recs;
    void* rtmp;
    void* stmp;
    size_t rtmp_bytes, stmp_bytes;
    Control* ctl;
};

static size_t carve_prep(Carver& cv, PrepBufs& b, uint32_t n, uint64_t m, bool copy_in,
                         uint64_t tb_total) {
    b.ctl = cv.take<Control>(1);
    if (copy_in) {
        b.eu = cv.take<int32_t>(m);
        b.ev = cv.take<int32_t>(m);
        b.sg = cv.take<int8_t>(m);
    }
    b.deg = cv.take<uint32_t>(n);
    b.k0 = cv.take<uint32_t>(n);
    b.v0 = cv.take<uint32_t>(n);
    b.k1 = cv.take<uint32_t>(n);
    b.v1 = cv.take<uint32_t>(n);
    b.flag = cv.take<uint32_t>(n);
    b.cnt_u = cv.take<uint32_t>(n + 1);
    b.sidx_of = cv.take<uint32_t>(n);
    b.rowdeg = cv.take<uint32_t>(n);
    b.rowcross = cv.take<uint32_t>(n);
    b.row_ptr = cv.take<uint32_t>(n + 1);
    b.cursor = cv.take<uint32_t>(n);
    b.vx = cv.take<uint2>(n);
    b.col_in = cv.take<uint32_t>(2 * m);
    b.col = cv.take<uint32_t>(2 * m + kColPad);
    b.lowcnt = cv.take<uint32_t>(n);
    b.mptr = cv.take<uint32_t>(n + 1);
    b.recs = cv.take<uint4>(m);
    b.wu = cv.take<u64>(n);
    b.tb = cv.take<uint32_t>(tb_total);
    b.hp = cv.take<uint32_t>(n);
    b.hp_off = cv.take<uint32_t>(n + 1);
    b.lr = cv.take<u64>(n);
    b.lr_off = cv.take<u64>(n + 1);
    b.lf = cv.take<uint32_t>(n);
    b.lf_off = cv.take<uint32_t>(n + 1);
    b.gs = cv.take<uint32_t>(n);
    b.gs_off = cv.take<uint32_t>(n + 1);
    b.tc = cv.take<uint32_t>(n);
    b.tc_off = cv.take<uint32_t>(n + 1);
    b.wsu = cv.take<u64>(n);
    b.swc = cv.take<u64>(n);
    b.swc_off = cv.take<u64>(n + 1);
    b.rtmp_bytes = radix_tmp_bytes(n);
    b.rtmp = cv.take<char>(b.rtmp_bytes);
    b.stmp_bytes = scan_tmp_bytes(n + 1);
    b.stmp = cv.take<char>(b.stmp_bytes);
    return cv.off;
}

static uint32_t bitlen(uint64_t x) {
    uint32_t b = 0;
    while (x) {
        b++;
        x >>= 1;
    }
    return b;
}

static float ev_ms(bbc_context* c, int a, int b) {
    float ms = 0;
    if (hipEventElapsedTime(&ms, c->ev[a], c->ev[b]) != hipSuccess) {
        (void)hipGetLastError();
        return 0;
    }
    return ms;
}

// ---------------------------------------------------------------------------
extern "C" {

int bbc_version(void) { return 10000; }

const char* bbc_status_string(bbc_status s) {
    switch (s) {
        case BBC_PENDING: return "pending";
        case BBC_OK: return "ok";
        case BBC_ERR_INVALID_ARG: return "invalid argument";
        case BBC_ERR_VERTEX_RANGE: return "vertex id out of range";
        case BBC_ERR_BAD_SIGN: return "edge sign not +1/-1";
        case BBC_ERR_DUPLICATE_EDGE: return "duplicate edge";
        case BBC_ERR_TOO_LARGE: return "graph too large";
        case BBC_ERR_OVERFLOW: return "count overflows int64";
        case BBC_ERR_OUT_OF_MEMORY: return "out of device memory";
        case BBC_ERR_DEVICE: return "HIP device error";
        case BBC_ERR_NOT_IMPLEMENTED: return "not implemented";
        case BBC_ERR_INTERNAL: return "internal capacity exceeded";
    }
    return "unknown status";
}

const char* bbc_last_error(const bbc_context* ctx) { return ctx ? ctx->err : ""; }

bbc_status bbc_create(int device, void* hip_stream, bbc_context** out) {
    if (!out) return BBC_ERR_INVALID_ARG;
    *out = nullptr;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev) {
        (void)hipGetLastError();
        return BBC_ERR_DEVICE;
    }
    bbc_context* c = new bbc_context();
    c->device = device;
    if (hipSetDevice(device) != hipSuccess) {
        delete c;
        return BBC_ERR_DEVICE;
    }
    int cus = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess ||
        cus <= 0)
        cus = 256;
    c->num_cus = (uint32_t)cus;
    if (hip_stream) {
        c->stream = (hipStream_t)hip_stream;
    } else {
        if (hipStreamCreate(&c->stream) != hipSuccess) {
            delete c;
            return BBC_ERR_DEVICE;
        }
        c->own_stream = true;
    }
    const char* b = getenv("BBC_MAX_DEVICE_BYTES");
    if (b && *b) c->budget = (size_t)strtoull(b, nullptr, 10);
    void* h = nullptr;
    if (hipHostMalloc(&h, sizeof(Control), hipHostMallocDefault) != hipSuccess) {
        bbc_destroy(c);
        return BBC_ERR_DEVICE;
    }
    c->host_ctl = (Control*)h;
    resolve_scratch(device);  // the device is current
    for (int i = 0; i < kNumEv; ++i)
        if (hipEventCreate(&c->ev[i]) != hipSuccess) {
            bbc_destroy(c);
            return BBC_ERR_DEVICE;
        }
    *out = c;
    return BBC_OK;
}

void bbc_destroy(bbc_context* c) {
    if (!c) return;
    (void)hipSetDevice(c->device);
    if (c->stream) (void)hipStreamSynchronize(c->stream);
    if (c->prep.base) (void)hipFree(c->prep.base);
    if (c->plan.base) (void)hipFree(c->plan.base);
    if (c->batch.base) (void)hipFree(c->batch.base);
    if (c->pv_host) (void)hipHostFree(c->pv_host);
    for (auto& g : c->seg)
        if (g.exec) (void)hipGraphExecDestroy(g.exec);
    if (c->host_ctl) (void)hipHostFree(c->host_ctl);
    for (int i = 0; i < kNumEv; ++i)
        if (c->ev[i]) (void)hipEventDestroy(c->ev[i]);
    if (c->own_stream && c->stream) (void)hipStreamDestroy(c->stream);
    (void)hipGetLastError();
    delete c;
}

bbc_status bbc_set_timing(bbc_context* c, int enabled) {
    if (!c) return BBC_ERR_INVALID_ARG;
    c->timing = enabled != 0;
    return BBC_OK;
}

bbc_status bbc_set_param(bbc_context* c, int param, int64_t value) {
    if (!c) return BBC_ERR_INVALID_ARG;
    switch (param) {
    case BBC_PARAM_HASH_TARGET:
        if (value < 64 || value > (1 << 20)) return BBC_ERR_INVALID_ARG;
        c->hash_target = (uint32_t)value;
        return BBC_OK;
    case BBC_PARAM_PROBE_LIMIT:
        if (value < 1 || value > (int64_t)bbc::kHashSlots) return BBC_ERR_INVALID_ARG;
        c->probe_limit = (uint32_t)value;
        return BBC_OK;
    case BBC_PARAM_CHUNK_WEDGES:
        if (value < 1024 || value > (1ll << 40)) return BBC_ERR_INVALID_ARG;
        c->chunk_min = (uint64_t)value;
        return BBC_OK;
    case BBC_PARAM_GRAPHS:
        if (value != 0 && value != 1) return BBC_ERR_INVALID_ARG;
        c->use_graphs = value != 0;
        return BBC_OK;
    case BBC_PARAM_LIGHT_MAX:
        if (value < 16 || value > (int64_t)bbc::kLightMax) return BBC_ERR_INVALID_ARG;
        c->light_max = (uint32_t)value;
        return BBC_OK;
    case BBC_PARAM_GRAB_DIV:
        if (value < 4 || value > 64) return BBC_ERR_INVALID_ARG;
        c->grab_div = (uint32_t)value;
        return BBC_OK;
    case BBC_PARAM_UNION_EDGES:
        if (value < (1 << 16) || value > (int64_t)bbc::kBatchMaxEdges) return BBC_ERR_INVALID_ARG;
        c->union_edges = (uint64_t)value;
        return BBC_OK;
    case BBC_PARAM_WAVE_SHARE:
        if (value < 0 || value > (1 << 20)) return BBC_ERR_INVALID_ARG;
        c->wave_share = (uint32_t)value;
        return BBC_OK;
    default:
        return BBC_ERR_INVALID_ARG;
    }
}

bbc_status bbc_get_param(const bbc_context* c, int param, int64_t* value) {
    if (!c || !value) return BBC_ERR_INVALID_ARG;
    switch (param) {
    case BBC_PARAM_HASH_TARGET: *value = c->hash_target; return BBC_OK;
    case BBC_PARAM_PROBE_LIMIT: *value = c->probe_limit; return BBC_OK;
    case BBC_PARAM_CHUNK_WEDGES: *value = (int64_t)c->chunk_min; return BBC_OK;
    case BBC_PARAM_GRAPHS: *value = c->use_graphs ? 1 : 0; return BBC_OK;
    case BBC_PARAM_GRAPH_CAPTURES: *value = c->graph_captures; return BBC_OK;
    case BBC_PARAM_GRAPH_REPLAYS: *value = c->graph_replays; return BBC_OK;
    case BBC_PARAM_LIGHT_MAX: *value = c->light_max; return BBC_OK;
    case BBC_PARAM_GRAB_DIV: *value = c->grab_div; return BBC_OK;
    case BBC_PARAM_UNION_EDGES: *value = (int64_t)c->union_edges; return BBC_OK;
    case BBC_PARAM_WAVE_SHARE: *value = c->wave_share; return BBC_OK;
    default: return BBC_ERR_INVALID_ARG;
    }
}

bbc_status bbc_last_phase_ms(const bbc_context* c, int phase, double* ms) {
    if (!c || !ms || phase < 0 || phase >= kNumPhases || !c->timing_valid) return BBC_ERR_INVALID_ARG;
    *ms = c->phase_ms[phase];
    return BBC_OK;
}

bbc_status bbc_last_stats(const bbc_context* c, int64_t* stats, int n) {
    if (!c || !stats || n < 0) return BBC_ERR_INVALID_ARG;
    for (int i = 0; i < n && i < 14; ++i) stats[i] = c->stats[i];
    return BBC_OK;
}

int64_t bbc_workspace_bytes(int32_t n_u, int32_t n_v, int64_t n_edges) {
    if (n_u < 0 || n_v < 0 || n_edges < 0) return -1;
    const uint64_t n64 = (uint64_t)n_u + (uint64_t)n_v;
    if (n64 >= (1ull << 30) || (uint64_t)n_edges >= kMaxEdges) return -1;
    const uint32_t n = (uint32_t)n64;
    const uint64_t m = (uint64_t)n_edges;
    const uint32_t nt0 = ((uint32_t)n_u + kTile - 1) / kTile, nt1 = ((uint32_t)n_v + kTile - 1) / kTile;
    const uint64_t tb = std::min<uint64_t>((uint64_t)n_u, m / (kLongDeg + 1)) * (nt1 + 1) +
                        std::min<uint64_t>((uint64_t)n_v, m / (kLongDeg + 1)) * (nt0 + 1);
    PrepBufs b;
    Carver probe(nullptr);
    const size_t prep = carve_prep(probe, b, n, m, true, tb);
    // planning workspace: about one piece per start plus record chunks and
    // merge rows; taken generously as 96 bytes per vertex and 8 per edge
    const size_t plan = 96ull * n + 8ull * m + 2 * short_wedge_chunk_slots(m) + (1u << 20);
    return (int64_t)(prep + plan);
}
}  // extern "C"

// ---------------------------------------------------------------------------
// One run of the counting pipeline over a graph, or over the union graph of a
// batch, whose edges are on the device (or on the host with copy_in).

struct BatchDev {
    uint32_t n_graphs;
    uint32_t max_side;       // largest |U| or |V| of a graph (bounds the degrees)
    const uint32_t* blk[2];  // device: sidx block starts per side (n_graphs + 1)
    u64* gres;               // device: per graph {balanced, unbalanced, wedges, -}
    u64* gerr;               // device: per graph first bad edge << 4 | code, ~0 if none
};

struct RunIn {
    uint32_t nu, nv;
    uint64_t m;
    const int32_t* eu;
    const int32_t* ev;
    const int8_t* sg;
    bool copy_in;            // eu/ev/sg are host pointers
    const BatchDev* bt;      // NULL: one graph
    const IngestArgs* ingest;  // batches: fills eu/ev/sg first (reports into the control block)
    bool per_vertex;         // per-vertex counts wanted (one graph only)
    int64_t* pv_host;        // host, n entries: where they are copied (NULL: left on the device)
};

struct RunOut {
    Control h;               // the control block after the run
    bool input_error;        // stopped after the input checks (h.edge_err / h.dup)
    uint32_t n_items, n_heavy;
    uint32_t n;
    const u64* pv_dev;       // per-vertex counts by input id on the device (per-vertex mode)
};

// Runs one device segment of the pipeline: eagerly, or (graph mode) as a HIP
// graph captured the first time its key is seen and replayed while the key
// stays the same.  The key holds every size, address and setting a launch of
// the segment depends on.  Segments record no memset nodes (all clearing is
// done by fill kernels) and no events.
template <class F>
static bbc_status run_segment(bbc_context* c, int which, const std::vector<uint64_t>& key,
                              F&& launches) {
    if (!c->use_graphs) return launches();
    hipStream_t st = c->stream;
    auto& slot = c->seg[which];
    if (!slot.exec || slot.key != key) {
        if (slot.exec) {
            HIPCHECK(c, hipGraphExecDestroy(slot.exec));
            slot.exec = nullptr;
        }
        slot.key.clear();
        HIPCHECK(c, hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
        const bbc_status s = launches();
        hipGraph_t g = nullptr;
        const hipError_t e = hipStreamEndCapture(st, &g);
        if (s) {
            if (g) (void)hipGraphDestroy(g);
            return s;
        }
        if (e != hipSuccess) return fail(c, BBC_ERR_DEVICE, "hipStreamEndCapture: %s", hipGetErrorString(e));
        const hipError_t e2 = hipGraphInstantiate(&slot.exec, g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        if (e2 != hipSuccess) {
            slot.exec = nullptr;
            return fail(c, BBC_ERR_DEVICE, "hipGraphInstantiate: %s", hipGetErrorString(e2));
        }
        slot.key = key;
        c->graph_captures++;
    } else {
        c->graph_replays++;
    }
    HIPCHECK(c, hipGraphLaunch(slot.exec, st));
    return BBC_OK;
}

static bbc_status run_pipeline(bbc_context* c, const RunIn& in, RunOut& ro) {
    hipStream_t st = c->stream;
    const uint32_t nu = in.nu, nv = in.nv, n = nu + nv;
    const uint64_t m = in.m;
    const bool copy_in = in.copy_in;
    const BatchDev* bt = in.bt;
    ro.input_error = false;
    ro.n_items = ro.n_heavy = 0;
    ro.n = n;
    ro.pv_dev = nullptr;

    Dims d;
    d.n_u = nu;
    d.n_v = nv;
    d.n = n;
    d.base[0] = 0;
    d.base[1] = nu;
    d.size[0] = nu;
    d.size[1] = nv;
    d.ntile[0] = (nu + kTile - 1) / kTile;
    d.ntile[1] = (nv + kTile - 1) / kTile;
    d.hash_target = c->hash_target;
    d.probe_limit = c->probe_limit;
    d.chunk_min = c->chunk_min;
    d.n_graphs = bt ? bt->n_graphs : 1u;
    d.blk[0] = bt ? bt->blk[0] : nullptr;
    d.blk[1] = bt ? bt->blk[1] : nullptr;
    d.gerr = bt ? bt->gerr : nullptr;
    d.rlist = nullptr;
    d.per_vertex = in.per_vertex ? 1u : 0u;
    d.light_window = kLightWindow16;
    d.light_max = c->light_max;
    d.grab_div = c->grab_div;
    d.wave_share = c->wave_share;
    // rows of side Y with more than kLongDeg entries: at most m / (kLongDeg + 1) per side
    uint64_t maxlong0 = std::min<uint64_t>(nu, m / (kLongDeg + 1));
    uint64_t maxlong1 = std::min<uint64_t>(nv, m / (kLongDeg + 1));
    d.tb_off[0] = 0;
    d.tb_off[1] = maxlong0 * (d.ntile[1] + 1);
    uint64_t tb_total = d.tb_off[1] + maxlong1 * (d.ntile[0] + 1);
    if (bt) tb_total = 0;  // a batch never splits a start into end-vertex tiles

    // ---- workspace
    PrepBufs b;
    char* prep_base = nullptr;
    {
        Carver probe(nullptr);
        size_t need = carve_prep(probe, b, n, m, copy_in, tb_total);
        bbc_status s = workspace(c, c->prep, need, &prep_base);
        if (s) return s;
        Carver cv(prep_base);
        carve_prep(cv, b, n, m, copy_in, tb_total);
    }
    const int32_t* eu = in.eu;
    const int32_t* ev = in.ev;
    const int8_t* sg = in.sg;
    if (copy_in) {
        HIPCHECK(c, hipMemcpyAsync(b.eu, in.eu, m * 4, hipMemcpyHostToDevice, st));
        HIPCHECK(c, hipMemcpyAsync(b.ev, in.ev, m * 4, hipMemcpyHostToDevice, st));
        HIPCHECK(c, hipMemcpyAsync(b.sg, in.sg, m, hipMemcpyHostToDevice, st));
        eu = b.eu;
        ev = b.ev;
        sg = b.sg;
    }
    const bool tm_out = c->timing;                   // events around the segments
    const bool tm = c->timing && !c->use_graphs;     // events between kernels
    const bool bt_on = bt != nullptr;
    const uint32_t deg_bits = bt ? bitlen(std::min<uint64_t>(m, bt->max_side)) : 0;
    const uint32_t g_bits = bt ? bitlen(bt->n_graphs - 1) : 0;
    if (bt && deg_bits + g_bits > 32)
        return fail(c, BBC_ERR_INTERNAL, "batch sort key needs %u bits", deg_bits + g_bits);
    // replay keys (graph mode only: an allocation-free call builds none)
    std::vector<uint64_t> keyA;
    if (c->use_graphs)
        keyA = {n, nu, nv, m, (uint64_t)eu, (uint64_t)ev, (uint64_t)sg,
                (uint64_t)prep_base, tb_total, d.hash_target, d.probe_limit,
                d.chunk_min, d.per_vertex, bt_on, deg_bits, g_bits, d.light_max, d.grab_div,
                d.wave_share};
    if (bt && c->use_graphs) {
        for (uint64_t x : {(uint64_t)bt->n_graphs, (uint64_t)bt->blk[0], (uint64_t)bt->blk[1],
                           (uint64_t)bt->gres, (uint64_t)bt->gerr})
            keyA.push_back(x);
    }
    if (in.ingest && c->use_graphs) {
        const IngestArgs& ia = *in.ingest;
        for (uint64_t x : {(uint64_t)ia.src_u, (uint64_t)ia.src_v, (uint64_t)ia.src_s,
                           (uint64_t)ia.src_off, (uint64_t)ia.dst_off, (uint64_t)ia.gnu,
                           (uint64_t)ia.gnv, (uint64_t)ia.uoff, (uint64_t)ia.voff,
                           (uint64_t)ia.n_graphs, (uint64_t)ia.m, (uint64_t)ia.eu,
                           (uint64_t)ia.ev, (uint64_t)ia.sg, (uint64_t)ia.gerr})
            keyA.push_back(x);
    }
    if (tm_out) HIPCHECK(c, hipEventRecord(c->ev[kEvStart], st));
    {
        Control z;
        memset(&z, 0, sizeof(z));
        z.edge_err = ~0ull;
        *c->host_ctl = z;  // read by the segment's upload (also when replayed)
    }
    uint32_t* inv = nullptr;
    bbc_status sA = run_segment(c, 0, keyA, [&]() -> bbc_status {
    // ---- control block
    HIPCHECK(c, hipMemcpyAsync(b.ctl, c->host_ctl, sizeof(Control), hipMemcpyHostToDevice, st));
    if (in.ingest) {
        IngestArgs ia = *in.ingest;
        ia.ctl = b.ctl;
        HIPCHECK(c, launch_ingest(ia, st));
    }

    // ---- 1. degrees + validation
    HIPCHECK(c, fill_u32(b.deg, 0, n, st));
    HIPCHECK(c, fill_u32(b.col + 2 * m, kColPadValue, kColPad, st));
    // every edge's slots in its two rows go to b.recs (free until the records)
    uint2* slots = reinterpret_cast<uint2*>(b.recs);
    HIPCHECK(c, launch_degree(eu, ev, sg, m, nu, nv, b.deg, slots, b.ctl, st));
    // ---- 2. priority order: stable sort of vertex ids by degree (by graph,
    // then degree, for a batch)
    if (bt) {
        uint32_t* key = b.rowdeg;  // free until the row degrees are assigned
        HIPCHECK(c, launch_batch_keys(b.deg, d, deg_bits, key, st));
        HIPCHECK(c, radix_sort_by_key(key, n, deg_bits + g_bits, b.k0, b.v0, b.k1, b.v1, b.rtmp,
                                      b.rtmp_bytes, &inv, st));
    } else {
        uint32_t maxdeg_bound = (uint32_t)std::min<uint64_t>(m, std::max(nu, nv));
        HIPCHECK(c, radix_sort_by_key(b.deg, n, bitlen(maxdeg_bound), b.k0, b.v0, b.k1, b.v1, b.rtmp,
                                      b.rtmp_bytes, &inv, st));
    }
    // ---- 3. per-side index and cross counts
    HIPCHECK(c, launch_sides(inv, n, nu, b.flag, st));
    HIPCHECK(c, scan_excl_u32(b.flag, b.cnt_u, n, b.stmp, b.stmp_bytes, st));
    HIPCHECK(c, launch_assign(inv, b.cnt_u, b.deg, n, nu, b.sidx_of, b.rowdeg, b.rowcross, st));
    if (bt) {
        // rows of a batch are in (graph, degree) order; the row sort works on
        // length classes, so it gets the rows in (side, length) order
        uint32_t* rlist = nullptr;
        HIPCHECK(c, launch_row_keys(b.rowdeg, d, deg_bits, b.flag, st));
        HIPCHECK(c, radix_sort_by_key(b.flag, n, deg_bits + 1, b.k0, b.v0, b.k1, b.v1, b.rtmp,
                                      b.rtmp_bytes, &rlist, st));
        d.rlist = rlist;
    }
    // ---- 4. CSR: offsets, scatter, per-row sort
    HIPCHECK(c, scan_excl_u32(b.rowdeg, b.row_ptr, n, b.stmp, b.stmp_bytes, st));
    HIPCHECK(c, launch_scatter(eu, ev, sg, m, nu, nv, b.sidx_of, b.row_ptr, slots, b.vx, b.col_in,
                               st));
    HIPCHECK(c, launch_row_sort(b.rowdeg, b.row_ptr, b.col_in, b.col, d, b.ctl, c->num_cus, st));
    if (bt) HIPCHECK(c, launch_dup_graphs(b.row_ptr, b.col, d, b.ctl, st));
    // ---- 5. middle counts, 6. records and W_u, 7. tile tables
    HIPCHECK(c, launch_lowcount(b.row_ptr, b.col, b.rowcross, n, b.lowcnt, st));
    HIPCHECK(c, scan_excl_u32(b.lowcnt, b.mptr, n, b.stmp, b.stmp_bytes, st));
    // every start's records in [mptr[u], mptr[u+1]), the long-middle ones
    // first; front[u] (kept in b.cursor) is where u's short ones begin
    HIPCHECK(c, copy_u32(b.mptr + 1, b.cursor, n, st));
    HIPCHECK(c, fill_u64(b.wu, 0, n, st));
    HIPCHECK(c, fill_u64(b.wsu, 0, n, st));
    HIPCHECK(c, launch_records(b.row_ptr, b.col, b.lowcnt, b.mptr, d, m, b.recs, b.wu, b.wsu,
                               b.cursor, st));
    if (!bt) HIPCHECK(c, launch_tile_table(b.row_ptr, b.col, d, b.ctl, b.tb, c->num_cus, st));
    if (tm) HIPCHECK(c, hipEventRecord(c->ev[kEvPrepEnd], st));

    // ---- planning: piece counts, offsets, totals
    HIPCHECK(c, launch_plan_count(b.wu, b.wsu, b.lowcnt, b.row_ptr, d, b.hp, b.lr, b.lf, b.gs, b.tc,
                                  b.swc, &b.ctl->wedges, &b.ctl->active_starts, b.ctl, st));
    if (bt) HIPCHECK(c, launch_graph_wedges(b.wu, d, bt->gres, st));
    {
        const uint32_t* ins[4] = {b.hp, b.lf, b.gs, b.tc};
        uint32_t* outs[4] = {b.hp_off, b.lf_off, b.gs_off, b.tc_off};
        HIPCHECK(c, scan_excl_u32_set(ins, outs, 4, n, b.stmp, b.stmp_bytes, st));
        const u64* ins64[2] = {b.lr, b.swc};
        u64* outs64[2] = {b.lr_off, b.swc_off};
        HIPCHECK(c, scan_excl_u64_set(ins64, outs64, 2, n, b.stmp, b.stmp_bytes, st));
    }
    HIPCHECK(c, launch_gather_totals(b.hp_off, b.lr_off, b.lf_off, b.gs_off, b.tc_off, b.swc_off, n,
                                     b.ctl, st));
    if (tm) HIPCHECK(c, hipEventRecord(c->ev[kEvPlanA], st));
    HIPCHECK(c, hipMemcpyAsync(c->host_ctl, b.ctl, sizeof(Control), hipMemcpyDeviceToHost, st));
    return BBC_OK;
    });
    if (sA) return sA;
    if (tm_out && c->use_graphs) HIPCHECK(c, hipEventRecord(c->ev[kEvPrepEnd], st));
    HIPCHECK(c, hipStreamSynchronize(st));
    Control h = *c->host_ctl;
    ro.h = h;
    if (h.edge_err != ~0ull || h.dup) {
        ro.input_error = true;
        return BBC_OK;
    }
    if (h.internal_err)
        return fail(c, BBC_ERR_INTERNAL, "a batch graph needs end-vertex tiles");

    // ---- planning: write the pieces and the light items
    if (h.tot_heavy + h.tot_light >= (1ull << 31))
        return fail(c, BBC_ERR_INTERNAL, "too many work pieces (%llu)",
                    (unsigned long long)(h.tot_heavy + h.tot_light));
    if (h.tot_sw >= (1ull << 32) || h.tot_tiles >= (1ull << 32) || h.tot_g >= (1ull << 32))
        return fail(c, BBC_ERR_INTERNAL, "planner totals exceed 32 bits (%llu %llu %llu)",
                    (unsigned long long)h.tot_sw, (unsigned long long)h.tot_tiles,
                    (unsigned long long)h.tot_g);
    const uint32_t n_heavy = (uint32_t)h.tot_heavy, n_light = (uint32_t)h.tot_light;
    const uint32_t n_wave = (uint32_t)std::min<u64>(h.n_wave, h.tot_heavy);
    const uint32_t n_dense = (uint32_t)std::min<u64>(h.n_dense_pieces, h.tot_heavy - n_wave);
    const uint64_t n_light_items64 = (h.tot_light_region + d.light_window - 1) / d.light_window;
    const uint32_t n_light_items = (uint32_t)n_light_items64;
    const uint32_t n_items = n_heavy + n_light_items;
    uint32_t first_long[2] = {h.cls[0][4] - d.base[0], h.cls[1][4] - d.base[1]};
    Piece* pieces;
    Piece* redo;  // halves of hashed pieces given up on: at most two per hashed piece
    u64* light_off;
    uint32_t* items_first;
    u64* G;
    uint32_t *hkey, *ok0, *ov0, *ok1, *ov1, *tile_piece, *sw_cnt, *sw_off, *sw_cur, *sw_list;
    uint32_t* sw_mid = nullptr;  // per-vertex mode: the middle row of each listed wedge
    uint16_t* sw_chunk;  // per-piece counts of single-start record chunks (count pass -> fill pass)
    u64 *pv = nullptr, *pv_out = nullptr;
    void* ortmp;
    const size_t ortmp_bytes = radix_tmp_bytes(n_heavy + 1);
    char* plan_base = nullptr;
    {
        auto carve_plan = [&](Carver& cv) {
            pieces = cv.take<Piece>((size_t)n_heavy + n_light);
            redo = cv.take<Piece>(2 * (size_t)(n_heavy - n_dense) + 1);
            light_off = cv.take<u64>((size_t)n_light + 1);
            items_first = cv.take<uint32_t>((size_t)n_light_items + 2);
            G = cv.take<u64>((size_t)h.tot_g + 1);
            hkey = cv.take<uint32_t>((size_t)n_heavy + 1);
            ok0 = cv.take<uint32_t>((size_t)n_heavy + 1);
            ov0 = cv.take<uint32_t>((size_t)n_heavy + 1);
            ok1 = cv.take<uint32_t>((size_t)n_heavy + 1);
            ov1 = cv.take<uint32_t>((size_t)n_heavy + 1);
            ortmp = cv.take<char>(ortmp_bytes);
            tile_piece = cv.take<uint32_t>((size_t)h.tot_tiles + 1);
            sw_cnt = cv.take<uint32_t>((size_t)n_heavy + 1);
            sw_off = cv.take<uint32_t>((size_t)n_heavy + 1);
            sw_cur = cv.take<uint32_t>((size_t)n_heavy + 1);
            sw_list = cv.take<uint32_t>((size_t)h.tot_sw + 1);
            sw_chunk = cv.take<uint16_t>(short_wedge_chunk_slots(m));
            if (in.per_vertex) {
                pv = cv.take<u64>(n);
                pv_out = cv.take<u64>(n);
                sw_mid = cv.take<uint32_t>((size_t)h.tot_sw + 1);
            }
            ro.pv_dev = pv_out;
            return cv.off;
        };
        Carver probe(nullptr);
        size_t need = carve_plan(probe);
        bbc_status s = workspace(c, c->plan, need, &plan_base);
        if (s) return s;
        Carver cv(plan_base);
        carve_plan(cv);
    }
    std::vector<uint64_t> keyB;
    if (c->use_graphs) keyB = keyA;
    if (c->use_graphs)
    for (uint64_t x : {(uint64_t)n_heavy, (uint64_t)n_dense, (uint64_t)n_wave, (uint64_t)n_light, (uint64_t)n_light_items, (uint64_t)h.tot_g,
                       (uint64_t)h.tot_sw, (uint64_t)h.tot_tiles, (uint64_t)plan_base, (uint64_t)first_long[0],
                       (uint64_t)first_long[1], (uint64_t)in.per_vertex, (uint64_t)in.pv_host})
        keyB.push_back(x);
    if (tm_out) HIPCHECK(c, hipEventRecord(c->ev[kEvPlanB], st));
    bbc_status sB = run_segment(c, 1, keyB, [&]() -> bbc_status {
    HIPCHECK(c, fill_u64(G, 0, (size_t)h.tot_g, st));
    if (pv) HIPCHECK(c, fill_u64(pv, 0, n, st));
    HIPCHECK(c, launch_plan_write(b.wu, b.lowcnt, b.row_ptr, b.mptr, b.cursor, b.hp_off, b.lr_off,
                                  b.lf_off, b.gs_off, b.tc_off, d, n_heavy, pieces, light_off, hkey,
                                  tile_piece, n_light, n_light_items, items_first, b.ctl, st));
    // bucket the short-middle wedges of split starts by piece
    HIPCHECK(c, fill_u32(sw_cnt, 0, (size_t)n_heavy + 1, st));
    if (tm) HIPCHECK(c, hipEventRecord(c->ev[kEvSwA], st));
    if (h.tot_sw > 0) {
        HIPCHECK(c, launch_short_wedges(b.recs, (uint32_t)m, b.col, b.cursor, b.tc, b.tc_off,
                                        b.hp_off, tile_piece, nu, sw_cnt, sw_cur, sw_list, sw_mid,
                                        sw_chunk, false, st));
    }
    HIPCHECK(c, scan_excl_u32(sw_cnt, sw_off, n_heavy, ortmp, ortmp_bytes, st));
    if (h.tot_sw > 0) {
        HIPCHECK(c, copy_u32(sw_off, sw_cur, n_heavy, st));
        HIPCHECK(c, launch_short_wedges(b.recs, (uint32_t)m, b.col, b.cursor, b.tc, b.tc_off,
                                        b.hp_off, tile_piece, nu, sw_cnt, sw_cur, sw_list, sw_mid,
                                        sw_chunk, true, st));
    }
    if (tm) HIPCHECK(c, hipEventRecord(c->ev[kEvSwB], st));
    uint32_t* order = nullptr;
    if (n_heavy > 0)  // heavy pieces, most expensive first
        HIPCHECK(c, radix_sort_by_key(hkey, n_heavy, 8, ok0, ov0, ok1, ov1, ortmp, ortmp_bytes,
                                      &order, st));
    if (tm) HIPCHECK(c, hipEventRecord(c->ev[kEvPlanC], st));

    // ---- wedge enumeration and bucket counting
    if (tm) HIPCHECK(c, hipEventRecord(c->ev[kEvWedgeA], st));
    HIPCHECK(c, launch_wedge(pieces, order, items_first, n_heavy, n_dense, n_wave, redo, n_items, b.recs, b.col, b.tb, d,
                             first_long, G, sw_off, sw_list, sw_mid, b.ctl,
                             bt ? bt->gres : nullptr, pv, (uint32_t)(2 * m),
                             c->num_cus, st));
    if (tm) HIPCHECK(c, hipEventRecord(c->ev[kEvWedgeB], st));
    if (pv) {
        HIPCHECK(c, launch_pv_out(pv, b.sidx_of, d, pv_out, st));
        if (in.pv_host)
            HIPCHECK(c, hipMemcpyAsync(in.pv_host, pv_out, 8ull * n, hipMemcpyDeviceToHost, st));
    }
    HIPCHECK(c, hipMemcpyAsync(c->host_ctl, b.ctl, sizeof(Control), hipMemcpyDeviceToHost, st));
    return BBC_OK;
    });
    if (sB) return sB;
    if (tm_out) HIPCHECK(c, hipEventRecord(c->ev[kEvEnd], st));
    HIPCHECK(c, hipStreamSynchronize(st));
    h = *c->host_ctl;
    ro.h = h;
    if (h.internal_err)
        return fail(c, BBC_ERR_INTERNAL,
                    "wedge kernel invariant broken (flags %u: 1 = an unsplit hashed piece gave up, "
                    "4 = a split piece met a short-middle record, 8 = a packed piece reached the "
                    "general kernel, 16 = a one-wave piece exceeds its counter slice)",
                    h.internal_err);
    if (tm_out && !c->use_graphs) {
        c->phase_ms[0] += ev_ms(c, kEvStart, kEvEnd);
        c->phase_ms[1] += ev_ms(c, kEvStart, kEvPrepEnd);
        c->phase_ms[2] += ev_ms(c, kEvWedgeA, kEvWedgeB);
        c->phase_ms[3] += ev_ms(c, kEvPrepEnd, kEvPlanA) + ev_ms(c, kEvPlanB, kEvPlanC);
        c->phase_ms[4] += ev_ms(c, kEvSwA, kEvSwB);
    } else if (tm_out) {  // graph mode: the two replayed segments
        c->phase_ms[0] += ev_ms(c, kEvStart, kEvEnd);
        c->phase_ms[1] += ev_ms(c, kEvStart, kEvPrepEnd);
        c->phase_ms[2] += ev_ms(c, kEvPlanB, kEvEnd);
    }
    ro.n_items = n_items;
    ro.n_heavy = n_heavy;
    return BBC_OK;
}

static void add_stats(bbc_context* c, const RunOut& ro, uint64_t m) {
    c->stats[0] += (int64_t)ro.n;
    c->stats[1] += (int64_t)m;
    c->stats[2] += (int64_t)ro.h.wedges;
    c->stats[3] += (int64_t)m;
    c->stats[4] += (int64_t)ro.n_items;
    c->stats[5] += (int64_t)ro.h.resplits;
    c->stats[6] += (int64_t)ro.h.active_starts;
    c->stats[7] += (int64_t)ro.n_heavy;
    c->stats[8] += (int64_t)ro.h.n_dense;
    c->stats[9] += (int64_t)ro.h.n_dense16;
    c->stats[10] += (int64_t)ro.h.n_hashed;
    c->stats[11] += (int64_t)ro.h.n_dense8;
    c->stats[12] += (int64_t)ro.h.n_dense4;
    c->stats[13] += (int64_t)ro.h.n_wave;
}

static void begin_call(bbc_context* c) {
    c->err[0] = 0;
    c->timing_valid = false;
    memset(c->stats, 0, sizeof(c->stats));
    for (double& p : c->phase_ms) p = 0;
}

extern "C" {

bbc_status bbc_count(bbc_context* c, int32_t n_u, int32_t n_v, int64_t n_edges,
                     const int32_t* edge_u, const int32_t* edge_v, const int8_t* edge_sign,
                     uint32_t flags, bbc_result* out, int64_t* per_vertex) {
    if (!c) return BBC_ERR_INVALID_ARG;
    begin_call(c);
    if (!out) return fail(c, BBC_ERR_INVALID_ARG, "out is NULL");
    if (n_u < 0 || n_v < 0 || n_edges < 0)
        return fail(c, BBC_ERR_INVALID_ARG, "negative size (n_u=%d n_v=%d n_edges=%lld)", n_u, n_v,
                    (long long)n_edges);
    if (flags & ~(uint32_t)(BBC_INPUT_ON_DEVICE | BBC_OUTPUT_ON_DEVICE | BBC_PER_VERTEX))
        return fail(c, BBC_ERR_INVALID_ARG, "unknown flag bits 0x%x", flags);
    if ((flags & BBC_OUTPUT_ON_DEVICE) && !(flags & BBC_PER_VERTEX))
        return fail(c, BBC_ERR_INVALID_ARG, "BBC_OUTPUT_ON_DEVICE without BBC_PER_VERTEX");
    const bool pv_on_device = (flags & BBC_OUTPUT_ON_DEVICE) != 0;
    if (n_edges > 0 && (!edge_u || !edge_v || !edge_sign))
        return fail(c, BBC_ERR_INVALID_ARG, "NULL edge array with n_edges=%lld", (long long)n_edges);
    if ((flags & BBC_PER_VERTEX) && !per_vertex)
        return fail(c, BBC_ERR_INVALID_ARG, "BBC_PER_VERTEX without per_vertex buffer");
    const uint64_t n64 = (uint64_t)n_u + (uint64_t)n_v;
    if (n64 >= (1ull << 30)) return fail(c, BBC_ERR_TOO_LARGE, "n_u + n_v = %llu >= 2^30", (unsigned long long)n64);
    if ((uint64_t)n_edges >= kMaxEdges)
        return fail(c, BBC_ERR_TOO_LARGE, "n_edges = %lld >= 2^31 - %u", (long long)n_edges, kColPad);
    if (n_edges == 0) {
        if ((flags & BBC_PER_VERTEX) && pv_on_device && n64 > 0) {
            HIPCHECK(c, hipSetDevice(c->device));
            HIPCHECK(c, fill_u64((u64*)per_vertex, 0, n64, c->stream));
            HIPCHECK(c, hipStreamSynchronize(c->stream));
        } else if (flags & BBC_PER_VERTEX) {
            memset(per_vertex, 0, 8ull * (size_t)n64);
        }
        out->balanced = out->unbalanced = out->wedges = 0;
        return BBC_OK;
    }
    HIPCHECK(c, hipSetDevice(c->device));
    const bool copy_in = !(flags & BBC_INPUT_ON_DEVICE);
    // per-vertex counts land in a context-owned host buffer first, so that the
    // caller's buffer is written only on success
    int64_t* pvh = nullptr;
    if ((flags & BBC_PER_VERTEX) && !pv_on_device) {
        const size_t bytes = 8ull * (size_t)n64;
        if (c->pv_host_cap < bytes) {
            if (c->pv_host) (void)hipHostFree(c->pv_host);
            c->pv_host = nullptr;
            c->pv_host_cap = 0;
            void* hp = nullptr;
            if (hipHostMalloc(&hp, bytes, hipHostMallocDefault) != hipSuccess) {
                (void)hipGetLastError();
                return fail(c, BBC_ERR_OUT_OF_MEMORY, "pinned host buffer of %zu bytes", bytes);
            }
            c->pv_host = (int64_t*)hp;
            c->pv_host_cap = bytes;
        }
        pvh = c->pv_host;
    }
    RunIn in{(uint32_t)n_u, (uint32_t)n_v, (uint64_t)n_edges, edge_u, edge_v, edge_sign, copy_in,
             nullptr, nullptr, (flags & BBC_PER_VERTEX) != 0, pvh};
    RunOut ro;
    bbc_status s = run_pipeline(c, in, ro);
    if (s) return s;
    const Control& h = ro.h;
    if (ro.input_error) {
        if (h.edge_err != ~0ull) {
            unsigned long long idx = h.edge_err >> 4;
            if ((h.edge_err & 15ull) == kErrRange)
                return fail(c, BBC_ERR_VERTEX_RANGE, "edge %llu: (u=%d, v=%d) outside |U|=%d, |V|=%d",
                            idx, copy_in ? edge_u[idx] : -1, copy_in ? edge_v[idx] : -1, n_u, n_v);
            return fail(c, BBC_ERR_BAD_SIGN, "edge %llu: sign %d is not +1/-1", idx,
                        copy_in ? (int)edge_sign[idx] : 0);
        }
        return fail(c, BBC_ERR_DUPLICATE_EDGE, "a (u, v) pair occurs more than once");
    }
    if (h.balanced > (u64)INT64_MAX || h.unbalanced > (u64)INT64_MAX || h.wedges > (u64)INT64_MAX)
        return fail(c, BBC_ERR_OVERFLOW, "a count exceeds INT64_MAX");
    if (pvh) {
        for (uint64_t x = 0; x < n64; ++x)
            if (pvh[x] < 0) return fail(c, BBC_ERR_OVERFLOW, "vertex %llu: count exceeds INT64_MAX",
                                        (unsigned long long)x);
        memcpy(per_vertex, pvh, 8ull * n64);
    }
    if (pv_on_device) {
        // every vertex count is at most the balanced total, checked above; the
        // caller's buffer is written only now, on success
        HIPCHECK(c, hipMemcpyAsync(per_vertex, ro.pv_dev, 8ull * n64, hipMemcpyDeviceToDevice,
                                   c->stream));
        HIPCHECK(c, hipStreamSynchronize(c->stream));
    }
    c->timing_valid = c->timing;
    add_stats(c, ro, (uint64_t)n_edges);
    out->balanced = (int64_t)h.balanced;
    out->unbalanced = (int64_t)h.unbalanced;
    out->wedges = (int64_t)h.wedges;
    return BBC_OK;
}

bbc_status bbc_count_noalloc(bbc_context* c, int32_t n_u, int32_t n_v, int64_t n_edges,
                             const int32_t* edge_u, const int32_t* edge_v,
                             const int8_t* edge_sign, uint32_t flags, bbc_result* out,
                             int64_t* per_vertex) {
    if (!c) return BBC_ERR_INVALID_ARG;
    if (!(flags & BBC_INPUT_ON_DEVICE)) {
        begin_call(c);
        return fail(c, BBC_ERR_INVALID_ARG, "bbc_count_noalloc needs BBC_INPUT_ON_DEVICE");
    }
    if ((flags & BBC_PER_VERTEX) && !(flags & BBC_OUTPUT_ON_DEVICE)) {
        begin_call(c);
        return fail(c, BBC_ERR_INVALID_ARG,
                    "bbc_count_noalloc: BBC_PER_VERTEX needs BBC_OUTPUT_ON_DEVICE");
    }
    char* base = scratch_ptr(c->device);
    if (!base) {
        begin_call(c);
        return fail(c, BBC_ERR_DEVICE, "the allocation-free scratch of device %d has no address",
                    c->device);
    }
    // the same pipeline as bbc_count, on the scratch and without graph replay
    // (whose capture and key lists allocate)
    c->fixed_base = base;
    c->fixed_cap = BBC_NOALLOC_SCRATCH_BYTES;
    c->fixed_used = 0;
    const bool graphs = c->use_graphs;
    c->use_graphs = false;
    const bbc_status s = bbc_count(c, n_u, n_v, n_edges, edge_u, edge_v, edge_sign, flags, out,
                                   per_vertex);
    c->use_graphs = graphs;
    c->fixed_base = nullptr;
    c->fixed_cap = c->fixed_used = 0;
    return s;
}

// ---------------------------------------------------------------------------
// Batches

static bbc_status status_of_code(u64 e) {
    switch (e & 15ull) {
        case kErrRange: return BBC_ERR_VERTEX_RANGE;
        case kErrSign: return BBC_ERR_BAD_SIGN;
        default: return BBC_ERR_DUPLICATE_EDGE;
    }
}

// Counts the included graphs `gl` (all small) as one union; graphs whose input
// is invalid get their status and the rest are counted again without them.
static bbc_status count_union(bbc_context* c, const std::vector<uint32_t>& all, const int32_t* n_u,
                              const int32_t* n_v, const int64_t* off, const int32_t* edge_u,
                              const int32_t* edge_v, const int8_t* edge_sign, bool on_device,
                              bbc_result* out, int32_t* status) {
    hipStream_t st = c->stream;
    std::vector<uint32_t> gl = all;
    while (!gl.empty()) {
        const uint32_t G = (uint32_t)gl.size();
        // host-side metadata of the included graphs
        std::vector<u64> src_off(G);
        std::vector<uint32_t> dst_off(G + 1), gnu(G), gnv(G), uoff(G + 1), voff(G + 1);
        uint32_t max_side = 1;
        dst_off[0] = uoff[0] = voff[0] = 0;
        for (uint32_t j = 0; j < G; ++j) {
            const uint32_t g = gl[j];
            // host input is copied packed (graph j's edges at dst_off[j]), so
            // graphs counted elsewhere are never copied
            src_off[j] = on_device ? (u64)off[g] : (u64)dst_off[j];
            gnu[j] = (uint32_t)n_u[g];
            gnv[j] = (uint32_t)n_v[g];
            dst_off[j + 1] = dst_off[j] + (uint32_t)(off[g + 1] - off[g]);
            uoff[j + 1] = uoff[j] + gnu[j];
            voff[j + 1] = voff[j] + gnv[j];
            max_side = std::max(max_side, std::max(gnu[j], gnv[j]));
        }
        const uint64_t m = dst_off[G];
        const uint32_t nu = uoff[G], nv = voff[G];
        const uint64_t src_m = on_device ? 0 : m;
        // workspace: metadata, union edges, source copy, per-graph results
        struct {
            u64 *src_off, *gres, *gerr;
            uint32_t *dst_off, *gnu, *gnv, *uoff, *voff;
            int32_t *eu, *ev, *su, *sv;
            int8_t *sg, *ss;
        } w;
        auto carve = [&](Carver& cv) {
            w.src_off = cv.take<u64>(G);
            w.gres = cv.take<u64>(4ull * G);
            w.gerr = cv.take<u64>(G);
            w.dst_off = cv.take<uint32_t>(G + 1);
            w.gnu = cv.take<uint32_t>(G);
            w.gnv = cv.take<uint32_t>(G);
            w.uoff = cv.take<uint32_t>(G + 1);
            w.voff = cv.take<uint32_t>(G + 1);
            w.eu = cv.take<int32_t>(m);
            w.ev = cv.take<int32_t>(m);
            w.sg = cv.take<int8_t>(m);
            w.su = cv.take<int32_t>(src_m);
            w.sv = cv.take<int32_t>(src_m);
            w.ss = cv.take<int8_t>(src_m);
            return cv.off;
        };
        {
            Carver probe(nullptr);
            bbc_status s = arena_reserve(c, c->batch, carve(probe));
            if (s) return s;
            Carver cv(c->batch.base);
            carve(cv);
        }
        HIPCHECK(c, hipMemcpyAsync(w.src_off, src_off.data(), 8ull * G, hipMemcpyHostToDevice, st));
        HIPCHECK(c, hipMemcpyAsync(w.dst_off, dst_off.data(), 4ull * (G + 1), hipMemcpyHostToDevice, st));
        HIPCHECK(c, hipMemcpyAsync(w.gnu, gnu.data(), 4ull * G, hipMemcpyHostToDevice, st));
        HIPCHECK(c, hipMemcpyAsync(w.gnv, gnv.data(), 4ull * G, hipMemcpyHostToDevice, st));
        HIPCHECK(c, hipMemcpyAsync(w.uoff, uoff.data(), 4ull * (G + 1), hipMemcpyHostToDevice, st));
        HIPCHECK(c, hipMemcpyAsync(w.voff, voff.data(), 4ull * (G + 1), hipMemcpyHostToDevice, st));
        const int32_t* su = edge_u;
        const int32_t* sv = edge_v;
        const int8_t* ss = edge_sign;
        if (!on_device) {
            // one copy per run of graphs whose edges follow each other in the input
            for (uint32_t j = 0; j < G;) {
                uint32_t k = j + 1;
                while (k < G && off[gl[k]] == off[gl[k - 1] + 1]) ++k;
                const int64_t e0 = off[gl[j]];
                const uint64_t d0 = dst_off[j], len = dst_off[k] - dst_off[j];
                if (len > 0) {
                    HIPCHECK(c, hipMemcpyAsync(w.su + d0, edge_u + e0, 4 * len, hipMemcpyHostToDevice, st));
                    HIPCHECK(c, hipMemcpyAsync(w.sv + d0, edge_v + e0, 4 * len, hipMemcpyHostToDevice, st));
                    HIPCHECK(c, hipMemcpyAsync(w.ss + d0, edge_sign + e0, len, hipMemcpyHostToDevice, st));
                }
                j = k;
            }
            su = w.su;
            sv = w.sv;
            ss = w.ss;
        }
        HIPCHECK(c, fill_u64(w.gres, 0, 4ull * G, st));
        HIPCHECK(c, fill_u64(w.gerr, ~0ull, G, st));
        RunIn in{nu, nv, m, w.eu, w.ev, w.sg, false, nullptr, nullptr, false, nullptr};
        BatchDev bd;
        bd.n_graphs = G;
        bd.max_side = max_side;
        bd.blk[0] = w.uoff;
        bd.blk[1] = w.voff;
        bd.gres = w.gres;
        bd.gerr = w.gerr;
        in.bt = &bd;
        IngestArgs ia;
        ia.src_u = su;
        ia.src_v = sv;
        ia.src_s = ss;
        ia.src_off = w.src_off;
        ia.dst_off = w.dst_off;
        ia.gnu = w.gnu;
        ia.gnv = w.gnv;
        ia.uoff = w.uoff;
        ia.voff = w.voff;
        ia.n_graphs = G;
        ia.m = m;
        ia.eu = w.eu;
        ia.ev = w.ev;
        ia.sg = w.sg;
        ia.gerr = w.gerr;
        ia.ctl = nullptr;  // set to the run's control block
        in.ingest = &ia;
        RunOut ro;
        bbc_status s = run_pipeline(c, in, ro);
        if (s) return s;
        // per-graph errors (from the ingest or the duplicate check)
        std::vector<u64> gerr(G);
        HIPCHECK(c, hipMemcpyAsync(gerr.data(), w.gerr, 8ull * G, hipMemcpyDeviceToHost, st));
        HIPCHECK(c, hipStreamSynchronize(st));
        std::vector<uint32_t> keep;
        for (uint32_t j = 0; j < G; ++j) {
            if (gerr[j] != ~0ull)
                status[gl[j]] = status_of_code(gerr[j]);
            else
                keep.push_back(gl[j]);
        }
        if (keep.size() != gl.size()) {  // count the valid graphs again without them
            gl.swap(keep);
            continue;
        }
        if (ro.input_error)
            return fail(c, BBC_ERR_INTERNAL, "batch input error without a per-graph cause");
        std::vector<u64> gres(4ull * G);
        HIPCHECK(c, hipMemcpyAsync(gres.data(), w.gres, 32ull * G, hipMemcpyDeviceToHost, st));
        HIPCHECK(c, hipStreamSynchronize(st));
        for (uint32_t j = 0; j < G; ++j) {
            const u64 bal = gres[4 * j], unb = gres[4 * j + 1], wed = gres[4 * j + 2];
            if (bal > (u64)INT64_MAX || unb > (u64)INT64_MAX || wed > (u64)INT64_MAX) {
                status[gl[j]] = BBC_ERR_OVERFLOW;
                continue;
            }
            out[gl[j]].balanced = (int64_t)bal;
            out[gl[j]].unbalanced = (int64_t)unb;
            out[gl[j]].wedges = (int64_t)wed;
        }
        add_stats(c, ro, m);
        break;
    }
    return BBC_OK;
}

bbc_status bbc_count_batch(bbc_context* c, int32_t n_graphs, const int32_t* n_u, const int32_t* n_v,
                           const int64_t* edge_offset, const int32_t* edge_u, const int32_t* edge_v,
                           const int8_t* edge_sign, uint32_t flags, bbc_result* out,
                           int32_t* status) {
    if (!c) return BBC_ERR_INVALID_ARG;
    begin_call(c);
    if (n_graphs < 0) return fail(c, BBC_ERR_INVALID_ARG, "n_graphs = %d", n_graphs);
    if (n_graphs == 0) return BBC_OK;
    if (!n_u || !n_v || !edge_offset || !out || !status)
        return fail(c, BBC_ERR_INVALID_ARG, "NULL size, offset or output array");
    if (flags & ~(uint32_t)BBC_INPUT_ON_DEVICE)
        return fail(c, BBC_ERR_INVALID_ARG, "unsupported flag bits 0x%x for a batch", flags);
    if (edge_offset[0] < 0) return fail(c, BBC_ERR_INVALID_ARG, "edge_offset[0] < 0");
    for (int32_t g = 0; g < n_graphs; ++g)
        if (edge_offset[g + 1] < edge_offset[g])
            return fail(c, BBC_ERR_INVALID_ARG, "edge_offset decreases at graph %d", g);
    if (edge_offset[n_graphs] > edge_offset[0] && (!edge_u || !edge_v || !edge_sign))
        return fail(c, BBC_ERR_INVALID_ARG, "NULL edge array");
    HIPCHECK(c, hipSetDevice(c->device));
    const bool on_device = (flags & BBC_INPUT_ON_DEVICE) != 0;
    // classify: empty / invalid sizes are settled here, large graphs run alone,
    // the rest go into unions of bounded size
    std::vector<uint32_t> small, big;
    for (int32_t g = 0; g < n_graphs; ++g) {
        out[g].balanced = out[g].unbalanced = out[g].wedges = 0;
        status[g] = BBC_OK;
        const int64_t mg = edge_offset[g + 1] - edge_offset[g];
        if (n_u[g] < 0 || n_v[g] < 0)
            status[g] = BBC_ERR_INVALID_ARG;
        else if ((uint64_t)n_u[g] + (uint64_t)n_v[g] >= (1ull << 30) || mg >= (1ll << 31))
            status[g] = BBC_ERR_TOO_LARGE;
        else if (mg == 0)
            continue;
        else if ((uint32_t)n_u[g] > kBatchSide || (uint32_t)n_v[g] > kBatchSide)
            big.push_back((uint32_t)g);
        else
            small.push_back((uint32_t)g);
    }
    int64_t stats[14] = {0};
    double ph[kNumPhases] = {0, 0, 0, 0, 0};
    auto keep_stats = [&]() {
        for (int i = 0; i < 14; ++i) stats[i] += c->stats[i];
        for (int i = 0; i < kNumPhases; ++i) ph[i] += c->phase_ms[i];
    };
    // unions: consecutive small graphs up to the size limits
    size_t i = 0;
    while (i < small.size()) {
        std::vector<uint32_t> gl;
        uint64_t me = 0, nn = 0;
        for (; i < small.size(); ++i) {
            const uint32_t g = small[i];
            const uint64_t mg = (uint64_t)(edge_offset[g + 1] - edge_offset[g]);
            const uint64_t ng = (uint64_t)n_u[g] + (uint64_t)n_v[g];
            if (!gl.empty() && (me + mg > c->union_edges || nn + ng > kBatchMaxVertices ||
                                gl.size() >= kBatchMaxGraphs))
                break;
            gl.push_back(g);
            me += mg;
            nn += ng;
        }
        memset(c->stats, 0, sizeof(c->stats));
        for (double& p : c->phase_ms) p = 0;
        bbc_status s = count_union(c, gl, n_u, n_v, edge_offset, edge_u, edge_v, edge_sign, on_device,
                                   out, status);
        if (s) return s;
        keep_stats();
    }
    // large graphs, one by one
    for (uint32_t g : big) {
        const int64_t e0 = edge_offset[g];
        bbc_result r;
        bbc_status s = bbc_count(c, n_u[g], n_v[g], edge_offset[g + 1] - e0, edge_u + e0,
                                 edge_v + e0, edge_sign + e0, flags, &r, nullptr);
        if (s == BBC_ERR_DEVICE || s == BBC_ERR_INTERNAL) return s;
        status[g] = s;
        if (s == BBC_OK) {
            out[g] = r;
            keep_stats();
        }
    }
    memcpy(c->stats, stats, sizeof(stats));
    for (int k = 0; k < kNumPhases; ++k) c->phase_ms[k] = ph[k];
    c->timing_valid = c->timing;
    c->err[0] = 0;
    return BBC_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Autotuner: coordinate search over the work-split tunables on the caller's
// own input, timing whole calls.

namespace {
struct TuneInput {
    int32_t n_graphs;
    const int32_t *n_u, *n_v;
    const int64_t* off;
    const int32_t *eu, *ev;
    const int8_t* sg;
    uint32_t flags;
};

// One timed call; *sum receives a checksum of every count (balanced,
// unbalanced, W of every graph) so that all settings can be compared.
bbc_status tune_call(bbc_context* c, const TuneInput& in, std::vector<bbc_result>& res,
                     std::vector<int32_t>& st, double* ms) {
    const auto t0 = std::chrono::steady_clock::now();
    bbc_status s;
    if (in.n_graphs == 1) {
        st[0] = BBC_OK;
        s = bbc_count(c, in.n_u[0], in.n_v[0], in.off[1] - in.off[0], in.eu + in.off[0],
                      in.ev + in.off[0], in.sg + in.off[0], in.flags, &res[0], nullptr);
    } else {
        s = bbc_count_batch(c, in.n_graphs, in.n_u, in.n_v, in.off, in.eu, in.ev, in.sg, in.flags,
                            res.data(), st.data());
    }
    *ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    return s;
}
}  // namespace

extern "C" {

bbc_status bbc_autotune(bbc_context* c, int32_t n_graphs, const int32_t* n_u, const int32_t* n_v,
                        const int64_t* edge_offset, const int32_t* edge_u, const int32_t* edge_v,
                        const int8_t* edge_sign, uint32_t flags, int32_t repeats,
                        int64_t* chosen, double* best_ms) {
    if (!c) return BBC_ERR_INVALID_ARG;
    if (n_graphs < 1 || !n_u || !n_v || !edge_offset || repeats < 1 || repeats > 100)
        return fail(c, BBC_ERR_INVALID_ARG, "autotune: bad sizes or repeats");
    if (flags & ~(uint32_t)BBC_INPUT_ON_DEVICE)
        return fail(c, BBC_ERR_INVALID_ARG, "autotune: unsupported flags 0x%x", flags);
    TuneInput in{n_graphs, n_u, n_v, edge_offset, edge_u, edge_v, edge_sign, flags};
    std::vector<bbc_result> res((size_t)n_graphs), ref((size_t)n_graphs);
    std::vector<int32_t> st((size_t)n_graphs), ref_st((size_t)n_graphs);
    // Every tunable, in the order of chosen[].  Which ones are searched depends
    // on the input: only graphs with more than 16384 vertices on a side cut
    // starts into end-vertex tiles, so only they make the hash target and the
    // probe limit matter; only a batch is split into unions.
    constexpr int kN = 6;
    const int pids[kN] = {BBC_PARAM_CHUNK_WEDGES, BBC_PARAM_HASH_TARGET, BBC_PARAM_PROBE_LIMIT,
                          BBC_PARAM_LIGHT_MAX, BBC_PARAM_GRAB_DIV, BBC_PARAM_UNION_EDGES};
    const bool batch = n_graphs > 1;
    bool tiles = !batch;  // some graph is counted alone (more than 16384 vertices on a side)
    for (int32_t g = 0; g < n_graphs && !tiles; ++g)
        tiles = (uint32_t)std::max(n_u[g], n_v[g]) > kBatchSide;
    const std::vector<int64_t> grid[kN] = {
        {16384, 65536, 262144, 1048576, 4194304},
        tiles ? std::vector<int64_t>{1024, 2048, 4096, 8192} : std::vector<int64_t>{},
        tiles ? std::vector<int64_t>{32, 256, 2048} : std::vector<int64_t>{},
        {512, 1024, 2048},
        {8, 16, 32},
        batch ? std::vector<int64_t>{1 << 24, 1 << 26, 1 << 28, 1 << 30} : std::vector<int64_t>{}};
    int64_t cur[kN];
    for (int k = 0; k < kN; ++k) bbc_get_param(c, pids[k], &cur[k]);
    int64_t saved[kN];
    for (int k = 0; k < kN; ++k) saved[k] = cur[k];
    auto restore = [&]() {
        for (int k = 0; k < kN; ++k) bbc_set_param(c, pids[k], saved[k]);
    };
    // reference counts and a warm workspace at the current settings
    double ms = 0;
    bbc_status s = tune_call(c, in, ref, ref_st, &ms);
    if (s) return s;
    auto timed = [&](double* best) -> bbc_status {
        *best = 1e300;
        for (int r = 0; r < repeats; ++r) {
            double t = 0;
            bbc_status e = tune_call(c, in, res, st, &t);
            if (e) return e;
            for (int32_t g = 0; g < n_graphs; ++g)
                if (st[g] != ref_st[g] || res[g].balanced != ref[g].balanced ||
                    res[g].unbalanced != ref[g].unbalanced || res[g].wedges != ref[g].wedges)
                    return fail(c, BBC_ERR_INTERNAL, "autotune: graph %d counted differently", g);
            *best = std::min(*best, t);
        }
        return BBC_OK;
    };
    double best = 0;
    s = timed(&best);
    if (s) {
        restore();
        return s;
    }
    for (int k = 0; k < kN; ++k) {
        int64_t keep = cur[k];
        for (int64_t v : grid[k]) {
            if (v == keep) continue;
            if (bbc_set_param(c, pids[k], v) != BBC_OK) continue;
            double t = 0;
            s = timed(&t);
            if (s) {
                restore();
                return s;
            }
            if (t < best * 0.97) {  // a clear gain only
                best = t;
                keep = v;
            }
        }
        cur[k] = keep;
        bbc_set_param(c, pids[k], keep);
    }
    if (chosen)
        for (int k = 0; k < kN; ++k) chosen[k] = cur[k];
    if (best_ms) *best_ms = best;
    return BBC_OK;
}

}  // extern "C"

