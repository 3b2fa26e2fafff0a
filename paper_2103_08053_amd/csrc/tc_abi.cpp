// C-ABI of the triangle-counting library: contexts, parameters, workspace
// layout and the orchestration of the device steps.  See trust_tc.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdarg>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "tc_internal.h"

// Count scratch of tc_graph_count_static: a library-owned buffer in every device's memory, so that
// entry point allocates nothing.  In host code `scratch` names a host-side stand-in, not a device
// address; the device address comes from hipGetSymbolAddress, taken once per device (static_scratch).
static __device__ __align__(256) unsigned char scratch[TC_STATIC_SCRATCH_BYTES];

struct tc_context {
    int device = 0;
    int cu_count = 0;
    size_t lds_per_block_max = 0;
    uint32_t big_lds_bytes = 0;  // dynamic LDS of the large-vertex kernel: all a workgroup may have
    uint32_t mid_lds_bytes = 0;  // the same kernel with two workgroups per CU: half a CU's LDS (0: unknown)
    tc_params p{};
    std::string err;
    bool timing = false;
    hipEvent_t ev[4] = {nullptr, nullptr, nullptr, nullptr};  // build start/end, count start/end
    bool have_build = false, have_count = false;
    hipStream_t capture_stream = nullptr;  // for tc_graph_count_replay and tc_count_graphs_replay
    struct Occ {
        uint32_t hub, sw, mu, S, pv, hk, threads, lds;
        int per_cu;
    };
    // tc_count_graphs: pinned host staging of the header and descriptors (a small ring, so an upload
    // still queued behind earlier work is never overwritten), and launch sequences captured per
    // (workspace, per-vertex mode, knobs).
    struct Stage {
        void* host = nullptr;
        size_t bytes = 0;
        hipEvent_t ev = nullptr;
        bool pending = false;
    };
    Stage stage[4];
    uint32_t stage_next = 0;
    struct MultiCapture {
        const void* ws;
        bool pv;
        tc_params p;
        hipGraph_t hg;
        hipGraphExec_t exec;
    };
    std::vector<MultiCapture> mcap;
    void* static_scratch = nullptr;  // this device's copy of the library-owned count scratch
    std::vector<Occ> occ;  // resident workgroups per CU, by kernel variant and launch shape
};

namespace {

// Device address of `scratch` on each device, resolved with that device current the first time a
// context is created on it (nullptr until then).
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mutex;
void* g_scratch_ptr[kMaxDevices] = {};

hipError_t static_scratch(int device, void** out) {
    if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_scratch_mutex);
    if (!g_scratch_ptr[device]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (!p) return hipErrorInvalidSymbol;
        g_scratch_ptr[device] = p;
    }
    *out = g_scratch_ptr[device];
    return hipSuccess;
}

}  // namespace

struct tc_graph {
    tc_context* ctx = nullptr;
    uint32_t n = 0;
    uint64_t m_in = 0;
    uint32_t k = 1;          // graphs in the batch (1 for a single graph)
    bool batch = false;
    tc_params p{};           // knobs the bins were sized with
    tc::BinCaps caps{};
    tc::GraphDev dev{};
    bool empty = false;      // n == 0 or m_in == 0: nothing on the device
    // captured count (tc_graph_count_replay)
    hipGraph_t hg = nullptr;
    hipGraphExec_t exec = nullptr;
    const void* key[3] = {nullptr, nullptr, nullptr};
};

namespace {

using tc::Layout;

constexpr size_t kAlign = 256;
constexpr size_t align_up(size_t x) { return (x + kAlign - 1) & ~(kAlign - 1); }

// The count scratch is used from the first 64 KB boundary in the caller's buffer (the layout reserves
// the slack).  With the per-vertex staging starting 256 B to 8 KB past a 2 MB boundary the per-vertex
// count at R-MAT scale 22 measured 18.2-18.3 ms against 17.25-17.4 ms from the boundary itself or
// 12 KB and more past it.
constexpr size_t kScratchAlign = 65536;
inline char* scratch_base(void* p) {
    return reinterpret_cast<char*>((reinterpret_cast<uintptr_t>(p) + kScratchAlign - 1) & ~(uintptr_t)(kScratchAlign - 1));
}

tc_status fail(tc_context* c, tc_status s, const char* fmt, ...) __attribute__((format(printf, 3, 4)));
tc_status fail(tc_context* c, tc_status s, const char* fmt, ...) {
    if (c) {
        char buf[512];
        va_list ap;
        va_start(ap, fmt);
        vsnprintf(buf, sizeof(buf), fmt, ap);
        va_end(ap);
        c->err = buf;
    }
    return s;
}

tc_status hip_fail(tc_context* c, hipError_t e, const char* where) {
    return fail(c, TC_E_DEVICE, "%s: %s", where, hipGetErrorString(e));
}

#define HIP_TRY(ctx, expr)                                     \
    do {                                                       \
        hipError_t e_ = (expr);                                \
        if (e_ != hipSuccess) return hip_fail(ctx, e_, #expr); \
    } while (0)

constexpr uint32_t kIntraFlags = TC_F_SUBWAVE_8 | TC_F_SUBWAVE_16 | TC_F_SUBWAVE_32 | TC_F_WAVE_LIST;

uint32_t subwave_lanes(uint32_t flags) {
    if (flags & TC_F_SUBWAVE_8) return 8;
    if (flags & TC_F_SUBWAVE_16) return 16;
    if (flags & TC_F_SUBWAVE_32) return 32;
    if (flags & TC_F_WAVE_LIST) return 64;
    return 0;
}

tc_status check_params(const tc_params* p) {
    if (!p || p->struct_size != sizeof(tc_params)) return TC_E_INVALID;
    if (p->wg_waves < 1 || p->wg_waves > tc::kMaxWaves) return TC_E_INVALID;
    if (p->wg_lds_bytes < 4096 || p->wg_lds_bytes > 131072 || p->wg_lds_bytes % 16) return TC_E_INVALID;
    // every wavefront keeps a probe queue in the LDS and a slice of at least 64 words
    if (p->wg_lds_bytes / 4 < p->wg_waves * (tc::kQueueWords + 64)) return TC_E_INVALID;
    if (p->slots_per_bucket != 1 && p->slots_per_bucket != 2 && p->slots_per_bucket != 4) return TC_E_INVALID;
    if (p->load_factor_pct < 10 || p->load_factor_pct > 100) return TC_E_INVALID;
    if (p->hash_kind > 1) return TC_E_INVALID;
    if (p->light_chunk < 1 || p->light_chunk > 256) return TC_E_INVALID;
    if (p->flags & ~(TC_F_NO_LPT | TC_F_FORCE_WG | TC_F_FORCE_HUB | TC_F_SCATTER_CSR | TC_F_WIDE_ADDR |
                     TC_F_FORCE_BIG | TC_F_ORDER_INDEGREE | TC_F_ORDER_COLLECTIVE | kIntraFlags | TC_F_NO_PACK |
                     TC_F_NO_MID | TC_F_RECORDS))
        return TC_E_INVALID;
    if (__builtin_popcount(p->flags & kIntraFlags) > 1) return TC_E_INVALID;
    if ((p->flags & TC_F_ORDER_INDEGREE) && (p->flags & TC_F_ORDER_COLLECTIVE)) return TC_E_INVALID;
    return TC_OK;
}

// LDS of the main launch.  While its workgroups take workgroup-bin vertices, the table region is
// the LDS minus the wavefronts' probe queues at its end; afterwards every wavefront owns a region
// of its own (1/wg_waves of the LDS): a table slice followed by its probe queue, or four
// packed-vertex tables (which need no queue).
uint32_t wg_table_words(const tc_params& p) { return p.wg_lds_bytes / 4 - p.wg_waves * tc::kQueueWords; }

// A wavefront's region, and the table slice at its start.
uint32_t wave_region_words(const tc_params& p) { return (p.wg_lds_bytes / 4 / p.wg_waves) & ~3u; }
uint32_t slice_words(const tc_params& p) { return wave_region_words(p) - tc::kQueueWords; }

// Table region of the large-vertex launch (16 wavefronts, all the LDS a workgroup may have), and of
// its half-LDS launch (two such workgroups per CU).
uint32_t big_table_words(const tc_context* ctx) { return ctx->big_lds_bytes / 4 - tc::kMaxWaves * tc::kQueueWords; }
uint32_t mid_table_words(const tc_context* ctx) {
    const uint32_t q = tc::kMidWaves * tc::kQueueWords;
    return ctx->mid_lds_bytes / 4 > q ? ctx->mid_lds_bytes / 4 - q : 0u;
}

// LDS words of a packed light vertex's table: a quarter of a wavefront slice.
uint32_t pack_region(const tc_params& p) { return (wave_region_words(p) / 4) & ~3u; }

tc::BinCaps bin_caps(const tc_context* ctx, const tc_params& p) {
    tc::BinCaps c{};
    // Capacities assume the per-vertex layout (the larger one), so one binning serves both modes,
    // and the filter of the LDS tables walked by virtual combination (not in the subwave modes).
    const bool filt = subwave_lanes(p.flags) == 0;
    c.wg_cap = tc::capacity(wg_table_words(p), p.slots_per_bucket, p.load_factor_pct, true, filt);
    c.wave_cap = tc::capacity(slice_words(p), p.slots_per_bucket, p.load_factor_pct, true, filt);
    if (p.wave_max_dplus && p.wave_max_dplus < c.wave_cap) c.wave_cap = p.wave_max_dplus;
    c.big_cap = tc::capacity(big_table_words(ctx), p.slots_per_bucket, p.load_factor_pct, true, true);
    if (c.big_cap < c.wg_cap) c.big_cap = c.wg_cap;
    // Half-LDS part of bin 1: out-degrees above the workgroup bin whose tables fit half a CU's LDS
    // (not when a forced bin asks for the full-LDS path).
    c.mid_cap = 0;
    if (!(p.flags & (TC_F_NO_MID | TC_F_FORCE_BIG | TC_F_FORCE_HUB | TC_F_FORCE_WG)) && mid_table_words(ctx)) {
        const uint32_t mc = tc::capacity(mid_table_words(ctx), p.slots_per_bucket, p.load_factor_pct, true, true);
        if (mc > c.wg_cap && mc < c.big_cap) c.mid_cap = mc;
    }
    c.force_wg = (p.flags & TC_F_FORCE_WG) != 0;
    c.force_hub = (p.flags & TC_F_FORCE_HUB) != 0;
    c.force_big = (p.flags & TC_F_FORCE_BIG) != 0;
    // Packed bin: out-degree up to 32 whose minimal table fits a quarter slice (subwave modes and
    // TC_F_NO_PACK keep one wavefront per vertex).
    c.pack_cap = 0;
    if (!(p.flags & (TC_F_NO_PACK | kIntraFlags))) {
        c.pack_cap = std::min<uint32_t>({tc::kPackMaxD, c.wave_cap,
                                         tc::capacity(pack_region(p), p.slots_per_bucket, p.load_factor_pct, true)});
        if (c.pack_cap < 2) c.pack_cap = 0;
    }
    c.lpt = (p.flags & TC_F_NO_LPT) == 0;
    c.scatter_csr = (p.flags & TC_F_SCATTER_CSR) != 0;
    c.order = (p.flags & TC_F_ORDER_INDEGREE) ? 1u : (p.flags & TC_F_ORDER_COLLECTIVE) ? 2u : 0u;
    return c;
}

// Out-degree bound after (degree, id) orientation: every out-neighbour of u
// has degree >= deg(u) >= d+(u), so d+(u)^2 <= 2m, and d+(u) < n.
uint32_t dplus_bound(uint32_t n, uint64_t m_in) {
    uint64_t b = (uint64_t)std::sqrt(2.0 * (double)m_in) + 2;
    if (b > n) b = n;
    if (b > m_in) b = m_in;
    return (uint32_t)b;
}

// Whether a graph of n vertices and m_in samples built with p gets the record layout: asked for, a
// build that sorts the oriented edges in rank order, and record positions and list starts below 2^31.
bool records_on(const tc_params& p, uint32_t n, uint64_t m_in) {
    return (p.flags & TC_F_RECORDS) &&
           !(p.flags & (TC_F_ORDER_INDEGREE | TC_F_ORDER_COLLECTIVE | TC_F_SCATTER_CSR)) &&
           tc::record_words(n, m_in) < (1ull << 31);
}

Layout layout(const tc_context* ctx, const tc_params& p, uint32_t n, uint64_t m_in, bool batch = false) {
    Layout L{};
    L.records = records_on(p, n, m_in);
    size_t o = 0;
    L.s_meta = o;  o = align_up(o + sizeof(tc::GraphMeta));
    L.s_off = o;   o = align_up(o + sizeof(int64_t) * ((size_t)n + 1));
    L.s_off32 = o; o = align_up(o + sizeof(uint32_t) * ((size_t)n + 1));
    L.s_col = o;   o = align_up(o + sizeof(uint32_t) * (size_t)m_in);
    L.s_rank = o;  o = align_up(o + sizeof(uint32_t) * (size_t)n);
    L.s_items = o; o = align_up(o + sizeof(uint32_t) * (size_t)n);
    L.s_gid = o;   o = align_up(o + (batch ? sizeof(uint32_t) * (size_t)n : 0));
    L.s_rec = o;   o = align_up(o + (L.records ? sizeof(uint32_t) * tc::record_words(n, m_in) : 0));
    L.s_place = o; o = align_up(o + (L.records ? 8 * ((size_t)n + 1) : 0));
    L.storage = o;

    o = 0;
    L.t_keys_a = o; o = align_up(o + 8 * (size_t)m_in);
    L.t_keys_b = o; o = align_up(o + 8 * (size_t)m_in);
    L.t_aux = o;    o = align_up(o + 8 * (size_t)m_in);
    L.t_deg = o;    o = align_up(o + 4 * ((size_t)n + 1));
    L.t_dplus = o;  o = align_up(o + 4 * ((size_t)n + 1));
    L.t_order = o;  o = align_up(o + 4 * (size_t)n);
    L.t_skey_a = o; o = align_up(o + 8 * (size_t)n);
    L.t_skey_b = o; o = align_up(o + 8 * (size_t)n);
    const bool relabel = (p.flags & (TC_F_ORDER_INDEGREE | TC_F_ORDER_COLLECTIVE)) != 0;
    L.relabel = relabel;
    L.t_rk_a = o;   o = align_up(o + (relabel ? 8 * (size_t)n : 0));
    L.t_rk_b = o;   o = align_up(o + (relabel ? 8 * (size_t)n : 0));
    L.t_off2 = o;   o = align_up(o + (relabel ? 8 * ((size_t)n + 1) : 0));
    L.t_place = o;  o = align_up(o + (L.records ? 16 * (tc::place_chunks(n) + 1) : 0));
    L.sort_tmp_bytes = align_up(tc::prep_sort_tmp_bytes(n, m_in));
    L.t_sort = o;   o = align_up(o + L.sort_tmp_bytes);
    L.temp = o;

    // Count scratch: per-vertex staging, global-memory tables, then the total and the queue heads.
    // The heads are the launch's hottest atomics; at the start of a 2 MB-aligned buffer (where a
    // separately allocated scratch begins) the per-vertex count at R-MAT scale 22 measured 18.8 ms
    // against 17.3-17.9 ms anywhere past its first 8 KB, so they go last.
    o = 0;
    // (record layout: the per-vertex counts are kept by record id)
    L.c_tv = o;     o = align_up(o + 8 * (L.records ? tc::record_words(n, m_in) : (size_t)n));
    const uint32_t dmax = dplus_bound(n, m_in);
    L.hub_words = tc::geometry(dmax, p.slots_per_bucket, tc::load_recip(p.load_factor_pct), true).words;
    uint32_t grid = p.grid_wgs ? p.grid_wgs : (uint32_t)std::max(1, ctx ? ctx->cu_count : 1);
    L.hub_wgs = std::min<uint32_t>(tc::kHubWgs, std::max<uint32_t>(1, grid));
    L.c_hub = o;    o = align_up(o + 4 * L.hub_words * L.hub_wgs);
    L.c_total = o;  o = align_up(o + 8);
    L.c_heads = o;  o = align_up(o + 4 * tc::kHeadWords);
    L.scratch = o + kScratchAlign;  // used from the first 64 KB boundary (scratch_base)
    return L;
}

tc::GraphDev graph_ptrs(void* storage, const Layout& L) {
    char* b = static_cast<char*>(storage);
    tc::GraphDev g;
    g.meta = reinterpret_cast<tc::GraphMeta*>(b + L.s_meta);
    g.off = reinterpret_cast<int64_t*>(b + L.s_off);
    g.off32 = reinterpret_cast<uint32_t*>(b + L.s_off32);
    g.col = reinterpret_cast<uint32_t*>(b + L.s_col);
    g.rank = reinterpret_cast<uint32_t*>(b + L.s_rank);
    g.items = reinterpret_cast<uint32_t*>(b + L.s_items);
    g.gid = nullptr;
    g.rec = L.records ? reinterpret_cast<uint32_t*>(b + L.s_rec) : nullptr;
    g.place = L.records ? reinterpret_cast<uint32_t*>(b + L.s_place) : nullptr;
    return g;
}

tc::BuildTemp temp_ptrs(void* temp, const Layout& L) {
    char* b = static_cast<char*>(temp);
    tc::BuildTemp t;
    t.keys_a = reinterpret_cast<unsigned long long*>(b + L.t_keys_a);
    t.keys_b = reinterpret_cast<unsigned long long*>(b + L.t_keys_b);
    t.aux = reinterpret_cast<uint32_t*>(b + L.t_aux);
    t.deg = reinterpret_cast<uint32_t*>(b + L.t_deg);
    t.dplus = reinterpret_cast<uint32_t*>(b + L.t_dplus);
    t.order = reinterpret_cast<uint32_t*>(b + L.t_order);
    t.skey_a = reinterpret_cast<unsigned long long*>(b + L.t_skey_a);
    t.skey_b = reinterpret_cast<unsigned long long*>(b + L.t_skey_b);
    const bool relabel = L.relabel;
    t.rk_a = relabel ? reinterpret_cast<unsigned long long*>(b + L.t_rk_a) : nullptr;
    t.rk_b = relabel ? reinterpret_cast<unsigned long long*>(b + L.t_rk_b) : nullptr;
    t.off2 = relabel ? reinterpret_cast<int64_t*>(b + L.t_off2) : nullptr;
    t.place_sz = L.records ? reinterpret_cast<unsigned long long*>(b + L.t_place) : nullptr;
    t.sort_tmp = b + L.t_sort;
    t.sort_tmp_bytes = L.sort_tmp_bytes;
    return t;
}

tc_status check_sizes(tc_context* ctx, uint64_t m_in) {
    if (m_in >= (1ull << 31)) return fail(ctx, TC_E_UNSUPPORTED, "m_in = %llu exceeds 2^31 - 1", (unsigned long long)m_in);
    return TC_OK;
}

tc_status use_device(tc_context* ctx) {
    HIP_TRY(ctx, hipSetDevice(ctx->device));
    return TC_OK;
}

tc_status build_into(tc_context* ctx, tc_graph* g, uint32_t n, uint64_t m_in, const uint32_t* src,
                     const uint32_t* dst, void* storage, void* temp, const Layout& L, hipStream_t s,
                     const tc::BatchIn* batch = nullptr) {
    g->ctx = ctx;
    g->n = n;
    g->m_in = m_in;
    g->batch = batch != nullptr;
    g->k = batch ? batch->k : 1;
    g->p = ctx->p;
    g->caps = bin_caps(ctx, ctx->p);
    g->caps.records = L.records;
    g->empty = (n == 0 || m_in == 0);
    if (g->empty) {
        g->dev = tc::GraphDev{};
        if (storage) {
            g->dev = graph_ptrs(storage, L);
            HIP_TRY(ctx, tc::fill_u32(g->dev.meta, 0, sizeof(tc::GraphMeta) / 4, s));
            HIP_TRY(ctx, tc::fill_u32(g->dev.off, 0, 2 * ((size_t)n + 1), s));
            HIP_TRY(ctx, tc::fill_u32(g->dev.rank, 0, n, s));
        }
        return TC_OK;
    }
    g->dev = graph_ptrs(storage, L);
    if (batch) g->dev.gid = reinterpret_cast<uint32_t*>(static_cast<char*>(storage) + L.s_gid);
    if (ctx->timing) HIP_TRY(ctx, hipEventRecord(ctx->ev[0], s));
    HIP_TRY(ctx, tc::prep_build(n, m_in, src, dst, g->dev, temp_ptrs(temp, L), g->caps, batch, s));
    if (ctx->timing) {
        HIP_TRY(ctx, hipEventRecord(ctx->ev[1], s));
        ctx->have_build = true;
    }
    return TC_OK;
}

// Launch shape of the main kernel (workgroups of wg_waves wavefronts, wg_lds_bytes of LDS) or of the
// large-vertex kernel (16 wavefronts, all the LDS a workgroup may have).
uint32_t launch_threads(const tc_params& p, bool hub) { return hub ? 64 * tc::kMaxWaves : 64 * p.wg_waves; }
uint32_t launch_lds(const tc_context* ctx, const tc_params& p, bool hub) {
    return hub ? ctx->big_lds_bytes : p.wg_lds_bytes;
}

tc_status occupancy(tc_context* ctx, const tc_params& p, bool pv, bool hub, int* per_cu, bool multi = false,
                    uint32_t lds_bytes = 0, uint32_t threads_override = 0) {
    const uint32_t threads = threads_override ? threads_override : launch_threads(p, hub);
    const uint32_t lds = lds_bytes ? lds_bytes : launch_lds(ctx, p, hub);
    const uint32_t sw = (!hub && !multi && subwave_lanes(p.flags)) ? 1u : 0u;
    const uint32_t mu = multi ? 1u : 0u;
    for (const auto& o : ctx->occ)
        if (o.hub == (uint32_t)hub && o.sw == sw && o.mu == mu && o.S == p.slots_per_bucket &&
            o.pv == (uint32_t)pv && o.hk == p.hash_kind && o.threads == threads && o.lds == lds) {
            *per_cu = o.per_cu;
            return TC_OK;
        }
    int q = 0;
    if (multi)
        HIP_TRY(ctx, tc::count_kernel_info_multi(hub, p.slots_per_bucket, pv, p.hash_kind, threads, lds, &q));
    else
        HIP_TRY(ctx, tc::count_kernel_info(hub, sw != 0, p.slots_per_bucket, pv, p.hash_kind, threads, lds, &q));
    // The query sets the kernel's dynamic-LDS limit to the size asked about; the large-vertex kernel
    // keeps the full-LDS limit, which its full-LDS launch needs (the half-LDS launch needs less).
    if (hub && lds < ctx->big_lds_bytes) {
        int q2 = 0;
        if (multi)
            HIP_TRY(ctx, tc::count_kernel_info_multi(true, p.slots_per_bucket, pv, p.hash_kind, threads,
                                                     ctx->big_lds_bytes, &q2));
        else
            HIP_TRY(ctx, tc::count_kernel_info(true, false, p.slots_per_bucket, pv, p.hash_kind, threads,
                                               ctx->big_lds_bytes, &q2));
    }
    if (q < 1) return fail(ctx, TC_E_INVALID, "kernel does not fit: %u threads, %u LDS bytes", threads, lds);
    ctx->occ.push_back({(uint32_t)hub, sw, mu, p.slots_per_bucket, (uint32_t)pv, p.hash_kind, threads, lds, q});
    *per_cu = q;
    return TC_OK;
}

// Whether any vertex can land in bins 0 or 1 (those need the large-vertex launch).
bool needs_hub_launch(const tc_graph* g) {
    return g->caps.force_hub || g->caps.force_big || dplus_bound(g->n, g->m_in) > g->caps.wg_cap;
}

// The count: clears, the persistent kernel and (per-vertex mode) the gather.
// d_totals has g->k entries.  With `record` false no timing events are recorded (stream capture).
tc_status count_into(tc_context* ctx, const tc_graph* g, uint64_t* d_totals, uint64_t* d_per_vertex, void* d_scr,
                     const Layout& L, hipStream_t s, bool record = true, uint32_t shard = 0, uint32_t shards = 1) {
    const tc_params& p = g->p;
    const bool pv = d_per_vertex != nullptr;
    char* b = scratch_base(d_scr);
    if (g->empty) {
        HIP_TRY(ctx, tc::fill_u32(d_totals, 0, 2 * (size_t)g->k, s));
        if (pv) HIP_TRY(ctx, tc::fill_u32(d_per_vertex, 0, 2 * (size_t)g->n, s));
        return TC_OK;
    }
    tc::CountArgs a{};
    a.meta = g->dev.meta;
    a.off = g->dev.off32;
    a.col = g->dev.col;
    a.items = g->dev.items;
    a.heads = reinterpret_cast<uint32_t*>(b + L.c_heads);
    a.gid = g->dev.gid;
    a.total = g->dev.gid ? nullptr : reinterpret_cast<unsigned long long*>(d_totals);
    a.totals = g->dev.gid ? reinterpret_cast<unsigned long long*>(d_totals) : nullptr;
    a.tv = pv ? reinterpret_cast<unsigned long long*>(b + L.c_tv) : nullptr;
    a.hub_scratch = reinterpret_cast<uint32_t*>(b + L.c_hub);
    a.hub_words = L.hub_words;
    a.hub_wgs = L.hub_wgs;
    a.slice_words = slice_words(p);
    a.lrecip = tc::load_recip(p.load_factor_pct);
    a.chunk = p.light_chunk;
    a.wide = tc::wide_list_addressing(g->m_in, (p.flags & TC_F_WIDE_ADDR) != 0) ? 1u : 0u;
    // Record layout: lists are read through the records, and ids (tables, tallies) are record ids.
    const size_t tv_words = g->dev.rec ? tc::record_words(g->n, g->m_in) : (size_t)g->n;
    if (g->dev.rec) {
        a.rec = g->dev.rec;
        a.col = g->dev.rec;
        a.place = g->dev.place;
        a.wide = tc::wide_list_addressing(tv_words, (p.flags & TC_F_WIDE_ADDR) != 0) ? 1u : 0u;
    }
    a.shard = shard;
    a.shards = shards;
    a.subwave = subwave_lanes(p.flags);
    a.pack_region = pack_region(p);
    const bool hub = needs_hub_launch(g);
    int per_cu = 0, per_cu_hub = 0, per_cu_mid = 0;
    if (tc_status st = occupancy(ctx, p, pv, false, &per_cu)) return st;
    if (hub)
        if (tc_status st = occupancy(ctx, p, pv, true, &per_cu_hub)) return st;
    if (hub && g->caps.mid_cap)
        if (tc_status st = occupancy(ctx, p, pv, true, &per_cu_mid, false, ctx->mid_lds_bytes, 64 * tc::kMidWaves))
            return st;
    const uint32_t grid = p.grid_wgs ? p.grid_wgs : (uint32_t)(per_cu * ctx->cu_count);
    const uint32_t grid_hub = p.grid_wgs ? p.grid_wgs : (uint32_t)(per_cu_hub * ctx->cu_count);
    const uint32_t grid_mid = p.grid_wgs ? p.grid_wgs : (uint32_t)(per_cu_mid * ctx->cu_count);
    if (grid_hub < a.hub_wgs) a.hub_wgs = grid_hub;
    HIP_TRY(ctx, tc::fill_u32(a.heads, 0, tc::kHeadWords, s));
    HIP_TRY(ctx, tc::fill_u32(d_totals, 0, 2 * (size_t)g->k, s));
    if (pv) {
        if (g->dev.rec) HIP_TRY(ctx, tc::clear_record_staging(a.tv, g->dev.place, g->n, s));
        else HIP_TRY(ctx, tc::fill_u32(a.tv, 0, 2 * tv_words, s));
    }
    const bool rec = record && ctx->timing;
    if (rec) HIP_TRY(ctx, hipEventRecord(ctx->ev[2], s));
    if (hub) {
        a.table_words = big_table_words(ctx);
        a.hub_part = 0;
        HIP_TRY(ctx, tc::count_launch(true, false, p.slots_per_bucket, pv, p.hash_kind, grid_hub, launch_threads(p, true),
                                      launch_lds(ctx, p, true), a, s));
        if (g->caps.mid_cap) {
            a.table_words = mid_table_words(ctx);
            a.hub_part = 1;
            HIP_TRY(ctx, tc::count_launch(true, false, p.slots_per_bucket, pv, p.hash_kind, grid_mid,
                                          64 * tc::kMidWaves, ctx->mid_lds_bytes, a, s));
            a.hub_part = 0;
        }
    }
    a.table_words = wg_table_words(p);
    HIP_TRY(ctx, tc::count_launch(false, a.subwave != 0, p.slots_per_bucket, pv, p.hash_kind, grid,
                                  launch_threads(p, false),
                                  p.wg_lds_bytes, a, s));
    if (rec) {
        HIP_TRY(ctx, hipEventRecord(ctx->ev[3], s));
        ctx->have_count = true;
    }
    if (pv)
        HIP_TRY(ctx, tc::gather_per_vertex(a.tv, g->dev.rank, g->n, g->dev.rec ? g->dev.place : nullptr,
                                           reinterpret_cast<unsigned long long*>(d_per_vertex), s));
    return TC_OK;
}

tc_status count_one_shot(tc_context* ctx, uint32_t n, uint64_t m_in, const uint32_t* d_src, const uint32_t* d_dst,
                         uint64_t* d_per_vertex, void* d_ws, const Layout& L, hipStream_t st, uint64_t* h_total);

// ---------------------------------------------------------------- several built graphs, one launch sequence

// Workspace of a multi-graph count: header | (80 KB in) queue heads | descriptors | per-bin fetch prefixes |
// per-vertex staging | global-memory tables.  The header and the heads sit at fixed offsets (the
// kernels are given those two addresses; everything else is read from the header); every other
// region grows with (k, n_total, hub_words), so the sizes of any call within a query's bounds fit
// the query's answer.
// The workspace is used from its first 64 KB boundary (scratch_base); the heads sit 16 KB past the next
// one, so never within the first 8 KB of a 2 MB page, and the per-vertex staging on a 64 KB boundary
// (see the count scratch layout).
constexpr size_t kMultiHeads = 65536 + 16384;
struct MultiLayout {
    size_t desc, pre, tv, hub, bytes;
    uint32_t hub_wgs;
};

MultiLayout multi_layout(const tc_context* ctx, const tc_params& p, uint32_t k, uint64_t n_total, bool pv,
                         uint64_t hub_words) {
    MultiLayout M{};
    size_t o = align_up(kMultiHeads + 4 * (size_t)tc::kHeadWords);
    M.desc = o;  o = align_up(o + sizeof(tc::MultiDesc) * (size_t)k);
    M.pre = o;   o = align_up(o + 4 * (size_t)tc::kBins * ((size_t)k + 1));
    o = (o + kScratchAlign - 1) & ~(kScratchAlign - 1);
    M.tv = o;    o = align_up(o + (pv ? 8 * (size_t)n_total : 0));
    const uint32_t grid = p.grid_wgs ? p.grid_wgs : (uint32_t)std::max(1, ctx ? ctx->cu_count : 1);
    M.hub_wgs = std::min<uint32_t>(tc::kHubWgs, std::max<uint32_t>(1, grid));
    M.hub = o;   o = align_up(o + 4 * (size_t)hub_words * M.hub_wgs);
    M.bytes = o + kScratchAlign;  // used from the first 64 KB boundary (scratch_base)
    return M;
}

// Words of one global-memory table region for a graph of n vertices and m_in samples.
uint64_t hub_words_for(const tc_params& p, uint32_t n, uint64_t m_in) {
    if (n == 0 || m_in == 0) return 0;
    return tc::geometry(dplus_bound(n, m_in), p.slots_per_bucket, tc::load_recip(p.load_factor_pct), true).words;
}

// The launches of a multi-graph count (clears and prefixes, large-vertex kernel, main kernel,
// per-vertex gather), every size read from the header at hdr.  `record`: timing events (not while
// capturing).  Launch shapes come from occupancy queries resolved beforehand.
tc_status multi_launches(tc_context* ctx, const tc_params& p, bool pv, tc::MultiHeader* hdr, uint32_t hub_wgs,
                         hipStream_t s, bool record) {
    int per_cu = 0, per_cu_hub = 0;
    if (tc_status st = occupancy(ctx, p, pv, false, &per_cu, true)) return st;
    if (tc_status st = occupancy(ctx, p, pv, true, &per_cu_hub, true)) return st;
    const uint32_t grid = p.grid_wgs ? p.grid_wgs : (uint32_t)(per_cu * ctx->cu_count);
    const uint32_t grid_hub = p.grid_wgs ? p.grid_wgs : (uint32_t)(per_cu_hub * ctx->cu_count);
    tc::CountArgs a{};
    a.multi = hdr;
    a.heads = reinterpret_cast<uint32_t*>(reinterpret_cast<char*>(hdr) + kMultiHeads);
    a.slice_words = slice_words(p);
    a.lrecip = tc::load_recip(p.load_factor_pct);
    a.chunk = p.light_chunk;
    a.pack_region = pack_region(p);
    a.subwave = 0;
    a.shard = 0;
    a.shards = 1;
    a.hub_wgs = std::min(hub_wgs, grid_hub);
    HIP_TRY(ctx, tc::multi_prepare(hdr, ctx->cu_count, s));
    const bool rec = record && ctx->timing;
    if (rec) HIP_TRY(ctx, hipEventRecord(ctx->ev[2], s));
    a.table_words = big_table_words(ctx);
    HIP_TRY(ctx, tc::count_launch_multi(true, p.slots_per_bucket, pv, p.hash_kind, grid_hub, launch_threads(p, true),
                                        launch_lds(ctx, p, true), a, s));
    a.table_words = wg_table_words(p);
    HIP_TRY(ctx, tc::count_launch_multi(false, p.slots_per_bucket, pv, p.hash_kind, grid, launch_threads(p, false),
                                        p.wg_lds_bytes, a, s));
    if (rec) {
        HIP_TRY(ctx, hipEventRecord(ctx->ev[3], s));
        ctx->have_count = true;
    }
    if (pv) HIP_TRY(ctx, tc::multi_gather(hdr, ctx->cu_count, s));
    return TC_OK;
}

void drop_capture(tc_graph* g) {
    if (g->exec) (void)hipGraphExecDestroy(g->exec);
    if (g->hg) (void)hipGraphDestroy(g->hg);
    g->exec = nullptr;
    g->hg = nullptr;
}

}  // namespace

extern "C" {

const char* tc_status_str(tc_status s) {
    switch (s) {
        case TC_OK: return "ok";
        case TC_E_INVALID: return "invalid argument";
        case TC_E_RANGE: return "vertex id out of range";
        case TC_E_NOMEM: return "workspace too small";
        case TC_E_DEVICE: return "device error";
        case TC_E_UNSUPPORTED: return "unsupported size";
        case TC_E_BUSY: return "busy";
    }
    return "unknown status";
}

const char* tc_last_error(const tc_context* ctx) { return ctx ? ctx->err.c_str() : ""; }

tc_status tc_default_params(tc_params* p) {
    if (!p) return TC_E_INVALID;
    std::memset(p, 0, sizeof(*p));
    p->struct_size = sizeof(tc_params);
    p->wg_waves = 8;
    p->wg_lds_bytes = 49152;
    p->wave_max_dplus = 0;
    p->slots_per_bucket = 4;
    p->load_factor_pct = 50;
    p->hash_kind = 0;
    p->light_chunk = 16;
    p->grid_wgs = 0;
    p->flags = 0;
    return TC_OK;
}

tc_status tc_create(int hip_device, const tc_params* p, tc_context** out) {
    if (!out) return TC_E_INVALID;
    *out = nullptr;
    tc_params q;
    if (p) q = *p; else tc_default_params(&q);
    if (check_params(&q) != TC_OK) return TC_E_INVALID;
    int count = 0;
    if (hipGetDeviceCount(&count) != hipSuccess || count <= 0) return TC_E_DEVICE;
    if (hip_device < 0 || hip_device >= count) return TC_E_DEVICE;
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, hip_device) != hipSuccess) return TC_E_DEVICE;
    if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0) return TC_E_DEVICE;
    tc_context* c = new (std::nothrow) tc_context();
    if (!c) return TC_E_NOMEM;
    c->device = hip_device;
    c->cu_count = prop.multiProcessorCount;
    // LDS a workgroup may use: the opt-in limit (past 64 KB needs hipFuncSetAttribute), within one CU's LDS.
    c->lds_per_block_max = std::max(prop.sharedMemPerBlock, prop.sharedMemPerBlockOptin);
    if (prop.maxSharedMemoryPerMultiProcessor)
        c->lds_per_block_max = std::min(c->lds_per_block_max, prop.maxSharedMemoryPerMultiProcessor);
    {
        uint32_t static_lds = 0;
        if (hipSetDevice(hip_device) != hipSuccess || tc::count_kernel_static_lds(&static_lds) != hipSuccess) {
            delete c;
            return TC_E_DEVICE;
        }
        c->big_lds_bytes = (uint32_t)((c->lds_per_block_max - static_lds) & ~(size_t)15);
        // Half-LDS launch: the largest LDS (within half a CU's, less the static part) at which the
        // large-vertex kernel is resident twice per CU (the runtime's accounting may add a little).
        if (prop.maxSharedMemoryPerMultiProcessor > 2 * (size_t)static_lds) {
            uint32_t lds = (uint32_t)((prop.maxSharedMemoryPerMultiProcessor / 2 - static_lds) & ~(size_t)15);
            for (int i = 0; i < 16 && lds > 4096; ++i, lds -= 256) {
                int per_cu = 0;
                if (tc::count_kernel_info(true, false, 4, true, 0, 64 * tc::kMidWaves, lds, &per_cu) != hipSuccess)
                    break;
                if (per_cu >= 2) {
                    c->mid_lds_bytes = lds;
                    break;
                }
            }
            int full = 0;  // back to the full-LDS limit (the queries above lowered it)
            if (tc::count_kernel_info(true, false, 4, true, 0, 64 * tc::kMaxWaves, c->big_lds_bytes, &full) !=
                hipSuccess) {
                delete c;
                return TC_E_DEVICE;
            }
        }
        if (static_scratch(hip_device, &c->static_scratch) != hipSuccess) {
            delete c;
            return TC_E_DEVICE;
        }
    }
    c->p = q;
    *out = c;
    return TC_OK;
}

tc_status tc_destroy(tc_context* ctx) {
    if (!ctx) return TC_OK;
    for (hipEvent_t& e : ctx->ev)
        if (e) (void)hipEventDestroy(e);
    for (auto& c : ctx->mcap) {
        if (c.exec) (void)hipGraphExecDestroy(c.exec);
        if (c.hg) (void)hipGraphDestroy(c.hg);
    }
    for (auto& st : ctx->stage) {
        if (st.ev) {
            (void)hipEventSynchronize(st.ev);
            (void)hipEventDestroy(st.ev);
        }
        if (st.host) (void)hipHostFree(st.host);
    }
    if (ctx->capture_stream) (void)hipStreamDestroy(ctx->capture_stream);
    delete ctx;
    return TC_OK;
}

tc_status tc_timing_enable(tc_context* ctx, int on) {
    if (!ctx) return TC_E_INVALID;
    if (on && !ctx->ev[0]) {
        if (tc_status s = use_device(ctx)) return s;
        for (hipEvent_t& e : ctx->ev) HIP_TRY(ctx, hipEventCreate(&e));
    }
    ctx->timing = on != 0;
    ctx->have_build = ctx->have_count = false;
    return TC_OK;
}

tc_status tc_timing_last(tc_context* ctx, float* build_ms, float* count_kernel_ms) {
    if (!ctx || !build_ms || !count_kernel_ms) return TC_E_INVALID;
    *build_ms = -1.0f;
    *count_kernel_ms = -1.0f;
    if (!ctx->timing) return TC_OK;
    if (ctx->have_build) {
        HIP_TRY(ctx, hipEventSynchronize(ctx->ev[1]));
        HIP_TRY(ctx, hipEventElapsedTime(build_ms, ctx->ev[0], ctx->ev[1]));
    }
    if (ctx->have_count) {
        HIP_TRY(ctx, hipEventSynchronize(ctx->ev[3]));
        HIP_TRY(ctx, hipEventElapsedTime(count_kernel_ms, ctx->ev[2], ctx->ev[3]));
    }
    return TC_OK;
}

tc_status tc_set_params(tc_context* ctx, const tc_params* p) {
    if (!ctx) return TC_E_INVALID;
    if (check_params(p) != TC_OK) return fail(ctx, TC_E_INVALID, "invalid tc_params");
    ctx->p = *p;
    return TC_OK;
}

tc_status tc_get_params(const tc_context* ctx, tc_params* out) {
    if (!ctx || !out) return TC_E_INVALID;
    *out = ctx->p;
    return TC_OK;
}

tc_status tc_workspace_bytes(const tc_context* ctx, uint32_t n, uint64_t m_in, uint64_t* bytes) {
    if (!ctx || !bytes) return TC_E_INVALID;
    if (m_in >= (1ull << 31)) return TC_E_UNSUPPORTED;
    const Layout L = layout(ctx, ctx->p, n, m_in);
    *bytes = L.storage + L.temp + L.scratch;
    return TC_OK;
}

tc_status tc_graph_footprint(const tc_context* ctx, uint32_t n, uint64_t m_in, uint64_t* storage_bytes,
                             uint64_t* temp_bytes) {
    if (!ctx || !storage_bytes || !temp_bytes) return TC_E_INVALID;
    if (m_in >= (1ull << 31)) return TC_E_UNSUPPORTED;
    const Layout L = layout(ctx, ctx->p, n, m_in);
    *storage_bytes = L.storage;
    *temp_bytes = L.temp;
    return TC_OK;
}

tc_status tc_count_scratch_bytes(const tc_context* ctx, uint32_t n, uint64_t m_in, uint64_t* bytes) {
    if (!ctx || !bytes) return TC_E_INVALID;
    if (m_in >= (1ull << 31)) return TC_E_UNSUPPORTED;
    *bytes = layout(ctx, ctx->p, n, m_in).scratch;
    return TC_OK;
}

tc_status tc_count(tc_context* ctx, uint32_t n, uint64_t m_in, const uint32_t* d_src, const uint32_t* d_dst,
                   uint64_t* d_per_vertex, void* d_ws, uint64_t ws_bytes, void* stream, uint64_t* h_total) {
    if (!ctx || !h_total) return TC_E_INVALID;
    ctx->err.clear();
    if (m_in && (!d_src || !d_dst)) return fail(ctx, TC_E_INVALID, "null edge arrays");
    if (tc_status s = check_sizes(ctx, m_in)) return s;
    const Layout L = layout(ctx, ctx->p, n, m_in);
    const uint64_t need = L.storage + L.temp + L.scratch;
    if (!d_ws || ws_bytes < need)
        return fail(ctx, TC_E_NOMEM, "workspace %llu bytes < %llu needed", (unsigned long long)ws_bytes,
                    (unsigned long long)need);
    if (tc_status s = use_device(ctx)) return s;
    return count_one_shot(ctx, n, m_in, d_src, d_dst, d_per_vertex, d_ws, L, static_cast<hipStream_t>(stream),
                          h_total);
}

}  // extern "C"

namespace {

// Clean, build and count in the workspace `d_ws` laid out by L (storage | temp | scratch), then read
// the total and the range flag back (synchronises the stream).
tc_status count_one_shot(tc_context* ctx, uint32_t n, uint64_t m_in, const uint32_t* d_src, const uint32_t* d_dst,
                         uint64_t* d_per_vertex, void* d_ws, const Layout& L, hipStream_t st, uint64_t* h_total) {
    char* ws = static_cast<char*>(d_ws);
    tc_graph g;
    if (tc_status s = build_into(ctx, &g, n, m_in, d_src, d_dst, ws, ws + L.storage, L, st)) return s;
    char* d_scr = ws + L.storage + L.temp;
    uint64_t* d_total = reinterpret_cast<uint64_t*>(scratch_base(d_scr) + L.c_total);
    if (tc_status s = count_into(ctx, &g, d_total, d_per_vertex, d_scr, L, st)) return s;
    uint64_t host[2] = {0, 0};
    HIP_TRY(ctx, hipMemcpyAsync(&host[0], d_total, 8, hipMemcpyDeviceToHost, st));
    unsigned int err = 0;
    if (!g.empty) HIP_TRY(ctx, hipMemcpyAsync(&err, &g.dev.meta->err, 4, hipMemcpyDeviceToHost, st));
    HIP_TRY(ctx, hipStreamSynchronize(st));
    if (err & 1u) return fail(ctx, TC_E_RANGE, "an input vertex id is >= n = %u", n);
    *h_total = host[0];
    return TC_OK;
}

}  // namespace

extern "C" {

tc_status tc_graph_build(tc_context* ctx, uint32_t n, uint64_t m_in, const uint32_t* d_src, const uint32_t* d_dst,
                         void* d_storage, uint64_t storage_bytes, void* d_temp, uint64_t temp_bytes, void* stream,
                         tc_graph** out) {
    if (!ctx || !out) return TC_E_INVALID;
    *out = nullptr;
    ctx->err.clear();
    if (m_in && (!d_src || !d_dst)) return fail(ctx, TC_E_INVALID, "null edge arrays");
    if (tc_status s = check_sizes(ctx, m_in)) return s;
    const Layout L = layout(ctx, ctx->p, n, m_in);
    if (!d_storage || storage_bytes < L.storage) return fail(ctx, TC_E_NOMEM, "storage too small");
    if (L.temp && (!d_temp || temp_bytes < L.temp)) return fail(ctx, TC_E_NOMEM, "temp too small");
    if (tc_status s = use_device(ctx)) return s;
    tc_graph* g = new (std::nothrow) tc_graph();
    if (!g) return TC_E_NOMEM;
    tc_status s = build_into(ctx, g, n, m_in, d_src, d_dst, d_storage, d_temp, L, static_cast<hipStream_t>(stream));
    if (s != TC_OK) { delete g; return s; }
    *out = g;
    return TC_OK;
}

tc_status tc_graph_count(tc_context* ctx, const tc_graph* g, uint64_t* d_total, uint64_t* d_per_vertex,
                         void* d_scratch, uint64_t scratch_bytes, void* stream) {
    if (!ctx || !g || !d_total) return TC_E_INVALID;
    if (g->k != 1) return fail(ctx, TC_E_INVALID, "a batch of %u graphs needs tc_graph_count_each", g->k);
    ctx->err.clear();
    const Layout L = layout(ctx, g->p, g->n, g->m_in);
    if (!d_scratch || scratch_bytes < L.scratch) return fail(ctx, TC_E_NOMEM, "scratch too small");
    if (tc_status s = use_device(ctx)) return s;
    return count_into(ctx, g, d_total, d_per_vertex, d_scratch, L, static_cast<hipStream_t>(stream));
}

tc_status tc_graph_count_static(tc_context* ctx, const tc_graph* g, uint64_t* d_total, uint64_t* d_per_vertex,
                                void* stream) {
    if (!ctx || !g || !d_total) return TC_E_INVALID;
    if (g->k != 1) return fail(ctx, TC_E_INVALID, "a batch of %u graphs: single graphs only", g->k);
    ctx->err.clear();
    if (!ctx->static_scratch) return fail(ctx, TC_E_DEVICE, "static scratch not resolved on device %d", ctx->device);
    const Layout L = layout(ctx, g->p, g->n, g->m_in);
    if (L.scratch > TC_STATIC_SCRATCH_BYTES)
        return fail(ctx, TC_E_NOMEM, "count scratch %llu bytes exceeds the static buffer of %llu bytes",
                    (unsigned long long)L.scratch, (unsigned long long)TC_STATIC_SCRATCH_BYTES);
    if (tc_status s = use_device(ctx)) return s;
    return count_into(ctx, g, d_total, d_per_vertex, ctx->static_scratch, L, static_cast<hipStream_t>(stream));
}

tc_status tc_graph_info_get(const tc_graph* g, void* stream, tc_graph_info* out) {
    if (!g || !out) return TC_E_INVALID;
    std::memset(out, 0, sizeof(*out));
    out->n = g->n;
    out->wave_cap = g->caps.wave_cap;
    out->wg_cap = g->caps.wg_cap;
    out->big_cap = g->caps.big_cap;
    out->records = g->dev.rec ? 1u : 0u;
    if (g->empty) return TC_OK;
    tc::GraphMeta m;
    if (hipSetDevice(g->ctx->device) != hipSuccess) return TC_E_DEVICE;
    hipStream_t st = static_cast<hipStream_t>(stream);
    if (hipMemcpyAsync(&m, g->dev.meta, sizeof(m), hipMemcpyDeviceToHost, st) != hipSuccess) return TC_E_DEVICE;
    if (hipStreamSynchronize(st) != hipSuccess) return TC_E_DEVICE;
    out->m = m.m;
    out->wedges_plus = m.wplus;
    out->max_dplus = m.max_dplus;
    out->n_hub = m.bins[0];
    out->n_big = m.bins[1];
    out->n_wg = m.bins[2];
    out->n_wave = m.bins[3];
    out->n_packed = m.bins[4];
    out->n_mid = m.bins[1] - m.big_full;
    out->mid_cap = g->caps.mid_cap;
    if (m.err & 1u) return TC_E_RANGE;
    return TC_OK;
}

tc_status tc_graph_bin_work(const tc_graph* g, void* stream, uint64_t work[6]) {
    if (!g || !work) return TC_E_INVALID;
    for (int i = 0; i < 6; ++i) work[i] = 0;
    if (g->empty) return TC_OK;
    tc::GraphMeta m;
    if (hipSetDevice(g->ctx->device) != hipSuccess) return TC_E_DEVICE;
    hipStream_t st = static_cast<hipStream_t>(stream);
    if (hipMemcpyAsync(&m, g->dev.meta, sizeof(m), hipMemcpyDeviceToHost, st) != hipSuccess) return TC_E_DEVICE;
    if (hipStreamSynchronize(st) != hipSuccess) return TC_E_DEVICE;
    for (int i = 0; i < 6; ++i) work[i] = m.bin_work[i];
    return TC_OK;
}

tc_status tc_graph_release(tc_graph* g) {
    if (!g) return TC_OK;
    drop_capture(g);
    delete g;
    return TC_OK;
}

tc_status tc_vc_locate(const uint32_t* incl_prefix, uint32_t d, uint32_t index, uint32_t* owner, uint32_t* offset) {
    if (!incl_prefix || !owner || !offset || d == 0 || index >= incl_prefix[d - 1]) return TC_E_INVALID;
    const uint32_t k = tc::vc_owner(d, index, [&](uint32_t j) { return incl_prefix[j]; });
    *owner = k;
    *offset = index - (k ? incl_prefix[k - 1] : 0u);
    return TC_OK;
}

tc_status tc_wide_list_addressing(uint64_t m_in, uint32_t flags, int* wide) {
    if (!wide) return TC_E_INVALID;
    *wide = tc::wide_list_addressing(m_in, (flags & TC_F_WIDE_ADDR) != 0) ? 1 : 0;
    return TC_OK;
}

tc_status tc_graph_k(const tc_graph* g, uint32_t* k) {
    if (!g || !k) return TC_E_INVALID;
    *k = g->k;
    return TC_OK;
}

tc_status tc_batch_footprint(const tc_context* ctx, uint32_t k, uint32_t n_total, uint64_t m_total,
                             uint64_t* storage_bytes, uint64_t* temp_bytes) {
    if (!ctx || !storage_bytes || !temp_bytes || k == 0) return TC_E_INVALID;
    if (m_total >= (1ull << 31)) return TC_E_UNSUPPORTED;
    const Layout L = layout(ctx, ctx->p, n_total, m_total, true);
    *storage_bytes = L.storage;
    *temp_bytes = L.temp;
    return TC_OK;
}

tc_status tc_batch_build(tc_context* ctx, uint32_t k, uint32_t n_total, uint64_t m_total, const uint64_t* d_voff,
                         const uint64_t* d_eoff, const uint32_t* d_src, const uint32_t* d_dst, void* d_storage,
                         uint64_t storage_bytes, void* d_temp, uint64_t temp_bytes, void* stream, tc_graph** out) {
    if (!ctx || !out) return TC_E_INVALID;
    *out = nullptr;
    ctx->err.clear();
    if (k == 0 || !d_voff || !d_eoff) return fail(ctx, TC_E_INVALID, "a batch needs k >= 1 and offset arrays");
    if (m_total && (!d_src || !d_dst)) return fail(ctx, TC_E_INVALID, "null edge arrays");
    if (tc_status s = check_sizes(ctx, m_total)) return s;
    const Layout L = layout(ctx, ctx->p, n_total, m_total, true);
    if (!d_storage || storage_bytes < L.storage) return fail(ctx, TC_E_NOMEM, "storage too small");
    if (L.temp && (!d_temp || temp_bytes < L.temp)) return fail(ctx, TC_E_NOMEM, "temp too small");
    if (tc_status s = use_device(ctx)) return s;
    tc_graph* g = new (std::nothrow) tc_graph();
    if (!g) return TC_E_NOMEM;
    const tc::BatchIn bi{reinterpret_cast<const unsigned long long*>(d_voff),
                         reinterpret_cast<const unsigned long long*>(d_eoff), k};
    tc_status s = build_into(ctx, g, n_total, m_total, d_src, d_dst, d_storage, d_temp, L,
                             static_cast<hipStream_t>(stream), &bi);
    if (s != TC_OK) { delete g; return s; }
    *out = g;
    return TC_OK;
}

tc_status tc_graph_count_shard(tc_context* ctx, const tc_graph* g, uint32_t shard, uint32_t shards,
                               uint64_t* d_totals, uint64_t* d_per_vertex, void* d_scratch, uint64_t scratch_bytes,
                               void* stream) {
    if (!ctx || !g || !d_totals) return TC_E_INVALID;
    if (shards == 0 || shard >= shards) return fail(ctx, TC_E_INVALID, "shard %u of %u", shard, shards);
    ctx->err.clear();
    const Layout L = layout(ctx, g->p, g->n, g->m_in, g->batch);
    if (!d_scratch || scratch_bytes < L.scratch) return fail(ctx, TC_E_NOMEM, "scratch too small");
    if (tc_status s = use_device(ctx)) return s;
    return count_into(ctx, g, d_totals, d_per_vertex, d_scratch, L, static_cast<hipStream_t>(stream), true, shard,
                      shards);
}

tc_status tc_graph_collisions(tc_context* ctx, const tc_graph* g, int per_vertex, void* d_scratch,
                              uint64_t scratch_bytes, void* stream, tc_collision_stats* out) {
    if (!ctx || !g || !out) return TC_E_INVALID;
    std::memset(out, 0, sizeof(*out));
    ctx->err.clear();
    if (g->empty) return TC_OK;
    const Layout L = layout(ctx, g->p, g->n, g->m_in, g->batch);
    if (!d_scratch || scratch_bytes < L.scratch) return fail(ctx, TC_E_NOMEM, "scratch too small");
    if (tc_status s = use_device(ctx)) return s;
    const tc_params& p = g->p;
    tc::DiagArgs a{};
    a.meta = g->dev.meta;
    a.off = g->dev.off;
    a.col = g->dev.col;
    a.items = g->dev.items;
    a.avail[0] = (uint32_t)L.hub_words;
    a.avail[1] = big_table_words(ctx);
    a.avail[2] = wg_table_words(p);
    a.avail[3] = slice_words(p);
    a.avail[4] = pack_region(p);
    const uint32_t filt = subwave_lanes(p.flags) == 0 ? 1u : 0u;
    a.filt[0] = 0;
    a.filt[1] = 1;
    a.filt[2] = filt;
    a.filt[3] = filt;
    a.filt[4] = 0;
    a.S = p.slots_per_bucket;
    a.lrecip = tc::load_recip(p.load_factor_pct);
    a.hash_kind = p.hash_kind;
    a.pv = per_vertex ? 1u : 0u;
    a.stats = reinterpret_cast<unsigned long long*>(scratch_base(d_scratch) + L.c_heads);
    hipStream_t s = static_cast<hipStream_t>(stream);
    HIP_TRY(ctx, tc::collision_stats(a, ctx->cu_count, s));
    unsigned long long h[4];
    HIP_TRY(ctx, hipMemcpyAsync(h, a.stats, sizeof(h), hipMemcpyDeviceToHost, s));
    HIP_TRY(ctx, hipStreamSynchronize(s));
    out->phi = h[0];
    out->sum_max_collision = h[1];
    out->tables = h[2];
    out->max_collision = h[3];
    return TC_OK;
}

tc_status tc_graph_count_simple(tc_context* ctx, const tc_graph* g, uint32_t mode, uint64_t* d_total,
                                void* d_scratch, uint64_t scratch_bytes, void* stream) {
    if (!ctx || !g || !d_total) return TC_E_INVALID;
    if (mode & ~(TC_SIMPLE_EDGE_CENTRIC | TC_SIMPLE_BUILD_ONLY)) return fail(ctx, TC_E_INVALID, "mode %u", mode);
    if (g->k != 1) return fail(ctx, TC_E_INVALID, "a batch of %u graphs: single graphs only", g->k);
    ctx->err.clear();
    const Layout L = layout(ctx, g->p, g->n, g->m_in, g->batch);
    if (!d_scratch || scratch_bytes < L.scratch) return fail(ctx, TC_E_NOMEM, "scratch too small");
    if (tc_status s = use_device(ctx)) return s;
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (g->empty) {
        HIP_TRY(ctx, tc::fill_u32(d_total, 0, 2, s));
        return TC_OK;
    }
    tc::GraphMeta m;
    HIP_TRY(ctx, hipMemcpyAsync(&m, g->dev.meta, sizeof(m), hipMemcpyDeviceToHost, s));
    HIP_TRY(ctx, hipStreamSynchronize(s));
    const tc_params& p = g->p;
    // Tables in the workgroup LDS of the count launch, or in all the LDS a workgroup may have.
    uint32_t lds = p.wg_lds_bytes, cap = 0;
    HIP_TRY(ctx, tc::simple_capacity(lds, p.load_factor_pct, &cap));
    if (m.max_dplus > cap) {
        lds = ctx->big_lds_bytes;
        HIP_TRY(ctx, tc::simple_capacity(lds, p.load_factor_pct, &cap));
    }
    if (m.max_dplus > cap)
        return fail(ctx, TC_E_UNSUPPORTED, "out-degree %u exceeds the LDS table limit %u", m.max_dplus, cap);
    tc::SimpleArgs a{};
    a.meta = g->dev.meta;
    a.off = g->dev.off;
    a.col = g->dev.col;
    a.items = g->dev.items;
    a.head = reinterpret_cast<uint32_t*>(scratch_base(d_scratch) + L.c_heads);
    a.total = reinterpret_cast<unsigned long long*>(d_total);
    a.lds_words = lds / 4;
    a.lrecip = tc::load_recip(p.load_factor_pct);
    HIP_TRY(ctx, tc::fill_u32(a.head, 0, 1, s));
    HIP_TRY(ctx, tc::fill_u32(d_total, 0, 2, s));
    const bool rec = ctx->timing;
    if (rec) HIP_TRY(ctx, hipEventRecord(ctx->ev[2], s));
    HIP_TRY(ctx, tc::simple_launch((mode & TC_SIMPLE_EDGE_CENTRIC) != 0, (mode & TC_SIMPLE_BUILD_ONLY) != 0, lds,
                                   ctx->cu_count, a, s));
    if (rec) {
        HIP_TRY(ctx, hipEventRecord(ctx->ev[3], s));
        ctx->have_count = true;
    }
    return TC_OK;
}

tc_status tc_graph_count_each(tc_context* ctx, const tc_graph* g, uint64_t* d_totals, uint64_t* d_per_vertex,
                              void* d_scratch, uint64_t scratch_bytes, void* stream) {
    if (!ctx || !g || !d_totals) return TC_E_INVALID;
    ctx->err.clear();
    const Layout L = layout(ctx, g->p, g->n, g->m_in, g->batch);
    if (!d_scratch || scratch_bytes < L.scratch) return fail(ctx, TC_E_NOMEM, "scratch too small");
    if (tc_status s = use_device(ctx)) return s;
    return count_into(ctx, g, d_totals, d_per_vertex, d_scratch, L, static_cast<hipStream_t>(stream));
}

tc_status tc_graph_count_replay(tc_context* ctx, tc_graph* g, uint64_t* d_totals, uint64_t* d_per_vertex,
                                void* d_scratch, uint64_t scratch_bytes, void* stream) {
    if (!ctx || !g || !d_totals) return TC_E_INVALID;
    ctx->err.clear();
    const Layout L = layout(ctx, g->p, g->n, g->m_in, g->batch);
    if (!d_scratch || scratch_bytes < L.scratch) return fail(ctx, TC_E_NOMEM, "scratch too small");
    if (tc_status s = use_device(ctx)) return s;
    const void* key[3] = {d_totals, d_per_vertex, d_scratch};
    if (!g->exec || std::memcmp(key, g->key, sizeof(key)) != 0) {
        drop_capture(g);
        if (!ctx->capture_stream) HIP_TRY(ctx, hipStreamCreateWithFlags(&ctx->capture_stream, hipStreamNonBlocking));
        int per_cu = 0;  // resolve launch shapes before capture (no attribute calls while capturing)
        if (!g->empty) {
            if (tc_status st = occupancy(ctx, g->p, d_per_vertex != nullptr, false, &per_cu)) return st;
            if (needs_hub_launch(g))
                if (tc_status st = occupancy(ctx, g->p, d_per_vertex != nullptr, true, &per_cu)) return st;
        }
        HIP_TRY(ctx, hipStreamBeginCapture(ctx->capture_stream, hipStreamCaptureModeThreadLocal));
        tc_status st = count_into(ctx, g, d_totals, d_per_vertex, d_scratch, L, ctx->capture_stream, false);
        hipGraph_t hg = nullptr;
        hipError_t e = hipStreamEndCapture(ctx->capture_stream, &hg);
        if (st != TC_OK) {
            if (hg) (void)hipGraphDestroy(hg);
            return st;
        }
        if (e != hipSuccess) return hip_fail(ctx, e, "hipStreamEndCapture");
        g->hg = hg;
        HIP_TRY(ctx, hipGraphInstantiate(&g->exec, g->hg, nullptr, nullptr, 0));
        std::memcpy(g->key, key, sizeof(key));
    }
    HIP_TRY(ctx, hipGraphLaunch(g->exec, static_cast<hipStream_t>(stream)));
    return TC_OK;
}

}  // extern "C"

namespace {

// A pinned staging slot of at least `bytes`, free to overwrite (its last upload has been read).
tc_status staging(tc_context* ctx, size_t bytes, tc_context::Stage** out) {
    tc_context::Stage& st = ctx->stage[ctx->stage_next];
    ctx->stage_next = (ctx->stage_next + 1) % (uint32_t)(sizeof(ctx->stage) / sizeof(ctx->stage[0]));
    if (!st.ev) HIP_TRY(ctx, hipEventCreateWithFlags(&st.ev, hipEventDisableTiming));
    if (st.pending) {
        HIP_TRY(ctx, hipEventSynchronize(st.ev));
        st.pending = false;
    }
    if (st.bytes < bytes) {
        if (st.host) HIP_TRY(ctx, hipHostFree(st.host));
        st.host = nullptr;
        st.bytes = 0;
        size_t cap = 65536;
        while (cap < bytes) cap *= 2;
        HIP_TRY(ctx, hipHostMalloc(&st.host, cap, hipHostMallocDefault));
        st.bytes = cap;
    }
    *out = &st;
    return TC_OK;
}

// tc_count_graphs and its replayed form: checks, the header and descriptors (one upload into the
// workspace), then the launches, direct or from the capture for (workspace, per-vertex mode, knobs).
tc_status count_graphs(tc_context* ctx, uint32_t k, tc_graph* const* graphs, uint64_t* d_totals,
                       uint64_t* const* d_per_vertex, void* d_ws, uint64_t ws_bytes, hipStream_t s, bool replay) {
    if (!ctx) return TC_E_INVALID;
    ctx->err.clear();
    if (k == 0 || !graphs || !d_totals) return fail(ctx, TC_E_INVALID, "k >= 1 graphs and a totals array are required");
    for (uint32_t g = 0; g < k; ++g) {
        if (!graphs[g]) return fail(ctx, TC_E_INVALID, "graph %u is null", g);
        if (graphs[g]->ctx->device != ctx->device) return fail(ctx, TC_E_INVALID, "graph %u is on another device", g);
        if (std::memcmp(&graphs[g]->p, &graphs[0]->p, sizeof(tc_params)) != 0)
            return fail(ctx, TC_E_INVALID, "graph %u was built with other parameters than graph 0", g);
    }
    const tc_params p = graphs[0]->p;
    if (subwave_lanes(p.flags))
        return fail(ctx, TC_E_UNSUPPORTED, "subwave intra-vertex modes count one graph at a time");
    const bool pv = d_per_vertex != nullptr;
    uint64_t n_total = 0, n_totals = 0, hub_words = 0;
    for (uint32_t g = 0; g < k; ++g) {
        const tc_graph* G = graphs[g];
        if (pv && G->n && !d_per_vertex[g]) return fail(ctx, TC_E_INVALID, "per-vertex output %u is null", g);
        n_total += G->n;
        n_totals += G->k;
        hub_words = std::max<uint64_t>(hub_words, hub_words_for(p, G->n, G->m_in));
    }
    if (n_total + (uint64_t)tc::kBins * k >= (1ull << 32))
        return fail(ctx, TC_E_UNSUPPORTED, "%llu vertices in one call (limit 2^32 - 1 - 5 k)",
                    (unsigned long long)n_total);
    const MultiLayout M = multi_layout(ctx, p, k, n_total, pv, hub_words);
    if (!d_ws || ws_bytes < M.bytes)
        return fail(ctx, TC_E_NOMEM, "workspace %llu bytes < %llu needed", (unsigned long long)ws_bytes,
                    (unsigned long long)M.bytes);
    if (tc_status st = use_device(ctx)) return st;

    // Header and descriptors, written to pinned memory (header, then the descriptors) and uploaded
    // with two copies (the heads lie between them in the workspace).
    const size_t hdr_bytes = sizeof(tc::MultiHeader), desc_bytes = sizeof(tc::MultiDesc) * (size_t)k;
    tc_context::Stage* st = nullptr;
    if (tc_status e = staging(ctx, hdr_bytes + desc_bytes, &st)) return e;
    char* ws = scratch_base(d_ws);
    char* h = static_cast<char*>(st->host);
    std::memset(h, 0, hdr_bytes);
    tc::MultiHeader* H = reinterpret_cast<tc::MultiHeader*>(h);
    H->k = k;
    H->pv = pv ? 1u : 0u;
    H->n_total = n_total;
    H->n_totals = n_totals;
    H->totals = reinterpret_cast<unsigned long long*>(d_totals);
    H->desc = reinterpret_cast<const tc::MultiDesc*>(ws + M.desc);
    H->pre = reinterpret_cast<uint32_t*>(ws + M.pre);
    H->tv = reinterpret_cast<unsigned long long*>(ws + M.tv);
    H->heads = reinterpret_cast<uint32_t*>(ws + kMultiHeads);
    H->hub = reinterpret_cast<uint32_t*>(ws + M.hub);
    H->hub_words = hub_words;
    const uint32_t pf[tc::kBins] = {1u, 1u, 1u, p.light_chunk, 4u * p.light_chunk};
    for (uint32_t b = 0; b < tc::kBins; ++b) H->per_fetch[b] = pf[b];
    tc::MultiDesc* D = reinterpret_cast<tc::MultiDesc*>(h + hdr_bytes);
    uint64_t tv0 = 0, t0 = 0;
    for (uint32_t g = 0; g < k; ++g) {
        const tc_graph* G = graphs[g];
        tc::MultiDesc& d = D[g];
        std::memset(&d, 0, sizeof(d));
        d.meta = G->empty ? nullptr : G->dev.meta;
        d.off = G->dev.off32;
        d.col = G->dev.col;
        d.items = G->dev.items;
        d.rank = G->dev.rank;
        d.gid = G->dev.gid;
        d.totals = reinterpret_cast<unsigned long long*>(d_totals + t0);
        d.out = pv ? reinterpret_cast<unsigned long long*>(d_per_vertex[g]) : nullptr;
        d.tv0 = tv0;
        d.n = G->n;
        d.wide = tc::wide_list_addressing(G->m_in, (p.flags & TC_F_WIDE_ADDR) != 0) ? 1u : 0u;
        tv0 += G->n;
        t0 += G->k;
    }
    HIP_TRY(ctx, hipMemcpyAsync(ws, h, hdr_bytes, hipMemcpyHostToDevice, s));
    HIP_TRY(ctx, hipMemcpyAsync(ws + M.desc, h + hdr_bytes, desc_bytes, hipMemcpyHostToDevice, s));
    HIP_TRY(ctx, hipEventRecord(st->ev, s));
    st->pending = true;

    tc::MultiHeader* hdr = reinterpret_cast<tc::MultiHeader*>(ws);
    if (!replay) return multi_launches(ctx, p, pv, hdr, M.hub_wgs, s, true);

    tc_context::MultiCapture* cap = nullptr;
    for (auto& c : ctx->mcap)
        if (c.ws == d_ws && c.pv == pv && std::memcmp(&c.p, &p, sizeof(p)) == 0) cap = &c;
    if (!cap) {
        if (!ctx->capture_stream) HIP_TRY(ctx, hipStreamCreateWithFlags(&ctx->capture_stream, hipStreamNonBlocking));
        int q = 0;  // launch shapes resolved before capture (no attribute calls while capturing)
        if (tc_status e = occupancy(ctx, p, pv, false, &q, true)) return e;
        if (tc_status e = occupancy(ctx, p, pv, true, &q, true)) return e;
        HIP_TRY(ctx, hipStreamBeginCapture(ctx->capture_stream, hipStreamCaptureModeThreadLocal));
        tc_status e = multi_launches(ctx, p, pv, hdr, M.hub_wgs, ctx->capture_stream, false);
        hipGraph_t hg = nullptr;
        hipError_t he = hipStreamEndCapture(ctx->capture_stream, &hg);
        if (e != TC_OK) {
            if (hg) (void)hipGraphDestroy(hg);
            return e;
        }
        if (he != hipSuccess) return hip_fail(ctx, he, "hipStreamEndCapture");
        hipGraphExec_t exec = nullptr;
        he = hipGraphInstantiate(&exec, hg, nullptr, nullptr, 0);
        if (he != hipSuccess) {
            (void)hipGraphDestroy(hg);
            return hip_fail(ctx, he, "hipGraphInstantiate");
        }
        ctx->mcap.push_back({d_ws, pv, p, hg, exec});
        cap = &ctx->mcap.back();
    }
    HIP_TRY(ctx, hipGraphLaunch(cap->exec, s));
    return TC_OK;
}

}  // namespace

extern "C" {

tc_status tc_count_graphs_bytes(const tc_context* ctx, uint32_t k, uint64_t n_total, uint64_t m_max, int per_vertex,
                                uint64_t* bytes) {
    if (!ctx || !bytes || k == 0) return TC_E_INVALID;
    if (m_max >= (1ull << 31) || n_total + (uint64_t)tc::kBins * k >= (1ull << 32)) return TC_E_UNSUPPORTED;
    const uint32_t nb = (uint32_t)std::min<uint64_t>(n_total, 0xFFFFFFFFull);
    *bytes = multi_layout(ctx, ctx->p, k, n_total, per_vertex != 0, hub_words_for(ctx->p, nb, m_max)).bytes;
    return TC_OK;
}

tc_status tc_count_graphs(tc_context* ctx, uint32_t k, tc_graph* const* graphs, uint64_t* d_totals,
                          uint64_t* const* d_per_vertex, void* d_ws, uint64_t ws_bytes, void* stream) {
    return count_graphs(ctx, k, graphs, d_totals, d_per_vertex, d_ws, ws_bytes, static_cast<hipStream_t>(stream),
                        false);
}

tc_status tc_count_graphs_replay(tc_context* ctx, uint32_t k, tc_graph* const* graphs, uint64_t* d_totals,
                                 uint64_t* const* d_per_vertex, void* d_ws, uint64_t ws_bytes, void* stream) {
    return count_graphs(ctx, k, graphs, d_totals, d_per_vertex, d_ws, ws_bytes, static_cast<hipStream_t>(stream),
                        true);
}

}  // extern "C"
