/*
 * trust_tc.h -- exact triangle counting on MI355X (gfx950) by vertex-centric,
 * hash-based list intersection on a degree-oriented CSR graph.
 *
 * Method: the vertex-centric hashing algorithm of the paper (Section 3,
 * Algorithm 1): for every vertex u a hash table of its out-neighbour list is
 * built once, then the out-neighbour list of every out-neighbour v of u is
 * probed against it; each hit closes one triangle.  The graph is first cleaned
 * (self-loops and duplicate edges dropped, pairs read as undirected; Section
 * 2.6) and oriented by rank-by-degree (Section 2.2), ties broken by vertex id,
 * so each triangle is found exactly once.  The result is the exact number of
 * 3-cliques of the undirected simple graph (Sections 1 and 2.1) and,
 * optionally, the number of triangles through each vertex.
 *
 * Conventions shared by every call:
 *   - Memory: every device buffer is owned by the caller.  The library never
 *     allocates or frees device memory; its scratch space comes from a
 *     caller-provided workspace sized by the matching *_bytes query (except
 *     tc_graph_count_static, whose scratch is a static buffer that every
 *     device holds for the life of the process).  Host
 *     memory is allocated only for the opaque handles and a context's pinned
 *     staging buffers (tc_count_graphs).
 *   - Ids: vertex ids are uint32 in [0, n), n <= 2^32 - 1.  Edge samples may
 *     repeat, appear in both directions or be self-loops; all are accepted and
 *     cleaned.  n = 0 or m_in = 0 gives a count of 0.
 *   - Counts are uint64.  Per-vertex counts are indexed by input vertex id and
 *     sum to 3 * total.
 *   - Streams: `stream` is a hipStream_t (passed as void*); NULL means the
 *     default stream.  All device work of a call is ordered on that stream.
 *   - Errors: every call returns a tc_status and never aborts or throws across
 *     the boundary.  tc_last_error() gives a message for the last failure on
 *     a context.  After TC_E_DEVICE the context should be destroyed.
 *   - Threads: a context may be used by one host thread at a time.
 */
#ifndef TRUST_TC_H
#define TRUST_TC_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    TC_OK = 0,
    TC_E_INVALID = 1,      /* null pointer where one is required, bad struct_size or parameter */
    TC_E_RANGE = 2,        /* an input vertex id is >= n */
    TC_E_NOMEM = 3,        /* workspace or storage smaller than the matching query returned */
    TC_E_DEVICE = 4,       /* HIP error or no usable gfx950 device */
    TC_E_UNSUPPORTED = 5,  /* size beyond the supported limits (m_in >= 2^31) */
    TC_E_BUSY = 6          /* reserved for admission control by callers */
} tc_status;

/* Tuning knobs.  None of them changes any result, only speed; every
 * combination accepted by tc_create / tc_set_params gives bit-identical counts. */
typedef struct tc_params {
    uint32_t struct_size;       /* = sizeof(tc_params) */
    uint32_t wg_waves;          /* wavefronts per workgroup, 1..16 (workgroup = 64 * wg_waves lanes) */
    uint32_t wg_lds_bytes;      /* LDS per workgroup for hash tables, 4096..131072 */
    uint32_t wave_max_dplus;    /* out-degree at or below which one wavefront owns a vertex
                                   (capped by what fits in wg_lds_bytes / wg_waves); 0 = largest that fits */
    uint32_t slots_per_bucket;  /* S: 1, 2 or 4 slots per hash bucket */
    uint32_t load_factor_pct;   /* buckets B = smallest power of two with B*S*load >= d+, and B >= d+; 10..100 */
    uint32_t hash_kind;         /* 0: low bits of the id (the degree rank, or the record id with
                                   TC_F_RECORDS); 1: multiplicative (Fibonacci) hash */
    uint32_t light_chunk;       /* vertices a wavefront takes per queue access, 1..256 */
    uint32_t grid_wgs;          /* persistent grid size in workgroups; 0 = fill the device */
    uint32_t flags;             /* TC_F_* below */
} tc_params;

#define TC_F_NO_LPT     0x1u    /* keep rank order instead of largest-work-first within each bin */
#define TC_F_FORCE_WG   0x2u    /* every vertex goes to the workgroup bin (tests) */
#define TC_F_FORCE_HUB  0x4u    /* every vertex goes to the global-memory table bin (tests) */
#define TC_F_SCATTER_CSR 0x8u   /* build the CSR by an atomic counting sort (list order unspecified) instead
                                   of the default stable radix sort of the oriented edges by row */
#define TC_F_WIDE_ADDR  0x10u   /* 64-bit list addressing even below 2^30 edges (tests) */
#define TC_F_FORCE_BIG  0x20u   /* every vertex goes to the large-LDS-table bin (tests) */
/* Vertex order used as the hash ids (paper Section 4.1, reordering; the orientation stays the
 * (degree, id) one).  Default: the (degree, id) rank.  At most one of: */
#define TC_F_ORDER_INDEGREE   0x40u  /* continuous ids by oriented in-degree, largest first */
#define TC_F_ORDER_COLLECTIVE 0x80u  /* vertices by collective degree W(u), largest first, give their
                                        not-yet-numbered out-neighbours the next ids in list order */
/* Intra-vertex work assignment of the probe (paper Section 4.2).  Default: virtual combination.
 * At most one of (the build is the same; counts use the parameters the graph was built with): */
#define TC_F_SUBWAVE_8   0x100u  /* groups of 8 lanes, one out-neighbour list per group */
#define TC_F_SUBWAVE_16  0x200u  /* groups of 16 lanes */
#define TC_F_SUBWAVE_32  0x400u  /* groups of 32 lanes */
#define TC_F_WAVE_LIST   0x800u  /* one list per wavefront at a time (warp-centric) */
#define TC_F_NO_PACK     0x1000u /* no packed bin: one wavefront per light vertex (default: when vertices
                                    with out-degree <= 32 and W(u) <= 512 are at least half of the
                                    wavefront-size tables, they share wavefronts, 4 x 16 lanes when
                                    out-degrees are <= 16, else 2 x 32 lanes) */
#define TC_F_NO_MID      0x2000u /* every large-LDS-bin vertex in the full-LDS launch (one workgroup per
                                    CU); default: those whose tables fit half a CU's LDS are counted by a
                                    second launch with two workgroups per CU */
#define TC_F_RECORDS     0x4000u /* the build also lays each vertex's out-degree and out-list out as one
                                    record (d+, then the neighbours' records' ids), and single-graph
                                    counts read lists through it: a 2-hop list starts in the line of its
                                    length instead of behind a separate offset load, and a record of at
                                    most 32 words that would straddle a 128-byte line starts at the next
                                    one (lists name records by position with its low 5 bits XORed with
                                    those of its line index, so that hashing by low bits still spreads
                                    them).  Not with the TC_F_ORDER_* relabellings or TC_F_SCATTER_CSR
                                    (ignored there), nor where R = 2 m_in + n + 32 (ceil(n / 64) + 1)
                                    reaches 2^31; the
                                    graph's storage grows by 4 R + 8 (n + 1) bytes, the build's
                                    temporaries by 16 (ceil(n / 64) + 1) and a per-vertex count's
                                    scratch by 8 (R - n) bytes */

/* Opaque handles. */
typedef struct tc_context tc_context;
typedef struct tc_graph tc_graph;

/* Summary of a built graph (all in the cleaned, oriented graph). */
typedef struct tc_graph_info {
    uint64_t n;           /* vertex count */
    uint64_t m;           /* undirected edges after cleaning = oriented edges */
    uint64_t wedges_plus; /* W+ = sum over oriented (u,v) of d+(v): the number of 2-hop probes */
    uint32_t max_dplus;   /* largest out-degree */
    uint32_t n_hub;       /* vertices in the global-memory table bin (too large for any LDS table) */
    uint32_t n_wg;        /* vertices in the workgroup (LDS) bin */
    uint32_t n_wave;      /* vertices in the wavefront (LDS) bin */
    uint32_t wave_cap;    /* out-degree limits used for the bins */
    uint32_t wg_cap;
    uint32_t n_big;       /* vertices in the large-LDS bin (one workgroup per CU with all of its LDS) */
    uint32_t big_cap;     /* out-degree limit of the large-LDS bin */
    uint32_t n_packed;    /* light vertices (out-degree <= 32, W(u) <= 512) packed 2-4 to a wavefront; only
                             when they are at least half of the wavefront-size tables */
    uint32_t n_mid;       /* vertices of the large-LDS bin (counted in n_big) whose tables fit half a CU's
                             LDS: a second launch counts them with two workgroups per CU */
    uint32_t mid_cap;     /* out-degree limit of that part (0: no such launch) */
    uint32_t records;     /* 1: built with the record layout (TC_F_RECORDS), which single-graph counts read */
} tc_graph_info;

/* Fill *p with the default knobs (struct_size set). */
tc_status tc_default_params(tc_params* p);

/* Create a context on HIP device `hip_device` (must be gfx950).  p may be NULL
 * for the defaults; it is copied. */
tc_status tc_create(int hip_device, const tc_params* p, tc_context** out);
tc_status tc_destroy(tc_context* ctx);
tc_status tc_set_params(tc_context* ctx, const tc_params* p);
tc_status tc_get_params(const tc_context* ctx, tc_params* out);

const char* tc_status_str(tc_status s);
/* Message of the last failure on ctx ("" if none).  Valid until the next call on ctx. */
const char* tc_last_error(const tc_context* ctx);

/* ---------------------------------------------------------------- one-shot count
 * Bytes of device workspace tc_count needs for a graph of n vertices and m_in
 * input edge samples (an upper bound, independent of the edge values). */
tc_status tc_workspace_bytes(const tc_context* ctx, uint32_t n, uint64_t m_in, uint64_t* bytes);

/* Count the triangles of the undirected simple graph given by the samples
 * (d_src[i], d_dst[i]), i < m_in (device arrays, read only, borrowed for the
 * call).  d_per_vertex: NULL, or device uint64[n] overwritten with the number
 * of triangles through each vertex.  d_ws: device workspace of ws_bytes >=
 * tc_workspace_bytes(); its contents are clobbered.  Synchronises `stream`
 * and writes the total to *h_total (host) on TC_OK. */
tc_status tc_count(tc_context* ctx, uint32_t n, uint64_t m_in, const uint32_t* d_src,
                   const uint32_t* d_dst, uint64_t* d_per_vertex, void* d_ws, uint64_t ws_bytes,
                   void* stream, uint64_t* h_total);

/* ---------------------------------------------------------------- build once, count many
 * tc_graph_footprint: device bytes a built graph keeps (storage) and the
 * transient bytes its build needs (temp), for n vertices and m_in samples. */
tc_status tc_graph_footprint(const tc_context* ctx, uint32_t n, uint64_t m_in,
                             uint64_t* storage_bytes, uint64_t* temp_bytes);

/* Clean, orient and lay out the graph in d_storage (caller-owned, must stay
 * alive until tc_graph_release) and schedule its vertices into bins.  d_temp
 * may be reused by the caller once the stream has passed this call.
 * Asynchronous on `stream`; input range errors are reported by the next
 * synchronous call on the graph (tc_graph_info_get). */
tc_status tc_graph_build(tc_context* ctx, uint32_t n, uint64_t m_in, const uint32_t* d_src,
                         const uint32_t* d_dst, void* d_storage, uint64_t storage_bytes,
                         void* d_temp, uint64_t temp_bytes, void* stream, tc_graph** out);

/* Device scratch bytes one tc_graph_count call needs (per-vertex staging,
 * queue heads, global-memory tables for the bin of vertices too large for any
 * LDS table). */
tc_status tc_count_scratch_bytes(const tc_context* ctx, uint32_t n, uint64_t m_in, uint64_t* bytes);

/* Count the triangles of a built graph.  Asynchronous: the total is written
 * to d_total (device uint64); d_per_vertex as in tc_count.  This call is one
 * persistent kernel launch (preceded, when some out-degree may exceed the
 * workgroup bin's limit, by one launch for the large-vertex bins) plus, with
 * d_per_vertex, one gather launch. */
tc_status tc_graph_count(tc_context* ctx, const tc_graph* g, uint64_t* d_total,
                         uint64_t* d_per_vertex, void* d_scratch, uint64_t scratch_bytes,
                         void* stream);

/* For callers that cannot allocate device memory (code under HIP graph capture, tight serving
 * loops, harnesses that forbid hipMalloc): tc_graph_count with its count scratch in a library-owned
 * static device buffer of TC_STATIC_SCRATCH_BYTES instead of a caller workspace.  Each device the
 * library runs on holds its own copy of that buffer until the process ends; the call itself
 * allocates nothing.  TC_E_NOMEM when the graph's scratch (tc_count_scratch_bytes with the graph's
 * n and m_in) exceeds the buffer, TC_E_INVALID for a batch handle.  The buffer keeps the last
 * call's contents (every call clears what it needs zeroed), and all calls on one device share it:
 * calls that overlap on one device (other streams, other host threads) race, so order them on one
 * stream.  Asynchronous on `stream`, as tc_graph_count. */
#define TC_STATIC_SCRATCH_BYTES (128ull << 20)
tc_status tc_graph_count_static(tc_context* ctx, const tc_graph* g, uint64_t* d_total, uint64_t* d_per_vertex,
                                void* stream);

/* Synchronise `stream` and read the graph's summary; returns TC_E_RANGE if
 * the build saw an id >= n. */
tc_status tc_graph_info_get(const tc_graph* g, void* stream, tc_graph_info* out);

/* Work per bin: work[b] = sum of W(u) (the collective degree, u's number of
 * 2-hop probes) over the vertices of bin b, b = 0 global-memory table, 1
 * large LDS table, 2 workgroup, 3 wavefront, 4 packed, 5 skipped; the sum is
 * W+.  Synchronises `stream`. */
tc_status tc_graph_bin_work(const tc_graph* g, void* stream, uint64_t work[6]);

/* Free the handle (host memory only; the storage stays the caller's). */
tc_status tc_graph_release(tc_graph* g);

/* ---------------------------------------------------------------- batches of graphs
 * k graphs in one call.  Graph g has n_g vertices (local ids 0..n_g-1) and
 * the edge samples [eoff[g], eoff[g+1]) of the concatenated arrays d_src /
 * d_dst; voff[g] = n_0 + ... + n_{g-1} and voff[k] = n_total, eoff[k] =
 * m_total (device uint64 arrays of k+1 entries, read during the build).
 * The batch is cleaned, oriented and binned as one disjoint union (a
 * disjoint union's triangles are the union of its parts' triangles), so one
 * set of preprocessing launches and ONE persistent count launch serve all k
 * graphs.  A local id >= n_g is a range error for the batch.
 * Sizes: storage / temp as for one graph of n_total vertices and m_total
 * samples plus 4 * n_total bytes (graph index of every vertex); see
 * tc_batch_footprint. */
tc_status tc_batch_footprint(const tc_context* ctx, uint32_t k, uint32_t n_total, uint64_t m_total,
                             uint64_t* storage_bytes, uint64_t* temp_bytes);
tc_status tc_batch_build(tc_context* ctx, uint32_t k, uint32_t n_total, uint64_t m_total,
                         const uint64_t* d_voff, const uint64_t* d_eoff, const uint32_t* d_src,
                         const uint32_t* d_dst, void* d_storage, uint64_t storage_bytes, void* d_temp,
                         uint64_t temp_bytes, void* stream, tc_graph** out);

/* Count a built graph or batch, one total per graph: d_totals is a device
 * uint64[k] (k = 1 for tc_graph_build graphs).  d_per_vertex: NULL or device
 * uint64[n_total], indexed by position in the concatenated vertex ranges.
 * Asynchronous; scratch as for tc_graph_count (tc_count_scratch_bytes with
 * n_total and m_total). */
tc_status tc_graph_count_each(tc_context* ctx, const tc_graph* g, uint64_t* d_totals, uint64_t* d_per_vertex,
                              void* d_scratch, uint64_t scratch_bytes, void* stream);

/* Workload partitioning (paper Section 5.1): count only the triangles whose
 * table owner u (the endpoint earliest in (degree, id) order, i.e. lowest
 * rank) has rank(u) mod shards == shard.  Ranks follow degree, so every
 * shard gets a similar mix of heavy and light vertices.  d_totals (device
 * uint64[k], one per graph) and d_per_vertex (NULL or device uint64[n]) are
 * overwritten with that shard's share; summing the shards 0..shards-1 gives
 * exactly what tc_graph_count_each gives.  Each shard runs the same launches
 * over the whole vertex list, skipping vertices of other shards, so shards
 * can go to different devices holding the same graph.  TC_E_INVALID when
 * shards == 0 or shard >= shards; scratch as for tc_graph_count_each.
 * Asynchronous on `stream`. */
tc_status tc_graph_count_shard(tc_context* ctx, const tc_graph* g, uint32_t shard, uint32_t shards,
                               uint64_t* d_totals, uint64_t* d_per_vertex, void* d_scratch, uint64_t scratch_bytes,
                               void* stream);

/* Collision statistics of the hash tables a count of g builds (paper Section
 * 4.1, Equation 2): for every vertex with a table, the bucket count is the
 * one the count kernels use (per-vertex mode sizes tables differently, hence
 * the flag) and max collision(u) is the largest number of out-neighbours of
 * u sharing a home bucket.  A diagnostic (e.g. for comparing vertex orders or
 * hash kinds); counts are not touched.  Uses d_scratch as tc_graph_count
 * does; synchronous on `stream`. */
typedef struct tc_collision_stats {
    uint64_t phi;               /* sum over tables of W(u) * max collision(u), W(u) = sum of d+(v), v in N+(u) */
    uint64_t sum_max_collision; /* sum over tables of max collision(u) */
    uint64_t tables;            /* vertices with a table (d+ >= 2 and W(u) > 0) */
    uint64_t max_collision;     /* largest max collision(u) */
} tc_collision_stats;
tc_status tc_graph_collisions(tc_context* ctx, const tc_graph* g, int per_vertex, void* d_scratch,
                              uint64_t scratch_bytes, void* stream, tc_collision_stats* out);

/* The plain designs of paper Section 3.3 on the same hash tables, for the
 * table-construction ablation: one workgroup per vertex, lane-by-lane
 * lookups, tables in wg_lds_bytes of LDS (all the LDS a workgroup may have
 * when some out-degree needs it).  Mode bits:
 *   TC_SIMPLE_EDGE_CENTRIC: Algorithm 2, the table of N+(u) is built again
 *     for every oriented edge (u, v) (otherwise once per vertex);
 *   TC_SIMPLE_BUILD_ONLY: tables only, no intersection (the count is 0), so
 *     the launch time is the construction time.
 * Writes the total to d_total (device uint64) for a single graph (k = 1);
 * TC_E_UNSUPPORTED when some out-degree does not fit the LDS table.  Uses
 * d_scratch as tc_graph_count does.  Reads the graph summary first
 * (synchronises `stream`), then launches asynchronously; with timing on, the
 * launch is what tc_timing_last reports as the count. */
#define TC_SIMPLE_EDGE_CENTRIC 0x1u
#define TC_SIMPLE_BUILD_ONLY   0x2u
tc_status tc_graph_count_simple(tc_context* ctx, const tc_graph* g, uint32_t mode, uint64_t* d_total,
                                void* d_scratch, uint64_t scratch_bytes, void* stream);

/* As tc_graph_count_each, but the device work (the clears, the count
 * kernel and the per-vertex gather) is captured once into a HIP graph on a
 * stream owned by ctx and replayed on `stream` by later calls with the same
 * arguments (re-captured when they change).  For callers that launch the
 * same count repeatedly with minimal host overhead. */
tc_status tc_graph_count_replay(tc_context* ctx, tc_graph* g, uint64_t* d_totals, uint64_t* d_per_vertex,
                                void* d_scratch, uint64_t scratch_bytes, void* stream);

/* Number of graphs (k) of a built graph or batch. */
tc_status tc_graph_k(const tc_graph* g, uint32_t* k);

/* ---------------------------------------------------------------- many built graphs, one launch
 * The problem of the paper (Sections 1 and 2.1: the triangle count of each undirected simple graph)
 * over k graphs that were built independently (tc_graph_build or tc_batch_build handles, resident on
 * this context's device): ONE persistent count launch serves all of them (plus the large-vertex
 * launch, a set-up launch before them and, with per-vertex output, one gather launch after).
 *
 * tc_count_graphs_bytes: device workspace for any call with at most k handles whose vertex counts
 * sum to at most n_total and whose handles have at most m_max edge samples each, for graphs built
 * with the context's current parameters, with per-vertex output (per_vertex != 0: 8 n_total bytes
 * more) or without.  TC_E_UNSUPPORTED when m_max >= 2^31 or n_total + 5 k >= 2^32.
 *
 * tc_count_graphs: graphs[0..k-1] are handles built with identical tc_params (TC_E_INVALID
 * otherwise; TC_E_UNSUPPORTED for the subwave intra-vertex flags).  d_totals: device uint64 array
 * with one entry per graph: handle g (a batch handle holds k_g graphs, a single graph 1) writes
 * entries [t_g, t_g + k_g), t_g = k_0 + ... + k_{g-1}; they are overwritten, not added to.
 * d_per_vertex: NULL, or a host array of k device pointers, entry g a uint64[n_g] that receives
 * the triangles through each vertex of handle g (input-id order; may be NULL when n_g = 0).
 * d_ws: device workspace of ws_bytes (TC_E_NOMEM if smaller than these graphs need); its contents
 * are clobbered.  Asynchronous on `stream`: the handles' builds must be ordered before it (same
 * stream, or an event), and the call copies a header and one 80-byte descriptor per handle from
 * context-owned pinned host memory into the start of d_ws (pinned host buffers are the only memory
 * a context allocates for itself, apart from the handles).  Calls that share a workspace must be
 * ordered on one stream.
 *
 * tc_count_graphs_replay: the same, but the device launches are captured once into a HIP graph per
 * (workspace address, per-vertex on or off, tc_params) and replayed after the descriptor upload.
 * The launches read k, the descriptors and every size from the workspace, so one capture serves
 * every later call, whatever graphs and k it brings (within the workspace's size). */
tc_status tc_count_graphs_bytes(const tc_context* ctx, uint32_t k, uint64_t n_total, uint64_t m_max, int per_vertex,
                                uint64_t* bytes);
tc_status tc_count_graphs(tc_context* ctx, uint32_t k, tc_graph* const* graphs, uint64_t* d_totals,
                          uint64_t* const* d_per_vertex, void* d_ws, uint64_t ws_bytes, void* stream);
tc_status tc_count_graphs_replay(tc_context* ctx, uint32_t k, tc_graph* const* graphs, uint64_t* d_totals,
                                 uint64_t* const* d_per_vertex, void* d_ws, uint64_t ws_bytes, void* stream);

/* ---------------------------------------------------------------- host-side helpers (no device work)
 * tc_vc_locate: the index map of virtual combination (paper Section 4.2),
 * evaluated on the host by the same code the count kernels run on the
 * device.  The out-neighbour lists N+(v_0..v_{d-1}) of a vertex are read as
 * one flattened sequence; incl_prefix[k] = |N+(v_0)| + ... + |N+(v_k)| (host
 * array of d entries, non-decreasing).  Flattened index `index` belongs to
 * list *owner = the first k with incl_prefix[k] > index, at position *offset =
 * index - incl_prefix[k - 1] (index itself for k = 0).  TC_E_INVALID when a
 * pointer is null, d = 0 or index >= incl_prefix[d - 1].
 *
 * tc_wide_list_addressing: whether a count of a graph with m_in edge samples
 * walks the lists with 64-bit word addressing (*wide = 1) instead of 32-bit
 * byte offsets (*wide = 0).  Wide when 4 * m_in + 256 >= 2^32 (a lane may
 * step 256 bytes past the last list before it moves on) or when `flags`
 * holds TC_F_WIDE_ADDR.  TC_E_INVALID when wide is null. */
tc_status tc_vc_locate(const uint32_t* incl_prefix, uint32_t d, uint32_t index, uint32_t* owner, uint32_t* offset);
tc_status tc_wide_list_addressing(uint64_t m_in, uint32_t flags, int* wide);

/* ---------------------------------------------------------------- timing
 * With timing on, every tc_count / tc_graph_build / tc_graph_count records
 * HIP events on its stream around its device steps (events owned by ctx).
 * tc_timing_last waits for the last recorded events and returns, in
 * milliseconds, the last build (clean, orient, CSR, bins) and the last count
 * kernel launches alone (large-vertex and main kernel); a value is -1 if that step has not run since timing
 * was switched on. */
tc_status tc_timing_enable(tc_context* ctx, int on);
tc_status tc_timing_last(tc_context* ctx, float* build_ms, float* count_kernel_ms);

#ifdef __cplusplus
}
#endif
#endif /* TRUST_TC_H */
