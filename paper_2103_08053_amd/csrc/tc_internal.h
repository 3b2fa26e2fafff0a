// Internal declarations of the device path (not part of the public ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "trust_tc.h"

namespace tc {

constexpr uint32_t kEmpty = 0xFFFFFFFFu;  // empty hash slot; never a valid id (ids < n <= 2^32 - 1)
constexpr uint32_t kMaxWaves = 16;
// Wavefronts of a workgroup of the half-LDS large-vertex launch.  The kernel's scalar registers allow 7
// wavefronts per SIMD: two 12-wavefront workgroups (3 per SIMD each) are resident together, where two
// 16-wavefront ones are not, and capping the kernel at 8 per SIMD spills scalar registers (measured
// slower than one workgroup per CU).
constexpr uint32_t kMidWaves = 12;
constexpr uint32_t kHubWgs = 128;        // workgroups that take global-memory-table vertices
// Queue heads of the count launches: bins 0-2, kWaveQueues sub-queues of each wavefront bin, then the
// half-LDS part of bin 1, each counter in a 128-byte line of its own (kHeadStride words apart).
constexpr uint32_t kWaveQueues = 8;
constexpr uint32_t kHeadStride = 32;
constexpr uint32_t kMidHead = 3 + 2 * kWaveQueues;
constexpr uint32_t kHeadWords = (kMidHead + 1) * kHeadStride;
// Packed bin: out-degree at most 32 and collective degree W(u) at most this (a few steps of 16 lanes).
constexpr uint32_t kPackMaxWork = 512;
constexpr uint32_t kPackMaxD = 32;

// Device-resident summary of a built graph (first 256 bytes of its storage).
struct GraphMeta {
    unsigned long long m;           // oriented edges
    unsigned long long wplus;       // W+ = sum over oriented (u, v) of d+(v)
    unsigned int big_full;          // bin-1 vertices whose tables need more than half a CU's LDS (first in bin 1)
    unsigned int max_dplus;
    unsigned int err;               // bit 0: some input id >= n
    // vertex counts: global-memory tables, large LDS tables (one workgroup per CU), workgroup LDS
    // tables, wavefront LDS slices, light vertices packed several per wavefront, skipped (d+ < 2 or
    // no 2-hop work)
    unsigned int bins[6];
    unsigned int wave_cands, pack_cands;  // census before binning: wavefront-size tables, and packable ones
    unsigned long long bin_work[6];       // sum of W(u) over the vertices of each bin
    unsigned int pad[36];
};
static_assert(sizeof(GraphMeta) == 256, "meta is one 256-byte block");

// Hash-table geometry for a vertex with d out-neighbours, shared by the host
// (capacity per bin) and the kernels (layout in LDS or in global memory).
// Layout in 32-bit words:
//   slots[B*S] | len[B] | pad to 4 | P[2d] | (per-vertex mode) tslot[B*S] | tally[d] | pad to 4 |
//   (filtered tables) filt[fw]
// B is the smallest power of two with B*S > d and B*S*load >= d, so every
// probe chain ends at a bucket with a free slot.  filt is a bit vector of 32*fw
// bits (a power of two) with bit hash(w) set for every element w: a probe whose
// bit is clear cannot be in the table and skips the bucket lookup.
struct Geometry {
    uint32_t B, mask, o_len, o_P, o_tslot, o_tally, o_filt, fbits, words;
};

// A wavefront's queue of probes that passed the filter, at the end of each count launch's LDS:
// kQueueEntries entries of two words (the probed id and, in per-vertex mode, its out-neighbour
// index), then one two-word dummy entry per lane (lanes without a survivor write there, so the
// appends need no lane mask).
constexpr uint32_t kQueueEntries = 64;
constexpr uint32_t kQueueWords = 2 * (kQueueEntries + 64);

// Bucket of element w in a table of B (power of two) buckets: kind 0 takes the low bits of the id
// (ids are degree ranks), kind 1 a multiplicative (Fibonacci) hash.
template <int HK>
__device__ __forceinline__ uint32_t hash_of(uint32_t w, uint32_t B) {
    if constexpr (HK == 0) return w & (B - 1);
    else return (uint32_t)(((uint64_t)(w * 0x9E3779B1u) * B) >> 32);
}

// Smallest power of two >= x, and largest power of two <= x (0 for x = 0).
__host__ __device__ inline uint32_t pow2_ceil(uint32_t x) { return x <= 1 ? 1u : 1u << (32 - __builtin_clz(x - 1)); }
__host__ __device__ inline uint32_t pow2_floor(uint32_t x) { return x ? 1u << (31 - __builtin_clz(x)) : 0u; }

// Slots per element a load factor asks for, in 16-bit fixed point (rounded up): ceil(100 * 2^16 / load).
// Host and device size tables from this same value, so a vertex binned by the host fits on the device.
__host__ __device__ inline uint32_t load_recip(uint32_t load_pct) { return (100u * 65536u + load_pct - 1) / load_pct; }

// Filter words for d elements: at least 16 bits per element (at most 1/16 of the bits set, so at
// most about 6% of the probes that miss pass the filter), at most 64.
__host__ __device__ inline uint32_t filter_words_min(uint32_t d) { return pow2_ceil(d) > 2u ? pow2_ceil(d) / 2u : 1u; }
__host__ __device__ inline uint32_t filter_words_max(uint32_t d) { return 2u * pow2_ceil(d); }

// Layout for d elements in B buckets with a filter of fw words (0: none).
__host__ __device__ inline Geometry geometry_b(uint32_t d, uint32_t S, uint32_t B, bool pv, uint32_t fw = 0) {
    Geometry g;
    g.B = B;
    g.mask = B - 1;
    g.o_len = B * S;
    g.o_P = (g.o_len + B + 3u) & ~3u;
    g.o_tslot = g.o_P + 2 * d;
    g.o_tally = g.o_tslot + (pv ? B * S : 0);
    g.o_filt = (g.o_tally + (pv ? d : 0) + 3u) & ~3u;
    g.fbits = 32u * fw;
    g.words = (g.o_filt + fw + 3u) & ~3u;
    return g;
}

// The smallest table the load factor allows (used to decide which bin a vertex fits):
// B*S > d and B*S >= d * 100 / load (lrecip = load_recip(load)); with `filt`, the smallest filter.
__host__ __device__ inline Geometry geometry(uint32_t d, uint32_t S, uint32_t lrecip, bool pv, bool filt = false) {
    uint32_t need = d / S + 1;
    const uint64_t slots = ((uint64_t)d * lrecip + 65535u) >> 16;
    const uint32_t c = (uint32_t)((slots + S - 1) / S);
    if (c > need) need = c;
    return geometry_b(d, S, pow2_ceil(need), pv, filt ? filter_words_min(d) : 0u);
}

// The table actually used in a region of `avail` words (at least the minimal geometry).
// Filtered tables (the LDS tables probed through the filter) keep the minimal B and give the room
// to the filter: the largest power-of-two filter up to 64 bits per element.  Unfiltered tables
// take the largest power-of-two B at least the minimal one that fits and holds at most
// max(64, 8 d) slots, so a vertex whose region has room gets a lightly loaded table (fewer full
// buckets to walk); words(B) <= B (S (1 + pv) + 1) + (2 + pv) d + 8 bounds that layout, which gives
// B in closed form.
__host__ __device__ inline Geometry geometry_fit(uint32_t d, uint32_t S, uint32_t lrecip, bool pv, uint32_t avail,
                                                 bool filt = false) {
    const Geometry g = geometry(d, S, lrecip, pv, filt);
    if (filt) {
        const uint32_t room = avail > g.o_filt ? avail - g.o_filt : 0u;
        uint32_t fw = room >= 4u ? pow2_floor(room) : 0u;  // a power of two >= 4 needs no padding
        const uint32_t fmax = filter_words_max(d);
        if (fw > fmax) fw = fmax;
        if (fw <= g.fbits / 32u) return g;
        return geometry_b(d, S, g.B, pv, fw);
    }
    const uint32_t cap_slots = d > 8u ? 8u * d : 64u;
    uint32_t B = pow2_floor(cap_slots / S);
    const uint32_t fixed = (pv ? 3u : 2u) * d + 8u;
    const uint32_t per_b = S * (pv ? 2u : 1u) + 1u;
    const uint32_t bw = avail > fixed ? pow2_floor((avail - fixed) / per_b) : 0u;
    if (bw < B) B = bw;
    if (B <= g.B) return g;
    const Geometry h = geometry_b(d, S, B, pv);
    return h.words <= avail ? h : g;
}

// Virtual combination (paper Section 4.2): the out-neighbour lists N+(v_0), ..., N+(v_{d-1}) are
// read as one flattened sequence; incl(k) is the inclusive prefix |N+(v_0)| + ... + |N+(v_k)|.
// Flattened index i belongs to the first k with incl(k) > i, at position i - incl(k - 1) of that
// list.  `incl` is any accessor of the prefix (the kernels read it from their records in LDS);
// d >= 1.  An index at or past incl(d - 1) maps to d - 1.
template <typename Incl>
__host__ __device__ inline uint32_t vc_owner(uint32_t d, uint32_t i, Incl incl) {
    uint32_t l = 0, r = d - 1;
    while (l < r) {
        const uint32_t mid = (l + r) >> 1;
        if (incl(mid) > i) r = mid; else l = mid + 1;
    }
    return l;
}

// The probe's 32-bit list cursor holds byte offsets into col: a lane may step up to 256 bytes past
// the end of its last list before it moves on, so 32-bit offsets hold while 4 m + 256 < 2^32.  Past
// that (or when asked), the cursor is a word index with 64-bit addressing.
__host__ __device__ inline bool wide_list_addressing(uint64_t m_in, bool forced) {
    return forced || 4ull * m_in + 256ull >= (1ull << 32);
}

// Largest d whose table fits in `words` 32-bit words (0 if none).
inline uint32_t capacity(uint32_t words, uint32_t S, uint32_t load_pct, bool pv, bool filt = false) {
    const uint32_t lr = load_recip(load_pct);
    uint32_t lo = 0, hi = words;  // words(d) >= 2d, so d <= words / 2
    while (lo < hi) {
        uint32_t mid = lo + (hi - lo + 1) / 2;
        if (geometry(mid, S, lr, pv, filt).words <= words) lo = mid; else hi = mid - 1;
    }
    return lo;
}

// Pointers into a built graph's storage (rank space: vertex r is the r-th in (degree, id) order).
struct GraphDev {
    GraphMeta* meta;
    int64_t* off;       // [n + 1] CSR offsets of the oriented graph
    uint32_t* off32;    // [n + 1] the same offsets in 32 bits (m_in < 2^31), read by the count kernels
    uint32_t* col;      // [m_in] out-neighbour lists (first meta->m entries used)
    uint32_t* rank;     // [n] input id -> rank
    uint32_t* items;    // [n] scheduled vertices by bin (global table, large LDS, workgroup, wavefront, packed, skipped)
    uint32_t* gid;      // [n] graph index of each rank (batches only, else null)
    uint32_t* rec;      // [record_words(n, m_in)] vertex records (record layout only, else null): rank
                        // r's record at p(r) holds d+(r), then rec_id(p(v)) of each out-neighbour v
    uint32_t* place;    // [2 (n + 1)] record layout: {p(r), d+(r)} of every rank r; entry n holds the
                        // records' extent (words up to the end of the last one)
};

// Batch description for the build (device arrays of k + 1 offsets).
struct BatchIn {
    const unsigned long long* voff;
    const unsigned long long* eoff;
    uint32_t k;
};

struct BuildTemp {
    unsigned long long* keys_a;
    unsigned long long* keys_b;
    uint32_t* aux;       // [2 m_in]: sorted upper endpoints, then the sorted oriented keys
    uint32_t* deg;       // [n + 1]; reused as the fill cursor
    uint32_t* dplus;     // [n + 1]
    uint32_t* order;     // [n]
    unsigned long long* skey_a;  // [n]
    unsigned long long* skey_b;  // [n]
    // relabelling (vertex orders other than the rank; null otherwise)
    unsigned long long* rk_a;    // [n]
    unsigned long long* rk_b;    // [n]
    int64_t* off2;               // [n + 1]
    unsigned long long* place_sz;  // [2 (place_chunks(n) + 1)] record layout: words per chunk, then the chunk bases
    void* sort_tmp;
    size_t sort_tmp_bytes;
};

struct BinCaps {
    uint32_t wave_cap, wg_cap, big_cap;
    uint32_t mid_cap;   // bin-1 out-degrees counted with half a CU's LDS, two workgroups per CU (0: none)
    uint32_t pack_cap;  // out-degree limit of the packed bin (0: no packing)
    bool force_wg, force_hub, force_big, lpt, scatter_csr;
    bool records;       // build the record layout (GraphDev::rec)
    uint32_t order;  // hash-id order: 0 (degree, id) rank, 1 in-degree, 2 collective degree
};

// Record placement: records go in rank order, kPlaceChunk ranks at a time from a 32-word (128-byte)
// line boundary, and a record of at most 32 words that would straddle a line boundary starts at the
// next one instead (the words skipped are fewer than the record's own), so the extent stays below
// record_words(n, m_in).
constexpr uint32_t kPlaceChunk = 64;
__host__ __device__ inline uint64_t place_chunks(uint32_t n) { return ((uint64_t)n + kPlaceChunk - 1) / kPlaceChunk; }
__host__ __device__ inline uint64_t record_words(uint32_t n, uint64_t m_in) { return 2 * m_in + n + 32 * (place_chunks(n) + 1); }
// Id of the record at position p, and position of the record with id p (the map is its own inverse):
// the low 5 bits XORed with those of the line index, so that records moved to a line start still
// spread over hash buckets by their low bits.  Ids stay within p's 32-word line.
__host__ __device__ inline uint32_t rec_id(uint32_t p) { return p ^ ((p >> 5) & 31u); }

struct Layout {
    size_t storage, temp, scratch;
    // storage offsets
    size_t s_meta, s_off, s_off32, s_col, s_rank, s_items, s_gid, s_rec, s_place;
    // temp offsets
    size_t t_keys_a, t_keys_b, t_aux, t_deg, t_dplus, t_order, t_skey_a, t_skey_b, t_rk_a, t_rk_b, t_off2, t_place,
        t_sort;
    size_t sort_tmp_bytes;
    bool relabel;  // temp holds the relabelling arrays
    bool records;  // storage holds the record layout, per-vertex scratch is indexed by record id
    // scratch offsets
    size_t c_tv, c_heads, c_total, c_hub;
    uint64_t hub_words;
    uint32_t hub_wgs;
};

// Several built graphs counted by one launch sequence (tc_count_graphs).  The host writes a
// MultiHeader and one MultiDesc per graph handle into the start of the caller's workspace before
// the launches; every size the launches need (k, vertex totals, table sizes) is read from there,
// so one captured launch sequence serves any set of graphs that fits the workspace.
constexpr uint32_t kBins = 5;  // scheduled bins: global table, large LDS, workgroup, wavefront, packed
struct MultiDesc {
    const GraphMeta* meta;           // null when the handle holds no scheduled vertex (empty graph)
    const uint32_t* off;             // [n + 1] 32-bit CSR offsets
    const uint32_t* col;
    const uint32_t* items;
    const uint32_t* rank;            // [n] input id -> rank (for the per-vertex gather)
    const uint32_t* gid;             // batch handles: graph of each rank; else null
    unsigned long long* totals;      // the handle's k totals (one for a single graph)
    unsigned long long* out;         // per-vertex output, input-id order, or null
    unsigned long long tv0;          // first entry of the handle's per-vertex staging
    uint32_t n;
    uint32_t wide;                   // 64-bit list addressing in the probe
};
static_assert(sizeof(MultiDesc) == 80, "descriptor layout is shared with the host");
struct MultiHeader {
    uint32_t k;                      // graph handles
    uint32_t pv;                     // per-vertex output requested
    unsigned long long n_total;      // sum of the handles' vertex counts (per-vertex staging entries)
    unsigned long long n_totals;     // sum of the handles' graph counts (entries of the totals array)
    unsigned long long* totals;      // all totals, handle after handle
    const MultiDesc* desc;           // [k]
    uint32_t* pre;                   // [kBins][k + 1]: exclusive prefix over handles of each bin's fetches
    unsigned long long* tv;          // [n_total] per-vertex staging in rank space
    uint32_t* heads;                 // [kHeadWords] queue heads
    uint32_t* hub;                   // global-memory tables: hub_wgs regions of hub_words words
    unsigned long long hub_words;
    uint32_t per_fetch[kBins];       // vertices per queue fetch of each bin (host-written)
    uint32_t items_tot[kBins];       // scheduled vertices of each bin over all handles (device-written)
    uint32_t fetch_tot[kBins];       // fetches of each bin over all handles (device-written)
    uint32_t pad[29];
};
static_assert(sizeof(MultiHeader) == 256, "header is one 256-byte block");

struct CountArgs {
    const MultiHeader* multi;        // several graphs (per-graph fields below come from its descriptors)
    const GraphMeta* meta;
    const uint32_t* off;  // [n + 1] 32-bit CSR offsets (half the cache footprint of the 64-bit ones)
    const uint32_t* col;
    const uint32_t* items;
    uint32_t* heads;                 // [kHeadWords] queue heads (zeroed before the launches)
    unsigned long long* total;       // [1] (zeroed before launch); single-graph mode
    const uint32_t* gid;             // [n] graph of each rank (batch mode), or null
    unsigned long long* totals;      // [k] per-graph totals (batch mode, zeroed before launch)
    unsigned long long* tv;          // [n] per-vertex counts in rank space, or null
    uint32_t* hub_scratch;           // hub_wgs * hub_words words
    unsigned long long hub_words;
    uint32_t hub_wgs;                // workgroups of the large-table launch that take global-table vertices
    uint32_t hub_part;               // large-vertex kernel: 0 bin 0 and the full-LDS part of bin 1 (all of
                                     // it in multi-graph mode), 1 the half-LDS part of bin 1
    uint32_t slice_words;            // per-wavefront LDS table slice (each wavefront region: the slice,
                                     // then its probe queue of kQueueWords)
    uint32_t table_words;            // LDS words of the workgroup table region (of this launch); the
                                     // wavefronts' probe queues (kQueueWords each) follow it
    uint32_t lrecip;                 // load_recip(load factor)
    uint32_t chunk;
    uint32_t pack_region;            // LDS words of a packed vertex's table (a quarter of a wavefront slice)
    uint32_t subwave;                // 0: virtual combination; 8/16/32/64: lanes per out-neighbour list
    uint32_t shard, shards;          // count only table owners u (rank) with u % shards == shard
    uint32_t wide;                   // col spans 4 GiB or more: 64-bit addressing in the probe
    const uint32_t* rec;             // record layout (col == rec): ids are record ids (rec_id of the
                                     // position), tv is indexed by them, and with p = rec_id(w) vertex
                                     // w's list is rec[p + 1, p + 1 + rec[p])
    const uint32_t* place;           // record layout: {p(u), d+(u)} of rank u at place[2u]
};

// tc_prep.hip
size_t prep_sort_tmp_bytes(uint32_t n, uint64_t m_in);
hipError_t prep_build(uint32_t n, uint64_t m_in, const uint32_t* src, const uint32_t* dst,
                      const GraphDev& g, const BuildTemp& t, const BinCaps& caps, const BatchIn* batch,
                      hipStream_t stream);
hipError_t fill_u32(void* p, uint32_t value, size_t words, hipStream_t stream);
// out[x] = tv[id(rank[x])] with id(r) = r, or the record id rec_id(place[2r]) when place is given.
hipError_t gather_per_vertex(const unsigned long long* tv, const uint32_t* rank, uint32_t n, const uint32_t* place,
                             unsigned long long* out, hipStream_t stream);
// Zeroes the record layout's per-vertex staging at every record's start (place[2r], r < n): the only
// entries a count adds to.
hipError_t clear_record_staging(unsigned long long* tv, const uint32_t* place, uint32_t n, hipStream_t stream);

// tc_diag.hip: per-table collision statistics of a built graph (the cost model of Equation 2) for
// the tables the count kernels build; avail[bin] = table words of bins 0-4.  stats = {phi,
// sum of max collisions, tables, largest collision} (zeroed here).
struct DiagArgs {
    const GraphMeta* meta;
    const int64_t* off;
    const uint32_t* col;
    const uint32_t* items;
    uint32_t avail[5];
    uint32_t filt[5];                // whether the count's tables of each bin carry a filter
    uint32_t S, lrecip, hash_kind, pv;
    unsigned long long* stats;
};
hipError_t collision_stats(const DiagArgs& a, int cu_count, hipStream_t stream);

// tc_edge.hip: the plain reference designs of Section 3.3 on the same tables, for the construction
// ablation: vertex-centric (one table per vertex) or edge-centric (Algorithm 2: the table of N+(u)
// rebuilt for every edge (u, v)), one workgroup per vertex, lane-by-lane lookups; optionally tables
// only.  Tables are in LDS (lds_words); every scheduled vertex must fit.
struct SimpleArgs {
    const GraphMeta* meta;
    const int64_t* off;
    const uint32_t* col;
    const uint32_t* items;
    uint32_t* head;                  // [1], zeroed before the launch
    unsigned long long* total;       // [1], zeroed before the launch
    uint32_t lds_words, lrecip;
};
constexpr uint32_t kSimpleThreads = 256;
constexpr uint32_t kSimpleS = 4;
hipError_t simple_capacity(uint32_t lds_bytes, uint32_t load_pct, uint32_t* max_d);
hipError_t simple_launch(bool edge, bool build_only, uint32_t lds_bytes, int cu_count, const SimpleArgs& a,
                         hipStream_t stream);

// tc_count.hip: the multi-graph steps around the count launches, all sized from the header at
// `hdr`: clear the totals, queue heads and per-vertex staging and form the per-bin fetch prefixes
// (before), and map the staging back to each handle's input ids (after, per-vertex mode).
hipError_t multi_prepare(MultiHeader* hdr, int cu_count, hipStream_t stream);
hipError_t multi_gather(const MultiHeader* hdr, int cu_count, hipStream_t stream);

// tc_count.hip.  `hub` selects the large-vertex kernel (bins 0 and 1) instead of the main one; `sw` the
// main kernel with subwave probe assignment.
hipError_t count_kernel_info(bool hub, bool sw, uint32_t S, bool pv, uint32_t hash_kind, uint32_t threads,
                             uint32_t lds_bytes, int* blocks_per_cu);
hipError_t count_kernel_static_lds(uint32_t* bytes);
hipError_t count_launch(bool hub, bool sw, uint32_t S, bool pv, uint32_t hash_kind, uint32_t grid, uint32_t threads,
                        uint32_t lds_bytes, const CountArgs& a, hipStream_t stream);
// `multi` selects the kernel variants that take their graphs from a.multi.
hipError_t count_kernel_info_multi(bool hub, uint32_t S, bool pv, uint32_t hash_kind, uint32_t threads,
                                   uint32_t lds_bytes, int* blocks_per_cu);
hipError_t count_launch_multi(bool hub, uint32_t S, bool pv, uint32_t hash_kind, uint32_t grid, uint32_t threads,
                              uint32_t lds_bytes, const CountArgs& a, hipStream_t stream);

}  // namespace tc
