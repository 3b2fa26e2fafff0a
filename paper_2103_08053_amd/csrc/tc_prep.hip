// Device preprocessing: clean, orient and lay out the graph, then bin its vertices.
//
//  1. canonicalise: each sample (a, b) becomes the key (min << nb) | max;
//     self-loops and out-of-range ids become a sentinel that sorts last
//     (cleaning rules of the paper, Section 2.6: duplicates and self-loops
//     removed, directed pairs read as undirected); single graphs form the
//     keys as the sort reads its input;
//  2. radix sort; distinct edges are the first keys of runs of equal keys
//     (duplicates stay in place and are skipped downstream);
//  3. degree of every vertex (distinct edges per run of equal lower ids, in
//     the pass that flags the runs; runs of the sorted upper endpoints), then
//     its rank in (degree, id) order;
//  4. orientation by rank-by-degree (Section 2.2): the edge runs from the
//     lower-ranked to the higher-ranked endpoint, and every id is replaced by
//     its rank, so out-neighbour lists hold ranks and hashing the low bits of
//     a rank spreads neighbours of similar degree over consecutive buckets
//     (the reordering idea of Section 4.1; other orders are optional);
//  5. CSR: stable radix sort of the oriented keys by row, row lengths from key
//     runs, scan (int64 offsets);
//  5c (optional): the record layout: rank r's record at p(r) holds d+(r) and then the record id
//     rec_id(p(v)) of each out-neighbour v; records go in rank order, a short one moved to the next
//     128-byte line where it would straddle one (placed first, written during the scan of step 6,
//     which gathers d+(v) anyway);
//  6. scheduling (Section 4.3): out-degree d+ and collective work
//     W(u) = sum of d+(v) over out-neighbours v (the collective degree of
//     Equation 2); vertices with d+ < 2 or W = 0 are skipped, the rest go by
//     d+ to a global-memory-table bin, a large-LDS bin, a workgroup bin, a
//     wavefront bin or (light vertices, when they dominate) a packed bin, and
//     each bin is ordered by decreasing W (largest work first).
#include <algorithm>
#include <cstring>

#include <rocprim/rocprim.hpp>

#include "tc_internal.h"

namespace tc {
namespace {

constexpr int kThreads = 256;

inline uint32_t grid_for(uint64_t items) {
    uint64_t g = (items + kThreads - 1) / kThreads;
    if (g > 65536) g = 65536;
    if (g == 0) g = 1;
    return (uint32_t)g;
}

inline uint32_t id_bits(uint32_t n) {  // bits to hold any id < n (at least 1)
    uint32_t b = 1;
    while (b < 32 && (1ull << b) < (uint64_t)n) ++b;
    return b;
}

// Key sorts of the build over m_in samples.  64-bit keys sort in onesweep passes of 9-bit digits
// (1024-thread blocks, 8 keys per thread): on gfx950 this beat the library's default 8-bit passes
// at every size measured (44 bits of 2^26 keys 2.03 vs 2.44 ms, 50 bits of 2^29 keys 19.3 vs
// 22.1 ms, rows-only 25 bits of 2^29 keys 10.3 vs 13.3 ms).  32-bit keys take 9-bit digits (16 keys
// per thread) only where that saves a pass (26 bits of 2^29 keys 8.1 vs 9.8 ms; at 23 bits the
// default's three passes are faster).  The size query takes the same path as the sort.
using Onesweep9x64 = rocprim::radix_sort_config<
    rocprim::default_config, rocprim::default_config,
    rocprim::radix_sort_onesweep_config<rocprim::kernel_config<1024, 8>, rocprim::kernel_config<1024, 8>, 9,
                                        rocprim::block_radix_rank_algorithm::match>>;
using Onesweep9x32 = rocprim::radix_sort_config<
    rocprim::default_config, rocprim::default_config,
    rocprim::radix_sort_onesweep_config<rocprim::kernel_config<1024, 16>, rocprim::kernel_config<1024, 16>, 9,
                                        rocprim::block_radix_rank_algorithm::match>>;

template <typename In>
hipError_t sort_keys(void* tmp, size_t& bytes, In in, unsigned long long* out, size_t count, uint32_t lo, uint32_t hi,
                     hipStream_t stream) {
    return rocprim::radix_sort_keys<Onesweep9x64>(tmp, bytes, in, out, count, lo, hi, stream);
}

hipError_t sort_keys(void* tmp, size_t& bytes, uint32_t* in, uint32_t* out, size_t count, uint32_t lo, uint32_t hi,
                     hipStream_t stream) {
    const uint32_t bits = hi - lo;
    if ((bits + 8) / 9 < (bits + 7) / 8)
        return rocprim::radix_sort_keys<Onesweep9x32>(tmp, bytes, in, out, count, lo, hi, stream);
    return rocprim::radix_sort_keys(tmp, bytes, in, out, count, lo, hi, stream);
}

// 32-bit keys with their original positions as values (per-vertex sorts), by the same rule.
hipError_t sort_pairs(void* tmp, size_t& bytes, uint32_t* kin, uint32_t* kout, uint32_t* vout, size_t count,
                      uint32_t hi, hipStream_t stream) {
    const auto pos = rocprim::counting_iterator<uint32_t>(0);
    if ((hi + 8) / 9 < (hi + 7) / 8)
        return rocprim::radix_sort_pairs<Onesweep9x32>(tmp, bytes, kin, kout, pos, vout, count, 0, hi, stream);
    return rocprim::radix_sort_pairs(tmp, bytes, kin, kout, pos, vout, count, 0, hi, stream);
}

// Bits of any vertex degree: at most min(n - 1, 2 m_in).
uint32_t degree_bits(uint32_t n, uint64_t m_in) {
    const uint64_t dmax = (uint64_t)n - 1 < 2 * m_in ? (uint64_t)n - 1 : 2 * m_in;
    uint32_t b = 1;
    while (b < 32 && (1ull << b) <= dmax) ++b;
    return b;
}

constexpr uint32_t kScheduleBits = 27;  // schedule keys: bin (0-5) << 24 | 24-bit reversed work

// Canonical key of sample i, formed as the sort reads its input (its key histogram reads the samples,
// its first step stores the keys in its own buffer); an out-of-range id raises the range error and
// gives the sentinel.
struct CanonKey {
    const uint32_t* src;
    const uint32_t* dst;
    uint32_t n, nb;
    unsigned long long sentinel;
    GraphMeta* meta;
    __device__ unsigned long long operator()(uint64_t i) const {
        const uint32_t a = src[i], b = dst[i];
        if (a >= n || b >= n) {
            if (!meta->err) atomicOr(&meta->err, 1u);
            return sentinel;
        }
        if (a == b) return sentinel;
        const uint32_t lo = a < b ? a : b, hi = a < b ? b : a;
        return ((unsigned long long)lo << nb) | hi;
    }
};

// d+(col[e]) for edge e (0 past the last edge), for the collective-degree scan.
struct HeadOutDegree {
    const uint32_t* col;
    const uint32_t* dplus;
    const GraphMeta* meta;
    __device__ unsigned long long operator()(uint64_t e) const {
        return e < meta->m ? (unsigned long long)dplus[col[e]] : 0ull;
    }
};

// Record layout: for edge e (row r, head v: the sorted oriented key r << nb | v) the scan reads d+(v)
// from v's placement {p(v), d+(v)} (one 8-byte load), and writes v's record id into r's record as a side
// effect (element e - off32[r] of the list behind r's header); the row's first edge also writes the
// row's header d+(r).  Row r's own placement and offset are read in row order.  Idempotent if
// evaluated twice.
struct RecordHead {
    const unsigned long long* okeys;
    const uint32_t* off32;
    const uint2* place;
    uint32_t* rec;
    uint32_t nb;
    unsigned long long mask;
    const GraphMeta* meta;
    __device__ unsigned long long operator()(uint64_t e) const {
        if (e >= meta->m) return 0ull;
        const unsigned long long k = okeys[e];
        const uint32_t r = (uint32_t)(k >> nb), v = (uint32_t)(k & mask);
        const uint2 pv = place[v], pr = place[r];
        const uint32_t i = (uint32_t)e - off32[r];
        rec[pr.x + 1u + i] = rec_id(pv.x);
        if (i == 0) rec[pr.x] = pr.y;
        return (unsigned long long)pv.y;
    }
};

// Record placement (kPlaceChunk ranks per thread, in rank order): the start of a record of s words
// at cursor c, moved to the next 32-word line boundary when s <= 32 and the record would straddle one.
__device__ __forceinline__ uint32_t place_at(uint32_t c, uint32_t s) {
    return (s <= 32u && (c & 31u) + s > 32u) ? ((c + 31u) & ~31u) : c;
}

// Words of each chunk of records, rounded up to a line (chunks start on line boundaries); entry
// `chunks` is 0, so that an exclusive scan gives the chunk bases and, last, the extent.
__global__ void k_place_size(const uint32_t* __restrict__ off32, uint32_t n, unsigned long long* __restrict__ csz) {
    const uint32_t chunks = (uint32_t)place_chunks(n);
    for (uint32_t c = blockIdx.x * blockDim.x + threadIdx.x; c <= chunks; c += gridDim.x * blockDim.x) {
        if (c == chunks) { csz[c] = 0; continue; }
        const uint32_t r0 = c * kPlaceChunk, r1 = r0 + kPlaceChunk < n ? r0 + kPlaceChunk : n;
        uint32_t cur = 0;
        for (uint32_t r = r0; r < r1; ++r) {
            const uint32_t sz = off32[r + 1] - off32[r] + 1u;
            cur = place_at(cur, sz) + sz;
        }
        csz[c] = (cur + 31u) & ~31u;
    }
}

// {p(r), d+(r)} of every rank from the chunk bases; entry n gets {extent, 0}.
__global__ void k_place_write(const uint32_t* __restrict__ off32, uint32_t n,
                              const unsigned long long* __restrict__ cbase, uint2* __restrict__ place) {
    const uint32_t chunks = (uint32_t)place_chunks(n);
    for (uint32_t c = blockIdx.x * blockDim.x + threadIdx.x; c <= chunks; c += gridDim.x * blockDim.x) {
        if (c == chunks) { place[n] = make_uint2((uint32_t)cbase[chunks], 0u); continue; }
        const uint32_t r0 = c * kPlaceChunk, r1 = r0 + kPlaceChunk < n ? r0 + kPlaceChunk : n;
        uint32_t cur = (uint32_t)cbase[c];
        for (uint32_t r = r0; r < r1; ++r) {
            const uint32_t d = off32[r + 1] - off32[r];
            cur = place_at(cur, d + 1u);
            place[r] = make_uint2(cur, d);
            cur += d + 1u;
        }
    }
}

// Zeroes the record layout's per-vertex staging where the count adds to it: at every record's start
// (the ids the count handles are record ids), in rank order.
__global__ void k_clear_record_starts(unsigned long long* __restrict__ tv, const uint32_t* __restrict__ place,
                                      uint32_t n) {
    for (uint32_t r = blockIdx.x * blockDim.x + threadIdx.x; r < n; r += gridDim.x * blockDim.x)
        tv[rec_id(place[2 * (uint64_t)r])] = 0ull;
}

__device__ __forceinline__ bool first_of_run(const unsigned long long* keys, uint64_t i, unsigned long long sentinel) {
    const unsigned long long k = keys[i];
    return k != sentinel && (i == 0 || keys[i - 1] != k);
}

// The CSR offsets narrowed to 32 bits for the count kernels (m_in < 2^31): at 2^25 vertices the
// 64-bit array (268 MB) no longer fits the Infinity Cache, the 32-bit one (134 MB) does.
__global__ void k_narrow(const int64_t* __restrict__ off, uint64_t n1, uint32_t* __restrict__ off32) {
    for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < n1; i += (uint64_t)gridDim.x * blockDim.x)
        off32[i] = (uint32_t)off[i];
}

__global__ void k_fill_u32(uint32_t* p, uint32_t v, size_t words) {
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < words; i += (size_t)gridDim.x * blockDim.x)
        p[i] = v;
}

// Largest g in [0, k) with off[g] <= x (off is non-decreasing, off[0] = 0).
__device__ __forceinline__ uint32_t owner(const unsigned long long* off, uint32_t k, unsigned long long x) {
    uint32_t lo = 0, hi = k - 1;
    while (lo < hi) {
        const uint32_t mid = (lo + hi + 1) >> 1;
        if (off[mid] <= x) lo = mid; else hi = mid - 1;
    }
    return lo;
}

// Batch form: sample e belongs to graph g with eoff[g] <= e < eoff[g+1]; its
// local ids are shifted by voff[g].  Local ids >= n_g, and union ids >= n
// (malformed offsets), are range errors.
__global__ void k_canon_batch(const uint32_t* __restrict__ src, const uint32_t* __restrict__ dst, uint64_t m_in,
                              uint32_t n, uint32_t nb, unsigned long long sentinel,
                              const unsigned long long* __restrict__ voff, const unsigned long long* __restrict__ eoff,
                              uint32_t k, unsigned long long* __restrict__ keys, GraphMeta* meta) {
    uint32_t bad = 0;
    if (blockIdx.x == 0 && threadIdx.x == 0 &&
        (voff[0] != 0 || eoff[0] != 0 || voff[k] != n || eoff[k] != m_in))
        bad = 1;
    // The graph of sample i: one binary search per block and step (its first sample), then each
    // thread moves forward over the few graphs a run of blockDim samples can span.
    __shared__ uint32_t s_g;
    for (uint64_t base = blockIdx.x * (uint64_t)blockDim.x; base < m_in; base += (uint64_t)gridDim.x * blockDim.x) {
        if (threadIdx.x == 0) s_g = owner(eoff, k, base);
        __syncthreads();
        const uint64_t i = base + threadIdx.x;
        uint32_t g = s_g;
        __syncthreads();
        if (i >= m_in) continue;
        while (g + 1 < k && eoff[g + 1] <= i) ++g;
        const unsigned long long v0 = voff[g], ng = voff[g + 1] - v0;
        const unsigned long long a = (unsigned long long)src[i] + v0, b = (unsigned long long)dst[i] + v0;
        unsigned long long key;
        if (src[i] >= ng || dst[i] >= ng || a >= n || b >= n) { bad = 1; key = sentinel; }
        else if (a == b) key = sentinel;
        else {
            const unsigned long long lo = a < b ? a : b, hi = a < b ? b : a;
            key = (lo << nb) | hi;
        }
        keys[i] = key;
    }
    if (bad) atomicOr(&meta->err, 1u);
}

// Graph index of every vertex in rank space.
__global__ void k_gid(const uint32_t* __restrict__ order, uint32_t n, const unsigned long long* __restrict__ voff,
                      uint32_t k, uint32_t* __restrict__ gid) {
    for (uint32_t r = blockIdx.x * blockDim.x + threadIdx.x; r < n; r += gridDim.x * blockDim.x)
        gid[r] = owner(voff, k, order[r]);
}

// One pass over the sorted keys (duplicates in place, sentinels last).  A distinct edge is the first
// key of its run of equal keys.  upper[i] = its upper id, or (duplicates and sentinels) a value above
// every id (bit nb set, or all ones when ids take 32 bits) so it sorts last.  Its lower id gets one
// degree: a wavefront walks a chunk of kRunChunk consecutive keys 64 at a time; equal lower ids are
// contiguous lanes (groups, found by ballot), the last lane of each group adds the group's distinct
// edges, and the group reaching the wavefront's last lane carries over to the next step, so a long
// run (a hub's row) costs one atomic per chunk (the sentinel's lower bits match no valid lower id,
// which is below n - 1).  m = the number of distinct edges, one atomic per workgroup.
constexpr uint32_t kRunChunk = 64 * 32;

__global__ void k_runs(const unsigned long long* __restrict__ keys, uint32_t nb, uint64_t cap,
                       unsigned long long sentinel, uint32_t* __restrict__ upper, uint32_t* __restrict__ deg,
                       GraphMeta* meta) {
    const unsigned long long mask = (nb >= 32) ? 0xFFFFFFFFull : ((1ull << nb) - 1);
    const uint32_t above = nb >= 32 ? 0xFFFFFFFFu : (1u << nb);
    const uint32_t lane = threadIdx.x & 63u;
    __shared__ unsigned long long s_m;
    if (threadIdx.x == 0) s_m = 0;
    __syncthreads();
    unsigned long long firsts = 0;
    const unsigned long long upto = lane == 63 ? ~0ull : ((2ull << lane) - 1);  // lanes 0..lane
    const uint64_t waves = (uint64_t)gridDim.x * (blockDim.x >> 6);
    // wavefront-uniform trip counts: every lane takes part in the ballots
    for (uint64_t c0 = (blockIdx.x * (uint64_t)(blockDim.x >> 6) + (threadIdx.x >> 6)) * kRunChunk; c0 < cap;
         c0 += waves * kRunChunk) {
        uint32_t clo = 0xFFFFFFFFu, cc = 0;  // carried group (uniform)
        for (uint32_t st = 0; st < kRunChunk && c0 + st < cap; st += 64) {
            const uint64_t i = c0 + st + lane;
            bool first = false;
            uint32_t lo = 0xFFFFFFFFu;
            if (i < cap) {
                const unsigned long long k = keys[i];
                first = k != sentinel && (i == 0 || keys[i - 1] != k);
                lo = (uint32_t)(k >> nb);
                upper[i] = first ? (uint32_t)(k & mask) : above;
            }
            const uint32_t lo_prev = (uint32_t)__shfl_up((int)lo, 1, 64);
            const unsigned long long F = __ballot(first);
            const unsigned long long H = __ballot(lane == 0 || lo != lo_prev);  // group starts
            const uint32_t s = 63u - (uint32_t)__builtin_clzll(H & upto);      // this lane's group start
            const uint32_t c = (uint32_t)__popcll((F & upto) >> s);            // its firsts up to this lane
            const bool merge = __builtin_amdgcn_readfirstlane(lo) == clo;     // first group continues the carry
            const uint32_t tail = 63u - (uint32_t)__builtin_clzll(H);          // start of lane 63's group
            if (lane != 63 && ((H >> (lane + 1)) & 1ull)) {                    // last lane of an inner group
                const uint32_t cnt = c + ((s == 0 && merge) ? cc : 0u);
                if (cnt) atomicAdd(&deg[lo], cnt);
            }
            const uint32_t c63 = (uint32_t)__builtin_amdgcn_readlane((int)c, 63);
            const uint32_t lo63 = (uint32_t)__builtin_amdgcn_readlane((int)lo, 63);
            if (tail == 0 && merge) {
                cc += c63;
            } else {
                if (!merge && cc && lane == 0) atomicAdd(&deg[clo], cc);
                clo = lo63;
                cc = c63;
            }
            if (lane == 0) firsts += (unsigned long long)__popcll(F);
        }
        if (cc && lane == 0) atomicAdd(&deg[clo], cc);
    }
    if (lane == 0 && firsts) atomicAdd(&s_m, firsts);
    __syncthreads();
    if (threadIdx.x == 0 && s_m) atomicAdd(&meta->m, s_m);
}

// Upper endpoints' degrees: the sorted upper ids of the distinct edges, counted by run length (the
// run's first element subtracts its index, its last adds index + 1; two atomics per run, mod 2^32:
// no counter is hammered by a hub vertex).
__global__ void k_degree(const uint32_t* __restrict__ upper, uint64_t cap, const GraphMeta* meta,
                         uint32_t* __restrict__ deg) {
    const uint64_t m = meta->m;
    for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < cap; i += (uint64_t)gridDim.x * blockDim.x) {
        if (i < m) {
            const uint32_t hi = upper[i];
            if (i == 0 || upper[i - 1] != hi) atomicSub(&deg[hi], (uint32_t)i);
            if (i + 1 == m || upper[i + 1] != hi) atomicAdd(&deg[hi], (uint32_t)(i + 1));
        }
    }
}

__global__ void k_rank(const uint32_t* __restrict__ order, uint32_t n, uint32_t* __restrict__ rank) {
    for (uint32_t r = blockIdx.x * blockDim.x + threadIdx.x; r < n; r += gridDim.x * blockDim.x)
        rank[order[r]] = r;
}

__global__ void k_orient_count(const unsigned long long* __restrict__ keys, uint32_t nb, uint64_t cap,
                               unsigned long long sentinel, const uint32_t* __restrict__ rank,
                               uint32_t* __restrict__ dplus) {
    const unsigned long long mask = (nb >= 32) ? 0xFFFFFFFFull : ((1ull << nb) - 1);
    for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < cap; i += (uint64_t)gridDim.x * blockDim.x) {
        if (!first_of_run(keys, i, sentinel)) continue;
        const unsigned long long k = keys[i];
        const uint32_t ra = rank[(uint32_t)(k >> nb)], rb = rank[(uint32_t)(k & mask)];
        atomicAdd(&dplus[ra < rb ? ra : rb], 1u);
    }
}

__global__ void k_orient_fill(const unsigned long long* __restrict__ keys, uint32_t nb, uint64_t cap,
                              unsigned long long sentinel, const uint32_t* __restrict__ rank,
                              const int64_t* __restrict__ off, uint32_t* __restrict__ cursor,
                              uint32_t* __restrict__ col) {
    const unsigned long long mask = (nb >= 32) ? 0xFFFFFFFFull : ((1ull << nb) - 1);
    for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < cap; i += (uint64_t)gridDim.x * blockDim.x) {
        if (!first_of_run(keys, i, sentinel)) continue;
        const unsigned long long k = keys[i];
        const uint32_t ra = rank[(uint32_t)(k >> nb)], rb = rank[(uint32_t)(k & mask)];
        const uint32_t s = ra < rb ? ra : rb, d = ra < rb ? rb : ra;
        const uint32_t pos = atomicAdd(&cursor[s], 1u);
        col[off[s] + pos] = d;
    }
}

// Oriented keys (rank_lo << nb | rank_hi) of the distinct edges for a
// sort-based CSR build; duplicates and sentinels stay the sentinel (sort last).
__global__ void k_orient_keys(const unsigned long long* __restrict__ keys, uint32_t nb, uint64_t cap,
                              const uint32_t* __restrict__ rank, unsigned long long sentinel,
                              unsigned long long* __restrict__ okeys) {
    const unsigned long long mask = (nb >= 32) ? 0xFFFFFFFFull : ((1ull << nb) - 1);
    for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < cap; i += (uint64_t)gridDim.x * blockDim.x) {
        if (first_of_run(keys, i, sentinel)) {
            const unsigned long long k = keys[i];
            const uint32_t ra = rank[(uint32_t)(k >> nb)], rb = rank[(uint32_t)(k & mask)];
            okeys[i] = ((unsigned long long)(ra < rb ? ra : rb) << nb) | (ra < rb ? rb : ra);
        } else {
            okeys[i] = sentinel;
        }
    }
}

// From sorted oriented keys: col[i] = head, and d+ of each row as its run
// length (the run's first key subtracts its index, its last adds index + 1).
__global__ void k_csr_runs(const unsigned long long* __restrict__ okeys, uint32_t nb, uint64_t cap,
                           const GraphMeta* meta, uint32_t* __restrict__ dplus, uint32_t* __restrict__ col) {
    const uint64_t m = meta->m;
    const unsigned long long mask = (nb >= 32) ? 0xFFFFFFFFull : ((1ull << nb) - 1);
    for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < cap && i < m; i += (uint64_t)gridDim.x * blockDim.x) {
        const unsigned long long k = okeys[i];
        const uint32_t s = (uint32_t)(k >> nb);
        col[i] = (uint32_t)(k & mask);
        if (i == 0 || (uint32_t)(okeys[i - 1] >> nb) != s) atomicSub(&dplus[s], (uint32_t)i);
        if (i + 1 == m || (uint32_t)(okeys[i + 1] >> nb) != s) atomicAdd(&dplus[s], (uint32_t)(i + 1));
    }
}

// Census for the packed bin: vertices that would get a wavefront-size table, and how many of them
// are light enough to pack (out-degree <= pack_cap, W(u) <= kPackMaxWork).  Packing pays when light
// vertices dominate (their per-vertex fixed work is what it shares); the schedule packs only then.
__global__ void k_pack_census(const int64_t* __restrict__ off, const unsigned long long* __restrict__ wscan,
                              uint32_t n, BinCaps caps, GraphMeta* meta) {
    uint32_t wc = 0, pc = 0;
    for (uint32_t r = blockIdx.x * blockDim.x + threadIdx.x; r < n; r += gridDim.x * blockDim.x) {
        const int64_t b = off[r], e = off[r + 1];
        const uint32_t d = (uint32_t)(e - b);
        const unsigned long long w = d ? wscan[e - 1] - (b ? wscan[b - 1] : 0ull) : 0ull;
        if (d < 2 || w == 0 || caps.force_hub || caps.force_big || caps.force_wg || d > caps.wave_cap) continue;
        ++wc;
        pc += (d <= caps.pack_cap && w <= kPackMaxWork) ? 1u : 0u;
    }
    for (int o = 32; o > 0; o >>= 1) {
        wc += __shfl_xor(wc, o);
        pc += __shfl_xor(pc, o);
    }
    if ((threadIdx.x & 63) == 0 && wc) {
        atomicAdd(&meta->wave_cands, wc);
        atomicAdd(&meta->pack_cands, pc);
    }
}

// One thread per vertex: d+, W(u) = sum of d+(v) over v in N+(u) (from the
// inclusive scan of d+(col[e]) over the edges), bin, and the sort key
// (bin << 24 | reversed work, clamped to 24 bits).  Bins: 0 global-memory table (too large for
// any LDS table), 1 large LDS table (whole LDS of a workgroup, one per CU),
// 2 workgroup LDS table, 3 wavefront LDS slice, 4 light vertices packed
// several to a wavefront, 5 skipped.  Bin 1 is split in two parts, each by decreasing work: first
// the vertices whose tables need more than half a CU's LDS (counted by one workgroup per CU), then
// those up to caps.mid_cap (two workgroups per CU); the work field there takes 23 bits.
__global__ void k_schedule(const int64_t* __restrict__ off, const unsigned long long* __restrict__ wscan, uint32_t n,
                           BinCaps caps, GraphMeta* meta, uint32_t* __restrict__ skey, uint32_t* __restrict__ rec,
                           const uint32_t* __restrict__ place) {
    __shared__ unsigned long long s_w;
    __shared__ unsigned int s_max, s_bins[6], s_full;
    __shared__ unsigned long long s_bw[6];
    if (threadIdx.x < 6) {
        s_bins[threadIdx.x] = 0;
        s_bw[threadIdx.x] = 0;
    }
    if (threadIdx.x == 0) { s_w = 0; s_max = 0; s_full = 0; }
    __syncthreads();
    const unsigned long long kWorkMax = (1ull << 24) - 1;  // larger work ties: LPT order is a heuristic
    const unsigned long long kWorkMax1 = (1ull << 23) - 1;  // bin 1: below the part bit
    const uint32_t pack_cap = (caps.pack_cap && 2ull * meta->pack_cands >= meta->wave_cands) ? caps.pack_cap : 0u;
    // Per-thread partials, reduced across the wave, then one LDS atomic per wave.
    unsigned long long wsum = 0;
    uint32_t dmax = 0, nb0 = 0, nb1 = 0, nb2 = 0, nb3 = 0, nb4 = 0, nb5 = 0, nfull = 0;
    unsigned long long bw[6] = {0, 0, 0, 0, 0, 0};
    for (uint32_t r = blockIdx.x * blockDim.x + threadIdx.x; r < n; r += gridDim.x * blockDim.x) {
        const int64_t b = off[r], e = off[r + 1];
        const uint32_t d = (uint32_t)(e - b);
        const unsigned long long w = d ? wscan[e - 1] - (b ? wscan[b - 1] : 0ull) : 0ull;
        if (rec && d == 0) rec[place[2 * r]] = 0;  // the header of a row without edges (the others: in the W scan)
        uint32_t bin;
        if (d < 2 || w == 0) bin = 5;
        else if (caps.force_hub || d > caps.big_cap) bin = 0;
        else if (caps.force_big || d > caps.wg_cap) bin = 1;
        else if (caps.force_wg || d > caps.wave_cap) bin = 2;
        else if (d <= pack_cap && w <= kPackMaxWork) bin = 4;
        else bin = 3;
        if (bin == 1) {
            const uint32_t half = d <= caps.mid_cap ? 1u : 0u;
            const unsigned long long wk = w > kWorkMax1 ? kWorkMax1 : w;
            skey[r] = (1u << 24) | (half << 23) | (uint32_t)(caps.lpt ? (kWorkMax1 - wk) : 0ull);
            nfull += half ^ 1u;
        } else {
            const unsigned long long wk = w > kWorkMax ? kWorkMax : w;
            skey[r] = (bin << 24) | (uint32_t)(caps.lpt ? (kWorkMax - wk) : 0ull);
        }
        wsum += w;
#pragma unroll
        for (int q = 0; q < 6; ++q) bw[q] += (bin == (uint32_t)q) ? w : 0ull;
        dmax = d > dmax ? d : dmax;
        nb0 += bin == 0;
        nb1 += bin == 1;
        nb2 += bin == 2;
        nb3 += bin == 3;
        nb4 += bin == 4;
        nb5 += bin == 5;
    }
    for (int o = 32; o > 0; o >>= 1) {
        wsum += __shfl_xor(wsum, o);
#pragma unroll
        for (int q = 0; q < 6; ++q) bw[q] += __shfl_xor(bw[q], o);
        const uint32_t dm = __shfl_xor(dmax, o);
        dmax = dm > dmax ? dm : dmax;
        nb0 += __shfl_xor(nb0, o);
        nb1 += __shfl_xor(nb1, o);
        nb2 += __shfl_xor(nb2, o);
        nb3 += __shfl_xor(nb3, o);
        nb4 += __shfl_xor(nb4, o);
        nb5 += __shfl_xor(nb5, o);
        nfull += __shfl_xor(nfull, o);
    }
    if ((threadIdx.x & 63) == 0) {
        atomicAdd(&s_w, wsum);
        atomicMax(&s_max, dmax);
        atomicAdd(&s_bins[0], nb0);
        atomicAdd(&s_bins[1], nb1);
        atomicAdd(&s_bins[2], nb2);
        atomicAdd(&s_bins[3], nb3);
        atomicAdd(&s_bins[4], nb4);
        atomicAdd(&s_bins[5], nb5);
        if (nfull) atomicAdd(&s_full, nfull);
#pragma unroll
        for (int q = 0; q < 6; ++q)
            if (bw[q]) atomicAdd(&s_bw[q], bw[q]);
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        atomicAdd(&meta->wplus, s_w);
        atomicMax(&meta->max_dplus, s_max);
        if (s_full) atomicAdd(&meta->big_full, s_full);
        for (int i = 0; i < 6; ++i) atomicAdd(&meta->bins[i], s_bins[i]);
        for (int i = 0; i < 6; ++i)
            if (s_bw[i]) atomicAdd(&meta->bin_work[i], s_bw[i]);
    }
}

// ---- vertex orders for the hash ids (Section 4.1, reordering)

// In-degree order: larger oriented in-degree d-(r) = deg(r) - d+(r) first, ties by rank.
__global__ void k_key_indegree(const uint32_t* __restrict__ deg_sorted, const uint32_t* __restrict__ dplus,
                               uint32_t n, unsigned long long* __restrict__ key) {
    for (uint32_t r = blockIdx.x * blockDim.x + threadIdx.x; r < n; r += gridDim.x * blockDim.x) {
        const uint32_t din = deg_sorted[r] - dplus[r];
        key[r] = ((unsigned long long)(0xFFFFFFFFu - din) << 32) | r;
    }
}

// Collective degree W(r) (from the inclusive scan of d+(col[e])), larger first, ties by rank.
__global__ void k_key_collective(const int64_t* __restrict__ off, const unsigned long long* __restrict__ wscan,
                                 uint32_t n, unsigned long long* __restrict__ key) {
    for (uint32_t r = blockIdx.x * blockDim.x + threadIdx.x; r < n; r += gridDim.x * blockDim.x) {
        const int64_t b = off[r], e = off[r + 1];
        unsigned long long w = e > b ? wscan[e - 1] - (b ? wscan[b - 1] : 0ull) : 0ull;
        if (w > 0xFFFFFFFFull) w = 0xFFFFFFFFull;
        key[r] = ((0xFFFFFFFFull - w) << 32) | r;
    }
}

// Greedy numbering of the collective order, in parallel: vertices taken in W order hand the next ids
// to their not-yet-numbered out-neighbours in list order, so v's id follows its first claim, the
// smallest (position of u in W order, position of v in u's list) over its in-edges u -> v.
// One wavefront per row.
__global__ void k_claim(const int64_t* __restrict__ off, const uint32_t* __restrict__ col,
                        const uint32_t* __restrict__ posw, uint32_t n, unsigned long long* __restrict__ claim) {
    const uint32_t lane = threadIdx.x & 63u;
    const uint32_t nwv = (gridDim.x * blockDim.x) >> 6;
    for (uint32_t r = (blockIdx.x * blockDim.x + threadIdx.x) >> 6; r < n; r += nwv) {
        const int64_t b = off[r];
        const uint32_t d = (uint32_t)(off[r + 1] - b);
        const unsigned long long hi = (unsigned long long)posw[r] << 32;
        for (uint32_t j = lane; j < d; j += 64) atomicMin(&claim[col[b + j]], hi | j);
    }
}

// Unclaimed vertices (no in-edges) follow every claimed one, by rank.
__global__ void k_key_claimed(uint32_t n, unsigned long long* __restrict__ claim) {
    for (uint32_t r = blockIdx.x * blockDim.x + threadIdx.x; r < n; r += gridDim.x * blockDim.x)
        if (claim[r] == ~0ull) claim[r] = (0xFFFFFFFFull << 32) | r;
}

__global__ void k_perm_dplus(const uint32_t* __restrict__ dplus, const uint32_t* __restrict__ pi, uint32_t n,
                             uint32_t* __restrict__ nd) {
    for (uint32_t r = blockIdx.x * blockDim.x + threadIdx.x; r < n; r += gridDim.x * blockDim.x) {
        nd[pi[r]] = dplus[r];
        if (r == 0) nd[n] = 0;
    }
}

// Row r of the CSR becomes row pi[r] with every entry v mapped to pi[v].  One wavefront per row.
__global__ void k_relabel_rows(const int64_t* __restrict__ off, const uint32_t* __restrict__ col,
                               const uint32_t* __restrict__ pi, const int64_t* __restrict__ off2, uint32_t n,
                               uint32_t* __restrict__ col2) {
    const uint32_t lane = threadIdx.x & 63u;
    const uint32_t nwv = (gridDim.x * blockDim.x) >> 6;
    for (uint32_t r = (blockIdx.x * blockDim.x + threadIdx.x) >> 6; r < n; r += nwv) {
        const int64_t b = off[r];
        const uint32_t d = (uint32_t)(off[r + 1] - b);
        const int64_t b2 = off2[pi[r]];
        for (uint32_t j = lane; j < d; j += 64) col2[b2 + j] = pi[col[b + j]];
    }
}

__global__ void k_compose(uint32_t* __restrict__ rank, const uint32_t* __restrict__ pi, uint32_t n) {
    for (uint32_t x = blockIdx.x * blockDim.x + threadIdx.x; x < n; x += gridDim.x * blockDim.x) rank[x] = pi[rank[x]];
}

__global__ void k_scatter_u32(const uint32_t* __restrict__ in, const uint32_t* __restrict__ pi, uint32_t n,
                              uint32_t* __restrict__ out) {
    for (uint32_t r = blockIdx.x * blockDim.x + threadIdx.x; r < n; r += gridDim.x * blockDim.x) out[pi[r]] = in[r];
}

__global__ void k_gather(const unsigned long long* __restrict__ tv, const uint32_t* __restrict__ rank, uint32_t n,
                         const uint32_t* __restrict__ place, unsigned long long* __restrict__ out) {
    for (uint32_t x = blockIdx.x * blockDim.x + threadIdx.x; x < n; x += gridDim.x * blockDim.x) {
        const uint32_t r = rank[x];
        out[x] = tv[place ? rec_id(place[2 * (uint64_t)r]) : r];
    }
}

#define TC_TRY(expr)                        \
    do {                                    \
        hipError_t e_ = (expr);             \
        if (e_ != hipSuccess) return e_;    \
    } while (0)

}  // namespace

hipError_t fill_u32(void* p, uint32_t value, size_t words, hipStream_t stream) {
    if (words == 0) return hipSuccess;
    hipLaunchKernelGGL(k_fill_u32, dim3(grid_for(words)), dim3(kThreads), 0, stream, (uint32_t*)p, value, words);
    return hipGetLastError();
}

hipError_t gather_per_vertex(const unsigned long long* tv, const uint32_t* rank, uint32_t n, const uint32_t* place,
                             unsigned long long* out, hipStream_t stream) {
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_gather, dim3(grid_for(n)), dim3(kThreads), 0, stream, tv, rank, n, place, out);
    return hipGetLastError();
}

hipError_t clear_record_staging(unsigned long long* tv, const uint32_t* place, uint32_t n, hipStream_t stream) {
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_clear_record_starts, dim3(grid_for(n)), dim3(kThreads), 0, stream, tv, place, n);
    return hipGetLastError();
}

size_t prep_sort_tmp_bytes(uint32_t n, uint64_t m_in) {
    size_t best = 0, sz = 0;
    const uint32_t nb = id_bits(n);
    unsigned long long* k64 = nullptr;
    uint32_t* u32p = nullptr;
    if (sort_keys(nullptr, sz, k64, k64, (size_t)m_in, 0, 2 * nb, 0) == hipSuccess && sz > best) best = sz;
    sz = 0;
    {
        auto keys = rocprim::make_transform_iterator(rocprim::make_counting_iterator<uint64_t>(0),
                                                     CanonKey{u32p, u32p, n, nb, 0ull, nullptr});
        if (sort_keys(nullptr, sz, keys, k64, (size_t)m_in, 0, 2 * nb, 0) == hipSuccess && sz > best) best = sz;
    }
    sz = 0;
    if (sort_keys(nullptr, sz, k64, k64, (size_t)m_in, nb, 2 * nb, 0) == hipSuccess && sz > best) best = sz;
    sz = 0;
    if (sort_keys(nullptr, sz, u32p, u32p, (size_t)m_in, 0, nb < 32 ? nb + 1 : 32, 0) == hipSuccess && sz > best)
        best = sz;
    sz = 0;
    if (rocprim::radix_sort_pairs(nullptr, sz, u32p, u32p, rocprim::counting_iterator<uint32_t>(0), u32p,
                                  (size_t)n, 0, 32) == hipSuccess && sz > best) best = sz;
    sz = 0;
    {
        auto heads = rocprim::make_transform_iterator(rocprim::make_counting_iterator<uint64_t>(0),
                                                      HeadOutDegree{u32p, u32p, nullptr});
        if (rocprim::inclusive_scan(nullptr, sz, heads, k64, (size_t)m_in, rocprim::plus<unsigned long long>()) ==
                hipSuccess && sz > best) best = sz;
        sz = 0;
        if (rocprim::exclusive_scan(nullptr, sz, k64, k64, (unsigned long long)0, (size_t)place_chunks(n) + 1,
                                    rocprim::plus<unsigned long long>()) == hipSuccess && sz > best) best = sz;
        sz = 0;
        auto rheads = rocprim::make_transform_iterator(rocprim::make_counting_iterator<uint64_t>(0),
                                                       RecordHead{k64, u32p, nullptr, u32p, 1u, 1ull, nullptr});
        if (rocprim::inclusive_scan(nullptr, sz, rheads, k64, (size_t)m_in, rocprim::plus<unsigned long long>()) ==
                hipSuccess && sz > best) best = sz;
        sz = 0;
    }
    {
        size_t q = 0;
        if (rocprim::radix_sort_pairs(nullptr, q, k64, k64, rocprim::counting_iterator<uint32_t>(0), u32p, (size_t)n, 0,
                                      64) == hipSuccess && q > best) best = q;
    }
    sz = 0;
    if (sort_pairs(nullptr, sz, u32p, u32p, u32p, (size_t)n, degree_bits(n, m_in), 0) == hipSuccess && sz > best)
        best = sz;
    sz = 0;
    if (sort_pairs(nullptr, sz, u32p, u32p, u32p, (size_t)n, kScheduleBits, 0) == hipSuccess && sz > best) best = sz;
    sz = 0;
    int64_t* i64p = nullptr;
    if (rocprim::exclusive_scan(nullptr, sz, u32p, i64p, (unsigned long long)0, (size_t)n + 1,
                                rocprim::plus<unsigned long long>()) == hipSuccess && sz > best) best = sz;
    sz = 0;
    if (rocprim::radix_sort_pairs(nullptr, sz, k64, k64, rocprim::counting_iterator<uint32_t>(0), u32p,
                                  (size_t)n, 0, 42) == hipSuccess && sz > best) best = sz;
    return best;
}

// Relabel the oriented rank-space CSR into another order of hash ids (the orientation stays).
hipError_t relabel(uint32_t n, const GraphDev& g, const BuildTemp& t, const BatchIn* batch, uint32_t order,
                   uint64_t m_in, hipStream_t stream) {
    size_t tmp;
    const uint32_t wave_grid = std::min<uint32_t>(grid_for((uint64_t)n * 64), 8192u);
    if (order == 1) {
        hipLaunchKernelGGL(k_key_indegree, dim3(grid_for(n)), dim3(kThreads), 0, stream,
                           reinterpret_cast<const uint32_t*>(t.skey_a), t.dplus, n, t.rk_a);
        TC_TRY(hipGetLastError());
    } else {
        unsigned long long* wscan = t.keys_a;
        auto heads = rocprim::make_transform_iterator(rocprim::make_counting_iterator<uint64_t>(0),
                                                      HeadOutDegree{g.col, t.dplus, g.meta});
        tmp = t.sort_tmp_bytes;
        TC_TRY(rocprim::inclusive_scan(t.sort_tmp, tmp, heads, wscan, (size_t)m_in,
                                       rocprim::plus<unsigned long long>(), stream));
        hipLaunchKernelGGL(k_key_collective, dim3(grid_for(n)), dim3(kThreads), 0, stream, g.off, wscan, n, t.rk_a);
        TC_TRY(hipGetLastError());
        tmp = t.sort_tmp_bytes;
        TC_TRY(rocprim::radix_sort_pairs(t.sort_tmp, tmp, t.rk_a, t.rk_b, rocprim::counting_iterator<uint32_t>(0),
                                         t.order, (size_t)n, 0, 64, stream));
        uint32_t* posw = reinterpret_cast<uint32_t*>(t.skey_b);
        hipLaunchKernelGGL(k_rank, dim3(grid_for(n)), dim3(kThreads), 0, stream, t.order, n, posw);
        TC_TRY(hipGetLastError());
        TC_TRY(fill_u32(t.rk_a, 0xFFFFFFFFu, 2 * (size_t)n, stream));
        hipLaunchKernelGGL(k_claim, dim3(wave_grid), dim3(kThreads), 0, stream, g.off, g.col, posw, n, t.rk_a);
        TC_TRY(hipGetLastError());
        hipLaunchKernelGGL(k_key_claimed, dim3(grid_for(n)), dim3(kThreads), 0, stream, n, t.rk_a);
        TC_TRY(hipGetLastError());
    }
    tmp = t.sort_tmp_bytes;
    TC_TRY(rocprim::radix_sort_pairs(t.sort_tmp, tmp, t.rk_a, t.rk_b, rocprim::counting_iterator<uint32_t>(0),
                                     t.order, (size_t)n, 0, 64, stream));
    uint32_t* pi = t.deg;  // new id of every rank
    hipLaunchKernelGGL(k_rank, dim3(grid_for(n)), dim3(kThreads), 0, stream, t.order, n, pi);
    TC_TRY(hipGetLastError());
    uint32_t* nd = reinterpret_cast<uint32_t*>(t.skey_b);  // out-degrees by new id, [n + 1]
    hipLaunchKernelGGL(k_perm_dplus, dim3(grid_for(n)), dim3(kThreads), 0, stream, t.dplus, pi, n, nd);
    TC_TRY(hipGetLastError());
    tmp = t.sort_tmp_bytes;
    TC_TRY(rocprim::exclusive_scan(t.sort_tmp, tmp, nd, t.off2, (unsigned long long)0, (size_t)n + 1,
                                   rocprim::plus<unsigned long long>(), stream));
    uint32_t* col2 = reinterpret_cast<uint32_t*>(t.keys_b);
    hipLaunchKernelGGL(k_relabel_rows, dim3(wave_grid), dim3(kThreads), 0, stream, g.off, g.col, pi, t.off2, n, col2);
    TC_TRY(hipGetLastError());
    TC_TRY(hipMemcpyAsync(g.col, col2, 4 * (size_t)m_in, hipMemcpyDeviceToDevice, stream));
    TC_TRY(hipMemcpyAsync(g.off, t.off2, 8 * ((size_t)n + 1), hipMemcpyDeviceToDevice, stream));
    TC_TRY(hipMemcpyAsync(t.dplus, nd, 4 * ((size_t)n + 1), hipMemcpyDeviceToDevice, stream));
    hipLaunchKernelGGL(k_compose, dim3(grid_for(n)), dim3(kThreads), 0, stream, g.rank, pi, n);
    TC_TRY(hipGetLastError());
    if (batch) {
        TC_TRY(hipMemcpyAsync(t.order, g.gid, 4 * (size_t)n, hipMemcpyDeviceToDevice, stream));
        hipLaunchKernelGGL(k_scatter_u32, dim3(grid_for(n)), dim3(kThreads), 0, stream, t.order, pi, n, g.gid);
        TC_TRY(hipGetLastError());
    }
    return hipSuccess;
}

hipError_t prep_build(uint32_t n, uint64_t m_in, const uint32_t* src, const uint32_t* dst, const GraphDev& g,
                      const BuildTemp& t, const BinCaps& caps, const BatchIn* batch, hipStream_t stream) {
    const uint32_t nb = id_bits(n);
    const unsigned long long sentinel = (2 * nb >= 64) ? ~0ull : ((1ull << (2 * nb)) - 1);
    size_t tmp = t.sort_tmp_bytes;

    TC_TRY(fill_u32(g.meta, 0, sizeof(GraphMeta) / 4, stream));
    TC_TRY(fill_u32(t.deg, 0, (size_t)n + 1, stream));
    TC_TRY(fill_u32(t.dplus, 0, (size_t)n + 1, stream));

    // 1-2: canonical keys, sort (batches form the keys first: each sample's graph is searched for).
    tmp = t.sort_tmp_bytes;
    if (batch) {
        hipLaunchKernelGGL(k_canon_batch, dim3(grid_for(m_in)), dim3(kThreads), 0, stream, src, dst, m_in, n, nb,
                           sentinel, batch->voff, batch->eoff, batch->k, t.keys_a, g.meta);
        TC_TRY(hipGetLastError());
        TC_TRY(sort_keys(t.sort_tmp, tmp, t.keys_a, t.keys_b, (size_t)m_in, 0, 2 * nb, stream));
    } else {
        auto keys = rocprim::make_transform_iterator(rocprim::make_counting_iterator<uint64_t>(0),
                                                     CanonKey{src, dst, n, nb, sentinel, g.meta});
        TC_TRY(sort_keys(t.sort_tmp, tmp, keys, t.keys_b, (size_t)m_in, 0, 2 * nb, stream));
    }

    // 3: distinct edges and degree (lower ids in the run pass, upper ids from runs of the sorted upper
    // endpoints), rank in (degree, id) order (stable sort keeps ids ascending among equal degrees).
    {
        uint32_t* up_a = t.aux;
        uint32_t* up_b = t.aux + m_in;
        const uint64_t chunks = (m_in + kRunChunk - 1) / kRunChunk;  // one wavefront each (4 per block)
        hipLaunchKernelGGL(k_runs, dim3(grid_for(chunks * 64)), dim3(kThreads), 0, stream, t.keys_b, nb, m_in, sentinel,
                           up_a, t.deg, g.meta);
        TC_TRY(hipGetLastError());
        tmp = t.sort_tmp_bytes;
        TC_TRY(sort_keys(t.sort_tmp, tmp, up_a, up_b, (size_t)m_in, 0, nb < 32 ? nb + 1 : 32, stream));
        hipLaunchKernelGGL(k_degree, dim3(grid_for(m_in)), dim3(kThreads), 0, stream, up_b, m_in, g.meta, t.deg);
        TC_TRY(hipGetLastError());
    }
    uint32_t* deg_sorted = reinterpret_cast<uint32_t*>(t.skey_a);
    tmp = t.sort_tmp_bytes;
    TC_TRY(sort_pairs(t.sort_tmp, tmp, t.deg, deg_sorted, t.order, (size_t)n, degree_bits(n, m_in), stream));
    hipLaunchKernelGGL(k_rank, dim3(grid_for(n)), dim3(kThreads), 0, stream, t.order, n, g.rank);
    TC_TRY(hipGetLastError());
    if (batch) {
        hipLaunchKernelGGL(k_gid, dim3(grid_for(n)), dim3(kThreads), 0, stream, t.order, n, batch->voff, batch->k,
                           g.gid);
        TC_TRY(hipGetLastError());
    }

    // 4-5: orientation and CSR in rank space.
    if (!caps.scatter_csr) {
        // Sort the oriented keys by row only (the high nb bits; radix sort is stable, so each list keeps
        // the canonical-key order; lists need no order for hashing): rows come out contiguous.  The
        // sentinel's row bits exceed every valid row, so unused entries sort last.
        unsigned long long* okeys = t.keys_a;
        unsigned long long* osorted = reinterpret_cast<unsigned long long*>(t.aux);
        hipLaunchKernelGGL(k_orient_keys, dim3(grid_for(m_in)), dim3(kThreads), 0, stream, t.keys_b, nb, m_in, g.rank,
                           sentinel, okeys);
        TC_TRY(hipGetLastError());
        tmp = t.sort_tmp_bytes;
        TC_TRY(sort_keys(t.sort_tmp, tmp, okeys, osorted, (size_t)m_in, nb, 2 * nb, stream));
        hipLaunchKernelGGL(k_csr_runs, dim3(grid_for(m_in)), dim3(kThreads), 0, stream, osorted, nb, m_in, g.meta,
                           t.dplus, g.col);
        TC_TRY(hipGetLastError());
        tmp = t.sort_tmp_bytes;
        TC_TRY(rocprim::exclusive_scan(t.sort_tmp, tmp, t.dplus, g.off, (unsigned long long)0, (size_t)n + 1,
                                       rocprim::plus<unsigned long long>(), stream));
    } else {
        // Counting sort: out-degrees, offsets, then an atomic scatter (list order unspecified).
        hipLaunchKernelGGL(k_orient_count, dim3(grid_for(m_in)), dim3(kThreads), 0, stream, t.keys_b, nb, m_in,
                           sentinel, g.rank, t.dplus);
        TC_TRY(hipGetLastError());
        tmp = t.sort_tmp_bytes;
        TC_TRY(rocprim::exclusive_scan(t.sort_tmp, tmp, t.dplus, g.off, (unsigned long long)0, (size_t)n + 1,
                                       rocprim::plus<unsigned long long>(), stream));
        TC_TRY(fill_u32(t.deg, 0, (size_t)n + 1, stream));
        hipLaunchKernelGGL(k_orient_fill, dim3(grid_for(m_in)), dim3(kThreads), 0, stream, t.keys_b, nb, m_in,
                           sentinel, g.rank, g.off, t.deg, g.col);
        TC_TRY(hipGetLastError());
    }

    // 5b (optional): hash ids in another vertex order.
    if (caps.order) TC_TRY(relabel(n, g, t, batch, caps.order, m_in, stream));

    hipLaunchKernelGGL(k_narrow, dim3(grid_for((uint64_t)n + 1)), dim3(kThreads), 0, stream, g.off, (uint64_t)n + 1,
                       g.off32);
    TC_TRY(hipGetLastError());

    // 6: bins and largest-work-first order; W(u) from a scan of d+(col[e]).
    unsigned long long* wscan = reinterpret_cast<unsigned long long*>(t.keys_a);
    // 5c with it: records are placed first ({p(r), d+(r)} per rank), then the scan's gather of d+(v)
    // reads v's placement, whose p(v) goes into the records (the sorted oriented keys give each edge's
    // row; no relabelling or counting-sort build here).  Rows without edges get their header in
    // k_schedule.
    uint32_t* rec = (caps.records && !caps.order && !caps.scatter_csr) ? g.rec : nullptr;
    if (rec) {
        const uint64_t chunks = place_chunks(n);
        hipLaunchKernelGGL(k_place_size, dim3(grid_for(chunks + 1)), dim3(kThreads), 0, stream, g.off32, n,
                           t.place_sz);
        TC_TRY(hipGetLastError());
        tmp = t.sort_tmp_bytes;
        unsigned long long* cbase = t.place_sz + chunks + 1;
        TC_TRY(rocprim::exclusive_scan(t.sort_tmp, tmp, t.place_sz, cbase, (unsigned long long)0,
                                       (size_t)chunks + 1, rocprim::plus<unsigned long long>(), stream));
        uint2* place = reinterpret_cast<uint2*>(g.place);
        hipLaunchKernelGGL(k_place_write, dim3(grid_for(chunks + 1)), dim3(kThreads), 0, stream, g.off32, n,
                           cbase, place);
        TC_TRY(hipGetLastError());
        const unsigned long long mask = (nb >= 32) ? 0xFFFFFFFFull : ((1ull << nb) - 1);
        auto heads = rocprim::make_transform_iterator(
            rocprim::make_counting_iterator<uint64_t>(0),
            RecordHead{reinterpret_cast<const unsigned long long*>(t.aux), g.off32, place, rec, nb, mask, g.meta});
        tmp = t.sort_tmp_bytes;
        TC_TRY(rocprim::inclusive_scan(t.sort_tmp, tmp, heads, wscan, (size_t)m_in,
                                       rocprim::plus<unsigned long long>(), stream));
    } else {
        auto heads = rocprim::make_transform_iterator(rocprim::make_counting_iterator<uint64_t>(0),
                                                      HeadOutDegree{g.col, t.dplus, g.meta});
        tmp = t.sort_tmp_bytes;
        TC_TRY(rocprim::inclusive_scan(t.sort_tmp, tmp, heads, wscan, (size_t)m_in,
                                       rocprim::plus<unsigned long long>(), stream));
    }
    if (caps.pack_cap) {
        hipLaunchKernelGGL(k_pack_census, dim3(std::min(grid_for(n), 1024u)), dim3(kThreads), 0, stream, g.off, wscan,
                           n, caps, g.meta);
        TC_TRY(hipGetLastError());
    }
    // at most 1024 blocks: each block ends with a few global atomics on the same summary words
    uint32_t* skey = reinterpret_cast<uint32_t*>(t.skey_a);
    hipLaunchKernelGGL(k_schedule, dim3(std::min(grid_for(n), 1024u)), dim3(kThreads), 0, stream, g.off, wscan, n, caps, g.meta,
                       skey, rec, rec ? g.place : nullptr);
    TC_TRY(hipGetLastError());
    tmp = t.sort_tmp_bytes;
    TC_TRY(sort_pairs(t.sort_tmp, tmp, skey, reinterpret_cast<uint32_t*>(t.skey_b), g.items, (size_t)n, kScheduleBits,
                      stream));
    return hipSuccess;
}

}  // namespace tc
