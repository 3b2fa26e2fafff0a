// The counting kernels: vertex-centric hashing (paper Section 3, Algorithm 1)
// on the oriented rank-space CSR, for gfx950.
//
// Two persistent launches.  A "group" owns one vertex u at a time:
//   * large-vertex launch (one workgroup of 16 wavefronts per CU, all of its
//     LDS): bin 0, out-degree too large for any LDS table, table in a
//     global-memory region of the workgroup; bin 1, table in the LDS;
//   * main launch: bin 2, the whole workgroup with the table in its LDS;
//     bin 3, one 64-lane wavefront with the table in its slice of the LDS;
//     bin 4, light vertices 4 (16 lanes each) or 2 (32 lanes each) to a
//     wavefront, each table in a quarter of the slice.
// This is the degree-aware resource assignment of Section 4.3 (a CTA for
// large vertices, a warp for small ones; vertices with fewer than two
// out-neighbours skipped), with atomic dynamic work fetching (one vertex per
// fetch for workgroups, `chunk` vertices per fetch for wavefronts).
//
// Per vertex u (d = d+(u) out-neighbours):
//   build  : buckets B (power of two), S slots each, len[] counters.  Every
//            w in N+(u) takes a slot with an atomic add on len[hash(w)]
//            (Algorithm 1, hashTableConstruction); a full bucket passes the
//            element on to the next bucket (the linear-probing overflow rule
//            of Section 3.2).  Slots of a bucket are contiguous, so one
//            8- or 16-byte LDS read fetches a whole bucket; unused slots hold
//            0xFFFFFFFF, which ends a probe.
//   records: for each out-neighbour v_k, its 2-hop list start and the
//            inclusive prefix of d+(v_k) (virtual combination, Section 4.2):
//            flattened 2-hop index i belongs to the first k whose prefix
//            exceeds i, at local offset i - exclusive prefix.
//   probe  : lanes walk the flattened 2-hop index space 64 at a time, so
//            consecutive lanes read consecutive words of the same list
//            (coalesced); each lane keeps a cursor (k, end, base) that only
//            moves forward.  Each w is looked up in its bucket (Algorithm 1,
//            intersection / linearSearch); a hit is one triangle (u, v_k, w).
//            A lookup that must continue to the next bucket is parked in
//            registers and resumed with other parked lookups, so chains never
//            stall a whole wavefront (LDS tables; the global-memory tables
//            walk chains lane by lane).
//   reduce : each lane counts its hits; the wavefront sums them with DPP lane
//            moves, the workgroup in LDS, and one atomic per workgroup adds
//            the launch's share to the total.  For a batch of graphs each
//            vertex's hits go to its graph's total instead.
// Per-vertex mode adds, per hit, an LDS tally on the matched slot (its
// element is the triangle's w) and a register tally for v_k (added to an LDS
// tally when the lane leaves v_k's list); after the probe, u's hits and the
// non-zero tallies go to the per-vertex array with one global atomic each.
#include <type_traits>

#include "tc_internal.h"
#include "tc_wave.h"

namespace tc {
namespace {

__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

template <bool WG>
__device__ __forceinline__ void group_sync() {
    if constexpr (WG) __syncthreads();
    else wave_sync();
}

typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

template <int S>
struct Bucket {
    uint32_t v[S];
};

template <int S>
__device__ __forceinline__ Bucket<S> read_bucket(const uint32_t* slots, uint32_t b) {
    Bucket<S> r;
    if constexpr (S == 1) {
        r.v[0] = slots[b];
    } else if constexpr (S == 2) {
        const u32x2 x = *reinterpret_cast<const u32x2*>(slots + 2 * b);
        r.v[0] = x.x; r.v[1] = x.y;
    } else {
        const u32x4 x = *reinterpret_cast<const u32x4*>(slots + 4 * b);
        r.v[0] = x.x; r.v[1] = x.y; r.v[2] = x.z; r.v[3] = x.w;
    }
    return r;
}

// Bucket contains w (bitwise OR of compares, so the lane mask stays a
// compare result and a ballot of it is a plain scalar OR).
template <int S>
__device__ __forceinline__ bool bucket_has(const Bucket<S>& v, uint32_t w) {
    bool f = v.v[0] == w;
#pragma unroll
    for (int j = 1; j < S; ++j) f = f | (v.v[j] == w);
    return f;
}

// Lanes whose bucket contains their w, as a wave mask.  Each compare is
// balloted on its own so the masks stay scalar (a ballot of an OR of
// compares would be rebuilt through vector registers).
template <int S>
__device__ __forceinline__ unsigned long long ballot_has(const Bucket<S>& v, uint32_t w) {
    unsigned long long m = __ballot(v.v[0] == w);
#pragma unroll
    for (int j = 1; j < S; ++j) m |= __ballot(v.v[j] == w);
    return m;
}

// This lane's bit of a wave mask, as a lane predicate (the mask itself is the predicate: no vector
// shift, and, or compare of the 64-bit value).
__device__ __forceinline__ bool lane_in(unsigned long long mask) {
    return __builtin_amdgcn_inverse_ballot_w64(mask);
}

// Byte offset of w within a bucket that contains it (j * 4).
template <int S>
__device__ __forceinline__ uint32_t bucket_pos4(const Bucket<S>& v, uint32_t w) {
    uint32_t j4 = 4u * (S - 1);
#pragma unroll
    for (int j = S - 2; j >= 0; --j) j4 = (v.v[j] == w) ? 4u * j : j4;
    return j4;
}

// Index of w within a bucket that contains it.
template <int S>
__device__ __forceinline__ uint32_t bucket_pos(const Bucket<S>& v, uint32_t w) {
    uint32_t j0 = S - 1;
#pragma unroll
    for (int j = S - 2; j >= 0; --j) j0 = (v.v[j] == w) ? (uint32_t)j : j0;
    return j0;
}

// One bucket step of a lookup: hit (slot index in *s), or "continue at the
// next bucket" (bucket full and w not in it), or a miss (neither).
template <int S>
__device__ __forceinline__ void bucket_step(const Bucket<S>& v, uint32_t w, uint32_t b, bool act, bool* hit,
                                            bool* cont, uint32_t* s) {
    bool found = false;
    uint32_t j0 = 0;
#pragma unroll
    for (int j = S - 1; j >= 0; --j)
        if (v.v[j] == w) { found = true; j0 = (uint32_t)j; }
    *hit = act && found;
    *cont = act && !found && v.v[S - 1] != kEmpty;
    *s = b * S + j0;
}

// Full lookup by walking the chain lane by lane (used for global-memory tables).
template <int S, int HK>
__device__ __forceinline__ bool lookup_chain(const uint32_t* slots, uint32_t w, uint32_t B, uint32_t* slot) {
    uint32_t b = hash_of<HK>(w, B);
    for (uint32_t t = 0; t < B; ++t) {
        const Bucket<S> v = read_bucket<S>(slots, b);
        bool hit, cont;
        bool act = true;
        bucket_step<S>(v, w, b, act, &hit, &cont, slot);
        if (hit) return true;
        if (!cont) return false;
        b = (b + 1) & (B - 1);
    }
    return false;
}

constexpr int kUnroll = 4;  // chunks per load group (the filter code spells out four)
static_assert(kUnroll == 4, "filter_group initialises four lane masks");

struct Probe {
    const uint32_t* __restrict__ col;
    const uint32_t* slots;
    const u32x2* P;
    uint32_t* tslot;  // per-slot hit tallies (per-vertex mode): the slot's element is the triangle's w
    uint32_t* tally;  // per-out-neighbour hit tallies (per-vertex mode): v_k of the triangle
    uint32_t B;
    const uint32_t* filt;  // filter bit vector of fbits bits (LDS tables)
    uint32_t fbits;
    uint32_t flog;         // log2 of the filter's words
    uint32_t* queue;       // this wavefront's queue: entries {id, k}, kQueueEntries then 64 dummies
};

// This lane's position among the set lanes of a wave mask (number of set lanes below it).
__device__ __forceinline__ uint32_t lanes_below(unsigned long long m) {
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}

template <int S, bool PV>
__device__ __forceinline__ void tally_hit(const Probe& pr, uint32_t s, uint32_t k) {
    if constexpr (PV) {
        atomicAdd(&pr.tslot[s], 1u);
        atomicAdd(&pr.tally[k], 1u);
    }
}

// Slot tally of a hit in bucket b at byte offset j4 of the bucket.
template <int S>
__device__ __forceinline__ void tally_slot4(const Probe& pr, uint32_t b, uint32_t j4) {
    atomicAdd(reinterpret_cast<uint32_t*>(reinterpret_cast<char*>(pr.tslot) + b * (4u * S) + j4), 1u);
}

// Probe the flattened 2-hop range [lo, hi) of the current vertex with one
// wavefront, walking it in chunks of 64 consecutive indices (consecutive
// lanes read consecutive words of a list).  Returns the hits (uniform).
//
// Each lane keeps a forward-only cursor as a position in col: `pos` (the
// word it reads next) and `lim` (end of the current list).  A chunk step is
// pos += 64; when pos passes lim the lane moves on to the next list(s) of the
// virtual combination, carrying the overshoot.  With col under 4 GiB the
// position is kept as a 32-bit byte offset and loads take the scalar-base
// form (no 64-bit address arithmetic per chunk).
//
// Filter and queue: most probes miss (a few percent hit on skewed graphs), so
// every probed id first tests its bit of the table's filter (one 4-byte LDS
// read); only ids whose bit is set (the hits and a few percent of the misses)
// are appended to the wavefront's queue in LDS.  When the queue cannot take a
// chunk's survivors, its entries are looked up together, one per lane, in the
// bucket table (Algorithm 1's intersection step), so the full lookup runs on a
// nearly full wavefront instead of on every chunk.  The queue keeps the order
// of the flattened index, so its entries' out-neighbour indices k are
// non-decreasing: per-vertex tallies of v_k are added once per run of equal k.
//
// A lookup whose bucket is full without a match must continue at the next
// bucket.  Instead of walking that chain while the other 63 lanes wait, the
// lane parks it (w, bucket[, k]) in registers; parked lookups take one
// bucket step together when 32 lanes hold one, when a lane that holds one
// needs to park another, and at the end of the range.
//
// Loads for the next group of kUnroll chunks are issued before the current
// group is filtered (two register sets used in turn); leftover chunks are
// taken in groups of up to kUnroll and the ragged last chunk with a lane
// predicate.
template <int S, bool PV, int HK, bool WIDE>
__device__ __forceinline__ unsigned long long probe_range_lds(const Probe& pr, uint32_t d, uint32_t lo, uint32_t hi,
                                                              int lane) {
    if (lo >= hi) return 0;
    const uint32_t bmask = pr.B - 1;
    uint32_t hits = 0;  // uniform (W < 2^32)
    // Cursor: record k holds the lane's next flattened index ii; pos = base_k + ii.
    uint32_t k, pos, lim, base;
    {
        const uint32_t ii0 = lo + (uint32_t)lane;
        const uint32_t key = ii0 < hi ? ii0 : hi - 1;
        k = vc_owner(d, key, [&](uint32_t j) { return pr.P[j].x; });
        const u32x2 rec = pr.P[k];
        base = rec.y;
        pos = base + ii0;
        lim = base + rec.x;
    }
    // 32-bit byte offsets (narrow) or word indices with 64-bit addressing (wide).
    const uint32_t step = WIDE ? 64u : 256u;
    uint32_t cur = WIDE ? pos : pos * 4u, end = WIDE ? lim : lim * 4u;

    auto advance = [&]() {  // cur >= end: move to the record holding the lane's index
        const uint32_t ii = (WIDE ? cur : cur >> 2) - base;
        uint32_t e;
        do {
            ++k;
            const u32x2 rec = pr.P[k];
            e = rec.x;
            base = rec.y;
        } while (ii >= e);
        cur = WIDE ? base + ii : (base + ii) * 4u;
        end = WIDE ? base + e : (base + e) * 4u;
    };
    auto load = [&]() -> uint32_t {
        if constexpr (WIDE) return pr.col[cur];
        else return *reinterpret_cast<const uint32_t*>(reinterpret_cast<const char*>(pr.col) + cur);
    };

    // Parked lookups: word, bucket (and k in per-vertex mode), mask of lanes holding one.
    uint32_t pw = 0, pb = 0, pk = 0;
    unsigned long long pm = 0;

    auto step_parked = [&]() {
        const unsigned long long mine = pm;
        const uint32_t b = (pb + 1) & bmask;
        const Bucket<S> v = read_bucket<S>(pr.slots, b);
        const unsigned long long hm = ballot_has<S>(v, pw) & mine;
        const unsigned long long cmask = __ballot(v.v[S - 1] != kEmpty) & mine & ~hm;
        hits += (uint32_t)__popcll(hm);
        if constexpr (PV) {
            if (lane_in(hm)) {
                tally_slot4<S>(pr, b, bucket_pos4<S>(v, pw));
                atomicAdd(&pr.tally[pk], 1u);
            }
        }
        pb = lane_in(cmask) ? b : pb;
        pm = cmask;
    };

    // Look up the qn queued ids (lane i takes entry i) in the bucket table.
    uint32_t qn = 0;  // uniform: queued entries
    u32x2* const queue = reinterpret_cast<u32x2*>(pr.queue);
    auto flush = [&]() {
        wave_sync();  // the queue writes of every lane are visible
        const bool act = (uint32_t)lane < qn;
        const unsigned long long am = qn >= 64u ? ~0ull : ((1ull << qn) - 1ull);
        uint32_t w = 0, kk = 0;
        {
            const u32x2 e = queue[lane];  // entries past qn are stale or dummies: masked off by am
            w = e.x;
            if constexpr (PV) kk = e.y;
        }
        const uint32_t b = hash_of<HK>(w, pr.B);
        const Bucket<S> v = read_bucket<S>(pr.slots, b);
        const unsigned long long hm = ballot_has<S>(v, w) & am;
        const unsigned long long cm = __ballot(v.v[S - 1] != kEmpty) & am & ~hm;
        hits += (uint32_t)__popcll(hm);
        if constexpr (PV) {
            const bool hit = lane_in(hm);
            if (hit) tally_slot4<S>(pr, b, bucket_pos4<S>(v, w));
            // tally[k] += hits of each run of equal k: the run's last lane adds the hits up to and
            // including it, the run's first lane subtracts the hits below it (modulo 2^32).
            // k of the lanes below and above (wave_shr:1 / wave_shl:1 lane moves; the end lanes get ~0)
            const uint32_t kprev = (uint32_t)__builtin_amdgcn_update_dpp(-1, (int)kk, 0x138, 0xf, 0xf, false);
            const uint32_t knext = (uint32_t)__builtin_amdgcn_update_dpp(-1, (int)kk, 0x130, 0xf, 0xf, false);
            const uint32_t below = lanes_below(hm);
            const bool first = act && (lane == 0 || kprev != kk);
            const bool last = act && ((uint32_t)lane + 1u == qn || knext != kk);
            const uint32_t upto = below + (hit ? 1u : 0u);
            if (last && upto) atomicAdd(&pr.tally[kk], upto);
            if (first && below) atomicSub(&pr.tally[kk], below);
        }
        if (cm) {
            while (cm & pm) step_parked();
            const bool cont = lane_in(cm);
            pw = cont ? w : pw;
            pb = cont ? b : pb;
            if constexpr (PV) pk = cont ? kk : pk;
            pm |= cm;
            if (__builtin_amdgcn_readfirstlane((uint32_t)__popcll(pm)) >= 32u) step_parked();
        }
        wave_sync();  // every lane has read its entry before the queue is refilled
        qn = 0;
    };

    // A group of up to kUnroll chunks (lanes in am[j]) through the filter: the filter words of all
    // chunks are read first, then the survivors go to the queue in chunk order (looked up first
    // when they would overflow it).  Every lane writes: a survivor to its queue position, any other
    // lane to its own dummy entry.
    auto append = [&](const unsigned long long sm, uint32_t w, uint32_t kk) {
        const uint32_t at = lane_in(sm) ? qn + lanes_below(sm) : kQueueEntries + (uint32_t)lane;
        if constexpr (PV) queue[at] = u32x2{w, kk};
        else queue[at].x = w;
        qn += (uint32_t)__popcll(sm);
    };
    auto filter_group = [&](const uint32_t (&w)[kUnroll], const uint32_t (&kk)[kUnroll],
                            const unsigned long long (&am)[kUnroll], uint32_t gcount) {
        uint32_t fw[kUnroll];
#pragma unroll
        for (int j = 0; j < kUnroll; ++j) {
            uint32_t word;
            if constexpr (HK == 0) word = __builtin_amdgcn_ubfe(w[j], 5u, pr.flog);  // bits [5, 5 + flog) of the id
            else word = hash_of<HK>(w[j], pr.fbits) >> 5;
            fw[j] = (uint32_t)j < gcount ? pr.filt[word] : 0u;
        }
        unsigned long long sm[kUnroll];
        uint32_t tot = 0;
#pragma unroll
        for (int j = 0; j < kUnroll; ++j) {
            uint32_t bit;
            if constexpr (HK == 0) bit = __builtin_amdgcn_ubfe(fw[j], w[j], 1u);  // the offset takes w's low 5 bits
            else bit = (fw[j] >> (hash_of<HK>(w[j], pr.fbits) & 31u)) & 1u;
            sm[j] = __builtin_amdgcn_ballot_w64(bit != 0u) & am[j];
            tot += (uint32_t)__popcll(sm[j]);
        }
        if (tot == 0) return;
        if (qn + tot > kQueueEntries) flush();
        if (tot <= kQueueEntries) {
#pragma unroll
            for (int j = 0; j < kUnroll; ++j) append(sm[j], w[j], kk[j]);
        } else {  // more survivors than the queue holds: chunk by chunk
#pragma unroll
            for (int j = 0; j < kUnroll; ++j) {
                if (qn + (uint32_t)__popcll(sm[j]) > kQueueEntries) flush();
                append(sm[j], w[j], kk[j]);
            }
        }
    };

    // Full chunk: every lane active.
    auto fetch = [&](uint32_t& w, uint32_t& kk) {
        const unsigned long long adv = __builtin_amdgcn_ballot_w64(cur >= end);
        if (adv) {  // uniform test first: most chunks need no lane to advance
            if (lane_in(adv)) advance();
        }
        w = load();
        if constexpr (PV) kk = k;
        cur += step;
    };
    const unsigned long long all[kUnroll] = {~0ull, ~0ull, ~0ull, ~0ull};

    const uint32_t nfull = (hi - lo) >> 6;
    uint32_t c = 0;
    if (nfull >= 2u * kUnroll) {
        uint32_t wa[kUnroll], ka[kUnroll], wb[kUnroll], kb[kUnroll];
#pragma unroll
        for (int j = 0; j < kUnroll; ++j) { ka[j] = 0; kb[j] = 0; fetch(wa[j], ka[j]); }
        c = kUnroll;
        // invariant: group A (fetched) is pending; c chunks fetched
        while (c + 2u * kUnroll <= nfull) {
#pragma unroll
            for (int j = 0; j < kUnroll; ++j) fetch(wb[j], kb[j]);
            filter_group(wa, ka, all, kUnroll);
#pragma unroll
            for (int j = 0; j < kUnroll; ++j) fetch(wa[j], ka[j]);
            filter_group(wb, kb, all, kUnroll);
            c += 2u * kUnroll;
        }
        filter_group(wa, ka, all, kUnroll);
    }
    // Remaining chunks (leftover full ones, then the ragged last one, whose lanes past hi sit out) in
    // groups of up to kUnroll: every load of a group is issued before the group is filtered.
    uint32_t left = nfull - c + ((lo + (nfull << 6) < hi) ? 1u : 0u);
    while (left) {
        const uint32_t gcount = left < (uint32_t)kUnroll ? left : (uint32_t)kUnroll;
        uint32_t w[kUnroll], kk[kUnroll];
        unsigned long long am[kUnroll];
#pragma unroll
        for (int j = 0; j < kUnroll; ++j) {
            w[j] = 0;
            kk[j] = 0;
            am[j] = 0;
            if ((uint32_t)j < gcount) {
                if (c < nfull) {
                    fetch(w[j], kk[j]);
                    am[j] = ~0ull;
                    ++c;
                } else {
                    const bool act = lo + (nfull << 6) + (uint32_t)lane < hi;
                    if (act) {
                        if (cur >= end) advance();
                        w[j] = load();
                    }
                    kk[j] = k;
                    am[j] = __ballot(act);
                }
            }
        }
        filter_group(w, kk, am, gcount);
        left -= gcount;
    }
    if (qn) flush();
    while (pm) step_parked();
    return hits;
}

// The same walk with a per-lane cursor and lane-by-lane chain lookups, for
// tables in global memory (bin 0: too large for any LDS table).
template <int S, bool PV, int HK>
__device__ __forceinline__ unsigned long long probe_range_global(const Probe& pr, uint32_t d, uint32_t lo,
                                                                 uint32_t hi, int lane) {
    unsigned long long hits = 0;
    if (lo >= hi) return 0;
    uint32_t i = lo + (uint32_t)lane;
    uint32_t k = 0, end = 0, base = 0;
    if (i < hi) {
        k = vc_owner(d, i, [&](uint32_t j) { return pr.P[j].x; });
        const u32x2 rec = pr.P[k];
        end = rec.x;
        base = rec.y;
    }
    for (; i - (uint32_t)lane < hi; i += 64u) {
        bool hit = false;
        uint32_t s = 0;
        if (i < hi) {
            while (i >= end) {
                ++k;
                const u32x2 rec = pr.P[k];
                end = rec.x;
                base = rec.y;
            }
            const uint32_t w = pr.col[(uint32_t)(base + i)];
            hit = lookup_chain<S, HK>(pr.slots, w, pr.B, &s);
        }
        hits += (unsigned long long)__popcll(__ballot(hit));
        if (hit) tally_hit<S, PV>(pr, s, k);
    }
    return hits;
}

template <int S, bool PV, int HK, bool DEFER>
__device__ __forceinline__ unsigned long long probe_range(const Probe& pr, uint32_t d, uint32_t lo, uint32_t hi,
                                                          int lane, bool wide) {
    if constexpr (DEFER) {
        if (wide) return probe_range_lds<S, PV, HK, true>(pr, d, lo, hi, lane);
        return probe_range_lds<S, PV, HK, false>(pr, d, lo, hi, lane);
    } else {
        return probe_range_global<S, PV, HK>(pr, d, lo, hi, lane);
    }
}

// Process vertex u with a group of `gsz` lanes (one wavefront, or the workgroup when WG).
// Subwave intra-vertex assignment (the alternative to virtual combination that Section 4.2 compares
// against): the wavefront is cut into groups of `sw` lanes (sw = 64: one list per wavefront, the
// warp-centric baseline), global group gi of gn takes the out-neighbour records k = gi, gi + gn, ...,
// and its lanes walk N+(v_k) with stride sw, each lane looking its element up along the bucket chain.
// Instantiated in kernels of its own, so the default kernels carry none of it.
template <int S, bool PV, int HK>
__device__ __forceinline__ unsigned long long probe_subwave(const Probe& pr, uint32_t d, uint32_t gi0, uint32_t gn,
                                                         uint32_t sw, int lane) {
    const uint32_t sub = (uint32_t)lane / sw, in = (uint32_t)lane % sw, per_wave = 64u / sw;
    uint32_t hits = 0;
    for (uint32_t k0 = gi0 * per_wave; k0 < d; k0 += gn * per_wave) {  // uniform: the wavefront's groups
        const uint32_t k = k0 + sub;
        uint32_t len = 0, start = 0;
        if (k < d) {
            const uint32_t excl = k ? pr.P[k - 1].x : 0u;
            const u32x2 rec = pr.P[k];
            len = rec.x - excl;
            start = rec.y + excl;
        }
        for (uint32_t t = in; t < len; t += sw) {
            const uint32_t w = pr.col[(uint64_t)start + t];
            uint32_t slot;
            if (lookup_chain<S, HK>(pr.slots, w, pr.B, &slot)) {
                ++hits;
                if constexpr (PV) {
                    atomicAdd(&pr.tslot[slot], 1u);
                    atomicAdd(&pr.tally[k], 1u);
                }
            }
        }
    }
    return wave_sum(hits);
}

struct NoMid {
    __device__ void operator()() const {}
};

// 2-hop list of vertex w: col[start, start + len).  Record layout: w is a record id (its position
// p = rec_id(w)), the length heads the record and the list follows it in the same line; otherwise w
// is a rank and the bounds come from the offsets (a line of their own).
__device__ __forceinline__ void list_of(const CountArgs& a, uint32_t w, uint32_t& start, uint32_t& len) {
    if (a.rec) {
        const uint32_t p = rec_id(w);
        len = a.rec[p];
        start = p + 1u;
    } else {
        start = a.off[w];
        len = a.off[w + 1] - start;
    }
}

// Table owner u (a rank) as the lists name it (its record id, or u), and where its own list
// starts in col.
__device__ __forceinline__ uint32_t own_id(const CountArgs& a, uint32_t u) {
    return a.rec ? rec_id(a.place[2u * u]) : u;
}
__device__ __forceinline__ uint32_t own_start(const CountArgs& a, uint32_t u) {
    return a.rec ? a.place[2u * u] + 1u : a.off[u];
}

// u's list is col[beg, beg + d) (uniform values).  With `pre` (one wavefront, d <= 64; uniform) the
// lane's list element and that element's list (start, length) were loaded by the caller (xw, xo, xl).
// `mid` runs after the table is built and before the probe (the caller issues its next loads there).
template <int S, bool PV, int HK, bool WG, bool DEFER, typename Mid = NoMid, bool SW = false>
__device__ __forceinline__ void process(const CountArgs& a, uint32_t u, int64_t beg, uint32_t d, uint32_t* tbl,
                                        uint64_t avail, int gl, int gsz, int gwave, int gnw, int lane,
                                        uint32_t* s_wsum, unsigned long long& acc, uint32_t* queue,
                                        bool pre = false, uint32_t xw = 0, uint32_t xo = 0, uint32_t xl = 0,
                                        Mid mid = Mid{}, uint32_t part = 0, uint32_t parts = 1) {
    gwave = __builtin_amdgcn_readfirstlane(gwave);
    // LDS tables walked by virtual combination carry a filter (the global-memory tables and the
    // subwave modes look every id up along its chain).
    constexpr bool FILT = DEFER && !SW;
    const Geometry g = geometry_fit(d, S, a.lrecip, PV, (uint32_t)avail, FILT);
    uint32_t* slots = tbl;
    uint32_t* len = tbl + g.o_len;
    u32x2* P = reinterpret_cast<u32x2*>(tbl + g.o_P);
    uint32_t* tslot = tbl + g.o_tslot;
    uint32_t* tally = tbl + g.o_tally;
    uint32_t* filt = tbl + g.o_filt;
    const uint32_t fwords = g.fbits / 32u;

    for (uint32_t x = gl; x < g.B * S; x += gsz) slots[x] = kEmpty;
    for (uint32_t x = gl; x < g.B; x += gsz) len[x] = 0;
    if constexpr (PV) {
        for (uint32_t x = gl; x < g.B * S; x += gsz) tslot[x] = 0;
        for (uint32_t x = gl; x < d; x += gsz) tally[x] = 0;
    }
    if constexpr (FILT)
        for (uint32_t x = gl; x < fwords; x += gsz) filt[x] = 0;
    group_sync<WG>();

    // Build the table of N+(u) (and its filter); record each out-neighbour's 2-hop list (length, start).
    auto insert = [&](uint32_t w) {
        uint32_t b = hash_of<HK>(w, g.B), pos;
        for (;;) {
            pos = atomicAdd(&len[b], 1u);
            if (pos < (uint32_t)S) break;
            b = (b + 1) & g.mask;
        }
        slots[b * S + pos] = w;
        if constexpr (FILT) {
            const uint32_t f = hash_of<HK>(w, g.fbits);
            atomicOr(&filt[f >> 5], 1u << (f & 31u));
        }
    };
    if (!WG && pre) {
        if ((uint32_t)gl < d) {
            insert(xw);
            P[gl] = u32x2{xl, xo};
        }
    } else {
        for (uint32_t p = gl; p < d; p += gsz) {
            const uint32_t w = a.col[beg + p];
            insert(w);
            uint32_t st, ln;
            list_of(a, w, st, ln);
            P[p] = u32x2{ln, st};
        }
    }
    group_sync<WG>();

    // Inclusive prefix of the 2-hop lengths; base = start - exclusive prefix (mod 2^32).
    uint32_t carry = 0;
    for (uint32_t t0 = 0; t0 < d; t0 += gsz) {
        const uint32_t p = t0 + gl;
        u32x2 r = u32x2{0u, 0u};
        if (p < d) r = P[p];
        uint32_t incl = wave_incl_scan(r.x), tot;
        if constexpr (WG) {
            if (lane == 63) s_wsum[gwave] = incl;
            __syncthreads();
            uint32_t pre = 0;
            tot = 0;
            for (int w = 0; w < gnw; ++w) {
                const uint32_t t = s_wsum[w];
                if (w < gwave) pre += t;
                tot += t;
            }
            __syncthreads();
            incl += pre;
        } else {
            tot = (uint32_t)__builtin_amdgcn_readlane((int)incl, 63);
        }
        if (p < d) {
            const uint32_t e = carry + incl;
            P[p] = u32x2{e, r.y - (e - r.x)};
        }
        carry += tot;
    }
    group_sync<WG>();

    mid();

    // Probe: the group's wavefronts split [0, W) into contiguous ranges.
    const uint32_t W = __builtin_amdgcn_readfirstlane(carry);
    // With parts > 1 several groups take the same vertex, each its share of [0, W) (tallies and hits
    // are sums, so partial flushes add up).
    const uint32_t r = part * (uint32_t)gnw + (uint32_t)gwave, rn = parts * (uint32_t)gnw;
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)(((uint64_t)W * r) / rn));
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(((uint64_t)W * (r + 1)) / rn));
    const Probe pr{a.col, slots, P, tslot, tally, g.B, filt, g.fbits,
                   fwords ? 31u - (uint32_t)__builtin_clz(fwords) : 0u, queue};
    unsigned long long hits;
    if constexpr (SW) hits = probe_subwave<S, PV, HK>(pr, d, r, rn, a.subwave, lane);
    else hits = probe_range<S, PV, HK, DEFER>(pr, d, lo, hi, lane, a.wide);
    if (a.gid) {
        if (lane == 0 && hits) atomicAdd(&a.totals[a.gid[u]], hits);
    } else {
        acc += hits;
    }

    if constexpr (PV) {
        if (lane == 0 && hits) atomicAdd(&a.tv[own_id(a, u)], hits);
        group_sync<WG>();
        for (uint32_t p = gl; p < d; p += gsz) {
            const uint32_t t = tally[p];
            if (t) atomicAdd(&a.tv[a.col[beg + p]], (unsigned long long)t);
        }
        for (uint32_t x = gl; x < g.B * S; x += gsz) {
            const uint32_t t = tslot[x];
            if (t) atomicAdd(&a.tv[slots[x]], (unsigned long long)t);
        }
    }
    group_sync<WG>();  // the table memory is reused by the next vertex
}

// Inclusive prefix sum within groups of G lanes (16 or 32) by DPP row moves.
template <int G>
__device__ __forceinline__ uint32_t group_incl_scan(uint32_t v) {
    v = dpp_add<0x111, 0xf>(v);  // row_shr:1
    v = dpp_add<0x112, 0xf>(v);  // row_shr:2
    v = dpp_add<0x114, 0xf>(v);  // row_shr:4
    v = dpp_add<0x118, 0xf>(v);  // row_shr:8
    if constexpr (G == 32) v = dpp_add<0x142, 0xa>(v);  // row_bcast:15 into rows 1 and 3
    return v;
}

// Several light vertices in one wavefront: group g = lane / G (64 / G groups) takes the vertex
// (ug, list at col[bg, bg + dg)) when `has`, with its table in the g-th part of the wavefront's LDS
// slice (`region` words each), and walks its own flattened 2-hop index space G lanes at a time
// (loads of kUnroll steps issued before they are looked up; each lookup reads its home bucket in
// straight-line code, and the chain is walked lane by lane only when some lane's home bucket is full
// without its id, which the lightly loaded tables of small vertices make rare: a loop around every
// lookup kept the scalar unit 73% busy at Erdos-Renyi 2^25 with the record layout).  The per-vertex fixed work
// (clears, build, records, reductions, flushes) is shared by the groups instead of paid per vertex.
template <int S, bool PV, int HK, int G>
__device__ __forceinline__ void process_packed(const CountArgs& a, uint32_t ug, uint32_t bg, uint32_t dg, bool has,
                                               uint32_t* slice, uint32_t region, int lane,
                                               unsigned long long& acc) {
    const uint32_t g = (uint32_t)lane / G, gl = (uint32_t)lane % G;
    const uint32_t d = has ? dg : 0u;
    const Geometry geo = geometry_fit(d, S, a.lrecip, PV, region);
    uint32_t* base = slice + g * (64u / G == 4 ? region : 2u * region);
    uint32_t* slots = base;
    uint32_t* len = base + geo.o_len;
    u32x2* P = reinterpret_cast<u32x2*>(base + geo.o_P);
    uint32_t* tslot = base + geo.o_tslot;
    uint32_t* tally = base + geo.o_tally;
    for (uint32_t x = gl; x < geo.B * S; x += G) slots[x] = kEmpty;
    for (uint32_t x = gl; x < geo.B; x += G) len[x] = 0;
    if constexpr (PV) {
        for (uint32_t x = gl; x < geo.B * S; x += G) tslot[x] = 0;
        if (gl < d) tally[gl] = 0;
    }
    wave_sync();
    // Build (one element per lane: d <= G) and the 2-hop records.
    uint32_t lv = 0, o0 = 0;
    if (gl < d) {
        const uint32_t w = a.col[(uint64_t)bg + gl];
        uint32_t b = hash_of<HK>(w, geo.B), pos;
        for (;;) {
            pos = atomicAdd(&len[b], 1u);
            if (pos < (uint32_t)S) break;
            b = (b + 1) & geo.mask;
        }
        slots[b * S + pos] = w;
        list_of(a, w, o0, lv);
    }
    const uint32_t incl = group_incl_scan<G>(lv);
    const uint32_t W = (uint32_t)__shfl((int)incl, (int)(g * G + G - 1), 64);
    if (gl < d) P[gl] = u32x2{incl, o0 - (incl - lv)};
    wave_sync();
    // Probe: step c covers indices c * G + gl of the group's range [0, W).
    uint32_t steps = (W + G - 1) / G, m = steps;
    for (int o = G; o < 64; o <<= 1) {
        const uint32_t t = (uint32_t)__shfl_xor((int)m, o, 64);
        m = t > m ? t : m;
    }
    const uint32_t maxsteps = __builtin_amdgcn_readfirstlane(m);
    uint32_t k = 0, cur = 0, end = 0, hits = 0;
    if (gl < W) {
        k = vc_owner(d, gl, [&](uint32_t j) { return P[j].x; });
        const u32x2 rec = P[k];
        cur = rec.y + gl;
        end = rec.y + rec.x;
    }
    for (uint32_t c0 = 0; c0 < maxsteps; c0 += kUnroll) {
        uint32_t w[kUnroll], kk[kUnroll];
        bool act[kUnroll];
#pragma unroll
        for (int j = 0; j < kUnroll; ++j) {
            const uint32_t ii = (c0 + j) * G + gl;
            act[j] = ii < W;
            w[j] = 0;
            kk[j] = k;
            if (act[j]) {
                while (cur >= end) {
                    ++k;
                    const u32x2 rec = P[k];
                    cur = rec.y + ii;
                    end = rec.y + rec.x;
                }
                w[j] = a.col[cur];
                kk[j] = k;
                cur += G;
            }
        }
#pragma unroll
        for (int j = 0; j < kUnroll; ++j) {
            // the home bucket for every lane in straight-line code; the chain walk only when some
            // lane's home bucket is full without its id (rare in these lightly loaded tables)
            const uint32_t b = hash_of<HK>(w[j], geo.B);
            const Bucket<S> v = read_bucket<S>(slots, b);
            bool hit, cont;
            uint32_t slot;
            bucket_step<S>(v, w[j], b, act[j], &hit, &cont, &slot);
            if (__builtin_amdgcn_ballot_w64(cont)) {
                if (cont) {
                    uint32_t bb = (b + 1) & geo.mask;
                    for (uint32_t t = 1; t < geo.B; ++t) {
                        const Bucket<S> u = read_bucket<S>(slots, bb);
                        bool c2;
                        bucket_step<S>(u, w[j], bb, true, &hit, &c2, &slot);
                        if (hit || !c2) break;
                        bb = (bb + 1) & geo.mask;
                    }
                }
            }
            if (hit) {
                ++hits;
                if constexpr (PV) {
                    atomicAdd(&tslot[slot], 1u);
                    atomicAdd(&tally[kk[j]], 1u);
                }
            }
        }
    }
    // Per-group totals (lane G - 1 of each group holds its group's sum).
    const uint32_t hs = group_incl_scan<G>(hits);
    const bool last = gl == G - 1;
    if (a.gid) {
        if (last && has && hs) atomicAdd(&a.totals[a.gid[ug]], (unsigned long long)hs);
    } else {
        uint32_t sum = 0;
#pragma unroll
        for (int q = 0; q < 64 / G; ++q) sum += (uint32_t)__builtin_amdgcn_readlane((int)hs, q * G + G - 1);
        acc += sum;
    }
    if constexpr (PV) {
        if (last && has && hs) atomicAdd(&a.tv[own_id(a, ug)], (unsigned long long)hs);
        wave_sync();
        if (gl < d) {
            const uint32_t t = tally[gl];
            if (t) atomicAdd(&a.tv[a.col[(uint64_t)bg + gl]], (unsigned long long)t);
        }
        for (uint32_t x = gl; x < geo.B * S; x += G) {
            const uint32_t t = tslot[x];
            if (t) atomicAdd(&a.tv[slots[x]], (unsigned long long)t);
        }
    }
    wave_sync();  // the slice is reused by the next vertex
}

// Workgroup-owned vertex: its list from the offsets, then process().
// Whether this launch counts the triangles owned by u (workload partitioning: u % shards == shard).
__device__ __forceinline__ bool in_shard(const CountArgs& a, uint32_t u) {
    return a.shards <= 1 || u % a.shards == a.shard;
}

// Several graphs in one launch (a.multi): the handle whose fetches of a bin hold the launch-wide
// fetch c is the last g < k with pre[g] <= c (pre: exclusive prefix over the handles of the bin's
// fetches, pre[0] = 0 <= c < pre[k]; a handle without fetches repeats its successor's value and is
// passed over).  A 64-way search by the whole wavefront, one round per factor of 64 in k.
__device__ __forceinline__ uint32_t find_graph(const uint32_t* pre, uint32_t k, uint32_t c, int lane) {
    uint32_t lo = 0, hi = k;  // pre[lo] <= c, and hi == k or pre[hi] > c
    while (hi - lo > 1) {
        const uint32_t step = (hi - lo + 63) / 64;
        const uint32_t p = lo + (uint32_t)lane * step;
        const unsigned long long ok = __ballot(p < hi && pre[p] <= c);  // lane 0: pre[lo] <= c
        lo += (uint32_t)(63 - __builtin_clzll(ok)) * step;
        hi = (lo + step < hi) ? lo + step : hi;
        lo = __builtin_amdgcn_readfirstlane(lo);
        hi = __builtin_amdgcn_readfirstlane(hi);
    }
    return lo;
}

// The launch-wide arguments with the per-graph fields of handle d.
__device__ __forceinline__ CountArgs graph_view(const CountArgs& a, const MultiDesc& d) {
    CountArgs v = a;
    v.meta = d.meta;
    v.off = d.off;
    v.col = d.col;
    v.items = d.items;
    v.gid = d.gid;
    v.totals = d.totals;
    v.total = d.totals;
    v.tv = a.multi->tv + d.tv0;
    v.wide = d.wide;
    return v;
}

// First item of bin `bin` in a graph's item list (the bins are stored one after another).
__device__ __forceinline__ uint32_t bin_base(const GraphMeta* m, uint32_t bin) {
    uint32_t b = 0;
    for (uint32_t i = 0; i < bin; ++i) b += m->bins[i];
    return b;
}

// Wavefront total of a multi-graph launch: hits of single graphs accumulate in `acc` while they
// belong to the same graph and go to that graph's total when the wavefront moves to another one.
struct AccSink {
    unsigned long long* dst = nullptr;
    __device__ __forceinline__ void to(unsigned long long* next, unsigned long long& acc, int lane) {
        if (next == dst) return;
        if (acc && dst && lane == 0) atomicAdd(dst, acc);
        acc = 0;
        dst = next;
    }
};

template <int S, bool PV, int HK, bool DEFER, bool SW = false>
__device__ __forceinline__ void process_wg(const CountArgs& a, uint32_t u, uint32_t* tbl, uint64_t avail, int tid,
                                           int wave, int nw, int lane, uint32_t* s_wsum, unsigned long long& acc,
                                           uint32_t* queue, uint32_t part = 0, uint32_t parts = 1) {
    u = __builtin_amdgcn_readfirstlane(u);
    if (!in_shard(a, u)) return;
    const int64_t beg = own_start(a, u);
    const uint32_t d = __builtin_amdgcn_readfirstlane(a.off[u + 1] - a.off[u]);
    process<S, PV, HK, true, DEFER, NoMid, SW>(a, u, beg, d, tbl, avail, tid, blockDim.x, wave, nw, lane, s_wsum, acc,
                                               queue, false, 0u, 0u, 0u, NoMid{}, part, parts);
}

// Tickets of a large-vertex bin of n vertices for `wgs` workgroups: when the bin has fewer vertices
// than workgroups, each vertex is split into `parts` tickets (consecutive), one per share of its work.
__device__ __forceinline__ uint32_t parts_for(uint32_t n, uint32_t wgs) {
    return (n && wgs > n) ? wgs / n : 1u;
}

// Sum of the workgroup's per-wavefront totals, one atomic per workgroup.
__device__ __forceinline__ void add_workgroup_total(const CountArgs& a, unsigned long long acc,
                                                    unsigned long long* s_acc, int tid, int lane, int wave, int nw) {
    if (lane == 0) s_acc[wave] = acc;
    __syncthreads();
    if (tid == 0) {
        unsigned long long sum = 0;
        for (int w = 0; w < nw; ++w) sum += s_acc[w];
        if (sum && a.total) atomicAdd(a.total, sum);
    }
}

// Large vertices (bins 0 and 1), launched before the main kernel with one
// workgroup per CU and the whole LDS: bin 1 tables fill the workgroup's LDS;
// bin 0 tables (too large for any LDS) live in global memory, one region per
// participating workgroup (the first hub_wgs workgroups).  The bin-1 vertices
// whose tables fit half a CU's LDS go to a second launch of the same kernel
// (hub_part 1) with half the LDS per workgroup, so two workgroups share a CU:
// one builds or clears its table while the other probes, with twice the
// wavefronts in flight to cover the list reads.
template <int S, bool PV, int HK, bool MULTI>
__global__ void __launch_bounds__(1024) __attribute__((amdgpu_waves_per_eu(6))) tc_hub_kernel(CountArgs a) {
    extern __shared__ __align__(16) uint32_t lds[];
    __shared__ uint32_t s_wsum[kMaxWaves];
    __shared__ unsigned long long s_acc[kMaxWaves];
    __shared__ uint32_t s_item;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, nw = blockDim.x >> 6;
    unsigned long long acc = 0;
    AccSink sink;
    // Bin-1 items [lo1, hi1) taken by this launch from queue head1: the full-LDS part (all of bin 1 in
    // multi-graph mode) with bin 0, or the half-LDS part alone.
    uint32_t n_hub, lo1 = 0, hi1, head1 = 1, base1 = 0;
    if constexpr (MULTI) {
        n_hub = a.multi->items_tot[0];
        hi1 = a.multi->items_tot[1];
    } else {
        n_hub = a.meta->bins[0];
        base1 = n_hub;  // bin 1 follows bin 0 in the item order
        hi1 = a.meta->big_full;
        if (a.hub_part) {
            n_hub = 0;
            lo1 = hi1;
            hi1 = a.meta->bins[1];
            head1 = kMidHead;
        }
    }
    const uint32_t n_big = hi1 - lo1;
    if (n_hub + n_big == 0) return;
    uint32_t* const queue = lds + a.table_words + (size_t)wave * kQueueWords;
    // Item j of bin `bin` (launch-wide index in multi-graph mode) with its graph's arguments.
    auto run = [&](uint32_t bin, uint32_t j, uint32_t* tbl, uint64_t avail, uint32_t part, uint32_t parts, auto wg) {
        if constexpr (MULTI) {
            const MultiHeader* H = a.multi;
            const uint32_t* pre = H->pre + (size_t)bin * (H->k + 1);
            const uint32_t g = find_graph(pre, H->k, j, lane);
            const MultiDesc& d = H->desc[g];
            const CountArgs v = graph_view(a, d);
            sink.to(d.totals, acc, lane);
            process_wg<S, PV, HK, decltype(wg)::value>(v, d.items[bin_base(d.meta, bin) + j - pre[g]], tbl, avail, tid,
                                                       wave, nw, lane, s_wsum, acc, queue, part, parts);
        } else {
            process_wg<S, PV, HK, decltype(wg)::value>(a, a.items[(bin ? base1 : 0u) + j], tbl, avail, tid, wave, nw,
                                                       lane, s_wsum, acc, queue, part, parts);
        }
    };

    if (blockIdx.x < a.hub_wgs && n_hub) {
        const unsigned long long hub_words = MULTI ? a.multi->hub_words : a.hub_words;
        uint32_t* gt = (MULTI ? a.multi->hub : a.hub_scratch) + (size_t)blockIdx.x * hub_words;
        const uint32_t parts = parts_for(n_hub, a.hub_wgs);
        for (;;) {
            if (tid == 0) s_item = atomicAdd(&a.heads[0 * kHeadStride], 1u);
            __syncthreads();
            const uint32_t t = s_item;
            __syncthreads();
            if (t >= n_hub * parts) break;
            run(0u, t / parts, gt, hub_words, t % parts, parts, std::false_type{});
        }
    }
    if (n_big) {
        const uint32_t parts = parts_for(n_big, gridDim.x);
        for (;;) {
            if (tid == 0) s_item = atomicAdd(&a.heads[head1 * kHeadStride], 1u);
            __syncthreads();
            const uint32_t t = s_item;
            __syncthreads();
            if (t >= n_big * parts) break;
            run(1u, lo1 + t / parts, lds, a.table_words, t % parts, parts, std::true_type{});
        }
    }
    if constexpr (MULTI) sink.to(nullptr, acc, lane);
    else add_workgroup_total(a, acc, s_acc, tid, lane, wave, nw);
}

// Everything else (bins 2-4): a persistent grid filling the GPU.  SW: subwave probe assignment;
// MULTI: the graphs come from a.multi.
template <int S, bool PV, int HK, bool SW, bool MULTI>
__global__ void __launch_bounds__(1024) __attribute__((amdgpu_waves_per_eu(6))) tc_count_kernel(CountArgs a) {
    extern __shared__ __align__(16) uint32_t lds[];
    __shared__ uint32_t s_wsum[kMaxWaves];
    __shared__ unsigned long long s_acc[kMaxWaves];
    __shared__ uint32_t s_item;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, nw = blockDim.x >> 6;
    unsigned long long acc = 0;
    AccSink sink;
    uint32_t n_before, n_wg, n_wave, n_pack;
    if constexpr (MULTI) {
        n_before = 0;  // items are found per graph
        n_wg = a.multi->items_tot[2];
        n_wave = a.multi->items_tot[3];
        n_pack = a.multi->items_tot[4];
    } else {
        n_before = a.meta->bins[0] + a.meta->bins[1];
        n_wg = a.meta->bins[2];
        n_wave = a.meta->bins[3];
        n_pack = a.meta->bins[4];
    }

    uint32_t* const queue = lds + a.table_words + (size_t)wave * kQueueWords;  // this wavefront's probe queue
    // Workgroup bin: the table fills the workgroup's table region.
    if (n_wg) {
        for (;;) {
            if (tid == 0) s_item = atomicAdd(&a.heads[2 * kHeadStride], 1u);
            __syncthreads();
            const uint32_t j = s_item;
            __syncthreads();
            if (j >= n_wg) break;
            if constexpr (MULTI) {
                const MultiHeader* H = a.multi;
                const uint32_t* pre = H->pre + 2u * (H->k + 1);
                const uint32_t g = find_graph(pre, H->k, j, lane);
                const MultiDesc& d = H->desc[g];
                const CountArgs v = graph_view(a, d);
                sink.to(d.totals, acc, lane);
                process_wg<S, PV, HK, true, SW>(v, d.items[bin_base(d.meta, 2) + j - pre[g]], lds, a.table_words, tid,
                                                wave, nw, lane, s_wsum, acc, queue);
            } else {
                process_wg<S, PV, HK, true, SW>(a, a.items[n_before + j], lds, a.table_words, tid, wave, nw, lane,
                                                s_wsum, acc, queue);
            }
        }
    }
    // Wavefront bins: each wavefront owns a slice of the LDS and takes `per_fetch` vertices at a time.
    // Chunk c of a bin belongs to sub-queue c % kWaveQueues (interleaved, so every sub-queue keeps the
    // largest-work-first order); each sub-queue counter has a cache line of its own, which spreads
    // the fetch atomics of a launch with millions of light vertices over kWaveQueues addresses.  A
    // wavefront starts on sub-queue blockIdx % kWaveQueues (one per XCD with round-robin dispatch),
    // moves on when its sub-queue is drained, and requests its next chunk before working on the
    // current one.  `work(args, base, j0, j1)` processes items base + [j0, j1) of the bin with the
    // arguments of their graph (in multi-graph mode a chunk never spans two graphs).
    // The wavefront's own region (after the workgroup bin): a table slice and its probe queue, or
    // four packed-vertex tables.
    uint32_t* slice = lds + (size_t)wave * (a.slice_words + kQueueWords);
    uint32_t* const slice_queue = slice + a.slice_words;
    auto drain = [&](uint32_t bin, uint32_t n_bin, uint32_t base1, uint32_t per_fetch, uint32_t head0,
                     auto&& work) {
        const uint32_t nchunks = MULTI ? a.multi->fetch_tot[bin] : (n_bin + per_fetch - 1) / per_fetch;
        uint32_t q = blockIdx.x % kWaveQueues, drained = 0;
        auto request = [&]() -> uint32_t {
            uint32_t c = 0;
            if (lane == 0) c = atomicAdd(&a.heads[(head0 + q) * kHeadStride], 1u);
            return c;
        };
        // Chunk index from a sub-queue ticket, moving on through drained sub-queues (nchunks: all done).
        auto settle = [&](uint32_t ticket) -> uint32_t {
            for (;;) {
                const uint32_t g = __builtin_amdgcn_readfirstlane(ticket) * kWaveQueues + q;
                if (g < nchunks) return g;
                if (++drained >= kWaveQueues) return nchunks;
                q = (q + 1) % kWaveQueues;
                ticket = request();
            }
        };
        uint32_t cur = settle(request());
        while (cur < nchunks) {
            const uint32_t ticket = request();  // next chunk, settled after this one
            if constexpr (MULTI) {
                const MultiHeader* H = a.multi;
                const uint32_t* pre = H->pre + (size_t)bin * (H->k + 1);
                const uint32_t g = find_graph(pre, H->k, cur, lane);
                const MultiDesc& d = H->desc[g];
                const uint32_t nb = d.meta->bins[bin];
                const uint32_t j0 = (cur - pre[g]) * per_fetch;
                sink.to(d.totals, acc, lane);
                work(graph_view(a, d), bin_base(d.meta, bin), j0, (j0 + per_fetch < nb) ? j0 + per_fetch : nb);
            } else {
                const uint32_t j0 = cur * per_fetch;
                work(a, base1, j0, (j0 + per_fetch < n_bin) ? j0 + per_fetch : n_bin);
            }
            cur = settle(ticket);
        }
    };
    // Bin 3: one vertex per wavefront.
    drain(3u, n_wave, n_before + n_wg, a.chunk, 3u, [&](const CountArgs& v, uint32_t base, uint32_t j0, uint32_t j1) {
        // The vertices of a fetch and their list bounds are loaded by the wavefront at once
        // (lane i holds the i-th), so each vertex starts without two dependent loads.
        for (uint32_t b0 = j0; b0 < j1; b0 += 64) {
            const uint32_t cnt = (j1 - b0 < 64u) ? j1 - b0 : 64u;
            uint32_t vu = 0, vb = 0, vd = 0;  // list starts stay below 2^31 (m < 2^31; records: m + n < 2^31)
            if ((uint32_t)lane < cnt) {
                vu = v.items[base + b0 + lane];
                vb = own_start(v, vu);
                vd = v.off[vu + 1] - v.off[vu];
            }
            // Two-stage prefetch for lists of at most 64: the next vertex's list is loaded while
            // this one's table is built, and its elements' list bounds while this one is probed.
            uint32_t xw = 0, xo = 0, xl = 0;
            auto prime = [&](uint32_t i0) {  // vertex i0's list element and its bounds, loaded now
                const int64_t beg0 = (int64_t)__builtin_amdgcn_readlane(vb, i0);
                const uint32_t d0 = __builtin_amdgcn_readlane(vd, i0);
                xw = xo = xl = 0;
                if (d0 <= 64u && (uint32_t)lane < d0) {
                    xw = v.col[beg0 + lane];
                    list_of(v, xw, xo, xl);
                }
            };
            prime(0);
            for (uint32_t i = 0; i < cnt; ++i) {
                const uint32_t u = __builtin_amdgcn_readlane(vu, i);
                const int64_t beg = (int64_t)__builtin_amdgcn_readlane(vb, i);
                const uint32_t d = __builtin_amdgcn_readlane(vd, i);
                const uint32_t inext = i + 1 < cnt ? i + 1 : i;
                const int64_t beg_n = (int64_t)__builtin_amdgcn_readlane(vb, inext);
                const uint32_t d_n = i + 1 < cnt ? __builtin_amdgcn_readlane(vd, inext) : 0u;
                const bool pre_n = d_n <= 64u && (uint32_t)lane < d_n;
                uint32_t nw = 0, no = 0, nl = 0;
                if (pre_n) nw = v.col[beg_n + lane];
                auto mid = [&]() {
                    if (pre_n) list_of(v, nw, no, nl);
                };
                if (in_shard(v, u))
                    process<S, PV, HK, false, true, decltype(mid), SW>(v, u, beg, d, slice, a.slice_words, lane,
                                                                       64, 0, 1, lane, nullptr, acc, slice_queue,
                                                                       d <= 64u,
                                                                       xw, xo, xl, mid);
                else
                    mid();
                xw = nw;
                xo = no;
                xl = nl;
            }
        }
    });
    // Bin 4: light vertices (out-degree <= 32, small collective degree) packed several to a
    // wavefront: 4 x 16 lanes when the next 3 or 4 have out-degree <= 16, else 2 x 32 lanes.
    if constexpr (!SW) {
        drain(4u, n_pack, n_before + n_wg + n_wave, 4u * a.chunk, 3u + kWaveQueues,
              [&](const CountArgs& v, uint32_t base, uint32_t j0, uint32_t j1) {
            for (uint32_t b0 = j0; b0 < j1; b0 += 64) {
                const uint32_t cnt = (j1 - b0 < 64u) ? j1 - b0 : 64u;
                uint32_t vu = 0, vb = 0, vd = 0;
                if ((uint32_t)lane < cnt) {
                    vu = v.items[base + b0 + lane];
                    vb = own_start(v, vu);
                    vd = v.off[vu + 1] - v.off[vu];
                }
                for (uint32_t i = 0; i < cnt;) {
                    uint32_t n16 = 0;
                    while (n16 < 4 && i + n16 < cnt && __builtin_amdgcn_readlane(vd, i + n16) <= 16u) ++n16;
                    const bool use16 = n16 >= 3;
                    const uint32_t np = use16 ? n16 : (i + 1 < cnt ? 2u : 1u);
                    const uint32_t gsz = use16 ? 16u : 32u;
                    const uint32_t gi = (uint32_t)lane / gsz;
                    const int src = (int)(i + (gi < np ? gi : np - 1));
                    const uint32_t ug = (uint32_t)__shfl((int)vu, src, 64);
                    const uint32_t bg = (uint32_t)__shfl((int)vb, src, 64);
                    const uint32_t dg = (uint32_t)__shfl((int)vd, src, 64);
                    const bool has = gi < np && in_shard(v, ug);
                    if (use16)
                        process_packed<S, PV, HK, 16>(v, ug, bg, dg, has, slice, a.pack_region, lane, acc);
                    else
                        process_packed<S, PV, HK, 32>(v, ug, bg, dg, has, slice, a.pack_region, lane, acc);
                    i += np;
                }
            }
        });
    }
    if constexpr (MULTI) sink.to(nullptr, acc, lane);
    else add_workgroup_total(a, acc, s_acc, tid, lane, wave, nw);
}

typedef void (*KernelFn)(CountArgs);

template <int S, bool HUB, bool SW, bool MULTI>
KernelFn pick_hk(bool pv, uint32_t hk) {
    if constexpr (HUB) {
        if (pv) return hk ? tc_hub_kernel<S, true, 1, MULTI> : tc_hub_kernel<S, true, 0, MULTI>;
        return hk ? tc_hub_kernel<S, false, 1, MULTI> : tc_hub_kernel<S, false, 0, MULTI>;
    } else {
        if (pv) return hk ? tc_count_kernel<S, true, 1, SW, MULTI> : tc_count_kernel<S, true, 0, SW, MULTI>;
        return hk ? tc_count_kernel<S, false, 1, SW, MULTI> : tc_count_kernel<S, false, 0, SW, MULTI>;
    }
}

template <bool HUB, bool SW, bool MULTI>
KernelFn pick(uint32_t S, bool pv, uint32_t hk) {
    switch (S) {
        case 1: return pick_hk<1, HUB, SW, MULTI>(pv, hk);
        case 2: return pick_hk<2, HUB, SW, MULTI>(pv, hk);
        case 4: return pick_hk<4, HUB, SW, MULTI>(pv, hk);
        default: return nullptr;
    }
}

// Kernel variant: the large-vertex kernel or the main one; subwave probe assignment (main kernel,
// single graph only); graphs from a multi-graph header.
KernelFn pick_kernel(bool hub, bool sw, bool multi, uint32_t S, bool pv, uint32_t hk) {
    if (multi) return hub ? pick<true, false, true>(S, pv, hk) : pick<false, false, true>(S, pv, hk);
    if (hub) return pick<true, false, false>(S, pv, hk);
    return sw ? pick<false, true, false>(S, pv, hk) : pick<false, false, false>(S, pv, hk);
}

hipError_t kernel_info(KernelFn f, uint32_t threads, uint32_t lds_bytes, int* blocks_per_cu) {
    if (!f) return hipErrorInvalidValue;
    if (lds_bytes > 65536) {
        hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(f),
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds_bytes);
        if (e != hipSuccess) return e;
    }
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, reinterpret_cast<const void*>(f),
                                                        (int)threads, (size_t)lds_bytes);
}

}  // namespace

hipError_t count_kernel_info(bool hub, bool sw, uint32_t S, bool pv, uint32_t hash_kind, uint32_t threads,
                             uint32_t lds_bytes, int* blocks_per_cu) {
    return kernel_info(pick_kernel(hub, sw, false, S, pv, hash_kind), threads, lds_bytes, blocks_per_cu);
}

hipError_t count_kernel_info_multi(bool hub, uint32_t S, bool pv, uint32_t hash_kind, uint32_t threads,
                                   uint32_t lds_bytes, int* blocks_per_cu) {
    return kernel_info(pick_kernel(hub, false, true, S, pv, hash_kind), threads, lds_bytes, blocks_per_cu);
}

hipError_t count_kernel_static_lds(uint32_t* bytes) {
    hipFuncAttributes attr{};
    uint32_t most = 0;
    for (int multi = 0; multi < 2; ++multi) {
        hipError_t e = hipFuncGetAttributes(&attr,
                                            reinterpret_cast<const void*>(pick_kernel(true, false, multi, 4, true, 0)));
        if (e != hipSuccess) return e;
        if ((uint32_t)attr.sharedSizeBytes > most) most = (uint32_t)attr.sharedSizeBytes;
    }
    *bytes = most;
    return hipSuccess;
}

hipError_t count_launch(bool hub, bool sw, uint32_t S, bool pv, uint32_t hash_kind, uint32_t grid, uint32_t threads,
                        uint32_t lds_bytes, const CountArgs& a, hipStream_t stream) {
    KernelFn f = pick_kernel(hub, sw, false, S, pv, hash_kind);
    if (!f) return hipErrorInvalidValue;
    hipLaunchKernelGGL(f, dim3(grid), dim3(threads), lds_bytes, stream, a);
    return hipGetLastError();
}

hipError_t count_launch_multi(bool hub, uint32_t S, bool pv, uint32_t hash_kind, uint32_t grid, uint32_t threads,
                              uint32_t lds_bytes, const CountArgs& a, hipStream_t stream) {
    KernelFn f = pick_kernel(hub, false, true, S, pv, hash_kind);
    if (!f) return hipErrorInvalidValue;
    hipLaunchKernelGGL(f, dim3(grid), dim3(threads), lds_bytes, stream, a);
    return hipGetLastError();
}

namespace {

// Multi-graph set-up: every workgroup clears a grid-stride share of the totals and (per-vertex mode)
// of the staging; workgroup 0 clears the queue heads and forms, for every bin, the exclusive prefix
// over the handles of their fetch counts (ceil(bin size / per_fetch)) and the bin totals.
__global__ void __launch_bounds__(1024) k_multi_prepare(MultiHeader* H) {
    const uint32_t tid = threadIdx.x, lane = tid & 63u, wave = tid >> 6, nw = blockDim.x >> 6;
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + tid; i < H->n_totals; i += stride) H->totals[i] = 0;
    if (H->pv)
        for (size_t i = (size_t)blockIdx.x * blockDim.x + tid; i < H->n_total; i += stride) H->tv[i] = 0;
    if (blockIdx.x != 0) return;
    __shared__ uint32_t s_wave[kBins][kMaxWaves];
    __shared__ uint32_t s_carry[kBins], s_items[kBins];
    for (uint32_t i = tid; i < kHeadWords; i += blockDim.x) H->heads[i] = 0;
    if (tid < kBins) {
        s_carry[tid] = 0;
        s_items[tid] = 0;
    }
    __syncthreads();
    const uint32_t k = H->k;
    for (uint32_t g0 = 0; g0 < k; g0 += blockDim.x) {
        const uint32_t g = g0 + tid;
        uint32_t f[kBins];
        const GraphMeta* m = g < k ? H->desc[g].meta : nullptr;
#pragma unroll
        for (uint32_t b = 0; b < kBins; ++b) {
            const uint32_t nb = m ? m->bins[b] : 0u;
            if (nb) atomicAdd(&s_items[b], nb);
            f[b] = (nb + H->per_fetch[b] - 1) / H->per_fetch[b];
        }
        uint32_t incl[kBins];
#pragma unroll
        for (uint32_t b = 0; b < kBins; ++b) {
            incl[b] = wave_incl_scan(f[b]);
            if (lane == 63) s_wave[b][wave] = incl[b];
        }
        __syncthreads();
#pragma unroll
        for (uint32_t b = 0; b < kBins; ++b) {
            uint32_t before = s_carry[b];
            for (uint32_t w = 0; w < wave; ++w) before += s_wave[b][w];
            if (g < k) H->pre[b * (k + 1) + g] = before + incl[b] - f[b];
        }
        __syncthreads();
        if (tid < kBins) {
            uint32_t t = 0;
            for (uint32_t w = 0; w < nw; ++w) t += s_wave[tid][w];
            s_carry[tid] += t;
        }
        __syncthreads();
    }
    if (tid < kBins) {
        H->pre[tid * (k + 1) + k] = s_carry[tid];
        H->fetch_tot[tid] = s_carry[tid];
        H->items_tot[tid] = s_items[tid];
    }
}

// Per-vertex output of a multi-graph count: staging entry tv0_g + r holds rank r of handle g, so
// input vertex x of handle g gets tv[tv0_g + rank_g[x]].  Position p of [0, n_total) is vertex
// p - tv0_g of the last handle g with tv0_g <= p (handles are laid out one after another); each
// workgroup takes a contiguous range, each thread finds its handle once and walks forward.
__global__ void __launch_bounds__(256) k_multi_gather(const MultiHeader* H) {
    const unsigned long long n = H->n_total;
    const uint32_t k = H->k;
    const unsigned long long per = (n + gridDim.x - 1) / gridDim.x;
    const unsigned long long p1 = (per * (blockIdx.x + 1) < n) ? per * (blockIdx.x + 1) : n;
    unsigned long long p = per * blockIdx.x + threadIdx.x;
    if (p >= p1) return;
    const MultiDesc* D = H->desc;
    uint32_t lo = 0, hi = k - 1;
    while (lo < hi) {
        const uint32_t mid = (lo + hi + 1) / 2;
        if (D[mid].tv0 <= p) lo = mid; else hi = mid - 1;
    }
    uint32_t g = lo;
    for (; p < p1; p += blockDim.x) {
        while (g + 1 < k && D[g + 1].tv0 <= p) ++g;
        const MultiDesc& d = D[g];
        const unsigned long long x = p - d.tv0;
        d.out[x] = H->tv[d.tv0 + d.rank[x]];
    }
}

}  // namespace

hipError_t multi_prepare(MultiHeader* hdr, int cu_count, hipStream_t stream) {
    hipLaunchKernelGGL(k_multi_prepare, dim3((uint32_t)(cu_count > 0 ? cu_count : 1)), dim3(1024), 0, stream, hdr);
    return hipGetLastError();
}

hipError_t multi_gather(const MultiHeader* hdr, int cu_count, hipStream_t stream) {
    hipLaunchKernelGGL(k_multi_gather, dim3((uint32_t)(cu_count > 0 ? 4 * cu_count : 1)), dim3(256), 0, stream, hdr);
    return hipGetLastError();
}

}  // namespace tc
