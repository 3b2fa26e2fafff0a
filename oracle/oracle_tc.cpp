// CPU oracle for exact triangle counting.  TEST INFRASTRUCTURE ONLY.
//
// Only the test suite, the smoke check and the benchmark's CPU-baseline leg
// may load this library.  It shares no code with the device path: no headers,
// no helpers, no tables.  It is written to be slow and obviously correct.
//
// What it computes (plain definitions, paper Sections 1 and 2.1):
//   * E = { {u,v} : u != v and (u,v) or (v,u) appears in the input } -- the
//     input is cleaned by dropping self-loops and duplicate edges and by
//     reading every pair as undirected (paper Section 2.6, the three dataset
//     transformation steps; orphan removal is not needed because an isolated
//     vertex is in no triangle).
//   * T = number of 3-element vertex sets whose three pairs are all in E.
//   * t(x) = number of those sets that contain x (so sum_x t(x) = 3 T).
//
// How (oracle_count): the intersection family of Section 2.2, in its
// merge-path form, on the rank-by-degree orientation of Section 2.2.
// Each undirected edge keeps one direction, from the endpoint that comes
// first in (degree, id) order to the other; the paper states only that the
// edge leaving the larger-degree endpoint is dropped, and ties are broken by
// vertex id here.  Every triangle {a,b,c} with a before b before c is then
// found exactly once, as c in N+(a) and N+(b), by a two-pointer scan of the
// two sorted lists.  std::sort / std::unique serve as library steps.
//
// oracle_vertex_counts evaluates t(x) for a few queried vertices straight
// from the definition, with no orientation: t(x) = (1/2) sum over neighbours
// y of |N(x) intersect N(y)|, the number of edges among the neighbours of x.
#include <algorithm>
#include <chrono>
#include <cstdint>
#include <cstring>
#include <vector>
#include <omp.h>

namespace {

using u32 = uint32_t;
using u64 = uint64_t;

double now_s() {
    return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

// Cleaned undirected edge set as sorted, unique keys (min << 32 | max).
// Returns false if an id is out of range.
bool clean_edges(u32 n, u64 m_in, const u32* src, const u32* dst, std::vector<u64>& keys) {
    keys.clear();
    keys.reserve(m_in);
    for (u64 i = 0; i < m_in; ++i) {
        u32 a = src[i], b = dst[i];
        if (a >= n || b >= n) return false;
        if (a == b) continue;                 // self-loop dropped
        u32 lo = a < b ? a : b, hi = a < b ? b : a;
        keys.push_back((u64(lo) << 32) | hi);  // direction dropped
    }
    std::sort(keys.begin(), keys.end());
    keys.erase(std::unique(keys.begin(), keys.end()), keys.end());  // duplicates dropped
    return true;
}

}  // namespace

extern "C" {

struct oracle_stats {
    u64 m;                 // undirected edges after cleaning (= oriented edges)
    u64 wedges_plus;       // W+ = sum over oriented (x,y) of d+(y): the 2-hop list lengths probed
    u64 max_dplus;         // largest out-degree after orientation
    u64 counted_vertices;  // vertices x whose N+(x) was processed (all, or the sample)
    u64 counted_edges;     // oriented edges (x, y) processed
    u64 counted_wedges;    // sum of d+(y) over the processed (x, y)
    double t_clean_s;      // cleaning + orientation + list build
    double t_count_s;      // merge intersections
    int threads;           // OpenMP threads used by the count
};

// Total (and optionally per-vertex) triangle count.
// stride > 1 processes only vertices x with x % stride == 0 (a bounded sample
// for timing; the total is then partial).  per_vertex, if non-null, has n
// entries and is overwritten.  Returns 0, or 2 if an id is >= n.
int oracle_count(u32 n, u64 m_in, const u32* src, const u32* dst, int nthreads, u32 stride,
                 u64* total, u64* per_vertex, oracle_stats* st) {
    if (nthreads > 0) omp_set_num_threads(nthreads);
    if (stride == 0) stride = 1;
    double t0 = now_s();
    std::vector<u64> keys;
    if (!clean_edges(n, m_in, src, dst, keys)) return 2;
    const u64 m = keys.size();

    // Undirected degree after cleaning.
    std::vector<u64> deg(n, 0);
    for (u64 k : keys) { deg[k >> 32]++; deg[k & 0xffffffffu]++; }
    // x precedes y in (degree, id) order.
    auto precedes = [&](u32 x, u32 y) { return deg[x] < deg[y] || (deg[x] == deg[y] && x < y); };

    // Oriented adjacency N+(x), each list sorted by id.
    std::vector<u64> off(size_t(n) + 1, 0);
    for (u64 k : keys) {
        u32 a = u32(k >> 32), b = u32(k);
        off[size_t(precedes(a, b) ? a : b) + 1]++;
    }
    for (size_t x = 0; x < n; ++x) off[x + 1] += off[x];
    std::vector<u32> nbr(m);
    {
        std::vector<u64> fill(off.begin(), off.end() - 1);
        for (u64 k : keys) {
            u32 a = u32(k >> 32), b = u32(k);
            if (precedes(a, b)) nbr[fill[a]++] = b; else nbr[fill[b]++] = a;
        }
    }
    std::vector<u64>().swap(keys);
#pragma omp parallel for schedule(dynamic, 256)
    for (int64_t x = 0; x < int64_t(n); ++x) std::sort(nbr.begin() + off[x], nbr.begin() + off[x + 1]);
    double t1 = now_s();

    if (per_vertex) std::memset(per_vertex, 0, sizeof(u64) * n);
    u64 T = 0, wplus = 0, maxdp = 0, cv = 0, ce = 0, cw = 0;
    int used = 1;
#pragma omp parallel reduction(+ : T, wplus, cv, ce, cw) reduction(max : maxdp)
    {
#pragma omp single
        used = omp_get_num_threads();
#pragma omp for schedule(dynamic, 64)
        for (int64_t xi = 0; xi < int64_t(n); ++xi) {
            const u32 x = u32(xi);
            const u64 xb = off[x], xe = off[x + 1];
            if (xe - xb > maxdp) maxdp = xe - xb;
            for (u64 p = xb; p < xe; ++p) wplus += off[nbr[p] + 1] - off[nbr[p]];
            if (x % stride) continue;
            cv++;
            for (u64 p = xb; p < xe; ++p) {
                const u32 y = nbr[p];
                u64 i = xb, j = off[y];
                const u64 je = off[y + 1];
                ce++;
                cw += je - j;
                // Two-pointer merge: advance the pointer at the smaller value;
                // equal values are a common neighbour z, i.e. a triangle x, y, z.
                while (i < xe && j < je) {
                    const u32 a = nbr[i], b = nbr[j];
                    if (a < b) ++i;
                    else if (b < a) ++j;
                    else {
                        T++;
                        if (per_vertex) {
#pragma omp atomic
                            per_vertex[x]++;
#pragma omp atomic
                            per_vertex[y]++;
#pragma omp atomic
                            per_vertex[a]++;
                        }
                        ++i; ++j;
                    }
                }
            }
        }
    }
    double t2 = now_s();
    *total = T;
    if (st) {
        st->m = m; st->wedges_plus = wplus; st->max_dplus = maxdp;
        st->counted_vertices = cv; st->counted_edges = ce; st->counted_wedges = cw;
        st->t_clean_s = t1 - t0; st->t_count_s = t2 - t1; st->threads = used;
    }
    return 0;
}

// t(x) for each queried x, straight from the definition (edges among the
// neighbours of x), on the cleaned undirected graph.  Returns 0 or 2.
int oracle_vertex_counts(u32 n, u64 m_in, const u32* src, const u32* dst, u64 nq, const u32* q,
                         u64* out, int nthreads) {
    if (nthreads > 0) omp_set_num_threads(nthreads);
    std::vector<u64> keys;
    if (!clean_edges(n, m_in, src, dst, keys)) return 2;
    for (u64 i = 0; i < nq; ++i) if (q[i] >= n) return 2;
    // Undirected adjacency, both directions, sorted lists.
    std::vector<u64> off(size_t(n) + 1, 0);
    for (u64 k : keys) { off[(k >> 32) + 1]++; off[(k & 0xffffffffu) + 1]++; }
    for (size_t x = 0; x < n; ++x) off[x + 1] += off[x];
    std::vector<u32> adj(2 * keys.size());
    {
        std::vector<u64> fill(off.begin(), off.end() - 1);
        for (u64 k : keys) {
            u32 a = u32(k >> 32), b = u32(k);
            adj[fill[a]++] = b;
            adj[fill[b]++] = a;
        }
    }
    std::vector<u64>().swap(keys);
#pragma omp parallel for schedule(dynamic, 256)
    for (int64_t x = 0; x < int64_t(n); ++x) std::sort(adj.begin() + off[x], adj.begin() + off[x + 1]);
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t t = 0; t < int64_t(nq); ++t) {
        const u32 x = q[t];
        u64 s = 0;
        for (u64 p = off[x]; p < off[x + 1]; ++p) {
            const u32 y = adj[p];
            u64 i = off[x], j = off[y];
            while (i < off[x + 1] && j < off[y + 1]) {
                if (adj[i] < adj[j]) ++i;
                else if (adj[j] < adj[i]) ++j;
                else { ++s; ++i; ++j; }
            }
        }
        out[t] = s / 2;  // each edge {y, z} among the neighbours is seen from y and from z
    }
    return 0;
}

// The cleaned graph's oriented CSR in (degree, id) order, for comparing a
// device-built CSR against: out_deg[n] receives d+(x), out_nbr receives the
// concatenated sorted N+(x) lists in id order (capacity m_in).  Returns the
// number of oriented edges through *m_out.  Returns 0 or 2.
int oracle_oriented(u32 n, u64 m_in, const u32* src, const u32* dst, u32* deg_out, u32* dplus_out,
                    u32* nbr_out, u64* m_out) {
    std::vector<u64> keys;
    if (!clean_edges(n, m_in, src, dst, keys)) return 2;
    std::vector<u64> deg(n, 0);
    for (u64 k : keys) { deg[k >> 32]++; deg[k & 0xffffffffu]++; }
    auto precedes = [&](u32 x, u32 y) { return deg[x] < deg[y] || (deg[x] == deg[y] && x < y); };
    std::vector<std::vector<u32>> lists(n);
    for (u64 k : keys) {
        u32 a = u32(k >> 32), b = u32(k);
        if (precedes(a, b)) lists[a].push_back(b); else lists[b].push_back(a);
    }
    u64 e = 0;
    for (u32 x = 0; x < n; ++x) {
        std::sort(lists[x].begin(), lists[x].end());
        deg_out[x] = u32(deg[x]);
        dplus_out[x] = u32(lists[x].size());
        for (u32 y : lists[x]) nbr_out[e++] = y;
    }
    *m_out = e;
    return 0;
}

}  // extern "C"
