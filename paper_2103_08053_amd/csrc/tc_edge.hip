// Plain vertex-centric and edge-centric hashing (paper Section 3.3, Algorithms 1 and 2) for the
// construction-cost ablation.
//
// Both designs use the same table (B buckets of S = 4 slots, atomic len[] insertion with the
// next-bucket overflow rule, minimal B for the load factor) and the same lookup (lane by lane along
// the bucket chain).  One workgroup owns a vertex u at a time:
//   vertex-centric: build the table of N+(u) once, then probe N+(v) for every v in N+(u);
//   edge-centric  : for every v in N+(u), build the table of N+(u) again, then probe N+(v)
//                   (every oriented edge (u, v) is its own task, as in Algorithm 2).
// With build_only the probes are skipped (the count is 0): the launch then measures table
// construction alone.  Vertices are fetched 16 at a time.  Not the production path (that is tc_count.hip); both count exactly.
#include "tc_internal.h"

namespace tc {
namespace {

constexpr uint32_t kSimpleChunk = 16;  // vertices per queue fetch (one counter serves the whole grid)

__device__ __forceinline__ bool lookup(const uint32_t* slots, uint32_t w, uint32_t B) {
    uint32_t b = hash_of<0>(w, B);
    for (uint32_t t = 0; t < B; ++t) {
        const uint32_t* s = slots + b * kSimpleS;
        bool full = true;
#pragma unroll
        for (uint32_t j = 0; j < kSimpleS; ++j) {
            const uint32_t x = s[j];
            if (x == w) return true;
            if (x == kEmpty) full = false;
        }
        if (!full) return false;
        b = (b + 1) & (B - 1);
    }
    return false;
}

template <bool EDGE, bool BUILD_ONLY>
__global__ void __launch_bounds__(kSimpleThreads) k_simple(SimpleArgs a) {
    extern __shared__ __align__(16) uint32_t tbl[];
    __shared__ uint32_t s_item;
    __shared__ unsigned long long s_acc[kSimpleThreads / 64];
    const uint32_t tid = threadIdx.x;
    const uint32_t n_tab = a.meta->bins[0] + a.meta->bins[1] + a.meta->bins[2] + a.meta->bins[3] + a.meta->bins[4];
    unsigned long long acc = 0;
    for (;;) {
        if (tid == 0) s_item = atomicAdd(a.head, kSimpleChunk);
        __syncthreads();
        const uint32_t j0 = s_item;
        __syncthreads();
        if (j0 >= n_tab) break;
        const uint32_t j1 = j0 + kSimpleChunk < n_tab ? j0 + kSimpleChunk : n_tab;
        for (uint32_t j = j0; j < j1; ++j) {
        const uint32_t u = a.items[j];
        const int64_t beg = a.off[u];
        const uint32_t d = (uint32_t)(a.off[u + 1] - beg);
        const Geometry g = geometry(d, kSimpleS, a.lrecip, false);
        uint32_t* slots = tbl;
        uint32_t* len = tbl + g.o_len;
        auto build = [&]() {
            for (uint32_t x = tid; x < g.B * kSimpleS; x += blockDim.x) slots[x] = kEmpty;
            for (uint32_t x = tid; x < g.B; x += blockDim.x) len[x] = 0;
            __syncthreads();
            for (uint32_t p = tid; p < d; p += blockDim.x) {
                const uint32_t w = a.col[beg + p];
                uint32_t b = hash_of<0>(w, g.B), pos;
                for (;;) {
                    pos = atomicAdd(&len[b], 1u);
                    if (pos < kSimpleS) break;
                    b = (b + 1) & g.mask;
                }
                slots[b * kSimpleS + pos] = w;
            }
            __syncthreads();
        };
        if (!EDGE) build();
        for (uint32_t k = 0; k < d; ++k) {
            if (EDGE) build();
            if (!BUILD_ONLY) {
                const uint32_t v = a.col[beg + k];
                const int64_t vb = a.off[v];
                const uint32_t dv = (uint32_t)(a.off[v + 1] - vb);
                for (uint32_t t = tid; t < dv; t += blockDim.x) acc += lookup(slots, a.col[vb + t], g.B) ? 1u : 0u;
            }
            if (EDGE) __syncthreads();  // the next edge rebuilds the table
        }
        __syncthreads();
        }
    }
    // block sum, one atomic
    unsigned long long v = acc;
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    if ((tid & 63) == 0) s_acc[tid >> 6] = v;
    __syncthreads();
    if (tid == 0) {
        unsigned long long sum = 0;
        for (uint32_t w = 0; w < kSimpleThreads / 64; ++w) sum += s_acc[w];
        if (sum) atomicAdd(a.total, sum);
    }
}

typedef void (*SimpleFn)(SimpleArgs);

SimpleFn pick(bool edge, bool build_only) {
    if (edge) return build_only ? k_simple<true, true> : k_simple<true, false>;
    return build_only ? k_simple<false, true> : k_simple<false, false>;
}

}  // namespace

hipError_t simple_capacity(uint32_t lds_bytes, uint32_t load_pct, uint32_t* max_d) {
    const uint32_t words = lds_bytes / 4, lr = load_recip(load_pct);
    uint32_t lo = 0, hi = words;
    while (lo < hi) {
        const uint32_t mid = lo + (hi - lo + 1) / 2;
        if (geometry(mid, kSimpleS, lr, false).words <= words) lo = mid; else hi = mid - 1;
    }
    *max_d = lo;
    return hipSuccess;
}

hipError_t simple_launch(bool edge, bool build_only, uint32_t lds_bytes, int cu_count, const SimpleArgs& a,
                         hipStream_t stream) {
    const SimpleFn f = pick(edge, build_only);
    if (lds_bytes > 65536) {
        if (hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(f),
                                               hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds_bytes))
            return e;
    }
    int per_cu = 0;
    if (hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, reinterpret_cast<const void*>(f),
                                                                    (int)kSimpleThreads, lds_bytes))
        return e;
    if (per_cu < 1) return hipErrorInvalidConfiguration;
    hipLaunchKernelGGL(f, dim3((uint32_t)(per_cu * (cu_count > 0 ? cu_count : 1))), dim3(kSimpleThreads), lds_bytes,
                       stream, a);
    return hipGetLastError();
}

}  // namespace tc
