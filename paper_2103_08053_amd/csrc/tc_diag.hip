// Collision statistics of the hash tables the count kernels build (paper Section 4.1, Equation 2).
//
// For every scheduled vertex u (bins 0-4) this recomputes the bucket count B of u's table exactly
// as the count kernels size it (same bin capacity, same geometry) and histograms the home bucket
// hash(w) of every w in N+(u).  The maximum bucket load is the "max collision" of u; the estimate of
// Equation 2 weighs it with the collective degree W(u) = sum of d+(v) over v in N+(u):
//     phi = sum over u of W(u) * max collision(u).
// A diagnostic: it does not touch the counts and is not on the counting path.
#include "tc_internal.h"

namespace tc {
namespace {

constexpr uint32_t kDiagThreads = 256;
constexpr uint32_t kPassBuckets = 32768;  // LDS counters per histogram pass (128 KB)

template <int HK>
__global__ void __launch_bounds__(kDiagThreads) k_collisions(DiagArgs a) {
    extern __shared__ uint32_t cnt[];  // kPassBuckets counters
    __shared__ unsigned long long s_w;
    __shared__ uint32_t s_max;
    const uint32_t nb0 = a.meta->bins[0], nb1 = a.meta->bins[1], nb2 = a.meta->bins[2], nb3 = a.meta->bins[3];
    const uint32_t total = nb0 + nb1 + nb2 + nb3 + a.meta->bins[4];
    unsigned long long phi = 0, summax = 0, tables = 0;
    uint32_t maxall = 0;
    for (uint32_t j = blockIdx.x; j < total; j += gridDim.x) {
        const uint32_t bin = j < nb0 ? 0u : j < nb0 + nb1 ? 1u : j < nb0 + nb1 + nb2 ? 2u
                           : j < nb0 + nb1 + nb2 + nb3 ? 3u : 4u;
        const uint32_t u = a.items[j];
        const int64_t beg = a.off[u];
        const uint32_t d = (uint32_t)(a.off[u + 1] - beg);
        const Geometry g = geometry_fit(d, a.S, a.lrecip, a.pv != 0, a.avail[bin], a.filt[bin] != 0);
        if (threadIdx.x == 0) { s_w = 0; s_max = 0; }
        __syncthreads();
        unsigned long long w_part = 0;
        for (uint32_t p = threadIdx.x; p < d; p += blockDim.x) {
            const uint32_t v = a.col[beg + p];
            w_part += (unsigned long long)(a.off[v + 1] - a.off[v]);
        }
        atomicAdd(&s_w, w_part);
        uint32_t mx = 0;
        for (uint32_t b0 = 0; b0 < g.B; b0 += kPassBuckets) {
            const uint32_t nbk = g.B - b0 < kPassBuckets ? g.B - b0 : kPassBuckets;
            for (uint32_t x = threadIdx.x; x < nbk; x += blockDim.x) cnt[x] = 0;
            __syncthreads();
            for (uint32_t p = threadIdx.x; p < d; p += blockDim.x) {
                const uint32_t h = hash_of<HK>(a.col[beg + p], g.B);
                if (h >= b0 && h < b0 + nbk) atomicAdd(&cnt[h - b0], 1u);
            }
            __syncthreads();
            for (uint32_t x = threadIdx.x; x < nbk; x += blockDim.x) mx = cnt[x] > mx ? cnt[x] : mx;
            __syncthreads();
        }
        atomicMax(&s_max, mx);
        __syncthreads();
        if (threadIdx.x == 0) {
            phi += s_w * s_max;
            summax += s_max;
            tables += 1;
            maxall = s_max > maxall ? s_max : maxall;
        }
        __syncthreads();
    }
    if (threadIdx.x == 0 && tables) {
        atomicAdd(&a.stats[0], phi);
        atomicAdd(&a.stats[1], summax);
        atomicAdd(&a.stats[2], tables);
        atomicMax(&a.stats[3], (unsigned long long)maxall);
    }
}

__global__ void k_zero4(unsigned long long* p) {
    if (threadIdx.x < 4) p[threadIdx.x] = 0;
}

}  // namespace

hipError_t collision_stats(const DiagArgs& a, int cu_count, hipStream_t stream) {
    hipLaunchKernelGGL(k_zero4, dim3(1), dim3(64), 0, stream, a.stats);
    if (hipError_t e = hipGetLastError()) return e;
    const auto f = a.hash_kind ? k_collisions<1> : k_collisions<0>;
    const size_t lds = 4 * (size_t)kPassBuckets;
    if (hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(f),
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds))
        return e;
    hipLaunchKernelGGL(f, dim3(4 * (uint32_t)(cu_count > 0 ? cu_count : 1)), dim3(kDiagThreads), lds, stream, a);
    return hipGetLastError();
}

}  // namespace tc
