// Cost-balanced split of a tree's bodies into Morton-contiguous target ranges.
//
// The paper names the varying work per particle and the tree rebuilt at every
// step as the obstacles to static load balance (section 1).  The split here is
// the cost-zone method (Singh, Holt, Totsuka, Gupta and Hennessy, 1995) on the
// Morton order of the current tree, over items that are either bodies or the
// 64-body walk groups.  A body costs one plus what a previous counting walk
// measured for it (its interactions, or its share of its group's wavefront
// work); a group costs its body count plus its wavefront work.  Range j of G
// starts at the first item boundary m whose exclusive prefix cost P(m) reaches
// j/G of the total T (smallest m with G P(m) >= j T; P(0) = 0), a body rank or,
// for groups, rank min(64 m, n).
//
// Three launches: prefix sums within chunks of kShardChunk items, a scan of the
// chunk totals, then one binary search per boundary over P(m) =
// chunk_prefix[(m - 1) / kShardChunk] + local[m - 1].
#include "bh_common.h"

namespace bh {

constexpr uint32_t kShardChunk = 1024;   // ranks per chunk: 256 threads x 4

// Cost of item s: body of rank s (its costs gathered in the caller's order), or
// walk group s (bodies [64 s, min(64 s + 64, n)), its cost read in rank order).
__device__ __forceinline__ unsigned long long item_cost(const uint32_t *idx, const int64_t *ca, const int64_t *cb,
                                                        const int64_t *gc, uint32_t n, uint32_t s) {
    if (gc) {
        const uint32_t lo = s * (uint32_t)kGroup;
        return (unsigned long long)(n - lo < (uint32_t)kGroup ? n - lo : (uint32_t)kGroup) +
               (unsigned long long)gc[s];
    }
    const uint32_t i = idx[s];
    unsigned long long c = 1;
    if (ca) c += (unsigned long long)ca[i];
    if (cb) c += (unsigned long long)cb[i];
    return c;
}

__device__ __forceinline__ unsigned long long wave_incl_scan(unsigned long long x, int lane) {
    for (int o = 1; o < 64; o <<= 1) {
        const unsigned long long y = __shfl_up(x, o, 64);
        if (lane >= o) x += y;
    }
    return x;
}

// loc[s] = sum of the costs from the start of s's chunk through item s (m items);
// csum[c] = chunk c's total.
__global__ void __launch_bounds__(256) k_shard_local(const uint32_t *idx, const int64_t *ca, const int64_t *cb,
                                                     const int64_t *gc, uint32_t n, uint32_t m,
                                                     unsigned long long *loc, unsigned long long *csum) {
    __shared__ unsigned long long wsum[4];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const uint32_t base = blockIdx.x * kShardChunk + 4 * threadIdx.x;
    unsigned long long c[4], run = 0;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        run += base + q < m ? item_cost(idx, ca, cb, gc, n, base + q) : 0ull;
        c[q] = run;
    }
    const unsigned long long x = wave_incl_scan(run, lane);
    if (lane == 63) wsum[wave] = x;
    __syncthreads();
    unsigned long long wpre = 0;
    for (int w = 0; w < wave; ++w) wpre += wsum[w];
    const unsigned long long pre = wpre + x - run;   // costs of this chunk before this thread's ranks
#pragma unroll
    for (int q = 0; q < 4; ++q)
        if (base + q < m) loc[base + q] = pre + c[q];
    if (threadIdx.x == 255) csum[blockIdx.x] = wpre + x;
}

// Exclusive scan of the nc chunk totals in place; csum[nc] = T.
__global__ void __launch_bounds__(1024) k_shard_scan(unsigned long long *csum, uint32_t nc) {
    __shared__ unsigned long long wsum[16];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    unsigned long long carry = 0;
    for (uint32_t b = 0; b < nc; b += 1024) {
        const uint32_t t = b + threadIdx.x;
        const unsigned long long v = t < nc ? csum[t] : 0ull;
        const unsigned long long x = wave_incl_scan(v, lane);
        if (lane == 63) wsum[wave] = x;
        __syncthreads();
        unsigned long long wpre = 0, tot = 0;
        for (int w = 0; w < 16; ++w) {
            if (w < wave) wpre += wsum[w];
            tot += wsum[w];
        }
        if (t < nc) csum[t] = carry + wpre + x - v;
        carry += tot;
        __syncthreads();   // wsum is rewritten by the next round
    }
    if (threadIdx.x == 0) csum[nc] = carry;
}

// bounds[j] = min(unit x, n) for the smallest item boundary x in [0, m] with
// G P(x) >= j T (j = 0..G); unit = 1 for bodies, 64 for groups.
__global__ void __launch_bounds__(256) k_shard_search(const unsigned long long *loc, const unsigned long long *csum,
                                                      uint32_t m, uint32_t nc, uint32_t G, uint32_t unit, uint32_t n,
                                                      int64_t *bounds) {
    const uint32_t j = blockIdx.x * 256 + threadIdx.x;
    if (j > G) return;
    if (j == 0) {
        bounds[0] = 0;
        return;
    }
    const unsigned __int128 want = (unsigned __int128)j * csum[nc];
    uint32_t lo = 1, hi = m;   // P(m) = T, so x = m always qualifies
    while (lo < hi) {
        const uint32_t mid = lo + (hi - lo) / 2;
        const unsigned long long P = csum[(mid - 1) / kShardChunk] + loc[mid - 1];
        if ((unsigned __int128)G * P >= want) hi = mid;
        else lo = mid + 1;
    }
    const unsigned long long r = (unsigned long long)lo * unit;
    bounds[j] = (int64_t)(r < n ? r : n);
}

hipError_t launch_shard_bounds(const ForestDev &f, uint32_t n, const int64_t *cost_a, const int64_t *cost_b,
                               const int64_t *group_cost, uint32_t G, int64_t *bounds, hipStream_t s) {
    const uint32_t unit = group_cost ? (uint32_t)kGroup : 1u;
    const uint32_t m = (n + unit - 1) / unit;   // items
    const uint32_t nc = (m + kShardChunk - 1) / kShardChunk;
    // scratch: the sort's alternate keys (n >= m values) and the bounding-box tile table
    // (6 per 4096 bodies >= nc + 1 values), both idle between builds
    unsigned long long *loc = reinterpret_cast<unsigned long long *>(f.keys_alt);
    unsigned long long *csum = f.tile_mm;
    hipLaunchKernelGGL(k_shard_local, dim3(nc), dim3(256), 0, s, f.idx, cost_a, cost_b, group_cost, n, m, loc, csum);
    hipLaunchKernelGGL(k_shard_scan, dim3(1), dim3(1024), 0, s, csum, nc);
    hipLaunchKernelGGL(k_shard_search, dim3((G + 256) / 256), dim3(256), 0, s, loc, csum, m, nc, G, unit, n, bounds);
    return hipGetLastError();
}

}  // namespace bh
