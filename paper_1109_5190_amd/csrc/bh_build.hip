// Octree construction and upward pass on gfx950.
//
// Build (paper section 1: cubes subdivided recursively until a cube holds at
// most leaf_cap particles; Fig. 2):
//   bbox      per-simulation FP64 min/max (order-free integer atomics)
//   keys      root cube [lo, lo + 2^k)^3, 21-bit quantisation, 63-bit Morton key
//   sort      stable LSD radix sort of (key, row), 8 passes of 8 bits; a pass is
//             tile histogram -> one global exclusive scan -> LDS-ranked scatter
//   permute   FP64 state and FP32 walk copies into key order
//   lcp       common-prefix level of neighbouring keys
//   mark/fill canonical compressed octree straight from the sorted keys:
//             a cube is a node iff it is a leaf of the cube hierarchy or it
//             holds more than leaf_cap particles spread over >= 2 sub-cubes;
//             node ids are the depth-first preorder (sort by (first, level))
// Upward (section 1: centre of mass of each cube): leaves sum their particles
// in key order, inner nodes their children in octant order, level by level.
#include "bh_common.h"

namespace bh {

// ============================================================== utilities ===

__global__ void k_fill_u32(uint32_t *p, uint32_t v, size_t n) {
    size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    size_t stride = (size_t)gridDim.x * blockDim.x;
    for (; i < n; i += stride) p[i] = v;
}

hipError_t launch_fill_u32(uint32_t *p, uint32_t v, size_t n, hipStream_t s) {
    if (n == 0) return hipSuccess;
    unsigned blocks = (unsigned)((n + 255) / 256);
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL(k_fill_u32, dim3(blocks), dim3(256), 0, s, p, v, n);
    return hipGetLastError();
}

// The per-tile streaming kernels (bbox, keys, sort histogram and scatter) give
// a 4096-particle tile 1024 threads (16 wavefronts, 4 particles each), so that
// enough loads are in flight with one tile per compute unit.
constexpr int kSortThreads = 1024;
constexpr int kSortWaves = kSortThreads / 64;

// Inclusive scan of one value per thread over the block (any multiple of 64
// threads; lds_waves holds one entry per wavefront).
__device__ inline uint32_t block_inclusive_scan_256(uint32_t v, uint32_t *lds_waves /*4*/) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        uint32_t t = __shfl_up(v, d, 64);
        if (lane >= d) v += t;
    }
    if (lane == 63) lds_waves[wave] = v;
    __syncthreads();
    uint32_t add = 0;
    for (int w = 0; w < wave; ++w) add += lds_waves[w];
    __syncthreads();
    return v + add;
}

// ----------------------------------------------------------------- scans ---
// Exclusive scan of f(in[i]), i in [0, n), into out[0..n] (out[n] = total).
// f = identity (kind 0) or popcount (kind 1).  Three kernels: block reduce,
// one-block scan of the block sums, block scan + offset.
constexpr int kScanItems = 8;
constexpr int kScanBlock = 256 * kScanItems;

template <int KIND>
__device__ __forceinline__ uint32_t scan_f(uint32_t v) {
    if (KIND == 1) return (uint32_t)__popc(v);
    return v;
}

template <int KIND>
__global__ void __launch_bounds__(256) k_scan_reduce(const uint32_t *in, uint32_t n, uint32_t *bsum) {
    __shared__ uint32_t w[4];
    size_t b0 = (size_t)blockIdx.x * kScanBlock;
    uint32_t s = 0;
#pragma unroll
    for (int j = 0; j < kScanItems; ++j) {
        size_t i = b0 + (size_t)j * 256 + threadIdx.x;
        if (i < n) s += scan_f<KIND>(in[i]);
    }
    uint32_t inc = block_inclusive_scan_256(s, w);
    if (threadIdx.x == 255) bsum[blockIdx.x] = inc;
}

__global__ void __launch_bounds__(256) k_scan_top(uint32_t *bsum, uint32_t nb, uint32_t *total_out) {
    __shared__ uint32_t w[4];
    __shared__ uint32_t last;
    uint32_t carry = 0;
    for (uint32_t c0 = 0; c0 < nb; c0 += 256) {
        uint32_t i = c0 + threadIdx.x;
        uint32_t v = i < nb ? bsum[i] : 0;
        uint32_t inc = block_inclusive_scan_256(v, w);
        if (i < nb) bsum[i] = carry + inc - v;
        if (threadIdx.x == 255) last = inc;
        __syncthreads();
        carry += last;
        __syncthreads();
    }
    if (threadIdx.x == 0) *total_out = carry;
}

template <int KIND>
__global__ void __launch_bounds__(256) k_scan_down(const uint32_t *in, uint32_t n, const uint32_t *bsum,
                                                   uint32_t *out) {
    __shared__ uint32_t w[4];
    size_t b0 = (size_t)blockIdx.x * kScanBlock + (size_t)threadIdx.x * kScanItems;
    uint32_t v[kScanItems];
    uint32_t s = 0;
#pragma unroll
    for (int j = 0; j < kScanItems; ++j) {
        size_t i = b0 + j;
        v[j] = i < n ? scan_f<KIND>(in[i]) : 0;
        s += v[j];
    }
    uint32_t inc = block_inclusive_scan_256(s, w);
    uint32_t run = bsum[blockIdx.x] + inc - s;
#pragma unroll
    for (int j = 0; j < kScanItems; ++j) {
        size_t i = b0 + j;
        if (i < n) out[i] = run;
        run += v[j];
    }
}

// One block of 1024 threads for arrays up to kScanSingleMax: each thread scans a
// contiguous run, then the run totals are scanned across the block.
constexpr uint32_t kScanSingleMax = 1u << 17;

__global__ void __launch_bounds__(1024) k_scan_single(const uint32_t *in, uint32_t n, uint32_t *out) {
    __shared__ uint32_t wsum[16];
    const uint32_t per = (n + 1023) / 1024;
    const uint32_t b0 = threadIdx.x * per;
    uint32_t s = 0;
    for (uint32_t j = 0; j < per; ++j) {
        const uint32_t i = b0 + j;
        if (i < n) s += in[i];
    }
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    uint32_t v = s;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        uint32_t t = __shfl_up(v, d, 64);
        if (lane >= d) v += t;
    }
    if (lane == 63) wsum[wave] = v;
    __syncthreads();
    uint32_t add = 0;
    for (int w = 0; w < wave; ++w) add += wsum[w];
    uint32_t run = add + v - s;
    if (threadIdx.x == 1023) out[n] = add + v;
    __syncthreads();
    for (uint32_t j = 0; j < per; ++j) {
        const uint32_t i = b0 + j;
        if (i < n) {
            const uint32_t x = in[i];
            out[i] = run;
            run += x;
        }
    }
}

static hipError_t scan_exclusive(const uint32_t *in, uint32_t n, uint32_t *out, uint32_t *tmp, int kind,
                                 hipStream_t s) {
    if (kind == 0 && n <= kScanSingleMax) {
        hipLaunchKernelGGL(k_scan_single, dim3(1), dim3(1024), 0, s, in, n, out);
        return hipGetLastError();
    }
    uint32_t nb = (n + kScanBlock - 1) / kScanBlock;
    if (nb == 0) nb = 1;
    if (kind == 1) hipLaunchKernelGGL(k_scan_reduce<1>, dim3(nb), dim3(256), 0, s, in, n, tmp);
    else hipLaunchKernelGGL(k_scan_reduce<0>, dim3(nb), dim3(256), 0, s, in, n, tmp);
    hipLaunchKernelGGL(k_scan_top, dim3(1), dim3(256), 0, s, tmp, nb, out + n);
    if (kind == 1) hipLaunchKernelGGL(k_scan_down<1>, dim3(nb), dim3(256), 0, s, in, n, tmp, out);
    else hipLaunchKernelGGL(k_scan_down<0>, dim3(nb), dim3(256), 0, s, in, n, tmp, out);
    return hipGetLastError();
}

// ================================================================= segids ===

__global__ void k_segid(ForestDev f) {
    const TileDesc td = f.tiles[blockIdx.x];
    for (uint32_t j = threadIdx.x; j < td.count; j += blockDim.x) f.segid[td.start + j] = td.seg;
}

hipError_t launch_segid(const ForestDev &f, hipStream_t s) {
    if (f.ntiles) hipLaunchKernelGGL(k_segid, dim3(f.ntiles), dim3(256), 0, s, f);
    return hipGetLastError();
}

// =================================================================== bbox ===

__global__ void __launch_bounds__(kSortThreads) k_bbox(ForestDev f, const double *pos, const double *mass) {
    const TileDesc td = f.tiles[blockIdx.x];
    const SegDesc &sd = f.seg[td.seg];
    const double *pb = seg_base(pos, sd.pos, sd, 3);
    const double *mb = seg_base(mass, sd.mass, sd, 1);
    const uint32_t j0 = td.start - sd.start;
    // a new build: the previous tree's inconsistency flag no longer applies
    if (blockIdx.x == 0 && threadIdx.x == 0) f.err[kErrWordTree] = 0;
    double mn[3] = {INFINITY, INFINITY, INFINITY}, mx[3] = {-INFINITY, -INFINITY, -INFINITY};
    bool bad = false;
    for (uint32_t j = threadIdx.x; j < td.count; j += kSortThreads) {
        size_t i = (size_t)j0 + j;
        double v[3];
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            v[d] = pb[3 * i + d];
            mn[d] = fmin(mn[d], v[d]);
            mx[d] = fmax(mx[d], v[d]);
        }
        const double m = mb[i];
        bad |= !isfinite(v[0]) || !isfinite(v[1]) || !isfinite(v[2]) || !isfinite(m);
        // the particle as one aligned record, for the gather into key order
        f.pk[(size_t)td.start + j] = make_double4(v[0], v[1], v[2], m);
    }
    // a non-finite coordinate or mass (fmin/fmax would pass over a NaN) is reported
    if (__builtin_amdgcn_ballot_w64(bad) && (threadIdx.x & 63) == 0) atomicOr(f.err, kErrNonFinite);
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        for (int o = 32; o > 0; o >>= 1) {
            mn[d] = fmin(mn[d], __shfl_xor(mn[d], o, 64));
            mx[d] = fmax(mx[d], __shfl_xor(mx[d], o, 64));
        }
    }
    __shared__ double wmn[kSortWaves][3], wmx[kSortWaves][3];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (lane == 0)
        for (int d = 0; d < 3; ++d) { wmn[wave][d] = mn[d]; wmx[wave][d] = mx[d]; }
    __syncthreads();
    if (threadIdx.x < 3) {
        const int d = threadIdx.x;
        double a = wmn[0][d], b = wmx[0][d];
        for (int w = 1; w < kSortWaves; ++w) {
            a = fmin(a, wmn[w][d]);
            b = fmax(b, wmx[w][d]);
        }
        f.tile_mm[6 * (size_t)blockIdx.x + d] = ord_enc(a);
        f.tile_mm[6 * (size_t)blockIdx.x + 3 + d] = ord_enc(b);
    }
}

// Per simulation: min/max over its tiles' partials (integer images: exact, order-free).
__global__ void __launch_bounds__(256) k_bbox_reduce(ForestDev f) {
    const SegDesc &sd = f.seg[blockIdx.x];
    __shared__ unsigned long long red[6][256];
    unsigned long long v[6] = {~0ull, ~0ull, ~0ull, 0ull, 0ull, 0ull};
    for (uint32_t t = threadIdx.x; t < sd.ntiles; t += 256) {
        const unsigned long long *p = f.tile_mm + 6 * (size_t)(sd.tile_base + t);
        for (int d = 0; d < 3; ++d) {
            v[d] = p[d] < v[d] ? p[d] : v[d];
            v[3 + d] = p[3 + d] > v[3 + d] ? p[3 + d] : v[3 + d];
        }
    }
    for (int d = 0; d < 6; ++d) red[d][threadIdx.x] = v[d];
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o)
            for (int d = 0; d < 3; ++d) {
                unsigned long long a = red[d][threadIdx.x + o], b = red[3 + d][threadIdx.x + o];
                if (a < red[d][threadIdx.x]) red[d][threadIdx.x] = a;
                if (b > red[3 + d][threadIdx.x]) red[3 + d][threadIdx.x] = b;
            }
        __syncthreads();
    }
    if (threadIdx.x < 3) {
        f.st[blockIdx.x].mn[threadIdx.x] = red[threadIdx.x][0];
        f.st[blockIdx.x].mx[threadIdx.x] = red[3 + threadIdx.x][0];
    }
    if (threadIdx.x == 0) f.st[blockIdx.x].nn = 0;
}

// =================================================================== keys ===
// q_d = floor(fl(x_d - lo_d) * 2^(21-k)); key = interleave with x the MSB of each digit.

__global__ void __launch_bounds__(kSortThreads) k_keys(ForestDev f, const double *pos) {
    const TileDesc td = f.tiles[blockIdx.x];
    __shared__ double lo_s[3], scale_s;
    if (threadIdx.x == 0) {
        SegState &st = f.st[td.seg];
        double lo[3], hi[3], ext = 0.0;
        for (int d = 0; d < 3; ++d) {
            lo[d] = ord_dec(st.mn[d]);
            hi[d] = ord_dec(st.mx[d]);
            double e = __dsub_rn(hi[d], lo[d]);
            if (e > ext) ext = e;
        }
        int k = 0;
        if (ext > 0.0) frexp(ext, &k);
        for (int d = 0; d < 3; ++d) lo_s[d] = lo[d];
        scale_s = ldexp(1.0, kMaxLevel - k);
        if (blockIdx.x == f.seg[td.seg].tile_base) {
            for (int d = 0; d < 3; ++d) {
                st.lo[d] = lo[d];
                st.cref[d] = 0.5 * lo[d] + 0.5 * hi[d];
            }
            st.k = k;
            st.L = ldexp(1.0, k);
        }
    }
    __syncthreads();
    const double scale = scale_s;
    const SegDesc &sd = f.seg[td.seg];
    const double *pb = seg_base(pos, sd.pos, sd, 3);
    const uint32_t j0 = td.start - sd.start;
    for (uint32_t j = threadIdx.x; j < td.count; j += kSortThreads) {
        size_t i = (size_t)td.start + j;
        uint64_t q[3];
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            double c = floor(__dmul_rn(__dsub_rn(pb[3 * ((size_t)j0 + j) + d], lo_s[d]), scale));
            c = fmin(fmax(c, 0.0), 2097151.0);
            q[d] = (uint64_t)c;
        }
        f.keys[i] = (spread3(q[0]) << 2) | (spread3(q[1]) << 1) | spread3(q[2]);
        f.idx[i] = (uint32_t)i;
    }
}

// =================================================================== sort ===
// Stable within a tile: items are ranked in element order with wave-level
// digit matching (8 ballots) and per-wave LDS counters.

__device__ __forceinline__ uint64_t match_digit(uint32_t dig, uint64_t valid) {
    uint64_t peers = valid;
#pragma unroll
    for (int b = 0; b < 8; ++b) {
        uint64_t m = __ballot((dig >> b) & 1u);
        peers &= ((dig >> b) & 1u) ? m : ~m;
    }
    return peers;
}



template <int T>
__global__ void __launch_bounds__(T) k_sort_hist(ForestDev f, const uint64_t *keys, int shift) {
    __shared__ uint32_t hist[(T / 64)][256];
    const TileDesc td = f.tiles[blockIdx.x];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    for (int d = lane; d < 256; d += 64) hist[wave][d] = 0;
    __syncthreads();
    const uint64_t lt = (1ull << lane) - 1ull;
    uint32_t dg[(kTile / T)];
    bool ok[(kTile / T)];
#pragma unroll
    for (int j = 0; j < (kTile / T); ++j) {
        const uint32_t e = (uint32_t)wave * 64 * (kTile / T) + (uint32_t)j * 64 + lane;
        ok[j] = e < td.count;
        dg[j] = ok[j] ? (uint32_t)(keys[(size_t)td.start + e] >> shift) & 255u : 0u;
    }
#pragma unroll
    for (int j = 0; j < (kTile / T); ++j) {
        const uint64_t peers = match_digit(dg[j], __ballot(ok[j]));
        if (ok[j] && (peers & lt) == 0) hist[wave][dg[j]] += (uint32_t)__popcll(peers);
    }
    __syncthreads();
    if (threadIdx.x < 256) {
        const uint32_t d = threadIdx.x;
        uint32_t t = 0;
#pragma unroll
        for (int w = 0; w < (T / 64); ++w) t += hist[w][d];
        f.cnt[256u * blockIdx.x + d] = t;
    }
}

// Digit d (one block per digit): exclusive scan of the tile counts over the tiles of
// each simulation (tiles of a simulation are contiguous), in place; the
// simulation's total of digit d goes to segtot[seg][d].
__global__ void __launch_bounds__(256) k_sort_colscan(ForestDev f) {
    __shared__ uint32_t w[4];
    __shared__ uint32_t last;
    const uint32_t d = blockIdx.x;
    uint32_t carry = 0;
    for (uint32_t c0 = 0; c0 < f.ntiles; c0 += 256) {
        const uint32_t j = c0 + threadIdx.x;
        const bool ok = j < f.ntiles;
        const uint32_t v = ok ? f.cnt[256u * j + d] : 0u;
        const uint32_t incl = block_inclusive_scan_256(v, w) + carry;
        const uint32_t excl = incl - v;
        uint32_t sid = 0;
        if (ok) {
            sid = f.tiles[j].seg;
            if (j == f.seg[sid].tile_base) f.segp[256u * sid + d] = excl;
        }
        if (threadIdx.x == 255) last = incl;
        __syncthreads();
        if (ok) {
            const SegDesc &sd = f.seg[sid];
            const uint32_t b = f.segp[256u * sid + d];
            f.cnt[256u * j + d] = excl - b;
            if (j == sd.tile_base + sd.ntiles - 1) f.segtot[256u * sid + d] = incl - b;
        }
        carry = last;
        __syncthreads();
    }
}

template <int T>
__global__ void __launch_bounds__(T) k_sort_scatter(ForestDev f, const uint64_t *kin, const uint32_t *iin,
                                                               uint64_t *kout, uint32_t *iout, int shift) {
    __shared__ uint64_t skey[kTile];
    __shared__ uint32_t sidx[kTile];
    __shared__ uint32_t whist[(T / 64)][256];
    __shared__ uint32_t lstart[256];
    __shared__ uint32_t gbase[256];
    __shared__ uint32_t wtot[(T / 64)];
    const TileDesc td = f.tiles[blockIdx.x];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const uint64_t lt = (1ull << lane) - 1ull;
    for (int d = lane; d < 256; d += 64) whist[wave][d] = 0;
    __syncthreads();

    uint64_t key[(kTile / T)];
    uint32_t idv[(kTile / T)];
    uint32_t rank[(kTile / T)];
#pragma unroll
    for (int j = 0; j < (kTile / T); ++j) {
        uint32_t e = (uint32_t)wave * 64 * (kTile / T) + (uint32_t)j * 64 + lane;
        bool valid = e < td.count;
        key[j] = valid ? kin[(size_t)td.start + e] : 0ull;
        idv[j] = valid ? iin[(size_t)td.start + e] : 0u;
    }
#pragma unroll
    for (int j = 0; j < (kTile / T); ++j) {
        uint32_t e = (uint32_t)wave * 64 * (kTile / T) + (uint32_t)j * 64 + lane;
        bool valid = e < td.count;
        uint32_t dig = (uint32_t)(key[j] >> shift) & 255u;
        uint64_t peers = match_digit(dig, __ballot(valid));
        uint32_t before = valid ? whist[wave][dig] : 0u;
        rank[j] = before + (uint32_t)__popcll(peers & lt);
        if (valid && (peers & lt) == 0) whist[wave][dig] = before + (uint32_t)__popcll(peers);
    }
    __syncthreads();
    // per digit (threads 0..255): offsets of the waves, tile-local start, global base; every
    // thread takes part in the block scans (the others with 0, after all digits)
    {
        const uint32_t d = threadIdx.x;
        uint32_t tot = 0;
        uint32_t c[(T / 64)];
        if (d < 256) {
#pragma unroll
            for (int w = 0; w < (T / 64); ++w) {
                c[w] = whist[w][d];
                tot += c[w];
            }
        }
        const uint32_t inc = block_inclusive_scan_256(tot, wtot);
        const SegDesc &sd = f.seg[td.seg];
        const uint32_t tot_d = d < 256 ? f.segtot[256u * td.seg + d] : 0u;
        const uint32_t dinc = block_inclusive_scan_256(tot_d, wtot);
        if (d < 256) {
            lstart[d] = inc - tot;
            uint32_t run = 0;
#pragma unroll
            for (int w = 0; w < (T / 64); ++w) {
                whist[w][d] = run;
                run += c[w];
            }
            gbase[d] = sd.start + (dinc - tot_d) + f.cnt[256u * blockIdx.x + d];
        }
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < (kTile / T); ++j) {
        uint32_t e = (uint32_t)wave * 64 * (kTile / T) + (uint32_t)j * 64 + lane;
        if (e < td.count) {
            uint32_t dig = (uint32_t)(key[j] >> shift) & 255u;
            uint32_t p = lstart[dig] + whist[wave][dig] + rank[j];
            skey[p] = key[j];
            sidx[p] = idv[j];
        }
    }
    __syncthreads();
    for (uint32_t q = threadIdx.x; q < td.count; q += T) {
        uint64_t k = skey[q];
        uint32_t dig = (uint32_t)(k >> shift) & 255u;
        uint32_t o = gbase[dig] + (q - lstart[dig]);
        kout[o] = k;
        iout[o] = sidx[q];
    }
}

// ================================================================ permute ===

// One pass over the sorted rows r in [0, ntot]: the state in key order (gathered
// from the packed records), the common-prefix level of neighbouring keys (-1 at
// the first row of each simulation and at the end), the cleared node-start masks,
// and the node tables cleared for the fill pass (two ids per row: the node
// capacity is twice the rows).
__global__ void k_permute_lcp(ForestDev f) {
    const uint32_t r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r > f.ntot) return;
    for (uint32_t g = r; g < f.mcap; g += f.ntot + 1) {
        f.nchild[g] = 0;
        f.nparent[g] = kNone;
        f.ncrank[g] = kNone;
    }
    int8_t v = -1;
    if (r < f.ntot) {
        f.mask[r] = 0;
        const uint32_t s = f.segid[r];
        const SegDesc &sd = f.seg[s];
        if (r != sd.start) {
            const uint64_t x = f.keys[r - 1] ^ f.keys[r];
            v = x == 0 ? (int8_t)kMaxLevel : (int8_t)((__clzll((long long)x) - 1) / 3);
        }
        const size_t li = f.idx[r] - sd.start;
        if (li >= sd.n) {   // cannot happen after a correct sort
            flag_tree(f);
        } else {
            const double4 p = f.pk[sd.start + li];
            f.spos[3 * (size_t)r] = p.x;
            f.spos[3 * (size_t)r + 1] = p.y;
            f.spos[3 * (size_t)r + 2] = p.z;
            f.smass[r] = p.w;
        }
    }
    f.lcp[r] = v;
}

// ==================================================================== lcp ===
// lcp[p], p in [0, ntot]: octant digits shared by keys p-1 and p (21 if equal),
// -1 at the first row of a simulation and at ntot.  Also clears mask.


// ============================================================ node marking ===

struct Seg { uint32_t lo, hi, cap; };

__device__ __forceinline__ Seg seg_of(const ForestDev &f, uint32_t r) {
    const SegDesc &sd = f.seg[f.segid[r]];
    Seg s;
    s.lo = sd.start;
    s.hi = sd.start + sd.n;
    s.cap = (uint32_t)sd.leaf_cap;
    return s;
}

// Level of the leaf holding row r: one below the deepest cube (level <= 20) with more
// than cap particles.  Returns 0 when the whole simulation fits one leaf.
__device__ inline int leaf_level(const ForestDev &f, uint32_t r, const Seg &sg) {
    if (sg.hi - sg.lo <= sg.cap) return 0;
    int h;
    if (sg.cap == 1) {
        int a = f.lcp[r], b = f.lcp[r + 1];
        h = a > b ? a : b;
        if (h > kMaxLevel - 1) h = kMaxLevel - 1;
    } else {
        int lo = 0, hi = kMaxLevel;          // cnt(lo) > cap, level hi excluded
        while (hi - lo > 1) {
            int mid = (lo + hi) >> 1;
            uint32_t a = cell_left(f.keys, r, mid, sg.lo);
            uint32_t b = cell_right(f.keys, r, mid, sg.hi);
            if (b - a > sg.cap) lo = mid; else hi = mid;
        }
        h = lo;
    }
    return h + 1;
}

__device__ __forceinline__ uint32_t node_id(const ForestDev &f, uint32_t first, int level) {
    return f.base[first] + (uint32_t)__popc(f.mask[first] & ((1u << level) - 1u));
}

// Mark pass: every node sets bit `level` of mask[first].  The row that starts a
// leaf keeps the leaf's level (rlam) and end (idx_alt); the boundary row that
// owns an internal node keeps the node's rows [q, R) (keys_alt), for the fill.
__global__ void __launch_bounds__(256) k_mark(ForestDev f) {
    uint32_t r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r < f.ntot) {
        const Seg sg = seg_of(f, r);
        uint2 *own = reinterpret_cast<uint2 *>(f.keys_alt);
        // cube edges: a neighbour sharing fewer than L digits (lcp < L) closes a level-L cube
        // at once; only longer runs need the key search
        const int l = f.lcp[r], lr = f.lcp[r + 1];
        // leaf holding r, marked by its first row
        const int lam = leaf_level(f, r, sg);
        const uint32_t a = lam == 0 ? sg.lo : (l < lam ? r : cell_left(f.keys, r, lam, sg.lo));
        if (a == r) {
            atomicOr(&f.mask[a], 1u << lam);
            f.rlam[r] = (uint8_t)lam;
            f.idx_alt[r] = lam == 0 ? sg.hi : (lr < lam ? r + 1 : cell_right(f.keys, r, lam, sg.hi));
        }
        // inner node owned by boundary r (the first split of its cube)
        uint2 node = make_uint2(kNone, kNone);
        if (l >= 0 && l < kMaxLevel) {
            const uint32_t q = f.lcp[r - 1] <= l ? r - 1 : cell_left(f.keys, r - 1, l + 1, sg.lo);
            if (q == sg.lo || f.lcp[q] < l) {
                const uint32_t R = lr < l ? r + 1 : cell_right(f.keys, r, l, sg.hi);
                if (R - q > sg.cap) {
                    atomicOr(&f.mask[q], 1u << l);
                    node = make_uint2(q, R);
                }
            }
        }
        own[r] = node;
    }
}

constexpr uint32_t kInner = 0xFFFFFFFFu;   // nchild of an internal node until its children are linked


// Fill pass: node records (level, first rows, count) at their preorder ids.
__global__ void __launch_bounds__(256) k_fill(ForestDev f) {
    uint32_t r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r < f.ntot) {
        const uint32_t s = f.segid[r];
        const uint32_t lo = f.seg[s].start;
        const uint32_t m = f.mask[r];
        const uint2 node = reinterpret_cast<const uint2 *>(f.keys_alt)[r];
        if (node.x != kNone) {
            // internal node: a later boundary owns it; its first row q carries the mask bit
            const uint32_t q = node.x;
            const int l = f.lcp[r];
            const uint32_t g = node_id(f, q, l);
            f.nlevel[g] = (uint8_t)l;
            f.nfirst[g] = q;
            f.ncount[g] = node.y - q;
            f.nchild[g] = kInner;
            if (q == lo && (f.mask[q] & ((1u << l) - 1u)) == 0) {
                f.nparent[g] = kNone;
                f.ncrank[g] = s;
                f.st[s].nbase = g;
            }
        }
        if (m != 0) {
            // the leaf starting at r, if any: the deepest node starting at r
            const int lam = f.rlam[r];
            if (lam > kMaxLevel || m >> lam != 1u) {
                flag_tree(f);   // the deepest node starting at a row must be its leaf
            } else {
                const uint32_t g = node_id(f, r, lam);
                f.nlevel[g] = (uint8_t)lam;
                f.nfirst[g] = r;
                f.ncount[g] = f.idx_alt[r] - r;
                f.nchild[g] = 0;
                if (r == lo && (m & ((1u << lam) - 1u)) == 0) {
                    f.nparent[g] = kNone;
                    f.ncrank[g] = s;
                    f.st[s].nbase = g;
                }
            }
        }
    }
}

// Child links.  In depth-first preorder the first child of internal node g is
// g + 1 and each next sibling is the first node starting at the row after the
// previous child's rows (base[end]); the walk over them gives each child its
// parent and octant rank, and g its child count.
__global__ void __launch_bounds__(256) k_link(ForestDev f) {
    const uint32_t g = blockIdx.x * blockDim.x + threadIdx.x;
    const uint32_t mtot = f.base[f.ntot];
    if (g >= mtot || f.nchild[g] != kInner) return;
    const uint32_t R = f.nfirst[g] + f.ncount[g];
    uint32_t c = g + 1, k = 0;
    bool bad = false;
    for (;;) {
        if (c >= mtot || k >= 8) { bad = true; break; }
        f.nparent[c] = g;
        f.ncrank[c] = k++;
        const uint32_t a = f.nfirst[c], e = a + f.ncount[c];
        if (e >= R || e > f.ntot || e <= a) { bad = e != R; break; }
        c = f.base[e];
    }
    if (bad || k < 2) {
        flag_tree(f);
        k = 0;
    }
    f.nchild[g] = k;
}

// Walk slots: roots take slots [0, nseg); the children of node g take
// [nseg + cs[g], nseg + cs[g] + nchild[g]) in octant order.  Each block also
// lists its internal nodes sorted by level (a counting sort in LDS) with the
// slots the upward pass needs.
__global__ void __launch_bounds__(256) k_slots(ForestDev f) {
    __shared__ uint32_t hist[kMaxLevel + 1], start[kMaxLevel + 2];
    if (threadIdx.x <= kMaxLevel) hist[threadIdx.x] = 0;
    __syncthreads();
    const uint32_t g = blockIdx.x * blockDim.x + threadIdx.x;
    const uint32_t mtot = f.base[f.ntot];
    int lvl = -1;
    uint32_t rank = 0;
    uint4 entry = make_uint4(0, 0, 0, 0);
    if (g < mtot) {
        const uint32_t p = f.nparent[g];
        const uint32_t rk = f.ncrank[g];
        uint32_t sl = kNone;
        if (p == kNone) {
            if (rk < f.nseg) {
                sl = rk;
                // the simulation's node count, from its root
                const SegDesc &sd = f.seg[rk];
                f.st[rk].nn = f.base[sd.start + sd.n] - f.base[sd.start];
            }
        } else if (p < mtot && rk < 8) {
            sl = f.nseg + f.cs[p] + rk;
        }
        if (sl >= mtot) {
            flag_tree(f);
        } else {
            f.slot_of[g] = sl;
            const uint32_t nc = f.nchild[g];
            if (nc != 0) {
                lvl = f.nlevel[g];
                rank = atomicAdd(&hist[lvl], 1u);
                const uint32_t quad = f.uQ ? f.seg[f.segid[f.nfirst[g]]].quad : 0u;
                entry = make_uint4(sl, f.nseg + f.cs[g], nc, quad);
            }
        }
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t run = 0;
        for (int l = 0; l <= kMaxLevel; ++l) {
            start[l] = run;
            run += hist[l];
        }
        start[kMaxLevel + 1] = run;
    }
    __syncthreads();
    if (threadIdx.x <= kMaxLevel + 1)
        f.blk_lvl[(size_t)blockIdx.x * (kMaxLevel + 2) + threadIdx.x] = (uint16_t)start[threadIdx.x];
    if (lvl >= 0) f.lvl_list[(size_t)blockIdx.x * blockDim.x + start[lvl] + rank] = entry;
}


hipError_t launch_build(const ForestDev &f, const double *pos, const double *mass, hipStream_t s) {
    hipLaunchKernelGGL(k_bbox, dim3(f.ntiles), dim3(kSortThreads), 0, s, f, pos, mass);
    hipLaunchKernelGGL(k_bbox_reduce, dim3(f.nseg), dim3(256), 0, s, f);
    hipLaunchKernelGGL(k_keys, dim3(f.ntiles), dim3(kSortThreads), 0, s, f, pos);
    // 8 stable passes of 8 bits: the result returns to (keys, idx)
    uint64_t *kin = f.keys, *kout = f.keys_alt;
    uint32_t *iin = f.idx, *iout = f.idx_alt;
    for (int pass = 0; pass < 8; ++pass) {
        int shift = 8 * pass;
        // the histogram takes 1024 threads per tile; the scatter (67 KB of LDS at 1024 threads)
        // does too while there are at most two tiles per compute unit, and otherwise keeps
        // more tiles resident with 256-thread blocks
        hipLaunchKernelGGL(k_sort_hist<1024>, dim3(f.ntiles), dim3(1024), 0, s, f, kin, shift);
        hipLaunchKernelGGL(k_sort_colscan, dim3(256), dim3(256), 0, s, f);
        if (f.ntiles <= 512)
            hipLaunchKernelGGL(k_sort_scatter<1024>, dim3(f.ntiles), dim3(1024), 0, s, f, kin, iin, kout, iout, shift);
        else
            hipLaunchKernelGGL(k_sort_scatter<256>, dim3(f.ntiles), dim3(256), 0, s, f, kin, iin, kout, iout, shift);
        uint64_t *tk = kin; kin = kout; kout = tk;
        uint32_t *ti = iin; iin = iout; iout = ti;
    }
    const unsigned nb = (f.ntot + 255) / 256;
    hipLaunchKernelGGL(k_permute_lcp, dim3((f.ntot + 1 + 255) / 256), dim3(256), 0, s, f);
    hipLaunchKernelGGL(k_mark, dim3(nb), dim3(256), 0, s, f);
    hipError_t e = scan_exclusive(f.mask, f.ntot, f.base, f.scan_tmp, 1, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_fill, dim3(nb), dim3(256), 0, s, f);
    const unsigned mb = (f.mcap + 255) / 256;
    hipLaunchKernelGGL(k_link, dim3(mb), dim3(256), 0, s, f);
    e = scan_exclusive(f.nchild, f.mcap, f.cs, f.scan_tmp, 0, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_slots, dim3(mb), dim3(256), 0, s, f);
    return hipGetLastError();
}

// ================================================================= upward ===

// Upward pass, level by level from the deepest level: a launch sums the leaves
// (particles in key order), then one launch per level sums each internal node's
// children in octant order, over that level's node list.  The kernel
// boundaries order the levels; no device-scope fences are needed.

__global__ void k_up_leaf(ForestDev f) {
    const uint32_t g = blockIdx.x * blockDim.x + threadIdx.x;
    const uint32_t mtot = f.base[f.ntot];
    if (g >= mtot || f.nchild[g] != 0) return;
    const uint32_t a = f.nfirst[g], b = a + f.ncount[g];
    const uint32_t sl = f.slot_of[g];
    if (a >= f.ntot || b > f.ntot || b <= a || sl >= mtot) { flag_tree(f); return; }
    double M = 0.0, Sx = 0.0, Sy = 0.0, Sz = 0.0;
    for (uint32_t r = a; r < b; ++r) {
        const double m = f.smass[r];
        M = __dadd_rn(M, m);
        Sx = __dadd_rn(Sx, __dmul_rn(m, f.spos[3 * (size_t)r]));
        Sy = __dadd_rn(Sy, __dmul_rn(m, f.spos[3 * (size_t)r + 1]));
        Sz = __dadd_rn(Sz, __dmul_rn(m, f.spos[3 * (size_t)r + 2]));
    }
    f.uM[sl] = M;
    f.uS[3 * (size_t)sl] = Sx;
    f.uS[3 * (size_t)sl + 1] = Sy;
    f.uS[3 * (size_t)sl + 2] = Sz;
    if (f.uQ && f.seg[f.segid[a]].quad) {
        // second moments about the leaf's centre of mass, from its particles in key order
        const double cx = Sx / M, cy = Sy / M, cz = Sz / M;
        double q[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
        for (uint32_t r = a; r < b; ++r) {
            const double m = f.smass[r];
            const double x = f.spos[3 * (size_t)r] - cx, y = f.spos[3 * (size_t)r + 1] - cy,
                         z = f.spos[3 * (size_t)r + 2] - cz;
            q[0] += m * x * x;
            q[1] += m * y * y;
            q[2] += m * z * z;
            q[3] += m * x * y;
            q[4] += m * x * z;
            q[5] += m * y * z;
        }
        for (int k = 0; k < 6; ++k) f.uQ[6 * (size_t)sl + k] = q[k];
    }
}

// One wavefront per block of 256 node ids: its level-`level` internal nodes,
// whose children occupy consecutive walk slots.
__global__ void __launch_bounds__(256) k_up_level(ForestDev f, int level, uint32_t nblk) {
    const uint32_t lane = threadIdx.x & 63;
    const uint32_t mtot = f.base[f.ntot];
    for (uint32_t b = blockIdx.x * 4 + (threadIdx.x >> 6); b < nblk; b += gridDim.x * 4) {
        const uint16_t *bl = f.blk_lvl + (size_t)b * (kMaxLevel + 2);
        const uint32_t begin = bl[level], end = bl[level + 1];
        for (uint32_t i = begin + lane; i < end; i += 64) {
            const uint4 e = f.lvl_list[(size_t)b * 256 + i];
            const uint32_t sl = e.x, c0 = e.y, nc = e.z;
            if (sl >= mtot || nc < 2 || nc > 8 || c0 + nc > mtot) { flag_tree(f); continue; }
            double M = 0.0, Sx = 0.0, Sy = 0.0, Sz = 0.0;
            for (uint32_t k = 0; k < nc; ++k) {
                const size_t c = c0 + k;
                M = __dadd_rn(M, f.uM[c]);
                Sx = __dadd_rn(Sx, f.uS[3 * c]);
                Sy = __dadd_rn(Sy, f.uS[3 * c + 1]);
                Sz = __dadd_rn(Sz, f.uS[3 * c + 2]);
            }
            f.uM[sl] = M;
            f.uS[3 * (size_t)sl] = Sx;
            f.uS[3 * (size_t)sl + 1] = Sy;
            f.uS[3 * (size_t)sl + 2] = Sz;
            if (e.w) {
                // second moments by the parallel-axis rule: each child's moments about its own
                // centre plus its mass times the offset of that centre from this node's
                const double cx = Sx / M, cy = Sy / M, cz = Sz / M;
                double q[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
                for (uint32_t k = 0; k < nc; ++k) {
                    const size_t c = c0 + k;
                    const double mc = f.uM[c];
                    // a massless child adds nothing (its own centre, 0/0, is undefined)
                    if (mc == 0.0) continue;
                    const double x = f.uS[3 * c] / mc - cx, y = f.uS[3 * c + 1] / mc - cy,
                                 z = f.uS[3 * c + 2] / mc - cz;
                    const double *qc = f.uQ + 6 * c;
                    q[0] += qc[0] + mc * x * x;
                    q[1] += qc[1] + mc * y * y;
                    q[2] += qc[2] + mc * z * z;
                    q[3] += qc[3] + mc * x * y;
                    q[4] += qc[4] + mc * x * z;
                    q[5] += qc[5] + mc * y * z;
                }
                for (int k = 0; k < 6; ++k) f.uQ[6 * (size_t)sl + k] = q[k];
            }
        }
    }
}

// r^2 of the opening test r^2 < theta^2 D^2 of a level-`level` cube whose first
// key is `key`, centre of mass c and side s (paper section 3 uses the side;
// section 6 lists other ways of computing the criterion as future work).
// Cube geometry from the key: Q = the cube's integer corner (low 21 - level bits
// of each quantised coordinate cleared), h = L 2^-21, w = 2^(21 - level):
// corner lo + Q h, far corner lo + (Q + w) h, centre lo + (2Q + w) h/2, each one
// rounding of an exact product.  b_max: e = max(c - corner, far - c) per axis,
// r^2 = (ex^2 + ey^2) + ez^2.  Offset (D > s/theta + delta): delta = |c - centre|,
// r = s + theta delta.
__device__ double open_radius2(uint64_t key, int level, const double c[3], double s, const SegState &st,
                               const SegDesc &sd) {
    if (sd.open == kOpenSide) return __dmul_rn(s, s);
    const double h = ldexp(st.L, -kMaxLevel);
    const uint32_t w = 1u << (kMaxLevel - level);
    double e[3];
    for (int a = 0; a < 3; ++a) {
        const uint32_t Q = compact3(key >> (2 - a)) & ~(w - 1u);
        if (sd.open == kOpenBmax) {
            const double lo = __dadd_rn(st.lo[a], __dmul_rn((double)Q, h));
            const double hi = __dadd_rn(st.lo[a], __dmul_rn((double)(Q + w), h));
            const double u = __dsub_rn(c[a], lo), v = __dsub_rn(hi, c[a]);
            e[a] = u > v ? u : v;
        } else {
            const double ctr = __dadd_rn(st.lo[a], __dmul_rn((double)(2u * Q + w), __dmul_rn(0.5, h)));
            e[a] = __dsub_rn(c[a], ctr);
        }
    }
    const double e2 = __dadd_rn(__dadd_rn(__dmul_rn(e[0], e[0]), __dmul_rn(e[1], e[1])), __dmul_rn(e[2], e[2]));
    if (sd.open == kOpenBmax) return e2;
    const double r = __dadd_rn(s, __dmul_rn(sd.theta, __dsqrt_rn(e2)));
    return __dmul_rn(r, r);
}

// com = S / M, then the walk record of the node at its slot.
__global__ void k_records(ForestDev f) {
    uint32_t g = blockIdx.x * blockDim.x + threadIdx.x;
    uint32_t mtot = f.base[f.ntot];
    if (g >= mtot) return;
    const uint32_t sl = f.slot_of[g];
    if (sl >= mtot) {
        flag_tree(f);
        return;
    }
    const double M = f.uM[sl];
    double c[3];
    for (int d = 0; d < 3; ++d) c[d] = f.uS[3 * (size_t)sl + d] / M;
    const uint32_t sid = f.segid[f.nfirst[g]];
    const SegDesc &sd = f.seg[sid];
    const SegState &st = f.st[sid];
    const int level = f.nlevel[g];
    const uint32_t nc = f.nchild[g];
    const uint32_t link = nc ? f.nseg + f.cs[g] : f.nfirst[g];
    const uint32_t cnt = nc ? nc : (f.ncount[g] | kLeafBit);
    if ((nc && (nc < 2 || nc > 8 || link + nc > mtot)) ||
        (!nc && (link >= f.ntot || f.ncount[g] == 0 || link + f.ncount[g] > f.ntot))) {
        flag_tree(f);
        return;
    }
    const double s = ldexp(st.L, -level);
    const double r2 = open_radius2(f.keys[f.nfirst[g]], level, c, s, st, sd);
    if (sd.precision == 1) {
        WRec32 w;
        w.cx = c[0];
        w.cy = c[1];
        w.cz = c[2];
        w.m = (float)M;
        // FP32 opening test: accept iff |d|^2 + eps^2 > r^2 / theta^2 + eps^2 (the walk adds
        // its rounding band); S is kept only when it and eps^2 are well inside the FP32 range,
        // otherwise every test of this node is decided in FP64.
        const double u = 5.9604644775390625e-8;   // 2^-24
        const double eps2 = sd.eps * sd.eps;
        const float eps2f = (float)eps2;
        const bool eps_ok = eps2 == 0.0 || (eps2 > 1e-30 && eps2 < 1e30 && eps2f > 0.0f);
        if (sd.theta == 0.0) {
            w.Sh = INFINITY;   // nothing is ever accepted
            w.band0 = 0.0f;
            w.band1 = 0.0f;
        } else {
            const double S = r2 / (sd.theta * sd.theta) + eps2;
            if (eps_ok && r2 > 1e-30 && S > 1e-30 && S < 1e30) {
                w.Sh = (float)(S * (1.0 + 8.0 * u));   // the walk's band edges start from S (1 + 8u)
                w.band0 = (float)(16.0 * u * S * (1.0 + 1e-6));
                w.band1 = (float)(8.0 * u * sqrt(r2) / sd.theta * (1.0 + 1e-6));
            } else {
                w.Sh = 0.0f;
                w.band0 = INFINITY;
                w.band1 = 0.0f;
            }
        }
        w.link = link;
        w.cnt = cnt;
        w.gid = g;
        w.level = (uint32_t)level;
        w.r2 = r2;
        f.w32[sl] = w;
        if (sd.quad) {
            const double *q = f.uQ + 6 * (size_t)sl;
            f.q32[2 * (size_t)sl] = make_float4((float)q[0], (float)q[1], (float)q[2], (float)q[3]);
            f.q32[2 * (size_t)sl + 1] = make_float4((float)q[4], (float)q[5], (float)(q[0] + q[1] + q[2]), 0.0f);
        }
    } else {
        WRec64 w;
        w.x = c[0];
        w.y = c[1];
        w.z = c[2];
        w.m = M;
        w.S = r2;
        w.link = link;
        w.cnt = cnt;
        w.gid = g;
        w.level = (uint32_t)level;
        w.pad = 0.0;
        f.w64[sl] = w;
        if (sd.quad)
            for (int k = 0; k < 6; ++k) f.q64[6 * (size_t)sl + k] = f.uQ[6 * (size_t)sl + k];
    }
}

// Group criterion: each body's group is the largest cube holding at most kGroupCap
// bodies (its parent holds more, or it is the root); a leaf of more than kGroupCap
// coincident bodies at the depth limit is cut into runs of kGroupCap in key order.
// One thread per group cube writes the group's bounding box (FP64 min and max of
// its bodies' coordinates) to each member's row.
__global__ void __launch_bounds__(256) k_group_boxes(ForestDev f) {
    const uint32_t g = blockIdx.x * blockDim.x + threadIdx.x;
    const uint32_t mtot = f.base[f.ntot];
    if (g >= mtot) return;
    const uint32_t first = f.nfirst[g], cnt = f.ncount[g];
    if (first >= f.ntot || cnt == 0 || cnt > f.ntot - first) return;   // flagged by the build
    if (!f.seg[f.segid[first]].group) return;
    const uint32_t par = f.nparent[g];
    const bool top = par == kNone || (par < mtot && f.ncount[par] > (uint32_t)kGroupCap);
    if (!top || (cnt > (uint32_t)kGroupCap && f.nchild[g] != 0)) return;
    for (uint32_t r0 = first; r0 < first + cnt; r0 += kGroupCap) {
        const uint32_t r1 = r0 + kGroupCap < first + cnt ? r0 + kGroupCap : first + cnt;
        double lo[3], hi[3];
        for (int d = 0; d < 3; ++d) lo[d] = hi[d] = f.spos[3 * (size_t)r0 + d];
        for (uint32_t r = r0 + 1; r < r1; ++r)
            for (int d = 0; d < 3; ++d) {
                const double v = f.spos[3 * (size_t)r + d];
                lo[d] = v < lo[d] ? v : lo[d];
                hi[d] = v > hi[d] ? v : hi[d];
            }
        for (uint32_t r = r0; r < r1; ++r)
            for (int d = 0; d < 3; ++d) {
                f.gbox[6 * (size_t)r + d] = lo[d];
                f.gbox[6 * (size_t)r + 3 + d] = hi[d];
            }
    }
}

hipError_t launch_upward(const ForestDev &f, hipStream_t s) {
    const unsigned mb = (f.mcap + 255) / 256;
    if (f.gbox) hipLaunchKernelGGL(k_group_boxes, dim3(mb), dim3(256), 0, s, f);
    hipLaunchKernelGGL(k_up_leaf, dim3(mb), dim3(256), 0, s, f);
    // one wavefront per list block; the lists cover the node ids [0, mcap) in blocks of 256
    const unsigned nblk = mb;
    const unsigned lb = (nblk + 3) / 4;   // one wavefront per list block
    for (int l = kMaxLevel - 1; l >= 0; --l)
        hipLaunchKernelGGL(k_up_level, dim3(lb), dim3(256), 0, s, f, l, nblk);
    hipLaunchKernelGGL(k_records, dim3(mb), dim3(256), 0, s, f);
    return hipGetLastError();
}

// ================================================================= export ===
// Canonical arrays of simulation `seg` in its own numbering (ranks and node ids
// relative to the simulation).

__global__ void k_export_particles(ForestDev f, uint32_t seg, uint64_t *keys, uint32_t *perm) {
    const SegDesc &sd = f.seg[seg];
    uint32_t r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= sd.n) return;
    if (keys) keys[r] = f.keys[sd.start + r];
    if (perm) perm[r] = f.idx[sd.start + r] - sd.start;
}

__global__ void k_export_nodes(ForestDev f, uint32_t seg, int32_t *level, uint32_t *first, uint32_t *count,
                               int32_t *parent, double *M, double *com) {
    const SegDesc &sd = f.seg[seg];
    const SegState &st = f.st[seg];
    uint32_t j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= st.nn) return;
    uint32_t g = st.nbase + j;
    if (level) level[j] = f.nlevel[g];
    if (first) first[j] = f.nfirst[g] - sd.start;
    if (count) count[j] = f.ncount[g];
    if (parent) parent[j] = f.nparent[g] == kNone ? -1 : (int32_t)(f.nparent[g] - st.nbase);
    // mass and centre of mass by walk slot, the centre divided exactly as the records do
    const uint32_t sl = f.slot_of[g];
    if (M) M[j] = f.uM[sl];
    if (com)
        for (int d = 0; d < 3; ++d) com[3 * (size_t)j + d] = f.uS[3 * (size_t)sl + d] / f.uM[sl];
}

hipError_t launch_export(const ForestDev &f, uint32_t seg, uint64_t *keys, uint32_t *perm, int32_t *level,
                         uint32_t *first, uint32_t *count, int32_t *parent, double *M, double *com,
                         hipStream_t s) {
    hipLaunchKernelGGL(k_export_particles, dim3((f.ntot + 255) / 256), dim3(256), 0, s, f, seg, keys, perm);
    hipLaunchKernelGGL(k_export_nodes, dim3((f.mcap + 255) / 256), dim3(256), 0, s, f, seg, level, first, count,
                       parent, M, com);
    return hipGetLastError();
}

}  // namespace bh
