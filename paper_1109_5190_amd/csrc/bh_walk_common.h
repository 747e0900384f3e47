// Shared device code of the force-walk kernels (per-body FP32 and FP64 walks,
// group-criterion walks, two-phase interaction lists): wave-level helpers,
// output descriptor and per-wavefront LDS layouts.
//
// Force walk on gfx950 (paper section 3: a remote cube is treated as one body
// only if its distance D from the body exceeds r/theta; the force stage is the
// computationally dominant part).
//
// One wavefront walks the tree for a group of 64 key-consecutive bodies, one
// body per lane.  The LDS stack holds (first child slot, number of children,
// lane mask) entries: a lane takes part in a cube only if it opened every
// ancestor, so each lane meets exactly the cubes of its own per-body walk and
// its interaction set is the per-body set of the method.
//
// Per popped entry, lane c loads child c's record (children are contiguous)
// and stages it in LDS; every lane then reads each child by broadcast.
// Per-lane predicates are formed as wave masks (one compare each, written to
// scalar registers) and combined with scalar logic, so a cube visit costs the
// distance, one fused opening test, two compares and, for accepting lanes,
// the softened monopole.  Opened leaves are queued (rank, lane mask) and their
// particles are loaded and converted 64 at a time.  No matrix cores: this is
// not a contraction.
//
// FP64 mode: the opening test s^2 < theta^2 D^2 is evaluated exactly as the
// oracle writes it; pair terms in FP64 with a Newton-refined rsqrt.
// FP32 mode: see k_walk32.
#pragma once
#include "bh_common.h"

namespace bh {

constexpr float kU32 = 5.9604644775390625e-8f;   // 2^-24
constexpr uint32_t kFlushWork = 64;              // pair terms (upper bound) between Kahan folds

__device__ __forceinline__ uint32_t uni(uint32_t v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ __forceinline__ uint64_t uni64(uint64_t v) {
    return ((uint64_t)uni((uint32_t)(v >> 32)) << 32) | uni((uint32_t)v);
}
__device__ __forceinline__ uint64_t ballot(bool p) { return __builtin_amdgcn_ballot_w64(p); }
__device__ __forceinline__ bool in_mask(uint64_t m) { return __builtin_amdgcn_inverse_ballot_w64(m); }

// Orders LDS traffic between lanes of one wavefront (no instruction is emitted:
// the wavefront executes in lockstep and its LDS operations complete in order;
// this only keeps the compiler from moving accesses across the hand-off).
__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ __forceinline__ void kahan_add(float &s, float &c, float v) {
    float y = v - c;
    float t = s + y;
    c = (t - s) - y;
    s = t;
}

// FP64 reciprocal square root: the hardware estimate refined by one Newton step
// y <- y + y (1 - x y^2) / 2 (the error is squared: well inside the 1e-10 force gate).
__device__ __forceinline__ double rsqrt64(double x) {
    const double y = __builtin_amdgcn_rsq(x);
    const double e = fma(-x * y, y, 1.0);
    return fma(0.5 * y, e, y);
}

__device__ __forceinline__ unsigned long long wave_sum_u(unsigned long long v) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// Self exclusion of a leaf pair: the lane whose body has rank jq (if in this group).
__device__ __forceinline__ uint64_t self_bit(uint32_t jq, uint32_t gstart) {
    uint32_t d = jq - gstart;
    return d < 64u ? (1ull << d) : 0ull;
}

struct WalkOut {
    double *acc, *pot;
    int64_t *n_mono, *n_p2p;
    uint64_t *hash;
    uint32_t wlo = 0, whi = 0xffffffffu;   // bodies written and counted: sorted ranks [wlo, whi)
    int64_t *work = nullptr;               // counting walks: the group's wavefront work per body
    int64_t *gwork = nullptr;              // counting walks: the wavefront work of each walk group
};

struct WaveLds32 {
    uint4 stk[kStackMax];
    float4 sa[8];          // child: centre rel g (x, y, z), mass
    float sbh[8], sbl[8];  // child: accept above sbh, decide in FP64 at or above sbl (this wavefront)
    uint2 sl[8];           // child: link, cnt
    uint2 sc[8];           // child: gid, level
    union {
        struct {
            float4 sq0[8], sq1[8];             // second moments (xx yy zz xy) (xz yz tr 0)
        } q;                                   // child, quadrupole walks
        struct {
            double cx[8], cy[8], cz[8], r2[8]; // FP64 centre of mass, r^2 of the test
        } g;                                   // child, group-criterion walks
    } x;
    uint32_t irank[64];    // queued leaf particles: rank
    uint64_t imask[64];    //                        lane mask
    float4 pst[64];        //                        position rel g, mass (unsoftened walks:
                           //                        32 particles as (hi, mass), (lo, 0))
    uint4 ovf[8];          // opened leaves that did not fit the queue: first rank, count, mask
};

// The FP32 walk records of a stack entry's children (at most 8, consecutive), read by
// lane c with buffer loads through one scalar resource whose base is the first
// child's record, so the per-lane address is a 32-bit offset (no 64-bit vector
// address arithmetic per entry); lanes past the 8 records read zeros.
typedef unsigned int v4u32 __attribute__((ext_vector_type(4)));
constexpr int kBufferWord3 = 0x00020000;   // buffer resource word 3 for raw 32-bit access (gfx9 family)
struct ChildRecs32 {
    __amdgpu_buffer_rsrc_t rs;
    __device__ __forceinline__ explicit ChildRecs32(const WRec32 *first)
        : rs(__builtin_amdgcn_make_buffer_rsrc(const_cast<WRec32 *>(first), (short)0, 8 * (int)sizeof(WRec32),
                                               kBufferWord3)) {}
    // record fields by 16-byte quarter: (cx, cy), (cz, m, Sh), (band0, band1, link, cnt), (gid, level, r2)
    __device__ __forceinline__ v4u32 q(uint32_t lane_off, uint32_t quarter) const {
        return __builtin_amdgcn_raw_buffer_load_b128(rs, (int)lane_off, (int)(16u * quarter), 0);
    }
};
__device__ __forceinline__ double as_f64(uint32_t lo, uint32_t hi) { return __hiloint2double((int)hi, (int)lo); }

// Opening thresholds of a child for one wavefront (FP32 walks): E2 > hi accepts,
// E2 < lo opens, anything between is decided in FP64.  q: the child's centre
// relative to the wavefront's reference g; rw: bound of |x - g|_inf over its bodies.
// With rho >= |q|_inf + rw and B = band0 + rho (band1 + 16 u^2 rho) the record's
// Sh >= S (1 + 6u) gives hi >= S + B and Sh (1 - 20u) - B (1 + 4u) <= S - B (lo
// rounds to a negative value, which never opens, when B exceeds it); B = inf
// (thresholds outside the FP32 range) sends every lane to FP64.
__device__ __forceinline__ float2 open_band(const WRec32 &w, float qx, float qy, float qz, float rw) {
    const float rho = fmaf(fmaxf(fabsf(qx), fmaxf(fabsf(qy), fabsf(qz))), 1.0f + 4.0f * kU32, rw);
    const float B = fmaf(rho, fmaf(16.0f * kU32 * kU32, rho, w.band1), w.band0);
    return make_float2(fmaf(B, 1.0f + 4.0f * kU32, w.Sh), fmaf(B, -(1.0f + 4.0f * kU32), w.Sh * (1.0f - 20.0f * kU32)));
}


template <bool QUAD>
struct WaveLds64 {
    uint4 stk[kStackMax];
    double4 sa[8];              // child: centre of mass, mass
    double sS[8];               // child: r^2 of the opening test
    uint4 sb[8];                // child: link, cnt, gid, level
    double sq[QUAD ? 8 * 6 : 1];// child (quadrupole walks): second moments (xx yy zz xy xz yz)
    uint32_t irank[64];         // queued leaf particles: rank
    uint64_t imask[64];         //                        lane mask
    double4 pst[32];            //                        position, mass (32 at a time)
};

// Group criterion (a variant, not the paper's per-body test): the cube is accepted
// for every body of a group iff r^2 < theta^2 D^2, D the distance from the cube's
// centre of mass c to the group's bounding box [lo, hi] (0 inside it), evaluated
// in FP64 exactly as the oracle writes it.
__device__ __forceinline__ bool group_accepts(double cx, double cy, double cz, double r2, const double lo[3],
                                              const double hi[3], double theta2) {
    const double c[3] = {cx, cy, cz};
    double dd[3];
    for (int k = 0; k < 3; ++k) {
        const double u = __dsub_rn(lo[k], c[k]), v = __dsub_rn(c[k], hi[k]);
        const double w = u > v ? u : v;
        dd[k] = w > 0.0 ? w : 0.0;
    }
    const double D2 = __dadd_rn(__dadd_rn(__dmul_rn(dd[0], dd[0]), __dmul_rn(dd[1], dd[1])), __dmul_rn(dd[2], dd[2]));
    return r2 < __dmul_rn(theta2, D2);
}

// Launchers of one kernel family each (defined in their own translation unit):
// shape, the launch shape (wavefronts per workgroup, each walking one 64-body group
// at a time, and the persistent bit); stats: the counting variant (totals, per-body
// counts and checksums); pot: also the potential.  Each launches the variants
// (expansion order, softening, opening test) its forest holds.
void launch_walk32_family(const ForestDev &f, const WalkOut &o, bool stats, bool pot, int shape, hipStream_t s);
void launch_walk64_family(const ForestDev &f, const WalkOut &o, bool stats, bool pot, int shape, hipStream_t s);

}  // namespace bh
