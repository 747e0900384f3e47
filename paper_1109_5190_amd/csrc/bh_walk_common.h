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

// Softened monopole factors in FP64 for x = |d|^2 + eps^2 > 0: w3 = m x^(-3/2) and (POT)
// mr = m x^(-1/2).  From the hardware estimate y of x^(-1/2) and its residual
// e = 1 - x y^2, m y^3 (1 + 3e/2) and m y (1 + e/2) are the first-order corrections:
// relative errors of about 7.5 and 1.5 times the square of the estimate's error, like
// one Newton step on y, but with two dependent operations fewer before the sums.
template <bool POT>
__device__ __forceinline__ void mono64(double x, double m, double &w3, double &mr) {
    const double y = __builtin_amdgcn_rsq(x);
    const double y2 = y * y;
    const double my = m * y;
    const double e = fma(-x, y2, 1.0);
    const double my3 = my * y2;
    w3 = fma(1.5 * my3, e, my3);
    if (POT) mr = fma(0.5 * my, e, my);
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

// Force sums of one lane's body in the FP32 walks and in their list replay: FP32
// partial sums folded into Kahan-compensated totals after at most kFlushWork
// terms, and the queue of opened leaves whose particles are taken as pairs after
// each stack entry (queued particles in queue order, then the leaves that did not
// fit, 64 particles at a time).  Pair terms are loaded and converted
// lane-parallel, then added one particle per pass.  STATS: pair counts,
// interaction-set checksums and the wavefront's pair iterations as well.
template <bool STATS, bool POT, bool SOFT>
struct Sums32 {
    const ForestDev &f;
    WaveLds32 &L;
    const int lane;
    const uint32_t r, gstart;          // this lane's row; the group's first row
    const double gx, gy, gz;           // the wavefront's reference point g
    const float tx, ty, tz, eps2;      // this lane's body relative to g; softening^2
    const uint64_t pair_base;          // STATS: checksum offset of particle terms (node count)
    const uint32_t seg_start;          // STATS: the simulation's first row
    float ax = 0.f, ay = 0.f, az = 0.f, ap = 0.f;      // partial sums
    float sx = 0.f, sy = 0.f, sz = 0.f, sp = 0.f;      // Kahan sums
    float cx = 0.f, cy = 0.f, cz = 0.f, cp = 0.f;      // Kahan compensations
    uint32_t work = 0;   // terms added to the partial sums since the last fold (wave-uniform)
    uint32_t qn = 0;     // queued leaf particles (wave-uniform)
    uint32_t nov = 0;    // leaves in L.ovf (wave-uniform)
    uint32_t np2p = 0;   // STATS: this body's particle terms
    uint32_t wwork = 0;  // STATS: the wavefront's child tests and pair iterations (uniform)
    uint64_t h = 0;      // STATS: this body's interaction-set checksum

    __device__ __forceinline__ void fold() {
        kahan_add(sx, cx, ax); ax = 0.f;
        kahan_add(sy, cy, ay); ay = 0.f;
        kahan_add(sz, cz, az); az = 0.f;
        if (POT) { kahan_add(sp, cp, ap); ap = 0.f; }
        work = 0;
    }
    __device__ __forceinline__ void pair(float px, float py, float pz, float pm) {
        const float dx = px - tx, dy = py - ty, dz = pz - tz;
        const float r2 = fmaf(dz, dz, fmaf(dy, dy, fmaf(dx, dx, eps2)));
        if (SOFT || r2 > 0.0f) {
            const float ri = __builtin_amdgcn_rsqf(r2);
            const float mr = pm * ri;
            const float w3 = mr * ri * ri;
            ax = fmaf(w3, dx, ax);
            ay = fmaf(w3, dy, ay);
            az = fmaf(w3, dz, az);
            if (POT) ap -= mr;
        }
    }
    __device__ __forceinline__ void count_pair(uint32_t jq) {
        if (STATS) {
            ++np2p;
            h += mix64(pair_base + (uint64_t)(f.idx[jq] - seg_start));
        }
    }
    __device__ __forceinline__ void pair_batch() {
        if (qn == 0) return;
        if (STATS) wwork += qn;
        if (work + qn > kFlushWork) fold();
        work += qn;
        if (!SOFT) {
            // without softening a pair can be far closer than the group's extent: each side
            // is split as x - g = hi + lo (FP32 pair), so the difference of a close pair,
            // (hi_j - hi_i) + (lo_j - lo_i), carries u |d| instead of u |x - g|
            const float tlx = (float)(__dsub_rn(f.spos[3 * (size_t)r], gx) - (double)tx);
            const float tly = (float)(__dsub_rn(f.spos[3 * (size_t)r + 1], gy) - (double)ty);
            const float tlz = (float)(__dsub_rn(f.spos[3 * (size_t)r + 2], gz) - (double)tz);
            for (uint32_t k0 = 0; k0 < qn; k0 += 32) {
                const uint32_t nb = qn - k0 < 32u ? qn - k0 : 32u;
                wave_sync();
                if ((uint32_t)lane < nb) {
                    const size_t j = L.irank[k0 + lane];
                    const double ex_ = __dsub_rn(f.spos[3 * j], gx), ey = __dsub_rn(f.spos[3 * j + 1], gy),
                                 ez = __dsub_rn(f.spos[3 * j + 2], gz);
                    const float hx = (float)ex_, hy = (float)ey, hz = (float)ez;
                    L.pst[2 * lane] = make_float4(hx, hy, hz, (float)f.smass[j]);
                    L.pst[2 * lane + 1] = make_float4((float)(ex_ - (double)hx), (float)(ey - (double)hy),
                                                      (float)(ez - (double)hz), 0.0f);
                }
                wave_sync();
                for (uint32_t k = 0; k < nb; ++k) {
                    const uint32_t jq = uni(L.irank[k0 + k]);
                    const uint64_t m = uni64(L.imask[k0 + k]) & ~self_bit(jq, gstart);
                    if (in_mask(m)) {
                        const float4 ph = L.pst[2 * k], pl = L.pst[2 * k + 1];
                        const float dx = (ph.x - tx) + (pl.x - tlx), dy = (ph.y - ty) + (pl.y - tly),
                                    dz = (ph.z - tz) + (pl.z - tlz);
                        const float r2 = fmaf(dz, dz, fmaf(dy, dy, dx * dx));
                        if (r2 > 0.0f) {
                            const float ri = __builtin_amdgcn_rsqf(r2);
                            const float mr = ph.w * ri;
                            const float w3 = mr * ri * ri;
                            ax = fmaf(w3, dx, ax);
                            ay = fmaf(w3, dy, ay);
                            az = fmaf(w3, dz, az);
                            if (POT) ap -= mr;
                        }
                        count_pair(jq);
                    }
                }
            }
            qn = 0;
            wave_sync();
            return;
        }
        wave_sync();
        if ((uint32_t)lane < qn) {
            const size_t j = L.irank[lane];
            L.pst[lane] = make_float4((float)__dsub_rn(f.spos[3 * j], gx), (float)__dsub_rn(f.spos[3 * j + 1], gy),
                                      (float)__dsub_rn(f.spos[3 * j + 2], gz), (float)f.smass[j]);
        }
        wave_sync();
        for (uint32_t k = 0; k < qn; ++k) {
            const uint32_t jq = uni(L.irank[k]);
            const uint64_t m = uni64(L.imask[k]) & ~self_bit(jq, gstart);
            if (in_mask(m)) {
                const float4 p = L.pst[k];
                pair(p.x, p.y, p.z, p.w);
                count_pair(jq);
            }
        }
        qn = 0;
        wave_sync();
    }
    // an opened leaf of np particles from rank `first`, for the lanes of m
    __device__ __forceinline__ void queue_leaf(uint32_t first, uint32_t np, uint64_t m) {
        if (qn + np <= 64u) {
            if ((uint32_t)lane < np) {
                L.irank[qn + lane] = first + lane;
                L.imask[qn + lane] = m;
            }
            qn += np;
        } else {
            if (lane == 0) L.ovf[nov] = make_uint4(first, np, (uint32_t)m, (uint32_t)(m >> 32));
            ++nov;
        }
    }
    __device__ __forceinline__ void flush() {
        pair_batch();
        for (uint32_t k = 0; k < nov; ++k) {
            const uint4 lf = L.ovf[k];
            const uint32_t first = uni(lf.x), np = uni(lf.y);
            const uint64_t m = ((uint64_t)uni(lf.w) << 32) | uni(lf.z);
            for (uint32_t b0 = 0; b0 < np; b0 += 64) {
                const uint32_t nb = np - b0 < 64u ? np - b0 : 64u;
                wave_sync();
                if ((uint32_t)lane < nb) {
                    L.irank[lane] = first + b0 + lane;
                    L.imask[lane] = m;
                }
                qn = nb;
                pair_batch();
            }
        }
        nov = 0;
    }
};

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

// Stages the children of a stack entry (at most 8, consecutive walk slots from
// `link`) in LDS, lane c for child c: centre relative to the wavefront's reference
// point g, mass, link and count, and per variant the FP32 band edges (per-body
// test), the FP64 centre and r^2 (group criterion), node id and level (IDS), the
// second moments (QUAD).
template <bool IDS, bool QUAD, bool GROUP>
__device__ __forceinline__ void stage_children32(const ForestDev &f, WaveLds32 &L, int lane, uint32_t link,
                                                 uint32_t nch, double gx, double gy, double gz, float rw) {
    if ((uint32_t)lane < nch) {
        const ChildRecs32 cr(f.w32 + link);
        const uint32_t lane_off = (uint32_t)lane * (uint32_t)sizeof(WRec32);   // byte offset of lane c's record
        const v4u32 r0 = cr.q(lane_off, 0), r1 = cr.q(lane_off, 1), r2q = cr.q(lane_off, 2);
        WRec32 w;
        w.cx = as_f64(r0.x, r0.y);
        w.cy = as_f64(r0.z, r0.w);
        w.cz = as_f64(r1.x, r1.y);
        w.m = __uint_as_float(r1.z);
        w.Sh = __uint_as_float(r1.w);
        w.band0 = __uint_as_float(r2q.x);
        w.band1 = __uint_as_float(r2q.y);
        w.link = r2q.z;
        w.cnt = r2q.w;
        if (IDS || GROUP) {
            const v4u32 r3 = cr.q(lane_off, 3);
            w.gid = r3.x;
            w.level = r3.y;
            w.r2 = as_f64(r3.z, r3.w);
        }
        const float qx = (float)__dsub_rn(w.cx, gx);
        const float qy = (float)__dsub_rn(w.cy, gy);
        const float qz = (float)__dsub_rn(w.cz, gz);
        L.sa[lane] = make_float4(qx, qy, qz, w.m);
        if (GROUP) {
            L.x.g.cx[lane] = w.cx;
            L.x.g.cy[lane] = w.cy;
            L.x.g.cz[lane] = w.cz;
            L.x.g.r2[lane] = w.r2;
        } else {
            const float2 band = open_band(w, qx, qy, qz, rw);
            L.sbh[lane] = band.x;
            L.sbl[lane] = band.y;
        }
        L.sl[lane] = make_uint2(w.link, w.cnt);
        if (IDS) L.sc[lane] = make_uint2(w.gid, w.level);
        if (QUAD) {
            L.x.q.sq0[lane] = f.q32[2 * (size_t)(link + lane)];
            L.x.q.sq1[lane] = f.q32[2 * (size_t)(link + lane) + 1];
        }
    }
}

// The opening test of the cube at walk slot `slot` for the body of sorted row r,
// decided exactly in FP64 as the oracle evaluates it (lanes whose FP32 distance lies
// within the rounding band of the threshold).
__device__ __forceinline__ bool exact_accept32(const ForestDev &f, uint32_t slot, uint32_t r, double theta) {
    const WRec32 &wc = f.w32[slot];
    const double *xp = f.spos + 3 * (size_t)r;
    const double ex_ = __dsub_rn(wc.cx, xp[0]), ey = __dsub_rn(wc.cy, xp[1]), ez = __dsub_rn(wc.cz, xp[2]);
    const double ED2 = __dadd_rn(__dadd_rn(__dmul_rn(ex_, ex_), __dmul_rn(ey, ey)), __dmul_rn(ez, ez));
    return wc.r2 < __dmul_rn(__dmul_rn(theta, theta), ED2);
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

// Stages the children of a stack entry (FP64 walks), lane c for child c: centre and
// mass, r^2 of the opening test, link, count, node id and level, and (QUAD) the
// second moments.
template <bool QUAD, class Lds>
__device__ __forceinline__ void stage_children64(const ForestDev &f, Lds &L, int lane, uint32_t link, uint32_t nch) {
    if ((uint32_t)lane < nch) {
        const WRec64 *wb = f.w64 + link;   // wave-uniform base, lane offset
        const WRec64 &w = wb[lane];
        L.sa[lane] = make_double4(w.x, w.y, w.z, w.m);
        L.sS[lane] = w.S;
        L.sb[lane] = make_uint4(w.link, w.cnt, w.gid, w.level);
        if (QUAD)
            for (int k = 0; k < 6; ++k) L.sq[6 * lane + k] = f.q64[6 * (size_t)(link + lane) + k];
    }
}

// Force sums of one lane's body in the FP64 walks and in their list replay, and the
// queue of opened leaves whose particles are taken as pairs (32 at a time, loaded
// lane-parallel).  STATS: pair counts, interaction-set checksums and the
// wavefront's pair iterations as well.
template <bool STATS, bool POT, class Lds>
struct Sums64 {
    const ForestDev &f;
    Lds &L;
    const int lane;
    const uint32_t gstart;             // the group's first row
    const double tx, ty, tz, eps2;     // this lane's body; softening^2
    const uint64_t pair_base;          // STATS: checksum offset of particle terms (node count)
    const uint32_t seg_start;          // STATS: the simulation's first row
    double ax = 0.0, ay = 0.0, az = 0.0, ap = 0.0;
    uint32_t qn = 0;     // queued leaf particles (wave-uniform)
    uint32_t np2p = 0;   // STATS: this body's particle terms
    uint32_t wwork = 0;  // STATS: the wavefront's child tests and pair iterations (uniform)
    uint64_t h = 0;      // STATS: this body's interaction-set checksum

    __device__ __forceinline__ void pair(double px, double py, double pz, double pm) {
        const double dx = px - tx, dy = py - ty, dz = pz - tz;
        const double r2 = fma(dz, dz, fma(dy, dy, fma(dx, dx, eps2)));
        if (eps2 > 0.0 || r2 > 0.0) {
            double w3, mr = 0.0;
            mono64<POT>(r2, pm, w3, mr);
            ax = fma(w3, dx, ax);
            ay = fma(w3, dy, ay);
            az = fma(w3, dz, az);
            if (POT) ap -= mr;
        }
    }
    __device__ __forceinline__ void flush_leaves() {
        if (qn == 0) return;
        if (STATS) wwork += qn;
        for (uint32_t k0 = 0; k0 < qn; k0 += 32) {
            const uint32_t nb = qn - k0 < 32u ? qn - k0 : 32u;
            wave_sync();
            if ((uint32_t)lane < nb) {
                const size_t j = L.irank[k0 + lane];
                L.pst[lane] = make_double4(f.spos[3 * j], f.spos[3 * j + 1], f.spos[3 * j + 2], f.smass[j]);
            }
            wave_sync();
            for (uint32_t k = 0; k < nb; ++k) {
                const uint32_t jq = uni(L.irank[k0 + k]);
                const uint64_t m = uni64(L.imask[k0 + k]) & ~self_bit(jq, gstart);
                if (in_mask(m)) {
                    const double4 p = L.pst[k];
                    pair(p.x, p.y, p.z, p.w);
                    if (STATS) {
                        ++np2p;
                        h += mix64(pair_base + (uint64_t)(f.idx[jq] - seg_start));
                    }
                }
            }
        }
        qn = 0;
        wave_sync();
    }
    // an opened leaf of np particles from rank `first`, for the lanes of m: queued, after
    // the queue's particles when it does not fit; a leaf of more than 64 goes alone
    __device__ __forceinline__ void queue_leaf(uint32_t first, uint32_t np, uint64_t m) {
        if (np <= 64u) {
            if (qn + np > 64u) flush_leaves();
            if ((uint32_t)lane < np) {
                L.irank[qn + lane] = first + lane;
                L.imask[qn + lane] = m;
            }
            qn += np;
        } else {
            flush_leaves();
            for (uint32_t b0 = 0; b0 < np; b0 += 64) {
                const uint32_t nq = np - b0 < 64u ? np - b0 : 64u;
                if ((uint32_t)lane < nq) {
                    L.irank[lane] = first + b0 + lane;
                    L.imask[lane] = m;
                }
                qn = nq;
                flush_leaves();
            }
        }
    }
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
