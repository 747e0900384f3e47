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
    float2 sb[8];          // child: accept above hi, decide in FP64 at or above lo (this wavefront)
    uint2 sl[8];           // child: link, cnt
    uint2 sc[8];           // child: gid, level
    float4 sq0[8], sq1[8]; // child (quadrupole walks): second moments (xx yy zz xy) (xz yz tr 0)
    uint32_t irank[64];    // queued leaf particles: rank
    uint64_t imask[64];    //                        lane mask
    float4 pst[64];        //                        position rel g, mass (unsoftened walks:
                           //                        32 particles as (hi, mass), (lo, 0))
};

// ------------------------------------------------------------- FP32 walk ---
// Each wavefront re-expresses coordinates relative to its own FP64 reference
// point g (its first body): FP32 differences then carry errors of order
// u |d| + u |x - g| rather than u |x - origin|.
//
// Opening test in FP32: for theta > 0 the method accepts iff s^2 < theta^2 D^2,
// i.e. iff E2 = |d|^2 + eps^2 exceeds S = s^2 / theta^2 + eps^2 (E2 is the
// softened distance the monopole needs anyway, so the test costs one compare).
// With rho an upper bound of |com - g|_inf + |x - g|_inf and u = 2^-24, the
// computed E2 - S differs from the exact D^2 - s^2 / theta^2 by less than
//   B = 16 u S + rho (8 u s / theta + 16 u^2 rho)
// wherever the two could differ in sign (first-order terms about half of
// these, the rho^2 term covers the case of a target within FP32 resolution of
// a small cube).  Per child and wavefront the walk stages hi >= S + B and
// lo <= S - B: E2 > hi accepts, E2 < lo opens, and the rare lanes in between
// repeat the test in FP64 exactly as the oracle evaluates it.  Pair terms go
// into FP32 partial sums that are folded into Kahan-compensated totals after
// at most 64 terms.
template <bool STATS, bool POT, int W, bool QUAD, bool SOFT>
__global__ void __launch_bounds__(64 * W) k_walk32(ForestDev f, WalkOut out) {
    __shared__ WaveLds32 lds_all[W];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    WaveLds32 &L = lds_all[wave];
    const uint32_t gi = blockIdx.x * W + wave;
    if (gi >= f.ngroups) return;
    if (uni(*f.err) & kErrTree) return;   // tree inconsistent: never walk it
    const GroupDesc gd = f.groups[gi];
    const uint32_t sid = uni(gd.seg);
    const SegDesc &sd = f.seg[sid];
    if (sd.precision != 1 || sd.group || (sd.quad != 0) != QUAD || unsoftened(sd.eps) == SOFT) return;
    const SegState &st = f.st[sid];
    const uint32_t gstart = uni(gd.start);
    const bool live = (uint32_t)lane < gd.count;
    const uint32_t r = gstart + (live ? (uint32_t)lane : 0u);
    const double gx = f.spos[3 * (size_t)gstart], gy = f.spos[3 * (size_t)gstart + 1],
                 gz = f.spos[3 * (size_t)gstart + 2];
    const float tx = (float)__dsub_rn(f.spos[3 * (size_t)r], gx);
    const float ty = (float)__dsub_rn(f.spos[3 * (size_t)r + 1], gy);
    const float tz = (float)__dsub_rn(f.spos[3 * (size_t)r + 2], gz);
    float rw = live ? fmaxf(fabsf(tx), fmaxf(fabsf(ty), fabsf(tz))) : 0.0f;
    for (int o = 32; o > 0; o >>= 1) rw = fmaxf(rw, __shfl_xor(rw, o, 64));
    rw = __uint_as_float(uni(__float_as_uint(rw))) * (1.0f + 4.0f * kU32);
    const double theta = sd.theta;
    const float eps2 = (float)(sd.eps * sd.eps);
    const float band2 = 16.0f * kU32 * kU32;   // 16 u^2
    constexpr bool soft = SOFT;

    float ax = 0.f, ay = 0.f, az = 0.f, ap = 0.f;            // partial sums
    float sx = 0.f, sy = 0.f, sz = 0.f, sp_ = 0.f;           // Kahan sums
    float cx = 0.f, cy = 0.f, cz = 0.f, cp = 0.f;            // Kahan compensations
    uint32_t nmono = 0, np2p = 0, nvis = 0, nfb = 0;
    uint32_t wvis = 0, went = 0, wacc = 0, wleaf = 0;         // wave-level counters (uniform)
    uint64_t h = 0;
    uint32_t work = 0;   // terms added to the partial sums since the last fold (wave-uniform)
    uint32_t qn = 0;     // queued leaf particles (wave-uniform)
    auto fold = [&]() {
        kahan_add(sx, cx, ax); ax = 0.f;
        kahan_add(sy, cy, ay); ay = 0.f;
        kahan_add(sz, cz, az); az = 0.f;
        if (POT) { kahan_add(sp_, cp, ap); ap = 0.f; }
        work = 0;
    };
    auto pair = [&](float px, float py, float pz, float pm) {
        const float dx = px - tx, dy = py - ty, dz = pz - tz;
        const float r2 = fmaf(dz, dz, fmaf(dy, dy, fmaf(dx, dx, eps2)));
        if (soft || r2 > 0.0f) {
            const float ri = __builtin_amdgcn_rsqf(r2);
            const float mr = pm * ri;
            const float w3 = mr * ri * ri;
            ax = fmaf(w3, dx, ax);
            ay = fmaf(w3, dy, ay);
            az = fmaf(w3, dz, az);
            if (POT) ap -= mr;
        }
    };
    // queued leaf particles: load and convert lane-parallel, then one pass per particle
    uint32_t wwork = 0;   // wavefront work: child tests and pair iterations (uniform)
    auto flush_leaves = [&]() {
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
                        if (STATS) {
                            ++np2p;
                            h += mix64((uint64_t)st.nn + (uint64_t)(f.idx[jq] - sd.start));
                        }
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
                if (STATS) {
                    ++np2p;
                    h += mix64((uint64_t)st.nn + (uint64_t)(f.idx[jq] - sd.start));
                }
            }
        }
        qn = 0;
        wave_sync();
    };

    int sp = 0;
    const uint64_t m0 = ballot(live);
    if (lane == 0) L.stk[0] = make_uint4(sid, 1u, (uint32_t)m0, (uint32_t)(m0 >> 32));
    wave_sync();
    sp = 1;
    while (sp > 0) {
        --sp;
        const uint4 e = L.stk[sp];
        const uint32_t link = uni(e.x), nch = uni(e.y);
        if (STATS) wwork += nch;
        const uint64_t emask = ((uint64_t)uni(e.w) << 32) | uni(e.z);
        wave_sync();
        if ((uint32_t)lane < nch) {
            const WRec32 &w = f.w32[link + lane];
            const float qx = (float)__dsub_rn(w.cx, gx);
            const float qy = (float)__dsub_rn(w.cy, gy);
            const float qz = (float)__dsub_rn(w.cz, gz);
            const float rho = fmaf(fmaxf(fabsf(qx), fmaxf(fabsf(qy), fabsf(qz))), 1.0f + 4.0f * kU32, rw);
            const float B = fmaf(rho, fmaf(band2, rho, w.band1), w.band0);
            L.sa[lane] = make_float4(qx, qy, qz, w.m);
            L.sb[lane] = make_float2((w.Sp + B) * (1.0f + 4.0f * kU32), fmaxf(w.Sp - B, 0.0f) * (1.0f - 4.0f * kU32));
            L.sl[lane] = make_uint2(w.link, w.cnt);
            L.sc[lane] = make_uint2(w.gid, w.level);
            if (QUAD) {
                L.sq0[lane] = f.q32[2 * (size_t)(link + lane)];
                L.sq1[lane] = f.q32[2 * (size_t)(link + lane) + 1];
            }
        }
        wave_sync();
        if (work + nch > kFlushWork) fold();
        work += nch;
        if (STATS) { wvis += nch; ++went; }
#pragma unroll
        for (uint32_t c = 0; c < 8; ++c) {
            if (c >= nch) break;
            const float4 qa = L.sa[c];
            const float dx = qa.x - tx, dy = qa.y - ty, dz = qa.z - tz;
            const float E2 = fmaf(dz, dz, fmaf(dy, dy, fmaf(dx, dx, eps2)));
            uint64_t accm = ballot(E2 > L.sb[c].x) & emask;
            uint64_t open = emask & ~accm;
            if (open) {
                const uint64_t ambm = ballot(!(E2 < L.sb[c].y)) & open;
                if (ambm) {
                    // within the FP32 rounding bound of the threshold: decide exactly in FP64
                    bool ex = false;
                    if (in_mask(ambm)) {
                        const WRec32 &wc = f.w32[link + c];
                        const double cm[3] = {wc.cx, wc.cy, wc.cz};
                        const double *xp = f.spos + 3 * (size_t)r;
                        const double ex_ = __dsub_rn(cm[0], xp[0]), ey = __dsub_rn(cm[1], xp[1]),
                                     ez = __dsub_rn(cm[2], xp[2]);
                        const double ED2 =
                            __dadd_rn(__dadd_rn(__dmul_rn(ex_, ex_), __dmul_rn(ey, ey)), __dmul_rn(ez, ez));
                        ex = f.w32[link + c].r2 < __dmul_rn(__dmul_rn(theta, theta), ED2);
                        if (STATS) ++nfb;
                    }
                    accm |= ballot(ex) & ambm;
                    open = emask & ~accm;
                }
                if (open) {
                    const uint2 ql = L.sl[c];
                    const uint32_t qlink = uni(ql.x), qcnt = uni(ql.y);
                    if (qcnt & kLeafBit) {
                        const uint32_t np = qcnt & ~kLeafBit;
                        if (STATS) ++wleaf;
                        if (np <= 64u) {
                            if (qn + np > 64u) flush_leaves();
                            if ((uint32_t)lane < np) {
                                L.irank[qn + lane] = qlink + lane;
                                L.imask[qn + lane] = open;
                            }
                            qn += np;
                        } else {
                            // a leaf of more than 64 particles (coincident particles at the depth limit)
                            flush_leaves();
                            for (uint32_t b0 = 0; b0 < np; b0 += 64) {
                                const uint32_t nb = np - b0 < 64u ? np - b0 : 64u;
                                if ((uint32_t)lane < nb) {
                                    L.irank[lane] = qlink + b0 + lane;
                                    L.imask[lane] = open;
                                }
                                qn = nb;
                                flush_leaves();
                            }
                        }
                    } else if (sp < kStackMax) {
                        if (lane == 0) L.stk[sp] = make_uint4(qlink, qcnt, (uint32_t)open, (uint32_t)(open >> 32));
                        wave_sync();
                        ++sp;
                    } else if (lane == 0) {
                        atomicOr(f.err, kErrStack);   // result void; the walk still drains
                    }
                }
            }
            if (STATS) {
                if (in_mask(emask)) ++nvis;
                if (accm) ++wacc;
            }
            if (in_mask(accm)) {
                // softened monopole, executed by the accepting lanes only
                __asm__ volatile("");
                const float ri = __builtin_amdgcn_rsqf(E2);
                const float mr = qa.w * ri;
                const float ri2 = ri * ri;
                float w3 = mr * ri2;
                if (QUAD) {
                    // + G [5 A d / (2 s^7) - (3 S.d - tr S d) / s^5],  A = 3 d.S.d - s^2 tr S
                    const float4 s0 = L.sq0[c], s1 = L.sq1[c];
                    const float sdx = fmaf(s0.x, dx, fmaf(s0.w, dy, s1.x * dz));
                    const float sdy = fmaf(s0.w, dx, fmaf(s0.y, dy, s1.y * dz));
                    const float sdz = fmaf(s1.x, dx, fmaf(s1.y, dy, s0.z * dz));
                    const float A = fmaf(3.0f, fmaf(dx, sdx, fmaf(dy, sdy, dz * sdz)), -E2 * s1.z);
                    const float ri5 = ri2 * ri2 * ri;
                    float qx = -ri5 * fmaf(3.0f, sdx, -s1.z * dx) + 2.5f * A * ri5 * ri2 * dx;
                    float qy = -ri5 * fmaf(3.0f, sdy, -s1.z * dy) + 2.5f * A * ri5 * ri2 * dy;
                    float qz = -ri5 * fmaf(3.0f, sdz, -s1.z * dz) + 2.5f * A * ri5 * ri2 * dz;
                    float qp = -0.5f * A * ri5;
                    // tr S > M s^2: the body is close to (or inside) the cube, the terms of the
                    // expansion nearly cancel and FP32 loses them; those lanes take it in FP64
                    const uint64_t hard = ballot(s1.z > qa.w * E2) & accm;
                    if (hard) {
                        if (in_mask(hard)) {
                            const WRec32 &wc = f.w32[link + c];
                            const double cm[3] = {wc.cx, wc.cy, wc.cz};
                            const double *xp = f.spos + 3 * (size_t)r;
                            const double *S = f.uQ + 6 * (size_t)(link + c);
                            const double ex_ = cm[0] - xp[0], ey = cm[1] - xp[1], ez = cm[2] - xp[2];
                            const double e2 = ((ex_ * ex_ + ey * ey) + ez * ez) + (double)sd.eps * sd.eps;
                            const double tr = (S[0] + S[1]) + S[2];
                            const double sx = fma(S[0], ex_, fma(S[3], ey, S[4] * ez));
                            const double sy = fma(S[3], ex_, fma(S[1], ey, S[5] * ez));
                            const double sz = fma(S[4], ex_, fma(S[5], ey, S[2] * ez));
                            const double A64 = fma(3.0, fma(ex_, sx, fma(ey, sy, ez * sz)), -e2 * tr);
                            const double rinv = 1.0 / sqrt(e2);
                            const double r5 = rinv * rinv * rinv * rinv * rinv, r7 = r5 * rinv * rinv;
                            qx = (float)(2.5 * A64 * r7 * ex_ - r5 * fma(3.0, sx, -tr * ex_));
                            qy = (float)(2.5 * A64 * r7 * ey - r5 * fma(3.0, sy, -tr * ey));
                            qz = (float)(2.5 * A64 * r7 * ez - r5 * fma(3.0, sz, -tr * ez));
                            qp = (float)(-0.5 * A64 * r5);
                        }
                    }
                    ax += qx;
                    ay += qy;
                    az += qz;
                    if (POT) ap += qp;
                }
                ax = fmaf(w3, dx, ax);
                ay = fmaf(w3, dy, ay);
                az = fmaf(w3, dz, az);
                if (POT) ap -= mr;
                if (STATS) {
                    ++nmono;
                    h += mix64((uint64_t)(L.sc[c].x - st.nbase));
                }
            }
        }
    }
    flush_leaves();
    fold();
    const bool own = live && r >= out.wlo && r < out.whi;
    if (STATS && out.gwork && lane == 0) out.gwork[(gstart - sd.start) / kGroup] = (int64_t)wwork;
    if (own) {
        const uint32_t i = f.idx[r];
        const size_t li = i - sd.start;
        const double G = sd.G;
        double *accb = seg_base(out.acc, sd.acc, sd, 3);
        accb[3 * li] = G * ((double)sx - (double)cx);
        accb[3 * li + 1] = G * ((double)sy - (double)cy);
        accb[3 * li + 2] = G * ((double)sz - (double)cz);
        if (POT) {
            double *potb = seg_base(out.pot, sd.pot, sd, 1);
            if (potb) potb[li] = G * ((double)sp_ - (double)cp);
        }
        if (STATS) {
            if (out.n_mono) out.n_mono[i] = nmono;
            if (out.n_p2p) out.n_p2p[i] = np2p;
            if (out.hash) out.hash[i] = h;
            if (out.work) {   // the group's wavefront work, spread evenly over its bodies
                const uint64_t wg = wwork, k = (uint32_t)lane, c = gd.count;
                out.work[i] = (int64_t)((wg * (k + 1)) / c - (wg * k) / c);
            }
        }
    }
    if (STATS) {
        unsigned long long a = wave_sum_u(own ? nmono : 0), b = wave_sum_u(own ? np2p : 0);
        unsigned long long v = wave_sum_u(own ? nvis : 0), fb = wave_sum_u(own ? nfb : 0);
        if (lane == 0) {
            atomicAdd(&f.stats[0], a);
            atomicAdd(&f.stats[1], b);
            atomicAdd(&f.stats[2], v);
            atomicAdd(&f.stats[3], fb);
            atomicAdd(&f.stats[4], (unsigned long long)wvis);
            atomicAdd(&f.stats[5], (unsigned long long)went);
            atomicAdd(&f.stats[6], (unsigned long long)wacc);
            atomicAdd(&f.stats[7], (unsigned long long)wleaf);
        }
    }
}

// ------------------------------------------------------------- FP64 walk ---

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

template <bool STATS, bool POT, int W, bool QUAD>
__global__ void __launch_bounds__(64 * W) k_walk64(ForestDev f, WalkOut out) {
    __shared__ WaveLds64<QUAD> lds_all[W];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    WaveLds64<QUAD> &L = lds_all[wave];
    const uint32_t gi = blockIdx.x * W + wave;
    if (gi >= f.ngroups) return;
    if (uni(*f.err) & kErrTree) return;   // tree inconsistent: never walk it
    const GroupDesc gd = f.groups[gi];
    const uint32_t sid = uni(gd.seg);
    const SegDesc &sd = f.seg[sid];
    if (sd.precision != 0 || sd.group || (sd.quad != 0) != QUAD) return;
    const SegState &st = f.st[sid];
    const uint32_t gstart = uni(gd.start);
    const bool live = (uint32_t)lane < gd.count;
    const uint32_t r = gstart + (live ? (uint32_t)lane : 0u);
    const double tx = f.spos[3 * (size_t)r], ty = f.spos[3 * (size_t)r + 1], tz = f.spos[3 * (size_t)r + 2];
    const double theta2 = __dmul_rn(sd.theta, sd.theta);
    const double eps2 = __dmul_rn(sd.eps, sd.eps);
    const bool soft = eps2 > 0.0;

    double ax = 0.0, ay = 0.0, az = 0.0, ap = 0.0;
    uint32_t nmono = 0, np2p = 0, nvis = 0;
    uint64_t h = 0;
    uint32_t qn = 0;
    auto pair = [&](double px, double py, double pz, double pm) {
        const double dx = px - tx, dy = py - ty, dz = pz - tz;
        const double r2 = fma(dz, dz, fma(dy, dy, fma(dx, dx, eps2)));
        if (soft || r2 > 0.0) {
            const double ri = rsqrt64(r2);
            const double mr = pm * ri;
            const double w3 = mr * ri * ri;
            ax = fma(w3, dx, ax);
            ay = fma(w3, dy, ay);
            az = fma(w3, dz, az);
            if (POT) ap -= mr;
        }
    };
    uint32_t wwork = 0;   // wavefront work: child tests and pair iterations (uniform)
    auto flush_leaves = [&]() {
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
                        h += mix64((uint64_t)st.nn + (uint64_t)(f.idx[jq] - sd.start));
                    }
                }
            }
        }
        qn = 0;
        wave_sync();
    };

    int sp = 0;
    const uint64_t m0 = ballot(live);
    if (lane == 0) L.stk[0] = make_uint4(sid, 1u, (uint32_t)m0, (uint32_t)(m0 >> 32));
    wave_sync();
    sp = 1;
    while (sp > 0) {
        --sp;
        const uint4 e = L.stk[sp];
        const uint32_t link = uni(e.x), nch = uni(e.y);
        if (STATS) wwork += nch;
        const uint64_t emask = ((uint64_t)uni(e.w) << 32) | uni(e.z);
        wave_sync();
        if ((uint32_t)lane < nch) {
            const WRec64 &w = f.w64[link + lane];
            L.sa[lane] = make_double4(w.x, w.y, w.z, w.m);
            L.sS[lane] = w.S;
            L.sb[lane] = make_uint4(w.link, w.cnt, w.gid, w.level);
            if (QUAD)
                for (int k = 0; k < 6; ++k) L.sq[6 * lane + k] = f.q64[6 * (size_t)(link + lane) + k];
        }
        wave_sync();
#pragma unroll
        for (uint32_t c = 0; c < 8; ++c) {
            if (c >= nch) break;
            const double4 qa = L.sa[c];
            const double S = L.sS[c];
            const double dx = __dsub_rn(qa.x, tx), dy = __dsub_rn(qa.y, ty), dz = __dsub_rn(qa.z, tz);
            const double D2 = __dadd_rn(__dadd_rn(__dmul_rn(dx, dx), __dmul_rn(dy, dy)), __dmul_rn(dz, dz));
            const uint64_t accm = ballot(S < __dmul_rn(theta2, D2)) & emask;
            if (STATS && in_mask(emask)) ++nvis;
            const uint64_t open = emask & ~accm;
            if (open) {
                const uint4 qb = L.sb[c];
                const uint32_t qlink = uni(qb.x), qcnt = uni(qb.y);
                if (qcnt & kLeafBit) {
                    const uint32_t np = qcnt & ~kLeafBit;
                    if (np <= 64u) {
                        if (qn + np > 64u) flush_leaves();
                        if ((uint32_t)lane < np) {
                            L.irank[qn + lane] = qlink + lane;
                            L.imask[qn + lane] = open;
                        }
                        qn += np;
                    } else {
                        flush_leaves();
                        for (uint32_t b0 = 0; b0 < np; b0 += 64) {
                            const uint32_t nb = np - b0 < 64u ? np - b0 : 64u;
                            if ((uint32_t)lane < nb) {
                                L.irank[lane] = qlink + b0 + lane;
                                L.imask[lane] = open;
                            }
                            qn = nb;
                            flush_leaves();
                        }
                    }
                } else if (sp < kStackMax) {
                    if (lane == 0) L.stk[sp] = make_uint4(qlink, qcnt, (uint32_t)open, (uint32_t)(open >> 32));
                    wave_sync();
                    ++sp;
                } else if (lane == 0) {
                    atomicOr(f.err, kErrStack);   // result void; the walk still drains
                }
            }
            if (in_mask(accm)) {
                // softened monopole, executed by the accepting lanes only
                __asm__ volatile("");
                const double E2 = D2 + eps2;
                const double ri = rsqrt64(E2);
                const double mr = qa.w * ri;
                const double ri2 = ri * ri;
                double w3 = mr * ri2;
                if (QUAD) {
                    const double *q = &L.sq[6 * c];
                    const double sdx = fma(q[0], dx, fma(q[3], dy, q[4] * dz));
                    const double sdy = fma(q[3], dx, fma(q[1], dy, q[5] * dz));
                    const double sdz = fma(q[4], dx, fma(q[5], dy, q[2] * dz));
                    const double tr = (q[0] + q[1]) + q[2];
                    const double A = fma(3.0, fma(dx, sdx, fma(dy, sdy, dz * sdz)), -E2 * tr);
                    const double ri5 = ri2 * ri2 * ri;
                    w3 = fma(2.5 * A, ri5 * ri2, w3);
                    ax = fma(-ri5, fma(3.0, sdx, -tr * dx), ax);
                    ay = fma(-ri5, fma(3.0, sdy, -tr * dy), ay);
                    az = fma(-ri5, fma(3.0, sdz, -tr * dz), az);
                    if (POT) ap -= 0.5 * A * ri5;
                }
                ax = fma(w3, dx, ax);
                ay = fma(w3, dy, ay);
                az = fma(w3, dz, az);
                if (POT) ap -= mr;
                if (STATS) {
                    ++nmono;
                    h += mix64((uint64_t)(L.sb[c].z - st.nbase));
                }
            }
        }
    }
    flush_leaves();
    const bool own = live && r >= out.wlo && r < out.whi;
    if (STATS && out.gwork && lane == 0) out.gwork[(gstart - sd.start) / kGroup] = (int64_t)wwork;
    if (own) {
        const uint32_t i = f.idx[r];
        const size_t li = i - sd.start;
        const double G = sd.G;
        double *accb = seg_base(out.acc, sd.acc, sd, 3);
        accb[3 * li] = G * ax;
        accb[3 * li + 1] = G * ay;
        accb[3 * li + 2] = G * az;
        if (POT) {
            double *potb = seg_base(out.pot, sd.pot, sd, 1);
            if (potb) potb[li] = G * ap;
        }
        if (STATS) {
            if (out.n_mono) out.n_mono[i] = nmono;
            if (out.n_p2p) out.n_p2p[i] = np2p;
            if (out.hash) out.hash[i] = h;
            if (out.work) {   // the group's wavefront work, spread evenly over its bodies
                const uint64_t wg = wwork, k = (uint32_t)lane, c = gd.count;
                out.work[i] = (int64_t)((wg * (k + 1)) / c - (wg * k) / c);
            }
        }
    }
    if (STATS) {
        unsigned long long a = wave_sum_u(own ? nmono : 0), b = wave_sum_u(own ? np2p : 0);
        unsigned long long v = wave_sum_u(own ? nvis : 0);
        if (lane == 0) {
            atomicAdd(&f.stats[0], a);
            atomicAdd(&f.stats[1], b);
            atomicAdd(&f.stats[2], v);
        }
    }
}

// ------------------------------------------------- group-criterion walk ---
// A variant of the opening test: the 64 bodies of a walk group share one decision
// per cube, taken in FP64 against the group's bounding box exactly as the oracle
// writes it (D from the centre of mass to the box, strict side^2 < theta^2 D^2).
// Each staging lane decides for its child, so a decision costs one FP64 test per
// child per wavefront, and every live lane evaluates every accepted cube: no
// partial lane masks.  Pair differences of opened leaves use the FP32 hi/lo split
// of x - g (accurate also without softening).

struct GLds32 {
    uint2 stk[kStackMax];  // (first child slot, children)
    float4 sa[8];          // child: centre rel g, mass
    uint2 sl[8];           // child: link, cnt
    uint32_t sg[8];        // child: gid
    uint32_t irank[64];    // queued leaf particles (every live lane takes part)
    float4 pst[64];        // 32 staged particles: (hi, mass), (lo, 0)
};

__device__ __forceinline__ double wave_min64(double v) {
    for (int o = 32; o > 0; o >>= 1) v = fmin(v, __shfl_xor(v, o, 64));
    return v;
}
__device__ __forceinline__ double wave_max64(double v) {
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
    return v;
}
__device__ __forceinline__ double unid(double v) {
    const uint64_t b = (uint64_t)__double_as_longlong(v);
    return __longlong_as_double((long long)uni64(b));
}

// Group decision for a cube with centre c and level `level`: as the oracle evaluates it.
__device__ __forceinline__ bool group_accepts(double cx, double cy, double cz, int level, const double blo[3],
                                              const double bhi[3], double theta2, double L) {
    double dd[3];
    const double c[3] = {cx, cy, cz};
    for (int k = 0; k < 3; ++k) {
        const double u = __dsub_rn(blo[k], c[k]), v = __dsub_rn(c[k], bhi[k]);
        const double w = u > v ? u : v;
        dd[k] = w > 0.0 ? w : 0.0;
    }
    const double D2 = __dadd_rn(__dadd_rn(__dmul_rn(dd[0], dd[0]), __dmul_rn(dd[1], dd[1])), __dmul_rn(dd[2], dd[2]));
    const double s = ldexp(L, -level);
    return __dmul_rn(s, s) < __dmul_rn(theta2, D2);
}

template <bool STATS, bool POT>
__global__ void __launch_bounds__(256) k_gwalk32(ForestDev f, WalkOut out) {
    __shared__ GLds32 lds_all[4];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    GLds32 &L = lds_all[wave];
    const uint32_t gi = blockIdx.x * 4 + wave;
    if (gi >= f.ngroups) return;
    if (uni(*f.err) & kErrTree) return;
    const GroupDesc gd = f.groups[gi];
    const uint32_t sid = uni(gd.seg);
    const SegDesc &sd = f.seg[sid];
    if (sd.precision != 1 || !sd.group) return;
    const SegState &st = f.st[sid];
    const uint32_t gstart = uni(gd.start);
    const bool live = (uint32_t)lane < gd.count;
    const uint32_t r = gstart + (live ? (uint32_t)lane : 0u);
    const double gx = f.spos[3 * (size_t)gstart], gy = f.spos[3 * (size_t)gstart + 1],
                 gz = f.spos[3 * (size_t)gstart + 2];
    const double xr = f.spos[3 * (size_t)r], yr = f.spos[3 * (size_t)r + 1], zr = f.spos[3 * (size_t)r + 2];
    const double ex = __dsub_rn(xr, gx), ey = __dsub_rn(yr, gy), ez = __dsub_rn(zr, gz);
    const float tx = (float)ex, ty = (float)ey, tz = (float)ez;
    const float tlx = (float)(ex - (double)tx), tly = (float)(ey - (double)ty), tlz = (float)(ez - (double)tz);
    double blo[3], bhi[3];
    blo[0] = unid(wave_min64(live ? xr : INFINITY));
    blo[1] = unid(wave_min64(live ? yr : INFINITY));
    blo[2] = unid(wave_min64(live ? zr : INFINITY));
    bhi[0] = unid(wave_max64(live ? xr : -INFINITY));
    bhi[1] = unid(wave_max64(live ? yr : -INFINITY));
    bhi[2] = unid(wave_max64(live ? zr : -INFINITY));
    const double theta2 = __dmul_rn(sd.theta, sd.theta);
    const double Lside = st.L;
    const float eps2 = (float)(sd.eps * sd.eps);
    const bool soft = eps2 > 0.0f;
    const uint64_t live_mask = ballot(live);

    float ax = 0.f, ay = 0.f, az = 0.f, ap = 0.f;
    float sx = 0.f, sy = 0.f, sz = 0.f, sp_ = 0.f;
    float cx = 0.f, cy = 0.f, cz = 0.f, cp = 0.f;
    uint32_t nmono = 0, np2p = 0, nvis = 0;
    uint32_t wvis = 0, went = 0, wacc = 0, wleaf = 0;
    uint64_t h = 0;
    uint32_t work = 0, qn = 0;
    auto fold = [&]() {
        kahan_add(sx, cx, ax); ax = 0.f;
        kahan_add(sy, cy, ay); ay = 0.f;
        kahan_add(sz, cz, az); az = 0.f;
        if (POT) { kahan_add(sp_, cp, ap); ap = 0.f; }
        work = 0;
    };
    uint32_t wwork = 0;   // wavefront work: child tests and pair iterations (uniform)
    auto flush_leaves = [&]() {
        if (qn == 0) return;
        if (STATS) wwork += qn;
        if (work + qn > kFlushWork) fold();
        work += qn;
        for (uint32_t k0 = 0; k0 < qn; k0 += 32) {
            const uint32_t nb = qn - k0 < 32u ? qn - k0 : 32u;
            wave_sync();
            if ((uint32_t)lane < nb) {
                const size_t j = L.irank[k0 + lane];
                const double px = __dsub_rn(f.spos[3 * j], gx), py = __dsub_rn(f.spos[3 * j + 1], gy),
                             pz = __dsub_rn(f.spos[3 * j + 2], gz);
                const float hx = (float)px, hy = (float)py, hz = (float)pz;
                L.pst[2 * lane] = make_float4(hx, hy, hz, (float)f.smass[j]);
                L.pst[2 * lane + 1] = make_float4((float)(px - (double)hx), (float)(py - (double)hy),
                                                  (float)(pz - (double)hz), 0.0f);
            }
            wave_sync();
            for (uint32_t k = 0; k < nb; ++k) {
                const uint32_t jq = uni(L.irank[k0 + k]);
                const uint64_t m = live_mask & ~self_bit(jq, gstart);
                if (in_mask(m)) {
                    const float4 ph = L.pst[2 * k], pl = L.pst[2 * k + 1];
                    const float dx = (ph.x - tx) + (pl.x - tlx), dy = (ph.y - ty) + (pl.y - tly),
                                dz = (ph.z - tz) + (pl.z - tlz);
                    const float r2 = fmaf(dz, dz, fmaf(dy, dy, fmaf(dx, dx, eps2)));
                    if (soft || r2 > 0.0f) {
                        const float ri = __builtin_amdgcn_rsqf(r2);
                        const float mr = ph.w * ri;
                        const float w3 = mr * ri * ri;
                        ax = fmaf(w3, dx, ax);
                        ay = fmaf(w3, dy, ay);
                        az = fmaf(w3, dz, az);
                        if (POT) ap -= mr;
                    }
                    if (STATS) {
                        ++np2p;
                        h += mix64((uint64_t)st.nn + (uint64_t)(f.idx[jq] - sd.start));
                    }
                }
            }
        }
        qn = 0;
        wave_sync();
    };

    int sp = 0;
    if (lane == 0) L.stk[0] = make_uint2(sid, 1u);
    wave_sync();
    sp = 1;
    while (sp > 0) {
        --sp;
        const uint2 e = L.stk[sp];
        const uint32_t link = uni(e.x), nch = uni(e.y);
        if (STATS) wwork += nch;
        wave_sync();
        bool acc_c = false;
        if ((uint32_t)lane < nch) {
            const WRec32 &w = f.w32[link + lane];
            acc_c = group_accepts(w.cx, w.cy, w.cz, (int)w.level, blo, bhi, theta2, Lside);
            L.sa[lane] = make_float4((float)__dsub_rn(w.cx, gx), (float)__dsub_rn(w.cy, gy),
                                     (float)__dsub_rn(w.cz, gz), w.m);
            L.sl[lane] = make_uint2(w.link, w.cnt);
            L.sg[lane] = w.gid;
        }
        const uint64_t accb = ballot(acc_c);
        wave_sync();
        if (work + nch > kFlushWork) fold();
        work += nch;
        if (STATS) {
            wvis += nch;
            ++went;
            if (live) nvis += nch;
        }
        for (uint32_t c = 0; c < 8; ++c) {
            if (c >= nch) break;
            if ((accb >> c) & 1u) {
                const float4 qa = L.sa[c];
                const float dx = qa.x - tx, dy = qa.y - ty, dz = qa.z - tz;
                const float E2 = fmaf(dz, dz, fmaf(dy, dy, fmaf(dx, dx, eps2)));
                const float ri = __builtin_amdgcn_rsqf(E2);
                const float mr = qa.w * ri;
                const float w3 = mr * ri * ri;
                ax = fmaf(w3, dx, ax);
                ay = fmaf(w3, dy, ay);
                az = fmaf(w3, dz, az);
                if (POT) ap -= mr;
                if (STATS) {
                    ++wacc;
                    ++nmono;
                    h += mix64((uint64_t)(L.sg[c] - st.nbase));
                }
            } else {
                const uint2 ql = L.sl[c];
                const uint32_t qlink = uni(ql.x), qcnt = uni(ql.y);
                if (qcnt & kLeafBit) {
                    const uint32_t np = qcnt & ~kLeafBit;
                    if (STATS) ++wleaf;
                    if (np <= 64u) {
                        if (qn + np > 64u) flush_leaves();
                        if ((uint32_t)lane < np) L.irank[qn + lane] = qlink + lane;
                        qn += np;
                    } else {
                        flush_leaves();
                        for (uint32_t b0 = 0; b0 < np; b0 += 64) {
                            const uint32_t nb = np - b0 < 64u ? np - b0 : 64u;
                            if ((uint32_t)lane < nb) L.irank[lane] = qlink + b0 + lane;
                            qn = nb;
                            flush_leaves();
                        }
                    }
                } else if (sp < kStackMax) {
                    if (lane == 0) L.stk[sp] = make_uint2(qlink, qcnt);
                    wave_sync();
                    ++sp;
                } else if (lane == 0) {
                    atomicOr(f.err, kErrStack);
                }
            }
        }
    }
    flush_leaves();
    fold();
    const bool own = live && r >= out.wlo && r < out.whi;
    if (STATS && out.gwork && lane == 0) out.gwork[(gstart - sd.start) / kGroup] = (int64_t)wwork;
    if (own) {
        const uint32_t i = f.idx[r];
        const size_t li = i - sd.start;
        const double G = sd.G;
        double *accb = seg_base(out.acc, sd.acc, sd, 3);
        accb[3 * li] = G * ((double)sx - (double)cx);
        accb[3 * li + 1] = G * ((double)sy - (double)cy);
        accb[3 * li + 2] = G * ((double)sz - (double)cz);
        if (POT) {
            double *potb = seg_base(out.pot, sd.pot, sd, 1);
            if (potb) potb[li] = G * ((double)sp_ - (double)cp);
        }
        if (STATS) {
            if (out.n_mono) out.n_mono[i] = nmono;
            if (out.n_p2p) out.n_p2p[i] = np2p;
            if (out.hash) out.hash[i] = h;
            if (out.work) {   // the group's wavefront work, spread evenly over its bodies
                const uint64_t wg = wwork, k = (uint32_t)lane, c = gd.count;
                out.work[i] = (int64_t)((wg * (k + 1)) / c - (wg * k) / c);
            }
        }
    }
    if (STATS) {
        unsigned long long a = wave_sum_u(own ? nmono : 0), b = wave_sum_u(own ? np2p : 0);
        unsigned long long v = wave_sum_u(own ? nvis : 0);
        if (lane == 0) {
            atomicAdd(&f.stats[0], a);
            atomicAdd(&f.stats[1], b);
            atomicAdd(&f.stats[2], v);
            atomicAdd(&f.stats[4], (unsigned long long)wvis);
            atomicAdd(&f.stats[5], (unsigned long long)went);
            atomicAdd(&f.stats[6], (unsigned long long)wacc);
            atomicAdd(&f.stats[7], (unsigned long long)wleaf);
        }
    }
}

struct GLds64 {
    uint2 stk[kStackMax];
    double4 sa[8];         // child: centre of mass, mass
    uint2 sl[8];
    uint32_t sg[8];
    uint32_t irank[64];
    double4 pst[64];
};

template <bool STATS, bool POT>
__global__ void __launch_bounds__(256) k_gwalk64(ForestDev f, WalkOut out) {
    __shared__ GLds64 lds_all[4];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    GLds64 &L = lds_all[wave];
    const uint32_t gi = blockIdx.x * 4 + wave;
    if (gi >= f.ngroups) return;
    if (uni(*f.err) & kErrTree) return;
    const GroupDesc gd = f.groups[gi];
    const uint32_t sid = uni(gd.seg);
    const SegDesc &sd = f.seg[sid];
    if (sd.precision != 0 || !sd.group) return;
    const SegState &st = f.st[sid];
    const uint32_t gstart = uni(gd.start);
    const bool live = (uint32_t)lane < gd.count;
    const uint32_t r = gstart + (live ? (uint32_t)lane : 0u);
    const double tx = f.spos[3 * (size_t)r], ty = f.spos[3 * (size_t)r + 1], tz = f.spos[3 * (size_t)r + 2];
    double blo[3], bhi[3];
    blo[0] = unid(wave_min64(live ? tx : INFINITY));
    blo[1] = unid(wave_min64(live ? ty : INFINITY));
    blo[2] = unid(wave_min64(live ? tz : INFINITY));
    bhi[0] = unid(wave_max64(live ? tx : -INFINITY));
    bhi[1] = unid(wave_max64(live ? ty : -INFINITY));
    bhi[2] = unid(wave_max64(live ? tz : -INFINITY));
    const double theta2 = __dmul_rn(sd.theta, sd.theta);
    const double Lside = st.L;
    const double eps2 = __dmul_rn(sd.eps, sd.eps);
    const bool soft = eps2 > 0.0;
    const uint64_t live_mask = ballot(live);

    double ax = 0.0, ay = 0.0, az = 0.0, ap = 0.0;
    uint32_t nmono = 0, np2p = 0, nvis = 0;
    uint64_t h = 0;
    uint32_t qn = 0;
    uint32_t wwork = 0;   // wavefront work: child tests and pair iterations (uniform)
    auto flush_leaves = [&]() {
        if (qn == 0) return;
        if (STATS) wwork += qn;
        wave_sync();
        if ((uint32_t)lane < qn) {
            const size_t j = L.irank[lane];
            L.pst[lane] = make_double4(f.spos[3 * j], f.spos[3 * j + 1], f.spos[3 * j + 2], f.smass[j]);
        }
        wave_sync();
        for (uint32_t k = 0; k < qn; ++k) {
            const uint32_t jq = uni(L.irank[k]);
            const uint64_t m = live_mask & ~self_bit(jq, gstart);
            if (in_mask(m)) {
                const double4 p = L.pst[k];
                const double dx = p.x - tx, dy = p.y - ty, dz = p.z - tz;
                const double r2 = fma(dz, dz, fma(dy, dy, fma(dx, dx, eps2)));
                if (soft || r2 > 0.0) {
                    const double ri = rsqrt64(r2);
                    const double mr = p.w * ri;
                    const double w3 = mr * ri * ri;
                    ax = fma(w3, dx, ax);
                    ay = fma(w3, dy, ay);
                    az = fma(w3, dz, az);
                    if (POT) ap -= mr;
                }
                if (STATS) {
                    ++np2p;
                    h += mix64((uint64_t)st.nn + (uint64_t)(f.idx[jq] - sd.start));
                }
            }
        }
        qn = 0;
        wave_sync();
    };

    int sp = 0;
    if (lane == 0) L.stk[0] = make_uint2(sid, 1u);
    wave_sync();
    sp = 1;
    while (sp > 0) {
        --sp;
        const uint2 e = L.stk[sp];
        const uint32_t link = uni(e.x), nch = uni(e.y);
        if (STATS) wwork += nch;
        wave_sync();
        bool acc_c = false;
        if ((uint32_t)lane < nch) {
            const WRec64 &w = f.w64[link + lane];
            acc_c = group_accepts(w.x, w.y, w.z, (int)w.level, blo, bhi, theta2, Lside);
            L.sa[lane] = make_double4(w.x, w.y, w.z, w.m);
            L.sl[lane] = make_uint2(w.link, w.cnt);
            L.sg[lane] = w.gid;
        }
        const uint64_t accb = ballot(acc_c);
        wave_sync();
        if (STATS && live) nvis += nch;
        for (uint32_t c = 0; c < 8; ++c) {
            if (c >= nch) break;
            if ((accb >> c) & 1u) {
                const double4 qa = L.sa[c];
                const double dx = qa.x - tx, dy = qa.y - ty, dz = qa.z - tz;
                const double E2 = fma(dz, dz, fma(dy, dy, fma(dx, dx, eps2)));
                const double ri = rsqrt64(E2);
                const double mr = qa.w * ri;
                const double w3 = mr * ri * ri;
                ax = fma(w3, dx, ax);
                ay = fma(w3, dy, ay);
                az = fma(w3, dz, az);
                if (POT) ap -= mr;
                if (STATS) {
                    ++nmono;
                    h += mix64((uint64_t)(L.sg[c] - st.nbase));
                }
            } else {
                const uint2 ql = L.sl[c];
                const uint32_t qlink = uni(ql.x), qcnt = uni(ql.y);
                if (qcnt & kLeafBit) {
                    const uint32_t np = qcnt & ~kLeafBit;
                    if (np <= 64u) {
                        if (qn + np > 64u) flush_leaves();
                        if ((uint32_t)lane < np) L.irank[qn + lane] = qlink + lane;
                        qn += np;
                    } else {
                        flush_leaves();
                        for (uint32_t b0 = 0; b0 < np; b0 += 64) {
                            const uint32_t nb = np - b0 < 64u ? np - b0 : 64u;
                            if ((uint32_t)lane < nb) L.irank[lane] = qlink + b0 + lane;
                            qn = nb;
                            flush_leaves();
                        }
                    }
                } else if (sp < kStackMax) {
                    if (lane == 0) L.stk[sp] = make_uint2(qlink, qcnt);
                    wave_sync();
                    ++sp;
                } else if (lane == 0) {
                    atomicOr(f.err, kErrStack);
                }
            }
        }
    }
    flush_leaves();
    const bool own = live && r >= out.wlo && r < out.whi;
    if (STATS && out.gwork && lane == 0) out.gwork[(gstart - sd.start) / kGroup] = (int64_t)wwork;
    if (own) {
        const uint32_t i = f.idx[r];
        const size_t li = i - sd.start;
        const double G = sd.G;
        double *accb = seg_base(out.acc, sd.acc, sd, 3);
        accb[3 * li] = G * ax;
        accb[3 * li + 1] = G * ay;
        accb[3 * li + 2] = G * az;
        if (POT) {
            double *potb = seg_base(out.pot, sd.pot, sd, 1);
            if (potb) potb[li] = G * ap;
        }
        if (STATS) {
            if (out.n_mono) out.n_mono[i] = nmono;
            if (out.n_p2p) out.n_p2p[i] = np2p;
            if (out.hash) out.hash[i] = h;
            if (out.work) {   // the group's wavefront work, spread evenly over its bodies
                const uint64_t wg = wwork, k = (uint32_t)lane, c = gd.count;
                out.work[i] = (int64_t)((wg * (k + 1)) / c - (wg * k) / c);
            }
        }
    }
    if (STATS) {
        unsigned long long a = wave_sum_u(own ? nmono : 0), b = wave_sum_u(own ? np2p : 0);
        unsigned long long v = wave_sum_u(own ? nvis : 0);
        if (lane == 0) {
            atomicAdd(&f.stats[0], a);
            atomicAdd(&f.stats[1], b);
            atomicAdd(&f.stats[2], v);
        }
    }
}

// Walk launches: W wavefronts (one 64-body group each) per workgroup, one kernel
// per precision and expansion order present.  The launch shape does not change
// any result (each group's arithmetic is its own); forests pick it by
// measurement (bh_forest_autotune).
// ------------------------------------------------ two-phase walk (lists) ---
// The force stage as the paper structures it (section 3): every body's list of
// cubes and particles is materialised first (flattened, here per walk group:
// the entries of all 64 bodies of a group in walk order, each with the mask of
// the bodies it applies to), then evaluated.  Phase one takes exactly the
// decisions of k_walk32 and records what k_walk32 would evaluate, in its
// order: the start of each stack entry (its child count, which times the
// Kahan folds), each opened leaf (particle range, mask) and each accepted cube
// (walk slot, node id, mask).  Phase two replays the lists with k_walk32's
// arithmetic, so both give the same bits.  Per-body walks of either precision
// and expansion order.

constexpr uint32_t kListEntry = 0xffffffffu;   // a == kListEntry: stack entry, b = children
constexpr uint32_t kListLeaf = 0x80000000u;    // b & kListLeaf: leaf, a = first rank, b = particles
constexpr uint32_t kListNone = 0xffffffffu;    // end of a group's chunk chain

template <int W>
__global__ void __launch_bounds__(64 * W) k_lists32(ForestDev f, ListDev ld) {
    __shared__ WaveLds32 lds_all[W];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    WaveLds32 &L = lds_all[wave];
    const uint32_t gi = blockIdx.x * W + wave;
    if (gi >= f.ngroups) return;
    if (uni(*f.err) & kErrTree) return;
    const GroupDesc gd = f.groups[gi];
    const uint32_t sid = uni(gd.seg);
    const SegDesc &sd = f.seg[sid];
    if (sd.precision != 1 || sd.group) return;   // refused by the host
    const SegState &st = f.st[sid];
    const uint32_t gstart = uni(gd.start);
    const bool live = (uint32_t)lane < gd.count;
    const uint32_t r = gstart + (live ? (uint32_t)lane : 0u);
    const double gx = f.spos[3 * (size_t)gstart], gy = f.spos[3 * (size_t)gstart + 1],
                 gz = f.spos[3 * (size_t)gstart + 2];
    const float tx = (float)__dsub_rn(f.spos[3 * (size_t)r], gx);
    const float ty = (float)__dsub_rn(f.spos[3 * (size_t)r + 1], gy);
    const float tz = (float)__dsub_rn(f.spos[3 * (size_t)r + 2], gz);
    float rw = live ? fmaxf(fabsf(tx), fmaxf(fabsf(ty), fabsf(tz))) : 0.0f;
    for (int o = 32; o > 0; o >>= 1) rw = fmaxf(rw, __shfl_xor(rw, o, 64));
    rw = __uint_as_float(uni(__float_as_uint(rw))) * (1.0f + 4.0f * kU32);
    const double theta = sd.theta;
    const float eps2 = (float)(sd.eps * sd.eps);
    const float band2 = 16.0f * kU32 * kU32;

    uint32_t ne = 0, total = 0, prev = kListNone;   // wave-uniform
    unsigned long long res = 0;                      // next reserved local chunk index
    uint32_t nres = 0;                               // reserved chunks left
    uint4 mine = make_uint4(0, 0, 0, 0);             // entry `lane` of the chunk being filled
    auto flush_chunk = [&]() {
        // group gi takes chunk ids part + kListParts t from the counter of part = gi mod
        // kListParts (counters on separate 256-byte lines), kListReserve at a time, so that few
        // waves meet on one address
        const uint32_t part = gi % kListParts;
        if (nres == 0) {
            unsigned long long base = 0;
            if (lane == 0) base = atomicAdd(ld.ctr + (size_t)part * 32, (unsigned long long)kListReserve);
            res = __shfl(base, 0, 64);
            nres = kListReserve;
        }
        const unsigned long long id = res * kListParts + part;
        ++res;
        --nres;
        if (id < ld.nchunks) {
            if ((uint32_t)lane < ne) ld.ent[id * 64 + lane] = mine;
            if (lane == 0) {
                if (prev == kListNone) ld.head[gi] = (uint32_t)id;
                else ld.next[prev] = (uint32_t)id;
                ld.next[id] = kListNone;
            }
        }
        prev = id < ld.nchunks ? (uint32_t)id : kListNone;
        total += ne;
        ne = 0;
    };
    // the chunk being filled lives in registers: entry k in lane k
    auto emit = [&](uint32_t a, uint32_t b, uint64_t m) {
        if ((uint32_t)lane == ne) mine = make_uint4(a, b, (uint32_t)m, (uint32_t)(m >> 32));
        if (++ne == 64) flush_chunk();
    };

    int sp = 0;
    const uint64_t m0 = ballot(live);
    if (lane == 0) L.stk[0] = make_uint4(sid, 1u, (uint32_t)m0, (uint32_t)(m0 >> 32));
    wave_sync();
    sp = 1;
    while (sp > 0) {
        --sp;
        const uint4 e = L.stk[sp];
        const uint32_t link = uni(e.x), nch = uni(e.y);
        const uint64_t emask = ((uint64_t)uni(e.w) << 32) | uni(e.z);
        wave_sync();
        if ((uint32_t)lane < nch) {
            const WRec32 &w = f.w32[link + lane];
            const float qx = (float)__dsub_rn(w.cx, gx);
            const float qy = (float)__dsub_rn(w.cy, gy);
            const float qz = (float)__dsub_rn(w.cz, gz);
            const float rho = fmaf(fmaxf(fabsf(qx), fmaxf(fabsf(qy), fabsf(qz))), 1.0f + 4.0f * kU32, rw);
            const float B = fmaf(rho, fmaf(band2, rho, w.band1), w.band0);
            L.sa[lane] = make_float4(qx, qy, qz, w.m);
            L.sb[lane] = make_float2((w.Sp + B) * (1.0f + 4.0f * kU32), fmaxf(w.Sp - B, 0.0f) * (1.0f - 4.0f * kU32));
            L.sl[lane] = make_uint2(w.link, w.cnt);
            L.sc[lane] = make_uint2(w.gid, w.level);
        }
        wave_sync();
        emit(kListEntry, nch, 0);
#pragma unroll
        for (uint32_t c = 0; c < 8; ++c) {
            if (c >= nch) break;
            const float4 qa = L.sa[c];
            const float dx = qa.x - tx, dy = qa.y - ty, dz = qa.z - tz;
            const float E2 = fmaf(dz, dz, fmaf(dy, dy, fmaf(dx, dx, eps2)));
            uint64_t accm = ballot(E2 > L.sb[c].x) & emask;
            uint64_t open = emask & ~accm;
            if (open) {
                const uint64_t ambm = ballot(!(E2 < L.sb[c].y)) & open;
                if (ambm) {
                    bool ex = false;
                    if (in_mask(ambm)) {
                        const WRec32 &wc = f.w32[link + c];
                        const double cm[3] = {wc.cx, wc.cy, wc.cz};
                        const double *xp = f.spos + 3 * (size_t)r;
                        const double ex_ = __dsub_rn(cm[0], xp[0]), ey = __dsub_rn(cm[1], xp[1]),
                                     ez = __dsub_rn(cm[2], xp[2]);
                        const double ED2 =
                            __dadd_rn(__dadd_rn(__dmul_rn(ex_, ex_), __dmul_rn(ey, ey)), __dmul_rn(ez, ez));
                        ex = f.w32[link + c].r2 < __dmul_rn(__dmul_rn(theta, theta), ED2);
                    }
                    accm |= ballot(ex) & ambm;
                    open = emask & ~accm;
                }
            }
            if (open) {
                const uint2 ql = L.sl[c];
                const uint32_t qlink = uni(ql.x), qcnt = uni(ql.y);
                if (qcnt & kLeafBit) {
                    emit(qlink, kListLeaf | (qcnt & ~kLeafBit), open);
                } else if (sp < kStackMax) {
                    if (lane == 0) L.stk[sp] = make_uint4(qlink, qcnt, (uint32_t)open, (uint32_t)(open >> 32));
                    wave_sync();
                    ++sp;
                } else if (lane == 0) {
                    atomicOr(f.err, kErrStack);
                }
            }
            if (accm) emit(link + c, uni(L.sc[c].x), accm);
        }
    }
    if (ne) flush_chunk();
    if (lane == 0) ld.count[gi] = total;
}

template <bool POT, bool SOFT, int W, bool QUAD>
__global__ void __launch_bounds__(64 * W) k_lists_eval32(ForestDev f, ListDev ld, WalkOut out) {
    __shared__ WaveLds32 lds_all[W];
    __shared__ float4 mst_all[W][64];   // accepted cubes of the current chunk: centre rel g, mass
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    WaveLds32 &L = lds_all[wave];
    float4 *mst = mst_all[wave];
    const uint32_t gi = blockIdx.x * W + wave;
    if (gi >= f.ngroups) return;
    if (uni(*f.err) & (kErrTree | kErrStack)) return;
    const GroupDesc gd = f.groups[gi];
    const uint32_t sid = uni(gd.seg);
    const SegDesc &sd = f.seg[sid];
    if (sd.precision != 1 || sd.group || (sd.quad != 0) != QUAD || unsoftened(sd.eps) == SOFT) return;
    const uint32_t gstart = uni(gd.start);
    const bool live = (uint32_t)lane < gd.count;
    const uint32_t r = gstart + (live ? (uint32_t)lane : 0u);
    const double gx = f.spos[3 * (size_t)gstart], gy = f.spos[3 * (size_t)gstart + 1],
                 gz = f.spos[3 * (size_t)gstart + 2];
    const float tx = (float)__dsub_rn(f.spos[3 * (size_t)r], gx);
    const float ty = (float)__dsub_rn(f.spos[3 * (size_t)r + 1], gy);
    const float tz = (float)__dsub_rn(f.spos[3 * (size_t)r + 2], gz);
    const float eps2 = (float)(sd.eps * sd.eps);
    constexpr bool soft = SOFT;

    float ax = 0.f, ay = 0.f, az = 0.f, ap = 0.f;
    float sx = 0.f, sy = 0.f, sz = 0.f, sp_ = 0.f;
    float cx = 0.f, cy = 0.f, cz = 0.f, cp = 0.f;
    uint32_t work = 0, qn = 0;
    auto fold = [&]() {
        kahan_add(sx, cx, ax); ax = 0.f;
        kahan_add(sy, cy, ay); ay = 0.f;
        kahan_add(sz, cz, az); az = 0.f;
        if (POT) { kahan_add(sp_, cp, ap); ap = 0.f; }
        work = 0;
    };
    auto pair = [&](float px, float py, float pz, float pm) {
        const float dx = px - tx, dy = py - ty, dz = pz - tz;
        const float r2 = fmaf(dz, dz, fmaf(dy, dy, fmaf(dx, dx, eps2)));
        if (soft || r2 > 0.0f) {
            const float ri = __builtin_amdgcn_rsqf(r2);
            const float mr = pm * ri;
            const float w3 = mr * ri * ri;
            ax = fmaf(w3, dx, ax);
            ay = fmaf(w3, dy, ay);
            az = fmaf(w3, dz, az);
            if (POT) ap -= mr;
        }
    };
    auto flush_leaves = [&]() {
        if (qn == 0) return;
        if (work + qn > kFlushWork) fold();
        work += qn;
        if (!SOFT) {
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
            }
        }
        qn = 0;
        wave_sync();
    };

    const uint32_t n = uni(ld.count[gi]);
    uint32_t chunk = uni(ld.head[gi]);
    for (uint32_t k0 = 0; k0 < n; k0 += 64) {
        const uint32_t nb = n - k0 < 64u ? n - k0 : 64u;
        const uint4 mine = (uint32_t)lane < nb ? ld.ent[(size_t)chunk * 64 + lane] : make_uint4(0, 0, 0, 0);
        // the chunk's accepted cubes, converted lane-parallel as the walk stages children
        wave_sync();
        if ((uint32_t)lane < nb && mine.x != kListEntry && !(mine.y & kListLeaf)) {
            const WRec32 &w = f.w32[mine.x];
            mst[lane] = make_float4((float)__dsub_rn(w.cx, gx), (float)__dsub_rn(w.cy, gy),
                                    (float)__dsub_rn(w.cz, gz), w.m);
        }
        wave_sync();
        for (uint32_t k = 0; k < nb; ++k) {
            const uint32_t a = (uint32_t)__builtin_amdgcn_readlane(mine.x, k);
            const uint32_t b = (uint32_t)__builtin_amdgcn_readlane(mine.y, k);
            const uint64_t m = ((uint64_t)(uint32_t)__builtin_amdgcn_readlane(mine.w, k) << 32) |
                               (uint64_t)(uint32_t)__builtin_amdgcn_readlane(mine.z, k);
            if (a == kListEntry) {
                if (work + b > kFlushWork) fold();
                work += b;
            } else if (b & kListLeaf) {
                const uint32_t np = b & ~kListLeaf;
                if (np <= 64u) {
                    if (qn + np > 64u) flush_leaves();
                    if ((uint32_t)lane < np) {
                        L.irank[qn + lane] = a + lane;
                        L.imask[qn + lane] = m;
                    }
                    qn += np;
                } else {
                    flush_leaves();
                    for (uint32_t b0 = 0; b0 < np; b0 += 64) {
                        const uint32_t nq = np - b0 < 64u ? np - b0 : 64u;
                        if ((uint32_t)lane < nq) {
                            L.irank[lane] = a + b0 + lane;
                            L.imask[lane] = m;
                        }
                        qn = nq;
                        flush_leaves();
                    }
                }
            } else if (in_mask(m)) {
                const float4 qa = mst[k];
                const float dx = qa.x - tx, dy = qa.y - ty, dz = qa.z - tz;
                const float E2 = fmaf(dz, dz, fmaf(dy, dy, fmaf(dx, dx, eps2)));
                const float ri = __builtin_amdgcn_rsqf(E2);
                const float mr = qa.w * ri;
                const float ri2 = ri * ri;
                const float w3 = mr * ri2;
                if (QUAD) {
                    // the walk's quadrupole term, from the moments of walk slot a
                    const float4 s0 = f.q32[2 * (size_t)a], s1 = f.q32[2 * (size_t)a + 1];
                    const float sdx = fmaf(s0.x, dx, fmaf(s0.w, dy, s1.x * dz));
                    const float sdy = fmaf(s0.w, dx, fmaf(s0.y, dy, s1.y * dz));
                    const float sdz = fmaf(s1.x, dx, fmaf(s1.y, dy, s0.z * dz));
                    const float A = fmaf(3.0f, fmaf(dx, sdx, fmaf(dy, sdy, dz * sdz)), -E2 * s1.z);
                    const float ri5 = ri2 * ri2 * ri;
                    float qx = -ri5 * fmaf(3.0f, sdx, -s1.z * dx) + 2.5f * A * ri5 * ri2 * dx;
                    float qy = -ri5 * fmaf(3.0f, sdy, -s1.z * dy) + 2.5f * A * ri5 * ri2 * dy;
                    float qz = -ri5 * fmaf(3.0f, sdz, -s1.z * dz) + 2.5f * A * ri5 * ri2 * dz;
                    float qp = -0.5f * A * ri5;
                    const uint64_t hard = ballot(s1.z > qa.w * E2) & m;
                    if (hard) {
                        if (in_mask(hard)) {
                            const WRec32 &wc = f.w32[a];
                            const double cm[3] = {wc.cx, wc.cy, wc.cz};
                            const double *xp = f.spos + 3 * (size_t)r;
                            const double *S = f.uQ + 6 * (size_t)a;
                            const double ex_ = cm[0] - xp[0], ey = cm[1] - xp[1], ez = cm[2] - xp[2];
                            const double e2 = ((ex_ * ex_ + ey * ey) + ez * ez) + (double)sd.eps * sd.eps;
                            const double tr = (S[0] + S[1]) + S[2];
                            const double sx = fma(S[0], ex_, fma(S[3], ey, S[4] * ez));
                            const double sy = fma(S[3], ex_, fma(S[1], ey, S[5] * ez));
                            const double sz = fma(S[4], ex_, fma(S[5], ey, S[2] * ez));
                            const double A64 = fma(3.0, fma(ex_, sx, fma(ey, sy, ez * sz)), -e2 * tr);
                            const double rinv = 1.0 / sqrt(e2);
                            const double r5 = rinv * rinv * rinv * rinv * rinv, r7 = r5 * rinv * rinv;
                            qx = (float)(2.5 * A64 * r7 * ex_ - r5 * fma(3.0, sx, -tr * ex_));
                            qy = (float)(2.5 * A64 * r7 * ey - r5 * fma(3.0, sy, -tr * ey));
                            qz = (float)(2.5 * A64 * r7 * ez - r5 * fma(3.0, sz, -tr * ez));
                            qp = (float)(-0.5 * A64 * r5);
                        }
                    }
                    ax += qx;
                    ay += qy;
                    az += qz;
                    if (POT) ap += qp;
                }
                ax = fmaf(w3, dx, ax);
                ay = fmaf(w3, dy, ay);
                az = fmaf(w3, dz, az);
                if (POT) ap -= mr;
            }
        }
        chunk = uni(ld.next[chunk]);
    }
    flush_leaves();
    fold();
    if (live) {
        const uint32_t i = f.idx[r];
        const size_t li = i - sd.start;
        const double G = sd.G;
        double *accb = seg_base(out.acc, sd.acc, sd, 3);
        accb[3 * li] = G * ((double)sx - (double)cx);
        accb[3 * li + 1] = G * ((double)sy - (double)cy);
        accb[3 * li + 2] = G * ((double)sz - (double)cz);
        if (POT) {
            double *potb = seg_base(out.pot, sd.pot, sd, 1);
            if (potb) potb[li] = G * ((double)sp_ - (double)cp);
        }
    }
}

// FP64 lists: k_walk64's decisions and order (no compensated sums, so no stack
// entry records); phase two replays them with k_walk64's arithmetic.
template <int W>
__global__ void __launch_bounds__(64 * W) k_lists64(ForestDev f, ListDev ld) {
    __shared__ WaveLds64<false> lds_all[W];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    WaveLds64<false> &L = lds_all[wave];
    const uint32_t gi = blockIdx.x * W + wave;
    if (gi >= f.ngroups) return;
    if (uni(*f.err) & kErrTree) return;
    const GroupDesc gd = f.groups[gi];
    const uint32_t sid = uni(gd.seg);
    const SegDesc &sd = f.seg[sid];
    if (sd.precision != 0 || sd.group) return;   // refused by the host
    const uint32_t gstart = uni(gd.start);
    const bool live = (uint32_t)lane < gd.count;
    const uint32_t r = gstart + (live ? (uint32_t)lane : 0u);
    const double tx = f.spos[3 * (size_t)r], ty = f.spos[3 * (size_t)r + 1], tz = f.spos[3 * (size_t)r + 2];
    const double theta2 = __dmul_rn(sd.theta, sd.theta);

    uint32_t ne = 0, total = 0, prev = kListNone;
    unsigned long long res = 0;
    uint32_t nres = 0;
    uint4 mine = make_uint4(0, 0, 0, 0);
    auto flush_chunk = [&]() {
        const uint32_t part = gi % kListParts;
        if (nres == 0) {
            unsigned long long base = 0;
            if (lane == 0) base = atomicAdd(ld.ctr + (size_t)part * 32, (unsigned long long)kListReserve);
            res = __shfl(base, 0, 64);
            nres = kListReserve;
        }
        const unsigned long long id = res * kListParts + part;
        ++res;
        --nres;
        if (id < ld.nchunks) {
            if ((uint32_t)lane < ne) ld.ent[id * 64 + lane] = mine;
            if (lane == 0) {
                if (prev == kListNone) ld.head[gi] = (uint32_t)id;
                else ld.next[prev] = (uint32_t)id;
                ld.next[id] = kListNone;
            }
        }
        prev = id < ld.nchunks ? (uint32_t)id : kListNone;
        total += ne;
        ne = 0;
    };
    auto emit = [&](uint32_t a, uint32_t b, uint64_t m) {
        if ((uint32_t)lane == ne) mine = make_uint4(a, b, (uint32_t)m, (uint32_t)(m >> 32));
        if (++ne == 64) flush_chunk();
    };

    int sp = 0;
    const uint64_t m0 = ballot(live);
    if (lane == 0) L.stk[0] = make_uint4(sid, 1u, (uint32_t)m0, (uint32_t)(m0 >> 32));
    wave_sync();
    sp = 1;
    while (sp > 0) {
        --sp;
        const uint4 e = L.stk[sp];
        const uint32_t link = uni(e.x), nch = uni(e.y);
        const uint64_t emask = ((uint64_t)uni(e.w) << 32) | uni(e.z);
        wave_sync();
        if ((uint32_t)lane < nch) {
            const WRec64 &w = f.w64[link + lane];
            L.sa[lane] = make_double4(w.x, w.y, w.z, w.m);
            L.sS[lane] = w.S;
            L.sb[lane] = make_uint4(w.link, w.cnt, w.gid, w.level);
        }
        wave_sync();
#pragma unroll
        for (uint32_t c = 0; c < 8; ++c) {
            if (c >= nch) break;
            const double4 qa = L.sa[c];
            const double S = L.sS[c];
            const double dx = __dsub_rn(qa.x, tx), dy = __dsub_rn(qa.y, ty), dz = __dsub_rn(qa.z, tz);
            const double D2 = __dadd_rn(__dadd_rn(__dmul_rn(dx, dx), __dmul_rn(dy, dy)), __dmul_rn(dz, dz));
            const uint64_t accm = ballot(S < __dmul_rn(theta2, D2)) & emask;
            const uint64_t open = emask & ~accm;
            if (open) {
                const uint4 qb = L.sb[c];
                const uint32_t qlink = uni(qb.x), qcnt = uni(qb.y);
                if (qcnt & kLeafBit) {
                    emit(qlink, kListLeaf | (qcnt & ~kLeafBit), open);
                } else if (sp < kStackMax) {
                    if (lane == 0) L.stk[sp] = make_uint4(qlink, qcnt, (uint32_t)open, (uint32_t)(open >> 32));
                    wave_sync();
                    ++sp;
                } else if (lane == 0) {
                    atomicOr(f.err, kErrStack);
                }
            }
            if (accm) emit(link + c, uni(L.sb[c].z), accm);
        }
    }
    if (ne) flush_chunk();
    if (lane == 0) ld.count[gi] = total;
}

template <bool POT, bool QUAD>
__global__ void __launch_bounds__(256) k_lists_eval64(ForestDev f, ListDev ld, WalkOut out) {
    __shared__ WaveLds64<false> lds_all[4];
    __shared__ double4 mst_all[4][64];   // accepted cubes of the current chunk: centre, mass
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    WaveLds64<false> &L = lds_all[wave];
    double4 *mst = mst_all[wave];
    const uint32_t gi = blockIdx.x * 4 + wave;
    if (gi >= f.ngroups) return;
    if (uni(*f.err) & (kErrTree | kErrStack)) return;
    const GroupDesc gd = f.groups[gi];
    const uint32_t sid = uni(gd.seg);
    const SegDesc &sd = f.seg[sid];
    if (sd.precision != 0 || sd.group || (sd.quad != 0) != QUAD) return;
    const uint32_t gstart = uni(gd.start);
    const bool live = (uint32_t)lane < gd.count;
    const uint32_t r = gstart + (live ? (uint32_t)lane : 0u);
    const double tx = f.spos[3 * (size_t)r], ty = f.spos[3 * (size_t)r + 1], tz = f.spos[3 * (size_t)r + 2];
    const double eps2 = __dmul_rn(sd.eps, sd.eps);
    const bool soft = eps2 > 0.0;

    double ax = 0.0, ay = 0.0, az = 0.0, ap = 0.0;
    uint32_t qn = 0;
    auto pair = [&](double px, double py, double pz, double pm) {
        const double dx = px - tx, dy = py - ty, dz = pz - tz;
        const double r2 = fma(dz, dz, fma(dy, dy, fma(dx, dx, eps2)));
        if (soft || r2 > 0.0) {
            const double ri = rsqrt64(r2);
            const double mr = pm * ri;
            const double w3 = mr * ri * ri;
            ax = fma(w3, dx, ax);
            ay = fma(w3, dy, ay);
            az = fma(w3, dz, az);
            if (POT) ap -= mr;
        }
    };
    auto flush_leaves = [&]() {
        if (qn == 0) return;
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
                }
            }
        }
        qn = 0;
        wave_sync();
    };

    const uint32_t n = uni(ld.count[gi]);
    uint32_t chunk = uni(ld.head[gi]);
    for (uint32_t k0 = 0; k0 < n; k0 += 64) {
        const uint32_t nb = n - k0 < 64u ? n - k0 : 64u;
        const uint4 mine = (uint32_t)lane < nb ? ld.ent[(size_t)chunk * 64 + lane] : make_uint4(0, 0, 0, 0);
        wave_sync();
        if ((uint32_t)lane < nb && mine.x != kListEntry && !(mine.y & kListLeaf)) {
            const WRec64 &w = f.w64[mine.x];
            mst[lane] = make_double4(w.x, w.y, w.z, w.m);
        }
        wave_sync();
        for (uint32_t k = 0; k < nb; ++k) {
            const uint32_t a = (uint32_t)__builtin_amdgcn_readlane(mine.x, k);
            const uint32_t b = (uint32_t)__builtin_amdgcn_readlane(mine.y, k);
            const uint64_t m = ((uint64_t)(uint32_t)__builtin_amdgcn_readlane(mine.w, k) << 32) |
                               (uint64_t)(uint32_t)__builtin_amdgcn_readlane(mine.z, k);
            if (a == kListEntry) continue;
            if (b & kListLeaf) {
                const uint32_t np = b & ~kListLeaf;
                if (np <= 64u) {
                    if (qn + np > 64u) flush_leaves();
                    if ((uint32_t)lane < np) {
                        L.irank[qn + lane] = a + lane;
                        L.imask[qn + lane] = m;
                    }
                    qn += np;
                } else {
                    flush_leaves();
                    for (uint32_t b0 = 0; b0 < np; b0 += 64) {
                        const uint32_t nq = np - b0 < 64u ? np - b0 : 64u;
                        if ((uint32_t)lane < nq) {
                            L.irank[lane] = a + b0 + lane;
                            L.imask[lane] = m;
                        }
                        qn = nq;
                        flush_leaves();
                    }
                }
            } else if (in_mask(m)) {
                const double4 qa = mst[k];
                const double dx = __dsub_rn(qa.x, tx), dy = __dsub_rn(qa.y, ty), dz = __dsub_rn(qa.z, tz);
                const double D2 = __dadd_rn(__dadd_rn(__dmul_rn(dx, dx), __dmul_rn(dy, dy)), __dmul_rn(dz, dz));
                const double E2 = D2 + eps2;
                const double ri = rsqrt64(E2);
                const double mr = qa.w * ri;
                const double ri2 = ri * ri;
                double w3 = mr * ri2;
                if (QUAD) {
                    // the walk's quadrupole term, from the moments of walk slot a
                    const double *q = f.q64 + 6 * (size_t)a;
                    const double sdx = fma(q[0], dx, fma(q[3], dy, q[4] * dz));
                    const double sdy = fma(q[3], dx, fma(q[1], dy, q[5] * dz));
                    const double sdz = fma(q[4], dx, fma(q[5], dy, q[2] * dz));
                    const double tr = (q[0] + q[1]) + q[2];
                    const double A = fma(3.0, fma(dx, sdx, fma(dy, sdy, dz * sdz)), -E2 * tr);
                    const double ri5 = ri2 * ri2 * ri;
                    w3 = fma(2.5 * A, ri5 * ri2, w3);
                    ax = fma(-ri5, fma(3.0, sdx, -tr * dx), ax);
                    ay = fma(-ri5, fma(3.0, sdy, -tr * dy), ay);
                    az = fma(-ri5, fma(3.0, sdz, -tr * dz), az);
                    if (POT) ap -= 0.5 * A * ri5;
                }
                ax = fma(w3, dx, ax);
                ay = fma(w3, dy, ay);
                az = fma(w3, dz, az);
                if (POT) ap -= mr;
            }
        }
        chunk = uni(ld.next[chunk]);
    }
    flush_leaves();
    if (live) {
        const uint32_t i = f.idx[r];
        const size_t li = i - sd.start;
        const double G = sd.G;
        double *accb = seg_base(out.acc, sd.acc, sd, 3);
        accb[3 * li] = G * ax;
        accb[3 * li + 1] = G * ay;
        accb[3 * li + 2] = G * az;
        if (POT) {
            double *potb = seg_base(out.pot, sd.pot, sd, 1);
            if (potb) potb[li] = G * ap;
        }
    }
}

hipError_t launch_lists_build(const ForestDev &f, const ListDev &ld, hipStream_t s) {
    if (f.ngroups == 0) return hipSuccess;
    if (f.has32) hipLaunchKernelGGL((k_lists32<4>), dim3((f.ngroups + 3) / 4), dim3(256), 0, s, f, ld);
    if (f.has64) hipLaunchKernelGGL((k_lists64<4>), dim3((f.ngroups + 3) / 4), dim3(256), 0, s, f, ld);
    return hipGetLastError();
}

template <bool POT>
static void launch_lists_eval_p(const ForestDev &f, const ListDev &ld, const WalkOut &o, hipStream_t s) {
    const dim3 g((f.ngroups + 3) / 4), b(256);
    if (f.has32 & var_bit(false, false)) hipLaunchKernelGGL((k_lists_eval32<POT, true, 4, false>), g, b, 0, s, f, ld, o);
    if (f.has32 & var_bit(true, false)) hipLaunchKernelGGL((k_lists_eval32<POT, true, 4, true>), g, b, 0, s, f, ld, o);
    if (f.has32 & var_bit(false, true)) hipLaunchKernelGGL((k_lists_eval32<POT, false, 4, false>), g, b, 0, s, f, ld, o);
    if (f.has32 & var_bit(true, true)) hipLaunchKernelGGL((k_lists_eval32<POT, false, 4, true>), g, b, 0, s, f, ld, o);
    if (f.has64 & (var_bit(false, false) | var_bit(false, true)))
        hipLaunchKernelGGL((k_lists_eval64<POT, false>), g, b, 0, s, f, ld, o);
    if (f.has64 & kVarQuadBits) hipLaunchKernelGGL((k_lists_eval64<POT, true>), g, b, 0, s, f, ld, o);
}

hipError_t launch_lists_eval(const ForestDev &f, const ListDev &ld, bool want_pot, double *acc, double *pot,
                             hipStream_t s) {
    if (f.ngroups == 0) return hipSuccess;
    WalkOut o{acc, pot, nullptr, nullptr, nullptr};
    if (want_pot) launch_lists_eval_p<true>(f, ld, o, s);
    else launch_lists_eval_p<false>(f, ld, o, s);
    return hipGetLastError();
}

template <bool STATS, bool POT, int W>
static void launch_walk_sp(const ForestDev &f, const WalkOut &o, hipStream_t s) {
    const unsigned blocks = (f.ngroups + W - 1) / W;
    const dim3 g(blocks), b(64 * W);
    if (f.has32 & var_bit(false, false)) hipLaunchKernelGGL((k_walk32<STATS, POT, W, false, true>), g, b, 0, s, f, o);
    if (f.has32 & var_bit(true, false)) hipLaunchKernelGGL((k_walk32<STATS, POT, W, true, true>), g, b, 0, s, f, o);
    if (f.has32 & var_bit(false, true)) hipLaunchKernelGGL((k_walk32<STATS, POT, W, false, false>), g, b, 0, s, f, o);
    if (f.has32 & var_bit(true, true)) hipLaunchKernelGGL((k_walk32<STATS, POT, W, true, false>), g, b, 0, s, f, o);
    if (f.has64 & (var_bit(false, false) | var_bit(false, true)))
        hipLaunchKernelGGL((k_walk64<STATS, POT, W, false>), g, b, 0, s, f, o);
    if (f.has64 & kVarQuadBits) hipLaunchKernelGGL((k_walk64<STATS, POT, W, true>), g, b, 0, s, f, o);
    const dim3 g4((f.ngroups + 3) / 4), b4(256);
    if (f.has32 & kVarGroup) hipLaunchKernelGGL((k_gwalk32<STATS, POT>), g4, b4, 0, s, f, o);
    if (f.has64 & kVarGroup) hipLaunchKernelGGL((k_gwalk64<STATS, POT>), g4, b4, 0, s, f, o);
}

template <int W>
static void launch_walk_w(const ForestDev &f, bool want_pot, const WalkOut &o, hipStream_t s) {
    if (want_pot) launch_walk_sp<false, true, W>(f, o, s);
    else launch_walk_sp<false, false, W>(f, o, s);
}

hipError_t launch_walk(const ForestDev &f, bool stats, bool want_pot, double *acc, double *pot, int64_t *n_mono,
                       int64_t *n_p2p, uint64_t *hash, hipStream_t s, int waves, uint32_t wlo, uint32_t whi,
                       int64_t *work, int64_t *gwork) {
    WalkOut o{acc, pot, n_mono, n_p2p, hash, wlo, whi, work, gwork};
    if (f.ngroups == 0) return hipSuccess;
    if (stats) {   // the counting walks use one launch shape
        if (want_pot) launch_walk_sp<true, true, 4>(f, o, s);
        else launch_walk_sp<true, false, 4>(f, o, s);
        return hipGetLastError();
    }
    switch (waves) {
        case 1: launch_walk_w<1>(f, want_pot, o, s); break;
        case 2: launch_walk_w<2>(f, want_pot, o, s); break;
        case 8: launch_walk_w<8>(f, want_pot, o, s); break;
        default: launch_walk_w<4>(f, want_pot, o, s); break;
    }
    return hipGetLastError();
}

}  // namespace bh
