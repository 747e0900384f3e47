// FP32-mode force walk (see k_walk32).
#include "bh_walk_common.h"

namespace bh {

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
//
// GROUP (the group-criterion variant): each lane decides with its group's
// bounding box instead of its own position, in FP64 as the oracle writes it
// (group_accepts), so the FP32 band is not used; pair and monopole terms are the
// per-body walk's.
//
// One walk group (gi < f.ngroups) on one wavefront with its LDS block L.
template <bool STATS, bool POT, bool QUAD, bool SOFT, bool GROUP>
__device__ __forceinline__ void walk32_group(const ForestDev &f, const WalkOut &out, WaveLds32 &L, const int lane,
                                             const uint32_t gi) {
    const GroupDesc gd = f.groups[gi];
    const uint32_t sid = uni(gd.seg);
    const SegDesc &sd = f.seg[sid];
    if (sd.precision != 1 || (sd.group != 0) != GROUP || (sd.quad != 0) != QUAD || unsoftened(sd.eps) == SOFT)
        return;
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
    double blo[3], bhi[3];   // GROUP: this lane's group box
    if (GROUP)
        for (int d = 0; d < 3; ++d) {
            blo[d] = f.gbox[6 * (size_t)r + d];
            bhi[d] = f.gbox[6 * (size_t)r + 3 + d];
        }
    const double theta2 = __dmul_rn(theta, theta);
    const float eps2 = (float)(sd.eps * sd.eps);

    Sums32<STATS, POT, SOFT> sums{f, L, lane, r, gstart, gx, gy, gz, tx, ty, tz, eps2,
                               STATS ? (uint64_t)st.nn : 0ull, STATS ? sd.start : 0u};
    uint32_t nmono = 0, nvis = 0, nfb = 0;
    uint32_t wvis = 0, went = 0, wacc = 0, wleaf = 0;         // wave-level counters (uniform)

    // Depth-first stack of (first child slot, children, lane mask); the most recent
    // push stays in scalar registers and is the next pop, so only entries pushed
    // beneath another one go through LDS.
    int sp = 0;
    bool pend = true;
    uint32_t p_link = sid, p_cnt = 1u;
    uint64_t p_mask = ballot(live);
    for (;;) {
        uint32_t link, nch;
        uint64_t emask;
        if (pend) {
            link = p_link;
            nch = p_cnt;
            emask = p_mask;
            pend = false;
        } else {
            if (sp == 0) break;
            --sp;
            const uint4 e = L.stk[sp];
            link = uni(e.x);
            nch = uni(e.y);
            emask = ((uint64_t)uni(e.w) << 32) | uni(e.z);
        }
        if (STATS) sums.wwork += nch;
        wave_sync();
        stage_children32<STATS, QUAD, GROUP>(f, L, lane, link, nch, gx, gy, gz, rw);
        wave_sync();
        if (sums.work + nch > kFlushWork) sums.fold();
        sums.work += nch;
        if (STATS) { wvis += nch; ++went; }
#pragma unroll
        for (uint32_t c = 0; c < 8; ++c) {
            if (c >= nch) break;
            const float4 qa = L.sa[c];
            const float dx = qa.x - tx, dy = qa.y - ty, dz = qa.z - tz;
            const float E2 = fmaf(dz, dz, fmaf(dy, dy, fmaf(dx, dx, eps2)));
            uint64_t accm, open;
            if (GROUP) {
                accm = ballot(group_accepts(L.x.g.cx[c], L.x.g.cy[c], L.x.g.cz[c], L.x.g.r2[c], blo, bhi, theta2)) &
                       emask;
                open = emask & ~accm;
            } else {
                // the lanes of the entry that do not accept (an and-not that sets the scalar condition
                // for the branch below), then the accepting ones
                open = emask & ~ballot(E2 > L.sbh[c]);
                accm = emask & ~open;
            }
            if (open) {
                const uint64_t ambm = GROUP ? 0 : ballot(!(E2 < L.sbl[c])) & open;
                if (ambm) {
                    // within the FP32 rounding bound of the threshold: decide exactly in FP64
                    bool ex = false;
                    if (in_mask(ambm)) {
                        ex = exact_accept32(f, link + c, r, theta);
                        if (STATS) ++nfb;
                    }
                    accm |= ballot(ex) & ambm;
                    open = emask & ~accm;
                }
                if (open) {
                    const uint2 ql = L.sl[c];
                    const uint32_t qlink = uni(ql.x), qcnt = uni(ql.y);
                    if (qcnt & kLeafBit) {
                        // queued; its pairs are taken after this entry
                        const uint32_t np = qcnt & ~kLeafBit;
                        if (STATS) ++wleaf;
                        sums.queue_leaf(qlink, np, open);
                    } else {
                        if (pend) {   // the pending entry goes beneath the new one
                            if (sp < kStackMax) {
                                if (lane == 0)
                                    L.stk[sp] = make_uint4(p_link, p_cnt, (uint32_t)p_mask, (uint32_t)(p_mask >> 32));
                                ++sp;
                            } else if (lane == 0) {
                                atomicOr(f.err, kErrStack);   // result void; the walk still drains
                            }
                        }
                        pend = true;
                        p_link = qlink;
                        p_cnt = qcnt;
                        p_mask = open;
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
                    const float4 s0 = L.x.q.sq0[c], s1 = L.x.q.sq1[c];
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
                    sums.ax += qx;
                    sums.ay += qy;
                    sums.az += qz;
                    if (POT) sums.ap += qp;
                }
                sums.ax = fmaf(w3, dx, sums.ax);
                sums.ay = fmaf(w3, dy, sums.ay);
                sums.az = fmaf(w3, dz, sums.az);
                if (POT) sums.ap -= mr;
                if (STATS) {
                    ++nmono;
                    sums.h += mix64((uint64_t)(L.sc[c].x - st.nbase));
                }
            }
        }
        // room for the next entry's eight children: at most 56 queued particles, no overflow
        if (sums.qn > 56u || sums.nov) sums.flush();
    }
    sums.flush();
    sums.fold();
    const bool own = live && r >= out.wlo && r < out.whi;
    if (STATS && out.gwork && lane == 0) out.gwork[(gstart - sd.start) / kGroup] = (int64_t)sums.wwork;
    if (own) {
        const uint32_t i = f.idx[r];
        const size_t li = i - sd.start;
        const double G = sd.G;
        double *accb = seg_base(out.acc, sd.acc, sd, 3);
        if (accb) {   // null: a counting walk for the checksums only
            accb[3 * li] = G * ((double)sums.sx - (double)sums.cx);
            accb[3 * li + 1] = G * ((double)sums.sy - (double)sums.cy);
            accb[3 * li + 2] = G * ((double)sums.sz - (double)sums.cz);
        }
        if (POT) {
            double *potb = seg_base(out.pot, sd.pot, sd, 1);
            if (potb) potb[li] = G * ((double)sums.sp - (double)sums.cp);
        }
        if (STATS) {
            if (out.n_mono) out.n_mono[i] = nmono;
            if (out.n_p2p) out.n_p2p[i] = sums.np2p;
            if (out.hash) out.hash[i] = sums.h;
            if (out.work) {   // the group's wavefront work, spread evenly over its bodies
                const uint64_t wg = sums.wwork, k = (uint32_t)lane, c = gd.count;
                out.work[i] = (int64_t)((wg * (k + 1)) / c - (wg * k) / c);
            }
        }
    }
    if (STATS) {
        unsigned long long a = wave_sum_u(own ? nmono : 0), b = wave_sum_u(own ? sums.np2p : 0);
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


// Walk launches.  Grid form: W wavefronts per workgroup, wavefront w of workgroup b
// walks group b W + w.  Persistent form (PERSIST): as many workgroups as the device
// holds at once; each wavefront takes the next group index from the counter q (one
// atomic add per group, zero at launch) until the index passes the last group, so
// a wavefront that finishes early starts another group at once and a workgroup's
// LDS is held only while groups remain.  The form changes no result.
template <bool STATS, bool POT, int W, bool QUAD, bool SOFT, bool GROUP, bool PERSIST>
__global__ void __launch_bounds__(64 * W, (PERSIST && SOFT && !QUAD && !POT) ? 8 : 1) k_walk32(ForestDev f, WalkOut out, uint32_t *q) {
    __shared__ WaveLds32 lds_all[W];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (uni(f.err[kErrWordTree]) & kErrTree) return;   // tree inconsistent: never walk it
    if (!PERSIST) {
        const uint32_t gi = blockIdx.x * W + wave;
        if (gi < f.ngroups) walk32_group<STATS, POT, QUAD, SOFT, GROUP>(f, out, lds_all[wave], lane, gi);
        return;
    }
    for (;;) {
        uint32_t gi = 0;
        if (lane == 0) gi = atomicAdd(q, 1u);
        gi = uni((uint32_t)__shfl((int)gi, 0, 64));
        if (gi >= f.ngroups) break;
        wave_sync();
        walk32_group<STATS, POT, QUAD, SOFT, GROUP>(f, out, lds_all[wave], lane, gi);
    }
}

// Variant v of the FP32 family: (QUAD, SOFT, GROUP), its counter slot is v.
template <bool STATS, bool POT, int W, bool PERSIST>
static void launch_w32(const ForestDev &f, const WalkOut &o, hipStream_t s) {
    const uint32_t nb = (f.ngroups + W - 1) / W;
#define BH_W32(v, QUAD, SOFT, GROUP)                                                                       \
    if (f.has32 & var_bit(QUAD, !(SOFT), GROUP)) {                                                        \
        auto k = k_walk32<STATS, POT, W, QUAD, SOFT, GROUP, PERSIST>;                                     \
        const dim3 g(PERSIST ? persistent_blocks((const void *)k, nb, 64 * W) : nb), b(64 * W);           \
        hipLaunchKernelGGL(k, g, b, 0, s, f, o, f.wq + (v));                                             \
    }
    BH_W32(0, false, true, false);
    BH_W32(1, true, true, false);
    BH_W32(2, false, false, false);
    BH_W32(3, true, false, false);
    BH_W32(4, false, true, true);
    BH_W32(5, false, false, true);
#undef BH_W32
}

template <bool POT, bool PERSIST>
static void launch_w32_shape(const ForestDev &f, const WalkOut &o, int W, hipStream_t s) {
    switch (W) {
        case 1: launch_w32<false, POT, 1, PERSIST>(f, o, s); break;
        case 2: launch_w32<false, POT, 2, PERSIST>(f, o, s); break;
        case 8: launch_w32<false, POT, 8, PERSIST>(f, o, s); break;
        default: launch_w32<false, POT, 4, PERSIST>(f, o, s); break;
    }
}

void launch_walk32_family(const ForestDev &f, const WalkOut &o, bool stats, bool pot, int shape, hipStream_t s) {
    if (!f.has32) return;
    const int W = shape & kWalkWavesMask;
    const bool persist = (shape & kWalkPersistent) != 0;
    if (stats) {   // the counting walks use one launch shape
        if (pot) launch_w32<true, true, 4, false>(f, o, s);
        else launch_w32<true, false, 4, false>(f, o, s);
    } else if (persist) {
        if (pot) launch_w32_shape<true, true>(f, o, W, s);
        else launch_w32_shape<false, true>(f, o, W, s);
    } else if (pot) {
        launch_w32_shape<true, false>(f, o, W, s);
    } else {
        launch_w32_shape<false, false>(f, o, W, s);
    }
}

}  // namespace bh
