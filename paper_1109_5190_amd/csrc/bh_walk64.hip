// FP64-mode force walk (see k_walk64).
#include "bh_walk_common.h"

namespace bh {

// ------------------------------------------------------------- FP64 walk ---


// GROUP (the group-criterion variant): each lane tests cubes against its group's
// bounding box (group_accepts) instead of its own position.
//
// One walk group (gi < f.ngroups) on one wavefront with its LDS block L.
template <bool STATS, bool POT, bool QUAD, bool GROUP>
__device__ __forceinline__ void walk64_group(const ForestDev &f, const WalkOut &out, WaveLds64<QUAD> &L,
                                             const int lane, const uint32_t gi) {
    const GroupDesc gd = f.groups[gi];
    const uint32_t sid = uni(gd.seg);
    const SegDesc &sd = f.seg[sid];
    if (sd.precision != 0 || (sd.group != 0) != GROUP || (sd.quad != 0) != QUAD) return;
    const SegState &st = f.st[sid];
    const uint32_t gstart = uni(gd.start);
    const bool live = (uint32_t)lane < gd.count;
    const uint32_t r = gstart + (live ? (uint32_t)lane : 0u);
    const double tx = f.spos[3 * (size_t)r], ty = f.spos[3 * (size_t)r + 1], tz = f.spos[3 * (size_t)r + 2];
    const double theta2 = __dmul_rn(sd.theta, sd.theta);
    double blo[3], bhi[3];   // GROUP: this lane's group box
    if (GROUP)
        for (int d = 0; d < 3; ++d) {
            blo[d] = f.gbox[6 * (size_t)r + d];
            bhi[d] = f.gbox[6 * (size_t)r + 3 + d];
        }
    const double eps2 = __dmul_rn(sd.eps, sd.eps);
    Sums64<STATS, POT, WaveLds64<QUAD>> sums{f, L, lane, gstart, tx, ty, tz, eps2,
                                          STATS ? (uint64_t)st.nn : 0ull, STATS ? sd.start : 0u};
    uint32_t nmono = 0, nvis = 0;

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
        stage_children64<QUAD>(f, L, lane, link, nch);
        wave_sync();
#pragma unroll
        for (uint32_t c = 0; c < 8; ++c) {
            if (c >= nch) break;
            const double4 qa = L.sa[c];
            const double S = L.sS[c];
            const double dx = __dsub_rn(qa.x, tx), dy = __dsub_rn(qa.y, ty), dz = __dsub_rn(qa.z, tz);
            const double D2 = __dadd_rn(__dadd_rn(__dmul_rn(dx, dx), __dmul_rn(dy, dy)), __dmul_rn(dz, dz));
            const uint64_t accm =
                ballot(GROUP ? group_accepts(qa.x, qa.y, qa.z, S, blo, bhi, theta2) : S < __dmul_rn(theta2, D2)) & emask;
            if (STATS && in_mask(emask)) ++nvis;
            const uint64_t open = emask & ~accm;
            if (open) {
                const uint4 qb = L.sb[c];
                const uint32_t qlink = uni(qb.x), qcnt = uni(qb.y);
                if (qcnt & kLeafBit) {
                    sums.queue_leaf(qlink, qcnt & ~kLeafBit, open);
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
            if (in_mask(accm)) {
                // softened monopole, executed by the accepting lanes only
                __asm__ volatile("");
                const double E2 = D2 + eps2;
                double w3, mr = 0.0;
                if (!QUAD) mono64<POT>(E2, qa.w, w3, mr);
                if (QUAD) {
                    const double ri = rsqrt64(E2);
                    const double ri2 = ri * ri;
                    mr = qa.w * ri;
                    w3 = mr * ri2;
                    const double *q = &L.sq[6 * c];
                    const double sdx = fma(q[0], dx, fma(q[3], dy, q[4] * dz));
                    const double sdy = fma(q[3], dx, fma(q[1], dy, q[5] * dz));
                    const double sdz = fma(q[4], dx, fma(q[5], dy, q[2] * dz));
                    const double tr = (q[0] + q[1]) + q[2];
                    const double A = fma(3.0, fma(dx, sdx, fma(dy, sdy, dz * sdz)), -E2 * tr);
                    const double ri5 = ri2 * ri2 * ri;
                    w3 = fma(2.5 * A, ri5 * ri2, w3);
                    sums.ax = fma(-ri5, fma(3.0, sdx, -tr * dx), sums.ax);
                    sums.ay = fma(-ri5, fma(3.0, sdy, -tr * dy), sums.ay);
                    sums.az = fma(-ri5, fma(3.0, sdz, -tr * dz), sums.az);
                    if (POT) sums.ap -= 0.5 * A * ri5;
                }
                sums.ax = fma(w3, dx, sums.ax);
                sums.ay = fma(w3, dy, sums.ay);
                sums.az = fma(w3, dz, sums.az);
                if (POT) sums.ap -= mr;
                if (STATS) {
                    ++nmono;
                    sums.h += mix64((uint64_t)(L.sb[c].z - st.nbase));
                }
            }
        }
    }
    sums.flush_leaves();
    const bool own = live && r >= out.wlo && r < out.whi;
    if (STATS && out.gwork && lane == 0) out.gwork[(gstart - sd.start) / kGroup] = (int64_t)sums.wwork;
    if (own) {
        const uint32_t i = f.idx[r];
        const size_t li = i - sd.start;
        const double G = sd.G;
        double *accb = seg_base(out.acc, sd.acc, sd, 3);
        if (accb) {   // null: a counting walk for the checksums only
            accb[3 * li] = G * sums.ax;
            accb[3 * li + 1] = G * sums.ay;
            accb[3 * li + 2] = G * sums.az;
        }
        if (POT) {
            double *potb = seg_base(out.pot, sd.pot, sd, 1);
            if (potb) potb[li] = G * sums.ap;
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
        unsigned long long v = wave_sum_u(own ? nvis : 0);
        if (lane == 0) {
            atomicAdd(&f.stats[0], a);
            atomicAdd(&f.stats[1], b);
            atomicAdd(&f.stats[2], v);
        }
    }
}


// Grid and persistent launch forms, as for the FP32 walk.
template <bool STATS, bool POT, int W, bool QUAD, bool GROUP, bool PERSIST>
__global__ void __launch_bounds__(64 * W, (PERSIST && !QUAD && !POT && !GROUP) ? 7 : 1) k_walk64(ForestDev f, WalkOut out, uint32_t *q) {
    __shared__ WaveLds64<QUAD> lds_all[W];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (uni(f.err[kErrWordTree]) & kErrTree) return;   // tree inconsistent: never walk it
    if (!PERSIST) {
        const uint32_t gi = blockIdx.x * W + wave;
        if (gi < f.ngroups) walk64_group<STATS, POT, QUAD, GROUP>(f, out, lds_all[wave], lane, gi);
        return;
    }
    for (;;) {
        uint32_t gi = 0;
        if (lane == 0) gi = atomicAdd(q, 1u);
        gi = uni((uint32_t)__shfl((int)gi, 0, 64));
        if (gi >= f.ngroups) break;
        wave_sync();
        walk64_group<STATS, POT, QUAD, GROUP>(f, out, lds_all[wave], lane, gi);
    }
}

// Variant v of the FP64 family: (QUAD, GROUP), its counter slot is 8 + v.
template <bool STATS, bool POT, int W, bool PERSIST>
static void launch_w64(const ForestDev &f, const WalkOut &o, hipStream_t s) {
    const uint32_t nb = (f.ngroups + W - 1) / W;
#define BH_W64(v, present, QUAD, GROUP)                                                                    \
    if (present) {                                                                                        \
        auto k = k_walk64<STATS, POT, W, QUAD, GROUP, PERSIST>;                                          \
        const dim3 g(PERSIST ? persistent_blocks((const void *)k, nb, 64 * W) : nb), b(64 * W);           \
        hipLaunchKernelGGL(k, g, b, 0, s, f, o, f.wq + 8 + (v));                                         \
    }
    BH_W64(0, f.has64 & (var_bit(false, false) | var_bit(false, true)), false, false);
    BH_W64(1, f.has64 & kVarQuadBits, true, false);
    BH_W64(2, f.has64 & kVarGroupBits, false, true);
#undef BH_W64
}

template <bool POT, bool PERSIST>
static void launch_w64_shape(const ForestDev &f, const WalkOut &o, int W, hipStream_t s) {
    switch (W) {
        case 1: launch_w64<false, POT, 1, PERSIST>(f, o, s); break;
        case 2: launch_w64<false, POT, 2, PERSIST>(f, o, s); break;
        case 8: launch_w64<false, POT, 8, PERSIST>(f, o, s); break;
        default: launch_w64<false, POT, 4, PERSIST>(f, o, s); break;
    }
}

void launch_walk64_family(const ForestDev &f, const WalkOut &o, bool stats, bool pot, int shape, hipStream_t s) {
    if (!f.has64) return;
    const int W = shape & kWalkWavesMask;
    const bool persist = (shape & kWalkPersistent) != 0;
    if (stats) {   // the counting walks use one launch shape
        if (pot) launch_w64<true, true, 4, false>(f, o, s);
        else launch_w64<true, false, 4, false>(f, o, s);
    } else if (persist) {
        if (pot) launch_w64_shape<true, true>(f, o, W, s);
        else launch_w64_shape<false, true>(f, o, W, s);
    } else if (pot) {
        launch_w64_shape<true, false>(f, o, W, s);
    } else {
        launch_w64_shape<false, false>(f, o, W, s);
    }
}

}  // namespace bh
