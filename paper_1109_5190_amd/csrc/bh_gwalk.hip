// Group-criterion force walks (FP32 and FP64).
#include "bh_walk_common.h"

namespace bh {

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
    if (uni(f.err[kErrWordTree]) & kErrTree) return;
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
        if (accb) {   // null: a counting walk for the checksums only
            accb[3 * li] = G * ((double)sx - (double)cx);
            accb[3 * li + 1] = G * ((double)sy - (double)cy);
            accb[3 * li + 2] = G * ((double)sz - (double)cz);
        }
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
    if (uni(f.err[kErrWordTree]) & kErrTree) return;
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
        if (accb) {   // null: a counting walk for the checksums only
            accb[3 * li] = G * ax;
            accb[3 * li + 1] = G * ay;
            accb[3 * li + 2] = G * az;
        }
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


template <bool STATS, bool POT>
static void launch_g(const ForestDev &f, const WalkOut &o, hipStream_t s) {
    const dim3 g4((f.ngroups + 3) / 4), b4(256);
    if (f.has32 & kVarGroup) hipLaunchKernelGGL((k_gwalk32<STATS, POT>), g4, b4, 0, s, f, o);
    if (f.has64 & kVarGroup) hipLaunchKernelGGL((k_gwalk64<STATS, POT>), g4, b4, 0, s, f, o);
}

void launch_gwalk_family(const ForestDev &f, const WalkOut &o, bool stats, bool pot, hipStream_t s) {
    if (!((f.has32 | f.has64) & kVarGroup)) return;
    if (stats) {
        if (pot) launch_g<true, true>(f, o, s);
        else launch_g<true, false>(f, o, s);
    } else {
        if (pot) launch_g<false, true>(f, o, s);
        else launch_g<false, false>(f, o, s);
    }
}

}  // namespace bh
