// Force walk on gfx950 (paper section 3: a remote cube is treated as one body
// only if its distance D from the body exceeds r/theta; the force stage is the
// computationally dominant part).
//
// One wavefront walks the tree for a group of 64 key-consecutive bodies, one
// body per lane.  The stack lives in LDS and holds (first child slot, number of
// children, lane mask) entries: a lane takes part in a node only if it opened
// every ancestor, so each lane meets exactly the cubes of its own per-body
// walk and its interaction set is the per-body set of the method.  Node
// records are read with wave-uniform (scalar) loads.  Monopoles and leaf pairs
// use a softened kernel on the VALU; no matrix cores (not a contraction).
//
// FP64 mode: the opening test s^2 < theta^2 D^2 and all arithmetic in FP64.
// FP32 mode: coordinates relative to the simulation's bbox centre in FP32;
// the test is evaluated in FP32 and, when |theta^2 D^2 - s^2| lies within its
// rounding bound, re-evaluated exactly in FP64 from the FP64 centre of mass
// and position; pair terms in FP32 summed into per-lane partial sums that are
// folded into Kahan-compensated totals after at most 64 terms.
#include "bh_common.h"

namespace bh {

constexpr float kU32 = 5.9604644775390625e-8f;   // 2^-24
constexpr uint32_t kFlushWork = 64;              // pair terms (upper bound) between Kahan folds

__device__ __forceinline__ uint32_t uni(uint32_t v) { return __builtin_amdgcn_readfirstlane(v); }

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

// Newton-refined FP64 reciprocal square root: y <- y + y (1 - x y^2) / 2, twice.
__device__ __forceinline__ double rsqrt64(double x) {
    double y = __builtin_amdgcn_rsq(x);
#pragma unroll
    for (int it = 0; it < 2; ++it) {
        double e = fma(-x * y, y, 1.0);
        y = fma(0.5 * y, e, y);
    }
    return y;
}

__device__ __forceinline__ double wave_sum_d(double v) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}
__device__ __forceinline__ unsigned long long wave_sum_u(unsigned long long v) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

struct WalkOut {
    double *acc, *pot;
    int64_t *n_mono, *n_p2p;
    uint64_t *hash;
};

// ------------------------------------------------------------- FP32 walk ---
// Each wavefront re-expresses coordinates relative to its own FP64 reference
// point g (its first body), so FP32 differences carry errors of order
// u |d| + u |x - g| rather than u |x - origin|.  The children of a popped stack
// entry are loaded and converted lane-parallel (lane c takes child c: FP64
// centre minus g, rounded to FP32, plus the per-child rounding band of the
// opening test) and staged in LDS, from which every lane reads them by
// broadcast.  Leaf particles are staged the same way, 64 at a time.
//
// Opening test in FP32: T = theta^2 D2 - s^2 (one fma).  With
// rho = |com - g|_inf + |x - g|_inf (upper bounds) and u = 2^-24,
//   |T - (theta^2 |com - x|^2 - s^2)| <= 16 u s^2 + rho (8 u s theta + 4 u^2 theta^2 rho)
// (a factor two above the first-order bound), so outside that band the FP32
// sign is the sign of the exact test; inside it the test is repeated in FP64
// exactly as the oracle evaluates it.

struct Stage {
    float x, y, z, m;     // centre relative to g (FP32), mass
    float S, band;        // side^2, rounding band for this wavefront
    uint32_t link, cnt;
    uint32_t gid, level, pad0, pad1;
};

template <bool STATS, bool POT>
__global__ void __launch_bounds__(kWalkThreads) k_walk32(ForestDev f, WalkOut out) {
    constexpr int W = kWalkThreads / 64;
    __shared__ uint4 stk[W][kStackMax];
    __shared__ Stage stage[W][8];
    __shared__ float4 pst[W][64];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const uint32_t gi = blockIdx.x * W + wave;
    if (gi >= f.ngroups) return;
    if (uni(*f.err) & kErrTree) return;   // tree inconsistent: never walk it
    const GroupDesc gd = f.groups[gi];
    const uint32_t sid = uni(gd.seg);
    const SegDesc &sd = f.seg[sid];
    if (sd.precision != 1) return;
    const SegState &st = f.st[sid];
    const bool live = (uint32_t)lane < gd.count;
    const uint32_t r = gd.start + (live ? (uint32_t)lane : 0u);
    const uint32_t r0 = uni(gd.start);
    const double gx = f.spos[3 * (size_t)r0], gy = f.spos[3 * (size_t)r0 + 1], gz = f.spos[3 * (size_t)r0 + 2];
    const float tx = (float)__dsub_rn(f.spos[3 * (size_t)r], gx);
    const float ty = (float)__dsub_rn(f.spos[3 * (size_t)r + 1], gy);
    const float tz = (float)__dsub_rn(f.spos[3 * (size_t)r + 2], gz);
    float rw = live ? fmaxf(fabsf(tx), fmaxf(fabsf(ty), fabsf(tz))) : 0.0f;
    for (int o = 32; o > 0; o >>= 1) rw = fmaxf(rw, __shfl_xor(rw, o, 64));
    rw = __uint_as_float(uni(__float_as_uint(rw))) * (1.0f + 4.0f * kU32);
    const double theta = sd.theta;
    const float theta2 = (float)(theta * theta);
    const float band2 = (float)(4.0 * 3.552713678800501e-15 * theta * theta);   // 4 u^2 theta^2
    const float eps2 = (float)(sd.eps * sd.eps);

    float ax = 0.f, ay = 0.f, az = 0.f, ap = 0.f;            // partial sums
    float sx = 0.f, sy = 0.f, sz = 0.f, sp_ = 0.f;           // Kahan sums
    float cx = 0.f, cy = 0.f, cz = 0.f, cp = 0.f;            // Kahan compensations
    uint32_t nmono = 0, np2p = 0, nvis = 0, nfb = 0;
    uint64_t h = 0;

    uint64_t m0 = __ballot(live);
    int sp = 0;
    if (lane == 0) stk[wave][0] = make_uint4(sid, 1u, (uint32_t)m0, (uint32_t)(m0 >> 32));
    wave_sync();
    sp = 1;
    uint32_t work = 0;   // terms added to the partial sums since the last fold (wave-uniform)
    auto fold = [&]() {
        kahan_add(sx, cx, ax); ax = 0.f;
        kahan_add(sy, cy, ay); ay = 0.f;
        kahan_add(sz, cz, az); az = 0.f;
        if (POT) { kahan_add(sp_, cp, ap); ap = 0.f; }
        work = 0;
    };
    while (sp > 0) {
        --sp;
        const uint4 e = stk[wave][sp];
        const uint32_t link = uni(e.x), nch = uni(e.y);
        const uint64_t emask = ((uint64_t)uni(e.w) << 32) | uni(e.z);
        const bool act = (emask >> lane) & 1ull;
        wave_sync();
        if ((uint32_t)lane < nch) {
            const WRec32 &w = f.w32[link + lane];
            Stage q;
            q.x = (float)__dsub_rn(w.cx, gx);
            q.y = (float)__dsub_rn(w.cy, gy);
            q.z = (float)__dsub_rn(w.cz, gz);
            q.m = w.m;
            q.S = w.S;
            const float rho = fmaxf(fabsf(q.x), fmaxf(fabsf(q.y), fabsf(q.z))) * (1.0f + 4.0f * kU32) + rw;
            q.band = fmaf(rho, fmaf(band2, rho, w.band1), w.band0);
            q.link = w.link;
            q.cnt = w.cnt;
            q.gid = w.gid;
            q.level = w.level;
            q.pad0 = q.pad1 = 0;
            stage[wave][lane] = q;
        }
        wave_sync();
        if (work + nch > kFlushWork) fold();
        work += nch;
        for (uint32_t c = 0; c < nch; ++c) {
            const Stage q = stage[wave][c];
            const float dx = q.x - tx, dy = q.y - ty, dz = q.z - tz;
            const float D2 = fmaf(dz, dz, fmaf(dy, dy, dx * dx));
            const float T = fmaf(theta2, D2, -q.S);
            bool acc = T > 0.0f;
            if (act && !(fabsf(T) > q.band)) {
                // within the FP32 rounding bound of the threshold: decide exactly in FP64
                const double *cm = f.nS + 3 * (size_t)uni(q.gid);
                const double *xp = f.spos + 3 * (size_t)r;
                double ex = __dsub_rn(cm[0], xp[0]), ey = __dsub_rn(cm[1], xp[1]), ez = __dsub_rn(cm[2], xp[2]);
                double ED2 = __dadd_rn(__dadd_rn(__dmul_rn(ex, ex), __dmul_rn(ey, ey)), __dmul_rn(ez, ez));
                double s = ldexp(st.L, -(int)uni(q.level));
                acc = __dmul_rn(s, s) < __dmul_rn(__dmul_rn(theta, theta), ED2);
                if (STATS) ++nfb;
            }
            acc = acc && act;
            if (STATS && act) ++nvis;
            if (acc) {
                const float r2 = D2 + eps2;
                const float ri = __builtin_amdgcn_rsqf(r2);
                const float mr = q.m * ri;
                const float w3 = mr * ri * ri;
                ax = fmaf(w3, dx, ax);
                ay = fmaf(w3, dy, ay);
                az = fmaf(w3, dz, az);
                if (POT) ap -= mr;
                if (STATS) {
                    ++nmono;
                    h += mix64((uint64_t)(q.gid - st.nbase));
                }
            }
            const uint64_t open = __ballot(act && !acc);
            if (open) {
                const uint32_t qcnt = uni(q.cnt), qlink = uni(q.link);
                if (qcnt & kLeafBit) {
                    const uint32_t np = qcnt & ~kLeafBit;
                    const bool me = (open >> lane) & 1ull;
                    for (uint32_t b0 = 0; b0 < np; b0 += 64) {
                        const uint32_t nb = np - b0 < 64u ? np - b0 : 64u;
                        wave_sync();
                        if ((uint32_t)lane < nb) {
                            const size_t j = (size_t)qlink + b0 + lane;
                            pst[wave][lane] = make_float4((float)__dsub_rn(f.spos[3 * j], gx),
                                                          (float)__dsub_rn(f.spos[3 * j + 1], gy),
                                                          (float)__dsub_rn(f.spos[3 * j + 2], gz), (float)f.smass[j]);
                        }
                        wave_sync();
                        if (work + nb > kFlushWork) fold();
                        work += nb;
                        for (uint32_t k = 0; k < nb; ++k) {
                            const float4 p = pst[wave][k];
                            const uint32_t jq = qlink + b0 + k;
                            if (me && jq != r) {
                                const float px = p.x - tx, py = p.y - ty, pz = p.z - tz;
                                const float r2 = fmaf(pz, pz, fmaf(py, py, fmaf(px, px, eps2)));
                                if (r2 > 0.0f) {
                                    const float ri = __builtin_amdgcn_rsqf(r2);
                                    const float mr = p.w * ri;
                                    const float w3 = mr * ri * ri;
                                    ax = fmaf(w3, px, ax);
                                    ay = fmaf(w3, py, ay);
                                    az = fmaf(w3, pz, az);
                                    if (POT) ap -= mr;
                                }
                                if (STATS) {
                                    ++np2p;
                                    h += mix64((uint64_t)st.nn + (uint64_t)(f.idx[jq] - sd.start));
                                }
                            }
                        }
                    }
                } else {
                    if (sp >= kStackMax) {
                        if (lane == 0) atomicOr(f.err, kErrStack);
                        sp = 0;
                        break;
                    }
                    if (lane == 0) stk[wave][sp] = make_uint4(qlink, qcnt, (uint32_t)open, (uint32_t)(open >> 32));
                    wave_sync();
                    ++sp;
                }
            }
        }
    }
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
        if (STATS) {
            if (out.n_mono) out.n_mono[i] = nmono;
            if (out.n_p2p) out.n_p2p[i] = np2p;
            if (out.hash) out.hash[i] = h;
        }
    }
    if (STATS) {
        unsigned long long a = wave_sum_u(live ? nmono : 0), b = wave_sum_u(live ? np2p : 0);
        unsigned long long v = wave_sum_u(live ? nvis : 0), fb = wave_sum_u(live ? nfb : 0);
        if (lane == 0) {
            atomicAdd(&f.stats[0], a);
            atomicAdd(&f.stats[1], b);
            atomicAdd(&f.stats[2], v);
            atomicAdd(&f.stats[3], fb);
        }
    }
}

// ------------------------------------------------------------- FP64 walk ---

template <bool STATS, bool POT>
__global__ void __launch_bounds__(kWalkThreads) k_walk64(ForestDev f, WalkOut out) {
    __shared__ uint4 stk[kWalkThreads / 64][kStackMax];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const uint32_t gi = blockIdx.x * (kWalkThreads / 64) + wave;
    if (gi >= f.ngroups) return;
    if (uni(*f.err) & kErrTree) return;   // tree inconsistent: never walk it
    const GroupDesc gd = f.groups[gi];
    const uint32_t sid = uni(gd.seg);
    const SegDesc &sd = f.seg[sid];
    if (sd.precision != 0) return;
    const SegState &st = f.st[sid];
    const bool live = (uint32_t)lane < gd.count;
    const uint32_t r = gd.start + (live ? (uint32_t)lane : 0u);
    const double tx = f.spos[3 * (size_t)r], ty = f.spos[3 * (size_t)r + 1], tz = f.spos[3 * (size_t)r + 2];
    const double theta2 = __dmul_rn(sd.theta, sd.theta);
    const double eps2 = __dmul_rn(sd.eps, sd.eps);

    double ax = 0.0, ay = 0.0, az = 0.0, ap = 0.0;
    uint32_t nmono = 0, np2p = 0, nvis = 0;
    uint64_t h = 0;

    uint64_t m0 = __ballot(live);
    int sp = 0;
    if (lane == 0) stk[wave][0] = make_uint4(sid, 1u, (uint32_t)m0, (uint32_t)(m0 >> 32));
    wave_sync();
    sp = 1;
    while (sp > 0) {
        --sp;
        const uint4 e = stk[wave][sp];
        const uint32_t link = uni(e.x), nch = uni(e.y);
        const uint64_t emask = ((uint64_t)uni(e.w) << 32) | uni(e.z);
        const bool act = (emask >> lane) & 1ull;
        for (uint32_t c = 0; c < nch; ++c) {
            const WRec64 w = f.w64[link + c];
            const double dx = __dsub_rn(w.x, tx), dy = __dsub_rn(w.y, ty), dz = __dsub_rn(w.z, tz);
            const double D2 = __dadd_rn(__dadd_rn(__dmul_rn(dx, dx), __dmul_rn(dy, dy)), __dmul_rn(dz, dz));
            const bool acc = act && (w.S < __dmul_rn(theta2, D2));
            if (STATS && act) ++nvis;
            if (acc) {
                const double ri = rsqrt64(D2 + eps2);
                const double mr = w.m * ri;
                const double w3 = mr * ri * ri;
                ax = fma(w3, dx, ax);
                ay = fma(w3, dy, ay);
                az = fma(w3, dz, az);
                if (POT) ap -= mr;
                if (STATS) {
                    ++nmono;
                    h += mix64((uint64_t)(w.gid - st.nbase));
                }
            }
            const uint64_t open = __ballot(act && !acc);
            if (open) {
                if (w.cnt & kLeafBit) {
                    const uint32_t np = w.cnt & ~kLeafBit;
                    const bool me = (open >> lane) & 1ull;
                    for (uint32_t q = w.link; q < w.link + np; ++q) {
                        const double qx = f.spos[3 * (size_t)q], qy = f.spos[3 * (size_t)q + 1],
                                     qz = f.spos[3 * (size_t)q + 2], qm = f.smass[q];
                        if (me && q != r) {
                            const double px = qx - tx, py = qy - ty, pz = qz - tz;
                            const double r2 = fma(pz, pz, fma(py, py, fma(px, px, eps2)));
                            if (r2 > 0.0) {
                                const double ri = rsqrt64(r2);
                                const double mr = qm * ri;
                                const double w3 = mr * ri * ri;
                                ax = fma(w3, px, ax);
                                ay = fma(w3, py, ay);
                                az = fma(w3, pz, az);
                                if (POT) ap -= mr;
                            }
                            if (STATS) {
                                ++np2p;
                                h += mix64((uint64_t)st.nn + (uint64_t)(f.idx[q] - sd.start));
                            }
                        }
                    }
                } else {
                    if (sp >= kStackMax) {
                        if (lane == 0) atomicOr(f.err, kErrStack);
                        sp = 0;
                        break;
                    }
                    if (lane == 0) stk[wave][sp] = make_uint4(w.link, w.cnt, (uint32_t)open, (uint32_t)(open >> 32));
                    wave_sync();
                    ++sp;
                }
            }
        }
    }
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
        if (STATS) {
            if (out.n_mono) out.n_mono[i] = nmono;
            if (out.n_p2p) out.n_p2p[i] = np2p;
            if (out.hash) out.hash[i] = h;
        }
    }
    if (STATS) {
        unsigned long long a = wave_sum_u(live ? nmono : 0), b = wave_sum_u(live ? np2p : 0);
        unsigned long long v = wave_sum_u(live ? nvis : 0);
        if (lane == 0) {
            atomicAdd(&f.stats[0], a);
            atomicAdd(&f.stats[1], b);
            atomicAdd(&f.stats[2], v);
        }
    }
}

hipError_t launch_walk(const ForestDev &f, bool stats, bool want_pot, double *acc, double *pot, int64_t *n_mono,
                       int64_t *n_p2p, uint64_t *hash, hipStream_t s) {
    WalkOut o{acc, pot, n_mono, n_p2p, hash};
    const unsigned blocks = (f.ngroups + (kWalkThreads / 64) - 1) / (kWalkThreads / 64);
    if (blocks == 0) return hipSuccess;
    const dim3 g(blocks), b(kWalkThreads);
    if (f.has32) {
        if (stats) {
            if (want_pot) hipLaunchKernelGGL((k_walk32<true, true>), g, b, 0, s, f, o);
            else hipLaunchKernelGGL((k_walk32<true, false>), g, b, 0, s, f, o);
        } else {
            if (want_pot) hipLaunchKernelGGL((k_walk32<false, true>), g, b, 0, s, f, o);
            else hipLaunchKernelGGL((k_walk32<false, false>), g, b, 0, s, f, o);
        }
    }
    if (f.has64) {
        if (stats) {
            if (want_pot) hipLaunchKernelGGL((k_walk64<true, true>), g, b, 0, s, f, o);
            else hipLaunchKernelGGL((k_walk64<true, false>), g, b, 0, s, f, o);
        } else {
            if (want_pot) hipLaunchKernelGGL((k_walk64<false, true>), g, b, 0, s, f, o);
            else hipLaunchKernelGGL((k_walk64<false, false>), g, b, 0, s, f, o);
        }
    }
    return hipGetLastError();
}

}  // namespace bh
