// Two-phase force stage: interaction lists written, then evaluated.
#include "bh_walk_common.h"

namespace bh {

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
    if (uni(f.err[kErrWordTree]) & kErrTree) return;
    const GroupDesc gd = f.groups[gi];
    const uint32_t sid = uni(gd.seg);
    const SegDesc &sd = f.seg[sid];
    if (sd.precision != 1 || sd.group) return;   // refused by the host
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
        stage_children32<true, false, false>(f, L, lane, link, nch, gx, gy, gz, rw);
        wave_sync();
        emit(kListEntry, nch, 0);
#pragma unroll
        for (uint32_t c = 0; c < 8; ++c) {
            if (c >= nch) break;
            const float4 qa = L.sa[c];
            const float dx = qa.x - tx, dy = qa.y - ty, dz = qa.z - tz;
            const float E2 = fmaf(dz, dz, fmaf(dy, dy, fmaf(dx, dx, eps2)));
            uint64_t accm = ballot(E2 > L.sbh[c]) & emask;
            uint64_t open = emask & ~accm;
            if (open) {
                const uint64_t ambm = ballot(!(E2 < L.sbl[c])) & open;
                if (ambm) {
                    bool ex = false;
                    if (in_mask(ambm)) ex = exact_accept32(f, link + c, r, theta);
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
    if (uni(f.err[kErrWordTree]) & kErrTree) return;
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
    // the walk's force sums and leaf pairs (after each stack entry, the queued particles,
    // then the leaves that did not fit the queue)
    Sums32<false, POT, SOFT> sums{f, L, lane, r, gstart, gx, gy, gz, tx, ty, tz, eps2, 0ull, 0u};

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
                if (sums.qn > 56u || sums.nov) sums.flush();   // the previous entry's pairs
                if (sums.work + b > kFlushWork) sums.fold();
                sums.work += b;
            } else if (b & kListLeaf) {
                wave_sync();
                sums.queue_leaf(a, b & ~kListLeaf, m);
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
                    sums.ax += qx;
                    sums.ay += qy;
                    sums.az += qz;
                    if (POT) sums.ap += qp;
                }
                sums.ax = fmaf(w3, dx, sums.ax);
                sums.ay = fmaf(w3, dy, sums.ay);
                sums.az = fmaf(w3, dz, sums.az);
                if (POT) sums.ap -= mr;
            }
        }
        chunk = uni(ld.next[chunk]);
    }
    sums.flush();
    sums.fold();
    if (live) {
        const uint32_t i = f.idx[r];
        const size_t li = i - sd.start;
        const double G = sd.G;
        double *accb = seg_base(out.acc, sd.acc, sd, 3);
        accb[3 * li] = G * ((double)sums.sx - (double)sums.cx);
        accb[3 * li + 1] = G * ((double)sums.sy - (double)sums.cy);
        accb[3 * li + 2] = G * ((double)sums.sz - (double)sums.cz);
        if (POT) {
            double *potb = seg_base(out.pot, sd.pot, sd, 1);
            if (potb) potb[li] = G * ((double)sums.sp - (double)sums.cp);
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
    if (uni(f.err[kErrWordTree]) & kErrTree) return;
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
        stage_children64<false>(f, L, lane, link, nch);
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
    if (uni(f.err[kErrWordTree]) & kErrTree) return;
    const GroupDesc gd = f.groups[gi];
    const uint32_t sid = uni(gd.seg);
    const SegDesc &sd = f.seg[sid];
    if (sd.precision != 0 || sd.group || (sd.quad != 0) != QUAD) return;
    const uint32_t gstart = uni(gd.start);
    const bool live = (uint32_t)lane < gd.count;
    const uint32_t r = gstart + (live ? (uint32_t)lane : 0u);
    const double tx = f.spos[3 * (size_t)r], ty = f.spos[3 * (size_t)r + 1], tz = f.spos[3 * (size_t)r + 2];
    const double eps2 = __dmul_rn(sd.eps, sd.eps);
    Sums64<false, POT, WaveLds64<false>> sums{f, L, lane, gstart, tx, ty, tz, eps2, 0ull, 0u};

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
                sums.queue_leaf(a, b & ~kListLeaf, m);
            } else if (in_mask(m)) {
                const double4 qa = mst[k];
                const double dx = __dsub_rn(qa.x, tx), dy = __dsub_rn(qa.y, ty), dz = __dsub_rn(qa.z, tz);
                const double D2 = __dadd_rn(__dadd_rn(__dmul_rn(dx, dx), __dmul_rn(dy, dy)), __dmul_rn(dz, dz));
                const double E2 = D2 + eps2;
                double w3, mr = 0.0;
                if (!QUAD) mono64<POT>(E2, qa.w, w3, mr);
                if (QUAD) {
                    const double ri = rsqrt64(E2);
                    const double ri2 = ri * ri;
                    mr = qa.w * ri;
                    w3 = mr * ri2;
                    // the walk's quadrupole term, from the moments of walk slot a
                    const double *q = f.q64 + 6 * (size_t)a;
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
            }
        }
        chunk = uni(ld.next[chunk]);
    }
    sums.flush_leaves();
    if (live) {
        const uint32_t i = f.idx[r];
        const size_t li = i - sd.start;
        const double G = sd.G;
        double *accb = seg_base(out.acc, sd.acc, sd, 3);
        accb[3 * li] = G * sums.ax;
        accb[3 * li + 1] = G * sums.ay;
        accb[3 * li + 2] = G * sums.az;
        if (POT) {
            double *potb = seg_base(out.pot, sd.pot, sd, 1);
            if (potb) potb[li] = G * sums.ap;
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



}  // namespace bh
