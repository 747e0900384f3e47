// Time integration, energy diagnostics and device-side initial conditions.
//
// The paper iterates force evaluations on a tree rebuilt every iteration
// (section 1, load-balancing item; section 3, global barrier at tree
// construction) without naming an integrator; the library advances with
// kick-drift-kick leapfrog in FP64:
//   v += (dt/2) a ; x += dt v ; (rebuild, forces) ; v += (dt/2) a.
#include "bh_common.h"

namespace bh {

// ------------------------------------------------------------------ KDK ---

// kSub blocks per tile (a tile holds up to 4096 particles, 12288 FP64 words per
// array), so that a streaming launch keeps enough loads in flight; the tile's
// simulation decides (phase) whether this half-kick or drift applies to it in
// this iteration; phase_mask 0 applies it everywhere.
constexpr uint32_t kSub = 4;

__global__ void __launch_bounds__(256) k_kick(ForestDev f, double *vel, const double *acc, uint32_t phase_mask) {
    const TileDesc td = f.tiles[blockIdx.x / kSub];
    const SegDesc &sd = f.seg[td.seg];
    if (phase_mask && !(sd.phase & phase_mask)) return;
    double *vb = seg_base(vel, sd.vel, sd, 3);
    const double *ab = seg_base(acc, (const double *)sd.acc, sd, 3);
    const double h = __dmul_rn(0.5, sd.dt);
    const size_t j0 = 3 * (size_t)(td.start - sd.start);
    for (uint32_t j = (blockIdx.x % kSub) * 256 + threadIdx.x; j < 3 * td.count; j += 256 * kSub)
        vb[j0 + j] = __dadd_rn(vb[j0 + j], __dmul_rn(h, ab[j0 + j]));
}

__global__ void __launch_bounds__(256) k_drift(ForestDev f, double *pos, const double *vel, uint32_t phase_mask) {
    const TileDesc td = f.tiles[blockIdx.x / kSub];
    const SegDesc &sd = f.seg[td.seg];
    if (phase_mask && !(sd.phase & phase_mask)) return;
    double *pb = seg_base(pos, (double *)sd.pos, sd, 3);
    const double *vb = seg_base(vel, (const double *)sd.vel, sd, 3);
    const size_t j0 = 3 * (size_t)(td.start - sd.start);
    for (uint32_t j = (blockIdx.x % kSub) * 256 + threadIdx.x; j < 3 * td.count; j += 256 * kSub)
        pb[j0 + j] = __dadd_rn(pb[j0 + j], __dmul_rn(sd.dt, vb[j0 + j]));
}

// The closing half-kick of one step, the opening half-kick of the next and its
// drift in one pass over the state: the same three roundings, in the same
// order, as k_kick, k_kick, k_drift.
__global__ void __launch_bounds__(256) k_kick_kick_drift(ForestDev f, double *pos, double *vel, const double *acc) {
    const TileDesc td = f.tiles[blockIdx.x / kSub];
    const SegDesc &sd = f.seg[td.seg];
    double *pb = seg_base(pos, (double *)sd.pos, sd, 3);
    double *vb = seg_base(vel, sd.vel, sd, 3);
    const double *ab = seg_base(acc, (const double *)sd.acc, sd, 3);
    const double h = __dmul_rn(0.5, sd.dt);
    const size_t j0 = 3 * (size_t)(td.start - sd.start);
    for (uint32_t j = (blockIdx.x % kSub) * 256 + threadIdx.x; j < 3 * td.count; j += 256 * kSub) {
        const double ha = __dmul_rn(h, ab[j0 + j]);
        const double v = __dadd_rn(__dadd_rn(vb[j0 + j], ha), ha);
        vb[j0 + j] = v;
        pb[j0 + j] = __dadd_rn(pb[j0 + j], __dmul_rn(sd.dt, v));
    }
}

hipError_t launch_kick(const ForestDev &f, double *vel, const double *acc, uint32_t phase_mask, hipStream_t s) {
    if (f.ntiles) hipLaunchKernelGGL(k_kick, dim3(f.ntiles * kSub), dim3(256), 0, s, f, vel, acc, phase_mask);
    return hipGetLastError();
}

hipError_t launch_drift(const ForestDev &f, double *pos, const double *vel, uint32_t phase_mask, hipStream_t s) {
    if (f.ntiles) hipLaunchKernelGGL(k_drift, dim3(f.ntiles * kSub), dim3(256), 0, s, f, pos, vel, phase_mask);
    return hipGetLastError();
}

hipError_t launch_kick_kick_drift(const ForestDev &f, double *pos, double *vel, const double *acc, hipStream_t s) {
    if (f.ntiles) hipLaunchKernelGGL(k_kick_kick_drift, dim3(f.ntiles * kSub), dim3(256), 0, s, f, pos, vel, acc);
    return hipGetLastError();
}

// --------------------------------------------------------------- energy ---
// Per simulation: K = 1/2 sum m |v|^2, W = 1/2 sum m phi (one block per simulation,
// fixed reduction order so repeated runs agree bit for bit).

__global__ void __launch_bounds__(256) k_energy(ForestDev f, const double *vel, const double *mass, const double *pot,
                                                double *out) {
    __shared__ double sk[256], sw[256];
    const SegDesc &sd = f.seg[blockIdx.x];
    const double *vb = seg_base(vel, (const double *)sd.vel, sd, 3);
    const double *mb = seg_base(mass, sd.mass, sd, 1);
    const double *pb = seg_base(pot, (const double *)sd.pot, sd, 1);
    double K = 0.0, W = 0.0;
    for (uint32_t i = threadIdx.x; i < sd.n; i += 256) {
        const double *v = vb + 3 * (size_t)i;
        K += mb[i] * ((v[0] * v[0] + v[1] * v[1]) + v[2] * v[2]);
        if (pb) W += mb[i] * pb[i];
    }
    sk[threadIdx.x] = K;
    sw[threadIdx.x] = W;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) {
            sk[threadIdx.x] += sk[threadIdx.x + o];
            sw[threadIdx.x] += sw[threadIdx.x + o];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        out[2 * blockIdx.x] = 0.5 * sk[0];
        out[2 * blockIdx.x + 1] = 0.5 * sw[0];
    }
}

hipError_t launch_energy(const ForestDev &f, const double *vel, const double *mass, const double *pot, double *out2,
                         hipStream_t s) {
    hipLaunchKernelGGL(k_energy, dim3(f.nseg), dim3(256), 0, s, f, vel, mass, pot, out2);
    return hipGetLastError();
}

// ---------------------------------------------------- initial conditions ---
// Philox4x32-10 (Salmon et al. 2011); counter (i_lo, i_hi, call, tag), key from the seed.

struct P4 { uint32_t x, y, z, w; };

__device__ inline P4 philox(P4 c, uint32_t k0, uint32_t k1) {
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint64_t p0 = (uint64_t)0xD2511F53u * c.x;
        const uint64_t p1 = (uint64_t)0xCD9E8D57u * c.z;
        P4 n;
        n.x = (uint32_t)(p1 >> 32) ^ c.y ^ k0;
        n.y = (uint32_t)p1;
        n.z = (uint32_t)(p0 >> 32) ^ c.w ^ k1;
        n.w = (uint32_t)p0;
        c = n;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    return c;
}

__device__ __forceinline__ double u53(uint32_t a, uint32_t b) {
    return ((double)(a >> 5) * 67108864.0 + (double)(b >> 6) + 0.5) * 1.1102230246251565e-16;
}

constexpr uint32_t kPlummerTag = 1, kCubeTag = 2;
constexpr uint32_t kIcBlocks = 256;   // blocks of the generator: one partial-sum record (6 FP64) each
constexpr double kMassCut = 0.999;

__device__ inline void draw2(uint64_t i, uint32_t call, uint32_t tag, uint64_t seed, double &u0, double &u1) {
    P4 c{(uint32_t)i, (uint32_t)(i >> 32), call, tag};
    P4 o = philox(c, (uint32_t)seed, (uint32_t)(seed >> 32));
    u0 = u53(o.x, o.y);
    u1 = u53(o.z, o.w);
}

__global__ void k_ic(int kind, int64_t n, uint64_t seed, double a, double M, double *pos, double *vel,
                     double *mass, double *part, uint32_t *err) {
    __shared__ double red[6][256];
    double acc6[6] = {0, 0, 0, 0, 0, 0};
    const double m = M / (double)n;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
        double x[3], v[3], mi;
        if (kind == 0) {
            double x1, x2, x3, x6, x7, unused;
            draw2((uint64_t)i, 0, kPlummerTag, seed, x1, x2);
            draw2((uint64_t)i, 1, kPlummerTag, seed, x3, x6);
            draw2((uint64_t)i, 2, kPlummerTag, seed, x7, unused);
            const double frac = kMassCut * x1;
            const double r = 1.0 / sqrt(pow(frac, -2.0 / 3.0) - 1.0);
            const double z = (1.0 - 2.0 * x2) * r;
            const double rho = sqrt(fmax(r * r - z * z, 0.0));
            const double phi = 2.0 * M_PI * x3;
            x[0] = rho * cos(phi) * a;
            x[1] = rho * sin(phi) * a;
            x[2] = z * a;
            double q = 0.0;
            bool ok = false;
            for (uint32_t call = 3; call <= 403; ++call) {
                double x4, x5;
                draw2((uint64_t)i, call, kPlummerTag, seed, x4, x5);
                if (0.1 * x5 < x4 * x4 * pow(1.0 - x4 * x4, 3.5)) { q = x4; ok = true; break; }
            }
            if (!ok) {   // no acceptance: reported, and the velocities are left non-finite
                atomicOr(err, kErrNonFinite);
                q = NAN;
            }
            const double sp = q * sqrt(2.0 * M / a) * pow(1.0 + r * r, -0.25);
            const double vz = (1.0 - 2.0 * x6) * sp;
            const double vr = sqrt(fmax(sp * sp - vz * vz, 0.0));
            const double psi = 2.0 * M_PI * x7;
            v[0] = vr * cos(psi);
            v[1] = vr * sin(psi);
            v[2] = vz;
            mi = m;
        } else {
            double u0, u1, u2, u3;
            draw2((uint64_t)i, 0, kCubeTag, seed, u0, u1);
            draw2((uint64_t)i, 1, kCubeTag, seed, u2, u3);
            x[0] = (2.0 * u0 - 1.0) * a;
            x[1] = (2.0 * u1 - 1.0) * a;
            x[2] = (2.0 * u2 - 1.0) * a;
            v[0] = v[1] = v[2] = 0.0;
            mi = (0.5 + u3) * M / (double)n;
        }
        for (int d = 0; d < 3; ++d) {
            pos[3 * i + d] = x[d];
            vel[3 * i + d] = v[d];
            acc6[d] += mi * x[d];
            acc6[3 + d] += mi * v[d];
        }
        mass[i] = mi;
    }
    for (int d = 0; d < 6; ++d) red[d][threadIdx.x] = acc6[d];
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o)
            for (int d = 0; d < 6; ++d) red[d][threadIdx.x] += red[d][threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x < 6) part[6 * blockIdx.x + threadIdx.x] = red[threadIdx.x][0];
}

// Shift a Plummer sphere to its centre-of-mass frame (partial sums from k_ic).
__global__ void k_ic_shift(int64_t n, double M, double *pos, double *vel, const double *part, int nblk) {
    __shared__ double sh[6];
    if (threadIdx.x < 6) {
        double s = 0.0;
        for (int b = 0; b < nblk; ++b) s += part[6 * b + threadIdx.x];
        sh[threadIdx.x] = s / M;
    }
    __syncthreads();
    for (int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x; j < 3 * n; j += (int64_t)gridDim.x * 256) {
        const int d = (int)(j % 3);
        pos[j] -= sh[d];
        vel[j] -= sh[3 + d];
    }
}

size_t ic_scratch_bytes() { return sizeof(double) * 6 * kIcBlocks; }

hipError_t launch_ic(int kind, int64_t n, uint64_t seed, double a, double M, double *pos, double *vel,
                     double *mass, double *part, uint32_t *err, hipStream_t s) {
    hipLaunchKernelGGL(k_ic, dim3(kIcBlocks), dim3(256), 0, s, kind, n, seed, a, M, pos, vel, mass, part, err);
    if (kind == 0) hipLaunchKernelGGL(k_ic_shift, dim3(512), dim3(256), 0, s, n, M, pos, vel, part, (int)kIcBlocks);
    return hipGetLastError();
}

}  // namespace bh
