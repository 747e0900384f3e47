// Shared definitions of the MI355X Barnes-Hut library: device data layouts,
// small device helpers and the host-side launcher prototypes.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace bh {

constexpr int kMaxLevel = 21;          // 63-bit Morton keys: 21 octant digits
constexpr int kTile = 4096;            // particles per sort / bbox tile
constexpr int kGroup = 64;             // walk targets per wavefront
constexpr int kWalkWaves[4] = {1, 2, 4, 8};   // walk launch shapes: wavefronts per block
constexpr int kWalkWavesMask = 0xff;          // launch shape: wavefronts per block in the low byte,
constexpr int kWalkPersistent = 0x100;        //   this bit for the persistent form (work queue)
constexpr int kWalkQueues = 16;               // persistent walks: one group counter per walk variant
constexpr int kStackMax = 160;         // >= 1 + 7 * 21 entries of (child block, lane mask)
constexpr uint32_t kLeafBit = 0x80000000u;
constexpr uint32_t kNone = 0xffffffffu;

// Device error words (ForestDev::err).  Word 0 gathers the fault bits until a
// synchronising call reports and clears them; word 1 holds kErrTree for the
// current tree only (cleared by every build): the walks skip an inconsistent tree.
constexpr uint32_t kErrStack = 1u;
constexpr uint32_t kErrNonFinite = 2u;  // non-finite position or mass, or a failed generator draw
constexpr uint32_t kErrTree = 4u;       // inconsistent tree
constexpr int kErrWordTree = 1;

// Per simulation, fixed while its membership in a forest lasts (host written).
struct SegDesc {
    uint32_t start, n;          // rows [start, start + n) of the forest's sorted/concatenated index space
    uint32_t tile_base, ntiles; // sort tiles of this simulation
    uint32_t group_base, ngroups;
    int32_t leaf_cap, precision;
    double theta, eps, G;
    double dt;
    // this simulation's state, indexed 0..n-1 (used when a launch is given no concatenated arrays)
    const double *pos, *mass;
    double *vel, *acc, *pot;
    uint32_t phase;             // kPhase* bits: which parts of a step apply this iteration
    uint32_t quad;              // 1: accepted cubes add their quadrupole term
    uint32_t group;             // 1: group criterion (a cube is accepted for all bodies of a group cube)
    uint32_t open;              // kOpen*: opening radius r of the test r^2 < theta^2 D^2
};

constexpr uint32_t kOpenSide = 0u, kOpenBmax = 1u, kOpenOffset = 2u;

constexpr uint32_t kPhaseDrift = 1u, kPhaseKick2 = 2u, kPhaseKick1 = 4u;

// Per simulation, written on the device by every build.
struct SegState {
    unsigned long long mn[3], mx[3];   // order-preserving integer images of the bbox
    double lo[3];                      // root cube minimum corner
    double cref[3];                    // FP32 coordinate origin (bbox centre)
    double L;                          // root cube side 2^k
    int32_t k;
    uint32_t nbase;                    // global id of the root node
    uint32_t nn;                       // nodes of this simulation
    uint32_t pad[3];
};

struct TileDesc { uint32_t start, count, seg, pad; };
struct GroupDesc { uint32_t start, count, seg, pad; };

// Walk record of a node, FP32 mode (indexed by walk slot: children of a node are contiguous).
// The centre of mass stays FP64 so that every wavefront can re-express it relative to its
// own reference point before rounding to FP32.
struct WRec32 {
    double cx, cy, cz;         // centre of mass (FP64)
    float m;                   // mass (FP32)
    float Sh;                  // S (1 + 8u) of S = r^2 / theta^2 + eps^2, rounded (FP32; +inf when theta = 0)
    float band0;               // 16 u S (inf: S outside FP32 range, always decide in FP64)
    float band1;               // 8 u r / theta
    uint32_t link;             // internal: first child slot; leaf: first particle rank
    uint32_t cnt;              // internal: children; leaf: particles | kLeafBit
    uint32_t gid;              // global node id (depth-first preorder)
    uint32_t level;
    double r2;                 // r^2 of the exact FP64 test r^2 < theta^2 D^2 (side^2 by default)
};

// Walk record of a node, FP64 mode.
struct WRec64 {
    double x, y, z, m;
    double S;                  // r^2 of the test r^2 < theta^2 D^2 (side^2 by default)
    uint32_t link, cnt, gid, level;
    double pad;
};
static_assert(sizeof(WRec32) == 64 && sizeof(WRec64) == 64, "walk records are one 64-byte line");

// Device-side views of one forest's buffers (all sub-allocated from the caller's workspace).
struct ForestDev {
    uint32_t nseg, ntot, ntiles, ngroups, mcap;   // current membership (mcap = 2 ntot)
    uint32_t has32, has64;                        // per precision: walk variants present, var_bit()
    SegDesc *seg;
    SegState *st;
    TileDesc *tiles;
    GroupDesc *groups;
    uint32_t *segid;            // per particle row
    uint64_t *keys, *keys_alt;  // sort ping-pong
    uint32_t *idx, *idx_alt;    // idx ends as perm: sorted rank -> original row
    uint32_t *cnt;              // sort digit counts, 256 per tile (tile-major)
    uint32_t *segtot, *segp;    // sort: per simulation and digit, total and scan base
    uint32_t *scan_tmp;         // block sums of the scans
    double *spos, *smass;       // sorted state (FP64)
    double4 *pk;                // per row in the caller's order: (x, y, z, m), one aligned 32-byte
                                // record for the permute's gather
    int8_t *lcp;                // common-prefix level of neighbouring keys, -1 at segment edges
    uint32_t *mask;             // per row: bit l set if a node of level l starts at this row
    uint32_t *base;             // exclusive scan of popcount(mask): global node id base
    uint8_t *nlevel;            // per node
    uint32_t *nchild;           // per node (scan input: number of children)
    uint32_t *nfirst, *ncount, *nparent, *ncrank;
    uint32_t *cs;               // exclusive scan of nchild
    uint32_t *slot_of;          // walk slot of each node
    uint4 *lvl_list;            // per block of 256 node ids: its internal nodes sorted by level,
                                //   as (slot, first child slot, children, quadrupole flag)
    uint16_t *blk_lvl;          // per such block: start of each level in its list (23 entries)
    double *uM, *uS;            // upward pass: mass and mass-weighted position sums by walk slot
    double *uQ;                 // upward pass: second moments about the centre of mass by slot (6), quadrupole forests
    float4 *q32;                // FP32 walk: second moments by slot, (xx yy zz xy) (xz yz tr 0)
    double *q64;                // FP64 walk: second moments by slot (xx yy zz xy xz yz)
    uint8_t *rlam;              // per row that starts a leaf: the leaf's level
    unsigned long long *tile_mm; // per tile: integer images of the bbox min (3) and max (3)
    WRec32 *w32;
    WRec64 *w64;
    uint32_t *err;              // device error word
    unsigned long long *stats;  // 4 totals (n_mono, n_p2p, n_visits, n_fallback)
    double *red;                // reduction scratch (energy)
    double *pot;                // potential scratch (ntot)
    double *gbox;               // group criterion, per sorted row: its group's bounding box lo[3], hi[3]
    uint32_t *wq;               // persistent walks: next group index, per walk variant (kWalkQueues)
};

// ---------------------------------------------------------------- helpers ---

// An inconsistent tree: reported, and its walks skipped.
__device__ __forceinline__ void flag_tree(const ForestDev &f) {
    atomicOr(f.err, kErrTree);
    atomicOr(f.err + kErrWordTree, kErrTree);
}

// Walk variant of a simulation: expansion order, whether its FP32 softening is zero and
// whether it uses the group criterion (one bit each of ForestDev::has32 / has64; the
// FP64 walk ignores the softening bit; the quadrupole is not combined with groups).
constexpr uint32_t kVarQuad = 1u, kVarUnsoft = 2u, kVarGroup = 4u;
__host__ __device__ __forceinline__ uint32_t var_bit(bool quad, bool unsoft, bool group = false) {
    return 1u << ((quad ? kVarQuad : 0u) | (unsoft ? kVarUnsoft : 0u) | (group ? kVarGroup : 0u));
}
constexpr uint32_t kVarQuadBits = (1u << kVarQuad) | (1u << (kVarQuad | kVarUnsoft));
constexpr uint32_t kVarGroupBits = (1u << kVarGroup) | (1u << (kVarGroup | kVarUnsoft));
constexpr int kGroupCap = 64;   // group criterion: a group is a largest cube of at most this many bodies

// A simulation's FP32 walk is unsoftened when eps^2 rounds to zero in FP32.
__host__ __device__ __forceinline__ bool unsoftened(double eps) { return !((float)(eps * eps) > 0.0f); }

// Base of a simulation's rows: the concatenated array shifted to its first row,
// or the simulation's own array.
template <typename T>
__device__ __forceinline__ T *seg_base(T *cat, T *own, const SegDesc &sd, int width) {
    return cat ? cat + (size_t)width * sd.start : own;
}

__device__ __forceinline__ unsigned long long ord_enc(double v) {
    unsigned long long b = (unsigned long long)__double_as_longlong(v);
    return (b & 0x8000000000000000ull) ? ~b : (b | 0x8000000000000000ull);
}
__device__ __forceinline__ double ord_dec(unsigned long long e) {
    unsigned long long b = (e & 0x8000000000000000ull) ? (e & 0x7fffffffffffffffull) : ~e;
    return __longlong_as_double((long long)b);
}

// Inverse of spread3: bits 3b of v gathered to bit b.
__device__ __forceinline__ uint32_t compact3(uint64_t v) {
    v &= 0x1249249249249249ull;
    v = (v ^ (v >> 2)) & 0x10c30c30c30c30c3ull;
    v = (v ^ (v >> 4)) & 0x100f00f00f00f00full;
    v = (v ^ (v >> 8)) & 0x001f0000ff0000ffull;
    v = (v ^ (v >> 16)) & 0x001f00000000ffffull;
    v = (v ^ (v >> 32)) & 0x00000000001fffffull;
    return (uint32_t)v;
}

// Morton spread: bit b of v moves to bit 3b (v < 2^21).
__device__ __forceinline__ uint64_t spread3(uint64_t v) {
    v &= 0x1fffffull;
    v = (v | (v << 32)) & 0x1f00000000ffffull;
    v = (v | (v << 16)) & 0x1f0000ff0000ffull;
    v = (v | (v << 8)) & 0x100f00f00f00f00full;
    v = (v | (v << 4)) & 0x10c30c30c30c30c3ull;
    v = (v | (v << 2)) & 0x1249249249249249ull;
    return v;
}

// SplitMix64 finalizer of x + golden gamma (interaction-set checksum).
__device__ __forceinline__ uint64_t mix64(uint64_t x) {
    uint64_t z = x + 0x9e3779b97f4a7c15ull;
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
    return z ^ (z >> 31);
}

// Edge of row r's level-`level` cube within sorted keys [lo, hi): RIGHT gives one
// past its last row, otherwise its first row.  Rows of one cube are contiguous,
// so membership is monotone in the distance from r; the search probes up to 8
// rows per round (independent loads): first at power-of-two distances in
// growing batches, then at 8 evenly spaced points of the bracketing interval,
// so a cube of n rows costs a few dependent rounds (about 2 + log_9 n for big
// cubes) instead of 2 log_2 n dependent loads.
template <bool RIGHT>
struct CellProbe {
    const uint64_t *K;
    uint32_t r, avail;   // rows available beyond r in the search direction
    int sh;
    uint64_t P;
    __device__ __forceinline__ bool inside(uint32_t d) const {
        return d <= avail && (K[RIGHT ? r + d : r - d] >> sh) == P;
    }
    // One round of NE probes at distances 2^E0 .. 2^(E0+NE-1); true once the edge is bracketed.
    template <int E0, int NE>
    __device__ __forceinline__ bool round(uint32_t &good, uint32_t &bad) const {
        int nin = 0;
#pragma unroll
        for (int k = 0; k < NE; ++k) nin += inside(1u << (E0 + k)) ? 1 : 0;   // the inside probes form a prefix
        if (nin > 0) good = 1u << (E0 + nin - 1);
        if (nin < NE) {
            const uint32_t d = 1u << (E0 + nin);
            if (d < bad) bad = d;
            return true;
        }
        return false;
    }
};

template <bool RIGHT>
__device__ __noinline__ uint32_t cell_edge(const uint64_t *K, uint32_t r, int level, uint32_t lo, uint32_t hi) {
    if (level <= 0) return RIGHT ? hi : lo;
    const int sh = 3 * (kMaxLevel - level);
    const CellProbe<RIGHT> pb{K, r, RIGHT ? hi - 1 - r : r - lo, sh, K[r] >> sh};
    // distances from r: inside(good) holds (good = 0 is r itself), inside(bad) does not
    uint32_t good = 0, bad = pb.avail + 1;
    (void)(pb.template round<0, 2>(good, bad) || pb.template round<2, 4>(good, bad) ||
           pb.template round<6, 8>(good, bad) || pb.template round<14, 8>(good, bad) ||
           pb.template round<22, 8>(good, bad) || pb.template round<30, 1>(good, bad));
    while (bad - good > 1) {
        const uint32_t span = bad - good;
        int nin = 0;
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            const uint32_t o = span <= 9 ? (uint32_t)(k + 1) : (uint32_t)((uint64_t)span * (k + 1) / 9);
            nin += (o < span && pb.inside(good + o)) ? 1 : 0;
        }
        const uint32_t g0 = good;
        if (nin > 0) good = g0 + (span <= 9 ? (uint32_t)nin : (uint32_t)((uint64_t)span * nin / 9));
        if (nin < 8) {
            const uint32_t o = span <= 9 ? (uint32_t)(nin + 1) : (uint32_t)((uint64_t)span * (nin + 1) / 9);
            if (o < span) bad = g0 + o;
        }
    }
    return RIGHT ? r + bad : r - good;
}

// First row q in [lo, r] whose key shares r's level-`level` cube (keys sorted on [lo, hi)).
__device__ inline uint32_t cell_left(const uint64_t *K, uint32_t r, int level, uint32_t lo) {
    return cell_edge<false>(K, r, level, lo, 0u);
}

// One past the last row q in [r, hi) whose key shares r's level-`level` cube.
__device__ inline uint32_t cell_right(const uint64_t *K, uint32_t r, int level, uint32_t hi) {
    return cell_edge<true>(K, r, level, 0u, hi);
}

// ------------------------------------------------------ launcher prototypes ---
// All launchers enqueue on `s` and return hipGetLastError().

hipError_t launch_build(const ForestDev &f, const double *pos, const double *mass,
                        hipStream_t s);                          // bbox .. tree topology
hipError_t launch_upward(const ForestDev &f, hipStream_t s);     // masses, centres, walk records
// Walks the groups of f (a copy may point at a sub-range of them); outputs and
// totals only for the bodies of sorted ranks [wlo, whi).  Counting walks, each
// nullable: work, each body's share of its group's wavefront work; gwork, that
// work per walk group (indexed by the group's first rank / 64 in its simulation).
// shape: wavefronts per workgroup, with kWalkPersistent for the persistent form
// (counting walks always take the grid form with 4).
hipError_t launch_walk(const ForestDev &f, bool stats, bool want_pot, double *acc, double *pot, int64_t *n_mono,
                       int64_t *n_p2p, uint64_t *hash, hipStream_t s, int shape = 4, uint32_t wlo = 0,
                       uint32_t whi = 0xffffffffu, int64_t *work = nullptr, int64_t *gwork = nullptr);
// Workgroups of a persistent launch of `kernel` with `block` threads: as many as the
// current device holds at once, at most nb.
uint32_t persistent_blocks(const void *kernel, uint32_t nb, int block);
// Cost zones over n bodies: per body (gathered through the sort order from two
// caller-order arrays) when group_cost is null, else per 64-body walk group (group
// g costs its body count plus group_cost[g]; bounds on group boundaries).
hipError_t launch_shard_bounds(const ForestDev &f, uint32_t n, const int64_t *cost_a, const int64_t *cost_b,
                               const int64_t *group_cost, uint32_t G, int64_t *bounds, hipStream_t s);
// phase_mask 0: every simulation; else only those whose SegDesc.phase has a bit of the mask.
hipError_t launch_kick(const ForestDev &f, double *vel, const double *acc, uint32_t phase_mask, hipStream_t s);
hipError_t launch_drift(const ForestDev &f, double *pos, const double *vel, uint32_t phase_mask, hipStream_t s);
// Interaction lists of one forest (two-phase walk): entries (a, b, mask lo, mask hi) in
// chunks of 64, chained per walk group.
constexpr uint32_t kListParts = 256;   // chunk counters; group g takes chunks g mod 256 + 256 t
constexpr uint32_t kListReserve = 4;   // chunks a wave reserves per counter update
struct ListDev {
    uint4 *ent;
    uint32_t *head, *count, *next;   // per group: first chunk, entries; per chunk: next chunk
    unsigned long long *ctr;         // kListParts counters, 32 apart: chunks taken from each
                                     // (beyond nchunks: counted, not written)
    uint32_t nchunks;
};
hipError_t launch_lists_build(const ForestDev &f, const ListDev &ld, hipStream_t s);
hipError_t launch_lists_eval(const ForestDev &f, const ListDev &ld, bool want_pot, double *acc, double *pot,
                             hipStream_t s);
hipError_t launch_kick_kick_drift(const ForestDev &f, double *pos, double *vel, const double *acc, hipStream_t s);
hipError_t launch_energy(const ForestDev &f, const double *vel, const double *mass, const double *pot,
                         double *out2, hipStream_t s);
hipError_t launch_export(const ForestDev &f, uint32_t seg, uint64_t *keys, uint32_t *perm, int32_t *level,
                         uint32_t *first, uint32_t *count, int32_t *parent, double *M, double *com,
                         hipStream_t s);
// Initial conditions; part: ic_scratch_bytes() of partial sums; err: the word that
// receives kErrNonFinite when a velocity draw fails.
size_t ic_scratch_bytes();
hipError_t launch_ic(int kind, int64_t n, uint64_t seed, double a, double M, double *pos, double *vel,
                     double *mass, double *part, uint32_t *err, hipStream_t s);
hipError_t launch_fill_u32(uint32_t *p, uint32_t v, size_t n, hipStream_t s);
hipError_t launch_segid(const ForestDev &f, hipStream_t s);

}  // namespace bh
