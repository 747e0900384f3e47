// C ABI of libbh.so: contexts, workspace planning, trees, simulations and
// forests.  Every entry point validates its arguments, enqueues kernels on the
// context's stream and returns a bh_status; no exception crosses the ABI.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include <unistd.h>

#include "bh.h"
#include "bh_common.h"
#include "bh_host.h"
#include "bh_internal.h"

using namespace bh;

static thread_local std::string g_err;

bh_status bh_fail(bh_status st, const std::string &msg) {
    g_err = msg;
    return st;
}

#define HIPCHK(x)                                                                              \
    do {                                                                                       \
        hipError_t e_ = (x);                                                                   \
        if (e_ != hipSuccess) return bh_fail(BH_E_DEVICE, std::string(#x) + ": " + hipGetErrorString(e_)); \
    } while (0)

// ------------------------------------------------------------- validation ---

bh_status bh_check_params(const bh_params *p) {
    if (!p) return bh_fail(BH_E_INVAL, "params is NULL");
    if (!std::isfinite(p->theta) || p->theta < 0.0) return bh_fail(BH_E_INVAL, "theta must be finite and >= 0");
    if (!std::isfinite(p->eps) || p->eps < 0.0) return bh_fail(BH_E_INVAL, "eps must be finite and >= 0");
    if (!std::isfinite(p->G)) return bh_fail(BH_E_INVAL, "G must be finite");
    if (p->leaf_cap < 1 || p->leaf_cap > 64) return bh_fail(BH_E_INVAL, "leaf_cap must be in [1, 64]");
    if (p->precision != BH_FP64 && p->precision != BH_FP32) return bh_fail(BH_E_INVAL, "precision must be BH_FP64 or BH_FP32");
    if (p->flags & ~(uint32_t)(BH_QUADRUPOLE | BH_GROUP_CRITERION | BH_OPEN_BMAX | BH_OPEN_OFFSET | BH_REQ_RELEASE))
        return bh_fail(BH_E_INVAL, "unknown bits in flags");
    if ((p->flags & BH_QUADRUPOLE) && (p->flags & BH_GROUP_CRITERION))
        return bh_fail(BH_E_INVAL, "BH_QUADRUPOLE and BH_GROUP_CRITERION are not combined");
    if ((p->flags & BH_OPEN_BMAX) && (p->flags & BH_OPEN_OFFSET))
        return bh_fail(BH_E_INVAL, "BH_OPEN_BMAX and BH_OPEN_OFFSET exclude each other");
    if ((p->flags & (BH_OPEN_BMAX | BH_OPEN_OFFSET)) && (p->flags & BH_GROUP_CRITERION))
        return bh_fail(BH_E_INVAL, "the group criterion is defined with the cube side only");
    return BH_OK;
}

// ------------------------------------------------------------- planning ---


// Host tables of a forest membership: segment descriptors (state pointers left
// null: the concatenated arrays are passed to each launch), sort tiles and walk groups.
void bh_forest_tables(ForestHost &F, int32_t nseg, const int64_t *n, const bh_params *p) {
    F.seg.assign(nseg, SegDesc{});
    F.tiles.clear();
    F.groups.clear();
    uint64_t ntot = 0;
    uint32_t has32 = 0, has64 = 0;
    for (int32_t s = 0; s < nseg; ++s) {
        SegDesc &d = F.seg[s];
        d.start = (uint32_t)ntot;
        d.n = (uint32_t)n[s];
        d.tile_base = (uint32_t)F.tiles.size();
        d.ntiles = (uint32_t)((n[s] + kTile - 1) / kTile);
        d.group_base = (uint32_t)F.groups.size();
        d.ngroups = (uint32_t)((n[s] + kGroup - 1) / kGroup);
        d.leaf_cap = p[s].leaf_cap;
        d.precision = p[s].precision;
        d.theta = p[s].theta;
        d.eps = p[s].eps;
        d.G = p[s].G;
        d.dt = 0.0;
        d.quad = (p[s].flags & BH_QUADRUPOLE) ? 1u : 0u;
        d.group = (p[s].flags & BH_GROUP_CRITERION) ? 1u : 0u;
        d.open = (p[s].flags & BH_OPEN_BMAX) ? kOpenBmax : (p[s].flags & BH_OPEN_OFFSET) ? kOpenOffset : kOpenSide;
        (p[s].precision == BH_FP32 ? has32 : has64) |= var_bit(d.quad != 0, unsoftened(d.eps), d.group != 0);
        for (uint32_t t = 0; t < d.ntiles; ++t) {
            uint32_t st = d.start + t * kTile;
            uint32_t c = (uint32_t)std::min<int64_t>(kTile, n[s] - (int64_t)t * kTile);
            F.tiles.push_back(TileDesc{st, c, (uint32_t)s, 0});
        }
        for (uint32_t g = 0; g < d.ngroups; ++g) {
            uint32_t st = d.start + g * kGroup;
            uint32_t c = (uint32_t)std::min<int64_t>(kGroup, n[s] - (int64_t)g * kGroup);
            F.groups.push_back(GroupDesc{st, c, (uint32_t)s, 0});
        }
        ntot += (uint64_t)n[s];
    }
    ForestDev &D = F.dev;
    D.nseg = (uint32_t)nseg;
    D.ntot = (uint32_t)ntot;
    D.ntiles = (uint32_t)F.tiles.size();
    D.ngroups = (uint32_t)F.groups.size();
    D.mcap = (uint32_t)(2 * ntot);
    D.has32 = has32;
    D.has64 = has64;
}

// Capacities that cover the current tables.
ForestCaps bh_caps_of(const ForestHost &F) {
    ForestCaps c;
    c.nseg = F.dev.nseg;
    c.ntot = F.dev.ntot;
    c.ntiles = F.dev.ntiles;
    c.ngroups = F.dev.ngroups;
    c.fp32 = F.dev.has32 != 0;
    c.fp64 = F.dev.has64 != 0;
    c.quad = ((F.dev.has32 | F.dev.has64) & kVarQuadBits) != 0;
    c.group = ((F.dev.has32 | F.dev.has64) & kVarGroupBits) != 0;
    return c;
}

// Lays out the device buffers for capacities `c` in `ws` (or only measures them when
// ws == NULL).  Returns the bytes needed (0 when the sizes overflow).  Counts in F.dev
// are left untouched.
size_t bh_forest_carve(ForestHost &F, const ForestCaps &cap, char *ws) {
    ForestDev &D = F.dev;
    const size_t N = cap.ntot, Mc = 2 * (size_t)cap.ntot, S = cap.nseg;
    const size_t scan_len = std::max<size_t>(std::max<size_t>(256 * (size_t)cap.ntiles, N), Mc);
    const size_t blocks = (Mc + 255) / 256;
    // (pointer, count, element size) in carve order
    struct Slot {
        void **p;
        size_t count, elem;
    };
    const Slot slots[] = {
        {(void **)&D.seg, S, sizeof(SegDesc)},
        {(void **)&D.st, S, sizeof(SegState)},
        {(void **)&D.tiles, cap.ntiles, sizeof(TileDesc)},
        {(void **)&D.groups, cap.ngroups, sizeof(GroupDesc)},
        {(void **)&D.segid, N, 4},
        {(void **)&D.keys, N, 8},
        {(void **)&D.keys_alt, N, 8},
        {(void **)&D.idx, N, 4},
        {(void **)&D.idx_alt, N, 4},
        {(void **)&D.cnt, 256 * (size_t)cap.ntiles + 1, 4},
        {(void **)&D.segtot, 256 * S, 4},
        {(void **)&D.segp, 256 * S, 4},
        {(void **)&D.scan_tmp, scan_len / 2048 + 2, 4},
        {(void **)&D.spos, 3 * N, 8},
        {(void **)&D.smass, N, 8},
        {(void **)&D.pk, N, sizeof(double4)},
        {(void **)&D.lcp, N + 1, 1},
        {(void **)&D.mask, N, 4},
        {(void **)&D.base, N + 1, 4},
        {(void **)&D.nlevel, Mc, 1},
        {(void **)&D.nchild, Mc + 1, 4},
        {(void **)&D.nfirst, Mc, 4},
        {(void **)&D.ncount, Mc, 4},
        {(void **)&D.nparent, Mc, 4},
        {(void **)&D.ncrank, Mc, 4},
        {(void **)&D.cs, Mc + 1, 4},
        {(void **)&D.slot_of, Mc, 4},
        {(void **)&D.lvl_list, 256 * blocks, sizeof(uint4)},
        {(void **)&D.blk_lvl, (kMaxLevel + 2) * blocks, 2},
        {(void **)&D.uM, Mc, 8},
        {(void **)&D.uS, 3 * Mc, 8},
        {(void **)&D.rlam, N, 1},
        {(void **)&D.tile_mm, 6 * (size_t)cap.ntiles, 8},
        {(void **)&D.w32, cap.fp32 ? Mc : 0, sizeof(WRec32)},
        {(void **)&D.w64, cap.fp64 ? Mc : 0, sizeof(WRec64)},
        {(void **)&D.uQ, cap.quad ? 6 * Mc : 0, 8},
        {(void **)&D.q32, cap.quad && cap.fp32 ? 2 * Mc : 0, sizeof(float4)},
        {(void **)&D.q64, cap.quad && cap.fp64 ? 6 * Mc : 0, 8},
        {(void **)&D.err, 64, 4},
        {(void **)&D.stats, 8, 8},
        {(void **)&D.red, 2 * S, 8},
        {(void **)&D.pot, N, 8},
        {(void **)&D.gbox, cap.group ? 6 * N : 0, 8},
        {(void **)&D.wq, kWalkQueues, 4},
    };
    std::vector<bh_host::Region> regions;
    for (const Slot &sl : slots) regions.push_back(bh_host::Region{sl.count, sl.elem});
    std::vector<size_t> off;
    size_t total = 0;
    if (!bh_host::layout(regions, off, total)) return 0;
    for (size_t i = 0; i < regions.size(); ++i)
        *slots[i].p = (ws && regions[i].count) ? (void *)(ws + off[i]) : nullptr;
    F.caps = cap;
    F.ws = ws;
    F.ws_bytes = total;
    return total;
}

size_t bh_plan_forest(ForestHost &F, int32_t nseg, const int64_t *n, const bh_params *p, char *ws) {
    bh_forest_tables(F, nseg, n, p);
    return bh_forest_carve(F, bh_caps_of(F), ws);
}

static bh_status validate_sizes(int32_t nseg, const int64_t *n, const bh_params *p) {
    if (nseg < 1) return bh_fail(BH_E_INVAL, "need at least one simulation");
    if (!n || !p) return bh_fail(BH_E_INVAL, "NULL size or params array");
    int64_t tot = 0;
    for (int32_t s = 0; s < nseg; ++s) {
        if (n[s] < 1) return bh_fail(BH_E_INVAL, "every simulation needs n >= 1");
        bh_status st = bh_check_params(&p[s]);
        if (st != BH_OK) return st;
        tot += n[s];
        if (tot > (int64_t)0x3fffffff) return bh_fail(BH_E_INVAL, "too many particles (limit 2^30 - 1 per call)");
    }
    return BH_OK;
}

bh_status bh_forest_upload_tables(ForestHost &F) {
    hipStream_t s = F.ctx->stream;
    ForestDev &D = F.dev;
    const ForestCaps &c = F.caps;
    if (D.nseg > c.nseg || D.ntot > c.ntot || D.ntiles > c.ntiles || D.ngroups > c.ngroups ||
        (D.has32 && !c.fp32) || (D.has64 && !c.fp64) || (((D.has32 | D.has64) & kVarQuadBits) && !c.quad) ||
        (((D.has32 | D.has64) & kVarGroupBits) && !c.group))
        return bh_fail(BH_E_NOMEM, "forest membership exceeds the planned capacity");
    HIPCHK(hipMemcpyAsync(D.seg, F.seg.data(), sizeof(SegDesc) * F.seg.size(), hipMemcpyHostToDevice, s));
    if (!F.tiles.empty())
        HIPCHK(hipMemcpyAsync(D.tiles, F.tiles.data(), sizeof(TileDesc) * F.tiles.size(), hipMemcpyHostToDevice, s));
    if (!F.groups.empty())
        HIPCHK(hipMemcpyAsync(D.groups, F.groups.data(), sizeof(GroupDesc) * F.groups.size(), hipMemcpyHostToDevice, s));
    HIPCHK(launch_segid(D, s));
    // the host tables must outlive the copies
    HIPCHK(hipStreamSynchronize(s));
    return BH_OK;
}

bh_status bh_forest_init(bh_ctx *ctx, ForestHost &F, int32_t nseg, const int64_t *n, const bh_params *p, void *ws,
                         size_t ws_bytes) {
    if (!ws) return bh_fail(BH_E_INVAL, "workspace is NULL");
    if (((uintptr_t)ws & 255) != 0) return bh_fail(BH_E_INVAL, "workspace must be 256-byte aligned");
    size_t need = bh_plan_forest(F, nseg, n, p, nullptr);
    if (need == 0) return bh_fail(BH_E_NOMEM, "workspace size overflows");
    if (ws_bytes < need) return bh_fail(BH_E_NOMEM, "workspace too small: need " + std::to_string(need) + " bytes");
    bh_plan_forest(F, nseg, n, p, (char *)ws);
    F.ctx = ctx;
    HIPCHK(launch_fill_u32(F.dev.err, 0, 64, ctx->stream));
    HIPCHK(launch_fill_u32((uint32_t *)F.dev.stats, 0, 16, ctx->stream));
    return bh_forest_upload_tables(F);
}

bh_status bh_forest_upload_seg(ForestHost &F) {
    HIPCHK(hipMemcpyAsync(F.dev.seg, F.seg.data(), sizeof(SegDesc) * F.seg.size(), hipMemcpyHostToDevice,
                          F.ctx->stream));
    // keep the host table alive until the copy has been consumed
    HIPCHK(hipStreamSynchronize(F.ctx->stream));
    return BH_OK;
}

bh_status bh_forest_eval(ForestHost &F, const double *pos, const double *mass, double *acc, double *pot,
                         bool want_pot, hipStream_t s) {
    if (!s) s = F.ctx->stream;
    HIPCHK(launch_build(F.dev, pos, mass, s));
    HIPCHK(launch_upward(F.dev, s));
    HIPCHK(launch_walk(F.dev, false, want_pot, acc, pot, nullptr, nullptr, nullptr, s, F.walk_shape));
    return BH_OK;
}

bh_status bh_forest_kdk(ForestHost &F, double *pos, double *vel, const double *mass, double *acc, hipStream_t s) {
    if (!s) s = F.ctx->stream;
    HIPCHK(launch_kick(F.dev, vel, acc, 0, s));
    HIPCHK(launch_drift(F.dev, pos, vel, 0, s));
    bh_status st = bh_forest_eval(F, pos, mass, acc, nullptr, false, s);
    if (st != BH_OK) return st;
    HIPCHK(launch_kick(F.dev, vel, acc, 0, s));
    return BH_OK;
}

// nsteps KDK steps; between two steps the closing half-kick, the next opening
// half-kick and its drift run as one fused pass (same roundings, same order).
bh_status bh_forest_kdk_steps(ForestHost &F, double *pos, double *vel, const double *mass, double *acc,
                              int32_t nsteps, hipStream_t s) {
    if (nsteps <= 0) return BH_OK;
    if (!s) s = F.ctx->stream;
    HIPCHK(launch_kick(F.dev, vel, acc, 0, s));
    HIPCHK(launch_drift(F.dev, pos, vel, 0, s));
    for (int32_t k = 0; k < nsteps; ++k) {
        if (k > 0) HIPCHK(launch_kick_kick_drift(F.dev, pos, vel, acc, s));
        bh_status st = bh_forest_eval(F, pos, mass, acc, nullptr, false, s);
        if (st != BH_OK) return st;
    }
    HIPCHK(launch_kick(F.dev, vel, acc, 0, s));
    return BH_OK;
}

void bh_ctx_attach(bh_ctx *ctx, ForestHost *F) {
    if (ctx) ctx->live.push_back(F);
}

void bh_ctx_detach(bh_ctx *ctx, ForestHost *F) {
    if (!ctx) return;
    for (size_t i = 0; i < ctx->live.size(); ++i)
        if (ctx->live[i] == F) {
            ctx->live.erase(ctx->live.begin() + (long)i);
            return;
        }
}

// Reports the fault bits gathered since the last report, and clears them.
bh_status bh_forest_check_err(ForestHost &F) {
    uint32_t e = 0;
    HIPCHK(hipMemcpyAsync(&e, F.dev.err, sizeof(uint32_t), hipMemcpyDeviceToHost, F.ctx->stream));
    HIPCHK(hipStreamSynchronize(F.ctx->stream));
    if (e) HIPCHK(launch_fill_u32(F.dev.err, 0, 1, F.ctx->stream));
    if (e & kErrStack) return bh_fail(BH_E_OVERFLOW, "walk stack overflow");
    if (e & kErrTree) return bh_fail(BH_E_DEVICE, "inconsistent tree detected on the device");
    if (e & kErrNonFinite) return bh_fail(BH_E_DEVICE, "device fault flag: non-finite position or mass");
    return BH_OK;
}

namespace {
struct EventPair {
    hipEvent_t a = nullptr, b = nullptr;
    ~EventPair() {
        if (a) (void)hipEventDestroy(a);
        if (b) (void)hipEventDestroy(b);
    }
};
}  // namespace

// --------------------------------------------------------- static scratch ---
// Device memory of the entry points that allocate nothing (bh_ic_generate_static):
// one array per GPU, held until the process ends.  Host code never passes the
// array's name to a kernel (on the host it is only a stand-in for the symbol); it
// uses the device address that hipGetSymbolAddress returns for the current device,
// looked up once per device when a context is created on it.
constexpr size_t kStaticScratchBytes = 16384;
static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};
}  // namespace

static bh_status static_scratch_init(int device) {
    if (device < 0 || device >= kMaxDevices) return bh_fail(BH_E_INVAL, "device index beyond the library's table");
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (g_scratch_ptr[device]) return BH_OK;
    void *ptr = nullptr;   // device `device` is current (the caller set it)
    hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr)
        return bh_fail(BH_E_DEVICE, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    g_scratch_ptr[device] = ptr;
    return BH_OK;
}

static void *static_scratch(int device) {
    if (device < 0 || device >= kMaxDevices) return nullptr;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    return g_scratch_ptr[device];
}

// ---------------------------------------------------------------- context ---

extern "C" {

const char *bh_last_error(void) { return g_err.c_str(); }
const char *bh_version(void) { return "bh-mi355x 0.1"; }

bh_status bh_ctx_create(int device, void *hip_stream, bh_ctx **out) {
    if (!out) return bh_fail(BH_E_INVAL, "out is NULL");
    int ndev = 0;
    HIPCHK(hipGetDeviceCount(&ndev));
    if (device < 0 || device >= ndev) return bh_fail(BH_E_INVAL, "no such device");
    HIPCHK(hipSetDevice(device));
    bh_status sst = static_scratch_init(device);
    if (sst != BH_OK) return sst;
    bh_ctx *c = new (std::nothrow) bh_ctx();
    if (!c) return bh_fail(BH_E_NOMEM, "host allocation failed");
    c->device = device;
    c->stream = (hipStream_t)hip_stream;
    *out = c;
    return BH_OK;
}

bh_status bh_ctx_destroy(bh_ctx *ctx) {
    if (!ctx) return BH_OK;
    (void)hipSetDevice(ctx->device);
    (void)hipStreamSynchronize(ctx->stream);
    for (ForestHost *F : ctx->live) F->ctx = nullptr;   // handles outliving their context
    delete ctx;
    return BH_OK;
}

bh_status bh_ctx_sync(bh_ctx *ctx) {
    if (!ctx) return bh_fail(BH_E_INVAL, "ctx is NULL");
    HIPCHK(hipStreamSynchronize(ctx->stream));
    for (ForestHost *F : ctx->live) {
        bh_status st = bh_forest_check_err(*F);
        if (st != BH_OK) return st;
    }
    return BH_OK;
}

// ------------------------------------------------------------------- tree ---

size_t bh_workspace_bytes(int64_t n, const bh_params *p) {
    if (n < 1 || !p || bh_check_params(p) != BH_OK) return 0;
    ForestHost F;
    return bh_plan_forest(F, 1, &n, p, nullptr);
}

bh_status bh_build(bh_ctx *ctx, int64_t n, const double *pos, const double *mass, const bh_params *p, void *ws,
                   size_t ws_bytes, bh_tree **out) {
    if (!ctx || !out || !pos || !mass) return bh_fail(BH_E_INVAL, "NULL argument");
    bh_status st = validate_sizes(1, &n, p);
    if (st != BH_OK) return st;
    bh_tree *t = new (std::nothrow) bh_tree();
    if (!t) return bh_fail(BH_E_NOMEM, "host allocation failed");
    st = bh_forest_init(ctx, t->F, 1, &n, p, ws, ws_bytes);
    if (st != BH_OK) {
        delete t;
        return st;
    }
    t->pos = pos;
    t->mass = mass;
    hipError_t e = launch_build(t->F.dev, pos, mass, ctx->stream);
    if (e != hipSuccess) {
        delete t;
        return bh_fail(BH_E_DEVICE, std::string("build launch: ") + hipGetErrorString(e));
    }
    bh_ctx_attach(ctx, &t->F);
    *out = t;
    return BH_OK;
}

bh_status bh_rebuild(bh_ctx *ctx, bh_tree *t, const double *pos, const double *mass) {
    if (!ctx || !t || !pos || !mass) return bh_fail(BH_E_INVAL, "NULL argument");
    if (t->F.ctx != ctx) return bh_fail(BH_E_INVAL, "handle created on another context, or its context was destroyed");
    t->pos = pos;
    t->mass = mass;
    t->upward_done = false;
    t->lists_buf = nullptr;
    HIPCHK(launch_build(t->F.dev, pos, mass, ctx->stream));
    return BH_OK;
}

bh_status bh_upward(bh_ctx *ctx, bh_tree *t) {
    if (!ctx || !t) return bh_fail(BH_E_INVAL, "NULL argument");
    if (t->F.ctx != ctx) return bh_fail(BH_E_INVAL, "handle created on another context, or its context was destroyed");
    HIPCHK(launch_upward(t->F.dev, ctx->stream));
    t->upward_done = true;
    t->lists_buf = nullptr;
    return BH_OK;
}

// ------------------------------------------------------ interaction lists ---

namespace {

using bh_host::list_chunks_for;
using bh_host::list_layout;
using bh_host::ListLayout;

ListDev list_dev(void *buf, size_t ngroups, size_t nchunks) {
    const ListLayout l = list_layout(ngroups, nchunks);
    char *b = static_cast<char *>(buf);
    ListDev d;
    d.ctr = reinterpret_cast<unsigned long long *>(b);
    d.head = reinterpret_cast<uint32_t *>(b + l.head);
    d.count = reinterpret_cast<uint32_t *>(b + l.count);
    d.next = reinterpret_cast<uint32_t *>(b + l.next);
    d.ent = reinterpret_cast<uint4 *>(b + l.ent);
    d.nchunks = (uint32_t)nchunks;
    return d;
}

bh_status lists_supported(const bh_tree *t) {
    for (const SegDesc &d : t->F.seg)
        if (d.group) return bh_fail(BH_E_INVAL, "interaction lists: trees with the per-body test only");
    return BH_OK;
}

}  // namespace

static_assert(sizeof(bh_list_entry) == bh_host::kListEntryBytes && kListParts == bh_host::kListPartitions,
              "list layout constants");

bh_status bh_lists_build(bh_ctx *ctx, bh_tree *t, void *buf, size_t bytes, size_t *bytes_needed) {
    if (!ctx || !t || !buf) return bh_fail(BH_E_INVAL, "NULL argument");
    if (t->F.ctx != ctx) return bh_fail(BH_E_INVAL, "handle created on another context, or its context was destroyed");
    if (reinterpret_cast<uintptr_t>(buf) % 256) return bh_fail(BH_E_INVAL, "list buffer must be 256-byte aligned");
    if (!t->upward_done) return bh_fail(BH_E_INVAL, "bh_upward must run before bh_lists_build");
    bh_status st = lists_supported(t);
    if (st != BH_OK) return st;
    t->lists_buf = nullptr;
    const size_t ng = t->F.dev.ngroups;
    if (bytes < list_layout(ng, 0).total) {
        // not even the counters and group tables fit: a lower bound (one chunk per group)
        if (bytes_needed) *bytes_needed = list_layout(ng, ng).total;
        return bh_fail(BH_E_NOMEM, "list buffer too small for its tables");
    }
    const size_t nc = list_chunks_for(ng, bytes);   // may be 0: the walk then only counts
    const ListDev ld = list_dev(buf, ng, nc);
    HIPCHK(launch_fill_u32(reinterpret_cast<uint32_t *>(ld.ctr), 0, 64 * kListParts, ctx->stream));
    HIPCHK(launch_lists_build(t->F.dev, ld, ctx->stream));
    std::vector<unsigned long long> taken(32 * kListParts);
    HIPCHK(hipMemcpyAsync(taken.data(), ld.ctr, sizeof(unsigned long long) * taken.size(), hipMemcpyDeviceToHost,
                          ctx->stream));
    st = bh_forest_check_err(t->F);
    if (st != BH_OK) return st;
    // chunk ids of partition k are k + kListParts t: the lists need ids up to the largest one
    // reserved (a wave reserves kListReserve at a time and may leave some unused)
    size_t span = 0;
    for (uint32_t k = 0; k < kListParts; ++k) {
        const unsigned long long n = taken[32 * (size_t)k];
        if (n) span = std::max<size_t>(span, (size_t)(n - 1) * kListParts + k + 1);
    }
    const size_t need = list_layout(ng, span).total;
    if (bytes_needed) *bytes_needed = need;
    if (span > nc) return bh_fail(BH_E_NOMEM, "list buffer too small for these lists (see bytes_needed)");
    t->lists_buf = buf;
    t->lists_chunks = (uint32_t)nc;
    return BH_OK;
}

bh_status bh_lists_forces(bh_ctx *ctx, bh_tree *t, const void *buf, double *acc, double *pot) {
    if (!ctx || !t || !buf || !acc) return bh_fail(BH_E_INVAL, "NULL argument");
    if (t->F.ctx != ctx) return bh_fail(BH_E_INVAL, "handle created on another context, or its context was destroyed");
    if (!t->lists_buf || t->lists_buf != buf)
        return bh_fail(BH_E_INVAL, "no interaction lists of the current tree in this buffer");
    const ListDev ld = list_dev(const_cast<void *>(buf), t->F.dev.ngroups, t->lists_chunks);
    HIPCHK(launch_lists_eval(t->F.dev, ld, pot != nullptr, acc, pot, ctx->stream));
    return BH_OK;
}

bh_status bh_forces(bh_ctx *ctx, bh_tree *t, double *acc, double *pot) {
    if (!ctx || !t || !acc) return bh_fail(BH_E_INVAL, "NULL argument");
    if (t->F.ctx != ctx) return bh_fail(BH_E_INVAL, "handle created on another context, or its context was destroyed");
    if (!t->upward_done) return bh_fail(BH_E_INVAL, "bh_upward must run before bh_forces");
    HIPCHK(launch_walk(t->F.dev, false, pot != nullptr, acc, pot, nullptr, nullptr, nullptr, ctx->stream,
                       t->F.walk_shape));
    return BH_OK;
}

bh_status bh_forces_stats(bh_ctx *ctx, bh_tree *t, double *acc, double *pot, int64_t *n_mono, int64_t *n_p2p,
                          uint64_t *hash, bh_stats *totals) {
    if (!ctx || !t || !acc) return bh_fail(BH_E_INVAL, "NULL argument");
    if (t->F.ctx != ctx) return bh_fail(BH_E_INVAL, "handle created on another context, or its context was destroyed");
    if (!t->upward_done) return bh_fail(BH_E_INVAL, "bh_upward must run before bh_forces_stats");
    EventPair ev;
    HIPCHK(hipEventCreate(&ev.a));
    HIPCHK(hipEventCreate(&ev.b));
    HIPCHK(launch_fill_u32((uint32_t *)t->F.dev.stats, 0, 16, ctx->stream));
    HIPCHK(hipEventRecord(ev.a, ctx->stream));
    HIPCHK(launch_walk(t->F.dev, true, pot != nullptr, acc, pot, n_mono, n_p2p, hash, ctx->stream,
                       t->F.walk_shape));
    HIPCHK(hipEventRecord(ev.b, ctx->stream));
    unsigned long long h[8];
    HIPCHK(hipMemcpyAsync(h, t->F.dev.stats, sizeof(h), hipMemcpyDeviceToHost, ctx->stream));
    bh_status st = bh_forest_check_err(t->F);
    if (st != BH_OK) return st;
    float ms = 0.0f;
    HIPCHK(hipEventElapsedTime(&ms, ev.a, ev.b));
    if (totals) {
        totals->n_mono = h[0];
        totals->n_p2p = h[1];
        totals->n_visits = h[2];
        totals->n_fallback = h[3];
        totals->wave_visits = h[4];
        totals->wave_entries = h[5];
        totals->wave_accepts = h[6];
        totals->wave_leaves = h[7];
        totals->t_ms = ms;
    }
    return BH_OK;
}

bh_status bh_forces_range(bh_ctx *ctx, bh_tree *t, int64_t first, int64_t count, double *acc, double *pot,
                          int64_t *n_mono, int64_t *n_p2p, int64_t *work, int64_t *group_work) {
    if (!ctx || !t || !acc) return bh_fail(BH_E_INVAL, "NULL argument");
    if (t->F.ctx != ctx) return bh_fail(BH_E_INVAL, "handle created on another context, or its context was destroyed");
    if (!t->upward_done) return bh_fail(BH_E_INVAL, "bh_upward must run before bh_forces_range");
    const int64_t n = t->F.dev.ntot;
    if (first < 0 || count < 0 || first > n || count > n - first)
        return bh_fail(BH_E_INVAL, "target range outside [0, n)");
    if (count == 0) return BH_OK;
    // the 64-body groups of a tree cover sorted ranks [64 g, 64 g + 64)
    ForestDev D = t->F.dev;
    const int64_t g0 = first / kGroup, g1 = (first + count + kGroup - 1) / kGroup;
    D.groups += g0;
    D.ngroups = (uint32_t)(g1 - g0);
    const bool stats = n_mono || n_p2p || work || group_work;
    if (stats) HIPCHK(launch_fill_u32((uint32_t *)t->F.dev.stats, 0, 16, ctx->stream));
    // a part of the groups loses less to the launch's tail with one wavefront per workgroup
    // (the whole tree keeps its own shape); the shape changes no result
    const int waves = count == n ? t->F.walk_shape : 1;
    HIPCHK(launch_walk(D, stats, pot != nullptr, acc, pot, n_mono, n_p2p, nullptr, ctx->stream, waves,
                       (uint32_t)first, (uint32_t)(first + count), work, group_work));
    return BH_OK;
}

bh_status bh_shard_bounds(bh_ctx *ctx, bh_tree *t, const int64_t *cost_a, const int64_t *cost_b, int32_t G,
                          int64_t *bounds) {
    if (!ctx || !t || !bounds) return bh_fail(BH_E_INVAL, "NULL argument");
    if (t->F.ctx != ctx) return bh_fail(BH_E_INVAL, "handle created on another context, or its context was destroyed");
    if (G < 1 || G > 65536) return bh_fail(BH_E_INVAL, "G must be in [1, 65536]");
    if (!t->upward_done) return bh_fail(BH_E_INVAL, "the tree must be built (bh_upward) before bh_shard_bounds");
    HIPCHK(launch_shard_bounds(t->F.dev, t->F.dev.ntot, cost_a, cost_b, nullptr, (uint32_t)G, bounds, ctx->stream));
    return BH_OK;
}

bh_status bh_shard_bounds_groups(bh_ctx *ctx, bh_tree *t, const int64_t *group_work, int32_t G, int64_t *bounds) {
    if (!ctx || !t || !group_work || !bounds) return bh_fail(BH_E_INVAL, "NULL argument");
    if (t->F.ctx != ctx) return bh_fail(BH_E_INVAL, "handle created on another context, or its context was destroyed");
    if (G < 1 || G > 65536) return bh_fail(BH_E_INVAL, "G must be in [1, 65536]");
    if (!t->upward_done) return bh_fail(BH_E_INVAL, "the tree must be built (bh_upward) before bh_shard_bounds_groups");
    HIPCHK(launch_shard_bounds(t->F.dev, t->F.dev.ntot, nullptr, nullptr, group_work, (uint32_t)G, bounds,
                               ctx->stream));
    return BH_OK;
}

bh_status bh_tree_info(bh_ctx *ctx, bh_tree *t, int64_t *n_nodes, double lo[3], int32_t *k) {
    if (!ctx || !t) return bh_fail(BH_E_INVAL, "NULL argument");
    if (t->F.ctx != ctx) return bh_fail(BH_E_INVAL, "handle created on another context, or its context was destroyed");
    SegState s;
    HIPCHK(hipMemcpyAsync(&s, t->F.dev.st, sizeof(SegState), hipMemcpyDeviceToHost, ctx->stream));
    bh_status st = bh_forest_check_err(t->F);
    if (st != BH_OK) return st;
    if (n_nodes) *n_nodes = s.nn;
    if (lo) for (int d = 0; d < 3; ++d) lo[d] = s.lo[d];
    if (k) *k = s.k;
    return BH_OK;
}

bh_status bh_tree_export(bh_ctx *ctx, bh_tree *t, uint64_t *keys, uint32_t *perm, int32_t *level, uint32_t *first,
                         uint32_t *count, int32_t *parent, double *M, double *com, int64_t *n_nodes,
                         uint64_t *isect_hash) {
    if (!ctx || !t) return bh_fail(BH_E_INVAL, "NULL argument");
    if (t->F.ctx != ctx) return bh_fail(BH_E_INVAL, "handle created on another context, or its context was destroyed");
    if ((M || com || isect_hash) && !t->upward_done)
        return bh_fail(BH_E_INVAL, "bh_upward must run before exporting M, com or the checksums");
    HIPCHK(launch_export(t->F.dev, 0, keys, perm, level, first, count, parent, M, com, ctx->stream));
    if (isect_hash)   // the counting walk, writing only the per-body checksums
        HIPCHK(launch_walk(t->F.dev, true, false, nullptr, nullptr, nullptr, nullptr, isect_hash, ctx->stream,
                           t->F.walk_shape));
    if (n_nodes || isect_hash) {
        SegState st;
        HIPCHK(hipMemcpyAsync(&st, t->F.dev.st, sizeof(SegState), hipMemcpyDeviceToHost, ctx->stream));
        bh_status rs = bh_forest_check_err(t->F);
        if (rs != BH_OK) return rs;
        if (n_nodes) *n_nodes = st.nn;
    }
    return BH_OK;
}

bh_status bh_tree_free(bh_ctx *ctx, bh_tree *t) {
    if (t) bh_ctx_detach(t->F.ctx, &t->F);
    (void)ctx;
    delete t;
    return BH_OK;
}

// ------------------------------------------------------------- simulation ---

size_t bh_sim_workspace_bytes(int64_t n, const bh_params *p) { return bh_workspace_bytes(n, p); }

bh_status bh_sim_create(bh_ctx *ctx, int64_t n, double *pos, double *vel, const double *mass, double *acc,
                        const bh_params *p, void *ws, size_t ws_bytes, bh_sim **out) {
    if (!ctx || !out || !pos || !vel || !mass || !acc) return bh_fail(BH_E_INVAL, "NULL argument");
    bh_status st = validate_sizes(1, &n, p);
    if (st != BH_OK) return st;
    bh_sim *sm = new (std::nothrow) bh_sim();
    if (!sm) return bh_fail(BH_E_NOMEM, "host allocation failed");
    st = bh_forest_init(ctx, sm->F, 1, &n, p, ws, ws_bytes);
    if (st != BH_OK) {
        delete sm;
        return st;
    }
    sm->pos = pos;
    sm->vel = vel;
    sm->mass = mass;
    sm->acc = acc;
    bh_ctx_attach(ctx, &sm->F);
    *out = sm;
    return BH_OK;
}

bh_status bh_step(bh_ctx *ctx, bh_sim *sm, int32_t nsteps, double dt) {
    if (!ctx || !sm) return bh_fail(BH_E_INVAL, "NULL argument");
    if (sm->F.ctx != ctx) return bh_fail(BH_E_INVAL, "handle created on another context, or its context was destroyed");
    if (nsteps < 0 || !std::isfinite(dt)) return bh_fail(BH_E_INVAL, "nsteps must be >= 0 and dt finite");
    if (sm->F.seg[0].dt != dt) {
        sm->F.seg[0].dt = dt;
        bh_status st = bh_forest_upload_seg(sm->F);
        if (st != BH_OK) return st;
    }
    if (!sm->have_acc) {
        bh_status st = bh_forest_eval(sm->F, sm->pos, sm->mass, sm->acc, nullptr, false, nullptr);
        if (st != BH_OK) return st;
        sm->have_acc = true;
    }
    return bh_forest_kdk_steps(sm->F, sm->pos, sm->vel, sm->mass, sm->acc, nsteps, nullptr);
}

bh_status bh_energy(bh_ctx *ctx, bh_sim *sm, double out_KW[2]) {
    if (!ctx || !sm || !out_KW) return bh_fail(BH_E_INVAL, "NULL argument");
    if (sm->F.ctx != ctx) return bh_fail(BH_E_INVAL, "handle created on another context, or its context was destroyed");
    bh_status st = bh_forest_eval(sm->F, sm->pos, sm->mass, sm->acc, sm->F.dev.pot, true, nullptr);
    if (st != BH_OK) return st;
    sm->have_acc = true;
    HIPCHK(launch_energy(sm->F.dev, sm->vel, sm->mass, sm->F.dev.pot, sm->F.dev.red, ctx->stream));
    double kw[2];
    HIPCHK(hipMemcpyAsync(kw, sm->F.dev.red, sizeof(kw), hipMemcpyDeviceToHost, ctx->stream));
    st = bh_forest_check_err(sm->F);
    if (st != BH_OK) return st;
    out_KW[0] = kw[0];
    out_KW[1] = kw[1];
    return BH_OK;
}

bh_status bh_sim_destroy(bh_ctx *ctx, bh_sim *sm) {
    if (sm) bh_ctx_detach(sm->F.ctx, &sm->F);
    (void)ctx;
    delete sm;
    return BH_OK;
}

// ----------------------------------------------------------------- forest ---

size_t bh_forest_workspace_bytes(int32_t n_sims, const int64_t *n, const bh_params *per_sim) {
    if (validate_sizes(n_sims, n, per_sim) != BH_OK) return 0;
    ForestHost F;
    return bh_plan_forest(F, n_sims, n, per_sim, nullptr);
}

bh_status bh_forest_create(bh_ctx *ctx, int32_t n_sims, const int64_t *n, const bh_params *per_sim, double *pos,
                           double *vel, const double *mass, double *acc, void *ws, size_t ws_bytes, bh_forest **out) {
    if (!ctx || !out || !pos || !vel || !mass || !acc) return bh_fail(BH_E_INVAL, "NULL argument");
    bh_status st = validate_sizes(n_sims, n, per_sim);
    if (st != BH_OK) return st;
    bh_forest *fo = new (std::nothrow) bh_forest();
    if (!fo) return bh_fail(BH_E_NOMEM, "host allocation failed");
    st = bh_forest_init(ctx, fo->F, n_sims, n, per_sim, ws, ws_bytes);
    if (st != BH_OK) {
        delete fo;
        return st;
    }
    fo->pos = pos;
    fo->vel = vel;
    fo->mass = mass;
    fo->acc = acc;
    bh_ctx_attach(ctx, &fo->F);
    *out = fo;
    return BH_OK;
}

static bh_status forest_set_dt(bh_forest *fo, const double *dt) {
    bool changed = false;
    for (size_t s = 0; s < fo->F.seg.size(); ++s) {
        if (!std::isfinite(dt[s])) return bh_fail(BH_E_INVAL, "dt must be finite");
        if (fo->F.seg[s].dt != dt[s]) {
            fo->F.seg[s].dt = dt[s];
            changed = true;
        }
    }
    if (changed) {
        if (fo->graph) {
            (void)hipGraphExecDestroy(fo->graph);
            fo->graph = nullptr;
        }
        return bh_forest_upload_seg(fo->F);
    }
    return BH_OK;
}

bh_status bh_forest_step(bh_ctx *ctx, bh_forest *fo, int32_t nsteps, const double *dt) {
    if (!ctx || !fo || !dt) return bh_fail(BH_E_INVAL, "NULL argument");
    if (fo->F.ctx != ctx) return bh_fail(BH_E_INVAL, "handle created on another context, or its context was destroyed");
    if (nsteps < 0) return bh_fail(BH_E_INVAL, "nsteps must be >= 0");
    bh_status st = forest_set_dt(fo, dt);
    if (st != BH_OK) return st;
    if (!fo->have_acc) {
        st = bh_forest_eval(fo->F, fo->pos, fo->mass, fo->acc, nullptr, false, nullptr);
        if (st != BH_OK) return st;
        fo->have_acc = true;
    }
    return bh_forest_kdk_steps(fo->F, fo->pos, fo->vel, fo->mass, fo->acc, nsteps, nullptr);
}

bh_status bh_forest_forces(bh_ctx *ctx, bh_forest *fo, double *pot) {
    if (!ctx || !fo) return bh_fail(BH_E_INVAL, "NULL argument");
    if (fo->F.ctx != ctx) return bh_fail(BH_E_INVAL, "handle created on another context, or its context was destroyed");
    bh_status st = bh_forest_eval(fo->F, fo->pos, fo->mass, fo->acc, pot, pot != nullptr, nullptr);
    if (st == BH_OK) fo->have_acc = true;
    return st;
}

bh_status bh_forest_step_graph(bh_ctx *ctx, bh_forest *fo, int32_t nsteps, const double *dt) {
    if (!ctx || !fo || !dt) return bh_fail(BH_E_INVAL, "NULL argument");
    if (fo->F.ctx != ctx) return bh_fail(BH_E_INVAL, "handle created on another context, or its context was destroyed");
    if (nsteps < 0) return bh_fail(BH_E_INVAL, "nsteps must be >= 0");
    bh_status st = forest_set_dt(fo, dt);
    if (st != BH_OK) return st;
    if (!fo->have_acc) {
        st = bh_forest_eval(fo->F, fo->pos, fo->mass, fo->acc, nullptr, false, nullptr);
        if (st != BH_OK) return st;
        fo->have_acc = true;
    }
    // a graph is recorded on a private stream (the caller's stream may be the null
    // stream, which cannot be captured) and replayed on the caller's stream
    hipStream_t s = ctx->stream;
    if (!fo->graph) {
        if (!fo->cap_stream) HIPCHK(hipStreamCreateWithFlags(&fo->cap_stream, hipStreamNonBlocking));
        hipGraph_t g = nullptr;
        HIPCHK(hipStreamBeginCapture(fo->cap_stream, hipStreamCaptureModeThreadLocal));
        bh_status cst = bh_forest_kdk(fo->F, fo->pos, fo->vel, fo->mass, fo->acc, fo->cap_stream);
        hipError_t ee = hipStreamEndCapture(fo->cap_stream, &g);
        if (cst != BH_OK) {
            if (g) (void)hipGraphDestroy(g);
            return cst;
        }
        HIPCHK(ee);
        hipError_t ie = hipGraphInstantiate(&fo->graph, g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        HIPCHK(ie);
    }
    for (int32_t k = 0; k < nsteps; ++k) HIPCHK(hipGraphLaunch(fo->graph, s));
    return BH_OK;
}


// ------------------------------------------------------------- autotuner ---

static std::mutex g_tune_mu;
static bh_host::TuneCache g_tune;
static bool g_tune_env_read = false;

static bool valid_walk_shape(int32_t shape) { return bh_host::valid_shape(shape); }

static int tune_shape(int k) { return kWalkWaves[k & 3] | (k >= 4 ? kWalkPersistent : 0); }

// The key a forest's tuned shape is kept under.
static bh_host::TuneKey tune_key(const ForestHost &F) {
    bh_host::TuneKey k;
    hipDeviceProp_t pr;
    if (hipGetDeviceProperties(&pr, F.ctx->device) == hipSuccess) {
        std::string arch(pr.gcnArchName);
        k.device = arch.substr(0, arch.find(':')) + ":" + std::to_string(pr.multiProcessorCount);
    } else {
        k.device = "device" + std::to_string(F.ctx->device);
    }
    k.n_log2 = bh_host::floor_log2(F.dev.ntot);
    k.sims_log2 = bh_host::floor_log2(F.dev.nseg);
    double wt = 0.0, tot = 0.0;
    for (const SegDesc &d : F.seg) {
        wt += (double)d.n * d.theta;
        tot += (double)d.n;
    }
    const double th = tot > 0.0 ? wt / tot : 0.0;
    k.theta_c = (int)std::lround(std::min(th, 1.0e4) * 100.0);
    k.precision = F.dev.has32 && F.dev.has64 ? "mixed" : F.dev.has32 ? "fp32" : "fp64";
    return k;
}

static bool read_file(const char *path, std::string &out) {
    FILE *fp = std::fopen(path, "rb");
    if (!fp) return false;
    char buf[4096];
    size_t r;
    out.clear();
    while ((r = std::fread(buf, 1, sizeof buf, fp)) > 0) {
        out.append(buf, r);
        if (out.size() > (64u << 20)) {   // no tuning cache is this large
            std::fclose(fp);
            return false;
        }
    }
    const bool ok = !std::ferror(fp);
    std::fclose(fp);
    return ok;
}

// Caller holds g_tune_mu.
static bh_status tune_load_locked(const char *path, bool missing_ok) {
    std::string text, err;
    if (!read_file(path, text)) {
        if (missing_ok) {
            FILE *fp = std::fopen(path, "rb");
            if (!fp) return BH_OK;   // no file yet: an empty cache
            std::fclose(fp);
        }
        return bh_fail(BH_E_IO, std::string("cannot read tuning cache ") + path);
    }
    if (!g_tune.merge_json(text, err)) return bh_fail(BH_E_IO, std::string("tuning cache ") + path + ": " + err);
    return BH_OK;
}

static bh_status tune_save_locked(const char *path) {
    const std::string text = g_tune.to_json();
    // a per-process temporary name, renamed over the file: concurrent writers do not
    // interleave, and a reader sees one whole file or the other
    const std::string tmp = std::string(path) + ".tmp" + std::to_string((long)getpid());
    FILE *fp = std::fopen(tmp.c_str(), "wb");
    if (!fp) return bh_fail(BH_E_IO, std::string("cannot write tuning cache ") + path);
    const bool ok = std::fwrite(text.data(), 1, text.size(), fp) == text.size();
    if (std::fclose(fp) != 0 || !ok || std::rename(tmp.c_str(), path) != 0) {
        std::remove(tmp.c_str());
        return bh_fail(BH_E_IO, std::string("cannot write tuning cache ") + path);
    }
    return BH_OK;
}

bh_status bh_tune_cache_load(const char *path) {
    if (!path) return bh_fail(BH_E_INVAL, "NULL path");
    std::lock_guard<std::mutex> lk(g_tune_mu);
    return tune_load_locked(path, false);
}

bh_status bh_tune_cache_save(const char *path) {
    if (!path) return bh_fail(BH_E_INVAL, "NULL path");
    std::lock_guard<std::mutex> lk(g_tune_mu);
    return tune_save_locked(path);
}

bh_status bh_tune_cache_clear(void) {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tune.clear();
    return BH_OK;
}

int64_t bh_tune_cache_size(void) {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    return (int64_t)g_tune.size();
}

static void forest_take_shape(bh_forest *fo, int shape) {
    if (shape != fo->F.walk_shape) {
        fo->F.walk_shape = shape;
        if (fo->graph) {   // recorded with the previous launch shape
            (void)hipGraphExecDestroy(fo->graph);
            fo->graph = nullptr;
        }
    }
}

bh_status bh_tree_set_walk_shape(bh_ctx *ctx, bh_tree *t, int32_t shape) {
    if (!ctx || !t) return bh_fail(BH_E_INVAL, "NULL argument");
    if (t->F.ctx != ctx) return bh_fail(BH_E_INVAL, "handle created on another context, or its context was destroyed");
    if (!valid_walk_shape(shape)) return bh_fail(BH_E_INVAL, "shape must be 1, 2, 4 or 8, optionally | BH_WALK_PERSISTENT");
    t->F.walk_shape = shape;
    return BH_OK;
}

bh_status bh_sim_set_walk_shape(bh_ctx *ctx, bh_sim *sm, int32_t shape) {
    if (!ctx || !sm) return bh_fail(BH_E_INVAL, "NULL argument");
    if (sm->F.ctx != ctx) return bh_fail(BH_E_INVAL, "handle created on another context, or its context was destroyed");
    if (!valid_walk_shape(shape)) return bh_fail(BH_E_INVAL, "shape must be 1, 2, 4 or 8, optionally | BH_WALK_PERSISTENT");
    sm->F.walk_shape = shape;
    return BH_OK;
}

bh_status bh_forest_set_walk_shape(bh_ctx *ctx, bh_forest *fo, int32_t shape) {
    if (!ctx || !fo) return bh_fail(BH_E_INVAL, "NULL argument");
    if (fo->F.ctx != ctx) return bh_fail(BH_E_INVAL, "handle created on another context, or its context was destroyed");
    if (!valid_walk_shape(shape)) return bh_fail(BH_E_INVAL, "shape must be 1, 2, 4 or 8, optionally | BH_WALK_PERSISTENT");
    forest_take_shape(fo, shape);
    return BH_OK;
}

bh_status bh_forest_autotune(bh_ctx *ctx, bh_forest *fo, uint32_t flags, int32_t *shape_out, double *ms_out) {
    if (!ctx || !fo) return bh_fail(BH_E_INVAL, "NULL argument");
    if (fo->F.ctx != ctx) return bh_fail(BH_E_INVAL, "handle created on another context, or its context was destroyed");
    if (flags & ~BH_TUNE_CACHED) return bh_fail(BH_E_INVAL, "unknown bits in flags");
    hipStream_t s = ctx->stream;
    ForestHost &F = fo->F;
    const char *env = std::getenv("BH_TUNE_CACHE");
    const bh_host::TuneKey key = tune_key(F);
    bh_host::TuneEntry hit;
    bool cached = false;
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        if (env && *env && !g_tune_env_read) {
            bh_status st = tune_load_locked(env, true);
            if (st != BH_OK) return st;
            g_tune_env_read = true;
        }
        cached = (flags & BH_TUNE_CACHED) && g_tune.find(key, hit) && valid_walk_shape(hit.shape);
    }
    HIPCHK(launch_build(F.dev, fo->pos, fo->mass, s));
    HIPCHK(launch_upward(F.dev, s));
    int best_shape = F.walk_shape;
    float best = 0.0f;
    if (cached) {
        best_shape = hit.shape;
        HIPCHK(launch_walk(F.dev, false, false, fo->acc, nullptr, nullptr, nullptr, nullptr, s, best_shape));
        if (ms_out)
            for (int k = 0; k < BH_TUNE_SHAPES; ++k) ms_out[k] = -1.0;
    } else {
        EventPair ev;
        HIPCHK(hipEventCreate(&ev.a));
        HIPCHK(hipEventCreate(&ev.b));
        constexpr int kReps = 2;
        for (int k = 0; k < BH_TUNE_SHAPES; ++k) {
            const int w = tune_shape(k);
            HIPCHK(launch_walk(F.dev, false, false, fo->acc, nullptr, nullptr, nullptr, nullptr, s, w));   // warm-up
            HIPCHK(hipEventRecord(ev.a, s));
            for (int r = 0; r < kReps; ++r)
                HIPCHK(launch_walk(F.dev, false, false, fo->acc, nullptr, nullptr, nullptr, nullptr, s, w));
            HIPCHK(hipEventRecord(ev.b, s));
            HIPCHK(hipEventSynchronize(ev.b));
            float ms = 0.0f;
            HIPCHK(hipEventElapsedTime(&ms, ev.a, ev.b));
            ms /= kReps;
            if (ms_out) ms_out[k] = ms;
            if (k == 0 || ms < best) {
                best = ms;
                best_shape = w;
            }
        }
    }
    bh_status st = bh_forest_check_err(F);
    if (st != BH_OK) return st;
    forest_take_shape(fo, best_shape);
    fo->have_acc = true;
    if (!cached) {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        g_tune.put(key, bh_host::TuneEntry{best_shape, (double)best});
        if (env && *env) {
            st = tune_save_locked(env);
            if (st != BH_OK) return st;
        }
    }
    if (shape_out) *shape_out = best_shape;
    return BH_OK;
}

bh_status bh_forest_destroy(bh_ctx *ctx, bh_forest *fo) {
    (void)ctx;
    if (!fo) return BH_OK;
    bh_ctx_detach(fo->F.ctx, &fo->F);
    if (fo->graph) (void)hipGraphExecDestroy(fo->graph);
    if (fo->cap_stream) (void)hipStreamDestroy(fo->cap_stream);
    delete fo;
    return BH_OK;
}

bh_status bh_forest_energy(bh_ctx *ctx, bh_forest *fo, double *out_KW) {
    if (!ctx || !fo || !out_KW) return bh_fail(BH_E_INVAL, "NULL argument");
    if (fo->F.ctx != ctx) return bh_fail(BH_E_INVAL, "handle created on another context, or its context was destroyed");
    bh_status st = bh_forest_eval(fo->F, fo->pos, fo->mass, fo->acc, fo->F.dev.pot, true, nullptr);
    if (st != BH_OK) return st;
    fo->have_acc = true;
    HIPCHK(launch_energy(fo->F.dev, fo->vel, fo->mass, fo->F.dev.pot, fo->F.dev.red, ctx->stream));
    HIPCHK(hipMemcpyAsync(out_KW, fo->F.dev.red, sizeof(double) * 2 * fo->F.seg.size(), hipMemcpyDeviceToHost,
                          ctx->stream));
    return bh_forest_check_err(fo->F);
}

// ---------------------------------------------------- initial conditions ---

// Workspace of bh_ic_generate: the generator's partial sums, then its fault word.
static size_t ic_flag_offset() { return (ic_scratch_bytes() + 255) & ~(size_t)255; }

size_t bh_ic_workspace_bytes(void) { return ic_flag_offset() + 256; }

bh_status bh_ic_generate(bh_ctx *ctx, int32_t kind, int64_t n, uint64_t seed, double a, double M, double *pos,
                         double *vel, double *mass, void *ws, size_t ws_bytes) {
    if (!ctx || !pos || !vel || !mass || !ws) return bh_fail(BH_E_INVAL, "NULL argument");
    if (((uintptr_t)ws & 255) != 0) return bh_fail(BH_E_INVAL, "workspace must be 256-byte aligned");
    if (ws_bytes < bh_ic_workspace_bytes())
        return bh_fail(BH_E_NOMEM, "workspace too small: need " + std::to_string(bh_ic_workspace_bytes()) + " bytes");
    if (kind != 0 && kind != 1) return bh_fail(BH_E_INVAL, "kind must be 0 (Plummer) or 1 (cube)");
    if (n < 1 || n > (int64_t)0x3fffffff) return bh_fail(BH_E_INVAL, "n out of range");
    if (!(a > 0.0) || !(M > 0.0) || !std::isfinite(a) || !std::isfinite(M))
        return bh_fail(BH_E_INVAL, "a and M must be positive and finite");
    uint32_t *flag = reinterpret_cast<uint32_t *>(static_cast<char *>(ws) + ic_flag_offset());
    HIPCHK(launch_fill_u32(flag, 0, 1, ctx->stream));
    HIPCHK(launch_ic(kind, n, seed, a, M, pos, vel, mass, static_cast<double *>(ws), flag, ctx->stream));
    uint32_t e = 0;
    HIPCHK(hipMemcpyAsync(&e, flag, sizeof(e), hipMemcpyDeviceToHost, ctx->stream));
    HIPCHK(hipStreamSynchronize(ctx->stream));
    if (e) return bh_fail(BH_E_DEVICE, "initial conditions: a velocity draw found no acceptance in 401 tries");
    return BH_OK;
}

bh_status bh_ic_generate_static(bh_ctx *ctx, int32_t kind, int64_t n, uint64_t seed, double a, double M,
                                double *pos, double *vel, double *mass) {
    if (!ctx || !pos || !vel || !mass) return bh_fail(BH_E_INVAL, "NULL argument");
    if (kind != 0 && kind != 1) return bh_fail(BH_E_INVAL, "kind must be 0 (Plummer) or 1 (cube)");
    if (n < 1 || n > (int64_t)0x3fffffff) return bh_fail(BH_E_INVAL, "n out of range (1 .. 2^30 - 1)");
    if (!(a > 0.0) || !(M > 0.0) || !std::isfinite(a) || !std::isfinite(M))
        return bh_fail(BH_E_INVAL, "a and M must be positive and finite");
    if (bh_ic_workspace_bytes() > kStaticScratchBytes)
        return bh_fail(BH_E_NOMEM, "the generator's scratch exceeds the static array (" +
                                       std::to_string(kStaticScratchBytes) + " bytes)");
    char *base = static_cast<char *>(static_scratch(ctx->device));
    if (!base) return bh_fail(BH_E_DEVICE, "no static scratch on this device (context not initialised)");
    uint32_t *flag = reinterpret_cast<uint32_t *>(base + ic_flag_offset());
    HIPCHK(launch_fill_u32(flag, 0, 1, ctx->stream));
    HIPCHK(launch_ic(kind, n, seed, a, M, pos, vel, mass, reinterpret_cast<double *>(base), flag, ctx->stream));
    return BH_OK;
}

}  // extern "C"
