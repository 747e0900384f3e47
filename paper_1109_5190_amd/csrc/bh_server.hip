// Continuous-batching request server.
//
// Requests (n particles, steps, initial-condition kind and seed, parameters)
// are queued first-come first-served.  A server thread owns a HIP stream and
// loops: admit queued requests while the slot count, the resident-particle cap
// and the caller's arena allow; generate their initial conditions on the
// device; advance every resident simulation by one iteration of one forest
// launch sequence; retire the ones that finished.  Simulations at different
// step indices share the iteration through per-simulation phase bits:
//   a newly admitted one only evaluates a(x0) and applies the first half-kick;
//   a running one drifts, is re-evaluated, takes its second half-kick and, if
//   steps remain, the first half-kick of its next step.
// The arithmetic and its order per simulation are those of bh_step, so a
// request's result does not depend on what else was resident.
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <deque>
#include <map>
#include <mutex>
#include <new>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "bh.h"
#include "bh_common.h"
#include "bh_host.h"
#include "bh_internal.h"

using namespace bh;

namespace {

enum { kQueued = 0, kRunning = 1, kDone = 2, kFailed = 3, kCancelled = 4 };
constexpr uint32_t kReqReleaseAtEnd = 1u;   // bh_params.flags bit: free the state when done (no fetch)

size_t align256(size_t v) { return (v + 255) & ~(size_t)255; }

struct Req {
    uint64_t id = 0;
    bh_request r{};
    int state = kQueued;
    int steps_done = 0;
    double t_submit = 0, t_admit = 0, t_done = 0, K = 0, W = 0;
    size_t off = 0, bytes = 0;
    bool has_mem = false, fresh = false, cancel = false, fetching = false;
    double *pos = nullptr, *vel = nullptr, *acc = nullptr, *mass = nullptr, *pot = nullptr;
};

size_t state_bytes(int64_t n) { return align256((size_t)n * 11 * sizeof(double)); }

}  // namespace

struct bh_server {
    bh_ctx *ctx = nullptr;
    hipStream_t stream = nullptr;
    hipStream_t fetch_stream = nullptr;   // copies of finished requests, apart from the iterations
    bh_ctx sctx;                 // the server's own context (its stream)
    char *arena = nullptr;
    size_t arena_bytes = 0, ws_bytes = 0;
    double *scratch = nullptr;   // initial-condition reductions (partial sums)
    int32_t max_slots = 0;
    int64_t max_resident = 0;
    ForestHost F;
    bh_host::Arena mem;
    std::mutex mu;
    std::condition_variable cv;
    std::deque<uint64_t> queue;
    std::unordered_map<uint64_t, Req> reqs;
    std::vector<uint64_t> resident;
    int64_t resident_particles = 0;
    uint64_t next_id = 1;
    bool stop = false;
    std::string fault;
    std::thread th;
    std::chrono::steady_clock::time_point t0;

    double now() const {
        return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    }
    void loop();
    bool iterate(std::vector<uint64_t> &ids);
};

bool bh_server::iterate(std::vector<uint64_t> &ids) {
    // tables of this iteration's membership (state pointers per simulation)
    std::vector<int64_t> ns;
    std::vector<bh_params> ps;
    std::vector<Req *> rs;
    {
        std::lock_guard<std::mutex> lk(mu);
        for (uint64_t id : ids) {
            Req &q = reqs[id];
            rs.push_back(&q);
            ns.push_back(q.r.n);
            ps.push_back(q.r.p);
        }
    }
    const int32_t nseg = (int32_t)rs.size();
    bh_forest_tables(F, nseg, ns.data(), ps.data());
    bool any_finish = false;
    std::vector<bool> finish(nseg, false);
    for (int32_t s = 0; s < nseg; ++s) {
        Req &q = *rs[s];
        SegDesc &d = F.seg[s];
        d.pos = q.pos;
        d.mass = q.mass;
        d.vel = q.vel;
        d.acc = q.acc;
        d.dt = q.r.dt;
        uint32_t ph = 0;
        if (q.fresh) {
            if (q.r.steps > 0) ph |= kPhaseKick1;
            else finish[s] = true;
        } else {
            ph |= kPhaseDrift | kPhaseKick2;
            if (q.steps_done + 1 < q.r.steps) ph |= kPhaseKick1;
            else finish[s] = true;
        }
        d.phase = ph;
        d.pot = finish[s] ? q.pot : nullptr;
        any_finish |= finish[s];
    }
    if (bh_forest_upload_tables(F) != BH_OK) return false;
    hipStream_t s = stream;
    const ForestDev &D = F.dev;
    if (launch_drift(D, nullptr, nullptr, kPhaseDrift, s) != hipSuccess) return false;
    if (launch_build(D, nullptr, nullptr, s) != hipSuccess) return false;
    if (launch_upward(D, s) != hipSuccess) return false;
    if (launch_walk(D, false, any_finish, nullptr, nullptr, nullptr, nullptr, nullptr, s, F.walk_shape) != hipSuccess) return false;
    if (launch_kick(D, nullptr, nullptr, kPhaseKick2, s) != hipSuccess) return false;
    if (launch_kick(D, nullptr, nullptr, kPhaseKick1, s) != hipSuccess) return false;
    std::vector<double> kw(2 * (size_t)nseg, 0.0);
    if (any_finish) {
        if (launch_energy(D, nullptr, nullptr, nullptr, D.red, s) != hipSuccess) return false;
        if (hipMemcpyAsync(kw.data(), D.red, sizeof(double) * kw.size(), hipMemcpyDeviceToHost, s) != hipSuccess)
            return false;
    }
    uint32_t e = 0;
    if (hipMemcpyAsync(&e, D.err, sizeof(uint32_t), hipMemcpyDeviceToHost, s) != hipSuccess) return false;
    if (hipStreamSynchronize(s) != hipSuccess) return false;
    if (e) return false;
    const double t = now();
    std::lock_guard<std::mutex> lk(mu);
    std::vector<uint64_t> keep;
    for (int32_t k = 0; k < nseg; ++k) {
        Req &q = *rs[k];
        if (q.fresh) q.fresh = false;
        else q.steps_done++;
        if (finish[k]) {
            q.state = kDone;
            q.t_done = t;
            q.K = kw[2 * k];
            q.W = kw[2 * k + 1];
            resident_particles -= q.r.n;
            if (q.r.p.flags & kReqReleaseAtEnd) {
                mem.release(q.off, q.bytes);
                q.has_mem = false;
            }
        } else if (q.cancel) {
            q.state = kCancelled;
            resident_particles -= q.r.n;
            mem.release(q.off, q.bytes);
            q.has_mem = false;
        } else {
            keep.push_back(q.id);
        }
    }
    resident.swap(keep);
    cv.notify_all();
    return true;
}

void bh_server::loop() {
    (void)hipSetDevice(ctx->device);
    for (;;) {
        std::vector<uint64_t> fresh, ids;
        {
            std::unique_lock<std::mutex> lk(mu);
            for (;;) {
                // admission, first come first served: stop at the first request that does not fit
                int32_t slots = (int32_t)resident.size();
                const auto admitted = bh_host::admit_fcfs(
                    queue,
                    [this](uint64_t id) {
                        const Req &q = reqs[id];
                        return bh_host::Queued{q.r.n, q.bytes, q.state == kCancelled};
                    },
                    bh_host::Caps{max_slots, max_resident}, slots, resident_particles, mem);
                for (const auto &ad : admitted) {
                    Req &q = reqs[ad.first];
                    q.off = ad.second;
                    q.has_mem = true;
                    char *b = arena + q.off;
                    const size_t n = (size_t)q.r.n;
                    q.pos = (double *)b;
                    q.vel = q.pos + 3 * n;
                    q.acc = q.vel + 3 * n;
                    q.mass = q.acc + 3 * n;
                    q.pot = q.mass + n;
                    q.state = kRunning;
                    q.t_admit = now();
                    q.fresh = true;
                    resident.push_back(q.id);
                    fresh.push_back(q.id);
                }
                if (!resident.empty()) break;
                if (stop) return;
                cv.wait_for(lk, std::chrono::milliseconds(2));
            }
            ids = resident;
        }
        // the error word covers this iteration only: initial conditions, tree, walk
        bool ok = launch_fill_u32(F.dev.err, 0, 64, stream) == hipSuccess;
        for (uint64_t id : fresh) {
            Req *q;
            {
                std::lock_guard<std::mutex> lk(mu);
                q = &reqs[id];
            }
            if (ok && launch_ic(q->r.ic_kind, q->r.n, q->r.seed, 1.0, 1.0, q->pos, q->vel, q->mass, scratch,
                                F.dev.err, stream) != hipSuccess)
                ok = false;
        }
        if (ok) ok = iterate(ids);
        if (!ok) {
            std::lock_guard<std::mutex> lk(mu);
            fault = "device error or fault flag (non-finite state, generator failure, inconsistent tree) "
                    "in a server iteration";
            for (uint64_t id : ids) {
                Req &q = reqs[id];
                q.state = kFailed;
                q.t_done = now();
                if (q.has_mem) {
                    mem.release(q.off, q.bytes);
                    q.has_mem = false;
                }
            }
            resident.clear();
            resident_particles = 0;
            cv.notify_all();
        }
    }
}

extern "C" {

bh_status bh_server_create(bh_ctx *ctx, void *arena, size_t arena_bytes, int32_t max_slots,
                           int64_t max_resident_particles, bh_server **out) {
    if (!ctx || !arena || !out) return bh_fail(BH_E_INVAL, "NULL argument");
    if (((uintptr_t)arena & 255) != 0) return bh_fail(BH_E_INVAL, "arena must be 256-byte aligned");
    if (max_slots < 1 || max_resident_particles < 1 || max_resident_particles > (int64_t)0x3fffffff)
        return bh_fail(BH_E_INVAL, "bad slot or particle cap");
    bh_server *sv = new (std::nothrow) bh_server();
    if (!sv) return bh_fail(BH_E_NOMEM, "host allocation failed");
    sv->ctx = ctx;
    sv->arena = (char *)arena;
    sv->arena_bytes = arena_bytes;
    sv->max_slots = max_slots;
    sv->max_resident = max_resident_particles;
    ForestCaps cap;
    cap.nseg = (uint32_t)max_slots;
    cap.ntot = (uint32_t)max_resident_particles;
    cap.ntiles = (uint32_t)(max_resident_particles / kTile + max_slots + 1);
    cap.ngroups = (uint32_t)(max_resident_particles / kGroup + max_slots + 1);
    cap.fp32 = cap.fp64 = true;
    cap.quad = true;
    cap.group = true;
    size_t ws = bh_forest_carve(sv->F, cap, nullptr);
    const size_t scratch_bytes = align256(ic_scratch_bytes());
    if (ws == 0 || ws + scratch_bytes >= arena_bytes) {
        delete sv;
        return bh_fail(BH_E_NOMEM, "arena too small for the tree workspace: need more than " +
                                       std::to_string(ws + scratch_bytes) + " bytes");
    }
    bh_forest_carve(sv->F, cap, (char *)arena);
    sv->ws_bytes = align256(ws);
    sv->scratch = (double *)(sv->arena + sv->ws_bytes);
    sv->mem.init(sv->ws_bytes + scratch_bytes, arena_bytes - sv->ws_bytes - scratch_bytes);
    hipError_t e = hipSetDevice(ctx->device);
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&sv->stream, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&sv->fetch_stream, hipStreamNonBlocking);
    if (e != hipSuccess) {
        if (sv->stream) (void)hipStreamDestroy(sv->stream);
        delete sv;
        return bh_fail(BH_E_DEVICE, std::string("stream creation: ") + hipGetErrorString(e));
    }
    sv->sctx.device = ctx->device;
    sv->sctx.stream = sv->stream;
    sv->F.ctx = &sv->sctx;
    e = launch_fill_u32(sv->F.dev.err, 0, 64, sv->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(sv->stream);
    if (e != hipSuccess) {
        (void)hipStreamDestroy(sv->stream);
        (void)hipStreamDestroy(sv->fetch_stream);
        delete sv;
        return bh_fail(BH_E_DEVICE, std::string("server init: ") + hipGetErrorString(e));
    }
    sv->t0 = std::chrono::steady_clock::now();
    sv->th = std::thread([sv] { sv->loop(); });
    *out = sv;
    return BH_OK;
}

bh_status bh_server_submit(bh_server *sv, const bh_request *req, uint64_t *id) {
    if (!sv || !req || !id) return bh_fail(BH_E_INVAL, "NULL argument");
    if (req->n < 1 || req->steps < 0 || (req->ic_kind != 0 && req->ic_kind != 1) || !std::isfinite(req->dt))
        return bh_fail(BH_E_INVAL, "bad request");
    bh_status st = bh_check_params(&req->p);
    if (st != BH_OK) return st;
    const size_t bytes = state_bytes(req->n);
    if (bh_host::never_fits(req->n, bytes, bh_host::Caps{sv->max_slots, sv->max_resident}, sv->mem))
        return bh_fail(BH_E_NOMEM, "request can never fit the server's arena or particle cap");
    std::lock_guard<std::mutex> lk(sv->mu);
    if (sv->stop) return bh_fail(BH_E_INVAL, "server is shutting down");
    Req q;
    q.id = sv->next_id++;
    q.r = *req;
    q.bytes = bytes;
    q.t_submit = sv->now();
    sv->reqs[q.id] = q;
    sv->queue.push_back(q.id);
    *id = q.id;
    sv->cv.notify_all();
    return BH_OK;
}

bh_status bh_server_poll(bh_server *sv, uint64_t id, bh_result *res) {
    if (!sv) return bh_fail(BH_E_INVAL, "NULL argument");
    std::lock_guard<std::mutex> lk(sv->mu);
    auto it = sv->reqs.find(id);
    if (it == sv->reqs.end()) return bh_fail(BH_E_NOTFOUND, "unknown request id");
    const Req &q = it->second;
    if (res) {
        res->state = q.state;
        res->steps_done = q.steps_done;
        res->t_submit = q.t_submit;
        res->t_admit = q.t_admit;
        res->t_done = q.t_done;
        res->K = q.K;
        res->W = q.W;
    }
    if (q.state == kDone) return BH_OK;
    if (q.state == kCancelled) return bh_fail(BH_E_CANCELLED, "request was cancelled");
    if (q.state == kFailed) return bh_fail(BH_E_DEVICE, sv->fault.empty() ? "request failed" : sv->fault);
    return BH_E_BUSY;
}

bh_status bh_server_fetch(bh_server *sv, uint64_t id, double *pos, double *vel) {
    if (!sv) return bh_fail(BH_E_INVAL, "NULL argument");
    const double *src_pos = nullptr, *src_vel = nullptr;
    size_t bytes3 = 0;
    {
        std::lock_guard<std::mutex> lk(sv->mu);
        auto it = sv->reqs.find(id);
        if (it == sv->reqs.end()) return bh_fail(BH_E_NOTFOUND, "unknown request id");
        Req &q = it->second;
        if (q.state == kQueued || q.state == kRunning) return bh_fail(BH_E_BUSY, "request not finished");
        if (q.state != kDone) return bh_fail(BH_E_INVAL, "request did not complete");
        if (!q.has_mem || q.fetching) return bh_fail(BH_E_INVAL, "request state was released (or already fetched)");
        q.fetching = true;   // the state stays allocated until the copies are done
        src_pos = q.pos;
        src_vel = q.vel;
        bytes3 = sizeof(double) * 3 * (size_t)q.r.n;
    }
    // a finished request's state is written by no later iteration: copy it on a stream of
    // its own, without waiting for the iteration in flight and without holding the lock
    hipError_t e = hipSuccess;
    if (pos) e = hipMemcpyAsync(pos, src_pos, bytes3, hipMemcpyDefault, sv->fetch_stream);
    if (e == hipSuccess && vel) e = hipMemcpyAsync(vel, src_vel, bytes3, hipMemcpyDefault, sv->fetch_stream);
    if (e == hipSuccess) e = hipStreamSynchronize(sv->fetch_stream);
    std::lock_guard<std::mutex> lk(sv->mu);
    Req &q = sv->reqs[id];
    q.fetching = false;
    if (e != hipSuccess) return bh_fail(BH_E_DEVICE, std::string("fetch copy: ") + hipGetErrorString(e));
    sv->mem.release(q.off, q.bytes);
    q.has_mem = false;
    sv->cv.notify_all();
    return BH_OK;
}

bh_status bh_server_cancel(bh_server *sv, uint64_t id) {
    if (!sv) return bh_fail(BH_E_INVAL, "NULL argument");
    std::lock_guard<std::mutex> lk(sv->mu);
    auto it = sv->reqs.find(id);
    if (it == sv->reqs.end()) return bh_fail(BH_E_NOTFOUND, "unknown request id");
    Req &q = it->second;
    if (q.state == kQueued) q.state = kCancelled;
    else if (q.state == kRunning) q.cancel = true;
    return BH_OK;
}

double bh_server_now(bh_server *sv) { return sv ? sv->now() : 0.0; }

bh_status bh_server_destroy(bh_server *sv) {
    if (!sv) return BH_OK;
    {
        std::lock_guard<std::mutex> lk(sv->mu);
        sv->stop = true;
        sv->cv.notify_all();
    }
    if (sv->th.joinable()) sv->th.join();
    (void)hipStreamSynchronize(sv->stream);
    (void)hipStreamDestroy(sv->stream);
    (void)hipStreamSynchronize(sv->fetch_stream);
    (void)hipStreamDestroy(sv->fetch_stream);
    delete sv;
    return BH_OK;
}

}  // extern "C"
