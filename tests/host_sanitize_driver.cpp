// Exercises the library's host-only logic (workspace layouts, interaction-list
// buffer layouts, the server's first-fit arena and its first-come first-served
// admission, the tuning cache and its JSON reader) for a build under
// AddressSanitizer and UndefinedBehaviorSanitizer,
// and checks its invariants against plain reference models.  Test
// infrastructure: exit status 0 and "all cases ok" when every check holds.
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <deque>
#include <map>
#include <random>
#include <vector>

#include "../paper_1109_5190_amd/csrc/bh_host.h"

using namespace bh_host;

static int failures = 0;
#define CHECK(c)                                                          \
    do {                                                                  \
        if (!(c)) {                                                       \
            std::fprintf(stderr, "check failed at line %d: %s\n", __LINE__, #c); \
            ++failures;                                                   \
        }                                                                 \
    } while (0)

static void layouts(std::mt19937_64 &rng) {
    for (int t = 0; t < 2000; ++t) {
        std::vector<Region> r(1 + rng() % 48);
        for (auto &x : r) {
            x.count = (rng() % 4 == 0) ? 0 : rng() % 100000;
            x.elem = 1 + rng() % 64;
        }
        std::vector<size_t> off;
        size_t total = 0;
        CHECK(layout(r, off, total));
        size_t end = 0;
        for (size_t i = 0; i < r.size(); ++i) {
            CHECK(off[i] % kAlign == 0);
            CHECK(off[i] >= end);
            end = off[i] + r[i].count * r[i].elem;
        }
        CHECK(total >= end + kAlign - 1 && total % 1 == 0);
    }
    // sizes that overflow are refused, not wrapped
    std::vector<size_t> off;
    size_t total = 7;
    CHECK(!layout({{SIZE_MAX / 2, 4}}, off, total));
    CHECK(!layout({{SIZE_MAX / 16, 8}, {SIZE_MAX / 16, 8}, {SIZE_MAX / 16, 8}}, off, total));
    CHECK(total == 7);
    size_t a;
    CHECK(!align_up(SIZE_MAX - 3, a));
    CHECK(align_up(0, a) && a == 0);
    CHECK(align_up(1, a) && a == 256);
}

static void list_layouts(std::mt19937_64 &rng) {
    for (int t = 0; t < 3000; ++t) {
        const size_t ng = rng() % 200000;
        const size_t bytes = rng() % (size_t(1) << 30);
        const size_t c = list_chunks_for(ng, bytes);
        const ListLayout l = list_layout(ng, c);
        CHECK(l.head % kAlign == 0 && l.count % kAlign == 0 && l.next % kAlign == 0 && l.ent % kAlign == 0);
        CHECK(l.count >= l.head + 4 * ng && l.next >= l.count + 4 * ng && l.ent >= l.next + 4 * c);
        if (c > 0) CHECK(l.total <= bytes);
        if (c < 0xffffffffu && bytes > list_layout(ng, 0).total + kAlign)
            CHECK(list_layout(ng, c + 1).total > bytes - kAlign);
    }
}

// Arena against a bitmap of 256-byte units.
static void arena(std::mt19937_64 &rng) {
    for (int t = 0; t < 200; ++t) {
        const size_t base = (rng() % 64) * kAlign;
        const size_t units = 1 + rng() % 4096;
        const size_t bytes = units * kAlign + rng() % kAlign;   // a ragged tail is never handed out
        Arena A;
        A.init(base, bytes);
        CHECK(A.capacity() == units * kAlign);
        std::vector<char> used(units, 0);
        std::map<size_t, size_t> live;   // offset -> requested bytes
        for (int op = 0; op < 3000; ++op) {
            if (live.empty() || rng() % 3) {
                const size_t want = 1 + rng() % (units * kAlign / 4 + 1);
                size_t off = 0;
                if (A.alloc(want, off)) {
                    size_t b;
                    CHECK(align_up(want, b));
                    CHECK(off >= base && off % kAlign == 0 && off + b <= base + units * kAlign);
                    for (size_t u = (off - base) / kAlign; u < (off - base + b) / kAlign; ++u) {
                        CHECK(!used[u]);
                        used[u] = 1;
                    }
                    live[off] = want;
                } else {
                    // first fit: no free run of that many units exists
                    size_t b;
                    CHECK(align_up(want, b));
                    size_t run = 0, best = 0;
                    for (size_t u = 0; u < units; ++u) {
                        run = used[u] ? 0 : run + 1;
                        if (run > best) best = run;
                    }
                    CHECK(best * kAlign < b);
                }
            } else {
                auto it = live.begin();
                std::advance(it, (long)(rng() % live.size()));
                size_t b;
                CHECK(align_up(it->second, b));
                for (size_t u = (it->first - base) / kAlign; u < (it->first - base + b) / kAlign; ++u) used[u] = 0;
                A.release(it->first, it->second);
                live.erase(it);
            }
            size_t nfree = 0;
            for (char c : used) nfree += !c;
            CHECK(A.free_bytes() == nfree * kAlign);
            // free blocks never touch: they are merged on release
            size_t prev_end = SIZE_MAX;
            for (const auto &kv : A.blocks()) {
                CHECK(kv.first != prev_end);
                prev_end = kv.first + kv.second;
            }
        }
        for (const auto &kv : live) A.release(kv.first, kv.second);
        CHECK(A.blocks().size() == 1 && A.free_bytes() == units * kAlign);
    }
}

static void admission(std::mt19937_64 &rng) {
    for (int t = 0; t < 300; ++t) {
        Arena A;
        const size_t cap = (1 + rng() % 512) * kAlign;
        A.init(0, cap);
        const Caps caps{(int32_t)(1 + rng() % 8), (int64_t)(1 + rng() % 100000)};
        std::map<uint64_t, Queued> reqs;
        std::deque<uint64_t> q;
        for (uint64_t id = 1; id <= 40; ++id) {
            Queued r{(int64_t)(1 + rng() % 40000), (size_t)(1 + rng() % (cap / 2 + 1)), rng() % 7 == 0};
            if (never_fits(r.n, r.bytes, caps, A)) continue;   // refused at submission
            reqs[id] = r;
            q.push_back(id);
        }
        int32_t slots = (int32_t)(rng() % 2);
        int64_t resident = (int64_t)(rng() % 1000);
        if (resident > caps.max_resident) resident = caps.max_resident;
        const std::deque<uint64_t> before = q;
        const int32_t s0 = slots;
        const int64_t r0 = resident;
        const auto got = admit_fcfs(q, [&](uint64_t id) { return reqs.at(id); }, caps, slots, resident, A);
        // admitted requests are the non-cancelled ones of a prefix of the queue, in order
        size_t k = 0, i = 0;
        int64_t adds = 0;
        for (; i < before.size() && k < got.size(); ++i) {
            const Queued &r = reqs.at(before[i]);
            if (r.cancelled) continue;
            CHECK(got[k].first == before[i]);
            adds += r.n;
            ++k;
        }
        CHECK(k == got.size());
        CHECK(slots == s0 + (int32_t)got.size() && resident == r0 + adds);
        CHECK(slots <= caps.max_slots || got.empty());
        CHECK(resident <= caps.max_resident || got.empty());
        // the queue keeps the rest, starting at the first request that did not fit
        while (i < before.size() && reqs.at(before[i]).cancelled) ++i;
        if (!q.empty()) {
            CHECK(q.front() == before[i]);
            CHECK(!reqs.at(q.front()).cancelled);
        }
        // admitted blocks are disjoint
        std::vector<std::pair<size_t, size_t>> blk;
        for (const auto &g : got) blk.push_back({g.second, reqs.at(g.first).bytes});
        for (size_t a = 0; a < blk.size(); ++a)
            for (size_t b = a + 1; b < blk.size(); ++b) {
                size_t ea, eb;
                align_up(blk[a].second, ea);
                align_up(blk[b].second, eb);
                CHECK(blk[a].first + ea <= blk[b].first || blk[b].first + eb <= blk[a].first);
            }
    }
    // a request of exactly the arena's capacity fits an empty arena; one byte more never does
    Arena A;
    A.init(4096, 10 * kAlign + 17);
    const Caps caps{4, 1000};
    CHECK(!never_fits(10, 10 * kAlign, caps, A));
    CHECK(never_fits(10, 10 * kAlign + 1, caps, A));
    CHECK(never_fits(1001, 256, caps, A));
    std::map<uint64_t, Queued> reqs{{1, {10, 10 * kAlign, false}}};
    std::deque<uint64_t> q{1};
    int32_t slots = 0;
    int64_t resident = 0;
    const auto got = admit_fcfs(q, [&](uint64_t id) { return reqs.at(id); }, caps, slots, resident, A);
    CHECK(got.size() == 1 && got[0].second == 4096 && q.empty());
}

static TuneKey random_key(std::mt19937_64 &rng) {
    static const char *devs[] = {"gfx950:256", "gfx942:304", "a\"b\\c", "tab\there"};
    static const char *precs[] = {"fp32", "fp64", "mixed"};
    TuneKey k;
    k.device = devs[rng() % 4];
    k.n_log2 = (int)(rng() % 63);
    k.sims_log2 = (int)(rng() % 32);
    k.theta_c = (int)(rng() % 1000001);
    k.precision = precs[rng() % 3];
    return k;
}

static void tune_cache(std::mt19937_64 &rng) {
    static const int shapes[] = {1, 2, 4, 8, 0x101, 0x102, 0x104, 0x108};
    // round trips: what is written reads back as the same entries
    for (int t = 0; t < 300; ++t) {
        TuneCache c;
        std::map<TuneKey, TuneEntry> model;
        const int n = (int)(rng() % 20);
        for (int i = 0; i < n; ++i) {
            const TuneKey k = random_key(rng);
            const TuneEntry e{shapes[rng() % 8], (double)(rng() % 100000) / 8.0};
            c.put(k, e);
            model[k] = e;
        }
        CHECK(c.size() == model.size());
        TuneCache d;
        std::string err;
        CHECK(d.merge_json(c.to_json(), err));
        CHECK(d.size() == model.size());
        for (const auto &kv : model) {
            TuneEntry e;
            CHECK(d.find(kv.first, e) && e.shape == kv.second.shape && std::fabs(e.ms - kv.second.ms) <= 1e-5 * (1 + kv.second.ms));
        }
        // mutated texts: parse or refuse, never read out of bounds; a refusal leaves the cache as it was
        const std::string text = c.to_json();
        for (int m = 0; m < 40; ++m) {
            std::string x = text;
            const int kind = (int)(rng() % 4);
            if (x.empty()) break;
            const size_t at = rng() % x.size();
            if (kind == 0) x[at] = (char)(rng() % 256);
            else if (kind == 1) x.erase(at, 1 + rng() % 8);
            else if (kind == 2) x.insert(at, 1, "{}[]\",:\\0e-9tn"[rng() % 14]);
            else x.resize(at);
            TuneCache e = d;
            const size_t before = e.size();
            std::string er;
            if (!e.merge_json(x, er)) {
                CHECK(e.size() == before && !er.empty());
            }
        }
    }
    // schema errors are refused with the cache unchanged
    const char *bad[] = {
        "", "[]", "{}", "null", "{\"format\": \"bh-tune-cache\", \"version\": 2, \"entries\": []}",
        "{\"format\": \"other\", \"version\": 1, \"entries\": []}",
        "{\"format\": \"bh-tune-cache\", \"version\": 1, \"entries\": {}}",
        "{\"format\": \"bh-tune-cache\", \"version\": 1, \"entries\": [], \"x\": 1}",
        "{\"format\": \"bh-tune-cache\", \"version\": 1, \"entries\": [{\"device\": \"g\", \"n_log2\": 3, "
        "\"sims_log2\": 0, \"theta\": 0.5, \"precision\": \"fp32\", \"shape\": 3, \"ms\": 1}]}",
        "{\"format\": \"bh-tune-cache\", \"version\": 1, \"entries\": [{\"device\": \"g\", \"n_log2\": 3.5, "
        "\"sims_log2\": 0, \"theta\": 0.5, \"precision\": \"fp32\", \"shape\": 4, \"ms\": 1}]}",
        "{\"format\": \"bh-tune-cache\", \"version\": 1, \"entries\": [{\"device\": \"g\", \"n_log2\": 3, "
        "\"sims_log2\": 0, \"theta\": 0.5, \"precision\": \"fp16\", \"shape\": 4, \"ms\": 1}]}",
        "{\"format\": \"bh-tune-cache\", \"version\": 1, \"entries\": [{\"device\": \"g\", \"n_log2\": 3, "
        "\"sims_log2\": 0, \"theta\": 0.5, \"precision\": \"fp32\", \"shape\": 4, \"ms\": -1}]}",
        "{\"format\": \"bh-tune-cache\", \"version\": 1, \"entries\": [{\"device\": \"g\", \"n_log2\": 3, "
        "\"sims_log2\": 0, \"theta\": 0.5, \"precision\": \"fp32\", \"shape\": -1e300, \"ms\": 1}]}",
        "{\"format\": \"bh-tune-cache\", \"version\": 1, \"version\": 1, \"entries\": []}",
        "{\"format\": \"bh-tune-cache\", \"version\": 1, \"entries\": [1e999]}",
        "[[[[[[[[[[[[[[[[[[[[[[[[[[[[[[[[[[[[[[[[[]]]]]]]]]]]]]]]]]]]]]]]]]]]]]]]]]]]]]]]]]",
    };
    TuneCache c;
    c.put(TuneKey{"gfx950:256", 20, 0, 50, "fp32"}, TuneEntry{4, 2.5});
    for (const char *b : bad) {
        std::string err;
        CHECK(!c.merge_json(b, err));
        CHECK(c.size() == 1 && !err.empty());
    }
    std::string err;
    CHECK(c.merge_json("{\"format\": \"bh-tune-cache\", \"version\": 1, \"entries\": []}", err) && c.size() == 1);
    CHECK(valid_shape(0x104) && !valid_shape(0x200) && !valid_shape(3) && !valid_shape(-4) && !valid_shape(0));
    CHECK(floor_log2(0) == 0 && floor_log2(1) == 0 && floor_log2(1048576) == 20 && floor_log2(1048575) == 19);
}

int main() {
    std::mt19937_64 rng(20260201);
    layouts(rng);
    list_layouts(rng);
    arena(rng);
    admission(rng);
    tune_cache(rng);
    if (failures) {
        std::fprintf(stderr, "%d checks failed\n", failures);
        return 1;
    }
    std::printf("all cases ok\n");
    return 0;
}
