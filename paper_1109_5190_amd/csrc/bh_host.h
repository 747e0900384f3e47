// Host-only logic of the library, free of HIP types so that it also builds with a
// plain C++ compiler (and its sanitizers): the layout of a workspace as aligned
// regions, the server's first-fit arena over byte offsets, and its first-come
// first-served admission of queued requests.
#pragma once
#include <cstddef>
#include <cstdint>
#include <deque>
#include <iterator>
#include <map>
#include <utility>
#include <vector>

namespace bh_host {

constexpr size_t kAlign = 256;

// Rounds v up to a multiple of 256; false when that overflows.
inline bool align_up(size_t v, size_t &out) {
    if (v > SIZE_MAX - (kAlign - 1)) return false;
    out = (v + kAlign - 1) & ~(kAlign - 1);
    return true;
}

// One region of a workspace: `count` elements of `elem` bytes (count 0: absent).
struct Region {
    size_t count, elem;
};

// Offsets of `r` laid out in order, each 256-byte aligned, and the total
// (the end of the last region plus one alignment unit of slack).  Returns false
// (total untouched) when a size overflows size_t.
inline bool layout(const std::vector<Region> &r, std::vector<size_t> &off, size_t &total) {
    off.assign(r.size(), 0);
    size_t at = 0;
    for (size_t i = 0; i < r.size(); ++i) {
        if (!align_up(at, at)) return false;
        off[i] = at;
        if (r[i].elem && r[i].count > SIZE_MAX / r[i].elem) return false;
        const size_t b = r[i].count * r[i].elem;
        if (b > SIZE_MAX - at) return false;
        at += b;
    }
    if (at > SIZE_MAX - kAlign) return false;
    total = at + kAlign;
    return true;
}

// Layout of an interaction-list buffer: 256 chunk counters 256 bytes apart, then
// per group its first chunk and entry count, per chunk its successor, then the
// entries (64 per chunk, 16 bytes each), each table 256-byte aligned.
constexpr size_t kListPartitions = 256, kListEntryBytes = 16, kListChunk = 64;
struct ListLayout {
    size_t head, count, next, ent, total;
};

inline ListLayout list_layout(size_t ngroups, size_t nchunks) {
    ListLayout l;
    l.head = 256 * kListPartitions;
    align_up(l.head + 4 * ngroups, l.count);
    align_up(l.count + 4 * ngroups, l.next);
    align_up(l.next + 4 * nchunks, l.ent);
    l.total = l.ent + kListEntryBytes * kListChunk * nchunks;
    return l;
}

// Largest chunk count whose layout fits in `bytes` (0 also when not even the tables
// fit), at most 2^32 - 1.
inline size_t list_chunks_for(size_t ngroups, size_t bytes) {
    const size_t fixed = list_layout(ngroups, 0).total;
    if (bytes <= fixed + kAlign) return 0;
    size_t c = (bytes - fixed - kAlign) / (4 + kListEntryBytes * kListChunk);
    if (c > 0xffffffffu) c = 0xffffffffu;
    while (c > 0 && list_layout(ngroups, c).total > bytes) --c;
    return c;
}

// First-fit allocator over byte offsets of an arena (bookkeeping only: it never
// touches the arena's memory).  Sizes are rounded up to 256 bytes.
class Arena {
public:
    void init(size_t off, size_t bytes) {
        free_.clear();
        cap_ = 0;
        size_t b = bytes & ~(kAlign - 1);   // whole units only
        if (b) free_[off] = b;
        cap_ = b;
    }
    // Largest block a request can ever get (the whole arena when it is empty).
    size_t capacity() const { return cap_; }
    bool alloc(size_t bytes, size_t &off) {
        if (!align_up(bytes, bytes) || bytes == 0) return false;
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second >= bytes) {
                off = it->first;
                const size_t rest = it->second - bytes;
                free_.erase(it);
                if (rest) free_[off + bytes] = rest;
                return true;
            }
        }
        return false;
    }
    // Returns a block obtained from alloc (same size); neighbouring free blocks merge.
    void release(size_t off, size_t bytes) {
        if (!align_up(bytes, bytes) || bytes == 0) return;
        auto it = free_.emplace(off, bytes).first;
        auto nx = std::next(it);
        if (nx != free_.end() && it->first + it->second == nx->first) {
            it->second += nx->second;
            free_.erase(nx);
        }
        if (it != free_.begin()) {
            auto pv = std::prev(it);
            if (pv->first + pv->second == it->first) {
                pv->second += it->second;
                free_.erase(it);
            }
        }
    }
    size_t free_bytes() const {
        size_t s = 0;
        for (const auto &kv : free_) s += kv.second;
        return s;
    }
    const std::map<size_t, size_t> &blocks() const { return free_; }

private:
    std::map<size_t, size_t> free_;   // offset -> bytes
    size_t cap_ = 0;
};

// Server caps a request is admitted against.
struct Caps {
    int32_t max_slots;
    int64_t max_resident;
};

// A request that can never be admitted: more particles than the resident cap,
// or a state larger than the arena's whole capacity.
inline bool never_fits(int64_t n, size_t bytes, const Caps &c, const Arena &mem) {
    size_t b;
    return n > c.max_resident || !align_up(bytes, b) || b > mem.capacity();
}

struct Queued {
    int64_t n;
    size_t bytes;
    bool cancelled;
};

// First-come first-served admission: takes requests from the front of `queue`
// (ids, looked up by get(id) -> Queued) while the slot count, the resident-particle
// cap and the arena allow; cancelled requests are dropped from the queue; stops at
// the first request that does not fit.  Returns the admitted (id, arena offset)
// pairs in order and updates the resident counts.
template <class Get>
std::vector<std::pair<uint64_t, size_t>> admit_fcfs(std::deque<uint64_t> &queue, Get get, const Caps &c,
                                                    int32_t &slots_used, int64_t &resident, Arena &mem) {
    std::vector<std::pair<uint64_t, size_t>> out;
    while (!queue.empty()) {
        const uint64_t id = queue.front();
        const Queued q = get(id);
        if (q.cancelled) {
            queue.pop_front();
            continue;
        }
        if (slots_used >= c.max_slots || resident + q.n > c.max_resident) break;
        size_t off;
        if (!mem.alloc(q.bytes, off)) break;
        out.emplace_back(id, off);
        ++slots_used;
        resident += q.n;
        queue.pop_front();
    }
    return out;
}

}  // namespace bh_host
