// Host-only logic of the library, free of HIP types so that it also builds with a
// plain C++ compiler (and its sanitizers): the layout of a workspace as aligned
// regions, the server's first-fit arena over byte offsets, its first-come
// first-served admission of queued requests, and the autotuner's cache of walk
// launch shapes with its JSON form.
#pragma once
#include <cmath>
#include <cstddef>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <deque>
#include <iterator>
#include <map>
#include <memory>
#include <string>
#include <tuple>
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

// ------------------------------------------------------------ tuning cache ---

// Walk launch shapes: wavefronts per workgroup (1, 2, 4, 8) in the low byte, bit
// 0x100 for the persistent form.
constexpr int kShapePersistent = 0x100;
inline bool valid_shape(long s) {
    if (s < 0 || (s & ~(long)(0xff | kShapePersistent))) return false;
    const long w = s & 0xff;
    return w == 1 || w == 2 || w == 4 || w == 8;
}

// What a tuned shape is kept for: the device (architecture and compute units), the
// size class floor(log2 bodies) and floor(log2 simulations), theta (the body-weighted
// mean, in hundredths) and the precision mix ("fp32", "fp64" or "mixed").
struct TuneKey {
    std::string device;
    int n_log2 = 0, sims_log2 = 0, theta_c = 0;
    std::string precision;
    bool operator<(const TuneKey &o) const {
        return std::tie(device, n_log2, sims_log2, theta_c, precision) <
               std::tie(o.device, o.n_log2, o.sims_log2, o.theta_c, o.precision);
    }
};

struct TuneEntry {
    int shape = 4;
    double ms = 0.0;   // the walk time it was chosen with
};

inline int floor_log2(uint64_t v) {
    int k = -1;
    while (v) {
        v >>= 1;
        ++k;
    }
    return k < 0 ? 0 : k;
}

// A parsed JSON value (objects keep their members in order; no duplicates allowed).
struct JVal {
    enum Kind { Null, Bool, Num, Str, Arr, Obj } kind = Null;
    bool b = false;
    double num = 0.0;
    std::string str;
    std::vector<JVal> arr;
    std::vector<std::pair<std::string, JVal>> obj;
};

// Strict recursive-descent JSON reader with a nesting limit; false (with a message)
// on any syntax error.  Strings take the escapes \" \\ \/ \b \f \n \r \t and \u00XX.
class JReader {
public:
    JReader(const std::string &t) : t_(t) {}
    bool parse(JVal &v, std::string &err) {
        if (!value(v, 0)) {
            err = msg_ + " at byte " + std::to_string(i_);
            return false;
        }
        ws();
        if (i_ != t_.size()) {
            err = "trailing characters at byte " + std::to_string(i_);
            return false;
        }
        return true;
    }

private:
    const std::string &t_;
    size_t i_ = 0;
    std::string msg_;
    static constexpr int kDepth = 16;
    bool fail(const char *m) {
        msg_ = m;
        return false;
    }
    void ws() {
        while (i_ < t_.size() && (t_[i_] == ' ' || t_[i_] == '\t' || t_[i_] == '\n' || t_[i_] == '\r')) ++i_;
    }
    bool lit(const char *w) {
        size_t k = 0;
        while (w[k]) {
            if (i_ + k >= t_.size() || t_[i_ + k] != w[k]) return fail("bad literal");
            ++k;
        }
        i_ += k;
        return true;
    }
    static int hex(char c) {
        if (c >= '0' && c <= '9') return c - '0';
        if (c >= 'a' && c <= 'f') return c - 'a' + 10;
        if (c >= 'A' && c <= 'F') return c - 'A' + 10;
        return -1;
    }
    bool string(std::string &out) {
        if (i_ >= t_.size() || t_[i_] != '"') return fail("expected a string");
        ++i_;
        out.clear();
        while (i_ < t_.size()) {
            const char c = t_[i_++];
            if (c == '"') return true;
            if ((unsigned char)c < 0x20) return fail("control character in a string");
            if (c != '\\') {
                out.push_back(c);
                continue;
            }
            if (i_ >= t_.size()) break;
            const char e = t_[i_++];
            switch (e) {
                case '"': out.push_back('"'); break;
                case '\\': out.push_back('\\'); break;
                case '/': out.push_back('/'); break;
                case 'b': out.push_back('\b'); break;
                case 'f': out.push_back('\f'); break;
                case 'n': out.push_back('\n'); break;
                case 'r': out.push_back('\r'); break;
                case 't': out.push_back('\t'); break;
                case 'u': {
                    if (i_ + 4 > t_.size()) return fail("short \\u escape");
                    int v = 0;
                    for (int k = 0; k < 4; ++k) {
                        const int h = hex(t_[i_ + k]);
                        if (h < 0) return fail("bad \\u escape");
                        v = 16 * v + h;
                    }
                    if (v > 0x7f) return fail("only ASCII \\u escapes are accepted");
                    out.push_back((char)v);
                    i_ += 4;
                    break;
                }
                default: return fail("bad escape");
            }
        }
        return fail("unterminated string");
    }
    bool number(double &out) {
        const size_t b = i_;
        if (i_ < t_.size() && t_[i_] == '-') ++i_;
        if (i_ >= t_.size() || !(t_[i_] >= '0' && t_[i_] <= '9')) return fail("bad number");
        if (t_[i_] == '0') ++i_;
        else while (i_ < t_.size() && t_[i_] >= '0' && t_[i_] <= '9') ++i_;
        if (i_ < t_.size() && t_[i_] == '.') {
            ++i_;
            if (i_ >= t_.size() || !(t_[i_] >= '0' && t_[i_] <= '9')) return fail("bad fraction");
            while (i_ < t_.size() && t_[i_] >= '0' && t_[i_] <= '9') ++i_;
        }
        if (i_ < t_.size() && (t_[i_] == 'e' || t_[i_] == 'E')) {
            ++i_;
            if (i_ < t_.size() && (t_[i_] == '+' || t_[i_] == '-')) ++i_;
            if (i_ >= t_.size() || !(t_[i_] >= '0' && t_[i_] <= '9')) return fail("bad exponent");
            while (i_ < t_.size() && t_[i_] >= '0' && t_[i_] <= '9') ++i_;
        }
        out = std::strtod(t_.substr(b, i_ - b).c_str(), nullptr);
        if (!std::isfinite(out)) return fail("number out of range");
        return true;
    }
    bool value(JVal &v, int depth) {
        if (depth > kDepth) return fail("nesting too deep");
        ws();
        if (i_ >= t_.size()) return fail("unexpected end");
        const char c = t_[i_];
        if (c == '{') {
            ++i_;
            v.kind = JVal::Obj;
            ws();
            if (i_ < t_.size() && t_[i_] == '}') {
                ++i_;
                return true;
            }
            for (;;) {
                ws();
                std::string k;
                if (!string(k)) return false;
                for (const auto &m : v.obj)
                    if (m.first == k) return fail("duplicate key");
                ws();
                if (i_ >= t_.size() || t_[i_] != ':') return fail("expected ':'");
                ++i_;
                JVal m;
                if (!value(m, depth + 1)) return false;
                v.obj.emplace_back(std::move(k), std::move(m));
                ws();
                if (i_ < t_.size() && t_[i_] == ',') {
                    ++i_;
                    continue;
                }
                if (i_ < t_.size() && t_[i_] == '}') {
                    ++i_;
                    return true;
                }
                return fail("expected ',' or '}'");
            }
        }
        if (c == '[') {
            ++i_;
            v.kind = JVal::Arr;
            ws();
            if (i_ < t_.size() && t_[i_] == ']') {
                ++i_;
                return true;
            }
            for (;;) {
                JVal m;
                if (!value(m, depth + 1)) return false;
                v.arr.push_back(std::move(m));
                ws();
                if (i_ < t_.size() && t_[i_] == ',') {
                    ++i_;
                    continue;
                }
                if (i_ < t_.size() && t_[i_] == ']') {
                    ++i_;
                    return true;
                }
                return fail("expected ',' or ']'");
            }
        }
        if (c == '"') {
            v.kind = JVal::Str;
            return string(v.str);
        }
        if (c == 't' || c == 'f') {
            v.kind = JVal::Bool;
            v.b = c == 't';
            return lit(v.b ? "true" : "false");
        }
        if (c == 'n') {
            v.kind = JVal::Null;
            return lit("null");
        }
        v.kind = JVal::Num;
        return number(v.num);
    }
};

inline std::string json_string(const std::string &s) {
    std::string o = "\"";
    for (const char c : s) {
        if (c == '"' || c == '\\') {
            o.push_back('\\');
            o.push_back(c);
        } else if ((unsigned char)c < 0x20) {
            char b[8];
            std::snprintf(b, sizeof b, "\\u%04x", (unsigned)(unsigned char)c);
            o += b;
        } else {
            o.push_back(c);
        }
    }
    return o + "\"";
}

// The autotuner's cache.  JSON form:
//   {"format": "bh-tune-cache", "version": 1, "entries": [
//     {"device": "gfx950:256", "n_log2": 20, "sims_log2": 0, "theta": 0.5,
//      "precision": "fp32", "shape": 4, "ms": 2.77}, ...]}
class TuneCache {
public:
    bool find(const TuneKey &k, TuneEntry &e) const {
        auto it = m_.find(k);
        if (it == m_.end()) return false;
        e = it->second;
        return true;
    }
    void put(const TuneKey &k, const TuneEntry &e) { m_[k] = e; }
    size_t size() const { return m_.size(); }
    void clear() { m_.clear(); }

    std::string to_json() const {
        std::string o = "{\"format\": \"bh-tune-cache\", \"version\": 1, \"entries\": [";
        bool first = true;
        for (const auto &kv : m_) {
            char num[160];
            std::snprintf(num, sizeof num,
                          ", \"n_log2\": %d, \"sims_log2\": %d, \"theta\": %.2f, \"precision\": ", kv.first.n_log2,
                          kv.first.sims_log2, kv.first.theta_c / 100.0);
            char tail[96];
            std::snprintf(tail, sizeof tail, ", \"shape\": %d, \"ms\": %.6g}", kv.second.shape, kv.second.ms);
            o += first ? "\n  " : ",\n  ";
            o += "{\"device\": " + json_string(kv.first.device) + num + json_string(kv.first.precision) + tail;
            first = false;
        }
        return o + "\n]}\n";
    }

    // Adds the entries of `text` (replacing equal keys).  All or nothing: on any
    // syntax or schema error the cache is unchanged and `err` says why.
    bool merge_json(const std::string &text, std::string &err) {
        JVal root;
        if (!JReader(text).parse(root, err)) return false;
        if (root.kind != JVal::Obj) return bad(err, "top level is not an object");
        const JVal *fmt = member(root, "format"), *ver = member(root, "version"), *ents = member(root, "entries");
        if (!fmt || fmt->kind != JVal::Str || fmt->str != "bh-tune-cache") return bad(err, "not a bh-tune-cache file");
        if (!ver || ver->kind != JVal::Num || ver->num != 1.0) return bad(err, "unsupported version");
        if (!ents || ents->kind != JVal::Arr) return bad(err, "entries is not an array");
        if (root.obj.size() != 3) return bad(err, "unknown top-level key");
        std::vector<std::pair<TuneKey, TuneEntry>> add;
        for (const JVal &e : ents->arr) {
            if (e.kind != JVal::Obj || e.obj.size() != 7) return bad(err, "an entry needs exactly its 7 keys");
            const JVal *dv = member(e, "device"), *nl = member(e, "n_log2"), *sl = member(e, "sims_log2"),
                       *th = member(e, "theta"), *pr = member(e, "precision"), *sh = member(e, "shape"),
                       *ms = member(e, "ms");
            if (!dv || dv->kind != JVal::Str || dv->str.empty() || dv->str.size() > 128)
                return bad(err, "bad device");
            if (!int_in(nl, 0, 62) || !int_in(sl, 0, 31)) return bad(err, "bad size class");
            if (!th || th->kind != JVal::Num || !(th->num >= 0.0) || th->num > 1.0e4) return bad(err, "bad theta");
            if (!pr || pr->kind != JVal::Str || (pr->str != "fp32" && pr->str != "fp64" && pr->str != "mixed"))
                return bad(err, "bad precision");
            if (!sh || sh->kind != JVal::Num || sh->num != std::floor(sh->num) || sh->num < 0.0 || sh->num > 1e6 ||
                !valid_shape((long)sh->num))
                return bad(err, "bad shape");
            if (!ms || ms->kind != JVal::Num || !(ms->num >= 0.0)) return bad(err, "bad ms");
            TuneKey k;
            k.device = dv->str;
            k.n_log2 = (int)nl->num;
            k.sims_log2 = (int)sl->num;
            k.theta_c = (int)std::lround(th->num * 100.0);
            k.precision = pr->str;
            add.push_back({k, TuneEntry{(int)sh->num, ms->num}});
        }
        for (const auto &kv : add) m_[kv.first] = kv.second;
        return true;
    }

private:
    std::map<TuneKey, TuneEntry> m_;
    static bool bad(std::string &err, const char *m) {
        err = m;
        return false;
    }
    static const JVal *member(const JVal &o, const char *k) {
        for (const auto &m : o.obj)
            if (m.first == k) return &m.second;
        return nullptr;
    }
    static bool int_in(const JVal *v, int lo, int hi) {
        return v && v->kind == JVal::Num && v->num == std::floor(v->num) && v->num >= lo && v->num <= hi;
    }
};

}  // namespace bh_host
