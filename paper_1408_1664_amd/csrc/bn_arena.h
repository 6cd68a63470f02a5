// Chunked best-fit arena for the server's device workspaces.
//
// Requests get blocks carved from a few large chunks that the arena
// allocates rarely and keeps (a device allocation per request costs more
// than a small solve, and freeing device memory synchronises the device). A
// chunk is kChunk bytes, or one request when larger, and the chunks together
// stay within a byte limit (the server's memory budget). Free ranges of each
// chunk (offset -> length, multiples of the granule) are kept coalesced; a
// request takes the smallest free range that fits over every chunk. When
// none fits, a new chunk is allocated; when that would pass the limit or the
// allocation fails, chunks with nothing in use are released first. With no
// block in use every chunk is empty, so a request within the limit then
// always gets its block (if the device has the memory).
//
// Mem supplies the underlying memory: static bool alloc(size_t, void **)
// and static void release(void *). Plain C++: the server instantiates it
// with device memory, the host tests with a counting host allocator.
#pragma once
#include <stddef.h>

#include <algorithm>
#include <iterator>
#include <map>
#include <vector>

namespace bnk {

template <class Mem>
class Arena {
   public:
    static constexpr size_t kGranule = (size_t)2 << 20;
    static constexpr size_t kChunk = (size_t)4 << 30;
    explicit Arena(size_t limit, size_t chunk = kChunk) : limit_(limit), chunk_(chunk) {}
    ~Arena() {
        for (auto &c : chunks_) Mem::release(c.base);
    }
    Arena(const Arena &) = delete;
    Arena &operator=(const Arena &) = delete;

    // a block of at least bytes (rounded up to the granule); false if the
    // limit or the memory cannot provide it now
    bool get(size_t bytes, void **p, size_t *got) {
        const size_t need = (bytes + kGranule - 1) / kGranule * kGranule;
        bool ok = take(need, p) || (grow(need) && take(need, p));
        if (!ok) {
            release_empty();
            ok = grow(need) && take(need, p);
        }
        if (ok) *got = need;
        return ok;
    }
    // return a block of get(); bytes is the size get() reported
    void put(void *p, size_t bytes) {
        char *q = static_cast<char *>(p);
        for (auto &c : chunks_) {
            if (q < c.base || q >= c.base + c.size) continue;
            size_t off = (size_t)(q - c.base), len = bytes;
            auto next = c.free.lower_bound(off);
            if (next != c.free.end() && off + len == next->first) {   // merge with the next range
                len += next->second;
                next = c.free.erase(next);
            }
            if (next != c.free.begin()) {                             // and with the previous one
                auto prev = std::prev(next);
                if (prev->first + prev->second == off) {
                    prev->second += len;
                    return;
                }
            }
            c.free.emplace(off, len);
            return;
        }
    }
    size_t bytes_held() const {
        size_t t = 0;
        for (const auto &c : chunks_) t += c.size;
        return t;
    }
    size_t chunks() const { return chunks_.size(); }
    size_t free_ranges() const {
        size_t k = 0;
        for (const auto &c : chunks_) k += c.free.size();
        return k;
    }

   private:
    struct Chunk {
        char *base;
        size_t size;
        std::map<size_t, size_t> free;   // offset -> length
    };
    bool take(size_t need, void **p) {
        Chunk *bc = nullptr;
        std::map<size_t, size_t>::iterator best;
        for (auto &c : chunks_)
            for (auto it = c.free.begin(); it != c.free.end(); ++it)
                if (it->second >= need && (!bc || it->second < best->second)) {
                    bc = &c;
                    best = it;
                }
        if (!bc) return false;
        const size_t off = best->first, len = best->second;
        bc->free.erase(best);
        if (len > need) bc->free.emplace(off + need, len - need);
        *p = bc->base + off;
        return true;
    }
    bool grow(size_t need) {
        size_t size = std::max(need, std::min(chunk_, limit_));
        if (bytes_held() + size > limit_) size = need;
        if (bytes_held() + size > limit_) return false;
        void *b = nullptr;
        if (!Mem::alloc(size, &b)) return false;
        Chunk c{static_cast<char *>(b), size, {}};
        c.free.emplace(0, size);
        chunks_.push_back(std::move(c));
        return true;
    }
    void release_empty() {
        for (size_t k = 0; k < chunks_.size();) {
            Chunk &c = chunks_[k];
            if (c.free.size() == 1 && c.free.begin()->first == 0 && c.free.begin()->second == c.size) {
                Mem::release(c.base);
                chunks_.erase(chunks_.begin() + k);
            } else {
                ++k;
            }
        }
    }
    size_t limit_, chunk_;
    std::vector<Chunk> chunks_;
};

}  // namespace bnk
