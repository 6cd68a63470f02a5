// Host checks of the server's workspace arena (bn_arena.h) over a counting
// host allocator; prints one line per check and exits nonzero on a failure.
#include <cstdio>
#include <cstdlib>
#include <set>

#include "../../paper_1408_1664_amd/csrc/bn_arena.h"

namespace {
int g_allocs = 0, g_live = 0, g_fail_next = 0;
std::set<void *> g_blocks;
struct HostMem {
    static bool alloc(size_t bytes, void **p) {
        if (g_fail_next > 0) {
            --g_fail_next;
            return false;
        }
        *p = std::malloc(bytes);   // never touched: only its address range matters
        if (!*p) return false;
        ++g_allocs;
        ++g_live;
        g_blocks.insert(*p);
        return true;
    }
    static void release(void *p) {
        if (!g_blocks.erase(p)) std::abort();
        std::free(p);
        --g_live;
    }
};
using A = bnk::Arena<HostMem>;
constexpr size_t MiB = (size_t)1 << 20;
int failures = 0;
void check(bool ok, const char *what) {
    std::printf("%s %s\n", ok ? "ok  " : "FAIL", what);
    if (!ok) ++failures;
}
}  // namespace

int main() {
    {   // rounding, one chunk for several blocks, coalescing back to one range
        A a(1024 * MiB, 64 * MiB);
        void *p1, *p2, *p3;
        size_t g1, g2, g3;
        check(a.get(1, &p1, &g1) && g1 == 2 * MiB, "a 1-byte request takes one 2 MiB granule");
        check(a.get(5 * MiB, &p2, &g2) && g2 == 6 * MiB, "5 MiB rounds up to 6 MiB");
        check(a.get(8 * MiB, &p3, &g3) && g3 == 8 * MiB, "8 MiB stays 8 MiB");
        check(a.chunks() == 1 && g_allocs == 1 && a.bytes_held() == 64 * MiB,
              "the three blocks share one 64 MiB chunk");
        check(static_cast<char *>(p2) == static_cast<char *>(p1) + 2 * MiB &&
                  static_cast<char *>(p3) == static_cast<char *>(p2) + 6 * MiB,
              "blocks are carved in address order");
        a.put(p1, g1);
        a.put(p3, g3);
        check(a.free_ranges() == 2, "two separated free ranges");
        a.put(p2, g2);
        check(a.free_ranges() == 1, "returning the middle block coalesces both neighbours");
    }
    check(g_live == 0, "the arena releases its chunks when destroyed");
    {   // best fit over the free ranges
        A a(1024 * MiB, 64 * MiB);
        void *p[5];
        size_t g[5];
        const size_t sz[5] = {6, 2, 4, 2, 30};
        for (int k = 0; k < 5; ++k) a.get(sz[k] * MiB, &p[k], &g[k]);
        a.put(p[0], g[0]);   // a 6 MiB hole
        a.put(p[2], g[2]);   // a 4 MiB hole
        void *q;
        size_t gq;
        check(a.get(4 * MiB, &q, &gq) && q == p[2], "a 4 MiB request takes the 4 MiB hole");
        void *r;
        size_t gr;
        check(a.get(3 * MiB, &r, &gr) && r == p[0], "a 3 MiB request takes the 6 MiB hole");
        check(a.chunks() == 1, "no new chunk while a hole fits");
    }
    {   // the limit: chunks never exceed it, a request waits for returns
        A a(8 * MiB, 64 * MiB);
        void *p1, *p2;
        size_t g1, g2;
        check(a.get(6 * MiB, &p1, &g1) && a.bytes_held() == 8 * MiB,
              "under a limit below the chunk size the chunk is the limit");
        check(!a.get(4 * MiB, &p2, &g2), "a request beyond what the limit leaves is refused");
        a.put(p1, g1);
        check(a.get(4 * MiB, &p2, &g2), "after the return it is served");
        check(a.bytes_held() <= 8 * MiB, "the arena never holds more than the limit");
    }
    {   // empty chunks give way to a larger request
        A a(100 * MiB, 40 * MiB);
        void *p1, *p2, *p3;
        size_t g1, g2, g3;
        a.get(30 * MiB, &p1, &g1);
        a.get(30 * MiB, &p2, &g2);   // a second 40 MiB chunk
        check(a.chunks() == 2 && a.bytes_held() == 80 * MiB, "two chunks of 40 MiB");
        a.put(p1, g1);
        a.put(p2, g2);
        check(a.get(90 * MiB, &p3, &g3) && a.chunks() == 1 && a.bytes_held() == 90 * MiB,
              "a 90 MiB request releases the empty chunks and gets a chunk of its own");
        a.put(p3, g3);
    }
    {   // an allocation failure of the memory itself
        A a(1024 * MiB, 64 * MiB);
        void *p1;
        size_t g1;
        g_fail_next = 2;   // the first grow and the one after releasing empty chunks
        check(!a.get(4 * MiB, &p1, &g1) && a.chunks() == 0, "a failing allocation is reported");
        check(a.get(4 * MiB, &p1, &g1), "the next request succeeds");
        a.put(p1, g1);
    }
    check(g_live == 0, "no chunk outlives its arena");
    return failures == 0 ? 0 : 1;
}
