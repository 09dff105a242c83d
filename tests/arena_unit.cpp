// Unit checks of the serving loop's host bookkeeping (gom_arena.h), built with g++ by
// tests/test_host_units.py.  Prints "ok" and exits 0 when every check holds.
#include "gom_arena.h"

#include <cstdio>
#include <cstdlib>
#include <random>
#include <set>
#include <stdexcept>
#include <vector>

using gom::ArenaBlocks;

#define CHECK(c)                                                             \
    do {                                                                     \
        if (!(c)) {                                                          \
            std::fprintf(stderr, "check failed at line %d: %s\n", __LINE__, #c); \
            std::exit(1);                                                    \
        }                                                                    \
    } while (0)

struct Job {
    int id;
    bool retired;
};

static void allocator_basics() {
    ArenaBlocks a(4096 + 100);  // rounded down to whole 256-byte units
    CHECK(a.total() == 4096 && a.free_bytes() == 4096 && a.free_blocks() == 1);
    size_t o1, o2, o3, o4;
    CHECK(a.alloc(1, &o1) && o1 == 0);          // rounds up to 256
    CHECK(a.alloc(300, &o2) && o2 == 256);      // 512
    CHECK(a.alloc(1024, &o3) && o3 == 768);
    CHECK(a.free_bytes() == 4096 - 256 - 512 - 1024);
    CHECK(!a.alloc(4096, &o4));                 // too large: nothing changes
    CHECK(a.free_bytes() == 4096 - 1792);
    a.release(o2, 300);                         // hole [256, 768)
    CHECK(a.free_blocks() == 2);
    CHECK(a.alloc(512, &o4) && o4 == 256);      // first fit takes the hole
    a.release(o4, 512);
    a.release(o1, 1);                           // merges with the hole: [0, 768)
    CHECK(a.free_blocks() == 2 && a.largest_free() == 4096 - 1792);
    a.release(o3, 1024);                        // merges both sides: one block again
    CHECK(a.free_blocks() == 1 && a.free_bytes() == 4096 && a.largest_free() == 4096);
}

// Random allocations and frees against a byte map: blocks never overlap, stay inside the
// arena, and all frees restore one block.
static void allocator_random() {
    const size_t total = 1 << 20;
    ArenaBlocks a(total);
    std::vector<unsigned char> owner(total / 256, 0);
    struct Live { size_t off, size; };
    std::vector<Live> live;
    std::mt19937_64 rng(7);
    for (int it = 0; it < 20000; ++it) {
        if (live.empty() || rng() % 3 != 0) {
            const size_t want = 1 + rng() % (48 * 1024);
            size_t off;
            const size_t before = a.free_bytes();
            if (a.alloc(want, &off)) {
                const size_t units = (want + 255) / 256;
                CHECK(off % 256 == 0 && off + units * 256 <= total);
                for (size_t u = off / 256; u < off / 256 + units; ++u) {
                    CHECK(owner[u] == 0);
                    owner[u] = 1;
                }
                CHECK(a.free_bytes() == before - units * 256);
                live.push_back({off, want});
            } else {
                CHECK(a.largest_free() < ((want + 255) & ~size_t(255)));
            }
        } else {
            const size_t k = rng() % live.size();
            const Live l = live[k];
            live.erase(live.begin() + (long)k);
            const size_t units = (l.size + 255) / 256;
            for (size_t u = l.off / 256; u < l.off / 256 + units; ++u) owner[u] = 0;
            a.release(l.off, l.size);
        }
        size_t used = 0;
        for (unsigned char o : owner) used += o;
        CHECK(a.free_bytes() == total - used * 256);
    }
    for (const Live &l : live) a.release(l.off, l.size);
    CHECK(a.free_blocks() == 1 && a.free_bytes() == total);
}

// A pass that retires some jobs and then ends early (an error return or an exception) still
// removes exactly the retired ones, in order.
static int pass(std::vector<Job> &active, const std::set<int> &finish, int fail_at, bool thrw) {
    gom::RetiredSweep<Job> sweep{active};
    for (Job &j : active) {
        if (j.id == fail_at) {
            if (thrw) throw std::runtime_error("device");
            return -5;
        }
        if (finish.count(j.id)) j.retired = true;
    }
    return 0;
}

static void retire_bookkeeping() {
    std::vector<Job> active;
    for (int i = 0; i < 8; ++i) active.push_back({i, false});
    CHECK(pass(active, {1, 3, 6}, 5, false) == -5);     // 1 and 3 retired before the error
    CHECK(active.size() == 6);
    const int want1[] = {0, 2, 4, 5, 6, 7};
    for (size_t k = 0; k < active.size(); ++k) CHECK(active[k].id == want1[k]);
    bool caught = false;
    try {
        pass(active, {0, 7}, 6, true);                  // 0 retired, exception at 6
    } catch (const std::exception &) {
        caught = true;
    }
    CHECK(caught && active.size() == 5);
    const int want2[] = {2, 4, 5, 6, 7};
    for (size_t k = 0; k < active.size(); ++k) CHECK(active[k].id == want2[k]);
    CHECK(pass(active, {2, 4, 5, 6, 7}, -1, false) == 0 && active.empty());
}

int main() {
    allocator_basics();
    allocator_random();
    retire_bookkeeping();
    std::printf("ok\n");
    return 0;
}
