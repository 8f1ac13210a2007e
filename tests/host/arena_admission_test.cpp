// CPU test of the serving loop's host bookkeeping (paper_1707_05062_amd/csrc/kohler_arena.h): the
// image arena's first-fit allocator and in-order admission, driven by a stub executor that stands
// in for the GPU (launches "complete" when the test says so). Built with g++ under AddressSanitizer
// and UndefinedBehaviorSanitizer by tests/test_host_sanitizers.py; exits non-zero on a failure.
#include <cstdio>
#include <cstdlib>
#include <random>
#include <unordered_map>

#include "kohler_arena.h"

using kohler::Arena;
using kohler::kAlign;

static int failures = 0;
#define CHECK(cond)                                                          \
    do {                                                                     \
        if (!(cond)) {                                                       \
            std::fprintf(stderr, "%s:%d: check failed: %s\n", __FILE__, __LINE__, #cond); \
            ++failures;                                                      \
        }                                                                    \
    } while (0)

struct Req {
    bool on_device = false;
    size_t bytes = 0;
    unsigned char *labels = nullptr;
    bool labels_on_device = false;
    int64_t H = 1, W = 1;
    int slot = -1;
    bool has_arena = false, has_label_block = false;
    size_t arena_off = 0, label_off = 0;
};

// Arena: first fit, 256-byte blocks, merging of free neighbours, peak tracking.
static void test_arena() {
    Arena a;
    a.reset(4096);
    size_t o1, o2, o3, o4;
    CHECK(a.alloc(1, &o1) && o1 == 0);          // rounded up to one block
    CHECK(a.alloc(300, &o2) && o2 == 256);      // two blocks
    CHECK(a.alloc(256, &o3) && o3 == 768);
    CHECK(a.used() == 1024 && a.peak() == 1024);
    a.release(o2, 300);                          // hole [256, 768)
    CHECK(a.alloc(512, &o4) && o4 == 256);      // first fit reuses the hole
    a.release(o4, 512);
    a.release(o1, 1);
    a.release(o3, 256);                          // everything merges back into one range
    CHECK(a.used() == 0);
    size_t big;
    CHECK(a.alloc(4096, &big) && big == 0);      // only possible if the free ranges merged
    CHECK(!a.alloc(1, &o1));                     // full
    a.release(big, 4096);
    // random alloc/release against a shadow map of blocks: no overlap, always inside [0, cap)
    std::mt19937 rng(7);
    std::map<size_t, size_t> live;
    a.reset(1 << 20);
    for (int step = 0; step < 20000; ++step) {
        if (live.empty() || rng() % 3) {
            const size_t n = 1 + rng() % 20000;
            size_t off;
            if (a.alloc(n, &off)) {
                const size_t len = kohler::round_up(n, kAlign);
                CHECK(off % kAlign == 0 && off + len <= a.capacity());
                auto next = live.lower_bound(off);
                if (next != live.end()) CHECK(off + kohler::round_up(next->second, kAlign) > off && off + len <= next->first);
                if (next != live.begin()) {
                    auto prev = std::prev(next);
                    CHECK(prev->first + kohler::round_up(prev->second, kAlign) <= off);
                }
                live[off] = n;
            }
        } else {
            auto it = live.begin();
            std::advance(it, rng() % live.size());
            a.release(it->first, it->second);
            live.erase(it);
        }
    }
    for (auto &kv : live) a.release(kv.first, kv.second);
    CHECK(a.used() == 0);
    size_t all;
    CHECK(a.alloc(1 << 20, &all) && all == 0);
}

// Admission order with a stub executor: requests are admitted in arrival order; a host image that
// does not fit blocks the ones behind it; slots and max_batch bound a launch; blocks return on
// completion and the waiting head is admitted next.
static void test_admission() {
    std::unordered_map<uint64_t, Req> reqs;
    std::deque<uint64_t> queue;
    Arena arena;
    arena.reset(10 * kAlign);
    std::vector<int> free_slots = {3, 2, 1, 0};
    auto get = [&](uint64_t t) -> Req & { return reqs.at(t); };
    auto add = [&](uint64_t t, size_t bytes, bool on_device, bool host_labels = false, int64_t H = 1, int64_t W = 1) {
        Req r;
        r.bytes = bytes;
        r.on_device = on_device;
        static unsigned char dummy[1];
        if (host_labels) r.labels = dummy;
        r.H = H;
        r.W = W;
        reqs[t] = r;
        queue.push_back(t);
    };
    add(1, 3 * kAlign, false);
    add(2, 6 * kAlign, false);
    add(3, 5 * kAlign, false);  // does not fit after 1 and 2 (1 block left)
    add(4, 1, false);           // would fit, but must not overtake 3
    add(5, 1 << 30, true);      // on the device: needs no arena
    std::vector<uint64_t> out;
    kohler::admit_in_order(queue, get, arena, free_slots, 8, out);
    CHECK(out.size() == 2 && out[0] == 1 && out[1] == 2);
    CHECK(queue.size() == 3 && queue.front() == 3);
    CHECK(reqs[1].has_arena && reqs[2].has_arena && reqs[1].arena_off != reqs[2].arena_off);
    CHECK(reqs[1].slot == 0 && reqs[2].slot == 1);
    // stub executor: request 1's launch completes, its block and slot come back
    arena.release(reqs[1].arena_off, reqs[1].bytes);
    free_slots.push_back(reqs[1].slot);
    out.clear();
    kohler::admit_in_order(queue, get, arena, free_slots, 8, out);
    CHECK(out.empty());  // 3 needs 5 blocks, 4 are free
    arena.release(reqs[2].arena_off, reqs[2].bytes);
    free_slots.push_back(reqs[2].slot);
    out.clear();
    kohler::admit_in_order(queue, get, arena, free_slots, 2, out);  // max_batch 2
    CHECK(out.size() == 2 && out[0] == 3 && out[1] == 4 && queue.size() == 1);
    out.clear();
    kohler::admit_in_order(queue, get, arena, free_slots, 8, out);
    CHECK(out.size() == 1 && out[0] == 5 && !reqs[5].has_arena);
    CHECK(free_slots.size() == 1);
    // labels to host memory take a block of H * W bytes of their own; when it does not fit, the
    // image block taken for the same request is given back
    arena.release(reqs[3].arena_off, reqs[3].bytes);
    arena.release(reqs[4].arena_off, reqs[4].bytes);
    CHECK(arena.used() == 0);
    free_slots = {0};
    add(6, 8 * kAlign, false, true, 4, 200);  // image 8 blocks + labels 800 bytes = 4 blocks > 10
    out.clear();
    kohler::admit_in_order(queue, get, arena, free_slots, 8, out);
    CHECK(out.empty() && arena.used() == 0 && !reqs[6].has_arena && !reqs[6].has_label_block);
    queue.clear();
    add(7, 5 * kAlign, false, true, 4, 200);
    kohler::admit_in_order(queue, get, arena, free_slots, 8, out);
    CHECK(out.size() == 1 && reqs[7].has_arena && reqs[7].has_label_block && arena.used() == 9 * kAlign);
    // no slot: nothing admitted
    add(8, 1, true);
    out.clear();
    kohler::admit_in_order(queue, get, arena, free_slots, 8, out);
    CHECK(out.empty() && queue.size() == 1);
}

int main() {
    test_arena();
    test_admission();
    if (failures) {
        std::fprintf(stderr, "%d check(s) failed\n", failures);
        return 1;
    }
    std::printf("arena and admission: ok\n");
    return 0;
}
