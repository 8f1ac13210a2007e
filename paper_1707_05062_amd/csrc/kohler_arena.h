// Host-side admission bookkeeping of the serving loop (kohler_server.cpp): the image arena's
// first-fit allocator and the in-order admission of queued requests. Plain C++ with no HIP
// dependency, so that it can also be built and tested on the CPU under sanitizers. Not installed.
#pragma once

#include <algorithm>
#include <cstddef>
#include <cstdint>
#include <deque>
#include <iterator>
#include <map>
#include <vector>

namespace kohler {

constexpr size_t kAlign = 256;

inline size_t round_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

// First-fit allocator over the byte range [0, cap) of the image arena; blocks are multiples of
// 256 bytes and free neighbours are merged.
class Arena {
public:
    void reset(size_t cap) {
        cap_ = cap;
        used_ = peak_ = 0;
        free_.clear();
        if (cap) free_[0] = cap;
    }
    size_t capacity() const { return cap_; }
    size_t used() const { return used_; }
    size_t peak() const { return peak_; }
    bool alloc(size_t bytes, size_t *off) {
        bytes = round_up(std::max<size_t>(bytes, 1), kAlign);
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second < bytes) continue;
            const size_t start = it->first, rest = it->second - bytes;
            free_.erase(it);
            if (rest) free_[start + bytes] = rest;
            *off = start;
            used_ += bytes;
            peak_ = std::max(peak_, used_);
            return true;
        }
        return false;
    }
    void release(size_t off, size_t bytes) {
        bytes = round_up(std::max<size_t>(bytes, 1), kAlign);
        used_ -= bytes;
        auto next = free_.lower_bound(off);
        if (next != free_.end() && off + bytes == next->first) {
            bytes += next->second;
            next = free_.erase(next);
        }
        if (next != free_.begin()) {
            auto prev = std::prev(next);
            if (prev->first + prev->second == off) {
                prev->second += bytes;
                return;
            }
        }
        free_[off] = bytes;
    }

private:
    size_t cap_ = 0, used_ = 0, peak_ = 0;
    std::map<size_t, size_t> free_;  // offset -> length
};

// Admission of the head of the queue into one launch, in arrival order: a request is admitted when a
// slot is free and, for an image in host memory, its copy fits the arena (and, for labels going to
// host memory, their block too); the first request that does not fit stops the admission (later,
// smaller requests do not overtake it). At most max_batch requests. `get(ticket)` returns the
// request, whose fields on_device, bytes, labels, labels_on_device, H, W are read and slot,
// has_arena, arena_off, has_label_block, label_off are set. Admitted tickets are appended to `out`
// and removed from the queue.
template <class Get>
void admit_in_order(std::deque<uint64_t> &queue, Get get, Arena &arena, std::vector<int> &free_slots, int max_batch,
                    std::vector<uint64_t> &out) {
    while (!queue.empty() && (int)out.size() < max_batch && !free_slots.empty()) {
        const uint64_t t = queue.front();
        auto &r = get(t);
        size_t off = 0, loff = 0;
        const bool need_img = !r.on_device, need_lab = r.labels && !r.labels_on_device;
        if (need_img && !arena.alloc(r.bytes, &off)) break;  // the head waits for arena room
        if (need_lab && !arena.alloc((size_t)(r.H * r.W), &loff)) {
            if (need_img) arena.release(off, r.bytes);
            break;
        }
        if (need_img) {
            r.has_arena = true;
            r.arena_off = off;
        }
        if (need_lab) {
            r.has_label_block = true;
            r.label_off = loff;
        }
        r.slot = free_slots.back();
        free_slots.pop_back();
        out.push_back(t);
        queue.pop_front();
    }
}

}  // namespace kohler
