// Host-only admission logic of the request loop: a first-fit arena over the server's
// device memory and FIFO admission into rounds of at most `max_round` frames.
// Nothing here touches a device, so it is exercised on the CPU by a plain C++ test.
#ifndef SSVB_SCHED_H
#define SSVB_SCHED_H

#include <stdint.h>

#include <deque>
#include <iterator>
#include <map>
#include <utility>
#include <vector>

namespace ssvb {

// First-fit allocator over [0, size): free blocks kept sorted by offset and merged with
// their neighbours on release; every block is a multiple of `align`.
class Arena {
public:
    explicit Arena(uint64_t size = 0, uint64_t align = 256) { reset(size, align); }

    void reset(uint64_t size, uint64_t align = 256) {
        align_ = align ? align : 1;
        size_ = size / align_ * align_;
        free_.clear();
        if (size_) free_[0] = size_;
        in_use_ = peak_ = 0;
    }

    uint64_t round_up(uint64_t n) const { return (n + align_ - 1) / align_ * align_; }

    // Lowest-offset free block that holds `bytes` (rounded up); false if none does.
    bool alloc(uint64_t bytes, uint64_t* off) {
        const uint64_t n = round_up(bytes ? bytes : 1);
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second < n) continue;
            const uint64_t o = it->first, len = it->second;
            free_.erase(it);
            if (len > n) free_[o + n] = len - n;
            in_use_ += n;
            if (in_use_ > peak_) peak_ = in_use_;
            *off = o;
            return true;
        }
        return false;
    }

    // Return a block obtained from alloc with the same `bytes`.
    void release(uint64_t off, uint64_t bytes) {
        uint64_t n = round_up(bytes ? bytes : 1);
        in_use_ -= n;
        auto next = free_.lower_bound(off);
        if (next != free_.end() && off + n == next->first) {  // merge with the block after
            n += next->second;
            next = free_.erase(next);
        }
        if (next != free_.begin()) {  // merge with the block before
            auto prev = std::prev(next);
            if (prev->first + prev->second == off) {
                prev->second += n;
                return;
            }
        }
        free_[off] = n;
    }

    uint64_t size() const { return size_; }
    uint64_t in_use() const { return in_use_; }
    uint64_t peak() const { return peak_; }
    uint64_t largest_free() const {
        uint64_t m = 0;
        for (const auto& b : free_) m = b.second > m ? b.second : m;
        return m;
    }
    size_t free_blocks() const { return free_.size(); }

    // Free blocks are disjoint, aligned, not adjacent, inside [0, size), and together
    // with the bytes in use cover the whole arena.
    bool check() const {
        uint64_t end = 0, total = 0;
        bool first = true;
        for (const auto& b : free_) {
            if (b.second == 0 || b.first % align_ || b.second % align_) return false;
            if (!first && b.first <= end) return false;  // overlapping or adjacent (unmerged)
            end = b.first + b.second;
            if (end > size_) return false;
            total += b.second;
            first = false;
        }
        return total + in_use_ == size_;
    }

private:
    std::map<uint64_t, uint64_t> free_;  // offset -> length
    uint64_t size_ = 0, align_ = 256, in_use_ = 0, peak_ = 0;
};

// FIFO admission: requests wait in arrival order; the head is admitted when its
// footprint fits in the arena (a later request never overtakes it, so large frames are
// not starved); admitted requests are handed out in rounds of at most `max_round`, in
// admission order; finishing a request returns its memory.
class Admission {
public:
    Admission(uint64_t arena_bytes = 0, int max_round = 64, uint64_t align = 256)
        : arena_(arena_bytes, align), max_round_(max_round > 0 ? max_round : 1) {}

    Arena& arena() { return arena_; }
    const Arena& arena() const { return arena_; }

    // Would a request of `bytes` ever fit?
    bool fits_at_all(uint64_t bytes) const { return arena_.round_up(bytes ? bytes : 1) <= arena_.size(); }

    void submit(uint64_t ticket, uint64_t bytes) { fifo_.push_back({ticket, bytes}); }

    // Admit from the head of the queue while it fits: appends (ticket, offset).
    int admit(std::vector<std::pair<uint64_t, uint64_t>>& out) {
        int n = 0;
        while (!fifo_.empty()) {
            uint64_t off = 0;
            if (!arena_.alloc(fifo_.front().second, &off)) break;
            const auto r = fifo_.front();
            fifo_.pop_front();
            resident_[r.first] = {off, r.second};
            ready_.push_back(r.first);
            out.push_back({r.first, off});
            ++n;
        }
        return n;
    }

    // Up to max_round admitted requests not yet in a round, oldest first.
    int take_round(std::vector<uint64_t>& out) {
        int n = 0;
        while (!ready_.empty() && n < max_round_) {
            out.push_back(ready_.front());
            ready_.pop_front();
            ++n;
        }
        return n;
    }

    // The request's round is over (or it was cancelled after admission): free its memory.
    bool finish(uint64_t ticket) {
        auto it = resident_.find(ticket);
        if (it == resident_.end()) return false;
        arena_.release(it->second.first, it->second.second);
        resident_.erase(it);
        return true;
    }

    // Drop every request still waiting for memory; returns their tickets.
    std::vector<uint64_t> cancel_queued() {
        std::vector<uint64_t> t;
        for (const auto& r : fifo_) t.push_back(r.first);
        fifo_.clear();
        return t;
    }

    // Drop every admitted request not yet in a round (memory is freed); returns tickets.
    std::vector<uint64_t> cancel_ready() {
        std::vector<uint64_t> t(ready_.begin(), ready_.end());
        ready_.clear();
        for (uint64_t k : t) finish(k);
        return t;
    }

    size_t queued() const { return fifo_.size(); }
    size_t ready() const { return ready_.size(); }
    size_t resident() const { return resident_.size(); }

private:
    Arena arena_;
    int max_round_;
    std::deque<std::pair<uint64_t, uint64_t>> fifo_;  // (ticket, bytes) waiting for memory
    std::deque<uint64_t> ready_;                      // admitted, not yet in a round
    std::map<uint64_t, std::pair<uint64_t, uint64_t>> resident_;  // ticket -> (offset, bytes)
};

}  // namespace ssvb

#endif
