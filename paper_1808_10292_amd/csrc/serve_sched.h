// Admission and batching policy of the sort server (host code only, no HIP):
// which queued requests start next, on which stream slot, grouped how.
//
//   - A request's footprint is the HBM it occupies while in flight (its key
//     buffers plus the workspace of its sort).  The sum over requests in
//     flight never exceeds the cap; a request larger than the cap is refused
//     at submission.
//   - Requests are admitted in arrival order.  When the oldest waiting request
//     does not fit in the remaining memory, or no stream slot is free,
//     admission stops (no later request overtakes a waiting one, except as
//     below), and resumes when a running batch completes.
//   - A small request (n <= small_max) at the head opens a batch that also
//     takes every later queued small request of the same key type, in arrival
//     order, while the batch size limit and the memory cap allow: one launch
//     sorts them all.  A large request runs alone in its slot.
#pragma once

#include <stddef.h>
#include <stdint.h>

#include <deque>
#include <vector>

namespace rsort {

struct ServeRequest {
    uint64_t ticket = 0;
    int key_type = 0;        // 0 = u32, 1 = u64
    uint64_t n = 0;
    uint64_t footprint = 0;  // bytes of HBM while in flight
    double t_submit = 0.0;   // seconds, host clock
    const void* keys_in = nullptr;
    void* keys_out = nullptr;
    void* ready = nullptr;   // event the request's sort waits for (opaque here)
};

struct ServeBatch {
    int slot = -1;
    bool small = false;
    int key_type = 0;
    uint64_t footprint = 0;
    std::vector<ServeRequest> reqs;
};

class ServeScheduler {
public:
    ServeScheduler(uint64_t cap_bytes, int num_slots, uint64_t small_max, size_t max_batch)
        : cap_(cap_bytes), small_max_(small_max), max_batch_(max_batch ? max_batch : 1),
          slot_busy_(num_slots > 0 ? num_slots : 1, false), slot_fp_(slot_busy_.size(), 0)
    {
    }

    bool admissible(uint64_t footprint) const { return footprint <= cap_; }
    void push(const ServeRequest& r) { queue_.push_back(r); }

    std::vector<ServeBatch> admit()
    {
        std::vector<ServeBatch> out;
        while (!queue_.empty()) {
            const int slot = free_slot();
            if (slot < 0) break;
            const ServeRequest head = queue_.front();
            if (used_ + head.footprint > cap_) break;
            ServeBatch b;
            b.slot = slot;
            b.key_type = head.key_type;
            b.small = head.n <= small_max_;
            b.footprint = head.footprint;
            b.reqs.push_back(head);
            queue_.pop_front();
            if (b.small) {
                for (auto it = queue_.begin(); it != queue_.end() && b.reqs.size() < max_batch_;) {
                    if (it->key_type == b.key_type && it->n <= small_max_ &&
                        used_ + b.footprint + it->footprint <= cap_) {
                        b.footprint += it->footprint;
                        b.reqs.push_back(*it);
                        it = queue_.erase(it);
                    } else {
                        ++it;
                    }
                }
            }
            used_ += b.footprint;
            if (used_ > max_used_) max_used_ = used_;
            slot_busy_[slot] = true;
            slot_fp_[slot] = b.footprint;
            out.push_back(std::move(b));
        }
        return out;
    }

    // The batch running in `slot` has completed.
    void release(int slot)
    {
        if (slot < 0 || (size_t)slot >= slot_busy_.size() || !slot_busy_[slot]) return;
        used_ -= slot_fp_[slot];
        slot_fp_[slot] = 0;
        slot_busy_[slot] = false;
    }

    size_t queued() const { return queue_.size(); }
    uint64_t used() const { return used_; }
    uint64_t max_used() const { return max_used_; }
    void reset_max_used() { max_used_ = used_; }
    uint64_t cap() const { return cap_; }
    size_t busy_slots() const
    {
        size_t c = 0;
        for (bool b : slot_busy_) c += b;
        return c;
    }
    int num_slots() const { return (int)slot_busy_.size(); }

private:
    int free_slot() const
    {
        for (size_t i = 0; i < slot_busy_.size(); ++i)
            if (!slot_busy_[i]) return (int)i;
        return -1;
    }

    uint64_t cap_;
    uint64_t small_max_;
    size_t max_batch_;
    uint64_t used_ = 0;
    uint64_t max_used_ = 0;
    std::vector<bool> slot_busy_;
    std::vector<uint64_t> slot_fp_;
    std::deque<ServeRequest> queue_;
};

}  // namespace rsort
