// Admission control of the serving loop: a FIFO of submitted tasks, admitted
// in order once (a) the descriptor ring slot their sequence number maps to is
// free, (b) their bytes fit the HBM budget and (c) their tiles fit the
// device tile map.  The paper runs one accelerator task at a time per worker
// to avoid contention (`--cores 1`, sec. 3.1.5); here tasks share the GPU and
// this controller is what keeps them within the memory the device can give.
// Pure host logic with no clock or device dependency, so it is unit-tested on
// the CPU.
#pragma once

#include <cstdint>
#include <deque>
#include <vector>

namespace sparkcl {

struct Pending {
    uint64_t ticket = 0;
    uint64_t bytes = 0;  // charged against the budget while in flight
    uint32_t ntiles = 0; // tile-map entries while in flight
    uint64_t t_arrive = 0;
    uint32_t user = 0;   // caller's index into its own task storage
    // A staged task (inputs in host memory) is admitted against the budget
    // and tile map alone; it takes a ring slot (and its sequence number) only
    // once its inputs have been copied to the device, so a copy in progress
    // never holds up the tasks admitted after it.
    bool staged = false;
};

constexpr uint64_t kNoSeq = ~0ull;

struct Admitted {
    Pending p;
    uint64_t seq = kNoSeq; // kNoSeq: a staged task that has no slot yet
    uint32_t slot = 0;
    bool has_slot() const { return seq != kNoSeq; }
};

enum class AdmitBlock { NONE, EMPTY, SLOT, BUDGET, TILES };

class Admission {
  public:
    Admission(uint64_t budget, uint32_t slots, uint64_t tile_cap)
        : budget_(budget), busy_(slots, 0), tile_cap_(tile_cap)
    {
    }

    // Whether a task of this size could ever be admitted.
    bool fits_at_all(uint64_t bytes, uint32_t ntiles) const
    {
        return bytes <= budget_ && ntiles <= tile_cap_;
    }

    void push(const Pending &p) { q_.push_back(p); }
    size_t pending() const { return q_.size(); }

    // What stops the head of the queue from being admitted right now.
    AdmitBlock head_block() const
    {
        if (q_.empty())
            return AdmitBlock::EMPTY;
        const Pending &h = q_.front();
        if (!h.staged && !slot_free())
            return AdmitBlock::SLOT;
        if (in_use_ + h.bytes > budget_)
            return AdmitBlock::BUDGET;
        if (tiles_ + h.ntiles > tile_cap_)
            return AdmitBlock::TILES;
        return AdmitBlock::NONE;
    }

    // Admits the head (the caller checked head_block() == NONE).  A staged
    // head is charged but gets no slot (take_slot later).
    Admitted admit_head()
    {
        Admitted a;
        a.p = q_.front();
        q_.pop_front();
        if (!a.p.staged)
            take_slot(a);
        in_use_ += a.p.bytes;
        tiles_ += a.p.ntiles;
        if (in_use_ > peak_)
            peak_ = in_use_;
        ++in_flight_;
        return a;
    }

    // Whether the ring slot of the next sequence number is free.
    bool slot_free() const { return !busy_[slot_of(next_seq_)]; }

    // Gives an admitted staged task the next sequence number and its ring
    // slot (the caller checked slot_free()).
    void take_slot(Admitted &a)
    {
        a.seq = next_seq_++;
        a.slot = slot_of(a.seq);
        busy_[a.slot] = 1;
    }

    // Undo an admission whose device resources could not be obtained; the
    // task goes back to the head of the queue (a slotted one must be the
    // latest admission and returns its sequence number).
    void unadmit(const Admitted &a)
    {
        if (a.has_slot()) {
            busy_[a.slot] = 0;
            --next_seq_;
        }
        in_use_ -= a.p.bytes;
        tiles_ -= a.p.ntiles;
        --in_flight_;
        q_.push_front(a.p);
    }

    void complete(const Admitted &a)
    {
        if (a.has_slot())
            busy_[a.slot] = 0;
        in_use_ -= a.p.bytes;
        tiles_ -= a.p.ntiles;
        --in_flight_;
    }

    // Drop every queued task (shutdown); returns them.
    std::deque<Pending> take_queue()
    {
        std::deque<Pending> out;
        out.swap(q_);
        return out;
    }

    uint32_t slot_of(uint64_t seq) const { return (uint32_t)(seq % busy_.size()); }
    uint64_t next_seq() const { return next_seq_; }
    uint64_t in_use() const { return in_use_; }
    uint64_t peak() const { return peak_; }
    uint64_t tiles_in_flight() const { return tiles_; }
    uint64_t in_flight() const { return in_flight_; }
    uint64_t budget() const { return budget_; }

  private:
    uint64_t budget_;
    std::vector<uint8_t> busy_;
    uint64_t tile_cap_;
    std::deque<Pending> q_;
    uint64_t next_seq_ = 0, in_use_ = 0, peak_ = 0, tiles_ = 0, in_flight_ = 0;
};

} // namespace sparkcl
