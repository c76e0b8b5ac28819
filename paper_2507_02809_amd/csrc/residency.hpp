// Admission of persistent grids (plain C++, no HIP: the host logic is tested on the CPU).
//
// The forward-substitution kernels of P^-1 are persistent: their workgroups wait for each other at
// device-wide barriers, so every workgroup of such a grid must be resident at the same time, also
// when several of them run side by side on different streams.  They are ordinary launches; what
// keeps them co-resident is this budget, taken before a grid's first launch and given back after
// the host has seen its last one finish.
//
// Model of the device.  The command processor deals the workgroups of one dispatch to the XCDs in
// turn (workgroup i to XCD i mod nxcd; MI355X: 8 XCDs of 32 CUs), and a workgroup can only run on
// a CU of its own XCD.  A persistent grid of g > 1 workgroups therefore puts at most ceil(g/nxcd)
// of them on any one XCD; a grid of one workgroup never waits (its barriers are no-ops) and needs
// nothing.  Charging every XCD ceil(g/nxcd) "CU slots", and keeping the total charge within the
// CUs per XCD, guarantees that the waiting workgroups of all admitted grids fit on distinct CUs
// even if no two of them share a CU (every kernel's workgroup fits one CU on its own, which the
// launcher checks by occupancy).  Other, non-persistent kernels only delay a persistent workgroup:
// they finish without waiting on anything.
#pragma once

#include <algorithm>
#include <condition_variable>
#include <mutex>

namespace tsfde {

// CU slots a persistent grid of `grid` workgroups takes on every XCD
inline int residency_slots(int grid, int nxcd) {
    if (grid <= 1) return 0;
    nxcd = std::max(1, nxcd);
    return (grid + nxcd - 1) / nxcd;
}

// largest grid whose charge fits `slots` per XCD
inline int residency_max_grid(int slots, int nxcd) { return std::max(1, slots) * std::max(1, nxcd); }

// A per-device pool of CU slots (the CUs of one XCD).  acquire() blocks the calling host thread
// until the charge fits; release() gives it back and wakes the waiters.
class ResidencyBudget {
  public:
    explicit ResidencyBudget(int slots = 0) : total_(slots), free_(slots) {}

    void reset(int slots) {
        std::lock_guard<std::mutex> lk(mx_);
        total_ = free_ = slots;
    }
    int total() const { return total_; }
    int available() {
        std::lock_guard<std::mutex> lk(mx_);
        return free_;
    }

    // takes `need` slots (0 <= need <= total), waiting for them if other grids hold them
    void acquire(int need) {
        if (need <= 0) return;
        std::unique_lock<std::mutex> lk(mx_);
        need = std::min(need, total_);
        cv_.wait(lk, [&] { return free_ >= need; });
        free_ -= need;
    }

    void release(int need) {
        if (need <= 0) return;
        {
            std::lock_guard<std::mutex> lk(mx_);
            free_ = std::min(total_, free_ + std::min(need, total_));
        }
        cv_.notify_all();
    }

  private:
    std::mutex mx_;
    std::condition_variable cv_;
    int total_;
    int free_;
};

// Slots held by one P^-1 application; release() is idempotent, the destructor releases.
class ResidencyTicket {
  public:
    ResidencyTicket() = default;
    ResidencyTicket(const ResidencyTicket&) = delete;
    ResidencyTicket& operator=(const ResidencyTicket&) = delete;
    ~ResidencyTicket() { release(); }

    void hold(ResidencyBudget* b, int need) {
        release();
        if (!b || need <= 0) return;
        need = std::min(need, b->total());
        b->acquire(need);
        budget_ = b;
        need_ = need;
    }
    void release() {
        if (budget_) budget_->release(need_);
        budget_ = nullptr;
        need_ = 0;
    }
    int held() const { return need_; }

  private:
    ResidencyBudget* budget_ = nullptr;
    int need_ = 0;
};

}  // namespace tsfde
