// Process-wide gate for cooperative launches.
//
// A cooperative launch needs every one of its workgroups resident at once
// and spins at grid barriers; two of them in flight on one device together
// could each hold part of the machine while waiting for the rest.  Every
// path of the library that launches a cooperative kernel (mcm_match's
// persistent launch, mcm_konig_cover, mcm_bfs_levels, the multi-graph
// launch of mcm_match_batched and of the request server, the entry point
// without allocation) therefore enters this gate before the launch and
// leaves it only once the launch has completed.
//
// An owner (a stream on which the launches follow one another, so that they
// never overlap on the device) may enter again while it is inside; another
// owner waits until the count drops to zero.  An owner that is inside does
// not get in again while another owner waits, so a server that keeps
// launching cannot starve a caller of mcm_match.
//
// Host-only C++ (no HIP), so that the CPU tests can exercise it directly.
#pragma once
#include <chrono>
#include <condition_variable>
#include <cstdint>
#include <mutex>

namespace mcm {

class CoopGate {
  public:
    // Blocks until `owner` may launch, then counts one launch in.
    void enter(const void *owner)
    {
        std::unique_lock<std::mutex> lk(mu_);
        ++waiting_;
        cv_.wait(lk, [&] { return count_ == 0 || (owner_ == owner && waiting_ == 1); });
        --waiting_;
        owner_ = owner;
        ++count_;
    }
    // Non-blocking form: true if a launch was counted in.  A caller that
    // waits in enter() goes first, even when the count is zero.
    bool try_enter(const void *owner)
    {
        std::lock_guard<std::mutex> lk(mu_);
        if (waiting_ != 0 || (count_ != 0 && owner_ != owner)) return false;
        owner_ = owner;
        ++count_;
        return true;
    }
    // A counted launch of `owner` has completed.
    void leave(const void *owner)
    {
        std::lock_guard<std::mutex> lk(mu_);
        if (count_ > 0 && owner_ == owner && --count_ == 0) owner_ = nullptr;
        cv_.notify_all();
    }
    int in_flight()
    {
        std::lock_guard<std::mutex> lk(mu_);
        return count_;
    }

  private:
    std::mutex mu_;
    std::condition_variable cv_;
    const void *owner_ = nullptr;
    int count_ = 0;
    int waiting_ = 0;
};

// The one gate of the process.
CoopGate &coop_gate();

}  // namespace mcm
