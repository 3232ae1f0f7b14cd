// CPU check of the cooperative-launch gate (paper_1303_1379_amd/csrc/mcm_gate.h):
// threads stand in for callers of the library, a "launch" is a short sleep
// during which the thread records itself as running on the device.
//   * callers with distinct owners (mcm_match on their own streams) never
//     have launches in flight at the same time;
//   * one owner (a server's compute stream) may hold several launches;
//   * a caller that waits gets in although the server keeps trying to launch.
// Prints "ok" and exits 0, or prints what failed and exits 1.
#include <atomic>
#include <chrono>
#include <cstdio>
#include <thread>
#include <vector>

#include "mcm_gate.h"

namespace mcm {
CoopGate &coop_gate()
{
    static CoopGate g;
    return g;
}
}  // namespace mcm

using namespace std::chrono;

static std::atomic<int> g_owners_running{0};  // distinct owners with launches in flight
static std::atomic<int> g_bad{0};

int main()
{
    mcm::CoopGate &gate = mcm::coop_gate();
    int tok[8];
    // 1. six callers, distinct owners, 200 launches each
    {
        std::vector<std::thread> th;
        for (int t = 0; t < 6; ++t)
            th.emplace_back([&, t] {
                for (int i = 0; i < 200; ++i) {
                    gate.enter(&tok[t]);
                    if (g_owners_running.fetch_add(1) != 0) g_bad.fetch_add(1);
                    std::this_thread::sleep_for(microseconds(20));
                    g_owners_running.fetch_sub(1);
                    gate.leave(&tok[t]);
                }
            });
        for (auto &x : th) x.join();
        if (g_bad.load()) { std::printf("distinct owners overlapped %d times\n", g_bad.load()); return 1; }
        if (gate.in_flight() != 0) { std::printf("count left at %d\n", gate.in_flight()); return 1; }
    }
    // 2. one owner holds two launches; another owner cannot get in meanwhile
    {
        if (!gate.try_enter(&tok[6]) || !gate.try_enter(&tok[6])) { std::printf("owner re-entry refused\n"); return 1; }
        if (gate.try_enter(&tok[7])) { std::printf("second owner admitted\n"); return 1; }
        gate.leave(&tok[6]);
        if (gate.try_enter(&tok[7])) { std::printf("second owner admitted with one launch left\n"); return 1; }
        gate.leave(&tok[6]);
        if (!gate.try_enter(&tok[7])) { std::printf("second owner refused on an empty gate\n"); return 1; }
        gate.leave(&tok[7]);
    }
    // 3. a server thread keeps launching (try_enter, two in flight, completions
    //    after 50 us); a caller that waits must get in within a bound, and
    //    never while a server launch is in flight
    {
        std::atomic<bool> stop{false};
        std::atomic<int> server_running{0};
        std::thread server([&] {
            std::vector<steady_clock::time_point> inflight;
            while (!stop.load()) {
                const auto now = steady_clock::now();
                for (size_t i = 0; i < inflight.size();)
                    if (now - inflight[i] > microseconds(50)) {
                        inflight.erase(inflight.begin() + i);
                        server_running.fetch_sub(1);
                        gate.leave(&tok[6]);
                    } else {
                        ++i;
                    }
                if (inflight.size() < 2 && gate.try_enter(&tok[6])) {
                    server_running.fetch_add(1);
                    inflight.push_back(steady_clock::now());
                }
                std::this_thread::yield();
            }
            for (size_t i = 0; i < inflight.size(); ++i) {
                server_running.fetch_sub(1);
                gate.leave(&tok[6]);
            }
        });
        int got = 0;
        for (int i = 0; i < 50; ++i) {
            const auto t0 = steady_clock::now();
            gate.enter(&tok[0]);
            if (server_running.load() != 0) g_bad.fetch_add(1);
            if (steady_clock::now() - t0 > seconds(2)) g_bad.fetch_add(1000);
            std::this_thread::sleep_for(microseconds(30));
            if (server_running.load() != 0) g_bad.fetch_add(1);
            gate.leave(&tok[0]);
            ++got;
            std::this_thread::sleep_for(microseconds(100));
        }
        stop.store(true);
        server.join();
        if (g_bad.load()) { std::printf("caller overlapped or starved: %d\n", g_bad.load()); return 1; }
        if (got != 50 || gate.in_flight() != 0) { std::printf("caller got %d, count %d\n", got, gate.in_flight()); return 1; }
    }
    std::printf("ok\n");
    return 0;
}
