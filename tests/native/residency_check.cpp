// Host check of the persistent-grid admission logic (paper_2507_02809_amd/csrc/residency.hpp):
// the CU-slot charge of a grid, and that concurrent holders never exceed the pool and never deadlock.
#include <atomic>
#include <chrono>
#include <cstdio>
#include <random>
#include <thread>
#include <vector>

#include "residency.hpp"

using namespace tsfde;

static int fails = 0;
#define CHECK(c)                                                     \
    do {                                                             \
        if (!(c)) {                                                  \
            std::fprintf(stderr, "check failed: %s (line %d)\n", #c, __LINE__); \
            ++fails;                                                 \
        }                                                            \
    } while (0)

int main() {
    // charge per XCD: nothing for one workgroup (no barrier waits), ceil(g / 8) otherwise
    CHECK(residency_slots(0, 8) == 0);
    CHECK(residency_slots(1, 8) == 0);
    CHECK(residency_slots(2, 8) == 1);
    CHECK(residency_slots(8, 8) == 1);
    CHECK(residency_slots(9, 8) == 2);
    CHECK(residency_slots(33, 8) == 5);
    CHECK(residency_slots(256, 8) == 32);
    CHECK(residency_max_grid(32, 8) == 256);
    // a grid of at most residency_max_grid(slots) workgroups is charged at most `slots`
    for (int s = 1; s <= 40; ++s)
        for (int g = 1; g <= residency_max_grid(s, 8); ++g) CHECK(residency_slots(g, 8) <= s);
    // the largest per-problem grid of a batch (256 CUs / 8 problems) times 8 problems fills the pool exactly
    CHECK(8 * residency_slots(256 / 8, 8) == 256 / 8);

    // tickets: hold, idempotent release, release by the destructor
    ResidencyBudget pool(32);
    {
        ResidencyTicket t;
        t.hold(&pool, 5);
        CHECK(pool.available() == 27 && t.held() == 5);
        t.release();
        t.release();
        CHECK(pool.available() == 32 && t.held() == 0);
        t.hold(&pool, 7);
        CHECK(pool.available() == 25);
    }
    CHECK(pool.available() == 32);

    // concurrent holders: the slots in use never exceed the pool, every thread finishes
    std::atomic<int> in_use{0}, peak{0}, done{0};
    std::vector<std::thread> th;
    for (int w = 0; w < 16; ++w)
        th.emplace_back([&, w] {
            std::mt19937 rng(1234 + w);
            std::uniform_int_distribution<int> grid(1, 256);
            for (int k = 0; k < 300; ++k) {
                const int g = grid(rng);
                ResidencyTicket t;
                t.hold(&pool, residency_slots(g, 8));
                const int now = in_use.fetch_add(t.held()) + t.held();
                int p = peak.load();
                while (now > p && !peak.compare_exchange_weak(p, now)) {
                }
                std::this_thread::sleep_for(std::chrono::microseconds(20));
                in_use.fetch_sub(t.held());
            }
            done.fetch_add(1);
        });
    for (auto& t : th) t.join();
    CHECK(done.load() == 16);
    CHECK(peak.load() <= 32);
    CHECK(peak.load() > 0);
    CHECK(pool.available() == 32);
    if (fails) return 1;
    std::printf("residency ok (peak %d of 32 slots)\n", peak.load());
    return 0;
}
