// Host check of the LDS budget of the dense transform passes (paper_2507_02809_amd/csrc/
// transform_lds.hpp): the static partial sums are counted, and the largest N that passes the check
// fits 160 KB while N + 1 does not, for the Hartley (Np = N) and sine (Np = 2(N+1)) tables, d = 1, 2.
#include <cstdio>

#include "transform_lds.hpp"

using namespace tsfde;

int main() {
    int fails = 0;
    for (int d = 1; d <= 2; ++d) {
        for (int sine = 0; sine <= 1; ++sine) {
            auto Np = [&](int N) { return sine ? 2 * (N + 1) : N; };
            int last = 0;
            for (int N = 1; N < 40000; ++N)
                if (dense_blocks_fit(d, N, Np(N))) last = N;
            const int nrow = d == 2 ? last : 1;
            const size_t used = pass_lds(last, Np(last), nrow, sizeof(double));
            const size_t over = pass_lds(last + 1, Np(last + 1), d == 2 ? last + 1 : 1, sizeof(double));
            // the static array of 4 x 64 doubles is part of every launch
            const size_t dyn = pass_dyn_lds(last, Np(last), nrow, sizeof(double));
            if (!(used <= kPassLdsBytes && over > kPassLdsBytes && used == dyn + 4 * 64 * sizeof(double))) {
                std::fprintf(stderr, "d=%d sine=%d: last N %d uses %zu, N+1 uses %zu\n", d, sine, last, used, over);
                ++fails;
            }
            std::printf("d=%d %s: largest N %d (%zu bytes)\n", d, sine ? "sine" : "cas", last, used);
        }
    }
    if (fails) return 1;
    std::printf("transform lds ok\n");
    return 0;
}
