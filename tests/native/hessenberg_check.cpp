// Reads n and an n x n row-major matrix from stdin, prints the eigenvalues of its upper Hessenberg
// part (paper_2507_02809_amd/csrc/hessenberg.hpp), one "re im" pair per line, or "fail".
#include <cstdio>
#include <vector>

#include "hessenberg.hpp"

int main() {
    int n = 0;
    while (std::scanf("%d", &n) == 1) {
        std::vector<double> H((size_t)n * n);
        for (auto& v : H)
            if (std::scanf("%lf", &v) != 1) return 2;
        std::vector<double> re, im;
        if (!tsfde::hessenberg_eigenvalues(H, n, re, im)) {
            std::printf("fail\n");
            continue;
        }
        for (int i = 0; i < n; ++i) std::printf("%.17g %.17g\n", re[i], im[i]);
        std::printf("end\n");
    }
    return 0;
}
