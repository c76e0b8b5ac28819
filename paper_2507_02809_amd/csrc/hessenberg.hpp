// Eigenvalues of a small real upper Hessenberg matrix (plain C++, host only): the Ritz values of the
// Arnoldi matrices that tsfde_arnoldi returns.  Francis' implicit double-shift QR iteration as given
// by Golub and Van Loan (Matrix Computations, the Francis QR step and the practical QR algorithm of
// the unsymmetric eigenvalue chapter): the active window [lo, hi] is shrunk at negligible subdiagonal
// entries, 1 x 1 and 2 x 2 diagonal blocks give the eigenvalues, and each step chases a 3 x 3
// Householder bulge from the top of the window to its bottom.  Only the window is updated, since
// only eigenvalues are wanted.
#pragma once

#include <cmath>
#include <vector>

namespace tsfde {

namespace hess_detail {

// eigenvalues of [[a, b], [c, d]]
inline void eig2(double a, double b, double c, double d, double& re1, double& im1, double& re2, double& im2) {
    const double half_tr = 0.5 * (a + d);
    const double det = a * d - b * c;
    const double disc = half_tr * half_tr - det;
    if (disc >= 0.0) {
        // the root of larger magnitude from the sum, the other from the product (no cancellation)
        const double r = std::sqrt(disc);
        const double big = half_tr >= 0.0 ? half_tr + r : half_tr - r;
        re1 = big;
        re2 = big != 0.0 ? det / big : 0.0;
        im1 = im2 = 0.0;
    } else {
        const double r = std::sqrt(-disc);
        re1 = re2 = half_tr;
        im1 = r;
        im2 = -r;
    }
}

// a Householder vector v (v[0] = 1) and beta with (I - beta v v^T) x = alpha e_1, for x of length 2 or 3
inline void house(const double* x, int len, double* v, double& beta) {
    double sigma = 0.0;
    for (int i = 1; i < len; ++i) sigma += x[i] * x[i];
    v[0] = 1.0;
    for (int i = 1; i < len; ++i) v[i] = x[i];
    if (sigma == 0.0) {
        beta = 0.0;
        return;
    }
    const double mu = std::sqrt(x[0] * x[0] + sigma);
    const double v0 = x[0] <= 0.0 ? x[0] - mu : -sigma / (x[0] + mu);
    beta = 2.0 * v0 * v0 / (sigma + v0 * v0);
    for (int i = 1; i < len; ++i) v[i] /= v0;
}

}  // namespace hess_detail

// H: n x n, row-major, upper Hessenberg (entries below the first subdiagonal are ignored); it is
// overwritten.  Returns false if the iteration did not converge (more than 60 steps for one window
// without a deflation); the eigenvalues found are then incomplete.
inline bool hessenberg_eigenvalues(std::vector<double>& H, int n, std::vector<double>& re, std::vector<double>& im) {
    using namespace hess_detail;
    re.assign(n, 0.0);
    im.assign(n, 0.0);
    auto h = [&](int i, int j) -> double& { return H[(size_t)i * n + j]; };
    const double eps = 2.220446049250313e-16;
    double norm = 0.0;  // for windows whose diagonal vanishes
    for (int i = 0; i < n; ++i)
        for (int j = (i > 0 ? i - 1 : 0); j < n; ++j) norm += std::fabs(h(i, j));
    int hi = n - 1;
    int steps = 0;
    while (hi >= 0) {
        // the window [lo, hi]: lo just below the lowest negligible subdiagonal entry
        int lo = hi;
        while (lo > 0) {
            double s = std::fabs(h(lo - 1, lo - 1)) + std::fabs(h(lo, lo));
            if (s == 0.0) s = norm;
            if (std::fabs(h(lo, lo - 1)) <= eps * s) {
                h(lo, lo - 1) = 0.0;
                break;
            }
            --lo;
        }
        if (lo == hi) {
            re[hi] = h(hi, hi);
            im[hi] = 0.0;
            --hi;
            steps = 0;
            continue;
        }
        if (lo == hi - 1) {
            eig2(h(hi - 1, hi - 1), h(hi - 1, hi), h(hi, hi - 1), h(hi, hi), re[hi - 1], im[hi - 1], re[hi], im[hi]);
            hi -= 2;
            steps = 0;
            continue;
        }
        if (++steps > 60) return false;
        // shifts: the eigenvalues of the trailing 2 x 2 block (through their sum and product); every
        // tenth step an ad hoc pair from the size of the last subdiagonal entries breaks cycles
        double s = h(hi - 1, hi - 1) + h(hi, hi);
        double t = h(hi - 1, hi - 1) * h(hi, hi) - h(hi - 1, hi) * h(hi, hi - 1);
        if (steps % 10 == 0) {
            const double w = std::fabs(h(hi, hi - 1)) + std::fabs(h(hi - 1, hi - 2));
            s = 1.5 * w;
            t = w * w;
        }
        // first column of (H - s1 I)(H - s2 I) = H^2 - s H + t I, nonzero in its first three entries
        double x[3];
        x[0] = h(lo, lo) * h(lo, lo) + h(lo, lo + 1) * h(lo + 1, lo) - s * h(lo, lo) + t;
        x[1] = h(lo + 1, lo) * (h(lo, lo) + h(lo + 1, lo + 1) - s);
        x[2] = h(lo + 1, lo) * h(lo + 2, lo + 1);
        for (int k = lo; k <= hi - 2; ++k) {
            double v[3], beta;
            house(x, 3, v, beta);
            if (beta != 0.0) {
                const int c0 = k > lo ? k - 1 : lo;
                for (int j = c0; j <= hi; ++j) {  // rows k..k+2
                    const double d = h(k, j) + v[1] * h(k + 1, j) + v[2] * h(k + 2, j);
                    h(k, j) -= beta * d;
                    h(k + 1, j) -= beta * d * v[1];
                    h(k + 2, j) -= beta * d * v[2];
                }
                const int r1 = k + 3 < hi ? k + 3 : hi;
                for (int i = lo; i <= r1; ++i) {  // columns k..k+2
                    const double d = h(i, k) + v[1] * h(i, k + 1) + v[2] * h(i, k + 2);
                    h(i, k) -= beta * d;
                    h(i, k + 1) -= beta * d * v[1];
                    h(i, k + 2) -= beta * d * v[2];
                }
            }
            x[0] = h(k + 1, k);
            x[1] = h(k + 2, k);
            x[2] = k < hi - 2 ? h(k + 3, k) : 0.0;
        }
        // the last 2 x 2 reflection restores the Hessenberg form at the bottom of the window
        {
            double v[2], beta;
            house(x, 2, v, beta);
            if (beta != 0.0) {
                const int k = hi - 1;
                for (int j = k - 1; j <= hi; ++j) {
                    const double d = h(k, j) + v[1] * h(k + 1, j);
                    h(k, j) -= beta * d;
                    h(k + 1, j) -= beta * d * v[1];
                }
                for (int i = lo; i <= hi; ++i) {
                    const double d = h(i, k) + v[1] * h(i, k + 1);
                    h(i, k) -= beta * d;
                    h(i, k + 1) -= beta * d * v[1];
                }
            }
        }
        // entries below the subdiagonal are rounding noise of the bulge chase
        for (int i = lo + 2; i <= hi; ++i)
            for (int j = lo; j < i - 1; ++j) h(i, j) = 0.0;
    }
    return true;
}

}  // namespace tsfde
