// Level-symmetric S_N quadrature sets (phi = sum_m w_m psi_m, eq. angular_quad),
// weights normalised to sum to 4 pi.
//
// Cosine levels mu_i^2 = mu_1^2 + (i - 1) * 2 (1 - 3 mu_1^2) / (N - 2); the points
// of one octant are the level triples (i, j, k) with i + j + k = N/2 + 2.  The
// weight is constant on each permutation class; S4 has one class and mu_1 fixed
// by the fourth moment (2 mu_1^4 + mu_2^4 = 3/5), S8 uses the tabulated
// mu_1 = 0.2182179 and three classes whose weights satisfy normalisation,
// <mu^4> = 1/5 and <mu^6> = 1/7.
#include <algorithm>
#include <array>
#include <cmath>
#include <map>
#include <vector>

#include "common.h"

namespace pair {

static void solve_small(std::vector<std::vector<double>>& A, std::vector<double>& b) {
    const int n = static_cast<int>(b.size());
    for (int p = 0; p < n; ++p) {
        int piv = p;
        for (int r = p + 1; r < n; ++r)
            if (std::fabs(A[r][p]) > std::fabs(A[piv][p])) piv = r;
        std::swap(A[p], A[piv]);
        std::swap(b[p], b[piv]);
        for (int r = p + 1; r < n; ++r) {
            double l = A[r][p] / A[p][p];
            for (int c = p; c < n; ++c) A[r][c] -= l * A[p][c];
            b[r] -= l * b[p];
        }
    }
    for (int r = n - 1; r >= 0; --r) {
        double s = b[r];
        for (int c = r + 1; c < n; ++c) s -= A[r][c] * b[c];
        b[r] = s / A[r][r];
    }
}

int level_symmetric(int order, std::vector<double>& omega, std::vector<double>& w) {
    if (order != 2 && order != 4 && order != 8) return -1;
    const int nlev = order / 2;
    std::vector<double> mu(nlev);
    if (order == 2) {
        mu[0] = 1.0 / std::sqrt(3.0);
    } else {
        double mu1sq;
        if (order == 4) {
            // 6 u^2 - 4 u + 2/5 = 0, smaller root
            mu1sq = (4.0 - std::sqrt(16.0 - 9.6)) / 12.0;
        } else {
            const double mu1 = 0.2182179;
            mu1sq = mu1 * mu1;
        }
        const double D = 2.0 * (1.0 - 3.0 * mu1sq) / (order - 2);
        for (int i = 0; i < nlev; ++i) mu[i] = std::sqrt(mu1sq + i * D);
    }
    std::vector<std::array<int, 3>> trip;
    const int sum = nlev + 2;
    for (int i = 1; i <= nlev; ++i)
        for (int j = 1; j <= nlev; ++j) {
            int k = sum - i - j;
            if (k >= 1 && k <= nlev) trip.push_back({i, j, k});
        }
    auto cls = [](std::array<int, 3> t) {
        std::sort(t.begin(), t.end());
        return t;
    };
    std::map<std::array<int, 3>, int> classes;
    for (auto& t : trip) classes.emplace(cls(t), 0);
    int ci = 0;
    for (auto& kv : classes) kv.second = ci++;
    const int nc = static_cast<int>(classes.size());
    std::vector<double> wc(nc);
    if (nc == 1) {
        wc[0] = 1.0 / trip.size();
    } else {
        std::vector<std::vector<double>> A(nc, std::vector<double>(nc, 0.0));
        std::vector<double> rhs(nc, 0.0);
        const int pw[2] = {4, 6};
        const double mom[2] = {1.0 / 5.0, 1.0 / 7.0};
        for (auto& t : trip) {
            int c = classes[cls(t)];
            A[0][c] += 1.0;
            for (int r = 1; r < nc; ++r) A[r][c] += std::pow(mu[t[0] - 1], pw[r - 1]);
        }
        rhs[0] = 1.0;
        for (int r = 1; r < nc; ++r) rhs[r] = mom[r - 1];
        solve_small(A, rhs);
        wc = rhs;
    }
    omega.clear();
    w.clear();
    const double fourpi = 4.0 * M_PI;
    for (int o = 0; o < 8; ++o) {
        const double sx = (o & 1) ? -1.0 : 1.0, sy = (o & 2) ? -1.0 : 1.0, sz = (o & 4) ? -1.0 : 1.0;
        for (auto& t : trip) {
            omega.push_back(sx * mu[t[0] - 1]);
            omega.push_back(sy * mu[t[1] - 1]);
            omega.push_back(sz * mu[t[2] - 1]);
            w.push_back(wc[classes[cls(t)]] * fourpi / 8.0);
        }
    }
    return static_cast<int>(w.size());
}

}  // namespace pair
