// Host check of the tet tile schedule for tiles with upwind cycles
// (csrc/tet_schedule.cpp), built with the address and undefined-behaviour
// sanitizers by tests/test_host_schedule.py.  Random tiles with planted
// cycles; every output is checked against brute force: the tile's elements
// once each, strongly connected sets by mutual reachability inside the tile,
// each set contiguous with its first position and size recorded, levels equal
// to the longest upwind path of the condensed graph, each level's single
// elements before its sets, dense level tables.  Prints "ok" and exits 0.
#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <random>
#include <vector>

#include "tet_schedule.h"

using pair::CyclicSchedule;

static int fail(const char* what, long a, long b) {
    std::printf("FAIL %s (%ld, %ld)\n", what, a, b);
    return 1;
}

struct Case {
    int64_t Em;
    int B, T;
    std::vector<int32_t> tile_of, tile_ptr, nbr;   // nbr [3][B Em], batch-global
};

// Elements of each tile in a random order; in-tile edges from a random DAG
// (edge e -> u only from a later to an earlier element of the order) plus
// planted cycles of length 2..cmax; some edges to other tiles (ignored by the
// schedule); empty slots.
static Case make_case(std::mt19937_64& rng, int64_t Em, int B, int T, int cmax, int ncyc) {
    Case c{Em, B, T, {}, {}, {}};
    c.tile_of.resize(Em);
    std::uniform_int_distribution<int> tile(0, T - 1);
    for (int64_t e = 0; e < Em; ++e) c.tile_of[e] = tile(rng);
    c.tile_ptr.assign(T + 1, 0);
    for (int64_t e = 0; e < Em; ++e) ++c.tile_ptr[c.tile_of[e] + 1];
    for (int t = 0; t < T; ++t) c.tile_ptr[t + 1] += c.tile_ptr[t];
    std::vector<std::vector<int32_t>> members(T);
    for (int64_t e = 0; e < Em; ++e) members[c.tile_of[e]].push_back(static_cast<int32_t>(e));
    const int64_t nel = Em * B;
    c.nbr.assign(3 * nel, -1);
    std::uniform_real_distribution<double> u01(0.0, 1.0);
    for (int m = 0; m < B; ++m) {
        const int64_t mE = static_cast<int64_t>(m) * Em;
        for (int t = 0; t < T; ++t) {
            std::vector<int32_t> ord = members[t];
            std::shuffle(ord.begin(), ord.end(), rng);
            const int n = static_cast<int>(ord.size());
            for (int q = 0; q < n; ++q)
                for (int sl = 0; sl < 3; ++sl) {
                    const double r = u01(rng);
                    int32_t u = -1;
                    if (r < 0.55 && q > 0) u = ord[std::uniform_int_distribution<int>(0, q - 1)(rng)];
                    else if (r < 0.75) {
                        u = static_cast<int32_t>(std::uniform_int_distribution<int64_t>(0, Em - 1)(rng));
                        if (c.tile_of[u] == t) u = -1;   // edges of this kind leave the tile
                    }
                    if (u == ord[q]) u = -1;
                    c.nbr[sl * nel + mE + ord[q]] = u < 0 ? -1 : static_cast<int32_t>(mE + u);
                }
            // planted cycles on disjoint runs of consecutive positions of the
            // order, each element pointing to the next: the DAG edges only
            // point to earlier positions, so no path re-enters a run and each
            // cycle is its own strongly connected set (of at most cmax)
            for (int k = 0; k < ncyc; ++k) {
                const int start = k * cmax;
                const int len = std::uniform_int_distribution<int>(2, cmax)(rng);
                if (start + len > n) break;
                for (int q = 0; q < len; ++q) {
                    const int32_t e = ord[start + q], u = ord[start + (q + 1) % len];
                    const int sl = std::uniform_int_distribution<int>(0, 2)(rng);
                    c.nbr[sl * nel + mE + e] = static_cast<int32_t>(mE + u);
                }
            }
        }
    }
    return c;
}

// Check one case; expect_large: a set above the limit must be reported.
static int check(const Case& c, bool expect_large) {
    const int64_t Em = c.Em, nel = Em * c.B;
    const CyclicSchedule s = pair::tet_schedule_cyclic(c.nbr, nel, Em, c.B, c.T, c.tile_of, c.tile_ptr);
    int largest = 1, Lmax_bf = 0;
    bool any_large = false;
    std::vector<std::vector<int>> level_of(static_cast<size_t>(c.B) * c.T);
    for (int m = 0; m < c.B; ++m) {
        const int64_t mE = static_cast<int64_t>(m) * Em;
        for (int t = 0; t < c.T; ++t) {
            const int n = c.tile_ptr[t + 1] - c.tile_ptr[t];
            std::vector<int32_t> el;
            std::vector<int> loc(Em, -1);
            for (int64_t e = 0; e < Em; ++e)
                if (c.tile_of[e] == t) { loc[e] = static_cast<int>(el.size()); el.push_back(static_cast<int32_t>(e)); }
            // in-tile dependency adjacency and reachability (closure)
            std::vector<std::vector<char>> R(n, std::vector<char>(n, 0));
            std::vector<std::vector<int>> dep(n);
            for (int a = 0; a < n; ++a)
                for (int sl = 0; sl < 3; ++sl) {
                    const int32_t u = c.nbr[sl * nel + mE + el[a]];
                    if (u < 0 || c.tile_of[u - mE] != t) continue;
                    dep[a].push_back(loc[u - mE]);
                    R[a][loc[u - mE]] = 1;
                }
            for (int k = 0; k < n; ++k)
                for (int a = 0; a < n; ++a)
                    if (R[a][k])
                        for (int b = 0; b < n; ++b)
                            if (R[k][b]) R[a][b] = 1;
            // components by mutual reachability
            std::vector<int> comp(n, -1), csz;
            for (int a = 0; a < n; ++a) {
                if (comp[a] >= 0) continue;
                comp[a] = static_cast<int>(csz.size());
                int sz = 1;
                for (int b = a + 1; b < n; ++b)
                    if (comp[b] < 0 && R[a][b] && R[b][a]) { comp[b] = comp[a]; ++sz; }
                csz.push_back(sz);
                largest = std::max(largest, sz);
                if (sz > pair::kSccMax) any_large = true;
            }
            // levels of the condensed graph: longest path, by repeated relaxation
            std::vector<int> cl(csz.size(), 0);
            for (bool ch = true; ch;) {
                ch = false;
                for (int a = 0; a < n; ++a)
                    for (int b : dep[a])
                        if (comp[b] != comp[a] && cl[comp[a]] < cl[comp[b]] + 1) { cl[comp[a]] = cl[comp[b]] + 1; ch = true; }
            }
            std::vector<int> lv(n);
            for (int a = 0; a < n; ++a) { lv[a] = cl[comp[a]]; Lmax_bf = std::max(Lmax_bf, lv[a]); }
            level_of[m * c.T + t] = lv;
            if (expect_large) continue;
            // the schedule's positions for this tile
            const int64_t k0 = mE + c.tile_ptr[t];
            std::vector<int> seen(n, 0);
            for (int q = 0; q < n; ++q) {
                const int32_t e = s.order[k0 + q];
                if (e < 0 || e >= Em || c.tile_of[e] != t) return fail("element outside its tile", m, q);
                if (seen[loc[e]]++) return fail("element twice", m, q);
            }
            const int64_t w = static_cast<int64_t>(m) * c.T + t;
            const int32_t* L = s.lvl.data() + w * (s.Lmax + 2);
            const int32_t* LS = s.lvls.data() + w * (s.Lmax + 1);
            if (L[s.Lmax + 1] != n) return fail("tile size entry", m, t);
            for (int Lv = 0; Lv <= s.Lmax; ++Lv) {
                if (!(L[Lv] <= LS[Lv] && LS[Lv] <= L[Lv + 1])) return fail("level table order", m, Lv);
                for (int q = L[Lv]; q < L[Lv + 1]; ++q) {
                    const int a = loc[s.order[k0 + q]];
                    if (lv[a] != Lv) return fail("level differs from the longest path", lv[a], Lv);
                    const bool single = csz[comp[a]] == 1;
                    if (single != (q < LS[Lv])) return fail("single elements before the sets", m, q);
                    const int32_t info = s.scc[k0 + q];
                    if (single) {
                        if (info != 0) return fail("scc entry of a single element", m, q);
                        continue;
                    }
                    const int first = info & 0xffff, sz = info >> 16;
                    if (sz != csz[comp[a]]) return fail("set size", sz, csz[comp[a]]);
                    if (q < first || q >= first + sz) return fail("position outside its set", q, first);
                    for (int q2 = first; q2 < first + sz; ++q2)
                        if (comp[loc[s.order[k0 + q2]]] != comp[a]) return fail("set not contiguous", q, q2);
                }
            }
            for (int Lv = 0; Lv <= s.Lmax + 1; ++Lv)
                if (Lv > 0 && L[Lv] < L[Lv - 1]) return fail("level starts decrease", m, Lv);
        }
    }
    if (expect_large) return s.too_large && any_large ? 0 : fail("a set above the limit not reported", largest, 0);
    if (s.too_large || any_large) return fail("unexpected large set", largest, 0);
    if (s.Lmax != Lmax_bf) return fail("Lmax", s.Lmax, Lmax_bf);
    if (s.max_set != largest) return fail("max_set", s.max_set, largest);
    return 0;
}

int main() {
    std::mt19937_64 rng(20240611);
    int cases = 0, with_sets = 0, over = 0, largest = 1;
    // acyclic-only, small cycles, many tiles, one tile
    const int shapes[][5] = {{120, 2, 6, 2, 0}, {300, 3, 9, 5, 3}, {400, 2, 1, 4, 6},
                             {250, 4, 25, 3, 2}, {60, 1, 3, 8, 2}, {500, 2, 12, 6, 4}};
    for (const auto& sh : shapes)
        for (int rep = 0; rep < 4; ++rep) {
            const Case c = make_case(rng, sh[0], sh[1], sh[2], sh[3], sh[4]);
            // random DAG edges plus cycles can merge into larger sets: decide by brute force
            bool big = false;
            {
                const CyclicSchedule s = pair::tet_schedule_cyclic(c.nbr, c.Em * c.B, c.Em, c.B, c.T, c.tile_of, c.tile_ptr);
                big = s.too_large;
                if (!big && s.max_set > 1) ++with_sets;
                if (!big) largest = std::max(largest, s.max_set);
                over += big ? 1 : 0;
            }
            if (check(c, big)) return 1;
            ++cases;
        }
    // a planted cycle of 20 elements inside one tile must be reported
    Case big = make_case(rng, 80, 1, 1, 2, 0);
    for (int q = 0; q < 20; ++q) big.nbr[0 * 80 + q] = (q + 1) % 20;
    if (check(big, true)) return 1;
    // the random cases must exercise sets inside the limit, not only the error
    if (with_sets < cases / 2) return fail("too few cases with strongly connected sets", with_sets, cases);
    std::printf("ok %d cases, %d with sets (largest %d), %d over the limit\n", cases + 1, with_sets, largest, over);
    return 0;
}
