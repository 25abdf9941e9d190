// Host schedule of tet tiles whose upwind graphs have cycles (plain C++: no
// HIP, so that it can be built and checked on its own).
#include "tet_schedule.h"

#include <algorithm>
#include <thread>
#include <utility>

namespace pair {

CyclicSchedule tet_schedule_cyclic(const std::vector<int32_t>& nbr, int64_t nel, int64_t Em, int B, int T,
                                   const std::vector<int32_t>& tile_of, const std::vector<int32_t>& tile_ptr) {
    // member-independent: the elements of every tile and each element's index in it
    std::vector<int32_t> elems(Em), loc(Em), fill(tile_ptr.begin(), tile_ptr.end() - 1);
    for (int64_t e = 0; e < Em; ++e) {
        const int t = tile_of[e];
        loc[e] = fill[t] - tile_ptr[t];
        elems[fill[t]++] = static_cast<int32_t>(e);
    }
    struct Out {
        std::vector<int32_t> pos_elem, pos_scc, lstart, sstart;
    };
    const int64_t work = static_cast<int64_t>(B) * T;
    std::vector<Out> out(work);
    std::vector<int> err(work, 0);
    auto run = [&](int64_t w) {
        const int64_t m = w / T, mE = m * Em;
        const int t = static_cast<int>(w - m * T);
        const int n = tile_ptr[t + 1] - tile_ptr[t];
        const int32_t* te = elems.data() + tile_ptr[t];
        auto dep = [&](int i, int sl) -> int {   // in-tile upwind neighbour of node i through slot sl, or -1
            const int32_t u = nbr[static_cast<int64_t>(sl) * nel + mE + te[i]];
            if (u < 0 || tile_of[u - mE] != t) return -1;
            return loc[u - mE];
        };
        // Tarjan, iterative: frames (node, next slot)
        std::vector<int> index(n, -1), low(n, 0), comp(n, -1), stack, csize;
        std::vector<char> on(n, 0);
        std::vector<std::pair<int, int>> frames;
        int counter = 0, ncomp = 0;
        for (int r = 0; r < n; ++r) {
            if (index[r] >= 0) continue;
            frames.push_back({r, 0});
            index[r] = low[r] = counter++;
            stack.push_back(r);
            on[r] = 1;
            while (!frames.empty()) {
                auto& f = frames.back();
                const int v = f.first;
                if (f.second < 3) {
                    const int u = dep(v, f.second++);
                    if (u < 0) continue;
                    if (index[u] < 0) {
                        index[u] = low[u] = counter++;
                        stack.push_back(u);
                        on[u] = 1;
                        frames.push_back({u, 0});
                    } else if (on[u]) {
                        low[v] = std::min(low[v], index[u]);
                    }
                    continue;
                }
                if (low[v] == index[v]) {
                    int sz = 0, x;
                    do {
                        x = stack.back();
                        stack.pop_back();
                        on[x] = 0;
                        comp[x] = ncomp;
                        ++sz;
                    } while (x != v);
                    csize.push_back(sz);
                    ++ncomp;
                }
                frames.pop_back();
                if (!frames.empty()) {
                    const int pv = frames.back().first;
                    low[pv] = std::min(low[pv], low[v]);
                }
            }
        }
        // component levels in completion order (every upwind component first)
        std::vector<int> clev(ncomp, 0);
        std::vector<std::vector<int>> members(ncomp);
        for (int i = 0; i < n; ++i) members[comp[i]].push_back(i);
        int Lt = 0;
        for (int c = 0; c < ncomp; ++c) {
            if (csize[c] > kSccMax) err[w] = 1;
            int L = 0;
            for (int i : members[c])
                for (int sl = 0; sl < 3; ++sl) {
                    const int u = dep(i, sl);
                    if (u >= 0 && comp[u] != c) L = std::max(L, clev[comp[u]] + 1);
                }
            clev[c] = L;
            Lt = std::max(Lt, L);
        }
        Out& o = out[w];
        o.lstart.assign(Lt + 2, 0);
        o.sstart.assign(Lt + 1, 0);
        o.pos_elem.reserve(n);
        o.pos_scc.reserve(n);
        std::vector<std::vector<int>> single(Lt + 1), sets(Lt + 1);
        for (int c = 0; c < ncomp; ++c) (csize[c] == 1 ? single : sets)[clev[c]].push_back(c);
        for (int L = 0; L <= Lt; ++L) {
            o.lstart[L] = static_cast<int32_t>(o.pos_elem.size());
            for (int c : single[L]) {
                o.pos_elem.push_back(te[members[c][0]]);
                o.pos_scc.push_back(0);
            }
            o.sstart[L] = static_cast<int32_t>(o.pos_elem.size());
            for (int c : sets[L]) {
                const int first = static_cast<int>(o.pos_elem.size());
                for (int i : members[c]) {
                    o.pos_elem.push_back(te[i]);
                    o.pos_scc.push_back(first | (csize[c] << 16));
                }
            }
        }
        o.lstart[Lt + 1] = n;
    };
    const int nth = static_cast<int>(std::max<int64_t>(1, std::min<int64_t>(
        {16, static_cast<int64_t>(std::thread::hardware_concurrency()), work})));
    std::vector<std::thread> th;
    for (int i = 0; i < nth; ++i)
        th.emplace_back([&, i] {
            for (int64_t w = i; w < work; w += nth) run(w);
        });
    for (auto& x : th) x.join();
    CyclicSchedule cs;
    for (int64_t w = 0; w < work; ++w)
        if (err[w]) cs.too_large = true;
    if (cs.too_large) return cs;
    for (const Out& o : out) cs.Lmax = std::max(cs.Lmax, static_cast<int>(o.sstart.size()) - 1);
    const int Lmax = cs.Lmax;
    cs.order.assign(nel, 0);
    cs.scc.assign(nel, 0);
    cs.lvl.assign(static_cast<size_t>(work) * (Lmax + 2), 0);
    cs.lvls.assign(static_cast<size_t>(work) * (Lmax + 1), 0);
    for (int64_t w = 0; w < work; ++w) {
        const int64_t m = w / T;
        const int t = static_cast<int>(w - m * T);
        const Out& o = out[w];
        const int n = tile_ptr[t + 1] - tile_ptr[t];
        const int Lt = static_cast<int>(o.sstart.size()) - 1;
        const int64_t k0 = m * Em + tile_ptr[t];
        for (int q = 0; q < n; ++q) {
            cs.order[k0 + q] = o.pos_elem[q];
            cs.scc[k0 + q] = o.pos_scc[q];
            if (o.pos_scc[q]) cs.max_set = std::max(cs.max_set, o.pos_scc[q] >> 16);
        }
        for (int L = 0; L <= Lmax + 1; ++L) cs.lvl[w * (Lmax + 2) + L] = L <= Lt ? o.lstart[L] : n;
        for (int L = 0; L <= Lmax; ++L) cs.lvls[w * (Lmax + 1) + L] = L <= Lt ? o.sstart[L] : n;
    }
    return cs;
}


}  // namespace pair
