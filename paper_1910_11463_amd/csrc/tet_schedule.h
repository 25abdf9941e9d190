// Host schedule of tet tiles whose upwind graphs have cycles.
#pragma once

#include <cstdint>
#include <vector>

namespace pair {

constexpr int kSccMax = 16;   // elements of one strongly connected set the tile kernel solves (64 rows)

// Per member m < B and tile t < T: the strongly connected components of the
// upwind graph restricted to the tile (Tarjan's algorithm, iterative; a
// component is completed after every component it depends on, so completion
// order is an upwind order), levels of the condensed graph (longest upwind
// path inside the tile), and the positions: per level its single elements,
// then its components, each contiguous.
//   nbr: [3][nel] batch-global upwind neighbour of every batch element per
//        slot (-1: none), nel = B Em, members consecutive;
//   tile_of: [Em] tile of every element; tile_ptr: [T + 1] tile offsets.
// Outputs per batch position k = m Em + tile_ptr[t] + q: order (member-local
// element), scc (first position in the tile | size << 16 for elements of
// components of two or more, else 0); per (member, tile) w = m T + t: level
// starts lvl[w (Lmax + 2) + L] (L > the tile's last level: the tile's size;
// the last entry is the tile's size) and component starts lvls[w (Lmax + 1) + L]
// (the level's end where it has none).  too_large: some component has more
// than kSccMax elements (the outputs are then not filled).
struct CyclicSchedule {
    std::vector<int32_t> order, scc, lvl, lvls;
    int Lmax = 0, max_set = 1;
    bool too_large = false;
};

CyclicSchedule tet_schedule_cyclic(const std::vector<int32_t>& nbr, int64_t nel, int64_t Em, int B, int T,
                                   const std::vector<int32_t>& tile_of, const std::vector<int32_t>& tile_ptr);

}  // namespace pair
