// Work list of a persistent batched launch (plain C++, no HIP: the scheduling
// logic is also compiled and checked on the host by the tests).
//
// A persistent launch runs a fixed number of workgroups that take work items
// from one queue, in ticket order, until the queue is empty.  An item is one
// workgroup of one round of one grid.  Round k of a grid reads what round k-1
// of the same grid wrote, so it may start only once every wave of that
// grid's earlier rounds has finished: each grid has a completion counter
// (waves done), and each round a threshold `need` on it.  Grids are
// independent of each other.
//
// Items are ordered by round index first (all grids' round 0, then all round
// 1, ...), the largest grids first within a round index, and by workgroup
// within a round.  Every item then depends only on items with smaller
// tickets.  A workgroup that holds a ticket is running, so the item with the
// smallest unfinished ticket never waits on anything unfinished: the queue
// always makes progress, whatever the number of resident workgroups.
#pragma once

#include <stdint.h>

#include <algorithm>
#include <numeric>
#include <vector>

namespace s5d {

struct PersistRound {
  int32_t grid;   // index of the grid (completion counter)
  int32_t round;  // round index within the grid's schedule
  int32_t need;   // waves of this grid that must be done before the round starts
  int32_t first;  // ticket of the round's first item
  int32_t blocks; // workgroups of the round
};

struct PersistItem {
  int32_t round;  // index into the round table
  int32_t block;  // workgroup of that round's own launch
};

// blocks[g][k]: workgroups of round k of grid g; waves_per_block: waves each
// workgroup counts when it finishes.  Fills the round table and the items.
// Returns false if a count overflows 32 bits.
inline bool persist_schedule(const std::vector<std::vector<int32_t>>& blocks, int32_t waves_per_block,
                             std::vector<PersistRound>& rounds, std::vector<PersistItem>& items) {
  rounds.clear();
  items.clear();
  const size_t n = blocks.size();
  size_t kmax = 0;
  for (const auto& b : blocks) kmax = std::max(kmax, b.size());
  // the largest grids (by workgroups of their first round) first in each round index
  std::vector<size_t> order(n);
  std::iota(order.begin(), order.end(), size_t{0});
  std::stable_sort(order.begin(), order.end(), [&](size_t a, size_t b) {
    const int64_t wa = blocks[a].empty() ? 0 : blocks[a][0], wb = blocks[b].empty() ? 0 : blocks[b][0];
    return wa > wb;
  });
  std::vector<int64_t> done_before(n, 0);  // waves of the grid's rounds already listed
  int64_t ticket = 0;
  for (size_t k = 0; k < kmax; ++k) {
    for (size_t g : order) {
      if (k >= blocks[g].size()) continue;
      const int64_t nb = blocks[g][k];
      if (nb < 0 || done_before[g] > INT32_MAX || ticket + nb > INT32_MAX) return false;
      PersistRound r;
      r.grid = static_cast<int32_t>(g);
      r.round = static_cast<int32_t>(k);
      r.need = static_cast<int32_t>(done_before[g]);
      r.first = static_cast<int32_t>(ticket);
      r.blocks = static_cast<int32_t>(nb);
      const int32_t ri = static_cast<int32_t>(rounds.size());
      rounds.push_back(r);
      for (int64_t b = 0; b < nb; ++b) items.push_back(PersistItem{ri, static_cast<int32_t>(b)});
      ticket += nb;
      done_before[g] += nb * waves_per_block;
    }
  }
  return true;
}

}  // namespace s5d
