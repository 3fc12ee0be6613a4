// Host check of the persistent work list (persist_schedule.h), compiled and
// run by test_persist_schedule_cpu.py.  Usage: persist_schedule_check SEED
// GRIDS WORKERS.  Draws GRIDS grids with 0..12 rounds of 1..40 workgroups
// each, builds the work list, checks its invariants, then simulates WORKERS
// persistent workgroups that take tickets in order, wait on their grid's
// counter and finish in random order; the queue must drain.  Prints "ok" or
// the first violation.
#include <cstdio>
#include <cstdlib>
#include <random>
#include <vector>

#include "persist_schedule.h"

int main(int argc, char** argv) {
  if (argc != 4) {
    std::printf("usage: %s SEED GRIDS WORKERS\n", argv[0]);
    return 2;
  }
  const unsigned seed = static_cast<unsigned>(std::atoi(argv[1]));
  const int ngrids = std::atoi(argv[2]), nworkers = std::atoi(argv[3]);
  const int wpb = 4;  // waves per workgroup
  std::mt19937 rng(seed);
  std::vector<std::vector<int32_t>> blocks(ngrids);
  for (auto& b : blocks) {
    const int nr = static_cast<int>(rng() % 13);
    for (int k = 0; k < nr; ++k) b.push_back(1 + static_cast<int32_t>(rng() % 40));
  }
  std::vector<s5d::PersistRound> rounds;
  std::vector<s5d::PersistItem> items;
  if (!s5d::persist_schedule(blocks, wpb, rounds, items)) {
    std::printf("schedule failed\n");
    return 1;
  }
  // every (grid, round, workgroup) exactly once; rounds consistent
  std::vector<std::vector<std::vector<int>>> seen(ngrids);
  for (int g = 0; g < ngrids; ++g) {
    seen[g].resize(blocks[g].size());
    for (size_t k = 0; k < blocks[g].size(); ++k) seen[g][k].assign(blocks[g][k], 0);
  }
  for (size_t t = 0; t < items.size(); ++t) {
    const s5d::PersistItem& it = items[t];
    if (it.round < 0 || static_cast<size_t>(it.round) >= rounds.size()) {
      std::printf("item %zu: bad round index\n", t);
      return 1;
    }
    const s5d::PersistRound& r = rounds[it.round];
    if (it.block < 0 || it.block >= r.blocks || static_cast<int64_t>(t) != r.first + it.block) {
      std::printf("item %zu: block %d outside its round\n", t, it.block);
      return 1;
    }
    if (seen[r.grid][r.round][it.block]++) {
      std::printf("item %zu listed twice\n", t);
      return 1;
    }
  }
  for (int g = 0; g < ngrids; ++g)
    for (size_t k = 0; k < blocks[g].size(); ++k)
      for (int c : seen[g][k])
        if (c != 1) {
          std::printf("grid %d round %zu: a workgroup is missing\n", g, k);
          return 1;
        }
  // thresholds: every wave of the grid's earlier rounds, nothing more; and
  // every earlier round of the grid has smaller tickets
  for (const s5d::PersistRound& r : rounds) {
    int64_t want = 0;
    for (int k = 0; k < r.round; ++k) want += static_cast<int64_t>(blocks[r.grid][k]) * wpb;
    if (r.need != want) {
      std::printf("grid %d round %d: need %d, expected %lld\n", r.grid, r.round, r.need, static_cast<long long>(want));
      return 1;
    }
    for (const s5d::PersistRound& q : rounds)
      if (q.grid == r.grid && q.round < r.round && q.first + q.blocks > r.first) {
        std::printf("grid %d: round %d is queued after round %d\n", r.grid, q.round, r.round);
        return 1;
      }
  }
  // simulation: workers take tickets in order, wait for their threshold,
  // then run for a random number of steps; finishing adds the waves
  std::vector<int64_t> done(ngrids, 0);
  struct Worker {
    int64_t ticket = -1;
    int left = 0;
  };
  std::vector<Worker> w(nworkers);
  int64_t next = 0, finished = 0, idle_steps = 0;
  const int64_t n = static_cast<int64_t>(items.size());
  while (finished < n) {
    Worker& x = w[rng() % nworkers];
    bool progress = false;
    if (x.ticket < 0) {
      if (next < n) {
        x.ticket = next++;
        x.left = -1;  // not started
        progress = true;
      }
    } else {
      const s5d::PersistRound& r = rounds[items[x.ticket].round];
      if (x.left < 0) {
        if (done[r.grid] >= r.need) {
          x.left = 1 + static_cast<int>(rng() % 3);
          progress = true;
        }
      } else if (--x.left == 0) {
        done[r.grid] += wpb;
        ++finished;
        x.ticket = -1;
        progress = true;
      } else {
        progress = true;
      }
    }
    idle_steps = progress ? 0 : idle_steps + 1;
    if (idle_steps > 100000LL * nworkers) {
      std::printf("no progress: %lld of %lld items finished\n", static_cast<long long>(finished),
                  static_cast<long long>(n));
      return 1;
    }
  }
  std::printf("ok %zu rounds %zu items\n", rounds.size(), items.size());
  return 0;
}
