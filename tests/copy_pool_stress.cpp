// Host-side stress test of the ring drain's copy pool (copy_pool.h): many
// short runs back to back, each with its own function object and counters
// that die when the run returns.  Every chunk must run exactly once per run;
// built with -fsanitize=thread, a worker that touched a finished run's state
// would be reported as a race.
#include <cstdio>
#include <cstdlib>
#include <random>
#include <vector>

#include "../paper_1309_7963_amd/csrc/copy_pool.h"

int main(int argc, char** argv) {
  const int runs = argc > 1 ? atoi(argv[1]) : 20000;
  const int workers = argc > 2 ? atoi(argv[2]) : 4;
  std::mt19937 rng(12345);
  incdev::CopyPool pool(workers);
  long long total = 0;
  for (int r = 0; r < runs; ++r) {
    const int n = 1 + (int)(rng() % 48);
    std::vector<std::atomic<int>> hits(n);
    for (auto& h : hits) h.store(0);
    {
      std::function<void(int)> fn = [&hits, n](int c) {
        if (c < 0 || c >= n) abort();
        hits[c].fetch_add(1);
      };
      pool.run(n, fn);
    }
    for (int c = 0; c < n; ++c) {
      if (hits[c].load() != 1) {
        fprintf(stderr, "run %d: chunk %d ran %d times\n", r, c, hits[c].load());
        return 1;
      }
    }
    total += n;
  }
  printf("ok %d runs %lld chunks\n", runs, total);
  return 0;
}
