// Driver of the host MCTS search (mcts_tree.h) for CPU runs (test infrastructure): drives
// MctsSearch with a synthetic evaluator, a fixed function of the order key that the Python
// test computes identically, and prints the evaluated keys in evaluation order.  Built
// host-only, with sanitizers.
//   mcts_driver task kcap P budget seed
#include <cstdio>
#include <cstdlib>
#include <vector>

#include "../../paper_2609_21803_amd/csrc/mcts_tree.h"

static unsigned long long fmix(unsigned long long h) {
  h ^= h >> 33;
  h *= 0xff51afd7ed558ccdull;
  h ^= h >> 33;
  h *= 0xc4ceb9fe1a85ec53ull;
  h ^= h >> 33;
  return h;
}

int main(int argc, char** argv) {
  if (argc != 6) return 2;
  const int task = atoi(argv[1]), kcap = atoi(argv[2]);
  const long long P = atoll(argv[3]), budget = atoll(argv[4]);
  const unsigned long long seed = strtoull(argv[5], nullptr, 10);
  comet::MctsSearch S;
  S.init(task, kcap, task == COMET_TASK_FLIP ? 845 : 12, 0.8, seed, P, budget, 100.0, 1e-5);
  std::vector<double> J, v;
  while (S.begin_batch()) {
    J.clear();
    v.clear();
    for (unsigned long long k : S.fresh) {
      const unsigned long long h = fmix(k);
      J.push_back(0.1 + (double)(h % 10007ull) / 10007.0);
      v.push_back(((h >> 20) % 3ull == 0ull) ? 0.0 : (double)((h >> 32) % 1000ull) * 1e-5);
    }
    S.end_batch(J.data(), v.data());
  }
  for (unsigned long long k : S.evaluated) printf("%llu\n", k);
  printf("batches %lld\n", S.batches);
  return 0;
}
