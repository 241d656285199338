// mcts_tree.h -- the MCTS allocation policy's tree and batch logic (host code), used by
// the device expansion's policy 2 and buildable alone on the CPU.
#pragma once
#include <algorithm>
#include <cmath>
#include <unordered_map>
#include <utility>
#include <vector>

#include "../../include/comet.h"
#include "keys.h"

namespace comet {

// MCTS allocation (policy 2): UCT over order prefixes on the host, one device evaluation
// per batch of batch_B selections.  Actions of a prefix of length d: "stop" (d >= 1) then
// "append id" (d < kcap) for the ids, in order, that keep it in the task's language; a
// node with untried actions expands the first, otherwise the walk takes the child of
// largest W/N + c sqrt(ln N_parent / N) (first on ties); every node of a path gets its
// visit at selection time (virtual loss).  A new "append" child of length d is completed by
// a rollout: K = d + out(8r) mod (kcap - d + 1), then for j = d .. K-1 the admissible id
// number out(8r+1+j) mod (count), out() being the SplitMix64 stream of sample_seed and r
// the rollout number.  Evaluated orders are cached (the budget counts distinct orders); a
// selection whose new order would exceed the budget is undone and ends the batch.  After
// the evaluation, the best value so far is updated and each path adds its reward: pushing
// J_best / J for feasible orders (0 otherwise), flipping M_best / M.  The search ends at
// the budget, when nothing is left untried and a batch brings no new order, or after 64
// batches in a row without one; then the refinement of the expansion.
// ---------------------------------------------------------------------------------
struct MctsNode {
  int len;
  int pre[KEY_MAXSEG];
  bool stop;
  std::vector<int> acts;   // untried actions (from `next`), -1 = stop
  size_t next = 0;
  std::vector<int> kids;   // child node indices in action order
  long long N = 0;
  double W = 0.0;
};

inline unsigned long long splitmix64_host(unsigned long long seed, unsigned long long i) {
  unsigned long long z = seed + (i + 1ull) * 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

struct MctsTree {
  int task, kcap, M;
  double c;
  unsigned long long seed, rollouts = 0;
  long long untried = 0;
  std::vector<MctsNode> nodes;

  bool admissible(const int* m, int n) const {
    return admissible_key(task, key_make(n, m, key_bits(task)));
  }
  void ids_after(const int* m, int n, std::vector<int>& out) const {
    out.clear();
    int q[KEY_MAXSEG];
    for (int i = 0; i < n; ++i) q[i] = m[i];
    for (int a = 0; a < M; ++a) {
      q[n] = a;
      if (admissible(q, n + 1)) out.push_back(a);
    }
  }
  int make(const int* pre, int len, bool stop) {
    MctsNode nd;
    nd.len = len;
    for (int i = 0; i < KEY_MAXSEG; ++i) nd.pre[i] = (i < len) ? pre[i] : 0;
    nd.stop = stop;
    if (!stop) {
      if (len >= 1) nd.acts.push_back(-1);
      if (len < kcap) {
        std::vector<int> ids;
        ids_after(pre, len, ids);
        nd.acts.insert(nd.acts.end(), ids.begin(), ids.end());
      }
    }
    untried += (long long)nd.acts.size();
    nodes.push_back(std::move(nd));
    return (int)nodes.size() - 1;
  }
  double uct(int parent, int child) const {
#pragma clang fp contract(off)
    const double n = (double)nodes[child].N;
    const double q = nodes[child].W / n;
    const double e = c * std::sqrt(std::log((double)nodes[parent].N) / n);
    return q + e;
  }
  // one selection: the path (node indices) and the order it yields
  void select(std::vector<int>& path, int* order, int& K) {
    path.clear();
    int v = 0;
    path.push_back(v);
    for (;;) {
      MctsNode& nd = nodes[v];
      if (nd.next < nd.acts.size()) {
        const int a = nd.acts[nd.next++];
        --untried;
        int pre[KEY_MAXSEG];
        for (int i = 0; i < nodes[v].len; ++i) pre[i] = nodes[v].pre[i];
        int len = nodes[v].len;
        bool stop = (a == -1);
        if (!stop) pre[len++] = a;
        const int ch = make(pre, len, stop);
        nodes[v].kids.push_back(ch);
        path.push_back(ch);
        break;
      }
      if (nd.kids.empty()) break;
      int best = -1;
      double bval = -INFINITY;
      for (int ch : nd.kids) {
        const double u = uct(v, ch);
        if (u > bval) {
          best = ch;
          bval = u;
        }
      }
      v = best;
      path.push_back(v);
    }
    const MctsNode& leaf = nodes[path.back()];
    K = leaf.len;
    for (int i = 0; i < K; ++i) order[i] = leaf.pre[i];
    if (!leaf.stop) rollout(order, K);
    for (int i : path) ++nodes[i].N;
  }
  void rollout(int* m, int& K) {
    const unsigned long long r = rollouts++;
    const int d = K;
    if (d >= kcap) return;
    const int target = d + (int)(splitmix64_host(seed, 8ull * r) % (unsigned long long)(kcap - d + 1));
    std::vector<int> cand;
    for (int j = d; j < target; ++j) {
      ids_after(m, K, cand);
      if (cand.empty()) break;
      m[K++] = cand[splitmix64_host(seed, 8ull * r + 1ull + (unsigned long long)j) % cand.size()];
    }
  }
};


// The search's batch logic around the evaluator: begin_batch() selects up to batch_B
// orders (fresh: the distinct new ones to evaluate, in selection order), end_batch() takes
// their (J, v), updates the cache and the best value, adds the rewards along every
// selected path and decides whether the search is over.
struct MctsSearch {
  MctsTree T;
  long long batch_B = 0, eval_budget = 0;
  double mu_merit = 100.0, eps = 1e-5;
  std::unordered_map<unsigned long long, std::pair<double, double>> cache;
  std::vector<unsigned long long> fresh, evaluated;
  std::vector<std::pair<std::vector<int>, unsigned long long>> sel;
  std::vector<int> path;
  long long nV = 0, batches = 0;
  int stall = 0;
  bool done = false;
  double best = INFINITY;

  void init(int task, int kcap, int M, double c, unsigned long long seed, long long B, long long budget,
            double mu, double eps_feas) {
    T.task = task;
    T.kcap = kcap;
    T.M = M;
    T.c = c;
    T.seed = seed;
    T.make(nullptr, 0, false);
    batch_B = B;
    eval_budget = budget;
    mu_merit = mu;
    eps = eps_feas;
  }
  double merit(double J, double v) const {
#pragma clang fp contract(off)
    return (std::isfinite(J) && std::isfinite(v)) ? J + mu_merit * std::fmax(v - eps, 0.0) : INFINITY;
  }
  bool begin_batch() {
    if (done || nV >= eval_budget || batches >= 1000000) return false;
    sel.clear();
    fresh.clear();
    for (long long q = 0; q < batch_B; ++q) {
      int order[KEY_MAXSEG], K = 0;
      T.select(path, order, K);
      const unsigned long long k = key_make(K, order, key_bits(T.task));
      if (!cache.count(k) && std::find(fresh.begin(), fresh.end(), k) == fresh.end()) {
        if (nV + (long long)fresh.size() >= eval_budget) {
          for (int i : path) --T.nodes[i].N;   // not taken
          break;
        }
        fresh.push_back(k);
      }
      sel.emplace_back(path, k);
    }
    ++batches;
    return true;
  }
  void end_batch(const double* J, const double* v) {
    const bool flip = (T.task == COMET_TASK_FLIP);
    const long long n = (long long)fresh.size();
    for (long long i = 0; i < n; ++i) {
      cache[fresh[i]] = {J[i], v[i]};
      evaluated.push_back(fresh[i]);
      if (flip) best = std::fmin(best, merit(J[i], v[i]));
      else if (v[i] <= eps && std::isfinite(J[i])) best = std::fmin(best, J[i]);
    }
    nV += n;
    for (const auto& sp : sel) {
      const auto& r = cache[sp.second];
      double rew = 0.0;
      if (flip) {
        const double Mi = merit(r.first, r.second);
        if (std::isfinite(Mi) && Mi > 0.0) rew = best / Mi;
      } else if (r.second <= eps && std::isfinite(r.first) && r.first > 0.0) {
        rew = best / r.first;
      }
      for (int i : sp.first) T.nodes[i].W += rew;
    }
    stall = (n > 0) ? 0 : stall + 1;
    if (n == 0 && (T.untried == 0 || stall >= 64)) done = true;
  }
};

}  // namespace comet
