// expand.hip -- greedy contact-mode expansion (Alg. 1, Sec. III-B) on the device.
//
// The evaluated set V lives in device memory as (key, J, v, merit) rows plus an
// open-addressing hash set of keys (V together with the batch under construction).
// One round: evaluate the batch F_s with the persistent solver; append the scores to V;
// rank V by (merit of Eq. 5, key) with a stable LSD radix sort; for the W best-ranked
// orders generate every r-edit neighbour by its enumeration index in parallel (parent
// rank major, index minor, so the flat position is the traversal order of Alg. 1); keep
// the first occurrence of every unseen key (atomic minimum of the position per key);
// compact in position order and admit the first B orders as F_{s+1}.  After the last
// round the K_ref best feasible orders are re-solved with the refinement budget and the
// best refined feasible one is returned.  The whole loop, sizes included, stays on the
// device, so it is captured once as a HIP graph and replayed.
//
// Keys pack (K, m_0, ..., m_5): K << 60 | m_0 << 50 | m_1 << 40 | ... (10 bits per id), so
// comparing keys compares the segment count first and then the ids lexicographically.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <unordered_map>
#include <vector>

#include "internal.h"
#include "keys.h"
#include "mcts_tree.h"

namespace comet {

constexpr unsigned long long EMPTY = 0ull;
constexpr int SCAN_BLOCK = 256, SCAN_ITEMS = 4, SCAN_TILE = SCAN_BLOCK * SCAN_ITEMS;
constexpr int RS_TILE = 256;

// Number of raw one-edit neighbours: substitutions K(M-1), deletions K (K > 1),
// insertions (K+1) M (K < K_cap).
__host__ __device__ inline int raw1_count(int K, int M, int kcap) {
  return K * (M - 1) + (K > 1 ? K : 0) + (K < kcap ? (K + 1) * M : 0);
}

// The e-th raw one-edit neighbour in enumeration order (substitutions by position then
// id, skipping the current id; deletions by position; insertions by position then id).
// Returns 0 when e is out of range.
__host__ __device__ inline unsigned long long raw1_decode(unsigned long long p, int e, int M, int kcap, int w) {
  int m[KEY_MAXSEG], q[KEY_MAXSEG + 1];
  const int K = key_len(p);
  for (int i = 0; i < K; ++i) m[i] = key_mode(p, i, w);
  const int nsub = K * (M - 1), ndel = (K > 1) ? K : 0, nins = (K < kcap) ? (K + 1) * M : 0;
  if (e < 0) return EMPTY;
  if (e < nsub) {
    const int i = e / (M - 1), j = e % (M - 1);
    for (int t = 0; t < K; ++t) q[t] = m[t];
    q[i] = (j < m[i]) ? j : j + 1;
    return key_make(K, q, w);
  }
  e -= nsub;
  if (e < ndel) {
    int t = 0;
    for (int j = 0; j < K; ++j)
      if (j != e) q[t++] = m[j];
    return key_make(K - 1, q, w);
  }
  e -= ndel;
  if (e < nins) {
    const int i = e / M, id = e % M;
    int t = 0;
    for (int j = 0; j < i; ++j) q[t++] = m[j];
    q[t++] = id;
    for (int j = i; j < K; ++j) q[t++] = m[j];
    return key_make(K + 1, q, w);
  }
  return EMPTY;
}

// e-th raw neighbour within r edits: the one-edit list, then for every entry of that
// list (in order) its own one-edit list, each padded to raw1max slots.  For a task with a
// language an entry of the one-edit list outside it starts no second edit (Sec. III-B:
// every intermediate order of an r-edit path stays admissible).
__host__ __device__ inline unsigned long long raw_decode(unsigned long long p, long long e, int M, int kcap, int radius,
                                                          int raw1max, int task) {
  const int w = key_bits(task);
  const int n1 = raw1_count(key_len(p), M, kcap);
  if (e < n1) return raw1_decode(p, (int)e, M, kcap, w);
  if (radius < 2) return EMPTY;
  const long long t = e - n1;
  const long long q = t / raw1max;
  const int e2 = (int)(t % raw1max);
  if (q >= n1) return EMPTY;
  const unsigned long long k1 = raw1_decode(p, (int)q, M, kcap, w);
  if (!admissible_key(task, k1)) return EMPTY;
  return (e2 < raw1_count(key_len(k1), M, kcap)) ? raw1_decode(k1, e2, M, kcap, w) : EMPTY;
}

// Table slot of a key.  Keys carry their information in the high bits (segment count and
// the leading ids), so the slot must depend on every bit: the 64-bit finaliser of
// MurmurHash3 (Appleby) mixes them into the low bits the mask keeps.
__device__ inline unsigned long long hash_slot(unsigned long long k, unsigned long long mask) {
  k ^= k >> 33;
  k *= 0xff51afd7ed558ccdull;
  k ^= k >> 33;
  k *= 0xc4ceb9fe1a85ec53ull;
  k ^= k >> 33;
  return k & mask;
}

__device__ inline void set_insert(unsigned long long* tab, unsigned long long mask, unsigned long long k) {
  unsigned long long s = hash_slot(k, mask);
  for (;;) {
    const unsigned long long prev = atomicCAS(&tab[s], EMPTY, k);
    if (prev == EMPTY || prev == k) return;
    s = (s + 1) & mask;
  }
}

__device__ inline bool set_has(const unsigned long long* tab, unsigned long long mask, unsigned long long k) {
  unsigned long long s = hash_slot(k, mask);
  for (;;) {
    const unsigned long long v = tab[s];
    if (v == k) return true;
    if (v == EMPTY) return false;
    s = (s + 1) & mask;
  }
}

// insert k if absent and lower its recorded first position to pos
__device__ inline void first_insert(unsigned long long* keys, unsigned* minpos, unsigned long long mask,
                                    unsigned long long k, unsigned pos) {
  unsigned long long s = hash_slot(k, mask);
  for (;;) {
    const unsigned long long prev = atomicCAS(&keys[s], EMPTY, k);
    if (prev == EMPTY || prev == k) {
      atomicMin(&minpos[s], pos);
      return;
    }
    s = (s + 1) & mask;
  }
}

__device__ inline unsigned first_lookup(const unsigned long long* keys, const unsigned* minpos,
                                        unsigned long long mask, unsigned long long k) {
  unsigned long long s = hash_slot(k, mask);
  for (;;) {
    const unsigned long long v = keys[s];
    if (v == k) return minpos[s];
    if (v == EMPTY) return 0xFFFFFFFFu;
    s = (s + 1) & mask;
  }
}

// double -> unsigned with the same order (NaN ranks as +inf)
__device__ inline unsigned long long order_bits(double d) {
  if (isnan(d)) d = INFINITY;
  if (d == 0.0) d = 0.0;
  const unsigned long long u = (unsigned long long)__double_as_longlong(d);
  return (u >> 63) ? ~u : (u | 0x8000000000000000ull);
}

// ---------------------------------------------------------------------------------
// Generic device utilities: fill, exclusive scan of uint32 (sizes on the device),
// stable LSD radix sort of (hi, lo) 128-bit keys with a 32-bit payload.
// ---------------------------------------------------------------------------------
__global__ void k_fill_u64(unsigned long long* p, unsigned long long v, long long n) {
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
    p[i] = v;
}
__global__ void k_fill_u32(unsigned* p, unsigned v, long long n) {
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
    p[i] = v;
}

__device__ inline long long dev_n(const long long* n_dev, long long n_host) { return n_dev ? *n_dev : n_host; }

// per-tile sums
__global__ __launch_bounds__(SCAN_BLOCK) void k_scan_reduce(const unsigned* in, const long long* n_dev, long long n_host,
                                                            unsigned* tile_sums) {
  __shared__ unsigned sh[SCAN_BLOCK];
  const long long n = dev_n(n_dev, n_host);
  const long long base = (long long)blockIdx.x * SCAN_TILE;
  unsigned s = 0;
  for (int i = 0; i < SCAN_ITEMS; ++i) {
    const long long j = base + (long long)threadIdx.x * SCAN_ITEMS + i;
    if (j < n) s += in[j];
  }
  sh[threadIdx.x] = s;
  __syncthreads();
  for (int o = SCAN_BLOCK / 2; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) sh[threadIdx.x] += sh[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) tile_sums[blockIdx.x] = sh[0];
}

// exclusive scan of the tile sums in one block; total to *total
__global__ __launch_bounds__(1024) void k_scan_tiles(unsigned* tile_sums, long long ntiles, unsigned long long* total) {
  __shared__ unsigned sh[1024];
  const long long per = (ntiles + 1023) / 1024;
  const long long b0 = (long long)threadIdx.x * per;
  unsigned s = 0;
  for (long long i = 0; i < per; ++i)
    if (b0 + i < ntiles) s += tile_sums[b0 + i];
  sh[threadIdx.x] = s;
  __syncthreads();
  for (int o = 1; o < 1024; o <<= 1) {  // inclusive Hillis-Steele
    const unsigned v = ((int)threadIdx.x >= o) ? sh[threadIdx.x - o] : 0u;
    __syncthreads();
    sh[threadIdx.x] += v;
    __syncthreads();
  }
  unsigned run = (threadIdx.x == 0) ? 0u : sh[threadIdx.x - 1];
  for (long long i = 0; i < per; ++i)
    if (b0 + i < ntiles) {
      const unsigned c = tile_sums[b0 + i];
      tile_sums[b0 + i] = run;
      run += c;
    }
  if (threadIdx.x == 1023 && total) *total = sh[1023];
}

// exclusive scan within each tile plus the tile offset
__global__ __launch_bounds__(SCAN_BLOCK) void k_scan_apply(const unsigned* in, const long long* n_dev, long long n_host,
                                                           const unsigned* tile_off, unsigned* out) {
  __shared__ unsigned sh[SCAN_BLOCK];
  const long long n = dev_n(n_dev, n_host);
  const long long base = (long long)blockIdx.x * SCAN_TILE + (long long)threadIdx.x * SCAN_ITEMS;
  unsigned v[SCAN_ITEMS], s = 0;
  for (int i = 0; i < SCAN_ITEMS; ++i) {
    v[i] = (base + i < n) ? in[base + i] : 0u;
    s += v[i];
  }
  sh[threadIdx.x] = s;
  __syncthreads();
  for (int o = 1; o < SCAN_BLOCK; o <<= 1) {
    const unsigned t = ((int)threadIdx.x >= o) ? sh[threadIdx.x - o] : 0u;
    __syncthreads();
    sh[threadIdx.x] += t;
    __syncthreads();
  }
  unsigned run = tile_off[blockIdx.x] + ((threadIdx.x == 0) ? 0u : sh[threadIdx.x - 1]);
  for (int i = 0; i < SCAN_ITEMS; ++i) {
    if (base + i < n) out[base + i] = run;
    run += v[i];
  }
}

struct Scanner {
  unsigned* tiles = nullptr;
  long long max_tiles = 0;
  // exclusive scan in -> out over n (device size if n_dev, capacity nmax for the grid)
  void run(hipStream_t s, const unsigned* in, unsigned* out, const long long* n_dev, long long nmax,
           unsigned long long* total) {
    const long long nt = std::max<long long>(1, (nmax + SCAN_TILE - 1) / SCAN_TILE);
    hipLaunchKernelGGL(k_scan_reduce, dim3((unsigned)nt), dim3(SCAN_BLOCK), 0, s, in, n_dev, nmax, tiles);
    hipLaunchKernelGGL(k_scan_tiles, dim3(1), dim3(1024), 0, s, tiles, nt, total);
    hipLaunchKernelGGL(k_scan_apply, dim3((unsigned)nt), dim3(SCAN_BLOCK), 0, s, in, n_dev, nmax, tiles, out);
  }
};

__device__ inline unsigned rs_digit(unsigned long long hi, unsigned long long lo, int pass) {
  return (pass < 8) ? (unsigned)((lo >> (8 * pass)) & 255ull) : (unsigned)((hi >> (8 * (pass - 8))) & 255ull);
}

// digit histogram of each tile, stored digit-major: counts[d * ntiles + tile]
__global__ __launch_bounds__(RS_TILE) void k_rs_count(const unsigned long long* hi, const unsigned long long* lo,
                                                      const long long* n_dev, int pass, long long ntiles,
                                                      unsigned* counts) {
  __shared__ unsigned h[256];
  h[threadIdx.x] = 0;
  __syncthreads();
  const long long n = *n_dev;
  const long long i = (long long)blockIdx.x * RS_TILE + threadIdx.x;
  if (i < n) atomicAdd(&h[rs_digit(hi[i], lo[i], pass)], 1u);
  __syncthreads();
  counts[(long long)threadIdx.x * ntiles + blockIdx.x] = h[threadIdx.x];
}

// stable scatter: destination = scanned offset of (digit, tile) + rank among equal
// digits earlier in the tile
__global__ __launch_bounds__(RS_TILE) void k_rs_scatter(const unsigned long long* hi, const unsigned long long* lo,
                                                        const unsigned* val, const long long* n_dev, int pass,
                                                        long long ntiles, const unsigned* offs, unsigned long long* hi2,
                                                        unsigned long long* lo2, unsigned* val2) {
  __shared__ unsigned dg[RS_TILE];
  const long long n = *n_dev;
  const long long i = (long long)blockIdx.x * RS_TILE + threadIdx.x;
  const bool in = i < n;
  const unsigned d = in ? rs_digit(hi[i], lo[i], pass) : 0xFFFFu;
  dg[threadIdx.x] = d;
  __syncthreads();
  if (!in) return;
  unsigned r = 0;
  for (unsigned j = 0; j < threadIdx.x; ++j) r += (dg[j] == d) ? 1u : 0u;
  const unsigned dst = offs[(long long)d * ntiles + blockIdx.x] + r;
  hi2[dst] = hi[i];
  lo2[dst] = lo[i];
  val2[dst] = val[i];
}

// ---------------------------------------------------------------------------------
// Expansion kernels
// ---------------------------------------------------------------------------------
struct ExpCounters {
  long long nV;                  // evaluated orders
  long long nF;                  // orders in the current batch
  long long room;                // capacity of the next batch
  long long nRef;                // orders in the refinement batch
  long long rounds;              // evaluation rounds run
  long long n_feas;              // feasible evaluated orders
  unsigned long long first_feas; // 1-based evaluation index of the first feasible order (0 = none)
  unsigned long long kept;       // unseen first-occurrence candidates of the last generation
  unsigned long long t_start, t_first;
  unsigned long long best_key;
  long long best_row;
  double best_J, best_v;
  long long nCand;               // candidate slots of the current generation
  unsigned long long draw_base;  // sampling: number of the next round's first draw
};

struct ExpCfg {
  int M, kcap, radius, W, raw1max, knots_per_segment, n_total, k_ref;
  int task, row;                 // task, trajectory row width (x_k, u_k)
  int policy;                    // 0 expansion, 1 uniform sampling
  unsigned long long sseed;      // sampling: SplitMix64 seed
  long long draws;               // sampling: draws per round
  long long rawmax, Bmax, budget, Vcap;
  unsigned long long vmask, cmask;
  double eps, mu_merit;
};

__global__ void k_exp_init(ExpCounters* C) {
  C->nV = 0; C->nF = 0; C->room = 0; C->nRef = 0; C->rounds = 0; C->n_feas = 0;
  C->first_feas = ~0ull; C->kept = 0; C->t_first = ~0ull; C->best_key = 0; C->best_row = -1;
  C->best_J = NAN; C->best_v = INFINITY; C->nCand = 0; C->draw_base = 0;
  C->t_start = (unsigned long long)wall_clock64();
}

// seed: every order with 1..kmax segments in key order, capped at the batch / budget
__global__ void k_seed(ExpCfg g, int kmax, long long n_seed, ExpCounters* C, unsigned long long* F,
                       unsigned long long* vset) {
  const long long cap = min(g.Bmax, g.budget);
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t == 0) C->nF = min(n_seed, cap);
  if (t >= n_seed || t >= cap) return;
  long long c = t, cnt = g.M;
  int K = 1;
  while (K < kmax && c >= cnt) {
    c -= cnt;
    ++K;
    cnt *= g.M;
  }
  int q[KEY_MAXSEG];
  for (int i = K - 1; i >= 0; --i) {
    q[i] = (int)(c % g.M);
    c /= g.M;
  }
  const unsigned long long k = key_make(K, q, key_bits(g.task));
  F[t] = k;
  set_insert(vset, g.vmask, k);
}

// seed as candidates (languages with a filter): slot t holds the t-th order of 1..kmax
// segments in key order, or EMPTY if it is not admissible; the candidate pipeline then
// keeps the admissible ones in order.  Pushing with free motion enumerates its language
// directly (slot t = the t-th admissible order, read off the continuation counts fc): its
// product space of eight segments (16^8 orders) is too large to filter.
__global__ void k_seed_cand(ExpCfg g, int kmax, long long n_seed, ExpCounters* C, unsigned long long* ckey,
                            unsigned long long* hkeys, unsigned* hmin, FreeCounts fc) {
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t == 0) {
    C->nCand = n_seed;
    C->room = min(g.Bmax, g.budget);
    C->kept = 0;
  }
  if (t >= n_seed) return;
  unsigned long long k;
  if (is_free_task(g.task)) {
    long long c = t;
    int K = 1;
    for (long long n = free_count_len(fc, 1); K < kmax && c >= n; n = free_count_len(fc, K)) {
      c -= n;
      ++K;
    }
    k = free_unrank(fc, K, c);
  } else {
    long long c = t, cnt = g.M;
    int K = 1;
    while (K < kmax && c >= cnt) {
      c -= cnt;
      ++K;
      cnt *= g.M;
    }
    int q[KEY_MAXSEG];
    for (int i = K - 1; i >= 0; --i) {
      q[i] = (int)(c % g.M);
      c /= g.M;
    }
    k = key_make(K, q, key_bits(g.task));
    if (!admissible_key(g.task, k)) k = EMPTY;
  }
  ckey[t] = k;
  if (k != EMPTY) first_insert(hkeys, hmin, g.cmask, k, (unsigned)t);
}

// batch keys -> evaluator inputs (segment counts, ids, interval allocation)
__global__ void k_build(ExpCfg g, const long long* n_dev, const unsigned long long* F, int32_t* nseg, int32_t* modes,
                        int32_t* knots, int smax) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= *n_dev) return;
  const unsigned long long k = F[i];
  const int K = key_len(k);
  nseg[i] = K;
  for (int j = 0; j < smax; ++j) {
    const bool live = j < K;
    modes[i * smax + j] = live ? key_mode(k, j, key_bits(g.task)) : 0;
    int n = 0;
    if (live) n = (g.knots_per_segment > 0) ? g.knots_per_segment : g.n_total / K + ((j < g.n_total % K) ? 1 : 0);
    knots[i * smax + j] = n;
  }
}

// Eq. (5); the product and the sum are rounded separately (no fused multiply-add), so the
// merit of an order is the same number whichever side computes it.
__device__ inline double merit_of(double J, double v, double eps, double mu) {
#pragma clang fp contract(off)
  if (isnan(J) || isnan(v)) return INFINITY;
  const double M = J + mu * fmax(v - eps, 0.0);
  return isnan(M) ? INFINITY : M;
}

__global__ void k_append(ExpCfg g, ExpCounters* C, const unsigned long long* F, const double* J, const double* v,
                         unsigned long long* vkey, double* vJ, double* vv, double* vM) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const bool in = i < C->nF;
  const long long j = C->nV + i;
  bool feas = false;
  if (in) {
    vkey[j] = F[i];
    vJ[j] = J[i];
    vv[j] = v[i];
    vM[j] = merit_of(J[i], v[i], g.eps, g.mu_merit);
    feas = v[i] <= g.eps;
  }
  // one update of the counters per wave: the feasible lanes' count, and the first of them
  // (lanes hold consecutive positions, so the lowest feasible lane has the smallest j)
  const unsigned long long m = __ballot(feas);
  if (m) {
    const int lead = __ffsll((long long)m) - 1;
    if ((int)(threadIdx.x & 63) == lead) {
      atomicAdd((unsigned long long*)&C->n_feas, (unsigned long long)__popcll(m));
      atomicMin(&C->first_feas, (unsigned long long)(j + 1));
    }
  }
}

__global__ void k_advance(ExpCfg g, ExpCounters* C) {
  C->nV += C->nF;
  if (C->nF > 0) C->rounds += 1;
  C->nF = 0;
  C->room = max(0ll, min(g.Bmax, g.budget - C->nV));
  C->nCand = (C->room > 0) ? (g.policy ? g.draws : (long long)min((long long)g.W, C->nV) * g.rawmax) : 0;
  C->kept = 0;
}

// output i of the SplitMix64 stream seeded with `seed`
__device__ inline unsigned long long splitmix64_out(unsigned long long seed, unsigned long long i) {
  unsigned long long z = seed + (i + 1ull) * 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

// uniform sampling: draw C->draw_base + t for slot t < nCand; outside the language or
// already evaluated -> EMPTY; first occurrences are marked as for generated candidates.
// Free motion draws the index of an admissible order of K segments and unranks it (fc):
// its eight-segment orders are too rare in the product space to find by rejection.
__global__ void k_sample(ExpCfg g, const ExpCounters* C, const unsigned long long* vset, unsigned long long* ckey,
                         unsigned long long* hkeys, unsigned* hmin, FreeCounts fc) {
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= C->nCand) return;
  const unsigned long long c = C->draw_base + (unsigned long long)t;
  const int K = 1 + (int)(splitmix64_out(g.sseed, 8ull * c) % (unsigned long long)g.kcap);
  unsigned long long k;
  if (is_free_task(g.task)) {
    const unsigned long long n = (unsigned long long)free_count_len(fc, K);
    k = free_unrank(fc, K, (long long)(splitmix64_out(g.sseed, 8ull * c + 1ull) % n));
  } else {
    int m[KEY_MAXSEG] = {};
    for (int j = 0; j < K; ++j) m[j] = (int)(splitmix64_out(g.sseed, 8ull * c + 1ull + j) % (unsigned long long)g.M);
    k = key_make(K, m, key_bits(g.task));
    if (!admissible_key(g.task, k)) k = EMPTY;
  }
  if (k != EMPTY && set_has(vset, g.vmask, k)) k = EMPTY;
  ckey[t] = k;
  if (k != EMPTY) first_insert(hkeys, hmin, g.cmask, k, (unsigned)t);
}

// first sampled batch: room and draw count; later rounds move the draw numbers on
__global__ void k_sample_start(ExpCfg g, ExpCounters* C) {
  C->room = min(g.Bmax, g.budget);
  C->nCand = g.draws;
  C->kept = 0;
}
__global__ void k_sample_done(ExpCfg g, ExpCounters* C) {
  C->nF = min((long long)C->kept, C->room);
  C->draw_base += (unsigned long long)g.draws;
}

// ranking keys: (merit, key) or, for refinement, (J if feasible else +inf, key)
__global__ void k_rank_keys(ExpCfg g, const ExpCounters* C, int refine, const unsigned long long* vkey, const double* vJ,
                            const double* vv, const double* vM, unsigned long long* hi, unsigned long long* lo,
                            unsigned* idx) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= C->nV) return;
  const double r = refine ? ((vv[i] <= g.eps && isfinite(vJ[i])) ? vJ[i] : INFINITY) : vM[i];
  hi[i] = order_bits(r);
  lo[i] = vkey[i];
  idx[i] = (unsigned)i;
}

// candidates of the W best-ranked orders, flat position = rank * rawmax + index
__global__ void k_gen(ExpCfg g, const ExpCounters* C, const unsigned* ranked, const unsigned long long* vkey,
                      const unsigned long long* vset, unsigned long long* ckey, unsigned long long* hkeys,
                      unsigned* hmin) {
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= C->nCand) return;
  const long long p = t / g.rawmax, e = t % g.rawmax;
  const unsigned long long parent = vkey[ranked[p]];
  unsigned long long k = raw_decode(parent, e, g.M, g.kcap, g.radius, g.raw1max, g.task);
  if (k != EMPTY && !admissible_key(g.task, k)) k = EMPTY;
  if (k != EMPTY && set_has(vset, g.vmask, k)) k = EMPTY;
  ckey[t] = k;
  if (k != EMPTY) first_insert(hkeys, hmin, g.cmask, k, (unsigned)t);
}

__global__ void k_first(ExpCfg g, const ExpCounters* C, const unsigned long long* ckey, const unsigned long long* hkeys,
                        const unsigned* hmin, unsigned* flag) {
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= C->nCand) return;
  const unsigned long long k = ckey[t];
  flag[t] = (k != EMPTY && first_lookup(hkeys, hmin, g.cmask, k) == (unsigned)t) ? 1u : 0u;
}

__global__ void k_compact(ExpCfg g, ExpCounters* C, const unsigned long long* ckey, const unsigned* flag,
                          const unsigned* pos, unsigned long long* F, unsigned long long* vset) {
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= C->nCand || !flag[t]) return;
  const long long r = pos[t];
  if (r < C->room) {
    F[r] = ckey[t];
    set_insert(vset, g.vmask, ckey[t]);
  }
}

__global__ void k_set_batch(ExpCounters* C) { C->nF = min((long long)C->kept, C->room); }

__global__ void k_vset_fill(ExpCfg g, const unsigned long long* keys, long long n, unsigned long long* vset) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) set_insert(vset, g.vmask, keys[i]);
}

// refinement batch: the first min(K_ref, #feasible) orders of the refinement ranking
__global__ void k_ref_batch(ExpCfg g, ExpCounters* C, const unsigned* ranked, const unsigned long long* vkey,
                            const double* vJ, const double* vv, unsigned long long* F) {
  const long long r = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const long long nr = min((long long)g.k_ref, C->nV);
  if (r >= nr) return;
  const unsigned i = ranked[r];
  const bool ok = vv[i] <= g.eps && isfinite(vJ[i]);
  F[r] = ok ? vkey[i] : EMPTY;
  if (ok) atomicMax((unsigned long long*)&C->nRef, (unsigned long long)(r + 1));
}

__global__ void k_pick_best(ExpCfg g, ExpCounters* C, const unsigned long long* F, const double* J, const double* v) {
  unsigned long long bk = 0;
  double bJ = NAN, bv = INFINITY;
  long long row = -1;
  for (long long r = 0; r < C->nRef; ++r) {
    if (!(v[r] <= g.eps) || !isfinite(J[r])) continue;
    if (bk == 0 || J[r] < bJ || (J[r] == bJ && F[r] < bk)) {
      bk = F[r];
      bJ = J[r];
      bv = v[r];
      row = r;
    }
  }
  C->best_key = bk;
  C->best_J = bJ;
  C->best_v = bv;
  C->best_row = row;
}

// learned ordering: predicted merit expm1(cost head) + mu (1 - sigmoid(logit)), ties by key
__global__ void k_learned_keys(ExpCfg g, const ExpCounters* C, const float* Y, int O, const unsigned long long* F,
                               unsigned long long* hi, unsigned long long* lo, unsigned* idx) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= C->nF) return;
  const double p = 1.0 / (1.0 + exp(-(double)Y[i * O + 0]));
  const double m = expm1(fmin((double)Y[i * O + 1], 50.0)) + g.mu_merit * (1.0 - p);
  hi[i] = order_bits(m);
  lo[i] = F[i];
  idx[i] = (unsigned)i;
}

// gather the batch into queue order: tmp arrays, then back
__global__ void k_gather_batch(const ExpCounters* C, const unsigned* perm, const unsigned long long* F,
                               const int32_t* nseg, const int32_t* modes, const int32_t* knots, int smax,
                               unsigned long long* F2, int32_t* nseg2, int32_t* modes2, int32_t* knots2) {
  const long long r = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= C->nF) return;
  const long long i = perm[r];
  F2[r] = F[i];
  nseg2[r] = nseg[i];
  for (int j = 0; j < smax; ++j) {
    modes2[r * smax + j] = modes[i * smax + j];
    knots2[r * smax + j] = knots[i * smax + j];
  }
}

__global__ void k_copy_batch(const ExpCounters* C, const unsigned long long* F2, const int32_t* nseg2,
                             const int32_t* modes2, const int32_t* knots2, int smax, unsigned long long* F, int32_t* nseg,
                             int32_t* modes, int32_t* knots) {
  const long long r = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= C->nF) return;
  F[r] = F2[r];
  nseg[r] = nseg2[r];
  for (int j = 0; j < smax; ++j) {
    modes[r * smax + j] = modes2[r * smax + j];
    knots[r * smax + j] = knots2[r * smax + j];
  }
}

__global__ void k_gather_warm(const ExpCounters* C, const unsigned* perm, const float* src, long long row,
                              float* dst) {
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const long long r = t / row, c = t % row;
  if (r >= C->nF) return;
  dst[t] = src[(long long)perm[r] * row + c];
}

__global__ void k_best_out(ExpCfg g, const ExpCounters* C, const float* rtraj, int nmax1, int32_t* best_nseg,
                           int32_t* best_modes, int32_t* best_knots, float* best_cost, float* best_viol,
                           float* best_traj, int smax) {
  const int t = threadIdx.x;
  const unsigned long long k = C->best_key;
  const int K = key_len(k);
  if (t == 0) {
    *best_nseg = (k == 0) ? 0 : K;
    *best_cost = (float)C->best_J;
    *best_viol = (float)C->best_v;
  }
  if (t < smax) {
    const bool live = (k != 0) && t < K;
    best_modes[t] = live ? key_mode(k, t, key_bits(g.task)) : 0;
    best_knots[t] = live ? ((g.knots_per_segment > 0) ? g.knots_per_segment
                                                      : g.n_total / K + ((t < g.n_total % K) ? 1 : 0))
                         : 0;
  }
  if (best_traj)
    for (int i = t; i < nmax1 * g.row; i += blockDim.x)
      best_traj[i] = (C->best_row >= 0) ? rtraj[C->best_row * (long long)nmax1 * g.row + i] : 0.f;
}

}  // namespace comet

// ==================================================================================
// Host: work space, graph, ABI
// ==================================================================================
using namespace comet;

struct comet_expand_ws {
  ExpCfg cfg;
  comet_expand_params prm;
  long long ntiles_rs = 0;
  // device buffers
  ExpCounters* C = nullptr;
  unsigned long long *vkey = nullptr, *vset = nullptr;
  double *vJ = nullptr, *vv = nullptr, *vM = nullptr;
  unsigned long long *s_hi[2] = {nullptr, nullptr}, *s_lo[2] = {nullptr, nullptr};
  unsigned* s_idx[2] = {nullptr, nullptr};
  unsigned* rs_counts = nullptr;
  unsigned long long *ckey = nullptr, *hkeys = nullptr;
  unsigned *hmin = nullptr, *cflag = nullptr, *cpos = nullptr;
  Scanner scan;
  unsigned long long* F = nullptr;
  int32_t *fnseg = nullptr, *fmodes = nullptr, *fknots = nullptr;
  float *ecost = nullptr, *eviol = nullptr, *rtraj = nullptr;
  uint8_t* efeas = nullptr;
  double *ecost64 = nullptr, *eviol64 = nullptr;
  float *ix0 = nullptr, *igoal = nullptr, *iinst = nullptr;
  int32_t *o_nseg = nullptr, *o_modes = nullptr, *o_knots = nullptr;
  float *o_cost = nullptr, *o_viol = nullptr, *o_traj = nullptr;
  long long* dev_nV = nullptr;     // scratch scalars for expand_next
  unsigned long long* F2 = nullptr;  // learned mode: batch in predicted-merit order
  int32_t *fnseg2 = nullptr, *fmodes2 = nullptr, *fknots2 = nullptr;
  float *warm_tmp = nullptr, *warm = nullptr;
  comet_mlp* learned = nullptr;      // network the captured graph uses (null = plain)
  long long ccap = 0;                // candidate slots allocated (ckey, cflag, cpos)
  hipGraphExec_t gexec = nullptr;
  bool graph_valid = false;
  double wall_khz = 100000.0;
};

namespace comet {

void destroy_expand_ws(comet_ctx* c) {
  comet_expand_ws* w = c->xws;
  if (!w) return;
  if (w->gexec) (void)hipGraphExecDestroy(w->gexec);
  void* ptrs[] = {w->C, w->vkey, w->vset, w->vJ, w->vv, w->vM, w->s_hi[0], w->s_hi[1], w->s_lo[0], w->s_lo[1],
                  w->s_idx[0], w->s_idx[1], w->rs_counts, w->ckey, w->hkeys, w->hmin, w->cflag, w->cpos,
                  w->scan.tiles, w->F, w->fnseg, w->fmodes, w->fknots, w->ecost, w->eviol, w->rtraj, w->efeas,
                  w->ecost64, w->eviol64, w->ix0, w->igoal, w->iinst, w->o_nseg, w->o_modes, w->o_knots,
                  w->o_cost, w->o_viol, w->o_traj, w->dev_nV, w->F2, w->fnseg2, w->fmodes2, w->fknots2,
                  w->warm_tmp, w->warm};
  for (void* p : ptrs)
    if (p) (void)hipFree(p);
  delete w;
  c->xws = nullptr;
}

}  // namespace comet

namespace {

unsigned long long pow2_at_least(unsigned long long n) {
  unsigned long long p = 16;
  while (p < n) p <<= 1;
  return p;
}

unsigned blocks(long long n, int bs) { return (unsigned)std::max<long long>(1, (n + bs - 1) / bs); }

comet_status check_expand_params(comet_ctx* c, const comet_expand_params* p) {
  if (!p) return fail_msg(c, COMET_EINVAL, "null expand params");
  if (p->kcap < 1 || p->kcap > c->max_segments) return fail_msg(c, COMET_EINVAL, "kcap outside [1, max_segments]");
  if (p->radius < 1 || p->radius > 2) return fail_msg(c, COMET_EINVAL, "radius must be 1 or 2");
  if (p->rounds < 0 || p->frontier_W < 1 || p->batch_B < 1 || p->eval_budget < 1 || p->k_ref < 0)
    return fail_msg(c, COMET_EINVAL, "bad expand sizes");
  if (p->batch_B > c->max_batch || p->k_ref > c->max_batch)
    return fail_msg(c, COMET_EINVAL, "batch_B and k_ref must not exceed the context's max_batch");
  if (p->seed_max_segments < 1) return fail_msg(c, COMET_EINVAL, "seed_max_segments must be >= 1");
  const long long N = (p->knots_per_segment > 0) ? (long long)p->knots_per_segment * p->kcap : p->n_total;
  if (N < 1 || N > c->max_intervals || (p->knots_per_segment <= 0 && p->n_total < p->kcap))
    return fail_msg(c, COMET_EINVAL, "interval allocation exceeds max_intervals (or n_total < kcap)");
  if (!(p->mu_merit >= 0)) return fail_msg(c, COMET_EINVAL, "mu_merit must be >= 0");
  if (p->policy != COMET_POLICY_EXPAND && p->policy != COMET_POLICY_UNIFORM && p->policy != COMET_POLICY_MCTS)
    return fail_msg(c, COMET_EINVAL, "unknown search policy");
  if (p->policy == COMET_POLICY_MCTS && !(p->uct_c >= 0.0 && std::isfinite(p->uct_c)))
    return fail_msg(c, COMET_EINVAL, "uct_c must be finite and >= 0");
  if (p->policy == COMET_POLICY_UNIFORM && (p->sample_draws < 1 || p->sample_draws > (1ll << 27)))
    return fail_msg(c, COMET_EINVAL, "sample_draws must be in [1, 2^27]");
  return COMET_OK;
}

// slots of the seed pass: every order of 1..kmax segments of the product space (filtered
// on the device by the task's language), or, with free motion, its admissible orders only
long long seed_slots(int task, int M, int kmax) {
  long long n = 0, t = 1;
  if (is_free_task(task)) {
    const FreeCounts f = free_counts();
    for (int K = 1; K <= kmax; ++K) n += free_count_len(f, K);
    return n;
  }
  for (int K = 1; K <= kmax; ++K) {
    t *= M;
    n += t;
  }
  return n;
}

comet_status ensure_ws(comet_ctx* c, const comet_expand_params* p) {
  const bool flip = (c->task == COMET_TASK_FLIP), lang = task_has_language(c->task);
  const int M = flip ? 845 : (is_free_task(c->task) ? push_free::NMODES : push::NMODES);
  const int rowW = flip ? 17
                   : c->task == COMET_TASK_PUSH_TIMED ? 8
                   : c->task == COMET_TASK_PUSH_FREE ? 9
                   : c->task == COMET_TASK_PUSH_FREE_TIMED ? 10 : 7;
  int raw1max = 0;
  for (int K = 1; K <= p->kcap; ++K) raw1max = std::max(raw1max, raw1_count(K, M, p->kcap));
  const long long rawmax = (p->radius >= 2) ? (long long)raw1max + (long long)raw1max * raw1max : raw1max;
  const long long n_seed = seed_slots(c->task, M, std::min(p->seed_max_segments, p->kcap));
  const bool sampling = p->policy == COMET_POLICY_UNIFORM;
  const long long ncand = (p->policy == COMET_POLICY_MCTS) ? 1
                          : sampling ? p->sample_draws : std::max(rawmax * p->frontier_W, lang ? n_seed : 0ll);
  if (ncand > (1ll << 27)) return fail_msg(c, COMET_EINVAL, "frontier_W x neighbourhood size exceeds 2^27 candidates");
  const long long Vcap = p->eval_budget + p->batch_B + 16;
  comet_expand_ws* w = c->xws;
  const bool fits = w && w->cfg.Vcap >= Vcap && w->ccap >= ncand && w->cfg.Bmax >= p->batch_B &&
                    w->cfg.k_ref >= p->k_ref;
  ExpCfg g;
  g.M = M;
  g.task = c->task;
  g.row = rowW;
  g.kcap = p->kcap;
  g.radius = p->radius;
  g.W = p->frontier_W;
  g.raw1max = raw1max;
  g.rawmax = rawmax;
  g.knots_per_segment = p->knots_per_segment;
  g.n_total = p->n_total;
  g.k_ref = p->k_ref;
  g.Bmax = p->batch_B;
  g.budget = p->eval_budget;
  g.eps = c->prm.eps_feas;
  g.mu_merit = p->mu_merit;
  g.policy = p->policy;
  g.sseed = p->sample_seed;
  g.draws = sampling ? p->sample_draws : 0;
  if (fits) {
    g.Vcap = w->cfg.Vcap;
    g.vmask = w->cfg.vmask;
    g.cmask = w->cfg.cmask;
    const bool same = std::memcmp(&w->prm, p, sizeof(*p)) == 0;
    w->cfg = g;
    w->prm = *p;
    if (!same) w->graph_valid = false;
    return COMET_OK;
  }
  destroy_expand_ws(c);
  w = new comet_expand_ws();
  c->xws = w;
  g.Vcap = Vcap;
  const unsigned long long HV = pow2_at_least(2ull * (unsigned long long)Vcap);
  const unsigned long long HC = pow2_at_least(2ull * (unsigned long long)ncand + 16);
  g.vmask = HV - 1;
  g.cmask = HC - 1;
  w->cfg = g;
  w->prm = *p;
  w->ntiles_rs = (Vcap + RS_TILE - 1) / RS_TILE;
  const long long nmax1 = c->max_intervals + 1;
  const long long kref = std::max(1, p->k_ref);
  const long long BR = std::max<long long>(p->batch_B, kref);
  bool ok = true;
  auto A = [&](void** ptr, size_t bytes) { ok = ok && hipMalloc(ptr, std::max<size_t>(bytes, 8)) == hipSuccess; };
  A((void**)&w->C, sizeof(ExpCounters));
  A((void**)&w->vkey, 8 * Vcap);
  A((void**)&w->vset, 8 * HV);
  A((void**)&w->vJ, 8 * Vcap);
  A((void**)&w->vv, 8 * Vcap);
  A((void**)&w->vM, 8 * Vcap);
  for (int i = 0; i < 2; ++i) {
    A((void**)&w->s_hi[i], 8 * Vcap);
    A((void**)&w->s_lo[i], 8 * Vcap);
    A((void**)&w->s_idx[i], 4 * Vcap);
  }
  A((void**)&w->rs_counts, 4 * 256 * w->ntiles_rs);
  w->ccap = ncand;
  A((void**)&w->ckey, 8 * ncand);
  A((void**)&w->cflag, 4 * ncand);
  A((void**)&w->cpos, 4 * ncand);
  A((void**)&w->hkeys, 8 * HC);
  A((void**)&w->hmin, 4 * HC);
  const long long max_scan = std::max<long long>(ncand, 256 * w->ntiles_rs);
  w->scan.max_tiles = (max_scan + SCAN_TILE - 1) / SCAN_TILE + 1;
  A((void**)&w->scan.tiles, 4 * w->scan.max_tiles);
  A((void**)&w->F, 8 * BR);
  A((void**)&w->fnseg, 4 * BR);
  A((void**)&w->fmodes, 4 * BR * c->max_segments);
  A((void**)&w->fknots, 4 * BR * c->max_segments);
  A((void**)&w->ecost, 4 * BR);
  A((void**)&w->eviol, 4 * BR);
  A((void**)&w->efeas, BR);
  A((void**)&w->ecost64, 8 * BR);
  A((void**)&w->eviol64, 8 * BR);
  A((void**)&w->rtraj, 4 * kref * nmax1 * rowW);
  A((void**)&w->ix0, 4 * 8);
  A((void**)&w->igoal, 4 * 4);
  A((void**)&w->iinst, 4 * 4);
  A((void**)&w->o_nseg, 4);
  A((void**)&w->o_modes, 4 * c->max_segments);
  A((void**)&w->o_knots, 4 * c->max_segments);
  A((void**)&w->o_cost, 4);
  A((void**)&w->o_viol, 4);
  A((void**)&w->o_traj, 4 * nmax1 * rowW);
  A((void**)&w->dev_nV, 8 * 4);
  A((void**)&w->F2, 8 * BR);
  A((void**)&w->fnseg2, 4 * BR);
  A((void**)&w->fmodes2, 4 * BR * c->max_segments);
  A((void**)&w->fknots2, 4 * BR * c->max_segments);
  A((void**)&w->warm_tmp, 4 * BR * nmax1 * rowW);
  A((void**)&w->warm, 4 * BR * nmax1 * rowW);
  if (!ok) {
    (void)hipGetLastError();
    destroy_expand_ws(c);
    return fail_msg(c, COMET_ENOMEM, "expansion work space does not fit");
  }
  int khz = 0;
  if (hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, c->device) == hipSuccess && khz > 0)
    w->wall_khz = khz;
  return COMET_OK;
}

// stable sort of s_*[0] (first *n entries) by (hi, lo); returns the buffer holding the result
int enqueue_sort(comet_ctx* c, hipStream_t s, const long long* nV) {
  comet_expand_ws* w = c->xws;
  int cur = 0;
  for (int pass = 0; pass < 16; ++pass) {
    hipLaunchKernelGGL(k_rs_count, dim3((unsigned)w->ntiles_rs), dim3(RS_TILE), 0, s, w->s_hi[cur], w->s_lo[cur], nV,
                       pass, w->ntiles_rs, w->rs_counts);
    w->scan.run(s, w->rs_counts, w->rs_counts, nullptr, 256 * w->ntiles_rs, nullptr);
    hipLaunchKernelGGL(k_rs_scatter, dim3((unsigned)w->ntiles_rs), dim3(RS_TILE), 0, s, w->s_hi[cur], w->s_lo[cur],
                       w->s_idx[cur], nV, pass, w->ntiles_rs, w->rs_counts, w->s_hi[cur ^ 1], w->s_lo[cur ^ 1],
                       w->s_idx[cur ^ 1]);
    cur ^= 1;
  }
  return cur;
}

// rank V (first nV entries) into s_idx[result]; returns which buffer holds the order
int enqueue_rank(comet_ctx* c, hipStream_t s, int refine) {
  comet_expand_ws* w = c->xws;
  const ExpCfg& g = w->cfg;
  hipLaunchKernelGGL(k_rank_keys, dim3(blocks(g.Vcap, 256)), dim3(256), 0, s, g, w->C, refine, w->vkey, w->vJ, w->vv,
                     w->vM, w->s_hi[0], w->s_lo[0], w->s_idx[0]);
  return enqueue_sort(c, s, &w->C->nV);
}

// next batch from the ranked V: generate, first occurrences, compact (sets C->nF)
// next batch by uniform sampling: draw, first occurrences, compact (sets C->nF)
void enqueue_sample_batch(comet_ctx* c, hipStream_t s) {
  comet_expand_ws* w = c->xws;
  const ExpCfg& g = w->cfg;
  const long long ncand = g.draws;
  hipLaunchKernelGGL(k_fill_u64, dim3(blocks(g.cmask + 1, 256 * 8)), dim3(256), 0, s, w->hkeys, EMPTY,
                     (long long)(g.cmask + 1));
  hipLaunchKernelGGL(k_fill_u32, dim3(blocks(g.cmask + 1, 256 * 8)), dim3(256), 0, s, w->hmin, 0xFFFFFFFFu,
                     (long long)(g.cmask + 1));
  hipLaunchKernelGGL(k_sample, dim3(blocks(ncand, 256)), dim3(256), 0, s, g, w->C, w->vset, w->ckey, w->hkeys,
                     w->hmin, free_counts());
  hipLaunchKernelGGL(k_first, dim3(blocks(ncand, 256)), dim3(256), 0, s, g, w->C, w->ckey, w->hkeys, w->hmin,
                     w->cflag);
  w->scan.run(s, w->cflag, w->cpos, &w->C->nCand, ncand, &w->C->kept);
  hipLaunchKernelGGL(k_compact, dim3(blocks(ncand, 256)), dim3(256), 0, s, g, w->C, w->ckey, w->cflag, w->cpos, w->F,
                     w->vset);
  hipLaunchKernelGGL(k_sample_done, dim3(1), dim3(1), 0, s, g, w->C);
}

void enqueue_next_batch(comet_ctx* c, hipStream_t s) {
  comet_expand_ws* w = c->xws;
  const ExpCfg& g = w->cfg;
  if (g.policy == COMET_POLICY_UNIFORM) {
    enqueue_sample_batch(c, s);
    return;
  }
  const long long ncand = (long long)g.W * g.rawmax;
  const int cur = enqueue_rank(c, s, 0);
  hipLaunchKernelGGL(k_fill_u64, dim3(blocks(g.cmask + 1, 256 * 8)), dim3(256), 0, s, w->hkeys, EMPTY,
                     (long long)(g.cmask + 1));
  hipLaunchKernelGGL(k_fill_u32, dim3(blocks(g.cmask + 1, 256 * 8)), dim3(256), 0, s, w->hmin, 0xFFFFFFFFu,
                     (long long)(g.cmask + 1));
  hipLaunchKernelGGL(k_gen, dim3(blocks(ncand, 256)), dim3(256), 0, s, g, w->C, w->s_idx[cur], w->vkey, w->vset,
                     w->ckey, w->hkeys, w->hmin);
  hipLaunchKernelGGL(k_first, dim3(blocks(ncand, 256)), dim3(256), 0, s, g, w->C, w->ckey, w->hkeys, w->hmin,
                     w->cflag);
  w->scan.run(s, w->cflag, w->cpos, &w->C->nCand, ncand, &w->C->kept);
  hipLaunchKernelGGL(k_compact, dim3(blocks(ncand, 256)), dim3(256), 0, s, g, w->C, w->ckey, w->cflag, w->cpos, w->F,
                     w->vset);
  hipLaunchKernelGGL(k_set_batch, dim3(1), dim3(1), 0, s, w->C);
}

comet_status enqueue_evaluate_batch(comet_ctx* c, hipStream_t s, const long long* n_dev, long long nmax, int refine,
                                    float* traj, unsigned long long* t_first, comet_mlp* learned) {
  comet_expand_ws* w = c->xws;
  hipLaunchKernelGGL(k_build, dim3(blocks(nmax, 256)), dim3(256), 0, s, w->cfg, n_dev, w->F, w->fnseg, w->fmodes,
                     w->fknots, c->max_segments);
  const int smax = c->max_segments;
  const long long row = (long long)(c->max_intervals + 1) * w->cfg.row;
  if (learned) {
    // network scores and warm starts; the batch is evaluated in predicted-merit order
    mlp_encode_dev(learned, c->task, s, nmax, n_dev, w->ix0, w->igoal, w->iinst, 0, w->fnseg, w->fmodes, w->fknots,
                   smax);
    mlp_forward(learned, s, (int)nmax, n_dev);
    const int O = mlp_out_dim(learned);
    hipLaunchKernelGGL(k_learned_keys, dim3(blocks(nmax, 256)), dim3(256), 0, s, w->cfg, w->C, mlp_output(learned), O,
                       w->F, w->s_hi[0], w->s_lo[0], w->s_idx[0]);
    const int cur = enqueue_sort(c, s, n_dev);
    const unsigned* perm = w->s_idx[cur];
    mlp_decode_warm_dev(learned, c->task, s, nmax, n_dev, w->ix0, 0, w->fnseg, w->fmodes, w->fknots, smax,
                        c->max_intervals, w->warm_tmp);
    hipLaunchKernelGGL(k_gather_batch, dim3(blocks(nmax, 256)), dim3(256), 0, s, w->C, perm, w->F, w->fnseg,
                       w->fmodes, w->fknots, smax, w->F2, w->fnseg2, w->fmodes2, w->fknots2);
    hipLaunchKernelGGL(k_copy_batch, dim3(blocks(nmax, 256)), dim3(256), 0, s, w->C, w->F2, w->fnseg2, w->fmodes2,
                       w->fknots2, smax, w->F, w->fnseg, w->fmodes, w->fknots);
    hipLaunchKernelGGL(k_gather_warm, dim3(blocks(nmax * row, 256)), dim3(256), 0, s, w->C, perm, w->warm_tmp, row,
                       w->warm);
  }
  EvalLaunch L;
  L.warm = (learned && w->prm.learned_warm) ? w->warm : nullptr;
  L.no_sort = learned != nullptr;
  L.B_dev = (const int64_t*)n_dev;
  L.B_max = nmax;
  L.x0 = w->ix0; L.goal = w->igoal; L.inst = w->iinst; L.inst_stride = 0;
  L.nseg = w->fnseg; L.modes = w->fmodes; L.knots = w->fknots;
  L.refine = refine;
  L.cost = w->ecost; L.viol = w->eviol; L.feas = w->efeas; L.traj = traj;
  L.cost64 = w->ecost64; L.viol64 = w->eviol64; L.t_first = t_first;
  if (c->task == COMET_TASK_FLIP) return launch_flip(c, s, L);
  return launch_evaluate(c, s, L);
}

// refinement of the k_ref best feasible evaluated orders and the returned plan
comet_status enqueue_refine_and_output(comet_ctx* c, hipStream_t s) {
  comet_expand_ws* w = c->xws;
  const ExpCfg& g = w->cfg;
  const comet_expand_params& p = w->prm;
  if (p.k_ref > 0) {
    const int cur = enqueue_rank(c, s, 1);
    hipLaunchKernelGGL(k_ref_batch, dim3(blocks(p.k_ref, 256)), dim3(256), 0, s, g, w->C, w->s_idx[cur], w->vkey,
                       w->vJ, w->vv, w->F);
    comet_status st = enqueue_evaluate_batch(c, s, &w->C->nRef, p.k_ref, 1, w->rtraj, nullptr, nullptr);
    if (st != COMET_OK) return st;
    hipLaunchKernelGGL(k_pick_best, dim3(1), dim3(1), 0, s, g, w->C, w->F, w->ecost64, w->eviol64);
  }
  hipLaunchKernelGGL(k_best_out, dim3(1), dim3(256), 0, s, g, w->C, w->rtraj, c->max_intervals + 1, w->o_nseg,
                     w->o_modes, w->o_knots, w->o_cost, w->o_viol, w->o_traj, c->max_segments);
  return hipGetLastError() == hipSuccess ? COMET_OK : fail_msg(c, COMET_EHIP, "expansion launch failed");
}

comet_status enqueue_expand(comet_ctx* c, hipStream_t s) {
  comet_expand_ws* w = c->xws;
  const ExpCfg& g = w->cfg;
  const comet_expand_params& p = w->prm;
  hipLaunchKernelGGL(k_exp_init, dim3(1), dim3(1), 0, s, w->C);
  hipLaunchKernelGGL(k_fill_u64, dim3(blocks(g.vmask + 1, 256 * 8)), dim3(256), 0, s, w->vset, EMPTY,
                     (long long)(g.vmask + 1));
  const int kmax = std::min(p.seed_max_segments, p.kcap);
  const long long n_seed = seed_slots(g.task, g.M, kmax);
  if (g.policy == COMET_POLICY_UNIFORM) {
    hipLaunchKernelGGL(k_sample_start, dim3(1), dim3(1), 0, s, g, w->C);
    enqueue_sample_batch(c, s);
  } else if (task_has_language(g.task)) {
    // a task language filters the seed: all orders of 1..kmax segments as candidates,
    // kept in key order by the candidate pipeline
    hipLaunchKernelGGL(k_fill_u64, dim3(blocks(g.cmask + 1, 256 * 8)), dim3(256), 0, s, w->hkeys, EMPTY,
                       (long long)(g.cmask + 1));
    hipLaunchKernelGGL(k_fill_u32, dim3(blocks(g.cmask + 1, 256 * 8)), dim3(256), 0, s, w->hmin, 0xFFFFFFFFu,
                       (long long)(g.cmask + 1));
    hipLaunchKernelGGL(k_seed_cand, dim3(blocks(n_seed, 256)), dim3(256), 0, s, g, kmax, n_seed, w->C, w->ckey,
                       w->hkeys, w->hmin, free_counts());
    hipLaunchKernelGGL(k_first, dim3(blocks(n_seed, 256)), dim3(256), 0, s, g, w->C, w->ckey, w->hkeys, w->hmin,
                       w->cflag);
    w->scan.run(s, w->cflag, w->cpos, &w->C->nCand, n_seed, &w->C->kept);
    hipLaunchKernelGGL(k_compact, dim3(blocks(n_seed, 256)), dim3(256), 0, s, g, w->C, w->ckey, w->cflag, w->cpos,
                       w->F, w->vset);
    hipLaunchKernelGGL(k_set_batch, dim3(1), dim3(1), 0, s, w->C);
  } else {
    hipLaunchKernelGGL(k_seed, dim3(blocks(n_seed, 256)), dim3(256), 0, s, g, kmax, n_seed, w->C, w->F, w->vset);
  }
  for (int r = 0; r <= p.rounds; ++r) {
    comet_status st = enqueue_evaluate_batch(c, s, &w->C->nF, g.Bmax, 0, nullptr, &w->C->t_first, w->learned);
    if (st != COMET_OK) return st;
    hipLaunchKernelGGL(k_append, dim3(blocks(g.Bmax, 256)), dim3(256), 0, s, g, w->C, w->F, w->ecost64, w->eviol64,
                       w->vkey, w->vJ, w->vv, w->vM);
    hipLaunchKernelGGL(k_advance, dim3(1), dim3(1), 0, s, g, w->C);
    if (r < p.rounds) enqueue_next_batch(c, s);
  }
  return enqueue_refine_and_output(c, s);
}

// ---------------------------------------------------------------------------------
__global__ void k_set_batch_n(ExpCounters* C, long long n) { C->nF = n; }

comet_status run_mcts(comet_ctx* c, hipStream_t s) {
  comet_expand_ws* w = c->xws;
  const ExpCfg& g = w->cfg;
  const comet_expand_params& p = w->prm;
  const double eps = g.eps;
  hipLaunchKernelGGL(k_exp_init, dim3(1), dim3(1), 0, s, w->C);
  MctsSearch S;
  S.init(g.task, g.kcap, g.M, p.uct_c, p.sample_seed, p.batch_B, p.eval_budget, p.mu_merit, eps);
  std::vector<double> hJ, hv;
  while (S.begin_batch()) {
    const long long n = (long long)S.fresh.size();
    if (n > 0) {
      if (hipMemcpyAsync(w->F, S.fresh.data(), 8 * n, hipMemcpyHostToDevice, s) != hipSuccess)
        return fail_msg(c, COMET_EHIP, "MCTS batch upload failed");
      hipLaunchKernelGGL(k_set_batch_n, dim3(1), dim3(1), 0, s, w->C, n);
      comet_status st = enqueue_evaluate_batch(c, s, &w->C->nF, n, 0, nullptr, &w->C->t_first, nullptr);
      if (st != COMET_OK) return st;
      hipLaunchKernelGGL(k_append, dim3(blocks(n, 256)), dim3(256), 0, s, g, w->C, w->F, w->ecost64, w->eviol64,
                         w->vkey, w->vJ, w->vv, w->vM);
      hipLaunchKernelGGL(k_advance, dim3(1), dim3(1), 0, s, g, w->C);
      hJ.resize(n);
      hv.resize(n);
      (void)hipMemcpyAsync(hJ.data(), w->ecost64, 8 * n, hipMemcpyDeviceToHost, s);
      (void)hipMemcpyAsync(hv.data(), w->eviol64, 8 * n, hipMemcpyDeviceToHost, s);
      if (hipStreamSynchronize(s) != hipSuccess) return fail_msg(c, COMET_EHIP, "MCTS evaluation failed");
    }
    S.end_batch(hJ.data(), hv.data());
  }
  return enqueue_refine_and_output(c, s);
}

}  // namespace

extern "C" {

comet_status comet_expand(comet_ctx* c, void* stream, const float* x0, const float* goal, const float* inst,
                          const comet_expand_params* params, comet_mlp* learned, int32_t* best_nseg,
                          int32_t* best_modes, int32_t* best_knots, float* best_cost, float* best_viol,
                          float* best_traj, comet_expand_stats* stats) {
  if (!c) return COMET_EINVAL;
  if (!x0 || !goal || !inst || !best_nseg || !best_modes || !best_knots || !best_cost || !best_viol)
    return fail_msg(c, COMET_EINVAL, "null input or output pointer");
  comet_status st = check_expand_params(c, params);
  if (st != COMET_OK) return st;
  const bool flip = (c->task == COMET_TASK_FLIP);
  if (learned && (mlp_max_batch(learned) < params->batch_B || mlp_in_dim(learned) < mlp_task_in_dim(c->task) ||
                  mlp_warm_segments(learned) < mlp_task_segments(c->task)))
    return fail_msg(c, COMET_EINVAL,
                    "learned network: max_batch < batch_B, or in_dim / out_dim too small for the task's encoding "
                    "(in_dim >= " + std::to_string(mlp_task_in_dim(c->task)) + ", out_dim >= " +
                        std::to_string(mlp_task_out_dim(c->task)) + ")");
  if (learned && params->policy == COMET_POLICY_MCTS)
    return fail_msg(c, COMET_EINVAL, "the learned network ranks expansion or sampling batches, not MCTS");
  st = ensure_ws(c, params);
  if (st != COMET_OK) return st;
  comet_expand_ws* w = c->xws;
  if (w->learned != learned) {
    w->learned = learned;
    w->graph_valid = false;
  }
  hipStream_t us = (hipStream_t)stream;
  if (!c->gstream && hipStreamCreateWithFlags(&c->gstream, hipStreamNonBlocking) != hipSuccess)
    return fail_msg(c, COMET_EHIP, "stream creation failed");
  hipStream_t gs = c->gstream;
  // inputs into the work space, ordered after the caller's stream
  hipEvent_t e_in, e_t0, e_t1;
  if (hipEventCreate(&e_in) != hipSuccess || hipEventCreate(&e_t0) != hipSuccess || hipEventCreate(&e_t1) != hipSuccess)
    return fail_msg(c, COMET_EHIP, "event creation failed");
  (void)hipMemcpyAsync(w->ix0, x0, 4 * (flip ? 8 : (is_free_task(c->task) ? push_free::NX : push::NX)),
                       hipMemcpyDeviceToDevice, us);
  (void)hipMemcpyAsync(w->igoal, goal, 4 * (flip ? 2 : 3), hipMemcpyDeviceToDevice, us);
  (void)hipMemcpyAsync(w->iinst, inst, 4 * 1, hipMemcpyDeviceToDevice, us);
  (void)hipEventRecord(e_in, us);
  (void)hipStreamWaitEvent(gs, e_in, 0);
  if (params->policy == COMET_POLICY_MCTS) {
    (void)hipEventRecord(e_t0, gs);
    const comet_status ms = run_mcts(c, gs);
    (void)hipEventRecord(e_t1, gs);
    if (ms != COMET_OK) {
      (void)hipStreamSynchronize(gs);
      (void)hipEventDestroy(e_in);
      (void)hipEventDestroy(e_t0);
      (void)hipEventDestroy(e_t1);
      return ms;
    }
  } else {
  if (!w->graph_valid) {
    if (w->gexec) {
      (void)hipGraphExecDestroy(w->gexec);
      w->gexec = nullptr;
    }
    hipGraph_t graph;
    if (hipStreamBeginCapture(gs, hipStreamCaptureModeThreadLocal) != hipSuccess)
      return fail_msg(c, COMET_EHIP, "stream capture failed to start");
    comet_status es = enqueue_expand(c, gs);
    hipError_t ce = hipStreamEndCapture(gs, &graph);
    if (es != COMET_OK) return es;
    if (ce != hipSuccess) return fail_msg(c, COMET_EHIP, "stream capture failed");
    const hipError_t ie = hipGraphInstantiate(&w->gexec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (ie != hipSuccess) return fail_msg(c, COMET_EHIP, "graph instantiation failed");
    w->graph_valid = true;
  }
  (void)hipEventRecord(e_t0, gs);
  if (hipGraphLaunch(w->gexec, gs) != hipSuccess) return fail_msg(c, COMET_EHIP, "graph launch failed");
  (void)hipEventRecord(e_t1, gs);
  }
  // outputs to the caller
  (void)hipMemcpyAsync(best_nseg, w->o_nseg, 4, hipMemcpyDeviceToDevice, gs);
  (void)hipMemcpyAsync(best_modes, w->o_modes, 4 * c->max_segments, hipMemcpyDeviceToDevice, gs);
  (void)hipMemcpyAsync(best_knots, w->o_knots, 4 * c->max_segments, hipMemcpyDeviceToDevice, gs);
  (void)hipMemcpyAsync(best_cost, w->o_cost, 4, hipMemcpyDeviceToDevice, gs);
  (void)hipMemcpyAsync(best_viol, w->o_viol, 4, hipMemcpyDeviceToDevice, gs);
  if (best_traj)
    (void)hipMemcpyAsync(best_traj, w->o_traj, 4 * (size_t)(c->max_intervals + 1) * w->cfg.row,
                         hipMemcpyDeviceToDevice, gs);
  ExpCounters hc;
  (void)hipMemcpyAsync(&hc, w->C, sizeof hc, hipMemcpyDeviceToHost, gs);
  const hipError_t se = hipStreamSynchronize(gs);
  float ms = 0.f;
  (void)hipEventElapsedTime(&ms, e_t0, e_t1);
  (void)hipEventDestroy(e_in);
  (void)hipEventDestroy(e_t0);
  (void)hipEventDestroy(e_t1);
  if (se != hipSuccess) return fail_msg(c, COMET_EHIP, "expansion failed on the device");
  if (stats) {
    stats->evaluated = hc.nV;
    stats->rounds_done = (int32_t)hc.rounds;
    stats->n_feasible = (int32_t)hc.n_feas;
    stats->first_feasible_index = (hc.first_feas == ~0ull) ? 0 : (int64_t)hc.first_feas;
    stats->t_first_feasible_ms =
        (hc.t_first != ~0ull && hc.t_first >= hc.t_start) ? (double)(hc.t_first - hc.t_start) / w->wall_khz : -1.0;
    stats->t_total_ms = ms;
    stats->n_refined = (int32_t)hc.nRef;
    stats->reserved = 0;
  }
  return COMET_OK;
}

comet_status comet_expand_next(comet_ctx* c, void* stream, int64_t n, const uint64_t* keys, const double* merit,
                               const comet_expand_params* params, int64_t room, uint64_t* out_keys,
                               int64_t* out_n) {
  if (!c) return COMET_EINVAL;
  if (n < 0 || (n > 0 && (!keys || !merit)) || !out_keys || !out_n) return fail_msg(c, COMET_EINVAL, "bad arguments");
  comet_status st = check_expand_params(c, params);
  if (st == COMET_OK && params->policy != COMET_POLICY_EXPAND)
    return fail_msg(c, COMET_EINVAL, "comet_expand_next builds expansion batches (policy 0)");
  if (st != COMET_OK) return st;
  if (n > params->eval_budget + params->batch_B) return fail_msg(c, COMET_EINVAL, "n exceeds eval_budget + batch_B");
  if (room < 0 || room > params->batch_B) return fail_msg(c, COMET_EINVAL, "room outside [0, batch_B]");
  st = ensure_ws(c, params);
  if (st != COMET_OK) return st;
  comet_expand_ws* w = c->xws;
  hipStream_t s = (hipStream_t)stream;
  const ExpCfg& g = w->cfg;
  // V := given keys and merits; counters describe a finished round with the given room
  ExpCounters hc;
  std::memset(&hc, 0, sizeof hc);
  hc.nV = n;
  hc.room = room;
  hc.nCand = (room > 0) ? std::min<long long>(g.W, n) * g.rawmax : 0;
  hc.best_row = -1;
  if (n > 0) {
    (void)hipMemcpyAsync(w->vkey, keys, 8 * n, hipMemcpyDeviceToDevice, s);
    (void)hipMemcpyAsync(w->vM, merit, 8 * n, hipMemcpyDeviceToDevice, s);
  }
  (void)hipMemcpyAsync(w->C, &hc, sizeof hc, hipMemcpyHostToDevice, s);
  hipLaunchKernelGGL(k_fill_u64, dim3(blocks(g.vmask + 1, 256 * 8)), dim3(256), 0, s, w->vset, EMPTY,
                     (long long)(g.vmask + 1));
  if (n > 0) hipLaunchKernelGGL(k_vset_fill, dim3(blocks(n, 256)), dim3(256), 0, s, g, w->vkey, n, w->vset);
  enqueue_next_batch(c, s);
  (void)hipMemcpyAsync(out_n, &w->C->nF, 8, hipMemcpyDeviceToDevice, s);
  (void)hipMemcpyAsync(out_keys, w->F, 8 * (size_t)room, hipMemcpyDeviceToDevice, s);
  if (hipStreamSynchronize(s) != hipSuccess) return fail_msg(c, COMET_EHIP, "expand_next failed on the device");
  w->graph_valid = false;  // the expansion graph must be re-captured after direct use of the work space
  return COMET_OK;
}

comet_status comet_expand_trace(comet_ctx* c, void* stream, int64_t cap, uint64_t* keys, double* J, double* v,
                                int64_t* n_out) {
  if (!c || !c->xws || !n_out) return fail_msg(c, COMET_ESTATE, "no expansion has run on this context");
  comet_expand_ws* w = c->xws;
  hipStream_t s = (hipStream_t)stream;
  long long nV = 0;
  if (hipMemcpyAsync(&nV, &w->C->nV, 8, hipMemcpyDeviceToHost, s) != hipSuccess || hipStreamSynchronize(s) != hipSuccess)
    return fail_msg(c, COMET_EHIP, "reading the expansion counters failed");
  const long long n = std::min<long long>(nV, cap);
  if (n > 0) {
    if (keys) (void)hipMemcpyAsync(keys, w->vkey, 8 * n, hipMemcpyDeviceToDevice, s);
    if (J) (void)hipMemcpyAsync(J, w->vJ, 8 * n, hipMemcpyDeviceToDevice, s);
    if (v) (void)hipMemcpyAsync(v, w->vv, 8 * n, hipMemcpyDeviceToDevice, s);
  }
  (void)hipMemcpyAsync(n_out, &nV, 8, hipMemcpyHostToDevice, s);
  if (hipStreamSynchronize(s) != hipSuccess) return fail_msg(c, COMET_EHIP, "copying the trace failed");
  return COMET_OK;
}

}  // extern "C"
