// keys.h -- order keys and the languages of the flipping and free-motion pushing tasks,
// shared by the device expansion and the host MCTS tree.
//
// Keys pack (K, m_0, ..., m_{K-1}) as K << 60 followed by the ids from bit 59 down, w bits
// each: w = 10 for the pushing, timed-pushing and flipping tasks (up to 6 segments), w = 4
// for the 16 ids of pushing with free motion (up to 8 segments).  Comparing two keys of a
// task compares the segment count first and then the ids lexicographically.
#pragma once
#include <hip/hip_runtime.h>

#include "../../include/comet.h"

namespace comet {

constexpr int KEY_MAXSEG = 8;   // the longest order a key holds (free motion; the others stop at 6)
// pushing with free motion, with the fixed step or with optimised timing: one language
__host__ __device__ constexpr bool is_free_task(int task) {
  return task == COMET_TASK_PUSH_FREE || task == COMET_TASK_PUSH_FREE_TIMED;
}
__host__ __device__ constexpr int key_bits(int task) { return is_free_task(task) ? 4 : 10; }
__host__ __device__ inline int key_len(unsigned long long k) { return (int)(k >> 60); }
__host__ __device__ inline int key_mode(unsigned long long k, int i, int w) {
  return (int)((k >> (60 - w * (i + 1))) & ((1ull << w) - 1ull));
}
__host__ __device__ inline unsigned long long key_make(int K, const int* m, int w) {
  unsigned long long k = (unsigned long long)K << 60;
  for (int i = 0; i < K; ++i) k |= (unsigned long long)m[i] << (60 - w * (i + 1));
  return k;
}


// Admissibility of a flipping order (the transition rules of Sec. IV-B, with the readings
// of the flip model): fingers never share a face; a finger changes face only through a
// free segment; a pivot keeps at least one finger in contact; no two consecutive segments
// are equal; consecutive pivots keep their direction; no finger touches the face on the
// table (the support face while supported; the support and the landing face in a pivot).
// Ids: (f1 * 13 + f2) * 5 + g, finger 0 free / 1 + 3 face + slip; the support starts on
// face 3 and a pivot run followed by a supported segment lands on the next face.
__host__ __device__ inline bool flip_admissible_key(unsigned long long k) {
  const int K = key_len(k);
  int fs = 3, prev_g = -1, prev_id = -1, pa = -1, pb = -1;
  for (int j = 0; j < K; ++j) {
    const int id = key_mode(k, j, 10);
    if (id >= 845 || id == prev_id) return false;
    const int g = id % 5, c2 = (id / 5) % 13, c1 = id / 65;
    if (g >= 3 && prev_g >= 3 && g != prev_g) return false;
    if (g <= 2 && prev_g >= 3) fs = (fs + (prev_g == 3 ? 3 : 1)) & 3;
    const int a = c1 ? (c1 - 1) / 3 : -1, b = c2 ? (c2 - 1) / 3 : -1;
    if (a >= 0 && a == b) return false;
    if (g >= 3 && a < 0 && b < 0) return false;
    if (a == fs || b == fs) return false;
    if (g >= 3) {
      const int landing = (fs + (g == 3 ? 3 : 1)) & 3;
      if (a == landing || b == landing) return false;
    }
    if ((pa >= 0 && a >= 0 && pa != a) || (pb >= 0 && b >= 0 && pb != b)) return false;
    pa = a;
    pb = b;
    prev_g = g;
    prev_id = id;
  }
  return true;
}

// Admissibility of a free-motion pushing order (the transition rules of Sec. III-A with
// the readings of the free-motion model): ids 0..11 are contacts (face id / 3), 12..15 free
// motion in front of face id - 12; no two consecutive segments are equal; a contact keeps
// its face (it may change its slip) until a free segment; leaving contact on face j enters
// the region in front of face j and a contact on face j starts from there; a free region
// connects to the regions of the neighbouring faces.
__host__ __device__ inline bool free_step_ok(int a, int b) {
  if (a == b) return false;
  const bool ca = a < 12, cb = b < 12;
  const int fa = ca ? a / 3 : a - 12, fb = cb ? b / 3 : b - 12;
  if (ca || cb) return fa == fb;
  return ((fb - fa + 4) & 3) == 1 || ((fa - fb + 4) & 3) == 1;
}
__host__ __device__ inline bool free_admissible_key(unsigned long long k) {
  const int K = key_len(k);
  if (K < 1 || K > 8) return false;
  for (int j = 0; j < K; ++j) {
    const int id = key_mode(k, j, 4);
    if (j > 0 && !free_step_ok(key_mode(k, j - 1, 4), id)) return false;
  }
  return true;
}

// Counts of admissible free-motion continuations: c[r][a] = the number of id sequences of
// length r that may follow id a (c[0][a] = 1).  The t-th admissible order of K segments in
// key order is read off them position by position (free_unrank).
struct FreeCounts {
  unsigned c[8][16];
};
inline FreeCounts free_counts() {
  FreeCounts f;
  for (int a = 0; a < 16; ++a) f.c[0][a] = 1;
  for (int r = 1; r < 8; ++r)
    for (int a = 0; a < 16; ++a) {
      unsigned s = 0;
      for (int b = 0; b < 16; ++b)
        if (free_step_ok(a, b)) s += f.c[r - 1][b];
      f.c[r][a] = s;
    }
  return f;
}
// number of admissible orders of exactly K segments
__host__ __device__ inline long long free_count_len(const FreeCounts& f, int K) {
  long long s = 0;
  for (int a = 0; a < 16; ++a) s += f.c[K - 1][a];
  return s;
}
// the t-th (from 0) admissible order of K segments in key order
__host__ __device__ inline unsigned long long free_unrank(const FreeCounts& f, int K, long long t) {
  int m[KEY_MAXSEG];
  int prev = -1;
  for (int d = 0; d < K; ++d) {
    const int rest = K - 1 - d;
    for (int b = 0; b < 16; ++b) {
      if (prev >= 0 && !free_step_ok(prev, b)) continue;
      const long long n = f.c[rest][b];
      if (t < n) {
        m[d] = b;
        break;
      }
      t -= n;
    }
    prev = m[d];
  }
  return key_make(K, m, 4);
}

// a task's language: flipping and free-motion pushing restrict the orders, the other
// pushing tasks evaluate every order of their product space
__host__ __device__ inline bool task_has_language(int task) {
  return task == COMET_TASK_FLIP || is_free_task(task);
}
__host__ __device__ inline bool admissible_key(int task, unsigned long long k) {
  return task == COMET_TASK_FLIP ? flip_admissible_key(k) : (is_free_task(task) ? free_admissible_key(k) : true);
}

}  // namespace comet
