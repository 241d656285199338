// keys.h -- order keys and the languages of the flipping and free-motion pushing tasks,
// shared by the device expansion and the host MCTS tree.
//
// Keys pack (K, m_0, ..., m_5): K << 60 | m_0 << 50 | m_1 << 40 | ... (10 bits per id), so
// comparing keys compares the segment count first and then the ids lexicographically.
#pragma once
#include <hip/hip_runtime.h>

#include "../../include/comet.h"

namespace comet {

__host__ __device__ inline int key_len(unsigned long long k) { return (int)(k >> 60); }
__host__ __device__ inline int key_mode(unsigned long long k, int i) { return (int)((k >> (50 - 10 * i)) & 1023ull); }
__host__ __device__ inline unsigned long long key_make(int K, const int* m) {
  unsigned long long k = (unsigned long long)K << 60;
  for (int i = 0; i < K; ++i) k |= (unsigned long long)m[i] << (50 - 10 * i);
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
    const int id = key_mode(k, j);
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
__host__ __device__ inline bool free_admissible_key(unsigned long long k) {
  const int K = key_len(k);
  int prev = -1;
  for (int j = 0; j < K; ++j) {
    const int id = key_mode(k, j);
    if (id >= 16) return false;
    if (prev >= 0) {
      if (id == prev) return false;
      const bool ca = prev < 12, cb = id < 12;
      const int fa = ca ? prev / 3 : prev - 12, fb = cb ? id / 3 : id - 12;
      if (ca || cb) {
        if (fa != fb) return false;
      } else if (((fb - fa + 4) & 3) != 1 && ((fa - fb + 4) & 3) != 1) {
        return false;
      }
    }
    prev = id;
  }
  return true;
}

// a task's language: flipping and free-motion pushing restrict the orders, the other
// pushing tasks evaluate every order of their product space
__host__ __device__ inline bool task_has_language(int task) {
  return task == COMET_TASK_FLIP || task == COMET_TASK_PUSH_FREE;
}
__host__ __device__ inline bool admissible_key(int task, unsigned long long k) {
  return task == COMET_TASK_FLIP ? flip_admissible_key(k) : (task == COMET_TASK_PUSH_FREE ? free_admissible_key(k) : true);
}

}  // namespace comet
