// keys.h -- order keys and the flipping language, shared by the device expansion and the
// host MCTS tree.
//
// Keys pack (K, m_0, ..., m_5): K << 60 | m_0 << 50 | m_1 << 40 | ... (10 bits per id), so
// comparing keys compares the segment count first and then the ids lexicographically.
#pragma once
#include <hip/hip_runtime.h>

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

}  // namespace comet
