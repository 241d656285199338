// mlp.hip -- learned proposal / warm-start network with hand-written BF16 MFMA kernels.
//
// Network: in_dim -> hidden (x layers, exact-erf GELU) -> out_dim, linear head.  Weights
// are kept as FP32 master copies; the GEMM operands (weights, inputs, hidden activations,
// back-propagated gradients) are rounded to BF16 (round to nearest even) and every product
// accumulates in FP32 on the matrix cores (v_mfma_f32_16x16x32_bf16 on gfx950).
// Heads of the output row: [0] feasibility logit, [1] predicted log(1 + J), [2 ..] the warm
// start: per segment slot 15 samples at normalised times i/14 of 8 channels.
// Loss (mean over the batch): BCE(logit, feasible) + masked MSE of the cost head on
// feasible samples + masked MSE of the warm-start head; optimiser AdamW on FP32 masters.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "internal.h"
#include "keys.h"

namespace comet {

typedef unsigned short bf16;
typedef __attribute__((__vector_size__(8 * sizeof(short)))) short bf16x8;
typedef __attribute__((__vector_size__(4 * sizeof(short)))) short bf16x4;
typedef __attribute__((__vector_size__(4 * sizeof(float)))) float f32x4;

constexpr int WS_SLOTS = 15, WS_CH = 8;
constexpr int SEG_SLOT = 64, POSE_DIMS = 16;

__host__ __device__ inline bf16 to_bf16(float f) {
  unsigned u;
  std::memcpy(&u, &f, 4);
  if ((u & 0x7F800000u) == 0x7F800000u && (u & 0x007FFFFFu)) return (bf16)((u >> 16) | 0x0040u);  // quiet NaN
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (bf16)(u >> 16);
}
__host__ __device__ inline float from_bf16(bf16 h) {
  const unsigned u = (unsigned)h << 16;
  float f;
  std::memcpy(&f, &u, 4);
  return f;
}

__device__ inline float gelu(float z) { return 0.5f * z * (1.0f + erff(z * 0.70710678118654752f)); }
__device__ inline float gelu_grad(float z) {
  return 0.5f * (1.0f + erff(z * 0.70710678118654752f)) + z * 0.39894228040143268f * expf(-0.5f * z * z);
}

// ---------------------------------------------------------------------------------
// GEMM: C(m, n) = sum_k A(m, k) B(k, n) with BF16 operands and FP32 accumulation on the
// matrix cores.  Operand layouts (template flags): A_K -- A(m, k) = A[m*lda + k] (the
// contraction index is contiguous), else A(m, k) = A[k*lda + m]; B_K -- B(k, n) =
// Bp[n*ldb + k], else B(k, n) = Bp[k*ldb + n].  Requirements (checked on the host): the
// contiguous extent of each operand and its leading dimension are multiples of 8 and the
// base pointers 16-byte aligned, so every global load is one 16-byte vector.
// Block tile 128 x 64, K step 32, 256 threads = 4 waves in 2 x 2, each wave 64 x 32 (4 x 2
// tiles of v_mfma_f32_16x16x32_bf16).  Tiles are staged through a double-buffered LDS ring
// (one barrier per K step, the next step's global loads in flight during the products).
// gridDim.z > 1 splits the contraction: block z sums k in [z*kc, (z+1)*kc) and writes its
// partial sums to slab z of the output (EPI_PARTIAL).
// ---------------------------------------------------------------------------------
enum { EPI_HIDDEN = 0, EPI_OUT = 1, EPI_DX = 2, EPI_PARTIAL = 3 };

struct Epi {
  const float* bias;   // [N] (EPI_HIDDEN, EPI_OUT)
  float* z;            // FP32 pre-activation out (EPI_HIDDEN; null when no backward pass follows) /
                       // FP32 result (EPI_OUT, EPI_PARTIAL)
  bf16* h;             // BF16 activation (EPI_HIDDEN) / BF16 gradient (EPI_DX)
  const float* zprev;  // pre-activation of the layer below (EPI_DX)
  long ldc;            // row stride of the outputs
  long slab;           // EPI_PARTIAL: elements between the partial-sum slabs
  bf16* ht;            // optional (EPI_HIDDEN, EPI_DX): the BF16 output again, transposed: ht[n * ldt + m]
  long ldt;            // row stride of ht (a multiple of 4)
  float* colpart;      // EPI_DX: column sums of dZ over each wave's 64 rows, row 2 * (M-tile) + wm,
                       // stride ldc (the layer's bias gradient is their sum; dZ itself is not stored)
};

constexpr int GBM = 128, GBN = 64, GBK = 32, GLD = GBK + 8;   // LDS row: 32 bf16 + 8 pad (80 bytes)
constexpr int MAX_SPLIT = 32;      // contraction splits of a weight-gradient GEMM
constexpr int COLSUM_ROWS = 256;   // partial rows of the bias-gradient column sums

// One operand tile of R rows (m or n) x GBK (k) into registers.  K-contiguous: vector v
// covers row v/4, k = (v%4)*8 .. +8.  Row-contiguous: vector v covers k = v/(R/8),
// rows ((v % (R/8))*8 .. +8).  Out-of-range vectors load zeros.
template <int R, bool KC>
struct TileLoader {
  static constexpr int NV = R * GBK / 8 / 256;   // vectors per thread
  bf16x8 v[NV];
  __device__ void load(const bf16* __restrict__ p, long ld, int r0, int rlim, int k0, int klim, int t) {
#pragma unroll
    for (int j = 0; j < NV; ++j) {
      const int id = t + 256 * j;
      int r, k;
      if (KC) {
        r = id >> 2;
        k = (id & 3) * 8;
      } else {
        k = id / (R / 8);
        r = (id % (R / 8)) * 8;
      }
      const int gr = r0 + r, gk = k0 + k;
      const bool in = KC ? (gr < rlim && gk < klim) : (gr < rlim && gk < klim);
      if (in) {
        const bf16* q = KC ? p + (long)gr * ld + gk : p + (long)gk * ld + gr;
        v[j] = *reinterpret_cast<const bf16x8*>(q);
      } else {
        v[j] = bf16x8{0, 0, 0, 0, 0, 0, 0, 0};
      }
    }
  }
  __device__ void store(bf16 (*S)[GLD], int t) const {
#pragma unroll
    for (int j = 0; j < NV; ++j) {
      const int id = t + 256 * j;
      if (KC) {
        *reinterpret_cast<bf16x8*>(&S[id >> 2][(id & 3) * 8]) = v[j];
      } else {
        const int k = id / (R / 8), r = (id % (R / 8)) * 8;
#pragma unroll
        for (int i = 0; i < 8; ++i) S[r + i][k] = (bf16)v[j][i];
      }
    }
  }
};

template <bool A_K, bool B_K, int EPI>
__global__ __launch_bounds__(256) void k_gemm(int M, int N, int K, const bf16* __restrict__ A, long lda,
                                              const bf16* __restrict__ Bp, long ldb, Epi ep, const long long* M_dev,
                                              int kc) {
  __shared__ __attribute__((aligned(16))) bf16 As[2][GBM][GLD];
  __shared__ __attribute__((aligned(16))) bf16 Bs[2][GBN][GLD];
  if (M_dev) M = (int)min((long long)M, *M_dev);
  // XCD-aware tile order.  The dispatcher places workgroup L (x fastest) on XCD L mod 8, so
  // with the identity mapping the N-tiles of one M-tile (consecutive L) land on eight
  // different L2 caches and each re-reads the same A rows from memory.  When the tiles of
  // a z-plane are a multiple of 8, XCD x takes the contiguous range [x T/8, (x+1) T/8) of
  // the row-major (M-tile, N-tile) order instead, so the N-tiles of an M-tile share an L2.
  int bx = blockIdx.x, by = blockIdx.y;
  {
    const int nbx = gridDim.x, T = nbx * gridDim.y;
    if ((T & 7) == 0) {
      const int L = blockIdx.y * nbx + blockIdx.x;
      const int q = (L & 7) * (T >> 3) + (L >> 3);
      bx = q % nbx;
      by = q / nbx;
    }
  }
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  const int wm = w >> 1, wn = w & 1;
  const int m0 = by * GBM, n0 = bx * GBN;
  if (m0 >= M) return;
  const int kb = blockIdx.z * kc, ke = min(K, kb + kc);
  f32x4 acc[4][2];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
  TileLoader<GBM, A_K> la;
  TileLoader<GBN, B_K> lb;
  const int steps = (ke - kb + GBK - 1) / GBK;
  if (steps > 0) {
    la.load(A, lda, m0, M, kb, ke, t);
    lb.load(Bp, ldb, n0, N, kb, ke, t);
    la.store(As[0], t);
    lb.store(Bs[0], t);
  }
  __syncthreads();
  const int kq = (lane >> 4) * 8;
  for (int st = 0; st < steps; ++st) {
    const int cur = st & 1;
    const bool more = st + 1 < steps;
    if (more) {   // next tiles in flight while this step's products run
      la.load(A, lda, m0, M, kb + (st + 1) * GBK, ke, t);
      lb.load(Bp, ldb, n0, N, kb + (st + 1) * GBK, ke, t);
    }
    bf16x8 a[4], b[2];
#pragma unroll
    for (int i = 0; i < 4; ++i) a[i] = *reinterpret_cast<const bf16x8*>(&As[cur][wm * 64 + i * 16 + (lane & 15)][kq]);
#pragma unroll
    for (int j = 0; j < 2; ++j) b[j] = *reinterpret_cast<const bf16x8*>(&Bs[cur][wn * 32 + j * 16 + (lane & 15)][kq]);
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j) acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[i], b[j], acc[i][j], 0, 0, 0);
    if (more) {
      la.store(As[cur ^ 1], t);
      lb.store(Bs[cur ^ 1], t);
    }
    __syncthreads();
  }
  // accumulator layout: lane holds rows 4*(lane/16) + r, column lane%16 of each 16x16 tile
  float* zo = ep.z + (EPI == EPI_PARTIAL ? (long)blockIdx.z * ep.slab : 0L);
  constexpr bool TR = (EPI == EPI_HIDDEN || EPI == EPI_DX);
  // transposed tile [n - n0][m - m0] over the operand ring (the loop's last barrier has
  // passed, so no wave still reads it)
  static_assert(GBN * (GBM + 8) <= 2 * GBM * GLD, "transposed tile exceeds the A ring");
  bf16 (*Tt)[GBM + 8] = reinterpret_cast<bf16 (*)[GBM + 8]>(&As[0][0][0]);
  float cs[2] = {0.f, 0.f};   // EPI_DX: this lane's share of the wave's column sums (column j)
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      const int mb = m0 + wm * 64 + i * 16 + (lane >> 4) * 4;
      const int n = n0 + wn * 32 + j * 16 + (lane & 15);
      if (n >= N) continue;
      bf16x4 tv = bf16x4{0, 0, 0, 0};
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int m = mb + r;
        if (m >= M) continue;
        const float v = acc[i][j][r];
        const long o = (long)m * ep.ldc + n;
        if (EPI == EPI_HIDDEN) {
          const float z = v + ep.bias[n];
          if (zo) zo[o] = z;
          const bf16 hb = to_bf16(gelu(z));
          ep.h[o] = hb;
          tv[r] = (short)hb;
        } else if (EPI == EPI_OUT) {
          zo[o] = v + ep.bias[n];
        } else if (EPI == EPI_DX) {
          const float d = v * gelu_grad(ep.zprev[o]);
          cs[j] += d;
          const bf16 hb = to_bf16(d);
          ep.h[o] = hb;
          tv[r] = (short)hb;
        } else {
          zo[o] = v;
        }
      }
      // the transposed copy is staged in LDS (the operand ring is free after the last step)
      if (TR && ep.ht) *reinterpret_cast<bf16x4*>(&Tt[n - n0][mb - m0]) = tv;
    }
  if (EPI == EPI_DX) {
    // lanes l, l^16, l^32, l^48 hold the same column over the wave's 4 row groups
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      float v = cs[j];
      v += __shfl_xor(v, 16);
      v += __shfl_xor(v, 32);
      const int n = n0 + wn * 32 + j * 16 + lane;
      if (lane < 16 && n < N) ep.colpart[(long)(2 * by + wm) * ep.ldc + n] = v;
    }
  }
  if (TR && ep.ht) {
    // write the 64 x 128 transposed block tile row by row, 16 bytes per thread and chunk
    __syncthreads();
#pragma unroll
    for (int c = 0; c < GBN * GBM / 8 / 256; ++c) {
      const int id = t + 256 * c, row = id / (GBM / 8), col = (id % (GBM / 8)) * 8;
      const int n = n0 + row, m = m0 + col;
      if (n >= N || m >= M) continue;
      bf16* q = ep.ht + (long)n * ep.ldt + m;
      if (m + 7 < M) {
        *reinterpret_cast<bf16x8*>(q) = *reinterpret_cast<const bf16x8*>(&Tt[row][col]);
      } else {
        for (int r = 0; r < M - m; ++r) q[r] = Tt[row][col + r];
      }
    }
  }
}

// out[c * ldo + r] = in[r * ldi + c] for a rows x cols BF16 matrix, through 64 x 64 LDS tiles.
// Both sides move pairs of BF16 values as 4-byte words: cols, ldi and ldo are even, rows a
// multiple of 8 and the buffers 4-byte aligned (the callers' layouts).  The LDS row stride
// of 65 values keeps the column reads on distinct banks.
__global__ __launch_bounds__(256) void k_transpose_bf16(const bf16* __restrict__ in, long ldi, int rows, int cols,
                                                        bf16* __restrict__ out, long ldo) {
  __shared__ bf16 tile[64][65];
  const int r0 = blockIdx.y * 64, c0 = blockIdx.x * 64, p = threadIdx.x & 31, q = threadIdx.x >> 5;
#pragma unroll
  for (int k = 0; k < 8; ++k) {   // row q + 8k of the tile, columns 2p, 2p + 1
    const int r = r0 + q + 8 * k, c = c0 + 2 * p;
    unsigned v = 0;
    if (r < rows && c < cols) v = *reinterpret_cast<const unsigned*>(in + (long)r * ldi + c);
    tile[q + 8 * k][2 * p] = (bf16)(v & 0xffffu);
    tile[q + 8 * k][2 * p + 1] = (bf16)(v >> 16);
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < 8; ++k) {   // output row c = column q + 8k of the tile, input rows 2p, 2p + 1
    const int c = c0 + q + 8 * k, r = r0 + 2 * p;
    if (c >= cols || r >= rows) continue;
    const unsigned v = (unsigned)tile[2 * p][q + 8 * k] | ((unsigned)tile[2 * p + 1][q + 8 * k] << 16);
    if (r + 1 < rows) *reinterpret_cast<unsigned*>(out + (long)c * ldo + r) = v;
    else out[(long)c * ldo + r] = (bf16)(v & 0xffffu);
  }
}

// sum of S partial-sum slabs of n floats each
__global__ void k_sum_slabs(const float* __restrict__ part, int S, long n, float* __restrict__ out) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  float s = 0.f;
  for (int z = 0; z < S; ++z) s += part[(long)z * n + i];
  out[i] = s;
}

// out[i] = sum_z part[z * n + i] for many slabs S: 64 columns per block, the slabs split
// over 4 thread phases (deterministic order: each phase in slab order, then phase order)
__global__ __launch_bounds__(256) void k_sum_rows(const float* __restrict__ part, int S, long n,
                                                  float* __restrict__ out) {
  __shared__ float red[4][64];
  const int c = threadIdx.x & 63, ph = threadIdx.x >> 6;
  const long i = (long)blockIdx.x * 64 + c;
  float s = 0.f;
  if (i < n)
#pragma unroll 8
    for (int z = ph; z < S; z += 4) s += part[(long)z * n + i];
  red[ph][c] = s;
  __syncthreads();
  if (ph == 0 && i < n) out[i] = red[0][c] + red[1][c] + red[2][c] + red[3][c];
}

// A hidden layer's gradients in one launch: blocks [0, nbw) add the weight gradient's
// split-K slabs as k_sum_slabs does, the remaining blocks add the bias gradient's partial
// rows as k_sum_rows does (the same summation orders, so the same values).
__global__ __launch_bounds__(256) void k_sum_grads(const float* __restrict__ slabs, int S, long nw,
                                                   float* __restrict__ outw, int nbw, const float* __restrict__ rows,
                                                   int R, long nb, float* __restrict__ outb) {
  __shared__ float red[4][64];
  if ((int)blockIdx.x < nbw) {
    const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nw) return;
    float s = 0.f;
    for (int z = 0; z < S; ++z) s += slabs[(long)z * nw + i];
    outw[i] = s;
    return;
  }
  const int c = threadIdx.x & 63, ph = threadIdx.x >> 6;
  const long i = (long)(blockIdx.x - nbw) * 64 + c;
  float s = 0.f;
  if (i < nb)
#pragma unroll 8
    for (int z = ph; z < R; z += 4) s += rows[(long)z * nb + i];
  red[ph][c] = s;
  __syncthreads();
  if (ph == 0 && i < nb) outb[i] = red[0][c] + red[1][c] + red[2][c] + red[3][c];
}

// column sums of an FP32 [M][N] matrix (bias gradients), in two deterministic stages:
// block (x, y) covers 256 columns (64 threads x 4 consecutive columns, 16-byte loads) and
// rows y*4 + phase + k * gridDim.y * 4 (4 row phases), writing part[y][n]; k_sum_rows then
// adds the gridDim.y partial rows.  N must be a multiple of 4.
__global__ __launch_bounds__(256) void k_colsum_part(const float* __restrict__ X, int M, int N,
                                                     float* __restrict__ part) {
  __shared__ f32x4 red[4][64];
  const int c = threadIdx.x & 63, ph = threadIdx.x >> 6;
  const int n = blockIdx.x * 256 + c * 4;
  f32x4 s = f32x4{0.f, 0.f, 0.f, 0.f};
  if (n < N)
    for (int m = blockIdx.y * 4 + ph; m < M; m += gridDim.y * 4) s += *reinterpret_cast<const f32x4*>(X + (long)m * N + n);
  red[ph][c] = s;
  __syncthreads();
  if (ph == 0 && n < N) {
    const f32x4 t = red[0][c] + red[1][c] + red[2][c] + red[3][c];
    *reinterpret_cast<f32x4*>(part + (long)blockIdx.y * N + n) = t;
  }
}

__global__ void k_to_bf16(const float* x, bf16* y, long n) {
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x)
    y[i] = to_bf16(x[i]);
}
// W [N][K] fp32 -> Wb [N][K] bf16 and WT [K][N] bf16
__global__ void k_refresh(const float* W, int N, int K, bf16* Wb, bf16* WT) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (long)N * K) return;
  const int n = (int)(i / K), k = (int)(i % K);
  const bf16 h = to_bf16(W[i]);
  Wb[i] = h;
  WT[(long)k * N + n] = h;
}

// ---------------------------------------------------------------------------------
// Loss and output gradient.  Y [B][O] FP32.  dY written FP32 and BF16.
// loss[0] = mean BCE, loss[1] = cost MSE over feasible, loss[2] = warm MSE over mask.
// ---------------------------------------------------------------------------------
// cnt[0] += sum of feasible flags, cnt[1] += sum of mask entries (cnt zeroed before)
// Loss reductions run in two deterministic stages: LOSS_BLOCKS blocks stride over the
// elements and write one partial per block, k_reduce_partials adds them in block order.
constexpr int LOSS_BLOCKS = 1024;

// sum over the 256 threads of a block; the result is valid in thread 0
__device__ inline float block_sum(float v, float* red) {
  for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o);
  __syncthreads();
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  return red[0] + red[1] + red[2] + red[3];
}

// partials of the two normalisers: feasible samples, warm-start mask entries (the mask
// [B][W] is read as float4: W is a multiple of 4)
__global__ __launch_bounds__(256) void k_loss_counts(int B, int W, const float* y_feas, const float* mask,
                                                     float* part) {
  __shared__ float red[4];
  const unsigned n4 = (unsigned)B * (unsigned)(W / 4), stride = gridDim.x * blockDim.x;
  const unsigned t0 = blockIdx.x * blockDim.x + threadIdx.x;
  const float4* m4 = reinterpret_cast<const float4*>(mask);
  float c = 0.f, a = 0.f;
  for (unsigned i = t0; i < n4; i += stride) {
    const float4 v = m4[i];
    c += (v.x + v.y) + (v.z + v.w);
  }
  for (unsigned i = t0; i < (unsigned)B; i += stride) a += y_feas[i];
  const float sa = block_sum(a, red);
  const float sc = block_sum(c, red);
  if (threadIdx.x == 0) {
    part[blockIdx.x * 4 + 0] = sa;
    part[blockIdx.x * 4 + 1] = sc;
  }
}

// out[j] = sum over the nb block partials of component j (j < ncomp); one block of 256
// threads, each summing a fixed stride of partials, then a fixed-order block reduction
__global__ __launch_bounds__(256) void k_reduce_partials(const float* part, int nb, int ncomp, float* out) {
  __shared__ float red[4];
  for (int j = 0; j < ncomp; ++j) {
    float s = 0.f;
    for (int b = threadIdx.x; b < nb; b += blockDim.x) s += part[b * 4 + j];
    s = block_sum(s, red);
    if (threadIdx.x == 0) out[j] = s;
  }
}

// dL/dY of the combined loss and per-block partials of the three loss terms.  Threads
// stride over pairs of adjacent outputs: O and W are even and the warm-start block starts
// at column 2, so every pair is 8-byte aligned in Y, dY and the targets and its two BF16
// gradients fill one 4-byte word.  B * O < 2^31 (checked by the caller).
__global__ __launch_bounds__(256) void k_loss_grad(int B, int O, int Wn, const float* Y, const float* y_feas,
                                                   const float* y_cost, const float* y_traj, const float* mask,
                                                   const float* cnt, float* dY, bf16* dYb, float* part) {
  __shared__ float red[4];
  const float inv_b = 1.f / (float)B, inv_f = 1.f / fmaxf(cnt[0], 1.f), inv_m = 1.f / fmaxf(cnt[1], 1.f);
  const unsigned half = (unsigned)O / 2u, n = (unsigned)B * half, stride = gridDim.x * blockDim.x;
  float acc0 = 0.f, acc1 = 0.f, acc2 = 0.f;
  for (unsigned t = blockIdx.x * blockDim.x + threadIdx.x; t < n; t += stride) {
    const unsigned b = t / half, p = t - b * half;
    const long i = (long)b * O + 2 * p;
    const float2 y = *reinterpret_cast<const float2*>(Y + i);
    float gx = 0.f, gy = 0.f;
    if (p == 0) {                                     // feasibility logit, predicted cost
      const float yv = y_feas[b], x = y.x;
      acc0 += fmaxf(x, 0.f) - x * yv + log1pf(expf(-fabsf(x)));
      gx = (1.f / (1.f + expf(-x)) - yv) * inv_b;
      const float d = y.y - y_cost[b];
      acc1 += yv * d * d;
      gy = 2.f * yv * d * inv_f;
    } else if (2 * p - 2 < (unsigned)Wn) {            // warm-start samples
      const long e = (long)b * Wn + (2 * p - 2);
      const float2 m = *reinterpret_cast<const float2*>(mask + e);
      const float2 yt = *reinterpret_cast<const float2*>(y_traj + e);
      const float d0 = y.x - yt.x, d1 = y.y - yt.y;
      acc2 += m.x * d0 * d0 + m.y * d1 * d1;
      gx = 2.f * m.x * d0 * inv_m;
      gy = 2.f * m.y * d1 * inv_m;
    }
    *reinterpret_cast<float2*>(dY + i) = make_float2(gx, gy);
    *reinterpret_cast<unsigned*>(dYb + i) = (unsigned)to_bf16(gx) | ((unsigned)to_bf16(gy) << 16);
  }
  const float s0 = block_sum(acc0, red);
  const float s1 = block_sum(acc1, red);
  const float s2 = block_sum(acc2, red);
  if (threadIdx.x == 0) {
    part[blockIdx.x * 4 + 0] = s0 * inv_b;
    part[blockIdx.x * 4 + 1] = s1 * inv_f;
    part[blockIdx.x * 4 + 2] = s2 * inv_m;
  }
}

// AdamW fused with the BF16 refresh of the weights it updates: one pass over the flat
// parameter vector; an element of a layer's weight block also writes its BF16 copy and the
// transposed copy (the values an AdamW pass followed by k_refresh would write).
constexpr int MAX_LINEAR = 17;   // layers <= 16 hidden, plus the output layer
struct LayerTable {
  int nl;
  long long woff[MAX_LINEAR], boff[MAX_LINEAR], wboff[MAX_LINEAR];
  int N[MAX_LINEAR], K[MAX_LINEAR];
};
__global__ void k_adamw_refresh(float* w, float* m, float* v, const float* g, long n, float lr, float b1, float b2,
                                float eps, float wd, float bc1, float bc2, LayerTable T, bf16* Wb, bf16* WT) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float gi = g[i];
  const float mi = b1 * m[i] + (1.f - b1) * gi;
  const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  const float mh = mi / bc1, vh = vi / bc2;
  const float wn = w[i] - lr * (mh / (sqrtf(vh) + eps) + wd * w[i]);
  w[i] = wn;
  int l = 0;
  while (l + 1 < T.nl && i >= T.woff[l + 1]) ++l;
  if (i < T.boff[l]) {   // weight block of layer l: W [N][K] row-major
    const long j = i - T.woff[l];
    const int K = T.K[l], N = T.N[l];
    const int r = (int)(j / K), c = (int)(j % K);
    const bf16 h = to_bf16(wn);
    Wb[T.wboff[l] + j] = h;
    WT[T.wboff[l] + (long)c * N + r] = h;
  }
}

__global__ void k_zero(float* p, long n) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0.f;
}

// deterministic initialisation: uniform(-1/sqrt(K), 1/sqrt(K)) from a counter-based hash
__device__ inline unsigned long long splitmix(unsigned long long x) {
  x += 0x9E3779B97F4A7C15ull;
  x = (x ^ (x >> 30)) * 0xBF58476D1CE4E5B9ull;
  x = (x ^ (x >> 27)) * 0x94D049BB133111EBull;
  return x ^ (x >> 31);
}
__global__ void k_init_uniform(float* w, long n, float scale, unsigned long long seed, long offset) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const unsigned long long r = splitmix(seed ^ splitmix((unsigned long long)(offset + i)));
  const float u = (float)((r >> 40) * (1.0 / 16777216.0));  // [0, 1)
  w[i] = (2.f * u - 1.f) * scale;
}

// ---------------------------------------------------------------------------------
// Input encoding of a planar-pushing order (416 values, BF16):
//   [0:16)   start (x, y, cos th, sin th), goal (x, y, cos th, sin th), goal - start
//            (x, y, th), pusher friction, 4 zeros;
//   [16 + 64 j, 16 + 64 (j+1))  segment j: one-hot mode id (12), intervals / 15, present flag,
//            zeros; absent segments are all zero;  [400:416) zeros.
// ---------------------------------------------------------------------------------
__global__ void k_encode_push(long B, const float* x0, const float* goal, const float* inst, int inst_stride,
                              const int32_t* nseg, const int32_t* modes, const int32_t* knots, int smax, int in_dim,
                              bf16* X, const long long* B_dev) {
  const long Bn = B_dev ? *B_dev : B;
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= Bn * in_dim) return;
  const long b = i / in_dim;
  const int d = (int)(i % in_dim);
  const long bi = b * inst_stride;
  float v = 0.f;
  if (d < POSE_DIMS) {
    const float sx = x0[bi * 4 + 0], sy = x0[bi * 4 + 1], st = x0[bi * 4 + 2];
    const float gx = goal[bi * 3 + 0], gy = goal[bi * 3 + 1], gt = goal[bi * 3 + 2];
    switch (d) {
      case 0: v = sx; break;
      case 1: v = sy; break;
      case 2: v = cosf(st); break;
      case 3: v = sinf(st); break;
      case 4: v = gx; break;
      case 5: v = gy; break;
      case 6: v = cosf(gt); break;
      case 7: v = sinf(gt); break;
      case 8: v = gx - sx; break;
      case 9: v = gy - sy; break;
      case 10: v = gt - st; break;
      case 11: v = inst[bi]; break;
      default: v = 0.f;
    }
  } else if (d < POSE_DIMS + 6 * SEG_SLOT) {
    const int j = (d - POSE_DIMS) / SEG_SLOT, q = (d - POSE_DIMS) % SEG_SLOT;
    const int K = nseg[b];
    if (j < K && j < smax) {
      const int m = modes[b * smax + j];
      if (q < push::NMODES) v = (q == m) ? 1.f : 0.f;
      else if (q == push::NMODES) v = (float)knots[b * smax + j] / 15.f;
      else if (q == push::NMODES + 1) v = 1.f;
    }
  }
  X[i] = to_bf16(v);
}

// ---------------------------------------------------------------------------------
// Warm-start targets and decoding.  Segment j covers knots k0 .. k0 + n_j of the
// trajectory rows (x_k, u_k); slot i samples normalised time i / 14 by linear
// interpolation between neighbouring rows; channel 7 is zero.
// ---------------------------------------------------------------------------------
// Flipping orders: pose block (start px, py, cos, sin; goal px, 0, cos, sin; goal - start
// px, 0, angle; table friction) then 6 segment slots of 64: factorised one-hot of the id
// (finger 1 code 0..12, finger 2 code 13..25, table mode 26..30), intervals / 15 at 31,
// presence flag at 32.
constexpr int FLIP_KN = 31, FLIP_PRESENT = 32;
__global__ void k_encode_flip(long B, const float* x0, const float* goal, const float* inst, int inst_stride,
                              const int32_t* nseg, const int32_t* modes, const int32_t* knots, int smax, int in_dim,
                              bf16* X, const long long* B_dev) {
  const long Bn = B_dev ? *B_dev : B;
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= Bn * in_dim) return;
  const long b = i / in_dim;
  const int d = (int)(i % in_dim);
  const long bi = b * inst_stride;
  float v = 0.f;
  if (d < POSE_DIMS) {
    const float sx = x0[bi * 8 + 0], sy = x0[bi * 8 + 1], st = x0[bi * 8 + 2];
    const float gx = goal[bi * 2 + 0], gt = goal[bi * 2 + 1];
    switch (d) {
      case 0: v = sx; break;
      case 1: v = sy; break;
      case 2: v = cosf(st); break;
      case 3: v = sinf(st); break;
      case 4: v = gx; break;
      case 6: v = cosf(gt); break;
      case 7: v = sinf(gt); break;
      case 8: v = gx - sx; break;
      case 10: v = gt - st; break;
      case 11: v = inst[bi]; break;
      default: v = 0.f;
    }
  } else if (d < POSE_DIMS + 6 * SEG_SLOT) {
    const int j = (d - POSE_DIMS) / SEG_SLOT, q = (d - POSE_DIMS) % SEG_SLOT;
    const int K = nseg[b];
    if (j < K && j < smax) {
      const int m = modes[b * smax + j];
      const int g = m % 5, f2 = (m / 5) % 13, f1 = m / 65;
      if (q < 13) v = (q == f1) ? 1.f : 0.f;
      else if (q < 26) v = (q - 13 == f2) ? 1.f : 0.f;
      else if (q < 31) v = (q - 26 == g) ? 1.f : 0.f;
      else if (q == FLIP_KN) v = (float)knots[b * smax + j] / 15.f;
      else if (q == FLIP_PRESENT) v = 1.f;
    }
  }
  X[i] = to_bf16(v);
}

// Free-motion pushing orders (up to 8 segments): the pushing pose block (start state with
// the slider pose, goal, goal - start, pusher friction) plus the pusher's start position
// (body frame) at 12 and 13, then 8 segment slots of 64: one-hot of the 16 ids, intervals
// / 15 at 16, presence flag at 17.
constexpr int FREE_SEGS = 8, FREE_KN = 16, FREE_PRESENT = 17;
__global__ void k_encode_free(long B, const float* x0, const float* goal, const float* inst, int inst_stride,
                              const int32_t* nseg, const int32_t* modes, const int32_t* knots, int smax, int in_dim,
                              bf16* X, const long long* B_dev) {
  const long Bn = B_dev ? *B_dev : B;
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= Bn * in_dim) return;
  const long b = i / in_dim;
  const int d = (int)(i % in_dim);
  const long bi = b * inst_stride;
  float v = 0.f;
  if (d < POSE_DIMS) {
    const float sx = x0[bi * 5 + 0], sy = x0[bi * 5 + 1], st = x0[bi * 5 + 2];
    const float gx = goal[bi * 3 + 0], gy = goal[bi * 3 + 1], gt = goal[bi * 3 + 2];
    switch (d) {
      case 0: v = sx; break;
      case 1: v = sy; break;
      case 2: v = cosf(st); break;
      case 3: v = sinf(st); break;
      case 4: v = gx; break;
      case 5: v = gy; break;
      case 6: v = cosf(gt); break;
      case 7: v = sinf(gt); break;
      case 8: v = gx - sx; break;
      case 9: v = gy - sy; break;
      case 10: v = gt - st; break;
      case 11: v = inst[bi]; break;
      case 12: v = x0[bi * 5 + 3]; break;
      case 13: v = x0[bi * 5 + 4]; break;
      default: v = 0.f;
    }
  } else if (d < POSE_DIMS + FREE_SEGS * SEG_SLOT) {
    const int j = (d - POSE_DIMS) / SEG_SLOT, q = (d - POSE_DIMS) % SEG_SLOT;
    const int K = nseg[b];
    if (j < K && j < smax) {
      const int m = modes[b * smax + j];
      if (q < push_free::NMODES) v = (q == m) ? 1.f : 0.f;
      else if (q == FREE_KN) v = (float)knots[b * smax + j] / 15.f;
      else if (q == FREE_PRESENT) v = 1.f;
    }
  }
  X[i] = to_bf16(v);
}

// Segment count of a sequence whose live knot counts are each >= 1 and sum to at most
// nmax, else 0 (the sequence is then treated as empty).  Counts are compared with the room
// left, so no sum of large counts can wrap.
__device__ inline int checked_segments(const int32_t* nseg, const int32_t* knots, long b, int smax, int nmax) {
  const int K = nseg[b];
  if (K < 1 || K > smax) return 0;
  int N = 0;
  for (int j = 0; j < K; ++j) {
    const int n = knots[b * smax + j];
    if (n < 1 || n > nmax - N) return 0;
    N += n;
  }
  return K;
}

// Warm-start targets: per segment (nsegs slots: 6, or 8 for free motion), 15 samples at
// normalised times i/14 by linear interpolation of the trajectory rows; channels
// 0..nch-1, channel c read from row column c except channel 7 from column col7 (pushing:
// the 7 state and control entries; timed pushing: the same and the duration; flipping:
// the 8 states; free motion: the 5 states and the two forces, with optimised timing the
// duration from column 9), row width `row`.
__global__ void k_targets(long B, const float* traj, int nmax, int row, int nch, int col7, int nsegs,
                          const int32_t* nseg, const int32_t* knots, int smax, const uint8_t* feas, const float* cost,
                          float* y_feas, float* y_cost, float* y_traj, float* mask) {
  const long b = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= B) return;
  const int K = checked_segments(nseg, knots, b, smax, nmax);
  const float f = feas[b] ? 1.f : 0.f;
  y_feas[b] = f;
  y_cost[b] = feas[b] ? log1pf(fmaxf(cost[b], 0.f)) : 0.f;
  const float* T = traj + b * (long)(nmax + 1) * row;
  int k0 = 0;
  for (int j = 0; j < nsegs; ++j) {
    const bool live = j < K;
    const int nj = live ? knots[b * smax + j] : 0;
    for (int i = 0; i < WS_SLOTS; ++i) {
      const float p = (float)i / (WS_SLOTS - 1) * (float)nj;
      const int k = min((int)floorf(p), max(nj - 1, 0));
      const float fr = p - (float)k;
      for (int c = 0; c < WS_CH; ++c) {
        const long e = b * ((long)nsegs * WS_SLOTS * WS_CH) + ((long)j * WS_SLOTS + i) * WS_CH + c;
        const int col = (c == 7) ? col7 : c;
        float val = 0.f;
        if (live && c < nch) {
          const float a0 = T[(k0 + k) * row + col], a1 = T[(k0 + min(k + 1, nj)) * row + col];
          val = a0 + fr * (a1 - a0);
        }
        y_traj[e] = val;
        mask[e] = (live && c < nch) ? f : 0.f;
      }
    }
    k0 += nj;
  }
}

// Pushing warm start: rows (x_k, u_k) interpolated from the network samples at every knot,
// the start state at knot 0, row N with u = 0.  width 7 (fixed step) or 8 (optimised
// timing: channel 7 is the interval duration, clamped to its bounds).
__global__ void k_decode_warm(long B, const long long* B_dev, const float* Y, int O, const float* x0, int inst_stride,
                              const int32_t* nseg, const int32_t* knots, int smax, int nmax, int width, float* warm) {
  const long Bn = B_dev ? *B_dev : B;
  const long b = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= Bn) return;
  const int K = checked_segments(nseg, knots, b, smax, nmax);
  const float* y = Y + b * (long)O + 2;
  float* Wr = warm + b * (long)(nmax + 1) * width;
  for (int r = 0; r < (nmax + 1) * width; ++r) Wr[r] = 0.f;
  int k0 = 0;
  for (int j = 0; j < K && j < smax; ++j) {
    const int nj = knots[b * smax + j];
    for (int k = 0; k <= nj && k0 + k <= nmax; ++k) {
      const float p = (nj > 0) ? (float)k / (float)nj * (WS_SLOTS - 1) : 0.f;
      const int i = min((int)floorf(p), WS_SLOTS - 2);
      const float fr = p - (float)i;
      for (int c = 0; c < width; ++c) {
        const float a0 = y[((long)j * WS_SLOTS + i) * WS_CH + c], a1 = y[((long)j * WS_SLOTS + i + 1) * WS_CH + c];
        float val = a0 + fr * (a1 - a0);
        if (c == 7) val = fminf(fmaxf(val, (float)push_timed::H_MIN), (float)push_timed::H_MAX);
        Wr[(k0 + k) * width + c] = val;
      }
    }
    k0 += nj;
  }
  for (int c = 0; c < 4; ++c) Wr[c] = x0[b * inst_stride * 4 + c];
  if (k0 <= nmax)
    for (int c = 4; c < width; ++c) Wr[k0 * width + c] = 0.f;
}

// Flipping warm start: states (8 channels) interpolated from the network samples at every
// knot, the start state at knot 0; controls from the states and the mode: accelerations
// and face-coordinate rates by forward differences, contact fingers pressing with mg/2
// (sliding ones on the cone edge), free fingers zero; row N has u = 0.
__global__ void k_decode_warm_flip(long B, const long long* B_dev, const float* Y, int O, const float* x0,
                                   int inst_stride, const int32_t* nseg, const int32_t* modes, const int32_t* knots,
                                   int smax, int nmax, float* warm) {
  constexpr int ROWF = 17;
  constexpr float MG = 0.5f * 9.81f, MUF = 0.5f, DT = 0.1f;
  const long Bn = B_dev ? *B_dev : B;
  const long b = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= Bn) return;
  const int K = checked_segments(nseg, knots, b, smax, nmax);
  const float* y = Y + b * (long)O + 2;
  float* Wr = warm + b * (long)(nmax + 1) * ROWF;
  for (int r = 0; r < (nmax + 1) * ROWF; ++r) Wr[r] = 0.f;
  int k0 = 0;
  for (int j = 0; j < K && j < smax; ++j) {
    const int nj = knots[b * smax + j];
    for (int k = 0; k <= nj && k0 + k <= nmax; ++k) {
      const float p = (nj > 0) ? (float)k / (float)nj * (WS_SLOTS - 1) : 0.f;
      const int i = min((int)floorf(p), WS_SLOTS - 2);
      const float fr = p - (float)i;
      for (int c = 0; c < 8; ++c) {
        const float a0 = y[((long)j * WS_SLOTS + i) * WS_CH + c], a1 = y[((long)j * WS_SLOTS + i + 1) * WS_CH + c];
        Wr[(k0 + k) * ROWF + c] = a0 + fr * (a1 - a0);
      }
    }
    k0 += nj;
  }
  const int N = min(k0, nmax);
  for (int c = 0; c < 8; ++c) Wr[c] = x0[b * inst_stride * 8 + c];
  int kk = 0;
  for (int j = 0; j < K && j < smax; ++j) {
    const int m = modes[b * smax + j], nj = knots[b * smax + j];
    const int fc[2] = {m / 65, (m / 5) % 13};
    for (int t = 0; t < nj && kk < N; ++t, ++kk) {
      float* u = Wr + kk * ROWF + 8;
      const float* xa = Wr + kk * ROWF;
      const float* xb = Wr + (kk + 1) * ROWF;
      for (int c = 0; c < 3; ++c) u[c] = (xb[3 + c] - xa[3 + c]) / DT;
      for (int f = 0; f < 2; ++f) {
        float fn = 0.f, ft = 0.f;
        if (fc[f] != 0) {
          const int slip = (fc[f] - 1) % 3;
          fn = 0.5f * MG;
          ft = (slip == 0) ? 0.f : ((slip == 1) ? MUF * fn : -MUF * fn);
        }
        u[3 + 3 * f] = fn;
        u[4 + 3 * f] = ft;
        u[5 + 3 * f] = (xb[6 + f] - xa[6 + f]) / DT;
      }
    }
  }
}

// Free-motion warm start: states (x, y, theta, p_x, p_y) and forces (F_n, F_t) interpolated
// from the network samples at every knot, with optimised timing also the duration
// (channel 7, clamped to its bounds); the start state at knot 0; the pusher velocity of
// interval k as the forward difference (p_{k+1} - p_k) / h_k of the decoded positions
// (h_k = dt with the fixed step), so the pusher defect rows hold; row N has u = 0.
// Row width 9 (u = F_n, F_t, v_x, v_y) or 10 (and h).
__global__ void k_decode_warm_free(long B, const long long* B_dev, const float* Y, int O, const float* x0,
                                   int inst_stride, const int32_t* nseg, const int32_t* knots, int smax, int nmax,
                                   int timed, float* warm) {
  const int width = timed ? 10 : 9;
  const long Bn = B_dev ? *B_dev : B;
  const long b = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= Bn) return;
  const int K = checked_segments(nseg, knots, b, smax, nmax);
  const float* y = Y + b * (long)O + 2;
  float* Wr = warm + b * (long)(nmax + 1) * width;
  for (int r = 0; r < (nmax + 1) * width; ++r) Wr[r] = 0.f;
  int k0 = 0;
  for (int j = 0; j < K && j < smax; ++j) {
    const int nj = knots[b * smax + j];
    for (int k = 0; k <= nj && k0 + k <= nmax; ++k) {
      const float p = (nj > 0) ? (float)k / (float)nj * (WS_SLOTS - 1) : 0.f;
      const int i = min((int)floorf(p), WS_SLOTS - 2);
      const float fr = p - (float)i;
      for (int c = 0; c < (timed ? 8 : 7); ++c) {
        const float a0 = y[((long)j * WS_SLOTS + i) * WS_CH + c], a1 = y[((long)j * WS_SLOTS + i + 1) * WS_CH + c];
        const float val = a0 + fr * (a1 - a0);
        if (c < 7)
          Wr[(k0 + k) * width + c] = val;
        else
          Wr[(k0 + k) * width + 9] =
              fminf(fmaxf(val, (float)push_free_timed::H_MIN), (float)push_free_timed::H_MAX);
      }
    }
    k0 += nj;
  }
  const int N = min(k0, nmax);
  for (int c = 0; c < 5; ++c) Wr[c] = x0[b * inst_stride * 5 + c];
  for (int k = 0; k < N; ++k) {
    float* r = Wr + k * width;
    const float h = timed ? r[9] : (float)push_free::DT;
    r[7] = (r[width + 3] - r[3]) / h;
    r[8] = (r[width + 4] - r[4]) / h;
  }
  for (int c = 5; c < width; ++c) Wr[N * width + c] = 0.f;
}

}  // namespace comet

// ==================================================================================
// Host side
// ==================================================================================
using namespace comet;

struct comet_mlp {
  int in_dim, hidden, layers, out_dim;
  int wsegs;                           // segments of the warm-start block: min(8, (out_dim - 2) / 120)
  long long max_batch;
  int nl;                              // linear layers = layers + 1
  std::vector<int> K, N;               // per linear layer: in, out
  std::vector<long long> woff, boff;   // offsets into the flat parameter vector
  long long n_params = 0;
  float *P = nullptr, *G = nullptr, *Mm = nullptr, *Vv = nullptr;  // master params, grads, Adam moments
  bf16 *Wb = nullptr, *WT = nullptr;                              // BF16 weights and transposes (concatenated)
  std::vector<long long> wboff;        // offsets of each layer's weights in Wb / WT
  bf16* X0 = nullptr;                  // encoded input [B][in]
  std::vector<float*> Z;               // pre-activations [B][hidden] per hidden layer
  std::vector<bf16*> H;                // activations (H[0] = X0) [B][dim]
  float *Y = nullptr, *dY = nullptr;   // output and its gradient [B][out]
  bf16 *dYb = nullptr;
  // backward buffers, one per layer so that the two streams of the backward pass never
  // wait for a buffer to be free: dzc[l] per-wave column sums of the hidden gradient that
  // layer l's input product leaves [2 ceil(B/128)][hidden]; dZl[l] BF16 gradient of hidden
  // layer l [B][hidden]
  std::vector<float*> dzc;
  std::vector<bf16*> dZl;
  float *cnt = nullptr, *lossd = nullptr;
  float* part = nullptr;               // partial sums: split weight gradients / bias column sums
  float* red = nullptr;                // per-block partials of the loss reductions [LOSS_BLOCKS][4]
  // batch-contiguous BF16 copies for the weight-gradient products (training, B % 8 == 0):
  // HT[l] = H[l]^T [K_l][ldt], GT = the current layer's output gradient transposed [N][ldt]
  std::vector<bf16*> HT;
  std::vector<bf16*> GTl;              // GTl[l] = layer l's output gradient transposed [N_l][ldt]
  long ldt = 0;
  long long step = 0;
  // the backward pass runs the chain of input-gradient products on the caller's stream and
  // each layer's weight gradient and bias sums beside it on this stream: evB[l] = layer l's
  // input gradient done, done = all weight gradients done
  hipStream_t aux = nullptr;
  hipEvent_t fork = nullptr, done = nullptr;
  std::vector<hipEvent_t> evB;
};

namespace {

unsigned nblk(long long n, int bs) { return (unsigned)std::max<long long>(1, (n + bs - 1) / bs); }

// operand requirements of k_gemm: contiguous extents, leading dimensions and base
// addresses allow 16-byte vector loads
bool vec_ok(const void* p, long ld, long contiguous_extent) {
  return ((uintptr_t)p % 16 == 0) && ld % 8 == 0 && contiguous_extent % 8 == 0;
}

// launches k_gemm; returns the number of contraction splits (partial-sum slabs) used
template <bool A_K, bool B_K, int EPI>
int gemm(hipStream_t s, int M, int N, int K, const bf16* A, long lda, const bf16* Bp, long ldb, const Epi& ep,
         const long long* M_dev = nullptr, int split = 1) {
  const int kc = split > 1 ? (int)((((long)K + split - 1) / split + GBK - 1) / GBK * GBK) : std::max(K, 1);
  const int nz = split > 1 ? (K + kc - 1) / kc : 1;
  dim3 grid(nblk(N, GBN), nblk(M, GBM), nz);
  hipLaunchKernelGGL((k_gemm<A_K, B_K, EPI>), grid, dim3(256), 0, s, M, N, K, A, lda, Bp, ldb, ep, M_dev, kc);
  return nz;
}

// splits of the batch contraction of a weight-gradient GEMM: about 512 blocks (two per
// CU), at least 256 batch rows per split.  Each split adds an FP32 slab of the gradient
// that k_sum_slabs reads back; aiming at 1,024 blocks doubled that traffic and made the
// 8,192-sample training step 6 % slower, aiming at 256 left the products short of blocks.
int wgrad_splits(int M, int N, int B) {
  const long blocks = (long)nblk(N, GBN) * nblk(M, GBM);
  const long want = (512 + blocks - 1) / blocks;
  return (int)std::max<long>(1, std::min<long>({want, (long)B / 256, (long)MAX_SPLIT}));
}

void refresh_weights(comet_mlp* m, hipStream_t s) {
  for (int l = 0; l < m->nl; ++l) {
    const long long n = (long long)m->N[l] * m->K[l];
    hipLaunchKernelGGL(k_refresh, dim3(nblk(n, 256)), dim3(256), 0, s, m->P + m->woff[l], m->N[l], m->K[l],
                       m->Wb + m->wboff[l], m->WT + m->wboff[l]);
  }
}

}  // namespace

namespace comet {

void mlp_forward_t(comet_mlp* m, hipStream_t s, int B, const long long* B_dev, bool keep_transposed, bool train);

// forward for B rows of m->H[0] (at most *B_dev rows if given); Y filled.
void mlp_forward(comet_mlp* m, hipStream_t s, int B, const long long* B_dev) {
  mlp_forward_t(m, s, B, B_dev, false, false);
}

// forward; with keep_transposed the hidden activations are also written transposed (HT);
// the FP32 pre-activations Z, which only the backward pass reads, are written when training
void mlp_forward_t(comet_mlp* m, hipStream_t s, int B, const long long* B_dev, bool keep_transposed, bool train) {
  for (int l = 0; l < m->nl; ++l) {
    const int K = m->K[l], N = m->N[l];
    Epi ep{};
    ep.bias = m->P + m->boff[l];
    ep.ldc = N;
    const bf16* Wl = m->Wb + m->wboff[l];
    if (l < m->nl - 1) {
      ep.z = train ? m->Z[l] : nullptr;
      ep.h = m->H[l + 1];
      if (keep_transposed) {
        ep.ht = m->HT[l + 1];
        ep.ldt = m->ldt;
      }
      gemm<true, true, EPI_HIDDEN>(s, B, N, K, m->H[l], K, Wl, K, ep, B_dev);
    } else {
      ep.z = m->Y;
      gemm<true, true, EPI_OUT>(s, B, N, K, m->H[l], K, Wl, K, ep, B_dev);
    }
  }
}

// hooks for the expansion graph (sizes on the device)
int mlp_in_dim(const comet_mlp* m) { return m->in_dim; }
int mlp_out_dim(const comet_mlp* m) { return m->out_dim; }
long long mlp_max_batch(const comet_mlp* m) { return m->max_batch; }
const float* mlp_output(const comet_mlp* m) { return m->Y; }

void mlp_encode_dev(comet_mlp* m, int task, hipStream_t s, long long Bmax, const long long* B_dev, const float* x0,
                    const float* goal, const float* inst, int inst_stride, const int32_t* nseg, const int32_t* modes,
                    const int32_t* knots, int smax) {
  auto kern = task == COMET_TASK_FLIP ? k_encode_flip : (is_free_task(task) ? k_encode_free : k_encode_push);
  hipLaunchKernelGGL(kern, dim3(nblk(Bmax * m->in_dim, 256)), dim3(256), 0, s, (long)Bmax, x0, goal, inst,
                     inst_stride, nseg, modes, knots, smax, m->in_dim, m->H[0], B_dev);
}

void mlp_decode_warm_dev(comet_mlp* m, int task, hipStream_t s, long long Bmax, const long long* B_dev,
                         const float* x0, int inst_stride, const int32_t* nseg, const int32_t* modes,
                         const int32_t* knots, int smax, int nmax, float* warm) {
  if (task == COMET_TASK_FLIP)
    hipLaunchKernelGGL(k_decode_warm_flip, dim3(nblk(Bmax, 128)), dim3(128), 0, s, (long)Bmax, B_dev, m->Y,
                       m->out_dim, x0, inst_stride, nseg, modes, knots, smax, nmax, warm);
  else if (is_free_task(task))
    hipLaunchKernelGGL(k_decode_warm_free, dim3(nblk(Bmax, 128)), dim3(128), 0, s, (long)Bmax, B_dev, m->Y,
                       m->out_dim, x0, inst_stride, nseg, knots, smax, nmax,
                       task == COMET_TASK_PUSH_FREE_TIMED ? 1 : 0, warm);
  else
    hipLaunchKernelGGL(k_decode_warm, dim3(nblk(Bmax, 128)), dim3(128), 0, s, (long)Bmax, B_dev, m->Y, m->out_dim,
                       x0, inst_stride, nseg, knots, smax, nmax, task == COMET_TASK_PUSH_TIMED ? 8 : 7, warm);
}

// segments of an order and of the warm-start block, and the encoded width, per task
int mlp_task_segments(int task) { return is_free_task(task) ? FREE_SEGS : 6; }
int mlp_task_in_dim(int task) { return POSE_DIMS + mlp_task_segments(task) * SEG_SLOT; }
int mlp_task_out_dim(int task) { return 2 + mlp_task_segments(task) * WS_SLOTS * WS_CH; }
int mlp_warm_segments(const comet_mlp* m) { return m->wsegs; }

}  // namespace comet

extern "C" {

comet_status comet_mlp_create(int32_t in_dim, int32_t hidden, int32_t layers, int32_t out_dim, int64_t max_batch,
                              uint64_t seed, comet_mlp** out) {
  if (!out || in_dim < 8 || hidden < 8 || layers < 1 || layers > 16 || out_dim < 2 + 6 * WS_SLOTS * WS_CH ||
      max_batch < 1 || in_dim % 8 || hidden % 8 || out_dim % 8)
    return COMET_EINVAL;
  *out = nullptr;
  comet_mlp* m = new comet_mlp();
  m->in_dim = in_dim;
  m->hidden = hidden;
  m->layers = layers;
  m->out_dim = out_dim;
  m->wsegs = std::min(FREE_SEGS, (out_dim - 2) / (WS_SLOTS * WS_CH));
  m->max_batch = max_batch;
  m->nl = layers + 1;
  long long off = 0, woff = 0;
  for (int l = 0; l < m->nl; ++l) {
    const int K = (l == 0) ? in_dim : hidden, N = (l == m->nl - 1) ? out_dim : hidden;
    m->K.push_back(K);
    m->N.push_back(N);
    m->woff.push_back(off);
    off += (long long)N * K;
    m->boff.push_back(off);
    off += N;
    m->wboff.push_back(woff);
    woff += (long long)N * K;
  }
  m->n_params = off;
  bool ok = true;
  auto A = [&](void** p, size_t bytes) { ok = ok && hipMalloc(p, std::max<size_t>(bytes, 8)) == hipSuccess; };
  A((void**)&m->P, 4 * off);
  A((void**)&m->G, 4 * off);
  A((void**)&m->Mm, 4 * off);
  A((void**)&m->Vv, 4 * off);
  A((void**)&m->Wb, 2 * woff);
  A((void**)&m->WT, 2 * woff);
  const long long B = max_batch;
  m->H.assign(m->nl, nullptr);
  m->Z.assign(m->nl - 1, nullptr);
  A((void**)&m->H[0], 2 * B * in_dim);
  for (int l = 1; l < m->nl; ++l) A((void**)&m->H[l], 2 * B * hidden);
  for (int l = 0; l < m->nl - 1; ++l) A((void**)&m->Z[l], 4 * B * hidden);
  m->X0 = m->H[0];
  A((void**)&m->Y, 4 * B * out_dim);
  A((void**)&m->dY, 4 * B * out_dim);
  A((void**)&m->dYb, 2 * B * out_dim);
  m->dzc.assign(m->nl, nullptr);
  m->dZl.assign(m->nl, nullptr);
  for (int l = 1; l < m->nl; ++l) A((void**)&m->dzc[l], 4 * 2 * ((B + GBM - 1) / GBM) * hidden);
  for (int l = 0; l < m->nl - 1; ++l) A((void**)&m->dZl[l], 2 * B * hidden);
  m->ldt = (long)((B + 7) / 8 * 8);
  m->HT.assign(m->nl, nullptr);
  for (int l = 0; l < m->nl; ++l) A((void**)&m->HT[l], 2 * (size_t)m->K[l] * m->ldt);
  m->GTl.assign(m->nl, nullptr);
  for (int l = 0; l < m->nl; ++l) A((void**)&m->GTl[l], 2 * (size_t)m->N[l] * m->ldt);
  ok = ok && hipStreamCreateWithFlags(&m->aux, hipStreamNonBlocking) == hipSuccess;
  ok = ok && hipEventCreateWithFlags(&m->fork, hipEventDisableTiming) == hipSuccess;
  ok = ok && hipEventCreateWithFlags(&m->done, hipEventDisableTiming) == hipSuccess;
  m->evB.assign(m->nl, nullptr);
  for (int l = 0; l < m->nl; ++l)
    ok = ok && hipEventCreateWithFlags(&m->evB[l], hipEventDisableTiming) == hipSuccess;
  A((void**)&m->cnt, 4 * 4);
  A((void**)&m->lossd, 4 * 4);
  {
    long long max_nk = 0, max_n = 0;
    for (int l = 0; l < m->nl; ++l) {
      max_nk = std::max(max_nk, (long long)m->N[l] * m->K[l]);
      max_n = std::max(max_n, (long long)m->N[l]);
    }
    A((void**)&m->part, 4 * std::max<long long>(MAX_SPLIT * max_nk, COLSUM_ROWS * max_n));
  }
  A((void**)&m->red, 4 * 4 * LOSS_BLOCKS);
  if (!ok) {
    (void)hipGetLastError();
    comet_mlp_destroy(m);
    return COMET_ENOMEM;
  }
  for (int l = 0; l < m->nl; ++l) {
    const long long nw = (long long)m->N[l] * m->K[l];
    hipLaunchKernelGGL(k_init_uniform, dim3(nblk(nw, 256)), dim3(256), 0, 0, m->P + m->woff[l], (long)nw,
                       1.0f / std::sqrt((float)m->K[l]), (unsigned long long)seed, (long)m->woff[l]);
    hipLaunchKernelGGL(k_zero, dim3(nblk(m->N[l], 256)), dim3(256), 0, 0, m->P + m->boff[l], (long)m->N[l]);
  }
  hipLaunchKernelGGL(k_zero, dim3(nblk(off, 256)), dim3(256), 0, 0, m->Mm, (long)off);
  hipLaunchKernelGGL(k_zero, dim3(nblk(off, 256)), dim3(256), 0, 0, m->Vv, (long)off);
  hipLaunchKernelGGL(k_zero, dim3(nblk(off, 256)), dim3(256), 0, 0, m->G, (long)off);
  refresh_weights(m, 0);
  if (hipDeviceSynchronize() != hipSuccess) {
    comet_mlp_destroy(m);
    return COMET_EHIP;
  }
  *out = m;
  return COMET_OK;
}

void comet_mlp_destroy(comet_mlp* m) {
  if (!m) return;
  std::vector<void*> ps = {m->P, m->G, m->Mm, m->Vv, m->Wb, m->WT, m->Y, m->dY, m->dYb, m->cnt, m->lossd, m->part,
                           m->red};
  for (auto* h : m->H) ps.push_back(h);
  for (auto* z : m->Z) ps.push_back(z);
  for (auto* h : m->HT) ps.push_back(h);
  for (auto* h : m->GTl) ps.push_back(h);
  for (auto* h : m->dZl) ps.push_back(h);
  for (auto* h : m->dzc) ps.push_back(h);
  for (void* p : ps)
    if (p) (void)hipFree(p);
  for (auto* e : m->evB)
    if (e) (void)hipEventDestroy(e);
  if (m->fork) (void)hipEventDestroy(m->fork);
  if (m->done) (void)hipEventDestroy(m->done);
  if (m->aux) (void)hipStreamDestroy(m->aux);
  delete m;
}

comet_status comet_mlp_num_params(const comet_mlp* m, int64_t* n) {
  if (!m || !n) return COMET_EINVAL;
  *n = m->n_params;
  return COMET_OK;
}

comet_status comet_mlp_params(comet_mlp* m, void* stream, int32_t set, float* flat) {
  if (!m || !flat) return COMET_EINVAL;
  hipStream_t s = (hipStream_t)stream;
  if (set) {
    if (hipMemcpyAsync(m->P, flat, 4 * m->n_params, hipMemcpyDeviceToDevice, s) != hipSuccess) return COMET_EHIP;
    refresh_weights(m, s);
    hipLaunchKernelGGL(k_zero, dim3(nblk(m->n_params, 256)), dim3(256), 0, s, m->Mm, (long)m->n_params);
    hipLaunchKernelGGL(k_zero, dim3(nblk(m->n_params, 256)), dim3(256), 0, s, m->Vv, (long)m->n_params);
    m->step = 0;
  } else {
    if (hipMemcpyAsync(flat, m->P, 4 * m->n_params, hipMemcpyDeviceToDevice, s) != hipSuccess) return COMET_EHIP;
  }
  return hipGetLastError() == hipSuccess ? COMET_OK : COMET_EHIP;
}

comet_status comet_mlp_grads(comet_mlp* m, void* stream, float* flat) {
  if (!m || !flat) return COMET_EINVAL;
  return hipMemcpyAsync(flat, m->G, 4 * m->n_params, hipMemcpyDeviceToDevice, (hipStream_t)stream) == hipSuccess
             ? COMET_OK
             : COMET_EHIP;
}

comet_status comet_mlp_forward(comet_mlp* m, void* stream, int64_t B, const uint16_t* x_bf16, float* out) {
  if (!m || B < 0 || B > m->max_batch) return COMET_EINVAL;
  if (B == 0) return COMET_OK;   // empty batch: no array is touched, pointers may be NULL
  if (!x_bf16 || !out) return COMET_EINVAL;
  hipStream_t s = (hipStream_t)stream;
  if (hipMemcpyAsync(m->H[0], x_bf16, 2 * B * m->in_dim, hipMemcpyDeviceToDevice, s) != hipSuccess) return COMET_EHIP;
  mlp_forward(m, s, (int)B, nullptr);
  if (hipMemcpyAsync(out, m->Y, 4 * B * m->out_dim, hipMemcpyDeviceToDevice, s) != hipSuccess) return COMET_EHIP;
  return hipGetLastError() == hipSuccess ? COMET_OK : COMET_EHIP;
}

comet_status comet_mlp_train_step(comet_mlp* m, void* stream, int64_t B, const uint16_t* x_bf16, const float* y_feas,
                                  const float* y_cost, const float* y_traj, const float* traj_mask, float lr,
                                  float weight_decay, float* loss) {
  if (!m || !x_bf16 || !y_feas || !y_cost || !y_traj || !traj_mask) return COMET_EINVAL;
  if (B < 1 || B > m->max_batch || B * (int64_t)m->out_dim >= (1ll << 31) || !(lr >= 0.f)) return COMET_EINVAL;
  // the loss kernel reads the warm-start targets in pairs and the mask in fours
  if ((uintptr_t)y_traj % 8 || (uintptr_t)traj_mask % 16) return COMET_EINVAL;
  hipStream_t s = (hipStream_t)stream;
  const int Bi = (int)B, O = m->out_dim, Wn = m->wsegs * WS_SLOTS * WS_CH;
  if (hipMemcpyAsync(m->H[0], x_bf16, 2 * B * m->in_dim, hipMemcpyDeviceToDevice, s) != hipSuccess) return COMET_EHIP;
  // With B a multiple of 8 the weight gradients contract over batch-contiguous copies of
  // their operands (16-byte loads straight into the matrix-core tiles): the hidden
  // activations and the hidden gradients are written transposed by the epilogues that
  // produce them, the input and the output gradient by k_transpose_bf16.  Otherwise the
  // products read the row-major tensors and transpose through LDS.
  const bool tr = (Bi % 8 == 0);
  if (tr)
    hipLaunchKernelGGL(k_transpose_bf16, dim3(nblk(m->in_dim, 64), nblk(Bi, 64)), dim3(256), 0, s, m->H[0],
                       (long)m->in_dim, Bi, m->in_dim, m->HT[0], m->ldt);
  mlp_forward_t(m, s, Bi, nullptr, tr, true);
  hipLaunchKernelGGL(k_loss_counts, dim3(LOSS_BLOCKS), dim3(256), 0, s, Bi, Wn, y_feas, traj_mask, m->red);
  hipLaunchKernelGGL(k_reduce_partials, dim3(1), dim3(256), 0, s, m->red, LOSS_BLOCKS, 2, m->cnt);
  hipLaunchKernelGGL(k_loss_grad, dim3(LOSS_BLOCKS), dim3(256), 0, s, Bi, O, Wn, m->Y, y_feas, y_cost, y_traj,
                     traj_mask, m->cnt, m->dY, m->dYb, m->red);
  hipLaunchKernelGGL(k_reduce_partials, dim3(1), dim3(256), 0, s, m->red, LOSS_BLOCKS, 3, m->lossd);
  const int L = m->nl;
  if (tr)
    hipLaunchKernelGGL(k_transpose_bf16, dim3(nblk(O, 64), nblk(Bi, 64)), dim3(256), 0, s, m->dYb, (long)O, Bi, O,
                       m->GTl[L - 1], m->ldt);
  // backward through the linear layers: the chain of input-gradient products runs on the
  // caller's stream; each layer's weight gradient and bias sums run beside it on m->aux,
  // after the input product that produced the gradient they read (event evB[l+1]).
  // Every gradient buffer belongs to one layer, so neither stream waits for a buffer.
  if (hipEventRecord(m->fork, s) != hipSuccess || hipStreamWaitEvent(m->aux, m->fork, 0) != hipSuccess)
    return COMET_EHIP;
  for (int l = L - 1; l >= 1; --l) {
    // dZ_{l-1} [B][K] = (G [B][N] . W_l [N][K]) * gelu'(Z_{l-1}), W_l read through its
    // transpose so both operands are contraction-contiguous
    const int K = m->K[l], N = m->N[l];
    const bf16* g = (l == L - 1) ? m->dYb : m->dZl[l];
    Epi ex{};
    ex.colpart = m->dzc[l];
    ex.h = m->dZl[l - 1];
    ex.zprev = m->Z[l - 1];
    ex.ldc = K;
    if (tr) {   // layer l-1's weight gradient reads it transposed
      ex.ht = m->GTl[l - 1];
      ex.ldt = m->ldt;
    }
    gemm<true, true, EPI_DX>(s, Bi, K, N, g, N, m->WT + m->wboff[l], N, ex);
    if (hipEventRecord(m->evB[l], s) != hipSuccess) return COMET_EHIP;
  }
  for (int l = L - 1; l >= 0; --l) {
    const int K = m->K[l], N = m->N[l];
    if (l < L - 1 && hipStreamWaitEvent(m->aux, m->evB[l + 1], 0) != hipSuccess) return COMET_EHIP;
    // dW_l [N][K] = G^T [N][B] . H_l [B][K]: contraction over the batch, split into
    // partial-sum slabs that k_sum_slabs adds
    const int split = wgrad_splits(N, K, Bi);
    Epi ew{};
    ew.z = m->part;
    ew.ldc = K;
    ew.slab = (long)N * K;
    const bf16* g = (l == L - 1) ? m->dYb : m->dZl[l];
    const int nzs = tr ? gemm<true, true, EPI_PARTIAL>(m->aux, N, K, Bi, m->GTl[l], m->ldt, m->HT[l], m->ldt, ew,
                                                       nullptr, split)
                       : gemm<false, false, EPI_PARTIAL>(m->aux, N, K, Bi, g, N, m->H[l], K, ew, nullptr, split);
    if (l == L - 1) {   // output layer: column sums of the FP32 loss gradient (they reuse m->part)
      hipLaunchKernelGGL(k_sum_slabs, dim3(nblk((long long)N * K, 256)), dim3(256), 0, m->aux, m->part, nzs,
                         (long)N * K, m->G + m->woff[l]);
      const int ry = std::max(1, std::min(COLSUM_ROWS, (Bi + 31) / 32));
      hipLaunchKernelGGL(k_colsum_part, dim3(nblk(N, 256), ry), dim3(256), 0, m->aux, m->dY, Bi, N, m->part);
      hipLaunchKernelGGL(k_sum_rows, dim3(nblk(N, 64)), dim3(256), 0, m->aux, m->part, ry, (long)N,
                         m->G + m->boff[l]);
    } else {            // hidden layers: the slabs and the per-wave column sums left by layer
                        // l+1's input product, in one launch
      const int nbw = (int)nblk((long long)N * K, 256);
      hipLaunchKernelGGL(k_sum_grads, dim3(nbw + (int)nblk(N, 64)), dim3(256), 0, m->aux, m->part, nzs,
                         (long)N * K, m->G + m->woff[l], nbw, m->dzc[l + 1], 2 * (int)nblk(Bi, GBM), (long)N,
                         m->G + m->boff[l]);
    }
  }
  if (hipEventRecord(m->done, m->aux) != hipSuccess || hipStreamWaitEvent(s, m->done, 0) != hipSuccess)
    return COMET_EHIP;
  // AdamW on the FP32 masters, then refresh the BF16 copies
  m->step += 1;
  const float b1 = 0.9f, b2 = 0.999f;
  const float bc1 = 1.f - std::pow(b1, (float)m->step), bc2 = 1.f - std::pow(b2, (float)m->step);
  LayerTable T{};
  T.nl = m->nl;
  for (int l = 0; l < m->nl; ++l) {
    T.woff[l] = m->woff[l];
    T.boff[l] = m->boff[l];
    T.wboff[l] = m->wboff[l];
    T.N[l] = m->N[l];
    T.K[l] = m->K[l];
  }
  hipLaunchKernelGGL(k_adamw_refresh, dim3(nblk(m->n_params, 256)), dim3(256), 0, s, m->P, m->Mm, m->Vv, m->G,
                     (long)m->n_params, lr, b1, b2, 1e-8f, weight_decay, bc1, bc2, T, m->Wb, m->WT);
  if (loss && hipMemcpyAsync(loss, m->lossd, 4 * 3, hipMemcpyDeviceToDevice, s) != hipSuccess) return COMET_EHIP;
  return hipGetLastError() == hipSuccess ? COMET_OK : COMET_EHIP;
}

static bool mlp_task_ok(int task) {
  return task == COMET_TASK_PUSH || task == COMET_TASK_FLIP || task == COMET_TASK_PUSH_TIMED || is_free_task(task);
}

comet_status comet_mlp_encode(comet_task task, void* stream, int64_t B, const float* x0, const float* goal,
                              const float* inst, const int32_t* nseg, const int32_t* modes, const int32_t* knots,
                              int32_t smax, int32_t in_dim, uint16_t* x_bf16) {
  if (!mlp_task_ok(task) || B < 0 || smax < 1 || smax > mlp_task_segments(task) || in_dim < mlp_task_in_dim(task))
    return COMET_EINVAL;
  if (B == 0) return COMET_OK;   // empty batch: no array is touched, pointers may be NULL
  if (!x0 || !goal || !inst || !nseg || !modes || !knots || !x_bf16) return COMET_EINVAL;
  auto kern = task == COMET_TASK_FLIP ? k_encode_flip : (is_free_task(task) ? k_encode_free : k_encode_push);
  hipLaunchKernelGGL(kern, dim3(nblk(B * in_dim, 256)), dim3(256), 0, (hipStream_t)stream, (long)B, x0, goal, inst, 1,
                     nseg, modes, knots, smax, in_dim, (bf16*)x_bf16, (const long long*)nullptr);
  return hipGetLastError() == hipSuccess ? COMET_OK : COMET_EHIP;
}

comet_status comet_mlp_targets(comet_task task, void* stream, int64_t B, const float* traj, int32_t nmax,
                               const int32_t* nseg, const int32_t* knots, int32_t smax, const uint8_t* feasible,
                               const float* cost, float* y_feas, float* y_cost, float* y_traj, float* traj_mask) {
  if (!mlp_task_ok(task) || B < 0 || smax < 1 || smax > mlp_task_segments(task) || nmax < 1) return COMET_EINVAL;
  if (B == 0) return COMET_OK;   // empty batch: no array is touched, pointers may be NULL
  if (!traj || !nseg || !knots || !feasible || !cost || !y_feas || !y_cost || !y_traj || !traj_mask)
    return COMET_EINVAL;
  // trajectory row width, the channels sampled and the column of channel 7: pushing (x, u)
  // 7 channels; timed pushing 8 (with the duration); flipping the 8 states of a 17-wide
  // row; free motion the 5 states and 2 forces of a 9-wide row, with optimised timing also
  // the duration from column 9 of a 10-wide row
  int row = 7, nch = 7, col7 = 7;
  switch (task) {
    case COMET_TASK_FLIP: row = 17; nch = 8; break;
    case COMET_TASK_PUSH_TIMED: row = 8; nch = 8; break;
    case COMET_TASK_PUSH_FREE: row = 9; break;
    case COMET_TASK_PUSH_FREE_TIMED: row = 10; nch = 8; col7 = 9; break;
    default: break;
  }
  hipLaunchKernelGGL(k_targets, dim3(nblk(B, 128)), dim3(128), 0, (hipStream_t)stream, (long)B, traj, nmax, row, nch,
                     col7, mlp_task_segments(task), nseg, knots, smax, feasible, cost, y_feas, y_cost, y_traj,
                     traj_mask);
  return hipGetLastError() == hipSuccess ? COMET_OK : COMET_EHIP;
}

comet_status comet_mlp_decode_warm(comet_task task, void* stream, int64_t B, const float* out, int32_t out_dim,
                                   const float* x0, const int32_t* nseg, const int32_t* modes, const int32_t* knots,
                                   int32_t smax, int32_t nmax, float* warm) {
  if (!mlp_task_ok(task) || B < 0 || smax < 1 || smax > mlp_task_segments(task) || nmax < 1 ||
      out_dim < mlp_task_out_dim(task))
    return COMET_EINVAL;
  if (B == 0) return COMET_OK;   // empty batch: no array is touched, pointers may be NULL
  if (!out || !x0 || !nseg || !knots || !warm || (task == COMET_TASK_FLIP && !modes)) return COMET_EINVAL;
  if (task == COMET_TASK_FLIP)
    hipLaunchKernelGGL(k_decode_warm_flip, dim3(nblk(B, 128)), dim3(128), 0, (hipStream_t)stream, (long)B,
                       (const long long*)nullptr, out, out_dim, x0, 1, nseg, modes, knots, smax, nmax, warm);
  else if (is_free_task(task))
    hipLaunchKernelGGL(k_decode_warm_free, dim3(nblk(B, 128)), dim3(128), 0, (hipStream_t)stream, (long)B,
                       (const long long*)nullptr, out, out_dim, x0, 1, nseg, knots, smax, nmax,
                       task == COMET_TASK_PUSH_FREE_TIMED ? 1 : 0, warm);
  else
    hipLaunchKernelGGL(k_decode_warm, dim3(nblk(B, 128)), dim3(128), 0, (hipStream_t)stream, (long)B,
                       (const long long*)nullptr, out, out_dim, x0, 1, nseg, knots, smax, nmax,
                       task == COMET_TASK_PUSH_TIMED ? 8 : 7, warm);
  return hipGetLastError() == hipSuccess ? COMET_OK : COMET_EHIP;
}

}  // extern "C"
