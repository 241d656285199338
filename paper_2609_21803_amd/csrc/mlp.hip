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

namespace comet {

typedef unsigned short bf16;
typedef __attribute__((__vector_size__(8 * sizeof(short)))) short bf16x8;
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
// GEMM: C(m, n) = sum_k A(m, k) B(k, n), A(m,k) = A[m*am + k*ak], B(k,n) = Bp[n*bn + k*bk],
// BF16 operands, FP32 accumulation.  Block tile 64 x 64, K step 32, 4 waves of 32 x 32
// (2 x 2 MFMA 16x16x32 tiles).  A_K / B_K: the contraction index is the contiguous one.
// ---------------------------------------------------------------------------------
enum { EPI_HIDDEN = 0, EPI_OUT = 1, EPI_DX = 2, EPI_PLAIN = 3 };

struct Epi {
  const float* bias;   // [N] (EPI_HIDDEN, EPI_OUT)
  float* z;            // FP32 pre-activation out (EPI_HIDDEN) / FP32 result (EPI_OUT, EPI_PLAIN) / dZ (EPI_DX)
  bf16* h;             // BF16 activation (EPI_HIDDEN) / BF16 gradient (EPI_DX)
  const float* zprev;  // pre-activation of the layer below (EPI_DX)
  long ldc;            // row stride of the outputs
};

constexpr int GBM = 64, GBN = 64, GBK = 32, GPAD = 8;

template <bool A_K, bool B_K, int EPI>
__global__ __launch_bounds__(256) void k_gemm(int M, int N, int K, const bf16* __restrict__ A, long am, long ak,
                                              const bf16* __restrict__ Bp, long bn, long bk, Epi ep,
                                              const long long* M_dev) {
  __shared__ bf16 As[GBM][GBK + GPAD];
  __shared__ bf16 Bs[GBN][GBK + GPAD];
  if (M_dev) M = (int)min((long long)M, *M_dev);
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  const int wm = w >> 1, wn = w & 1;
  const int m0 = blockIdx.y * GBM, n0 = blockIdx.x * GBN;
  if (m0 >= M) return;
  f32x4 acc[2][2];
  for (int i = 0; i < 2; ++i)
    for (int j = 0; j < 2; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
  for (int k0 = 0; k0 < K; k0 += GBK) {
    // A tile -> As[m][k]
    if (A_K) {
      const int r = t >> 2, kc = (t & 3) * 8;
      const int m = m0 + r;
      for (int i = 0; i < 8; ++i) {
        const int k = k0 + kc + i;
        As[r][kc + i] = (m < M && k < K) ? A[(long)m * am + (long)k * ak] : (bf16)0;
      }
    } else {
      const int kk = t >> 3, mc = (t & 7) * 8;
      const int k = k0 + kk;
      for (int i = 0; i < 8; ++i) {
        const int m = m0 + mc + i;
        As[mc + i][kk] = (m < M && k < K) ? A[(long)m * am + (long)k * ak] : (bf16)0;
      }
    }
    // B tile -> Bs[n][k]
    if (B_K) {
      const int r = t >> 2, kc = (t & 3) * 8;
      const int n = n0 + r;
      for (int i = 0; i < 8; ++i) {
        const int k = k0 + kc + i;
        Bs[r][kc + i] = (n < N && k < K) ? Bp[(long)n * bn + (long)k * bk] : (bf16)0;
      }
    } else {
      const int kk = t >> 3, nc = (t & 7) * 8;
      const int k = k0 + kk;
      for (int i = 0; i < 8; ++i) {
        const int n = n0 + nc + i;
        Bs[nc + i][kk] = (n < N && k < K) ? Bp[(long)n * bn + (long)k * bk] : (bf16)0;
      }
    }
    __syncthreads();
    const int kq = (lane >> 4) * 8;
    bf16x8 a[2], b[2];
    for (int i = 0; i < 2; ++i) {
      const int r = wm * 32 + i * 16 + (lane & 15);
      a[i] = *reinterpret_cast<const bf16x8*>(&As[r][kq]);
    }
    for (int j = 0; j < 2; ++j) {
      const int c = wn * 32 + j * 16 + (lane & 15);
      b[j] = *reinterpret_cast<const bf16x8*>(&Bs[c][kq]);
    }
    for (int i = 0; i < 2; ++i)
      for (int j = 0; j < 2; ++j) acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[i], b[j], acc[i][j], 0, 0, 0);
    __syncthreads();
  }
  // accumulator layout: lane holds rows 4*(lane/16) + r, column lane%16 of each 16x16 tile
  for (int i = 0; i < 2; ++i)
    for (int j = 0; j < 2; ++j)
      for (int r = 0; r < 4; ++r) {
        const int m = m0 + wm * 32 + i * 16 + (lane >> 4) * 4 + r;
        const int n = n0 + wn * 32 + j * 16 + (lane & 15);
        if (m >= M || n >= N) continue;
        const float v = acc[i][j][r];
        const long o = (long)m * ep.ldc + n;
        if (EPI == EPI_HIDDEN) {
          const float z = v + ep.bias[n];
          ep.z[o] = z;
          ep.h[o] = to_bf16(gelu(z));
        } else if (EPI == EPI_OUT) {
          ep.z[o] = v + ep.bias[n];
        } else if (EPI == EPI_DX) {
          const float d = v * gelu_grad(ep.zprev[o]);
          ep.z[o] = d;
          ep.h[o] = to_bf16(d);
        } else {
          ep.z[o] = v;
        }
      }
}

// column sums of an FP32 [M][N] matrix (bias gradients)
__global__ void k_colsum(const float* X, int M, int N, float* out) {
  const int n = blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= N) return;
  float s = 0.f;
  for (int m = 0; m < M; ++m) s += X[(long)m * N + n];
  out[n] = s;
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
__global__ void k_loss_counts(int B, int W, const float* y_feas, const float* mask, float* cnt) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  const long n = (long)B * W;
  float c = (i < n) ? mask[i] : 0.f;
  float a = (i < B) ? y_feas[i] : 0.f;
  for (int o = 32; o >= 1; o >>= 1) {
    c += __shfl_xor(c, o);
    a += __shfl_xor(a, o);
  }
  if ((threadIdx.x & 63) == 0) {
    if (c != 0.f) atomicAdd(&cnt[1], c);
    if (a != 0.f) atomicAdd(&cnt[0], a);
  }
}

__global__ void k_loss_grad(int B, int O, int Wn, const float* Y, const float* y_feas, const float* y_cost,
                            const float* y_traj, const float* mask, const float* cnt, float* dY, bf16* dYb,
                            float* loss_terms) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (long)B * O) return;
  const int b = (int)(i / O), o = (int)(i % O);
  const float nf = fmaxf(cnt[0], 1.f), nm = fmaxf(cnt[1], 1.f);
  float g = 0.f, l = 0.f;
  int term = -1;
  if (o == 0) {
    const float x = Y[i], yv = y_feas[b];
    l = fmaxf(x, 0.f) - x * yv + log1pf(expf(-fabsf(x)));
    g = (1.f / (1.f + expf(-x)) - yv) / (float)B;
    l /= (float)B;
    term = 0;
  } else if (o == 1) {
    const float f = y_feas[b], d = Y[i] - y_cost[b];
    l = f * d * d / nf;
    g = 2.f * f * d / nf;
    term = 1;
  } else if (o - 2 < Wn) {
    const long e = (long)b * Wn + (o - 2);
    const float m = mask[e], d = Y[i] - y_traj[e];
    l = m * d * d / nm;
    g = 2.f * m * d / nm;
    term = 2;
  }
  dY[i] = g;
  dYb[i] = to_bf16(g);
  if (term >= 0 && l != 0.f) atomicAdd(&loss_terms[term], l);
}

__global__ void k_adamw(float* w, float* m, float* v, const float* g, long n, float lr, float b1, float b2, float eps,
                        float wd, float bc1, float bc2) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float gi = g[i];
  const float mi = b1 * m[i] + (1.f - b1) * gi;
  const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  const float mh = mi / bc1, vh = vi / bc2;
  w[i] -= lr * (mh / (sqrtf(vh) + eps) + wd * w[i]);
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
__global__ void k_targets(long B, const float* traj, int nmax, const int32_t* nseg, const int32_t* knots, int smax,
                          const uint8_t* feas, const float* cost, float* y_feas, float* y_cost, float* y_traj,
                          float* mask) {
  const long b = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= B) return;
  const int K = nseg[b];
  const float f = feas[b] ? 1.f : 0.f;
  y_feas[b] = f;
  y_cost[b] = feas[b] ? log1pf(fmaxf(cost[b], 0.f)) : 0.f;
  const float* T = traj + b * (long)(nmax + 1) * 7;
  int k0 = 0;
  for (int j = 0; j < 6; ++j) {
    const bool live = j < K && j < smax;
    const int nj = live ? knots[b * smax + j] : 0;
    for (int i = 0; i < WS_SLOTS; ++i) {
      const float p = (float)i / (WS_SLOTS - 1) * (float)nj;
      const int k = min((int)floorf(p), max(nj - 1, 0));
      const float fr = p - (float)k;
      for (int c = 0; c < WS_CH; ++c) {
        const long e = b * (6L * WS_SLOTS * WS_CH) + ((long)j * WS_SLOTS + i) * WS_CH + c;
        float val = 0.f;
        if (live && c < 7) {
          const float a0 = T[(k0 + k) * 7 + c], a1 = T[(k0 + min(k + 1, nj)) * 7 + c];
          val = a0 + fr * (a1 - a0);
        }
        y_traj[e] = val;
        mask[e] = (live && c < 7) ? f : 0.f;
      }
    }
    k0 += nj;
  }
}

__global__ void k_decode_warm(long B, const long long* B_dev, const float* Y, int O, const float* x0, int inst_stride,
                              const int32_t* nseg, const int32_t* knots, int smax, int nmax, float* warm) {
  const long Bn = B_dev ? *B_dev : B;
  const long b = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= Bn) return;
  const int K = nseg[b];
  const float* y = Y + b * (long)O + 2;
  float* Wr = warm + b * (long)(nmax + 1) * 7;
  for (int r = 0; r < (nmax + 1) * 7; ++r) Wr[r] = 0.f;
  int k0 = 0;
  for (int j = 0; j < K && j < smax; ++j) {
    const int nj = knots[b * smax + j];
    for (int k = 0; k <= nj && k0 + k <= nmax; ++k) {
      const float p = (nj > 0) ? (float)k / (float)nj * (WS_SLOTS - 1) : 0.f;
      const int i = min((int)floorf(p), WS_SLOTS - 2);
      const float fr = p - (float)i;
      for (int c = 0; c < 7; ++c) {
        const float a0 = y[((long)j * WS_SLOTS + i) * WS_CH + c], a1 = y[((long)j * WS_SLOTS + i + 1) * WS_CH + c];
        Wr[(k0 + k) * 7 + c] = a0 + fr * (a1 - a0);
      }
    }
    k0 += nj;
  }
  for (int c = 0; c < 4; ++c) Wr[c] = x0[b * inst_stride * 4 + c];
  if (k0 <= nmax)
    for (int c = 4; c < 7; ++c) Wr[k0 * 7 + c] = 0.f;
}

}  // namespace comet

// ==================================================================================
// Host side
// ==================================================================================
using namespace comet;

struct comet_mlp {
  int in_dim, hidden, layers, out_dim;
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
  float *dZ = nullptr;                 // FP32 gradient buffer [B][hidden]
  bf16 *dZb[2] = {nullptr, nullptr};   // BF16 gradient ping-pong [B][max(hidden, out)]
  float *cnt = nullptr, *lossd = nullptr;
  long long step = 0;
};

namespace {

unsigned nblk(long long n, int bs) { return (unsigned)std::max<long long>(1, (n + bs - 1) / bs); }

template <bool A_K, bool B_K, int EPI>
void gemm(hipStream_t s, int M, int N, int K, const bf16* A, long am, long ak, const bf16* Bp, long bn, long bk,
          const Epi& ep, const long long* M_dev = nullptr) {
  dim3 grid(nblk(N, GBN), nblk(M, GBM));
  hipLaunchKernelGGL((k_gemm<A_K, B_K, EPI>), grid, dim3(256), 0, s, M, N, K, A, am, ak, Bp, bn, bk, ep, M_dev);
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

// forward for B rows of m->H[0] (at most *B_dev rows if given); Y filled.
void mlp_forward(comet_mlp* m, hipStream_t s, int B, const long long* B_dev) {
  for (int l = 0; l < m->nl; ++l) {
    const int K = m->K[l], N = m->N[l];
    Epi ep{};
    ep.bias = m->P + m->boff[l];
    ep.ldc = N;
    const bf16* Wl = m->Wb + m->wboff[l];
    if (l < m->nl - 1) {
      ep.z = m->Z[l];
      ep.h = m->H[l + 1];
      gemm<true, true, EPI_HIDDEN>(s, B, N, K, m->H[l], K, 1, Wl, K, 1, ep, B_dev);
    } else {
      ep.z = m->Y;
      gemm<true, true, EPI_OUT>(s, B, N, K, m->H[l], K, 1, Wl, K, 1, ep, B_dev);
    }
  }
}

// hooks for the expansion graph (sizes on the device)
int mlp_in_dim(const comet_mlp* m) { return m->in_dim; }
int mlp_out_dim(const comet_mlp* m) { return m->out_dim; }
long long mlp_max_batch(const comet_mlp* m) { return m->max_batch; }
const float* mlp_output(const comet_mlp* m) { return m->Y; }

void mlp_encode_dev(comet_mlp* m, hipStream_t s, long long Bmax, const long long* B_dev, const float* x0,
                    const float* goal, const float* inst, int inst_stride, const int32_t* nseg, const int32_t* modes,
                    const int32_t* knots, int smax) {
  hipLaunchKernelGGL(k_encode_push, dim3(nblk(Bmax * m->in_dim, 256)), dim3(256), 0, s, (long)Bmax, x0, goal, inst,
                     inst_stride, nseg, modes, knots, smax, m->in_dim, m->H[0], B_dev);
}

void mlp_decode_warm_dev(comet_mlp* m, hipStream_t s, long long Bmax, const long long* B_dev, const float* x0,
                         int inst_stride, const int32_t* nseg, const int32_t* knots, int smax, int nmax, float* warm) {
  hipLaunchKernelGGL(k_decode_warm, dim3(nblk(Bmax, 128)), dim3(128), 0, s, (long)Bmax, B_dev, m->Y, m->out_dim, x0,
                     inst_stride, nseg, knots, smax, nmax, warm);
}

}  // namespace comet

extern "C" {

comet_status comet_mlp_create(int32_t in_dim, int32_t hidden, int32_t layers, int32_t out_dim, int64_t max_batch,
                              uint64_t seed, comet_mlp** out) {
  if (!out || in_dim < 1 || hidden < 1 || layers < 1 || layers > 16 || out_dim < 2 + 6 * WS_SLOTS * WS_CH ||
      max_batch < 1)
    return COMET_EINVAL;
  *out = nullptr;
  comet_mlp* m = new comet_mlp();
  m->in_dim = in_dim;
  m->hidden = hidden;
  m->layers = layers;
  m->out_dim = out_dim;
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
  A((void**)&m->dZ, 4 * B * hidden);
  A((void**)&m->dZb[0], 2 * B * std::max(hidden, out_dim));
  A((void**)&m->dZb[1], 2 * B * std::max(hidden, out_dim));
  A((void**)&m->cnt, 4 * 4);
  A((void**)&m->lossd, 4 * 4);
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
  std::vector<void*> ps = {m->P, m->G, m->Mm, m->Vv, m->Wb, m->WT, m->Y, m->dY, m->dYb, m->dZ, m->dZb[0], m->dZb[1],
                           m->cnt, m->lossd};
  for (auto* h : m->H) ps.push_back(h);
  for (auto* z : m->Z) ps.push_back(z);
  for (void* p : ps)
    if (p) (void)hipFree(p);
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
  if (!m || !x_bf16 || !out) return COMET_EINVAL;
  if (B < 0 || B > m->max_batch) return COMET_EINVAL;
  if (B == 0) return COMET_OK;
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
  if (B < 1 || B > m->max_batch || !(lr >= 0.f)) return COMET_EINVAL;
  hipStream_t s = (hipStream_t)stream;
  const int Bi = (int)B, O = m->out_dim, Wn = 6 * WS_SLOTS * WS_CH;
  if (hipMemcpyAsync(m->H[0], x_bf16, 2 * B * m->in_dim, hipMemcpyDeviceToDevice, s) != hipSuccess) return COMET_EHIP;
  mlp_forward(m, s, Bi, nullptr);
  hipLaunchKernelGGL(k_zero, dim3(1), dim3(64), 0, s, m->lossd, 4L);
  hipLaunchKernelGGL(k_zero, dim3(1), dim3(64), 0, s, m->cnt, 4L);
  hipLaunchKernelGGL(k_loss_counts, dim3(nblk((long long)B * Wn, 256)), dim3(256), 0, s, Bi, Wn, y_feas, traj_mask,
                     m->cnt);
  hipLaunchKernelGGL(k_loss_grad, dim3(nblk((long long)B * O, 256)), dim3(256), 0, s, Bi, O, Wn, m->Y, y_feas, y_cost,
                     y_traj, traj_mask, m->cnt, m->dY, m->dYb, m->lossd);
  // backward through the linear layers
  const bf16* g = m->dYb;
  const float* g32 = m->dY;
  int cur = 0;
  for (int l = m->nl - 1; l >= 0; --l) {
    const int K = m->K[l], N = m->N[l];
    // dW_l [N][K] = G^T [N][B] . H_l [B][K]   (contraction over the batch)
    Epi ew{};
    ew.z = m->G + m->woff[l];
    ew.ldc = K;
    gemm<false, false, EPI_PLAIN>(s, N, K, Bi, g, 1, N, m->H[l], 1, K, ew);
    hipLaunchKernelGGL(k_colsum, dim3(nblk(N, 256)), dim3(256), 0, s, g32, Bi, N, m->G + m->boff[l]);
    if (l > 0) {
      // dZ_{l-1} [B][K] = (G [B][N] . W_l [N][K]) * gelu'(Z_{l-1})
      Epi ex{};
      ex.z = m->dZ;
      ex.h = m->dZb[cur];
      ex.zprev = m->Z[l - 1];
      ex.ldc = K;
      gemm<true, false, EPI_DX>(s, Bi, K, N, g, N, 1, m->Wb + m->wboff[l], 1, K, ex);
      g = m->dZb[cur];
      g32 = m->dZ;
      cur ^= 1;
    }
  }
  // AdamW on the FP32 masters, then refresh the BF16 copies
  m->step += 1;
  const float b1 = 0.9f, b2 = 0.999f;
  const float bc1 = 1.f - std::pow(b1, (float)m->step), bc2 = 1.f - std::pow(b2, (float)m->step);
  hipLaunchKernelGGL(k_adamw, dim3(nblk(m->n_params, 256)), dim3(256), 0, s, m->P, m->Mm, m->Vv, m->G,
                     (long)m->n_params, lr, b1, b2, 1e-8f, weight_decay, bc1, bc2);
  refresh_weights(m, s);
  if (loss && hipMemcpyAsync(loss, m->lossd, 4 * 3, hipMemcpyDeviceToDevice, s) != hipSuccess) return COMET_EHIP;
  return hipGetLastError() == hipSuccess ? COMET_OK : COMET_EHIP;
}

comet_status comet_mlp_encode(comet_task task, void* stream, int64_t B, const float* x0, const float* goal,
                              const float* inst, const int32_t* nseg, const int32_t* modes, const int32_t* knots,
                              int32_t smax, int32_t in_dim, uint16_t* x_bf16) {
  if (task != COMET_TASK_PUSH || !x0 || !goal || !inst || !nseg || !modes || !knots || !x_bf16) return COMET_EINVAL;
  if (B < 0 || smax < 1 || smax > 6 || in_dim < POSE_DIMS + 6 * SEG_SLOT) return COMET_EINVAL;
  if (B == 0) return COMET_OK;
  hipLaunchKernelGGL(k_encode_push, dim3(nblk(B * in_dim, 256)), dim3(256), 0, (hipStream_t)stream, (long)B, x0, goal,
                     inst, 1, nseg, modes, knots, smax, in_dim, (bf16*)x_bf16, (const long long*)nullptr);
  return hipGetLastError() == hipSuccess ? COMET_OK : COMET_EHIP;
}

comet_status comet_mlp_targets(void* stream, int64_t B, const float* traj, int32_t nmax, const int32_t* nseg,
                               const int32_t* knots, int32_t smax, const uint8_t* feasible, const float* cost,
                               float* y_feas, float* y_cost, float* y_traj, float* traj_mask) {
  if (!traj || !nseg || !knots || !feasible || !cost || !y_feas || !y_cost || !y_traj || !traj_mask) return COMET_EINVAL;
  if (B < 0 || smax < 1 || smax > 6 || nmax < 1) return COMET_EINVAL;
  if (B == 0) return COMET_OK;
  hipLaunchKernelGGL(k_targets, dim3(nblk(B, 128)), dim3(128), 0, (hipStream_t)stream, (long)B, traj, nmax, nseg,
                     knots, smax, feasible, cost, y_feas, y_cost, y_traj, traj_mask);
  return hipGetLastError() == hipSuccess ? COMET_OK : COMET_EHIP;
}

comet_status comet_mlp_decode_warm(void* stream, int64_t B, const float* out, int32_t out_dim, const float* x0,
                                   const int32_t* nseg, const int32_t* knots, int32_t smax, int32_t nmax, float* warm) {
  if (!out || !x0 || !nseg || !knots || !warm || out_dim < 2 + 6 * WS_SLOTS * WS_CH) return COMET_EINVAL;
  if (B < 0 || smax < 1 || smax > 6 || nmax < 1) return COMET_EINVAL;
  if (B == 0) return COMET_OK;
  hipLaunchKernelGGL(k_decode_warm, dim3(nblk(B, 128)), dim3(128), 0, (hipStream_t)stream, (long)B,
                     (const long long*)nullptr, out, out_dim, x0, 1, nseg, knots, smax, nmax, warm);
  return hipGetLastError() == hipSuccess ? COMET_OK : COMET_EHIP;
}

}  // extern "C"
