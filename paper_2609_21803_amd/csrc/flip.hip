// flip.hip -- batched mode-conditioned TO evaluator for bimanual flipping of a box in a
// vertical plane (the bimanual task of Sec. IV-B: quasi-static wrench balance with the table
// reaction eliminated, fingers on faces with Coulomb cones, support transitions by
// pivoting), solved with the augmented-Lagrangian / Gauss-Newton scheme of Sec. III-C.
//
// Mapping: one candidate order per 64-lane wavefront (one block).  With 17 stage unknowns
// (u_k, x_{k+1}) the per-stage algebra (32 x 25 row Jacobian, 25 x 25 Gauss-Newton block,
// 17 x 17 factorisation with 9 right-hand sides) is too large for one lane's registers, so
// it is spread over the lanes: lanes over rows for the linearisation (Jacobian rows staged
// in LDS), the Gauss-Newton block assembled on the FP64 matrix cores, lane i holding row i
// of the bordered block in registers for the elimination and the back substitution (pivot
// row broadcast by readlane), lanes over intervals for the trial steps and the
// feasibility, multiplier and scoring passes.  All arithmetic is
// FP64: the blocks carry 1/mu-scaled rank-deficient terms as in the pushing task.
//
// Task model (state, controls, rows, units): see include/comet.h, COMET_TASK_FLIP.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>

#include "internal.h"

namespace comet {
namespace flip {

constexpr int NX = 8, NU = 9, NW = 17, NV = 25, NE = 17, NI = 15, NR = 32, NT = 5;
constexpr int NMODES = 845;
constexpr int ROW = NX + NU;   // trajectory row (x_k, u_k)
constexpr double BW = 0.2, BH = 0.1, MG = 0.5 * 9.81, MUF = 0.5, DT = 0.1;
constexpr double WA = 1e-2, WF = 1.0, WS = 1e-2;
constexpr double HALF_PI = 1.5707963267948966;
constexpr int MAX_TRIALS = 16;

// u indices inside the row arguments v = (x_k, u_k, x_{k+1})
constexpr int V_AX = 8, V_X1 = NX + NU;
__host__ __device__ constexpr int v_fn(int i) { return 11 + 3 * i; }
__host__ __device__ constexpr int v_ft(int i) { return 12 + 3 * i; }
__host__ __device__ constexpr int v_sd(int i) { return 13 + 3 * i; }

// face j: outward normal at angle j pi/2, counter-clockwise tangent, distance from the
// centre, half length
struct Face {
  double nx, ny, tx, ty, h, l;
};
__host__ __device__ inline Face face(int j) {
  Face f;
  f.nx = (j == 0) ? 1.0 : (j == 2) ? -1.0 : 0.0;
  f.ny = (j == 1) ? 1.0 : (j == 3) ? -1.0 : 0.0;
  f.tx = -f.ny;
  f.ty = f.nx;
  f.h = (j % 2 == 0) ? 0.5 * BW : 0.5 * BH;
  f.l = (j % 2 == 0) ? 0.5 * BH : 0.5 * BW;
  return f;
}

// per-interval contact parameters, packed: f1 | f2 << 4 | g << 8 | fs << 11 | land << 13 |
// (turns + 8) << 14, the support angle being turns * pi/2
__host__ __device__ inline int pack(int f1, int f2, int g, int fs, int land, int turns) {
  return f1 | (f2 << 4) | (g << 8) | (fs << 11) | (land << 13) | ((turns + 8) << 14);
}
struct Stage {
  int f[2], g, fs, land;
  double ths, mu_g;
};
__device__ inline Stage unpack(int p, double mu_g) {
  Stage s;
  s.f[0] = p & 15;
  s.f[1] = (p >> 4) & 15;
  s.g = (p >> 8) & 7;
  s.fs = (p >> 11) & 3;
  s.land = (p >> 13) & 1;
  s.ths = (double)(((p >> 14) & 15) - 8) * HALF_PI;
  s.mu_g = mu_g;
  return s;
}

// Quantities shared by the rows of one interval: body and world finger forces, moments
// about the centre, the table reaction and their derivatives.
struct Wrench {
  double c, s, c1, s1;               // cos / sin of th_k and th_{k+1}
  double Fbx[2], Fby[2];             // body-frame finger forces
  double tau[2];                     // moments about the centre
  double rx, ry;                     // table reaction (world)
  double drx_dth, dry_dth;
  double drx_dfn[2], dry_dfn[2], drx_dft[2], dry_dft[2];
  Face ff[2];
};

// with the sines and cosines of th_k (s, c) and th_{k+1} (s1, c1) given
__device__ __forceinline__ void wrench_sc(const Stage& S, const double* v, double s, double c, double s1, double c1,
                                          Wrench& w) {
  w.s = s;
  w.c = c;
  w.s1 = s1;
  w.c1 = c1;
  double Fwx = 0.0, Fwy = 0.0;
  for (int i = 0; i < 2; ++i) {
    w.Fbx[i] = w.Fby[i] = w.tau[i] = 0.0;
    w.drx_dfn[i] = w.dry_dfn[i] = w.drx_dft[i] = w.dry_dft[i] = 0.0;
    if (S.f[i] == 0) continue;
    const Face F = face((S.f[i] - 1) / 3);
    w.ff[i] = F;
    const double fn = v[v_fn(i)], ft = v[v_ft(i)], si = v[6 + i];
    w.Fbx[i] = -fn * F.nx + ft * F.tx;
    w.Fby[i] = -fn * F.ny + ft * F.ty;
    w.tau[i] = F.h * ft + si * fn;
    Fwx += w.c * w.Fbx[i] - w.s * w.Fby[i];
    Fwy += w.s * w.Fbx[i] + w.c * w.Fby[i];
    // r = -(sum of world forces) + (0, mg)
    w.drx_dfn[i] = w.c * F.nx - w.s * F.ny;
    w.dry_dfn[i] = w.s * F.nx + w.c * F.ny;
    w.drx_dft[i] = -(w.c * F.tx - w.s * F.ty);
    w.dry_dft[i] = -(w.s * F.tx + w.c * F.ty);
  }
  w.rx = -Fwx;
  w.ry = MG - Fwy;
  w.drx_dth = Fwy;
  w.dry_dth = -Fwx;
}

__device__ __forceinline__ void wrench(const Stage& S, const double* v, Wrench& w) {
  double s, c, s1, c1;
  sincos(v[2], &s, &c);
  sincos(v[V_X1 + 2], &s1, &c1);
  wrench_sc(S, v, s, c, s1, c1, w);
}

// gradient of the linear combination p rx + q ry of the table reaction into a[]
template <bool JAC>
__device__ inline void d_comb(const Wrench& w, double p, double q, double* a) {
  if (!JAC) return;
  a[2] += p * w.drx_dth + q * w.dry_dth;
  for (int i = 0; i < 2; ++i) {
    a[v_fn(i)] += p * w.drx_dfn[i] + q * w.dry_dfn[i];
    a[v_ft(i)] += p * w.drx_dft[i] + q * w.dry_dft[i];
  }
}

// Row r of interval k at v = (x_k, u_k, x_{k+1}); a[] (NV entries, zeroed by the caller)
// receives its gradient when JAC.  Slots: 0..7 defects; 8..11 finger equalities (two per
// finger); 12..16 table equalities; 17..26 finger inequalities (five per finger); 27..31
// table inequalities.
template <bool JAC>
__device__ __forceinline__ void row(const Stage& S, const Wrench& w, int r, const double* v, double& c, double* a,
                                    int& en) {
  c = 0.0;
  en = 0;
  if (r < 8) {
    // x_{k+1} = x_k + dt * rate: twist for the pose, accelerations for the twist, slip
    // rates for the face coordinates
    const int ri = (r < 3) ? r + 3 : (r < 6) ? r + 5 : (r == 6) ? 13 : 16;
    c = v[V_X1 + r] - (v[r] + DT * v[ri]);
    en = 1;
    if (JAC) {
      a[V_X1 + r] += 1.0;
      a[r] -= 1.0;
      a[ri] -= DT;
    }
    return;
  }
  if (r < 12) {   // finger equalities
    const int i = (r - 8) >> 1, e = (r - 8) & 1;
    const int code = S.f[i];
    if (code == 0) {
      const int idx = e ? v_ft(i) : v_fn(i);
      c = v[idx] / MG;
      en = 1;
      if (JAC) a[idx] += 1.0 / MG;
      return;
    }
    if (e) return;
    const int slip = (code - 1) % 3;
    if (slip == 0) {
      c = v[v_sd(i)];
      en = 1;
      if (JAC) a[v_sd(i)] += 1.0;
    } else {
      const double sg = (slip == 1) ? 1.0 : -1.0;
      c = (v[v_ft(i)] - sg * MUF * v[v_fn(i)]) / MG;
      en = 1;
      if (JAC) {
        a[v_ft(i)] += 1.0 / MG;
        a[v_fn(i)] -= sg * MUF / MG;
      }
    }
    return;
  }
  if (r >= 17 && r < 27) {   // finger inequalities
    const int i = (r - 17) / 5, q = (r - 17) % 5;
    const int code = S.f[i];
    if (code == 0) return;
    const int slip = (code - 1) % 3;
    const double fn = v[v_fn(i)], ft = v[v_ft(i)];
    if (q == 0) {
      c = -fn / MG;
      en = 1;
      if (JAC) a[v_fn(i)] -= 1.0 / MG;
    } else if (q == 1) {
      en = 1;
      if (slip == 0) {
        c = (ft - MUF * fn) / MG;
        if (JAC) {
          a[v_ft(i)] += 1.0 / MG;
          a[v_fn(i)] -= MUF / MG;
        }
      } else {
        const double sg = (slip == 1) ? 1.0 : -1.0;
        c = -sg * v[v_sd(i)];
        if (JAC) a[v_sd(i)] -= sg;
      }
    } else if (q == 2) {
      if (slip != 0) return;
      c = (-ft - MUF * fn) / MG;
      en = 1;
      if (JAC) {
        a[v_ft(i)] -= 1.0 / MG;
        a[v_fn(i)] -= MUF / MG;
      }
    } else {
      const double l = w.ff[i].l, sgn = (q == 3) ? 1.0 : -1.0;
      c = sgn * v[6 + i] - l;
      en = 1;
      if (JAC) a[6 + i] += sgn;
    }
    return;
  }
  // table rows
  const Face F = face(S.fs);
  const double mu = S.mu_g;
  if (r == 27) {
    c = -w.ry / MG;
    en = 1;
    d_comb<JAC>(w, 0.0, -1.0 / MG, a);
    return;
  }
  if (S.g <= 2) {   // supported on face fs
    switch (r) {
      case 12:
        if (!S.land) return;
        c = v[2] - S.ths;
        en = 1;
        if (JAC) a[2] += 1.0;
        return;
      case 13:
        c = v[5];
        en = 1;
        if (JAC) a[5] += 1.0;
        return;
      case 14:
        c = v[4];
        en = 1;
        if (JAC) a[4] += 1.0;
        return;
      case 15:
        en = 1;
        if (S.g == 0) {
          c = v[3];
          if (JAC) a[3] += 1.0;
        } else {
          const double sg = (S.g == 1) ? 1.0 : -1.0;
          c = (w.rx + sg * mu * w.ry) / MG;
          d_comb<JAC>(w, 1.0 / MG, sg * mu / MG, a);
        }
        return;
      case 28:
      case 29: {
        const double sg = (r == 28) ? 1.0 : -1.0;
        const double k = 1.0 / (MG * BW);
        c = (sg * (w.tau[0] + w.tau[1] + F.h * w.rx) - F.l * w.ry) * k;
        en = 1;
        if (JAC) {
          d_comb<JAC>(w, sg * F.h * k, -F.l * k, a);
          for (int i = 0; i < 2; ++i) {
            if (S.f[i] == 0) continue;
            a[v_ft(i)] += sg * w.ff[i].h * k;
            a[v_fn(i)] += sg * v[6 + i] * k;
            a[6 + i] += sg * v[v_fn(i)] * k;
          }
        }
        return;
      }
      case 30:
        en = 1;
        if (S.g == 0) {
          c = (w.rx - mu * w.ry) / MG;
          d_comb<JAC>(w, 1.0 / MG, -mu / MG, a);
        } else {
          const double sg = (S.g == 1) ? 1.0 : -1.0;
          c = -sg * v[3];
          if (JAC) a[3] -= sg;
        }
        return;
      case 31:
        if (S.g != 0) return;
        c = (-w.rx - mu * w.ry) / MG;
        en = 1;
        d_comb<JAC>(w, -1.0 / MG, -mu / MG, a);
        return;
      default:
        return;
    }
  }
  // pivot about the left (g = 3) or right (g = 4) corner of the support face
  const double dir = (S.g == 3) ? 1.0 : -1.0;
  const double cbx = F.h * F.nx - dir * F.l * F.tx, cby = F.h * F.ny - dir * F.l * F.ty;
  switch (r) {
    case 12:
      c = (v[V_X1] + w.c1 * cbx - w.s1 * cby) - (v[0] + w.c * cbx - w.s * cby);
      en = 1;
      if (JAC) {
        a[V_X1] += 1.0;
        a[V_X1 + 2] += -w.s1 * cbx - w.c1 * cby;
        a[0] -= 1.0;
        a[2] += w.s * cbx + w.c * cby;
      }
      return;
    case 13:
      c = v[V_X1 + 1] + w.s1 * cbx + w.c1 * cby;
      en = 1;
      if (JAC) {
        a[V_X1 + 1] += 1.0;
        a[V_X1 + 2] += w.c1 * cbx - w.s1 * cby;
      }
      return;
    case 14: {
      const double k = 1.0 / (MG * BW);
      double mom = MG * (w.c * cbx - w.s * cby);
      for (int i = 0; i < 2; ++i) mom += w.tau[i] - (cbx * w.Fby[i] - cby * w.Fbx[i]);
      c = mom * k;
      en = 1;
      if (JAC) {
        a[2] += MG * (-w.s * cbx - w.c * cby) * k;
        for (int i = 0; i < 2; ++i) {
          if (S.f[i] == 0) continue;
          const Face& G = w.ff[i];
          a[v_fn(i)] += (v[6 + i] + cbx * G.ny - cby * G.nx) * k;
          a[v_ft(i)] += (G.h - (cbx * G.ty - cby * G.tx)) * k;
          a[6 + i] += v[v_fn(i)] * k;
        }
      }
      return;
    }
    case 28:
      c = -dir * (v[V_X1 + 2] - S.ths);
      en = 1;
      if (JAC) a[V_X1 + 2] -= dir;
      return;
    case 29:
      c = dir * (v[V_X1 + 2] - S.ths) - HALF_PI;
      en = 1;
      if (JAC) a[V_X1 + 2] += dir;
      return;
    case 30:
      c = (w.rx - mu * w.ry) / MG;
      en = 1;
      d_comb<JAC>(w, 1.0 / MG, -mu / MG, a);
      return;
    case 31:
      c = (-w.rx - mu * w.ry) / MG;
      en = 1;
      d_comb<JAC>(w, -1.0 / MG, -mu / MG, a);
      return;
    default:
      return;
  }
}

__device__ inline double cost_weight(int i) {
  return (i < 3) ? WA : ((i == 5 || i == 8) ? WS : WF / (MG * MG));
}

// terminal rows: (px, th) at the goal, zero twist; row t depends on x_N[term_idx[t]]
__device__ inline int term_idx(int t) { return (t == 0) ? 0 : (t == 1) ? 2 : (t + 1); }

struct FlipArgs {
  int64_t B;
  const int64_t* Bdev;
  int64_t inst_stride;            // 1: per-order instance, 0: one instance for the batch
  unsigned long long* t_first;    // device timestamp of the first feasible solve (or null)
  int smax, nmax;
  const float *x0, *goal, *inst;
  const int32_t *nseg, *modes, *knots;
  const float* warm;
  float *cost, *viol;
  uint8_t* feas;
  float* traj;
  int32_t* stats;
  double *cost64, *viol64;
  double *z, *dz, *g, *lam, *nu, *kk, *KK;
  int* code;
  unsigned* err;
  DevParams prm;
};

struct Shm {
  double A[NR][NV + 1];
  double cr[NR], wr[NR], yr[NR];
  double M[NV + 1][NV + 2];   // bordered Gauss-Newton block, lower triangle (see sweep)
  double Pm[NX][NX + 1], pv[NX];
  double h[NV];
  double v[NV];           // row arguments of the interval being linearised
  double carry[NX];
  double dx[NX];
  double trial[MAX_TRIALS];
  double xk0[NX];
  double goal[2];
  double mu_g;
  int N, valid, fail;
};

// value of x in lane `src` (a compile-time or wave-uniform lane index), in every lane
__device__ __forceinline__ double bcast(double x, int src) {
  const unsigned long long u = (unsigned long long)__double_as_longlong(x);
  const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)u, src);
  const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(u >> 32), src);
  return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

// a value known to be the same in every lane, moved to scalar registers
__device__ __forceinline__ double uniform(double x) {
  const unsigned long long u = (unsigned long long)__double_as_longlong(x);
  const unsigned lo = (unsigned)__builtin_amdgcn_readfirstlane((int)(unsigned)u);
  const unsigned hi = (unsigned)__builtin_amdgcn_readfirstlane((int)(unsigned)(u >> 32));
  return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

// sum over the 64 lanes (result in every lane)
__device__ inline double wave_sum(double v) {
  for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o);
  return v;
}
__device__ inline double wave_max(double v) {
  for (int o = 32; o >= 1; o >>= 1) v = fmax(v, __shfl_xor(v, o));
  return v;
}

// row arguments v = (x_k, u_k, x_{k+1}) of interval k from z (+ alpha dz)
__device__ inline void load_args(const FlipArgs& A, const Shm& sh, int64_t b, int k, double alpha, double* v) {
  const double* z = A.z + (b * A.nmax) * NW;
  const double* dz = A.dz + (b * A.nmax) * NW;
  for (int i = 0; i < NX; ++i)
    v[i] = (k == 0) ? sh.xk0[i] : z[(k - 1) * NW + NU + i] + (alpha != 0.0 ? alpha * dz[(k - 1) * NW + NU + i] : 0.0);
  for (int i = 0; i < NW; ++i) v[NX + i] = z[k * NW + i] + (alpha != 0.0 ? alpha * dz[k * NW + i] : 0.0);
}

// merit contribution of interval k (cost + rows) at v, and of the terminal rows if k = N-1;
// (s0, c0), (s1, c1): sine and cosine of th_k and th_{k+1}
__device__ __forceinline__ double stage_merit(const FlipArgs& A, const Shm& sh, int64_t b, int k, const double* v,
                                              double s0, double c0, double s1, double c1, double mu,
                                              const double* lamT) {
  const Stage S = unpack(A.code[b * A.nmax + k], sh.mu_g);
  Wrench w;
  wrench_sc(S, v, s0, c0, s1, c1, w);
  double phi = 0.0;
  for (int i = 0; i < NU; ++i) phi += DT * cost_weight(i) * v[NX + i] * v[NX + i];
  const double* lam = A.lam + (b * A.nmax + k) * NE;
  const double* nu = A.nu + (b * A.nmax + k) * NI;
#pragma unroll
  for (int r = 0; r < NR; ++r) {
    double c;
    int en;
    row<false>(S, w, r, v, c, nullptr, en);
    if (!en) continue;
    if (r < NE) {
      phi += lam[r] * c + c * c / (2.0 * mu);
    } else {
      const double n = nu[r - NE];
      const double t = fmax(n + c / mu, 0.0);
      phi += 0.5 * mu * (t * t - n * n);
    }
  }
  if (k == sh.N - 1) {
    const double* xN = v + V_X1;
    for (int t = 0; t < NT; ++t) {
      const double c = xN[term_idx(t)] - ((t == 0) ? sh.goal[0] : (t == 1) ? sh.goal[1] : 0.0);
      phi += lamT[t] * c + c * c / (2.0 * mu);
    }
  }
  return phi;
}

typedef double f64x4 __attribute__((ext_vector_type(4)));

// Factorisation of one interval's bordered block, held in LDS as its lower triangle (see
// sweep), with one block row per lane: lane i < 26 mirrors row i into registers (entry (i, j)
// from (max, min)).  Symmetric elimination of the 17 w pivots: the pivot row p is broadcast
// from lane p by readlane and every lane below it updates its whole row,
// M[i][j] -= M[i][p] M[j][p] / d_p, so the mirrored rows stay exact transposes of each other
// (the product is commutative).  After the elimination, column p of the rows below p holds
// the unit lower factor times d_p, and columns 17..25 of rows 0..16 hold d_p (L^{-1} [Q_wx,
// q_w])[p]; the back substitution X[p] = (z_p - sum_{i>p} M[i][p] X[i]) / d_p runs from the
// last pivot, lane i solving its row for all nine right-hand sides and broadcasting them.
// Lane p < 17 then writes gain row p (k = -X[:, q_w], K = -X[:, Q_wx]); lanes 17..24 write
// the value function of x_k (trailing block and border).  Returns 1 if a pivot is not
// positive and finite (S not positive definite); gains and value function are then left as
// they were.
__device__ __forceinline__ int factor_rows(const FlipArgs& A, Shm& sh, int lane, int64_t b, int k) {
  constexpr int NB = NV + 1;
  const int li = lane < NB ? lane : 0;
  double m[NB];
#pragma unroll
  for (int j = 0; j < NB; ++j) m[j] = (j <= li) ? sh.M[li][j] : sh.M[j][li];
  double idv = 0.0;   // inverse of this lane's pivot
#pragma unroll
  for (int p = 0; p < NW; ++p) {
    const double d = bcast(m[p], p);
    if (!(d > 0.0) || !isfinite(d)) return 1;
    const double id = 1.0 / d;
    if (lane == p) idv = id;
    double mp[NB];
#pragma unroll
    for (int j = p + 1; j < NB; ++j) mp[j] = bcast(m[j], p);
    if (lane > p && lane < NB) {
      const double mi = m[p];
#pragma unroll
      for (int j = p + 1; j < NB; ++j) m[j] = m[j] - mi * mp[j] * id;
    }
  }
  double x[NX + 1];
#pragma unroll
  for (int c = 0; c <= NX; ++c) x[c] = m[NW + c];
#pragma unroll
  for (int i = NW - 1; i >= 0; --i) {
    if (lane == i) {
#pragma unroll
      for (int c = 0; c <= NX; ++c) x[c] = x[c] * idv;
    }
    double xi[NX + 1];
#pragma unroll
    for (int c = 0; c <= NX; ++c) xi[c] = bcast(x[c], i);
    if (lane < i) {
      const double mli = m[i];
#pragma unroll
      for (int c = 0; c <= NX; ++c) x[c] = x[c] - mli * xi[c];
    }
  }
  if (lane < NW) {
    double* kk = A.kk + (b * A.nmax + k) * NW;
    double* KK = A.KK + ((b * A.nmax + k) * NW + lane) * NX;
#pragma unroll
    for (int c = 0; c < NX; ++c) KK[c] = -x[c];
    kk[lane] = -x[NX];
  } else if (lane < NV) {
#pragma unroll
    for (int j = 0; j < NX; ++j) sh.Pm[lane - NW][j] = m[NW + j];
    sh.pv[lane - NW] = m[NV];
  }
  return 0;
}

// Backward sweep over the intervals.  Always computes the merit phi and the gradient g of
// phi (stored per interval in A.g); with `factor`, also the Riccati recursion with damping
// rho, storing the gains.  Returns 1 if every factorisation succeeded (or factor is false).
//
// Factorisation of one interval.  The Gauss-Newton block over (w_k, x_k), w_k = (u_k,
// x_{k+1}), is bordered by the gradient q and held in LDS as the lower triangle of the
// order-26 matrix  [[S, Q_wx, q_w], [Q_xw, Q_xx, q_x], [q_w', q_x', .]]  in the variable
// order (u_k, x_{k+1}, x_k, 1).  Its row part sum_r w_r a_r a_r' (and the row gradient
// sum_r y_r a_r in the border row) is one dense 26 x 32 x 26 product on the FP64 matrix
// cores.  Symmetric elimination of the 17 w pivots (factor_rows: one block row per lane)
// leaves, by the Schur complement, the value function (P, p) of x_k in the trailing block
// and L^{-1} [Q_wx, q_w] (scaled by the pivots) in the eliminated columns; a back
// substitution over the pivot rows then gives the gains.  The pivots are the squares of
// the Cholesky diagonal of S, so a non-positive pivot is the positive-definiteness
// failure.
__device__ __forceinline__ int sweep(const FlipArgs& A, Shm& sh, int64_t b, bool factor, double mu,
                                     double rho, const double* lamT, double& phi_out, double& gnorm_out) {
  const int lane = threadIdx.x, N = sh.N;
  const double imu = 1.0 / mu;
  double phi_acc = 0.0, gmax = 0.0;
  int ok = 1;
  // terminal value function V_N and the terminal part of the gradient
  {
    const double* z = A.z + (b * A.nmax) * NW;
    const double* xN = z + (N - 1) * NW + NU;
    if (lane < NX) {
      sh.pv[lane] = 0.0;
      sh.carry[lane] = 0.0;
      for (int j = 0; j < NX; ++j) sh.Pm[lane][j] = 0.0;
    }
    __syncthreads();
    if (lane == 0) {
      for (int t = 0; t < NT; ++t) {
        const int j = term_idx(t);
        const double c = xN[j] - ((t == 0) ? sh.goal[0] : (t == 1) ? sh.goal[1] : 0.0);
        const double y = lamT[t] + c * imu;
        sh.pv[j] += y;
        sh.carry[j] += y;
        sh.Pm[j][j] += imu;
        phi_acc += lamT[t] * c + c * c / (2.0 * mu);
      }
    }
    __syncthreads();
  }
  // interval k's row arguments (lanes < 25), row multiplier (lanes < 32) and contact code
  // are loaded one interval ahead, so their memory latency overlaps the previous interval
  const double* zb = A.z + (b * A.nmax) * NW;
  double v_pre = 0.0, m_pre = 0.0;
  int code_pre = 0;
  auto prefetch = [&](int k) {
    if (lane < NV) v_pre = (lane < NX) ? ((k == 0) ? sh.xk0[lane] : zb[(k - 1) * NW + NU + lane]) : zb[k * NW + lane - NX];
    if (lane < NE)
      m_pre = A.lam[(b * A.nmax + k) * NE + lane];
    else if (lane < NR)
      m_pre = A.nu[(b * A.nmax + k) * NI + lane - NE];
    code_pre = A.code[b * A.nmax + k];
  };
  prefetch(N - 1);
  // sine and cosine of th_{k+1}, carried from interval k+1 (where it was th_k)
  double sn1, cs1;
  sincos(zb[(N - 1) * NW + NU + 2], &sn1, &cs1);
  for (int k = N - 1; k >= 0; --k) {
    const Stage S = unpack(code_pre, sh.mu_g);
    if (lane < NV) sh.v[lane] = v_pre;
    const double m_row = m_pre;
    if (k > 0) prefetch(k - 1);
    if (lane < NR)
      for (int j = 0; j < NV; ++j) sh.A[lane][j] = 0.0;
    __syncthreads();
    const double* v = sh.v;
    // rows: lane r evaluates row r and writes its gradient into A[r]
    double sn0, cs0;
    sincos(v[2], &sn0, &cs0);
    if (lane < NR) {
      Wrench w;
      wrench_sc(S, v, sn0, cs0, sn1, cs1, w);
      double c;
      int en;
      row<true>(S, w, lane, v, c, sh.A[lane], en);
      double y = 0.0, wt = 0.0;
      if (en) {
        if (lane < NE) {
          const double l = m_row;
          y = l + c * imu;
          wt = imu;
          phi_acc += l * c + c * c / (2.0 * mu);
        } else {
          const double n = m_row;
          const double t = n + c * imu;
          y = (t > 0.0) ? t : 0.0;
          wt = (t > 0.0) ? imu : 0.0;
          phi_acc += 0.5 * mu * (y * y - n * n);
        }
      }
      sh.cr[lane] = c;
      sh.yr[lane] = y;
      sh.wr[lane] = wt;
    } else if (lane < NR + NU) {
      const int i = lane - NR;
      const double u = v[NX + i];
      phi_acc += DT * cost_weight(i) * u * u;
    }
    __syncthreads();
    const bool fac = factor && ok;   // the same in every lane
    if (fac) {
      // row part of the block on the matrix cores: tile (I, J) of D = (W A)' A, rows of
      // tile-row 1 include the border row y' A (index NV)
      const int c16 = lane & 15, kq = lane >> 4;
      const int n1 = 16 + c16;
      const int v0 = NX + c16;                                  // variable of block index c16
      const int v1 = (n1 < NW) ? NX + n1 : n1 - NW;             // of block index n1 (if < NV)
      f64x4 d00 = {0.0, 0.0, 0.0, 0.0}, d10 = {0.0, 0.0, 0.0, 0.0}, d11 = {0.0, 0.0, 0.0, 0.0};
#pragma unroll 2
      for (int s4 = 0; s4 < NR / 4; ++s4) {
        const int r = 4 * s4 + kq;
        const double wr = sh.wr[r];
        const double b0 = sh.A[r][v0];
        const double b1 = (n1 < NV) ? sh.A[r][v1] : 0.0;
        const double a1 = (n1 < NV) ? wr * b1 : ((n1 == NV) ? sh.yr[r] : 0.0);
        d00 = __builtin_amdgcn_mfma_f64_16x16x4f64(wr * b0, b0, d00, 0, 0, 0);
        d10 = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b0, d10, 0, 0, 0);
        d11 = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b1, d11, 0, 0, 0);
      }
      // register q of lane l holds entry (l / 16 + 4 q, l % 16) of a tile
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int i = kq + 4 * q;
        sh.M[i][c16] = d00[q];
        if (16 + i <= NV) {
          sh.M[16 + i][c16] = d10[q];
          if (n1 <= NV) sh.M[16 + i][n1] = d11[q];
        }
      }
      __syncthreads();
    }
    // stage gradient h (no value function) and the gradient of phi for w_k
    if (lane < NV) {
      double s = 0.0;
      if (fac) {
        s = sh.M[NV][(lane < NX) ? NW + lane : lane - NX];
      } else {
        for (int r = 0; r < NR; ++r) {
          const double y = uniform(sh.yr[r]);   // same for every lane: a scalar branch skips zero rows
          if (y != 0.0) s += y * sh.A[r][lane];
        }
      }
      if (lane >= NX && lane < NX + NU) s += 2.0 * DT * cost_weight(lane - NX) * v[lane];
      sh.h[lane] = s;
    }
    __syncthreads();
    if (lane < NW) {
      const double gw = sh.h[NX + lane] + ((lane >= NU) ? sh.carry[lane - NU] : 0.0);
      A.g[(b * A.nmax + k) * NW + lane] = gw;
      gmax = fmax(gmax, fabs(gw));
    }
    __syncthreads();
    if (lane < NX) sh.carry[lane] = sh.h[lane];   // x_k part goes to the previous interval's w
    sn1 = sn0;
    cs1 = cs0;
    if (fac) {
      // cost Hessian and damping on the w diagonal, value function of x_{k+1} (P into the
      // x_{k+1} block, p into the border), border = stage gradient q
      if (lane < NW) {
        double dg = rho;
        if (lane < NU) dg += 2.0 * DT * cost_weight(lane);
        else dg += sh.Pm[lane - NU][lane - NU];
        sh.M[lane][lane] += dg;
        sh.M[NV][lane] = sh.h[NX + lane] + ((lane >= NU) ? sh.pv[lane - NU] : 0.0);
      } else if (lane < NV) {
        sh.M[NV][lane] = sh.h[lane - NW];
      }
      {
        const int i = lane / NX, j = lane % NX;
        if (j < i) sh.M[NU + i][NU + j] += sh.Pm[i][j];
      }
      __syncthreads();
      if (factor_rows(A, sh, lane, b, k)) ok = 0;
    }
    __syncthreads();
  }
  phi_out = wave_sum(phi_acc);
  gnorm_out = wave_max(gmax);
  return ok;
}

// forward pass: dw_k = k_k + K_k dx_k, dx_0 = 0
__device__ __forceinline__ void forward(const FlipArgs& A, Shm& sh, int64_t b) {
  const int lane = threadIdx.x;
  if (lane < NX) sh.dx[lane] = 0.0;
  __syncthreads();
  for (int k = 0; k < sh.N; ++k) {
    double d = 0.0;
    if (lane < NW) {
      d = A.kk[(b * A.nmax + k) * NW + lane];
      const double* K = A.KK + ((b * A.nmax + k) * NW + lane) * NX;
      for (int j = 0; j < NX; ++j) d += K[j] * sh.dx[j];
      A.dz[(b * A.nmax + k) * NW + lane] = d;
    }
    __syncthreads();
    if (lane >= NU && lane < NW) sh.dx[lane - NU] = d;
    __syncthreads();
  }
}

// lanes over intervals, one trial step after the other: phi(z + alpha_t dz) for t < T.
// Each lane takes the sine and cosine of its th_{k+1}; those of th_k come from the lane
// below (th_0 does not move: dx_0 = 0), or across a 64-interval chunk boundary from lane 63.
__device__ __forceinline__ void trials(const FlipArgs& A, Shm& sh, int64_t b, int T, double mu, const double* lamT) {
  const int lane = threadIdx.x, N = sh.N;
  double sx0, cx0;
  sincos(sh.xk0[2], &sx0, &cx0);
  for (int t = 0; t < T; ++t) {
    const double alpha = ldexp(1.0, -t);
    double acc = 0.0, sp = sx0, cp = cx0;
    for (int k0 = 0; k0 < N; k0 += 64) {
      const int k = k0 + lane;
      const bool on = k < N;
      double v[NV];
      double s1 = 0.0, c1 = 1.0;
      if (on) {
        load_args(A, sh, b, k, alpha, v);
        sincos(v[V_X1 + 2], &s1, &c1);
      }
      double s0 = __shfl_up(s1, 1), c0 = __shfl_up(c1, 1);
      if (lane == 0) {
        s0 = sp;
        c0 = cp;
      }
      sp = bcast(s1, 63);
      cp = bcast(c1, 63);
      if (on) acc += stage_merit(A, sh, b, k, v, s0, c0, s1, c1, mu, lamT);
    }
    const double s = wave_sum(acc);
    if (lane == 0) sh.trial[t] = s;
  }
  __syncthreads();
}

// lanes over intervals: scaled feasibility and complementarity at z; optionally the
// multiplier update lam += c/mu, nu = [nu + c/mu]_+
__device__ __forceinline__ void viol_pass(const FlipArgs& A, Shm& sh, int64_t b, double mu, bool update, double* lamT, double& vs,
                          double& rc) {
  const int lane = threadIdx.x, N = sh.N;
  double vmax = 0.0, qmax = 0.0;
  for (int k = lane; k < N; k += 64) {
    const Stage S = unpack(A.code[b * A.nmax + k], sh.mu_g);
    double v[NV];
    load_args(A, sh, b, k, 0.0, v);
    Wrench w;
    wrench(S, v, w);
    double* lam = A.lam + (b * A.nmax + k) * NE;
    double* nu = A.nu + (b * A.nmax + k) * NI;
#pragma unroll
    for (int r = 0; r < NR; ++r) {
      double c;
      int en;
      row<false>(S, w, r, v, c, nullptr, en);
      if (!en) continue;
      if (r < NE) {
        vmax = fmax(vmax, fabs(c));
        if (update) lam[r] += c / mu;
      } else {
        const double n = nu[r - NE];
        vmax = fmax(vmax, fmax(c, 0.0));
        qmax = fmax(qmax, fabs(fmin(-c, n)));
        if (update) nu[r - NE] = fmax(n + c / mu, 0.0);
      }
    }
  }
  vs = wave_max(vmax);
  rc = wave_max(qmax);
  // terminal rows (every lane computes them identically)
  const double* xN = A.z + (b * A.nmax + N - 1) * NW + NU;
  for (int t = 0; t < NT; ++t) {
    const double c = xN[term_idx(t)] - ((t == 0) ? sh.goal[0] : (t == 1) ? sh.goal[1] : 0.0);
    vs = fmax(vs, fabs(c));
    if (update) lamT[t] += c / mu;
  }
  __syncthreads();
}

// Eq. (4): objective and violation of z in the task's units
__device__ __forceinline__ void score_pass(const FlipArgs& A, Shm& sh, int64_t b, double& J, double& vi) {
  const int lane = threadIdx.x, N = sh.N;
  double jacc = 0.0, vmax = 0.0;
  for (int k = lane; k < N; k += 64) {
    const Stage S = unpack(A.code[b * A.nmax + k], sh.mu_g);
    double v[NV];
    load_args(A, sh, b, k, 0.0, v);
    Wrench w;
    wrench(S, v, w);
    for (int i = 0; i < NU; ++i) jacc += DT * cost_weight(i) * v[NX + i] * v[NX + i];
#pragma unroll
    for (int r = 0; r < NR; ++r) {
      double c;
      int en;
      row<false>(S, w, r, v, c, nullptr, en);
      if (!en) continue;
      vmax = fmax(vmax, (r < NE) ? fabs(c) : fmax(c, 0.0));
    }
  }
  J = wave_sum(jacc);
  vi = wave_max(vmax);
  const double* xN = A.z + (b * A.nmax + N - 1) * NW + NU;
  for (int t = 0; t < NT; ++t) {
    const double c = xN[term_idx(t)] - ((t == 0) ? sh.goal[0] : (t == 1) ? sh.goal[1] : 0.0);
    vi = fmax(vi, fabs(c));
  }
}

// Kinematic initial guess (one lane): face-supported segments hold the pose (stick) or
// slide it 5 cm, a pivot run turns the box about its corner to the landing angle (or the
// goal angle if the order ends in it); twists and accelerations by finite differences;
// contact fingers press with mg/2, sliding ones on the cone edge.
__device__ __forceinline__ void initial_guess(const FlipArgs& A, const Shm& sh, int64_t b) {
  const int N = sh.N;
  double* z = A.z + (b * A.nmax) * NW;
  // pass 1: poses at knots 1..N into z's x_{k+1} slots (px, py, th)
  double px = sh.xk0[0], py = sh.xk0[1], th = sh.xk0[2];
  int k = 0;
  while (k < N) {
    const Stage S = unpack(A.code[b * A.nmax + k], sh.mu_g);
    int e = k;
    if (S.g <= 2) {
      const double d = (S.g == 0) ? 0.0 : ((S.g == 1) ? 0.05 : -0.05);
      while (e < N) {
        const Stage Se = unpack(A.code[b * A.nmax + e], sh.mu_g);
        if (Se.g != S.g || (e > k && Se.land)) break;
        ++e;
      }
      const Face F = face(S.fs);
      for (int s = k + 1; s <= e; ++s) {
        const double a = (double)(s - k) / (double)(e - k);
        z[(s - 1) * NW + NU + 0] = px + d * a;
        z[(s - 1) * NW + NU + 1] = F.h;
        z[(s - 1) * NW + NU + 2] = S.ths;
      }
      px += d;
      py = F.h;
      th = S.ths;
    } else {
      const double dir = (S.g == 3) ? 1.0 : -1.0;
      while (e < N && unpack(A.code[b * A.nmax + e], sh.mu_g).g == S.g) ++e;
      const Face F = face(S.fs);
      const double cbx = F.h * F.nx - dir * F.l * F.tx, cby = F.h * F.ny - dir * F.l * F.ty;
      const double cwx = px + cos(th) * cbx - sin(th) * cby;
      const double cwy = py + sin(th) * cbx + cos(th) * cby;
      double th_end;
      if (e < N) {
        th_end = S.ths + dir * HALF_PI;
      } else {
        const double lo = (dir > 0) ? S.ths : S.ths - HALF_PI;
        const double hi = (dir > 0) ? S.ths + HALF_PI : S.ths;
        th_end = fmin(fmax(sh.goal[1], lo), hi);
      }
      for (int s = k + 1; s <= e; ++s) {
        const double a = (double)(s - k) / (double)(e - k);
        const double ts = th + (th_end - th) * a;
        z[(s - 1) * NW + NU + 0] = cwx - (cos(ts) * cbx - sin(ts) * cby);
        z[(s - 1) * NW + NU + 1] = cwy - (sin(ts) * cbx + cos(ts) * cby);
        z[(s - 1) * NW + NU + 2] = ts;
      }
      px = z[(e - 1) * NW + NU + 0];
      py = z[(e - 1) * NW + NU + 1];
      th = z[(e - 1) * NW + NU + 2];
    }
    k = e;
  }
  // pass 2: twists at knots 1..N-1 by forward differences, zero at N
  for (int s = 1; s <= N; ++s)
    for (int i = 0; i < 3; ++i) {
      double vel = 0.0;
      if (s < N) {
        const double p1 = z[s * NW + NU + i], p0 = z[(s - 1) * NW + NU + i];
        vel = (p1 - p0) / DT;
      }
      z[(s - 1) * NW + NU + 3 + i] = vel;
    }
  // pass 3: controls
  for (int kk = 0; kk < N; ++kk) {
    const Stage S = unpack(A.code[b * A.nmax + kk], sh.mu_g);
    double* w = z + kk * NW;
    for (int i = 0; i < 3; ++i) {
      const double v0 = (kk == 0) ? sh.xk0[3 + i] : z[(kk - 1) * NW + NU + 3 + i];
      w[i] = (w[NU + 3 + i] - v0) / DT;
    }
    for (int f = 0; f < 2; ++f) {
      double fn = 0.0, ft = 0.0;
      if (S.f[f] != 0) {
        const int slip = (S.f[f] - 1) % 3;
        fn = 0.5 * MG;
        ft = (slip == 0) ? 0.0 : ((slip == 1) ? MUF * fn : -MUF * fn);
      }
      w[3 + 3 * f] = fn;
      w[4 + 3 * f] = ft;
      w[5 + 3 * f] = 0.0;
    }
    w[NU + 6] = sh.xk0[6];
    w[NU + 7] = sh.xk0[7];
  }
}

__global__ __launch_bounds__(64, 2) void k_flip_solve(FlipArgs A) {
  __shared__ Shm sh;
  const int lane = threadIdx.x;
  const int64_t b = blockIdx.x;
  const int64_t Bn = A.Bdev ? *A.Bdev : A.B;
  if (b >= Bn) return;
  const DevParams& prm = A.prm;
  // sequence set-up (one lane): contact parameters per interval with the support
  // bookkeeping of the pivots
  if (lane == 0) {
    int valid = 1, N = 0;
    const int K = A.nseg[b];
    if (K < 1 || K > A.smax) valid = 0;
    const int64_t bi = b * A.inst_stride;
    for (int i = 0; i < NX; ++i) {
      sh.xk0[i] = (double)A.x0[bi * NX + i];
      if (!isfinite(sh.xk0[i])) valid = 0;
    }
    sh.goal[0] = (double)A.goal[bi * 2 + 0];
    sh.goal[1] = (double)A.goal[bi * 2 + 1];
    sh.mu_g = (double)A.inst[bi];
    if (!isfinite(sh.goal[0]) || !isfinite(sh.goal[1]) || !(sh.mu_g > 0.0) || !isfinite(sh.mu_g)) valid = 0;
    int fs = 3, turns = 0, prev_g = -1;
    for (int j = 0; valid && j < K; ++j) {
      const int id = A.modes[b * A.smax + j], n = A.knots[b * A.smax + j];
      if (id < 0 || id >= NMODES || n < 1 || n > A.nmax - N) {   // room left, so no sum can wrap
        valid = 0;
        break;
      }
      const int g = id % 5, f2 = (id / 5) % 13, f1 = id / 65;
      if (g >= 3 && prev_g >= 3 && g != prev_g) {
        valid = 0;
        break;
      }
      if (g <= 2 && prev_g >= 3) {
        const int dir = (prev_g == 3) ? 1 : -1;
        fs = ((fs - dir) % 4 + 4) % 4;
        turns += dir;
      }
      for (int t = 0; t < n; ++t, ++N)
        A.code[b * A.nmax + N] = pack(f1, f2, g, fs, (t == 0 && g <= 2 && prev_g >= 3) ? 1 : 0, turns);
      prev_g = g;
    }
    if (turns < -8 || turns > 7) valid = 0;
    sh.valid = valid;
    sh.N = N;
  }
  __syncthreads();
  const int N = sh.N;
  if (!sh.valid) {
    if (lane == 0) {
      A.cost[b] = __builtin_nan("");
      A.viol[b] = __builtin_inff();
      A.feas[b] = 0;
      if (A.cost64) A.cost64[b] = __builtin_nan("");
      if (A.viol64) A.viol64[b] = __builtin_inf();
      if (A.stats)
        for (int i = 0; i < 4; ++i) A.stats[b * 4 + i] = (i == 3) ? 3 : 0;
      atomicAdd(A.err, 1u);
    }
    if (A.traj)
      for (int i = lane; i < (A.nmax + 1) * ROW; i += 64) A.traj[b * (int64_t)(A.nmax + 1) * ROW + i] = 0.f;
    return;
  }
  // primal start: warm start or the kinematic guess; multipliers zero
  double* z = A.z + (b * A.nmax) * NW;
  if (A.warm) {
    const float* W = A.warm + b * (int64_t)(A.nmax + 1) * ROW;
    for (int e = lane; e < N * NW; e += 64) {
      const int k = e / NW, i = e % NW;
      z[e] = (i < NU) ? (double)W[k * ROW + NX + i] : (double)W[(k + 1) * ROW + (i - NU)];
    }
  } else if (lane == 0) {
    initial_guess(A, sh, b);
  }
  for (int e = lane; e < N * NE; e += 64) A.lam[b * A.nmax * NE + e] = 0.0;
  for (int e = lane; e < N * NI; e += 64) A.nu[b * A.nmax * NI + e] = 0.0;
  __syncthreads();

  double mu = A.warm ? prm.mu0_warm : prm.mu0;
  double eta = pow(mu, 0.1), omega = mu, rho = prm.rho0;
  double lamT[NT] = {0, 0, 0, 0, 0};
  int al_iters = 0, gn_iters = 0, cfails = 0, status = 0;
  const int T = min(max(prm.ls_trials, 1), MAX_TRIALS);
  for (int al = 0; al < prm.al_max; ++al) {
    int rejects = 0;
    al_iters = al + 1;
    for (int it = 0; it < prm.gn_max; ++it) {
      double phi0, gnorm;
      int ok = sweep(A, sh, b, true, mu, rho, lamT, phi0, gnorm);
      if (gnorm <= omega) break;
      int tries = 0;
      while (!ok && tries < prm.chol_retries) {
        ++cfails;
        rho = fmax(10.0 * rho, 1e-8);
        ++tries;
        double p2, g2;
        ok = sweep(A, sh, b, true, mu, rho, lamT, p2, g2);
      }
      if (!ok) ++cfails;
      ++gn_iters;
      int best = -1;
      double alpha = 1.0;
      if (ok) {
        forward(A, sh, b);
        double ddp = 0.0;
        for (int e = lane; e < N * NW; e += 64) ddp += A.g[b * A.nmax * NW + e] * A.dz[b * A.nmax * NW + e];
        const double dd = wave_sum(ddp);
        if (dd < 0.0 && isfinite(phi0)) {
          trials(A, sh, b, T, mu, lamT);
          for (int t = 0; t < T; ++t) {
            const double ph = sh.trial[t];
            if (isfinite(ph) && ph <= phi0 + prm.armijo_c1 * alpha * dd) {
              best = t;
              break;
            }
            alpha *= 0.5;
          }
          if (best >= 0)
            for (int e = lane; e < N * NW; e += 64) z[e] += alpha * A.dz[b * A.nmax * NW + e];
          __syncthreads();
        }
      }
      if (best >= 0) {
        rho = fmax(rho / 3.0, prm.rho_min);
        rejects = 0;
      } else {
        rho = fmin(10.0 * rho, prm.rho_max);
        if (++rejects >= prm.max_rejects) break;
      }
    }
    // outer update at the final inner iterate
    double vs, rc, phi_u, gnorm;
    viol_pass(A, sh, b, mu, false, lamT, vs, rc);
    (void)sweep(A, sh, b, false, mu, rho, lamT, phi_u, gnorm);
    double zbad = 0.0;
    for (int e = lane; e < N * NW; e += 64) zbad = fmax(zbad, isfinite(z[e]) ? 0.0 : 1.0);
    zbad = wave_max(zbad);
    if (!isfinite(vs) || !isfinite(gnorm) || zbad > 0.0) {
      status = 2;
      break;
    }
    if (vs <= eta) {
      if (vs <= prm.eta_star && gnorm <= prm.omega_star && rc <= prm.rc_star) {
        status = 1;
        break;
      }
      double v2, r2;
      viol_pass(A, sh, b, mu, true, lamT, v2, r2);
      eta = fmax(eta * pow(mu, 0.9), prm.eta_star);
      omega = fmax(omega * mu, prm.omega_star);
    } else {
      mu = fmax(0.1 * mu, prm.mu_min);
      eta = fmax(pow(mu, 0.1), prm.eta_star);
      omega = fmax(mu, prm.omega_star);
    }
  }
  double J = __builtin_nan(""), vi = __builtin_inf();
  if (status != 2) score_pass(A, sh, b, J, vi);
  if (!isfinite(J) || !isfinite(vi)) {
    J = __builtin_nan("");
    vi = __builtin_inf();
    status = 2;
  }
  if (lane == 0) {
    A.cost[b] = (float)J;
    A.viol[b] = (float)vi;
    A.feas[b] = (vi <= prm.eps_feas) ? 1 : 0;
    if (A.t_first && vi <= prm.eps_feas) atomicMin(A.t_first, (unsigned long long)wall_clock64());
    if (A.cost64) A.cost64[b] = J;
    if (A.viol64) A.viol64[b] = vi;
    if (A.stats) {
      A.stats[b * 4 + 0] = al_iters;
      A.stats[b * 4 + 1] = gn_iters;
      A.stats[b * 4 + 2] = cfails;
      A.stats[b * 4 + 3] = status;
    }
  }
  if (A.traj) {
    float* Tr = A.traj + b * (int64_t)(A.nmax + 1) * ROW;
    for (int e = lane; e < (A.nmax + 1) * ROW; e += 64) {
      const int k = e / ROW, i = e % ROW;
      double val = 0.0;
      if (k <= N) {
        if (i < NX) val = (k == 0) ? sh.xk0[i] : z[(k - 1) * NW + NU + i];
        else if (k < N) val = z[k * NW + (i - NX)];
      }
      Tr[e] = (float)val;
    }
  }
}

}  // namespace flip

// per-sequence work space of the flip task: z, dz, g, kk (17 per interval), lam (17),
// nu (15), KK (136), all FP64; packed contact parameters (int)
size_t flip_ws_doubles_per_interval() {
  return (size_t)flip::NW * 4 + flip::NE + flip::NI + (size_t)flip::NW * flip::NX;
}

comet_status flip_create_ws(comet_ctx* c) {
  const size_t R = (size_t)c->max_batch * (size_t)c->max_intervals;
  if (hipMalloc(&c->fws, sizeof(double) * R * flip_ws_doubles_per_interval()) != hipSuccess ||
      hipMalloc(&c->fcode, sizeof(int) * R) != hipSuccess) {
    (void)hipGetLastError();
    return COMET_ENOMEM;
  }
  int nb = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, flip::k_flip_solve, 64, 0) != hipSuccess || nb < 1) nb = 1;
  c->occ_blocks_per_cu = nb;
  return COMET_OK;
}

void flip_destroy_ws(comet_ctx* c) {
  if (c->fws) (void)hipFree(c->fws);
  if (c->fcode) (void)hipFree(c->fcode);
  c->fws = nullptr;
  c->fcode = nullptr;
}

comet_status launch_flip(comet_ctx* c, hipStream_t s, const EvalLaunch& L) {
  flip::FlipArgs A;
  std::memset(&A, 0, sizeof A);
  A.B = L.B;
  A.Bdev = L.B_dev;
  A.smax = c->max_segments;
  A.nmax = c->max_intervals;
  A.x0 = L.x0; A.goal = L.goal; A.inst = L.inst; A.inst_stride = L.inst_stride;
  A.t_first = L.t_first;
  A.nseg = L.nseg; A.modes = L.modes; A.knots = L.knots; A.warm = L.warm;
  A.cost = L.cost; A.viol = L.viol; A.feas = L.feas; A.traj = L.traj; A.stats = L.stats;
  A.cost64 = L.cost64; A.viol64 = L.viol64;
  const size_t R = (size_t)c->max_batch * (size_t)c->max_intervals;
  double* p = c->fws;
  A.z = p; p += R * flip::NW;
  A.dz = p; p += R * flip::NW;
  A.g = p; p += R * flip::NW;
  A.kk = p; p += R * flip::NW;
  A.lam = p; p += R * flip::NE;
  A.nu = p; p += R * flip::NI;
  A.KK = p;
  A.code = c->fcode;
  A.err = c->err;
  const comet_solver_params& q = c->prm;
  A.prm.al_max = L.refine ? q.ref_al_max : q.al_max;
  A.prm.gn_max = L.refine ? q.ref_gn_max : q.gn_max;
  A.prm.chol_retries = q.chol_retries;
  A.prm.ls_trials = q.ls_trials;
  A.prm.max_rejects = q.max_rejects;
  A.prm.mu0 = q.mu0; A.prm.mu_min = q.mu_min; A.prm.rho0 = q.rho0; A.prm.rho_min = q.rho_min;
  A.prm.rho_max = q.rho_max; A.prm.armijo_c1 = q.armijo_c1; A.prm.eta_star = q.eta_star;
  A.prm.omega_star = q.omega_star; A.prm.rc_star = q.rc_star; A.prm.eps_feas = q.eps_feas;
  A.prm.mu0_warm = q.mu0_warm;
  const int64_t Bmax = L.B_dev ? L.B_max : L.B;
  hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
  (void)hipStreamIsCapturing(s, &cap);
  const bool timed = (cap == hipStreamCaptureStatusNone);
  if (timed) (void)hipEventRecord(c->ev0, s);
  hipLaunchKernelGGL(flip::k_flip_solve, dim3((unsigned)std::max<int64_t>(1, Bmax)), dim3(64), 0, s, A);
  if (timed) (void)hipEventRecord(c->ev1, s);
  c->timed = timed;
  if (hipGetLastError() != hipSuccess) return fail_msg(c, COMET_EHIP, "flip kernel launch failed");
  return COMET_OK;
}

}  // namespace comet
