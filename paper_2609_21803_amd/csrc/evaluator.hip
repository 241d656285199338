// evaluator.hip -- batched mode-conditioned TO evaluator for MI355X (gfx950).
//
// One contact-mode order per lane.  Every lane runs its own augmented-Lagrangian /
// Gauss-Newton solve (Sec. III-C) as a flat state machine: each trip of the wave loop is
// one Gauss-Newton iteration (backward Riccati sweep, forward pass with all trial step
// lengths, step application) for every lane still inside an inner loop, followed by the
// outer update of the lanes whose inner loop ended.  Lanes of a wave never wait for each
// other's inner loops.  The grid is persistent: a lane whose solve ends takes the next
// order from a device work queue (the device form of the paper's reusable pool of slots
// with independent stopping, Sec. III-C), so heterogeneous solve times do not idle the
// wave until the queue is drained.  The queue can be ordered by interval count so that
// the lanes of a wave sweep similar lengths.
//
// Numerics: the model Jacobian, the gains and the forward pass run in FP32; the
// primal trajectory is stored in FP64 and the row residuals (whose rounding, divided by
// the penalty, sets the floor of the stationarity test) and merit sums are FP64; the
// Riccati recursion (block assembly A^T A / mu,
// Cholesky of S_k, gains, value update) runs in FP64 because the assembled blocks carry
// 1/mu-scaled rank-deficient terms whose small eigenvalues FP32 rounding of the
// assembly would erase.
//
// Work space (device, structure of arrays over sequence slots, so that a wave's 64 lanes
// touch 64 consecutive words for every field): primal, multipliers, gains, step and
// interval codes, one row per interval.  Inside a wave the rows are end-aligned so that
// the backward sweep of sequences of different length stays in lock-step on the same row.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "internal.h"

namespace comet {

using namespace push;

__device__ inline int wave_max(int v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v = max(v, __shfl_xor(v, o));
  return v;
}

__device__ inline bool wave_any(bool p) { return __ballot(p) != 0; }

// --------------------------------------------------------------------------------
// Per-lane view of one sequence's work space.
// --------------------------------------------------------------------------------
struct Lane {
  const EvalArgs* A;
  int64_t slot;        // work-space slot (one per resident lane)
  int64_t seq;         // sequence being solved, -1 if none
  int N, off;          // intervals, row offset (rows end-aligned to the work-space height)
  double x0[NX], goal[3], mu;

  __device__ double& z(int k, int f) const { return A->zd[((int64_t)(off + k) * NW + f) * A->S + slot]; }
  __device__ float& lam(int k, int r) const { return A->lam[((int64_t)(off + k) * NE + r) * A->S + slot]; }
  __device__ float& nu(int k, int r) const { return A->nu[((int64_t)(off + k) * NE + r) * A->S + slot]; }
  __device__ float& gain(int k, int f) const { return A->gains[((int64_t)(off + k) * NGAIN + f) * A->S + slot]; }
  __device__ float& dz(int k, int f) const { return A->dz[((int64_t)(off + k) * NW + f) * A->S + slot]; }
  __device__ int code(int k) const { return A->code[(int64_t)(off + k) * A->S + slot]; }

  __device__ void load_x(int k, double* x) const {  // x_k
    if (k == 0) {
      for (int i = 0; i < NX; ++i) x[i] = x0[i];
    } else {
      for (int i = 0; i < NX; ++i) x[i] = z(k - 1, NU + i);
    }
  }
  __device__ void load_w(int k, double* u, double* x1) const {
    for (int i = 0; i < NU; ++i) u[i] = z(k, i);
    for (int i = 0; i < NX; ++i) x1[i] = z(k, NU + i);
  }
};

// scaled residuals of one interval; multiplier estimates; merit contribution
struct RowEval {
  double c[NR];       // scaled residuals
  int en[NR];
  float J[NR][NV];    // scaled Jacobian (nz entries only)
};

template <bool JAC>
__device__ inline void eval_interval(const EvalArgs& A, const double* xk, const double* uk, const double* x1,
                                     int code, double mu, RowEval& R, const double* sc = nullptr) {
  if (sc) rows_sc<float>(xk, uk, x1, code, mu, sc[0], sc[1], R.c, JAC ? R.J : nullptr, R.en);
  else rows<float>(xk, uk, x1, code, mu, R.c, JAC ? R.J : nullptr, R.en);
  const bool stick = ((code >> 2) & 3) == 0;
#pragma unroll
  for (int r = 0; r < NR; ++r) {
    const double is = A.inv_scale[row_type(r, stick)];
    R.c[r] *= is;
    if (JAC) {
#pragma unroll
      for (int i = 0; i < NV; ++i)
        if (nz(r, i)) R.J[r][i] *= float(is);
    }
  }
}

// residuals only (no Jacobian), scaled by the given per-row factors
__device__ inline void eval_rows_scaled(const double* xk, const double* uk, const double* x1, int code, double mu,
                                        const double* sc, const double* isc, RowEval& R) {
  rows_sc<float>(xk, uk, x1, code, mu, sc[0], sc[1], R.c, nullptr, R.en);
#pragma unroll
  for (int r = 0; r < NR; ++r) R.c[r] *= isc[r];
}

// terminal rows, scaled
__device__ inline void eval_terminal(const EvalArgs& A, const double* xN, const double* goal, double* c) {
  c[0] = (xN[0] - goal[0]) * A.inv_scale[T_TXY];
  c[1] = (xN[1] - goal[1]) * A.inv_scale[T_TXY];
  c[2] = (xN[2] - goal[2]) * A.inv_scale[T_TTH];
}

// merit contribution of one interval's rows given multipliers
__device__ inline double merit_rows(const RowEval& R, const float* lam, const float* nu, double mu, double imu) {
  double phi = 0.0;
  const double hi = 0.5 * imu, hm = 0.5 * mu;
#pragma unroll
  for (int r = 0; r < NE; ++r)
    if (R.en[r]) phi += double(lam[r]) * R.c[r] + R.c[r] * R.c[r] * hi;
#pragma unroll
  for (int r = 0; r < NE; ++r) {
    if (!R.en[NE + r]) continue;
    const double n = nu[r];
    const double t = fmax(n + R.c[NE + r] * imu, 0.0);
    phi += hm * (t * t - n * n);
  }
  return phi;
}

// --------------------------------------------------------------------------------
// Sweeps over the intervals of the lanes selected by `on`.  All lanes iterate the same
// end-aligned row index; lane-local interval k = row - off.
// --------------------------------------------------------------------------------
struct FactorOut {
  double phi0, D, gnorm;
  bool ok;
};

// inputs of one interval for the backward sweep: x_k, u_k, multipliers, mode code, and the
// step directions of x_k and u_k when a step z += ap dz is pending
struct StageIn {
  double xk[NX], uk[NU];
  float dxk[NX], duk[NU];
  float lm[NE], nv[NE];
  int code;
};

__device__ inline void load_stage(const Lane& L, int k, StageIn& s, double ap) {
  L.load_x(k, s.xk);
#pragma unroll
  for (int i = 0; i < NU; ++i) s.uk[i] = L.z(k, i);
  if (ap != 0.0) {
#pragma unroll
    for (int i = 0; i < NX; ++i) s.dxk[i] = (k > 0) ? L.dz(k - 1, NU + i) : 0.f;
#pragma unroll
    for (int i = 0; i < NU; ++i) s.duk[i] = L.dz(k, i);
  }
#pragma unroll
  for (int r = 0; r < NE; ++r) {
    s.lm[r] = L.lam(k, r);
    s.nv[r] = L.nu(k, r);
  }
  s.code = L.code(k);
}

// the accepted step of the previous trip, applied to the entries of z that interval k
// reads (u_k, and x_k for k > 0) and written back: every entry of z once per sweep
__device__ inline void apply_stage(const Lane& L, int k, StageIn& s, double ap) {
  if (ap == 0.0) return;
  if (k > 0) {
#pragma unroll
    for (int i = 0; i < NX; ++i) {
      s.xk[i] += ap * double(s.dxk[i]);
      L.z(k - 1, NU + i) = s.xk[i];
    }
  }
#pragma unroll
  for (int i = 0; i < NU; ++i) {
    s.uk[i] += ap * double(s.duk[i]);
    L.z(k, i) = s.uk[i];
  }
}

// inputs of one interval for the forward sweep: u_k, x_{k+1}, gains, multipliers, code
struct FwdIn {
  double uk[NU], x1[NX];
  float g[NGAIN];
  float lm[NE], nv[NE];
  int code;
};

__device__ inline void load_fwd(const Lane& L, int k, FwdIn& s) {
  L.load_w(k, s.uk, s.x1);
#pragma unroll
  for (int i = 0; i < NGAIN; ++i) s.g[i] = L.gain(k, i);
#pragma unroll
  for (int r = 0; r < NE; ++r) {
    s.lm[r] = L.lam(k, r);
    s.nv[r] = L.nu(k, r);
  }
  s.code = L.code(k);
}

// Backward sweep: gradient, merit, Riccati factorisation and gains at the current z.
// With FACTOR = false it only returns the gradient norm (outer stationarity test),
// together with the scaled violation and complementarity residual.
template <bool FACTOR>
// With upd set, the first-order multiplier update (lam += c/mu, nu = [nu + c/mu]_+, at the
// current iterate) is applied row by row before the rows are used.  A step accepted in the
// previous trip (z += ap dz, ap != 0) is applied to z as the sweep reads it.
__device__ void sweep_backward(const Lane& L, int Nw, bool on, double mu, double imu, double rho, double* lamT,
                               bool upd, double ap, FactorOut& out, double& vs, double& rc) {
  const EvalArgs& A = *L.A;
  double P[NX][NX], p[NX], gx[NX];
  double xk1[NX];
  out.phi0 = 0.0;
  out.D = 0.0;
  out.gnorm = 0.0;
  out.ok = true;
  vs = 0.0;
  rc = 0.0;
  if (on) {
    // terminal value function V_N and terminal gradient
    double xN[NX], cT[NT];
    L.load_x(L.N, xN);
    if (ap != 0.0) {
#pragma unroll
      for (int i = 0; i < NX; ++i) {
        xN[i] += ap * double(L.dz(L.N - 1, NU + i));
        L.z(L.N - 1, NU + i) = xN[i];
      }
    }
    eval_terminal(A, xN, L.goal, cT);
    const double sT[NT] = {A.inv_scale[T_TXY], A.inv_scale[T_TXY], A.inv_scale[T_TTH]};
#pragma unroll
    for (int i = 0; i < NX; ++i) {
      p[i] = 0.0;
      gx[i] = 0.0;
#pragma unroll
      for (int j = 0; j < NX; ++j) P[i][j] = 0.0;
    }
#pragma unroll
    for (int r = 0; r < NT; ++r) {
      if (upd) lamT[r] += cT[r] * imu;
      const double y = lamT[r] + cT[r] * imu;
      out.phi0 += lamT[r] * cT[r] + cT[r] * cT[r] * (0.5 * imu);
      p[r] = y * sT[r];
      gx[r] = y * sT[r];
      P[r][r] = sT[r] * sT[r] * imu;
      vs = fmax(vs, fabs(cT[r]));
    }
#pragma unroll
    for (int i = 0; i < NX; ++i) xk1[i] = xN[i];
  }
  // software pipelining: the loads of stage k-1 are issued before stage k is computed;
  // x_{k+1} of a stage is the x_k of the stage after it
  StageIn nxt;
  double x1c[NX];
  if (on) {
    load_stage(L, L.N - 1, nxt, ap);
#pragma unroll
    for (int i = 0; i < NX; ++i) x1c[i] = xk1[i];
  }
  for (int t = 0; t < Nw; ++t) {
    const int k = L.N - 1 - t;
    if (!on || k < 0) continue;
    StageIn cur = nxt;
    if (k >= 1) load_stage(L, k - 1, nxt, ap);
    apply_stage(L, k, cur, ap);
    double xk[NX], uk[NU], x1[NX];
#pragma unroll
    for (int i = 0; i < NX; ++i) {
      xk[i] = cur.xk[i];
      x1[i] = x1c[i];
      x1c[i] = cur.xk[i];
    }
#pragma unroll
    for (int i = 0; i < NU; ++i) uk[i] = cur.uk[i];
    RowEval R;
    const int code = cur.code;
    eval_interval<true>(A, xk, uk, x1, code, L.mu, R);
    float lm[NE], nv[NE];
#pragma unroll
    for (int r = 0; r < NE; ++r) {
      lm[r] = cur.lm[r];
      nv[r] = cur.nv[r];
    }
    if (upd) {
#pragma unroll
      for (int r = 0; r < NE; ++r) {
        if (R.en[r]) {
          lm[r] = float(double(lm[r]) + R.c[r] * imu);
          L.lam(k, r) = lm[r];
        }
        if (R.en[NE + r]) {
          nv[r] = float(fmax(double(nv[r]) + R.c[NE + r] * imu, 0.0));
          L.nu(k, r) = nv[r];
        }
      }
    }
    // multiplier estimates y and curvature weights w
    double y[NR], w[NR];
#pragma unroll
    for (int r = 0; r < NE; ++r) {
      y[r] = R.en[r] ? double(lm[r]) + R.c[r] * imu : 0.0;
      w[r] = R.en[r] ? imu : 0.0;
      if (R.en[r]) vs = fmax(vs, fabs(R.c[r]));
    }
#pragma unroll
    for (int r = 0; r < NE; ++r) {
      const double tt = double(nv[r]) + R.c[NE + r] * imu;
      const bool act = R.en[NE + r] && tt > 0.0;
      y[NE + r] = act ? tt : 0.0;
      w[NE + r] = act ? imu : 0.0;
      if (R.en[NE + r]) {
        vs = fmax(vs, fmax(R.c[NE + r], 0.0));
        rc = fmax(rc, fabs(fmin(-R.c[NE + r], double(nv[r]))));
      }
    }
    out.phi0 += stage_cost(uk) + merit_rows(R, lm, nv, mu, imu);
    // gradient over v = (x_k, w_k): h = sum_r y_r a_r + cost gradient
    double h[NV];
#pragma unroll
    for (int i = 0; i < NV; ++i) h[i] = 0.0;
#pragma unroll
    for (int r = 0; r < NR; ++r)
#pragma unroll
      for (int i = 0; i < NV; ++i)
        if (nz(r, i)) h[i] += y[r] * double(R.J[r][i]);
    h[VFN] += HF * uk[0];
    h[VFT] += HF * uk[1];
    h[VVS] += HV * uk[2];
    // gradient of w_k = own rows + next interval's rows through x_{k+1}
#pragma unroll
    for (int i = 0; i < NW; ++i) {
      const double g = h[NX + i] + (i >= NU ? gx[i - NU] : 0.0);
      out.gnorm = fmax(out.gnorm, fabs(g));
    }
#pragma unroll
    for (int i = 0; i < NX; ++i) gx[i] = h[i];
    if (!FACTOR || !out.ok) continue;

    // ---- block assembly (FP64): G = sum_r w_r a_r a_r^T + cost Hessian, lower triangle
    double G[NV][NV];
#pragma unroll
    for (int i = 0; i < NV; ++i)
#pragma unroll
      for (int j = 0; j < NV; ++j) G[i][j] = 0.0;
#pragma unroll
    for (int r = 0; r < NR; ++r) {
      double a[NV];
#pragma unroll
      for (int i = 0; i < NV; ++i) a[i] = nz(r, i) ? double(R.J[r][i]) : 0.0;
#pragma unroll
      for (int i = 0; i < NV; ++i)
#pragma unroll
        for (int j = 0; j <= i; ++j)
          if (nz(r, i) && nz(r, j)) G[i][j] += w[r] * a[i] * a[j];
    }
    G[VFN][VFN] += HF;
    G[VFT][VFT] += HF;
    G[VVS][VVS] += HV;
    // S = Q_ww + embed(P_{k+1}) + rho I ; qh = q_w + embed(p_{k+1})
    double Sm[NW][NW], qh[NW], Qwx[NW][NX];
#pragma unroll
    for (int i = 0; i < NW; ++i) {
#pragma unroll
      for (int j = 0; j <= i; ++j) Sm[i][j] = G[NX + i][NX + j];
      Sm[i][i] += rho;
      qh[i] = h[NX + i];
#pragma unroll
      for (int j = 0; j < NX; ++j) Qwx[i][j] = G[NX + i][j];
    }
#pragma unroll
    for (int i = 0; i < NX; ++i) {
      qh[NU + i] += p[i];
#pragma unroll
      for (int j = 0; j <= i; ++j) Sm[NU + i][NU + j] += P[i][j];
    }
    // Cholesky S = L L^T without pivoting, in place (lower triangle)
    bool ok = true;
    double ipiv[NW];
#pragma unroll
    for (int j = 0; j < NW; ++j) {
      double d = Sm[j][j];
#pragma unroll
      for (int q = 0; q < j; ++q) d -= Sm[j][q] * Sm[j][q];
      ok = ok && (d > 0.0) && isfinite(d);
      const double dd = fmax(d, 1e-300);
      double inv = __builtin_amdgcn_rsq(dd);
      inv = inv * (1.5 - 0.5 * dd * inv * inv);  // one Newton step
      ipiv[j] = inv;
      Sm[j][j] = dd * inv;
#pragma unroll
      for (int i = j + 1; i < NW; ++i) {
        double s2 = Sm[i][j];
#pragma unroll
        for (int q = 0; q < j; ++q) s2 -= Sm[i][q] * Sm[j][q];
        Sm[i][j] = s2 * inv;
      }
    }
    if (!ok) {
      out.ok = false;
      continue;
    }
    // Y = L^-1 Qwx, yv = L^-1 qh
#pragma unroll
    for (int i = 0; i < NW; ++i) {
      const double inv = ipiv[i];
#pragma unroll
      for (int q = 0; q < i; ++q) {
        qh[i] -= Sm[i][q] * qh[q];
#pragma unroll
        for (int j = 0; j < NX; ++j) Qwx[i][j] -= Sm[i][q] * Qwx[q][j];
      }
      qh[i] *= inv;
#pragma unroll
      for (int j = 0; j < NX; ++j) Qwx[i][j] *= inv;
    }
    // value function: P = Q_xx - Y^T Y, p = q_x - Y^T y ; model decrease D += -y^T y
#pragma unroll
    for (int i = 0; i < NX; ++i) {
      double pi = h[i];
#pragma unroll
      for (int q = 0; q < NW; ++q) pi -= Qwx[q][i] * qh[q];
      p[i] = pi;
#pragma unroll
      for (int j = 0; j <= i; ++j) {
        double pij = G[i][j];
#pragma unroll
        for (int q = 0; q < NW; ++q) pij -= Qwx[q][i] * Qwx[q][j];
        P[i][j] = pij;
        P[j][i] = pij;
      }
    }
#pragma unroll
    for (int q = 0; q < NW; ++q) out.D -= qh[q] * qh[q];
    // gains: k = -L^-T y, K = -L^-T Y (back substitution)
#pragma unroll
    for (int i = NW - 1; i >= 0; --i) {
      const double inv = ipiv[i];
#pragma unroll
      for (int q = i + 1; q < NW; ++q) {
        qh[i] -= Sm[q][i] * qh[q];
#pragma unroll
        for (int j = 0; j < NX; ++j) Qwx[i][j] -= Sm[q][i] * Qwx[q][j];
      }
      qh[i] *= inv;
#pragma unroll
      for (int j = 0; j < NX; ++j) Qwx[i][j] *= inv;
    }
#pragma unroll
    for (int i = 0; i < NW; ++i) {
      L.gain(k, i) = float(-qh[i]);
#pragma unroll
      for (int j = 0; j < NX; ++j) L.gain(k, NW + i * NX + j) = float(-Qwx[i][j]);
    }
  }
}

// Forward pass: dz from the gains (stored), merit at every trial step length.  The trial
// loop is unrolled over TU >= T slots so that each trial's merit accumulator phi[i] is a
// fixed register (a run-time trial index would select among all accumulators per trial).
template <int TU>
__device__ void sweep_forward(const Lane& L, int Nw, bool on, double mu, double imu, const double* lamT, int T,
                              double* phi) {
  const EvalArgs& A = *L.A;
  float dx[NX] = {0.f, 0.f, 0.f, 0.f};
  double xk[NX];
#pragma unroll
  for (int i = 0; i < MAX_TRIALS; ++i) phi[i] = 0.0;
  FwdIn nxt;
  if (on) {
    L.load_x(0, xk);
    load_fwd(L, 0, nxt);
  }
  for (int t = 0; t < Nw; ++t) {
    const int k = t - (Nw - L.N);
    if (!on || k < 0) continue;
    const FwdIn cur = nxt;
    if (k + 1 < L.N) load_fwd(L, k + 1, nxt);   // next stage's loads in flight during this stage
    double uk[NU], x1[NX];
#pragma unroll
    for (int i = 0; i < NU; ++i) uk[i] = cur.uk[i];
#pragma unroll
    for (int i = 0; i < NX; ++i) x1[i] = cur.x1[i];
    float dw[NW];
#pragma unroll
    for (int i = 0; i < NW; ++i) {
      float s = cur.g[i];
#pragma unroll
      for (int j = 0; j < NX; ++j) s += cur.g[NW + i * NX + j] * dx[j];
      dw[i] = s;
      L.dz(k, i) = s;
    }
    float lm[NE], nv[NE];
#pragma unroll
    for (int r = 0; r < NE; ++r) {
      lm[r] = cur.lm[r];
      nv[r] = cur.nv[r];
    }
    const int code = cur.code;
    // per-interval constants of the trial steps: row scale factors and the directions in FP64
    double isc[NR], dxd[NX], dwd[NW];
    {
      const bool stick = ((code >> 2) & 3) == 0;
#pragma unroll
      for (int r = 0; r < NR; ++r) isc[r] = A.inv_scale[row_type(r, stick)];
#pragma unroll
      for (int q = 0; q < NX; ++q) dxd[q] = double(dx[q]);
#pragma unroll
      for (int q = 0; q < NW; ++q) dwd[q] = double(dw[q]);
    }
    // sin / cos of theta_k + a_i, a_i = 2^-i dtheta: one sincos of theta_k and of the
    // smallest a_i, then angle doubling towards a_0 and angle addition
    double sb, cb, sa, ca;
    sincos_d(xk[2], &sb, &cb);
    double alpha = ldexp(1.0, -(T - 1));
    sincos_d(alpha * double(dx[2]), &sa, &ca);
#pragma unroll
    for (int i = TU - 1; i >= 0; --i) {
      if (i >= T) continue;   // the same in every lane
      double xt[NX], ut[NU], x1t[NX];
#pragma unroll
      for (int q = 0; q < NX; ++q) {
        xt[q] = xk[q] + alpha * dxd[q];
        x1t[q] = x1[q] + alpha * dwd[NU + q];
      }
#pragma unroll
      for (int q = 0; q < NU; ++q) ut[q] = uk[q] + alpha * dwd[q];
      const double sc[2] = {sb * ca + cb * sa, cb * ca - sb * sa};
      RowEval R;
      eval_rows_scaled(xt, ut, x1t, code, L.mu, sc, isc, R);
      phi[i] += stage_cost(ut) + merit_rows(R, lm, nv, mu, imu);
      const double s2 = 2.0 * sa * ca, c2 = ca * ca - sa * sa;
      sa = s2;
      ca = c2;
      alpha *= 2.0;
    }
#pragma unroll
    for (int q = 0; q < NX; ++q) {
      xk[q] = x1[q];
      dx[q] = dw[NU + q];
    }
  }
  if (on) {
    double alpha = 1.0;
#pragma unroll
    for (int i = 0; i < TU; ++i) {
      if (i >= T) break;
      double xt[NX], cT[NT];
#pragma unroll
      for (int q = 0; q < NX; ++q) xt[q] = xk[q] + alpha * double(dx[q]);
      eval_terminal(A, xt, L.goal, cT);
      double contrib = 0.0;
#pragma unroll
      for (int r = 0; r < NT; ++r) contrib += lamT[r] * cT[r] + cT[r] * cT[r] * (0.5 * imu);
      phi[i] += contrib;
      alpha *= 0.5;
    }
  }
}

// physical-unit score (Eq. 4) and trajectory output
__device__ void sweep_score(const Lane& L, int Nw, bool on, double& J, double& v) {
  const EvalArgs& A = *L.A;
  J = 0.0;
  v = 0.0;
  for (int t = 0; t < Nw; ++t) {
    const int k = t - (Nw - L.N);
    if (!on || k < 0) continue;
    double xk[NX], uk[NU], x1[NX], c[NR];
    int en[NR];
    L.load_x(k, xk);
    L.load_w(k, uk, x1);
    rows<float>(xk, uk, x1, L.code(k), L.mu, c, (float(*)[NV]) nullptr, en);
    J += stage_cost(uk);
#pragma unroll
    for (int r = 0; r < NE; ++r)
      if (en[r]) v = fmax(v, fabs(c[r]));
#pragma unroll
    for (int r = NE; r < NR; ++r)
      if (en[r]) v = fmax(v, fmax(c[r], 0.0));
    if (!isfinite(J) || !isfinite(c[0]) || !isfinite(c[1]) || !isfinite(c[2]) || !isfinite(c[3])) v = INFINITY;
    if (A.traj) {
      float* T = A.traj + (L.seq * (int64_t)(A.nmax + 1) + k) * (NX + NU);
#pragma unroll
      for (int i = 0; i < NX; ++i) T[i] = float(xk[i]);
#pragma unroll
      for (int i = 0; i < NU; ++i) T[NX + i] = float(uk[i]);
    }
  }
  if (on) {
    double xN[NX];
    L.load_x(L.N, xN);
    v = fmax(v, fabs(xN[0] - L.goal[0]));
    v = fmax(v, fabs(xN[1] - L.goal[1]));
    v = fmax(v, fabs(xN[2] - L.goal[2]));
    if (A.traj) {
      float* T = A.traj + (L.seq * (int64_t)(A.nmax + 1) + L.N) * (NX + NU);
#pragma unroll
      for (int i = 0; i < NX; ++i) T[i] = float(xN[i]);
#pragma unroll
      for (int i = 0; i < NU; ++i) T[NX + i] = 0.f;
    }
  }
}

// --------------------------------------------------------------------------------
// Sequence intake: validate, write interval codes, initial guess and zero multipliers
// into the lane's rows.  Invalid sequences are scored infeasible right away.
// --------------------------------------------------------------------------------
__device__ bool load_sequence(Lane& L, int64_t b) {
  const EvalArgs& A = *L.A;
  int K = A.nseg[b];
  bool valid = (K >= 1 && K <= A.smax);
  int N = 0;
  for (int j = 0; j < MAXSEG; ++j) {
    if (!valid || j >= K) break;
    const int m = A.modes[b * A.smax + j], n = A.knots[b * A.smax + j];
    if (m < 0 || m >= NMODES || n < 1) valid = false;
    N += n;
  }
  if (N > A.nmax) valid = false;
  const int64_t bi = b * A.inst_stride;
  for (int i = 0; i < NX; ++i) {
    L.x0[i] = A.x0[bi * NX + i];
    valid = valid && isfinite(L.x0[i]);
  }
  for (int i = 0; i < 3; ++i) {
    L.goal[i] = A.goal[bi * 3 + i];
    valid = valid && isfinite(L.goal[i]);
  }
  L.mu = A.inst[bi];
  valid = valid && isfinite(L.mu);
  if (!valid) {
    atomicAdd(A.err, 1u);
    A.cost[b] = NAN;
    A.viol[b] = INFINITY;
    A.feas[b] = 0;
    if (A.cost64) {
      A.cost64[b] = NAN;
      A.viol64[b] = INFINITY;
    }
    if (A.stats) {
      A.stats[b * 4 + 0] = 0;
      A.stats[b * 4 + 1] = 0;
      A.stats[b * 4 + 2] = 0;
      A.stats[b * 4 + 3] = 3;
    }
    if (A.traj)
      for (int i = 0; i < (A.nmax + 1) * (NX + NU); ++i) A.traj[b * (int64_t)(A.nmax + 1) * (NX + NU) + i] = 0.f;
    return false;
  }
  L.seq = b;
  L.N = N;
  L.off = A.nmax - N;
  int k = 0;
  for (int j = 0; j < K; ++j) {
    const int m = A.modes[b * A.smax + j], n = A.knots[b * A.smax + j];
    const int mnext = (j + 1 < K) ? A.modes[b * A.smax + j + 1] : m;
    for (int i = 0; i < n; ++i, ++k) {
      const int smask = (i == n - 1 && (mnext / 3) != (m / 3)) ? 0 : 1;
      A.code[(int64_t)(L.off + k) * A.S + L.slot] = (uint8_t)make_code(m, smask);
    }
  }
  const double fn = 0.05 * FMAX;
  for (int k2 = 0; k2 < N; ++k2) {
    const int c = L.code(k2);
    const int slip = (c >> 2) & 3;
    const double sg = (slip == 1) ? 1.0 : ((slip == 2) ? -1.0 : 0.0);
    if (A.warm) {
      const float* W = A.warm + b * (int64_t)(A.nmax + 1) * (NX + NU);
      for (int i = 0; i < NU; ++i) L.z(k2, i) = W[k2 * (NX + NU) + NX + i];
      for (int i = 0; i < NX; ++i) L.z(k2, NU + i) = W[(k2 + 1) * (NX + NU) + i];
    } else {
      const double tfrac = double(k2 + 1) / double(N);
      L.z(k2, 0) = fn;
      L.z(k2, 1) = sg * L.mu * fn;
      L.z(k2, 2) = 0.0;
      for (int i = 0; i < 3; ++i) L.z(k2, NU + i) = L.x0[i] + (L.goal[i] - L.x0[i]) * tfrac;
      L.z(k2, NU + 3) = L.x0[3];
    }
    for (int r = 0; r < NE; ++r) {
      L.lam(k2, r) = 0.f;
      L.nu(k2, r) = 0.f;
    }
  }
  return true;
}

// Solver state of one lane.
struct SolverState {
  double mu, imu, eta, omega, rho, lamT[NT];
  int al, gn_in, gn_tot, rejects, tries, cfails, status;
  bool upd, outer_pending;   // multiplier update to apply in the next sweep; outer test due next sweep
  __device__ void reset(const DevParams& prm, bool warm) {
    mu = warm ? prm.mu0_warm : prm.mu0;
    imu = 1.0 / mu;
    eta = pow(mu, 0.1);
    omega = mu;
    rho = prm.rho0;
    lamT[0] = lamT[1] = lamT[2] = 0.0;
    al = gn_in = gn_tot = rejects = tries = cfails = status = 0;
    upd = outer_pending = false;
  }
};

// --------------------------------------------------------------------------------
// The solver kernel: persistent, one sequence per lane at a time, 64 lanes per block.
// --------------------------------------------------------------------------------
__global__ __launch_bounds__(WAVE) void k_push_solve(EvalArgs A) {
  const int lane = threadIdx.x;
  const DevParams& prm = A.prm;
  Lane L;
  L.A = &A;
  L.slot = (int64_t)blockIdx.x * WAVE + lane;
  L.seq = -1;
  L.N = 0;
  L.off = A.nmax;
  SolverState st;
  st.reset(prm, false);
  bool exhausted = false;
  double pend = 0.0;   // step length of an accepted step not yet applied to z
  const int64_t Bn = A.Bdev ? *A.Bdev : A.B;
  const int T = min(max(prm.ls_trials, 1), MAX_TRIALS);

  for (;;) {
    // intake: lanes without a sequence pop the queue (one atomic per wave)
    for (;;) {
      const bool need = (L.seq < 0) && !exhausted;
      const unsigned long long m = __ballot(need);
      if (!m) break;
      const int leader = __ffsll((long long)m) - 1;
      unsigned long long base = 0;
      if (lane == leader) base = atomicAdd(A.qhead, (unsigned long long)__popcll(m));
      base = __shfl(base, leader);
      if (need) {
        const unsigned long long q = base + __popcll(m & ((1ull << lane) - 1ull));
        if (q >= (unsigned long long)Bn) {
          exhausted = true;
        } else {
          const int64_t b = A.order ? (int64_t)A.order[q] : (int64_t)q;
          pend = 0.0;
          if (load_sequence(L, b)) st.reset(prm, A.warm != nullptr);
        }
      }
    }
    const bool active = L.seq >= 0;
    if (!wave_any(active)) break;
    const int Nw = wave_max(active ? L.N : 0);

    // One backward sweep per trip: gradient, merit, factorisation -- and, at the same
    // iterate, the scaled violation, complementarity and stationarity that the outer test
    // needs (pending multiplier updates are applied inside the sweep).
    FactorOut fo;
    double vsv, rcv;
    sweep_backward<true>(L, Nw, active, st.mu, st.imu, st.rho, st.lamT, active && st.upd, active ? pend : 0.0, fo,
                         vsv, rcv);
    pend = 0.0;
    if (active) st.upd = false;
    bool step = false, outer_now = false, accepted = false;
    double alpha_acc = 0.0;
    if (active) {
      if (st.outer_pending) {
        // the inner loop ended with an accepted step: this sweep saw the new iterate
        st.outer_pending = false;
        outer_now = true;
      } else if (fo.gnorm <= st.omega) {
        outer_now = true;
      } else if (!fo.ok) {
        ++st.cfails;
        if (st.tries < prm.chol_retries) {
          st.rho = fmax(10.0 * st.rho, 1e-8);
          ++st.tries;
        } else {
          st.tries = 0;
          ++st.gn_in;
          ++st.gn_tot;
          st.rho = fmin(10.0 * st.rho, prm.rho_max);
          if (++st.rejects >= prm.max_rejects || st.gn_in >= prm.gn_max) outer_now = true;
        }
      } else {
        st.tries = 0;
        ++st.gn_in;
        ++st.gn_tot;
        if (fo.D < 0.0 && isfinite(fo.phi0)) {
          step = true;
        } else {
          st.rho = fmin(10.0 * st.rho, prm.rho_max);
          if (++st.rejects >= prm.max_rejects || st.gn_in >= prm.gn_max) outer_now = true;
        }
      }
    }
    if (wave_any(step)) {
      double phi[MAX_TRIALS];
      // the default eight trials take the short unrolled variant
      if (T <= 8)
        sweep_forward<8>(L, Nw, step, st.mu, st.imu, st.lamT, T, phi);
      else
        sweep_forward<MAX_TRIALS>(L, Nw, step, st.mu, st.imu, st.lamT, T, phi);
      if (step) {
        int best = -1;
        double alpha = 1.0, a_best = 0.0;
#pragma unroll
        for (int i = 0; i < MAX_TRIALS; ++i) {
          if (i >= T) break;
          const double ph = phi[i];
          if (best < 0 && isfinite(ph) && ph <= fo.phi0 + prm.armijo_c1 * alpha * fo.D) {
            best = i;
            a_best = alpha;
          }
          alpha *= 0.5;
        }
        if (best >= 0) {
          accepted = true;
          alpha_acc = a_best;
          st.rho = fmax(st.rho / 3.0, prm.rho_min);
          st.rejects = 0;
          if (st.gn_in >= prm.gn_max) st.outer_pending = true;  // outer test at the new iterate, next trip
        } else {
          st.rho = fmin(10.0 * st.rho, prm.rho_max);
          ++st.rejects;
          if (st.rejects >= prm.max_rejects || st.gn_in >= prm.gn_max) outer_now = true;  // iterate unchanged
        }
      }
    }
    // an accepted step is applied by the next trip's backward sweep as it reads z
    if (accepted) pend = alpha_acc;
    bool fin = false;
    if (outer_now) {
      ++st.al;
      st.gn_in = 0;
      st.rejects = 0;
      if (!isfinite(vsv) || !isfinite(fo.gnorm)) {
        st.status = 2;
        fin = true;
      } else if (vsv <= st.eta) {
        if (vsv <= prm.eta_star && fo.gnorm <= prm.omega_star && rcv <= prm.rc_star) {
          st.status = 1;
          fin = true;
        } else {
          st.upd = true;
          st.eta = fmax(st.eta * pow(st.mu, 0.9), prm.eta_star);
          st.omega = fmax(st.omega * st.mu, prm.omega_star);
        }
      } else {
        st.mu = fmax(0.1 * st.mu, prm.mu_min);
        st.imu = 1.0 / st.mu;
        st.eta = fmax(pow(st.mu, 0.1), prm.eta_star);
        st.omega = fmax(st.mu, prm.omega_star);
      }
      if (!fin && st.al >= prm.al_max) {
        st.status = 0;
        fin = true;
        st.upd = false;
      }
    }
    if (wave_any(fin)) {
      double J, v;
      sweep_score(L, Nw, fin, J, v);
      if (fin) {
        const int64_t b = L.seq;
        if (st.status == 2 || !isfinite(J) || !isfinite(v)) {
          J = NAN;
          v = INFINITY;
          st.status = 2;
        }
        A.cost[b] = float(J);
        A.viol[b] = float(v);
        A.feas[b] = (v <= prm.eps_feas) ? 1 : 0;
        if (A.cost64) {
          A.cost64[b] = J;
          A.viol64[b] = v;
        }
        if (A.t_first && v <= prm.eps_feas) atomicMin(A.t_first, (unsigned long long)wall_clock64());
        if (A.stats) {
          A.stats[b * 4 + 0] = st.al;
          A.stats[b * 4 + 1] = st.gn_tot;
          A.stats[b * 4 + 2] = st.cfails;
          A.stats[b * 4 + 3] = st.status;
        }
        if (A.traj) {  // zero rows beyond N
          for (int k = L.N + 1; k <= A.nmax; ++k)
            for (int i = 0; i < NX + NU; ++i) A.traj[(b * (int64_t)(A.nmax + 1) + k) * (NX + NU) + i] = 0.f;
        }
        L.seq = -1;
      }
    }
  }
}

// --------------------------------------------------------------------------------
// Queue set-up kernels: reset the head, and (optionally) order the sequences by
// decreasing interval count with a counting sort (histogram, scan, scatter).
// --------------------------------------------------------------------------------
__global__ void k_queue_reset(unsigned long long* qhead, int* hist, int nbins) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i == 0) *qhead = 0ull;
  if (hist && i < nbins) hist[i] = 0;
}

__device__ inline int seq_len(const EvalArgs& A, int64_t b) {
  const int K = A.nseg[b];
  if (K < 1 || K > A.smax) return 0;
  int N = 0;
  for (int j = 0; j < K; ++j) N += max(A.knots[b * A.smax + j], 0);
  return min(N, A.nmax + 1);
}

__global__ void k_queue_hist(EvalArgs A, int* hist) {
  const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t Bn = A.Bdev ? *A.Bdev : A.B;
  if (b < Bn) atomicAdd(&hist[seq_len(A, b)], 1);
}

// exclusive scan over bins in decreasing length order (one block)
__global__ void k_queue_scan(int* hist, int nbins) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    int acc = 0;
    for (int n = nbins - 1; n >= 0; --n) {
      const int c = hist[n];
      hist[n] = acc;
      acc += c;
    }
  }
}

__global__ void k_queue_scatter(EvalArgs A, int* hist, int* order) {
  const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t Bn = A.Bdev ? *A.Bdev : A.B;
  if (b < Bn) order[atomicAdd(&hist[seq_len(A, b)], 1)] = (int)b;
}

}  // namespace comet

// ==================================================================================
// Host side: context, row scales, C ABI.
// ==================================================================================
namespace {

comet_status fail(comet_ctx* c, comet_status s, const std::string& m) { return comet::fail_msg(c, s, m); }

// Row scales: for every row type, the median 2-norm of its physical Jacobian row over the
// schedule-derived initial guesses of a fixed sample of orders (all 144 two-segment orders,
// 5 + 5 intervals, start at rest at the origin, goal (0.1, 0.1, pi/4), pusher friction
// 0.4); median of an even count = mean of the two middle values.  Evaluated in double on
// the host with the same model code the device uses.
void compute_scales(double* out) {
  using namespace comet::push;
  std::vector<double> vals[NTYPES];
  const double x0[NX] = {0, 0, 0, 0}, goal[3] = {0.1, 0.1, M_PI / 4.0}, mu = 0.4;
  for (int m1 = 0; m1 < NMODES; ++m1)
    for (int m2 = 0; m2 < NMODES; ++m2) {
      const int N = 10;
      int code[N];
      for (int k = 0; k < N; ++k) {
        const int m = k < 5 ? m1 : m2;
        const int smask = (k == 4 && (m2 / 3) != (m1 / 3)) ? 0 : 1;
        code[k] = make_code(m, smask);
      }
      double xs[N + 1][NX], us[N][NU];
      for (int i = 0; i < NX; ++i) xs[0][i] = x0[i];
      for (int k = 0; k < N; ++k) {
        const int slip = (code[k] >> 2) & 3;
        const double sg = slip == 1 ? 1.0 : (slip == 2 ? -1.0 : 0.0);
        us[k][0] = 0.05 * FMAX;
        us[k][1] = sg * mu * us[k][0];
        us[k][2] = 0.0;
        const double t = double(k + 1) / N;
        for (int i = 0; i < 3; ++i) xs[k + 1][i] = x0[i] + (goal[i] - x0[i]) * t;
        xs[k + 1][3] = x0[3];
      }
      for (int k = 0; k < N; ++k) {
        double c[NR], J[NR][NV];
        int en[NR];
        for (int r = 0; r < NR; ++r)
          for (int i = 0; i < NV; ++i) J[r][i] = 0.0;
        rows<double>(xs[k], us[k], xs[k + 1], code[k], mu, c, J, en);
        const bool stick = ((code[k] >> 2) & 3) == 0;
        for (int r = 0; r < NR; ++r) {
          if (!en[r]) continue;
          double n2 = 0.0;
          for (int i = 0; i < NV; ++i) n2 += J[r][i] * J[r][i];
          vals[row_type(r, stick)].push_back(std::sqrt(n2));
        }
      }
      for (int r = 0; r < 2; ++r) vals[T_TXY].push_back(1.0);
      vals[T_TTH].push_back(1.0);
    }
  for (int t = 0; t < NTYPES; ++t) {
    std::vector<double>& v = vals[t];
    std::sort(v.begin(), v.end());
    const size_t n = v.size();
    out[t] = (n == 0) ? 1.0 : ((n % 2) ? v[n / 2] : 0.5 * (v[n / 2 - 1] + v[n / 2]));
  }
}

}  // namespace

namespace comet {

comet_status fail_msg(comet_ctx* c, comet_status st, const std::string& m) {
  if (c) c->msg = m;
  return st;
}

comet_status launch_evaluate(comet_ctx* c, hipStream_t s, const EvalLaunch& L) {
  EvalArgs A;
  std::memset(&A, 0, sizeof A);
  A.B = L.B;
  A.Bdev = L.B_dev;
  A.smax = c->max_segments;
  A.nmax = c->max_intervals;
  A.S = c->S;
  A.x0 = L.x0; A.goal = L.goal; A.inst = L.inst; A.inst_stride = L.inst_stride;
  A.nseg = L.nseg; A.modes = L.modes; A.knots = L.knots; A.warm = L.warm;
  A.cost = L.cost; A.viol = L.viol; A.feas = L.feas; A.traj = L.traj; A.stats = L.stats;
  A.cost64 = L.cost64; A.viol64 = L.viol64; A.t_first = L.t_first;
  A.zd = c->zd; A.lam = c->lam; A.nu = c->nu; A.gains = c->gains; A.dz = c->dz; A.code = c->code; A.err = c->err;
  A.qhead = c->qhead;
  A.order = (c->sched.sort_by_length && !L.no_sort) ? c->order : nullptr;
  const comet_solver_params& p = c->prm;
  A.prm.al_max = L.refine ? p.ref_al_max : p.al_max;
  A.prm.gn_max = L.refine ? p.ref_gn_max : p.gn_max;
  A.prm.chol_retries = p.chol_retries;
  A.prm.ls_trials = p.ls_trials;
  A.prm.max_rejects = p.max_rejects;
  A.prm.mu0 = p.mu0; A.prm.mu_min = p.mu_min; A.prm.rho0 = p.rho0; A.prm.rho_min = p.rho_min;
  A.prm.rho_max = p.rho_max; A.prm.armijo_c1 = p.armijo_c1; A.prm.eta_star = p.eta_star;
  A.prm.omega_star = p.omega_star; A.prm.rc_star = p.rc_star; A.prm.eps_feas = p.eps_feas;
  A.prm.mu0_warm = p.mu0_warm;
  for (int t = 0; t < NTYPES; ++t) A.inv_scale[t] = 1.0 / c->scale[t];
  const int64_t Bmax = L.B_dev ? L.B_max : L.B;
  const int64_t blocks_needed = (Bmax + WAVE - 1) / WAVE;
  const int wpc = c->sched.waves_per_cu > 0 ? c->sched.waves_per_cu : c->occ_blocks_per_cu;
  const unsigned grid = (unsigned)std::max<int64_t>(1, std::min<int64_t>(blocks_needed, (int64_t)wpc * c->n_cu));
  const int nbins = c->max_intervals + 2;
  hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
  (void)hipStreamIsCapturing(s, &cap);
  const bool timed = (cap == hipStreamCaptureStatusNone);
  hipLaunchKernelGGL(k_queue_reset, dim3((nbins + 255) / 256), dim3(256), 0, s, c->qhead,
                     A.order ? c->hist : (int*)nullptr, nbins);
  if (A.order) {
    const unsigned gb = (unsigned)std::max<int64_t>(1, (Bmax + 255) / 256);
    hipLaunchKernelGGL(k_queue_hist, dim3(gb), dim3(256), 0, s, A, c->hist);
    hipLaunchKernelGGL(k_queue_scan, dim3(1), dim3(64), 0, s, c->hist, nbins);
    hipLaunchKernelGGL(k_queue_scatter, dim3(gb), dim3(256), 0, s, A, c->hist, c->order);
  }
  if (timed) (void)hipEventRecord(c->ev0, s);
  hipLaunchKernelGGL(k_push_solve, dim3(grid), dim3(WAVE), 0, s, A);
  if (timed) (void)hipEventRecord(c->ev1, s);
  c->timed = timed;
  if (hipGetLastError() != hipSuccess) return fail_msg(c, COMET_EHIP, "kernel launch failed");
  return COMET_OK;
}

}  // namespace comet

extern "C" {

void comet_default_params(comet_solver_params* p) {
  if (!p) return;
  p->al_max = 20;
  p->gn_max = 10;
  p->ref_al_max = 40;
  p->ref_gn_max = 25;
  p->chol_retries = 6;
  p->ls_trials = 8;
  p->max_rejects = 4;
  p->reserved = 0;
  p->mu0 = 1e-2;
  p->mu_min = 1e-4;
  p->rho0 = 1e-4;
  p->rho_min = 1e-8;
  p->rho_max = 1e8;
  p->armijo_c1 = 1e-4;
  p->eta_star = 1e-6;
  p->omega_star = 1e-4;
  p->rc_star = 1e-6;
  p->eps_feas = 1e-5;
  p->mu0_warm = 1e-4;
}

comet_status comet_create(comet_task task, const comet_solver_params* params, int64_t max_batch,
                          int32_t max_segments, int32_t max_intervals, comet_ctx** out) {
  if (!out) return COMET_EINVAL;
  *out = nullptr;
  if ((task != COMET_TASK_PUSH && task != COMET_TASK_FLIP) || max_batch < 1 || max_segments < 1 ||
      max_segments > comet::MAXSEG ||
      max_intervals < 1 || max_intervals > comet::MAXN)
    return COMET_EINVAL;
  comet_ctx* c = new comet_ctx();
  c->task = task;
  if (params) c->prm = *params;
  else comet_default_params(&c->prm);
  if (c->prm.ls_trials < 1 || c->prm.ls_trials > comet::MAX_TRIALS || c->prm.al_max < 1 || c->prm.gn_max < 1 ||
      !(c->prm.mu0 > 0) || !(c->prm.mu_min > 0) || !(c->prm.mu0_warm > 0)) {
    delete c;
    return COMET_EINVAL;
  }
  c->max_batch = max_batch;
  c->S = (max_batch + 63) / 64 * 64;
  c->max_segments = max_segments;
  c->max_intervals = max_intervals;
  (void)hipGetDevice(&c->device);
  compute_scales(c->scale);
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, c->device) != hipSuccess) {
    delete c;
    return COMET_EHIP;
  }
  c->n_cu = prop.multiProcessorCount;
  if (task == COMET_TASK_FLIP) {
    comet_status st = comet::flip_create_ws(c);
    if (st == COMET_OK && (hipMalloc(&c->err, sizeof(unsigned)) != hipSuccess ||
                           hipMemset(c->err, 0, sizeof(unsigned)) != hipSuccess ||
                           hipEventCreate(&c->ev0) != hipSuccess || hipEventCreate(&c->ev1) != hipSuccess))
      st = COMET_EHIP;
    if (st != COMET_OK) {
      comet_destroy(c);
      return st;
    }
    *out = c;
    return COMET_OK;
  }
  int nb = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, comet::k_push_solve, comet::WAVE, 0) != hipSuccess || nb < 1)
    nb = 1;
  c->occ_blocks_per_cu = nb;
  const int64_t R = max_intervals, S = c->S;
  using namespace comet::push;
  bool okm = hipMalloc(&c->zd, sizeof(double) * R * NW * S) == hipSuccess &&
             hipMalloc(&c->lam, sizeof(float) * R * NE * S) == hipSuccess &&
             hipMalloc(&c->nu, sizeof(float) * R * NE * S) == hipSuccess &&
             hipMalloc(&c->gains, sizeof(float) * R * NGAIN * S) == hipSuccess &&
             hipMalloc(&c->dz, sizeof(float) * R * NW * S) == hipSuccess &&
             hipMalloc(&c->code, sizeof(uint8_t) * R * S) == hipSuccess &&
             hipMalloc(&c->err, sizeof(unsigned)) == hipSuccess &&
             hipMalloc(&c->qhead, sizeof(unsigned long long)) == hipSuccess &&
             hipMalloc(&c->hist, sizeof(int) * (R + 2)) == hipSuccess &&
             hipMalloc(&c->order, sizeof(int) * max_batch) == hipSuccess;
  if (!okm) {
    (void)hipGetLastError();
    comet_destroy(c);
    return COMET_ENOMEM;
  }
  if (hipMemset(c->err, 0, sizeof(unsigned)) != hipSuccess || hipEventCreate(&c->ev0) != hipSuccess ||
      hipEventCreate(&c->ev1) != hipSuccess) {
    comet_destroy(c);
    return COMET_EHIP;
  }
  *out = c;
  return COMET_OK;
}

void comet_destroy(comet_ctx* c) {
  if (!c) return;
  comet::destroy_expand_ws(c);
  comet::flip_destroy_ws(c);
  if (c->gstream) (void)hipStreamDestroy(c->gstream);
  if (c->zd) (void)hipFree(c->zd);
  if (c->lam) (void)hipFree(c->lam);
  if (c->nu) (void)hipFree(c->nu);
  if (c->gains) (void)hipFree(c->gains);
  if (c->dz) (void)hipFree(c->dz);
  if (c->code) (void)hipFree(c->code);
  if (c->err) (void)hipFree(c->err);
  if (c->qhead) (void)hipFree(c->qhead);
  if (c->hist) (void)hipFree(c->hist);
  if (c->order) (void)hipFree(c->order);
  if (c->ev0) (void)hipEventDestroy(c->ev0);
  if (c->ev1) (void)hipEventDestroy(c->ev1);
  delete c;
}

const char* comet_last_error(const comet_ctx* c) { return c ? c->msg.c_str() : "null context"; }

comet_status comet_dims(const comet_ctx* c, int32_t* nx, int32_t* nu, int32_t* np, int32_t* nm, int32_t* ms,
                        int32_t* mi, int64_t* mb) {
  if (!c) return COMET_EINVAL;
  const bool fl = (c->task == COMET_TASK_FLIP);
  if (nx) *nx = fl ? 8 : comet::push::NX;
  if (nu) *nu = fl ? 9 : comet::push::NU;
  if (np) *np = 1;
  if (nm) *nm = fl ? 845 : comet::push::NMODES;
  if (ms) *ms = c->max_segments;
  if (mi) *mi = c->max_intervals;
  if (mb) *mb = c->max_batch;
  return COMET_OK;
}

comet_status comet_row_scales(const comet_ctx* c, double* out, int32_t n) {
  if (!c || !out || n < comet::push::NTYPES || c->task != COMET_TASK_PUSH) return COMET_EINVAL;
  for (int t = 0; t < comet::push::NTYPES; ++t) out[t] = c->scale[t];
  return COMET_OK;
}

comet_status comet_check(comet_ctx* c, void* stream) {
  if (!c) return COMET_EINVAL;
  unsigned h = 0;
  if (hipStreamSynchronize((hipStream_t)stream) != hipSuccess) return fail(c, COMET_EHIP, "stream synchronize failed");
  if (hipMemcpy(&h, c->err, sizeof(unsigned), hipMemcpyDeviceToHost) != hipSuccess ||
      hipMemset(c->err, 0, sizeof(unsigned)) != hipSuccess)
    return fail(c, COMET_EHIP, "reading the device error counter failed");
  if (h) return fail(c, COMET_EINVAL, std::to_string(h) + " sequence(s) had invalid device data");
  return COMET_OK;
}

comet_status comet_evaluate(comet_ctx* c, void* stream, int64_t B, const float* x0, const float* goal,
                            const float* inst, const int32_t* nseg, const int32_t* modes, const int32_t* knots,
                            const float* warm, int32_t refine, float* cost, float* viol, uint8_t* feasible,
                            float* traj, int32_t* stats) {
  if (!c) return COMET_EINVAL;
  if (B == 0) return COMET_OK;
  if (B < 0 || B > c->max_batch) return fail(c, COMET_EINVAL, "batch size outside [0, max_batch]");
  if (!x0 || !goal || !inst || !nseg || !modes || !knots || !cost || !viol || !feasible)
    return fail(c, COMET_EINVAL, "null input or output pointer");
  if (refine != 0 && refine != 1) return fail(c, COMET_EINVAL, "refine must be 0 or 1");
  comet::EvalLaunch L;
  L.B = B;
  L.B_max = B;
  L.x0 = x0; L.goal = goal; L.inst = inst; L.inst_stride = 1;
  L.nseg = nseg; L.modes = modes; L.knots = knots; L.warm = warm; L.refine = refine;
  L.cost = cost; L.viol = viol; L.feas = feasible; L.traj = traj; L.stats = stats;
  if (c->task == COMET_TASK_FLIP) return comet::launch_flip(c, (hipStream_t)stream, L);
  return comet::launch_evaluate(c, (hipStream_t)stream, L);
}

comet_status comet_set_schedule(comet_ctx* c, const comet_schedule* sc) {
  if (!c || !sc || sc->waves_per_cu < 0 || sc->waves_per_cu > 64) return fail(c, COMET_EINVAL, "bad schedule");
  c->sched = *sc;
  return COMET_OK;
}

comet_status comet_get_schedule(const comet_ctx* c, comet_schedule* sc, int32_t* occupancy_waves_per_cu,
                                int32_t* n_cu) {
  if (!c || !sc) return COMET_EINVAL;
  *sc = c->sched;
  if (occupancy_waves_per_cu) *occupancy_waves_per_cu = c->occ_blocks_per_cu;
  if (n_cu) *n_cu = c->n_cu;
  return COMET_OK;
}

comet_status comet_autotune(comet_ctx* c, void* stream, int64_t B, const float* x0, const float* goal,
                            const float* inst, const int32_t* nseg, const int32_t* modes, const int32_t* knots,
                            float* cost, float* viol, uint8_t* feasible, float* traj, int32_t* stats,
                            comet_schedule* best, float* best_ms) {
  if (!c) return COMET_EINVAL;
  hipStream_t s = (hipStream_t)stream;
  hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
  (void)hipStreamIsCapturing(s, &cap);
  if (cap != hipStreamCaptureStatusNone) return fail(c, COMET_ESTATE, "autotune cannot run under stream capture");
  const int occ = c->occ_blocks_per_cu;
  const int mult[3] = {1, 2, 4};
  comet_schedule keep = c->sched, top = keep;
  float top_ms = 1e30f;
  for (int sort = 0; sort < 2; ++sort)
    for (int m = 0; m < 3; ++m) {
      comet_schedule cand{occ * mult[m], sort};
      c->sched = cand;
      comet_status st = comet_evaluate(c, stream, B, x0, goal, inst, nseg, modes, knots, nullptr, 0, cost, viol,
                                        feasible, traj, stats);
      if (st != COMET_OK) {
        c->sched = keep;
        return st;
      }
      if (hipStreamSynchronize(s) != hipSuccess) {
        c->sched = keep;
        return fail(c, COMET_EHIP, "synchronize failed during autotune");
      }
      float ms = 0.f;
      if (hipEventElapsedTime(&ms, c->ev0, c->ev1) != hipSuccess) ms = 1e30f;
      if (ms < top_ms) {
        top_ms = ms;
        top = cand;
      }
    }
  c->sched = top;
  if (best) *best = top;
  if (best_ms) *best_ms = top_ms;
  return COMET_OK;
}

comet_status comet_last_kernel_ms(comet_ctx* c, float* ms) {
  if (!c || !ms) return COMET_EINVAL;
  if (!c->timed) return fail(c, COMET_ESTATE, "last evaluate was captured, not timed");
  if (hipEventElapsedTime(ms, c->ev0, c->ev1) != hipSuccess) return fail(c, COMET_EHIP, "event query failed");
  return COMET_OK;
}

}  // extern "C"
