// push_model.h -- planar pusher-slider task model for the gfx950 evaluator.
//
// One interval k of a mode-conditioned TO (Eq. 2) links x_k, u_k, x_{k+1} through the
// defect d_k = x_{k+1} - F_k(x_k, u_k; m) (Sec. III-C, shared representation) and carries
// the mode's contact rows in fixed positions; rows a mode does not use are masked.
//
// Mechanics (readings of what the paper leaves unstated): square slider of side a, mass
// m, ground friction mu_g, f_max = mu_g m g; ellipsoidal limit surface with the
// uniform-pressure radius c_ls = a (sqrt2 + asinh 1) / 6; quasi-static law: body twist =
// (v_ref / f_max) (F_x, F_y, M / c_ls^2); contact point p = (a/2) n + s t on face j with
// outward normal n at angle j pi/2 and tangent t = (-n_y, n_x); force on the slider
// F = -F_n n + F_t t, so the moment about the centre is M = (a/2) F_t + s F_n; explicit Euler
// with dt = 0.1 s.
//
// State x = (x, y, theta, s), control u = (F_n, F_t, v_s).  Row slots per interval:
//   0..3 defects (slot 3, the contact-coordinate row, is masked on the last interval of a
//        segment whose successor uses another face: the pusher relocates);
//   4    stick: v_s = 0              slide(sigma): F_t - sigma mu F_n = 0
//   5    -F_n <= 0
//   6    stick: F_t - mu F_n <= 0    slide(sigma): -sigma v_s <= 0
//   7    stick: -F_t - mu F_n <= 0   slide: masked
//   8,9  s_{k+1} - a/2 <= 0,  -s_{k+1} - a/2 <= 0
// Terminal rows (x_N, y_N, theta_N) - goal = 0.
// Objective: sum_k dt [ (F_n^2 + F_t^2) / f_max^2 + w_v (v_s / v_ref)^2 ].
#pragma once
#include <hip/hip_runtime.h>

#include <cmath>

#include "dmath.h"

namespace comet {
namespace push {

constexpr int NX = 4, NU = 3, NW = 7, NV = 11, NR = 10, NE = 5, NI = NR - NE, NT = 3;
constexpr int NMODES = 12, NTYPES = 12, NGAIN = NW + NW * NX;
// the forward sweep loads an interval's gains one interval ahead (they stay in registers
// while the trial steps of the current interval run)
constexpr bool PREFETCH_GAINS = true;
constexpr double SIDE = 0.1, MASS = 1.0, GRAV = 9.81, MU_G = 0.5, VREF = 1.0, DT = 0.1, WV = 1.0;
constexpr double FMAX = MU_G * MASS * GRAV;
constexpr double CLS = SIDE * (1.4142135623730951 + 0.88137358701954305) / 6.0;  // sqrt2 + asinh(1)
constexpr double K1 = VREF / FMAX;          // translational gain of the limit surface
constexpr double KM = K1 / (CLS * CLS);     // rotational gain
constexpr double HALF = 0.5 * SIDE;

// column indices of v = (x_k, u_k, x_{k+1})
enum { VX = 0, VY, VTH, VS_, VFN, VFT, VVS, VX1, VY1, VTH1, VS1 };
// row types of the internal scaling
enum { T_DX, T_DY, T_DTH, T_DS, T_STICK, T_SLIDE, T_FN, T_CONE, T_SLIP, T_FACE, T_TXY, T_TTH };

// Union over modes of the structural nonzeros of each row (slot) of the interval Jacobian.
__host__ __device__ constexpr bool nz(int r, int i) {
  return (r == 0) ? (i == VX || i == VTH || i == VFN || i == VFT || i == VX1)
       : (r == 1) ? (i == VY || i == VTH || i == VFN || i == VFT || i == VY1)
       : (r == 2) ? (i == VTH || i == VS_ || i == VFN || i == VFT || i == VTH1)
       : (r == 3) ? (i == VS_ || i == VVS || i == VS1)
       : (r == 4 || r == 6) ? (i == VFN || i == VFT || i == VVS)
       : (r == 5) ? (i == VFN)
       : (r == 7) ? (i == VFN || i == VFT)
       : (i == VS1);
}

// Mode code of an interval: bits 0-1 face, bits 2-3 slip (0 stick, 1 slide+, 2 slide-),
// bit 4 set when the contact-coordinate defect is enabled.
__host__ __device__ inline int make_code(int mode, int smask) { return (mode / 3) | ((mode % 3) << 2) | (smask << 4); }

template <typename T>
__host__ __device__ inline void face_dirs(int f, T& nx, T& ny) {
  nx = T((f == 0) - (f == 2));
  ny = T((f == 1) - (f == 3));
}

// Row residuals (physical units) in double and, if J != nullptr, the Jacobian in T
// precision laid out densely over the 11 columns (only the nz() entries are written);
// en[r] = 1 if the row is enabled.  The residuals, including the trigonometric terms of
// the nonlinear increment F_k, are always evaluated in double: near a solution the solver
// divides them by the penalty parameter, so their rounding error sets the floor of the
// stationarity measure.
template <typename T>
__host__ __device__ inline void rows_sc(const double* xk, const double* uk, const double* x1, int code, double mu,
                                        double st, double ct, double* c, T (*J)[NV], int* en);

// rows() with sin and cos of theta_k computed here
template <typename T>
__host__ __device__ inline void rows(const double* xk, const double* uk, const double* x1, int code, double mu,
                                     double* c, T (*J)[NV], int* en) {
  double st, ct;
  sincos_d(xk[2], &st, &ct);
  rows_sc<T>(xk, uk, x1, code, mu, st, ct, c, J, en);
}

// rows() given st = sin(theta_k), ct = cos(theta_k)
template <typename T>
__host__ __device__ inline void rows_sc(const double* xk, const double* uk, const double* x1, int code, double mu,
                                        double st, double ct, double* c, T (*J)[NV], int* en) {
  const int face = code & 3, slip = (code >> 2) & 3, smask = (code >> 4) & 1;
  const bool stick = (slip == 0);
  const double sg = (slip == 1) ? 1.0 : ((slip == 2) ? -1.0 : 0.0);
  double nx, ny;
  face_dirs<double>(face, nx, ny);
  const double tx = -ny, ty = nx;
  const double th = xk[2], s = xk[3], Fn = uk[0], Ft = uk[1];
  const double Fbx = -Fn * nx + Ft * tx, Fby = -Fn * ny + Ft * ty;
  const double M = HALF * Ft + s * Fn;
  (void)th;
  const double xi_x = K1 * Fbx, xi_y = K1 * Fby, xi_t = KM * M;
  const double vx = ct * xi_x - st * xi_y, vy = st * xi_x + ct * xi_y;
  c[0] = (x1[0] - xk[0]) - DT * vx;
  c[1] = (x1[1] - xk[1]) - DT * vy;
  c[2] = (x1[2] - xk[2]) - DT * xi_t;
  c[3] = smask ? (x1[3] - xk[3]) - DT * uk[2] : 0.0;
  c[4] = stick ? uk[2] : uk[1] - sg * mu * uk[0];
  c[5] = -uk[0];
  c[6] = stick ? uk[1] - mu * uk[0] : -sg * uk[2];
  c[7] = stick ? -uk[1] - mu * uk[0] : 0.0;
  c[8] = x1[3] - HALF;
  c[9] = -x1[3] - HALF;
  en[0] = en[1] = en[2] = 1;
  en[3] = smask;
  en[4] = en[5] = en[6] = 1;
  en[7] = stick ? 1 : 0;
  en[8] = en[9] = 1;
  if (J) {
    const T k1 = T(K1), km = T(KM), dt = T(DT), half = T(HALF);
    const T stT = T(st), ctT = T(ct), nxT = T(nx), nyT = T(ny), txT = T(tx), tyT = T(ty);
    const T muT = T(mu), sgT = T(sg), vxT = T(vx), vyT = T(vy), FnT = T(Fn), sT = T(s);
    const T dvx_dFn = k1 * (ctT * (-nxT) - stT * (-nyT)), dvy_dFn = k1 * (stT * (-nxT) + ctT * (-nyT));
    const T dvx_dFt = k1 * (ctT * txT - stT * tyT), dvy_dFt = k1 * (stT * txT + ctT * tyT);
    J[0][VX] = T(-1); J[0][VTH] = dt * vyT; J[0][VFN] = -dt * dvx_dFn; J[0][VFT] = -dt * dvx_dFt; J[0][VX1] = T(1);
    J[1][VY] = T(-1); J[1][VTH] = -dt * vxT; J[1][VFN] = -dt * dvy_dFn; J[1][VFT] = -dt * dvy_dFt; J[1][VY1] = T(1);
    J[2][VTH] = T(-1); J[2][VS_] = -dt * km * FnT; J[2][VFN] = -dt * km * sT; J[2][VFT] = -dt * km * half;
    J[2][VTH1] = T(1);
    const T sm = smask ? T(1) : T(0);
    J[3][VS_] = -sm; J[3][VVS] = -dt * sm; J[3][VS1] = sm;
    J[4][VFN] = stick ? T(0) : -sgT * muT; J[4][VFT] = stick ? T(0) : T(1); J[4][VVS] = stick ? T(1) : T(0);
    J[5][VFN] = T(-1);
    J[6][VFN] = stick ? -muT : T(0); J[6][VFT] = stick ? T(1) : T(0); J[6][VVS] = stick ? T(0) : -sgT;
    J[7][VFN] = stick ? -muT : T(0); J[7][VFT] = stick ? T(-1) : T(0);
    J[8][VS1] = T(1);
    J[9][VS1] = T(-1);
  }
}

// row type of each slot for the scaling; depends only on stick / slide
__host__ __device__ inline int row_type(int r, bool stick) {
  switch (r) {
    case 0: return T_DX;
    case 1: return T_DY;
    case 2: return T_DTH;
    case 3: return T_DS;
    case 4: return stick ? T_STICK : T_SLIDE;
    case 5: return T_FN;
    case 6: return stick ? T_CONE : T_SLIP;
    case 7: return T_CONE;
    default: return T_FACE;
  }
}

// stage cost and its gradient / constant diagonal Hessian w.r.t. u
__host__ __device__ inline double stage_cost(const double* u) {
  return DT * ((u[0] * u[0] + u[1] * u[1]) / (FMAX * FMAX) + WV * u[2] * u[2] / (VREF * VREF));
}
constexpr double HF = DT * 2.0 / (FMAX * FMAX), HV = DT * 2.0 * WV / (VREF * VREF);

// cost gradient added into the gradient over v, and the (constant) cost Hessian into the
// lower triangle of the block over v
__host__ __device__ inline void add_cost_grad(const double* u, double* h) {
  h[VFN] += HF * u[0];
  h[VFT] += HF * u[1];
  h[VVS] += HV * u[2];
}
__host__ __device__ inline void add_cost_hess(const double* u, double (*G)[NV]) {
  (void)u;
  G[VFN][VFN] += HF;
  G[VFT][VFT] += HF;
  G[VVS][VVS] += HV;
}

// schedule-derived initial controls: normal force fn, tangential force on the cone edge
// (sg = +-1 sliding, 0 sticking), no slip
__host__ __device__ inline void initial_u(double fn, double sg, double mu, double* u) {
  u[0] = fn;
  u[1] = sg * mu * fn;
  u[2] = 0.0;
}

}  // namespace push

// --------------------------------------------------------------------------------------
// Optimised timing (Sec. III-C: the interval durations become controls; the pushing
// configuration of Sec. IV-A optimises the time step under a duration bound).  Readings:
// the duration h_k of every interval is a fourth control, bounded per interval by
// h_min <= h_k <= h_max, every defect steps by h_k instead of dt, and the objective
// charges sum_k h_k [ (F_n^2 + F_t^2) / f_max^2 + w_v (v_s / v_ref)^2 + w_T ].  Its
// Hessian model keeps the exact force/velocity block 2 h diag(...) (at max(h, h_min / 2))
// and drops the (u, h) and (h, h) entries, with which the exact Hessian is indefinite;
// the duration direction takes its curvature from the rows and the proximal term.
// Rows 0..9 are those of the fixed-step model; rows 10, 11 are h - h_max <= 0 and
// h_min - h <= 0.
// --------------------------------------------------------------------------------------
namespace push_timed {

constexpr int NX = 4, NU = 4, NW = 8, NV = 12, NR = 12, NE = 5, NI = NR - NE, NT = 3;
constexpr int NMODES = 12, NTYPES = 13, NGAIN = NW + NW * NX;
// the larger stage leaves no registers for gains in flight (prefetched, they spilled in
// the trial loop and cost 20 % of the kernel time): they are loaded at use
constexpr bool PREFETCH_GAINS = false;
using push::SIDE;
using push::MASS;
using push::GRAV;
using push::MU_G;
using push::VREF;
using push::DT;
using push::WV;
using push::FMAX;
using push::CLS;
using push::K1;
using push::KM;
using push::HALF;
using push::make_code;
using push::face_dirs;
constexpr double H_MIN = 0.02, H_MAX = 0.2, W_T = 0.01;

// column indices of v = (x_k, u_k, x_{k+1}), u_k = (F_n, F_t, v_s, h)
enum { VX = 0, VY, VTH, VS_, VFN, VFT, VVS, VH, VX1, VY1, VTH1, VS1 };
// row types of the internal scaling: those of the fixed-step model, then the duration rows
enum { T_DX, T_DY, T_DTH, T_DS, T_STICK, T_SLIDE, T_FN, T_CONE, T_SLIP, T_FACE, T_TXY, T_TTH, T_DUR };

__host__ __device__ constexpr bool nz(int r, int i) {
  return (r == 0) ? (i == VX || i == VTH || i == VFN || i == VFT || i == VH || i == VX1)
       : (r == 1) ? (i == VY || i == VTH || i == VFN || i == VFT || i == VH || i == VY1)
       : (r == 2) ? (i == VTH || i == VS_ || i == VFN || i == VFT || i == VH || i == VTH1)
       : (r == 3) ? (i == VS_ || i == VVS || i == VH || i == VS1)
       : (r == 4 || r == 6) ? (i == VFN || i == VFT || i == VVS)
       : (r == 5) ? (i == VFN)
       : (r == 7) ? (i == VFN || i == VFT)
       : (r == 8 || r == 9) ? (i == VS1)
       : (i == VH);
}

template <typename T>
__host__ __device__ inline void rows_sc(const double* xk, const double* uk, const double* x1, int code, double mu,
                                        double st, double ct, double* c, T (*J)[NV], int* en) {
  const int face = code & 3, slip = (code >> 2) & 3, smask = (code >> 4) & 1;
  const bool stick = (slip == 0);
  const double sg = (slip == 1) ? 1.0 : ((slip == 2) ? -1.0 : 0.0);
  double nx, ny;
  face_dirs<double>(face, nx, ny);
  const double tx = -ny, ty = nx;
  const double s = xk[3], Fn = uk[0], Ft = uk[1], h = uk[3];
  const double Fbx = -Fn * nx + Ft * tx, Fby = -Fn * ny + Ft * ty;
  const double M = HALF * Ft + s * Fn;
  const double xi_x = K1 * Fbx, xi_y = K1 * Fby, xi_t = KM * M;
  const double vx = ct * xi_x - st * xi_y, vy = st * xi_x + ct * xi_y;
  c[0] = (x1[0] - xk[0]) - h * vx;
  c[1] = (x1[1] - xk[1]) - h * vy;
  c[2] = (x1[2] - xk[2]) - h * xi_t;
  c[3] = smask ? (x1[3] - xk[3]) - h * uk[2] : 0.0;
  c[4] = stick ? uk[2] : uk[1] - sg * mu * uk[0];
  c[5] = -uk[0];
  c[6] = stick ? uk[1] - mu * uk[0] : -sg * uk[2];
  c[7] = stick ? -uk[1] - mu * uk[0] : 0.0;
  c[8] = x1[3] - HALF;
  c[9] = -x1[3] - HALF;
  c[10] = h - H_MAX;
  c[11] = H_MIN - h;
  en[0] = en[1] = en[2] = 1;
  en[3] = smask;
  en[4] = en[5] = en[6] = 1;
  en[7] = stick ? 1 : 0;
  en[8] = en[9] = en[10] = en[11] = 1;
  if (J) {
    const T k1 = T(K1), km = T(KM), hT = T(h), half = T(HALF);
    const T stT = T(st), ctT = T(ct), nxT = T(nx), nyT = T(ny), txT = T(tx), tyT = T(ty);
    const T muT = T(mu), sgT = T(sg), vxT = T(vx), vyT = T(vy), FnT = T(Fn), sT = T(s);
    const T dvx_dFn = k1 * (ctT * (-nxT) - stT * (-nyT)), dvy_dFn = k1 * (stT * (-nxT) + ctT * (-nyT));
    const T dvx_dFt = k1 * (ctT * txT - stT * tyT), dvy_dFt = k1 * (stT * txT + ctT * tyT);
    J[0][VX] = T(-1); J[0][VTH] = hT * vyT; J[0][VFN] = -hT * dvx_dFn; J[0][VFT] = -hT * dvx_dFt;
    J[0][VH] = -vxT; J[0][VX1] = T(1);
    J[1][VY] = T(-1); J[1][VTH] = -hT * vxT; J[1][VFN] = -hT * dvy_dFn; J[1][VFT] = -hT * dvy_dFt;
    J[1][VH] = -vyT; J[1][VY1] = T(1);
    J[2][VTH] = T(-1); J[2][VS_] = -hT * km * FnT; J[2][VFN] = -hT * km * sT; J[2][VFT] = -hT * km * half;
    J[2][VH] = -T(xi_t); J[2][VTH1] = T(1);
    const T sm = smask ? T(1) : T(0);
    J[3][VS_] = -sm; J[3][VVS] = -hT * sm; J[3][VH] = -sm * T(uk[2]); J[3][VS1] = sm;
    J[4][VFN] = stick ? T(0) : -sgT * muT; J[4][VFT] = stick ? T(0) : T(1); J[4][VVS] = stick ? T(1) : T(0);
    J[5][VFN] = T(-1);
    J[6][VFN] = stick ? -muT : T(0); J[6][VFT] = stick ? T(1) : T(0); J[6][VVS] = stick ? T(0) : -sgT;
    J[7][VFN] = stick ? -muT : T(0); J[7][VFT] = stick ? T(-1) : T(0);
    J[8][VS1] = T(1);
    J[9][VS1] = T(-1);
    J[10][VH] = T(1);
    J[11][VH] = T(-1);
  }
}

template <typename T>
__host__ __device__ inline void rows(const double* xk, const double* uk, const double* x1, int code, double mu,
                                     double* c, T (*J)[NV], int* en) {
  double st, ct;
  sincos_d(xk[2], &st, &ct);
  rows_sc<T>(xk, uk, x1, code, mu, st, ct, c, J, en);
}

__host__ __device__ inline int row_type(int r, bool stick) { return r >= 10 ? T_DUR : push::row_type(r, stick); }

constexpr double CF = 1.0 / (FMAX * FMAX), CV = WV / (VREF * VREF);

__host__ __device__ inline double stage_cost(const double* u) {
  return u[3] * ((u[0] * u[0] + u[1] * u[1]) * CF + CV * u[2] * u[2] + W_T);
}
__host__ __device__ inline void add_cost_grad(const double* u, double* h) {
  h[VFN] += 2.0 * CF * u[3] * u[0];
  h[VFT] += 2.0 * CF * u[3] * u[1];
  h[VVS] += 2.0 * CV * u[3] * u[2];
  h[VH] += (u[0] * u[0] + u[1] * u[1]) * CF + CV * u[2] * u[2] + W_T;
}
__host__ __device__ inline void add_cost_hess(const double* u, double (*G)[NV]) {
  const double he = fmax(u[3], 0.5 * H_MIN);
  G[VFN][VFN] += 2.0 * CF * he;
  G[VFT][VFT] += 2.0 * CF * he;
  G[VVS][VVS] += 2.0 * CV * he;
}
__host__ __device__ inline void initial_u(double fn, double sg, double mu, double* u) {
  push::initial_u(fn, sg, mu, u);
  u[3] = DT;
}

}  // namespace push_timed
}  // namespace comet
