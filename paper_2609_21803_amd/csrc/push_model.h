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

// row type of slot r for an interval's mode code (the solver's lookup of the row scale)
__host__ __device__ inline int rtype(int r, int code) { return row_type(r, ((code >> 2) & 3) == 0); }

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
__host__ __device__ inline int rtype(int r, int code) { return row_type(r, ((code >> 2) & 3) == 0); }

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

// --------------------------------------------------------------------------------------
// Free-motion pushing (the admissible language of Sec. III-A: modes are contact events or
// free motion, and a contact changes faces only through a free-motion segment).  Readings
// of the model: the state adds the point pusher's position p in the slider frame, x = (x,
// y, theta, p_x, p_y); the control is u = (F_n, F_t, v_x, v_y), the contact force and the
// pusher's velocity in the slider frame, and p_{k+1} = p_k + dt v.  The slider moves by the
// quasi-static law of the fixed-step model with the moment M = p x F, which on face j
// (p = (a/2) n + s t) is (a/2) F_t + s F_n.  Mode ids 0..11: contact on face id / 3 with
// slip id % 3; ids 12..15: free motion in front of face id - 12 (the half-plane n . p >=
// a/2).  Mode code: face | kind << 2, kind 0 stick, 1 slide+, 2 slide-, 3 free.
// Row slots (equalities first):
//   0..4  defects (pose and pusher position)
//   contact: 5 n.p_k - a/2 = 0, 6 n.v = 0, 7 stick t.v = 0 | slide F_t - sg mu F_n = 0,
//            8 -F_n <= 0, 9 stick F_t - mu F_n <= 0 | slide -sg t.v <= 0,
//            10 stick -F_t - mu F_n <= 0, 11, 12 +-t.p_{k+1} - a/2 <= 0, 13, 14 +-t.p_k - a/2 <= 0
//   free:    5 F_n = 0, 6 F_t = 0, 8 a/2 - n.p_k <= 0, 9 a/2 - n.p_{k+1} <= 0 (no penetration)
// Terminal rows (x_N, y_N, theta_N) - goal = 0.  Objective sum_k dt [ (F_n^2 + F_t^2) /
// f_max^2 + w_v |v|^2 / v_ref^2 ].
// --------------------------------------------------------------------------------------
namespace push_free {

constexpr int NX = 5, NU = 4, NW = 9, NV = 14, NR = 15, NE = 8, NI = NR - NE, NT = 3;
constexpr int NMODES = 16, NTYPES = 16, NGAIN = NW + NW * NX;
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
using push::face_dirs;
constexpr double DFREE = 0.02;   // initial guess: a free segment's knots this far in front of its face

enum { VX = 0, VY, VTH, VPX, VPY, VFN, VFT, VVX, VVY, VX1, VY1, VTH1, VPX1, VPY1 };
// row types of the internal scaling (n.p - a/2 and n.v share one)
enum { T_DX, T_DY, T_DTH, T_DPX, T_DPY, T_ONF, T_STICK, T_SLIDE, T_FREEF, T_FN, T_CONE, T_SLIP, T_NPEN, T_FACE,
       T_TXY, T_TTH };

__host__ __device__ inline int make_code(int mode, int smask) {
  (void)smask;
  return mode < 12 ? (mode / 3) | ((mode % 3) << 2) : (mode - 12) | (3 << 2);
}

__host__ __device__ constexpr bool nz(int r, int i) {
  return (r == 0) ? (i == VX || i == VTH || i == VFN || i == VFT || i == VX1)
       : (r == 1) ? (i == VY || i == VTH || i == VFN || i == VFT || i == VY1)
       : (r == 2) ? (i == VTH || i == VPX || i == VPY || i == VFN || i == VFT || i == VTH1)
       : (r == 3) ? (i == VPX || i == VVX || i == VPX1)
       : (r == 4) ? (i == VPY || i == VVY || i == VPY1)
       : (r == 5 || r == 8) ? (i == VPX || i == VPY || i == VFN)
       : (r == 6) ? (i == VVX || i == VVY || i == VFT)
       : (r == 7) ? (i == VVX || i == VVY || i == VFN || i == VFT)
       : (r == 9) ? (i == VPX1 || i == VPY1 || i == VVX || i == VVY || i == VFN || i == VFT)
       : (r == 10) ? (i == VFN || i == VFT)
       : (r == 11 || r == 12) ? (i == VPX1 || i == VPY1)
       : (i == VPX || i == VPY);
}

// residuals in double, the Jacobian (every structural entry of the union, zeros where the
// mode has none) in T
template <typename T>
__host__ __device__ inline void rows_sc(const double* xk, const double* uk, const double* x1, int code, double mu,
                                        double st, double ct, double* c, T (*J)[NV], int* en) {
  const int face = code & 3, kind = (code >> 2) & 3;
  const bool fr = (kind == 3), stick = (kind == 0);
  const double sg = (kind == 1) ? 1.0 : ((kind == 2) ? -1.0 : 0.0);
  double nx, ny;
  face_dirs<double>(face, nx, ny);
  const double tx = -ny, ty = nx;
  const double px = xk[3], py = xk[4], Fn = uk[0], Ft = uk[1], vx = uk[2], vy = uk[3];
  const double px1 = x1[3], py1 = x1[4];
  const double Fbx = -Fn * nx + Ft * tx, Fby = -Fn * ny + Ft * ty;
  const double M = px * Fby - py * Fbx;
  const double xi_x = K1 * Fbx, xi_y = K1 * Fby, xi_t = KM * M;
  const double wx = ct * xi_x - st * xi_y, wy = st * xi_x + ct * xi_y;
  const double pn = nx * px + ny * py, pt = tx * px + ty * py;
  const double p1n = nx * px1 + ny * py1, p1t = tx * px1 + ty * py1;
  const double vn = nx * vx + ny * vy, vt = tx * vx + ty * vy;
  c[0] = (x1[0] - xk[0]) - DT * wx;
  c[1] = (x1[1] - xk[1]) - DT * wy;
  c[2] = (x1[2] - xk[2]) - DT * xi_t;
  c[3] = (px1 - px) - DT * vx;
  c[4] = (py1 - py) - DT * vy;
  c[5] = fr ? Fn : pn - HALF;
  c[6] = fr ? Ft : vn;
  c[7] = fr ? 0.0 : (stick ? vt : Ft - sg * mu * Fn);
  c[8] = fr ? HALF - pn : -Fn;
  c[9] = fr ? HALF - p1n : (stick ? Ft - mu * Fn : -sg * vt);
  c[10] = (!fr && stick) ? -Ft - mu * Fn : 0.0;
  c[11] = fr ? 0.0 : p1t - HALF;
  c[12] = fr ? 0.0 : -p1t - HALF;
  c[13] = fr ? 0.0 : pt - HALF;
  c[14] = fr ? 0.0 : -pt - HALF;
  en[0] = en[1] = en[2] = en[3] = en[4] = en[5] = en[6] = 1;
  en[7] = fr ? 0 : 1;
  en[8] = en[9] = 1;
  en[10] = (!fr && stick) ? 1 : 0;
  en[11] = en[12] = en[13] = en[14] = fr ? 0 : 1;
  if (J) {
    const T k1 = T(K1), km = T(KM), dt = T(DT), one = T(1), zero = T(0);
    const T stT = T(st), ctT = T(ct), nxT = T(nx), nyT = T(ny), txT = T(tx), tyT = T(ty);
    const T muT = T(mu), sgT = T(sg), wxT = T(wx), wyT = T(wy), FbxT = T(Fbx), FbyT = T(Fby);
    const T pxT = T(px), pyT = T(py);
    const T dwx_dFn = k1 * (ctT * (-nxT) - stT * (-nyT)), dwy_dFn = k1 * (stT * (-nxT) + ctT * (-nyT));
    const T dwx_dFt = k1 * (ctT * txT - stT * tyT), dwy_dFt = k1 * (stT * txT + ctT * tyT);
    J[0][VX] = -one; J[0][VTH] = dt * wyT; J[0][VFN] = -dt * dwx_dFn; J[0][VFT] = -dt * dwx_dFt; J[0][VX1] = one;
    J[1][VY] = -one; J[1][VTH] = -dt * wxT; J[1][VFN] = -dt * dwy_dFn; J[1][VFT] = -dt * dwy_dFt; J[1][VY1] = one;
    J[2][VTH] = -one; J[2][VPX] = -dt * km * FbyT; J[2][VPY] = dt * km * FbxT;
    J[2][VFN] = -dt * km * (-pxT * nyT + pyT * nxT); J[2][VFT] = -dt * km * (pxT * tyT - pyT * txT);
    J[2][VTH1] = one;
    J[3][VPX] = -one; J[3][VVX] = -dt; J[3][VPX1] = one;
    J[4][VPY] = -one; J[4][VVY] = -dt; J[4][VPY1] = one;
    J[5][VPX] = fr ? zero : nxT; J[5][VPY] = fr ? zero : nyT; J[5][VFN] = fr ? one : zero;
    J[6][VVX] = fr ? zero : nxT; J[6][VVY] = fr ? zero : nyT; J[6][VFT] = fr ? one : zero;
    J[7][VVX] = (!fr && stick) ? txT : zero; J[7][VVY] = (!fr && stick) ? tyT : zero;
    J[7][VFN] = (!fr && !stick) ? -sgT * muT : zero; J[7][VFT] = (!fr && !stick) ? one : zero;
    J[8][VPX] = fr ? -nxT : zero; J[8][VPY] = fr ? -nyT : zero; J[8][VFN] = fr ? zero : -one;
    J[9][VPX1] = fr ? -nxT : zero; J[9][VPY1] = fr ? -nyT : zero;
    J[9][VVX] = (!fr && !stick) ? -sgT * txT : zero; J[9][VVY] = (!fr && !stick) ? -sgT * tyT : zero;
    J[9][VFN] = (!fr && stick) ? -muT : zero; J[9][VFT] = (!fr && stick) ? one : zero;
    J[10][VFN] = (!fr && stick) ? -muT : zero; J[10][VFT] = (!fr && stick) ? -one : zero;
    J[11][VPX1] = fr ? zero : txT; J[11][VPY1] = fr ? zero : tyT;
    J[12][VPX1] = fr ? zero : -txT; J[12][VPY1] = fr ? zero : -tyT;
    J[13][VPX] = fr ? zero : txT; J[13][VPY] = fr ? zero : tyT;
    J[14][VPX] = fr ? zero : -txT; J[14][VPY] = fr ? zero : -tyT;
  }
}

template <typename T>
__host__ __device__ inline void rows(const double* xk, const double* uk, const double* x1, int code, double mu,
                                     double* c, T (*J)[NV], int* en) {
  double st, ct;
  sincos_d(xk[2], &st, &ct);
  rows_sc<T>(xk, uk, x1, code, mu, st, ct, c, J, en);
}

__host__ __device__ inline int rtype(int r, int code) {
  const int kind = (code >> 2) & 3;
  const bool fr = (kind == 3), stick = (kind == 0);
  switch (r) {
    case 0: return T_DX;
    case 1: return T_DY;
    case 2: return T_DTH;
    case 3: return T_DPX;
    case 4: return T_DPY;
    case 5:
    case 6: return fr ? T_FREEF : T_ONF;
    case 7: return stick ? T_STICK : T_SLIDE;
    case 8: return fr ? T_NPEN : T_FN;
    case 9: return fr ? T_NPEN : (stick ? T_CONE : T_SLIP);
    case 10: return T_CONE;
    default: return T_FACE;
  }
}

constexpr double HF = DT * 2.0 / (FMAX * FMAX), HV = DT * 2.0 * WV / (VREF * VREF);
__host__ __device__ inline double stage_cost(const double* u) {
  return DT * ((u[0] * u[0] + u[1] * u[1]) / (FMAX * FMAX) + WV * (u[2] * u[2] + u[3] * u[3]) / (VREF * VREF));
}
__host__ __device__ inline void add_cost_grad(const double* u, double* h) {
  h[VFN] += HF * u[0];
  h[VFT] += HF * u[1];
  h[VVX] += HV * u[2];
  h[VVY] += HV * u[3];
}
__host__ __device__ inline void add_cost_hess(const double* u, double (*G)[NV]) {
  (void)u;
  G[VFN][VFN] += HF;
  G[VFT][VFT] += HF;
  G[VVX][VVX] += HV;
  G[VVY][VVY] += HV;
}

// Schedule-derived initial guess of one interval (the paper's construction: the pusher is
// placed on each scheduled face during each contact segment): the interval's end knot p1
// at the face centre for contact, DFREE in front of the face for free motion; the velocity
// that moves the pusher from p0 there in one step; F_n = fn with F_t on the cone edge for
// sliding contact, no force in free motion.
__host__ __device__ inline void initial_knot(int code, double fn, double mu, const double* p0, double* u, double* p1) {
  const int face = code & 3, kind = (code >> 2) & 3;
  double nx, ny;
  face_dirs<double>(face, nx, ny);
  const double d = (kind == 3) ? HALF + DFREE : HALF;
  const double sg = (kind == 1) ? 1.0 : ((kind == 2) ? -1.0 : 0.0);
  p1[0] = d * nx;
  p1[1] = d * ny;
  u[0] = (kind == 3) ? 0.0 : fn;
  u[1] = (kind == 3) ? 0.0 : sg * mu * fn;
  u[2] = (p1[0] - p0[0]) / DT;
  u[3] = (p1[1] - p0[1]) / DT;
}

}  // namespace push_free

// --------------------------------------------------------------------------------------
// Free-motion pushing with optimised timing (the paper's pushing transcription: the
// language of Sec. III-A with interval durations as controls, Sec. III-C / IV-A).  The
// free-motion model above with u = (F_n, F_t, v_x, v_y, h): every defect steps by the
// interval's duration h, rows 15, 16 bound it (h_min - h <= 0, h - h_max <= 0; unit rows,
// scaled as the face-bound rows), the objective charges sum_k h [ q(u_k) + w_T ], and the
// Gauss-Newton cost Hessian keeps the force and velocity block only.
// --------------------------------------------------------------------------------------
namespace push_free_timed {

constexpr int NX = 5, NU = 5, NW = 10, NV = 15, NR = 17, NE = 8, NI = NR - NE, NT = 3;
constexpr int NMODES = 16, NTYPES = 16, NGAIN = NW + NW * NX;
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
using push::face_dirs;
constexpr double DFREE = 0.02;   // initial guess: a free segment's knots this far in front of its face
constexpr double H_MIN = 0.02, H_MAX = 0.2, W_T = 0.01;   // duration bounds, time charge

enum { VX = 0, VY, VTH, VPX, VPY, VFN, VFT, VVX, VVY, VH, VX1, VY1, VTH1, VPX1, VPY1 };
// row types of the internal scaling (n.p - a/2 and n.v share one)
enum { T_DX, T_DY, T_DTH, T_DPX, T_DPY, T_ONF, T_STICK, T_SLIDE, T_FREEF, T_FN, T_CONE, T_SLIP, T_NPEN, T_FACE,
       T_TXY, T_TTH };

__host__ __device__ inline int make_code(int mode, int smask) {
  (void)smask;
  return mode < 12 ? (mode / 3) | ((mode % 3) << 2) : (mode - 12) | (3 << 2);
}

__host__ __device__ constexpr bool nz(int r, int i) {
  return (r == 0) ? (i == VX || i == VTH || i == VFN || i == VFT || i == VH || i == VX1)
       : (r == 1) ? (i == VY || i == VTH || i == VFN || i == VFT || i == VH || i == VY1)
       : (r == 2) ? (i == VTH || i == VPX || i == VPY || i == VFN || i == VFT || i == VH || i == VTH1)
       : (r == 3) ? (i == VPX || i == VVX || i == VH || i == VPX1)
       : (r == 4) ? (i == VPY || i == VVY || i == VH || i == VPY1)
       : (r == 5 || r == 8) ? (i == VPX || i == VPY || i == VFN)
       : (r == 6) ? (i == VVX || i == VVY || i == VFT)
       : (r == 7) ? (i == VVX || i == VVY || i == VFN || i == VFT)
       : (r == 9) ? (i == VPX1 || i == VPY1 || i == VVX || i == VVY || i == VFN || i == VFT)
       : (r == 10) ? (i == VFN || i == VFT)
       : (r == 11 || r == 12) ? (i == VPX1 || i == VPY1)
       : (r == 13 || r == 14) ? (i == VPX || i == VPY)
       : (i == VH);
}

// residuals in double, the Jacobian (every structural entry of the union, zeros where the
// mode has none) in T
template <typename T>
__host__ __device__ inline void rows_sc(const double* xk, const double* uk, const double* x1, int code, double mu,
                                        double st, double ct, double* c, T (*J)[NV], int* en) {
  const int face = code & 3, kind = (code >> 2) & 3;
  const bool fr = (kind == 3), stick = (kind == 0);
  const double sg = (kind == 1) ? 1.0 : ((kind == 2) ? -1.0 : 0.0);
  double nx, ny;
  face_dirs<double>(face, nx, ny);
  const double tx = -ny, ty = nx;
  const double px = xk[3], py = xk[4], Fn = uk[0], Ft = uk[1], vx = uk[2], vy = uk[3], h = uk[4];
  const double px1 = x1[3], py1 = x1[4];
  const double Fbx = -Fn * nx + Ft * tx, Fby = -Fn * ny + Ft * ty;
  const double M = px * Fby - py * Fbx;
  const double xi_x = K1 * Fbx, xi_y = K1 * Fby, xi_t = KM * M;
  const double wx = ct * xi_x - st * xi_y, wy = st * xi_x + ct * xi_y;
  const double pn = nx * px + ny * py, pt = tx * px + ty * py;
  const double p1n = nx * px1 + ny * py1, p1t = tx * px1 + ty * py1;
  const double vn = nx * vx + ny * vy, vt = tx * vx + ty * vy;
  c[0] = (x1[0] - xk[0]) - h * wx;
  c[1] = (x1[1] - xk[1]) - h * wy;
  c[2] = (x1[2] - xk[2]) - h * xi_t;
  c[3] = (px1 - px) - h * vx;
  c[4] = (py1 - py) - h * vy;
  c[5] = fr ? Fn : pn - HALF;
  c[6] = fr ? Ft : vn;
  c[7] = fr ? 0.0 : (stick ? vt : Ft - sg * mu * Fn);
  c[8] = fr ? HALF - pn : -Fn;
  c[9] = fr ? HALF - p1n : (stick ? Ft - mu * Fn : -sg * vt);
  c[10] = (!fr && stick) ? -Ft - mu * Fn : 0.0;
  c[11] = fr ? 0.0 : p1t - HALF;
  c[12] = fr ? 0.0 : -p1t - HALF;
  c[13] = fr ? 0.0 : pt - HALF;
  c[14] = fr ? 0.0 : -pt - HALF;
  en[0] = en[1] = en[2] = en[3] = en[4] = en[5] = en[6] = 1;
  en[7] = fr ? 0 : 1;
  en[8] = en[9] = 1;
  en[10] = (!fr && stick) ? 1 : 0;
  en[11] = en[12] = en[13] = en[14] = fr ? 0 : 1;
  c[15] = H_MIN - h;
  c[16] = h - H_MAX;
  en[15] = en[16] = 1;
  if (J) {
    const T k1 = T(K1), km = T(KM), dt = T(h), one = T(1), zero = T(0);
    const T stT = T(st), ctT = T(ct), nxT = T(nx), nyT = T(ny), txT = T(tx), tyT = T(ty);
    const T muT = T(mu), sgT = T(sg), wxT = T(wx), wyT = T(wy), FbxT = T(Fbx), FbyT = T(Fby);
    const T pxT = T(px), pyT = T(py);
    const T dwx_dFn = k1 * (ctT * (-nxT) - stT * (-nyT)), dwy_dFn = k1 * (stT * (-nxT) + ctT * (-nyT));
    const T dwx_dFt = k1 * (ctT * txT - stT * tyT), dwy_dFt = k1 * (stT * txT + ctT * tyT);
    J[0][VX] = -one; J[0][VTH] = dt * wyT; J[0][VFN] = -dt * dwx_dFn; J[0][VFT] = -dt * dwx_dFt; J[0][VX1] = one;
    J[1][VY] = -one; J[1][VTH] = -dt * wxT; J[1][VFN] = -dt * dwy_dFn; J[1][VFT] = -dt * dwy_dFt; J[1][VY1] = one;
    J[2][VTH] = -one; J[2][VPX] = -dt * km * FbyT; J[2][VPY] = dt * km * FbxT;
    J[2][VFN] = -dt * km * (-pxT * nyT + pyT * nxT); J[2][VFT] = -dt * km * (pxT * tyT - pyT * txT);
    J[2][VTH1] = one;
    J[3][VPX] = -one; J[3][VVX] = -dt; J[3][VPX1] = one;
    J[4][VPY] = -one; J[4][VVY] = -dt; J[4][VPY1] = one;
    J[5][VPX] = fr ? zero : nxT; J[5][VPY] = fr ? zero : nyT; J[5][VFN] = fr ? one : zero;
    J[6][VVX] = fr ? zero : nxT; J[6][VVY] = fr ? zero : nyT; J[6][VFT] = fr ? one : zero;
    J[7][VVX] = (!fr && stick) ? txT : zero; J[7][VVY] = (!fr && stick) ? tyT : zero;
    J[7][VFN] = (!fr && !stick) ? -sgT * muT : zero; J[7][VFT] = (!fr && !stick) ? one : zero;
    J[8][VPX] = fr ? -nxT : zero; J[8][VPY] = fr ? -nyT : zero; J[8][VFN] = fr ? zero : -one;
    J[9][VPX1] = fr ? -nxT : zero; J[9][VPY1] = fr ? -nyT : zero;
    J[9][VVX] = (!fr && !stick) ? -sgT * txT : zero; J[9][VVY] = (!fr && !stick) ? -sgT * tyT : zero;
    J[9][VFN] = (!fr && stick) ? -muT : zero; J[9][VFT] = (!fr && stick) ? one : zero;
    J[10][VFN] = (!fr && stick) ? -muT : zero; J[10][VFT] = (!fr && stick) ? -one : zero;
    J[11][VPX1] = fr ? zero : txT; J[11][VPY1] = fr ? zero : tyT;
    J[12][VPX1] = fr ? zero : -txT; J[12][VPY1] = fr ? zero : -tyT;
    J[13][VPX] = fr ? zero : txT; J[13][VPY] = fr ? zero : tyT;
    J[14][VPX] = fr ? zero : -txT; J[14][VPY] = fr ? zero : -tyT;
    // the duration column: each defect steps by h
    J[0][VH] = -wxT; J[1][VH] = -wyT; J[2][VH] = -T(xi_t); J[3][VH] = -T(vx); J[4][VH] = -T(vy);
    J[15][VH] = -one;
    J[16][VH] = one;
  }
}

template <typename T>
__host__ __device__ inline void rows(const double* xk, const double* uk, const double* x1, int code, double mu,
                                     double* c, T (*J)[NV], int* en) {
  double st, ct;
  sincos_d(xk[2], &st, &ct);
  rows_sc<T>(xk, uk, x1, code, mu, st, ct, c, J, en);
}

__host__ __device__ inline int rtype(int r, int code) {
  const int kind = (code >> 2) & 3;
  const bool fr = (kind == 3), stick = (kind == 0);
  switch (r) {
    case 0: return T_DX;
    case 1: return T_DY;
    case 2: return T_DTH;
    case 3: return T_DPX;
    case 4: return T_DPY;
    case 5:
    case 6: return fr ? T_FREEF : T_ONF;
    case 7: return stick ? T_STICK : T_SLIDE;
    case 8: return fr ? T_NPEN : T_FN;
    case 9: return fr ? T_NPEN : (stick ? T_CONE : T_SLIP);
    case 10: return T_CONE;
    default: return T_FACE;
  }
}

constexpr double CF = 1.0 / (FMAX * FMAX), CV = WV / (VREF * VREF);
__host__ __device__ inline double stage_cost(const double* u) {
  return u[4] * ((u[0] * u[0] + u[1] * u[1]) * CF + CV * (u[2] * u[2] + u[3] * u[3]) + W_T);
}
__host__ __device__ inline void add_cost_grad(const double* u, double* h) {
  h[VFN] += 2.0 * CF * u[4] * u[0];
  h[VFT] += 2.0 * CF * u[4] * u[1];
  h[VVX] += 2.0 * CV * u[4] * u[2];
  h[VVY] += 2.0 * CV * u[4] * u[3];
  h[VH] += (u[0] * u[0] + u[1] * u[1]) * CF + CV * (u[2] * u[2] + u[3] * u[3]) + W_T;
}
// Gauss-Newton model of the cost Hessian: the exact force and velocity block 2h diag at
// max(h, h_min / 2), without the (u, h) and (h, h) entries (as the timed pushing model)
__host__ __device__ inline void add_cost_hess(const double* u, double (*G)[NV]) {
  const double he = fmax(u[4], 0.5 * H_MIN);
  G[VFN][VFN] += 2.0 * CF * he;
  G[VFT][VFT] += 2.0 * CF * he;
  G[VVX][VVX] += 2.0 * CV * he;
  G[VVY][VVY] += 2.0 * CV * he;
}

// Schedule-derived initial guess of one interval (the paper's construction: the pusher is
// placed on each scheduled face during each contact segment): the interval's end knot p1
// at the face centre for contact, DFREE in front of the face for free motion; the velocity
// that moves the pusher from p0 there in one step; F_n = fn with F_t on the cone edge for
// sliding contact, no force in free motion.
__host__ __device__ inline void initial_knot(int code, double fn, double mu, const double* p0, double* u, double* p1) {
  const int face = code & 3, kind = (code >> 2) & 3;
  double nx, ny;
  face_dirs<double>(face, nx, ny);
  const double d = (kind == 3) ? HALF + DFREE : HALF;
  const double sg = (kind == 1) ? 1.0 : ((kind == 2) ? -1.0 : 0.0);
  p1[0] = d * nx;
  p1[1] = d * ny;
  u[0] = (kind == 3) ? 0.0 : fn;
  u[1] = (kind == 3) ? 0.0 : sg * mu * fn;
  u[2] = (p1[0] - p0[0]) / DT;
  u[3] = (p1[1] - p0[1]) / DT;
  u[4] = DT;
}

}  // namespace push_free_timed
}  // namespace comet
