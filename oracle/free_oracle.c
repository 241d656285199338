/* free_oracle.c -- FP64 CPU oracle of planar pushing with free-motion segments (the
 * admissible language of Sec. III-A: modes are contact events or free motion, a contact
 * changes faces only through a free-motion segment).  TEST INFRASTRUCTURE ONLY: the
 * tests, the smoke check and the bench's CPU baseline call it; the HIP library never does.
 *
 * Model (readings; the paper states the rules, not this model):
 *   state x = (x, y, theta, p_x, p_y): slider pose in the world and the point pusher's
 *   position in the slider frame; control u = (F_n, F_t, v_x, v_y): contact force (normal,
 *   tangential) and the pusher's velocity in the slider frame.  Square slider, ellipsoidal
 *   limit surface and explicit Euler step as in the pushing task; the moment about the
 *   centre is M = p x F, which on face j (p = (a/2) n + s t) is (a/2) F_t + s F_n.
 *   Modes: ids 0..11 contact on face id/3 with slip id%3 (stick, slide+, slide-); ids
 *   12..15 free motion in region id-12, the half-plane in front of that face.
 *   Rows per interval (slots; equalities first):
 *     0..4  defects x_{k+1} - x_k - dt f(x_k, u_k)
 *     contact:  5 n.p_k - a/2 = 0 ; 6 n.v = 0 ; 7 stick t.v = 0 | slide F_t - sg mu F_n = 0
 *               8 -F_n <= 0 ; 9 stick F_t - mu F_n <= 0 | slide -sg t.v <= 0 ;
 *               10 stick -F_t - mu F_n <= 0 ; 11,12 +-t.p_{k+1} - a/2 <= 0 ;
 *               13,14 +-t.p_k - a/2 <= 0
 *     free:     5 F_n = 0 ; 6 F_t = 0 ; 8 a/2 - n.p_k <= 0 ; 9 a/2 - n.p_{k+1} <= 0
 *   terminal rows (x_N, y_N, theta_N) = goal; the pusher ends anywhere.
 *   Objective sum_k dt [ (F_n^2 + F_t^2) / f_max^2 + w_v |v|^2 / v_ref^2 ].
 * Optimised timing (-DFREE_TIMED): u = (F_n, F_t, v_x, v_y, h) with the duration h of the
 *   interval, every defect steps by h, rows 15, 16: h_min - h <= 0, h - h_max <= 0 (their
 *   unit Jacobian rows share the scale type of the face-bound rows), objective
 *   sum_k h [ ... + w_T ], Gauss-Newton cost Hessian 2 max(h, h_min / 2) on the force and
 *   velocity entries, none on h (as the timed pushing oracle).
 * Solver: the augmented-Lagrangian Gauss-Newton scheme of Sec. III-C with the same
 * readings as the pushing oracle (comet_oracle.c): PHR merit, Riccati recursion with
 * Cholesky and damping retries, backtracking over a fixed number of trial steps, the
 * multiplier / penalty schedule, row scaling by median Jacobian-row norms, Eq. (4) score.
 * Compile: gcc -O2 -ffp-contract=off -fno-fast-math -shared -fPIC -pthread. */
#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define QNX 5
#ifdef FREE_TIMED
/* optimised timing (built as its own library with -DFREE_TIMED): the duration h_k of every  */
/* interval is a fifth control, bounded per interval, and the objective charges time        */
#define QNU 5
#define QNW 10
#define QNV 15
#define QNR 17
#define QNE 8
#define QNI 9
#else
#define QNU 4
#define QNW 9
#define QNV 14
#define QNR 15
#define QNE 8
#define QNI 7
#endif
#define IX1 (QNX + QNU) /* column of x_{k+1} in v = (x_k, u_k, x_{k+1}) */
#define QNT 3
#define QMODES 16
#define MAXSEG 8
#define MAXN 512

static const double Q_A = 0.1, Q_MASS = 1.0, Q_G = 9.81, Q_MUG = 0.5;
static const double Q_VREF = 1.0, Q_DT = 0.1, Q_WV = 1.0;
static const double Q_DFREE = 0.02; /* initial guess: free-motion waypoint this far in front of its face */
#ifdef FREE_TIMED
static const double Q_HMIN = 0.02, Q_HMAX = 0.2, Q_WT = 0.01; /* duration bounds and time charge */
#endif
static double q_fmax(void) { return Q_MUG * Q_MASS * Q_G; }
static double q_cls(void) { return Q_A * (sqrt(2.0) + log(1.0 + sqrt(2.0))) / 6.0; }
static const double QFACE_N[4][2] = {{1, 0}, {0, 1}, {-1, 0}, {0, -1}};

/* row types of the internal scaling (the pusher-on-face rows, n.p - a/2 and n.v, share one) */
enum { T_DX, T_DY, T_DTH, T_DPX, T_DPY, T_ONF, T_STICK, T_SLIDE, T_FREEF, T_FN, T_CONE, T_SLIP, T_NPEN, T_FACE,
       T_TXY, T_TTH, QTYPES };

typedef struct {
  int32_t al_max, gn_max, chol_retries, ls_trials, max_rejects;
  int32_t timed; /* unused here (the layout is the pushing oracle's) */
  double mu0, mu_min, rho0, rho_min, rho_max, armijo_c1;
  double eta_star, omega_star, rc_star, eps_feas;
  double mu0_warm;
  int32_t round32; /* test switch (0 = plain FP64), as in the pushing oracle: rounds to float32 bit 0 the */
                   /* step, bit 1 the multipliers, bit 2 the scaled Jacobians, bit 3 the gains with the */
                   /* forward recursion; results with bits set are perturbations, not the oracle's answer */
} QParams;

typedef struct {
  int N;
  int face[MAXN], kind[MAXN]; /* kind: 0 stick, 1 slide+, 2 slide-, 3 free */
  double mu;
  double x0[QNX], goal[3];
  const double *scale;
  int round_jac; /* test switch: scaled Jacobians rounded to float32 */
  int round_fwd; /* test switch: gains and the forward recursion in float32 */
} QProb;

/* ------------------------------------------------------------------------------ */
/* Rows of one interval in physical units; v = (x_k[5], u_k[4], x_{k+1}[5]).        */
/* ------------------------------------------------------------------------------ */
static void q_rows(int face, int kind, double mu, const double *v, double *c, double J[QNR][QNV], int *en,
                   int *type) {
#ifdef FREE_TIMED
  const double dt = v[9];
#else
  const double dt = Q_DT;
#endif
  const double fmax = q_fmax(), cls2 = q_cls() * q_cls(), k1 = Q_VREF / fmax, h = 0.5 * Q_A;
  const double nx = QFACE_N[face][0], ny = QFACE_N[face][1], tx = -ny, ty = nx;
  const double th = v[2], px = v[3], py = v[4], Fn = v[5], Ft = v[6], vx = v[7], vy = v[8];
  const double px1 = v[IX1 + 3], py1 = v[IX1 + 4];
  const double Fbx = -Fn * nx + Ft * tx, Fby = -Fn * ny + Ft * ty;
  const double M = px * Fby - py * Fbx;
  const double xi_x = k1 * Fbx, xi_y = k1 * Fby, xi_t = k1 * M / cls2;
  const double ct = cos(th), st = sin(th);
  const double wx = ct * xi_x - st * xi_y, wy = st * xi_x + ct * xi_y;
  const double dwx_dFn = k1 * (ct * (-nx) - st * (-ny)), dwy_dFn = k1 * (st * (-nx) + ct * (-ny));
  const double dwx_dFt = k1 * (ct * tx - st * ty), dwy_dFt = k1 * (st * tx + ct * ty);
  const double km = dt * k1 / cls2;
  int r, j;
  for (r = 0; r < QNR; ++r) {
    c[r] = 0.0;
    en[r] = 0;
    type[r] = T_FACE;
    for (j = 0; j < QNV; ++j) J[r][j] = 0.0;
  }
  c[0] = v[IX1] - v[0] - dt * wx;
  J[0][0] = -1; J[0][2] = dt * wy; J[0][5] = -dt * dwx_dFn; J[0][6] = -dt * dwx_dFt; J[0][IX1] = 1;
  c[1] = v[IX1 + 1] - v[1] - dt * wy;
  J[1][1] = -1; J[1][2] = -dt * wx; J[1][5] = -dt * dwy_dFn; J[1][6] = -dt * dwy_dFt; J[1][IX1 + 1] = 1;
  c[2] = v[IX1 + 2] - th - dt * xi_t;
  J[2][2] = -1; J[2][3] = -km * Fby; J[2][4] = km * Fbx; J[2][5] = -km * (-px * ny + py * nx);
  J[2][6] = -km * (px * ty - py * tx); J[2][IX1 + 2] = 1;
  c[3] = px1 - px - dt * vx;
  J[3][3] = -1; J[3][7] = -dt; J[3][IX1 + 3] = 1;
  c[4] = py1 - py - dt * vy;
  J[4][4] = -1; J[4][8] = -dt; J[4][IX1 + 4] = 1;
  en[0] = en[1] = en[2] = en[3] = en[4] = 1;
  type[0] = T_DX; type[1] = T_DY; type[2] = T_DTH; type[3] = T_DPX; type[4] = T_DPY;
#ifdef FREE_TIMED
  J[0][9] = -wx; J[1][9] = -wy; J[2][9] = -xi_t; J[3][9] = -vx; J[4][9] = -vy;
  c[15] = Q_HMIN - dt; J[15][9] = -1; en[15] = 1; type[15] = T_FACE;
  c[16] = dt - Q_HMAX; J[16][9] = 1; en[16] = 1; type[16] = T_FACE;
#endif
  if (kind == 3) {
    c[5] = Fn; J[5][5] = 1; en[5] = 1; type[5] = T_FREEF;
    c[6] = Ft; J[6][6] = 1; en[6] = 1; type[6] = T_FREEF;
    c[8] = h - (nx * px + ny * py); J[8][3] = -nx; J[8][4] = -ny; en[8] = 1; type[8] = T_NPEN;
    c[9] = h - (nx * px1 + ny * py1); J[9][IX1 + 3] = -nx; J[9][IX1 + 4] = -ny; en[9] = 1; type[9] = T_NPEN;
    return;
  }
  c[5] = nx * px + ny * py - h; J[5][3] = nx; J[5][4] = ny; en[5] = 1; type[5] = T_ONF;
  c[6] = nx * vx + ny * vy; J[6][7] = nx; J[6][8] = ny; en[6] = 1; type[6] = T_ONF;
  if (kind == 0) {
    c[7] = tx * vx + ty * vy; J[7][7] = tx; J[7][8] = ty; type[7] = T_STICK;
  } else {
    const double sg = (kind == 1) ? 1.0 : -1.0;
    c[7] = Ft - sg * mu * Fn; J[7][6] = 1; J[7][5] = -sg * mu; type[7] = T_SLIDE;
  }
  en[7] = 1;
  c[8] = -Fn; J[8][5] = -1; en[8] = 1; type[8] = T_FN;
  if (kind == 0) {
    c[9] = Ft - mu * Fn; J[9][6] = 1; J[9][5] = -mu; type[9] = T_CONE;
    c[10] = -Ft - mu * Fn; J[10][6] = -1; J[10][5] = -mu; en[10] = 1; type[10] = T_CONE;
  } else {
    const double sg = (kind == 1) ? 1.0 : -1.0;
    c[9] = -sg * (tx * vx + ty * vy); J[9][7] = -sg * tx; J[9][8] = -sg * ty; type[9] = T_SLIP;
  }
  en[9] = 1;
  c[11] = tx * px1 + ty * py1 - h; J[11][IX1 + 3] = tx; J[11][IX1 + 4] = ty;
  c[12] = -(tx * px1 + ty * py1) - h; J[12][IX1 + 3] = -tx; J[12][IX1 + 4] = -ty;
  c[13] = tx * px + ty * py - h; J[13][3] = tx; J[13][4] = ty;
  c[14] = -(tx * px + ty * py) - h; J[14][3] = -tx; J[14][4] = -ty;
  en[11] = en[12] = en[13] = en[14] = 1;
}

static void q_term(const double *goal, const double *xN, double *c, double J[QNT][QNX], int *type) {
  int r, j;
  for (r = 0; r < QNT; ++r) {
    c[r] = xN[r] - goal[r];
    for (j = 0; j < QNX; ++j) J[r][j] = (r == j) ? 1.0 : 0.0;
  }
  type[0] = T_TXY; type[1] = T_TXY; type[2] = T_TTH;
}

/* stage cost dt q(u), its gradient and (constant, diagonal) Hessian; hu [QNU][QNU] */
static double q_cost(const double *u, double *gu, double hu[QNU][QNU]) {
#ifdef FREE_TIMED
  const double fm2 = q_fmax() * q_fmax(), vr2 = Q_VREF * Q_VREF, dt = u[4], hm = fmax(u[4], 0.5 * Q_HMIN);
  const double q = (u[0] * u[0] + u[1] * u[1]) / fm2 + Q_WV * (u[2] * u[2] + u[3] * u[3]) / vr2 + Q_WT;
  int i, j;
  if (gu) {
    gu[0] = dt * 2.0 * u[0] / fm2;
    gu[1] = dt * 2.0 * u[1] / fm2;
    gu[2] = dt * 2.0 * Q_WV * u[2] / vr2;
    gu[3] = dt * 2.0 * Q_WV * u[3] / vr2;
    gu[4] = q;
  }
  if (hu) {
    for (i = 0; i < QNU; ++i)
      for (j = 0; j < QNU; ++j) hu[i][j] = 0.0;
    hu[0][0] = hu[1][1] = hm * 2.0 / fm2;
    hu[2][2] = hu[3][3] = hm * 2.0 * Q_WV / vr2;
  }
  return dt * q;
#else
  const double fm2 = q_fmax() * q_fmax(), vr2 = Q_VREF * Q_VREF, dt = Q_DT;
  int i, j;
  if (gu) {
    gu[0] = dt * 2.0 * u[0] / fm2;
    gu[1] = dt * 2.0 * u[1] / fm2;
    gu[2] = dt * 2.0 * Q_WV * u[2] / vr2;
    gu[3] = dt * 2.0 * Q_WV * u[3] / vr2;
  }
  if (hu) {
    for (i = 0; i < QNU; ++i)
      for (j = 0; j < QNU; ++j) hu[i][j] = 0.0;
    hu[0][0] = hu[1][1] = dt * 2.0 / fm2;
    hu[2][2] = hu[3][3] = dt * 2.0 * Q_WV / vr2;
  }
  return dt * ((u[0] * u[0] + u[1] * u[1]) / fm2 + Q_WV * (u[2] * u[2] + u[3] * u[3]) / vr2);
#endif
}

/* primal layout z[k*QNW + 0..3] = u_k, z[k*QNW + 4..8] = x_{k+1} */
static void q_args(const QProb *P, const double *z, int k, double *v) {
  int i;
  const double *xk = (k == 0) ? P->x0 : &z[(k - 1) * QNW + QNU];
  for (i = 0; i < QNX; ++i) v[i] = xk[i];
  for (i = 0; i < QNU; ++i) v[QNX + i] = z[k * QNW + i];
  for (i = 0; i < QNX; ++i) v[QNX + QNU + i] = z[k * QNW + QNU + i];
}

static void q_scaled(const QProb *P, const double *z, int k, double *c, double J[QNR][QNV], int *en) {
  double v[QNV];
  int type[QNR], r, j;
  q_args(P, z, k, v);
  q_rows(P->face[k], P->kind[k], P->mu, v, c, J, en, type);
  for (r = 0; r < QNR; ++r) {
    const double sc = P->scale[type[r]];
    c[r] /= sc;
    for (j = 0; j < QNV; ++j) J[r][j] /= sc;
    if (P->round_jac)
      for (j = 0; j < QNV; ++j) J[r][j] = (double)(float)J[r][j];
  }
}

static void q_term_scaled(const QProb *P, const double *z, double *c, double J[QNT][QNX]) {
  int type[QNT], r, j;
  q_term(P->goal, &z[(P->N - 1) * QNW + QNU], c, J, type);
  for (r = 0; r < QNT; ++r) {
    const double sc = P->scale[type[r]];
    c[r] /= sc;
    for (j = 0; j < QNX; ++j) J[r][j] /= sc;
  }
}

typedef struct {
  double *lam, *nu, lamT[QNT];
  double mu;
} QDual;

static double q_merit(const QProb *P, const double *z, const QDual *D) {
  double phi = 0.0, c[QNR], J[QNR][QNV], cT[QNT], JT[QNT][QNX];
  int en[QNR], k, r;
  for (k = 0; k < P->N; ++k) {
    phi += q_cost(&z[k * QNW], NULL, NULL);
    q_scaled(P, z, k, c, J, en);
    for (r = 0; r < QNE; ++r)
      if (en[r]) phi += D->lam[k * QNE + r] * c[r] + c[r] * c[r] / (2.0 * D->mu);
    for (r = QNE; r < QNR; ++r)
      if (en[r]) {
        const double nu = D->nu[k * QNI + (r - QNE)];
        const double t = fmax(nu + c[r] / D->mu, 0.0);
        phi += 0.5 * D->mu * (t * t - nu * nu);
      }
  }
  q_term_scaled(P, z, cT, JT);
  for (r = 0; r < QNT; ++r) phi += D->lamT[r] * cT[r] + cT[r] * cT[r] / (2.0 * D->mu);
  return phi;
}

static double q_weight(int r, int en, double c, double lam, double nu, double mu, int *active) {
  if (!en) {
    *active = 0;
    return 0.0;
  }
  if (r < QNE) {
    *active = 1;
    return lam + c / mu;
  }
  {
    const double t = nu + c / mu;
    *active = (t > 0.0);
    return (t > 0.0) ? t : 0.0;
  }
}

static void q_gradient(const QProb *P, const double *z, const QDual *D, double *g) {
  double c[QNR], J[QNR][QNV], cT[QNT], JT[QNT][QNX], gu[QNU];
  int en[QNR], k, r, j, act;
  memset(g, 0, sizeof(double) * QNW * P->N);
  for (k = 0; k < P->N; ++k) {
    q_cost(&z[k * QNW], gu, NULL);
    for (j = 0; j < QNU; ++j) g[k * QNW + j] += gu[j];
    q_scaled(P, z, k, c, J, en);
    for (r = 0; r < QNR; ++r) {
      const double lam = (r < QNE) ? D->lam[k * QNE + r] : 0.0;
      const double nuv = (r >= QNE) ? D->nu[k * QNI + r - QNE] : 0.0;
      const double w = q_weight(r, en[r], c[r], lam, nuv, D->mu, &act);
      if (w == 0.0) continue;
      if (k > 0)
        for (j = 0; j < QNX; ++j) g[(k - 1) * QNW + QNU + j] += w * J[r][j];
      for (j = 0; j < QNW; ++j) g[k * QNW + j] += w * J[r][QNX + j];
    }
  }
  q_term_scaled(P, z, cT, JT);
  for (r = 0; r < QNT; ++r) {
    const double w = D->lamT[r] + cT[r] / D->mu;
    for (j = 0; j < QNX; ++j) g[(P->N - 1) * QNW + QNU + j] += w * JT[r][j];
  }
}

static int q_cholesky(int n, double *A, int lda) {
  int i, j, k;
  for (j = 0; j < n; ++j) {
    double d = A[j * lda + j];
    for (k = 0; k < j; ++k) d -= A[j * lda + k] * A[j * lda + k];
    if (!(d > 0.0) || !isfinite(d)) return 0;
    d = sqrt(d);
    A[j * lda + j] = d;
    for (i = j + 1; i < n; ++i) {
      double s = A[i * lda + j];
      for (k = 0; k < j; ++k) s -= A[i * lda + k] * A[j * lda + k];
      A[i * lda + j] = s / d;
    }
  }
  return 1;
}

static void q_chol_solve(int n, const double *L, int lda, double *b) {
  int i, k;
  for (i = 0; i < n; ++i) {
    double s = b[i];
    for (k = 0; k < i; ++k) s -= L[i * lda + k] * b[k];
    b[i] = s / L[i * lda + i];
  }
  for (i = n - 1; i >= 0; --i) {
    double s = b[i];
    for (k = i + 1; k < n; ++k) s -= L[k * lda + i] * b[k];
    b[i] = s / L[i * lda + i];
  }
}

/* one regularised Gauss-Newton step by the backward Riccati recursion (see comet_oracle.c) */
static int q_gn_step(const QProb *P, const double *z, const QDual *D, double rho, double *dz) {
  const int N = P->N;
  double Pm[QNX][QNX], pv[QNX];
  double *kk = (double *)malloc(sizeof(double) * N * QNW);
  double *KK = (double *)malloc(sizeof(double) * N * QNW * QNX);
  double c[QNR], J[QNR][QNV], cT[QNT], JT[QNT][QNX], gu[QNU], hu[QNU][QNU];
  int en[QNR], k, r, i, j, act, ok = 1;
  q_term_scaled(P, z, cT, JT);
  for (i = 0; i < QNX; ++i) {
    pv[i] = 0;
    for (j = 0; j < QNX; ++j) Pm[i][j] = 0;
  }
  for (r = 0; r < QNT; ++r) {
    const double w = D->lamT[r] + cT[r] / D->mu;
    for (i = 0; i < QNX; ++i) {
      pv[i] += w * JT[r][i];
      for (j = 0; j < QNX; ++j) Pm[i][j] += JT[r][i] * JT[r][j] / D->mu;
    }
  }
  for (k = N - 1; k >= 0 && ok; --k) {
    double G[QNV][QNV], h[QNV], S[QNW * QNW], rhs[QNW];
    memset(G, 0, sizeof G);
    memset(h, 0, sizeof h);
    q_cost(&z[k * QNW], gu, hu);
    for (i = 0; i < QNU; ++i) {
      h[QNX + i] += gu[i];
      for (j = 0; j < QNU; ++j) G[QNX + i][QNX + j] += hu[i][j];
    }
    q_scaled(P, z, k, c, J, en);
    for (r = 0; r < QNR; ++r) {
      const double lam = (r < QNE) ? D->lam[k * QNE + r] : 0.0;
      const double nuv = (r >= QNE) ? D->nu[k * QNI + r - QNE] : 0.0;
      const double w = q_weight(r, en[r], c[r], lam, nuv, D->mu, &act);
      for (i = 0; i < QNV; ++i) h[i] += w * J[r][i];
      if (act)
        for (i = 0; i < QNV; ++i)
          for (j = 0; j < QNV; ++j) G[i][j] += J[r][i] * J[r][j] / D->mu;
    }
    for (i = 0; i < QNX; ++i) {
      h[QNX + QNU + i] += pv[i];
      for (j = 0; j < QNX; ++j) G[QNX + QNU + i][QNX + QNU + j] += Pm[i][j];
    }
    for (i = 0; i < QNW; ++i)
      for (j = 0; j < QNW; ++j) S[i * QNW + j] = G[QNX + i][QNX + j] + (i == j ? rho : 0.0);
    if (!q_cholesky(QNW, S, QNW)) {
      ok = 0;
      break;
    }
    for (i = 0; i < QNW; ++i) rhs[i] = -h[QNX + i];
    q_chol_solve(QNW, S, QNW, rhs);
    for (i = 0; i < QNW; ++i) kk[k * QNW + i] = rhs[i];
    for (j = 0; j < QNX; ++j) {
      for (i = 0; i < QNW; ++i) rhs[i] = -G[QNX + i][j];
      q_chol_solve(QNW, S, QNW, rhs);
      for (i = 0; i < QNW; ++i) KK[(k * QNW + i) * QNX + j] = rhs[i];
    }
    {
      double Pn[QNX][QNX], pn[QNX];
      for (i = 0; i < QNX; ++i) {
        pn[i] = h[i];
        for (r = 0; r < QNW; ++r) pn[i] += G[i][QNX + r] * kk[k * QNW + r];
        for (j = 0; j < QNX; ++j) {
          Pn[i][j] = G[i][j];
          for (r = 0; r < QNW; ++r) Pn[i][j] += G[i][QNX + r] * KK[(k * QNW + r) * QNX + j];
        }
      }
      for (i = 0; i < QNX; ++i) {
        pv[i] = pn[i];
        for (j = 0; j < QNX; ++j) Pm[i][j] = 0.5 * (Pn[i][j] + Pn[j][i]);
      }
    }
  }
  if (ok && P->round_fwd) {
    float dxf[QNX] = {0, 0, 0, 0, 0};
    for (k = 0; k < N; ++k) {
      for (i = 0; i < QNW; ++i) {
        float s = (float)kk[k * QNW + i];
        for (j = 0; j < QNX; ++j) s += (float)KK[(k * QNW + i) * QNX + j] * dxf[j];
        dz[k * QNW + i] = s;
      }
      for (j = 0; j < QNX; ++j) dxf[j] = (float)dz[k * QNW + QNU + j];
    }
  } else if (ok) {
    double dx[QNX] = {0, 0, 0, 0, 0};
    for (k = 0; k < N; ++k) {
      for (i = 0; i < QNW; ++i) {
        double s = kk[k * QNW + i];
        for (j = 0; j < QNX; ++j) s += KK[(k * QNW + i) * QNX + j] * dx[j];
        dz[k * QNW + i] = s;
      }
      for (j = 0; j < QNX; ++j) dx[j] = dz[k * QNW + QNU + j];
    }
  }
  free(kk);
  free(KK);
  return ok;
}

static void q_scaled_viol(const QProb *P, const double *z, const QDual *D, double *vs, double *rc) {
  double c[QNR], J[QNR][QNV], cT[QNT], JT[QNT][QNX];
  int en[QNR], k, r;
  double v = 0.0, q = 0.0;
  for (k = 0; k < P->N; ++k) {
    q_scaled(P, z, k, c, J, en);
    for (r = 0; r < QNR; ++r) {
      if (!en[r]) continue;
      if (r < QNE) v = fmax(v, fabs(c[r]));
      else {
        const double nu = D->nu[k * QNI + r - QNE];
        v = fmax(v, fmax(c[r], 0.0));
        q = fmax(q, fabs(fmin(-c[r], nu)));
      }
    }
  }
  q_term_scaled(P, z, cT, JT);
  for (r = 0; r < QNT; ++r) v = fmax(v, fabs(cT[r]));
  *vs = v;
  *rc = q;
}

static void q_update_duals(const QProb *P, const double *z, QDual *D) {
  double c[QNR], J[QNR][QNV], cT[QNT], JT[QNT][QNX];
  int en[QNR], k, r;
  for (k = 0; k < P->N; ++k) {
    q_scaled(P, z, k, c, J, en);
    for (r = 0; r < QNR; ++r) {
      if (!en[r]) continue;
      if (r < QNE) D->lam[k * QNE + r] += c[r] / D->mu;
      else {
        double *nu = &D->nu[k * QNI + r - QNE];
        *nu = fmax(*nu + c[r] / D->mu, 0.0);
      }
    }
  }
  q_term_scaled(P, z, cT, JT);
  for (r = 0; r < QNT; ++r) D->lamT[r] += cT[r] / D->mu;
}

/* objective and violation in physical units, Eq. (4) */
static void q_score(const QProb *P, const double *z, double *Jout, double *vout) {
  double c[QNR], J[QNR][QNV], cT[QNT], JT[QNT][QNX], v[QNV];
  int en[QNR], type[QNR], ttype[QNT], k, r;
  double obj = 0.0, vi = 0.0;
  for (k = 0; k < P->N; ++k) {
    obj += q_cost(&z[k * QNW], NULL, NULL);
    q_args(P, z, k, v);
    q_rows(P->face[k], P->kind[k], P->mu, v, c, J, en, type);
    for (r = 0; r < QNR; ++r) {
      if (!en[r]) continue;
      vi = fmax(vi, (r < QNE) ? fabs(c[r]) : fmax(c[r], 0.0));
    }
  }
  q_term(P->goal, &z[(P->N - 1) * QNW + QNU], cT, JT, ttype);
  for (r = 0; r < QNT; ++r) vi = fmax(vi, fabs(cT[r]));
  *Jout = obj;
  *vout = vi;
}

/* Schedule-derived initial guess: the pose interpolated from start to goal; the pusher   */
/* placed on the scheduled face (its centre) during a contact segment and a fixed         */
/* distance in front of the face during a free segment, each knot at its interval's       */
/* place, with the velocity that moves it there in one step; F_n = 0.05 f_max with F_t on  */
/* the cone edge for sliding contact, no force in free motion.                             */
static void q_initial(const QProb *P, double *z) {
  const double fn = 0.05 * q_fmax(), h = 0.5 * Q_A;
  double p[2] = {P->x0[3], P->x0[4]};
  int k, i;
  for (k = 0; k < P->N; ++k) {
    const int f = P->face[k], kind = P->kind[k];
    const double d = (kind == 3) ? h + Q_DFREE : h;
    const double p1x = d * QFACE_N[f][0], p1y = d * QFACE_N[f][1];
    const double t = (double)(k + 1) / (double)P->N;
    const double sg = (kind == 1) ? 1.0 : ((kind == 2) ? -1.0 : 0.0);
    z[k * QNW + 0] = (kind == 3) ? 0.0 : fn;
    z[k * QNW + 1] = (kind == 3) ? 0.0 : sg * P->mu * fn;
    z[k * QNW + 2] = (p1x - p[0]) / Q_DT;
    z[k * QNW + 3] = (p1y - p[1]) / Q_DT;
#ifdef FREE_TIMED
    z[k * QNW + 4] = Q_DT;
#endif
    for (i = 0; i < 3; ++i) z[k * QNW + QNU + i] = P->x0[i] + (P->goal[i] - P->x0[i]) * t;
    z[k * QNW + QNU + 3] = p1x;
    z[k * QNW + QNU + 4] = p1y;
    p[0] = p1x;
    p[1] = p1y;
  }
}

static int q_setup(QProb *P, int nseg, const int32_t *modes, const int32_t *knots, const double *x0,
                   const double *goal, double mu, const double *scale) {
  int j, i, k = 0;
  P->round_jac = 0;
  P->round_fwd = 0;
  if (nseg < 1 || nseg > MAXSEG) return 0;
  for (j = 0; j < nseg; ++j) {
    const int m = modes[j];
    if (m < 0 || m >= QMODES || knots[j] < 1) return 0;
    for (i = 0; i < knots[j]; ++i) {
      if (k >= MAXN) return 0;
      P->face[k] = (m < 12) ? m / 3 : m - 12;
      P->kind[k] = (m < 12) ? m % 3 : 3;
      ++k;
    }
  }
  P->N = k;
  P->mu = mu;
  for (i = 0; i < QNX; ++i) P->x0[i] = x0[i];
  for (i = 0; i < 3; ++i) P->goal[i] = goal[i];
  P->scale = scale;
  if (!isfinite(mu)) return 0;
  for (i = 0; i < QNX; ++i) if (!isfinite(x0[i])) return 0;
  for (i = 0; i < 3; ++i) if (!isfinite(goal[i])) return 0;
  return 1;
}

/* Row scales: for each row type the median 2-norm of its physical Jacobian row over the  */
/* initial guesses of all 256 two-segment orders (5 + 5 intervals), slider at rest at the */
/* origin, pusher at (0, -0.08) in front of face 3, goal (0.1, 0.1, pi/4), friction 0.4;   */
/* median of an even count = mean of the two middle values; terminal rows 1.              */
static int q_cmp(const void *a, const void *b) {
  const double x = *(const double *)a, y = *(const double *)b;
  return (x < y) ? -1 : (x > y) ? 1 : 0;
}
static double g_qscale[QTYPES];
static int g_qscale_ready = 0;
static pthread_mutex_t g_qscale_lock = PTHREAD_MUTEX_INITIALIZER;

static void q_compute_scales(double *out) {
  static double buf[QTYPES][256 * 10 * QNR];     /* at most QNR rows of one type per interval */
  int cnt[QTYPES], t, m1, m2, k, r, j;
  double ones[QTYPES];
  const double x0[QNX] = {0, 0, 0, 0, -0.08}, goal[3] = {0.1, 0.1, M_PI / 4.0};
  for (t = 0; t < QTYPES; ++t) {
    cnt[t] = 0;
    ones[t] = 1.0;
  }
  for (m1 = 0; m1 < QMODES; ++m1)
    for (m2 = 0; m2 < QMODES; ++m2) {
      QProb P;
      int32_t modes[2] = {m1, m2}, knots[2] = {5, 5};
      double z[10 * QNW], v[QNV], c[QNR], J[QNR][QNV];
      int en[QNR], type[QNR];
      q_setup(&P, 2, modes, knots, x0, goal, 0.4, ones);
      q_initial(&P, z);
      for (k = 0; k < P.N; ++k) {
        q_args(&P, z, k, v);
        q_rows(P.face[k], P.kind[k], P.mu, v, c, J, en, type);
        for (r = 0; r < QNR; ++r) {
          double nrm = 0.0;
          if (!en[r]) continue;
          for (j = 0; j < QNV; ++j) nrm += J[r][j] * J[r][j];
          buf[type[r]][cnt[type[r]]++] = sqrt(nrm);
        }
      }
    }
  for (t = 0; t < QTYPES; ++t) {
    const int n = cnt[t];
    if (n == 0) {
      out[t] = 1.0;
      continue;
    }
    qsort(buf[t], (size_t)n, sizeof(double), q_cmp);
    out[t] = (n % 2) ? buf[t][n / 2] : 0.5 * (buf[t][n / 2 - 1] + buf[t][n / 2]);
  }
}

static const double *q_scales(void) {
  pthread_mutex_lock(&g_qscale_lock);
  if (!g_qscale_ready) {
    q_compute_scales(g_qscale);
    g_qscale_ready = 1;
  }
  pthread_mutex_unlock(&g_qscale_lock);
  return g_qscale;
}

typedef struct {
  int al_iters, gn_iters, chol_fails, status;
} QStats;

static int q_finite(const double *a, int n) {
  int i;
  for (i = 0; i < n; ++i)
    if (!isfinite(a[i])) return 0;
  return 1;
}

/* the augmented-Lagrangian outer loop with the Gauss-Newton inner loop */
static void q_solve(const QProb *P, const QParams *prm, int warm, double *z, QStats *st) {
  const int N = P->N, nz = N * QNW;
  double *g = (double *)malloc(sizeof(double) * nz);
  double *dz = (double *)malloc(sizeof(double) * nz);
  double *zt = (double *)malloc(sizeof(double) * nz);
  double *phi = (double *)malloc(sizeof(double) * (size_t)prm->ls_trials);
  QDual D;
  double eta, omega, rho = prm->rho0;
  int al, i;
  D.lam = (double *)calloc((size_t)N * QNE, sizeof(double));
  D.nu = (double *)calloc((size_t)N * QNI, sizeof(double));
  D.lamT[0] = D.lamT[1] = D.lamT[2] = 0.0;
  D.mu = warm ? prm->mu0_warm : prm->mu0;
  eta = pow(D.mu, 0.1);
  omega = D.mu;
  st->al_iters = st->gn_iters = st->chol_fails = 0;
  st->status = 0;
  for (al = 0; al < prm->al_max; ++al) {
    int it, rejects = 0;
    double vs, rc, gnorm;
    st->al_iters = al + 1;
    for (it = 0; it < prm->gn_max; ++it) {
      double phi0, dd;
      int tries = 0, ok, best = -1;
      q_gradient(P, z, &D, g);
      gnorm = 0.0;
      for (i = 0; i < nz; ++i) gnorm = fmax(gnorm, fabs(g[i]));
      if (gnorm <= omega) break;
      phi0 = q_merit(P, z, &D);
      ok = q_gn_step(P, z, &D, rho, dz);
      while (!ok && tries < prm->chol_retries) {
        st->chol_fails++;
        rho = fmax(10.0 * rho, 1e-8);
        ++tries;
        ok = q_gn_step(P, z, &D, rho, dz);
      }
      if (!ok) st->chol_fails++;
      if (ok && (prm->round32 & 1))
        for (i = 0; i < nz; ++i) dz[i] = (double)(float)dz[i];
      st->gn_iters++;
      dd = 0.0;
      if (ok)
        for (i = 0; i < nz; ++i) dd += g[i] * dz[i];
      if (ok && dd < 0.0 && isfinite(phi0)) {
        int t;
        double alpha = 1.0;
        for (t = 0; t < prm->ls_trials; ++t) {
          for (i = 0; i < nz; ++i) zt[i] = z[i] + alpha * dz[i];
          phi[t] = q_merit(P, zt, &D);
          alpha *= 0.5;
        }
        alpha = 1.0;
        for (t = 0; t < prm->ls_trials; ++t) {
          if (isfinite(phi[t]) && phi[t] <= phi0 + prm->armijo_c1 * alpha * dd) {
            best = t;
            break;
          }
          alpha *= 0.5;
        }
        if (best >= 0)
          for (i = 0; i < nz; ++i) z[i] += alpha * dz[i];
      }
      if (best >= 0) {
        rho = fmax(rho / 3.0, prm->rho_min);
        rejects = 0;
      } else {
        rho = fmin(10.0 * rho, prm->rho_max);
        if (++rejects >= prm->max_rejects) break;
      }
    }
    q_scaled_viol(P, z, &D, &vs, &rc);
    q_gradient(P, z, &D, g);
    gnorm = 0.0;
    for (i = 0; i < nz; ++i) gnorm = fmax(gnorm, fabs(g[i]));
    if (!isfinite(vs) || !isfinite(gnorm) || !q_finite(z, nz)) {
      st->status = 2;
      break;
    }
    if (vs <= eta) {
      if (vs <= prm->eta_star && gnorm <= prm->omega_star && rc <= prm->rc_star) {
        st->status = 1;
        break;
      }
      q_update_duals(P, z, &D);
      if (prm->round32 & 2) {
        for (i = 0; i < N * QNE; ++i) D.lam[i] = (double)(float)D.lam[i];
        for (i = 0; i < N * QNI; ++i) D.nu[i] = (double)(float)D.nu[i];
      }
      eta = fmax(eta * pow(D.mu, 0.9), prm->eta_star);
      omega = fmax(omega * D.mu, prm->omega_star);
    } else {
      D.mu = fmax(0.1 * D.mu, prm->mu_min);
      eta = fmax(pow(D.mu, 0.1), prm->eta_star);
      omega = fmax(D.mu, prm->omega_star);
    }
  }
  free(g);
  free(dz);
  free(zt);
  free(phi);
  free(D.lam);
  free(D.nu);
}

/* ------------------------------------------------------------------------------ */
/* Batched evaluation, one sequence per thread.  x0 [B][5] (pose, pusher in the     */
/* slider frame), goal [B][3], inst [B] (pusher friction).  traj [B][nmax+1][QNX+QNU] */
/* rows (x_k, u_k), u_N = 0, rows beyond N zero; stats [B][4].                       */
/* ------------------------------------------------------------------------------ */
typedef struct {
  int64_t B;
  int32_t smax, nmax;
  const double *x0, *goal, *inst, *warm;
  const int32_t *nseg, *modes, *knots;
  const QParams *prm;
  double *cost, *viol, *traj;
  uint8_t *feas;
  int32_t *stats;
  int64_t next;
  pthread_mutex_t lock;
} QJob;

static void q_eval_one(QJob *E, int64_t b) {
  const int rw = QNX + QNU;
  QProb *P = (QProb *)malloc(sizeof(QProb));
  double *z;
  QStats st = {0, 0, 0, 2};
  double J = NAN, v = INFINITY;
  int k, i;
  int ok = q_setup(P, E->nseg[b], &E->modes[b * E->smax], &E->knots[b * E->smax], &E->x0[b * QNX],
                   &E->goal[b * 3], E->inst[b], q_scales());
  if (ok && P->N > E->nmax) ok = 0;
  if (ok) {
    P->round_jac = (E->prm->round32 & 4) != 0;
    P->round_fwd = (E->prm->round32 & 8) != 0;
  }
  if (E->traj) memset(&E->traj[b * (E->nmax + 1) * rw], 0, sizeof(double) * (size_t)(E->nmax + 1) * rw);
  if (!ok) {
    E->cost[b] = NAN;
    E->viol[b] = INFINITY;
    E->feas[b] = 0;
    if (E->stats)
      for (i = 0; i < 4; ++i) E->stats[b * 4 + i] = (i == 3) ? 3 : 0;
    free(P);
    return;
  }
  z = (double *)malloc(sizeof(double) * P->N * QNW);
  if (E->warm) {
    const double *w = &E->warm[b * (E->nmax + 1) * rw];
    for (k = 0; k < P->N; ++k) {
      for (i = 0; i < QNU; ++i) z[k * QNW + i] = w[k * rw + QNX + i];
      for (i = 0; i < QNX; ++i) z[k * QNW + QNU + i] = w[(k + 1) * rw + i];
    }
  } else {
    q_initial(P, z);
  }
  q_solve(P, E->prm, E->warm != NULL, z, &st);
  if (st.status != 2) q_score(P, z, &J, &v);
  if (!isfinite(J) || !isfinite(v)) {
    J = NAN;
    v = INFINITY;
    st.status = 2;
  }
  E->cost[b] = J;
  E->viol[b] = v;
  E->feas[b] = (v <= E->prm->eps_feas) ? 1 : 0;
  if (E->stats) {
    E->stats[b * 4 + 0] = st.al_iters;
    E->stats[b * 4 + 1] = st.gn_iters;
    E->stats[b * 4 + 2] = st.chol_fails;
    E->stats[b * 4 + 3] = st.status;
  }
  if (E->traj) {
    double *T = &E->traj[b * (E->nmax + 1) * rw];
    for (i = 0; i < QNX; ++i) T[i] = P->x0[i];
    for (k = 0; k < P->N; ++k) {
      for (i = 0; i < QNU; ++i) T[k * rw + QNX + i] = z[k * QNW + i];
      for (i = 0; i < QNX; ++i) T[(k + 1) * rw + i] = z[k * QNW + QNU + i];
    }
  }
  free(z);
  free(P);
}

static void *q_worker(void *arg) {
  QJob *E = (QJob *)arg;
  for (;;) {
    int64_t b;
    pthread_mutex_lock(&E->lock);
    b = E->next++;
    pthread_mutex_unlock(&E->lock);
    if (b >= E->B) break;
    q_eval_one(E, b);
  }
  return NULL;
}

int free_evaluate(int64_t B, int32_t smax, int32_t nmax, const double *x0, const double *goal, const double *inst,
                  const int32_t *nseg, const int32_t *modes, const int32_t *knots, const double *warm,
                  const QParams *prm, int32_t nthreads, double *cost, double *viol, uint8_t *feas, double *traj,
                  int32_t *stats) {
  QJob E;
  pthread_t th[256];
  int t;
  if (B < 0 || smax < 1 || smax > MAXSEG || nmax < 1 || nmax > MAXN || !prm) return -1;
  memset(&E, 0, sizeof E);
  E.B = B; E.smax = smax; E.nmax = nmax;
  E.x0 = x0; E.goal = goal; E.inst = inst; E.warm = warm;
  E.nseg = nseg; E.modes = modes; E.knots = knots; E.prm = prm;
  E.cost = cost; E.viol = viol; E.feas = feas; E.traj = traj; E.stats = stats;
  pthread_mutex_init(&E.lock, NULL);
  if (nthreads < 1) nthreads = 1;
  if (nthreads > 256) nthreads = 256;
  if (nthreads == 1 || B <= 1) {
    q_worker(&E);
  } else {
    for (t = 0; t < nthreads; ++t) pthread_create(&th[t], NULL, q_worker, &E);
    for (t = 0; t < nthreads; ++t) pthread_join(th[t], NULL);
  }
  pthread_mutex_destroy(&E.lock);
  return 0;
}

/* ------------------------------------------------------------------------------ */
/* Pins and tests: the model and the solver pieces for one sequence.                */
/* ------------------------------------------------------------------------------ */
int free_scales(double *out) {
  const double *s = q_scales();
  int t;
  for (t = 0; t < QTYPES; ++t) out[t] = s[t];
  return QTYPES;
}

/* rows of one interval at v (physical units): c [15], J [15][14] row-major, en [15], type [15] */
int free_rows(int32_t mode, double mu, const double *v, double *c, double *J, int32_t *en, int32_t *type) {
  double JJ[QNR][QNV];
  int e[QNR], ty[QNR], r, j;
  if (mode < 0 || mode >= QMODES) return -1;
  q_rows(mode < 12 ? mode / 3 : mode - 12, mode < 12 ? mode % 3 : 3, mu, v, c, JJ, e, ty);
  for (r = 0; r < QNR; ++r) {
    en[r] = e[r];
    type[r] = ty[r];
    for (j = 0; j < QNV; ++j) J[r * QNV + j] = JJ[r][j];
  }
  return 0;
}

double free_cost(const double *u, double *gu) { return q_cost(u, gu, NULL); }

int free_initial(int32_t nseg, const int32_t *modes, const int32_t *knots, const double *x0, const double *goal,
                 double mu, double *z) {
  QProb P;
  if (!q_setup(&P, nseg, modes, knots, x0, goal, mu, q_scales())) return -1;
  q_initial(&P, z);
  return P.N;
}

/* Eq. (4) of a given primal z [N*9] */
int free_score(int32_t nseg, const int32_t *modes, const int32_t *knots, const double *x0, const double *goal,
               double mu, const double *z, double *J, double *v) {
  QProb P;
  if (!q_setup(&P, nseg, modes, knots, x0, goal, mu, q_scales())) return -1;
  q_score(&P, z, J, v);
  return 0;
}

/* merit, its gradient and one Gauss-Newton step at (z, lam [N*8], nu [N*7], lamT [3], mu) */
int free_merit_grad_step(int32_t nseg, const int32_t *modes, const int32_t *knots, const double *x0,
                         const double *goal, double mu_f, const double *z, const double *lam, const double *nu,
                         const double *lamT, double mu, double rho, double *phi, double *g, double *dz) {
  QProb P;
  QDual D;
  int ok;
  if (!q_setup(&P, nseg, modes, knots, x0, goal, mu_f, q_scales())) return -1;
  D.lam = (double *)lam;
  D.nu = (double *)nu;
  D.lamT[0] = lamT[0]; D.lamT[1] = lamT[1]; D.lamT[2] = lamT[2];
  D.mu = mu;
  *phi = q_merit(&P, z, &D);
  q_gradient(&P, z, &D, g);
  ok = q_gn_step(&P, z, &D, rho, dz);
  return ok ? 0 : 1;
}

/* ================================================================================ */
/* The admissible language (Sec. III-A) and the greedy expansion's batch step.      */
/* ================================================================================ */
/* Transition rules (reading of the rules Sec. III-A states): no two consecutive      */
/* segments share a mode; a contact keeps its face until a free segment (contact on    */
/* face j may change only its slip); leaving contact on face j enters the free region  */
/* in front of face j, and a contact on face j starts from that region; free regions   */
/* connect to the regions of the neighbouring faces (they overlap at the corners).     */
static int q_step_ok(int a, int b) {
  const int ca = a < 12, cb = b < 12, fa = ca ? a / 3 : a - 12, fb = cb ? b / 3 : b - 12;
  if (a == b) return 0;
  if (ca && cb) return fa == fb;
  if (ca != cb) return fa == fb;
  return ((fb - fa + 4) & 3) == 1 || ((fa - fb + 4) & 3) == 1;
}

int free_admissible(int32_t K, const int32_t *modes) {
  int j;
  if (K < 1 || K > MAXSEG) return 0;
  for (j = 0; j < K; ++j)
    if (modes[j] < 0 || modes[j] >= QMODES) return 0;
  for (j = 1; j < K; ++j)
    if (!q_step_ok(modes[j - 1], modes[j])) return 0;
  return 1;
}

/* keys: K << 60 | m_0 << 56 | m_1 << 52 | ... (4 bits per id, up to 8 segments), so that */
/* comparing keys compares the segment count, then the ids lexicographically             */
typedef uint64_t QKey;
static QKey qkey_make(int K, const int *m) {
  QKey k = (QKey)K << 60;
  int i;
  for (i = 0; i < K; ++i) k |= (QKey)m[i] << (56 - 4 * i);
  return k;
}
static int qkey_len(QKey k) { return (int)(k >> 60); }
static int qkey_mode(QKey k, int i) { return (int)((k >> (56 - 4 * i)) & 15u); }
static int qkey_admissible(QKey k) {
  int32_t m[MAXSEG];
  int K = qkey_len(k), i;
  if (K < 1 || K > MAXSEG) return 0;
  for (i = 0; i < K; ++i) m[i] = qkey_mode(k, i);
  return free_admissible(K, m);
}

typedef struct {
  QKey *slot;
  int64_t cap;
} QSet;
static void qset_init(QSet *S, int64_t n) {
  int64_t c = 16;
  while (c < 2 * n + 16) c <<= 1;
  S->cap = c;
  S->slot = (QKey *)calloc((size_t)c, sizeof(QKey));
}
static uint64_t qmix(uint64_t x) {
  x ^= x >> 33; x *= 0xff51afd7ed558ccdULL;
  x ^= x >> 33; x *= 0xc4ceb9fe1a85ec53ULL;
  x ^= x >> 33;
  return x;
}
static int qset_has(const QSet *S, QKey k) {
  int64_t i = (int64_t)(qmix(k) & (uint64_t)(S->cap - 1));
  while (S->slot[i]) {
    if (S->slot[i] == k) return 1;
    i = (i + 1) & (S->cap - 1);
  }
  return 0;
}
static void qset_add(QSet *S, QKey k) {
  int64_t i = (int64_t)(qmix(k) & (uint64_t)(S->cap - 1));
  while (S->slot[i]) {
    if (S->slot[i] == k) return;
    i = (i + 1) & (S->cap - 1);
  }
  S->slot[i] = k;
}

/* one-edit list in the fixed order: substitutions (position, id ascending), deletions */
/* (K > 1), insertions (position 0..K, id ascending; K < kcap); repeats kept           */
static int64_t qneigh1(QKey p, int kcap, QKey *out) {
  int K = qkey_len(p), m[MAXSEG], q[MAXSEG], i, j, id;
  int64_t n = 0;
  for (i = 0; i < K; ++i) m[i] = qkey_mode(p, i);
  for (i = 0; i < K; ++i)
    for (id = 0; id < QMODES; ++id) {
      if (id == m[i]) continue;
      for (j = 0; j < K; ++j) q[j] = m[j];
      q[i] = id;
      out[n++] = qkey_make(K, q);
    }
  if (K > 1)
    for (i = 0; i < K; ++i) {
      int t = 0;
      for (j = 0; j < K; ++j)
        if (j != i) q[t++] = m[j];
      out[n++] = qkey_make(K - 1, q);
    }
  if (K < kcap)
    for (i = 0; i <= K; ++i)
      for (id = 0; id < QMODES; ++id) {
        int t = 0;
        for (j = 0; j < i; ++j) q[t++] = m[j];
        q[t++] = id;
        for (j = i; j < K; ++j) q[t++] = m[j];
        out[n++] = qkey_make(K + 1, q);
      }
  return n;
}

/* r-edit neighbourhood (r in {1, 2}, Sec. III-B): the one-edit list, then the one-edit */
/* lists of its admissible entries in order (every intermediate order stays in the     */
/* language); first occurrence wins, the order itself excluded; admissible orders only */
static int64_t qneigh(QKey p, int kcap, int r, QKey *out) {
  const int64_t cap1 = (int64_t)(2 * kcap + 2) * QMODES + 16;
  QKey *l1 = (QKey *)malloc(sizeof(QKey) * (size_t)cap1);
  QKey *l2 = (QKey *)malloc(sizeof(QKey) * (size_t)cap1);
  int64_t n1 = qneigh1(p, kcap, l1), n = 0, i, j;
  QSet seen;
  qset_init(&seen, (r >= 2) ? n1 * cap1 + n1 : n1);
  qset_add(&seen, p);
  for (i = 0; i < n1; ++i)
    if (!qset_has(&seen, l1[i])) {
      qset_add(&seen, l1[i]);
      if (qkey_admissible(l1[i])) out[n++] = l1[i];
    }
  if (r >= 2)
    for (i = 0; i < n1; ++i) {
      int64_t n2;
      if (!qkey_admissible(l1[i])) continue;
      n2 = qneigh1(l1[i], kcap, l2);
      for (j = 0; j < n2; ++j)
        if (!qset_has(&seen, l2[j])) {
          qset_add(&seen, l2[j]);
          if (qkey_admissible(l2[j])) out[n++] = l2[j];
        }
    }
  free(l1);
  free(l2);
  free(seen.slot);
  return n;
}

int64_t free_neighbours(uint64_t key, int32_t kcap, int32_t radius, uint64_t *out) {
  return qneigh((QKey)key, kcap, radius, (QKey *)out);
}

/* seed: the admissible orders of 1..kmax segments in key order, at most cap.  For each  */
/* length, a depth-first walk that tries the ids of every position in ascending order   */
/* and extends only admissible prefixes (the product space of eight segments, 16^8      */
/* orders, is too large to filter)                                                      */
static void q_seed_walk(int K, int d, int *q, int64_t cap, int64_t *n, uint64_t *out) {
  int id;
  if (d == K) {
    if (*n < cap) out[(*n)++] = qkey_make(K, q);
    return;
  }
  for (id = 0; id < QMODES && *n < cap; ++id) {
    if (d > 0 && !q_step_ok(q[d - 1], id)) continue;
    q[d] = id;
    q_seed_walk(K, d + 1, q, cap, n, out);
  }
}

int64_t free_seed(int32_t kmax, int64_t cap, uint64_t *out) {
  int64_t n = 0;
  int K, q[MAXSEG];
  if (kmax > MAXSEG) kmax = MAXSEG;
  for (K = 1; K <= kmax && n < cap; ++K) q_seed_walk(K, 0, q, cap, &n, out);
  return n;
}

typedef struct {
  QKey key;
  double M;
} QEntry;
static int q_cmp_entry(const void *a, const void *b) {
  const QEntry *x = (const QEntry *)a, *y = (const QEntry *)b;
  if (x->M < y->M) return -1;
  if (x->M > y->M) return 1;
  return (x->key < y->key) ? -1 : (x->key > y->key) ? 1 : 0;
}

/* one batch-construction step of Alg. 1: rank the evaluated orders by (merit, key),     */
/* traverse at most W parents, admit their unseen admissible r-edit neighbours in order  */
/* until `room` are admitted                                                             */
int64_t free_expand_next(int64_t n, const uint64_t *keys, const double *merit, int32_t kcap, int32_t radius,
                         int32_t frontier_W, int64_t room, uint64_t *out_keys) {
  QEntry *R = (QEntry *)malloc(sizeof(QEntry) * (size_t)(n + 1));
  const int64_t cap1 = (int64_t)(2 * kcap + 2) * QMODES + 16;
  QKey *nb = (QKey *)malloc(sizeof(QKey) * (size_t)(radius >= 2 ? cap1 * cap1 : cap1));
  QSet seen;
  int64_t i, j, nF = 0;
  qset_init(&seen, n + room + 16);
  for (i = 0; i < n; ++i) {
    R[i].key = keys[i];
    R[i].M = isnan(merit[i]) ? INFINITY : merit[i];
    qset_add(&seen, keys[i]);
  }
  qsort(R, (size_t)n, sizeof(QEntry), q_cmp_entry);
  for (i = 0; i < n && i < frontier_W && nF < room; ++i) {
    const int64_t m = qneigh(R[i].key, kcap, radius, nb);
    for (j = 0; j < m && nF < room; ++j)
      if (!qset_has(&seen, nb[j])) {
        qset_add(&seen, nb[j]);
        out_keys[nF++] = nb[j];
      }
  }
  free(R);
  free(nb);
  free(seen.slot);
  return nF;
}
