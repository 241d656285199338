/*
 * comet_oracle.c -- FP64 CPU oracle of the mode-conditioned trajectory-optimisation
 * (TO) evaluator and of the greedy contact-mode expansion.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link, load or call this
 * file; only the tests, the smoke check and the CPU-baseline leg of the benchmark do.
 * It shares no code, header, table or constant generator with the HIP library.
 *
 * Plain and slow on purpose: dense per-stage matrices, full gradient vectors, a full
 * re-evaluation of the merit at every trial step, one sequence per thread.  Compile
 * with -O2 -ffp-contract=off (no fused multiply-add, no fast-math).
 *
 * What it follows (paper sections / equations):
 *   - Eq. (2)  mode-conditioned NLP for a fixed contact-mode order;
 *   - Sec. III-C "Shared representation across contact modes": N control intervals,
 *     defects d_k = x_{k+1} - F_k(x_k,u_k;m), masked rows in fixed positions;
 *   - Sec. III-C "Fixed-workspace local solves": S_k = H_k + rho I + A_k^T A_k / mu over
 *     the n_u+n_x unknowns (u_k, x_{k+1}); Cholesky without pivoting as PD test,
 *     failed attempts raise the damping, exhausted retries reject the step; a forward
 *     pass assembles the step and several trial step lengths are scored;
 *   - Sec. IV-A "CoMET configurations": schedule-derived initial guess, rows scaled by
 *     their median Jacobian-row norm over sample orders;
 *   - Sec. III-C "Stopping and scoring" and Eq. (4): score in physical units,
 *     feasible iff v <= eps_feas; Eq. (5): merit M = J + mu_merit max(v - eps, 0);
 *   - Alg. 1 and Sec. III-B: seed, ranking by merit, r-edit neighbourhoods,
 *     batch construction, refinement of the best feasible orders.
 * Readings of what the paper leaves open (pusher-slider mechanics, the augmented-
 * Lagrangian schedule, tolerances, tie-breaks) are listed in the design notes of the
 * repository; each is restated where it is used below.
 */
#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------------------ */
/* Pushing task constants.  Square slider of side a and mass m; ground friction     */
/* mu_g (reading: 0.5), f_max = mu_g m g; ellipsoidal limit surface with the        */
/* uniform-pressure radius c_ls = a (sqrt2 + ln(1+sqrt2)) / 6; velocity scale v_ref. */
/* ------------------------------------------------------------------------------ */
#define PNX 4  /* x, y, theta, s                                   */
#define PNU 4  /* at most: F_n, F_t, v_s (and h, timed)            */
#define PNW 8  /* at most: stage unknowns (u_k, x_{k+1})            */
#define PNV 12 /* at most: row arguments (x_k, u_k, x_{k+1})         */
#define PNR 12 /* at most: path rows per interval, equalities first  */
#define PNE 5  /* equality rows per interval                        */
#define PNI 7  /* at most: inequality rows per interval              */
#define PNT 3  /* terminal rows */
#define MAXSEG 6
#define MAXN 512

static const double P_A = 0.1, P_MASS = 1.0, P_G = 9.81, P_MUG = 0.5;
static const double P_VREF = 1.0, P_DT = 0.1, P_WV = 1.0;
/* Optimised timing (reading): the interval duration h is a fourth control, bounded per   */
/* interval by h_min <= h <= h_max, and the objective charges the elapsed time with the   */
/* weight w_T; a fixed-step problem uses h = P_DT.                                        */
static const double P_HMIN = 0.02, P_HMAX = 0.2, P_WT = 0.01;
static double p_fmax(void) { return P_MUG * P_MASS * P_G; }
static double p_cls(void) { return P_A * (sqrt(2.0) + log(1.0 + sqrt(2.0))) / 6.0; }

/* outward face normals in the body frame, face j at angle j*pi/2 */
static const double FACE_N[4][2] = {{1, 0}, {0, 1}, {-1, 0}, {0, -1}};

/* row types for the internal scaling */
enum { T_DX, T_DY, T_DTH, T_DS, T_STICK, T_SLIDE, T_FN, T_CONE, T_SLIP, T_FACE, T_TXY, T_TTH, T_DUR, NTYPES };

typedef struct {
  int32_t al_max, gn_max, chol_retries, ls_trials, max_rejects;
  int32_t timed; /* 1: the optimised-timing pushing problem */
  double mu0, mu_min, rho0, rho_min, rho_max, armijo_c1;
  double eta_star, omega_star, rc_star, eps_feas;
  double mu0_warm; /* initial penalty of a solve started from a given (warm) primal */
  /* Test switch (0 = plain FP64).  Rounds quantities to float32 as they are produced, to  */
  /* ask whether a result is determined at float32 precision at all: bit 0 the Gauss-    */
  /* Newton step direction, bit 1 the multipliers after each update, bit 2 the scaled    */
  /* row Jacobians, bit 3 the gains with the forward recursion run in float32, bit 4 the */
  /* gains alone.  Results with bits set are perturbations, not the oracle's answer.     */
  int32_t round32;
} OracleParams;

/* one mode-conditioned problem (one candidate order on one instance) */
typedef struct {
  int N;
  int timed;              /* interval durations are controls                      */
  int nu, nw, nv, nr, ni; /* controls, stage unknowns, row arguments, rows, ineqs */
  int face[MAXN], slip[MAXN], smask[MAXN]; /* slip: 0 stick, 1 slide+, 2 slide- */
  double mu;
  double x0[PNX], goal[3];
  const double *scale; /* NTYPES row scales */
  int round_jac;       /* test switch: scaled Jacobians rounded to float32 */
  int round_fwd;       /* test switch: gains and forward recursion in float32 */
  int round_gain;      /* test switch: gains rounded to float32, recursion in FP64 */
} PushProb;

/* ------------------------------------------------------------------------------ */
/* Rows of one interval, physical units.                                          */
/* v = (x_k[4], u_k[nu], x_{k+1}[4]), u = (F_n, F_t, v_s) or, with optimised timing, */
/* (F_n, F_t, v_s, h); the step is dt = P_DT or dt = h.  Row slots:                   */
/*  0..3 defects x_{k+1} - x_k - dt f(x_k,u_k)   (slot 3 masked at a face change)  */
/*  4    stick: v_s = 0 ;  slide(sigma): F_t - sigma mu F_n = 0                     */
/*  5    -F_n <= 0                                                                  */
/*  6    stick: F_t - mu F_n <= 0 ;  slide: -sigma v_s <= 0                         */
/*  7    stick: -F_t - mu F_n <= 0 ; slide: disabled                                */
/*  8,9  s_{k+1} - a/2 <= 0 ,  -s_{k+1} - a/2 <= 0                                  */
/*  10,11 (timed only) h - h_max <= 0 ,  h_min - h <= 0                            */
/* Quasi-static law (reading): body twist = (v_ref/f_max) (F_x, F_y, M / c_ls^2),   */
/* contact point p = (a/2) n + s t, force on the slider F = -F_n n + F_t t, so the  */
/* moment about the centre is M = p x F = (a/2) F_t + s F_n; explicit Euler.        */
/* ------------------------------------------------------------------------------ */
static void push_rows(int timed, int face, int slip, int smask, double mu, const double *v,
                      double *c, double J[PNR][PNV], int *en, int *type) {
  const int nu = timed ? 4 : 3, nr = timed ? 12 : 10, c1 = 4 + nu; /* c1: first column of x_{k+1} */
  const double fmax = p_fmax(), cls2 = p_cls() * p_cls(), k1 = P_VREF / fmax;
  const double dt = timed ? v[7] : P_DT;
  const double nx = FACE_N[face][0], ny = FACE_N[face][1];
  const double tx = -ny, ty = nx;
  const double x = v[0], y = v[1], th = v[2], s = v[3];
  const double Fn = v[4], Ft = v[5], vs = v[6];
  const double x1 = v[c1], y1 = v[c1 + 1], th1 = v[c1 + 2], s1 = v[c1 + 3];
  const double Fbx = -Fn * nx + Ft * tx, Fby = -Fn * ny + Ft * ty;
  const double M = 0.5 * P_A * Ft + s * Fn;
  const double xi_x = k1 * Fbx, xi_y = k1 * Fby, xi_t = k1 * M / cls2;
  const double ct = cos(th), st = sin(th);
  const double vx = ct * xi_x - st * xi_y, vy = st * xi_x + ct * xi_y;
  /* derivatives of the world velocity w.r.t. F_n and F_t */
  const double dvx_dFn = k1 * (ct * (-nx) - st * (-ny)), dvy_dFn = k1 * (st * (-nx) + ct * (-ny));
  const double dvx_dFt = k1 * (ct * tx - st * ty), dvy_dFt = k1 * (st * tx + ct * ty);
  int r, j;
  for (r = 0; r < PNR; ++r) {
    c[r] = 0.0;
    en[r] = 0;
    type[r] = T_FACE;
    for (j = 0; j < PNV; ++j) J[r][j] = 0.0;
  }
  /* defects; with optimised timing d/dh of "- h f" is "- f" */
  c[0] = x1 - x - dt * vx;
  J[0][0] = -1; J[0][2] = dt * vy; J[0][4] = -dt * dvx_dFn; J[0][5] = -dt * dvx_dFt; J[0][c1] = 1;
  c[1] = y1 - y - dt * vy;
  J[1][1] = -1; J[1][2] = -dt * vx; J[1][4] = -dt * dvy_dFn; J[1][5] = -dt * dvy_dFt; J[1][c1 + 1] = 1;
  c[2] = th1 - th - dt * xi_t;
  J[2][2] = -1; J[2][3] = -dt * k1 * Fn / cls2; J[2][4] = -dt * k1 * s / cls2;
  J[2][5] = -dt * k1 * 0.5 * P_A / cls2; J[2][c1 + 2] = 1;
  c[3] = s1 - s - dt * vs;
  J[3][3] = -1; J[3][6] = -dt; J[3][c1 + 3] = 1;
  if (timed) {
    J[0][7] = -vx;
    J[1][7] = -vy;
    J[2][7] = -xi_t;
    J[3][7] = -vs;
  }
  en[0] = en[1] = en[2] = 1;
  en[3] = smask;
  type[0] = T_DX; type[1] = T_DY; type[2] = T_DTH; type[3] = T_DS;
  /* mode equality */
  if (slip == 0) {
    c[4] = vs; J[4][6] = 1; type[4] = T_STICK;
  } else {
    const double sg = (slip == 1) ? 1.0 : -1.0;
    c[4] = Ft - sg * mu * Fn; J[4][5] = 1; J[4][4] = -sg * mu; type[4] = T_SLIDE;
  }
  en[4] = 1;
  /* inequalities */
  c[5] = -Fn; J[5][4] = -1; en[5] = 1; type[5] = T_FN;
  if (slip == 0) {
    c[6] = Ft - mu * Fn; J[6][5] = 1; J[6][4] = -mu; en[6] = 1; type[6] = T_CONE;
    c[7] = -Ft - mu * Fn; J[7][5] = -1; J[7][4] = -mu; en[7] = 1; type[7] = T_CONE;
  } else {
    const double sg = (slip == 1) ? 1.0 : -1.0;
    c[6] = -sg * vs; J[6][6] = -sg; en[6] = 1; type[6] = T_SLIP;
    c[7] = 0; en[7] = 0; type[7] = T_CONE;
  }
  c[8] = s1 - 0.5 * P_A; J[8][c1 + 3] = 1; en[8] = 1; type[8] = T_FACE;
  c[9] = -s1 - 0.5 * P_A; J[9][c1 + 3] = -1; en[9] = 1; type[9] = T_FACE;
  if (timed) {
    c[10] = v[7] - P_HMAX; J[10][7] = 1; en[10] = 1; type[10] = T_DUR;
    c[11] = P_HMIN - v[7]; J[11][7] = -1; en[11] = 1; type[11] = T_DUR;
  }
  for (r = 0; r < nr; ++r)
    if (!en[r]) {
      c[r] = 0;
      for (j = 0; j < PNV; ++j) J[r][j] = 0;
    }
}

/* terminal rows (x_N, y_N, theta_N) - goal, theta not wrapped */
static void push_term(const double *goal, const double *xN, double *c, double J[PNT][PNX], int *type) {
  int r, j;
  for (r = 0; r < PNT; ++r) {
    c[r] = xN[r] - goal[r];
    for (j = 0; j < PNX; ++j) J[r][j] = (r == j) ? 1.0 : 0.0;
  }
  type[0] = T_TXY; type[1] = T_TXY; type[2] = T_TTH;
}


/* Stage cost.  Fixed step: dt q(u) with q = (F_n^2 + F_t^2)/f_max^2 + w_v (v_s/v_ref)^2, */
/* gradient and its (constant, diagonal) Hessian.  Optimised timing: h (q(u) + w_T) with   */
/* the exact gradient; the Hessian model keeps the force/velocity block of the exact      */
/* Hessian, 2 h diag(weights of q), taken at h_e = max(h, h_min / 2), and drops the mixed */
/* (u, h) and (h, h) entries, with which the exact Hessian is indefinite (reading: the    */
/* duration direction takes its curvature from the active rows and the proximal term).   */
/* hu: [PNU][PNU], full.                                                                   */
static double push_cost(int timed, const double *u, double *gu, double hu[PNU][PNU]) {
  const double fm2 = p_fmax() * p_fmax(), vr2 = P_VREF * P_VREF;
  const double h = timed ? u[3] : P_DT;
  const double q = (u[0] * u[0] + u[1] * u[1]) / fm2 + P_WV * u[2] * u[2] / vr2;
  int i, j;
  if (gu) {
    gu[0] = h * 2.0 * u[0] / fm2;
    gu[1] = h * 2.0 * u[1] / fm2;
    gu[2] = h * 2.0 * P_WV * u[2] / vr2;
    if (timed) gu[3] = q + P_WT;
  }
  if (hu) {
    const double he = timed ? fmax(h, 0.5 * P_HMIN) : h;
    for (i = 0; i < PNU; ++i)
      for (j = 0; j < PNU; ++j) hu[i][j] = 0.0;
    hu[0][0] = he * 2.0 / fm2;
    hu[1][1] = he * 2.0 / fm2;
    hu[2][2] = he * 2.0 * P_WV / vr2;
  }
  return timed ? h * (q + P_WT) : h * q;
}

/* ------------------------------------------------------------------------------ */
/* Primal layout: z[k*nw + 0..nu-1] = u_k, z[k*nw + nu..nu+3] = x_{k+1},            */
/* k = 0..N-1, nw = nu + 4 (nu = 3, or 4 with optimised timing).                     */
/* ------------------------------------------------------------------------------ */
static void stage_args(const PushProb *P, const double *z, int k, double *v) {
  int i;
  const int nu = P->nu, nw = P->nw;
  const double *xk = (k == 0) ? P->x0 : &z[(k - 1) * nw + nu];
  for (i = 0; i < PNV; ++i) v[i] = 0.0;
  for (i = 0; i < PNX; ++i) v[i] = xk[i];
  for (i = 0; i < nu; ++i) v[PNX + i] = z[k * nw + i];
  for (i = 0; i < PNX; ++i) v[PNX + nu + i] = z[k * nw + nu + i];
}

/* scaled rows of interval k: c~ = c / sigma_type, J~ likewise */
static void stage_scaled(const PushProb *P, const double *z, int k, double *c, double J[PNR][PNV], int *en) {
  double v[PNV];
  int type[PNR], r, j;
  stage_args(P, z, k, v);
  push_rows(P->timed, P->face[k], P->slip[k], P->smask[k], P->mu, v, c, J, en, type);
  for (r = 0; r < P->nr; ++r) {
    const double sc = P->scale[type[r]];
    c[r] /= sc;
    for (j = 0; j < PNV; ++j) J[r][j] /= sc;
    if (P->round_jac)
      for (j = 0; j < PNV; ++j) J[r][j] = (double)(float)J[r][j];
  }
}

static void term_scaled(const PushProb *P, const double *z, double *c, double J[PNT][PNX]) {
  int type[PNT], r, j;
  push_term(P->goal, &z[(P->N - 1) * P->nw + P->nu], c, J, type);
  for (r = 0; r < PNT; ++r) {
    const double sc = P->scale[type[r]];
    c[r] /= sc;
    for (j = 0; j < PNX; ++j) J[r][j] /= sc;
  }
}

/* ------------------------------------------------------------------------------ */
/* Augmented-Lagrangian merit (reading: classic PHR form, mu = 1/penalty).          */
/*   phi = J + sum_eq (lam c + c^2/(2 mu)) + sum_in (mu/2)([nu + c/mu]_+^2 - nu^2)   */
/* lam: [N][5] equality multipliers (slots 0..4), nu: [N][ni] inequality multipliers */
/* (slots 5..nr-1; ni = 5, or 7 with optimised timing), lamT[3] terminal ones.       */
/* ------------------------------------------------------------------------------ */
typedef struct {
  double *lam, *nu, lamT[PNT];
  double mu;
} Dual;

static double merit(const PushProb *P, const double *z, const Dual *D) {
  double phi = 0.0, c[PNR], J[PNR][PNV], cT[PNT], JT[PNT][PNX];
  int en[PNR], k, r;
  for (k = 0; k < P->N; ++k) {
    phi += push_cost(P->timed, &z[k * P->nw], NULL, NULL);
    stage_scaled(P, z, k, c, J, en);
    for (r = 0; r < PNE; ++r)
      if (en[r]) phi += D->lam[k * PNE + r] * c[r] + c[r] * c[r] / (2.0 * D->mu);
    for (r = PNE; r < P->nr; ++r)
      if (en[r]) {
        const double nu = D->nu[k * P->ni + (r - PNE)];
        const double t = fmax(nu + c[r] / D->mu, 0.0);
        phi += 0.5 * D->mu * (t * t - nu * nu);
      }
  }
  term_scaled(P, z, cT, JT);
  for (r = 0; r < PNT; ++r) phi += D->lamT[r] * cT[r] + cT[r] * cT[r] / (2.0 * D->mu);
  return phi;
}

/* multiplier estimate of a row: d phi / d c~ ; returns 0 for a disabled row, and    */
/* sets *active for rows that enter the Gauss-Newton curvature                       */
static double row_weight(int r, int en, double c, double lam, double nu, double mu, int *active) {
  if (!en) {
    *active = 0;
    return 0.0;
  }
  if (r < PNE) {
    *active = 1;
    return lam + c / mu;
  }
  {
    const double t = nu + c / mu;
    *active = (t > 0.0);
    return (t > 0.0) ? t : 0.0;
  }
}

/* gradient of phi w.r.t. z (size nw N) */
static void gradient(const PushProb *P, const double *z, const Dual *D, double *g) {
  double c[PNR], J[PNR][PNV], cT[PNT], JT[PNT][PNX], gu[PNU];
  const int nu = P->nu, nw = P->nw;
  int en[PNR], k, r, j, act;
  memset(g, 0, sizeof(double) * nw * P->N);
  for (k = 0; k < P->N; ++k) {
    push_cost(P->timed, &z[k * nw], gu, NULL);
    for (j = 0; j < nu; ++j) g[k * nw + j] += gu[j];
    stage_scaled(P, z, k, c, J, en);
    for (r = 0; r < P->nr; ++r) {
      const double lam = (r < PNE) ? D->lam[k * PNE + r] : 0.0;
      const double nuv = (r >= PNE) ? D->nu[k * P->ni + r - PNE] : 0.0;
      const double w = row_weight(r, en[r], c[r], lam, nuv, D->mu, &act);
      if (w == 0.0) continue;
      /* x_k columns belong to the previous stage's x_{k+1} (x_0 is fixed) */
      if (k > 0)
        for (j = 0; j < PNX; ++j) g[(k - 1) * nw + nu + j] += w * J[r][j];
      for (j = 0; j < nw; ++j) g[k * nw + j] += w * J[r][PNX + j];
    }
  }
  term_scaled(P, z, cT, JT);
  for (r = 0; r < PNT; ++r) {
    const double w = D->lamT[r] + cT[r] / D->mu;
    for (j = 0; j < PNX; ++j) g[(P->N - 1) * nw + nu + j] += w * JT[r][j];
  }
}

/* ------------------------------------------------------------------------------ */
/* Dense Cholesky without pivoting, n <= 17.  Returns 0 if a pivot is not positive. */
/* ------------------------------------------------------------------------------ */
static int cholesky(int n, double *A, int lda) {
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

/* solve L L^T x = b in place */
static void chol_solve(int n, const double *L, int lda, double *b) {
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

/* ------------------------------------------------------------------------------ */
/* One regularised Gauss-Newton step by the backward Riccati recursion.             */
/* Model: m(dz) = g^T dz + 1/2 dz^T (H + rho I) dz, H = cost Hessian                */
/*        + (1/mu) sum over equality and active inequality rows of a a^T.           */
/* Stage k owns w_k = (u_k, x_{k+1}); its local quadratic is over y = (x_k, w_k).  */
/* Returns 1 on success, 0 when a Cholesky factorisation fails.                     */
/* ------------------------------------------------------------------------------ */
static int gn_step(const PushProb *P, const double *z, const Dual *D, double rho, double *dz) {
  const int N = P->N, nu = P->nu, nw = P->nw, nv = P->nv;
  double Pm[PNX][PNX], pv[PNX];
  double *kk = (double *)malloc(sizeof(double) * N * nw);
  double *KK = (double *)malloc(sizeof(double) * N * nw * PNX);
  double c[PNR], J[PNR][PNV], cT[PNT], JT[PNT][PNX], gu[PNU], hu[PNU][PNU];
  int en[PNR], k, r, i, j, act, ok = 1;
  /* terminal value function V_N */
  term_scaled(P, z, cT, JT);
  for (i = 0; i < PNX; ++i) {
    pv[i] = 0;
    for (j = 0; j < PNX; ++j) Pm[i][j] = 0;
  }
  for (r = 0; r < PNT; ++r) {
    const double w = D->lamT[r] + cT[r] / D->mu;
    for (i = 0; i < PNX; ++i) {
      pv[i] += w * JT[r][i];
      for (j = 0; j < PNX; ++j) Pm[i][j] += JT[r][i] * JT[r][j] / D->mu;
    }
  }
  for (k = N - 1; k >= 0 && ok; --k) {
    double G[PNV][PNV], h[PNV], S[PNW * PNW], rhs[PNW];
    memset(G, 0, sizeof G);
    memset(h, 0, sizeof h);
    push_cost(P->timed, &z[k * nw], gu, hu);
    for (i = 0; i < nu; ++i) {
      h[PNX + i] += gu[i];
      for (j = 0; j < nu; ++j) G[PNX + i][PNX + j] += hu[i][j];
    }
    stage_scaled(P, z, k, c, J, en);
    for (r = 0; r < P->nr; ++r) {
      const double lam = (r < PNE) ? D->lam[k * PNE + r] : 0.0;
      const double nuv = (r >= PNE) ? D->nu[k * P->ni + r - PNE] : 0.0;
      const double w = row_weight(r, en[r], c[r], lam, nuv, D->mu, &act);
      for (i = 0; i < nv; ++i) h[i] += w * J[r][i];
      if (act)
        for (i = 0; i < nv; ++i)
          for (j = 0; j < nv; ++j) G[i][j] += J[r][i] * J[r][j] / D->mu;
    }
    /* value function of x_{k+1}, the last four entries of y */
    for (i = 0; i < PNX; ++i) {
      h[PNX + nu + i] += pv[i];
      for (j = 0; j < PNX; ++j) G[PNX + nu + i][PNX + nu + j] += Pm[i][j];
    }
    for (i = 0; i < nw; ++i)
      for (j = 0; j < nw; ++j) S[i * nw + j] = G[PNX + i][PNX + j] + (i == j ? rho : 0.0);
    if (!cholesky(nw, S, nw)) {
      ok = 0;
      break;
    }
    /* gains: k = -S^-1 q_w, K = -S^-1 Q_wx */
    for (i = 0; i < nw; ++i) rhs[i] = -h[PNX + i];
    chol_solve(nw, S, nw, rhs);
    for (i = 0; i < nw; ++i) kk[k * nw + i] = rhs[i];
    for (j = 0; j < PNX; ++j) {
      for (i = 0; i < nw; ++i) rhs[i] = -G[PNX + i][j];
      chol_solve(nw, S, nw, rhs);
      for (i = 0; i < nw; ++i) KK[(k * nw + i) * PNX + j] = rhs[i];
    }
    /* value: P = Q_xx + Q_xw K, p = q_x + Q_xw k */
    {
      double Pn[PNX][PNX], pn[PNX];
      for (i = 0; i < PNX; ++i) {
        pn[i] = h[i];
        for (r = 0; r < nw; ++r) pn[i] += G[i][PNX + r] * kk[k * nw + r];
        for (j = 0; j < PNX; ++j) {
          Pn[i][j] = G[i][j];
          for (r = 0; r < nw; ++r) Pn[i][j] += G[i][PNX + r] * KK[(k * nw + r) * PNX + j];
        }
      }
      for (i = 0; i < PNX; ++i) {
        pv[i] = pn[i];
        for (j = 0; j < PNX; ++j) Pm[i][j] = 0.5 * (Pn[i][j] + Pn[j][i]);
      }
    }
  }
  if (ok && P->round_fwd) {
    float dxf[PNX] = {0, 0, 0, 0};
    for (k = 0; k < N; ++k) {
      for (i = 0; i < nw; ++i) {
        float s = (float)kk[k * nw + i];
        for (j = 0; j < PNX; ++j) s += (float)KK[(k * nw + i) * PNX + j] * dxf[j];
        dz[k * nw + i] = s;
      }
      for (j = 0; j < PNX; ++j) dxf[j] = (float)dz[k * nw + nu + j];
    }
  } else if (ok) {
    double dx[PNX] = {0, 0, 0, 0};
    for (k = 0; k < N; ++k) {
      for (i = 0; i < nw; ++i) {
        double s = P->round_gain ? (double)(float)kk[k * nw + i] : kk[k * nw + i];
        for (j = 0; j < PNX; ++j)
          s += (P->round_gain ? (double)(float)KK[(k * nw + i) * PNX + j] : KK[(k * nw + i) * PNX + j]) * dx[j];
        dz[k * nw + i] = s;
      }
      for (j = 0; j < PNX; ++j) dx[j] = dz[k * nw + nu + j];
    }
  }
  free(kk);
  free(KK);
  return ok;
}

/* scaled feasibility v_s, complementarity r_c at z */
static void scaled_viol(const PushProb *P, const double *z, const Dual *D, double *vs, double *rc) {
  double c[PNR], J[PNR][PNV], cT[PNT], JT[PNT][PNX];
  int en[PNR], k, r;
  double v = 0.0, q = 0.0;
  for (k = 0; k < P->N; ++k) {
    stage_scaled(P, z, k, c, J, en);
    for (r = 0; r < P->nr; ++r) {
      if (!en[r]) continue;
      if (r < PNE) v = fmax(v, fabs(c[r]));
      else {
        const double nu = D->nu[k * P->ni + r - PNE];
        v = fmax(v, fmax(c[r], 0.0));
        q = fmax(q, fabs(fmin(-c[r], nu)));
      }
    }
  }
  term_scaled(P, z, cT, JT);
  for (r = 0; r < PNT; ++r) v = fmax(v, fabs(cT[r]));
  *vs = v;
  *rc = q;
}

/* first-order multiplier update lam += c/mu, nu = [nu + c/mu]_+ */
static void update_duals(const PushProb *P, const double *z, Dual *D) {
  double c[PNR], J[PNR][PNV], cT[PNT], JT[PNT][PNX];
  int en[PNR], k, r;
  for (k = 0; k < P->N; ++k) {
    stage_scaled(P, z, k, c, J, en);
    for (r = 0; r < P->nr; ++r) {
      if (!en[r]) continue;
      if (r < PNE) D->lam[k * PNE + r] += c[r] / D->mu;
      else {
        double *nu = &D->nu[k * P->ni + r - PNE];
        *nu = fmax(*nu + c[r] / D->mu, 0.0);
      }
    }
  }
  term_scaled(P, z, cT, JT);
  for (r = 0; r < PNT; ++r) D->lamT[r] += cT[r] / D->mu;
}

/* test switch: multipliers rounded to float32 */
static void round_duals(const PushProb *P, Dual *D) {
  int i;
  for (i = 0; i < P->N * PNE; ++i) D->lam[i] = (double)(float)D->lam[i];
  for (i = 0; i < P->N * P->ni; ++i) D->nu[i] = (double)(float)D->nu[i];
}

/* objective and violation in physical units, Eq. (4) */
static void score(const PushProb *P, const double *z, double *Jout, double *vout) {
  double c[PNR], J[PNR][PNV], cT[PNT], JT[PNT][PNX], v[PNV];
  int en[PNR], type[PNR], ttype[PNT], k, r;
  double obj = 0.0, vi = 0.0;
  for (k = 0; k < P->N; ++k) {
    obj += push_cost(P->timed, &z[k * P->nw], NULL, NULL);
    stage_args(P, z, k, v);
    push_rows(P->timed, P->face[k], P->slip[k], P->smask[k], P->mu, v, c, J, en, type);
    for (r = 0; r < P->nr; ++r) {
      if (!en[r]) continue;
      vi = fmax(vi, (r < PNE) ? fabs(c[r]) : fmax(c[r], 0.0));
    }
  }
  push_term(P->goal, &z[(P->N - 1) * P->nw + P->nu], cT, JT, ttype);
  for (r = 0; r < PNT; ++r) vi = fmax(vi, fabs(cT[r]));
  *Jout = obj;
  *vout = vi;
}

/* schedule-derived initial guess: pose interpolated start->goal, contact coordinate */
/* held at its start value, F_n = 0.05 f_max, F_t on the cone edge for sliding; with  */
/* optimised timing every interval starts at the fixed step, h = P_DT.                */
static void initial_guess(const PushProb *P, double *z) {
  const double fn = 0.05 * p_fmax();
  const int nu = P->nu, nw = P->nw;
  int k, i;
  for (k = 0; k < P->N; ++k) {
    const double sg = (P->slip[k] == 0) ? 0.0 : ((P->slip[k] == 1) ? 1.0 : -1.0);
    const double t = (double)(k + 1) / (double)P->N;
    z[k * nw + 0] = fn;
    z[k * nw + 1] = sg * P->mu * fn;
    z[k * nw + 2] = 0.0;
    if (P->timed) z[k * nw + 3] = P_DT;
    for (i = 0; i < 3; ++i) z[k * nw + nu + i] = P->x0[i] + (P->goal[i] - P->x0[i]) * t;
    z[k * nw + nu + 3] = P->x0[3];
  }
}

/* ------------------------------------------------------------------------------ */
/* Problem setup from (nseg, modes, knots).  Push mode id = 3*face + slip.          */
/* The s-row of the last interval of a segment is masked when the next segment     */
/* uses another face (instantaneous relocation of the pusher).                      */
/* ------------------------------------------------------------------------------ */
static int setup_push(PushProb *P, int timed, int nseg, const int32_t *modes, const int32_t *knots,
                      const double *x0, const double *goal, double mu, const double *scale) {
  int j, i, k = 0;
  P->timed = timed ? 1 : 0;
  P->round_jac = 0;
  P->round_fwd = 0;
  P->round_gain = 0;
  P->nu = timed ? 4 : 3;
  P->nw = P->nu + PNX;
  P->nv = P->nw + PNX;
  P->nr = timed ? 12 : 10;
  P->ni = P->nr - PNE;
  if (nseg < 1 || nseg > MAXSEG) return 0;
  for (j = 0; j < nseg; ++j) {
    if (modes[j] < 0 || modes[j] >= 12 || knots[j] < 1) return 0;
    for (i = 0; i < knots[j]; ++i) {
      if (k >= MAXN) return 0;
      P->face[k] = modes[j] / 3;
      P->slip[k] = modes[j] % 3;
      P->smask[k] = 1;
      ++k;
    }
    if (j + 1 < nseg && (modes[j + 1] / 3) != (modes[j] / 3)) P->smask[k - 1] = 0;
  }
  P->N = k;
  P->mu = mu;
  for (i = 0; i < PNX; ++i) P->x0[i] = x0[i];
  for (i = 0; i < 3; ++i) P->goal[i] = goal[i];
  P->scale = scale;
  if (!isfinite(mu)) return 0;
  for (i = 0; i < PNX; ++i) if (!isfinite(x0[i])) return 0;
  for (i = 0; i < 3; ++i) if (!isfinite(goal[i])) return 0;
  return 1;
}

/* ------------------------------------------------------------------------------ */
/* Row scales: for each row type, the median 2-norm of its (physical) Jacobian row  */
/* over the schedule-derived initial guesses of a fixed sample of orders: all 144  */
/* two-segment orders, 5+5 intervals, start at rest at the origin, goal            */
/* (0.1, 0.1, pi/4), pusher friction 0.4.  Median of an even count = mean of the   */
/* two middle values.                                                              */
/* ------------------------------------------------------------------------------ */
static int cmp_double(const void *a, const void *b) {
  const double x = *(const double *)a, y = *(const double *)b;
  return (x < y) ? -1 : (x > y) ? 1 : 0;
}

static double g_push_scale[2][NTYPES];
static int g_push_scale_ready[2] = {0, 0};
static pthread_mutex_t g_scale_lock = PTHREAD_MUTEX_INITIALIZER;

static void compute_push_scales(int timed, double *out) {
  static double buf[NTYPES][144 * 10 * 2 + 8];
  int cnt[NTYPES];
  double ones[NTYPES];
  const double x0[4] = {0, 0, 0, 0}, goal[3] = {0.1, 0.1, M_PI / 4.0};
  int m1, m2, t, k, r, j;
  for (t = 0; t < NTYPES; ++t) {
    cnt[t] = 0;
    ones[t] = 1.0;
  }
  for (m1 = 0; m1 < 12; ++m1)
    for (m2 = 0; m2 < 12; ++m2) {
      PushProb P;
      int32_t modes[2] = {m1, m2}, knots[2] = {5, 5};
      double z[10 * PNW], v[PNV], c[PNR], J[PNR][PNV], cT[PNT], JT[PNT][PNX];
      int en[PNR], type[PNR], tt[PNT];
      setup_push(&P, timed, 2, modes, knots, x0, goal, 0.4, ones);
      initial_guess(&P, z);
      for (k = 0; k < P.N; ++k) {
        stage_args(&P, z, k, v);
        push_rows(timed, P.face[k], P.slip[k], P.smask[k], P.mu, v, c, J, en, type);
        for (r = 0; r < P.nr; ++r) {
          double nrm = 0.0;
          if (!en[r]) continue;
          for (j = 0; j < PNV; ++j) nrm += J[r][j] * J[r][j];
          buf[type[r]][cnt[type[r]]++] = sqrt(nrm);
        }
      }
      push_term(P.goal, &z[(P.N - 1) * P.nw + P.nu], cT, JT, tt);
      for (r = 0; r < PNT; ++r) {
        double nrm = 0.0;
        for (j = 0; j < PNX; ++j) nrm += JT[r][j] * JT[r][j];
        buf[tt[r]][cnt[tt[r]]++] = sqrt(nrm);
      }
    }
  for (t = 0; t < NTYPES; ++t) {
    const int n = cnt[t];
    if (n == 0) {           /* a type the model does not have */
      out[t] = 1.0;
      continue;
    }
    qsort(buf[t], (size_t)n, sizeof(double), cmp_double);
    out[t] = (n % 2) ? buf[t][n / 2] : 0.5 * (buf[t][n / 2 - 1] + buf[t][n / 2]);
  }
}

static const double *push_scales(int timed) {
  timed = timed ? 1 : 0;
  pthread_mutex_lock(&g_scale_lock);
  if (!g_push_scale_ready[timed]) {
    compute_push_scales(timed, g_push_scale[timed]);
    g_push_scale_ready[timed] = 1;
  }
  pthread_mutex_unlock(&g_scale_lock);
  return g_push_scale[timed];
}

/* ------------------------------------------------------------------------------ */
/* The solver: AL outer loop, Gauss-Newton inner loop (reading of Sec. III-C).      */
/* ------------------------------------------------------------------------------ */
typedef struct {
  int al_iters, gn_iters, chol_fails, status; /* status: 1 converged, 0 budget, 2 non-finite */
} SolveStats;

static int all_finite(const double *a, int n) {
  int i;
  for (i = 0; i < n; ++i)
    if (!isfinite(a[i])) return 0;
  return 1;
}

static void solve(const PushProb *P, const OracleParams *prm, int warm, double *z, SolveStats *st) {
  const int N = P->N, nz = N * P->nw;
  double *g = (double *)malloc(sizeof(double) * nz);
  double *dz = (double *)malloc(sizeof(double) * nz);
  double *zt = (double *)malloc(sizeof(double) * nz);
  double *phi = (double *)malloc(sizeof(double) * (size_t)prm->ls_trials);
  Dual D;
  double eta, omega, rho = prm->rho0;
  int al, i;
  D.lam = (double *)calloc((size_t)N * PNE, sizeof(double));
  D.nu = (double *)calloc((size_t)N * P->ni, sizeof(double));
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
      gradient(P, z, &D, g);
      gnorm = 0.0;
      for (i = 0; i < nz; ++i) gnorm = fmax(gnorm, fabs(g[i]));
      if (gnorm <= omega) break;
      phi0 = merit(P, z, &D);
      ok = gn_step(P, z, &D, rho, dz);
      while (!ok && tries < prm->chol_retries) {
        st->chol_fails++;
        rho = fmax(10.0 * rho, 1e-8);
        ++tries;
        ok = gn_step(P, z, &D, rho, dz);
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
          phi[t] = merit(P, zt, &D);
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
        if (best >= 0) {
          for (i = 0; i < nz; ++i) z[i] += alpha * dz[i];
        }
      }
      if (best >= 0) {
        rho = fmax(rho / 3.0, prm->rho_min);
        rejects = 0;
      } else {
        rho = fmin(10.0 * rho, prm->rho_max);
        if (++rejects >= prm->max_rejects) break;
      }
    }
    /* outer update at the final inner iterate */
    scaled_viol(P, z, &D, &vs, &rc);
    gradient(P, z, &D, g);
    gnorm = 0.0;
    for (i = 0; i < nz; ++i) gnorm = fmax(gnorm, fabs(g[i]));
    if (!isfinite(vs) || !isfinite(gnorm) || !all_finite(z, nz)) {
      st->status = 2;
      break;
    }
    if (vs <= eta) {
      if (vs <= prm->eta_star && gnorm <= prm->omega_star && rc <= prm->rc_star) {
        st->status = 1;
        break;
      }
      update_duals(P, z, &D);
      if (prm->round32 & 2) round_duals(P, &D);
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
/* Batched evaluation over sequences, one sequence per thread.                      */
/* traj: [B][nmax+1][4+nu] rows (x_k, u_k), row N has u = 0, rows beyond N zero.    */
/* stats: [B][4] = (AL iterations, GN iterations, Cholesky failures, status).       */
/* ------------------------------------------------------------------------------ */
typedef struct {
  int64_t B;
  int32_t smax, nmax;
  const double *x0, *goal, *inst, *warm;
  const int32_t *nseg, *modes, *knots;
  const OracleParams *prm;
  double *cost, *viol, *traj;
  uint8_t *feas;
  int32_t *stats;
  int64_t next;
  pthread_mutex_t lock;
} EvalJob;

static void eval_one(EvalJob *E, int64_t b) {
  PushProb *P = (PushProb *)malloc(sizeof(PushProb));
  const int timed = E->prm->timed != 0, rw = PNX + (timed ? 4 : 3); /* trajectory row width */
  const double *scale = push_scales(timed);
  double *z;
  SolveStats st = {0, 0, 0, 2};
  double J = NAN, v = INFINITY;
  int k, i;
  int ok = setup_push(P, timed, E->nseg[b], &E->modes[b * E->smax], &E->knots[b * E->smax], &E->x0[b * PNX],
                      &E->goal[b * 3], E->inst[b], scale);
  if (ok && P->N > E->nmax) ok = 0;
  if (ok) {
    P->round_jac = (E->prm->round32 & 4) != 0;
    P->round_fwd = (E->prm->round32 & 8) != 0;
    P->round_gain = (E->prm->round32 & 16) != 0;
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
  z = (double *)malloc(sizeof(double) * P->N * P->nw);
  if (E->warm) {
    const double *w = &E->warm[b * (E->nmax + 1) * rw];
    for (k = 0; k < P->N; ++k) {
      for (i = 0; i < P->nu; ++i) z[k * P->nw + i] = w[k * rw + PNX + i];
      for (i = 0; i < PNX; ++i) z[k * P->nw + P->nu + i] = w[(k + 1) * rw + i];
    }
  } else {
    initial_guess(P, z);
  }
  solve(P, E->prm, E->warm != NULL, z, &st);
  if (st.status != 2) score(P, z, &J, &v);
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
    for (i = 0; i < PNX; ++i) T[i] = P->x0[i];
    for (k = 0; k < P->N; ++k) {
      for (i = 0; i < P->nu; ++i) T[k * rw + PNX + i] = z[k * P->nw + i];
      for (i = 0; i < PNX; ++i) T[(k + 1) * rw + i] = z[k * P->nw + P->nu + i];
    }
  }
  free(z);
  free(P);
}

static void *eval_worker(void *arg) {
  EvalJob *E = (EvalJob *)arg;
  for (;;) {
    int64_t b;
    pthread_mutex_lock(&E->lock);
    b = E->next++;
    pthread_mutex_unlock(&E->lock);
    if (b >= E->B) break;
    eval_one(E, b);
  }
  return NULL;
}

static void run_eval(EvalJob *E, int nthreads) {
  pthread_t th[256];
  int t;
  E->next = 0;
  pthread_mutex_init(&E->lock, NULL);
  if (nthreads < 1) nthreads = 1;
  if (nthreads > 256) nthreads = 256;
  if (nthreads == 1 || E->B <= 1) {
    eval_worker(E);
  } else {
    for (t = 0; t < nthreads; ++t) pthread_create(&th[t], NULL, eval_worker, E);
    for (t = 0; t < nthreads; ++t) pthread_join(th[t], NULL);
  }
  pthread_mutex_destroy(&E->lock);
}

int oracle_evaluate(int64_t B, int32_t smax, int32_t nmax, const double *x0, const double *goal,
                    const double *inst, const int32_t *nseg, const int32_t *modes, const int32_t *knots,
                    const double *warm, const OracleParams *prm, int32_t nthreads, double *cost, double *viol,
                    uint8_t *feas, double *traj, int32_t *stats) {
  EvalJob E;
  if (B < 0 || smax < 1 || smax > MAXSEG || nmax < 1 || nmax > MAXN || !prm) return -1;
  memset(&E, 0, sizeof E);
  E.B = B; E.smax = smax; E.nmax = nmax;
  E.x0 = x0; E.goal = goal; E.inst = inst; E.warm = warm;
  E.nseg = nseg; E.modes = modes; E.knots = knots; E.prm = prm;
  E.cost = cost; E.viol = viol; E.feas = feas; E.traj = traj; E.stats = stats;
  run_eval(&E, nthreads);
  return 0;
}

/* ------------------------------------------------------------------------------ */
/* Debug entry points used by the pins: one sequence, given primal and duals.       */
/* z: [N*nw] in the (u_k, x_{k+1}) layout; lam [N*5], nu [N*ni], lamT [3].         */
/* ------------------------------------------------------------------------------ */
int oracle_push_scales(int32_t timed, double *out) {
  const double *s = push_scales(timed);
  int t;
  for (t = 0; t < NTYPES; ++t) out[t] = s[t];
  return NTYPES;
}

int oracle_push_rows(int32_t timed, int32_t face, int32_t slip, int32_t smask, double mu, const double *v,
                     double *c, double *J, int32_t *en) {
  double JJ[PNR][PNV], cc[PNR];
  int e[PNR], type[PNR], r, j;
  const int nr = timed ? 12 : 10, nv = timed ? 12 : 11;
  push_rows(timed, face, slip, smask, mu, v, cc, JJ, e, type);
  for (r = 0; r < nr; ++r) {
    c[r] = cc[r];
    en[r] = e[r];
    for (j = 0; j < nv; ++j) J[r * nv + j] = JJ[r][j];
  }
  return 0;
}

/* stage cost, its gradient (nu) and Hessian model (nu x nu, row-major) */
double oracle_push_cost(int32_t timed, const double *u, double *gu, double *hu) {
  double H[PNU][PNU];
  const int nu = timed ? 4 : 3;
  int i, j;
  const double J = push_cost(timed, u, gu, H);
  for (i = 0; i < nu; ++i)
    for (j = 0; j < nu; ++j) hu[i * nu + j] = H[i][j];
  return J;
}

static int debug_setup(PushProb *P, int32_t timed, int32_t nseg, const int32_t *modes, const int32_t *knots,
                       const double *x0, const double *goal, double mu) {
  return setup_push(P, timed, nseg, modes, knots, x0, goal, mu, push_scales(timed));
}

int oracle_push_initial(int32_t timed, int32_t nseg, const int32_t *modes, const int32_t *knots, const double *x0,
                        const double *goal, double mu, double *z) {
  PushProb P;
  if (!debug_setup(&P, timed, nseg, modes, knots, x0, goal, mu)) return -1;
  initial_guess(&P, z);
  return P.N;
}

int oracle_push_merit(int32_t timed, int32_t nseg, const int32_t *modes, const int32_t *knots, const double *x0,
                      const double *goal, double mu, const double *z, const double *lam, const double *nu,
                      const double *lamT, double mu_al, double *phi_out, double *grad_out) {
  PushProb P;
  Dual D;
  if (!debug_setup(&P, timed, nseg, modes, knots, x0, goal, mu)) return -1;
  D.lam = (double *)lam;
  D.nu = (double *)nu;
  D.lamT[0] = lamT[0]; D.lamT[1] = lamT[1]; D.lamT[2] = lamT[2];
  D.mu = mu_al;
  if (phi_out) *phi_out = merit(&P, z, &D);
  if (grad_out) gradient(&P, z, &D, grad_out);
  return P.N;
}

int oracle_push_step(int32_t timed, int32_t nseg, const int32_t *modes, const int32_t *knots, const double *x0,
                     const double *goal, double mu, const double *z, const double *lam, const double *nu,
                     const double *lamT, double mu_al, double rho, double *dz) {
  PushProb P;
  Dual D;
  if (!debug_setup(&P, timed, nseg, modes, knots, x0, goal, mu)) return -1;
  D.lam = (double *)lam;
  D.nu = (double *)nu;
  D.lamT[0] = lamT[0]; D.lamT[1] = lamT[1]; D.lamT[2] = lamT[2];
  D.mu = mu_al;
  return gn_step(&P, z, &D, rho, dz) ? P.N : 0;
}

/* scaled rows and Jacobians per stage (for the dense-KKT pin):                     */
/* c [N*nr], J [N*nr*nv], en [N*nr], cT [3], JT [3*4]                                */
int oracle_push_blocks(int32_t timed, int32_t nseg, const int32_t *modes, const int32_t *knots, const double *x0,
                       const double *goal, double mu, const double *z, double *c, double *J, int32_t *en,
                       double *cT, double *JT) {
  PushProb P;
  double cc[PNR], JJ[PNR][PNV], ct[PNT], Jt[PNT][PNX];
  int e[PNR], k, r, j;
  if (!debug_setup(&P, timed, nseg, modes, knots, x0, goal, mu)) return -1;
  for (k = 0; k < P.N; ++k) {
    stage_scaled(&P, z, k, cc, JJ, e);
    for (r = 0; r < P.nr; ++r) {
      c[k * P.nr + r] = cc[r];
      en[k * P.nr + r] = e[r];
      for (j = 0; j < P.nv; ++j) J[(k * P.nr + r) * P.nv + j] = JJ[r][j];
    }
  }
  term_scaled(&P, z, ct, Jt);
  for (r = 0; r < PNT; ++r) {
    cT[r] = ct[r];
    for (j = 0; j < PNX; ++j) JT[r * PNX + j] = Jt[r][j];
  }
  return P.N;
}

int oracle_push_score(int32_t timed, int32_t nseg, const int32_t *modes, const int32_t *knots, const double *x0,
                      const double *goal, double mu, const double *z, double *J, double *v) {
  PushProb P;
  if (!debug_setup(&P, timed, nseg, modes, knots, x0, goal, mu)) return -1;
  score(&P, z, J, v);
  return P.N;
}

/* ================================================================================ */
/* Greedy contact-mode expansion (Alg. 1, Sec. III-B).                              */
/* ================================================================================ */
/* A contact-mode order is (K, m_0..m_{K-1}); its key packs K and the ids so that   */
/* comparing keys compares (K, m_0, m_1, ...) lexicographically:                     */
/*   key = K << 60 | m_0 << 50 | m_1 << 40 | ... | m_5 << 0, 10 bits per id.         */
typedef uint64_t Key;

static Key key_make(int K, const int *m) {
  Key k = (Key)K << 60;
  int i;
  for (i = 0; i < K; ++i) k |= (Key)m[i] << (50 - 10 * i);
  return k;
}

static int key_len(Key k) { return (int)(k >> 60); }
static int key_mode(Key k, int i) { return (int)((k >> (50 - 10 * i)) & 1023u); }

/* open-addressing set of keys */
typedef struct {
  Key *slot;
  int64_t cap;
} KeySet;

static void set_init(KeySet *S, int64_t n) {
  int64_t c = 16;
  while (c < 2 * n + 16) c <<= 1;
  S->cap = c;
  S->slot = (Key *)calloc((size_t)c, sizeof(Key));
}
static uint64_t mix64(uint64_t x) {
  x ^= x >> 33; x *= 0xff51afd7ed558ccdULL;
  x ^= x >> 33; x *= 0xc4ceb9fe1a85ec53ULL;
  x ^= x >> 33;
  return x;
}
static int set_has(const KeySet *S, Key k) {
  int64_t i = (int64_t)(mix64(k) & (uint64_t)(S->cap - 1));
  while (S->slot[i]) {
    if (S->slot[i] == k) return 1;
    i = (i + 1) & (S->cap - 1);
  }
  return 0;
}
static void set_add(KeySet *S, Key k) {
  int64_t i = (int64_t)(mix64(k) & (uint64_t)(S->cap - 1));
  while (S->slot[i]) {
    if (S->slot[i] == k) return;
    i = (i + 1) & (S->cap - 1);
  }
  S->slot[i] = k;
}

/* One-edit neighbourhood in the fixed enumeration order (reading):                 */
/*   substitutions (position ascending, new id ascending, skipping the same id),    */
/*   deletions (position ascending, only if K > 1),                                 */
/*   insertions (position 0..K ascending, id ascending, only if K < K_cap).         */
/* Repeats inside the list are kept here; the caller skips already-seen orders.     */
static int64_t neighbours1(Key p, int n_modes, int kcap, Key *out) {
  int K = key_len(p), m[MAXSEG], q[MAXSEG], i, j, id;
  int64_t n = 0;
  for (i = 0; i < K; ++i) m[i] = key_mode(p, i);
  for (i = 0; i < K; ++i)
    for (id = 0; id < n_modes; ++id) {
      if (id == m[i]) continue;
      for (j = 0; j < K; ++j) q[j] = m[j];
      q[i] = id;
      out[n++] = key_make(K, q);
    }
  if (K > 1)
    for (i = 0; i < K; ++i) {
      int t = 0;
      for (j = 0; j < K; ++j)
        if (j != i) q[t++] = m[j];
      out[n++] = key_make(K - 1, q);
    }
  if (K < kcap)
    for (i = 0; i <= K; ++i)
      for (id = 0; id < n_modes; ++id) {
        int t = 0;
        for (j = 0; j < i; ++j) q[t++] = m[j];
        q[t++] = id;
        for (j = i; j < K; ++j) q[t++] = m[j];
        out[n++] = key_make(K + 1, q);
      }
  return n;
}

/* r-edit neighbourhood: breadth-first over one-edit lists, first occurrence wins,  */
/* the order itself excluded.  r in {1, 2}.                                          */
static int64_t neighbours(Key p, int n_modes, int kcap, int r, Key *out, Key *tmp) {
  int64_t n1 = neighbours1(p, n_modes, kcap, out), n = 0, i, j;
  KeySet seen;
  if (r <= 1) {
    /* drop in-list repeats, keep first occurrence */
    set_init(&seen, n1 + 1);
    set_add(&seen, p);
    for (i = 0; i < n1; ++i)
      if (!set_has(&seen, out[i])) {
        set_add(&seen, out[i]);
        out[n++] = out[i];
      }
    free(seen.slot);
    return n;
  }
  {
    Key *lvl1 = (Key *)malloc(sizeof(Key) * (size_t)n1);
    int64_t m1 = 0;
    set_init(&seen, n1 * (int64_t)(2 * n_modes * (kcap + 1) + 8));
    set_add(&seen, p);
    for (i = 0; i < n1; ++i)
      if (!set_has(&seen, out[i])) {
        set_add(&seen, out[i]);
        lvl1[m1++] = out[i];
      }
    for (i = 0; i < m1; ++i) out[n++] = lvl1[i];
    for (i = 0; i < m1; ++i) {
      int64_t n2 = neighbours1(lvl1[i], n_modes, kcap, tmp);
      for (j = 0; j < n2; ++j)
        if (!set_has(&seen, tmp[j])) {
          set_add(&seen, tmp[j]);
          out[n++] = tmp[j];
        }
    }
    free(lvl1);
    free(seen.slot);
    return n;
  }
}

int64_t oracle_neighbours(uint64_t key, int32_t n_modes, int32_t kcap, int32_t radius, uint64_t *out) {
  Key *tmp = (Key *)malloc(sizeof(Key) * 4096);
  int64_t n = neighbours((Key)key, n_modes, kcap, radius, (Key *)out, tmp);
  free(tmp);
  return n;
}

typedef struct {
  int32_t kcap, seed_max_segments, radius, rounds, frontier_W, knots_per_segment, k_ref, n_total;
  int64_t batch_B, eval_budget;
  double mu_merit;
} OracleExpandParams;

typedef struct {
  Key key;
  double J, v, M;
} Entry;

/* ranking by (merit, key); NaN merit ranks as +inf */
static int cmp_entry_merit(const void *a, const void *b) {
  const Entry *x = (const Entry *)a, *y = (const Entry *)b;
  const double mx = isnan(x->M) ? INFINITY : x->M, my = isnan(y->M) ? INFINITY : y->M;
  if (mx < my) return -1;
  if (mx > my) return 1;
  return (x->key < y->key) ? -1 : (x->key > y->key) ? 1 : 0;
}

static double merit_of(double J, double v, double eps, double mu_merit) {
  double M;
  if (isnan(J) || isnan(v)) return INFINITY;
  M = J + mu_merit * fmax(v - eps, 0.0);
  return isnan(M) ? INFINITY : M;
}

/* Eq. (5) merit of one evaluated order, exported for the tests */
double oracle_merit(double J, double v, double eps, double mu_merit) { return merit_of(J, v, eps, mu_merit); }

/* knot allocation of an order: a fixed count per segment, or (if that is 0) a      */
/* total of n_total intervals split as evenly as possible, the remainder going to   */
/* the earliest segments.                                                           */
static void allocate_knots(int K, int per_seg, int n_total, int32_t *knots) {
  int j;
  for (j = 0; j < K; ++j) {
    if (per_seg > 0) knots[j] = per_seg;
    else knots[j] = n_total / K + ((j < n_total % K) ? 1 : 0);
  }
}

/* evaluate a list of keys on one instance with the given budget */
static void eval_keys(const Key *keys, int64_t n, const double *x0, const double *goal, double mu,
                      const OracleExpandParams *ep, const OracleParams *prm, int nthreads, double *J, double *v,
                      int32_t *stats) {
  int32_t *nseg = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n + 1));
  int32_t *modes = (int32_t *)calloc((size_t)(n + 1) * MAXSEG, sizeof(int32_t));
  int32_t *knots = (int32_t *)calloc((size_t)(n + 1) * MAXSEG, sizeof(int32_t));
  double *X0 = (double *)malloc(sizeof(double) * (size_t)(n + 1) * PNX);
  double *G = (double *)malloc(sizeof(double) * (size_t)(n + 1) * 3);
  double *I = (double *)malloc(sizeof(double) * (size_t)(n + 1));
  uint8_t *f = (uint8_t *)malloc((size_t)(n + 1));
  int64_t b;
  int i, nmax = 1;
  for (b = 0; b < n; ++b) {
    const int K = key_len(keys[b]);
    int tot = 0;
    nseg[b] = K;
    for (i = 0; i < K; ++i) modes[b * MAXSEG + i] = key_mode(keys[b], i);
    allocate_knots(K, ep->knots_per_segment, ep->n_total, &knots[b * MAXSEG]);
    for (i = 0; i < K; ++i) tot += knots[b * MAXSEG + i];
    if (tot > nmax) nmax = tot;
    for (i = 0; i < PNX; ++i) X0[b * PNX + i] = x0[i];
    for (i = 0; i < 3; ++i) G[b * 3 + i] = goal[i];
    I[b] = mu;
  }
  oracle_evaluate(n, MAXSEG, nmax, X0, G, I, nseg, modes, knots, NULL, prm, nthreads, J, v, f, NULL, stats);
  free(nseg); free(modes); free(knots); free(X0); free(G); free(I); free(f);
}

/* Greedy expansion with refinement.  Output: the best refined feasible order       */
/* (best_key = 0 if none), its refined cost and violation, and counters:            */
/* counters[0] = orders evaluated, [1] = rounds run, [2] = feasible orders found,     */
/* [3] = evaluation index (1-based, in round/batch order) of the first feasible one. */
/* The list of evaluated keys with (J, v) is returned in eval order if requested.    */
int oracle_expand(const double *x0, const double *goal, double mu, const OracleExpandParams *ep,
                  const OracleParams *prm_exp, const OracleParams *prm_ref, int32_t nthreads, uint64_t *best_key,
                  double *best_J, double *best_v, int64_t *counters, uint64_t *eval_keys_out,
                  double *eval_J_out, double *eval_v_out, int64_t eval_cap) {
  const int n_modes = 12;
  int64_t cap = ep->eval_budget + 16, nV = 0, nF = 0, i, j;
  Entry *V = (Entry *)malloc(sizeof(Entry) * (size_t)cap);
  Entry *R = (Entry *)malloc(sizeof(Entry) * (size_t)cap);
  Key *F = (Key *)malloc(sizeof(Key) * (size_t)(ep->batch_B + 16));
  Key *nb = (Key *)malloc(sizeof(Key) * 1000000);
  Key *tmp = (Key *)malloc(sizeof(Key) * 4096);
  double *J = (double *)malloc(sizeof(double) * (size_t)(ep->batch_B + 16));
  double *v = (double *)malloc(sizeof(double) * (size_t)(ep->batch_B + 16));
  KeySet seen;
  int s, K, q[MAXSEG];
  int64_t first_feasible = 0, n_feas = 0, rounds_run = 0;
  set_init(&seen, cap);
  /* seed: all orders with at most seed_max_segments segments, in key order */
  {
    int kmax = ep->seed_max_segments < ep->kcap ? ep->seed_max_segments : ep->kcap;
    for (K = 1; K <= kmax; ++K) {
      int64_t total = 1, c;
      for (i = 0; i < K; ++i) total *= n_modes;
      for (c = 0; c < total && nF < ep->batch_B && nF < ep->eval_budget; ++c) {
        int64_t t = c;
        for (i = K - 1; i >= 0; --i) {
          q[i] = (int)(t % n_modes);
          t /= n_modes;
        }
        F[nF++] = key_make(K, q);
      }
    }
    for (i = 0; i < nF; ++i) set_add(&seen, F[i]);
  }
  for (s = 0; nF > 0 && s <= ep->rounds; ++s) {
    int64_t room;
    eval_keys(F, nF, x0, goal, mu, ep, prm_exp, nthreads, J, v, NULL);
    ++rounds_run;
    for (i = 0; i < nF; ++i) {
      V[nV].key = F[i];
      V[nV].J = J[i];
      V[nV].v = v[i];
      V[nV].M = merit_of(J[i], v[i], prm_exp->eps_feas, ep->mu_merit);
      if (eval_keys_out && nV < eval_cap) {
        eval_keys_out[nV] = F[i];
        eval_J_out[nV] = J[i];
        eval_v_out[nV] = v[i];
      }
      if (v[i] <= prm_exp->eps_feas) {
        ++n_feas;
        if (!first_feasible) first_feasible = nV + 1;
      }
      ++nV;
    }
    nF = 0;
    if (s == ep->rounds) break;
    room = ep->batch_B;
    if (ep->eval_budget - nV < room) room = ep->eval_budget - nV;
    if (room <= 0) break;
    /* rank V and build the next batch */
    memcpy(R, V, sizeof(Entry) * (size_t)nV);
    qsort(R, (size_t)nV, sizeof(Entry), cmp_entry_merit);
    for (i = 0; i < nV && i < ep->frontier_W && nF < room; ++i) {
      int64_t n = neighbours(R[i].key, n_modes, ep->kcap, ep->radius, nb, tmp);
      for (j = 0; j < n && nF < room; ++j)
        if (!set_has(&seen, nb[j])) {
          set_add(&seen, nb[j]);
          F[nF++] = nb[j];
        }
    }
  }
  counters[0] = nV;
  counters[1] = rounds_run;
  counters[2] = n_feas;
  counters[3] = first_feasible;
  /* refinement: the k_ref feasible orders of smallest J (ties by key), re-solved   */
  /* from the schedule-derived start with the refinement budget                    */
  {
    int64_t nR = 0, nref;
    Key *rk;
    double *rJ, *rv;
    for (i = 0; i < nV; ++i)
      if (V[i].v <= prm_exp->eps_feas && isfinite(V[i].J)) {
        R[nR] = V[i];
        R[nR].M = V[i].J;
        ++nR;
      }
    qsort(R, (size_t)nR, sizeof(Entry), cmp_entry_merit);
    nref = nR < ep->k_ref ? nR : ep->k_ref;
    rk = (Key *)malloc(sizeof(Key) * (size_t)(nref + 1));
    rJ = (double *)malloc(sizeof(double) * (size_t)(nref + 1));
    rv = (double *)malloc(sizeof(double) * (size_t)(nref + 1));
    for (i = 0; i < nref; ++i) rk[i] = R[i].key;
    if (nref > 0) eval_keys(rk, nref, x0, goal, mu, ep, prm_ref, nthreads, rJ, rv, NULL);
    *best_key = 0;
    *best_J = NAN;
    *best_v = INFINITY;
    for (i = 0; i < nref; ++i) {
      if (!(rv[i] <= prm_ref->eps_feas) || !isfinite(rJ[i])) continue;
      if (*best_key == 0 || rJ[i] < *best_J || (rJ[i] == *best_J && rk[i] < *best_key)) {
        *best_key = rk[i];
        *best_J = rJ[i];
        *best_v = rv[i];
      }
    }
    free(rk); free(rJ); free(rv);
  }
  free(V); free(R); free(F); free(nb); free(tmp); free(J); free(v);
  free(seen.slot);
  return 0;
}

/* One batch-construction step of Alg. 1 on given merits: rank the evaluated orders by  */
/* (merit, key), traverse at most W of them, append their unseen r-edit neighbours in  */
/* enumeration order until `room` orders are admitted.  keys/merit: the evaluated set  */
/* V (n entries, merit NaN ranks as +inf).  Returns the number admitted (out_keys).      */
int64_t oracle_expand_next(int64_t n, const uint64_t *keys, const double *merit, int32_t n_modes, int32_t kcap,
                           int32_t radius, int32_t frontier_W, int64_t room, uint64_t *out_keys) {
  Entry *R = (Entry *)malloc(sizeof(Entry) * (size_t)(n + 1));
  Key *nb = (Key *)malloc(sizeof(Key) * 4000000);
  Key *tmp = (Key *)malloc(sizeof(Key) * 65536);
  KeySet seen;
  int64_t i, j, nF = 0;
  set_init(&seen, n + room + 16);
  for (i = 0; i < n; ++i) {
    R[i].key = keys[i];
    R[i].M = isnan(merit[i]) ? INFINITY : merit[i];
    R[i].J = R[i].v = 0.0;
    set_add(&seen, keys[i]);
  }
  qsort(R, (size_t)n, sizeof(Entry), cmp_entry_merit);
  for (i = 0; i < n && i < frontier_W && nF < room; ++i) {
    int64_t m = neighbours(R[i].key, n_modes, kcap, radius, nb, tmp);
    for (j = 0; j < m && nF < room; ++j)
      if (!set_has(&seen, nb[j])) {
        set_add(&seen, nb[j]);
        out_keys[nF++] = nb[j];
      }
  }
  free(R); free(nb); free(tmp); free(seen.slot);
  return nF;
}

/* Full enumeration of every order with 1..kcap segments (kmin..kcap if kmin > 1),  */
/* then the same refinement: the reference the expansion is compared with.          */
int oracle_enumerate(const double *x0, const double *goal, double mu, int32_t kmin, const OracleExpandParams *ep,
                     const OracleParams *prm_exp, const OracleParams *prm_ref, int32_t nthreads,
                     uint64_t *best_key, double *best_J, double *best_v, int64_t *n_eval) {
  const int n_modes = 12;
  int64_t total = 0, n = 0, i, c, nR = 0, nref;
  int K, q[MAXSEG];
  Key *keys;
  double *J, *v, *rJ, *rv;
  Entry *R;
  for (K = kmin; K <= ep->kcap; ++K) {
    int64_t t = 1;
    for (i = 0; i < K; ++i) t *= n_modes;
    total += t;
  }
  keys = (Key *)malloc(sizeof(Key) * (size_t)total);
  J = (double *)malloc(sizeof(double) * (size_t)total);
  v = (double *)malloc(sizeof(double) * (size_t)total);
  R = (Entry *)malloc(sizeof(Entry) * (size_t)total);
  for (K = kmin; K <= ep->kcap; ++K) {
    int64_t t = 1;
    for (i = 0; i < K; ++i) t *= n_modes;
    for (c = 0; c < t; ++c) {
      int64_t u = c;
      for (i = K - 1; i >= 0; --i) {
        q[i] = (int)(u % n_modes);
        u /= n_modes;
      }
      keys[n++] = key_make(K, q);
    }
  }
  eval_keys(keys, n, x0, goal, mu, ep, prm_exp, nthreads, J, v, NULL);
  for (i = 0; i < n; ++i)
    if (v[i] <= prm_exp->eps_feas && isfinite(J[i])) {
      R[nR].key = keys[i];
      R[nR].J = J[i];
      R[nR].v = v[i];
      R[nR].M = J[i];
      ++nR;
    }
  qsort(R, (size_t)nR, sizeof(Entry), cmp_entry_merit);
  nref = nR < ep->k_ref ? nR : ep->k_ref;
  rJ = (double *)malloc(sizeof(double) * (size_t)(nref + 1));
  rv = (double *)malloc(sizeof(double) * (size_t)(nref + 1));
  for (i = 0; i < nref; ++i) keys[i] = R[i].key;
  if (nref > 0) eval_keys(keys, nref, x0, goal, mu, ep, prm_ref, nthreads, rJ, rv, NULL);
  *best_key = 0;
  *best_J = NAN;
  *best_v = INFINITY;
  for (i = 0; i < nref; ++i) {
    if (!(rv[i] <= prm_ref->eps_feas) || !isfinite(rJ[i])) continue;
    if (*best_key == 0 || rJ[i] < *best_J || (rJ[i] == *best_J && keys[i] < *best_key)) {
      *best_key = keys[i];
      *best_J = rJ[i];
      *best_v = rv[i];
    }
  }
  *n_eval = n;
  free(keys); free(J); free(v); free(R); free(rJ); free(rv);
  return 0;
}
