/*
 * flip_oracle.c -- FP64 CPU oracle of the mode-conditioned TO for bimanual flipping
 * of a box in a vertical plane, and of its contact-mode language.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link, load or call this
 * file; only the tests and the smoke check do.  It shares no code, header, table or
 * constant generator with the HIP library.
 *
 * Plain and slow on purpose: the row Jacobians come from complex-step differentiation
 * of the residual code (exact to rounding for these analytic rows), every stage builds
 * dense matrices over its 25 arguments, the merit is re-evaluated in full at every trial
 * step, one sequence per thread.  Compile with -O2 -ffp-contract=off.
 *
 * What it follows: Eq. (2) for a fixed contact-mode order; the transcription of
 * Sec. III-C (defects x_{k+1} - F(x_k, u_k), masked rows in fixed slots); the local
 * solves S_k = H_k + rho I + A^T A / mu over w_k = (u_k, x_{k+1}) with the Cholesky PD
 * test and damping retries; trial step lengths; Eq. (4) scoring.  The task model is the
 * bimanual flip of Sec. IV-B (quasi-static wrench balance with the table reaction
 * eliminated, fingers on faces with Coulomb cones, support transitions by pivoting) on
 * the box of the benchmark configuration.  Readings of what the paper leaves open are
 * restated where they are used:
 *   - box W x H = 0.2 x 0.1 m, 0.5 kg, gravity -y, ground line y = 0; table friction
 *     mu_g per instance, finger friction mu_f = 0.5; dt = 0.1 s; explicit Euler;
 *   - state (px, py, th, vx, vy, om, s1, s2), controls (ax, ay, al, f1n, f1t, sd1, f2n,
 *     f2t, sd2): the pose moves with the twist, the twist with the accelerations, the
 *     finger face coordinates with their rates; forces do not drive the motion, they
 *     must balance gravity and the table reaction (quasi-static);
 *   - rows are stated non-dimensionally (forces / mg, moments / (mg W)), which is the
 *     row scaling of this task and also the unit of its score;
 *   - mode id = (f1 * 13 + f2) * 5 + g; finger code 0 free, 1 + 3 face + slip (slip 0
 *     stick, 1 slide+, 2 slide-); ground g: 0 stick, 1 slide+, 2 slide-, 3 pivot about
 *     the left corner of the support face (counter-clockwise), 4 pivot about the right
 *     corner (clockwise);
 *   - the support face starts as face 3 (the -y face, resting on the long side); a
 *     pivot run followed by a face-supported segment lands on the neighbouring face.
 */
#include <complex.h>
#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define FNX 8
#define FNU 9
#define FNW 17 /* stage unknowns (u_k, x_{k+1}) */
#define FNV 25 /* row arguments (x_k, u_k, x_{k+1}) */
#define FNE 17 /* equality slots */
#define FNI 15 /* inequality slots */
#define FNR 32
#define FNT 5 /* terminal rows */
#define FMAXSEG 6
#define FMAXN 512
#define FNMODES 845

static const double F_W = 0.2, F_H = 0.1, F_MASS = 0.5, F_G = 9.81, F_MUF = 0.5, F_DT = 0.1;
static const double F_WA = 1e-2, F_WF = 1.0, F_WS = 1e-2;
static double f_mg(void) { return F_MASS * F_G; }

/* face j of the box: outward normal n_j at angle j pi/2, counter-clockwise tangent t_j, */
/* distance from the centre h_j, half length l_j                                        */
static void face_geom(int j, double *n, double *t, double *h, double *l) {
  static const double NN[4][2] = {{1, 0}, {0, 1}, {-1, 0}, {0, -1}};
  n[0] = NN[j][0];
  n[1] = NN[j][1];
  t[0] = -n[1];
  t[1] = n[0];
  *h = (j % 2 == 0) ? 0.5 * F_W : 0.5 * F_H;
  *l = (j % 2 == 0) ? 0.5 * F_H : 0.5 * F_W;
}

typedef struct {
  double mu_g;
  int N;
  double x0[FNX], goal[2]; /* goal (px, th) */
  /* per interval */
  int fcode[FMAXN][2]; /* finger codes */
  int g[FMAXN];        /* ground mode */
  int fs[FMAXN];       /* support face */
  double ths[FMAXN];   /* support angle */
  int land[FMAXN];     /* first interval of a face-supported segment after a pivot */
} FlipProb;

typedef struct {
  int32_t al_max, gn_max, chol_retries, ls_trials, max_rejects, pad_;
  double mu0, mu_min, rho0, rho_min, rho_max, armijo_c1;
  double eta_star, omega_star, rc_star, eps_feas;
  double mu0_warm;
} FlipParams;

/* ------------------------------------------------------------------------------ */
/* Rows of interval k as complex functions of v = (x_k, u_k, x_{k+1}).               */
/* Slots 0..7 defects; 8..11 finger equalities (two per finger); 12..16 ground       */
/* equalities; 17..26 finger inequalities (five per finger); 27..31 ground           */
/* inequalities.  en[r] = 0 marks a masked slot (its value is 0).                    */
/* ------------------------------------------------------------------------------ */
typedef double complex cplx;

static void flip_rows_c(const FlipProb *P, int k, const cplx *v, cplx *c, int *en) {
  const double mg = f_mg(), dt = F_DT;
  const cplx *x = v, *u = v + FNX, *x1 = v + FNX + FNU;
  cplx cs = ccos(x[2]), sn = csin(x[2]);
  cplx Fw[2][2], tau[2], Fb[2][2];
  cplx rx, ry, tauF;
  int i, r;
  for (r = 0; r < FNR; ++r) {
    c[r] = 0;
    en[r] = 0;
  }
  /* defects */
  {
    const cplx rate[FNX] = {x[3], x[4], x[5], u[0], u[1], u[2], u[5], u[8]};
    for (i = 0; i < FNX; ++i) {
      c[i] = x1[i] - (x[i] + dt * rate[i]);
      en[i] = 1;
    }
  }
  /* fingers: body-frame force, world force, moment about the centre */
  for (i = 0; i < 2; ++i) {
    const int code = P->fcode[k][i];
    const cplx fn = u[3 + 3 * i], ft = u[4 + 3 * i], sd = u[5 + 3 * i], s = x[6 + i];
    const int e = 8 + 2 * i, q = 17 + 5 * i;
    if (code == 0) {
      Fb[i][0] = Fb[i][1] = 0;
      tau[i] = 0;
      c[e] = fn / mg;
      c[e + 1] = ft / mg;
      en[e] = en[e + 1] = 1;
    } else {
      const int face = (code - 1) / 3, slip = (code - 1) % 3;
      double n[2], t[2], h, l;
      face_geom(face, n, t, &h, &l);
      Fb[i][0] = -fn * n[0] + ft * t[0];
      Fb[i][1] = -fn * n[1] + ft * t[1];
      tau[i] = h * ft + s * fn; /* (h n + s t) x (-fn n + ft t) */
      c[q] = -fn / mg;
      en[q] = 1;
      if (slip == 0) {
        c[e] = sd;
        en[e] = 1;
        c[q + 1] = (ft - F_MUF * fn) / mg;
        c[q + 2] = (-ft - F_MUF * fn) / mg;
        en[q + 1] = en[q + 2] = 1;
      } else {
        const double sg = (slip == 1) ? 1.0 : -1.0;
        c[e] = (ft - sg * F_MUF * fn) / mg;
        en[e] = 1;
        c[q + 1] = -sg * sd;
        en[q + 1] = 1;
      }
      c[q + 3] = s - l;
      c[q + 4] = -s - l;
      en[q + 3] = en[q + 4] = 1;
    }
    Fw[i][0] = cs * Fb[i][0] - sn * Fb[i][1];
    Fw[i][1] = sn * Fb[i][0] + cs * Fb[i][1];
  }
  /* table reaction from the force balance */
  rx = -(Fw[0][0] + Fw[1][0]);
  ry = mg - (Fw[0][1] + Fw[1][1]);
  tauF = tau[0] + tau[1];
  c[27] = -ry / mg;
  en[27] = 1;
  {
    const int g = P->g[k];
    double n[2], t[2], h, l;
    face_geom(P->fs[k], n, t, &h, &l);
    if (g <= 2) {
      /* supported on face fs: pose held by a zero twist; the centre of pressure     */
      /* -(tauF + h rx) / ry lies on the support face                                */
      if (P->land[k]) {
        c[12] = x[2] - P->ths[k];
        en[12] = 1;
      }
      c[13] = x[5];
      c[14] = x[4];
      en[13] = en[14] = 1;
      c[28] = (tauF + h * rx - l * ry) / (mg * F_W);
      c[29] = (-tauF - h * rx - l * ry) / (mg * F_W);
      en[28] = en[29] = 1;
      if (g == 0) {
        c[15] = x[3];
        en[15] = 1;
        c[30] = (rx - P->mu_g * ry) / mg;
        c[31] = (-rx - P->mu_g * ry) / mg;
        en[30] = en[31] = 1;
      } else {
        const double sg = (g == 1) ? 1.0 : -1.0;
        c[15] = (rx + sg * P->mu_g * ry) / mg; /* friction opposes the sliding */
        en[15] = 1;
        c[30] = -sg * x[3];
        en[30] = 1;
      }
    } else {
      /* pivot about a corner of the support face: the corner keeps its place on the */
      /* ground, the moment about it balances, the reaction stays in its cone, the   */
      /* angle stays between the support and the landing orientation                 */
      const double dir = (g == 3) ? 1.0 : -1.0;
      const double cb[2] = {h * n[0] - dir * l * t[0], h * n[1] - dir * l * t[1]};
      const cplx cs1 = ccos(x1[2]), sn1 = csin(x1[2]);
      const cplx Pk = x[0] + cs * cb[0] - sn * cb[1];
      const cplx Pk1x = x1[0] + cs1 * cb[0] - sn1 * cb[1];
      const cplx Pk1y = x1[1] + sn1 * cb[0] + cs1 * cb[1];
      const cplx grav = mg * (cs * cb[0] - sn * cb[1]); /* -c x g_body */
      cplx mom = grav;
      for (i = 0; i < 2; ++i) mom += tau[i] - (cb[0] * Fb[i][1] - cb[1] * Fb[i][0]);
      c[12] = Pk1x - Pk;
      c[13] = Pk1y;
      c[14] = mom / (mg * F_W);
      en[12] = en[13] = en[14] = 1;
      c[28] = -dir * (x1[2] - P->ths[k]);
      c[29] = dir * (x1[2] - P->ths[k]) - 0.5 * M_PI;
      c[30] = (rx - P->mu_g * ry) / mg;
      c[31] = (-rx - P->mu_g * ry) / mg;
      en[28] = en[29] = en[30] = en[31] = 1;
    }
  }
}

/* real rows and their Jacobian by complex steps */
static void flip_rows(const FlipProb *P, int k, const double *v, double *c, double J[FNR][FNV], int *en) {
  const double hstep = 1e-30;
  cplx vc[FNV], cc[FNR];
  int j, r;
  for (j = 0; j < FNV; ++j) vc[j] = v[j];
  flip_rows_c(P, k, vc, cc, en);
  for (r = 0; r < FNR; ++r) c[r] = creal(cc[r]);
  if (!J) return;
  for (j = 0; j < FNV; ++j) {
    int e2[FNR];
    vc[j] = v[j] + I * hstep;
    flip_rows_c(P, k, vc, cc, e2);
    for (r = 0; r < FNR; ++r) J[r][j] = cimag(cc[r]) / hstep;
    vc[j] = v[j];
  }
}

/* terminal rows: (px, th) at the goal, zero twist */
static void flip_term(const FlipProb *P, const double *xN, double *c, double J[FNT][FNX]) {
  int r, j;
  c[0] = xN[0] - P->goal[0];
  c[1] = xN[2] - P->goal[1];
  c[2] = xN[3];
  c[3] = xN[4];
  c[4] = xN[5];
  if (!J) return;
  for (r = 0; r < FNT; ++r)
    for (j = 0; j < FNX; ++j) J[r][j] = 0.0;
  J[0][0] = J[1][2] = J[2][3] = J[3][4] = J[4][5] = 1.0;
}

/* stage cost dt [w_a |accel|^2 + w_f sum |f_i|^2 / (mg)^2 + w_s sum sd_i^2]; gradient */
/* and (diagonal) Hessian over u                                                      */
static double flip_cost(const double *u, double *gu, double *hu) {
  const double mg2 = f_mg() * f_mg();
  double w[FNU];
  double J = 0.0;
  int i;
  w[0] = w[1] = w[2] = F_WA;
  w[3] = w[4] = w[6] = w[7] = F_WF / mg2;
  w[5] = w[8] = F_WS;
  for (i = 0; i < FNU; ++i) {
    J += F_DT * w[i] * u[i] * u[i];
    if (gu) gu[i] = 2.0 * F_DT * w[i] * u[i];
    if (hu) hu[i] = 2.0 * F_DT * w[i];
  }
  return J;
}

/* ------------------------------------------------------------------------------ */
/* Sequence set-up: per-interval contact parameters from the mode order, with the    */
/* support bookkeeping of the pivots.  Returns 0 for an invalid order.               */
/* ------------------------------------------------------------------------------ */
static int flip_decode(int id, int *f1, int *f2, int *g) {
  if (id < 0 || id >= FNMODES) return 0;
  *g = id % 5;
  *f2 = (id / 5) % 13;
  *f1 = id / 65;
  return 1;
}

static int setup_flip(FlipProb *P, int nseg, const int32_t *modes, const int32_t *knots, const double *x0,
                      const double *goal, double mu_g) {
  int j, k = 0, i, fs = 3, prev_g = -1;
  double ths = 0.0;
  if (nseg < 1 || nseg > FMAXSEG || !(mu_g > 0.0) || !isfinite(mu_g)) return 0;
  for (i = 0; i < FNX; ++i)
    if (!isfinite(x0[i])) return 0;
  if (!isfinite(goal[0]) || !isfinite(goal[1])) return 0;
  P->mu_g = mu_g;
  for (i = 0; i < FNX; ++i) P->x0[i] = x0[i];
  P->goal[0] = goal[0];
  P->goal[1] = goal[1];
  for (j = 0; j < nseg; ++j) {
    int f1, f2, g, t;
    if (!flip_decode(modes[j], &f1, &f2, &g) || knots[j] < 1) return 0;
    if (g >= 3 && prev_g >= 3 && g != prev_g) return 0; /* a pivot run keeps its corner */
    if (g <= 2 && prev_g >= 3) {                        /* landing on the next face  */
      const int dir = (prev_g == 3) ? 1 : -1;
      fs = ((fs - dir) % 4 + 4) % 4;
      ths += dir * 0.5 * M_PI;
    }
    for (t = 0; t < knots[j]; ++t, ++k) {
      if (k >= FMAXN) return 0;
      P->fcode[k][0] = f1;
      P->fcode[k][1] = f2;
      P->g[k] = g;
      P->fs[k] = fs;
      P->ths[k] = ths;
      P->land[k] = (t == 0 && g <= 2 && prev_g >= 3) ? 1 : 0;
    }
    prev_g = g;
  }
  P->N = k;
  return 1;
}

/* ------------------------------------------------------------------------------ */
/* Kinematic initial guess (the construction the paper uses for its warm starts,     */
/* read as: follow the support chain).  Face-supported segments hold the pose (stick) */
/* or slide it 5 cm; a pivot run turns the box about its corner to the landing angle  */
/* (or to the goal angle when the order ends in it); twists and accelerations by      */
/* finite differences; contact fingers press with mg/2, sliding ones on the cone edge. */
/* ------------------------------------------------------------------------------ */
static void initial_guess_flip(const FlipProb *P, double *z) {
  const int N = P->N;
  double *pose = (double *)malloc(sizeof(double) * 3 * (N + 1));
  double *vel = (double *)malloc(sizeof(double) * 3 * (N + 1));
  double px = P->x0[0], py = P->x0[1], th = P->x0[2];
  int k = 0, i;
  pose[0] = px;
  pose[1] = py;
  pose[2] = th;
  while (k < N) {
    const int g = P->g[k];
    int e = k;
    if (g <= 2) {
      const double d = (g == 0) ? 0.0 : ((g == 1) ? 0.05 : -0.05);
      double n[2], t[2], h, l;
      int s;
      while (e < N && P->g[e] == g && !(e > k && P->land[e])) ++e;
      /* one segment of equal ground mode; consecutive face segments handled in turn */
      face_geom(P->fs[k], n, t, &h, &l);
      for (s = k + 1; s <= e; ++s) {
        const double a = (double)(s - k) / (double)(e - k);
        pose[3 * s + 0] = px + d * a;
        pose[3 * s + 1] = h;
        pose[3 * s + 2] = P->ths[k];
      }
      px += d;
      py = h;
      th = P->ths[k];
    } else {
      const double dir = (g == 3) ? 1.0 : -1.0;
      double n[2], t[2], h, l, cb[2], cw[2], th_end;
      int s;
      while (e < N && P->g[e] == g) ++e;
      face_geom(P->fs[k], n, t, &h, &l);
      cb[0] = h * n[0] - dir * l * t[0];
      cb[1] = h * n[1] - dir * l * t[1];
      cw[0] = px + cos(th) * cb[0] - sin(th) * cb[1];
      cw[1] = py + sin(th) * cb[0] + cos(th) * cb[1];
      if (e < N) {
        th_end = P->ths[k] + dir * 0.5 * M_PI;
      } else {
        const double lo = (dir > 0) ? P->ths[k] : P->ths[k] - 0.5 * M_PI;
        const double hi = (dir > 0) ? P->ths[k] + 0.5 * M_PI : P->ths[k];
        th_end = fmin(fmax(P->goal[1], lo), hi);
      }
      for (s = k + 1; s <= e; ++s) {
        const double a = (double)(s - k) / (double)(e - k);
        const double ts = th + (th_end - th) * a;
        pose[3 * s + 0] = cw[0] - (cos(ts) * cb[0] - sin(ts) * cb[1]);
        pose[3 * s + 1] = cw[1] - (sin(ts) * cb[0] + cos(ts) * cb[1]);
        pose[3 * s + 2] = ts;
      }
      px = pose[3 * e + 0];
      py = pose[3 * e + 1];
      th = pose[3 * e + 2];
    }
    k = e;
  }
  for (i = 0; i < 3; ++i) vel[i] = P->x0[3 + i];
  for (k = 1; k < N; ++k)
    for (i = 0; i < 3; ++i) vel[3 * k + i] = (pose[3 * (k + 1) + i] - pose[3 * k + i]) / F_DT;
  for (i = 0; i < 3; ++i) vel[3 * N + i] = 0.0;
  for (k = 0; k < N; ++k) {
    double *w = &z[k * FNW];
    int f;
    for (i = 0; i < 3; ++i) w[i] = (vel[3 * (k + 1) + i] - vel[3 * k + i]) / F_DT;
    for (f = 0; f < 2; ++f) {
      const int code = P->fcode[k][f];
      double fn = 0.0, ft = 0.0;
      if (code != 0) {
        const int slip = (code - 1) % 3;
        fn = 0.5 * f_mg();
        ft = (slip == 0) ? 0.0 : ((slip == 1) ? F_MUF * fn : -F_MUF * fn);
      }
      w[3 + 3 * f] = fn;
      w[4 + 3 * f] = ft;
      w[5 + 3 * f] = 0.0;
    }
    for (i = 0; i < 3; ++i) w[FNU + i] = pose[3 * (k + 1) + i];
    for (i = 0; i < 3; ++i) w[FNU + 3 + i] = vel[3 * (k + 1) + i];
    w[FNU + 6] = P->x0[6];
    w[FNU + 7] = P->x0[7];
  }
  free(pose);
  free(vel);
}

/* ------------------------------------------------------------------------------ */
/* Solver: the same augmented-Lagrangian / Gauss-Newton algorithm as the pushing     */
/* oracle, over the flip dimensions.                                                 */
/* ------------------------------------------------------------------------------ */
static void stage_args(const FlipProb *P, const double *z, int k, double *v) {
  int i;
  const double *xk = (k == 0) ? P->x0 : &z[(k - 1) * FNW + FNU];
  for (i = 0; i < FNX; ++i) v[i] = xk[i];
  for (i = 0; i < FNW; ++i) v[FNX + i] = z[k * FNW + i];
}

typedef struct {
  double *lam, *nu, lamT[FNT];
  double mu;
} Dual;

static double merit(const FlipProb *P, const double *z, const Dual *D) {
  double phi = 0.0, v[FNV], c[FNR], cT[FNT];
  int en[FNR], k, r;
  for (k = 0; k < P->N; ++k) {
    phi += flip_cost(&z[k * FNW], NULL, NULL);
    stage_args(P, z, k, v);
    flip_rows(P, k, v, c, NULL, en);
    for (r = 0; r < FNE; ++r)
      if (en[r]) phi += D->lam[k * FNE + r] * c[r] + c[r] * c[r] / (2.0 * D->mu);
    for (r = FNE; r < FNR; ++r)
      if (en[r]) {
        const double nu = D->nu[k * FNI + (r - FNE)];
        const double t = fmax(nu + c[r] / D->mu, 0.0);
        phi += 0.5 * D->mu * (t * t - nu * nu);
      }
  }
  flip_term(P, &z[(P->N - 1) * FNW + FNU], cT, NULL);
  for (r = 0; r < FNT; ++r) phi += D->lamT[r] * cT[r] + cT[r] * cT[r] / (2.0 * D->mu);
  return phi;
}

static double row_weight(int r, int en, double c, double lam, double nu, double mu, int *active) {
  if (!en) {
    *active = 0;
    return 0.0;
  }
  if (r < FNE) {
    *active = 1;
    return lam + c / mu;
  }
  {
    const double t = nu + c / mu;
    *active = (t > 0.0);
    return (t > 0.0) ? t : 0.0;
  }
}

static void gradient(const FlipProb *P, const double *z, const Dual *D, double *g) {
  double v[FNV], c[FNR], J[FNR][FNV], cT[FNT], JT[FNT][FNX], gu[FNU];
  int en[FNR], k, r, j, act;
  memset(g, 0, sizeof(double) * FNW * P->N);
  for (k = 0; k < P->N; ++k) {
    flip_cost(&z[k * FNW], gu, NULL);
    for (j = 0; j < FNU; ++j) g[k * FNW + j] += gu[j];
    stage_args(P, z, k, v);
    flip_rows(P, k, v, c, J, en);
    for (r = 0; r < FNR; ++r) {
      const double lam = (r < FNE) ? D->lam[k * FNE + r] : 0.0;
      const double nu = (r >= FNE) ? D->nu[k * FNI + r - FNE] : 0.0;
      const double w = row_weight(r, en[r], c[r], lam, nu, D->mu, &act);
      if (w == 0.0) continue;
      if (k > 0)
        for (j = 0; j < FNX; ++j) g[(k - 1) * FNW + FNU + j] += w * J[r][j];
      for (j = 0; j < FNW; ++j) g[k * FNW + j] += w * J[r][FNX + j];
    }
  }
  flip_term(P, &z[(P->N - 1) * FNW + FNU], cT, JT);
  for (r = 0; r < FNT; ++r) {
    const double w = D->lamT[r] + cT[r] / D->mu;
    for (j = 0; j < FNX; ++j) g[(P->N - 1) * FNW + FNU + j] += w * JT[r][j];
  }
}

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

/* one regularised Gauss-Newton step by the backward Riccati recursion over the       */
/* stages' 25 arguments y = (x_k, w_k); 1 on success, 0 on a failed factorisation     */
static int gn_step(const FlipProb *P, const double *z, const Dual *D, double rho, double *dz) {
  const int N = P->N;
  double Pm[FNX][FNX], pv[FNX];
  double *kk = (double *)malloc(sizeof(double) * N * FNW);
  double *KK = (double *)malloc(sizeof(double) * N * FNW * FNX);
  double v[FNV], c[FNR], J[FNR][FNV], cT[FNT], JT[FNT][FNX], gu[FNU], hu[FNU];
  int en[FNR], k, r, i, j, act, ok = 1;
  flip_term(P, &z[(N - 1) * FNW + FNU], cT, JT);
  for (i = 0; i < FNX; ++i) {
    pv[i] = 0;
    for (j = 0; j < FNX; ++j) Pm[i][j] = 0;
  }
  for (r = 0; r < FNT; ++r) {
    const double w = D->lamT[r] + cT[r] / D->mu;
    for (i = 0; i < FNX; ++i) {
      pv[i] += w * JT[r][i];
      for (j = 0; j < FNX; ++j) Pm[i][j] += JT[r][i] * JT[r][j] / D->mu;
    }
  }
  for (k = N - 1; k >= 0 && ok; --k) {
    double G[FNV][FNV], h[FNV], S[FNW * FNW], rhs[FNW];
    memset(G, 0, sizeof G);
    memset(h, 0, sizeof h);
    flip_cost(&z[k * FNW], gu, hu);
    for (i = 0; i < FNU; ++i) {
      h[FNX + i] += gu[i];
      G[FNX + i][FNX + i] += hu[i];
    }
    stage_args(P, z, k, v);
    flip_rows(P, k, v, c, J, en);
    for (r = 0; r < FNR; ++r) {
      const double lam = (r < FNE) ? D->lam[k * FNE + r] : 0.0;
      const double nu = (r >= FNE) ? D->nu[k * FNI + r - FNE] : 0.0;
      const double w = row_weight(r, en[r], c[r], lam, nu, D->mu, &act);
      for (i = 0; i < FNV; ++i) h[i] += w * J[r][i];
      if (act)
        for (i = 0; i < FNV; ++i)
          for (j = 0; j < FNV; ++j) G[i][j] += J[r][i] * J[r][j] / D->mu;
    }
    for (i = 0; i < FNX; ++i) {
      h[FNX + FNU + i] += pv[i];
      for (j = 0; j < FNX; ++j) G[FNX + FNU + i][FNX + FNU + j] += Pm[i][j];
    }
    for (i = 0; i < FNW; ++i)
      for (j = 0; j < FNW; ++j) S[i * FNW + j] = G[FNX + i][FNX + j] + (i == j ? rho : 0.0);
    if (!cholesky(FNW, S, FNW)) {
      ok = 0;
      break;
    }
    for (i = 0; i < FNW; ++i) rhs[i] = -h[FNX + i];
    chol_solve(FNW, S, FNW, rhs);
    for (i = 0; i < FNW; ++i) kk[k * FNW + i] = rhs[i];
    for (j = 0; j < FNX; ++j) {
      for (i = 0; i < FNW; ++i) rhs[i] = -G[FNX + i][j];
      chol_solve(FNW, S, FNW, rhs);
      for (i = 0; i < FNW; ++i) KK[(k * FNW + i) * FNX + j] = rhs[i];
    }
    {
      double Pn[FNX][FNX], pn[FNX];
      for (i = 0; i < FNX; ++i) {
        pn[i] = h[i];
        for (r = 0; r < FNW; ++r) pn[i] += G[i][FNX + r] * kk[k * FNW + r];
        for (j = 0; j < FNX; ++j) {
          Pn[i][j] = G[i][j];
          for (r = 0; r < FNW; ++r) Pn[i][j] += G[i][FNX + r] * KK[(k * FNW + r) * FNX + j];
        }
      }
      for (i = 0; i < FNX; ++i) {
        pv[i] = pn[i];
        for (j = 0; j < FNX; ++j) Pm[i][j] = 0.5 * (Pn[i][j] + Pn[j][i]);
      }
    }
  }
  if (ok) {
    double dx[FNX];
    for (j = 0; j < FNX; ++j) dx[j] = 0.0;
    for (k = 0; k < N; ++k) {
      for (i = 0; i < FNW; ++i) {
        double s = kk[k * FNW + i];
        for (j = 0; j < FNX; ++j) s += KK[(k * FNW + i) * FNX + j] * dx[j];
        dz[k * FNW + i] = s;
      }
      for (j = 0; j < FNX; ++j) dx[j] = dz[k * FNW + FNU + j];
    }
  }
  free(kk);
  free(KK);
  return ok;
}

static void scaled_viol(const FlipProb *P, const double *z, const Dual *D, double *vs, double *rc) {
  double v[FNV], c[FNR], cT[FNT];
  int en[FNR], k, r;
  double vi = 0.0, q = 0.0;
  for (k = 0; k < P->N; ++k) {
    stage_args(P, z, k, v);
    flip_rows(P, k, v, c, NULL, en);
    for (r = 0; r < FNR; ++r) {
      if (!en[r]) continue;
      if (r < FNE) vi = fmax(vi, fabs(c[r]));
      else {
        const double nu = D->nu[k * FNI + r - FNE];
        vi = fmax(vi, fmax(c[r], 0.0));
        q = fmax(q, fabs(fmin(-c[r], nu)));
      }
    }
  }
  flip_term(P, &z[(P->N - 1) * FNW + FNU], cT, NULL);
  for (r = 0; r < FNT; ++r) vi = fmax(vi, fabs(cT[r]));
  *vs = vi;
  *rc = q;
}

static void update_duals(const FlipProb *P, const double *z, Dual *D) {
  double v[FNV], c[FNR], cT[FNT];
  int en[FNR], k, r;
  for (k = 0; k < P->N; ++k) {
    stage_args(P, z, k, v);
    flip_rows(P, k, v, c, NULL, en);
    for (r = 0; r < FNR; ++r) {
      if (!en[r]) continue;
      if (r < FNE) D->lam[k * FNE + r] += c[r] / D->mu;
      else {
        double *nu = &D->nu[k * FNI + r - FNE];
        *nu = fmax(*nu + c[r] / D->mu, 0.0);
      }
    }
  }
  flip_term(P, &z[(P->N - 1) * FNW + FNU], cT, NULL);
  for (r = 0; r < FNT; ++r) D->lamT[r] += cT[r] / D->mu;
}

/* objective and violation, Eq. (4); the rows are already in the task's units */
static void score(const FlipProb *P, const double *z, double *Jout, double *vout) {
  double v[FNV], c[FNR], cT[FNT];
  int en[FNR], k, r;
  double obj = 0.0, vi = 0.0;
  for (k = 0; k < P->N; ++k) {
    obj += flip_cost(&z[k * FNW], NULL, NULL);
    stage_args(P, z, k, v);
    flip_rows(P, k, v, c, NULL, en);
    for (r = 0; r < FNR; ++r) {
      if (!en[r]) continue;
      vi = fmax(vi, (r < FNE) ? fabs(c[r]) : fmax(c[r], 0.0));
    }
  }
  flip_term(P, &z[(P->N - 1) * FNW + FNU], cT, NULL);
  for (r = 0; r < FNT; ++r) vi = fmax(vi, fabs(cT[r]));
  *Jout = obj;
  *vout = vi;
}

typedef struct {
  int al_iters, gn_iters, chol_fails, status;
} SolveStats;

static int all_finite(const double *a, int n) {
  int i;
  for (i = 0; i < n; ++i)
    if (!isfinite(a[i])) return 0;
  return 1;
}

static void solve(const FlipProb *P, const FlipParams *prm, int warm, double *z, SolveStats *st) {
  const int N = P->N, nz = N * FNW;
  double *g = (double *)malloc(sizeof(double) * nz);
  double *dz = (double *)malloc(sizeof(double) * nz);
  double *zt = (double *)malloc(sizeof(double) * nz);
  double *phi = (double *)malloc(sizeof(double) * (size_t)prm->ls_trials);
  Dual D;
  double eta, omega, rho = prm->rho0;
  int al, i;
  D.lam = (double *)calloc((size_t)N * FNE, sizeof(double));
  D.nu = (double *)calloc((size_t)N * FNI, sizeof(double));
  for (i = 0; i < FNT; ++i) D.lamT[i] = 0.0;
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
/* Batched evaluation, one sequence per thread.  x0 [B][8], goal [B][2] (px, th),    */
/* inst [B] (table friction), traj [B][nmax+1][17] rows (x_k, u_k), row N has u = 0. */
/* ------------------------------------------------------------------------------ */
typedef struct {
  int64_t B, next;
  int smax, nmax;
  const double *x0, *goal, *inst, *warm;
  const int32_t *nseg, *modes, *knots;
  const FlipParams *prm;
  double *cost, *viol, *traj;
  uint8_t *feas;
  int32_t *stats;
  pthread_mutex_t lock;
} FlipJob;

#define FROW (FNX + FNU)

static void eval_one(FlipJob *E, int64_t b) {
  FlipProb *P = (FlipProb *)malloc(sizeof(FlipProb));
  double *z;
  SolveStats st = {0, 0, 0, 2};
  double J = NAN, v = INFINITY;
  int k, i;
  int ok = setup_flip(P, E->nseg[b], &E->modes[b * E->smax], &E->knots[b * E->smax], &E->x0[b * FNX],
                      &E->goal[b * 2], E->inst[b]);
  if (ok && P->N > E->nmax) ok = 0;
  if (E->traj) memset(&E->traj[b * (E->nmax + 1) * FROW], 0, sizeof(double) * (size_t)(E->nmax + 1) * FROW);
  if (!ok) {
    E->cost[b] = NAN;
    E->viol[b] = INFINITY;
    E->feas[b] = 0;
    if (E->stats)
      for (i = 0; i < 4; ++i) E->stats[b * 4 + i] = (i == 3) ? 3 : 0;
    free(P);
    return;
  }
  z = (double *)malloc(sizeof(double) * P->N * FNW);
  if (E->warm) {
    const double *w = &E->warm[b * (E->nmax + 1) * FROW];
    for (k = 0; k < P->N; ++k) {
      for (i = 0; i < FNU; ++i) z[k * FNW + i] = w[k * FROW + FNX + i];
      for (i = 0; i < FNX; ++i) z[k * FNW + FNU + i] = w[(k + 1) * FROW + i];
    }
  } else {
    initial_guess_flip(P, z);
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
    double *T = &E->traj[b * (E->nmax + 1) * FROW];
    for (i = 0; i < FNX; ++i) T[i] = P->x0[i];
    for (k = 0; k < P->N; ++k) {
      for (i = 0; i < FNU; ++i) T[k * FROW + FNX + i] = z[k * FNW + i];
      for (i = 0; i < FNX; ++i) T[(k + 1) * FROW + i] = z[k * FNW + FNU + i];
    }
  }
  free(z);
  free(P);
}

static void *eval_worker(void *arg) {
  FlipJob *E = (FlipJob *)arg;
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

int flip_evaluate(int64_t B, int32_t smax, int32_t nmax, const double *x0, const double *goal, const double *inst,
                  const int32_t *nseg, const int32_t *modes, const int32_t *knots, const double *warm,
                  const FlipParams *prm, int32_t nthreads, double *cost, double *viol, uint8_t *feas, double *traj,
                  int32_t *stats) {
  FlipJob E;
  pthread_t th[256];
  int t;
  if (B < 0 || smax < 1 || smax > FMAXSEG || nmax < 1 || nmax > FMAXN || !prm) return -1;
  memset(&E, 0, sizeof E);
  E.B = B; E.smax = smax; E.nmax = nmax;
  E.x0 = x0; E.goal = goal; E.inst = inst; E.warm = warm;
  E.nseg = nseg; E.modes = modes; E.knots = knots; E.prm = prm;
  E.cost = cost; E.viol = viol; E.feas = feas; E.traj = traj; E.stats = stats;
  pthread_mutex_init(&E.lock, NULL);
  if (nthreads < 1) nthreads = 1;
  if (nthreads > 256) nthreads = 256;
  if (nthreads == 1 || B <= 1) {
    eval_worker(&E);
  } else {
    for (t = 0; t < nthreads; ++t) pthread_create(&th[t], NULL, eval_worker, &E);
    for (t = 0; t < nthreads; ++t) pthread_join(th[t], NULL);
  }
  pthread_mutex_destroy(&E.lock);
  return 0;
}

/* ------------------------------------------------------------------------------ */
/* Debug entry points for the pins.                                                  */
/* ------------------------------------------------------------------------------ */
static int debug_setup(FlipProb *P, int32_t nseg, const int32_t *modes, const int32_t *knots, const double *x0,
                       const double *goal, double mu_g) {
  return setup_flip(P, nseg, modes, knots, x0, goal, mu_g);
}

/* rows of interval k at arguments v [25]: c [32], J [32][25] (complex step), en [32] */
int flip_rows_at(int32_t nseg, const int32_t *modes, const int32_t *knots, const double *x0, const double *goal,
                 double mu_g, int32_t k, const double *v, double *c, double *J, int32_t *en) {
  FlipProb *P = (FlipProb *)malloc(sizeof(FlipProb));
  double Jl[FNR][FNV];
  int e[FNR], r, j;
  if (!debug_setup(P, nseg, modes, knots, x0, goal, mu_g) || k < 0 || k >= P->N) {
    free(P);
    return -1;
  }
  flip_rows(P, k, v, c, Jl, e);
  for (r = 0; r < FNR; ++r) {
    en[r] = e[r];
    for (j = 0; j < FNV; ++j) J[r * FNV + j] = Jl[r][j];
  }
  free(P);
  return 0;
}

/* rows of interval k evaluated in plain real arithmetic (no complex step) */
int flip_rows_real(int32_t nseg, const int32_t *modes, const int32_t *knots, const double *x0,
                   const double *goal, double mu_g, int32_t k, const double *v, double *c, int32_t *en) {
  FlipProb *P = (FlipProb *)malloc(sizeof(FlipProb));
  double Jl[FNR][FNV];
  int e[FNR], r;
  (void)Jl;
  if (!debug_setup(P, nseg, modes, knots, x0, goal, mu_g) || k < 0 || k >= P->N) {
    free(P);
    return -1;
  }
  flip_rows(P, k, v, c, NULL, e);
  for (r = 0; r < FNR; ++r) en[r] = e[r];
  free(P);
  return 0;
}

/* per-interval contact parameters: [N][6] = (f1, f2, g, fs, land, 0) and ths [N] */
int flip_setup_info(int32_t nseg, const int32_t *modes, const int32_t *knots, int32_t *info, double *ths,
                    int32_t *n_out) {
  FlipProb *P = (FlipProb *)malloc(sizeof(FlipProb));
  const double x0[FNX] = {0, 0.05, 0, 0, 0, 0, 0, 0}, goal[2] = {0, 0};
  int k;
  if (!debug_setup(P, nseg, modes, knots, x0, goal, 0.7)) {
    free(P);
    return -1;
  }
  for (k = 0; k < P->N; ++k) {
    info[k * 6 + 0] = P->fcode[k][0];
    info[k * 6 + 1] = P->fcode[k][1];
    info[k * 6 + 2] = P->g[k];
    info[k * 6 + 3] = P->fs[k];
    info[k * 6 + 4] = P->land[k];
    info[k * 6 + 5] = 0;
    ths[k] = P->ths[k];
  }
  *n_out = P->N;
  free(P);
  return 0;
}

/* schedule-derived initial guess z [N*17] */
int flip_initial(int32_t nseg, const int32_t *modes, const int32_t *knots, const double *x0, const double *goal,
                 double mu_g, double *z) {
  FlipProb *P = (FlipProb *)malloc(sizeof(FlipProb));
  if (!debug_setup(P, nseg, modes, knots, x0, goal, mu_g)) {
    free(P);
    return -1;
  }
  initial_guess_flip(P, z);
  free(P);
  return 0;
}

/* merit, gradient and Gauss-Newton step at (z, duals) */
int flip_merit_grad_step(int32_t nseg, const int32_t *modes, const int32_t *knots, const double *x0,
                         const double *goal, double mu_g, const double *z, const double *lam, const double *nu,
                         const double *lamT, double mu, double rho, double *phi, double *g, double *dz) {
  FlipProb *P = (FlipProb *)malloc(sizeof(FlipProb));
  Dual D;
  int i, ok;
  if (!debug_setup(P, nseg, modes, knots, x0, goal, mu_g)) {
    free(P);
    return -1;
  }
  D.lam = (double *)lam;
  D.nu = (double *)nu;
  for (i = 0; i < FNT; ++i) D.lamT[i] = lamT[i];
  D.mu = mu;
  *phi = merit(P, z, &D);
  gradient(P, z, &D, g);
  ok = gn_step(P, z, &D, rho, dz);
  free(P);
  return ok ? 0 : 1;
}

/* objective and violation of z */
int flip_score(int32_t nseg, const int32_t *modes, const int32_t *knots, const double *x0, const double *goal,
               double mu_g, const double *z, double *J, double *v) {
  FlipProb *P = (FlipProb *)malloc(sizeof(FlipProb));
  if (!debug_setup(P, nseg, modes, knots, x0, goal, mu_g)) {
    free(P);
    return -1;
  }
  score(P, z, J, v);
  free(P);
  return 0;
}

/* ------------------------------------------------------------------------------ */
/* Language of admissible orders (Sec. IV-B, transition rules, with the readings:    */
/* fingers never share a face; a finger changes face only through a free segment; a  */
/* pivot has at least one finger in contact; no two consecutive segments are equal;  */
/* consecutive pivots keep their direction; no finger touches the face on the table  */
/* (the support face while face-supported; the support and the landing face during a */
/* pivot); K <= 6).  Returns 1 if the order is admissible.                           */
/* ------------------------------------------------------------------------------ */
int flip_admissible(int32_t K, const int32_t *modes) {
  int j, fs = 3, prev_g = -1, pf[2] = {-1, -1}, prev_id = -1;
  if (K < 1 || K > FMAXSEG) return 0;
  for (j = 0; j < K; ++j) {
    int f[2], g, i, face[2];
    if (!flip_decode(modes[j], &f[0], &f[1], &g)) return 0;
    if (modes[j] == prev_id) return 0;
    if (g >= 3 && prev_g >= 3 && g != prev_g) return 0;
    if (g <= 2 && prev_g >= 3) {
      const int dir = (prev_g == 3) ? 1 : -1;
      fs = ((fs - dir) % 4 + 4) % 4;
    }
    for (i = 0; i < 2; ++i) face[i] = f[i] ? (f[i] - 1) / 3 : -1;
    if (face[0] >= 0 && face[0] == face[1]) return 0;
    if (g >= 3 && face[0] < 0 && face[1] < 0) return 0;
    for (i = 0; i < 2; ++i) {
      if (face[i] < 0) continue;
      if (face[i] == fs) return 0;
      if (g >= 3) {
        const int dir = (g == 3) ? 1 : -1;
        const int landing = ((fs - dir) % 4 + 4) % 4;
        if (face[i] == landing) return 0;
      }
      if (pf[i] >= 0 && pf[i] != face[i]) return 0;
    }
    for (i = 0; i < 2; ++i) pf[i] = face[i];
    prev_g = g;
    prev_id = modes[j];
  }
  return 1;
}

/* ================================================================================ */
/* Greedy contact-mode expansion (Alg. 1) over the flip language.                    */
/* ================================================================================ */
/* key = K << 60 | m_0 << 50 | ... | m_5 << 0 (10 bits per id): comparing keys       */
/* compares (K, m_0, m_1, ...) lexicographically.                                    */
typedef uint64_t FKey;

static FKey fkey_make(int K, const int *m) {
  FKey k = (FKey)K << 60;
  int i;
  for (i = 0; i < K; ++i) k |= (FKey)m[i] << (50 - 10 * i);
  return k;
}
static int fkey_len(FKey k) { return (int)(k >> 60); }
static int fkey_mode(FKey k, int i) { return (int)((k >> (50 - 10 * i)) & 1023u); }

static int admissible_key(FKey k) {
  int32_t m[FMAXSEG];
  int i, K = fkey_len(k);
  for (i = 0; i < K; ++i) m[i] = fkey_mode(k, i);
  return flip_admissible(K, m);
}

typedef struct {
  FKey *slot;
  int64_t cap;
} FSet;

static void fset_init(FSet *S, int64_t n) {
  int64_t c = 16;
  while (c < 2 * n + 16) c <<= 1;
  S->cap = c;
  S->slot = (FKey *)calloc((size_t)c, sizeof(FKey));
}
static uint64_t fmix(uint64_t x) {
  x ^= x >> 33; x *= 0xff51afd7ed558ccdULL;
  x ^= x >> 33; x *= 0xc4ceb9fe1a85ec53ULL;
  x ^= x >> 33;
  return x;
}
static int fset_has(const FSet *S, FKey k) {
  int64_t i = (int64_t)(fmix(k) & (uint64_t)(S->cap - 1));
  while (S->slot[i]) {
    if (S->slot[i] == k) return 1;
    i = (i + 1) & (S->cap - 1);
  }
  return 0;
}
static void fset_add(FSet *S, FKey k) {
  int64_t i = (int64_t)(fmix(k) & (uint64_t)(S->cap - 1));
  while (S->slot[i]) {
    if (S->slot[i] == k) return;
    i = (i + 1) & (S->cap - 1);
  }
  S->slot[i] = k;
}

/* one-edit list in enumeration order: substitutions (position, then id, skipping   */
/* the current id), deletions (position; K > 1), insertions (position 0..K, then id; */
/* K < kcap); in-list repeats kept                                                   */
static int64_t fneigh1(FKey p, int kcap, FKey *out) {
  int K = fkey_len(p), m[FMAXSEG], q[FMAXSEG], i, j, id;
  int64_t n = 0;
  for (i = 0; i < K; ++i) m[i] = fkey_mode(p, i);
  for (i = 0; i < K; ++i)
    for (id = 0; id < FNMODES; ++id) {
      if (id == m[i]) continue;
      for (j = 0; j < K; ++j) q[j] = m[j];
      q[i] = id;
      out[n++] = fkey_make(K, q);
    }
  if (K > 1)
    for (i = 0; i < K; ++i) {
      int t = 0;
      for (j = 0; j < K; ++j)
        if (j != i) q[t++] = m[j];
      out[n++] = fkey_make(K - 1, q);
    }
  if (K < kcap)
    for (i = 0; i <= K; ++i)
      for (id = 0; id < FNMODES; ++id) {
        int t = 0;
        for (j = 0; j < i; ++j) q[t++] = m[j];
        q[t++] = id;
        for (j = i; j < K; ++j) q[t++] = m[j];
        out[n++] = fkey_make(K + 1, q);
      }
  return n;
}

/* r-edit neighbourhood (r in {1, 2}, Sec. III-B): the one-edit list, then the        */
/* one-edit lists of its admissible entries in order (every intermediate order of a   */
/* two-edit path stays in the language); first occurrence wins, the order itself      */
/* excluded; only admissible orders are returned                                       */
static int64_t fneigh(FKey p, int kcap, int r, FKey *out) {
  int64_t cap1 = (int64_t)(2 * kcap + 2) * FNMODES + 16;
  FKey *l1 = (FKey *)malloc(sizeof(FKey) * (size_t)cap1);
  FKey *l2 = (FKey *)malloc(sizeof(FKey) * (size_t)cap1);
  int64_t n1 = fneigh1(p, kcap, l1), n = 0, i, j;
  FSet seen;
  fset_init(&seen, (r >= 2) ? n1 * cap1 / 4 + n1 : n1);
  fset_add(&seen, p);
  for (i = 0; i < n1; ++i)
    if (!fset_has(&seen, l1[i])) {
      fset_add(&seen, l1[i]);
      if (admissible_key(l1[i])) out[n++] = l1[i];
    }
  if (r >= 2)
    for (i = 0; i < n1; ++i) {
      int64_t n2;
      if (!admissible_key(l1[i])) continue;
      n2 = fneigh1(l1[i], kcap, l2);
      for (j = 0; j < n2; ++j)
        if (!fset_has(&seen, l2[j])) {
          fset_add(&seen, l2[j]);
          if (admissible_key(l2[j])) out[n++] = l2[j];
        }
    }
  free(l1);
  free(l2);
  free(seen.slot);
  return n;
}

typedef struct {
  FKey key;
  double J, v, M;
} FEntry;

static int cmp_fentry(const void *a, const void *b) {
  const FEntry *x = (const FEntry *)a, *y = (const FEntry *)b;
  const double mx = isnan(x->M) ? INFINITY : x->M, my = isnan(y->M) ? INFINITY : y->M;
  if (mx < my) return -1;
  if (mx > my) return 1;
  return (x->key < y->key) ? -1 : (x->key > y->key) ? 1 : 0;
}

/* seed: admissible orders of 1..kmax segments in key order, at most cap */
int64_t flip_seed(int32_t kmax, int64_t cap, uint64_t *out) {
  int64_t n = 0;
  int K, i, q[FMAXSEG];
  for (K = 1; K <= kmax && n < cap; ++K) {
    int64_t total = 1, c;
    for (i = 0; i < K; ++i) total *= FNMODES;
    for (c = 0; c < total && n < cap; ++c) {
      int64_t t = c;
      for (i = K - 1; i >= 0; --i) {
        q[i] = (int)(t % FNMODES);
        t /= FNMODES;
      }
      {
        FKey k = fkey_make(K, q);
        if (admissible_key(k)) out[n++] = k;
      }
    }
  }
  return n;
}

/* one batch-construction step: rank V by (merit, key), traverse at most W parents,   */
/* admit their unseen admissible r-edit neighbours in order until `room` are admitted */
int64_t flip_expand_next(int64_t n, const uint64_t *keys, const double *merit, int32_t kcap, int32_t radius,
                         int32_t frontier_W, int64_t room, uint64_t *out_keys) {
  FEntry *R = (FEntry *)malloc(sizeof(FEntry) * (size_t)(n + 1));
  int64_t cap = (radius >= 2) ? 40000000 : (int64_t)(2 * kcap + 2) * FNMODES + 16;
  FKey *nb = (FKey *)malloc(sizeof(FKey) * (size_t)cap);
  FSet seen;
  int64_t i, j, nF = 0;
  fset_init(&seen, n + room + 16);
  for (i = 0; i < n; ++i) {
    R[i].key = keys[i];
    R[i].M = isnan(merit[i]) ? INFINITY : merit[i];
    R[i].J = R[i].v = 0.0;
    fset_add(&seen, keys[i]);
  }
  qsort(R, (size_t)n, sizeof(FEntry), cmp_fentry);
  for (i = 0; i < n && i < frontier_W && nF < room; ++i) {
    int64_t m = fneigh(R[i].key, kcap, radius, nb);
    for (j = 0; j < m && nF < room; ++j)
      if (!fset_has(&seen, nb[j])) {
        fset_add(&seen, nb[j]);
        out_keys[nF++] = nb[j];
      }
  }
  free(R);
  free(nb);
  free(seen.slot);
  return nF;
}

typedef struct {
  int32_t kcap, seed_max_segments, radius, rounds, frontier_W, knots_per_segment, k_ref, n_total;
  int64_t batch_B, eval_budget;
  double mu_merit;
} FlipExpandParams;

static void fknots(int K, const FlipExpandParams *ep, int32_t *kn) {
  int j;
  for (j = 0; j < K; ++j)
    kn[j] = (ep->knots_per_segment > 0) ? ep->knots_per_segment
                                        : ep->n_total / K + ((j < ep->n_total % K) ? 1 : 0);
}

static void feval_keys(const FKey *keys, int64_t n, const double *x0, const double *goal, double mu_g,
                       const FlipExpandParams *ep, const FlipParams *prm, int nthreads, double *J, double *v) {
  int32_t *nseg = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n + 1));
  int32_t *modes = (int32_t *)calloc((size_t)(n + 1) * FMAXSEG, sizeof(int32_t));
  int32_t *kn = (int32_t *)calloc((size_t)(n + 1) * FMAXSEG, sizeof(int32_t));
  double *X0 = (double *)malloc(sizeof(double) * (size_t)(n + 1) * FNX);
  double *G = (double *)malloc(sizeof(double) * (size_t)(n + 1) * 2);
  double *Iv = (double *)malloc(sizeof(double) * (size_t)(n + 1));
  uint8_t *f = (uint8_t *)malloc((size_t)(n + 1));
  int64_t b;
  int i, nmax = 1;
  for (b = 0; b < n; ++b) {
    const int K = fkey_len(keys[b]);
    int tot = 0;
    nseg[b] = K;
    for (i = 0; i < K; ++i) modes[b * FMAXSEG + i] = fkey_mode(keys[b], i);
    fknots(K, ep, &kn[b * FMAXSEG]);
    for (i = 0; i < K; ++i) tot += kn[b * FMAXSEG + i];
    if (tot > nmax) nmax = tot;
    for (i = 0; i < FNX; ++i) X0[b * FNX + i] = x0[i];
    G[b * 2 + 0] = goal[0];
    G[b * 2 + 1] = goal[1];
    Iv[b] = mu_g;
  }
  flip_evaluate(n, FMAXSEG, nmax, X0, G, Iv, nseg, modes, kn, NULL, prm, nthreads, J, v, f, NULL, NULL);
  free(nseg); free(modes); free(kn); free(X0); free(G); free(Iv); free(f);
}

/* Greedy expansion with refinement on one instance: counters = (evaluated, rounds,   */
/* feasible found, 1-based evaluation index of the first feasible order); the        */
/* evaluated keys with (J, v) in evaluation order if eval_keys_out is given.          */
int flip_expand(const double *x0, const double *goal, double mu_g, const FlipExpandParams *ep,
                const FlipParams *prm_exp, const FlipParams *prm_ref, int32_t nthreads, uint64_t *best_key,
                double *best_J, double *best_v, int64_t *counters, uint64_t *eval_keys_out, double *eval_J_out,
                double *eval_v_out, int64_t eval_cap) {
  int64_t cap = ep->eval_budget + 16, nV = 0, nF = 0, i;
  FEntry *V = (FEntry *)malloc(sizeof(FEntry) * (size_t)cap);
  FEntry *R = (FEntry *)malloc(sizeof(FEntry) * (size_t)cap);
  FKey *F = (FKey *)malloc(sizeof(FKey) * (size_t)(ep->batch_B + 16));
  double *J = (double *)malloc(sizeof(double) * (size_t)(ep->batch_B + 16));
  double *v = (double *)malloc(sizeof(double) * (size_t)(ep->batch_B + 16));
  int s;
  int64_t first_feasible = 0, n_feas = 0, rounds_run = 0;
  {
    const int kmax = ep->seed_max_segments < ep->kcap ? ep->seed_max_segments : ep->kcap;
    int64_t lim = ep->batch_B < ep->eval_budget ? ep->batch_B : ep->eval_budget;
    nF = flip_seed(kmax, lim, F);
  }
  for (s = 0; nF > 0 && s <= ep->rounds; ++s) {
    int64_t room;
    feval_keys(F, nF, x0, goal, mu_g, ep, prm_exp, nthreads, J, v);
    ++rounds_run;
    for (i = 0; i < nF; ++i) {
      double M = NAN;
      if (!isnan(J[i]) && !isnan(v[i])) M = J[i] + ep->mu_merit * fmax(v[i] - prm_exp->eps_feas, 0.0);
      V[nV].key = F[i];
      V[nV].J = J[i];
      V[nV].v = v[i];
      V[nV].M = isnan(M) ? INFINITY : M;
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
    {
      uint64_t *keys = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)nV);
      double *mer = (double *)malloc(sizeof(double) * (size_t)nV);
      for (i = 0; i < nV; ++i) {
        keys[i] = V[i].key;
        mer[i] = V[i].M;
      }
      nF = flip_expand_next(nV, keys, mer, ep->kcap, ep->radius, ep->frontier_W, room, F);
      free(keys);
      free(mer);
    }
  }
  counters[0] = nV;
  counters[1] = rounds_run;
  counters[2] = n_feas;
  counters[3] = first_feasible;
  {
    int64_t nR = 0, nref;
    FKey *rk;
    double *rJ, *rv;
    for (i = 0; i < nV; ++i)
      if (V[i].v <= prm_exp->eps_feas && isfinite(V[i].J)) {
        R[nR] = V[i];
        R[nR].M = V[i].J;
        ++nR;
      }
    qsort(R, (size_t)nR, sizeof(FEntry), cmp_fentry);
    nref = nR < ep->k_ref ? nR : ep->k_ref;
    rk = (FKey *)malloc(sizeof(FKey) * (size_t)(nref + 1));
    rJ = (double *)malloc(sizeof(double) * (size_t)(nref + 1));
    rv = (double *)malloc(sizeof(double) * (size_t)(nref + 1));
    for (i = 0; i < nref; ++i) rk[i] = R[i].key;
    if (nref > 0) feval_keys(rk, nref, x0, goal, mu_g, ep, prm_ref, nthreads, rJ, rv);
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
  free(V); free(R); free(F); free(J); free(v);
  return 0;
}
