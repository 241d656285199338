/* Driver for sanitizer builds of the FP64 oracles (test infrastructure, CPU only).
 *
 * Compiled together with one oracle source (-DPUSH includes the pushing oracle, with
 * -DPUSH_TIMED its optimised-timing problem, -DFLIP
 * the flipping oracle, -DFREE the free-motion pushing oracle, with -DFREE_TIMED its
 * optimised-timing build) under AddressSanitizer + UndefinedBehaviorSanitizer or
 * ThreadSanitizer.  Reads a batch from a binary file, solves it with the oracle on
 * `nthreads` threads (and, with `expand` set, runs one greedy expansion on the batch's
 * first instance), and writes the results to a binary file for comparison with the
 * plain build.
 *
 * Input:  int64 B; int32 smax, nmax, nthreads, expand; double x0[B*NXD], goal[B*NGD],
 *         inst[B]; int32 nseg[B], modes[B*smax], knots[B*smax].
 * Output: double cost[B], viol[B]; uint8 feas[B]; int32 stats[B*4]; then, with expand,
 *         uint64 best key; double best J, best v; int64 counters[4] (free motion: int64 n,
 *         uint64 seed keys[n], int64 m, uint64 batch keys[m]).
 */
#include <stdio.h>
#include <stdlib.h>

#ifdef PUSH
#include "../../oracle/comet_oracle.c"
#define NXD 4
#define NGD 3
typedef OracleParams DrvParams;
#define EVALUATE oracle_evaluate
#define EXPAND oracle_expand
typedef OracleExpandParams DrvExpand;
#elif defined(FREE)
/* free-motion pushing; with -DFREE_TIMED the optimised-timing build of the same source */
#include "../../oracle/free_oracle.c"
#define NXD 5
#define NGD 3
typedef QParams DrvParams;
#define EVALUATE free_evaluate
#else
#include "../../oracle/flip_oracle.c"
#define NXD 8
#define NGD 2
typedef FlipParams DrvParams;
#define EVALUATE flip_evaluate
#define EXPAND flip_expand
typedef FlipExpandParams DrvExpand;
#endif

static void *read_n(FILE *f, size_t sz, size_t n) {
  void *p = calloc(n ? n : 1, sz);
  if (!p || fread(p, sz, n, f) != n) {
    fprintf(stderr, "short input\n");
    exit(2);
  }
  return p;
}

int main(int argc, char **argv) {
  FILE *f, *g;
  int64_t B;
  int32_t hdr[4];
  double *x0, *goal, *inst, *cost, *viol, *traj;
  int32_t *nseg, *modes, *knots, *stats;
  uint8_t *feas;
  DrvParams prm;
  if (argc != 3 || !(f = fopen(argv[1], "rb"))) return 2;
  if (fread(&B, 8, 1, f) != 1 || fread(hdr, 4, 4, f) != 4) return 2;
  x0 = (double *)read_n(f, 8, (size_t)B * NXD);
  goal = (double *)read_n(f, 8, (size_t)B * NGD);
  inst = (double *)read_n(f, 8, (size_t)B);
  nseg = (int32_t *)read_n(f, 4, (size_t)B);
  modes = (int32_t *)read_n(f, 4, (size_t)B * hdr[0]);
  knots = (int32_t *)read_n(f, 4, (size_t)B * hdr[0]);
  fclose(f);
  memset(&prm, 0, sizeof prm);
  prm.al_max = 20; prm.gn_max = 10; prm.chol_retries = 6; prm.ls_trials = 8; prm.max_rejects = 4;
  prm.mu0 = 1e-2; prm.mu_min = 1e-4; prm.rho0 = 1e-4; prm.rho_min = 1e-8; prm.rho_max = 1e8;
  prm.armijo_c1 = 1e-4; prm.eta_star = 1e-6; prm.omega_star = 1e-4; prm.rc_star = 1e-6;
  prm.eps_feas = 1e-5; prm.mu0_warm = 1e-4;
#if defined(PUSH_TIMED)
  prm.timed = 1;
#endif
  cost = (double *)calloc((size_t)B, 8);
  viol = (double *)calloc((size_t)B, 8);
  feas = (uint8_t *)calloc((size_t)B, 1);
  stats = (int32_t *)calloc((size_t)B * 4, 4);
  traj = (double *)calloc((size_t)B * (hdr[1] + 1) * 17, 8);
  if (EVALUATE(B, hdr[0], hdr[1], x0, goal, inst, nseg, modes, knots, NULL, &prm, hdr[2], cost, viol, feas, traj,
               stats) != 0)
    return 3;
  if (!(g = fopen(argv[2], "wb"))) return 2;
  fwrite(cost, 8, (size_t)B, g);
  fwrite(viol, 8, (size_t)B, g);
  fwrite(feas, 1, (size_t)B, g);
  fwrite(stats, 4, (size_t)B * 4, g);
#ifdef FREE
  /* the free-motion oracle has no whole-search driver: with `expand`, its language pieces
   * instead -- the seed of up to four segments, then one batch step (kcap 6, r = 2, W = 16,
   * room 4096) on merits (7919 i mod 1000) / 1000 */
  if (hdr[3]) {
    uint64_t *sk = (uint64_t *)calloc(2048, 8), *nk = (uint64_t *)calloc(4096, 8);
    int64_t ns = free_seed(4, 2048, sk), nn, i;
    double *mer = (double *)calloc((size_t)ns, 8);
    for (i = 0; i < ns; ++i) mer[i] = (double)((i * 7919) % 1000) / 1000.0;
    nn = free_expand_next(ns, sk, mer, 6, 2, 16, 4096, nk);
    fwrite(&ns, 8, 1, g);
    fwrite(sk, 8, (size_t)ns, g);
    fwrite(&nn, 8, 1, g);
    fwrite(nk, 8, (size_t)nn, g);
    free(sk); free(nk); free(mer);
  }
#else
  if (hdr[3]) {
    DrvExpand ep;
    DrvParams ref = prm;
    uint64_t key = 0;
    double J = 0, v = 0;
    int64_t ctr[4] = {0, 0, 0, 0};
    memset(&ep, 0, sizeof ep);
    ep.kcap = 2; ep.seed_max_segments = 1; ep.radius = 2; ep.rounds = 1; ep.frontier_W = 8;
    ep.knots_per_segment = 5; ep.k_ref = 4; ep.batch_B = 300; ep.eval_budget = 900; ep.mu_merit = 100.0;
    ref.al_max = 40;
    ref.gn_max = 25;
    EXPAND(x0, goal, inst[0], &ep, &prm, &ref, hdr[2], &key, &J, &v, ctr, NULL, NULL, NULL, 0);
    fwrite(&key, 8, 1, g);
    fwrite(&J, 8, 1, g);
    fwrite(&v, 8, 1, g);
    fwrite(ctr, 8, 4, g);
  }
#endif
  fclose(g);
  free(x0); free(goal); free(inst); free(nseg); free(modes); free(knots);
  free(cost); free(viol); free(feas); free(stats); free(traj);
  return 0;
}
