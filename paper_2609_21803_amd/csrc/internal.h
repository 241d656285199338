// internal.h -- definitions shared by the evaluator and the expansion (not part of the ABI).
#pragma once
#include <hip/hip_runtime.h>

#include <string>

#include "../../include/comet.h"
#include "push_model.h"

namespace comet {

constexpr int MAXSEG = 6;        // segments per order: pushing, timed pushing and flipping
constexpr int MAXSEG_FREE = 8;   // pushing with free motion (its 16 ids pack into 4-bit key fields)
constexpr int MAXN = 512;
constexpr int MAX_TRIALS = 16;
constexpr int WAVE = 64;
constexpr int MAX_TYPES = 16;   // row-scale types of any pushing model

struct DevParams {
  int al_max, gn_max, chol_retries, ls_trials, max_rejects;
  double mu0, mu_min, rho0, rho_min, rho_max, armijo_c1, eta_star, omega_star, rc_star, eps_feas;
  double mu0_warm;
};

struct EvalArgs {
  int64_t B;
  int smax, nmax;                 // segment slots per sequence, max intervals (work-space rows)
  int64_t S;                      // slot stride of the work space
  const float* x0;
  const float* goal;
  const float* inst;
  const int* nseg;
  const int* modes;
  const int* knots;
  const float* warm;
  float* cost;
  float* viol;
  uint8_t* feas;
  float* traj;
  int* stats;
  double* zd;                     // [row][NW][S]  (u_k, x_{k+1})
  float* lam;                     // [row][NE][S]
  float* nu;                      // [row][NI][S]
  float* gains;                   // [row][NW + NW NX][S] (k, K row-major NW x NX)
  float* dz;                      // [row][NW][S]
  uint8_t* code;                  // [row][S]
  const int64_t* Bdev;            // batch size read from device memory (graph capture), or null
  int inst_stride;                // 1: x0/goal/inst per sequence, 0: one instance for all
  double* cost64;                 // optional double-precision cost / violation outputs
  double* viol64;
  unsigned long long* t_first;    // optional: earliest wall-clock tick of a feasible finish
  const int* order;               // queue order of the sequences (null = identity)
  unsigned long long* qhead;      // work-queue head
  unsigned* err;
  DevParams prm;
  double inv_scale[MAX_TYPES];
};

// One evaluation launch: inputs, outputs and where the batch size lives.
struct EvalLaunch {
  int64_t B = 0;                   // host batch size (ignored if B_dev is set)
  const int64_t* B_dev = nullptr;  // device batch size (for captured graphs)
  int64_t B_max = 0;               // upper bound of the batch size (grid sizing)
  const float *x0 = nullptr, *goal = nullptr, *inst = nullptr;
  int inst_stride = 1;
  const int32_t *nseg = nullptr, *modes = nullptr, *knots = nullptr;
  const float* warm = nullptr;
  int refine = 0;
  float *cost = nullptr, *viol = nullptr;
  uint8_t* feas = nullptr;
  float* traj = nullptr;
  int32_t* stats = nullptr;
  double *cost64 = nullptr, *viol64 = nullptr;
  unsigned long long* t_first = nullptr;
  bool no_sort = false;            // keep the caller's order in the work queue
};

}  // namespace comet

struct comet_expand_ws;  // expansion work space (expand.hip)

struct comet_ctx {
  int task;
  comet_solver_params prm;
  int64_t max_batch, S;
  int max_segments, max_intervals;
  int device;
  double scale[comet::MAX_TYPES];
  double* zd = nullptr;
  float* lam = nullptr;
  float* nu = nullptr;
  float* gains = nullptr;
  float* dz = nullptr;
  uint8_t* code = nullptr;
  unsigned* err = nullptr;
  unsigned long long* qhead = nullptr;
  int* hist = nullptr;
  int* order = nullptr;
  hipEvent_t ev0 = nullptr, ev1 = nullptr;
  bool timed = false;
  int n_cu = 0, occ_blocks_per_cu = 1;
  comet_schedule sched{0, 1};   // occupancy limit, length-sorted queue
  hipStream_t gstream = nullptr;   // internal stream for captured graphs
  comet_expand_ws* xws = nullptr;
  double* fws = nullptr;      // flip task work space (FP64 per interval)
  int* fcode = nullptr;       // flip task packed contact parameters per interval
  std::string msg;
};


namespace comet {
comet_status launch_evaluate(comet_ctx* c, hipStream_t s, const EvalLaunch& L);
// flip task (flip.hip)
comet_status flip_create_ws(comet_ctx* c);
void flip_destroy_ws(comet_ctx* c);
comet_status launch_flip(comet_ctx* c, hipStream_t s, const EvalLaunch& L);
// learned network hooks (mlp.hip)
int mlp_in_dim(const comet_mlp* m);
int mlp_out_dim(const comet_mlp* m);
int mlp_warm_segments(const comet_mlp* m);   // segments the warm-start block holds
int mlp_task_segments(int task);             // segments the task's encodings hold (6, free motion 8)
int mlp_task_in_dim(int task);               // smallest in_dim of the task's encoding
int mlp_task_out_dim(int task);              // smallest out_dim of the task's warm-start block
long long mlp_max_batch(const comet_mlp* m);
const float* mlp_output(const comet_mlp* m);
void mlp_forward(comet_mlp* m, hipStream_t s, int B, const long long* B_dev);
void mlp_encode_dev(comet_mlp* m, int task, hipStream_t s, long long Bmax, const long long* B_dev, const float* x0,
                    const float* goal, const float* inst, int inst_stride, const int32_t* nseg, const int32_t* modes,
                    const int32_t* knots, int smax);
void mlp_decode_warm_dev(comet_mlp* m, int task, hipStream_t s, long long Bmax, const long long* B_dev,
                         const float* x0, int inst_stride, const int32_t* nseg, const int32_t* modes,
                         const int32_t* knots, int smax, int nmax, float* warm);
comet_status fail_msg(comet_ctx* c, comet_status st, const std::string& m);
// failure of a call without a context: the message is kept per thread (comet_last_error(NULL))
comet_status fail_global(comet_status st, const std::string& m);
void destroy_expand_ws(comet_ctx* c);
}  // namespace comet
