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
#include <mutex>
#include <string>
#include <vector>

#include "internal.h"
#include "keys.h"

namespace comet {

__device__ inline int wave_max(int v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v = max(v, __shfl_xor(v, o));
  return v;
}

__device__ inline bool wave_any(bool p) { return __ballot(p) != 0; }

namespace fixed_step {
using namespace push;
#include "push_solver.inc"
}  // namespace fixed_step

namespace timed_step {
using namespace push_timed;
#include "push_solver.inc"
}  // namespace timed_step

namespace free_step {
constexpr int MAXSEG = MAXSEG_FREE;   // orders of up to eight segments
using namespace push_free;
#define PUSH_MODEL_FREE 1
#include "push_solver.inc"
#undef PUSH_MODEL_FREE
}  // namespace free_step

namespace free_timed_step {
constexpr int MAXSEG = MAXSEG_FREE;   // orders of up to eight segments
using namespace push_free_timed;
#define PUSH_MODEL_FREE 1
#include "push_solver.inc"
#undef PUSH_MODEL_FREE
}  // namespace free_timed_step

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
  // each count is clamped to nmax + 1 and the sum saturates there, so it cannot wrap
  const int cap = A.nmax + 1;
  int N = 0;
  for (int j = 0; j < K; ++j) N = min(N + min(max(A.knots[b * A.smax + j], 0), cap), cap);
  return N;
}

// Counts per length are gathered in LDS first and added to the global bins once per block
// and length: a batch of equal lengths would otherwise serialise every order's atomic on
// one address.
__global__ void k_queue_hist(EvalArgs A, int* hist, int nbins) {
  __shared__ int lh[MAXN + 2];
  for (int i = threadIdx.x; i < nbins; i += blockDim.x) lh[i] = 0;
  __syncthreads();
  const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t Bn = A.Bdev ? *A.Bdev : A.B;
  if (b < Bn) atomicAdd(&lh[seq_len(A, b)], 1);
  __syncthreads();
  for (int i = threadIdx.x; i < nbins; i += blockDim.x)
    if (lh[i]) atomicAdd(&hist[i], lh[i]);
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

// each block reserves one range per length in the bins' running offsets and places its
// orders in it by their rank within the block
__global__ void k_queue_scatter(EvalArgs A, int* hist, int* order, int nbins) {
  __shared__ int lh[MAXN + 2];
  __shared__ int base[MAXN + 2];
  for (int i = threadIdx.x; i < nbins; i += blockDim.x) lh[i] = 0;
  __syncthreads();
  const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t Bn = A.Bdev ? *A.Bdev : A.B;
  int len = 0, rank = 0;
  if (b < Bn) {
    len = seq_len(A, b);
    rank = atomicAdd(&lh[len], 1);
  }
  __syncthreads();
  for (int i = threadIdx.x; i < nbins; i += blockDim.x)
    if (lh[i]) base[i] = atomicAdd(&hist[i], lh[i]);
  __syncthreads();
  if (b < Bn) order[base[len] + rank] = (int)b;
}

}  // namespace comet

// ==================================================================================
// Host side: context, row scales, C ABI.
// ==================================================================================
namespace {

comet_status fail(comet_ctx* c, comet_status s, const std::string& m) { return comet::fail_msg(c, s, m); }

}  // namespace

namespace comet {

comet_status fail_msg(comet_ctx* c, comet_status st, const std::string& m) {
  if (c) c->msg = m;
  return st;
}

thread_local std::string g_msg;   // last failure of a call without a context

comet_status fail_global(comet_status st, const std::string& m) {
  g_msg = m;
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
  for (int t = 0; t < MAX_TYPES; ++t) A.inv_scale[t] = 1.0 / c->scale[t];
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
    hipLaunchKernelGGL(k_queue_hist, dim3(gb), dim3(256), 0, s, A, c->hist, nbins);
    hipLaunchKernelGGL(k_queue_scan, dim3(1), dim3(64), 0, s, c->hist, nbins);
    hipLaunchKernelGGL(k_queue_scatter, dim3(gb), dim3(256), 0, s, A, c->hist, c->order, nbins);
  }
  if (timed && c->ev0) (void)hipEventRecord(c->ev0, s);
  if (c->task == COMET_TASK_PUSH_TIMED)
    hipLaunchKernelGGL(timed_step::k_push_solve, dim3(grid), dim3(WAVE), 0, s, A);
  else if (c->task == COMET_TASK_PUSH_FREE)
    hipLaunchKernelGGL(free_step::k_push_solve, dim3(grid), dim3(WAVE), 0, s, A);
  else if (c->task == COMET_TASK_PUSH_FREE_TIMED)
    hipLaunchKernelGGL(free_timed_step::k_push_solve, dim3(grid), dim3(WAVE), 0, s, A);
  else
    hipLaunchKernelGGL(fixed_step::k_push_solve, dim3(grid), dim3(WAVE), 0, s, A);
  if (timed && c->ev1) (void)hipEventRecord(c->ev1, s);
  c->timed = timed && c->ev0;
  if (hipGetLastError() != hipSuccess) return fail_msg(c, COMET_EHIP, "kernel launch failed");
  return COMET_OK;
}

}  // namespace comet

// ==================================================================================
// Allocation-free evaluation (pushing tasks): the work space of the solver lives in a
// static device array of every GPU the library runs on, instead of in a context's pools.
// ==================================================================================
namespace comet {

constexpr size_t NOALLOC_BYTES = size_t(64) << 20;
static __device__ __align__(256) unsigned char scratch[NOALLOC_BYTES];

// per device: the address of its copy of `scratch` (host code never uses the array's name
// as an address), its CU count, the solver kernels' occupancy and both models' row scales
struct NoallocDevice {
  bool ready = false;
  unsigned char* ptr = nullptr;
  int n_cu = 0, occ[2] = {1, 1};
  double scale[2][MAX_TYPES];
};
constexpr int NOALLOC_MAX_DEVICES = 64;
static NoallocDevice g_noalloc[NOALLOC_MAX_DEVICES];
static std::mutex g_noalloc_lock;

// Set-up of the current device, once: the symbol address, device properties, occupancy and
// row scales.  Later calls on the device only read these.
static comet_status noalloc_setup(int dev, NoallocDevice** out) {
  if (dev < 0 || dev >= NOALLOC_MAX_DEVICES) return fail_global(COMET_EINVAL, "device index out of range");
  std::lock_guard<std::mutex> g(g_noalloc_lock);
  NoallocDevice& d = g_noalloc[dev];
  if (!d.ready) {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p)
      return fail_global(COMET_EHIP, "hipGetSymbolAddress of the scratch array failed");
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, dev) != hipSuccess) return fail_global(COMET_EHIP, "device properties");
    int nb0 = 0, nb1 = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb0, fixed_step::k_push_solve, WAVE, 0) != hipSuccess || nb0 < 1)
      nb0 = 1;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb1, timed_step::k_push_solve, WAVE, 0) != hipSuccess || nb1 < 1)
      nb1 = 1;
    for (int t = 0; t < MAX_TYPES; ++t) d.scale[0][t] = d.scale[1][t] = 1.0;
    fixed_step::compute_scales(d.scale[0]);
    timed_step::compute_scales(d.scale[1]);
    d.ptr = (unsigned char*)p;
    d.n_cu = prop.multiProcessorCount;
    d.occ[0] = nb0;
    d.occ[1] = nb1;
    d.ready = true;
  }
  *out = &d;
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
  if ((task != COMET_TASK_PUSH && task != COMET_TASK_FLIP && task != COMET_TASK_PUSH_TIMED &&
       task != COMET_TASK_PUSH_FREE && task != COMET_TASK_PUSH_FREE_TIMED) || max_batch < 1 ||
      max_segments < 1 ||
      max_segments > (comet::is_free_task(task) ? comet::MAXSEG_FREE : comet::MAXSEG) ||
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
  const bool timed = (task == COMET_TASK_PUSH_TIMED), freem = (task == COMET_TASK_PUSH_FREE),
             freet = (task == COMET_TASK_PUSH_FREE_TIMED);
  for (int t = 0; t < comet::MAX_TYPES; ++t) c->scale[t] = 1.0;
  if (timed) comet::timed_step::compute_scales(c->scale);
  else if (freem) comet::free_step::compute_scales(c->scale);
  else if (freet) comet::free_timed_step::compute_scales(c->scale);
  else comet::fixed_step::compute_scales(c->scale);
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
  const hipError_t oe =
      timed ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, comet::timed_step::k_push_solve, comet::WAVE, 0)
      : freem ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, comet::free_step::k_push_solve, comet::WAVE, 0)
      : freet ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, comet::free_timed_step::k_push_solve, comet::WAVE, 0)
              : hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, comet::fixed_step::k_push_solve, comet::WAVE, 0);
  if (oe != hipSuccess || nb < 1) nb = 1;
  c->occ_blocks_per_cu = nb;
  const int64_t R = max_intervals, S = c->S;
  // per-interval work-space widths of the task's model
  const int64_t NW = timed ? comet::push_timed::NW
                     : freem ? comet::push_free::NW : freet ? comet::push_free_timed::NW : comet::push::NW;
  const int64_t NE = timed ? comet::push_timed::NE
                     : freem ? comet::push_free::NE : freet ? comet::push_free_timed::NE : comet::push::NE;
  const int64_t NI = timed ? comet::push_timed::NI
                     : freem ? comet::push_free::NI : freet ? comet::push_free_timed::NI : comet::push::NI;
  const int64_t NGAIN = timed ? comet::push_timed::NGAIN
                        : freem ? comet::push_free::NGAIN : freet ? comet::push_free_timed::NGAIN : comet::push::NGAIN;
  bool okm = hipMalloc(&c->zd, sizeof(double) * R * NW * S) == hipSuccess &&
             hipMalloc(&c->lam, sizeof(float) * R * NE * S) == hipSuccess &&
             hipMalloc(&c->nu, sizeof(float) * R * NI * S) == hipSuccess &&
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

const char* comet_last_error(const comet_ctx* c) { return c ? c->msg.c_str() : comet::g_msg.c_str(); }

comet_status comet_dims(const comet_ctx* c, int32_t* nx, int32_t* nu, int32_t* np, int32_t* nm, int32_t* ms,
                        int32_t* mi, int64_t* mb) {
  if (!c) return COMET_EINVAL;
  const bool fl = (c->task == COMET_TASK_FLIP), fr = comet::is_free_task(c->task);
  if (nx) *nx = fl ? 8 : (fr ? comet::push_free::NX : comet::push::NX);
  if (nu)
    *nu = fl ? 9
          : c->task == COMET_TASK_PUSH_TIMED ? comet::push_timed::NU
          : c->task == COMET_TASK_PUSH_FREE_TIMED ? comet::push_free_timed::NU
          : fr ? comet::push_free::NU : comet::push::NU;
  if (np) *np = 1;
  if (nm) *nm = fl ? 845 : (fr ? comet::push_free::NMODES : comet::push::NMODES);
  if (ms) *ms = c->max_segments;
  if (mi) *mi = c->max_intervals;
  if (mb) *mb = c->max_batch;
  return COMET_OK;
}

comet_status comet_row_scales(const comet_ctx* c, double* out, int32_t n) {
  if (!c || !out || c->task == COMET_TASK_FLIP) return COMET_EINVAL;
  const int nt = (c->task == COMET_TASK_PUSH_TIMED) ? comet::push_timed::NTYPES
                 : comet::is_free_task(c->task) ? comet::push_free::NTYPES : comet::push::NTYPES;
  if (n < nt) return COMET_EINVAL;
  for (int t = 0; t < nt; ++t) out[t] = c->scale[t];
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

comet_status comet_evaluate_noalloc(comet_task task, const comet_solver_params* params, void* stream, int64_t B,
                                    int32_t max_segments, int32_t max_intervals, const float* x0, const float* goal,
                                    const float* inst, const int32_t* nseg, const int32_t* modes, const int32_t* knots,
                                    float* cost, float* viol, uint8_t* feasible, float* traj, int32_t* stats) {
  using namespace comet;
  if (task != COMET_TASK_PUSH && task != COMET_TASK_PUSH_TIMED)
    return fail_global(COMET_EINVAL, "the allocation-free evaluation serves the pushing tasks");
  if (B < 0 || max_segments < 1 || max_segments > MAXSEG || max_intervals < 1 || max_intervals > MAXN)
    return fail_global(COMET_EINVAL, "B, max_segments or max_intervals out of range");
  if (B == 0) return COMET_OK;
  if (!x0 || !goal || !inst || !nseg || !modes || !knots || !cost || !viol || !feasible)
    return fail_global(COMET_EINVAL, "null input or output pointer");
  comet_solver_params prm;
  if (params) prm = *params;
  else comet_default_params(&prm);
  if (prm.ls_trials < 1 || prm.ls_trials > MAX_TRIALS || prm.al_max < 1 || prm.gn_max < 1 || !(prm.mu0 > 0) ||
      !(prm.mu_min > 0) || !(prm.mu0_warm > 0))
    return fail_global(COMET_EINVAL, "bad solver parameters");
  const bool timed = (task == COMET_TASK_PUSH_TIMED);
  const int64_t NW = timed ? push_timed::NW : push::NW, NE = timed ? push_timed::NE : push::NE;
  const int64_t NI = timed ? push_timed::NI : push::NI, NG = timed ? push_timed::NGAIN : push::NGAIN;
  const int64_t S = (B + 63) / 64 * 64, R = max_intervals;
  // layout of the scratch array, every region 256-byte aligned
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t at = off;
    off = (off + bytes + 255) / 256 * 256;
    return at;
  };
  const size_t o_zd = take(sizeof(double) * R * NW * S), o_lam = take(sizeof(float) * R * NE * S);
  const size_t o_nu = take(sizeof(float) * R * NI * S), o_gain = take(sizeof(float) * R * NG * S);
  const size_t o_dz = take(sizeof(float) * R * NW * S), o_code = take((size_t)R * S);
  const size_t o_q = take(sizeof(unsigned long long)), o_err = take(sizeof(unsigned));
  const size_t o_hist = take(sizeof(int) * (R + 2)), o_order = take(sizeof(int) * B);
  if (off > NOALLOC_BYTES)
    return fail_global(COMET_EINVAL, "batch x intervals exceed the allocation-free work space (64 MiB)");
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return fail_global(COMET_EHIP, "no current device");
  NoallocDevice* nd = nullptr;
  comet_status st = noalloc_setup(dev, &nd);
  if (st != COMET_OK) return st;
  // a context on the stack pointing into the device's scratch array: no pools, no events
  comet_ctx c;
  c.task = task;
  c.prm = prm;
  c.max_batch = B;
  c.S = S;
  c.max_segments = max_segments;
  c.max_intervals = max_intervals;
  c.device = dev;
  for (int t = 0; t < MAX_TYPES; ++t) c.scale[t] = nd->scale[timed ? 1 : 0][t];
  unsigned char* base = nd->ptr;
  c.zd = (double*)(base + o_zd);
  c.lam = (float*)(base + o_lam);
  c.nu = (float*)(base + o_nu);
  c.gains = (float*)(base + o_gain);
  c.dz = (float*)(base + o_dz);
  c.code = base + o_code;
  c.qhead = (unsigned long long*)(base + o_q);
  c.err = (unsigned*)(base + o_err);
  c.hist = (int*)(base + o_hist);
  c.order = (int*)(base + o_order);
  c.n_cu = nd->n_cu;
  c.occ_blocks_per_cu = nd->occ[timed ? 1 : 0];
  EvalLaunch L;
  L.B = B;
  L.B_max = B;
  L.x0 = x0; L.goal = goal; L.inst = inst; L.inst_stride = 1;
  L.nseg = nseg; L.modes = modes; L.knots = knots;
  L.cost = cost; L.viol = viol; L.feas = feasible; L.traj = traj; L.stats = stats;
  st = launch_evaluate(&c, (hipStream_t)stream, L);
  if (st != COMET_OK) return fail_global(st, c.msg);
  return COMET_OK;
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
