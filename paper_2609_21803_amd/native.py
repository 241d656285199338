"""ctypes binding of the C ABI in ``include/comet.h`` (argument marshalling only).

Every step of the evaluator runs in the HIP library ``libcomet.so``; this module only
turns torch tensors into device pointers and the caller's stream into a HIP stream
handle.  It raises if the library is missing or the GPU is absent: there is no CPU
fallback.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass, fields

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libcomet.so")

COMET_OK, COMET_EINVAL, COMET_EHIP, COMET_ENOMEM, COMET_ESTATE = 0, -1, -2, -3, -4
TASK_PUSH, TASK_FLIP, TASK_PUSH_TIMED, TASK_PUSH_FREE, TASK_PUSH_FREE_TIMED = 0, 1, 2, 3, 4
POLICY_EXPAND, POLICY_UNIFORM, POLICY_MCTS = 0, 1, 2
ROW_WIDTH = {TASK_PUSH: 7, TASK_FLIP: 17, TASK_PUSH_TIMED: 8, TASK_PUSH_FREE: 9, TASK_PUSH_FREE_TIMED: 10}   # trajectory row (x_k, u_k)


class SolverParamsC(C.Structure):
    _fields_ = [("al_max", C.c_int32), ("gn_max", C.c_int32), ("ref_al_max", C.c_int32), ("ref_gn_max", C.c_int32),
                ("chol_retries", C.c_int32), ("ls_trials", C.c_int32), ("max_rejects", C.c_int32),
                ("reserved", C.c_int32), ("mu0", C.c_double), ("mu_min", C.c_double), ("rho0", C.c_double),
                ("rho_min", C.c_double), ("rho_max", C.c_double), ("armijo_c1", C.c_double),
                ("eta_star", C.c_double), ("omega_star", C.c_double), ("rc_star", C.c_double),
                ("eps_feas", C.c_double), ("mu0_warm", C.c_double)]


class ScheduleC(C.Structure):
    _fields_ = [("waves_per_cu", C.c_int32), ("sort_by_length", C.c_int32)]


class ExpandParamsC(C.Structure):
    _fields_ = [("kcap", C.c_int32), ("seed_max_segments", C.c_int32), ("radius", C.c_int32), ("rounds", C.c_int32),
                ("frontier_W", C.c_int32), ("knots_per_segment", C.c_int32), ("k_ref", C.c_int32),
                ("n_total", C.c_int32), ("learned_warm", C.c_int32), ("policy", C.c_int32), ("batch_B", C.c_int64),
                ("eval_budget", C.c_int64), ("mu_merit", C.c_double), ("sample_seed", C.c_uint64),
                ("sample_draws", C.c_int64), ("uct_c", C.c_double)]


class ExpandStatsC(C.Structure):
    _fields_ = [("evaluated", C.c_int64), ("rounds_done", C.c_int32), ("n_feasible", C.c_int32),
                ("first_feasible_index", C.c_int64), ("t_first_feasible_ms", C.c_double),
                ("t_total_ms", C.c_double), ("n_refined", C.c_int32), ("reserved", C.c_int32)]


@dataclass
class ExpandParams:
    kcap: int = 3
    seed_max_segments: int = 2
    radius: int = 1
    rounds: int = 8
    frontier_W: int = 4096
    knots_per_segment: int = 8
    k_ref: int = 64
    n_total: int = 24
    learned_warm: int = 1
    policy: int = 0            # 0 expansion (Alg. 1), 1 uniform sampling
    batch_B: int = 131072
    eval_budget: int = 200000
    mu_merit: float = 100.0
    sample_seed: int = 0       # uniform sampling: SplitMix64 seed
    sample_draws: int = 65536  # uniform sampling: draws per round
    uct_c: float = 0.8         # MCTS exploration constant

    def c(self) -> ExpandParamsC:
        return ExpandParamsC(*[getattr(self, f.name) for f in fields(self)])


class CometError(RuntimeError):
    pass


_lib = None


def lib():
    """Load libcomet.so (built by ``__graft_entry__.build()``); raise if it is missing."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise CometError(f"HIP library not built: {LIB_PATH} (run __graft_entry__.build())")
        L = C.CDLL(LIB_PATH)
        P = C.c_void_p
        L.comet_default_params.argtypes = [C.POINTER(SolverParamsC)]
        L.comet_default_params.restype = None
        L.comet_create.argtypes = [C.c_int, C.POINTER(SolverParamsC), C.c_int64, C.c_int32, C.c_int32,
                                   C.POINTER(P)]
        L.comet_create.restype = C.c_int
        L.comet_destroy.argtypes = [P]
        L.comet_destroy.restype = None
        L.comet_last_error.argtypes = [P]
        L.comet_last_error.restype = C.c_char_p
        L.comet_dims.argtypes = [P] + [C.POINTER(C.c_int32)] * 6 + [C.POINTER(C.c_int64)]
        L.comet_dims.restype = C.c_int
        L.comet_row_scales.argtypes = [P, P, C.c_int32]
        L.comet_row_scales.restype = C.c_int
        L.comet_check.argtypes = [P, P]
        L.comet_check.restype = C.c_int
        L.comet_evaluate.argtypes = [P, P, C.c_int64] + [P] * 7 + [C.c_int32] + [P] * 5
        L.comet_evaluate.restype = C.c_int
        L.comet_evaluate_noalloc.argtypes = [C.c_int, C.POINTER(SolverParamsC), P, C.c_int64, C.c_int32, C.c_int32] + \
            [P] * 11
        L.comet_evaluate_noalloc.restype = C.c_int
        L.comet_set_schedule.argtypes = [P, C.POINTER(ScheduleC)]
        L.comet_set_schedule.restype = C.c_int
        L.comet_get_schedule.argtypes = [P, C.POINTER(ScheduleC), C.POINTER(C.c_int32), C.POINTER(C.c_int32)]
        L.comet_get_schedule.restype = C.c_int
        L.comet_autotune.argtypes = [P, P, C.c_int64] + [P] * 11 + [C.POINTER(ScheduleC), C.POINTER(C.c_float)]
        L.comet_autotune.restype = C.c_int
        L.comet_expand.argtypes = [P, P, P, P, P, C.POINTER(ExpandParamsC), P, P, P, P, P, P, P,
                                   C.POINTER(ExpandStatsC)]
        L.comet_expand.restype = C.c_int
        L.comet_expand_next.argtypes = [P, P, C.c_int64, P, P, C.POINTER(ExpandParamsC), C.c_int64, P, P]
        L.comet_expand_next.restype = C.c_int
        L.comet_expand_trace.argtypes = [P, P, C.c_int64, P, P, P, P]
        L.comet_expand_trace.restype = C.c_int
        L.comet_mlp_create.argtypes = [C.c_int32, C.c_int32, C.c_int32, C.c_int32, C.c_int64, C.c_uint64, C.POINTER(P)]
        L.comet_mlp_create.restype = C.c_int
        L.comet_mlp_destroy.argtypes = [P]
        L.comet_mlp_destroy.restype = None
        L.comet_mlp_num_params.argtypes = [P, C.POINTER(C.c_int64)]
        L.comet_mlp_num_params.restype = C.c_int
        L.comet_mlp_params.argtypes = [P, P, C.c_int32, P]
        L.comet_mlp_params.restype = C.c_int
        L.comet_mlp_grads.argtypes = [P, P, P]
        L.comet_mlp_grads.restype = C.c_int
        L.comet_mlp_forward.argtypes = [P, P, C.c_int64, P, P]
        L.comet_mlp_forward.restype = C.c_int
        L.comet_mlp_train_step.argtypes = [P, P, C.c_int64, P, P, P, P, P, C.c_float, C.c_float, P]
        L.comet_mlp_train_step.restype = C.c_int
        L.comet_mlp_encode.argtypes = [C.c_int, P, C.c_int64, P, P, P, P, P, P, C.c_int32, C.c_int32, P]
        L.comet_mlp_encode.restype = C.c_int
        L.comet_mlp_targets.argtypes = [C.c_int, P, C.c_int64, P, C.c_int32, P, P, C.c_int32, P, P, P, P, P, P]
        L.comet_mlp_targets.restype = C.c_int
        L.comet_mlp_decode_warm.argtypes = [C.c_int, P, C.c_int64, P, C.c_int32, P, P, P, P, C.c_int32, C.c_int32,
                                            P]
        L.comet_mlp_decode_warm.restype = C.c_int
        L.comet_last_kernel_ms.argtypes = [P, C.POINTER(C.c_float)]
        L.comet_last_kernel_ms.restype = C.c_int
        L.comet_probe_peaks.argtypes = [P, P]
        L.comet_probe_peaks.restype = C.c_int
        _lib = L
    return _lib


@dataclass
class SolverParams:
    al_max: int = 20
    gn_max: int = 10
    ref_al_max: int = 40
    ref_gn_max: int = 25
    chol_retries: int = 6
    ls_trials: int = 8
    max_rejects: int = 4
    reserved: int = 0
    mu0: float = 1e-2
    mu_min: float = 1e-4
    rho0: float = 1e-4
    rho_min: float = 1e-8
    rho_max: float = 1e8
    armijo_c1: float = 1e-4
    eta_star: float = 1e-6
    omega_star: float = 1e-4
    rc_star: float = 1e-6
    eps_feas: float = 1e-5
    mu0_warm: float = 1e-4

    def c(self) -> SolverParamsC:
        return SolverParamsC(*[getattr(self, f.name) for f in fields(self)])

    @staticmethod
    def library_defaults() -> "SolverParams":
        p = SolverParamsC()
        lib().comet_default_params(C.byref(p))
        return SolverParams(*[getattr(p, f) for f, _ in SolverParamsC._fields_])


def _ptr(t):
    if t is None:
        return None
    if not t.is_cuda or not t.is_contiguous():
        raise CometError("expected a contiguous tensor on the GPU")
    return C.c_void_p(t.data_ptr())


def _stream(stream=None):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


def _torch_device_first():
    """Initialise torch's device runtime before the library's first device call: torch
    owns the device memory and streams handed to the library, and its runtime must be
    the first to open the device in the process."""
    import torch
    torch.cuda.current_device()


def check(rc: int, ctx=None):
    if rc != COMET_OK:
        msg = lib().comet_last_error(ctx).decode()
        raise CometError(f"comet call failed with status {rc}: {msg}")


class Context:
    """One evaluator context (work space for max_batch sequences) on the current device."""

    def __init__(self, max_batch: int, max_segments: int = 6, max_intervals: int = 24,
                 params: SolverParams | None = None, task: int = TASK_PUSH):
        _torch_device_first()
        self._h = C.c_void_p()
        self.params = params or SolverParams()
        p = self.params.c()
        rc = lib().comet_create(task, C.byref(p), int(max_batch), int(max_segments), int(max_intervals),
                                C.byref(self._h))
        if rc != COMET_OK:
            raise CometError(f"comet_create failed with status {rc}")
        self.task = int(task)
        self.max_batch, self.max_segments, self.max_intervals = int(max_batch), int(max_segments), int(max_intervals)

    def close(self):
        if self._h:
            lib().comet_destroy(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def dims(self):
        v = [C.c_int32() for _ in range(6)]
        mb = C.c_int64()
        check(lib().comet_dims(self._h, *[C.byref(x) for x in v], C.byref(mb)), self._h)
        return dict(nx=v[0].value, nu=v[1].value, n_inst=v[2].value, n_modes=v[3].value,
                    max_segments=v[4].value, max_intervals=v[5].value, max_batch=mb.value)

    def row_scales(self):
        import numpy as np
        out = np.zeros(16)
        check(lib().comet_row_scales(self._h, out.ctypes.data_as(C.c_void_p), 16), self._h)
        return out[:{TASK_PUSH_TIMED: 13, TASK_PUSH_FREE: 16, TASK_PUSH_FREE_TIMED: 16}.get(self.task, 12)]

    def check(self, stream=None):
        check(lib().comet_check(self._h, _stream(stream)), self._h)

    def kernel_ms(self) -> float:
        ms = C.c_float()
        check(lib().comet_last_kernel_ms(self._h, C.byref(ms)), self._h)
        return ms.value

    def schedule(self):
        sc = ScheduleC()
        occ, ncu = C.c_int32(), C.c_int32()
        check(lib().comet_get_schedule(self._h, C.byref(sc), C.byref(occ), C.byref(ncu)), self._h)
        return dict(waves_per_cu=sc.waves_per_cu, sort_by_length=sc.sort_by_length, occupancy=occ.value,
                    n_cu=ncu.value)

    def set_schedule(self, waves_per_cu=0, sort_by_length=0):
        sc = ScheduleC(int(waves_per_cu), int(sort_by_length))
        check(lib().comet_set_schedule(self._h, C.byref(sc)), self._h)

    def autotune(self, x0, goal, inst, nseg, modes, knots, out: dict, stream=None):
        """Time every candidate schedule on this batch, keep the fastest; returns (schedule, ms)."""
        sc = ScheduleC()
        ms = C.c_float()
        rc = lib().comet_autotune(self._h, _stream(stream), int(nseg.shape[0]), _ptr(x0), _ptr(goal), _ptr(inst),
                                  _ptr(nseg), _ptr(modes), _ptr(knots), _ptr(out["cost"]), _ptr(out["viol"]),
                                  _ptr(out["feasible"]), _ptr(out.get("traj")), _ptr(out.get("stats")),
                                  C.byref(sc), C.byref(ms))
        check(rc, self._h)
        return dict(waves_per_cu=sc.waves_per_cu, sort_by_length=sc.sort_by_length), ms.value

    def evaluate(self, x0, goal, inst, nseg, modes, knots, warm=None, refine=0, cost=None, viol=None,
                 feasible=None, traj=None, stats=None, want_traj=True, want_stats=True, stream=None):
        """Device tensors in, device tensors out (allocated here when not given)."""
        import torch
        B = int(nseg.shape[0])
        dev = nseg.device
        if cost is None:
            cost = torch.empty(B, dtype=torch.float32, device=dev)
        if viol is None:
            viol = torch.empty(B, dtype=torch.float32, device=dev)
        if feasible is None:
            feasible = torch.empty(B, dtype=torch.uint8, device=dev)
        if traj is None and want_traj:
            traj = torch.empty((B, self.max_intervals + 1, ROW_WIDTH[self.task]), dtype=torch.float32, device=dev)
        if stats is None and want_stats:
            stats = torch.empty((B, 4), dtype=torch.int32, device=dev)
        rc = lib().comet_evaluate(self._h, _stream(stream), B, _ptr(x0), _ptr(goal), _ptr(inst), _ptr(nseg),
                                  _ptr(modes), _ptr(knots), _ptr(warm), int(refine), _ptr(cost), _ptr(viol),
                                  _ptr(feasible), _ptr(traj), _ptr(stats))
        check(rc, self._h)
        return dict(cost=cost, viol=viol, feasible=feasible, traj=traj, stats=stats)


def expand(ctx: "Context", x0, goal, inst, params: ExpandParams, learned=None, stream=None):
    """Greedy expansion on one instance (device tensors; pushing: x0 [4], goal [3], inst [1];
    free-motion pushing: x0 [5]; flipping: x0 [8], goal [2], inst [1])."""
    import torch
    dev = x0.device
    S, N = ctx.max_segments, ctx.max_intervals
    o = dict(nseg=torch.zeros(1, dtype=torch.int32, device=dev), modes=torch.zeros(S, dtype=torch.int32, device=dev),
             knots=torch.zeros(S, dtype=torch.int32, device=dev), cost=torch.zeros(1, device=dev),
             viol=torch.zeros(1, device=dev), traj=torch.zeros((N + 1, ROW_WIDTH[ctx.task]), device=dev))
    st = ExpandStatsC()
    pc = params.c()
    rc = lib().comet_expand(ctx._h, _stream(stream), _ptr(x0), _ptr(goal), _ptr(inst), C.byref(pc),
                            None if learned is None else learned.handle(), _ptr(o["nseg"]), _ptr(o["modes"]),
                            _ptr(o["knots"]), _ptr(o["cost"]), _ptr(o["viol"]), _ptr(o["traj"]), C.byref(st))
    check(rc, ctx._h)
    stats = {f: getattr(st, f) for f, _ in ExpandStatsC._fields_}
    return o, stats


def expand_next(ctx: "Context", keys, merit, params: ExpandParams, room: int, stream=None):
    """One batch-construction step on device tensors keys (uint64 as int64) and merit (float64)."""
    import torch
    dev = merit.device
    out = torch.zeros(max(int(room), 1), dtype=torch.int64, device=dev)
    n = torch.zeros(1, dtype=torch.int64, device=dev)
    pc = params.c()
    rc = lib().comet_expand_next(ctx._h, _stream(stream), int(keys.shape[0]), _ptr(keys), _ptr(merit), C.byref(pc),
                                 int(room), _ptr(out), _ptr(n))
    check(rc, ctx._h)
    return out[: int(n.item())]


def probe_peaks(stream=None) -> dict:
    """Measured peak rates of the current device (comet_probe_peaks)."""
    import numpy as np
    _torch_device_first()
    out = np.zeros(4)
    st = _stream(stream)
    check(lib().comet_probe_peaks(st, out.ctypes.data_as(C.c_void_p)))
    return dict(fp32_fma_tflops=float(out[0]), fp64_fma_tflops=float(out[1]), bf16_mfma_tflops=float(out[2]),
                copy_gbs=float(out[3]))


def expand_trace(ctx: "Context", cap: int = 1 << 20, stream=None):
    import torch
    keys = torch.zeros(cap, dtype=torch.int64, device="cuda")
    J = torch.zeros(cap, dtype=torch.float64, device="cuda")
    v = torch.zeros(cap, dtype=torch.float64, device="cuda")
    n = torch.zeros(1, dtype=torch.int64, device="cuda")
    check(lib().comet_expand_trace(ctx._h, _stream(stream), cap, _ptr(keys), _ptr(J), _ptr(v), _ptr(n)), ctx._h)
    k = int(n.item())
    return keys[:k], J[:k], v[:k]


class MLP:
    """Learned proposal / warm-start network (BF16 matrix-core kernels)."""
    IN, HIDDEN, LAYERS, OUT = 416, 512, 4, 736

    def __init__(self, max_batch=8192, seed=0, in_dim=IN, hidden=HIDDEN, layers=LAYERS, out_dim=OUT):
        _torch_device_first()
        self._h = C.c_void_p()
        rc = lib().comet_mlp_create(in_dim, hidden, layers, out_dim, int(max_batch), int(seed), C.byref(self._h))
        if rc != COMET_OK:
            raise CometError(f"comet_mlp_create failed with status {rc}")
        self.in_dim, self.hidden, self.layers, self.out_dim, self.max_batch = in_dim, hidden, layers, out_dim, max_batch
        n = C.c_int64()
        check(lib().comet_mlp_num_params(self._h, C.byref(n)))
        self.n_params = n.value

    def handle(self):
        return self._h

    def close(self):
        if self._h:
            lib().comet_mlp_destroy(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def get_params(self):
        import torch
        out = torch.empty(self.n_params, dtype=torch.float32, device="cuda")
        check(lib().comet_mlp_params(self._h, _stream(), 0, _ptr(out)))
        return out

    def set_params(self, flat):
        check(lib().comet_mlp_params(self._h, _stream(), 1, _ptr(flat)))

    def grads(self):
        import torch
        out = torch.empty(self.n_params, dtype=torch.float32, device="cuda")
        check(lib().comet_mlp_grads(self._h, _stream(), _ptr(out)))
        return out

    def forward(self, x_bf16):
        import torch
        B = int(x_bf16.shape[0])
        out = torch.empty((B, self.out_dim), dtype=torch.float32, device="cuda")
        check(lib().comet_mlp_forward(self._h, _stream(), B, _ptr(x_bf16), _ptr(out)))
        return out

    def train_step(self, x_bf16, y_feas, y_cost, y_traj, mask, lr, weight_decay=1e-4):
        import torch
        loss = torch.zeros(3, dtype=torch.float32, device="cuda")
        check(lib().comet_mlp_train_step(self._h, _stream(), int(x_bf16.shape[0]), _ptr(x_bf16), _ptr(y_feas),
                                         _ptr(y_cost), _ptr(y_traj), _ptr(mask), float(lr), float(weight_decay),
                                         _ptr(loss)))
        return loss


def mlp_segments(task) -> int:
    """Segments an encoding and a warm-start block hold: 8 for free motion, else 6."""
    return 8 if task in (TASK_PUSH_FREE, TASK_PUSH_FREE_TIMED) else 6


def mlp_dims(task) -> tuple[int, int]:
    """(in_dim, out_dim) of a network for the task: 16 + 64 S inputs, 2 + 120 S outputs
    (S segments), rounded up to multiples of 8."""
    S = mlp_segments(task)
    r8 = lambda n: (n + 7) // 8 * 8
    return (416, 736) if S == 6 else (r8(16 + 64 * S), r8(2 + 120 * S))


def mlp_encode(d: dict, in_dim=None, task=TASK_PUSH):
    """Encode device batches (as from to_device) for the network: [B, in_dim] BF16 bits."""
    import torch
    in_dim = in_dim or mlp_dims(task)[0]
    B = int(d["nseg"].shape[0])
    smax = int(d["modes"].shape[1])
    x = torch.empty((B, in_dim), dtype=torch.int16, device="cuda")
    check(lib().comet_mlp_encode(task, _stream(), B, _ptr(d["x0"]), _ptr(d["goal"]), _ptr(d["inst"]),
                                 _ptr(d["nseg"]), _ptr(d["modes"]), _ptr(d["knots"]), smax, in_dim, _ptr(x)))
    return x


def mlp_targets(d: dict, out: dict, nmax: int, task=TASK_PUSH):
    import torch
    B = int(d["nseg"].shape[0])
    smax = int(d["modes"].shape[1])
    f = lambda *s: torch.empty(s, dtype=torch.float32, device="cuda")
    W = 120 * mlp_segments(task)
    yf, yc, yt, m = f(B), f(B), f(B, W), f(B, W)
    check(lib().comet_mlp_targets(task, _stream(), B, _ptr(out["traj"]), nmax, _ptr(d["nseg"]), _ptr(d["knots"]), smax,
                                  _ptr(out["feasible"]), _ptr(out["cost"]), _ptr(yf), _ptr(yc), _ptr(yt), _ptr(m)))
    return yf, yc, yt, m


def mlp_decode_warm(y, d: dict, nmax: int, task=TASK_PUSH):
    import torch
    B = int(d["nseg"].shape[0])
    smax = int(d["modes"].shape[1])
    w = torch.empty((B, nmax + 1, ROW_WIDTH[task]), dtype=torch.float32, device="cuda")
    check(lib().comet_mlp_decode_warm(task, _stream(), B, _ptr(y), int(y.shape[1]), _ptr(d["x0"]), _ptr(d["nseg"]),
                                      _ptr(d["modes"]), _ptr(d["knots"]), smax, nmax, _ptr(w)))
    return w


def evaluate_noalloc(x0, goal, inst, nseg, modes, knots, max_intervals: int, task=TASK_PUSH,
                     params: "SolverParams | None" = None, out: dict | None = None, stream=None):
    """comet_evaluate_noalloc: the context-free, allocation-free evaluation (pushing tasks).
    Outputs are allocated here by torch unless given in `out` (the library call itself
    allocates nothing)."""
    import torch
    B = int(nseg.shape[0])
    dev = nseg.device
    row = ROW_WIDTH[task]
    if out is None:
        out = dict(cost=torch.empty(B, dtype=torch.float32, device=dev), viol=torch.empty(B, dtype=torch.float32, device=dev),
                   feasible=torch.empty(B, dtype=torch.uint8, device=dev),
                   traj=torch.empty((B, max_intervals + 1, row), dtype=torch.float32, device=dev),
                   stats=torch.empty((B, 4), dtype=torch.int32, device=dev))
    pc = None if params is None else C.byref(params.c())
    rc = lib().comet_evaluate_noalloc(int(task), pc, _stream(stream), B, int(modes.shape[1]), int(max_intervals),
                                      _ptr(x0), _ptr(goal), _ptr(inst), _ptr(nseg), _ptr(modes), _ptr(knots),
                                      _ptr(out["cost"]), _ptr(out["viol"]), _ptr(out["feasible"]), _ptr(out.get("traj")),
                                      _ptr(out.get("stats")))
    check(rc)
    return out


def to_device(batch: dict, device="cuda"):
    """Seeded host arrays (see instances.py) -> device tensors in the ABI dtypes."""
    import torch
    f32 = lambda a: torch.as_tensor(a, dtype=torch.float32).contiguous().to(device)
    i32 = lambda a: torch.as_tensor(a, dtype=torch.int32).contiguous().to(device)
    return dict(x0=f32(batch["x0"]), goal=f32(batch["goal"]), inst=f32(batch["inst"]), nseg=i32(batch["nseg"]),
                modes=i32(batch["modes"]), knots=i32(batch["knots"]))
