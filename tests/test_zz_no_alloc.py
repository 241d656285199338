"""The allocation-free evaluation (comet_evaluate_noalloc) against comet_evaluate: two calls
in a row on one GPU's shared scratch array, the second with a smaller batch, and the
optimised-timing task; every output equal bit for bit (same kernel, same arithmetic; a
sequence's result does not depend on the work-space slot it is solved in).  Requests
beyond the 64 MiB work space are rejected before any launch."""
import numpy as np
import pytest

from paper_2609_21803_amd import instances as I

pytestmark = pytest.mark.gpu


def _ref(b, nmax, task):
    import torch
    from paper_2609_21803_amd import native
    ctx = native.Context(max_batch=len(b["nseg"]), max_segments=6, max_intervals=nmax, task=task)
    out = ctx.evaluate(**native.to_device(b))
    torch.cuda.synchronize()
    return {k: v.cpu().numpy() for k, v in out.items()}


def _noalloc(b, nmax, task):
    import torch
    from paper_2609_21803_amd import native
    d = native.to_device(b)
    out = native.evaluate_noalloc(**d, max_intervals=nmax, task=task)
    torch.cuda.synchronize()
    return {k: v.cpu().numpy() for k, v in out.items()}


def _same(a, b):
    for k in ("cost", "viol", "feasible", "traj", "stats"):
        assert np.array_equal(a[k], b[k], equal_nan=True), k


def test_noalloc_equals_context_evaluate_on_two_calls_in_a_row():
    from paper_2609_21803_amd import native
    big = I.push_hetero(B=1800, seed=31, kmax=4, nmax=10)          # up to 40 intervals
    small = I.subset(I.push_tiny(seed=5), np.arange(0, 1152, 3))    # 384 orders, 10 intervals
    _same(_noalloc(big, 40, native.TASK_PUSH), _ref(big, 40, native.TASK_PUSH))
    _same(_noalloc(small, 10, native.TASK_PUSH), _ref(small, 10, native.TASK_PUSH))
    # optimised timing (its own model in the same array), then the fixed step again
    _same(_noalloc(small, 10, native.TASK_PUSH_TIMED), _ref(small, 10, native.TASK_PUSH_TIMED))
    _same(_noalloc(big, 40, native.TASK_PUSH), _ref(big, 40, native.TASK_PUSH))


def test_noalloc_rejects_what_does_not_fit_and_other_tasks():
    import torch
    from paper_2609_21803_amd import native
    b = I.push_hetero(B=64, seed=3)
    d = native.to_device(b)
    with pytest.raises(native.CometError):
        native.evaluate_noalloc(**d, max_intervals=600, task=native.TASK_PUSH,
                                out=dict(cost=torch.empty(64, device="cuda"), viol=torch.empty(64, device="cuda"),
                                         feasible=torch.empty(64, dtype=torch.uint8, device="cuda")))
    big = {k: v.repeat(*([64] + [1] * (v.dim() - 1))) for k, v in d.items()}   # 4,096 orders x 75 intervals
    with pytest.raises(native.CometError):
        native.evaluate_noalloc(**big, max_intervals=75, task=native.TASK_PUSH)
    with pytest.raises(native.CometError):
        native.evaluate_noalloc(**d, max_intervals=75, task=native.TASK_FLIP)
    with pytest.raises(native.CometError):
        native.evaluate_noalloc(**d, max_intervals=75, task=native.TASK_PUSH_FREE)
    e = {k: v[:0] for k, v in d.items()}
    o = native.evaluate_noalloc(**e, max_intervals=75, task=native.TASK_PUSH)   # B = 0: no-op
    assert o["cost"].numel() == 0
