"""Host logic of the learned-proposal helpers (CPU): key decoding for both key layouts
against the oracles' own key functions, the even split of an order's intervals (the
expansion's allocation when knots_per_segment is 0), the per-task network widths, and the
rank statistic behind the feasibility AUC against brute force."""
import numpy as np
import pytest


def test_decode_keys_matches_the_oracle_key_layouts():
    import torch
    from oracle import free as F
    from paper_2609_21803_amd import learned
    keys = F.seed(8)
    pick = np.random.default_rng(3).choice(len(keys), 500, replace=False)
    k = torch.as_tensor(keys[pick].view(np.int64))
    nseg, modes = learned.decode_keys(k, smax=8, bits=4)
    for i, p in enumerate(pick):
        m = F.key_modes(int(keys[p]))
        assert int(nseg[i]) == len(m)
        assert modes[i, :len(m)].tolist() == m and not modes[i, len(m):].any()
    # ten-bit ids (pushing, timed pushing, flipping): K << 60 then ids from bit 50 down
    ids = [[3, 845 - 1, 0, 17, 512, 9], [11], [0, 0]]
    raw = [(len(m) << 60) | sum(v << (50 - 10 * j) for j, v in enumerate(m)) for m in ids]
    nseg, modes = learned.decode_keys(torch.tensor(raw, dtype=torch.int64), smax=6)
    for i, m in enumerate(ids):
        assert int(nseg[i]) == len(m) and modes[i, :len(m)].tolist() == m and not modes[i, len(m):].any()


@pytest.mark.parametrize("n_total", [8, 24, 50])
def test_split_knots_is_even_with_the_remainder_first(n_total):
    import torch
    from paper_2609_21803_amd import learned
    nseg = torch.arange(1, 9, dtype=torch.int32)
    kn = learned.split_knots(nseg, 8, n_total).numpy()
    for K in range(1, 9):
        row = kn[K - 1]
        assert row.sum() == n_total and np.all(row[K:] == 0)
        assert row[:K].max() - row[:K].min() <= 1 and np.all(np.diff(row[:K]) <= 0)
        assert np.all(row[:K] == [n_total // K + (j < n_total % K) for j in range(K)])


def test_network_widths_per_task():
    from paper_2609_21803_amd import native
    assert native.mlp_dims(native.TASK_PUSH) == (416, 736) == native.mlp_dims(native.TASK_FLIP)
    assert native.mlp_dims(native.TASK_PUSH_TIMED) == (416, 736)
    for t in (native.TASK_PUSH_FREE, native.TASK_PUSH_FREE_TIMED):
        i, o = native.mlp_dims(t)
        assert (i, o) == (528, 968) and i >= 16 + 64 * 8 and o >= 2 + 120 * 8 and i % 8 == 0 and o % 8 == 0


def test_auc_equals_pairwise_count():
    from paper_2609_21803_amd import learned
    rng = np.random.default_rng(5)
    s = rng.integers(0, 6, 200).astype(float)          # many ties
    y = rng.random(200) < 0.3
    pos, neg = s[y], s[~y]
    brute = ((pos[:, None] > neg[None, :]).sum() + 0.5 * (pos[:, None] == neg[None, :]).sum()) / (len(pos) * len(neg))
    assert abs(learned.auc(s, y) - brute) < 1e-12
    assert np.isnan(learned.auc(s, np.zeros(200, bool)))
