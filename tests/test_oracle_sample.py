"""Pins of the uniform-sampling oracle: the SplitMix64 generator against its published test
vectors, the draw rule's distribution, sampling without replacement, and coverage of a
small language (every admissible single-segment flip order exactly once; all twelve
single-segment pushing orders)."""
import collections

import numpy as np

from oracle import sample as S


def test_splitmix64_published_vectors():
    # seed 1234567 (the vector of the reference implementation's test suites) and seed 0
    assert [S.splitmix64(1234567, i) for i in range(5)] == [
        6457827717110365317, 3203168211198807973, 9817491932198370423, 4593380528125082431, 16408922859458223821]
    assert S.splitmix64(0, 0) == 0xE220A8397B1DCDAF and S.splitmix64(0, 1) == 0x6E789E6AA1B965F4
    idx = np.arange(1000, dtype=np.uint64)
    assert S.splitmix64_array(99, idx).tolist() == [S.splitmix64(99, i) for i in range(1000)]


def test_draws_are_uniform_in_length_and_ids():
    d = S.draws(seed=7, first=0, n=60000, kcap=3, n_modes=12)
    K = collections.Counter(len(m) for m in d)
    assert set(K) == {1, 2, 3} and all(abs(K[k] / 60000 - 1 / 3) < 0.01 for k in K)
    ids = collections.Counter(m[0] for m in d)
    assert all(abs(ids[i] / 60000 - 1 / 12) < 0.006 for i in range(12))
    # draw c uses outputs 8c .. 8c+K: the same draw from a later start
    assert S.draws(7, 123, 5, 3, 12) == d[123:128]


def test_rounds_sample_without_replacement_and_only_admissible_orders():
    from oracle import flip as F
    seen = set()
    for s in range(3):
        b = S.sample_round(1, seed=3, first=s * 20000, n_draws=20000, kcap=2, seen=seen, room=500)
        assert len(b) == len(set(b)) and not (set(b) & seen)
        assert all(F.admissible(S.key_modes(k)) for k in b)
        seen.update(b)
    assert len(seen) > 500


def test_small_languages_are_covered_exactly_once():
    from oracle import flip as F
    seen = set()
    for s in range(40):
        seen.update(S.sample_round(1, seed=11, first=s * 4000, n_draws=4000, kcap=1, seen=set(seen), room=10 ** 6))
    single = {int(k) for k in F.seed(1)}
    assert seen == single and len(single) == 279
    seen = set()
    for s in range(4):
        seen.update(S.sample_round(0, seed=5, first=s * 200, n_draws=200, kcap=1, seen=set(seen), room=10 ** 6))
    assert seen == {S.key_make([i]) for i in range(12)}
