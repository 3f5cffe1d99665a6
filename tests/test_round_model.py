"""The multi-pick round's certification rule, modelled on the CPU
(tests/round_model.py), gives the oracle's sequence: random, tie-heavy,
duplicated and planar clouds under many group counts, lookahead depths and
list caps (small caps force the cut of a long list at a key boundary)."""
import numpy as np
import pytest

import oracle
import round_model


def _cloud(rng, kind, n):
    if kind == 0:
        return rng.random((n, 3), dtype=np.float32)
    if kind == 1:
        return rng.integers(0, 4, size=(n, 3)).astype(np.float32)              # heavy ties
    if kind == 2:
        return np.repeat(rng.random((max(1, n // 4), 3), dtype=np.float32), 4, axis=0)  # duplicates
    if kind == 3:
        return np.c_[rng.integers(0, 8, size=(n, 2)), np.zeros(n)].astype(np.float32)  # planar lattice
    if kind == 4:
        return (rng.normal(size=(n, 3)) * 3).astype(np.float32)
    return rng.integers(0, 2, size=(n, 3)).astype(np.float32)                  # 8 distinct points


@pytest.mark.parametrize("seed", range(6))
def test_round_model_matches_oracle(oracle_lib, seed):
    rng = np.random.default_rng(100 + seed)
    for it in range(8):
        P = _cloud(rng, (seed + it) % 6, int(rng.integers(2, 260)))
        n = len(P)
        m = int(rng.integers(1, n + 1))
        s = int(rng.integers(0, n))
        G = int(rng.choice([1, 2, 3, 5, 8, 16, 64]))
        R = int(rng.choice([2, 3, 4, 8]))
        klist = int(rng.choice([4, 16, 128]))
        ri, rd = oracle_lib.fps(P, m, s)
        gi, gd, _, _ = round_model.run(P, m, s, G, R, klist=klist)
        assert np.array_equal(gi, ri), (seed, it, n, m, s, G, R, klist)
        assert np.array_equal(gd.view(np.uint32), rd.view(np.uint32)), (seed, it, n, m, s, G, R, klist)


def test_round_model_settles_many_picks_per_round(oracle_lib):
    # the point of the rule: far fewer rounds than selections
    P = np.random.default_rng(7).random((600, 3), dtype=np.float32)
    ri, _ = oracle_lib.fps(P, 300, 0)
    gi, _, rounds, _ = round_model.run(P, 300, 0, 32, 2)
    assert np.array_equal(gi, ri)
    assert rounds < 300 // 3
