"""Host logic of the surrogate sweep (no GPU): the held-out split used to
calibrate the ensemble spread, and the fallback rule's default multiplier."""
import numpy as np

from paper_2405_03474_amd import sweep


def test_split_holdout_partitions():
    tr, ho = sweep.split_holdout(1000, 0.1, seed=3)
    assert len(ho) == 100 and len(tr) == 900
    assert np.array_equal(np.sort(np.concatenate([tr, ho])), np.arange(1000))
    tr2, ho2 = sweep.split_holdout(1000, 0.1, seed=3)
    assert np.array_equal(ho, ho2)                      # seeded


def test_default_rule_is_the_raw_spread():
    cfg = sweep.Config()
    assert cfg.kappa == 1.0 and cfg.rel_tol == 1e-3
