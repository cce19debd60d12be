"""Host logic of the cost model (no GPU): the record arrays and their masks, the slab-scale
mapping, and the regret bookkeeping."""
import math

import numpy as np

from paper_2305_17813_amd import costmodel as CM
from paper_2305_17813_amd import native


def _records():
    rec = CM.Records()
    rng = np.random.default_rng(0)
    for i in range(4):  # timing records: no slab scale
        rec.X.append(rng.normal(size=CM.N_IN).astype(np.float32))
        rec.t_incr.append(1.0 + i)
        rec.t_rec.append(10.0 / (1 + i))
        rec.algo.append(i % len(CM.ALGOS))
        rec.state.append(i)
        rec.slab_scale.append(float("nan"))
    for i in range(2):  # slab-scale records: no timings
        rec.scale_ms[len(rec.X)] = (3.0, 2.0, 4.0)
        rec.X.append(rng.normal(size=CM.N_IN).astype(np.float32))
        rec.t_incr.append(float("nan"))
        rec.t_rec.append(float("nan"))
        rec.algo.append(-1)
        rec.state.append(100 + i)
        rec.slab_scale.append(math.log2(1.0))
    return rec


def test_record_arrays_mask_what_a_record_lacks():
    X, T, M, ti, tr, algo, state = _records().arrays()
    assert X.shape == (6, CM.N_IN) and T.shape == (6, 3) and M.shape == (6, 3)
    assert np.isfinite(T).all()
    assert (M[:4] == [1, 1, 0]).all() and (M[4:] == [0, 0, 1]).all()
    assert np.allclose(T[:4, 0], np.log([1, 2, 3, 4])) and np.allclose(T[:4, 1], np.log(10.0 / np.arange(1, 5)))
    assert (T[4:, :2] == 0).all() and (T[4:, 2] == 0).all()  # log2(1) = 0


def test_load_factor_for_scales():
    assert CM.load_factor_for(1.0) == CM.BASE_LOAD_FACTOR
    assert math.isclose(CM.load_factor_for(2.0), CM.BASE_LOAD_FACTOR / 2)
    assert math.isclose(CM.load_factor_for(0.5), CM.BASE_LOAD_FACTOR * 2)


class _Fixed(CM.CostModel):
    """A cost model whose predictions are given (no MLP)."""

    def __init__(self, y):
        self.y = np.asarray(y, np.float32)

    def predict(self, X):
        return self.y[: np.atleast_2d(X).shape[0]]


def test_slab_scale_picks_the_nearest_measured_scale_in_log2():
    y = [[0, 0, -3.0], [0, 0, -0.6], [0, 0, -0.4], [0, 0, 0.49], [0, 0, 0.51], [0, 0, 5.0]]
    picks = _Fixed(y).slab_scale(np.zeros((6, CM.N_IN)))
    assert picks.tolist() == [0.5, 0.5, 1.0, 1.0, 2.0, 2.0]


def test_scale_regret_and_choice_rule():
    rec = _records()
    cm = _Fixed([[0, 0, 1.0]] * 2)  # predicts scale 2 for both slab records
    r = CM.scale_regret(cm, rec, [4, 5, 0])  # a timing record index is ignored
    assert r == {"policy_ms": 8.0, "best_ms": 4.0, "default_ms": 4.0}
    # log ms predictions: a recompute is taken only when predicted RECOMPUTE_MARGIN faster
    choice = _Fixed([[1.0, 2.0, 0], [3.0, 2.0, 0], [2.1, 2.0, 0]]).choose(np.zeros((3, CM.N_IN)))
    assert choice.tolist() == [native.INCR, native.RECOMPUTE, native.INCR]
    choice = choice[:2]
    reg = CM.regret(np.array([1.0, 5.0]), np.array([2.0, 3.0]), choice)
    assert reg["policy_ms"] == 4.0 and reg["best_ms"] == 4.0 and reg["always_incremental_ms"] == 6.0
