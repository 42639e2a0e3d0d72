"""Host-side logic of the learned regridding policy (CPU): the probability
threshold for a target patch recall, the patch metrics, and the run
statistics.  The predictor is replaced by a stub that returns fixed logits."""
import math

import numpy as np
import pytest

torch = pytest.importorskip("torch")
from paper_2508_05020_amd import learned  # noqa: E402


class StubPredictor:
    """forward(x) -> logits [B, cells]; patch b's cell logits all equal
    scores[b] except one cell at scores[b] + 0 (the max is scores[b])."""

    def __init__(self, scores, cells=16, max_batch=4):
        self.scores = np.asarray(scores, np.float32)
        self.cells = cells
        self.max_batch = max_batch

    def forward(self, x):
        idx = x[:, 0, 0].long().numpy()
        z = np.repeat(self.scores[idx][:, None] - 5.0, self.cells, axis=1)
        z[:, 3] = self.scores[idx]
        return torch.from_numpy(z)


def _data(npatch, positive):
    x = torch.zeros(npatch, 4, 4, dtype=torch.int16)
    x[:, 0, 0] = torch.arange(npatch, dtype=torch.int16)
    y = np.zeros((npatch, 16), np.uint8)
    for b in positive:
        y[b, 5] = 1
    return learned.Dataset(x, y, 4)


def test_tau_meets_recall_and_is_tight():
    scores = np.linspace(-4.0, 5.0, 40)
    positive = list(range(0, 40, 2))
    data = _data(40, positive)
    pred = StubPredictor(scores)
    for recall in (0.5, 0.9, 0.99):
        tau = learned.choose_tau(pred, data, recall=recall)
        assert 0.0 < tau < 1.0
        met = learned.patch_metrics(pred, data, tau)
        assert met["recall"] >= recall
        # tight: the lowest flagged positive is the k-th smallest positive score
        zt = math.log(tau / (1.0 - tau))
        pos_scores = np.sort(scores[positive])
        k = int(math.floor((1.0 - recall) * len(pos_scores)))
        assert pos_scores[k] > zt >= pos_scores[k] - 2e-3
        assert met["positive"] == pytest.approx(0.5)


def test_tau_stays_inside_the_unit_interval_for_saturated_logits():
    data = _data(8, [0, 1, 2, 3])
    tau = learned.choose_tau(StubPredictor([60.0] * 8), data, recall=0.9)
    assert 0.0 < tau < 1.0 and tau == pytest.approx(1.0 / (1.0 + math.exp(-15.0)))
    tau = learned.choose_tau(StubPredictor([-60.0] * 8), data, recall=0.9)
    assert 0.0 < tau < 1.0 and tau == pytest.approx(1.0 / (1.0 + math.exp(15.0)))


def test_tau_without_positive_patches():
    assert learned.choose_tau(StubPredictor(np.zeros(6)), _data(6, []), recall=0.99) == 0.5


def test_run_stats():
    st = learned.RunStats("plain", 100, 2.0, 0.5, 25, 3, 4, 10)
    d = st.as_dict()
    assert d["wall_per_tsim"] == pytest.approx(4.0)
    assert d["coverage"] == pytest.approx(0.96)
    assert learned.RunStats("plain", 1, 1.0, 0.0, 0, 0, 0, 0).wall_per_tsim == float("inf")
