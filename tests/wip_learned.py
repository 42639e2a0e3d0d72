"""What the trained refinement predictor gains over regridding without it
(GPU).  The network is trained by the library's own kernels on tags that the
solver generates, then three regrid policies advance the same seeded run
under the plain-tag judge with fallback, so every policy advances on meshes
that cover the plain tags:

  plain every 2 steps, plain every 8 steps, learned every 8 steps.

The gain is counted in regrid operations, which is what the network is for:
the learned policy needs fewer fallbacks than plain regridding at the same
interval, and fewer regrids in total than plain regridding every 2 steps.
Wall-clock figures are printed, not asserted."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

N = 16
STEPS = 48


@pytest.fixture(scope="module")
def setup():
    from paper_2508_05020_amd import amr, learned, workloads as W
    seeds = [4000, 4001, 4002]
    mean, std = learned.input_statistics([learned.uniform_config(64, N)], seeds[:1], steps=8)
    data = learned.build_dataset((64, 128), seeds, steps=32, horizon=8, stride=2,
                                 mean=mean, std=std, n=N)
    pos = float(data.y.mean())
    pos_weight = float(min(100.0, (1.0 - pos) / max(pos, 1e-6)))
    cfg = W.AMRConfig(name="learned-eval", dim=2, base_cells=128, patch_cells=[N] * 4,
                      periodic=[True, True], ic="quadrants_blobs", tag_buffer=2,
                      max_patches=8192)
    return amr, learned, W, cfg, data, mean, std, pos_weight


def _hier(amr, W, cfg, seed):
    h = amr.Hierarchy(cfg)
    amr.init_from_ic(h, W.initial_data(cfg, seed))
    return h


def test_learned_regridding_gain(setup):
    amr, learned, W, cfg, data, mean, std, pos_weight = setup
    seed = 4100
    h_bl = _hier(amr, W, cfg, seed)
    pred = amr.Predictor(h_bl, N, mean, std, pos_weight=pos_weight, max_batch=256)
    pred.set_weights(learned.init_weights(seed=1))
    losses = learned.train(pred, data, epochs=8, lr=2e-3, batch=64)
    assert losses[-1] < 0.7 * losses[0], losses
    tau = learned.choose_tau(pred, data, recall=0.995)

    runs = {}
    for name, every, policy in (("B2", 2, "plain"), ("B8", 8, "plain"), ("BL", 8, "learned")):
        h = h_bl if policy == "learned" else _hier(amr, W, cfg, seed)
        runs[name] = learned.run_policy(h, STEPS, every, policy,
                                        pred if policy == "learned" else None, tau, judge=True)
        print(name, runs[name].as_dict())
    b2, b8, bl = runs["B2"], runs["B8"], runs["BL"]
    # the network forecasts where tags appear: fewer fallbacks than plain
    # regridding at the same interval
    assert bl.fallbacks < b8.fallbacks, (bl.as_dict(), b8.as_dict())
    # and fewer regrid operations than plain regridding every 2 steps
    assert bl.regrids + bl.fallbacks < b2.regrids + b2.fallbacks, (bl.as_dict(), b2.as_dict())
    # all three advanced the same physical time to within the step-size spread
    assert abs(bl.t_sim - b2.t_sim) <= 0.05 * b2.t_sim
