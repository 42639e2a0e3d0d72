"""What the trained 3D refinement predictor gains over regridding without it
(GPU).  The 3D network (8^3 tiles) is trained by the library's own kernels on
tags from single-level runs of the blast + density-perturbation generator at
the resolutions of the hierarchy's levels, then one seeded 4-level run
(16^3 base, 8^3 patches) advances under three regrid policies, each under the
plain-tag judge with fallback:

  plain every 2 steps, plain every 16 steps, learned every 16 steps (two
  predict + regrid rounds per regrid, so that a forecast feature can gain
  two levels at once).

The gain is counted in judge failures and regrid operations, which do not
depend on timing.  Wall-clock figures are printed, not asserted."""
import pytest

pytestmark = pytest.mark.gpu

N = 8
H = 16
STEPS = 64


@pytest.fixture(scope="module")
def setup():
    from paper_2508_05020_amd import amr, learned, workloads as W
    cfg = W.AMRConfig(name="learned3-eval", dim=3, base_cells=16, patch_cells=[N] * 4,
                      periodic=[True] * 3, ic="blasts_perturbed", tag_buffer=1,
                      max_patches=32768)
    seeds = [5000, 5001]
    resolutions = (16, 32, 64, 128)
    mean, std = learned.input_statistics([learned.uniform_config(16, N, tag_buffer=1, dim=3)],
                                         seeds[:1], steps=8)
    data = learned.build_dataset(resolutions, seeds, steps=40, horizon=H, stride=4, mean=mean,
                                 std=std, n=N, tag_buffer=1, dim=3)
    val = learned.build_dataset(resolutions[-2:], [5100], steps=40, horizon=H, stride=4,
                                mean=mean, std=std, n=N, tag_buffer=1, dim=3)
    pos = float(data.y.mean())
    pos_weight = float(min(100.0, (1.0 - pos) / max(pos, 1e-6)))
    return amr, learned, W, cfg, data, val, mean, std, pos_weight


def _hier(amr, W, cfg, seed=5100):
    h = amr.Hierarchy(cfg)
    amr.init_from_ic(h, W.initial_data(cfg, seed))
    return h


def test_learned_regridding_gain_3d(setup):
    amr, learned, W, cfg, data, val, mean, std, pos_weight = setup
    h = _hier(amr, W, cfg)
    learned.run_policy(h, 8, 2, "plain", judge=True)   # warm-up outside the comparison
    h.close()

    h_bl = _hier(amr, W, cfg)
    pred = amr.Predictor(h_bl, N, mean, std, pos_weight=pos_weight, max_batch=256)
    pred.set_weights(learned.init_weights(seed=1, dim=3))
    losses = learned.train(pred, data, epochs=10, lr=2e-3, batch=64)
    assert losses[-1] < 0.7 * losses[0], losses
    tau = learned.choose_tau(pred, val, recall=0.99)
    met = learned.patch_metrics(pred, val, tau)
    print("validation", met, "tau", tau)
    assert met["recall"] >= 0.98
    pred.predict(0, tau)

    runs = {}
    for name, every, policy in (("plain2", 2, "plain"), ("plain16", H, "plain"),
                                ("learned16", H, "learned")):
        h = h_bl if policy == "learned" else _hier(amr, W, cfg)
        runs[name] = learned.run_policy(h, STEPS, every, policy,
                                        pred if policy == "learned" else None, tau, judge=True,
                                        rounds=2)
        print(name, runs[name].as_dict())
    p2, p16, l16 = runs["plain2"], runs["plain16"], runs["learned16"]
    assert abs(l16.t_sim - p2.t_sim) <= 0.02 * p2.t_sim
    # identical (full) plain-tag coverage: after every step the judge's
    # plain regrids leave no tagged cell outside the finest leaves
    for r in runs.values():
        assert r.uncovered_steps == 0 and r.as_dict()["coverage"] == 1.0, r.as_dict()
    # forecasting: at most half the judge failures of plain regridding at the
    # same interval
    assert l16.fallbacks <= 0.5 * p16.fallbacks, (l16.as_dict(), p16.as_dict())
    assert l16.regrids + l16.fallbacks < 0.5 * (p2.regrids + p2.fallbacks)
    pred.close()
