"""The learned refinement predictor's HIP kernels against the CPU reference
(GPU).  MFMA lane layout; input gather bitwise; forward logits against the
BF16-emulating reference; gradients against the FP64 reference backward; the
Adam step; training lowers the loss on the solver's own tags."""
import numpy as np
import pytest

from oracle import cnn
from tests import _harness as H

pytestmark = pytest.mark.gpu

N16 = 16


@pytest.fixture(scope="module")
def amr():
    import paper_2508_05020_amd.amr as A
    return A


def _bits_to_f32(x_int16):
    u = x_int16.cpu().numpy().view(np.uint16).astype(np.uint32) << 16
    return u.view(np.float32)


def _f32_to_bits(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a, np.float32)).to(torch.bfloat16).view(torch.int16)


def _to_oracle_x(x_int16, n):
    f = _bits_to_f32(x_int16).reshape(x_int16.shape[0], n + 6, n + 6, 4)
    return np.transpose(f, (0, 3, 1, 2)).astype(np.float64)


def _params_from_flat(w):
    w = np.asarray(w, np.float64)
    o = 0
    W1 = w[o:o + 576].reshape(16, 4, 3, 3); o += 576
    b1 = w[o:o + 16]; o += 16
    W2 = w[o:o + 2304].reshape(16, 16, 3, 3); o += 2304
    b2 = w[o:o + 16]; o += 16
    W3 = w[o:o + 144].reshape(1, 16, 3, 3); o += 144
    b3 = w[o:o + 1]
    return [W1, b1, W2, b2, W3, b3]


def _flat(params):
    return np.concatenate([np.asarray(p, np.float64).ravel() for p in params])


NORM_MEAN = (0.8, 0.0, 0.0, 0.9)
NORM_STD = (0.4, 0.3, 0.3, 0.4)


def _setup(amr):
    o, h, pid_of, key_of = H.mirror_case("2d", amr)
    pred = amr.Predictor(h, N16, NORM_MEAN, NORM_STD, pos_weight=4.0, max_batch=64)
    leaves = [pid_of[k] for k in o.forest.leaves() if o.cfg.patch_cells[k[0]] == N16][:48]
    return o, h, pid_of, key_of, pred, leaves


def test_mfma_lane_layout(amr):
    import torch
    from paper_2508_05020_amd import workloads as W
    cfg = W.AMRConfig(name="t", dim=2, base_cells=64, patch_cells=[16], periodic=[True, True],
                      max_patches=64)
    h = amr.Hierarchy(cfg)
    rng = np.random.default_rng(0)
    A = rng.integers(-8, 8, size=(16, 16)).astype(np.float32)
    B = rng.integers(-8, 8, size=(16, 16)).astype(np.float32)
    a = _f32_to_bits(A).cuda()
    b = _f32_to_bits(B).cuda()
    d = torch.zeros(256, dtype=torch.float32, device="cuda")
    amr.mfma_selftest(h, a, b, d)
    got = d.cpu().numpy().reshape(16, 16)
    assert np.array_equal(got, A @ B)


def test_gather_bitwise(amr):
    o, h, pid_of, key_of, pred, leaves = _setup(amr)
    x = pred.gather(0, leaves)
    o.fill_ghosts(0, o.forest.leaves())
    g = o.cfg.gamma
    istd = [np.float32(1.0) / np.float32(s) for s in NORM_STD]
    for b, pid in enumerate(leaves):
        a = o.U[0][key_of[pid]][:, 1:-1, 1:-1]   # cells -3 .. n+2
        rho, mx, my, E = a
        ux = mx / rho
        uy = my / rho
        ke = mx * ux
        ke = ke + my * uy
        ke = 0.5 * ke
        p = (g - 1.0) * (E - ke)
        ref = []
        for c, f in enumerate((rho, ux, uy, p)):
            z = (f - np.float64(np.float32(NORM_MEAN[c]))) * np.float64(istd[c])
            ref.append(cnn.bf16_round(z.astype(np.float32)))
        ref = np.stack(ref, axis=-1).reshape(-1, 4)
        got = _bits_to_f32(x[b])
        assert np.array_equal(got, ref), pid


def test_forward_matches_bf16_reference(amr):
    o, h, pid_of, key_of, pred, leaves = _setup(amr)
    params = cnn.init_params(4, 16, 2, seed=11)
    params = [p + 0.05 * np.random.default_rng(1).normal(size=np.shape(p)) for p in params]
    pred.set_weights(_flat(params))
    x = pred.gather(0, leaves)
    z = pred.forward(x).cpu().numpy().reshape(len(leaves), N16, N16)
    ref, _ = cnn.forward(_to_oracle_x(x, N16), _params_from_flat(pred.get_weights()), bf16=True)
    scale = np.max(np.abs(ref))
    assert np.max(np.abs(z - ref)) <= 2e-2 * scale, (np.max(np.abs(z - ref)), scale)


def test_gradients_match_reference(amr):
    import torch
    o, h, pid_of, key_of, pred, leaves = _setup(amr)
    params = cnn.init_params(4, 16, 2, seed=12)
    pred.set_weights(_flat(params))
    x = pred.gather(0, leaves)
    refine, coarsen, cells = h.tag(0, cell_tags=True)
    labels = _labels(h, cells, leaves, N16)
    grads = torch.zeros(pred.nparams, dtype=torch.float32, device="cuda")
    loss = pred.train_step(x, torch.from_numpy(labels).cuda(), lr=0.0, grads=grads)
    g = grads.cpu().numpy()
    w_bf = cnn.bf16_round(pred.get_weights())
    rl, rg = cnn.backward(_to_oracle_x(x, N16), _params_from_flat(w_bf),
                          labels.reshape(len(leaves), N16, N16).astype(float), 4.0)
    assert loss.item() == pytest.approx(rl, rel=2e-2)
    ref = _flat(rg)
    offs = [0, 576, 592, 2896, 2912, 3056, 3057]
    # per parameter block: element-wise, max |g - ref| against the block's
    # largest reference gradient, and the L2 relative error
    for a, b in zip(offs[:-1], offs[1:]):
        scale = max(float(np.max(np.abs(ref[a:b]))), 1e-12)
        elem = float(np.max(np.abs(g[a:b] - ref[a:b]))) / scale
        l2 = np.linalg.norm(g[a:b] - ref[a:b]) / max(np.linalg.norm(ref[a:b]), 1e-12)
        print(f"block [{a}, {b}): element-wise {elem:.3e}, L2 {l2:.3e}")
        assert elem <= 2e-2 and l2 <= 2e-2, (a, b, elem, l2)


def test_adam_step_matches_reference(amr):
    import torch
    o, h, pid_of, key_of, pred, leaves = _setup(amr)
    params = cnn.init_params(4, 16, 2, seed=13)
    pred.set_weights(_flat(params))
    w0 = pred.get_weights()
    x = pred.gather(0, leaves)
    refine, coarsen, cells = h.tag(0, cell_tags=True)
    labels = torch.from_numpy(_labels(h, cells, leaves, N16)).cuda()
    grads = torch.zeros(pred.nparams, dtype=torch.float32, device="cuda")
    pred.train_step(x, labels, lr=1e-3, grads=grads)
    w1 = pred.get_weights()
    exp, _, _ = cnn.adam_step([w0], [grads.cpu().numpy()], [np.zeros_like(w0)],
                              [np.zeros_like(w0)], 1, 1e-3)
    assert np.allclose(w1, exp[0], rtol=1e-5, atol=1e-7)


def test_training_lowers_loss(amr):
    import torch
    o, h, pid_of, key_of, pred, leaves = _setup(amr)
    pred.set_weights(_flat(cnn.init_params(4, 16, 2, seed=14)))
    x = pred.gather(0, leaves)
    refine, coarsen, cells = h.tag(0, cell_tags=True)
    labels = torch.from_numpy(_labels(h, cells, leaves, N16)).cuda()
    first = pred.train_step(x, labels, lr=3e-3).item()
    for _ in range(150):
        last = pred.train_step(x, labels, lr=3e-3).item()
    assert last < 0.5 * first, (first, last)


def _labels(h, cells, leaves, n):
    flat = cells.cpu().numpy()
    out = np.zeros((len(leaves), n * n), np.uint8)
    for b, pid in enumerate(leaves):
        off = h.offset(pid) // h.nvar
        box = flat[off:off + (n + 8) ** 2].reshape(n + 8, n + 8)
        out[b] = box[4:-4, 4:-4].ravel()
    return out
