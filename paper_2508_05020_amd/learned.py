"""Learned refinement predictor: training data, training loop and the
regridding policies that use it.  Every numerical step runs in libamr
(gather, forward, backward, Adam, tagging, regridding); this module only
sequences calls and moves small host-side arrays.

Labels come from the solver itself: for a patch at step t, a cell is positive
when the plain gradient tagger tags it (after dilation) at any step in
(t, t + horizon].  Training data are recorded on single-level periodic runs
at several resolutions (the 2D quadrant + blob generator, or the 3D blast +
perturbation generator), so that the network sees features at the cell sizes
of several AMR levels.  In 3D a training patch is one 8^3 tile.

Policies (wall-clock per unit simulated time is the figure of merit):
  plain  -- gradient tagging + regrid every ``every`` steps;
  learned -- every ``every`` steps regrid with refine = plain | predicted and
             coarsen = plain & predicted.
With the judge on, after every step the plain tagger checks that every tagged
cell lies in a leaf of the finest level allowed, and an immediate plain regrid
follows when one does not (the fallback).  Every policy run under the judge
therefore advances on meshes that cover the plain tags at the same rate, and
the policies differ only in how many regrids and fallbacks that costs.
"""
from __future__ import annotations

import dataclasses
import math
import sys
import time
from typing import Dict, List, Optional, Sequence

import numpy as np

from . import amr as A
from . import workloads as W


def net_shape(dim: int):
    """(input channels, hidden channels, taps) of the network."""
    return (4, 16, 9) if dim == 2 else (5, 8, 27)


def init_weights(seed: int, dim: int = 2) -> np.ndarray:
    """He-normal weights, zero biases, in the flat parameter layout of the
    library: W1 [ch][cin][taps], b1, W2 [ch][ch][taps], b2, W3 [ch][taps], b3
    with (cin, ch, taps) = (4, 16, 3x3) in 2D and (5, 8, 3x3x3) in 3D."""
    c0, c1, k = net_shape(dim)
    rng = np.random.default_rng(seed)
    parts = [rng.normal(0.0, math.sqrt(2.0 / (c0 * k)), c1 * c0 * k), np.zeros(c1),
             rng.normal(0.0, math.sqrt(2.0 / (c1 * k)), c1 * c1 * k), np.zeros(c1),
             rng.normal(0.0, math.sqrt(2.0 / (c1 * k)), c1 * k), np.zeros(1)]
    return np.concatenate(parts).astype(np.float32)


def uniform_config(base: int, n: int = 32, tag_buffer: int = 2, cfl: float = 0.5,
                   max_patches: int = 4096, dim: int = 2) -> W.AMRConfig:
    ic = "quadrants_blobs" if dim == 2 else "blasts_perturbed"
    return W.AMRConfig(name=f"uniform{base}", dim=dim, base_cells=base, patch_cells=[n],
                       periodic=[True] * dim, cfl=cfl, tag_buffer=tag_buffer,
                       ic=ic, max_patches=max_patches, regrid_interval=0)


def _interior_index(h: A.Hierarchy, pids: Sequence[int], n: int):
    """Device index of the interior cells of the given patches in the
    hierarchy's cell-tag layout, [len(pids), n^d] (row-major interior)."""
    torch = A._torch()
    d = h.cfg.dim
    box = np.arange((n + 8) ** d, dtype=np.int64).reshape((n + 8,) * d)
    inner = box[(slice(4, -4),) * d].ravel()
    base = np.array([h.offset(pid) // h.nvar for pid in pids], np.int64)
    return torch.from_numpy(base[:, None] + inner[None, :]).to(h.device)


def record(cfg: W.AMRConfig, seed: int, steps: int, horizon: int, stride: int,
           mean, std):
    """Input tiles (device, BF16 bits) and labels (host) of one uniform run."""
    torch = A._torch()
    h = A.Hierarchy(cfg)
    A.init_from_ic(h, W.initial_data(cfg, seed))
    n = cfg.patch_cells[0]
    pred = A.Predictor(h, n, mean, std, max_batch=1)
    pids = [r["pid"] for r in h.patch_table()]
    idx = _interior_index(h, pids, n)
    xs, tags = [], []
    snaps = []
    for t in range(steps + horizon + 1):
        if t < steps and t % stride == 0:
            xs.append(pred.gather(0, pids))
            snaps.append(t)
        _, _, cells = h.tag(0, cell_tags=True)
        tags.append(cells[idx].cpu().numpy())
        h.step()
    ys = []
    for t in snaps:
        y = tags[t + 1].copy()
        for s in range(t + 2, t + horizon + 1):
            y |= tags[s]
        ys.append(y)
    pred.close()
    h.close()
    return torch.cat(xs), np.concatenate(ys)


def input_statistics(cfgs, seeds, steps=16):
    """Per-channel mean and standard deviation of (rho, u, v, p) (2D) or
    (rho, u, v, w, p) (3D) over the recorded pixels (inputs gathered without
    normalisation)."""
    vals = []
    for cfg in cfgs:
        nch = cfg.dim + 2
        for seed in seeds:
            x, _ = record(cfg, seed, steps, horizon=1, stride=4, mean=(0,) * nch, std=(1,) * nch)
            u = x.cpu().numpy().view(np.uint16).astype(np.uint32) << 16
            vals.append(u.view(np.float32).reshape(-1, x.shape[-1])[:, :nch])
    v = np.concatenate(vals).astype(np.float64)
    return v.mean(axis=0), np.maximum(v.std(axis=0), 1e-3)


@dataclasses.dataclass
class Dataset:
    x: object            # torch int16 [S, (n+6)^d, channels] on the device
    y: np.ndarray        # uint8 [S, n^d]
    n: int


def build_dataset(resolutions: Sequence[int], seeds: Sequence[int], steps: int, horizon: int,
                  stride: int, mean, std, n: int = 32, tag_buffer: int = 2,
                  dim: int = 2) -> Dataset:
    """Inputs and labels of single-level runs at the given resolutions, the
    labels dilated by `tag_buffer` cells like the tagger they forecast."""
    torch = A._torch()
    xs, ys = [], []
    for base in resolutions:
        cfg = uniform_config(base, n, tag_buffer=tag_buffer, dim=dim,
                             max_patches=max(4096, (base // n) ** dim))
        for seed in seeds:
            x, y = record(cfg, seed, steps, horizon, stride, mean, std)
            xs.append(x)
            ys.append(y)
    return Dataset(torch.cat(xs), np.concatenate(ys), n)


def train(pred: A.Predictor, data: Dataset, epochs: int, lr: float, batch: int, seed: int = 0,
          log=None) -> List[float]:
    torch = A._torch()
    rng = np.random.default_rng(seed)
    S = data.x.shape[0]
    ydev = torch.from_numpy(data.y).to(data.x.device)
    losses = []
    for ep in range(epochs):
        perm = rng.permutation(S)
        tot, cnt = 0.0, 0
        for b0 in range(0, S - batch + 1, batch):
            idx = torch.from_numpy(perm[b0:b0 + batch]).to(data.x.device)
            loss = pred.train_step(data.x.index_select(0, idx).contiguous(),
                                   ydev.index_select(0, idx).contiguous(), lr)
            tot += loss.item()
            cnt += 1
        losses.append(tot / max(1, cnt))
        if log:
            log(f"epoch {ep}: loss {losses[-1]:.4f}")
    return losses


def patch_scores(pred: A.Predictor, x) -> np.ndarray:
    """Max logit per patch."""
    out = []
    for b0 in range(0, x.shape[0], pred.max_batch):
        z = pred.forward(x[b0:b0 + pred.max_batch].contiguous())
        out.append(z.max(dim=1).values.cpu().numpy())
    return np.concatenate(out)


def choose_tau(pred: A.Predictor, data: Dataset, recall: float = 0.995) -> float:
    """Probability threshold flagging at least `recall` of the patches that
    have a positive cell."""
    s = patch_scores(pred, data.x)
    pos = data.y.reshape(data.y.shape[0], -1).any(axis=1)
    if not pos.any():
        return 0.5
    zs = np.sort(s[pos])
    k = int(math.floor((1.0 - recall) * len(zs)))
    # the threshold as a probability strictly inside (0, 1) in float32 terms
    zt = float(np.clip(zs[k] - 1e-3, -15.0, 15.0))
    return float(1.0 / (1.0 + math.exp(-zt)))


def patch_metrics(pred: A.Predictor, data: Dataset, tau: float) -> Dict[str, float]:
    s = patch_scores(pred, data.x)
    zt = math.log(tau / (1.0 - tau))
    flag = s > zt
    pos = data.y.reshape(data.y.shape[0], -1).any(axis=1)
    tp = int((flag & pos).sum())
    return {"recall": tp / max(1, int(pos.sum())), "flagged": float(flag.mean()),
            "positive": float(pos.mean())}


# ---------------------------------------------------------------------------
# regridding policies
# ---------------------------------------------------------------------------


@dataclasses.dataclass
class RunStats:
    policy: str
    steps: int
    wall_s: float
    t_sim: float
    regrids: int
    fallbacks: int
    uncovered_steps: int
    cell_updates: int
    capacity_retries: int = 0   # learned regrids whose refinement did not fit the pools

    @property
    def wall_per_tsim(self) -> float:
        return self.wall_s / self.t_sim if self.t_sim > 0 else float("inf")

    def as_dict(self):
        d = dataclasses.asdict(self)
        d["wall_per_tsim"] = self.wall_per_tsim
        d["coverage"] = 1.0 - self.uncovered_steps / max(1, self.steps)
        return d


def learned_regrid(h: A.Hierarchy, pred: A.Predictor, tau: float, rounds: int = 1) -> int:
    """Up to `rounds` regrids with refine = predicted | plain tags and
    coarsen = predicted-quiet & plain coarsen requests (the first round only
    coarsens), each round predicting on the leaves the previous one created;
    returns the number of rounds that changed the mesh."""
    changed = 0
    for r in range(rounds):
        pr, pc = pred.predict(0, tau)
        tr, tc, _ = h.tag(0)
        # combined on the host: the flags come back for the host regrid anyway
        ref = pr.cpu().numpy() | tr.cpu().numpy()
        coa = (pc.cpu().numpy() & tc.cpu().numpy()) if r == 0 else np.zeros_like(ref)
        if not ref.any() and not coa.any():
            break
        nc, nd = h.regrid(ref, coa)
        if nc == 0 and nd == 0:
            break
        changed += 1
    return changed


def cover(h: A.Hierarchy, max_rounds: int) -> int:
    """The judge's fallback: plain regrids until the plain tagger finds no
    tagged cell outside the finest leaves (each regrid can add one level), at
    most ``max_rounds``; returns the regrids made, or -1 when the mesh still
    misses tags after them."""
    made = 0
    while h.judge():
        if made == max_rounds:
            return -1
        h.adapt()
        made += 1
    return made


def run_policy(h: A.Hierarchy, steps: int, every: int, policy: str = "plain",
               pred: Optional[A.Predictor] = None, tau: float = 0.5,
               judge: bool = False, rounds: int = 1, regrid_buffer: Optional[int] = None,
               capacity_retries: int = 3, progress: int = 0) -> RunStats:
    """Advance `steps` steps under a regrid policy; wall time includes
    tagging, prediction, judging and regridding.

    Every `every` steps the policy regrids (plain tags, or the predicted and
    plain requests together), with the tag dilation `regrid_buffer` when
    given (the hierarchy's own otherwise).  With the judge on, after every
    step (and its scheduled regrid) the plain tagger at the hierarchy's own
    dilation checks that the mesh the next step runs on covers every tagged
    cell; when it does not, plain regrids follow until it does (at most
    max_levels - 1, the fallback).  A step whose mesh still misses tags after
    that counts as uncovered, so coverage is the fraction of steps that ran
    on a mesh covering the plain tags."""
    torch = A._torch()
    dt = torch.zeros(1, dtype=torch.float64, device=h.device)
    tsim = torch.zeros(1, dtype=torch.float64, device=h.device)
    regrids = fallbacks = uncovered = cells = capacity = 0
    own_buffer = h.cfg.tag_buffer
    max_rounds = h.cfg.max_levels - 1
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for s in range(1, steps + 1):
        cells += h.leaf_cells()
        h.step(dt)
        tsim += dt
        if every > 0 and s % every == 0:
            regrids += 1
            if regrid_buffer is not None:
                h.set_tag_buffer(regrid_buffer)
            if policy == "plain":
                h.adapt()
            else:
                # a predicted refinement that does not fit the patch pools
                # leaves the mesh unchanged (the regrid is transactional):
                # retry with a stricter threshold (1 - tau halved), then
                # fall back to a plain regrid
                t = tau
                for attempt in range(capacity_retries + 1):
                    try:
                        learned_regrid(h, pred, t, rounds)
                        break
                    except A.AMRError as e:
                        if e.status != A.E_CAPACITY:
                            raise
                        capacity += 1
                        t = 0.5 * (1.0 + t)
                else:
                    h.adapt()
                    fallbacks += 1
            if regrid_buffer is not None:
                h.set_tag_buffer(own_buffer)
        if judge and s < steps:
            made = cover(h, max_rounds)
            if made != 0:
                fallbacks += 1
            if made < 0:
                uncovered += 1
        if progress and s % progress == 0:
            print(f"[policy] {policy}: step {s}/{steps}, {time.perf_counter() - t0:.1f} s",
                  file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    return RunStats(policy, steps, wall, float(tsim.item()), regrids, fallbacks, uncovered, cells,
                    capacity)
