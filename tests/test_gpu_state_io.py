"""Patch state transfer through the C-ABI (GPU): whole patch arrays up and
down in any pid order (copies merged over patches adjacent in a level's
pool), and the primitive upload of Eq. (4), (6), m_j = rho u_j and
E = p / (gamma - 1) + rho |u|^2 / 2, against the same conversion on the host,
bit for bit, with ghost cells left untouched."""
import numpy as np
import pytest

from paper_2508_05020_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def amr():
    import paper_2508_05020_amd.amr as A
    return A


def _refined(amr, d, base, max_patches=8192, seed=0):
    cfg = W.AMRConfig(name="io", dim=d, base_cells=base, patch_cells=[8, 8, 8],
                      periodic=[True] * d, max_patches=max_patches)
    h = amr.Hierarchy(cfg)
    rng = np.random.default_rng(seed)
    for lev in range(2):
        table = h.patch_table()
        rq = np.zeros(cfg.max_patches, np.uint8)
        leaves = [t["pid"] for t in table if t["nchildren"] == 0 and t["level"] == lev]
        rq[rng.choice(leaves, max(1, len(leaves) // 6), replace=False)] = 1
        h.regrid(rq, np.zeros_like(rq))
    table = h.patch_table()
    assert len({t["level"] for t in table}) == 3
    return cfg, h, {t["pid"]: t["level"] for t in table}


def _host_conserved(prim, d, gamma):
    rho, p = prim[0], prim[d + 1]
    out = np.empty_like(prim)
    out[0] = rho
    uu = None
    for j in range(d):
        u = prim[1 + j]
        uu = u * u if j == 0 else uu + u * u
        out[1 + j] = rho * u
    out[d + 1] = p / (gamma - 1.0) + 0.5 * rho * uu
    return out


def _random_patch(rng, shape):
    return rng.standard_normal(shape)


@pytest.mark.parametrize("d", [1, 2, 3])
def test_state_roundtrip_any_order(d, amr):
    cfg, h, levels = _refined(amr, d, {1: 128, 2: 64, 3: 32}[d])
    rng = np.random.default_rng(10 + d)
    pids = sorted(levels)
    shapes = {p: a.shape for p, a in h.get_state(0, pids, levels).items()}
    first = {p: rng.standard_normal(shapes[p]) for p in pids}
    h.set_state(1, first)                                   # pool order: long runs
    order = [int(p) for p in rng.permutation(pids)]
    got = h.get_state(1, order, levels)                     # scattered: short runs
    assert all(np.array_equal(got[p], first[p]) for p in pids)
    second = {p: rng.standard_normal(shapes[p]) for p in order}
    h.set_state(1, second)
    got = h.get_state(1, pids[::-1], levels)
    assert all(np.array_equal(got[p], second[p]) for p in pids)
    sub = pids[1::3]
    got = h.get_state(1, sub, levels)
    assert all(np.array_equal(got[p], second[p]) for p in sub)


def _check_prim_upload(h, cfg, levels, order, rng):
    d = cfg.dim
    pids = sorted(levels)
    shapes = {p: a.shape for p, a in h.get_state(0, pids, levels).items()}
    sentinel = {p: np.full(shapes[p], -7.25) for p in pids}
    h.set_state(0, sentinel)
    prims = {}
    for p in order:
        n = cfg.patch_cells[levels[p]]
        a = rng.standard_normal((d + 2,) + (n,) * d)
        a[0] = rng.uniform(0.1, 3.0, a[0].shape)
        a[d + 1] = rng.uniform(0.1, 3.0, a[0].shape)
        prims[p] = a
    h.set_state_prim(0, prims)
    got = h.get_state(0, pids, levels)
    inner = (slice(None),) + (slice(4, -4),) * d
    for p in pids:
        ref = np.array(sentinel[p])
        if p in prims:
            ref[inner] = _host_conserved(prims[p], d, cfg.gamma)
        assert np.array_equal(got[p], ref), p


@pytest.mark.parametrize("d", [1, 2, 3])
def test_set_state_prim_matches_host_conversion(d, amr):
    cfg, h, levels = _refined(amr, d, {1: 128, 2: 64, 3: 32}[d])
    rng = np.random.default_rng(20 + d)
    pids = sorted(levels)
    order = [int(p) for p in rng.permutation(pids)][: (2 * len(pids)) // 3]
    _check_prim_upload(h, cfg, levels, order, rng)


def test_set_state_prim_many_batches(amr):
    """More than 64 Ki patches and 128 MiB of primitives in one call: the
    upload goes through the staging buffer in several batches."""
    cfg = W.AMRConfig(name="io", dim=2, base_cells=2048, patch_cells=[8, 8],
                      periodic=[True, True], max_patches=65536 + 4096,
                      level_capacity=(65536, 4096))
    h = amr.Hierarchy(cfg)
    rq = np.zeros(cfg.max_patches, np.uint8)
    rq[np.random.default_rng(3).choice(65536, 700, replace=False)] = 1
    h.regrid(rq, np.zeros_like(rq))
    levels = {t["pid"]: t["level"] for t in h.patch_table()}
    assert len(levels) > 65536
    rng = np.random.default_rng(4)
    _check_prim_upload(h, cfg, levels, [int(p) for p in rng.permutation(sorted(levels))], rng)


def test_set_state_inactive_pid_writes_nothing(amr):
    cfg, h, levels = _refined(amr, 2, 64)
    pids = sorted(levels)
    shapes = {p: a.shape for p, a in h.get_state(0, pids, levels).items()}
    before = h.get_state(0, pids, levels)
    free = next(p for p in range(cfg.max_patches) if p not in levels)
    bad = {pids[0]: np.zeros(shapes[pids[0]]), free: np.zeros(shapes[pids[0]])}
    with pytest.raises(amr.AMRError):
        h.set_state(0, bad)
    n = cfg.patch_cells[levels[pids[0]]]
    with pytest.raises(amr.AMRError):
        h.set_state_prim(0, {pids[0]: np.ones((4, n, n)), free: np.ones((4, n, n))})
    after = h.get_state(0, pids, levels)
    assert all(np.array_equal(after[p], before[p]) for p in pids)
