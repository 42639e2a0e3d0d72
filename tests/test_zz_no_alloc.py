"""The primitive upload that allocates nothing (GPU, through the C-ABI).

amr_set_state_prim_noalloc stages through the library's fixed per-GPU
scratch array instead of an allocator buffer; its result must be the one
amr_set_state_prim gives, bit for bit, on two calls in a row (the second
smaller, so that the first call's leftovers in the scratch would show), and
a call larger than the scratch must be refused before anything is copied."""
import numpy as np
import pytest

from paper_2508_05020_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def amr():
    import paper_2508_05020_amd.amr as A
    return A


def _pair(amr, d, base):
    cfg = W.AMRConfig(name="na", dim=d, base_cells=base, patch_cells=[8, 8, 8],
                      periodic=[True] * d, max_patches=8192)
    hs = [amr.Hierarchy(cfg), amr.Hierarchy(cfg)]
    rng = np.random.default_rng(40 + d)
    for lev in range(2):
        table = hs[0].patch_table()
        rq = np.zeros(cfg.max_patches, np.uint8)
        leaves = [t["pid"] for t in table if t["nchildren"] == 0 and t["level"] == lev]
        rq[rng.choice(leaves, max(1, len(leaves) // 5), replace=False)] = 1
        for h in hs:
            h.regrid(rq, np.zeros_like(rq))
    table = hs[0].patch_table()
    assert table == hs[1].patch_table()
    return cfg, hs, {t["pid"]: t["level"] for t in table}


def _prims(rng, cfg, pids, levels):
    d = cfg.dim
    out = {}
    for p in pids:
        n = cfg.patch_cells[levels[p]]
        a = rng.uniform(-1.0, 1.0, (d + 2,) + (n,) * d)
        a[0] = rng.uniform(0.2, 2.0, a[0].shape)
        a[d + 1] = rng.uniform(0.2, 2.0, a[0].shape)
        out[p] = a
    return out


@pytest.mark.parametrize("d", [1, 2, 3])
def test_noalloc_upload_equals_allocating_upload(d, amr):
    cfg, (h1, h2), levels = _pair(amr, d, {1: 256, 2: 64, 3: 32}[d])
    rng = np.random.default_rng(7 + d)
    pids = sorted(levels)
    print(f"no-alloc upload: d={d}, {len(pids)} patches", flush=True)
    first = _prims(rng, cfg, pids, levels)
    h1.set_state_prim(0, first)
    h2.set_state_prim_noalloc(0, first)
    a, b = h1.get_state(0, pids, levels), h2.get_state(0, pids, levels)
    for p in pids:
        assert np.array_equal(a[p], b[p]), p
    # second call: a smaller, shuffled subset with new values
    sub = [int(p) for p in rng.permutation(pids)[: max(1, len(pids) // 3)]]
    second = _prims(rng, cfg, sub, levels)
    h1.set_state_prim(0, second)
    h2.set_state_prim_noalloc(0, second)
    a, b = h1.get_state(0, pids, levels), h2.get_state(0, pids, levels)
    for p in pids:
        assert np.array_equal(a[p], b[p]), p
    # and the conversion itself: interior of a re-uploaded patch
    g = cfg.gamma
    p = sub[0]
    pr = second[p]
    inner = b[p][(slice(None),) + (slice(4, -4),) * d]
    assert np.array_equal(inner[0], pr[0])
    assert np.array_equal(inner[1], pr[0] * pr[1])
    h1.close()
    h2.close()


def test_noalloc_upload_refuses_more_than_its_scratch(amr):
    cfg = W.AMRConfig(name="na", dim=3, base_cells=128, patch_cells=[32],
                      periodic=[True] * 3, max_patches=128)
    h = amr.Hierarchy(cfg)
    table = h.patch_table()
    levels = {t["pid"]: 0 for t in table}
    per = 5 * 32 ** 3 * 8
    npat = amr.NOALLOC_SCRATCH_BYTES // per + 1          # one patch too many
    assert npat <= len(table)
    prims = {t["pid"]: np.ones((5, 32, 32, 32)) for t in table[:npat]}
    before = h.get_state(0, list(prims), levels)
    with pytest.raises(amr.AMRError) as e:
        h.set_state_prim_noalloc(0, prims)
    assert e.value.status == -1 and "scratch" in str(e.value)
    after = h.get_state(0, list(prims), levels)
    for p in prims:
        assert np.array_equal(before[p], after[p])
    # a call that fits still works on the same hierarchy
    fit = dict(list(prims.items())[: npat - 1])
    h.set_state_prim_noalloc(0, fit)
    got = h.get_state(0, list(fit), levels)
    for p in fit:
        assert np.array_equal(got[p][(slice(None),) + (slice(4, -4),) * 3][0], fit[p][0])
    h.close()
