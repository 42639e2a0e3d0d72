"""C-ABI checks that need no GPU: the library loads, exports every function
include/amr.h declares, rejects invalid configurations before touching the
device, and its host-side mesh adaptation (Algorithms 1-2) reproduces the
oracle's meshes for the same request sequences."""
import os
import random
import re
import subprocess

import pytest

from paper_2508_05020_amd import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "amr.h")


def _lib():
    import paper_2508_05020_amd.amr as A
    return A


def test_header_functions_exported():
    A = _lib()
    names = set(re.findall(r"\b(amr_\w+)\s*\(", open(HEADER).read()))
    assert len(names) >= 20
    out = subprocess.run(["nm", "-D", "--defined-only", A.LIB_PATH], capture_output=True,
                         text=True, check=True).stdout
    syms = {line.split()[-1] for line in out.splitlines() if line.strip()}
    missing = sorted(n for n in names if n not in syms)
    assert not missing, missing
    # the binding covers exactly the declared functions
    assert set(A.EXPORTED) == names


@pytest.mark.parametrize("field,value", [("dim", 4), ("max_levels", 0), ("gamma", 1.0),
                                         ("cfl", 0.0), ("tag_buffer", 4), ("max_patches", 0)])
def test_invalid_config_rejected_without_device(field, value):
    import ctypes as C
    A = _lib()
    cfg = W.config("c1")
    c = A.make_config(cfg)
    setattr(c, field, value)
    h = C.c_void_p()
    st = A._lib.amr_create_hierarchy(C.byref(c), None, None, C.byref(h))
    assert st == -1
    assert A._lib.amr_last_error(h)
    A._lib.amr_destroy_hierarchy(h)


def test_patch_size_rules_rejected():
    import ctypes as C
    A = _lib()
    cfg = W.AMRConfig(name="x", dim=2, base_cells=64, patch_cells=[32, 12], periodic=[True, True])
    c = A.make_config(cfg)
    h = C.c_void_p()
    assert A._lib.amr_create_hierarchy(C.byref(c), None, None, C.byref(h)) == -1
    A._lib.amr_destroy_hierarchy(h)


def _random_rounds(cfg, seed, nround=8, coarsen_every=2, rule="text"):
    from oracle.mesh import Forest
    f = Forest(cfg, coarsen_rule=rule)
    rnd = random.Random(seed)
    rounds = []
    for it in range(nround):
        leaves = [k for k in f.leaves() if k[0] < cfg.max_levels - 1]
        ref = rnd.sample(leaves, max(1, len(leaves) // 5)) if leaves else []
        nonleaf = [k for k in f.keys() if not f.is_leaf(k)]
        coa = rnd.sample(nonleaf, len(nonleaf) // 2) if (it % coarsen_every == 1) else []
        f.regrid(ref, coa)
        f.validate()
        rounds.append((ref, coa))
    return f, rounds


@pytest.mark.parametrize("case", [
    dict(dim=1, base_cells=128, patch_cells=[8, 8, 8, 8], periodic=[False]),
    dict(dim=2, base_cells=64, patch_cells=[16, 16, 16, 16], periodic=[True, True]),
    dict(dim=2, base_cells=64, patch_cells=[32, 16, 16], periodic=[False, True]),
    dict(dim=3, base_cells=32, patch_cells=[16, 16, 8], periodic=[True, True, True]),
    dict(dim=3, base_cells=32, patch_cells=[8, 8, 8], periodic=[False, True, False]),
])
@pytest.mark.parametrize("rule", ["text", "literal"])
def test_forest_replay_matches_oracle(case, rule):
    A = _lib()
    cfg = W.AMRConfig(name="m", max_patches=200000, **case)
    for seed in range(3):
        f, rounds = _random_rounds(cfg, seed, rule=rule)
        lib = A.forest_replay(cfg, rounds,
                              coarsen_rule=A.COARSEN_LITERAL if rule == "literal" else A.COARSEN_TEXT)
        mine = sorted((k[0], k[1], len(f.children[k])) for k in f.keys())
        theirs = sorted((r[0], r[1], r[3]) for r in lib)
        assert mine == theirs


def test_forest_replay_capacity_error():
    A = _lib()
    cfg = W.AMRConfig(name="m", dim=2, base_cells=64, patch_cells=[16, 16], periodic=[True, True],
                      max_patches=16 + 8)
    with pytest.raises(A.AMRError) as e:
        A.forest_replay(cfg, [([(0, (0, 0)), (0, (2, 2)), (0, (0, 2))], [])])
    assert e.value.status == -2


@pytest.mark.parametrize("dim,base,nrefine,small_cap", [(1, 65536, 300, 6000),
                                                      (2, 1024, 300, 9000),
                                                      (3, 256, 80, 20000)])
def test_forest_replay_order_large(dim, base, nrefine, small_cap):
    """Active patches come out in (level, z, y, x) order from both host
    paths: the level-map scan (capacity large against the maps) and the
    packed-key radix sort (capacity small against the maps, >= 4096 keys)."""
    A = _lib()
    rnd = random.Random(dim)
    np0 = base // 16
    coords = [tuple(rnd.randrange(np0) for _ in range(dim)) for _ in range(nrefine)]
    nsub, c0 = nrefine * 2 // 5, nrefine * 2 // 3
    rounds = [([(0, c) for c in coords], []),
              ([(1, tuple(2 * x + rnd.randrange(2) for x in c)) for c in coords[:nsub]], []),
              ([], [(0, c) for c in coords[c0:c0 + nrefine // 5]])]
    outs = []
    for mp in (small_cap, 400000):
        cfg = W.AMRConfig(name="m", dim=dim, base_cells=base, patch_cells=[16, 16, 16],
                          periodic=[True] * dim, max_patches=mp)
        outs.append([(r[0], r[1], r[3]) for r in A.forest_replay(cfg, rounds)])
    assert len(outs[0]) > 4096
    assert outs[0] == outs[1]
    assert outs[0] == sorted(outs[0], key=lambda r: (r[0], r[1][::-1]))
