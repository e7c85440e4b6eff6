"""Host logic of libchns (no GPU needed): the product mesh builder against the
oracle mesh and the brute-force reference, bit for bit, and the C ABI's
exported symbols against include/chns.h."""
import ctypes
import os
import re

import numpy as np
import pytest

from paper_1912_12453_amd import chns
from paper_1912_12453_amd import workloads as W
from tests import bruteforce_mesh as BF

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_library_exports_every_declared_symbol():
    L = chns.lib()
    header = open(os.path.join(ROOT, "include", "chns.h")).read()
    names = set(re.findall(r"\b(chns_[a-z_0-9]+)\s*\(", header))
    assert len(names) >= 12
    for name in sorted(names):
        assert hasattr(L, name), name
        assert isinstance(getattr(L, name), ctypes._CFuncPtr)


def same_mesh(pm, om):
    a = pm.arrays()
    np.testing.assert_array_equal(a["leaves"], om.leaves)
    np.testing.assert_array_equal(a["elem"], om.elem)
    np.testing.assert_array_equal(a["nodes"], om.nodes)
    np.testing.assert_array_equal(a["bflags"], om.bflags)
    np.testing.assert_array_equal(a["hang_xyz"], om.hang_xyz)
    np.testing.assert_array_equal(a["hang_off"], om.hang_off)
    np.testing.assert_array_equal(a["hang_ids"], om.hang_ids)
    np.testing.assert_array_equal(a["hang_w"], om.hang_w)


@pytest.mark.parametrize("seed,trees,D,p", [
    (0, (1, 1, 1), 3, 0.5), (1, (1, 1, 1), 4, 0.35), (2, (2, 1, 1), 3, 0.45),
    (3, (1, 1, 2), 3, 0.5), (4, (1, 1, 1), 5, 0.25), (5, (1, 2, 1), 3, 0.6),
    (6, (3, 2, 1), 3, 0.4), (7, (1, 1, 4), 4, 0.3),
])
def test_random_trees_match_oracle(orc, seed, trees, D, p):
    leaves = W.random_leaves(trees, D, seed, p_split=p, level_min=1)
    pm = chns.Mesh(trees, 0, D, leaves=leaves)
    om = orc.Mesh(trees, 0, D, leaves=leaves)
    same_mesh(pm, om)


def test_tiny_tree_matches_bruteforce():
    leaves = W.random_leaves((1, 1, 1), 3, 42, p_split=0.5, level_min=1)
    pm = chns.Mesh((1, 1, 1), 0, 3, leaves=leaves)
    ref = BF.build(leaves, 3)
    a = pm.arrays()
    assert [tuple(r) for r in a["leaves"].tolist()] == ref["leaves"]
    assert [tuple(r) for r in a["nodes"].tolist()] == ref["nodes"]
    assert a["elem"].tolist() == ref["elem"]


@pytest.mark.parametrize("wl", ["drop8", "bubble6", "rt5", "serving"])
def test_refined_workload_meshes_match_oracle(orc, wl):
    if wl == "drop8":
        w = W.drop16(level=3)
    elif wl == "bubble6":
        w = W.bubble(level_max=6, level_min=3)
    elif wl == "rt5":
        w = W.rt(level_max=5, level_min=2)
    else:
        w = W.serving_stream(n_requests=3, seed=4, level_range=(5, 6))[1].workload
    ms = w.mesh
    pm = chns.Mesh.from_spec(ms)
    om = orc.Mesh(ms.trees, ms.level_min, ms.level_max, ms.phi0, ms.band)
    same_mesh(pm, om)
    assert pm.n_leaves == om.n_leaves


@pytest.mark.slow
def test_bubble_level8_matches_oracle(orc):
    w = W.bubble(level_max=8, level_min=4)
    pm = chns.Mesh.from_spec(w.mesh)
    om = orc.Mesh(w.mesh.trees, w.mesh.level_min, w.mesh.level_max, w.mesh.phi0, w.mesh.band)
    same_mesh(pm, om)
    assert pm.stats.n_hanging > 1000


def test_mesh_errors():
    with pytest.raises(chns.ChnsError):
        chns.Mesh((1, 1, 1), 0, 2, leaves=np.array([[0, 0, 0, 1]], np.int32))
    with pytest.raises(chns.ChnsError):
        chns.Mesh((1, 1, 1), 3, 2)
    with pytest.raises(chns.ChnsError):
        chns.Mesh((0, 1, 1), 0, 2)
