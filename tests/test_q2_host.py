"""Host logic of the library's cG(2) numbering (no GPU needed): the 27 node
refs per leaf, the node and hanging-node coordinates and the quadratic
constraint rows and the wall / pressure-pin flags equal the oracle's, bit for
bit, on adaptive meshes with 2:1 faces and edges."""
import numpy as np
import pytest

import oracle
from paper_1912_12453_amd import chns
from paper_1912_12453_amd import workloads as W

CASES = [("random", (1, 1, 1), 2, 4, 7), ("random", (1, 1, 1), 1, 4, 11), ("random", (1, 1, 1), 2, 5, 5),
         ("random", (2, 1, 1), 1, 4, 3), ("drop", (1, 1, 1), 2, 5, 0), ("rt", (1, 1, 4), 2, 4, 0)]


def meshes(kind, trees, lmin, lmax, seed):
    if kind == "random":
        leaves = W.random_leaves(trees, lmax, seed, p_split=0.35, level_min=lmin)
        return (chns.Mesh(trees, 0, lmax, leaves=leaves), oracle.Mesh(trees, 0, lmax, leaves=leaves))
    if kind == "drop":
        phi0 = W.drops_phi([(np.array([0.4, 0.45, 0.5]), 0.2)], 0.05, -1.0)
    else:
        phi0 = W.rt(level_max=lmax).mesh.phi0
    return (chns.Mesh(trees, lmin, lmax, phi0, 0.9), oracle.Mesh(trees, lmin, lmax, phi0, 0.9))


@pytest.mark.parametrize("kind,trees,lmin,lmax,seed", CASES)
def test_q2_numbering_matches_oracle(kind, trees, lmin, lmax, seed):
    pm, om = meshes(kind, trees, lmin, lmax, seed)
    assert pm.n_leaves == om.n_leaves
    a = pm.q2_arrays()
    q = om.q2()
    np.testing.assert_array_equal(a["elem"], q.elem)
    np.testing.assert_array_equal(a["nodes"], q.node_xyz())
    np.testing.assert_array_equal(a["hang_xyz"], q.hang_coords())
    np.testing.assert_array_equal(a["hang_off"], q.hang_off)
    np.testing.assert_array_equal(a["hang_ids"], q.hang_ids)
    np.testing.assert_array_equal(a["hang_w"], q.hang_w)
    np.testing.assert_array_equal(a["bflags"], q.bflags)
    if kind != "rt":
        assert a["hang_xyz"].shape[0] > 0
