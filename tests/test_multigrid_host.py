"""Host side of the octree multigrid hierarchy (chns_mesh_coarsen,
chns_mesh_transfer), checked against what the definitions fix: the coarse
tree is the fine tree with its finest sibling groups merged (and therefore
2:1 balanced), its nodes are fine nodes, and prolongation evaluates the
coarse trilinear field, so it reproduces every trilinear polynomial exactly
and forms a partition of unity."""
import numpy as np
import pytest

from paper_1912_12453_amd import chns
from paper_1912_12453_amd import workloads as W
from tests import bruteforce_mesh as BF


def trilinear(xyz):
    x, y, z = xyz[:, 0], xyz[:, 1], xyz[:, 2]
    return 1.0 + 2.0 * x - 3.0 * y + 0.5 * z + 1.25 * x * y - 0.75 * y * z + 0.5 * x * z + 0.25 * x * y * z


def make_mesh(name):
    if name == "random":
        return chns.Mesh(trees=(1, 1, 1), level_min=1, level_max=4,
                         leaves=W.random_leaves((1, 1, 1), 4, seed=3, p_split=0.45, level_min=1))
    if name == "brick":
        return chns.Mesh(trees=(2, 1, 1), level_min=1, level_max=3,
                         leaves=W.random_leaves((2, 1, 1), 3, seed=5, p_split=0.5, level_min=1))
    if name == "bubble6":
        return chns.Mesh.from_spec(W.bubble(level_max=6, level_min=3).mesh)
    return chns.Mesh(trees=(1, 1, 1), level_min=3, level_max=3)


@pytest.mark.parametrize("name", ["random", "brick", "bubble6", "uniform"])
def test_coarsening_and_transfer(name):
    fine = make_mesh(name)
    coarse = fine.coarsen()
    fa, ca = fine.arrays(), coarse.arrays()
    D = fine.level_max
    # coarse leaves = fine leaves with the finest sibling groups merged
    exp = set()
    for x, y, z, l in fa["leaves"]:
        if l == D:  # the parent, in units of the coarser grid
            exp.add(((x & ~1) >> 1, (y & ~1) >> 1, (z & ~1) >> 1, D - 1))
        else:
            exp.add((x >> 1, y >> 1, z >> 1, int(l)))
    got = {tuple(int(v) for v in r) for r in ca["leaves"]}
    assert got == exp
    # still 2:1 balanced (the brute-force balancer changes nothing)
    if coarse.n_leaves <= 4096:
        lv = [tuple(int(v) for v in r) for r in ca["leaves"]]
        assert sorted(BF.balance(lv, D - 1)) == sorted(lv)
    # coarse nodes are fine independent nodes; injection points at them
    p_off, p_idx, p_w, inj = fine.transfer(coarse)
    assert np.array_equal(fa["nodes"][inj], 2 * ca["nodes"])
    # P evaluates the coarse trilinear field: exact on trilinear polynomials
    xf, _ = fine.nodes()
    xc, _ = coarse.nodes()
    uc = trilinear(xc)
    uf = np.array([np.dot(p_w[p_off[i]:p_off[i + 1]], uc[p_idx[p_off[i]:p_off[i + 1]]])
                   for i in range(fine.n_nodes)])
    assert np.allclose(uf, trilinear(xf), rtol=0, atol=1e-13)
    # partition of unity, positive dyadic weights, sorted unique coarse ids
    sums = np.add.reduceat(p_w, p_off[:-1])
    assert np.array_equal(sums, np.ones(fine.n_nodes))
    assert (p_w > 0).all()
    assert np.all(np.mod(p_w * 2.0 ** 40, 1.0) == 0)  # dyadic
    for i in range(min(fine.n_nodes, 2000)):
        ids = p_idx[p_off[i]:p_off[i + 1]]
        assert (np.diff(ids) > 0).all()
    # at a coarse node the fine value is that node's value alone
    assert np.array_equal(p_off[inj + 1] - p_off[inj], np.ones(coarse.n_nodes, np.int32))
    assert np.array_equal(p_idx[p_off[inj]], np.arange(coarse.n_nodes))


def test_coarsening_reaches_uniform_and_stops():
    m = chns.Mesh(trees=(1, 1, 1), level_min=2, level_max=2)
    c = m.coarsen()
    assert c.level_max == 1 and c.n_leaves == 8
    c0 = c.coarsen()
    assert c0.n_leaves == 1
    with pytest.raises(chns.ChnsError):
        c0.coarsen()
