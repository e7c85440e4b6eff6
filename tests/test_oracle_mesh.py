"""Pins of the oracle's octree mesh (Sec. 4) against closed forms and a
brute-force geometric reference on tiny trees."""
from fractions import Fraction

import numpy as np
import pytest

from paper_1912_12453_amd import workloads as W
from tests import bruteforce_mesh as BF


def _mesh_dict(m):
    cons = {}
    for h in range(m.hang_xyz.shape[0]):
        a, b = m.hang_off[h], m.hang_off[h + 1]
        cons[h] = [(int(i), Fraction(float(w))) for i, w in zip(m.hang_ids[a:b], m.hang_w[a:b])]
    return {
        "leaves": [tuple(int(v) for v in r) for r in m.leaves],
        "nodes": [tuple(int(v) for v in r) for r in m.nodes],
        "hanging": [tuple(int(v) for v in r) for r in m.hang_xyz],
        "constraints": cons,
        "elem": [[int(v) for v in r] for r in m.elem],
    }


@pytest.mark.parametrize("level", [0, 1, 2, 3, 4])
def test_uniform_counts(orc, level):
    m = orc.Mesh((1, 1, 1), level, level)
    assert m.n_leaves == 8 ** level
    assert m.n_nodes == (2 ** level + 1) ** 3
    assert m.hang_xyz.shape[0] == 0
    # boundary nodes: all but the interior lattice
    assert int((m.bflags & 1).sum()) == (2 ** level + 1) ** 3 - max(2 ** level - 1, 0) ** 3
    assert m.bflags[0] & 2 and (m.bflags[1:] & 2).sum() == 0


def test_brick_counts(orc):
    m = orc.Mesh((1, 1, 4), 2, 2)
    assert m.n_leaves == 4 * 64
    assert m.n_nodes == 5 * 5 * 17


def test_config_drop16_counts(orc):
    w = W.drop16()
    m = orc.Mesh(w.mesh.trees, w.mesh.level_min, w.mesh.level_max)
    assert (m.n_leaves, m.n_nodes) == (4096, 4913)


@pytest.mark.parametrize("seed,trees,D,p", [
    (0, (1, 1, 1), 3, 0.5), (1, (1, 1, 1), 4, 0.35), (2, (2, 1, 1), 3, 0.45),
    (3, (1, 1, 2), 3, 0.5), (4, (1, 1, 1), 4, 0.3), (5, (1, 2, 1), 3, 0.6),
])
def test_bruteforce_random_trees(orc, seed, trees, D, p):
    leaves = W.random_leaves(trees, D, seed, p_split=p, level_min=1)
    m = orc.Mesh(trees, 0, D, leaves=leaves)
    ref = BF.build(leaves, D)
    got = _mesh_dict(m)
    assert got["leaves"] == ref["leaves"]
    assert got["nodes"] == ref["nodes"]
    assert got["hanging"] == ref["hanging"]
    assert got["elem"] == ref["elem"]
    assert got["constraints"] == ref["constraints"]
    assert len(ref["hanging"]) > 0


def test_balance_is_idempotent_and_ordered(orc):
    leaves = W.random_leaves((1, 1, 1), 5, 11, p_split=0.3)
    m = orc.Mesh((1, 1, 1), 0, 5, leaves=leaves)
    m2 = orc.Mesh((1, 1, 1), 0, 5, leaves=m.leaves)
    assert np.array_equal(m.leaves, m2.leaves)
    keys = [BF.morton(*map(int, r[:3])) for r in m.leaves]
    assert keys == sorted(keys) and len(set(keys)) == len(keys)
    nk = [BF.morton(*map(int, r)) for r in m.nodes]
    assert nk == sorted(nk)


def test_continuity_of_constrained_space(orc):
    """The constraints make the trilinear space continuous: every leaf whose
    closure contains a corner, edge midpoint or face centre of another leaf
    interpolates the same value there."""
    leaves = W.random_leaves((1, 1, 1), 4, 21, p_split=0.35, level_min=1)
    m = orc.Mesh((1, 1, 1), 0, 4, leaves=leaves)
    assert m.hang_xyz.shape[0] > 0
    D = m.level_max
    rng = np.random.default_rng(0)
    u = rng.normal(size=m.n_nodes)
    hv = np.zeros(m.hang_xyz.shape[0])
    for h in range(len(hv)):
        a, b = m.hang_off[h], m.hang_off[h + 1]
        hv[h] = (m.hang_w[a:b] * u[m.hang_ids[a:b]]).sum()
    cv = np.where(m.elem >= 0, u[np.maximum(m.elem, 0)], hv[np.maximum(-1 - m.elem, 0)])

    def interp(e, P):
        x, y, z, l = (int(v) for v in m.leaves[e])
        s = 1 << (D - l)
        t = [(P[0] - x) / s, (P[1] - y) / s, (P[2] - z) / s]
        val = 0.0
        for c in range(8):
            w = 1.0
            for d in range(3):
                w *= t[d] if (c >> d) & 1 else 1 - t[d]
            val += w * cv[e, c]
        return val

    pts = set()
    for x, y, z, l in m.leaves:
        s = 1 << (D - int(l))
        for i in range(3):
            for j in range(3):
                for k in range(3):
                    pts.add((int(x) + i * s // 2, int(y) + j * s // 2, int(z) + k * s // 2))
    L = m.leaves.astype(np.int64)
    S = (1 << (D - L[:, 3]))
    checked = 0
    for P in pts:
        inside = np.all((L[:, :3] <= np.array(P)) & (np.array(P) <= L[:, :3] + S[:, None]), axis=1)
        vals = [interp(e, P) for e in np.nonzero(inside)[0]]
        assert max(vals) - min(vals) < 1e-12
        checked += len(vals) > 1
    assert checked > 100


def test_refinement_indicator_levels(orc):
    """Top-down refinement: leaves away from the interface stay at level_min;
    the leaf containing an interface point reaches level_max."""
    w = W.bubble(level_max=6, level_min=3)
    m = orc.Mesh(w.mesh.trees, w.mesh.level_min, w.mesh.level_max, w.mesh.phi0, w.mesh.band)
    assert m.leaves[:, 3].min() == 3 and m.leaves[:, 3].max() == 6
    D = m.level_max
    # a point on the bubble surface
    P = np.array([0.5 + 0.15, 0.3, 0.5]) * 2 ** D
    L = m.leaves.astype(np.int64)
    S = (1 << (D - L[:, 3]))
    inside = np.all((L[:, :3] <= P) & (P < L[:, :3] + S[:, None]), axis=1)
    assert L[inside, 3].max() == 6
    # a corner of the domain, far from the bubble
    inside0 = np.all(L[:, :3] == 0, axis=1)
    assert L[inside0, 3][0] == 3


def test_invalid_leaves_rejected(orc):
    with pytest.raises(ValueError):
        orc.Mesh((1, 1, 1), 0, 2, leaves=np.array([[0, 0, 0, 1]], np.int32))
    with pytest.raises(ValueError):
        orc.Mesh((1, 1, 1), 0, 2, leaves=np.array([[1, 0, 0, 2]] * 64, np.int32))


def _small_sphere(centre, r, eps):
    c = np.asarray(centre, float)

    def f(P):
        P = np.asarray(P, float)
        return np.tanh((np.linalg.norm(P - c, axis=-1) - r) / eps)
    return f


@pytest.mark.parametrize("centre,r,lmin,lmax,trees", [
    ((0.25, 0.25, 0.25), 0.05, 1, 4, (1, 1, 1)),      # seen first by a level-1 centre sample
    ((0.625, 0.375, 0.125), 0.03, 2, 5, (1, 1, 1)),   # by a level-2 centre sample
    ((1.25, 0.75, 0.25), 0.04, 1, 4, (2, 1, 1)),      # in the second tree of a brick
    ((0.3, 0.55, 0.7), 0.22, 1, 4, (1, 1, 1)),        # corners and centres both matter
])
def test_refinement_matches_bruteforce(orc, centre, r, lmin, lmax, trees):
    """The refinement rule (Sec. 4 "Refinement", reading A18) against a
    one-octant-at-a-time restatement followed by the brute-force balance.  The
    indicator is a sphere much smaller than the octants whose centre it sits
    at, so the split at those octants comes from the centre sample alone."""
    phi0 = _small_sphere(centre, r, 0.004)
    m = orc.Mesh(trees, lmin, lmax, phi0=lambda P: phi0(P), band=0.9)
    ref = BF.balance(BF.refine(trees, lmin, lmax, phi0, 0.9), lmax)
    assert [tuple(int(v) for v in L) for L in m.leaves] == ref
    assert max(L[3] for L in ref) == lmax
