"""Remeshing and intergrid transfer (host side: chns_mesh_remesh,
chns_mesh_interp_weights), checked against definitions: the transfer
evaluates the source mesh's trilinear field, so it is the identity onto the
same mesh and reproduces every trilinear polynomial between unrelated
meshes; the remeshed octree is the one the oracle's own mesh builder makes
when its refinement indicator is the old field, evaluated here by an
independent numpy routine on the oracle's mesh arrays."""
import numpy as np
import pytest

from paper_1912_12453_amd import chns
from paper_1912_12453_amd import workloads as W


def trilinear(xyz):
    x, y, z = xyz[:, 0], xyz[:, 1], xyz[:, 2]
    return 0.5 - x + 2.0 * y + 0.25 * z + 1.5 * x * y - 0.5 * x * z + 0.75 * y * z - 2.0 * x * y * z


def apply(off, idx, w, u):
    return np.array([np.dot(w[off[i]:off[i + 1]], u[idx[off[i]:off[i + 1]]]) for i in range(len(off) - 1)])


def test_transfer_onto_itself_is_identity():
    m = chns.Mesh((1, 1, 1), 0, 4, leaves=W.random_leaves((1, 1, 1), 4, 11, p_split=0.4, level_min=1))
    off, idx, w = m.interp_weights(m)
    assert np.array_equal(off, np.arange(m.n_nodes + 1))
    assert np.array_equal(idx, np.arange(m.n_nodes))
    assert np.array_equal(w, np.ones(m.n_nodes))


@pytest.mark.parametrize("trees,seeds", [((1, 1, 1), (3, 4)), ((1, 2, 1), (5, 6)), ((2, 1, 1), (7, 8))])
def test_transfer_between_unrelated_meshes(trees, seeds):
    a = chns.Mesh(trees, 0, 4, leaves=W.random_leaves(trees, 4, seeds[0], p_split=0.45, level_min=1))
    b = chns.Mesh(trees, 0, 3, leaves=W.random_leaves(trees, 3, seeds[1], p_split=0.5, level_min=1))
    for src, dst in ((a, b), (b, a)):
        off, idx, w = src.interp_weights(dst)
        xs, _ = src.nodes()
        xd, _ = dst.nodes()
        assert np.allclose(apply(off, idx, w, trilinear(xs)), trilinear(xd), rtol=0, atol=1e-13)
        assert np.array_equal(np.add.reduceat(w, off[:-1]), np.ones(dst.n_nodes))
        assert (w > 0).all() and np.all(np.mod(w * 2.0 ** 40, 1.0) == 0)


def field_evaluator(om, phi):
    """The trilinear field of nodal values phi on oracle mesh om, at points:
    locate a leaf whose closed cube holds the point, weight its corners, and
    expand hanging corners through their constraints."""
    D = om.level_max
    leaves = om.leaves.astype(np.int64)
    side = (1 << (D - leaves[:, 3])).astype(np.int64)
    ext = np.array(om.trees, dtype=np.int64) << D

    def f(xyz):
        out = np.empty(len(xyz))
        for t, x in enumerate(xyz):
            s = x * 2.0 ** D
            q = np.clip(np.floor(s), 0, ext - 1).astype(np.int64)
            inside = np.all((leaves[:, :3] <= q) & (q < leaves[:, :3] + side[:, None]), axis=1)
            e = int(np.flatnonzero(inside)[0])
            xi = np.clip((s - leaves[e, :3]) / side[e], 0.0, 1.0)
            acc = {}
            for k in range(8):
                wk = ((xi[0] if k & 1 else 1 - xi[0]) * (xi[1] if k & 2 else 1 - xi[1]) *
                      (xi[2] if k & 4 else 1 - xi[2]))
                if wk == 0.0:
                    continue
                ref = int(om.elem[e, k])
                if ref >= 0:
                    acc[ref] = acc.get(ref, 0.0) + wk
                else:
                    h = -1 - ref
                    for j in range(int(om.hang_off[h]), int(om.hang_off[h + 1])):
                        i = int(om.hang_ids[j])
                        acc[i] = acc.get(i, 0.0) + wk * float(om.hang_w[j])
            v = 0.0
            for i in sorted(acc):
                v += acc[i] * float(phi[i])
            out[t] = v
        return out
    return f


def test_remesh_matches_oracle_builder_on_the_old_field(orc):
    w = W.bubble(level_max=5, level_min=2)
    ms = w.mesh
    old_o = orc.Mesh(ms.trees, ms.level_min, ms.level_max, ms.phi0, ms.band)
    old_p = chns.Mesh.from_spec(ms)
    # the bubble has moved up by 0.1: phi at the old nodes
    moved = W.sphere_phi((0.5, 0.4, 0.5), 0.15, 0.02, inside=-1.0)
    phi = moved(old_o.node_xyz())
    U = np.zeros((old_p.n_nodes, 6))
    U[:, 0] = phi
    new_p = old_p.remesh(U, 2, 5, 0.9)
    new_o = orc.Mesh(ms.trees, 2, 5, field_evaluator(old_o, phi), 0.9)
    a = new_p.arrays()
    assert np.array_equal(a["leaves"], new_o.leaves)
    assert np.array_equal(a["elem"], new_o.elem)
    assert np.array_equal(a["nodes"], new_o.nodes)
    # the refined band follows the moved interface: it differs from the old mesh
    assert not np.array_equal(a["leaves"], old_o.leaves)


def test_remesh_to_the_same_criterion_keeps_the_mesh():
    """With phi the old mesh's own indicator sampled at its nodes and a
    uniform level, remeshing returns the same mesh."""
    m = chns.Mesh((1, 1, 1), 3, 3)
    U = np.zeros((m.n_nodes, 6))
    U[:, 0] = 1.0
    r = m.remesh(U, 3, 3, 0.9)
    assert np.array_equal(r.arrays()["leaves"], m.arrays()["leaves"])
