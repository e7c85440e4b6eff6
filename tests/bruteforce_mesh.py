"""Brute-force octree reference for tiny trees (pure Python, O(n^2)).

Restates the mesh definitions geometrically, with no neighbour search:
* 2:1 balance: repeatedly split any leaf whose closure touches the closure of
  a leaf more than one level finer, until no such pair remains;
* a leaf corner is hanging iff it lies in the closure of some leaf without
  being one of that leaf's vertices;
* a hanging corner's value is the trilinear interpolant, at the corner, of
  the corner values of the coarsest leaf in which it hangs (ties: smallest
  Morton anchor), with hanging corners of that leaf substituted recursively;
* independent and hanging nodes are each numbered in Morton order, x in the
  lowest bit of each bit triple.
"""
from fractions import Fraction


def morton(x, y, z, bits=24):
    k = 0
    for b in range(bits):
        k |= ((x >> b) & 1) << (3 * b)
        k |= ((y >> b) & 1) << (3 * b + 1)
        k |= ((z >> b) & 1) << (3 * b + 2)
    return k


def size(D, level):
    return 1 << (D - level)


def touches(a, b, D):
    sa, sb = size(D, a[3]), size(D, b[3])
    for d in range(3):
        if a[d] + sa < b[d] or b[d] + sb < a[d]:
            return False
    return True


def children(L, D):
    h = size(D, L[3] + 1)
    return [(L[0] + (h if c & 1 else 0), L[1] + (h if c & 2 else 0), L[2] + (h if c & 4 else 0),
             L[3] + 1) for c in range(8)]


def balance(leaves, D):
    leaves = [tuple(int(v) for v in L) for L in leaves]
    while True:
        bad = None
        for a in leaves:
            for b in leaves:
                if a[3] < b[3] - 1 and touches(a, b, D):
                    bad = a
                    break
            if bad:
                break
        if bad is None:
            return sorted(leaves, key=lambda L: morton(L[0], L[1], L[2]))
        leaves.remove(bad)
        leaves.extend(children(bad, D))


def corners(L, D):
    s = size(D, L[3])
    return [(L[0] + (s if c & 1 else 0), L[1] + (s if c & 2 else 0), L[2] + (s if c & 4 else 0))
            for c in range(8)]


def in_closure(P, L, D):
    s = size(D, L[3])
    return all(L[d] <= P[d] <= L[d] + s for d in range(3))


def is_vertex(P, L, D):
    s = size(D, L[3])
    return all(P[d] in (L[d], L[d] + s) for d in range(3))


def build(leaves, D):
    """Returns a dict with the balanced leaves, independent nodes, hanging nodes,
    constraints {hanging index: [(node id, Fraction weight)]}, and the element
    table (corner refs: id >= 0 node, -1-h hanging)."""
    L = balance(leaves, D)
    pts = set()
    for lf in L:
        pts.update(corners(lf, D))
    hang_owner = {}
    for P in pts:
        cands = [lf for lf in L if in_closure(P, lf, D) and not is_vertex(P, lf, D)]
        if cands:
            cands.sort(key=lambda lf: (lf[3], morton(lf[0], lf[1], lf[2])))
            hang_owner[P] = cands[0]
    indep = sorted([P for P in pts if P not in hang_owner], key=lambda P: morton(*P))
    hang = sorted(hang_owner, key=lambda P: morton(*P))
    nid = {P: i for i, P in enumerate(indep)}
    hid = {P: i for i, P in enumerate(hang)}

    memo = {}

    def value(P):
        if P in nid:
            return {nid[P]: Fraction(1)}
        if P in memo:
            return memo[P]
        lf = hang_owner[P]
        s = size(D, lf[3])
        acc = {}
        for c, Q in enumerate(corners(lf, D)):
            w = Fraction(1)
            for d in range(3):
                t = Fraction(P[d] - lf[d], s)
                w *= t if (c >> d) & 1 else (1 - t)
            if w == 0:
                continue
            for k, v in value(Q).items():
                acc[k] = acc.get(k, Fraction(0)) + w * v
        memo[P] = {k: v for k, v in acc.items() if v != 0}
        return memo[P]

    cons = {hid[P]: sorted(value(P).items()) for P in hang}
    elem = []
    for lf in L:
        row = []
        for Q in corners(lf, D):
            row.append(nid[Q] if Q in nid else -1 - hid[Q])
        elem.append(row)
    return {"leaves": L, "nodes": indep, "hanging": hang, "constraints": cons, "elem": elem}


def refine(trees, level_min, level_max, phi0, band):
    """Top-down refinement of a brick of unit trees (integer unit 2^-level_max),
    one octant at a time: an octant below level_max splits when it is below
    level_min, or when any of nine samples of phi0 (its 8 corners and its
    centre) has |phi0| < band, or the samples take both signs.  Returns the
    unbalanced leaves (x, y, z, level)."""
    D = level_max
    out = []
    stack = [(i << D, j << D, k << D, 0) for k in range(trees[2]) for j in range(trees[1])
             for i in range(trees[0])]
    unit = 2.0 ** -D
    while stack:
        L = stack.pop()
        l = L[3]
        if l == level_max:
            out.append(L)
            continue
        if l < level_min:
            split = True
        else:
            s = size(D, l)
            pts = [tuple(q * unit for q in P) for P in corners(L, D)]
            pts.append(tuple((L[d] + s // 2) * unit for d in range(3)))
            vals = [float(phi0(P)) for P in pts]
            split = (any(abs(v) < band for v in vals)
                     or (any(v > 0 for v in vals) and any(v < 0 for v in vals)))
        if split:
            stack.extend(children(L, D))
        else:
            out.append(L)
    return out
