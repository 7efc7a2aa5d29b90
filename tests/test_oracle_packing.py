"""Pins of the oracle's particle-in-kernel contact detection and packing step (supplementary
material, particle-in-kernel technique; main text, near-contact handling and cell packing)
against closed forms, an independent library search and the physics of the packing run."""
import numpy as np
import pytest
import scipy.spatial

import npfem_inputs as I
import oracle as O


def _types(meshes, mat=I.PLT_MATERIAL):
    return {k: O.CellType(x, t, mat, I.DT) for k, (x, t) in meshes.items()}


def test_vertex_normals_of_regular_polyhedra_are_radial():
    """Vertices of the octahedron and icosahedron lie on the unit sphere and every vertex
    star is symmetric, so the outward normal is x / |x|; a rigid motion rotates it."""
    rng = np.random.default_rng(3)
    for fn in (I.octahedron, I.icosahedron):
        x, t = fn()
        n = O.vertex_normals(x[None], t)[0]
        assert np.abs(n - x / np.linalg.norm(x, axis=1, keepdims=True)).max() < 1e-14
        R = I.random_rotations(rng, 1)[0]
        nr = O.vertex_normals((x @ R.T + [5.0, -2.0, 1.0])[None], t)[0]
        assert np.abs(nr - n @ R.T).max() < 1e-13


def test_closest_foreign_vertex_matches_a_kd_tree():
    """Platelets overlapping in a small box: for every vertex, scipy's KD-tree over the other
    cells' vertices (nearest neighbour within the radius) gives the same neighbour."""
    tids = np.array([I.PLT] * 7, dtype=np.int32)
    b = I.make_batch(tids, seed=21, translate=4.0)
    cell_of = np.repeat(np.arange(b.n_cells), np.diff(b.offsets))
    r = 0.6
    got = O.closest_foreign_vertex(b.x0, cell_of, r, np.float64)
    want = np.full(b.v_total, -1)
    pts = b.x0.T
    for c in range(b.n_cells):
        others = np.nonzero(cell_of != c)[0]
        tree = scipy.spatial.cKDTree(pts[others])
        d, k = tree.query(pts[cell_of == c], distance_upper_bound=r)
        hit = np.isfinite(d)
        want[np.nonzero(cell_of == c)[0][hit]] = others[k[hit]]
    assert (want >= 0).mean() > 0.2           # the box packs the cells: many contacts
    assert np.array_equal(got, want)


def test_equal_distances_pick_the_smallest_index_and_own_cell_is_ignored():
    x = np.array([[0.0, 0.5, -0.5, 0.1, 0.5],
                  [0.0, 0.0, 0.0, 0.0, 0.0],
                  [0.0, 0.0, 0.0, 0.0, 0.0]])
    cell_of = np.array([0, 2, 1, 0, 3])
    j = O.closest_foreign_vertex(x, cell_of, 1.0, np.float32)
    # vertex 0: own-cell vertex 3 at 0.1 is ignored; 1, 2 and 4 are foreign, 1 and 4 tie at
    # 0.5 with 2 -> the smallest index, 1
    assert j[0] == 1
    # the radius is strict: nothing at distance exactly 0.5 with radius 0.5
    assert O.closest_foreign_vertex(x, cell_of, 0.5, np.float32)[0] == -1


def test_projection_points_of_two_octahedra_closed_form():
    """Unit octahedra at the origin and at (1.5, 0, 0): only the facing apices (1, 0, 0) and
    (0.5, 0, 0) are within 0.8 of a foreign vertex; each is projected to the other's apex
    plus the separation along that apex's outward normal (-x and +x)."""
    x, t = I.octahedron()
    ot = _types({0: (x, t)})
    X = np.concatenate([x.T, (x + [1.5, 0.0, 0.0]).T], axis=1)
    offsets = np.array([0, 6, 12])
    p, w, j = O.pik_contacts(ot, [0, 0], offsets, X, 0.8, 0.3, 7.0)
    a, bb = 1, 6 + 3                       # A's (1,0,0) and B's local (-1,0,0) = (0.5,0,0)
    assert j[a] == bb and j[bb] == a
    assert np.allclose(p[:, a], [0.5 - 0.3, 0.0, 0.0], atol=1e-15)
    assert np.allclose(p[:, bb], [1.0 + 0.3, 0.0, 0.0], atol=1e-15)
    assert w[a] == 7.0 and w[bb] == 7.0
    rest = np.setdiff1d(np.arange(12), [a, bb])
    assert np.all(w[rest] == 0.0) and np.all(j[rest] == -1)
    assert np.array_equal(p[:, rest], X[:, rest])


@pytest.mark.parametrize("dtype", [np.float32, np.float64])
def test_packing_separates_two_overlapping_platelets(dtype):
    """Two platelets interpenetrating by 40 % of their thickness, at rest and without external
    force: the packing steps push them apart until no vertex has a foreign vertex within the
    kernel."""
    inp = I.cell_type_inputs()
    xp, tp, mp = inp[I.PLT]
    ot = {I.PLT: O.CellType(xp, tp, mp, I.DT)}
    P = I.PACKING
    thick = np.ptp(xp[:, 2])
    X = np.concatenate([xp.T, (xp + [0.3, 0.2, 0.6 * thick]).T], axis=1)
    X = X.astype(np.float32).astype(np.float64)
    offsets = np.array([0, xp.shape[0], 2 * xp.shape[0]])
    types = [I.PLT, I.PLT]
    v = np.zeros_like(X)
    _, w0, _ = O.pik_contacts(ot, types, offsets, X, P["radius"], P["separation"], P["weight"], dtype)
    counts = [(w0 > 0).sum()]
    for _ in range(80):
        X, v, w = O.packing_step(ot, types, offsets, X, v, P["n_pd_iters"], P["radius"],
                                 P["separation"], P["weight"], dtype)
        X = X.astype(dtype).astype(np.float64)
        v = v.astype(dtype).astype(np.float64)
        counts.append((w > 0).sum())
        if counts[-1] == 0:
            break
    assert counts[0] > 20 and counts[-1] == 0, counts
    cz = [X[2, :66].mean(), X[2, 66:].mean()]
    assert cz[1] - cz[0] > 0.6 * thick           # moved apart along the overlap axis
    assert np.all(np.isfinite(X))
    print("contacting vertices per step:", counts)
