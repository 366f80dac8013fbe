"""The synthetic box meshes themselves: box_mesh on a cube is cartesian_mesh,
and on any box every lattice vertex is used by exactly the elements whose
closed boxes contain it."""
import numpy as np
import pytest

import meshgen


@pytest.mark.parametrize("n,p", [(1, 1), (2, 3), (3, 2)])
def test_box_mesh_on_a_cube_is_cartesian_mesh(n, p):
    a, b = meshgen.cartesian_mesh(n, p, 0.1), meshgen.box_mesh(n, n, n, p, 0.1)
    assert np.array_equal(a["elem_dofs"], b["elem_dofs"])
    assert np.array_equal(a["coords"], b["coords"])
    assert a["ndofs"] == b["ndofs"] and a["nel"] == b["nel"]


@pytest.mark.parametrize("box,p", [((3, 2, 1), 2), ((1, 1, 4), 3), ((2, 3, 2), 1)])
def test_box_mesh_incidence(box, p):
    m = meshgen.box_mesh(*box, p)
    L = [n * p + 1 for n in box]
    counts = np.bincount(m["elem_dofs"].reshape(-1), minlength=m["ndofs"])
    v = np.arange(m["ndofs"])
    X, Y, Z = v % L[0], (v // L[0]) % L[1], v // (L[0] * L[1])

    def per_axis(c, n):
        # a point on an interior element face along this axis lies in two elements
        return np.where((c % p == 0) & (c > 0) & (c < n * p), 2, 1)

    assert np.array_equal(counts, per_axis(X, box[0]) * per_axis(Y, box[1]) * per_axis(Z, box[2]))
    # the perturbed lattice keeps the box corners where they were
    assert np.allclose(m["coords"][0], 0.0)
    assert np.allclose(m["coords"][-1], np.array(box) / max(box))


@pytest.mark.parametrize("n,p", [(1, 1), (3, 2), (2, 5)])
def test_box_mesh_2d_on_a_square_is_cartesian_mesh_2d(n, p):
    a, b = meshgen.cartesian_mesh_2d(n, p, 0.1), meshgen.box_mesh_2d(n, n, p, 0.1)
    assert np.array_equal(a["elem_dofs"], b["elem_dofs"])
    assert np.array_equal(a["coords"], b["coords"])
    assert a["ndofs"] == b["ndofs"] and a["nel"] == b["nel"]


@pytest.mark.parametrize("box,p", [((3, 2), 2), ((1, 4), 3), ((5, 2), 1)])
def test_box_mesh_2d_incidence(box, p):
    m = meshgen.box_mesh_2d(*box, p)
    L = [n * p + 1 for n in box]
    counts = np.bincount(m["elem_dofs"].reshape(-1), minlength=m["ndofs"])
    v = np.arange(m["ndofs"])
    X, Y = v % L[0], v // L[0]

    def per_axis(c, n):
        return np.where((c % p == 0) & (c > 0) & (c < n * p), 2, 1)

    assert np.array_equal(counts, per_axis(X, box[0]) * per_axis(Y, box[1]))
    # local vertex i + (p+1) j of element (ex, ey) is lattice point (p ex + i, p ey + j)
    e = box[0] + 0 if box[1] > 1 else 0
    ex, ey = e % box[0], e // box[0]
    q = p + 1
    for l in range(q * q):
        assert m["elem_dofs"][e][l] == (p * ex + l % q) + L[0] * (p * ey + l // q)
    assert np.allclose(m["coords"][0], 0.0)
    assert np.allclose(m["coords"][-1], np.array(box) / max(box))


@pytest.mark.parametrize("n,p", [(1, 2), (2, 3), (3, 1)])
def test_face_map_box_on_a_cube_is_face_map(n, p):
    a, na = meshgen.face_map(n, p)
    b, nb = meshgen.face_map_box(n, n, n, p)
    assert na == nb and np.array_equal(a, b)


@pytest.mark.parametrize("box,p", [((3, 2, 1), 2), ((1, 2, 3), 1)])
def test_face_map_box_matches_vertices(box, p):
    """Every face once per macro element holding it (2 on the faces between
    two elements, 1 elsewhere), and the same faces as derived from the vertex
    map alone."""
    m = meshgen.box_mesh(*box, p)
    fm, nf = meshgen.face_map_box(*box, p)
    counts = np.bincount(fm.reshape(-1), minlength=nf)
    M = [n * p for n in box]
    nshared = (box[0] - 1) * M[1] * M[2] + (box[1] - 1) * M[0] * M[2] + (box[2] - 1) * M[0] * M[1]
    assert nf == (M[0] + 1) * M[1] * M[2] + M[0] * (M[1] + 1) * M[2] + M[0] * M[1] * (M[2] + 1)
    assert np.sort(counts).tolist() == [1] * (nf - nshared) + [2] * nshared
    fv, nfv = meshgen.face_map_from_vertices(m["elem_dofs"], p)
    assert nfv == nf
    # the two numberings differ by a relabelling of the faces: the same
    # partition of (element, local face) slots into faces
    pairs = {}
    for a, b in zip(np.abs(fm).reshape(-1).tolist(), (np.where(fv < 0, -1 - fv, fv)).reshape(-1).tolist()):
        assert pairs.setdefault(a, b) == b
    assert len(set(pairs.values())) == nf


@pytest.mark.parametrize("n,p", [(1, 2), (2, 3), (3, 1)])
def test_nd_edge_map_box_on_a_cube_is_nd_edge_map(n, p):
    a, na = meshgen.nd_edge_map(n, p)
    b, nb = meshgen.nd_edge_map_box(n, n, n, p)
    assert na == nb and np.array_equal(a, b)


@pytest.mark.parametrize("box,p", [((3, 2, 1), 2), ((1, 2, 3), 1), ((2, 1, 2), 3)])
def test_nd_edge_map_box_matches_vertices(box, p):
    """The edge count of the box's lattice, every edge along its axis (no
    reversed entries), and the same edges as derived from the vertex map
    alone: the same partition of (element, local edge) slots into edges, and
    the same orientation (box vertex ids grow along every axis)."""
    m = meshgen.box_mesh(*box, p)
    em, ne = meshgen.nd_edge_map_box(*box, p)
    M = [n * p for n in box]
    assert ne == M[0] * (M[1] + 1) * (M[2] + 1) + (M[0] + 1) * M[1] * (M[2] + 1) + (M[0] + 1) * (M[1] + 1) * M[2]
    assert em.min() >= 0 and set(np.unique(em).tolist()) == set(range(ne))
    ev, nev = meshgen.edge_map_from_vertices(m["elem_dofs"], p)
    assert nev == ne and ev.min() >= 0
    pairs = {}
    for a, b in zip(em.reshape(-1).tolist(), ev.reshape(-1).tolist()):
        assert pairs.setdefault(a, b) == b
    assert len(set(pairs.values())) == ne
