"""Seeded synthetic inputs for low-order-refined (LOR) assembly.

This module builds the *inputs* of the assembly only: node coordinates of the
Gauss-Lobatto-refined hexahedral mesh, the element-to-vertex and element-to-edge
maps, per-subelement coefficients and cotangents.  It contains none of the
assembly arithmetic (no shape functions, quadrature, Jacobians or sums), so both
the CPU oracle and the GPU path can take their inputs from here without sharing
any of the method's code.

Conventions (section "The low-order-refined mesh" of the paper: each degree-p
hexahedron is cut at the tensor Gauss-Lobatto lattice into p^3 subelements):

* Element e = ex + n*(ey + n*ez) of an n x n x n Cartesian coarse mesh of the
  unit cube.  Local vertex l = i + (p+1)*(j + (p+1)*k), i,j,k in [0, p].
* Global lattice has N = n*p + 1 points per axis; global vertex id
  X + N*(Y + N*Z) with X = p*ex + i (lexicographic, x fastest).
* Subelement s = i + p*(j + p*k), i,j,k in [0, p); its corner (a,b,c) is local
  vertex (i+a, j+b, k+c).
* Local edges (lowest-order Nedelec on the LOR mesh): x-edges first, index
  i + p*(j + (p+1)*k) with i < p; then y-edges at offset p*(p+1)^2, index
  i + (p+1)*(j + p*k) with j < p; then z-edges at offset 2*p*(p+1)^2, index
  i + (p+1)*(j + (p+1)*k) with k < p.  Each local edge points along +axis.
* Global edges: with M = n*p, N = M + 1: x-edges X + M*(Y + N*Z); y-edges
  M*N^2 + X + N*(Y + M*Z); z-edges 2*M*N^2 + X + N*(Y + N*Z); each points along
  +axis.  A map entry v >= 0 means global edge v with the same orientation as the
  local edge; v < 0 means global edge -1-v with the opposite orientation (the
  orientation-in-the-sign convention of the processor-local assembly step A2).
"""
from __future__ import annotations

import math

import numpy as np
import torch

__all__ = [
    "gll_points",
    "cartesian_mesh",
    "cartesian_mesh_2d",
    "box_mesh_2d",
    "affine_mesh",
    "nd_edge_map",
    "nd_edge_map_box",
    "face_map",
    "face_map_box",
    "kappa_field",
    "kappa_field_2d",
    "cotangent",
    "renumber_vertices",
    "permute_elements",
    "reorient_elements",
    "flip_edge_signs",
    "boundary_vertices",
    "boundary_edges",
    "random_dofs",
    "ho_nodes",
    "prism_mesh",
    "polygon_mesh_2d",
    "tri_split_mesh",
    "tri_split_mesh_2d",
    "edge_map_from_vertices",
    "face_map_from_vertices",
    "CONFIGS",
    "config_mesh",
]


def gll_points(p: int) -> np.ndarray:
    """The p+1 Gauss-Lobatto points mapped to [0, 1], ascending, float64.

    Endpoints 0 and 1; the interior points are the roots of P_p' (derivative of
    the degree-p Legendre polynomial) on [-1, 1].  The set is symmetrised so that
    t_i + t_{p-i} = 1 up to one rounding.
    """
    if p < 1:
        raise ValueError("p must be >= 1")
    if p == 1:
        r = np.array([-1.0, 1.0])
    else:
        inner = np.polynomial.legendre.Legendre.basis(p).deriv().roots().real
        r = np.concatenate([[-1.0], np.sort(inner), [1.0]])
    r = 0.5 * (r - r[::-1])
    return 0.5 * (r + 1.0)


def _lattice_1d(n: int, p: int) -> np.ndarray:
    """Reference coordinate in [0,1] of each of the N = n*p+1 lattice points."""
    t = gll_points(p)
    x = np.empty(n * p + 1)
    for e in range(n):
        x[e * p:(e + 1) * p + 1] = (e + t) / n
    x[0], x[-1] = 0.0, 1.0
    return x


def _elem_dofs(n: int, p: int) -> np.ndarray:
    N = n * p + 1
    q = p + 1
    ex, ey, ez = np.meshgrid(np.arange(n), np.arange(n), np.arange(n), indexing="ij")
    # element id e = ex + n*(ey + n*ez): order so that ex varies fastest
    ex = ex.transpose(2, 1, 0).reshape(-1)
    ey = ey.transpose(2, 1, 0).reshape(-1)
    ez = ez.transpose(2, 1, 0).reshape(-1)
    i, j, k = np.meshgrid(np.arange(q), np.arange(q), np.arange(q), indexing="ij")
    i = i.transpose(2, 1, 0).reshape(-1)
    j = j.transpose(2, 1, 0).reshape(-1)
    k = k.transpose(2, 1, 0).reshape(-1)
    X = p * ex[:, None] + i[None, :]
    Y = p * ey[:, None] + j[None, :]
    Z = p * ez[:, None] + k[None, :]
    g = X + N * (Y + N * Z)
    return g.astype(np.int32)


def cartesian_mesh(n: int, p: int, amp: float = 0.0) -> dict:
    """n^3 hexes of degree p on the unit cube, LOR vertices perturbed by

        x' = x + A sin(2 pi y) sin(2 pi z)   (and cyclically for y', z'),

    with A = amp / n (amp is the amplitude in units of the coarse element size
    h = 1/n).  The map is applied to every Gauss-Lobatto lattice vertex.
    Returns a dict with coords [N^3, 3] float64, elem_dofs [n^3, (p+1)^3] int32,
    n, p, N, nel, ndofs.
    """
    N = n * p + 1
    x1 = _lattice_1d(n, p)
    X, Y, Z = np.meshgrid(x1, x1, x1, indexing="ij")
    X = X.transpose(2, 1, 0).reshape(-1)
    Y = Y.transpose(2, 1, 0).reshape(-1)
    Z = Z.transpose(2, 1, 0).reshape(-1)
    A = amp / n
    if A != 0.0:
        tp = 2.0 * math.pi
        sx, sy, sz = np.sin(tp * X), np.sin(tp * Y), np.sin(tp * Z)
        X, Y, Z = X + A * sy * sz, Y + A * sz * sx, Z + A * sx * sy
    coords = np.stack([X, Y, Z], axis=1).astype(np.float64)
    return {
        "coords": coords,
        "elem_dofs": _elem_dofs(n, p),
        "n": n,
        "p": p,
        "N": N,
        "nel": n ** 3,
        "ndofs": N ** 3,
    }


def box_mesh(nx: int, ny: int, nz: int, p: int, amp: float = 0.0) -> dict:
    """nx x ny x nz hexes of degree p on the box [0, nx/m] x [0, ny/m] x [0, nz/m]
    (m = max(nx, ny, nz)), numbered like cartesian_mesh: element
    ex + nx (ey + ny ez), lattice vertex X + LX (Y + LY Z) with LX = nx p + 1
    (and so on), local vertex i + (p+1)(j + (p+1)k); every lattice vertex moved
    by the map of cartesian_mesh with A = amp / m.  box_mesh(n, n, n, p, amp)
    equals cartesian_mesh(n, p, amp)."""
    m = max(nx, ny, nz)
    q = p + 1
    L = (nx * p + 1, ny * p + 1, nz * p + 1)
    x1 = [_lattice_1d(n, p) * (n / m) for n in (nx, ny, nz)]
    Z, Y, X = np.meshgrid(x1[2], x1[1], x1[0], indexing="ij")
    X, Y, Z = X.reshape(-1), Y.reshape(-1), Z.reshape(-1)
    A = amp / m
    if A != 0.0:
        tp = 2.0 * math.pi
        sx, sy, sz = np.sin(tp * X), np.sin(tp * Y), np.sin(tp * Z)
        X, Y, Z = X + A * sy * sz, Y + A * sz * sx, Z + A * sx * sy
    coords = np.stack([X, Y, Z], axis=1).astype(np.float64)
    e = np.arange(nx * ny * nz)
    ex, ey, ez = e % nx, (e // nx) % ny, e // (nx * ny)
    l = np.arange(q ** 3)
    i, j, k = l % q, (l // q) % q, l // (q * q)
    g = (p * ex[:, None] + i) + L[0] * ((p * ey[:, None] + j) + L[1] * (p * ez[:, None] + k))
    return {
        "coords": coords,
        "elem_dofs": g.astype(np.int32),
        "p": p,
        "box": (nx, ny, nz),
        "nel": nx * ny * nz,
        "ndofs": L[0] * L[1] * L[2],
    }


def cartesian_mesh_2d(n: int, p: int, amp: float = 0.0) -> dict:
    """n^2 quadrilaterals of degree p on the unit square (the 2D variant):
    element e = ex + n*ey, local vertex i + (p+1)*j, global vertex X + N*Y with
    N = n*p + 1 on the Gauss-Lobatto lattice, every lattice vertex moved by
        x' = x + A sin(2 pi y),  y' = y + A sin(2 pi x),   A = amp / n.
    Returns coords [N^2, 2] float64, elem_dofs [n^2, (p+1)^2] int32, n, p, N,
    nel, ndofs."""
    N = n * p + 1
    q = p + 1
    x1 = _lattice_1d(n, p)
    X, Y = np.meshgrid(x1, x1, indexing="xy")   # [Y][X]
    X, Y = X.reshape(-1), Y.reshape(-1)
    A = amp / n
    if A != 0.0:
        tp = 2.0 * math.pi
        X, Y = X + A * np.sin(tp * Y), Y + A * np.sin(tp * X)
    e = np.arange(n * n)
    ex, ey = e % n, e // n
    j, i = np.meshgrid(np.arange(q), np.arange(q), indexing="ij")
    i, j = i.reshape(-1), j.reshape(-1)          # local vertex i + q*j
    g = (p * ex[:, None] + i[None, :]) + N * (p * ey[:, None] + j[None, :])
    return {"coords": np.stack([X, Y], axis=1).astype(np.float64), "elem_dofs": g.astype(np.int32),
            "n": n, "p": p, "N": N, "nel": n * n, "ndofs": N * N}


def box_mesh_2d(nx: int, ny: int, p: int, amp: float = 0.0) -> dict:
    """nx x ny quadrilaterals of degree p on [0, nx/m] x [0, ny/m] (m = max(nx, ny)),
    numbered like cartesian_mesh_2d: element ex + nx*ey, lattice vertex X + LX*Y
    with LX = nx*p + 1, local vertex i + (p+1)*j; every lattice vertex moved by
    the map of cartesian_mesh_2d with A = amp / m.  box_mesh_2d(n, n, p, amp)
    equals cartesian_mesh_2d(n, p, amp)."""
    m = max(nx, ny)
    q = p + 1
    LX, LY = nx * p + 1, ny * p + 1
    X, Y = np.meshgrid(_lattice_1d(nx, p) * (nx / m), _lattice_1d(ny, p) * (ny / m), indexing="xy")
    X, Y = X.reshape(-1), Y.reshape(-1)
    A = amp / m
    if A != 0.0:
        tp = 2.0 * math.pi
        X, Y = X + A * np.sin(tp * Y), Y + A * np.sin(tp * X)
    e = np.arange(nx * ny)
    ex, ey = e % nx, e // nx
    l = np.arange(q * q)
    i, j = l % q, l // q
    g = (p * ex[:, None] + i) + LX * (p * ey[:, None] + j)
    return {"coords": np.stack([X, Y], axis=1).astype(np.float64), "elem_dofs": g.astype(np.int32), "p": p,
            "box": (nx, ny), "nel": nx * ny, "ndofs": LX * LY}


def affine_mesh(n: int, p: int, A: np.ndarray, t: np.ndarray) -> dict:
    """Cartesian Gauss-Lobatto lattice mapped by x -> A x + t (parallelepipeds)."""
    m = cartesian_mesh(n, p, 0.0)
    m["coords"] = m["coords"] @ np.asarray(A, dtype=np.float64).T + np.asarray(t, dtype=np.float64)
    return m


def nd_edge_map(n: int, p: int) -> tuple[np.ndarray, int]:
    """Signed element-to-edge map [n^3, 3p(p+1)^2] int32 and the edge count."""
    M = n * p
    N = M + 1
    q = p + 1
    ne = n ** 3
    e = np.arange(ne)
    ex, ey, ez = e % n, (e // n) % n, e // (n * n)
    out = np.empty((ne, 3 * p * q * q), dtype=np.int64)
    off = 0
    # x-edges: i < p, j,k <= p
    for k in range(q):
        for j in range(q):
            for i in range(p):
                ll = i + p * (j + q * k)
                X, Y, Z = p * ex + i, p * ey + j, p * ez + k
                out[:, ll] = X + M * (Y + N * Z)
    off = p * q * q
    for k in range(q):
        for j in range(p):
            for i in range(q):
                ll = off + i + q * (j + p * k)
                X, Y, Z = p * ex + i, p * ey + j, p * ez + k
                out[:, ll] = M * N * N + X + N * (Y + M * Z)
    off = 2 * p * q * q
    for k in range(p):
        for j in range(q):
            for i in range(q):
                ll = off + i + q * (j + q * k)
                X, Y, Z = p * ex + i, p * ey + j, p * ez + k
                out[:, ll] = 2 * M * N * N + X + N * (Y + N * Z)
    return out.astype(np.int32), 3 * M * N * N


def nd_edge_map_box(nx: int, ny: int, nz: int, p: int) -> tuple[np.ndarray, int]:
    """nd_edge_map for the nx x ny x nz elements of box_mesh: the same local
    edges; global edges with cells (MX, MY, MZ) = (nx p, ny p, nz p) per axis:
    x-edges X + MX*(Y + (MY+1)*Z); y-edges OY + X + (MX+1)*(Y + MY*Z) with
    OY = MX (MY+1) (MZ+1); z-edges OZ + X + (MX+1)*(Y + (MY+1)*Z) with
    OZ = OY + (MX+1) MY (MZ+1).  nd_edge_map_box(n, n, n, p) equals
    nd_edge_map(n, p)."""
    MX, MY, MZ = nx * p, ny * p, nz * p
    q = p + 1
    ne = nx * ny * nz
    e = np.arange(ne)
    ex, ey, ez = e % nx, (e // nx) % ny, e // (nx * ny)
    OY = MX * (MY + 1) * (MZ + 1)
    OZ = OY + (MX + 1) * MY * (MZ + 1)
    out = np.empty((ne, 3 * p * q * q), dtype=np.int64)
    for k in range(q):
        for j in range(q):
            for i in range(p):
                X, Y, Z = p * ex + i, p * ey + j, p * ez + k
                out[:, i + p * (j + q * k)] = X + MX * (Y + (MY + 1) * Z)
    off = p * q * q
    for k in range(q):
        for j in range(p):
            for i in range(q):
                X, Y, Z = p * ex + i, p * ey + j, p * ez + k
                out[:, off + i + q * (j + p * k)] = OY + X + (MX + 1) * (Y + MY * Z)
    off = 2 * p * q * q
    for k in range(p):
        for j in range(q):
            for i in range(q):
                X, Y, Z = p * ex + i, p * ey + j, p * ez + k
                out[:, off + i + q * (j + q * k)] = OZ + X + (MX + 1) * (Y + (MY + 1) * Z)
    return out.astype(np.int32), OZ + (MX + 1) * (MY + 1) * MZ


def face_map(n: int, p: int) -> tuple[np.ndarray, int]:
    """Signed element-to-face map [n^3, 3p^2(p+1)] int32 of the LOR mesh faces
    (the lowest-order Raviart-Thomas dofs) and the face count.

    Local faces: x-faces (normal +x) first, index i + (p+1)*(j + p*k) with
    i <= p, j, k < p; then y-faces at offset p^2(p+1), index i + p*(j + (p+1)*k)
    with j <= p; then z-faces at offset 2p^2(p+1), index i + p*(j + p*k) with
    k <= p.  Global faces, M = n*p, N = M + 1: x-faces X + N*(Y + M*Z); y-faces
    N*M^2 + X + M*(Y + N*Z); z-faces 2*N*M^2 + X + M*(Y + M*Z); every face
    normal points along +axis, and a negative entry -1-f means face f with the
    opposite orientation (as for edges)."""
    M = n * p
    N = M + 1
    q = p + 1
    ne = n ** 3
    e = np.arange(ne)
    ex, ey, ez = e % n, (e // n) % n, e // (n * n)
    out = np.empty((ne, 3 * p * p * q), dtype=np.int64)
    for k in range(p):
        for j in range(p):
            for i in range(q):
                X, Y, Z = p * ex + i, p * ey + j, p * ez + k
                out[:, i + q * (j + p * k)] = X + N * (Y + M * Z)
    off = p * p * q
    for k in range(p):
        for j in range(q):
            for i in range(p):
                X, Y, Z = p * ex + i, p * ey + j, p * ez + k
                out[:, off + i + p * (j + q * k)] = N * M * M + X + M * (Y + N * Z)
    off = 2 * p * p * q
    for k in range(q):
        for j in range(p):
            for i in range(p):
                X, Y, Z = p * ex + i, p * ey + j, p * ez + k
                out[:, off + i + p * (j + p * k)] = 2 * N * M * M + X + M * (Y + M * Z)
    return out.astype(np.int32), 3 * N * M * M


def face_map_box(nx: int, ny: int, nz: int, p: int) -> tuple[np.ndarray, int]:
    """face_map for the nx x ny x nz elements of box_mesh: the same local
    faces; global faces with cells (MX, MY, MZ) = (nx p, ny p, nz p) per axis:
    x-faces X + (MX+1)*(Y + MY*Z); y-faces OY + X + MX*(Y + (MY+1)*Z) with
    OY = (MX+1) MY MZ; z-faces OZ + X + MX*(Y + MY*Z) with OZ = OY + MX (MY+1) MZ.
    face_map_box(n, n, n, p) equals face_map(n, p)."""
    MX, MY, MZ = nx * p, ny * p, nz * p
    q = p + 1
    ne = nx * ny * nz
    e = np.arange(ne)
    ex, ey, ez = e % nx, (e // nx) % ny, e // (nx * ny)
    OY = (MX + 1) * MY * MZ
    OZ = OY + MX * (MY + 1) * MZ
    out = np.empty((ne, 3 * p * p * q), dtype=np.int64)
    for k in range(p):
        for j in range(p):
            for i in range(q):
                X, Y, Z = p * ex + i, p * ey + j, p * ez + k
                out[:, i + q * (j + p * k)] = X + (MX + 1) * (Y + MY * Z)
    off = p * p * q
    for k in range(p):
        for j in range(q):
            for i in range(p):
                X, Y, Z = p * ex + i, p * ey + j, p * ez + k
                out[:, off + i + p * (j + q * k)] = OY + X + MX * (Y + (MY + 1) * Z)
    off = 2 * p * p * q
    for k in range(q):
        for j in range(p):
            for i in range(p):
                X, Y, Z = p * ex + i, p * ey + j, p * ez + k
                out[:, off + i + p * (j + p * k)] = OZ + X + MX * (Y + MY * Z)
    return out.astype(np.int32), OZ + MX * MY * (MZ + 1)


def kappa_field(nel: int, p: int, sigma: float, seed: int = 0, batch: int | None = None,
                ) -> torch.Tensor:
    """Log-normal per-subelement coefficient exp(sigma * z), z ~ N(0, 1).

    Draw order: torch.Generator('cpu').manual_seed(seed), then one randn of shape
    (B, nel, p, p, p) (index [b][e][k][j][i]), float64.  Returned with shape
    (nel, p^3) when batch is None, else (batch, nel, p^3); subelement index
    s = i + p*(j + p*k).
    """
    g = torch.Generator(device="cpu")
    g.manual_seed(seed)
    B = 1 if batch is None else batch
    z = torch.randn((B, nel, p, p, p), generator=g, dtype=torch.float64)
    k = torch.exp(sigma * z).reshape(B, nel, p ** 3)
    return k[0] if batch is None else k


def kappa_field_2d(nel: int, p: int, sigma: float, seed: int = 0) -> torch.Tensor:
    """2D counterpart of kappa_field: exp(sigma z) per subelement, z drawn as
    randn((nel, p, p)) (index [e][j][i], subelement i + p*j), float64."""
    g = torch.Generator(device="cpu")
    g.manual_seed(seed)
    z = torch.randn((nel, p, p), generator=g, dtype=torch.float64)
    return torch.exp(sigma * z).reshape(nel, p * p)


def cotangent(batch: int, nnz: int, seed: int = 1) -> torch.Tensor:
    """Gaussian cotangent on the CSR values, shape (batch, nnz), float64."""
    g = torch.Generator(device="cpu")
    g.manual_seed(seed)
    return torch.randn((batch, nnz), generator=g, dtype=torch.float64)


# ---------------------------------------------------------------- perturbations

def renumber_vertices(mesh: dict, seed: int) -> tuple[dict, np.ndarray]:
    """Random relabelling of the global vertices: new id = perm[old id]."""
    rng = np.random.default_rng(seed)
    perm = rng.permutation(mesh["ndofs"]).astype(np.int64)
    out = dict(mesh)
    coords = np.empty_like(mesh["coords"])
    coords[perm] = mesh["coords"]
    out["coords"] = coords
    out["elem_dofs"] = perm[mesh["elem_dofs"].astype(np.int64)].astype(np.int32)
    return out, perm


def permute_elements(mesh: dict, seed: int) -> tuple[dict, np.ndarray]:
    """Random reordering of the elements: new element r holds old element order[r]."""
    rng = np.random.default_rng(seed)
    order = rng.permutation(mesh["nel"]).astype(np.int64)
    out = dict(mesh)
    out["elem_dofs"] = np.ascontiguousarray(mesh["elem_dofs"][order])
    return out, order


def _cube_symmetries() -> list[tuple[tuple[int, int, int], tuple[bool, bool, bool]]]:
    """The 24 rotations of the cube as (axis permutation, axis reversal): the
    signed permutations of determinant +1, so that positively oriented elements
    stay positively oriented."""
    import itertools
    out = []
    for perm in itertools.permutations(range(3)):
        inv = sum(1 for a in range(3) for b in range(a + 1, 3) if perm[a] > perm[b])
        for flips in itertools.product([False, True], repeat=3):
            if (inv + sum(flips)) % 2 == 0:
                out.append((perm, flips))
    return out


def _sym_lattice_index(q: int, perm, flips) -> np.ndarray:
    """For a (q x q x q) lattice (index i + q(j + q k)), the source index of every
    destination index under the symmetry: new[c] = old[src[c]]."""
    idx = np.arange(q ** 3)
    c = [idx % q, (idx // q) % q, idx // (q * q)]
    src = [None, None, None]
    for d in range(3):
        v = c[d]
        src[perm[d]] = (q - 1 - v) if flips[d] else v
    return src[0] + q * (src[1] + q * src[2])


def reorient_elements(mesh: dict, seed: int, kappa: torch.Tensor | None = None,
                      elem_edges: np.ndarray | None = None):
    """Give every element an independent random local orientation (one of the 24
    cube rotations applied to its local lattice).  The assembled LOR matrix is
    unchanged; only the local numbering (and the local edge directions) differ.

    Returns (mesh', kappa', elem_edges') with kappa [.., nel, p^3] permuted the
    same way and the signed edge map re-signed where a local edge now points the
    other way.
    """
    p = mesh["p"]
    q = p + 1
    syms = _cube_symmetries()
    rng = np.random.default_rng(seed)
    choice = rng.integers(0, len(syms), size=mesh["nel"])
    ed = mesh["elem_dofs"].copy()
    kap = None if kappa is None else kappa.clone()
    ee = None if elem_edges is None else elem_edges.copy()
    for si, (perm, flips) in enumerate(syms):
        sel = np.nonzero(choice == si)[0]
        if sel.size == 0:
            continue
        vsrc = _sym_lattice_index(q, perm, flips)
        ed[sel] = mesh["elem_dofs"][sel][:, vsrc]
        if kap is not None:
            ssrc = torch.from_numpy(_sym_lattice_index(p, perm, flips))
            ks = torch.from_numpy(sel)
            kap[..., ks, :] = kappa[..., ks, :][..., ssrc]
        if ee is not None:
            esrc, esgn = _sym_edge_index(p, perm, flips)
            old = elem_edges[sel][:, esrc].astype(np.int64)
            neg = old < 0
            gid = np.where(neg, -1 - old, old)
            sgn = np.where(neg, -1, 1) * esgn[None, :]
            ee[sel] = np.where(sgn > 0, gid, -1 - gid).astype(np.int32)
    out = dict(mesh)
    out["elem_dofs"] = ed
    return out, kap, ee


def _local_edges(p: int):
    """List of (axis, i, j, k) for every local edge in local numbering."""
    q = p + 1
    out = []
    for k in range(q):
        for j in range(q):
            for i in range(p):
                out.append((0, i, j, k))
    for k in range(q):
        for j in range(p):
            for i in range(q):
                out.append((1, i, j, k))
    for k in range(p):
        for j in range(q):
            for i in range(q):
                out.append((2, i, j, k))
    return out


def _sym_edge_index(p: int, perm, flips):
    """Edge analogue of _sym_lattice_index: returns (src, sign) so that the new
    local edge c is the old local edge src[c], traversed with relative sign
    sign[c] (-1 when the symmetry reverses it)."""
    q = p + 1
    edges = _local_edges(p)
    lookup = {e: n for n, e in enumerate(edges)}
    src = np.empty(len(edges), dtype=np.int64)
    sgn = np.empty(len(edges), dtype=np.int64)
    for c, (ax, i, j, k) in enumerate(edges):
        # new edge from new-vertex v0=(i,j,k) to v1=v0+unit(ax)
        v0 = [i, j, k]
        v1 = [i, j, k]
        v1[ax] += 1
        o0 = [0, 0, 0]
        o1 = [0, 0, 0]
        for d in range(3):
            o0[perm[d]] = (q - 1 - v0[d]) if flips[d] else v0[d]
            o1[perm[d]] = (q - 1 - v1[d]) if flips[d] else v1[d]
        oax = perm[ax]
        if o1[oax] > o0[oax]:
            base, s = o0, 1
        else:
            base, s = o1, -1
        src[c] = lookup[(oax, base[0], base[1], base[2])]
        sgn[c] = s
    return src, sgn


def flip_edge_signs(elem_edges: np.ndarray, nedges: int, seed: int):
    """Reverse the global orientation of a random half of the edges (or of the
    faces, given a signed face map).  Returns the new signed map and the +-1
    vector S with A' = S A S."""
    rng = np.random.default_rng(seed)
    s = np.where(rng.random(nedges) < 0.5, -1, 1).astype(np.int64)
    old = elem_edges.astype(np.int64)
    neg = old < 0
    gid = np.where(neg, -1 - old, old)
    sg = np.where(neg, -1, 1) * s[gid]
    return np.where(sg > 0, gid, -1 - gid).astype(np.int32), s


def ho_nodes(n: int, q: int, amp: float = 0.0) -> np.ndarray:
    """Nodes of a degree-q high-order mesh of the n^3 cube as an E-vector
    [n^3][(q+1)^3][3]: the same curved map as cartesian_mesh, evaluated at
    each element's tensor Gauss-Lobatto points of degree q (local node
    i + (q+1)(j + (q+1)k))."""
    m = cartesian_mesh(n, q, amp)
    return np.ascontiguousarray(m["coords"][m["elem_dofs"]])


# ---------------------------------------------------------------- essential dofs

def boundary_vertices(n: int, p: int) -> np.ndarray:
    """Ids (ascending, int32) of the lattice vertices on the boundary of the
    cube: X, Y or Z equal to 0 or M = n*p."""
    N = n * p + 1
    g = np.arange(N ** 3, dtype=np.int64)
    X, Y, Z = g % N, (g // N) % N, g // (N * N)
    on = (X == 0) | (X == N - 1) | (Y == 0) | (Y == N - 1) | (Z == 0) | (Z == N - 1)
    return g[on].astype(np.int32)


def boundary_edges(n: int, p: int) -> np.ndarray:
    """Ids (ascending, int32) of the edges lying in the boundary of the cube
    (tangential edges, the essential dofs of H(curl)): an x-edge at (X, Y, Z)
    lies in the boundary iff Y or Z is 0 or M, and cyclically."""
    M = n * p
    N = M + 1
    out = []
    a = np.arange(M * N * N, dtype=np.int64)
    # x-edges X + M*(Y + N*Z)
    Y, Z = (a // M) % N, a // (M * N)
    out.append(a[(Y == 0) | (Y == M) | (Z == 0) | (Z == M)])
    # y-edges M*N^2 + X + N*(Y + M*Z)
    X, Z = a % N, a // (N * M)
    out.append(M * N * N + a[(X == 0) | (X == M) | (Z == 0) | (Z == M)])
    # z-edges 2*M*N^2 + X + N*(Y + N*Z)
    X, Y = a % N, (a // N) % N
    out.append(2 * M * N * N + a[(X == 0) | (X == M) | (Y == 0) | (Y == M)])
    return np.concatenate(out).astype(np.int32)


def random_dofs(ndofs: int, count: int, seed: int, duplicates: bool = True) -> np.ndarray:
    """`count` random dof ids in [0, ndofs) (with repeats if duplicates), in
    random order, int32.  Draw order: numpy default_rng(seed), then integers or
    a permutation."""
    rng = np.random.default_rng(seed)
    if duplicates:
        return rng.integers(0, ndofs, size=count).astype(np.int32)
    return rng.permutation(ndofs)[:count].astype(np.int32)


# ---------------------------------------------------------------- unstructured

def prism_mesh(p: int, sides: int = 3, layers: int = 2, amp: float = 0.0) -> dict:
    """A conforming hexahedral mesh that is not a Cartesian grid: the regular
    `sides`-gon of circumradius 1 is cut into `sides` quadrilaterals around its
    centre C (quadrilateral k has the corners C, the midpoint M_{k-1} of side
    k-1, the polygon vertex P_k and the midpoint M_k, with P_k at angle
    2 pi k / sides and side k joining P_k and P_{k+1}), and the polygon is
    extruded over z in [0, 1] in `layers` layers.  The edge through C is shared
    by `sides` elements per layer (3 or 5: irregular valence), the polygon
    vertices by one.  Element e = k + sides * l; its local corner (a, b, c) is
    C, M_{k-1}, P_k, M_k for (a, b) = (0,0), (1,0), (1,1), (0,1), at height
    (l + c) / layers; lattice points come from the bilinear-in-plane map at the
    Gauss-Lobatto points.  Points shared by neighbouring elements are merged by
    their coordinates snapped to 1e-9, and the global ids follow the sorted
    snapped coordinates.  With amp != 0, every lattice vertex is then moved by
        x' = x + A sin(2 pi y) sin(2 pi z)   (and cyclically),   A = amp / 2.
    Returns coords, elem_dofs, p, sides, layers, nel, ndofs (as cartesian_mesh,
    without n and N)."""
    if sides < 3 or layers < 1:
        raise ValueError("sides >= 3 and layers >= 1")
    q = p + 1
    t = gll_points(p)
    ang = 2.0 * math.pi * np.arange(sides) / sides
    P = np.stack([np.cos(ang), np.sin(ang)], axis=1)
    Mid = 0.5 * (P + np.roll(P, -1, axis=0))          # Mid[k] joins P[k] and P[k+1]
    C = np.zeros(2)
    # local lattice parameters, index i + q*(j + q*k)
    kk, jj, ii = np.meshgrid(np.arange(q), np.arange(q), np.arange(q), indexing="ij")
    xi, eta, zeta = t[ii.reshape(-1)], t[jj.reshape(-1)], t[kk.reshape(-1)]
    pts = []
    for l in range(layers):
        for k in range(sides):
            c00, c10, c11, c01 = C, Mid[k - 1], P[k], Mid[k]
            xy = (((1 - xi) * (1 - eta))[:, None] * c00 + (xi * (1 - eta))[:, None] * c10
                  + (xi * eta)[:, None] * c11 + ((1 - xi) * eta)[:, None] * c01)
            z = (l + zeta) / layers
            pts.append(np.concatenate([xy, z[:, None]], axis=1))
    pts = np.concatenate(pts, axis=0)
    key = np.round(pts * 1e9).astype(np.int64)
    uniq, inv = np.unique(key, axis=0, return_inverse=True)
    first = np.full(len(uniq), -1, dtype=np.int64)
    order = np.arange(len(inv))[::-1]
    first[inv.reshape(-1)[order]] = order               # one representative per merged point
    coords = pts[first].copy()
    expect = (1 + sides * p + sides * p * p) * (layers * p + 1)
    if len(uniq) != expect:
        raise RuntimeError(f"lattice merge gave {len(uniq)} vertices, expected {expect}")
    A = amp / 2.0
    if A != 0.0:
        tp = 2.0 * math.pi
        X, Y, Z = coords[:, 0], coords[:, 1], coords[:, 2]
        sx, sy, sz = np.sin(tp * X), np.sin(tp * Y), np.sin(tp * Z)
        coords = np.stack([X + A * sy * sz, Y + A * sz * sx, Z + A * sx * sy], axis=1)
    nel = sides * layers
    return {"coords": np.ascontiguousarray(coords, dtype=np.float64),
            "elem_dofs": inv.reshape(nel, q ** 3).astype(np.int32),
            "p": p, "sides": sides, "layers": layers, "nel": nel, "ndofs": len(uniq)}


def polygon_mesh_2d(p: int, sides: int = 3, amp: float = 0.0) -> dict:
    """The 2D counterpart of prism_mesh: the regular `sides`-gon of
    circumradius 1 cut into `sides` quadrilaterals around its centre (corner
    (a, b) of quadrilateral k is C, M_{k-1}, P_k, M_k for (0,0), (1,0), (1,1),
    (0,1)), so the centre is shared by `sides` elements.  Local vertex i + q*j;
    lattice points merged by coordinates snapped to 1e-9, global ids following
    the sorted snapped coordinates; with amp != 0 every lattice vertex is moved
    by x' = x + A sin(2 pi y), y' = y + A sin(2 pi x), A = amp / 2.  Returns
    coords [ndofs, 2], elem_dofs [sides, (p+1)^2], p, sides, nel, ndofs."""
    if sides < 3:
        raise ValueError("sides >= 3")
    q = p + 1
    t = gll_points(p)
    ang = 2.0 * math.pi * np.arange(sides) / sides
    P = np.stack([np.cos(ang), np.sin(ang)], axis=1)
    Mid = 0.5 * (P + np.roll(P, -1, axis=0))
    jj, ii = np.meshgrid(np.arange(q), np.arange(q), indexing="ij")
    xi, eta = t[ii.reshape(-1)], t[jj.reshape(-1)]
    pts = []
    for k in range(sides):
        c10, c11, c01 = Mid[k - 1], P[k], Mid[k]       # c00 is the centre (0, 0)
        pts.append((xi * (1 - eta))[:, None] * c10 + (xi * eta)[:, None] * c11 + ((1 - xi) * eta)[:, None] * c01)
    pts = np.concatenate(pts, axis=0)
    key = np.round(pts * 1e9).astype(np.int64)
    uniq, inv = np.unique(key, axis=0, return_inverse=True)
    first = np.full(len(uniq), -1, dtype=np.int64)
    order = np.arange(len(inv))[::-1]
    first[inv.reshape(-1)[order]] = order
    coords = pts[first].copy()
    expect = 1 + sides * p + sides * p * p
    if len(uniq) != expect:
        raise RuntimeError(f"lattice merge gave {len(uniq)} vertices, expected {expect}")
    A = amp / 2.0
    if A != 0.0:
        tp = 2.0 * math.pi
        X, Y = coords[:, 0], coords[:, 1]
        coords = np.stack([X + A * np.sin(tp * Y), Y + A * np.sin(tp * X)], axis=1)
    return {"coords": np.ascontiguousarray(coords, dtype=np.float64),
            "elem_dofs": inv.reshape(sides, q * q).astype(np.int32),
            "p": p, "sides": sides, "nel": sides, "ndofs": len(uniq)}


def _merge_points(pts: np.ndarray, nel: int, nloc: int, expect: int) -> tuple[np.ndarray, np.ndarray]:
    """Global ids of lattice points shared by neighbouring elements: points are
    merged by their coordinates snapped to 1e-9 (ids follow the sorted snapped
    coordinates); returns (coords [ndofs, d], elem_dofs [nel, nloc])."""
    key = np.round(pts * 1e9).astype(np.int64)
    uniq, inv = np.unique(key, axis=0, return_inverse=True)
    if len(uniq) != expect:
        raise RuntimeError(f"lattice merge gave {len(uniq)} vertices, expected {expect}")
    first = np.full(len(uniq), -1, dtype=np.int64)
    order = np.arange(len(inv))[::-1]
    first[inv.reshape(-1)[order]] = order
    return pts[first].copy(), inv.reshape(nel, nloc).astype(np.int32)


def _tri_split_quads(n: int) -> np.ndarray:
    """Corners [6 n^2, 4, 2] of the quadrilaterals of the unit square cut into
    n x n cells, each cell into two triangles by its (0,0)-(1,1) diagonal, each
    triangle (A, B, C), counter-clockwise, into three quadrilaterals around its
    centroid G: (A, M_AB, G, M_CA), (B, M_BC, G, M_AB), (C, M_CA, G, M_BC) as
    local corners (0,0), (1,0), (1,1), (0,1).  Quadrilateral index
    3 (2 (cx + n cy) + t) + corner."""
    quads = []
    for cy in range(n):
        for cx in range(n):
            v00 = np.array([cx, cy], dtype=np.float64) / n
            v10, v11, v01 = v00 + [1.0 / n, 0.0], v00 + [1.0 / n, 1.0 / n], v00 + [0.0, 1.0 / n]
            for A, B, C in ((v00, v10, v11), (v00, v11, v01)):
                G = (A + B + C) / 3.0
                mab, mbc, mca = 0.5 * (A + B), 0.5 * (B + C), 0.5 * (C + A)
                quads += [(A, mab, G, mca), (B, mbc, G, mab), (C, mca, G, mbc)]
    return np.array(quads)


def _tri_split_count(n: int, p: int) -> int:
    """Lattice points of the planar mesh of _tri_split_quads(n) at degree p."""
    return ((n + 1) ** 2 + 2 * n * n + 3 * n * n + 2 * n + (p - 1) * (12 * n * n + 4 * n)
            + 6 * n * n * (p - 1) ** 2)


def tri_split_mesh(n: int, layers: int, p: int, amp: float = 0.0) -> dict:
    """A conforming hexahedral mesh of the unit cube with irregular valence
    throughout: the quadrilaterals of _tri_split_quads(n) (vertex valence 3 at
    the centroids, 4 at the edge midpoints, up to 6 at the grid vertices)
    extruded over z in [0, 1] in `layers` layers; element
    e = quad + 6 n^2 * layer, local corner (a, b, c) at quad corner (a, b) and
    height (layer + c) / layers; Gauss-Lobatto lattice from the
    bilinear-in-plane map; shared points merged by coordinates (count checked
    against its closed form); with amp != 0 every lattice vertex is moved by
    the sinusoidal map of cartesian_mesh with A = amp / n.  Returns coords,
    elem_dofs, p, n, layers, nel, ndofs."""
    q = p + 1
    t = gll_points(p)
    Q = _tri_split_quads(n)
    nq = len(Q)
    kk, jj, ii = np.meshgrid(np.arange(q), np.arange(q), np.arange(q), indexing="ij")
    xi, eta, zeta = t[ii.reshape(-1)], t[jj.reshape(-1)], t[kk.reshape(-1)]
    w = np.stack([(1 - xi) * (1 - eta), xi * (1 - eta), xi * eta, (1 - xi) * eta], axis=1)   # [q^3, 4]
    xy = np.einsum("lc,qcd->qld", w, Q)                                                        # [nq, q^3, 2]
    pts = []
    for l in range(layers):
        z = np.broadcast_to(((l + zeta) / layers)[None, :, None], (nq, q ** 3, 1))
        pts.append(np.concatenate([xy, z], axis=2))
    pts = np.concatenate(pts, axis=0).reshape(-1, 3)
    # planar lattice: vertices (n+1)^2, centroids 2n^2, edge midpoints 3n^2+2n,
    # plus p-1 interior points on each of the 12n^2+4n quadrilateral edges (two
    # halves of every triangle edge, three spokes per triangle) and (p-1)^2
    # inside each of the 6n^2 quadrilaterals
    n2d = _tri_split_count(n, p)
    coords, ed = _merge_points(pts, nq * layers, q ** 3, n2d * (layers * p + 1))
    A = amp / n
    if A != 0.0:
        tp = 2.0 * math.pi
        X, Y, Z = coords[:, 0], coords[:, 1], coords[:, 2]
        sx, sy, sz = np.sin(tp * X), np.sin(tp * Y), np.sin(tp * Z)
        coords = np.stack([X + A * sy * sz, Y + A * sz * sx, Z + A * sx * sy], axis=1)
    return {"coords": np.ascontiguousarray(coords, dtype=np.float64), "elem_dofs": ed, "p": p, "n": n,
            "layers": layers, "nel": nq * layers, "ndofs": len(coords)}


def tri_split_mesh_2d(n: int, p: int, amp: float = 0.0) -> dict:
    """The planar quadrilateral mesh of tri_split_mesh (local vertex i + q*j),
    moved with amp != 0 by the sinusoidal map of cartesian_mesh_2d (A = amp/n)."""
    q = p + 1
    t = gll_points(p)
    Q = _tri_split_quads(n)
    jj, ii = np.meshgrid(np.arange(q), np.arange(q), indexing="ij")
    xi, eta = t[ii.reshape(-1)], t[jj.reshape(-1)]
    w = np.stack([(1 - xi) * (1 - eta), xi * (1 - eta), xi * eta, (1 - xi) * eta], axis=1)
    pts = np.einsum("lc,qcd->qld", w, Q).reshape(-1, 2)
    coords, ed = _merge_points(pts, len(Q), q * q, _tri_split_count(n, p))
    A = amp / n
    if A != 0.0:
        tp = 2.0 * math.pi
        X, Y = coords[:, 0], coords[:, 1]
        coords = np.stack([X + A * np.sin(tp * Y), Y + A * np.sin(tp * X)], axis=1)
    return {"coords": np.ascontiguousarray(coords, dtype=np.float64), "elem_dofs": ed, "p": p, "n": n,
            "nel": len(Q), "ndofs": len(coords)}


def edge_map_from_vertices(elem_dofs: np.ndarray, p: int) -> tuple[np.ndarray, int]:
    """Signed element-to-edge map of any conforming LOR hex mesh, from its
    vertex map alone: the local edges (numbered as in the module docstring, each
    along +axis from its first to its second local vertex) are merged by their
    two global vertex ids; global edge ids follow the sorted (lower id, higher
    id) pairs, and every global edge points from its lower to its higher vertex
    id, so an entry is -1-g where the local edge runs the other way."""
    q = p + 1
    v0, v1 = [], []
    for axis, stride, (ni, nj, nk) in ((0, 1, (p, q, q)), (1, q, (q, p, q)), (2, q * q, (q, q, p))):
        k, j, i = np.meshgrid(np.arange(nk), np.arange(nj), np.arange(ni), indexing="ij")
        a = (i + q * (j + q * k)).reshape(-1)
        v0.append(a)
        v1.append(a + stride)
    v0, v1 = np.concatenate(v0), np.concatenate(v1)
    g0 = elem_dofs[:, v0].astype(np.int64)
    g1 = elem_dofs[:, v1].astype(np.int64)
    lo, hi = np.minimum(g0, g1), np.maximum(g0, g1)
    key = np.stack([lo.reshape(-1), hi.reshape(-1)], axis=1)
    uniq, inv = np.unique(key, axis=0, return_inverse=True)
    gid = inv.reshape(g0.shape)
    out = np.where(g0 < g1, gid, -1 - gid)
    return out.astype(np.int32), len(uniq)


def face_map_from_vertices(elem_dofs: np.ndarray, p: int) -> tuple[np.ndarray, int]:
    """Signed element-to-face map of any conforming LOR hex mesh (local faces
    numbered as in face_map), from its vertex map alone.  Each local face lists
    its 4 vertices in the cyclic order whose right-hand normal is the local
    +axis; faces are merged by their sorted vertex ids (global ids follow the
    sorted 4-tuples).  The global normal of a face is the one of the cyclic
    order that, started at its lowest vertex id, visits the lower of that
    vertex's two neighbours first; an entry is -1-f where the local normal is
    the opposite one."""
    q = p + 1
    cyc = []
    # x-faces at i (0..p), spanning (j, j+1) x (k, k+1): normal +x = e_y x e_z
    k, j, i = np.meshgrid(np.arange(p), np.arange(p), np.arange(q), indexing="ij")
    b = (i + q * (j + q * k)).reshape(-1)
    cyc.append(np.stack([b, b + q, b + q + q * q, b + q * q], axis=1))
    # y-faces at j (0..p), spanning (i, i+1) x (k, k+1): normal +y = e_z x e_x
    k, j, i = np.meshgrid(np.arange(p), np.arange(q), np.arange(p), indexing="ij")
    b = (i + q * (j + q * k)).reshape(-1)
    cyc.append(np.stack([b, b + q * q, b + q * q + 1, b + 1], axis=1))
    # z-faces at k (0..p), spanning (i, i+1) x (j, j+1): normal +z = e_x x e_y
    k, j, i = np.meshgrid(np.arange(q), np.arange(p), np.arange(p), indexing="ij")
    b = (i + q * (j + q * k)).reshape(-1)
    cyc.append(np.stack([b, b + 1, b + 1 + q, b + q], axis=1))
    cyc = np.concatenate(cyc, axis=0)                   # [nlocf, 4] local vertices
    g = elem_dofs[:, cyc].astype(np.int64)               # [nel, nlocf, 4]
    key = np.sort(g, axis=2).reshape(-1, 4)
    uniq, inv = np.unique(key, axis=0, return_inverse=True)
    gid = inv.reshape(g.shape[:2])
    m = np.argmin(g, axis=2)
    nxt = np.take_along_axis(g, ((m + 1) % 4)[..., None], axis=2)[..., 0]
    prv = np.take_along_axis(g, ((m + 3) % 4)[..., None], axis=2)[..., 0]
    out = np.where(nxt < prv, gid, -1 - gid)
    return out.astype(np.int32), len(uniq)


# ---------------------------------------------------------------- named workloads

#: The named workloads: (space, n, p, amp, sigma, beta, batch).
CONFIGS = {
    "c1_h1_p2_uniform": dict(space="h1", n=4, p=2, amp=0.0, sigma=0.0, beta=0.0, batch=1),
    "c2_h1_p4_curved": dict(space="h1", n=16, p=4, amp=0.1, sigma=1.0, beta=1.0, batch=1),
    "c3_h1_p6_curved": dict(space="h1", n=32, p=6, amp=0.1, sigma=2.0, beta=1.0, batch=1),
    "c4_nd_p3_curved": dict(space="nd", n=24, p=3, amp=0.1, sigma=1.0, beta=1.0, batch=1),
    "c5_h1_p4_backward": dict(space="h1", n=16, p=4, amp=0.1, sigma=1.0, beta=1.0, batch=8),
    "c6_rt_p3_curved": dict(space="rt", n=24, p=3, amp=0.1, sigma=1.0, beta=1.0, batch=1),
    "c7_h1_2d_p6_curved": dict(space="h1_2d", n=512, p=6, amp=0.1, sigma=2.0, beta=1.0, batch=1),
    # the headline form on an unstructured mesh of the same size: tri_split_mesh(16, 21 layers)
    "c8_h1_p6_trisplit": dict(space="h1_tri", n=16, layers=21, p=6, amp=0.1, sigma=2.0, beta=1.0, batch=1),
}


def config_mesh(name: str, seed: int = 0) -> dict:
    """Mesh, coefficients (and edge map for H(curl)) of a named workload."""
    c = CONFIGS[name]
    if c["space"] == "h1_2d":
        m = cartesian_mesh_2d(c["n"], c["p"], c["amp"])
        m["kappa"] = kappa_field_2d(m["nel"], c["p"], c["sigma"], seed)
        m["beta"] = c["beta"]
        m["config"] = dict(c, name=name)
        return m
    if c["space"] == "h1_tri":
        m = tri_split_mesh(c["n"], c["layers"], c["p"], c["amp"])
    else:
        m = cartesian_mesh(c["n"], c["p"], c["amp"])
    if c["sigma"] == 0.0:
        kap = torch.ones((m["nel"], c["p"] ** 3), dtype=torch.float64)
        if c["batch"] > 1:
            kap = kap.expand(c["batch"], -1, -1).contiguous()
    else:
        kap = kappa_field(m["nel"], c["p"], c["sigma"], seed,
                          batch=None if c["batch"] == 1 else c["batch"])
    m["kappa"] = kap
    m["beta"] = c["beta"]
    m["config"] = dict(c, name=name)
    if c["space"] == "nd":
        ee, ned = nd_edge_map(c["n"], c["p"])
        m["elem_edges"] = ee
        m["nedges"] = ned
    if c["space"] == "rt":
        fm, nf = face_map(c["n"], c["p"])
        m["elem_faces"] = fm
        m["nfaces"] = nf
    return m
