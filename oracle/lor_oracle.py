"""CPU FP64 oracle for low-order-refined (LOR) matrix assembly.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path imports, calls or links
this module; only the tests, the smoke check and the CPU-baseline leg of the
benchmark use it.  It shares no code with the HIP path (the only common import
is the seeded input generator, which holds none of the method's arithmetic).

What it computes is the plain definition of the LOR matrices, written out:

* Section "The low-order-refined mesh": every degree-p hexahedron is split at its
  tensor Gauss-Lobatto lattice into p^3 subelements; the subelement vertices are
  the mapped lattice points (given here as node coordinates).
* Section "Poisson problem": the LOR space is the p=1 (trilinear, Q1) H1 space on
  the refined mesh, with the same degrees of freedom as the high-order space; its
  stiffness matrix (kappa grad u, grad v) and mass matrix (beta u, v) are the
  standard element-by-element assembled finite element matrices.
* Section "Vector finite elements": the lowest-order interpolation-histopolation
  H(curl) case is the standard lowest-order Nedelec element on the refined mesh;
  its curl-curl (kappa curl u, curl v) and mass (beta u, v) matrices.
* Step A2 (processor-local assembly): the orientation of a vector basis function
  is carried by the sign of its degree of freedom.
* Section "Adaptive mesh refinement": for conforming meshes the LOR matrix is the
  element-by-element assembly Lambda^T A_hat Lambda, which is what the COO-then-
  sort below computes (COO = the unassembled block-diagonal A_hat, the sort and
  segment sum = the Boolean assembly operator).

Readings of points the paper leaves open (the HIP path takes the same ones):
* Subelement quadrature: 2x2x2 Gauss-Legendre (weights 1/8 on the unit cube).
* Coefficients: kappa constant per subelement, beta a scalar (or, for tests, a
  per-subelement tensor).  Consistent (not lumped) mass.
* CSR form: full symmetric storage, columns sorted ascending and unique, every
  structurally present entry kept even where its value cancels to ~0.
* Inverted subelements (det J <= 0 at a quadrature point) raise ValueError.

Every function is in float64 and differentiable (torch autograd) in the node
coordinates and the coefficients, which gives the reference gradient of the
adjoint kernel.  "Parity unpinned" functions: none.  tests/test_oracle_pins.py
pins every whole-matrix function against closed forms, invariants, exact
sequences or brute force, and every row-subset function (h1_rows, nd_rows,
rt_rows, h1_rows_2d, the references of the full-size parity tests) against the
rows of its pinned whole-matrix form.
"""
from __future__ import annotations

import math

import torch

__all__ = [
    "GAUSS_T",
    "h1_subelement_vertices",
    "h1_subelement_matrices",
    "nd_subelement_edges",
    "nd_subelement_matrices",
    "coo_to_csr",
    "h1_matrix",
    "h1_rows",
    "nd_matrix",
    "nd_rows",
    "h1_matrix_2d",
    "h1_rows_2d",
    "rt_subelement_faces",
    "rt_subelement_matrices",
    "rt_matrix",
    "rt_rows",
    "discrete_gradient",
    "eliminate_bc",
    "discrete_curl",
    "lagrange_matrix",
    "interp_nodes",
    "evec_to_tvec",
    "csr_to_dense",
    "csr_to_scipy",
]

#: 2-point Gauss-Legendre abscissae on [0, 1]; each weight is 1/2.
GAUSS_T = (0.5 - 0.5 / math.sqrt(3.0), 0.5 + 0.5 / math.sqrt(3.0))


def _l(a: int, t: float) -> float:
    """1D linear Lagrange function on [0,1]: l_0(t) = 1 - t, l_1(t) = t."""
    return t if a == 1 else 1.0 - t


def _dl(a: int) -> float:
    return 1.0 if a == 1 else -1.0


def _quad_points():
    """The 8 tensor Gauss points q = q1 + 2 q2 + 4 q3 and weight 1/8 each."""
    pts = []
    for q3 in range(2):
        for q2 in range(2):
            for q1 in range(2):
                pts.append((GAUSS_T[q1], GAUSS_T[q2], GAUSS_T[q3]))
    return pts, 1.0 / 8.0


# ------------------------------------------------------------------------- H1

def _q1_reference():
    """Trilinear shape functions phi[q, v] and reference gradients g[q, v, c] at
    the Gauss points; vertex v = a + 2b + 4c sits at reference corner (a, b, c)."""
    pts, w = _quad_points()
    phi = torch.zeros(8, 8, dtype=torch.float64)
    grad = torch.zeros(8, 8, 3, dtype=torch.float64)
    for q, (x, y, z) in enumerate(pts):
        for v in range(8):
            a, b, c = v & 1, (v >> 1) & 1, (v >> 2) & 1
            phi[q, v] = _l(a, x) * _l(b, y) * _l(c, z)
            grad[q, v, 0] = _dl(a) * _l(b, y) * _l(c, z)
            grad[q, v, 1] = _l(a, x) * _dl(b) * _l(c, z)
            grad[q, v, 2] = _l(a, x) * _l(b, y) * _dl(c)
    return phi, grad, w


def h1_subelement_vertices(elem_dofs: torch.Tensor, p: int) -> torch.Tensor:
    """Global vertex ids [nel, p^3, 8] of every subelement (LOR mesh section):
    subelement s = i + p(j + p k) of element e has corner (a,b,c) at local
    lattice vertex (i+a) + (p+1)((j+b) + (p+1)(k+c))."""
    q = p + 1
    ed = torch.as_tensor(elem_dofs).to(torch.int64)
    idx = torch.empty(p ** 3, 8, dtype=torch.int64)
    for k in range(p):
        for j in range(p):
            for i in range(p):
                s = i + p * (j + p * k)
                for v in range(8):
                    a, b, c = v & 1, (v >> 1) & 1, (v >> 2) & 1
                    idx[s, v] = (i + a) + q * ((j + b) + q * (k + c))
    return ed[:, idx]


def h1_subelement_matrices(X: torch.Tensor, kappa: torch.Tensor, beta) -> torch.Tensor:
    """Q1 stiffness + mass of trilinear subelements, 2x2x2 Gauss.

    X: [S, 8, 3] vertex coordinates; kappa: [S]; beta: scalar or [S].
    Returns A^s = K^s + M^s, [S, 8, 8], with
      K_uv = sum_q w kappa det(J) (J^-T g_u).(J^-T g_v),
      M_uv = sum_q w beta  det(J) phi_u phi_v,
    J_rc = d x_r / d xi_c = sum_v X_v,r g_v,c.
    """
    phi, grad, w = _q1_reference()
    J = torch.einsum("svr,qvc->sqrc", X, grad)            # [S, 8, 3, 3]
    det = torch.linalg.det(J)                              # [S, 8]
    if bool((det <= 0).any()):
        raise ValueError("inverted LOR subelement (det J <= 0 at a quadrature point)")
    Jinv = torch.linalg.inv(J)
    gp = torch.einsum("qvr,sqrc->sqvc", grad, Jinv)        # physical gradients
    kap = torch.as_tensor(kappa, dtype=torch.float64)
    K = torch.einsum("sq,sqvc,squc->svu", w * det, gp, gp) * kap[:, None, None]
    bet = torch.as_tensor(beta, dtype=torch.float64)
    Mq = torch.einsum("qv,qu->qvu", phi, phi)              # [8, 8, 8]
    M = torch.einsum("sq,qvu->svu", w * det, Mq)
    M = M * (bet[:, None, None] if bet.dim() == 1 else bet)
    return K + M


# --------------------------------------------------------------------- H(curl)

def _nd_reference():
    """Lowest-order Nedelec reference basis N[q, a, 3] and curls C[q, a, 3] at the
    Gauss points.  Edge a: x-edges (b,c) -> b + 2c, y-edges (a,c) -> 4 + a + 2c,
    z-edges (a,b) -> 8 + a + 2b; each points along +axis and has unit tangential
    moment on its own edge."""
    pts, w = _quad_points()
    N = torch.zeros(8, 12, 3, dtype=torch.float64)
    C = torch.zeros(8, 12, 3, dtype=torch.float64)
    for q, (x, y, z) in enumerate(pts):
        for b in range(2):
            for c in range(2):
                n = b + 2 * c
                N[q, n, 0] = _l(b, y) * _l(c, z)
                C[q, n, 1] = _l(b, y) * _dl(c)
                C[q, n, 2] = -_dl(b) * _l(c, z)
        for a in range(2):
            for c in range(2):
                n = 4 + a + 2 * c
                N[q, n, 1] = _l(a, x) * _l(c, z)
                C[q, n, 0] = -_l(a, x) * _dl(c)
                C[q, n, 2] = _dl(a) * _l(c, z)
        for a in range(2):
            for b in range(2):
                n = 8 + a + 2 * b
                N[q, n, 2] = _l(a, x) * _l(b, y)
                C[q, n, 0] = _l(a, x) * _dl(b)
                C[q, n, 1] = -_dl(a) * _l(b, y)
    return N, C, w


def nd_subelement_edges(elem_edges: torch.Tensor, p: int):
    """Global edge ids and orientation signs [nel, p^3, 12] of every subelement."""
    q = p + 1
    ee = torch.as_tensor(elem_edges).to(torch.int64)
    idx = torch.empty(p ** 3, 12, dtype=torch.int64)
    ox, oy, oz = 0, p * q * q, 2 * p * q * q
    for k in range(p):
        for j in range(p):
            for i in range(p):
                s = i + p * (j + p * k)
                for b in range(2):
                    for c in range(2):
                        idx[s, b + 2 * c] = ox + i + p * ((j + b) + q * (k + c))
                for a in range(2):
                    for c in range(2):
                        idx[s, 4 + a + 2 * c] = oy + (i + a) + q * (j + p * (k + c))
                for a in range(2):
                    for b in range(2):
                        idx[s, 8 + a + 2 * b] = oz + (i + a) + q * ((j + b) + q * k)
    raw = ee[:, idx]
    sign = torch.where(raw < 0, -1.0, 1.0).to(torch.float64)
    gid = torch.where(raw < 0, -1 - raw, raw)
    return gid, sign


def nd_subelement_matrices(X: torch.Tensor, kappa: torch.Tensor, beta) -> torch.Tensor:
    """Lowest-order Nedelec curl-curl + mass of trilinear subelements, 2x2x2 Gauss,
    in the local (+axis) orientation.  Covariant Piola map: N = J^-T N_hat,
    curl N = J C_hat / det J.
      K_ab = sum_q w kappa det(J) curlN_a . curlN_b,
      M_ab = sum_q w beta  det(J) N_a . N_b.
    X: [S, 8, 3]; returns [S, 12, 12]."""
    _, grad, _ = _q1_reference()
    Nr, Cr, w = _nd_reference()
    J = torch.einsum("svr,qvc->sqrc", X, grad)
    det = torch.linalg.det(J)
    if bool((det <= 0).any()):
        raise ValueError("inverted LOR subelement (det J <= 0 at a quadrature point)")
    Jinv = torch.linalg.inv(J)
    Nphys = torch.einsum("qar,sqrc->sqac", Nr, Jinv)               # N_hat^T J^-1
    Cphys = torch.einsum("sqrc,qac->sqar", J, Cr) / det[:, :, None, None]
    kap = torch.as_tensor(kappa, dtype=torch.float64)
    bet = torch.as_tensor(beta, dtype=torch.float64)
    K = torch.einsum("sq,sqac,sqbc->sab", w * det, Cphys, Cphys) * kap[:, None, None]
    M = torch.einsum("sq,sqac,sqbc->sab", w * det, Nphys, Nphys)
    M = M * (bet[:, None, None] if bet.dim() == 1 else bet)
    return K + M


# ------------------------------------------------------------------ H1 in 2D

def _q1_reference_2d():
    """Bilinear shape functions phi[q, v] and reference gradients g[q, v, c] at
    the 2x2 Gauss points q = q1 + 2 q2 (weight 1/4); vertex v = a + 2b at
    reference corner (a, b)."""
    phi = torch.zeros(4, 4, dtype=torch.float64)
    grad = torch.zeros(4, 4, 2, dtype=torch.float64)
    for q2 in range(2):
        for q1 in range(2):
            q = q1 + 2 * q2
            x, y = GAUSS_T[q1], GAUSS_T[q2]
            for v in range(4):
                a, b = v & 1, v >> 1
                phi[q, v] = _l(a, x) * _l(b, y)
                grad[q, v, 0] = _dl(a) * _l(b, y)
                grad[q, v, 1] = _l(a, x) * _dl(b)
    return phi, grad, 0.25


def _coo_h1_2d(coords, elem_dofs, p, kappa, beta, elems=None):
    """The 2D variant of the LOR mesh and matrix (p x p bilinear subelements
    per quadrilateral macro element, Q1 diffusion + mass, 2x2 Gauss):
      K_uv = sum_q w kappa det(J) (J^-T g_u).(J^-T g_v),  M_uv = sum_q w beta det(J) phi_u phi_v."""
    X = _as_f64(coords)
    kap = _as_f64(kappa)
    ed = torch.as_tensor(elem_dofs).to(torch.int64)
    if elems is not None:
        elems = torch.as_tensor(elems, dtype=torch.int64)
        ed, kap = ed[elems], kap[elems]
    q = p + 1
    idx = torch.empty(p * p, 4, dtype=torch.int64)
    for j in range(p):
        for i in range(p):
            for v in range(4):
                a, b = v & 1, v >> 1
                idx[i + p * j, v] = (i + a) + q * (j + b)
    sv = ed[:, idx].reshape(-1, 4)
    Xs = X[sv]                                                   # [S, 4, 2]
    phi, grad, w = _q1_reference_2d()
    J = torch.einsum("svr,qvc->sqrc", Xs, grad)
    det = torch.linalg.det(J)
    if bool((det <= 0).any()):
        raise ValueError("inverted LOR subelement (det J <= 0 at a quadrature point)")
    Jinv = torch.linalg.inv(J)
    gp = torch.einsum("qvr,sqrc->sqvc", grad, Jinv)
    K = torch.einsum("sq,sqvc,squc->svu", w * det, gp, gp) * kap.reshape(-1)[:, None, None]
    M = torch.einsum("sq,qv,qu->svu", w * det, phi, phi) * float(beta)
    A = K + M
    R = sv[:, :, None].expand(-1, 4, 4).reshape(-1)
    C = sv[:, None, :].expand(-1, 4, 4).reshape(-1)
    return R, C, A.reshape(-1)


def h1_matrix_2d(coords, elem_dofs, p: int, kappa, beta, ndofs: int | None = None):
    """Assembled 2D LOR H1 matrix in CSR (9 nonzeros per interior row)."""
    R, C, V = _coo_h1_2d(coords, elem_dofs, p, kappa, beta)
    n = int(ndofs) if ndofs is not None else int(torch.as_tensor(coords).shape[0])
    return coo_to_csr(R, C, V, n)


def h1_rows_2d(coords, elem_dofs, p: int, kappa, beta, rows):
    """The listed rows of the 2D LOR H1 matrix (same definition as h1_matrix_2d)."""
    rows = torch.unique(torch.as_tensor(rows, dtype=torch.int64))
    ed = torch.as_tensor(elem_dofs).to(torch.int64)
    elems = _elements_touching(ed, rows)
    R, C, V = _coo_h1_2d(coords, elem_dofs, p, kappa, beta, elems=elems)
    keep = torch.isin(R, rows)
    R, C, V = R[keep], C[keep], V[keep]
    pos = torch.searchsorted(rows, R)
    stride = int(C.max().item()) + 1 if C.numel() else 1
    key = pos * stride + C
    order = torch.argsort(key, stable=True)
    uniq, inverse = torch.unique_consecutive(key[order], return_inverse=True)
    values = torch.zeros(uniq.numel(), dtype=torch.float64).index_add(0, inverse, V[order])
    r = uniq // stride
    col_idx = uniq - r * stride
    counts = torch.bincount(r, minlength=rows.numel())
    row_ptr = torch.zeros(rows.numel() + 1, dtype=torch.int64)
    row_ptr[1:] = torch.cumsum(counts, 0)
    return rows, row_ptr, col_idx, values


# --------------------------------------------------------------------- H(div)

def _rt_reference():
    """Lowest-order Raviart-Thomas reference basis R[q, a, 3] and divergences
    D[a] at the Gauss points.  Face a: x-faces (xi = a0) -> a0, y-faces
    (eta = b) -> 2 + b, z-faces (zeta = c) -> 4 + c; each has unit flux through
    its own face with the +axis normal and none through the others:
    x-face a0: (l_a0(xi), 0, 0), divergence l_a0' = +-1, and cyclically."""
    pts, w = _quad_points()
    R = torch.zeros(8, 6, 3, dtype=torch.float64)
    D = torch.zeros(6, dtype=torch.float64)
    for q, (x, y, z) in enumerate(pts):
        for t in range(2):
            R[q, t, 0] = _l(t, x)
            R[q, 2 + t, 1] = _l(t, y)
            R[q, 4 + t, 2] = _l(t, z)
    for t in range(2):
        D[t] = D[2 + t] = D[4 + t] = _dl(t)
    return R, D, w


def rt_subelement_faces(elem_faces: torch.Tensor, p: int):
    """Global face ids and orientation signs [nel, p^3, 6] of every subelement
    (local faces as in the input generator's face map)."""
    q = p + 1
    fm = torch.as_tensor(elem_faces).to(torch.int64)
    idx = torch.empty(p ** 3, 6, dtype=torch.int64)
    ox, oy, oz = 0, p * p * q, 2 * p * p * q
    for k in range(p):
        for j in range(p):
            for i in range(p):
                s = i + p * (j + p * k)
                for t in range(2):
                    idx[s, t] = ox + (i + t) + q * (j + p * k)
                    idx[s, 2 + t] = oy + i + p * ((j + t) + q * k)
                    idx[s, 4 + t] = oz + i + p * (j + p * (k + t))
    raw = fm[:, idx]
    sign = torch.where(raw < 0, -1.0, 1.0).to(torch.float64)
    gid = torch.where(raw < 0, -1 - raw, raw)
    return gid, sign


def rt_subelement_matrices(X: torch.Tensor, kappa: torch.Tensor, beta) -> torch.Tensor:
    """Lowest-order Raviart-Thomas div-div + mass of trilinear subelements,
    2x2x2 Gauss, in the local (+axis) orientation.  Contravariant Piola map:
    N = J R_hat / det J, div N = D_hat / det J.
      K_ab = sum_q w kappa det(J) divN_a divN_b,
      M_ab = sum_q w beta  det(J) N_a . N_b.
    X: [S, 8, 3]; returns [S, 6, 6]."""
    _, grad, _ = _q1_reference()
    Rr, Dr, w = _rt_reference()
    J = torch.einsum("svr,qvc->sqrc", X, grad)
    det = torch.linalg.det(J)
    if bool((det <= 0).any()):
        raise ValueError("inverted LOR subelement (det J <= 0 at a quadrature point)")
    Nphys = torch.einsum("sqrc,qac->sqar", J, Rr) / det[:, :, None, None]
    Dphys = Dr[None, None, :] / det[:, :, None]
    kap = torch.as_tensor(kappa, dtype=torch.float64)
    bet = torch.as_tensor(beta, dtype=torch.float64)
    K = torch.einsum("sq,sqa,sqb->sab", w * det, Dphys, Dphys) * kap[:, None, None]
    M = torch.einsum("sq,sqac,sqbc->sab", w * det, Nphys, Nphys)
    M = M * (bet[:, None, None] if bet.dim() == 1 else bet)
    return K + M


def _coo_rt(coords, elem_dofs, elem_faces, p, kappa, beta, elems=None, chunk=4096):
    coords = _as_f64(coords)
    kappa = _as_f64(kappa)
    ed = torch.as_tensor(elem_dofs)
    fm = torch.as_tensor(elem_faces)
    if elems is not None:
        elems = torch.as_tensor(elems, dtype=torch.int64)
        ed, fm, kappa = ed[elems], fm[elems], kappa[elems]
        if isinstance(beta, torch.Tensor) and beta.dim() > 0:
            beta = beta[elems]
    R, C, V = [], [], []
    nel = ed.shape[0]
    for e0 in range(0, nel, chunk):
        e1 = min(nel, e0 + chunk)
        sv = h1_subelement_vertices(ed[e0:e1], p).reshape(-1, 8)
        gid, sg = rt_subelement_faces(fm[e0:e1], p)
        gid = gid.reshape(-1, 6)
        sg = sg.reshape(-1, 6)
        X = coords[sv]
        kap = kappa[e0:e1].reshape(-1)
        bet = beta[e0:e1].reshape(-1) if (isinstance(beta, torch.Tensor) and beta.dim() > 0) else beta
        A = rt_subelement_matrices(X, kap, bet) * (sg[:, :, None] * sg[:, None, :])
        R.append(gid[:, :, None].expand(-1, 6, 6).reshape(-1))
        C.append(gid[:, None, :].expand(-1, 6, 6).reshape(-1))
        V.append(A.reshape(-1))
    return torch.cat(R), torch.cat(C), torch.cat(V)


def rt_matrix(coords, elem_dofs, elem_faces, p: int, kappa, beta, nfaces: int):
    """Assembled LOR H(div) matrix (kappa div-div + beta mass) in CSR; rows and
    columns are global faces with the orientation given by the sign of the
    signed face map (the lowest-order Raviart-Thomas element on the refined
    mesh, the lowest-order interpolation-histopolation case)."""
    R, C, V = _coo_rt(coords, elem_dofs, elem_faces, p, kappa, beta)
    return coo_to_csr(R, C, V, nfaces)


def rt_rows(coords, elem_dofs, elem_faces, p: int, kappa, beta, rows):
    """The listed rows of the H(div) LOR matrix (same definition as rt_matrix)."""
    rows = torch.unique(torch.as_tensor(rows, dtype=torch.int64))
    fm = torch.as_tensor(elem_faces).to(torch.int64)
    gid = torch.where(fm < 0, -1 - fm, fm)
    elems = _elements_touching(gid, rows)
    R, C, V = _coo_rt(coords, elem_dofs, elem_faces, p, kappa, beta, elems=elems)
    keep = torch.isin(R, rows)
    R, C, V = R[keep], C[keep], V[keep]
    pos = torch.searchsorted(rows, R)
    stride = int(C.max().item()) + 1 if C.numel() else 1
    key = pos * stride + C
    order = torch.argsort(key, stable=True)
    ks = key[order]
    uniq, inverse = torch.unique_consecutive(ks, return_inverse=True)
    values = torch.zeros(uniq.numel(), dtype=torch.float64).index_add(0, inverse, V[order])
    r = uniq // stride
    col_idx = uniq - r * stride
    counts = torch.bincount(r, minlength=rows.numel())
    row_ptr = torch.zeros(rows.numel() + 1, dtype=torch.int64)
    row_ptr[1:] = torch.cumsum(counts, 0)
    return rows, row_ptr, col_idx, values


# ------------------------------------------------------------------ assembly

def coo_to_csr(rows: torch.Tensor, cols: torch.Tensor, vals: torch.Tensor, nrows: int):
    """Sum duplicate (row, col) entries: stable sort by row*nrows + col, unique
    keys become the pattern, values are segment sums (index_add_, differentiable).
    Returns row_ptr [nrows+1] int64, col_idx [nnz] int64, values [nnz] float64."""
    key = rows.to(torch.int64) * int(nrows) + cols.to(torch.int64)
    order = torch.argsort(key, stable=True)
    ks = key[order]
    uniq, inverse = torch.unique_consecutive(ks, return_inverse=True)
    values = torch.zeros(uniq.numel(), dtype=torch.float64)
    values = values.index_add(0, inverse, vals[order])
    r = uniq // int(nrows)
    col_idx = uniq - r * int(nrows)
    counts = torch.bincount(r, minlength=int(nrows))
    row_ptr = torch.zeros(int(nrows) + 1, dtype=torch.int64)
    row_ptr[1:] = torch.cumsum(counts, 0)
    return row_ptr, col_idx, values


def _as_f64(x) -> torch.Tensor:
    if isinstance(x, torch.Tensor):
        return x if x.dtype == torch.float64 else x.to(torch.float64)
    return torch.as_tensor(x, dtype=torch.float64)


def _coo_h1(coords, elem_dofs, p, kappa, beta, elems=None, chunk=4096):
    coords = _as_f64(coords)
    kappa = _as_f64(kappa)
    ed = torch.as_tensor(elem_dofs)
    if elems is not None:
        elems = torch.as_tensor(elems, dtype=torch.int64)
        ed = ed[elems]
        kappa = kappa[elems]
        if isinstance(beta, torch.Tensor) and beta.dim() > 0:
            beta = beta[elems]
    R, C, V = [], [], []
    nel = ed.shape[0]
    for e0 in range(0, nel, chunk):
        e1 = min(nel, e0 + chunk)
        sv = h1_subelement_vertices(ed[e0:e1], p).reshape(-1, 8)
        X = coords[sv]                                          # [S, 8, 3]
        kap = kappa[e0:e1].reshape(-1)
        bet = beta[e0:e1].reshape(-1) if (isinstance(beta, torch.Tensor) and beta.dim() > 0) else beta
        A = h1_subelement_matrices(X, kap, bet)                # [S, 8, 8]
        R.append(sv[:, :, None].expand(-1, 8, 8).reshape(-1))
        C.append(sv[:, None, :].expand(-1, 8, 8).reshape(-1))
        V.append(A.reshape(-1))
    return torch.cat(R), torch.cat(C), torch.cat(V)


def h1_matrix(coords, elem_dofs, p: int, kappa, beta, ndofs: int | None = None):
    """Assembled LOR H1 matrix (kappa-diffusion + beta-mass) in CSR.

    coords [ndofs, 3] float64, elem_dofs [nel, (p+1)^3], kappa [nel, p^3],
    beta scalar (or [nel, p^3]).  Returns (row_ptr, col_idx, values)."""
    coords = _as_f64(coords)
    nd = coords.shape[0] if ndofs is None else ndofs
    R, C, V = _coo_h1(coords, elem_dofs, p, kappa, beta)
    return coo_to_csr(R, C, V, nd)


def _elements_touching(elem_ids: torch.Tensor, rows: torch.Tensor) -> torch.Tensor:
    hit = torch.isin(elem_ids, rows).any(dim=1)
    return torch.nonzero(hit).reshape(-1)


def h1_rows(coords, elem_dofs, p: int, kappa, beta, rows):
    """The listed rows of the H1 LOR matrix, computed from only the subelements
    that touch them (same definition as h1_matrix).  Returns, for the sorted
    unique rows, (rows, row_ptr, col_idx, values)."""
    rows = torch.unique(torch.as_tensor(rows, dtype=torch.int64))
    ed = torch.as_tensor(elem_dofs).to(torch.int64)
    elems = _elements_touching(ed, rows)
    R, C, V = _coo_h1(coords, ed, p, kappa, beta, elems=elems)
    keep = torch.isin(R, rows)
    R, C, V = R[keep], C[keep], V[keep]
    pos = torch.searchsorted(rows, R)
    # key on (row position, global column); columns range over all vertices
    stride = int(C.max().item()) + 1 if C.numel() else 1
    key = pos * stride + C
    order = torch.argsort(key, stable=True)
    ks = key[order]
    uniq, inverse = torch.unique_consecutive(ks, return_inverse=True)
    values = torch.zeros(uniq.numel(), dtype=torch.float64).index_add(0, inverse, V[order])
    r = uniq // stride
    col_idx = uniq - r * stride
    counts = torch.bincount(r, minlength=rows.numel())
    row_ptr = torch.zeros(rows.numel() + 1, dtype=torch.int64)
    row_ptr[1:] = torch.cumsum(counts, 0)
    return rows, row_ptr, col_idx, values


def _coo_nd(coords, elem_dofs, elem_edges, p, kappa, beta, elems=None, chunk=4096):
    coords = _as_f64(coords)
    kappa = _as_f64(kappa)
    ed = torch.as_tensor(elem_dofs)
    ee = torch.as_tensor(elem_edges)
    if elems is not None:
        elems = torch.as_tensor(elems, dtype=torch.int64)
        ed, ee, kappa = ed[elems], ee[elems], kappa[elems]
        if isinstance(beta, torch.Tensor) and beta.dim() > 0:
            beta = beta[elems]
    R, C, V = [], [], []
    nel = ed.shape[0]
    for e0 in range(0, nel, chunk):
        e1 = min(nel, e0 + chunk)
        sv = h1_subelement_vertices(ed[e0:e1], p).reshape(-1, 8)
        gid, sg = nd_subelement_edges(ee[e0:e1], p)
        gid = gid.reshape(-1, 12)
        sg = sg.reshape(-1, 12)
        X = coords[sv]
        kap = kappa[e0:e1].reshape(-1)
        bet = beta[e0:e1].reshape(-1) if (isinstance(beta, torch.Tensor) and beta.dim() > 0) else beta
        A = nd_subelement_matrices(X, kap, bet) * (sg[:, :, None] * sg[:, None, :])
        R.append(gid[:, :, None].expand(-1, 12, 12).reshape(-1))
        C.append(gid[:, None, :].expand(-1, 12, 12).reshape(-1))
        V.append(A.reshape(-1))
    return torch.cat(R), torch.cat(C), torch.cat(V)


def nd_matrix(coords, elem_dofs, elem_edges, p: int, kappa, beta, nedges: int):
    """Assembled LOR H(curl) matrix (kappa curl-curl + beta mass) in CSR; rows and
    columns are global edges with the orientation given by the sign of the signed
    edge map."""
    R, C, V = _coo_nd(coords, elem_dofs, elem_edges, p, kappa, beta)
    return coo_to_csr(R, C, V, nedges)


def nd_rows(coords, elem_dofs, elem_edges, p: int, kappa, beta, rows):
    """The listed rows of the H(curl) LOR matrix (same definition as nd_matrix)."""
    rows = torch.unique(torch.as_tensor(rows, dtype=torch.int64))
    ee = torch.as_tensor(elem_edges).to(torch.int64)
    gid = torch.where(ee < 0, -1 - ee, ee)
    elems = _elements_touching(gid, rows)
    R, C, V = _coo_nd(coords, elem_dofs, elem_edges, p, kappa, beta, elems=elems)
    keep = torch.isin(R, rows)
    R, C, V = R[keep], C[keep], V[keep]
    pos = torch.searchsorted(rows, R)
    stride = int(C.max().item()) + 1 if C.numel() else 1
    key = pos * stride + C
    order = torch.argsort(key, stable=True)
    ks = key[order]
    uniq, inverse = torch.unique_consecutive(ks, return_inverse=True)
    values = torch.zeros(uniq.numel(), dtype=torch.float64).index_add(0, inverse, V[order])
    r = uniq // stride
    col_idx = uniq - r * stride
    counts = torch.bincount(r, minlength=rows.numel())
    row_ptr = torch.zeros(rows.numel() + 1, dtype=torch.int64)
    row_ptr[1:] = torch.cumsum(counts, 0)
    return rows, row_ptr, col_idx, values


# ------------------------------------------------------- auxiliary: gradient

def discrete_gradient(elem_dofs, elem_edges, p: int, nedges: int):
    """Discrete gradient (vertices -> edges) of the LOR mesh in CSR, as in the
    algorithm for the discrete gradient matrix (auxiliary computations of Step
    S1.2): row i (an edge) has I[i] = 2i, J = (first vertex, second vertex) of
    its local edge, A = (-sigma, +sigma) with sigma the orientation sign.
    Returns (row_ptr, col_idx, values) with 2 entries per row (col order as
    defined, not sorted).  The algorithm takes each edge from one element (its
    element map and local index); here that is the edge's first incidence, the
    lowest element and then the lowest local edge.  The row is the same sparse
    vector whichever element supplies it; only the order of its two entries
    can differ where elements are reoriented."""
    q = p + 1
    ed = torch.as_tensor(elem_dofs).to(torch.int64)
    ee = torch.as_tensor(elem_edges).to(torch.int64)
    nloc = 3 * p * q * q
    v0 = torch.empty(nloc, dtype=torch.int64)
    v1 = torch.empty(nloc, dtype=torch.int64)
    n = 0
    for ax, (nx, ny, nz) in enumerate([(p, q, q), (q, p, q), (q, q, p)]):
        for k in range(nz):
            for j in range(ny):
                for i in range(nx):
                    a = [i, j, k]
                    b = [i, j, k]
                    b[ax] += 1
                    v0[n] = a[0] + q * (a[1] + q * a[2])
                    v1[n] = b[0] + q * (b[1] + q * b[2])
                    n += 1
    raw = ee.reshape(-1)
    gid = torch.where(raw < 0, -1 - raw, raw)
    flat = torch.arange(gid.numel())
    none = gid.numel()
    first = torch.full((nedges,), none, dtype=torch.int64).scatter_reduce(0, gid, flat, reduce="amin")
    if bool((first == none).any()):
        raise ValueError("edge map does not cover every edge")
    e, l = first // nloc, first % nloc
    sig = torch.where(raw[first] < 0, -1.0, 1.0).to(torch.float64)
    J = torch.stack([ed[e, v0[l]], ed[e, v1[l]]], dim=1)
    A = torch.stack([-sig, sig], dim=1)
    row_ptr = torch.arange(0, 2 * nedges + 1, 2, dtype=torch.int64)
    return row_ptr, J.reshape(-1), A.reshape(-1)


# ------------------------------------------------------- auxiliary: curl

def _local_face_edges(p: int):
    """For every local face of a degree-p macro element, its 4 local edges and
    the sign of each in the face's boundary circulation (right-hand rule about
    the face normal, which points along +axis): x-face boundary runs +y, +z,
    -y, -z; y-face +z, +x, -z, -x; z-face +x, +y, -x, -y (Stokes: the flux of
    curl u through the face is the circulation of u around it)."""
    q = p + 1

    def xe(i, j, k):
        return i + p * (j + q * k)

    def ye(i, j, k):
        return p * q * q + i + q * (j + p * k)

    def ze(i, j, k):
        return 2 * p * q * q + i + q * (j + q * k)

    out = []
    for k in range(p):
        for j in range(p):
            for i in range(q):
                out.append([(ye(i, j, k), 1), (ze(i, j + 1, k), 1), (ye(i, j, k + 1), -1), (ze(i, j, k), -1)])
    for k in range(p):
        for j in range(q):
            for i in range(p):
                out.append([(ze(i, j, k), 1), (xe(i, j, k + 1), 1), (ze(i + 1, j, k), -1), (xe(i, j, k), -1)])
    for k in range(q):
        for j in range(p):
            for i in range(p):
                out.append([(xe(i, j, k), 1), (ye(i + 1, j, k), 1), (xe(i, j + 1, k), -1), (ye(i, j, k), -1)])
    return out


def discrete_curl(elem_edges, elem_faces, p: int, nfaces: int):
    """Discrete curl (LOR edges -> LOR faces) in CSR (auxiliary computations of
    Step S1.2): row f (a face) has 4 entries, one per edge of the face, equal
    to sigma_f * sigma_e * s, with s the edge's sign in the face circulation on
    the reference macro element and sigma_f, sigma_e the orientation signs of
    the signed face and edge maps.  As for the gradient, each face is taken
    from its first incidence (lowest element, then lowest local face); the
    entries keep the local circulation order (+, +, -, - before the signs).
    Returns (row_ptr, col_idx, values)."""
    fe = torch.as_tensor(elem_faces).to(torch.int64)
    ee = torch.as_tensor(elem_edges).to(torch.int64)
    nlocf = fe.shape[1]
    tab = _local_face_edges(p)
    if len(tab) != nlocf:
        raise ValueError("face map does not match p")
    le = torch.tensor([[t[0] for t in row] for row in tab], dtype=torch.int64)   # [nlocf, 4]
    ls = torch.tensor([[t[1] for t in row] for row in tab], dtype=torch.float64)
    raw = fe.reshape(-1)
    gid = torch.where(raw < 0, -1 - raw, raw)
    flat = torch.arange(gid.numel())
    none = gid.numel()
    first = torch.full((nfaces,), none, dtype=torch.int64).scatter_reduce(0, gid, flat, reduce="amin")
    if bool((first == none).any()):
        raise ValueError("face map does not cover every face")
    e, lf = first // nlocf, first % nlocf
    sf = torch.where(raw[first] < 0, -1.0, 1.0).to(torch.float64)
    eraw = ee[e[:, None], le[lf]]                                                 # [nfaces, 4]
    J = torch.where(eraw < 0, -1 - eraw, eraw)
    se = torch.where(eraw < 0, -1.0, 1.0).to(torch.float64)
    A = sf[:, None] * se * ls[lf]
    row_ptr = torch.arange(0, 4 * nfaces + 1, 4, dtype=torch.int64)
    return row_ptr, J.reshape(-1), A.reshape(-1)


# ------------------------------------------ auxiliary: LOR coordinate vector

def lagrange_matrix(src, dst) -> torch.Tensor:
    """B[a][i] = l_i(dst[a]), l_i the Lagrange polynomial of the points `src`
    (l_i(src[m]) = delta_im), written as the product formula."""
    src = [float(t) for t in src]
    dst = [float(t) for t in dst]
    B = torch.empty(len(dst), len(src), dtype=torch.float64)
    for a, x in enumerate(dst):
        for i, xi in enumerate(src):
            v = 1.0
            for m, xm in enumerate(src):
                if m != i:
                    v *= (x - xm) / (xi - xm)
            B[a, i] = v
    return B


def interp_nodes(nodes, p: int, q: int) -> torch.Tensor:
    """Coordinates of the LOR vertices of every element as an E-vector
    (auxiliary computations of Step S1.2 and the coordinate-vector results of
    Section 4): the high-order mesh of degree q, given by its nodes at the
    tensor Gauss-Lobatto points of degree q, is evaluated at the tensor
    Gauss-Lobatto lattice of degree p with the tensor-product Lagrange basis,
    X_out[e][a + (p+1)(b + (p+1)c)] = sum_ijk l_i(x_a) l_j(x_b) l_k(x_c) X[e][i + (q+1)(j + (q+1)k)].
    nodes [nel][(q+1)^3][ncomp] -> [nel][(p+1)^3][ncomp], float64."""
    import meshgen  # the point sets are those that define the inputs
    X = torch.as_tensor(nodes, dtype=torch.float64)
    nel, _, nc = X.shape
    B = lagrange_matrix(meshgen.gll_points(q), meshgen.gll_points(p))
    X = X.reshape(nel, q + 1, q + 1, q + 1, nc)  # [e][k][j][i][comp]
    out = torch.einsum("ai,bj,ck,ekjid->ecbad", B, B, B, X)
    return out.reshape(nel, (p + 1) ** 3, nc)


def evec_to_tvec(evec, elem_map, ndofs: int) -> torch.Tensor:
    """E-vector -> T-vector (deduplication with the element restriction map,
    one value per degree of freedom): every dof takes the value of its first
    incidence, the lowest element and then the lowest local index.
    evec [nel][nloc][ncomp], elem_map [nel][nloc] -> [ndofs][ncomp]."""
    E = torch.as_tensor(evec, dtype=torch.float64)
    nc = E.shape[-1]
    g = torch.as_tensor(elem_map).to(torch.int64).reshape(-1)
    flat = torch.arange(g.numel())
    none = g.numel()
    first = torch.full((ndofs,), none, dtype=torch.int64).scatter_reduce(0, g, flat, reduce="amin")
    if bool((first == none).any()):
        raise ValueError("element map does not cover every dof")
    return E.reshape(-1, nc)[first]


# ------------------------------------------------- boundary-condition elimination

DIAG_POLICIES = ("one", "keep", "zero")


def eliminate_bc(row_ptr, col_idx, values, ess, diag_policy: str = "one", rows=None):
    """Step A4 of the processor-local assembly (Section 3, Step S1.2), one
    process: the rows and the columns of the essential degrees of freedom are
    eliminated, i.e. every entry (r, c) with r or c essential becomes 0, except
    the diagonal entry (i, i) of an essential i, which becomes 1 ("one", the
    usual choice the paper names), keeps its value ("keep") or becomes 0
    ("zero").  The essential set is held as a Boolean marker over the
    degrees of freedom, as in the paper.

    row_ptr, col_idx: CSR arrays; values [nnz] or [batch, nnz]; ess: indices of
    the essential dofs (duplicates allowed, each must lie in [0, n)); rows: the
    global row id of each CSR row, for a block of sampled rows (default
    0..n-1).  The marker has n = len(row_ptr) - 1 entries, or, with rows given,
    one more than the largest row, column or essential index.
    Returns (eliminated values, marker)."""
    row_ptr = torch.as_tensor(row_ptr).to(torch.int64)
    col_idx = torch.as_tensor(col_idx).to(torch.int64)
    values = torch.as_tensor(values)
    ess = torch.as_tensor(ess).to(torch.int64).reshape(-1)
    if diag_policy not in DIAG_POLICIES:
        raise ValueError(f"diag_policy must be one of {DIAG_POLICIES}")
    nloc = row_ptr.numel() - 1
    if rows is None:
        rows = torch.arange(nloc)
        n = nloc
    else:
        rows = torch.as_tensor(rows).to(torch.int64)
        n = int(max(rows.max().item() if rows.numel() else -1, col_idx.max().item() if col_idx.numel() else -1,
                    ess.max().item() if ess.numel() else -1)) + 1
    if ess.numel() and (int(ess.min()) < 0 or int(ess.max()) >= n):
        raise IndexError("essential dof outside [0, n)")
    marker = torch.zeros(n, dtype=torch.bool)
    marker[ess] = True
    r = torch.repeat_interleave(rows, row_ptr[1:] - row_ptr[:-1])
    hit = marker[r] | marker[col_idx]
    on_diag = r == col_idx
    out = values.clone()
    out[..., hit & ~on_diag] = 0
    if diag_policy == "one":
        out[..., hit & on_diag] = 1
    elif diag_policy == "zero":
        out[..., hit & on_diag] = 0
    return out, marker


# ---------------------------------------------------------------- utilities

def csr_to_dense(row_ptr, col_idx, values, ncols: int | None = None) -> torch.Tensor:
    n = row_ptr.numel() - 1
    m = n if ncols is None else ncols
    rows = torch.repeat_interleave(torch.arange(n), row_ptr[1:] - row_ptr[:-1])
    D = torch.zeros(n, m, dtype=values.dtype)
    D.index_put_((rows, col_idx.to(torch.int64)), values, accumulate=True)
    return D


def csr_to_scipy(row_ptr, col_idx, values, ncols: int | None = None):
    import scipy.sparse as sp
    n = row_ptr.numel() - 1
    m = n if ncols is None else ncols
    return sp.csr_matrix((values.detach().numpy(), col_idx.numpy(), row_ptr.numpy()), shape=(n, m))
