"""Pins of the CPU oracle against what the paper and the mathematics fix.

Each test derives its expected value by a route that does not go through the
oracle's code: lattice counting with 1D element matrices, conservation laws
(partition of unity, exact volumes), exactness of the 2-point rule on affine
cells, an independent dense brute-force assembly, the de Rham exact sequence,
and the paper's printed pattern counts.  A dropped term, a wrong sign or index
or a transposed Jacobian in the oracle fails at least one of them.
"""
import itertools
import json
import math
import os

import numpy as np
import pytest
import torch

import meshgen
from oracle import lor_oracle as orc

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def dense(rp, ci, v, n=None):
    return orc.csr_to_dense(rp, ci, v, n).numpy()


def lattice_xyz(g, N):
    g = np.asarray(g, dtype=np.int64)
    return np.stack([g % N, (g // N) % N, g // (N * N)], axis=-1)


# ----------------------------------------------------------- closed forms (C1)

def _expected_uniform(N, h, kind):
    """Assembled Q1 matrix on a uniform lattice of N^3 points, spacing h, from
    lattice counting: entry (i, j) = (#cells holding both) x (cell-matrix entry
    for the pair), with the cell matrix built from 1D linear element matrices
    S = [[1,-1],[-1,1]]/h and M = h/6 [[2,1],[1,2]] by tensor products."""
    S1 = np.array([[1.0, -1.0], [-1.0, 1.0]]) / h
    M1 = h / 6.0 * np.array([[2.0, 1.0], [1.0, 2.0]])
    if kind == "K":
        cell = (np.kron(np.kron(M1, M1), S1) + np.kron(np.kron(M1, S1), M1)
                + np.kron(np.kron(S1, M1), M1))
    else:
        cell = np.kron(np.kron(M1, M1), M1)
    # kron order puts the x-index fastest: corner v = a + 2b + 4c
    n = N ** 3
    A = np.zeros((n, n))
    for cz, cy, cx in itertools.product(range(N - 1), repeat=3):
        ids = []
        for c, b, a in itertools.product(range(2), repeat=3):
            ids.append((cx + a) + N * ((cy + b) + N * (cz + c)))
        ids = np.array(ids)
        # ids enumerated with a fastest within (c, b, a) loops -> v = a + 2b + 4c
        A[np.ix_(ids, ids)] += cell
    return A


@pytest.mark.parametrize("kind", ["K", "M"])
def test_uniform_cube_closed_form(kind):
    """C1 (4^3 hexes, p=2, undistorted): every row, boundary rows included."""
    m = meshgen.cartesian_mesh(4, 2, 0.0)
    N = m["N"]
    h = 1.0 / (N - 1)
    kap = torch.ones(m["nel"], 8, dtype=torch.float64) * (1.0 if kind == "K" else 0.0)
    beta = 0.0 if kind == "K" else 1.0
    rp, ci, v = orc.h1_matrix(m["coords"], m["elem_dofs"], 2, kap, beta)
    assert rp[-1].item() == (3 * N - 2) ** 3
    A = dense(rp, ci, v)
    E = _expected_uniform(N, h, kind)
    scale = np.abs(E).max()
    assert np.abs(A - E).max() <= 1e-14 * scale
    # interior stencil values quoted in the plan: 8h/3, 0, -h/6, -h/12
    if kind == "K":
        g = 4 + N * (4 + N * 4)
        row = {tuple(lattice_xyz(c, N) - lattice_xyz(g, N)): A[g, c] for c in np.nonzero(E[g])[0]}
        assert abs(A[g, g] - 8 * h / 3) < 1e-15
        assert abs(row[(1, 1, 0)] + h / 6) < 1e-15
        assert abs(row[(1, 1, 1)] + h / 12) < 1e-15
        assert abs(A[g, g + 1]) < 1e-15


# ------------------------------------------------------- conservation / exactness

def test_diffusion_row_sums_vanish():
    m = meshgen.cartesian_mesh(3, 3, 0.18)         # strongly curved (A = 0.06)
    kap = meshgen.kappa_field(m["nel"], 3, 2.0, seed=3)
    rp, ci, v = orc.h1_matrix(m["coords"], m["elem_dofs"], 3, kap, 0.0)
    A = orc.csr_to_scipy(rp, ci, v)
    rs = np.abs(np.asarray(A.sum(axis=1)).ravel())
    rmax = np.asarray(abs(A).max(axis=1).todense()).ravel()
    assert (rs <= 1e-14 * rmax).all()


def test_symmetry():
    m = meshgen.cartesian_mesh(3, 3, 0.18)
    kap = meshgen.kappa_field(m["nel"], 3, 1.0, seed=4)
    rp, ci, v = orc.h1_matrix(m["coords"], m["elem_dofs"], 3, kap, 1.0)
    A = orc.csr_to_scipy(rp, ci, v)
    D = abs(A - A.T).max()
    assert D <= 1e-15 * abs(A).max()
    # pattern is structurally symmetric
    assert (A != 0).nnz == (A.T != 0).nnz


@pytest.mark.parametrize("n,p,amp", [(4, 4, 0.1), (3, 5, 0.18), (2, 6, 0.12)])
def test_mass_total_is_domain_volume(n, p, amp):
    """Sum of all mass entries = volume of the union of trilinear subelements.
    The sinusoidal map moves each face of the unit cube only along its normal,
    by a bump whose trapezoid-weighted lattice sum vanishes (lattice symmetric
    about 1/2), so that union has volume exactly 1."""
    m = meshgen.cartesian_mesh(n, p, amp)
    kap = torch.zeros(m["nel"], p ** 3, dtype=torch.float64)
    rp, ci, v = orc.h1_matrix(m["coords"], m["elem_dofs"], p, kap, 1.0)
    assert abs(v.sum().item() - 1.0) <= 1e-13


def _affine():
    A = np.array([[1.3, 0.4, -0.2], [0.1, 0.9, 0.3], [-0.25, 0.2, 1.1]])
    t = np.array([0.3, -0.7, 1.9])
    return A, t


@pytest.mark.parametrize("p", [2, 3])
def test_affine_energy(p):
    """On parallelepiped cells the 2-point rule is exact for |grad u|^2 and u^2
    with u affine: U^T K U = |a|^2 sum_s kappa_s vol_s and
    U^T M U = beta * int (a.x + c)^2."""
    n = 2
    Am, t = _affine()
    m = meshgen.affine_mesh(n, p, Am, t)
    kap = meshgen.kappa_field(m["nel"], p, 1.0, seed=7)
    a = np.array([0.7, -1.1, 0.4])
    c = 0.35
    X = m["coords"]
    U = torch.from_numpy(X @ a + c)
    detA = np.linalg.det(Am)
    # subelement volumes from the lattice spacings
    tt = meshgen.gll_points(p)
    dt = np.diff(tt) / n
    vol = np.einsum("i,j,k->kji", dt, dt, dt).reshape(-1) * detA   # s = i + p(j + p k)
    rp, ci, v = orc.h1_matrix(X, m["elem_dofs"], p, kap, 0.0)
    K = orc.csr_to_scipy(rp, ci, v)
    want = float(a @ a) * float((kap.numpy() * vol[None, :]).sum())
    got = float(U.numpy() @ (K @ U.numpy()))
    assert abs(got - want) <= 1e-12 * abs(want)
    beta = 2.5
    rp, ci, v = orc.h1_matrix(X, m["elem_dofs"], p, torch.zeros_like(kap), beta)
    M = orc.csr_to_scipy(rp, ci, v)
    alpha = Am.T @ a
    gamma = float(a @ t) + c
    integral = detA * ((alpha.sum() / 2 + gamma) ** 2 + float(alpha @ alpha) / 12.0)
    got = float(U.numpy() @ (M @ U.numpy()))
    assert abs(got - beta * integral) <= 1e-12 * abs(beta * integral)


# ------------------------------------------------------------ brute force (p=2)

def _brute_force_dense(coords, elem_dofs, p, kappa, beta, npts):
    """Independent dense assembly: explicit loops over subelements, quadrature
    points and vertex pairs, Jacobian from explicit shape derivatives, physical
    gradients by solving J^T y = grad_ref."""
    xg, wg = np.polynomial.legendre.leggauss(npts)
    xg = 0.5 * (xg + 1.0)
    wg = 0.5 * wg
    q = p + 1
    nd = coords.shape[0]
    A = np.zeros((nd, nd))
    corners = [(a, b, c) for c in range(2) for b in range(2) for a in range(2)]
    for e in range(elem_dofs.shape[0]):
        for k in range(p):
            for j in range(p):
                for i in range(p):
                    s = i + p * (j + p * k)
                    ids = [elem_dofs[e, (i + a) + q * ((j + b) + q * (k + c))] for (a, b, c) in corners]
                    Xs = coords[ids]
                    Ke = np.zeros((8, 8))
                    for (x1, w1) in zip(xg, wg):
                        for (x2, w2) in zip(xg, wg):
                            for (x3, w3) in zip(xg, wg):
                                N = np.empty(8)
                                dN = np.empty((8, 3))
                                for v, (a, b, c) in enumerate(corners):
                                    fa = x1 if a else 1 - x1
                                    fb = x2 if b else 1 - x2
                                    fc = x3 if c else 1 - x3
                                    da = 1.0 if a else -1.0
                                    db = 1.0 if b else -1.0
                                    dc = 1.0 if c else -1.0
                                    N[v] = fa * fb * fc
                                    dN[v] = (da * fb * fc, fa * db * fc, fa * fb * dc)
                                J = Xs.T @ dN          # J[r, c] = sum_v X[v, r] dN[v, c]
                                dJ = np.linalg.det(J)
                                G = np.linalg.solve(J.T, dN.T).T
                                w = w1 * w2 * w3 * dJ
                                Ke += w * (kappa[e, s] * (G @ G.T) + beta * np.outer(N, N))
                    A[np.ix_(ids, ids)] += Ke
    return A


def test_brute_force_dense_curved():
    m = meshgen.cartesian_mesh(2, 2, 0.12)
    kap = meshgen.kappa_field(m["nel"], 2, 1.0, seed=11)
    rp, ci, v = orc.h1_matrix(m["coords"], m["elem_dofs"], 2, kap, 0.6)
    B = _brute_force_dense(m["coords"], m["elem_dofs"], 2, kap.numpy(), 0.6, 2)
    A = dense(rp, ci, v)
    assert np.abs(A - B).max() <= 1e-14 * np.abs(B).max()
    # pattern: every stored entry is a lattice neighbour pair, and nothing else
    assert ((A != 0) | (B == 0)).all()


def test_brute_force_affine_exact_rule():
    """On affine cells the 2-point rule equals a 4-point rule (exactness)."""
    Am, t = _affine()
    m = meshgen.affine_mesh(2, 2, Am, t)
    kap = meshgen.kappa_field(m["nel"], 2, 1.0, seed=12)
    rp, ci, v = orc.h1_matrix(m["coords"], m["elem_dofs"], 2, kap, 1.3)
    B = _brute_force_dense(m["coords"], m["elem_dofs"], 2, kap.numpy(), 1.3, 4)
    A = dense(rp, ci, v)
    assert np.abs(A - B).max() <= 1e-13 * np.abs(B).max()


# ------------------------------------------------------------- invariances

def test_vertex_renumbering_is_a_permutation():
    m = meshgen.cartesian_mesh(3, 2, 0.18)
    kap = meshgen.kappa_field(m["nel"], 2, 1.0, seed=5)
    rp, ci, v = orc.h1_matrix(m["coords"], m["elem_dofs"], 2, kap, 1.0)
    m2, perm = meshgen.renumber_vertices(m, seed=9)
    rp2, ci2, v2 = orc.h1_matrix(m2["coords"], m2["elem_dofs"], 2, kap, 1.0)
    A = dense(rp, ci, v)
    A2 = dense(rp2, ci2, v2)
    P = np.zeros_like(A)
    P[perm, np.arange(len(perm))] = 1.0
    assert np.abs(A2 - P @ A @ P.T).max() <= 1e-15 * np.abs(A).max()
    # row lengths travel with the rows
    assert np.array_equal(np.diff(rp2.numpy())[perm], np.diff(rp.numpy()))


def test_element_permutation_and_reorientation():
    m = meshgen.cartesian_mesh(3, 3, 0.18)
    kap = meshgen.kappa_field(m["nel"], 3, 1.0, seed=6)
    rp, ci, v = orc.h1_matrix(m["coords"], m["elem_dofs"], 3, kap, 1.0)
    m2, order = meshgen.permute_elements(m, seed=1)
    rp2, ci2, v2 = orc.h1_matrix(m2["coords"], m2["elem_dofs"], 3, kap[torch.from_numpy(order)], 1.0)
    assert torch.equal(rp, rp2) and torch.equal(ci, ci2)
    assert (v - v2).abs().max() <= 1e-15 * v.abs().max()
    m3, kap3, _ = meshgen.reorient_elements(m, seed=2, kappa=kap)
    rp3, ci3, v3 = orc.h1_matrix(m3["coords"], m3["elem_dofs"], 3, kap3, 1.0)
    assert torch.equal(rp, rp3) and torch.equal(ci, ci3)
    assert (v - v3).abs().max() <= 1e-14 * v.abs().max()


# -------------------------------------------------------------- pattern counts

@pytest.mark.parametrize("n,p", [(1, 1), (2, 1), (2, 2), (3, 2), (2, 3), (1, 4), (2, 4)])
def test_h1_pattern_count(n, p):
    m = meshgen.cartesian_mesh(n, p, 0.0)
    kap = torch.ones(m["nel"], p ** 3, dtype=torch.float64)
    rp, ci, v = orc.h1_matrix(m["coords"], m["elem_dofs"], p, kap, 1.0)
    N = m["N"]
    assert rp[-1].item() == (3 * N - 2) ** 3
    counts = (rp[1:] - rp[:-1]).numpy()
    assert counts.max() == min(3, N) ** 3 and counts.min() == 8


def test_paper_printed_counts_follow_the_lattice_formula():
    """The paper prints the 3D p=6 / 32768-element and 2D p=6 / 262144-element
    Helmholtz problem sizes; the lattice count that the oracle satisfies above,
    (3N-2)^d with N = n p + 1, reproduces them exactly."""
    with open(os.path.join(GOLDEN, "paper_counts.json")) as f:
        g = json.load(f)
    d3 = g["h1_3d"]
    n = round(d3["elements"] ** (1 / 3))
    N = n * d3["p"] + 1
    assert n ** 3 == d3["elements"]
    assert N ** 3 == d3["dofs"] and (3 * N - 2) ** 3 == d3["nnz"]
    d2 = g["h1_2d"]
    n2 = round(math.sqrt(d2["elements"]))
    N2 = n2 * d2["p"] + 1
    assert N2 ** 2 == d2["dofs"] and (3 * N2 - 2) ** 2 == d2["nnz"]


def test_h1_pattern_count_moderate_size():
    """A mid-size p=6 mesh: nnz from the oracle equals (3N-2)^3."""
    m = meshgen.cartesian_mesh(3, 6, 0.1)
    kap = torch.ones(m["nel"], 216, dtype=torch.float64)
    rp, _, _ = orc.h1_matrix(m["coords"], m["elem_dofs"], 6, kap, 1.0)
    assert rp[-1].item() == (3 * m["N"] - 2) ** 3


def test_rows_subset_matches_full():
    m = meshgen.cartesian_mesh(3, 3, 0.18)
    kap = meshgen.kappa_field(m["nel"], 3, 1.0, seed=8)
    rp, ci, v = orc.h1_matrix(m["coords"], m["elem_dofs"], 3, kap, 1.0)
    rows = torch.tensor([0, 5, 77, 400, m["ndofs"] - 1, 313])
    r, rp2, ci2, v2 = orc.h1_rows(m["coords"], m["elem_dofs"], 3, kap, 1.0, rows)
    for n, g in enumerate(r.tolist()):
        a, b = rp[g].item(), rp[g + 1].item()
        c, d = rp2[n].item(), rp2[n + 1].item()
        assert torch.equal(ci[a:b], ci2[c:d])
        assert (v[a:b] - v2[c:d]).abs().max() <= 1e-15 * v[a:b].abs().max()


# ----------------------------------------------------------------- H(curl)

def _nd_setup(n, p, amp, seed, reorient=False, flip=False):
    m = meshgen.cartesian_mesh(n, p, amp)
    ee, ned = meshgen.nd_edge_map(n, p)
    kap = meshgen.kappa_field(m["nel"], p, 1.0, seed=seed)
    if reorient:
        m, kap, ee = meshgen.reorient_elements(m, seed=seed + 1, kappa=kap, elem_edges=ee)
    S = None
    if flip:
        ee, S = meshgen.flip_edge_signs(ee, ned, seed=seed + 2)
    return m, ee, ned, kap, S


def _gradient_from_topology(m, ee, ned, p):
    """Discrete gradient written from its definition in this test: for every
    local edge of every element, the row of its global edge gets -sigma at the
    first local vertex and +sigma at the second."""
    q = p + 1
    G = np.zeros((ned, m["ndofs"]))
    loc = []
    for ax, dims in enumerate([(p, q, q), (q, p, q), (q, q, p)]):
        for k in range(dims[2]):
            for j in range(dims[1]):
                for i in range(dims[0]):
                    a = [i, j, k]
                    b = list(a)
                    b[ax] += 1
                    loc.append((a[0] + q * (a[1] + q * a[2]), b[0] + q * (b[1] + q * b[2])))
    ed = m["elem_dofs"]
    for e in range(m["nel"]):
        for l, (v0, v1) in enumerate(loc):
            raw = int(ee[e, l])
            g = raw if raw >= 0 else -1 - raw
            s = 1.0 if raw >= 0 else -1.0
            G[g, :] = 0.0
            G[g, ed[e, v0]] = -s
            G[g, ed[e, v1]] = s
    return G


@pytest.mark.parametrize("reorient,flip", [(False, False), (True, True)])
def test_nd_exact_sequence(reorient, flip):
    """curl grad = 0 on every trilinear cell:  K_curl G = 0.  And the gradients
    of the Q1 basis are Nedelec fields with coefficients G:  G^T M_nd(c) G =
    K_h1(c) with the same per-subelement coefficient c and quadrature."""
    p = 2
    m, ee, ned, kap, _ = _nd_setup(2, p, 0.12, seed=21, reorient=reorient, flip=flip)
    G = _gradient_from_topology(m, ee, ned, p)
    rp, ci, v = orc.nd_matrix(m["coords"], m["elem_dofs"], ee, p, kap, 0.0, ned)
    Kc = dense(rp, ci, v, ned)
    assert np.abs(Kc @ G).max() <= 1e-13 * np.abs(Kc).max()
    rp, ci, v = orc.nd_matrix(m["coords"], m["elem_dofs"], ee, p, torch.zeros_like(kap), kap, ned)
    Mn = dense(rp, ci, v, ned)
    rp, ci, v = orc.h1_matrix(m["coords"], m["elem_dofs"], p, kap, 0.0)
    Kh = dense(rp, ci, v)
    assert np.abs(G.T @ Mn @ G - Kh).max() <= 1e-13 * np.abs(Kh).max()
    # the oracle's discrete gradient (the algorithm's CSR form) is the same map
    grp, gci, gv = orc.discrete_gradient(m["elem_dofs"], ee, p, ned)
    assert np.abs(dense(grp, gci, gv, m["ndofs"]) - G).max() == 0.0


def test_nd_affine_fields():
    """u = a x X + b on parallelepipeds: curl u = 2a, so U^T K U = kappa |2a|^2 vol;
    and for constant u, U^T M U = beta |u|^2 vol.  Edge DOF = u(mid) . (v1 - v0)."""
    p = 2
    Am, t = _affine()
    m = meshgen.affine_mesh(2, p, Am, t)
    ee, ned = meshgen.nd_edge_map(2, p)
    kap = torch.full((m["nel"], p ** 3), 1.7, dtype=torch.float64)
    G = _gradient_from_topology(m, ee, ned, p)
    X = m["coords"]
    # edge endpoints from the gradient rows
    v0 = np.argmax(G < 0, axis=1)
    v1 = np.argmax(G > 0, axis=1)
    mid = 0.5 * (X[v0] + X[v1])
    tan = X[v1] - X[v0]
    a = np.array([0.3, -0.8, 0.5])
    b = np.array([1.1, 0.2, -0.6])
    U = np.einsum("ij,ij->i", np.cross(a, mid) + b, tan)
    vol = np.linalg.det(Am)
    rp, ci, v = orc.nd_matrix(X, m["elem_dofs"], ee, p, kap, 0.0, ned)
    K = dense(rp, ci, v, ned)
    assert abs(U @ K @ U - 1.7 * 4 * (a @ a) * vol) <= 1e-12 * 1.7 * 4 * (a @ a) * vol
    Uc = tan @ b
    rp, ci, v = orc.nd_matrix(X, m["elem_dofs"], ee, p, torch.zeros_like(kap), 2.0, ned)
    M = dense(rp, ci, v, ned)
    assert abs(Uc @ M @ Uc - 2.0 * (b @ b) * vol) <= 1e-12 * 2.0 * (b @ b) * vol


def test_nd_sign_flip():
    p = 2
    m, ee, ned, kap, _ = _nd_setup(2, p, 0.12, seed=31)
    rp, ci, v = orc.nd_matrix(m["coords"], m["elem_dofs"], ee, p, kap, 1.0, ned)
    ee2, S = meshgen.flip_edge_signs(ee, ned, seed=5)
    rp2, ci2, v2 = orc.nd_matrix(m["coords"], m["elem_dofs"], ee2, p, kap, 1.0, ned)
    A = dense(rp, ci, v, ned)
    A2 = dense(rp2, ci2, v2, ned)
    assert np.abs(A2 - S[:, None] * A * S[None, :]).max() == 0.0


@pytest.mark.parametrize("n,p", [(1, 2), (2, 1), (1, 3), (2, 2), (1, 5)])
def test_nd_pattern_count(n, p):
    """Cartesian count 3M(3M+1)(11M+1), M = n p; interior rows hold 33 (the
    paper's 'about 33 nonzeros per row' for the Nedelec LOR system)."""
    m, ee, ned, kap, _ = _nd_setup(n, p, 0.0, seed=1)
    rp, ci, v = orc.nd_matrix(m["coords"], m["elem_dofs"], ee, p, kap, 1.0, ned)
    M = n * p
    assert rp[-1].item() == 3 * M * (3 * M + 1) * (11 * M + 1)
    assert (rp[1:] - rp[:-1]).max().item() == (33 if M >= 2 else (rp[1:] - rp[:-1]).max().item())


def test_nd_symmetric_and_rows_subset():
    p = 3
    m, ee, ned, kap, _ = _nd_setup(2, p, 0.12, seed=41, reorient=True, flip=True)
    rp, ci, v = orc.nd_matrix(m["coords"], m["elem_dofs"], ee, p, kap, 1.0, ned)
    A = orc.csr_to_scipy(rp, ci, v, ned)
    assert abs(A - A.T).max() <= 1e-15 * abs(A).max()
    rows = torch.tensor([0, 3, 100, ned - 1])
    r, rp2, ci2, v2 = orc.nd_rows(m["coords"], m["elem_dofs"], ee, p, kap, 1.0, rows)
    for n, g in enumerate(r.tolist()):
        a, b = rp[g].item(), rp[g + 1].item()
        c, d = rp2[n].item(), rp2[n + 1].item()
        assert torch.equal(ci[a:b], ci2[c:d])
        assert (v[a:b] - v2[c:d]).abs().max() <= 1e-15 * v[a:b].abs().max()


# ------------------------------------------------------------------ gradients

def test_oracle_gradient_kappa_closed_form_and_fd():
    """L = <Gbar, A(kappa, X)>: dL/dkappa_s = <Gbar|s, K^s(kappa=1)> (linear), and
    central differences in the coordinates (step 1e-6) match autograd."""
    p = 2
    m = meshgen.cartesian_mesh(2, p, 0.12)
    kap = meshgen.kappa_field(m["nel"], p, 1.0, seed=2).requires_grad_(True)
    X = torch.from_numpy(m["coords"]).clone().requires_grad_(True)
    rp, ci, v = orc.h1_matrix(X, m["elem_dofs"], p, kap, 0.8)
    Gb = meshgen.cotangent(1, v.numel(), seed=1)[0]
    L = (Gb * v).sum()
    gk, gx = torch.autograd.grad(L, (kap, X))
    # closed form for kappa: per-subelement unit-kappa matrices, contracted with
    # the cotangent at each subelement entry's CSR position
    sv = orc.h1_subelement_vertices(torch.from_numpy(m["elem_dofs"]), p).reshape(-1, 8)
    with torch.no_grad():
        K1 = orc.h1_subelement_matrices(X[sv], torch.ones(sv.shape[0], dtype=torch.float64), 0.0)
    pos = {}
    for r in range(rp.numel() - 1):
        for q in range(rp[r].item(), rp[r + 1].item()):
            pos[(r, ci[q].item())] = q
    want = torch.zeros(sv.shape[0], dtype=torch.float64)
    for s in range(sv.shape[0]):
        acc = 0.0
        for u in range(8):
            for w in range(8):
                acc += Gb[pos[(sv[s, u].item(), sv[s, w].item())]].item() * K1[s, u, w].item()
        want[s] = acc
    assert (gk.reshape(-1) - want).abs().max() <= 1e-12 * want.abs().max()
    gen = torch.Generator().manual_seed(3)
    eps = 1e-6
    for _ in range(3):
        d = torch.randn(X.shape, generator=gen, dtype=torch.float64)
        d /= d.norm()
        with torch.no_grad():
            vp = orc.h1_matrix(X + eps * d, m["elem_dofs"], p, kap, 0.8)[2]
            vm = orc.h1_matrix(X - eps * d, m["elem_dofs"], p, kap, 0.8)[2]
        fd = ((Gb * vp).sum() - (Gb * vm).sum()).item() / (2 * eps)
        ad = (gx * d).sum().item()
        assert abs(fd - ad) <= 1e-6 * (abs(ad) + 1.0)


def test_inverted_subelement_raises():
    m = meshgen.cartesian_mesh(1, 2, 0.0)
    X = m["coords"].copy()
    # push the centre vertex through a corner of the domain: inverts cells
    X[13] = [1.5, 1.5, 1.5]
    kap = torch.ones(1, 8, dtype=torch.float64)
    with pytest.raises(ValueError):
        orc.h1_matrix(X, m["elem_dofs"], 2, kap, 1.0)


# -------------------------------------------- boundary-condition elimination (A4)

def _elim_case(space):
    if space == "h1":
        m = meshgen.cartesian_mesh(2, 2, 0.1)
        kap = meshgen.kappa_field(m["nel"], 2, 1.0, seed=3)
        rp, ci, v = orc.h1_matrix(m["coords"], m["elem_dofs"], 2, kap, 1.0)
        return rp, ci, v, m["ndofs"]
    m = meshgen.cartesian_mesh(2, 2, 0.1)
    ee, ned = meshgen.nd_edge_map(2, 2)
    kap = meshgen.kappa_field(m["nel"], 2, 1.0, seed=4)
    rp, ci, v = orc.nd_matrix(m["coords"], m["elem_dofs"], ee, 2, kap, 0.7, ned)
    return rp, ci, v, ned


@pytest.mark.parametrize("space", ["h1", "nd"])
@pytest.mark.parametrize("policy", ["one", "keep", "zero"])
def test_elimination_is_a_projection(space, policy):
    """With P = diag(1 - marker), eliminating rows and columns is
    P A P + (I - P) D, D = I ("one"), diag(A) ("keep") or 0 ("zero"): checked
    with dense matrix products instead of the oracle's entrywise rule, on a
    random essential set with repeats."""
    rp, ci, v, n = _elim_case(space)
    ess = meshgen.random_dofs(n, n // 3, seed=5)
    out, marker = orc.eliminate_bc(rp, ci, v, ess, policy)
    mk = np.zeros(n)
    mk[ess] = 1.0
    assert np.array_equal(marker.numpy(), mk > 0)
    A = dense(rp, ci, v)
    P = np.diag(1.0 - mk)
    D = {"one": np.eye(n), "keep": np.diag(np.diag(A)), "zero": np.zeros((n, n))}[policy]
    assert np.array_equal(dense(rp, ci, out), P @ A @ P + (np.eye(n) - P) @ D)
    # symmetric in, symmetric out (to the rounding asymmetry of A itself);
    # the pattern itself is kept (zeros stay stored)
    E = dense(rp, ci, out)
    assert np.all(np.abs(E - E.T) <= np.abs(A - A.T))
    assert out.shape == v.shape


def test_elimination_dirichlet_solve():
    """The eliminated system with right-hand side [f - A g on free rows; g on
    essential rows] has the solution of the reduced problem A_ff u_f =
    f_f - A_fe g_e, u_e = g_e (textbook Dirichlet elimination)."""
    rp, ci, v, n = _elim_case("h1")
    bnd = meshgen.boundary_vertices(2, 2)
    out, _ = orc.eliminate_bc(rp, ci, v, bnd, "one")
    A = dense(rp, ci, v)
    rng = np.random.default_rng(7)
    f = rng.standard_normal(n)
    g = np.zeros(n)
    g[bnd] = rng.standard_normal(bnd.size)
    free = np.setdiff1d(np.arange(n), bnd)
    b = f - A @ g
    b[bnd] = g[bnd]
    u = np.linalg.solve(dense(rp, ci, out), b)
    uf = np.linalg.solve(A[np.ix_(free, free)], f[free] - A[np.ix_(free, bnd)] @ g[bnd])
    assert np.abs(u[bnd] - g[bnd]).max() <= 1e-13
    assert np.abs(u[free] - uf).max() <= 1e-10 * np.abs(uf).max()


def test_elimination_edge_cases():
    rp, ci, v, n = _elim_case("h1")
    out, marker = orc.eliminate_bc(rp, ci, v, np.zeros(0, np.int32))
    assert torch.equal(out, v) and not bool(marker.any())
    out, _ = orc.eliminate_bc(rp, ci, v, np.arange(n))
    assert np.array_equal(dense(rp, ci, out), np.eye(n))
    vb = torch.stack([v, 2 * v, -v])  # batched values: each batch entry on its own
    ess = meshgen.random_dofs(n, 20, seed=9)
    ob, _ = orc.eliminate_bc(rp, ci, vb, ess, "keep")
    for b in range(3):
        assert torch.equal(ob[b], orc.eliminate_bc(rp, ci, vb[b], ess, "keep")[0])
    # a block of sampled rows gives the rows of the whole result
    rows = torch.tensor([3, 11, 20])
    sub_rp = torch.cat([torch.zeros(1, dtype=torch.int64), torch.cumsum(rp[rows + 1] - rp[rows], 0)])
    idx = torch.cat([torch.arange(rp[r], rp[r + 1]) for r in rows.tolist()])
    full, _ = orc.eliminate_bc(rp, ci, v, ess, "one")
    part, _ = orc.eliminate_bc(sub_rp, ci[idx], v[idx], ess, "one", rows=rows)
    assert torch.equal(part, full[idx])
    with pytest.raises(IndexError):
        orc.eliminate_bc(rp, ci, v, [n])


def test_discrete_gradient_first_incidence_order():
    """On reoriented elements with flipped edge signs, each row of the
    discrete gradient comes from the edge's first incidence (lowest element,
    then lowest local edge), found here by a plain loop; the row is the same
    sparse vector as the topological definition."""
    p = 2
    m = meshgen.cartesian_mesh(2, p, 0.0)
    ee, ned = meshgen.nd_edge_map(2, p)
    m, _, ee = meshgen.reorient_elements(m, seed=3, kappa=None, elem_edges=ee)
    ee, _ = meshgen.flip_edge_signs(ee, ned, seed=4)
    rp, ci, v = orc.discrete_gradient(m["elem_dofs"], ee, p, ned)
    q = p + 1
    loc = []
    for ax, dims in enumerate([(p, q, q), (q, p, q), (q, q, p)]):
        for k in range(dims[2]):
            for j in range(dims[1]):
                for i in range(dims[0]):
                    a = [i, j, k]
                    b = list(a)
                    b[ax] += 1
                    loc.append((a[0] + q * (a[1] + q * a[2]), b[0] + q * (b[1] + q * b[2])))
    done = set()
    for e in range(m["nel"]):
        for l, (v0, v1) in enumerate(loc):
            raw = int(ee[e, l])
            g = raw if raw >= 0 else -1 - raw
            if g in done:
                continue
            done.add(g)
            s = 1.0 if raw >= 0 else -1.0
            assert ci[2 * g].item() == m["elem_dofs"][e, v0] and ci[2 * g + 1].item() == m["elem_dofs"][e, v1]
            assert v[2 * g].item() == -s and v[2 * g + 1].item() == s
    assert len(done) == ned and torch.equal(rp, torch.arange(0, 2 * ned + 1, 2))
    G = _gradient_from_topology(m, ee, ned, p)
    assert np.array_equal(dense(rp, ci, v, m["ndofs"]), G)


# ------------------------------------------------ LOR coordinate vector (aux)

def test_interp_nodes_identity_when_degrees_match():
    """q = p: the Lagrange basis at its own nodes is the identity, exactly."""
    X = meshgen.ho_nodes(2, 3, 0.1)
    assert np.array_equal(orc.interp_nodes(X, 3, 3).numpy(), X)


@pytest.mark.parametrize("q,p", [(1, 6), (2, 4), (3, 5), (2, 2)])
def test_interp_nodes_reproduces_polynomial_maps(q, p):
    """A map whose components are polynomials of degree <= q in each variable
    is reproduced exactly (to rounding) at the degree-p lattice: the nodes are
    the map at the degree-q lattice, the expected values the map at the
    degree-p lattice, both evaluated here directly."""
    def f(P):
        x, y, z = P[..., 0], P[..., 1], P[..., 2]
        d = min(q, 2)
        return np.stack([x + 0.3 * y ** d - 0.2 * x * z, y - 0.1 * (x * y) ** (d - 1) * z + 0.05,
                         z + 0.2 * x ** d * y - 0.1], axis=-1)
    mq = meshgen.cartesian_mesh(2, q, 0.0)
    mp = meshgen.cartesian_mesh(2, p, 0.0)
    nodes = f(mq["coords"])[mq["elem_dofs"]]
    want = f(mp["coords"])[mp["elem_dofs"]]
    got = orc.interp_nodes(nodes, p, q).numpy()
    assert np.abs(got - want).max() <= 1e-14


def test_interp_nodes_trilinear_gives_the_lattice():
    """q = 1 from the 8 corners of each element of an affine mesh gives the
    Gauss-Lobatto lattice of the same affine mesh (the input generator's own
    lattice), as an E-vector; deduplicated it is the vertex coordinate array."""
    A = np.array([[1.0, 0.2, 0.0], [0.1, 0.9, 0.3], [0.0, -0.2, 1.1]])
    t = np.array([0.3, -0.1, 2.0])
    m1 = meshgen.affine_mesh(3, 1, A, t)
    m6 = meshgen.affine_mesh(3, 6, A, t)
    E = orc.interp_nodes(m1["coords"][m1["elem_dofs"]], 6, 1)
    assert np.abs(E.numpy() - m6["coords"][m6["elem_dofs"]]).max() <= 1e-14
    T = orc.evec_to_tvec(E, m6["elem_dofs"], m6["ndofs"])
    assert np.abs(T.numpy() - m6["coords"]).max() <= 1e-14


def test_evec_to_tvec_first_incidence():
    """Every dof takes the value of its first incidence (lowest element, then
    lowest local index), found here by a plain loop over a renumbered mesh
    whose E-vector differs per element."""
    m, _ = meshgen.renumber_vertices(meshgen.cartesian_mesh(2, 2, 0.0), seed=1)
    ed = m["elem_dofs"]
    E = np.zeros(ed.shape + (2,))
    E[..., 0] = np.arange(ed.size).reshape(ed.shape)
    E[..., 1] = -ed
    T = orc.evec_to_tvec(E, ed, m["ndofs"]).numpy()
    seen = {}
    for e in range(ed.shape[0]):
        for l in range(ed.shape[1]):
            seen.setdefault(int(ed[e, l]), (e, l))
    assert len(seen) == m["ndofs"]
    for g, (e, l) in seen.items():
        assert T[g, 0] == e * ed.shape[1] + l and T[g, 1] == -g
    with pytest.raises(ValueError):
        orc.evec_to_tvec(E, ed, m["ndofs"] + 1)


# ------------------------------------------------------- discrete curl (aux)

def _curl_setup(n, p, seed):
    A = np.array([[1.0, 0.3, -0.1], [0.05, 0.9, 0.2], [0.1, -0.15, 1.2]])
    t = np.array([0.2, -0.4, 0.1])
    m = meshgen.affine_mesh(n, p, A, t)
    ee, ned = meshgen.nd_edge_map(n, p)
    fm, nf = meshgen.face_map(n, p)
    ee, se = meshgen.flip_edge_signs(ee, ned, seed=seed)
    fm, sf = meshgen.flip_edge_signs(fm, nf, seed=seed + 1)
    return m, ee, ned, se, fm, nf, sf


@pytest.mark.parametrize("n,p", [(2, 1), (2, 2), (1, 4)])
def test_discrete_curl_stokes_and_exact_sequence(n, p):
    """On an affine mesh with randomly flipped edge and face orientations:
    (1) C G = 0 exactly (curl of a gradient); (2) Stokes: for u = a x X + b,
    with edge dofs u(mid).(v1 - v0) (exact for linear u) and face dofs
    curl u . (t1 x t2) = 2a . (t1 x t2) over each parallelogram face (t1, t2
    its lattice edge vectors ordered so that t1 x t2 points along the face's
    +axis normal), C U equals F.  Geometry and numbering are rebuilt here from
    the lattice, not taken from the oracle."""
    m, ee, ned, se, fm, nf, sf = _curl_setup(n, p, seed=n + p)
    rp, ci, v = orc.discrete_curl(ee, fm, p, nf)
    C = dense(rp, ci, v, ned)
    grp, gci, gv = orc.discrete_gradient(m["elem_dofs"], ee, p, ned)
    assert np.abs(C @ dense(grp, gci, gv, m["ndofs"])).max() == 0.0
    M = n * p
    N = M + 1
    X = m["coords"]

    def P(x, y, z):
        return X[x + N * (y + N * z)]
    a = np.array([0.4, -0.7, 0.25])
    b = np.array([0.1, 0.3, -0.2])
    U = np.zeros(ned)
    for g in range(ned):
        if g < M * N * N:
            x, y, z = g % M, (g // M) % N, g // (M * N)
            v0, v1 = P(x, y, z), P(x + 1, y, z)
        elif g < 2 * M * N * N:
            h = g - M * N * N
            x, y, z = h % N, (h // N) % M, h // (N * M)
            v0, v1 = P(x, y, z), P(x, y + 1, z)
        else:
            h = g - 2 * M * N * N
            x, y, z = h % N, (h // N) % N, h // (N * N)
            v0, v1 = P(x, y, z), P(x, y, z + 1)
        mid = 0.5 * (v0 + v1)
        U[g] = se[g] * (np.cross(a, mid) + b) @ (v1 - v0)
    F = np.zeros(nf)
    for f in range(nf):
        if f < N * M * M:
            x, y, z = f % N, (f // N) % M, f // (N * M)
            o = P(x, y, z)
            t1, t2 = P(x, y + 1, z) - o, P(x, y, z + 1) - o
        elif f < 2 * N * M * M:
            h = f - N * M * M
            x, y, z = h % M, (h // M) % N, h // (M * N)
            o = P(x, y, z)
            t1, t2 = P(x, y, z + 1) - o, P(x + 1, y, z) - o
        else:
            h = f - 2 * N * M * M
            x, y, z = h % M, (h // M) % M, h // (M * M)
            o = P(x, y, z)
            t1, t2 = P(x + 1, y, z) - o, P(x, y + 1, z) - o
        F[f] = sf[f] * (2 * a) @ np.cross(t1, t2)
    assert np.abs(C @ U - F).max() <= 1e-13 * max(1.0, np.abs(F).max())


def test_discrete_curl_first_incidence_rows():
    """Each face row comes from the face's first incidence: checked with a
    plain loop over elements and local faces, rebuilding the 4 boundary edges
    of every local face from its lattice position."""
    p = 2
    q = p + 1
    m, ee, ned, se, fm, nf, sf = _curl_setup(2, p, seed=7)
    rp, ci, v = orc.discrete_curl(ee, fm, p, nf)

    def xe(i, j, k):
        return i + p * (j + q * k)

    def ye(i, j, k):
        return p * q * q + i + q * (j + p * k)

    def ze(i, j, k):
        return 2 * p * q * q + i + q * (j + q * k)
    loc = {}
    for k in range(p):
        for j in range(p):
            for i in range(q):
                loc[i + q * (j + p * k)] = [(ye(i, j, k), 1), (ze(i, j + 1, k), 1), (ye(i, j, k + 1), -1),
                                            (ze(i, j, k), -1)]
    for k in range(p):
        for j in range(q):
            for i in range(p):
                loc[p * p * q + i + p * (j + q * k)] = [(ze(i, j, k), 1), (xe(i, j, k + 1), 1),
                                                        (ze(i + 1, j, k), -1), (xe(i, j, k), -1)]
    for k in range(q):
        for j in range(p):
            for i in range(p):
                loc[2 * p * p * q + i + p * (j + p * k)] = [(xe(i, j, k), 1), (ye(i + 1, j, k), 1),
                                                            (xe(i, j + 1, k), -1), (ye(i, j, k), -1)]
    done = set()
    for e in range(fm.shape[0]):
        for lf in range(fm.shape[1]):
            raw = int(fm[e, lf])
            f = raw if raw >= 0 else -1 - raw
            if f in done:
                continue
            done.add(f)
            s_f = 1 if raw >= 0 else -1
            for slot, (le, s) in enumerate(loc[lf]):
                r = int(ee[e, le])
                g = r if r >= 0 else -1 - r
                s_e = 1 if r >= 0 else -1
                assert ci[4 * f + slot].item() == g and v[4 * f + slot].item() == s_f * s_e * s
    assert len(done) == nf and torch.equal(rp, torch.arange(0, 4 * nf + 1, 4))


# ------------------------------------------------------------------- H(div)

def _rt_setup(n, p, amp, seed):
    m = meshgen.cartesian_mesh(n, p, amp)
    ee, ned = meshgen.nd_edge_map(n, p)
    fm, nf = meshgen.face_map(n, p)
    ee, _ = meshgen.flip_edge_signs(ee, ned, seed=seed)
    fm, _ = meshgen.flip_edge_signs(fm, nf, seed=seed + 1)
    kap = meshgen.kappa_field(m["nel"], p, 1.0, seed=seed + 2)
    return m, ee, ned, fm, nf, kap


@pytest.mark.parametrize("n,p", [(2, 2), (1, 3)])
def test_rt_exact_sequence(n, p):
    """With the (pinned) discrete curl C, on a curved mesh with flipped edge
    and face orientations: K_div C = 0 (div of a curl) and, with the RT mass
    weighted by kappa per subelement, C^T M_RT C = K_curl, the (pinned) ND
    curl-curl with the same kappa (curl N_e = sum_f C_fe RT_f pointwise under
    the Piola maps, same 2x2x2 rule)."""
    m, ee, ned, fm, nf, kap = _rt_setup(n, p, 0.1, seed=n + 3 * p)
    crp, cci, cv = orc.discrete_curl(ee, fm, p, nf)
    C = dense(crp, cci, cv, ned)
    rp, ci, v = orc.rt_matrix(m["coords"], m["elem_dofs"], fm, p, kap, 0.0, nf)
    K = dense(rp, ci, v)
    assert np.abs(K @ C).max() <= 1e-14 * np.abs(K).max() * np.abs(C).sum(axis=0).max()
    rp, ci, v = orc.rt_matrix(m["coords"], m["elem_dofs"], fm, p, torch.zeros_like(kap), kap, nf)
    Mrt = dense(rp, ci, v)
    rp, ci, v = orc.nd_matrix(m["coords"], m["elem_dofs"], ee, p, kap, 0.0, ned)
    Kc = dense(rp, ci, v)
    assert np.abs(C.T @ Mrt @ C - Kc).max() <= 1e-13 * np.abs(Kc).max()
    assert np.abs(K - K.T).max() <= 1e-14 * np.abs(K).max()


def test_rt_affine_fields():
    """On a parallelepiped mesh, for u = alpha X + b (div u = 3 alpha), face
    dofs = flux u(centre).(t1 x t2) (exact for linear u on a parallelogram):
    U^T K U = kappa (3 alpha)^2 vol; for constant u, U^T M U = beta |u|^2 vol.
    Faces and their vectors are rebuilt here from the lattice."""
    p, n = 2, 2
    Am, t = _affine()
    m = meshgen.affine_mesh(n, p, Am, t)
    fm, nf = meshgen.face_map(n, p)
    M_, N = n * p, n * p + 1
    X = m["coords"]

    def P(x, y, z):
        return X[x + N * (y + N * z)]
    centres, areas = np.zeros((nf, 3)), np.zeros((nf, 3))
    for f in range(nf):
        if f < N * M_ * M_:
            x, y, z = f % N, (f // N) % M_, f // (N * M_)
            o = P(x, y, z)
            t1, t2 = P(x, y + 1, z) - o, P(x, y, z + 1) - o
        elif f < 2 * N * M_ * M_:
            h = f - N * M_ * M_
            x, y, z = h % M_, (h // M_) % N, h // (M_ * N)
            o = P(x, y, z)
            t1, t2 = P(x, y, z + 1) - o, P(x + 1, y, z) - o
        else:
            h = f - 2 * N * M_ * M_
            x, y, z = h % M_, (h // M_) % M_, h // (M_ * M_)
            o = P(x, y, z)
            t1, t2 = P(x + 1, y, z) - o, P(x, y + 1, z) - o
        centres[f] = o + 0.5 * (t1 + t2)
        areas[f] = np.cross(t1, t2)
    vol = np.linalg.det(Am)
    alpha, b = 0.7, np.array([0.2, -0.5, 0.9])
    U = np.einsum("ij,ij->i", alpha * centres + b, areas)
    kap = torch.full((m["nel"], p ** 3), 1.3, dtype=torch.float64)
    rp, ci, v = orc.rt_matrix(X, m["elem_dofs"], fm, p, kap, 0.0, nf)
    K = dense(rp, ci, v)
    assert abs(U @ K @ U - 1.3 * 9 * alpha ** 2 * vol) <= 1e-12 * 1.3 * 9 * alpha ** 2 * vol
    Uc = areas @ b
    rp, ci, v = orc.rt_matrix(X, m["elem_dofs"], fm, p, torch.zeros_like(kap), 0.6, nf)
    Mm = dense(rp, ci, v)
    assert abs(Uc @ Mm @ Uc - 0.6 * (b @ b) * vol) <= 1e-12 * 0.6 * (b @ b) * vol


def test_rt_pattern_count_and_sign_flip():
    """nnz = nfaces + 30 M^3 on an M^3 lattice (every face couples to itself
    and to the 5 other faces of each of its one or two subelements); flipping
    face orientations gives S A S."""
    n, p = 2, 2
    m = meshgen.cartesian_mesh(n, p, 0.1)
    fm, nf = meshgen.face_map(n, p)
    kap = meshgen.kappa_field(m["nel"], p, 1.0, seed=4)
    rp, ci, v = orc.rt_matrix(m["coords"], m["elem_dofs"], fm, p, kap, 0.8, nf)
    M_ = n * p
    assert rp[-1].item() == nf + 30 * M_ ** 3
    cnt = (rp[1:] - rp[:-1])
    assert int(cnt.max()) == 11 and int(cnt.min()) == 6
    fm2, S = meshgen.flip_edge_signs(fm, nf, seed=6)
    rp2, ci2, v2 = orc.rt_matrix(m["coords"], m["elem_dofs"], fm2, p, kap, 0.8, nf)
    A, A2 = dense(rp, ci, v), dense(rp2, ci2, v2)
    assert np.abs(A2 - S[:, None] * A * S[None, :]).max() <= 1e-14 * np.abs(A).max()


def _rows_match(rp, ci, v, r, rp2, ci2, v2):
    """The rows (r, rp2, ci2, v2) of a row-subset call equal the same rows of
    the whole matrix: columns bit for bit, values to 1e-15 of the row maximum."""
    for n, g in enumerate(r.tolist()):
        a, b = rp[g].item(), rp[g + 1].item()
        c, d = rp2[n].item(), rp2[n + 1].item()
        assert torch.equal(ci[a:b], ci2[c:d]), g
        assert (v[a:b] - v2[c:d]).abs().max() <= 1e-15 * v[a:b].abs().max(), g


@pytest.mark.parametrize("reorient", [False, True])
def test_rt_rows_match_the_whole_matrix(reorient):
    """rt_rows (the row-subset form used as the reference at full size) gives
    exactly the rows of rt_matrix, whose own pins are the exact sequence, the
    affine fields and the sign flip: curved mesh, flipped face signs, and
    optionally every element rotated by a random cube symmetry (face map then
    derived from the rotated vertex map)."""
    n, p = 2, 3
    m, ee, ned, fm, nf, kap = _rt_setup(n, p, 0.12, seed=17)
    if reorient:
        # rotated local frames; faces (and their orientation) re-derived from
        # the rotated vertex map
        m, kap, _ = meshgen.reorient_elements(m, seed=18, kappa=kap)
        fm, nf = meshgen.face_map_from_vertices(m["elem_dofs"], p)
    rp, ci, v = orc.rt_matrix(m["coords"], m["elem_dofs"], fm, p, kap, 0.7, nf)
    rows = torch.tensor([0, 1, 37, nf // 2, nf // 3 + 5, nf - 1, 200])
    r, rp2, ci2, v2 = orc.rt_rows(m["coords"], m["elem_dofs"], fm, p, kap, 0.7, rows)
    assert torch.equal(r, torch.unique(rows))
    _rows_match(rp, ci, v, r, rp2, ci2, v2)
    # every row at once: the subset form reproduces the whole CSR matrix
    r, rp2, ci2, v2 = orc.rt_rows(m["coords"], m["elem_dofs"], fm, p, kap, 0.7, torch.arange(nf))
    assert torch.equal(rp2, rp) and torch.equal(ci2, ci)
    assert (v2 - v).abs().max() <= 1e-15 * v.abs().max()


# ----------------------------------------------------------------- H1 in 2D

def test_h1_2d_closed_form_uniform_square():
    """Uniform lattice (p <= 2, where the Gauss-Lobatto points are
    equispaced): every entry equals (#cells holding both vertices) x (the
    bilinear cell-matrix entry for their offset), stiffness 2/3, -1/6, -1/3
    and mass h^2 (1/9, 1/18, 1/36) for offsets differing in 0, 1, 2
    coordinates -- derived from 1D element matrices by tensor products."""
    n, p = 3, 2
    m = meshgen.cartesian_mesh_2d(n, p, 0.0)
    N = m["N"]
    h = 1.0 / (N - 1)
    kap = torch.full((m["nel"], p * p), 1.7, dtype=torch.float64)
    rp, ci, v = orc.h1_matrix_2d(m["coords"], m["elem_dofs"], p, kap, 0.9)
    S1 = np.array([[1.0, -1.0], [-1.0, 1.0]])
    M1 = np.array([[2.0, 1.0], [1.0, 2.0]]) / 6.0
    Kc = 1.7 * (np.kron(M1, S1) + np.kron(S1, M1))   # cell matrix, vertex a + 2b
    Mc = 0.9 * h * h * np.kron(M1, M1)
    want = np.zeros((N * N, N * N))
    for cy in range(N - 1):
        for cx in range(N - 1):
            g = [(cx + a) + N * (cy + b) for b in range(2) for a in range(2)]
            for u in range(4):
                for w in range(4):
                    want[g[u], g[w]] += Kc[u, w] + Mc[u, w]
    A = dense(rp, ci, v)
    assert np.abs(A - want).max() <= 1e-14 * np.abs(want).max()
    c = N * 2 + 2
    assert abs(A[c, c] - 1.7 * 8 / 3 - 0.9 * 4 * h * h / 9) <= 1e-14


def test_h1_2d_row_sums_and_area():
    """Curved quads, random kappa: stiffness rows sum to 0 (constants are in
    the kernel); with kappa = 0 and beta = 1 the sum of all entries is the
    area of the bilinear mesh, computed here cell by cell with the shoelace
    formula (2x2 Gauss integrates det J of a bilinear map exactly)."""
    n, p = 3, 4
    m = meshgen.cartesian_mesh_2d(n, p, 0.15)
    kap = meshgen.kappa_field_2d(m["nel"], p, 1.0, seed=2)
    rp, ci, v = orc.h1_matrix_2d(m["coords"], m["elem_dofs"], p, kap, 0.0)
    A = dense(rp, ci, v)
    assert np.abs(A.sum(axis=1)).max() <= 1e-13 * np.abs(A).max()
    assert np.abs(A - A.T).max() <= 1e-14 * np.abs(A).max()
    rp, ci, v = orc.h1_matrix_2d(m["coords"], m["elem_dofs"], p, torch.zeros_like(kap), 1.0)
    X = m["coords"]
    N = m["N"]
    area = 0.0
    for cy in range(N - 1):
        for cx in range(N - 1):
            P = [X[(cx + a) + N * (cy + b)] for a, b in ((0, 0), (1, 0), (1, 1), (0, 1))]
            area += 0.5 * sum(P[k][0] * P[(k + 1) % 4][1] - P[(k + 1) % 4][0] * P[k][1] for k in range(4))
    assert abs(float(v.sum()) - area) <= 1e-13


def test_h1_2d_affine_energy_and_pattern():
    """Affine map x -> B x + t: for u = a . x, U^T K U = kappa |a|^2 area;
    nnz = (3N - 2)^2 and 9 entries per interior row (the 2D counts of
    Section 4.1 follow from the same formula, see the count pin)."""
    n, p = 2, 3
    m = meshgen.cartesian_mesh_2d(n, p, 0.0)
    B = np.array([[1.2, 0.3], [-0.2, 0.8]])
    X = m["coords"] @ B.T + np.array([0.4, -1.0])
    kap = torch.full((m["nel"], p * p), 0.6, dtype=torch.float64)
    rp, ci, v = orc.h1_matrix_2d(X, m["elem_dofs"], p, kap, 0.0)
    a = np.array([0.7, -1.1])
    U = X @ a
    K = dense(rp, ci, v)
    want = 0.6 * (a @ a) * np.linalg.det(B)
    assert abs(U @ K @ U - want) <= 1e-12 * want
    N = m["N"]
    assert rp[-1].item() == (3 * N - 2) ** 2
    assert int((rp[1:] - rp[:-1]).max()) == 9


@pytest.mark.parametrize("mesh", ["cartesian", "polygon"])
def test_h1_rows_2d_match_the_whole_matrix(mesh):
    """h1_rows_2d (the row-subset form used as the reference at full size)
    gives exactly the rows of h1_matrix_2d, whose own pins are the closed
    form, zero row sums, area and affine energy: curved Cartesian and
    irregular-valence polygon meshes, random kappa, beta != 0."""
    p = 3
    m = meshgen.cartesian_mesh_2d(3, p, 0.15) if mesh == "cartesian" else meshgen.polygon_mesh_2d(p, 5, 0.15)
    nd = m["coords"].shape[0]
    kap = meshgen.kappa_field_2d(m["nel"], p, 1.0, seed=5)
    rp, ci, v = orc.h1_matrix_2d(m["coords"], m["elem_dofs"], p, kap, 0.9, nd)
    rows = torch.tensor([0, 3, nd // 2, nd - 1, 11, 3])
    r, rp2, ci2, v2 = orc.h1_rows_2d(m["coords"], m["elem_dofs"], p, kap, 0.9, rows)
    assert torch.equal(r, torch.unique(rows))
    _rows_match(rp, ci, v, r, rp2, ci2, v2)
    r, rp2, ci2, v2 = orc.h1_rows_2d(m["coords"], m["elem_dofs"], p, kap, 0.9, torch.arange(nd))
    assert torch.equal(rp2, rp) and torch.equal(ci2, ci)
    assert (v2 - v).abs().max() <= 1e-15 * v.abs().max()


# ------------------------------------------------- irregular-valence hex meshes

PRISMS = [(3, 2, 2), (5, 2, 2), (3, 1, 3)]   # (sides, layers, p)


@pytest.mark.parametrize("sides,layers,p", PRISMS)
def test_prism_h1_invariants_and_axis_rows(sides, layers, p):
    """The polygon prism has an axis edge shared by `sides` elements per layer.
    With flat faces the subelements tile the prism exactly and det J is
    bilinear on each, so the 2-point rule gives total mass = polygon area x 1.
    On a curved copy the diffusion rows sum to zero and K is symmetric.  A
    vertex on the axis at an interior lattice level couples to the centre, the
    first spoke point and the first diagonal point of every quadrilateral on
    three levels: 3 (1 + 2 sides) columns."""
    m = meshgen.prism_mesh(p, sides, layers, 0.0)
    kap = meshgen.kappa_field(m["nel"], p, 1.0, seed=7)
    rp, ci, v = orc.h1_matrix(m["coords"], m["elem_dofs"], p, torch.zeros_like(kap), 1.0)
    area = 0.5 * sides * math.sin(2.0 * math.pi / sides)
    assert abs(float(v.sum()) - area) <= 1e-13
    X = m["coords"]
    on_axis = np.flatnonzero((np.abs(X[:, 0]) < 1e-12) & (np.abs(X[:, 1]) < 1e-12))
    assert len(on_axis) == layers * p + 1
    lengths = (rp[1:] - rp[:-1]).numpy()
    for g in on_axis:
        z = X[g, 2]
        levels = 2 if (z < 1e-12 or z > 1.0 - 1e-12) else 3
        assert lengths[g] == levels * (1 + 2 * sides)
    mc = meshgen.prism_mesh(p, sides, layers, 0.15)
    rp, ci, v = orc.h1_matrix(mc["coords"], mc["elem_dofs"], p, kap, 0.0)
    K = dense(rp, ci, v)
    assert np.abs(K.sum(axis=1)).max() <= 1e-13 * np.abs(K).max()
    assert np.abs(K - K.T).max() <= 1e-15 * np.abs(K).max()


@pytest.mark.parametrize("sides,layers,p", PRISMS)
def test_prism_nd_rt_exact_sequences(sides, layers, p):
    """On the curved polygon prism, with edge and face maps built from the
    vertex map alone: K_curl G = 0 and G^T M_ND G = K_H1 (the gradient written
    from its definition here), K_div C = 0 and C^T M_RT C = K_curl (the discrete
    curl of the oracle).  A face or edge whose orientation disagreed between
    two elements would break the second identity of each pair."""
    m = meshgen.prism_mesh(p, sides, layers, 0.15)
    ee, ned = meshgen.edge_map_from_vertices(m["elem_dofs"], p)
    fm, nf = meshgen.face_map_from_vertices(m["elem_dofs"], p)
    kap = meshgen.kappa_field(m["nel"], p, 1.0, seed=sides + 10 * p)
    G = _gradient_from_topology(m, ee, ned, p)
    rp, ci, v = orc.nd_matrix(m["coords"], m["elem_dofs"], ee, p, kap, 0.0, ned)
    Kc = dense(rp, ci, v, ned)
    assert np.abs(Kc @ G).max() <= 1e-13 * np.abs(Kc).max()
    rp, ci, v = orc.nd_matrix(m["coords"], m["elem_dofs"], ee, p, torch.zeros_like(kap), kap, ned)
    Mn = dense(rp, ci, v, ned)
    rp, ci, v = orc.h1_matrix(m["coords"], m["elem_dofs"], p, kap, 0.0)
    Kh = dense(rp, ci, v)
    assert np.abs(G.T @ Mn @ G - Kh).max() <= 1e-13 * np.abs(Kh).max()
    crp, cci, cv = orc.discrete_curl(ee, fm, p, nf)
    C = dense(crp, cci, cv, ned)
    rp, ci, v = orc.rt_matrix(m["coords"], m["elem_dofs"], fm, p, kap, 0.0, nf)
    Kd = dense(rp, ci, v, nf)
    assert np.abs(Kd @ C).max() <= 1e-14 * np.abs(Kd).max() * np.abs(C).sum(axis=0).max()
    rp, ci, v = orc.rt_matrix(m["coords"], m["elem_dofs"], fm, p, torch.zeros_like(kap), kap, nf)
    Mrt = dense(rp, ci, v, nf)
    assert np.abs(C.T @ Mrt @ C - Kc).max() <= 1e-13 * np.abs(Kc).max()


@pytest.mark.parametrize("sides,p", [(3, 2), (5, 3), (5, 1)])
def test_polygon_2d_invariants(sides, p):
    """The 2D polygon mesh (centre shared by `sides` quadrilaterals): total
    mass = polygon area (flat bilinear cells tile it exactly, det J bilinear),
    zero diffusion row sums and symmetry on a curved copy, and the centre row
    couples 1 + 2 sides vertices."""
    m = meshgen.polygon_mesh_2d(p, sides, 0.0)
    kap = meshgen.kappa_field_2d(m["nel"], p, 1.0, seed=sides)
    rp, ci, v = orc.h1_matrix_2d(m["coords"], m["elem_dofs"], p, torch.zeros_like(kap), 1.0, m["ndofs"])
    area = 0.5 * sides * math.sin(2.0 * math.pi / sides)
    assert abs(float(v.sum()) - area) <= 1e-13
    c = int(np.flatnonzero(np.abs(m["coords"]).sum(axis=1) < 1e-12)[0])
    assert int(rp[c + 1] - rp[c]) == 1 + 2 * sides
    mc = meshgen.polygon_mesh_2d(p, sides, 0.15)
    rp, ci, v = orc.h1_matrix_2d(mc["coords"], mc["elem_dofs"], p, kap, 0.0, mc["ndofs"])
    K = dense(rp, ci, v)
    assert np.abs(K.sum(axis=1)).max() <= 1e-13 * np.abs(K).max()
    assert np.abs(K - K.T).max() <= 1e-15 * np.abs(K).max()


@pytest.mark.parametrize("n,layers,p", [(2, 1, 2), (2, 2, 1), (1, 2, 3)])
def test_tri_split_invariants_and_exact_sequences(n, layers, p):
    """The triangle-split hex mesh of the unit cube (valence 3, 4 and 6):
    total mass = 1 with flat faces; on a curved copy zero diffusion row sums,
    symmetry, and the ND and RT exact sequences with vertex-derived edge and
    face maps; rows at valence-6 vertices inside the cube couple 3 x 13
    vertices."""
    m = meshgen.tri_split_mesh(n, layers, p, 0.0)
    kap = meshgen.kappa_field(m["nel"], p, 1.0, seed=11)
    rp, ci, v = orc.h1_matrix(m["coords"], m["elem_dofs"], p, torch.zeros_like(kap), 1.0)
    assert abs(float(v.sum()) - 1.0) <= 1e-13
    if n >= 2 and layers * p >= 2:
        assert int((rp[1:] - rp[:-1]).max()) == 39
    mc = meshgen.tri_split_mesh(n, layers, p, 0.12)
    rp, ci, v = orc.h1_matrix(mc["coords"], mc["elem_dofs"], p, kap, 0.0)
    Kh = dense(rp, ci, v)
    assert np.abs(Kh.sum(axis=1)).max() <= 1e-13 * np.abs(Kh).max()
    assert np.abs(Kh - Kh.T).max() <= 1e-15 * np.abs(Kh).max()
    ee, ned = meshgen.edge_map_from_vertices(mc["elem_dofs"], p)
    fm, nf = meshgen.face_map_from_vertices(mc["elem_dofs"], p)
    G = _gradient_from_topology(mc, ee, ned, p)
    rp, ci, v = orc.nd_matrix(mc["coords"], mc["elem_dofs"], ee, p, kap, 0.0, ned)
    Kc = dense(rp, ci, v, ned)
    assert np.abs(Kc @ G).max() <= 1e-13 * np.abs(Kc).max()
    rp, ci, v = orc.nd_matrix(mc["coords"], mc["elem_dofs"], ee, p, torch.zeros_like(kap), kap, ned)
    assert np.abs(G.T @ dense(rp, ci, v, ned) @ G - Kh).max() <= 1e-13 * np.abs(Kh).max()
    crp, cci, cv = orc.discrete_curl(ee, fm, p, nf)
    C = dense(crp, cci, cv, ned)
    rp, ci, v = orc.rt_matrix(mc["coords"], mc["elem_dofs"], fm, p, torch.zeros_like(kap), kap, nf)
    assert np.abs(C.T @ dense(rp, ci, v, nf) @ C - Kc).max() <= 1e-13 * np.abs(Kc).max()
    rp, ci, v = orc.rt_matrix(mc["coords"], mc["elem_dofs"], fm, p, kap, 0.0, nf)
    Kd = dense(rp, ci, v, nf)
    assert np.abs(Kd @ C).max() <= 1e-14 * np.abs(Kd).max() * np.abs(C).sum(axis=0).max()


@pytest.mark.parametrize("n,p", [(2, 1), (2, 2), (2, 3), (1, 4)])
def test_vertex_derived_maps_match_the_cartesian_maps(n, p):
    """The generic edge and face maps built from the vertex map alone agree with
    the Cartesian formulas up to a relabelling of the ids and, per face, one
    global sign: the same local entities are merged, and two elements sharing
    an entity agree (or disagree) on its orientation in both maps alike.  On the
    lexicographic lattice every edge runs from the lower to the higher vertex
    id, so the generic edge signs are all positive, as the Cartesian ones."""
    m = meshgen.cartesian_mesh(n, p, 0.0)

    def dec(a):
        return np.where(a < 0, -1 - a, a)

    ee, ned = meshgen.nd_edge_map(n, p)
    eg, ng = meshgen.edge_map_from_vertices(m["elem_dofs"], p)
    assert ng == ned and (eg >= 0).all() and (ee >= 0).all()
    pairs = set(zip(dec(ee).ravel().tolist(), dec(eg).ravel().tolist()))
    assert len(pairs) == ned                       # a bijection between the two id sets
    fm, nf = meshgen.face_map(n, p)
    fg, nf2 = meshgen.face_map_from_vertices(m["elem_dofs"], p)
    assert nf2 == nf
    pairs = set(zip(dec(fm).ravel().tolist(), dec(fg).ravel().tolist()))
    assert len(pairs) == nf
    rel = {}
    for f, r in zip(dec(fm).ravel().tolist(), (np.sign(fm + 0.5) * np.sign(fg + 0.5)).ravel().tolist()):
        assert rel.setdefault(f, r) == r           # one relative sign per face
