"""GPU parity on hexahedral meshes that are not Cartesian grids, with the edge
and face maps built from the vertex map alone: the polygon prism (an axis edge
shared by 3 or 5 elements per layer, rows of 21 or 33 vertex columns on the
axis, more than 8 colours) and the triangle-split cube (valence 3, 4 and 6
everywhere, rows of up to 39 vertex columns, hundreds of elements, so every
colour spans several groups per workgroup)."""
import sys

import numpy as np
import pytest
import torch

import meshgen
import paper_2210_12253_amd as lor
from oracle import lor_oracle as orc
from tests.gpu_helpers import row_rel_err, transpose_perm

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda:0")

CASES = [(3, 2, 2), (5, 2, 3), (5, 1, 5), (3, 2, 6)]   # (sides, layers, p)


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _mesh(sides, layers, p):
    m = meshgen.prism_mesh(p, sides, layers, 0.12)
    kap = meshgen.kappa_field(m["nel"], p, 1.0, seed=sides + 10 * p)
    return m, kap


def _check(pat, rp, ci, v64, v32, v):
    assert pat.nnz == rp[-1].item()
    assert torch.equal(pat.row_ptr.cpu().to(torch.int64), rp)
    assert torch.equal(pat.col_idx.cpu().to(torch.int64), ci)
    e64, e32 = row_rel_err(rp, ci, v64, ci, v), row_rel_err(rp, ci, v32, ci, v)
    _say(f"  colours {pat.ncolors} nnz {pat.nnz} fp64 {e64:.2e} fp32 {e32:.2e}")
    assert e64 <= 1e-12 and e32 <= 1e-6
    t = torch.from_numpy(transpose_perm(rp, ci))
    assert torch.equal(v64, v64[t]) and torch.equal(v32, v32[t])


@pytest.mark.parametrize("case", CASES, ids=[f"s{c[0]}l{c[1]}p{c[2]}" for c in CASES])
def test_prism_h1_parity(case):
    sides, layers, p = case
    _say("h1 prism", case)
    m, kap = _mesh(sides, layers, p)
    rp, ci, v = orc.h1_matrix(m["coords"], m["elem_dofs"], p, kap, 1.0)
    ed = torch.from_numpy(m["elem_dofs"])
    pat = lor.lor_pattern(lor.LOR_H1, p, ed.to(DEV), m["ndofs"])
    if layers == 2:
        assert pat.ncolors >= 2 * sides   # every element touches the axis vertex of the middle level
    x = torch.from_numpy(m["coords"])
    v64 = lor.lor_assemble_h1(pat, ed, x, kap, 1.0).cpu()
    v32 = lor.lor_assemble_h1(pat, ed, x, kap.float(), 1.0, dtype=torch.float32, fp64_fallback=True).cpu()
    torch.cuda.synchronize()
    _check(pat, rp, ci, v64, v32, v)
    assert torch.equal(v64, lor.lor_assemble_h1(pat, ed, x, kap, 1.0).cpu())


@pytest.mark.parametrize("case", [c for c in CASES if c[2] <= 5], ids=[f"s{c[0]}l{c[1]}p{c[2]}" for c in CASES
                                                                    if c[2] <= 5])
def test_prism_nd_parity(case):
    sides, layers, p = case
    _say("nd prism", case)
    m, kap = _mesh(sides, layers, p)
    ee, ned = meshgen.edge_map_from_vertices(m["elem_dofs"], p)
    rp, ci, v = orc.nd_matrix(m["coords"], m["elem_dofs"], ee, p, kap, 0.8, ned)
    pat = lor.lor_pattern(lor.LOR_ND, p, torch.from_numpy(ee).to(DEV), ned)
    args = (torch.from_numpy(m["elem_dofs"]), torch.from_numpy(ee), torch.from_numpy(m["coords"]))
    v64 = lor.lor_assemble_nd(pat, *args, kap, 0.8, m["ndofs"]).cpu()
    v32 = lor.lor_assemble_nd(pat, *args, kap.float(), 0.8, m["ndofs"], dtype=torch.float32,
                              fp64_fallback=True).cpu()
    torch.cuda.synchronize()
    _check(pat, rp, ci, v64, v32, v)


@pytest.mark.parametrize("case", CASES, ids=[f"s{c[0]}l{c[1]}p{c[2]}" for c in CASES])
def test_prism_rt_parity(case):
    sides, layers, p = case
    _say("rt prism", case)
    m, kap = _mesh(sides, layers, p)
    fm, nf = meshgen.face_map_from_vertices(m["elem_dofs"], p)
    rp, ci, v = orc.rt_matrix(m["coords"], m["elem_dofs"], fm, p, kap, 1.3, nf)
    pat = lor.lor_pattern(lor.LOR_RT, p, torch.from_numpy(fm).to(DEV), nf)
    args = (torch.from_numpy(m["elem_dofs"]), torch.from_numpy(fm), torch.from_numpy(m["coords"]))
    v64 = lor.lor_assemble_rt(pat, *args, kap, 1.3, m["ndofs"]).cpu()
    v32 = lor.lor_assemble_rt(pat, *args, kap.float(), 1.3, m["ndofs"], dtype=torch.float32,
                              fp64_fallback=True).cpu()
    torch.cuda.synchronize()
    _check(pat, rp, ci, v64, v32, v)


@pytest.mark.parametrize("case", [(3, 2), (5, 3), (5, 6)], ids=["s3p2", "s5p3", "s5p6"])
def test_polygon_2d_parity(case):
    """2D H1 on the polygon cut into quadrilaterals around its centre (the
    centre row couples 1 + 2 sides vertices)."""
    sides, p = case
    _say("h1_2d polygon", case)
    m = meshgen.polygon_mesh_2d(p, sides, 0.12)
    kap = meshgen.kappa_field_2d(m["nel"], p, 1.0, seed=sides * p)
    rp, ci, v = orc.h1_matrix_2d(m["coords"], m["elem_dofs"], p, kap, 0.7, m["ndofs"])
    ed, x = torch.from_numpy(m["elem_dofs"]), torch.from_numpy(m["coords"])
    pat = lor.lor_pattern(lor.LOR_H1_2D, p, ed.to(DEV), m["ndofs"])
    assert pat.ncolors >= sides
    v64 = lor.lor_assemble_h1_2d(pat, ed, x, kap, 0.7).cpu()
    v32 = lor.lor_assemble_h1_2d(pat, ed, x, kap.float(), 0.7, dtype=torch.float32, fp64_fallback=True).cpu()
    torch.cuda.synchronize()
    _check(pat, rp, ci, v64, v32, v)


@pytest.mark.parametrize("case", [(3, 2, 2, 2), (5, 1, 3, 3)], ids=["s3l2p2B2", "s5l1p3B3"])
def test_prism_backward_parity(case):
    """The adjoint on the prism against autograd through the oracle."""
    from tests.test_gpu_backward import oracle_loss_grads
    sides, layers, p, batch = case
    _say("backward prism", case)
    m = meshgen.prism_mesh(p, sides, layers, 0.12)
    kap = meshgen.kappa_field(m["nel"], p, 1.0, seed=5, batch=batch)
    rp, ci, _ = orc.h1_matrix(m["coords"], m["elem_dofs"], p, kap[0], 0.7)
    cot = meshgen.cotangent(batch, rp[-1].item(), seed=1)
    gk_ref, gx_ref = oracle_loss_grads(m, p, kap, 0.7, cot, rp, ci)
    ed, x = torch.from_numpy(m["elem_dofs"]), torch.from_numpy(m["coords"])
    pat = lor.lor_pattern(lor.LOR_H1, p, ed.to(DEV), m["ndofs"])
    for dtype, tol in ((torch.float64, 1e-10), (torch.float32, 1e-5)):
        gk, gx = lor.lor_assemble_backward(pat, ed, x, kap.to(dtype), 0.7, cot.to(dtype), dtype=dtype)
        torch.cuda.synchronize()
        ek = float((gk.cpu().double() - gk_ref).abs().max() / gk_ref.abs().max())
        ex = float((gx.cpu() - gx_ref).abs().max() / gx_ref.abs().max())
        _say(f"  {dtype}: kappa {ek:.2e} coords {ex:.2e}")
        assert ek <= tol and ex <= tol


@pytest.mark.parametrize("case", [(3, 2, 2), (5, 2, 3)], ids=["s3l2p2", "s5l2p3"])
def test_prism_discrete_gradient_and_curl(case):
    """Bit-exact discrete gradient and curl on the prism (first incidence from
    the schedule and from the face-owner pass on an irregular mesh)."""
    sides, layers, p = case
    _say("aux prism", case)
    m = meshgen.prism_mesh(p, sides, layers, 0.0)
    ee, ned = meshgen.edge_map_from_vertices(m["elem_dofs"], p)
    fm, nf = meshgen.face_map_from_vertices(m["elem_dofs"], p)
    rp, ci, v = orc.discrete_gradient(m["elem_dofs"], ee, p, ned)
    pat = lor.lor_pattern(lor.LOR_ND, p, torch.from_numpy(ee).to(DEV), ned)
    grp, gci, gv = lor.lor_discrete_gradient(pat, m["elem_dofs"], ee, m["ndofs"])
    torch.cuda.synchronize()
    assert torch.equal(grp.cpu().to(torch.int64), rp)
    assert torch.equal(gci.cpu().to(torch.int64), ci)
    assert torch.equal(gv.cpu(), v)
    rp, ci, v = orc.discrete_curl(ee, fm, p, nf)
    crp, cci, cv = lor.lor_discrete_curl(p, ee, fm, ned, nf, device=DEV)
    torch.cuda.synchronize()
    assert torch.equal(crp.cpu().to(torch.int64), rp)
    assert torch.equal(cci.cpu().to(torch.int64), ci)
    assert torch.equal(cv.cpu(), v)


TRI = [(6, 3, 2), (4, 2, 3), (2, 2, 6), (3, 1, 5)]   # (n, layers, p)


@pytest.mark.parametrize("case", TRI, ids=[f"n{c[0]}l{c[1]}p{c[2]}" for c in TRI])
def test_tri_split_parity(case):
    n, layers, p = case
    _say("tri-split", case)
    m = meshgen.tri_split_mesh(n, layers, p, 0.1)
    kap = meshgen.kappa_field(m["nel"], p, 1.0, seed=n + 10 * p)
    ed, x = torch.from_numpy(m["elem_dofs"]), torch.from_numpy(m["coords"])
    rp, ci, v = orc.h1_matrix(m["coords"], m["elem_dofs"], p, kap, 1.0)
    pat = lor.lor_pattern(lor.LOR_H1, p, ed.to(DEV), m["ndofs"])
    v64 = lor.lor_assemble_h1(pat, ed, x, kap, 1.0).cpu()
    v32 = lor.lor_assemble_h1(pat, ed, x, kap.float(), 1.0, dtype=torch.float32, fp64_fallback=True).cpu()
    torch.cuda.synchronize()
    _check(pat, rp, ci, v64, v32, v)
    if p <= 5:
        ee, ned = meshgen.edge_map_from_vertices(m["elem_dofs"], p)
        rp, ci, v = orc.nd_matrix(m["coords"], m["elem_dofs"], ee, p, kap, 0.8, ned)
        pat = lor.lor_pattern(lor.LOR_ND, p, torch.from_numpy(ee).to(DEV), ned)
        v64 = lor.lor_assemble_nd(pat, ed, torch.from_numpy(ee), x, kap, 0.8, m["ndofs"]).cpu()
        v32 = lor.lor_assemble_nd(pat, ed, torch.from_numpy(ee), x, kap.float(), 0.8, m["ndofs"],
                                  dtype=torch.float32, fp64_fallback=True).cpu()
        torch.cuda.synchronize()
        _check(pat, rp, ci, v64, v32, v)
    fm, nf = meshgen.face_map_from_vertices(m["elem_dofs"], p)
    rp, ci, v = orc.rt_matrix(m["coords"], m["elem_dofs"], fm, p, kap, 1.3, nf)
    pat = lor.lor_pattern(lor.LOR_RT, p, torch.from_numpy(fm).to(DEV), nf)
    v64 = lor.lor_assemble_rt(pat, ed, torch.from_numpy(fm), x, kap, 1.3, m["ndofs"]).cpu()
    v32 = lor.lor_assemble_rt(pat, ed, torch.from_numpy(fm), x, kap.float(), 1.3, m["ndofs"],
                              dtype=torch.float32, fp64_fallback=True).cpu()
    torch.cuda.synchronize()
    _check(pat, rp, ci, v64, v32, v)


@pytest.mark.parametrize("case", [(8, 4), (4, 6), (6, 1)], ids=["n8p4", "n4p6", "n6p1"])
def test_tri_split_2d_parity(case):
    n, p = case
    _say("tri-split 2d", case)
    m = meshgen.tri_split_mesh_2d(n, p, 0.1)
    kap = meshgen.kappa_field_2d(m["nel"], p, 1.0, seed=n * p)
    rp, ci, v = orc.h1_matrix_2d(m["coords"], m["elem_dofs"], p, kap, 0.7, m["ndofs"])
    ed, x = torch.from_numpy(m["elem_dofs"]), torch.from_numpy(m["coords"])
    pat = lor.lor_pattern(lor.LOR_H1_2D, p, ed.to(DEV), m["ndofs"])
    v64 = lor.lor_assemble_h1_2d(pat, ed, x, kap, 0.7).cpu()
    v32 = lor.lor_assemble_h1_2d(pat, ed, x, kap.float(), 0.7, dtype=torch.float32, fp64_fallback=True).cpu()
    torch.cuda.synchronize()
    _check(pat, rp, ci, v64, v32, v)


def test_tri_split_backward_and_aux():
    """The adjoint (batch 2) and the bit-exact discrete gradient and curl on
    the triangle-split cube, n = 3, 2 layers, p = 3 (108 elements)."""
    from tests.test_gpu_backward import oracle_loss_grads
    n, layers, p = 3, 2, 3
    m = meshgen.tri_split_mesh(n, layers, p, 0.1)
    kap = meshgen.kappa_field(m["nel"], p, 1.0, seed=9, batch=2)
    rp, ci, _ = orc.h1_matrix(m["coords"], m["elem_dofs"], p, kap[0], 0.7)
    cot = meshgen.cotangent(2, rp[-1].item(), seed=1)
    gk_ref, gx_ref = oracle_loss_grads(m, p, kap, 0.7, cot, rp, ci)
    ed, x = torch.from_numpy(m["elem_dofs"]), torch.from_numpy(m["coords"])
    pat = lor.lor_pattern(lor.LOR_H1, p, ed.to(DEV), m["ndofs"])
    for dtype, tol in ((torch.float64, 1e-10), (torch.float32, 1e-5)):
        gk, gx = lor.lor_assemble_backward(pat, ed, x, kap.to(dtype), 0.7, cot.to(dtype), dtype=dtype)
        torch.cuda.synchronize()
        ek = float((gk.cpu().double() - gk_ref).abs().max() / gk_ref.abs().max())
        ex = float((gx.cpu() - gx_ref).abs().max() / gx_ref.abs().max())
        _say(f"  backward {dtype}: kappa {ek:.2e} coords {ex:.2e}")
        assert ek <= tol and ex <= tol
    ee, ned = meshgen.edge_map_from_vertices(m["elem_dofs"], p)
    fm, nf = meshgen.face_map_from_vertices(m["elem_dofs"], p)
    rp, ci, v = orc.discrete_gradient(m["elem_dofs"], ee, p, ned)
    pat = lor.lor_pattern(lor.LOR_ND, p, torch.from_numpy(ee).to(DEV), ned)
    grp, gci, gv = lor.lor_discrete_gradient(pat, m["elem_dofs"], ee, m["ndofs"])
    torch.cuda.synchronize()
    assert torch.equal(grp.cpu().to(torch.int64), rp) and torch.equal(gci.cpu().to(torch.int64), ci)
    assert torch.equal(gv.cpu(), v)
    rp, ci, v = orc.discrete_curl(ee, fm, p, nf)
    crp, cci, cv = lor.lor_discrete_curl(p, ee, fm, ned, nf, device=DEV)
    torch.cuda.synchronize()
    assert torch.equal(crp.cpu().to(torch.int64), rp) and torch.equal(cci.cpu().to(torch.int64), ci)
    assert torch.equal(cv.cpu(), v)


def test_tri_split_headline_size():
    """The headline form on the triangle-split mesh at the headline size
    (32,256 hexahedra, p = 6, 7,071,487 rows), in the launch configuration the
    benchmark times: sampled rows (including vertices of valence 3 and 6)
    against the oracle in FP64 and FP32, the whole-matrix properties, and the
    total of all entries equal to the unit volume (the boundary lattice is
    symmetric about 1/2 on every face, so the sinusoidal map keeps it)."""
    from tests.gpu_helpers import check_whole_matrix
    m = meshgen.config_mesh("c8_h1_p6_trisplit")
    ed, x = torch.from_numpy(m["elem_dofs"]), torch.from_numpy(m["coords"])
    pat = lor.lor_pattern(lor.LOR_H1, 6, ed.to(DEV), m["ndofs"])
    v64 = lor.lor_assemble_h1(pat, ed, x, m["kappa"], 1.0)
    v32 = lor.lor_assemble_h1(pat, ed, x, m["kappa"].float(), 1.0, dtype=torch.float32, fp64_fallback=True)
    torch.cuda.synchronize()
    grp = pat.row_ptr.cpu().to(torch.int64)
    lens = grp[1:] - grp[:-1]
    rng = np.random.default_rng(2)
    longest = torch.nonzero(lens == lens.max()).flatten()[:20].tolist()     # valence-6 vertices
    pick = longest + [0, m["ndofs"] - 1] + list(rng.integers(0, m["ndofs"], size=300))
    rows, rp, ci, v = orc.h1_rows(m["coords"], m["elem_dofs"], 6, m["kappa"], 1.0, torch.tensor(pick))
    idx = torch.cat([torch.arange(grp[r], grp[r + 1]) for r in rows.tolist()])
    assert torch.equal(pat.col_idx.cpu().to(torch.int64)[idx], ci)
    e64 = row_rel_err(rp, ci, v64.cpu()[idx], ci, v)
    e32 = row_rel_err(rp, ci, v32.cpu()[idx], ci, v)
    s64, a64 = float(v64.sum()), float(v64.abs().sum())
    _say(f"  colours {pat.ncolors} max row {int(lens.max())} fp64 {e64:.2e} fp32 {e32:.2e} sum-1 {s64 - 1:.2e} "
         f"|A| {a64:.3e}")
    assert int(lens.max()) == 39
    assert e64 <= 1e-12 and e32 <= 1e-6
    check_whole_matrix(pat, v64, v32)
    assert abs(s64 - 1.0) <= 1e-17 * a64
