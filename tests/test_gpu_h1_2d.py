"""GPU parity of the 2D LOR H1 path against the CPU oracle, through the C ABI."""
import json
import os
import sys

import numpy as np
import pytest
import torch

import meshgen
import paper_2210_12253_amd as lor
from oracle import lor_oracle as orc
from tests.gpu_helpers import check_whole_matrix, row_rel_err, transpose_perm

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda:0")
GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _assemble(pat, m, kap, beta, dtype=torch.float64, **kw):
    v = lor.lor_assemble_h1_2d(pat, torch.from_numpy(m["elem_dofs"]), torch.from_numpy(m["coords"]), kap, beta,
                               dtype=dtype, **kw)
    torch.cuda.synchronize()
    return v.cpu()


CASES = [(3, 1, 0.1, False), (4, 2, 0.12, True), (3, 3, 0.1, False), (2, 4, 0.1, True), (2, 5, 0.1, False),
         (3, 6, 0.1, True)]


@pytest.mark.parametrize("case", CASES, ids=[f"n{c[0]}p{c[1]}-r{int(c[3])}" for c in CASES])
def test_h1_2d_small_parity(case):
    n, p, amp, renumber = case
    _say("case", case)
    m = meshgen.cartesian_mesh_2d(n, p, amp)
    if renumber:
        m, _ = meshgen.renumber_vertices(m, seed=n + p)
    kap = meshgen.kappa_field_2d(m["nel"], p, 1.0, seed=n * p)
    rp, ci, v = orc.h1_matrix_2d(m["coords"], m["elem_dofs"], p, kap, 0.7, m["ndofs"])
    pat = lor.lor_pattern(lor.LOR_H1_2D, p, torch.from_numpy(m["elem_dofs"]).to(DEV), m["ndofs"])
    assert torch.equal(pat.row_ptr.cpu().to(torch.int64), rp)
    assert torch.equal(pat.col_idx.cpu().to(torch.int64), ci)
    v64 = _assemble(pat, m, kap, 0.7)
    v32 = _assemble(pat, m, kap.float(), 0.7, dtype=torch.float32, fp64_fallback=True)
    e64 = row_rel_err(rp, ci, v64, ci, v)
    e32 = row_rel_err(rp, ci, v32, ci, v)
    _say(f"  fp64 {e64:.2e} fp32 {e32:.2e} colours {pat.ncolors}")
    assert e64 <= 1e-12 and e32 <= 1e-6
    assert torch.equal(v64, v64[transpose_perm(rp, ci)])


BOX2D = [(12, 5, 6, 0.1, True), (7, 9, 1, 0.15, False), (3, 4, 3, 0.1, True), (1, 1, 2, 0.0, False),
         (70, 1, 1, 0.05, True)]


@pytest.mark.parametrize("case", BOX2D, ids=[f"{c[0]}x{c[1]}p{c[2]}-perm{int(c[4])}" for c in BOX2D])
def test_h1_2d_owner_parity(case):
    """2D box lattices (also rectangular, with the elements in any order) get
    the owner-computes schedule; both kernels in both forms against the
    oracle, every row (row-relative 1e-12 FP64, 1e-6 FP32), the owner kernel
    bitwise symmetric and deterministic.  12 x 5 at p = 6 spans two strips
    of 64 cells (72 cells per line) and several segments along y; 70 x 1 at
    p = 1 two strips with a short last one."""
    nx, ny, p, amp, perm = case
    _say("case", case)
    m = meshgen.box_mesh_2d(nx, ny, p, amp)
    kap = meshgen.kappa_field_2d(m["nel"], p, 1.0, seed=nx + ny + p)
    if perm:
        m, order = meshgen.permute_elements(m, seed=nx * ny)
        kap = kap[torch.from_numpy(order)]
    rp, ci, v = orc.h1_matrix_2d(m["coords"], m["elem_dofs"], p, kap, 0.6, m["ndofs"])
    pat = lor.lor_pattern(lor.LOR_H1_2D, p, torch.from_numpy(m["elem_dofs"]).to(DEV), m["ndofs"])
    assert pat.owner
    assert torch.equal(pat.row_ptr.cpu().to(torch.int64), rp)
    assert torch.equal(pat.col_idx.cpu().to(torch.int64), ci)
    tp = transpose_perm(rp, ci)
    for kern in ("owner", "colored"):
        diag = torch.zeros(2, dtype=torch.int32, device=DEV)
        v64 = _assemble(pat, m, kap, 0.6, kernel=kern, diag=diag)
        v32 = _assemble(pat, m, kap.float(), 0.6, dtype=torch.float32, fp64_fallback=True, kernel=kern)
        e64 = row_rel_err(rp, ci, v64, ci, v)
        e32 = row_rel_err(rp, ci, v32, ci, v)
        _say(f"  {kern}: fp64 {e64:.2e} fp32 {e32:.2e} diag {diag.cpu().tolist()}")
        assert e64 <= 1e-12 and e32 <= 1e-6
        assert diag.cpu().tolist() == [0, 0]
        assert torch.equal(v64, v64[tp]) and torch.equal(v32, v32[tp])
        if kern == "owner":
            assert torch.equal(v64, _assemble(pat, m, kap, 0.6, kernel=kern))


def test_h1_2d_owner_not_a_box():
    """Renumbered vertices: no owner-computes schedule; asking for it fails
    with LOR_EUNSUPPORTED and the default takes the coloured kernel."""
    m = meshgen.cartesian_mesh_2d(3, 2, 0.1)
    m, _ = meshgen.renumber_vertices(m, seed=4)
    kap = meshgen.kappa_field_2d(m["nel"], 2, 1.0, seed=1)
    pat = lor.lor_pattern(lor.LOR_H1_2D, 2, torch.from_numpy(m["elem_dofs"]).to(DEV), m["ndofs"])
    assert not pat.owner
    with pytest.raises(lor.LorError):
        _assemble(pat, m, kap, 0.5, kernel="owner")
    assert torch.equal(_assemble(pat, m, kap, 0.5), _assemble(pat, m, kap, 0.5, kernel="colored"))


def test_h1_2d_closed_form_uniform():
    """Uniform square, kappa = 1, beta = 0: interior rows are the Q1 9-point
    stencil 8/3, -1/3 (printed form of the bilinear Laplacian)."""
    n, p = 4, 2
    m = meshgen.cartesian_mesh_2d(n, p, 0.0)
    kap = torch.ones((m["nel"], p * p), dtype=torch.float64)
    pat = lor.lor_pattern(lor.LOR_H1_2D, p, torch.from_numpy(m["elem_dofs"]).to(DEV), m["ndofs"])
    v = _assemble(pat, m, kap, 0.0)
    N = m["N"]
    rp = pat.row_ptr.cpu().long()
    ci = pat.col_idx.cpu().long()
    c = N * 3 + 3
    row = dict(zip(ci[rp[c]:rp[c + 1]].tolist(), v[rp[c]:rp[c + 1]].tolist()))
    assert abs(row[c] - 8.0 / 3.0) <= 1e-14
    for d in (1, -1, N, -N, N + 1, N - 1, -N + 1, -N - 1):
        assert abs(row[c + d] + 1.0 / 3.0) <= 1e-14


def test_h1_2d_full_size_counts_and_sampled_rows():
    """The paper's 2D workload (Section 4.1): 512^2 elements at p = 6 give
    9,443,329 rows and 84,953,089 nonzeros; sampled rows against the oracle."""
    with open(os.path.join(GOLDEN, "paper_counts.json")) as f:
        g = json.load(f)["h1_2d"]
    m = meshgen.config_mesh("c7_h1_2d_p6_curved")
    pat = lor.lor_pattern(lor.LOR_H1_2D, 6, torch.from_numpy(m["elem_dofs"]).to(DEV), m["ndofs"])
    assert m["nel"] == g["elements"] and pat.nrows == g["dofs"] and pat.nnz == g["nnz"]
    v64 = _assemble(pat, m, m["kappa"], m["beta"])
    v32 = _assemble(pat, m, m["kappa"].float(), m["beta"], dtype=torch.float32, fp64_fallback=True)
    N = m["N"]
    rng = np.random.default_rng(0)
    pick = [0, N - 1, N * N - 1, (N // 2) * (N + 1), 6 + 6 * N] + list(rng.integers(0, N * N, size=400))
    rows, rp, ci, v = orc.h1_rows_2d(m["coords"], m["elem_dofs"], 6, m["kappa"], m["beta"], torch.tensor(pick))
    grp = pat.row_ptr.cpu().to(torch.int64)
    idx = torch.cat([torch.arange(grp[r], grp[r + 1]) for r in rows.tolist()])
    assert torch.equal(pat.col_idx.cpu().to(torch.int64)[idx], ci)
    e64 = row_rel_err(rp, ci, v64[idx], ci, v)
    e32 = row_rel_err(rp, ci, v32[idx], ci, v)
    assert pat.owner  # the default above is the owner-computes kernel; the coloured one too
    c64 = _assemble(pat, m, m["kappa"], m["beta"], kernel="colored")
    c32 = _assemble(pat, m, m["kappa"].float(), m["beta"], dtype=torch.float32, fp64_fallback=True, kernel="colored")
    ec64 = row_rel_err(rp, ci, c64[idx], ci, v)
    ec32 = row_rel_err(rp, ci, c32[idx], ci, v)
    _say(f"sampled rows: owner fp64 {e64:.2e} fp32 {e32:.2e}; coloured fp64 {ec64:.2e} fp32 {ec32:.2e}")
    assert e64 <= 1e-12 and e32 <= 1e-6 and ec64 <= 1e-12 and ec32 <= 1e-6
    del c64, c32
    # the whole matrix: sorted rows, symmetric pattern, bitwise symmetric
    # values; and with zero diffusion row sums the entries add up to the area
    # of the mapped square, which is 1 (the boundary displacements A sin(2 pi t)
    # cancel over the lattice, symmetric about 1/2)
    check_whole_matrix(pat, v64.to(DEV), v32.to(DEV))
    s64, a64 = float(v64.sum()), float(v64.abs().sum())
    _say(f"sum fp64 {s64:.15f} (|A| {a64:.3e})")
    assert abs(s64 - 1.0) <= 1e-16 * a64


def test_h1_2d_fp32_fallback_batch_and_empty():
    """A pinched vertex sends its subelements through the FP64 path of the FP32
    form (diag[0]); a batch of kappa fields equals the single calls; an empty
    mesh launches nothing."""
    m = meshgen.cartesian_mesh_2d(1, 2, 0.0)
    X = m["coords"].copy()
    X[4] = [0.96, 0.5]   # corner-Jacobian ratio 12.5 in the two right subelements
    m["coords"] = X
    kap = torch.ones(1, 4, dtype=torch.float64)
    rp, ci, v = orc.h1_matrix_2d(X, m["elem_dofs"], 2, kap, 1.0, m["ndofs"])
    pat = lor.lor_pattern(lor.LOR_H1_2D, 2, torch.from_numpy(m["elem_dofs"]).to(DEV), m["ndofs"])
    diag = torch.zeros(2, dtype=torch.int32, device=DEV)
    v32 = _assemble(pat, m, kap.float(), 1.0, dtype=torch.float32, fp64_fallback=True, det_ratio_thresh=10.0,
                    diag=diag)
    d = diag.cpu().tolist()
    assert d[0] > 0 and d[1] == 0
    assert row_rel_err(rp, ci, v32, ci, v) <= 1e-6
    m = meshgen.cartesian_mesh_2d(3, 3, 0.1)
    pat = lor.lor_pattern(lor.LOR_H1_2D, 3, torch.from_numpy(m["elem_dofs"]).to(DEV), m["ndofs"])
    kb = torch.stack([meshgen.kappa_field_2d(m["nel"], 3, 1.0, seed=s) for s in range(3)])
    vb = _assemble(pat, m, kb, 0.4)
    for b in range(3):
        assert torch.equal(vb[b], _assemble(pat, m, kb[b], 0.4))
    pat0 = lor.lor_pattern(lor.LOR_H1_2D, 2, torch.zeros((0, 9), dtype=torch.int32, device=DEV), 4)
    out = lor.lor_assemble_h1_2d(pat0, torch.zeros((0, 9), dtype=torch.int32), torch.zeros((4, 2), dtype=torch.float64),
                                 torch.zeros((0, 4), dtype=torch.float64), 1.0)
    torch.cuda.synchronize()
    assert pat0.nnz == 0 and out.numel() == 0
