"""GPU parity of the owner-computes H1 kernel (every row summed once and
written whole) against the CPU oracle, and its agreement with the coloured
kernel, through the C ABI.  Which meshes get the owner-computes schedule is
checked too: lattice-continuing meshes (Cartesian, elements permuted) do;
renumbered vertices, rotated elements and irregular-valence meshes do not."""
import sys

import pytest
import torch

import meshgen
import paper_2210_12253_amd as lor
from oracle import lor_oracle as orc
from tests.gpu_helpers import row_rel_err, transpose_perm

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda:0")


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _pattern(m):
    return lor.lor_pattern(lor.LOR_H1, m["p"], torch.from_numpy(m["elem_dofs"]).to(DEV), m["ndofs"])


def _assemble(pat, m, kap, beta, dtype=torch.float64, **kw):
    v = lor.lor_assemble_h1(pat, torch.from_numpy(m["elem_dofs"]), torch.from_numpy(m["coords"]), kap, beta,
                            dtype=dtype, **kw)
    torch.cuda.synchronize()
    return v.cpu()


def _mesh(n, p, amp, sigma, pert, seed=0):
    m = meshgen.cartesian_mesh(n, p, amp)
    kap = meshgen.kappa_field(m["nel"], p, sigma, seed=seed)
    if pert == "permute":
        m, order = meshgen.permute_elements(m, seed=seed + 4)
        kap = kap[torch.from_numpy(order)]
    elif pert == "renumber":
        m, _ = meshgen.renumber_vertices(m, seed=seed + 3)
    elif pert == "reorient":
        m, kap, _ = meshgen.reorient_elements(m, seed=seed + 5, kappa=kap)
    return m, kap


def test_owner_schedule_eligibility():
    for p in range(1, 7):
        m, _ = _mesh(2, p, 0.1, 1.0, None)
        assert _pattern(m).owner, p
    for pert, want in (("permute", True), ("renumber", False), ("reorient", False)):
        m, _ = _mesh(3, 2, 0.1, 1.0, pert)
        assert _pattern(m).owner == want, pert
    pm = meshgen.prism_mesh(3, sides=5, layers=2, amp=0.1)
    assert not lor.lor_pattern(lor.LOR_H1, 3, torch.from_numpy(pm["elem_dofs"]).to(DEV), pm["ndofs"]).owner
    ts = meshgen.tri_split_mesh(2, 2, 2, amp=0.1)
    assert not lor.lor_pattern(lor.LOR_H1, 2, torch.from_numpy(ts["elem_dofs"]).to(DEV), ts["ndofs"]).owner


# (n, p, amp, sigma, beta, perturbation): np > 7 cells gives several 8 x 8
# tiles per plane (overlapping by one cell), np > 8 several z-segments (a
# segment above the bottom starts with the layer below it)
CASES = [
    (2, 1, 0.1, 1.0, 1.0, None),
    (5, 1, 0.1, 1.0, 0.5, "permute"),
    (5, 2, 0.15, 1.0, 1.0, None),
    (3, 2, 0.0, 0.0, 0.0, None),
    (6, 3, 0.12, 2.0, 1.0, "permute"),
    (2, 4, 0.12, 1.0, 1.0, None),
    (5, 4, 0.1, 1.0, 1.0, "permute"),
    (3, 5, 0.12, 1.0, 1.0, None),
    (9, 5, 0.1, 1.0, 1.0, None),
    (2, 6, 0.12, 2.0, 1.0, "permute"),
    (9, 6, 0.1, 2.0, 1.0, None),
]


@pytest.mark.parametrize("case", CASES, ids=[f"n{c[0]}p{c[1]}-{c[5]}" for c in CASES])
def test_owner_small_parity(case):
    n, p, amp, sigma, beta, pert = case
    _say("owner case", case)
    m, kap = _mesh(n, p, amp, sigma, pert)
    if sigma == 0.0:
        kap = torch.ones_like(kap)
    rp, ci, v = orc.h1_matrix(m["coords"], m["elem_dofs"], p, kap, beta)
    pat = _pattern(m)
    assert pat.owner
    assert torch.equal(pat.row_ptr.cpu().to(torch.int64), rp)
    assert torch.equal(pat.col_idx.cpu().to(torch.int64), ci)
    # every entry is written: poison the output first
    out = torch.full((pat.nnz,), float("nan"), dtype=torch.float64, device=DEV)
    v64 = _assemble(pat, m, kap, beta, kernel="owner", out=out)
    assert row_rel_err(rp, ci, v64, ci, v) <= 1e-12
    out32 = torch.full((pat.nnz,), float("nan"), dtype=torch.float32, device=DEV)
    v32 = _assemble(pat, m, kap.float(), beta, dtype=torch.float32, kernel="owner", out=out32)
    assert row_rel_err(rp, ci, v32, ci, v) <= 1e-6
    # determinism and bitwise symmetry
    assert torch.equal(v64, _assemble(pat, m, kap, beta, kernel="owner"))
    t = torch.from_numpy(transpose_perm(rp, ci))
    assert torch.equal(v64, v64[t])
    assert torch.equal(v32, v32[t])
    # same matrix as the coloured kernel, up to the order of the sums
    vc = _assemble(pat, m, kap, beta, kernel="colored")
    assert row_rel_err(rp, ci, v64, ci, vc) <= 1e-13
    # the default is the owner-computes kernel on this mesh
    assert torch.equal(_assemble(pat, m, kap.float(), beta, dtype=torch.float32), v32)
    assert torch.equal(_assemble(pat, m, kap, beta), v64)


def test_owner_batch_matches_single():
    m = meshgen.cartesian_mesh(5, 3, 0.1)
    kb = meshgen.kappa_field(m["nel"], 3, 1.0, seed=2, batch=3)
    pat = _pattern(m)
    vb = _assemble(pat, m, kb, 0.7, kernel="owner")
    for b in range(3):
        assert torch.equal(vb[b], _assemble(pat, m, kb[b], 0.7, kernel="owner"))
    vb32 = _assemble(pat, m, kb.float(), 0.7, dtype=torch.float32, kernel="owner")
    for b in range(3):
        assert torch.equal(vb32[b], _assemble(pat, m, kb[b].float(), 0.7, dtype=torch.float32, kernel="owner"))


def test_owner_fp32_fallback_and_counters():
    """The pinched vertex of the coloured kernel's fallback test: the
    owner-computes kernel counts each fallback cell once (not again where a
    neighbouring tile integrates it too) and matches the oracle to 1e-6."""
    m = meshgen.cartesian_mesh(2, 2, 0.0)
    X = m["coords"].copy()
    N = m["N"]
    c = 1 + N * (1 + N * 1)        # an interior vertex of element 0
    X[c] = X[c] + [0.23, 0.0, 0.0]
    m["coords"] = X
    kap = torch.ones(m["nel"], 8, dtype=torch.float64)
    rp, ci, v = orc.h1_matrix(X, m["elem_dofs"], 2, kap, 1.0)
    pat = _pattern(m)
    assert pat.owner
    counts = {}
    for kern in ("owner", "colored"):
        diag = torch.zeros(2, dtype=torch.int32, device=DEV)
        v32 = _assemble(pat, m, kap.float(), 1.0, dtype=torch.float32, fp64_fallback=True, det_ratio_thresh=10.0,
                        diag=diag, kernel=kern)
        counts[kern] = diag.cpu().tolist()
        assert row_rel_err(rp, ci, v32, ci, v) <= 1e-6
    assert counts["owner"] == counts["colored"] and counts["owner"][0] > 0


def test_owner_inverted_cells_counted_once():
    m = meshgen.cartesian_mesh(3, 2, 0.0)
    X = m["coords"].copy()
    N = m["N"]
    c = 2 + N * (2 + N * 2)        # shared by 8 elements
    X[c] = X[c] + [0.3, 0.3, 0.3]  # past its neighbours: some cells invert
    m["coords"] = X
    kap = torch.ones(m["nel"], 8, dtype=torch.float64)
    pat = _pattern(m)
    counts = {}
    for kern in ("owner", "colored"):
        diag = torch.zeros(2, dtype=torch.int32, device=DEV)
        _assemble(pat, m, kap, 1.0, diag=diag, kernel=kern)
        counts[kern] = diag.cpu().tolist()
    assert counts["owner"] == counts["colored"] and counts["owner"][1] > 0


def test_owner_flag_errors():
    m, kap = _mesh(2, 2, 0.1, 1.0, "renumber")
    pat = _pattern(m)
    assert not pat.owner
    with pytest.raises(lor.LorError, match="owner-computes"):
        _assemble(pat, m, kap, 1.0, kernel="owner")
    # auto falls back to the coloured kernel
    rp, ci, v = orc.h1_matrix(m["coords"], m["elem_dofs"], 2, kap, 1.0)
    assert row_rel_err(rp, ci, _assemble(pat, m, kap, 1.0), ci, v) <= 1e-12
    lib = lor.load_library()
    rc = lib.lor_assemble_h1(2, pat.nel, pat.nrows, 1, 0x1000, 0x1000, 0x1000, 1.0, 0x1000,
                             lor.lor.ctypes.byref(pat.sched), 0x1000, 0, lor.lor.LOR_COLORED | lor.lor.LOR_OWNER,
                             10.0, None, None)
    assert rc == lor.lor.LOR_EINVAL
