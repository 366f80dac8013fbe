"""GPU parity of the unstructured comparator (explicit LOR mesh, per-element
dense matrices, atomic adds) against the CPU oracle, through the C ABI."""
import sys

import numpy as np
import pytest
import torch

import meshgen
import paper_2210_12253_amd as lor
from oracle import lor_oracle as orc
from tests.gpu_helpers import row_rel_err

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda:0")


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.mark.parametrize("n,p", [(2, 1), (2, 3), (1, 6)])
def test_refine_map_matches_oracle(n, p):
    m, _ = meshgen.renumber_vertices(meshgen.cartesian_mesh(n, p, 0.0), seed=n + p)
    want = orc.h1_subelement_vertices(torch.from_numpy(m["elem_dofs"]), p).reshape(-1, 8)
    got = lor.lor_refine_map(p, m["elem_dofs"], device=DEV)
    torch.cuda.synchronize()
    assert torch.equal(got.cpu().to(torch.int64), want.to(torch.int64))


CASES = [(2, 1, 0.1), (3, 2, 0.12), (2, 3, 0.1), (1, 4, 0.1), (1, 6, 0.1)]


@pytest.mark.parametrize("case", CASES, ids=[f"n{c[0]}p{c[1]}" for c in CASES])
def test_unstructured_small_parity(case):
    n, p, amp = case
    _say("case", case)
    m = meshgen.cartesian_mesh(n, p, amp)
    kap = meshgen.kappa_field(m["nel"], p, 1.0, seed=n + p)
    rp, ci, v = orc.h1_matrix(m["coords"], m["elem_dofs"], p, kap, 0.8)
    pat = lor.lor_pattern(lor.LOR_H1, p, torch.from_numpy(m["elem_dofs"]).to(DEV), m["ndofs"])
    sub = lor.lor_refine_map(p, m["elem_dofs"], device=DEV)
    diag = torch.zeros(2, dtype=torch.int32, device=DEV)
    got = lor.lor_assemble_h1_unstructured(pat, sub, m["coords"], kap, 0.8, diag=diag)
    torch.cuda.synchronize()
    assert diag.cpu().tolist() == [0, 0]
    e = row_rel_err(rp, ci, got.cpu(), ci, v)
    _say(f"  row-rel err {e:.2e}")
    assert e <= 1e-12


def test_unstructured_full_size_sampled_rows():
    """The headline mesh (p=6, 32^3): sampled rows against the oracle, and the
    whole matrix against the macro-element kernel (two independent GPU paths,
    agreeing to rounding)."""
    m = meshgen.config_mesh("c3_h1_p6_curved")
    ed = torch.from_numpy(m["elem_dofs"]).to(DEV)
    pat = lor.lor_pattern(lor.LOR_H1, 6, ed, m["ndofs"])
    sub = lor.lor_refine_map(6, ed, device=DEV)
    got = lor.lor_assemble_h1_unstructured(pat, sub, m["coords"], m["kappa"], m["beta"])
    macro = lor.lor_assemble_h1(pat, ed, m["coords"], m["kappa"], m["beta"])
    torch.cuda.synchronize()
    N = m["N"]
    rng = np.random.default_rng(1)
    pick = [0, N * N - 1, (N // 2) * (1 + N + N * N)] + list(rng.integers(0, N ** 3, size=200))
    rows, rp, ci, v = orc.h1_rows(m["coords"], m["elem_dofs"], 6, m["kappa"], m["beta"], torch.tensor(pick))
    grp = pat.row_ptr.cpu().to(torch.int64)
    idx = torch.cat([torch.arange(grp[r], grp[r + 1]) for r in rows.tolist()])
    assert row_rel_err(rp, ci, got.cpu()[idx], ci, v) <= 1e-12
    rowmax = torch.zeros(pat.nrows, dtype=torch.float64, device=DEV)
    r_of = torch.repeat_interleave(torch.arange(pat.nrows, device=DEV),
                                   (pat.row_ptr[1:] - pat.row_ptr[:-1]).long())
    rowmax.scatter_reduce_(0, r_of, macro.abs(), reduce="amax")
    rel = ((got - macro).abs() / rowmax[r_of]).max()
    assert float(rel) <= 1e-12
