"""GPU parity of essential-BC elimination (step A4) against the CPU oracle,
through the C ABI (Python binding).  Elimination only copies, zeroes or sets
entries to 1, so the comparison is bit-exact."""
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


def _oracle_pattern(space, n, p):
    """CSR pattern (and a vertex/edge count) from the oracle's assembly."""
    m = meshgen.cartesian_mesh(n, p, 0.1)
    kap = meshgen.kappa_field(m["nel"], p, 1.0, seed=n + p)
    if space == "h1":
        rp, ci, _ = orc.h1_matrix(m["coords"], m["elem_dofs"], p, kap, 1.0)
        return rp, ci, m["ndofs"], meshgen.boundary_vertices(n, p)
    ee, ned = meshgen.nd_edge_map(n, p)
    rp, ci, _ = orc.nd_matrix(m["coords"], m["elem_dofs"], ee, p, kap, 1.0, ned)
    return rp, ci, ned, meshgen.boundary_edges(n, p)


def _pattern_on_device(rp, ci, nrows):
    rpd = rp.to(torch.int32).to(DEV)
    cid = ci.to(torch.int32).to(DEV)
    return lor.Pattern(lor.LOR_H1, 1, 0, nrows, int(rp[-1]), rpd, cid, None, None)


def _ess_sets(nrows, bnd):
    return {
        "random_repeats": meshgen.random_dofs(nrows, max(1, nrows // 4), seed=nrows),
        "boundary": bnd,
        "empty": np.zeros(0, np.int32),
        "all": np.arange(nrows, dtype=np.int32)[::-1].copy(),
    }


CASES = [("h1", 3, 2), ("h1", 2, 1), ("h1", 1, 6), ("nd", 2, 2), ("nd", 1, 3)]


@pytest.mark.parametrize("case", CASES, ids=[f"{c[0]}-n{c[1]}p{c[2]}" for c in CASES])
def test_elim_small_parity(case):
    space, n, p = case
    rp, ci, nrows, bnd = _oracle_pattern(space, n, p)
    pat = _pattern_on_device(rp, ci, nrows)
    nnz = pat.nnz
    for ess_name, ess in _ess_sets(nrows, bnd).items():
        for policy in ("one", "keep", "zero"):
            for dtype, batch in ((torch.float64, 1), (torch.float32, 3)):
                _say("case", case, ess_name, policy, dtype, batch)
                v0 = meshgen.cotangent(batch, nnz, seed=len(ess) + 7).to(dtype)
                v0 = v0[0] if batch == 1 else v0
                exp, mk = orc.eliminate_bc(rp, ci, v0, ess, policy)
                vd = v0.to(DEV).contiguous()
                diag = torch.zeros(2, dtype=torch.int32, device=DEV)
                marker = lor.lor_eliminate_bc(pat, vd, torch.from_numpy(ess), policy, diag=diag)
                torch.cuda.synchronize()
                assert torch.equal(vd.cpu(), exp), (ess_name, policy, dtype)
                assert torch.equal(marker.cpu().bool(), mk)
                assert diag.cpu().tolist() == [0, 0]


def test_elim_after_gpu_assembly_matches_oracle():
    """What a caller does: GPU pattern, GPU assembly, GPU elimination of the
    boundary; against the oracle's assembly and elimination of the same mesh."""
    n, p = 3, 3
    m = meshgen.cartesian_mesh(n, p, 0.1)
    kap = meshgen.kappa_field(m["nel"], p, 1.0, seed=2)
    bnd = meshgen.boundary_vertices(n, p)
    rp, ci, v = orc.h1_matrix(m["coords"], m["elem_dofs"], p, kap, 1.0)
    exp, _ = orc.eliminate_bc(rp, ci, v, bnd, "one")
    pat = lor.lor_pattern(lor.LOR_H1, p, torch.from_numpy(m["elem_dofs"]).to(DEV), m["ndofs"])
    vd = lor.lor_assemble_h1(pat, torch.from_numpy(m["elem_dofs"]), torch.from_numpy(m["coords"]), kap, 1.0)
    lor.lor_eliminate_bc(pat, vd, torch.from_numpy(bnd))
    torch.cuda.synchronize()
    got = vd.cpu()
    assert torch.equal(pat.col_idx.cpu().to(torch.int64), ci)
    assert row_rel_err(rp, ci, got, ci, exp) <= 1e-12
    rows = torch.repeat_interleave(torch.arange(m["ndofs"]), rp[1:] - rp[:-1])
    mk = torch.zeros(m["ndofs"], dtype=torch.bool)
    mk[torch.from_numpy(bnd).long()] = True
    hit = mk[rows] | mk[ci]
    assert torch.equal(got[hit], exp[hit])  # eliminated entries: exactly 0 or 1


def test_elim_out_of_range_and_asymmetric_counts():
    rp, ci, nrows, bnd = _oracle_pattern("h1", 2, 1)
    pat = _pattern_on_device(rp, ci, nrows)
    ess = np.array([5, -3, nrows, 7, nrows + 100], dtype=np.int32)
    v0 = meshgen.cotangent(1, pat.nnz, seed=3)[0]
    exp, _ = orc.eliminate_bc(rp, ci, v0, ess[(ess >= 0) & (ess < nrows)], "one")
    vd = v0.to(DEV)
    diag = torch.zeros(2, dtype=torch.int32, device=DEV)
    lor.lor_eliminate_bc(pat, vd, torch.from_numpy(ess), "one", diag=diag)
    torch.cuda.synchronize()
    assert diag.cpu().tolist() == [3, 0]
    assert torch.equal(vd.cpu(), exp)
    # a pattern without the transposed entry (1, 0): counted, the rest done
    rp2 = torch.tensor([0, 2, 3, 4])
    ci2 = torch.tensor([0, 1, 1, 2])
    pat2 = _pattern_on_device(rp2, ci2, 3)
    vd = torch.tensor([4.0, -1.0, 5.0, 6.0], dtype=torch.float64, device=DEV)
    diag.zero_()
    lor.lor_eliminate_bc(pat2, vd, torch.tensor([0], dtype=torch.int32), "one", diag=diag)
    torch.cuda.synchronize()
    assert diag.cpu().tolist() == [0, 1]
    assert vd.cpu().tolist() == [1.0, 0.0, 5.0, 6.0]


def _full_size(space):
    if space == "h1":
        m = meshgen.config_mesh("c3_h1_p6_curved")
        pat = lor.lor_pattern(lor.LOR_H1, 6, torch.from_numpy(m["elem_dofs"]).to(DEV), m["ndofs"])
        v = lor.lor_assemble_h1(pat, torch.from_numpy(m["elem_dofs"]), torch.from_numpy(m["coords"]),
                                m["kappa"], m["beta"])
        return m, pat, v, meshgen.boundary_vertices(m["n"], m["p"])
    m = meshgen.config_mesh("c4_nd_p3_curved")
    pat = lor.lor_pattern(lor.LOR_ND, 3, torch.from_numpy(m["elem_edges"]).to(DEV), m["nedges"])
    v = lor.lor_assemble_nd(pat, torch.from_numpy(m["elem_dofs"]), torch.from_numpy(m["elem_edges"]),
                            torch.from_numpy(m["coords"]), m["kappa"], m["beta"], m["ndofs"])
    return m, pat, v, meshgen.boundary_edges(m["n"], m["p"])


@pytest.mark.parametrize("space", ["h1", "nd"])
def test_elim_full_size(space):
    """Full workloads (H1 p=6 on 32^3, H(curl) p=3 on 24^3), boundary dofs
    eliminated in the launch configuration the benchmark times: every entry
    is checked against the definition (eliminated entries exactly 0 or 1, all
    others bitwise unchanged), and sampled rows against the oracle."""
    m, pat, v, bnd = _full_size(space)
    _say(space, "rows", pat.nrows, "nnz", pat.nnz, "essential", bnd.size)
    before = v.clone()
    diag = torch.zeros(2, dtype=torch.int32, device=DEV)
    marker = lor.lor_eliminate_bc(pat, v, torch.from_numpy(bnd), "one", diag=diag)
    torch.cuda.synchronize()
    assert diag.cpu().tolist() == [0, 0]
    mk = torch.zeros(pat.nrows, dtype=torch.bool, device=DEV)
    mk[torch.from_numpy(bnd).long().to(DEV)] = True
    assert torch.equal(marker.bool(), mk)
    rp = pat.row_ptr.to(torch.int64)
    rows = torch.repeat_interleave(torch.arange(pat.nrows, device=DEV), rp[1:] - rp[:-1])
    ci = pat.col_idx.to(torch.int64)
    hit = mk[rows] | mk[ci]
    on_diag = rows == ci
    assert torch.equal(v[~hit], before[~hit])
    assert bool((v[hit & ~on_diag] == 0).all()) and bool((v[hit & on_diag] == 1).all())
    del rows, ci, hit, on_diag, before
    # sampled rows against the oracle (assembly of those rows + elimination)
    N = m["N"]
    if space == "h1":
        pick = [0, 1, N, N + 1, N * N + N + 1, 2 * N * N + 2 * N + 2, (N // 2) * (1 + N + N * N), N ** 3 - 1]
        rows_s, rps, cis, vs = orc.h1_rows(m["coords"], m["elem_dofs"], 6, m["kappa"], m["beta"], torch.tensor(pick))
    else:
        M = N - 1
        pick = [0, 1, M + 1, M * (N + 1) + 1, M * N * N + N + 1, 2 * M * N * N + N * N + N + 1, M * N * N - 1]
        rows_s, rps, cis, vs = orc.nd_rows(m["coords"], m["elem_dofs"], m["elem_edges"], 3, m["kappa"], m["beta"],
                                           torch.tensor(pick))
    exp, _ = orc.eliminate_bc(rps, cis, vs, bnd, "one", rows=rows_s)
    grp = pat.row_ptr.cpu().to(torch.int64)
    idx = torch.cat([torch.arange(grp[r], grp[r + 1]) for r in rows_s.tolist()])
    got = v.cpu()[idx]
    assert torch.equal(pat.col_idx.cpu().to(torch.int64)[idx], cis)
    assert row_rel_err(rps, cis, got, cis, exp) <= 1e-12
    mkc = torch.zeros(pat.nrows, dtype=torch.bool)
    mkc[torch.from_numpy(bnd).long()] = True
    rr = torch.repeat_interleave(rows_s, rps[1:] - rps[:-1])
    hs = mkc[rr] | mkc[cis]
    assert int(hs.sum()) > 0 and torch.equal(got[hs], exp[hs])
