"""GPU parity of the LOR H(div) (lowest-order Raviart-Thomas) path against the
CPU oracle, through the C ABI (Python binding)."""
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


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _setup(n, p, amp, sigma, seed, flip=False, renumber=False):
    m = meshgen.cartesian_mesh(n, p, amp)
    fm, nf = meshgen.face_map(n, p)
    kap = meshgen.kappa_field(m["nel"], p, sigma, seed=seed)
    if flip:
        fm, _ = meshgen.flip_edge_signs(fm, nf, seed=seed + 2)
    if renumber:
        m, _ = meshgen.renumber_vertices(m, seed=seed + 3)
    return m, fm, nf, kap


def _assemble(pat, m, fm, kap, beta, dtype=torch.float64, **kw):
    v = lor.lor_assemble_rt(pat, torch.from_numpy(m["elem_dofs"]), torch.from_numpy(fm),
                            torch.from_numpy(m["coords"]), kap, beta, m["ndofs"], dtype=dtype, **kw)
    torch.cuda.synchronize()
    return v.cpu()


CASES = [
    # (n, p, amp, sigma, beta, flip, renumber)
    (2, 1, 0.1, 1.0, 1.0, False, False),
    (2, 2, 0.12, 1.0, 0.5, True, True),
    (3, 3, 0.1, 1.0, 1.0, False, False),
    (2, 3, 0.12, 2.0, 1.0, True, False),
    (1, 4, 0.1, 1.0, 1.0, True, True),
    (1, 5, 0.1, 1.0, 2.0, False, True),
    (1, 6, 0.1, 1.0, 1.0, True, False),
]


@pytest.mark.parametrize("case", CASES, ids=[f"n{c[0]}p{c[1]}-f{int(c[5])}r{int(c[6])}" for c in CASES])
def test_rt_small_parity(case):
    n, p, amp, sigma, beta, fl, rn = case
    _say("case", case)
    m, fm, nf, kap = _setup(n, p, amp, sigma, seed=n + 10 * p, flip=fl, renumber=rn)
    rp, ci, v = orc.rt_matrix(m["coords"], m["elem_dofs"], fm, p, kap, beta, nf)
    pat = lor.lor_pattern(lor.LOR_RT, p, torch.from_numpy(fm).to(DEV), nf)
    assert pat.nnz == rp[-1].item() == nf + 30 * (n * p) ** 3
    assert torch.equal(pat.row_ptr.cpu().to(torch.int64), rp)
    assert torch.equal(pat.col_idx.cpu().to(torch.int64), ci)
    v64 = _assemble(pat, m, fm, kap, beta)
    e64 = row_rel_err(rp, ci, v64, ci, v)
    v32 = _assemble(pat, m, fm, kap.float(), beta, dtype=torch.float32, fp64_fallback=True)
    e32 = row_rel_err(rp, ci, v32, ci, v)
    _say(f"  fp64 {e64:.2e} fp32 {e32:.2e}")
    assert e64 <= 1e-12 and e32 <= 1e-6
    t = transpose_perm(rp, ci)
    assert torch.equal(v64, v64[t])  # bitwise symmetric


BOXRT = [(3, 3, 3, 1, 0.1, True, False, False), (2, 3, 1, 3, 0.12, False, True, True),
         (5, 1, 2, 3, 0.1, True, True, False), (1, 1, 1, 6, 0.1, False, False, True),
         (2, 2, 2, 4, 0.1, True, False, True)]


@pytest.mark.parametrize("case", BOXRT, ids=[f"{c[0]}x{c[1]}x{c[2]}p{c[3]}-f{int(c[5])}r{int(c[6])}e{int(c[7])}"
                                             for c in BOXRT])
def test_rt_owner_parity(case):
    """Face lattices (also rectangular boxes, flipped face orientations,
    renumbered vertices, elements in any order) get the owner-computes
    schedule; both kernels in both forms against the oracle, every row, the
    owner kernel bitwise symmetric and deterministic.  5 x 1 x 2 at p = 3
    spans three tiles of 8 cells along x (15 cells), 2 x 2 x 2 at p = 4 two
    along each of x and y."""
    nx, ny, nz, p, amp, flip, renumber, perm = case
    _say("case", case)
    m = meshgen.box_mesh(nx, ny, nz, p, amp)
    fm, nf = meshgen.face_map_box(nx, ny, nz, p)
    kap = meshgen.kappa_field(m["nel"], p, 1.0, seed=nx + ny + nz + p)
    if flip:
        fm, _ = meshgen.flip_edge_signs(fm, nf, seed=p)
    if renumber:
        m, _ = meshgen.renumber_vertices(m, seed=p + 1)
    if perm:
        m, order = meshgen.permute_elements(m, seed=nx * ny * nz)
        fm = np.ascontiguousarray(fm[order])
        kap = kap[torch.from_numpy(order)]
    rp, ci, v = orc.rt_matrix(m["coords"], m["elem_dofs"], fm, p, kap, 0.8, nf)
    pat = lor.lor_pattern(lor.LOR_RT, p, torch.from_numpy(fm).to(DEV), nf)
    assert pat.owner
    assert torch.equal(pat.row_ptr.cpu().to(torch.int64), rp)
    assert torch.equal(pat.col_idx.cpu().to(torch.int64), ci)
    tp = transpose_perm(rp, ci)
    for kern in ("owner", "colored"):
        diag = torch.zeros(2, dtype=torch.int32, device=DEV)
        v64 = _assemble(pat, m, fm, kap, 0.8, kernel=kern, diag=diag)
        v32 = _assemble(pat, m, fm, kap.float(), 0.8, dtype=torch.float32, fp64_fallback=True, kernel=kern)
        e64 = row_rel_err(rp, ci, v64, ci, v)
        e32 = row_rel_err(rp, ci, v32, ci, v)
        _say(f"  {kern}: fp64 {e64:.2e} fp32 {e32:.2e} diag {diag.cpu().tolist()}")
        assert e64 <= 1e-12 and e32 <= 1e-6
        assert diag.cpu().tolist() == [0, 0]
        assert torch.equal(v64, v64[tp]) and torch.equal(v32, v32[tp])
        if kern == "owner":
            assert torch.equal(v64, _assemble(pat, m, fm, kap, 0.8, kernel=kern))


def test_rt_owner_not_a_face_lattice():
    """Reoriented elements: no face lattice, LOR_OWNER fails with
    LOR_EUNSUPPORTED, the default takes the coloured kernel."""
    m = meshgen.cartesian_mesh(2, 2, 0.1)
    fm, nf = meshgen.face_map(2, 2)
    kap = meshgen.kappa_field(m["nel"], 2, 1.0, seed=3)
    m2, kap2, _ = meshgen.reorient_elements(m, seed=5, kappa=kap)
    fm2, nf2 = meshgen.face_map_from_vertices(m2["elem_dofs"], 2)
    assert nf2 == nf
    pat = lor.lor_pattern(lor.LOR_RT, 2, torch.from_numpy(fm2).to(DEV), nf)
    assert not pat.owner
    with pytest.raises(lor.LorError):
        _assemble(pat, m2, fm2, kap2, 0.5, kernel="owner")
    rp, ci, v = orc.rt_matrix(m2["coords"], m2["elem_dofs"], fm2, 2, kap2, 0.5, nf)
    assert row_rel_err(rp, ci, _assemble(pat, m2, fm2, kap2, 0.5), ci, v) <= 1e-12


def test_rt_batch_matches_single_and_is_deterministic():
    m, fm, nf, _ = _setup(2, 3, 0.1, 1.0, seed=1)
    kb = meshgen.kappa_field(m["nel"], 3, 1.0, seed=4, batch=3)
    pat = lor.lor_pattern(lor.LOR_RT, 3, torch.from_numpy(fm).to(DEV), nf)
    vb = _assemble(pat, m, fm, kb, 0.7)
    for b in range(3):
        assert torch.equal(vb[b], _assemble(pat, m, fm, kb[b], 0.7))
    assert torch.equal(vb, _assemble(pat, m, fm, kb, 0.7))


def test_rt_full_size_sampled_rows_and_exact_sequence():
    """p=3 on 24^3 curved hexes (1,135,296 faces): the pattern count, sampled
    rows (boundary and interior faces of every orientation) against the
    oracle in FP64 and FP32, and K_div C = 0 with the GPU's own discrete curl
    (kappa-only matrix)."""
    m = meshgen.config_mesh("c6_rt_p3_curved")
    fm, nf = m["elem_faces"], m["nfaces"]
    pat = lor.lor_pattern(lor.LOR_RT, 3, torch.from_numpy(fm).to(DEV), nf)
    M = 72
    assert nf == 1135296 and pat.nnz == nf + 30 * M ** 3
    v64 = _assemble(pat, m, fm, m["kappa"], m["beta"])
    v32 = _assemble(pat, m, fm, m["kappa"].float(), m["beta"], dtype=torch.float32, fp64_fallback=True)
    N = M + 1
    rng = np.random.default_rng(0)
    pick = [0, 1, N, N * M - 1, N * M * M + 5, 2 * N * M * M + M * M + 7, nf - 1]
    pick += list(rng.integers(0, nf, size=300))
    rows, rp, ci, v = orc.rt_rows(m["coords"], m["elem_dofs"], fm, 3, m["kappa"], m["beta"], torch.tensor(pick))
    grp = pat.row_ptr.cpu().to(torch.int64)
    idx = torch.cat([torch.arange(grp[r], grp[r + 1]) for r in rows.tolist()])
    assert torch.equal(pat.col_idx.cpu().to(torch.int64)[idx], ci)
    e64 = row_rel_err(rp, ci, v64[idx], ci, v)
    e32 = row_rel_err(rp, ci, v32[idx], ci, v)
    _say(f"sampled rows: fp64 {e64:.2e} fp32 {e32:.2e}")
    assert e64 <= 1e-12 and e32 <= 1e-6
    check_whole_matrix(pat, v64.to(DEV), v32.to(DEV))
    ee, ned = meshgen.nd_edge_map(24, 3)
    crp, cci, cv = lor.lor_discrete_curl(3, ee, fm, ned, nf, device=DEV)
    kd = _assemble(pat, m, fm, m["kappa"], 0.0)
    K = orc.csr_to_scipy(pat.row_ptr.cpu().long(), pat.col_idx.cpu().long(), kd, nf)
    C = orc.csr_to_scipy(crp.cpu().long(), cci.cpu().long(), cv.cpu(), ned)
    x = rng.standard_normal(ned)
    y = K @ (C @ x)
    assert np.abs(y).max() <= 1e-11 * np.abs(K.data).max() * np.abs(x).max()


def test_rt_fp32_fallback_and_empty():
    """A pinched vertex (corner-Jacobian ratio above 10) sends its subelements
    through the FP64 path of the FP32 form (counted in diag[0]); an empty mesh
    launches nothing."""
    m, fm, nf, _ = _setup(1, 2, 0.0, 1.0, seed=3)
    X = m["coords"].copy()
    X[13] = [0.96, 0.5, 0.5]
    m["coords"] = X
    kap = torch.ones(1, 8, dtype=torch.float64)
    rp, ci, v = orc.rt_matrix(X, m["elem_dofs"], fm, 2, kap, 1.0, nf)
    pat = lor.lor_pattern(lor.LOR_RT, 2, torch.from_numpy(fm).to(DEV), nf)
    diag = torch.zeros(2, dtype=torch.int32, device=DEV)
    v32 = _assemble(pat, m, fm, kap.float(), 1.0, dtype=torch.float32, fp64_fallback=True, det_ratio_thresh=10.0,
                    diag=diag)
    d = diag.cpu().tolist()
    assert d[0] > 0 and d[1] == 0
    assert row_rel_err(rp, ci, v32, ci, v) <= 1e-6
    pat0 = lor.lor_pattern(lor.LOR_RT, 2, torch.zeros((0, 36), dtype=torch.int32, device=DEV), 5)
    out = lor.lor_assemble_rt(pat0, torch.zeros((0, 27), dtype=torch.int32), torch.zeros((0, 36), dtype=torch.int32),
                              torch.zeros((5, 3), dtype=torch.float64), torch.zeros((0, 8), dtype=torch.float64), 1.0, 5)
    torch.cuda.synchronize()
    assert pat0.nnz == 0 and out.numel() == 0
