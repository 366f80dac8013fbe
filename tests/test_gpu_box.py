"""Box-lattice H1 meshes (elements tiling a box, lexicographic vertex ids,
elements in any order): the pattern, colours and rank tables then come from
closed forms instead of searches.  Checked here on boxes that are not cubes
-- one element thick along some axes, a single element, odd and even counts
-- against the CPU oracle: the pattern bit for bit, both value kernels to the
usual bounds, the colour count (two colours per axis with more than one
element) and that a mesh which is not a box lattice (two vertex ids swapped)
takes the general path and still matches the oracle."""
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

BOXES = [
    (1, 1, 1, 3, None),
    (3, 2, 1, 2, None),
    (1, 3, 2, 2, "permute"),
    (4, 1, 2, 1, None),
    (2, 3, 4, 2, "permute"),
    (5, 2, 3, 3, None),
    (1, 1, 4, 4, "permute"),
]


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _mesh(nx, ny, nz, p, pert, seed=0):
    m = meshgen.box_mesh(nx, ny, nz, p, 0.12)
    kap = meshgen.kappa_field(m["nel"], p, 1.5, seed=seed)
    if pert == "permute":
        m, order = meshgen.permute_elements(m, seed=seed + 7)
        kap = kap[torch.from_numpy(order)]
    return m, kap


def _values(pat, m, kap, beta, dtype=torch.float64, **kw):
    v = lor.lor_assemble_h1(pat, torch.from_numpy(m["elem_dofs"]), torch.from_numpy(m["coords"]), kap, beta,
                            dtype=dtype, **kw)
    torch.cuda.synchronize()
    return v.cpu()


@pytest.mark.parametrize("case", BOXES, ids=[f"{c[0]}x{c[1]}x{c[2]}p{c[3]}-{c[4]}" for c in BOXES])
def test_box_lattice_parity(case):
    nx, ny, nz, p, pert = case
    _say("box", case)
    m, kap = _mesh(nx, ny, nz, p, pert)
    rp, ci, v = orc.h1_matrix(m["coords"], m["elem_dofs"], p, kap, 0.8)
    pat = lor.lor_pattern(lor.LOR_H1, p, torch.from_numpy(m["elem_dofs"]).to(DEV), m["ndofs"])
    assert pat.owner
    assert tuple(pat.sched.box) == (nx, ny, nz)
    assert pat.ncolors == 2 ** sum(n > 1 for n in (nx, ny, nz))
    assert pat.sched.nclass <= 64
    assert torch.equal(pat.row_ptr.cpu().to(torch.int64), rp)
    assert torch.equal(pat.col_idx.cpu().to(torch.int64), ci)
    t = torch.from_numpy(transpose_perm(rp, ci))
    for kern in ("owner", "colored"):
        v64 = _values(pat, m, kap, 0.8, kernel=kern)
        assert row_rel_err(rp, ci, v64, ci, v) <= 1e-12, kern
        assert torch.equal(v64, v64[t]), kern
        v32 = _values(pat, m, kap.float(), 0.8, dtype=torch.float32, kernel=kern)
        assert row_rel_err(rp, ci, v32, ci, v) <= 1e-6, kern


def test_box_colours_are_proper_and_ordered():
    """Elements of one colour share no vertex, and the colour order lists each
    colour's elements in increasing element index."""
    m, _ = _mesh(3, 2, 4, 2, "permute")
    pat = lor.lor_pattern(lor.LOR_H1, 2, torch.from_numpy(m["elem_dofs"]).to(DEV), m["ndofs"])
    s = pat.sched
    raw = pat.sched_dev.cpu().numpy()
    order = np.frombuffer(raw[s.off_order:s.off_order + 4 * m["nel"]].tobytes(), dtype=np.int32)
    color = np.frombuffer(raw[s.off_color:s.off_color + 4 * m["nel"]].tobytes(), dtype=np.int32)
    assert sorted(order.tolist()) == list(range(m["nel"]))
    for c in range(s.ncolors):
        els = order[s.color_ptr[c]:s.color_ptr[c + 1]]
        assert np.all(np.diff(els) > 0) and np.all(color[els] == c)
        verts = m["elem_dofs"][els].reshape(-1)
        assert len(np.unique(verts)) == verts.size, c


def test_not_a_box_lattice_takes_the_general_path():
    m, kap = _mesh(3, 2, 2, 2, None)
    ed = m["elem_dofs"].copy()
    a, b = 5, 17                    # swap two vertex ids (and their coordinates)
    ed = np.where(ed == a, -1, ed)
    ed = np.where(ed == b, a, ed)
    ed = np.where(ed == -1, b, ed).astype(np.int32)
    X = m["coords"].copy()
    X[[a, b]] = X[[b, a]]
    m = dict(m, elem_dofs=ed, coords=X)
    rp, ci, v = orc.h1_matrix(X, ed, 2, kap, 1.0)
    pat = lor.lor_pattern(lor.LOR_H1, 2, torch.from_numpy(ed).to(DEV), m["ndofs"])
    assert not pat.owner
    assert torch.equal(pat.row_ptr.cpu().to(torch.int64), rp)
    assert torch.equal(pat.col_idx.cpu().to(torch.int64), ci)
    assert row_rel_err(rp, ci, _values(pat, m, kap, 1.0), ci, v) <= 1e-12
