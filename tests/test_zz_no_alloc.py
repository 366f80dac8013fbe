"""The allocation-free backward entry point (lor_assemble_backward_noalloc,
workspace built into the library) against lor_assemble_backward with a caller
workspace, through the C ABI: two calls in a row on one GPU, the second on a
smaller mesh and batch, so that it runs on what the first left in the shared
workspace.  The kernels are the same, so the results must agree bit for bit."""
import sys

import pytest
import torch

import meshgen
import paper_2210_12253_amd as lor

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda:0")


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _case(n, p, batch, dtype, seed):
    m = meshgen.cartesian_mesh(n, p, 0.12)
    ed = torch.from_numpy(m["elem_dofs"]).to(DEV)
    x = torch.from_numpy(m["coords"]).to(DEV)
    pat = lor.lor_pattern(lor.LOR_H1, p, ed, m["ndofs"])
    kap = meshgen.kappa_field(m["nel"], p, 1.0, seed=seed, batch=batch).to(DEV, dtype)
    cot = meshgen.cotangent(batch, pat.nnz, seed=seed + 1).to(DEV, dtype)
    return pat, ed, x, kap, cot


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_noalloc_backward_matches_the_workspace_call(dtype):
    lib = lor.load_library()
    assert lib.lor_backward_noalloc_max_workspace() == 32 << 20
    # first call: 4^3 elements at p = 4, batch 3; second: 2^3 at p = 3, batch 2
    for n, p, batch, seed in ((4, 4, 3, 11), (2, 3, 2, 21)):
        _say(f"noalloc backward n={n} p={p} batch={batch} dtype={dtype}")
        pat, ed, x, kap, cot = _case(n, p, batch, dtype, seed)
        gk_ref, gx_ref = lor.lor_assemble_backward(pat, ed, x, kap, 0.8, cot, dtype=dtype)
        gk = torch.full_like(kap, float("nan"))
        gx = torch.full((pat.nrows, 3), float("nan"), dtype=torch.float64, device=DEV)
        lor.lor_assemble_backward_noalloc(pat, ed, x, kap, 0.8, cot, dtype=dtype, grad_kappa=gk, grad_coords=gx)
        torch.cuda.synchronize()
        assert torch.equal(gk, gk_ref), "grad kappa differs from the workspace entry point"
        assert torch.equal(gx, gx_ref), "grad coords differ from the workspace entry point"
        assert bool(torch.isfinite(gx).all())


def test_noalloc_backward_rejects_a_mesh_beyond_the_workspace():
    """The host check names the limit; nothing is launched."""
    lib = lor.load_library()
    pat, ed, x, kap, cot = _case(1, 2, 1, torch.float64, 3)
    gk = torch.empty_like(kap)
    gx = torch.empty((pat.nrows, 3), dtype=torch.float64, device=DEV)
    nel_big = (32 << 20) // (24 * 27) + 1
    rc = lib.lor_assemble_backward_noalloc(2, nel_big, pat.nrows, 1, ed.data_ptr(), x.data_ptr(), kap.data_ptr(),
                                           1.0, pat.row_ptr.data_ptr(), lor.lor.ctypes.byref(pat.sched),
                                           cot.data_ptr(), gk.data_ptr(), gx.data_ptr(), lor.LOR_F64, None)
    assert rc == lor.lor.LOR_EUNSUPPORTED
    assert b"built-in workspace" in lib.lor_last_error()
