"""FP32 form, quality report: extreme eigenvalues of the FP64 LOR matrix
preconditioned by its FP32 form (the pencil A64 x = lambda A32 x on the same
pattern).  Nothing in the paper fixes these values (parity unpinned); the
test checks that both ends stay within a loose bound of 1 and prints them."""
import sys

import pytest
import torch

import bench
import meshgen
import paper_2210_12253_amd as lor

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda:0")


def test_fp32_pencil_extreme_eigenvalues():
    m = meshgen.cartesian_mesh(6, 4, 0.1 / 6)
    kap = meshgen.kappa_field(m["nel"], 4, 2.0, seed=0)
    ed = torch.from_numpy(m["elem_dofs"]).to(DEV)
    x = torch.from_numpy(m["coords"]).to(DEV)
    pat = lor.lor_pattern(lor.LOR_H1, 4, ed, m["ndofs"])
    v64 = lor.lor_assemble_h1(pat, ed, x, kap.to(DEV), 1.0)
    v32 = lor.lor_assemble_h1(pat, ed, x, kap.to(DEV).float(), 1.0, dtype=torch.float32, fp64_fallback=True)
    torch.cuda.synchronize()
    r = bench.pencil_extreme_eigs(pat.row_ptr, pat.col_idx, v64, v32, m["ndofs"], niter=300)
    print(f"n6 p4 ({m['ndofs']} rows): lambda_max - 1 = {r['lambda_max_minus_1']:.3e}, "
          f"1 - lambda_min = {r['one_minus_lambda_min']:.3e}", flush=True)
    sys.stdout.flush()
    assert abs(r["lambda_max_minus_1"]) <= 1e-4
    assert abs(r["one_minus_lambda_min"]) <= 1e-4
