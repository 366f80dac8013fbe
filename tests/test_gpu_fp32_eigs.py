"""FP32 form, quality report: extreme eigenvalues of the FP64 LOR matrix
preconditioned by its FP32 form (the pencil A64 x = lambda A32 x on the same
pattern), by the Lanczos routine the benchmark reports.  Nothing in the paper
fixes these values (parity unpinned); the test checks the Lanczos extremes
against a dense generalized eigensolve of the same two matrices, that the
reported pairs have converged, and that both ends stay within a loose bound
of 1."""
import sys

import numpy as np
import pytest
import scipy.linalg as sl
import torch

import bench
import meshgen
import paper_2210_12253_amd as lor
from oracle import lor_oracle as orc

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda:0")


def test_fp32_pencil_extreme_eigenvalues():
    m = meshgen.cartesian_mesh(4, 4, 0.1 / 4)
    kap = meshgen.kappa_field(m["nel"], 4, 2.0, seed=0)
    ed = torch.from_numpy(m["elem_dofs"]).to(DEV)
    x = torch.from_numpy(m["coords"]).to(DEV)
    pat = lor.lor_pattern(lor.LOR_H1, 4, ed, m["ndofs"])
    v64 = lor.lor_assemble_h1(pat, ed, x, kap.to(DEV), 1.0)
    v32 = lor.lor_assemble_h1(pat, ed, x, kap.to(DEV).float(), 1.0, dtype=torch.float32, fp64_fallback=True)
    torch.cuda.synchronize()
    r = bench.pencil_extreme_eigs(pat.row_ptr, pat.col_idx, v64, v32, m["ndofs"])
    print(f"n4 p4 ({m['ndofs']} rows): lambda_max - 1 = {r['lambda_max_minus_1']:.6e}, "
          f"1 - lambda_min = {r['one_minus_lambda_min']:.6e}, residuals {r['relative_residual']}", flush=True)
    sys.stdout.flush()
    assert r["converged"]
    # dense generalized eigenvalues of (A64 - A32, A32)
    a32 = v32.double().cpu()
    d = (v64.cpu() - a32)
    B = orc.csr_to_dense(pat.row_ptr.cpu().long(), pat.col_idx.cpu().long(), a32).numpy()
    E = orc.csr_to_dense(pat.row_ptr.cpu().long(), pat.col_idx.cpu().long(), d).numpy()
    w = sl.eigh(E, B, eigvals_only=True)
    print(f"dense: max {w[-1]:.6e}, min {w[0]:.6e}", flush=True)
    assert abs(r["lambda_max_minus_1"] - w[-1]) <= 1e-6 * abs(w[-1])
    assert abs(r["one_minus_lambda_min"] + w[0]) <= 1e-6 * abs(w[0])
    assert np.abs(w).max() <= 1e-4
