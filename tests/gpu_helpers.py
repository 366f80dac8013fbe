"""Helpers shared by the GPU parity tests (comparison metrics only)."""
import numpy as np
import torch


def row_rel_err(rp, ci_a, va, ci_b, vb):
    """max over rows of max_j |A_ij - B_ij| / max_j |B_ij| on identical patterns."""
    rp = torch.as_tensor(rp).to(torch.int64).cpu()
    assert torch.equal(torch.as_tensor(ci_a).cpu().to(torch.int64), torch.as_tensor(ci_b).cpu().to(torch.int64))
    va = torch.as_tensor(va).cpu().to(torch.float64)
    vb = torch.as_tensor(vb).cpu().to(torch.float64)
    n = rp.numel() - 1
    rows = torch.repeat_interleave(torch.arange(n), rp[1:] - rp[:-1])
    d = (va - vb).abs()
    num = torch.zeros(n, dtype=torch.float64).scatter_reduce(0, rows, d, reduce="amax", include_self=True)
    den = torch.zeros(n, dtype=torch.float64).scatter_reduce(0, rows, vb.abs(), reduce="amax", include_self=True)
    ok = den > 0
    if not bool(ok.any()):
        return float(num.max()) if num.numel() else 0.0
    return float((num[ok] / den[ok]).max())


def transpose_perm(rp, ci):
    """Index t with values[t[k]] = the entry (j, i) of entry k = (i, j)."""
    rp = np.asarray(torch.as_tensor(rp).cpu(), dtype=np.int64)
    ci = np.asarray(torch.as_tensor(ci).cpu(), dtype=np.int64)
    n = rp.size - 1
    rows = np.repeat(np.arange(n), np.diff(rp))
    key = rows * n + ci
    tkey = ci * n + rows
    order = np.argsort(key)
    pos = np.searchsorted(key[order], tkey)
    return order[pos]


def check_whole_matrix(pat, *values):
    """Properties of a complete assembled matrix that hold at any size, checked
    on the device: columns strictly increasing in every row, a symmetric
    pattern (the transpose of every entry present exactly once) and bitwise
    symmetric values for every given value array (same pattern)."""
    dev = pat.row_ptr.device
    rp = pat.row_ptr.to(torch.int64)
    ci = pat.col_idx.to(torch.int64)
    n = pat.nrows
    rows = torch.repeat_interleave(torch.arange(n, device=dev), rp[1:] - rp[:-1])
    same_row = rows[1:] == rows[:-1]
    assert bool((ci[1:][same_row] > ci[:-1][same_row]).all()), "columns not strictly increasing"
    del same_row
    key = rows * n + ci
    tkey = ci * n + rows
    del rows
    order = torch.argsort(tkey)
    assert torch.equal(tkey[order], key), "pattern not symmetric"
    del tkey, key
    for v in values:
        v = v.reshape(-1, pat.nnz)
        assert torch.equal(v[:, order], v), "values not bitwise symmetric"
