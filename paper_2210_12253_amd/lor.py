"""Python binding of the LOR assembly C ABI (include/lor.h).

Argument marshalling only: every step of the assembly runs in the HIP kernels
of liblor.so.  PyTorch provides device memory and the current stream.  If the
library has not been built the import fails loudly -- there is no fallback.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liblor.so")

LOR_OK, LOR_EINVAL, LOR_EOVERFLOW, LOR_EDEVICE, LOR_EUNSUPPORTED = 0, -1, -2, -3, -4
LOR_H1, LOR_ND, LOR_RT, LOR_H1_2D = 0, 1, 2, 3
LOR_F64, LOR_F32 = 0, 1
LOR_MAX_P = 6
LOR_MAX_COLORS = 64
LOR_FP64_FALLBACK = 0x1
LOR_COLORED = 0x2
LOR_OWNER = 0x4
_KERNEL_FLAGS = {"auto": 0, "colored": LOR_COLORED, "owner": LOR_OWNER}
LOR_DIAG_ONE, LOR_DIAG_KEEP, LOR_DIAG_ZERO = 0, 1, 2
_DIAG_POLICY = {"one": LOR_DIAG_ONE, "keep": LOR_DIAG_KEEP, "zero": LOR_DIAG_ZERO}

ABI_SYMBOLS = (
    "lor_pattern",
    "lor_assemble_h1",
    "lor_assemble_nd",
    "lor_assemble_rt",
    "lor_assemble_h1_2d",
    "lor_assemble_backward",
    "lor_refine_map",
    "lor_assemble_h1_unstructured",
    "lor_backward_workspace",
    "lor_pattern_workspace",
    "lor_assemble_backward_noalloc",
    "lor_backward_noalloc_max_workspace",
    "lor_eliminate_bc",
    "lor_discrete_gradient",
    "lor_discrete_curl",
    "lor_interp_nodes",
    "lor_evec_to_tvec",
    "lor_sched_bytes",
    "lor_last_error",
    "lor_abi_version",
)


class LorError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"[{code}] {msg}")
        self.code = code


class LorSched(ctypes.Structure):
    _fields_ = [
        ("space", ctypes.c_int32),
        ("p", ctypes.c_int32),
        ("nel", ctypes.c_int64),
        ("nrows", ctypes.c_int64),
        ("nnz", ctypes.c_int64),
        ("nloc", ctypes.c_int32),
        ("nent", ctypes.c_int32),
        ("ncolors", ctypes.c_int32),
        ("max_row_nnz", ctypes.c_int32),
        ("color_ptr", ctypes.c_int32 * (LOR_MAX_COLORS + 1)),
        ("nclass", ctypes.c_int64),
        ("tab_stride", ctypes.c_int64),
        ("dev_bytes", ctypes.c_size_t),
        ("dev", ctypes.c_void_p),
        ("off_order", ctypes.c_size_t),
        ("off_color", ctypes.c_size_t),
        ("off_class", ctypes.c_size_t),
        ("off_tables", ctypes.c_size_t),
        ("off_inc_ptr", ctypes.c_size_t),
        ("off_inc_list", ctypes.c_size_t),
        ("off_st_ptr", ctypes.c_size_t),
        ("off_st_col", ctypes.c_size_t),
        ("off_ent_row", ctypes.c_size_t),
        ("off_recipe", ctypes.c_size_t),
        ("off_zero", ctypes.c_size_t),
        ("off_order_class", ctypes.c_size_t),
        ("off_elem3d", ctypes.c_size_t),
        ("off_base", ctypes.c_size_t),
        ("owner", ctypes.c_int32),
        ("box", ctypes.c_int32 * 3),
        ("reserved", ctypes.c_size_t * 3),
    ]


_lib = None


def load_library(path: str = LIB_PATH) -> ctypes.CDLL:
    """Load liblor.so (raises if it is missing: build it with __graft_entry__.build())."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"HIP library {path} not built; run `python -c 'import __graft_entry__ as g; g.build()'`")
    lib = ctypes.CDLL(path)
    vp, i32, i64, u32, f64, sz = (ctypes.c_void_p, ctypes.c_int, ctypes.c_int64, ctypes.c_uint, ctypes.c_double,
                                  ctypes.c_size_t)
    lib.lor_pattern.argtypes = [i32, i32, i64, i64, vp, vp, ctypes.POINTER(ctypes.c_int64), vp,
                                ctypes.POINTER(LorSched), vp]
    lib.lor_pattern.restype = i32
    lib.lor_assemble_h1.argtypes = [i32, i64, i64, i32, vp, vp, vp, f64, vp, ctypes.POINTER(LorSched), vp, i32, u32,
                                    f64, vp, vp]
    lib.lor_assemble_h1.restype = i32
    lib.lor_assemble_nd.argtypes = [i32, i64, i64, i64, i32, vp, vp, vp, vp, f64, vp, ctypes.POINTER(LorSched), vp,
                                    i32, u32, f64, vp, vp]
    lib.lor_assemble_nd.restype = i32
    lib.lor_assemble_rt.argtypes = [i32, i64, i64, i64, i32, vp, vp, vp, vp, f64, vp, ctypes.POINTER(LorSched), vp,
                                    i32, u32, f64, vp, vp]
    lib.lor_assemble_rt.restype = i32
    lib.lor_assemble_h1_2d.argtypes = [i32, i64, i64, i32, vp, vp, vp, f64, vp, ctypes.POINTER(LorSched), vp, i32,
                                       u32, f64, vp, vp]
    lib.lor_assemble_h1_2d.restype = i32
    lib.lor_assemble_backward.argtypes = [i32, i64, i64, i32, vp, vp, vp, f64, vp, ctypes.POINTER(LorSched), vp, vp,
                                          vp, vp, i32, vp]
    lib.lor_assemble_backward.restype = i32
    lib.lor_assemble_backward_noalloc.argtypes = [i32, i64, i64, i32, vp, vp, vp, f64, vp,
                                                  ctypes.POINTER(LorSched), vp, vp, vp, i32, vp]
    lib.lor_assemble_backward_noalloc.restype = i32
    lib.lor_backward_noalloc_max_workspace.argtypes = []
    lib.lor_backward_noalloc_max_workspace.restype = sz
    lib.lor_eliminate_bc.argtypes = [i64, i64, i32, vp, vp, vp, i32, i64, vp, vp, i32, vp, vp]
    lib.lor_eliminate_bc.restype = i32
    lib.lor_discrete_gradient.argtypes = [i32, i64, i64, i64, vp, vp, ctypes.POINTER(LorSched), vp, vp, vp, i32,
                                          vp, vp]
    lib.lor_discrete_gradient.restype = i32
    lib.lor_discrete_curl.argtypes = [i32, i64, i64, i64, vp, vp, vp, vp, vp, vp, i32, vp, vp]
    lib.lor_discrete_curl.restype = i32
    lib.lor_interp_nodes.argtypes = [i32, i32, i64, i32, vp, vp, vp]
    lib.lor_interp_nodes.restype = i32
    lib.lor_evec_to_tvec.argtypes = [i32, i64, i64, ctypes.POINTER(LorSched), i32, vp, vp, vp, vp]
    lib.lor_evec_to_tvec.restype = i32
    lib.lor_refine_map.argtypes = [i32, i64, vp, vp, vp]
    lib.lor_refine_map.restype = i32
    lib.lor_assemble_h1_unstructured.argtypes = [i64, i64, i64, vp, vp, vp, f64, vp, vp, vp, vp, vp]
    lib.lor_assemble_h1_unstructured.restype = i32
    lib.lor_backward_workspace.argtypes = [i32, i64, i32, i32]
    lib.lor_backward_workspace.restype = sz
    lib.lor_pattern_workspace.argtypes = [i32, i32, i64, i64]
    lib.lor_pattern_workspace.restype = sz
    lib.lor_sched_bytes.argtypes = []
    lib.lor_sched_bytes.restype = sz
    lib.lor_last_error.argtypes = []
    lib.lor_last_error.restype = ctypes.c_char_p
    lib.lor_abi_version.argtypes = []
    lib.lor_abi_version.restype = i32
    if lib.lor_sched_bytes() != ctypes.sizeof(LorSched):
        raise ImportError("lor_sched layout mismatch between liblor.so and the binding")
    _lib = lib
    return lib


def _check(rc: int) -> None:
    if rc != LOR_OK:
        msg = _lib.lor_last_error().decode() if _lib is not None else ""
        raise LorError(rc, msg)


def _ptr(t: torch.Tensor | None) -> int | None:
    return None if t is None else t.data_ptr()


def _stream() -> int:
    return torch.cuda.current_stream().cuda_stream


def _dev_tensor(t, dtype, name, device) -> torch.Tensor:
    t = torch.as_tensor(t)
    if t.dtype != dtype:
        t = t.to(dtype)
    if t.device != device:
        t = t.to(device)
    if not t.is_contiguous():
        t = t.contiguous()
    return t


def _out(out, shape, dtype, device, name="out") -> torch.Tensor:
    """A caller-supplied output (or workspace) buffer must match exactly: the
    kernels write every element of it and nothing beyond."""
    shape = tuple(int(x) for x in shape)
    if out is None:
        return torch.empty(shape, dtype=dtype, device=device)
    if tuple(out.shape) != shape or out.dtype != dtype or out.device != device or not out.is_contiguous():
        raise ValueError(f"{name} must be a contiguous {dtype} tensor of shape {shape} on {device}")
    return out


def _need(t: torch.Tensor, numel: int, name: str) -> None:
    """The kernels index every array by the pattern's sizes: a wrong size would
    make them read or write outside it, so it is rejected here."""
    if t.numel() != int(numel):
        raise ValueError(f"{name} has {t.numel()} elements, expected {int(numel)}")


def _diag(diag, n: int, device):
    if diag is None:
        return None
    if diag.dtype != torch.int32 or diag.device != device or diag.numel() < n or not diag.is_contiguous():
        raise ValueError(f"diag must be a contiguous int32 tensor of at least {n} elements on {device}")
    return diag


def _dtype_code(dtype) -> int:
    if dtype == torch.float64:
        return LOR_F64
    if dtype == torch.float32:
        return LOR_F32
    raise ValueError("dtype must be torch.float64 or torch.float32")


@dataclass
class Pattern:
    """CSR pattern + assembly schedule of one mesh (built once, reused)."""
    space: int
    p: int
    nel: int
    nrows: int
    nnz: int
    row_ptr: torch.Tensor
    col_idx: torch.Tensor
    sched: LorSched
    sched_dev: torch.Tensor

    @property
    def ncolors(self) -> int:
        return int(self.sched.ncolors)

    @property
    def owner(self) -> bool:
        """True if the mesh has the owner-computes schedule (an H1 box lattice,
        3D or 2D, an H(curl) edge lattice or an H(div) face lattice)."""
        return bool(self.sched.owner)


def lor_pattern(space: int, p: int, elem_map: torch.Tensor, nrows: int, device=None) -> Pattern:
    """Pattern and schedule (lor_pattern phases 1 and 2) on the current CUDA device."""
    lib = load_library()
    device = torch.device("cuda") if device is None else torch.device(device)
    em = _dev_tensor(elem_map, torch.int32, "elem_map", device)
    nloc = {LOR_H1: (p + 1) ** 3, LOR_ND: 3 * p * (p + 1) ** 2, LOR_RT: 3 * p * p * (p + 1),
            LOR_H1_2D: (p + 1) ** 2}.get(space)
    if nloc is None:
        raise ValueError("space must be LOR_H1, LOR_ND, LOR_RT or LOR_H1_2D")
    if em.dim() != 2 or em.shape[1] != nloc:
        raise ValueError(f"elem_map must have shape [nel, {nloc}] for this space and p")
    nel = em.shape[0]
    row_ptr = torch.empty(nrows + 1, dtype=torch.int32, device=device)
    nnz = ctypes.c_int64(0)
    sched = LorSched()
    st = _stream()
    _check(lib.lor_pattern(space, p, nel, nrows, _ptr(em), _ptr(row_ptr), ctypes.byref(nnz), None,
                           ctypes.byref(sched), st))
    col_idx = torch.empty(max(1, nnz.value), dtype=torch.int32, device=device)[: nnz.value]
    sched_dev = torch.empty(int(sched.dev_bytes), dtype=torch.uint8, device=device)
    sched.dev = sched_dev.data_ptr()
    cptr = col_idx.data_ptr() if nnz.value > 0 else torch.empty(1, dtype=torch.int32, device=device).data_ptr()
    _check(lib.lor_pattern(space, p, nel, nrows, _ptr(em), _ptr(row_ptr), ctypes.byref(nnz), cptr,
                           ctypes.byref(sched), st))
    return Pattern(space, p, nel, nrows, nnz.value, row_ptr, col_idx, sched, sched_dev)


def lor_assemble_h1(pat: Pattern, elem_dofs, coords, kappa, beta: float, dtype=torch.float64,
                    fp64_fallback: bool = False, det_ratio_thresh: float = 10.0,
                    diag: torch.Tensor | None = None, out: torch.Tensor | None = None,
                    kernel: str = "auto") -> torch.Tensor:
    """Values of the H1 LOR matrix, [nnz] (or [batch, nnz] for kappa [batch, nel, p^3]).
    kernel: "auto" (owner-computes where the schedule has it, else coloured),
    "owner" or "colored"."""
    if kernel not in _KERNEL_FLAGS:
        raise ValueError("kernel must be 'auto', 'owner' or 'colored'")
    lib = load_library()
    dev = pat.row_ptr.device
    ed = _dev_tensor(elem_dofs, torch.int32, "elem_dofs", dev)
    x = _dev_tensor(coords, torch.float64, "coords", dev)
    k = _dev_tensor(kappa, dtype, "kappa", dev)
    batched = k.dim() == 3
    batch = k.shape[0] if batched else 1
    p = pat.p
    _need(ed, pat.nel * (p + 1) ** 3, "elem_dofs")
    _need(x, pat.nrows * 3, "coords")
    _need(k, batch * pat.nel * p ** 3, "kappa")
    diag = _diag(diag, 2, dev)
    out = _out(out, (batch, pat.nnz) if batched else (pat.nnz,), dtype, dev)
    flags = (LOR_FP64_FALLBACK if fp64_fallback else 0) | _KERNEL_FLAGS[kernel]
    _check(lib.lor_assemble_h1(pat.p, pat.nel, pat.nrows, batch, _ptr(ed), _ptr(x), _ptr(k), float(beta),
                               _ptr(pat.row_ptr), ctypes.byref(pat.sched), _ptr(out), _dtype_code(dtype), flags,
                               float(det_ratio_thresh), _ptr(diag), _stream()))
    return out


def lor_assemble_nd(pat: Pattern, elem_dofs, elem_edges, coords, kappa, beta: float, ndofs_h1: int,
                    dtype=torch.float64, fp64_fallback: bool = False, det_ratio_thresh: float = 10.0,
                    diag: torch.Tensor | None = None, out: torch.Tensor | None = None,
                    kernel: str = "auto") -> torch.Tensor:
    """Values of the H(curl) LOR matrix, [nnz] (or [batch, nnz]).  kernel:
    "auto" (owner-computes when the edge map is an edge lattice, else
    coloured), "owner" or "colored"."""
    if kernel not in _KERNEL_FLAGS:
        raise ValueError("kernel must be 'auto', 'owner' or 'colored'")
    lib = load_library()
    dev = pat.row_ptr.device
    ed = _dev_tensor(elem_dofs, torch.int32, "elem_dofs", dev)
    ee = _dev_tensor(elem_edges, torch.int32, "elem_edges", dev)
    x = _dev_tensor(coords, torch.float64, "coords", dev)
    k = _dev_tensor(kappa, dtype, "kappa", dev)
    batched = k.dim() == 3
    batch = k.shape[0] if batched else 1
    p = pat.p
    _need(ed, pat.nel * (p + 1) ** 3, "elem_dofs")
    _need(ee, pat.nel * 3 * p * (p + 1) ** 2, "elem_edges")
    _need(x, ndofs_h1 * 3, "coords")
    _need(k, batch * pat.nel * p ** 3, "kappa")
    diag = _diag(diag, 2, dev)
    out = _out(out, (batch, pat.nnz) if batched else (pat.nnz,), dtype, dev)
    flags = (LOR_FP64_FALLBACK if fp64_fallback else 0) | _KERNEL_FLAGS[kernel]
    _check(lib.lor_assemble_nd(pat.p, pat.nel, ndofs_h1, pat.nrows, batch, _ptr(ed), _ptr(ee), _ptr(x), _ptr(k),
                               float(beta), _ptr(pat.row_ptr), ctypes.byref(pat.sched), _ptr(out),
                               _dtype_code(dtype), flags, float(det_ratio_thresh), _ptr(diag), _stream()))
    return out


def lor_assemble_h1_2d(pat: Pattern, elem_dofs, coords, kappa, beta: float, dtype=torch.float64,
                       fp64_fallback: bool = False, det_ratio_thresh: float = 10.0,
                       diag: torch.Tensor | None = None, out: torch.Tensor | None = None,
                       kernel: str = "auto") -> torch.Tensor:
    """Values of the 2D H1 LOR matrix, [nnz] (or [batch, nnz] for kappa [batch, nel, p^2]).
    kernel: "auto" (owner-computes on a 2D box lattice, else coloured),
    "owner" or "colored"."""
    if kernel not in _KERNEL_FLAGS:
        raise ValueError("kernel must be 'auto', 'owner' or 'colored'")
    lib = load_library()
    dev = pat.row_ptr.device
    ed = _dev_tensor(elem_dofs, torch.int32, "elem_dofs", dev)
    x = _dev_tensor(coords, torch.float64, "coords", dev)
    k = _dev_tensor(kappa, dtype, "kappa", dev)
    batched = k.dim() == 3
    batch = k.shape[0] if batched else 1
    p = pat.p
    _need(ed, pat.nel * (p + 1) ** 2, "elem_dofs")
    _need(x, pat.nrows * 2, "coords")
    _need(k, batch * pat.nel * p ** 2, "kappa")
    diag = _diag(diag, 2, dev)
    out = _out(out, (batch, pat.nnz) if batched else (pat.nnz,), dtype, dev)
    flags = (LOR_FP64_FALLBACK if fp64_fallback else 0) | _KERNEL_FLAGS[kernel]
    _check(lib.lor_assemble_h1_2d(pat.p, pat.nel, pat.nrows, batch, _ptr(ed), _ptr(x), _ptr(k), float(beta),
                                  _ptr(pat.row_ptr), ctypes.byref(pat.sched), _ptr(out), _dtype_code(dtype), flags,
                                  float(det_ratio_thresh), _ptr(diag), _stream()))
    return out


def lor_assemble_rt(pat: Pattern, elem_dofs, elem_faces, coords, kappa, beta: float, ndofs_h1: int,
                    dtype=torch.float64, fp64_fallback: bool = False, det_ratio_thresh: float = 10.0,
                    diag: torch.Tensor | None = None, out: torch.Tensor | None = None,
                    kernel: str = "auto") -> torch.Tensor:
    """Values of the H(div) LOR matrix, [nnz] (or [batch, nnz]).  kernel:
    "auto" (owner-computes when the face map is a face lattice, else
    coloured), "owner" or "colored"."""
    if kernel not in _KERNEL_FLAGS:
        raise ValueError("kernel must be 'auto', 'owner' or 'colored'")
    lib = load_library()
    dev = pat.row_ptr.device
    ed = _dev_tensor(elem_dofs, torch.int32, "elem_dofs", dev)
    fm = _dev_tensor(elem_faces, torch.int32, "elem_faces", dev)
    x = _dev_tensor(coords, torch.float64, "coords", dev)
    k = _dev_tensor(kappa, dtype, "kappa", dev)
    batched = k.dim() == 3
    batch = k.shape[0] if batched else 1
    p = pat.p
    _need(ed, pat.nel * (p + 1) ** 3, "elem_dofs")
    _need(fm, pat.nel * 3 * p * p * (p + 1), "elem_faces")
    _need(x, ndofs_h1 * 3, "coords")
    _need(k, batch * pat.nel * p ** 3, "kappa")
    diag = _diag(diag, 2, dev)
    out = _out(out, (batch, pat.nnz) if batched else (pat.nnz,), dtype, dev)
    flags = (LOR_FP64_FALLBACK if fp64_fallback else 0) | _KERNEL_FLAGS[kernel]
    _check(lib.lor_assemble_rt(pat.p, pat.nel, ndofs_h1, pat.nrows, batch, _ptr(ed), _ptr(fm), _ptr(x), _ptr(k),
                               float(beta), _ptr(pat.row_ptr), ctypes.byref(pat.sched), _ptr(out),
                               _dtype_code(dtype), flags, float(det_ratio_thresh), _ptr(diag), _stream()))
    return out


def lor_assemble_backward(pat: Pattern, elem_dofs, coords, kappa, beta: float, grad_values,
                          dtype=torch.float64, workspace: torch.Tensor | None = None):
    """Adjoint of lor_assemble_h1: returns (grad_kappa like kappa, grad_coords [ndofs, 3] FP64)."""
    lib = load_library()
    dev = pat.row_ptr.device
    ed = _dev_tensor(elem_dofs, torch.int32, "elem_dofs", dev)
    x = _dev_tensor(coords, torch.float64, "coords", dev)
    k = _dev_tensor(kappa, dtype, "kappa", dev)
    gv = _dev_tensor(grad_values, dtype, "grad_values", dev)
    batched = k.dim() == 3
    batch = k.shape[0] if batched else 1
    p = pat.p
    _need(ed, pat.nel * (p + 1) ** 3, "elem_dofs")
    _need(x, pat.nrows * 3, "coords")
    _need(k, batch * pat.nel * p ** 3, "kappa")
    _need(gv, batch * pat.nnz, "grad_values")
    gk = torch.empty_like(k)
    gx = torch.empty((pat.nrows, 3), dtype=torch.float64, device=dev)
    wbytes = max(1, int(lib.lor_backward_workspace(pat.p, pat.nel, batch, _dtype_code(dtype))))
    if workspace is None:
        workspace = torch.empty(wbytes, dtype=torch.uint8, device=dev)
    elif workspace.device != dev or not workspace.is_contiguous() or \
            workspace.numel() * workspace.element_size() < wbytes:
        raise ValueError(f"workspace must be a contiguous device buffer of at least {wbytes} bytes")
    _check(lib.lor_assemble_backward(pat.p, pat.nel, pat.nrows, batch, _ptr(ed), _ptr(x), _ptr(k), float(beta),
                                     _ptr(pat.row_ptr), ctypes.byref(pat.sched), _ptr(gv), _ptr(gk), _ptr(gx),
                                     _ptr(workspace), _dtype_code(dtype), _stream()))
    return gk, gx


def lor_assemble_backward_noalloc(pat: Pattern, elem_dofs, coords, kappa, beta: float, grad_values,
                                  dtype=torch.float64, grad_kappa: torch.Tensor | None = None,
                                  grad_coords: torch.Tensor | None = None):
    """lor_assemble_backward through the entry point that allocates nothing on
    the device (its workspace is built into the library, one per GPU; calls
    that overlap on one GPU race).  Inputs must already be device tensors of
    the right dtype and outputs may be passed in, so that a captured call
    allocates nothing either.  Returns (grad_kappa, grad_coords)."""
    lib = load_library()
    dev = pat.row_ptr.device
    ed = _dev_tensor(elem_dofs, torch.int32, "elem_dofs", dev)
    x = _dev_tensor(coords, torch.float64, "coords", dev)
    k = _dev_tensor(kappa, dtype, "kappa", dev)
    gv = _dev_tensor(grad_values, dtype, "grad_values", dev)
    batch = k.shape[0] if k.dim() == 3 else 1
    p = pat.p
    _need(ed, pat.nel * (p + 1) ** 3, "elem_dofs")
    _need(x, pat.nrows * 3, "coords")
    _need(k, batch * pat.nel * p ** 3, "kappa")
    _need(gv, batch * pat.nnz, "grad_values")
    gk = _out(grad_kappa, tuple(k.shape), dtype, dev, "grad_kappa")
    gx = _out(grad_coords, (pat.nrows, 3), torch.float64, dev, "grad_coords")
    _check(lib.lor_assemble_backward_noalloc(pat.p, pat.nel, pat.nrows, batch, _ptr(ed), _ptr(x), _ptr(k),
                                             float(beta), _ptr(pat.row_ptr), ctypes.byref(pat.sched), _ptr(gv),
                                             _ptr(gk), _ptr(gx), _dtype_code(dtype), _stream()))
    return gk, gx


def lor_eliminate_bc(pat: Pattern, values: torch.Tensor, ess_dofs, diag_policy: str = "one",
                     marker: torch.Tensor | None = None, diag: torch.Tensor | None = None) -> torch.Tensor:
    """Eliminate the rows and columns of the essential dofs from `values`
    ([nnz] or [batch, nnz], FP64 or FP32, on the pattern's device) in place;
    returns the uint8 marker [nrows]."""
    lib = load_library()
    dev = pat.row_ptr.device
    if values.device != dev or not values.is_contiguous():
        raise ValueError("values must be a contiguous tensor on the pattern's device (modified in place)")
    if values.shape[-1] != pat.nnz or values.dim() not in (1, 2):
        raise ValueError("values must have shape [nnz] or [batch, nnz]")
    if diag_policy not in _DIAG_POLICY:
        raise ValueError(f"diag_policy must be one of {tuple(_DIAG_POLICY)}")
    ess = _dev_tensor(ess_dofs, torch.int32, "ess_dofs", dev).reshape(-1)
    batch = values.shape[0] if values.dim() == 2 else 1
    marker = _out(marker, (pat.nrows,), torch.uint8, dev, "marker")
    diag = _diag(diag, 2, dev)
    _check(lib.lor_eliminate_bc(pat.nrows, pat.nnz, batch, _ptr(pat.row_ptr), _ptr(pat.col_idx), _ptr(values),
                                _dtype_code(values.dtype), ess.numel(), _ptr(ess), _ptr(marker),
                                _DIAG_POLICY[diag_policy], _ptr(diag), _stream()))
    return marker


def lor_discrete_gradient(pat: Pattern, elem_dofs, elem_edges, ndofs_h1: int, dtype=torch.float64,
                          diag: torch.Tensor | None = None, out=None):
    """Discrete gradient (vertices -> edges) in CSR: (row_ptr, col_idx, values)
    with two entries per row; `pat` is the H(curl) pattern of elem_edges.
    `out` may hold preallocated (row_ptr, col_idx, values)."""
    lib = load_library()
    dev = pat.row_ptr.device
    ed = _dev_tensor(elem_dofs, torch.int32, "elem_dofs", dev)
    ee = _dev_tensor(elem_edges, torch.int32, "elem_edges", dev)
    p = pat.p
    _need(ed, pat.nel * (p + 1) ** 3, "elem_dofs")
    _need(ee, pat.nel * 3 * p * (p + 1) ** 2, "elem_edges")
    diag = _diag(diag, 2, dev)
    rp, ci, v = out if out is not None else (None, None, None)
    rp = _out(rp, (pat.nrows + 1,), torch.int32, dev, "row_ptr")
    ci = _out(ci, (2 * pat.nrows,), torch.int32, dev, "col_idx")
    v = _out(v, (2 * pat.nrows,), dtype, dev, "values")
    _check(lib.lor_discrete_gradient(pat.p, pat.nel, ndofs_h1, pat.nrows, _ptr(ed), _ptr(ee), ctypes.byref(pat.sched),
                                     _ptr(rp), _ptr(ci), _ptr(v), _dtype_code(dtype), _ptr(diag), _stream()))
    return rp, ci, v


def lor_discrete_curl(p: int, elem_edges, elem_faces, nedges: int, nfaces: int, dtype=torch.float64,
                      diag: torch.Tensor | None = None, workspace: torch.Tensor | None = None, out=None,
                      device=None):
    """Discrete curl (edges -> faces) in CSR: (row_ptr, col_idx, values) with
    four entries per row.  `out` may hold preallocated outputs."""
    lib = load_library()
    dev = torch.device("cuda") if device is None else torch.device(device)
    ee = _dev_tensor(elem_edges, torch.int32, "elem_edges", dev)
    fm = _dev_tensor(elem_faces, torch.int32, "elem_faces", dev)
    nel = fm.shape[0] if fm.dim() == 2 else 0
    _need(fm, nel * 3 * p * p * (p + 1), "elem_faces")
    _need(ee, nel * 3 * p * (p + 1) ** 2, "elem_edges")
    diag = _diag(diag, 2, dev)
    workspace = _out(workspace, (nfaces,), torch.int32, dev, "workspace")
    rp, ci, v = out if out is not None else (None, None, None)
    rp = _out(rp, (nfaces + 1,), torch.int32, dev, "row_ptr")
    ci = _out(ci, (4 * nfaces,), torch.int32, dev, "col_idx")
    v = _out(v, (4 * nfaces,), dtype, dev, "values")
    _check(lib.lor_discrete_curl(p, nel, nedges, nfaces, _ptr(ee), _ptr(fm), _ptr(workspace), _ptr(rp), _ptr(ci),
                                 _ptr(v), _dtype_code(dtype), _ptr(diag), _stream()))
    return rp, ci, v


def lor_interp_nodes(nodes, p: int, q: int, out: torch.Tensor | None = None) -> torch.Tensor:
    """High-order mesh nodes [nel, (q+1)^3, ncomp] -> LOR lattice E-vector
    [nel, (p+1)^3, ncomp] (float64, on the current CUDA device)."""
    lib = load_library()
    dev = torch.device("cuda") if not (torch.is_tensor(nodes) and nodes.is_cuda) else nodes.device
    X = _dev_tensor(nodes, torch.float64, "nodes", dev)
    if X.dim() != 3 or X.shape[1] != (q + 1) ** 3 or not 1 <= X.shape[2] <= 3:
        raise ValueError("nodes must have shape [nel, (q+1)^3, ncomp] with ncomp in 1..3")
    nel, _, nc = X.shape
    out = _out(out, (nel, (p + 1) ** 3, nc), torch.float64, dev)
    _check(lib.lor_interp_nodes(p, q, nel, nc, _ptr(X), _ptr(out), _stream()))
    return out


def lor_evec_to_tvec(pat: Pattern, evec: torch.Tensor, diag: torch.Tensor | None = None,
                     out: torch.Tensor | None = None) -> torch.Tensor:
    """E-vector [nel, (p+1)^3, ncomp] -> T-vector [nrows, ncomp] by first
    incidence; `pat` is the H1 pattern of the element map."""
    lib = load_library()
    dev = pat.row_ptr.device
    E = _dev_tensor(evec, torch.float64, "evec", dev)
    if E.dim() != 3 or E.shape[0] != pat.nel or E.shape[1] != (pat.p + 1) ** 3:
        raise ValueError("evec must have shape [nel, (p+1)^3, ncomp]")
    nc = E.shape[2]
    diag = _diag(diag, 1, dev)
    out = _out(out, (pat.nrows, nc), torch.float64, dev)
    _check(lib.lor_evec_to_tvec(pat.p, pat.nel, pat.nrows, ctypes.byref(pat.sched), nc, _ptr(E), _ptr(out),
                                _ptr(diag), _stream()))
    return out


def lor_refine_map(p: int, elem_dofs, device=None, out: torch.Tensor | None = None) -> torch.Tensor:
    """Explicit LOR mesh: [nel * p^3, 8] int32 vertex ids of every subelement."""
    lib = load_library()
    dev = torch.device("cuda") if device is None else torch.device(device)
    ed = _dev_tensor(elem_dofs, torch.int32, "elem_dofs", dev)
    nel = ed.shape[0] if ed.dim() == 2 else 0
    _need(ed, nel * (p + 1) ** 3, "elem_dofs")
    out = _out(out, (nel * p ** 3, 8), torch.int32, dev)
    _check(lib.lor_refine_map(p, nel, _ptr(ed), _ptr(out), _stream()))
    return out


def lor_assemble_h1_unstructured(pat: Pattern, sub_map, coords, kappa, beta: float,
                                 diag: torch.Tensor | None = None, out: torch.Tensor | None = None) -> torch.Tensor:
    """The generic comparator: the H1 LOR matrix (FP64) from the explicit LOR
    mesh with per-element dense matrices and atomic adds (not bitwise
    reproducible).  `pat` supplies the CSR pattern; kappa is per subelement."""
    lib = load_library()
    dev = pat.row_ptr.device
    sm = _dev_tensor(sub_map, torch.int32, "sub_map", dev)
    x = _dev_tensor(coords, torch.float64, "coords", dev)
    k = _dev_tensor(kappa, torch.float64, "kappa", dev).reshape(-1)
    if sm.dim() != 2 or sm.shape[1] != 8 or k.numel() != sm.shape[0]:
        raise ValueError("sub_map must be [nsub, 8] and kappa hold one value per element")
    _need(x, pat.nrows * 3, "coords")
    diag = _diag(diag, 2, dev)
    out = _out(out, (pat.nnz,), torch.float64, dev)
    _check(lib.lor_assemble_h1_unstructured(sm.shape[0], pat.nrows, pat.nnz, _ptr(sm), _ptr(x), _ptr(k), float(beta),
                                            _ptr(pat.row_ptr), _ptr(pat.col_idx), _ptr(out), _ptr(diag), _stream()))
    return out


class LorH1(torch.autograd.Function):
    """values = assemble_h1(coords, kappa); backward through the hand-written adjoint
    kernel (geometry recomputed, not stored).  beta gets no gradient."""

    @staticmethod
    def forward(ctx, coords, kappa, beta, pat, elem_dofs):
        dtype = kappa.dtype
        vals = lor_assemble_h1(pat, elem_dofs, coords, kappa, beta, dtype=dtype)
        ctx.save_for_backward(coords, kappa)
        ctx.pat, ctx.elem_dofs, ctx.beta = pat, elem_dofs, beta
        return vals

    @staticmethod
    def backward(ctx, grad_values):
        coords, kappa = ctx.saved_tensors
        gk, gx = lor_assemble_backward(ctx.pat, ctx.elem_dofs, coords, kappa, ctx.beta,
                                       grad_values.contiguous(), dtype=kappa.dtype)
        return gx.to(coords.dtype).reshape(coords.shape), gk.reshape(kappa.shape), None, None, None
