"""MI355X-native (gfx950) assembly of low-order-refined (LOR) matrices.

The compute path is the HIP library liblor.so (C ABI in include/lor.h); this
package is its Python binding.
"""
from .lor import (  # noqa: F401
    LOR_DIAG_KEEP,
    LOR_DIAG_ONE,
    LOR_DIAG_ZERO,
    LOR_F32,
    LOR_F64,
    LOR_H1,
    LOR_H1_2D,
    LOR_ND,
    LOR_RT,
    LorError,
    LorH1,
    Pattern,
    load_library,
    lor_assemble_backward,
    lor_assemble_backward_noalloc,
    lor_assemble_h1,
    lor_assemble_h1_2d,
    lor_assemble_h1_unstructured,
    lor_assemble_nd,
    lor_assemble_rt,
    lor_discrete_curl,
    lor_discrete_gradient,
    lor_eliminate_bc,
    lor_evec_to_tvec,
    lor_interp_nodes,
    lor_pattern,
    lor_refine_map,
)
