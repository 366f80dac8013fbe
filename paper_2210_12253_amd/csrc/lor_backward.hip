// Adjoint of the LOR H1 assembly with respect to kappa and the coordinates.
#include "lor_common.hpp"

extern "C" size_t lor_backward_workspace(int p, int64_t nel) {
  if (p < 1 || p > LOR_MAX_P || nel < 0) return 0;
  return sizeof(double) * 3 * static_cast<size_t>(nel) * lor::nloc_h1(p);
}

extern "C" int lor_assemble_backward(int p, int64_t nel, int64_t ndofs, int batch, const int32_t* elem_dofs,
                                     const double* coords, const void* kappa, double beta, const int32_t* row_ptr,
                                     const lor_sched* sched, const void* grad_values, void* grad_kappa,
                                     double* grad_coords, void* workspace, int dtype, void* stream) {
  lor::clear_error();
  LOR_FAIL(LOR_EUNSUPPORTED, "lor_assemble_backward is not built yet");
}
