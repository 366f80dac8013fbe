// Values of the LOR H(curl) matrix (lowest-order Nedelec on the refined mesh).
#include "lor_common.hpp"

extern "C" int lor_assemble_nd(int p, int64_t nel, int64_t ndofs_h1, int64_t nedges, int batch,
                               const int32_t* elem_dofs, const int32_t* elem_edges, const double* coords,
                               const void* kappa, double beta, const int32_t* row_ptr, const lor_sched* sched,
                               void* values, int dtype, unsigned flags, double det_ratio_thresh, int32_t* diag,
                               void* stream) {
  lor::clear_error();
  LOR_FAIL(LOR_EUNSUPPORTED, "lor_assemble_nd is not built yet");
}
