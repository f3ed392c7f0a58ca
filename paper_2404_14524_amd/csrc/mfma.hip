// BF16 matrix-core sketch (placeholder until the MFMA kernels land).
#include "common.hpp"
#include "kernels.hpp"

namespace nys {
int sketch_bf16(nys_handle h, const nys_matrix*, const double*, const double*, int, double*) {
  return set_error(h, NYS_EINVAL, "BF16 sketch not built");
}
}  // namespace nys
