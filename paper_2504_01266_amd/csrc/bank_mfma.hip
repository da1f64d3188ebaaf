// BF16 filter bank on the matrix cores: placeholder until the kernels land.
#include "f2d_host.hpp"

namespace f2d {

f2d_status bank_forward_bf16(const Problem&, const f2d_tensor*, hipStream_t) {
  return fail(F2D_EUNSUPPORTED, "bf16 banks are not implemented yet");
}

size_t bank_backward_bf16_workspace(const Problem&) { return 256; }

f2d_status bank_backward_bf16(const Problem&, const f2d_tensor&, const f2d_tensor*, float*, void*, size_t,
                              hipStream_t) {
  return fail(F2D_EUNSUPPORTED, "bf16 banks are not implemented yet");
}

}  // namespace f2d
