// Stand-ins for the fused-pass launchers in the sanitized host build: the host driver never
// launches a kernel, and leaving fused_kernels.hip out keeps its device code (minutes of
// compilation) out of the build. Every stand-in reports an invalid launch.
#include "fused.h"

namespace qsv {

template <typename R>
hipError_t launch_fused_forward(const PassItem*, int, int64_t, int64_t, int, int, bool, int,
                                hipStream_t) {
  return hipErrorInvalidValue;
}
template <typename R>
hipError_t launch_fused_backward(const PassItem*, int, int64_t, int64_t, int, int, bool, int,
                                 hipStream_t, bool) {
  return hipErrorInvalidValue;
}
template hipError_t launch_fused_forward<double>(const PassItem*, int, int64_t, int64_t, int, int,
                                                 bool, int, hipStream_t);
template hipError_t launch_fused_forward<float>(const PassItem*, int, int64_t, int64_t, int, int,
                                                bool, int, hipStream_t);
template hipError_t launch_fused_backward<double>(const PassItem*, int, int64_t, int64_t, int,
                                                  int, bool, int, hipStream_t, bool);
template hipError_t launch_fused_backward<float>(const PassItem*, int, int64_t, int64_t, int, int,
                                                 bool, int, hipStream_t, bool);

}  // namespace qsv
