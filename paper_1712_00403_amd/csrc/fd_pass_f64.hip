// Pass kernels instantiated for precision class 0 (f64).
#include "fd_pass.inc"
#include "fd_pass3.inc"

namespace fdk {
template hipError_t launch_p<0>(const PassArgs&, int, hipStream_t);
template hipError_t launch2_p<0>(const PassArgs&, int, int, size_t, hipStream_t);
template hipError_t launch3_p<0>(const PassArgs&, int, int, size_t, hipStream_t);
}  // namespace fdk
