// Pass kernels instantiated for precision class 0 (f64).
#include "fd_pass.inc"

namespace fdk {
template hipError_t launch_p<0>(const PassArgs&, int, hipStream_t);
}  // namespace fdk
