// Pass kernels instantiated for precision class 3 (f16).
#include "fd_pass.inc"

namespace fdk {
template hipError_t launch_p<3>(const PassArgs&, int, hipStream_t);
}  // namespace fdk
