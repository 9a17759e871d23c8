// Pass kernels instantiated for precision class 1 (f32).
#include "fd_pass.inc"

namespace fdk {
template hipError_t launch_p<1>(const PassArgs&, int, hipStream_t);
}  // namespace fdk
