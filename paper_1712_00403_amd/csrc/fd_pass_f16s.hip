// Pass kernels instantiated for precision class 5 (f16s).
#include "fd_pass.inc"

namespace fdk {
template hipError_t launch_p<5>(const PassArgs&, int, hipStream_t);
}  // namespace fdk
