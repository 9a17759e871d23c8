// Pass kernels instantiated for precision class 2 (bf16).
#include "fd_pass.inc"

namespace fdk {
template hipError_t launch_p<2>(const PassArgs&, int, hipStream_t);
}  // namespace fdk
