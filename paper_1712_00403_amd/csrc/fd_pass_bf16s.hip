// Pass kernels instantiated for precision class 4 (bf16s).
#include "fd_pass.inc"

namespace fdk {
template hipError_t launch_p<4>(const PassArgs&, int, hipStream_t);
}  // namespace fdk
