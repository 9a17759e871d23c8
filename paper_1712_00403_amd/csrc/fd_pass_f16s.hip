// Pass kernels instantiated for precision class 5 (f16s).
#include "fd_pass.inc"
#include "fd_pass2.inc"
#include "fd_pass3.inc"

namespace fdk {
template hipError_t launch_p<5>(const PassArgs&, int, hipStream_t);
template hipError_t launch2_p<5>(const PassArgs&, int, int, size_t, hipStream_t);
template hipError_t launch3_p<5>(const PassArgs&, int, int, size_t, hipStream_t);
}  // namespace fdk
