// Pass kernels instantiated for precision class 3 (f16).
#include "fd_pass.inc"
#include "fd_pass2.inc"
#include "fd_pass3.inc"

namespace fdk {
template hipError_t launch_p<3>(const PassArgs&, int, hipStream_t);
template hipError_t launch2_p<3>(const PassArgs&, int, int, size_t, hipStream_t);
template hipError_t launch3_p<3>(const PassArgs&, int, int, size_t, hipStream_t);
template hipError_t launch3_p<8>(const PassArgs&, int, int, size_t, hipStream_t);  // 16-bit data
}  // namespace fdk
