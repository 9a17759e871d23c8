// Batched persistent kernel instantiated for precision class 3 (f16).
#include "fd_pass.inc"
#include "fd_pass2.inc"
#include "fd_batch.inc"

namespace fdk {
template hipError_t batch_launch_p<3>(const BatchArgs&, int, size_t, hipStream_t);
template hipError_t batch_resident_p<3>(size_t, int*);
template hipError_t batch_seg_launch_p<3>(const BatchArgs&, int, int, size_t, hipStream_t);
template hipError_t batch_seg_resident_p<3>(size_t, int*);
template hipError_t launch_seg3_p<8>(const BatchDesc*, const BatchSeg&, int, size_t, hipStream_t);  // 16-bit data
}  // namespace fdk
