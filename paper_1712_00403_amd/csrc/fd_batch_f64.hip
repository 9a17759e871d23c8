// Batched persistent kernel instantiated for precision class 0 (f64).
#include "fd_pass.inc"
#include "fd_pass2.inc"
#include "fd_batch.inc"

namespace fdk {
template hipError_t batch_launch_p<0>(const BatchArgs&, int, size_t, hipStream_t);
template hipError_t batch_resident_p<0>(size_t, int*);
template hipError_t batch_seg_launch_p<0>(const BatchArgs&, int, int, size_t, hipStream_t);
template hipError_t batch_seg_resident_p<0>(size_t, int*);
}  // namespace fdk
