// Batched persistent kernel instantiated for precision class 2 (bf16).
#include "fd_pass.inc"
#include "fd_pass2.inc"
#include "fd_batch.inc"

namespace fdk {
template hipError_t batch_launch_p<2>(const BatchArgs&, int, size_t, hipStream_t);
template hipError_t batch_resident_p<2>(size_t, int*);
}  // namespace fdk
