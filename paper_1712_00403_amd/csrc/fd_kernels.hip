// Launch dispatch and host-side packing of the factors for the pass kernels.
#include <hip/hip_runtime.h>

#include <cstring>

#include "fd_internal.h"

namespace fdk {

template <int P> hipError_t launch_p(const PassArgs& args, int max_mt, hipStream_t stream);
extern template hipError_t launch_p<0>(const PassArgs&, int, hipStream_t);
extern template hipError_t launch_p<1>(const PassArgs&, int, hipStream_t);
extern template hipError_t launch_p<2>(const PassArgs&, int, hipStream_t);
extern template hipError_t launch_p<3>(const PassArgs&, int, hipStream_t);
extern template hipError_t launch_p<4>(const PassArgs&, int, hipStream_t);
extern template hipError_t launch_p<5>(const PassArgs&, int, hipStream_t);

int mfma_kstep(int prec) { return (prec <= 1) ? 4 : 32; }

static size_t elem_bytes(int prec) { return prec == 0 ? 8 : prec == 1 ? 4 : 2; }

size_t packed_bytes(int n, int prec) {
  const int ks = mfma_kstep(prec);
  const size_t MT = (n + 15) / 16, KS = (n + ks - 1) / ks;
  const size_t per = MT * KS * 16 * ks * elem_bytes(prec);
  return (prec == 4 || prec == 5) ? 2 * per : per;
}

static uint16_t to_bf16(float x) {
  uint32_t u;
  std::memcpy(&u, &x, 4);
  if ((u & 0x7f800000u) == 0x7f800000u) return uint16_t(u >> 16);  // inf / nan
  const uint32_t lsb = (u >> 16) & 1u;
  u += 0x7fffu + lsb;  // round to nearest even
  return uint16_t(u >> 16);
}
static float from_bf16(uint16_t h) {
  uint32_t u = uint32_t(h) << 16;
  float x;
  std::memcpy(&x, &u, 4);
  return x;
}

void pack_factor(int n, const double* F, int prec, void* dst) {
  const int ks = mfma_kstep(prec);
  const int kw = ks / 4;
  const int MT = (n + 15) / 16, KS = (n + ks - 1) / ks;
  const size_t count = size_t(MT) * KS * 64 * kw;
  auto val = [&](int r, int c) -> double { return (r < n && c < n) ? F[r + size_t(n) * c] : 0.0; };
  for (int mt = 0; mt < MT; ++mt)
    for (int k = 0; k < KS; ++k)
      for (int l = 0; l < 64; ++l)
        for (int j = 0; j < kw; ++j) {
          const int r = mt * 16 + (l & 15);
          const int c = k * ks + kw * (l >> 4) + j;
          const size_t idx = ((size_t(mt) * KS + k) * 64 + l) * kw + j;
          const double v = val(r, c);
          if (prec == 0) {
            reinterpret_cast<double*>(dst)[idx] = v;
          } else if (prec == 1) {
            reinterpret_cast<float*>(dst)[idx] = float(v);
          } else if (prec == 2 || prec == 4) {
            const uint16_t h = to_bf16(float(v));
            reinterpret_cast<uint16_t*>(dst)[idx] = h;
            if (prec == 4) reinterpret_cast<uint16_t*>(dst)[count + idx] = to_bf16(float(v - double(from_bf16(h))));
          } else {
            const _Float16 h = (_Float16)float(v);
            reinterpret_cast<_Float16*>(dst)[idx] = h;
            if (prec == 5) reinterpret_cast<_Float16*>(dst)[count + idx] = (_Float16)float(v - double((float)h));
          }
        }
}

hipError_t launch_pass(const PassArgs& args, int prec, int max_mt, hipStream_t stream) {
  if (args.total_tiles <= 0) return hipSuccess;
  switch (prec) {
    case 0: return launch_p<0>(args, max_mt, stream);
    case 1: return launch_p<1>(args, max_mt, stream);
    case 2: return launch_p<2>(args, max_mt, stream);
    case 3: return launch_p<3>(args, max_mt, stream);
    case 4: return launch_p<4>(args, max_mt, stream);
    case 5: return launch_p<5>(args, max_mt, stream);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace fdk
