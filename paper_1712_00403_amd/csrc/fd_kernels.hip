// Launch dispatch and host-side packing of the factors for the pass kernels.
#include <hip/hip_runtime.h>

#include <cstring>

#include "fd_internal.h"
#include "fd_pass3.inc"

namespace fdk {

template <int P> hipError_t launch_p(const PassArgs& args, int max_mt, hipStream_t stream);
extern template hipError_t launch_p<0>(const PassArgs&, int, hipStream_t);
extern template hipError_t launch_p<1>(const PassArgs&, int, hipStream_t);
extern template hipError_t launch_p<2>(const PassArgs&, int, hipStream_t);
extern template hipError_t launch_p<3>(const PassArgs&, int, hipStream_t);
extern template hipError_t launch_p<4>(const PassArgs&, int, hipStream_t);
extern template hipError_t launch_p<5>(const PassArgs&, int, hipStream_t);

static size_t elem_bytes(int prec);
static uint16_t to_bf16(float x);
static float from_bf16(uint16_t h);

template <int P>
hipError_t launch2_p(const PassArgs& args, int mode, int mt_bucket, size_t smem, hipStream_t stream);
extern template hipError_t launch2_p<0>(const PassArgs&, int, int, size_t, hipStream_t);
extern template hipError_t launch2_p<1>(const PassArgs&, int, int, size_t, hipStream_t);
extern template hipError_t launch2_p<2>(const PassArgs&, int, int, size_t, hipStream_t);
extern template hipError_t launch2_p<3>(const PassArgs&, int, int, size_t, hipStream_t);
extern template hipError_t launch2_p<4>(const PassArgs&, int, int, size_t, hipStream_t);
extern template hipError_t launch2_p<5>(const PassArgs&, int, int, size_t, hipStream_t);

template <int P>
static bool v2_plan_p(int mode, int max_n, int max_mt, int* bucket, int* chunk, size_t* smem) {
  const int b = v2_mt<P>(max_mt);
  if (b > v2_max_mt<P>()) return false;
  const size_t bytes = v2_lds_bytes<P>(max_n, mode == 2);
  if (bytes > 160 * 1024) return false;
  *bucket = b;
  *chunk = kV2Waves * 16 * v2_pt<P>(b, mode);
  *smem = bytes;
  return true;
}

template <int P>
hipError_t launch3_p(const PassArgs& args, int mode, int mt, size_t smem, hipStream_t stream);
extern template hipError_t launch3_p<0>(const PassArgs&, int, int, size_t, hipStream_t);
extern template hipError_t launch3_p<1>(const PassArgs&, int, int, size_t, hipStream_t);
extern template hipError_t launch3_p<2>(const PassArgs&, int, int, size_t, hipStream_t);
extern template hipError_t launch3_p<3>(const PassArgs&, int, int, size_t, hipStream_t);
extern template hipError_t launch3_p<4>(const PassArgs&, int, int, size_t, hipStream_t);
extern template hipError_t launch3_p<5>(const PassArgs&, int, int, size_t, hipStream_t);
extern template hipError_t launch3_p<6>(const PassArgs&, int, int, size_t, hipStream_t);
extern template hipError_t launch3_p<7>(const PassArgs&, int, int, size_t, hipStream_t);
extern template hipError_t launch3_p<8>(const PassArgs&, int, int, size_t, hipStream_t);

int v2_max_mt_of(int prec) { return prec == 0 ? v2_max_mt<0>() : prec == 1 ? v2_max_mt<1>() : v2_max_mt<2>(); }

template <int P>
static bool v3_plan_p(int mode, int max_n, int mt, int* chunk, size_t* smem) {
  if (mt < 1 || mt > v3_max_mt<P>(mode)) return false;
  (void)max_n;
  const size_t bytes = v3_lds_bytes<P>(mt, mode);
  if (bytes > 160 * 1024) return false;
  *chunk = v3_np<P>(mt, mode);
  *smem = bytes;
  return true;
}

int v3_mt(int prec, int mt) { return prec >= 2 ? (mt + 1) / 2 * 2 : mt; }

bool v3_plan(int prec, int mode, int max_n, int mt, int* chunk, size_t* smem) {
  if (mode == 3 && prec != 0) return false;  // (forward + Lambda pass: FP64 only)
  if (prec == 0) return v3_plan_p<0>(mode, max_n, mt, chunk, smem);
  if (prec == 1) return v3_plan_p<1>(mode, max_n, mt, chunk, smem);
  if (prec == 2) return v3_plan_p<2>(mode, max_n, v3_mt(prec, mt), chunk, smem);
  if (prec == 3) return v3_plan_p<3>(mode, max_n, v3_mt(prec, mt), chunk, smem);
  if (prec == 4) return v3_plan_p<4>(mode, max_n, v3_mt(prec, mt), chunk, smem);
  if (prec == 5) return v3_plan_p<5>(mode, max_n, v3_mt(prec, mt), chunk, smem);
  if (prec == 6) return v3_plan_p<6>(mode, max_n, v3_mt(prec, mt), chunk, smem);
  // 16-bit data classes: the fused last-mode pass only
  if (prec == 7 && mode == 2) return v3_plan_p<7>(mode, max_n, v3_mt(prec, mt), chunk, smem);
  if (prec == 8 && mode == 2) return v3_plan_p<8>(mode, max_n, v3_mt(prec, mt), chunk, smem);
  return false;
}

hipError_t launch_pass3(const PassArgs& args, int prec, int mode, int mt, size_t smem, hipStream_t stream) {
  if (args.total_tiles <= 0) return hipSuccess;
  if (prec == 0) return launch3_p<0>(args, mode, mt, smem, stream);
  if (prec == 1) return launch3_p<1>(args, mode, mt, smem, stream);
  if (prec == 2) return launch3_p<2>(args, mode, v3_mt(prec, mt), smem, stream);
  if (prec == 3) return launch3_p<3>(args, mode, v3_mt(prec, mt), smem, stream);
  if (prec == 4) return launch3_p<4>(args, mode, v3_mt(prec, mt), smem, stream);
  if (prec == 5) return launch3_p<5>(args, mode, v3_mt(prec, mt), smem, stream);
  if (prec == 6) return launch3_p<6>(args, mode, v3_mt(prec, mt), smem, stream);
  if (prec == 7) return launch3_p<7>(args, mode, v3_mt(prec, mt), smem, stream);
  if (prec == 8) return launch3_p<8>(args, mode, v3_mt(prec, mt), smem, stream);
  return hipErrorInvalidValue;
}

bool v2_plan(int prec, int mode, int max_n, int max_mt, int* bucket, int* chunk, size_t* smem) {
  switch (prec) {
    case 0: return v2_plan_p<0>(mode, max_n, max_mt, bucket, chunk, smem);
    case 1: return v2_plan_p<1>(mode, max_n, max_mt, bucket, chunk, smem);
    case 2: return v2_plan_p<2>(mode, max_n, max_mt, bucket, chunk, smem);
    case 3: return v2_plan_p<3>(mode, max_n, max_mt, bucket, chunk, smem);
    case 4: return v2_plan_p<4>(mode, max_n, max_mt, bucket, chunk, smem);
    case 5: return v2_plan_p<5>(mode, max_n, max_mt, bucket, chunk, smem);
    default: return false;
  }
}

hipError_t launch_pass2(const PassArgs& args, int prec, int mode, int bucket, size_t smem,
                        hipStream_t stream) {
  if (args.total_tiles <= 0) return hipSuccess;
  switch (prec) {
    case 0: return launch2_p<0>(args, mode, bucket, smem, stream);
    case 1: return launch2_p<1>(args, mode, bucket, smem, stream);
    case 2: return launch2_p<2>(args, mode, bucket, smem, stream);
    case 3: return launch2_p<3>(args, mode, bucket, smem, stream);
    case 4: return launch2_p<4>(args, mode, bucket, smem, stream);
    case 5: return launch2_p<5>(args, mode, bucket, smem, stream);
    default: return hipErrorInvalidValue;
  }
}

// ---------------------------------------------------------------- batched launch
template <int P> hipError_t batch_launch_p(const BatchArgs&, int, size_t, hipStream_t);
template <int P> hipError_t batch_resident_p(size_t, int*);
extern template hipError_t batch_launch_p<0>(const BatchArgs&, int, size_t, hipStream_t);
extern template hipError_t batch_launch_p<1>(const BatchArgs&, int, size_t, hipStream_t);
extern template hipError_t batch_launch_p<2>(const BatchArgs&, int, size_t, hipStream_t);
extern template hipError_t batch_launch_p<3>(const BatchArgs&, int, size_t, hipStream_t);
extern template hipError_t batch_launch_p<4>(const BatchArgs&, int, size_t, hipStream_t);
extern template hipError_t batch_launch_p<5>(const BatchArgs&, int, size_t, hipStream_t);
extern template hipError_t batch_resident_p<0>(size_t, int*);
extern template hipError_t batch_resident_p<1>(size_t, int*);
extern template hipError_t batch_resident_p<2>(size_t, int*);
extern template hipError_t batch_resident_p<3>(size_t, int*);
extern template hipError_t batch_resident_p<4>(size_t, int*);
extern template hipError_t batch_resident_p<5>(size_t, int*);

int batch_mt(int prec, int mt);
template <int P> static int batch_chunk_p(int mode, int mt, int narrow) {
  return kV2Waves * 16 * (narrow ? 1 : v2_pt<P>(batch_mt(P, mt), mode));
}

int batch_chunk(int prec, int mode, int mt, int narrow) {
  switch (prec) {
    case 0: return batch_chunk_p<0>(mode, mt, narrow);
    case 1: return batch_chunk_p<1>(mode, mt, narrow);
    case 2: return batch_chunk_p<2>(mode, mt, narrow);
    case 3: return batch_chunk_p<3>(mode, mt, narrow);
    case 4: return batch_chunk_p<4>(mode, mt, narrow);
    default: return batch_chunk_p<5>(mode, mt, narrow);
  }
}

template <int P> static void batch_plan3_p(int mode, int mt, int* chunk, size_t* smem) {
  *chunk = v3_np<P>(mt, mode, kV2Waves);
  *smem = v3_lds_bytes<P>(mt, mode, kV2Waves);
}

bool batch_plan3(int prec, int mode, int mt, int* body_mt, int* chunk, size_t* smem) {
  if (prec > 3 || mode < 0 || mode > 2) return false;
  const int m = v3_mt(prec, mt);
  if (m < 1 || m > kBatchMaxMT) return false;
  switch (prec) {
    case 0: batch_plan3_p<0>(mode, m, chunk, smem); break;
    case 1: batch_plan3_p<1>(mode, m, chunk, smem); break;
    case 2: batch_plan3_p<2>(mode, m, chunk, smem); break;
    default: batch_plan3_p<3>(mode, m, chunk, smem); break;
  }
  *body_mt = m;
  return *smem <= 160 * 1024;
}

int batch_mt(int prec, int mt) {
  (void)prec;
  return (mt + 1) / 2 * 2;
}

size_t batch_lds_bytes(int prec, int n, bool fused) {
  switch (prec) {
    case 0: return v2_lds_bytes<0>(n, fused);
    case 1: return v2_lds_bytes<1>(n, fused);
    case 2: return v2_lds_bytes<2>(n, fused);
    case 3: return v2_lds_bytes<3>(n, fused);
    case 4: return v2_lds_bytes<4>(n, fused);
    default: return v2_lds_bytes<5>(n, fused);
  }
}

hipError_t batch_resident(int prec, size_t smem, int* per_cu) {
  switch (prec) {
    case 0: return batch_resident_p<0>(smem, per_cu);
    case 1: return batch_resident_p<1>(smem, per_cu);
    case 2: return batch_resident_p<2>(smem, per_cu);
    case 3: return batch_resident_p<3>(smem, per_cu);
    case 4: return batch_resident_p<4>(smem, per_cu);
    default: return batch_resident_p<5>(smem, per_cu);
  }
}

template <int P> hipError_t batch_seg_launch_p(const BatchArgs&, int, int, size_t, hipStream_t);
template <int P> hipError_t batch_seg_resident_p(size_t, int*);
extern template hipError_t batch_seg_launch_p<0>(const BatchArgs&, int, int, size_t, hipStream_t);
extern template hipError_t batch_seg_launch_p<1>(const BatchArgs&, int, int, size_t, hipStream_t);
extern template hipError_t batch_seg_launch_p<2>(const BatchArgs&, int, int, size_t, hipStream_t);
extern template hipError_t batch_seg_launch_p<3>(const BatchArgs&, int, int, size_t, hipStream_t);
extern template hipError_t batch_seg_launch_p<4>(const BatchArgs&, int, int, size_t, hipStream_t);
extern template hipError_t batch_seg_launch_p<5>(const BatchArgs&, int, int, size_t, hipStream_t);
extern template hipError_t batch_seg_resident_p<0>(size_t, int*);
extern template hipError_t batch_seg_resident_p<1>(size_t, int*);
extern template hipError_t batch_seg_resident_p<2>(size_t, int*);
extern template hipError_t batch_seg_resident_p<3>(size_t, int*);
extern template hipError_t batch_seg_resident_p<4>(size_t, int*);
extern template hipError_t batch_seg_resident_p<5>(size_t, int*);

hipError_t batch_seg_launch(const BatchArgs& args, int prec, int k, int grid, size_t smem, hipStream_t stream) {
  switch (prec) {
    case 0: return batch_seg_launch_p<0>(args, k, grid, smem, stream);
    case 1: return batch_seg_launch_p<1>(args, k, grid, smem, stream);
    case 2: return batch_seg_launch_p<2>(args, k, grid, smem, stream);
    case 3: return batch_seg_launch_p<3>(args, k, grid, smem, stream);
    case 4: return batch_seg_launch_p<4>(args, k, grid, smem, stream);
    default: return batch_seg_launch_p<5>(args, k, grid, smem, stream);
  }
}

hipError_t batch_seg_resident(int prec, size_t smem, int* per_cu) {
  switch (prec) {
    case 0: return batch_seg_resident_p<0>(smem, per_cu);
    case 1: return batch_seg_resident_p<1>(smem, per_cu);
    case 2: return batch_seg_resident_p<2>(smem, per_cu);
    case 3: return batch_seg_resident_p<3>(smem, per_cu);
    case 4: return batch_seg_resident_p<4>(smem, per_cu);
    default: return batch_seg_resident_p<5>(smem, per_cu);
  }
}

extern template hipError_t launch_seg3_p<7>(const BatchDesc*, const BatchSeg&, int, size_t, hipStream_t);
extern template hipError_t launch_seg3_p<8>(const BatchDesc*, const BatchSeg&, int, size_t, hipStream_t);

hipError_t launch_seg3(const BatchDesc* table, const BatchSeg& sg, int prec, int mt, size_t smem,
                       hipStream_t stream) {
  if (prec == 7) return launch_seg3_p<7>(table, sg, v3_mt(prec, mt), smem, stream);
  if (prec == 8) return launch_seg3_p<8>(table, sg, v3_mt(prec, mt), smem, stream);
  return hipErrorInvalidValue;
}

hipError_t batch_launch(const BatchArgs& args, int prec, int grid, size_t smem, hipStream_t stream) {
  switch (prec) {
    case 0: return batch_launch_p<0>(args, grid, smem, stream);
    case 1: return batch_launch_p<1>(args, grid, smem, stream);
    case 2: return batch_launch_p<2>(args, grid, smem, stream);
    case 3: return batch_launch_p<3>(args, grid, smem, stream);
    case 4: return batch_launch_p<4>(args, grid, smem, stream);
    default: return batch_launch_p<5>(args, grid, smem, stream);
  }
}

__global__ void fd_batch_reset_kernel(uint32_t* barrier, int32_t* error) {
  if (threadIdx.x == 0) {
    *barrier = 0u;
    *error = 0;
  }
}

hipError_t batch_reset(uint32_t* barrier, int32_t* error, hipStream_t stream) {
  hipLaunchKernelGGL(fd_batch_reset_kernel, dim3(1), dim3(64), 0, stream, barrier, error);
  return hipGetLastError();
}

size_t lam_table_bytes(const PassArgs& args) {
  size_t e = 0;
  for (int k = 0; k < args.count; ++k) {
    const PassDesc& v = args.u[k];
    e += size_t(v.lam_ndim == 3 ? v.n1 + v.A / v.n1 : v.A) + size_t(v.n);
  }
  return e * sizeof(float);
}

size_t plain_bytes(int n, int prec) {
  if (prec == 6) return 0;  // the FP8 class has pipelined images only
  const size_t per = size_t(n) * n * elem_bytes(prec);
  return (prec == 4 || prec == 5) ? 2 * per : per;
}

int v3_ld(int n, int prec) {
  // = rows: the fused pass contracts over all 16 MT rows (MT even for 16-bit)
  const int r = prec >= 2 ? 32 : 16;
  return (n + r - 1) / r * r;
}

size_t v3_factor_bytes(int n, int prec) {
  if (prec < 0 || prec > 6) return 0;
  const size_t eb = prec == 0 ? 8 : (prec == 1 ? 4 : 2);
  const size_t planes = (prec == 4 || prec == 5) ? 2 : 1;  // split classes: hi plane, then lo plane
  return planes * size_t(v3_ld(n, prec)) * v3_ld(n, prec) * eb;
}

void v3_factor(int n, const double* F, int prec, bool second, void* dst) {
  const int ld = v3_ld(n, prec);
  std::memset(dst, 0, v3_factor_bytes(n, prec));
  for (int r = 0; r < n; ++r)
    for (int c = 0; c < n; ++c) {
      int pos = c;
      // second product of the fused pass: the first product's accumulator
      // registers are the operand, so the columns follow their layout
      if (second && prec == 1) pos = (c & ~15) | (4 * (c & 3) + ((c & 15) >> 2));
      if (second && prec >= 2) {
        // within 32 columns: column 4 g + j at 8 g + j, column 16 + 4 g + j at 8 g + 4 + j
        const int w = c & 31, hi = w >> 4, g = (w & 15) >> 2, j = w & 3;
        pos = (c & ~31) | (8 * g + 4 * hi + j);
      }
      // FP64/FP32: rows with bit 3 set swap the halves of each 16-byte chunk
      // (the LDS bank layout of the pipelined kernels, rhalf)
      if (prec == 0) pos ^= rhalf(r);
      if (prec == 1) pos ^= 2 * rhalf(r);
      const double v = F[r + size_t(n) * c];
      const size_t idx = size_t(r) * ld + pos;
      const size_t lo = size_t(ld) * ld;  // the lo plane of the split classes
      if (prec == 0) {
        reinterpret_cast<double*>(dst)[idx] = v;
      } else if (prec == 1) {
        reinterpret_cast<float*>(dst)[idx] = float(v);
      } else if (prec == 2 || prec == 4) {
        const uint16_t h = to_bf16(float(v));
        reinterpret_cast<uint16_t*>(dst)[idx] = h;
        if (prec == 4) reinterpret_cast<uint16_t*>(dst)[lo + idx] = to_bf16(float(v - double(from_bf16(h))));
      } else {
        const _Float16 h = (_Float16)float(v);
        reinterpret_cast<_Float16*>(dst)[idx] = h;
        if (prec == 5) reinterpret_cast<_Float16*>(dst)[lo + idx] = (_Float16)float(v - double((float)h));
      }
    }
}

void v3_factor_f32(int n, const double* F, bool second, float scale, float* dst) {
  const int ld = v3_ld(n, 6);
  std::memset(dst, 0, sizeof(float) * size_t(ld) * ld);
  for (int r = 0; r < n; ++r)
    for (int c = 0; c < n; ++c) {
      int pos = c;
      if (second) {  // as the 16-bit classes: column 4 g + j at 8 g + j, 16 + 4 g + j at 8 g + 4 + j
        const int w = c & 31, hi = w >> 4, g = (w & 15) >> 2, j = w & 3;
        pos = (c & ~31) | (8 * g + 4 * hi + j);
      }
      dst[size_t(r) * ld + pos] = float(F[r + size_t(n) * c] * double(scale));
    }
}

void plain_factor(int n, const double* F, int prec, void* dst) {
  const size_t nn = size_t(n) * n;
  for (int r = 0; r < n; ++r)
    for (int c = 0; c < n; ++c) {
      const double v = F[r + size_t(n) * c];
      const size_t idx = size_t(r) * n + c;  // row-major
      if (prec == 0) {
        reinterpret_cast<double*>(dst)[idx] = v;
      } else if (prec == 1) {
        reinterpret_cast<float*>(dst)[idx] = float(v);
      } else if (prec == 2 || prec == 4) {
        const uint16_t h = to_bf16(float(v));
        reinterpret_cast<uint16_t*>(dst)[idx] = h;
        if (prec == 4) reinterpret_cast<uint16_t*>(dst)[nn + idx] = to_bf16(float(v - double(from_bf16(h))));
      } else {
        const _Float16 h = (_Float16)float(v);
        reinterpret_cast<_Float16*>(dst)[idx] = h;
        if (prec == 5) reinterpret_cast<_Float16*>(dst)[nn + idx] = (_Float16)float(v - double((float)h));
      }
    }
}

int mfma_kstep(int prec) { return (prec <= 1) ? 4 : 32; }

static size_t elem_bytes(int prec) { return prec == 0 ? 8 : prec == 1 ? 4 : 2; }

size_t packed_bytes(int n, int prec) {
  if (prec == 6) return 0;
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
