// Banded Cholesky solves of the pressure-mass block P_Q = M_d (x) .. (x) M_1
// (the O(degree n) route of Sec. 5.2 for P_Q, eq. precQ), one mode per launch.
//
// Mode i applies M_i^{-1} = L_i^{-T} L_i^{-1} along the contracted index of
// the tensor view (a, i, b) at a + A i + A n b: a forward sweep with L_i, then
// a backward sweep with L_i^T, each a recurrence over i that reads the last
// `bw` results. A workgroup owns 64 pencils: it stages them in LDS with
// coalesced loads (rows of 64 consecutive pencils when A > 1, the contiguous
// pencils themselves when A = 1), one thread sweeps each pencil in LDS, and
// the results leave with coalesced stores (modes with A = 1, or a band wider
// than 8); the other modes run one thread per pencil straight from global
// memory with register windows (fd_band_strided_kernel). The band of L_i
// (bw + 1 rows of n: row 0 the reciprocal diagonal) is read with uniform
// addresses (broadcast). Arithmetic in the compute type T
// (FP64 for FP64 plans, FP32 otherwise). Tiles read all of their pencils
// before they write, so the pass may run in place.
#include <hip/hip_runtime.h>

#include <utility>

#include "fd_internal.h"

namespace fdk {

constexpr int kBandP = 64;  // pencils per workgroup (one per thread)

template <class T>
__global__ __launch_bounds__(kBandP) void fd_band_kernel(const BandArgs a) {
  extern __shared__ __align__(16) unsigned char smem_band[];
  const BandDesc& d = a.u;
  const int n = d.n, bw = d.bw, A = d.A;
  const int tid = threadIdx.x;
  const int tile = blockIdx.x;
  const int rhs = tile / d.tiles_per_rhs;
  const int64_t q0 = int64_t(tile - rhs * d.tiles_per_rhs) * kBandP;
  const int64_t NQ = int64_t(A) * d.B;
  T* fac = reinterpret_cast<T*>(smem_band);            // (bw + 1) x n
  T* x = fac + size_t(bw + 1) * n;                       // n rows of kBandP + 1
  constexpr int XS = kBandP + 1;
  const T* gfac = static_cast<const T*>(d.fac);
  for (int e = tid; e < (bw + 1) * n; e += kBandP) fac[e] = gfac[e];
  const T* in = static_cast<const T*>(d.in) + int64_t(rhs) * d.ld;
  T* out = static_cast<T*>(d.out) + int64_t(rhs) * d.ld;
  const int np = int(NQ - q0 < kBandP ? NQ - q0 : kBandP);  // pencils of this tile
  if (A == 1) {
    // pencil q occupies [q n, q n + n): the tile is one contiguous run
    const int64_t base = q0 * n;
    for (int e = tid; e < np * n; e += kBandP) {
      const int p = e / n, i = e - p * n;
      x[i * XS + p] = in[base + e];
    }
  } else {
    const bool ok = tid < np;
    const int64_t q = q0 + tid;
    const int64_t pb = ok ? (q % A) + int64_t(A) * n * (q / A) : 0;
    for (int i = 0; i < n; ++i) x[i * XS + tid] = ok ? in[pb + int64_t(A) * i] : T(0);
  }
  __syncthreads();
  if (tid < np) {
    T* col = x + tid;
    // L y = x
    for (int i = 0; i < n; ++i) {
      T s = col[i * XS];
      for (int j = 1; j <= bw && j <= i; ++j) s -= fac[j * n + i] * col[(i - j) * XS];
      col[i * XS] = s * fac[i];
    }
    // L^T z = y
    for (int i = n - 1; i >= 0; --i) {
      T s = col[i * XS];
      for (int j = 1; j <= bw && i + j < n; ++j) s -= fac[j * n + i + j] * col[(i + j) * XS];
      col[i * XS] = s * fac[i];
    }
  }
  __syncthreads();
  if (A == 1) {
    const int64_t base = q0 * n;
    for (int e = tid; e < np * n; e += kBandP) {
      const int p = e / n, i = e - p * n;
      out[base + e] = x[i * XS + p];
    }
  } else if (tid < np) {
    const int64_t q = q0 + tid;
    const int64_t pb = (q % A) + int64_t(A) * n * (q / A);
    for (int i = 0; i < n; ++i) out[pb + int64_t(A) * i] = x[i * XS + tid];
  }
}

// Modes with A > 1: consecutive pencils are consecutive addresses, so one
// thread per pencil reads and writes global memory directly (coalesced over
// the wavefront) and keeps the last BW results of each sweep in registers;
// no LDS, so many wavefronts per CU hide the latency of the recurrences.
// The forward sweep writes L^{-1} x into out, the backward sweep reads it back
// (the same thread's own stores; L2-resident) and overwrites it with the
// result. The band is read with wavefront-uniform indices.
template <class T, int BW>
__global__ __launch_bounds__(256) void fd_band_strided_kernel(const BandArgs a) {
  const BandDesc& d = a.u;
  const int n = d.n;
  const int64_t A = d.A;
  const int tiles_per_rhs = d.tiles_per_rhs;
  const int rhs = blockIdx.x / tiles_per_rhs;
  const int64_t q = int64_t(blockIdx.x - rhs * tiles_per_rhs) * 256 + threadIdx.x;
  const int64_t NQ = A * d.B;
  if (q >= NQ) return;
  const T* __restrict__ fac = static_cast<const T*>(d.fac);
  const T* in = static_cast<const T*>(d.in) + int64_t(rhs) * d.ld + (q % A) + A * n * (q / A);
  T* out = static_cast<T*>(d.out) + int64_t(rhs) * d.ld + (q % A) + A * n * (q / A);
  T w[BW];
#pragma unroll
  for (int j = 0; j < BW; ++j) w[j] = T(0);
  // L y = x (w[j] = y_{i-1-j})
  for (int i = 0; i < n; ++i) {
    T s = in[A * i];
#pragma unroll
    for (int j = 0; j < BW; ++j)
      if (j < i) s -= fac[(j + 1) * n + i] * w[j];
    const T y = s * fac[i];
#pragma unroll
    for (int j = BW - 1; j > 0; --j) w[j] = w[j - 1];
    w[0] = y;
    out[A * i] = y;
  }
  // L^T z = y (w[j] = z_{i+1+j})
#pragma unroll
  for (int j = 0; j < BW; ++j) w[j] = T(0);
  for (int i = n - 1; i >= 0; --i) {
    T s = out[A * i];
#pragma unroll
    for (int j = 0; j < BW; ++j)
      if (i + j + 1 < n) s -= fac[(j + 1) * n + i + j + 1] * w[j];
    const T z = s * fac[i];
#pragma unroll
    for (int j = BW - 1; j > 0; --j) w[j] = w[j - 1];
    w[0] = z;
    out[A * i] = z;
  }
}

template <class T, int BW>
static hipError_t launch_strided(const BandArgs& args, hipStream_t stream) {
  const int64_t NQ = int64_t(args.u.A) * args.u.B;
  BandArgs a = args;
  a.u.tiles_per_rhs = int((NQ + 255) / 256);
  const int64_t tiles = int64_t(a.u.tiles_per_rhs) * a.u.nrhs;
  if (tiles <= 0) return hipSuccess;
  hipLaunchKernelGGL((fd_band_strided_kernel<T, BW>), dim3(unsigned(tiles)), dim3(256), 0, stream, a);
  return hipGetLastError();
}

template <class T, int... I>
static hipError_t launch_strided_bw(const BandArgs& args, hipStream_t stream, std::integer_sequence<int, I...>) {
  hipError_t res = hipErrorInvalidValue;
  (void)((args.u.bw == I + 1 ? (res = launch_strided<T, I + 1>(args, stream), true) : false) || ...);
  return res;
}

constexpr int kBandStridedMaxBW = 8;  // register windows instantiated for bandwidths 1..8

size_t band_lds_bytes(int n, int bw, bool f64) {
  return (size_t(bw + 1) * n + size_t(n) * (kBandP + 1)) * (f64 ? 8 : 4);
}

hipError_t launch_band(const BandArgs& args, bool f64, hipStream_t stream) {
  if (args.u.A > 1 && args.u.bw >= 1 && args.u.bw <= kBandStridedMaxBW) {
    using seq = std::make_integer_sequence<int, kBandStridedMaxBW>;
    return f64 ? launch_strided_bw<double>(args, stream, seq{}) : launch_strided_bw<float>(args, stream, seq{});
  }
  const size_t smem = band_lds_bytes(args.u.n, args.u.bw, f64);
  const int tiles = args.u.tiles_per_rhs * args.u.nrhs;
  if (tiles <= 0) return hipSuccess;
  if (f64) {
    static const hipError_t attr = hipFuncSetAttribute(reinterpret_cast<const void*>(fd_band_kernel<double>),
                                                       hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
    if (attr != hipSuccess) return attr;
    hipLaunchKernelGGL(fd_band_kernel<double>, dim3(tiles), dim3(kBandP), smem, stream, args);
  } else {
    static const hipError_t attr = hipFuncSetAttribute(reinterpret_cast<const void*>(fd_band_kernel<float>),
                                                       hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
    if (attr != hipSuccess) return attr;
    hipLaunchKernelGGL(fd_band_kernel<float>, dim3(tiles), dim3(kBandP), smem, stream, args);
  }
  return hipGetLastError();
}

int band_tiles_per_rhs(int64_t pencils) { return int((pencils + kBandP - 1) / kBandP); }

}  // namespace fdk
