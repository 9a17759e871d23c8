// Internal types shared by the C-ABI layer and the HIP kernels.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>
#include <vector>

#include "../../include/fd.h"

namespace fdk {

// Pencil tile processed by one workgroup: 4 wavefronts x 16 pencils.
constexpr int kWaves = 4;
constexpr int kTileP = 16 * kWaves;
constexpr int kMaxN = 256;        // largest factor order
constexpr int kMaxMT = kMaxN / 16;
constexpr int kMaxDesc = 8;       // work units per launch (kernel-argument table)

enum PassFlags : int32_t {
  kFuseLambda = 1,   // mode product with F1, divide by Lambda, mode product with F2
  kPreScale = 2,     // multiply the input by scale[] while loading
  kPostScale = 4,    // multiply the output by scale[] while storing
};

// One mode-k pass over nrhs tensors of one plan.
// Tensor view of a residual: element (a, i, b) at a + A*i + A*n*b, with
// a in [0,A), i in [0,n) the contracted index, b in [0,B). Residual j starts
// at j*ld. A pencil is a fixed (a, b); pencils are numbered q = a + A*b.
struct PassDesc {
  const void* in;
  void* out;
  const void* f1;       // packed factor fragments of the (first) mode product
  const void* f2;       // packed factor fragments of the second product (fused pass)
  const void* pf1;      // plain row-major factor (LDS-resident kernels), hi then lo plane
  const void* pf2;      // plain row-major factor of the second product
  const void* pv1;      // padded row-major factor (pipelined kernels; FP64/FP32 plans)
  const void* pv2;      // padded factor of the second product (FP32: columns permuted)
  const void* scale;    // pre/post scale vector (N entries, I/O type)
  const double* d[3];   // eigenvalues per direction (fused pass)
  double w[3];          // direction weights (fused pass)
  int64_t ld;           // elements between residual vectors
  int64_t tile_begin;   // first workgroup index of this unit
  int32_t A, n, B;      // tensor view
  int32_t nrhs;
  int32_t MT, KS;       // output row tiles (16) and contraction steps of the MFMA
  int32_t flags;
  int32_t lam_ndim;     // 2 or 3: how a pencil index splits into direction indices
  int32_t n1;           // first direction size (3D fused pass: a = i1 + n1*i2)
  int32_t tiles_per_rhs;
};

struct PassArgs {
  int32_t count;
  int32_t total_tiles;
  PassDesc u[kMaxDesc];
};

// Storage/compute class of a plan: 0 = FP64 MFMA, 1 = FP32 MFMA,
// 2 = BF16 MFMA, 3 = FP16 MFMA, 4 = BF16 split, 5 = FP16 split.
hipError_t launch_pass(const PassArgs& args, int prec, int max_mt, hipStream_t stream);

// LDS-resident-factor kernels. mode: 0 contracted index fastest, 1 pencil
// index fastest, 2 fused last mode. v2_plan() picks the row-tile bucket and
// reports the pencils per workgroup and LDS bytes, or returns false when the
// factor does not fit in LDS.
bool v2_plan(int prec, int mode, int max_n, int max_mt, int* bucket, int* chunk, size_t* smem);
hipError_t launch_pass2(const PassArgs& args, int prec, int mode, int bucket, size_t smem,
                        hipStream_t stream);
// Pipelined kernels (FP64/FP32, factor and pencil blocks streamed into LDS
// stages by direct global->LDS loads). mt is the exact row-tile count.
bool v3_plan(int prec, int mode, int max_n, int mt, int* chunk, size_t* smem);
hipError_t launch_pass3(const PassArgs& args, int prec, int mode, int mt, size_t smem, hipStream_t stream);
// Bytes of one plain factor (n x n in the storage type, hi and lo planes for split).
size_t plain_bytes(int n, int prec);
void plain_factor(int n, const double* F, int prec, void* dst);
// Padded factor image of the pipelined kernels (FP64/FP32 plans only):
// round_up(n, 16) rows of v3_ld(n, prec) = round_up(n, 16) entries,
// row-major, zero padded.
// `second` stores the image used as the second product of the fused pass
// (FP32: within every 16 columns, column 4g + r sits at position 4r + g).
int v3_ld(int n, int prec);
size_t v3_factor_bytes(int n, int prec);
void v3_factor(int n, const double* F, int prec, bool second, void* dst);

// Bytes of one packed factor (fragment order) for order n and precision.
size_t packed_bytes(int n, int prec);
// Pack F (n x n, F[r + n*c] = row r, column c; the product computes
// out[r] = sum_c F[r][c] in[c]) into MFMA fragment order. For the split
// precisions the low parts follow the high parts in the same buffer.
void pack_factor(int n, const double* F, int prec, void* dst);
int mfma_kstep(int prec);

}  // namespace fdk
