// Internal types shared by the C-ABI layer and the HIP kernels.
#pragma once
#include <hip/hip_runtime.h>

#include <atomic>
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
constexpr int kMaxDevices = 64;   // per-device launch state

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
  // FP16 range scaling (powers of two, 1 for the other classes): the input is
  // multiplied by xscale before its conversion to FP16, the fused pass's
  // second operand by qscale, the FP32 result by oscale = 1 / (xscale qscale)
  float xscale, qscale, oscale;
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
  int32_t sA;           // 16-bit data classes: elements between consecutive i (A otherwise)
};

// ---- one persistent launch per batched apply (fd_batch.inc)
constexpr int kBatchMaxMT = 8;             // factor order n <= 128
constexpr uint32_t kBatchSpin = 1u << 22;  // about a second of s_sleep per barrier wait

struct BatchDesc {
  PassDesc u;        // u.tile_begin: first tile of this pass within its stage
  int32_t mode;      // 0 contract-fast, 1 pencil-fast, 2 fused
  int32_t mt;        // row tiles of the body (batch_mt, or v3_mt for the pipelined body)
  int32_t scale;     // 0 none, 1 scale on load, 2 scale on store (mode 0 only)
  int32_t pad;
};

// Bodies of a batch segment: LDS-resident factor with the register-budget
// tile width or one 16-pencil tile per wavefront; pipelined LDS ring.
constexpr int32_t kBodyWide = 0, kBodyNarrow = 1, kBodyPipelined = 2;

// Descriptors [d0, d1) of one stage that share one body (mode, mt, scale,
// body); their tiles are [t0, t1) of the stage.
struct BatchSeg {
  int32_t d0, d1, t0, t1;
  int32_t mode, mt, scale, body;
};

struct BatchArgs {
  const BatchDesc* desc;   // ordered by stage, then body, then tile_begin
  const BatchSeg* seg;     // ordered by stage
  uint32_t* barrier;       // arrival counter
  int32_t* error;          // set to 1 if a barrier wait gave up
  uint32_t base;           // arrivals counted by earlier launches of this batch
  int32_t stage_seg[6];    // segments of stage s: [stage_seg[s], stage_seg[s+1])
  int32_t last_stage;      // last stage with tiles (no barrier after it)
};

struct PassArgs {
  int32_t count;
  int32_t total_tiles;
  int32_t lam_lds;      // pipelined divide passes: 1 = the weighted eigenvalues of every unit sit in LDS
  PassDesc u[kMaxDesc];
};

// ---- slab passes of 3D BF16/FP16 plans (fd_slab.hip)
// One workgroup takes one i3-slab (n1 x n2 entries, contiguous) of one
// residual and applies both in-plane products, out[j1, j2] =
// sum_{i1, i2} F1[j1, i1] F2[j2, i2] x[i1, i2], with the slab and the
// intermediate in LDS. Between the slab passes and the fused last-mode pass
// the tensor lives in z as 16 bits per entry ("16-bit layout"): entry
// (i1, i2, i3) of residual j at 16-bit index 2 j ld + off16 + 2 A i3 + i1 +
// n1 i2 of z (A = n1 n2, off16 = A rounded down to even), i.e. in the upper
// half of the bytes that the FP32 plane i3 of that residual occupies. A slab
// pass therefore reads and writes inside the FP32 footprint of its own slab
// only, which keeps z == r and the final FP32 store race-free.
constexpr int kSlabMaxMT = 9;   // n1, n2 <= 144
constexpr int kSlabWaves = 9;   // 3 x 3 wavefronts, each a block of output tiles

struct SlabDesc {
  const void* in;       // FP32 vectors (in16 == 0) or z in the 16-bit layout
  void* out;            // z: FP32 (out16 == 0) or the 16-bit layout
  const void* f1;       // padded row-major factor image of the product along i1 (ldf1 entries a row)
  const void* f2;       // the same along i2
  const void* scale;    // D^{-1/2} in the 16-bit type, applied on load (pre) or store (post), or
                        // null; plane i3 at (n1 + (n1 & 1)) n2 i3, rows of n1 + (n1 & 1) entries
                        // (an odd row ends with a zero)
  int64_t ld;           // FP32 elements between residual vectors
  int64_t tile_begin;   // first slab of this unit within the launch
  int32_t n1, n2, n3, nrhs;
  int32_t ldf1, ldf2;
  int32_t in16, out16;
  int32_t post;         // 1: scale multiplies the output, 0: the input
  // FP16 range scaling (powers of two, 1 for BF16): input before its
  // conversion, first product's accumulators before theirs, output
  float s_in, s_mid, s_out;
};

struct SlabArgs {
  int32_t count;
  int32_t total_tiles;
  SlabDesc u[kMaxDesc];
};

// The units of a slab launch in a device table (fixed batches): u[0, count)
// ordered by tile_begin. Each workgroup takes one contiguous range of slabs,
// so that it restages the factors only where its range crosses into the
// next unit.
struct SlabTab {
  const SlabDesc* u;
  int32_t count;
  int32_t total_tiles;
};

// 16-bit element offset of the 16-bit layout within each plane of A entries
__host__ __device__ inline int64_t slab_off16(int64_t A) { return A & ~int64_t(1); }
size_t slab_lds_bytes(int mt);
// prec: 2 (BF16) or 3 (FP16); mt: row tiles of max(n1, n2), <= kSlabMaxMT
hipError_t launch_slab(const SlabArgs& args, int prec, int mt, hipStream_t stream);
// fwd: in16 == 0 for every unit; sc: every unit has a scale (the host groups so)
hipError_t launch_slab_tab(const SlabTab& tab, int prec, int mt, bool fwd, bool sc, hipStream_t stream);

// LDS bytes of the weighted-eigenvalue tables of a divide pass (w_0 d_0, w_1 d_1
// and w_l d_l of every unit, FP32), placed after the pipeline ring.
size_t lam_table_bytes(const PassArgs& args);

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
// Largest row-tile count of the pipelined kernels of a class.
int v2_max_mt_of(int prec);
// FP8 split class: the FP32 image of a pipelined factor scaled by `scale`
// (ld x ld floats, ld = v3_ld(n, 6)), and its device conversion to the FP8
// hi/lo image (`entries` a multiple of 8; asynchronous on `stream`).
void v3_factor_f32(int n, const double* F, bool second, float scale, float* dst);
hipError_t fp8s_image(const float* src, void* dst, int64_t entries, hipStream_t stream);
hipError_t launch_pass3(const PassArgs& args, int prec, int mode, int mt, size_t smem, hipStream_t stream);
// The fused last-mode pass of 16-bit data (classes 7, 8) over one segment of
// a device table of passes (fixed batches; factor orders may differ per
// pass): tiles [sg.t0, sg.t1), passes [sg.d0, sg.d1); mt as v3_plan.
hipError_t launch_seg3(const BatchDesc* table, const BatchSeg& sg, int prec, int mt, size_t smem,
                       hipStream_t stream);
// Bytes of one plain factor (n x n in the storage type, hi and lo planes for split).
// Batched persistent launch: pencils per tile and LDS bytes of a pass body,
// resident workgroups per CU, launch, counter reset.
// `narrow`: one pencil tile per wavefront instead of the register-budget default.
int batch_chunk(int prec, int mode, int mt, int narrow);
// The pipelined body of a batch pass (FP64/FP32/BF16/FP16, kV2Waves
// wavefronts): row tiles it runs with, pencils per tile and LDS bytes, or
// false if the class has none or n exceeds the batch limit.
bool batch_plan3(int prec, int mode, int mt, int* body_mt, int* chunk, size_t* smem);
int batch_mt(int prec, int mt);
size_t batch_lds_bytes(int prec, int n, bool fused);
hipError_t batch_resident(int prec, size_t smem, int* per_cu);
hipError_t batch_launch(const BatchArgs& args, int prec, int grid, size_t smem, hipStream_t stream);
hipError_t batch_reset(uint32_t* barrier, int32_t* error, hipStream_t stream);
// The segment route: segment k of the batch's tables as one launch of its own
// (args.desc, args.seg as the persistent launch; barrier fields unused).
hipError_t batch_seg_launch(const BatchArgs& args, int prec, int k, int grid, size_t smem, hipStream_t stream);
hipError_t batch_seg_resident(int prec, size_t smem, int* per_cu);

// ---- banded Cholesky solves of the pressure-mass block (fd_banded.hip)
struct BandDesc {
  const void* in;       // I/O type: double for FP64 plans, float otherwise
  void* out;
  const void* fac;      // (bw + 1) x n in the compute type: row 0 = 1 / L(i,i), row j = L(i, i - j)
  int64_t ld;           // elements between residual vectors
  int32_t A, n, B;      // tensor view of the mode (as PassDesc)
  int32_t nrhs, bw;
  int32_t tiles_per_rhs;
};
struct BandArgs {
  BandDesc u;
};
constexpr int kMaxBand = 16;
size_t band_lds_bytes(int n, int bw, bool f64);
int band_tiles_per_rhs(int64_t pencils);
hipError_t launch_band(const BandArgs& args, bool f64, hipStream_t stream);

size_t plain_bytes(int n, int prec);
void plain_factor(int n, const double* F, int prec, void* dst);
// Padded factor image of the pipelined kernels (FP64, FP32, BF16, FP16
// plans): v3_ld(n, prec) rows and columns (n rounded up to 16, to 32 for the
// 16-bit classes), row-major, zero padded.
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
