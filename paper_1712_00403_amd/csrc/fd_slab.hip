// Slab passes of 3D BF16/FP16 plans: the products along directions 1 and 2
// of Algorithm 1, steps 2 and 4 (Sec. 5.2), for one i3-slab at a time.
//
// A slab X (n1 x n2, contiguous in a vector with i1 fastest) goes through
//   P1: Y^T(i2, j1) = sum_i1 X(i1, i2) F1(j1, i1)   A = X, B = F1
//   P2: Z^T(j2, j1) = sum_i2 F2(j2, i2) Y(j1, i2)   A = F2, B = Y
// on 16x16x32 MFMA tiles with FP32 accumulation, every operand read from
// LDS. A workgroup (one per CU at orders above 112, several below) keeps
// both factors in LDS for as long as its slabs belong to one unit, and
// stages each slab in 16 bits (row i2 holds
// the i1 entries, P1's contraction index); P1's accumulators, converted to
// 16 bits, become the rows j1 of Y with i2 contiguous (P2's contraction
// index) in the same LDS image; P2's accumulators hold runs of 16
// consecutive j1 per lane group, so the stores of Z are 32- or 64-byte runs.
// Nine wavefronts split each product's output into 3 x 3 blocks of TB x TB
// tiles, so a fragment read from LDS feeds TB MFMAs.
//
// LDS images: one 64-byte row segment per row and 32-entry contraction
// block, block after block; 16-byte chunk c of row r at position
// c ^ rsw(r) (the layout of the pipelined pass kernels), so that the lanes of
// a fragment read (16 rows, one chunk per lane group) and of a staging store
// hit distinct banks.
//
// Rounding: every entry is rounded to the 16-bit type once before each
// product, exactly as the pencil passes do at their fragment reads, so the
// 16-bit layout between passes (SlabDesc) changes no result. FP16 plans scale
// by powers of two (s_in, s_mid, s_out) to stay in range; BF16 plans use 1.
// Coefficient-aware blocks scale by D^{-1/2} (Sec. 6), read in the 16-bit
// type: the forward pass on load, the backward pass in its epilogue.
//
// Units come from the kernel arguments (up to kMaxDesc per launch, slabs
// strided over the grid) or from a device table (fixed batches, a
// contiguous range of slabs per workgroup).
#include <hip/hip_runtime.h>

#include <atomic>

#include "fd_internal.h"
#include "fd_pass3.inc"

namespace fdk {

template <int P> struct SlabT;
template <> struct SlabT<2> { using s = __bf16; using frag = bf16x8; using v4 = __bf16 __attribute__((ext_vector_type(4))); };
template <> struct SlabT<3> { using s = _Float16; using frag = f16x8; using v4 = _Float16 __attribute__((ext_vector_type(4))); };

// 32-entry contraction blocks of the largest order; bytes of one block of an
// image (ROWS rows of 64 bytes, plus 64 so that consecutive blocks start 16
// banks apart)
__host__ __device__ constexpr int slab_kt(int mt) { return (mt + 1) / 2; }
__host__ __device__ constexpr int slab_bs(int mt) { return 16 * mt * 64 + 64; }

size_t slab_lds_bytes(int mt) { return 3 * size_t(slab_kt(mt)) * size_t(slab_bs(mt)); }
// backward passes with a scale and at most 7 row tiles: the slab's D^{-1/2}
// in LDS as well (16 mt rows of 16 mt + 16 entries, 16-bit)
__host__ __device__ constexpr bool slab_scale_lds(bool fwd, bool sc, int mt) { return !fwd && sc && mt <= 7; }
__host__ __device__ constexpr int slab_sci_bytes(int mt) { return 16 * mt * (16 * mt + 16) * 2; }

typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

// Byte offset of 16-bit entry (r, col) in an image.
template <int BS> __device__ __forceinline__ int slab_at(int r, int col) {
  return (col >> 5) * BS + r * 64 + ((((col >> 3) & 3) ^ rsw(r)) << 4) + ((col & 7) << 1);
}

// Barrier without a memory fence: LDS traffic is complete (lgkmcnt) and the
// previous slab's stores and the next slab's loads stay in flight.
__device__ __forceinline__ void slab_barrier() {
  asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");
  __builtin_amdgcn_s_barrier();
  asm volatile("" ::: "memory");
}

template <class S>
__device__ __forceinline__ void bstore16(__amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff, S v) {
  __builtin_amdgcn_raw_buffer_store_b16(__builtin_bit_cast(unsigned short, v), r, voff, soff, 0);
}

// Position of slab `tile` of a launch: unit, residual, plane.
struct SlabPos {
  int ui, rhs, i3;
  bool valid;
};

// Unit sources of a slab launch (free functions on the kernel argument).
// Kernel-argument table (at most kMaxDesc units): slabs blockIdx.x +
// k gridDim.x; the unit of a slab found by a scan of the table.
__device__ __forceinline__ const SlabDesc& slab_unit(const SlabArgs& args, int ui) { return args.u[ui]; }
__device__ __forceinline__ void slab_range(const SlabArgs& args, int* t0, int* t1, int* step) {
  *t0 = (int)blockIdx.x;
  *t1 = args.total_tiles;
  *step = (int)gridDim.x;
}
__device__ __forceinline__ SlabPos slab_pos(const SlabArgs& args, int tile, const SlabPos&) {
  SlabPos p;
  p.valid = tile < args.total_tiles;
  int ui = 0;
#pragma unroll 1
  for (int k = 1; k < args.count; ++k)
    if (tile >= args.u[k].tile_begin) ui = k;
  p.ui = ui;
  const int tl = p.valid ? tile - (int)args.u[ui].tile_begin : 0;
  p.rhs = tl / args.u[ui].n3;
  p.i3 = tl - p.rhs * args.u[ui].n3;
  return p;
}

// Device table: a contiguous range of slabs per workgroup; the unit of the
// first slab by bisection, of the following ones by stepping forward from
// the previous slab's unit. The table is read through the constant address
// space (scalar loads; it does not change during a launch).
typedef const SlabDesc __attribute__((address_space(4))) SlabDescC;
__device__ __forceinline__ SlabDescC& slab_unit(const SlabTab& t, int ui) { return ((SlabDescC*)t.u)[ui]; }
__device__ __forceinline__ void slab_range(const SlabTab& t, int* t0, int* t1, int* step) {
  const int G = (int)gridDim.x, w = (int)blockIdx.x;
  const int per = t.total_tiles / G, rem = t.total_tiles - per * G;
  *t0 = w * per + (w < rem ? w : rem);
  *t1 = *t0 + per + (w < rem ? 1 : 0);
  *step = 1;
}
__device__ __forceinline__ SlabPos slab_pos(const SlabTab& t, int tile, const SlabPos& hint) {
  SlabPos p;
  p.valid = tile < t.total_tiles;
  int ui = hint.ui;
  if (!hint.valid) {
    int lo = 0, hi = t.count - 1;  // last unit whose first slab is <= tile
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (slab_unit(t, mid).tile_begin <= tile) lo = mid;
      else hi = mid - 1;
    }
    ui = lo;
  } else {
    while (ui + 1 < t.count && slab_unit(t, ui + 1).tile_begin <= tile) ++ui;
  }
  p.ui = ui;
  const int tl = p.valid ? tile - (int)slab_unit(t, ui).tile_begin : 0;
  p.rhs = tl / slab_unit(t, ui).n3;
  p.i3 = tl - p.rhs * slab_unit(t, ui).n3;
  return p;
}

// FWD: the forward slab pass (FP32 input, pre-scaled by D^{-1/2} if SC, 16-bit
// output); otherwise the backward one (16-bit input, FP32 output, post-scaled
// if SC). Both are template parameters so that the load and store sequences
// are straight-line code with a fixed number of memory instructions per
// slab, which keeps the compiler's wait counts exact across the slab loop.
template <int P, int MT, bool FWD, bool SC, class Src>
__global__ __launch_bounds__(64 * kSlabWaves) __attribute__((amdgpu_waves_per_eu(3)))
void fd_slab_kernel(const Src args) {
  using S = typename SlabT<P>::s;
  using frag = typename SlabT<P>::frag;
  using v4 = typename SlabT<P>::v4;
  typedef S s2 __attribute__((ext_vector_type(2)));
  typedef float fl2 __attribute__((ext_vector_type(2)));
  typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));
  constexpr int W = kSlabWaves;
  constexpr int KT = slab_kt(MT), BS = slab_bs(MT), ROWS = 16 * MT;
  constexpr int TB = (MT + 2) / 3;          // tiles of a wavefront along each output dimension
  constexpr int NT = 64 * W;                // threads
  constexpr int XB = KT * BS;               // bytes of one LDS image
  // X staging: wavefront w takes rows w + W k (k < KA) with lane l holding
  // columns 2l, 2l + 1, and (orders above 128) rows 8 (w + W k) + l / 8 with
  // columns 128 + 2 (l % 8), + 1 (k < KB)
  constexpr int KA = (ROWS + W - 1) / W;
  constexpr bool TAILC = MT > 8;
  constexpr int KB = TAILC ? (ROWS + 8 * W - 1) / (8 * W) : 1;
  constexpr int WC = TAILC ? 144 : (32 * KT < 128 ? 32 * KT : 128);  // columns the staging writes
  extern __shared__ __align__(16) unsigned char lds[];
  unsigned char* const xs = lds;            // X, then Y (16-bit)
  unsigned char* const fs1 = lds + XB;      // F1 rows j1, columns i1
  unsigned char* const fs2 = lds + 2 * XB;  // F2 rows j2, columns i2
  // backward pass with a scale: D^{-1/2} of the slab in LDS (SCL; row j2,
  // n1p + 16 entries a row) for the epilogue, or (orders above 112) loaded
  // one slab ahead into registers (SCB)
  constexpr bool SCL = slab_scale_lds(FWD, SC, MT);
  unsigned char* const sci = lds + 3 * XB;

  const int tid0 = threadIdx.x;
  const int wave = __builtin_amdgcn_readfirstlane(tid0 >> 6);
  __builtin_assume(wave >= 0 && wave < W);
  const int wa = wave / 3, wb = wave - 3 * (wave / 3);

  // The next slab's input is loaded into registers while the current slab
  // computes. FWD: xa holds the FP32 pair of a row (lane l: 2l, 2l + 1),
  // xb0/xb1 the tail pair. Backward: xa[.][0]/xp hold the two 16-bit entries
  // of the pair, xb0/xb1 those of the tail pair.
  u32x2 xa[KA];
  uint32_t xp[FWD ? 1 : KA], xb0[KB], xb1[KB];
  // D^{-1/2} in 16 bits, rows of n1 + (n1 & 1) entries (SlabDesc::scale):
  // sa[k] the pair (2l, 2l + 1) of row k's, sbp[k] the tail pair
  uint32_t sa[SC ? KA : 1], sbp[SC ? KB : 1];
  auto scale2 = [](uint32_t w) -> fl2 {
    const s2 h = __builtin_bit_cast(s2, w);
    return fl2{(float)h[0], (float)h[1]};
  };
  auto prefetch = [&](const SlabPos& q, int lane) {
    auto& u = slab_unit(args, q.ui);
    const int n1 = u.n1, n2 = u.n2, A = n1 * n2;
    // (row offsets go in the scalar offset; an out-of-range vector offset
    // stays out of range with it: A * 4 < 2^31)
    if constexpr (FWD) {
      const __amdgpu_buffer_rsrc_t rin =
          make_rsrc(reinterpret_cast<const float*>(u.in) + ((int64_t)q.rhs * u.ld + (int64_t)A * q.i3), (uint32_t)A * 4);
      const int n1p = n1 + (n1 & 1);
      const __amdgpu_buffer_rsrc_t rsc =
          make_rsrc(SC ? static_cast<const S*>(u.scale) + (int64_t)n1p * n2 * q.i3 : nullptr,
                    SC ? (uint32_t)(n1p * n2) * 2 : 0u);
      // pair (2l, 2l + 1); the lone last entry of an odd row (2l = n1 - 1)
      // comes as the second half of the pair (2l - 1, 2l) (its scale as the
      // first half of the scale pair (2l, 2l + 1), the second a zero pad)
      const uint32_t vf = 2 * lane + 1 < n1 ? (uint32_t)(8 * lane) : 2 * lane + 1 == n1 ? (uint32_t)(8 * lane - 4) : kOOB;
      const uint32_t vs = 2 * lane < n1 ? (uint32_t)(4 * lane) : kOOB;
#pragma unroll
      for (int k = 0; k < KA; ++k) {
        const int r = wave + W * k;
        const int so = (r < n2 ? r : 0) * n1 * 4;
        const uint32_t of = r < n2 ? vf : kOOB;
        xa[k] = __builtin_bit_cast(u32x2, __builtin_amdgcn_raw_buffer_load_b64(rin, of, so, 0));
        if constexpr (SC)
          sa[k] = __builtin_amdgcn_raw_buffer_load_b32(rsc, r < n2 ? vs : kOOB, (r < n2 ? r : 0) * n1p * 2, 0);
      }
      if constexpr (TAILC) {
#pragma unroll
        for (int k = 0; k < KB; ++k) {
          const int r = 8 * (wave + W * k) + (lane >> 3), c = 128 + 2 * (lane & 7);
          const uint32_t o0 = r < n2 && c < n1 ? (uint32_t)((r * n1 + c) * 4) : kOOB;
          const uint32_t o1 = r < n2 && c + 1 < n1 ? (uint32_t)((r * n1 + c + 1) * 4) : kOOB;
          xb0[k] = __builtin_amdgcn_raw_buffer_load_b32(rin, o0, 0, 0);
          xb1[k] = __builtin_amdgcn_raw_buffer_load_b32(rin, o1, 0, 0);
          if constexpr (SC)
            sbp[k] = __builtin_amdgcn_raw_buffer_load_b32(
                rsc, r < n2 && c < n1 ? (uint32_t)((r * n1p + c) * 2) : kOOB, 0, 0);
        }
      }
    } else {
      const __amdgpu_buffer_rsrc_t rin = make_rsrc(
          reinterpret_cast<const S*>(u.in) + (2 * (int64_t)q.rhs * u.ld + slab_off16(A) + 2 * (int64_t)A * q.i3),
          (uint32_t)A * 2);
      const uint32_t v0 = 2 * lane < n1 ? (uint32_t)(4 * lane) : kOOB;
      const uint32_t v1 = 2 * lane + 1 < n1 ? (uint32_t)(4 * lane + 2) : kOOB;
      const int n1p = n1 + (n1 & 1);
      const __amdgpu_buffer_rsrc_t rsc =
          make_rsrc(SCL ? static_cast<const S*>(u.scale) + (int64_t)n1p * n2 * q.i3 : nullptr,
                    SCL ? (uint32_t)(n1p * n2) * 2 : 0u);
      const uint32_t vs = 2 * lane < n1 ? (uint32_t)(4 * lane) : kOOB;
#pragma unroll
      for (int k = 0; k < KA; ++k) {
        const int r = wave + W * k;
        const int so = (r < n2 ? r : 0) * n1 * 2;
        xa[k][0] = __builtin_amdgcn_raw_buffer_load_b16(rin, r < n2 ? v0 : kOOB, so, 0);
        xp[k] = __builtin_amdgcn_raw_buffer_load_b16(rin, r < n2 ? v1 : kOOB, so, 0);
        if constexpr (SCL)
          sa[k] = __builtin_amdgcn_raw_buffer_load_b32(rsc, r < n2 ? vs : kOOB, (r < n2 ? r : 0) * n1p * 2, 0);
      }
      if constexpr (TAILC) {
#pragma unroll
        for (int k = 0; k < KB; ++k) {
          const int r = 8 * (wave + W * k) + (lane >> 3), c = 128 + 2 * (lane & 7);
          const uint32_t o0 = r < n2 && c < n1 ? (uint32_t)((r * n1 + c) * 2) : kOOB;
          const uint32_t o1 = r < n2 && c + 1 < n1 ? (uint32_t)((r * n1 + c + 1) * 2) : kOOB;
          xb0[k] = __builtin_amdgcn_raw_buffer_load_b16(rin, o0, 0, 0);
          xb1[k] = __builtin_amdgcn_raw_buffer_load_b16(rin, o1, 0, 0);
        }
      }
    }
  };

  // Results of the previous slab: its stores are issued in the next
  // iteration, before the next prefetch, so that the prefetched data are
  // always the youngest memory operations when they are waited for (the
  // vector memory counter completes in order: a prefetch issued before a
  // slab's stores could only be waited for together with them).
  v4 zh[TB][TB];
  f4 zf[TB][TB];
  // SCB: D^{-1/2} at the entries of zf, loaded one slab ahead of its use (a
  // load right before the store that needs it would expose the memory
  // latency in every slab)
  constexpr bool SCB = !FWD && SC && !SCL;
  f4 zsc[SCB ? TB : 1][SCB ? TB : 1];
  // Z(j1, j2) of slab `tile`: lane group g's 16 lanes hold 16 consecutive
  // j1; every thread issues the same 4 TB^2 stores (invalid ones at an
  // out-of-range offset, dropped); offset = a per-lane vector part + a
  // uniform scalar part per tile and row
  auto store_z = [&](const SlabPos& ps, int lane) {
    const int g = lane >> 4, l16 = lane & 15;
    auto& u = slab_unit(args, ps.ui);
    const int n1 = u.n1, n2 = u.n2, A = n1 * n2;
    constexpr int EB = FWD ? 2 : 4;
    const uint32_t vlane = (uint32_t)(l16 + 4 * g * n1) * EB;  // j1 = .. + l16, j2 = .. + 4 g
    const int64_t plane = FWD ? 2 * (int64_t)ps.rhs * u.ld + slab_off16(A) + 2 * (int64_t)A * ps.i3
                              : (int64_t)ps.rhs * u.ld + (int64_t)A * ps.i3;
    const __amdgpu_buffer_rsrc_t rout = FWD ? make_rsrc(reinterpret_cast<S*>(u.out) + plane, (uint32_t)A * 2)
                                            : make_rsrc(reinterpret_cast<float*>(u.out) + plane, (uint32_t)A * 4);
#pragma unroll
    for (int t = 0; t < TB; ++t)
#pragma unroll
      for (int q = 0; q < TB; ++q) {
        const int j2t = 16 * (wa * TB + t), j1t = 16 * (wb * TB + q);
        // a tile wholly inside n1 x n2 stores without per-lane bounds
        const bool inner = wa * TB + t < MT && wb * TB + q < MT && j1t + 16 <= n1 && j2t + 16 <= n2;
        const bool okl = wa * TB + t < MT && wb * TB + q < MT && l16 + j1t < n1;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const uint32_t so = (uint32_t)(j1t + n1 * (j2t + r)) * EB;
          const uint32_t vo = inner || (okl && j2t + 4 * g + r < n2) ? vlane : kOOB;
          if constexpr (FWD) {
            bstore16(rout, vo, so, zh[t][q][r]);
          } else {
            float zr = zf[t][q][r];
            if constexpr (SCB) zr *= zsc[t][q][r];
            __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(uint32_t, zr), rout, vo, so, 0);
          }
        }
      }
  };
  // the scale entries store_z(ps) multiplies by (same offsets)
  auto load_scale = [&](const SlabPos& ps, int lane) {
    const int g = lane >> 4, l16 = lane & 15;
    auto& u = slab_unit(args, ps.ui);
    const int n1 = u.n1, n2 = u.n2, n1p = n1 + (n1 & 1);
    const uint32_t vlane = (uint32_t)(l16 + 4 * g * n1p) * 2;
    const __amdgpu_buffer_rsrc_t rsc =
        make_rsrc(static_cast<const S*>(u.scale) + (int64_t)n1p * n2 * ps.i3, (uint32_t)(n1p * n2) * 2);
#pragma unroll
    for (int t = 0; t < TB; ++t)
#pragma unroll
      for (int q = 0; q < TB; ++q) {
        const int j2t = 16 * (wa * TB + t), j1t = 16 * (wb * TB + q);
        const bool inner = wa * TB + t < MT && wb * TB + q < MT && j1t + 16 <= n1 && j2t + 16 <= n2;
        const bool okl = wa * TB + t < MT && wb * TB + q < MT && l16 + j1t < n1;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const uint32_t so = (uint32_t)(j1t + n1p * (j2t + r)) * 2;
          const uint32_t vo = inner || (okl && j2t + 4 * g + r < n2) ? vlane : kOOB;
          zsc[t][q][r] = (float)__builtin_bit_cast(S, (unsigned short)__builtin_amdgcn_raw_buffer_load_b16(rsc, vo, so, 0));
        }
      }
  };
  int t_begin = 0, t_end = 0, t_step = 1;
  slab_range(args, &t_begin, &t_end, &t_step);
  SlabPos nxt = slab_pos(args, t_begin, SlabPos{0, 0, 0, false});
  if (nxt.valid && t_begin < t_end) prefetch(nxt, tid0 & 63);
  int staged = -1;  // unit whose factors are in LDS
  SlabPos prevp{0, 0, 0, false};  // the slab whose results wait in zh / zf

  for (int tile = t_begin; tile < t_end; tile += t_step) {
    // (the thread index passes through an empty asm each slab so that the
    // offsets derived from it are recomputed here rather than hoisted out of
    // the loop and spilled)
    int tid = tid0;
    asm volatile("" : "+v"(tid));
    const int lane = tid & 63, g = lane >> 4, l16 = lane & 15;
    const SlabPos cur = nxt;
    auto& u = slab_unit(args, cur.ui);
    const int n1 = u.n1, n2 = u.n2;

    // ---- the previous slab is done with the LDS
    slab_barrier();
    if (cur.ui != staged) {
      // factors of a new unit: 16-byte chunks of the padded images (entries
      // past an image read 0); chunk index -> (row, block, chunk)
      staged = cur.ui;
      const __amdgpu_buffer_rsrc_t rf1 = make_rsrc(u.f1, (uint32_t)u.ldf1 * u.ldf1 * 2);
      const __amdgpu_buffer_rsrc_t rf2 = make_rsrc(u.f2, (uint32_t)u.ldf2 * u.ldf2 * 2);
      for (int c = tid; c < ROWS * 4 * KT; c += NT) {
        const int row = c / (4 * KT), col = 8 * (c - row * (4 * KT));
        const uint32_t o1 = row < u.ldf1 && col < u.ldf1 ? (uint32_t)(row * u.ldf1 + col) * 2 : kOOB;
        const uint32_t o2 = row < u.ldf2 && col < u.ldf2 ? (uint32_t)(row * u.ldf2 + col) * 2 : kOOB;
        const int at = slab_at<BS>(row, col);
        *reinterpret_cast<u32x4*>(fs1 + at) = __builtin_amdgcn_raw_buffer_load_b128(rf1, o1, 0, 0);
        *reinterpret_cast<u32x4*>(fs2 + at) = __builtin_amdgcn_raw_buffer_load_b128(rf2, o2, 0, 0);
      }
    }

    // ---- stage X: entry (i1, i2) at row i2, column i1, in 16 bits; every
    // LDS entry the products read is written for every slab (data, or zero
    // past n1 and n2), so no value of an earlier slab reaches this one
    {
      const float s_in = u.s_in;
      auto cvt2 = [&](fl2 x) -> uint32_t {
        if (P == 3 || SC) x *= s_in;  // (FP16 range scale; 1 for BF16)
        return __builtin_bit_cast(uint32_t, __builtin_convertvector(x, s2));
      };
      // rows >= n2 and columns >= n1 get the zeros their out-of-range loads
      // returned; lane l's pair sits in block l / 16, chunk (l / 4) % 4 of
      // the row (the row's swizzle is uniform: rows w + W k)
      const int lpart = (lane >> 4) * BS + wave * 64 + (((lane >> 2) & 3) << 4) + ((lane & 3) << 2);
      if (4 * lane < 64 * KT) {
#pragma unroll
        for (int k = 0; k < KA; ++k) {
          const int r = wave + W * k;
          if (W * (k + 1) <= ROWS || r < ROWS) {
            uint32_t v;
            if constexpr (FWD) {
              fl2 x = __builtin_bit_cast(fl2, xa[k]);
              if (2 * lane + 1 == n1) x = fl2{x[1], 0.0f};  // the lone last entry
              if constexpr (SC) x *= scale2(sa[k]);
              v = cvt2(x);
            } else {
              v = (xa[k][0] & 0xffffu) | (xp[k] << 16);
              if constexpr (SCL) {
                const int n1p = n1 + (n1 & 1);
                if (r < n2 && 2 * lane < n1p)
                  *reinterpret_cast<uint32_t*>(sci + 2 * (r * (n1p + 16) + 2 * lane)) = sa[k];
              }
            }
            *reinterpret_cast<uint32_t*>(xs + ((lpart ^ (rsw(r) << 4)) + W * 64 * k)) = v;
          }
        }
      }
      if constexpr (TAILC) {
#pragma unroll
        for (int k = 0; k < KB; ++k) {
          const int r = 8 * (wave + W * k) + (lane >> 3);
          if (r < ROWS) {
            uint32_t v;
            if constexpr (FWD) {
              fl2 x = {__builtin_bit_cast(float, xb0[k]), __builtin_bit_cast(float, xb1[k])};
              if constexpr (SC) x *= scale2(sbp[k]);
              v = cvt2(x);
            } else {
              v = (xb0[k] & 0xffffu) | (xb1[k] << 16);
            }
            *reinterpret_cast<uint32_t*>(xs + slab_at<BS>(r, 128 + 2 * (lane & 7))) = n1 > 128 ? v : 0u;
          }
        }
      }
      // columns [WC, 32 KT) of every row (whole 16-byte chunks)
      constexpr int CW = (32 * KT - WC) / 8;  // chunks per row past WC
      if constexpr (CW > 0) {
        for (int c = tid; c < ROWS * CW; c += NT) {
          const int r = c / CW;
          *reinterpret_cast<u32x4*>(xs + slab_at<BS>(r, WC + 8 * (c - r * CW))) = u32x4{0u, 0u, 0u, 0u};
        }
      }
    }
    // the previous slab's stores, then the next slab's input, stream while
    // this one computes
    if (prevp.valid) store_z(prevp, lane);
    nxt = slab_pos(args, tile + t_step, cur);
    if (nxt.valid && tile + t_step < t_end) prefetch(nxt, lane);
    if constexpr (SCB) load_scale(cur, lane);
    slab_barrier();

    // Fragment reads: row 16 T + l16 (T uniform), chunk g of block s; the
    // swizzle depends on l16 only. Tiles past MT (uniform) read tile MT - 1
    // and skip their MFMAs.
    const int fpart = l16 * 64 + ((g ^ rsw(l16)) << 4);
    auto tile_at = [&](int T) { return (T < MT ? T : MT - 1) * 1024 + fpart; };

    // ---- P1: Y^T tiles (i2 tile wa TB + t, j1 tile wb TB + q)
    f4 acc[TB][TB];
#pragma unroll
    for (int t = 0; t < TB; ++t)
#pragma unroll
      for (int q = 0; q < TB; ++q) acc[t][q] = f4{0.f, 0.f, 0.f, 0.f};
    const int kt1 = (n1 + 31) >> 5;
#pragma unroll
    for (int s = 0; s < KT; ++s) {
      if (s < kt1) {
        frag a[TB], b[TB];
#pragma unroll
        for (int t = 0; t < TB; ++t) a[t] = *reinterpret_cast<const frag*>(xs + s * BS + tile_at(wa * TB + t));
#pragma unroll
        for (int q = 0; q < TB; ++q) b[q] = *reinterpret_cast<const frag*>(fs1 + s * BS + tile_at(wb * TB + q));
#pragma unroll
        for (int t = 0; t < TB; ++t)
#pragma unroll
          for (int q = 0; q < TB; ++q)
            if (wa * TB + t < MT && wb * TB + q < MT) acc[t][q] = mma(a[t], b[q], acc[t][q]);
      }
    }
    slab_barrier();  // every read of X is done

    // ---- Y rows j1, columns i2 (4 consecutive i2 per lane and tile: half a
    // chunk)
    {
      const float s_mid = u.s_mid;
#pragma unroll
      for (int t = 0; t < TB; ++t)
#pragma unroll
        for (int q = 0; q < TB; ++q) {
          if (wa * TB + t < MT && wb * TB + q < MT) {
            const int i2 = 16 * (wa * TB + t) + 4 * g, j1 = 16 * (wb * TB + q) + l16;
            f4 y = acc[t][q];
            if constexpr (P == 3) y *= s_mid;  // (FP16 range scale)
            *reinterpret_cast<v4*>(xs + slab_at<BS>(j1, i2)) = __builtin_convertvector(y, v4);
          }
        }
    }
    slab_barrier();

    // ---- P2: Z^T tiles (A = F2 rows j2, tile wa TB + t; B = Y rows j1, tile
    // wb TB + q): a lane group's 16 lanes hold 16 consecutive j1
#pragma unroll
    for (int t = 0; t < TB; ++t)
#pragma unroll
      for (int q = 0; q < TB; ++q) acc[t][q] = f4{0.f, 0.f, 0.f, 0.f};
    const int kt2 = (n2 + 31) >> 5;
#pragma unroll
    for (int s = 0; s < KT; ++s) {
      if (s < kt2) {
        frag a[TB], b[TB];
#pragma unroll
        for (int t = 0; t < TB; ++t) a[t] = *reinterpret_cast<const frag*>(fs2 + s * BS + tile_at(wa * TB + t));
#pragma unroll
        for (int q = 0; q < TB; ++q) b[q] = *reinterpret_cast<const frag*>(xs + s * BS + tile_at(wb * TB + q));
#pragma unroll
        for (int t = 0; t < TB; ++t)
#pragma unroll
          for (int q = 0; q < TB; ++q)
            if (wa * TB + t < MT && wb * TB + q < MT) acc[t][q] = mma(a[t], b[q], acc[t][q]);
      }
    }

    // ---- keep Z for the next iteration's stores (scaled; FWD in 16 bits)
#pragma unroll
    for (int t = 0; t < TB; ++t)
#pragma unroll
      for (int q = 0; q < TB; ++q) {
        f4 z = acc[t][q];
        if constexpr (P == 3 || !FWD) z *= u.s_out;
        if constexpr (SCL) {
          // D^{-1/2} at (j1, j2) from the slab's LDS image (entries past
          // the slab read clamped positions: their results are not stored)
          const int SR = n1 + (n1 & 1) + 16;
          const int j1 = 16 * (wb * TB + q) + l16, j1c = j1 < SR ? j1 : SR - 1;
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const int j2 = 16 * (wa * TB + t) + 4 * g + r, j2c = j2 < ROWS ? j2 : ROWS - 1;
            z[r] *= (float)*reinterpret_cast<const S*>(sci + 2 * (j2c * SR + j1c));
          }
        }
        if constexpr (FWD) zh[t][q] = __builtin_convertvector(z, v4);
        else zf[t][q] = z;
      }
    prevp = cur;
  }
  if (prevp.valid) store_z(prevp, tid0 & 63);
}

template <int P, int MT, bool FWD, bool SC, class Src>
static hipError_t launch_slab_m(const Src& args, hipStream_t stream) {
  auto kern = fd_slab_kernel<P, MT, FWD, SC, Src>;
  const size_t smem = slab_lds_bytes(MT) + (slab_scale_lds(FWD, SC, MT) ? slab_sci_bytes(MT) : 0);
  // once per process (thread-safe initialisation of a function-local static)
  static const hipError_t attr = hipFuncSetAttribute(reinterpret_cast<const void*>(kern),
                                                     hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
  if (attr != hipSuccess) return attr;
  // workgroups resident on the device at once, per device (racing threads
  // compute the same value)
  static std::atomic<int> resident_of[kMaxDevices];
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  int resident = resident_of[dev].load(std::memory_order_relaxed);
  if (resident == 0) {
    int cus = 0, per_cu = 0;
    e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (e == hipSuccess)
      e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, reinterpret_cast<const void*>(kern),
                                                       64 * kSlabWaves, smem);
    if (e != hipSuccess) return e;
    resident = cus * (per_cu > 0 ? per_cu : 1);
    resident_of[dev].store(resident, std::memory_order_relaxed);
  }
  const int grid = args.total_tiles < resident ? args.total_tiles : resident;
  hipLaunchKernelGGL(kern, dim3(grid), dim3(64 * kSlabWaves), smem, stream, args);
  return hipGetLastError();
}

template <int P, int MT, class Src>
static hipError_t launch_slab_mt(const Src& args, bool fwd, bool sc, hipStream_t stream) {
  if (fwd)
    return sc ? launch_slab_m<P, MT, true, true>(args, stream) : launch_slab_m<P, MT, true, false>(args, stream);
  return sc ? launch_slab_m<P, MT, false, true>(args, stream) : launch_slab_m<P, MT, false, false>(args, stream);
}

template <int P, class Src, int... I>
static hipError_t launch_slab_sel(const Src& args, int mt, bool fwd, bool sc, hipStream_t stream,
                                  std::integer_sequence<int, I...>) {
  hipError_t res = hipErrorInvalidValue;
  (void)((mt == I + 1 ? (res = launch_slab_mt<P, I + 1>(args, fwd, sc, stream), true) : false) || ...);
  return res;
}

hipError_t launch_slab(const SlabArgs& args, int prec, int mt, hipStream_t stream) {
  if (args.total_tiles <= 0) return hipSuccess;
  // one direction and one scaling per launch (the host groups units so)
  const bool fwd = args.u[0].in16 == 0, sc = args.u[0].scale != nullptr;
  for (int k = 1; k < args.count; ++k)
    if ((args.u[k].in16 == 0) != fwd || (args.u[k].scale != nullptr) != sc) return hipErrorInvalidValue;
  using seq = std::make_integer_sequence<int, kSlabMaxMT>;
  if (prec == 2) return launch_slab_sel<2>(args, mt, fwd, sc, stream, seq{});
  if (prec == 3) return launch_slab_sel<3>(args, mt, fwd, sc, stream, seq{});
  return hipErrorInvalidValue;
}

hipError_t launch_slab_tab(const SlabTab& tab, int prec, int mt, bool fwd, bool sc, hipStream_t stream) {
  if (tab.total_tiles <= 0) return hipSuccess;
  if (tab.count < 1 || !tab.u) return hipErrorInvalidValue;
  using seq = std::make_integer_sequence<int, kSlabMaxMT>;
  if (prec == 2) return launch_slab_sel<2>(tab, mt, fwd, sc, stream, seq{});
  if (prec == 3) return launch_slab_sel<3>(tab, mt, fwd, sc, stream, seq{});
  return hipErrorInvalidValue;
}

}  // namespace fdk
