// C ABI of libfd (declared in include/fd.h): plan setup on the host in FP64,
// device upload of the packed factors, and the pass schedule of Algorithm 1.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <functional>
#include <map>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "../../include/fd.h"
#include "fd_host.h"
#include "fd_internal.h"

struct fd_plan_s {
  int ndim = 0;
  int n[3] = {1, 1, 1};
  int prec = 0;
  bool mass_only = false;
  int64_t N = 0;
  double w[3] = {1, 1, 1};
  std::vector<double> U[3], d[3];
  // device memory (one allocation)
  void* dev = nullptr;
  size_t dev_bytes = 0;
  const void* f_fwd[3] = {nullptr, nullptr, nullptr};  // packed U_i^T
  const void* f_bwd[3] = {nullptr, nullptr, nullptr};  // packed U_i
  const void* p_fwd[3] = {nullptr, nullptr, nullptr};  // plain row-major U_i^T
  const void* p_bwd[3] = {nullptr, nullptr, nullptr};  // plain row-major U_i
  const void* v_fwd[3] = {nullptr, nullptr, nullptr};  // padded U_i^T (pipelined kernels)
  const void* v_bwd[3] = {nullptr, nullptr, nullptr};  // padded U_i
  const void* v_snd[3] = {nullptr, nullptr, nullptr};  // padded U_i as second product of the fused pass
  const double* d_dev[3] = {nullptr, nullptr, nullptr};
  double lam_w[3] = {1, 1, 1};                          // weights used for Lambda on device
  float xs[5] = {1, 1, 1, 1, 1}, qs = 1.0f;             // FP16 / FP8 range scaling per stage
  float fs[3] = {1, 1, 1};                              // FP8: scale of the factor images per direction
  const void* scale_dev = nullptr;                      // D^{-1/2}, I/O type
  const void* scale16 = nullptr;                        // slab route: D^{-1/2} in 16 bits (SlabDesc::scale)
  int MT[3] = {0, 0, 0}, KS[3] = {0, 0, 0};
  int device = 0;
  int family_cap = 3;  // most capable kernel family the plan's passes may use
  // slab route (3D BF16/FP16, n1, n2 <= 144): stage 0 and 4 are slab passes
  // over both in-plane modes and the tensor stays in the 16-bit layout of z
  // until the last one; stages 1 and 3 are empty. xs_sb: FP16 scale of the
  // backward slab pass's intermediate (after the last and first modes).
  bool slab = false;
  float xs_sb = 1.0f;
  // banded route of a mass-only block (fd_setup_mass_banded): per direction
  // the band of the Cholesky factor of M_i on the device
  bool banded = false;
  int bw[3] = {0, 0, 0};
  const void* bfac[3] = {nullptr, nullptr, nullptr};
};

struct fd_batch_s {
  int device = 0;
  int prec = 0;
  std::vector<fd_work> works;
  // per body choice (kBodyWide, kBodyNarrow, kBodyPipelined: the passes that
  // have a pipelined body, the others wide) the passes of each stage as
  // descriptors and body segments (stage-local indices)
  struct Layout {
    std::vector<fdk::BatchDesc> desc[5];
    std::vector<fdk::BatchSeg> seg[5];
    std::vector<size_t> seg_smem[5];  // LDS bytes of each segment's body (segment route)
    int64_t tiles[5] = {0, 0, 0, 0, 0};
    bool differs[5] = {false, false, false, false, false};  // some pass of the stage runs another body than wide
  } lay[3];
  int width[5] = {0, 0, 0, 0, 0};  // body choice per stage
  int stage_seg[6] = {0, 0, 0, 0, 0, 0};
  int64_t max_tiles = 0;
  size_t smem = 0;
  int last_stage = -1;
  int phases = 0;         // barrier phases per launch
  void* dev = nullptr;    // descriptors and segments of the current widths
  size_t dev_cap = 0;
  void* ctl = nullptr;    // barrier counter and error flag
  // segment route (configuration bit kBatchSegments): every segment of the
  // uploaded tables as a launch of its own, in stage order; per uploaded
  // segment its LDS bytes and grid
  bool use_segments = false;
  std::vector<size_t> up_smem;
  std::vector<int> up_grid;
  uint32_t arrivals = 0;  // barrier arrivals counted so far
  int cus = 0;
  bool tuned = false;
  // Staged route (configuration word kBatchStaged; batches whose works are
  // all slab-route plans, 3D BF16/FP16): one launch per stage and row-tile
  // group instead of the persistent launch, the slab passes of stages 0 and
  // 4 and the 16-bit fused pass of stage 2 reading their units from device
  // tables, so the tensor crosses HBM three times in 16 bits between passes.
  struct StagedLaunch {
    int stage;        // 0, 2 or 4
    int mt;           // slab: row tiles of max(n1, n2); fused: of the last order
    bool sc;          // slab: the units scale by D^{-1/2}; fused: eigenvalue tables in LDS
    bool walk;        // fused: units one by one over contiguous tile ranges (else tiles strided)
    size_t off;       // byte offset of the units (SlabDesc or BatchDesc) in sdev
    int count;        // units
    int64_t tiles;
    size_t smem;      // fused: LDS bytes
    int max_n;
  };
  std::vector<StagedLaunch> staged;
  void* sdev = nullptr;
  size_t sdev_bytes = 0;
  bool use_staged = false;
};

namespace {

thread_local std::string g_err;

// Device bytes the library holds (plans, batch tables, setup temporaries)
// and the cap of fd_set_device_limit (0: none). An allocation that would pass
// the cap fails as on an exhausted device, before hipMalloc is called; the
// bytes are reserved before the call, so concurrent setups cannot pass the
// cap together.
std::atomic<size_t> g_dev_limit{0};
std::atomic<size_t> g_dev_held{0};

hipError_t dev_alloc(void** ptr, size_t bytes) {
  *ptr = nullptr;
  const size_t lim = g_dev_limit.load();
  size_t cur = g_dev_held.load();
  do {
    if (lim && (cur > lim || bytes > lim - cur)) return hipErrorOutOfMemory;
  } while (!g_dev_held.compare_exchange_weak(cur, cur + bytes));
  hipError_t e = hipMalloc(ptr, bytes);
  if (e != hipSuccess) {
    *ptr = nullptr;
    g_dev_held.fetch_sub(bytes);
  }
  return e;
}

hipError_t dev_free(void* ptr, size_t bytes) {
  if (!ptr) return hipSuccess;
  const hipError_t e = hipFree(ptr);
  g_dev_held.fetch_sub(bytes);
  return e;
}

struct StageRecord {
  int stage;
  hipEvent_t start, end;
};
struct LaunchRecord {
  int stage, family, n, prec;
  hipEvent_t start, end;
};
bool g_timing = false;
std::vector<StageRecord> g_records;
std::vector<LaunchRecord> g_launch_records;
std::vector<fd_launch_time> g_launch_stats;  // filled by fd_timing_read

fd_status fail(fd_status s, const std::string& msg) {
  g_err = msg;
  return s;
}

fd_status hip_fail(hipError_t e, const char* what) {
  return fail(FD_E_HIP, std::string(what) + ": " + hipGetErrorString(e));
}

bool io_is_f64(int prec) { return prec == FD_F64; }

// ---- pass schedule
// 3D: stage 0 mode-1 forward (pre-scale), 1 mode-2 forward, 2 mode-3 forward
//     + Lambda^{-1} + mode-3 backward, 3 mode-2 backward, 4 mode-1 backward
//     (post-scale).
// 2D: stage 0 mode-1 forward, 2 mode-2 fused, 4 mode-1 backward.
constexpr int kStages = 5;

// `slab_route`: false for callers that run every plan on the five-stage
// schedule (the persistent batch).
bool unit_pass(const fd_plan_s* p, const fd_work& wk, int stage, fdk::PassDesc& u, bool slab_route = true) {
  std::memset(&u, 0, sizeof(u));
  if (p->banded) return false;  // runs the banded solves instead (band_pass)
  const bool slab = slab_route && p->slab;
  if (slab && stage != 2) return false;  // slab passes (slab_pass)
  const int n1 = p->n[0], n2 = p->n[1], n3 = p->n[2];
  u.in = wk.z;
  u.out = wk.z;
  u.ld = wk.ld;
  u.nrhs = wk.nrhs;
  u.scale = p->scale_dev;
  int dir = -1;
  bool fwd = false, fused = false;
  if (p->ndim == 3) {
    switch (stage) {
      case 0: dir = 0; u.A = 1; u.n = n1; u.B = n2 * n3; u.in = wk.r; fwd = true;
              if (p->scale_dev) u.flags |= fdk::kPreScale; break;
      case 1: dir = 1; u.A = n1; u.n = n2; u.B = n3; fwd = true; break;
      case 2: dir = 2; u.A = n1 * n2; u.n = n3; u.B = 1; fused = true; break;
      case 3: dir = 1; u.A = n1; u.n = n2; u.B = n3; break;
      case 4: dir = 0; u.A = 1; u.n = n1; u.B = n2 * n3;
              if (p->scale_dev) u.flags |= fdk::kPostScale; break;
    }
  } else {
    switch (stage) {
      case 0: dir = 0; u.A = 1; u.n = n1; u.B = n2; u.in = wk.r; fwd = true;
              if (p->scale_dev) u.flags |= fdk::kPreScale; break;
      case 2: dir = 1; u.A = n1; u.n = n2; u.B = 1; fused = true; break;
      case 4: dir = 0; u.A = 1; u.n = n1; u.B = n2;
              if (p->scale_dev) u.flags |= fdk::kPostScale; break;
      default: return false;
    }
  }
  if (fused) {
    u.flags |= fdk::kFuseLambda;
    u.f1 = p->f_fwd[dir];
    u.f2 = p->f_bwd[dir];
    u.pf1 = p->p_fwd[dir];
    u.pf2 = p->p_bwd[dir];
    u.pv1 = p->v_fwd[dir];
    u.pv2 = p->v_snd[dir];
  } else {
    u.f1 = fwd ? p->f_fwd[dir] : p->f_bwd[dir];
    u.pf1 = fwd ? p->p_fwd[dir] : p->p_bwd[dir];
    u.pv1 = fwd ? p->v_fwd[dir] : p->v_bwd[dir];
  }
  u.xscale = p->xs[stage];
  u.qscale = fused ? p->qs : 1.0f;
  // (FP8: the factor images carry fs per product)
  u.oscale = 1.0f / (u.xscale * u.qscale * p->fs[dir] * (fused ? p->fs[dir] : 1.0f));
  u.MT = p->MT[dir];
  u.KS = p->KS[dir];
  u.lam_ndim = p->ndim;
  u.n1 = n1;
  u.sA = u.A;
  for (int i = 0; i < 3; ++i) {
    u.d[i] = p->d_dev[i];
    u.w[i] = p->lam_w[i];
  }
  if (slab) {
    // fused last-mode pass on the 16-bit layout: z viewed as 16-bit entries
    // from the plane offset, residuals 2 ld apart, planes 2 A apart; its FP16
    // input is already scaled, its output carries the backward slab pass's
    // input scale
    const int64_t A = int64_t(n1) * n2;
    u.in = static_cast<const char*>(wk.z) + 2 * fdk::slab_off16(A);
    u.out = static_cast<char*>(wk.z) + 2 * fdk::slab_off16(A);
    u.ld = 2 * wk.ld;
    u.sA = int32_t(2 * A);
    u.xscale = 1.0f;
    u.oscale = p->xs[3] / (p->xs[2] * p->qs);
  }
  return true;
}

// Effective precision class of the pass of `p` in `stage`: the fused pass of a
// slab-route plan reads and writes 16-bit data (classes 7 and 8).
int unit_class(const fd_plan_s* p, int stage) {
  if (p->slab && stage == 2) return p->prec == FD_BF16 ? 7 : 8;
  return p->prec;
}

// Slab pass of a slab-route plan: stage 0 reads r (FP32, pre-scaled by
// D^{-1/2} if the plan has one) and writes the 16-bit layout of z; stage 4
// reads that layout and writes FP32 z (post-scaled).
bool slab_pass(const fd_plan_s* p, const fd_work& wk, int stage, fdk::SlabDesc& d) {
  if (!p->slab || wk.nrhs == 0 || (stage != 0 && stage != 4)) return false;
  std::memset(&d, 0, sizeof(d));
  const bool fwd = stage == 0;
  d.in = fwd ? wk.r : wk.z;
  d.out = wk.z;
  d.f1 = fwd ? p->v_fwd[0] : p->v_bwd[0];
  d.f2 = fwd ? p->v_fwd[1] : p->v_bwd[1];
  d.scale = p->scale16;
  d.post = fwd ? 0 : 1;
  d.ld = wk.ld;
  d.n1 = p->n[0];
  d.n2 = p->n[1];
  d.n3 = p->n[2];
  d.nrhs = wk.nrhs;
  d.ldf1 = fdk::v3_ld(p->n[0], p->prec);
  d.ldf2 = fdk::v3_ld(p->n[1], p->prec);
  d.in16 = fwd ? 0 : 1;
  d.out16 = fwd ? 1 : 0;
  if (fwd) {
    d.s_in = p->xs[0];
    d.s_mid = p->xs[1] / p->xs[0];
    d.s_out = p->xs[2] / p->xs[1];
  } else {
    d.s_in = 1.0f;
    d.s_mid = p->xs_sb / p->xs[3];
    d.s_out = 1.0f / p->xs_sb;
  }
  return true;
}

int slab_mt(const fd_plan_s* p) { return std::max(p->MT[0], p->MT[1]); }

int stage_mode(const fdk::PassDesc& u) {
  if (u.flags & fdk::kFuseLambda) return 2;
  return u.A == 1 ? 0 : 1;
}

// Mode `stage` of the banded route (stages 0..ndim-1: mode 1 reads r and
// writes z, the later modes run in place on z).
bool band_pass(const fd_plan_s* p, const fd_work& wk, int stage, fdk::BandArgs& a) {
  if (!p->banded || stage >= p->ndim || wk.nrhs == 0) return false;
  std::memset(&a, 0, sizeof(a));
  fdk::BandDesc& u = a.u;
  int A = 1, B = 1;
  for (int i = 0; i < stage; ++i) A *= p->n[i];
  for (int i = stage + 1; i < p->ndim; ++i) B *= p->n[i];
  u.in = stage == 0 ? wk.r : wk.z;
  u.out = wk.z;
  u.fac = p->bfac[stage];
  u.ld = wk.ld;
  u.A = A;
  u.n = p->n[stage];
  u.B = B;
  u.nrhs = wk.nrhs;
  u.bw = p->bw[stage];
  u.tiles_per_rhs = fdk::band_tiles_per_rhs(int64_t(A) * B);
  return true;
}

fd_status validate_work(const fd_work& wk) {
  if (!wk.plan) return fail(FD_E_ARG, "fd_apply: NULL plan");
  if (wk.nrhs < 0) return fail(FD_E_ARG, "fd_apply: nrhs < 0");
  if (wk.nrhs == 0) return FD_OK;
  if (!wk.r || !wk.z) return fail(FD_E_ARG, "fd_apply: NULL vector pointer");
  if (wk.ld < wk.plan->N) return fail(FD_E_ARG, "fd_apply: ld smaller than the plan size");
  const size_t eb = io_is_f64(wk.plan->prec) ? 8 : 4;
  const char* r0 = static_cast<const char*>(wk.r);
  const char* z0 = static_cast<const char*>(wk.z);
  const size_t span = (size_t(wk.nrhs - 1) * size_t(wk.ld) + size_t(wk.plan->N)) * eb;
  if (r0 != z0 && r0 < z0 + span && z0 < r0 + span)
    return fail(FD_E_ARG, "fd_apply: r and z overlap without being equal");
  return FD_OK;
}

fd_status run_work(int count, const fd_work* work, hipStream_t stream) {
  // the most capable kernel family every plan of the call allows (the
  // default picks the most capable family a unit fits)
  int kernel_family = 3;
  for (int i = 0; i < count; ++i)
    if (work[i].plan) kernel_family = std::min(kernel_family, work[i].plan->family_cap);
  for (int i = 0; i < count; ++i) {
    fd_status s = validate_work(work[i]);
    if (s != FD_OK) return s;
  }
  const bool f64 = count > 0 && io_is_f64(work[0].plan->prec);
  for (int i = 0; i < count; ++i)
    if (io_is_f64(work[i].plan->prec) != f64)
      return fail(FD_E_ARG, "fd_apply_batched: FP64 and FP32-I/O plans in one call");
  for (int stage = 0; stage < kStages; ++stage) {
    StageRecord rec{stage, nullptr, nullptr};
    if (g_timing) {
      bool any = false;
      for (int i = 0; i < count; ++i) {
        fdk::PassDesc probe;
        fdk::BandArgs bprobe;
        fdk::SlabDesc sprobe;
        if (work[i].nrhs > 0 && (unit_pass(work[i].plan, work[i], stage, probe) ||
                                 band_pass(work[i].plan, work[i], stage, bprobe) ||
                                 slab_pass(work[i].plan, work[i], stage, sprobe)))
          any = true;
      }
      if (any) {
        hipError_t e = hipEventCreate(&rec.start);
        if (e == hipSuccess) e = hipEventCreate(&rec.end);
        if (e == hipSuccess) e = hipEventRecord(rec.start, stream);
        if (e != hipSuccess) return hip_fail(e, "timing event");
      }
    }
    for (int prec = 0; prec <= 8; ++prec) {
      // units of this stage and precision class
      std::vector<fdk::PassDesc> units, split_fwd, split_bwd;
      int mode = -1;
      for (int i = 0; i < count; ++i) {
        const fd_work& wk = work[i];
        if (wk.nrhs == 0 || unit_class(wk.plan, stage) != prec) continue;
        fdk::PassDesc u;
        if (!unit_pass(wk.plan, wk, stage, u)) continue;
        mode = stage_mode(u);
        // FP64 last-mode passes beyond the fused pipelined kernel (n > 144)
        // but within the single-pass one run as two pipelined passes: the
        // forward product with Lambda^{-1} applied before its store (mode 3),
        // then the backward product in place (mode 1)
        int c3 = 0;
        size_t s3 = 0;
        if (kernel_family >= 3 && prec == FD_F64 && mode == 2 && !fdk::v3_plan(prec, 2, u.n, u.MT, &c3, &s3) &&
            fdk::v3_plan(prec, 3, u.n, u.MT, &c3, &s3) && fdk::v3_plan(prec, 1, u.n, u.MT, &c3, &s3)) {
          split_fwd.push_back(u);
          fdk::PassDesc v = u;
          v.in = u.out;
          v.flags &= ~fdk::kFuseLambda;
          v.pv1 = wk.plan->v_bwd[wk.plan->ndim - 1];
          split_bwd.push_back(v);
          continue;
        }
        units.push_back(u);
      }
      auto run_units = [&](std::vector<fdk::PassDesc>& units, int mode) -> fd_status {
        // Kernel families: 3 = pipelined LDS GEMM (FP64/FP32), 2 = factor resident
        // in LDS, 1 = factor fragments from global memory. Family 3 launches
        // group units of one factor order n, family 2 units of one row-tile
        // count; family 1 takes the rest in one launch.
        std::vector<int> group(units.size(), -1);  // family * 1000 + n or row tiles
        for (size_t k = 0; k < units.size(); ++k) {
          int b = 0, c = 0;
          size_t sm = 0;
          const bool pre = (units[k].flags & fdk::kPreScale) != 0;
          // the pipelined family (FP64/FP32) loads raw input straight into LDS
          // and stores raw accumulators, so passes that scale their input or
          // output run on family 2
          const bool post = (units[k].flags & fdk::kPostScale) != 0;
          if (kernel_family >= 3 && !pre && !post && fdk::v3_plan(prec, mode, units[k].n, units[k].MT, &c, &sm))
            group[k] = 3000 + units[k].n;
          else if (prec >= 7)  // (16-bit data has the pipelined body only)
            return fail(FD_E_HIP, "internal: no kernel for a 16-bit data pass");
          else if (kernel_family >= 2 && fdk::v2_plan(prec, mode, units[k].n, units[k].MT, &b, &c, &sm))
            group[k] = 2000 + b;
          else
            group[k] = 1000;
        }
        std::vector<int> keys(group.begin(), group.end());
        std::sort(keys.begin(), keys.end());
        keys.erase(std::unique(keys.begin(), keys.end()), keys.end());
        for (int key : keys) {
          const int fam = key / 1000;
          int max_n = 0, max_mt = 1;
          for (size_t k = 0; k < units.size(); ++k)
            if (group[k] == key) {
              max_n = std::max(max_n, units[k].n);
              max_mt = std::max(max_mt, units[k].MT);
            }
          int bucket = 0, chunk = fdk::kTileP;
          size_t smem = 0;
          bool ok = true;
          if (fam == 3) ok = fdk::v3_plan(prec, mode, max_n, max_mt, &chunk, &smem);
          if (fam == 2) ok = fdk::v2_plan(prec, mode, max_n, max_mt, &bucket, &chunk, &smem);
          if (!ok) return fail(FD_E_HIP, "internal: kernel plan changed");
          fdk::PassArgs args;
          args.lam_lds = 0;
          args.count = 0;
          args.total_tiles = 0;
          int launch_mt = 1;
          auto flush = [&]() -> fd_status {
            if (args.count == 0) return FD_OK;
            LaunchRecord lr{stage, fam, max_n, prec, nullptr, nullptr};
            if (g_timing) {
              hipError_t e = hipEventCreate(&lr.start);
              if (e == hipSuccess) e = hipEventCreate(&lr.end);
              if (e == hipSuccess) e = hipEventRecord(lr.start, stream);
              if (e != hipSuccess) return hip_fail(e, "timing event");
            }
            hipError_t e = fam == 3 ? fdk::launch_pass3(args, prec, mode, max_mt, smem, stream)
                         : fam == 2 ? fdk::launch_pass2(args, prec, mode, bucket, smem, stream)
                                    : fdk::launch_pass(args, prec, launch_mt, stream);
            if (g_timing && e == hipSuccess) {
              e = hipEventRecord(lr.end, stream);
              if (e == hipSuccess) g_launch_records.push_back(lr);
            }
            args.count = 0;
            args.total_tiles = 0;
            launch_mt = 1;
            if (e != hipSuccess) return hip_fail(e, "kernel launch");
            return FD_OK;
          };
          for (size_t k = 0; k < units.size(); ++k) {
            if (group[k] != key) continue;
            fdk::PassDesc u = units[k];
            const int64_t NQ = int64_t(u.A) * u.B;
            u.tiles_per_rhs = int32_t((NQ + chunk - 1) / chunk);
            const int64_t tiles = int64_t(u.tiles_per_rhs) * u.nrhs;
            if (tiles > 0x7fffffffLL) return fail(FD_E_ARG, "fd_apply: too many tiles in one call");
            if (args.count == fdk::kMaxDesc || int64_t(args.total_tiles) + tiles > 0x7fffffffLL) {
              fd_status s = flush();
              if (s != FD_OK) return s;
            }
            u.tile_begin = args.total_tiles;
            args.u[args.count++] = u;
            args.total_tiles += int32_t(tiles);
            launch_mt = std::max(launch_mt, u.MT);
          }
          fd_status s = flush();
          if (s != FD_OK) return s;
        }
        return FD_OK;
      };
      if (!units.empty()) {
        fd_status s = run_units(units, mode);
        if (s != FD_OK) return s;
      }
      if (!split_fwd.empty()) {
        fd_status s = run_units(split_fwd, 3);
        if (s == FD_OK) s = run_units(split_bwd, 1);
        if (s != FD_OK) return s;
      }
    }
    // banded route of mass-only blocks: one launch per work and mode
    for (int i = 0; i < count; ++i) {
      fdk::BandArgs ba;
      if (!band_pass(work[i].plan, work[i], stage, ba)) continue;
      LaunchRecord lr{stage, 4, ba.u.n, work[i].plan->prec, nullptr, nullptr};
      if (g_timing) {
        hipError_t e = hipEventCreate(&lr.start);
        if (e == hipSuccess) e = hipEventCreate(&lr.end);
        if (e == hipSuccess) e = hipEventRecord(lr.start, stream);
        if (e != hipSuccess) return hip_fail(e, "timing event");
      }
      if (int64_t(ba.u.tiles_per_rhs) * ba.u.nrhs > 0x7fffffffLL)
        return fail(FD_E_ARG, "fd_apply: too many tiles in one call");
      hipError_t e = fdk::launch_band(ba, io_is_f64(work[i].plan->prec), stream);
      if (e != hipSuccess) return hip_fail(e, "banded kernel launch");
      if (g_timing) {
        e = hipEventRecord(lr.end, stream);
        if (e != hipSuccess) return hip_fail(e, "timing event");
        g_launch_records.push_back(lr);
      }
    }
    // slab passes: one launch per precision, row-tile count and scaling, up
    // to kMaxDesc works each
    for (int prec = 2; prec <= 3; ++prec)
      for (int mt = 1; mt <= fdk::kSlabMaxMT; ++mt)
        for (int sc = 0; sc <= 1; ++sc) {
        fdk::SlabArgs sa;
        sa.count = 0;
        sa.total_tiles = 0;
        int max_n = 0;
        auto flush = [&]() -> fd_status {
          if (sa.count == 0) return FD_OK;
          LaunchRecord lr{stage, 5, max_n, prec, nullptr, nullptr};
          if (g_timing) {
            hipError_t e = hipEventCreate(&lr.start);
            if (e == hipSuccess) e = hipEventCreate(&lr.end);
            if (e == hipSuccess) e = hipEventRecord(lr.start, stream);
            if (e != hipSuccess) return hip_fail(e, "timing event");
          }
          hipError_t e = fdk::launch_slab(sa, prec, mt, stream);
          if (e != hipSuccess) return hip_fail(e, "slab kernel launch");
          if (g_timing) {
            e = hipEventRecord(lr.end, stream);
            if (e != hipSuccess) return hip_fail(e, "timing event");
            g_launch_records.push_back(lr);
          }
          sa.count = 0;
          sa.total_tiles = 0;
          max_n = 0;
          return FD_OK;
        };
        for (int i = 0; i < count; ++i) {
          const fd_plan_s* p = work[i].plan;
          fdk::SlabDesc d;
          if (p->prec != prec || slab_mt(p) != mt || (p->scale_dev != nullptr) != (sc == 1) ||
              !slab_pass(p, work[i], stage, d))
            continue;
          const int64_t tiles = int64_t(d.n3) * d.nrhs;
          if (tiles > 0x7fffffffLL) return fail(FD_E_ARG, "fd_apply: too many tiles in one call");
          if (sa.count == fdk::kMaxDesc || int64_t(sa.total_tiles) + tiles > 0x7fffffffLL) {
            fd_status s = flush();
            if (s != FD_OK) return s;
          }
          d.tile_begin = sa.total_tiles;
          sa.u[sa.count++] = d;
          sa.total_tiles += int32_t(tiles);
          max_n = std::max(max_n, std::max(d.n1, d.n2));
        }
        fd_status s = flush();
        if (s != FD_OK) return s;
      }
    if (rec.start) {
      hipError_t e = hipEventRecord(rec.end, stream);
      if (e != hipSuccess) return hip_fail(e, "timing event");
      g_records.push_back(rec);
    }
  }
  return FD_OK;
}

// ---------------------------------------------------------------- persistent batch

// Descriptor of the pass of `wk` in `stage` with body choice `choice`
// (kBodyWide, kBodyNarrow, kBodyPipelined; passes without a pipelined body
// run wide), its body and the LDS bytes it needs; false if the work has no
// pass in that stage.
static bool batch_pass(int prec, const fd_work& wk, int stage, int choice, int* body, fdk::BatchDesc* out,
                       size_t* smem) {
  fdk::PassDesc u;
  if (wk.nrhs == 0 || !unit_pass(wk.plan, wk, stage, u, false)) return false;
  fdk::BatchDesc bd{};
  bd.u = u;
  bd.mode = stage_mode(u);
  bd.scale = (u.flags & fdk::kPreScale) ? 1 : (u.flags & fdk::kPostScale) ? 2 : 0;
  int b = choice == fdk::kBodyNarrow ? fdk::kBodyNarrow : fdk::kBodyWide;
  int chunk = 0, mt3 = 0;
  size_t sm3 = 0;
  // the pipelined body loads raw input straight into LDS and stores raw
  // accumulators: passes that scale either run an LDS-resident body
  if (choice == fdk::kBodyPipelined && bd.scale == 0 && u.pv1 &&
      fdk::batch_plan3(prec, bd.mode, u.MT, &mt3, &chunk, &sm3)) {
    b = fdk::kBodyPipelined;
    bd.mt = mt3;
    *smem = sm3;
  } else {
    bd.mt = fdk::batch_mt(prec, u.MT);
    chunk = fdk::batch_chunk(prec, bd.mode, u.MT, b == fdk::kBodyNarrow);
    *smem = fdk::batch_lds_bytes(prec, u.n, bd.mode == 2);
  }
  const int64_t NQ = int64_t(u.A) * u.B;
  bd.u.tiles_per_rhs = int32_t((NQ + chunk - 1) / chunk);
  *body = b;
  *out = bd;
  return true;
}

// Order of the passes inside a stage (segments of equal keys): largest
// row-tile count first, then body, mode and scaling.
static std::tuple<int, int, int, int> batch_key(int body, const fdk::BatchDesc& bd) {
  return std::make_tuple(-bd.mt, body, bd.mode, bd.scale);
}

static fd_status batch_build_layout(fd_batch_s* b, int choice) {
  auto& L = b->lay[choice];
  for (int stage = 0; stage < kStages; ++stage) {
    auto& D = L.desc[stage];
    auto& S = L.seg[stage];
    D.clear();
    S.clear();
    L.differs[stage] = false;
    // passes of this stage, grouped by body (kind, mode, row tiles, scaling)
    std::vector<std::pair<int, fdk::BatchDesc>> passes;  // (body, descriptor)
    std::vector<size_t> pass_smem;
    for (const fd_work& wk : b->works) {
      int body = 0;
      fdk::BatchDesc bd;
      size_t sm = 0;
      if (!batch_pass(b->prec, wk, stage, choice, &body, &bd, &sm)) continue;
      b->smem = std::max(b->smem, sm);
      if (body != fdk::kBodyWide) L.differs[stage] = true;
      passes.emplace_back(body, bd);
      pass_smem.push_back(sm);
    }
    // segments of a stage run one after another on every workgroup: the
    // largest row-tile counts first, so that the tiles left when workgroups
    // reach the stage's barrier are the cheapest ones
    auto key = [](const std::pair<int, fdk::BatchDesc>& x) { return batch_key(x.first, x.second); };
    std::vector<size_t> order(passes.size());
    for (size_t i = 0; i < order.size(); ++i) order[i] = i;
    std::stable_sort(order.begin(), order.end(), [&](size_t x, size_t y) { return key(passes[x]) < key(passes[y]); });
    {
      std::vector<std::pair<int, fdk::BatchDesc>> sorted;
      std::vector<size_t> sorted_smem;
      for (size_t i : order) {
        sorted.push_back(passes[i]);
        sorted_smem.push_back(pass_smem[i]);
      }
      passes.swap(sorted);
      pass_smem.swap(sorted_smem);
    }
    L.seg_smem[stage].clear();
    int64_t t = 0;
    for (size_t i = 0; i < passes.size(); ++i) {
      fdk::BatchDesc bd = passes[i].second;
      if (i == 0 || key(passes[i - 1]) != key(passes[i])) {
        L.seg_smem[stage].push_back(0);
        fdk::BatchSeg sg{};
        sg.d0 = int(D.size());
        sg.t0 = int(t);
        sg.mode = bd.mode;
        sg.mt = bd.mt;
        sg.scale = bd.scale;
        sg.body = passes[i].first;
        S.push_back(sg);
      }
      bd.u.tile_begin = t;
      t += int64_t(bd.u.tiles_per_rhs) * bd.u.nrhs;
      if (t > 0x7fffffffLL) return fail(FD_E_ARG, "fd_batch_create: too many tiles in one stage");
      L.seg_smem[stage].back() = std::max(L.seg_smem[stage].back(), pass_smem[i]);
      D.push_back(bd);
      S.back().d1 = int(D.size());
      S.back().t1 = int(t);
    }
    L.tiles[stage] = t;
  }
  return FD_OK;
}

// Uploads the descriptors and segments of the chosen body of every stage.
static fd_status batch_upload(fd_batch_s* b) {
  std::vector<fdk::BatchDesc> desc;
  std::vector<fdk::BatchSeg> seg;
  b->max_tiles = 0;
  b->up_smem.clear();
  b->up_grid.clear();
  for (int st = 0; st < kStages; ++st) {
    const auto& L = b->lay[b->width[st]];
    b->stage_seg[st] = int(seg.size());
    const int base = int(desc.size());
    for (size_t k = 0; k < L.seg[st].size(); ++k) {
      fdk::BatchSeg sg = L.seg[st][k];
      sg.d0 += base;
      sg.d1 += base;
      seg.push_back(sg);
      // the segment route's launch: its own LDS, as many workgroups as fit
      const size_t sm = L.seg_smem[st][k];
      int per_cu = 0;
      hipError_t e = fdk::batch_seg_resident(b->prec, sm, &per_cu);
      if (e != hipSuccess) return hip_fail(e, "batch occupancy");
      b->up_smem.push_back(sm);
      b->up_grid.push_back(int(std::min<int64_t>(int64_t(b->cus) * std::max(per_cu, 1), sg.t1 - sg.t0)));
    }
    desc.insert(desc.end(), L.desc[st].begin(), L.desc[st].end());
    b->max_tiles = std::max(b->max_tiles, L.tiles[st]);
  }
  b->stage_seg[kStages] = int(seg.size());
  const size_t db = desc.size() * sizeof(fdk::BatchDesc), sb = seg.size() * sizeof(fdk::BatchSeg);
  if (db + sb > b->dev_cap) {
    (void)dev_free(b->dev, b->dev_cap);
    b->dev = nullptr;
    b->dev_cap = 0;
    hipError_t e = dev_alloc(&b->dev, db + sb + 256);
    if (e != hipSuccess) return e == hipErrorOutOfMemory ? fail(FD_E_NOMEM, "fd_batch") : hip_fail(e, "hipMalloc");
    b->dev_cap = db + sb + 256;
  }
  // the device may still run an apply that reads the old tables
  hipError_t e = hipDeviceSynchronize();
  if (e == hipSuccess) e = hipMemcpy(b->dev, desc.data(), db, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(static_cast<unsigned char*>(b->dev) + db, seg.data(), sb, hipMemcpyHostToDevice);
  if (e != hipSuccess) return hip_fail(e, "hipMemcpy");
  return FD_OK;
}

static fd_status batch_launch_staged(fd_batch_s* b, hipStream_t stream);

static fd_status batch_launch(fd_batch_s* b, hipStream_t stream) {
  if (b->use_staged) return batch_launch_staged(b, stream);
  if (b->max_tiles == 0) return FD_OK;
  if (b->use_segments) {
    fdk::BatchArgs a{};
    size_t nd = 0;
    for (int st = 0; st < kStages; ++st) nd += b->lay[b->width[st]].desc[st].size();
    unsigned char* base = static_cast<unsigned char*>(b->dev);
    a.desc = reinterpret_cast<const fdk::BatchDesc*>(base);
    a.seg = reinterpret_cast<const fdk::BatchSeg*>(base + nd * sizeof(fdk::BatchDesc));
    for (int k = 0; k < b->stage_seg[kStages]; ++k) {
      hipError_t e = fdk::batch_seg_launch(a, b->prec, k, b->up_grid[size_t(k)], b->up_smem[size_t(k)], stream);
      if (e != hipSuccess) return hip_fail(e, "batch segment launch");
    }
    return FD_OK;
  }
  // one 8-wavefront workgroup per CU: the pass bodies are called functions
  // with a stack, and the scratch the runtime grants is sized for that
  const int64_t grid = std::min<int64_t>(b->cus, b->max_tiles);
  uint32_t* bar = static_cast<uint32_t*>(b->ctl);
  int32_t* err = reinterpret_cast<int32_t*>(static_cast<unsigned char*>(b->ctl) + 128);
  // the arrival counter only grows: restart it before it could wrap
  if (uint64_t(b->arrivals) + uint64_t(b->phases) * uint64_t(grid) >= 0x80000000ull) {
    hipError_t e = fdk::batch_reset(bar, err, stream);
    if (e != hipSuccess) return hip_fail(e, "batch reset");
    b->arrivals = 0;
  }
  fdk::BatchArgs a{};
  size_t nd = 0;
  for (int st = 0; st < kStages; ++st) nd += b->lay[b->width[st]].desc[st].size();
  unsigned char* base = static_cast<unsigned char*>(b->dev);
  a.desc = reinterpret_cast<const fdk::BatchDesc*>(base);
  a.seg = reinterpret_cast<const fdk::BatchSeg*>(base + nd * sizeof(fdk::BatchDesc));
  a.barrier = bar;
  a.error = err;
  a.base = b->arrivals;
  for (int i = 0; i <= kStages; ++i) a.stage_seg[i] = b->stage_seg[i];
  a.last_stage = b->last_stage;
  hipError_t e = fdk::batch_launch(a, b->prec, int(grid), b->smem, stream);
  if (e != hipSuccess) return hip_fail(e, "batch kernel launch");
  b->arrivals += uint32_t(b->phases) * uint32_t(grid);  // every workgroup passes each barrier once
  return FD_OK;
}

// Works a persistent batch accepts: valid works of one precision class with
// every factor order <= 128, FP8 split excluded.
static fd_status batch_validate(int32_t count, const fd_work* work, const char* who) {
  for (int i = 0; i < count; ++i) {
    fd_status s = validate_work(work[i]);
    if (s != FD_OK) return s;
    for (int d = 0; d < work[i].plan->ndim; ++d)
      if (work[i].plan->n[d] > 16 * fdk::kBatchMaxMT)
        return fail(FD_E_UNSUPPORTED, std::string(who) + ": factor order above 128 (use fd_apply_batched)");
    if (work[i].plan->prec != work[0].plan->prec)
      return fail(FD_E_UNSUPPORTED, std::string(who) + ": plans of different precision classes");
    if (work[i].plan->banded)
      return fail(FD_E_UNSUPPORTED, std::string(who) + ": banded mass plans run through fd_apply_batched only");
  }
  if (count > 0 && work[0].plan->prec == FD_FP8_SPLIT)
    return fail(FD_E_UNSUPPORTED, std::string(who) + ": no persistent-batch body for FD_FP8_SPLIT");
  return FD_OK;
}

// Configuration words beyond the ten bits of the body choices: the staged
// route, and the segment route (with the body choices of its segments).
constexpr int kBatchStaged = 1 << 10;
constexpr int kBatchSegments = 1 << 11;

// two bits per stage: the body choice of stage s in bits 2s, 2s + 1
static int batch_config(const fd_batch_s* b) {
  if (b->use_staged) return kBatchStaged;
  int c = 0;
  for (int st = 0; st < kStages; ++st) c |= b->width[st] << (2 * st);
  return c | (b->use_segments ? kBatchSegments : 0);
}

// Lays out and uploads the staged route when every work with residuals is a
// slab-route plan; otherwise leaves it empty (not available).
static fd_status batch_build_staged(fd_batch_s* b) {
  b->staged.clear();
  if (b->prec != FD_BF16 && b->prec != FD_F16) return FD_OK;
  bool any = false;
  for (const fd_work& wk : b->works) {
    if (wk.nrhs == 0) continue;
    if (!wk.plan->slab) return FD_OK;
    any = true;
  }
  if (!any) return FD_OK;
  const int cls = b->prec == FD_BF16 ? 7 : 8;
  std::vector<unsigned char> image;
  auto put = [&](const void* src, size_t bytes) {
    const size_t off = (image.size() + 255) & ~size_t(255);
    image.resize(off + bytes);
    std::memcpy(image.data() + off, src, bytes);
    return off;
  };
  for (int stage = 0; stage < kStages; stage += 2) {
    if (stage == 2) {
      // fused passes grouped by the (even) row-tile count of the last order
      std::map<int, std::vector<fdk::BatchDesc>, std::greater<int>> groups;
      std::map<int, std::pair<size_t, int>> plan_of;  // group -> (LDS bytes, largest order)
      std::map<int, size_t> lam_of;                     // group -> largest eigenvalue table
      for (const fd_work& wk : b->works) {
        fdk::PassDesc u;
        if (wk.nrhs == 0 || !unit_pass(wk.plan, wk, 2, u)) continue;
        int chunk = 0;
        size_t sm = 0;
        const int mt = (u.MT + 1) / 2 * 2;
        if (!fdk::v3_plan(cls, 2, u.n, mt, &chunk, &sm)) return fail(FD_E_HIP, "internal: no 16-bit fused pass");
        u.tiles_per_rhs = int32_t((int64_t(u.A) * u.B + chunk - 1) / chunk);
        fdk::BatchDesc bd{};
        bd.u = u;
        bd.mode = 2;
        bd.mt = mt;
        bd.scale = 0;
        groups[mt].push_back(bd);
        auto& pl = plan_of[mt];
        pl.first = sm;
        pl.second = std::max(pl.second, u.n);
        auto& tb = lam_of[mt];  // the unit's weighted eigenvalues in LDS (FP32)
        tb = std::max(tb, sizeof(float) * size_t(u.n1 + u.A / u.n1 + u.n));
      }
      for (auto& [mt, D] : groups) {
        int64_t t = 0;
        for (auto& bd : D) {
          bd.u.tile_begin = t;
          t += int64_t(bd.u.tiles_per_rhs) * bd.u.nrhs;
        }
        if (t > 0x7fffffffLL) return fail(FD_E_ARG, "fd_batch_create: too many tiles in one launch");
        // the eigenvalue tables sit after the ring when they fit the LDS
        const bool lam = plan_of[mt].first + lam_of[mt] <= 160 * 1024;
        fd_batch_s::StagedLaunch L{2, mt, lam, lam, put(D.data(), D.size() * sizeof(fdk::BatchDesc)),
                                   int(D.size()), t, plan_of[mt].first + (lam ? lam_of[mt] : 0), plan_of[mt].second};
        b->staged.push_back(L);
      }
    } else {
      // slab passes grouped by row-tile count and scaling
      std::map<std::pair<int, int>, std::vector<fdk::SlabDesc>, std::greater<std::pair<int, int>>> groups;
      for (const fd_work& wk : b->works) {
        fdk::SlabDesc d;
        if (!slab_pass(wk.plan, wk, stage, d)) continue;
        groups[{slab_mt(wk.plan), d.scale ? 1 : 0}].push_back(d);
      }
      for (auto& [key, D] : groups) {
        int64_t t = 0;
        int max_n = 0;
        for (auto& d : D) {
          d.tile_begin = t;
          t += int64_t(d.n3) * d.nrhs;
          max_n = std::max(max_n, std::max(d.n1, d.n2));
        }
        if (t > 0x7fffffffLL) return fail(FD_E_ARG, "fd_batch_create: too many tiles in one launch");
        fd_batch_s::StagedLaunch L{stage, key.first, key.second == 1, false,
                                   put(D.data(), D.size() * sizeof(fdk::SlabDesc)), int(D.size()), t, 0, max_n};
        b->staged.push_back(L);
      }
    }
  }
  hipError_t e = dev_alloc(&b->sdev, image.size());
  if (e == hipSuccess) b->sdev_bytes = image.size();
  if (e != hipSuccess) {
    b->sdev = nullptr;
    b->staged.clear();
    return e == hipErrorOutOfMemory ? fail(FD_E_NOMEM, "fd_batch") : hip_fail(e, "hipMalloc");
  }
  e = hipMemcpy(b->sdev, image.data(), image.size(), hipMemcpyHostToDevice);
  if (e != hipSuccess) return hip_fail(e, "hipMemcpy");
  return FD_OK;
}

static hipError_t staged_launch_one(fd_batch_s* b, const fd_batch_s::StagedLaunch& L, hipStream_t stream) {
  const int cls = b->prec == FD_BF16 ? 7 : 8;
  const unsigned char* base = static_cast<const unsigned char*>(b->sdev) + L.off;
  if (L.stage == 2) {
    fdk::BatchSeg sg{};
    sg.d0 = 0;
    sg.d1 = L.count;
    sg.t0 = 0;
    sg.t1 = int(L.tiles);
    sg.mode = 2;
    sg.mt = L.mt;
    sg.scale = L.sc ? 1 : 0;  // (fused launches: the eigenvalue tables go to LDS)
    sg.body = L.walk ? 1 : 0;
    return fdk::launch_seg3(reinterpret_cast<const fdk::BatchDesc*>(base), sg, cls, L.mt, L.smem, stream);
  }
  fdk::SlabTab t{reinterpret_cast<const fdk::SlabDesc*>(base), L.count, int(L.tiles)};
  return fdk::launch_slab_tab(t, b->prec, L.mt, L.stage == 0, L.sc, stream);
}

// The staged route: its launches in stage order on `stream`. (Launching the
// independent launches of a stage on forked streams gained nothing: each
// launch fills the device.)
static fd_status batch_launch_staged(fd_batch_s* b, hipStream_t stream) {
  const int cls = b->prec == FD_BF16 ? 7 : 8;
  StageRecord rec{-1, nullptr, nullptr};
  auto close_stage = [&]() -> fd_status {
    if (!rec.start) return FD_OK;
    hipError_t e = hipEventRecord(rec.end, stream);
    if (e != hipSuccess) return hip_fail(e, "timing event");
    g_records.push_back(rec);
    rec = StageRecord{-1, nullptr, nullptr};
    return FD_OK;
  };
  for (const auto& L : b->staged) {
    if (g_timing && L.stage != rec.stage) {
      fd_status s = close_stage();
      if (s != FD_OK) return s;
      rec.stage = L.stage;
      hipError_t e = hipEventCreate(&rec.start);
      if (e == hipSuccess) e = hipEventCreate(&rec.end);
      if (e == hipSuccess) e = hipEventRecord(rec.start, stream);
      if (e != hipSuccess) return hip_fail(e, "timing event");
    }
    LaunchRecord lr{L.stage, L.stage == 2 ? 3 : 5, L.max_n, L.stage == 2 ? cls : b->prec, nullptr, nullptr};
    if (g_timing) {
      hipError_t e = hipEventCreate(&lr.start);
      if (e == hipSuccess) e = hipEventCreate(&lr.end);
      if (e == hipSuccess) e = hipEventRecord(lr.start, stream);
      if (e != hipSuccess) return hip_fail(e, "timing event");
    }
    hipError_t e = staged_launch_one(b, L, stream);
    if (e != hipSuccess) return hip_fail(e, "staged batch launch");
    if (g_timing) {
      e = hipEventRecord(lr.end, stream);
      if (e != hipSuccess) return hip_fail(e, "timing event");
      g_launch_records.push_back(lr);
    }
  }
  return close_stage();
}

// ---------------------------------------------------------------- allocation-free persistent apply
//
// fd_apply_persistent_static runs a list of works as one persistent launch,
// like fd_batch_apply, without allocating: the barrier counter, the error
// flag and the pass tables live in the file-scope device array `scratch`
// (one copy per GPU, kStaticBytes, held until the process ends). Host code
// never passes `scratch` itself: the per-device address from
// hipGetSymbolAddress is kept in g_static[device].ptr and used everywhere.

constexpr size_t kStaticBytes = size_t(2) << 20;  // tables + control words per device
constexpr size_t kStaticCtl = 256;                // barrier counter at 0, error flag at 128
constexpr int kStaticMaxDesc = int((kStaticBytes - kStaticCtl) / sizeof(fdk::BatchDesc));
constexpr int kStaticMaxDevices = 64;

struct StaticDevice {
  unsigned char* ptr = nullptr;  // device address of `scratch` on this device
  int cus = 0;
};
StaticDevice g_static[kStaticMaxDevices];
std::mutex g_static_mu;  // the host staging below is shared by all callers

// host staging of one call: passes of a stage before ordering, their order,
// then the uploaded image (descriptors followed by segments)
fdk::BatchDesc g_cand[kStaticMaxDesc];
int g_cand_body[kStaticMaxDesc];
int g_ord[kStaticMaxDesc];
fdk::BatchSeg g_seg[kStaticMaxDesc];
alignas(256) unsigned char g_image[kStaticBytes - kStaticCtl];

}  // namespace

static __device__ __align__(256) unsigned char scratch[kStaticBytes];

namespace {

// Per-device set-up (with that device current): the address of this
// device's copy of `scratch`, and its CU count.
fd_status static_device(int dev, StaticDevice** out) {
  if (dev < 0 || dev >= kStaticMaxDevices) return fail(FD_E_UNSUPPORTED, "fd_apply_persistent_static: device index");
  StaticDevice& sd = g_static[dev];
  if (!sd.ptr) {
    void* p = nullptr;
    hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress(scratch)");
    int cus = 0;
    e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (e != hipSuccess) return hip_fail(e, "hipDeviceGetAttribute");
    sd.cus = cus;
    sd.ptr = static_cast<unsigned char*>(p);
  }
  *out = &sd;
  return FD_OK;
}

}  // namespace

extern "C" {

const char* fd_last_error(void) { return g_err.c_str(); }

fd_status fd_timing_enable(int32_t enable) {
  g_timing = enable != 0;
  return FD_OK;
}

fd_status fd_timing_read(double* ms, int32_t* count) {
  if (!ms || !count) return fail(FD_E_ARG, "fd_timing_read: NULL output");
  for (int s = 0; s < kStages; ++s) {
    ms[s] = 0.0;
    count[s] = 0;
  }
  fd_status st = FD_OK;
  for (auto& r : g_records) {
    float t = 0.0f;
    hipError_t e = hipEventSynchronize(r.end);
    if (e == hipSuccess) e = hipEventElapsedTime(&t, r.start, r.end);
    if (e != hipSuccess && st == FD_OK) st = hip_fail(e, "fd_timing_read");
    ms[r.stage] += t;
    count[r.stage] += 1;
    (void)hipEventDestroy(r.start);
    (void)hipEventDestroy(r.end);
  }
  g_records.clear();
  g_launch_stats.clear();
  for (auto& r : g_launch_records) {
    float t = 0.0f;
    hipError_t e = hipEventSynchronize(r.end);
    if (e == hipSuccess) e = hipEventElapsedTime(&t, r.start, r.end);
    if (e != hipSuccess && st == FD_OK) st = hip_fail(e, "fd_timing_read");
    fd_launch_time* slot = nullptr;
    for (auto& c : g_launch_stats)
      if (c.stage == r.stage && c.family == r.family && c.n == r.n && c.prec == r.prec) slot = &c;
    if (!slot) {
      g_launch_stats.push_back(fd_launch_time{r.stage, r.family, r.n, r.prec, 0.0, 0});
      slot = &g_launch_stats.back();
    }
    slot->ms += t;
    slot->count += 1;
    (void)hipEventDestroy(r.start);
    (void)hipEventDestroy(r.end);
  }
  g_launch_records.clear();
  return st;
}

fd_status fd_timing_launches(int32_t capacity, fd_launch_time* out, int32_t* n_out) {
  if (!n_out || (capacity > 0 && !out)) return fail(FD_E_ARG, "fd_timing_launches: NULL output");
  *n_out = int32_t(g_launch_stats.size());
  for (int32_t i = 0; i < capacity && i < *n_out; ++i) out[i] = g_launch_stats[size_t(i)];
  return FD_OK;
}

fd_status fd_assemble_1d(int32_t n_el, int32_t degree, int32_t regularity, int32_t dirichlet,
                         int32_t npts, const double* tau_q, const double* mu_q, int32_t* n_out,
                         double* K, double* M) {
  if (!n_out) return fail(FD_E_ARG, "fd_assemble_1d: NULL n_out");
  int m = 0;
  if (fdh::assemble_1d(n_el, degree, regularity, dirichlet, npts, tau_q, mu_q, &m, K, M) != 0)
    return fail(FD_E_ARG, "fd_assemble_1d: invalid n_el/degree/regularity/npts");
  *n_out = m;
  return FD_OK;
}

fd_status fd_nitsche_stiffness_1d(int32_t n_el, int32_t degree, int32_t regularity, double c_pen, int32_t* n_out,
                                  double* K) {
  if (!n_out) return fail(FD_E_ARG, "fd_nitsche_stiffness_1d: NULL n_out");
  int m = 0;
  if (fdh::nitsche_stiffness_1d(n_el, degree, regularity, c_pen, &m, K) != 0)
    return fail(FD_E_ARG, "fd_nitsche_stiffness_1d: invalid n_el/degree/regularity or c_pen < 0");
  *n_out = m;
  return FD_OK;
}

fd_status fd_mixed_1d(int32_t n_el, int32_t deg_a, int32_t reg_a, int32_t da, int32_t deg_b, int32_t reg_b,
                      int32_t db, int32_t npts, int32_t* ma, int32_t* mb, double* X) {
  if (!ma || !mb) return fail(FD_E_ARG, "fd_mixed_1d: NULL size outputs");
  int a = 0, b = 0;
  if (npts <= 0) npts = std::max(deg_a, deg_b) + 2;
  if (fdh::mixed_1d(n_el, deg_a, reg_a, da, deg_b, reg_b, db, npts, &a, &b, X) != 0)
    return fail(FD_E_ARG, "fd_mixed_1d: invalid spaces, derivative orders or npts");
  *ma = a;
  *mb = b;
  return FD_OK;
}

fd_status fd_quadrature_1d(int32_t n_el, int32_t npts, double* x, double* w) {
  if (n_el < 1 || npts < 1 || npts > 16 || !x || !w) return fail(FD_E_ARG, "fd_quadrature_1d: bad arguments");
  fdh::element_quadrature(n_el, npts, x, w);
  return FD_OK;
}

fd_status fd_geometry_coefficients(int32_t ndim, int64_t npts, const double* jac, const double* nu,
                                   int32_t component, double* C, double* q_weight) {
  const int rc = fdh::geometry_coefficients(ndim, npts, jac, nu, component, C, q_weight);
  if (rc == 1) return fail(FD_E_ARG, "fd_geometry_coefficients: bad arguments");
  if (rc == 2) return fail(FD_E_ARG, "fd_geometry_coefficients: singular Jacobian or nu <= 0");
  return FD_OK;
}

fd_status fd_separable_factors(int32_t ndim, const int32_t* nq, const double* c, int64_t stride,
                               int32_t sweeps, double tol, double* tau, double* mu) {
  const int rc = fdh::separable_factors(ndim, nq, c, stride, sweeps, tol, tau, mu);
  if (rc == 1) return fail(FD_E_ARG, "fd_separable_factors: bad arguments");
  if (rc == 2) return fail(FD_E_ARG, "fd_separable_factors: coefficient entry <= 0");
  return FD_OK;
}

fd_status fd_operator_diagonal(int32_t ndim, const int32_t* n_el, int32_t degree, int32_t regularity,
                               int32_t dirichlet, int32_t npts, int32_t order, const double* coef,
                               double* diag) {
  if (fdh::operator_diagonal(ndim, n_el, degree, regularity, dirichlet, npts, order, coef, diag))
    return fail(FD_E_ARG, "fd_operator_diagonal: bad arguments");
  return FD_OK;
}

fd_status fd_factor_1d(int32_t n, const double* K, const double* M, double* U, double* d) {
  const char* why = "";
  const int rc = fdh::factor_1d(n, K, M, U, d, &why);
  if (rc == 1) return fail(FD_E_ARG, std::string("fd_factor_1d: ") + why);
  if (rc == 2) return fail(FD_E_NOTSPD, std::string("fd_factor_1d: ") + why);
  return FD_OK;
}

fd_status fd_setup(int32_t ndim, const int32_t* n, const double* const* K, const double* const* M,
                   const double* w, const double* diag_target, fd_precision prec, fd_plan* out) {
  if (!out) return fail(FD_E_ARG, "fd_setup: NULL out");
  *out = nullptr;
  if (ndim != 2 && ndim != 3) return fail(FD_E_ARG, "fd_setup: ndim must be 2 or 3");
  if (!n || !M) return fail(FD_E_ARG, "fd_setup: NULL n or M");
  if (int(prec) < 0 || int(prec) > 6) return fail(FD_E_ARG, "fd_setup: unknown precision");
  if (prec == FD_FP8_SPLIT) {
    // only the pipelined kernels have an FP8 body: no input/output scaling,
    // every order within their row tiles
    if (diag_target) return fail(FD_E_UNSUPPORTED, "fd_setup: FD_FP8_SPLIT plans take no diag_target");
    for (int i = 0; i < ndim && n; ++i)
      if (n[i] > 16 * fdk::v2_max_mt_of(FD_FP8_SPLIT))
        return fail(FD_E_UNSUPPORTED, "fd_setup: FD_FP8_SPLIT needs every n[i] <= 224");
  }
  auto p = new (std::nothrow) fd_plan_s();
  if (!p) return fail(FD_E_NOMEM, "fd_setup: host allocation");
  p->ndim = ndim;
  p->prec = int(prec);
  p->mass_only = (K == nullptr);
  // FD_KERNEL=v1 / v2 at setup caps the kernel family of the plan's passes
  // (diagnostics and tests of the fallback kernels)
  if (const char* kenv = std::getenv("FD_KERNEL")) {
    if (std::strcmp(kenv, "v1") == 0) p->family_cap = 1;
    else if (std::strcmp(kenv, "v2") == 0) p->family_cap = 2;
  }
  p->N = 1;
  for (int i = 0; i < ndim; ++i) {
    if (n[i] < 2 || n[i] > fdk::kMaxN) {
      delete p;
      return fail(FD_E_ARG, "fd_setup: each n[i] must be in [2, 256]");
    }
    if (!M[i] || (K && !K[i])) {
      delete p;
      return fail(FD_E_ARG, "fd_setup: NULL factor matrix");
    }
    p->n[i] = n[i];
    p->N *= n[i];
    p->w[i] = w ? w[i] : 1.0;
    if (!(p->w[i] > 0.0)) {
      delete p;
      return fail(FD_E_ARG, "fd_setup: weights must be > 0");
    }
  }
  // Buffer offsets inside one vector are 32-bit byte offsets with an
  // always-out-of-range value at 2^31: N * 8 bytes must stay below it.
  if (p->N >= (int64_t(1) << 28)) {
    delete p;
    return fail(FD_E_ARG, "fd_setup: prod(n) must be below 2^28");
  }
  // Step 1 of Algorithm 1 in FP64 on the host.
  for (int i = 0; i < ndim; ++i) {
    p->U[i].resize(size_t(n[i]) * n[i]);
    p->d[i].resize(n[i]);
    const char* why = "";
    const int rc = fdh::factor_1d(n[i], K ? K[i] : nullptr, M[i], p->U[i].data(), p->d[i].data(), &why);
    if (rc != 0) {
      delete p;
      return fail(rc == 2 ? FD_E_NOTSPD : FD_E_ARG, std::string("fd_setup: direction ") +
                                                         std::to_string(i + 1) + ": " + why);
    }
  }
  // Lambda must be positive: its smallest entry is sum_i w_i min(d_i).
  std::vector<double> dl[3];
  if (p->mass_only) {
    for (int i = 0; i < ndim; ++i) {
      dl[i].assign(n[i], i == 0 ? 1.0 : 0.0);
      p->lam_w[i] = 1.0;
    }
  } else {
    double lmin = 0.0;
    for (int i = 0; i < ndim; ++i) {
      lmin += p->w[i] * p->d[i][0];
      dl[i] = p->d[i];
      p->lam_w[i] = p->w[i];
    }
    if (!(lmin > 0.0)) {
      delete p;
      return fail(FD_E_NOTSPD, "fd_setup: the Kronecker-sum eigenvalues are not all positive");
    }
  }
  // Coefficient-aware scaling (Sec. 6): D = target / diag(P), scale = D^{-1/2}.
  std::vector<double> scale;
  if (diag_target) {
    scale.resize(p->N);
    const int n1 = p->n[0], n2 = p->n[1], n3 = ndim == 3 ? p->n[2] : 1;
    for (int64_t idx = 0; idx < p->N; ++idx) {
      const int i1 = int(idx % n1), i2 = int((idx / n1) % n2), i3 = int(idx / (int64_t(n1) * n2));
      const int ii[3] = {i1, i2, i3};
      double diagP = 0.0;
      if (p->mass_only) {
        diagP = 1.0;
        for (int k = 0; k < ndim; ++k) diagP *= M[k][ii[k] + size_t(p->n[k]) * ii[k]];
      } else {
        for (int k = 0; k < ndim; ++k) {
          double t = p->w[k] * K[k][ii[k] + size_t(p->n[k]) * ii[k]];
          for (int l = 0; l < ndim; ++l)
            if (l != k) t *= M[l][ii[l] + size_t(p->n[l]) * ii[l]];
          diagP += t;
        }
      }
      const double D = diag_target[idx] / diagP;
      if (!(D > 0.0) || !std::isfinite(D)) {
        delete p;
        return fail(FD_E_NOTSPD, "fd_setup: diag_target / diag(P) must be positive and finite");
      }
      scale[idx] = 1.0 / std::sqrt(D);
    }
    (void)n3;
  }
  // FP16 range (largest finite 65504): each pass converts its FP32 input to
  // FP16, so the input of every pass is scaled by a power of two that brings
  // its expected RMS to 1, and the result is scaled back (exact). The model
  // takes white residual entries of RMS r0 (the RMS of D^{-1/2} when scaled):
  // a product along mode i by U_i^T or U_i keeps the entries' variances in
  // product form, entry k scaled by c_i[k_i] = ||column k_i of U_i||^2, and
  // the division by Lambda divides entry k by Lambda(k)^2. So the mean square
  // after the forward products along modes 0..j is prod_{i<=j} mean(c_i), and
  // after the division and backward products along modes in `back` it is the
  // mean over k of prod_i c_i[k_i] prod_{i in back} c_i[k_i] / Lambda(k)^2,
  // estimated on 4096 fixed multi-indices.
  // FP8 (largest finite 448): the same model with the RMS of every converted
  // tensor placed at 4, and each factor image scaled by the power of two that
  // puts its largest entry in [112, 224); the output scale undoes both.
  const bool fp8 = p->prec == FD_FP8_SPLIT;
  if (fp8) {
    for (int i = 0; i < ndim; ++i) {
      double mx = 0.0;
      for (double v : p->U[i]) mx = std::max(mx, std::fabs(v));
      p->fs[i] = mx > 0 ? float(std::ldexp(1.0, int(std::floor(std::log2(224.0 / mx))))) : 1.0f;
    }
  }
  if (p->prec == FD_F16 || p->prec == FD_F16_SPLIT || fp8) {
    std::vector<double> cn[3];  // squared column norms of U_i
    double gain[3] = {1, 1, 1};
    for (int i = 0; i < ndim; ++i) {
      cn[i].assign(n[i], 0.0);
      for (int k = 0; k < n[i]; ++k)
        for (int m = 0; m < n[i]; ++m) cn[i][k] += p->U[i][m + size_t(n[i]) * k] * p->U[i][m + size_t(n[i]) * k];
      double f = 0.0;
      for (double v : cn[i]) f += v;
      gain[i] = std::sqrt(f / n[i]);
    }
    double r0 = 1.0;
    if (diag_target) {
      double ss = 0.0;
      for (double v : scale) ss += v * v;
      r0 = std::sqrt(ss / double(p->N));
    }
    const int last = ndim - 1;
    // mean squares after the division (sq[0]) and after the backward products
    // along modes last, last-1 (sq[1], sq[2])
    double sq[3] = {0.0, 0.0, 0.0}, sq_sb = 0.0;
    {
      uint64_t st = 0x9E3779B97F4A7C15ull;
      for (int t = 0; t < 4096; ++t) {
        double lam = 0.0, w = 1.0;
        int k[3] = {0, 0, 0};
        for (int i = 0; i < ndim; ++i) {
          st = st * 6364136223846793005ull + 1442695040888963407ull;
          k[i] = int((st >> 33) % uint64_t(n[i]));
          lam += p->lam_w[i] * dl[i][k[i]];
          w *= cn[i][k[i]];
        }
        if (p->mass_only) lam = 1.0;
        const double v = w / (lam * lam);
        sq[0] += v;
        sq[1] += v * cn[last][k[last]];
        if (ndim == 3) sq[2] += v * cn[last][k[last]] * cn[1][k[1]];
        // slab route: the backward slab pass's intermediate follows the
        // products along the last and the first mode
        if (ndim == 3) sq_sb += v * cn[last][k[last]] * cn[0][k[0]];
      }
      for (double& v : sq) v /= 4096.0;
      sq_sb /= 4096.0;
    }
    const double target = fp8 ? 4.0 : 1.0;
    auto pow2 = [target](double rms) {
      return float(std::ldexp(1.0, -int(std::lround(std::log2(rms / target)))));
    };
    double in = r0;
    for (int i = 0; i < last; ++i) {  // forward passes before the fused one
      p->xs[i] = pow2(in);
      in *= gain[i];
    }
    const int fused_stage = 2;  // 3D: stages 0, 1 then 2; 2D: stage 0 then 2
    p->xs[fused_stage] = pow2(in);
    // the fused pass converts acc / Lambda, where acc carries its input scale
    // and the factor image scale
    p->qs = pow2(r0 * std::sqrt(sq[0]) * p->xs[fused_stage] * p->fs[last]);
    if (ndim == 3) {
      p->xs[3] = pow2(r0 * std::sqrt(sq[1]));
      p->xs[4] = pow2(r0 * std::sqrt(sq[2]));
      p->xs_sb = pow2(r0 * std::sqrt(sq_sb));
    } else {
      p->xs[4] = pow2(r0 * std::sqrt(sq[1]));
      p->xs[0] = pow2(r0);
    }
  }
  // Slab route of 3D BF16/FP16 plans (in-plane orders within the slab kernel,
  // the last order within the 16-bit fused pass); FD_SLAB=0 at setup keeps
  // the five-stage schedule (diagnostics, tests of both routes)
  if (ndim == 3 && (p->prec == FD_BF16 || p->prec == FD_F16) && p->family_cap >= 3 &&
      n[0] <= 16 * fdk::kSlabMaxMT && n[1] <= 16 * fdk::kSlabMaxMT) {
    int c3 = 0;
    size_t s3 = 0;
    const char* senv = std::getenv("FD_SLAB");
    p->slab = !(senv && std::strcmp(senv, "0") == 0) &&
              fdk::v3_plan(p->prec == FD_BF16 ? 7 : 8, 2, n[2], (n[2] + 15) / 16, &c3, &s3);
  }
  // Pack U_i^T (forward) and U_i (backward) in fragment order.
  const int ks = fdk::mfma_kstep(p->prec);
  size_t off[3][2], offp[3][2], offv[3][3], offd[3], offs = 0, total = 0;
  auto align = [](size_t x) { return (x + 255) & ~size_t(255); };
  for (int i = 0; i < ndim; ++i) {
    p->MT[i] = (n[i] + 15) / 16;
    p->KS[i] = (n[i] + ks - 1) / ks;
    const size_t pb = fdk::packed_bytes(n[i], p->prec);
    off[i][0] = total; total = align(total + pb);
    off[i][1] = total; total = align(total + pb);
    const size_t qb = fdk::plain_bytes(n[i], p->prec);
    offp[i][0] = total; total = align(total + qb);
    offp[i][1] = total; total = align(total + qb);
    const size_t vb = fdk::v3_factor_bytes(n[i], p->prec);
    for (int j = 0; j < 3; ++j) { offv[i][j] = total; total = align(total + vb); }
    offd[i] = total; total = align(total + sizeof(double) * n[i]);
  }
  const size_t eb = io_is_f64(p->prec) ? 8 : 4;
  if (diag_target) { offs = total; total = align(total + eb * size_t(p->N)); }
  // slab route: D^{-1/2} once more in the plan's 16-bit type, rows padded to
  // an even length, so that the slab passes read it in aligned pairs
  size_t offs16 = 0;
  const int64_t n1p = n[0] + (n[0] & 1);
  if (diag_target && p->slab) {
    offs16 = total;
    total = align(total + 2 * size_t(n1p) * n[1] * n[2]);
  }
  std::vector<unsigned char> host(total, 0);
  std::vector<double> Ft;
  std::vector<float> stage8[3];
  for (int i = 0; i < ndim; ++i) {
    const int m = n[i];
    Ft.assign(size_t(m) * m, 0.0);
    for (int r = 0; r < m; ++r)
      for (int c = 0; c < m; ++c) Ft[r + size_t(m) * c] = p->U[i][c + size_t(m) * r];
    if (fp8) {
      // FP32 images (scaled), converted to FP8 hi/lo on the device below
      const size_t e = size_t(fdk::v3_ld(m, p->prec)) * fdk::v3_ld(m, p->prec);
      stage8[i].assign(3 * e, 0.0f);
      fdk::v3_factor_f32(m, Ft.data(), false, p->fs[i], stage8[i].data());
      fdk::v3_factor_f32(m, p->U[i].data(), false, p->fs[i], stage8[i].data() + e);
      fdk::v3_factor_f32(m, p->U[i].data(), true, p->fs[i], stage8[i].data() + 2 * e);
      std::memcpy(host.data() + offd[i], dl[i].data(), sizeof(double) * m);
      continue;
    }
    fdk::pack_factor(m, Ft.data(), p->prec, host.data() + off[i][0]);
    fdk::pack_factor(m, p->U[i].data(), p->prec, host.data() + off[i][1]);
    fdk::plain_factor(m, Ft.data(), p->prec, host.data() + offp[i][0]);
    fdk::plain_factor(m, p->U[i].data(), p->prec, host.data() + offp[i][1]);
    if (fdk::v3_factor_bytes(m, p->prec)) {
      fdk::v3_factor(m, Ft.data(), p->prec, false, host.data() + offv[i][0]);
      fdk::v3_factor(m, p->U[i].data(), p->prec, false, host.data() + offv[i][1]);
      fdk::v3_factor(m, p->U[i].data(), p->prec, true, host.data() + offv[i][2]);
    }
    std::memcpy(host.data() + offd[i], dl[i].data(), sizeof(double) * m);
  }
  if (diag_target) {
    if (eb == 8) std::memcpy(host.data() + offs, scale.data(), 8 * size_t(p->N));
    else
      for (int64_t k = 0; k < p->N; ++k) reinterpret_cast<float*>(host.data() + offs)[k] = float(scale[k]);
  }
  if (diag_target && p->slab) {
    uint16_t* s16 = reinterpret_cast<uint16_t*>(host.data() + offs16);
    for (int64_t k = 0; k < int64_t(n[1]) * n[2]; ++k)
      for (int i1 = 0; i1 < n[0]; ++i1) {
        const float v = float(scale[k * n[0] + i1]);
        uint16_t h;
        if (p->prec == FD_BF16) {
          uint32_t b;
          std::memcpy(&b, &v, 4);
          h = uint16_t((b + 0x7fffu + ((b >> 16) & 1u)) >> 16);  // round to nearest even
        } else {
          const _Float16 f = (_Float16)v;
          std::memcpy(&h, &f, 2);
        }
        s16[k * n1p + i1] = h;
      }
  }
  hipError_t e = hipGetDevice(&p->device);
  if (e != hipSuccess) { delete p; return hip_fail(e, "hipGetDevice"); }
  e = dev_alloc(&p->dev, total);
  if (e != hipSuccess) {
    delete p;
    return e == hipErrorOutOfMemory ? fail(FD_E_NOMEM, "fd_setup: device allocation") : hip_fail(e, "hipMalloc");
  }
  e = hipMemcpy(p->dev, host.data(), total, hipMemcpyHostToDevice);
  if (e != hipSuccess) {
    (void)dev_free(p->dev, total);
    delete p;
    return hip_fail(e, "hipMemcpy");
  }
  p->dev_bytes = total;
  unsigned char* base = static_cast<unsigned char*>(p->dev);
  if (fp8) {
    size_t sb = 0;
    for (int i = 0; i < ndim; ++i) sb = std::max(sb, stage8[i].size() * sizeof(float));
    void* tmp = nullptr;
    e = dev_alloc(&tmp, sb);
    for (int i = 0; i < ndim && e == hipSuccess; ++i) {
      const int64_t ent = int64_t(fdk::v3_ld(n[i], p->prec)) * fdk::v3_ld(n[i], p->prec);
      e = hipMemcpy(tmp, stage8[i].data(), stage8[i].size() * sizeof(float), hipMemcpyHostToDevice);
      for (int j = 0; j < 3 && e == hipSuccess; ++j)
        e = fdk::fp8s_image(static_cast<const float*>(tmp) + j * ent, base + offv[i][j], ent, nullptr);
      if (e == hipSuccess) e = hipDeviceSynchronize();
    }
    (void)dev_free(tmp, sb);
    if (e != hipSuccess) {
      (void)dev_free(p->dev, total);
      delete p;
      return e == hipErrorOutOfMemory ? fail(FD_E_NOMEM, "fd_setup: device allocation") : hip_fail(e, "FP8 images");
    }
  }
  for (int i = 0; i < ndim; ++i) {
    p->f_fwd[i] = base + off[i][0];
    p->f_bwd[i] = base + off[i][1];
    p->p_fwd[i] = base + offp[i][0];
    p->p_bwd[i] = base + offp[i][1];
    if (fdk::v3_factor_bytes(n[i], p->prec)) {
      p->v_fwd[i] = base + offv[i][0];
      p->v_bwd[i] = base + offv[i][1];
      p->v_snd[i] = base + offv[i][2];
    }
    p->d_dev[i] = reinterpret_cast<const double*>(base + offd[i]);
  }
  if (diag_target) p->scale_dev = base + offs;
  if (diag_target && p->slab) p->scale16 = base + offs16;
  *out = p;
  return FD_OK;
}

fd_status fd_destroy(fd_plan plan) {
  if (!plan) return FD_OK;
  if (plan->dev) {
    hipError_t e = dev_free(plan->dev, plan->dev_bytes);
    plan->dev = nullptr;
    delete plan;
    if (e != hipSuccess) return hip_fail(e, "hipFree");
    return FD_OK;
  }
  delete plan;
  return FD_OK;
}

int64_t fd_plan_size(fd_plan plan) { return plan ? plan->N : 0; }

size_t fd_plan_device_bytes(fd_plan plan) { return plan ? plan->dev_bytes : 0; }

fd_status fd_set_device_limit(size_t bytes) {
  g_dev_limit.store(bytes);
  return FD_OK;
}

size_t fd_device_bytes_held(void) { return g_dev_held.load(); }

size_t fd_workspace_bytes(fd_plan plan, int32_t nrhs) {
  (void)plan;
  (void)nrhs;
  return 0;
}

fd_status fd_setup_mass_banded(int32_t ndim, const int32_t* n, const double* const* M, fd_precision prec,
                               fd_plan* out) {
  if (!out) return fail(FD_E_ARG, "fd_setup_mass_banded: NULL out");
  *out = nullptr;
  if (ndim != 2 && ndim != 3) return fail(FD_E_ARG, "fd_setup_mass_banded: ndim must be 2 or 3");
  if (!n || !M) return fail(FD_E_ARG, "fd_setup_mass_banded: NULL n or M");
  if (int(prec) < 0 || int(prec) > 6) return fail(FD_E_ARG, "fd_setup_mass_banded: unknown precision");
  auto p = new (std::nothrow) fd_plan_s();
  if (!p) return fail(FD_E_NOMEM, "fd_setup_mass_banded: host allocation");
  p->ndim = ndim;
  p->prec = int(prec);
  p->mass_only = true;
  p->banded = true;
  p->N = 1;
  std::vector<double> fac[3];
  const bool f64 = io_is_f64(p->prec);
  const size_t eb = f64 ? 8 : 4;
  size_t offs[3], total = 0;
  for (int i = 0; i < ndim; ++i) {
    if (n[i] < 2 || n[i] > fdk::kMaxN || !M[i]) {
      delete p;
      return fail(FD_E_ARG, "fd_setup_mass_banded: each n[i] must be in [2, 256] with M[i] given");
    }
    p->n[i] = n[i];
    p->N *= n[i];
    int bw = 0;
    const int rc0 = fdh::band_cholesky(n[i], M[i], fdk::kMaxBand, &bw, nullptr, nullptr);
    if (rc0 != 0) {
      delete p;
      return fail(FD_E_ARG, "fd_setup_mass_banded: M[" + std::to_string(i) + "] asymmetric or bandwidth above 16");
    }
    p->bw[i] = bw;
    fac[i].assign(size_t(bw + 1) * n[i], 0.0);
    // rows 1..bw of the band and, in row 0, the reciprocal diagonal
    const int rc = fdh::band_cholesky(n[i], M[i], fdk::kMaxBand, &bw, fac[i].data(), fac[i].data());
    if (rc != 0) {
      delete p;
      return fail(FD_E_NOTSPD, "fd_setup_mass_banded: M[" + std::to_string(i) + "] is not positive definite");
    }
    offs[i] = total;
    total += (fac[i].size() * eb + 255) & ~size_t(255);
  }
  if (p->N >= (int64_t(1) << 28)) {
    delete p;
    return fail(FD_E_ARG, "fd_setup_mass_banded: prod(n) must be below 2^28");
  }
  hipError_t e = hipGetDevice(&p->device);
  if (e == hipSuccess) e = dev_alloc(&p->dev, total);
  if (e != hipSuccess) {
    p->dev = nullptr;
    delete p;
    return e == hipErrorOutOfMemory ? fail(FD_E_NOMEM, "fd_setup_mass_banded: device memory")
                                    : hip_fail(e, "fd_setup_mass_banded");
  }
  p->dev_bytes = total;
  std::vector<unsigned char> host(total, 0);
  for (int i = 0; i < ndim; ++i) {
    unsigned char* dst = host.data() + offs[i];
    for (size_t k = 0; k < fac[i].size(); ++k) {
      if (f64) {
        std::memcpy(dst + 8 * k, &fac[i][k], 8);
      } else {
        const float v = float(fac[i][k]);
        std::memcpy(dst + 4 * k, &v, 4);
      }
    }
    p->bfac[i] = static_cast<unsigned char*>(p->dev) + offs[i];
  }
  e = hipMemcpy(p->dev, host.data(), total, hipMemcpyHostToDevice);
  if (e != hipSuccess) {
    fd_destroy(p);
    return hip_fail(e, "fd_setup_mass_banded: upload");
  }
  *out = p;
  return FD_OK;
}

fd_status fd_plan_factors(fd_plan plan, int32_t dir, double* U, double* d) {
  if (!plan || dir < 0 || dir >= plan->ndim) return fail(FD_E_ARG, "fd_plan_factors: bad plan or direction");
  if (plan->banded) return fail(FD_E_UNSUPPORTED, "fd_plan_factors: a banded mass plan holds no eigenvectors");
  const int m = plan->n[dir];
  if (U) std::memcpy(U, plan->U[dir].data(), sizeof(double) * m * m);
  if (d) std::memcpy(d, plan->d[dir].data(), sizeof(double) * m);
  return FD_OK;
}

fd_status fd_apply(fd_plan plan, const void* r, void* z, int32_t nrhs, int64_t ld, void* stream) {
  fd_work wk;
  wk.plan = plan;
  wk.r = r;
  wk.z = z;
  wk.nrhs = nrhs;
  wk.ld = ld;
  return run_work(1, &wk, static_cast<hipStream_t>(stream));
}

fd_status fd_batch_create(int32_t count, const fd_work* work, fd_batch* out) {
  if (!out || count < 1 || !work) return fail(FD_E_ARG, "fd_batch_create: bad arguments");
  *out = nullptr;
  {
    fd_status s = batch_validate(count, work, "fd_batch_create");
    if (s != FD_OK) return s;
  }
  auto* b = new fd_batch_s;
  b->prec = work[0].plan->prec;
  b->works.assign(work, work + count);
  hipError_t e = hipGetDevice(&b->device);
  if (e == hipSuccess) e = hipDeviceGetAttribute(&b->cus, hipDeviceAttributeMultiprocessorCount, b->device);
  if (e != hipSuccess) {
    delete b;
    return hip_fail(e, "fd_batch_create");
  }
  fd_status s = FD_OK;
  for (int c = 0; c < 3 && s == FD_OK; ++c) s = batch_build_layout(b, c);
  if (s == FD_OK && b->smem > 160 * 1024) s = fail(FD_E_UNSUPPORTED, "fd_batch_create: factor image exceeds LDS");
  int per_cu = 0;
  if (s == FD_OK) {
    e = fdk::batch_resident(b->prec, b->smem, &per_cu);
    if (e != hipSuccess) s = hip_fail(e, "batch occupancy");
    else if (per_cu < 1) s = fail(FD_E_UNSUPPORTED, "fd_batch_create: batch kernel does not fit a CU");
  }
  if (s == FD_OK) {
    for (int st = 0; st < kStages; ++st)
      if (b->lay[0].tiles[st] > 0) b->last_stage = st;
    for (int st = 0; st < b->last_stage; ++st)
      if (b->lay[0].tiles[st] > 0) ++b->phases;
    s = batch_upload(b);
  }
  if (s == FD_OK) s = batch_build_staged(b);
  if (s == FD_OK) {
    e = dev_alloc(&b->ctl, 256);
    if (e == hipSuccess) e = hipMemset(b->ctl, 0, 256);
    if (e != hipSuccess) s = hip_fail(e, "fd_batch_create");
  }
  if (s != FD_OK) {
    fd_batch_destroy(b);
    return s;
  }
  *out = b;
  return FD_OK;
}

fd_status fd_batch_apply(fd_batch b, void* stream) {
  if (!b) return fail(FD_E_ARG, "fd_batch_apply: NULL batch");
  return batch_launch(b, static_cast<hipStream_t>(stream));
}

fd_status fd_batch_tune(fd_batch b, void* stream, int32_t reps, int32_t* choice) {
  if (!b || reps < 1) return fail(FD_E_ARG, "fd_batch_tune: bad arguments");
  hipStream_t st = static_cast<hipStream_t>(stream);
  hipEvent_t e0 = nullptr, e1 = nullptr;
  hipError_t e = hipEventCreate(&e0);
  if (e == hipSuccess) e = hipEventCreate(&e1);
  if (e != hipSuccess) return hip_fail(e, "fd_batch_tune");
  auto time_current = [&](float* ms) -> fd_status {
    fd_status s = batch_launch(b, st);  // warm-up
    hipError_t er = hipEventRecord(e0, st);
    for (int r = 0; r < reps && s == FD_OK && er == hipSuccess; ++r) s = batch_launch(b, st);
    if (er == hipSuccess) er = hipEventRecord(e1, st);
    if (er == hipSuccess) er = hipEventSynchronize(e1);
    if (er == hipSuccess) er = hipEventElapsedTime(ms, e0, e1);
    if (s == FD_OK && er != hipSuccess) s = hip_fail(er, "fd_batch_tune");
    if (s == FD_OK) s = fd_batch_check(b);
    return s;
  };
  // greedy over stages: each stage keeps the body choice that made the whole
  // apply fastest, given the choices already made for the earlier stages
  b->use_staged = false;
  b->use_segments = false;
  for (int i = 0; i < kStages; ++i) b->width[i] = 0;
  fd_status s = batch_upload(b);
  float best = 0.0f;
  if (s == FD_OK) s = time_current(&best);
  for (int stage = 0; stage < kStages && s == FD_OK; ++stage) {
    int keep = 0;
    for (int c = 1; c < 3 && s == FD_OK; ++c) {
      if (!b->lay[c].differs[stage]) continue;
      b->width[stage] = c;
      s = batch_upload(b);
      float ms = 0.0f;
      if (s == FD_OK) s = time_current(&ms);
      if (s == FD_OK && ms < best) {
        best = ms;
        keep = c;
      }
    }
    b->width[stage] = keep;
  }
  if (s == FD_OK) s = batch_upload(b);
  // the segment route with the chosen bodies
  if (s == FD_OK) {
    b->use_segments = true;
    float ms = 0.0f;
    s = time_current(&ms);
    if (s == FD_OK && ms < best) best = ms;
    else b->use_segments = false;
  }
  // the staged route, where the batch has one: first per fused launch the
  // faster of unit-by-unit (eigenvalues in LDS) and strided tiles, timed
  // alone, then the route as a whole against the persistent launch
  if (s == FD_OK && !b->staged.empty()) {
    for (auto& L : b->staged) {
      if (L.stage != 2 || !L.sc || s != FD_OK) continue;
      float t_mode[2] = {0.0f, 0.0f};
      for (int m = 0; m < 2 && s == FD_OK; ++m) {
        L.walk = m == 1;
        hipError_t er = staged_launch_one(b, L, st);  // warm-up
        if (er == hipSuccess) er = hipEventRecord(e0, st);
        for (int r = 0; r < reps && er == hipSuccess; ++r) er = staged_launch_one(b, L, st);
        if (er == hipSuccess) er = hipEventRecord(e1, st);
        if (er == hipSuccess) er = hipEventSynchronize(e1);
        if (er == hipSuccess) er = hipEventElapsedTime(&t_mode[m], e0, e1);
        if (er != hipSuccess) s = hip_fail(er, "fd_batch_tune");
      }
      L.walk = t_mode[1] <= t_mode[0];
    }
    b->use_staged = true;
    float ms = 0.0f;
    if (s == FD_OK) s = time_current(&ms);
    b->use_staged = s == FD_OK && ms < best;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (s != FD_OK) return s;
  b->tuned = true;
  if (choice) *choice = batch_config(b);
  return FD_OK;
}

fd_status fd_batch_set_config(fd_batch b, int32_t config) {
  if (b && config == kBatchStaged) {
    if (b->staged.empty())
      return fail(FD_E_UNSUPPORTED, "fd_batch_set_config: the batch has no staged route (not all slab-route plans)");
    hipError_t e = hipDeviceSynchronize();
    if (e != hipSuccess) return hip_fail(e, "fd_batch_set_config");
    b->use_staged = true;
    return FD_OK;
  }
  if (!b || config < 0 || (config & ~kBatchSegments) >= (1 << (2 * kStages)))
    return fail(FD_E_ARG, "fd_batch_set_config: bad arguments");
  b->use_staged = false;
  b->use_segments = (config & kBatchSegments) != 0;
  config &= ~kBatchSegments;
  for (int st = 0; st < kStages; ++st)
    if (((config >> (2 * st)) & 3) == 3) return fail(FD_E_ARG, "fd_batch_set_config: body choice 3");
  for (int st = 0; st < kStages; ++st) b->width[st] = (config >> (2 * st)) & 3;
  return batch_upload(b);
}

fd_status fd_batch_info(fd_batch b, int64_t* tiles, int32_t* grid, int32_t* config) {
  if (!b) return fail(FD_E_ARG, "fd_batch_info: NULL batch");
  if (tiles) {
    int64_t t = 0;
    if (b->use_staged)
      for (const auto& L : b->staged) t += L.tiles;
    else
      for (int st = 0; st < kStages; ++st) t += b->lay[b->width[st]].tiles[st];
    *tiles = t;
  }
  if (grid) *grid = int32_t(std::min<int64_t>(b->cus, b->max_tiles));  // (the persistent launch's)
  if (config) *config = batch_config(b);
  return FD_OK;
}

fd_status fd_batch_signature(fd_batch b, uint64_t* sig) {
  if (!b || !sig) return fail(FD_E_ARG, "fd_batch_signature: bad arguments");
  // FNV-1a over what the layout and the tuned configuration depend on: the
  // device's CU count, the precision class and per work the plan's shape,
  // route, scaling and the number of residuals (not the buffers)
  uint64_t h = 1469598103934665603ull;
  auto mix = [&h](int64_t v) {
    for (int i = 0; i < 8; ++i) {
      h ^= uint64_t(v >> (8 * i)) & 0xffu;
      h *= 1099511628211ull;
    }
  };
  mix(b->cus);
  mix(b->prec);
  mix(int64_t(b->works.size()));
  for (const fd_work& wk : b->works) {
    const fd_plan_s* p = wk.plan;
    mix(p->ndim);
    for (int i = 0; i < 3; ++i) mix(p->n[i]);
    mix(p->mass_only);
    mix(p->slab);
    mix(p->scale_dev != nullptr);
    mix(wk.nrhs);
  }
  *sig = h;
  return FD_OK;
}

fd_status fd_batch_check(fd_batch b) {
  if (!b) return fail(FD_E_ARG, "fd_batch_check: NULL batch");
  hipError_t e = hipDeviceSynchronize();
  if (e != hipSuccess) return hip_fail(e, "fd_batch_check");
  int32_t flag = 0;
  e = hipMemcpy(&flag, static_cast<unsigned char*>(b->ctl) + 128, sizeof(flag), hipMemcpyDeviceToHost);
  if (e != hipSuccess) return hip_fail(e, "fd_batch_check");
  if (flag) {
    // restart the counter so that the batch can run again
    uint32_t* bar = static_cast<uint32_t*>(b->ctl);
    int32_t* err = reinterpret_cast<int32_t*>(static_cast<unsigned char*>(b->ctl) + 128);
    e = fdk::batch_reset(bar, err, nullptr);
    if (e == hipSuccess) e = hipDeviceSynchronize();
    b->arrivals = 0;
    return fail(FD_E_HIP, "fd_batch_apply: a grid barrier wait gave up (grid not fully resident)");
  }
  return FD_OK;
}

fd_status fd_batch_destroy(fd_batch b) {
  if (!b) return FD_OK;
  (void)dev_free(b->dev, b->dev_cap);
  (void)dev_free(b->ctl, 256);
  (void)dev_free(b->sdev, b->sdev_bytes);
  delete b;
  return FD_OK;
}

fd_status fd_apply_batched(int32_t count, const fd_work* work, void* stream) {
  if (count < 0 || (count > 0 && !work)) return fail(FD_E_ARG, "fd_apply_batched: bad count/work");
  return run_work(count, work, static_cast<hipStream_t>(stream));
}

fd_status fd_apply_persistent_static(int32_t count, const fd_work* work, int32_t config, int32_t* status,
                                     void* stream) {
  if (count < 0 || (count > 0 && !work)) return fail(FD_E_ARG, "fd_apply_persistent_static: bad arguments");
  if (config < 0 || config >= (1 << (2 * kStages)))
    return fail(FD_E_ARG, "fd_apply_persistent_static: configuration word out of range");
  for (int st = 0; st < kStages; ++st)
    if (((config >> (2 * st)) & 3) == 3) return fail(FD_E_ARG, "fd_apply_persistent_static: body choice 3");
  fd_status s = batch_validate(count, work, "fd_apply_persistent_static");
  if (s != FD_OK) return s;
  hipStream_t st = static_cast<hipStream_t>(stream);
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
  std::lock_guard<std::mutex> lock(g_static_mu);
  StaticDevice* sd = nullptr;
  s = static_device(dev, &sd);
  if (s != FD_OK) return s;
  const int prec = count > 0 ? work[0].plan->prec : FD_F64;
  // the pass tables of every stage, in the layout fd_batch_create builds
  fdk::BatchArgs a{};
  int nd = 0, ns = 0, last_stage = -1;
  int64_t max_tiles = 0;
  size_t smem = 0;
  for (int stage = 0; stage < kStages; ++stage) {
    const int choice = (config >> (2 * stage)) & 3;
    int nc = 0;
    for (int i = 0; i < count; ++i) {
      if (nd + nc == kStaticMaxDesc)
        return fail(FD_E_ARG, "fd_apply_persistent_static: more passes than the " +
                                  std::to_string(kStaticMaxDesc) + " descriptors of the 2 MiB static table");
      size_t sm = 0;
      if (!batch_pass(prec, work[i], stage, choice, &g_cand_body[nc], &g_cand[nc], &sm)) continue;
      smem = std::max(smem, sm);
      g_ord[nc] = nc;
      ++nc;
    }
    // stable order of the keys (ties keep the work order)
    std::sort(g_ord, g_ord + nc, [](int x, int y) {
      const auto kx = batch_key(g_cand_body[x], g_cand[x]), ky = batch_key(g_cand_body[y], g_cand[y]);
      return kx < ky || (kx == ky && x < y);
    });
    a.stage_seg[stage] = ns;
    auto* desc = reinterpret_cast<fdk::BatchDesc*>(g_image);
    int64_t t = 0;
    for (int k = 0; k < nc; ++k) {
      const int c = g_ord[k];
      fdk::BatchDesc bd = g_cand[c];
      if (k == 0 || batch_key(g_cand_body[g_ord[k - 1]], g_cand[g_ord[k - 1]]) != batch_key(g_cand_body[c], bd)) {
        fdk::BatchSeg sg{};
        sg.d0 = nd;
        sg.t0 = int(t);
        sg.mode = bd.mode;
        sg.mt = bd.mt;
        sg.scale = bd.scale;
        sg.body = g_cand_body[c];
        g_seg[ns++] = sg;
      }
      bd.u.tile_begin = t;
      t += int64_t(bd.u.tiles_per_rhs) * bd.u.nrhs;
      if (t > 0x7fffffffLL) return fail(FD_E_ARG, "fd_apply_persistent_static: too many tiles in one stage");
      desc[nd++] = bd;
      g_seg[ns - 1].d1 = nd;
      g_seg[ns - 1].t1 = int(t);
    }
    if (t > 0) last_stage = stage;
    max_tiles = std::max(max_tiles, t);
  }
  a.stage_seg[kStages] = ns;
  const size_t db = size_t(nd) * sizeof(fdk::BatchDesc), sb = size_t(ns) * sizeof(fdk::BatchSeg);
  if (kStaticCtl + db + sb > kStaticBytes)
    return fail(FD_E_ARG, "fd_apply_persistent_static: pass tables of " + std::to_string(db + sb) +
                              " bytes exceed the 2 MiB static table");
  if (smem > 160 * 1024) return fail(FD_E_UNSUPPORTED, "fd_apply_persistent_static: factor image exceeds LDS");
  std::memcpy(g_image + db, g_seg, sb);
  uint32_t* bar = reinterpret_cast<uint32_t*>(sd->ptr);
  int32_t* err = status ? status : reinterpret_cast<int32_t*>(sd->ptr + 128);
  // the counter and the flag start at zero (a fill kernel, no memset node)
  e = fdk::batch_reset(bar, err, st);
  if (e != hipSuccess) return hip_fail(e, "batch reset");
  if (max_tiles == 0) return FD_OK;
  int per_cu = 0;
  e = fdk::batch_resident(prec, smem, &per_cu);
  if (e != hipSuccess) return hip_fail(e, "batch occupancy");
  if (per_cu < 1) return fail(FD_E_UNSUPPORTED, "fd_apply_persistent_static: batch kernel does not fit a CU");
  // pageable source: the runtime has consumed g_image when the call returns
  e = hipMemcpyAsync(sd->ptr + kStaticCtl, g_image, db + sb, hipMemcpyHostToDevice, st);
  if (e != hipSuccess) return hip_fail(e, "hipMemcpyAsync (pass tables)");
  a.desc = reinterpret_cast<const fdk::BatchDesc*>(sd->ptr + kStaticCtl);
  a.seg = reinterpret_cast<const fdk::BatchSeg*>(sd->ptr + kStaticCtl + db);
  a.barrier = bar;
  a.error = err;
  a.base = 0;
  a.last_stage = last_stage;
  const int64_t grid = std::min<int64_t>(sd->cus, max_tiles);
  e = fdk::batch_launch(a, prec, int(grid), smem, st);
  if (e != hipSuccess) return hip_fail(e, "batch kernel launch");
  return FD_OK;
}

}  // extern "C"
