// Host side of the svdv C-ABI: argument validation, configuration checks, the
// stage-1 panel/update schedule (Algorithm 1) with its TSQR tree plan, the
// per-(device, stream) workspace cache and the dispatch to the HIP kernels.
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

#include "../../include/svdv.h"
#include "kernels.hpp"

using namespace svdv;

namespace {

thread_local std::string g_last_error;

// Optional per-stage event timing (see svdv_timing in the header).
// Per kernel class (0: trailing update, 1: panel), every launch of the last
// timed call is bracketed by an event pair and its algorithmic flops and bytes
// are recorded on the host.
struct KernelLog {
  std::vector<hipEvent_t> ev;  // pool, pairs (2i, 2i+1)
  std::vector<double> flops, bytes;
  size_t used = 0;
  void reset() {
    used = 0;
    flops.clear();
    bytes.clear();
  }
  hipEvent_t next() {
    if (used == ev.size()) {
      hipEvent_t e = nullptr;
      hipEventCreate(&e);
      ev.push_back(e);
    }
    return ev[used++];
  }
};
struct Timing {
  bool enabled = false;
  bool kernels = false;  // also bracket every stage-1 launch (svdv_timing(2))
  bool valid = false;
  hipEvent_t ev[7] = {};
  hipEvent_t cev[2] = {};  // around the bulge-chase launch, on the stream it runs on
  KernelLog klog[2];
  void mark(int i, hipStream_t st) {
    if (!enabled) return;
    if (!ev[i]) hipEventCreate(&ev[i]);
    hipEventRecord(ev[i], st);
  }
  void chase_mark(int i, hipStream_t st) {
    if (!enabled) return;
    if (!cev[i]) hipEventCreate(&cev[i]);
    hipEventRecord(cev[i], st);
  }
  void begin_call() {
    valid = false;
    klog[0].reset();
    klog[1].reset();
  }
  void kbegin(int kind, hipStream_t st) {
    if (kernels) hipEventRecord(klog[kind].next(), st);
  }
  void kend(int kind, hipStream_t st, double fl, double by) {
    if (!kernels) return;
    hipEventRecord(klog[kind].next(), st);
    klog[kind].flops.push_back(fl);
    klog[kind].bytes.push_back(by);
  }
};
thread_local Timing g_timing;

int fail(int status, const std::string& msg) {
  g_last_error = msg;
  return status;
}
int fail_hip(hipError_t e, const char* where) {
  g_last_error = std::string(where) + ": " + hipGetErrorString(e);
  return SVDV_ERR_HIP;
}
#define HIPCHK(expr)                              \
  do {                                            \
    hipError_t _e = (expr);                       \
    if (_e != hipSuccess) return fail_hip(_e, #expr); \
  } while (0)

bool is_pow2_in(int v, int lo, int hi) { return v >= lo && v <= hi && (v & (v - 1)) == 0; }

int elem_size(int dtype) { return dtype == SVDV_F32 ? 4 : 8; }

// ----------------------------------------------------------------------------
// configuration
// ----------------------------------------------------------------------------

template <typename T>
bool larfb_ok(int tile, int threads, int ib) {
  const int KT = tile / 16, NW = threads / 64;
  return larfb_valid<T>(KT, ib, NW);
}

int check_config_impl(int64_t m, int64_t n, int dtype, const svdv_config& c) {
  if (dtype != SVDV_F32 && dtype != SVDV_F64) return fail(SVDV_ERR_INVALID_ARG, "dtype must be SVDV_F32 or SVDV_F64");
  if (!(c.tile == 16 || c.tile == 32 || c.tile == 64 || c.tile == 128))
    return fail(SVDV_ERR_UNSUPPORTED, "tile must be one of 16, 32, 64, 128");
  if (!is_pow2_in(c.threads, 64, 1024)) return fail(SVDV_ERR_UNSUPPORTED, "threads must be 64, 128, 256, 512 or 1024");
  if (!(c.inner_block == 1 || c.inner_block == 2 || c.inner_block == 4 || c.inner_block == 8))
    return fail(SVDV_ERR_UNSUPPORTED, "inner_block must be 1, 2, 4 or 8");
  if (c.sweep_width < 1 || c.sweep_width > 8) return fail(SVDV_ERR_UNSUPPORTED, "sweep_width must be in 1..8");
  if (c.update_precision != 0 && c.update_precision != 2 && c.update_precision != 3)
    return fail(SVDV_ERR_UNSUPPORTED, "update_precision must be 0 (input precision), 2 (BF16) or 3 (FP16)");
  if (c.update_precision != 0 &&
      (dtype != SVDV_F32 || c.tile > 64 || !larfb_reg_valid<float>(c.tile / 16, c.inner_block, c.threads / 64)))
    return fail(SVDV_ERR_UNSUPPORTED, "BF16/FP16 trailing updates need float32 input, a tile of at most 64 (the "
                                      "float64 panel must fit in LDS) and a configuration whose strip fits in registers");
  if (dtype == SVDV_F64 && c.tile > 64) return fail(SVDV_ERR_UNSUPPORTED, "float64 supports tiles up to 64");
  const bool ok = dtype == SVDV_F32 ? larfb_ok<float>(c.tile, c.threads, c.inner_block)
                                    : larfb_ok<double>(c.tile, c.threads, c.inner_block);
  if (!ok) return fail(SVDV_ERR_UNSUPPORTED, "trailing-update tile exceeds the register budget for this workgroup size");
  if (chase_lds_bytes(c.tile, c.sweep_width) > 160 * 1024 - 1024)
    return fail(SVDV_ERR_UNSUPPORTED, "bulge-chase LDS exceeds 160 KiB for this tile and sweep width");
  (void)m;
  (void)n;
  return SVDV_OK;
}

struct TunedCell {
  int64_t n;
  int32_t dtype, tile, threads, inner_block, sweep_width;
};
#include "tuned_table.inc"

// The default configuration: the auto-tuner's measured best of the cell with
// the same dtype whose size is nearest to min(m, n) on a log scale (ties go to
// the larger cell), if the library accepts it for (m, n); otherwise tile 16 with
// the widest trailing-update workgroup that fits its registers (1024 threads in
// float32, 256 in float64), inner block 1 and sweep width 4.
svdv_config default_config(int64_t m, int64_t n, int dtype) {
  svdv_config c;
  c.tile = 16;
  c.threads = dtype == SVDV_F32 ? 1024 : 256;
  c.inner_block = 1;
  c.sweep_width = 4;
  c.update_precision = 0;
  const double k = (double)std::max<int64_t>(1, std::min(m, n));
  const TunedCell* best = nullptr;
  double bd = 0.0;
  for (const TunedCell& t : kTunedCells) {
    if (t.dtype != dtype || t.n <= 0) continue;
    const double d = std::fabs(std::log2((double)t.n) - std::log2(k));
    if (!best || d < bd - 1e-12 || (std::fabs(d - bd) <= 1e-12 && t.n > best->n)) {
      best = &t;
      bd = d;
    }
  }
  if (best) {
    svdv_config t = c;
    t.tile = best->tile;
    t.threads = best->threads;
    t.inner_block = best->inner_block;
    t.sweep_width = best->sweep_width;
    const std::string saved = g_last_error;
    if (check_config_impl(m, n, dtype, t) == SVDV_OK) c = t;
    g_last_error = saved;
  }
  return c;
}

// ----------------------------------------------------------------------------
// TSQR tree plan for one panel of height h and width bw
// ----------------------------------------------------------------------------

struct Level {
  int64_t h;           // rows at this level
  int64_t chunk_rows;  // rows per chunk
  int32_t P;           // chunks
  RowMap rm;
  int64_t ldv;         // leading dimension of this level's V (h rounded up to 16)
  int64_t voff;        // offset (elements) of this level's V in the V workspace
  int64_t toff;        // offset (elements) of this level's T factors
};

// 4-row vector access in the trailing update: float, rows contiguous, and every
// 4-row group of C and of V starting on a 16-byte boundary.
template <typename T>
int larfb_vec_ok(const LarfbArgs<T>& a) {
  if (sizeof(T) != 4 || a.M.rs != 1) return 0;
  const RowMap& r = a.rm;
  const bool rows4 = r.base % 4 == 0 && r.chunk_stride % 4 == 0 && (r.per_unit == 0 || (r.per_unit % 4 == 0 &&
                                                                                          r.unit_stride % 4 == 0));
  const bool mat4 = (reinterpret_cast<uintptr_t>(a.M.p) % 16) == 0 && a.M.cs % 4 == 0;
  const bool v4 = (reinterpret_cast<uintptr_t>(a.V) % 16) == 0 && a.ldv % 4 == 0 && a.chunk_rows % 4 == 0;
  return rows4 && mat4 && v4 ? 1 : 0;
}
// V alone: 16-byte loads of 4 consecutive reflector rows (float only).
template <typename T>
int larfb_vecv_ok(const LarfbArgs<T>& a) {
  if (sizeof(T) != 4) return 0;
  return (reinterpret_cast<uintptr_t>(a.V) % 16) == 0 && a.ldv % 4 == 0 && a.chunk_rows % 4 == 0 ? 1 : 0;
}

std::vector<Level> plan_panel(int64_t r0, int64_t h, int bw, int tile, int hmax) {
  std::vector<Level> L;
  int64_t voff = 0, toff = 0;
  // level 1
  int64_t P = 1, cr = h;
  if (h > hmax) {
    for (P = (h + hmax - 1) / hmax;; ++P) {
      cr = ((h + P - 1) / P + 15) / 16 * 16;
      if (cr > hmax) continue;
      const int64_t rem = h - (P - 1) * cr;
      if (rem >= bw && rem <= hmax && rem > 0) break;
    }
  }
  Level l1;
  l1.h = h;
  l1.chunk_rows = cr;
  l1.P = (int32_t)P;
  l1.rm = RowMap{r0, cr, 0, 0};
  l1.ldv = (h + 15) / 16 * 16;
  l1.voff = voff;
  l1.toff = toff;
  voff += l1.ldv * tile;
  toff += P * (int64_t)tile * tile;
  L.push_back(l1);
  int64_t U = cr;  // matrix rows between consecutive chunk tops of the previous level
  const int64_t F = hmax / bw;
  while (L.back().P > 1) {
    const int64_t units = L.back().P;
    Level lv;
    lv.h = units * bw;
    if (lv.h <= hmax) {
      lv.P = 1;
      lv.chunk_rows = lv.h;
      lv.rm = RowMap{r0, 0, U, bw};
    } else {
      lv.P = (int32_t)((units + F - 1) / F);
      lv.chunk_rows = F * bw;
      lv.rm = RowMap{r0, F * U, U, bw};
    }
    lv.ldv = (lv.h + 15) / 16 * 16;
    lv.voff = voff;
    lv.toff = toff;
    voff += lv.ldv * tile;
    toff += (int64_t)lv.P * tile * tile;
    L.push_back(lv);
    U = (lv.P > 1) ? F * U : U;
  }
  return L;
}

void panel_ws(int64_t h, int bw, int tile, int hmax, int64_t* vsz, int64_t* tsz) {
  auto L = plan_panel(0, h, bw, tile, hmax);
  int64_t v = 0, t = 0;
  for (auto& l : L) {
    v += l.ldv * tile;
    t += (int64_t)l.P * tile * tile;
  }
  *vsz = v;
  *tsz = t;
}

// ----------------------------------------------------------------------------
// workspace
// ----------------------------------------------------------------------------

struct Workspace {
  void* ptr = nullptr;
  size_t bytes = 0;
};
std::mutex g_mu;
std::map<std::pair<int, void*>, Workspace> g_ws;

// A second stream per (device, caller stream) for the upper levels of a TSQR tree,
// which run beside the trailing update of the level below (see run_panel_step),
// and the events that fork it from and join it to the caller's stream.
struct SideStream {
  hipStream_t s = nullptr;
  hipEvent_t ev[8] = {};
};
std::map<std::pair<int, void*>, SideStream> g_side;

int get_side(void* stream, SideStream** out) {
  int dev = 0;
  HIPCHK(hipGetDevice(&dev));
  std::lock_guard<std::mutex> lk(g_mu);
  SideStream& ss = g_side[{dev, stream}];
  if (!ss.s) {
    HIPCHK(hipStreamCreateWithFlags(&ss.s, hipStreamNonBlocking));  // default priority
    for (auto& e : ss.ev) HIPCHK(hipEventCreateWithFlags(&e, hipEventDisableTiming));
  }
  *out = &ss;
  return SVDV_OK;
}

int get_workspace(void* stream, size_t bytes, char** out) {
  int dev = 0;
  HIPCHK(hipGetDevice(&dev));
  std::lock_guard<std::mutex> lk(g_mu);
  Workspace& w = g_ws[{dev, stream}];
  if (w.bytes < bytes) {
    if (w.ptr) {
      HIPCHK(hipStreamSynchronize((hipStream_t)stream));
      HIPCHK(hipFree(w.ptr));
      w.ptr = nullptr;
      w.bytes = 0;
    }
    hipError_t e = hipMalloc(&w.ptr, bytes);
    if (e != hipSuccess) {
      w.ptr = nullptr;
      return fail(SVDV_ERR_NO_MEMORY, std::string("workspace hipMalloc failed: ") + hipGetErrorString(e));
    }
    w.bytes = bytes;
  }
  *out = (char*)w.ptr;
  return SVDV_OK;
}

size_t align_up(size_t x) { return (x + 255) / 256 * 256; }

// Persistent grid of the bulge chase: every workgroup must be resident at once.
int chase_grid(int ngroups, int b, int W) { return std::min<int>(ngroups, chase_max_groups_resident(b, W)); }

struct Layout {
  size_t W, V, T, Bs, progress, err, amax, exp, d, e, work, total;
};

Layout make_layout(int64_t M, int64_t N, int es, int tile, int hmax, int sweep_width, int64_t ldw) {
  Layout L{};
  size_t off = 0;
  auto take = [&](size_t bytes) {
    size_t o = off;
    off += align_up(bytes);
    return o;
  };
  int64_t vsz = 0, tsz = 0;
  panel_ws(M, std::min<int64_t>(tile, N), tile, hmax, &vsz, &tsz);
  L.W = take((size_t)ldw * N * es);
  L.V = take((size_t)vsz * es);
  L.T = take((size_t)tsz * es);
  L.Bs = take((size_t)N * 3 * tile * 8);
  const int64_t ngroups = (N + sweep_width - 1) / sweep_width + 1;
  L.progress = take((size_t)(ngroups + 1) * 4);
  L.err = take(8);
  L.amax = take(8);
  L.exp = take(8);
  L.d = take((size_t)N * 8);
  L.e = take((size_t)N * 8);
  L.work = take((size_t)bisect_work_doubles(N) * 8);
  L.total = off;
  return L;
}

// ----------------------------------------------------------------------------
// stage 1 driver
// ----------------------------------------------------------------------------

// One panel step: the TSQR levels of the panel, then the trailing update level by
// level.  The update of level 1 (the chunks' own reflectors, Q_1^T C) does not read
// what the levels above it compute: they factor the stacked R factors in the panel's
// columns and write their own V and T, while that update reads level 1's V and T and
// writes the trailing columns.  With a side stream, levels 2.. are factored there,
// forked after level 1's factorisation, so they run beside level 1's update; the
// update of level l waits for level l's factorisation.  Same kernels, same
// arithmetic, in either order.
template <typename T>
int run_panel_step(View<T> V, int64_t r0, int64_t pc, int64_t h, int bw, int64_t ncols, const svdv_config& cfg,
                   T* vws, T* tws, hipStream_t st, const SideStream* side) {
  const int hmax = chunk_qr_hmax<T>(cfg.tile);
  auto levels = plan_panel(r0, h, bw, cfg.tile, hmax);
  // per-kernel timing (svdv_timing(2)) keeps one stream, so that each launch's
  // events bracket that kernel alone and not its wait for a CU beside the update
  const bool fork = side != nullptr && !g_timing.kernels && levels.size() > 1 && levels.size() <= 8;
  for (size_t li = 0; li < levels.size(); ++li) {
    const auto& lv = levels[li];
    const hipStream_t sp = fork && li > 0 ? side->s : st;
    if (fork && li == 1) {
      HIPCHK(hipEventRecord(side->ev[0], st));
      HIPCHK(hipStreamWaitEvent(side->s, side->ev[0], 0));
    }
    ChunkQRArgs<T> a;
    a.M = V;
    a.pc = pc;
    a.bw = bw;
    a.rm = lv.rm;
    a.h = lv.h;
    a.chunk_rows = lv.chunk_rows;
    a.P = lv.P;
    a.V = vws + lv.voff;
    a.ldv = lv.ldv;
    a.Tm = tws + lv.toff;
    a.hp = cfg.update_precision != 0 ? 1 : 0;
    g_timing.kbegin(1, sp);
    HIPCHK(launch_chunk_qr<T>(cfg.tile, a, sp));
    // Householder QR of P chunks of (chunk rows x bw): 2 r bw^2 flops, panel read and written once
    g_timing.kend(1, sp, 2.0 * (double)lv.h * bw * bw, 2.0 * sizeof(T) * (double)lv.h * bw);
    if (fork && li > 0) HIPCHK(hipEventRecord(side->ev[li], side->s));
  }
  if (pc + bw < ncols) {
    for (size_t li = 0; li < levels.size(); ++li) {
      const auto& lv = levels[li];
      if (fork && li > 0) HIPCHK(hipStreamWaitEvent(st, side->ev[li], 0));
      LarfbArgs<T> a;
      a.M = V;
      a.rm = lv.rm;
      a.h = lv.h;
      a.chunk_rows = lv.chunk_rows;
      a.P = lv.P;
      a.col0 = pc + bw;
      a.col1 = ncols;
      a.V = vws + lv.voff;
      a.ldv = lv.ldv;
      a.Tm = tws + lv.toff;
      a.ldt = cfg.tile;
      a.k = (int32_t)(lv.P == 1 ? std::min<int64_t>(bw, lv.h) : bw);
      a.vec = larfb_vec_ok(a);
      a.vecv = larfb_vecv_ok(a);
      a.prec = cfg.update_precision;
      g_timing.kbegin(0, st);
      HIPCHK(launch_larfb<T>(cfg.tile, cfg.threads / 64, cfg.inner_block, a, st));
      // C (rows x w) read and written once, V (rows x k) read once; 4 rows w k flops
      const double w = (double)(a.col1 - a.col0);
      g_timing.kend(0, st, 4.0 * (double)lv.h * w * a.k, sizeof(T) * ((double)lv.h * w * 2.0 + (double)lv.h * a.k));
    }
  } else if (fork) {
    HIPCHK(hipStreamWaitEvent(st, side->ev[levels.size() - 1], 0));  // the last panel: join before the band is read
  }
  return SVDV_OK;
}

template <typename T>
int run_stage1(T* W, int64_t ldw, int64_t M, int64_t N, const svdv_config& cfg, T* vws, T* tws, hipStream_t st,
               const SideStream* side) {
  const int b = cfg.tile;
  const View<T> colv{W, 1, ldw};
  const View<T> rowv{W, ldw, 1};
  for (int64_t k0 = 0; k0 < N; k0 += b) {
    const int bw = (int)std::min<int64_t>(b, N - k0);
    // QR sweep: tile column, rows k0..M-1, update columns k0+bw..N-1
    int rc = run_panel_step<T>(colv, k0, k0, M - k0, bw, N, cfg, vws, tws, st, side);
    if (rc) return rc;
    // LQ sweep: tile row k0..k0+b-1, columns k0+b..N-1 (QR of the transposed view),
    // update rows k0+b..M-1 (view columns)
    const int64_t c1 = k0 + b;
    if (c1 < N) {
      rc = run_panel_step<T>(rowv, c1, k0, N - c1, b, M, cfg, vws, tws, st, side);
      if (rc) return rc;
    }
  }
  return SVDV_OK;
}

// ----------------------------------------------------------------------------
// argument checks shared by the entry points
// ----------------------------------------------------------------------------

int check_matrix_args(const void* A, int64_t m, int64_t n, int64_t lda, int dtype) {
  if (dtype != SVDV_F32 && dtype != SVDV_F64) return fail(SVDV_ERR_INVALID_ARG, "dtype must be SVDV_F32 or SVDV_F64");
  if (m < 0 || n < 0) return fail(SVDV_ERR_INVALID_ARG, "m and n must be >= 0");
  if (lda < std::max<int64_t>(1, m)) return fail(SVDV_ERR_INVALID_ARG, "lda must be >= max(1, m)");
  if (m > 0 && n > 0 && A == nullptr) return fail(SVDV_ERR_INVALID_ARG, "A is NULL");
  if (m > (int64_t)1 << 20 || n > (int64_t)1 << 20) return fail(SVDV_ERR_UNSUPPORTED, "dimension above 2^20");
  return SVDV_OK;
}

// ext_ws (optional): a caller-provided workspace of ext_bytes bytes used instead of
// the cached allocation; a layout larger than it is rejected before any GPU work.
template <typename T>
int svd_values_t(const T* A, int64_t m, int64_t n, int64_t lda, T* S, hipStream_t st, const svdv_config& cfg,
                 double* band_out, int64_t ldband, double* d_out, double* e_out, char* ext_ws = nullptr,
                 size_t ext_bytes = 0) {
  const int transpose = m < n;
  const int64_t M = transpose ? n : m, N = transpose ? m : n;
  const int64_t ldw = (M + 15) / 16 * 16;
  const int hmax = chunk_qr_hmax<T>(cfg.tile);
  Layout L = make_layout(M, N, sizeof(T), cfg.tile, hmax, cfg.sweep_width, ldw);
  char* ws = nullptr;
  int rc = SVDV_OK;
  if (ext_ws) {
    if (L.total > ext_bytes)
      return fail(SVDV_ERR_UNSUPPORTED, "workspace of " + std::to_string(L.total) + " bytes exceeds the fixed array of " +
                                            std::to_string(ext_bytes) + " bytes");
    ws = ext_ws;
  } else {
    rc = get_workspace(st, L.total, &ws);
    if (rc) return rc;
  }
  T* W = (T*)(ws + L.W);
  T* vws = (T*)(ws + L.V);
  T* tws = (T*)(ws + L.T);
  double* Bs = (double*)(ws + L.Bs);
  int* progress = (int*)(ws + L.progress);
  int* err = (int*)(ws + L.err);
  unsigned long long* amax = (unsigned long long*)(ws + L.amax);
  int* expo = (int*)(ws + L.exp);
  double* d = d_out ? d_out : (double*)(ws + L.d);
  double* e = e_out ? e_out : (double*)(ws + L.e);
  double* work = (double*)(ws + L.work);

  // the allocation-free path (ext_ws) creates nothing: its panel levels stay on one stream
  SideStream* side = nullptr;
  if (!ext_ws) {
    rc = get_side(st, &side);
    if (rc) return rc;
  }
  g_timing.begin_call();
  g_timing.mark(0, st);
  HIPCHK(launch_stage_in<T>(A, m, n, lda, transpose, W, ldw, amax, expo, st));
  g_timing.mark(1, st);
  rc = run_stage1<T>(W, ldw, M, N, cfg, vws, tws, st, side);
  if (rc) return rc;
  g_timing.mark(2, st);
  if (band_out) {
    HIPCHK(launch_band_extract<T>(W, ldw, N, cfg.tile, band_out, ldband, expo, st));
    return SVDV_OK;
  }
  HIPCHK(launch_band_pack<T>(W, ldw, N, cfg.tile, Bs, 3 * cfg.tile, expo, 0, st));
  g_timing.mark(3, st);
  ChaseArgs ca{};
  ca.Bs = Bs;
  ca.ldb = 3 * cfg.tile;
  ca.n = N;
  ca.b = cfg.tile;
  ca.W = cfg.sweep_width;
  ca.ngroups = (int32_t)std::max<int64_t>(1, (N - 1 + cfg.sweep_width - 1) / cfg.sweep_width);
  ca.progress = progress;
  ca.err = err;
  ca.d = d;
  ca.e = e;
  int grid = chase_grid(ca.ngroups, cfg.tile, cfg.sweep_width);
  if (grid < 1) return fail(SVDV_ERR_UNSUPPORTED, "bulge-chase kernel cannot be resident with this configuration");
  hipLaunchKernelGGL(k_fill_i32, dim3(1), dim3(64), 0, st, err, 0, (int64_t)1);
  g_timing.chase_mark(0, st);
  HIPCHK(launch_chase(ca, grid, st));
  g_timing.chase_mark(1, st);
  g_timing.mark(4, st);
  if (S) HIPCHK(launch_bisect<T>(d, e, N, S, work, expo, 0, st, err));
  g_timing.mark(5, st);
  g_timing.valid = g_timing.enabled;
  return SVDV_OK;
}

// ----------------------------------------------------------------------------
// fixed device array of the allocation-free entry point
// ----------------------------------------------------------------------------
// Each GPU the library runs on holds its own copy of `scratch` from the module's
// load until the process ends.  In host code the name is only a stand-in for the
// symbol: the device address of a GPU's copy comes from hipGetSymbolAddress with
// that GPU current, looked up once per device and kept here.
constexpr size_t kNoallocBytes = (size_t)SVDV_NOALLOC_SCRATCH_BYTES;
__device__ __align__(256) char scratch[kNoallocBytes];
std::mutex g_scratch_mu;
std::map<int, char*> g_scratch_ptr;

int scratch_address(char** out) {
  int dev = 0;
  HIPCHK(hipGetDevice(&dev));
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  auto it = g_scratch_ptr.find(dev);
  if (it == g_scratch_ptr.end()) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || p == nullptr) return fail_hip(e, "hipGetSymbolAddress(scratch)");
    it = g_scratch_ptr.emplace(dev, (char*)p).first;
  }
  *out = it->second;
  return SVDV_OK;
}

// ----------------------------------------------------------------------------
// batched driver: every stage runs once for the whole batch, matrix i taking
// its share of each launch through per-matrix argument tables in device
// memory; the launch sequence is captured in a hipGraph and replayed while the
// shapes stay the same (only the pointer table is refreshed between calls).
// ----------------------------------------------------------------------------

struct BatchPlan {
  // key
  int dtype = -1;
  svdv_config cfg{};
  std::vector<int64_t> m, n, lda, soff;
  // device memory: tables + per-matrix workspaces
  char* mem = nullptr;
  size_t bytes = 0;
  size_t mats_off = 0;             // BatchMat<T>[count] (refreshed per call)
  std::vector<char> mats_host;     // host copy of that table
  std::vector<int> idx;            // plan order -> batch index (matrices with min(m, n) > 0, N descending)
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  std::function<int(hipStream_t)> record;  // enqueues the launch sequence (built with the tables)
  void release() {
    if (exec) hipGraphExecDestroy(exec);
    if (graph) hipGraphDestroy(graph);
    if (mem) hipFree(mem);
    exec = nullptr;
    graph = nullptr;
    mem = nullptr;
  }
};
// Cached batched plans, one per (device, stream, configuration): a batch whose
// matrices take different configurations keeps one plan per configuration.
struct BatchKey {
  int dev;
  void* stream;
  int32_t tile, threads, inner_block, sweep_width, precision;
  bool operator<(const BatchKey& o) const {
    return std::tie(dev, stream, tile, threads, inner_block, sweep_width, precision) <
           std::tie(o.dev, o.stream, o.tile, o.threads, o.inner_block, o.sweep_width, o.precision);
  }
};
std::map<BatchKey, BatchPlan> g_batch;

// Builds the plan's tables and workspaces (uploaded here, before any capture)
// and the recorder of its launch sequence.
template <typename T>
int batched_build(BatchPlan& P, const void* const* A_array, void* S) {
  const svdv_config& cfg = P.cfg;
  const int b = cfg.tile, W = cfg.sweep_width;
  const int cnt = (int)P.idx.size();
  // sizes in plan order
  std::vector<int64_t> Mv(cnt), Nv(cnt), ldw(cnt), ldv(cnt), ng(cnt);
  int64_t maxN = 0, maxM = 0, total_groups = 0, total_vals = 0;
  for (int i = 0; i < cnt; ++i) {
    const int q = P.idx[i];
    Mv[i] = std::max(P.m[q], P.n[q]);
    Nv[i] = std::min(P.m[q], P.n[q]);
    ldw[i] = (Mv[i] + 15) / 16 * 16;
    ldv[i] = ldw[i];
    ng[i] = std::max<int64_t>(0, (Nv[i] - 1 + W - 1) / W);
    maxN = std::max(maxN, Nv[i]);
    maxM = std::max(maxM, Mv[i]);
    total_groups += ng[i];
    total_vals += Nv[i];
  }
  const int64_t steps = (maxN + b - 1) / b;
  // layout
  size_t off = 0;
  auto take = [&](size_t bytes) {
    size_t o = off;
    off += align_up(bytes);
    return o;
  };
  P.mats_off = take(sizeof(BatchMat<T>) * cnt);
  const size_t qr_off = take(sizeof(ChunkQRArgs<T>) * cnt * steps), lq_off = take(sizeof(ChunkQRArgs<T>) * cnt * steps);
  const size_t uq_off = take(sizeof(LarfbArgs<T>) * cnt * steps), ul_off = take(sizeof(LarfbArgs<T>) * cnt * steps);
  const size_t ch_off = take(sizeof(ChaseArgs) * cnt);
  const size_t ord_off = take(sizeof(int) * 2 * std::max<int64_t>(1, total_groups));
  const size_t vmat_off = take(sizeof(int) * std::max<int64_t>(1, total_vals));
  const size_t voff_off = take(sizeof(int64_t) * cnt);
  // progress counters of every matrix (ng + 1 each), then the ticket and the error flag: one fill clears them
  std::vector<int64_t> prog(cnt);
  int64_t nprog = 0;
  for (int i = 0; i < cnt; ++i) {
    prog[i] = nprog;
    nprog += ng[i] + 1;
  }
  const size_t prog_off = take(sizeof(int) * (nprog + 2));
  const size_t amax_off = take(sizeof(unsigned long long) * cnt);
  const size_t exp_off = take(sizeof(int) * cnt);
  std::vector<size_t> w_off(cnt), v_off(cnt), t_off(cnt), bs_off(cnt), d_off(cnt), e_off(cnt), wk_off(cnt);
  for (int i = 0; i < cnt; ++i) {
    w_off[i] = take(sizeof(T) * ldw[i] * Nv[i]);
    v_off[i] = take(sizeof(T) * ldv[i] * b);
    t_off[i] = take(sizeof(T) * b * b);
    bs_off[i] = take(sizeof(double) * Nv[i] * 3 * b);
    d_off[i] = take(sizeof(double) * Nv[i]);
    e_off[i] = take(sizeof(double) * Nv[i]);
    wk_off[i] = take(sizeof(double) * bisect_work_doubles(Nv[i]));
  }
  if (off > P.bytes) {
    if (P.mem) HIPCHK(hipFree(P.mem));
    P.mem = nullptr;
    hipError_t e = hipMalloc(&P.mem, off);
    if (e != hipSuccess) return fail(SVDV_ERR_NO_MEMORY, "batched workspace hipMalloc failed");
    P.bytes = off;
  }
  char* base = P.mem;
  // host tables
  std::vector<BatchMat<T>> mats(cnt);
  for (int i = 0; i < cnt; ++i) {
    const int q = P.idx[i];
    BatchMat<T>& t = mats[i];
    t.A = (const T*)A_array[q];
    t.m = P.m[q];
    t.n = P.n[q];
    t.lda = P.lda[q];
    t.transpose = P.m[q] < P.n[q];
    t.M = Mv[i];
    t.N = Nv[i];
    t.W = (T*)(base + w_off[i]);
    t.ldw = ldw[i];
    t.amax = (unsigned long long*)(base + amax_off) + i;
    t.exp = (int*)(base + exp_off) + i;
    t.Bs = (double*)(base + bs_off[i]);
    t.d = (double*)(base + d_off[i]);
    t.e = (double*)(base + e_off[i]);
    t.work = (double*)(base + wk_off[i]);
    t.S = (T*)S + P.soff[q];
  }
  std::vector<ChunkQRArgs<T>> qr(cnt * steps), lq(cnt * steps);
  std::vector<LarfbArgs<T>> uq(cnt * steps), ul(cnt * steps);
  std::vector<int> n_qr(steps, 0), n_lq(steps, 0), vec_qr(steps, 1), vec_lq(steps, 1);
  std::vector<int64_t> mc_qr(steps, 0), mc_lq(steps, 0);
  std::vector<int64_t> lo_qr(steps, INT64_MAX), hi_qr(steps, 0), lo_lq(steps, INT64_MAX), hi_lq(steps, 0);
  for (int64_t k = 0; k < steps; ++k) {
    const int64_t k0 = k * b;
    for (int i = 0; i < cnt; ++i) {
      if (Nv[i] <= k0) break;  // N descending: the active matrices are a prefix
      T* Wp = mats[i].W;
      T* Vp = (T*)(base + v_off[i]);
      T* Tp = (T*)(base + t_off[i]);
      const int bw = (int)std::min<int64_t>(b, Nv[i] - k0);
      {  // QR sweep of the tile column
        const int64_t h = Mv[i] - k0;
        ChunkQRArgs<T>& a = qr[k * cnt + i];
        a.M = View<T>{Wp, 1, ldw[i]};
        a.pc = k0;
        a.bw = bw;
        a.rm = RowMap{k0, h, 0, 0};
        a.h = h;
        a.chunk_rows = h;
        a.P = 1;
        a.V = Vp;
        a.ldv = (h + 15) / 16 * 16;
        a.Tm = Tp;
        a.hp = cfg.update_precision != 0 ? 1 : 0;
        LarfbArgs<T>& u = uq[k * cnt + i];
        u.M = a.M;
        u.rm = a.rm;
        u.h = h;
        u.chunk_rows = h;
        u.P = 1;
        u.col0 = k0 + bw;
        u.col1 = Nv[i];
        u.V = Vp;
        u.ldv = a.ldv;
        u.Tm = Tp;
        u.ldt = b;
        u.k = (int32_t)std::min<int64_t>(bw, h);
        u.prec = cfg.update_precision;
        u.vec = larfb_vec_ok(u);
        u.vecv = larfb_vecv_ok(u);
        vec_qr[k] &= u.vec;
        mc_qr[k] = std::max<int64_t>(mc_qr[k], u.col1 - u.col0);
        if (u.col1 > u.col0) {
          lo_qr[k] = std::min<int64_t>(lo_qr[k], h);
          hi_qr[k] = std::max<int64_t>(hi_qr[k], h);
        }
        n_qr[k] = i + 1;
      }
      const int64_t c1 = k0 + b;
      if (c1 < Nv[i]) {  // LQ sweep of the tile row
        const int64_t h = Nv[i] - c1;
        ChunkQRArgs<T>& a = lq[k * cnt + i];
        a.M = View<T>{Wp, ldw[i], 1};
        a.pc = k0;
        a.bw = b;
        a.rm = RowMap{c1, h, 0, 0};
        a.h = h;
        a.chunk_rows = h;
        a.P = 1;
        a.V = Vp;
        a.ldv = (h + 15) / 16 * 16;
        a.Tm = Tp;
        a.hp = cfg.update_precision != 0 ? 1 : 0;
        LarfbArgs<T>& u = ul[k * cnt + i];
        u.M = a.M;
        u.rm = a.rm;
        u.h = h;
        u.chunk_rows = h;
        u.P = 1;
        u.col0 = k0 + b;
        u.col1 = Mv[i];
        u.V = Vp;
        u.ldv = a.ldv;
        u.Tm = Tp;
        u.ldt = b;
        u.k = (int32_t)std::min<int64_t>(b, h);
        u.prec = cfg.update_precision;
        u.vec = larfb_vec_ok(u);
        u.vecv = larfb_vecv_ok(u);
        vec_lq[k] &= u.vec;
        mc_lq[k] = std::max<int64_t>(mc_lq[k], u.col1 - u.col0);
        if (u.col1 > u.col0) {
          lo_lq[k] = std::min<int64_t>(lo_lq[k], h);
          hi_lq[k] = std::max<int64_t>(hi_lq[k], h);
        }
        n_lq[k] = i + 1;
      }
    }
  }
  int* progress = (int*)(base + prog_off);
  int* ticket = progress + nprog;
  int* err = ticket + 1;
  std::vector<ChaseArgs> ch(cnt);
  for (int i = 0; i < cnt; ++i) {
    ChaseArgs& c = ch[i];
    c = ChaseArgs{};
    c.Bs = mats[i].Bs;
    c.ldb = 3 * b;
    c.n = Nv[i];
    c.b = b;
    c.W = W;
    c.ngroups = (int32_t)ng[i];
    c.progress = progress + prog[i];
    c.err = err;
    c.d = mats[i].d;
    c.e = mats[i].e;
  }
  std::vector<int> order;
  order.reserve(2 * total_groups);
  for (int64_t r = 0;; ++r) {  // round robin over matrices: predecessors keep smaller tickets
    bool any = false;
    for (int i = 0; i < cnt; ++i)
      if (r < ng[i]) {
        order.push_back(i);
        order.push_back((int)r);
        any = true;
      }
    if (!any) break;
  }
  std::vector<int> vmat(total_vals);
  std::vector<int64_t> voff(cnt);
  for (int i = 0, v = 0; i < cnt; ++i) {
    voff[i] = v;
    for (int64_t j = 0; j < Nv[i]; ++j) vmat[v++] = i;
  }
  // upload (synchronous, before anything is recorded)
  auto up = [&](size_t o, const void* src, size_t bytes) -> hipError_t {
    return bytes ? hipMemcpy(base + o, src, bytes, hipMemcpyHostToDevice) : hipSuccess;
  };
  HIPCHK(up(P.mats_off, mats.data(), sizeof(BatchMat<T>) * cnt));
  HIPCHK(up(qr_off, qr.data(), sizeof(ChunkQRArgs<T>) * qr.size()));
  HIPCHK(up(lq_off, lq.data(), sizeof(ChunkQRArgs<T>) * lq.size()));
  HIPCHK(up(uq_off, uq.data(), sizeof(LarfbArgs<T>) * uq.size()));
  HIPCHK(up(ul_off, ul.data(), sizeof(LarfbArgs<T>) * ul.size()));
  HIPCHK(up(ch_off, ch.data(), sizeof(ChaseArgs) * cnt));
  HIPCHK(up(ord_off, order.data(), sizeof(int) * order.size()));
  HIPCHK(up(vmat_off, vmat.data(), sizeof(int) * vmat.size()));
  HIPCHK(up(voff_off, voff.data(), sizeof(int64_t) * cnt));
  P.mats_host.assign((const char*)mats.data(), (const char*)mats.data() + sizeof(BatchMat<T>) * cnt);

  // ---- the launch sequence ----
  const int nw = cfg.threads / 64, ib = cfg.inner_block, prec = cfg.update_precision;
  const int hp = prec != 0 ? 1 : 0;  // panels in float64 arithmetic when the updates run in BF16/FP16
  ChaseArgs L{};
  L.b = b;
  L.W = W;
  L.ldb = 3 * b;
  L.tab = (const ChaseArgs*)(base + ch_off);
  L.order = (const int*)(base + ord_off);
  L.ticket = ticket;
  L.total = (int32_t)total_groups;
  L.err = err;
  const int grid = std::max(1, chase_grid((int)std::max<int64_t>(1, total_groups), b, W));
  const size_t mats_off = P.mats_off;
  P.record = [=](hipStream_t st) -> int {
    const BatchMat<T>* dmats = (const BatchMat<T>*)(base + mats_off);
    HIPCHK(launch_stage_in_batched<T>(dmats, cnt, (unsigned long long*)(base + amax_off), maxM * maxN, st));
    for (int64_t k = 0; k < steps; ++k) {
      HIPCHK(launch_chunk_qr_batched<T>(b, (const ChunkQRArgs<T>*)(base + qr_off) + k * cnt, n_qr[k], hp, st));
      HIPCHK(launch_larfb_batched<T>(b, nw, ib, prec, vec_qr[k], (const LarfbArgs<T>*)(base + uq_off) + k * cnt,
                                     n_qr[k], mc_qr[k], lo_qr[k], hi_qr[k], st));
      if (n_lq[k] > 0) {
        HIPCHK(launch_chunk_qr_batched<T>(b, (const ChunkQRArgs<T>*)(base + lq_off) + k * cnt, n_lq[k], hp, st));
        HIPCHK(launch_larfb_batched<T>(b, nw, ib, prec, vec_lq[k], (const LarfbArgs<T>*)(base + ul_off) + k * cnt,
                                       n_lq[k], mc_lq[k], lo_lq[k], hi_lq[k], st));
      }
    }
    HIPCHK(launch_band_pack_batched<T>(dmats, cnt, b, maxN, st));
    HIPCHK(launch_chase_batched(L, grid, cnt, maxN, progress, nprog + 2, st));
    HIPCHK(launch_bisect_batched<T>(dmats, cnt, (const int*)(base + vmat_off), (const int64_t*)(base + voff_off),
                                    total_vals, maxN, st, err));
    return SVDV_OK;
  };
  return SVDV_OK;
}

// Stream on which batched graphs are captured (the caller's stream may be the
// legacy default stream, which cannot be captured); one per device, default priority.
int capture_stream(hipStream_t* out) {
  static std::map<int, hipStream_t> streams;
  int dev = 0;
  HIPCHK(hipGetDevice(&dev));
  hipStream_t& s = streams[dev];
  if (!s) HIPCHK(hipStreamCreateWithFlags(&s, hipStreamNonBlocking));
  *out = s;
  return SVDV_OK;
}

template <typename T>
int batched_run(BatchPlan& P, const void* const* A_array, void* S, hipStream_t st) {
  if (!P.exec) {
    // tables first (plain copies), then the launch sequence recorded into a graph
    int rc = batched_build<T>(P, A_array, S);
    if (rc) return rc;
    hipStream_t cs = nullptr;
    rc = capture_stream(&cs);
    if (rc) return rc;
    HIPCHK(hipStreamBeginCapture(cs, hipStreamCaptureModeRelaxed));
    rc = P.record(cs);
    hipGraph_t g = nullptr;
    hipError_t ce = hipStreamEndCapture(cs, &g);
    if (rc) {
      if (g) hipGraphDestroy(g);
      return rc;
    }
    HIPCHK(ce);
    P.graph = g;
    HIPCHK(hipGraphInstantiate(&P.exec, P.graph, nullptr, nullptr, 0));
  } else {
    // same shapes: refresh the input / output pointers of the matrix table if they changed
    const int cnt = (int)P.idx.size();
    std::vector<BatchMat<T>> mats(cnt);
    std::memcpy(mats.data(), P.mats_host.data(), sizeof(BatchMat<T>) * cnt);
    bool changed = false;
    for (int i = 0; i < cnt; ++i) {
      const int q = P.idx[i];
      const T* a = (const T*)A_array[q];
      T* s = (T*)S + P.soff[q];
      if (mats[i].A != a || mats[i].S != s) {
        mats[i].A = a;
        mats[i].S = s;
        changed = true;
      }
    }
    if (changed) {
      HIPCHK(hipStreamSynchronize(st));  // earlier replays may still read the table
      HIPCHK(hipMemcpy(P.mem + P.mats_off, mats.data(), sizeof(BatchMat<T>) * cnt, hipMemcpyHostToDevice));
      P.mats_host.assign((const char*)mats.data(), (const char*)mats.data() + sizeof(BatchMat<T>) * cnt);
    }
  }
  HIPCHK(hipGraphLaunch(P.exec, st));
  return SVDV_OK;
}

}  // namespace

namespace svdv {
// Records an error detail for svdv_last_error (used by the other source files).
int report_error(int status, const char* msg) { return fail(status, msg); }
}  // namespace svdv

// ============================================================================
// C ABI
// ============================================================================

extern "C" {

const char* svdv_status_string(int status) {
  switch (status) {
    case SVDV_OK: return "SVDV_OK";
    case SVDV_ERR_INVALID_ARG: return "SVDV_ERR_INVALID_ARG";
    case SVDV_ERR_UNSUPPORTED: return "SVDV_ERR_UNSUPPORTED";
    case SVDV_ERR_NO_MEMORY: return "SVDV_ERR_NO_MEMORY";
    case SVDV_ERR_HIP: return "SVDV_ERR_HIP";
  }
  return "unknown svdv status";
}

const char* svdv_last_error(void) { return g_last_error.c_str(); }

int svdv_default_config(int64_t m, int64_t n, int32_t dtype, svdv_config* out) {
  if (!out) return fail(SVDV_ERR_INVALID_ARG, "out is NULL");
  if (dtype != SVDV_F32 && dtype != SVDV_F64) return fail(SVDV_ERR_INVALID_ARG, "dtype must be SVDV_F32 or SVDV_F64");
  *out = default_config(m, n, dtype);
  return SVDV_OK;
}

int svdv_check_config(int64_t m, int64_t n, int32_t dtype, const svdv_config* cfg) {
  if (!cfg) return fail(SVDV_ERR_INVALID_ARG, "cfg is NULL");
  return check_config_impl(m, n, dtype, *cfg);
}

int svd_values_ex(const void* A, int64_t m, int64_t n, int64_t lda, int32_t dtype, void* S, void* stream,
                  const svdv_config* cfg) {
  int rc = check_matrix_args(A, m, n, lda, dtype);
  if (rc) return rc;
  const int64_t k = std::min(m, n);
  if (k == 0) return SVDV_OK;
  if (!S) return fail(SVDV_ERR_INVALID_ARG, "S is NULL");
  svdv_config c = cfg ? *cfg : default_config(m, n, dtype);
  rc = check_config_impl(m, n, dtype, c);
  if (rc) return rc;
  hipStream_t st = (hipStream_t)stream;
  if (dtype == SVDV_F32)
    return svd_values_t<float>((const float*)A, m, n, lda, (float*)S, st, c, nullptr, 0, nullptr, nullptr);
  return svd_values_t<double>((const double*)A, m, n, lda, (double*)S, st, c, nullptr, 0, nullptr, nullptr);
}

int svd_values(const void* A, int64_t m, int64_t n, int64_t lda, int32_t dtype, void* S, void* stream) {
  return svd_values_ex(A, m, n, lda, dtype, S, stream, nullptr);
}

int svd_values_noalloc(const void* A, int64_t m, int64_t n, int64_t lda, int32_t dtype, void* S, void* stream,
                       const svdv_config* cfg) {
  int rc = check_matrix_args(A, m, n, lda, dtype);
  if (rc) return rc;
  const int64_t k = std::min(m, n);
  if (k == 0) return SVDV_OK;
  if (!S) return fail(SVDV_ERR_INVALID_ARG, "S is NULL");
  svdv_config c = cfg ? *cfg : default_config(m, n, dtype);
  rc = check_config_impl(m, n, dtype, c);
  if (rc) return rc;
  char* ws = nullptr;
  rc = scratch_address(&ws);
  if (rc) return rc;
  hipStream_t st = (hipStream_t)stream;
  // no event creation on this path: per-stage timing is left off for the call
  const bool timing = g_timing.enabled;
  g_timing.enabled = false;
  if (dtype == SVDV_F32)
    rc = svd_values_t<float>((const float*)A, m, n, lda, (float*)S, st, c, nullptr, 0, nullptr, nullptr, ws,
                             kNoallocBytes);
  else
    rc = svd_values_t<double>((const double*)A, m, n, lda, (double*)S, st, c, nullptr, 0, nullptr, nullptr, ws,
                              kNoallocBytes);
  g_timing.enabled = timing;
  return rc;
}

int64_t svdv_noalloc_capacity(void) { return (int64_t)kNoallocBytes; }

int svdv_stage_band(const void* A, int64_t m, int64_t n, int64_t lda, int32_t dtype, double* band, int64_t ldband,
                    void* stream, const svdv_config* cfg) {
  int rc = check_matrix_args(A, m, n, lda, dtype);
  if (rc) return rc;
  const int64_t k = std::min(m, n);
  if (k == 0) return SVDV_OK;
  svdv_config c = cfg ? *cfg : default_config(m, n, dtype);
  rc = check_config_impl(m, n, dtype, c);
  if (rc) return rc;
  if (!band) return fail(SVDV_ERR_INVALID_ARG, "band is NULL");
  if (ldband < c.tile + 1) return fail(SVDV_ERR_INVALID_ARG, "ldband must be >= tile + 1");
  hipStream_t st = (hipStream_t)stream;
  if (dtype == SVDV_F32)
    return svd_values_t<float>((const float*)A, m, n, lda, nullptr, st, c, band, ldband, nullptr, nullptr);
  return svd_values_t<double>((const double*)A, m, n, lda, nullptr, st, c, band, ldband, nullptr, nullptr);
}

int svdv_stage_bidiag(const double* band, int64_t n, int64_t b, int64_t ldband, double* d, double* e, void* stream,
                      const svdv_config* cfg) {
  if (n < 0) return fail(SVDV_ERR_INVALID_ARG, "n must be >= 0");
  if (n == 0) return SVDV_OK;
  if (!band || !d || (n > 1 && !e)) return fail(SVDV_ERR_INVALID_ARG, "NULL pointer");
  if (!(b == 16 || b == 32 || b == 64 || b == 128)) return fail(SVDV_ERR_UNSUPPORTED, "b must be 16, 32, 64 or 128");
  if (ldband < b + 1) return fail(SVDV_ERR_INVALID_ARG, "ldband must be >= b + 1");
  svdv_config c = cfg ? *cfg : default_config(n, n, SVDV_F64);
  c.tile = (int32_t)b;
  if (c.sweep_width < 1 || c.sweep_width > 8) return fail(SVDV_ERR_UNSUPPORTED, "sweep_width must be in 1..8");
  if (chase_lds_bytes((int)b, c.sweep_width) > 160 * 1024 - 1024)
    return fail(SVDV_ERR_UNSUPPORTED, "bulge-chase LDS exceeds 160 KiB for this b and sweep width");
  hipStream_t st = (hipStream_t)stream;
  Layout L = make_layout(n, n, 8, (int)b, 256, c.sweep_width, n);
  char* ws = nullptr;
  int rc = get_workspace(st, L.total, &ws);
  if (rc) return rc;
  double* Bs = (double*)(ws + L.Bs);
  int* err = (int*)(ws + L.err);
  hipLaunchKernelGGL(k_fill_i32, dim3(1), dim3(64), 0, st, err, 0, (int64_t)1);
  HIPCHK(launch_band_import(band, ldband, n, (int)b, Bs, 3 * b, err, st));  // sets err for a non-finite band
  // the band as given may lie anywhere in the float64 range: scale it by a power of
  // two into [0.5, 1) (exact) and scale d and e back at the end
  int* expo = (int*)(ws + L.exp);
  HIPCHK(launch_band_scale(Bs, 3 * b, n, (unsigned long long*)(ws + L.amax), expo, st));
  ChaseArgs ca{};
  ca.Bs = Bs;
  ca.ldb = 3 * b;
  ca.n = n;
  ca.b = (int32_t)b;
  ca.W = c.sweep_width;
  ca.ngroups = (int32_t)std::max<int64_t>(1, (n - 1 + c.sweep_width - 1) / c.sweep_width);
  ca.progress = (int*)(ws + L.progress);
  ca.err = err;
  ca.d = d;
  ca.e = e ? e : (double*)(ws + L.e);
  int grid = chase_grid(ca.ngroups, (int)b, c.sweep_width);
  if (grid < 1) return fail(SVDV_ERR_UNSUPPORTED, "bulge-chase kernel cannot be resident with this configuration");
  HIPCHK(launch_chase(ca, grid, st));
  // a non-finite band, or a bounded wait that gave up (the chase unfinished): d and e
  // become NaN; otherwise they are scaled back
  hipLaunchKernelGGL(k_finish_de, dim3(std::max<int64_t>(1, std::min<int64_t>(1024, (n + 255) / 256))), dim3(256), 0,
                     st, ca.err, expo, d, ca.e, n);
  HIPCHK(hipGetLastError());
  return SVDV_OK;
}

int svdv_stage_values(const double* d, const double* e, int64_t n, int32_t out_dtype, void* S, void* stream) {
  if (n < 0) return fail(SVDV_ERR_INVALID_ARG, "n must be >= 0");
  if (out_dtype != SVDV_F32 && out_dtype != SVDV_F64) return fail(SVDV_ERR_INVALID_ARG, "bad out_dtype");
  if (n == 0) return SVDV_OK;
  if (!d || !S || (n > 1 && !e)) return fail(SVDV_ERR_INVALID_ARG, "NULL pointer");
  hipStream_t st = (hipStream_t)stream;
  Layout L = make_layout(n, n, 8, 16, 256, 1, n);
  char* ws = nullptr;
  int rc = get_workspace(st, L.total, &ws);
  if (rc) return rc;
  int* expo = (int*)(ws + L.exp);
  double* work = (double*)(ws + L.work);
  hipLaunchKernelGGL(k_fill_i32, dim3(1), dim3(64), 0, st, expo, 0, (int64_t)1);
  const double* ee = e ? e : d;  // n == 1: e is never read
  if (out_dtype == SVDV_F32) HIPCHK(launch_bisect<float>(d, ee, n, (float*)S, work, expo, 0, st));
  else HIPCHK(launch_bisect<double>(d, ee, n, (double*)S, work, expo, 0, st));
  return SVDV_OK;
}

int svdv_apply_qt(const void* V, int64_t ldv, const void* Tm, int64_t ldt, void* C, int64_t ldc, int64_t h, int64_t w,
                  int64_t k, int32_t dtype, int32_t side, void* stream, const svdv_config* cfg) {
  if (dtype != SVDV_F32 && dtype != SVDV_F64) return fail(SVDV_ERR_INVALID_ARG, "bad dtype");
  if (h < 0 || w < 0 || k < 0) return fail(SVDV_ERR_INVALID_ARG, "negative size");
  if (side != 0 && side != 1) return fail(SVDV_ERR_INVALID_ARG, "side must be 0 (left) or 1 (right)");
  if (h == 0 || w == 0 || k == 0) return SVDV_OK;
  if (!V || !Tm || !C) return fail(SVDV_ERR_INVALID_ARG, "NULL pointer");
  const int64_t vrows = side == 0 ? h : w;
  if (ldc < h || ldv < vrows || ldt < k) return fail(SVDV_ERR_INVALID_ARG, "leading dimension too small");
  if (k > vrows) return fail(SVDV_ERR_INVALID_ARG, "k exceeds the reflector length");
  svdv_config c = cfg ? *cfg : default_config(h, w, dtype);
  int rc = check_config_impl(h, w, dtype, c);
  if (rc) return rc;
  if (k > c.tile) return fail(SVDV_ERR_UNSUPPORTED, "k exceeds cfg->tile");
  const bool tall = vrows > 32768 / c.tile;
  // a tall panel runs split over row blocks when the register strip exists for this
  // configuration, else the streaming form
  const bool split = tall && (dtype == SVDV_F32 ? larfb_split_ok<float>(c.tile, c.threads / 64, c.inner_block)
                                                : larfb_split_ok<double>(c.tile, c.threads / 64, c.inner_block));
  const bool stream_ok = dtype == SVDV_F32 ? larfb_stream_valid<float>(c.tile / 16, c.inner_block, c.threads / 64)
                                            : larfb_stream_valid<double>(c.tile / 16, c.inner_block, c.threads / 64);
  if (tall && c.update_precision != 0)
    return fail(SVDV_ERR_UNSUPPORTED, "BF16/FP16 updates need a reflector length of at most 32768 / cfg->tile");
  if (tall && !split && !stream_ok)
    return fail(SVDV_ERR_UNSUPPORTED, "reflector length exceeds 32768 / cfg->tile, which this configuration "
                                      "(threads, inner_block) only handles in registers");
  hipStream_t st = (hipStream_t)stream;
  auto run = [&](auto* Cp, auto* Vp, auto* Tp) -> int {
    typedef std::remove_pointer_t<decltype(Cp)> T;
    LarfbArgs<T> a;
    a.M = side == 0 ? View<T>{Cp, 1, ldc} : View<T>{Cp, ldc, 1};
    a.rm = RowMap{0, 0, 0, 0};
    a.h = vrows;
    a.chunk_rows = vrows;
    a.P = 1;
    a.col0 = 0;
    a.col1 = side == 0 ? w : h;
    a.V = Vp;
    a.ldv = ldv;
    a.Tm = Tp;
    a.ldt = ldt;
    a.k = (int32_t)k;
    a.vec = larfb_vec_ok(a);
      a.vecv = larfb_vecv_ok(a);
    a.prec = c.update_precision;
    if (split) {
      const int64_t elems = larfb_split_work<T>(c.tile, c.threads / 64, c.inner_block, vrows, a.col1 - a.col0);
      char* ws = nullptr;
      const int wrc = get_workspace(st, (size_t)elems * sizeof(T), &ws);
      if (wrc) return wrc;
      HIPCHK(launch_larfb_split<T>(c.tile, c.threads / 64, c.inner_block, a, (T*)ws, st));
      return SVDV_OK;
    }
    HIPCHK(launch_larfb<T>(c.tile, c.threads / 64, c.inner_block, a, st));
    return SVDV_OK;
  };
  if (dtype == SVDV_F32) return run((float*)C, (const float*)V, (const float*)Tm);
  return run((double*)C, (const double*)V, (const double*)Tm);
}

}  // extern "C"

namespace {

// Streams (default priority, non-blocking) and events of the concurrent groups of a
// batch, created once per device and kept until the process ends.
int group_streams(int count, std::vector<hipStream_t>& out) {
  static std::mutex mu;
  static std::map<int, std::vector<hipStream_t>> pool;
  int dev = 0;
  HIPCHK(hipGetDevice(&dev));
  std::lock_guard<std::mutex> lk(mu);
  std::vector<hipStream_t>& v = pool[dev];
  while ((int)v.size() < count) {
    hipStream_t s = nullptr;
    HIPCHK(hipStreamCreateWithFlags(&s, hipStreamNonBlocking));
    v.push_back(s);
  }
  out.assign(v.begin(), v.begin() + count);
  return SVDV_OK;
}
int group_event(int i, hipEvent_t* out) {
  static std::mutex mu;
  static std::map<std::pair<int, int>, hipEvent_t> pool;
  int dev = 0;
  HIPCHK(hipGetDevice(&dev));
  std::lock_guard<std::mutex> lk(mu);
  hipEvent_t& e = pool[{dev, i}];
  if (!e) HIPCHK(hipEventCreateWithFlags(&e, hipEventDisableTiming));
  *out = e;
  return SVDV_OK;
}

// One batch (or one group of a batch) under one configuration.
int batched_with_config(const void* const* A_array, const int64_t* m, const int64_t* n, const int64_t* lda,
                        int64_t batch, int32_t dtype, void* S, const int64_t* S_offset, void* stream,
                        const svdv_config& c, int64_t maxdim) {
  const bool reg_ok = dtype == SVDV_F32 ? larfb_reg_valid<float>(c.tile / 16, c.inner_block, c.threads / 64)
                                        : larfb_reg_valid<double>(c.tile / 16, c.inner_block, c.threads / 64);
  const int hmax = dtype == SVDV_F32 ? chunk_qr_hmax<float>(c.tile) : chunk_qr_hmax<double>(c.tile);
  if (!reg_ok || maxdim > hmax) {
    // outside the batched kernels' reach (a strip that does not fit in registers, or
    // matrices taller than one panel chunk): the matrices run one after another
    const int es = elem_size(dtype);
    for (int64_t i = 0; i < batch; ++i) {
      const int rc = svd_values_ex(A_array[i], m[i], n[i], lda[i], dtype, (char*)S + S_offset[i] * es, stream, &c);
      if (rc) return rc;
    }
    return SVDV_OK;
  }
  int dev = 0;
  HIPCHK(hipGetDevice(&dev));
  std::lock_guard<std::mutex> lk(g_mu);
  BatchPlan& P = g_batch[BatchKey{dev, stream, c.tile, c.threads, c.inner_block, c.sweep_width, c.update_precision}];
  const std::vector<int64_t> mv(m, m + batch), nv(n, n + batch), lv(lda, lda + batch), ov(S_offset, S_offset + batch);
  const bool same = P.exec && P.dtype == dtype && std::memcmp(&P.cfg, &c, sizeof(c)) == 0 && P.m == mv && P.n == nv &&
                    P.lda == lv && P.soff == ov;
  if (!same) {
    if (P.exec || P.mem) HIPCHK(hipStreamSynchronize((hipStream_t)stream));
    P.release();
    P.bytes = 0;
    P.dtype = dtype;
    P.cfg = c;
    P.m = mv;
    P.n = nv;
    P.lda = lv;
    P.soff = ov;
    P.idx.clear();
    for (int64_t i = 0; i < batch; ++i)
      if (std::min(m[i], n[i]) > 0) P.idx.push_back((int)i);
    std::stable_sort(P.idx.begin(), P.idx.end(),
                     [&](int a, int b) { return std::min(m[a], n[a]) > std::min(m[b], n[b]); });
    if (P.idx.empty()) return SVDV_OK;
  }
  if (P.idx.empty()) return SVDV_OK;
  hipStream_t st = (hipStream_t)stream;
  if (dtype == SVDV_F32) return batched_run<float>(P, A_array, S, st);
  return batched_run<double>(P, A_array, S, st);
}

}  // namespace

extern "C" {

int svd_values_batched(const void* const* A_array, const int64_t* m, const int64_t* n, const int64_t* lda, int64_t batch,
                       int32_t dtype, void* S, const int64_t* S_offset, void* stream, const svdv_config* cfg) {
  if (batch < 0) return fail(SVDV_ERR_INVALID_ARG, "batch must be >= 0");
  if (batch == 0) return SVDV_OK;
  if (batch > (1 << 20)) return fail(SVDV_ERR_UNSUPPORTED, "batch above 2^20");
  if (!A_array || !m || !n || !lda || !S_offset || !S) return fail(SVDV_ERR_INVALID_ARG, "NULL pointer");
  int64_t maxdim = 1;
  for (int64_t i = 0; i < batch; ++i) {
    int rc = check_matrix_args(A_array[i], m[i], n[i], lda[i], dtype);
    if (rc) return rc;
    if (S_offset[i] < 0) return fail(SVDV_ERR_INVALID_ARG, "negative S_offset");
    maxdim = std::max<int64_t>(maxdim, std::max(m[i], n[i]));
  }
  if (cfg) {
    const int rc = check_config_impl(maxdim, maxdim, dtype, *cfg);
    if (rc) return rc;
    return batched_with_config(A_array, m, n, lda, batch, dtype, S, S_offset, stream, *cfg, maxdim);
  }
  // per-size tuned defaults: the matrices are grouped by the configuration the tuned
  // table gives their size, and each group runs as one batch (in order of first appearance)
  std::vector<svdv_config> cfgs;
  std::vector<std::vector<int64_t>> members;
  for (int64_t i = 0; i < batch; ++i) {
    svdv_config c = default_config(m[i], n[i], dtype);
    // a group runs in the batched kernels only with a register-strip update: keep the
    // tuned tile and sweep width, and take the widest such workgroup otherwise
    const bool reg = dtype == SVDV_F32 ? larfb_reg_valid<float>(c.tile / 16, c.inner_block, c.threads / 64)
                                       : larfb_reg_valid<double>(c.tile / 16, c.inner_block, c.threads / 64);
    if (!reg) {
      for (int th : {1024, 512, 256, 128}) {
        const bool ok = dtype == SVDV_F32 ? larfb_reg_valid<float>(c.tile / 16, 1, th / 64)
                                          : larfb_reg_valid<double>(c.tile / 16, 1, th / 64);
        if (ok) {
          c.threads = th;
          c.inner_block = 1;
          break;
        }
      }
    }
    size_t g = 0;
    while (g < cfgs.size() && std::memcmp(&cfgs[g], &c, sizeof(c)) != 0) ++g;
    if (g == cfgs.size()) {
      cfgs.push_back(c);
      members.emplace_back();
    }
    members[g].push_back(i);
  }
  // groups run concurrently: each on a stream of its own, forked from and joined
  // back to the caller's stream (one group runs on the caller's stream itself)
  hipStream_t st = (hipStream_t)stream;
  std::vector<hipStream_t> gst(cfgs.size(), st);
  if (cfgs.size() > 1) {
    int rc = group_streams((int)cfgs.size(), gst);
    if (rc) return rc;
    hipEvent_t fork = nullptr;
    rc = group_event(0, &fork);
    if (rc) return rc;
    HIPCHK(hipEventRecord(fork, st));
    for (size_t g = 0; g < cfgs.size(); ++g) HIPCHK(hipStreamWaitEvent(gst[g], fork, 0));
  }
  for (size_t g = 0; g < cfgs.size(); ++g) {
    const std::vector<int64_t>& ix = members[g];
    std::vector<const void*> a(ix.size());
    std::vector<int64_t> mm(ix.size()), nn(ix.size()), ll(ix.size()), oo(ix.size());
    int64_t gmax = 1;
    for (size_t q = 0; q < ix.size(); ++q) {
      a[q] = A_array[ix[q]];
      mm[q] = m[ix[q]];
      nn[q] = n[ix[q]];
      ll[q] = lda[ix[q]];
      oo[q] = S_offset[ix[q]];
      gmax = std::max<int64_t>(gmax, std::max(mm[q], nn[q]));
    }
    int rc = check_config_impl(gmax, gmax, dtype, cfgs[g]);
    if (rc) return rc;
    rc = batched_with_config(a.data(), mm.data(), nn.data(), ll.data(), (int64_t)ix.size(), dtype, S, oo.data(),
                             (void*)gst[g], cfgs[g], gmax);
    if (rc) return rc;
  }
  if (cfgs.size() > 1) {
    for (size_t g = 0; g < cfgs.size(); ++g) {
      hipEvent_t join = nullptr;
      int rc = group_event(1 + (int)g, &join);
      if (rc) return rc;
      HIPCHK(hipEventRecord(join, gst[g]));
      HIPCHK(hipStreamWaitEvent(st, join, 0));
    }
  }
  return SVDV_OK;
}

int svdv_timing(int enable) {
  g_timing.enabled = enable != 0;
  g_timing.kernels = enable >= 2;
  g_timing.valid = false;
  return SVDV_OK;
}

int svdv_last_timing(double* ms, int n) {
  if (!ms || n < 0) return fail(SVDV_ERR_INVALID_ARG, "bad output array");
  if (!g_timing.valid) return fail(SVDV_ERR_INVALID_ARG, "no timed call recorded (enable svdv_timing first)");
  HIPCHK(hipEventSynchronize(g_timing.ev[5]));
  int k = 0;
  for (int i = 0; i < 5 && k < n; ++i, ++k) {
    float t = 0.f;
    HIPCHK(hipEventElapsedTime(&t, g_timing.ev[i], g_timing.ev[i + 1]));
    ms[k] = t;
  }
  if (k < n) {
    float t = 0.f;
    HIPCHK(hipEventElapsedTime(&t, g_timing.ev[0], g_timing.ev[5]));
    ms[k++] = t;
  }
  if (k < n) {  // the bulge-chase launch itself, on its own stream
    float t = 0.f;
    HIPCHK(hipEventElapsedTime(&t, g_timing.cev[0], g_timing.cev[1]));
    ms[k++] = t;
  }
  return k;
}

int svdv_last_kernel_stats(int kind, double* out, int n) {
  if (!out || n < 4) return fail(SVDV_ERR_INVALID_ARG, "out needs 4 entries");
  if (kind != 0 && kind != 1) return fail(SVDV_ERR_INVALID_ARG, "kind must be 0 (trailing update) or 1 (panel)");
  if (!g_timing.valid) return fail(SVDV_ERR_INVALID_ARG, "no timed call recorded (enable svdv_timing first)");
  const KernelLog& L = g_timing.klog[kind];
  const size_t launches = L.flops.size();
  double ms = 0.0, fl = 0.0, by = 0.0;
  if (launches) HIPCHK(hipEventSynchronize(L.ev[2 * launches - 1]));
  for (size_t i = 0; i < launches; ++i) {
    float t = 0.f;
    HIPCHK(hipEventElapsedTime(&t, L.ev[2 * i], L.ev[2 * i + 1]));
    ms += t;
    fl += L.flops[i];
    by += L.bytes[i];
  }
  out[0] = (double)launches;
  out[1] = ms;
  out[2] = fl;
  out[3] = by;
  return 4;
}

int svdv_release(void) {
  std::lock_guard<std::mutex> lk(g_mu);
  for (auto& kv : g_ws) {
    if (kv.second.ptr) {
      hipSetDevice(kv.first.first);
      hipStreamSynchronize((hipStream_t)kv.first.second);
      hipFree(kv.second.ptr);
    }
  }
  g_ws.clear();
  for (auto& kv : g_batch) {
    hipSetDevice(kv.first.dev);
    hipStreamSynchronize((hipStream_t)kv.first.stream);
    kv.second.release();
  }
  g_batch.clear();
  for (auto& kv : g_side) {
    hipSetDevice(kv.first.first);
    hipStreamSynchronize(kv.second.s);
    for (auto& e : kv.second.ev) hipEventDestroy(e);
    hipStreamDestroy(kv.second.s);
  }
  g_side.clear();
  return SVDV_OK;
}

}  // extern "C"
