// Stage 2: upper band (bandwidth b) -> upper bidiagonal by Householder bulge
// chasing.  The paper names this step only ("finally to bidiagonal"); the
// reading taken here: sweep s makes row s bidiagonal and chases the bulge it
// creates down the band.  A sweep is a chain of tasks (p, c):
//   right reflector on columns c..c+L-1 annihilating row p beyond column c,
//   applied to rows p..c+L-1 (this creates fill below the diagonal);
//   left reflector on rows c..c+L-1 annihilating column c below the diagonal,
//   applied to columns c..c+L+b-1 (this creates fill beyond the band);
// with p_0 = s, c_0 = s+1, then p <- c, c <- c+b, and L = min(b, n-c).
//
// Dependencies: task j of sweep s+1 overlaps tasks j and j+1 of sweep s in
// whole rows and columns, and task j+2 in a single element; tasks further apart
// are disjoint.  So a sweep may start task j once its predecessor has finished
// task j+1 (and written the one element task j+2 shares with it), and any
// schedule obeying that gives bitwise the same result.
//
// Kernels: b = 16 runs k_chase_flow (lag-2 schedule, LDS window, loader and
// storer waves, no per-step barrier); b = 32 runs the windowed k_chase_win
// (lag 3, one barrier per step); larger b the direct k_chase.  In all of them a
// persistent grid takes groups of W consecutive sweeps in increasing order from
// a ticket counter, so the predecessor of every group being worked on is held by
// a workgroup that is already running: no schedule can wait on a workgroup that
// was never made resident, whatever the occupancy.  Group g waits for group
// g-1's last sweep through a progress counter.  Band data crosses workgroups
// (and XCDs, whose L2 caches are not coherent with each other) only as
// device-scope accesses (coherent at device level), and progress is published
// only after the stores it covers have completed.
#include "common.hpp"
#include "kernels.hpp"

namespace svdv {

// Optional step trace of one group (diagnostic builds only, -DSVDV_CHASE_TRACE,
// group SVDV_TRACE_GROUP, default 0): eight timestamps per step of the 100 MHz
// real-time counter.
#ifdef SVDV_CHASE_TRACE
#ifndef SVDV_TRACE_GROUP
#define SVDV_TRACE_GROUP 0
#endif
__device__ uint64_t g_chase_trace[8 * 1024];
#define CHASE_MARK_IF(cond, gi, t, k)                                          \
  do {                                                                         \
    if ((cond) && (gi) == SVDV_TRACE_GROUP && (t) < 1024)                      \
      g_chase_trace[(t) * 8 + (k)] = __builtin_amdgcn_s_memrealtime();         \
  } while (0)
#else
#define CHASE_MARK_IF(cond, gi, t, k) \
  do {                                \
  } while (0)
#endif
#define CHASE_MARK(gi, t, k) CHASE_MARK_IF(threadIdx.x == 0, gi, t, k)

__device__ __forceinline__ double bld(const double* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void bst(double* p, double v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

struct ChaseCtx {
  double* Bs;
  int64_t ldb;
  int64_t n;
  int b;
  int LO;
  __device__ __forceinline__ double* at(int64_t i, int64_t j) const { return Bs + i * ldb + (j - i + LO); }
};

// One task, executed by one wave.  tile: LDS scratch of 64*(b+1) doubles; vb: b doubles.
__device__ void chase_task(const ChaseCtx& X, int64_t p, int64_t c, double* tile, double* vb) {
  const int lane = threadIdx.x & 63;
  const int b = X.b;
  const int L = (int)((X.n - c) < b ? (X.n - c) : b);
  const int64_t rend = c + L < X.n ? c + L : X.n;
  const int64_t cend = c + L + b < X.n ? c + L + b : X.n;
  const int ldt = b + 1;

  // ---------------- right reflector: row p, columns c .. c+L-1 ----------------
  for (int half = 0; half * 64 < L; ++half) {
    const int l = half * 64 + lane;
    double xl = l < L ? bld(X.at(p, c + l)) : 0.0;
    tile[l] = xl;  // temporary: x in tile[0..L)
  }
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  double tau, beta, scal;
  {
    // norm over up to 128 elements: each lane sums its (up to 2) tail entries
    double ss = 0.0;
    for (int half = 0; half * 64 < L; ++half) {
      const int l = half * 64 + lane;
      if (l >= 1 && l < L) ss += tile[l] * tile[l];
    }
    ss = wave_sum(ss);
    const double alpha = tile[0];
    beta = alpha;
    scal = 0.0;
    tau = 0.0;
    if (ss > 0.0) {
      const double nrm = sqrt(alpha * alpha + ss);
      beta = alpha >= 0.0 ? -nrm : nrm;
      scal = nr_div(1.0, alpha - beta);  // divisors >= sqrt(ss), normal whenever ss > 0
      tau = nr_div(beta - alpha, beta);
    }
  }
  for (int half = 0; half * 64 < L; ++half) {
    const int l = half * 64 + lane;
    if (l < L) {
      vb[l] = l == 0 ? 1.0 : tile[l] * scal;
      bst(X.at(p, c + l), l == 0 ? beta : 0.0);
    }
  }
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  if (tau != 0.0) {
    for (int64_t r0 = p + 1; r0 < rend; r0 += 64) {
      const int nr = (int)((rend - r0) < 64 ? (rend - r0) : 64);
      for (int e = lane; e < nr * L; e += 64) {
        const int rr = e / L, l = e - rr * L;
        tile[rr * ldt + l] = bld(X.at(r0 + rr, c + l));
      }
      __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
      if (lane < nr) {
        double dot = 0.0;
        for (int l = 0; l < L; ++l) dot += tile[lane * ldt + l] * vb[l];
        const double td = tau * dot;
        for (int l = 0; l < L; ++l) tile[lane * ldt + l] -= td * vb[l];
      }
      __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
      for (int e = lane; e < nr * L; e += 64) {
        const int rr = e / L, l = e - rr * L;
        bst(X.at(r0 + rr, c + l), tile[rr * ldt + l]);
      }
      __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    }
  }

  // ---------------- left reflector: column c, rows c .. c+L-1 ----------------
  for (int half = 0; half * 64 < L; ++half) {
    const int l = half * 64 + lane;
    tile[l] = l < L ? bld(X.at(c + l, c)) : 0.0;
  }
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  {
    double ss = 0.0;
    for (int half = 0; half * 64 < L; ++half) {
      const int l = half * 64 + lane;
      if (l >= 1 && l < L) ss += tile[l] * tile[l];
    }
    ss = wave_sum(ss);
    const double alpha = tile[0];
    beta = alpha;
    scal = 0.0;
    tau = 0.0;
    if (ss > 0.0) {
      const double nrm = sqrt(alpha * alpha + ss);
      beta = alpha >= 0.0 ? -nrm : nrm;
      scal = nr_div(1.0, alpha - beta);  // divisors >= sqrt(ss), normal whenever ss > 0
      tau = nr_div(beta - alpha, beta);
    }
  }
  for (int half = 0; half * 64 < L; ++half) {
    const int l = half * 64 + lane;
    if (l < L) {
      vb[l] = l == 0 ? 1.0 : tile[l] * scal;
      bst(X.at(c + l, c), l == 0 ? beta : 0.0);
    }
  }
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  if (tau != 0.0) {
    const int ldc = 65;
    for (int64_t q0 = c + 1; q0 < cend; q0 += 64) {
      const int nq = (int)((cend - q0) < 64 ? (cend - q0) : 64);
      for (int e = lane; e < nq * L; e += 64) {
        const int l = e / nq, qq = e - l * nq;
        tile[l * ldc + qq] = bld(X.at(c + l, q0 + qq));
      }
      __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
      if (lane < nq) {
        double dot = 0.0;
        for (int l = 0; l < L; ++l) dot += vb[l] * tile[l * ldc + lane];
        const double td = tau * dot;
        for (int l = 0; l < L; ++l) tile[l * ldc + lane] -= td * vb[l];
      }
      __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
      for (int e = lane; e < nq * L; e += 64) {
        const int l = e / nq, qq = e - l * nq;
        bst(X.at(c + l, q0 + qq), tile[l * ldc + qq]);
      }
      __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    }
  }
}

// Next group for this workgroup: a ticket from the launch's counter (zeroed
// before the launch), mapped to (matrix, group) by the order table of a batched
// launch (tickets of one matrix's groups are increasing, so every predecessor
// holds a smaller ticket), or to group = ticket for one matrix.  Every thread
// gets the same result; gi < 0 when no group is left.
__device__ __forceinline__ ChaseArgs take_group(const ChaseArgs& L, int& gi) {
  __shared__ int s_ticket;
  if (threadIdx.x == 0) s_ticket = atomicAdd(L.ticket, 1);
  __syncthreads();
  const int tk = __builtin_amdgcn_readfirstlane(s_ticket);  // uniform: keep the schedule scalar
  __syncthreads();
  if (tk >= L.total) {
    gi = -1;
    return L;
  }
  if (L.order == nullptr) {
    gi = tk;
    return L;
  }
  gi = L.order[2 * tk + 1];
  return L.tab[L.order[2 * tk]];
}

__device__ __forceinline__ int ntasks_of(int64_t s, int64_t n, int b) {
  if (s >= n - 1) return 0;
  return (int)((n - 1 - s + b - 1) / b);
}

template <int B>
__device__ __forceinline__ int ntasks_b(int64_t s, int64_t n) {
  const int r = (int)(n - 1 - s);
  return r > 0 ? (r + B - 1) / B : 0;
}

size_t chase_lds_bytes(int b, int W) {
  // per wave: a 64 x (b+1) tile (also used as b x 65 for the left part) + b reflector entries
  const int tile = 64 * (b + 1) > b * 65 ? 64 * (b + 1) : b * 65;
  return (size_t)W * (tile + b) * sizeof(double);
}

__global__ void k_chase(ChaseArgs L) {
  extern __shared__ __align__(16) double lds[];
  const int wv = threadIdx.x >> 6;
  const int W = L.W;
  const int b = L.b;
  const int tile_elems = 64 * (b + 1) > b * 65 ? 64 * (b + 1) : b * 65;
  double* tile = lds + (size_t)wv * (tile_elems + b);
  double* vb = tile + tile_elems;
  __shared__ int s_giveup;

  for (;;) {
    int gi;
    const ChaseArgs a = take_group(L, gi);
    if (gi < 0) break;
    const int64_t n = a.n;
    const ChaseCtx X{a.Bs, a.ldb, a.n, b, b - 1};
    const int64_t s0 = (int64_t)gi * W;
    const int nsw = (int)((n - 1 - s0) < W ? (n - 1 - s0) : W);
    int tend = 0;
    for (int i = 0; i < nsw; ++i) {
      const int te = 3 * i + ntasks_of(s0 + i, n, b);
      tend = te > tend ? te : tend;
    }
    const int prev_total = gi > 0 ? ntasks_of(s0 - 1, n, b) : 0;
    const int last_total = ntasks_of(s0 + nsw - 1, n, b);
    int known = gi > 0 ? 0 : 1 << 30;  // cached progress of the previous group (thread 0)
    if (threadIdx.x == 0) s_giveup = 0;
    __syncthreads();
    for (int t = 0; t < tend; ++t) {
      if (gi > 0 && threadIdx.x == 0) {
        const int need = (t + 3) < prev_total ? (t + 3) : prev_total;
        if (known < need) {
          const uint64_t t0 = __builtin_amdgcn_s_memrealtime();
          while (true) {
            known = __hip_atomic_load(&a.progress[gi - 1], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            if (known >= need) break;
            if (__builtin_amdgcn_s_memrealtime() - t0 > 1000000000ull ||  // 10 s at 100 MHz
                __hip_atomic_load(a.err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0) {
              atomicAdd(a.err, 1);
              s_giveup = 1;
              break;
            }
            __builtin_amdgcn_s_sleep(1);
          }
        }
      }
      __syncthreads();
      if (s_giveup) break;
      if (wv < nsw) {
        const int64_t s = s0 + wv;
        const int jt = t - 3 * wv;
        if (jt >= 0 && jt < ntasks_of(s, n, b)) {
          const int64_t c = s + 1 + (int64_t)jt * b;
          const int64_t p = jt == 0 ? s : c - b;
          chase_task(X, p, c, tile, vb);
        }
      }
      __builtin_amdgcn_s_waitcnt(0);
      __syncthreads();
      if (threadIdx.x == 0) {
        int done = t - 3 * (nsw - 1) + 1;
        done = done < 0 ? 0 : (done > last_total ? last_total : done);
        __hip_atomic_store(&a.progress[gi], done, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      }
    }
    if (threadIdx.x == 0)
      __hip_atomic_store(&a.progress[gi], last_total, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// Windowed chase (b = 32): the rows a group is working on live in LDS.
// ---------------------------------------------------------------------------
//
// The group's rows form a sliding window kept in an LDS ring buffer (row r in
// slot r mod R, each slot one band row of 3b entries).  Per step: rows the
// group's first sweep needs at the next step are loaded from global memory
// while the current step computes (prefetch distance 1), every wave runs its
// task entirely in LDS, and rows no unfinished sweep of the group will touch
// again are written back.  Global memory is therefore off the critical path
// except for the hand-off between consecutive groups, which is ordered by the
// progress counter (published after the write-back stores completed).

template <int B>
struct WinGeom {
  static constexpr int LO = B - 1;
  static constexpr int RW = 3 * B;      // entries of a band row (global and LDS)
  static constexpr int RS = 3 * B + 2;  // LDS slot stride (see win_task)
  // the windowed kernel always runs at least 4 waves (the extra ones only move rows)
  static constexpr int MIN_WAVES = 4;
  static constexpr int PF = (B * RW + 64 * MIN_WAVES - 1) / (64 * MIN_WAVES);  // prefetch registers per thread
};

__host__ __device__ inline int win_rows(int b, int W) { return (3 * W + 2) * b + 2; }

size_t chase_win_lds_bytes(int b, int W) {
  if (b != 16 && b != 32) return (size_t)1 << 40;
  return ((size_t)(win_rows(b, W) + 1) * (3 * b + 2) + (size_t)16 * b) * sizeof(double);  // ring + zero slot + reflector slots
}

// Ring slot of row r: (r - base) mod R (base <= every row the window holds;
// the difference is below 2^31).  Column j of row r sits at offset j - r + (B-1)
// of the slot.
__device__ __forceinline__ int ring_slot(int64_t r, int64_t base, int R) {
  return (int)((uint32_t)(r - base) % (uint32_t)R);
}

// Householder reflector H = I - tau v v^T with H x = beta e_1, for the vector x
// held one entry per lane (lanes >= L hold 0).  v is returned per lane (v_0 = 1,
// zero beyond L); x = 0 below its first entry gives tau = 0 (H = I).
template <int B>
__device__ __forceinline__ void wave_reflector(double x, int lane, int L, double& beta, double& tau, double& v) {
  const double sq = (lane >= 1 && lane < L) ? x * x : 0.0;  // L <= B: only the first B lanes contribute
  const double ss = B <= 16 ? row_sum16(sq) : row_sum32(sq);
  const double alpha = lane_value(x, 0);
  double scal = 0.0;
  beta = alpha;
  tau = 0.0;
  if (ss > 0.0) {
    const double nrm = sqrt(alpha * alpha + ss);
    beta = alpha >= 0.0 ? -nrm : nrm;
    scal = nr_div(1.0, alpha - beta);  // divisors >= sqrt(ss), normal whenever ss > 0
    tau = nr_div(beta - alpha, beta);
  }
  v = lane < L ? (lane == 0 ? 1.0 : x * scal) : 0.0;
}

// One task (p, c) on the window, executed by one wave.  Every lane loads its
// whole row (right update) or column (left update) into registers before the
// reflector is formed, so those loads overlap the reduction; the reflector
// entries then go through the wave's LDS slot `vbw` (B doubles) and come back
// to every lane as wide broadcast reads.  The loops run over all B entries
// whatever L is: the reflector is zero beyond L, the right update then reads
// and rewrites band positions past column n (zeros), and the left update reads
// rows past n from the zero slot `zs` (a slot kept at zero), so no entry
// changes and no loop needs a branch.  The slot stride is 3B+2: a column of the
// band walks the slots with stride 3B+1 (odd), which spreads the lanes of the
// right update over distinct banks.  LDS operations of one wave complete in
// order, so each phase sees the previous phase's stores.
template <int B>
__device__ __forceinline__ void win_task(lds_f64* win, lds_f64* vbw, int R, int zs, int64_t base, int64_t n, int64_t p,
                                         int64_t c) {
  constexpr int RS = WinGeom<B>::RS, LO = WinGeom<B>::LO;
  // the reflector comes back through LDS (B = 16) or lane reads into scalar
  // registers (B = 32, where vector registers would not hold it beside the row)
  constexpr bool kVrLds = B <= 16;
  const int lane = threadIdx.x & 63;
  const int L = (int)((n - c) < B ? (n - c) : B);
  const int nr = (int)(c + L - p - 1);                              // rows p+1 .. c+L-1
  const int nq = (int)((c + L + B < n ? c + L + B : n) - c - 1);   // columns c+1 .. min(c+L+B, n)-1
  const int sp = ring_slot(p, base, R), sc = ring_slot(c, base, R);
  const int dc = (int)(c - p);

  // ---- right reflector on row p, columns c..c+L-1 (element (p, c+l) at rowp[l]) ----
  lds_f64* rowp = win + sp * RS + (dc + LO);
  double x = lane < L ? rowp[lane] : 0.0;
  // lanes past the last row read (and later leave alone) row p+1, so the loads
  // need no branch and overlap the reduction below
  const int lr = lane < nr ? lane : 0;
  int sr = sp + 1 + lr;
  sr = sr >= R ? sr - R : sr;
  lds_f64* row = win + sr * RS + (dc - 1 - lr + LO);  // element (p+1+lr, c+l) at row[l]
  double xr[B];
#pragma unroll
  for (int l = 0; l < B; ++l) xr[l] = row[l];
  double beta, tau, v;
  wave_reflector<B>(x, lane, L, beta, tau, v);
  if (lane < L) rowp[lane] = lane == 0 ? beta : 0.0;
  if (kVrLds && lane < B) vbw[lane] = v;
  double vr[B];
  auto vget = [&](int l) -> double { return vr[l]; };
  auto vfetch = [&]() {
#pragma unroll
    for (int l = 0; l < B; ++l) vr[l] = kVrLds ? vbw[l] : lane_value(v, l);
  };
  if (tau != 0.0) {
    vfetch();
    if (lane < nr) {
      double dot = 0.0;
#pragma unroll
      for (int l = 0; l < B; ++l) dot += xr[l] * vget(l);
      const double td = tau * dot;
#pragma unroll
      for (int l = 0; l < B; ++l) row[l] = xr[l] - td * vget(l);
    }
  }

  // ---- left reflector on column c, rows c..c+L-1 (element (c+l, c) at slot(c+l), offset LO-l) ----
  int sx = sc + lane;
  sx = sx >= R ? sx - R : sx;
  x = lane < L ? win[sx * RS + LO - lane] : 0.0;
  int so[B];     // slot of row c+l (the zero slot past row n-1)
  double xc[B];  // element (c+l, c+1+lane) at offset 1+lane-l+LO of that slot
#pragma unroll
  for (int l = 0; l < B; ++l) {
    int sl = sc + l;
    sl = sl >= R ? sl - R : sl;
    so[l] = l < L ? sl : zs;
  }
  const int lq = lane < nq ? lane : 0;  // as above: lanes past the last column read column c+1
#pragma unroll
  for (int l = 0; l < B; ++l) xc[l] = win[so[l] * RS + 1 + lq - l + LO];
  wave_reflector<B>(x, lane, L, beta, tau, v);
  if (lane < L) win[sx * RS + LO - lane] = lane == 0 ? beta : 0.0;
  if (kVrLds && lane < B) vbw[lane] = v;
  if (tau != 0.0) {
    vfetch();
    if (lane < nq) {
      double dot = 0.0;
#pragma unroll
      for (int l = 0; l < B; ++l) dot += vget(l) * xc[l];
      const double td = tau * dot;
#pragma unroll
      for (int l = 0; l < B; ++l) win[so[l] * RS + 1 + lane - l + LO] = xc[l] - td * vget(l);
    }
  }
}

// First row the (unfinished) sweep s0+i will touch at its task j (j <= 0: it has not started).
__device__ __forceinline__ int64_t sweep_front(int64_t s, int j, int b) {
  return j <= 0 ? s : s + 1 + (int64_t)(j - 1) * b;
}

template <int B>
__global__ void __launch_bounds__(512) k_chase_win(ChaseArgs L) {
  constexpr int RW = WinGeom<B>::RW, RS = WinGeom<B>::RS, PF = WinGeom<B>::PF;
  extern __shared__ __align__(16) double lds[];
  const int W = L.W;
  const int R = win_rows(B, W);
  lds_f64* win = (lds_f64*)lds;
  for (int e = threadIdx.x; e < RS; e += blockDim.x) win[R * RS + e] = 0.0;  // zero slot
  const int wv = threadIdx.x >> 6;
  const int nthr = blockDim.x;
  const int tid = threadIdx.x;
  __shared__ int s_giveup;

  for (;;) {
    int gi;
    const ChaseArgs a = take_group(L, gi);
    if (gi < 0) break;
    const int64_t n = a.n;
    const int64_t s0 = (int64_t)gi * W;
    const int nsw = (int)((n - 1 - s0) < W ? (n - 1 - s0) : W);
    int tend = 0;
    for (int i = 0; i < nsw; ++i) {
      const int te = 3 * i + ntasks_b<B>(s0 + i, n);
      tend = te > tend ? te : tend;
    }
    const int prev_total = gi > 0 ? ntasks_b<B>(s0 - 1, n) : 0;
    const int last_total = ntasks_b<B>(s0 + nsw - 1, n);
    const int first_total = ntasks_b<B>(s0, n);
    // rows the group's first sweep needs up to (and including) step t: [s0, front_end(t))
    auto front_end = [&](int t) -> int64_t {
      const int tt = t < first_total - 1 ? t : first_total - 1;
      const int64_t e = s0 + 1 + (int64_t)(tt + 1) * B;
      return e < n ? e : n;
    };
    // wait until the previous group's last sweep completed `need` tasks (bounded)
    auto wait_prev = [&](int need) {
      if (gi == 0 || threadIdx.x != 0) return;
      need = need < prev_total ? need : prev_total;
      const uint64_t t0 = __builtin_amdgcn_s_memrealtime();
      while (__hip_atomic_load(&a.progress[gi - 1], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < need) {
        if (__builtin_amdgcn_s_memrealtime() - t0 > 1000000000ull ||  // 10 s at 100 MHz
            __hip_atomic_load(a.err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0) {
          atomicAdd(a.err, 1);
          s_giveup = 1;
          return;
        }
        __builtin_amdgcn_s_sleep(1);
      }
    };
    if (threadIdx.x == 0) s_giveup = 0;
    __syncthreads();
    // initial rows (those step 0 needs): sweep s0-1 must have finished its tasks 0..2
    wait_prev(3);
    __syncthreads();
    int64_t lo = s0, hi = s_giveup ? s0 : front_end(0);
    for (int64_t e = tid; e < (hi - lo) * RW; e += nthr) {
      const int64_t r = lo + e / RW;
      const int col = (int)(e % RW);
      win[ring_slot(r, 0, R) * RS + col] = bld(a.Bs + r * a.ldb + col);
    }
    __syncthreads();

    for (int t = 0; t < tend && !s_giveup; ++t) {
      // rows for step t+1 may be loaded once sweep s0-1 finished task t+3
      wait_prev(t + 4);
      __syncthreads();
      if (s_giveup) break;
      const int64_t nhi = front_end(t + 1);
      double pf[PF];
      const int64_t npf = (nhi - hi) * RW;
#pragma unroll
      for (int k = 0; k < PF; ++k) {
        const int64_t e = tid + (int64_t)k * nthr;
        pf[k] = e < npf ? bld(a.Bs + hi * a.ldb + e) : 0.0;
      }
      // compute: wave i runs task t-3i of sweep s0+i
      if (wv < nsw) {
        const int64_t s = s0 + wv;
        const int jt = t - 3 * wv;
        if (jt >= 0 && jt < ntasks_b<B>(s, n)) {
          const int64_t c = s + 1 + (int64_t)jt * B;
          const int64_t p = jt == 0 ? s : c - B;
          win_task<B>(win, win + (R + 1) * RS + wv * B, R, R, 0, n, p, c);
        }
      }
      __syncthreads();
      // write back rows no unfinished sweep of the group touches again
      // (the minimum over all unfinished sweeps: a sweep that has not started yet
      // still needs its own first row)
      int64_t nlo = n;
      for (int i = 0; i < nsw; ++i) {
        const int jn = t + 1 - 3 * i;
        if (jn < ntasks_b<B>(s0 + i, n)) {
          const int64_t f = sweep_front(s0 + i, jn, B);
          nlo = f < nlo ? f : nlo;
        }
      }
      nlo = nlo < hi ? nlo : hi;
      for (int64_t e = tid; e < (nlo - lo) * RW; e += nthr) {
        const int64_t r = lo + e / RW;
        const int col = (int)(e % RW);
        bst(a.Bs + r * a.ldb + col, win[ring_slot(r, 0, R) * RS + col]);
      }
      lo = nlo;
#pragma unroll
      for (int k = 0; k < PF; ++k) {
        const int64_t e = tid + (int64_t)k * nthr;
        if (e < npf) {
          const int64_t r = hi + e / RW;
          win[ring_slot(r, 0, R) * RS + (int)(e % RW)] = pf[k];
        }
      }
      hi = nhi;
      __builtin_amdgcn_s_waitcnt(0);
      __syncthreads();
      if (threadIdx.x == 0) {
        int done = t - 3 * (nsw - 1) + 1;
        done = done < 0 ? 0 : (done > last_total - 1 ? last_total - 1 : done);
        __hip_atomic_store(&a.progress[gi], done, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      }
    }
    // flush the rest of the window, then mark the group complete
    for (int64_t e = tid; e < (hi - lo) * RW; e += nthr) {
      const int64_t r = lo + e / RW;
      const int col = (int)(e % RW);
      bst(a.Bs + r * a.ldb + col, win[ring_slot(r, 0, R) * RS + col]);
    }
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    if (threadIdx.x == 0)
      __hip_atomic_store(&a.progress[gi], last_total, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// Pipelined chase (b = 16): lag-2 schedule, reflectors formed by every lane
// from a broadcast copy of the vector, row movers that keep global-memory
// latency off the tasks' path, and no workgroup barrier per step.
// ---------------------------------------------------------------------------
//
// Lag 2.  Task j of sweep s+1 and task j+2 of sweep s share exactly one band
// element, (p, c) of the latter: its right reflector reads it as alpha and
// overwrites it with beta at the very start, and the former's left update
// (whose last row is p and last column c) reads and rewrites it near its end.
// Every other element of the two tasks is disjoint, and tasks further apart
// are disjoint, so the two may run in the same step if the left update of
// sweep s+1 waits for the beta of sweep s: wave i publishes the step number
// in an LDS flag right after writing its beta, and wave i+1 waits for it
// before loading its left-update operands.  Wave i runs task t - 2i of sweep
// s0 + i at step t, so a sweep costs two steps instead of three.
//
// Task arithmetic.  With x the vector to annihilate (x_0 = alpha, tail x_1..),
// beta = -sgn(alpha) ||x||, v = (1, x_1 / (alpha - beta), ...) and
// tau = (beta - alpha) / beta (LAPACK's dlarfg convention), the update of a
// vector y is y - tau (v^T y) v with v^T y = y_0 + D / (alpha - beta) and
// D = sum_{l >= 1} x_l y_l.  Every lane reads the whole of x (broadcast LDS
// reads), so D starts as soon as the operands arrive, beside the norm, and no
// lane exchange is needed for the norm or the coefficients; every lane forms
// them with the same instructions, hence bitwise the same values.
//
// Movers and the schedule without a per-step barrier: see k_chase_flow.

__device__ __forceinline__ int uni_i32(int v) { return __builtin_amdgcn_readfirstlane(v); }
// Global-memory pointer types: accesses through them are global (not flat)
// instructions, counted by vmcnt only, so in-flight loads never hold up a wait
// on LDS operations.
typedef __attribute__((address_space(1))) double glb_f64;
typedef __attribute__((address_space(1))) f64x2 glb_f64x2;
typedef __attribute__((address_space(1))) int glb_i32;
typedef int i32x4 __attribute__((ext_vector_type(4)));
constexpr int kDevScope = 16;  // buffer-access cache policy: sc1 (device scope)
__device__ __forceinline__ int64_t uni_i64(int64_t v) {
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)v);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)((uint64_t)v >> 32));
  return (int64_t)(((uint64_t)hi << 32) | lo);
}

// Ring slot (r - base) mod R by a multiply-high with m = floor(2^32 / R): the
// quotient estimate is at most one below the true one for r - base < 2^24 (rows
// are below 2^20), so one correction gives the remainder.
__host__ __device__ inline uint32_t ring_magic(int R) { return (uint32_t)(0xffffffffu / (uint32_t)R); }
__device__ __forceinline__ int ring_slot_m(int64_t r, int64_t base, int R, uint32_t m) {
  const uint32_t d = (uint32_t)(r - base);
  const uint32_t q = __umulhi(d, m);
  uint32_t s = d - q * (uint32_t)R;
  s = s >= (uint32_t)R ? s - (uint32_t)R : s;
  return (int)s;
}

struct PipeRefl {
  double beta, scal, tau;
};

// The task arithmetic below is written out operation by operation (explicit
// fma where one is meant, no contraction of the rest), so that every copy of it
// -- the two left-update paths of a task -- rounds identically and the chase is
// bitwise the same for every schedule.

// Sum over l = 1 .. B-1 of a_l * b_l in four interleaved partial sums, added
// pairwise: the same order wherever it is used.
template <int B>
__device__ __forceinline__ double pipe_dot1(const double (&a)[B], const double (&b)[B]) {
#pragma clang fp contract(off)
  double q0 = 0.0, q1 = 0.0, q2 = 0.0, q3 = 0.0;
#pragma unroll
  for (int l = 1; l < B; ++l) {
    if ((l & 3) == 0) q0 = fma(a[l], b[l], q0);
    if ((l & 3) == 1) q1 = fma(a[l], b[l], q1);
    if ((l & 3) == 2) q2 = fma(a[l], b[l], q2);
    if ((l & 3) == 3) q3 = fma(a[l], b[l], q3);
  }
  return (q0 + q1) + (q2 + q3);
}

template <int B>
__device__ __forceinline__ PipeRefl pipe_refl(const double (&x)[B]) {
#pragma clang fp contract(off)
  const double ss = pipe_dot1<B>(x, x);
  const double alpha = x[0];
  PipeRefl r;
  r.beta = alpha;
  r.scal = 0.0;
  r.tau = 0.0;
  if (ss > 0.0) {
    const double nrm = sqrt(fma(alpha, alpha, ss));
    r.beta = alpha >= 0.0 ? -nrm : nrm;
    r.scal = nr_div(1.0, alpha - r.beta);  // |alpha - beta| >= sqrt(ss): normal whenever ss > 0
    r.tau = nr_div(r.beta - alpha, r.beta);
  }
  return r;
}

// y <- (I - tau v v^T) y, with D = sum_{l >= 1} x_l y_l (tau = 0 leaves y bitwise unchanged)
template <int B>
__device__ __forceinline__ void pipe_apply(const PipeRefl& r, const double (&x)[B], double (&y)[B], double D) {
#pragma clang fp contract(off)
  const double w = r.tau * fma(r.scal, D, y[0]);
  const double ws = w * r.scal;
  y[0] -= w;
#pragma unroll
  for (int l = 1; l < B; ++l) y[l] = fma(-ws, x[l], y[l]);
}

// Task (p, c) on the window, one wave.  `mine`: this wave's beta flag (set to t
// after the right reflector's beta is written), `prev`: the flag of the wave of
// the previous sweep when that sweep has a task at this step (else null).
// Lanes past the last row (right update) or column (left update) read the first
// one again and store nothing, so the loads need no branch.  Returns false if
// the wait for `prev` gave up (*fail set elsewhere, or a 1 s bound).
template <int B>
__device__ __forceinline__ bool pipe_task(lds_f64* win, int R, uint32_t rmagic, int64_t s0, int64_t n, int64_t p,
                                          int64_t c, int* mine, const int* prev, int t, const int* fail) {
  constexpr int RS = 3 * B + 2, LO = B - 1;
  const int lane = threadIdx.x & 63;
  const int L = uni_i32((int)((n - c) < B ? (n - c) : B));
  const int nr = uni_i32((int)(c + L - p - 1));                                  // rows p+1 .. c+L-1
  const int nq = uni_i32((int)(((c + L + B) < n ? (c + L + B) : n) - c - 1));   // columns c+1 .. c+nq
  const int dc = uni_i32((int)(c - p));
  const int sp = uni_i32(ring_slot_m(p, s0, R, rmagic));
  const int sc = uni_i32(ring_slot_m(c, s0, R, rmagic));

  // ---------------- right reflector: row p, columns c .. c+B-1 ----------------
  lds_f64* rowp = win + sp * RS + (dc + LO);
  double x[B], y[B];
#pragma unroll
  for (int l = 0; l < B; ++l) x[l] = rowp[l];  // one address for every lane: broadcast
  const int lr = lane < nr ? lane : 0;
  int sr = sp + 1 + lr;
  sr = sr >= R ? sr - R : sr;
  lds_f64* row = win + sr * RS + (dc - 1 - lr + LO);  // element (p+1+lr, c+l) at row[l]
#pragma unroll
  for (int l = 0; l < B; ++l) y[l] = row[l];
  double D = pipe_dot1<B>(x, y);
  PipeRefl r = pipe_refl<B>(x);
  if (lane < B) rowp[lane] = lane == 0 ? r.beta : 0.0;
  if (lane == 0) __hip_atomic_store(mine, t, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_WORKGROUP);
  pipe_apply<B>(r, x, y, D);
  if (lane < nr) {
#pragma unroll
    for (int l = 0; l < B; ++l) row[l] = y[l];
  }

  // ---------------- left reflector: column c, rows c .. c+B-1 ----------------
  bool ok = true;
  if (prev != nullptr && __hip_atomic_load(prev, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_WORKGROUP) < t) {
    const uint64_t t0 = __builtin_amdgcn_s_memrealtime();
    for (;;) {
      __builtin_amdgcn_s_sleep(1);
      if (__hip_atomic_load(prev, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_WORKGROUP) >= t) break;
      if (__hip_atomic_load(fail, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP) != 0 ||
          __builtin_amdgcn_s_memrealtime() - t0 > 100000000ull) {  // 1 s at 100 MHz
        ok = false;
        break;
      }
    }
  }
  const int lq = lane < nq ? lane : 0;  // column c+1+lq
  if (sc + B <= R && L == B) {
    // rows c .. c+B-1 in consecutive slots: element (c+m, c) at colx[m (RS-1)],
    // element (c+m, c+1+lq) at coly[m (RS-1)]
    const lds_f64* colx = win + sc * RS + LO;
    lds_f64* coly = win + sc * RS + (1 + lq + LO);
#pragma unroll
    for (int m = 0; m < B; ++m) x[m] = colx[m * (RS - 1)];
#pragma unroll
    for (int m = 0; m < B; ++m) y[m] = coly[m * (RS - 1)];
    D = pipe_dot1<B>(x, y);
    r = pipe_refl<B>(x);
    if (lane < B) win[(sc + lane) * RS + LO - lane] = lane == 0 ? r.beta : 0.0;
    pipe_apply<B>(r, x, y, D);
    if (lane < nq) {
#pragma unroll
      for (int m = 0; m < B; ++m) coly[m * (RS - 1)] = y[m];
    }
  } else {
    // wrapping window or rows past n - 1 (read from the zero slot R, never written)
    int so[B];
#pragma unroll
    for (int m = 0; m < B; ++m) {
      int sm = sc + m;
      sm = sm >= R ? sm - R : sm;
      so[m] = m < L ? sm : R;
    }
#pragma unroll
    for (int m = 0; m < B; ++m) x[m] = win[so[m] * RS + LO - m];
#pragma unroll
    for (int m = 0; m < B; ++m) y[m] = win[so[m] * RS + 1 + lq - m + LO];
    D = pipe_dot1<B>(x, y);
    r = pipe_refl<B>(x);
    if (lane < L) {
      int sm = sc + lane;
      sm = sm >= R ? sm - R : sm;
      win[sm * RS + LO - lane] = lane == 0 ? r.beta : 0.0;
    }
    pipe_apply<B>(r, x, y, D);
    if (lane < nq) {
#pragma unroll
      for (int m = 0; m < B; ++m)
        if (m < L) win[so[m] * RS + 1 + lq - m + LO] = y[m];
    }
  }
  return ok;
}

// Barrier-free schedule.  The waves of a workgroup synchronise through
// counters in LDS instead of a workgroup barrier per step:
//   s_done[i]  last step compute wave i has finished; wave i starts step t once
//              wave i-1 finished step t-1 (and wave 0 once the rows of step t
//              are in the window).  Every wave passes every step;
//   s_filled   last step whose rows are in the window;
//   s_stored   last duty whose rows have been read out of the window for storing
//              (their slots may be refilled K duties later);
//   s_conf     last duty whose stores are known to be complete in memory.
// A wave that runs ahead of its successor is always safe (the later sweep only
// falls further behind); one that would fall behind waits.  Two kinds of mover
// waves take duties in turn.  Loader k (of ML) at duty t = k, k + ML, ... fills
// the rows of step t + 1 (loaded at its previous duty) and loads those of step
// t + ML + 1; it runs ahead of the compute waves.  Storer k (of MS) at duty
// t = k, k + MS, ... reads out the rows no task touches after step t - 1 once
// every compute wave has finished that step, stores them, waits for the stores
// to complete and publishes the progress they allow; it trails the compute
// waves.  Neither is on the compute waves' path, which carries only task
// latency and counter hand-offs.
//
// Hand-off between groups.  Band rows cross workgroups (and XCDs, whose L2
// caches are not coherent with each other) only as relaxed device-scope atomic
// loads and stores, which go to the device's coherence point.  A group publishes
// a progress value only after the stores it covers have completed there (the
// mover's own wait on its memory counter, confirmed in duty order), and a group
// issues the loads of rows only after it has read a progress value that covers
// them; a compiler-only fence keeps the compiler from moving memory operations
// across either point.  Agent-scope release/acquire fences would add a
// write-back or an invalidation of the whole L2 cache per hand-off; measured in
// this kernel they lengthen every mover duty by microseconds, so the ordering
// rests on completion of device-scope accesses instead.

constexpr int kFlowLoaders = 2;  // ML
constexpr int kFlowStorers = 2;  // MS
constexpr int kFlowSlack = 2;  // K: extra ring rows (in units of b) between storing and refilling a slot
constexpr int kFlowMaxW = 8;
// Instantiations by width.  A workgroup of at most 8 waves (two per SIMD) may use
// 256 VGPRs per lane, which the task needs without spilling; 12 waves allow 168
// and spill.  So widths up to 4 run with two loaders and two storers, widths 5
// and 6 with one of each (8 waves), and only 7 and 8 with 12 waves.
constexpr int kFlowNarrowW = 4;
constexpr int kFlowMidW = 6;

__host__ __device__ inline int flow_rows(int b, int W) { return (2 * W + 3 + kFlowSlack) * b; }

size_t chase_flow_lds_bytes(int b, int W) {
  return (size_t)(flow_rows(b, W) + 1) * (3 * b + 2) * sizeof(double);  // ring + zero slot
}

// Wait until the LDS counter reaches v (acquire).  Gives up (false) when *fail
// is set or after 10 s.
__device__ __forceinline__ bool lds_wait_ge(const int* ctr, int v, const int* fail) {
  if (uni_i32(__hip_atomic_load(ctr, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_WORKGROUP)) >= v) return true;
  const uint64_t t0 = __builtin_amdgcn_s_memrealtime();
  for (;;) {
    __builtin_amdgcn_s_sleep(1);
    if (uni_i32(__hip_atomic_load(ctr, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_WORKGROUP)) >= v) return true;
    if (uni_i32(__hip_atomic_load(fail, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP)) != 0 ||
        __builtin_amdgcn_s_memrealtime() - t0 > 1000000000ull)
      return false;
  }
}
__device__ __forceinline__ void lds_set(int* ctr, int v) {
  if ((threadIdx.x & 63) == 0) __hip_atomic_store(ctr, v, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_WORKGROUP);
}

template <int B, int ML, int MS, int K, int WMAX>
__global__ void __launch_bounds__(64 * (WMAX + ML + MS)) k_chase_flow(ChaseArgs Lg) {
  constexpr int RW = 3 * B, RS = RW + 2, MT = 64;
  constexpr int KP = (B * RW / 2 + MT - 1) / MT;  // pairs of doubles per mover lane for B rows
  extern __shared__ __align__(16) double lds[];
  __shared__ int s_done[WMAX], s_beta[WMAX];
  __shared__ int s_filled, s_stored, s_conf, s_fail;
  const int W = uni_i32(Lg.W);
  const int R = (2 * W + 3 + K) * B;
  const uint32_t rmagic = ring_magic(R);
  lds_f64* win = (lds_f64*)lds;
  const int wv = uni_i32(threadIdx.x >> 6);
  const int tid = threadIdx.x;
  const int mt = tid & 63;
  const bool mover = wv >= W;
  const int mk = wv - W;  // mover index (mover waves only)
  for (int e = tid; e < RS; e += blockDim.x) win[R * RS + e] = 0.0;  // zero slot

  // pair k of a mover lane within a block of rows: row prow[k], columns pcol[k], pcol[k] + 1
  int prow[KP], pcol[KP];
#pragma unroll
  for (int k = 0; k < KP; ++k) {
    const int q = mt + k * MT;
    prow[k] = q / (RW / 2);
    pcol[k] = 2 * (q % (RW / 2));
  }

  for (;;) {
    int gi;
    const ChaseArgs a = take_group(Lg, gi);
    if (gi < 0) break;
    gi = uni_i32(gi);
    const int64_t n = uni_i64(a.n);
    double* Bs = a.Bs;
    glb_i32* progress = (glb_i32*)a.progress;
    glb_i32* err = (glb_i32*)a.err;
    const int64_t s0 = (int64_t)gi * W;
    const int sbase = (int)(s0 * RW * (int64_t)sizeof(double));  // byte offset of row s0 (rows below 2^20)
    const int nsw = uni_i32((int)((n - 1 - s0) < W ? (n - 1 - s0) : W));
    const int64_t sl = s0 + nsw - 1;
    const int first_total = ntasks_b<B>(s0, n);
    const int last_total = ntasks_b<B>(sl, n);
    const int prev_total = gi > 0 ? ntasks_b<B>(s0 - 1, n) : 0;
    int tend = 0;
    for (int i = 0; i < nsw; ++i) {
      const int te = 2 * i + ntasks_b<B>(s0 + i, n);
      tend = te > tend ? te : tend;
    }
    // rows the group's first sweep needs up to (and including) step u: [s0, fe(u))
    auto fe = [&](int u) -> int64_t {
      if (u < 0) return s0;
      const int uu = u < first_total - 1 ? u : first_total - 1;
      const int64_t e = s0 + 1 + (int64_t)(uu + 1) * B;
      return e < n ? e : n;
    };
    // rows no sweep of the group touches after step t (rows below fe(t) only): the
    // lowest front of the unfinished sweeps.  The last sweep finishes last (sweeps
    // of one group differ by at most one task, and it starts 2 steps after its
    // predecessor); once started its front is the lowest, and before that the
    // first sweep not yet started (front = its first row) is.
    auto final_after = [&](int t) -> int64_t {
      const int64_t f_e = fe(t);
      const int jn = t + 1 - 2 * (nsw - 1);
      if (jn >= last_total) return f_e;
      int64_t f;
      if (jn <= 0) {
        const int i0 = (t + 2) / 2 > 0 ? (t + 2) / 2 : 0;  // first sweep whose task t+1-2i is not positive
        f = s0 + i0;
      } else {
        f = sweep_front(sl, jn, B);
      }
      return f < f_e ? f : f_e;
    };
    // progress the successor may rely on once every step up to t is finished and
    // the rows below Lr are stored: tasks of the last sweep done, capped by the
    // rows the successor's step P-3 needs (below sl + 2 + (P-2) B)
    auto allowed = [&](int t, int64_t Lr) -> int {
      int d = t - 2 * (nsw - 1) + 1;
      d = d < 0 ? 0 : (d > last_total ? last_total : d);
      if (Lr < n) {
        const int64_t q = Lr - sl - 2;
        const int br = q >= 0 ? (int)(q / B) + 2 : 0;
        d = br < d ? br : d;
      }
      return d;
    };
    auto giveup = [&]() {
      if (mt == 0) {
        __hip_atomic_fetch_add(err, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __hip_atomic_store(&s_fail, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
      }
    };
    // bounded wait (one mover wave) until the predecessor's progress reaches `need`
    auto wait_prev = [&](int need, int& known) -> bool {
      need = need < prev_total ? need : prev_total;
      if (gi == 0 || known >= need) return true;
      const uint64_t t0 = __builtin_amdgcn_s_memrealtime();
      for (;;) {
        known = uni_i32(__hip_atomic_load(&progress[gi - 1], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
        if (known >= need) return true;
        if (__builtin_amdgcn_s_memrealtime() - t0 > 1000000000ull ||  // 10 s at 100 MHz
            __hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0 ||
            __hip_atomic_load(&s_fail, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP) != 0)
          return false;
        __builtin_amdgcn_s_sleep(1);
      }
    };
    auto slot = [&](int64_t r) -> int { return ring_slot_m(r, s0, R, rmagic); };
    auto pair_lds = [&](int s_r0, int k) -> lds_f64x2* {
      int sq = s_r0 + prow[k];
      sq = sq >= R ? sq - R : sq;
      return (lds_f64x2*)(win + sq * RS + pcol[k]);
    };
    // Band rows move as 16-byte buffer accesses at device scope (sc1: coherent at
    // the device level, like the relaxed device-scope atomics they stand for);
    // the resource covers the matrix's n rows, so nothing outside them is touched.
    const __amdgpu_buffer_rsrc_t brs =
        __builtin_amdgcn_make_buffer_rsrc(Bs, (short)0, (int)(n * RW * (int64_t)sizeof(double)), 0x00020000);
    // global <-> registers <-> window for a block of at most B rows [r0, r1)
    auto blk_load = [&](int64_t r0, int64_t r1, f64x2 (&buf)[KP]) {
      const int np = (int)(r1 - r0) * (RW / 2);
      const int base = (int)((r0 - s0) * RW * (int64_t)sizeof(double));
#pragma unroll
      for (int k = 0; k < KP; ++k)
        if (mt + k * MT < np)
          buf[k] = __builtin_bit_cast(f64x2, __builtin_amdgcn_raw_buffer_load_b128(brs, (mt + k * MT) * 16, base + sbase,
                                                                                    kDevScope));
    };
    auto blk_fill = [&](int64_t r0, int64_t r1, const f64x2 (&buf)[KP]) {
      const int rows = (int)(r1 - r0);
      const int s_r0 = slot(r0);
#pragma unroll
      for (int k = 0; k < KP; ++k)
        if (prow[k] < rows) *pair_lds(s_r0, k) = buf[k];
    };
    // rows [r0, r1) read out of the window and stored at device scope; `read_out`
    // is called once every row has left the window (before the last stores issue)
    auto store_rows = [&](int64_t r0, int64_t r1, auto read_out) {
      for (int64_t rb = r0; rb < r1; rb += B) {
        const int64_t re = r1 - rb < B ? r1 : rb + B;
        const int rows = (int)(re - rb);
        const int np = rows * (RW / 2);
        const int s_r0 = slot(rb);
        f64x2 vals[KP];
#pragma unroll
        for (int k = 0; k < KP; ++k) vals[k] = prow[k] < rows ? *pair_lds(s_r0, k) : f64x2{0.0, 0.0};
        if (re == r1) read_out();
        const int base = (int)((rb - s0) * RW * (int64_t)sizeof(double));
#pragma unroll
        for (int k = 0; k < KP; ++k)
          if (mt + k * MT < np)
            __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(i32x4, vals[k]), brs, (mt + k * MT) * 16,
                                                   base + sbase, kDevScope);
      }
      if (r0 >= r1) read_out();
    };

    if (tid == 0) {
      s_filled = -1;
      s_stored = -1;
      s_conf = -1;
      s_fail = 0;
    }
    if (tid < WMAX) {
      s_done[tid] = -1;
      s_beta[tid] = -1;
    }
    __syncthreads();
    // prologue: rows of steps 0 .. ML, loaded by the loaders together (after the
    // predecessor's progress allows step ML)
    int known = 0;
    if (mover && mk < ML) {
      if (wait_prev(ML + 3, known)) {
        __atomic_signal_fence(__ATOMIC_SEQ_CST);
        const int64_t hi = fe(ML);
        for (int64_t rb = s0 + (int64_t)mk * B; rb < hi; rb += (int64_t)ML * B) {
          f64x2 buf[KP];
          const int64_t re = hi - rb < B ? hi : rb + B;
          blk_load(rb, re, buf);
          blk_fill(rb, re, buf);
        }
      } else {
        giveup();
      }
    }
    __syncthreads();
    if (tid == 0) s_filled = ML;
    __syncthreads();

    if (!mover) {
      if (wv < nsw) {
        const int64_t s = s0 + wv;
        const int nt = ntasks_b<B>(s, n);
        const int ntp = wv > 0 ? ntasks_b<B>(s - 1, n) : 0;
        for (int t = 0; t < tend; ++t) {
          const bool ok = wv == 0 ? lds_wait_ge(&s_filled, t, &s_fail) : lds_wait_ge(&s_done[wv - 1], t - 1, &s_fail);
          if (!ok) {
            giveup();
            break;
          }
          CHASE_MARK_IF(mt == 0 && wv == 0, gi, t, 0);
          const int jt = t - 2 * wv;
          if (jt >= 0 && jt < nt) {
            const int64_t c = s + 1 + (int64_t)jt * B;
            const int64_t p = jt == 0 ? s : c - B;
            // the previous sweep's task jt+2 runs at the same step: wait for its beta
            const int* prevf = (wv > 0 && jt + 2 < ntp) ? &s_beta[wv - 1] : nullptr;
            if (!pipe_task<B>(win, R, rmagic, s0, n, p, c, &s_beta[wv], prevf, t, &s_fail)) {
              giveup();
              break;
            }
          }
          lds_set(&s_done[wv], t);
          CHASE_MARK_IF(mt == 0 && wv == 0, gi, t, 1);
          CHASE_MARK_IF(mt == 0 && wv == nsw - 1, gi, t, 2);
        }
      }
    } else if (mk < ML) {
      // loader mk: duties t = mk, mk + ML, ...
      f64x2 regs[KP];
      int pend = 0;
      bool have_pend = false;
      for (int t = mk; t < tend; t += ML) {
        CHASE_MARK_IF(mt == 0, gi, t, 3);
        // rows of step t + 1 (loaded at duty t - ML) into the window, in step order,
        // into slots whose rows were read out at least K duties ago
        if (t >= ML) {
          __builtin_amdgcn_s_waitcnt(0);
          if (!lds_wait_ge(&s_stored, t - 1 - K, &s_fail) || !lds_wait_ge(&s_filled, t, &s_fail)) {
            giveup();
            break;
          }
          blk_fill(fe(t), fe(t + 1), regs);
          lds_set(&s_filled, t + 1);
        }
        CHASE_MARK_IF(mt == 0, gi, t, 4);
        // rows of step t + ML + 1, once the predecessor's progress allows them
        if (have_pend) known = pend > known ? pend : known;
        const int64_t r0 = fe(t + ML), r1 = fe(t + ML + 1);
        if (r1 > r0) {
          if (!wait_prev(t + ML + 4, known)) {
            giveup();
            break;
          }
          __atomic_signal_fence(__ATOMIC_SEQ_CST);
          blk_load(r0, r1, regs);
        }
        CHASE_MARK_IF(mt == 0, gi, t, 5);
        if (gi > 0) {
          pend = __hip_atomic_load(&progress[gi - 1], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          have_pend = true;
        }
      }
      __builtin_amdgcn_s_waitcnt(0);
    } else {
      // storer mk - ML: duties t = mk - ML, mk - ML + MS, ...
      for (int t = mk - ML; t < tend; t += MS) {
        // rows final after step t - 1, read out in duty order once every wave has
        // finished that step (a wave may finish a step before its predecessor
        // does: the order only binds starts), then stored
        bool ready = lds_wait_ge(&s_stored, t - 1, &s_fail);
        for (int i = nsw - 1; i >= 0 && ready; --i) ready = lds_wait_ge(&s_done[i], t - 1, &s_fail);
        if (!ready) {
          giveup();
          break;
        }
        CHASE_MARK_IF(mt == 0, gi, t, 6);
        const int64_t hi = final_after(t - 1);
        store_rows(final_after(t - 2), hi, [&]() { lds_set(&s_stored, t); });
        // stores complete: confirm in duty order and publish what they allow
        __builtin_amdgcn_s_waitcnt(0);
        __atomic_signal_fence(__ATOMIC_SEQ_CST);
        if (!lds_wait_ge(&s_conf, t - 1, &s_fail)) {
          giveup();
          break;
        }
        if (mt == 0) {
          const int P = allowed(t - 1, hi);
          if (P > 0)
            __hip_atomic_fetch_max(&progress[gi], P < last_total ? P : last_total - 1, __ATOMIC_RELAXED,
                                   __HIP_MEMORY_SCOPE_AGENT);
        }
        lds_set(&s_conf, t);
        CHASE_MARK_IF(mt == 0, gi, t, 7);
      }
      __builtin_amdgcn_s_waitcnt(0);
    }
    // epilogue: every wave is through its steps; store the rest of the window, then
    // mark the group complete
    __syncthreads();
    const bool failed = __hip_atomic_load(&s_fail, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP) != 0;
    if (mover && mk == ML && !failed) {
      store_rows(final_after(tend - 2), fe(tend - 1), []() {});
      __builtin_amdgcn_s_waitcnt(0);
      __atomic_signal_fence(__ATOMIC_SEQ_CST);
      if (mt == 0)
        __hip_atomic_fetch_max(&progress[gi], last_total, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    __syncthreads();
  }
}

// d_i = B(i, i), e_i = B(i, i+1) once every sweep has finished (next kernel in the stream).
__device__ __forceinline__ void chase_extract_body(const double* __restrict__ Bs, int64_t ldb, int64_t n, int b,
                                                   double* d, double* e) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    d[i] = Bs[i * ldb + (b - 1)];
    if (i + 1 < n) e[i] = Bs[i * ldb + b];
  }
}
__global__ void k_chase_extract(const double* __restrict__ Bs, int64_t ldb, int64_t n, int b, double* d, double* e) {
  chase_extract_body(Bs, ldb, n, b, d, e);
}
__global__ void k_chase_extract_b(const ChaseArgs* __restrict__ tab) {
  const ChaseArgs& a = tab[blockIdx.y];
  chase_extract_body(a.Bs, a.ldb, a.n, a.b, a.d, a.e);
}

static bool use_pipe(int b, int W) { return b == 16 && W <= kFlowMaxW && chase_flow_lds_bytes(b, W) <= 159 * 1024; }
static bool use_window(int b, int W) { return b == 32 && chase_win_lds_bytes(b, W) <= 159 * 1024; }

static const void* chase_fn(int b, int W) {
  if (use_pipe(b, W)) {
    if (W <= kFlowNarrowW) return (const void*)k_chase_flow<16, kFlowLoaders, kFlowStorers, kFlowSlack, kFlowNarrowW>;
    if (W <= kFlowMidW) return (const void*)k_chase_flow<16, 1, 1, kFlowSlack, kFlowMidW>;
    return (const void*)k_chase_flow<16, kFlowLoaders, kFlowStorers, kFlowSlack, kFlowMaxW>;
  }
  if (use_window(b, W)) return (const void*)k_chase_win<32>;
  return (const void*)k_chase;
}

static int chase_threads(int b, int W) {
  if (use_pipe(b, W)) return 64 * (W + (W > kFlowNarrowW && W <= kFlowMidW ? 2 : kFlowLoaders + kFlowStorers));
  return use_window(b, W) ? 64 * (W > WinGeom<32>::MIN_WAVES ? W : WinGeom<32>::MIN_WAVES) : 64 * W;
}

static size_t chase_launch_lds(int b, int W) {
  if (use_pipe(b, W)) return chase_flow_lds_bytes(b, W);
  return use_window(b, W) ? chase_win_lds_bytes(b, W) : chase_lds_bytes(b, W);
}

static hipError_t chase_set_lds(const void* fn, size_t lds) {
  hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  return e;
}

int chase_max_groups_resident(int b, int W) {
  int dev = 0, cus = 0, per = 0;
  const void* fn = chase_fn(b, W);
  const size_t lds = chase_launch_lds(b, W);
  if (chase_set_lds(fn, lds) != hipSuccess) return 0;
  if (hipGetDevice(&dev) != hipSuccess) return 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, fn, chase_threads(b, W), lds) != hipSuccess) return 0;
  return per * cus;
}

static hipError_t launch_chase_kernel(const ChaseArgs& a, int grid, hipStream_t st) {
  const void* fn = chase_fn(a.b, a.W);
  const size_t lds = chase_launch_lds(a.b, a.W);
  hipError_t e = chase_set_lds(fn, lds);
  if (e != hipSuccess) return e;
  {
    const dim3 block(chase_threads(a.b, a.W));
    if (fn == (const void*)k_chase_flow<16, kFlowLoaders, kFlowStorers, kFlowSlack, kFlowNarrowW>)
      hipLaunchKernelGGL((k_chase_flow<16, kFlowLoaders, kFlowStorers, kFlowSlack, kFlowNarrowW>), dim3(grid), block,
                         lds, st, a);
    else if (fn == (const void*)k_chase_flow<16, 1, 1, kFlowSlack, kFlowMidW>)
      hipLaunchKernelGGL((k_chase_flow<16, 1, 1, kFlowSlack, kFlowMidW>), dim3(grid), block, lds, st, a);
    else if (fn == (const void*)k_chase_flow<16, kFlowLoaders, kFlowStorers, kFlowSlack, kFlowMaxW>)
      hipLaunchKernelGGL((k_chase_flow<16, kFlowLoaders, kFlowStorers, kFlowSlack, kFlowMaxW>), dim3(grid), block, lds,
                         st, a);
    else if (fn == (const void*)k_chase_win<32>) hipLaunchKernelGGL(k_chase_win<32>, dim3(grid), block, lds, st, a);
    else hipLaunchKernelGGL(k_chase, dim3(grid), block, lds, st, a);
  }
  return hipGetLastError();
}

hipError_t launch_chase(const ChaseArgs& a0, int grid, hipStream_t st) {
  ChaseArgs a = a0;
  a.tab = nullptr;
  a.order = nullptr;
  a.ticket = a.progress + a.ngroups;  // zeroed with the progress counters
  a.total = a.ngroups;
  if (a.n > 1) {
    hipLaunchKernelGGL(k_fill_i32, dim3(64), dim3(256), 0, st, a.progress, 0, (int64_t)a.ngroups + 1);
    hipError_t e = launch_chase_kernel(a, grid, st);
    if (e != hipSuccess) return e;
  }
  const int g = (int)((a.n + 255) / 256);
  hipLaunchKernelGGL(k_chase_extract, dim3(g < 1 ? 1 : (g > 4096 ? 4096 : g)), dim3(256), 0, st, a.Bs, a.ldb, a.n,
                     a.b, a.d, a.e);
  return hipGetLastError();
}

hipError_t launch_chase_batched(const ChaseArgs& L, int grid, int count, int64_t max_n, int* zero_base,
                                int64_t zero_count, hipStream_t st) {
  hipLaunchKernelGGL(k_fill_i32, dim3(64), dim3(256), 0, st, zero_base, 0, zero_count);  // progress + ticket
  if (L.total > 0) {
    hipError_t e = launch_chase_kernel(L, grid, st);
    if (e != hipSuccess) return e;
  }
  const int g = (int)((max_n + 255) / 256);
  hipLaunchKernelGGL(k_chase_extract_b, dim3(g < 1 ? 1 : (g > 64 ? 64 : g), count), dim3(256), 0, st, L.tab);
  return hipGetLastError();
}

}  // namespace svdv

#ifdef SVDV_CHASE_TRACE
extern "C" int svdv_chase_trace(uint64_t* out, int count) {
  return (int)hipMemcpyFromSymbol(out, HIP_SYMBOL(svdv::g_chase_trace), (size_t)count * 8);
}
#endif
