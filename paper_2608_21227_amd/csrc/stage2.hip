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
// Dependencies: task j of sweep s+1 overlaps tasks j, j+1, j+2 of sweep s (the
// last by one element), so it may start once sweep s has finished task j+2.
// Tasks of different sweeps that respect this lag touch disjoint data, so any
// schedule obeying it gives bitwise the same result.
//
// Schedule: sweeps are cut into groups of W consecutive sweeps; one workgroup
// (W waves) owns a group and advances its sweeps in lockstep -- at step t the
// wave of sweep s0+i runs task t-3i -- with a workgroup barrier between steps.
// A persistent grid takes groups in increasing order from a ticket counter, so
// the predecessor of every group being worked on is held by a workgroup that is
// already running: no schedule can wait on a workgroup that was never made
// resident, whatever the occupancy.  Group g waits for group g-1's last sweep
// through a progress counter.  Band data crosses
// workgroups (and XCDs, whose L2 caches are not coherent with each other), so
// every band access is a relaxed device-scope atomic (coherent at device
// level), and progress is published only after the step's stores completed.
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
// Windowed chase (b = 16 or 32): the rows a group is working on live in LDS.
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
// Windowed chase with mover waves (b = 16): the window of k_chase_win, with all
// global-memory traffic taken off the tasks' path.
// ---------------------------------------------------------------------------
//
// Waves 0..W-1 only compute (wave i runs task t-3i of sweep s0+i at step t);
// the kSpecMovers = 2 waves after them move rows, during the tasks of the same
// step, side by side.  At step t the storer wave
//   1. waits for its own stores of step t-1,
//   2. (one lane) publishes the progress whose rows were stored at step t-2,
//   3. stores the rows no sweep of the group touches after step t-1;
// and the loader wave
//   1. waits for its own loads of step t-1 and writes those rows (needed at
//      step t+1) into the window,
//   2. waits until the predecessor group finished the tasks step t+2 depends
//      on, and requests the rows of step t+2.
// One workgroup barrier ends a step.  Rows written in (3) are beyond every row
// the tasks of step t touch, and rows stored in (4) are below them, so the
// movers never race the tasks.  The hand-off between consecutive groups costs
// about four steps.

constexpr int kSpecMovers = 2;
constexpr int kSpecMaxW = 6;

__host__ __device__ inline int spec_rows(int b, int W) { return (3 * W + 6) * b; }

size_t chase_spec_lds_bytes(int b, int W) {
  return ((size_t)(spec_rows(b, W) + 1) * (3 * b + 2) + (size_t)16 * b) * sizeof(double);  // ring + zero slot + reflector slots
}

template <int B>
__global__ void __launch_bounds__(64 * (kSpecMaxW + kSpecMovers)) k_chase_spec(ChaseArgs L) {
  constexpr int RW = 3 * B, RS = RW + 2, MT = 64;
  constexpr int KP = (B * RW / 2 + MT - 1) / MT;  // pairs of doubles per mover lane for B rows
  extern __shared__ __align__(16) double lds[];
  __shared__ int s_flag;
  const int W = L.W;
  const int R = spec_rows(B, W);
  lds_f64* win = (lds_f64*)lds;
  const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), tid = threadIdx.x;  // wv: wave-uniform
  const bool mover = wv >= W;
  const bool storer = wv == W;  // the first mover wave stores and publishes, the second loads
  const int mt = tid & 63;      // lane within the mover wave
  for (int e = tid; e < RS; e += blockDim.x) win[R * RS + e] = 0.0;  // zero slot

  for (;;) {
    int gi;
    const ChaseArgs a = take_group(L, gi);
    if (gi < 0) break;
    const int64_t n = a.n;
    const int64_t s0 = (int64_t)gi * W;
    const int nsw = (int)((n - 1 - s0) < W ? (n - 1 - s0) : W);
    const int64_t sl = s0 + nsw - 1;
    int tend = 0;
    for (int i = 0; i < nsw; ++i) {
      const int te = 3 * i + ntasks_b<B>(s0 + i, n);
      tend = te > tend ? te : tend;
    }
    const int prev_total = gi > 0 ? ntasks_b<B>(s0 - 1, n) : 0;
    const int last_total = ntasks_b<B>(sl, n);
    const int first_total = ntasks_b<B>(s0, n);
    auto slot = [&](int64_t r) -> int { return ring_slot(r, s0, R); };
    // rows the group's first sweep needs up to (and including) step t: [s0, front_end(t))
    auto front_end = [&](int t) -> int64_t {
      const int tt = t < first_total - 1 ? t : first_total - 1;
      const int64_t e = s0 + 1 + (int64_t)(tt + 1) * B;
      return e < n ? e : n;
    };
    // rows no sweep of the group touches after step t
    auto final_after = [&](int t) -> int64_t {
      int64_t lo = n;
      for (int i = 0; i < nsw; ++i) {
        const int jn = t + 1 - 3 * i;
        if (jn < ntasks_b<B>(s0 + i, n)) {
          const int64_t f = sweep_front(s0 + i, jn, B);
          lo = f < lo ? f : lo;
        }
      }
      const int64_t cap = front_end(t);
      return lo < cap ? lo : cap;
    };
    // tasks of the last sweep completed after step t
    auto done_after = [&](int t) -> int {
      int d = t - 3 * (nsw - 1) + 1;
      return d < 0 ? 0 : (d > last_total ? last_total : d);
    };
    // progress that rows [.., L) written back allow (the next group's step j
    // needs rows below sl + 2 + (j+1) b and progress j + 3)
    auto by_rows = [&](int64_t L) -> int { return L - sl - 1 >= 0 ? (int)((L - sl - 1) / B) + 1 : 0; };
    // each mover wave waits until the previous group's last sweep completed `need` tasks (bounded)
    auto wait_prev = [&](int need) {
      if (gi == 0) return;
      need = need < prev_total ? need : prev_total;
      const uint64_t t0 = __builtin_amdgcn_s_memrealtime();
      while (__hip_atomic_load(&a.progress[gi - 1], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < need) {
        if (__builtin_amdgcn_s_memrealtime() - t0 > 1000000000ull ||  // 10 s at 100 MHz
            __hip_atomic_load(a.err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0) {
          if ((tid & 63) == 0) atomicAdd(a.err, 1);
          s_flag = 1;
          return;
        }
        __builtin_amdgcn_s_sleep(1);
      }
    };
    if (tid == 0) s_flag = 0;
    __syncthreads();
    // row movers: a block of rows [r0, r1) is contiguous in the chase storage (row
    // stride RW = 3B); it is moved as pairs of doubles, pair q = (row r0 + q / (RW/2),
    // columns 2 (q % (RW/2)) and the next), thread mt taking pairs mt + k MT.  On the
    // LDS side a pair is one 16-byte access (slot stride and RW are even).
    auto mv_load = [&](int64_t r0, int64_t r1, f64x2 (&buf)[KP]) {
      const int np = (int)(r1 - r0) * (RW / 2);
      const double* src = a.Bs + r0 * RW + 2 * mt;
#pragma unroll
      for (int k = 0; k < KP; ++k) {
        const bool ok = mt + k * MT < np;
        buf[k].x = ok ? bld(src + 2 * k * MT) : 0.0;
        buf[k].y = ok ? bld(src + 2 * k * MT + 1) : 0.0;
      }
    };
    // pair k of this thread: row prow[k] of the block, columns pcol[k], pcol[k] + 1
    // (the same for every block, so computed once)
    int prow[KP], pcol[KP];
#pragma unroll
    for (int k = 0; k < KP; ++k) {
      const int q = mt + k * MT;
      prow[k] = q / (RW / 2);
      pcol[k] = 2 * (q % (RW / 2));
    }
    auto pair_lds = [&](int s_r0, int k) -> lds_f64x2* {
      int sl = s_r0 + prow[k];
      sl = sl >= R ? sl - R : sl;
      return (lds_f64x2*)(win + sl * RS + pcol[k]);
    };
    auto mv_fill = [&](int64_t r0, int64_t r1, const f64x2 (&buf)[KP]) {
      const int rows = (int)(r1 - r0);
      const int s_r0 = slot(r0);
#pragma unroll
      for (int k = 0; k < KP; ++k)
        if (prow[k] < rows) *pair_lds(s_r0, k) = buf[k];
    };
    auto mv_store = [&](int64_t r0, int64_t r1) {
      // up to B rows per batch (more only when the last sweep starts): LDS reads, then stores
      for (int64_t rb = r0; rb < r1; rb += B) {
        const int64_t re = r1 - rb < B ? r1 : rb + B;
        const int np = (int)(re - rb) * (RW / 2);
        const int rows = (int)(re - rb);
        const int s_r0 = slot(rb);
        f64x2 vals[KP];
#pragma unroll
        for (int k = 0; k < KP; ++k) vals[k] = prow[k] < rows ? *pair_lds(s_r0, k) : f64x2{0.0, 0.0};
        double* dst = a.Bs + rb * RW + 2 * mt;
#pragma unroll
        for (int k = 0; k < KP; ++k)
          if (mt + k * MT < np) {
            bst(dst + 2 * k * MT, vals[k].x);
            bst(dst + 2 * k * MT + 1, vals[k].y);
          }
      }
    };
    // prologue: rows of steps 0 and 1, loaded directly
    if (mover && !storer) {
      wait_prev(4);
      if (!s_flag) {
        const int64_t hi1 = front_end(1);
        for (int64_t rb = s0; rb < hi1; rb += B) {
          f64x2 buf[KP];
          const int64_t re = hi1 - rb < B ? hi1 : rb + B;
          mv_load(rb, re, buf);
          mv_fill(rb, re, buf);
        }
      }
    }
    __syncthreads();
    int64_t lo = s0;         // rows below lo have been stored
    int64_t lo_hist[3] = {s0, s0, s0};  // lo after the stores of steps t-1, t-2, t-3
    int published = 0;
    f64x2 regs[KP];
    for (int t = 0; t < tend && !s_flag; ++t) {
      CHASE_MARK(gi, t, 0);
      if (!mover) {
        if (wv < nsw) {
          const int64_t s = s0 + wv;
          const int jt = t - 3 * wv;
          if (jt >= 0 && jt < ntasks_b<B>(s, n)) {
            const int64_t c = s + 1 + (int64_t)jt * B;
            const int64_t p = jt == 0 ? s : c - B;
            win_task<B>(win, win + (R + 1) * RS + wv * B, R, R, s0, n, p, c);
          }
        }
        CHASE_MARK(gi, t, 1);
      } else if (storer) {
        // 1. own stores of step t-1 complete
        __builtin_amdgcn_s_waitcnt(0);
        CHASE_MARK_IF(mt == 0, gi, t, 3);
        // 2. publish: the rows stored at step t-2 are long complete
        if (mt == 0 && t >= 2) {
          int P = done_after(t - 3 >= 0 ? t - 3 : -1);
          const int br = by_rows(lo_hist[1]);
          P = br < P ? br : P;
          P = P < last_total - 1 ? P : last_total - 1;
          if (P > published) {
            published = P;
            __hip_atomic_store(&a.progress[gi], P, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          }
        }
        // 3. store the rows final after step t-1
        if (t >= 1) {
          const int64_t nlo = final_after(t - 1);
          mv_store(lo, nlo);
          lo = nlo > lo ? nlo : lo;
        }
        lo_hist[2] = lo_hist[1];
        lo_hist[1] = lo_hist[0];
        lo_hist[0] = lo;
        CHASE_MARK_IF(mt == 0, gi, t, 4);
      } else {
        // 1. own loads of step t-1 complete; their rows (needed at step t+1) into the window
        __builtin_amdgcn_s_waitcnt(0);
        if (t >= 1) mv_fill(front_end(t), front_end(t + 1), regs);
        // 2. rows of step t+2
        wait_prev(t + 5);
        CHASE_MARK_IF(mt == 0, gi, t, 5);
        if (!s_flag) mv_load(front_end(t + 1), front_end(t + 2), regs);
        CHASE_MARK_IF(mt == 0, gi, t, 6);
      }
      __syncthreads();
      CHASE_MARK(gi, t, 2);
    }
    // epilogue: store the rest of the window, then mark the group complete
    if (storer) {
      __builtin_amdgcn_s_waitcnt(0);
      mv_store(lo, front_end(tend));
      __builtin_amdgcn_s_waitcnt(0);
    }
    __syncthreads();
    if (storer && mt == 0 && !s_flag)
      __hip_atomic_store(&a.progress[gi], last_total, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
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

static bool use_spec(int b, int W) { return b == 16 && W <= kSpecMaxW && chase_spec_lds_bytes(b, W) <= 159 * 1024; }
static bool use_window(int b, int W) {
  return !use_spec(b, W) && (b == 16 || b == 32) && chase_win_lds_bytes(b, W) <= 159 * 1024;
}

static const void* chase_fn(int b, int W) {
  if (use_spec(b, W)) return (const void*)k_chase_spec<16>;
  if (use_window(b, W)) return b == 16 ? (const void*)k_chase_win<16> : (const void*)k_chase_win<32>;
  return (const void*)k_chase;
}

static int chase_threads(int b, int W) {
  if (use_spec(b, W)) return 64 * (W + kSpecMovers);
  return use_window(b, W) ? 64 * (W > WinGeom<16>::MIN_WAVES ? W : WinGeom<16>::MIN_WAVES) : 64 * W;
}

static size_t chase_launch_lds(int b, int W) {
  if (use_spec(b, W)) return chase_spec_lds_bytes(b, W);
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
    if (fn == (const void*)k_chase_spec<16>) hipLaunchKernelGGL(k_chase_spec<16>, dim3(grid), block, lds, st, a);
    else if (fn == (const void*)k_chase_win<16>) hipLaunchKernelGGL(k_chase_win<16>, dim3(grid), block, lds, st, a);
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
