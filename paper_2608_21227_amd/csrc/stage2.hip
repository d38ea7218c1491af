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
// Groups are handed out round-robin to a persistent grid; group g waits for
// group g-1's last sweep through a progress counter.  Band data crosses
// workgroups (and XCDs, whose L2 caches are not coherent with each other), so
// every band access is a relaxed device-scope atomic (coherent at device
// level), and progress is published only after the step's stores completed.
#include "common.hpp"
#include "kernels.hpp"

namespace svdv {

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
      scal = 1.0 / (alpha - beta);
      tau = (beta - alpha) / beta;
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
      scal = 1.0 / (alpha - beta);
      tau = (beta - alpha) / beta;
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

__device__ __forceinline__ int ntasks_of(int64_t s, int64_t n, int b) {
  if (s >= n - 1) return 0;
  return (int)((n - 1 - s + b - 1) / b);
}

size_t chase_lds_bytes(int b, int W) {
  // per wave: a 64 x (b+1) tile (also used as b x 65 for the left part) + b reflector entries
  const int tile = 64 * (b + 1) > b * 65 ? 64 * (b + 1) : b * 65;
  return (size_t)W * (tile + b) * sizeof(double);
}

__global__ void k_chase(ChaseArgs a) {
  extern __shared__ __align__(16) double lds[];
  const int wv = threadIdx.x >> 6;
  const int W = a.W;
  const int b = a.b;
  const int tile_elems = 64 * (b + 1) > b * 65 ? 64 * (b + 1) : b * 65;
  double* tile = lds + (size_t)wv * (tile_elems + b);
  double* vb = tile + tile_elems;
  ChaseCtx X{a.Bs, a.ldb, a.n, b, b - 1};
  const int64_t n = a.n;
  __shared__ int s_giveup;

  for (int gi = blockIdx.x; gi < a.ngroups; gi += gridDim.x) {
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
  static constexpr int RS = 3 * B + 1;  // LDS slot stride (odd: fewer bank conflicts)
  // the windowed kernel always runs at least 4 waves (the extra ones only move rows)
  static constexpr int MIN_WAVES = 4;
  static constexpr int PF = (B * RW + 64 * MIN_WAVES - 1) / (64 * MIN_WAVES);  // prefetch registers per thread
};

__host__ __device__ inline int win_rows(int b, int W) { return (3 * W + 2) * b + 2; }

size_t chase_win_lds_bytes(int b, int W) {
  if (b != 16 && b != 32) return (size_t)1 << 40;
  return ((size_t)win_rows(b, W) * (3 * b + 1) + (size_t)(W > 4 ? W : 4) * 64) * sizeof(double);
}

template <int B>
__device__ __forceinline__ double& welem(double* win, int R, int64_t i, int64_t j) {
  return win[(int)((uint64_t)i % (uint64_t)R) * WinGeom<B>::RS + (int)(j - i + WinGeom<B>::LO)];
}

template <int B>
__device__ void win_task(double* win, int R, int64_t n, int64_t p, int64_t c, double* vb) {
  constexpr int RS = WinGeom<B>::RS, LO = WinGeom<B>::LO;
  const int lane = threadIdx.x & 63;
  const int L = (int)((n - c) < B ? (n - c) : B);
  const int64_t rend = c + L < n ? c + L : n;
  const int64_t cend = c + L + B < n ? c + L + B : n;

  // right reflector on row p, columns c..c+L-1
  double x = lane < L ? welem<B>(win, R, p, c + lane) : 0.0;
  double ss = wave_sum((lane >= 1 && lane < L) ? x * x : 0.0);
  double alpha = __shfl(x, 0, kWave);
  double beta = alpha, tau = 0.0, scal = 0.0;
  if (ss > 0.0) {
    const double nrm = sqrt(alpha * alpha + ss);
    beta = alpha >= 0.0 ? -nrm : nrm;
    scal = 1.0 / (alpha - beta);
    tau = (beta - alpha) / beta;
  }
  if (lane < L) {
    vb[lane] = lane == 0 ? 1.0 : x * scal;
    welem<B>(win, R, p, c + lane) = lane == 0 ? beta : 0.0;
  }
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  if (tau != 0.0) {
    const int64_t r = p + 1 + lane;
    if (r < rend) {
      double* row = win + (int)((uint64_t)r % (uint64_t)R) * RS + (int)(c - r + LO);
      double dot = 0.0;
#pragma unroll 8
      for (int l = 0; l < L; ++l) dot += row[l] * vb[l];
      const double td = tau * dot;
#pragma unroll 8
      for (int l = 0; l < L; ++l) row[l] -= td * vb[l];
    }
  }
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");

  // left reflector on column c, rows c..c+L-1
  x = lane < L ? welem<B>(win, R, c + lane, c) : 0.0;
  ss = wave_sum((lane >= 1 && lane < L) ? x * x : 0.0);
  alpha = __shfl(x, 0, kWave);
  beta = alpha;
  tau = 0.0;
  scal = 0.0;
  if (ss > 0.0) {
    const double nrm = sqrt(alpha * alpha + ss);
    beta = alpha >= 0.0 ? -nrm : nrm;
    scal = 1.0 / (alpha - beta);
    tau = (beta - alpha) / beta;
  }
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  if (lane < L) {
    vb[lane] = lane == 0 ? 1.0 : x * scal;
    welem<B>(win, R, c + lane, c) = lane == 0 ? beta : 0.0;
  }
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  if (tau != 0.0) {
    const int64_t q = c + 1 + lane;
    if (q < cend) {
      const int sc = (int)((uint64_t)c % (uint64_t)R);
      double dot = 0.0;
      for (int l = 0; l < L; ++l) {
        int sl = sc + l;
        sl = sl >= R ? sl - R : sl;
        dot += vb[l] * win[sl * RS + (int)(q - c - l + LO)];
      }
      const double td = tau * dot;
      for (int l = 0; l < L; ++l) {
        int sl = sc + l;
        sl = sl >= R ? sl - R : sl;
        win[sl * RS + (int)(q - c - l + LO)] -= td * vb[l];
      }
    }
  }
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
}

// First row the (unfinished) sweep s0+i will touch at its task j (j <= 0: it has not started).
__device__ __forceinline__ int64_t sweep_front(int64_t s, int j, int b) {
  return j <= 0 ? s : s + 1 + (int64_t)(j - 1) * b;
}

template <int B>
__global__ void __launch_bounds__(512) k_chase_win(ChaseArgs a) {
  constexpr int RW = WinGeom<B>::RW, RS = WinGeom<B>::RS, PF = WinGeom<B>::PF;
  extern __shared__ __align__(16) double lds[];
  const int W = a.W;
  const int R = win_rows(B, W);
  double* win = lds;
  const int wv = threadIdx.x >> 6;
  double* vb = lds + (size_t)R * RS + wv * 64;
  const int nthr = blockDim.x;
  const int tid = threadIdx.x;
  const int64_t n = a.n;
  __shared__ int s_giveup;

  for (int gi = blockIdx.x; gi < a.ngroups; gi += gridDim.x) {
    const int64_t s0 = (int64_t)gi * W;
    const int nsw = (int)((n - 1 - s0) < W ? (n - 1 - s0) : W);
    int tend = 0;
    for (int i = 0; i < nsw; ++i) {
      const int te = 3 * i + ntasks_of(s0 + i, n, B);
      tend = te > tend ? te : tend;
    }
    const int prev_total = gi > 0 ? ntasks_of(s0 - 1, n, B) : 0;
    const int last_total = ntasks_of(s0 + nsw - 1, n, B);
    const int first_total = ntasks_of(s0, n, B);
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
      win[(int)((uint64_t)r % (uint64_t)R) * RS + col] = bld(a.Bs + r * a.ldb + col);
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
        if (jt >= 0 && jt < ntasks_of(s, n, B)) {
          const int64_t c = s + 1 + (int64_t)jt * B;
          const int64_t p = jt == 0 ? s : c - B;
          win_task<B>(win, R, n, p, c, vb);
        }
      }
      __syncthreads();
      // write back rows no unfinished sweep of the group touches again
      // (the minimum over all unfinished sweeps: a sweep that has not started yet
      // still needs its own first row)
      int64_t nlo = n;
      for (int i = 0; i < nsw; ++i) {
        const int jn = t + 1 - 3 * i;
        if (jn < ntasks_of(s0 + i, n, B)) {
          const int64_t f = sweep_front(s0 + i, jn, B);
          nlo = f < nlo ? f : nlo;
        }
      }
      nlo = nlo < hi ? nlo : hi;
      for (int64_t e = tid; e < (nlo - lo) * RW; e += nthr) {
        const int64_t r = lo + e / RW;
        const int col = (int)(e % RW);
        bst(a.Bs + r * a.ldb + col, win[(int)((uint64_t)r % (uint64_t)R) * RS + col]);
      }
      lo = nlo;
#pragma unroll
      for (int k = 0; k < PF; ++k) {
        const int64_t e = tid + (int64_t)k * nthr;
        if (e < npf) {
          const int64_t r = hi + e / RW;
          win[(int)((uint64_t)r % (uint64_t)R) * RS + (int)(e % RW)] = pf[k];
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
      bst(a.Bs + r * a.ldb + col, win[(int)((uint64_t)r % (uint64_t)R) * RS + col]);
    }
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    if (threadIdx.x == 0)
      __hip_atomic_store(&a.progress[gi], last_total, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __syncthreads();
  }
}

// d_i = B(i, i), e_i = B(i, i+1) once every sweep has finished (next kernel in the stream).
__global__ void k_chase_extract(const double* __restrict__ Bs, int64_t ldb, int64_t n, int b, double* d, double* e) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    d[i] = Bs[i * ldb + (b - 1)];
    if (i + 1 < n) e[i] = Bs[i * ldb + b];
  }
}

static bool use_window(int b, int W) { return (b == 16 || b == 32) && chase_win_lds_bytes(b, W) <= 159 * 1024; }

static const void* chase_fn(int b, int W) {
  if (use_window(b, W)) return b == 16 ? (const void*)k_chase_win<16> : (const void*)k_chase_win<32>;
  return (const void*)k_chase;
}

static int chase_threads(int b, int W) {
  return use_window(b, W) ? 64 * (W > WinGeom<16>::MIN_WAVES ? W : WinGeom<16>::MIN_WAVES) : 64 * W;
}

static size_t chase_launch_lds(int b, int W) { return use_window(b, W) ? chase_win_lds_bytes(b, W) : chase_lds_bytes(b, W); }

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

hipError_t launch_chase(const ChaseArgs& a, int grid, hipStream_t st) {
  const void* fn = chase_fn(a.b, a.W);
  const size_t lds = chase_launch_lds(a.b, a.W);
  hipError_t e = chase_set_lds(fn, lds);
  if (e != hipSuccess) return e;
  if (a.n > 1) {
    hipLaunchKernelGGL(k_fill_i32, dim3(64), dim3(256), 0, st, a.progress, 0, (int64_t)a.ngroups + 1);
    const dim3 block(chase_threads(a.b, a.W));
    if (fn == (const void*)k_chase_win<16>) hipLaunchKernelGGL(k_chase_win<16>, dim3(grid), block, lds, st, a);
    else if (fn == (const void*)k_chase_win<32>) hipLaunchKernelGGL(k_chase_win<32>, dim3(grid), block, lds, st, a);
    else hipLaunchKernelGGL(k_chase, dim3(grid), block, lds, st, a);
  }
  const int g = (int)((a.n + 255) / 256);
  hipLaunchKernelGGL(k_chase_extract, dim3(g < 1 ? 1 : (g > 4096 ? 4096 : g)), dim3(256), 0, st, a.Bs, a.ldb, a.n,
                     a.b, a.d, a.e);
  return hipGetLastError();
}

}  // namespace svdv
