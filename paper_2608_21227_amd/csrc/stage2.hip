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
            if (__builtin_amdgcn_s_memrealtime() - t0 > 1000000000ull) {  // 10 s at 100 MHz
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

// d_i = B(i, i), e_i = B(i, i+1) once every sweep has finished (next kernel in the stream).
__global__ void k_chase_extract(const double* __restrict__ Bs, int64_t ldb, int64_t n, int b, double* d, double* e) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    d[i] = Bs[i * ldb + (b - 1)];
    if (i + 1 < n) e[i] = Bs[i * ldb + b];
  }
}

static hipError_t chase_set_lds(size_t lds) {
  static size_t configured = 0;
  if (lds > configured) {
    hipError_t e = hipFuncSetAttribute((const void*)k_chase, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    configured = lds;
  }
  return hipSuccess;
}

int chase_max_groups_resident(int b, int W) {
  int dev = 0, cus = 0, per = 0;
  const size_t lds = chase_lds_bytes(b, W);
  if (chase_set_lds(lds) != hipSuccess) return 0;
  if (hipGetDevice(&dev) != hipSuccess) return 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, (const void*)k_chase, W * 64, lds) != hipSuccess) return 0;
  return per * cus;
}

hipError_t launch_chase(const ChaseArgs& a, int grid, hipStream_t st) {
  const size_t lds = chase_lds_bytes(a.b, a.W);
  hipError_t e = chase_set_lds(lds);
  if (e != hipSuccess) return e;
  if (a.n > 1) {
    hipLaunchKernelGGL(k_fill_i32, dim3(64), dim3(256), 0, st, a.progress, 0, (int64_t)a.ngroups + 1);
    hipLaunchKernelGGL(k_chase, dim3(grid), dim3(a.W * 64), lds, st, a);
  }
  const int g = (int)((a.n + 255) / 256);
  hipLaunchKernelGGL(k_chase_extract, dim3(g < 1 ? 1 : (g > 4096 ? 4096 : g)), dim3(256), 0, st, a.Bs, a.ldb, a.n,
                     a.b, a.d, a.e);
  return hipGetLastError();
}

}  // namespace svdv
