// Stage 3: singular values of the upper bidiagonal B = bidiag(d, e), float64.
// The paper names this step only ("and diagonal form"); the reading taken here
// is bisection on Sturm counts.  count(x) = #{sigma_i < x} is the number of
// negative pivots of the LDL^T factorisation of B^T B - x^2 I, obtained from
// B's entries by the stationary qd recurrence
//     s_1 = -x^2;  D+_i = d_i^2 + s_i;  s_{i+1} = e_i^2 s_i / D+_i - x^2,
// (a pivot smaller than pivmin in magnitude is replaced by -pivmin).
// Each singular value is located by multisection: a team of LPS lanes
// evaluates the count at LPS interior points of the current interval, which
// shrinks it by a factor LPS+1 per round, until it is narrower than 4u times
// the bound max|d| + max|e| on sigma_max.
#include "common.hpp"
#include "kernels.hpp"
#include <float.h>

namespace svdv {

// work layout: dd[n], ee[n], then [2*n] = bound, [2*n+1] = pivmin
__device__ __forceinline__ void bisect_prep_body(const double* __restrict__ d, const double* __restrict__ e, int64_t n,
                                                 double* work) {
  __shared__ double smax[3][256];
  double md = 0.0, me = 0.0, me2 = 0.0;
  for (int64_t i = threadIdx.x; i < n; i += blockDim.x) {
    const double di = d[i];
    const double ei = i + 1 < n ? e[i] : 0.0;
    work[i] = di * di;
    work[n + i] = ei * ei;
    md = fmax(md, fabs(di));
    me = fmax(me, fabs(ei));
    me2 = fmax(me2, ei * ei);
  }
  smax[0][threadIdx.x] = md;
  smax[1][threadIdx.x] = me;
  smax[2][threadIdx.x] = me2;
  __syncthreads();
  for (int s = blockDim.x / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s)
      for (int k = 0; k < 3; ++k) smax[k][threadIdx.x] = fmax(smax[k][threadIdx.x], smax[k][threadIdx.x + s]);
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    work[2 * n] = (smax[0][0] + smax[1][0]) * (1.0 + 1e-14) + DBL_MIN;
    work[2 * n + 1] = DBL_MIN * fmax(1.0, smax[2][0]);
  }
}

__global__ void k_bisect_prep(const double* __restrict__ d, const double* __restrict__ e, int64_t n, double* work) {
  bisect_prep_body(d, e, n, work);
}
template <typename T>
__global__ void k_bisect_prep_b(const BatchMat<T>* __restrict__ tab) {
  const BatchMat<T>& t = tab[blockIdx.x];
  bisect_prep_body(t.d, t.e, t.N, t.work);
}

__device__ __forceinline__ int sturm_count(const double* __restrict__ dd, const double* __restrict__ ee, int64_t n,
                                           double x, double pivmin) {
  const double t = x * x;
  double s = -t;
  int cnt = 0;
  for (int64_t i = 0; i + 1 < n; ++i) {
    double dp = dd[i] + s;
    if (fabs(dp) < pivmin) dp = -pivmin;
    cnt += dp < 0.0;
    s = ee[i] * (s / dp) - t;
  }
  double dp = dd[n - 1] + s;
  if (fabs(dp) < pivmin) dp = -pivmin;
  cnt += dp < 0.0;
  return cnt;
}

// One team of lps lanes locates value k (k-th smallest) of the bidiagonal whose
// prepared work array is `work`; inactive teams (active = false) still take part
// in the wave-wide votes.
template <typename T>
__device__ __forceinline__ void bisect_team(const double* __restrict__ work, int64_t n, T* __restrict__ S,
                                            const int* exp_in, int64_t k, bool active, int lps) {
  const double* dd = work;
  const double* ee = work + n;
  const double bound = active ? work[2 * n] : 0.0;
  const double pivmin = active ? work[2 * n + 1] : 0.0;
  const int lane = threadIdx.x & 63;
  const int team_in_wave = lane / lps, j = lane % lps;
  double lo = 0.0, hi = bound;
  const double tol = 4.0 * DBL_EPSILON * bound;
  const uint64_t team_mask = (lps == 64) ? ~0ull : (((1ull << lps) - 1) << (team_in_wave * lps));
  for (int it = 0; it < 80; ++it) {
    // every lane of the wave runs the same number of rounds (wave-uniform control)
    const bool need = active && (hi - lo > tol);
    if (!__any(need)) break;
    const double x = lo + (hi - lo) * (double)(j + 1) / (double)(lps + 1);
    const int cnt = active ? sturm_count(dd, ee, n, x, pivmin) : 0;
    const uint64_t ball = __ballot(cnt > k) & team_mask;
    if (need) {
      if (ball == 0) {
        lo = lo + (hi - lo) * (double)lps / (double)(lps + 1);
      } else {
        const int first = __builtin_ctzll(ball) - team_in_wave * lps;  // smallest point with count > k
        const double nhi = lo + (hi - lo) * (double)(first + 1) / (double)(lps + 1);
        const double nlo = first == 0 ? lo : lo + (hi - lo) * (double)first / (double)(lps + 1);
        lo = nlo;
        hi = nhi;
      }
    }
  }
  if (active && j == 0) {
    const int e = *exp_in;
    S[n - 1 - k] = (T)ldexp(0.5 * (lo + hi), e);
  }
}

template <typename T>
__global__ void k_bisect(const double* __restrict__ work, int64_t n, T* __restrict__ S, const int* exp_in, int lps,
                         const int* fail_flag) {
  const int lane = threadIdx.x & 63;
  const int teams_per_wave = 64 / lps;
  const int64_t k = ((int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6)) * teams_per_wave + lane / lps;
  if (fail_flag != nullptr && *fail_flag != 0) {  // the bidiagonal is not valid: fail loudly
    if (k < n && lane % lps == 0) S[n - 1 - k] = (T)__builtin_nan("");
    return;
  }
  bisect_team(work, n, S, exp_in, k, k < n, lps);
}

// Batched form: value v of the flattened batch belongs to matrix vmat[v] as its
// value v - voff[vmat[v]].
template <typename T>
__global__ void k_bisect_b(const BatchMat<T>* __restrict__ tab, const int* __restrict__ vmat,
                           const int64_t* __restrict__ voff, int64_t total, int lps) {
  const int lane = threadIdx.x & 63;
  const int teams_per_wave = 64 / lps;
  const int64_t v = ((int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6)) * teams_per_wave + lane / lps;
  const bool active = v < total;
  const int mi = active ? vmat[v] : 0;
  const BatchMat<T>& t = tab[mi];
  bisect_team(t.work, t.N, t.S, t.exp, active ? v - voff[mi] : 0, active, lps);
}

template <typename T>
hipError_t launch_bisect(const double* d, const double* e, int64_t n, T* S, double* work, const int* exp_in, int lps,
                         hipStream_t st, const int* fail_flag) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_bisect_prep, dim3(1), dim3(256), 0, st, d, e, n, work);
  const int teams_per_block = 256 / lps;
  const int64_t blocks = (n + teams_per_block - 1) / teams_per_block;
  hipLaunchKernelGGL(k_bisect<T>, dim3((unsigned)blocks), dim3(256), 0, st, work, n, S, exp_in, lps, fail_flag);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_bisect_batched(const BatchMat<T>* tab, int count, const int* vmat, const int64_t* voff, int64_t total,
                                 int lps, hipStream_t st) {
  if (count <= 0 || total <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_bisect_prep_b<T>, dim3(count), dim3(256), 0, st, tab);
  const int teams_per_block = 256 / lps;
  const int64_t blocks = (total + teams_per_block - 1) / teams_per_block;
  hipLaunchKernelGGL(k_bisect_b<T>, dim3((unsigned)blocks), dim3(256), 0, st, tab, vmat, voff, total, lps);
  return hipGetLastError();
}
template hipError_t launch_bisect_batched<float>(const BatchMat<float>*, int, const int*, const int64_t*, int64_t, int,
                                                 hipStream_t);
template hipError_t launch_bisect_batched<double>(const BatchMat<double>*, int, const int*, const int64_t*, int64_t,
                                                  int, hipStream_t);
template hipError_t launch_bisect<float>(const double*, const double*, int64_t, float*, double*, const int*, int,
                                         hipStream_t, const int*);
template hipError_t launch_bisect<double>(const double*, const double*, int64_t, double*, double*, const int*, int,
                                          hipStream_t, const int*);

}  // namespace svdv
