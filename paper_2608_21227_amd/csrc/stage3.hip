// Stage 3: singular values of the upper bidiagonal B = bidiag(d, e), float64.
// The paper names this step only ("and diagonal form"); the reading taken here
// is bisection on Sturm counts.  count(x) = #{sigma_i < x} is the number of
// negative pivots of the LDL^T factorisation of B^T B - x^2 I, obtained from
// B's entries by the stationary qd recurrence
//     s_1 = -x^2;  D+_i = d_i^2 + s_i;  s_{i+1} = e_i^2 s_i / D+_i - x^2,
// (a pivot smaller than pivmin in magnitude is replaced by -pivmin; pivmin is a
// power of two far below the rounding error, chosen so that no pivot or
// reciprocal leaves the normal range).
// Counts on a shared grid of 16 n points give every singular value a starting
// cell; a team of LPS lanes then multisects it: LPS interior points of the
// current interval per round, which shrink it by a factor LPS+1, until it is
// narrower than the tolerance (4u times the bound max|d| + max|e| on
// sigma_max for float64 output, 2^-32 times it for float32 output).
#include "common.hpp"
#include "kernels.hpp"
#include <float.h>

namespace svdv {

// work layout: dd[n], ee[n] (the squares of d and e scaled by 2^-k), then
// [2*n] = bound, [2*n+1] = pivmin, [2*n+2] = k, then the grid counts.
// d and e are scaled by the power of two 2^-k that brings max(|d|, |e|) into
// [0.5, 1) (exact), so that the squares and the pivot bounds below hold for any
// finite input; the output stage scales the values back by 2^k.
__device__ __forceinline__ void bisect_prep_body(const double* __restrict__ d, const double* __restrict__ e, int64_t n,
                                                 double* work) {
  __shared__ double smax[3][256];
  __shared__ int s_k;
  double md = 0.0, me = 0.0, bad = 0.0;
  for (int64_t i = threadIdx.x; i < n; i += blockDim.x) {
    const double di = d[i];
    const double ei = i + 1 < n ? e[i] : 0.0;
    md = fmax(md, fabs(di));
    me = fmax(me, fabs(ei));
    if (!isfinite(di) || !isfinite(ei)) bad = 1.0;
  }
  smax[0][threadIdx.x] = md;
  smax[1][threadIdx.x] = me;
  smax[2][threadIdx.x] = bad;
  __syncthreads();
  for (int s = blockDim.x / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s)
      for (int k = 0; k < 3; ++k) smax[k][threadIdx.x] = fmax(smax[k][threadIdx.x], smax[k][threadIdx.x + s]);
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const double mx = fmax(smax[0][0], smax[1][0]);
    s_k = (smax[2][0] == 0.0 && mx > 0.0) ? ilogb(mx) + 1 : 0;
  }
  __syncthreads();
  const int k = s_k;
  for (int64_t i = threadIdx.x; i < n; i += blockDim.x) {
    const double di = ldexp(d[i], -k);
    const double ei = i + 1 < n ? ldexp(e[i], -k) : 0.0;
    work[i] = di * di;
    work[n + i] = ei * ei;
  }
  if (threadIdx.x == 0) {
    // a NaN or an infinity in d or e: the bound is NaN, which every search stops
    // on at once and the output stage writes as NaN
    const double bound = smax[2][0] != 0.0 ? __builtin_nan("")
                                           : ldexp(smax[0][0] + smax[1][0], -k) * (1.0 + 1e-14) + DBL_MIN;
    work[2 * n] = bound;
    // pivmin = 2^p >= bound^2 2^-896.  With G = bound^2 >= d_i^2, e_i^2, x^2 every
    // |s_i| <= 2 G^2 / pivmin + G <= 2^897 G and every |D+_i| >= pivmin, so all
    // pivots and their reciprocals stay normal (G <= 4 after the scaling).  Pivots
    // this small are a perturbation far below the rounding error of the reduction.
    work[2 * n + 1] = isfinite(bound) ? ldexp(1.0, max(2 * ilogb(bound) + 2 - 896, -1000)) : 1.0;
    work[2 * n + 2] = (double)k;
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

// One step of the recurrence, s' = e^2 s / D+ - x^2, as fma(e^2 s, r, -x^2) with
// r = 1/D+ from the hardware reciprocal refined once by Newton's step: e^2 s is
// formed beside the reciprocal, so the dependent chain per step is the pivot, the
// reciprocal, its refinement and one fma.  Each operation has a relative error of
// a few units in the last place, which keeps the count's backward stability.
__device__ __forceinline__ double sturm_step(double s, double dp, double e2, double t) {
  const double es = e2 * s;
  double r = __builtin_amdgcn_rcp(dp);
  r = fma(r, fma(-dp, r, 1.0), r);
  return fma(es, r, -t);
}

// Sturm count of one shift x: the number of negative pivots (the choice of
// pivmin keeps every pivot and its reciprocal normal).  d_i^2 and e_i^2 are
// fetched 8 steps at a time (wave-uniform addresses, so scalar loads that are in
// flight while the previous 8 steps run).  pivmin is a power of two, so
// |D+| < pivmin is decided exactly on the high 32 bits of D+; the sign bit of
// the (possibly replaced) pivot is the count.
__device__ __forceinline__ int sturm_count(const double* __restrict__ dd, const double* __restrict__ ee, int64_t n,
                                           double x, double pivmin) {
  const double t = x * x;
  const uint32_t piv_hi = (uint32_t)(__double_as_longlong(pivmin) >> 32);
  const double negpiv = -pivmin;
  double s = -t;
  int cnt = 0;
  auto pivot = [&](double di) {
    double dp = di + s;
    const uint32_t hi = (uint32_t)(__double_as_longlong(dp) >> 32);
    const bool tiny = (hi & 0x7fffffffu) < piv_hi;
    dp = tiny ? negpiv : dp;
    cnt += tiny ? 1 : (int)(hi >> 31);
    return dp;
  };
  int64_t i = 0;
  for (; i + 8 < n; i += 8) {
    double dv[8], ev[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      dv[u] = dd[i + u];
      ev[u] = ee[i + u];
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) s = sturm_step(s, pivot(dv[u]), ev[u], t);
  }
  for (; i + 1 < n; ++i) s = sturm_step(s, pivot(dd[i]), ee[i], t);
  pivot(dd[n - 1]);  // last pivot (no e beyond it)
  return cnt;
}

// Shared count grid: counts at G = 16 n points x_g = bound (g + 1) / (G + 1),
// evaluated once for all values (one lane per point).  Every value's search then
// starts from the grid cell that holds it instead of from [0, bound], which
// saves the first rounds of multisection that all values would repeat.
__device__ __forceinline__ double grid_x(double bound, int64_t g, int64_t G) {
  return bound * (double)(g + 1) / (double)(G + 1);
}

__device__ __forceinline__ void bisect_grid_body(const double* __restrict__ work, int64_t n, int64_t g0) {
  const int64_t G = bisect_grid_points(n);
  const int64_t g = g0 + threadIdx.x;
  const double bound = work[2 * n], pivmin = work[2 * n + 1];
  const int c = sturm_count(work, work + n, n, grid_x(bound, g < G ? g : G - 1, G), pivmin);
  if (g < G) bisect_grid_counts(const_cast<double*>(work), n)[g] = c;
}

__global__ void __launch_bounds__(256) k_bisect_grid(const double* __restrict__ work, int64_t n) {
  bisect_grid_body(work, n, (int64_t)blockIdx.x * blockDim.x);
}

template <typename T>
__global__ void __launch_bounds__(256) k_bisect_grid_b(const BatchMat<T>* __restrict__ tab) {
  const BatchMat<T>& t = tab[blockIdx.y];
  const int64_t g0 = (int64_t)blockIdx.x * blockDim.x;
  if (g0 >= bisect_grid_points(t.N)) return;  // whole workgroup leaves together
  bisect_grid_body(t.work, t.N, g0);
}

// One team of lps lanes locates value k (k-th smallest) of the bidiagonal whose
// prepared work array is `work`; inactive teams (active = false) still take part
// in the wave-wide votes.
//  1. Grid search: an lps-ary search over the grid counts finds the cell
//     (x_{g-1}, x_g] with count(x_{g-1}) <= k < count(x_g) (x_{-1} = 0, x_G = bound).
//  2. Multisection: each round the team's lanes evaluate lps interior points of
//     the interval, which shrinks it (lps + 1)-fold, until it is narrower than
//     tol: 4u bound for float64 output, 2^-32 bound for float32 output (far
//     below float32's rounding of any value above 2^-8 sigma_max, and below the
//     float32 reduction's own error for every value).
template <typename T>
__device__ __forceinline__ void bisect_team(const double* __restrict__ work, int64_t n, T* __restrict__ S,
                                            const int* exp_in, int64_t k, bool active, int lps) {
  const double* dd = work;
  const double* ee = work + n;
  const int* gc = bisect_grid_counts(work, n);
  const int64_t G = bisect_grid_points(n);
  const double bound = active ? work[2 * n] : 0.0;
  const double pivmin = active ? work[2 * n + 1] : 0.0;
  const int lane = threadIdx.x & 63;
  const int team_in_wave = lane / lps, j = lane % lps;
  const int team_base = team_in_wave * lps;
  const uint64_t team_mask = (lps == 64) ? ~0ull : (((1ull << lps) - 1) << team_base);

  // 1. grid search, invariant count(lo_i) <= k < count(hi_i)
  int64_t lo_i = -1, hi_i = G;
  while (__any(active && hi_i - lo_i > 1)) {
    const int64_t m = hi_i - lo_i - 1;  // interior indices lo_i+1 .. hi_i-1
    const bool live = active && m > 0;
    const int64_t pj = lo_i + 1 + (j * m) / lps;
    const bool above = live && gc[pj] > k;
    const uint64_t ball = __ballot(above) & team_mask;
    if (live) {
      if (ball == 0) {
        lo_i = lo_i + 1 + ((int64_t)(lps - 1) * m) / lps;
      } else {
        const int f = __builtin_ctzll(ball) - team_base;
        hi_i = lo_i + 1 + ((int64_t)f * m) / lps;
        if (f > 0) lo_i = lo_i + 1 + ((int64_t)(f - 1) * m) / lps;
      }
    }
  }
  double lo = lo_i < 0 ? 0.0 : grid_x(bound, lo_i, G);
  double hi = hi_i >= G ? bound : grid_x(bound, hi_i, G);

  // 2. multisection
  const double npts = (double)(lps + 1);
  const double tol = sizeof(T) == 4 ? ldexp(bound, -32) : 4.0 * DBL_EPSILON * bound;
  for (int it = 0; it < 80; ++it) {
    // every lane of the wave runs the same number of rounds (wave-uniform control)
    const bool need = active && (hi - lo > tol);
    if (!__any(need)) break;
    const double x = lo + (hi - lo) * (double)(j + 1) / npts;
    const bool above = active && sturm_count(dd, ee, n, x, pivmin) > k;
    // first point (in x order) whose count exceeds k (counts increase with x)
    const uint64_t ball = __ballot(above) & team_mask;
    if (need) {
      if (ball == 0) {
        lo = lo + (hi - lo) * (npts - 1.0) / npts;
      } else {
        const int first = __builtin_ctzll(ball) - team_base;
        const double nhi = lo + (hi - lo) * (double)(first + 1) / npts;
        const double nlo = first == 0 ? lo : lo + (hi - lo) * (double)first / npts;
        lo = nlo;
        hi = nhi;
      }
    }
  }
  if (active && j == 0) {
    const int e = *exp_in;
    // NaN for an input with a NaN or an infinity (marked in the exponent at
    // staging, or in the bound by the preparation of d and e); otherwise the
    // value scaled back by the preparation's 2^k and the staging's 2^e
    S[n - 1 - k] = (e == kExpNonFinite || !isfinite(bound))
                       ? (T)__builtin_nan("")
                       : (T)ldexp(0.5 * (lo + hi), e + (int)work[2 * n + 2]);
  }
}

template <typename T>
__global__ void __launch_bounds__(256) k_bisect(const double* __restrict__ work, int64_t n, T* __restrict__ S,
                                                const int* exp_in, int lps, const int* fail_flag) {
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
// When fail_flag holds a nonzero value (a bounded wait of the batch's chase gave
// up) every output value of the batch is NaN.
template <typename T>
__global__ void __launch_bounds__(256) k_bisect_b(const BatchMat<T>* __restrict__ tab, const int* __restrict__ vmat,
                                                  const int64_t* __restrict__ voff, int64_t total, int lps,
                                                  const int* fail_flag) {
  const int lane = threadIdx.x & 63;
  const int teams_per_wave = 64 / lps;
  const int64_t v = ((int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6)) * teams_per_wave + lane / lps;
  const bool active = v < total;
  const int mi = active ? vmat[v] : 0;
  const BatchMat<T>& t = tab[mi];
  if (fail_flag != nullptr && *fail_flag != 0) {
    if (active && lane % lps == 0) t.S[t.N - 1 - (v - voff[mi])] = (T)__builtin_nan("");
    return;
  }
  bisect_team(t.work, t.N, t.S, t.exp, active ? v - voff[mi] : 0, active, lps);
}

// Lanes per value: about 64K lanes in all (one wave per SIMD) when there are
// enough values, at most 64 (one wave) per value.
static int bisect_lps(int64_t values) {
  int lps = 8;
  while (lps < 64 && (int64_t)lps * values < 65536) lps *= 2;
  return lps;
}

template <typename T>
hipError_t launch_bisect(const double* d, const double* e, int64_t n, T* S, double* work, const int* exp_in, int lps,
                         hipStream_t st, const int* fail_flag) {
  if (n <= 0) return hipSuccess;
  if (lps <= 0) lps = bisect_lps(n);
  if (lps != 8 && lps != 16 && lps != 32 && lps != 64) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_bisect_prep, dim3(1), dim3(256), 0, st, d, e, n, work);
  const int64_t G = bisect_grid_points(n);
  hipLaunchKernelGGL(k_bisect_grid, dim3((unsigned)((G + 255) / 256)), dim3(256), 0, st, work, n);
  const int teams_per_block = 256 / lps;
  const int64_t blocks = (n + teams_per_block - 1) / teams_per_block;
  hipLaunchKernelGGL(k_bisect<T>, dim3((unsigned)blocks), dim3(256), 0, st, work, n, S, exp_in, lps, fail_flag);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_bisect_batched(const BatchMat<T>* tab, int count, const int* vmat, const int64_t* voff, int64_t total,
                                 int64_t max_n, hipStream_t st, const int* fail_flag) {
  if (count <= 0 || total <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_bisect_prep_b<T>, dim3(count), dim3(256), 0, st, tab);
  const int64_t G = bisect_grid_points(max_n);
  hipLaunchKernelGGL(k_bisect_grid_b<T>, dim3((unsigned)((G + 255) / 256), (unsigned)count), dim3(256), 0, st, tab);
  const int lps = bisect_lps(total);
  const int teams_per_block = 256 / lps;
  const int64_t blocks = (total + teams_per_block - 1) / teams_per_block;
  hipLaunchKernelGGL(k_bisect_b<T>, dim3((unsigned)blocks), dim3(256), 0, st, tab, vmat, voff, total, lps,
                     fail_flag);
  return hipGetLastError();
}
template hipError_t launch_bisect_batched<float>(const BatchMat<float>*, int, const int*, const int64_t*, int64_t, int64_t,
                                                 hipStream_t, const int*);
template hipError_t launch_bisect_batched<double>(const BatchMat<double>*, int, const int*, const int64_t*, int64_t,
                                                  int64_t, hipStream_t, const int*);
template hipError_t launch_bisect<float>(const double*, const double*, int64_t, float*, double*, const int*, int,
                                         hipStream_t, const int*);
template hipError_t launch_bisect<double>(const double*, const double*, int64_t, double*, double*, const int*, int,
                                          hipStream_t, const int*);

}  // namespace svdv
