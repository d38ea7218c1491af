// Stage 1 of the two-stage singular-value method: reduction of a dense matrix to
// upper band form with bandwidth TS (Algorithm 1 of the paper).  For every
// diagonal tile k: QR sweep (panel factorisation of the tile column, then the
// trailing update from the left) and LQ sweep (the same on the tile row, applied
// from the right).  The LQ sweep runs the same kernels on the transposed view.
//
// Panel factorisation (the paper's GEQRT/TSQRT step): a tall-skinny QR done as a
// tree.  Level-1 chunks of up to 64*RPT rows are factored independently, one
// workgroup each, with the chunk held in registers; the R factors of a level are
// stacked and factored again at the next level until one chunk remains.  Every
// level stores its Householder vectors V (unit lower trapezoidal) and the
// compact-WY factor T (Q = I - V T V^T).
//
// Trailing update (the paper's UNMQR/TSMQR step, Algorithm 2): C <- Q^T C per
// chunk and per level, in compact-WY form C -= V (T^T (V^T C)), with the three
// products on the MFMA units.  Each wave owns IB 16-column tiles and walks the
// chunk's rows twice (V^T C, then the rank-k update); nothing is shared between
// waves, so no LDS and no barriers are needed.
#include <algorithm>
#include <type_traits>

#include "common.hpp"
#include "kernels.hpp"

namespace svdv {

// Optional phase trace of the panel kernel (diagnostic builds only, -DSVDV_PANEL_TRACE):
// for each of the first 4096 launches of workgroup 0, five timestamps of the 100 MHz counter.
#ifdef SVDV_PANEL_TRACE
__device__ uint64_t g_panel_trace[5 * 4096];
__device__ int g_panel_calls;
#define PANEL_MARK(slot, k)                                                        \
  do {                                                                             \
    if (threadIdx.x == 0 && (slot) >= 0 && (slot) < 4096)                          \
      g_panel_trace[(slot) * 5 + (k)] = __builtin_amdgcn_s_memrealtime();          \
  } while (0)
#else
#define PANEL_MARK(slot, k) \
  do {                      \
  } while (0)
#endif

__global__ void k_fill_u64(unsigned long long* p, unsigned long long v, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) p[i] = v;
}
__global__ void k_fill_i32(int* p, int v, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) p[i] = v;
}
__global__ void k_fill_f64(double* p, double v, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) p[i] = v;
}
// d[0 .. n) and e[0 .. n-1) of stage 2 run alone: NaN when *flag is nonzero (a
// non-finite band, or a chase that gave up a bounded wait), so no caller reads them
// as valid; otherwise scaled back by 2^(*exp), the power of two the band was scaled by.
__global__ void k_finish_de(const int* flag, const int* exp, double* d, double* e, int64_t n) {
  const bool bad = *flag != 0;
  const int k = bad ? 0 : *exp;
  const double q = __builtin_nan("");
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    d[i] = bad ? q : ldexp(d[i], k);
    if (i + 1 < n) e[i] = bad ? q : ldexp(e[i], k);
  }
}

// ---------------------------------------------------------------------------
// a1: input staging -- max |a|, then copy (optionally transposed) scaled by 2^-e
// ---------------------------------------------------------------------------

__device__ __forceinline__ unsigned long long abs_bits(double x) {
  return (unsigned long long)__double_as_longlong(fabs(x));
}

template <typename T>
__device__ __forceinline__ void absmax_body(const T* __restrict__ A, int64_t m, int64_t n, int64_t lda,
                                            unsigned long long* out) {
  double mx = 0.0;
  int64_t total = m * n;
  for (int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; idx < total; idx += (int64_t)gridDim.x * blockDim.x) {
    int64_t j = idx / m, i = idx - j * m;
    double v = fabs((double)A[i + j * lda]);
    if (v != v || v > mx) mx = v;  // a NaN, once met, stays (no comparison replaces it)
  }
  unsigned long long b = abs_bits(mx);
  for (int off = 32; off > 0; off >>= 1) {
    unsigned long long o = __shfl_xor(b, off, kWave);
    b = o > b ? o : b;
  }
  __shared__ unsigned long long wmax[16];
  if ((threadIdx.x & 63) == 0) wmax[threadIdx.x >> 6] = b;
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int w = 1; w < (int)(blockDim.x >> 6); ++w) b = wmax[w] > b ? wmax[w] : b;
    atomicMax(out, b);
  }
}
template <typename T>
__global__ void k_absmax(const T* __restrict__ A, int64_t m, int64_t n, int64_t lda, unsigned long long* out) {
  absmax_body(A, m, n, lda, out);
}

// exponent e with max*2^-e in [0.5, 1); 0 if max is zero or not finite
__device__ __forceinline__ int scale_exponent(unsigned long long bits) {
  double mx = __longlong_as_double((long long)bits);
  if (!(mx > 0.0) || !isfinite(mx)) return 0;
  int e;
  frexp(mx, &e);
  return e;
}

template <typename T>
__device__ __forceinline__ void copy_scale_body(const T* __restrict__ A, int64_t m, int64_t n, int64_t lda,
                                                int transpose, T* __restrict__ W, int64_t ldw,
                                                const unsigned long long* amax, int* exp_out) {
  int e = scale_exponent(*amax);
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    const double mx = __longlong_as_double((long long)*amax);
    *exp_out = isfinite(mx) ? e : kExpNonFinite;  // the data is copied unscaled either way
  }
  // W is M x N with M = transpose ? n : m
  int64_t M = transpose ? n : m, N = transpose ? m : n;
  int64_t total = M * N;
  for (int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; idx < total; idx += (int64_t)gridDim.x * blockDim.x) {
    int64_t j = idx / M, i = idx - j * M;
    T v = transpose ? A[j + i * lda] : A[i + j * lda];
    W[i + j * ldw] = (T)ldexp((double)v, -e);
  }
}
template <typename T>
__global__ void k_copy_scale(const T* __restrict__ A, int64_t m, int64_t n, int64_t lda, int transpose,
                             T* __restrict__ W, int64_t ldw, const unsigned long long* amax, int* exp_out) {
  copy_scale_body(A, m, n, lda, transpose, W, ldw, amax, exp_out);
}

// ---------------------------------------------------------------------------
// a2/a4: chunk QR (one TSQR chunk per workgroup, chunk in registers)
// ---------------------------------------------------------------------------
//
// Thread layout: NW = 16 waves; wave w owns columns [w*CPT, (w+1)*CPT); lane l
// owns rows q = i*64 + l, i < RPT.  Column sums are wave reductions.

template <typename TC, int TILE, int RPT>
struct ChunkQRCfg {
  static constexpr int NW = 16;
  static constexpr int CPT = TILE / NW;
  static constexpr int HMAX = 64 * RPT;
  // 64-row blocks transposed per barrier pair when loading (stage area <= 64 KiB)
  static constexpr int CQB0 = (64 * 1024) / (64 * (TILE + 1) * (int)sizeof(TC));
  static constexpr int CQB = CQB0 >= RPT ? RPT : (CQB0 >= 8 ? 8 : (CQB0 >= 4 ? 4 : (CQB0 >= 2 ? 2 : 1)));
};

// T: storage type of the matrix, V and T factors; TC: arithmetic type of the
// factorisation (float64 for float32 storage when the trailing updates run in
// BF16/FP16: the panel factorisation itself stays float64 there).
template <typename T, int TILE, int RPT, typename TC = T>
__device__ __forceinline__ void chunk_qr_body(const ChunkQRArgs<T>& a, const int c) {
  typedef ChunkQRCfg<TC, TILE, RPT> C;
  constexpr int CPT = C::CPT;
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
  const int64_t row0 = (int64_t)c * a.chunk_rows;
  const int Hc = (int)(c == a.P - 1 ? a.h - row0 : a.chunk_rows);
  const int bw = a.bw;
  const int kr = Hc < bw ? Hc : bw;

  extern __shared__ __align__(16) unsigned char smem_raw[];
  // LDS: stage [CQB*64][TILE+1] (also reused as Mtmp at the end) | vbuf[2][HMAX] | taus[TILE] | Tl[TILE][TILE+1]
  TC* stage = reinterpret_cast<TC*>(smem_raw);
  TC* Mtmp = stage;
  TC* vbuf = stage + C::CQB * 64 * (TILE + 1);
  TC* taus = vbuf + 2 * C::HMAX;
  TC* Tl = taus + TILE;
  constexpr int LDT = TILE + 1;

  TC x[RPT][CPT];

#ifdef SVDV_PANEL_TRACE
  __shared__ int s_slot;
  if (threadIdx.x == 0) s_slot = (blockIdx.x == 0 && c == 0) ? atomicAdd(&g_panel_calls, 1) : -1;
  __syncthreads();
  const int slot = s_slot;
#else
  const int slot = -1;
#endif
  PANEL_MARK(slot, 0);
  // ---- load the chunk, with the global loads issued in bursts ----
  // rows contiguous (QR sweep): lane l reads rows i*64+l of its columns directly
  // (coalesced along rows).  Otherwise (LQ sweep) threads read along the
  // memory-contiguous columns and the blocks are transposed through LDS, CQB
  // 64-row blocks (loaded together) per barrier pair.
  auto fetch = [&](int q, int col) -> TC {
    TC v = TC(0);
    if (q < Hc && col < bw) {
      v = (TC)a.M.at(a.rm.row(c, q), a.pc + col);
      if (a.rm.per_unit != 0 && (q % a.rm.per_unit) > col) v = TC(0);
    }
    return v;
  };
  if (a.M.rs == 1) {
#pragma unroll
    for (int i = 0; i < RPT; ++i)
#pragma unroll
      for (int cc = 0; cc < CPT; ++cc) x[i][cc] = fetch(i * 64 + l, w * CPT + cc);
  } else {
    constexpr int EPT = TILE / 16;  // elements of one 64 x TILE block per thread
    constexpr int CQB = C::CQB;
    // the next group of blocks is requested before this one goes through LDS, so
    // the global loads of consecutive groups overlap instead of queueing
    TC tmp[CQB][EPT], nxt[CQB][EPT];
#pragma unroll
    for (int ib = 0; ib < CQB; ++ib)
#pragma unroll
      for (int k = 0; k < EPT; ++k) {
        const int t = threadIdx.x + k * 1024;
        tmp[ib][k] = fetch(ib * 64 + t / TILE, t % TILE);
      }
#pragma unroll
    for (int i0 = 0; i0 < RPT; i0 += CQB) {
      if (i0 + CQB < RPT) {
#pragma unroll
        for (int ib = 0; ib < CQB; ++ib)
#pragma unroll
          for (int k = 0; k < EPT; ++k) {
            const int t = threadIdx.x + k * 1024;
            nxt[ib][k] = fetch((i0 + CQB + ib) * 64 + t / TILE, t % TILE);
          }
      }
#pragma unroll
      for (int ib = 0; ib < CQB; ++ib)
#pragma unroll
        for (int k = 0; k < EPT; ++k) {
          const int t = threadIdx.x + k * 1024;
          stage[(ib * 64 + t / TILE) * (TILE + 1) + t % TILE] = tmp[ib][k];
        }
      __syncthreads();
#pragma unroll
      for (int ib = 0; ib < CQB; ++ib)
#pragma unroll
        for (int cc = 0; cc < CPT; ++cc) x[i0 + ib][cc] = stage[(ib * 64 + l) * (TILE + 1) + w * CPT + cc];
      __syncthreads();
      if (i0 + CQB < RPT) {
#pragma unroll
        for (int ib = 0; ib < CQB; ++ib)
#pragma unroll
          for (int k = 0; k < EPT; ++k) tmp[ib][k] = nxt[ib][k];
      }
    }
  }

  PANEL_MARK(slot, 1);
  // Compact-WY factor T (upper triangular, LAPACK's forward columnwise form):
  // T[j][j] = tau_j and T[0:j, j] = -tau_j T[0:j, 0:j] Y[0:j, j] with
  // Y[k][j] = v_k^T v_j, which the column loop collects in Tl's strict upper
  // part during iteration j.  For tiles up to 32 wave 0 forms column j-1 of T
  // right after the barrier of iteration j (its own columns are finished by
  // then, or nearly), lane i holding row i of T in registers, so T costs no
  // time of its own; wider tiles build T after the loop by recursive doubling.
  constexpr bool kTinLoop = TILE <= 32;
  TC trow[kTinLoop ? TILE : 1];
#pragma unroll
  for (int k = 0; k < (kTinLoop ? TILE : 1); ++k) trow[k] = TC(0);
  auto t_column = [&](int jj) {
    if constexpr (kTinLoop) {
      const TC tj = taus[jj];
      TC acc = TC(0);
#pragma unroll
      for (int k = 0; k < TILE; ++k)
        if (k < jj && k >= l) acc += trow[k] * Tl[k * LDT + jj];
      const TC val = l < jj ? -tj * acc : (l == jj ? tj : TC(0));
#pragma unroll
      for (int k = 0; k < TILE; ++k)
        if (k == jj) trow[k] = val;
    }
  };
  // ---- Householder loop over the panel columns ----
  for (int j = 0; j < kr; ++j) {
    const int ow = j / CPT, oc = j % CPT;
    TC* vb = vbuf + (j & 1) * C::HMAX;
    if (w == ow) {
      double sp[4] = {0.0, 0.0, 0.0, 0.0}, alpha_l = 0.0;
#pragma unroll
      for (int i = 0; i < RPT; ++i) {
        const int q = i * 64 + l;
        double v = 0.0;
#pragma unroll
        for (int cc = 0; cc < CPT; ++cc) if (cc == oc) v = (double)x[i][cc];
        if (q > j) sp[i & 3] += v * v;
        if (q == j) alpha_l = v;
      }
      const double ss = wave_sum((sp[0] + sp[1]) + (sp[2] + sp[3]));
      const double alpha = lane_value(alpha_l, j & 63);
      double beta = alpha, tau = 0.0, scal = 0.0;
      if (ss > 0.0) {
        const double nrm = sqrt(alpha * alpha + ss);
        beta = alpha >= 0.0 ? -nrm : nrm;
        // divisors >= sqrt(ss) >= 2^-537, normal with normal reciprocals
        tau = nr_div(beta - alpha, beta);
        scal = nr_div(1.0, alpha - beta);
      }
#pragma unroll
      for (int i = 0; i < RPT; ++i) {
        const int q = i * 64 + l;
#pragma unroll
        for (int cc = 0; cc < CPT; ++cc) {
          if (cc != oc) continue;
          TC v = x[i][cc];
          TC vv;
          if (q > j) { v = (TC)((double)v * scal); vv = v; }
          else if (q == j) { vv = TC(1); v = (TC)beta; }
          else vv = TC(0);
          x[i][cc] = v;
          vb[q] = vv;
        }
      }
      if (l == 0) { taus[j] = (TC)tau; Tl[j * LDT + j] = (TC)tau; }
    }
    __syncthreads();
    if (kTinLoop && w == 0 && j >= 1) t_column(j - 1);
    const TC tau = taus[j];
    // v is kept in registers when the chunk leaves room for it, else re-read from LDS
    constexpr bool kCacheV = RPT * ((int)sizeof(TC) / 4) * (CPT + 1) <= 96;
    TC vr[kCacheV ? RPT : 1];
    if constexpr (kCacheV) {
#pragma unroll
      for (int i = 0; i < RPT; ++i) vr[i] = vb[i * 64 + l];
    }
    auto vget = [&](int i) -> TC {
      if constexpr (kCacheV) return vr[i];
      else return vb[i * 64 + l];
    };
#pragma unroll
    for (int cc = 0; cc < CPT; ++cc) {
      const int gc = w * CPT + cc;
      if (gc == j || gc >= bw) continue;
      // four independent partial sums shorten the dependent FMA chain
      TC dp[4] = {TC(0), TC(0), TC(0), TC(0)};
#pragma unroll
      for (int i = 0; i < RPT; ++i) dp[i & 3] += vget(i) * x[i][cc];
      TC d = wave_sum((dp[0] + dp[1]) + (dp[2] + dp[3]));
      if (gc > j) {
        const TC td = tau * d;
#pragma unroll
        for (int i = 0; i < RPT; ++i) x[i][cc] -= td * vget(i);
      } else if (l == 0) {
        Tl[gc * LDT + j] = d;  // Y[gc][j] = v_gc^T v_j
      }
    }
  }
  __syncthreads();

  PANEL_MARK(slot, 2);
  if constexpr (kTinLoop) {
    // last column of T, then the rows of T into Tl for the output stage
    if (w == 0 && kr >= 1) {
      t_column(kr - 1);
      if (l < TILE) {
#pragma unroll
        for (int k = 0; k < TILE; ++k)
          if (k >= l) Tl[l * LDT + k] = trow[k];
      }
    }
    __syncthreads();
  }
  // ---- (wider tiles) T = inverse of (diag(1/tau) + strict upper of V^T V), by doubling ----
  for (int bs = 1; !kTinLoop && bs < kr; bs *= 2) {
    const int npair = (kr + 2 * bs - 1) / (2 * bs);
    // M = Y_AB * T_BB
    for (int t = threadIdx.x; t < npair * bs * bs; t += blockDim.x) {
      const int p = t / (bs * bs), r = (t / bs) % bs, cidx = t % bs;
      const int i0 = p * 2 * bs, ia = i0 + r, ib = i0 + bs + cidx;
      TC s = TC(0);
      if (ib < kr) {
        for (int lq = i0 + bs; lq <= ib; ++lq) s += Tl[ia * LDT + lq] * Tl[lq * LDT + ib];
      }
      Mtmp[t] = s;
    }
    __syncthreads();
    // T_AB = -T_AA * M
    for (int t = threadIdx.x; t < npair * bs * bs; t += blockDim.x) {
      const int p = t / (bs * bs), r = (t / bs) % bs, cidx = t % bs;
      const int i0 = p * 2 * bs, ia = i0 + r, ib = i0 + bs + cidx;
      if (ib < kr) {
        TC s = TC(0);
        for (int lq = ia; lq < i0 + bs; ++lq) s += Tl[ia * LDT + lq] * Mtmp[p * bs * bs + (lq - i0) * bs + cidx];
        Tl[ia * LDT + ib] = -s;
      }
    }
    __syncthreads();
  }

  PANEL_MARK(slot, 3);
  // ---- outputs: T (TILE x TILE, column-major, zero outside kr), V, R ----
  T* Tout = a.Tm + (int64_t)c * TILE * TILE;
  for (int t = threadIdx.x; t < TILE * TILE; t += blockDim.x) {
    const int r = t % TILE, col = t / TILE;
    Tout[t] = (r < kr && col < kr && r <= col) ? (T)Tl[r * LDT + col] : T(0);
  }
#pragma unroll
  for (int cc = 0; cc < CPT; ++cc) {
    const int gc = w * CPT + cc;
    if (gc >= kr) continue;
#pragma unroll
    for (int i = 0; i < RPT; ++i) {
      const int q = i * 64 + l;
      if (q >= Hc) continue;
      const T v = q > gc ? (T)x[i][cc] : (q == gc ? T(1) : T(0));
      a.V[(row0 + q) + (int64_t)gc * a.ldv] = v;
    }
  }
  // R: upper triangle of the top kr rows (q <= gc, q < kr), all bw columns.
#pragma unroll
  for (int cc = 0; cc < CPT; ++cc) {
    const int gc = w * CPT + cc;
    if (gc >= bw) continue;
#pragma unroll
    for (int i = 0; i < RPT; ++i) {
      const int q = i * 64 + l;
      if (q < kr && q <= gc) a.M.at(a.rm.row(c, q), a.pc + gc) = (T)x[i][cc];
    }
  }
  PANEL_MARK(slot, 4);
}

template <typename T, int TILE, int RPT, typename TC>
__global__ __launch_bounds__(1024) void k_chunk_qr(ChunkQRArgs<T> a) {
  chunk_qr_body<T, TILE, RPT, TC>(a, blockIdx.x);
}

// Batched form: one single-chunk panel per matrix, matrix blockIdx.x of the table.
// A single chunk shorter than the capacity (the upper levels of a TSQR tree, the
// panels of small or nearly finished matrices) runs the same body with fewer rows
// per lane -- 2, 8 or 16, the fewest that hold it -- so that the per-column work
// scales with the rows present, not with the capacity.  Returns the rows per lane
// to use (RPT itself when no smaller tier applies).
template <int RPT>
__host__ __device__ inline int chunk_tier(int P, int64_t h) {
  if (P != 1) return RPT;
  if (RPT > 2 && h <= 64 * 2) return 2;
  if (RPT > 8 && h <= 64 * 8) return 8;
  if (RPT > 16 && h <= 64 * 16) return 16;
  return RPT;
}

template <typename T, int TILE, int RPT, typename TC>
__global__ __launch_bounds__(1024) void k_chunk_qr_b(const ChunkQRArgs<T>* __restrict__ tab) {
  const ChunkQRArgs<T>& a = tab[blockIdx.x];
  switch (chunk_tier<RPT>(a.P, a.h)) {  // the same choice as a single call
    case 2:
      if constexpr (RPT > 2) { chunk_qr_body<T, TILE, 2, TC>(a, 0); return; }
      break;
    case 8:
      if constexpr (RPT > 8) { chunk_qr_body<T, TILE, 8, TC>(a, 0); return; }
      break;
    case 16:
      if constexpr (RPT > 16) { chunk_qr_body<T, TILE, 16, TC>(a, 0); return; }
      break;
  }
  chunk_qr_body<T, TILE, RPT, TC>(a, 0);
}

// ---------------------------------------------------------------------------
// a3/a5: trailing update  C <- (I - V T V^T)^T C  on MFMA
// ---------------------------------------------------------------------------

// ---------------------------------------------------------------------------
// a6: band pack -- W (dtype T, column-major) -> chase storage (float64, row-major,
// row i holds columns i-(b-1) .. i+2b-1 at offsets 0 .. 3b-2; width ldb)
// ---------------------------------------------------------------------------

template <typename T>
__device__ __forceinline__ void band_pack_body(const T* __restrict__ W, int64_t ldw, int64_t n, int b,
                                               double* __restrict__ Bs, int64_t ldb, const int* exp_in, int unscale) {
  const int64_t total = n * ldb;
  const int e = unscale ? *exp_in : 0;
  for (int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; idx < total; idx += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = idx / ldb;
    const int d = (int)(idx - i * ldb);
    const int64_t j = i + d - (b - 1);
    double v = 0.0;
    if (j >= i && j <= i + b && j < n) v = ldexp((double)W[i + j * ldw], e);
    Bs[idx] = v;
  }
}
template <typename T>
__global__ void k_band_pack(const T* __restrict__ W, int64_t ldw, int64_t n, int b, double* __restrict__ Bs, int64_t ldb,
                            const int* exp_in, int unscale) {
  band_pack_body(W, ldw, n, b, Bs, ldb, exp_in, unscale);
}

// ---------------------------------------------------------------------------
// batched forms of staging and band packing: matrix blockIdx.y of the table
// ---------------------------------------------------------------------------
template <typename T>
__global__ void k_absmax_b(const BatchMat<T>* __restrict__ tab) {
  const BatchMat<T>& t = tab[blockIdx.y];
  absmax_body(t.A, t.m, t.n, t.lda, t.amax);
}
template <typename T>
__global__ void k_copy_scale_b(const BatchMat<T>* __restrict__ tab) {
  const BatchMat<T>& t = tab[blockIdx.y];
  copy_scale_body(t.A, t.m, t.n, t.lda, t.transpose, t.W, t.ldw, t.amax, t.exp);
}
template <typename T>
__global__ void k_band_pack_b(const BatchMat<T>* __restrict__ tab, int b) {
  const BatchMat<T>& t = tab[blockIdx.y];
  band_pack_body(t.W, t.ldw, t.N, b, t.Bs, 3 * b, t.exp, 0);
}

// External band layout (band[i*ldband + d] = B(i, i+d), d = 0..b) <-> chase storage.
template <typename T>
__global__ void k_band_extract(const T* __restrict__ W, int64_t ldw, int64_t n, int b, double* __restrict__ out,
                               int64_t ldo, const int* exp_in) {
  const int64_t total = n * (b + 1);
  const int e = *exp_in;
  const bool nonfinite = e == kExpNonFinite;
  for (int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; idx < total; idx += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = idx / (b + 1);
    const int d = (int)(idx - i * (b + 1));
    const int64_t j = i + d;
    out[i * ldo + d] = nonfinite ? __builtin_nan("") : (j < n ? ldexp((double)W[i + j * ldw], e) : 0.0);
  }
}

// A NaN or an infinity among the band's entries sets *nonfinite (the chase then
// gives up at once and its d and e are written as NaN).
__global__ void k_band_import(const double* __restrict__ in, int64_t ldi, int64_t n, int b, double* __restrict__ Bs,
                              int64_t ldb, int* nonfinite) {
  const int64_t total = n * ldb;
  bool bad = false;
  for (int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; idx < total; idx += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = idx / ldb;
    const int d = (int)(idx - i * ldb);
    const int64_t off = d - (b - 1);
    const double v = (off >= 0 && off <= b && i + off < n) ? in[i * ldi + off] : 0.0;
    bad = bad || !isfinite(v);
    Bs[idx] = v;
  }
  if (bad) __hip_atomic_store(nonfinite, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// ---------------------------------------------------------------------------
// host-side launchers
// ---------------------------------------------------------------------------

static inline int grid_for(int64_t total, int block) {
  int64_t g = (total + block - 1) / block;
  if (g > 8192) g = 8192;
  if (g < 1) g = 1;
  return (int)g;
}

template <typename T>
hipError_t launch_stage_in(const T* A, int64_t m, int64_t n, int64_t lda, int transpose, T* W, int64_t ldw,
                           unsigned long long* amax, int* exp_out, hipStream_t st) {
  hipLaunchKernelGGL(k_fill_u64, dim3(1), dim3(64), 0, st, amax, 1ull * 0, (int64_t)1);
  hipLaunchKernelGGL(k_absmax<T>, dim3(std::min(grid_for(m * n, 256), 1024)), dim3(256), 0, st, A, m, n, lda, amax);
  hipLaunchKernelGGL(k_copy_scale<T>, dim3(grid_for(m * n, 256)), dim3(256), 0, st, A, m, n, lda, transpose, W, ldw,
                     amax, exp_out);
  return hipGetLastError();
}

template <typename TC, int TILE, int RPT>
static size_t chunk_qr_lds() {
  return sizeof(TC) * (ChunkQRCfg<TC, TILE, RPT>::CQB * 64 * (TILE + 1) + 2 * 64 * RPT + TILE + TILE * (TILE + 1));
}

template <typename T, int TILE, int RPT, typename TC = T>
static hipError_t launch_cqr(const ChunkQRArgs<T>& a, hipStream_t st) {
  if constexpr (sizeof(TC) == 8 && TILE > 64) {
    return hipErrorInvalidConfiguration;
  } else {
    if constexpr (std::is_same<T, float>::value && std::is_same<TC, float>::value) {
      if (a.hp) return launch_cqr<T, TILE, RPT, double>(a, st);
    }
    const size_t lds = chunk_qr_lds<TC, TILE, RPT>();
    static bool configured = false;
    if (!configured) {
      hipError_t e = hipFuncSetAttribute((const void*)k_chunk_qr<T, TILE, RPT, TC>,
                                         hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
      if (e != hipSuccess) return e;
      configured = true;
    }
    const int tier = chunk_tier<RPT>(a.P, a.h);
    if constexpr (RPT > 2) {
      if (tier == 2) return launch_cqr<T, TILE, 2, TC>(a, st);
    }
    if constexpr (RPT > 8) {
      if (tier == 8) return launch_cqr<T, TILE, 8, TC>(a, st);
    }
    if constexpr (RPT > 16) {
      if (tier == 16) return launch_cqr<T, TILE, 16, TC>(a, st);
    }
    hipLaunchKernelGGL((k_chunk_qr<T, TILE, RPT, TC>), dim3(a.P), dim3(1024), lds, st, a);
    return hipGetLastError();
  }
}

template <typename T>
int chunk_qr_hmax(int tile) {
  switch (tile) {
    case 16: return 64 * ChunkRPT<T, 16>::value;
    case 32: return 64 * ChunkRPT<T, 32>::value;
    case 64: return 64 * ChunkRPT<T, 64>::value;
    case 128: return 64 * ChunkRPT<T, 128>::value;
  }
  return 0;
}
template int chunk_qr_hmax<float>(int);
template int chunk_qr_hmax<double>(int);

template <typename T, int TILE, int RPT, typename TC = T>
static hipError_t launch_cqr_b(const ChunkQRArgs<T>* tab, int count, int hp, hipStream_t st) {
  if constexpr (sizeof(TC) == 8 && TILE > 64) {
    return hipErrorInvalidConfiguration;
  } else {
    if constexpr (std::is_same<T, float>::value && std::is_same<TC, float>::value) {
      if (hp) return launch_cqr_b<T, TILE, RPT, double>(tab, count, hp, st);
    }
    const size_t lds = chunk_qr_lds<TC, TILE, RPT>();
    static bool configured = false;
    if (!configured) {
      hipError_t e = hipFuncSetAttribute((const void*)k_chunk_qr_b<T, TILE, RPT, TC>,
                                         hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
      if (e != hipSuccess) return e;
      configured = true;
    }
    hipLaunchKernelGGL((k_chunk_qr_b<T, TILE, RPT, TC>), dim3(count), dim3(1024), lds, st, tab);
    return hipGetLastError();
  }
}

template <typename T>
hipError_t launch_chunk_qr_batched(int tile, const ChunkQRArgs<T>* tab, int count, int hp, hipStream_t st) {
  if (count <= 0) return hipSuccess;
  switch (tile) {
    case 16: return launch_cqr_b<T, 16, ChunkRPT<T, 16>::value>(tab, count, hp, st);
    case 32: return launch_cqr_b<T, 32, ChunkRPT<T, 32>::value>(tab, count, hp, st);
    case 64: return launch_cqr_b<T, 64, ChunkRPT<T, 64>::value>(tab, count, hp, st);
    case 128: return launch_cqr_b<T, 128, ChunkRPT<T, 128>::value>(tab, count, hp, st);
  }
  return hipErrorInvalidValue;
}

template <typename T>
hipError_t launch_stage_in_batched(const BatchMat<T>* tab, int count, unsigned long long* amax_all, int64_t max_elems,
                                   hipStream_t st) {
  if (count <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill_u64, dim3(std::max(1, std::min(64, (count + 255) / 256))), dim3(256), 0, st, amax_all,
                     0ull, (int64_t)count);
  const int gx = std::max(1, std::min(grid_for(max_elems, 256), 64));
  hipLaunchKernelGGL(k_absmax_b<T>, dim3(gx, count), dim3(256), 0, st, tab);
  hipLaunchKernelGGL(k_copy_scale_b<T>, dim3(gx, count), dim3(256), 0, st, tab);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_band_pack_batched(const BatchMat<T>* tab, int count, int b, int64_t max_n, hipStream_t st) {
  if (count <= 0) return hipSuccess;
  const int gx = std::max(1, std::min(grid_for(max_n * 3 * b, 256), 64));
  hipLaunchKernelGGL(k_band_pack_b<T>, dim3(gx, count), dim3(256), 0, st, tab, b);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_chunk_qr(int tile, const ChunkQRArgs<T>& a, hipStream_t st) {
  switch (tile) {
    case 16: return launch_cqr<T, 16, ChunkRPT<T, 16>::value>(a, st);
    case 32: return launch_cqr<T, 32, ChunkRPT<T, 32>::value>(a, st);
    case 64: return launch_cqr<T, 64, ChunkRPT<T, 64>::value>(a, st);
    case 128: return launch_cqr<T, 128, ChunkRPT<T, 128>::value>(a, st);
  }
  return hipErrorInvalidValue;
}

template <typename T>
hipError_t launch_band_pack(const T* W, int64_t ldw, int64_t n, int b, double* Bs, int64_t ldb, const int* exp_in,
                            int unscale, hipStream_t st) {
  hipLaunchKernelGGL(k_band_pack<T>, dim3(grid_for(n * ldb, 256)), dim3(256), 0, st, W, ldw, n, b, Bs, ldb, exp_in,
                     unscale);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_band_extract(const T* W, int64_t ldw, int64_t n, int b, double* out, int64_t ldo, const int* exp_in,
                               hipStream_t st) {
  hipLaunchKernelGGL(k_band_extract<T>, dim3(grid_for(n * (b + 1), 256)), dim3(256), 0, st, W, ldw, n, b, out, ldo,
                     exp_in);
  return hipGetLastError();
}

// In-place exact scaling of the chase storage by 2^-e, e = scale_exponent(*amax), so
// that the chase's norms neither overflow nor underflow for any finite band; *exp_out
// receives e (the marker of a non-finite input leaves the data as it is).
__global__ void k_scale_inplace(double* p, int64_t count, const unsigned long long* amax, int* exp_out) {
  const int e = scale_exponent(*amax);
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    const double mx = __longlong_as_double((long long)*amax);
    *exp_out = isfinite(mx) ? e : kExpNonFinite;
  }
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < count; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = ldexp(p[i], -e);
}

hipError_t launch_band_scale(double* Bs, int64_t ldb, int64_t n, unsigned long long* amax, int* exp_out,
                             hipStream_t st) {
  hipLaunchKernelGGL(k_fill_u64, dim3(1), dim3(64), 0, st, amax, 0ull, (int64_t)1);
  hipLaunchKernelGGL(k_absmax<double>, dim3(std::min(grid_for(n * ldb, 256), 1024)), dim3(256), 0, st, Bs, ldb, n,
                     ldb, amax);
  hipLaunchKernelGGL(k_scale_inplace, dim3(grid_for(n * ldb, 256)), dim3(256), 0, st, Bs, n * ldb, amax, exp_out);
  return hipGetLastError();
}

hipError_t launch_band_import(const double* in, int64_t ldi, int64_t n, int b, double* Bs, int64_t ldb, int* nonfinite,
                              hipStream_t st) {
  hipLaunchKernelGGL(k_band_import, dim3(grid_for(n * ldb, 256)), dim3(256), 0, st, in, ldi, n, b, Bs, ldb, nonfinite);
  return hipGetLastError();
}

#define SVDV_INST(T)                                                                                             \
  template hipError_t launch_stage_in<T>(const T*, int64_t, int64_t, int64_t, int, T*, int64_t, unsigned long long*, \
                                         int*, hipStream_t);                                                      \
  template hipError_t launch_chunk_qr<T>(int, const ChunkQRArgs<T>&, hipStream_t);                               \
  template hipError_t launch_chunk_qr_batched<T>(int, const ChunkQRArgs<T>*, int, int, hipStream_t);             \
  template hipError_t launch_stage_in_batched<T>(const BatchMat<T>*, int, unsigned long long*, int64_t, hipStream_t); \
  template hipError_t launch_band_pack_batched<T>(const BatchMat<T>*, int, int, int64_t, hipStream_t);          \
  template hipError_t launch_band_pack<T>(const T*, int64_t, int64_t, int, double*, int64_t, const int*, int,     \
                                          hipStream_t);                                                           \
  template hipError_t launch_band_extract<T>(const T*, int64_t, int64_t, int, double*, int64_t, const int*,       \
                                             hipStream_t);
SVDV_INST(float)
SVDV_INST(double)

}  // namespace svdv

#ifdef SVDV_PANEL_TRACE
extern "C" int svdv_panel_trace(uint64_t* out, int count) {
  return (int)hipMemcpyFromSymbol(out, HIP_SYMBOL(svdv::g_panel_trace), (size_t)count * 8);
}
#endif
