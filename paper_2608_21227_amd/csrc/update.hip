// Stage-1 trailing update, the operation the paper's Algorithm 2 performs and
// auto-tunes: apply the orthogonal factor of a panel to the trailing matrix.
// Here it is done in compact-WY form, C <- (I - V T V^T)^T C = C - V (T^T (V^T C)),
// one TSQR chunk (rows of V) and one 16*IB-column strip of C per workgroup.
//
// The strip stays in registers between the two products, so C crosses HBM
// once each way:
//
//   load    the NW waves take the chunk's 16-row slabs round-robin (SPW slabs
//           each) and issue every load of their slabs at once; with rows
//           contiguous in memory (QR sweep) each lane loads 4 consecutive rows
//           of one column as one 16-byte access;
//   pass 1  Z = V^T C on the MFMA units, a partial Z per wave;
//   reduce  Z = sum of the NW partials in LDS (fixed order: deterministic);
//   small   Z' = T^T Z (vector FMAs, from LDS);
//   pass 2  C -= V Z' on the MFMA units, accumulating into the C registers,
//           which are then stored.
//
// The paper's tunables map onto this kernel as: threads = NW * 64 (waves that
// share a column strip and split its rows, like the split-K "K" of Algorithm 2),
// inner_block = IB (16-column MFMA tiles per workgroup, like "CPB").
#include <algorithm>
#include <type_traits>
#include "common.hpp"
#include "kernels.hpp"

namespace svdv {

// MFMA operand layout used throughout (16x16x4): lane (g, nl) = (lane / 16, lane % 16).
// The C registers of a slab hold rows acc_row<T>(g, i), i = 0..3, of column nl: the
// K index of pass 1 and the output rows of pass 2 use the same assignment, so the
// pass-2 accumulator starts from, and ends in, the registers that were loaded.

// Loads rows q0 + acc_row(g, i) (i = 0..3) of view column `col` (zero outside the
// chunk or the strip).
template <typename T, bool VEC>
__device__ __forceinline__ void load_c(const LarfbArgs<T>& a, int c, int Hc, int q0, int g, int64_t col, T (&x)[4]) {
  const bool cok = col < a.col1;
  if constexpr (VEC) {
    // float, rows contiguous: rows q0+4g .. q0+4g+3 are consecutive in memory
    const int qa = q0 + 4 * g;
    if (cok && qa + 3 < Hc) {
      const float4 v = *reinterpret_cast<const float4*>(&a.M.at(a.rm.row(c, qa), col));
      x[0] = v.x;
      x[1] = v.y;
      x[2] = v.z;
      x[3] = v.w;
      return;
    }
  }
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int q = q0 + acc_row<T>(g, i);
    x[i] = (cok && q < Hc) ? a.M.at(a.rm.row(c, q), col) : T(0);
  }
}

template <typename T, bool VEC>
__device__ __forceinline__ void store_c(const LarfbArgs<T>& a, int c, int Hc, int q0, int g, int64_t col,
                                        const typename Acc<T>::type& x) {
  if (col >= a.col1) return;
  if constexpr (VEC) {
    const int qa = q0 + 4 * g;
    if (qa + 3 < Hc) {
      *reinterpret_cast<float4*>(&a.M.at(a.rm.row(c, qa), col)) = float4{x[0], x[1], x[2], x[3]};
      return;
    }
  }
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int q = q0 + acc_row<T>(g, i);
    if (q < Hc) a.M.at(a.rm.row(c, q), col) = x[i];
  }
}

// Pass-1 operand: V^T rows (reflector r = 16 mt + nl), K = rows q0 + acc_row(g, i).
template <typename T, bool VEC>
__device__ __forceinline__ void load_v1(const LarfbArgs<T>& a, const T* V, int Hc, int q0, int g, int r, T (&x)[4]) {
  const bool rok = r < a.k;
  if constexpr (sizeof(T) == 4) {
    const int qa = q0 + 4 * g;
    if ((VEC || a.vecv) && rok && qa + 3 < Hc) {
      const float4 v = *reinterpret_cast<const float4*>(V + qa + (int64_t)r * a.ldv);
      x[0] = v.x;
      x[1] = v.y;
      x[2] = v.z;
      x[3] = v.w;
      return;
    }
  }
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int q = q0 + acc_row<T>(g, i);
    x[i] = (rok && q < Hc) ? V[q + (int64_t)r * a.ldv] : T(0);
  }
}

// PREC 0: MFMA in T; PREC 2 / 3 (T = float): BF16 / FP16 operands, float32 accumulation.
// MODE 0: the whole update of the strip.  MODE 2 (the split form of a single panel
// taller than the registers hold): the strip's Z' = T^T V^T C comes from zw[strip],
// written by the split form's first pass and reduction, and only pass 2 runs.
template <typename T, int KT, int IB, int NW, int SPW, bool VEC, int PREC, int MODE = 0>
__device__ __forceinline__ void larfb_reg_body(const LarfbArgs<T>& a, const int strip, const int c, T* zw = nullptr) {
  typedef typename Acc<T>::type AccT;
  constexpr int KR = KT * 16, CB = IB * 16;
  // MODE 2 with strips of 32 or more columns loads each slab's V just before its
  // transpose rather than with the strip: fewer registers live, more workgroups per
  // CU (with 16-column strips the early loads measured faster)
  constexpr bool kLateV = MODE == 2 && IB >= 2;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  // [NW][KR][CB] partial sums (slot 0 then holds Z); in pass 2 the same space holds
  // each wave's [16][KR + 4] V slab being transposed
  T* Zs = reinterpret_cast<T*>(smem_raw);
  T* Zp = Zs + (larfb_reg_lds_elems(KT, IB, NW) - KR * CB);  // [KR][CB] Z' = T^T Z
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int g = lane >> 4, nl = lane & 15;
  const int64_t row0 = (int64_t)c * a.chunk_rows;
  const int Hc = (int)(c == a.P - 1 ? a.h - row0 : a.chunk_rows);
  const int k = a.k;
  const int64_t colbase = a.col0 + (int64_t)strip * CB;
  const T* V = a.V + row0;
  const T* Tm = a.Tm + (int64_t)c * a.ldt * a.ldt;
  const int nslab = (Hc + 15) >> 4;

  // ---------------- load the strip and the pass-1 operands ----------------
  T cr[SPW][IB][4];
  T vr[SPW][KT][4];
#pragma unroll
  for (int j = 0; j < SPW; ++j) {
    const int s = wv + j * NW;
    const int q0 = s * 16;
    if (s < nslab) {
#pragma unroll
      for (int nt = 0; nt < IB; ++nt) load_c<T, VEC>(a, c, Hc, q0, g, colbase + nt * 16 + nl, cr[j][nt]);
      if constexpr (!kLateV) {
#pragma unroll
        for (int mt = 0; mt < KT; ++mt) load_v1<T, VEC>(a, V, Hc, q0, g, mt * 16 + nl, vr[j][mt]);
      }
    } else {
#pragma unroll
      for (int nt = 0; nt < IB; ++nt)
#pragma unroll
        for (int i = 0; i < 4; ++i) cr[j][nt][i] = T(0);
#pragma unroll
      for (int mt = 0; mt < KT; ++mt)
#pragma unroll
        for (int i = 0; i < 4; ++i) vr[j][mt][i] = T(0);
    }
  }

  // ---------------- pass 1: partial Z = V^T C ----------------
  AccT Z[KT][IB];
#pragma unroll
  for (int mt = 0; mt < KT; ++mt)
#pragma unroll
    for (int nt = 0; nt < IB; ++nt) Z[mt][nt] = AccT{0, 0, 0, 0};
  if constexpr (MODE == 2) {
    // Z' comes from the split form's reduction
  } else if constexpr (PREC == 0) {
#pragma unroll
    for (int j = 0; j < SPW; ++j)
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int mt = 0; mt < KT; ++mt)
#pragma unroll
          for (int nt = 0; nt < IB; ++nt) Z[mt][nt] = mfma16(vr[j][mt][i], cr[j][nt][i], Z[mt][nt]);
  } else {
    // one 16x16x16 instruction per slab: K = the 16 rows, lane (g, nl) holding rows 4g..4g+3
#pragma unroll
    for (int j = 0; j < SPW; ++j)
#pragma unroll
      for (int mt = 0; mt < KT; ++mt)
#pragma unroll
        for (int nt = 0; nt < IB; ++nt) Z[mt][nt] = mfma16x16<PREC>(vr[j][mt], cr[j][nt], Z[mt][nt]);
  }

  // pass-2 operand (reflectors along K, rows along lanes), formed per slab in pass 2
  // A[m = row][k = reflector]: lane (g, nl) holds -V[q0 + nl][r], r = 4 kk + g (K = 4 per
  // instruction) or, for the 16x16x16 forms, r = 16 (kk / 4) + 4 g + kk % 4
  T va[SPW][KR / 4];

  // ---------------- reduce the NW partials (fixed order) ----------------
  if constexpr (MODE != 2) {
    T* mine = Zs + (size_t)wv * KR * CB;
#pragma unroll
    for (int mt = 0; mt < KT; ++mt)
#pragma unroll
      for (int nt = 0; nt < IB; ++nt)
#pragma unroll
        for (int r = 0; r < 4; ++r) mine[(mt * 16 + acc_row<T>(g, r)) * CB + nt * 16 + nl] = Z[mt][nt][r];
  }
  if constexpr (MODE != 2) {
    __syncthreads();
    for (int e = threadIdx.x; e < KR * CB; e += NW * 64) {
      T acc = Zs[e];
      for (int w = 1; w < NW; ++w) acc += Zs[(size_t)w * KR * CB + e];
      Zs[e] = acc;
    }
    __syncthreads();
  }
  if constexpr (MODE == 0) {
    // ---------------- Z' = T^T Z (T upper triangular, k x k) ----------------
    for (int e = threadIdx.x; e < KR * CB; e += NW * 64) {
      const int i = e / CB, col = e - i * CB;
      T acc = T(0);
      if (i < k) {
        // all T loads of the sum issued together (one cache round trip, not KR in a row)
        T tv[KR];
#pragma unroll
        for (int l = 0; l < KR; ++l) tv[l] = l <= i ? Tm[l + (int64_t)i * a.ldt] : T(0);
#pragma unroll
        for (int l = 0; l < KR; ++l)
          if (l <= i) acc += tv[l] * Zs[l * CB + col];
      }
      Zp[e] = acc;
    }
    __syncthreads();
  }

  // ---------------- pass 2: C -= V Z', accumulated into the strip registers ----------------
  // B[k = reflector][n = column]: lane (g, nl) holds Z'[4 kk + g][16 nt + nl]
  const T* zsrc = MODE == 2 ? zw + (int64_t)strip * (KR * CB) : Zp;
  T zb[KR / 4][IB];
#pragma unroll
  for (int kk = 0; kk < KR / 4; ++kk) {
    const int r = PREC == 0 ? 4 * kk + g : 16 * (kk / 4) + 4 * g + kk % 4;
#pragma unroll
    for (int nt = 0; nt < IB; ++nt) zb[kk][nt] = zsrc[r * CB + nt * 16 + nl];
  }
#pragma unroll
  for (int j = 0; j < SPW; ++j) {
    const int s = wv + j * NW;
    if (s >= nslab) break;
    AccT acc[IB];
#pragma unroll
    for (int nt = 0; nt < IB; ++nt) acc[nt] = AccT{cr[j][nt][0], cr[j][nt][1], cr[j][nt][2], cr[j][nt][3]};
    {
      // vr[j][mt][i] = V[row acc_row(g, i)][reflector 16 mt + nl] of this slab (zero
      // outside the chunk and past k), transposed through this wave's LDS slab:
      // va[j][kk] needs row nl, reflector r(kk, g).  The Zs space is free here (Z'
      // was formed behind a barrier) and each wave touches only its own slab.
      T* buf = Zs + (size_t)wv * 16 * (KR + 4);
      if constexpr (kLateV) {
#pragma unroll
        for (int mt = 0; mt < KT; ++mt) load_v1<T, VEC>(a, V, Hc, s * 16, g, mt * 16 + nl, vr[j][mt]);
      }
#pragma unroll
      for (int mt = 0; mt < KT; ++mt)
#pragma unroll
        for (int i = 0; i < 4; ++i) buf[acc_row<T>(g, i) * (KR + 4) + mt * 16 + nl] = vr[j][mt][i];
      __builtin_amdgcn_wave_barrier();
#pragma unroll
      for (int kk = 0; kk < KR / 4; ++kk) {
        const int r = PREC == 0 ? 4 * kk + g : 16 * (kk / 4) + 4 * g + kk % 4;
        va[j][kk] = -buf[nl * (KR + 4) + r];
      }
      __builtin_amdgcn_wave_barrier();
    }
    if constexpr (PREC == 0) {
#pragma unroll
      for (int kk = 0; kk < KR / 4; ++kk)
#pragma unroll
        for (int nt = 0; nt < IB; ++nt) acc[nt] = mfma16(va[j][kk], zb[kk][nt], acc[nt]);
    } else {
#pragma unroll
      for (int kt = 0; kt < KT; ++kt)
#pragma unroll
        for (int nt = 0; nt < IB; ++nt) {
          const float av[4] = {va[j][4 * kt], va[j][4 * kt + 1], va[j][4 * kt + 2], va[j][4 * kt + 3]};
          const float bv[4] = {zb[4 * kt][nt], zb[4 * kt + 1][nt], zb[4 * kt + 2][nt], zb[4 * kt + 3][nt]};
          acc[nt] = mfma16x16<PREC>(av, bv, acc[nt]);
        }
    }
#pragma unroll
    for (int nt = 0; nt < IB; ++nt) store_c<T, VEC>(a, c, Hc, s * 16, g, colbase + nt * 16 + nl, acc[nt]);
  }
}

// Workgroups are dispatched to the 8 XCDs round-robin by linear workgroup id, and
// each XCD has its own L2.  Neighbouring strips share 128-byte lines when the
// strip runs along memory rows (LQ sweep: 16 floats = half a line), so the
// linear ids are permuted to put strips 2j and 2j+1 on workgroups id and id + 8
// (same XCD): the second half of each line is then an L2 hit, not a second HBM
// read.  Groups of 16 ids are permuted; a ragged tail keeps its ids.
__device__ __forceinline__ int64_t xcd_pair_id(int64_t id, int64_t count) {
  const int64_t full = count / 16 * 16;
  if (id >= full) return id;
  const int64_t g = id / 16, r = id % 16;
  return g * 16 + (r % 8) * 2 + r / 8;
}

template <typename T, int KT, int IB, int NW, int SPW, bool VEC, int PREC>
__global__ void __launch_bounds__(NW * 64) k_larfb_reg(LarfbArgs<T> a) {
  const int64_t id = xcd_pair_id(blockIdx.x + (int64_t)blockIdx.y * gridDim.x, (int64_t)gridDim.x * gridDim.y);
  larfb_reg_body<T, KT, IB, NW, SPW, VEC, PREC>(a, (int)(id % gridDim.x), (int)(id / gridDim.x));
}

// Split form of one tall panel (reflectors longer than a strip's registers hold).
// First pass, grid (strips, row ranges): Z = V^T C over rows [c R1, (c + 1) R1) of
// the strip, summed register block by register block (SPW x NW slabs of 16 rows)
// in row order, the NW wave partials then added in fixed order; written to
// zw[c * strips + strip].  C is only read.
template <typename T, int KT, int IB, int NW, int SPW, bool VEC>
__global__ void __launch_bounds__(NW * 64) k_larfb_split_p1(LarfbArgs<T> a, T* zw) {
  typedef typename Acc<T>::type AccT;
  constexpr int KR = KT * 16, CB = IB * 16, R0 = SPW * NW * 16;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  T* Zs = reinterpret_cast<T*>(smem_raw);  // [NW][KR][CB] wave partials
  const int64_t id = xcd_pair_id(blockIdx.x + (int64_t)blockIdx.y * gridDim.x, (int64_t)gridDim.x * gridDim.y);
  const int strip = (int)(id % gridDim.x), c = (int)(id / gridDim.x);
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int g = lane >> 4, nl = lane & 15;
  const int64_t row0 = (int64_t)c * a.chunk_rows;
  const int Hc = (int)(c == a.P - 1 ? a.h - row0 : a.chunk_rows);
  const int64_t colbase = a.col0 + (int64_t)strip * CB;
  const T* V = a.V + row0;
  AccT Z[KT][IB];
#pragma unroll
  for (int mt = 0; mt < KT; ++mt)
#pragma unroll
    for (int nt = 0; nt < IB; ++nt) Z[mt][nt] = AccT{0, 0, 0, 0};
  // with strips of 32 or more columns a block's slabs are taken in two halves (the
  // same slab order, so the same sums): half the registers live, more workgroups per CU
  constexpr int SH = (IB >= 2 && SPW % 2 == 0) ? SPW / 2 : SPW;
  for (int base = 0; base < Hc; base += R0) {
#pragma unroll
    for (int j0 = 0; j0 < SPW; j0 += SH) {
      T cr[SH][IB][4], vr[SH][KT][4];
#pragma unroll
      for (int jj = 0; jj < SH; ++jj) {
        const int q0 = base + (wv + (j0 + jj) * NW) * 16;
#pragma unroll
        for (int nt = 0; nt < IB; ++nt) load_c<T, VEC>(a, c, Hc, q0, g, colbase + nt * 16 + nl, cr[jj][nt]);
#pragma unroll
        for (int mt = 0; mt < KT; ++mt) load_v1<T, VEC>(a, V, Hc, q0, g, mt * 16 + nl, vr[jj][mt]);
      }
#pragma unroll
      for (int jj = 0; jj < SH; ++jj)
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
          for (int mt = 0; mt < KT; ++mt)
#pragma unroll
            for (int nt = 0; nt < IB; ++nt) Z[mt][nt] = mfma16(vr[jj][mt][i], cr[jj][nt][i], Z[mt][nt]);
    }
  }
  T* mine = Zs + (size_t)wv * KR * CB;
#pragma unroll
  for (int mt = 0; mt < KT; ++mt)
#pragma unroll
    for (int nt = 0; nt < IB; ++nt)
#pragma unroll
      for (int r = 0; r < 4; ++r) mine[(mt * 16 + acc_row<T>(g, r)) * CB + nt * 16 + nl] = Z[mt][nt][r];
  __syncthreads();
  T* out = zw + ((int64_t)c * gridDim.x + strip) * (KR * CB);
  for (int e = threadIdx.x; e < KR * CB; e += NW * 64) {
    T acc = Zs[e];
    for (int w = 1; w < NW; ++w) acc += Zs[(size_t)w * KR * CB + e];
    out[e] = acc;
  }
}

// Split form, second pass, grid (strips, register blocks of R0 rows): C -= V Z'
// with the strip's Z' from zw[strip]; LDS holds one 16-row V slab per wave.
template <typename T, int KT, int IB, int NW, int SPW, bool VEC>
__global__ void __launch_bounds__(NW * 64) k_larfb_split_p2(LarfbArgs<T> a, T* zw) {
  const int64_t id = xcd_pair_id(blockIdx.x + (int64_t)blockIdx.y * gridDim.x, (int64_t)gridDim.x * gridDim.y);
  larfb_reg_body<T, KT, IB, NW, SPW, VEC, 0, 2>(a, (int)(id % gridDim.x), (int)(id / gridDim.x), zw);
}

// Z = sum of the P blocks' partial Z in block order, then Z' = T^T Z (T the panel's
// k x k upper triangular factor); one workgroup per strip.
template <typename T, int KT, int IB>
__global__ void __launch_bounds__(256) k_larfb_split_z(const T* __restrict__ zpart, T* __restrict__ zprime, int P,
                                                       const T* __restrict__ Tm, int64_t ldt, int k) {
  constexpr int KR = KT * 16, CB = IB * 16;
  __shared__ T Zs[KR * CB];
  const int strip = blockIdx.x, nstrips = gridDim.x;
  for (int e = threadIdx.x; e < KR * CB; e += blockDim.x) {
    T acc = T(0);
    for (int c = 0; c < P; ++c) acc += zpart[((int64_t)c * nstrips + strip) * (KR * CB) + e];
    Zs[e] = acc;
  }
  __syncthreads();
  for (int e = threadIdx.x; e < KR * CB; e += blockDim.x) {
    const int i = e / CB, col = e - i * CB;
    T acc = T(0);
    if (i < k)
      for (int l = 0; l <= i; ++l) acc += Tm[l + (int64_t)i * ldt] * Zs[l * CB + col];
    zprime[(int64_t)strip * (KR * CB) + e] = acc;
  }
}

// Batched form: matrix blockIdx.z of the table (single-chunk panels); strips past
// that matrix's columns return at once (before any barrier).
template <typename T, int KT, int IB, int NW, int SPW, bool VEC, int PREC>
__global__ void __launch_bounds__(NW * 64) k_larfb_reg_b(const LarfbArgs<T>* __restrict__ tab, int64_t h_lo,
                                                         int64_t h_hi) {
  const int64_t id = xcd_pair_id(blockIdx.x + (int64_t)blockIdx.z * gridDim.x, (int64_t)gridDim.x * gridDim.z);
  const int strip = (int)(id % gridDim.x);
  const LarfbArgs<T>& a = tab[id / gridDim.x];
  // matrices of height in (h_lo, h_hi] only (the others are another launch's)
  if (a.col0 + (int64_t)strip * IB * 16 >= a.col1 || a.k <= 0 || a.h <= h_lo || a.h > h_hi) return;
  larfb_reg_body<T, KT, IB, NW, SPW, VEC, PREC>(a, strip, 0);
}

// Streaming variant, for strips that do not fit in registers: C is read in
// pass 1, read again and written in pass 2, with the next 16-row slab of each
// wave prefetched while the current one is multiplied.
template <typename T, int KT, int IB>
__device__ __forceinline__ void load_slab1(const LarfbArgs<T>& a, const T* V, int c, int Hc, int64_t colbase, int s,
                                           int g, int nl, T (&cb)[IB][4], T (&av)[KT][4]) {
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int q = s * 16 + acc_row<T>(g, i);
    const bool rok = q < Hc;
    const int64_t gr = rok ? a.rm.row(c, q) : 0;
#pragma unroll
    for (int nt = 0; nt < IB; ++nt) {
      const int64_t col = colbase + nt * 16 + nl;
      cb[nt][i] = (rok && col < a.col1) ? a.M.at(gr, col) : T(0);
    }
#pragma unroll
    for (int mt = 0; mt < KT; ++mt) {
      const int r = mt * 16 + nl;
      av[mt][i] = (rok && r < a.k) ? V[q + (int64_t)r * a.ldv] : T(0);
    }
  }
}

template <typename T, int KT, int IB>
__device__ __forceinline__ void load_slab2(const LarfbArgs<T>& a, const T* V, int c, int Hc, int64_t colbase, int s,
                                           int g, int nl, T (&cd)[IB][4], T (&va)[KT][4], int64_t (&grow)[4]) {
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int q = s * 16 + acc_row<T>(g, i);
    const bool rok = q < Hc;
    grow[i] = rok ? a.rm.row(c, q) : -1;
#pragma unroll
    for (int nt = 0; nt < IB; ++nt) {
      const int64_t col = colbase + nt * 16 + nl;
      cd[nt][i] = (rok && col < a.col1) ? a.M.at(grow[i], col) : T(0);
    }
  }
  const int qa = s * 16 + nl;
  const bool aok = qa < Hc;
#pragma unroll
  for (int ot = 0; ot < KT; ++ot)
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int r = ot * 16 + acc_row<T>(g, i);
      va[ot][i] = (aok && r < a.k) ? -V[qa + (int64_t)r * a.ldv] : T(0);
    }
}

template <typename T, int KT, int IB, int NW>
__global__ void __launch_bounds__(NW * 64) k_larfb_stream(LarfbArgs<T> a) {
  typedef typename Acc<T>::type AccT;
  constexpr int KR = KT * 16, CB = IB * 16;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  T* Zs = reinterpret_cast<T*>(smem_raw);  // [NW][KR][CB] partial sums; slot 0 then holds Z
  T* Zp = Zs + (size_t)NW * KR * CB;       // [KR][CB] Z' = T^T Z
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int g = lane >> 4, nl = lane & 15;
  const int c = blockIdx.y;
  const int64_t row0 = (int64_t)c * a.chunk_rows;
  const int Hc = (int)(c == a.P - 1 ? a.h - row0 : a.chunk_rows);
  const int k = a.k;
  const int64_t colbase = a.col0 + (int64_t)blockIdx.x * CB;
  const T* V = a.V + row0;
  const T* Tm = a.Tm + (int64_t)c * a.ldt * a.ldt;
  const int nslab = (Hc + 15) >> 4;

  // ---------------- pass 1: partial Z = V^T C over this wave's slabs ----------------
  AccT Z[KT][IB];
#pragma unroll
  for (int mt = 0; mt < KT; ++mt)
#pragma unroll
    for (int nt = 0; nt < IB; ++nt) Z[mt][nt] = AccT{0, 0, 0, 0};
  {
    T cbA[IB][4], avA[KT][4], cbB[IB][4], avB[KT][4];
    auto mul = [&](T (&cb)[IB][4], T (&av)[KT][4]) {
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int mt = 0; mt < KT; ++mt)
#pragma unroll
          for (int nt = 0; nt < IB; ++nt) Z[mt][nt] = mfma16(av[mt][i], cb[nt][i], Z[mt][nt]);
    };
    int s = wv;
    if (s < nslab) load_slab1<T, KT, IB>(a, V, c, Hc, colbase, s, g, nl, cbA, avA);
    for (; s < nslab; s += 2 * NW) {
      const int s1 = s + NW;
      if (s1 < nslab) load_slab1<T, KT, IB>(a, V, c, Hc, colbase, s1, g, nl, cbB, avB);
      mul(cbA, avA);
      if (s1 >= nslab) break;
      const int s2 = s1 + NW;
      if (s2 < nslab) load_slab1<T, KT, IB>(a, V, c, Hc, colbase, s2, g, nl, cbA, avA);
      mul(cbB, avB);
    }
  }
  // ---------------- reduce the NW partials (fixed order) ----------------
  {
    T* mine = Zs + (size_t)wv * KR * CB;
#pragma unroll
    for (int mt = 0; mt < KT; ++mt)
#pragma unroll
      for (int nt = 0; nt < IB; ++nt)
#pragma unroll
        for (int r = 0; r < 4; ++r) mine[(mt * 16 + acc_row<T>(g, r)) * CB + nt * 16 + nl] = Z[mt][nt][r];
  }
  __syncthreads();
  for (int e = threadIdx.x; e < KR * CB; e += NW * 64) {
    T acc = Zs[e];
    for (int w = 1; w < NW; ++w) acc += Zs[(size_t)w * KR * CB + e];
    Zs[e] = acc;
  }
  __syncthreads();
  // ---------------- Z' = T^T Z (T upper triangular, k x k) ----------------
  for (int e = threadIdx.x; e < KR * CB; e += NW * 64) {
    const int i = e / CB, col = e - i * CB;
    T acc = T(0);
    if (i < k) {
      // all T loads of the sum issued together (one cache round trip, not KR in a row)
      T tv[KR];
#pragma unroll
      for (int l = 0; l < KR; ++l) tv[l] = l <= i ? Tm[l + (int64_t)i * a.ldt] : T(0);
#pragma unroll
      for (int l = 0; l < KR; ++l)
        if (l <= i) acc += tv[l] * Zs[l * CB + col];
    }
    Zp[e] = acc;
  }
  __syncthreads();

  // ---------------- pass 2: C -= V Z' ----------------
  T zb[KT][4][IB];
#pragma unroll
  for (int ot = 0; ot < KT; ++ot)
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int nt = 0; nt < IB; ++nt) zb[ot][i][nt] = Zp[(ot * 16 + acc_row<T>(g, i)) * CB + nt * 16 + nl];

  T cdA[IB][4], vaA[KT][4], cdB[IB][4], vaB[KT][4];
  int64_t grA[4], grB[4];
  auto upd = [&](T (&cd)[IB][4], T (&va)[KT][4], int64_t (&gr)[4]) {
    AccT acc[IB];
#pragma unroll
    for (int nt = 0; nt < IB; ++nt) acc[nt] = AccT{cd[nt][0], cd[nt][1], cd[nt][2], cd[nt][3]};
#pragma unroll
    for (int ot = 0; ot < KT; ++ot)
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int nt = 0; nt < IB; ++nt) acc[nt] = mfma16(va[ot][i], zb[ot][i][nt], acc[nt]);
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      if (gr[i] < 0) continue;
#pragma unroll
      for (int nt = 0; nt < IB; ++nt) {
        const int64_t col = colbase + nt * 16 + nl;
        if (col < a.col1) a.M.at(gr[i], col) = acc[nt][i];
      }
    }
  };
  int s = wv;
  if (s < nslab) load_slab2<T, KT, IB>(a, V, c, Hc, colbase, s, g, nl, cdA, vaA, grA);
  for (; s < nslab; s += 2 * NW) {
    const int s1 = s + NW;
    if (s1 < nslab) load_slab2<T, KT, IB>(a, V, c, Hc, colbase, s1, g, nl, cdB, vaB, grB);
    upd(cdA, vaA, grA);
    if (s1 >= nslab) break;
    const int s2 = s1 + NW;
    if (s2 < nslab) load_slab2<T, KT, IB>(a, V, c, Hc, colbase, s2, g, nl, cdA, vaA, grA);
    upd(cdB, vaB, grB);
  }
}

template <typename T, int KT, int IB, int NW, bool VEC, int PREC>
static hipError_t launch_larfb_reg(const LarfbArgs<T>& a, hipStream_t st) {
  constexpr int SPW = larfb_spw(KT * 16, NW);
  constexpr size_t lds = larfb_reg_lds<T>(KT, IB, NW);
  static bool configured = false;
  if (!configured) {
    hipError_t e = hipFuncSetAttribute((const void*)k_larfb_reg<T, KT, IB, NW, SPW, VEC, PREC>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    configured = true;
  }
  const int64_t ncols = a.col1 - a.col0;
  const dim3 grid((unsigned)((ncols + IB * 16 - 1) / (IB * 16)), (unsigned)a.P);
  hipLaunchKernelGGL((k_larfb_reg<T, KT, IB, NW, SPW, VEC, PREC>), grid, dim3(NW * 64), lds, st, a);
  return hipGetLastError();
}

// Single chunks of at most kSmallUpdateRows rows (the upper levels of a TSQR tree,
// small or nearly finished matrices, batches of small matrices) use the register
// strip with 4 waves of 8 slabs (256 threads) at tile 16, whatever the configured
// thread count: four workgroups fit on a CU instead of one, and a strip holds
// exactly such a chunk.  Single and batched calls make the same choice per matrix.
constexpr int kSmallUpdateRows = 512;
template <typename T>
inline bool small_update_ok(int tile, int ib) { return tile == 16 && (sizeof(T) == 4 ? ib <= 2 : ib == 1); }
inline bool small_update_rows(int P, int64_t h) { return P == 1 && h <= kSmallUpdateRows; }

template <typename T, int IB, bool VEC, int PREC>
static hipError_t launch_larfb_small(const LarfbArgs<T>& a, hipStream_t st) {
  constexpr size_t lds = larfb_reg_lds<T>(1, IB, 4);
  const int64_t ncols = a.col1 - a.col0;
  const dim3 grid((unsigned)((ncols + IB * 16 - 1) / (IB * 16)), 1);
  hipLaunchKernelGGL((k_larfb_reg<T, 1, IB, 4, 8, VEC, PREC>), grid, dim3(256), lds, st, a);
  return hipGetLastError();
}
template <typename T, int IB>
static hipError_t launch_larfb_small_ib(const LarfbArgs<T>& a, hipStream_t st) {
  if constexpr (sizeof(T) == 4) {
    switch (a.prec * 2 + (a.vec ? 1 : 0)) {
      case 0: return launch_larfb_small<T, IB, false, 0>(a, st);
      case 1: return launch_larfb_small<T, IB, true, 0>(a, st);
      case 4: return launch_larfb_small<T, IB, false, 2>(a, st);
      case 5: return launch_larfb_small<T, IB, true, 2>(a, st);
      case 6: return launch_larfb_small<T, IB, false, 3>(a, st);
      case 7: return launch_larfb_small<T, IB, true, 3>(a, st);
    }
    return hipErrorInvalidValue;
  } else {
    if (a.prec != 0) return hipErrorInvalidValue;
    return launch_larfb_small<T, IB, false, 0>(a, st);
  }
}

template <typename T, int IB, bool VEC, int PREC>
static hipError_t launch_larfb_small_b(const LarfbArgs<T>* tab, int count, int64_t max_ncols, hipStream_t st) {
  constexpr size_t lds = larfb_reg_lds<T>(1, IB, 4);
  const dim3 grid((unsigned)((max_ncols + IB * 16 - 1) / (IB * 16)), 1, (unsigned)count);
  hipLaunchKernelGGL((k_larfb_reg_b<T, 1, IB, 4, 8, VEC, PREC>), grid, dim3(256), lds, st, tab, (int64_t)0,
                     (int64_t)kSmallUpdateRows);
  return hipGetLastError();
}
template <typename T, int IB>
static hipError_t launch_larfb_small_b_ib(int prec, int vec, const LarfbArgs<T>* tab, int count, int64_t mc,
                                          hipStream_t st) {
  if constexpr (sizeof(T) == 4) {
    switch (prec * 2 + (vec ? 1 : 0)) {
      case 0: return launch_larfb_small_b<T, IB, false, 0>(tab, count, mc, st);
      case 1: return launch_larfb_small_b<T, IB, true, 0>(tab, count, mc, st);
      case 4: return launch_larfb_small_b<T, IB, false, 2>(tab, count, mc, st);
      case 5: return launch_larfb_small_b<T, IB, true, 2>(tab, count, mc, st);
      case 6: return launch_larfb_small_b<T, IB, false, 3>(tab, count, mc, st);
      case 7: return launch_larfb_small_b<T, IB, true, 3>(tab, count, mc, st);
    }
    return hipErrorInvalidValue;
  } else {
    if (prec != 0) return hipErrorInvalidValue;
    return launch_larfb_small_b<T, IB, false, 0>(tab, count, mc, st);
  }
}

template <typename T, int KT, int IB, int NW>
static hipError_t launch_larfb_stream(const LarfbArgs<T>& a, hipStream_t st) {
  constexpr size_t lds = larfb_lds<T>(KT, IB, NW);
  static bool configured = false;
  if (!configured) {
    hipError_t e = hipFuncSetAttribute((const void*)k_larfb_stream<T, KT, IB, NW>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    configured = true;
  }
  const int64_t ncols = a.col1 - a.col0;
  const dim3 grid((unsigned)((ncols + IB * 16 - 1) / (IB * 16)), (unsigned)a.P);
  hipLaunchKernelGGL((k_larfb_stream<T, KT, IB, NW>), grid, dim3(NW * 64), lds, st, a);
  return hipGetLastError();
}

template <typename T, int KT, int IB, int NW>
static hipError_t launch_larfb_nw(const LarfbArgs<T>& a, hipStream_t st) {
  // the register-strip kernel when the chunk fits in its registers, else the streaming one
  const int64_t cap = (int64_t)larfb_spw(KT * 16, NW) * NW * 16;
  const bool fits = a.chunk_rows <= cap && a.h - (int64_t)(a.P - 1) * a.chunk_rows <= cap;
  if constexpr (larfb_reg_valid<T>(KT, IB, NW)) {
    if (fits) {
      if constexpr (sizeof(T) == 4) {
        if (a.prec == 2) return a.vec ? launch_larfb_reg<T, KT, IB, NW, true, 2>(a, st)
                                      : launch_larfb_reg<T, KT, IB, NW, false, 2>(a, st);
        if (a.prec == 3) return a.vec ? launch_larfb_reg<T, KT, IB, NW, true, 3>(a, st)
                                      : launch_larfb_reg<T, KT, IB, NW, false, 3>(a, st);
        if (a.vec) return launch_larfb_reg<T, KT, IB, NW, true, 0>(a, st);
      }
      if (a.prec != 0) return hipErrorInvalidValue;
      return launch_larfb_reg<T, KT, IB, NW, false, 0>(a, st);
    }
  }
  if (a.prec != 0) return hipErrorInvalidValue;  // reduced precision only in the register-strip form
  if constexpr (larfb_stream_valid<T>(KT, IB, NW)) {
    return launch_larfb_stream<T, KT, IB, NW>(a, st);
  } else {
    return hipErrorInvalidValue;
  }
}

template <typename T, int KT, int IB>
static hipError_t launch_larfb_ib(int nw, const LarfbArgs<T>& a, hipStream_t st) {
  switch (nw) {
    case 1: return launch_larfb_nw<T, KT, IB, 1>(a, st);
    case 2: return launch_larfb_nw<T, KT, IB, 2>(a, st);
    case 4: return launch_larfb_nw<T, KT, IB, 4>(a, st);
    case 8: return launch_larfb_nw<T, KT, IB, 8>(a, st);
    case 16: return launch_larfb_nw<T, KT, IB, 16>(a, st);
  }
  return hipErrorInvalidConfiguration;
}

template <typename T, int KT>
static hipError_t launch_larfb_kt(int nw, int ib, const LarfbArgs<T>& a, hipStream_t st) {
  switch (ib) {
    case 1: return launch_larfb_ib<T, KT, 1>(nw, a, st);
    case 2: return launch_larfb_ib<T, KT, 2>(nw, a, st);
    case 4: return launch_larfb_ib<T, KT, 4>(nw, a, st);
    case 8: return launch_larfb_ib<T, KT, 8>(nw, a, st);
  }
  return hipErrorInvalidConfiguration;
}

template <typename T, int KT, int IB, int NW, bool VEC, int PREC>
static hipError_t launch_larfb_reg_b(const LarfbArgs<T>* tab, int count, int64_t max_ncols, int64_t h_lo,
                                     hipStream_t st) {
  constexpr int SPW = larfb_spw(KT * 16, NW);
  constexpr size_t lds = larfb_reg_lds<T>(KT, IB, NW);
  static bool configured = false;
  if (!configured) {
    hipError_t e = hipFuncSetAttribute((const void*)k_larfb_reg_b<T, KT, IB, NW, SPW, VEC, PREC>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    configured = true;
  }
  const dim3 grid((unsigned)((max_ncols + IB * 16 - 1) / (IB * 16)), 1, (unsigned)count);
  hipLaunchKernelGGL((k_larfb_reg_b<T, KT, IB, NW, SPW, VEC, PREC>), grid, dim3(NW * 64), lds, st, tab, h_lo,
                     (int64_t)INT64_MAX);
  return hipGetLastError();
}

template <typename T, int KT, int IB, int NW>
static hipError_t launch_larfb_b_nw(int prec, int vec, const LarfbArgs<T>* tab, int count, int64_t max_ncols,
                                    int64_t h_lo, hipStream_t st) {
  if constexpr (larfb_reg_valid<T>(KT, IB, NW)) {
    if constexpr (sizeof(T) == 4) {
      switch (prec * 2 + (vec ? 1 : 0)) {
        case 0: return launch_larfb_reg_b<T, KT, IB, NW, false, 0>(tab, count, max_ncols, h_lo, st);
        case 1: return launch_larfb_reg_b<T, KT, IB, NW, true, 0>(tab, count, max_ncols, h_lo, st);
        case 4: return launch_larfb_reg_b<T, KT, IB, NW, false, 2>(tab, count, max_ncols, h_lo, st);
        case 5: return launch_larfb_reg_b<T, KT, IB, NW, true, 2>(tab, count, max_ncols, h_lo, st);
        case 6: return launch_larfb_reg_b<T, KT, IB, NW, false, 3>(tab, count, max_ncols, h_lo, st);
        case 7: return launch_larfb_reg_b<T, KT, IB, NW, true, 3>(tab, count, max_ncols, h_lo, st);
      }
      return hipErrorInvalidValue;
    } else {
      if (prec != 0) return hipErrorInvalidValue;
      return launch_larfb_reg_b<T, KT, IB, NW, false, 0>(tab, count, max_ncols, h_lo, st);
    }
  } else {
    return hipErrorInvalidConfiguration;  // the batched path needs the register-strip form
  }
}

template <typename T, int KT, int IB>
static hipError_t launch_larfb_b_ib(int nw, int prec, int vec, const LarfbArgs<T>* tab, int count, int64_t mc,
                                    int64_t h_lo, hipStream_t st) {
  switch (nw) {
    case 1: return launch_larfb_b_nw<T, KT, IB, 1>(prec, vec, tab, count, mc, h_lo, st);
    case 2: return launch_larfb_b_nw<T, KT, IB, 2>(prec, vec, tab, count, mc, h_lo, st);
    case 4: return launch_larfb_b_nw<T, KT, IB, 4>(prec, vec, tab, count, mc, h_lo, st);
    case 8: return launch_larfb_b_nw<T, KT, IB, 8>(prec, vec, tab, count, mc, h_lo, st);
    case 16: return launch_larfb_b_nw<T, KT, IB, 16>(prec, vec, tab, count, mc, h_lo, st);
  }
  return hipErrorInvalidConfiguration;
}

template <typename T, int KT>
static hipError_t launch_larfb_b_kt(int nw, int ib, int prec, int vec, const LarfbArgs<T>* tab, int count, int64_t mc,
                                    int64_t h_lo, hipStream_t st) {
  switch (ib) {
    case 1: return launch_larfb_b_ib<T, KT, 1>(nw, prec, vec, tab, count, mc, h_lo, st);
    case 2: return launch_larfb_b_ib<T, KT, 2>(nw, prec, vec, tab, count, mc, h_lo, st);
    case 4: return launch_larfb_b_ib<T, KT, 4>(nw, prec, vec, tab, count, mc, h_lo, st);
    case 8: return launch_larfb_b_ib<T, KT, 8>(nw, prec, vec, tab, count, mc, h_lo, st);
  }
  return hipErrorInvalidConfiguration;
}

// ---- split form of one tall panel ----
// Rows per first-pass workgroup: whole register blocks of R0 rows, enough row ranges
// that strips x ranges reaches about 4096 workgroups, and no more, so the partial
// sums (KR x CB per workgroup) stay a small fraction of C.
static int64_t split_p1_rows(int64_t h, int64_t nstrips, int64_t R0) {
  const int64_t nb = (h + R0 - 1) / R0;
  const int64_t ranges = std::max<int64_t>(1, std::min<int64_t>(nb, (4096 + nstrips - 1) / nstrips));
  return (nb + ranges - 1) / ranges * R0;
}

template <typename T, int KT, int IB, int NW, bool VEC>
static hipError_t launch_larfb_split_v(const LarfbArgs<T>& a0, T* zw, hipStream_t st) {
  constexpr int SPW = larfb_spw(KT * 16, NW), KR = KT * 16, CB = IB * 16;
  constexpr int64_t R0 = (int64_t)SPW * NW * 16;  // rows of one register block
  constexpr size_t lds1 = (size_t)NW * KR * CB * sizeof(T);
  constexpr size_t lds2 = larfb_reg_lds<T>(KT, IB, NW);  // pass 2 uses the per-wave transpose slabs
  const int64_t nstrips = (a0.col1 - a0.col0 + CB - 1) / CB;
  LarfbArgs<T> a1 = a0, a2 = a0;
  a1.chunk_rows = split_p1_rows(a0.h, nstrips, R0);  // first pass: row ranges of whole blocks
  a1.P = (int32_t)((a0.h + a1.chunk_rows - 1) / a1.chunk_rows);
  a1.rm.chunk_stride = a1.chunk_rows;
  a2.chunk_rows = R0;  // second pass: one register block per workgroup
  a2.P = (int32_t)((a0.h + R0 - 1) / R0);
  a2.rm.chunk_stride = R0;
  if (a2.P > 65535) return hipErrorInvalidValue;  // grid y limit
  T* zpart = zw;
  T* zprime = zw + (int64_t)a1.P * nstrips * KR * CB;
  static bool configured = false;
  if (!configured) {
    hipError_t e = hipFuncSetAttribute((const void*)k_larfb_split_p1<T, KT, IB, NW, SPW, VEC>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds1);
    if (e == hipSuccess)
      e = hipFuncSetAttribute((const void*)k_larfb_split_p2<T, KT, IB, NW, SPW, VEC>,
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds2);
    if (e != hipSuccess) return e;
    configured = true;
  }
  hipLaunchKernelGGL((k_larfb_split_p1<T, KT, IB, NW, SPW, VEC>), dim3((unsigned)nstrips, (unsigned)a1.P),
                     dim3(NW * 64), lds1, st, a1, zpart);
  hipLaunchKernelGGL((k_larfb_split_z<T, KT, IB>), dim3((unsigned)nstrips), dim3(256), 0, st, (const T*)zpart, zprime,
                     (int)a1.P, a0.Tm, a0.ldt, a0.k);
  hipLaunchKernelGGL((k_larfb_split_p2<T, KT, IB, NW, SPW, VEC>), dim3((unsigned)nstrips, (unsigned)a2.P),
                     dim3(NW * 64), lds2, st, a2, zprime);
  return hipGetLastError();
}
template <typename T, int KT, int IB, int NW>
static hipError_t launch_larfb_split_nw(const LarfbArgs<T>& a, T* zw, hipStream_t st) {
  if constexpr (larfb_reg_valid<T>(KT, IB, NW)) {
    if constexpr (sizeof(T) == 4) {
      if (a.vec) return launch_larfb_split_v<T, KT, IB, NW, true>(a, zw, st);
    }
    return launch_larfb_split_v<T, KT, IB, NW, false>(a, zw, st);
  } else {
    return hipErrorInvalidConfiguration;
  }
}
template <typename T, int KT, int IB>
static hipError_t launch_larfb_split_ib(int nw, const LarfbArgs<T>& a, T* zw, hipStream_t st) {
  switch (nw) {
    case 8: return launch_larfb_split_nw<T, KT, IB, 8>(a, zw, st);
    case 16: return launch_larfb_split_nw<T, KT, IB, 16>(a, zw, st);
  }
  return hipErrorInvalidConfiguration;
}
template <typename T, int KT>
static hipError_t launch_larfb_split_kt(int nw, int ib, const LarfbArgs<T>& a, T* zw, hipStream_t st) {
  switch (ib) {
    case 1: return launch_larfb_split_ib<T, KT, 1>(nw, a, zw, st);
    case 2: return launch_larfb_split_ib<T, KT, 2>(nw, a, zw, st);
    case 4: return launch_larfb_split_ib<T, KT, 4>(nw, a, zw, st);
    case 8: return launch_larfb_split_ib<T, KT, 8>(nw, a, zw, st);
  }
  return hipErrorInvalidConfiguration;
}

template <typename T>
bool larfb_split_ok(int tile, int nw, int ib) {
  const int kt = tile / 16;
  auto ok = [&](auto KTc) {
    constexpr int KT = decltype(KTc)::value;
    switch (nw * 16 + ib) {
      case 8 * 16 + 1: return larfb_reg_valid<T>(KT, 1, 8);
      case 8 * 16 + 2: return larfb_reg_valid<T>(KT, 2, 8);
      case 8 * 16 + 4: return larfb_reg_valid<T>(KT, 4, 8);
      case 8 * 16 + 8: return larfb_reg_valid<T>(KT, 8, 8);
      case 16 * 16 + 1: return larfb_reg_valid<T>(KT, 1, 16);
      case 16 * 16 + 2: return larfb_reg_valid<T>(KT, 2, 16);
      case 16 * 16 + 4: return larfb_reg_valid<T>(KT, 4, 16);
      case 16 * 16 + 8: return larfb_reg_valid<T>(KT, 8, 16);
    }
    return false;
  };
  switch (kt) {
    case 1: return ok(std::integral_constant<int, 1>{});
    case 2: return ok(std::integral_constant<int, 2>{});
    case 4: return ok(std::integral_constant<int, 4>{});
    case 8: return ok(std::integral_constant<int, 8>{});
  }
  return false;
}

template <typename T>
int64_t larfb_split_work(int tile, int nw, int ib, int64_t h, int64_t ncols) {
  const int64_t R0 = (int64_t)larfb_spw(tile, nw) * nw * 16;
  const int64_t CB = 16 * ib, nstrips = (ncols + CB - 1) / CB;
  const int64_t R1 = split_p1_rows(h, nstrips, R0), P1 = (h + R1 - 1) / R1;
  return (P1 + 1) * nstrips * tile * CB;
}

template <typename T>
hipError_t launch_larfb_split(int tile, int nw, int ib, const LarfbArgs<T>& a, T* zw, hipStream_t st) {
  if (a.col1 <= a.col0 || a.k <= 0) return hipSuccess;
  if (a.prec != 0) return hipErrorInvalidValue;
  switch (tile) {
    case 16: return launch_larfb_split_kt<T, 1>(nw, ib, a, zw, st);
    case 32: return launch_larfb_split_kt<T, 2>(nw, ib, a, zw, st);
    case 64: return launch_larfb_split_kt<T, 4>(nw, ib, a, zw, st);
    case 128: return launch_larfb_split_kt<T, 8>(nw, ib, a, zw, st);
  }
  return hipErrorInvalidValue;
}
template bool larfb_split_ok<float>(int, int, int);
template bool larfb_split_ok<double>(int, int, int);
template int64_t larfb_split_work<float>(int, int, int, int64_t, int64_t);
template int64_t larfb_split_work<double>(int, int, int, int64_t, int64_t);
template hipError_t launch_larfb_split<float>(int, int, int, const LarfbArgs<float>&, float*, hipStream_t);
template hipError_t launch_larfb_split<double>(int, int, int, const LarfbArgs<double>&, double*, hipStream_t);

template <typename T>
hipError_t launch_larfb_batched(int tile, int nw, int ib, int prec, int vec, const LarfbArgs<T>* tab, int count,
                                int64_t max_ncols, int64_t min_rows, int64_t max_rows, hipStream_t st) {
  if (count <= 0 || max_ncols <= 0) return hipSuccess;
  int64_t h_lo = 0;  // the general launch takes the matrices taller than h_lo
  if (small_update_ok<T>(tile, ib) && min_rows <= kSmallUpdateRows) {
    hipError_t e = ib == 1 ? launch_larfb_small_b_ib<T, 1>(prec, vec, tab, count, max_ncols, st)
                           : launch_larfb_small_b_ib<T, 2>(prec, vec, tab, count, max_ncols, st);
    if (e != hipSuccess) return e;
    if (max_rows <= kSmallUpdateRows) return hipSuccess;
    h_lo = kSmallUpdateRows;
  }
  switch (tile) {
    case 16: return launch_larfb_b_kt<T, 1>(nw, ib, prec, vec, tab, count, max_ncols, h_lo, st);
    case 32: return launch_larfb_b_kt<T, 2>(nw, ib, prec, vec, tab, count, max_ncols, h_lo, st);
    case 64: return launch_larfb_b_kt<T, 4>(nw, ib, prec, vec, tab, count, max_ncols, h_lo, st);
    case 128: return launch_larfb_b_kt<T, 8>(nw, ib, prec, vec, tab, count, max_ncols, h_lo, st);
  }
  return hipErrorInvalidValue;
}

template <typename T>
hipError_t launch_larfb(int tile, int nw, int ib, const LarfbArgs<T>& a, hipStream_t st) {
  if (a.col1 <= a.col0 || a.k <= 0) return hipSuccess;
  if (small_update_ok<T>(tile, ib) && small_update_rows(a.P, a.h))
    return ib == 1 ? launch_larfb_small_ib<T, 1>(a, st) : launch_larfb_small_ib<T, 2>(a, st);
  switch (tile) {
    case 16: return launch_larfb_kt<T, 1>(nw, ib, a, st);
    case 32: return launch_larfb_kt<T, 2>(nw, ib, a, st);
    case 64: return launch_larfb_kt<T, 4>(nw, ib, a, st);
    case 128: return launch_larfb_kt<T, 8>(nw, ib, a, st);
  }
  return hipErrorInvalidValue;
}

template hipError_t launch_larfb<float>(int, int, int, const LarfbArgs<float>&, hipStream_t);
template hipError_t launch_larfb<double>(int, int, int, const LarfbArgs<double>&, hipStream_t);
template hipError_t launch_larfb_batched<float>(int, int, int, int, int, const LarfbArgs<float>*, int, int64_t,
                                                int64_t, int64_t, hipStream_t);
template hipError_t launch_larfb_batched<double>(int, int, int, int, int, const LarfbArgs<double>*, int, int64_t,
                                                 int64_t, int64_t, hipStream_t);

}  // namespace svdv
