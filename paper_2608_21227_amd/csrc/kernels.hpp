// Kernel argument blocks, compile-time configuration tables and launcher
// declarations shared by the stage sources and the host pipeline.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>
#include "common.hpp"

namespace svdv {

// Records an error detail for svdv_last_error and returns status.
int report_error(int status, const char* msg);

// Rows per lane of the chunk-QR kernel (16 waves, one chunk in registers):
// 64 * RPT rows * TILE columns = 32 elements per thread (16 for float64 at
// tile 16, whose single column per wave would otherwise not fit in registers).
template <typename T, int TILE> struct ChunkRPT {
  static constexpr int value = (sizeof(T) == 8 && TILE == 16 ? 256 : 512) / TILE;
};

template <typename T>
struct ChunkQRArgs {
  View<T> M;          // matrix view holding the panel (column-major or transposed)
  int64_t pc;         // first panel column (view coordinates)
  int32_t bw;         // panel width
  RowMap rm;          // rows of chunk c
  int64_t h;          // total rows at this tree level
  int64_t chunk_rows; // rows per chunk (the last chunk takes the remainder)
  int32_t P;          // chunks at this level
  T* V;               // Householder vectors, chunk c at rows [c*chunk_rows, ...), leading dim ldv
  int64_t ldv;
  T* Tm;              // compact-WY factors, chunk c at Tm + c*TILE*TILE (TILE x TILE column-major)
  int32_t hp;         // float32 storage factored in float64 arithmetic (BF16/FP16 trailing updates)
};

template <typename T>
struct LarfbArgs {
  View<T> M;          // matrix view holding C
  RowMap rm;          // rows of chunk c (same map as the factorisation of that level)
  int64_t h, chunk_rows;
  int32_t P;
  int64_t col0, col1; // view columns to update
  const T* V;
  int64_t ldv;
  const T* Tm;
  int64_t ldt;        // = TILE (per-chunk T is ldt x ldt)
  int32_t k;          // reflectors per chunk
  int32_t vec;        // 1: view rows contiguous in memory and every 4-row group of C and V
                      // 16-byte aligned (float only), so 4 rows load as one access
  int32_t prec;       // MFMA operand precision: 0 = T, 2 = BF16, 3 = FP16 (float only)
  int32_t vecv = 0;   // 1: V alone allows 16-byte loads of 4 rows (float only; C may not,
                      // as in the LQ sweep, whose view rows are memory columns)
};

// Slabs (16 rows) per wave of the trailing update: enough for the largest chunk a
// panel level can have (at most the chunk-QR capacity, 32768 / tile rows).
constexpr int larfb_spw(int tile, int NW) { return ((32768 / tile + 15) / 16 + NW - 1) / NW; }
// Register estimates (32-bit registers per lane), calibrated against the
// compiler's resource report so that no configuration taken spills to scratch.
//  register-strip kernel: the strip (SPW x IB tiles), V operands (SPW x KT tiles),
//  Z and Z' (KT x IB tiles each) and addressing;
//  streaming kernel: Z and Z' tiles, two slabs of C and of V in flight.
template <typename T>
constexpr int larfb_reg_regs(int KT, int IB, int NW) {
  return (larfb_spw(KT * 16, NW) * 4 * (IB + KT) + 8 * KT * IB + 48) * (int)(sizeof(T) / 4);
}
template <typename T>
constexpr int larfb_stream_regs(int KT, int IB) {
  return (2 * KT * IB * 4 + 3 * IB * 4 + 2 * KT * 4 + 48) * (int)(sizeof(T) / 4);
}
constexpr int larfb_reg_budget(int NW) { return NW >= 16 ? 128 : (NW >= 8 ? 240 : 0); }
constexpr int larfb_stream_budget(int NW) { return NW >= 16 ? 96 : (NW >= 8 ? 176 : 256); }
// LDS: NW partial Z tiles plus Z' (each KT*16 x IB*16).
template <typename T>
constexpr size_t larfb_lds(int KT, int IB, int NW) {
  return (size_t)(NW + 1) * (KT * 16) * (IB * 16) * sizeof(T);
}
// Register-strip kernel: the partial Z tiles, or (once Z' is formed) one 16-row
// V slab per wave being transposed for pass 2 (rows padded by 4), then Z'.
constexpr int64_t larfb_reg_lds_elems(int KT, int IB, int NW) {
  const int64_t kr = KT * 16, cb = IB * 16;
  return (NW * kr * cb > NW * 16 * (kr + 4) ? NW * kr * cb : NW * 16 * (kr + 4)) + kr * cb;
}
template <typename T>
constexpr size_t larfb_reg_lds(int KT, int IB, int NW) {
  return (size_t)larfb_reg_lds_elems(KT, IB, NW) * sizeof(T);
}
template <typename T>
constexpr bool larfb_reg_valid(int KT, int IB, int NW) {
  return larfb_reg_regs<T>(KT, IB, NW) <= larfb_reg_budget(NW) && larfb_reg_lds<T>(KT, IB, NW) <= 128 * 1024;
}
template <typename T>
constexpr bool larfb_stream_valid(int KT, int IB, int NW) {
  return larfb_stream_regs<T>(KT, IB) <= larfb_stream_budget(NW) && !(sizeof(T) == 8 && KT > 4) &&
         larfb_lds<T>(KT, IB, NW) <= 128 * 1024;
}
template <typename T>
constexpr bool larfb_valid(int KT, int IB, int NW) {
  return larfb_reg_valid<T>(KT, IB, NW) || larfb_stream_valid<T>(KT, IB, NW);
}

// One matrix of a batch: its input, output and workspace pieces (device pointers).
template <typename T>
struct BatchMat {
  const T* A;            // input, column-major, lda
  int64_t m, n, lda;
  int32_t transpose;     // 1 when m < n (the transpose is reduced)
  int64_t M, N;          // reduced matrix (M >= N)
  T* W;                  // working copy, M x N, leading dimension ldw
  int64_t ldw;
  unsigned long long* amax;
  int* exp;              // power-of-two scale exponent
  double* Bs;            // chase storage (N x 3b)
  double* d;
  double* e;
  double* work;          // bisection work (bisect_work_doubles(N))
  T* S;                  // output singular values (min(m, n))
};

// Fill kernels (used instead of hipMemsetAsync so that every step can be captured in a graph).
__global__ void k_fill_u64(unsigned long long* p, unsigned long long v, int64_t n);
__global__ void k_fill_i32(int* p, int v, int64_t n);
__global__ void k_fill_f64(double* p, double v, int64_t n);
__global__ void k_finish_de(const int* flag, const int* exp, double* d, double* e, int64_t n);

template <typename T>
hipError_t launch_stage_in(const T* A, int64_t m, int64_t n, int64_t lda, int transpose, T* W, int64_t ldw,
                           unsigned long long* amax, int* exp_out, hipStream_t st);
template <typename T> int chunk_qr_hmax(int tile);
template <typename T> hipError_t launch_chunk_qr(int tile, const ChunkQRArgs<T>& a, hipStream_t st);
// Batched forms (argument tables in device memory, one entry per matrix).
template <typename T> hipError_t launch_chunk_qr_batched(int tile, const ChunkQRArgs<T>* tab, int count, int hp,
                                                          hipStream_t st);
template <typename T>
hipError_t launch_stage_in_batched(const BatchMat<T>* tab, int count, unsigned long long* amax_all, int64_t max_elems,
                                   hipStream_t st);
template <typename T>
hipError_t launch_band_pack_batched(const BatchMat<T>* tab, int count, int b, int64_t max_n, hipStream_t st);
template <typename T>
// min_rows / max_rows: the smallest and largest panel height h of the step's matrices.
hipError_t launch_larfb_batched(int tile, int nw, int ib, int prec, int vec, const LarfbArgs<T>* tab, int count,
                                int64_t max_ncols, int64_t min_rows, int64_t max_rows, hipStream_t st);
template <typename T> hipError_t launch_larfb(int tile, int nw, int ib, const LarfbArgs<T>& a, hipStream_t st);
// Split form of one panel taller than a register strip (a.P == 1, a.h rows):
// row blocks of the strip capacity; zw: larfb_split_work() elements of device
// workspace.  Available when the register-strip kernel is (larfb_split_ok).
template <typename T> bool larfb_split_ok(int tile, int nw, int ib);
template <typename T> int64_t larfb_split_work(int tile, int nw, int ib, int64_t h, int64_t ncols);
template <typename T>
hipError_t launch_larfb_split(int tile, int nw, int ib, const LarfbArgs<T>& a, T* zw, hipStream_t st);
template <typename T>
hipError_t launch_band_pack(const T* W, int64_t ldw, int64_t n, int b, double* Bs, int64_t ldb, const int* exp_in,
                            int unscale, hipStream_t st);
template <typename T>
hipError_t launch_band_extract(const T* W, int64_t ldw, int64_t n, int b, double* out, int64_t ldo, const int* exp_in,
                               hipStream_t st);
hipError_t launch_band_import(const double* in, int64_t ldi, int64_t n, int b, double* Bs, int64_t ldb, int* nonfinite,
                              hipStream_t st);
// max |Bs| over n rows of ldb entries, then Bs scaled in place by the power of two
// 2^-e that brings it into [0.5, 1); *exp_out receives e
hipError_t launch_band_scale(double* Bs, int64_t ldb, int64_t n, unsigned long long* amax, int* exp_out,
                             hipStream_t st);

// Stage 2.
struct ChaseArgs {
  double* Bs;          // chase storage, row-major, row i at Bs + i*ldb; column j at offset j - i + (b-1)
                       // (ldb = 3b: the windowed kernels rely on it)
  int64_t ldb;
  int64_t n;
  int32_t b;
  int32_t W;           // sweeps per workgroup (sweep width)
  int32_t ngroups;     // ceil((n-1) / W)
  int32_t* progress;   // per group: tasks completed by its last sweep; entry ngroups is the
                       // group ticket (ngroups + 1 entries, zeroed before launch)
  int32_t* err;        // set when a bounded wait gives up
  double* d;
  double* e;
  // launch-level fields (set by the launchers): group tickets come from *ticket;
  // a batched launch maps ticket t to matrix order[2t] (its arguments tab[...])
  // and group order[2t+1]; total = number of tickets.
  const ChaseArgs* tab;
  const int* order;
  int* ticket;
  int32_t total;
};
size_t chase_lds_bytes(int b, int W);
int chase_max_groups_resident(int b, int W);
hipError_t launch_chase(const ChaseArgs& a, int grid, hipStream_t st);
// Batched chase: L carries b, W, tab, order, ticket and total; zero_base[0 .. zero_count)
// (every matrix's progress counters and the ticket) is cleared first; then d, e of every
// matrix are extracted.
hipError_t launch_chase_batched(const ChaseArgs& L, int grid, int count, int64_t max_n, int* zero_base,
                                int64_t zero_count, hipStream_t st);

// Stage 3.
// Work array of an n x n bidiagonal: d_i^2 [n], e_i^2 [n], bound, pivmin, then
// the int32 counts of the shared grid (bisect_grid_points(n) of them).
__host__ __device__ inline int64_t bisect_grid_points(int64_t n) { return 16 * n; }
__host__ __device__ inline int64_t bisect_work_doubles(int64_t n) { return 2 * n + 3 + (bisect_grid_points(n) + 1) / 2; }
__host__ __device__ inline int* bisect_grid_counts(double* work, int64_t n) { return (int*)(work + 2 * n + 3); }
__host__ __device__ inline const int* bisect_grid_counts(const double* work, int64_t n) {
  return (const int*)(work + 2 * n + 3);
}
// lanes_per_value: 8, 16, 32 or 64, or 0 to choose from n.
// fail_flag (optional): when it holds a nonzero value (a bounded wait of the chase
// gave up), every output value is NaN.
template <typename T>
hipError_t launch_bisect(const double* d, const double* e, int64_t n, T* S, double* work, const int* exp_in,
                         int lanes_per_value, hipStream_t st, const int* fail_flag = nullptr);
// Batched: value v (0 <= v < total) of the flattened batch is value v - voff[vmat[v]] of matrix vmat[v];
// max_n is the largest N of the batch; fail_flag as above, for the whole batch.
template <typename T>
hipError_t launch_bisect_batched(const BatchMat<T>* tab, int count, const int* vmat, const int64_t* voff, int64_t total,
                                 int64_t max_n, hipStream_t st, const int* fail_flag);

}  // namespace svdv
