// (+,*) FP64 inner product at FP64 accuracy from BF16 slices on the matrix
// cores — the split scheme of Ozaki, Ogita, Oishi & Rump (Numer. Algorithms 59,
// 2012), with signed digits. The (+,*) case of Eq. inner (Section I) on the
// flattened M x K and K x N views.
//
// Scheme. Row i of A is scaled by 2^-e_i and column j of B by 2^-f_j, where
// 2^e is the smallest power of two above the row (column) maximum, so scaled
// entries x lie in (-1, 1). Each x is written as signed base-2^9 digits
//     x = sum_s sigma_s 2^-(8 + 9 s),  |sigma_s| <= 256,
// every digit an integer that BF16 holds exactly (stored times its weight
// 2^-9s, still exact). With S digits per operand the pairs (s, t), s + t < S
// are kept; pairs of equal level d = s + t carry the same weight
// 2^-(16 + 9 d), so they share one FP32 accumulator per level:
//     D_ij = 2^(e_i + f_j - 16) * sum_d 2^-9d T_d[i, j],
//     T_d = sum_{s+t=d} sigma^A_s . sigma^B_t   (integer-valued).
// Products of digits are at most 2^16, so an FP32 level accumulator is exact
// over a bounded number of k values; the product kernel (split_gemm.hpp) folds
// each level into FP64 within that bound and scales back by 2^(e_i + f_j) at
// the end.
//
// Data layout. Slices are written once, in the operand layout of
// v_mfma_f32_32x32x16_bf16: a "chunk" is the 32 x 16 (A) or 16 x 32 (B)
// fragment of one slice, 64 lanes x 8 BF16 = 1 KiB, lane l holding row (col)
// l % 32 and k = 8 * (l / 32) .. + 7. Chunks are ordered
// [row block][k block][slice], so the slices of consecutive k blocks of one
// row block are one contiguous run. The product kernel copies runs straight
// into LDS with global_load_lds_dwordx4 (no staging registers) and each wave
// reads a fragment back as one conflict-free ds_read_b128.
//
// This file holds the row/column scans, the slicing kernels and the launch
// plan; the product kernel is in split_gemm.hpp.
#include "common.hpp"
#include "internal.hpp"
#include "split_gemm.hpp"
#include "split_gemm_f8.hpp"

namespace moa {

namespace {

using split::exponent_of_max;
using split::kBeta;
constexpr int kFlushK = 64;  // K is padded to a multiple of this

// Slice-pair kernel layout by slice count. Up to 5 slices: 4 x 2 waves of
// 32 x 64 (128 x 128 tile, two waves per SIMD), one 16-k block per LDS stage,
// four stages in rotation (all 160 KiB of LDS; 11.79-11.89 ms against
// 12.08 ms with three at 8192^3, S = 5, same box); against 2 x 4 waves of
// 32 x 32 (64 x 128 tile) a 16-k block reads 27% fewer LDS bytes per MFMA and
// a third fewer slice bytes per flop. 6 and 7 slices need more fragment
// registers and keep 32 x 32 per wave: 2 x 4 waves (6) or 2 x 2 (7), two 16-k
// blocks per stage, two stages.
template <int S>
struct Layout {
  static constexpr bool kWide = S <= 5;
  static constexpr int WMW = kWide ? 4 : 2, WNW = kWide ? 2 : (S <= 6 ? 4 : 2), WN = kWide ? 2 : 1;
  static constexpr int SKB = kWide ? 1 : 2, NBUF = kWide ? 4 : 2;
  // The pipelined loop (buffer loads into LDS) for the wide layout; its
  // per-stream descriptors need the stream's slice bytes below 2^31.
  static constexpr bool PIPE = kWide;
  using C = split::Cfg<S, WMW, WNW, WN, SKB, NBUF>;
};

static void tile_of(int S, int *bm, int *bn) {
  *bm = S <= 5 ? 128 : 64;
  *bn = S <= 6 ? 128 : 64;
}

// Row maxima of |A| (M x K row-major): one wave per row; IEEE bit pattern out.
__global__ __launch_bounds__(256) void k_scan_rows(const double *__restrict__ A, int64_t M, int64_t K,
                                                   uint64_t *__restrict__ rowmax, int64_t Mp) {
  const int64_t row = (int64_t)blockIdx.x * 4 + threadIdx.x / 64;
  const int lane = threadIdx.x % 64;
  if (row >= Mp) return;
  double mx = 0.0;
  if (row < M)
    for (int64_t k = lane; k < K; k += 64) mx = fmax(mx, fabs(A[row * K + k]));
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) mx = fmax(mx, __shfl_xor(mx, o));
  if (lane == 0) rowmax[row] = (uint64_t)__double_as_longlong(mx);
}

__global__ __launch_bounds__(256) void k_zero_u64(uint64_t *p, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) p[i] = 0;
}

// Column maxima of |B| (K x N row-major): thread per column over a band of
// rows; bands merged with an atomic max on the bit pattern (monotonic for
// non-negative doubles).
__global__ __launch_bounds__(256) void k_scan_cols(const double *__restrict__ B, int64_t K, int64_t N, int64_t band,
                                                   uint64_t *__restrict__ colmax) {
  const int64_t col = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int64_t k0 = (int64_t)blockIdx.y * band;
  if (col >= N) return;
  const int64_t k1 = (k0 + band) < K ? (k0 + band) : K;
  double mx = 0.0;
  for (int64_t k = k0; k < k1; ++k) mx = fmax(mx, fabs(B[k * N + col]));
  if (mx > 0.0) atomicMax((unsigned long long *)&colmax[col], (unsigned long long)__double_as_longlong(mx));
}

// Signed digits of 8 consecutive-k values of one row (A) or column (B):
// sig[s] holds digit s of each of the 8 values times its weight 2^(-9 s), as
// BF16 (exact: |digit| <= 256 needs 8 significant bits, and the power of two
// only moves the exponent). With weighted digits every slice-pair product
// carries the weight of its level, so levels can share accumulators.
template <int S>
__device__ __forceinline__ void digits8(const double v[8], int e, bf16x8 sig[S]) {
#pragma unroll
  for (int q = 0; q < 8; ++q) {
    double r = ldexp(v[q], kBeta - 1 - e);  // x * 2^(beta-1), exact
#pragma unroll
    for (int s = 0; s < S; ++s) {
      const double d = rint(r);
      sig[s][q] = (__bf16)(float)(d * __builtin_ldexp(1.0, -kBeta * s));
      r = (r - d) * (double)(1 << kBeta);
    }
  }
}

// INT8 slices (MOA_SPLIT_INT8): signed digits of 7 bits, |digit| <= 64,
// chunk = 64 lanes x 16 INT8 (a 32 x 32 operand of v_mfma_i32_32x32x32_i8,
// lane l holding row/col l % 32 and k = 16 * (l / 32) .. + 15).
template <int S>
__device__ __forceinline__ void digits16_i8(const double v[16], int e, split::i8::intx4 sig[S]) {
  constexpr int kB = split::i8::kBeta;
#pragma unroll
  for (int s = 0; s < S; ++s) sig[s] = split::i8::intx4{0, 0, 0, 0};
#pragma unroll
  for (int q = 0; q < 16; ++q) {
    double r = ldexp(v[q], kB - 1 - e);  // x * 2^(beta-1), exact
#pragma unroll
    for (int s = 0; s < S; ++s) {
      const double d = rint(r);
      sig[s][q / 4] |= ((int)d & 0xff) << (8 * (q % 4));
      r = (r - d) * (double)(1 << kB);
    }
  }
}

// FP8 slices (MOA_SPLIT_FP8): signed digits of 5 bits, |digit| <= 16, each
// an E4M3 value exactly (4 significant bits); chunk = 64 lanes x 32 FP8 (a
// 32 x 64 operand of v_mfma_scale_f32_32x32x64_f8f6f4, lane l holding
// row/col l % 32 and k = 32 * (l / 32) .. + 31), stored as two 1-KiB halves
// (lane l's bytes 0-15, then its bytes 16-31) so each half is one
// 16-byte-per-lane copy. sig[s][h]: the 16 digits of slice s in half h.
template <int S>
__device__ __forceinline__ void digits32_f8(const double v[32], int e, split::f8::intx4 sig[S][2]) {
  constexpr int kB = split::f8::kBeta;
#pragma unroll
  for (int s = 0; s < S; ++s) sig[s][0] = sig[s][1] = split::f8::intx4{0, 0, 0, 0};
#pragma unroll
  for (int q = 0; q < 32; q += 2) {
    double r0 = ldexp(v[q], kB - 1 - e), r1 = ldexp(v[q + 1], kB - 1 - e);  // x * 2^(beta-1), exact
#pragma unroll
    for (int s = 0; s < S; ++s) {
      const double d0 = rint(r0), d1 = rint(r1);
      // Two digits into bytes 0-1 (q % 4 == 0) or 2-3 of the dword; exact.
      const int old = sig[s][q / 16][(q % 16) / 4];
      const int w = (q % 4 == 0) ? __builtin_amdgcn_cvt_pk_fp8_f32((float)d0, (float)d1, 0, false)
                                 : __builtin_amdgcn_cvt_pk_fp8_f32((float)d0, (float)d1, old, true);
      sig[s][q / 16][(q % 16) / 4] = w;
      r0 = (r0 - d0) * (double)(1 << kB);
      r1 = (r1 - d1) * (double)(1 << kB);
    }
  }
}

// A slices. A wave owns one chunk: row block mb (32 rows) and k block kb (CK =
// 16 k for BF16, 32 for INT8, 64 for FP8). It copies the chunk's block of A into its own
// LDS region with row-contiguous loads (CK lanes per row, 64 / CK rows per
// load), then each lane reads back the values of its operand slot (row l % 32,
// k = CK / 2 * (l / 32) ..) and writes their digits. Loading A directly in the
// operand layout would make every load instruction touch 64 rows. The INT8
// block (32 x 32) is staged 16 rows at a time, so the LDS a workgroup needs
// stays small enough for 8 waves per SIMD (32 rows at once: 0.272 ms, 16 at a
// time: 0.231 ms at 8192^2); the FP8 block (32 x 64) likewise.
// F: slice format, 0 = BF16, 1 = INT8, 2 = FP8.
template <int S, int F>
__global__ __launch_bounds__(256) void k_slice_a(const double *__restrict__ A, int64_t M, int64_t K,
                                                 const uint64_t *__restrict__ rowmax, int64_t KB, int64_t nchunks,
                                                 void *__restrict__ Apk) {
  constexpr bool I8 = F == 1, F8 = F == 2;
  constexpr int CK = F8 ? 64 : I8 ? 32 : 16, VL = CK / 2, RPL = kWave / CK;
  constexpr int ROWS = (I8 || F8) ? 16 : 32;  // rows staged per pass
  constexpr int LS = CK + 2;          // padded row stride (doubles) of the staged block
  __shared__ double tile[4][ROWS * LS];
  const int lane = threadIdx.x % kWave;
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
  const int64_t blk = (int64_t)blockIdx.x * 4 + w;  // (mb, kb) pair index
  const bool live = blk < nchunks;
  const int64_t mb = live ? blk / KB : 0, kb = live ? blk % KB : 0;
  double *T = tile[w];
  const int r = lane % 32, h = lane / 32;
  const int e = live ? exponent_of_max(rowmax[mb * 32 + r]) : 0;
  [[maybe_unused]] split::i8::intx4 sig8[S];
  [[maybe_unused]] bf16x8 sig16[S];
  [[maybe_unused]] split::f8::intx4 sigf[S][2];
#pragma unroll
  for (int pass = 0; pass < 32 / ROWS; ++pass) {
    if (live) {
      const int64_t col = kb * CK + lane % CK;
#pragma unroll
      for (int j = 0; j < ROWS / RPL; ++j) {
        const int rr = j * RPL + lane / CK;
        const int64_t row = mb * 32 + pass * ROWS + rr;
        T[rr * LS + lane % CK] = (row < M && col < K) ? A[row * K + col] : 0.0;
      }
    }
    __syncthreads();
    // Lanes whose row was staged in this pass take their values.
    if (live && r / ROWS == pass) {
      double v[VL];
#pragma unroll
      for (int q = 0; q < VL; ++q) v[q] = T[(r % ROWS) * LS + h * VL + q];
      if constexpr (F8)
        digits32_f8<S>(v, e, sigf);
      else if constexpr (I8)
        digits16_i8<S>(v, e, sig8);
      else
        digits8<S>(v, e, sig16);
    }
    if (pass + 1 < 32 / ROWS) __syncthreads();  // the block is refilled next pass
  }
  if (!live) return;
  if constexpr (F8) {
    split::f8::intx4 *dst = (split::f8::intx4 *)Apk + (blk * S) * 128 + lane;
#pragma unroll
    for (int s = 0; s < S; ++s) {
      dst[s * 128] = sigf[s][0];
      dst[s * 128 + 64] = sigf[s][1];
    }
  } else if constexpr (I8) {
    split::i8::intx4 *dst = (split::i8::intx4 *)Apk + (blk * S) * 64 + lane;
#pragma unroll
    for (int s = 0; s < S; ++s) dst[s * 64] = sig8[s];
  } else {
    bf16x8 *dst = (bf16x8 *)Apk + (blk * S) * 64 + lane;
#pragma unroll
    for (int s = 0; s < S; ++s) dst[s * 64] = sig16[s];
  }
}

// B slices: thread = (column block nb, k block kb, lane).
template <int S>
__global__ __launch_bounds__(256) void k_slice_b(const double *__restrict__ B, int64_t K, int64_t N,
                                                 const uint64_t *__restrict__ colmax, int64_t KB, int64_t nchunks,
                                                 bf16x8 *__restrict__ Bpk) {
  const int64_t blk = (int64_t)blockIdx.x * 4 + threadIdx.x / 64;
  if (blk >= nchunks) return;
  const int lane = threadIdx.x % 64;
  const int64_t nb = blk / KB, kb = blk % KB;
  const int64_t col = nb * 32 + lane % 32;
  const int64_t k0 = kb * 16 + (lane / 32) * 8;
  double v[8];
#pragma unroll
  for (int q = 0; q < 8; ++q) v[q] = (col < N && k0 + q < K) ? B[(k0 + q) * N + col] : 0.0;
  const int e = (col < N) ? exponent_of_max(colmax[col]) : 0;
  bf16x8 sig[S];
  digits8<S>(v, e, sig);
  bf16x8 *dst = Bpk + (blk * S) * 64 + lane;
#pragma unroll
  for (int s = 0; s < S; ++s) dst[s * 64] = sig[s];
}

// INT8 B slices: as k_slice_b with 32-k chunks of INT8 digits.
template <int S>
__global__ __launch_bounds__(256) void k_slice_b_i8(const double *__restrict__ B, int64_t K, int64_t N,
                                                    const uint64_t *__restrict__ colmax, int64_t KB, int64_t nchunks,
                                                    split::i8::intx4 *__restrict__ Bpk) {
  const int64_t blk = (int64_t)blockIdx.x * 4 + threadIdx.x / 64;
  if (blk >= nchunks) return;
  const int lane = threadIdx.x % 64;
  const int64_t nb = blk / KB, kb = blk % KB;
  const int64_t col = nb * 32 + lane % 32;
  const int64_t k0 = kb * 32 + (lane / 32) * 16;
  double v[16];
#pragma unroll
  for (int q = 0; q < 16; ++q) v[q] = (col < N && k0 + q < K) ? B[(k0 + q) * N + col] : 0.0;
  const int e = (col < N) ? exponent_of_max(colmax[col]) : 0;
  split::i8::intx4 sig[S];
  digits16_i8<S>(v, e, sig);
  split::i8::intx4 *dst = Bpk + (blk * S) * 64 + lane;
#pragma unroll
  for (int s = 0; s < S; ++s) dst[s * 64] = sig[s];
}

// FP8 B slices: as k_slice_b with 64-k chunks of FP8 digits in two halves.
template <int S>
__global__ __launch_bounds__(256) void k_slice_b_f8(const double *__restrict__ B, int64_t K, int64_t N,
                                                    const uint64_t *__restrict__ colmax, int64_t KB, int64_t nchunks,
                                                    split::f8::intx4 *__restrict__ Bpk) {
  const int64_t blk = (int64_t)blockIdx.x * 4 + threadIdx.x / 64;
  if (blk >= nchunks) return;
  const int lane = threadIdx.x % 64;
  const int64_t nb = blk / KB, kb = blk % KB;
  const int64_t col = nb * 32 + lane % 32;
  const int64_t k0 = kb * 64 + (lane / 32) * 32;
  double v[32];
#pragma unroll
  for (int q = 0; q < 32; ++q) v[q] = (col < N && k0 + q < K) ? B[(k0 + q) * N + col] : 0.0;
  const int e = (col < N) ? exponent_of_max(colmax[col]) : 0;
  split::f8::intx4 sig[S][2];
  digits32_f8<S>(v, e, sig);
  split::f8::intx4 *dst = Bpk + (blk * S) * 128 + lane;
#pragma unroll
  for (int s = 0; s < S; ++s) {
    dst[s * 128] = sig[s][0];
    dst[s * 128 + 64] = sig[s][1];
  }
}

// Scans shared by every format.
static void launch_scans(const SplitPlan &p, const double *A, const double *B, uint64_t *rowmax, uint64_t *colmax,
                         hipStream_t s) {
  hipLaunchKernelGGL(k_scan_rows, dim3((unsigned)((p.Mp + 3) / 4)), dim3(256), 0, s, A, p.M, p.K, rowmax, p.Mp);
  hipLaunchKernelGGL(k_zero_u64, dim3((unsigned)((p.Np + 255) / 256)), dim3(256), 0, s, colmax, p.Np);
  // Bands of 128 rows, or wider where K would need more than 65535 of them
  // (the grid's y extent).
  int64_t band = 128;
  while ((p.K + band - 1) / band > 65535) band *= 2;
  dim3 gcols((unsigned)((p.N + 255) / 256), (unsigned)((p.K + band - 1) / band));
  if (p.N > 0 && p.K > 0) hipLaunchKernelGGL(k_scan_cols, gcols, dim3(256), 0, s, B, p.K, p.N, band, colmax);
}

template <int S>
hipError_t launch_prepare_i8(const SplitPlan &p, const double *A, const double *B, void *ws, hipStream_t s) {
  char *w = (char *)ws;
  uint64_t *rowmax = (uint64_t *)(w + p.off_ea);
  uint64_t *colmax = (uint64_t *)(w + p.off_fb);
  auto *Apk = (split::i8::intx4 *)(w + p.off_ap);
  auto *Bpk = (split::i8::intx4 *)(w + p.off_bp);
  const int64_t KB = p.Kp / 32;
  launch_scans(p, A, B, rowmax, colmax, s);
  const int64_t cha = (p.Mp / 32) * KB, chb = (p.Np / 32) * KB;
  hipLaunchKernelGGL((k_slice_a<S, 1>), dim3((unsigned)((cha + 3) / 4)), dim3(256), 0, s, A, p.M, p.K, rowmax,
                     KB, cha, Apk);
  hipLaunchKernelGGL((k_slice_b_i8<S>), dim3((unsigned)((chb + 3) / 4)), dim3(256), 0, s, B, p.K, p.N, colmax, KB,
                     chb, Bpk);
  return hipGetLastError();
}

template <int S>
hipError_t launch_multiply_i8(const SplitPlan &p, double *D, void *ws, hipStream_t s) {
  char *w = (char *)ws;
  const uint64_t *rowmax = (const uint64_t *)(w + p.off_ea);
  const uint64_t *colmax = (const uint64_t *)(w + p.off_fb);
  const auto *Apk = (const split::i8::intx4 *)(w + p.off_ap);
  const auto *Bpk = (const split::i8::intx4 *)(w + p.off_bp);
  const int64_t KB = p.Kp / 32;
  using C = split::i8::Cfg<S, 2, 4>;
  const int64_t tmn = p.Mp / C::BM, tnn = p.Np / C::BN;
  // Pipelined loop while a chunk stream's slice bytes stay below 2^31.
  if (KB * S * 64 * 16 < ((int64_t)1 << 31))
    hipLaunchKernelGGL((split::i8::k_split_gemm_i8<S, 2, 4, true>), dim3((unsigned)(tmn * tnn)), dim3(C::kThreads), 0,
                       s, Apk, Bpk, rowmax, colmax, D, p.M, p.N, KB, tmn, tnn);
  else
    hipLaunchKernelGGL((split::i8::k_split_gemm_i8<S, 2, 4, false>), dim3((unsigned)(tmn * tnn)), dim3(C::kThreads), 0,
                       s, Apk, Bpk, rowmax, colmax, D, p.M, p.N, KB, tmn, tnn);
  return hipGetLastError();
}

template <int S>
hipError_t launch_prepare_f8(const SplitPlan &p, const double *A, const double *B, void *ws, hipStream_t s) {
  char *w = (char *)ws;
  uint64_t *rowmax = (uint64_t *)(w + p.off_ea);
  uint64_t *colmax = (uint64_t *)(w + p.off_fb);
  auto *Apk = (split::f8::intx4 *)(w + p.off_ap);
  auto *Bpk = (split::f8::intx4 *)(w + p.off_bp);
  const int64_t KB = p.Kp / 64;
  launch_scans(p, A, B, rowmax, colmax, s);
  const int64_t cha = (p.Mp / 32) * KB, chb = (p.Np / 32) * KB;
  hipLaunchKernelGGL((k_slice_a<S, 2>), dim3((unsigned)((cha + 3) / 4)), dim3(256), 0, s, A, p.M, p.K, rowmax, KB,
                     cha, Apk);
  hipLaunchKernelGGL((k_slice_b_f8<S>), dim3((unsigned)((chb + 3) / 4)), dim3(256), 0, s, B, p.K, p.N, colmax, KB,
                     chb, Bpk);
  return hipGetLastError();
}

template <int S>
hipError_t launch_multiply_f8(const SplitPlan &p, double *D, void *ws, hipStream_t s) {
  char *w = (char *)ws;
  const uint64_t *rowmax = (const uint64_t *)(w + p.off_ea);
  const uint64_t *colmax = (const uint64_t *)(w + p.off_fb);
  const auto *Apk = (const split::f8::intx4 *)(w + p.off_ap);
  const auto *Bpk = (const split::f8::intx4 *)(w + p.off_bp);
  const int64_t KB = p.Kp / 64;
  using C = split::f8::Cfg<S, 2, 2>;
  const int64_t tmn = p.Mp / C::BM, tnn = p.Np / C::BN;
  // The pipelined kernel, one launch per slab of 4096 k, while a tile's slice
  // bytes stay below 2^31 (its buffer descriptors' reach).
  if (C::MBW * KB * S * 2048 < ((int64_t)1 << 31) && C::NBW * KB * S * 2048 < ((int64_t)1 << 31)) {
    for (int64_t lo = 0; lo < KB; lo += split::f8::kFoldStages) {
      const int64_t hi = KB - lo < split::f8::kFoldStages ? KB : lo + split::f8::kFoldStages;
      hipLaunchKernelGGL((split::f8::k_split_gemm_f8_slab<S, 2, 2>), dim3((unsigned)(tmn * tnn)), dim3(C::kThreads),
                         0, s, Apk, Bpk, rowmax, colmax, D, p.M, p.N, KB, tmn, tnn, lo, hi);
    }
    return hipGetLastError();
  }
  hipLaunchKernelGGL((split::f8::k_split_gemm_f8<S, 2, 2>), dim3((unsigned)(tmn * tnn)), dim3(C::kThreads), 0, s,
                     Apk, Bpk, rowmax, colmax, D, p.M, p.N, KB, tmn, tnn);
  return hipGetLastError();
}

template <int S>
hipError_t launch_prepare_s(const SplitPlan &p, const double *A, const double *B, void *ws, hipStream_t s) {
  char *w = (char *)ws;
  uint64_t *rowmax = (uint64_t *)(w + p.off_ea);
  uint64_t *colmax = (uint64_t *)(w + p.off_fb);
  bf16x8 *Apk = (bf16x8 *)(w + p.off_ap);
  bf16x8 *Bpk = (bf16x8 *)(w + p.off_bp);
  const int64_t KB = p.Kp / 16;
  launch_scans(p, A, B, rowmax, colmax, s);
  const int64_t cha = (p.Mp / 32) * KB, chb = (p.Np / 32) * KB;
  hipLaunchKernelGGL((k_slice_a<S, 0>), dim3((unsigned)((cha + 3) / 4)), dim3(256), 0, s, A, p.M, p.K, rowmax, KB,
                     cha, Apk);
  hipLaunchKernelGGL((k_slice_b<S>), dim3((unsigned)((chb + 3) / 4)), dim3(256), 0, s, B, p.K, p.N, colmax, KB, chb,
                     Bpk);
  return hipGetLastError();
}

template <int S>
hipError_t launch_multiply_s(const SplitPlan &p, double *D, void *ws, hipStream_t s) {
  char *w = (char *)ws;
  const uint64_t *rowmax = (const uint64_t *)(w + p.off_ea);
  const uint64_t *colmax = (const uint64_t *)(w + p.off_fb);
  const bf16x8 *Apk = (const bf16x8 *)(w + p.off_ap);
  const bf16x8 *Bpk = (const bf16x8 *)(w + p.off_bp);
  const int64_t KB = p.Kp / 16;
  using L = Layout<S>;
  const int64_t tmn = p.Mp / L::C::BM, tnn = p.Np / L::C::BN;
  if (L::PIPE && KB * S * 64 * (int64_t)sizeof(bf16x8) < ((int64_t)1 << 31))
    hipLaunchKernelGGL((split::k_split_gemm<S, L::WMW, L::WNW, L::WN, L::SKB, L::NBUF, 1, L::PIPE>),
                       dim3((unsigned)(tmn * tnn)), dim3(L::C::kThreads), 0, s, Apk, Bpk, rowmax, colmax, D, p.M, p.N,
                       KB, tmn, tnn);
  else
    hipLaunchKernelGGL((split::k_split_gemm<S, L::WMW, L::WNW, L::WN, L::SKB, L::NBUF, 1, false>),
                       dim3((unsigned)(tmn * tnn)), dim3(L::C::kThreads), 0, s, Apk, Bpk, rowmax, colmax, D, p.M, p.N,
                       KB, tmn, tnn);
  return hipGetLastError();
}

}  // namespace

static int64_t round_up(int64_t x, int64_t m) { return (x + m - 1) / m * m; }
static size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

int split_max_slices(int fmt) {
  return fmt == MOA_SPLIT_FP8 ? 10 : (fmt == MOA_SPLIT_BF16 || fmt == MOA_SPLIT_INT8) ? 7 : 0;
}

bool split_plan(int64_t M, int64_t K, int64_t N, int fmt, int S, SplitPlan *p) {
  if (S < 1 || S > split_max_slices(fmt)) return false;
  p->M = M;
  p->K = K;
  p->N = N;
  p->fmt = fmt;
  p->S = S;
  int bm, bn, bytes;
  if (fmt == MOA_SPLIT_BF16) {
    p->beta = kBeta;
    tile_of(S, &bm, &bn);
    p->Kp = round_up(K > 0 ? K : 1, kFlushK);
    bytes = 2;
  } else if (fmt == MOA_SPLIT_INT8) {
    p->beta = split::i8::kBeta;
    bm = split::i8::Cfg<1, 2, 4>::BM;
    bn = split::i8::Cfg<1, 2, 4>::BN;
    p->Kp = round_up(K > 0 ? K : 1, 32);
    bytes = 1;
  } else {
    p->beta = split::f8::kBeta;
    bm = split::f8::Cfg<1, 2, 2>::BM;
    bn = split::f8::Cfg<1, 2, 2>::BN;
    p->Kp = round_up(K > 0 ? K : 1, 64);
    bytes = 1;
  }
  p->Mp = round_up(M > 0 ? M : 1, bm);
  p->Np = round_up(N > 0 ? N : 1, bn);
  size_t off = 0;
  p->off_ea = off;
  off = align256(off + sizeof(uint64_t) * (size_t)p->Mp);
  p->off_fb = off;
  off = align256(off + sizeof(uint64_t) * (size_t)p->Np);
  p->off_ap = off;
  off = align256(off + (size_t)bytes * (size_t)S * (size_t)p->Mp * (size_t)p->Kp);
  p->off_bp = off;
  off = align256(off + (size_t)bytes * (size_t)S * (size_t)p->Np * (size_t)p->Kp);
  p->total = off;
  return true;
}

hipError_t launch_split_prepare(const SplitPlan &p, const double *A, const double *B, void *ws, hipStream_t s) {
  if (p.fmt == MOA_SPLIT_FP8) {
    switch (p.S) {
      case 1: return launch_prepare_f8<1>(p, A, B, ws, s);
      case 2: return launch_prepare_f8<2>(p, A, B, ws, s);
      case 3: return launch_prepare_f8<3>(p, A, B, ws, s);
      case 4: return launch_prepare_f8<4>(p, A, B, ws, s);
      case 5: return launch_prepare_f8<5>(p, A, B, ws, s);
      case 6: return launch_prepare_f8<6>(p, A, B, ws, s);
      case 7: return launch_prepare_f8<7>(p, A, B, ws, s);
      case 8: return launch_prepare_f8<8>(p, A, B, ws, s);
      case 9: return launch_prepare_f8<9>(p, A, B, ws, s);
      case 10: return launch_prepare_f8<10>(p, A, B, ws, s);
    }
    return hipErrorInvalidValue;
  }
  if (p.fmt == MOA_SPLIT_INT8) {
    switch (p.S) {
      case 1: return launch_prepare_i8<1>(p, A, B, ws, s);
      case 2: return launch_prepare_i8<2>(p, A, B, ws, s);
      case 3: return launch_prepare_i8<3>(p, A, B, ws, s);
      case 4: return launch_prepare_i8<4>(p, A, B, ws, s);
      case 5: return launch_prepare_i8<5>(p, A, B, ws, s);
      case 6: return launch_prepare_i8<6>(p, A, B, ws, s);
      case 7: return launch_prepare_i8<7>(p, A, B, ws, s);
    }
    return hipErrorInvalidValue;
  }
  switch (p.S) {
    case 1: return launch_prepare_s<1>(p, A, B, ws, s);
    case 2: return launch_prepare_s<2>(p, A, B, ws, s);
    case 3: return launch_prepare_s<3>(p, A, B, ws, s);
    case 4: return launch_prepare_s<4>(p, A, B, ws, s);
    case 5: return launch_prepare_s<5>(p, A, B, ws, s);
    case 6: return launch_prepare_s<6>(p, A, B, ws, s);
    case 7: return launch_prepare_s<7>(p, A, B, ws, s);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_split_multiply(const SplitPlan &p, double *D, void *ws, hipStream_t s) {
  if (p.fmt == MOA_SPLIT_FP8) {
    switch (p.S) {
      case 1: return launch_multiply_f8<1>(p, D, ws, s);
      case 2: return launch_multiply_f8<2>(p, D, ws, s);
      case 3: return launch_multiply_f8<3>(p, D, ws, s);
      case 4: return launch_multiply_f8<4>(p, D, ws, s);
      case 5: return launch_multiply_f8<5>(p, D, ws, s);
      case 6: return launch_multiply_f8<6>(p, D, ws, s);
      case 7: return launch_multiply_f8<7>(p, D, ws, s);
      case 8: return launch_multiply_f8<8>(p, D, ws, s);
      case 9: return launch_multiply_f8<9>(p, D, ws, s);
      case 10: return launch_multiply_f8<10>(p, D, ws, s);
    }
    return hipErrorInvalidValue;
  }
  if (p.fmt == MOA_SPLIT_INT8) {
    switch (p.S) {
      case 1: return launch_multiply_i8<1>(p, D, ws, s);
      case 2: return launch_multiply_i8<2>(p, D, ws, s);
      case 3: return launch_multiply_i8<3>(p, D, ws, s);
      case 4: return launch_multiply_i8<4>(p, D, ws, s);
      case 5: return launch_multiply_i8<5>(p, D, ws, s);
      case 6: return launch_multiply_i8<6>(p, D, ws, s);
      case 7: return launch_multiply_i8<7>(p, D, ws, s);
    }
    return hipErrorInvalidValue;
  }
  switch (p.S) {
    case 1: return launch_multiply_s<1>(p, D, ws, s);
    case 2: return launch_multiply_s<2>(p, D, ws, s);
    case 3: return launch_multiply_s<3>(p, D, ws, s);
    case 4: return launch_multiply_s<4>(p, D, ws, s);
    case 5: return launch_multiply_s<5>(p, D, ws, s);
    case 6: return launch_multiply_s<6>(p, D, ws, s);
    case 7: return launch_multiply_s<7>(p, D, ws, s);
  }
  return hipErrorInvalidValue;
}

}  // namespace moa
