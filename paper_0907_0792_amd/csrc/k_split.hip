// (+,*) FP64 inner product at FP64 accuracy from BF16 slices on the matrix
// cores — the split scheme of Ozaki, Ogita, Oishi & Rump (Numer. Algorithms 59,
// 2012), with signed digits. The (+,*) case of Eq. inner (Section I) on the
// flattened M x K and K x N views.
//
// Scheme. Row i of A is scaled by 2^-e_i and column j of B by 2^-f_j, where
// 2^e is the smallest power of two above the row (column) maximum, so scaled
// entries x lie in (-1, 1). Each x is written as signed base-2^9 digits
//     x = sum_s sigma_s 2^-(8 + 9 s),  |sigma_s| <= 256,
// every digit an integer that BF16 holds exactly. With S digits per operand
// the pairs (s, t), s + t < S are kept; pairs of equal level d = s + t carry
// the same weight 2^-(16 + 9 d), so they share one FP32 accumulator per level:
//     D_ij = 2^(e_i + f_j - 16) * sum_d 2^-9d T_d[i, j],
//     T_d = sum_{s+t=d} sigma^A_s . sigma^B_t   (integer-valued).
// Products of digits are at most 2^16; a level-d accumulator receives at most
// (d+1) * 64 * 2^16 <= 2^24 in magnitude over a period of 64 k values for
// d <= 3, so its FP32 sum is exact; it is then folded into an FP64
// accumulator and restarted (levels >= 4 weigh at most 2^-52 of a level-0 unit
// and their FP32 rounding is far below FP64 rounding). Within one period the
// levels 0..3 combine exactly in FP64 (they span 51 bits), so each period adds
// one rounded FP64 term per output.
//
// Data layout. Slices are written once, in the operand layout of
// v_mfma_f32_32x32x16_bf16: a "chunk" is the 32 x 16 (A) or 16 x 32 (B)
// fragment of one slice, 64 lanes x 8 BF16 = 1 KiB, lane l holding row (col)
// l % 32 and k = 8 * (l / 32) .. + 7. Chunks are ordered
// [row block][k block][slice], so the slices of consecutive k blocks of one
// row block are one contiguous run. The product kernel copies runs straight
// into LDS with global_load_lds_dwordx4 (no staging registers) and each wave
// reads a fragment back as one conflict-free ds_read_b128.
#include "common.hpp"
#include "internal.hpp"

namespace moa {

namespace {

constexpr int kBeta = 9;               // BF16 digit width (|digit| <= 2^(beta-1) = 256)
constexpr int kFlushK = 64;            // exact-accumulation period in k
// 16-wide k blocks per LDS stage (two, unless the slices would overflow LDS).
template <int S>
constexpr int stage_kb() { return S <= 6 ? 2 : 1; }
constexpr int kSplitBM = 64;           // workgroup tile rows (2 waves x 32)
constexpr int kSplitWN = 2;            // 32-wide column blocks per wave
constexpr int kSplitBN = 64 * kSplitWN;  // workgroup tile columns (2 waves)

__device__ __forceinline__ int exponent_of_max(uint64_t bits) {
  // bits: IEEE pattern of a non-negative double. frexp exponent, 0 for 0.
  const double m = __longlong_as_double((long long)bits);
  if (m == 0.0) return 0;
  int e;
  (void)frexp(m, &e);
  return e;
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
// sig[s] holds digit s of each of the 8 values, as BF16.
template <int S>
__device__ __forceinline__ void digits8(const double v[8], int e, bf16x8 sig[S]) {
#pragma unroll
  for (int q = 0; q < 8; ++q) {
    double r = ldexp(v[q], kBeta - 1 - e);  // x * 2^(beta-1), exact
#pragma unroll
    for (int s = 0; s < S; ++s) {
      const double d = rint(r);
      sig[s][q] = (__bf16)(float)d;  // |d| <= 256: exact in BF16
      r = (r - d) * (double)(1 << kBeta);
    }
  }
}

// A slices: thread = (row block mb, k block kb, lane).
template <int S>
__global__ __launch_bounds__(256) void k_slice_a(const double *__restrict__ A, int64_t M, int64_t K,
                                                 const uint64_t *__restrict__ rowmax, int64_t KB, int64_t nchunks,
                                                 bf16x8 *__restrict__ Apk) {
  const int64_t blk = (int64_t)blockIdx.x * 4 + threadIdx.x / 64;  // (mb, kb) pair index
  if (blk >= nchunks) return;
  const int lane = threadIdx.x % 64;
  const int64_t mb = blk / KB, kb = blk % KB;
  const int64_t row = mb * 32 + lane % 32;
  const int64_t k0 = kb * 16 + (lane / 32) * 8;
  double v[8];
#pragma unroll
  for (int q = 0; q < 8; ++q) v[q] = (row < M && k0 + q < K) ? A[row * K + k0 + q] : 0.0;
  const int e = exponent_of_max(rowmax[row]);
  bf16x8 sig[S];
  digits8<S>(v, e, sig);
  bf16x8 *dst = Apk + (blk * S) * 64 + lane;
#pragma unroll
  for (int s = 0; s < S; ++s) dst[s * 64] = sig[s];
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

__device__ __forceinline__ floatx16 mfma_bf16(const bf16x8 &a, const bf16x8 &b, const floatx16 &c) {
  return __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, c, 0, 0, 0);
}

// The fused slice-pair product. Workgroup = 4 waves (2 x 2) owning a
// 64 x 128 tile of D; each wave a 32 x 64 block (two 32 x 32 accumulators per
// level).
template <int S>
__global__ __launch_bounds__(256, 1) void k_split_gemm(const bf16x8 *__restrict__ Apk, const bf16x8 *__restrict__ Bpk,
                                                       const uint64_t *__restrict__ rowmax,
                                                       const uint64_t *__restrict__ colmax, double *__restrict__ D,
                                                       int64_t M, int64_t N, int64_t KB, int64_t tiles_m,
                                                       int64_t tiles_n) {
  constexpr int WN = kSplitWN;
  constexpr int kStageKB = stage_kb<S>();
  constexpr int MBW = kSplitBM / 32;      // row blocks per workgroup
  constexpr int NBW = kSplitBN / 32;      // column blocks per workgroup
  constexpr int A_CH = MBW * kStageKB * S;  // chunks of A per stage
  constexpr int B_CH = NBW * kStageKB * S;
  constexpr int ST_CH = A_CH + B_CH;
  constexpr int PER_WAVE = ST_CH / 4;           // copies every wave issues
  constexpr int MAX_WAVE = (ST_CH + 3) / 4;     // copies the first waves issue
  constexpr int STAGES_PER_FLUSH = kFlushK / (16 * kStageKB);
  __shared__ bf16x8 lds[2][ST_CH * 64];

  int64_t tm, tn;
  grouped_tile(xcd_swizzle(blockIdx.x, tiles_m * tiles_n), tiles_m, tiles_n, 4, tm, tn);
  const int tid = threadIdx.x, lane = tid % 64, wave = tid / 64;
  const int wm = wave / 2, wn = wave % 2;

  // Chunk c of a stage: A chunks first ([mb][kb][s]), then B ([nb][kb][s]).
  auto issue_stage = [&](int64_t st, int buf) {
#pragma unroll
    for (int q = 0; q < MAX_WAVE; ++q) {
      const int c = wave + 4 * q;
      if (c >= ST_CH) break;
      const bf16x8 *src;
      if (c < A_CH) {
        const int mbl = c / (kStageKB * S), rest = c % (kStageKB * S);
        src = Apk + (((tm * MBW + mbl) * KB + st * kStageKB) * S + rest) * 64;
      } else {
        const int cb = c - A_CH;
        const int nbl = cb / (kStageKB * S), rest = cb % (kStageKB * S);
        src = Bpk + (((tn * NBW + nbl) * KB + st * kStageKB) * S + rest) * 64;
      }
      __builtin_amdgcn_global_load_lds((const void *)(src + lane), (__attribute__((address_space(3))) void *)&lds[buf][c * 64], 16, 0, 0);
    }
  };

  floatx16 acc[S][WN];
  double acc64[WN][16];
#pragma unroll
  for (int j = 0; j < WN; ++j)
#pragma unroll
    for (int v = 0; v < 16; ++v) acc64[j][v] = 0.0;
#pragma unroll
  for (int d = 0; d < S; ++d)
#pragma unroll
    for (int j = 0; j < WN; ++j)
#pragma unroll
      for (int v = 0; v < 16; ++v) acc[d][j][v] = 0.0f;

  const int64_t nstages = KB / kStageKB;
  issue_stage(0, 0);
  for (int64_t st = 0; st < nstages; ++st) {
    const int buf = (int)(st & 1);
    if (st + 1 < nstages) {
      issue_stage(st + 1, buf ^ 1);
      // Wait for this stage's copies; up to PER_WAVE of the next stage stay in
      // flight (a wave that issued one more waits for one of those too).
      __builtin_amdgcn_s_waitcnt(0x0F70 | PER_WAVE);
    } else {
      __builtin_amdgcn_s_waitcnt(0x0F70);
    }
    // Plain barrier, not __syncthreads(): its fence would also wait for the
    // next stage's copies. LDS is coherent within the workgroup, and each
    // wave has already waited for its own copies of this stage above.
    __builtin_amdgcn_s_barrier();
#pragma unroll
    for (int kbl = 0; kbl < kStageKB; ++kbl) {
      bf16x8 af[S], bfr[S][WN];
#pragma unroll
      for (int s = 0; s < S; ++s) af[s] = lds[buf][((wm * kStageKB + kbl) * S + s) * 64 + lane];
#pragma unroll
      for (int t = 0; t < S; ++t)
#pragma unroll
        for (int j = 0; j < WN; ++j)
          bfr[t][j] = lds[buf][A_CH * 64 + (((wn * WN + j) * kStageKB + kbl) * S + t) * 64 + lane];
#pragma unroll
      for (int s = 0; s < S; ++s)
#pragma unroll
        for (int t = 0; t + s < S; ++t)
#pragma unroll
          for (int j = 0; j < WN; ++j) acc[s + t][j] = mfma_bf16(af[s], bfr[t][j], acc[s + t][j]);
    }
    if ((st + 1) % STAGES_PER_FLUSH == 0 || st + 1 == nstages) {
      // Fold the period into FP64: sum_d 2^-9d T_d, innermost (smallest) first.
#pragma unroll
      for (int j = 0; j < WN; ++j)
#pragma unroll
        for (int v = 0; v < 16; ++v) {
          double p = (double)acc[S - 1][j][v];
#pragma unroll
          for (int d = S - 2; d >= 0; --d) p = fma(p, 0x1p-9, (double)acc[d][j][v]);
          acc64[j][v] += p;
        }
#pragma unroll
      for (int d = 0; d < S; ++d)
#pragma unroll
        for (int j = 0; j < WN; ++j)
#pragma unroll
          for (int v = 0; v < 16; ++v) acc[d][j][v] = 0.0f;
    }
    // Every wave is done reading `buf` before the next iteration refills it.
    __builtin_amdgcn_s_waitcnt(0xC07F);  // lgkmcnt(0)
    __builtin_amdgcn_s_barrier();
  }

  // Epilogue: exact power-of-two descaling, D[i, j] = 2^(e_i + f_j - 16) * acc.
  const int64_t col_base = tn * kSplitBN + wn * (32 * WN);
  const int64_t row_base = tm * kSplitBM + wm * 32;
#pragma unroll
  for (int j = 0; j < WN; ++j) {
    const int64_t gn = col_base + j * 32 + lane % 32;
    const int fe = (gn < N) ? exponent_of_max(colmax[gn]) : 0;
#pragma unroll
    for (int v = 0; v < 16; ++v) {
      const int64_t gm = row_base + (v / 4) * 8 + (lane / 32) * 4 + (v % 4);
      if (gm < M && gn < N) {
        const int ee = exponent_of_max(rowmax[gm]);
        D[gm * N + gn] = ldexp(acc64[j][v], ee + fe - 2 * (kBeta - 1));
      }
    }
  }
}

template <int S>
hipError_t launch_prepare_s(const SplitPlan &p, const double *A, const double *B, void *ws, hipStream_t s) {
  char *w = (char *)ws;
  uint64_t *rowmax = (uint64_t *)(w + p.off_ea);
  uint64_t *colmax = (uint64_t *)(w + p.off_fb);
  bf16x8 *Apk = (bf16x8 *)(w + p.off_ap);
  bf16x8 *Bpk = (bf16x8 *)(w + p.off_bp);
  const int64_t KB = p.Kp / 16;
  hipLaunchKernelGGL(k_scan_rows, dim3((unsigned)((p.Mp + 3) / 4)), dim3(256), 0, s, A, p.M, p.K, rowmax, p.Mp);
  hipLaunchKernelGGL(k_zero_u64, dim3((unsigned)((p.Np + 255) / 256)), dim3(256), 0, s, colmax, p.Np);
  const int64_t band = 128;
  dim3 gcols((unsigned)((p.N + 255) / 256), (unsigned)((p.K + band - 1) / band));
  if (p.N > 0 && p.K > 0) hipLaunchKernelGGL(k_scan_cols, gcols, dim3(256), 0, s, B, p.K, p.N, band, colmax);
  const int64_t cha = (p.Mp / 32) * KB, chb = (p.Np / 32) * KB;
  hipLaunchKernelGGL((k_slice_a<S>), dim3((unsigned)((cha + 3) / 4)), dim3(256), 0, s, A, p.M, p.K, rowmax, KB, cha,
                     Apk);
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
  const int64_t tmn = p.Mp / kSplitBM, tnn = p.Np / kSplitBN;
  hipLaunchKernelGGL((k_split_gemm<S>), dim3((unsigned)(tmn * tnn)), dim3(256), 0, s, Apk, Bpk, rowmax, colmax, D,
                     p.M, p.N, KB, tmn, tnn);
  return hipGetLastError();
}

}  // namespace

static int64_t round_up(int64_t x, int64_t m) { return (x + m - 1) / m * m; }
static size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

bool split_plan(int64_t M, int64_t K, int64_t N, int fmt, int S, SplitPlan *p) {
  if (fmt != MOA_SPLIT_BF16 || S < 1 || S > MOA_SPLIT_MAX_SLICES) return false;
  p->M = M;
  p->K = K;
  p->N = N;
  p->fmt = fmt;
  p->S = S;
  p->beta = kBeta;
  p->Mp = round_up(M > 0 ? M : 1, kSplitBM);
  p->Np = round_up(N > 0 ? N : 1, kSplitBN);
  p->Kp = round_up(K > 0 ? K : 1, kFlushK);
  size_t off = 0;
  p->off_ea = off;
  off = align256(off + sizeof(uint64_t) * (size_t)p->Mp);
  p->off_fb = off;
  off = align256(off + sizeof(uint64_t) * (size_t)p->Np);
  p->off_ap = off;
  off = align256(off + 2 * (size_t)S * (size_t)p->Mp * (size_t)p->Kp);
  p->off_bp = off;
  off = align256(off + 2 * (size_t)S * (size_t)p->Np * (size_t)p->Kp);
  p->total = off;
  return true;
}

hipError_t launch_split_prepare(const SplitPlan &p, const double *A, const double *B, void *ws, hipStream_t s) {
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
