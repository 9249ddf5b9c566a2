// Fused slice-pair product of the split (Ozaki) FP64 inner product.
//
// Inputs are the fragment-packed BF16 slices of A and B written by the slicing
// kernels (see k_split.hip): chunk = 64 lanes x 8 BF16 = one 32x16 (A) or
// 16x32 (B) operand of v_mfma_f32_32x32x16_bf16, chunks ordered
// [row block][k block (16)][slice].
//
// Workgroup = WMW x WNW waves; a wave owns a 32 x (32*WN) block of D. Per
// level d = s + t of the kept slice pairs (s + t < S) a wave keeps one FP32
// accumulator per 32x32 block. Digits are at most 2^8 in magnitude, so each
// product is at most 2^16 and a level with (d+1) pairs stays exactly
// representable in FP32 for 256/(d+1) k values. Each level is folded into the
// FP64 accumulator (times its weight 2^-9d, exact) at its own period:
//     level 0: every 256 k   (exact)
//     level 1: every 128 k   (exact)
//     level 2: every  64 k   (exact)
//     level 3: every 256 k   (FP32 rounding possible only beyond 2^24, at a
//                             weight of 2^-43: far below FP64 rounding of the
//                             result)
//     level >= 4: at the end (weight <= 2^-52)
// The fold points repeat every 256 k (16 k blocks), so one cycle is unrolled
// and every fold point, and every period start (whose first MFMA takes C = 0
// instead of a zeroed accumulator), is known at compile time. A shorter tail
// (K not a multiple of 256) folds levels 0..3 every 64 k.
//
// A and B chunks are copied global -> LDS with global_load_lds_dwordx4 (no
// staging registers). An LDS stage holds kSKB 16-wide k blocks of the tile's
// slices; kNBuf stages rotate, so copies run kNBuf - 1 stages ahead of the
// MFMAs and one barrier per stage suffices: the buffer refilled at stage st
// was last read at stage st - 1, which every wave has left once it passes the
// barrier of stage st. Each wave reads its fragments as conflict-free
// ds_read_b128. Two stages of two k blocks measured slightly faster than four
// of one (half the barriers, twice the MFMAs between them).
#pragma once

#include <utility>

#include "common.hpp"

namespace moa {
namespace split {

constexpr int kBeta = 9;    // BF16 digit width: |digit| <= 2^(beta-1) = 256
constexpr int kSKB = 2;       // 16-wide k blocks per LDS stage
constexpr int kNBuf = 2;      // LDS stages in rotation
constexpr int kCycleKB = 16;  // unrolled cycle: 256 k
constexpr int kCycleSt = kCycleKB / kSKB;
static_assert(kCycleKB % kSKB == 0 && 4 % kSKB == 0, "a 64-k tail step must be whole stages");

// s_waitcnt immediate: wait until at most n vector-memory operations of this
// wave are outstanding (vmcnt split over bits 3:0 and 15:14; lgkm/exp: no wait).
__host__ __device__ constexpr int vmcnt_imm(int n) { return 0x0F70 | (n & 15) | ((n >> 4) << 14); }

// Fold period of level d in k blocks (0 = only at the end).
__host__ __device__ constexpr int period_kb(int d) {
  return d == 0 ? 16 : d == 1 ? 8 : d == 2 ? 4 : d == 3 ? 16 : 0;
}

template <int S, int WMW, int WNW, int WN>
struct Cfg {
  static constexpr int kWaves = WMW * WNW;
  static constexpr int kThreads = 64 * kWaves;
  static constexpr int BM = 32 * WMW;
  static constexpr int BN = 32 * WN * WNW;
  static constexpr int MBW = BM / 32, NBW = BN / 32;
  static constexpr int A_CH = MBW * kSKB * S;
  static constexpr int B_CH = NBW * kSKB * S;
  static constexpr int ST_CH = A_CH + B_CH;
  static constexpr int PER_WAVE = ST_CH / kWaves;                  // copies per stage, later waves
  static constexpr int MAX_WAVE = (ST_CH + kWaves - 1) / kWaves;  // copies per stage, first waves
  static constexpr int EXTRA = ST_CH % kWaves;                     // waves that issue MAX_WAVE
};

__device__ __forceinline__ floatx16 mfma_bf16(const bf16x8 &a, const bf16x8 &b, const floatx16 &c) {
  return __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, c, 0, 0, 0);
}

__device__ __forceinline__ int exponent_of_max(uint64_t bits) {
  // bits: IEEE pattern of a non-negative double. frexp exponent, 0 for 0.
  const double m = __longlong_as_double((long long)bits);
  if (m == 0.0) return 0;
  int e;
  (void)frexp(m, &e);
  return e;
}

template <int S, int WMW, int WNW, int WN, int MINB>
__global__ __launch_bounds__(64 * WMW * WNW, MINB) void k_split_gemm(
    const bf16x8 *__restrict__ Apk, const bf16x8 *__restrict__ Bpk, const uint64_t *__restrict__ rowmax,
    const uint64_t *__restrict__ colmax, double *__restrict__ D, int64_t M, int64_t N, int64_t KB, int64_t tiles_m,
    int64_t tiles_n) {
  using C = Cfg<S, WMW, WNW, WN>;
  __shared__ bf16x8 lds[kNBuf][C::ST_CH * 64];

  int64_t tm, tn;
  // Each XCD walks its share of the tiles 4 tile rows at a time (8192^3:
  // 14.52-14.59 ms against 14.72-14.78 ms with 8 rows, 14.89 with 2; the
  // concurrently resident tiles of an XCD then span 256 x 1024 of D).
  grouped_tile(xcd_swizzle(blockIdx.x, tiles_m * tiles_n), tiles_m, tiles_n, 4, tm, tn);
  const int tid = threadIdx.x, lane = tid % 64;
  // Wave index as a wave-uniform (scalar) value, so chunk addresses are scalar.
  const int wave = __builtin_amdgcn_readfirstlane(tid / 64);
  const int wm = wave / WNW, wn = wave % WNW;

  auto issue_stage = [&](int64_t st, int buf) {
#pragma unroll
    for (int q = 0; q < C::MAX_WAVE; ++q) {
      const int c = wave + C::kWaves * q;
      if (c >= C::ST_CH) break;
      const bf16x8 *src;
      if (c < C::A_CH) {
        const int mbl = c / (kSKB * S), rest = c % (kSKB * S);
        src = Apk + (((tm * C::MBW + mbl) * KB + st * kSKB) * S + rest) * 64;
      } else {
        const int cb = c - C::A_CH;
        const int nbl = cb / (kSKB * S), rest = cb % (kSKB * S);
        src = Bpk + (((tn * C::NBW + nbl) * KB + st * kSKB) * S + rest) * 64;
      }
      __builtin_amdgcn_global_load_lds((const void *)(src + lane),
                                       (__attribute__((address_space(3))) void *)&lds[buf][c * 64], 16, 0, 0);
    }
  };

  floatx16 acc[S][WN];
  double acc64[WN][16];
  const floatx16 zero16 = {};
#pragma unroll
  for (int j = 0; j < WN; ++j)
#pragma unroll
    for (int v = 0; v < 16; ++v) acc64[j][v] = 0.0;
#pragma unroll
  for (int d = 0; d < S; ++d)
#pragma unroll
    for (int j = 0; j < WN; ++j) acc[d][j] = zero16;

  auto fold_level = [&](int d) {
    const double w = __builtin_ldexp(1.0, -kBeta * d);
#pragma unroll
    for (int j = 0; j < WN; ++j)
#pragma unroll
      for (int v = 0; v < 16; ++v) acc64[j][v] = fma((double)acc[d][j][v], w, acc64[j][v]);
  };

  // One 16-wide k block from LDS buffer `buf`. Q = position in the 256-k
  // cycle (compile time), or -1 in the tail (no period starts or folds).
  // All fragments are read first (one LDS round trip per stage), then the
  // MFMAs run round-robin over the levels, largest level first, so
  // consecutive MFMAs mostly update different accumulators.
  auto mma_kb = [&](int buf, int kbl, auto qc) {
    constexpr int Q = decltype(qc)::value;
    bf16x8 af[S], bfr[S][WN];
#pragma unroll
    for (int s = 0; s < S; ++s) af[s] = lds[buf][((wm * kSKB + kbl) * S + s) * 64 + lane];
#pragma unroll
    for (int t = 0; t < S; ++t)
#pragma unroll
      for (int j = 0; j < WN; ++j)
        bfr[t][j] = lds[buf][C::A_CH * 64 + (((wn * WN + j) * kSKB + kbl) * S + t) * 64 + lane];
    __builtin_amdgcn_sched_barrier(0);
    // Round r issues, for each level d >= r (largest first), the pair
    // (s, t) = (r, d - r); rounds r = 0 .. S-1 cover every kept pair once.
#pragma unroll
    for (int r = 0; r < S; ++r)
#pragma unroll
      for (int d = S - 1; d >= r; --d)
#pragma unroll
        for (int j = 0; j < WN; ++j) {
          const bool start = Q >= 0 && r == 0 && period_kb(d) > 0 && Q % period_kb(d) == 0;
          acc[d][j] = mfma_bf16(af[r], bfr[d - r][j], start ? zero16 : acc[d][j]);
        }
    if constexpr (Q >= 0) {
#pragma unroll
      for (int d = 0; d < S; ++d)
        if (period_kb(d) > 0 && (Q + 1) % period_kb(d) == 0) fold_level(d);
    }
  };

  const int64_t nst = KB / kSKB;
  // Stage st: wait for its copies, barrier, refill the buffer of stage st - 1
  // with stage st + kNBuf - 1, then multiply its kSKB k blocks. I = position
  // of the stage in the 256-k cycle, or -1 in the tail.
  auto stage = [&](int64_t st, auto ic) {
    constexpr int I = decltype(ic)::value;
    const int buf = (int)(st % kNBuf);
    // Issued so far: stages up to st + kNBuf - 2. Stage st must be complete;
    // the kNBuf - 2 after it may stay in flight (all of them near the end).
    if (kNBuf > 2 && st + kNBuf - 2 < nst) {
      if (wave < C::EXTRA)
        __builtin_amdgcn_s_waitcnt(vmcnt_imm((kNBuf - 2) * C::MAX_WAVE));
      else
        __builtin_amdgcn_s_waitcnt(vmcnt_imm((kNBuf - 2) * C::PER_WAVE));
    } else {
      __builtin_amdgcn_s_waitcnt(vmcnt_imm(0));
    }
    // A plain barrier, not __syncthreads(): its fence would also wait for the
    // copies still in flight. LDS is coherent within the workgroup.
    __builtin_amdgcn_s_barrier();
    if (st + kNBuf - 1 < nst) issue_stage(st + kNBuf - 1, (int)((st + kNBuf - 1) % kNBuf));
    [&]<int... J>(std::integer_sequence<int, J...>) {
      (mma_kb(buf, J, std::integral_constant<int, I < 0 ? -1 : I * kSKB + J>{}), ...);
    }(std::make_integer_sequence<int, kSKB>{});
  };

  for (int i = 0; i < kNBuf - 1; ++i)
    if (i < nst) issue_stage(i, i);
  const int64_t ncyc = nst / kCycleSt;
  int64_t st = 0;
  for (int64_t cyc = 0; cyc < ncyc; ++cyc) {
    [&]<int... I>(std::integer_sequence<int, I...>) {
      (stage(st + I, std::integral_constant<int, I>{}), ...);
    }(std::make_integer_sequence<int, kCycleSt>{});
    st += kCycleSt;
  }
  if (st < nst) {
    // Tail: levels 0..3 restart from zero and fold every 64 k.
#pragma unroll
    for (int d = 0; d < S && d < 4; ++d)
#pragma unroll
      for (int j = 0; j < WN; ++j) acc[d][j] = zero16;
    for (; st < nst; st += 4 / kSKB) {
#pragma unroll
      for (int i = 0; i < 4 / kSKB; ++i) stage(st + i, std::integral_constant<int, -1>{});
#pragma unroll
      for (int d = 0; d < S && d < 4; ++d) {
        fold_level(d);
#pragma unroll
        for (int j = 0; j < WN; ++j) acc[d][j] = zero16;
      }
    }
  }
  // Levels that fold only at the end.
#pragma unroll
  for (int d = 4; d < S; ++d) fold_level(d);

  // Epilogue: exact power-of-two descaling, D[i, j] = 2^(e_i + f_j - 16) * acc.
  const int64_t col_base = tn * C::BN + wn * (32 * WN);
  const int64_t row_base = tm * C::BM + wm * 32;
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



// ---------------------------------------------------------------------------
// INT8 slices: signed digits of 7 bits (|digit| <= 64), so a digit product is
// at most 2^12 and v_mfma_i32_32x32x32_i8 accumulates every level exactly in
// INT32 for 8192 k (level d has d+1 <= 7 pairs: 7 * 8192 * 2^12 < 2^31). A
// level is folded into FP64 (times 2^-7d) only every 8192 k and at the end.
// Chunk = 64 lanes x 16 INT8 = one 32x32 operand (lane l: row/col l % 32,
// k = 16 * (l / 32) .. + 15); chunks ordered [row block][k block (32)][slice].
// LDS holds three 32-k stages in rotation (two in flight), one barrier per
// stage.
namespace i8 {

constexpr int kBeta = 7;
constexpr int kNBuf = 3;
constexpr int kFoldStages = 256;  // 8192 k

typedef __attribute__((__vector_size__(4 * sizeof(int)))) int intx4;
typedef __attribute__((__vector_size__(16 * sizeof(int)))) int intx16;

template <int S, int WMW, int WNW>
struct Cfg {
  static constexpr int kWaves = WMW * WNW;
  static constexpr int kThreads = 64 * kWaves;
  static constexpr int BM = 32 * WMW, BN = 32 * WNW;
  static constexpr int MBW = WMW, NBW = WNW;
  static constexpr int A_CH = MBW * S, B_CH = NBW * S, ST_CH = A_CH + B_CH;
  static constexpr int PER_WAVE = ST_CH / kWaves;
  static constexpr int MAX_WAVE = (ST_CH + kWaves - 1) / kWaves;
  static constexpr int EXTRA = ST_CH % kWaves;
};

template <int S, int WMW, int WNW>
__global__ __launch_bounds__(64 * WMW * WNW, 1) void k_split_gemm_i8(
    const intx4 *__restrict__ Apk, const intx4 *__restrict__ Bpk, const uint64_t *__restrict__ rowmax,
    const uint64_t *__restrict__ colmax, double *__restrict__ D, int64_t M, int64_t N, int64_t KB, int64_t tiles_m,
    int64_t tiles_n) {
  using C = Cfg<S, WMW, WNW>;
  __shared__ intx4 lds[kNBuf][C::ST_CH * 64];

  int64_t tm, tn;
  // 4 tile rows per group as in the BF16 kernel (12.94 ms against 13.03-13.14
  // ms with 8 rows at 8192^3).
  grouped_tile(xcd_swizzle(blockIdx.x, tiles_m * tiles_n), tiles_m, tiles_n, 4, tm, tn);
  const int tid = threadIdx.x, lane = tid % 64;
  const int wave = __builtin_amdgcn_readfirstlane(tid / 64);
  const int wm = wave / WNW, wn = wave % WNW;

  auto issue_stage = [&](int64_t st, int buf) {
#pragma unroll
    for (int q = 0; q < C::MAX_WAVE; ++q) {
      const int c = wave + C::kWaves * q;
      if (c >= C::ST_CH) break;
      const intx4 *src;
      if (c < C::A_CH) {
        const int mbl = c / S, s = c % S;
        src = Apk + (((tm * C::MBW + mbl) * KB + st) * S + s) * 64;
      } else {
        const int cb = c - C::A_CH;
        const int nbl = cb / S, t = cb % S;
        src = Bpk + (((tn * C::NBW + nbl) * KB + st) * S + t) * 64;
      }
      __builtin_amdgcn_global_load_lds((const void *)(src + lane),
                                       (__attribute__((address_space(3))) void *)&lds[buf][c * 64], 16, 0, 0);
    }
  };

  intx16 acc[S];
  double acc64[16];
  const intx16 zero16 = {};
#pragma unroll
  for (int v = 0; v < 16; ++v) acc64[v] = 0.0;
#pragma unroll
  for (int d = 0; d < S; ++d) acc[d] = zero16;

  auto fold_all = [&]() {
#pragma unroll
    for (int d = S - 1; d >= 0; --d) {
      const double w = __builtin_ldexp(1.0, -kBeta * d);
#pragma unroll
      for (int v = 0; v < 16; ++v) acc64[v] = fma((double)acc[d][v], w, acc64[v]);
      acc[d] = zero16;
    }
  };

  const int64_t nst = KB;
  issue_stage(0, 0);
  if (1 < nst) issue_stage(1, 1);
  for (int64_t st = 0; st < nst; ++st) {
    const int buf = (int)(st % kNBuf);
    // The copies of stage st + 1 may stay in flight.
    if (st + 1 < nst) {
      if (wave < C::EXTRA)
        __builtin_amdgcn_s_waitcnt(0x0F70 | C::MAX_WAVE);
      else
        __builtin_amdgcn_s_waitcnt(0x0F70 | C::PER_WAVE);
    } else {
      __builtin_amdgcn_s_waitcnt(0x0F70);
    }
    // Plain barrier (no fence): this stage is visible, and the buffer of
    // stage st - 1 is free for stage st + 2.
    __builtin_amdgcn_s_barrier();
    if (st + 2 < nst) issue_stage(st + 2, (int)((st + 2) % kNBuf));
    intx4 af[S], bfr[S];
#pragma unroll
    for (int s = 0; s < S; ++s) af[s] = lds[buf][(wm * S + s) * 64 + lane];
#pragma unroll
    for (int t = 0; t < S; ++t) bfr[t] = lds[buf][C::A_CH * 64 + (wn * S + t) * 64 + lane];
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int r = 0; r < S; ++r)
#pragma unroll
      for (int d = S - 1; d >= r; --d) acc[d] = __builtin_amdgcn_mfma_i32_32x32x32_i8(af[r], bfr[d - r], acc[d], 0, 0, 0);
    if ((st + 1) % kFoldStages == 0) fold_all();
  }
  if (nst % kFoldStages != 0) fold_all();

  // D[i, j] = 2^(e_i + f_j - 2(beta-1)) * acc.
  const int64_t gn = tn * C::BN + wn * 32 + lane % 32;
  const int fe = (gn < N) ? exponent_of_max(colmax[gn]) : 0;
#pragma unroll
  for (int v = 0; v < 16; ++v) {
    const int64_t gm = tm * C::BM + wm * 32 + (v / 4) * 8 + (lane / 32) * 4 + (v % 4);
    if (gm < M && gn < N) {
      const int ee = exponent_of_max(rowmax[gm]);
      D[gm * N + gn] = ldexp(acc64[v], ee + fe - 2 * (kBeta - 1));
    }
  }
}

}  // namespace i8

}  // namespace split
}  // namespace moa
