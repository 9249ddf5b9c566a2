#pragma once
// FP8 (E4M3) slice-pair kernel of the split product (the BF16 and INT8
// kernels are in split_gemm.hpp, whose helpers this one uses).

#include "split_gemm.hpp"

namespace moa {
namespace split {

// ---------------------------------------------------------------------------
// FP8 (E4M3) slices: signed digits of 5 bits (|digit| <= 16, exact in E4M3),
// so a digit product is at most 2^8 and a level with d + 1 pairs stays exact
// in FP32 for 2^16 / (d + 1) k values: with up to 10 slices the levels fold
// into FP64 (times 2^-5d) every 4096 k and at the end. MFMA:
// v_mfma_scale_f32_32x32x64_f8f6f4 with both formats E4M3 and unit scales.
// Chunk = 64 lanes x 32 FP8 = one 32x64 operand (lane l: row/col l % 32,
// k = 32 (l / 32) .. + 31; A and B use the same lane-to-k assignment, which is
// all an exact sum needs), stored as two 1-KiB halves, chunks ordered
// [row block][k block (64)][slice]. Workgroup = 2 x 2 waves of 32 x 32
// (64 x 64 tile), one wave per SIMD (the S level accumulators, the FP64 sums
// and S A fragments of 8 registers each need the whole register file). Two
// 64-k LDS stages in rotation, one barrier per stage; B fragments are read
// one slice at a time.
namespace f8 {

constexpr int kBeta = 5;
constexpr int kNBuf = 2;
constexpr int kFoldStages = 64;  // 4096 k

typedef __attribute__((__vector_size__(4 * sizeof(int)))) int intx4;
typedef __attribute__((__vector_size__(8 * sizeof(int)))) int intx8;

template <int S, int WMW, int WNW>
struct Cfg {
  static constexpr int kWaves = WMW * WNW;
  static constexpr int kThreads = 64 * kWaves;
  static constexpr int BM = 32 * WMW, BN = 32 * WNW;
  static constexpr int MBW = WMW, NBW = WNW;
  static constexpr int A_CH = MBW * S, B_CH = NBW * S, ST_CH = A_CH + B_CH;  // 2-KiB chunks per stage
  static constexpr int COPIES = 2 * ST_CH;                                   // 1-KiB copies per stage
  static constexpr int PER_WAVE = COPIES / kWaves;
  static constexpr int MAX_WAVE = (COPIES + kWaves - 1) / kWaves;
  static constexpr int EXTRA = COPIES % kWaves;
  static_assert(sizeof(intx4) * 128 * ST_CH * kNBuf <= 160 * 1024, "LDS stages exceed 160 KiB");
};

__device__ __forceinline__ floatx16 mfma_f8(const intx8 &a, const intx8 &b, const floatx16 &c) {
  // Formats 0 / 0: A and B are E4M3; scales 127 (E8M0 for 2^0).
  return __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(a, b, c, 0, 0, 0, 127, 0, 127);
}

template <int S, int WMW, int WNW>
__global__ __launch_bounds__(64 * WMW * WNW, 1) void k_split_gemm_f8(
    const intx4 *__restrict__ Apk, const intx4 *__restrict__ Bpk, const uint64_t *__restrict__ rowmax,
    const uint64_t *__restrict__ colmax, double *__restrict__ D, int64_t M, int64_t N, int64_t KB, int64_t tiles_m,
    int64_t tiles_n) {
  using C = Cfg<S, WMW, WNW>;
  __shared__ intx4 lds[kNBuf][C::ST_CH * 128];

  int64_t tm, tn;
  grouped_tile(xcd_swizzle(blockIdx.x, tiles_m * tiles_n), tiles_m, tiles_n, 4, tm, tn);
  const int tid = threadIdx.x, lane = tid % 64;
  const int wave = __builtin_amdgcn_readfirstlane(tid / 64);
  const int wm = wave / WNW, wn = wave % WNW;

  // Copy q of a stage: half (q % 2) of chunk q / 2.
  auto issue_stage = [&](int64_t st, int buf) {
#pragma unroll
    for (int qq = 0; qq < C::MAX_WAVE; ++qq) {
      const int q = wave + C::kWaves * qq;
      if (q >= C::COPIES) break;
      const int c = q / 2, half = q % 2;
      const intx4 *src;
      if (c < C::A_CH)
        src = Apk + (((tm * C::MBW + c / S) * KB + st) * S + c % S) * 128 + half * 64;
      else
        src = Bpk + (((tn * C::NBW + (c - C::A_CH) / S) * KB + st) * S + (c - C::A_CH) % S) * 128 + half * 64;
      __builtin_amdgcn_global_load_lds((const void *)(src + lane),
                                       (__attribute__((address_space(3))) void *)&lds[buf][c * 128 + half * 64], 16,
                                       0, 0);
    }
  };

  floatx16 acc[S];
  double acc64[16];
  const floatx16 zero16 = {};
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

  auto frag = [&](int buf, int c) {
    const intx4 lo = lds[buf][c * 128 + lane], hi = lds[buf][c * 128 + 64 + lane];
    return intx8{lo[0], lo[1], lo[2], lo[3], hi[0], hi[1], hi[2], hi[3]};
  };

  const int64_t nst = KB;
  issue_stage(0, 0);
  // Blocks of kFoldStages stages with the fold after each: inside a block
  // the level accumulators feed only matrix-core instructions, so they stay
  // in the accumulation registers (a fold inside the stage loop made the
  // compiler keep them in VGPRs and copy all of them in and out per stage).
  for (int64_t st0 = 0; st0 < nst; st0 += kFoldStages) {
    const int64_t st1 = (nst - st0) < kFoldStages ? nst : st0 + kFoldStages;
    for (int64_t st = st0; st < st1; ++st) {
      const int buf = (int)(st % kNBuf);
      __builtin_amdgcn_s_waitcnt(vmcnt_imm(0));
      // Plain barrier (no fence): this stage is visible, and the buffer of
      // stage st - 1 is free for stage st + 1.
      __builtin_amdgcn_s_barrier();
      if (st + 1 < nst) issue_stage(st + 1, (int)((st + 1) % kNBuf));
      intx8 af[S];
#pragma unroll
      for (int s = 0; s < S; ++s) af[s] = frag(buf, wm * S + s);
      // B slice t pairs with A slices s < S - t (level s + t).
#pragma unroll
      for (int t = 0; t < S; ++t) {
        const intx8 bf = frag(buf, C::A_CH + wn * S + t);
#pragma unroll
        for (int s = 0; s < S - t; ++s) acc[s + t] = mfma_f8(af[s], bf, acc[s + t]);
      }
    }
    fold_all();
  }

  // D[i, j] = 2^(e_i + f_j - 2(beta-1)) * acc.
  const int64_t gn = tn * C::BN + wn * 32 + lane % 32;
  const int fe = (gn < N) ? exponent_of_max(colmax[gn]) : 0;
  const int64_t row_base = tm * C::BM + wm * 32;
  const int e_lane = (row_base + lane % 32 < M) ? exponent_of_max(rowmax[row_base + lane % 32]) : 0;
#pragma unroll
  for (int v = 0; v < 16; ++v) {
    const int r = (v / 4) * 8 + (lane / 32) * 4 + (v % 4);
    const int ee = __shfl(e_lane, r);
    const int64_t gm = row_base + r;
    if (gm < M && gn < N) D[gm * N + gn] = ldexp(acc64[v], ee + fe - 2 * (kBeta - 1));
  }
}

}  // namespace f8

}  // namespace split
}  // namespace moa
