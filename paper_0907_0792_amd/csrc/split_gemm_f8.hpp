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

// Pipelined FP8 kernel over one slab of stages [st_lo, st_hi), at most
// kFoldStages of them (4096 k): the host launches it once per slab, and each
// launch folds its level accumulators into D once, at the end. A stage's A and
// B fragments all sit in registers (S of each); the barrier of stage st + 1
// comes after round 0 of stage st, and each fragment register is refilled
// with the next stage's right after its last MFMA (B fragment t: first MFMA
// of round S - 1 - t; A fragment r: last MFMA of round r), so LDS reads run
// under the matrix-core work. The copies are buffer loads into LDS, one
// descriptor per operand tile with the chunk's offset in the scalar offset
// (with global_load_lds in flight the compiler cannot order LDS reads and
// waits for all of them at every use). One fold per launch keeps the level
// accumulators in the accumulation registers; a fold inside this loop, with
// both operand sets live, made the compiler spill.
// Slab 0 writes D, later slabs add to it in the same order as the other
// kernel's folds, and the last slab applies the exact power-of-two descale.
template <int S, int WMW, int WNW>
__global__ __launch_bounds__(64 * WMW * WNW, 1) void k_split_gemm_f8_slab(
    const intx4 *__restrict__ Apk, const intx4 *__restrict__ Bpk, const uint64_t *__restrict__ rowmax,
    const uint64_t *__restrict__ colmax, double *__restrict__ D, int64_t M, int64_t N, int64_t KB, int64_t tiles_m,
    int64_t tiles_n, int64_t st_lo, int64_t st_hi) {
  using C = Cfg<S, WMW, WNW>;
  __shared__ intx4 lds[kNBuf][C::ST_CH * 128];

  int64_t tm, tn;
  grouped_tile(xcd_swizzle(blockIdx.x, tiles_m * tiles_n), tiles_m, tiles_n, 4, tm, tn);
  const int tid = threadIdx.x, lane = tid % 64;
  const int wave = __builtin_amdgcn_readfirstlane(tid / 64);
  __builtin_assume(wave >= 0 && wave < C::kWaves);
  const int wm = wave / WNW, wn = wave % WNW;

  const intx4 *abase = uniform_ptr(Apk + tm * C::MBW * KB * S * 128);
  const intx4 *bbase = uniform_ptr(Bpk + tn * C::NBW * KB * S * 128);
  const int a_bytes = (int)(C::MBW * KB * S * 2048), b_bytes = (int)(C::NBW * KB * S * 2048);
  // Copies of a stage: A copy q is half (q % 2) of A chunk q / 2, likewise
  // for B; every wave issues the same number of each.
  static_assert((2 * C::A_CH) % C::kWaves == 0 && (2 * C::B_CH) % C::kWaves == 0, "uneven copies");
  // voff: the lanes' offset, or one past every buffer (the loads then return
  // zeros and touch no memory), which lets a copy be skipped without a branch.
  constexpr int NA = 2 * C::A_CH / C::kWaves, NB = 2 * C::B_CH / C::kWaves;  // copies per wave
  auto copy_a = [&](int64_t st, int buf, int voff, int qq) {
    const int q = wave + C::kWaves * qq, c = q / 2, half = q % 2;
    copy16_to_lds(abase, a_bytes, &lds[buf][c * 128 + half * 64], voff,
                  (int)(((c / S) * KB * S + c % S + st * S) * 2048 + half * 1024));
  };
  auto copy_b = [&](int64_t st, int buf, int voff, int qq) {
    const int q = wave + C::kWaves * qq, c = q / 2, half = q % 2;
    copy16_to_lds(bbase, b_bytes, &lds[buf][(C::A_CH + c) * 128 + half * 64], voff,
                  (int)(((c / S) * KB * S + c % S + st * S) * 2048 + half * 1024));
  };
  auto issue_a = [&](int64_t st, int buf, int voff) {
#pragma unroll
    for (int qq = 0; qq < NA; ++qq) copy_a(st, buf, voff, qq);
  };
  auto issue_b = [&](int64_t st, int buf, int voff) {
#pragma unroll
    for (int qq = 0; qq < NB; ++qq) copy_b(st, buf, voff, qq);
  };
  constexpr int kNoCopy = (int)0x80000000u;
  // Stage x becomes readable: its copies are done and, after this wave's
  // LDS reads have drained, every wave has left the buffer that takes stage
  // x + 1 next (the stage before x, whose fragments are all in registers).
  // With one wave per SIMD nothing covers a burst of copies, so from three
  // slices on the copies of stage x + 1 are spread over the MFMAs of rounds
  // 1 (A) and 2 (B) of stage x - 1, one or two after each; with fewer, here.
  auto open_stage = [&](int64_t x) {
    __builtin_amdgcn_s_waitcnt(vmcnt_lgkm0_imm(0));
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_sched_barrier(0);
    if constexpr (S < 3)
      if (x + 1 < st_hi) {
        issue_a(x + 1, (int)((x + 1) % kNBuf), lane * 16);
        issue_b(x + 1, (int)((x + 1) % kNBuf), lane * 16);
      }
  };
  auto frag = [&](int buf, int c) {
    const intx4 lo = lds[buf][c * 128 + lane], hi = lds[buf][c * 128 + 64 + lane];
    return intx8{lo[0], lo[1], lo[2], lo[3], hi[0], hi[1], hi[2], hi[3]};
  };

  floatx16 acc[S];
  const floatx16 zero16 = {};
#pragma unroll
  for (int d = 0; d < S; ++d) acc[d] = zero16;
  asm volatile("" ::"s"(rowmax), "s"(colmax), "s"(D));
  intx8 af[S], bfr[S];
  issue_a(st_lo, (int)(st_lo % kNBuf), lane * 16);
  issue_b(st_lo, (int)(st_lo % kNBuf), lane * 16);
  open_stage(st_lo);
  if constexpr (S >= 3)
    if (st_lo + 1 < st_hi) {
      issue_a(st_lo + 1, (int)((st_lo + 1) % kNBuf), lane * 16);
      issue_b(st_lo + 1, (int)((st_lo + 1) % kNBuf), lane * 16);
    }
  {
    const int buf = (int)(st_lo % kNBuf);
#pragma unroll
    for (int r = 0; r < S; ++r) {
      bfr[S - 1 - r] = frag(buf, C::A_CH + wn * S + S - 1 - r);
      af[r] = frag(buf, wm * S + r);
    }
  }
  __builtin_amdgcn_sched_barrier(0);
  // The last stage runs the same body: it opens stage st_hi, which has no
  // copies (a barrier only), and refills the registers with LDS contents
  // nothing uses.
  for (int64_t st = st_lo; st < st_hi; ++st) {
    const int nbuf = (int)((st + 1) % kNBuf);
#pragma unroll
    for (int d = S - 1; d >= 0; --d) acc[d] = mfma_f8(af[0], bfr[d], acc[d]);
    __builtin_amdgcn_sched_barrier(0);
    open_stage(st + 1);
    bfr[S - 1] = frag(nbuf, C::A_CH + wn * S + S - 1);
    af[0] = frag(nbuf, wm * S);
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int r = 1; r < S; ++r) {
#pragma unroll
      for (int d = S - 1; d >= r; --d) {
        acc[d] = mfma_f8(af[r], bfr[d - r], acc[d]);
        __builtin_amdgcn_sched_barrier(0);
        if (d == S - 1) bfr[S - 1 - r] = frag(nbuf, C::A_CH + wn * S + S - 1 - r);
        // Stage st + 2 goes to the buffer of stage st, whose fragments every
        // wave has read (open_stage(st + 1) above). Copy qq follows MFMA
        // qq * len / n of its round. Past the slab's end the copies are
        // issued as no-ops, so no branch here lets the compiler move them.
        if constexpr (S >= 3) {
          if (r == 1 || r == 2) {
            const int voff = st + 2 < st_hi ? lane * 16 : kNoCopy;
            const int len = S - r, i = S - 1 - d;
#pragma unroll
            for (int qq = 0; qq < (r == 1 ? NA : NB); ++qq)
              if (qq * len / (r == 1 ? NA : NB) == i) {
                if (r == 1)
                  copy_a(st + 2, (int)(st % kNBuf), voff, qq);
                else
                  copy_b(st + 2, (int)(st % kNBuf), voff, qq);
              }
          }
        }
        __builtin_amdgcn_sched_barrier(0);
      }
      af[r] = frag(nbuf, wm * S + r);
      __builtin_amdgcn_sched_barrier(0);
    }
  }

  // The last stage issued no-op copies after its final wait: drain them so
  // that no copy into LDS is outstanding when the workgroup ends.
  __builtin_amdgcn_s_waitcnt(vmcnt_imm(0));

  // Fold into D: D[i, j] (+)= sum_d 2^-5d level_d, then on the last slab
  // D[i, j] = 2^(e_i + f_j - 2(beta-1)) * D[i, j].
  const bool first = st_lo == 0, last = st_hi == KB;
  const int64_t gn = tn * C::BN + wn * 32 + lane % 32;
  const int64_t row_base = tm * C::BM + wm * 32;
  const int fe = (last && gn < N) ? exponent_of_max(colmax[gn]) : 0;
  const int e_lane = (last && row_base + lane % 32 < M) ? exponent_of_max(rowmax[row_base + lane % 32]) : 0;
#pragma unroll
  for (int v = 0; v < 16; ++v) {
    const int r = (v / 4) * 8 + (lane / 32) * 4 + (v % 4);
    const int ee = __shfl(e_lane, r);
    const int64_t gm = row_base + r;
    if (gm < M && gn < N) {
      double t = first ? 0.0 : D[gm * N + gn];
#pragma unroll
      for (int d = S - 1; d >= 0; --d) t = fma((double)acc[d][v], __builtin_ldexp(1.0, -kBeta * d), t);
      D[gm * N + gn] = last ? ldexp(t, ee + fe - 2 * (kBeta - 1)) : t;
    }
  }
}

}  // namespace f8

}  // namespace split
}  // namespace moa
