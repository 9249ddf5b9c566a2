// Fused slice-pair product of the split (Ozaki) FP64 inner product.
//
// Inputs are the fragment-packed BF16 slices of A and B written by the slicing
// kernels (see k_split.hip): chunk = 64 lanes x 8 BF16 = one 32x16 (A) or
// 16x32 (B) operand of v_mfma_f32_32x32x16_bf16, chunks ordered
// [row block][k block (16)][slice]. Digit s is stored times its weight
// 2^-9s (exact in BF16), so a slice-pair product carries the weight of its
// level d = s + t.
//
// Workgroup = WMW x WNW waves; a wave owns a 32 x (32*WN) block of D. A wave
// keeps one FP32 accumulator per level and 32x32 block, except that 32 x 64
// wave blocks (WN = 2) have registers for four: levels from 3 up then share
// the fourth (MERGE). Digits are at most 2^8 in magnitude, so a product is at
// most 2^16 times its weight and a level with (d+1) pairs stays exact in FP32
// for 256/(d+1) k values. Each accumulator is folded into the FP64
// accumulator at its own period:
//     level 0:    every 256 k   (exact)
//     level 1:    every 128 k   (exact)
//     level 2:    every  64 k   (exact)
//     level 3:    every 256 k   (exact while partial sums stay below 2^24;
//                                weight 2^-27)
//     levels 4+:  at the end    (weight <= 2^-36)
//     merged 3+:  every 256 k   (levels 3 and 4 on one FP32 grid: a sum
//                                rounded to 2^-24 of a level-3 sum; on the
//                                2^[-8,8]-scaled workload about 3e-14 normwise
//                                of the result, a few percent of the scheme's
//                                own truncation error at 5 slices)
// A fold adds the accumulator into FP64 and zeroes it; the last fold of each
// accumulator comes after the last k block.
//
// A and B chunks are copied global -> LDS with global_load_lds_dwordx4 (no
// staging registers). An LDS stage holds SKB 16-wide k blocks of the tile's
// slices; NBUF stages rotate, so copies run NBUF - 1 stages ahead of the
// MFMAs and one barrier per stage suffices: the buffer refilled at stage st
// was last read at stage st - 1, which every wave has left once it passes the
// barrier of stage st. Each wave reads its fragments as conflict-free
// ds_read_b128: its S A fragments once per k block, then the S B fragments
// of one 32-column block at a time (a wave with WN = 2 holds 2S, not 3S,
// fragments, which is what lets 32 x 64 wave blocks run at two waves per
// SIMD).
//
// The 32 x 64 layout runs a pipelined form of the same loop (PIPE): copies are
// buffer loads into LDS, each stage's barrier sits inside the stage before
// it, and every fragment register is refilled right after its last MFMA, so
// the fragment reads overlap the matrix-core work instead of stalling all
// waves after each barrier. On the 8192^3, 5-slice product it takes 11.85-11.90
// ms against 12.45 ms for the plain loop (same box, same run).
#pragma once

#include <utility>

#include "common.hpp"

namespace moa {
namespace split {

constexpr int kBeta = 9;  // BF16 digit width: |digit| <= 2^(beta-1) = 256

// s_waitcnt immediate: wait until at most n vector-memory operations of this
// wave are outstanding (vmcnt split over bits 3:0 and 15:14; lgkm/exp: no wait).
__host__ __device__ constexpr int vmcnt_imm(int n) { return 0x0F70 | (n & 15) | ((n >> 4) << 14); }

// Accumulator of level d: its own, or with MERGE one shared by every level
// from 3 up.
template <bool MERGE>
__host__ __device__ constexpr int acc_of(int d) {
  return (MERGE && d > 3) ? 3 : d;
}

template <int S, int WMW, int WNW, int WN, int SKB, int NBUF>
struct Cfg {
  static constexpr int kWaves = WMW * WNW;
  static constexpr int kThreads = 64 * kWaves;
  static constexpr int BM = 32 * WMW;
  static constexpr int BN = 32 * WN * WNW;
  static constexpr int MBW = BM / 32, NBW = BN / 32;
  static constexpr int A_CH = MBW * SKB * S;
  static constexpr int B_CH = NBW * SKB * S;
  static constexpr int ST_CH = A_CH + B_CH;
  static constexpr int PER_WAVE = ST_CH / kWaves;                  // copies per stage, later waves
  static constexpr int MAX_WAVE = (ST_CH + kWaves - 1) / kWaves;  // copies per stage, first waves
  static constexpr int EXTRA = ST_CH % kWaves;                     // waves that issue MAX_WAVE
  // 32 x 64 wave blocks have registers for four accumulators per 32x32
  // block: levels from 3 up share the fourth (MERGE); otherwise one each.
  static constexpr bool MERGE = WN > 1;
  static constexpr int L = (MERGE && S > 4) ? 4 : S;              // accumulators per 32x32 block
  static_assert(4 % SKB == 0, "a 64-k group must be whole stages");
  static_assert(sizeof(bf16x8) * 64 * ST_CH * NBUF <= 160 * 1024, "LDS stages exceed 160 KiB");
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

// s_waitcnt immediate: at most n vector-memory operations outstanding and no
// LDS/scalar operation outstanding.
__host__ __device__ constexpr int vmcnt_lgkm0_imm(int n) { return 0x0070 | (n & 15) | ((n >> 4) << 14); }

// A wave-uniform pointer as a scalar value. readfirstlane returns a signed
// int: each half goes through uint32_t before widening, or a low half with
// bit 31 set would sign-extend over the high half.
template <typename T>
__device__ __forceinline__ const T *uniform_ptr(const T *p) {
  const uint64_t u = (uint64_t)p;
  const uint64_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)(u >> 32));
  const uint64_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)u);
  return (const T *)((hi << 32) | lo);
}

// 16 bytes per lane from base + voff + soff into LDS at dst + 16 * lane, by
// a buffer load whose descriptor covers nbytes from base.
__device__ __forceinline__ void copy16_to_lds(const void *base, int nbytes, void *dst, int voff, int soff) {
  __builtin_amdgcn_raw_ptr_buffer_load_lds(__builtin_amdgcn_make_buffer_rsrc((void *)base, (short)0, nbytes, 0x00020000),
                                           (__attribute__((address_space(3))) void *)dst, 16, voff, soff, 0, 0);
}

template <int S, int WMW, int WNW, int WN, int SKB, int NBUF, int MINB, bool PIPE = false>
__global__ __launch_bounds__(64 * WMW * WNW, MINB) void k_split_gemm(
    const bf16x8 *__restrict__ Apk, const bf16x8 *__restrict__ Bpk, const uint64_t *__restrict__ rowmax,
    const uint64_t *__restrict__ colmax, double *__restrict__ D, int64_t M, int64_t N, int64_t KB, int64_t tiles_m,
    int64_t tiles_n) {
  using C = Cfg<S, WMW, WNW, WN, SKB, NBUF>;
  constexpr int L = C::L;
  __shared__ bf16x8 lds[NBUF][C::ST_CH * 64];

  int64_t tm, tn;
  // Each XCD walks its share of the tiles 4 tile rows at a time.
  grouped_tile(xcd_swizzle(blockIdx.x, tiles_m * tiles_n), tiles_m, tiles_n, 4, tm, tn);
  const int tid = threadIdx.x, lane = tid % 64;
  // Wave index as a wave-uniform (scalar) value, so chunk addresses are scalar.
  const int wave = __builtin_amdgcn_readfirstlane(tid / 64);
  __builtin_assume(wave >= 0 && wave < C::kWaves);
  const int wm = wave / WNW, wn = wave % WNW;

  // Per-wave chunk bases at stage 0, forced wave-uniform so they live in
  // scalar registers: a copy is then the scalar base plus the stage offset,
  // with the lane's 16-byte offset as the only vector register (per-copy
  // 64-bit vector addresses, hoisted out of the unrolled stages, would fill
  // the register file).
  const bf16x8 *cbase[C::MAX_WAVE];
#pragma unroll
  for (int q = 0; q < C::MAX_WAVE; ++q) {
    const int c = wave + C::kWaves * q;
    const bf16x8 *p;
    if (c < C::A_CH) {
      const int mbl = c / (SKB * S), rest = c % (SKB * S);
      p = Apk + ((tm * C::MBW + mbl) * KB * S + rest) * 64;
    } else {
      const int cb = c - C::A_CH;
      const int nbl = cb / (SKB * S), rest = cb % (SKB * S);
      p = Bpk + ((tn * C::NBW + nbl) * KB * S + rest) * 64;
    }
    // readfirstlane returns a signed int: each half goes through uint32_t
    // before widening, or a low half with bit 31 set would sign-extend over
    // the high half.
    const uint64_t u = (uint64_t)p;
    const uint64_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)(u >> 32));
    const uint64_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)u);
    cbase[q] = (const bf16x8 *)((hi << 32) | lo);
  }
  auto issue_stage = [&](int64_t st, int buf) {
#pragma unroll
    for (int q = 0; q < C::MAX_WAVE; ++q) {
      const int c = wave + C::kWaves * q;
      if (c >= C::ST_CH) break;
      __builtin_amdgcn_global_load_lds((const void *)(cbase[q] + st * (SKB * S * 64) + lane),
                                       (__attribute__((address_space(3))) void *)&lds[buf][c * 64], 16, 0, 0);
    }
  };

  floatx16 acc[L][WN];
  double acc64[WN][16];
  const floatx16 zero16 = {};
#pragma unroll
  for (int j = 0; j < WN; ++j)
#pragma unroll
    for (int v = 0; v < 16; ++v) acc64[j][v] = 0.0;
#pragma unroll
  for (int l = 0; l < L; ++l)
#pragma unroll
    for (int j = 0; j < WN; ++j) acc[l][j] = zero16;

  auto fold = [&](int l) {
#pragma unroll
    for (int j = 0; j < WN; ++j)
#pragma unroll
      for (int v = 0; v < 16; ++v) acc64[j][v] += (double)acc[l][j][v];
#pragma unroll
    for (int j = 0; j < WN; ++j) acc[l][j] = zero16;
  };

  // One 16-wide k block from LDS buffer `buf`. For each 32-column block j:
  // read its S B fragments, then round r issues, for each level d >= r
  // (largest first), the pair (s, t) = (r, d - r), so consecutive MFMAs
  // mostly update different accumulators.
  auto mma_kb = [&](int buf, int kbl) {
    bf16x8 af[S], bfr[S];
#pragma unroll
    for (int s = 0; s < S; ++s) af[s] = lds[buf][((wm * SKB + kbl) * S + s) * 64 + lane];
    [&]<int... J>(std::integer_sequence<int, J...>) {
      ([&]<int j>(std::integral_constant<int, j>) {
#pragma unroll
        for (int t = 0; t < S; ++t)
          bfr[t] = lds[buf][C::A_CH * 64 + (((wn * WN + j) * SKB + kbl) * S + t) * 64 + lane];
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int r = 0; r < S; ++r)
#pragma unroll
          for (int d = S - 1; d >= r; --d) {
            constexpr bool MG = C::MERGE;
            acc[acc_of<MG>(d)][j] = mfma_bf16(af[r], bfr[d - r], acc[acc_of<MG>(d)][j]);
          }
        __builtin_amdgcn_sched_barrier(0);
      }(std::integral_constant<int, J>{}), ...);
    }(std::make_integer_sequence<int, WN>{});
  };

  const int64_t nst = KB / SKB;
  // Stage st: wait for its copies, barrier, refill the buffer of stage st - 1
  // with stage st + NBUF - 1, then multiply its SKB k blocks.
  auto stage = [&](int64_t st) {
    const int buf = (int)(st % NBUF);
    // Issued so far: stages up to st + NBUF - 2. Stage st must be complete;
    // the NBUF - 2 after it may stay in flight (all of them near the end).
    if (NBUF > 2 && st + NBUF - 2 < nst) {
      if (wave < C::EXTRA)
        __builtin_amdgcn_s_waitcnt(vmcnt_imm((NBUF - 2) * C::MAX_WAVE));
      else
        __builtin_amdgcn_s_waitcnt(vmcnt_imm((NBUF - 2) * C::PER_WAVE));
    } else {
      __builtin_amdgcn_s_waitcnt(vmcnt_imm(0));
    }
    // A plain barrier, not __syncthreads(): its fence would also wait for the
    // copies still in flight. LDS is coherent within the workgroup.
    __builtin_amdgcn_s_barrier();
    if (st + NBUF - 1 < nst) issue_stage(st + NBUF - 1, (int)((st + NBUF - 1) % NBUF));
#pragma unroll
    for (int kbl = 0; kbl < SKB; ++kbl) mma_kb(buf, kbl);
  };

  // Folds after the 64-k group g (K is padded to a multiple of 64): level 2
  // after every group, level 1 after every second, levels 0 and 3 (or the
  // merged accumulator) after every fourth, separate levels from 4 up only
  // after the last; every accumulator folds after the last group (a fold
  // zeroes it).
  auto fold_group = [&](int64_t g, bool last) {
    if constexpr (L > 2) fold(2);
    if constexpr (L > 1)
      if ((g & 1) == 1 || last) fold(1);
    if ((g & 3) == 3 || last) {
      fold(0);
      if constexpr (L > 3) fold(3);
    }
    if (last) {
#pragma unroll
      for (int l = 4; l < L; ++l) fold(l);
    }
  };

  if constexpr (PIPE) {
    // Pipelined form for 32 x 64 wave blocks and one k block per stage. The
    // stage barrier sits inside the previous stage, after the first round of
    // its second column block: by then the wave has read every fragment of
    // that stage into registers. Each fragment register is refilled for the
    // next column block (or the next stage) right after its last MFMA, so
    // the LDS reads run under the matrix-core work instead of in a burst
    // after every barrier, when all waves would wait on them together.
    // B fragment t is last used by the first MFMA of round S - 1 - t, A
    // fragment r by the last MFMA of round r.
    static_assert(WN == 2 && SKB == 1 && NBUF >= 3 && NBUF <= 4, "pipelined form: 32 x 64 wave blocks, 16-k stages");
    auto a_at = [&](int buf, int s) -> const bf16x8 & { return lds[buf][(wm * S + s) * 64 + lane]; };
    auto b_at = [&](int buf, int j, int t) -> const bf16x8 & {
      return lds[buf][C::A_CH * 64 + ((wn * WN + j) * S + t) * 64 + lane];
    };
    // Copies by buffer loads into LDS: chunk stream q of this wave gets a
    // descriptor at its stage-0 chunk covering its nst chunks (the host keeps
    // that below 2^31 bytes); the stage offset goes in the scalar offset.
    // With global_load_lds in flight the compiler cannot order LDS reads and
    // turns every wait for one fragment into a wait for all of them.
    const int stream_bytes = (int)(nst * (S * 64 * 16));
    auto issue_buf = [&](int64_t st, int buf) {
#pragma unroll
      for (int q = 0; q < C::MAX_WAVE; ++q) {
        const int c = wave + C::kWaves * q;
        if (c >= C::ST_CH) break;
        copy16_to_lds(cbase[q], stream_bytes, &lds[buf][c * 64], lane * 16, (int)st * (S * 64 * 16));
      }
    };
    // Copy q of stage st; voff = kNoCopy (an offset past the stream) makes it
    // a no-op that reads no memory, so a copy past the last stage needs no
    // branch.
    constexpr int kNoCopy = (int)0x80000000u;
    auto copy_one = [&](int64_t st, int buf, int voff, int q) {
      copy16_to_lds(cbase[q], stream_bytes, &lds[buf][(wave + C::kWaves * q) * 64], voff, (int)st * (S * 64 * 16));
    };
    // Stage x becomes readable: its copies are done (the ones of the stages
    // after it that are already issued may stay in flight), every wave has
    // left the fragments of stage x - 1, and that buffer is refilled with
    // stage x + NBUF - 1.
    static_assert(C::EXTRA == 0, "pipelined form: every wave issues the same copies");
    auto wait_vm = [&]<int N>() { __builtin_amdgcn_s_waitcnt(vmcnt_imm(N)); };
    auto open_stage = [&](int64_t x) {
      const int64_t later = nst - 1 - x;  // stages after x
      if (later >= NBUF - 2)
        wait_vm.template operator()<(NBUF - 2) * C::PER_WAVE>();
      else if (NBUF > 3 && later == 1)
        wait_vm.template operator()<C::PER_WAVE>();
      else
        wait_vm.template operator()<0>();
      __builtin_amdgcn_s_barrier();
      __builtin_amdgcn_sched_barrier(0);
      // With two slices or more the copies of stage x + NBUF - 1 are spread
      // over the MFMAs after this barrier (run_stage); with one, here.
      if constexpr (S == 1)
        if (x + NBUF - 1 < nst) issue_buf(x + NBUF - 1, (int)((x + NBUF - 1) % NBUF));
    };
    // The epilogue's kernel arguments are loaded here, before the loop: a
    // scalar load still in flight would make every LDS wait in the loop a
    // full drain (scalar loads complete out of order on the same counter).
    asm volatile("" ::"s"(rowmax), "s"(colmax), "s"(D));
    bf16x8 af[S], bfr[S];
#pragma unroll
    for (int i = 0; i < NBUF - 1; ++i)
      if (i < nst) issue_buf(i, i);
    open_stage(0);
    // Stage NBUF - 1: with two slices or more open_stage leaves its copies
    // to the stage body, which issues those of stage st + NBUF; the first
    // such stage is issued here.
    if constexpr (S >= 2)
      if (NBUF - 1 < nst) {
#pragma unroll
        for (int q = 0; q < C::PER_WAVE; ++q) copy_one(NBUF - 1, NBUF - 1, lane * 16, q);
      }
    // Same read order as the loop's refills, so the waits at the loop head
    // are the same from both sides.
#pragma unroll
    for (int r = 0; r < S; ++r) {
      bfr[S - 1 - r] = b_at(0, 0, S - 1 - r);
      af[r] = a_at(0, r);
    }
    __builtin_amdgcn_sched_barrier(0);
    constexpr bool MG = C::MERGE;
    // One stage; MORE: a next stage exists (every stage but the last), so
    // the body has no data-dependent branches around its LDS reads.
    auto run_stage = [&]<bool MORE>(int64_t st) {
      const int buf = (int)(st % NBUF), nbuf = (int)((st + 1) % NBUF);
      // Column block 0; its B fragments are replaced by block 1's.
#pragma unroll
      for (int r = 0; r < S; ++r)
#pragma unroll
        for (int d = S - 1; d >= r; --d) {
          acc[acc_of<MG>(d)][0] = mfma_bf16(af[r], bfr[d - r], acc[acc_of<MG>(d)][0]);
          if (d == S - 1) {
            __builtin_amdgcn_sched_barrier(0);
            bfr[S - 1 - r] = b_at(buf, 1, S - 1 - r);
            __builtin_amdgcn_sched_barrier(0);
          }
        }
      // Column block 1, round 0 (it reads every B fragment).
#pragma unroll
      for (int d = S - 1; d >= 0; --d) acc[acc_of<MG>(d)][1] = mfma_bf16(af[0], bfr[d], acc[acc_of<MG>(d)][1]);
      __builtin_amdgcn_sched_barrier(0);
      if constexpr (MORE) {
        open_stage(st + 1);
        bfr[S - 1] = b_at(nbuf, 0, S - 1);
        af[0] = a_at(nbuf, 0);
        __builtin_amdgcn_sched_barrier(0);
      }
      // Rounds 1.. of column block 1; fragments are replaced by the next
      // stage's as they retire, and the copies of stage st + NBUF (into the
      // buffer of stage st, which every wave has left) go one after every
      // few MFMAs: copy q follows MFMA q * T / PER_WAVE of these T.
      constexpr int T = S * (S - 1) / 2;
      const int voff = st + NBUF < nst ? lane * 16 : kNoCopy;
#pragma unroll
      for (int r = 1; r < S; ++r) {
#pragma unroll
        for (int d = S - 1; d >= r; --d) {
          acc[acc_of<MG>(d)][1] = mfma_bf16(af[r], bfr[d - r], acc[acc_of<MG>(d)][1]);
          if constexpr (MORE) {
            __builtin_amdgcn_sched_barrier(0);
            if (d == S - 1) bfr[S - 1 - r] = b_at(nbuf, 0, S - 1 - r);
            const int t = (r - 1) * S - (r - 1) * r / 2 + (S - 1 - d);
#pragma unroll
            for (int q = 0; q < C::PER_WAVE; ++q)
              if (q * T / C::PER_WAVE == t) copy_one(st + NBUF, buf, voff, q);
            __builtin_amdgcn_sched_barrier(0);
          }
        }
        if constexpr (MORE) {
          af[r] = a_at(nbuf, r);
          __builtin_amdgcn_sched_barrier(0);
        }
      }
      if ((st & 3) == 3) fold_group(st >> 2, !MORE);
    };
    for (int64_t st = 0; st + 1 < nst; ++st) run_stage.template operator()<true>(st);
    run_stage.template operator()<false>(nst - 1);
    // The last stages issued no-op copies after their final wait: drain them
    // so that no copy into LDS is outstanding when the workgroup ends.
    __builtin_amdgcn_s_waitcnt(vmcnt_imm(0));
  } else {
    for (int i = 0; i < NBUF - 1; ++i)
      if (i < nst) issue_stage(i, i);
    const int64_t ngroups = nst / (4 / SKB);
    for (int64_t g = 0; g < ngroups; ++g) {
#pragma unroll
      for (int i = 0; i < 4 / SKB; ++i) stage(g * (4 / SKB) + i);
      fold_group(g, g + 1 == ngroups);
    }
  }

  // Epilogue: exact power-of-two descaling, D[i, j] = 2^(e_i + f_j - 16) * acc.
  // Lane l < 32 reads the exponent of the wave's row l and hands it to the
  // lanes that store that row (one load per lane instead of 16, which the
  // compiler would hoist above the loop and keep in registers).
  const int64_t col_base = tn * C::BN + wn * (32 * WN);
  const int64_t row_base = tm * C::BM + wm * 32;
  const int e_lane = (row_base + lane % 32 < M) ? exponent_of_max(rowmax[row_base + lane % 32]) : 0;
#pragma unroll
  for (int j = 0; j < WN; ++j) {
    const int64_t gn = col_base + j * 32 + lane % 32;
    const int fe = (gn < N) ? exponent_of_max(colmax[gn]) : 0;
#pragma unroll
    for (int v = 0; v < 16; ++v) {
      const int r = (v / 4) * 8 + (lane / 32) * 4 + (v % 4);
      const int ee = __shfl(e_lane, r);
      const int64_t gm = row_base + r;
      if (gm < M && gn < N) D[gm * N + gn] = ldexp(acc64[j][v], ee + fe - 2 * (kBeta - 1));
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

template <int S, int WMW, int WNW, bool PIPE = false>
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
  __builtin_assume(wave >= 0 && wave < C::kWaves);
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
  if constexpr (PIPE) {
    // Pipelined form, as in the BF16 kernel: buffer loads into LDS (so the
    // compiler can wait for one fragment at a time), the barrier of stage
    // st + 1 after round 0 of stage st, and each fragment register refilled
    // with the next stage's right after its last MFMA (B fragment t: first
    // MFMA of round S - 1 - t; A fragment r: last MFMA of round r).
    const intx4 *qbase[C::MAX_WAVE];
#pragma unroll
    for (int q = 0; q < C::MAX_WAVE; ++q) {
      const int c = wave + C::kWaves * q;
      const intx4 *p;
      if (c < C::A_CH)
        p = Apk + ((tm * C::MBW + c / S) * KB * S + c % S) * 64;
      else
        p = Bpk + ((tn * C::NBW + (c - C::A_CH) / S) * KB * S + (c - C::A_CH) % S) * 64;
      qbase[q] = uniform_ptr(p);
    }
    const int stream_bytes = (int)(nst * (S * 64 * 16));
    auto issue_buf = [&](int64_t st, int buf) {
#pragma unroll
      for (int q = 0; q < C::MAX_WAVE; ++q) {
        const int c = wave + C::kWaves * q;
        if (c >= C::ST_CH) break;
        copy16_to_lds(qbase[q], stream_bytes, &lds[buf][c * 64], lane * 16, (int)st * (S * 64 * 16));
      }
    };
    // Copy q of stage st; voff = kNoCopy (an offset past the stream) makes it
    // a no-op that reads no memory, so a copy past the last stage needs no
    // branch.
    constexpr int kNoCopy = (int)0x80000000u;
    auto copy_one = [&](int64_t st, int buf, int voff, int q) {
      copy16_to_lds(qbase[q], stream_bytes, &lds[buf][(wave + C::kWaves * q) * 64], voff, (int)st * (S * 64 * 16));
    };
    // Stage x becomes readable: its copies are done (the next stage's may
    // stay in flight) and, after this wave's LDS reads have drained, every
    // wave has left the buffer that now takes stage x + 2.
    auto open_stage = [&](int64_t x) {
      if (x + 1 < nst) {
        if (wave < C::EXTRA)
          __builtin_amdgcn_s_waitcnt(vmcnt_lgkm0_imm(C::MAX_WAVE));
        else
          __builtin_amdgcn_s_waitcnt(vmcnt_lgkm0_imm(C::PER_WAVE));
      } else {
        __builtin_amdgcn_s_waitcnt(vmcnt_lgkm0_imm(0));
      }
      __builtin_amdgcn_s_barrier();
      __builtin_amdgcn_sched_barrier(0);
      // With two slices or more, every wave's first PER_WAVE copies of stage
      // x + 2 are spread over the MFMAs after this barrier (run_stage) and
      // only the extra copy of the first EXTRA waves goes here; with one
      // slice, all of them.
      if (x + 2 < nst) {
        if constexpr (S == 1) {
          issue_buf(x + 2, (int)((x + 2) % kNBuf));
        } else if constexpr (C::EXTRA > 0) {
          if (wave < C::EXTRA) copy_one(x + 2, (int)((x + 2) % kNBuf), lane * 16, C::PER_WAVE);
        }
      }
    };
    auto a_at = [&](int buf, int s) -> const intx4 & { return lds[buf][(wm * S + s) * 64 + lane]; };
    auto b_at = [&](int buf, int t) -> const intx4 & { return lds[buf][C::A_CH * 64 + (wn * S + t) * 64 + lane]; };
    asm volatile("" ::"s"(rowmax), "s"(colmax), "s"(D));
    intx4 af[S], bfr[S];
    issue_buf(0, 0);
    if (1 < nst) issue_buf(1, 1);
    open_stage(0);
    // Stage 2: with two slices or more open_stage issues only its extra
    // copy and leaves the others to the stage body, which issues those of
    // stage st + 3; the first such stage is issued here.
    if constexpr (S >= 2)
      if (2 < nst) {
#pragma unroll
        for (int q = 0; q < C::PER_WAVE; ++q) copy_one(2, 2, lane * 16, q);
      }
#pragma unroll
    for (int r = 0; r < S; ++r) {
      bfr[S - 1 - r] = b_at(0, S - 1 - r);
      af[r] = a_at(0, r);
    }
    __builtin_amdgcn_sched_barrier(0);
    auto run_stage = [&]<bool MORE>(int64_t st) {
      const int nbuf = (int)((st + 1) % kNBuf);
#pragma unroll
      for (int d = S - 1; d >= 0; --d) acc[d] = __builtin_amdgcn_mfma_i32_32x32x32_i8(af[0], bfr[d], acc[d], 0, 0, 0);
      __builtin_amdgcn_sched_barrier(0);
      if constexpr (MORE) {
        open_stage(st + 1);
        bfr[S - 1] = b_at(nbuf, S - 1);
        af[0] = a_at(nbuf, 0);
        __builtin_amdgcn_sched_barrier(0);
      }
      // Copies of stage st + 3 (into the buffer of stage st, which every
      // wave has left): copy q follows MFMA q * T / PER_WAVE of rounds 1...
      constexpr int T = S * (S - 1) / 2;
      const int voff = st + 3 < nst ? lane * 16 : kNoCopy;
#pragma unroll
      for (int r = 1; r < S; ++r) {
#pragma unroll
        for (int d = S - 1; d >= r; --d) {
          acc[d] = __builtin_amdgcn_mfma_i32_32x32x32_i8(af[r], bfr[d - r], acc[d], 0, 0, 0);
          if constexpr (MORE) {
            __builtin_amdgcn_sched_barrier(0);
            if (d == S - 1) bfr[S - 1 - r] = b_at(nbuf, S - 1 - r);
            const int t = (r - 1) * S - (r - 1) * r / 2 + (S - 1 - d);
#pragma unroll
            for (int q = 0; q < C::PER_WAVE; ++q)
              if (q * T / (C::PER_WAVE > 0 ? C::PER_WAVE : 1) == t) copy_one(st + 3, (int)(st % kNBuf), voff, q);
            __builtin_amdgcn_sched_barrier(0);
          }
        }
        if constexpr (MORE) {
          af[r] = a_at(nbuf, r);
          __builtin_amdgcn_sched_barrier(0);
        }
      }
      if ((st + 1) % kFoldStages == 0) fold_all();
    };
    for (int64_t st = 0; st + 1 < nst; ++st) run_stage.template operator()<true>(st);
    run_stage.template operator()<false>(nst - 1);
    // The last stages issued no-op copies after their final wait: drain them
    // so that no copy into LDS is outstanding when the workgroup ends.
    __builtin_amdgcn_s_waitcnt(vmcnt_imm(0));
  } else {
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
        for (int d = S - 1; d >= r; --d)
          acc[d] = __builtin_amdgcn_mfma_i32_32x32x32_i8(af[r], bfr[d - r], acc[d], 0, 0, 0);
      if ((st + 1) % kFoldStages == 0) fold_all();
    }
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
