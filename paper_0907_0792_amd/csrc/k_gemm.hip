// (+,*) inner product on the matrix cores: D (M x N) = A (M x K) . B (K x N).
//
// The (+,*) case of Eq. inner (Section I), which the paper notes is the
// standard matrix product, for FP64 (v_mfma_f64_16x16x4_f64) and FP32
// (v_mfma_f32_16x16x4_f32). Any rank reaches this kernel as the flattened
// M x K and K x N views.
//
// Workgroup = 4 waves (2 x 2), each owning a (16*WBM) x (16*WBN) block of D
// as WBM x WBN 16x16 accumulator tiles. A and B panels of BK = 16 k (32 for
// FP32) are staged in LDS (k-major, so one fragment read is 16 contiguous
// elements per k row);
// the next panel is fetched into registers while the current one is
// multiplied, as 16-byte vectors when the operands are aligned and their
// contiguous extents are multiples of the vector length (VEC).
// trans_a / trans_b read A stored K x M or B stored N x K, which
// is how the backward pass contracts over permuted axes without a transposed
// copy; the GEN variants read the strided (P, K, Q) views of a contraction
// over any axis pair.
#include <utility>

#include "common.hpp"
#include "gemm_tile.hpp"
#include "internal.hpp"

namespace moa {

// I = int32_t: the FP32 128 x 128 vector-panel kernel with 32-bit index
// arithmetic, where every offset fits; its registers then allow four
// workgroups per CU (a 20-byte spill), so 1024 tiles run in one round:
// 4096 x 512 . 512 x 4096 0.196 -> 0.169 ms, 8192^3 unchanged (8.70 ms).
template <typename T, int WBM, bool VEC, typename I>
constexpr int gemm_min_blocks() {
  return (sizeof(T) == 4 && WBM == 4 && VEC && sizeof(I) == 4) ? 4 : 2;
}

template <typename T, bool TA, bool TB, int WBM, int WBN, bool GEN, bool VEC, typename I = int64_t>
__global__ __launch_bounds__(256, (gemm_min_blocks<T, WBM, VEC, I>())) void k_gemm(
    const T *__restrict__ A, const T *__restrict__ B, T *__restrict__ D, int64_t M, int64_t K, int64_t N,
    int64_t tiles_m, int64_t tiles_n, int64_t Qa, int64_t Qb) {
  int64_t tm, tn;
  grouped_tile(xcd_swizzle(blockIdx.x, tiles_m * tiles_n), tiles_m, tiles_n, 8, tm, tn);
  // FP32 MFMAs run at twice the FP64 rate: 32-wide k panels halve the
  // barriers and panel stores per flop (below: except one tile).
  // Row-major staging of k-contiguous operands for the FP64 vector-panel
  // tiles, and for the FP32 128 x 128 tile with 32-bit indices, there with
  // 16-wide panels: its four workgroups per CU leave 128 registers, which
  // 32-wide panels plus the longer-lived fragments would exceed (FP32
  // 8192^3 8.57 -> 8.45 ms, 4096 x 512 . 512 x 4096 forward + backward
  // 0.546 -> 0.541 ms, same box). The other FP32 tiles keep 32-wide k-major
  // panels.
  constexpr bool F32I = sizeof(T) == 4 && sizeof(I) == 4 && WBM == 4 && VEC;
  constexpr bool RCL = (sizeof(T) == 8 && VEC) || F32I;
  gemm_tile<T, TA, TB, WBM, WBN, (sizeof(T) == 4 && !F32I) ? 32 : 16, GEN, false, VEC, I, RCL>(
      A, B, D, (I)M, (I)K, (I)N, (I)(tm * 32 * WBM), (I)(tn * 32 * WBN), (I)Qa, (I)Qb);
}

// Small grids (fewer 32 x 32 tiles than the GPU has SIMDs) with a long
// contraction: one 32 x 32 tile per workgroup of KG groups of 4 waves. Group
// g takes the k panels g, g + KG, g + 2 KG, ..., keeping DEPTH panels in
// flight in registers, so each wave waits out about nk / (KG DEPTH) load
// round trips instead of nk, and each SIMD holds KG waves instead of one.
// Panels are staged in two LDS buffers (one barrier per panel). The groups'
// partial tiles are summed in LDS in group order (deterministic). FP64 512^3:
// 15-17 us with the one-group kernel.
template <typename T, int KG, int BK, int DEPTH, bool VEC>
__global__ __launch_bounds__(256 * KG, 1) void k_gemm_splitk(const T *__restrict__ A, const T *__restrict__ B,
                                                             T *__restrict__ D, int64_t M, int64_t K, int64_t N,
                                                             int64_t tiles_m, int64_t tiles_n) {
  using MF = Mfma16<T>;
  using acc_t = typename MF::acc_t;
  constexpr int BM = 32, BN = 32, PAD = 2;
  constexpr int V = VEC ? 16 / (int)sizeof(T) : 1;
  constexpr int EA = BM * BK / 256, EB = BN * BK / 256;  // elements per thread per panel
  typedef __attribute__((__vector_size__(V * sizeof(T)))) T vec_t;
  // A is staged row-major (its rows are what the lanes load, 16-byte runs
  // along k), padded by 16 bytes so the 16 rows of a fragment read start in
  // different banks; B k-major.
  constexpr int PA = 16 / (int)sizeof(T);
  __shared__ T As[2][KG][BM][BK + PA];
  __shared__ T Bs[2][KG][BK][BN + PAD];
  static_assert(sizeof(As) >= sizeof(T) * 4 * 256 * (KG - 1), "reduction space");

  int64_t tm, tn;
  grouped_tile(xcd_swizzle(blockIdx.x, tiles_m * tiles_n), tiles_m, tiles_n, 8, tm, tn);
  const int64_t m0 = tm * BM, n0 = tn * BN;
  const int tid = threadIdx.x % 256, lane = tid % kWave;
  const int g = __builtin_amdgcn_readfirstlane(threadIdx.x / 256);
  const int wave = __builtin_amdgcn_readfirstlane(tid / kWave);
  const int wm = wave / 2, wn = wave % 2;

  // Loads are unconditional (an element past an edge reads element 0 and is
  // zeroed when stored), so they issue as straight-line code and the wait
  // before a store covers only that panel's loads, not the later ones.
  // (Whether an element is inside is recomputed at the store: keeping the
  // flags would cost registers.)
  vec_t ra[DEPTH][EA / V], rb[DEPTH][EB / V];
  auto a_in = [&](int e, int64_t k0) {
    const int f = tid + 256 * e;
    return m0 + f / (BK / V) < M && k0 + (f % (BK / V)) * V < K;
  };
  auto b_in = [&](int e, int64_t k0) {
    const int f = tid + 256 * e;
    return n0 + (f % (BN / V)) * V < N && k0 + f / (BN / V) < K;
  };
  auto load = [&](auto bufc, int64_t k0) {
    constexpr int buf = decltype(bufc)::value;
#pragma unroll
    for (int e = 0; e < EA / V; ++e) {
      const int f = tid + 256 * e;
      const int64_t gm = m0 + f / (BK / V), gk = k0 + (f % (BK / V)) * V;
      ra[buf][e] = *(const vec_t *)(A + (a_in(e, k0) ? gm * K + gk : 0));
    }
#pragma unroll
    for (int e = 0; e < EB / V; ++e) {
      const int f = tid + 256 * e;
      const int64_t gk = k0 + f / (BN / V), gn = n0 + (f % (BN / V)) * V;
      rb[buf][e] = *(const vec_t *)(B + (b_in(e, k0) ? gk * N + gn : 0));
    }
  };
  auto store = [&](auto bufc, int lb, int64_t k0) {
    constexpr int buf = decltype(bufc)::value;
#pragma unroll
    for (int e = 0; e < EA / V; ++e) {
      const int f = tid + 256 * e;
      const bool in = a_in(e, k0);
#pragma unroll
      for (int u = 0; u < V; ++u) As[lb][g][f / (BK / V)][(f % (BK / V)) * V + u] = in ? ra[buf][e][u] : T(0);
    }
#pragma unroll
    for (int e = 0; e < EB / V; ++e) {
      const int f = tid + 256 * e;
      const bool in = b_in(e, k0);
#pragma unroll
      for (int u = 0; u < V; ++u) Bs[lb][g][f / (BN / V)][(f % (BN / V)) * V + u] = in ? rb[buf][e][u] : T(0);
    }
  };

  // Two accumulators (even and odd k steps) break the MFMA dependency chain.
  acc_t acc[2];
#pragma unroll
  for (int h = 0; h < 2; ++h)
#pragma unroll
    for (int v = 0; v < 4; ++v) acc[h][v] = T(0);

  const int64_t nk = (K + BK - 1) / BK;
  const int64_t live = (nk + KG - 1) / KG;  // rounds with a panel for some group
  // Every group runs the same number of rounds, a multiple of DEPTH, so the
  // loop body has no branch around a load; rounds past `live` only load.
  const int64_t rounds = (live + DEPTH - 1) / DEPTH * DEPTH;
  // Round r multiplies panel r from LDS buffer r % 2 while the stores of
  // panel r + 1 (register set (r + 1) % DEPTH) fill the other buffer, which
  // every wave finished reading in round r - 1, and that register set is
  // refilled with panel r + 1 + DEPTH; one barrier ends the round. The MFMAs
  // of a round thus overlap the next panel's LDS stores.
  auto round = [&](int64_t r, auto bufc) {
    constexpr int nbuf = (decltype(bufc)::value + 1) % DEPTH;
    const int lb = (int)(r & 1);
    if (r < live) {
#pragma unroll
      for (int k4 = 0; k4 < BK; k4 += 4) {
        const T a = As[lb][g][wm * 16 + lane % 16][k4 + lane / 16];
        const T b = Bs[lb][g][k4 + lane / 16][wn * 16 + lane % 16];
        acc[(k4 / 4) & 1] = MF::run(a, b, acc[(k4 / 4) & 1]);
      }
    }
    store(std::integral_constant<int, nbuf>{}, lb ^ 1, ((r + 1) * KG + g) * BK);
    load(std::integral_constant<int, nbuf>{}, ((r + 1 + DEPTH) * KG + g) * BK);
    __syncthreads();
  };
  [&]<int... J>(std::integer_sequence<int, J...>) {
    (load(std::integral_constant<int, J>{}, ((int64_t)J * KG + g) * BK), ...);
  }(std::make_integer_sequence<int, DEPTH>{});
  store(std::integral_constant<int, 0>{}, 0, (int64_t)g * BK);
  load(std::integral_constant<int, 0>{}, ((int64_t)DEPTH * KG + g) * BK);
  __syncthreads();
  for (int64_t r = 0; r < rounds; r += DEPTH) {
    [&]<int... J>(std::integer_sequence<int, J...>) {
      (round(r + J, std::integral_constant<int, J>{}), ...);
    }(std::make_integer_sequence<int, DEPTH>{});
  }
#pragma unroll
  for (int v = 0; v < 4; ++v) acc[0][v] += acc[1][v];
  // Groups 1..KG-1 hand their partial tiles to group 0 through LDS.
  __syncthreads();
  T *red = &As[0][0][0][0];
  if (g > 0) {
#pragma unroll
    for (int v = 0; v < 4; ++v) red[((g - 1) * 4 + v) * 256 + tid] = acc[0][v];
  }
  __syncthreads();
  if (g == 0) {
#pragma unroll
    for (int q = 1; q < KG; ++q)
#pragma unroll
      for (int v = 0; v < 4; ++v) acc[0][v] += red[((q - 1) * 4 + v) * 256 + tid];
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int64_t gm = m0 + wm * 16 + MF::row(lane, v), gn = n0 + wn * 16 + lane % 16;
      if (gm < M && gn < N) D[gm * N + gn] = acc[0][v];
    }
  }
}

// Small grids with a contraction of at most 512: one 32 x 32 tile per
// workgroup of 16 waves, wave w taking k = 32 w .. 32 w + 31 of all four
// 16 x 16 blocks. Fragments go from memory straight into registers: in MFMA
// step s (of 8) the lanes 16 c + r (c = 0..3) supply k = 32 w + 8 c + s (any
// assignment of k to lanes and steps gives the same sum, as long as A and B
// use the same one), so a lane's A values of one block are 8 consecutive k
// (16-byte vectors) and its B values 8 rows of one column (each row read by
// 16 lanes as one run). Every load is issued before the first MFMA: one
// memory round trip per tile, no LDS staging, no barrier until the partial
// tiles are summed through LDS in wave order (deterministic).
template <typename T>
__global__ __launch_bounds__(1024, 1) void k_gemm_kslice(const T *__restrict__ A, const T *__restrict__ B,
                                                         T *__restrict__ D, int64_t M, int64_t K, int64_t N,
                                                         int64_t tiles_m, int64_t tiles_n) {
  using MF = Mfma16<T>;
  using acc_t = typename MF::acc_t;
  constexpr int V = 16 / (int)sizeof(T);
  typedef T vec_t __attribute__((ext_vector_type(V)));
  __shared__ T part[16][32 * 32];
  int64_t tm, tn;
  grouped_tile(xcd_swizzle(blockIdx.x, tiles_m * tiles_n), tiles_m, tiles_n, 8, tm, tn);
  const int64_t m0 = tm * 32, n0 = tn * 32;
  const int lane = threadIdx.x % kWave, w = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
  const int r = lane % 16, c = lane / 16;
  const int64_t kb = 32 * w + 8 * c;  // this lane's first k
  // A: rows m0 + 16 ib + r, k = kb .. kb + 7 (K % V == 0: a vector is wholly
  // inside or past K). B: rows kb .. kb + 7, column n0 + 16 jb + r.
  vec_t av[2][8 / V];
  T bv[2][8];
#pragma unroll
  for (int ib = 0; ib < 2; ++ib) {
    const int64_t row = m0 + 16 * ib + r;
#pragma unroll
    for (int q = 0; q < 8 / V; ++q) {
      const int64_t k = kb + V * q;
      av[ib][q] = (row < M && k < K) ? *(const vec_t *)(A + row * K + k) : vec_t{};
    }
  }
#pragma unroll
  for (int jb = 0; jb < 2; ++jb) {
    const int64_t col = n0 + 16 * jb + r;
#pragma unroll
    for (int s = 0; s < 8; ++s) {
      const int64_t k = kb + s;
      bv[jb][s] = (col < N && k < K) ? B[k * N + col] : T(0);
    }
  }
  acc_t acc[2][2];
#pragma unroll
  for (int ib = 0; ib < 2; ++ib)
#pragma unroll
    for (int jb = 0; jb < 2; ++jb)
#pragma unroll
      for (int v = 0; v < 4; ++v) acc[ib][jb][v] = T(0);
#pragma unroll
  for (int s = 0; s < 8; ++s)
#pragma unroll
    for (int ib = 0; ib < 2; ++ib)
#pragma unroll
      for (int jb = 0; jb < 2; ++jb) acc[ib][jb] = MF::run(av[ib][s / V][s % V], bv[jb][s], acc[ib][jb]);
#pragma unroll
  for (int ib = 0; ib < 2; ++ib)
#pragma unroll
    for (int jb = 0; jb < 2; ++jb)
#pragma unroll
      for (int v = 0; v < 4; ++v) part[w][(16 * ib + MF::row(lane, v)) * 32 + 16 * jb + r] = acc[ib][jb][v];
  __syncthreads();
  const int e = threadIdx.x;  // one element of the 32 x 32 tile per thread
  T sum = part[0][e];
#pragma unroll
  for (int q = 1; q < 16; ++q) sum += part[q][e];
  const int64_t gm = m0 + e / 32, gn = n0 + e % 32;
  if (gm < M && gn < N) D[gm * N + gn] = sum;
}

// Every offset of a tile of M x K . K x N (extents padded by a 128 tile) fits
// in 31 bits.
static bool fits_int32(int64_t M, int64_t K, int64_t N) {
  const int64_t lim = (int64_t)1 << 31;
  return (M + 128) * (K + 128) < lim && (K + 128) * (N + 128) < lim && (M + 128) * (N + 128) < lim;
}

// The largest tile that still gives the CUs enough workgroups: 128 x 128
// (1) from 512 tiles up, 64 x 64 (2) from 256 (one per CU), else 32 x 32 (3).
static int auto_tile(int64_t M, int64_t N) {
  const int64_t big = ((M + 127) / 128) * ((N + 127) / 128);
  const int64_t mid = ((M + 63) / 64) * ((N + 63) / 64);
  return big >= 512 ? 1 : mid >= 256 ? 2 : 3;
}

template <typename T, bool TA, bool TB, bool GEN, bool VEC>
static hipError_t launch_t(const T *A, const T *B, T *D, int64_t M, int64_t K, int64_t N, int tile, int64_t Qa,
                           int64_t Qb, hipStream_t s) {
  const bool automatic = tile == 0;
  if (tile == 0) tile = auto_tile(M, N);
  if (tile == 3) {
    const int64_t tmn = (M + 31) / 32, tnn = (N + 31) / 32;
    if (tmn * tnn > 0x7fffffff) return hipErrorInvalidConfiguration;
    if constexpr (!TA && !TB && !GEN) {
      // Fewer 32 x 32 tiles than SIMDs and a contraction of at least 256:
      // split it over four wave groups per tile.
      if constexpr (VEC) {
        // A contraction of 256..512: every fragment in registers at once.
        if (automatic && tmn * tnn < 1024 && K >= 256 && K <= 512) {
          hipLaunchKernelGGL((k_gemm_kslice<T>), dim3((unsigned)(tmn * tnn)), dim3(1024), 0, s, A, B, D, M, K, N,
                             tmn, tnn);
          return hipGetLastError();
        }
      }
      if (automatic && tmn * tnn < 1024 && K >= 256) {
        // 32-wide panels, two in flight per thread beyond the one in LDS.
        hipLaunchKernelGGL((k_gemm_splitk<T, 4, 32, 2, VEC>), dim3((unsigned)(tmn * tnn)), dim3(1024), 0, s, A, B, D,
                           M, K, N, tmn, tnn);
        return hipGetLastError();
      }
    }
    hipLaunchKernelGGL((k_gemm<T, TA, TB, 1, 1, GEN, VEC>), dim3((unsigned)(tmn * tnn)), dim3(256), 0, s, A, B, D, M, K,
                       N, tmn, tnn, Qa, Qb);
  } else if (tile == 1) {
    const int64_t tmn = (M + 127) / 128, tnn = (N + 127) / 128;
    if (tmn * tnn > 0x7fffffff) return hipErrorInvalidConfiguration;
    if constexpr (sizeof(T) == 4 && VEC && !GEN) {
      if (fits_int32(M, K, N)) {
        hipLaunchKernelGGL((k_gemm<T, TA, TB, 4, 4, GEN, VEC, int32_t>), dim3((unsigned)(tmn * tnn)), dim3(256), 0, s,
                           A, B, D, M, K, N, tmn, tnn, Qa, Qb);
        return hipGetLastError();
      }
    }
    hipLaunchKernelGGL((k_gemm<T, TA, TB, 4, 4, GEN, VEC>), dim3((unsigned)(tmn * tnn)), dim3(256), 0, s, A, B, D, M, K,
                       N, tmn, tnn, Qa, Qb);
  } else {
    const int64_t tmn = (M + 63) / 64, tnn = (N + 63) / 64;
    if (tmn * tnn > 0x7fffffff) return hipErrorInvalidConfiguration;
    hipLaunchKernelGGL((k_gemm<T, TA, TB, 2, 2, GEN, VEC>), dim3((unsigned)(tmn * tnn)), dim3(256), 0, s, A, B, D, M, K,
                       N, tmn, tnn, Qa, Qb);
  }
  return hipGetLastError();
}

template <typename T, bool GEN, bool VEC>
static hipError_t launch_tv(bool ta, bool tb, const T *A, const T *B, T *D, int64_t M, int64_t K, int64_t N, int tile,
                            int64_t Qa, int64_t Qb, hipStream_t s) {
  if (!ta && !tb) return launch_t<T, false, false, GEN, VEC>(A, B, D, M, K, N, tile, Qa, Qb, s);
  if (ta && !tb) return launch_t<T, true, false, GEN, VEC>(A, B, D, M, K, N, tile, Qa, Qb, s);
  if (!ta && tb) return launch_t<T, false, true, GEN, VEC>(A, B, D, M, K, N, tile, Qa, Qb, s);
  return launch_t<T, true, true, GEN, VEC>(A, B, D, M, K, N, tile, Qa, Qb, s);
}

// Vector panels need 16-byte aligned operands whose extents along the lanes'
// axis are multiples of the vector length: the stored row length of A and B,
// or for the strided views the inner extent Qa (Qb) when it is not 1 and K
// when it is.
template <typename T>
static bool vec_ok(const T *A, const T *B, int64_t a_run, int64_t b_run) {
  constexpr int64_t V = 16 / sizeof(T);
  return ((uintptr_t)A % 16) == 0 && ((uintptr_t)B % 16) == 0 && a_run % V == 0 && b_run % V == 0;
}

template <typename T, bool GEN>
static hipError_t launch_tt(bool ta, bool tb, bool vec, const T *A, const T *B, T *D, int64_t M, int64_t K, int64_t N,
                            int tile, int64_t Qa, int64_t Qb, hipStream_t s) {
  if (vec) return launch_tv<T, GEN, true>(ta, tb, A, B, D, M, K, N, tile, Qa, Qb, s);
  return launch_tv<T, GEN, false>(ta, tb, A, B, D, M, K, N, tile, Qa, Qb, s);
}

hipError_t launch_gemm(moa_dtype dt, bool trans_a, bool trans_b, const void *A, const void *B, void *D, int64_t M,
                       int64_t K, int64_t N, int tile, hipStream_t s) {
  if (M == 0 || N == 0) return hipSuccess;
  const int64_t a_run = trans_a ? M : K, b_run = trans_b ? K : N;
  if (dt == MOA_F64) {
    const double *a = (const double *)A, *b = (const double *)B;
    return launch_tt<double, false>(trans_a, trans_b, vec_ok(a, b, a_run, b_run), a, b, (double *)D, M, K, N, tile, 1,
                                    1, s);
  }
  if (dt == MOA_F32) {
    const float *a = (const float *)A, *b = (const float *)B;
    return launch_tt<float, false>(trans_a, trans_b, vec_ok(a, b, a_run, b_run), a, b, (float *)D, M, K, N, tile, 1, 1,
                                   s);
  }
  return hipErrorInvalidValue;
}

// Contraction over any axis pair: A, B read through their (P, K, Q) views.
// Lanes run along i when A's inner extent Qa exceeds 1 and along k when B's
// inner extent Qb is 1, so neighbouring lanes read neighbouring addresses.
hipError_t launch_gemm_strided(moa_dtype dt, const void *A, const void *B, void *D, int64_t M, int64_t K, int64_t N,
                               int64_t Qa, int64_t Qb, hipStream_t s) {
  if (M == 0 || N == 0) return hipSuccess;
  if (Qa <= 0 || Qb <= 0) return hipErrorInvalidValue;
  const bool ta = Qa != 1, tb = Qb == 1;
  const int64_t a_run = ta ? Qa : K, b_run = tb ? K : Qb;
  if (dt == MOA_F64) {
    const double *a = (const double *)A, *b = (const double *)B;
    return launch_tt<double, true>(ta, tb, vec_ok(a, b, a_run, b_run), a, b, (double *)D, M, K, N, 0, Qa, Qb, s);
  }
  if (dt == MOA_F32) {
    const float *a = (const float *)A, *b = (const float *)B;
    return launch_tt<float, true>(ta, tb, vec_ok(a, b, a_run, b_run), a, b, (float *)D, M, K, N, 0, Qa, Qb, s);
  }
  return hipErrorInvalidValue;
}

// The two products of the backward pass in one launch: workgroups [0, n0)
// take tiles of dA = G . B^T (B read as stored, K x N = (N x K)^T), the rest
// tiles of dB = A^T . G (A read as stored). One launch instead of two: no gap
// between them, and the second product's tiles fill the CUs the first one's
// tail leaves idle.
struct GemmJob {
  const void *A;
  const void *B;
  void *D;
  int64_t M, K, N, tiles_m, tiles_n;
};

template <typename T, int WBM, int WBN, int BK, bool VEC>
__global__ __launch_bounds__(256, 2) void k_gemm_grad_pair(GemmJob j0, GemmJob j1) {
  __shared__ __attribute__((aligned(16))) unsigned char smem[gemm_tile_lds_bytes<T, WBM, WBN, BK>()];
  const int64_t n0 = j0.tiles_m * j0.tiles_n;
  int64_t tm, tn;
  if ((int64_t)blockIdx.x < n0) {
    grouped_tile(xcd_swizzle(blockIdx.x, n0), j0.tiles_m, j0.tiles_n, 8, tm, tn);
    // dA = G . B^T reads both operands k-contiguous: row-major staging where
    // the registers allow it (tiles up to 64 x 64).
    gemm_tile_at<T, false, true, WBM, WBN, BK, false, false, VEC, int64_t, VEC && WBM <= 2>(
        (const T *)j0.A, (const T *)j0.B, (T *)j0.D, j0.M, j0.K, j0.N, tm * 32 * WBM, tn * 32 * WBN, (int64_t)1,
        (int64_t)1, smem);
  } else {
    const int64_t b = blockIdx.x - n0, n1 = j1.tiles_m * j1.tiles_n;
    grouped_tile(xcd_swizzle(b, n1), j1.tiles_m, j1.tiles_n, 8, tm, tn);
    gemm_tile_at<T, true, false, WBM, WBN, BK, false, false, VEC>((const T *)j1.A, (const T *)j1.B, (T *)j1.D, j1.M,
                                                                   j1.K, j1.N, tm * 32 * WBM, tn * 32 * WBN,
                                                                   (int64_t)1, (int64_t)1, smem);
  }
}

template <typename T, int WBM, int WBN, int BK, bool VEC>
static hipError_t launch_pair_t(GemmJob j0, GemmJob j1, hipStream_t s) {
  constexpr int sm = 32 * WBM, sn = 32 * WBN;
  j0.tiles_m = (j0.M + sm - 1) / sm;
  j0.tiles_n = (j0.N + sn - 1) / sn;
  j1.tiles_m = (j1.M + sm - 1) / sm;
  j1.tiles_n = (j1.N + sn - 1) / sn;
  const int64_t blocks = j0.tiles_m * j0.tiles_n + j1.tiles_m * j1.tiles_n;
  if (blocks > 0x7fffffff) return hipErrorInvalidConfiguration;
  hipLaunchKernelGGL((k_gemm_grad_pair<T, WBM, WBN, BK, VEC>), dim3((unsigned)blocks), dim3(256), 0, s, j0, j1);
  return hipGetLastError();
}

template <typename T>
static hipError_t launch_pair(const T *G, const T *A, const T *B, T *dA, T *dB, int64_t M, int64_t K, int64_t N,
                              hipStream_t s) {
  // dA (M x K) = G (M x N) . B^T ; dB (K x N) = A^T . G.
  const GemmJob j0{G, B, dA, M, N, K, 0, 0}, j1{A, G, dB, K, M, N, 0, 0};
  const int tile = auto_tile(M, K);
  const bool vec = vec_ok(G, B, N, N) && vec_ok(A, G, K, N);
  if (tile != auto_tile(K, N))  // different tile sizes: two launches
    return hipErrorNotSupported;
  constexpr int BK = sizeof(T) == 4 ? 32 : 16;
  if (tile == 1)
    return vec ? launch_pair_t<T, 4, 4, BK, true>(j0, j1, s) : launch_pair_t<T, 4, 4, BK, false>(j0, j1, s);
  // 64 x 64 tiles, 32-wide FP32 panels: on the 4096 x 4096 . 512 backward
  // pair 0.529 ms per forward + backward step, against 0.565 with 64-wide
  // panels and 0.532-0.541 with 128 x 64 tiles.
  if (tile == 2)
    return vec ? launch_pair_t<T, 2, 2, BK, true>(j0, j1, s) : launch_pair_t<T, 2, 2, BK, false>(j0, j1, s);
  return vec ? launch_pair_t<T, 1, 1, BK, true>(j0, j1, s) : launch_pair_t<T, 1, 1, BK, false>(j0, j1, s);
}

hipError_t launch_gemm_grad(moa_dtype dt, const void *G, const void *A, const void *B, void *dA, void *dB, int64_t M,
                            int64_t K, int64_t N, hipStream_t s) {
  hipError_t e = hipErrorNotSupported;
  if (M > 0 && K > 0 && N > 0) {
    if (dt == MOA_F64)
      e = launch_pair<double>((const double *)G, (const double *)A, (const double *)B, (double *)dA, (double *)dB,
                              M, K, N, s);
    else if (dt == MOA_F32)
      e = launch_pair<float>((const float *)G, (const float *)A, (const float *)B, (float *)dA, (float *)dB, M, K,
                             N, s);
  }
  if (e != hipErrorNotSupported) return e;
  // Tile sizes differ between the two products: one launch each.
  if ((e = launch_gemm(dt, false, true, G, B, dA, M, N, K, 0, s)) != hipSuccess) return e;
  return launch_gemm(dt, true, false, A, G, dB, K, M, N, 0, s);
}

}  // namespace moa
