// Matrix-core tile of the (+,*) inner product, shared by the single-product
// kernel and the persistent batch kernel.
#pragma once

#include "common.hpp"

namespace moa {

template <typename T>
struct Mfma16;

template <>
struct Mfma16<double> {
  using acc_t = doublex4;
  static __device__ __forceinline__ acc_t run(double a, double b, acc_t c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  // Output element v of lane l sits at row 4*v + l/16, column l%16.
  static __device__ __forceinline__ int row(int lane, int v) { return 4 * v + lane / 16; }
};

template <>
struct Mfma16<float> {
  using acc_t = floatx4;
  static __device__ __forceinline__ acc_t run(float a, float b, acc_t c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  // Output element v of lane l sits at row 4*(l/16) + v, column l%16.
  static __device__ __forceinline__ int row(int lane, int v) { return 4 * (lane / 16) + v; }
};

// LDS bytes of one tile's panels, for either layout of each operand
// (k-major: BK x (side + 2); row-major: side x (BK + 16 bytes)).
template <typename T, int WBM, int WBN, int BK>
constexpr int gemm_tile_lds_bytes() {
  constexpr int PA = 16 / (int)sizeof(T);
  constexpr int a = BK * (32 * WBM + 2) > 32 * WBM * (BK + PA) ? BK * (32 * WBM + 2) : 32 * WBM * (BK + PA);
  constexpr int b = BK * (32 * WBN + 2) > 32 * WBN * (BK + PA) ? BK * (32 * WBN + 2) : 32 * WBN * (BK + PA);
  return (int)sizeof(T) * (a + b);
}

// One BM x BN tile of D = A . B (BM = 32*WBM, BN = 32*WBN), computed by the
// 256 threads of a workgroup with BK-wide k panels. m0, n0: tile origin.
// GEN: A and B are the strided (P, K, Q) views of a contraction over any
// axis pair, A[i, k] = A[(i / Qa) K Qa + k Qa + i % Qa] and
// B[k, j] = B[(j / Qb) K Qb + k Qb + j % Qb]; TA, TB then only choose which
// index runs fastest across threads (TA: i, else k; TB: k, else j), so that
// neighbouring lanes read neighbouring addresses.
// SKIP: a wave issues no MFMA for its 16 x 16 blocks that lie wholly past
// M or N (small problems in a fixed tile: the matrix-core work then follows
// the problem's extents in steps of 16 instead of the tile's).
// VEC: panels are loaded as 16-byte vectors along the axis the lanes run on
// (4 FP32 or 2 FP64 per load: fewer load instructions and address
// registers). The caller guarantees 16-byte aligned A and B and extents along
// those axes that are multiples of the vector length (K for A, N for B, or M
// and K when transposed; with GEN, Qa and Qb wherever the lanes run along i
// or j), so a vector is either wholly inside the operand or wholly past its
// edge and its elements are adjacent in memory.
// I: index type. int32_t when the caller knows every offset of the tile
// (operand and result extents padded by a tile) fits in 31 bits: 32-bit
// address arithmetic takes fewer registers (small batched problems).
// smem: the panels' LDS (at least gemm_tile_lds_bytes, 16-byte aligned),
// given by the caller so that a kernel running tiles of several shapes holds
// one buffer sized for the largest instead of one per shape; gemm_tile below
// declares its own.
template <typename T, bool TA, bool TB, int WBM, int WBN, int BK = 16, bool GEN = false, bool SKIP = false,
          bool VEC = false, typename I = int64_t, bool RCL = false>
__device__ __forceinline__ void gemm_tile_at(const T *__restrict__ A, const T *__restrict__ B, T *__restrict__ D,
                                             I M, I K, I N, I m0, I n0, I Qa, I Qb, unsigned char *smem) {
  using MF = Mfma16<T>;
  using acc_t = typename MF::acc_t;
  constexpr int BM = 32 * WBM, BN = 32 * WBN;
  constexpr int PAD = 2;
  constexpr int EA = BM * BK / 256, EB = BN * BK / 256;
  constexpr int V = VEC ? 16 / (int)sizeof(T) : 1;  // elements per load
  typedef __attribute__((__vector_size__(V * sizeof(T)))) T vec_t;
  // Panel layouts. With RCL, an operand whose rows run along k in memory (A
  // as stored, or B read as stored N x K; not the strided views) is staged
  // row-major, rows of BK padded by 16 bytes: the loaded vectors are stored
  // whole (no transposing scatter of 4-byte stores, whose bank conflicts
  // stall the LDS), and a fragment is read as 16-byte vectors (below). It
  // keeps a row-major fragment's values live across steps, so it is enabled
  // only where the registers allow. Every other operand is staged k-major,
  // rows of the tile side padded by 2 elements.
  constexpr bool A_RC = RCL && !TA && !GEN, B_RC = RCL && TB && !GEN;
  constexpr int PA = 16 / (int)sizeof(T);
  constexpr int ABYTES = (int)sizeof(T) * (A_RC ? BM * (BK + PA) : BK * (BM + PAD));
  T(*As)[BM + PAD] = reinterpret_cast<T(*)[BM + PAD]>(smem);
  T(*Ar)[BK + PA] = reinterpret_cast<T(*)[BK + PA]>(smem);
  T(*Bs)[BN + PAD] = reinterpret_cast<T(*)[BN + PAD]>(smem + ABYTES);
  T(*Br)[BK + PA] = reinterpret_cast<T(*)[BK + PA]>(smem + ABYTES);

  const int tid = threadIdx.x, lane = tid % kWave, wave = __builtin_amdgcn_readfirstlane(tid / kWave);
  const int wm = wave / 2, wn = wave % 2;
  // Blocks of this wave inside the problem (all of them unless SKIP).
  int nbm = WBM, nbn = WBN;
  if constexpr (SKIP) {
    const I rm = M - (m0 + wm * (BM / 2)), rn = N - (n0 + wn * (BN / 2));
    nbm = rm <= 0 ? 0 : (rm >= 16 * WBM ? WBM : (int)((rm + 15) / 16));
    nbn = rn <= 0 ? 0 : (rn >= 16 * WBN ? WBN : (int)((rn + 15) / 16));
  }

  acc_t acc[WBM][WBN];
#pragma unroll
  for (int i = 0; i < WBM; ++i)
#pragma unroll
    for (int j = 0; j < WBN; ++j)
#pragma unroll
      for (int v = 0; v < 4; ++v) acc[i][j][v] = T(0);

  vec_t ra[EA / V], rb[EB / V];
  // GEN: the row/column part of each loaded element's address is the same for
  // every k panel; -1 marks a row or column past the edge.
  [[maybe_unused]] I abase[GEN ? EA / V : 1], bbase[GEN ? EB / V : 1];
  if constexpr (GEN) {
#pragma unroll
    for (int e = 0; e < EA / V; ++e) {
      const int f = tid + 256 * e;
      const I gm = m0 + (TA ? (f % (BM / V)) * V : f / (BK / V));
      abase[e] = gm < M ? (gm / Qa) * K * Qa + gm % Qa : -1;
    }
#pragma unroll
    for (int e = 0; e < EB / V; ++e) {
      const int f = tid + 256 * e;
      const I gn = n0 + (TB ? f / (BK / V) : (f % (BN / V)) * V);
      bbase[e] = gn < N ? (gn / Qb) * K * Qb + gn % Qb : -1;
    }
  }
  // Panel element f (vector f when VEC) of a thread: A runs along k unless TA
  // (then along i), B along j unless TB (then along k), so that neighbouring
  // lanes read neighbouring addresses.
  auto load = [&](I k0) {
#pragma unroll
    for (int e = 0; e < EA / V; ++e) {
      const int f = tid + 256 * e;
      I gm, gk;
      if constexpr (!TA) {
        gm = m0 + f / (BK / V);
        gk = k0 + (f % (BK / V)) * V;
      } else {
        gk = k0 + f / (BM / V);
        gm = m0 + (f % (BM / V)) * V;
      }
      const bool ok = gm < M && gk < K;
      if constexpr (GEN) {
        const bool in = abase[e] >= 0 && gk < K;
        if constexpr (VEC)
          ra[e] = in ? *(const vec_t *)(A + abase[e] + gk * Qa) : vec_t{};
        else
          ra[e][0] = in ? A[abase[e] + gk * Qa] : T(0);
      } else {
        const T *src = TA ? A + gk * M + gm : A + gm * K + gk;
        if constexpr (VEC)
          ra[e] = ok ? *(const vec_t *)src : vec_t{};
        else
          ra[e][0] = ok ? *src : T(0);
      }
    }
#pragma unroll
    for (int e = 0; e < EB / V; ++e) {
      const int f = tid + 256 * e;
      I gn, gk;
      if constexpr (!TB) {
        gk = k0 + f / (BN / V);
        gn = n0 + (f % (BN / V)) * V;
      } else {
        gn = n0 + f / (BK / V);
        gk = k0 + (f % (BK / V)) * V;
      }
      const bool ok = gn < N && gk < K;
      if constexpr (GEN) {
        const bool in = bbase[e] >= 0 && gk < K;
        if constexpr (VEC)
          rb[e] = in ? *(const vec_t *)(B + bbase[e] + gk * Qb) : vec_t{};
        else
          rb[e][0] = in ? B[bbase[e] + gk * Qb] : T(0);
      } else {
        const T *src = TB ? B + gn * K + gk : B + gk * N + gn;
        if constexpr (VEC)
          rb[e] = ok ? *(const vec_t *)src : vec_t{};
        else
          rb[e][0] = ok ? *src : T(0);
      }
    }
  };
  auto store = [&]() {
#pragma unroll
    for (int e = 0; e < EA / V; ++e) {
      const int f = tid + 256 * e;
      if constexpr (A_RC) {
        *(vec_t *)&Ar[f / (BK / V)][(f % (BK / V)) * V] = ra[e];
      } else {
#pragma unroll
        for (int u = 0; u < V; ++u) {
          if constexpr (!TA)
            As[(f % (BK / V)) * V + u][f / (BK / V)] = ra[e][u];
          else
            As[f / (BM / V)][(f % (BM / V)) * V + u] = ra[e][u];
        }
      }
    }
#pragma unroll
    for (int e = 0; e < EB / V; ++e) {
      const int f = tid + 256 * e;
      if constexpr (B_RC) {
        *(vec_t *)&Br[f / (BK / V)][(f % (BK / V)) * V] = rb[e];
      } else {
#pragma unroll
        for (int u = 0; u < V; ++u) {
          if constexpr (!TB)
            Bs[f / (BN / V)][(f % (BN / V)) * V + u] = rb[e][u];
          else
            Bs[(f % (BK / V)) * V + u][f / (BK / V)] = rb[e][u];
        }
      }
    }
  };

  // The panel's BK / 4 matrix-core steps assign k to lanes so that a
  // row-major operand's fragment is contiguous: in step s the lanes 16 g + r
  // (g = 0..3) supply k = g BK / 4 + s, so lane (r, g) needs k = g BK / 4 ..
  // g BK / 4 + BK / 4 - 1 of its row, read HS at a time as one 16-byte vector
  // (any assignment gives the same sum, as long as A and B use the same one).
  // k-major operands are read one element per step, as before.
  constexpr int KS = BK / 4, HS = 16 / (int)sizeof(T);
  typedef __attribute__((__vector_size__(16))) T v16_t;
  auto compute = [&]() {
    if constexpr (!A_RC && !B_RC) {
      // Both k-major: step k4 / 4 takes k = k4 + l / 16 in lane l.
#pragma unroll
      for (int k4 = 0; k4 < BK; k4 += 4) {
        T a[WBM], b[WBN];
#pragma unroll
        for (int i = 0; i < WBM; ++i) a[i] = As[k4 + lane / 16][wm * (BM / 2) + i * 16 + lane % 16];
#pragma unroll
        for (int j = 0; j < WBN; ++j) b[j] = Bs[k4 + lane / 16][wn * (BN / 2) + j * 16 + lane % 16];
#pragma unroll
        for (int i = 0; i < WBM; ++i)
#pragma unroll
          for (int j = 0; j < WBN; ++j)
            if (!SKIP || (i < nbm && j < nbn)) acc[i][j] = MF::run(a[i], b[j], acc[i][j]);
      }
      return;
    }
    const int r = lane % 16, g = lane / 16;
#pragma unroll
    for (int c = 0; c < KS / HS; ++c) {
      [[maybe_unused]] v16_t av[A_RC ? WBM : 1], bv[B_RC ? WBN : 1];
      if constexpr (A_RC) {
#pragma unroll
        for (int i = 0; i < WBM; ++i) av[i] = *(const v16_t *)&Ar[wm * (BM / 2) + i * 16 + r][g * KS + c * HS];
      }
      if constexpr (B_RC) {
#pragma unroll
        for (int j = 0; j < WBN; ++j) bv[j] = *(const v16_t *)&Br[wn * (BN / 2) + j * 16 + r][g * KS + c * HS];
      }
#pragma unroll
      for (int t = 0; t < HS; ++t) {
        const int kk = g * KS + c * HS + t;
        T a[WBM], b[WBN];
#pragma unroll
        for (int i = 0; i < WBM; ++i) {
          if constexpr (A_RC)
            a[i] = av[i][t];
          else
            a[i] = As[kk][wm * (BM / 2) + i * 16 + r];
        }
#pragma unroll
        for (int j = 0; j < WBN; ++j) {
          if constexpr (B_RC)
            b[j] = bv[j][t];
          else
            b[j] = Bs[kk][wn * (BN / 2) + j * 16 + r];
        }
#pragma unroll
        for (int i = 0; i < WBM; ++i)
#pragma unroll
          for (int j = 0; j < WBN; ++j)
            if (!SKIP || (i < nbm && j < nbn)) acc[i][j] = MF::run(a[i], b[j], acc[i][j]);
      }
    }
  };

  // The next panel is fetched into registers while this one is multiplied.
  const I nk = (K + BK - 1) / BK;
  if (nk > 0) load(0);
  for (I kt = 0; kt < nk; ++kt) {
    __syncthreads();
    store();
    __syncthreads();
    if (kt + 1 < nk) load((kt + 1) * BK);
    compute();
  }
  __syncthreads();  // LDS is reused by the caller's next tile
#pragma unroll
  for (int i = 0; i < WBM; ++i)
#pragma unroll
    for (int j = 0; j < WBN; ++j)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const I gm = m0 + wm * (BM / 2) + i * 16 + MF::row(lane, v);
        const I gn = n0 + wn * (BN / 2) + j * 16 + lane % 16;
        if (gm < M && gn < N) D[gm * N + gn] = acc[i][j][v];
      }
}

template <typename T, bool TA, bool TB, int WBM, int WBN, int BK = 16, bool GEN = false, bool SKIP = false,
          bool VEC = false, typename I = int64_t, bool RCL = false>
__device__ __forceinline__ void gemm_tile(const T *__restrict__ A, const T *__restrict__ B, T *__restrict__ D,
                                          I M, I K, I N, I m0, I n0, I Qa = 1, I Qb = 1) {
  __shared__ __attribute__((aligned(16))) unsigned char smem[gemm_tile_lds_bytes<T, WBM, WBN, BK>()];
  gemm_tile_at<T, TA, TB, WBM, WBN, BK, GEN, SKIP, VEC, I, RCL>(A, B, D, M, K, N, m0, n0, Qa, Qb, smem);
}

}  // namespace moa
