// Generic (op1, op2) inner product on the vector ALUs: the tile kernel and
// its launch for one (dtype, op1). Included by the units that instantiate
// simt_fold for their dtypes and folds (split over several units so they
// compile in parallel); the scheme is described in k_simt.hip.
#pragma once
#pragma clang fp contract(off)

#include "common.hpp"
#include "internal.hpp"

namespace moa {

template <typename T, int OP1, int OP2, int TM, int TN, bool VEC>
__global__ __launch_bounds__(256) void k_simt_inner(const T *__restrict__ A, const T *__restrict__ B,
                                                    T *__restrict__ D, int64_t M, int64_t K, int64_t N,
                                                    int64_t tiles_m, int64_t tiles_n, int64_t Qa, int64_t Qb) {
  constexpr int BM = 16 * TM, BN = 16 * TN, BK = 16;
  constexpr int PAD = 16 / sizeof(T);
  // Staged elements per thread and panel; V per load (VEC: 16 bytes).
  constexpr int EA = BM * BK / 256, EB = BN * BK / 256, V = VEC ? 16 / (int)sizeof(T) : 1;
  static_assert(EA % V == 0 && EB % V == 0, "vector staging needs whole vectors per thread");
  typedef __attribute__((__vector_size__(V * sizeof(T)))) T vec_t;
  __shared__ __attribute__((aligned(16))) T As[BK][BM + PAD];
  __shared__ __attribute__((aligned(16))) T Bs[BK][BN];

  int64_t tm, tn;
  const int64_t nt = tiles_m * tiles_n;
  grouped_tile(xcd_swizzle(blockIdx.x, nt), tiles_m, tiles_n, 8, tm, tn);
  const int64_t m0 = tm * BM, n0 = tn * BN;
  const int tid = threadIdx.x;
  const int tx = tid % 16, ty = tid / 16;

  T acc[TM][TN];
#pragma unroll
  for (int i = 0; i < TM; ++i)
#pragma unroll
    for (int j = 0; j < TN; ++j) acc[i][j] = fold_identity<OP1, T>();

  // Staging of A[m0:m0+BM, k0:k0+BK] (into As[k][m], transposed) and
  // B[k0:k0+BK, n0:n0+BN] (into Bs[k][n]). Slot p of a thread covers row r,
  // column c of the panel; lanes run along k for A and along j for B, except
  // for strided views where the other index is contiguous (A: Qa > 1, lanes
  // along i; B: Qb = 1, lanes along k). The view tests are wave-uniform and
  // sit outside the unrolled loops.
  const bool a_plain = VEC || Qa == 1, b_plain = VEC || Qb == N;
  auto a_slot = [&](int p, int &r, int &c) {
    const int idx = tid + 256 * p;
    if (a_plain) {
      r = idx / (BK / V);
      c = (idx % (BK / V)) * V;
    } else {
      r = idx % BM;
      c = idx / BM;
    }
  };
  auto b_slot = [&](int p, int &r, int &c) {
    const int idx = tid + 256 * p;
    if (b_plain || Qb != 1) {
      r = idx / (BN / V);
      c = (idx % (BN / V)) * V;
    } else {
      r = idx % BK;
      c = idx / BK;
    }
  };
  vec_t ra[EA / V], rb[EB / V];
  auto load = [&](int64_t k0) {
    if constexpr (VEC) {
#pragma unroll
      for (int p = 0; p < EA / V; ++p) {
        int r, c;
        a_slot(p, r, c);
        const int64_t gm = m0 + r, gk = k0 + c;
        ra[p] = (gm < M && gk < K) ? *(const vec_t *)(A + gm * K + gk) : vec_t{};
      }
#pragma unroll
      for (int p = 0; p < EB / V; ++p) {
        int r, c;
        b_slot(p, r, c);
        const int64_t gk = k0 + r, gn = n0 + c;
        rb[p] = (gk < K && gn < N) ? *(const vec_t *)(B + gk * N + gn) : vec_t{};
      }
    } else {
      if (Qa == 1) {
#pragma unroll
        for (int p = 0; p < EA; ++p) {
          int r, c;
          a_slot(p, r, c);
          const int64_t gm = m0 + r, gk = k0 + c;
          ra[p][0] = (gm < M && gk < K) ? A[gm * K + gk] : T(0);
        }
      } else {
#pragma unroll
        for (int p = 0; p < EA; ++p) {
          int r, c;
          a_slot(p, r, c);
          const int64_t gm = m0 + r, gk = k0 + c;
          ra[p][0] = (gm < M && gk < K) ? A[(gm / Qa) * K * Qa + gk * Qa + gm % Qa] : T(0);
        }
      }
      if (Qb == N) {
#pragma unroll
        for (int p = 0; p < EB; ++p) {
          int r, c;
          b_slot(p, r, c);
          const int64_t gk = k0 + r, gn = n0 + c;
          rb[p][0] = (gk < K && gn < N) ? B[gk * N + gn] : T(0);
        }
      } else {
#pragma unroll
        for (int p = 0; p < EB; ++p) {
          int r, c;
          b_slot(p, r, c);
          const int64_t gk = k0 + r, gn = n0 + c;
          rb[p][0] = (gk < K && gn < N) ? B[(gn / Qb) * K * Qb + gk * Qb + gn % Qb] : T(0);
        }
      }
    }
  };
  auto store = [&]() {
#pragma unroll
    for (int p = 0; p < EA / V; ++p) {
      int r, c;
      a_slot(p, r, c);
#pragma unroll
      for (int u = 0; u < V; ++u) As[c + u][r] = ra[p][u];
    }
#pragma unroll
    for (int p = 0; p < EB / V; ++p) {
      int r, c;
      b_slot(p, r, c);
      if constexpr (VEC)
        *(vec_t *)&Bs[r][c] = rb[p];
      else
        Bs[r][c] = rb[p][0];
    }
  };

  if (K > 0) load(0);
  for (int64_t k0 = 0; k0 < K; k0 += BK) {
    store();
    __syncthreads();
    if (k0 + BK < K) load(k0 + BK);
    const int kmax = (K - k0) < BK ? (int)(K - k0) : BK;
    if (kmax == BK && fold_reassociable<OP1, T>()) {
#pragma unroll
      for (int kk = 0; kk < BK; kk += 2) {
        T a0[TM], b0[TN], a1[TM], b1[TN];
#pragma unroll
        for (int i = 0; i < TM; ++i) {
          a0[i] = As[kk][ty * TM + i];
          a1[i] = As[kk + 1][ty * TM + i];
        }
#pragma unroll
        for (int j = 0; j < TN; ++j) {
          b0[j] = Bs[kk][tx * TN + j];
          b1[j] = Bs[kk + 1][tx * TN + j];
        }
#pragma unroll
        for (int i = 0; i < TM; ++i)
#pragma unroll
          for (int j = 0; j < TN; ++j)
            acc[i][j] = fold_pair<OP1>(acc[i][j], apply_op<OP2>(a0[i], b0[j]), apply_op<OP2>(a1[i], b1[j]));
      }
    } else if (kmax == BK) {
#pragma unroll
      for (int kk = 0; kk < BK; ++kk) {
        T a[TM], b[TN];
#pragma unroll
        for (int i = 0; i < TM; ++i) a[i] = As[kk][ty * TM + i];
#pragma unroll
        for (int j = 0; j < TN; ++j) b[j] = Bs[kk][tx * TN + j];
#pragma unroll
        for (int i = 0; i < TM; ++i)
#pragma unroll
          for (int j = 0; j < TN; ++j) acc[i][j] = apply_op<OP1>(acc[i][j], apply_op<OP2>(a[i], b[j]));
      }
    } else {
      for (int kk = 0; kk < kmax; ++kk) {
        T a[TM], b[TN];
#pragma unroll
        for (int i = 0; i < TM; ++i) a[i] = As[kk][ty * TM + i];
#pragma unroll
        for (int j = 0; j < TN; ++j) b[j] = Bs[kk][tx * TN + j];
#pragma unroll
        for (int i = 0; i < TM; ++i)
#pragma unroll
          for (int j = 0; j < TN; ++j) acc[i][j] = apply_op<OP1>(acc[i][j], apply_op<OP2>(a[i], b[j]));
      }
    }
    __syncthreads();
  }

#pragma unroll
  for (int i = 0; i < TM; ++i) {
    const int64_t gm = m0 + ty * TM + i;
    if (gm >= M) continue;
#pragma unroll
    for (int j = 0; j < TN; ++j) {
      const int64_t gn = n0 + tx * TN + j;
      if (gn < N) D[gm * N + gn] = acc[i][j];
    }
  }
}

template <typename T, int OP1, int OP2>
static hipError_t launch_tiles(const T *A, const T *B, T *D, int64_t M, int64_t K, int64_t N, int tile,
                               int64_t Qa, int64_t Qb, hipStream_t s) {
  // 16-byte staging loads: plain layout, aligned operands, rows of A and B
  // whole vectors (then a vector is wholly inside or wholly past an edge).
  constexpr int64_t V = 16 / sizeof(T);
  const bool vec = Qa == 1 && Qb == N && (uintptr_t)A % 16 == 0 && (uintptr_t)B % 16 == 0 && K % V == 0 &&
                   N % V == 0;
  int64_t tm, tn;
  if (tile == 8) {
    tm = (M + 127) / 128;
    tn = (N + 127) / 128;
    if (vec)
      hipLaunchKernelGGL((k_simt_inner<T, OP1, OP2, 8, 8, true>), dim3((unsigned)(tm * tn)), dim3(256), 0, s, A, B, D,
                         M, K, N, tm, tn, Qa, Qb);
    else
      hipLaunchKernelGGL((k_simt_inner<T, OP1, OP2, 8, 8, false>), dim3((unsigned)(tm * tn)), dim3(256), 0, s, A, B,
                         D, M, K, N, tm, tn, Qa, Qb);
  } else if (tile == 4) {
    tm = (M + 63) / 64;
    tn = (N + 63) / 64;
    if (vec)
      hipLaunchKernelGGL((k_simt_inner<T, OP1, OP2, 4, 4, true>), dim3((unsigned)(tm * tn)), dim3(256), 0, s, A, B, D,
                         M, K, N, tm, tn, Qa, Qb);
    else
      hipLaunchKernelGGL((k_simt_inner<T, OP1, OP2, 4, 4, false>), dim3((unsigned)(tm * tn)), dim3(256), 0, s, A, B,
                         D, M, K, N, tm, tn, Qa, Qb);
  } else {
    // 32 x 32 blocks stage 2 elements per thread: fewer than one vector.
    tm = (M + 31) / 32;
    tn = (N + 31) / 32;
    hipLaunchKernelGGL((k_simt_inner<T, OP1, OP2, 2, 2, false>), dim3((unsigned)(tm * tn)), dim3(256), 0, s, A, B, D,
                       M, K, N, tm, tn, Qa, Qb);
  }
  return hipGetLastError();
}

// D = A (op1 . op2) B for one dtype and fold, any element operation.
template <typename T, int OP1>
hipError_t simt_fold(moa_op op2, const T *A, const T *B, T *D, int64_t M, int64_t K, int64_t N, int tile,
                               int64_t Qa, int64_t Qb, hipStream_t s) {
  switch (op2) {
    case MOA_ADD: return launch_tiles<T, OP1, MOA_ADD>(A, B, D, M, K, N, tile, Qa, Qb, s);
    case MOA_SUB: return launch_tiles<T, OP1, MOA_SUB>(A, B, D, M, K, N, tile, Qa, Qb, s);
    case MOA_MUL: return launch_tiles<T, OP1, MOA_MUL>(A, B, D, M, K, N, tile, Qa, Qb, s);
    case MOA_MAX: return launch_tiles<T, OP1, MOA_MAX>(A, B, D, M, K, N, tile, Qa, Qb, s);
    case MOA_MIN: return launch_tiles<T, OP1, MOA_MIN>(A, B, D, M, K, N, tile, Qa, Qb, s);
    default: break;
  }
  if constexpr (T(1) / 2 == 0) {
    switch (op2) {
      case MOA_AND: return launch_tiles<T, OP1, MOA_AND>(A, B, D, M, K, N, tile, Qa, Qb, s);
      case MOA_OR: return launch_tiles<T, OP1, MOA_OR>(A, B, D, M, K, N, tile, Qa, Qb, s);
      case MOA_XOR: return launch_tiles<T, OP1, MOA_XOR>(A, B, D, M, K, N, tile, Qa, Qb, s);
      default: break;
    }
  } else {
    if (op2 == MOA_DIV) return launch_tiles<T, OP1, MOA_DIV>(A, B, D, M, K, N, tile, Qa, Qb, s);
  }
  return hipErrorInvalidValue;
}

}  // namespace moa
