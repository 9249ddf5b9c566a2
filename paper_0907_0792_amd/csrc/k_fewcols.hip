// Inner product with few result columns (N <= 16) and an association-
// independent fold: the contraction split over the lanes of a wave, then a
// wavefront reduction.
//
// D[i, j] = op1-fold over l of op2(A[i, l], B[l, j])   (Section I, Eq. inner)
//
// With few columns the row form (a row of B per element of A) leaves most
// lanes of a wave idle, so here the lanes share the fold over l instead. A
// workgroup owns 4 R rows of D (R per wave) and walks l in chunks of 256: the
// chunk's rows of B (256 N contiguous elements) are staged once in LDS, and
// within each span of 64 VW consecutive l (VW = elements per 16 bytes) lane q
// folds l = VW q .. VW q + VW - 1 for its R rows and all N columns, so every
// A load is one 16-byte vector per lane and 1 KiB per wave (A, the stream that
// dominates, is read once and coalesced). After the last chunk the 64 partial
// folds of each element are combined by a butterfly of cross-lane exchanges.
// The combination order differs from a sequential fold, so this path is used
// only for folds whose result does not depend on association: every int32
// fold (wrapping + and * included) and FP max/min.
#pragma clang fp contract(off)

#include <algorithm>

#include "common.hpp"
#include "internal.hpp"

namespace moa {

namespace {

constexpr int kChunk = 256;  // l per chunk

// vec: A is 16-byte aligned and K is a multiple of VW, so a lane's VW values
// are one aligned vector; otherwise they are loaded one by one.
template <typename T, int OP1, int OP2, int NC, int R>
__global__ __launch_bounds__(256) void k_fewcols(const T *__restrict__ A, const T *__restrict__ B, T *__restrict__ D,
                                                 int64_t M, int64_t K, int N, int vec) {
  constexpr int VW = 16 / (int)sizeof(T), SPAN = kWave * VW, NSPAN = kChunk / SPAN;
  typedef __attribute__((__vector_size__(16))) T vec_t;
  // Row l of a chunk sits at LDS row (l / SPAN) SPAN + (l % VW) 64 + (l % SPAN) / VW,
  // so the 64 lanes reading their u-th values read 64 consecutive rows: with
  // rows of exactly NC elements that is one contiguous block, read as 16-byte
  // vectors (a lane takes its row's NC values in NC / VW reads, and
  // neighbouring lanes read neighbouring 16 bytes).
  constexpr int SB = NC;
  constexpr int RV = (NC * (int)sizeof(T) + 15) / 16;  // 16-byte reads per row
  __shared__ __attribute__((aligned(16))) T Bs[kChunk * SB];
  const int tid = threadIdx.x, lane = tid % kWave;
  const int wave = __builtin_amdgcn_readfirstlane(tid / kWave);
  const int64_t i0 = ((int64_t)blockIdx.x * 4 + wave) * R;
  // Rows past M read row M - 1 (never stored), so every load is in bounds.
  const T *a[R];
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const int64_t i = i0 + r < M ? i0 + r : M - 1;
    a[r] = A + i * K;
  }
  T acc[R][NC];
#pragma unroll
  for (int r = 0; r < R; ++r)
#pragma unroll
    for (int c = 0; c < NC; ++c) acc[r][c] = fold_identity<OP1, T>();

  for (int64_t k0 = 0; k0 < K; k0 += kChunk) {
    const int kc = (K - k0) < kChunk ? (int)(K - k0) : kChunk;
    // A values of a full chunk are loaded first, so their latency overlaps
    // the staging of B and its barriers.
    T x[NSPAN][R][VW];
    if (kc == kChunk) {
#pragma unroll
      for (int h = 0; h < NSPAN; ++h)
#pragma unroll
        for (int r = 0; r < R; ++r) {
          const T *src = a[r] + k0 + h * SPAN + VW * lane;
          if (vec) {
            const vec_t v = *(const vec_t *)src;
#pragma unroll
            for (int u = 0; u < VW; ++u) x[h][r][u] = v[u];
          } else {
#pragma unroll
            for (int u = 0; u < VW; ++u) x[h][r][u] = src[u];
          }
        }
    }
    // Stage rows k0 .. k0 + kc - 1 of B (one contiguous block of kc N):
    // thread t takes column t % NP of rows t / NP + j 256 / NP (NP = NC
    // rounded up to a power of two, so no division by N). When N = NP and the
    // chunk is full that is element t + 256 j of the block: the loads are
    // unrolled with constant offsets and all issued before the first store.
    __syncthreads();
    {
      constexpr int NP = NC <= 1 ? 1 : NC <= 2 ? 2 : NC <= 4 ? 4 : NC <= 8 ? 8 : 16;
      constexpr int RPT = kChunk * NP / 256;  // rows per thread
      const int c = tid % NP;
      auto pos = [](int l) { return (l / SPAN) * SPAN + (l % VW) * kWave + (l % SPAN) / VW; };
      if (N == NP && kc == kChunk) {
        const T *src = B + k0 * NP + tid;
        T bv[RPT];
#pragma unroll
        for (int j = 0; j < RPT; ++j) bv[j] = src[256 * j];
#pragma unroll
        for (int j = 0; j < RPT; ++j) Bs[pos(tid / NP + j * (256 / NP)) * SB + c] = bv[j];
      } else if (c < N) {
        for (int l = tid / NP; l < kc; l += 256 / NP) Bs[pos(l) * SB + c] = B[(k0 + l) * N + c];
      }
    }
    __syncthreads();
#pragma unroll
    for (int h = 0; h < NSPAN; ++h) {
      const int l0 = h * SPAN + VW * lane;  // this lane's first l in the chunk
      if (kc == kChunk) {
#pragma unroll
        for (int u = 0; u < VW; u += 2) {  // pairs of terms (three-operand fold for int32)
          T b[2][RV * VW];
#pragma unroll
          for (int w = 0; w < 2; ++w) {
            const T *row = &Bs[(h * SPAN + (u + w) * kWave + lane) * SB];
            if constexpr (NC * sizeof(T) >= 16) {
#pragma unroll
              for (int q = 0; q < RV; ++q) {
                const vec_t v = *(const vec_t *)(row + q * VW);
#pragma unroll
                for (int e = 0; e < VW; ++e) b[w][q * VW + e] = v[e];
              }
            } else {
#pragma unroll
              for (int c = 0; c < NC; ++c) b[w][c] = row[c];
            }
          }
#pragma unroll
          for (int c = 0; c < NC; ++c)
            if (c < N) {
#pragma unroll
              for (int r = 0; r < R; ++r)
                acc[r][c] = fold_pair<OP1>(acc[r][c], apply_op<OP2>(x[h][r][u], b[0][c]),
                                           apply_op<OP2>(x[h][r][u + 1], b[1][c]));
            }
        }
      } else {
#pragma unroll
        for (int u = 0; u < VW; ++u) {
          const int l = l0 + u;
          if (l < kc) {
            T xt[R];
#pragma unroll
            for (int r = 0; r < R; ++r) xt[r] = a[r][k0 + l];
#pragma unroll
            for (int c = 0; c < NC; ++c)
              if (c < N) {
                const T bv = Bs[(h * SPAN + u * kWave + lane) * SB + c];
#pragma unroll
                for (int r = 0; r < R; ++r) acc[r][c] = apply_op<OP1>(acc[r][c], apply_op<OP2>(xt[r], bv));
              }
          }
        }
      }
    }
  }
  // Butterfly over the 64 lanes: afterwards every lane holds the full fold.
#pragma unroll
  for (int r = 0; r < R; ++r)
#pragma unroll
    for (int c = 0; c < NC; ++c)
#pragma unroll
      for (int m = kWave / 2; m >= 1; m /= 2) acc[r][c] = apply_op<OP1>(acc[r][c], __shfl_xor(acc[r][c], m));
  if (lane == 0) {
#pragma unroll
    for (int r = 0; r < R; ++r)
#pragma unroll
      for (int c = 0; c < NC; ++c)
        if (i0 + r < M && c < N) D[(i0 + r) * N + c] = acc[r][c];
  }
}

// B resident in LDS: when all of B (K rows of NC elements) fits in 128 KiB,
// one workgroup of 16 waves per CU stages it once, with the same permuted row
// placement, and then streams rows of A with no further barrier: wave groups
// of R rows are taken round-robin, each lane loading 16-byte runs of A one
// span ahead of the fold. No B chunk is re-staged per 256 l (no per-chunk
// loads, LDS stores or barriers).
constexpr int kResidentBytes = 128 * 1024;

template <typename T, int OP1, int OP2, int NC, int R>
__global__ __launch_bounds__(1024, 1) void k_fewcols_resident(const T *__restrict__ A, const T *__restrict__ B,
                                                              T *__restrict__ D, int64_t M, int K, int N) {
  constexpr int VW = 16 / (int)sizeof(T), SPAN = kWave * VW;
  constexpr int RV = (NC * (int)sizeof(T) + 15) / 16;  // 16-byte reads per staged row
  typedef __attribute__((__vector_size__(16))) T vec_t;
  __shared__ __attribute__((aligned(16))) T Bs[kResidentBytes / sizeof(T)];
  const int tid = threadIdx.x, lane = tid % kWave;
  const int wave = __builtin_amdgcn_readfirstlane(tid / kWave);
  auto pos = [](int l) { return (l / SPAN) * SPAN + (l % VW) * kWave + (l % SPAN) / VW; };
#pragma unroll 8
  for (int e = tid; e < K * NC; e += 1024) {
    const int l = e / NC, c = e % NC;
    Bs[pos(l) * NC + c] = c < N ? B[(int64_t)l * N + c] : T(0);
  }
  __syncthreads();
  const int nspan = K / SPAN;
  const int64_t groups = (M + R - 1) / R;
  for (int64_t g = (int64_t)blockIdx.x * 16 + wave; g < groups; g += (int64_t)gridDim.x * 16) {
    const T *a[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const int64_t i = g * R + r < M ? g * R + r : M - 1;  // rows past M repeat row M - 1, never stored
      a[r] = A + i * K + VW * lane;
    }
    T acc[R][NC];
#pragma unroll
    for (int r = 0; r < R; ++r)
#pragma unroll
      for (int c = 0; c < NC; ++c) acc[r][c] = fold_identity<OP1, T>();
    vec_t x[R], xn[R];
#pragma unroll
    for (int r = 0; r < R; ++r) x[r] = *(const vec_t *)a[r];
    for (int sp = 0; sp < nspan; ++sp) {
      if (sp + 1 < nspan) {
#pragma unroll
        for (int r = 0; r < R; ++r) xn[r] = *(const vec_t *)(a[r] + (sp + 1) * SPAN);
      }
#pragma unroll
      for (int u = 0; u < VW; u += 2) {
        T b[2][RV * VW];
#pragma unroll
        for (int w = 0; w < 2; ++w) {
          const T *row = &Bs[(sp * SPAN + (u + w) * kWave + lane) * NC];
          if constexpr (NC * sizeof(T) >= 16) {
#pragma unroll
            for (int q = 0; q < RV; ++q) {
              const vec_t v = *(const vec_t *)(row + q * VW);
#pragma unroll
              for (int e = 0; e < VW; ++e) b[w][q * VW + e] = v[e];
            }
          } else {
#pragma unroll
            for (int c = 0; c < NC; ++c) b[w][c] = row[c];
          }
        }
#pragma unroll
        for (int c = 0; c < NC; ++c)
          if (c < N) {
#pragma unroll
            for (int r = 0; r < R; ++r)
              acc[r][c] = fold_pair<OP1>(acc[r][c], apply_op<OP2>(x[r][u], b[0][c]), apply_op<OP2>(x[r][u + 1], b[1][c]));
          }
      }
#pragma unroll
      for (int r = 0; r < R; ++r) x[r] = xn[r];
    }
#pragma unroll
    for (int r = 0; r < R; ++r)
#pragma unroll
      for (int c = 0; c < NC; ++c)
#pragma unroll
        for (int m = kWave / 2; m >= 1; m /= 2) acc[r][c] = apply_op<OP1>(acc[r][c], __shfl_xor(acc[r][c], m));
    if (lane == 0) {
#pragma unroll
      for (int r = 0; r < R; ++r)
#pragma unroll
        for (int c = 0; c < NC; ++c)
          if (g * R + r < M && c < N) D[(g * R + r) * N + c] = acc[r][c];
    }
  }
}

int cu_count() {
  static int cached[64] = {};
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 256;
  if (cached[dev] == 0) {
    int n = 0;
    cached[dev] = (hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && n > 0) ? n : 256;
  }
  return cached[dev];
}

// Rows per wave (each staged B row, read as 16-byte vectors, feeds R terms
// per value): 4, measured on int32 (max,+) 65536 x 4096 . 4096 x 8 over ten
// back-to-back calls (0.234 ms; 2 rows: 0.247 ms).
template <typename T, int NC>
constexpr int rows_per_wave() {
  return 4;
}

template <typename T, int OP1, int OP2, int NC>
void launch_ncr(const T *A, const T *B, T *D, int64_t M, int64_t K, int64_t N, hipStream_t s) {
  constexpr int R = rows_per_wave<T, NC>();
  const int64_t blocks = (M + 4 * R - 1) / (4 * R);
  const int vec = ((uintptr_t)A % 16) == 0 && K % (16 / (int64_t)sizeof(T)) == 0;
  constexpr int64_t SPAN = kWave * (16 / (int64_t)sizeof(T));
  if (vec && K % SPAN == 0 && K * NC * (int64_t)sizeof(T) <= kResidentBytes) {
    // 16 waves per CU leave 128 registers per lane: fewer rows per wave for
    // wide (FP64, or 16-column) rows.
    constexpr int RR = (sizeof(T) * NC > 64) ? 1 : (sizeof(T) * NC > 32) ? 2 : R;
    const int64_t groups = (M + RR - 1) / RR;
    const int64_t grid = std::min<int64_t>(cu_count(), (groups + 15) / 16);
    hipLaunchKernelGGL((k_fewcols_resident<T, OP1, OP2, NC, RR>), dim3((unsigned)grid), dim3(1024), 0, s, A, B, D,
                       M, (int)K, (int)N);
    return;
  }
  hipLaunchKernelGGL((k_fewcols<T, OP1, OP2, NC, R>), dim3((unsigned)blocks), dim3(256), 0, s, A, B, D, M, K,
                     (int)N, vec);
}

template <typename T, int OP1, int OP2>
hipError_t launch_nc(const T *A, const T *B, T *D, int64_t M, int64_t K, int64_t N, hipStream_t s) {
  if ((M + 7) / 8 > 0x7fffffff) return hipErrorInvalidConfiguration;
  if (N == 1)
    launch_ncr<T, OP1, OP2, 1>(A, B, D, M, K, N, s);
  else if (N <= 4)
    launch_ncr<T, OP1, OP2, 4>(A, B, D, M, K, N, s);
  else if (N <= 8)
    launch_ncr<T, OP1, OP2, 8>(A, B, D, M, K, N, s);
  else if (N <= kFewColsMax)
    launch_ncr<T, OP1, OP2, 16>(A, B, D, M, K, N, s);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

template <typename T, int OP1>
hipError_t dispatch_op2(moa_op op2, const T *A, const T *B, T *D, int64_t M, int64_t K, int64_t N, hipStream_t s) {
  switch (op2) {
    case MOA_ADD: return launch_nc<T, OP1, MOA_ADD>(A, B, D, M, K, N, s);
    case MOA_SUB: return launch_nc<T, OP1, MOA_SUB>(A, B, D, M, K, N, s);
    case MOA_MUL: return launch_nc<T, OP1, MOA_MUL>(A, B, D, M, K, N, s);
    case MOA_MAX: return launch_nc<T, OP1, MOA_MAX>(A, B, D, M, K, N, s);
    case MOA_MIN: return launch_nc<T, OP1, MOA_MIN>(A, B, D, M, K, N, s);
    default: break;
  }
  if constexpr (T(1) / 2 == 0) {
    switch (op2) {
      case MOA_AND: return launch_nc<T, OP1, MOA_AND>(A, B, D, M, K, N, s);
      case MOA_OR: return launch_nc<T, OP1, MOA_OR>(A, B, D, M, K, N, s);
      case MOA_XOR: return launch_nc<T, OP1, MOA_XOR>(A, B, D, M, K, N, s);
      default: break;
    }
  } else {
    if (op2 == MOA_DIV) return launch_nc<T, OP1, MOA_DIV>(A, B, D, M, K, N, s);
  }
  return hipErrorInvalidValue;
}

template <typename T>
hipError_t dispatch_int(moa_op op1, moa_op op2, const T *A, const T *B, T *D, int64_t M, int64_t K, int64_t N,
                        hipStream_t s) {
  switch (op1) {
    case MOA_ADD: return dispatch_op2<T, MOA_ADD>(op2, A, B, D, M, K, N, s);
    case MOA_MUL: return dispatch_op2<T, MOA_MUL>(op2, A, B, D, M, K, N, s);
    case MOA_MAX: return dispatch_op2<T, MOA_MAX>(op2, A, B, D, M, K, N, s);
    case MOA_MIN: return dispatch_op2<T, MOA_MIN>(op2, A, B, D, M, K, N, s);
    case MOA_AND: return dispatch_op2<T, MOA_AND>(op2, A, B, D, M, K, N, s);
    case MOA_OR: return dispatch_op2<T, MOA_OR>(op2, A, B, D, M, K, N, s);
    case MOA_XOR: return dispatch_op2<T, MOA_XOR>(op2, A, B, D, M, K, N, s);
    default: break;
  }
  return hipErrorInvalidValue;
}

template <typename T>
hipError_t dispatch_fp(moa_op op1, moa_op op2, const T *A, const T *B, T *D, int64_t M, int64_t K, int64_t N,
                       hipStream_t s) {
  switch (op1) {
    case MOA_MAX: return dispatch_op2<T, MOA_MAX>(op2, A, B, D, M, K, N, s);
    case MOA_MIN: return dispatch_op2<T, MOA_MIN>(op2, A, B, D, M, K, N, s);
    default: break;
  }
  return hipErrorInvalidValue;
}

}  // namespace

bool fewcols_applies(moa_dtype dt, moa_op op1, int64_t M, int64_t K, int64_t N) {
  const bool assoc = dt == MOA_I32 || op1 == MOA_MAX || op1 == MOA_MIN;
  return assoc && N >= 1 && N <= kFewColsMax && K >= 256 && M >= 1;
}

hipError_t launch_fewcols_inner(moa_dtype dt, moa_op op1, moa_op op2, const void *A, const void *B, void *D,
                                int64_t M, int64_t K, int64_t N, hipStream_t s) {
  if (M == 0 || N == 0) return hipSuccess;
  if (!fewcols_applies(dt, op1, M, K, N)) return hipErrorInvalidValue;
  switch (dt) {
    case MOA_I32:
      return dispatch_int<int32_t>(op1, op2, (const int32_t *)A, (const int32_t *)B, (int32_t *)D, M, K, N, s);
    case MOA_F32: return dispatch_fp<float>(op1, op2, (const float *)A, (const float *)B, (float *)D, M, K, N, s);
    case MOA_F64: return dispatch_fp<double>(op1, op2, (const double *)A, (const double *)B, (double *)D, M, K, N, s);
    default: break;
  }
  return hipErrorInvalidValue;
}

}  // namespace moa
