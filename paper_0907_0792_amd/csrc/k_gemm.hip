// (+,*) inner product on the matrix cores: D (M x N) = A (M x K) . B (K x N).
//
// The (+,*) case of Eq. inner (Section I), which the paper notes is the
// standard matrix product, for FP64 (v_mfma_f64_16x16x4_f64) and FP32
// (v_mfma_f32_16x16x4_f32). Any rank reaches this kernel as the flattened
// M x K and K x N views.
//
// Workgroup = 4 waves (2 x 2), each owning a (16*WBM) x (16*WBN) block of D
// as WBM x WBN 16x16 accumulator tiles. A and B panels of BK = 16 are staged
// in LDS (k-major, so one fragment read is 16 contiguous elements per k row);
// the next panel is fetched into registers while the current one is
// multiplied. trans_a / trans_b read A stored K x M or B stored N x K, which
// is how the backward pass contracts over permuted axes without a transposed
// copy.
#include "common.hpp"
#include "gemm_tile.hpp"
#include "internal.hpp"

namespace moa {

template <typename T, bool TA, bool TB, int WBM, int WBN>
__global__ __launch_bounds__(256, 2) void k_gemm(const T *__restrict__ A, const T *__restrict__ B, T *__restrict__ D,
                                                  int64_t M, int64_t K, int64_t N, int64_t tiles_m,
                                                  int64_t tiles_n) {
  int64_t tm, tn;
  grouped_tile(xcd_swizzle(blockIdx.x, tiles_m * tiles_n), tiles_m, tiles_n, 8, tm, tn);
  gemm_tile<T, TA, TB, WBM, WBN>(A, B, D, M, K, N, tm * 32 * WBM, tn * 32 * WBN);
}

template <typename T, bool TA, bool TB>
static hipError_t launch_t(const T *A, const T *B, T *D, int64_t M, int64_t K, int64_t N, int tile, hipStream_t s) {
  if (tile == 0) {
    const int64_t big = ((M + 127) / 128) * ((N + 127) / 128);
    tile = big >= 512 ? 1 : 2;
  }
  if (tile == 1) {
    const int64_t tmn = (M + 127) / 128, tnn = (N + 127) / 128;
    if (tmn * tnn > 0x7fffffff) return hipErrorInvalidConfiguration;
    hipLaunchKernelGGL((k_gemm<T, TA, TB, 4, 4>), dim3((unsigned)(tmn * tnn)), dim3(256), 0, s, A, B, D, M, K, N,
                       tmn, tnn);
  } else {
    const int64_t tmn = (M + 63) / 64, tnn = (N + 63) / 64;
    if (tmn * tnn > 0x7fffffff) return hipErrorInvalidConfiguration;
    hipLaunchKernelGGL((k_gemm<T, TA, TB, 2, 2>), dim3((unsigned)(tmn * tnn)), dim3(256), 0, s, A, B, D, M, K, N,
                       tmn, tnn);
  }
  return hipGetLastError();
}

template <typename T>
static hipError_t launch_tt(bool ta, bool tb, const T *A, const T *B, T *D, int64_t M, int64_t K, int64_t N, int tile,
                            hipStream_t s) {
  if (!ta && !tb) return launch_t<T, false, false>(A, B, D, M, K, N, tile, s);
  if (ta && !tb) return launch_t<T, true, false>(A, B, D, M, K, N, tile, s);
  if (!ta && tb) return launch_t<T, false, true>(A, B, D, M, K, N, tile, s);
  return launch_t<T, true, true>(A, B, D, M, K, N, tile, s);
}

hipError_t launch_gemm(moa_dtype dt, bool trans_a, bool trans_b, const void *A, const void *B, void *D, int64_t M,
                       int64_t K, int64_t N, int tile, hipStream_t s) {
  if (M == 0 || N == 0) return hipSuccess;
  if (dt == MOA_F64)
    return launch_tt<double>(trans_a, trans_b, (const double *)A, (const double *)B, (double *)D, M, K, N, tile, s);
  if (dt == MOA_F32)
    return launch_tt<float>(trans_a, trans_b, (const float *)A, (const float *)B, (float *)D, M, K, N, tile, s);
  return hipErrorInvalidValue;
}

}  // namespace moa
