// Batches of uneven (+,*) inner products in one persistent launch.
//
// Each problem i is the (+,*) case of Eq. inner (Section I) on its own
// flattened M_i x K_i . K_i x N_i view. The batch is cut into work items
// (one output tile of one problem each), and a persistent grid (as many
// workgroups as fit on the GPU at once) runs them: at build time the items
// are dealt to the workgroups by the longest-processing-time rule on an
// estimated cost, so the workgroups finish close together. The launch has no
// state between replays, so the captured graph replays as is.
//
// Tile variants (per problem, from the tile table):
//   0: 32 x 32 tiles (one 16 x 16 MFMA block per wave)
//   1: 64 x 64 tiles (2 x 2 blocks per wave)
// The table maps (M, N, K) size buckets to a variant; moa_batch_autotune
// fills it by timing both variants on synthetic problems of each bucket.
// FP32 batches whose operands allow 32-bit byte offsets run the LDS-fed
// tile (batch_tile_lds16: buffer loads straight into an LDS ring); FP64 and
// larger FP32 batches run the register-staged tile of gemm_tile.hpp.
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <mutex>
#include <numeric>
#include <queue>
#include <random>
#include <string>
#include <vector>

#include "common.hpp"
#include "gemm_tile.hpp"
#include "internal.hpp"

namespace moa {
moa_status set_error(moa_status st, const char *msg);
moa_status validate_inner(moa_shape a, moa_shape b, int64_t *M, int64_t *K, int64_t *N);
}  // namespace moa

struct moa_batch {
  moa_dtype dt;
  int32_t n;
  int64_t items;
  moa::BatchItem *d_items;
  int64_t *d_first;  // grid + 1 offsets: workgroup g runs items [d_first[g], d_first[g + 1])
  hipGraph_t graph;
  hipGraphExec_t exec;
  int grid;
  bool idx32;  // every tile offset fits in 31 bits: 32-bit index arithmetic
  int kind;    // kernel: 0 LDS-fed FP32, 1 FP32 64-bit index, 2-3 FP64 (32/64-bit index)
};

namespace moa {
namespace {

constexpr int kVariants = 2;
constexpr int kTileSide[kVariants] = {32, 64};

// Size buckets: M and N split at 32, K at 128.
int bucket_of(int64_t M, int64_t N, int64_t K) {
  return (M > 32 ? 4 : 0) + (N > 32 ? 2 : 0) + (K > 128 ? 1 : 0);
}
constexpr int kBuckets = 8;

std::mutex g_table_mu;
// Default: 64 x 64 everywhere (with blocks past the edge skipped, the larger
// tile wins on the 10,000-problem mixed workload: 0.281 vs 0.430 ms for 32).
int g_table[kBuckets] = {1, 1, 1, 1, 1, 1, 1, 1};

// Register-staged tiles (FP64 batches, and FP32 batches whose offsets do not
// fit the LDS-fed tile below). I: index type of the tile arithmetic (int32_t
// when every offset of every problem, padded by a tile, fits in 31 bits:
// fewer registers, one more workgroup per CU).
template <typename T, typename I>
__global__ __launch_bounds__(256, 2) void k_batch(const BatchItem *__restrict__ items,
                                                   const int64_t *__restrict__ first) {
  // Workgroup g runs items first[g] .. first[g + 1] - 1 (its share, fixed at
  // build time). The next item's record is requested before this item's tile
  // starts, so its latency is hidden. One LDS buffer, sized for the larger
  // tile, serves both.
  __shared__ __attribute__((aligned(16))) unsigned char smem[gemm_tile_lds_bytes<T, 2, 2, 16>()];
  int64_t it = first[blockIdx.x];
  const int64_t end = first[blockIdx.x + 1];
  if (it >= end) return;
  BatchItem w = items[it];
  for (; it < end; ++it) {
    const BatchItem wn = items[it + 1 < end ? it + 1 : it];  // uniform: a scalar load
    const T *a = (const T *)w.A, *b = (const T *)w.B;
    T *d = (T *)w.D;
    // SKIP: blocks past the problem's edge issue no MFMA, so the matrix-core
    // work follows M and N in steps of 16 rather than the tile side.
    if (w.tile == 0)
      gemm_tile_at<T, false, false, 1, 1, 16, false, true, false, I>(a, b, d, w.M, w.K, w.N, w.m0, w.n0, 1, 1, smem);
    else
      gemm_tile_at<T, false, false, 2, 2, 16, false, true, false, I>(a, b, d, w.M, w.K, w.N, w.m0, w.n0, 1, 1, smem);
    w = wn;
  }
}

// FP32 tiles fed by buffer loads straight into LDS (32-bit offsets: used
// when every problem's A and B stay below 2^31 bytes and every tile offset
// fits in 31 bits). Nothing is staged through registers, so NS - 1 k panels
// of 16 are in flight per workgroup at no register cost; one barrier per
// panel. Elements past M, N or K get an offset past the buffer's size, and
// the buffer range check returns zero for them.
// Three panels: six workgroups per CU (LDS-bound), two panels in flight
// each. History on the 10,000-problem FP32 workload (same box per pair):
// loading 4 bytes per lane (four 256-byte rows per load, A blocks padded
// to 68 words) 0.2256 ms against 0.2343 with four panels and 0.243-0.246 ms
// for the register-staged tile; A fragment-ordered by 4-byte lanes (each
// load touching 16 rows) 0.281-0.287 ms; 16 bytes per lane (below)
// 0.2147-0.2173 ms against 0.2237-0.2277 ms for 4 bytes per lane, and
// 0.2385-0.2415 ms with four panels (five workgroups per CU).
constexpr int kLdsStages = 3;
constexpr int kLdsStageWords = 2 * 4 * 256;  // A then B: four 16 x 16 blocks each

// s_waitcnt immediate that waits until at most n vector-memory operations
// are outstanding (n < 64) and leaves the other counters alone.
constexpr int vmcnt_lds(int n) { return 0x0F70 | (n & 15) | ((n >> 4) << 14); }

// The tile is fed by 16-byte buffer loads: one instruction moves a whole
// 16 x 16 block (1 KiB). A block: lane l loads
// A[16 ib + l % 16][k0 + 4 (l / 16) .. + 3], which lands in 16-byte slot l,
// so word 64 ks + 4 i + c holds A[16 ib + i][k0 + 4 ks + c]: the fragment
// read of lane i + 16 c touches 64 different banks. B block: lane l loads
// B[k0 + l / 4][16 jb + 4 (l % 4) .. + 3], so word 16 k + j holds B[k0 + k][j]
// and the fragment word 64 ks + 16 c + j is again conflict-free. A 4-element
// run is loaded whole or not at all, so the last k panel (where runs may
// cross K, or for B the end of the buffer) loads the same layout with four
// 4-byte loads per block and masks each element: instruction t has lane l
// fill word 64 t + l. B columns past N inside a run hold other data, which
// reaches only D columns past N, which are not stored.
template <int WB, int NS>
__device__ __forceinline__ void batch_tile_lds16(const BatchItem &w, float *lds) {
  constexpr int NB = 2 * WB;                // 16-wide blocks per tile side
  constexpr int ASZ = 4 * 256;              // A words per stage (sized for WB = 2)
  constexpr int STAGE = kLdsStageWords;     // then B
  constexpr int BPW = NB / 2;               // blocks per wave per panel
  constexpr uint32_t kOut = 0x80000000u;    // an offset past every buffer
  using MF = Mfma16<float>;
  typedef __attribute__((address_space(3))) void *lds_ptr;
  const int lane = threadIdx.x % kWave, wave = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
  const int wm = wave / 2, wn = wave % 2;
  const int M = w.M, K = w.K, N = w.N, m0 = w.m0, n0 = w.n0;
  const __amdgpu_buffer_rsrc_t ra =
      __builtin_amdgcn_make_buffer_rsrc((void *)w.A, (short)0, (int)((uint32_t)M * (uint32_t)K * 4u), 0x00020000);
  const __amdgpu_buffer_rsrc_t rb =
      __builtin_amdgcn_make_buffer_rsrc((void *)w.B, (short)0, (int)((uint32_t)K * (uint32_t)N * 4u), 0x00020000);
  const int nk = (K + 15) / 16;
  // One block's loads for panel kt into stage buffer st (A or B fixed at
  // compile time, so each load names its descriptor directly).
  auto issue_block = [&]<bool ISA>(float *st, int blk, int kt) {
    const int k0 = 16 * kt;
    float *dst = st + (ISA ? 0 : ASZ) + blk * 256;
    if (kt + 1 < nk) {
      uint32_t off;
      if constexpr (ISA) {
        const int row = m0 + 16 * blk + lane % 16, k = k0 + 4 * (lane / 16);
        off = row < M ? ((uint32_t)row * (uint32_t)K + (uint32_t)k) * 4u : kOut;
      } else {
        const int k = k0 + lane / 4, col = n0 + 16 * blk + 4 * (lane % 4);
        off = col < N ? ((uint32_t)k * (uint32_t)N + (uint32_t)col) * 4u : kOut;
      }
      __builtin_amdgcn_raw_ptr_buffer_load_lds(ISA ? ra : rb, (lds_ptr)dst, 16, off, 0, 0, 0);
    } else {
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        uint32_t off;
        if constexpr (ISA) {
          const int row = m0 + 16 * blk + lane / 4, k = k0 + 4 * t + lane % 4;
          off = (row < M && k < K) ? ((uint32_t)row * (uint32_t)K + (uint32_t)k) * 4u : kOut;
        } else {
          const int k = k0 + 4 * t + lane / 16, col = n0 + 16 * blk + lane % 16;
          off = (k < K && col < N) ? ((uint32_t)k * (uint32_t)N + (uint32_t)col) * 4u : kOut;
        }
        __builtin_amdgcn_raw_ptr_buffer_load_lds(ISA ? ra : rb, (lds_ptr)(dst + 64 * t), 4, off, 0, 0, 0);
      }
    }
  };
  // Blocks of this wave: with 4 blocks a side, A block `wave` and B block
  // `wave`; with 2, waves 0-1 take the A blocks and waves 2-3 the B blocks.
  auto issue = [&](int buf, int kt) {
    float *st = lds + buf * STAGE;
    if constexpr (NB == 4) {
      issue_block.template operator()<true>(st, wave, kt);
      issue_block.template operator()<false>(st, wave, kt);
    } else {
      if (wave < 2)
        issue_block.template operator()<true>(st, wave, kt);
      else
        issue_block.template operator()<false>(st, wave - 2, kt);
    }
  };
  // Blocks of this wave inside the problem: no MFMA for the others.
  const int rm = M - (m0 + wm * 16 * WB), rn = N - (n0 + wn * 16 * WB);
  const int nbm = rm <= 0 ? 0 : (rm >= 16 * WB ? WB : (rm + 15) / 16);
  const int nbn = rn <= 0 ? 0 : (rn >= 16 * WB ? WB : (rn + 15) / 16);
  floatx4 acc[WB][WB];
#pragma unroll
  for (int i = 0; i < WB; ++i)
#pragma unroll
    for (int j = 0; j < WB; ++j) acc[i][j] = floatx4{0.f, 0.f, 0.f, 0.f};
  const int fi = lane % 16, fc = lane / 16;

#pragma unroll
  for (int st = 0; st < NS - 1; ++st)
    if (st < nk) issue(st, st);
  for (int kt = 0; kt < nk; ++kt) {
    // This wave's loads of panel kt are done once at most the later panels'
    // loads are outstanding (counted at BPW each; the last panel issues
    // more, so near the end the wait is stricter than needed); the barrier
    // then makes every wave's part visible and frees the buffer of panel
    // kt - 1.
    if (kt + NS - 2 < nk)
      __builtin_amdgcn_s_waitcnt(vmcnt_lds(BPW * (NS - 2)));
    else
      __builtin_amdgcn_s_waitcnt(vmcnt_lds(0));
    __builtin_amdgcn_s_barrier();
    if (kt + NS - 1 < nk) issue((kt + NS - 1) % NS, kt + NS - 1);
    const float *stage = lds + (kt % NS) * STAGE;
#pragma unroll
    for (int ks = 0; ks < 4; ++ks) {
      float a[WB], b[WB];
#pragma unroll
      for (int i = 0; i < WB; ++i) a[i] = stage[(wm * WB + i) * 256 + 64 * ks + 4 * fi + fc];
#pragma unroll
      for (int j = 0; j < WB; ++j) b[j] = stage[ASZ + (wn * WB + j) * 256 + 64 * ks + 16 * fc + fi];
#pragma unroll
      for (int i = 0; i < WB; ++i)
#pragma unroll
        for (int j = 0; j < WB; ++j)
          if (i < nbm && j < nbn) acc[i][j] = MF::run(a[i], b[j], acc[i][j]);
    }
  }
  // Every wave is done with the panels before the next item's loads reuse them.
  __builtin_amdgcn_s_barrier();
#pragma unroll
  for (int i = 0; i < WB; ++i)
#pragma unroll
    for (int j = 0; j < WB; ++j)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int gm = m0 + (wm * WB + i) * 16 + MF::row(lane, v);
        const int gn = n0 + (wn * WB + j) * 16 + lane % 16;
        if (gm < M && gn < N) ((float *)w.D)[(int64_t)gm * N + gn] = acc[i][j][v];
      }
}

template <int NS>
__global__ __launch_bounds__(256, 2) void k_batch_lds(const BatchItem *__restrict__ items,
                                                       const int64_t *__restrict__ first) {
  __shared__ __attribute__((aligned(16))) float lds[NS * kLdsStageWords];
  int64_t it = first[blockIdx.x];
  const int64_t end = first[blockIdx.x + 1];
  if (it >= end) return;
  BatchItem w = items[it];
  for (; it < end; ++it) {
    const BatchItem wn = items[it + 1 < end ? it + 1 : it];  // uniform: a scalar load
    if (w.tile == 0)
      batch_tile_lds16<1, NS>(w, lds);
    else
      batch_tile_lds16<2, NS>(w, lds);
    w = wn;
  }
}

// As many workgroups as can be resident at once (CUs x occupancy): every
// workgroup's share is fixed at build time, and one that had to wait for a
// free slot would run its share after everyone else.
template <typename F>
int persistent_grid(F kernel) {
  int dev = 0, cus = 256, per_cu = 4;
  if (hipGetDevice(&dev) == hipSuccess) {
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, dev) == hipSuccess && prop.multiProcessorCount > 0)
      cus = prop.multiProcessorCount;
  }
  int occ = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, kernel, 256, 0) == hipSuccess && occ > 0) per_cu = occ;
  return cus * per_cu;
}

moa_status hip_fail(hipError_t e, const char *what) {
  char buf[256];
  snprintf(buf, sizeof buf, "%s: %s", what, hipGetErrorString(e));
  return set_error(MOA_ERR_HIP, buf);
}

void free_batch(moa_batch *b) {
  if (!b) return;
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  if (b->d_items) (void)hipFree(b->d_items);
  if (b->d_first) (void)hipFree(b->d_first);
  delete b;
}

}  // namespace
}  // namespace moa

using namespace moa;

extern "C" {

moa_status moa_batch_build(int32_t n, const moa_shape *sa, const void *const *A, const moa_shape *sb,
                           const void *const *B, void *const *D, moa_dtype dt, void *stream, moa_batch **out) {
  if (!out) return set_error(MOA_ERR_NULL, "out is NULL");
  *out = nullptr;
  if (dt != MOA_F32 && dt != MOA_F64) return set_error(MOA_ERR_DTYPE, "batch needs MOA_F32 or MOA_F64");
  if (n < 0) return set_error(MOA_ERR_ARG, "negative batch size");
  if (n > 0 && (!sa || !sb || !A || !B || !D)) return set_error(MOA_ERR_NULL, "batch array is NULL");
  const size_t es = dt == MOA_F64 ? 8 : 4;
  std::vector<BatchDesc> desc((size_t)n);
  int table[kBuckets];
  {
    std::lock_guard<std::mutex> lk(g_table_mu);
    memcpy(table, g_table, sizeof table);
  }
  int64_t total_items = 0;
  bool idx32 = true, lds_ok = true;
  for (int32_t i = 0; i < n; ++i) {
    int64_t M, K, N;
    moa_status st = validate_inner(sa[i], sb[i], &M, &K, &N);
    if (st != MOA_OK) return st;
    if (M > INT32_MAX || N > INT32_MAX || K > INT32_MAX) return set_error(MOA_ERR_SIZE, "batch problem too large");
    // Offsets of a tile reach (extent + tile) x (extent + tile) at most.
    const int64_t lim = (int64_t)1 << 31;
    if ((M + 64) * (K + 64) >= lim || (K + 64) * (N + 64) >= lim || (M + 64) * (N + 64) >= lim) idx32 = false;
    // Buffer loads address A and B by 32-bit byte offsets, with 2^31 as the
    // out-of-range marker.
    if (M * K * (int64_t)es >= lim || K * N * (int64_t)es >= lim) lds_ok = false;
    if (M * K > 0 && !A[i]) return set_error(MOA_ERR_NULL, "A[i] is NULL");
    if (K * N > 0 && !B[i]) return set_error(MOA_ERR_NULL, "B[i] is NULL");
    if (M * N > 0 && !D[i]) return set_error(MOA_ERR_NULL, "D[i] is NULL");
    const uintptr_t d0 = (uintptr_t)D[i], d1 = d0 + (uintptr_t)(M * N) * es;
    const uintptr_t a0 = (uintptr_t)A[i], a1 = a0 + (uintptr_t)(M * K) * es;
    const uintptr_t b0 = (uintptr_t)B[i], b1 = b0 + (uintptr_t)(K * N) * es;
    if (M * N > 0 && ((M * K > 0 && d0 < a1 && a0 < d1) || (K * N > 0 && d0 < b1 && b0 < d1)))
      return set_error(MOA_ERR_ALIAS, "D[i] overlaps an input");
    const int v = table[bucket_of(M, N, K)];
    const int side = kTileSide[v];
    BatchDesc &d = desc[(size_t)i];
    d.A = A[i];
    d.B = B[i];
    d.D = D[i];
    d.M = (int32_t)M;
    d.K = (int32_t)K;
    d.N = (int32_t)N;
    d.tile = v;
    d.tiles_n = (int32_t)((N + side - 1) / side);
    const int64_t tiles = ((M + side - 1) / side) * d.tiles_n;
    total_items += (M * N > 0) ? tiles : 0;
  }
  // Work items, one per output tile. A tile of these small problems is bound
  // by load latency: its time is about a fixed cost plus one round trip per
  // 16-wide k panel, whatever the tile side, so its cost is 2 + ceil(K / 16)
  // panel times. The items are dealt to the persistent workgroups by the
  // longest-processing-time rule (costliest first, each to the workgroup
  // with the least work so far; ties to the lowest index), and each
  // workgroup's items are stored contiguously.
  // FP32 with 32-bit offsets everywhere: the LDS-fed tile; other FP32
  // batches the register-staged tile with 64-bit index arithmetic; FP64 the
  // register-staged tile with 32- or 64-bit index arithmetic.
  const int kind = dt == MOA_F32 ? (idx32 && lds_ok ? 0 : 1) : (idx32 ? 2 : 3);
  const int grid = kind == 0   ? persistent_grid(k_batch_lds<kLdsStages>)
                   : kind == 1 ? persistent_grid(k_batch<float, int64_t>)
                   : kind == 2 ? persistent_grid(k_batch<double, int32_t>)
                               : persistent_grid(k_batch<double, int64_t>);
  struct Tile {
    int32_t prob, t;
    int64_t cost;
  };
  std::vector<Tile> tiles_all;
  tiles_all.reserve((size_t)total_items);
  for (int32_t i = 0; i < n; ++i) {
    const BatchDesc &d = desc[(size_t)i];
    if ((int64_t)d.M * d.N == 0) continue;
    const int side = kTileSide[d.tile];
    const int64_t tiles = ((d.M + side - 1) / side) * (int64_t)d.tiles_n;
    for (int64_t t = 0; t < tiles; ++t) tiles_all.push_back(Tile{i, (int32_t)t, 2 + ((int64_t)d.K + 15) / 16});
  }
  std::stable_sort(tiles_all.begin(), tiles_all.end(), [](const Tile &x, const Tile &y) { return x.cost > y.cost; });
  std::vector<int32_t> owner(tiles_all.size());
  std::vector<int64_t> count((size_t)grid, 0);
  {
    typedef std::pair<int64_t, int32_t> Slot;  // (work so far, workgroup)
    std::priority_queue<Slot, std::vector<Slot>, std::greater<Slot>> heap;
    for (int32_t g = 0; g < grid; ++g) heap.push(Slot{0, g});
    for (size_t k = 0; k < tiles_all.size(); ++k) {
      Slot sl = heap.top();
      heap.pop();
      owner[k] = sl.second;
      ++count[(size_t)sl.second];
      sl.first += tiles_all[k].cost;
      heap.push(sl);
    }
  }
  std::vector<int64_t> first((size_t)grid + 1, 0);
  for (int32_t g = 0; g < grid; ++g) first[(size_t)g + 1] = first[(size_t)g] + count[(size_t)g];
  std::vector<BatchItem> items(tiles_all.size());
  {
    std::vector<int64_t> next(first.begin(), first.end() - 1);
    for (size_t k = 0; k < tiles_all.size(); ++k) {
      const BatchDesc &d = desc[(size_t)tiles_all[k].prob];
      const int side = kTileSide[d.tile];
      const int32_t t = tiles_all[k].t;
      items[(size_t)next[(size_t)owner[k]]++] =
          BatchItem{d.A, d.B, d.D, d.M, d.K, d.N, d.tile, t / d.tiles_n * side, t % d.tiles_n * side};
    }
  }

  moa_batch *b = new moa_batch();
  memset(b, 0, sizeof *b);
  b->dt = dt;
  b->n = n;
  b->items = (int64_t)items.size();
  b->idx32 = idx32;
  b->kind = kind;
  b->grid = grid;
  hipError_t e;
  hipStream_t cap = nullptr;
  if (!items.empty() && (e = hipMalloc(&b->d_items, sizeof(BatchItem) * items.size())) != hipSuccess) goto hip_error;
  if ((e = hipMalloc(&b->d_first, sizeof(int64_t) * first.size())) != hipSuccess) goto hip_error;
  // The work list and the shares are uploaded on `stream` (ordered after the
  // caller's earlier work there) and build waits for the copies, so the host
  // vectors may go.
  if (!items.empty() && (e = hipMemcpyAsync(b->d_items, items.data(), sizeof(BatchItem) * items.size(),
                                            hipMemcpyHostToDevice, (hipStream_t)stream)) != hipSuccess)
    goto hip_error;
  if ((e = hipMemcpyAsync(b->d_first, first.data(), sizeof(int64_t) * first.size(), hipMemcpyHostToDevice,
                          (hipStream_t)stream)) != hipSuccess)
    goto hip_error;
  if ((e = hipStreamSynchronize((hipStream_t)stream)) != hipSuccess) goto hip_error;
  // Capture the persistent launch on a private stream (capture is not allowed
  // on the legacy default stream); the graph is replayed on any stream.
  if ((e = hipStreamCreateWithFlags(&cap, hipStreamNonBlocking)) != hipSuccess) goto hip_error;
  if ((e = hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal)) != hipSuccess) goto hip_error;
  if (b->items > 0) {
    const dim3 g((unsigned)b->grid), t(256);
    switch (kind) {
      case 0: hipLaunchKernelGGL((k_batch_lds<kLdsStages>), g, t, 0, cap, b->d_items, b->d_first); break;
      case 1: hipLaunchKernelGGL((k_batch<float, int64_t>), g, t, 0, cap, b->d_items, b->d_first); break;
      case 2: hipLaunchKernelGGL((k_batch<double, int32_t>), g, t, 0, cap, b->d_items, b->d_first); break;
      default: hipLaunchKernelGGL((k_batch<double, int64_t>), g, t, 0, cap, b->d_items, b->d_first); break;
    }
  }
  if ((e = hipStreamEndCapture(cap, &b->graph)) != hipSuccess) goto hip_error;
  if ((e = hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0)) != hipSuccess) goto hip_error;
  (void)hipStreamDestroy(cap);
  *out = b;
  return MOA_OK;
hip_error:
  if (cap) (void)hipStreamDestroy(cap);
  free_batch(b);
  return hip_fail(e, "moa_batch_build");
}

moa_status moa_batch_run(moa_batch *b, void *stream) {
  if (!b) return set_error(MOA_ERR_NULL, "batch is NULL");
  if (b->items == 0) return MOA_OK;
  hipError_t e = hipGraphLaunch(b->exec, (hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(e, "moa_batch_run");
  return MOA_OK;
}

void moa_batch_free(moa_batch *b) { free_batch(b); }

moa_status moa_batch_info(const moa_batch *b, int64_t *work_items, int32_t *launches) {
  if (!b) return set_error(MOA_ERR_NULL, "batch is NULL");
  if (work_items) *work_items = b->items;
  if (launches) *launches = b->items > 0 ? 1 : 0;
  return MOA_OK;
}

moa_status moa_tile_table_get(char *buf, size_t len) {
  if (!buf || len == 0) return set_error(MOA_ERR_NULL, "buffer is NULL");
  std::string s;
  {
    std::lock_guard<std::mutex> lk(g_table_mu);
    for (int bk = 0; bk < kBuckets; ++bk) {
      char line[96];
      snprintf(line, sizeof line, "%s %s %s %d\n", (bk & 4) ? "M>32" : "M<=32", (bk & 2) ? "N>32" : "N<=32",
               (bk & 1) ? "K>128" : "K<=128", g_table[bk]);
      s += line;
    }
  }
  if (s.size() + 1 > len) return set_error(MOA_ERR_ARG, "buffer too small");
  memcpy(buf, s.c_str(), s.size() + 1);
  return MOA_OK;
}

// Bucket bit of one token: `hi` ("M>32") sets it, `lo` ("M<=32") clears it,
// anything else is an error (-1).
static int bucket_bit(const char *tok, const char *lo, const char *hi, int bit) {
  if (strcmp(tok, hi) == 0) return bit;
  if (strcmp(tok, lo) == 0) return 0;
  return -1;
}

moa_status moa_tile_table_set(const char *text) {
  if (!text) return set_error(MOA_ERR_NULL, "text is NULL");
  int t[kBuckets];
  for (int bk = 0; bk < kBuckets; ++bk) t[bk] = -1;
  const char *p = text;
  while (*p == '\n' || *p == ' ' || *p == '\t') ++p;
  while (*p) {
    char m[16], nn[16], k[16];
    int v, used = 0;
    if (sscanf(p, "%15s %15s %15s %d%n", m, nn, k, &v, &used) != 4)
      return set_error(MOA_ERR_ARG, "tile table line is not 'bucket_m bucket_n bucket_k variant'");
    if (v < 0 || v >= kVariants) return set_error(MOA_ERR_ARG, "tile variant out of range");
    const int bm = bucket_bit(m, "M<=32", "M>32", 4), bn = bucket_bit(nn, "N<=32", "N>32", 2),
              bkk = bucket_bit(k, "K<=128", "K>128", 1);
    if (bm < 0 || bn < 0 || bkk < 0) return set_error(MOA_ERR_ARG, "unknown bucket name in the tile table");
    const int bk = bm + bn + bkk;
    if (t[bk] >= 0) return set_error(MOA_ERR_ARG, "tile table sets a bucket twice");
    t[bk] = v;
    p += used;
    while (*p == '\n' || *p == ' ' || *p == '\t') ++p;
  }
  for (int bk = 0; bk < kBuckets; ++bk)
    if (t[bk] < 0) return set_error(MOA_ERR_ARG, "tile table needs one line per bucket");
  std::lock_guard<std::mutex> lk(g_table_mu);
  memcpy(g_table, t, sizeof t);
  return MOA_OK;
}

// Autotuner: for each size bucket, build synthetic batches that use only that
// bucket's shapes, time each tile variant (HIP events around graph replays on
// `stream`) and keep the fastest. Each batch holds enough problems to fill
// every CU many times over, as a production batch does; with a few hundred,
// the smaller tile won only by adding parallelism the real batch already has.
moa_status moa_batch_autotune(moa_dtype dt, int32_t reps, void *stream) {
  if (dt != MOA_F32 && dt != MOA_F64) return set_error(MOA_ERR_DTYPE, "autotune needs MOA_F32 or MOA_F64");
  if (reps < 1) reps = 5;
  const size_t es = dt == MOA_F64 ? 8 : 4;
  const int kProblems = 4096;
  hipStream_t s = (hipStream_t)stream;
  std::mt19937_64 rng(12345);
  int best[kBuckets];
  int saved[kBuckets];
  {
    std::lock_guard<std::mutex> lk(g_table_mu);
    memcpy(saved, g_table, sizeof saved);
  }
  void *pool = nullptr;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  hipError_t he;
  if ((he = hipEventCreate(&e0)) != hipSuccess || (he = hipEventCreate(&e1)) != hipSuccess)
    return hip_fail(he, "autotune events");
  moa_status result = MOA_OK;
  for (int bk = 0; bk < kBuckets && result == MOA_OK; ++bk) {
    std::vector<int64_t> dims(6 * (size_t)kProblems);
    size_t bytes = 0;
    std::vector<size_t> offA(kProblems), offB(kProblems), offD(kProblems);
    for (int i = 0; i < kProblems; ++i) {
      auto pick = [&](int lo, int hi) { return (int64_t)(lo + (int)(rng() % (uint64_t)(hi - lo + 1))); };
      const int64_t M = (bk & 4) ? pick(33, 64) : pick(4, 32);
      const int64_t N = (bk & 2) ? pick(33, 64) : pick(4, 32);
      const int64_t K = (bk & 1) ? pick(129, 512) : pick(16, 128);
      dims[6 * i + 0] = M;
      dims[6 * i + 1] = K;
      dims[6 * i + 2] = K;
      dims[6 * i + 3] = N;
      offA[i] = bytes;
      bytes += (size_t)(M * K) * es;
      offB[i] = bytes;
      bytes += (size_t)(K * N) * es;
      offD[i] = bytes;
      bytes += (size_t)(M * N) * es;
      bytes = (bytes + 255) & ~(size_t)255;
    }
    if ((he = hipMalloc(&pool, bytes)) != hipSuccess) {
      result = hip_fail(he, "autotune pool");
      break;
    }
    (void)hipMemsetAsync(pool, 0, bytes, s);
    std::vector<moa_shape> sa(kProblems), sb(kProblems);
    std::vector<const void *> pa(kProblems), pb(kProblems);
    std::vector<void *> pd(kProblems);
    for (int i = 0; i < kProblems; ++i) {
      sa[i] = moa_shape{2, &dims[6 * i + 0]};
      sb[i] = moa_shape{2, &dims[6 * i + 2]};
      pa[i] = (char *)pool + offA[i];
      pb[i] = (char *)pool + offB[i];
      pd[i] = (char *)pool + offD[i];
    }
    float best_ms = 1e30f;
    best[bk] = saved[bk];
    for (int v = 0; v < kVariants && result == MOA_OK; ++v) {
      {
        std::lock_guard<std::mutex> lk(g_table_mu);
        for (int q = 0; q < kBuckets; ++q) g_table[q] = v;
      }
      moa_batch *b = nullptr;
      moa_status st = moa_batch_build(kProblems, sa.data(), pa.data(), sb.data(), pb.data(), pd.data(), dt, stream, &b);
      if (st != MOA_OK) {
        result = st;
        break;
      }
      (void)moa_batch_run(b, stream);
      (void)hipEventRecord(e0, s);
      for (int r = 0; r < reps; ++r) (void)moa_batch_run(b, stream);
      (void)hipEventRecord(e1, s);
      if ((he = hipEventSynchronize(e1)) != hipSuccess) {
        moa_batch_free(b);
        result = hip_fail(he, "autotune timing");
        break;
      }
      float ms = 0.f;
      (void)hipEventElapsedTime(&ms, e0, e1);
      if (ms < best_ms) {
        best_ms = ms;
        best[bk] = v;
      }
      moa_batch_free(b);
    }
    (void)hipStreamSynchronize(s);
    (void)hipFree(pool);
    pool = nullptr;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  std::lock_guard<std::mutex> lk(g_table_mu);
  if (result == MOA_OK)
    memcpy(g_table, best, sizeof best);
  else
    memcpy(g_table, saved, sizeof saved);
  return result;
}

}  // extern "C"
