// Grouped FP64 GEMM engine on the CDNA matrix cores (v_mfma_f64_16x16x4).
//
// One workgroup (4 wave64) computes one BM x BN tile of one task.  Operand
// tiles of depth 16 are staged through two LDS buffers with coalesced global
// reads (k-contiguous or m/n-contiguous depending on the transpose flags):
// the next tile is loaded into registers while the current one feeds the
// matrix cores, then stored to the other buffer, one barrier per step.  LDS
// tiles are k-major so each MFMA operand read is 16 consecutive doubles.
// Stored rows of either operand may be gathered through an index list (rows
// of A = M index when A is not transposed, K index when it is; rows of B = K
// index when B is not transposed, N index when it is), which lets one task
// project a slab onto the OSVs of all neighbours of an orbital, form a
// 4-block pair K from two scattered row blocks, or contract gradient blocks
// of many pairs in one K-concatenated product.  A task may also store C^T
// (the coupling blocks are needed in both orientations).
#include "internal.hpp"

namespace mbe3 {

typedef double d4 __attribute__((ext_vector_type(4)));

template <int BM, int BN>
__global__ __launch_bounds__(256, 2) void gemm_tasks_kernel(
    const GemmTask *__restrict__ tasks, int n_tasks, GemmBases bases) {
  constexpr int BK = 16;
  // pitch = BM + 16: the four k-rows an MFMA read touches (lane / 16) start
  // 2 PA = 32 (mod 64) banks apart, so each half-wave reads distinct banks
  constexpr int PA = BM + 16;
  constexpr int PB = BN + 16;
  __shared__ double As[2][BK * PA];
  __shared__ double Bs[2][BK * PB];

  const int64_t tile = blockIdx.x;
  int lo = 0, hi = n_tasks - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (tasks[mid].tile_begin <= tile) lo = mid; else hi = mid - 1;
  }
  const GemmTask t = tasks[lo];
  const int64_t local = tile - t.tile_begin;
  const int m0 = (int)(local / t.tiles_n) * BM;
  const int n0 = (int)(local % t.tiles_n) * BN;
  const double *__restrict__ A = bases.p[t.a_buf] + t.a_off;
  const double *__restrict__ B = bases.p[t.b_buf] + t.b_off;
  double *__restrict__ C = bases.p[t.c_buf] + t.c_off;
  double *__restrict__ CT = t.ct_off >= 0 ? bases.p[t.c_buf] + t.ct_off : nullptr;
  const int32_t *__restrict__ rows = bases.rows;

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  constexpr int WM = BM / 2, WN = BN / 2;
  constexpr int TM = WM / 16, TN = WN / 16;
  const int wr = wave >> 1, wc = wave & 1;

  d4 acc[TM][TN];
#pragma unroll
  for (int i = 0; i < TM; ++i)
#pragma unroll
    for (int j = 0; j < TN; ++j) acc[i][j] = d4{0.0, 0.0, 0.0, 0.0};

  // A / B elements per thread: a tile of BM x 16 split evenly when that
  // gives a power of two per thread, else 8 per thread on the first
  // BM * 16 / 8 threads (the 96-wide tiles: 192 of 256 threads load)
  constexpr int EA0 = BM * BK / 256, EB0 = BN * BK / 256;
  constexpr int EA = (BK % EA0 == 0) ? EA0 : 8;
  constexpr int EB = (BK % EB0 == 0) ? EB0 : 8;
  const bool a_act = tid < BM * BK / EA;
  const bool b_act = tid < BN * BK / EB;

  // Per-thread source positions.  k-contiguous A (transA = 0): EA consecutive
  // k of one row; m-contiguous A (transA = 1): EA consecutive m of one k row.
  // B likewise.  Gathered rows are resolved per k-row as they come.
  const int a_tpr = BK / EA;
  const int a_r = tid / a_tpr, a_k = (tid % a_tpr) * EA;
  int64_t a_row = -1;
  if (a_act && !t.transA && m0 + a_r < t.M)
    a_row = (t.a_rows >= 0) ? rows[t.a_rows + m0 + a_r] : (m0 + a_r);
  const int a_tpk = BM / EA;
  const int a_kk = tid / a_tpk, a_mm = (tid % a_tpk) * EA;
  const int b_tpr = BK / EB;
  const int b_r = tid / b_tpr, b_k = (tid % b_tpr) * EB;
  int64_t b_row = -1;
  if (b_act && t.transB && n0 + b_r < t.N)
    b_row = (t.b_rows >= 0) ? rows[t.b_rows + n0 + b_r] : (n0 + b_r);
  const int b_tpk = BN / EB;
  const int b_kk = tid / b_tpk, b_nn = (tid % b_tpk) * EB;

  double ra[EA], rb[EB];  // the next tile, in flight during the products
#define MBE3_GEMM_LOAD(K0)                                                     \
  do {                                                                         \
    if (!t.transA) {                                                           \
      _Pragma("unroll") for (int e = 0; e < EA; ++e) {                         \
        const int k = (K0) + a_k + e;                                          \
        ra[e] = (a_row >= 0 && k < t.K) ? A[a_row * (int64_t)t.lda + k] : 0.0; \
      }                                                                        \
    } else {                                                                   \
      const int k = (K0) + a_kk;                                               \
      const int64_t krow = k < t.K ? (t.a_rows >= 0 ? rows[t.a_rows + k] : k) : 0; \
      _Pragma("unroll") for (int e = 0; e < EA; ++e) {                         \
        const int m = m0 + a_mm + e;                                           \
        ra[e] = (a_act && m < t.M && k < t.K) ? A[krow * t.lda + m] : 0.0;     \
      }                                                                        \
    }                                                                          \
    if (!t.transB) {                                                           \
      const int k = (K0) + b_kk;                                               \
      const int64_t krow = k < t.K ? (t.b_rows >= 0 ? rows[t.b_rows + k] : k) : 0; \
      _Pragma("unroll") for (int e = 0; e < EB; ++e) {                         \
        const int n = n0 + b_nn + e;                                           \
        rb[e] = (b_act && n < t.N && k < t.K) ? B[krow * t.ldb + n] : 0.0;     \
      }                                                                        \
    } else {                                                                   \
      _Pragma("unroll") for (int e = 0; e < EB; ++e) {                         \
        const int k = (K0) + b_k + e;                                          \
        rb[e] = (b_row >= 0 && k < t.K) ? B[b_row * (int64_t)t.ldb + k] : 0.0; \
      }                                                                        \
    }                                                                          \
  } while (0)
#define MBE3_GEMM_STORE(BUF)                                                   \
  do {                                                                         \
    double *as_ = As[BUF];                                                     \
    double *bs_ = Bs[BUF];                                                     \
    if (!a_act) {                                                              \
    } else if (!t.transA) {                                                    \
      _Pragma("unroll") for (int e = 0; e < EA; ++e) as_[(a_k + e) * PA + a_r] = ra[e]; \
    } else {                                                                   \
      _Pragma("unroll") for (int e = 0; e < EA; ++e) as_[a_kk * PA + a_mm + e] = ra[e]; \
    }                                                                          \
    if (!b_act) {                                                              \
    } else if (!t.transB) {                                                    \
      _Pragma("unroll") for (int e = 0; e < EB; ++e) bs_[b_kk * PB + b_nn + e] = rb[e]; \
    } else {                                                                   \
      _Pragma("unroll") for (int e = 0; e < EB; ++e) bs_[(b_k + e) * PB + b_r] = rb[e]; \
    }                                                                          \
  } while (0)

  MBE3_GEMM_LOAD(0);
  MBE3_GEMM_STORE(0);
  __syncthreads();
  int buf = 0;
  for (int k0 = 0; k0 < t.K; k0 += BK) {
    const bool more = k0 + BK < t.K;
    if (more) MBE3_GEMM_LOAD(k0 + BK);
    const double *as = As[buf];
    const double *bs = Bs[buf];
#pragma unroll
    for (int kk = 0; kk < BK; kk += 4) {
      const int kr = kk + (lane >> 4);
      double a[TM], b[TN];
#pragma unroll
      for (int i = 0; i < TM; ++i) a[i] = as[kr * PA + wr * WM + i * 16 + (lane & 15)];
#pragma unroll
      for (int j = 0; j < TN; ++j) b[j] = bs[kr * PB + wc * WN + j * 16 + (lane & 15)];
#pragma unroll
      for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int j = 0; j < TN; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[i], b[j], acc[i][j], 0, 0, 0);
    }
    // the other buffer was last read before the previous barrier
    if (more) MBE3_GEMM_STORE(buf ^ 1);
    __syncthreads();
    buf ^= 1;
  }
#undef MBE3_GEMM_LOAD
#undef MBE3_GEMM_STORE

  // ---- epilogue: D layout of v_mfma_f64_16x16x4: register v of lane l holds
  //      row (l / 16) + 4 v, column l % 16
#pragma unroll
  for (int i = 0; i < TM; ++i)
#pragma unroll
    for (int j = 0; j < TN; ++j) {
      const int n = n0 + wc * WN + j * 16 + (lane & 15);
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int m = m0 + wr * WM + i * 16 + (lane >> 4) + 4 * v;
        if (m < t.M && n < t.N) {
          double *c = C + (int64_t)m * t.ldc + n;
          double r = t.alpha * acc[i][j][v];
          if (t.beta != 0.0) r += t.beta * *c;
          *c = r;
          if (CT) CT[(int64_t)n * t.ldct + m] = r;
        }
      }
    }
}

int gemm_tile_m(GemmShape shape) {
  switch (shape) {
    case GEMM_128x128: return 128;
    case GEMM_32x32:
    case GEMM_32x128: return 32;
    case GEMM_96x96: return 96;
    default: return 64;
  }
}

int gemm_tile_n(GemmShape shape) {
  switch (shape) {
    case GEMM_32x32: return 32;
    case GEMM_64x64: return 64;
    case GEMM_96x96: return 96;
    default: return 128;
  }
}

const char *gemm_shape_name(GemmShape shape) {
  switch (shape) {
    case GEMM_64x64: return "64x64";
    case GEMM_128x128: return "128x128";
    case GEMM_32x32: return "32x32";
    case GEMM_32x128: return "32x128";
    case GEMM_64x128: return "64x128";
    case GEMM_96x96: return "96x96";
    default: return "?";
  }
}

int64_t gemm_tile_count(const GemmTask &t, GemmShape shape) {
  const int bm = gemm_tile_m(shape), bn = gemm_tile_n(shape);
  return (int64_t)((t.M + bm - 1) / bm) * ((t.N + bn - 1) / bn);
}

hipError_t launch_gemm_tasks(const GemmTask *d_tasks, int n_tasks,
                             int64_t n_tiles, const GemmBases &bases,
                             GemmShape shape, hipStream_t s) {
  if (n_tasks <= 0 || n_tiles <= 0) return hipSuccess;
  if (n_tiles > 0x7fffffffLL) return hipErrorInvalidValue;
  dim3 grid((unsigned)n_tiles), block(256);
  switch (shape) {
    case GEMM_64x64:
      hipLaunchKernelGGL((gemm_tasks_kernel<64, 64>), grid, block, 0, s, d_tasks,
                         n_tasks, bases);
      break;
    case GEMM_128x128:
      hipLaunchKernelGGL((gemm_tasks_kernel<128, 128>), grid, block, 0, s, d_tasks,
                         n_tasks, bases);
      break;
    case GEMM_32x32:
      hipLaunchKernelGGL((gemm_tasks_kernel<32, 32>), grid, block, 0, s, d_tasks,
                         n_tasks, bases);
      break;
    case GEMM_32x128:
      hipLaunchKernelGGL((gemm_tasks_kernel<32, 128>), grid, block, 0, s, d_tasks,
                         n_tasks, bases);
      break;
    case GEMM_64x128:
      hipLaunchKernelGGL((gemm_tasks_kernel<64, 128>), grid, block, 0, s, d_tasks,
                         n_tasks, bases);
      break;
    case GEMM_96x96:
      hipLaunchKernelGGL((gemm_tasks_kernel<96, 96>), grid, block, 0, s, d_tasks,
                         n_tasks, bases);
      break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace mbe3
