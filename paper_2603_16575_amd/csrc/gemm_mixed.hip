// Split-precision grouped GEMM for the projection (eq. osv_imua) and the
// pair exchange matrices (eq. osv_close_k) in the mixed form: each FP64
// operand is carried as three bf16 pieces x = h + m + l, and
//   a b ~ h_a h_b + h_a m_b + m_a h_b + h_a l_b + m_a m_b + l_a h_b
// (the projection: its pieces are relative roundings, so the dropped
// products are below 2^-24 relative; pair_K forms all nine) runs on
// v_mfma_f32_16x16x32_bf16 (each bf16 x bf16 product is exact in FP32).  The
// leading product h_a h_b of every 32-deep block is formed from a zero
// accumulator and added to an FP64 accumulator, so FP32 rounding touches it
// once per block instead of growing with K; the five correction products,
// 2^-8 and less of it, accumulate in FP32 over a few blocks at a time and
// are then added to the FP64 accumulator too.  Results are stored in FP64.
//
// C = A B^T with both operands K-contiguous: lane l of a wave holds row l%16
// of an A tile and row l%16 of a B tile (a column of B^T) with the eight
// consecutive k = 8 (l/16) + e, so every operand is one 16-byte load straight
// from global memory (no LDS, no barriers); the output register v of lane l
// is row 4 (l/16) + v, column l%16 of the 16 x 16 tile.  A workgroup of four
// waves (2 x 2) covers (32 TM) x (32 TN) outputs; the six products cycle
// over the TM x TN independent accumulators so no MFMA waits on its
// predecessor.  Requires K, lda, ldb and plane strides to be multiples of 8
// (the planes are zero padded).
#include "internal.hpp"

namespace mbe3 {

typedef __bf16 bf8 __attribute__((ext_vector_type(8)));
typedef unsigned u4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));

struct MixedArgs {
  const uint16_t *A, *B;
  int64_t a_ps, b_ps;
  double *C;
  const int32_t *rows;
};

// PF: load the next block's operands before this block's products (pays off
// for the small pair_K tiles; the 64 x 128 projection tile is better served
// by the occupancy the extra registers would cost).
// Correction products are summed in FP32 over MIXED_FLUSH 32-deep blocks,
// then added to the FP64 accumulator (a long FP32 sum would gather rounding
// error in proportion to K).  ALL forms all nine piece products: the pair_K
// operands carry fixed-point pieces on the grid of their row, so every
// element's third piece is grid noise of up to 2^-16 of the row's largest,
// and dropping l l would bias each diagonal entry of K by minus the sum of
// their squares.
constexpr int MIXED_FLUSH = 4;

template <int TM, int TN, bool PF, bool ALL>
__global__ __launch_bounds__(256) void gemm_mixed_kernel(
    const MixedTask *__restrict__ tasks, int n_tasks, MixedArgs g) {
  const int64_t tile = blockIdx.x;
  int lo = 0, hi = n_tasks - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (tasks[mid].tile_begin <= tile) lo = mid;
    else hi = mid - 1;
  }
  const MixedTask t = tasks[lo];
  const int64_t lt = tile - t.tile_begin;
  const int tm = (int)(lt / t.tiles_n);
  const int tn = (int)(lt - (int64_t)tm * t.tiles_n);
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int r16 = lane & 15, q = lane >> 4;
  const int mw = tm * 32 * TM + (wave >> 1) * 16 * TM;
  const int nw = tn * 32 * TN + (wave & 1) * 16 * TN;

  const u4 *ap[TM];
  const u4 *bp[TN];
  bool av[TM], bv[TN];
#pragma unroll
  for (int i = 0; i < TM; ++i) {
    const int row = mw + 16 * i + r16;
    av[i] = row < t.M;
    const int64_t pr = av[i] ? (t.a_rows >= 0 ? g.rows[t.a_rows + row] : row) : 0;
    ap[i] = reinterpret_cast<const u4 *>(g.A + t.a_off + pr * t.lda + 8 * q);
  }
#pragma unroll
  for (int j = 0; j < TN; ++j) {
    const int row = nw + 16 * j + r16;
    bv[j] = row < t.N;
    const int64_t pr = bv[j] ? (t.b_rows >= 0 ? g.rows[t.b_rows + row] : row) : 0;
    bp[j] = reinterpret_cast<const u4 *>(g.B + t.b_off + pr * t.ldb + 8 * q);
  }
  const int64_t aps = g.a_ps / 8, bps = g.b_ps / 8;  // plane strides in u4

  f4 acc[TM][TN];   // correction products, FP32 over MIXED_FLUSH blocks
  double dacc[TM][TN][4];  // FP64 sum of the blocks' leading products and flushes
#pragma unroll
  for (int i = 0; i < TM; ++i)
#pragma unroll
    for (int j = 0; j < TN; ++j) {
      acc[i][j] = f4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int v = 0; v < 4; ++v) dacc[i][j][v] = 0.0;
    }

  const u4 zero = {0u, 0u, 0u, 0u};
  // operands of the block at k0 (held) and of the next block (in flight)
  u4 a[3][TM], b[3][TN];
#define MBE3_LOAD(DA, DB, K0)                                                 \
  do {                                                                        \
    const bool kv_ = (K0) + 8 * q < t.K;                                      \
    const int ko_ = (K0) >> 3;                                                \
    _Pragma("unroll") for (int p = 0; p < 3; ++p) {                           \
      _Pragma("unroll") for (int i = 0; i < TM; ++i)                          \
        DA[p][i] = (av[i] && kv_) ? ap[i][p * aps + ko_] : zero;              \
      _Pragma("unroll") for (int j = 0; j < TN; ++j)                          \
        DB[p][j] = (bv[j] && kv_) ? bp[j][p * bps + ko_] : zero;              \
    }                                                                         \
  } while (0)
  if (PF) MBE3_LOAD(a, b, 0);
  int nblk = 0;
  for (int k0 = 0; k0 < t.K; k0 += 32) {
    u4 an[3][TM], bn[3][TN];
    if (!PF) MBE3_LOAD(a, b, k0);
    else if (k0 + 32 < t.K) MBE3_LOAD(an, bn, k0 + 32);
#define MBE3_PROD(PA, PB)                                                     \
  _Pragma("unroll") for (int i = 0; i < TM; ++i)                              \
    _Pragma("unroll") for (int j = 0; j < TN; ++j)                            \
      acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(                    \
          __builtin_bit_cast(bf8, a[PA][i]), __builtin_bit_cast(bf8, b[PB][j]), \
          acc[i][j], 0, 0, 0)
    if (ALL) {
      MBE3_PROD(2, 2);
      MBE3_PROD(2, 1);
      MBE3_PROD(1, 2);
    }
    MBE3_PROD(2, 0);
    MBE3_PROD(1, 1);
    MBE3_PROD(0, 2);
    MBE3_PROD(1, 0);
    MBE3_PROD(0, 1);
#undef MBE3_PROD
    if (++nblk == MIXED_FLUSH || k0 + 32 >= t.K) {
      nblk = 0;
#pragma unroll
      for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int j = 0; j < TN; ++j) {
#pragma unroll
          for (int v = 0; v < 4; ++v) dacc[i][j][v] += (double)acc[i][j][v];
          acc[i][j] = f4{0.f, 0.f, 0.f, 0.f};
        }
    }
    const f4 fz = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int i = 0; i < TM; ++i)
#pragma unroll
      for (int j = 0; j < TN; ++j) {
        const f4 t = __builtin_amdgcn_mfma_f32_16x16x32_bf16(
            __builtin_bit_cast(bf8, a[0][i]), __builtin_bit_cast(bf8, b[0][j]), fz, 0, 0, 0);
#pragma unroll
        for (int v = 0; v < 4; ++v) dacc[i][j][v] += (double)t[v];
      }
    if (PF && k0 + 32 < t.K) {
#pragma unroll
      for (int p = 0; p < 3; ++p) {
#pragma unroll
        for (int i = 0; i < TM; ++i) a[p][i] = an[p][i];
#pragma unroll
        for (int j = 0; j < TN; ++j) b[p][j] = bn[p][j];
      }
    }
  }
#undef MBE3_LOAD
#pragma unroll
  for (int i = 0; i < TM; ++i)
#pragma unroll
    for (int j = 0; j < TN; ++j) {
      const int n = nw + 16 * j + r16;
      if (n >= t.N) continue;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int m = mw + 16 * i + 4 * q + v;
        if (m < t.M)
          g.C[t.c_off + (int64_t)m * t.ldc + n] = dacc[i][j][v];
      }
    }
}

// The projection tile (64 x 128, relative pieces, six products) with its
// operands staged through LDS: each 32-deep block of the workgroup's A rows
// (64) and B rows (128), all three planes, is fetched once per workgroup
// (16-byte chunks, the next block in registers while the matrix cores work
// on the current one) instead of once per wave, and the waves read their
// fragments from LDS.  The products, their order and the FP64 flushes are
// those of gemm_mixed_kernel with TM = 2, TN = 4 (its per-wave loads gave
// the same results bit for bit at 16.9 instead of 13.7 ms per 160-LMO
// projection).
constexpr int LDS_ROW = 5;  // u4 per LDS row: 64 bytes of k plus 16 of pad
__global__ __launch_bounds__(256) void gemm_mixed_proj_lds_kernel(
    const MixedTask *__restrict__ tasks, int n_tasks, MixedArgs g) {
  constexpr int TM = 2, TN = 4;
  __shared__ u4 As[3 * 64 * LDS_ROW];
  __shared__ u4 Bs[3 * 128 * LDS_ROW];
  const int64_t tile = blockIdx.x;
  int lo = 0, hi = n_tasks - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (tasks[mid].tile_begin <= tile) lo = mid;
    else hi = mid - 1;
  }
  const MixedTask t = tasks[lo];
  const int64_t lt = tile - t.tile_begin;
  const int tm = (int)(lt / t.tiles_n);
  const int tn = (int)(lt - (int64_t)tm * t.tiles_n);
  const int tid = threadIdx.x;
  const int wave = tid >> 6, lane = tid & 63;
  const int r16 = lane & 15, q = lane >> 4;
  const int mw = tm * 64 + (wave >> 1) * 32;
  const int nw = tn * 128 + (wave & 1) * 64;

  // this thread's chunks: A row tid / 4 (three planes), B rows tid / 4 and
  // tid / 4 + 64 (three planes each), all at 16-byte column tid % 4
  const int lr = tid >> 2, kc = tid & 3;
  const u4 zero = {0u, 0u, 0u, 0u};
  const int ra = tm * 64 + lr, rb0 = tn * 128 + lr, rb1 = rb0 + 64;
  const bool va = ra < t.M, vb0 = rb0 < t.N, vb1 = rb1 < t.N;
  const u4 *pa = reinterpret_cast<const u4 *>(
      g.A + t.a_off + (va ? (t.a_rows >= 0 ? g.rows[t.a_rows + ra] : ra) : 0) * (int64_t)t.lda) + kc;
  const u4 *pb0 = reinterpret_cast<const u4 *>(
      g.B + t.b_off + (vb0 ? (t.b_rows >= 0 ? g.rows[t.b_rows + rb0] : rb0) : 0) * (int64_t)t.ldb) + kc;
  const u4 *pb1 = reinterpret_cast<const u4 *>(
      g.B + t.b_off + (vb1 ? (t.b_rows >= 0 ? g.rows[t.b_rows + rb1] : rb1) : 0) * (int64_t)t.ldb) + kc;
  const int64_t aps = g.a_ps / 8, bps = g.b_ps / 8;  // plane strides in u4
  u4 fa[3], fb0[3], fb1[3];
#define MBE3_FETCH(K0)                                                        \
  do {                                                                        \
    const bool kv_ = (K0) + 8 * kc < t.K;                                     \
    const int ko_ = (K0) >> 3;                                                \
    _Pragma("unroll") for (int p = 0; p < 3; ++p) {                           \
      fa[p] = (va && kv_) ? pa[p * aps + ko_] : zero;                         \
      fb0[p] = (vb0 && kv_) ? pb0[p * bps + ko_] : zero;                      \
      fb1[p] = (vb1 && kv_) ? pb1[p * bps + ko_] : zero;                      \
    }                                                                         \
  } while (0)

  f4 acc[TM][TN];
  double dacc[TM][TN][4];
#pragma unroll
  for (int i = 0; i < TM; ++i)
#pragma unroll
    for (int j = 0; j < TN; ++j) {
      acc[i][j] = f4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int v = 0; v < 4; ++v) dacc[i][j][v] = 0.0;
    }

  MBE3_FETCH(0);
  int nblk = 0;
  for (int k0 = 0; k0 < t.K; k0 += 32) {
    __syncthreads();  // the previous block's fragments are read
#pragma unroll
    for (int p = 0; p < 3; ++p) {
      As[(p * 64 + lr) * LDS_ROW + kc] = fa[p];
      Bs[(p * 128 + lr) * LDS_ROW + kc] = fb0[p];
      Bs[(p * 128 + lr + 64) * LDS_ROW + kc] = fb1[p];
    }
    __syncthreads();
    if (k0 + 32 < t.K) MBE3_FETCH(k0 + 32);
    u4 a[3][TM], b[3][TN];
#pragma unroll
    for (int p = 0; p < 3; ++p) {
#pragma unroll
      for (int i = 0; i < TM; ++i)
        a[p][i] = As[(p * 64 + (wave >> 1) * 32 + 16 * i + r16) * LDS_ROW + q];
#pragma unroll
      for (int j = 0; j < TN; ++j)
        b[p][j] = Bs[(p * 128 + (wave & 1) * 64 + 16 * j + r16) * LDS_ROW + q];
    }
#define MBE3_PROD(PA, PB)                                                     \
  _Pragma("unroll") for (int i = 0; i < TM; ++i)                              \
    _Pragma("unroll") for (int j = 0; j < TN; ++j)                            \
      acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(                    \
          __builtin_bit_cast(bf8, a[PA][i]), __builtin_bit_cast(bf8, b[PB][j]), \
          acc[i][j], 0, 0, 0)
    MBE3_PROD(2, 0);
    MBE3_PROD(1, 1);
    MBE3_PROD(0, 2);
    MBE3_PROD(1, 0);
    MBE3_PROD(0, 1);
#undef MBE3_PROD
    if (++nblk == MIXED_FLUSH || k0 + 32 >= t.K) {
      nblk = 0;
#pragma unroll
      for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int j = 0; j < TN; ++j) {
#pragma unroll
          for (int v = 0; v < 4; ++v) dacc[i][j][v] += (double)acc[i][j][v];
          acc[i][j] = f4{0.f, 0.f, 0.f, 0.f};
        }
    }
    const f4 fz = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int i = 0; i < TM; ++i)
#pragma unroll
      for (int j = 0; j < TN; ++j) {
        const f4 tt = __builtin_amdgcn_mfma_f32_16x16x32_bf16(
            __builtin_bit_cast(bf8, a[0][i]), __builtin_bit_cast(bf8, b[0][j]), fz, 0, 0, 0);
#pragma unroll
        for (int v = 0; v < 4; ++v) dacc[i][j][v] += (double)tt[v];
      }
  }
#undef MBE3_FETCH
#pragma unroll
  for (int i = 0; i < TM; ++i)
#pragma unroll
    for (int j = 0; j < TN; ++j) {
      const int n = nw + 16 * j + r16;
      if (n >= t.N) continue;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int m = mw + 16 * i + 4 * q + v;
        if (m < t.M)
          g.C[t.c_off + (int64_t)m * t.ldc + n] = dacc[i][j][v];
      }
    }
}

int mixed_tile_m(MixedShape shape) { return shape == MIXED_64x128 ? 64 : 32; }
int mixed_tile_n(MixedShape shape) { return shape == MIXED_64x128 ? 128 : 64; }

int64_t mixed_tile_count(const MixedTask &t, MixedShape shape) {
  const int bm = mixed_tile_m(shape), bn = mixed_tile_n(shape);
  return (int64_t)((t.M + bm - 1) / bm) * ((t.N + bn - 1) / bn);
}

hipError_t launch_gemm_mixed(const MixedTask *d_tasks, int n_tasks,
                             int64_t n_tiles, const uint16_t *A, int64_t a_ps,
                             const uint16_t *B, int64_t b_ps, double *C,
                             const int32_t *rows, MixedShape shape,
                             hipStream_t s) {
  if (n_tasks <= 0 || n_tiles <= 0) return hipSuccess;
  MixedArgs g{A, B, a_ps, b_ps, C, rows};
  if (shape == MIXED_64x128)
    hipLaunchKernelGGL(gemm_mixed_proj_lds_kernel, dim3((unsigned)n_tiles), dim3(256), 0, s,
                       d_tasks, n_tasks, g);
  else
    hipLaunchKernelGGL((gemm_mixed_kernel<1, 2, true, true>), dim3((unsigned)n_tiles),
                       dim3(256), 0, s, d_tasks, n_tasks, g);
  return hipGetLastError();
}

}  // namespace mbe3
