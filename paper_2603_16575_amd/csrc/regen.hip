// Counter-based regeneration of the RI slabs (ia|P), standing in for the
// paper's direct Gamma_i generator (Algorithm 1): nothing is stored between
// uses, every element is a pure function of (seed, i, a, P).
//
// Philox4x64-10 (Salmon, Moraes, Dror, Shaw, SC'11): ten rounds of two
// 64x64->128-bit products with the Philox multipliers, high halves xored into
// the other words with the round key, key bumped by the Weyl constants
// between rounds.  Box-Muller (1958) on the top 53 bits of words 0 and 1.
// One thread per element; consecutive threads take consecutive P so the
// slab is written as coalesced rows of the [n_vir][n_aux] tile.
#include "internal.hpp"

namespace mbe3 {

__device__ __forceinline__ void philox4x64_10(uint64_t &c0, uint64_t &c1,
                                              uint64_t &c2, uint64_t &c3,
                                              uint64_t k0, uint64_t k1) {
  const uint64_t M0 = 0xD2E7470EE14C6C93ull, M1 = 0xCA5A826395121157ull;
  const uint64_t W0 = 0x9E3779B97F4A7C15ull, W1 = 0xBB67AE8584CAA73Bull;
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    if (r) { k0 += W0; k1 += W1; }
    const uint64_t hi0 = __umul64hi(M0, c0), lo0 = M0 * c0;
    const uint64_t hi1 = __umul64hi(M1, c2), lo1 = M1 * c2;
    const uint64_t n0 = hi1 ^ c1 ^ k0;
    const uint64_t n2 = hi0 ^ c3 ^ k1;
    c0 = n0; c1 = lo1; c2 = n2; c3 = lo0;
  }
}

__device__ __forceinline__ double box_muller(uint64_t w0, uint64_t w1) {
  const double u1 = ((double)(w0 >> 11) + 0.5) * 0x1p-53;
  const double u2 = (double)(w1 >> 11) * 0x1p-53;
  return sqrt(-2.0 * log(u1)) * cos((2.0 * M_PI) * u2);
}

// Element (a, P) of LMO i: w_ia w_iP (cb z_0 + cd z_10), z_s the normal of
// the Philox block at counter (P, a, i, 0) under key (seed, s).  cb = 1,
// cd = 0 gives the slab B itself (bit for bit w_ia w_iP z_0); cb = 0, cd = 1
// the gradient probe direction Delta (stream 10); cb = 1, cd = t the shifted
// slab B + t Delta of a finite-difference check.  cb and cd are uniform over
// the launch, so the skipped draw is a uniform branch.
__global__ __launch_bounds__(256) void regen_slab_kernel(
    double *__restrict__ out, int i0, int nb, int n_vir, int n_aux,
    uint64_t seed, const double *__restrict__ w_ia,
    const double *__restrict__ w_iP, double cb, double cd) {
  const int64_t per = (int64_t)n_vir * n_aux;
  const int64_t total = per * nb;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int b = (int)(e / per);
    const int64_t r = e - (int64_t)b * per;
    const int a = (int)(r / n_aux);
    const int P = (int)(r - (int64_t)a * n_aux);
    const int i = i0 + b;
    double z = 0.0;
    if (cb != 0.0) {
      uint64_t c0 = (uint64_t)P, c1 = (uint64_t)a, c2 = (uint64_t)i, c3 = 0;
      philox4x64_10(c0, c1, c2, c3, seed, 0ull);
      z = box_muller(c0, c1);
      if (cb != 1.0) z *= cb;
    }
    if (cd != 0.0) {
      uint64_t c0 = (uint64_t)P, c1 = (uint64_t)a, c2 = (uint64_t)i, c3 = 0;
      philox4x64_10(c0, c1, c2, c3, seed, (uint64_t)PROBE_STREAM);
      z += cd * box_muller(c0, c1);
    }
    out[e] = (z * w_ia[(int64_t)i * n_vir + a]) * w_iP[(int64_t)i * n_aux + P];
  }
}

// ---------------------------------------------------------------------------
// Split-precision operands.  x = h + m + l with h = bf16(x), m = bf16(x - h),
// l = bf16(x - h - m), the remainders formed in FP64 (exact): 24 significant
// bits, |x - h - m - l| <= 2^-24 |x| up to the tail rounding.  Pieces are
// stored as three planes of bf16 bit patterns, rows padded with zeros to ldk.
// ---------------------------------------------------------------------------
// Round to the nearest bf16, ties to even: FP64 -> FP32 (nearest even) and
// FP32 -> bf16 on the bit pattern.  The pieces only need to be close, but
// unbiased rounding keeps their tails unbiased too.
__device__ __forceinline__ uint16_t bf16_bits(double x) {
  const uint32_t u = __builtin_bit_cast(uint32_t, (float)x);
  return (uint16_t)((u + 0x7FFFu + ((u >> 16) & 1u)) >> 16);
}
__device__ __forceinline__ double bf16_value(uint16_t u) {
  return (double)(float)__builtin_bit_cast(__bf16, u);
}
__device__ __forceinline__ void split3(double x, uint16_t *dst, int64_t ps) {
  const uint16_t h = bf16_bits(x);
  const double r1 = x - bf16_value(h);
  const uint16_t m = bf16_bits(r1);
  const double r2 = r1 - bf16_value(m);
  dst[0] = h;
  dst[ps] = m;
  dst[2 * ps] = bf16_bits(r2);
}

// Slabs of LMOs i0 .. i0 + nb - 1 regenerated straight into split planes in
// the transposed layout [b][P][a] (a fastest, row pitch ldk >= n_vir, zero
// padded), the K-contiguous operand of the projection.  With an explicit
// slab (device [n_occ][n_vir][n_aux]) its values are split instead.
__global__ __launch_bounds__(256) void regen_split_kernel(
    uint16_t *__restrict__ planes, int64_t ps, int i0, int nb, int n_vir,
    int n_aux, int ldk, uint64_t seed, const double *__restrict__ w_ia,
    const double *__restrict__ w_iP, const double *__restrict__ slab) {
  const int64_t per = (int64_t)n_aux * ldk;
  const int64_t total = per * nb;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int b = (int)(e / per);
    const int64_t r = e - (int64_t)b * per;
    const int P = (int)(r / ldk);
    const int a = (int)(r - (int64_t)P * ldk);
    const int i = i0 + b;
    double x = 0.0;
    if (a < n_vir) {
      if (slab) {
        x = slab[((int64_t)i * n_vir + a) * n_aux + P];
      } else {
        uint64_t c0 = (uint64_t)P, c1 = (uint64_t)a, c2 = (uint64_t)i, c3 = 0;
        philox4x64_10(c0, c1, c2, c3, seed, 0ull);
        const double z = box_muller(c0, c1);
        x = (z * w_ia[(int64_t)i * n_vir + a]) * w_iP[(int64_t)i * n_aux + P];
      }
    }
    split3(x, planes + e, ps);
  }
}

// Rows of a row-major FP64 matrix (rows x cols, leading dimension ld) into
// split planes with row pitch ldk >= cols (zero padded).
__global__ __launch_bounds__(256) void split_rows_kernel(
    const double *__restrict__ x, int64_t rows, int cols, int64_t ld,
    uint16_t *__restrict__ planes, int64_t ps, int ldk) {
  const int64_t total = rows * ldk;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t rw = e / ldk;
    const int c = (int)(e - rw * ldk);
    split3(c < cols ? x[rw * ld + c] : 0.0, planes + e, ps);
  }
}

// Rows for the pair_K operands: all three pieces on fixed-point grids of the
// row, x ~ (H1 + H2 / 256 + H3 / 65536) u with integers |Hk| <= 128 and
// u = 2^(e - 7), 2^e above the row's largest magnitude (representation error
// at most u / 2^17, i.e. 2^-23 of the row's largest).  A product of two
// pieces of two such rows is then an integer multiple of one unit per product
// class, at most 2^14 units, so every 32-deep block is summed exactly by the
// matrix cores.  Their product adder drops the bits of each product that lie
// far below the block's largest one, which biases a sum downward however the
// products' signs fall; exact classes leave no such bias.  One wave per row.
__global__ __launch_bounds__(256) void split_rows_fixed_kernel(
    const double *__restrict__ x, int64_t rows, int cols, int64_t ld,
    uint16_t *__restrict__ planes, int64_t ps, int ldk) {
  const int lane = threadIdx.x & 63;
  const int64_t rw = blockIdx.x * (int64_t)(blockDim.x >> 6) + (threadIdx.x >> 6);
  if (rw >= rows) return;
  const double *xr = x + rw * ld;
  double mx = 0.0;
  for (int c = lane; c < cols; c += 64) mx = fmax(mx, fabs(xr[c]));
  for (int o = 32; o > 0; o >>= 1) mx = fmax(mx, __shfl_xor(mx, o));
  int e = 0;
  if (mx > 0.0) frexp(mx, &e);  // mx < 2^e
  uint16_t *pr = planes + rw * ldk;
  for (int c = lane; c < ldk; c += 64) {
    double r = c < cols ? xr[c] : 0.0;
#pragma unroll
    for (int p = 0; p < 3; ++p) {  // |r| <= 2^(e - 8p) - 1/2 grid step
      const int sh = 7 + 8 * p;
      const double hv = rint(ldexp(r, sh - e));  // |hv| <= 128: exact in bf16
      pr[p * ps + c] = bf16_bits(ldexp(hv, e - sh));
      r -= ldexp(hv, e - sh);
    }
  }
}

static int64_t grid_for(int64_t total) {
  int64_t blocks = (total + 255) / 256;
  return blocks > 65536 ? 65536 : blocks;
}

hipError_t launch_regen_split(uint16_t *planes, int64_t ps, int i0, int nb,
                              int n_vir, int n_aux, int ldk, uint64_t seed,
                              const double *w_ia, const double *w_iP,
                              const double *slab, hipStream_t s) {
  const int64_t total = (int64_t)n_aux * ldk * nb;
  if (total <= 0) return hipSuccess;
  hipLaunchKernelGGL(regen_split_kernel, dim3((unsigned)grid_for(total)), dim3(256),
                     0, s, planes, ps, i0, nb, n_vir, n_aux, ldk, seed, w_ia,
                     w_iP, slab);
  return hipGetLastError();
}

hipError_t launch_split_rows(const double *x, int64_t rows, int cols, int64_t ld,
                             uint16_t *planes, int64_t ps, int ldk,
                             hipStream_t s) {
  const int64_t total = rows * ldk;
  if (total <= 0) return hipSuccess;
  hipLaunchKernelGGL(split_rows_kernel, dim3((unsigned)grid_for(total)), dim3(256),
                     0, s, x, rows, cols, ld, planes, ps, ldk);
  return hipGetLastError();
}

hipError_t launch_split_rows_fixed(const double *x, int64_t rows, int cols, int64_t ld,
                                   uint16_t *planes, int64_t ps, int ldk, hipStream_t s) {
  if (rows <= 0) return hipSuccess;
  const int64_t blocks = (rows + 3) / 4;
  if (blocks > 0x7fffffffLL) return hipErrorInvalidValue;
  hipLaunchKernelGGL(split_rows_fixed_kernel, dim3((unsigned)blocks), dim3(256), 0, s, x,
                     rows, cols, ld, planes, ps, ldk);
  return hipGetLastError();
}

hipError_t launch_regen_slab(double *out, int i0, int nb, int n_vir, int n_aux,
                             uint64_t seed, const double *w_ia,
                             const double *w_iP, double cb, double cd, hipStream_t s) {
  const int64_t total = (int64_t)n_vir * n_aux * nb;
  if (total <= 0) return hipSuccess;
  int64_t blocks = (total + 255) / 256;
  if (blocks > 65536) blocks = 65536;
  hipLaunchKernelGGL(regen_slab_kernel, dim3((unsigned)blocks), dim3(256), 0, s,
                     out, i0, nb, n_vir, n_aux, seed, w_ia, w_iP, cb, cd);
  return hipGetLastError();
}


// ---------------------------------------------------------------------------
// Sparse fitting domains (eq. sparse_fit_metric).  s_fit[i][P] is the sum
// over a of B_i[a][P]^2, one thread per (i, P), summed in increasing a; the
// slab elements are regenerated exactly as regen_slab_kernel writes them
// (or read from a given [n_occ][n_vir][n_aux] slab), so nothing is stored.
// Consecutive threads take consecutive P: the w_iP and given-slab reads are
// coalesced rows, w_ia a broadcast.
__global__ __launch_bounds__(256) void fit_metric_kernel(
    double *__restrict__ s_fit, int n_occ, int n_vir, int n_aux, uint64_t seed,
    const double *__restrict__ w_ia, const double *__restrict__ w_iP,
    const double *__restrict__ slab) {
  const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (e >= (int64_t)n_occ * n_aux) return;
  const int i = (int)(e / n_aux);
  const int P = (int)(e - (int64_t)i * n_aux);
  double s = 0.0;
  if (slab) {
    const double *b = slab + (int64_t)i * n_vir * n_aux + P;
    for (int a = 0; a < n_vir; ++a) {
      const double v = b[(int64_t)a * n_aux];
      s += v * v;
    }
  } else {
    const double wp = w_iP[e];
    const double *wa = w_ia + (int64_t)i * n_vir;
    for (int a = 0; a < n_vir; ++a) {
      uint64_t c0 = (uint64_t)P, c1 = (uint64_t)a, c2 = (uint64_t)i, c3 = 0;
      philox4x64_10(c0, c1, c2, c3, seed, 0ull);
      const double v = (box_muller(c0, c1) * wa[a]) * wp;
      s += v * v;
    }
  }
  s_fit[e] = s;
}

// Restriction of gamma-layout rows (Gamma~, or a gradient with respect to
// it) to the columns the fitting domains select for them (eq. osv_imua):
// a row of block (i, x), x != i, keeps P when P is in D_i or D_x; a row of
// the diagonal block (i, i) keeps P when P is in D_q for some q in N+(i),
// the union of the pair domains D_i u D_q of every pair that reads it
// (eq. osv_close_k).  D_q = {P : s_fit[q][P] > l_fit}.  Other elements
// become zero; kept elements are neither read nor written.  Threads run
// along P (coalesced), workgroups stride over rows.
__global__ __launch_bounds__(256) void fit_mask_kernel(
    double *__restrict__ g, int64_t rows, int n_aux,
    const int32_t *__restrict__ row_lmo, const int32_t *__restrict__ row_x,
    const int32_t *__restrict__ nbr_off, const int32_t *__restrict__ nbr,
    const double *__restrict__ s_fit, double l_fit) {
  const int P = blockIdx.x * 256 + threadIdx.x;
  if (P >= n_aux) return;
  for (int64_t row = blockIdx.y; row < rows; row += gridDim.y) {
    const int i = row_lmo[row], x = row_x[row];
    bool keep;
    if (x != i) {
      keep = s_fit[(int64_t)i * n_aux + P] > l_fit || s_fit[(int64_t)x * n_aux + P] > l_fit;
    } else {
      keep = false;
      for (int k = nbr_off[i]; k < nbr_off[i + 1] && !keep; ++k)
        keep = s_fit[(int64_t)nbr[k] * n_aux + P] > l_fit;
    }
    if (!keep) g[row * n_aux + P] = 0.0;
  }
}

// The kept columns of a batch of slabs, compacted: for LMO i = i0 + b with
// domain columns cols[col_off[i] .. col_off[i + 1]) (nc of them),
//   out[out_off[b] + a * nc + c] = B_i[a][cols[col_off[i] + c]],
// each element regenerated exactly as regen_slab_kernel writes it (or read
// from a given slab).  One workgroup row (blockIdx.y) per LMO of the batch.
__global__ __launch_bounds__(256) void regen_cols_kernel(
    double *__restrict__ out, const int64_t *__restrict__ out_off,
    const int32_t *__restrict__ cols, const int32_t *__restrict__ col_off, int i0,
    int n_vir, int n_aux, uint64_t seed, const double *__restrict__ w_ia,
    const double *__restrict__ w_iP, const double *__restrict__ slab) {
  const int i = i0 + (int)blockIdx.y;
  const int c0 = col_off[i], nc = col_off[i + 1] - c0;
  const int64_t total = (int64_t)n_vir * nc;
  double *o = out + out_off[blockIdx.y];
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int a = (int)(e / nc);
    const int P = cols[c0 + (int)(e - (int64_t)a * nc)];
    double v;
    if (slab) {
      v = slab[((int64_t)i * n_vir + a) * n_aux + P];
    } else {
      uint64_t k0 = (uint64_t)P, k1 = (uint64_t)a, k2 = (uint64_t)i, k3 = 0;
      philox4x64_10(k0, k1, k2, k3, seed, 0ull);
      v = (box_muller(k0, k1) * w_ia[(int64_t)i * n_vir + a]) * w_iP[(int64_t)i * n_aux + P];
    }
    o[e] = v;
  }
}

// Compacted gamma rows back into the dense layout: row r of LMO i (r from
// g_off[i]) holds its nc kept columns at gc[gc_off[i] + (r - g_off[i]) nc];
// they go to columns cols[col_off[i] + c] of the dense row (the others were
// zeroed before).  Threads along the kept columns, workgroups over rows.
__global__ __launch_bounds__(256) void fit_scatter_kernel(
    double *__restrict__ g, const double *__restrict__ gc, int64_t rows, int n_aux,
    const int32_t *__restrict__ row_lmo, const int64_t *__restrict__ g_off,
    const int64_t *__restrict__ gc_off, const int32_t *__restrict__ cols,
    const int32_t *__restrict__ col_off) {
  for (int64_t row = blockIdx.y; row < rows; row += gridDim.y) {
    const int i = row_lmo[row];
    const int c0 = col_off[i], nc = col_off[i + 1] - c0;
    const double *src = gc + gc_off[i] + (row - g_off[i]) * nc;
    for (int c = blockIdx.x * 256 + threadIdx.x; c < nc; c += gridDim.x * 256)
      g[row * n_aux + cols[c0 + c]] = src[c];
  }
}

hipError_t launch_regen_cols(double *out, const int64_t *out_off, const int32_t *cols,
                             const int32_t *col_off, int i0, int nb, int64_t max_elems,
                             int n_vir, int n_aux, uint64_t seed, const double *w_ia,
                             const double *w_iP, const double *slab, hipStream_t s) {
  if (nb <= 0 || max_elems <= 0) return hipSuccess;
  if (nb > 65535) return hipErrorInvalidValue;
  int64_t gx = (max_elems + 255) / 256;
  if (gx > 1024) gx = 1024;
  hipLaunchKernelGGL(regen_cols_kernel, dim3((unsigned)gx, (unsigned)nb), dim3(256), 0, s,
                     out, out_off, cols, col_off, i0, n_vir, n_aux, seed, w_ia, w_iP, slab);
  return hipGetLastError();
}

hipError_t launch_fit_scatter(double *g, const double *gc, int64_t rows, int n_aux,
                              int max_nc, const int32_t *row_lmo, const int64_t *g_off,
                              const int64_t *gc_off, const int32_t *cols,
                              const int32_t *col_off, hipStream_t s) {
  if (rows <= 0 || max_nc <= 0) return hipSuccess;
  const unsigned gx = (unsigned)((max_nc + 255) / 256);
  const unsigned gy = (unsigned)(rows < 4096 ? rows : 4096);
  hipLaunchKernelGGL(fit_scatter_kernel, dim3(gx, gy), dim3(256), 0, s, g, gc, rows, n_aux,
                     row_lmo, g_off, gc_off, cols, col_off);
  return hipGetLastError();
}

// Gaussian test rows of the randomized OSV range finder: row s, column a of
// batch member b (LMO i0 + b) is the Box-Muller normal of the Philox block at
// counter (a, s, i, 0) under key (seed, stream); rows [n_rows][n_vir] per
// member, members n_rows * n_vir apart.
__global__ __launch_bounds__(256) void regen_gauss_kernel(double *__restrict__ out, int i0,
                                                          int nb, int n_rows, int n_vir,
                                                          uint64_t seed, uint64_t stream) {
  const int64_t per = (int64_t)n_rows * n_vir;
  const int64_t total = per * nb;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int b = (int)(e / per);
    const int64_t r = e - (int64_t)b * per;
    const int srow = (int)(r / n_vir);
    const int a = (int)(r - (int64_t)srow * n_vir);
    uint64_t c0 = (uint64_t)a, c1 = (uint64_t)srow, c2 = (uint64_t)(i0 + b), c3 = 0;
    philox4x64_10(c0, c1, c2, c3, seed, stream);
    out[e] = box_muller(c0, c1);
  }
}

hipError_t launch_regen_gauss(double *out, int i0, int nb, int n_rows, int n_vir,
                              uint64_t seed, uint64_t stream, hipStream_t s) {
  const int64_t total = (int64_t)nb * n_rows * n_vir;
  if (total <= 0) return hipSuccess;
  int64_t blocks = (total + 255) / 256;
  if (blocks > 65536) blocks = 65536;
  hipLaunchKernelGGL(regen_gauss_kernel, dim3((unsigned)blocks), dim3(256), 0, s, out, i0, nb,
                     n_rows, n_vir, seed, stream);
  return hipGetLastError();
}

hipError_t launch_fit_metric(double *s_fit, int n_occ, int n_vir, int n_aux,
                             uint64_t seed, const double *w_ia, const double *w_iP,
                             const double *slab, hipStream_t s) {
  const int64_t total = (int64_t)n_occ * n_aux;
  if (total <= 0) return hipSuccess;
  const int64_t blocks = (total + 255) / 256;
  if (blocks > 0x7fffffffLL) return hipErrorInvalidValue;
  hipLaunchKernelGGL(fit_metric_kernel, dim3((unsigned)blocks), dim3(256), 0, s,
                     s_fit, n_occ, n_vir, n_aux, seed, w_ia, w_iP, slab);
  return hipGetLastError();
}

hipError_t launch_fit_mask(double *g, int64_t rows, int n_aux, const int32_t *row_lmo,
                           const int32_t *row_x, const int32_t *nbr_off,
                           const int32_t *nbr, const double *s_fit, double l_fit,
                           hipStream_t s) {
  if (rows <= 0 || n_aux <= 0) return hipSuccess;
  const unsigned gx = (unsigned)((n_aux + 255) / 256);
  const unsigned gy = (unsigned)(rows < 4096 ? rows : 4096);
  hipLaunchKernelGGL(fit_mask_kernel, dim3(gx, gy), dim3(256), 0, s, g, rows, n_aux,
                     row_lmo, row_x, nbr_off, nbr, s_fit, l_fit);
  return hipGetLastError();
}

}  // namespace mbe3
