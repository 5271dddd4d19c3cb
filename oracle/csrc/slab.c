/*
 * Oracle side (TEST INFRASTRUCTURE ONLY; the product path never loads this
 * file's library).  Plain C, no code shared with the HIP library.
 *
 * The regenerated RI slab that stands in for the fitted Gamma_i of the
 * paper's eq. fitting (direct Gamma_i generator, Algorithm 1):
 *   B_i[a][P] = (z * w_ia[a]) * w_iP[P]
 * with z the Box-Muller normal (Box & Muller, 1958) of words 0 and 1 of the
 * Philox4x64-10 block (Salmon, Moraes, Dror and Shaw, SC'11) at counter
 * (P, a, i, 0) under key (seed, stream):
 *   u1 = ((w0 >> 11) + 0.5) 2^-53,  u2 = (w1 >> 11) 2^-53,
 *   z  = sqrt(-2 ln u1) cos(2 pi u2).
 * The same definition as the numpy routine of the oracle, in C for the
 * large workloads (tens of millions of elements per slab).
 */
#include <math.h>
#include <stdint.h>

/* Philox4x64 round multipliers and key increments, as published. */
#define PH_M0 0xD2E7470EE14C6C93ULL
#define PH_M1 0xCA5A826395121157ULL
#define PH_W0 0x9E3779B97F4A7C15ULL
#define PH_W1 0xBB67AE8584CAA73BULL

static void philox4x64_10(const uint64_t in[4], uint64_t k0, uint64_t k1,
                          uint64_t out[4]) {
  uint64_t x0 = in[0], x1 = in[1], x2 = in[2], x3 = in[3];
  for (int r = 0; r < 10; ++r) {
    if (r) {
      k0 += PH_W0;
      k1 += PH_W1;
    }
    const unsigned __int128 p0 = (unsigned __int128)PH_M0 * x0;
    const unsigned __int128 p1 = (unsigned __int128)PH_M1 * x2;
    const uint64_t hi0 = (uint64_t)(p0 >> 64), lo0 = (uint64_t)p0;
    const uint64_t hi1 = (uint64_t)(p1 >> 64), lo1 = (uint64_t)p1;
    const uint64_t n0 = hi1 ^ x1 ^ k0, n2 = hi0 ^ x3 ^ k1;
    x0 = n0;
    x1 = lo1;
    x2 = n2;
    x3 = lo0;
  }
  out[0] = x0;
  out[1] = x1;
  out[2] = x2;
  out[3] = x3;
}

/* Raw Philox words for n counters (tests compare them with numpy's). */
void oracle_philox_raw(const uint64_t *ctr, int64_t n, uint64_t k0, uint64_t k1,
                       uint64_t *out) {
#pragma omp parallel for schedule(static)
  for (int64_t e = 0; e < n; ++e) philox4x64_10(ctr + 4 * e, k0, k1, out + 4 * e);
}

/* out[a * n_cols + c] = (z(cols[c], a) * w_row[a]) * w_col[cols[c]] for
   a < n_rows, with z at counter (cols[c], a, w2, 0) under key (k0, k1).
   w_row / w_col NULL means 1 (plain normals). */
void oracle_normal_slab(uint64_t k0, uint64_t k1, uint64_t w2, int64_t n_rows,
                        int64_t n_cols, const int64_t *cols, const double *w_row,
                        const double *w_col, double *out) {
  const double two53 = 1.0 / 9007199254740992.0; /* 2^-53 */
#pragma omp parallel for schedule(static)
  for (int64_t a = 0; a < n_rows; ++a) {
    for (int64_t c = 0; c < n_cols; ++c) {
      const uint64_t P = (uint64_t)cols[c];
      const uint64_t ctr[4] = {P, (uint64_t)a, w2, 0};
      uint64_t w[4];
      philox4x64_10(ctr, k0, k1, w);
      const double u1 = ((double)(w[0] >> 11) + 0.5) * two53;
      const double u2 = (double)(w[1] >> 11) * two53;
      double z = sqrt(-2.0 * log(u1)) * cos((2.0 * 3.141592653589793) * u2);
      if (w_row) z = z * w_row[a];
      if (w_col) z = z * w_col[P];
      out[a * n_cols + c] = z;
    }
  }
}
