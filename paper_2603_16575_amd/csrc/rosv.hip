// Randomized OSV generation (the paper's randomized OSV section, Alg. 3):
// the pieces between the grouped GEMMs that the C-ABI call plans.
//
//   rosv_tscale_kernel   T_ii[a][b] /= (f_aa + f_bb - 2 f_ii)   (eq. mp2_tkk,
//                        after T = B_D B_D^T over the fitting domain)
//   range_finder_kernel  the adaptive randomized range finder on the rows of
//                        Y = G T: one workgroup per LMO walks the accepted
//                        rows s = 1, 2, ... while the largest of the r
//                        pending row norms exceeds the stopping bound; each
//                        step orthogonalises the first pending row against
//                        the accepted rows (eq. rsvd_za), normalises it,
//                        appends the next sample orthogonalised against the
//                        earlier rows, and removes the new direction from
//                        every pending row
//   rosv_finalize_kernel singular values w = sqrt(eigenvalues of T~ T~^T)
//                        (eq. tii_rsvd via the Gram matrix), rows of
//                        Q_i^T = Q~^T Z (eq. back_q) ordered by decreasing w,
//                        those with w >= l_osv kept
//
// All reductions run in a fixed order (lane-strided partial sums, a xor
// butterfly per wave, the four waves in order), so results are
// reproducible bit for bit.
#include "internal.hpp"

namespace mbe3 {

__global__ __launch_bounds__(256) void rosv_tscale_kernel(
    double *__restrict__ T, int i0, int nb, int n_vir, const double *__restrict__ eps,
    const double *__restrict__ f, int n_occ) {
  const int64_t per = (int64_t)n_vir * n_vir;
  const int64_t total = per * nb;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int b = (int)(e / per);
    const int64_t r = e - (int64_t)b * per;
    const int a = (int)(r / n_vir), c = (int)(r - (int64_t)a * n_vir);
    const int i = i0 + b;
    T[e] = T[e] / (eps[a] + eps[c] - 2.0 * f[(int64_t)i * n_occ + i]);
  }
}

hipError_t launch_rosv_tscale(double *T, int i0, int nb, int n_vir, const double *eps,
                              const double *f, int n_occ, hipStream_t s) {
  const int64_t total = (int64_t)nb * n_vir * n_vir;
  if (total <= 0) return hipSuccess;
  int64_t blocks = (total + 255) / 256;
  if (blocks > 65536) blocks = 65536;
  hipLaunchKernelGGL(rosv_tscale_kernel, dim3((unsigned)blocks), dim3(256), 0, s, T, i0, nb,
                     n_vir, eps, f, n_occ);
  return hipGetLastError();
}

__device__ __forceinline__ double rf_wave_sum(double v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// Sum over the workgroup (256 threads) of one value per thread, fixed order.
__device__ double rf_block_sum(double v, double *red) {
  v = rf_wave_sum(v);
  const int w = threadIdx.x >> 6;
  __syncthreads();
  if ((threadIdx.x & 63) == 0) red[w] = v;
  __syncthreads();
  return ((red[0] + red[1]) + red[2]) + red[3];
}

// <x, y> over n elements by one wave (lane-strided, then the butterfly).
__device__ __forceinline__ double rf_wave_dot(const double *__restrict__ x,
                                              const double *__restrict__ y, int n) {
  double acc = 0.0;
  for (int a = threadIdx.x & 63; a < n; a += 64) acc += x[a] * y[a];
  return rf_wave_sum(acc);
}

// Y: [nb][r + n_max][n_vir] (G T, rows 0..r-1 pending first, then the later
// samples, overwritten as they are orthogonalised); Z: [nb][n_max][n_vir]
// (accepted rows, zero beyond the count); rows[b]: accepted count.
__global__ __launch_bounds__(256) void range_finder_kernel(double *__restrict__ Y,
                                                           double *__restrict__ Z,
                                                           int32_t *__restrict__ rows, int r,
                                                           int n_max, int n_vir,
                                                           double thr) {
  extern __shared__ double rf_sm[];
  double *coef = rf_sm;               // n_max dot products
  double *nrm = coef + n_max;         // r pending norms
  double *red = nrm + r;              // 4 wave partials
  int *ring = (int *)(red + 4);       // r pending row indices, oldest first
  __shared__ int stop;
  const int b = blockIdx.x;
  double *Yb = Y + (int64_t)b * (r + n_max) * n_vir;
  double *Zb = Z + (int64_t)b * n_max * n_vir;
  const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
  for (int j = threadIdx.x; j < r; j += 256) ring[j] = j;
  __syncthreads();
  int s = 0;
  for (;;) {
    // largest pending row norm against the stopping bound
    for (int j = wv; j < r; j += 4) {
      const double *y = Yb + (int64_t)ring[j] * n_vir;
      const double q = rf_wave_dot(y, y, n_vir);
      if (lane == 0) nrm[j] = sqrt(q);
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      double mx = 0.0;
      for (int j = 0; j < r; ++j) mx = fmax(mx, nrm[j]);
      stop = (s >= n_max) || !(mx > thr);
    }
    __syncthreads();
    if (stop) break;
    double *y = Yb + (int64_t)ring[0] * n_vir;
    double *z = Zb + (int64_t)s * n_vir;
    // z~ = y - (y Z^T) Z over the s accepted rows (eq. rsvd_za)
    for (int k = wv; k < s; k += 4) {
      const double c = rf_wave_dot(y, Zb + (int64_t)k * n_vir, n_vir);
      if (lane == 0) coef[k] = c;
    }
    __syncthreads();
    double part = 0.0;
    for (int a = threadIdx.x; a < n_vir; a += 256) {
      double v = 0.0;
      for (int k = 0; k < s; ++k) v += coef[k] * Zb[(int64_t)k * n_vir + a];
      v = y[a] - v;
      z[a] = v;
      part += v * v;
    }
    const double inv = 1.0 / sqrt(rf_block_sum(part, red));
    for (int a = threadIdx.x; a < n_vir; a += 256) z[a] *= inv;
    // the next sample, against the rows accepted before this step
    double *yn = Yb + (int64_t)(r + s) * n_vir;
    __syncthreads();
    for (int k = wv; k < s; k += 4) {
      const double c = rf_wave_dot(yn, Zb + (int64_t)k * n_vir, n_vir);
      if (lane == 0) coef[k] = c;
    }
    __syncthreads();
    for (int a = threadIdx.x; a < n_vir; a += 256) {
      double v = 0.0;
      for (int k = 0; k < s; ++k) v += coef[k] * Zb[(int64_t)k * n_vir + a];
      yn[a] = yn[a] - v;
    }
    __syncthreads();
    // shift the pending rows, the new sample last
    if (threadIdx.x == 0) {
      for (int j = 0; j + 1 < r; ++j) ring[j] = ring[j + 1];
      ring[r - 1] = r + s;
    }
    __syncthreads();
    // remove the accepted direction from every pending row
    for (int j = wv; j < r; j += 4) {
      const double c = rf_wave_dot(Yb + (int64_t)ring[j] * n_vir, z, n_vir);
      if (lane == 0) nrm[j] = c;
    }
    __syncthreads();
    for (int j = 0; j < r; ++j) {
      double *yj = Yb + (int64_t)ring[j] * n_vir;
      const double c = nrm[j];
      for (int a = threadIdx.x; a < n_vir; a += 256) yj[a] = yj[a] - c * z[a];
    }
    __syncthreads();
    ++s;
  }
  for (int64_t e = (int64_t)s * n_vir + threadIdx.x; e < (int64_t)n_max * n_vir; e += 256)
    Zb[e] = 0.0;
  if (threadIdx.x == 0) rows[b] = s;
}

hipError_t launch_range_finder(double *Y, double *Z, int32_t *rows, int nb, int r, int n_max,
                               int n_vir, double thr, hipStream_t s) {
  if (nb <= 0) return hipSuccess;
  const size_t smem = sizeof(double) * ((size_t)n_max + r + 4) + sizeof(int) * (size_t)r;
  hipLaunchKernelGGL(range_finder_kernel, dim3(nb), dim3(256), smem, s, Y, Z, rows, r, n_max,
                     n_vir, thr);
  return hipGetLastError();
}

// evals: [nb][D] eigenvalues of T~ T~^T ascending (sentinel beyond rows[b]);
// Qr: [nb][n_max][n_vir], row k = eigenvector k applied to Z (ascending
// order).  Output: Q_out rows of LMO i0 + b at (i0 + b) * n_max, decreasing
// w, only w >= l_osv, zero rows after; w_out likewise; n_osv[i0 + b].
__global__ __launch_bounds__(256) void rosv_finalize_kernel(
    const double *__restrict__ evals, int D, const double *__restrict__ Qr,
    const int32_t *__restrict__ rows, int i0, int n_max, int n_vir, double l_osv,
    double *__restrict__ Q_out, double *__restrict__ w_out, int32_t *__restrict__ n_osv,
    int32_t *__restrict__ rows_out) {
  __shared__ int keep;
  const int b = blockIdx.x;
  const int s = rows[b];
  const double *ev = evals + (int64_t)b * D;
  if (threadIdx.x == 0) {
    int k = 0;
    for (int j = s - 1; j >= 0; --j) {
      const double w = sqrt(fmax(ev[j], 0.0));
      if (w >= l_osv) ++k; else break;  // decreasing: the rest are smaller
    }
    keep = k;
    n_osv[i0 + b] = k;
    rows_out[i0 + b] = s;
  }
  __syncthreads();
  const int k = keep;
  double *qo = Q_out + (int64_t)(i0 + b) * n_max * n_vir;
  const double *qr = Qr + (int64_t)b * n_max * n_vir;
  for (int64_t e = threadIdx.x; e < (int64_t)n_max * n_vir; e += 256) {
    const int mu = (int)(e / n_vir);
    const int a = (int)(e - (int64_t)mu * n_vir);
    qo[e] = mu < k ? qr[(int64_t)(s - 1 - mu) * n_vir + a] : 0.0;
  }
  for (int mu = threadIdx.x; mu < n_max; mu += 256)
    w_out[(int64_t)(i0 + b) * n_max + mu] = mu < k ? sqrt(fmax(ev[s - 1 - mu], 0.0)) : 0.0;
}

hipError_t launch_rosv_finalize(const double *evals, int D, const double *Qr,
                                const int32_t *rows, int i0, int nb, int n_max, int n_vir,
                                double l_osv, double *Q_out, double *w_out, int32_t *n_osv,
                                int32_t *rows_out, hipStream_t s) {
  if (nb <= 0) return hipSuccess;
  hipLaunchKernelGGL(rosv_finalize_kernel, dim3(nb), dim3(256), 0, s, evals, D, Qr, rows, i0,
                     n_max, n_vir, l_osv, Q_out, w_out, n_osv, rows_out);
  return hipGetLastError();
}

}  // namespace mbe3
