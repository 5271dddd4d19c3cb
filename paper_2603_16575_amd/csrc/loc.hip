// Occupied-orbital localization (the paper's section on occupied orbital
// localization: Alg. 2, eq. loc_theta): Pipek-Mezey with Jacobi sweeps on
// Loewdin charges.
//
//   pm_charges_kernel  P^A_ij = sum_{alpha in A} C~_{alpha i} C~_{alpha j},
//                      stored P[(i n + j) n_atom + A] (atoms fastest, so a
//                      pair's three charge vectors and a row's update run
//                      along contiguous memory)
//   pm_jacobi_kernel   one workgroup walks the pairs i < j in order, as the
//                      algorithm does (each rotation changes the charges the
//                      next pair reads): a_ij and b_ij reduced over the
//                      atoms, 4 theta = atan2(b, -a), the increment
//                      sqrt(a^2 + b^2)(1 - cos 4 theta), then the rotation
//                      of the columns i, j of U and of the first and the
//                      second orbital index of every P^A, spread over the
//                      workgroup's threads; sweeps repeat while the last
//                      sweep's summed increment exceeds l_loc.
// Sums run in a fixed order (lane-strided, xor butterfly per wave, waves in
// order), so the result is reproducible bit for bit.
#include "internal.hpp"

namespace mbe3 {

__global__ __launch_bounds__(256) void pm_charges_kernel(const double *__restrict__ C,
                                                         const int32_t *__restrict__ ao_off,
                                                         int n, int na, double *__restrict__ P) {
  const int64_t total = (int64_t)n * n * na;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int A = (int)(e % na);
    const int64_t ij = e / na;
    const int i = (int)(ij / n), j = (int)(ij - (int64_t)i * n);
    double acc = 0.0;
    for (int al = ao_off[A]; al < ao_off[A + 1]; ++al)
      acc += C[(int64_t)al * n + i] * C[(int64_t)al * n + j];
    P[e] = acc;
  }
}

hipError_t launch_pm_charges(const double *C, const int32_t *ao_off, int n, int na, double *P,
                             hipStream_t s) {
  const int64_t total = (int64_t)n * n * na;
  if (total <= 0) return hipSuccess;
  int64_t blocks = (total + 255) / 256;
  if (blocks > 65536) blocks = 65536;
  hipLaunchKernelGGL(pm_charges_kernel, dim3((unsigned)blocks), dim3(256), 0, s, C, ao_off, n,
                     na, P);
  return hipGetLastError();
}

static constexpr int PM_THREADS = 1024;
static constexpr int PM_WAVES = PM_THREADS / 64;

__device__ __forceinline__ double pm_wave_sum(double v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// rec[2 * sweep] = summed increment of the sweep, rec[2 * sweep + 1] =
// rotations applied in it (as a double); rec[2 * max_sweeps] = sweeps run.
__global__ __launch_bounds__(PM_THREADS) void pm_jacobi_kernel(double *__restrict__ P,
                                                               double *__restrict__ U, int n,
                                                               int na, double l_loc,
                                                               int max_sweeps,
                                                               double *__restrict__ rec) {
  __shared__ double red_a[PM_WAVES], red_b[PM_WAVES];
  __shared__ double cs_c, cs_s;
  __shared__ int do_rot, go;
  const int tid = threadIdx.x, wv = tid >> 6, lane = tid & 63;
  for (int64_t e = tid; e < (int64_t)n * n; e += PM_THREADS)
    U[e] = (e / n == e % n) ? 1.0 : 0.0;
  double dL = 0.0;  // thread 0's running sweep sum
  int nrot = 0, sweep = 0;
  if (tid == 0) go = max_sweeps > 0;
  __syncthreads();
  while (go) {
    if (tid == 0) { dL = 0.0; nrot = 0; }
    for (int i = 0; i < n; ++i) {
      for (int j = i + 1; j < n; ++j) {
        const double *pij = P + ((int64_t)i * n + j) * na;
        const double *pii = P + ((int64_t)i * n + i) * na;
        const double *pjj = P + ((int64_t)j * n + j) * na;
        double pa = 0.0, pb = 0.0;
        for (int A = tid; A < na; A += PM_THREADS) {
          const double x = pij[A], d = pii[A] - pjj[A];
          pa += x * x - 0.25 * d * d;
          pb += x * d;
        }
        pa = pm_wave_sum(pa);
        pb = pm_wave_sum(pb);
        if (lane == 0) { red_a[wv] = pa; red_b[wv] = pb; }
        __syncthreads();
        if (tid == 0) {
          double a = 0.0, b = 0.0;
          for (int w = 0; w < PM_WAVES; ++w) { a += red_a[w]; b += red_b[w]; }
          const double th = 0.25 * atan2(b, -a);
          const double s = sin(th), c = cos(th);
          const int r = fabs(s) >= 1e-10;
          if (r) {
            dL += sqrt(a * a + b * b) * (1.0 - cos(4.0 * th));
            ++nrot;
          }
          cs_c = c; cs_s = s; do_rot = r;
        }
        __syncthreads();
        if (!do_rot) continue;  // uniform: every thread read the same flag
        const double c = cs_c, s = cs_s;
        for (int k = tid; k < n; k += PM_THREADS) {  // columns i, j of U
          const double ui = U[(int64_t)k * n + i], uj = U[(int64_t)k * n + j];
          U[(int64_t)k * n + i] = c * ui + s * uj;
          U[(int64_t)k * n + j] = c * uj - s * ui;
        }
        double *ri = P + (int64_t)i * n * na, *rj = P + (int64_t)j * n * na;
        for (int64_t e = tid; e < (int64_t)n * na; e += PM_THREADS) {  // first index
          const double x = ri[e], y = rj[e];
          ri[e] = c * x + s * y;
          rj[e] = c * y - s * x;
        }
        __syncthreads();
        for (int64_t e = tid; e < (int64_t)n * na; e += PM_THREADS) {  // second index
          const int k = (int)(e / na), A = (int)(e - (int64_t)k * na);
          double *qi = P + ((int64_t)k * n + i) * na + A;
          double *qj = P + ((int64_t)k * n + j) * na + A;
          const double x = *qi, y = *qj;
          *qi = c * x + s * y;
          *qj = c * y - s * x;
        }
        __syncthreads();
      }
    }
    if (tid == 0) {
      rec[2 * sweep] = dL;
      rec[2 * sweep + 1] = (double)nrot;
      ++sweep;
      go = (sweep < max_sweeps) && (dL > l_loc);
    }
    __syncthreads();
  }
  if (tid == 0) rec[2 * max_sweeps] = (double)sweep;
}

hipError_t launch_pm_jacobi(double *P, double *U, int n, int na, double l_loc, int max_sweeps,
                            double *rec, hipStream_t s) {
  hipLaunchKernelGGL(pm_jacobi_kernel, dim3(1), dim3(PM_THREADS), 0, s, P, U, n, na, l_loc,
                     max_sweeps, rec);
  return hipGetLastError();
}

}  // namespace mbe3
