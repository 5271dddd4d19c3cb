// Pair screening (eq. s2b) and the weak-pair energies (eqs. osv_weak_k,
// res_weak): the reductions that close the grouped GEMM chains planned by
// mbe3_screen and mbe3_weak_pairs.  One wave per pair; sums run lane-strided
// over the pair's block and end in a fixed xor tree, so every result is
// reproducible bit for bit.
#include "internal.hpp"

namespace mbe3 {

__device__ __forceinline__ double wave_sum(double v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  return v;
}

// s2b_ij = sum of the squares of the r_i x r_j block S_(i,j) = Q_i^T Q_j at
// k_off, divided by sqrt(r_i r_j).
__global__ __launch_bounds__(256) void s2b_kernel(const WeakPair *__restrict__ wp, int n,
                                                  const double *__restrict__ S,
                                                  double *__restrict__ out) {
  const int lane = threadIdx.x & 63;
  const int p = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (p >= n) return;
  const WeakPair w = wp[p];
  const double *s = S + w.k_off;
  const int m = w.ri * w.rj;
  double acc = 0.0;
  for (int e = lane; e < m; e += 64) acc += s[e] * s[e];
  acc = wave_sum(acc);
  if (lane == 0) out[p] = acc / sqrt((double)w.ri * (double)w.rj);
}

// e_ij = 4 sum_{a < rank_i, b < rank_j} K~_ab (K~_ab - f_ij D~_ab)
//                                       / (f_ii + f_jj - eps~_i[a] - eps~_j[b])
// with K~ = X_i^T K_(i,j) X_j and D~ = X_i^T (T_ii S_(i,j) + S_(i,j) T_jj) X_j
// (D_i x D_j blocks at t_off): the one-block amplitudes in the diagonal
// pairs' bases, contracted with K~.
__global__ __launch_bounds__(256) void weak_energy_kernel(
    const WeakPair *__restrict__ wp, int n, const double *__restrict__ Kt,
    const double *__restrict__ Dt, const double *__restrict__ et,
    const int32_t *__restrict__ rank, const double *__restrict__ f, int n_occ,
    double *__restrict__ e) {
  const int lane = threadIdx.x & 63;
  const int p = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (p >= n) return;
  const WeakPair w = wp[p];
  const int rki = rank[w.i], rkj = rank[w.j];
  const double fii = f[(int64_t)w.i * n_occ + w.i];
  const double fjj = f[(int64_t)w.j * n_occ + w.j];
  const double fij = f[(int64_t)w.i * n_occ + w.j];
  const double *kt = Kt + w.t_off;
  const double *dt = Dt + w.t_off;
  const double *ei = et + w.ei;
  const double *ej = et + w.ej;
  double acc = 0.0;
  for (int x = lane; x < rki * rkj; x += 64) {
    const int a = x / rkj, b = x - a * rkj;
    const int64_t ab = (int64_t)a * w.Dj + b;
    const double k = kt[ab];
    acc += k * (k - fij * dt[ab]) / (fii + fjj - ei[a] - ej[b]);
  }
  acc = wave_sum(acc);
  if (lane == 0) e[p] = 4.0 * acc;
}

hipError_t launch_s2b(const WeakPair *wp, int n, const double *S, double *out,
                      hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(s2b_kernel, dim3((unsigned)((n + 3) / 4)), dim3(256), 0, s, wp, n, S,
                     out);
  return hipGetLastError();
}

hipError_t launch_weak_energy(const WeakPair *wp, int n, const double *Kt, const double *Dt,
                              const double *et, const int32_t *rank, const double *f,
                              int n_occ, double *e, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(weak_energy_kernel, dim3((unsigned)((n + 3) / 4)), dim3(256), 0, s, wp,
                     n, Kt, Dt, et, rank, f, n_occ, e);
  return hipGetLastError();
}

}  // namespace mbe3
