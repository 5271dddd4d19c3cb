// MBE(3) energy reductions.
//
// E = sum_F c_F E_F with c_F the inclusion-exclusion coefficients of the
// MBE(3) sum (c_ijk = 1, c_ij = 1 - #trimers containing ij,
// c_i = 1 - #pairs containing i + #trimers containing i), evaluated in a
// fixed order in double-double arithmetic (Knuth's TwoSum and the exact
// product by fma), so the result does not depend on launch shape and is
// faithfully rounded for these magnitudes.  The monomer coefficients are
// large (order #trimers per orbital), so the cancellation in the sum is
// severe and plain summation would lose digits.
#include "internal.hpp"

namespace mbe3 {

struct dd {
  double hi, lo;
};

__device__ __forceinline__ dd two_sum(double a, double b) {
  const double s = a + b;
  const double bb = s - a;
  const double e = (a - (s - bb)) + (b - bb);
  return {s, e};
}

__device__ __forceinline__ dd dd_add(dd x, dd y) {
  dd s = two_sum(x.hi, y.hi);
  const double lo = s.lo + x.lo + y.lo;
  return two_sum(s.hi, lo);
}

__device__ __forceinline__ dd dd_mul_dd(double a, double b) {
  const double p = a * b;
  const double e = fma(a, b, -p);
  return {p, e};
}

// One workgroup of 1024 threads; thread k sums the strided subset k, k+1024,
// ...; then a fixed binary tree in LDS.
__global__ __launch_bounds__(1024) void mbe_sum_kernel(
    const double *__restrict__ e, const double *__restrict__ c, int64_t n,
    double *__restrict__ out2) {
  __shared__ double sh_hi[1024];
  __shared__ double sh_lo[1024];
  dd acc = {0.0, 0.0};
  for (int64_t k = threadIdx.x; k < n; k += 1024)
    acc = dd_add(acc, c ? dd_mul_dd(c[k], e[k]) : dd{e[k], 0.0});
  sh_hi[threadIdx.x] = acc.hi;
  sh_lo[threadIdx.x] = acc.lo;
  __syncthreads();
  for (int w = 512; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) {
      dd x = {sh_hi[threadIdx.x], sh_lo[threadIdx.x]};
      dd y = {sh_hi[threadIdx.x + w], sh_lo[threadIdx.x + w]};
      dd z = dd_add(x, y);
      sh_hi[threadIdx.x] = z.hi;
      sh_lo[threadIdx.x] = z.lo;
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    out2[0] = sh_hi[0] + sh_lo[0];
    out2[1] = sh_hi[0];
    out2[2] = sh_lo[0];
  }
}

hipError_t launch_mbe_sum(const double *e_frag, const double *coef, int64_t n,
                          double *out2, hipStream_t s) {
  hipLaunchKernelGGL(mbe_sum_kernel, dim3(1), dim3(1024), 0, s, e_frag, coef, n,
                     out2);
  return hipGetLastError();
}

// First-order energy change of a change of the pair integrals, per slot:
//   per_slot[s] = c_s <K_a,s - K_b,s, W_s>,  c_s = 2 (diagonal slot s < n_occ),
//                                              c_s = 4 (pair slot),
// with W the multipliers of fragment_solve (dE/dK_s = c_s W_s).  One
// workgroup per slot: each thread sums a strided share of the slot's
// elements in order, then a fixed tree in LDS.
__global__ __launch_bounds__(256) void slot_dot_kernel(
    const double *__restrict__ Ka, const double *__restrict__ Kb,
    const double *__restrict__ W, const int64_t *__restrict__ k_off, int n_occ,
    int64_t n_slot, double *__restrict__ per_slot) {
  __shared__ double sh[256];
  for (int64_t sl = blockIdx.x; sl < n_slot; sl += gridDim.x) {
    const int64_t o0 = k_off[sl], o1 = k_off[sl + 1];
    double acc = 0.0;
    for (int64_t e = o0 + threadIdx.x; e < o1; e += 256) acc += (Ka[e] - Kb[e]) * W[e];
    sh[threadIdx.x] = acc;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
      if ((int)threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
      __syncthreads();
    }
    if (threadIdx.x == 0) per_slot[sl] = (sl < n_occ ? 2.0 : 4.0) * sh[0];
    __syncthreads();
  }
}

hipError_t launch_slot_dot(const double *Ka, const double *Kb, const double *W,
                           const int64_t *k_off, int n_occ, int64_t n_slot,
                           double *per_slot, hipStream_t s) {
  if (n_slot <= 0) return hipSuccess;
  const unsigned blocks = (unsigned)(n_slot < 65536 ? n_slot : 65536);
  hipLaunchKernelGGL(slot_dot_kernel, dim3(blocks), dim3(256), 0, s, Ka, Kb, W, k_off,
                     n_occ, n_slot, per_slot);
  return hipGetLastError();
}

// Increments: sub[f][0..5] = fragment indices of the sub-fragments
// (monomers i, j, k then dimers ij, ik, jk; -1 when absent).
__global__ void increments_kernel(const double *__restrict__ e,
                                  const int32_t *__restrict__ sub, int64_t n,
                                  double *__restrict__ incr) {
  for (int64_t f = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; f < n;
       f += (int64_t)gridDim.x * blockDim.x) {
    const int32_t *s = sub + 6 * f;
    double v = e[f];
    if (s[3] >= 0) {  // trimer: E_ijk - dE_ij - dE_ik - dE_jk - E_i - E_j - E_k
      const double ei = e[s[0]], ej = e[s[1]], ek = e[s[2]];
      const double dij = e[s[3]] - ei - ej;
      const double dik = e[s[4]] - ei - ek;
      const double djk = e[s[5]] - ej - ek;
      v = v - dij - dik - djk - ei - ej - ek;
    } else if (s[1] >= 0) {  // dimer: E_ij - E_i - E_j
      v = v - e[s[0]] - e[s[1]];
    }
    incr[f] = v;
  }
}

hipError_t launch_increments(const double *e_frag, const int32_t *sub,
                             int64_t n, double *incr, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  int64_t blocks = (n + 255) / 256;
  if (blocks > 4096) blocks = 4096;
  hipLaunchKernelGGL(increments_kernel, dim3((unsigned)blocks), dim3(256), 0, s,
                     e_frag, sub, n, incr);
  return hipGetLastError();
}

}  // namespace mbe3
