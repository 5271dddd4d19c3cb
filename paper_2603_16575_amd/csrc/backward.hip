// Backward kernels: gradient of the MBE(3) energy with respect to the slabs
// (ia|P) and the occupied Fock matrix, from Hylleraas stationarity (each
// fragment energy is stationary in its amplitudes, so only explicit
// dependences on K and f contribute).
//
//   W~_t     = sum_F c_F (2 Y^F_t - Y^F_t^T)        multipliers, X basis
//   dE/dK_s  = 4 W_s (pairs), 2 W_s (diagonal)    W_s = X_s W~_s X_s^T
//   dE/dG~   : K_s = L_s R_s^T gives dL = G R, dR = G^T L, contracted per
//              destination block (i, x) in one K-concatenated product
//   dE/dB_i  = sum_x Q_x dG~_{i,x}                (projection-shaped GEMM)
//   dE/df_xy = -sum_F c_F sum_terms w <Y~, S~ Y S~^T> - (E~ terms)
// Every reduction runs in a fixed order: the results are deterministic.
#include "internal.hpp"

namespace mbe3 {

// W~_slot += sum_entries c Y~ (Y~ = 2Y - Y^T stored by the solver), one
// workgroup per work item (an element range of a slot); every element sums
// its entries in fragment order.  A thread keeps WT_J elements in registers
// and reads WT_U entries ahead before adding them in order, so that each
// round trip to memory carries WT_U * WT_J independent loads.
constexpr int WT_J = 2, WT_U = 8;
__global__ __launch_bounds__(256) void wtilde_kernel(
    const WSlot *__restrict__ slots, const WEntry *__restrict__ ents,
    const double *__restrict__ yfin, double *__restrict__ wt) {
  const WSlot sl = slots[blockIdx.x];
  for (int base = 0; base < sl.n; base += 256 * WT_J) {
    double acc[WT_J];
#pragma unroll
    for (int j = 0; j < WT_J; ++j) {
      const int e = base + (int)threadIdx.x + 256 * j;
      acc[j] = e < sl.n ? wt[sl.wt_off + e] : 0.0;
    }
    int k = sl.e_begin;
    for (; k + WT_U <= sl.e_end; k += WT_U) {
      double c[WT_U], y[WT_U][WT_J];
#pragma unroll
      for (int u = 0; u < WT_U; ++u) {
        const WEntry en = ents[k + u];
        c[u] = en.coef;
        const double *yp = yfin + en.yoff + sl.y0;
#pragma unroll
        for (int j = 0; j < WT_J; ++j) {
          const int e = base + (int)threadIdx.x + 256 * j;
          y[u][j] = e < sl.n ? yp[e] : 0.0;
        }
      }
#pragma unroll
      for (int u = 0; u < WT_U; ++u)
#pragma unroll
        for (int j = 0; j < WT_J; ++j) acc[j] += c[u] * y[u][j];
    }
    for (; k < sl.e_end; ++k) {
      const WEntry en = ents[k];
      const double *yp = yfin + en.yoff + sl.y0;
#pragma unroll
      for (int j = 0; j < WT_J; ++j) {
        const int e = base + (int)threadIdx.x + 256 * j;
        if (e < sl.n) acc[j] += en.coef * yp[e];
      }
    }
#pragma unroll
    for (int j = 0; j < WT_J; ++j) {
      const int e = base + (int)threadIdx.x + 256 * j;
      if (e < sl.n) wt[sl.wt_off + e] = acc[j];
    }
  }
}

hipError_t launch_wtilde(const WSlot *slots, int n_slots, const WEntry *ents,
                         const double *yfin, double *wt, hipStream_t s) {
  if (n_slots <= 0) return hipSuccess;
  hipLaunchKernelGGL(wtilde_kernel, dim3(n_slots), dim3(256), 0, s, slots, ents,
                     yfin, wt);
  return hipGetLastError();
}

// g[dst] += sum_entries scale * (term or target scalar): one wave per
// destination; lane l sums entries l, l + 64, ... and a fixed xor tree
// combines the lanes (deterministic).
__global__ __launch_bounds__(256) void fgrad_kernel(
    const GDest *__restrict__ dests, int n, const GEntry *__restrict__ ents,
    const double *__restrict__ gterm, const double *__restrict__ gdiag,
    double *__restrict__ g) {
  const int lane = threadIdx.x & 63;
  const int wpb = blockDim.x >> 6;
  for (int d = blockIdx.x * wpb + (threadIdx.x >> 6); d < n; d += gridDim.x * wpb) {
    const GDest gd = dests[d];
    double acc = 0.0;
    for (int k = gd.e_begin + lane; k < gd.e_end; k += 64) {
      const GEntry e = ents[k];
      acc += e.scale * (e.kind ? gdiag[e.idx] : gterm[e.idx]);
    }
    for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o);
    if (lane == 0) g[gd.dst] += acc;
  }
}

hipError_t launch_fgrad(const GDest *dests, int n, const GEntry *ents,
                        const double *gterm, const double *gdiag, double *g,
                        hipStream_t s) {
  if (n <= 0) return hipSuccess;
  int blocks = (n + 3) / 4;
  if (blocks > 4096) blocks = 4096;
  hipLaunchKernelGGL(fgrad_kernel, dim3(blocks), dim3(256), 0, s, dests, n, ents,
                     gterm, gdiag, g);
  return hipGetLastError();
}

// One segment of a destination's concatenated G block:
//   mode 0: W[rc0 + r][k]  mode 1: W[k][rc0 + r]  mode 2: W[r][k] + W[k][r]
__global__ __launch_bounds__(256) void ga_kernel(const GASeg *__restrict__ segs,
                                                 const double *__restrict__ W,
                                                 double mult,
                                                 double *__restrict__ ga) {
  const GASeg g = segs[blockIdx.x];
  const double *w = W + g.w_off;
  for (int e = threadIdx.x; e < g.rows * g.kseg; e += blockDim.x) {
    const int r = e / g.kseg, k = e - r * g.kseg;
    double v;
    if (g.mode == 0) v = w[(int64_t)(g.rc0 + r) * g.w_ld + k];
    else if (g.mode == 1) v = w[(int64_t)k * g.w_ld + g.rc0 + r];
    else v = w[(int64_t)r * g.w_ld + k] + w[(int64_t)k * g.w_ld + r];
    ga[g.ga_off + (int64_t)r * g.ga_ld + g.k0 + k] = (mult * g.scale) * v;
  }
}

hipError_t launch_ga(const GASeg *segs, int n, const double *W, double mult,
                     double *ga, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(ga_kernel, dim3(n), dim3(256), 0, s, segs, W, mult, ga);
  return hipGetLastError();
}

// Double-double dot product: fixed grid of partials, then one combine.
struct ddv {
  double hi, lo;
};
__device__ __forceinline__ ddv dd_two_sum(double a, double b) {
  const double s = a + b;
  const double bb = s - a;
  return {s, (a - (s - bb)) + (b - bb)};
}
__device__ __forceinline__ ddv dd_plus(ddv x, ddv y) {
  ddv s = dd_two_sum(x.hi, y.hi);
  return dd_two_sum(s.hi, s.lo + x.lo + y.lo);
}

constexpr int DOT_BLOCKS = 1024;

__global__ __launch_bounds__(256) void dot_partial_kernel(
    const double *__restrict__ x, const double *__restrict__ y, int64_t n,
    double *__restrict__ part) {
  __shared__ double hi[256], lo[256];
  ddv acc = {0.0, 0.0};
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n;
       e += (int64_t)gridDim.x * blockDim.x) {
    const double p = x[e] * y[e];
    const double pe = fma(x[e], y[e], -p);
    acc = dd_plus(acc, ddv{p, pe});
  }
  hi[threadIdx.x] = acc.hi;
  lo[threadIdx.x] = acc.lo;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) {
      ddv z = dd_plus(ddv{hi[threadIdx.x], lo[threadIdx.x]},
                      ddv{hi[threadIdx.x + w], lo[threadIdx.x + w]});
      hi[threadIdx.x] = z.hi;
      lo[threadIdx.x] = z.lo;
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    part[2 * blockIdx.x] = hi[0];
    part[2 * blockIdx.x + 1] = lo[0];
  }
}

__global__ void dot_final_kernel(const double *__restrict__ part, int nb,
                                 double scale, double *__restrict__ out) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    ddv acc = {0.0, 0.0};
    for (int b = 0; b < nb; ++b) acc = dd_plus(acc, ddv{part[2 * b], part[2 * b + 1]});
    out[0] = scale * (acc.hi + acc.lo);
  }
}

hipError_t launch_dot(const double *x, const double *y, int64_t n, double scale,
                      double *part /* 2 * DOT_BLOCKS */, double *out,
                      hipStream_t s) {
  hipLaunchKernelGGL(dot_partial_kernel, dim3(DOT_BLOCKS), dim3(256), 0, s, x, y,
                     n, part);
  hipLaunchKernelGGL(dot_final_kernel, dim3(1), dim3(64), 0, s, part, DOT_BLOCKS,
                     scale, out);
  return hipGetLastError();
}
int dot_partials() { return DOT_BLOCKS; }

// out[x][y] = scale (g[x][y] + g[y][x]) / 2
__global__ void fsym_kernel(const double *__restrict__ g, int n, double scale,
                            double *__restrict__ out) {
  for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < n * n;
       e += gridDim.x * blockDim.x) {
    const int x = e / n, y = e - x * n;
    out[e] = scale * 0.5 * (g[x * n + y] + g[y * n + x]);
  }
}

hipError_t launch_fsym(const double *g, int n, double scale, double *out,
                       hipStream_t s) {
  const int tot = n * n;
  int blocks = (tot + 255) / 256;
  if (blocks > 4096) blocks = 4096;
  hipLaunchKernelGGL(fsym_kernel, dim3(blocks), dim3(256), 0, s, g, n, scale, out);
  return hipGetLastError();
}

}  // namespace mbe3
