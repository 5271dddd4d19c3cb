// Preparation kernels: assembly of 4-block pair matrices from the OSV
// overlap / Fock block stores (eq. 4block_osv) and the eps-scaled copy of
// the packed OSVs used to form F_(x,y) = Q_x^T diag(eps) Q_y as a GEMM.
#include "internal.hpp"

namespace mbe3 {

__global__ __launch_bounds__(256) void assemble_kernel(
    const AssembleTask *__restrict__ tasks, const double *__restrict__ sstore,
    const double *__restrict__ fstore, double *__restrict__ out0,
    double *__restrict__ out1) {
  const AssembleTask t = tasks[blockIdx.x];
  const double *src = t.src_buf ? fstore : sstore;
  double *o = (t.out_buf ? out1 : out0) + t.out_off;
  const int rtot = t.rsz[0] + (t.nrb > 1 ? t.rsz[1] : 0);
  const int ctot = t.csz[0] + (t.ncb > 1 ? t.csz[1] : 0);
  const int lane = threadIdx.x & 63;
  // one wave per output row; the source blocks are picked with constant
  // indices (a dynamically indexed block table would live in scratch)
  for (int r = threadIdx.x >> 6; r < t.rows_out; r += blockDim.x >> 6) {
    const bool lower = r >= t.rsz[0];
    const int rl = lower ? r - t.rsz[0] : r;
    const BlockSrc bl = lower ? t.b[1][0] : t.b[0][0];
    const BlockSrc br = lower ? t.b[1][1] : t.b[0][1];
    for (int c = lane; c < t.cols_out; c += 64) {
      double v = 0.0;
      if (r < rtot && c < ctot) {
        const bool right = c >= t.csz[0];
        const int cl = right ? c - t.csz[0] : c;
        const int64_t off = right ? br.off : bl.off;
        const int64_t ld = right ? br.ld : bl.ld;
        const bool tr = right ? br.trans : bl.trans;
        v = tr ? src[off + cl * ld + rl] : src[off + rl * ld + cl];
      }
      o[(int64_t)r * t.ld_out + c] = v;
    }
  }
}

hipError_t launch_assemble(const AssembleTask *d_tasks, int n_tasks,
                           const double *sstore, const double *fstore,
                           double *out0, double *out1, hipStream_t s) {
  if (n_tasks <= 0) return hipSuccess;
  hipLaunchKernelGGL(assemble_kernel, dim3(n_tasks), dim3(256), 0, s, d_tasks,
                     sstore, fstore, out0, out1);
  return hipGetLastError();
}

__global__ __launch_bounds__(256) void scale_rows_kernel(
    double *__restrict__ out, const double *__restrict__ Q,
    const double *__restrict__ eps, int64_t total, int n_vir) {
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x)
    out[e] = Q[e] * eps[e % n_vir];
}

hipError_t launch_scale_rows(double *out, const double *Q, const double *eps,
                             int64_t rows, int n_vir, hipStream_t s) {
  const int64_t total = rows * n_vir;
  if (total <= 0) return hipSuccess;
  int64_t blocks = (total + 255) / 256;
  if (blocks > 16384) blocks = 16384;
  hipLaunchKernelGGL(scale_rows_kernel, dim3((unsigned)blocks), dim3(256), 0, s,
                     out, Q, eps, total, n_vir);
  return hipGetLastError();
}

__global__ void fill_kernel(double *p, double v, int64_t n) {
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n;
       e += (int64_t)gridDim.x * blockDim.x)
    p[e] = v;
}

hipError_t launch_fill(double *p, double v, int64_t n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  int64_t blocks = (n + 255) / 256;
  if (blocks > 16384) blocks = 16384;
  hipLaunchKernelGGL(fill_kernel, dim3((unsigned)blocks), dim3(256), 0, s, p, v, n);
  return hipGetLastError();
}

__global__ void fill_i32_kernel(int32_t *p, int32_t v, int64_t n) {
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n;
       e += (int64_t)gridDim.x * blockDim.x)
    p[e] = v;
}

hipError_t launch_fill_i32(int32_t *p, int32_t v, int64_t n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  int64_t blocks = (n + 255) / 256;
  if (blocks > 16384) blocks = 16384;
  hipLaunchKernelGGL(fill_i32_kernel, dim3((unsigned)blocks), dim3(256), 0, s, p, v, n);
  return hipGetLastError();
}

}  // namespace mbe3
