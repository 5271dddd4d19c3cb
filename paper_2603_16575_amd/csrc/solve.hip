// Fragment solver: the coupled residual equations of one 1-, 2- or 3-orbital
// fragment (eq. res_close restricted to the fragment, Algorithm 7) iterated
// to convergence inside one workgroup.
//
// Work is done in each pair's pseudo-canonical basis X (eq. prec_eig):
// T_pq = X Y X^T.  Then the pair's own Fock terms become diagonal,
//   X^T (F T S + S T F - f_pp S T S - f_qq S T S) X = -E~ o Y,
// and every coupling term f S_(t,s) T_s S_(s,t) becomes
//   f S~_(t,s) Y_s S~_(t,s)^T,   S~_(t,s) = X_t^T V_t^T V_s X_s,
// so one sweep is
//   R~_t = K~_t - E~_t o Y_t - sum_terms f S~ Y_s^(T) S~^T   (+ transpose for
//          diagonal pairs, whose two mirror terms are transposes),
//   converged if max |R~| < tol, else Y_t += R~_t / E~_t,
// which is the paper's update T += X (X^T R X / E~) X^T with the same
// iterates, without the per-sweep X transforms.  The Hylleraas energy
//   E_F = sum_t w_t <2 Y_t - Y_t^T, K~_t + R~_t>
// is accumulated in the same pass.
//
// Products run on v_mfma_f64_16x16x4 with operands read straight from the
// (L2-resident) per-workgroup scratch and the S~ stores; all pair blocks are
// zero padded to multiples of 16, so no tile needs masking.
#include "internal.hpp"

namespace mbe3 {

typedef double d4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ d4 mfma_f64(double a, double b, d4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

template <int MAXT>
__global__ __launch_bounds__(256) void solve_kernel(SolveArgs a) {
  __shared__ double red_d[8];
  __shared__ int red_i[8];
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int l16 = lane & 15;
  const int lq = lane >> 4;

  double *scr = a.scratch + (int64_t)blockIdx.x * a.scratch_stride;
  const int64_t ny_cap = (a.scratch_stride - 2LL * a.dmax * a.dmax) / 4;
  double *const Y0 = scr;
  double *const YT0 = scr + 2 * ny_cap;
  double *Z = scr + 4 * ny_cap;
  double *ACC = Z + (int64_t)a.dmax * a.dmax;

  for (int fi = blockIdx.x; fi < a.n_frag; fi += gridDim.x) {
    const FragDesc *__restrict__ fdp = a.frags + fi;
    const int f_nt = fdp->nt, f_ny = fdp->ny, f_frag = fdp->frag;
    const int f_tb = fdp->term_begin, f_te = fdp->term_end;
    for (int e = tid; e < f_ny; e += 256) {
      Y0[e] = 0.0;
      YT0[e] = 0.0;
    }
    __syncthreads();
    int cur = 0;
    for (int it = 0;; ++it) {
      double mres = 0.0, epart = 0.0;
      int bad = 0;
      double *const Ycb = Y0 + (cur ? ny_cap : 0);
      double *const YTcb = YT0 + (cur ? ny_cap : 0);
      double *const Ynb = Y0 + (cur ? 0 : ny_cap);
      double *const YTnb = YT0 + (cur ? 0 : ny_cap);
      for (int tl = 0; tl < f_nt; ++tl) {
        const SlotInfo sl = a.slots[fdp->slot[tl]];
        const int Dt = sl.D;
        const int nT = Dt >> 4;
        const int ntile = nT * nT;
        d4 acc[MAXT];
#pragma unroll
        for (int u = 0; u < MAXT; ++u) acc[u] = d4{0.0, 0.0, 0.0, 0.0};

        for (int ti = f_tb; ti < f_te; ++ti) {
          const Term tm = a.terms[ti];
          if (tm.target != tl) continue;
          const double coef = a.f_occ[(int64_t)tm.fx * a.n_occ + tm.fy];
          const int Ds = a.slots[fdp->slot[tm.src]].D;
          const double *__restrict__ Ys =
              (tm.trans ? YTcb : Ycb) + fdp->ysub[tm.src];
          const double *__restrict__ ST = (tm.st_buf ? a.st1 : a.st0) + tm.st_off;
          // Z = coef * S~'(Dt x Ds) . Ys^(T) (Ds x Ds), S~'[i][k] = ST[k*Dt+i];
          // stored column-major Z[j*Dt + i].
          const int nS = Ds >> 4;
          const int nZ = nT * nS;
          for (int zt = wave; zt < nZ; zt += 4) {
            const int zi = zt % nT, zj = zt / nT;
            d4 z = d4{0.0, 0.0, 0.0, 0.0};
            const double *ap = ST + zi * 16 + l16;
            const double *bp = Ys + zj * 16 + l16;
            for (int k0 = 0; k0 < Ds; k0 += 4) {
              const int k = k0 + lq;
              z = mfma_f64(ap[(int64_t)k * Dt], bp[(int64_t)k * Ds], z);
            }
            // D layout: register v of lane l is row l/16 + 4v, column l%16
            double *zp = Z + (int64_t)(zj * 16 + l16) * Dt + zi * 16 + lq;
#pragma unroll
            for (int v = 0; v < 4; ++v) zp[4 * v] = coef * z[v];
          }
          __syncthreads();
          // acc += Z (Dt x Ds) . S~'^T (Ds x Dt), S~'^T[k][j] = ST[k*Dt+j]
#pragma unroll
          for (int u = 0; u < MAXT; ++u) {
            const int tt = wave + 4 * u;
            if (tt < ntile) {
              const int ri = tt / nT, rj = tt - ri * nT;
              const double *ap = Z + ri * 16 + l16;
              const double *bp = ST + rj * 16 + l16;
              d4 c = acc[u];
              for (int k0 = 0; k0 < Ds; k0 += 4) {
                const int k = k0 + lq;
                c = mfma_f64(ap[(int64_t)k * Dt], bp[(int64_t)k * Dt], c);
              }
              acc[u] = c;
            }
          }
          __syncthreads();
        }

        const int sym = fdp->sym[tl];
        if (sym) {
#pragma unroll
          for (int u = 0; u < MAXT; ++u) {
            const int tt = wave + 4 * u;
            if (tt < ntile) {
              const int ri = tt / nT, rj = tt - ri * nT;
#pragma unroll
              for (int v = 0; v < 4; ++v)
                ACC[(int64_t)(ri * 16 + lq + 4 * v) * Dt + rj * 16 + l16] = acc[u][v];
            }
          }
          __syncthreads();
        }

        const int ysub = fdp->ysub[tl];
        const double *Yc = Ycb + ysub;
        const double *YTc = YTcb + ysub;
        double *Yn = Ynb + ysub;
        double *YTn = YTnb + ysub;
        const double *Kt = a.kt + sl.kt_off;
        const double *et = a.et + sl.et_off;
        const double fpq = a.f_occ[(int64_t)sl.p * a.n_occ + sl.p] +
                           a.f_occ[(int64_t)sl.q * a.n_occ + sl.q];
        const double w = (double)fdp->wgt[tl];
#pragma unroll
        for (int u = 0; u < MAXT; ++u) {
          const int tt = wave + 4 * u;
          if (tt < ntile) {
            const int ri = tt / nT, rj = tt - ri * nT;
            const int j = rj * 16 + l16;
            const double ej = et[j];
#pragma unroll
            for (int v = 0; v < 4; ++v) {
              const int i = ri * 16 + lq + 4 * v;
              double s = acc[u][v];
              if (sym) s += ACC[(int64_t)j * Dt + i];
              const int64_t ij = (int64_t)i * Dt + j;
              const double y = Yc[ij];
              const double yt = YTc[ij];
              const double den = fpq - et[i] - ej;
              const double r = Kt[ij] - den * y - s;
              const double ar = fabs(r);
              if (!(ar <= 1e300)) bad = 1;
              mres = fmax(mres, ar);
              epart += w * (2.0 * y - yt) * (Kt[ij] + r);
              const double yn = y + r / den;
              Yn[ij] = yn;
              YTn[(int64_t)j * Dt + i] = yn;
            }
          }
        }
        if (sym) __syncthreads();  // ACC is reused by the next target
      }

      // block reductions (fixed order: deterministic)
      for (int o = 32; o > 0; o >>= 1) {
        mres = fmax(mres, __shfl_xor(mres, o));
        epart += __shfl_xor(epart, o);
        bad |= __shfl_xor(bad, o);
      }
      if (lane == 0) {
        red_d[wave] = mres;
        red_d[4 + wave] = epart;
        red_i[wave] = bad;
      }
      __syncthreads();
      const double M = fmax(fmax(red_d[0], red_d[1]), fmax(red_d[2], red_d[3]));
      const double E = (red_d[4] + red_d[5]) + (red_d[6] + red_d[7]);
      const int B = red_i[0] | red_i[1] | red_i[2] | red_i[3];
      __syncthreads();
      const bool conv = M < a.tol;
      if (conv || B || it >= a.max_iter) {
        if (tid == 0) {
          a.e_frag[f_frag] = B ? __builtin_nan("") : E;
          a.iters[f_frag] = conv && !B ? it : -(a.max_iter + 1);
          int32_t *st = a.status + 2 * blockIdx.x;  // owned by this workgroup
          if (B) st[0] = 1;
          if (!conv && !B) st[1] = 1;
        }
        break;
      }
      cur ^= 1;
    }
    __syncthreads();
  }
}

int64_t solve_scratch_doubles(int ny_max, int dmax) {
  return 4LL * ny_max + 2LL * dmax * dmax;
}

hipError_t launch_solve(const SolveArgs &a, int n_wg, hipStream_t s) {
  if (a.n_frag <= 0) return hipSuccess;
  const int nt = a.dmax / 16;
  const int tiles = (nt * nt + 3) / 4;
  dim3 grid(n_wg), block(256);
  if (tiles <= 1)
    hipLaunchKernelGGL(solve_kernel<1>, grid, block, 0, s, a);
  else if (tiles <= 4)
    hipLaunchKernelGGL(solve_kernel<4>, grid, block, 0, s, a);
  else if (tiles <= 7)
    hipLaunchKernelGGL(solve_kernel<7>, grid, block, 0, s, a);
  else if (tiles <= 9)
    hipLaunchKernelGGL(solve_kernel<9>, grid, block, 0, s, a);
  else if (tiles <= 16)
    hipLaunchKernelGGL(solve_kernel<16>, grid, block, 0, s, a);
  else if (tiles <= 25)
    hipLaunchKernelGGL(solve_kernel<25>, grid, block, 0, s, a);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

}  // namespace mbe3
