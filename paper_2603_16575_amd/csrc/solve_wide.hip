// Fragment solver for pair dimensions beyond the LDS-resident design (D up
// to 160, configurations with r up to 80).  Same equations and sweep order as
// solve.hip (pseudo-canonical basis, eq. res_close restricted to the
// fragment, Algorithm 7, Hylleraas energy); only the data flow differs, so
// that a D_s x D_t block never has to sit in LDS or in registers whole:
//   - one wave per 16-row block of the largest pair (up to 10 waves);
//   - pass 1 (W = Z^T for the wave's row block, all D_s columns) streams
//     16-row panels of S~ and Y^(T) through LDS;
//   - pass 2 (the row block of S~^T Y S~) runs in two halves of the output
//     columns, each streaming the S~ panels again, and adds its half into a
//     per-workgroup term sum R in global memory (each element owned by one
//     lane, so no atomics);
//   - the residual, update and energy run one element per thread over R.
// Registers: pass 1 holds W (4 D_max/16 doubles per lane), which then goes to
// the workgroup's scratch; pass 2 holds half a row block of the output
// (2 D_max/16 doubles per lane) and reads W back four doubles at a time, so
// ten waves fit with three per SIMD.
#include "internal.hpp"

namespace mbe3 {

typedef double d4 __attribute__((ext_vector_type(4)));
typedef double d2 __attribute__((ext_vector_type(2)));

__device__ __forceinline__ d4 mfma64(double a, double b, d4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

template <int NW>
__device__ __forceinline__ double wide_sum(double v, double *red) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  double s = red[0];
#pragma unroll
  for (int w = 1; w < NW; ++w) s += red[w];
  __syncthreads();
  return s;
}

// Rows 16 m .. 16 m + 15 of a row-major block with rows of `len` doubles
// (a multiple of 16) into LDS, as coalesced 16-byte loads.
template <int NTH>
__device__ __forceinline__ void load_panel(const double *__restrict__ src, int len,
                                           double *dst) {
  const d2 *s2 = reinterpret_cast<const d2 *>(src);
  d2 *d = reinterpret_cast<d2 *>(dst);
  for (int e = threadIdx.x; e < 8 * len; e += NTH) d[e] = s2[e];
}

template <int MAXNT, bool GRAD>
__global__ __launch_bounds__(64 * MAXNT) __attribute__((amdgpu_waves_per_eu((MAXNT + 3) / 4)))
void solve_wide_kernel(SolveArgs a) {
  constexpr int NW = MAXNT;
  constexpr int NTH = 64 * NW;
  constexpr int HALF = (MAXNT + 1) / 2;
  extern __shared__ double lds[];
  __shared__ double red_d[2 * NW];
  __shared__ int red_i[NW];
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int l16 = lane & 15;
  const int lq = lane >> 4;
  double *const Sp = lds;                  // 16 rows of S~' (16 x D_t)
  double *const Yp = lds + 16 * a.dmax;    // 16 rows of Y^(T) (16 x D_s)

  double *scr = a.scratch + (int64_t)blockIdx.x * a.scratch_stride;
  const int64_t ny_cap = (a.scratch_stride - 2LL * a.dmax * a.dmax) / 4;
  double *const Y0 = scr;
  double *const YT0 = scr + 2 * ny_cap;
  double *const R = scr + 4 * ny_cap;      // term sum of the current target
  // pass-1 result of every wave: (MAXNT waves x MAXNT tiles x 64 lanes) d4,
  // i.e. 256 MAXNT^2 = D_max^2 doubles after R
  d4 *const Wg = reinterpret_cast<d4 *>(R + (int64_t)a.dmax * a.dmax);

  for (int fi = blockIdx.x; fi < a.n_frag; fi += gridDim.x) {
    const FragDesc *__restrict__ fdp = a.frags + fi;
    const int f_nt = fdp->nt, f_frag = fdp->frag;
    const int f_tb = fdp->term_begin, f_te = fdp->term_end;
    int cur = 0;
    bool gpass = false;  // GRAD: the extra pass at the converged amplitudes
    // amplitudes present: after a warm start from the solutions of the
    // fragment's own pairs (monomers, dimers), or after the first update
    bool hasY = false;
    if (fdp->warm_in && a.warm) {
      for (int tl = 0; tl < f_nt; ++tl) {
        const SlotInfo sl = a.slots[fdp->slot[tl]];
        const int D = sl.D;
        const double *src = a.warm + sl.kt_off;
        double *y = Y0 + fdp->ysub[tl];
        double *yt = YT0 + fdp->ysub[tl];
        for (int e = tid; e < D * D; e += NTH) {
          const int i = e / D, j = e - i * D;
          const double v = src[e];
          y[e] = v;
          yt[(int64_t)j * D + i] = v;
        }
      }
      __syncthreads();
      hasY = true;
    }
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
        const int sym = fdp->sym[tl];
        for (int e = tid; e < Dt * Dt; e += NTH) R[e] = 0.0;
        __syncthreads();
        if (hasY) {
          for (int ti = f_tb; ti < f_te; ++ti) {
            const Term tm = a.terms[ti];
            if (tm.target != tl) continue;
            const double coef =
                (GRAD && gpass) ? 1.0 : a.f_occ[(int64_t)tm.fx * a.n_occ + tm.fy];
            const int Ds = a.slots[fdp->slot[tm.src]].D;
            const int nS = Ds >> 4;
            const double *St = (tm.st_buf ? a.st1 : a.st0) + tm.st_off;
            const double *Ys = (tm.trans ? YTcb : Ycb) + fdp->ysub[tm.src];
            // pass 1: W[kb] = tile (kb, wave) of Z^T = (Y^(T))^T S~'
            d4 W[MAXNT];
#pragma unroll
            for (int kb = 0; kb < MAXNT; ++kb) W[kb] = d4{0.0, 0.0, 0.0, 0.0};
            for (int mp = 0; mp < nS; ++mp) {
              load_panel<NTH>(St + (int64_t)16 * mp * Dt, Dt, Sp);
              load_panel<NTH>(Ys + (int64_t)16 * mp * Ds, Ds, Yp);
              __syncthreads();
              if (wave < nT) {
#pragma unroll
                for (int mm = 0; mm < 4; ++mm) {
                  const int ml = 4 * mm + lq;
                  const double bv = Sp[ml * Dt + wave * 16 + l16];
#pragma unroll
                  for (int kb = 0; kb < MAXNT; ++kb)
                    if (kb < nS) W[kb] = mfma64(Yp[ml * Ds + kb * 16 + l16], bv, W[kb]);
                }
              }
              __syncthreads();
            }
            // W leaves the registers: each lane keeps its own tiles in the
            // workgroup's scratch and reads them back in pass 2 (same lane)
            if (wave < nT) {
#pragma unroll
              for (int kb = 0; kb < MAXNT; ++kb)
                if (kb < nS) Wg[(wave * MAXNT + kb) * 64 + lane] = W[kb];
            }
            // pass 2 in two halves of the output columns
#pragma unroll
            for (int h = 0; h < 2; ++h) {
              d4 acc[HALF];
#pragma unroll
              for (int jj = 0; jj < HALF; ++jj) acc[jj] = d4{0.0, 0.0, 0.0, 0.0};
              for (int kp = 0; kp < nS; ++kp) {
                load_panel<NTH>(St + (int64_t)16 * kp * Dt, Dt, Sp);
                __syncthreads();
                if (wave < nT) {
                  const d4 wk = Wg[(wave * MAXNT + kp) * 64 + lane];
#pragma unroll
                  for (int v = 0; v < 4; ++v) {
                    const double av = coef * wk[v];
                    const double *brow = Sp + (4 * v + lq) * Dt + l16;
#pragma unroll
                    for (int jj = 0; jj < HALF; ++jj) {
                      const int jb = h * HALF + jj;
                      if (jb < nT) acc[jj] = mfma64(av, brow[jb * 16], acc[jj]);
                    }
                  }
                }
                __syncthreads();
              }
              if (wave < nT) {
#pragma unroll
                for (int jj = 0; jj < HALF; ++jj) {
                  const int jb = h * HALF + jj;
                  if (jb < nT) {
#pragma unroll
                    for (int v = 0; v < 4; ++v)
                      R[(int64_t)(wave * 16 + lq + 4 * v) * Dt + jb * 16 + l16] += acc[jj][v];
                  }
                }
              }
            }
            if (GRAD && gpass) {
              // this term alone, contracted with Y~ = 2Y - Y^T (Y + Y^T for a
              // diagonal target, whose mirror term is folded); R cleared again
              __syncthreads();
              const double *Yc = Ycb + fdp->ysub[tl];
              const double *YTc = YTcb + fdp->ysub[tl];
              double part = 0.0;
              for (int e = tid; e < Dt * Dt; e += NTH) {
                const double wy = sym ? Yc[e] + YTc[e] : 2.0 * Yc[e] - YTc[e];
                part += wy * R[e];
                R[e] = 0.0;
              }
              const double tot = wide_sum<NW>(part, red_d);
              if (tid == 0) a.gterm[ti] = tot;
            }
          }
        }
        if (GRAD && gpass) {
          const double *Yc = Ycb + fdp->ysub[tl];
          const double *YTc = YTcb + fdp->ysub[tl];
          double part = 0.0;
          for (int e = tid; e < Dt * Dt; e += NTH) part += (2.0 * Yc[e] - YTc[e]) * Yc[e];
          const double tot = wide_sum<NW>(part, red_d);
          if (tid == 0) a.gdiag[6 * fi + tl] = tot;
          continue;
        }
        __syncthreads();  // R complete
        // ---- residual, energy, update: one element per thread ----
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
        for (int e = tid; e < Dt * Dt; e += NTH) {
          const int i = e / Dt, j = e - i * Dt;
          const double y = hasY ? Yc[e] : 0.0;
          const double yt = hasY ? YTc[e] : 0.0;
          const double s = sym ? R[e] + R[(int64_t)j * Dt + i] : R[e];
          const double kij = Kt[e];
          const double den = fpq - et[i] - et[j];
          const double r = kij - den * y - s;
          const double ar = fabs(r);
          if (!(ar <= 1e300)) bad = 1;
          mres = fmax(mres, ar);
          epart += w * (2.0 * y - yt) * (kij + r);
          const double yn = y + r / den;
          Yn[e] = yn;
          YTn[(int64_t)j * Dt + i] = yn;
        }
        __syncthreads();  // R is cleared by the next target
      }
      if (GRAD && gpass) break;
      for (int o = 32; o > 0; o >>= 1) {
        mres = fmax(mres, __shfl_xor(mres, o));
        epart += __shfl_xor(epart, o);
        bad |= __shfl_xor(bad, o);
      }
      if (lane == 0) {
        red_d[wave] = mres;
        red_d[NW + wave] = epart;
        red_i[wave] = bad;
      }
      __syncthreads();
      double M = red_d[0], E = red_d[NW];
      int B = red_i[0];
#pragma unroll
      for (int w2 = 1; w2 < NW; ++w2) {
        M = fmax(M, red_d[w2]);
        E += red_d[NW + w2];
        B |= red_i[w2];
      }
      __syncthreads();
      const bool conv = M < a.tol;
      if (conv || B || it >= a.max_iter) {
        if (tid == 0) {
          a.e_frag[f_frag] = B ? __builtin_nan("") : E;
          a.iters[f_frag] = conv && !B ? it : -(a.max_iter + 1);
          int32_t *st = a.status + 2 * blockIdx.x;
          if (B) st[0] = 1;
          if (!conv && !B) st[1] = 1;
        }
        if (fdp->warm_out >= 0 && a.warm) {
          // the fragment's own pair seeds the trimers that contain it: its
          // last amplitudes, converged or not (zero after a non-finite
          // residual), so every trimer starts from defined values
          const SlotInfo sl = a.slots[fdp->slot[fdp->warm_out]];
          const double *src = Ycb + fdp->ysub[fdp->warm_out];
          for (int e = tid; e < sl.D * sl.D; e += NTH)
            a.warm[sl.kt_off + e] = hasY && !B ? src[e] : 0.0;
        }
        if (GRAD && conv && !B) {
          if (!hasY) {
            for (int e = tid; e < fdp->ny; e += NTH) a.yfin[fdp->yout + e] = 0.0;
            for (int ti = f_tb + tid; ti < f_te; ti += NTH) a.gterm[ti] = 0.0;
            if (tid < f_nt) a.gdiag[6 * fi + tid] = 0.0;
            break;
          }
          for (int e = tid; e < fdp->ny; e += NTH)
            a.yfin[fdp->yout + e] = 2.0 * Ycb[e] - YTcb[e];
          __syncthreads();
          gpass = true;
          continue;
        }
        break;
      }
      hasY = true;
      cur ^= 1;
    }
  }
}

size_t solve_wide_lds_bytes(int dmax) { return (size_t)32 * dmax * sizeof(double); }

template <int NT, bool GRAD>
static hipError_t launch_wide_g(const SolveArgs &a, int n_wg, hipStream_t s) {
  const size_t smem = solve_wide_lds_bytes(a.dmax);
  hipError_t e = hipFuncSetAttribute((const void *)solve_wide_kernel<NT, GRAD>,
                                     hipFuncAttributeMaxDynamicSharedMemorySize,
                                     (int)smem);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((solve_wide_kernel<NT, GRAD>), dim3(n_wg), dim3(64 * NT), smem, s, a);
  return hipGetLastError();
}

template <int NT>
static hipError_t launch_wide_nt(const SolveArgs &a, int n_wg, hipStream_t s) {
  return a.yfin ? launch_wide_g<NT, true>(a, n_wg, s) : launch_wide_g<NT, false>(a, n_wg, s);
}

hipError_t launch_solve_wide(const SolveArgs &a, int n_wg, hipStream_t s) {
  if (a.n_frag <= 0) return hipSuccess;
  if (a.dmax % 16) return hipErrorInvalidValue;
  switch (a.dmax / 16) {
    case 7: return launch_wide_nt<7>(a, n_wg, s);
    case 8: return launch_wide_nt<8>(a, n_wg, s);
    case 9: return launch_wide_nt<9>(a, n_wg, s);
    case 10: return launch_wide_nt<10>(a, n_wg, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace mbe3
