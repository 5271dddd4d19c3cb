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
// Data flow of one term on the FP64 matrix cores (v_mfma_f64_16x16x4), with
// S~ stored as S~_(s,t) = S~'^T (D_s x D_t, row-major):
//   pass 1: each wave owns whole 16-row blocks ib of R~_t and accumulates
//      W = Z^T = (Y_s^(T))^T S~'^T over 16-row panels m of Y_s^(T) and S~;
//   pass 2: the MFMA output layout (register v of lane l holds row l/16 + 4v,
//      column l%16) is exactly the A-operand layout of the second product for
//      the four k-steps kb*16 + 4v, so Z never leaves the registers and
//      R~_t[ib, :] += Z[ib, :] S~'^T reads the S~ resident in LDS.
// Panels go global -> registers (prefetched one step ahead) -> LDS: the
// term's S~ panels land in a resident D_s x D_t block reused by pass 2 (which
// then needs no barrier and hides the next term's first load), the Y^(T)
// rows in two alternating 16-row buffers.  Only Y is kept in memory: a panel
// of Y^T (16 rows of it) is read as 16-column strips of Y's rows and
// transposed on its way into LDS, and the residual reads Y^T elements
// straight from Y, so each sweep writes its amplitudes once, coalesced.  LDS per workgroup is
// D_max^2 + 32 D_max doubles (16 D_max at D_max = 128, one Y buffer): two
// fragments share a CU up to 80-wide domains (four waves each), one above
// (eight waves, each owning one row block).  A diagonal pair's
// mirror terms f S~ Y S~^T and its transpose are formed once and symmetrised
// through LDS.
// Sweep 0 has T = 0, so R~ = K~ needs no product.  All pair blocks are zero
// padded to multiples of 16: no tile is masked.
#include "internal.hpp"

namespace mbe3 {

typedef double d4 __attribute__((ext_vector_type(4)));
typedef double d2 __attribute__((ext_vector_type(2)));

__device__ __forceinline__ d4 mfma_f64(double a, double b, d4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// Global-memory view of a pointer whose address space the compiler cannot
// see (one read back from LDS): loads through it are global loads, counted
// by vmcnt alone.  Through a generic pointer they would be flat loads, which
// also count in lgkmcnt, so every wait for an LDS access would wait for the
// prefetched panel as well.
typedef __attribute__((address_space(1))) const d2 gd2;
__device__ __forceinline__ const gd2 *as_global(const double *p) {
  return (const gd2 *)(p);
}

// s_waitcnt immediate of vmcnt(0) alone (gfx9 encoding: expcnt and lgkmcnt
// at their maxima)
constexpr int WAIT_VMCNT0 = 0x0F70;

// A fragment's terms and slots as the workgroup reads them, staged in LDS at
// the start of each fragment: every panel step and residual block then reads
// its descriptors from LDS instead of chasing term -> slot -> dimension
// through global memory (each hop a full memory round trip on the critical
// path of the panel pipeline).
struct TermLds {
  const double *st;  // row-major S~_(src, target)
  double coef;       // f_occ[fx][fy]; 1 in the gradient pass
  int32_t target, src, dt, ds, trans, pad_;
};
struct SlotLds {
  int64_t kt_off, et_off;
  double fpq;  // f_pp + f_qq
  int32_t D, ysub, sym, wgt;
};

// Sum / max of the per-wave partials r[0 .. N) as a fixed tree: the first
// half (the largest power of two below N) and the rest, recursively.
template <int N>
__device__ __forceinline__ double wave_tree_sum(const double *r) {
  if constexpr (N == 1) {
    return r[0];
  } else {
    constexpr int H = N > 4 ? 4 : (N > 2 ? 2 : 1);
    return wave_tree_sum<H>(r) + wave_tree_sum<N - H>(r + H);
  }
}
template <int N>
__device__ __forceinline__ double wave_tree_max(const double *r) {
  if constexpr (N == 1) {
    return r[0];
  } else {
    constexpr int H = N > 4 ? 4 : (N > 2 ? 2 : 1);
    return fmax(wave_tree_max<H>(r), wave_tree_max<N - H>(r + H));
  }
}

// Workgroup sum in a fixed order (wave shuffles, then the waves' tree).
template <int NW>
__device__ __forceinline__ double wg_sum(double v, double *red) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  const double s = wave_tree_sum<NW>(red);
  __syncthreads();
  return s;
}

// One term's products accumulated into acc (see the data flow above): pass 1
// streams the S~ and Y^(T) row panels into LDS and forms W = Z^T in
// registers, pass 2 reads the S~ resident in LDS.  Expects the panel
// pipeline state (pf, p_*), Dt/nT, Ds/nS, acc and the LDS pointers in scope.
#define MBE3_TERM_PRODUCTS(COEF)                                               \
  do {                                                                         \
    d4 W[MAXRB][MAXNT];                                                        \
    _Pragma("unroll") for (int rb = 0; rb < MAXRB; ++rb)                       \
      _Pragma("unroll") for (int kb = 0; kb < MAXNT; ++kb)                     \
        W[rb][kb] = d4{0.0, 0.0, 0.0, 0.0};                                    \
    __syncthreads(); /* the previous term's S~ is no longer read */            \
    for (int mp = 0; mp < nS; ++mp) {                                          \
      double *const yb = (mp & 1) ? yb1 : yb0;                                 \
      /* the panel in pf has landed; waiting here explicitly leaves no load   \
         outstanding on any path, so the next panel's loads issue back to     \
         back instead of each waiting for the one before */                  \
      __builtin_amdgcn_s_waitcnt(WAIT_VMCNT0);                                 \
      {                                                                        \
        d2 *s_ = reinterpret_cast<d2 *>(Sl + 16 * mp * Dt);                    \
        d2 *y_ = reinterpret_cast<d2 *>(yb);                                   \
        _Pragma("unroll") for (int u = 0; u < PFN; ++u) {                      \
          const int e = tid + NTH * u;                                         \
          if (e < p_n1) {                                                      \
            s_[e] = pf[u];                                                     \
          } else if (e - p_n1 < p_n2) {                                        \
            const int q_ = e - p_n1;                                           \
            if (p_tr) { /* Y[k][16 mp + c, c + 1] -> rows c, c + 1, col k */   \
              const int k_ = q_ >> 3, c_ = 2 * (q_ & 7);                       \
              yb[c_ * Ds + k_] = pf[u].x;                                      \
              yb[(c_ + 1) * Ds + k_] = pf[u].y;                                \
            } else {                                                           \
              y_[q_] = pf[u];                                                  \
            }                                                                  \
          }                                                                    \
        }                                                                      \
      }                                                                        \
      /* the next panel streams in under the products; a term's last panel   \
         prefetches the next term's first one */                              \
      MBE3_ADVANCE();                                                          \
      if (p_ti < f_te) MBE3_LOAD_PANEL();                                      \
      __syncthreads();                                                         \
      const double *STp = Sl + 16 * mp * Dt;                                   \
      _Pragma("unroll") for (int mm = 0; mm < 4; ++mm) {                       \
        const int ml = 4 * mm + lq;                                            \
        _Pragma("unroll") for (int rb = 0; rb < MAXRB; ++rb) {                 \
          const int ib = wave + NW * rb;                                       \
          if (ib < nT) {                                                       \
            const double bv = STp[ml * Dt + ib * 16 + l16];                    \
            _Pragma("unroll") for (int kb = 0; kb < MAXNT; ++kb)               \
              if (kb < nS)                                                     \
                W[rb][kb] = mfma_f64(yb[ml * Ds + kb * 16 + l16], bv, W[rb][kb]); \
          }                                                                    \
        }                                                                      \
      }                                                                        \
      /* one Y buffer: the next panel's store waits for these reads */        \
      if (!DBY) __syncthreads();                                               \
    }                                                                          \
    _Pragma("unroll") for (int kp = 0; kp < MAXNT; ++kp) {                     \
      if (kp < nS) {                                                           \
        _Pragma("unroll") for (int v = 0; v < 4; ++v) {                        \
          const double *brow = Sl + (kp * 16 + 4 * v + lq) * Dt + l16;         \
          _Pragma("unroll") for (int rb = 0; rb < MAXRB; ++rb) {               \
            const int ib = wave + NW * rb;                                     \
            if (ib < nT) {                                                     \
              const double av = (COEF) * W[rb][kp][v];                         \
              _Pragma("unroll") for (int jb = 0; jb < MAXNT; ++jb)             \
                if (jb < nT) acc[rb][jb] = mfma_f64(av, brow[jb * 16], acc[rb][jb]); \
            }                                                                  \
          }                                                                    \
        }                                                                      \
      }                                                                        \
    }                                                                          \
  } while (0)

// MAXNT: largest number of 16-blocks per pair dimension (dmax / 16).
// MODE 0: solve.  MODE 1: solve and store each converged fragment's Y at
// FragDesc::yout (zero if it converged at T = 0) for the gradient pass.
// MODE 2: the gradient pass alone, a separate launch over the same
// fragments: the stored Y goes back into the scratch, every term's product
// is formed once more with unit coefficient and contracted with Y~, and the
// store then receives Y~ = 2Y - Y^T for the multipliers.  Fragments that did
// not converge (iters < 0) are skipped.  Keeping the pass out of the solving
// launch keeps its registers out of the iterations.
template <int MAXNT, int MODE, int NW>
__global__ __launch_bounds__(64 * NW, MAXNT <= 5 ? 2 : 1) void solve_kernel(SolveArgs a) {
  constexpr bool ST = MODE == 1, GP = MODE == 2;
  extern __shared__ double lds[];
  constexpr int NTH = 64 * NW;                   // threads per workgroup
  constexpr int MAXRB = (MAXNT + NW - 1) / NW;   // row blocks per wave
  constexpr int PFN = (4 * MAXNT + NW - 1) / NW;  // panel slots per thread
  constexpr bool DBY = MAXNT <= 7;               // two Y panel buffers
  __shared__ double red_d[2 * NW];
  __shared__ int red_i[NW];
  __shared__ TermLds tc[MAX_FRAG_TERMS];
  __shared__ SlotLds sc[6];
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);  // uniform per wave
  const int l16 = lane & 15;
  const int lq = lane >> 4;
  // LDS: the term's whole S~ (D_s x D_t) stays resident for both passes; the
  // Y^(T) rows stream through two 16-row buffers.
  double *const Sl = lds;
  double *const yb0 = lds + (int64_t)a.dmax * a.dmax;
  double *const yb1 = DBY ? yb0 + 16 * a.dmax : yb0;

  double *scr = a.scratch + (int64_t)blockIdx.x * a.scratch_stride;
  const int64_t ny_cap = (a.scratch_stride - 2LL * a.dmax * a.dmax) / 4;
  double *const Y0 = scr;  // two buffers of ny_cap (current, next)

  d2 pf[PFN];  // next panel: S~ rows then Y^(T) rows

  for (int fi = blockIdx.x; fi < a.n_frag; fi += gridDim.x) {
    const FragDesc *__restrict__ fdp = a.frags + fi;
    const int f_nt = fdp->nt, f_frag = fdp->frag;
    const int f_tb = fdp->term_begin, f_te = fdp->term_end;
    int cur = 0;
    // amplitudes present: after a warm start from the solutions of the
    // fragment's own pairs (monomers, dimers), or after the first update
    bool hasY = false;
    if (GP && a.iters[f_frag] < 0) continue;  // uniform over the workgroup
    // stage the descriptors (the previous fragment's last reads of them came
    // before its closing barrier)
    if (tid < f_te - f_tb) {
      const Term t = a.terms[f_tb + tid];
      TermLds c;
      c.st = (t.st_buf ? a.st1 : a.st0) + t.st_off;
      c.coef = GP ? 1.0 : a.f_occ[(int64_t)t.fx * a.n_occ + t.fy];
      c.target = t.target;
      c.src = t.src;
      c.dt = a.slots[fdp->slot[t.target]].D;
      c.ds = a.slots[fdp->slot[t.src]].D;
      c.trans = t.trans;
      c.pad_ = 0;
      tc[tid] = c;
    } else if (tid >= 64 && tid - 64 < f_nt) {
      const int tl = tid - 64;
      const SlotInfo sl = a.slots[fdp->slot[tl]];
      SlotLds c;
      c.kt_off = sl.kt_off;
      c.et_off = sl.et_off;
      c.fpq = a.f_occ[(int64_t)sl.p * a.n_occ + sl.p] + a.f_occ[(int64_t)sl.q * a.n_occ + sl.q];
      c.D = sl.D;
      c.ysub = fdp->ysub[tl];
      c.sym = fdp->sym[tl];
      c.wgt = fdp->wgt[tl];
      sc[tl] = c;
    }
    __syncthreads();
    if (GP) {
      // the pass reads the stored Y in place; the contraction weights of
      // every target (Y + Y^T for a diagonal one, else 2Y - Y^T = Y~) go to
      // the second scratch buffer, Y~ of the diagonal targets to the third,
      // and <Y~_t, Y_t> to gdiag
      for (int tl = 0; tl < f_nt; ++tl) {
        const int D = sc[tl].D;
        const int sy = sc[tl].sym;
        const double *y = a.yfin + fdp->yout + sc[tl].ysub;
        double *wy = Y0 + ny_cap + sc[tl].ysub;
        double *yd = Y0 + 2 * ny_cap + sc[tl].ysub;
        double part = 0.0;
        for (int e = tid; e < D * D; e += NTH) {
          const int i = e / D, j = e - i * D;
          const double yv = y[e], yt = y[(int64_t)j * D + i];
          const double ytil = 2.0 * yv - yt;
          wy[e] = sy ? yv + yt : ytil;
          if (sy) yd[e] = ytil;
          part += ytil * yv;
        }
        const double tot = wg_sum<NW>(part, red_d);  // also orders the wy writes
        if (tid == 0) a.gdiag[6 * fi + tl] = tot;
      }
      hasY = true;
    } else if (fdp->warm_in && a.warm) {
      hasY = true;
    }
    // a warm-started fragment's first sweep reads the solutions of its own
    // pairs' fragments in place (warm store, one D x D block per slot)
    bool wsrc = !GP && fdp->warm_in && a.warm;
    for (int it = 0;; ++it) {
      double mres = 0.0, epart = 0.0;
      int bad = 0;
      double *const Ycb = GP ? a.yfin + fdp->yout : Y0 + (cur ? ny_cap : 0);
      double *const Ynb = Y0 + (cur ? 0 : ny_cap);
      // the current amplitudes of target / source slot tl
      auto ysrc = [&](int tl) -> const double * {
        return wsrc ? a.warm + sc[tl].kt_off : Ycb + sc[tl].ysub;
      };

      // ---- panel pipeline: step (ti, m) = rows 16m.. of S~ and of Y^(T) ----
      int p_ti = f_tb, p_m = 0;  // step held in pf
      int p_n1 = 0, p_n2 = 0;
      bool p_tr = false;  // the Y part of pf is a strip of Y columns
      // descriptors of term c_ti (the one the prefetch is in), read from LDS
      // once per term rather than once per panel
      int c_ti = -1, c_dt = 0, c_ds = 16;
      bool c_tr = false;
      const double *c_st = nullptr, *c_ys = nullptr;
#define MBE3_LOAD_PANEL()                                                      \
  do {                                                                         \
    if (p_ti != c_ti) { /* a new term: its descriptors, once */                \
      const TermLds &tm_ = tc[p_ti - f_tb];                                    \
      c_dt = __builtin_amdgcn_readfirstlane(tm_.dt);                           \
      c_ds = __builtin_amdgcn_readfirstlane(tm_.ds);                           \
      c_tr = __builtin_amdgcn_readfirstlane(tm_.trans) != 0;                   \
      c_st = tm_.st;                                                           \
      c_ys = ysrc(tm_.src);                                                    \
      c_ti = p_ti;                                                             \
    }                                                                          \
    const gd2 *st_ = as_global(c_st + (int64_t)16 * p_m * c_dt);               \
    /* rows 16m.. of Y, or (transposed source) columns 16m.. of every row */  \
    const gd2 *y_ = as_global(c_tr ? c_ys + 16 * p_m : c_ys + (int64_t)16 * p_m * c_ds); \
    p_n1 = 8 * c_dt;                                                           \
    p_n2 = 8 * c_ds;                                                           \
    p_tr = c_tr;                                                               \
    /* one unconditional load per slot from a selected address: no two      \
       loads of a step write the same registers, so none waits for another */\
    _Pragma("unroll") for (int u = 0; u < PFN; ++u) {                          \
      const int e = tid + NTH * u;                                             \
      const int q_ = e - p_n1;                                                 \
      /* slots past the panel load its first element (never stored) */       \
      const gd2 *src_ = e < p_n1 ? st_ + e                                     \
                        : q_ >= p_n2 ? st_                                     \
                        : p_tr ? y_ + (q_ >> 3) * (c_ds >> 1) + (q_ & 7)       \
                        : y_ + q_;                                             \
      pf[u] = *src_;                                                           \
    }                                                                          \
  } while (0)
#define MBE3_ADVANCE()                                                         \
  do {                                                                         \
    if (++p_m >= (c_ds >> 4)) { p_m = 0; ++p_ti; }                             \
  } while (0)

      if (hasY && f_tb < f_te) MBE3_LOAD_PANEL();

      for (int tl = 0; tl < f_nt; ++tl) {
        const SlotLds sl = sc[tl];
        const int Dt = __builtin_amdgcn_readfirstlane(sl.D);
        const int nT = Dt >> 4;
        d4 acc[MAXRB][MAXNT];
#pragma unroll
        for (int rb = 0; rb < MAXRB; ++rb)
#pragma unroll
          for (int jb = 0; jb < MAXNT; ++jb) acc[rb][jb] = d4{0.0, 0.0, 0.0, 0.0};

        if (hasY) {
          for (int ti = f_tb; ti < f_te; ++ti) {
            if (tc[ti - f_tb].target != tl) continue;
            const double coef = tc[ti - f_tb].coef;
            const int Ds = __builtin_amdgcn_readfirstlane(tc[ti - f_tb].ds);
            const int nS = Ds >> 4;
            MBE3_TERM_PRODUCTS(coef);
            if (GP) {
              // this term's product alone, contracted with Y~ = 2Y - Y^T
              // (Y + Y^T for a diagonal target, whose mirror term is folded)
              const double *Wy = Y0 + ny_cap + sl.ysub;
              double part = 0.0;
#pragma unroll
              for (int rb = 0; rb < MAXRB; ++rb) {
                const int ib = wave + NW * rb;
#pragma unroll
                for (int jb = 0; jb < MAXNT; ++jb) {
                  if (ib < nT && jb < nT) {
#pragma unroll
                    for (int v = 0; v < 4; ++v) {
                      const int i = ib * 16 + lq + 4 * v, j = jb * 16 + l16;
                      part += Wy[(int64_t)i * Dt + j] * acc[rb][jb][v];
                    }
                  }
                  acc[rb][jb] = d4{0.0, 0.0, 0.0, 0.0};
                }
              }
              const double tot = wg_sum<NW>(part, red_d);
              if (tid == 0) a.gterm[ti] = tot;
            }
          }
        }
        if (GP) continue;  // no residual in the gradient pass

        const int sym = sl.sym;
        if (sym) {  // diagonal pair: R~ gets acc + acc^T (mirror terms)
          __syncthreads();  // S~ of the last term is no longer read
#pragma unroll
          for (int rb = 0; rb < MAXRB; ++rb) {
            const int ib = wave + NW * rb;
            if (ib < nT) {
#pragma unroll
              for (int jb = 0; jb < MAXNT; ++jb)
                if (jb < nT) {
#pragma unroll
                  for (int v = 0; v < 4; ++v)
                    Sl[(ib * 16 + lq + 4 * v) * Dt + jb * 16 + l16] = acc[rb][jb][v];
                }
            }
          }
          __syncthreads();
        }

        // ---- residual, energy, update for the owned rows of target tl ----
        const int ysub = sl.ysub;
        const double *Yc = ysrc(tl);
        double *Yn = Ynb + ysub;
        const double *Kt = a.kt + sl.kt_off;
        const double *et = a.et + sl.et_off;
        const double fpq = sl.fpq;
        const double w = (double)sl.wgt;
#pragma unroll
        for (int rb = 0; rb < MAXRB; ++rb) {
          const int ib = wave + NW * rb;
          if (ib < nT) {
#pragma unroll
            for (int jb = 0; jb < MAXNT; ++jb) {
              if (jb < nT) {
                const int j = jb * 16 + l16;
                const double ej = et[j];
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                  const int i = ib * 16 + lq + 4 * v;
                  const int64_t ij = (int64_t)i * Dt + j;
                  const double y = hasY ? Yc[ij] : 0.0;
                  const double yt = hasY ? Yc[(int64_t)j * Dt + i] : 0.0;
                  const double kij = Kt[ij];
                  const double den = fpq - et[i] - ej;
                  const double sacc = sym ? acc[rb][jb][v] + Sl[j * Dt + i] : acc[rb][jb][v];
                  const double r = kij - den * y - sacc;
                  const double ar = fabs(r);
                  if (!(ar <= 1e300)) bad = 1;
                  mres = fmax(mres, ar);
                  epart += w * (2.0 * y - yt) * (kij + r);
                  const double yn = y + r / den;
                  Yn[ij] = yn;
                }
              }
            }
          }
        }
      }
      if (GP) {
        // Y~ over the stored Y (every read of it is done: the last term's
        // contraction ended in a workgroup barrier, its last panel fetched
        // nothing further)
        for (int tl = 0; tl < f_nt; ++tl) {
          const int D = sc[tl].D;
          const double *src = Y0 + (sc[tl].sym ? 2 : 1) * ny_cap + sc[tl].ysub;
          double *o = a.yfin + fdp->yout + sc[tl].ysub;
          for (int e = tid; e < D * D; e += NTH) o[e] = src[e];
        }
        __syncthreads();  // the scratch is read; the next fragment refills it
        break;
      }
      // block reductions (fixed order: deterministic)
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
      __syncthreads();  // also orders this sweep's Y writes before the next
      const double M = wave_tree_max<NW>(red_d);
      const double E = wave_tree_sum<NW>(red_d + NW);
      int B = 0;
#pragma unroll
      for (int w2 = 0; w2 < NW; ++w2) B |= red_i[w2];
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
        if (fdp->warm_out >= 0 && a.warm) {
          // the fragment's own pair seeds the trimers that contain it: its
          // last amplitudes, converged or not (zero after a non-finite
          // residual), so every trimer starts from defined values
          const SlotLds sl = sc[fdp->warm_out];
          const double *src = ysrc(fdp->warm_out);
          for (int e = tid; e < sl.D * sl.D; e += NTH)
            a.warm[sl.kt_off + e] = hasY && !B ? src[e] : 0.0;
        }
        if (ST && conv && !B) {
          // the converged amplitudes (zero if converged at T = 0) for the
          // gradient pass
          for (int tl = 0; tl < f_nt; ++tl) {
            const int D = sc[tl].D;
            const double *src = ysrc(tl);
            double *dst = a.yfin + fdp->yout + sc[tl].ysub;
            for (int e = tid; e < D * D; e += NTH) dst[e] = hasY ? src[e] : 0.0;
          }
        }
        __syncthreads();  // the scratch is read; the next fragment refills it
        break;
      }
      hasY = true;
      wsrc = false;
      cur ^= 1;
    }
  }
}
#undef MBE3_ADVANCE
#undef MBE3_LOAD_PANEL
#undef MBE3_TERM_PRODUCTS

int64_t solve_scratch_doubles(int ny_max, int dmax) {
  return 4LL * ny_max + 2LL * dmax * dmax;
}

// Waves per workgroup of the instance for chunks whose widest pair domain
// has NT 16-row blocks: four up to 80-wide domains (two workgroups share a
// CU), eight from 96 on, where the resident S~ block leaves room for one
// workgroup per CU.  Measured on the 512- and 160-LMO lattices against one
// wave per row block of the widest targets (five to eight waves): balanced
// rows but fewer waves to hide the panel loads, 3% and 20% slower.
template <int NT>
constexpr int solve_waves() { return NT <= 5 ? 4 : 8; }

// LDS of one workgroup: the resident S~ block and two 16-row Y panel
// buffers, one for the 128-wide instance (two would not leave room).
size_t solve_lds_bytes(int dmax) {
  const int ybuf = dmax <= 112 ? 32 : 16;
  return (size_t)(dmax * dmax + ybuf * dmax) * sizeof(double);
}

template <int NT, int MODE, int NW>
static hipError_t launch_nt_g(const SolveArgs &a, int n_wg, hipStream_t s, int *per_cu) {
  const size_t smem = solve_lds_bytes(a.dmax);
  hipError_t e = hipFuncSetAttribute((const void *)solve_kernel<NT, MODE, NW>,
                                     hipFuncAttributeMaxDynamicSharedMemorySize,
                                     (int)smem);
  if (e != hipSuccess) return e;
  if (per_cu)  // resident workgroups per CU for this instance
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(
        per_cu, (const void *)solve_kernel<NT, MODE, NW>, 64 * NW, smem);
  hipLaunchKernelGGL((solve_kernel<NT, MODE, NW>), dim3(n_wg), dim3(64 * NW), smem, s, a);
  return hipGetLastError();
}

template <int MODE>
static hipError_t launch_mode(const SolveArgs &a, int n_wg, hipStream_t s, int *per_cu) {
  if (!per_cu && a.n_frag <= 0) return hipSuccess;
  if (solve_lds_bytes(a.dmax) > 150 * 1024) return hipErrorInvalidValue;
  switch (a.dmax / 16) {
    case 1:
    case 2: return launch_nt_g<2, MODE, solve_waves<2>()>(a, n_wg, s, per_cu);
    case 3: return launch_nt_g<3, MODE, solve_waves<3>()>(a, n_wg, s, per_cu);
    case 4: return launch_nt_g<4, MODE, solve_waves<4>()>(a, n_wg, s, per_cu);
    case 5: return launch_nt_g<5, MODE, solve_waves<5>()>(a, n_wg, s, per_cu);
    case 6: return launch_nt_g<6, MODE, solve_waves<6>()>(a, n_wg, s, per_cu);
    case 7: return launch_nt_g<7, MODE, solve_waves<7>()>(a, n_wg, s, per_cu);
    case 8: return launch_nt_g<8, MODE, solve_waves<8>()>(a, n_wg, s, per_cu);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_solve(const SolveArgs &a, int n_wg, hipStream_t s) {
  return a.yfin ? launch_mode<1>(a, n_wg, s, nullptr) : launch_mode<0>(a, n_wg, s, nullptr);
}

hipError_t launch_solve_grad(const SolveArgs &a, int n_wg, hipStream_t s) {
  if (!a.yfin || !a.gterm || !a.gdiag) return hipErrorInvalidValue;
  return launch_mode<2>(a, n_wg, s, nullptr);
}

hipError_t solve_blocks_per_cu(const SolveArgs &a, int mode, int *per_cu) {
  *per_cu = 0;
  switch (mode) {
    case 0: return launch_mode<0>(a, 0, nullptr, per_cu);
    case 1: return launch_mode<1>(a, 0, nullptr, per_cu);
    default: return launch_mode<2>(a, 0, nullptr, per_cu);
  }
}

}  // namespace mbe3
