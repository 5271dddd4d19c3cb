// Batched symmetric eigensolvers for the pair preconditioner (eq. prec_eig).
// The generalized problem F x = e S x of a pair is reduced by canonical
// orthogonalisation (an overlap step, then a Fock step), so rank-deficient
// pair overlaps are handled by dropping overlap eigenvalues <= tau; the
// paper factors the overlap by Cholesky instead, which is the first try here
// too (cholesky_kernel), the eigen route taking over for slots it flags.
//
// Matrices whose workspace fits in LDS (order up to ~139) go to
// tridiag_qr_kernel: one wave per matrix, Householder reduction to
// tridiagonal form, the reflections accumulated in place, implicit QR steps
// with the Wilkinson shift, no workgroup barriers in the iteration.  Larger
// orders run cyclic Jacobi (jacobi_kernel) on a per-workgroup slice of global
// memory (L2 resident), the workgroups looping over their share of the
// tasks: the round-robin (circle) ordering lets n/2 disjoint rotations run
// concurrently, and a round applies J^T A J as independent 2x2 blocks
// J_k1^T A_(k1,k2) J_k2 (upper blocks only, mirrored) together with V <- V J.
//
// Rotation (Golub & Van Loan, sym.schur2): for a_pq != 0,
//   tau = (a_qq - a_pp) / (2 a_pq), t = sign(tau) / (|tau| + sqrt(1 + tau^2)),
//   c = 1 / sqrt(1 + t^2), s = t c, and A <- J^T A J with J_pp = J_qq = c,
//   J_pq = s, J_qp = -s, which zeroes a_pq.
#include <algorithm>

#include "internal.hpp"

namespace mbe3 {

static constexpr int JAC_MAX_SWEEPS = 40;
static constexpr double EV_SENTINEL = 1e30;

__device__ double block_sum(double v, double *red) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) red[w] = v;
  __syncthreads();
  double s = 0.0;
  const int nw = (blockDim.x + 63) >> 6;
  for (int i = 0; i < nw; ++i) s += red[i];
  return s;
}

__global__ __launch_bounds__(256) void jacobi_kernel(
    const EigTask *__restrict__ tasks, int n_tasks, const double *__restrict__ in,
    double *__restrict__ out, double *__restrict__ evals,
    int32_t *__restrict__ rank, int mode, double tau,
    const int32_t *__restrict__ only_flagged, int n_lo, int n_hi, double *gws,
    int64_t gstride) {
  // launched only for orders above the LDS limit, always on the global
  // workspace (a pointer known to be global: global, not flat, accesses)
  double *const sm = gws + (int64_t)blockIdx.x * gstride;
  for (int ti = blockIdx.x; ti < n_tasks; ti += gridDim.x) {
  const EigTask t = tasks[ti];
  if (t.n < n_lo || t.n > n_hi) continue;  // the other launch's task
  if (only_flagged && only_flagged[t.slot] == 0) continue;
  const int n = mode == 0 ? t.n : rank[t.slot];
  const int D = t.D;
  const int ld = n + 1;
  const int nh = (n + 1) >> 1;  // rotations per round
  double *A = sm;
  double *V = A + (size_t)n * ld;
  double *cs_c = V + (size_t)n * ld;
  double *cs_s = cs_c + nh + 1;
  double *lam = cs_s + nh + 1;
  double *red = lam + n + 1;
  int *pq = (int *)(red + 8);
  int *perm = pq + 2 * (nh + 1);
  const int tid = threadIdx.x;
  const int nt = blockDim.x;

  for (int e = tid; e < n * n; e += nt) {
    const int r = e / n, c = e - r * n;
    A[r * ld + c] = in[t.a_off + (int64_t)r * t.lda + c];
    V[r * ld + c] = (r == c) ? 1.0 : 0.0;
  }
  __syncthreads();

  const int nn = n + (n & 1);
  const int np = nn / 2;              // rotations per round
  const int nblk = np * (np + 1) / 2; // 2x2 blocks (k1 <= k2) of A
  for (int sweep = 0; sweep < JAC_MAX_SWEEPS && n > 1; ++sweep) {
    double off = 0.0, tot = 0.0;
    for (int e = tid; e < n * n; e += nt) {
      const int r = e / n, c = e - r * n;
      const double v = A[r * ld + c];
      tot += v * v;
      if (r != c) off += v * v;
    }
    off = block_sum(off, red);
    tot = block_sum(tot, red);
    if (!(off > 1e-30 * tot)) break;  // off-diagonal norm <= 1e-15 ||A||
    for (int round = 0; round < nn - 1; ++round) {
      // phase 1: the round's np disjoint rotations (circle ordering)
      if (tid < np) {
        const int k = tid;
        int a, b;
        if (k == 0) {
          a = round;
          b = nn - 1;
        } else {
          a = (round + k) % (nn - 1);
          b = (round - k + nn - 1) % (nn - 1);
        }
        const int p = a < b ? a : b, q = a < b ? b : a;
        double c = 1.0, s = 0.0;
        if (q < n) {
          const double apq = A[p * ld + q];
          if (apq != 0.0) {
            const double th = (A[q * ld + q] - A[p * ld + p]) / (2.0 * apq);
            double tt;
            if (fabs(th) > 1e150)
              tt = 0.5 / th;
            else
              tt = (th >= 0.0 ? 1.0 : -1.0) / (fabs(th) + sqrt(1.0 + th * th));
            c = 1.0 / sqrt(1.0 + tt * tt);
            s = tt * c;
          }
        }
        pq[2 * k] = p;
        pq[2 * k + 1] = q;
        cs_c[k] = c;
        cs_s[k] = s;
      }
      __syncthreads();
      // phase 2: A <- J^T A J as independent 2x2 blocks, V <- V J
      for (int e = tid; e < nblk; e += nt) {
        int k2 = (int)((sqrt(8.0 * e + 1.0) - 1.0) * 0.5);
        while (k2 * (k2 + 1) / 2 > e) --k2;
        while ((k2 + 1) * (k2 + 2) / 2 <= e) ++k2;
        const int k1 = e - k2 * (k2 + 1) / 2;  // k1 <= k2
        const double s1 = cs_s[k1], s2 = cs_s[k2];
        if (s1 == 0.0 && s2 == 0.0) continue;
        const double c1 = cs_c[k1], c2 = cs_c[k2];
        const int p1 = pq[2 * k1], q1 = pq[2 * k1 + 1];
        const int p2 = pq[2 * k2], q2 = pq[2 * k2 + 1];
        const bool h1 = q1 < n, h2 = q2 < n;  // second index exists
        const double b00 = A[p1 * ld + p2];
        const double b01 = h2 ? A[p1 * ld + q2] : 0.0;
        const double b10 = h1 ? A[q1 * ld + p2] : 0.0;
        const double b11 = (h1 && h2) ? A[q1 * ld + q2] : 0.0;
        // T = J1^T B (rows), B' = T J2 (columns)
        const double t00 = c1 * b00 - s1 * b10, t01 = c1 * b01 - s1 * b11;
        const double t10 = s1 * b00 + c1 * b10, t11 = s1 * b01 + c1 * b11;
        double n00 = c2 * t00 - s2 * t01, n01 = s2 * t00 + c2 * t01;
        double n10 = c2 * t10 - s2 * t11, n11 = s2 * t10 + c2 * t11;
        if (k1 == k2) { n01 = 0.0; n10 = 0.0; }  // rotated pair: zeroed
        A[p1 * ld + p2] = n00;
        if (h2) A[p1 * ld + q2] = n01;
        if (h1) A[q1 * ld + p2] = n10;
        if (h1 && h2) A[q1 * ld + q2] = n11;
        if (k1 != k2) {  // mirror into the lower block
          A[p2 * ld + p1] = n00;
          if (h2) A[q2 * ld + p1] = n01;
          if (h1) A[p2 * ld + q1] = n10;
          if (h1 && h2) A[q2 * ld + q1] = n11;
        }
      }
      for (int e = tid; e < np * n; e += nt) {
        const int k = e / n, i = e - k * n;
        const double s = cs_s[k];
        const int q = pq[2 * k + 1];
        if (q < n && s != 0.0) {
          const int p = pq[2 * k];
          const double c = cs_c[k];
          const double vp = V[i * ld + p], vq = V[i * ld + q];
          V[i * ld + p] = c * vp - s * vq;
          V[i * ld + q] = s * vp + c * vq;
        }
      }
      __syncthreads();
    }
  }

  // eigenvalues and ascending order (ties by index)
  for (int i = tid; i < n; i += nt) lam[i] = A[i * ld + i];
  __syncthreads();
  for (int i = tid; i < n; i += nt) {
    const double li = lam[i];
    int r = 0;
    for (int j = 0; j < n; ++j) {
      const double lj = lam[j];
      r += (lj < li) || (lj == li && j < i);
    }
    perm[r] = i;
  }
  __syncthreads();

  if (mode == 0) {
    __shared__ int first_kept;
    if (tid == 0) {
      int f = n;
      for (int r = 0; r < n; ++r)
        if (lam[perm[r]] > tau) { f = r; break; }
      first_kept = f;
      rank[t.slot] = n - f;
    }
    __syncthreads();
    const int f = first_kept, nk = n - f;
    for (int e = tid; e < n * D; e += nt) {
      const int r = e / D, c = e - r * D;
      double v = 0.0;
      if (c < nk) {
        const int src = perm[f + c];
        v = V[r * ld + src] / sqrt(lam[src]);
      }
      out[t.o_off + (int64_t)r * D + c] = v;
    }
    for (int c = tid; c < D; c += nt)
      evals[t.e_off + c] = c < nk ? lam[perm[f + c]] : EV_SENTINEL;
  } else {
    for (int e = tid; e < D * D; e += nt) {
      const int r = e / D, c = e - r * D;
      double v = 0.0;
      if (r < n && c < n) v = V[r * ld + perm[c]];
      out[t.o_off + (int64_t)r * D + c] = v;
    }
    for (int c = tid; c < D; c += nt)
      evals[t.e_off + c] = c < n ? lam[perm[c]] : EV_SENTINEL;
  }
  __syncthreads();  // the workspace is reused by the next task
  }
}

// Overlap step by Cholesky: S = L L^T in LDS (right-looking, one column per
// step), then L^{-1} column by column (forward substitution, one column per
// thread) and X0 = L^{-T}, which satisfies X0^T S X0 = 1 with the full rank.
// The slot keeps this basis only when ||L^{-1}||_F^2 < 1 / tau, which proves
// every eigenvalue of S above tau (the rank canonical orthogonalisation
// keeps is then n as well).  A pivot <= tau or a larger norm sets
// flag[slot] and leaves the slot to the canonical-orthogonalisation launch
// that follows.  GWS: the matrices live in a global-memory slice per
// workgroup (orders above the LDS limit); otherwise in LDS, through a pointer
// the compiler knows to be LDS (ds instructions, not flat ones).
template <bool GWS>
__global__ __launch_bounds__(256) void cholesky_kernel(
    const EigTask *__restrict__ tasks, int n_tasks, const double *__restrict__ in,
    double *__restrict__ out, double *__restrict__ evals,
    int32_t *__restrict__ rank, int32_t *__restrict__ flag, double tau, int n_lo,
    int n_hi, double *gws, int64_t gstride) {
  extern __shared__ double sm_dyn[];
  double *const sm = GWS ? gws + (int64_t)blockIdx.x * gstride : sm_dyn;
  __shared__ int failed;
  __shared__ double wsum[4];  // per-wave partial sums (256 threads)
  for (int ti = blockIdx.x; ti < n_tasks; ti += gridDim.x) {
  const EigTask t = tasks[ti];
  if (t.n < n_lo || t.n > n_hi) continue;  // the other launch's task
  const int n = t.n, D = t.D;
  // L and L^{-1} as packed lower triangles (row i starts at i (i + 1) / 2),
  // so that orders up to 142 fit 160 KB of LDS
  auto P = [](int i, int j) { return i * (i + 1) / 2 + j; };
  double *L = sm;                       // n (n + 1) / 2
  double *Li = sm + n * (n + 1) / 2;    // n (n + 1) / 2
  const int tid = threadIdx.x, nt = blockDim.x;
  for (int e = tid; e < n * n; e += nt) {
    const int r = e / n, c = e - r * n;
    if (c <= r) L[P(r, c)] = in[t.a_off + (int64_t)r * t.lda + c];
  }
  if (tid == 0) failed = 0;
  __syncthreads();
  for (int k = 0; k < n; ++k) {
    const double piv = L[P(k, k)];
    if (!(piv > tau)) {  // uniform: every thread reads the same value
      if (tid == 0) failed = 1;
      break;
    }
    const double lkk = sqrt(piv);
    const double inv = 1.0 / lkk;
    for (int i = k + 1 + tid; i < n; i += nt) L[P(i, k)] *= inv;
    __syncthreads();
    if (tid == 0) L[P(k, k)] = lkk;
    // trailing update of the lower triangle: the 256 threads as a 16 x 16
    // grid striding over its rows and columns (no triangular index to
    // invert per element)
    const int m = n - k - 1;  // trailing order
    const int ty = tid >> 4, tx = tid & 15;
    for (int ii = ty; ii < m; ii += 16) {
      const int i = k + 1 + ii;
      const double lik = L[P(i, k)];
      for (int jj = tx; jj <= ii; jj += 16) {
        const int j = k + 1 + jj;
        L[P(i, j)] -= lik * L[P(j, k)];
      }
    }
    __syncthreads();
  }
  __syncthreads();
  if (failed) {
    if (tid == 0) flag[t.slot] = 1;
    __syncthreads();
    continue;
  }
  // L^{-1}: four adjacent lanes solve L x = e_c for column c (rows >= c),
  // each summing the terms m2 = its lane (mod 4) of every row's dot product
  // (the long columns no longer hold one lane for the whole solve); the lane
  // that will read row i's value again is the one that stores it, and it
  // adds its square
  double ssq = 0.0;
  {
    const int sub = tid & 3;
    for (int c = tid >> 2; c < n; c += nt >> 2) {
      for (int i = c; i < n; ++i) {
        double part = 0.0;
        for (int m2 = c + sub; m2 < i; m2 += 4) part += L[P(i, m2)] * Li[P(m2, c)];
        part += __shfl_xor(part, 1, 64);
        part += __shfl_xor(part, 2, 64);
        const double v = (((i == c) ? 1.0 : 0.0) - part) / L[P(i, i)];
        if (sub == (i & 3)) {
          Li[P(i, c)] = v;
          ssq += v * v;
        }
      }
    }
  }
  // Positive pivots do not bound the smallest eigenvalue of S; the trace of
  // S^{-1} = L^{-T} L^{-1}, the squared Frobenius norm of L^{-1}, does:
  // 1 / lambda_min <= trace(S^{-1}).  So when ||L^{-1}||_F^2 < 1 / tau every
  // eigenvalue exceeds tau and canonical orthogonalisation would keep all n
  // directions too; otherwise the slot goes to that route (flag).  Fixed-
  // order sums: lane butterfly, then the four waves in order.
  for (int o = 32; o > 0; o >>= 1) ssq += __shfl_xor(ssq, o, 64);
  if ((tid & 63) == 0) wsum[tid >> 6] = ssq;
  __syncthreads();
  if (tid == 0) {
    double tr = 0.0;
    for (int w = 0; w < (nt + 63) / 64; ++w) tr += wsum[w];
    if (!(tr * tau < 1.0)) failed = 1;  // NaN fails too
  }
  __syncthreads();
  if (failed) {
    if (tid == 0) flag[t.slot] = 1;
    __syncthreads();
    continue;
  }
  // X0 = L^{-T}: X0[r][c] = Li[c][r], zero above the diagonal of Li
  for (int e = tid; e < n * D; e += nt) {
    const int r = e / D, c = e - r * D;
    out[t.o_off + (int64_t)r * D + c] = (c < n && c >= r) ? Li[P(c, r)] : 0.0;
  }
  for (int c = tid; c < D; c += nt) evals[t.e_off + c] = c < n ? 1.0 : EV_SENTINEL;
  if (tid == 0) {
    rank[t.slot] = n;
    flag[t.slot] = 0;
  }
  __syncthreads();  // the workspace is reused by the next task
  }
}

// ---------------------------------------------------------------------------
// Tridiagonal QR eigensolver, one wave per matrix (the default path).
//
// 1. Householder reduction A = Q T Q^T, T symmetric tridiagonal (Golub &
//    Van Loan, sec. 8.3.1): step k annihilates A[k+2:, k] with
//    H_k = I - tau_k v v^T, v = (1, v_{k+2}, ..., v_{n-1}), applied to the
//    trailing block as A22 <- A22 - v w^T - w v^T, p = tau A22 v,
//    w = p - (tau/2)(p.v) v.  v_{k+2..} is kept in column k.
// 2. Q = H_0 H_1 ... H_{n-3}, accumulated from the last reflector back to the
//    first over the same storage: the block of Q under construction
//    (rows and columns > k) never holds a reflector still to be applied.
// 3. Implicit symmetric QR steps with the Wilkinson shift (Golub & Van Loan,
//    Alg. 8.3.2) on the diagonal d and subdiagonal e: the bulge is chased
//    by Givens rotations that also rotate the columns of Q; a subdiagonal
//    entry at or below eps (|d_k| + |d_k+1|) splits the problem, and the
//    trailing unreduced block is iterated until its last entry splits off.
// Every lane evaluates the scalar recurrences of steps 1-3 itself (the same
// values in every lane, so no lane waits for another) and owns rows
// lane, lane + 64, ... for the vector work.  The matrix lives in LDS with an
// odd row pitch, the rows of a lane's column reads falling on distinct banks.
// ---------------------------------------------------------------------------
static __host__ __device__ inline int qr_pitch(int n) { return (n & 1) ? n : n + 1; }

static size_t qr_smem(int n) {
  return sizeof(double) * ((size_t)n * qr_pitch(n) + 5 * (size_t)n + 1) +
         sizeof(int) * ((size_t)n + 1);
}

__device__ inline double wave_sum(double v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  return v;
}

// 1 / sqrt(h) for h > 0: the hardware estimate and two Newton steps.
__device__ inline double rsqrt_nr(double h) {
  double y = __builtin_amdgcn_rsq(h);
  for (int it = 0; it < 2; ++it) {
    const double t = h * y;
    const double e = fma(-t, y, 1.0);
    y = fma(0.5 * y, e, y);
  }
  return y;
}

template <int RPL>
__global__ __launch_bounds__(64) void tridiag_qr_kernel(
    const EigTask *__restrict__ tasks, int n_tasks, const double *__restrict__ in,
    double *__restrict__ out, double *__restrict__ evals,
    int32_t *__restrict__ rank, int mode, double tau,
    const int32_t *__restrict__ only_flagged, int n_lo, int n_hi) {
  extern __shared__ double sm[];
  const int lane = threadIdx.x;
  for (int ti = blockIdx.x; ti < n_tasks; ti += gridDim.x) {
    const EigTask t = tasks[ti];
    if (t.n < n_lo || t.n > n_hi) continue;  // another launch's task
    if (only_flagged && only_flagged[t.slot] == 0) continue;
    const int n = mode == 0 ? t.n : rank[t.slot];
    const int D = t.D;
    const int ld = qr_pitch(n);
    double *const M = sm;
    double *const dd = M + (size_t)n * ld;
    double *const ee = dd + n;
    double *const vv = ee + n;
    double *const ww = vv + n;
    double *const taus = ww + n;
    int *const perm = reinterpret_cast<int *>(taus + n + 1);

    for (int e = lane; e < n * n; e += 64) {
      const int r = e / n, c = e - r * n;
      M[r * ld + c] = in[t.a_off + (int64_t)r * t.lda + c];
    }
    __syncthreads();

    // ---- 1. Householder reduction ----
    for (int k = 0; k + 2 < n; ++k) {
      double sig = 0.0;
#pragma unroll
      for (int j = 0; j < RPL; ++j) {
        const int i = lane + 64 * j;
        if (i >= k + 2 && i < n) {
          const double x = M[i * ld + k];
          sig += x * x;
        }
      }
      sig = wave_sum(sig);
      const double alpha = M[(k + 1) * ld + k];
      double tk = 0.0, beta = alpha;
      if (sig > 0.0) {
        const double nrm = sqrt(alpha * alpha + sig);
        beta = alpha >= 0.0 ? -nrm : nrm;
        tk = (beta - alpha) / beta;
        const double sc = 1.0 / (alpha - beta);
#pragma unroll
        for (int j = 0; j < RPL; ++j) {
          const int i = lane + 64 * j;
          if (i >= k + 2 && i < n) {
            const double v = M[i * ld + k] * sc;
            M[i * ld + k] = v;
            vv[i] = v;
          }
        }
        if (lane == 0) vv[k + 1] = 1.0;
      }
      if (lane == 0) {
        ee[k] = beta;
        taus[k] = tk;
        dd[k] = M[k * ld + k];
      }
      __syncthreads();
      if (tk != 0.0) {
        double p[RPL];
        double pv = 0.0;
#pragma unroll
        for (int j = 0; j < RPL; ++j) {
          const int i = lane + 64 * j;
          p[j] = 0.0;
          if (i >= k + 1 && i < n) {
            const double *row = M + i * ld;
            double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
            int c = k + 1;
            for (; c + 3 < n; c += 4) {  // four chains keep loads in flight
              a0 += row[c] * vv[c];
              a1 += row[c + 1] * vv[c + 1];
              a2 += row[c + 2] * vv[c + 2];
              a3 += row[c + 3] * vv[c + 3];
            }
            for (; c < n; ++c) a0 += row[c] * vv[c];
            p[j] = tk * ((a0 + a1) + (a2 + a3));
            pv += p[j] * vv[i];
          }
        }
        const double kk = 0.5 * tk * wave_sum(pv);
#pragma unroll
        for (int j = 0; j < RPL; ++j) {
          const int i = lane + 64 * j;
          if (i >= k + 1 && i < n) ww[i] = p[j] - kk * vv[i];
        }
        __syncthreads();
#pragma unroll
        for (int j = 0; j < RPL; ++j) {
          const int i = lane + 64 * j;
          if (i >= k + 1 && i < n) {
            const double vi = vv[i], wi = ww[i];
            double *row = M + i * ld;
#pragma unroll 4
            for (int c = k + 1; c < n; ++c) row[c] -= vi * ww[c] + wi * vv[c];
          }
        }
        __syncthreads();
      }
    }
    if (lane == 0 && n >= 1) {
      if (n >= 2) {
        dd[n - 2] = M[(n - 2) * ld + n - 2];
        ee[n - 2] = M[(n - 1) * ld + n - 2];
      }
      dd[n - 1] = M[(n - 1) * ld + n - 1];
      ee[n - 1] = 0.0;
    }
    __syncthreads();

    // ---- 2. Q in place, last reflector first ----
    if (n >= 2) {
      if (lane < 4) {
        const int r = n - 2 + (lane >> 1), c = n - 2 + (lane & 1);
        M[r * ld + c] = r == c ? 1.0 : 0.0;
      }
    } else if (n == 1 && lane == 0) {
      M[0] = 1.0;
    }
    __syncthreads();
    for (int k = n - 3; k >= 0; --k) {
      // row and column k + 1 of the block become the unit vector
      for (int c = k + 2 + lane; c < n; c += 64) {
        M[(k + 1) * ld + c] = 0.0;
        M[c * ld + k + 1] = 0.0;
      }
      if (lane == 0) M[(k + 1) * ld + k + 1] = 1.0;
      __syncthreads();
      const double tk = taus[k];
      if (tk != 0.0) {
        for (int c = k + 1 + lane; c < n; c += 64) {  // one column per lane
          double u0 = M[(k + 1) * ld + c], u1 = 0.0, u2 = 0.0, u3 = 0.0;
          int i = k + 2;
          for (; i + 3 < n; i += 4) {
            u0 += M[i * ld + k] * M[i * ld + c];
            u1 += M[(i + 1) * ld + k] * M[(i + 1) * ld + c];
            u2 += M[(i + 2) * ld + k] * M[(i + 2) * ld + c];
            u3 += M[(i + 3) * ld + k] * M[(i + 3) * ld + c];
          }
          for (; i < n; ++i) u0 += M[i * ld + k] * M[i * ld + c];
          const double u = tk * ((u0 + u1) + (u2 + u3));
          M[(k + 1) * ld + c] -= u;
#pragma unroll 4
          for (int i2 = k + 2; i2 < n; ++i2) M[i2 * ld + c] -= M[i2 * ld + k] * u;
        }
        __syncthreads();
      }
    }
    if (n >= 2) {
      for (int c = 1 + lane; c < n; c += 64) {
        M[c] = 0.0;
        M[c * ld] = 0.0;
      }
      if (lane == 0) M[0] = 1.0;
    }
    __syncthreads();

    // ---- 3. implicit QR steps with the Wilkinson shift ----
    constexpr double EPS = 2.220446049250313e-16;
    int m = n - 1;
    int steps = 0;
    const int max_steps = 30 * n + 30;
    while (m > 0 && steps < max_steps) {
      // l = 1 + the largest k < m with a negligible e[k] (0 if none): one
      // ballot over the lanes per 64 entries
      int l = 0;
#pragma unroll
      for (int j = RPL - 1; j >= 0; --j) {
        const int k = lane + 64 * j;
        const bool neg =
            k < m && fabs(ee[k]) <= EPS * (fabs(dd[k]) + fabs(dd[k + 1]));
        const unsigned long long b = __ballot(neg);
        if (l == 0 && b != 0ULL) l = 64 * j + 64 - __clzll((long long)b);
      }
      if (l == m) {  // d[m] has split off
        --m;
        continue;
      }
      ++steps;
      const double dm1 = dd[m - 1], dm = dd[m], b = ee[m - 1];
      const double del = 0.5 * (dm1 - dm);
      const double hyp = sqrt(del * del + b * b);
      const double mu = dm - b * b / (del + (del >= 0.0 ? hyp : -hyp));
      // d[k], e[k], d[k+1], e[k+1] and columns k, k+1 of Q travel in
      // registers; the next rotation's operands are loaded one step ahead
      double dk = dd[l], ek = ee[l];
      double dk1 = dd[l + 1];
      double ek1 = l + 1 < m ? ee[l + 1] : 0.0;
      double x = dk - mu, z = ek;
      double qc[RPL], qn[RPL];
#pragma unroll
      for (int j = 0; j < RPL; ++j) {
        const int i = lane + 64 * j;
        qc[j] = i < n ? M[i * ld + l] : 0.0;
        qn[j] = i < n ? M[i * ld + l + 1] : 0.0;
      }
      for (int k = l; k < m; ++k) {
        const double dk2 = k + 2 <= m ? dd[k + 2] : 0.0;
        const double ek2 = k + 2 < m ? ee[k + 2] : 0.0;
        double qnn[RPL];
#pragma unroll
        for (int j = 0; j < RPL; ++j) {
          const int i = lane + 64 * j;
          qnn[j] = (k + 2 <= m && i < n) ? M[i * ld + k + 2] : 0.0;
        }
        double c = 1.0, s = 0.0, r = x;
        const double hh = x * x + z * z;
        if (hh > 0.0) {
          const double ir = rsqrt_nr(hh);
          r = hh * ir;
          c = x * ir;
          s = -z * ir;
        }
        if (k > l) ee[k - 1] = r;  // the bulge is chased down: same value in every lane
        const double cs = c * s, c2 = c * c, s2 = s * s;
        const double nd0 = c2 * dk - 2.0 * cs * ek + s2 * dk1;
        const double nd1 = s2 * dk + 2.0 * cs * ek + c2 * dk1;
        const double ne = cs * (dk - dk1) + (c2 - s2) * ek;
        dd[k] = nd0;
#pragma unroll
        for (int j = 0; j < RPL; ++j) {  // column k is final, k + 1 carried
          const int i = lane + 64 * j;
          const double q0 = qc[j], q1 = qn[j];
          if (i < n) M[i * ld + k] = c * q0 - s * q1;
          qc[j] = s * q0 + c * q1;
          qn[j] = qnn[j];
        }
        if (k + 1 < m) {
          z = -s * ek1;  // new bulge at (k + 2, k)
          ek = c * ek1;
          x = ne;
          dk = nd1;
          dk1 = dk2;
          ek1 = ek2;
        } else {
          dd[k + 1] = nd1;
          ee[k] = ne;
        }
      }
#pragma unroll
      for (int j = 0; j < RPL; ++j) {
        const int i = lane + 64 * j;
        if (i < n) M[i * ld + m] = qc[j];
      }
    }
    const bool failed = m > 0;  // did not converge: reported as NaN eigenvalues
    __syncthreads();

    // ---- ascending order (ties by index) and outputs ----
    for (int i = lane; i < n; i += 64) {
      const double li = dd[i];
      int r = 0;
      for (int j = 0; j < n; ++j) {
        const double lj = dd[j];
        r += (lj < li) || (lj == li && j < i);
      }
      perm[r] = i;
    }
    __syncthreads();
    const double nanv = __builtin_nan("");
    if (mode == 0) {
      int f = n;
      for (int r = 0; r < n; ++r)
        if (dd[perm[r]] > tau) { f = r; break; }
      const int nk = n - f;
      if (lane == 0) rank[t.slot] = nk;
      for (int e = lane; e < n * D; e += 64) {
        const int r = e / D, c = e - r * D;
        double v = 0.0;
        if (c < nk) {
          const int src = perm[f + c];
          v = M[r * ld + src] / sqrt(dd[src]);
        }
        out[t.o_off + (int64_t)r * D + c] = v;
      }
      for (int c = lane; c < D; c += 64)
        evals[t.e_off + c] = c < nk ? (failed ? nanv : dd[perm[f + c]]) : EV_SENTINEL;
    } else {
      for (int e = lane; e < D * D; e += 64) {
        const int r = e / D, c = e - r * D;
        double v = 0.0;
        if (r < n && c < n) v = M[r * ld + perm[c]];
        out[t.o_off + (int64_t)r * D + c] = v;
      }
      for (int c = lane; c < D; c += 64)
        evals[t.e_off + c] = c < n ? (failed ? nanv : dd[perm[c]]) : EV_SENTINEL;
    }
    __syncthreads();  // the workspace is reused by the next task
  }
}

// ---------------------------------------------------------------------------
// Fock step (mode 1) in three launches.  In the fused kernel above the
// implicit QR steps take most of the time: the Givens chase is a serial
// chain of dependent FP64 operations, and while it runs the matrix Q holds
// the LDS, so above order ~90 one chase runs per CU.  Split:
//   house:  the Householder reduction and Q exactly as above (one wave per
//           matrix, in LDS); Q goes to the output block (pitch D), d and e
//           to the task's record;
//   chase:  the same implicit QR steps on d and e alone (2 KB of LDS per
//           wave, so chases fill the CU up to the wave limit), every step's
//           sweep bounds (l, m) and rotations (c, s) appended to the record;
//   apply:  Q back into LDS and the recorded rotations applied to its rows
//           in order with the fused kernel's arithmetic (column k + 2
//           loaded one rotation ahead, columns k, k + 1 carried in
//           registers), then the fused kernel's ordering and outputs.
// Record of a task (doubles at cws + w_off): d [D], e [D], sweep bounds
// [SC(D)] (two int32 each), rotations [2 RC(D)].  Typical solves need about
// 2n sweeps and 1.1 n^2 rotations; a task that would pass SC or RC is
// marked in redo[] and solved by the fused kernel afterwards.
// ---------------------------------------------------------------------------
static constexpr int SPLIT_MAX_ORDER = 128;
static __host__ __device__ inline int64_t chase_sc(int D) { return 4LL * D + 8; }
// rotations: about 1.1 n^2 plus up to 30 identity rotations per sweep that
// pad it to whole blocks of 16 columns
static __host__ __device__ inline int64_t chase_rc(int D) { return 2LL * D * D + 16 * chase_sc(D); }

int eig_split_max_order() { return SPLIT_MAX_ORDER; }
int64_t eig_chase_ws_doubles(int D) { return 2LL * D + chase_sc(D) + 2 * chase_rc(D); }

// rows x cols of a row-major global matrix (pitch gld) into LDS (pitch ld):
// rows over the four waves, columns over the lanes, eight loads of a wave
// in flight before their LDS stores (a load per iteration would wait out
// the memory latency every time).
__device__ __forceinline__ void copy_in_rows(double *M, int ld, const double *__restrict__ g,
                                             int64_t gld, int rows, int cols, int wv, int ln) {
  const int per_row = (cols + 63) / 64;
  const int total = ((rows - wv + 3) / 4) * per_row;  // this wave's (row, block) items
  for (int b = 0; b < total; b += 8) {
    double x[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int it = b + u;
      const int r = wv + 4 * (it / per_row), c = ln + 64 * (it % per_row);
      const bool ok = it < total && c < cols;
      const double y = g[ok ? (int64_t)r * gld + c : 0];  // index kept inside the matrix
      x[u] = ok ? y : 0.0;
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int it = b + u;
      const int r = wv + 4 * (it / per_row), c = ln + 64 * (it % per_row);
      if (it < total && c < cols) M[r * ld + c] = x[u];
    }
  }
}

// The reduction and Q of tridiag_qr_kernel with four waves per matrix (the
// LDS matrix allows one per CU): each row of the trailing block (reduction)
// and each column (Q) goes to a pair of adjacent lanes that split it by
// parity (orders up to 128), the two wave sums of a step become workgroup
// sums.
__global__ __launch_bounds__(256) void tridiag_house_kernel(
    const EigTask *__restrict__ tasks, int n_tasks, const double *__restrict__ in,
    double *__restrict__ out, const int32_t *__restrict__ rank, double *__restrict__ cws,
    int n_lo, int n_hi) {
  extern __shared__ double sm[];
  __shared__ double red[8];
  const int tid = threadIdx.x;
  for (int ti = blockIdx.x; ti < n_tasks; ti += gridDim.x) {
    const EigTask t = tasks[ti];
    const int n = rank[t.slot];
    // tasks without a record (order above the split path's) run fused
    if (t.w_off < 0 || n < n_lo || n > n_hi) continue;
    const int D = t.D;
    const int ld = qr_pitch(n);
    double *const M = sm;
    double *const dd = M + (size_t)n * ld;
    double *const ee = dd + n;
    double *const vv = ee + n;
    double *const ww = vv + n;
    double *const taus = ww + n;

    // rows over the four waves, columns over the lanes: coalesced, no
    // division, the loads of a row's column blocks in flight together
    const int wv = tid >> 6, ln = tid & 63;
    copy_in_rows(M, ld, in + t.a_off, t.lda, n, n, wv, ln);
    __syncthreads();
    // ---- Householder reduction (the steps of tridiag_qr_kernel) ----
    for (int k = 0; k + 2 < n; ++k) {
      double sig = 0.0;
      for (int i = k + 2 + tid; i < n; i += 256) {
        const double x = M[i * ld + k];
        sig += x * x;
      }
      sig = block_sum(sig, red);
      const double alpha = M[(k + 1) * ld + k];
      double tk = 0.0, beta = alpha;
      if (sig > 0.0) {
        const double nrm = sqrt(alpha * alpha + sig);
        beta = alpha >= 0.0 ? -nrm : nrm;
        tk = (beta - alpha) / beta;
        const double sc = 1.0 / (alpha - beta);
        for (int i = k + 2 + tid; i < n; i += 256) {
          const double v = M[i * ld + k] * sc;
          M[i * ld + k] = v;
          vv[i] = v;
        }
        if (tid == 0) vv[k + 1] = 1.0;
      }
      if (tid == 0) {
        ee[k] = beta;
        taus[k] = tk;
        dd[k] = M[k * ld + k];
      }
      __syncthreads();
      if (tk != 0.0) {
        // two adjacent lanes per row (orders up to 128 on 256 threads), each
        // taking the columns of one parity; the halves meet by a lane swap,
        // even columns first
        double pv = 0.0;
        double pj = 0.0;
        const int h = tid & 1;
        const int i = k + 1 + (tid >> 1);
        double part = 0.0;
        if (i < n) {
          const double *row = M + i * ld;
          double a0 = 0.0, a1 = 0.0;
          int c = k + 1 + h;
          for (; c + 2 < n; c += 4) {
            a0 += row[c] * vv[c];
            a1 += row[c + 2] * vv[c + 2];
          }
          for (; c < n; c += 2) a0 += row[c] * vv[c];
          part = a0 + a1;
        }
        const double other = __shfl_xor(part, 1);
        if (i < n) {
          pj = tk * (h == 0 ? part + other : other + part);
          if (h == 0) pv = pj * vv[i];
        }
        const double kk = 0.5 * tk * block_sum(pv, red);
        if (i < n && h == 0) ww[i] = pj - kk * vv[i];
        __syncthreads();
        if (i < n) {
          const double vi = vv[i], wi = ww[i];
          double *row = M + i * ld;
#pragma unroll 4
          for (int c = k + 1 + h; c < n; c += 2) row[c] -= vi * ww[c] + wi * vv[c];
        }
        __syncthreads();
      }
    }
    if (tid == 0 && n >= 1) {
      if (n >= 2) {
        dd[n - 2] = M[(n - 2) * ld + n - 2];
        ee[n - 2] = M[(n - 1) * ld + n - 2];
      }
      dd[n - 1] = M[(n - 1) * ld + n - 1];
      ee[n - 1] = 0.0;
    }
    __syncthreads();
    // ---- Q in place, last reflector first ----
    if (n >= 2) {
      if (tid < 4) {
        const int r = n - 2 + (tid >> 1), c = n - 2 + (tid & 1);
        M[r * ld + c] = r == c ? 1.0 : 0.0;
      }
    } else if (n == 1 && tid == 0) {
      M[0] = 1.0;
    }
    __syncthreads();
    for (int k = n - 3; k >= 0; --k) {
      for (int c = k + 2 + tid; c < n; c += 256) {
        M[(k + 1) * ld + c] = 0.0;
        M[c * ld + k + 1] = 0.0;
      }
      if (tid == 0) M[(k + 1) * ld + k + 1] = 1.0;
      __syncthreads();
      const double tk = taus[k];
      if (tk != 0.0) {
        // two adjacent lanes per column, each taking the rows of one parity
        // (both lanes of a pair run the same columns, so the swap partner is
        // always active)
        const int h = tid & 1;
        for (int c = k + 1 + (tid >> 1); c < n; c += 128) {
          double u0 = h == 0 ? M[(k + 1) * ld + c] : 0.0, u1 = 0.0;
          int i = k + 2 + h;
          for (; i + 2 < n; i += 4) {
            u0 += M[i * ld + k] * M[i * ld + c];
            u1 += M[(i + 2) * ld + k] * M[(i + 2) * ld + c];
          }
          for (; i < n; i += 2) u0 += M[i * ld + k] * M[i * ld + c];
          const double part = u0 + u1;
          const double other = __shfl_xor(part, 1);
          const double u = tk * (h == 0 ? part + other : other + part);
          if (h == 0) M[(k + 1) * ld + c] -= u;
#pragma unroll 4
          for (int i2 = k + 2 + h; i2 < n; i2 += 2) M[i2 * ld + c] -= M[i2 * ld + k] * u;
        }
        __syncthreads();
      }
    }
    if (n >= 2) {
      for (int c = 1 + tid; c < n; c += 256) {
        M[c] = 0.0;
        M[c * ld] = 0.0;
      }
      if (tid == 0) M[0] = 1.0;
    }
    __syncthreads();
    // ---- Q to the output block, d and e to the record ----
    for (int r = wv; r < n; r += 4)
      for (int c = ln; c < n; c += 64) out[t.o_off + (int64_t)r * D + c] = M[r * ld + c];
    double *const rec = cws + t.w_off;
    for (int i = tid; i < n; i += 256) {
      rec[i] = dd[i];
      rec[D + i] = ee[i];
    }
    __syncthreads();  // the workspace is reused by the next task
  }
}

__global__ __launch_bounds__(64) void tridiag_chase_kernel(
    const EigTask *__restrict__ tasks, int n_tasks, const int32_t *__restrict__ rank,
    double *__restrict__ cws, int32_t *__restrict__ meta, int n_lo, int n_hi) {
  __shared__ double dd[SPLIT_MAX_ORDER + 1], ee[SPLIT_MAX_ORDER + 1];
  constexpr int RPL = (SPLIT_MAX_ORDER + 63) / 64;
  const int lane = threadIdx.x;
  for (int ti = blockIdx.x; ti < n_tasks; ti += gridDim.x) {
    const EigTask t = tasks[ti];
    const int n = rank[t.slot];
    // tasks without a record (order above the split path's) run fused
    if (t.w_off < 0 || n < n_lo || n > n_hi) continue;
    const int D = t.D;
    double *const rec = cws + t.w_off;
    int32_t *const bounds = reinterpret_cast<int32_t *>(rec + 2 * D);
    double *const rot = rec + 2 * D + chase_sc(D);
    const int64_t cap_s = chase_sc(D), cap_r = chase_rc(D);
    for (int i = lane; i < n; i += 64) {
      dd[i] = rec[i];
      ee[i] = rec[D + i];
    }
    __syncthreads();
    // ---- the implicit QR steps of tridiag_qr_kernel on d and e alone ----
    constexpr double EPS = 2.220446049250313e-16;
    int m = n - 1;
    int steps = 0;
    const int max_steps = 30 * n + 30;
    int64_t ns = 0, nr = 0;
    int ovf = 0;
    while (m > 0 && steps < max_steps) {
      int l = 0;
#pragma unroll
      for (int j = RPL - 1; j >= 0; --j) {
        const int k = lane + 64 * j;
        const bool neg =
            k < m && fabs(ee[k]) <= EPS * (fabs(dd[k]) + fabs(dd[k + 1]));
        const unsigned long long b = __ballot(neg);
        if (l == 0 && b != 0ULL) l = 64 * j + 64 - __clzll((long long)b);
      }
      if (l == m) {
        --m;
        continue;
      }
      ++steps;
      // the sweep's record covers columns bl .. bm - 1 (whole 16-blocks):
      // identity rotations before l and from m on
      const int bl = l & ~15, bm = ((m - 1) | 15) + 1;
      if (ns >= cap_s || nr + (bm - bl) > cap_r) {  // the record is full
        ovf = 1;
        break;
      }
      if (lane == 0) {
        bounds[2 * ns] = l;
        bounds[2 * ns + 1] = m;
        for (int k = bl; k < l; ++k) {
          rot[2 * (nr + k - bl)] = 1.0;
          rot[2 * (nr + k - bl) + 1] = 0.0;
        }
        for (int k = m; k < bm; ++k) {
          rot[2 * (nr + k - bl)] = 1.0;
          rot[2 * (nr + k - bl) + 1] = 0.0;
        }
      }
      ++ns;
      nr += l - bl;  // the sweep's own rotations follow its leading pad
      const double dm1 = dd[m - 1], dm = dd[m], b = ee[m - 1];
      const double del = 0.5 * (dm1 - dm);
      const double hyp = sqrt(del * del + b * b);
      const double mu = dm - b * b / (del + (del >= 0.0 ? hyp : -hyp));
      double dk = dd[l], ek = ee[l];
      double dk1 = dd[l + 1];
      double ek1 = l + 1 < m ? ee[l + 1] : 0.0;
      double x = dk - mu, z = ek;
      for (int k = l; k < m; ++k) {
        const double dk2 = k + 2 <= m ? dd[k + 2] : 0.0;
        const double ek2 = k + 2 < m ? ee[k + 2] : 0.0;
        double c = 1.0, s = 0.0, r = x;
        const double hh = x * x + z * z;
        if (hh > 0.0) {
          const double ir = rsqrt_nr(hh);
          r = hh * ir;
          c = x * ir;
          s = -z * ir;
        }
        if (k > l) ee[k - 1] = r;
        const double cs = c * s, c2 = c * c, s2 = s * s;
        const double nd0 = c2 * dk - 2.0 * cs * ek + s2 * dk1;
        const double nd1 = s2 * dk + 2.0 * cs * ek + c2 * dk1;
        const double ne = cs * (dk - dk1) + (c2 - s2) * ek;
        dd[k] = nd0;
        if (lane == 0) {
          rot[2 * nr] = c;
          rot[2 * nr + 1] = s;
        }
        ++nr;
        if (k + 1 < m) {
          z = -s * ek1;
          ek = c * ek1;
          x = ne;
          dk = nd1;
          dk1 = dk2;
          ek1 = ek2;
        } else {
          dd[k + 1] = nd1;
          ee[k] = ne;
        }
      }
      nr += ((m - 1) | 15) + 1 - m;  // the trailing pad
    }
    __syncthreads();
    for (int i = lane; i < n; i += 64) rec[i] = dd[i];  // the eigenvalues, unsorted
    if (lane == 0) {
      int32_t *mt = meta + 4 * (int64_t)ti;
      mt[0] = (int32_t)ns;
      mt[1] = (int32_t)nr;
      mt[2] = (!ovf && m > 0) ? 1 : 0;  // did not converge
      mt[3] = ovf;
    }
    __syncthreads();  // dd and ee are reused by the next task
  }
}

// LDS of the apply launch: Q (n x pitch), d, the rotation stage, perm and
// the sweep bounds of the largest record.
static size_t apply_smem(int n, int stage) {
  return sizeof(double) * ((size_t)n * qr_pitch(n) + (size_t)n + 2 * (size_t)stage) +
         sizeof(int) * ((size_t)n + 1 + 2 * (size_t)chase_sc(SPLIT_MAX_ORDER));
}

// Four waves per matrix: the rotations act on the rows of Q independently,
// so row i belongs to lane i % RW of wave i / RW (RW = ceil(n_hi / 4) rows
// per wave), and the four SIMDs of the CU each carry a quarter of the rows
// through the whole record (the LDS matrix allows one matrix per CU).  The
// waves meet only at the stage refills.
__global__ __launch_bounds__(256) void tridiag_apply_kernel(
    const EigTask *__restrict__ tasks, int n_tasks, const int32_t *__restrict__ rank,
    const double *__restrict__ cws, const int32_t *__restrict__ meta,
    double *__restrict__ out, double *__restrict__ evals, int32_t *__restrict__ redo,
    int stage, int n_lo, int n_hi) {
  extern __shared__ double sm[];
  const int tid = threadIdx.x;
  const int rw = (n_hi + 3) / 4;  // rows per wave
  const int lane = tid & 63, wave = tid >> 6;
  const int my_row = lane < rw ? wave * rw + lane : -1;
  for (int ti = blockIdx.x; ti < n_tasks; ti += gridDim.x) {
    const EigTask t = tasks[ti];
    const int n = rank[t.slot];
    // tasks without a record (order above the split path's) run fused
    if (t.w_off < 0 || n < n_lo || n > n_hi) continue;
    const int32_t *mt = meta + 4 * (int64_t)ti;
    const int ns = mt[0];
    const int64_t nr = mt[1];
    const bool failed = mt[2] != 0;
    const int ovf = mt[3];
    if (tid == 0) redo[t.slot] = ovf;
    if (ovf) continue;  // the fused kernel solves it
    const int D = t.D;
    const int ld = qr_pitch(n);
    double *const M = sm;
    double *const dd = M + (size_t)n * ld;
    double *const st = dd + n;
    int *const perm = reinterpret_cast<int *>(st + 2 * stage);
    int *const bnd = perm + n + 1;  // the sweep bounds, staged once per task
    const double *const rec = cws + t.w_off;
    const int32_t *const bounds = reinterpret_cast<const int32_t *>(rec + 2 * D);
    const double *const rot = rec + 2 * D + chase_sc(D);
    copy_in_rows(M, ld, out + t.o_off, D, n, n, wave, lane);
    for (int i = tid; i < n; i += 256) dd[i] = rec[i];
    for (int e = tid; e < 2 * ns; e += 256) bnd[e] = bounds[e];
    __syncthreads();
    // ---- the recorded rotations, in order, on this thread's row ----
    // A sweep (l, m) rotates columns (k, k + 1) for k = l .. m - 1 in turn;
    // its record covers the whole 16-column blocks from bl = 16 floor(l/16)
    // to bm = 16 ceil(m/16), identity rotations (c = 1, s = 0, which leave
    // both values exactly as they are) outside [l, m).  Each block: the
    // row's 16 values and the 16 rotations come in at once, the rotations
    // run in registers (v[q] is column bl + 16 b + q, v[16] the next
    // block's first, carried).
    const int i = my_row < n ? my_row : -1;
    double *const Mi = M + (i >= 0 ? i : 0) * ld;
    int64_t j0 = 0, j1 = 0;  // rotations [j0, j1) are staged
    int64_t j = 0;           // first rotation of the sweep's record
    for (int h = 0; h < ns; ++h) {
      const int l = bnd[2 * h], m = bnd[2 * h + 1];
      const int bl = l & ~15, bm = ((m - 1) | 15) + 1;
      if (j + (bm - bl) > j1) {  // the sweep's record into the stage (uniform)
        __syncthreads();
        j0 = j;
        const int64_t cnt = nr - j0 < stage ? nr - j0 : stage;
        j1 = j0 + cnt;
        {
          double x[4];
#pragma unroll
          for (int u = 0; u < 4; ++u) {  // 2 * stage <= 1024 = 4 * 256
            const int64_t e = tid + 256 * u;
            const double y = rot[2 * j0 + (e < 2 * cnt ? e : 0)];  // index kept inside the record
            x[u] = e < 2 * cnt ? y : 0.0;
          }
#pragma unroll
          for (int u = 0; u < 4; ++u) {
            const int64_t e = tid + 256 * u;
            if (e < 2 * cnt) st[e] = x[u];
          }
        }
        __syncthreads();
      }
      const double *sr = st + 2 * (j - j0);  // rotation of column bl + 16 b + q at sr[2 (16 b + q)]
      double v[17];
      v[0] = (i >= 0) ? Mi[bl] : 0.0;
      for (int c0 = bl; c0 < bm; c0 += 16, sr += 32) {
        const bool inner = c0 + 16 < n;  // the block and its carry inside the row (uniform)
        if (inner) {
#pragma unroll
          for (int q = 1; q <= 16; ++q) v[q] = Mi[c0 + q];
        } else {
          // the row's last block: reads clamped into the row, columns past
          // it held at zero
#pragma unroll
          for (int q = 1; q <= 16; ++q) {
            const double x = Mi[c0 + q < n ? c0 + q : n - 1];
            v[q] = c0 + q < n ? x : 0.0;
          }
        }
#pragma unroll
        for (int q = 0; q < 16; ++q) {
          const double c = sr[2 * q], s = sr[2 * q + 1];
          const double q0 = v[q], q1 = v[q + 1];
          v[q] = c * q0 - s * q1;
          v[q + 1] = s * q0 + c * q1;
        }
        if (i >= 0) {
          if (inner) {
#pragma unroll
            for (int q = 0; q < 16; ++q) Mi[c0 + q] = v[q];
          } else {
#pragma unroll
            for (int q = 0; q < 16; ++q)
              if (c0 + q < n) Mi[c0 + q] = v[q];
          }
        }
        v[0] = v[16];
      }
      if (i >= 0 && bm < n) Mi[bm] = v[0];
      j += bm - bl;
    }
    __syncthreads();
    // ---- ascending order (ties by index) and the mode-1 outputs ----
    for (int r0 = tid; r0 < n; r0 += 256) {
      const double li = dd[r0];
      int r = 0;
      for (int q = 0; q < n; ++q) {
        const double lj = dd[q];
        r += (lj < li) || (lj == li && q < r0);
      }
      perm[r] = r0;
    }
    __syncthreads();
    const double nanv = __builtin_nan("");
    for (int r = wave; r < D; r += 4)
      for (int c = lane; c < D; c += 64) {
        double v = 0.0;
        if (r < n && c < n) v = M[r * ld + perm[c]];
        out[t.o_off + (int64_t)r * D + c] = v;
      }
    for (int c = tid; c < D; c += 256)
      evals[t.e_off + c] = c < n ? (failed ? nanv : dd[perm[c]]) : EV_SENTINEL;
    __syncthreads();  // the workspace is reused by the next task
  }
}

static size_t cholesky_smem(int n) { return sizeof(double) * (size_t)n * (n + 1); }

static size_t jacobi_smem(int n) {
  const int ld = n + 1, nh = (n + 1) / 2;
  return sizeof(double) * ((size_t)2 * n * ld + 2 * (nh + 1) + (n + 1) + 8) +
         sizeof(int) * (2 * (nh + 1) + n + 1);
}

static constexpr size_t EIG_LDS = 160 * 1024;

// Largest order whose workspace fits in LDS.
static int lds_order(size_t (*bytes)(int)) {
  int n = 1;
  while (bytes(n + 1) <= EIG_LDS) ++n;
  return n;
}

int64_t eig_workspace_doubles(int max_n) {
  const size_t b = std::max(jacobi_smem(max_n), cholesky_smem(max_n));
  return (int64_t)((b + 255) / 256 * 256 / sizeof(double));
}
int eig_lds_max_order() { return std::min(lds_order(jacobi_smem), lds_order(cholesky_smem)); }

// Launch the LDS variant for tasks of order <= the LDS limit and, if needed,
// the global-workspace variant (grid bounded by the workspace) for the rest.
template <class Launch>
static hipError_t two_launches(int n_tasks, int max_n, size_t (*bytes)(int),
                               double *gws, int64_t gws_doubles, Launch launch) {
  const int nl = lds_order(bytes);
  const int hi = std::min(max_n, nl);
  hipError_t e = launch(n_tasks, 0, hi, nullptr, (int64_t)0, bytes(hi));
  if (e != hipSuccess || max_n <= nl) return e;
  const int64_t stride = eig_workspace_doubles(max_n);
  if (!gws || gws_doubles < stride) return hipErrorInvalidValue;
  const int grid = (int)std::min<int64_t>(n_tasks, gws_doubles / stride);
  return launch(grid, nl + 1, max_n, gws, stride, (size_t)0);
}

hipError_t launch_cholesky(const EigTask *d_tasks, int n_tasks, int max_n,
                           const double *in, double *out, double *evals,
                           int32_t *rank, int32_t *flag, double tau, double *gws,
                           int64_t gws_doubles, hipStream_t s) {
  if (n_tasks <= 0) return hipSuccess;
  return two_launches(n_tasks, max_n, cholesky_smem, gws, gws_doubles,
                      [&](int grid, int lo, int hi, double *ws, int64_t stride,
                          size_t smem) -> hipError_t {
                        if (ws) {
                          hipLaunchKernelGGL(cholesky_kernel<true>, dim3(grid), dim3(256), 0,
                                             s, d_tasks, n_tasks, in, out, evals, rank,
                                             flag, tau, lo, hi, ws, stride);
                          return hipGetLastError();
                        }
                        hipError_t e = hipFuncSetAttribute(
                            (const void *)cholesky_kernel<false>,
                            hipFuncAttributeMaxDynamicSharedMemorySize, (int)smem);
                        if (e != hipSuccess) return e;
                        hipLaunchKernelGGL(cholesky_kernel<false>, dim3(grid), dim3(256),
                                           smem, s, d_tasks, n_tasks, in, out, evals,
                                           rank, flag, tau, lo, hi, ws, stride);
                        return hipGetLastError();
                      });
}

template <int RPL>
static hipError_t launch_qr(const EigTask *d_tasks, int n_tasks, int lo, int hi,
                            const double *in, double *out, double *evals,
                            int32_t *rank, int mode, double tau,
                            const int32_t *only_flagged, hipStream_t s) {
  const size_t smem = qr_smem(hi);
  hipError_t e = hipFuncSetAttribute((const void *)tridiag_qr_kernel<RPL>,
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)smem);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((tridiag_qr_kernel<RPL>), dim3(n_tasks), dim3(64), smem, s, d_tasks,
                     n_tasks, in, out, evals, rank, mode, tau, only_flagged, lo, hi);
  return hipGetLastError();
}

int eig_qr_max_order() { return std::min(lds_order(qr_smem), 192); }

hipError_t launch_eigh(const EigTask *d_tasks, int n_tasks, int max_n,
                       const double *in, double *out, double *evals, int32_t *rank,
                       int mode, double tau, const int32_t *only_flagged, double *gws,
                       int64_t gws_doubles, hipStream_t s) {
  if (n_tasks <= 0) return hipSuccess;
  // orders up to the LDS limit: one wave per matrix, in ranges of 64 rows
  // so that each launch reserves the LDS of its own largest order
  const int nq = eig_qr_max_order();
  hipError_t e = hipSuccess;
  for (int lo = 1; lo <= std::min(max_n, nq) && e == hipSuccess; lo += 64) {
    const int hi = std::min(std::min(max_n, nq), lo + 63);
    if (hi <= 64)
      e = launch_qr<1>(d_tasks, n_tasks, lo, hi, in, out, evals, rank, mode, tau,
                       only_flagged, s);
    else if (hi <= 128)
      e = launch_qr<2>(d_tasks, n_tasks, lo, hi, in, out, evals, rank, mode, tau,
                       only_flagged, s);
    else
      e = launch_qr<3>(d_tasks, n_tasks, lo, hi, in, out, evals, rank, mode, tau,
                       only_flagged, s);
  }
  if (e != hipSuccess || max_n <= nq) return e;
  // larger orders: cyclic Jacobi on a global-memory slice per workgroup
  const int64_t stride = eig_workspace_doubles(max_n);
  if (!gws || gws_doubles < stride) return hipErrorInvalidValue;
  const int grid = (int)std::min<int64_t>(n_tasks, gws_doubles / stride);
  hipLaunchKernelGGL(jacobi_kernel, dim3(grid), dim3(256), 0, s, d_tasks, n_tasks, in, out,
                     evals, rank, mode, tau, only_flagged, nq + 1, max_n, gws, stride);
  return hipGetLastError();
}

hipError_t launch_eigh_split(const EigTask *d_tasks, int n_tasks, int max_n,
                             const double *in, double *out, double *evals,
                             int32_t *rank, double *cws, int32_t *meta, int32_t *redo,
                             double *gws, int64_t gws_doubles, hipStream_t s) {
  if (n_tasks <= 0) return hipSuccess;
  if (!cws || !meta || !redo) return hipErrorInvalidValue;
  hipError_t e = hipSuccess;
  const int top = std::min(max_n, SPLIT_MAX_ORDER);
  for (int lo = 1; lo <= top && e == hipSuccess; lo += 64) {
    const int hi = std::min(top, lo + 63);
    // the split launches select tasks by their order rank[slot] (order 0,
    // an empty basis, in the first range); the fused fallback by t.n, the
    // range whose LDS it reserved: each task's redo flag is written by the
    // apply launch of its order's range, before the fallback of t.n's
    const int rlo = lo == 1 ? 0 : lo;
    const size_t hs = qr_smem(hi);
    // 512 staged rotations (8 KB) keep the record's reads off the chain;
    // more would only take LDS from other workgroups
    int stage = (int)std::min<int64_t>(512, ((int64_t)EIG_LDS - (int64_t)apply_smem(hi, 0)) / 16);
    stage = stage / 64 * 64;
    if (stage < 64) return hipErrorInvalidValue;
    const size_t as = apply_smem(hi, stage);
    if (hi <= 64) {
      e = hipFuncSetAttribute((const void *)tridiag_house_kernel,
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)hs);
      if (e == hipSuccess)
        e = hipFuncSetAttribute((const void *)tridiag_apply_kernel,
                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)as);
      if (e != hipSuccess) return e;
      hipLaunchKernelGGL(tridiag_house_kernel, dim3(n_tasks), dim3(256), hs, s, d_tasks,
                         n_tasks, in, out, rank, cws, rlo, hi);
      hipLaunchKernelGGL(tridiag_chase_kernel, dim3(n_tasks), dim3(64), 0, s, d_tasks,
                         n_tasks, rank, cws, meta, rlo, hi);
      hipLaunchKernelGGL(tridiag_apply_kernel, dim3(n_tasks), dim3(256), as, s, d_tasks,
                         n_tasks, rank, cws, meta, out, evals, redo, stage, rlo, hi);
      e = hipGetLastError();
      if (e == hipSuccess)  // records that overflowed: the fused kernel
        e = launch_qr<1>(d_tasks, n_tasks, lo, hi, in, out, evals, rank, 1, 0.0, redo, s);
    } else {
      e = hipFuncSetAttribute((const void *)tridiag_house_kernel,
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)hs);
      if (e == hipSuccess)
        e = hipFuncSetAttribute((const void *)tridiag_apply_kernel,
                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)as);
      if (e != hipSuccess) return e;
      hipLaunchKernelGGL(tridiag_house_kernel, dim3(n_tasks), dim3(256), hs, s, d_tasks,
                         n_tasks, in, out, rank, cws, rlo, hi);
      hipLaunchKernelGGL(tridiag_chase_kernel, dim3(n_tasks), dim3(64), 0, s, d_tasks,
                         n_tasks, rank, cws, meta, rlo, hi);
      hipLaunchKernelGGL(tridiag_apply_kernel, dim3(n_tasks), dim3(256), as, s, d_tasks,
                         n_tasks, rank, cws, meta, out, evals, redo, stage, rlo, hi);
      e = hipGetLastError();
      if (e == hipSuccess)
        e = launch_qr<2>(d_tasks, n_tasks, lo, hi, in, out, evals, rank, 1, 0.0, redo, s);
    }
  }
  if (e != hipSuccess || max_n <= SPLIT_MAX_ORDER) return e;
  // orders above the split path: the fused kernel, then cyclic Jacobi
  const int nq = eig_qr_max_order();
  for (int lo = SPLIT_MAX_ORDER + 1; lo <= std::min(max_n, nq) && e == hipSuccess; lo += 64) {
    const int hi = std::min(std::min(max_n, nq), lo + 63);
    e = launch_qr<3>(d_tasks, n_tasks, lo, hi, in, out, evals, rank, 1, 0.0, nullptr, s);
  }
  if (e != hipSuccess || max_n <= nq) return e;
  const int64_t stride = eig_workspace_doubles(max_n);
  if (!gws || gws_doubles < stride) return hipErrorInvalidValue;
  const int grid = (int)std::min<int64_t>(n_tasks, gws_doubles / stride);
  hipLaunchKernelGGL(jacobi_kernel, dim3(grid), dim3(256), 0, s, d_tasks, n_tasks, in, out,
                     evals, rank, 1, 0.0, nullptr, nq + 1, max_n, gws, stride);
  return hipGetLastError();
}

}  // namespace mbe3
