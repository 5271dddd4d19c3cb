/*
 * mbe3osv.h -- C-ABI of the MBE(3)-OSV-MP2 hot path on one AMD Instinct
 * MI355X (gfx950).
 *
 * Method: Liang & Yang, "Multi-GPU MBE(3)-OSV-MP2 for Performant Large-Scale
 * ab initio Calculations", arXiv:2603.16575.  The calls below follow the
 * paper's statement of the problem (section "MBE(3)-OSV-MP2 Method") and the
 * outputs of its Algorithms 5-7:
 *
 *   osv_project     regenerated RI slabs (ia|P) projected onto the OSVs of
 *                   every neighbour (eq. osv_imua; the slab stands in for the
 *                   fitted Gamma_i of eq. fitting / Algorithm 1)
 *   pair_K          4-block pair exchange matrices K_(pq,pq)
 *                   (eq. osv_close_k, Algorithm 6)
 *   fragment_solve  OSV overlap/Fock blocks (Algorithm 5), pair
 *                   preconditioner bases (eq. prec_eig) and the coupled
 *                   residual equations of every 1-, 2- and 3-orbital
 *                   fragment (eq. res_close, Algorithm 7)
 *   mbe3_energy     MBE(3) sum of fragment energies (eqs. tmbediag, tmbeoff)
 *   mbe3_backward   dE/d(ia|P) and dE/df_occ (derived from Hylleraas
 *                   stationarity; the paper names analytic gradients only as
 *                   future work)
 *
 * Conventions for every call:
 *   - Arrays are caller-owned.  "device" pointers are HIP device memory on
 *     the handle's device; "host" pointers are ordinary host memory.
 *   - All floating point data is IEEE double, row-major.
 *   - Every call is ordered on the handle's stream (hipStream_t passed as
 *     void*; NULL = the default stream).  In the forward path mbe3_energy
 *     (which returns the sum) and fragment_solve (which returns the
 *     fragments' convergence status) synchronise the stream when called
 *     directly; inside a recording neither does, and mbe3_graph_launch
 *     checks the status after each replay.  Other calls that synchronise
 *     say so below.
 *   - Every call returns an int status (MBE3_*).  On failure,
 *     mbe3_last_error() describes the cause.  No C++ exception crosses the
 *     ABI.  The library allocates its own device workspace (at create and
 *     on first use); it never frees or writes caller memory other than the
 *     documented outputs.
 *   - The handle is not thread safe; concurrent calls on one handle race.
 *
 * Index conventions:
 *   LMO i in [0, n_occ) has r[i] OSVs; q_off[i] = r[0] + ... + r[i-1].
 *   N+(i) = {i} united with every j such that the pair (i, j) is kept,
 *   in ascending order.
 *   Pair slots: slot s < n_occ is the diagonal pair (s, s); slot n_occ + m
 *   is kept pair m of the `pairs` list.  d_s = r[p] for (p, p) and
 *   r[p] + r[q] for (p, q); the pair domain is V_pq = [Q_p Q_q] (or Q_p).
 */
#ifndef MBE3OSV_H
#define MBE3OSV_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ------------------------------------------------------ */
#define MBE3_OK 0
#define MBE3_EINVAL (-1)     /* bad sizes, lists or arguments              */
#define MBE3_ENOMEM (-2)     /* device allocation failed / too large       */
#define MBE3_EHIP (-3)       /* a HIP runtime call failed                  */
#define MBE3_ENOCONV (-4)    /* a fragment hit max_iter (iters[f] < 0)     */
#define MBE3_ENONFINITE (-5) /* NaN/Inf met in a residual or an energy     */

/* Arithmetic of osv_project and pair_K (everything else is FP64 always). */
#define MBE3_FP64 0
/* Split precision (eq. osv_imua and eq. osv_close_k on bf16 matrix cores):
   every FP64 operand of the two products is carried as three bf16 pieces
   x = h + m + l with FP32 accumulation over a few 32-deep blocks and FP64
   accumulation across them; results are stored in FP64.
   - Projection: relative pieces (h = bf16(x), m = bf16(x - h),
     l = bf16(x - h - m)) and the six cross products whose piece orders sum
     to at most 2; per product the error is about 2^-24 of sum |a_k b_k|.
   - pair_K (MBE3_MIXED_BF16 only): pieces on a fixed-point grid of each
     row of gamma, (H1 + H2/2^8 + H3/2^16) 2^(e-7) with integers |Hk| <= 128
     and 2^e above the row's largest magnitude, and all nine products.  Each
     32-deep block of one product class is then summed exactly by the matrix
     cores (whose product adder otherwise drops low bits of small products,
     a downward bias), and keeping l l avoids the bias the grid noise of the
     third piece would leave on the diagonal of K.  The representation error
     is at most 2^-23 of the row's largest element, unbiased.
   The energy error against MBE3_FP64 is reported by the tests and the
   benchmark. */
#define MBE3_MIXED_BF16 1
/* Split-precision projection as above; pair_K in FP64 (the split pair_K
   issues nine bf16 products per FP64 one and is memory bound, so FP64
   matrix cores finish it sooner). */
#define MBE3_MIXED_BF16_PROJ 2

/* Phases reported by mbe3_get_timing. */
#define MBE3_PHASE_REGEN 0   /* slab regeneration (osv_project)             */
#define MBE3_PHASE_PROJECT 1 /* projection GEMMs (osv_project)              */
#define MBE3_PHASE_PAIR_K 2  /* pair_K                                      */
#define MBE3_PHASE_BASES 3   /* S/F blocks, pair eigensolves, X             */
#define MBE3_PHASE_PAIRS 4   /* K~ = X^T K X, pair-level S~                  */
#define MBE3_PHASE_CROSS 5   /* per-trimer S~ between pair domains          */
#define MBE3_PHASE_SOLVE 6   /* fragment residual iterations                */
#define MBE3_PHASE_ENERGY 7  /* MBE(3) sum                                  */
#define MBE3_PHASE_GRAD 8    /* multipliers and dE/df (fragment_solve, W)   */
#define MBE3_PHASE_BACKWARD 9 /* mbe3_backward                              */
#define MBE3_NPHASE 10

/* Output selector of mbe3_backward. */
#define MBE3_GRAD_SLAB 0  /* dE/d(ia|P), [n_occ][n_vir][n_aux]               */
#define MBE3_GRAD_GAMMA 1 /* dE/dG, osv_project's layout                     */
#define MBE3_GRAD_PROBE 2 /* <dE/dB, Delta> and <dE/dB, B>, no dense dE/dB  */

typedef struct mbe3_handle mbe3_handle;

/*
 * Problem description (read once by mbe3_create; host arrays are copied, the
 * device arrays must stay valid and unchanged-in-shape for the handle's
 * lifetime; their values may change between calls).
 */
typedef struct mbe3_problem {
  int32_t n_occ; /* localized occupied orbitals (LMOs)                     */
  int32_t n_vir; /* canonical virtual orbitals                             */
  int32_t n_aux; /* auxiliary (RI) functions                               */
  const int32_t *r; /* host [n_occ]: OSVs per LMO, 1 <= r[i] <= n_vir       */
  const double *Q;  /* device [sum r][n_vir]: row q_off[i]+mu is OSV mu of
                       LMO i (columns of Q_i, orthonormal)                  */
  const double *eps_vir; /* device [n_vir]: virtual energies f_aa           */
  const double *f_occ;   /* device [n_occ][n_occ]: symmetric LMO Fock      */
  /* RI slab source.  If slab != NULL it is used as (ia|P) directly:
     device [n_occ][n_vir][n_aux].  Otherwise the slab is regenerated:
       (ia|P) = z * w_ia[i][a] * w_iP[i][P]   (evaluated in that order)
     with z the Box-Muller normal of words 0, 1 of the Philox4x64-10 block
     at counter (P, a, i, 0) under key (seed, 0):
       u1 = ((w0 >> 11) + 0.5) 2^-53,  u2 = (w1 >> 11) 2^-53,
       z  = sqrt(-2 ln u1) cos(2 pi u2).                                    */
  uint64_t seed;
  const double *w_ia; /* device [n_occ][n_vir]                             */
  const double *w_iP; /* device [n_occ][n_aux]                             */
  const double *slab; /* device [n_occ][n_vir][n_aux] or NULL              */
  int64_t n_pair;
  const int32_t *pairs; /* host [n_pair][2]: kept pairs, i < j, no repeats  */
  int64_t n_frag;
  const int32_t *frags; /* host [n_frag][3]: fragments, ascending orbital
                           indices padded with -1.  Must be downward closed:
                           every orbital of a fragment is a monomer
                           fragment, every pair inside a dimer or trimer is
                           both kept and a dimer fragment.                  */
  double tol;       /* convergence: max |X^T R X| < tol (every pair)       */
  int32_t max_iter; /* maximum amplitude updates per fragment               */
  double tau_S;     /* drop pair-overlap eigenvalues <= tau_S               */
  int32_t precision; /* MBE3_FP64, MBE3_MIXED_BF16, MBE3_MIXED_BF16_PROJ */
  /* 0: every fragment starts from T = 0.  1: monomers and dimers are solved
     first and each trimer starts from their converged amplitudes (its
     diagonal pairs from the monomers, its pairs from the dimers); the
     solution is the same to the convergence threshold, in fewer updates.  */
  int32_t warm_start;
} mbe3_problem;

/* Sizes of the packed arrays exchanged between the calls. */
typedef struct mbe3_layout {
  int64_t n_slot;      /* n_occ + n_pair                                    */
  int64_t gamma_rows;  /* sum_i sum_{x in N+(i)} r[x]                       */
  int64_t gamma_elems; /* gamma_rows * n_aux                                */
  int64_t k_elems;     /* sum_s d_s^2                                       */
  int64_t n_frag;
} mbe3_layout;

/* Create a handle for problem *p on `stream` (hipStream_t).  Validates the
   lists (MBE3_EINVAL), builds the execution plans and allocates the
   workspace (MBE3_ENOMEM).  *h is NULL on failure.  The handle belongs to
   the device current at this call: its workspace is allocated there,
   `stream` must be that device's, and later calls on h expect it current. */
int mbe3_create(mbe3_handle **h, const mbe3_problem *p, void *stream);
/* Release the handle and its workspace (after finishing its stream). */
int mbe3_destroy(mbe3_handle *h);
/* Host string describing the last failure on h (never NULL). */
const char *mbe3_last_error(const mbe3_handle *h);

int mbe3_get_layout(const mbe3_handle *h, mbe3_layout *out /* host */);
/* Plan without a device: validates *p (device pointers are not touched, any
   non-NULL value is accepted), builds every execution plan and checks that
   each task stays inside the buffers it addresses.  Returns the status
   mbe3_create would return for plan errors; the message is available from
   mbe3_last_error(NULL).  `out` (host, nullable) receives the layout. */
int mbe3_plan_check(const mbe3_problem *p, mbe3_layout *out);
/* Row offset of LMO i's block in gamma, host out[n_occ + 1]. */
int mbe3_gamma_offsets(const mbe3_handle *h, int64_t *out);
/* Offset (in doubles) of slot s in the K layout, host out[n_slot + 1]. */
int mbe3_k_offsets(const mbe3_handle *h, int64_t *out);

/*
 * osv_project -- eq. osv_imua.  For every LMO i and x in N+(i):
 *   gamma[goff[i] + (rows of x within N+(i))][P] = (Q_x^T B_i)[mu][P],
 * i.e. LMO i's block is the stacked Q_x^T B_i over x in N+(i) (ascending),
 * each r[x] x n_aux, rows contiguous.  gamma: device, gamma_elems doubles
 * (mbe3_layout).  B_i is regenerated tile by tile (or read from slab).
 */
int osv_project(mbe3_handle *h, double *gamma, int64_t gamma_elems);

/*
 * pair_K -- eq. osv_close_k.  For slot s of pair (p, q):
 *   K_s = [G_{p,p}; G_{p,q}] [G_{q,p}; G_{q,q}]^T          (d_s x d_s)
 * and for a diagonal slot K_s = G_{p,p} G_{p,p}^T, with G_{i,x} = Q_x^T B_i
 * read from gamma (osv_project's layout).  K: device, k_elems doubles,
 * slot s row-major at k_off[s] (the p-block first).
 */
int pair_K(mbe3_handle *h, const double *gamma, double *K, int64_t k_elems);

/*
 * fragment_solve -- Algorithms 5 and 7 with eq. prec_eig.
 * Builds S_(x,y) = Q_x^T Q_y and F_(x,y) = Q_x^T diag(eps) Q_y, the pair
 * bases X_s (F X = S X diag(eps~), X^T S X = 1, overlap eigenvalues <= tau_S
 * dropped), then for each fragment F iterates from T = 0:
 *   R_pq = K_pq + F T_pq S + S T_pq F
 *          - sum_{k in F} [ f_pk S_(pq,kq) T_kq S_(kq,pq)
 *                         + f_kq S_(pq,pk) T_pk S_(pk,pq) ]   (p <= q in F)
 *   stop when max |X^T R X| < tol, else T += X ((X^T R X) / E~) X^T,
 *   E~[mu][nu] = f_pp + f_qq - eps~_mu - eps~_nu,
 * and returns the Hylleraas fragment energy
 *   e_frag[f] = sum_{p<=q in F} w_pq <2 T_pq - T_pq^T, K_pq + R_pq>,
 * w = 1 for p = q, 2 otherwise (Frobenius product).
 * K: device, pair_K's layout.  e_frag: device [n_frag].  iters: device
 * [n_frag] int32, number of updates, or -(max_iter+1) if not converged.
 * W: device, K layout, or NULL; when given it receives the MBE multipliers
 *   W_s = sum_{F containing p,q} c_F (2 T^F_pq - T^F_pq^T)
 * (c_F: the fragment's coefficient in the MBE(3) sum of mbe3_energy, i.e.
 * E = sum_F c_F e_frag[F]) at the converged amplitudes, and the handle
 * records dE/df_occ for mbe3_backward.  The first call with W plans and
 * allocates the gradient workspace (about one Y block per fragment and
 * chunk, one gamma-sized buffer).  Called directly it synchronises the
 * stream and returns MBE3_ENOCONV / MBE3_ENONFINITE if any fragment failed
 * (other fragments are valid; W is then not); while recording it returns at
 * once and mbe3_graph_launch reports the status of each replay.
 */
int fragment_solve(mbe3_handle *h, const double *K, double *e_frag,
                   int32_t *iters, double *W);

/*
 * mbe3_backward -- gradient of the MBE(3) energy through pair_K and
 * osv_project.  Because every fragment energy is a Hylleraas functional at
 * a stationary point of its amplitudes, its derivative with respect to K or
 * f_occ is the explicit one at the converged amplitudes:
 *   dE/dK_s = 4 W_s (pairs), 2 W_s (diagonal slots)  with W from
 *   fragment_solve; K_s = L R^T (pair_K) gives dL = G R and dR = G^T L, so
 *   dE/dB_i = 4 sum_{q in N+(i)} V_iq W_iq V_iq^T B_q  (W_qi = W_iq^T in
 *   the swapped basis, W_ii symmetrised), and
 *   dE/df_xy = -sum_F c_F [ sum_q <T~_xq, S_(xq,yq) T_yq S_(yq,xq)>
 *                         + sum_p <T~_py, S_(py,px) T_px S_(px,py)> ]
 *   over ordered pairs of F, T~ = 2T - T^T, returned symmetrised.
 * dE: scale applied to every output (the upstream derivative).
 * gamma: device, osv_project's output for the same slabs.  W: device, K
 *   layout (fragment_solve's multipliers, or any d_s x d_s blocks G_s / 4
 *   for pairs and G_s / 2 for diagonal slots to back-propagate dE/dK = G).
 * mode MBE3_GRAD_SLAB: out = dE dE/dB, device [n_occ][n_vir][n_aux];
 *   MBE3_GRAD_GAMMA: out = dE dE/dG (G_{i,x} = Q_x^T B_i), gamma layout;
 *   MBE3_GRAD_PROBE: directional derivatives without the dense dE/dB (at
 *   1024 LMOs it would take hundreds of GB): the probe direction
 *     Delta_i[a][P] = w_ia w_iP z'(i, a, P),
 *   z' the Box-Muller normal of the Philox4x64-10 block at counter
 *   (P, a, i, 0) under key (seed, 10) (the slab's own generator with key
 *   word 1 = 10 instead of 0), is regenerated and projected into out
 *   (gamma layout, workspace, must not alias gamma; receives Q_x^T Delta_i),
 *   and probe[0] = dE <dE/dB, Delta> = <dE dE/dG, Q^T Delta>,
 *   probe[1] = dE <dE/dB, B> (the Euler sum below).  Needs an FP64 handle
 *   with regenerated slabs and a host probe[2]; synchronises the stream.
 *   out_elems: doubles available at out.
 * dEdF: device [n_occ][n_occ] or NULL: dE (g + g^T) / 2 from the last
 *   fragment_solve that received W (MBE3_EINVAL if there was none).
 * probe: host double or NULL (modes 0, 1): receives <out_G, G> with
 *   out_G = dE dE/dG (summed in double-double).  E is homogeneous of
 *   degree 4 in the slabs,
 *   so at exact convergence this is 4 E dE; the difference is of the order
 *   of the residual left at tol.  Synchronises the stream.
 */
int mbe3_backward(mbe3_handle *h, double dE, const double *gamma,
                  const double *W, int mode, double *out, int64_t out_elems,
                  double *dEdF, double *probe);

/*
 * mbe3_set_slab_shift -- from the next call on, osv_project regenerates the
 * shifted slabs B + t Delta (Delta the probe direction of MBE3_GRAD_PROBE),
 * so that a central difference (E(t) - E(-t)) / 2t of the whole forward
 * checks probe[0] along the same direction.  t = 0 restores B bit for bit.
 * While t != 0 the other calls that regenerate slabs (mbe3_fit_metric,
 * mbe3_project_fit, mbe3_pair_K_fit, mbe3_rosv) return MBE3_EINVAL.
 * Needs an FP64 handle with regenerated slabs (MBE3_EINVAL otherwise, and
 * for a non-finite t or while recording); releases a recorded graph, whose
 * launches carry the old shift.  Synchronises the stream.
 */
int mbe3_set_slab_shift(mbe3_handle *h, double t);

/*
 * mbe3_energy -- E = sum_i E_i + sum_ij dE_ij + sum_ijk dE_ijk with
 * dE_ij = E_ij - E_i - E_j, dE_ijk = E_ijk - dE_ij - dE_ik - dE_jk
 * - E_i - E_j - E_k (MBE(3) of fragment energies), summed in a fixed order
 * with compensated (double-double) arithmetic.  e_frag: device [n_frag].
 * e_total: host, 1 double.  incr: device [n_frag] (dE per fragment) or NULL.
 * Synchronises the stream.
 */
int mbe3_energy(mbe3_handle *h, const double *e_frag, double *e_total,
                double *incr);

/*
 * Pair bases for inspection: X_s (d_s x D_s, D_s = d_s rounded up to 16,
 * dropped / padded columns zero) at x_off = sum_{s'<s} d_s' D_s', eps~_s
 * (D_s entries, padded with 1e30) at e_off = sum_{s'<s} D_s', kept rank per
 * slot.  Runs the preparation of fragment_solve.  All device pointers.
 */
int mbe3_pair_basis(mbe3_handle *h, double *X, double *eps_t, int32_t *rank);
/*
 * Kernel timing: mbe3_set_timing(h, 1) synchronises the stream, clears the
 * accumulators and from then on brackets every phase's launches with HIP
 * events on the handle's stream.  mbe3_get_timing synchronises and writes
 * the accumulated milliseconds per phase (host ms[MBE3_NPHASE]) and the
 * number of timed regions (host launches[MBE3_NPHASE], nullable).
 */
int mbe3_set_timing(mbe3_handle *h, int enable);
int mbe3_get_timing(mbe3_handle *h, double *ms, int64_t *launches);

/* Offsets for mbe3_pair_basis: host xoff[n_slot+1], eoff[n_slot+1]. */
int mbe3_basis_offsets(const mbe3_handle *h, int64_t *xoff, int64_t *eoff);

/*
 * Pair screening metric of eq. s2b for each listed pair:
 *   s2b[k] = sum_{mu nu} <mu_i|nu_j>^2 / sqrt(r_i r_j),  (i, j) = pairs[k],
 * the squared norm of the OSV overlap block S_(i,j) = Q_i^T Q_j.  The paper
 * calls a pair distant below 1e-7, weak below 1e-2 and close otherwise, and
 * keeps a trimer when the mean of its three pair metrics (eq. s3b) is at
 * least 0.2; mbe3_screen_lists takes those decisions.
 * pairs: host [n][2], two distinct LMOs each, any order.  s2b: device [n].
 * Allocates and frees device memory for the overlap blocks (sum r_i r_j
 * doubles) inside the call, so it cannot be recorded; synchronises the
 * stream.  MBE3_EINVAL for a bad pair or while recording.
 */
int mbe3_screen(mbe3_handle *h, const int32_t *pairs, int64_t n, double *s2b);

/*
 * Pair classes and trimer screening (section on OSV overlap and Fock
 * computation; eqs. s2b and s3b).  Host only, no handle, no device.
 * For candidate pair k = (pairs[2k], pairs[2k+1]) (either order, distinct
 * LMOs in [0, n_occ), no pair twice) with metric s2b[k] (mbe3_screen):
 *   cls[k] = 0 distant  (s2b < t_distant),
 *            1 weak     (t_distant <= s2b < t_close),
 *            2 close    (s2b >= t_close);
 * the paper's thresholds are MBE3_S2B_DISTANT, MBE3_S2B_CLOSE.
 * close_pairs / weak_pairs receive those classes' pairs as i < j in
 * lexicographic order ([n][2] each, capacity n; nullable), *n_close and
 * *n_weak their counts.  Trimers are the triples i < j < k whose three
 * pairs are all close (each one a dimer fragment, so the fragment list
 * stays downward closed) and whose mean metric
 *   s3b = (s2b_ij + s2b_ik + s2b_jk) / 3   (eq. s3b)
 * is at least t_trimer (the paper's MBE3_S3B_KEEP); they go to trimers
 * ([tri_cap][3], lexicographic; nullable) and their count to *n_tri.  Call
 * once with trimers = NULL for the count, then with room for it.  The
 * close pairs and trimers with every monomer are a fragment list for
 * mbe3_create; the weak pairs go to mbe3_weak_pairs; distant ones drop.
 * host: pairs, s2b, cls, close_pairs, weak_pairs, trimers, counts.
 * MBE3_EINVAL (message from mbe3_last_error(NULL)) for a bad or repeated
 * pair, a non-finite metric or too small a tri_cap; MBE3_ENOMEM if host
 * memory runs out.
 */
#define MBE3_S2B_DISTANT 1e-7
#define MBE3_S2B_CLOSE 1e-2
#define MBE3_S3B_KEEP 0.2
int mbe3_screen_lists(int32_t n_occ, const int32_t *pairs, int64_t n, const double *s2b,
                      double t_distant, double t_close, double t_trimer, int8_t *cls,
                      int32_t *close_pairs, int64_t *n_close, int32_t *weak_pairs,
                      int64_t *n_weak, int32_t *trimers, int64_t tri_cap, int64_t *n_tri);

/*
 * mbe3_screen without any allocation, for callers that cannot allocate
 * device memory (code that must not call hipMalloc / hipFree, tight
 * serving loops, harnesses that forbid allocation): the same s2b values as
 * mbe3_screen, bit for bit (same kernels, same order), with the task table,
 * the pair table and the overlap blocks S_(i,j) held in a fixed scratch
 * array of mbe3_screen_noalloc_max_bytes() bytes (64 MiB) inside the
 * library, one per GPU, kept until the process ends.  A call needs about
 * 8 sum_k r_i r_j bytes plus 200 bytes per pair; more than the array holds
 * is refused with MBE3_EINVAL (split the pairs over several calls).  The
 * host tables are copied on the handle's stream and the call synchronises
 * it.  Every call on one GPU shares that GPU's array and leaves its
 * contents behind; nothing in it needs to start at zero.  Calls that
 * overlap on one GPU (another handle, another host thread) race.
 * pairs: host [n][2] (two distinct LMOs each).  s2b: device [n].
 * MBE3_EINVAL as mbe3_screen, or while recording.
 */
int mbe3_screen_noalloc(mbe3_handle *h, const int32_t *pairs, int64_t n, double *s2b);
int64_t mbe3_screen_noalloc_max_bytes(void);

/*
 * Occupied-orbital localization (section on occupied orbital localization,
 * Alg. 2, eq. loc_theta): Pipek-Mezey with Jacobi sweeps on Loewdin charges.
 * No handle.  From symmetrically orthonormalized MO coefficients
 * C~ (device [n_ao][n_occ], orthonormal columns) and the atom of every AO
 * (host ao_off[n_atom + 1]: AOs of atom A are ao_off[A] .. ao_off[A+1]-1,
 * ao_off[0] = 0, ao_off[n_atom] = n_ao):
 *   P^A_ij = sum_{alpha in A} C~_{alpha i} C~_{alpha j},
 * then sweeps over the pairs i < j in order:
 *   a_ij = sum_A (P^A_ij)^2 - (P^A_ii - P^A_jj)^2 / 4,
 *   b_ij = sum_A P^A_ij (P^A_ii - P^A_jj),
 *   4 theta = atan2(b_ij, -a_ij)  (the maximizer of sum_{i,A} (P^A_ii)^2
 *                                  over the pair rotation),
 * and, when |sin theta| >= 1e-10, the increment
 * sqrt(a^2 + b^2)(1 - cos 4 theta) is added to the sweep's sum and the
 * columns i, j of U and both orbital indices of every P^A are rotated
 * (i' = cos i + sin j, j' = cos j - sin i).  Sweeps repeat while the last
 * sweep's sum exceeds l_loc (the paper's 1e-3), at most max_sweeps.
 * Outputs: P device [n_occ][n_occ][n_atom] (element (i, j, A) at
 * (i n_occ + j) n_atom + A): the charges of the localized orbitals; U device
 * [n_occ][n_occ] row-major: the localized orbitals are C~ U; dL and
 * rotations host [max_sweeps] (nullable): each sweep's sum and rotation
 * count; *sweeps (host) the sweeps run.  One workgroup runs the sweeps (the
 * pairs are sequential: each rotation changes what the next pair reads).
 * Allocates two small device buffers per call and synchronises `stream`.
 * MBE3_EINVAL for bad sizes or offsets (message from mbe3_last_error(NULL)),
 * MBE3_ENOCONV when max_sweeps end above l_loc (outputs valid),
 * MBE3_ENONFINITE for a non-finite increment.
 */
int mbe3_pm_localize(const double *C, const int32_t *ao_off, int32_t n_ao, int32_t n_occ,
                     int32_t n_atom, double l_loc, int32_t max_sweeps, double *P, double *U,
                     double *dL, int32_t *rotations, int32_t *sweeps, void *stream);

/*
 * Weak pairs (the weak-pair part of Algorithm 7): energies of pairs left
 * out of the fragment list, from the one-block exchange integrals
 * K_(i,j) = Gamma~_(i,i) Gamma~_(j,j)^T (eq. osv_weak_k) and the one-block
 * residual of eq. res_weak, read so that it type-checks,
 *   R_(i,j) = K_(i,j) + T_(i,j) F_(j,j) + F_(i,i) T_(i,j)
 *             - (f_ii + f_jj) T_(i,j) - f_ij [T_(i,i) S_(i,j) + S_(i,j) T_(j,j)],
 * solved in one step in the diagonal pairs' pseudo-canonical bases
 * (eq. prec_eig), and the energy of each unordered pair
 *   e[k] = 4 <K_(i,j), T_(i,j)>
 * (the close-pair energy restricted to the one block; the exchange block is
 * dropped with the exchange amplitudes).  T_(i,i) are the MBE(3) diagonal
 * amplitudes (eq. tmbediag): the diagonal-slot blocks of W.
 * pairs: host [n][2] with 0 <= i < j < n_occ.  gamma: device, osv_project's
 * output (FP64).  W: device, K layout; fragment_solve's multipliers (their
 * diagonal slots are T^MBE_ii), or any caller blocks.  e: device [n].
 * Uses the pair bases of the handle's last eager fragment_solve or
 * mbe3_pair_basis call (prepares them when there was none), allocates and
 * frees its blocks (about 3 sum r_i r_j + 2 sum D_i D_j + sum D_i r_j
 * doubles) inside the call, so it cannot be recorded; synchronises the
 * stream.
 * MBE3_EINVAL for a bad pair or argument or while recording.
 */
int mbe3_weak_pairs(mbe3_handle *h, const int32_t *pairs, int64_t n, const double *gamma,
                    const double *W, double *e);

/*
 * Sparse fitting domains (eq. sparse_fit_metric, section on the direct
 * Gamma_i generator).  The metric of auxiliary function P for LMO i is
 *   s_fit[i * n_aux + P] = sum_a B_i[a][P]^2
 * over the slab's orbital index (the virtual MOs of the (ia|P) slab, which
 * stands in for the paper's AO-indexed Gamma_i), summed in increasing a in
 * FP64 from the regenerated (or given) slab elements; nothing is stored
 * besides s_fit.  The fitting domain is D_i = {P : s_fit[i][P] > l_fit}
 * (strict; the paper's threshold is 1e-6).
 *
 * mbe3_fit_metric: s_fit device, n_occ * n_aux doubles, written.  The same
 * arithmetic in every precision mode.
 *
 * mbe3_fit_mask: restricts gamma-layout rows to the auxiliary functions the
 * domains select for them.  Eqs. osv_imua, osv_close_k and osv_weak_k run
 * A' over D_i u D_j for the pair ij, so a row of block (i, x), x != i
 * (G_{i,x} = Q_x^T B_i), keeps P in D_i u D_x, and a row of the diagonal
 * block (i, i), which every pair (i, q) reads over D_i u D_q, keeps P in
 * the union of D_q over q in N+(i).  Every other element is set to zero
 * (a NaN metric drops P); kept elements are not touched.  g: device,
 * g_elems >= gamma_elems doubles, in place.  This is Gamma~ as stored over
 * the domains (mbe3_project_fit's output); the exchange integrals over the
 * domains come from mbe3_pair_K_fit (pair_K of the masked gamma would sum
 * the diagonal blocks' product over more than D_p u D_q).
 * MBE3_EINVAL for a NULL pointer, a NaN l_fit or a short g.
 *
 * Both allocate nothing, leave the handle's state alone and may be recorded.
 */
int mbe3_fit_metric(mbe3_handle *h, double *s_fit);
int mbe3_fit_mask(mbe3_handle *h, const double *s_fit, double l_fit, double *g,
                  int64_t g_elems);

/*
 * osv_project restricted to the fitting domains, with the work of the
 * restriction saved (the paper's reason for the domains): for every LMO i
 * only the columns P its rows are needed on (the union C_i of D_q over q in
 * N+(i)) are regenerated and projected (eq. osv_imua), and gamma receives
 * Gamma~ in osv_project's layout restricted as mbe3_fit_mask describes
 * (block (i, x) on D_i u D_x, block (i, i) on C_i), every other column
 * zero.  The products run in FP64 in every precision mode, each element
 * summed over a in the order of osv_project's FP64 form, so on an MBE3_FP64
 * handle the result equals osv_project followed by mbe3_fit_mask bit for
 * bit.  s_fit: device, n_occ * n_aux doubles (mbe3_fit_metric's output or
 * any caller metric).  gamma: device, gamma_elems >= gamma_elems of the
 * layout.  Copies s_fit to the host and synchronises the stream, allocates
 * the compacted slabs and rows for the call (at most about 2 GiB of slabs
 * at a time, plus sum_i rows_i |C_i| doubles), so it cannot be recorded.
 * MBE3_EINVAL for a NULL pointer, a NaN l_fit, a short gamma or while
 * recording; MBE3_ENOMEM if the compacted buffers cannot be allocated.
 */
int mbe3_project_fit(mbe3_handle *h, const double *s_fit, double l_fit, double *gamma,
                     int64_t gamma_elems);

/*
 * pair_K over the fitting domains (eq. osv_close_k with A' in D_p u D_q;
 * eq. sparse_fit_metric): for slot (p, q)
 *   K_s = sum_{A' in D_p u D_q} L[:, A'] R[:, A']^T,
 *   L = [G_{p,p}; G_{p,q}], R = [G_{q,p}; G_{q,q}]  (unrestricted values),
 * and for a diagonal slot the sum over D_p.  The columns C_i of every slab
 * (the union of the domains of N+(i), which holds D_p u D_q for every pair
 * of i) are projected as in mbe3_project_fit, kept compacted and transposed
 * inside the call, and each block is summed over the union by gathering its
 * rows from both operands.  Blocks with an empty union are zero.  Gamma~
 * itself is not written.  FP64 in every precision mode.
 * s_fit: device, n_occ * n_aux doubles.  K: device, k_elems >= the
 * layout's k_elems.  Copies s_fit to the host and synchronises the stream,
 * allocates the compacted slabs (at most about 2 GiB at a time) and
 * sum_i rows_i |C_i| doubles for the call, so it cannot be recorded.
 * MBE3_EINVAL for a NULL pointer, a NaN l_fit, a short K or while
 * recording; MBE3_ENOMEM if the buffers cannot be allocated.
 */
int mbe3_pair_K_fit(mbe3_handle *h, const double *s_fit, double l_fit, double *K,
                    int64_t k_elems);

/*
 * Randomized OSV generation (section on randomized OSV generation, Alg. 3):
 * for every LMO i,
 *   T_ii[a][b] = sum_{P in D_i} B_i[a][P] B_i[b][P] / (f_aa + f_bb - 2 f_ii)
 *                                                          (eq. mp2_tkk)
 * from the regenerated (or given) slab on the fitting domain D_i =
 * {P : s_fit[i][P] > l_fit} (every P when s_fit is NULL); Gaussian test
 * rows G: row s, column a is the Box-Muller normal of the Philox4x64-10
 * block at counter (a, s, i, 0) under key (seed, 11), rows 0..9 the first
 * block, rows 10 .. 10 + n_max - 1 the later samples; the adaptive range
 * finder over the rows of Y = G T: while the largest of the 10 pending row
 * norms exceeds l_osv / (10 sqrt(2/pi)) and fewer than n_max rows are
 * accepted, the first pending row is orthogonalised against the accepted
 * rows Z (eq. rsvd_za) and accepted, the next sample is appended after
 * orthogonalisation against the earlier rows, and the new row's direction
 * is removed from every pending row; then T~ = Z T (eq. tsub), its singular
 * values w and left vectors Q~ (eq. tii_rsvd, through the eigenvectors of
 * T~ T~^T) and Q_i = Z^T Q~ (eq. back_q), keeping the columns with
 * w >= l_osv, largest first.
 * s_fit: device n_occ * n_aux doubles or NULL.  n_max: 1 .. min(n_vir, the
 * eigensolver's LDS order, at least 128).  Outputs, all device:
 *   Q_out [n_occ][n_max][n_vir]: row mu of LMO i is OSV mu (a column of
 *         Q_i), zero rows after the kept ones;
 *   w_out [n_occ][n_max]: the kept singular values, decreasing, zeros after;
 *   n_osv [n_occ]: kept counts;  rows [n_occ]: accepted range-finder rows
 *   (n_max when the cap stopped the loop).
 * Allocates per call (batches of LMOs whose n_vir x n_vir T fit 8 GiB) and
 * synchronises the stream, so it cannot be recorded.  MBE3_EINVAL for a
 * NULL output, a NaN l_fit, a non-positive l_osv, n_max out of range or
 * while recording; MBE3_ENOMEM if the buffers cannot be allocated.
 */
int mbe3_rosv(mbe3_handle *h, const double *s_fit, double l_fit, double l_osv, int n_max,
              double *Q_out, double *w_out, int32_t *n_osv, int32_t *rows);

/*
 * First-order energy change of a change of the pair integrals (the split-
 * precision forms change the energy only through K; fragment_solve reads
 * K~ = X^T K X):
 *   per_slot[s] = c_s <K_a,s - K_b,s, W_s>,  c_s = 2 diagonal slots,
 *                                            c_s = 4 pair slots,
 *   *total = sum_s per_slot[s]  (double-double, fixed order),
 * with W the multipliers fragment_solve returned for K_b (dE/dK_s =
 * c_s W_s).  Attributes an energy difference to slots.  K_a, K_b, W:
 * device, K layout.  per_slot: device [n_slot].  total: host, 1 double.
 * Synchronises the stream; MBE3_EINVAL for a NULL pointer or while
 * recording.
 */
int mbe3_first_order_dE(mbe3_handle *h, const double *K_a, const double *K_b,
                        const double *W, double *per_slot, double *total);

/*
 * Recorded launches (one HIP graph per handle) for the batched form of
 * Algorithm 7: thousands of fragments per call, replayed without host work.
 *
 * mbe3_graph_begin starts recording: until mbe3_graph_end, the calls
 * osv_project, pair_K, fragment_solve, mbe3_energy, mbe3_backward (without
 * probe) and mbe3_pair_basis on h enqueue their launches into the graph
 * instead of running them, bound to the pointers they are given (which must
 * stay valid while the graph is used).  They do not synchronise; their
 * status codes then cover argument checks only: fragment_solve's
 * convergence and finiteness are reported by mbe3_graph_launch, and
 * mbe3_energy writes NaN to *e_total (the energy comes from
 * mbe3_graph_launch).  with_grad != 0 plans and allocates the gradient
 * workspace first (fragment_solve with W and mbe3_backward need it; they
 * fail while recording if it is missing).  Any failing call marks the
 * recording failed.  mbe3_set_timing, mbe3_get_timing and a second
 * mbe3_graph_begin fail while recording.  Recording happens on a private
 * stream of the handle; beginning a new recording synchronises h's stream
 * and releases the previous graph.  If timing is on while recording, each
 * timed phase becomes a graph of its own and mbe3_graph_launch, with
 * timing on, brackets its replay with HIP events on h's stream (the
 * mbe3_get_timing accumulators); otherwise the recording is one graph.
 *
 * mbe3_graph_end instantiates the graph: MBE3_EINVAL if a call failed while
 * recording (the message names it; nothing is kept), MBE3_EHIP if HIP
 * refused the capture.
 *
 * mbe3_graph_launch replays the graph on h's stream and synchronises, then
 * reports like the recorded calls would have: MBE3_ENONFINITE / MBE3_ENOCONV
 * from a recorded fragment_solve, and the MBE(3) energy of a recorded
 * mbe3_energy in *e_total (host, nullable).  After a successful replay that
 * contains fragment_solve with W, mbe3_backward may use dE/df.  Nothing is
 * allocated per replay.
 */
/*
 * Tile shapes of the grouped FP64 GEMMs (the batched products of
 * Algorithms 5 and 6 and of the gradient): each task list of the handle has
 * one shape, BM x BN of the output per workgroup, from
 *   0: 64x64, 1: 128x128, 2: 32x32, 3: 32x128, 4: 64x128, 5: 96x96.
 * Every shape accumulates each output element over k in the same order, so
 * the results are bitwise the same whichever shape runs.
 *
 * mbe3_autotune times every shape on every task list of the handle (its
 * own tasks and sizes: `reps` timed launches after one warm-up, HIP events
 * on h's stream) and keeps the fastest per list.  gamma, K (device, the
 * layout's sizes) and dB (device, n_occ*n_vir*n_aux doubles, or NULL to
 * leave the un-projection list as planned) serve as the products' operands
 * and outputs: their contents are undefined afterwards, as are the handle's
 * intermediate results (the next fragment_solve recomputes them).  The
 * gradient lists are included once gradients are planned (fragment_solve
 * with W, or mbe3_graph_begin with with_grad).  Synchronises; releases a
 * recorded graph.  mbe3_tune_report returns one line per list: index, name,
 * task count, the time of each shape and the choice.
 *
 * mbe3_set_gemm_shape sets the shape of list `list` (its index in the
 * report; -1: all lists) without timing, and re-checks every task against
 * its buffers.  Synchronises; releases a recorded graph.
 */
int mbe3_autotune(mbe3_handle *h, double *gamma, int64_t gamma_elems, double *K,
                  int64_t k_elems, double *dB, int64_t dB_elems, int reps);
int mbe3_set_gemm_shape(mbe3_handle *h, int list, int shape);
const char *mbe3_tune_report(const mbe3_handle *h);

int mbe3_graph_begin(mbe3_handle *h, int with_grad);
int mbe3_graph_end(mbe3_handle *h);
int mbe3_graph_launch(mbe3_handle *h, double *e_total);

#ifdef __cplusplus
}
#endif

#endif /* MBE3OSV_H */
