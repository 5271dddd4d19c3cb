// Internal declarations shared by the HIP translation units of libmbe3osv.
// Each .hip file owns its kernels and exposes host launchers declared here.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace mbe3 {

// ---------------------------------------------------------------------------
// Grouped FP64 GEMM engine (gemm.hip)
//   C = alpha * op(A) op(B) + beta * C   for every task of a list, one
//   workgroup per BM x BN output tile.  Operands are addressed relative to a
//   small table of base pointers so that plans built once at create time can
//   be replayed on caller buffers.
// ---------------------------------------------------------------------------
enum { NBASE = 32 };
struct GemmBases {
  double *p[NBASE];
  const int32_t *rows;  // row-gather indices (see a_rows / b_rows)
};

struct GemmTask {
  int64_t a_off, b_off, c_off;  // element offsets into bases.p[*_buf]
  int64_t tile_begin;           // first tile of this task (prefix sum)
  int32_t a_buf, b_buf, c_buf;
  int32_t a_rows;  // >= 0: stored row r of A is physical row rows[a_rows + r]
                   // (r = m for transA = 0, r = k for transA = 1); -1: identity
  int32_t b_rows;  // >= 0: stored row r of B is physical row rows[b_rows + r]
                   // (r = k for transB = 0, r = n for transB = 1); -1: identity
  int32_t M, N, K, lda, ldb, ldc;
  int32_t transA, transB;
  int32_t tiles_n;
  int32_t ldct;    // leading dimension of the transposed copy
  int64_t ct_off;  // >= 0: C^T is also stored at this offset of c_buf
  double alpha, beta;
};

// Tile shape ids for launch_gemm_tasks (BM x BN of C per workgroup).  Every
// shape accumulates each output over k in the same order, so the results do
// not depend on the shape.
enum GemmShape {
  GEMM_64x64 = 0,
  GEMM_128x128 = 1,
  GEMM_32x32 = 2,
  GEMM_32x128 = 3,
  GEMM_64x128 = 4,
  GEMM_96x96 = 5,
  GEMM_NSHAPE = 6
};
int gemm_tile_m(GemmShape shape);
int gemm_tile_n(GemmShape shape);
const char *gemm_shape_name(GemmShape shape);
int64_t gemm_tile_count(const GemmTask &t, GemmShape shape);
hipError_t launch_gemm_tasks(const GemmTask *d_tasks, int n_tasks,
                             int64_t n_tiles, const GemmBases &bases,
                             GemmShape shape, hipStream_t s);

// ---------------------------------------------------------------------------
// Slab regeneration (regen.hip)
// ---------------------------------------------------------------------------
// Philox key word 1 of the gradient probe direction Delta (key word 1 of the
// slab itself is 0).
constexpr uint64_t PROBE_STREAM = 10;
// out[b][a][P] = w_ia w_iP (cb z_0 + cd z_10) for i = i0 + b: the slab
// (cb = 1, cd = 0), the probe direction (0, 1) or B + t Delta (1, t).
hipError_t launch_regen_slab(double *out, int i0, int nb, int n_vir, int n_aux,
                             uint64_t seed, const double *w_ia,
                             const double *w_iP, double cb, double cd, hipStream_t s);

// Sparse fitting metric s_fit[i][P] = sum_a B_i[a][P]^2 of the regenerated
// (slab == nullptr) or given slabs, and the restriction of gamma-layout rows
// to the columns the domains D_q = {P : s_fit[q][P] > l_fit} select for
// them: a row of block (i, x), x != i (LMO in row_lmo, block in row_x),
// keeps D_i u D_x; a row of block (i, i) keeps the union of D_q over q in
// N+(i) (CSR nbr_off / nbr) (regen.hip).
hipError_t launch_fit_metric(double *s_fit, int n_occ, int n_vir, int n_aux,
                             uint64_t seed, const double *w_ia, const double *w_iP,
                             const double *slab, hipStream_t s);
hipError_t launch_fit_mask(double *g, int64_t rows, int n_aux, const int32_t *row_lmo,
                           const int32_t *row_x, const int32_t *nbr_off,
                           const int32_t *nbr, const double *s_fit, double l_fit,
                           hipStream_t s);
// Projection over the fitting domains only: the kept columns of a batch of
// slabs compacted (LMO i's columns cols[col_off[i]..col_off[i+1]), batch
// member b at out_off[b]), and compacted gamma rows scattered back into the
// dense layout (regen.hip).
hipError_t launch_regen_cols(double *out, const int64_t *out_off, const int32_t *cols,
                             const int32_t *col_off, int i0, int nb, int64_t max_elems,
                             int n_vir, int n_aux, uint64_t seed, const double *w_ia,
                             const double *w_iP, const double *slab, hipStream_t s);
hipError_t launch_fit_scatter(double *g, const double *gc, int64_t rows, int n_aux,
                              int max_nc, const int32_t *row_lmo, const int64_t *g_off,
                              const int64_t *gc_off, const int32_t *cols,
                              const int32_t *col_off, hipStream_t s);

// Randomized OSV generation: Gaussian test rows (regen.hip, Philox key
// (seed, stream), counter (a, s, i, 0)); the Cauchy scaling of T_ii, the
// range finder and the final selection (rosv.hip).
hipError_t launch_regen_gauss(double *out, int i0, int nb, int n_rows, int n_vir,
                              uint64_t seed, uint64_t stream, hipStream_t s);
hipError_t launch_rosv_tscale(double *T, int i0, int nb, int n_vir, const double *eps,
                              const double *f, int n_occ, hipStream_t s);
hipError_t launch_range_finder(double *Y, double *Z, int32_t *rows, int nb, int r, int n_max,
                               int n_vir, double thr, hipStream_t s);
hipError_t launch_rosv_finalize(const double *evals, int D, const double *Qr,
                                const int32_t *rows, int i0, int nb, int n_max, int n_vir,
                                double l_osv, double *Q_out, double *w_out, int32_t *n_osv,
                                int32_t *rows_out, hipStream_t s);

// Pipek-Mezey localization (loc.hip): Loewdin charges P[(i n + j) na + A]
// from orthonormalized MO coefficients C [n_ao][n] with the AOs of atom A at
// ao_off[A] .. ao_off[A+1]-1 (device), and the Jacobi sweeps of one
// workgroup (rec: 2 doubles per sweep, then the sweep count).
hipError_t launch_pm_charges(const double *C, const int32_t *ao_off, int n, int na, double *P,
                             hipStream_t s);
hipError_t launch_pm_jacobi(double *P, double *U, int n, int na, double l_loc, int max_sweeps,
                            double *rec, hipStream_t s);

// Split-precision operands (regen.hip): three bf16 planes (bit patterns),
// plane stride ps elements, rows padded with zeros to ldk (a multiple of 8).
hipError_t launch_regen_split(uint16_t *planes, int64_t ps, int i0, int nb,
                              int n_vir, int n_aux, int ldk, uint64_t seed,
                              const double *w_ia, const double *w_iP,
                              const double *slab, hipStream_t s);
hipError_t launch_split_rows(const double *x, int64_t rows, int cols, int64_t ld,
                             uint16_t *planes, int64_t ps, int ldk,
                             hipStream_t s);
// The same planes with the leading piece on a fixed-point grid of each row
// (the pair_K operands: exact leading block sums on the matrix cores).
hipError_t launch_split_rows_fixed(const double *x, int64_t rows, int cols, int64_t ld,
                                   uint16_t *planes, int64_t ps, int ldk, hipStream_t s);

// ---------------------------------------------------------------------------
// Split-precision grouped GEMM (gemm_mixed.hip): C = A B^T in FP64 storage
// from three-piece bf16 operands, six cross products (pieces p + q <= 2) on
// v_mfma_f32_16x16x32_bf16 with FP32 accumulation.  A rows and B rows are
// K-contiguous (row pitch lda / ldb, multiples of 8), optionally gathered.
// ---------------------------------------------------------------------------
struct MixedTask {
  int64_t a_off, b_off, c_off;  // element offsets (A/B in plane 0, C)
  int64_t tile_begin;
  int32_t a_rows, b_rows;       // gather offsets into the row table, or -1
  int32_t M, N, K, lda, ldb, ldc;
  int32_t tiles_n, pad_;
};
enum MixedShape { MIXED_32x64 = 0, MIXED_64x128 = 1 };
int64_t mixed_tile_count(const MixedTask &t, MixedShape shape);
int mixed_tile_m(MixedShape shape);
int mixed_tile_n(MixedShape shape);
hipError_t launch_gemm_mixed(const MixedTask *d_tasks, int n_tasks,
                             int64_t n_tiles, const uint16_t *A, int64_t a_ps,
                             const uint16_t *B, int64_t b_ps, double *C,
                             const int32_t *rows, MixedShape shape,
                             hipStream_t s);

// ---------------------------------------------------------------------------
// Block assembly (prep.hip): out[r][c] for a matrix made of up to 2 x 2
// blocks of the S or F block store (or identity-free zero padding).
// ---------------------------------------------------------------------------
struct BlockSrc {
  int64_t off;   // offset of the source block (r_x x r_y row-major, ld = r_y)
  int32_t ld;    // leading dimension of the stored block
  int32_t trans; // 1: read the stored block transposed
};
struct AssembleTask {
  int64_t out_off;   // into the output base
  int32_t ld_out;    // output leading dimension
  int32_t nrb, ncb;  // number of row / column blocks (1 or 2)
  int32_t rsz[2], csz[2];  // block sizes
  int32_t rows_out, cols_out;  // total written region (>= sum of sizes:
                               // the remainder is zero-filled)
  int32_t src_buf;   // 0: S store, 1: F store
  int32_t out_buf;   // 0: out0, 1: out1
  BlockSrc b[2][2];
};
hipError_t launch_assemble(const AssembleTask *d_tasks, int n_tasks,
                           const double *sstore, const double *fstore,
                           double *out0, double *out1, hipStream_t s);
hipError_t launch_scale_rows(double *out, const double *Q, const double *eps,
                             int64_t rows, int n_vir, hipStream_t s);

// ---------------------------------------------------------------------------
// Batched symmetric Jacobi eigensolver (eigen.hip)
// ---------------------------------------------------------------------------
struct EigTask {
  int64_t a_off;    // input matrix (n x n, lda) in the input base
  int64_t o_off;    // output vectors (n_out x D, ld D) in the output base
  int64_t e_off;    // eigenvalues (D) in the eigenvalue base
  int32_t n;        // matrix order (mode 0); for mode 1 read from rank[slot]
  int32_t lda;
  int32_t D;        // padded column count of the outputs
  int32_t slot;     // slot id (rank array index)
  int64_t w_off;    // split Fock step: the task's record in the chase
                    // workspace (eig_chase_ws_doubles(D) doubles), or -1
};
// mode 0: overlap step.  Writes X0 = U_keep s^-1/2 (kept eigenvalues > tau,
//         ascending), zero columns up to D, rank[slot] = kept count;
//         eigenvalue array receives the kept eigenvalues (sentinel after).
// mode 1: Fock step.  Order = rank[slot].  Writes Z (D x D: eigenvectors in
//         the leading rank x rank block, zero elsewhere) and eps~ ascending
//         (sentinel 1e30 beyond rank).
// Tasks of order above eig_qr_max_order() run on a global workspace of
// gws_doubles (>= eig_workspace_doubles(max_n); one slice per workgroup).
// Orders up to eig_qr_max_order() by Householder reduction and implicit QR
// steps, one wave per matrix in LDS; larger orders by cyclic Jacobi.
hipError_t launch_eigh(const EigTask *d_tasks, int n_tasks, int max_n,
                       const double *in, double *out, double *evals, int32_t *rank,
                       int mode, double tau, const int32_t *only_flagged, double *gws,
                       int64_t gws_doubles, hipStream_t s);
int eig_qr_max_order();
// Split Fock step (mode 1 only) for orders up to eig_split_max_order():
// Householder reduction and Q per wave in LDS, then the implicit QR steps
// on (d, e) alone with every sweep's bounds and rotations recorded in the
// task's workspace record (ws + w_off, eig_chase_ws_doubles(D) doubles),
// then the rotations replayed onto Q and the outputs of launch_eigh's
// mode 1.  meta: device [n_tasks][4] int32 scratch; redo: device [n_slot]
// int32, set for tasks whose record overflowed (they are then solved by the
// fused kernel in the same call).  Larger orders as in launch_eigh.
int eig_split_max_order();
int64_t eig_chase_ws_doubles(int D);
hipError_t launch_eigh_split(const EigTask *d_tasks, int n_tasks, int max_n,
                             const double *in, double *out, double *evals,
                             int32_t *rank, double *cws, int32_t *meta, int32_t *redo,
                             double *gws, int64_t gws_doubles, hipStream_t s);
// Overlap step by Cholesky (X0 = L^-T, full rank).  Slots whose pivots drop
// to <= tau get flag[slot] = 1 and are redone by launch_eigh(mode 0,
// only_flagged = flag).
hipError_t launch_cholesky(const EigTask *d_tasks, int n_tasks, int max_n,
                           const double *in, double *out, double *evals,
                           int32_t *rank, int32_t *flag, double tau, double *gws,
                           int64_t gws_doubles, hipStream_t s);
int64_t eig_workspace_doubles(int max_n);
int eig_lds_max_order();

// ---------------------------------------------------------------------------
// Fragment solver (solve.hip)
// ---------------------------------------------------------------------------
struct SlotInfo {
  int32_t p, q;      // orbitals (p == q for diagonal slots)
  int32_t d, D;      // pair-domain dimension and padded X-basis dimension
  int64_t kt_off;    // K~ = X^T K X (D x D) in the K~ store
  int64_t et_off;    // eps~ (D) in the eps~ store
};
struct FragDesc {
  int32_t nt;           // number of pair slots (1, 3 or 6)
  int32_t frag;         // fragment index in the caller's list
  int32_t term_begin, term_end;
  int32_t slot[6];      // global slot ids, order: diagonals then pairs
  int32_t ysub[6];      // offset of each slot's D x D block in Y scratch
  int32_t sym[6];       // 1 for diagonal slots (residual symmetrised)
  int32_t wgt[6];       // energy weight 1 (diagonal) or 2 (pair)
  int32_t ny;           // sum of D^2 over the fragment's slots
  int32_t warm_in;      // 1: start every slot from the warm store, else T = 0
  int32_t warm_out;     // local slot whose converged Y goes to the warm store
                        // (the fragment's own pair: monomer 0, dimer 2), or -1
  int32_t pad_;
  double coef;          // MBE(3) coefficient c_F
  int64_t yout;         // offset of the converged Y blocks in the chunk store
};
struct Term {
  int32_t target, src;  // local slot indices within the fragment
  int32_t fx, fy;       // coefficient f_occ[fx][fy]
  int32_t trans;        // use Y_src^T
  int32_t st_buf;       // 0: pair-level S~ store, 1: per-chunk cross store
  int64_t st_off;       // row-major S~_(src,target)  (D_src x D_target)
};
// Most terms of one fragment: a trimer has two per diagonal target and four
// per pair target (the solver stages them in LDS).
constexpr int MAX_FRAG_TERMS = 18;
struct SolveArgs {
  const FragDesc *frags;
  const Term *terms;
  const SlotInfo *slots;
  const double *kt;      // K~ store
  const double *et;      // eps~ store
  const double *f_occ;
  const double *st0;     // pair-level S~ store
  const double *st1;     // cross S~ store of this chunk
  double *scratch;       // per-workgroup scratch
  int64_t scratch_stride;  // doubles per workgroup
  int32_t n_frag;        // fragments in this chunk
  int32_t n_occ;
  int32_t max_iter;
  int32_t dmax;          // largest D in the chunk
  double tol;
  double *e_frag;
  int32_t *iters;
  int32_t *status;       // [2 * workgroup]: non-finite seen, non-converged seen
  double *warm;          // converged Y per slot (K~ layout), or null
  // gradient mode (all null otherwise): Y~ = 2Y - Y^T of the converged
  // blocks per fragment (at FragDesc::yout; the LDS-resident solver stores Y
  // there and its gradient pass turns it into Y~), per-term contractions
  // <Y~_t, S~ Y_s^(T) S~^T> (<Y_t + Y_t^T, .> for diagonal targets) indexed
  // by term, and per-target <Y~_t, Y_t> at 6 * fragment + target.
  double *yfin;
  double *gterm;
  double *gdiag;
};
hipError_t launch_solve(const SolveArgs &a, int n_wg, hipStream_t s);
// The gradient pass over a chunk that launch_solve solved with yfin set (the
// same arguments and grid): per-term contractions, <Y~_t, Y_t>, and Y~ into
// the store.
hipError_t launch_solve_grad(const SolveArgs &a, int n_wg, hipStream_t s);
// Variant for 96 < dmax <= 160 (solve_wide.hip): one wave per 16-row block,
// panels streamed for both products, per-workgroup term sums in the scratch
// (which must hold 4 ny + 2 dmax^2 doubles, as solve_scratch_doubles gives).
hipError_t launch_solve_wide(const SolveArgs &a, int n_wg, hipStream_t s);
size_t solve_wide_lds_bytes(int dmax);
constexpr int SOLVE_LDS_DMAX = 128;  // largest dmax of the LDS-resident solver
// Resident workgroups per CU of the solver instance a chunk with a.dmax
// runs (mode 0 solve, 1 solve and store, 2 gradient pass).
hipError_t solve_blocks_per_cu(const SolveArgs &a, int mode, int *per_cu);
int64_t solve_scratch_doubles(int ny_max, int dmax);
size_t solve_lds_bytes(int dmax);

// ---------------------------------------------------------------------------
// Backward (backward.hip)
// ---------------------------------------------------------------------------
// W~ of one slot (D x D at wt_off) += sum of its entries [e_begin, e_end).
// One work item of the W~ reduction: elements [y0, y0 + n) of a slot's
// D x D block, summed over the entries [e_begin, e_end) (a slot in many
// fragments is split over several items by element range).
struct WSlot {
  int64_t wt_off;  // W~ offset of element y0
  int32_t n, e_begin, e_end, y0;
};
struct WEntry {
  int64_t yoff;  // converged Y~ = 2Y - Y^T block (D x D) in the chunk's store
  double coef;   // c_F
};
hipError_t launch_wtilde(const WSlot *slots, int n_slots, const WEntry *ents,
                         const double *yfin, double *wt, hipStream_t s);
// g[dst] += sum of scale * (kind ? gdiag[idx] : gterm[idx]) over the entries
// (one wave per destination, lane-strided partial sums, fixed shuffle tree).
struct GDest {
  int32_t dst, e_begin, e_end, pad_;
};
struct GEntry {
  double scale;
  int32_t kind, idx;
};
hipError_t launch_fgrad(const GDest *dests, int n, const GEntry *ents,
                        const double *gterm, const double *gdiag, double *g,
                        hipStream_t s);
// One segment of the concatenated multiplier block of a dGamma destination:
// ga[ga_off + r * ga_ld + k0 + k] = mult * scale * src(r, k), r < rows,
// k < kseg,
//   mode 0: W[rc0 + r][k], mode 1: W[k][rc0 + r], mode 2: W[r][k] + W[k][r]
// with W the d x d multiplier block at w_off (leading dimension w_ld).
struct GASeg {
  int64_t w_off, ga_off;
  int32_t w_ld, ga_ld, rc0, k0, rows, kseg, mode, pad_;
  double scale;
};
hipError_t launch_ga(const GASeg *segs, int n, const double *W, double mult,
                     double *ga, hipStream_t s);
// out[0] = scale * <x, y> in double-double arithmetic, fixed order; part
// holds 2 * dot_partials() doubles.
hipError_t launch_dot(const double *x, const double *y, int64_t n, double scale,
                      double *part, double *out, hipStream_t s);
int dot_partials();
// out = scale (g + g^T) / 2 for an n x n matrix.
hipError_t launch_fsym(const double *g, int n, double scale, double *out,
                       hipStream_t s);

// ---------------------------------------------------------------------------
// Reductions (reduce.hip)
// ---------------------------------------------------------------------------
hipError_t launch_mbe_sum(const double *e_frag, const double *coef, int64_t n,
                          double *out2, hipStream_t s);
// per_slot[s] = c_s <Ka_s - Kb_s, W_s> (c_s = 2 diagonal, 4 pair slots), one
// workgroup per slot, fixed-order sums (reduce.hip).  launch_mbe_sum with
// coef == nullptr sums its values with unit coefficients.
hipError_t launch_slot_dot(const double *Ka, const double *Kb, const double *W,
                           const int64_t *k_off, int n_occ, int64_t n_slot,
                           double *per_slot, hipStream_t s);
hipError_t launch_increments(const double *e_frag, const int32_t *sub,
                             int64_t n, double *incr, hipStream_t s);
hipError_t launch_fill(double *p, double v, int64_t n, hipStream_t s);

// ---------------------------------------------------------------------------
// Pair screening and weak pairs (weak.hip).  Per listed pair (i, j): its
// r_i x r_j blocks at k_off (S_(i,j), K_(i,j)), its D_i x D_j blocks at t_off
// (K~, D~) and the offsets of eps~ of the diagonal slots i and j.
// ---------------------------------------------------------------------------
struct WeakPair {
  int32_t i, j, ri, rj, Di, Dj;
  int64_t k_off, t_off, ei, ej;
};
hipError_t launch_s2b(const WeakPair *wp, int n, const double *S, double *out,
                      hipStream_t s);
hipError_t launch_weak_energy(const WeakPair *wp, int n, const double *Kt, const double *Dt,
                              const double *et, const int32_t *rank, const double *f,
                              int n_occ, double *e, hipStream_t s);
hipError_t launch_fill_i32(int32_t *p, int32_t v, int64_t n, hipStream_t s);

}  // namespace mbe3
