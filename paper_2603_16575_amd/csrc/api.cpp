// Host side of libmbe3osv: problem validation, execution plans (GEMM /
// assembly / eigen task tables and the fragment term tables, built once at
// create time and uploaded), workspace management and the C-ABI entry points
// declared in include/mbe3osv.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <iterator>
#include <map>
#include <mutex>
#include <new>
#include <string>
#include <unordered_map>
#include <vector>

#include "internal.hpp"
#include "mbe3osv.h"

using namespace mbe3;

namespace {

constexpr int DMAX_SUPPORTED = 160;  // largest padded pair dimension handled
constexpr int SOLVE_WG = 1024;       // persistent workgroups of the solver
constexpr int64_t SLAB_BUDGET = 2LL << 30;    // bytes of regenerated slabs
constexpr int64_t CHUNK_BUDGET = 12LL << 30;  // bytes of per-chunk stores

inline int round16(int x) { return (x + 15) & ~15; }
inline int64_t key2(int a, int b) { return ((int64_t)a << 32) | (uint32_t)b; }

// base-pointer ids of the GEMM engine
enum Base {
  B_Q = 0, B_EQ, B_SLAB, B_GAMMA, B_K, B_SS, B_FS, B_PS, B_PF, B_X0, B_X,
  B_TMP, B_FP, B_Z, B_KT, B_AT, B_MT, B_ST0, B_CA, B_CM, B_ST1,
  B_WT, B_W, B_GA, B_DG, B_DB,
  // call-time blocks of mbe3_screen / mbe3_weak_pairs
  B_PK, B_PS2, B_PM, B_PP, B_PKT, B_PDT, B_COUNT
};
static_assert(B_COUNT <= NBASE, "too many GEMM bases");

struct Chunk {
  std::vector<int> frag_ids;  // fragment indices (heavy first)
  // cross S~ GEMM lists (glists): outputs up to 64 wide, and wider
  int L_m = -1, L_mw = -1, L_s1 = -1, L_s1w = -1;
  AssembleTask *d_asm = nullptr;
  int n_asm = 0;
  FragDesc *d_frags = nullptr;
  int n_frag = 0;
  Term *d_terms = nullptr;
  int dmax = 16;
  int ny_max = 0;
  int64_t ny_total = 0;  // converged Y blocks of the chunk (gradient mode)
  int n_terms = 0;
  // gradient reductions of this chunk (planned on first use)
  WSlot *d_ws = nullptr;
  WEntry *d_we = nullptr;
  int n_ws = 0;
  GDest *d_gd = nullptr;
  GEntry *d_ge = nullptr;
  int n_gd = 0;
};

// One grouped-GEMM task list: its tasks (tile fields for `shape`), the
// device copy, and the row-gather table its tasks index (0: the plan's,
// 1: the gradient's).  The shape is the planner's default until
// mbe3_autotune measures the alternatives.
struct GemmList {
  std::string name;
  std::vector<GemmTask> host;
  GemmTask *d = nullptr;
  int64_t tiles = 0;
  GemmShape shape = GEMM_64x64;
  int rows_table = 0;
};

}  // namespace

struct mbe3_handle {
  // ---- problem ----
  int n_occ = 0, n_vir = 0, n_aux = 0;
  std::vector<int> r;
  std::vector<int64_t> q_off;
  const double *Q = nullptr, *eps = nullptr, *f = nullptr;
  const double *w_ia = nullptr, *w_iP = nullptr, *slab = nullptr;
  double slab_shift = 0.0;  // osv_project regenerates B + slab_shift * Delta
  uint64_t seed = 0;
  std::vector<std::array<int, 2>> pairs;
  std::vector<std::array<int, 3>> frags;
  double tol = 1e-8, tau_S = 1e-8;
  int max_iter = 100;
  int precision = MBE3_FP64;
  bool warm_start = false;
  double *warm = nullptr;  // converged Y of every slot's own fragment
  int ldk_vir = 0, ldk_aux = 0;  // padded row pitch of split planes
  hipStream_t stream = nullptr;
  std::string err;

  // ---- layout ----
  std::vector<std::vector<int>> nbr;
  std::vector<int64_t> g_off;
  std::unordered_map<int64_t, int64_t> grow;
  std::unordered_map<int64_t, int> pair_slot;
  int64_t n_slot = 0;
  std::vector<int> sp, sq, sd, sD;
  std::vector<int64_t> k_off, x_off, kt_off, et_off;
  std::unordered_map<int64_t, int64_t> sb_off;  // S/F block (x<=y) offsets
  int64_t sb_total = 0;
  int dmax = 16, dmin_max_pair = 0;
  std::vector<double> coef;
  std::vector<int> frag_cost_order;

  // ---- device workspace ----
  std::vector<void *> allocs;
  double *slab_buf = nullptr;
  int slab_nb = 1;
  double *eq = nullptr, *sstore = nullptr, *fstore = nullptr;
  double *ps = nullptr, *pf = nullptr, *x0 = nullptr, *xb = nullptr;
  double *tmp = nullptr, *fp = nullptr, *zb = nullptr, *kt = nullptr;
  double *et = nullptr, *ev0 = nullptr;
  int32_t *rank = nullptr;
  bool bases_done = false;  // X, eps~, rank computed by an eager preparation
  int32_t *sflag = nullptr;  // per slot: overlap not safely positive definite
  double *eig_ws = nullptr;  // eigensolver workspace for orders beyond LDS
  int64_t eig_ws_doubles = 0;
  double *cws = nullptr;     // records of the split Fock step (chase)
  int64_t cws_doubles = 0;
  int32_t *eig_meta = nullptr, *eig_redo = nullptr;
  double *at = nullptr, *mt = nullptr, *st0 = nullptr;
  double *ca = nullptr, *cm = nullptr, *st1 = nullptr;
  double *scratch = nullptr;
  int64_t scratch_stride = 0;
  int32_t *status = nullptr;
  int32_t *h_status = nullptr;
  double *d_coef = nullptr;
  int32_t *d_sub = nullptr;
  double *d_e3 = nullptr;
  unsigned char *noalloc_scratch = nullptr;  // this device's copy of `scratch`
  double *h_e3 = nullptr;
  int32_t *d_rows = nullptr;
  SlotInfo *d_slots = nullptr;

  // ---- plans ----
  std::vector<std::pair<int, int>> proj_batches;  // [i0, i1)
  std::vector<GemmList> glists;  // every GEMM task list of the handle
  std::vector<int> L_proj;       // indices into glists (-1: none)
  int L_pk = -1, L_pkw = -1, L_sf = -1;
  AssembleTask *d_asm_pair = nullptr;
  int n_asm_pair = 0;
  EigTask *d_eig0 = nullptr, *d_eig1 = nullptr;
  int L_m1 = -1, L_fp = -1, L_x = -1, L_m2 = -1, L_kt = -1;
  AssembleTask *d_asm_st = nullptr;
  int n_asm_st = 0;
  int L_stm = -1, L_st1 = -1;
  std::vector<Chunk> chunks;
  int64_t gamma_rows = 0;
  int64_t k_elems = 0;

  // ---- split-precision projection / pair_K (MBE3_MIXED_BF16) ----
  uint16_t *qplanes = nullptr, *splanes = nullptr, *gplanes = nullptr;
  int64_t q_ps = 0, s_ps = 0, g_ps = 0;  // plane strides (elements)
  std::vector<MixedTask *> d_mproj;
  std::vector<int64_t> t_mproj;
  MixedTask *d_mpk = nullptr;
  int64_t t_mpk = 0;
  int32_t *d_mrows = nullptr;
  int64_t *d_k_off = nullptr;    // k_off on the device
  int32_t *d_row_lmo = nullptr;  // LMO of every gamma row (fitting domains)
  int32_t *d_row_x = nullptr;    // OSV block (orbital x) of every gamma row
  int32_t *d_nbr_off = nullptr, *d_nbr = nullptr;  // N+(i) as CSR on the device
  std::vector<std::pair<std::string, std::vector<MixedTask>>> h_mixed;
  std::vector<int32_t> h_mrows;

  // ---- gradient (planned on first use) ----
  bool grad_planned = false;
  bool grad_ready = false;   // W and dE/df of the last fragment_solve are valid
  double *wt = nullptr;      // W~ per slot (K~ layout)
  double *yfin = nullptr, *gterm = nullptr, *gdiag = nullptr;
  double *graw = nullptr;    // unsymmetrised dE/df
  double *ga = nullptr, *dg = nullptr;
  double *dot_part = nullptr, *d_probe = nullptr, *h_probe = nullptr;
  int64_t yfin_max = 1, gterm_max = 1, gdiag_max = 1, ga_total = 1;
  int L_wm = -1, L_ww = -1, L_dg = -1, L_up = -1;
  std::vector<int32_t> h_grows;  // host copy of d_grows, for the bounds check
  GASeg *d_ga = nullptr;
  int n_ga = 0;
  int32_t *d_grows = nullptr;

  // ---- per-phase event timing (mbe3_set_timing) ----
  bool timing = false;
  struct Region { int phase; hipEvent_t a, b; };
  std::vector<Region> regions;
  std::vector<hipEvent_t> event_pool;
  size_t event_next = 0;
  double phase_ms[MBE3_NPHASE] = {0};
  int64_t phase_n[MBE3_NPHASE] = {0};

  // ---- HIP graph of a recorded call sequence (mbe3_graph_begin/end) ----
  hipStream_t user_stream = nullptr;  // the caller's stream while recording
  hipStream_t cap_stream = nullptr;   // private stream the calls record on
  bool recording = false, rec_failed = false;
  bool rec_solve = false, rec_grad = false, rec_energy = false;
  bool g_solve = false, g_grad = false, g_energy = false;  // in the graph
  // one segment per phase scope when timing is on (events go between the
  // segment launches), else a single segment
  struct Segment { int phase; hipGraph_t g; hipGraphExec_t x; };
  std::vector<Segment> segs;
  int seg_phase = -1;  // phase of the segment being recorded

  // ---- host mirrors of the plans, for the bounds check ----
  bool dry = false;  // plan only: no device allocation or copies
  int64_t at_total = 0, mt_total = 0, st0_total = 0;
  int64_t max_ca = 1, max_cm = 1, max_st1 = 1, n_rows = 0;
  std::string tune_report;  // last mbe3_autotune, one line per list
  std::vector<std::pair<std::array<int64_t, 2>, std::vector<AssembleTask>>> h_asm;
  std::vector<std::pair<int, std::vector<EigTask>>> h_eig;
  std::vector<std::vector<FragDesc>> h_fds;
  std::vector<std::vector<Term>> h_terms;
  std::vector<int32_t> h_rows;

  int fail(int code, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    err = buf;
    if (recording) rec_failed = true;
    return code;
  }
  ~mbe3_handle() {
    for (auto &sg : segs) {
      if (sg.x) (void)hipGraphExecDestroy(sg.x);
      if (sg.g) (void)hipGraphDestroy(sg.g);
    }
    if (cap_stream) (void)hipStreamDestroy(cap_stream);
    for (hipEvent_t e : event_pool) (void)hipEventDestroy(e);
    for (void *p : allocs) (void)hipFree(p);
    if (h_status) (void)hipHostFree(h_status);
    if (h_e3) (void)hipHostFree(h_e3);
    if (h_probe) (void)hipHostFree(h_probe);
  }
};

#define HIP_TRY(h, expr)                                                   \
  do {                                                                     \
    hipError_t e_ = (expr);                                                \
    if (e_ != hipSuccess)                                                  \
      return (h)->fail(MBE3_EHIP, "%s: %s (%s:%d)", #expr,                  \
                       hipGetErrorString(e_), __FILE__, __LINE__);         \
  } while (0)

namespace {

// Event pair around a group of launches of one phase (only when timing).
hipEvent_t next_event(mbe3_handle *h) {
  if (h->event_next == h->event_pool.size()) {
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    h->event_pool.push_back(e);
  }
  return h->event_pool[h->event_next++];
}
// Close the graph segment being recorded (kept if it holds any node) and
// start the next one, of phase `next`.
void cut_segment(mbe3_handle *h, int next, bool reopen) {
  hipGraph_t g = nullptr;
  hipError_t e = hipStreamEndCapture(h->cap_stream, &g);
  if (e == hipSuccess && g) {
    size_t n = 0;
    e = hipGraphGetNodes(g, nullptr, &n);
    if (e == hipSuccess && n > 0) {
      hipGraphExec_t x = nullptr;
      e = hipGraphInstantiateWithFlags(&x, g, 0);
      if (e == hipSuccess) {
        h->segs.push_back({h->seg_phase, g, x});
        g = nullptr;
      }
    }
  }
  if (g) (void)hipGraphDestroy(g);
  if (e != hipSuccess) {
    h->rec_failed = true;
    h->err = std::string("graph segment: ") + hipGetErrorString(e);
  }
  h->seg_phase = next;
  if (reopen && hipStreamBeginCapture(h->cap_stream, hipStreamCaptureModeRelaxed) != hipSuccess) {
    h->rec_failed = true;
    h->err = "hipStreamBeginCapture failed";
  }
}

// Times the launches of one phase: HIP events around them when timing is
// on; while recording with timing, a graph segment of their own.
struct PhaseScope {
  mbe3_handle *h;
  int phase;
  hipEvent_t a = nullptr;
  bool seg = false;
  PhaseScope(mbe3_handle *hh, int ph) : h(hh), phase(ph) {
    if (!h->timing) return;
    if (h->recording) {
      cut_segment(h, phase, true);
      seg = true;
    } else if ((a = next_event(h))) {
      (void)hipEventRecord(a, h->stream);
    }
  }
  ~PhaseScope() {
    if (seg) {
      cut_segment(h, -1, true);
      return;
    }
    if (!a) return;
    hipEvent_t b = next_event(h);
    if (!b) return;
    (void)hipEventRecord(b, h->stream);
    h->regions.push_back({phase, a, b});
  }
};

template <class T>
int dev_alloc(mbe3_handle *h, T **p, int64_t n) {
  *p = nullptr;
  if (h->dry) return MBE3_OK;
  if (n <= 0) n = 1;
  void *q = nullptr;
  hipError_t e = hipMalloc(&q, (size_t)n * sizeof(T));
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return h->fail(MBE3_ENOMEM, "hipMalloc of %lld bytes failed: %s",
                   (long long)(n * (int64_t)sizeof(T)), hipGetErrorString(e));
  }
  h->allocs.push_back(q);
  *p = (T *)q;
  return MBE3_OK;
}

template <class T>
int upload(mbe3_handle *h, T **dst, const std::vector<T> &v) {
  int rc = dev_alloc(h, dst, (int64_t)v.size());
  if (rc) return rc;
  if (!v.empty() && !h->dry)
    HIP_TRY(h, hipMemcpy(*dst, v.data(), v.size() * sizeof(T),
                         hipMemcpyHostToDevice));
  return MBE3_OK;
}

// Finalise a task list: tile prefix sums for the given shape.
int64_t finish_tasks(std::vector<GemmTask> &ts, GemmShape shape) {
  int64_t acc = 0;
  const int bn = gemm_tile_n(shape);
  for (auto &t : ts) {
    t.tiles_n = (t.N + bn - 1) / bn;
    t.tile_begin = acc;
    acc += gemm_tile_count(t, shape);
  }
  return acc;
}

// Register a task list (tiled for `shape`) with its device copy; *idx gets
// its index in h->glists.
int add_list(mbe3_handle *h, const std::string &name, std::vector<GemmTask> &ts,
             GemmShape shape, int rows_table, int *idx) {
  GemmList L;
  L.name = name;
  L.shape = shape;
  L.rows_table = rows_table;
  L.tiles = finish_tasks(ts, shape);
  L.host = ts;
  const int rc = upload(h, &L.d, ts);
  if (rc) return rc;
  *idx = (int)h->glists.size();
  h->glists.push_back(std::move(L));
  return MBE3_OK;
}

// Register a list as two: tasks whose output is at most 64 wide (planned
// 64x64 tiles) and the wider ones (planned 96x96), each with its own shape.
int add_split_lists(mbe3_handle *h, const std::string &name, const std::vector<GemmTask> &ts,
                    int *idx_narrow, int *idx_wide) {
  std::vector<GemmTask> nt, wt;
  for (const GemmTask &t : ts) (std::max(t.M, t.N) > 64 ? wt : nt).push_back(t);
  int rc;
  if (!nt.empty() && (rc = add_list(h, name, nt, GEMM_64x64, 0, idx_narrow))) return rc;
  if (!wt.empty() && (rc = add_list(h, name + " wide", wt, GEMM_96x96, 0, idx_wide))) return rc;
  return MBE3_OK;
}

hipError_t launch_list(mbe3_handle *h, int idx, const GemmBases &b, hipStream_t s) {
  if (idx < 0) return hipSuccess;
  const GemmList &L = h->glists[idx];
  return launch_gemm_tasks(L.d, (int)L.host.size(), L.tiles, b, L.shape, s);
}

GemmTask gemm(int a_buf, int64_t a_off, int lda, int transA, int b_buf,
              int64_t b_off, int ldb, int transB, int c_buf, int64_t c_off,
              int ldc, int M, int N, int K, double alpha = 1.0,
              double beta = 0.0) {
  GemmTask t;
  std::memset(&t, 0, sizeof t);
  t.a_buf = a_buf; t.a_off = a_off; t.lda = lda; t.transA = transA;
  t.b_buf = b_buf; t.b_off = b_off; t.ldb = ldb; t.transB = transB;
  t.c_buf = c_buf; t.c_off = c_off; t.ldc = ldc;
  t.M = M; t.N = N; t.K = K;
  t.alpha = alpha; t.beta = beta;
  t.a_rows = -1; t.b_rows = -1;
  t.ct_off = -1;
  return t;
}

int validate_and_copy(mbe3_handle *h, const mbe3_problem *p) {
  if (!p) return h->fail(MBE3_EINVAL, "problem is NULL");
  if (p->n_occ < 1 || p->n_vir < 1 || p->n_aux < 1)
    return h->fail(MBE3_EINVAL, "sizes must be positive (n_occ=%d n_vir=%d n_aux=%d)",
                   p->n_occ, p->n_vir, p->n_aux);
  if (!p->r || !p->Q || !p->eps_vir || !p->f_occ)
    return h->fail(MBE3_EINVAL, "r, Q, eps_vir and f_occ are required");
  if (!p->slab && (!p->w_ia || !p->w_iP))
    return h->fail(MBE3_EINVAL, "either slab or (w_ia, w_iP) must be given");
  if (!(p->tol > 0.0) || p->max_iter < 0 || !(p->tau_S >= 0.0))
    return h->fail(MBE3_EINVAL, "tol > 0, max_iter >= 0, tau_S >= 0 required");
  if (p->precision != MBE3_FP64 && p->precision != MBE3_MIXED_BF16 &&
      p->precision != MBE3_MIXED_BF16_PROJ)
    return h->fail(MBE3_EINVAL, "unsupported precision %d", p->precision);
  h->precision = p->precision;
  if (p->warm_start != 0 && p->warm_start != 1)
    return h->fail(MBE3_EINVAL, "warm_start must be 0 or 1");
  h->warm_start = p->warm_start == 1;
  h->ldk_vir = (p->n_vir + 7) & ~7;
  h->ldk_aux = (p->n_aux + 7) & ~7;
  h->n_occ = p->n_occ; h->n_vir = p->n_vir; h->n_aux = p->n_aux;
  h->Q = p->Q; h->eps = p->eps_vir; h->f = p->f_occ;
  h->w_ia = p->w_ia; h->w_iP = p->w_iP; h->slab = p->slab; h->seed = p->seed;
  h->tol = p->tol; h->tau_S = p->tau_S; h->max_iter = p->max_iter;
  h->r.assign(p->r, p->r + p->n_occ);
  h->q_off.assign(h->n_occ + 1, 0);
  for (int i = 0; i < h->n_occ; ++i) {
    if (h->r[i] < 1 || h->r[i] > h->n_vir)
      return h->fail(MBE3_EINVAL, "r[%d]=%d out of [1, n_vir]", i, h->r[i]);
    h->q_off[i + 1] = h->q_off[i] + h->r[i];
  }
  if (p->n_pair < 0 || (p->n_pair > 0 && !p->pairs))
    return h->fail(MBE3_EINVAL, "bad pair list");
  for (int64_t m = 0; m < p->n_pair; ++m) {
    const int a = p->pairs[2 * m], b = p->pairs[2 * m + 1];
    if (a < 0 || b >= h->n_occ || a >= b)
      return h->fail(MBE3_EINVAL, "pair %lld = (%d, %d) invalid", (long long)m, a, b);
    if (h->pair_slot.count(key2(a, b)))
      return h->fail(MBE3_EINVAL, "pair (%d, %d) repeated", a, b);
    h->pair_slot[key2(a, b)] = h->n_occ + (int)m;
    h->pairs.push_back({a, b});
  }
  if (p->n_frag < 1 || !p->frags) return h->fail(MBE3_EINVAL, "no fragments");
  std::map<std::array<int, 3>, int64_t> seen;
  for (int64_t m = 0; m < p->n_frag; ++m) {
    std::array<int, 3> o = {p->frags[3 * m], p->frags[3 * m + 1], p->frags[3 * m + 2]};
    int n = 0;
    while (n < 3 && o[n] >= 0) ++n;
    for (int k = n; k < 3; ++k)
      if (o[k] != -1) return h->fail(MBE3_EINVAL, "fragment %lld: bad padding", (long long)m);
    if (n == 0) return h->fail(MBE3_EINVAL, "fragment %lld is empty", (long long)m);
    for (int k = 0; k < n; ++k)
      if (o[k] >= h->n_occ || (k && o[k] <= o[k - 1]))
        return h->fail(MBE3_EINVAL, "fragment %lld: orbitals must be ascending and < n_occ",
                       (long long)m);
    if (seen.count(o)) return h->fail(MBE3_EINVAL, "fragment %lld repeated", (long long)m);
    seen[o] = m;
    h->frags.push_back(o);
  }
  // downward closure: every sub-fragment present, every inner pair kept
  for (auto &o : h->frags) {
    int n = o[2] >= 0 ? 3 : (o[1] >= 0 ? 2 : 1);
    for (int k = 0; k < n; ++k)
      if (!seen.count({o[k], -1, -1}))
        return h->fail(MBE3_EINVAL, "fragment (%d,%d,%d) lacks monomer %d", o[0], o[1], o[2], o[k]);
    for (int a = 0; a < n; ++a)
      for (int b = a + 1; b < n; ++b) {
        if (!h->pair_slot.count(key2(o[a], o[b])))
          return h->fail(MBE3_EINVAL, "fragment (%d,%d,%d): pair (%d,%d) not kept",
                         o[0], o[1], o[2], o[a], o[b]);
        if (n == 3 && !seen.count({o[a], o[b], -1}))
          return h->fail(MBE3_EINVAL, "fragment (%d,%d,%d) lacks dimer (%d,%d)",
                         o[0], o[1], o[2], o[a], o[b]);
      }
  }
  // MBE(3) coefficients and sub-fragment indices
  std::vector<int64_t> deg(h->n_occ, 0), tri_i(h->n_occ, 0);
  std::unordered_map<int64_t, int64_t> tri_ij;
  for (auto &o : h->frags) {
    if (o[1] >= 0 && o[2] < 0) { deg[o[0]]++; deg[o[1]]++; }
    if (o[2] >= 0) {
      tri_i[o[0]]++; tri_i[o[1]]++; tri_i[o[2]]++;
      tri_ij[key2(o[0], o[1])]++; tri_ij[key2(o[0], o[2])]++; tri_ij[key2(o[1], o[2])]++;
    }
  }
  h->coef.resize(h->frags.size());
  for (size_t m = 0; m < h->frags.size(); ++m) {
    auto &o = h->frags[m];
    if (o[1] < 0) h->coef[m] = (double)(1 - deg[o[0]] + tri_i[o[0]]);
    else if (o[2] < 0) {
      auto it = tri_ij.find(key2(o[0], o[1]));
      h->coef[m] = (double)(1 - (it == tri_ij.end() ? 0 : it->second));
    } else h->coef[m] = 1.0;
  }
  return MBE3_OK;
}

int build_layout(mbe3_handle *h) {
  const int n = h->n_occ;
  h->nbr.assign(n, {});
  for (int i = 0; i < n; ++i) h->nbr[i].push_back(i);
  for (auto &pq : h->pairs) {
    h->nbr[pq[0]].push_back(pq[1]);
    h->nbr[pq[1]].push_back(pq[0]);
  }
  h->g_off.assign(n + 1, 0);
  for (int i = 0; i < n; ++i) {
    std::sort(h->nbr[i].begin(), h->nbr[i].end());
    int64_t row = h->g_off[i];
    for (int x : h->nbr[i]) {
      h->grow[key2(i, x)] = row;
      row += h->r[x];
    }
    h->g_off[i + 1] = row;
  }
  h->gamma_rows = h->g_off[n];
  h->n_slot = n + (int64_t)h->pairs.size();
  h->sp.resize(h->n_slot); h->sq.resize(h->n_slot);
  h->sd.resize(h->n_slot); h->sD.resize(h->n_slot);
  h->k_off.assign(h->n_slot + 1, 0);
  h->x_off.assign(h->n_slot + 1, 0);
  h->kt_off.assign(h->n_slot + 1, 0);
  h->et_off.assign(h->n_slot + 1, 0);
  h->dmax = 16;
  for (int64_t s = 0; s < h->n_slot; ++s) {
    int p, q;
    if (s < n) { p = q = (int)s; }
    else { p = h->pairs[s - n][0]; q = h->pairs[s - n][1]; }
    const int d = p == q ? h->r[p] : h->r[p] + h->r[q];
    const int D = round16(d);
    h->sp[s] = p; h->sq[s] = q; h->sd[s] = d; h->sD[s] = D;
    h->dmax = std::max(h->dmax, D);
    h->k_off[s + 1] = h->k_off[s] + (int64_t)d * d;
    h->x_off[s + 1] = h->x_off[s] + (int64_t)d * D;
    h->kt_off[s + 1] = h->kt_off[s] + (int64_t)D * D;
    h->et_off[s + 1] = h->et_off[s] + D;
  }
  h->k_elems = h->k_off[h->n_slot];
  if (h->dmax > DMAX_SUPPORTED)
    return h->fail(MBE3_EINVAL, "pair dimension %d exceeds the supported %d",
                   h->dmax, DMAX_SUPPORTED);
  // S/F block store: (x, x) and kept (x, y), x < y
  h->sb_total = 0;
  for (int x = 0; x < n; ++x)
    for (int y : h->nbr[x])
      if (y >= x) {
        h->sb_off[key2(x, y)] = h->sb_total;
        h->sb_total += (int64_t)h->r[x] * h->r[y];
      }
  return MBE3_OK;
}

int slot_of(const mbe3_handle *h, int a, int b) {
  if (a == b) return a;
  if (a > b) std::swap(a, b);
  auto it = h->pair_slot.find(key2(a, b));
  return it == h->pair_slot.end() ? -1 : it->second;
}

// Block source for S_(a,b) (or F) in the block store.
BlockSrc bsrc(const mbe3_handle *h, int a, int b) {
  BlockSrc s;
  if (a <= b) {
    s.off = h->sb_off.at(key2(a, b));
    s.ld = h->r[b];
    s.trans = 0;
  } else {
    s.off = h->sb_off.at(key2(b, a));
    s.ld = h->r[a];
    s.trans = 1;
  }
  return s;
}

std::vector<int> slot_orbs(const mbe3_handle *h, int s) {
  if (h->sp[s] == h->sq[s]) return {h->sp[s]};
  return {h->sp[s], h->sq[s]};
}

// Assembly task for V_A^T M V_B with A = orbitals of slot (or list), into
// out_off with leading dimension ld_out; rows_out x cols_out region.
AssembleTask asm_task(const mbe3_handle *h, const std::vector<int> &ro,
                      const std::vector<int> &co, int src_buf, int out_buf,
                      int64_t out_off, int ld_out, int rows_out, int cols_out) {
  AssembleTask t;
  std::memset(&t, 0, sizeof t);
  t.out_off = out_off; t.ld_out = ld_out; t.src_buf = src_buf;
  t.out_buf = out_buf;
  t.nrb = (int)ro.size(); t.ncb = (int)co.size();
  for (int a = 0; a < t.nrb; ++a) t.rsz[a] = h->r[ro[a]];
  for (int b = 0; b < t.ncb; ++b) t.csz[b] = h->r[co[b]];
  t.rows_out = rows_out; t.cols_out = cols_out;
  for (int a = 0; a < t.nrb; ++a)
    for (int b = 0; b < t.ncb; ++b) t.b[a][b] = bsrc(h, ro[a], co[b]);
  return t;
}

int build_plans(mbe3_handle *h) {
  const int n = h->n_occ, nv = h->n_vir, na = h->n_aux;
  int rc;
  std::vector<int32_t> rows;

  // ---- projection: one GEMM per orbital, A rows gathered from Q ----
  const int64_t slab_elems = (int64_t)nv * na;
  // split projection in both mixed forms, split pair_K in MBE3_MIXED_BF16
  const bool mixed = h->precision != MBE3_FP64;
  const bool mixed_k = h->precision == MBE3_MIXED_BF16;
  if (mixed) {  // three bf16 planes per slab element
    int64_t nb = SLAB_BUDGET / ((int64_t)na * h->ldk_vir * 6);
    h->slab_nb = (int)std::max<int64_t>(1, std::min<int64_t>(nb, n));
  } else if (!h->slab) {
    int64_t nb = SLAB_BUDGET / (slab_elems * 8);
    nb = std::max<int64_t>(1, std::min<int64_t>(nb, n));
    h->slab_nb = (int)nb;
  } else {
    h->slab_nb = n;
  }
  for (int i0 = 0; i0 < n; i0 += h->slab_nb) {
    const int i1 = std::min(n, i0 + h->slab_nb);
    h->proj_batches.push_back({i0, i1});
    std::vector<GemmTask> ts;
    for (int i = i0; i < i1; ++i) {
      GemmTask t = gemm(B_Q, 0, nv, 0, B_SLAB,
                        (int64_t)(h->slab ? i : i - i0) * slab_elems, na, 0,
                        B_GAMMA, h->g_off[i] * na, na,
                        (int)(h->g_off[i + 1] - h->g_off[i]), na, nv);
      t.a_rows = (int32_t)rows.size();
      for (int x : h->nbr[i])
        for (int mu = 0; mu < h->r[x]; ++mu) rows.push_back((int32_t)(h->q_off[x] + mu));
      ts.push_back(t);
    }
    if (!mixed) {  // the split-precision form has its own task lists
      int li = -1;
      if ((rc = add_list(h, "project " + std::to_string(h->L_proj.size()), ts,
                         GEMM_128x128, 0, &li)))
        return rc;
      h->L_proj.push_back(li);
    }
  }

  // ---- pair K: K_s = L R^T with gathered rows of gamma; slots up to 64
  //      wide and wider ones in separate lists (own tile shapes) ----
  {
    std::vector<GemmTask> ts, tw;
    for (int64_t s = 0; s < h->n_slot; ++s) {
      const int p = h->sp[s], q = h->sq[s], d = h->sd[s];
      GemmTask t = gemm(B_GAMMA, 0, na, 0, B_GAMMA, 0, na, 1, B_K, h->k_off[s],
                        d, d, d, na);
      t.a_rows = (int32_t)rows.size();
      for (int x : slot_orbs(h, (int)s))
        for (int mu = 0; mu < h->r[x]; ++mu) rows.push_back((int32_t)(h->grow.at(key2(p, x)) + mu));
      t.b_rows = (int32_t)rows.size();
      for (int x : slot_orbs(h, (int)s))
        for (int mu = 0; mu < h->r[x]; ++mu) rows.push_back((int32_t)(h->grow.at(key2(q, x)) + mu));
      (d > 64 ? tw : ts).push_back(t);
    }
    if (!mixed_k && !ts.empty() &&
        (rc = add_list(h, "pair_K", ts, GEMM_64x64, 0, &h->L_pk)))
      return rc;
    if (!mixed_k && !tw.empty() &&
        (rc = add_list(h, "pair_K wide", tw, GEMM_96x96, 0, &h->L_pkw)))
      return rc;
  }
  h->n_rows = (int64_t)rows.size();
  h->h_rows = rows;
  if ((rc = upload(h, &h->d_rows, rows))) return rc;

  // ---- split-precision variants of the two products ----
  if (mixed) {
    std::vector<int32_t> mr;
    const int lv = h->ldk_vir, la = h->ldk_aux;
    auto finish = [](std::vector<MixedTask> &ts, MixedShape sh) {
      int64_t acc = 0;
      for (auto &t : ts) {
        t.tiles_n = (t.N + mixed_tile_n(sh) - 1) / mixed_tile_n(sh);
        t.tile_begin = acc;
        acc += mixed_tile_count(t, sh);
      }
      return acc;
    };
    for (auto &bt : h->proj_batches) {
      std::vector<MixedTask> ts;
      for (int i = bt.first; i < bt.second; ++i) {
        MixedTask t;
        std::memset(&t, 0, sizeof t);
        t.a_off = 0;
        t.a_rows = (int32_t)mr.size();
        for (int x : h->nbr[i])
          for (int mu = 0; mu < h->r[x]; ++mu) mr.push_back((int32_t)(h->q_off[x] + mu));
        t.b_off = (int64_t)(i - bt.first) * na * lv;
        t.b_rows = -1;
        t.c_off = h->g_off[i] * na;
        t.M = (int)(h->g_off[i + 1] - h->g_off[i]);
        t.N = na;
        t.K = lv;
        t.lda = lv; t.ldb = lv; t.ldc = na;
        ts.push_back(t);
      }
      h->t_mproj.push_back(finish(ts, MIXED_64x128));
      MixedTask *d = nullptr;
      if ((rc = upload(h, &d, ts))) return rc;
      h->d_mproj.push_back(d);
      h->h_mixed.push_back({"project (split)", ts});
    }
    if (mixed_k) {
      std::vector<MixedTask> ts;
      for (int64_t sl = 0; sl < h->n_slot; ++sl) {
        const int p = h->sp[sl], q = h->sq[sl], d = h->sd[sl];
        MixedTask t;
        std::memset(&t, 0, sizeof t);
        t.a_rows = (int32_t)mr.size();
        for (int x : slot_orbs(h, (int)sl))
          for (int mu = 0; mu < h->r[x]; ++mu) mr.push_back((int32_t)(h->grow.at(key2(p, x)) + mu));
        t.b_rows = (int32_t)mr.size();
        for (int x : slot_orbs(h, (int)sl))
          for (int mu = 0; mu < h->r[x]; ++mu) mr.push_back((int32_t)(h->grow.at(key2(q, x)) + mu));
        t.c_off = h->k_off[sl];
        t.M = d; t.N = d; t.K = la;
        t.lda = la; t.ldb = la; t.ldc = d;
        ts.push_back(t);
      }
      h->t_mpk = finish(ts, MIXED_32x64);
      if ((rc = upload(h, &h->d_mpk, ts))) return rc;
      h->h_mixed.push_back({"pair_K (split)", ts});
    }
    h->h_mrows = mr;
    if ((rc = upload(h, &h->d_mrows, mr))) return rc;
    h->q_ps = h->q_off[n] * lv;
    h->s_ps = (int64_t)h->slab_nb * na * lv;
    h->g_ps = mixed_k ? h->gamma_rows * la : 0;
  }

  // ---- S / F blocks ----
  {
    std::vector<GemmTask> ts;
    for (int x = 0; x < n; ++x)
      for (int y : h->nbr[x])
        if (y >= x) {
          const int64_t off = h->sb_off.at(key2(x, y));
          ts.push_back(gemm(B_Q, h->q_off[x] * nv, nv, 0, B_Q, h->q_off[y] * nv, nv, 1,
                            B_SS, off, h->r[y], h->r[x], h->r[y], nv));
          ts.push_back(gemm(B_Q, h->q_off[x] * nv, nv, 0, B_EQ, h->q_off[y] * nv, nv, 1,
                            B_FS, off, h->r[y], h->r[x], h->r[y], nv));
        }
    if ((rc = add_list(h, "S/F blocks", ts, GEMM_64x64, 0, &h->L_sf))) return rc;
  }

  // ---- pair 4-block S, F (k layout) and the basis pipeline ----
  {
    std::vector<AssembleTask> as;
    std::vector<EigTask> e0, e1;
    std::vector<GemmTask> m1, fpt, xt, m2, ktt;
    for (int64_t s = 0; s < h->n_slot; ++s) {
      const int d = h->sd[s], D = h->sD[s];
      const auto o = slot_orbs(h, (int)s);
      as.push_back(asm_task(h, o, o, 0, 0, h->k_off[s], d, d, d));  // S -> ps
      as.push_back(asm_task(h, o, o, 1, 1, h->k_off[s], d, d, d));  // F -> pf
      EigTask a;
      a.a_off = h->k_off[s]; a.lda = d; a.n = d; a.D = D; a.slot = (int)s;
      a.o_off = h->x_off[s]; a.e_off = h->et_off[s];
      a.w_off = -1;
      e0.push_back(a);
      EigTask b = a;
      b.a_off = h->kt_off[s]; b.lda = D; b.o_off = h->kt_off[s];
      if (d <= eig_split_max_order()) {  // the Fock step's chase record
        b.w_off = h->cws_doubles;
        h->cws_doubles += eig_chase_ws_doubles(D);
      }
      e1.push_back(b);
      // M1 = F X0 (d x D) -> tmp (x layout)
      m1.push_back(gemm(B_PF, h->k_off[s], d, 0, B_X0, h->x_off[s], D, 0, B_TMP,
                        h->x_off[s], D, d, D, d));
      // F' = X0^T M1 (D x D)
      fpt.push_back(gemm(B_X0, h->x_off[s], D, 1, B_TMP, h->x_off[s], D, 0, B_FP,
                         h->kt_off[s], D, D, D, d));
      // X = X0 Z (d x D)
      xt.push_back(gemm(B_X0, h->x_off[s], D, 0, B_Z, h->kt_off[s], D, 0, B_X,
                        h->x_off[s], D, d, D, D));
      // M2 = K X (d x D) -> tmp ; K~ = X^T M2 (D x D) -> kt
      m2.push_back(gemm(B_K, h->k_off[s], d, 0, B_X, h->x_off[s], D, 0, B_TMP,
                        h->x_off[s], D, d, D, d));
      ktt.push_back(gemm(B_X, h->x_off[s], D, 1, B_TMP, h->x_off[s], D, 0, B_KT,
                         h->kt_off[s], D, D, D, d));
    }
    h->n_asm_pair = (int)as.size();
    if ((rc = upload(h, &h->d_asm_pair, as))) return rc;
    if ((rc = upload(h, &h->d_eig0, e0))) return rc;
    if ((rc = upload(h, &h->d_eig1, e1))) return rc;
    h->h_asm.push_back({{B_PS, B_PF}, as});
    h->h_eig.push_back({0, e0});
    h->h_eig.push_back({1, e1});
    if ((rc = add_list(h, "M1", m1, GEMM_64x64, 0, &h->L_m1))) return rc;
    if ((rc = add_list(h, "F'", fpt, GEMM_64x64, 0, &h->L_fp))) return rc;
    if ((rc = add_list(h, "X", xt, GEMM_64x64, 0, &h->L_x))) return rc;
    if ((rc = add_list(h, "M2", m2, GEMM_64x64, 0, &h->L_m2))) return rc;
    if ((rc = add_list(h, "K~", ktt, GEMM_64x64, 0, &h->L_kt))) return rc;
  }

  // ---- pair-level S~ between a pair slot and its two diagonal slots ----
  // For slot t = (p, q) and u in {p, q}:
  //   A_tu = V_t^T Q_u (d_t x r_u), M = A_tu X_u (d_t x D_u),
  //   S~_(t,u) = X_t^T M (D_t x D_u), S~_(u,t) = M^T X_t (D_u x D_t).
  std::vector<int64_t> st0_tu(h->n_slot * 2, -1), st0_ut(h->n_slot * 2, -1);
  int64_t st0_total = 0;
  {
    std::vector<AssembleTask> as;
    std::vector<GemmTask> gm, g1;
    int64_t at_total = 0, mt_total = 0;
    for (int64_t s = n; s < h->n_slot; ++s) {
      const int dt = h->sd[s], Dt = h->sD[s];
      const auto o = slot_orbs(h, (int)s);
      for (int k = 0; k < 2; ++k) {
        const int u = o[k];
        const int ru = h->r[u], Du = h->sD[u];
        as.push_back(asm_task(h, o, {u}, 0, 0, at_total, ru, dt, ru));
        gm.push_back(gemm(B_AT, at_total, ru, 0, B_X, h->x_off[u], Du, 0, B_MT,
                          mt_total, Du, dt, Du, ru));
        // S~_(t,u) (Dt x Du) and, by the same task, its transpose S~_(u,t)
        st0_tu[2 * s + k] = st0_total;
        st0_ut[2 * s + k] = st0_total + (int64_t)Dt * Du;
        GemmTask t1 = gemm(B_X, h->x_off[s], Dt, 1, B_MT, mt_total, Du, 0, B_ST0,
                           st0_total, Du, Dt, Du, dt);
        t1.ct_off = st0_ut[2 * s + k];
        t1.ldct = Dt;
        g1.push_back(t1);
        st0_total += 2LL * Dt * Du;
        at_total += (int64_t)dt * ru;
        mt_total += (int64_t)dt * Du;
      }
    }
    h->n_asm_st = (int)as.size();
    h->h_asm.push_back({{B_AT, -1}, as});
    if ((rc = upload(h, &h->d_asm_st, as))) return rc;
    if (!gm.empty()) {
      if ((rc = add_list(h, "S~ M", gm, GEMM_64x64, 0, &h->L_stm))) return rc;
      if ((rc = add_list(h, "S~", g1, GEMM_64x64, 0, &h->L_st1))) return rc;
    }
    h->at_total = at_total; h->mt_total = mt_total; h->st0_total = st0_total;
    if ((rc = dev_alloc(h, &h->at, at_total))) return rc;
    if ((rc = dev_alloc(h, &h->mt, mt_total))) return rc;
    if ((rc = dev_alloc(h, &h->st0, st0_total))) return rc;
  }

  // ---- fragments: term tables and chunks ----
  std::vector<int64_t> cost(h->frags.size());
  for (size_t m = 0; m < h->frags.size(); ++m) {
    int64_t c = 0;
    for (int k = 0; k < 3; ++k)
      if (h->frags[m][k] >= 0) c += h->sD[h->frags[m][k]];
    const int nf = h->frags[m][2] >= 0 ? 3 : (h->frags[m][1] >= 0 ? 2 : 1);
    cost[m] = c * c * c * (nf == 3 ? 18 : (nf == 2 ? 4 : 1));
  }
  // the largest padded pair dimension among a fragment's slots: it picks the
  // solver kernel and its register / LDS layout for the whole chunk
  std::vector<int> fdim(h->frags.size());
  for (size_t m = 0; m < h->frags.size(); ++m) {
    const auto &o = h->frags[m];
    int d = 16;
    for (int a = 0; a < 3; ++a) {
      if (o[a] < 0) continue;
      d = std::max(d, h->sD[o[a]]);
      for (int b = a + 1; b < 3; ++b)
        if (o[b] >= 0) d = std::max(d, h->sD[slot_of(h, o[a], o[b])]);
    }
    fdim[m] = d;
  }
  // solver class of a fragment: the four-wave instances take every fragment
  // up to 80-wide pair domains (one chunk's instance is sized by its widest
  // fragment); each width above that has its own eight-wave instance, so
  // one class per width
  auto fclass = [&](int m) { return fdim[m] <= 80 ? 0 : fdim[m]; };
  std::vector<int> order(h->frags.size());
  for (size_t m = 0; m < order.size(); ++m) order[m] = (int)m;
  // with warm starts every monomer and dimer comes before the trimers (their
  // solutions seed the trimers' pairs); then by class, widest first, so
  // that each chunk holds one class; heavy first inside a class
  auto is_tri = [&](int m) { return h->frags[m][2] >= 0; };
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
    if (h->warm_start && is_tri(a) != is_tri(b)) return !is_tri(a);
    if (fclass(a) != fclass(b)) return fclass(a) > fclass(b);
    return cost[a] > cost[b];
  });

  Chunk cur;
  std::vector<FragDesc> fds;
  std::vector<Term> terms;
  std::vector<AssembleTask> cas;
  std::vector<GemmTask> cgm, cg1;
  int64_t ca_total = 0, cm_total = 0, st1_total = 0;
  int64_t max_ca = 1, max_cm = 1, max_st1 = 1;
  auto flush = [&](void) -> int {
    if (cur.frag_ids.empty()) return MBE3_OK;
    cur.n_frag = (int)fds.size();
    cur.n_terms = (int)terms.size();
    cur.n_asm = (int)cas.size();
    int rc2;
    h->h_fds.push_back(fds);
    h->h_terms.push_back(terms);
    h->h_asm.push_back({{B_CA, -1}, cas});
    if ((rc2 = upload(h, &cur.d_frags, fds))) return rc2;
    if ((rc2 = upload(h, &cur.d_terms, terms))) return rc2;
    if (!cas.empty()) {
      const std::string c = " " + std::to_string(h->chunks.size());
      if ((rc2 = upload(h, &cur.d_asm, cas))) return rc2;
      if ((rc2 = add_split_lists(h, "cross M" + c, cgm, &cur.L_m, &cur.L_mw))) return rc2;
      if ((rc2 = add_split_lists(h, "cross" + c, cg1, &cur.L_s1, &cur.L_s1w))) return rc2;
    }
    max_ca = std::max(max_ca, ca_total);
    max_cm = std::max(max_cm, cm_total);
    max_st1 = std::max(max_st1, st1_total);
    h->chunks.push_back(cur);
    cur = Chunk();
    fds.clear(); terms.clear(); cas.clear(); cgm.clear(); cg1.clear();
    ca_total = cm_total = st1_total = 0;
    return MBE3_OK;
  };

  for (int m : order) {
    const auto &o = h->frags[m];
    std::vector<int> F;
    for (int k = 0; k < 3; ++k)
      if (o[k] >= 0) F.push_back(o[k]);
    const int nf = (int)F.size();
    // local slots: diagonals, then pairs (ab, ac, bc)
    std::vector<int> ls;
    for (int x : F) ls.push_back(x);
    for (int a = 0; a < nf; ++a)
      for (int b = a + 1; b < nf; ++b) ls.push_back(slot_of(h, F[a], F[b]));
    // cross S~ needed by a trimer (bytes of this fragment's chunk stores)
    int64_t need = 0;
    if (nf == 3) {
      for (int a = 3; a < 6; ++a)
        for (int b = a + 1; b < 6; ++b) {
          const int64_t dt = h->sd[ls[a]], Dt = h->sD[ls[a]];
          const int64_t ds = h->sd[ls[b]], Ds = h->sD[ls[b]];
          need += (dt * ds + dt * Ds + 2 * Dt * Ds) * 8;
        }
    }
    const bool phase_change = !cur.frag_ids.empty() &&
                              ((h->warm_start && nf == 3 && !is_tri(cur.frag_ids.back())) ||
                               fclass(m) != fclass(cur.frag_ids.back()));
    if (!cur.frag_ids.empty() &&
        ((ca_total + cm_total + st1_total) * 8 + need > CHUNK_BUDGET || phase_change)) {
      if ((rc = flush())) return rc;
    }
    FragDesc fd;
    std::memset(&fd, 0, sizeof fd);
    fd.nt = (int)ls.size();
    fd.frag = m;
    fd.coef = h->coef[m];
    int ny = 0;
    for (int k = 0; k < fd.nt; ++k) {
      fd.slot[k] = ls[k];
      fd.ysub[k] = ny;
      const int D = h->sD[ls[k]];
      ny += D * D;
      fd.sym[k] = k < nf ? 1 : 0;
      fd.wgt[k] = k < nf ? 1 : 2;
      cur.dmax = std::max(cur.dmax, D);
    }
    fd.ny = ny;
    fd.warm_in = h->warm_start && nf == 3 ? 1 : 0;
    fd.warm_out = !h->warm_start ? -1 : (nf == 1 ? 0 : (nf == 2 ? 2 : -1));
    fd.yout = cur.ny_total;
    cur.ny_total += ny;
    cur.ny_max = std::max(cur.ny_max, ny);
    // cross S~ of this trimer: cross[a][b] = offset of row-major S~_(ls[a], ls[b])
    int64_t cross[6][6];
    for (auto &row : cross) for (auto &v : row) v = -1;
    if (nf == 3) {
      for (int a = 3; a < 6; ++a)
        for (int b = a + 1; b < 6; ++b) {
          const int t = ls[a], s = ls[b];
          const int dt = h->sd[t], Dt = h->sD[t], ds = h->sd[s], Ds = h->sD[s];
          cas.push_back(asm_task(h, slot_orbs(h, t), slot_orbs(h, s), 0, 0,
                                 ca_total, ds, dt, ds));
          // M = A X_s (dt x Ds)
          cgm.push_back(gemm(B_CA, ca_total, ds, 0, B_X, h->x_off[s], Ds, 0, B_CM,
                             cm_total, Ds, dt, Ds, ds));
          // S~_(t,s) = X_t^T M  (Dt x Ds), stored with its transpose
          // S~_(s,t) (Ds x Dt) by the same task
          cross[a][b] = st1_total;
          cross[b][a] = st1_total + (int64_t)Dt * Ds;
          GemmTask g1 = gemm(B_X, h->x_off[t], Dt, 1, B_CM, cm_total, Ds, 0, B_ST1,
                             st1_total, Ds, Dt, Ds, dt);
          g1.ct_off = cross[b][a];
          g1.ldct = Dt;
          cg1.push_back(g1);
          st1_total += 2LL * Dt * Ds;
          ca_total += (int64_t)dt * ds;
          cm_total += (int64_t)dt * Ds;
        }
    }
    auto local = [&](int a, int b) {  // local index of slot (a, b) orbitals
      const int s = slot_of(h, a, b);
      for (int k = 0; k < fd.nt; ++k)
        if (ls[k] == s) return k;
      return -1;
    };
    // pair-level S~ offsets: row-major S~_(u,t) (diag u, pair t) and S~_(t,u)
    auto st_ut = [&](int t, int u) {  // row-major S~_(u, t)
      const int k = (h->sp[t] == u) ? 0 : 1;
      return st0_ut[2 * t + k];
    };
    auto st_tu = [&](int t, int u) {  // row-major S~_(t, u)
      const int k = (h->sp[t] == u) ? 0 : 1;
      return st0_tu[2 * t + k];
    };
    fd.term_begin = (int)terms.size();
    for (int tl = 0; tl < fd.nt; ++tl) {
      const int t = ls[tl];
      const int p = h->sp[t], q = h->sq[t];
      if (p == q) {
        for (int k : F) {
          if (k == p) continue;
          Term tm;
          std::memset(&tm, 0, sizeof tm);
          const int s = slot_of(h, p, k);
          tm.target = tl; tm.src = local(p, k);
          tm.fx = p; tm.fy = k;
          tm.trans = k > p ? 1 : 0;  // T_kp from the stored (p,k)
          tm.st_buf = 0;
          tm.st_off = st_tu(s, p);   // row-major S~_(src=s, target=pp)
          terms.push_back(tm);
        }
      } else {
        // k = q in the first sum and k = p in the second (own diagonals)
        Term tm;
        std::memset(&tm, 0, sizeof tm);
        tm.target = tl; tm.fx = p; tm.fy = q; tm.st_buf = 0; tm.trans = 0;
        tm.src = local(q, q); tm.st_off = st_ut(t, q);
        terms.push_back(tm);
        tm.src = local(p, p); tm.st_off = st_ut(t, p);
        terms.push_back(tm);
        for (int r : F) {
          if (r == p || r == q) continue;
          // first sum, k = r: f_pr S_(pq,rq) T_rq S_(rq,pq)
          const int lrq = local(r, q), lpr = local(p, r);
          Term a;
          std::memset(&a, 0, sizeof a);
          a.target = tl; a.src = lrq; a.fx = p; a.fy = r;
          a.trans = r > q ? 1 : 0; a.st_buf = 1;
          a.st_off = cross[lrq][tl];
          terms.push_back(a);
          // second sum, k = r: f_rq S_(pq,pr) T_pr S_(pr,pq)
          Term b;
          std::memset(&b, 0, sizeof b);
          b.target = tl; b.src = lpr; b.fx = r; b.fy = q;
          b.trans = p > r ? 1 : 0; b.st_buf = 1;
          b.st_off = cross[lpr][tl];
          terms.push_back(b);
        }
      }
    }
    fd.term_end = (int)terms.size();
    fds.push_back(fd);
    cur.frag_ids.push_back(m);
  }
  if ((rc = flush())) return rc;
  h->max_ca = max_ca; h->max_cm = max_cm; h->max_st1 = max_st1;
  if ((rc = dev_alloc(h, &h->ca, max_ca))) return rc;
  if ((rc = dev_alloc(h, &h->cm, max_cm))) return rc;
  if ((rc = dev_alloc(h, &h->st1, max_st1))) return rc;

  // ---- slots, energies ----
  std::vector<SlotInfo> si(h->n_slot);
  for (int64_t s = 0; s < h->n_slot; ++s) {
    si[s].p = h->sp[s]; si[s].q = h->sq[s];
    si[s].d = h->sd[s]; si[s].D = h->sD[s];
    si[s].kt_off = h->kt_off[s]; si[s].et_off = h->et_off[s];
  }
  if ((rc = upload(h, &h->d_slots, si))) return rc;
  if ((rc = upload(h, &h->d_coef, h->coef))) return rc;
  {
    std::map<std::array<int, 3>, int> idx;
    for (size_t m = 0; m < h->frags.size(); ++m) idx[h->frags[m]] = (int)m;
    std::vector<int32_t> sub(6 * h->frags.size(), -1);
    for (size_t m = 0; m < h->frags.size(); ++m) {
      const auto &o = h->frags[m];
      if (o[1] < 0) continue;
      sub[6 * m + 0] = idx.at({o[0], -1, -1});
      sub[6 * m + 1] = idx.at({o[1], -1, -1});
      if (o[2] >= 0) {
        sub[6 * m + 2] = idx.at({o[2], -1, -1});
        sub[6 * m + 3] = idx.at({o[0], o[1], -1});
        sub[6 * m + 4] = idx.at({o[0], o[2], -1});
        sub[6 * m + 5] = idx.at({o[1], o[2], -1});
      }
    }
    if ((rc = upload(h, &h->d_sub, sub))) return rc;
  }
  return MBE3_OK;
}

int max_d(const mbe3_handle *h);

int alloc_workspace(mbe3_handle *h) {
  int rc;
  const int64_t nv = h->n_vir, na = h->n_aux;
  if (h->precision != MBE3_FP64) {
    if ((rc = dev_alloc(h, &h->qplanes, 3 * h->q_ps))) return rc;
    if ((rc = dev_alloc(h, &h->splanes, 3 * h->s_ps))) return rc;
    if (h->g_ps && (rc = dev_alloc(h, &h->gplanes, 3 * h->g_ps))) return rc;
  } else if (!h->slab &&
             (rc = dev_alloc(h, &h->slab_buf, (int64_t)h->slab_nb * nv * na))) {
    return rc;
  }
  {
    std::vector<int32_t> rl((size_t)h->gamma_rows), rx((size_t)h->gamma_rows);
    std::vector<int32_t> noff((size_t)h->n_occ + 1, 0), nb;
    for (int i = 0; i < h->n_occ; ++i) {
      int64_t row = h->g_off[i];
      for (int x : h->nbr[i]) {
        nb.push_back(x);
        for (int mu = 0; mu < h->r[x]; ++mu, ++row) {
          rl[(size_t)row] = i;
          rx[(size_t)row] = x;
        }
      }
      noff[(size_t)i + 1] = (int32_t)nb.size();
    }
    if ((rc = upload(h, &h->d_k_off, h->k_off)) ||
        (rc = upload(h, &h->d_row_lmo, rl)) || (rc = upload(h, &h->d_row_x, rx)) ||
        (rc = upload(h, &h->d_nbr_off, noff)) || (rc = upload(h, &h->d_nbr, nb)))
      return rc;
  }
  const int64_t nq = h->q_off[h->n_occ];
  if ((rc = dev_alloc(h, &h->eq, nq * nv))) return rc;
  if ((rc = dev_alloc(h, &h->sstore, h->sb_total))) return rc;
  if ((rc = dev_alloc(h, &h->fstore, h->sb_total))) return rc;
  if ((rc = dev_alloc(h, &h->ps, h->k_elems))) return rc;
  if ((rc = dev_alloc(h, &h->pf, h->k_elems))) return rc;
  const int64_t nx = h->x_off[h->n_slot], nkt = h->kt_off[h->n_slot];
  if ((rc = dev_alloc(h, &h->x0, nx))) return rc;
  if ((rc = dev_alloc(h, &h->xb, nx))) return rc;
  if ((rc = dev_alloc(h, &h->tmp, nx))) return rc;
  if ((rc = dev_alloc(h, &h->fp, nkt))) return rc;
  if ((rc = dev_alloc(h, &h->zb, nkt))) return rc;
  if ((rc = dev_alloc(h, &h->kt, nkt))) return rc;
  if ((rc = dev_alloc(h, &h->et, h->et_off[h->n_slot]))) return rc;
  if ((rc = dev_alloc(h, &h->ev0, h->et_off[h->n_slot]))) return rc;
  if ((rc = dev_alloc(h, &h->rank, h->n_slot))) return rc;
  if ((rc = dev_alloc(h, &h->sflag, h->n_slot))) return rc;
  if ((rc = dev_alloc(h, &h->cws, h->cws_doubles))) return rc;
  if ((rc = dev_alloc(h, &h->eig_meta, 4 * h->n_slot))) return rc;
  if ((rc = dev_alloc(h, &h->eig_redo, h->n_slot))) return rc;
  if (h->warm_start && (rc = dev_alloc(h, &h->warm, h->kt_off[h->n_slot]))) return rc;
  {
    const int md = max_d(h), nl = eig_lds_max_order();
    if (md > nl) {
      int64_t n_large = 0;
      for (int64_t sl = 0; sl < h->n_slot; ++sl) n_large += h->sd[sl] > nl;
      h->eig_ws_doubles = std::min<int64_t>(n_large, 1024) * eig_workspace_doubles(md);
      if ((rc = dev_alloc(h, &h->eig_ws, h->eig_ws_doubles))) return rc;
    }
  }
  int ny_max = 0, dmax = 16;
  for (auto &c : h->chunks) {
    ny_max = std::max(ny_max, c.ny_max);
    dmax = std::max(dmax, c.dmax);
  }
  h->scratch_stride = solve_scratch_doubles(ny_max, dmax);
  h->scratch_stride = (h->scratch_stride + 31) & ~31LL;
  if ((rc = dev_alloc(h, &h->scratch, h->scratch_stride * SOLVE_WG))) return rc;
  if ((rc = dev_alloc(h, &h->status, 2 * SOLVE_WG))) return rc;
  if ((rc = dev_alloc(h, &h->d_e3, 4))) return rc;
  if (h->dry) return MBE3_OK;
  HIP_TRY(h, hipHostMalloc((void **)&h->h_status, 2 * SOLVE_WG * sizeof(int32_t)));
  HIP_TRY(h, hipHostMalloc((void **)&h->h_e3, 4 * sizeof(double)));
  return MBE3_OK;
}

GemmBases bases(mbe3_handle *h) {
  GemmBases b;
  std::memset(&b, 0, sizeof b);
  b.p[B_Q] = const_cast<double *>(h->Q);
  b.p[B_EQ] = h->eq;
  b.p[B_SLAB] = h->slab ? const_cast<double *>(h->slab) : h->slab_buf;
  b.p[B_SS] = h->sstore;
  b.p[B_FS] = h->fstore;
  b.p[B_PS] = h->ps;
  b.p[B_PF] = h->pf;
  b.p[B_X0] = h->x0;
  b.p[B_X] = h->xb;
  b.p[B_TMP] = h->tmp;
  b.p[B_FP] = h->fp;
  b.p[B_Z] = h->zb;
  b.p[B_KT] = h->kt;
  b.p[B_AT] = h->at;
  b.p[B_MT] = h->mt;
  b.p[B_ST0] = h->st0;
  b.p[B_CA] = h->ca;
  b.p[B_CM] = h->cm;
  b.p[B_ST1] = h->st1;
  b.p[B_WT] = h->wt;
  b.p[B_GA] = h->ga;
  b.p[B_DG] = h->dg;
  b.rows = h->d_rows;
  return b;
}

int max_d(const mbe3_handle *h) {
  int m = 1;
  for (int64_t s = 0; s < h->n_slot; ++s) m = std::max(m, h->sd[s]);
  return m;
}

// Pair bases (Algorithm 5 blocks, eq. prec_eig) -- needs only Q and eps.
int prepare_bases(mbe3_handle *h) {
  PhaseScope ps_(h, MBE3_PHASE_BASES);
  hipStream_t s = h->stream;
  GemmBases b = bases(h);
  const int64_t nq = h->q_off[h->n_occ];
  HIP_TRY(h, launch_scale_rows(h->eq, h->Q, h->eps, nq, h->n_vir, s));
  HIP_TRY(h, launch_list(h, h->L_sf, b, s));
  HIP_TRY(h, launch_assemble(h->d_asm_pair, h->n_asm_pair, h->sstore, h->fstore,
                             h->ps, h->pf, s));
  const int md = max_d(h);
  HIP_TRY(h, launch_cholesky(h->d_eig0, (int)h->n_slot, md, h->ps, h->x0, h->ev0,
                             h->rank, h->sflag, h->tau_S, h->eig_ws,
                             h->eig_ws_doubles, s));
  HIP_TRY(h, launch_eigh(h->d_eig0, (int)h->n_slot, md, h->ps, h->x0, h->ev0,
                           h->rank, 0, h->tau_S, h->sflag, h->eig_ws,
                           h->eig_ws_doubles, s));
  HIP_TRY(h, launch_list(h, h->L_m1, b, s));
  HIP_TRY(h, launch_list(h, h->L_fp, b, s));
  HIP_TRY(h, launch_eigh_split(h->d_eig1, (int)h->n_slot, md, h->fp, h->zb, h->et,
                                 h->rank, h->cws, h->eig_meta, h->eig_redo, h->eig_ws,
                                 h->eig_ws_doubles, s));
  HIP_TRY(h, launch_list(h, h->L_x, b, s));
  if (!h->recording) h->bases_done = true;  // replays do not set it
  return MBE3_OK;
}

// K~ = X^T K X and the pair-level S~ blocks.
int prepare_pairs(mbe3_handle *h, const double *K) {
  hipStream_t s = h->stream;
  int rc = prepare_bases(h);
  if (rc) return rc;
  PhaseScope ps_(h, MBE3_PHASE_PAIRS);
  GemmBases b = bases(h);
  b.p[B_K] = const_cast<double *>(K);
  HIP_TRY(h, launch_list(h, h->L_m2, b, s));
  HIP_TRY(h, launch_list(h, h->L_kt, b, s));
  HIP_TRY(h, launch_assemble(h->d_asm_st, h->n_asm_st, h->sstore, h->fstore, h->at,
                             nullptr, s));
  HIP_TRY(h, launch_list(h, h->L_stm, b, s));
  HIP_TRY(h, launch_list(h, h->L_st1, b, s));
  return MBE3_OK;
}

// Bounds of one GEMM task list against the buffer sizes sz[] (in doubles)
// and the row-gather table it uses.
int check_gemm_list(mbe3_handle *h, const std::string &name,
                    const std::vector<GemmTask> &ts, const int64_t *sz,
                    const std::vector<int32_t> &rows, GemmShape shape) {
  const int tm = gemm_tile_m(shape), tn = gemm_tile_n(shape);
  auto bad = [&](const std::string &what, size_t k) {
    return h->fail(MBE3_EINVAL, "internal plan check failed: %s task %zu", what.c_str(), k);
  };
  const int64_t n_rows = (int64_t)rows.size();
  int64_t tb = 0;
  for (size_t k = 0; k < ts.size(); ++k) {
    const GemmTask &t = ts[k];
    if (t.a_buf < 0 || t.a_buf >= B_COUNT || t.b_buf < 0 || t.b_buf >= B_COUNT ||
        t.c_buf < 0 || t.c_buf >= B_COUNT)
      return bad(name + " (buffer id)", k);
    if (t.M < 1 || t.N < 1 || t.K < 1) return bad(name + " (empty)", k);
    if (t.tile_begin != tb) return bad(name + " (tile prefix)", k);
    if (t.tiles_n != (t.N + tn - 1) / tn) return bad(name + " (tiles_n)", k);
    tb += (int64_t)((t.M + tm - 1) / tm) * t.tiles_n;
    auto rmax = [&](int32_t off, int n, int64_t &out) {
      if (off < 0) { out = n - 1; return true; }
      if ((int64_t)off + n > n_rows) return false;
      int64_t m = -1;
      for (int e = 0; e < n; ++e) {
        if (rows[off + e] < 0) return false;
        m = std::max<int64_t>(m, rows[off + e]);
      }
      out = m;
      return true;
    };
    int64_t amax, bmax, r;
    if (!t.transA) {
      if (t.lda < t.K || !rmax(t.a_rows, t.M, r)) return bad(name + " (A rows)", k);
      amax = t.a_off + r * t.lda + t.K - 1;
    } else {
      if (t.lda < t.M || !rmax(t.a_rows, t.K, r)) return bad(name + " (A^T rows)", k);
      amax = t.a_off + r * t.lda + t.M - 1;
    }
    if (!t.transB) {
      if (t.ldb < t.N || !rmax(t.b_rows, t.K, r)) return bad(name + " (B rows)", k);
      bmax = t.b_off + r * t.ldb + t.N - 1;
    } else {
      if (t.ldb < t.K || !rmax(t.b_rows, t.N, r)) return bad(name + " (B^T rows)", k);
      bmax = t.b_off + r * t.ldb + t.K - 1;
    }
    const int64_t cmax = t.c_off + (int64_t)(t.M - 1) * t.ldc + t.N - 1;
    if (t.ldc < t.N) return bad(name + " (ldc)", k);
    if (t.a_off < 0 || amax >= sz[t.a_buf]) return bad(name + " (A bounds)", k);
    if (t.b_off < 0 || bmax >= sz[t.b_buf]) return bad(name + " (B bounds)", k);
    if (t.c_off < 0 || cmax >= sz[t.c_buf]) return bad(name + " (C bounds)", k);
    if (t.ct_off >= 0) {
      const int64_t ctmax = t.ct_off + (int64_t)(t.N - 1) * t.ldct + t.M - 1;
      if (t.ldct < t.M || ctmax >= sz[t.c_buf]) return bad(name + " (C^T bounds)", k);
    }
  }
  return MBE3_OK;
}

// Sizes (doubles) of every GEMM base; caller buffers at their required size.
void base_sizes(const mbe3_handle *h, int64_t *sz) {
  const int64_t nv = h->n_vir, na = h->n_aux;
  for (int k = 0; k < B_COUNT; ++k) sz[k] = 0;
  sz[B_Q] = sz[B_EQ] = h->q_off[h->n_occ] * nv;
  // the FP64 slab tile buffer exists only for regenerated slabs in FP64
  const int64_t slabs = h->slab ? (int64_t)h->n_occ
                                : (h->precision == MBE3_FP64 ? (int64_t)h->slab_nb : 0);
  sz[B_SLAB] = slabs * nv * na;
  sz[B_GAMMA] = sz[B_DG] = h->gamma_rows * na;
  sz[B_K] = sz[B_PS] = sz[B_PF] = sz[B_W] = h->k_elems;
  sz[B_SS] = sz[B_FS] = h->sb_total;
  sz[B_X0] = sz[B_X] = sz[B_TMP] = h->x_off[h->n_slot];
  sz[B_FP] = sz[B_Z] = sz[B_KT] = sz[B_WT] = h->kt_off[h->n_slot];
  sz[B_AT] = h->at_total;
  sz[B_MT] = h->mt_total;
  sz[B_ST0] = h->st0_total;
  sz[B_CA] = h->max_ca;
  sz[B_CM] = h->max_cm;
  sz[B_ST1] = h->max_st1;
  sz[B_GA] = h->ga_total;
  sz[B_DB] = (int64_t)h->n_occ * nv * na;
}

// Bounds of registered list li (its own shape and row table).
int check_list(mbe3_handle *h, int li, const int64_t *sz) {
  if (li < 0) return MBE3_OK;
  const GemmList &L = h->glists[li];
  return check_gemm_list(h, L.name, L.host, sz, L.rows_table ? h->h_grows : h->h_rows,
                         L.shape);
}

// Host-side bounds check of every plan against the buffers it addresses,
// run before any kernel of the plan is launched.  A failure here is a bug in
// the planner, reported as MBE3_EINVAL.
// Bounds of a split-precision task list: A rows inside a plane of a_ps
// elements, B rows inside b_ps, C inside c_size; 16-byte aligned operands.
int check_mixed_list(mbe3_handle *h, const std::string &name,
                     const std::vector<MixedTask> &ts, int64_t a_ps,
                     int64_t b_ps, int64_t c_size, MixedShape shape) {
  auto bad = [&](const std::string &what, size_t k) {
    return h->fail(MBE3_EINVAL, "internal plan check failed: %s task %zu", what.c_str(), k);
  };
  const std::vector<int32_t> &rows = h->h_mrows;
  int64_t tb = 0;
  for (size_t k = 0; k < ts.size(); ++k) {
    const MixedTask &t = ts[k];
    if (t.M < 1 || t.N < 1 || t.K < 1) return bad(name + " (empty)", k);
    if (t.K % 8 || t.lda % 8 || t.ldb % 8 || t.a_off % 8 || t.b_off % 8 ||
        t.lda < t.K || t.ldb < t.K || t.ldc < t.N)
      return bad(name + " (alignment)", k);
    if (t.tile_begin != tb) return bad(name + " (tile prefix)", k);
    tb += mixed_tile_count(t, shape);
    auto rmax = [&](int32_t off, int n, int64_t &out) {
      if (off < 0) { out = n - 1; return true; }
      if ((int64_t)off + n > (int64_t)rows.size()) return false;
      int64_t m = -1;
      for (int e = 0; e < n; ++e) {
        if (rows[off + e] < 0) return false;
        m = std::max<int64_t>(m, rows[off + e]);
      }
      out = m;
      return true;
    };
    int64_t ra, rb;
    if (!rmax(t.a_rows, t.M, ra) || t.a_off + ra * t.lda + t.K > a_ps)
      return bad(name + " (A bounds)", k);
    if (!rmax(t.b_rows, t.N, rb) || t.b_off + rb * t.ldb + t.K > b_ps)
      return bad(name + " (B bounds)", k);
    if (t.c_off < 0 || t.c_off + (int64_t)(t.M - 1) * t.ldc + t.N > c_size)
      return bad(name + " (C bounds)", k);
  }
  return MBE3_OK;
}

int validate_plans(mbe3_handle *h) {
  int64_t sz[B_COUNT];
  base_sizes(h, sz);
  if (h->precision != MBE3_FP64) {
    for (auto &pl : h->h_mixed) {
      const bool proj = pl.first[0] == 'p' && pl.first[1] == 'r';
      const int rc = proj ? check_mixed_list(h, pl.first, pl.second, h->q_ps, h->s_ps,
                                             h->gamma_rows * h->n_aux, MIXED_64x128)
                          : check_mixed_list(h, pl.first, pl.second, h->g_ps, h->g_ps,
                                             h->k_elems, MIXED_32x64);
      if (rc) return rc;
    }
  }
  auto bad = [&](const std::string &what, size_t k) {
    return h->fail(MBE3_EINVAL, "internal plan check failed: %s task %zu", what.c_str(), k);
  };
  for (size_t li = 0; li < h->glists.size(); ++li) {
    const int rc = check_list(h, (int)li, sz);
    if (rc) return rc;
  }
  for (auto &pl : h->h_asm) {
    for (size_t k = 0; k < pl.second.size(); ++k) {
      const AssembleTask &t = pl.second[k];
      const int64_t ob = pl.first[t.out_buf ? 1 : 0];
      if (ob < 0 || ob >= B_COUNT) return bad("assemble (out id)", k);
      if (t.ld_out < t.cols_out || t.rows_out < 1 || t.cols_out < 1)
        return bad("assemble (shape)", k);
      if (t.out_off < 0 || t.out_off + (int64_t)(t.rows_out - 1) * t.ld_out + t.cols_out - 1 >= sz[ob])
        return bad("assemble (out bounds)", k);
      if (t.nrb < 1 || t.nrb > 2 || t.ncb < 1 || t.ncb > 2) return bad("assemble (blocks)", k);
      for (int a = 0; a < t.nrb; ++a)
        for (int c = 0; c < t.ncb; ++c) {
          const BlockSrc &b = t.b[a][c];
          const int64_t last = b.trans ? b.off + (int64_t)(t.csz[c] - 1) * b.ld + t.rsz[a] - 1
                                       : b.off + (int64_t)(t.rsz[a] - 1) * b.ld + t.csz[c] - 1;
          if (b.off < 0 || last >= h->sb_total) return bad("assemble (source bounds)", k);
        }
    }
  }
  const int md = max_d(h);
  for (auto &pl : h->h_eig) {
    for (size_t k = 0; k < pl.second.size(); ++k) {
      const EigTask &t = pl.second[k];
      if (t.slot < 0 || t.slot >= h->n_slot || t.n > md || t.n > t.D) return bad("eigen (shape)", k);
      if (t.e_off < 0 || t.e_off + t.D > h->et_off[h->n_slot]) return bad("eigen (values)", k);
      if (pl.first == 0) {
        if (t.lda < t.n || t.a_off + (int64_t)(t.n - 1) * t.lda + t.n - 1 >= sz[B_PS])
          return bad("eigen (S input)", k);
        if (t.o_off + (int64_t)t.n * t.D > sz[B_X0]) return bad("eigen (X0 output)", k);
      } else {
        if (t.lda < t.D || t.a_off + (int64_t)(t.D - 1) * t.lda + t.D - 1 >= sz[B_FP])
          return bad("eigen (F input)", k);
        if (t.o_off + (int64_t)t.D * t.D > sz[B_Z]) return bad("eigen (Z output)", k);
        if (t.n <= eig_split_max_order() &&
            (t.w_off < 0 || t.w_off + eig_chase_ws_doubles(t.D) > h->cws_doubles))
          return bad("eigen (chase record)", k);
      }
    }
  }
  int dm = 16, nym = 0;
  for (auto &c : h->chunks) { dm = std::max(dm, c.dmax); nym = std::max(nym, c.ny_max); }
  const int64_t ny_cap = (h->scratch_stride - 2LL * dm * dm) / 4;
  if (dm > DMAX_SUPPORTED || nym > ny_cap) return bad("solve (scratch)", 0);
  for (size_t c = 0; c < h->h_fds.size(); ++c) {
    const auto &fds = h->h_fds[c];
    const auto &terms = h->h_terms[c];
    for (size_t k = 0; k < fds.size(); ++k) {
      const FragDesc &fd = fds[k];
      if (!(fd.nt == 1 || fd.nt == 3 || fd.nt == 6)) return bad("solve (nt)", k);
      if (fd.frag < 0 || fd.frag >= (int)h->frags.size()) return bad("solve (frag)", k);
      if (fd.term_begin < 0 || fd.term_end < fd.term_begin || fd.term_end > (int)terms.size())
        return bad("solve (terms)", k);
      if (fd.term_end - fd.term_begin > MAX_FRAG_TERMS) return bad("solve (term count)", k);
      for (int l = 0; l < fd.nt; ++l) {
        const int s = fd.slot[l];
        if (s < 0 || s >= h->n_slot) return bad("solve (slot)", k);
        const int D = h->sD[s];
        if (D > dm || fd.ysub[l] < 0 || fd.ysub[l] + D * D > fd.ny) return bad("solve (ysub)", k);
        if (h->kt_off[s] + (int64_t)D * D > sz[B_KT]) return bad("solve (K~)", k);
      }
      if (fd.ny > ny_cap) return bad("solve (ny)", k);
      for (int e = fd.term_begin; e < fd.term_end; ++e) {
        const Term &t = terms[e];
        if (t.target < 0 || t.target >= fd.nt || t.src < 0 || t.src >= fd.nt)
          return bad("solve (term slots)", k);
        if (t.fx < 0 || t.fx >= h->n_occ || t.fy < 0 || t.fy >= h->n_occ)
          return bad("solve (term f)", k);
        const int64_t dt = h->sD[fd.slot[t.target]], ds = h->sD[fd.slot[t.src]];
        const int64_t lim = t.st_buf ? sz[B_ST1] : sz[B_ST0];
        if (t.st_off < 0 || t.st_off + ds * dt > lim) return bad("solve (S~ bounds)", k);
      }
    }
  }
  return MBE3_OK;
}

// ---------------------------------------------------------------------------
// Gradient plans (built on the first call that asks for multipliers).
//   per chunk: W~ entries grouped by slot and f-gradient entries grouped by
//              destination f_xy, both in fragment order (deterministic);
//   W_s = X_s W~_s X_s^T for every slot;
//   dGamma~_{i,x} = GA_{i,x} [gathered Gamma~ rows], one product per
//              destination block, GA the concatenated multiplier segments;
//   dE/dB_i = sum_x Q_x dGamma~_{i,x} (gathered Q rows, transposed).
// ---------------------------------------------------------------------------
int build_grad_plans(mbe3_handle *h) {
  if (h->grad_planned) return MBE3_OK;
  if (h->recording)
    return h->fail(MBE3_EINVAL, "gradient plans allocate: start the recording with with_grad = 1");
  const int n = h->n_occ, na = h->n_aux, nv = h->n_vir;
  int rc;
  auto bad = [&](const char *what, size_t k) {
    return h->fail(MBE3_EINVAL, "internal plan check failed: gradient %s %zu", what, k);
  };
  int64_t ymax = 1, tmax = 1, gmax = 1;
  for (size_t c = 0; c < h->chunks.size(); ++c) {
    Chunk &ch = h->chunks[c];
    const auto &fds = h->h_fds[c];
    const auto &terms = h->h_terms[c];
    ymax = std::max(ymax, ch.ny_total);
    tmax = std::max<int64_t>(tmax, ch.n_terms);
    gmax = std::max<int64_t>(gmax, 6LL * ch.n_frag);
    std::map<int, std::vector<WEntry>> bs;
    std::map<int, std::vector<GEntry>> gs;
    for (size_t k = 0; k < fds.size(); ++k) {
      const FragDesc &fd = fds[k];
      for (int l = 0; l < fd.nt; ++l) {
        const int sl = fd.slot[l];
        const int64_t D = h->sD[sl];
        if (fd.yout < 0 || fd.yout + fd.ysub[l] + D * D > ch.ny_total) return bad("Y store", k);
        bs[sl].push_back({fd.yout + fd.ysub[l], fd.coef});
      }
      for (int e = fd.term_begin; e < fd.term_end; ++e) {
        const Term &t = terms[e];
        gs[t.fx * n + t.fy].push_back({-fd.coef * fd.wgt[t.target], 0, e});
      }
      // f_pp and f_qq inside E~ (both f_pp for a diagonal slot)
      for (int l = 0; l < fd.nt; ++l) {
        const int sl = fd.slot[l];
        const double sc = -fd.coef * fd.wgt[l];
        gs[h->sp[sl] * n + h->sp[sl]].push_back({sc, 1, (int32_t)(6 * k + l)});
        gs[h->sq[sl] * n + h->sq[sl]].push_back({sc, 1, (int32_t)(6 * k + l)});
      }
    }
    std::vector<WSlot> ws;
    std::vector<WEntry> we;
    for (auto &kv : bs) {
      // a slot found in many fragments is split over several work items by
      // element range (about 32 entries' worth of reads per 256 elements)
      const int D = h->sD[kv.first];
      const int nel = D * D;
      const int ne = (int)kv.second.size();
      const int pieces = std::max(1, std::min((ne + 31) / 32, (nel + 255) / 256));
      const int span = ((nel + pieces - 1) / pieces + 63) / 64 * 64;
      const int32_t eb = (int32_t)we.size();
      we.insert(we.end(), kv.second.begin(), kv.second.end());
      for (int y0 = 0; y0 < nel; y0 += span) {
        WSlot w;
        std::memset(&w, 0, sizeof w);
        w.wt_off = h->kt_off[kv.first] + y0;
        w.y0 = y0;
        w.n = std::min(span, nel - y0);
        w.e_begin = eb;
        w.e_end = (int32_t)we.size();
        ws.push_back(w);
      }
      // bounds: W~ block of the slot, each entry's Y~ block in the store
      if (h->kt_off[kv.first] + nel > h->kt_off[h->n_slot]) return bad("W~ slot", kv.first);
      for (const WEntry &e : kv.second)
        if (e.yoff < 0 || e.yoff + nel > ch.ny_total) return bad("W~ entry", kv.first);
    }
    std::vector<GDest> gd;
    std::vector<GEntry> ge;
    for (auto &kv : gs) {
      GDest d;
      std::memset(&d, 0, sizeof d);
      d.dst = kv.first;
      d.e_begin = (int32_t)ge.size();
      for (const GEntry &e : kv.second) {
        if (e.kind == 0 ? (e.idx < 0 || e.idx >= ch.n_terms)
                        : (e.idx < 0 || e.idx >= 6 * ch.n_frag))
          return bad("f entry", ge.size());
        ge.push_back(e);
      }
      d.e_end = (int32_t)ge.size();
      if (d.dst < 0 || d.dst >= n * n) return bad("f destination", gd.size());
      gd.push_back(d);
    }
    ch.n_ws = (int)ws.size();
    ch.n_gd = (int)gd.size();
    if ((rc = upload(h, &ch.d_ws, ws))) return rc;
    if ((rc = upload(h, &ch.d_we, we))) return rc;
    if ((rc = upload(h, &ch.d_gd, gd))) return rc;
    if ((rc = upload(h, &ch.d_ge, ge))) return rc;
  }
  h->yfin_max = ymax;
  h->gterm_max = tmax;
  h->gdiag_max = gmax;

  // ---- W_s = X_s W~_s X_s^T ----
  {
    std::vector<GemmTask> wm, ww;
    for (int64_t s = 0; s < h->n_slot; ++s) {
      const int d = h->sd[s], D = h->sD[s];
      wm.push_back(gemm(B_X, h->x_off[s], D, 0, B_WT, h->kt_off[s], D, 0, B_TMP,
                        h->x_off[s], D, d, D, D));
      ww.push_back(gemm(B_TMP, h->x_off[s], D, 0, B_X, h->x_off[s], D, 1, B_W,
                        h->k_off[s], d, d, d, D));
    }
    if ((rc = add_list(h, "W left", wm, GEMM_64x64, 0, &h->L_wm))) return rc;
    if ((rc = add_list(h, "W right", ww, GEMM_64x64, 0, &h->L_ww))) return rc;
  }
  // ---- dGamma~ per destination block (i, x) ----
  std::vector<int32_t> rows;
  std::vector<GASeg> segs;
  std::vector<GemmTask> dg, up;
  int64_t ga_total = 0;
  auto grows = [&](int i, int x) {  // rows of Gamma~_{i,x}
    const int64_t g0 = h->grow.at(key2(i, x));
    for (int mu = 0; mu < h->r[x]; ++mu) rows.push_back((int32_t)g0 + mu);
  };
  for (int i = 0; i < n; ++i) {
    for (int x : h->nbr[i]) {
      const int rx = h->r[x];
      // segments of this destination: (slot, rc0, mode, scale, right factor)
      struct Seg { int s, rc0, mode; double scale; int ra, xa, rb, xb; };
      std::vector<Seg> sl;
      auto add_pair = [&](int a, int b) {  // contribution through slot (a, b)
        const int s = slot_of(h, a, b);
        const int p = h->sp[s], q = h->sq[s];
        const int rc0 = (x == i) ? (i == p ? 0 : h->r[p]) : (i == p ? h->r[p] : 0);
        if (i == p)  // dL = G R, R = [Gamma~_{q,p}; Gamma~_{q,q}]
          sl.push_back({s, rc0, 0, 4.0, q, p, q, q});
        else         // dR = G^T L, L = [Gamma~_{p,p}; Gamma~_{p,q}]
          sl.push_back({s, rc0, 1, 4.0, p, p, p, q});
      };
      if (x == i) {
        sl.push_back({i, 0, 2, 2.0, i, i, -1, -1});  // K_ii = G~ G~^T
        for (int q : h->nbr[i])
          if (q != i) add_pair(i, q);
      } else {
        add_pair(i, x);
      }
      const int32_t brow = (int32_t)rows.size();
      const size_t seg0 = segs.size();
      int ktot = 0;
      for (const Seg &g : sl) {
        const int d = h->sd[g.s];
        GASeg a;
        std::memset(&a, 0, sizeof a);
        a.w_off = h->k_off[g.s];
        a.w_ld = d;
        a.ga_off = ga_total;
        a.rc0 = g.rc0;
        a.k0 = ktot;
        a.rows = rx;
        a.kseg = d;
        a.mode = g.mode;
        a.scale = g.scale;
        segs.push_back(a);
        grows(g.ra, g.xa);
        if (g.rb >= 0) grows(g.rb, g.xb);
        ktot += d;
      }
      for (size_t k = seg0; k < segs.size(); ++k) segs[k].ga_ld = ktot;
      if ((int)rows.size() - brow != ktot) return bad("gather rows", (size_t)i);
      GemmTask t = gemm(B_GA, ga_total, ktot, 0, B_GAMMA, 0, na, 0, B_DG,
                        h->grow.at(key2(i, x)) * na, na, rx, na, ktot);
      t.b_rows = brow;
      dg.push_back(t);
      ga_total += (int64_t)rx * ktot;
    }
    // dE/dB_i = [Q_x ...] dGamma~_i
    GemmTask t = gemm(B_Q, 0, nv, 1, B_DG, h->g_off[i] * na, na, 0, B_DB,
                      (int64_t)i * nv * na, na, nv, na,
                      (int)(h->g_off[i + 1] - h->g_off[i]));
    t.a_rows = (int32_t)rows.size();
    for (int x : h->nbr[i])
      for (int mu = 0; mu < h->r[x]; ++mu) rows.push_back((int32_t)(h->q_off[x] + mu));
    up.push_back(t);
  }
  h->ga_total = std::max<int64_t>(1, ga_total);
  h->n_ga = (int)segs.size();
  if ((rc = add_list(h, "dGamma", dg, GEMM_64x64, 1, &h->L_dg))) return rc;
  if ((rc = add_list(h, "unproject", up, GEMM_128x128, 1, &h->L_up))) return rc;
  if ((rc = upload(h, &h->d_ga, segs))) return rc;
  if ((rc = upload(h, &h->d_grows, rows))) return rc;
  h->h_grows = rows;

  // ---- bounds ----
  int64_t sz[B_COUNT];
  base_sizes(h, sz);
  for (int li : {h->L_wm, h->L_ww, h->L_dg, h->L_up})
    if ((rc = check_list(h, li, sz))) return rc;
  for (size_t k = 0; k < segs.size(); ++k) {
    const GASeg &a = segs[k];
    if (a.rows < 1 || a.kseg < 1 || a.k0 + a.kseg > a.ga_ld) return bad("segment shape", k);
    if (a.ga_off + (int64_t)(a.rows - 1) * a.ga_ld + a.k0 + a.kseg > h->ga_total)
      return bad("segment output", k);
    int64_t last;
    if (a.mode == 0) last = (int64_t)(a.rc0 + a.rows - 1) * a.w_ld + a.kseg - 1;
    else if (a.mode == 1) last = (int64_t)(a.kseg - 1) * a.w_ld + a.rc0 + a.rows - 1;
    else {
      if (a.rc0 != 0 || a.rows != a.kseg) return bad("segment symmetric", k);
      last = (int64_t)(a.kseg - 1) * a.w_ld + a.kseg - 1;
    }
    if (a.rc0 + a.rows > a.w_ld || a.w_off + last >= h->k_elems) return bad("segment input", k);
  }

  // ---- buffers ----
  if ((rc = dev_alloc(h, &h->wt, h->kt_off[h->n_slot]))) return rc;
  if ((rc = dev_alloc(h, &h->yfin, ymax))) return rc;
  if ((rc = dev_alloc(h, &h->gterm, tmax))) return rc;
  if ((rc = dev_alloc(h, &h->gdiag, gmax))) return rc;
  if ((rc = dev_alloc(h, &h->graw, (int64_t)n * n))) return rc;
  if ((rc = dev_alloc(h, &h->ga, h->ga_total))) return rc;
  if ((rc = dev_alloc(h, &h->dg, h->gamma_rows * na))) return rc;
  if ((rc = dev_alloc(h, &h->dot_part, 2LL * dot_partials()))) return rc;
  if ((rc = dev_alloc(h, &h->d_probe, 2))) return rc;
  if (!h->dry)
    HIP_TRY(h, hipHostMalloc((void **)&h->h_probe, 2 * sizeof(double)));
  h->grad_planned = true;
  return MBE3_OK;
}

}  // namespace

// ===========================================================================
// C-ABI
// ===========================================================================
static thread_local std::string g_create_error = "no handle";

// Status words of the last solve (host copy already synchronised).
int solve_status(mbe3_handle *h) {
  int bad = 0, nconv = 0;
  for (int k = 0; k < SOLVE_WG; ++k) {
    bad |= h->h_status[2 * k];
    nconv |= h->h_status[2 * k + 1];
  }
  if (bad) return h->fail(MBE3_ENONFINITE, "non-finite residual in some fragment (e_frag = NaN)");
  if (nconv) return h->fail(MBE3_ENOCONV, "some fragment did not converge in %d updates (iters < 0)",
                            h->max_iter);
  return MBE3_OK;
}

void release_graph(mbe3_handle *h) {
  for (auto &sg : h->segs) {
    if (sg.x) (void)hipGraphExecDestroy(sg.x);
    if (sg.g) (void)hipGraphDestroy(sg.g);
  }
  h->segs.clear();
  h->g_solve = h->g_grad = h->g_energy = false;
}

// Device memory of one call, released (after the stream has drained) when
// the call returns.
struct CallTemp {
  mbe3_handle *h;
  std::vector<void *> ps;
  explicit CallTemp(mbe3_handle *hh) : h(hh) {}
  ~CallTemp() {
    if (ps.empty()) return;
    (void)hipStreamSynchronize(h->stream);
    for (void *p : ps) (void)hipFree(p);
  }
  template <class T>
  int alloc(T **p, int64_t n) {
    void *q = nullptr;
    const hipError_t e = hipMalloc(&q, (size_t)std::max<int64_t>(n, 1) * sizeof(T));
    if (e != hipSuccess) {
      (void)hipGetLastError();
      return h->fail(MBE3_ENOMEM, "hipMalloc of %lld bytes failed: %s",
                     (long long)(n * (int64_t)sizeof(T)), hipGetErrorString(e));
    }
    ps.push_back(q);
    *p = (T *)q;
    return MBE3_OK;
  }
  template <class T>
  int upload(T **p, const std::vector<T> &v) {
    const int rc = alloc(p, (int64_t)v.size());
    if (rc || v.empty()) return rc;
    HIP_TRY(h, hipMemcpy(*p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice));
    return MBE3_OK;
  }
};

// Pairs of a screening / weak-pair call, checked and laid out: r_i x r_j
// blocks, D_i x D_j blocks and the X_i^T (.) temporaries (D_i x r_j).
static int weak_layout(mbe3_handle *h, const int32_t *pairs, int64_t n, bool ordered,
                       std::vector<WeakPair> &wp, int64_t *k_tot, int64_t *t_tot,
                       int64_t *p_tot, std::vector<int64_t> &p_off) {
  if (n > 0x7fffffffLL / 4) return h->fail(MBE3_EINVAL, "too many pairs (%lld)", (long long)n);
  wp.resize(n);
  p_off.resize(n);
  int64_t ko = 0, to = 0, po = 0;
  for (int64_t k = 0; k < n; ++k) {
    const int i = pairs[2 * k], j = pairs[2 * k + 1];
    if (i < 0 || j < 0 || i >= h->n_occ || j >= h->n_occ || i == j || (ordered && i > j))
      return h->fail(MBE3_EINVAL, "pair %lld (%d, %d) is not %s", (long long)k, i, j,
                     ordered ? "0 <= i < j < n_occ" : "two distinct LMOs");
    WeakPair w;
    w.i = i; w.j = j; w.ri = h->r[i]; w.rj = h->r[j];
    w.Di = h->sD[i]; w.Dj = h->sD[j];  // the diagonal slots i and j
    w.k_off = ko; w.t_off = to;
    w.ei = h->et_off[i]; w.ej = h->et_off[j];
    wp[k] = w;
    p_off[k] = po;
    ko += (int64_t)w.ri * w.rj;
    to += (int64_t)w.Di * w.Dj;
    po += (int64_t)w.Di * w.rj;
  }
  *k_tot = ko; *t_tot = to; *p_tot = po;
  return MBE3_OK;
}

// One call-time task list: bounds-checked against sz, tiled, uploaded and
// launched on the handle's stream.
static int run_call_list(mbe3_handle *h, CallTemp &tmp, const char *name,
                         std::vector<GemmTask> &ts, const int64_t *sz, const GemmBases &b,
                         GemmShape shape) {
  if (ts.empty()) return MBE3_OK;
  const int64_t tiles = finish_tasks(ts, shape);
  int rc = check_gemm_list(h, name, ts, sz, std::vector<int32_t>(), shape);
  if (rc) return rc;
  GemmTask *d = nullptr;
  if ((rc = tmp.upload(&d, ts))) return rc;
  HIP_TRY(h, launch_gemm_tasks(d, (int)ts.size(), tiles, b, shape, h->stream));
  return MBE3_OK;
}

// No C++ exception crosses the C-ABI: host-side planning (containers, map
// lookups) runs inside this guard, which turns one into a status.
template <class F>
static int no_throw(mbe3_handle *h, F &&f) {
  try {
    return f();
  } catch (const std::bad_alloc &) {
    return h->fail(MBE3_ENOMEM, "host allocation failed");
  } catch (const std::exception &e) {
    return h->fail(MBE3_EINVAL, "internal error: %s", e.what());
  } catch (...) {
    return h->fail(MBE3_EINVAL, "internal error");
  }
}

extern "C" {

// ---- scratch of the allocation-free entry point (mbe3_screen_noalloc) ----
// A fixed device array in the library's code object: every GPU the library
// runs on holds its own copy until the process ends.  In host code the
// array's name is not a device address; each device's address comes from
// hipGetSymbolAddress (with that device current), once, and only that
// address is ever handed to kernels or copies.
static constexpr size_t SCRATCH_BYTES = (size_t)64 << 20;  // 64 MiB
static __device__ __align__(256) unsigned char scratch[SCRATCH_BYTES];
static std::mutex g_scratch_mu;
static constexpr int SCRATCH_MAX_DEV = 64;
static unsigned char *g_scratch_dev[SCRATCH_MAX_DEV];

static int scratch_init(mbe3_handle *h) {
  int dev = 0;
  HIP_TRY(h, hipGetDevice(&dev));
  if (dev < 0 || dev >= SCRATCH_MAX_DEV)
    return h->fail(MBE3_EINVAL, "device %d beyond the scratch table", dev);
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_dev[dev]) {
    void *p = nullptr;
    HIP_TRY(h, hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    g_scratch_dev[dev] = (unsigned char *)p;
  }
  h->noalloc_scratch = g_scratch_dev[dev];
  return MBE3_OK;
}

static int64_t align256(int64_t b) { return (b + 255) / 256 * 256; }

// mbe3_screen with every buffer (task table, pair table, overlap blocks) in
// the device's scratch array instead of per-call allocations.
static int screen_noalloc_body(mbe3_handle *h, const int32_t *pairs, int64_t n,
                               double *s2b) {
  if (h->recording) return h->fail(MBE3_EINVAL, "mbe3_screen_noalloc synchronises: not recordable");
  if (!h->noalloc_scratch) return h->fail(MBE3_EINVAL, "scratch not initialised on this handle");
  if (n < 0 || (n > 0 && (!pairs || !s2b)))
    return h->fail(MBE3_EINVAL, "pairs and s2b required for n > 0");
  if (n == 0) return MBE3_OK;
  std::vector<WeakPair> wp;
  std::vector<int64_t> p_off;
  int64_t ko, to, po;
  int rc = weak_layout(h, pairs, n, false, wp, &ko, &to, &po, p_off);
  if (rc) return rc;
  const int nv = h->n_vir;
  std::vector<GemmTask> ts;
  for (const WeakPair &w : wp)  // S_(i,j) = Q_i^T Q_j (rows of the packed Q)
    ts.push_back(gemm(B_Q, h->q_off[w.i] * nv, nv, 0, B_Q, h->q_off[w.j] * nv, nv, 1,
                      B_PS2, w.k_off, w.rj, w.ri, w.rj, nv));
  const int64_t tiles = finish_tasks(ts, GEMM_32x32);
  int64_t sz[B_COUNT];
  base_sizes(h, sz);
  sz[B_PS2] = ko;
  if ((rc = check_gemm_list(h, "screen S (no alloc)", ts, sz, std::vector<int32_t>(),
                            GEMM_32x32)))
    return rc;
  const int64_t off_wp = align256((int64_t)(ts.size() * sizeof(GemmTask)));
  const int64_t off_s = align256(off_wp + n * (int64_t)sizeof(WeakPair));
  const int64_t need = off_s + ko * (int64_t)sizeof(double);
  if (need > (int64_t)SCRATCH_BYTES)
    return h->fail(MBE3_EINVAL,
                   "mbe3_screen_noalloc: %lld pairs need %lld bytes of scratch, the "
                   "library holds %lld; pass fewer pairs per call",
                   (long long)n, (long long)need, (long long)SCRATCH_BYTES);
  hipStream_t st = h->stream;
  GemmTask *d_ts = (GemmTask *)h->noalloc_scratch;
  WeakPair *d_wp = (WeakPair *)(h->noalloc_scratch + off_wp);
  double *S = (double *)(h->noalloc_scratch + off_s);
  HIP_TRY(h, hipMemcpyAsync(d_ts, ts.data(), ts.size() * sizeof(GemmTask),
                            hipMemcpyHostToDevice, st));
  HIP_TRY(h, hipMemcpyAsync(d_wp, wp.data(), wp.size() * sizeof(WeakPair),
                            hipMemcpyHostToDevice, st));
  GemmBases b = bases(h);
  b.p[B_PS2] = S;
  HIP_TRY(h, launch_gemm_tasks(d_ts, (int)ts.size(), tiles, b, GEMM_32x32, st));
  HIP_TRY(h, launch_s2b(d_wp, (int)n, S, s2b, st));
  // the host tables stay alive until the copies have run
  HIP_TRY(h, hipStreamSynchronize(st));
  return MBE3_OK;
}

int mbe3_screen_noalloc(mbe3_handle *h, const int32_t *pairs, int64_t n, double *s2b) {
  if (!h) return MBE3_EINVAL;
  return no_throw(h, [&] { return screen_noalloc_body(h, pairs, n, s2b); });
}

int64_t mbe3_screen_noalloc_max_bytes(void) { return (int64_t)SCRATCH_BYTES; }

int mbe3_create(mbe3_handle **out, const mbe3_problem *p, void *stream) {
  if (!out) return MBE3_EINVAL;
  *out = nullptr;
  mbe3_handle *h = new (std::nothrow) mbe3_handle();
  if (!h) return MBE3_ENOMEM;
  h->stream = (hipStream_t)stream;
  int rc = no_throw(h, [&] {
    int r = validate_and_copy(h, p);
    if (!r) r = build_layout(h);
    if (!r) r = build_plans(h);
    if (!r) r = alloc_workspace(h);
    if (!r) r = validate_plans(h);
    if (!r) r = scratch_init(h);
    return r;
  });
  if (rc) {
    g_create_error = h->err;
    delete h;
    return rc;
  }
  *out = h;
  return MBE3_OK;
}

int mbe3_plan_check(const mbe3_problem *p, mbe3_layout *out) {
  mbe3_handle *h = new (std::nothrow) mbe3_handle();
  if (!h) return MBE3_ENOMEM;
  h->dry = true;
  int rc = no_throw(h, [&] {
    int r = validate_and_copy(h, p);
    if (!r) r = build_layout(h);
    if (!r) r = build_plans(h);
    if (!r) r = alloc_workspace(h);
    if (!r) r = validate_plans(h);
    if (!r) r = build_grad_plans(h);
    return r;
  });
  // every tile shape mbe3_autotune may choose keeps every task in bounds
  for (int sh = 0; sh < GEMM_NSHAPE && !rc; ++sh) rc = mbe3_set_gemm_shape(h, -1, sh);
  if (!rc && out) mbe3_get_layout(h, out);
  g_create_error = rc ? h->err : std::string("ok");
  delete h;
  return rc;
}

// Pair classes and trimer screening (section on OSV overlap and Fock
// computation, eqs. s2b and s3b): host logic only, no handle.
int mbe3_screen_lists(int32_t n_occ, const int32_t *pairs, int64_t n, const double *s2b,
                      double t_distant, double t_close, double t_trimer, int8_t *cls,
                      int32_t *close_pairs, int64_t *n_close, int32_t *weak_pairs,
                      int64_t *n_weak, int32_t *trimers, int64_t tri_cap, int64_t *n_tri) {
  auto fail = [](const char *fmt, long long a, long long b) {
    char buf[256];
    snprintf(buf, sizeof buf, fmt, a, b);
    g_create_error = buf;
    return MBE3_EINVAL;
  };
  if (n_occ < 1 || n < 0 || (n > 0 && (!pairs || !s2b)) || !n_close || !n_weak || !n_tri)
    return fail("mbe3_screen_lists: bad arguments (n_occ %lld, n %lld)", n_occ, n);
  try {
    // normalised (i < j) pairs with their metric, keyed for lookup
    std::unordered_map<int64_t, double> close_s2b;
    std::vector<std::array<int32_t, 2>> cl, wk;
    std::unordered_map<int64_t, int64_t> seen;
    for (int64_t k = 0; k < n; ++k) {
      int32_t i = pairs[2 * k], j = pairs[2 * k + 1];
      if (i > j) std::swap(i, j);
      if (i < 0 || j >= n_occ || i == j)
        return fail("mbe3_screen_lists: pair %lld (%lld) out of range or repeated orbital",
                    k, (long long)pairs[2 * k]);
      const int64_t key = (int64_t)i * n_occ + j;
      if (!seen.emplace(key, k).second)
        return fail("mbe3_screen_lists: pair %lld repeats pair %lld", k, seen[key]);
      const double v = s2b[k];
      if (!std::isfinite(v))
        return fail("mbe3_screen_lists: s2b[%lld] of pair %lld is not finite", k, k);
      const int8_t c = v < t_distant ? 0 : (v < t_close ? 1 : 2);
      if (cls) cls[k] = c;
      if (c == 2) {
        cl.push_back({i, j});
        close_s2b[key] = v;
      } else if (c == 1) {
        wk.push_back({i, j});
      }
    }
    std::sort(cl.begin(), cl.end());
    std::sort(wk.begin(), wk.end());
    *n_close = (int64_t)cl.size();
    *n_weak = (int64_t)wk.size();
    if (close_pairs)
      for (size_t k = 0; k < cl.size(); ++k) {
        close_pairs[2 * k] = cl[k][0];
        close_pairs[2 * k + 1] = cl[k][1];
      }
    if (weak_pairs)
      for (size_t k = 0; k < wk.size(); ++k) {
        weak_pairs[2 * k] = wk[k][0];
        weak_pairs[2 * k + 1] = wk[k][1];
      }
    // trimers of three close pairs whose mean metric (eq. s3b) reaches t_trimer
    std::vector<std::vector<int32_t>> up((size_t)n_occ);  // close partners above i
    for (auto &pq : cl) up[(size_t)pq[0]].push_back(pq[1]);
    int64_t nt = 0;
    for (auto &pq : cl) {
      const int32_t i = pq[0], j = pq[1];
      const double sij = close_s2b[(int64_t)i * n_occ + j];
      for (int32_t k : up[(size_t)j]) {  // k > j, (j, k) close
        const auto ik = close_s2b.find((int64_t)i * n_occ + k);
        if (ik == close_s2b.end()) continue;
        const double sjk = close_s2b[(int64_t)j * n_occ + k];
        if ((sij + ik->second + sjk) / 3.0 >= t_trimer) {
          if (trimers) {
            if (nt >= tri_cap)
              return fail("mbe3_screen_lists: trimer %lld exceeds tri_cap = %lld", nt, tri_cap);
            trimers[3 * nt] = i;
            trimers[3 * nt + 1] = j;
            trimers[3 * nt + 2] = k;
          }
          ++nt;
        }
      }
    }
    *n_tri = nt;
  } catch (const std::bad_alloc &) {
    g_create_error = "mbe3_screen_lists: host allocation failed";
    return MBE3_ENOMEM;
  }
  g_create_error = "ok";
  return MBE3_OK;
}

// Pipek-Mezey localization with Jacobi sweeps (Alg. 2): no handle; errors
// through mbe3_last_error(NULL).
int mbe3_pm_localize(const double *C, const int32_t *ao_off, int32_t n_ao, int32_t n_occ,
                     int32_t n_atom, double l_loc, int32_t max_sweeps, double *P, double *U,
                     double *dL, int32_t *rotations, int32_t *sweeps, void *stream) {
  auto fail = [](int code, const char *msg) {
    g_create_error = msg;
    return code;
  };
  if (!C || !ao_off || !P || !U || !sweeps)
    return fail(MBE3_EINVAL, "mbe3_pm_localize: C, ao_off, P, U and sweeps are required");
  if (n_ao < 1 || n_occ < 1 || n_atom < 1 || max_sweeps < 1 || std::isnan(l_loc))
    return fail(MBE3_EINVAL, "mbe3_pm_localize: sizes and max_sweeps must be positive");
  if (ao_off[0] != 0 || ao_off[n_atom] != n_ao)
    return fail(MBE3_EINVAL, "mbe3_pm_localize: ao_off must run from 0 to n_ao");
  for (int A = 0; A < n_atom; ++A)
    if (ao_off[A + 1] < ao_off[A])
      return fail(MBE3_EINVAL, "mbe3_pm_localize: ao_off must not decrease");
  hipStream_t st = (hipStream_t)stream;
  int32_t *d_off = nullptr;
  double *d_rec = nullptr;
  auto release = [&] {
    if (d_off) (void)hipFree(d_off);
    if (d_rec) (void)hipFree(d_rec);
  };
  std::vector<double> rec((size_t)2 * max_sweeps + 1, 0.0);
  hipError_t e = hipMalloc((void **)&d_off, sizeof(int32_t) * ((size_t)n_atom + 1));
  if (e == hipSuccess) e = hipMalloc((void **)&d_rec, sizeof(double) * rec.size());
  if (e != hipSuccess) {
    (void)hipGetLastError();
    release();
    return fail(MBE3_ENOMEM, "mbe3_pm_localize: device allocation failed");
  }
  if (e == hipSuccess)
    e = hipMemcpyAsync(d_off, ao_off, sizeof(int32_t) * ((size_t)n_atom + 1),
                       hipMemcpyHostToDevice, st);
  if (e == hipSuccess) e = launch_pm_charges(C, d_off, n_occ, n_atom, P, st);
  if (e == hipSuccess) e = launch_pm_jacobi(P, U, n_occ, n_atom, l_loc, max_sweeps, d_rec, st);
  if (e == hipSuccess)
    e = hipMemcpyAsync(rec.data(), d_rec, sizeof(double) * rec.size(), hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  release();
  if (e != hipSuccess) {
    static thread_local char buf[256];
    snprintf(buf, sizeof buf, "mbe3_pm_localize: %s", hipGetErrorString(e));
    return fail(MBE3_EHIP, buf);
  }
  const int ns = (int)rec[2 * (size_t)max_sweeps];
  *sweeps = ns;
  for (int k = 0; k < ns; ++k) {
    if (dL) dL[k] = rec[2 * (size_t)k];
    if (rotations) rotations[k] = (int32_t)rec[2 * (size_t)k + 1];
  }
  if (ns > 0 && !std::isfinite(rec[2 * (size_t)(ns - 1)]))
    return fail(MBE3_ENONFINITE, "mbe3_pm_localize: non-finite increment");
  if (ns > 0 && rec[2 * (size_t)(ns - 1)] > l_loc)
    return fail(MBE3_ENOCONV, "mbe3_pm_localize: max_sweeps reached above l_loc");
  g_create_error = "ok";
  return MBE3_OK;
}

int mbe3_destroy(mbe3_handle *h) {
  if (!h) return MBE3_EINVAL;
  if (h->recording) {
    hipGraph_t g = nullptr;
    (void)hipStreamEndCapture(h->cap_stream, &g);
    if (g) (void)hipGraphDestroy(g);
    h->stream = h->user_stream;
    h->recording = false;
  }
  (void)hipStreamSynchronize(h->stream);
  delete h;
  return MBE3_OK;
}

const char *mbe3_last_error(const mbe3_handle *h) {
  if (!h) return g_create_error.c_str();
  return h->err.c_str();
}

int mbe3_get_layout(const mbe3_handle *h, mbe3_layout *o) {
  if (!h || !o) return MBE3_EINVAL;
  o->n_slot = h->n_slot;
  o->gamma_rows = h->gamma_rows;
  o->gamma_elems = h->gamma_rows * h->n_aux;
  o->k_elems = h->k_elems;
  o->n_frag = (int64_t)h->frags.size();
  return MBE3_OK;
}

int mbe3_gamma_offsets(const mbe3_handle *h, int64_t *o) {
  if (!h || !o) return MBE3_EINVAL;
  std::memcpy(o, h->g_off.data(), h->g_off.size() * sizeof(int64_t));
  return MBE3_OK;
}

int mbe3_k_offsets(const mbe3_handle *h, int64_t *o) {
  if (!h || !o) return MBE3_EINVAL;
  std::memcpy(o, h->k_off.data(), h->k_off.size() * sizeof(int64_t));
  return MBE3_OK;
}

int mbe3_basis_offsets(const mbe3_handle *h, int64_t *xoff, int64_t *eoff) {
  if (!h || !xoff || !eoff) return MBE3_EINVAL;
  std::memcpy(xoff, h->x_off.data(), h->x_off.size() * sizeof(int64_t));
  std::memcpy(eoff, h->et_off.data(), h->et_off.size() * sizeof(int64_t));
  return MBE3_OK;
}

int osv_project(mbe3_handle *h, double *gamma, int64_t gamma_elems) {
  if (!h) return MBE3_EINVAL;
  if (!gamma || gamma_elems < h->gamma_rows * h->n_aux)
    return h->fail(MBE3_EINVAL, "gamma needs %lld doubles, got %lld",
                   (long long)(h->gamma_rows * h->n_aux), (long long)gamma_elems);
  hipStream_t s = h->stream;
  if (h->precision != MBE3_FP64) {
    {
      PhaseScope ps_(h, MBE3_PHASE_REGEN);
      HIP_TRY(h, launch_split_rows(h->Q, h->q_off[h->n_occ], h->n_vir, h->n_vir,
                                   h->qplanes, h->q_ps, h->ldk_vir, s));
    }
    for (size_t k = 0; k < h->proj_batches.size(); ++k) {
      const int i0 = h->proj_batches[k].first, i1 = h->proj_batches[k].second;
      {
        PhaseScope ps_(h, MBE3_PHASE_REGEN);
        HIP_TRY(h, launch_regen_split(h->splanes, h->s_ps, i0, i1 - i0, h->n_vir,
                                      h->n_aux, h->ldk_vir, h->seed, h->w_ia,
                                      h->w_iP, h->slab, s));
      }
      PhaseScope ps_(h, MBE3_PHASE_PROJECT);
      HIP_TRY(h, launch_gemm_mixed(h->d_mproj[k], i1 - i0, h->t_mproj[k], h->qplanes,
                                   h->q_ps, h->splanes, h->s_ps, gamma, h->d_mrows,
                                   MIXED_64x128, s));
    }
    return MBE3_OK;
  }
  GemmBases b = bases(h);
  b.p[B_GAMMA] = gamma;
  for (size_t k = 0; k < h->proj_batches.size(); ++k) {
    const int i0 = h->proj_batches[k].first, i1 = h->proj_batches[k].second;
    if (!h->slab) {
      PhaseScope ps_(h, MBE3_PHASE_REGEN);
      HIP_TRY(h, launch_regen_slab(h->slab_buf, i0, i1 - i0, h->n_vir, h->n_aux,
                                   h->seed, h->w_ia, h->w_iP, 1.0, h->slab_shift, s));
    }
    PhaseScope ps_(h, MBE3_PHASE_PROJECT);
    HIP_TRY(h, launch_list(h, h->L_proj[k], b, s));
  }
  return MBE3_OK;
}

int pair_K(mbe3_handle *h, const double *gamma, double *K, int64_t k_elems) {
  if (!h) return MBE3_EINVAL;
  if (!gamma || !K || k_elems < h->k_elems)
    return h->fail(MBE3_EINVAL, "K needs %lld doubles, got %lld",
                   (long long)h->k_elems, (long long)k_elems);
  PhaseScope ps_(h, MBE3_PHASE_PAIR_K);
  if (h->precision == MBE3_MIXED_BF16) {
    HIP_TRY(h, launch_split_rows_fixed(gamma, h->gamma_rows, h->n_aux, h->n_aux,
                                       h->gplanes, h->g_ps, h->ldk_aux, h->stream));
    HIP_TRY(h, launch_gemm_mixed(h->d_mpk, (int)h->n_slot, h->t_mpk, h->gplanes, h->g_ps,
                                 h->gplanes, h->g_ps, K, h->d_mrows, MIXED_32x64,
                                 h->stream));
    return MBE3_OK;
  }
  GemmBases b = bases(h);
  b.p[B_GAMMA] = const_cast<double *>(gamma);
  b.p[B_K] = K;
  HIP_TRY(h, launch_list(h, h->L_pk, b, h->stream));
  HIP_TRY(h, launch_list(h, h->L_pkw, b, h->stream));
  return MBE3_OK;
}

int fragment_solve(mbe3_handle *h, const double *K, double *e_frag,
                   int32_t *iters, double *W) {
  if (!h) return MBE3_EINVAL;
  if (!K || !e_frag || !iters) return h->fail(MBE3_EINVAL, "K, e_frag, iters required");
  hipStream_t s = h->stream;
  if (!h->recording) h->grad_ready = false;
  int rc;
  if (W && (rc = no_throw(h, [&] { return build_grad_plans(h); }))) return rc;
  if ((rc = prepare_pairs(h, K))) return rc;
  GemmBases b = bases(h);
  HIP_TRY(h, launch_fill_i32(h->status, 0, 2 * SOLVE_WG, s));
  if (W) {
    PhaseScope ps_(h, MBE3_PHASE_GRAD);
    HIP_TRY(h, launch_fill(h->wt, 0.0, h->kt_off[h->n_slot], s));
    HIP_TRY(h, launch_fill(h->graw, 0.0, (int64_t)h->n_occ * h->n_occ, s));
  }
  for (auto &c : h->chunks) {
    if (c.n_asm) {
      PhaseScope ps_(h, MBE3_PHASE_CROSS);
      HIP_TRY(h, launch_assemble(c.d_asm, c.n_asm, h->sstore, h->fstore, h->ca,
                                 nullptr, s));
      HIP_TRY(h, launch_list(h, c.L_m, b, s));
      HIP_TRY(h, launch_list(h, c.L_mw, b, s));  // every M before the S~ that read it
      HIP_TRY(h, launch_list(h, c.L_s1, b, s));
      HIP_TRY(h, launch_list(h, c.L_s1w, b, s));
    }
    SolveArgs a;
    std::memset(&a, 0, sizeof a);
    a.frags = c.d_frags;
    a.terms = c.d_terms;
    a.slots = h->d_slots;
    a.kt = h->kt;
    a.et = h->et;
    a.f_occ = h->f;
    a.st0 = h->st0;
    a.st1 = h->st1;
    a.scratch = h->scratch;
    a.scratch_stride = h->scratch_stride;
    a.n_frag = c.n_frag;
    a.n_occ = h->n_occ;
    a.max_iter = h->max_iter;
    a.tol = h->tol;
    a.e_frag = e_frag;
    a.iters = iters;
    a.status = h->status;
    a.warm = h->warm;
    if (W) {
      a.yfin = h->yfin;
      a.gterm = h->gterm;
      a.gdiag = h->gdiag;
    }
    // the chunk's largest pair dimension picks the kernel and its LDS
    // layout; the scratch stride is the handle's (sized for the largest)
    a.dmax = c.dmax;
    if (c.dmax <= SOLVE_LDS_DMAX) {
      // persistent grid: as many workgroups as are resident on the 256 CUs
      // at once (registers and LDS of the instance), so that no workgroup
      // starts after others have finished their share
      int per_cu = 0, per_cu_g = 0;
      HIP_TRY(h, solve_blocks_per_cu(a, W ? 1 : 0, &per_cu));
      per_cu = std::max(1, per_cu);
      const int nwg = std::min(std::min(SOLVE_WG, c.n_frag), 256 * per_cu);
      {
        PhaseScope ps_(h, MBE3_PHASE_SOLVE);
        HIP_TRY(h, launch_solve(a, nwg, s));
      }
      if (W) {  // dE/df contractions and Y~ at the converged amplitudes
        HIP_TRY(h, solve_blocks_per_cu(a, 2, &per_cu_g));
        per_cu_g = std::max(1, per_cu_g);
        const int nwg_g = std::min(std::min(SOLVE_WG, c.n_frag), 256 * per_cu_g);
        PhaseScope ps_(h, MBE3_PHASE_GRAD);
        HIP_TRY(h, launch_solve_grad(a, nwg_g, s));
      }
    } else {
      const int nwg = std::min(std::min(SOLVE_WG, c.n_frag), 256);
      PhaseScope ps_(h, MBE3_PHASE_SOLVE);
      HIP_TRY(h, launch_solve_wide(a, nwg, s));
    }
    if (W) {
      // this chunk's share of W~ and dE/df (its Y store is reused next)
      PhaseScope ps_(h, MBE3_PHASE_GRAD);
      HIP_TRY(h, launch_wtilde(c.d_ws, c.n_ws, c.d_we, h->yfin, h->wt, s));
      HIP_TRY(h, launch_fgrad(c.d_gd, c.n_gd, c.d_ge, h->gterm, h->gdiag,
                              h->graw, s));
    }
  }
  if (W) {
    PhaseScope ps_(h, MBE3_PHASE_GRAD);
    b.p[B_W] = W;
    HIP_TRY(h, launch_list(h, h->L_wm, b, s));
    HIP_TRY(h, launch_list(h, h->L_ww, b, s));
  }
  HIP_TRY(h, hipMemcpyAsync(h->h_status, h->status, 2 * SOLVE_WG * sizeof(int32_t),
                            hipMemcpyDeviceToHost, s));
  if (h->recording) {  // checked by mbe3_graph_launch after each replay
    h->rec_solve = true;
    h->rec_grad = W != nullptr;
    return MBE3_OK;
  }
  HIP_TRY(h, hipStreamSynchronize(s));
  if ((rc = solve_status(h))) return rc;
  h->grad_ready = W != nullptr;
  return MBE3_OK;
}

int mbe3_backward(mbe3_handle *h, double dE, const double *gamma,
                  const double *W, int mode, double *out, int64_t out_elems,
                  double *dEdF, double *probe) {
  if (!h) return MBE3_EINVAL;
  if (!gamma || !W || !out) return h->fail(MBE3_EINVAL, "gamma, W and out required");
  if (mode != MBE3_GRAD_SLAB && mode != MBE3_GRAD_GAMMA && mode != MBE3_GRAD_PROBE)
    return h->fail(MBE3_EINVAL, "unknown gradient mode %d", mode);
  if (!std::isfinite(dE)) return h->fail(MBE3_EINVAL, "dE is not finite");
  const int64_t na = h->n_aux;
  const int64_t need = mode == MBE3_GRAD_SLAB ? (int64_t)h->n_occ * h->n_vir * na
                                              : h->gamma_rows * na;
  if (out_elems < need)
    return h->fail(MBE3_EINVAL, "out needs %lld doubles, got %lld", (long long)need,
                   (long long)out_elems);
  if (dEdF && !(h->recording ? h->rec_grad : h->grad_ready))
    return h->fail(MBE3_EINVAL, "dE/df needs a preceding successful fragment_solve with W");
  if (mode == MBE3_GRAD_PROBE) {
    if (!probe) return h->fail(MBE3_EINVAL, "MBE3_GRAD_PROBE needs probe[2]");
    if (h->precision != MBE3_FP64 || h->slab)
      return h->fail(MBE3_EINVAL, "MBE3_GRAD_PROBE needs an FP64 handle with regenerated slabs");
    if (out == gamma) return h->fail(MBE3_EINVAL, "MBE3_GRAD_PROBE: out must not be gamma");
  }
  if (probe && h->recording)
    return h->fail(MBE3_EINVAL, "the probe is read on the host: not available while recording");
  int rc = no_throw(h, [&] { return build_grad_plans(h); });
  if (rc) return rc;
  hipStream_t s = h->stream;
  double *dgam = mode == MBE3_GRAD_GAMMA ? out : h->dg;
  const int64_t gel = h->gamma_rows * na;
  {
    PhaseScope ps_(h, MBE3_PHASE_BACKWARD);
    GemmBases b = bases(h);
    b.rows = h->d_grows;
    b.p[B_GAMMA] = const_cast<double *>(gamma);
    b.p[B_W] = const_cast<double *>(W);
    b.p[B_DG] = dgam;
    b.p[B_DB] = out;
    HIP_TRY(h, launch_ga(h->d_ga, h->n_ga, W, dE, h->ga, s));
    HIP_TRY(h, launch_list(h, h->L_dg, b, s));
    if (mode == MBE3_GRAD_SLAB)
      HIP_TRY(h, launch_list(h, h->L_up, b, s));
    if (dEdF) HIP_TRY(h, launch_fsym(h->graw, h->n_occ, dE, dEdF, s));
  }
  if (mode == MBE3_GRAD_PROBE) {
    // <dE/dB, Delta> = sum_{i,x} <dE/dG_{i,x}, Q_x^T Delta_i>: Delta is
    // regenerated and projected into out with osv_project's own lists
    GemmBases b = bases(h);
    b.p[B_GAMMA] = out;
    for (size_t k = 0; k < h->proj_batches.size(); ++k) {
      const int i0 = h->proj_batches[k].first, i1 = h->proj_batches[k].second;
      {
        PhaseScope ps_(h, MBE3_PHASE_REGEN);
        HIP_TRY(h, launch_regen_slab(h->slab_buf, i0, i1 - i0, h->n_vir, h->n_aux, h->seed,
                                     h->w_ia, h->w_iP, 0.0, 1.0, s));
      }
      PhaseScope ps_(h, MBE3_PHASE_BACKWARD);
      HIP_TRY(h, launch_list(h, h->L_proj[k], b, s));
    }
    PhaseScope ps_(h, MBE3_PHASE_BACKWARD);
    HIP_TRY(h, launch_dot(dgam, out, gel, 1.0, h->dot_part, h->d_probe, s));
    HIP_TRY(h, launch_dot(dgam, gamma, gel, 1.0, h->dot_part, h->d_probe + 1, s));
    HIP_TRY(h, hipMemcpyAsync(h->h_probe, h->d_probe, 2 * sizeof(double),
                              hipMemcpyDeviceToHost, s));
    HIP_TRY(h, hipStreamSynchronize(s));
    probe[0] = h->h_probe[0];
    probe[1] = h->h_probe[1];
    return MBE3_OK;
  }
  if (probe) {
    {
      PhaseScope ps_(h, MBE3_PHASE_BACKWARD);
      HIP_TRY(h, launch_dot(dgam, gamma, gel, 1.0, h->dot_part, h->d_probe, s));
    }
    HIP_TRY(h, hipMemcpyAsync(h->h_probe, h->d_probe, sizeof(double),
                              hipMemcpyDeviceToHost, s));
    HIP_TRY(h, hipStreamSynchronize(s));
    *probe = *h->h_probe;
  }
  return MBE3_OK;
}

int mbe3_set_slab_shift(mbe3_handle *h, double t) {
  if (!h) return MBE3_EINVAL;
  if (!std::isfinite(t)) return h->fail(MBE3_EINVAL, "shift is not finite");
  if (h->recording) return h->fail(MBE3_EINVAL, "the shift cannot change while recording");
  if (t != 0.0 && (h->precision != MBE3_FP64 || h->slab))
    return h->fail(MBE3_EINVAL, "a slab shift needs an FP64 handle with regenerated slabs");
  HIP_TRY(h, hipStreamSynchronize(h->stream));
  release_graph(h);  // its regeneration launches carry the old shift
  h->slab_shift = t;
  return MBE3_OK;
}

int mbe3_energy(mbe3_handle *h, const double *e_frag, double *e_total,
                double *incr) {
  if (!h) return MBE3_EINVAL;
  if (!e_frag || !e_total) return h->fail(MBE3_EINVAL, "e_frag and e_total required");
  hipStream_t s = h->stream;
  const int64_t n = (int64_t)h->frags.size();
  {
    PhaseScope ps_(h, MBE3_PHASE_ENERGY);
    HIP_TRY(h, launch_mbe_sum(e_frag, h->d_coef, n, h->d_e3, s));
    if (incr) HIP_TRY(h, launch_increments(e_frag, h->d_sub, n, incr, s));
  }
  HIP_TRY(h, hipMemcpyAsync(h->h_e3, h->d_e3, 3 * sizeof(double),
                            hipMemcpyDeviceToHost, s));
  if (h->recording) {  // the energy comes back from mbe3_graph_launch
    h->rec_energy = true;
    *e_total = std::nan("");
    return MBE3_OK;
  }
  HIP_TRY(h, hipStreamSynchronize(s));
  *e_total = h->h_e3[0];
  if (!std::isfinite(*e_total))
    return h->fail(MBE3_ENONFINITE, "MBE(3) energy is not finite");
  return MBE3_OK;
}

int mbe3_first_order_dE(mbe3_handle *h, const double *K_a, const double *K_b,
                        const double *W, double *per_slot, double *total) {
  if (!h) return MBE3_EINVAL;
  if (!K_a || !K_b || !W || !per_slot || !total)
    return h->fail(MBE3_EINVAL, "K_a, K_b, W, per_slot and total required");
  if (h->recording) return h->fail(MBE3_EINVAL, "mbe3_first_order_dE synchronises: not recordable");
  hipStream_t s = h->stream;
  HIP_TRY(h, launch_slot_dot(K_a, K_b, W, h->d_k_off, h->n_occ, h->n_slot, per_slot, s));
  HIP_TRY(h, launch_mbe_sum(per_slot, nullptr, h->n_slot, h->d_e3, s));
  HIP_TRY(h, hipMemcpyAsync(h->h_e3, h->d_e3, 3 * sizeof(double), hipMemcpyDeviceToHost, s));
  HIP_TRY(h, hipStreamSynchronize(s));
  *total = h->h_e3[0];
  return MBE3_OK;
}

int mbe3_set_timing(mbe3_handle *h, int enable) {
  if (!h) return MBE3_EINVAL;
  if (h->recording) return h->fail(MBE3_EINVAL, "timing cannot change while recording");
  HIP_TRY(h, hipStreamSynchronize(h->stream));
  h->timing = enable != 0;
  h->regions.clear();
  h->event_next = 0;
  for (int k = 0; k < MBE3_NPHASE; ++k) { h->phase_ms[k] = 0.0; h->phase_n[k] = 0; }
  return MBE3_OK;
}

int mbe3_get_timing(mbe3_handle *h, double *ms, int64_t *launches) {
  if (!h || !ms) return MBE3_EINVAL;
  if (h->recording) return h->fail(MBE3_EINVAL, "timing is not readable while recording");
  HIP_TRY(h, hipStreamSynchronize(h->stream));
  for (auto &r : h->regions) {
    float t = 0.f;
    HIP_TRY(h, hipEventElapsedTime(&t, r.a, r.b));
    h->phase_ms[r.phase] += t;
    h->phase_n[r.phase] += 1;
  }
  h->regions.clear();
  h->event_next = 0;
  for (int k = 0; k < MBE3_NPHASE; ++k) {
    ms[k] = h->phase_ms[k];
    if (launches) launches[k] = h->phase_n[k];
  }
  return MBE3_OK;
}

int mbe3_pair_basis(mbe3_handle *h, double *X, double *eps_t, int32_t *rank) {
  if (!h) return MBE3_EINVAL;
  if (!X || !eps_t || !rank) return h->fail(MBE3_EINVAL, "X, eps_t, rank required");
  int rc = prepare_bases(h);
  if (rc) return rc;
  hipStream_t s = h->stream;
  HIP_TRY(h, hipMemcpyAsync(X, h->xb, h->x_off[h->n_slot] * sizeof(double),
                            hipMemcpyDeviceToDevice, s));
  HIP_TRY(h, hipMemcpyAsync(eps_t, h->et, h->et_off[h->n_slot] * sizeof(double),
                            hipMemcpyDeviceToDevice, s));
  HIP_TRY(h, hipMemcpyAsync(rank, h->rank, h->n_slot * sizeof(int32_t),
                            hipMemcpyDeviceToDevice, s));
  return MBE3_OK;
}

static int screen_body(mbe3_handle *h, const int32_t *pairs, int64_t n, double *s2b) {
  if (h->recording) return h->fail(MBE3_EINVAL, "mbe3_screen allocates: not recordable");
  if (n < 0 || (n > 0 && (!pairs || !s2b)))
    return h->fail(MBE3_EINVAL, "pairs and s2b required for n > 0");
  if (n == 0) return MBE3_OK;
  std::vector<WeakPair> wp;
  std::vector<int64_t> p_off;
  int64_t ko, to, po;
  int rc = weak_layout(h, pairs, n, false, wp, &ko, &to, &po, p_off);
  if (rc) return rc;
  CallTemp tmp(h);
  double *S = nullptr;
  WeakPair *d_wp = nullptr;
  if ((rc = tmp.alloc(&S, ko)) || (rc = tmp.upload(&d_wp, wp))) return rc;
  const int nv = h->n_vir;
  std::vector<GemmTask> ts;
  for (const WeakPair &w : wp)  // S_(i,j) = Q_i^T Q_j (rows of the packed Q)
    ts.push_back(gemm(B_Q, h->q_off[w.i] * nv, nv, 0, B_Q, h->q_off[w.j] * nv, nv, 1,
                      B_PS2, w.k_off, w.rj, w.ri, w.rj, nv));
  int64_t sz[B_COUNT];
  base_sizes(h, sz);
  sz[B_PS2] = ko;
  GemmBases b = bases(h);
  b.p[B_PS2] = S;
  if ((rc = run_call_list(h, tmp, "screen S", ts, sz, b, GEMM_32x32))) return rc;
  HIP_TRY(h, launch_s2b(d_wp, (int)n, S, s2b, h->stream));
  HIP_TRY(h, hipStreamSynchronize(h->stream));
  return MBE3_OK;
}

static int weak_body(mbe3_handle *h, const int32_t *pairs, int64_t n, const double *gamma,
                     const double *W, double *e) {
  if (h->recording) return h->fail(MBE3_EINVAL, "mbe3_weak_pairs allocates: not recordable");
  if (n < 0 || (n > 0 && (!pairs || !gamma || !W || !e)))
    return h->fail(MBE3_EINVAL, "pairs, gamma, W and e required for n > 0");
  if (n == 0) return MBE3_OK;
  std::vector<WeakPair> wp;
  std::vector<int64_t> p_off;
  int64_t ko, to, po;
  int rc = weak_layout(h, pairs, n, true, wp, &ko, &to, &po, p_off);
  if (rc) return rc;
  // X, eps~ and ranks of the diagonal slots: those of the last eager
  // preparation (fragment_solve, mbe3_pair_basis), else prepared here
  if (!h->bases_done && (rc = prepare_bases(h))) return rc;
  CallTemp tmp(h);
  double *Kb = nullptr, *Sb = nullptr, *Mb = nullptr, *Pb = nullptr, *Kt = nullptr,
         *Dt = nullptr;
  WeakPair *d_wp = nullptr;
  if ((rc = tmp.alloc(&Kb, ko)) || (rc = tmp.alloc(&Sb, ko)) || (rc = tmp.alloc(&Mb, ko)) ||
      (rc = tmp.alloc(&Pb, po)) || (rc = tmp.alloc(&Kt, to)) || (rc = tmp.alloc(&Dt, to)) ||
      (rc = tmp.upload(&d_wp, wp)))
    return rc;
  const int nv = h->n_vir, na = h->n_aux;
  std::vector<GemmTask> lk, ls, lm1, lm2, lxk, lkx, lxm, lmx;
  for (int64_t k = 0; k < n; ++k) {
    const WeakPair &w = wp[k];
    const auto fi = h->grow.find(key2(w.i, w.i)), fj = h->grow.find(key2(w.j, w.j));
    if (fi == h->grow.end() || fj == h->grow.end())  // every LMO projects onto itself
      return h->fail(MBE3_EINVAL, "internal: no gamma rows of (%d,%d) or (%d,%d)", w.i, w.i,
                     w.j, w.j);
    const int64_t gi = fi->second, gj = fj->second;
    // K_(i,j) = Gamma~_(i,i) Gamma~_(j,j)^T (eq. osv_weak_k)
    lk.push_back(gemm(B_GAMMA, gi * na, na, 0, B_GAMMA, gj * na, na, 1, B_PK, w.k_off,
                      w.rj, w.ri, w.rj, na));
    // S_(i,j) = Q_i^T Q_j
    ls.push_back(gemm(B_Q, h->q_off[w.i] * nv, nv, 0, B_Q, h->q_off[w.j] * nv, nv, 1,
                      B_PS2, w.k_off, w.rj, w.ri, w.rj, nv));
    // M = T_ii S_(i,j) + S_(i,j) T_jj, T_ii the diagonal slot blocks of W
    lm1.push_back(gemm(B_W, h->k_off[w.i], w.ri, 0, B_PS2, w.k_off, w.rj, 0, B_PM, w.k_off,
                       w.rj, w.ri, w.rj, w.ri));
    lm2.push_back(gemm(B_PS2, w.k_off, w.rj, 0, B_W, h->k_off[w.j], w.rj, 0, B_PM, w.k_off,
                       w.rj, w.ri, w.rj, w.rj, 1.0, 1.0));
    // K~ = X_i^T K X_j and D~ = X_i^T M X_j (X: d x D, row-major)
    lxk.push_back(gemm(B_X, h->x_off[w.i], w.Di, 1, B_PK, w.k_off, w.rj, 0, B_PP, p_off[k],
                       w.rj, w.Di, w.rj, w.ri));
    lkx.push_back(gemm(B_PP, p_off[k], w.rj, 0, B_X, h->x_off[w.j], w.Dj, 0, B_PKT, w.t_off,
                       w.Dj, w.Di, w.Dj, w.rj));
    lxm.push_back(gemm(B_X, h->x_off[w.i], w.Di, 1, B_PM, w.k_off, w.rj, 0, B_PP, p_off[k],
                       w.rj, w.Di, w.rj, w.ri));
    lmx.push_back(gemm(B_PP, p_off[k], w.rj, 0, B_X, h->x_off[w.j], w.Dj, 0, B_PDT, w.t_off,
                       w.Dj, w.Di, w.Dj, w.rj));
  }
  int64_t sz[B_COUNT];
  base_sizes(h, sz);
  sz[B_W] = h->k_elems;
  sz[B_PK] = sz[B_PS2] = sz[B_PM] = ko;
  sz[B_PP] = po;
  sz[B_PKT] = sz[B_PDT] = to;
  GemmBases b = bases(h);
  b.p[B_GAMMA] = const_cast<double *>(gamma);
  b.p[B_W] = const_cast<double *>(W);
  b.p[B_PK] = Kb; b.p[B_PS2] = Sb; b.p[B_PM] = Mb; b.p[B_PP] = Pb;
  b.p[B_PKT] = Kt; b.p[B_PDT] = Dt;
  // stream order: each list reads what the ones before it wrote
  if ((rc = run_call_list(h, tmp, "weak K", lk, sz, b, GEMM_32x32)) ||
      (rc = run_call_list(h, tmp, "weak S", ls, sz, b, GEMM_32x32)) ||
      (rc = run_call_list(h, tmp, "weak T S", lm1, sz, b, GEMM_32x32)) ||
      (rc = run_call_list(h, tmp, "weak S T", lm2, sz, b, GEMM_32x32)) ||
      (rc = run_call_list(h, tmp, "weak X^T K", lxk, sz, b, GEMM_32x32)) ||
      (rc = run_call_list(h, tmp, "weak K~", lkx, sz, b, GEMM_32x32)) ||
      (rc = run_call_list(h, tmp, "weak X^T M", lxm, sz, b, GEMM_32x32)) ||
      (rc = run_call_list(h, tmp, "weak D~", lmx, sz, b, GEMM_32x32)))
    return rc;
  HIP_TRY(h, launch_weak_energy(d_wp, (int)n, Kt, Dt, h->et, h->rank, h->f, h->n_occ, e,
                                h->stream));
  HIP_TRY(h, hipStreamSynchronize(h->stream));
  return MBE3_OK;
}

int mbe3_fit_metric(mbe3_handle *h, double *s_fit) {
  if (!h) return MBE3_EINVAL;
  if (h->slab_shift != 0.0)
    return h->fail(MBE3_EINVAL, "a slab shift is set: only osv_project regenerates B + t Delta");
  if (!s_fit) return h->fail(MBE3_EINVAL, "s_fit required");
  PhaseScope ps_(h, MBE3_PHASE_REGEN);
  HIP_TRY(h, launch_fit_metric(s_fit, h->n_occ, h->n_vir, h->n_aux, h->seed, h->w_ia,
                               h->w_iP, h->slab, h->stream));
  return MBE3_OK;
}

int mbe3_fit_mask(mbe3_handle *h, const double *s_fit, double l_fit, double *g,
                  int64_t g_elems) {
  if (!h) return MBE3_EINVAL;
  if (!s_fit || !g) return h->fail(MBE3_EINVAL, "s_fit and g required");
  if (std::isnan(l_fit)) return h->fail(MBE3_EINVAL, "l_fit is NaN");
  if (g_elems < h->gamma_rows * h->n_aux)
    return h->fail(MBE3_EINVAL, "g needs %lld doubles, got %lld",
                   (long long)(h->gamma_rows * h->n_aux), (long long)g_elems);
  PhaseScope ps_(h, MBE3_PHASE_PROJECT);
  HIP_TRY(h, launch_fit_mask(g, h->gamma_rows, h->n_aux, h->d_row_lmo, h->d_row_x,
                             h->d_nbr_off, h->d_nbr, s_fit, l_fit, h->stream));
  return MBE3_OK;
}

// The fitting domains from a device metric (copied back; the stream is
// synchronised): D_i = {P : s_fit[i][P] > l_fit} at dcols[dcol_off[i] ..
// dcol_off[i + 1]), ascending.  Every integral of eq. osv_close_k for a pair
// (p, q) sums over D_p u D_q (D_p for the diagonal slot), so LMO i's
// projected rows are needed on C_i = the union of D_q over q in N+(i):
// ccols[ccol_off[i] .. ccol_off[i + 1]), ascending.  batches: runs of LMOs
// whose compacted slabs (n_vir x |C_i| each) fit the slab budget together
// (at most 65535 per run, one workgroup row each); *cs_max the largest run.
static int fit_domains(mbe3_handle *h, const double *s_fit, double l_fit,
                       std::vector<int32_t> &dcols, std::vector<int32_t> &dcol_off,
                       std::vector<int32_t> &ccols, std::vector<int32_t> &ccol_off,
                       std::vector<std::pair<int, int>> &batches, int64_t *cs_max) {
  const int n = h->n_occ, nv = h->n_vir, na = h->n_aux;
  std::vector<double> sf((size_t)n * na);
  HIP_TRY(h, hipMemcpyAsync(sf.data(), s_fit, sf.size() * sizeof(double),
                            hipMemcpyDeviceToHost, h->stream));
  HIP_TRY(h, hipStreamSynchronize(h->stream));
  dcols.clear();
  dcol_off.assign((size_t)n + 1, 0);
  for (int i = 0; i < n; ++i) {
    for (int P = 0; P < na; ++P)
      if (sf[(size_t)i * na + P] > l_fit) dcols.push_back(P);
    dcol_off[i + 1] = (int32_t)dcols.size();
  }
  ccols.clear();
  ccol_off.assign((size_t)n + 1, 0);
  std::vector<char> mark((size_t)na);
  for (int i = 0; i < n; ++i) {
    std::fill(mark.begin(), mark.end(), 0);
    for (int q : h->nbr[i])
      for (int c = dcol_off[q]; c < dcol_off[q + 1]; ++c) mark[(size_t)dcols[c]] = 1;
    for (int P = 0; P < na; ++P)
      if (mark[(size_t)P]) ccols.push_back(P);
    ccol_off[i + 1] = (int32_t)ccols.size();
  }
  const int64_t budget = SLAB_BUDGET / (int64_t)sizeof(double);
  batches.clear();
  *cs_max = 0;
  for (int i0 = 0; i0 < n;) {
    int i1 = i0;
    int64_t tot = 0;
    while (i1 < n && i1 - i0 < 65535 &&
           (i1 == i0 || tot + (int64_t)nv * (ccol_off[i1 + 1] - ccol_off[i1]) <= budget)) {
      tot += (int64_t)nv * (ccol_off[i1 + 1] - ccol_off[i1]);
      ++i1;
    }
    batches.push_back({i0, i1});
    *cs_max = std::max(*cs_max, tot);
    i0 = i1;
  }
  return MBE3_OK;
}

// osv_project over the fitting domains only: per LMO i the columns C_i are
// listed on the host (s_fit copied back), regenerated compacted, projected
// by one GEMM per LMO over them and scattered into the zeroed dense gamma;
// the rows of blocks (i, x), x != i, are then cut to D_i u D_x by the mask
// kernel (eq. osv_imua).
static int project_fit_body(mbe3_handle *h, const double *s_fit, double l_fit, double *gamma,
                            int64_t gamma_elems) {
  if (h->slab_shift != 0.0)
    return h->fail(MBE3_EINVAL, "a slab shift is set: only osv_project regenerates B + t Delta");
  if (h->recording)
    return h->fail(MBE3_EINVAL, "mbe3_project_fit allocates: not recordable");
  if (!s_fit || !gamma) return h->fail(MBE3_EINVAL, "s_fit and gamma required");
  if (std::isnan(l_fit)) return h->fail(MBE3_EINVAL, "l_fit is NaN");
  const int n = h->n_occ, nv = h->n_vir, na = h->n_aux;
  if (gamma_elems < h->gamma_rows * na)
    return h->fail(MBE3_EINVAL, "gamma needs %lld doubles, got %lld",
                   (long long)(h->gamma_rows * na), (long long)gamma_elems);
  hipStream_t s = h->stream;
  std::vector<int32_t> dcols, dcol_off, cols, col_off;
  std::vector<std::pair<int, int>> batches;
  int64_t cs_max = 0;
  int rc = fit_domains(h, s_fit, l_fit, dcols, dcol_off, cols, col_off, batches, &cs_max);
  if (rc) return rc;
  std::vector<int64_t> gc_off((size_t)n + 1, 0);
  int max_nc = 0;
  for (int i = 0; i < n; ++i) {
    const int nc = col_off[i + 1] - col_off[i];
    max_nc = std::max(max_nc, nc);
    gc_off[i + 1] = gc_off[i] + (h->g_off[i + 1] - h->g_off[i]) * nc;
  }
  CallTemp tmp(h);
  int32_t *d_cols = nullptr, *d_col_off = nullptr;
  int64_t *d_goff = nullptr, *d_gcoff = nullptr;
  double *gc = nullptr, *cs = nullptr;
  if ((rc = tmp.upload(&d_cols, cols)) || (rc = tmp.upload(&d_col_off, col_off)) ||
      (rc = tmp.upload(&d_goff, h->g_off)) || (rc = tmp.upload(&d_gcoff, gc_off)) ||
      (rc = tmp.alloc(&gc, gc_off[n])) || (rc = tmp.alloc(&cs, cs_max)))
    return rc;
  HIP_TRY(h, launch_fill(gamma, 0.0, h->gamma_rows * na, s));
  int64_t sz[B_COUNT];
  base_sizes(h, sz);
  sz[B_SLAB] = cs_max;
  sz[B_GAMMA] = gc_off[n];
  for (const auto &bt : batches) {
    const int i0 = bt.first, i1 = bt.second;
    std::vector<int64_t> out_off;
    std::vector<GemmTask> ts;
    std::vector<int32_t> rows;
    int64_t off = 0, max_elems = 0;
    for (int i = i0; i < i1; ++i) {
      const int nc = col_off[i + 1] - col_off[i];
      out_off.push_back(off);
      max_elems = std::max<int64_t>(max_elems, (int64_t)nv * nc);
      if (nc > 0) {
        GemmTask t = gemm(B_Q, 0, nv, 0, B_SLAB, off, nc, 0, B_GAMMA, gc_off[i], nc,
                          (int)(h->g_off[i + 1] - h->g_off[i]), nc, nv);
        t.a_rows = (int32_t)rows.size();
        for (int x : h->nbr[i])
          for (int mu = 0; mu < h->r[x]; ++mu) rows.push_back((int32_t)(h->q_off[x] + mu));
        ts.push_back(t);
      }
      off += (int64_t)nv * nc;
    }
    if (ts.empty()) continue;
    int64_t *d_out_off = nullptr;
    int32_t *d_rows = nullptr;
    GemmTask *d_ts = nullptr;
    const int64_t tiles = finish_tasks(ts, GEMM_128x128);
    if ((rc = check_gemm_list(h, "project (fitting domains)", ts, sz, rows, GEMM_128x128)))
      return rc;
    if ((rc = tmp.upload(&d_out_off, out_off)) || (rc = tmp.upload(&d_rows, rows)) ||
        (rc = tmp.upload(&d_ts, ts)))
      return rc;
    {
      PhaseScope ps_(h, MBE3_PHASE_REGEN);
      HIP_TRY(h, launch_regen_cols(cs, d_out_off, d_cols, d_col_off, i0, i1 - i0, max_elems,
                                   nv, na, h->seed, h->w_ia, h->w_iP, h->slab, s));
    }
    PhaseScope ps_(h, MBE3_PHASE_PROJECT);
    GemmBases b = bases(h);
    b.p[B_SLAB] = cs;
    b.p[B_GAMMA] = gc;
    b.rows = d_rows;
    HIP_TRY(h, launch_gemm_tasks(d_ts, (int)ts.size(), tiles, b, GEMM_128x128, s));
  }
  HIP_TRY(h, launch_fit_scatter(gamma, gc, h->gamma_rows, na, max_nc, h->d_row_lmo, d_goff,
                                d_gcoff, d_cols, d_col_off, s));
  HIP_TRY(h, launch_fit_mask(gamma, h->gamma_rows, na, h->d_row_lmo, h->d_row_x,
                             h->d_nbr_off, h->d_nbr, s_fit, l_fit, s));
  return MBE3_OK;
}

// pair_K over the fitting domains (eq. osv_close_k, A' in D_p u D_q): the
// columns C_i projected as in project_fit but stored transposed and
// compacted (GT_i: column of C_i x gamma row of LMO i), then each K block of
// slot (p, q) summed over the union D_p u D_q (D_p for a diagonal slot) by
// gathering the union's rows of GT_p and GT_q, both of which hold it (k-row
// gathers of the grouped-GEMM engine).
static int pair_k_fit_body(mbe3_handle *h, const double *s_fit, double l_fit, double *K,
                           int64_t k_elems) {
  if (h->slab_shift != 0.0)
    return h->fail(MBE3_EINVAL, "a slab shift is set: only osv_project regenerates B + t Delta");
  if (h->recording)
    return h->fail(MBE3_EINVAL, "mbe3_pair_K_fit allocates: not recordable");
  if (!s_fit || !K) return h->fail(MBE3_EINVAL, "s_fit and K required");
  if (std::isnan(l_fit)) return h->fail(MBE3_EINVAL, "l_fit is NaN");
  if (k_elems < h->k_elems)
    return h->fail(MBE3_EINVAL, "K needs %lld doubles, got %lld", (long long)h->k_elems,
                   (long long)k_elems);
  const int n = h->n_occ, nv = h->n_vir, na = h->n_aux;
  hipStream_t s = h->stream;
  std::vector<int32_t> dcols, dcol_off, cols, col_off;
  std::vector<std::pair<int, int>> batches;
  int64_t cs_max = 0;
  int rc = fit_domains(h, s_fit, l_fit, dcols, dcol_off, cols, col_off, batches, &cs_max);
  if (rc) return rc;
  std::vector<int64_t> gt_off((size_t)n + 1, 0);
  for (int i = 0; i < n; ++i)
    gt_off[i + 1] = gt_off[i] + (h->g_off[i + 1] - h->g_off[i]) * (col_off[i + 1] - col_off[i]);
  CallTemp tmp(h);
  int32_t *d_cols = nullptr, *d_col_off = nullptr;
  double *gt = nullptr, *cs = nullptr;
  if ((rc = tmp.upload(&d_cols, cols)) || (rc = tmp.upload(&d_col_off, col_off)) ||
      (rc = tmp.alloc(&gt, gt_off[n])) || (rc = tmp.alloc(&cs, cs_max)))
    return rc;
  int64_t sz[B_COUNT];
  base_sizes(h, sz);
  sz[B_SLAB] = cs_max;
  sz[B_GAMMA] = gt_off[n];
  // GT_i = (B_i restricted to C_i)^T Q_{N+(i)}: A the compacted slab read
  // transposed, B the gathered rows of Q^T read transposed
  for (const auto &bt : batches) {
    const int i0 = bt.first, i1 = bt.second;
    std::vector<int64_t> out_off;
    std::vector<GemmTask> ts;
    std::vector<int32_t> rows;
    int64_t off = 0, max_elems = 0;
    for (int i = i0; i < i1; ++i) {
      const int nc = col_off[i + 1] - col_off[i];
      const int Mi = (int)(h->g_off[i + 1] - h->g_off[i]);
      out_off.push_back(off);
      max_elems = std::max<int64_t>(max_elems, (int64_t)nv * nc);
      if (nc > 0) {
        GemmTask t = gemm(B_SLAB, off, nc, 1, B_Q, 0, nv, 1, B_GAMMA, gt_off[i], Mi, nc, Mi,
                          nv);
        t.b_rows = (int32_t)rows.size();
        for (int x : h->nbr[i])
          for (int mu = 0; mu < h->r[x]; ++mu) rows.push_back((int32_t)(h->q_off[x] + mu));
        ts.push_back(t);
      }
      off += (int64_t)nv * nc;
    }
    if (ts.empty()) continue;
    int64_t *d_out_off = nullptr;
    int32_t *d_rows = nullptr;
    GemmTask *d_ts = nullptr;
    const int64_t tiles = finish_tasks(ts, GEMM_64x64);
    if ((rc = check_gemm_list(h, "project^T (fitting domains)", ts, sz, rows, GEMM_64x64)))
      return rc;
    if ((rc = tmp.upload(&d_out_off, out_off)) || (rc = tmp.upload(&d_rows, rows)) ||
        (rc = tmp.upload(&d_ts, ts)))
      return rc;
    {
      PhaseScope ps_(h, MBE3_PHASE_REGEN);
      HIP_TRY(h, launch_regen_cols(cs, d_out_off, d_cols, d_col_off, i0, i1 - i0, max_elems,
                                   nv, na, h->seed, h->w_ia, h->w_iP, h->slab, s));
    }
    PhaseScope ps_(h, MBE3_PHASE_PROJECT);
    GemmBases b = bases(h);
    b.p[B_SLAB] = cs;
    b.p[B_GAMMA] = gt;
    b.rows = d_rows;
    HIP_TRY(h, launch_gemm_tasks(d_ts, (int)ts.size(), tiles, b, GEMM_64x64, s));
  }
  // K blocks (x, y) of every slot over the union of the two domains
  std::vector<GemmTask> kt;
  std::vector<int32_t> krows;
  std::vector<int32_t> un, ip, iq;
  // positions of the ascending columns u in the ascending list C_i (every u
  // is in C_i: D_p, D_q are both in C_p and in C_q for a kept pair)
  auto positions = [&](int i, std::vector<int32_t> &out) -> bool {
    out.clear();
    int c = col_off[i];
    for (int32_t P : un) {
      while (c < col_off[i + 1] && cols[c] < P) ++c;
      if (c == col_off[i + 1] || cols[c] != P) return false;
      out.push_back(c - col_off[i]);
    }
    return true;
  };
  for (int sl = 0; sl < h->n_slot; ++sl) {
    const int p = h->sp[sl], q = h->sq[sl];
    un.clear();
    std::set_union(dcols.begin() + dcol_off[p], dcols.begin() + dcol_off[p + 1],
                   dcols.begin() + dcol_off[q], dcols.begin() + dcol_off[q + 1],
                   std::back_inserter(un));
    if (un.empty()) continue;
    if (!positions(p, ip) || !positions(q, iq))
      return h->fail(MBE3_EINVAL, "internal: union of D_%d and D_%d outside C", p, q);
    const int32_t ro_p = (int32_t)krows.size();
    krows.insert(krows.end(), ip.begin(), ip.end());
    const int32_t ro_q = (int32_t)krows.size();
    krows.insert(krows.end(), iq.begin(), iq.end());
    const int Mp = (int)(h->g_off[p + 1] - h->g_off[p]);
    const int Mq = (int)(h->g_off[q + 1] - h->g_off[q]);
    const int d = p == q ? h->r[p] : h->r[p] + h->r[q];
    const int xs[2] = {p, q};
    const int nx = p == q ? 1 : 2;
    int ro = 0;
    for (int xi = 0; xi < nx; ++xi) {
      const int x = xs[xi];
      const auto fx = h->grow.find(key2(p, x));
      if (fx == h->grow.end()) return h->fail(MBE3_EINVAL, "internal: no rows of (%d,%d)", p, x);
      int co = 0;
      for (int yi = 0; yi < nx; ++yi) {
        const int y = xs[yi];
        const auto fy = h->grow.find(key2(q, y));
        if (fy == h->grow.end())
          return h->fail(MBE3_EINVAL, "internal: no rows of (%d,%d)", q, y);
        GemmTask t = gemm(B_GAMMA, gt_off[p] + (fx->second - h->g_off[p]), Mp, 1, B_GAMMA,
                          gt_off[q] + (fy->second - h->g_off[q]), Mq, 0, B_K,
                          h->k_off[sl] + (int64_t)ro * d + co, d, h->r[x], h->r[y],
                          (int)ip.size());
        t.a_rows = ro_p;
        t.b_rows = ro_q;
        kt.push_back(t);
        co += h->r[y];
      }
      ro += h->r[x];
    }
  }
  HIP_TRY(h, launch_fill(K, 0.0, h->k_elems, s));
  if (!kt.empty()) {
    int32_t *d_krows = nullptr;
    GemmTask *d_kt = nullptr;
    const int64_t tiles = finish_tasks(kt, GEMM_32x32);
    if ((rc = check_gemm_list(h, "pair_K (fitting domains)", kt, sz, krows, GEMM_32x32)))
      return rc;
    if ((rc = tmp.upload(&d_krows, krows)) || (rc = tmp.upload(&d_kt, kt))) return rc;
    PhaseScope ps_(h, MBE3_PHASE_PAIR_K);
    GemmBases b = bases(h);
    b.p[B_GAMMA] = gt;
    b.p[B_K] = K;
    b.rows = d_krows;
    HIP_TRY(h, launch_gemm_tasks(d_kt, (int)kt.size(), tiles, b, GEMM_32x32, s));
  }
  return MBE3_OK;
}

// Randomized OSV generation (Alg. 3) for every LMO, in batches of LMOs whose
// T_ii fit a budget: compacted slab columns of D_i -> T = B_D B_D^T, the
// Cauchy scaling (eq. mp2_tkk) -> the Gaussian rows G (Philox stream 11)
// -> Y = G T -> range finder -> T~ = Z T -> M = T~ T~^T -> eigenvectors of
// M (eq. tii_rsvd through the Gram matrix) -> Q_i^T = Q~^T Z (eq. back_q)
// -> selection by w >= l_osv.
static constexpr int ROSV_R = 10;             // rows per stopping-test block
static constexpr uint64_t ROSV_STREAM = 11;   // Philox stream of G
static constexpr int64_t ROSV_BUDGET = 8LL << 30;  // bytes of T per batch

static int rosv_body(mbe3_handle *h, const double *s_fit, double l_fit, double l_osv,
                     int n_max, double *Q_out, double *w_out, int32_t *n_osv,
                     int32_t *rows_out) {
  if (h->slab_shift != 0.0)
    return h->fail(MBE3_EINVAL, "a slab shift is set: only osv_project regenerates B + t Delta");
  if (h->recording) return h->fail(MBE3_EINVAL, "mbe3_rosv allocates: not recordable");
  if (!Q_out || !w_out || !n_osv || !rows_out)
    return h->fail(MBE3_EINVAL, "Q_out, w_out, n_osv and rows required");
  if (s_fit && std::isnan(l_fit)) return h->fail(MBE3_EINVAL, "l_fit is NaN");
  if (!(l_osv > 0.0)) return h->fail(MBE3_EINVAL, "l_osv must be positive");
  const int n = h->n_occ, nv = h->n_vir, na = h->n_aux;
  if (n_max < 1 || n_max > nv || n_max > eig_qr_max_order())
    return h->fail(MBE3_EINVAL, "n_max = %d outside 1 .. min(n_vir, %d)", n_max,
                   eig_qr_max_order());
  hipStream_t st = h->stream;
  // fitting domains (all columns without a metric)
  std::vector<int32_t> cols, col_off((size_t)n + 1, 0);
  if (s_fit) {
    std::vector<double> sf((size_t)n * na);
    HIP_TRY(h, hipMemcpyAsync(sf.data(), s_fit, sf.size() * sizeof(double),
                              hipMemcpyDeviceToHost, st));
    HIP_TRY(h, hipStreamSynchronize(st));
    for (int i = 0; i < n; ++i) {
      for (int P = 0; P < na; ++P)
        if (sf[(size_t)i * na + P] > l_fit) cols.push_back(P);
      col_off[i + 1] = (int32_t)cols.size();
    }
  } else {
    for (int i = 0; i < n; ++i) {
      for (int P = 0; P < na; ++P) cols.push_back(P);
      col_off[i + 1] = (int32_t)cols.size();
    }
  }
  const int nr = ROSV_R + n_max;                 // Gaussian rows per LMO
  const int Dq = (n_max + 15) / 16 * 16;         // eigenvector pitch
  const int64_t t_elems = (int64_t)nv * nv;
  int nb_max = (int)std::max<int64_t>(1, std::min<int64_t>(
      ROSV_BUDGET / (t_elems * (int64_t)sizeof(double)), 65535));
  int64_t max_nc = 0;
  for (int i = 0; i < n; ++i) max_nc = std::max<int64_t>(max_nc, col_off[i + 1] - col_off[i]);
  nb_max = (int)std::min<int64_t>(nb_max, std::max<int64_t>(
      1, (SLAB_BUDGET / (int64_t)sizeof(double)) / std::max<int64_t>(1, nv * max_nc)));
  nb_max = std::min(nb_max, n);
  CallTemp tmp(h);
  int32_t *d_cols = nullptr, *d_col_off = nullptr, *d_rows = nullptr;
  double *cs = nullptr, *T = nullptr, *G = nullptr, *Y = nullptr, *Z = nullptr, *Tt = nullptr,
         *M = nullptr, *Qe = nullptr, *ev = nullptr, *Qr = nullptr;
  const int64_t cs_per = (int64_t)nv * std::max<int64_t>(1, max_nc);
  int rc;
  if ((rc = tmp.upload(&d_cols, cols)) || (rc = tmp.upload(&d_col_off, col_off)) ||
      (rc = tmp.alloc(&cs, (int64_t)nb_max * cs_per)) ||
      (rc = tmp.alloc(&T, (int64_t)nb_max * t_elems)) ||
      (rc = tmp.alloc(&G, (int64_t)nb_max * nr * nv)) ||
      (rc = tmp.alloc(&Y, (int64_t)nb_max * nr * nv)) ||
      (rc = tmp.alloc(&Z, (int64_t)nb_max * n_max * nv)) ||
      (rc = tmp.alloc(&Tt, (int64_t)nb_max * n_max * nv)) ||
      (rc = tmp.alloc(&M, (int64_t)nb_max * n_max * n_max)) ||
      (rc = tmp.alloc(&Qe, (int64_t)nb_max * Dq * Dq)) ||
      (rc = tmp.alloc(&ev, (int64_t)nb_max * Dq)) ||
      (rc = tmp.alloc(&Qr, (int64_t)nb_max * n_max * nv)) ||
      (rc = tmp.alloc(&d_rows, nb_max)))
    return rc;
  // operands of the call's products (base ids of the engine, call-time
  // pointers): compacted slabs, T, G, Y, Z, T~, M, eigenvectors, Q rows
  int64_t sz[B_COUNT];
  base_sizes(h, sz);
  sz[B_SLAB] = (int64_t)nb_max * cs_per;
  sz[B_PK] = (int64_t)nb_max * t_elems;
  sz[B_PS2] = (int64_t)nb_max * nr * nv;
  sz[B_K] = (int64_t)nb_max * nr * nv;
  sz[B_PM] = (int64_t)nb_max * n_max * nv;
  sz[B_PP] = (int64_t)nb_max * n_max * nv;
  sz[B_PKT] = (int64_t)nb_max * n_max * n_max;
  sz[B_PDT] = (int64_t)nb_max * Dq * Dq;
  sz[B_GAMMA] = (int64_t)nb_max * n_max * nv;
  GemmBases b = bases(h);
  b.p[B_SLAB] = cs;
  b.p[B_PK] = T;
  b.p[B_PS2] = G;
  b.p[B_K] = Y;
  b.p[B_PM] = Z;
  b.p[B_PP] = Tt;
  b.p[B_PKT] = M;
  b.p[B_PDT] = Qe;
  b.p[B_GAMMA] = Qr;
  const double thr = l_osv / (10.0 * std::sqrt(2.0 / 3.141592653589793));
  for (int i0 = 0; i0 < n; i0 += nb_max) {
    const int nb = std::min(nb_max, n - i0);
    std::vector<int64_t> out_off;
    std::vector<GemmTask> tT, tY, tTt, tM, tQ;
    std::vector<EigTask> et;
    int64_t off = 0;
    for (int k = 0; k < nb; ++k) {
      const int i = i0 + k;
      const int nc = col_off[i + 1] - col_off[i];
      out_off.push_back(off);
      const int64_t t0 = (int64_t)k * t_elems;
      const int64_t y0 = (int64_t)k * nr * nv, z0 = (int64_t)k * n_max * nv;
      if (nc > 0)  // T = B_D B_D^T (the compacted slab is n_vir x nc)
        tT.push_back(gemm(B_SLAB, off, nc, 0, B_SLAB, off, nc, 1, B_PK, t0, nv, nv, nv, nc));
      off += (int64_t)nv * nc;
      tY.push_back(gemm(B_PS2, y0, nv, 0, B_PK, t0, nv, 0, B_K, y0, nv, nr, nv, nv));  // Y = G T
      tTt.push_back(gemm(B_PM, z0, nv, 0, B_PK, t0, nv, 0, B_PP, z0, nv, n_max, nv, nv));  // Z T
      tM.push_back(gemm(B_PP, z0, nv, 0, B_PP, z0, nv, 1, B_PKT, (int64_t)k * n_max * n_max,
                        n_max, n_max, n_max, nv));  // M = T~ T~^T
      tQ.push_back(gemm(B_PDT, (int64_t)k * Dq * Dq, Dq, 1, B_PM, z0, nv, 0, B_GAMMA, z0, nv,
                        n_max, nv, n_max));  // rows of Q~^T Z
      EigTask e;
      std::memset(&e, 0, sizeof e);
      e.a_off = (int64_t)k * n_max * n_max;
      e.lda = n_max;
      e.n = n_max;  // selects the launch; the order is rows[k]
      e.D = Dq;
      e.o_off = (int64_t)k * Dq * Dq;
      e.e_off = (int64_t)k * Dq;
      e.slot = k;
      e.w_off = -1;
      et.push_back(e);
    }
    int64_t *d_out_off = nullptr;
    EigTask *d_et = nullptr;
    if ((rc = tmp.upload(&d_out_off, out_off)) || (rc = tmp.upload(&d_et, et))) return rc;
    HIP_TRY(h, launch_fill(T, 0.0, (int64_t)nb * t_elems, st));  // LMOs with empty domains
    HIP_TRY(h, launch_regen_cols(cs, d_out_off, d_cols, d_col_off, i0, nb, cs_per, nv, na,
                                 h->seed, h->w_ia, h->w_iP, h->slab, st));
    if ((rc = run_call_list(h, tmp, "rosv T", tT, sz, b, GEMM_128x128))) return rc;
    HIP_TRY(h, launch_rosv_tscale(T, i0, nb, nv, h->eps, h->f, n, st));
    HIP_TRY(h, launch_regen_gauss(G, i0, nb, nr, nv, h->seed, ROSV_STREAM, st));
    if ((rc = run_call_list(h, tmp, "rosv Y", tY, sz, b, GEMM_64x64))) return rc;
    HIP_TRY(h, launch_range_finder(Y, Z, d_rows, nb, ROSV_R, n_max, nv, thr, st));
    if ((rc = run_call_list(h, tmp, "rosv T~", tTt, sz, b, GEMM_64x64))) return rc;
    if ((rc = run_call_list(h, tmp, "rosv M", tM, sz, b, GEMM_64x64))) return rc;
    HIP_TRY(h, launch_eigh(d_et, nb, n_max, M, Qe, ev, d_rows, 1, 0.0, nullptr, h->eig_ws,
                           h->eig_ws_doubles, st));
    if ((rc = run_call_list(h, tmp, "rosv Q", tQ, sz, b, GEMM_64x64))) return rc;
    HIP_TRY(h, launch_rosv_finalize(ev, Dq, Qr, d_rows, i0, nb, n_max, nv, l_osv, Q_out, w_out,
                                    n_osv, rows_out, st));
  }
  HIP_TRY(h, hipStreamSynchronize(st));
  return MBE3_OK;
}

int mbe3_rosv(mbe3_handle *h, const double *s_fit, double l_fit, double l_osv, int n_max,
              double *Q_out, double *w_out, int32_t *n_osv, int32_t *rows) {
  if (!h) return MBE3_EINVAL;
  return no_throw(h, [&] {
    return rosv_body(h, s_fit, l_fit, l_osv, n_max, Q_out, w_out, n_osv, rows);
  });
}

int mbe3_pair_K_fit(mbe3_handle *h, const double *s_fit, double l_fit, double *K,
                    int64_t k_elems) {
  if (!h) return MBE3_EINVAL;
  return no_throw(h, [&] { return pair_k_fit_body(h, s_fit, l_fit, K, k_elems); });
}

int mbe3_project_fit(mbe3_handle *h, const double *s_fit, double l_fit, double *gamma,
                     int64_t gamma_elems) {
  if (!h) return MBE3_EINVAL;
  return no_throw(h, [&] { return project_fit_body(h, s_fit, l_fit, gamma, gamma_elems); });
}

int mbe3_screen(mbe3_handle *h, const int32_t *pairs, int64_t n, double *s2b) {
  if (!h) return MBE3_EINVAL;
  return no_throw(h, [&] { return screen_body(h, pairs, n, s2b); });
}

int mbe3_weak_pairs(mbe3_handle *h, const int32_t *pairs, int64_t n, const double *gamma,
                    const double *W, double *e) {
  if (!h) return MBE3_EINVAL;
  return no_throw(h, [&] { return weak_body(h, pairs, n, gamma, W, e); });
}

// Retile list li for `shape` and upload its tasks (stream idle).
static int set_list_shape(mbe3_handle *h, int li, GemmShape shape) {
  GemmList &L = h->glists[li];
  std::vector<GemmTask> ts = L.host;
  const int64_t tiles = finish_tasks(ts, shape);
  if (tiles > 0x7fffffffLL) return h->fail(MBE3_EINVAL, "%s: too many tiles for %s",
                                            L.name.c_str(), gemm_shape_name(shape));
  if (!ts.empty())
    HIP_TRY(h, hipMemcpy(L.d, ts.data(), ts.size() * sizeof(GemmTask),
                         hipMemcpyHostToDevice));
  L.host.swap(ts);
  L.tiles = tiles;
  L.shape = shape;
  return MBE3_OK;
}

int mbe3_autotune(mbe3_handle *h, double *gamma, int64_t gamma_elems, double *K,
                  int64_t k_elems, double *dB, int64_t dB_elems, int reps) {
  if (!h) return MBE3_EINVAL;
  if (h->dry) return h->fail(MBE3_EINVAL, "plan-only handle");
  if (h->recording) return h->fail(MBE3_EINVAL, "not available while recording");
  if (!gamma || gamma_elems < h->gamma_rows * h->n_aux || !K || k_elems < h->k_elems)
    return h->fail(MBE3_EINVAL, "gamma and K of the layout's sizes are required");
  const int64_t nb = (int64_t)h->n_occ * h->n_vir * h->n_aux;
  if (dB && dB_elems < nb) return h->fail(MBE3_EINVAL, "dB needs %lld doubles", (long long)nb);
  if (reps < 1) reps = 3;
  HIP_TRY(h, hipStreamSynchronize(h->stream));
  release_graph(h);  // its launches were recorded with the old tilings
  GemmBases b = bases(h);
  b.p[B_GAMMA] = gamma;
  b.p[B_K] = K;
  b.p[B_W] = K;  // W lists: the K layout stands in for the multipliers
  b.p[B_DB] = dB;
  GemmBases bg = b;
  bg.rows = h->d_grows;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  HIP_TRY(h, hipEventCreate(&e0));
  HIP_TRY(h, hipEventCreate(&e1));
  std::string rep;
  int rc = MBE3_OK;
  for (size_t li = 0; li < h->glists.size() && rc == MBE3_OK; ++li) {
    GemmList &L = h->glists[li];
    if (L.host.empty()) continue;
    if (L.name == "unproject" && !dB) continue;
    const GemmShape orig = L.shape;
    GemmShape best = orig;
    double best_ms = 1e300;
    char line[512];
    int pos = snprintf(line, sizeof line, "%zu %s (%zu tasks):", li, L.name.c_str(),
                       L.host.size());
    for (int sh = 0; sh < GEMM_NSHAPE && rc == MBE3_OK; ++sh) {
      if ((rc = set_list_shape(h, (int)li, (GemmShape)sh))) break;
      const GemmBases &bb = L.rows_table ? bg : b;
      hipError_t e = launch_list(h, (int)li, bb, h->stream);  // warm-up
      if (e == hipSuccess) e = hipEventRecord(e0, h->stream);
      for (int r = 0; r < reps && e == hipSuccess; ++r) e = launch_list(h, (int)li, bb, h->stream);
      if (e == hipSuccess) e = hipEventRecord(e1, h->stream);
      if (e == hipSuccess) e = hipEventSynchronize(e1);
      float ms = 0.f;
      if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
      if (e != hipSuccess) {
        rc = h->fail(MBE3_EHIP, "autotune %s %s: %s", L.name.c_str(),
                     gemm_shape_name((GemmShape)sh), hipGetErrorString(e));
        break;
      }
      const double per = ms / reps;
      if (pos < (int)sizeof line)
        pos += snprintf(line + pos, sizeof line - pos, " %s %.4f ms",
                        gemm_shape_name((GemmShape)sh), per);
      if (per < best_ms) { best_ms = per; best = (GemmShape)sh; }
    }
    if (rc) break;
    if ((rc = set_list_shape(h, (int)li, best))) break;
    rep += std::string(line) + " -> " + gemm_shape_name(best) + " (planned " +
           gemm_shape_name(orig) + ")\n";
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  h->tune_report = rep;
  return rc;
}

int mbe3_set_gemm_shape(mbe3_handle *h, int list, int shape) {
  if (!h) return MBE3_EINVAL;
  if (h->recording) return h->fail(MBE3_EINVAL, "not available while recording");
  if (shape < 0 || shape >= GEMM_NSHAPE) return h->fail(MBE3_EINVAL, "unknown shape %d", shape);
  if (list < -1 || list >= (int)h->glists.size())
    return h->fail(MBE3_EINVAL, "list %d out of range (%zu lists)", list, h->glists.size());
  if (!h->dry) HIP_TRY(h, hipStreamSynchronize(h->stream));
  release_graph(h);
  for (int li = 0; li < (int)h->glists.size(); ++li) {
    if (list >= 0 && li != list) continue;
    int rc;
    if (h->dry) {
      GemmList &L = h->glists[li];
      L.tiles = finish_tasks(L.host, (GemmShape)shape);
      L.shape = (GemmShape)shape;
    } else if ((rc = set_list_shape(h, li, (GemmShape)shape))) {
      return rc;
    }
  }
  int64_t sz[B_COUNT];
  base_sizes(h, sz);
  for (int li = 0; li < (int)h->glists.size(); ++li) {
    const int rc = check_list(h, li, sz);
    if (rc) return rc;
  }
  return MBE3_OK;
}

const char *mbe3_tune_report(const mbe3_handle *h) {
  if (!h) return "";
  return h->tune_report.c_str();
}

int mbe3_graph_begin(mbe3_handle *h, int with_grad) {
  if (!h) return MBE3_EINVAL;
  if (h->dry) return h->fail(MBE3_EINVAL, "plan-only handle");
  if (h->recording) return h->fail(MBE3_EINVAL, "already recording");
  int rc;
  if (with_grad && (rc = no_throw(h, [&] { return build_grad_plans(h); }))) return rc;
  if (!h->cap_stream)
    HIP_TRY(h, hipStreamCreateWithFlags(&h->cap_stream, hipStreamNonBlocking));
  HIP_TRY(h, hipStreamSynchronize(h->stream));  // a replay may still use the old graph
  release_graph(h);
  HIP_TRY(h, hipStreamBeginCapture(h->cap_stream, hipStreamCaptureModeRelaxed));
  h->user_stream = h->stream;
  h->stream = h->cap_stream;
  h->recording = true;
  h->rec_failed = false;
  h->rec_solve = h->rec_grad = h->rec_energy = false;
  h->seg_phase = -1;
  return MBE3_OK;
}

int mbe3_graph_end(mbe3_handle *h) {
  if (!h) return MBE3_EINVAL;
  if (!h->recording) return h->fail(MBE3_EINVAL, "not recording");
  cut_segment(h, -1, false);
  h->stream = h->user_stream;
  h->recording = false;
  if (h->rec_failed || h->segs.empty()) {
    release_graph(h);
    if (h->segs.empty() && !h->rec_failed) return h->fail(MBE3_EINVAL, "nothing was recorded");
    return h->fail(MBE3_EINVAL, "recording failed: %s", h->err.c_str());
  }
  h->g_solve = h->rec_solve;
  h->g_grad = h->rec_grad;
  h->g_energy = h->rec_energy;
  return MBE3_OK;
}

int mbe3_graph_launch(mbe3_handle *h, double *e_total) {
  if (!h) return MBE3_EINVAL;
  if (h->recording) return h->fail(MBE3_EINVAL, "still recording");
  if (h->segs.empty()) return h->fail(MBE3_EINVAL, "no recorded graph");
  for (auto &sg : h->segs) {
    hipEvent_t a = nullptr, b = nullptr;
    if (h->timing && sg.phase >= 0 && (a = next_event(h)))
      HIP_TRY(h, hipEventRecord(a, h->stream));
    HIP_TRY(h, hipGraphLaunch(sg.x, h->stream));
    if (a && (b = next_event(h))) {
      HIP_TRY(h, hipEventRecord(b, h->stream));
      h->regions.push_back({sg.phase, a, b});
    }
  }
  HIP_TRY(h, hipStreamSynchronize(h->stream));
  if (h->g_solve) {
    h->grad_ready = false;
    const int rc = solve_status(h);
    if (rc) return rc;
    h->grad_ready = h->g_grad;
  }
  if (h->g_energy && e_total) {
    *e_total = h->h_e3[0];
    if (!std::isfinite(*e_total))
      return h->fail(MBE3_ENONFINITE, "MBE(3) energy is not finite");
  }
  return MBE3_OK;
}

}  // extern "C"
