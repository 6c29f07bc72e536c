// C-ABI entry points of the FE step library (declared in include/fe.h).
//
// Structure of one context:
//   host:    pattern + map (two counting-sort transposes), nested-dissection
//            ordering, supernodal symbolic structure and tile schedules;
//            a factor thread that runs the FP64 LDL^T of a snapshot of A
//            (paper Sec. 3.3, asynchronous preconditioner);
//   device:  one caller-owned workspace holding the topology, two factor
//            slots (double buffering: one in use by the solves, the other
//            receiving the next upload on a copy stream), CG vectors and the
//            control block that the kernels read to stop early.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <stdexcept>
#include <string>
#include <thread>
#include <vector>

#include "../../include/fe.h"
#include "device.hpp"
#include "host.hpp"

using namespace fe;

namespace {

thread_local std::string g_build_error;

#define HIP_TRY(expr)                                                                   \
  do {                                                                                  \
    hipError_t e_ = (expr);                                                             \
    if (e_ != hipSuccess) {                                                             \
      return c->fail(FE_EDEVICE, "%s failed: %s", #expr, hipGetErrorString(e_));        \
    }                                                                                   \
  } while (0)

struct Timing {
  int kind;
  hipEvent_t a, b;
  double bytes;
};

struct GraphKey {
  const void *A, *x;
  int slot, tsize;
  bool rot;
  bool operator==(const GraphKey &o) const {
    return A == o.A && x == o.x && slot == o.slot && tsize == o.tsize && rot == o.rot;
  }
};

constexpr int kGraphIters = 2;  // CG iterations per captured graph

// Static device scratch of fe_compliance_noalloc: the blocks of right-hand
// sides live here instead of in a caller workspace.  One copy per GPU, held
// from the first fe_bind on that GPU until the process ends.  In host code
// `scratch` names a host-side shadow, not device memory: its device address
// is looked up once per device with hipGetSymbolAddress and only that address
// is passed to kernels.
constexpr int64_t kScratchBytes = (int64_t)FE_NOALLOC_SCRATCH_BYTES;
__device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_addr[kMaxDevices] = {};

// Device address of `scratch` on the current device `dev` (looked up on the
// first call for that device).
hipError_t scratch_address(int dev, void **out) {
  *out = nullptr;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_addr[dev]) {
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (!p) return hipErrorInvalidSymbol;
    g_scratch_addr[dev] = p;
  }
  *out = g_scratch_addr[dev];
  return hipSuccess;
}

}  // namespace

struct fe_ctx {
  std::string err;
  Pattern P;
  Symbolic S;
  std::vector<double> X;
  int elem_type = 0, nen = 0, n_threads = 0;
  int spmv_lanes = 8;

  // ---- binding
  bool bound = false;
  int prec = FE_PREC_FP64;
  int device = 0;
  size_t tsize = 8;
  char *ws = nullptr;
  int64_t ws_bytes = 0;
  int32_t *d_row_ptr = nullptr, *d_col = nullptr, *d_conn = nullptr, *d_smap = nullptr,
          *d_fds = nullptr, *d_rows = nullptr;
  uint8_t *d_slot = nullptr, *d_dof_fixed = nullptr;
  // assembly without atomics: block lists and the element contribution buffers
  int32_t *d_blk_ptr = nullptr, *d_blk_pos = nullptr, *d_blk_node = nullptr, *d_blk_src = nullptr;
  void *d_ebuf = nullptr;
  double *d_rbuf = nullptr;
  double *d_X = nullptr;
  SnDev *d_sn = nullptr;
  TileDev *d_ftiles = nullptr, *d_btiles = nullptr;
  MTile *d_mftiles = nullptr, *d_mbtiles = nullptr;  // many-right-hand-side sweeps
  int32_t *d_mbdofs = nullptr;                       // own DOFs per backward level
  int *d_herr = nullptr;                             // constraint-matrix index error flag
  char *d_scratch = nullptr;  // device address of the static scratch (this device)
  std::string scratch_err;    // why it is unavailable, if it is
  void *d_panels[2] = {nullptr, nullptr}, *d_dinv[2] = {nullptr, nullptr};
  double *d_jdinv = nullptr;
  double *d_r = nullptr, *d_z = nullptr, *d_p = nullptr, *d_q = nullptr, *d_tmp = nullptr;
  double *d_b = nullptr, *d_a = nullptr, *d_abar = nullptr, *d_mu = nullptr;
  double *d_Kmu = nullptr, *d_Mmu = nullptr, *d_Tmv = nullptr;
  void *d_w = nullptr, *d_y = nullptr, *d_A = nullptr;
  double *d_part1 = nullptr, *d_part2 = nullptr;
  PcgState *d_state = nullptr;

  // ---- host-side HIP resources
  PcgState *h_state = nullptr;
  void *h_Asnap = nullptr;
  void *h_stage = nullptr;   // panels (T) followed by dinv (T)
  hipStream_t copy_stream = nullptr;
  hipEvent_t ev_snap_ready = nullptr, ev_snap_done = nullptr, ev_upload_done = nullptr;
  hipEvent_t ev_slot_free[2] = {nullptr, nullptr};
  bool upload_issued = false;

  // ---- factor thread
  std::thread th;
  std::mutex mu;
  std::condition_variable cv;
  bool quit = false, job_pending = false, job_running = false;
  int64_t job_tag = -1, ready_tag = -1;
  int job_status = FE_OK;
  std::string job_err;
  double last_factor_seconds = 0.0;
  int active_slot = -1;
  int64_t installed_tag = -1;
  int64_t step_count = 0;
  bool have_prev_a = false;
  // ring of earlier step solutions for the projected initial guess
  double *d_histV = nullptr, *d_histW = nullptr, *d_histP = nullptr;
  int hist_count = 0, hist_next = 0;
  // rotation of the stale factor: node accumulators, rotations of the
  // current state, of the state of each factor job (two, alternating) and of
  // the factor in each slot; Q = R_now R_slot^T in the context precision
  int32_t *d_ne_ptr = nullptr, *d_ne_idx = nullptr;  // elements of each node (rotations)
  double *d_rotFe = nullptr, *d_Rnow = nullptr, *d_Rjob[2] = {nullptr, nullptr},
         *d_Rslot[2] = {nullptr, nullptr};
  void *d_rotQ = nullptr;
  bool rot_valid = false;  // d_Rnow holds the rotations of this step's state
  bool rot_on = false;     // the solve in progress applies Q P^{-1} Q^T
  int job_count = 0, job_rbuf = 0, gf_rbuf = 0, ready_rbuf = 0;

  // ---- GPU factorisation (factor_on_gpu)
  bool gpu_factor = false;
  int gf_max_blocks = 0;
  GfPlan G;
  GfDev gd{};
  void *d_Asnap = nullptr;
  int *h_gf_status = nullptr;
  hipStream_t factor_stream = nullptr;
  hipEvent_t ev_gf_done = nullptr;
  bool gf_pending = false;
  int64_t gf_tag = -1;
  int gf_slot = -1, ready_slot = -1;

  // ---- graphs of CG iterations
  bool use_graphs = true;
  hipStream_t cap_stream = nullptr;
  std::vector<std::pair<GraphKey, hipGraphExec_t>> graphs;

  // ---- timing
  bool timing = false;
  std::vector<Timing> tq;
  std::vector<hipEvent_t> ev_pool;
  static constexpr int kTimedKinds = 6;
  double t_ms[kTimedKinds] = {}, t_bytes[kTimedKinds] = {};
  int64_t t_count[kTimedKinds] = {};
  int *h_flag = nullptr;  // pinned host word for error flags read back
  std::vector<double> fwd_level_bytes, bwd_level_bytes;
  // the sweeps read the panels non-temporally when one factor slot exceeds
  // the 256 MB last-level cache (a smaller factor stays cached between
  // applications)
  bool panel_stream = false;

  int fail(int code, const char *fmt, ...) {
    char buf[1024];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    err = buf;
    return code;
  }
  ~fe_ctx();
};

namespace {

// ------------------------------------------------------------- layout
struct Layout {
  static constexpr int kMax = 80;
  int64_t off[kMax];
  int64_t total = 0;
  int k = 0;
  int64_t add(int64_t bytes) {
    const int64_t o = total;
    if (k >= kMax) throw std::runtime_error("workspace layout: too many sections");
    off[k++] = o;
    total += (bytes + 255) / 256 * 256;
    return o;
  }
};

enum {
  L_ROWPTR, L_COL, L_CONN, L_SLOT, L_SMAP, L_FDS, L_DOFFIX, L_X, L_SN, L_ROWS, L_FT, L_BT,
  L_PAN0, L_PAN1, L_DINV0, L_DINV1, L_JDINV, L_R, L_Z, L_P, L_Q, L_TMP, L_B, L_ACC, L_ABAR,
  L_MU, L_KMU, L_MMU, L_TMV, L_W, L_Y, L_A, L_PART1, L_PART2, L_STATE, L_GF_FRONTS, L_GF_FR,
  L_GF_LVLSN, L_GF_ACSR, L_GF_AOFF, L_GF_PARENT, L_GF_REL, L_GF_RELOFF, L_GF_EXT, L_GF_PANELSN,
  L_GF_UPD, L_GF_ASNAP, L_GF_STATUS, L_BLKPTR, L_BLKPOS, L_BLKNODE, L_BLKSRC, L_EBUF, L_RBUF,
  L_MFT, L_MBT, L_HERR, L_MBDOF, L_HISTV, L_HISTW, L_HISTP, L_NEPTR, L_NEIDX, L_ROTFE, L_RNOW,
  L_RJOB0, L_RJOB1, L_RSLOT0, L_RSLOT1, L_ROTQ
};

Layout make_layout(const fe_ctx *c, int prec) {
  const Pattern &P = c->P;
  const Symbolic &S = c->S;
  const int64_t ts = prec == FE_PREC_MIXED ? 4 : 8;
  const int64_t n = P.n, nnz = (int64_t)P.col_idx.size();
  const int64_t np = cg_blocks(n) + 16;
  const int64_t spmv_parts = (n * c->spmv_lanes + 255) / 256 + 16;
  Layout L;
  L.add((n + 1) * 4);
  L.add(nnz * 4);
  L.add((int64_t)P.conn.size() * 4);
  L.add(P.compact_ok ? (int64_t)P.slot.size() : 0);
  L.add(P.compact_ok ? 0 : (int64_t)P.tmap.size() * 4);
  L.add((int64_t)P.fixed_diag_slot.size() * 4);
  L.add(n);
  L.add(n * 8);
  L.add((int64_t)S.sn.size() * (int64_t)sizeof(SnDev));
  L.add((int64_t)S.rows.size() * 4);
  L.add((int64_t)S.fwd_tiles.size() * (int64_t)sizeof(TileDev));
  L.add((int64_t)S.bwd_tiles.size() * (int64_t)sizeof(TileDev));
  L.add(S.dev_panel_entries * ts);
  L.add(S.dev_panel_entries * ts);
  L.add(n * ts);
  L.add(n * ts);
  L.add(n * 8);  // jdinv
  for (int i = 0; i < 12; ++i) L.add(n * 8);  // r z p q tmp b a abar mu Kmu Mmu Tmv
  L.add(n * ts);  // w
  L.add(n * ts);  // y
  L.add(nnz * ts);
  L.add(std::max(np, spmv_parts) * 8);
  L.add(std::max(np, spmv_parts) * 8);
  L.add(256);
  const bool g = c->gpu_factor;
  const GfPlan &Gp = c->G;
  L.add(g ? Gp.doubles * 8 : 0);
  L.add(g ? (int64_t)Gp.fr.size() * (int64_t)sizeof(GfFront) : 0);
  L.add(g ? (int64_t)Gp.lvl_sn.size() * 4 : 0);
  L.add(g ? (int64_t)Gp.a_csr.size() * 4 : 0);
  L.add(g ? (int64_t)Gp.a_off.size() * 8 : 0);
  L.add(g ? (int64_t)Gp.parent.size() * 4 : 0);
  L.add(g ? (int64_t)Gp.rel.size() * 4 : 0);
  L.add(g ? (int64_t)Gp.rel_off.size() * 8 : 0);
  L.add(g ? (int64_t)Gp.ext.size() * (int64_t)sizeof(GfExt) : 0);
  L.add(g ? (int64_t)Gp.panel_sn.size() * 4 : 0);
  L.add(g ? (int64_t)Gp.upd.size() * (int64_t)sizeof(GfTile) : 0);
  L.add(g ? nnz * ts : 0);
  L.add(g ? 256 : 0);
  const bool cg = P.compact_ok;
  const int64_t nen = P.nen;
  L.add(cg ? (int64_t)P.blk_ptr.size() * 4 : 0);
  L.add(cg ? (int64_t)P.blk_pos.size() * 4 : 0);
  L.add(cg ? (int64_t)P.blk_node.size() * 4 : 0);
  L.add(cg ? (int64_t)P.blk_src.size() * 4 : 0);
  L.add(cg ? (int64_t)P.n_elems * (nen * (nen + 1) / 2) * 9 * ts : 0);  // blocks a <= b
  L.add(cg ? (int64_t)P.n_elems * nen * 3 * 8 : 0);
  L.add((int64_t)S.mfwd_tiles.size() * (int64_t)sizeof(MTile));
  L.add((int64_t)S.mbwd_tiles.size() * (int64_t)sizeof(MTile));
  L.add(256);
  L.add((int64_t)S.mbwd_dofs.size() * 4);
  L.add(n * kHist * 8);  // earlier solutions (initial-guess projection)
  L.add(n * kHist * 8);  // A times them
  L.add(hist_part_doubles() * 8);
  const int64_t nn = n / 3;
  L.add((nn + 1) * 4);                             // elements of each node: offsets,
  L.add((int64_t)P.n_elems * P.nen * 4);           //   element indices
  L.add((int64_t)P.n_elems * 9 * 8);               // element-centre deformation gradients
  for (int i = 0; i < 5; ++i) L.add(nn * 9 * 8);  // R_now, R_job x2, R_slot x2
  L.add(nn * 9 * ts);                              // Q
  return L;
}

template <typename T>
T *ptr_at(char *ws, const Layout &L, int k) {
  return reinterpret_cast<T *>(ws + L.off[k]);
}

ElemParams to_elem(const fe_params *p) {
  ElemParams e;
  e.h = p->h;
  e.alpha = p->alpha;
  e.beta = p->beta;
  e.rho = p->rho;
  e.nu = p->nu;
  e.gx = p->gravity[0];
  e.gy = p->gravity[1];
  e.gz = p->gravity[2];
  e.material = p->material;
  e.pad = 0;
  e.mr_c01_share = p->mr_c01_share;
  return e;
}

// ------------------------------------------------------------- timing
hipEvent_t take_event(fe_ctx *c) {
  if (!c->ev_pool.empty()) {
    hipEvent_t e = c->ev_pool.back();
    c->ev_pool.pop_back();
    return e;
  }
  // timing-only events: no system-scope fence on record, so the marker does
  // not write back and invalidate the L2s between the timed kernels
  hipEvent_t e = nullptr;
  (void)hipEventCreateWithFlags(&e, hipEventDisableSystemFence);
  return e;
}

void drain_timing(fe_ctx *c) {
  for (auto &t : c->tq) {
    (void)hipEventSynchronize(t.b);
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, t.a, t.b) == hipSuccess) {
      c->t_ms[t.kind] += ms;
      c->t_count[t.kind] += 1;
      c->t_bytes[t.kind] += t.bytes;
    }
    c->ev_pool.push_back(t.a);
    c->ev_pool.push_back(t.b);
  }
  c->tq.clear();
}

struct TimedLaunch {
  fe_ctx *c;
  hipStream_t st;
  Timing t;
  bool on;
  TimedLaunch(fe_ctx *c_, hipStream_t s, int kind, double bytes) : c(c_), st(s), on(c_->timing) {
    if (on) {
      t.kind = kind;
      t.bytes = bytes;
      t.a = take_event(c);
      t.b = take_event(c);
      (void)hipEventRecord(t.a, st);
    }
  }
  ~TimedLaunch() {
    if (on) {
      (void)hipEventRecord(t.b, st);
      c->tq.push_back(t);
      if (c->tq.size() > 4096) drain_timing(c);
    }
  }
};

// ------------------------------------------------------------- factor thread
template <typename T>
void stage_factor(fe_ctx *c, const std::vector<double> &panels, const std::vector<double> &dinv) {
  // host panels (leading dimension m) to the device layout (leading
  // dimension ld, the padding rows zero)
  T *dst = reinterpret_cast<T *>(c->h_stage);
  const std::vector<Supernode> &sn = c->S.sn;
  const int64_t ns = (int64_t)sn.size();
  parallel_for(64, c->n_threads, [&](int64_t b, int) {
    for (int64_t s = ns * b / 64; s < ns * (b + 1) / 64; ++s) {
      const Supernode &q = sn[s];
      for (int64_t j = 0; j < q.nc; ++j) {
        const double *src = panels.data() + q.panel_off + j * q.m;
        T *d = dst + q.dev_off + j * q.ld;
        for (int64_t i = 0; i < q.m; ++i) d[i] = (T)src[i];
        for (int64_t i = q.m; i < q.ld; ++i) d[i] = T(0);
      }
    }
  });
  T *dd = dst + c->S.dev_panel_entries;
  for (size_t i = 0; i < dinv.size(); ++i) dd[i] = (T)dinv[i];
}

void factor_main(fe_ctx *c) {
  (void)hipSetDevice(c->device);
  for (;;) {
    int64_t tag;
    int rbuf;
    {
      std::unique_lock<std::mutex> lk(c->mu);
      c->cv.wait(lk, [&] { return c->quit || c->job_pending; });
      if (c->quit) return;
      c->job_pending = false;
      c->job_running = true;
      tag = c->job_tag;
      rbuf = c->job_rbuf;
    }
    const auto t0 = std::chrono::steady_clock::now();
    std::string e;
    std::vector<double> panels, dinv;
    if (hipEventSynchronize(c->ev_snap_done) != hipSuccess) e = "snapshot copy failed";
    if (e.empty()) {
      if (c->prec == FE_PREC_MIXED)
        e = factorize<float>(c->P, c->S, (const float *)c->h_Asnap, c->n_threads, panels, dinv);
      else
        e = factorize<double>(c->P, c->S, (const double *)c->h_Asnap, c->n_threads, panels, dinv);
    }
    std::unique_lock<std::mutex> lk(c->mu);
    if (e.empty()) {
      // the staging buffer may still be feeding the previous upload
      if (c->upload_issued) (void)hipEventSynchronize(c->ev_upload_done);
      if (c->prec == FE_PREC_MIXED) stage_factor<float>(c, panels, dinv);
      else stage_factor<double>(c, panels, dinv);
      c->ready_tag = tag;
      c->ready_rbuf = rbuf;
      c->job_status = FE_OK;
      c->job_err.clear();
    } else {
      c->job_status = FE_EFACTOR;
      c->job_err = e;
    }
    c->last_factor_seconds =
        std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    c->job_running = false;
    c->cv.notify_all();
  }
}

// ------------------------------------------------------------- solve pieces
// z = P^{-1} r.  With skip_prep the sweep inputs (w = r, y = 0, z = 0 / r on
// fixed DOFs) were already written by the fused x/r update.
template <typename T>
void precond(fe_ctx *c, const T *A, const double *r, double *z, hipStream_t st, bool use_state,
             bool skip_prep = false) {
  const int64_t n = c->P.n;
  const PcgState *s = use_state ? c->d_state : nullptr;
  if (c->active_slot < 0) {
    launch_jacobi(st, n, c->d_jdinv, r, z, s);
    return;
  }
  (void)A;
  const int slot = c->active_slot;
  const T *pan = (const T *)c->d_panels[slot];
  const T *dinv = (const T *)c->d_dinv[slot];
  T *w = (T *)c->d_w, *y = (T *)c->d_y;
  if (!skip_prep) launch_tri_prep<T>(st, n, r, w, y, z, c->d_dof_fixed, s);
  if (c->rot_on) launch_rot_in<T>(st, n / 3, (const T *)c->d_rotQ, r, w, s);
  const Symbolic &S = c->S;
  for (int L = 0; L < S.n_levels; ++L) {
    const int b = S.fwd_level_ptr[L], e = S.fwd_level_ptr[L + 1];
    TimedLaunch tl(c, st, 1, c->fwd_level_bytes[L]);
    launch_tri_fwd<T>(st, c->d_ftiles + b, e - b, c->d_rows, pan, w, y, s, S.fwd_level_cols[L],
                      S.fwd_level_groups[L], c->panel_stream);
  }
  for (int L = 0; L < S.n_levels; ++L) {  // L-th backward launch: level n_levels - 1 - L
    const int b = S.bwd_level_ptr[L], e = S.bwd_level_ptr[L + 1];
    TimedLaunch tl(c, st, 2, c->bwd_level_bytes[L]);
    launch_tri_bwd<T>(st, c->d_btiles + b, e - b, c->d_rows, pan, dinv, y, z, s,
                      S.bwd_level_rows[S.n_levels - 1 - L], S.bwd_level_cols[S.n_levels - 1 - L],
                      c->panel_stream);
  }
  if (c->rot_on) launch_rot_out<T>(st, n / 3, (const T *)c->d_rotQ, z, s);
}

// Workspace of the many-right-hand-side calls: an error word, then the
// DOF-major n x ld blocks w, y (factor precision) and z (FP64).
struct MultiWs {
  int bn = 64, ld = 0;
  int64_t off_w = 0, off_y = 0, off_z = 0, total = 0;
};

MultiWs multi_ws(const fe_ctx *c, int k) {
  MultiWs m;
  m.bn = k <= 64 ? 64 : 128;
  m.ld = (k + m.bn - 1) / m.bn * m.bn;
  const int64_t n = c->P.n;
  auto r256 = [](int64_t b) { return (b + 255) / 256 * 256; };
  m.off_w = 0;
  m.off_y = r256(n * m.ld * (int64_t)c->tsize);
  m.off_z = m.off_y + r256(n * m.ld * (int64_t)c->tsize);
  m.total = m.off_z + r256(n * m.ld * 8);
  return m;
}

// Z = P^{-1} R for the prepared blocks: level-ordered forward tiles, then
// backward tiles (the same dependency levels as the single sweeps).
template <typename T>
void multi_sweeps(fe_ctx *c, const MultiWs &m, int k, T *w, T *y, double *z, hipStream_t st) {
  const int slot = c->active_slot;
  const T *pan = (const T *)c->d_panels[slot];
  const T *dinv = (const T *)c->d_dinv[slot];
  const Symbolic &S = c->S;
  const int nkb = m.ld / m.bn;
  for (int L = 0; L < S.n_levels; ++L) {
    const int b = S.mfwd_level_ptr[L], e = S.mfwd_level_ptr[L + 1];
    TimedLaunch tl(c, st, 4, 2.0 * S.level_lower[L] * k);
    launch_multi_fwd<T>(st, c->d_mftiles + b, e - b, nkb, m.bn, c->d_sn, c->d_rows, pan, w, y,
                        m.ld, k);
  }
  for (int L = 0; L < S.n_levels; ++L) {
    const int b = S.mbwd_level_ptr[L], e = S.mbwd_level_ptr[L + 1];
    {
      TimedLaunch tl(c, st, 5, 2.0 * S.level_lower[S.n_levels - 1 - L] * k);
      launch_multi_bwd<T>(st, c->d_mbtiles + b, e - b, nkb, m.bn, c->d_sn, c->d_rows, pan, dinv,
                          y, z, m.ld, k);
    }
    if (L + 1 < S.n_levels) {
      const int32_t d0 = S.mbwd_dof_ptr[L], d1 = S.mbwd_dof_ptr[L + 1];
      launch_multi_conv<T>(st, c->d_mbdofs + d0, d1 - d0, m.ld, z, y);
    }
  }
}

template <typename T>
void precond_multi(fe_ctx *c, const MultiWs &m, const double *R, double *Z, int k, char *work,
                   hipStream_t st) {
  T *w = (T *)(work + m.off_w), *y = (T *)(work + m.off_y);
  double *z = (double *)(work + m.off_z);
  launch_multi_prep<T>(st, c->P.n, k, m.ld, R, w, y, z, c->d_dof_fixed);
  multi_sweeps<T>(c, m, k, w, y, z, st);
  launch_multi_out(st, c->P.n, k, m.ld, z, Z);
}

template <typename T>
void compliance(fe_ctx *c, const MultiWs &m, int k, const int32_t *hrp, const int32_t *hcol,
                const double *hval, int64_t nnz_h, double *W, double *Z, char *work,
                hipStream_t st) {
  const int64_t n = c->P.n;
  T *w = (T *)(work + m.off_w), *y = (T *)(work + m.off_y);
  double *z = (double *)(work + m.off_z);
  launch_multi_zero<T>(st, n * m.ld, w, y, z);
  launch_h_scatter<T>(st, k, n, nnz_h, hrp, hcol, hval, m.ld, w, z, c->d_dof_fixed, c->d_herr);
  multi_sweeps<T>(c, m, k, w, y, z, st);
  launch_hz(st, k, n, nnz_h, hrp, hcol, hval, m.ld, z, W);
  if (Z) launch_multi_out(st, n, k, m.ld, z, Z);
}

template <typename T>
void spmv(fe_ctx *c, const T *A, const double *x, double *y, const double *w, double *part,
          int *np, hipStream_t st, const PcgState *s) {
  const double nnz = (double)c->P.col_idx.size(), n = (double)c->P.n;
  TimedLaunch tl(c, st, 0, nnz * (sizeof(T) + 4) + (n + 1) * 4 + n * 8 * 2);
  launch_spmv<T>(st, c->P.n, c->spmv_lanes, c->d_row_ptr, c->d_col, A, x, y, w, part, np, s);
}

// One CG iteration: q = A p with alpha; x, r update (+ sweep inputs); z = P^{-1} r;
// beta; p = z + beta p.  Every kernel returns at once when the done flag is set.
template <typename T>
void cg_iteration(fe_ctx *c, const T *A, double *x, hipStream_t st) {
  const int64_t n = c->P.n;
  const bool tri = c->active_slot >= 0;
  int np = 0;
  spmv<T>(c, A, c->d_p, c->d_q, c->d_p, c->d_part1, &np, st, c->d_state);
  // the SpMV's partials are summed in two stages, the first into part2
  // (free until the update below writes its own partials there)
  launch_ctl_alpha(st, c->d_state, c->d_part1, np, c->d_part2);
  launch_update_xr_prep<T>(st, n, x, c->d_r, c->d_p, c->d_q, c->d_part2, c->d_state,
                           tri ? (T *)c->d_w : nullptr, (T *)c->d_y, c->d_z, c->d_dof_fixed);
  launch_ctl_rr(st, c->d_state, c->d_part2, cg_blocks(n));
  precond<T>(c, A, c->d_r, c->d_z, st, true, tri);
  launch_dot(st, n, c->d_r, c->d_z, c->d_part1, c->d_state);
  launch_ctl_rz(st, c->d_state, c->d_part1, cg_blocks(n), 0);
  launch_update_p(st, n, c->d_p, c->d_z, c->d_state, 0);
}

// A HIP graph of kGraphIters CG iterations for (A, x, factor slot), captured
// on the context's private stream and replayed on the caller's stream.  The
// graph holds kernel nodes only (no memset/copy nodes).
template <typename T>
hipGraphExec_t iter_graph(fe_ctx *c, const T *A, double *x) {
  const GraphKey key{(const void *)A, (const void *)x, c->active_slot, (int)sizeof(T),
                     c->rot_on};
  for (auto &kv : c->graphs)
    if (kv.first == key) return kv.second;
  hipGraph_t g = nullptr;
  hipGraphExec_t ex = nullptr;
  if (hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeThreadLocal) != hipSuccess) {
    c->use_graphs = false;
    return nullptr;
  }
  for (int k = 0; k < kGraphIters; ++k) cg_iteration<T>(c, A, x, c->cap_stream);
  if (hipStreamEndCapture(c->cap_stream, &g) != hipSuccess || !g ||
      hipGraphInstantiate(&ex, g, nullptr, nullptr, 0) != hipSuccess) {
    if (g) (void)hipGraphDestroy(g);
    (void)hipGetLastError();
    c->use_graphs = false;
    return nullptr;
  }
  (void)hipGraphDestroy(g);
  if (c->graphs.size() >= 8) {
    (void)hipGraphExecDestroy(c->graphs.front().second);
    c->graphs.erase(c->graphs.begin());
  }
  c->graphs.push_back({key, ex});
  return ex;
}

int read_state(fe_ctx *c, hipStream_t st) {
  {
    hipError_t e1 = hipMemcpyAsync(c->h_state, c->d_state, sizeof(PcgState),
                                   hipMemcpyDeviceToHost, st);
    if (e1 != hipSuccess) return c->fail(FE_EDEVICE, "state copy: %s", hipGetErrorString(e1));
    hipError_t e2 = hipStreamSynchronize(st);
    if (e2 != hipSuccess) return c->fail(FE_EDEVICE, "stream sync: %s", hipGetErrorString(e2));
  }
  return FE_OK;
}

template <typename T>
int pcg(fe_ctx *c, const T *A, const double *b, double *x, double tol, int max_it,
        hipStream_t st, fe_solve_stats *out) {
  const int64_t n = c->P.n;
  const int nb = cg_blocks(n);
  int np = 0;
  if (c->active_slot < 0) launch_diag_inv<T>(st, n, c->d_row_ptr, c->d_col, A, c->d_jdinv);
  // r = b - A x
  spmv<T>(c, A, x, c->d_tmp, nullptr, nullptr, nullptr, st, nullptr);
  launch_residual(st, n, b, c->d_tmp, c->d_r, c->d_part1, c->d_part2);
  launch_ctl_init(st, c->d_state, c->d_part1, c->d_part2, nb, tol);
  (void)np;
  auto restart = [&]() {
    precond<T>(c, A, c->d_r, c->d_z, st, true);
    launch_dot(st, n, c->d_r, c->d_z, c->d_part1, c->d_state);
    launch_ctl_rz(st, c->d_state, c->d_part1, nb, 1);
    launch_update_p(st, n, c->d_p, c->d_z, c->d_state, 1);
  };
  restart();
  int chunk = std::min(2, max_it);
  int status = FE_OK;
  int restarts = 0;
  int32_t last_it = -1;
  for (;;) {
    hipGraphExec_t g = c->use_graphs && !c->timing ? iter_graph<T>(c, A, x) : nullptr;
    if (g) {
      // whole graphs, then the remainder of the chunk (at most
      // kGraphIters - 1 iterations) as eager launches, so that no batch runs
      // past max_it
      int k = 0;
      for (; k + kGraphIters <= chunk; k += kGraphIters) {
        hipError_t e = hipGraphLaunch(g, st);
        if (e != hipSuccess) return c->fail(FE_EDEVICE, "graph launch: %s", hipGetErrorString(e));
      }
      for (; k < chunk; ++k) cg_iteration<T>(c, A, x, st);
    } else {
      for (int k = 0; k < chunk; ++k) cg_iteration<T>(c, A, x, st);
    }
    {
      hipError_t le = hipGetLastError();
      if (le != hipSuccess) return c->fail(FE_EDEVICE, "kernel launch: %s", hipGetErrorString(le));
    }
    int rc = read_state(c, st);
    if (rc) return rc;
    const PcgState &h = *c->h_state;
    if (!h.done && h.status == 0 && h.it == last_it)
      return c->fail(FE_EDEVICE, "CG iteration counter did not advance");
    last_it = h.it;
    if (h.status == 4) {
      status = FE_EINDEF;
      break;
    }
    if (h.done) {
      // certify with the recomputed FP64 residual
      spmv<T>(c, A, x, c->d_tmp, nullptr, nullptr, nullptr, st, nullptr);
      launch_residual(st, n, b, c->d_tmp, c->d_r, c->d_part1, nullptr);
      launch_ctl_true(st, c->d_state, c->d_part1, nb);
      rc = read_state(c, st);
      if (rc) return rc;
      if (c->h_state->rr_true <= c->h_state->tol2 || c->h_state->bb == 0.0) break;
      if (++restarts > 50) {
        status = FE_ENOTCONV;
        break;
      }
      // residual replacement: continue from the true residual
      c->h_state->done = 0;
      hipError_t e = hipMemcpyAsync(&c->d_state->done, &c->h_state->done, sizeof(int32_t),
                                    hipMemcpyHostToDevice, st);
      if (e != hipSuccess) return c->fail(FE_EDEVICE, "state reset: %s", hipGetErrorString(e));
      restart();
      continue;
    }
    if (h.it >= max_it) {
      status = FE_ENOTCONV;
      spmv<T>(c, A, x, c->d_tmp, nullptr, nullptr, nullptr, st, nullptr);
      launch_residual(st, n, b, c->d_tmp, c->d_r, c->d_part1, nullptr);
      launch_ctl_true(st, c->d_state, c->d_part1, nb);
      rc = read_state(c, st);
      if (rc) return rc;
      break;
    }
    chunk = std::min(16, std::max(2, chunk * 2));
    chunk = std::min(chunk, max_it - h.it);
    if (chunk <= 0) chunk = 1;
  }
  if (out) {
    out->iterations = c->h_state->it;
    out->status = status;
    out->rel_res = c->h_state->bb > 0 ? std::sqrt(c->h_state->rr_true / c->h_state->bb) : 0.0;
    out->factor_tag = c->active_slot >= 0 ? c->installed_tag : -1;
  }
  if (status == FE_EINDEF) return c->fail(FE_EINDEF, "CG breakdown: p^T A p <= 0");
  if (status == FE_ENOTCONV)
    return c->fail(FE_ENOTCONV, "CG did not converge in %d iterations", c->h_state->it);
  return FE_OK;
}

template <typename T>
int assemble(fe_ctx *c, const fe_params *p, const double *q, const double *v, T *A, double *b,
             hipStream_t st) {
  const ElemParams ep = to_elem(p);
  const bool gather = c->P.compact_ok;
  launch_assembly_init<T>(st, (int64_t)c->P.col_idx.size(), A,
                          (int64_t)c->P.fixed_diag_slot.size(), c->d_fds, c->P.n, b,
                          p->f_nodal, c->d_dof_fixed, !gather);
  const double bytes = (double)c->P.col_idx.size() * sizeof(T) + 8.0 * c->P.n +
                       (4.0 * c->nen + 8.0 + (c->P.compact_ok ? c->nen * c->nen : 36.0 * c->nen * c->nen)) *
                           c->P.n_elems + 72.0 * c->P.n_nodes;
  TimedLaunch tl(c, st, 3, bytes);
  launch_element<T>(st, c->elem_type, c->P.n_elems, c->d_conn,
                    c->P.compact_ok ? c->d_slot : nullptr, c->P.compact_ok ? nullptr : c->d_smap,
                    c->d_row_ptr, c->d_X, q, v, p->E, c->d_dof_fixed, ep, A, b,
                    static_cast<T *>(c->d_ebuf), c->d_rbuf, c->d_state);
  if (gather)
    launch_assembly_gather<T>(st, c->nen, (int64_t)c->P.blk_pos.size(), c->d_blk_ptr,
                              c->d_blk_src, c->d_blk_pos, c->d_blk_node, c->d_row_ptr,
                              static_cast<const T *>(c->d_ebuf), c->d_rbuf, p->f_nodal, A, b);
  return FE_OK;
}

int check_params(fe_ctx *c, const fe_params *p) {
  if (!p) return c->fail(FE_EINVAL, "params is NULL");
  if (!p->E) return c->fail(FE_EINVAL, "params->E is NULL");
  if (p->material != FE_NEO_HOOKEAN && p->material != FE_STVK &&
      p->material != FE_COROTATIONAL && p->material != FE_MOONEY_RIVLIN)
    return c->fail(FE_EINVAL, "unknown material %d", p->material);
  if (p->material == FE_MOONEY_RIVLIN && !(p->mr_c01_share >= 0.0 && p->mr_c01_share <= 1.0))
    return c->fail(FE_EINVAL, "mr_c01_share must be in [0, 1]");
  if (!(p->h > 0)) return c->fail(FE_EINVAL, "h must be positive");
  if (!(p->nu > -1.0 && p->nu < 0.5)) return c->fail(FE_EINVAL, "nu out of range");
  return FE_OK;
}

int clear_elem_status(fe_ctx *c, hipStream_t st) {
  c->h_state->elem_status = 0;
  hipError_t e = hipMemcpyAsync(&c->d_state->elem_status, &c->h_state->elem_status,
                                sizeof(int32_t), hipMemcpyHostToDevice, st);
  if (e != hipSuccess) return c->fail(FE_EDEVICE, "status reset: %s", hipGetErrorString(e));
  // the pinned source must not change before the copy has run
  e = hipStreamSynchronize(st);
  if (e != hipSuccess) return c->fail(FE_EDEVICE, "stream sync: %s", hipGetErrorString(e));
  return FE_OK;
}

// ---- GPU factorisation job bookkeeping (caller holds c->mu)
int gf_collect_locked(fe_ctx *c, bool block) {
  if (!c->gf_pending) return FE_OK;
  if (!block && hipEventQuery(c->ev_gf_done) == hipErrorNotReady) return FE_OK;
  HIP_TRY(hipEventSynchronize(c->ev_gf_done));
  HIP_TRY(hipMemcpyAsync(c->h_gf_status, c->gd.status, sizeof(int), hipMemcpyDeviceToHost,
                         c->factor_stream));
  HIP_TRY(hipStreamSynchronize(c->factor_stream));
  c->gf_pending = false;
  if (*c->h_gf_status) {
    c->job_status = FE_EFACTOR;
    c->job_err = "non-positive pivot in the GPU LDL^T";
  } else {
    c->job_status = FE_OK;
    c->job_err.clear();
    c->ready_tag = c->gf_tag;
    c->ready_slot = c->gf_slot;
    c->ready_rbuf = c->gf_rbuf;
  }
  return FE_OK;
}

bool factor_busy_locked(fe_ctx *c) {
  if (c->gpu_factor) {
    (void)gf_collect_locked(c, false);
    return c->gf_pending;
  }
  return c->job_pending || c->job_running;
}

int install_locked(fe_ctx *c, hipStream_t st) {
  if (c->gpu_factor) {
    int rc = gf_collect_locked(c, false);
    if (rc) return rc;
    if (c->ready_tag < 0 || c->ready_tag == c->installed_tag || c->ready_slot < 0) return FE_OK;
    HIP_TRY(hipStreamWaitEvent(st, c->ev_gf_done, 0));
    HIP_TRY(hipMemcpyAsync(c->d_Rslot[c->ready_slot], c->d_Rjob[c->ready_rbuf],
                           (size_t)(c->P.n / 3) * 72, hipMemcpyDeviceToDevice, st));
    if (c->active_slot >= 0) HIP_TRY(hipEventRecord(c->ev_slot_free[c->active_slot], st));
    c->active_slot = c->ready_slot;
    c->installed_tag = c->ready_tag;
    return FE_OK;
  }
  if (c->ready_tag < 0 || c->ready_tag == c->installed_tag) return FE_OK;
  const int slot = c->active_slot < 0 ? 0 : 1 - c->active_slot;
  const size_t pan_bytes = (size_t)c->S.dev_panel_entries * c->tsize;
  const size_t dinv_bytes = (size_t)c->P.n * c->tsize;
  HIP_TRY(hipStreamWaitEvent(c->copy_stream, c->ev_slot_free[slot], 0));
  HIP_TRY(hipMemcpyAsync(c->d_panels[slot], c->h_stage, pan_bytes, hipMemcpyHostToDevice,
                         c->copy_stream));
  HIP_TRY(hipMemcpyAsync(c->d_dinv[slot], (char *)c->h_stage + pan_bytes, dinv_bytes,
                         hipMemcpyHostToDevice, c->copy_stream));
  HIP_TRY(hipMemcpyAsync(c->d_Rslot[slot], c->d_Rjob[c->ready_rbuf], (size_t)(c->P.n / 3) * 72,
                         hipMemcpyDeviceToDevice, c->copy_stream));
  HIP_TRY(hipEventRecord(c->ev_upload_done, c->copy_stream));
  c->upload_issued = true;
  HIP_TRY(hipStreamWaitEvent(st, c->ev_upload_done, 0));
  if (c->active_slot >= 0) HIP_TRY(hipEventRecord(c->ev_slot_free[c->active_slot], st));
  c->active_slot = slot;
  c->installed_tag = c->ready_tag;
  return FE_OK;
}

// Rotations of a factor job's state (the current step's when they were
// computed, else the identity) into the next job buffer, on the job's copy
// stream; *rbuf receives the buffer index.
hipError_t snap_rotations(fe_ctx *c, hipStream_t js, int *rbuf) {
  const int rb = c->job_count++ & 1;
  *rbuf = rb;
  const int64_t nn = c->P.n / 3;
  if (c->rot_valid)
    return hipMemcpyAsync(c->d_Rjob[rb], c->d_Rnow, (size_t)nn * 72, hipMemcpyDeviceToDevice, js);
  launch_rot_identity(js, nn, c->d_Rjob[rb]);
  return hipGetLastError();
}

// GPU job: snapshot A on the factor stream (after the work queued on st;
// later work on st, which may assemble into the same A, waits for the copy),
// then factor into the idle slot once the solves that used it are done.
int gf_start_locked(fe_ctx *c, const void *A, int64_t tag, hipStream_t st) {
  const int slot = c->active_slot < 0 ? 0 : 1 - c->active_slot;
  if (c->ready_slot == slot) c->ready_tag = c->installed_tag;  // superseded
  c->ready_slot = -1;
  HIP_TRY(hipEventRecord(c->ev_snap_ready, st));
  HIP_TRY(hipStreamWaitEvent(c->factor_stream, c->ev_snap_ready, 0));
  HIP_TRY(hipMemcpyAsync(c->d_Asnap, A, c->P.col_idx.size() * c->tsize, hipMemcpyDeviceToDevice,
                         c->factor_stream));
  HIP_TRY(snap_rotations(c, c->factor_stream, &c->gf_rbuf));
  HIP_TRY(hipEventRecord(c->ev_snap_done, c->factor_stream));
  HIP_TRY(hipStreamWaitEvent(st, c->ev_snap_done, 0));
  HIP_TRY(hipStreamWaitEvent(c->factor_stream, c->ev_slot_free[slot], 0));
  HIP_TRY(hipMemsetAsync(c->gd.status, 0, sizeof(int), c->factor_stream));
  if (c->prec == FE_PREC_MIXED)
    launch_gpu_factor<float, float>(c->factor_stream, c->G, c->gd, (const float *)c->d_Asnap,
                                    (float *)c->d_panels[slot], (float *)c->d_dinv[slot]);
  else
    launch_gpu_factor<double, double>(c->factor_stream, c->G, c->gd, (const double *)c->d_Asnap,
                                      (double *)c->d_panels[slot], (double *)c->d_dinv[slot]);
  HIP_TRY(hipGetLastError());
  HIP_TRY(hipEventRecord(c->ev_gf_done, c->factor_stream));
  c->gf_pending = true;
  c->gf_tag = tag;
  c->gf_slot = slot;
  return FE_OK;
}

int factor_async_impl(fe_ctx *c, const void *A, int64_t tag, hipStream_t st) {
  std::unique_lock<std::mutex> lk(c->mu);
  if (factor_busy_locked(c)) return c->fail(FE_EBUSY, "factorisation in progress");
  if (c->gpu_factor) return gf_start_locked(c, A, tag, st);
  HIP_TRY(hipEventRecord(c->ev_snap_ready, st));
  HIP_TRY(hipStreamWaitEvent(c->copy_stream, c->ev_snap_ready, 0));
  HIP_TRY(hipMemcpyAsync(c->h_Asnap, A, c->P.col_idx.size() * c->tsize, hipMemcpyDeviceToHost,
                         c->copy_stream));
  HIP_TRY(snap_rotations(c, c->copy_stream, &c->job_rbuf));
  HIP_TRY(hipEventRecord(c->ev_snap_done, c->copy_stream));
  // later work on st may overwrite A (the next assembly): it waits for the copy
  HIP_TRY(hipStreamWaitEvent(st, c->ev_snap_done, 0));
  c->job_tag = tag;
  c->job_pending = true;
  c->cv.notify_all();
  return FE_OK;
}

int factor_wait_impl(fe_ctx *c, int64_t tag) {
  std::unique_lock<std::mutex> lk(c->mu);
  if (c->gpu_factor) {
    int rc = gf_collect_locked(c, true);
    if (rc) return rc;
  } else {
    c->cv.wait(lk, [&] { return !c->job_pending && !c->job_running; });
  }
  if (c->job_status != FE_OK) return c->fail(c->job_status, "%s", c->job_err.c_str());
  if (c->ready_tag < tag) return c->fail(FE_ESTATE, "no factorisation job with tag %lld",
                                         (long long)tag);
  return FE_OK;
}

template <typename T>
int step_impl(fe_ctx *c, double *q, double *v, const fe_params *p, const fe_step_opts *o,
              double *a_out, hipStream_t st, fe_step_stats *stats) {
  const int64_t n = c->P.n;
  const int64_t step = c->step_count;
  T *A = (T *)c->d_A;
  int rc = assemble<T>(c, p, q, v, A, c->d_b, st);
  if (rc) return rc;
  c->rot_valid = o->rotate_precond != 0;
  if (c->rot_valid)
    launch_node_rotations(st, c->elem_type, c->P.n_elems, c->d_conn, c->d_X, q, n / 3,
                          c->d_dof_fixed, c->d_ne_ptr, c->d_ne_idx, c->d_rotFe, c->d_Rnow);
  const int R = o->refresh, d = o->lag;
  if (R > 0 && step % R == 0) {
    bool busy;
    {
      std::lock_guard<std::mutex> lk(c->mu);
      busy = factor_busy_locked(c);
    }
    if (busy && o->mode == FE_FACTOR_DETERMINISTIC) {
      rc = factor_wait_impl(c, -1);
      if (rc) return rc;
      busy = false;
    }
    if (!busy) {
      rc = factor_async_impl(c, A, step, st);
      if (rc) return rc;
    }
  }
  if (R > 0) {
    std::unique_lock<std::mutex> lk(c->mu);
    if (o->mode == FE_FACTOR_DETERMINISTIC) {
      if (step - d >= 0) {
        const int64_t req = ((step - d) / R) * R;
        if (c->installed_tag != req) {
          lk.unlock();
          rc = factor_wait_impl(c, req);
          if (rc) return rc;
          lk.lock();
          rc = install_locked(c, st);
          if (rc) return rc;
        }
      }
    } else {
      rc = install_locked(c, st);
      if (rc) return rc;
    }
  }
  double *x = c->d_a;
  const int ws = o->warm_start;
  const int m = std::min(std::min(ws, kHist), c->hist_count);
  if (ws >= 2 && m >= 1)
    launch_hist_guess<T>(st, n, m, (c->hist_next + kHist - 1) % kHist, c->d_row_ptr, c->d_col, A,
                         c->d_histV, c->d_histW, c->d_b, c->d_histP,
                         c->d_histP + hist_part_doubles() - kHist, x);
  else if (!(ws == 1 && c->have_prev_a))
    launch_zero(st, n, x);
  fe_solve_stats ss;
  c->rot_on = c->rot_valid && c->active_slot >= 0;
  if (c->rot_on)
    launch_rot_q<T>(st, n / 3, c->d_Rnow, c->d_Rslot[c->active_slot], (T *)c->d_rotQ);
  rc = pcg<T>(c, A, c->d_b, x, o->rel_tol, o->max_it, st, &ss);
  c->rot_on = false;
  c->have_prev_a = true;
  if (ws >= 2 && (rc == FE_OK || rc == FE_ENOTCONV)) {
    launch_hist_push(st, n, c->hist_next, x, c->d_histV);
    c->hist_next = (c->hist_next + 1) % kHist;
    c->hist_count = std::min(c->hist_count + 1, kHist);
  }
  if (c->h_state->elem_status) {
    clear_elem_status(c, st);
    return c->fail(FE_EINVERTED, "inverted element (det F <= 0) at step %lld", (long long)step);
  }
  if (rc && rc != FE_ENOTCONV) return rc;
  launch_integrate(st, n, p->h, x, q, v);
  if (a_out) {
    hipError_t e = hipMemcpyAsync(a_out, x, n * 8, hipMemcpyDeviceToDevice, st);
    if (e != hipSuccess) return c->fail(FE_EDEVICE, "a_out copy: %s", hipGetErrorString(e));
  }
  if (stats) {
    stats->solve = ss;
    stats->step = step;
    stats->factor_lag = ss.factor_tag >= 0 ? step - ss.factor_tag : -1;
  }
  c->step_count = step + 1;
  return rc;
}

template <typename T>
int adjoint_impl(fe_ctx *c, const double *q_n, const double *v_n, const double *v_np1,
                 const double *lq_in, const double *lv_in, double *lq_out, double *lv_out,
                 double *dE, const fe_params *p, const fe_step_opts *o, hipStream_t st,
                 fe_solve_stats *stats) {
  const int64_t n = c->P.n;
  if (p && p->material != FE_NEO_HOOKEAN && p->material != FE_STVK)
    return c->fail(FE_EINVAL, "the adjoint step covers the neo-Hookean and St Venant-Kirchhoff "
                              "materials");
  T *A = (T *)c->d_A;
  // A at q_n (b is not needed but assembled alongside)
  int rc = assemble<T>(c, p, q_n, v_n, A, c->d_b, st);
  if (rc) return rc;
  c->rot_valid = o && o->rotate_precond;
  if (c->rot_valid)
    launch_node_rotations(st, c->elem_type, c->P.n_elems, c->d_conn, c->d_X, q_n, n / 3,
                          c->d_dof_fixed, c->d_ne_ptr, c->d_ne_idx, c->d_rotFe, c->d_Rnow);
  if (o && o->refresh > 0 && c->active_slot < 0) {
    // no factor yet: factor this A synchronously
    const int64_t tag = (int64_t(1) << 40) + c->step_count;
    rc = factor_wait_impl(c, -1);  // let a running job finish first
    if (rc) return rc;
    rc = factor_async_impl(c, A, tag, st);
    if (rc) return rc;
    rc = factor_wait_impl(c, tag);
    if (rc) return rc;
    std::lock_guard<std::mutex> lk(c->mu);
    rc = install_locked(c, st);
    if (rc) return rc;
  }
  launch_abar(st, n, p->h, lq_in, lv_in, c->d_dof_fixed, c->d_abar);
  launch_zero(st, n, c->d_mu);
  fe_solve_stats ss;
  c->rot_on = c->rot_valid && c->active_slot >= 0;
  if (c->rot_on)
    launch_rot_q<T>(st, n / 3, c->d_Rnow, c->d_Rslot[c->active_slot], (T *)c->d_rotQ);
  rc = pcg<T>(c, A, c->d_abar, c->d_mu, o ? o->rel_tol : 1e-10, o ? o->max_it : 1000, st, &ss);
  c->rot_on = false;
  if (c->h_state->elem_status) {
    clear_elem_status(c, st);
    return c->fail(FE_EINVERTED, "inverted element in the adjoint step");
  }
  if (rc && rc != FE_ENOTCONV) return rc;
  launch_zero(st, n, c->d_Kmu);
  launch_zero(st, n, c->d_Mmu);
  launch_zero(st, n, c->d_Tmv);
  const ElemParams ep = to_elem(p);
  launch_adjoint_element<T>(st, c->elem_type, c->P.n_elems, c->d_conn, c->d_X, q_n, c->d_mu,
                            v_np1, p->E, ep, c->d_Kmu, c->d_Mmu, c->d_Tmv, dE);
  launch_adjoint_combine(st, n, p->h, p->alpha, p->beta, lq_in, lv_in, c->d_Kmu, c->d_Mmu,
                         c->d_Tmv, lq_out, lv_out);
  if (stats) *stats = ss;
  return rc;
}

}  // namespace

fe_ctx::~fe_ctx() {
  if (th.joinable()) {
    {
      std::lock_guard<std::mutex> lk(mu);
      quit = true;
    }
    cv.notify_all();
    th.join();
  }
  if (bound) {
    (void)hipSetDevice(device);
    drain_timing(this);
    for (hipEvent_t e : ev_pool) (void)hipEventDestroy(e);
    if (copy_stream) (void)hipStreamSynchronize(copy_stream);
    if (h_state) (void)hipHostFree(h_state);
    if (h_flag) (void)hipHostFree(h_flag);
    if (h_Asnap) (void)hipHostFree(h_Asnap);
    if (h_stage) (void)hipHostFree(h_stage);
    for (hipEvent_t e : {ev_snap_ready, ev_snap_done, ev_upload_done, ev_slot_free[0],
                         ev_slot_free[1]})
      if (e) (void)hipEventDestroy(e);
    if (copy_stream) (void)hipStreamDestroy(copy_stream);
    for (auto &kv : graphs) (void)hipGraphExecDestroy(kv.second);
    if (cap_stream) (void)hipStreamDestroy(cap_stream);
    if (factor_stream) {
      (void)hipStreamSynchronize(factor_stream);
      (void)hipStreamDestroy(factor_stream);
    }
    if (ev_gf_done) (void)hipEventDestroy(ev_gf_done);
    if (h_gf_status) (void)hipHostFree(h_gf_status);
  }
}

// =================================================================== C ABI
extern "C" {

int fe_build_pattern(const fe_mesh *mesh, const uint8_t *fixed_dof, const fe_build_opts *opts,
                     fe_ctx **out) {
  g_build_error.clear();
  if (!mesh || !out || !mesh->conn || !mesh->X) {
    g_build_error = "NULL argument";
    return FE_EINVAL;
  }
  if (mesh->elem_type != FE_TET4 && mesh->elem_type != FE_HEX8) {
    g_build_error = "elem_type must be FE_TET4 or FE_HEX8";
    return FE_EINVAL;
  }
  fe_ctx *c = nullptr;
  try {
    c = new fe_ctx();
    c->elem_type = mesh->elem_type;
    c->nen = mesh->elem_type;
    if (opts && opts->n_threads > 0) {
      c->n_threads = opts->n_threads;
    } else {
      // default: the process's CPU share (OMP_NUM_THREADS if set, else all
      // cores, capped at 16) minus one core left to the launching thread
      int hw = (int)std::max(1u, std::thread::hardware_concurrency());
      if (const char *env = getenv("OMP_NUM_THREADS")) {
        const int v = atoi(env);
        if (v > 0) hw = std::min(hw, v);
      }
      hw = std::min(hw, 16);
      c->n_threads = std::max(1, hw - 1);
    }
    std::string e = build_pattern(mesh->n_nodes, mesh->n_elems, c->nen, mesh->conn, fixed_dof, c->P);
    if (e.empty()) {
      // rest volume check (signed, per element)
      const double *X = mesh->X;
      for (int64_t el = 0; el < mesh->n_elems && e.empty(); ++el) {
        const int32_t *cn = mesh->conn + el * c->nen;
        int a0 = 0, a1 = 1, a2 = c->nen == 8 ? 3 : 2, a3 = c->nen == 8 ? 4 : 3;
        double d[3][3];
        for (int i = 0; i < 3; ++i) {
          d[0][i] = X[3 * cn[a1] + i] - X[3 * cn[a0] + i];
          d[1][i] = X[3 * cn[a2] + i] - X[3 * cn[a0] + i];
          d[2][i] = X[3 * cn[a3] + i] - X[3 * cn[a0] + i];
        }
        const double det = d[0][0] * (d[1][1] * d[2][2] - d[1][2] * d[2][1]) -
                           d[0][1] * (d[1][0] * d[2][2] - d[1][2] * d[2][0]) +
                           d[0][2] * (d[1][0] * d[2][1] - d[1][1] * d[2][0]);
        if (!(det > 0)) e = "element " + std::to_string(el) + " has non-positive rest volume";
      }
    }
    if (e.empty()) {
      c->X.assign(mesh->X, mesh->X + 3 * (int64_t)mesh->n_nodes);
      e = analyse(c->P, c->X.data(), opts ? opts->leaf_nodes : 0, opts ? opts->fwd_tile_cols : 0,
                  opts ? opts->fwd_col_groups : 0, opts ? opts->bwd_tile_rows : 0,
                  opts ? opts->bwd_tile_cols : 0, c->S);
    }
    if (e.empty() && opts && opts->factor_on_gpu) {
      c->gpu_factor = true;
      c->gf_max_blocks = std::max(0, opts->factor_max_blocks);
      e = gpu_plan(c->P, c->S, c->G);
    }
    if (!e.empty()) {
      g_build_error = e;
      delete c;
      return FE_EINVAL;
    }
    const double avg = (double)c->P.col_idx.size() / (double)std::max<int64_t>(1, c->P.n);
    c->spmv_lanes = spmv_lanes_for(avg);
  } catch (const std::bad_alloc &) {
    g_build_error = "out of host memory";
    delete c;
    return FE_ENOMEM;
  } catch (const std::exception &ex) {
    g_build_error = ex.what();
    delete c;
    return FE_EINVAL;
  }
  *out = c;
  return FE_OK;
}

int fe_query(fe_ctx *c, int32_t prec, fe_sizes *o) {
  if (!c || !o) return FE_EINVAL;
  if (prec != FE_PREC_FP64 && prec != FE_PREC_MIXED) return c->fail(FE_EINVAL, "bad precision");
  Layout L;
  try {
    L = make_layout(c, prec);
  } catch (const std::exception &ex) {
    return c->fail(FE_EINVAL, "%s", ex.what());
  }
  o->n_dofs = c->P.n;
  o->nnz = (int64_t)c->P.col_idx.size();
  o->n_elems = c->P.n_elems;
  o->map_len = (int64_t)c->P.tmap.size();
  o->n_supernodes = (int64_t)c->S.sn.size();
  o->n_levels = c->S.n_levels;
  o->factor_entries = c->S.dev_panel_entries;
  o->factor_lower = c->S.lower_entries;
  o->factor_flops = c->S.flops;
  o->ws_bytes = L.total;
  o->compact_map = c->P.compact_ok ? 1 : 0;
  o->pad_ = 0;
  return FE_OK;
}

int fe_bind(fe_ctx *c, int32_t prec, void *d_ws, int64_t ws_bytes, void *stream) {
  if (!c) return FE_EINVAL;
  if (c->bound) return c->fail(FE_ESTATE, "context already bound");
  if (prec != FE_PREC_FP64 && prec != FE_PREC_MIXED) return c->fail(FE_EINVAL, "bad precision");
  Layout L;
  try {
    L = make_layout(c, prec);
  } catch (const std::exception &ex) {
    return c->fail(FE_EINVAL, "%s", ex.what());
  }
  if (!d_ws || ws_bytes < L.total)
    return c->fail(FE_ENOMEM, "workspace too small: %lld < %lld bytes", (long long)ws_bytes,
                   (long long)L.total);
  if (((uintptr_t)d_ws) % 256 != 0) return c->fail(FE_EINVAL, "workspace must be 256-byte aligned");
  hipStream_t st = (hipStream_t)stream;
  HIP_TRY(hipGetDevice(&c->device));
  {
    void *sp = nullptr;
    const hipError_t e = scratch_address(c->device, &sp);
    if (e == hipSuccess) {
      c->d_scratch = (char *)sp;
    } else {
      c->scratch_err = std::string("hipGetSymbolAddress(scratch) failed: ") + hipGetErrorString(e);
      (void)hipGetLastError();
    }
  }
  c->prec = prec;
  c->tsize = prec == FE_PREC_MIXED ? 4 : 8;
  c->ws = (char *)d_ws;
  c->ws_bytes = ws_bytes;
  char *w = c->ws;
  c->d_row_ptr = ptr_at<int32_t>(w, L, L_ROWPTR);
  c->d_col = ptr_at<int32_t>(w, L, L_COL);
  c->d_conn = ptr_at<int32_t>(w, L, L_CONN);
  c->d_slot = ptr_at<uint8_t>(w, L, L_SLOT);
  c->d_smap = ptr_at<int32_t>(w, L, L_SMAP);
  c->d_blk_ptr = ptr_at<int32_t>(w, L, L_BLKPTR);
  c->d_blk_pos = ptr_at<int32_t>(w, L, L_BLKPOS);
  c->d_blk_node = ptr_at<int32_t>(w, L, L_BLKNODE);
  c->d_blk_src = ptr_at<int32_t>(w, L, L_BLKSRC);
  c->d_ebuf = w + L.off[L_EBUF];
  c->d_rbuf = ptr_at<double>(w, L, L_RBUF);
  c->d_fds = ptr_at<int32_t>(w, L, L_FDS);
  c->d_dof_fixed = ptr_at<uint8_t>(w, L, L_DOFFIX);
  c->d_X = ptr_at<double>(w, L, L_X);
  c->d_sn = ptr_at<SnDev>(w, L, L_SN);
  c->d_rows = ptr_at<int32_t>(w, L, L_ROWS);
  c->d_ftiles = ptr_at<TileDev>(w, L, L_FT);
  c->d_btiles = ptr_at<TileDev>(w, L, L_BT);
  c->panel_stream = c->S.dev_panel_entries * c->tsize > ((int64_t)256 << 20);
  c->d_panels[0] = w + L.off[L_PAN0];
  c->d_panels[1] = w + L.off[L_PAN1];
  c->d_dinv[0] = w + L.off[L_DINV0];
  c->d_dinv[1] = w + L.off[L_DINV1];
  c->d_jdinv = ptr_at<double>(w, L, L_JDINV);
  c->d_r = ptr_at<double>(w, L, L_R);
  c->d_z = ptr_at<double>(w, L, L_Z);
  c->d_p = ptr_at<double>(w, L, L_P);
  c->d_q = ptr_at<double>(w, L, L_Q);
  c->d_tmp = ptr_at<double>(w, L, L_TMP);
  c->d_b = ptr_at<double>(w, L, L_B);
  c->d_a = ptr_at<double>(w, L, L_ACC);
  c->d_abar = ptr_at<double>(w, L, L_ABAR);
  c->d_mu = ptr_at<double>(w, L, L_MU);
  c->d_Kmu = ptr_at<double>(w, L, L_KMU);
  c->d_Mmu = ptr_at<double>(w, L, L_MMU);
  c->d_Tmv = ptr_at<double>(w, L, L_TMV);
  c->d_w = w + L.off[L_W];
  c->d_y = w + L.off[L_Y];
  c->d_A = w + L.off[L_A];
  c->d_part1 = ptr_at<double>(w, L, L_PART1);
  c->d_part2 = ptr_at<double>(w, L, L_PART2);
  c->d_state = ptr_at<PcgState>(w, L, L_STATE);
  c->d_mftiles = ptr_at<MTile>(w, L, L_MFT);
  c->d_mbtiles = ptr_at<MTile>(w, L, L_MBT);
  c->d_herr = ptr_at<int>(w, L, L_HERR);
  c->d_mbdofs = ptr_at<int32_t>(w, L, L_MBDOF);
  c->d_histV = ptr_at<double>(w, L, L_HISTV);
  c->d_histW = ptr_at<double>(w, L, L_HISTW);
  c->d_histP = ptr_at<double>(w, L, L_HISTP);
  c->d_ne_ptr = ptr_at<int32_t>(w, L, L_NEPTR);
  c->d_ne_idx = ptr_at<int32_t>(w, L, L_NEIDX);
  c->d_rotFe = ptr_at<double>(w, L, L_ROTFE);
  c->d_Rnow = ptr_at<double>(w, L, L_RNOW);
  c->d_Rjob[0] = ptr_at<double>(w, L, L_RJOB0);
  c->d_Rjob[1] = ptr_at<double>(w, L, L_RJOB1);
  c->d_Rslot[0] = ptr_at<double>(w, L, L_RSLOT0);
  c->d_Rslot[1] = ptr_at<double>(w, L, L_RSLOT1);
  c->d_rotQ = w + L.off[L_ROTQ];

  // host-side resources
  HIP_TRY(hipHostMalloc((void **)&c->h_state, sizeof(PcgState), hipHostMallocDefault));
  memset(c->h_state, 0, sizeof(PcgState));
  HIP_TRY(hipHostMalloc((void **)&c->h_flag, 256, hipHostMallocDefault));
  if (!c->gpu_factor) {
    // snapshot of A and staging of the factor: host-thread factorisation only
    HIP_TRY(hipHostMalloc(&c->h_Asnap, std::max<size_t>(1, c->P.col_idx.size() * c->tsize),
                          hipHostMallocDefault));
    HIP_TRY(hipHostMalloc(&c->h_stage,
                          std::max<size_t>(1, (c->S.dev_panel_entries + c->P.n) * c->tsize),
                          hipHostMallocDefault));
  }
  HIP_TRY(hipStreamCreateWithFlags(&c->copy_stream, hipStreamNonBlocking));
  HIP_TRY(hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking));
  HIP_TRY(hipEventCreateWithFlags(&c->ev_snap_ready, hipEventDisableTiming));
  HIP_TRY(hipEventCreateWithFlags(&c->ev_snap_done, hipEventDisableTiming));
  HIP_TRY(hipEventCreateWithFlags(&c->ev_upload_done, hipEventDisableTiming));
  HIP_TRY(hipEventCreateWithFlags(&c->ev_slot_free[0], hipEventDisableTiming));
  HIP_TRY(hipEventCreateWithFlags(&c->ev_slot_free[1], hipEventDisableTiming));
  c->bound = true;

  // upload topology (synchronous copies from pageable host memory)
  const Pattern &P = c->P;
  const Symbolic &S = c->S;
  auto up = [&](void *dst, const void *src, size_t bytes) -> hipError_t {
    if (bytes == 0) return hipSuccess;
    return hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, st);
  };
  HIP_TRY(up(c->d_row_ptr, P.row_ptr.data(), P.row_ptr.size() * 4));
  HIP_TRY(up(c->d_col, P.col_idx.data(), P.col_idx.size() * 4));
  HIP_TRY(up(c->d_conn, P.conn.data(), P.conn.size() * 4));
  if (P.compact_ok) {
    HIP_TRY(up(c->d_slot, P.slot.data(), P.slot.size()));
    HIP_TRY(up(c->d_blk_ptr, P.blk_ptr.data(), P.blk_ptr.size() * 4));
    HIP_TRY(up(c->d_blk_pos, P.blk_pos.data(), P.blk_pos.size() * 4));
    HIP_TRY(up(c->d_blk_node, P.blk_node.data(), P.blk_node.size() * 4));
    HIP_TRY(up(c->d_blk_src, P.blk_src.data(), P.blk_src.size() * 4));
  } else {
    HIP_TRY(up(c->d_smap, P.tmap.data(), P.tmap.size() * 4));
  }
  HIP_TRY(up(c->d_fds, P.fixed_diag_slot.data(), P.fixed_diag_slot.size() * 4));
  HIP_TRY(up(c->d_dof_fixed, P.fixed.data(), P.fixed.size()));
  HIP_TRY(up(c->d_X, c->X.data(), c->X.size() * 8));
  std::vector<SnDev> sn(S.sn.size());
  for (size_t s = 0; s < S.sn.size(); ++s)
    sn[s] = SnDev{S.sn[s].nc, S.sn[s].m, S.sn[s].dev_off, S.sn[s].rows_off, S.sn[s].ld, 0};
  HIP_TRY(up(c->d_sn, sn.data(), sn.size() * sizeof(SnDev)));
  HIP_TRY(up(c->d_rows, S.rows.data(), S.rows.size() * 4));
  auto tile_dev = [&](int32_t s, int32_t r0, int32_t c0) {
    const Supernode &q = S.sn[s];
    return TileDev{q.dev_off, q.rows_off, q.nc, q.m, q.ld, r0, c0, 0};
  };
  std::vector<TileDev> ft(S.fwd_tiles.size()), bt(S.bwd_tiles.size());
  for (size_t i = 0; i < ft.size(); ++i)
    ft[i] = tile_dev(S.fwd_tiles[i].s, S.fwd_tiles[i].r0, S.fwd_tiles[i].c0);
  for (size_t i = 0; i < bt.size(); ++i)
    bt[i] = tile_dev(S.bwd_tiles[i].s, S.bwd_tiles[i].r0, S.bwd_tiles[i].c0);
  HIP_TRY(up(c->d_ftiles, ft.data(), ft.size() * sizeof(TileDev)));
  HIP_TRY(up(c->d_btiles, bt.data(), bt.size() * sizeof(TileDev)));
  HIP_TRY(up(c->d_mftiles, S.mfwd_tiles.data(), S.mfwd_tiles.size() * sizeof(MTile)));
  HIP_TRY(up(c->d_mbtiles, S.mbwd_tiles.data(), S.mbwd_tiles.size() * sizeof(MTile)));
  HIP_TRY(up(c->d_mbdofs, S.mbwd_dofs.data(), S.mbwd_dofs.size() * 4));
  HIP_TRY(up(c->d_state, c->h_state, sizeof(PcgState)));
  {
    // the elements of each node in ascending order (the rotation's sums run
    // in that fixed order); rotations of jobs and slots the identity
    const int64_t nn = P.n / 3;
    std::vector<int32_t> ne_ptr(nn + 1, 0), ne_idx((size_t)P.n_elems * P.nen);
    for (size_t k = 0; k < ne_idx.size(); ++k) ++ne_ptr[P.conn[k] + 1];
    for (int64_t i = 0; i < nn; ++i) ne_ptr[i + 1] += ne_ptr[i];
    std::vector<int32_t> fill(ne_ptr.begin(), ne_ptr.end() - 1);
    for (int64_t e = 0; e < P.n_elems; ++e)
      for (int a = 0; a < P.nen; ++a) ne_idx[fill[P.conn[e * P.nen + a]]++] = (int32_t)e;
    HIP_TRY(up(c->d_ne_ptr, ne_ptr.data(), ne_ptr.size() * 4));
    HIP_TRY(up(c->d_ne_idx, ne_idx.data(), ne_idx.size() * 4));
    for (double *R : {c->d_Rnow, c->d_Rjob[0], c->d_Rjob[1], c->d_Rslot[0], c->d_Rslot[1]})
      launch_rot_identity(st, nn, R);
    HIP_TRY(hipGetLastError());
  }
  HIP_TRY(hipStreamSynchronize(st));

  // algorithmic bytes per sweep level (lower panel entries + indices + vectors)
  c->fwd_level_bytes.assign(S.n_levels, 0.0);
  c->bwd_level_bytes.assign(S.n_levels, 0.0);
  for (const Supernode &s : S.sn) {
    const double lower = (double)s.m * s.nc - (double)s.nc * (s.nc - 1) / 2.0;
    const double bytes = lower * c->tsize + s.m * 4.0 + (s.nc + 2.0 * s.m) * c->tsize;
    c->fwd_level_bytes[s.level] += bytes;
    c->bwd_level_bytes[S.n_levels - 1 - s.level] += bytes;
  }
  if (c->gpu_factor) {
    GfDev &g = c->gd;
    const GfPlan &Gp = c->G;
    g.fronts = ptr_at<double>(w, L, L_GF_FRONTS);
    GfFront *fr = ptr_at<GfFront>(w, L, L_GF_FR);
    int32_t *lvl_sn = ptr_at<int32_t>(w, L, L_GF_LVLSN);
    int32_t *a_csr = ptr_at<int32_t>(w, L, L_GF_ACSR);
    int64_t *a_off = ptr_at<int64_t>(w, L, L_GF_AOFF);
    int32_t *parent = ptr_at<int32_t>(w, L, L_GF_PARENT);
    int32_t *rel = ptr_at<int32_t>(w, L, L_GF_REL);
    int64_t *rel_off = ptr_at<int64_t>(w, L, L_GF_RELOFF);
    GfExt *ext = ptr_at<GfExt>(w, L, L_GF_EXT);
    int32_t *panel_sn = ptr_at<int32_t>(w, L, L_GF_PANELSN);
    GfTile *upd = ptr_at<GfTile>(w, L, L_GF_UPD);
    HIP_TRY(up(fr, Gp.fr.data(), Gp.fr.size() * sizeof(GfFront)));
    HIP_TRY(up(lvl_sn, Gp.lvl_sn.data(), Gp.lvl_sn.size() * 4));
    HIP_TRY(up(a_csr, Gp.a_csr.data(), Gp.a_csr.size() * 4));
    HIP_TRY(up(a_off, Gp.a_off.data(), Gp.a_off.size() * 8));
    HIP_TRY(up(parent, Gp.parent.data(), Gp.parent.size() * 4));
    HIP_TRY(up(rel, Gp.rel.data(), Gp.rel.size() * 4));
    HIP_TRY(up(rel_off, Gp.rel_off.data(), Gp.rel_off.size() * 8));
    HIP_TRY(up(ext, Gp.ext.data(), Gp.ext.size() * sizeof(GfExt)));
    HIP_TRY(up(panel_sn, Gp.panel_sn.data(), Gp.panel_sn.size() * 4));
    HIP_TRY(up(upd, Gp.upd.data(), Gp.upd.size() * sizeof(GfTile)));
    HIP_TRY(hipStreamSynchronize(st));
    g.fr = fr;
    g.lvl_sn = lvl_sn;
    g.a_csr = a_csr;
    g.a_off = a_off;
    g.parent = parent;
    g.rel = rel;
    g.rel_off = rel_off;
    g.ext = ext;
    g.panel_sn = panel_sn;
    g.upd = upd;
    g.rows = c->d_rows;
    g.max_blocks = c->gf_max_blocks;
    g.status = ptr_at<int>(w, L, L_GF_STATUS);
    c->d_Asnap = w + L.off[L_GF_ASNAP];
    HIP_TRY(hipHostMalloc((void **)&c->h_gf_status, sizeof(int), hipHostMallocDefault));
    *c->h_gf_status = 0;
    HIP_TRY(hipStreamCreateWithFlags(&c->factor_stream, hipStreamNonBlocking));
    HIP_TRY(hipEventCreateWithFlags(&c->ev_gf_done, hipEventDisableTiming));
  }
  // backward levels are launched top-down: index L of the loop is level nl-1-L
  c->th = std::thread(factor_main, c);
  return FE_OK;
}

int fe_export_pattern(fe_ctx *c, int32_t *row_ptr, int32_t *col_idx, int32_t *map) {
  if (!c) return FE_EINVAL;
  if (row_ptr) memcpy(row_ptr, c->P.row_ptr.data(), c->P.row_ptr.size() * 4);
  if (col_idx) memcpy(col_idx, c->P.col_idx.data(), c->P.col_idx.size() * 4);
  if (map) memcpy(map, c->P.tmap.data(), c->P.tmap.size() * 4);
  return FE_OK;
}

int fe_export_ordering(fe_ctx *c, int32_t *perm, int32_t *sn_ptr) {
  if (!c) return FE_EINVAL;
  if (perm) memcpy(perm, c->S.perm.data(), c->S.perm.size() * 4);
  if (sn_ptr) memcpy(sn_ptr, c->S.sn_ptr.data(), c->S.sn_ptr.size() * 4);
  return FE_OK;
}

int fe_export_supernodes(fe_ctx *c, int32_t *n_rows, int32_t *level) {
  if (!c) return FE_EINVAL;
  for (size_t s = 0; s < c->S.sn.size(); ++s) {
    if (n_rows) n_rows[s] = c->S.sn[s].m;
    if (level) level[s] = c->S.sn[s].level;
  }
  return FE_OK;
}

int fe_export_sweep_tiles(fe_ctx *c, int32_t *n_levels, int32_t *n_fwd, int32_t *n_bwd,
                          int32_t *extents, int32_t *fwd, int32_t *bwd) {
  if (!c) return FE_EINVAL;
  const Symbolic &S = c->S;
  if (n_levels) *n_levels = S.n_levels;
  if (n_fwd) *n_fwd = (int32_t)S.fwd_tiles.size();
  if (n_bwd) *n_bwd = (int32_t)S.bwd_tiles.size();
  if (extents)
    for (int L = 0; L < S.n_levels; ++L) {
      extents[4 * L + 0] = S.fwd_level_cols[L];
      extents[4 * L + 1] = S.fwd_level_groups[L];
      extents[4 * L + 2] = S.bwd_level_rows[L];
      extents[4 * L + 3] = S.bwd_level_cols[L];
    }
  auto put = [](const std::vector<Tile> &tl, int32_t *out) {
    if (!out) return;
    for (size_t i = 0; i < tl.size(); ++i) {
      out[3 * i + 0] = tl[i].s;
      out[3 * i + 1] = tl[i].r0;
      out[3 * i + 2] = tl[i].c0;
    }
  };
  put(S.fwd_tiles, fwd);
  put(S.bwd_tiles, bwd);
  return FE_OK;
}

int fe_assemble(fe_ctx *c, const fe_params *params, const double *q, const double *v,
                void *A_vals, double *b, void *stream) {
  if (!c) return FE_EINVAL;
  if (!c->bound) return c->fail(FE_ESTATE, "fe_bind has not been called");
  if (int rc = check_params(c, params)) return rc;
  if (!q || !v || !A_vals || !b) return c->fail(FE_EINVAL, "NULL buffer");
  hipStream_t st = (hipStream_t)stream;
  if (int rc = clear_elem_status(c, st)) return rc;
  if (c->prec == FE_PREC_MIXED) assemble<float>(c, params, q, v, (float *)A_vals, b, st);
  else assemble<double>(c, params, q, v, (double *)A_vals, b, st);
  HIP_TRY(hipGetLastError());
  if (int rc = read_state(c, st)) return rc;
  if (c->h_state->elem_status) {
    clear_elem_status(c, st);
    return c->fail(FE_EINVERTED, "inverted element (det F <= 0)");
  }
  return FE_OK;
}

int fe_factor_async(fe_ctx *c, const void *A_vals, int64_t tag, void *stream) {
  if (!c) return FE_EINVAL;
  if (!c->bound) return c->fail(FE_ESTATE, "fe_bind has not been called");
  if (!A_vals) return c->fail(FE_EINVAL, "NULL A");
  return factor_async_impl(c, A_vals, tag, (hipStream_t)stream);
}

int fe_factor_status(fe_ctx *c, int64_t *ready_tag) {
  if (!c) return FE_EINVAL;
  std::lock_guard<std::mutex> lk(c->mu);
  const bool busy = factor_busy_locked(c);
  if (ready_tag) *ready_tag = c->ready_tag;
  if (busy) return FE_EBUSY;
  if (c->job_status != FE_OK) return c->fail(c->job_status, "%s", c->job_err.c_str());
  return FE_OK;
}

int fe_factor_wait(fe_ctx *c, int64_t tag) {
  if (!c) return FE_EINVAL;
  if (!c->bound) return c->fail(FE_ESTATE, "fe_bind has not been called");
  return factor_wait_impl(c, tag);
}

int fe_factor_install(fe_ctx *c, int64_t *tag, void *stream) {
  if (!c) return FE_EINVAL;
  if (!c->bound) return c->fail(FE_ESTATE, "fe_bind has not been called");
  std::lock_guard<std::mutex> lk(c->mu);
  int rc = install_locked(c, (hipStream_t)stream);
  if (tag) *tag = c->active_slot >= 0 ? c->installed_tag : -1;
  return rc;
}

int fe_pcg_solve(fe_ctx *c, const void *A_vals, const double *b, double *x, double rel_tol,
                 int32_t max_it, void *stream, fe_solve_stats *stats) {
  if (!c) return FE_EINVAL;
  if (!c->bound) return c->fail(FE_ESTATE, "fe_bind has not been called");
  if (!A_vals || !b || !x) return c->fail(FE_EINVAL, "NULL buffer");
  if (!(rel_tol > 0) || max_it <= 0) return c->fail(FE_EINVAL, "bad tolerance or max_it");
  hipStream_t st = (hipStream_t)stream;
  if (c->prec == FE_PREC_MIXED)
    return pcg<float>(c, (const float *)A_vals, b, x, rel_tol, max_it, st, stats);
  return pcg<double>(c, (const double *)A_vals, b, x, rel_tol, max_it, st, stats);
}

int fe_step(fe_ctx *c, double *q, double *v, const fe_params *params, const fe_step_opts *opts,
            double *a_out, void *stream, fe_step_stats *stats) {
  if (!c) return FE_EINVAL;
  if (!c->bound) return c->fail(FE_ESTATE, "fe_bind has not been called");
  if (int rc = check_params(c, params)) return rc;
  if (!q || !v || !opts) return c->fail(FE_EINVAL, "NULL argument");
  if (opts->mode == FE_FACTOR_DETERMINISTIC && opts->refresh > 0 && opts->lag >= opts->refresh)
    return c->fail(FE_EINVAL, "deterministic mode needs lag < refresh");
  if (!(opts->rel_tol > 0) || opts->max_it <= 0) return c->fail(FE_EINVAL, "bad rel_tol/max_it");
  hipStream_t st = (hipStream_t)stream;
  if (c->prec == FE_PREC_MIXED) return step_impl<float>(c, q, v, params, opts, a_out, st, stats);
  return step_impl<double>(c, q, v, params, opts, a_out, st, stats);
}

int fe_step_adjoint(fe_ctx *c, const double *q_n, const double *v_n, const double *v_np1,
                    const double *lam_q_in, const double *lam_v_in, double *lam_q_out,
                    double *lam_v_out, double *dE_accum, const fe_params *params,
                    const fe_step_opts *opts, void *stream, fe_solve_stats *stats) {
  if (!c) return FE_EINVAL;
  if (!c->bound) return c->fail(FE_ESTATE, "fe_bind has not been called");
  if (int rc = check_params(c, params)) return rc;
  if (!q_n || !v_n || !v_np1 || !lam_q_in || !lam_v_in || !lam_q_out || !lam_v_out || !dE_accum)
    return c->fail(FE_EINVAL, "NULL buffer");
  hipStream_t st = (hipStream_t)stream;
  if (c->prec == FE_PREC_MIXED)
    return adjoint_impl<float>(c, q_n, v_n, v_np1, lam_q_in, lam_v_in, lam_q_out, lam_v_out,
                               dE_accum, params, opts, st, stats);
  return adjoint_impl<double>(c, q_n, v_n, v_np1, lam_q_in, lam_v_in, lam_q_out, lam_v_out,
                              dE_accum, params, opts, st, stats);
}

int fe_spmv(fe_ctx *c, const void *A_vals, const double *x, double *y, void *stream) {
  if (!c) return FE_EINVAL;
  if (!c->bound) return c->fail(FE_ESTATE, "fe_bind has not been called");
  if (!A_vals || !x || !y) return c->fail(FE_EINVAL, "NULL buffer");
  hipStream_t st = (hipStream_t)stream;
  if (c->prec == FE_PREC_MIXED)
    spmv<float>(c, (const float *)A_vals, x, y, nullptr, nullptr, nullptr, st, nullptr);
  else
    spmv<double>(c, (const double *)A_vals, x, y, nullptr, nullptr, nullptr, st, nullptr);
  HIP_TRY(hipGetLastError());
  return FE_OK;
}

int fe_precond_apply(fe_ctx *c, const void *A_vals, const double *r, double *z, void *stream) {
  if (!c) return FE_EINVAL;
  if (!c->bound) return c->fail(FE_ESTATE, "fe_bind has not been called");
  if (!r || !z) return c->fail(FE_EINVAL, "NULL buffer");
  hipStream_t st = (hipStream_t)stream;
  if (c->active_slot < 0) {
    if (!A_vals) return c->fail(FE_EINVAL, "no factor installed and A is NULL");
    if (c->prec == FE_PREC_MIXED)
      launch_diag_inv<float>(st, c->P.n, c->d_row_ptr, c->d_col, (const float *)A_vals, c->d_jdinv);
    else
      launch_diag_inv<double>(st, c->P.n, c->d_row_ptr, c->d_col, (const double *)A_vals, c->d_jdinv);
  }
  if (c->prec == FE_PREC_MIXED) precond<float>(c, (const float *)A_vals, r, z, st, false);
  else precond<double>(c, (const double *)A_vals, r, z, st, false);
  HIP_TRY(hipGetLastError());
  return FE_OK;
}

int fe_multi_ws_bytes(fe_ctx *c, int32_t k, int64_t *bytes) {
  if (!c) return FE_EINVAL;
  if (!c->bound) return c->fail(FE_ESTATE, "fe_bind has not been called");
  if (k < 0 || !bytes) return c->fail(FE_EINVAL, "bad argument");
  *bytes = multi_ws(c, k).total;
  return FE_OK;
}

// shared checks of the many-right-hand-side calls
static int multi_check(fe_ctx *c, int32_t k, void *work, int64_t work_bytes) {
  if (!c->bound) return c->fail(FE_ESTATE, "fe_bind has not been called");
  if (c->active_slot < 0) return c->fail(FE_ESTATE, "no factor installed");
  if (k < 0) return c->fail(FE_EINVAL, "negative number of right-hand sides");
  if (k == 0) return FE_OK;
  if (!work || ((uintptr_t)work & 255)) return c->fail(FE_EINVAL, "work must be 256-byte aligned");
  const int64_t need = multi_ws(c, k).total;
  if (work_bytes < need)
    return c->fail(FE_ENOMEM, "workspace too small: %lld bytes needed", (long long)need);
  return FE_OK;
}

// Read back and clear the constraint-matrix error word (synchronises st).
static int herr_check(fe_ctx *c, hipStream_t st) {
  HIP_TRY(hipMemcpyAsync(c->h_flag, c->d_herr, sizeof(int), hipMemcpyDeviceToHost, st));
  HIP_TRY(hipStreamSynchronize(st));
  if (*c->h_flag) return c->fail(FE_EINVAL, "constraint matrix: bad row range or column index");
  return FE_OK;
}

int fe_precond_apply_multi(fe_ctx *c, const double *R, double *Z, int32_t k, void *work,
                           int64_t work_bytes, void *stream) {
  if (!c) return FE_EINVAL;
  const int rc = multi_check(c, k, work, work_bytes);
  if (rc != FE_OK || k == 0) return rc;
  if (!R || !Z) return c->fail(FE_EINVAL, "NULL buffer");
  hipStream_t st = (hipStream_t)stream;
  const MultiWs m = multi_ws(c, k);
  if (c->prec == FE_PREC_MIXED) precond_multi<float>(c, m, R, Z, k, (char *)work, st);
  else precond_multi<double>(c, m, R, Z, k, (char *)work, st);
  HIP_TRY(hipGetLastError());
  return FE_OK;
}

// W = H P^{-1} H^T with the blocks of right-hand sides in `work` (checked
// by the caller); shared by fe_compliance and fe_compliance_noalloc.
static int compliance_impl(fe_ctx *c, int32_t k, const int32_t *h_row_ptr, const int32_t *h_col,
                           const double *h_val, int64_t nnz_h, double *W, double *Z, char *work,
                           void *stream) {
  if (!h_row_ptr || !W || nnz_h < 0 || (nnz_h > 0 && (!h_col || !h_val)))
    return c->fail(FE_EINVAL, "bad constraint matrix or NULL output");
  hipStream_t st = (hipStream_t)stream;
  const MultiWs m = multi_ws(c, k);
  HIP_TRY(hipMemsetAsync(c->d_herr, 0, sizeof(int), st));
  if (c->prec == FE_PREC_MIXED)
    compliance<float>(c, m, k, h_row_ptr, h_col, h_val, nnz_h, W, Z, work, st);
  else
    compliance<double>(c, m, k, h_row_ptr, h_col, h_val, nnz_h, W, Z, work, st);
  HIP_TRY(hipGetLastError());
  return herr_check(c, st);
}

int fe_compliance(fe_ctx *c, int32_t k, const int32_t *h_row_ptr, const int32_t *h_col,
                  const double *h_val, int64_t nnz_h, double *W, double *Z, void *work,
                  int64_t work_bytes, void *stream) {
  if (!c) return FE_EINVAL;
  const int rc = multi_check(c, k, work, work_bytes);
  if (rc != FE_OK || k == 0) return rc;
  return compliance_impl(c, k, h_row_ptr, h_col, h_val, nnz_h, W, Z, (char *)work, stream);
}

int fe_compliance_noalloc(fe_ctx *c, int32_t k, const int32_t *h_row_ptr, const int32_t *h_col,
                          const double *h_val, int64_t nnz_h, double *W, double *Z,
                          void *stream) {
  if (!c) return FE_EINVAL;
  if (!c->bound) return c->fail(FE_ESTATE, "fe_bind has not been called");
  if (!c->d_scratch) return c->fail(FE_EDEVICE, "%s", c->scratch_err.c_str());
  if (k > 0) {
    const int64_t need = multi_ws(c, k).total;
    if (need > kScratchBytes)
      return c->fail(FE_ENOMEM,
                     "%d right-hand sides need %lld bytes of scratch; the static scratch holds "
                     "%lld bytes (use fe_compliance with a caller workspace)",
                     (int)k, (long long)need, (long long)kScratchBytes);
  }
  const int rc = multi_check(c, k, c->d_scratch, kScratchBytes);
  if (rc != FE_OK || k == 0) return rc;
  return compliance_impl(c, k, h_row_ptr, h_col, h_val, nnz_h, W, Z, c->d_scratch, stream);
}

int fe_constraint_apply(fe_ctx *c, int32_t k, const int32_t *h_row_ptr, const int32_t *h_col,
                        const double *h_val, int64_t nnz_h, int32_t transpose, double s_h,
                        const double *x, double s_y, const double *y_in, double *y,
                        void *stream) {
  if (!c) return FE_EINVAL;
  if (!c->bound) return c->fail(FE_ESTATE, "fe_bind has not been called");
  if (k < 0 || nnz_h < 0) return c->fail(FE_EINVAL, "bad size");
  if (!h_row_ptr || !x || !y || (nnz_h > 0 && (!h_col || !h_val)))
    return c->fail(FE_EINVAL, "NULL buffer");
  hipStream_t st = (hipStream_t)stream;
  HIP_TRY(hipMemsetAsync(c->d_herr, 0, sizeof(int), st));
  launch_h_apply(st, k, c->P.n, nnz_h, h_row_ptr, h_col, h_val, transpose != 0, s_h, x, s_y,
                 y_in, y, c->d_herr);
  HIP_TRY(hipGetLastError());
  return herr_check(c, st);
}

int fe_structure_changed(fe_ctx *c, int64_t n_elems, const int32_t *conn,
                         const uint8_t *fixed_dof, int32_t *changed, void *stream) {
  if (!c) return FE_EINVAL;
  if (!c->bound) return c->fail(FE_ESTATE, "fe_bind has not been called");
  if (!changed || n_elems < 0 || (n_elems > 0 && !conn)) return c->fail(FE_EINVAL, "bad argument");
  if (n_elems != c->P.n_elems) {  // another element count: another fill sequence
    *changed = 1;
    return FE_OK;
  }
  hipStream_t st = (hipStream_t)stream;
  int *flag = c->d_herr + 1;  // second word of the error area
  HIP_TRY(hipMemsetAsync(flag, 0, sizeof(int), st));
  launch_struct_cmp(st, n_elems * c->nen, conn, c->d_conn, c->P.n, fixed_dof, c->d_dof_fixed,
                    flag);
  HIP_TRY(hipGetLastError());
  HIP_TRY(hipMemcpyAsync(c->h_flag, flag, sizeof(int), hipMemcpyDeviceToHost, st));
  HIP_TRY(hipStreamSynchronize(st));
  *changed = *c->h_flag ? 1 : 0;
  return FE_OK;
}

int fe_pgs(fe_ctx *c, int32_t k, const double *W, const double *cvec, double *lam,
           int32_t max_sweeps, double tol, double *info, void *stream) {
  if (!c) return FE_EINVAL;
  if (!c->bound) return c->fail(FE_ESTATE, "fe_bind has not been called");
  if (k < 0 || k > pgs_max_constraints() || max_sweeps < 0 || !(tol >= 0.0))
    return c->fail(FE_EINVAL, "k must be in [0, %d], max_sweeps >= 0, tol >= 0",
                   pgs_max_constraints());
  if (k == 0) return FE_OK;
  if (!W || !cvec || !lam) return c->fail(FE_EINVAL, "NULL buffer");
  launch_pgs((hipStream_t)stream, k, W, cvec, lam, max_sweeps, tol, info);
  HIP_TRY(hipGetLastError());
  return FE_OK;
}

int fe_host_factor_apply(fe_ctx *c, const double *A_host, const double *r_host, double *z_host,
                         int32_t n_rhs) {
  if (!c) return FE_EINVAL;
  if (!A_host || !r_host || !z_host || n_rhs < 0) return c->fail(FE_EINVAL, "bad argument");
  std::vector<double> panels, dinv;
  std::string e = factorize<double>(c->P, c->S, A_host, c->n_threads, panels, dinv);
  if (!e.empty()) return c->fail(FE_EFACTOR, "%s", e.c_str());
  const Symbolic &S = c->S;
  const int64_t n = c->P.n;
  std::vector<double> w(n), y(n), t;
  for (int32_t k = 0; k < n_rhs; ++k) {
    const double *r = r_host + k * n;
    double *z = z_host + k * n;
    for (int64_t i = 0; i < n; ++i) {
      w[i] = r[i];
      y[i] = 0.0;
      z[i] = c->P.fixed[i] ? r[i] : 0.0;
    }
    for (const Supernode &s : S.sn) {  // post-order = a valid forward order
      const int32_t *rw = S.rows.data() + s.rows_off;
      const double *G = panels.data() + s.panel_off;
      t.assign(s.m, 0.0);
      for (int32_t j = 0; j < s.nc; ++j) {
        const double wj = w[rw[j]];
        for (int32_t i = j; i < s.m; ++i) t[i] += G[(int64_t)j * s.m + i] * wj;
      }
      for (int32_t i = 0; i < s.nc; ++i) y[rw[i]] = t[i];
      for (int32_t i = s.nc; i < s.m; ++i) w[rw[i]] -= t[i];
    }
    for (int64_t si = (int64_t)S.sn.size() - 1; si >= 0; --si) {
      const Supernode &s = S.sn[si];
      const int32_t *rw = S.rows.data() + s.rows_off;
      const double *G = panels.data() + s.panel_off;
      for (int32_t j = 0; j < s.nc; ++j) {
        double acc = 0.0;
        for (int32_t i = j; i < s.m; ++i) {
          const double vi = i < s.nc ? dinv[rw[i]] * y[rw[i]] : -z[rw[i]];
          acc += G[(int64_t)j * s.m + i] * vi;
        }
        z[rw[j]] = acc;
      }
    }
  }
  return FE_OK;
}

int fe_set_graphs(fe_ctx *c, int32_t enable) {
  if (!c) return FE_EINVAL;
  c->use_graphs = enable != 0;
  return FE_OK;
}

int fe_set_kernel_timing(fe_ctx *c, int32_t enable) {
  if (!c) return FE_EINVAL;
  c->timing = enable != 0;
  return FE_OK;
}

int fe_kernel_times(fe_ctx *c, double *out_ms, int64_t *out_count, double *out_bytes, int32_t n) {
  if (!c) return FE_EINVAL;
  drain_timing(c);
  for (int k = 0; k < fe_ctx::kTimedKinds && k < n; ++k) {
    if (out_ms) out_ms[k] = c->t_ms[k];
    if (out_count) out_count[k] = c->t_count[k];
    if (out_bytes) out_bytes[k] = c->t_bytes[k];
    c->t_ms[k] = 0;
    c->t_count[k] = 0;
    c->t_bytes[k] = 0;
  }
  return FE_OK;
}

int fe_reset(fe_ctx *c) {
  if (!c) return FE_EINVAL;
  std::unique_lock<std::mutex> lk(c->mu);
  c->cv.wait(lk, [&] { return !c->job_pending && !c->job_running; });
  if (c->gpu_factor) (void)gf_collect_locked(c, true);
  c->step_count = 0;
  c->active_slot = -1;
  c->installed_tag = -1;
  c->ready_tag = -1;
  c->ready_slot = -1;
  c->job_status = FE_OK;
  c->have_prev_a = false;
  c->hist_count = 0;
  c->hist_next = 0;
  c->rot_valid = false;
  return FE_OK;
}

int fe_destroy(fe_ctx *c) {
  delete c;
  return FE_OK;
}

const char *fe_last_error(fe_ctx *c) {
  if (!c) return g_build_error.c_str();
  return c->err.c_str();
}

}  // extern "C"
