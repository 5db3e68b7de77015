// C ABI of libfeti (include/feti.h): problem lifetime, device memory, and the
// orchestration of assembly, batched factorisation and the projected PCG.
//
// Solve (section 4.3 of the paper):
//   e = R^T f,  d = sum_i B_i K_i^+ f_i - b,  Q = G^T G,  lambda_0 = G Q^{-1} e,
//   r_0 = d - F lambda_0,  w = P r,  z = P M^{-1} w,  CG on P^T F,
//   gamma = Q^{-1} G^T (F lambda - d),  u_i = K_i^+ (f_i - B_i^T lambda) + R_i gamma_i.
// The PCG iterations are captured in a HIP graph (graph_block iterations per
// replay) with all scalars on the device; the host reads one flag per replay.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <memory>
#include <string>
#include <vector>

#include "feti_impl.h"
#include "k_pcg.h"

using namespace feti;

namespace {

thread_local std::string g_setup_error;
constexpr int kGmresRestart = 30;   // Krylov vectors per flexible GMRES cycle of the refinement
constexpr int kDualRestart = 100;   // Krylov vectors per cycle of the projected dual GMRES
constexpr int kGsMax = (kDualRestart > kGmresRestart ? kDualRestart : kGmresRestart) + 1;   // basis vectors

struct DeviceAlloc {
  void* (*fn)(size_t, void*, void*) = nullptr;
  void (*fr)(void*, void*) = nullptr;
  void* ctx = nullptr;
};

}  // namespace

struct feti_problem {
  HostPlan P;
  std::string err;
  feti_options opt{};
  hipStream_t stream = nullptr;
  bool own_stream = false;
  // stream of the coarse factorisation (concurrent with the local one), its
  // fork/join events and the host data its uploads read
  hipStream_t stream_c = nullptr;
  hipEvent_t ev_cfork = nullptr, ev_cjoin = nullptr;
  hipEvent_t ev_asm = nullptr, ev_modes = nullptr;   // assembly done; rigid modes done (coarse stream)
  hipEvent_t ev_ffork = nullptr, ev_fjoin = nullptr; // arena and ELL reset on the coarse stream
  int32_t* h_nmodes = nullptr;                        // pinned: kernel dimension per subdomain
  SubInfo* h_sub = nullptr;                           // pinned: subdomain table with the coarse layout
  SubInfo h_qsub{};
  std::vector<Task> h_qt;
  const int h_big = 0x7fffffff;
  // pinned copies of the PCG state after the two replays in flight
  PcgState* h_state = nullptr;
  hipEvent_t ev_rep[2] = {nullptr, nullptr};
  DeviceAlloc da;
  std::vector<void*> allocs;
  size_t bytes = 0;
  bool factored = false;
  bool factored_linear = false;
  // FETI_KERNEL6 at a stressed state: the dual solve is of an approximate
  // tangent, and the outer refinement against the exact sparse tangent
  // (as for mixed precision) recovers the exact step
  bool approx_tangent = false;
  // the factors of the next factorisation serve only as the preconditioner of
  // a refinement against the exact operator: non-positive pivots may be
  // replaced (modified Cholesky); modified_pivots counts them
  bool allow_modified = false;
  int modified_pivots = 0;
  int h_errinit[4] = {0, 0, 0, 0};
  bool refined_out = false;     // the last result is in d_uglob
  // FETI_LOAD_STIFFNESS in a Newton step: the assembled operator of the
  // refinement includes -tau d f_p / dU at the state ls_U
  bool ls_on = false;
  const double* ls_U = nullptr;
  double ls_tau = 0.0;
  // flexible GMRES of the refinement: restart length gm, Krylov vectors V
  // (gm + 1) and preconditioned vectors Z (gm) of n_dof entries, work vector,
  // dot-product partials (device and pinned host), Hessenberg and rotations
  // FETI_DUAL_GMRES: projected GMRES on the dual problem, restart length dm,
  // Krylov vectors V (dm + 1), preconditioned vectors Z (dm), work vector;
  // dual_target: absolute stopping target of a warm-started solve (or < 0)
  bool dual_gmres = false;
  int dm = 0;
  double *d_dv = nullptr, *d_dz = nullptr, *d_dw = nullptr;
  double dual_target = -1.0;
  std::vector<double> dg_H, dg_g, dg_c, dg_s, dg_y, dg_h;
  // FETI_WARM_START: multipliers of the previous call's first dual solve
  double* d_lamp = nullptr;
  int64_t* d_gdesc = nullptr;   // interface tile descriptors of the GEMV (gemv_descriptors)
  bool have_prev = false;
  double warm_scale = 0.0;
  int gm = 0;
  double *d_gv = nullptr, *d_gz = nullptr, *d_gw = nullptr, *d_gdots = nullptr, *h_gdots = nullptr;
  std::vector<double> gm_H, gm_g, gm_c, gm_s, gm_y, gm_h;
  int n_coarse = 0;
  int nq = 0;   // coarse tiles
  DevIdx di;

  // static device data
  SubInfo* d_sub = nullptr;
  Task* d_tasks = nullptr;
  double *d_xyz = nullptr, *d_mat = nullptr, *d_fib = nullptr, *d_body = nullptr, *d_dirval = nullptr;
  int64_t *d_hex8 = nullptr, *d_pface = nullptr, *d_loc_node = nullptr;
  int32_t *d_elem_mat = nullptr, *d_loc_pos = nullptr, *d_loc_sub = nullptr, *d_loc_ncopy = nullptr;
  uint8_t* d_dmask = nullptr;
  int32_t *d_ps_a = nullptr, *d_ps_b = nullptr, *d_ps_nbr = nullptr, *d_ps_c0 = nullptr, *d_ps_c1 = nullptr;
  int32_t *d_pc_e = nullptr, *d_pc_ab = nullptr, *d_diag_slot = nullptr, *d_ell_col = nullptr;
  int32_t* d_env = nullptr;   // tile envelopes of the local matrices
  int32_t *d_fpos_lnode = nullptr, *d_f_sub = nullptr;
  int8_t* d_fpos_comp = nullptr;
  int32_t *d_uc_ptr = nullptr, *d_pf_ptr = nullptr, *d_pf_ent = nullptr;
  int64_t* d_uc_idx = nullptr;
  int32_t *d_qp_s = nullptr, *d_qp_t = nullptr, *d_qp_ptr = nullptr;
  int64_t *d_qe_bs = nullptr, *d_qe_bt = nullptr;
  double* d_qe_c = nullptr;

  // assembly / factor data
  double *d_Ke = nullptr, *d_fint = nullptr, *d_fbody = nullptr, *d_ell_val = nullptr, *d_U = nullptr;
  double *d_fnodal = nullptr;
  void *d_arena = nullptr, *d_linv = nullptr, *d_W = nullptr, *d_X = nullptr, *d_S = nullptr;
  double *d_t = nullptr, *d_kb1 = nullptr, *d_kb2 = nullptr, *d_bb_val = nullptr;
  int32_t *d_bb_slot = nullptr, *d_bb_col = nullptr;
  double *d_rfull = nullptr, *d_rb = nullptr, *d_work = nullptr, *d_rho = nullptr, *d_wbm = nullptr;
  double* d_mpart = nullptr;   // partial sums of the rotation test (k_modes_sweep)
  int32_t *d_nmodes = nullptr, *d_err = nullptr;
  // coarse
  SubInfo* d_qsub = nullptr;
  Task* d_qtasks = nullptr;
  int qtask_cap = 0;
  int32_t* d_qbsub = nullptr;
  double *d_qarena = nullptr, *d_qlinv = nullptr, *d_qW = nullptr, *d_qX = nullptr, *d_qpart = nullptr;
  HostPlan::Launch q_xtiles{};
  // vectors
  double *d_f = nullptr, *d_w = nullptr, *d_u = nullptr, *d_ul = nullptr;
  double *d_xb = nullptr, *d_yb = nullptr, *d_vb = nullptr, *d_part = nullptr;
  double *d_lam = nullptr, *d_r = nullptr, *d_s = nullptr, *d_q = nullptr, *d_wv = nullptr, *d_zv = nullptr;
  double *d_tv = nullptr, *d_d = nullptr, *d_bv = nullptr;
  double *d_cg = nullptr, *d_calpha = nullptr, *d_gamma = nullptr, *d_e = nullptr;
  double *d_dvals = nullptr, *d_out = nullptr;
  double *d_f0 = nullptr, *d_uglob = nullptr, *d_zero = nullptr;
  double* d_qdense = nullptr;
  int32_t* d_bco = nullptr;
  int2* d_rco = nullptr;     // per multiplier row: coarse codes of its two entries
  int ldg = 0;
  // scratch of the dual iteration: `own` is allocated at set-up; `sc` is the
  // set the kernels use (own, or the library's static array in
  // feti_solve_noalloc)
  PcgScratch own, sc;
  void* noalloc_base = nullptr;   // device address of the static scratch array on this device
  bool use_graph = true;
  // pinned host copies of the CG history and of dot-product partials, and the
  // work arrays of the condition estimate (sized at set-up)
  double *h_hist = nullptr, *h_dots = nullptr;
  std::vector<double> lz_d, lz_e;
  // graph
  hipGraphExec_t graph = nullptr;
  int graph_iters = 0;
  hipEvent_t ev[6] = {};
  // FETI_PROFILE: event pairs around the F GEMV of every captured iteration and
  // around every factor-update launch
  bool profile = false;
  std::vector<hipEvent_t> ev_gemv, ev_upd;   // burst start/end; pairs around update launches
  int n_upd_recorded = 0;
  // autotuner of the update launches (FETI_AUTOTUNE): factorisation f < 4
  // times form f of every update launch (0: 64x64 tiles, 1: 128x64, 2: 64x64
  // double-buffered, 3: double-buffered in 16-wide chunks at four workgroups
  // per CU where the launch holds update tasks only, else as 2); from then on
  // each launch uses its fastest form.  All forms give identical factors.
  // Launches are identified by the first task of their 64x64 form.
  static constexpr int kForms = 4;
  bool autotune = false;
  int tune_phase = 0;                          // < kForms: measuring; kForms: decided
  std::vector<int32_t> upd_first;              // update launches, by first task
  std::vector<float> t_form[kForms];
  std::vector<uint8_t> use_form;
  std::vector<hipEvent_t> ev_tune;
  int n_wide = -1, n_db = -1;
  double prof_gemv_ms = 0.0, prof_upd_ms = 0.0, upd_flops = 0.0, gemv_bytes = 0.0;
  int prof_gemv_n = 0, prof_upd_n = 0;
};

namespace {

#define HIPCHK(expr)                                                              \
  do {                                                                            \
    hipError_t e_ = (expr);                                                       \
    if (e_ != hipSuccess) {                                                       \
      p->err = std::string("HIP error: ") + hipGetErrorString(e_) + " at " #expr; \
      return FETI_EDEVICE;                                                        \
    }                                                                             \
  } while (0)

template <typename T>
feti_status dalloc(feti_problem* p, T*& out, size_t n) {
  out = nullptr;
  if (n == 0) n = 1;
  const size_t bytes = n * sizeof(T);
  void* ptr = nullptr;
  if (p->da.fn) {
    ptr = p->da.fn(bytes, (void*)p->stream, p->da.ctx);
    if (!ptr) {
      p->err = "device allocation of " + std::to_string(bytes) + " bytes failed";
      return FETI_ENOMEM;
    }
  } else {
    if (hipMalloc(&ptr, bytes) != hipSuccess) {
      (void)hipGetLastError();
      p->err = "hipMalloc of " + std::to_string(bytes) + " bytes failed";
      return FETI_ENOMEM;
    }
  }
  p->allocs.push_back(ptr);
  p->bytes += bytes;
  out = (T*)ptr;
  return FETI_OK;
}

template <typename T>
feti_status upload(feti_problem* p, T*& out, const std::vector<T>& v) {
  feti_status s = dalloc(p, out, v.size());
  if (s != FETI_OK) return s;
  if (!v.empty()) HIPCHK(hipMemcpyAsync(out, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice, p->stream));
  return FETI_OK;
}

#define TRY(expr)                   \
  do {                              \
    feti_status s_ = (expr);        \
    if (s_ != FETI_OK) return s_;   \
  } while (0)

size_t elt(const feti_problem* p) { return p->P.mixed ? sizeof(float) : sizeof(double); }

// Dense launches on the subdomain batch in the working precision.

int update_index(const feti_problem* p, const HostPlan::Launch& L) {
  const auto it = std::lower_bound(p->upd_first.begin(), p->upd_first.end(), L.first);
  return (it != p->upd_first.end() && *it == L.first) ? (int)(it - p->upd_first.begin()) : -1;
}

void dense(feti_problem* p, const HostPlan::Launch& L) {
  hipStream_t stream = p->stream;
  const bool upd = is_update_kind(L.kind) && L.count > 0;
  const bool timed = p->profile && upd && 2 * p->n_upd_recorded + 1 < (int)p->ev_upd.size();
  void* W = p->d_W;
  int form = 0, idx = -1;
  if (upd && p->autotune && (idx = update_index(p, L)) >= 0 && L.wcount > 0)
    form = p->tune_phase < feti_problem::kForms ? p->tune_phase : p->use_form[idx];
  const bool tuning = idx >= 0 && p->tune_phase < feti_problem::kForms;
  const bool wide = form == 1;
  const Task* t = p->d_tasks + (wide ? L.wfirst : L.first);
  const int count = wide ? L.wcount : L.count, split = wide ? L.wsplit : L.split;
  if (timed) (void)hipEventRecord(p->ev_upd[2 * p->n_upd_recorded], stream);
  if (tuning) (void)hipEventRecord(p->ev_tune[2 * idx], stream);
  if (p->P.mixed)
    launch_dense<float>(L.kind, t, count, p->d_sub, (float*)p->d_arena, (float*)p->d_linv, (float*)W,
                        (float*)p->d_X, p->d_err, stream, split, form, L.ndiag);
  else
    launch_dense<double>(L.kind, t, count, p->d_sub, (double*)p->d_arena, (double*)p->d_linv, (double*)W,
                         (double*)p->d_X, p->d_err, stream, split, form, L.ndiag);
  if (tuning) (void)hipEventRecord(p->ev_tune[2 * idx + 1], stream);
  if (timed) (void)hipEventRecord(p->ev_upd[2 * p->n_upd_recorded++ + 1], stream);
}

// After a factorisation: collect the autotuner's timings and advance it.
void autotune_step(feti_problem* p) {
  if (!p->autotune || p->tune_phase >= feti_problem::kForms) return;
  auto& dst = p->t_form[p->tune_phase];
  for (size_t k = 0; k < p->upd_first.size(); ++k) {
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, p->ev_tune[2 * k], p->ev_tune[2 * k + 1]) != hipSuccess) {
      (void)hipGetLastError();
      ms = 0.f;
    }
    dst[k] = ms;
  }
  if (++p->tune_phase == feti_problem::kForms) {
    p->n_wide = p->n_db = 0;
    for (size_t k = 0; k < p->upd_first.size(); ++k) {
      int best = 0;
      for (int f = 1; f < feti_problem::kForms; ++f)
        if (p->t_form[f][k] > 0.f && p->t_form[f][k] < p->t_form[best][k]) best = f;
      p->use_form[k] = (uint8_t)best;
      p->n_wide += best == 1;
      p->n_db += best >= 2;
    }
  }
}

// yb = M xb over the trailing blocks of all subdomains.  iface_only: the rows
// and columns of DOFs without multipliers are left out (the dual operator and
// the Dirichlet preconditioner); otherwise the whole trailing block takes part
// (the local pseudo-inverse).
void symv_local(feti_problem* p, const void* M, const double* xb, double* yb, const PcgState* st,
                int iface_only) {
  const HostPlan::Launch& L = p->P.sched_xtiles;
  if (p->P.mixed)
    pcg_symv_desc<float>(p->d_gdesc, L.count, (const float*)M, xb, p->d_part, p->di.NB, p->di.b_sub, p->d_sub, yb,
                         st, p->stream, iface_only);
  else
    pcg_symv_desc<double>(p->d_gdesc, L.count, (const double*)M, xb, p->d_part, p->di.NB, p->di.b_sub, p->d_sub,
                          yb, st, p->stream, iface_only);
}

// z = K^+ g for every subdomain (full local vectors), see k_kp_band and k_kp_tiles.
template <typename T>
void kpinv_t(feti_problem* p, const double* g, double* z) {
  const HostPlan& P = p->P;
  const T* A = (const T*)p->d_arena;
  hipStream_t st = p->stream;
  local_kp_band<T>(0, P.n_sub, P.max_nt_i, p->d_sub, p->d_env, A, (const T*)p->d_linv, g, p->d_w, st);
  local_kp_tiles<T>(1, P.n_sub, P.max_nt_b, p->d_sub, p->d_env, A, p->d_w, nullptr, g, nullptr, p->d_kb1, st);
  symv_local(p, p->d_X, p->d_kb1, p->d_kb2, nullptr, 0);
  local_kp_tiles<T>(2, P.n_sub, P.max_nt_i, p->d_sub, p->d_env, A, nullptr, p->d_kb2, p->d_w, p->d_t, nullptr, st);
  local_kp_band<T>(3, P.n_sub, P.max_nt_i, p->d_sub, p->d_env, A, (const T*)p->d_linv, p->d_t, z, st);
  vec_set_b2f(p->di, p->d_kb2, z, st);
}

void kpinv(feti_problem* p, const double* g, double* z) {
  if (p->P.mixed) kpinv_t<float>(p, g, z);
  else kpinv_t<double>(p, g, z);
}

// z = K^+ (f - B^T lambda) after kpinv_b(f): the right-hand side differs from
// f on interface DOFs only, so the interior forward solve w = L_II^{-1} f_I
// (d_w) and f_b - L_bI w (d_kb1) left by kpinv_b still hold; only xb = B^T
// lambda is subtracted before the interface and backward passes.
template <typename T>
void kpinv_recover_t(feti_problem* p, const double* xb, double* z) {
  const HostPlan& P = p->P;
  const T* A = (const T*)p->d_arena;
  hipStream_t st = p->stream;
  vec_axpby(P.NB, -1.0, xb, 1.0, p->d_kb1, st);
  symv_local(p, p->d_X, p->d_kb1, p->d_kb2, nullptr, 0);
  local_kp_tiles<T>(2, P.n_sub, P.max_nt_i, p->d_sub, p->d_env, A, nullptr, p->d_kb2, p->d_w, p->d_t, nullptr, st);
  local_kp_band<T>(3, P.n_sub, P.max_nt_i, p->d_sub, p->d_env, A, (const T*)p->d_linv, p->d_t, z, st);
  vec_set_b2f(p->di, p->d_kb2, z, st);
}

// Interface part only, zb = (K^+ g)_b = X (g_b - L_bI L_II^{-1} g_I), as a
// b-space vector: the interior back substitution is not needed for B K^+ g.
template <typename T>
void kpinv_b_t(feti_problem* p, const double* g, double* zb) {
  const HostPlan& P = p->P;
  const T* A = (const T*)p->d_arena;
  hipStream_t st = p->stream;
  local_kp_band<T>(0, P.n_sub, P.max_nt_i, p->d_sub, p->d_env, A, (const T*)p->d_linv, g, p->d_w, st);
  local_kp_tiles<T>(1, P.n_sub, P.max_nt_b, p->d_sub, p->d_env, A, p->d_w, nullptr, g, nullptr, p->d_kb1, st);
  symv_local(p, p->d_X, p->d_kb1, zb, nullptr, 0);
}
void kpinv_b(feti_problem* p, const double* g, double* zb) {
  if (p->P.mixed) kpinv_b_t<float>(p, g, zb);
  else kpinv_b_t<double>(p, g, zb);
}

// alpha = Q^{-1} g on the coarse space (alpha = 0 without coarse space).
void coarse_solve(feti_problem* p, const double* g, double* alpha, const PcgState* st) {
  if (p->n_coarse == 0) return;
  pcg_symv<double>(p->d_qtasks + p->q_xtiles.first, p->q_xtiles.count, p->d_qsub, p->d_qX, g, p->d_qpart,
                   (int64_t)p->nq * TS, p->d_qbsub, alpha, st, p->stream, 0);
}

// Projection by the fused kernels: g = Rb^T B^T x per subdomain, a = Q^{-1} g
// (dense inverse), and per multiplier row out = x - G a (see k_proj_apply for
// the modes: 0 plain, 1 with the r/lambda update, 2 with the PCG dot products).
void project_fused(feti_problem* p, int mode, int init, double* x, double* out, const double* w, PcgState* st,
                   double* hist) {
  const int nc = p->n_coarse;
  if (nc) {
    pcg_proj_gt(p->P.n_sub, p->d_sub, p->di, p->d_rb, x, p->d_q, mode == 1, p->sc.gpart, p->ldg, st, p->stream);
    pcg_coarse_dense(nc, nc, p->d_qdense, p->sc.gpart, p->ldg, p->d_calpha, st, p->stream);
  }
  pcg_proj_apply(mode, init, p->di, nc > 0, p->d_rco, p->d_rb, p->d_calpha, x, p->d_q, p->d_s, p->d_lam, out, w,
                 p->sc.fpart, p->sc.ticket + 1, st, hist, p->stream);
}

// q = F v
void apply_F(feti_problem* p, const double* v, double* q, const double* base, double sgn, const PcgState* st) {
  pcg_gather(p->di, 0, v, p->d_xb, st, p->stream);
  symv_local(p, p->d_X, p->d_xb, p->d_yb, st, 1);
  pcg_scatter(p->di, 0, p->d_yb, base, sgn, q, st, p->stream);
}

// out = M^{-1} w (scaled rows B_D; lumped, Dirichlet or identity)
void precondition(feti_problem* p, const double* w, double* out, const PcgState* st) {
  pcg_gather(p->di, 1, w, p->d_xb, st, p->stream);
  const double* y = p->d_xb;
  if (p->P.precond == FETI_PREC_LUMPED) {
    pcg_lumped(p->di, p->P.w_bb, p->d_bb_col, p->d_bb_val, p->d_xb, p->d_yb, st, p->stream);
    y = p->d_yb;
  } else if (p->P.precond == FETI_PREC_DIRICHLET) {
    symv_local(p, p->d_S, p->d_xb, p->d_yb, st, 1);
    y = p->d_yb;
  }
  pcg_scatter(p->di, 1, y, nullptr, 1.0, out, st, p->stream);
}

// One PCG iteration (ten or eleven launches, all scalars on the device):
//   xb = B^T s with s = z + beta s formed on the fly;  y = X xb (tile phase,
//   ordered reduction);  q = B y, alpha, and G^T q from y;  a = Q^{-1} G^T q;
//   r -= alpha q, lambda += alpha s, w -= alpha (q - G a);
//   t = M^{-1} w with G^T t from the preconditioner's interface output;
//   a = Q^{-1} G^T t;  z = t - G a, beta and the stopping test.
void pcg_iteration(feti_problem* p) {
  PcgState* st = p->sc.state;
  hipStream_t s = p->stream;
  const int nc = p->n_coarse;
  pcg_gather_s(p->di, p->d_zv, p->d_s, p->d_xb, st, s);
  symv_local(p, p->d_X, p->d_xb, p->d_yb, st, 1);
  pcg_scatter_dot_alpha_gt(p->di, p->P.n_sub, nc > 0, p->d_sub, p->d_rb, p->d_yb, p->d_zv, p->d_s, p->d_q,
                           p->sc.apart, st, p->sc.gpart, p->ldg, s);
  if (nc) pcg_coarse_dense(nc, nc, p->d_qdense, p->sc.gpart, p->ldg, p->d_calpha, st, s);
  pcg_proj_apply(1, 0, p->di, nc > 0, p->d_rco, p->d_rb, p->d_calpha, p->d_r, p->d_q, p->d_s, p->d_lam, p->d_wv,
                 nullptr, p->sc.fpart, p->sc.ticket + 1, st, nullptr, s, p->sc.apart);
  // preconditioner
  pcg_gather(p->di, 1, p->d_wv, p->d_xb, st, s);
  const double* y = p->d_xb;
  if (p->P.precond == FETI_PREC_LUMPED) {
    pcg_lumped(p->di, p->P.w_bb, p->d_bb_col, p->d_bb_val, p->d_xb, p->d_yb, st, s);
    y = p->d_yb;
  } else if (p->P.precond == FETI_PREC_DIRICHLET) {
    symv_local(p, p->d_S, p->d_xb, p->d_yb, st, 1);
    y = p->d_yb;
  }
  pcg_scatter_w_gt(p->di, p->P.n_sub, nc > 0, p->d_sub, p->d_rb, y, p->d_tv, st, p->sc.gpart, p->ldg, s);
  if (nc) pcg_coarse_dense(nc, nc, p->d_qdense, p->sc.gpart, p->ldg, p->d_calpha, st, s);
  pcg_proj_apply(2, 0, p->di, nc > 0, p->d_rco, p->d_rb, p->d_calpha, p->d_tv, p->d_q, p->d_s, p->d_lam, p->d_zv,
                 p->d_wv, p->sc.fpart, p->sc.ticket + 1, st, p->sc.hist, s);
}

// Condition estimate from the recorded (alpha, beta): extreme eigenvalues of
// the Lanczos tridiagonal by bisection on Sturm sequences.
double lanczos_kappa(const double* h, int m, std::vector<double>& d, std::vector<double>& e) {
  if (m <= 0 || (int)d.size() < m || (int)e.size() < m) return 1.0;
  std::fill(e.begin(), e.begin() + m, 0.0);
  for (int k = 0; k < m; ++k) {
    const double a = h[2 * k], b = h[2 * k + 1];
    d[k] = 1.0 / a + (k > 0 ? h[2 * (k - 1) + 1] / h[2 * (k - 1)] : 0.0);
    if (k + 1 < m) e[k] = std::sqrt(std::max(b, 0.0)) / a;
  }
  auto count_below = [&](double x) {
    int c = 0;
    double q = d[0] - x;
    if (q < 0) c++;
    for (int k = 1; k < m; ++k) {
      const double den = std::fabs(q) < 1e-300 ? 1e-300 : q;
      q = d[k] - x - e[k - 1] * e[k - 1] / den;
      if (q < 0) c++;
    }
    return c;
  };
  double lo = 1e300, hi = -1e300;
  for (int k = 0; k < m; ++k) {
    const double r = (k > 0 ? std::fabs(e[k - 1]) : 0.0) + std::fabs(e[k]);
    lo = std::min(lo, d[k] - r);
    hi = std::max(hi, d[k] + r);
  }
  auto kth = [&](int k) {
    double a = lo, b = hi;
    for (int it = 0; it < 200; ++it) {
      const double mid = 0.5 * (a + b);
      if (count_below(mid) > k) b = mid;
      else a = mid;
    }
    return 0.5 * (a + b);
  };
  const double lmin = kth(0), lmax = kth(m - 1);
  return lmin > 0 ? lmax / lmin : 0.0;
}

// Whether a solve of this problem can be refined by the flexible GMRES
// (solve_refined): mixed precision, FETI_KERNEL6 or a kernel tolerance above
// the exact test on an HGO problem (an approximate stressed tangent), or the
// exact Newton step with the load stiffness.
bool refinable(const feti_problem* p) {
  return p->P.mixed || (p->opt.flags & (FETI_KERNEL6 | FETI_LOAD_STIFFNESS)) ||
         (p->P.any_hgo && p->opt.kernel_tol > 1e-12);
}

feti_status setup_device(feti_problem* p) {
  HostPlan& P = p->P;
  p->di.NB = P.NB;
  p->di.NF = P.NF;
  p->di.n_lam = P.n_lam;
  TRY(upload(p, p->d_sub, P.sub));
  TRY(upload(p, p->d_env, P.env));
  TRY(upload(p, p->d_tasks, P.tasks));
  {   // descriptors of the interface tiles for the dual-operator GEMV
    std::vector<int64_t> gd;
    const HostPlan::Launch& XL = P.sched_xtiles;
    gemv_descriptors(P.tasks.data() + XL.first, XL.count, P.sub.data(), gd);
    if (!gd.empty()) TRY(upload(p, p->d_gdesc, gd));
  }
  TRY(upload(p, p->d_xyz, P.xyz));
  TRY(upload(p, p->d_hex8, P.hex8));
  TRY(upload(p, p->d_elem_mat, P.elem_mat));
  {
    std::vector<double> m(7 * P.mat.size());
    for (size_t k = 0; k < P.mat.size(); ++k) {
      const auto& q = P.mat[k];
      double v[7] = {(double)q.kind, q.E, q.nu, q.c, q.k1, q.k2, q.kappa};
      std::copy(v, v + 7, m.begin() + 7 * k);
    }
    TRY(upload(p, p->d_mat, m));
  }
  if (!P.fibers.empty()) TRY(upload(p, p->d_fib, P.fibers));
  if (!P.body_force.empty()) TRY(upload(p, p->d_body, P.body_force));
  TRY(upload(p, p->d_dirval, P.dir_val));
  TRY(upload(p, p->d_dmask, P.dir_mask));
  TRY(upload(p, p->d_loc_node, P.loc_node));
  TRY(upload(p, p->d_loc_pos, P.loc_pos));
  TRY(upload(p, p->d_loc_sub, P.loc_sub));
  TRY(upload(p, p->d_loc_ncopy, P.loc_ncopy));
  TRY(upload(p, p->d_ps_a, P.ps_a));
  TRY(upload(p, p->d_ps_b, P.ps_b));
  TRY(upload(p, p->d_ps_nbr, P.ps_nbr));
  TRY(upload(p, p->d_ps_c0, P.ps_c0));
  TRY(upload(p, p->d_ps_c1, P.ps_c1));
  TRY(upload(p, p->d_pc_e, P.pc_e));
  TRY(upload(p, p->d_pc_ab, P.pc_ab));
  TRY(upload(p, p->d_diag_slot, P.diag_slot));
  TRY(upload(p, p->d_ell_col, P.ell_col));
  if (P.precond == FETI_PREC_LUMPED) {
    TRY(upload(p, p->d_bb_slot, P.bb_slot));
    TRY(upload(p, p->d_bb_col, P.bb_col));
    TRY(dalloc(p, p->d_bb_val, P.bb_slot.size()));
  }
  TRY(upload(p, p->d_fpos_lnode, P.fpos_lnode));
  TRY(upload(p, p->d_fpos_comp, P.fpos_comp));
  TRY(upload(p, p->d_f_sub, P.f_sub));
  TRY(upload(p, p->d_uc_ptr, P.uc_ptr));
  TRY(upload(p, p->d_uc_idx, P.uc_idx));
  if (!P.pface.empty()) {
    TRY(upload(p, p->d_pface, P.pface));
    TRY(upload(p, p->d_pf_ptr, P.pf_ptr));
    TRY(upload(p, p->d_pf_ent, P.pf_ent));
  }
  TRY(upload(p, p->d_qp_s, P.qp_s));
  TRY(upload(p, p->d_qp_t, P.qp_t));
  TRY(upload(p, p->d_qp_ptr, P.qp_ptr));
  TRY(upload(p, p->d_qe_bs, P.qe_bs));
  TRY(upload(p, p->d_qe_bt, P.qe_bt));
  TRY(upload(p, p->d_qe_c, P.qe_c));
  {
    int32_t *a, *b, *c, *e;
    double *f, *g, *h, *w;
    int64_t *r0, *r1, *rg, *b2f;
    TRY(upload(p, a, P.g_ptr));
    TRY(upload(p, b, P.g_row));
    TRY(upload(p, c, P.b_sub));
    TRY(upload(p, f, P.g_coef));
    TRY(upload(p, w, P.r_w));
    TRY(upload(p, g, P.r_c0));
    TRY(upload(p, h, P.r_c1));
    TRY(upload(p, r0, P.r_b0));
    TRY(upload(p, r1, P.r_b1));
    TRY(upload(p, rg, P.r_gdof));
    TRY(upload(p, b2f, P.b2full));
    e = p->d_f_sub;
    p->di.g_ptr = a;
    p->di.g_row = b;
    p->di.b_sub = c;
    p->di.f_sub = e;
    p->di.g_coef = f;
    p->di.r_w = w;
    p->di.r_c0 = g;
    p->di.r_c1 = h;
    p->di.r_b0 = r0;
    p->di.r_b1 = r1;
    p->di.r_gdof = rg;
    p->di.b2full = b2f;
    int32_t *cp, *cc;
    double *cv0, *cv1;
    TRY(upload(p, cp, P.c_ptr));
    TRY(upload(p, cc, P.c_col));
    TRY(upload(p, cv0, P.c_v0));
    TRY(upload(p, cv1, P.c_v1));
    p->di.c_ptr = cp;
    p->di.c_col = cc;
    p->di.c_v0 = cv0;
    p->di.c_v1 = cv1;
  }
  // working memory
  const size_t e = elt(p);
  const size_t nde = 3 * (size_t)P.npe;   // DOFs per element
  TRY(dalloc(p, p->d_Ke, (size_t)P.n_elems * nde * nde));
  TRY(dalloc(p, p->d_fint, (size_t)P.n_elems * nde));
  TRY(dalloc(p, p->d_fbody, (size_t)P.n_elems * nde));
  TRY(dalloc(p, p->d_ell_val, (size_t)P.NF * P.ellw));
  TRY(dalloc(p, p->d_U, (size_t)P.n_dof));
  TRY(dalloc(p, p->d_fnodal, (size_t)P.n_dof));
  {
    char *a, *l, *w, *x, *s = nullptr;
    TRY(dalloc(p, a, (size_t)P.n_tiles * e));
    TRY(dalloc(p, l, (size_t)P.n_linv * e));
    TRY(dalloc(p, w, (size_t)P.n_xtiles * e));
    TRY(dalloc(p, x, (size_t)P.n_xtiles * e));
    if (P.precond == FETI_PREC_DIRICHLET) TRY(dalloc(p, s, (size_t)P.n_xtiles * e));
    p->d_arena = a;
    p->d_linv = l;
    p->d_W = w;
    p->d_X = x;
    p->d_S = s;
  }
  TRY(dalloc(p, p->d_rfull, (size_t)P.NF * 6));
  TRY(dalloc(p, p->d_work, (size_t)P.NF * 6));
  TRY(dalloc(p, p->d_mpart, (size_t)P.n_sub * MODES_CH * 13));
  TRY(dalloc(p, p->d_rb, (size_t)P.NB * 6));
  TRY(dalloc(p, p->d_rho, (size_t)P.n_sub));
  TRY(dalloc(p, p->d_wbm, (size_t)P.n_sub * 9));
  TRY(dalloc(p, p->d_nmodes, (size_t)P.n_sub));
  TRY(dalloc(p, p->d_err, 8));
  HIPCHK(hipMemsetAsync(p->d_err, 0, 8 * sizeof(int), p->stream));
  // coarse space: at most 6 per subdomain
  const int max_coarse = 6 * P.n_sub;
  const int nq_max = (max_coarse + TS - 1) / TS;
  const size_t qt = (size_t)nq_max * (nq_max + 1) / 2 * TS2;
  TRY(dalloc(p, p->d_qsub, 1));
  TRY(dalloc(p, p->d_qarena, qt));
  TRY(dalloc(p, p->d_qlinv, (size_t)nq_max * TS2));
  TRY(dalloc(p, p->d_qW, qt));
  TRY(dalloc(p, p->d_qX, qt));
  TRY(dalloc(p, p->d_qpart, (size_t)nq_max * nq_max * TS));
  {
    std::vector<int32_t> z((size_t)nq_max * TS, 0);
    TRY(upload(p, p->d_qbsub, z));
  }
  p->qtask_cap = 4 * nq_max * nq_max + 4 * nq_max + 16;
  TRY(dalloc(p, p->d_qtasks, (size_t)p->qtask_cap * (nq_max + 2)));
  TRY(dalloc(p, p->d_cg, (size_t)nq_max * TS));
  TRY(dalloc(p, p->d_calpha, (size_t)nq_max * TS));
  TRY(dalloc(p, p->d_gamma, (size_t)nq_max * TS));
  TRY(dalloc(p, p->d_e, (size_t)nq_max * TS));
  // coarse vectors: padding entries stay zero (kernels write real entries only)
  vec_fill((int64_t)nq_max * TS, 0.0, p->d_cg, p->stream);
  vec_fill((int64_t)nq_max * TS, 0.0, p->d_calpha, p->stream);
  vec_fill((int64_t)nq_max * TS, 0.0, p->d_gamma, p->stream);
  vec_fill((int64_t)nq_max * TS, 0.0, p->d_e, p->stream);
  // vectors
  TRY(dalloc(p, p->d_f, (size_t)P.NF));
  TRY(dalloc(p, p->d_w, (size_t)P.NF));
  TRY(dalloc(p, p->d_u, (size_t)P.NF));
  TRY(dalloc(p, p->d_ul, (size_t)P.NF));
  TRY(dalloc(p, p->d_t, (size_t)P.NF));
  TRY(dalloc(p, p->d_kb1, (size_t)P.NB));
  TRY(dalloc(p, p->d_kb2, (size_t)P.NB));
  TRY(dalloc(p, p->d_xb, (size_t)P.NB));
  TRY(dalloc(p, p->d_yb, (size_t)P.NB));
  TRY(dalloc(p, p->d_vb, (size_t)P.NB));
  TRY(dalloc(p, p->d_part, (size_t)std::max<int64_t>(P.n_part, 1)));
  const size_t nl = (size_t)std::max<int64_t>(P.n_lam, 1);
  TRY(dalloc(p, p->d_lam, nl));
  TRY(dalloc(p, p->d_r, nl));
  TRY(dalloc(p, p->d_s, nl));
  TRY(dalloc(p, p->d_q, nl));
  TRY(dalloc(p, p->d_wv, nl));
  TRY(dalloc(p, p->d_zv, nl));
  TRY(dalloc(p, p->d_tv, nl));
  TRY(dalloc(p, p->d_d, nl));
  TRY(dalloc(p, p->d_bv, nl));
  if (p->opt.flags & FETI_WARM_START) TRY(dalloc(p, p->d_lamp, nl));
  TRY(dalloc(p, p->d_dvals, (size_t)P.n_dof));
  TRY(dalloc(p, p->d_out, (size_t)P.n_dof));
  // the flexible GMRES refinement runs for mixed precision, six-mode or
  // tolerance-selected kernels of stressed (HGO) tangents, and the exact
  // Newton step; its buffers exist exactly then (see refinable())
  const bool refine = refinable(p);
  if (refine || (p->opt.flags & FETI_PROFILE)) {   // refinement / residual report
    TRY(dalloc(p, p->d_f0, (size_t)P.NF));
    TRY(dalloc(p, p->d_uglob, (size_t)P.n_dof));
    TRY(dalloc(p, p->d_zero, (size_t)P.n_dof));
    vec_fill(P.n_dof, 0.0, p->d_zero, p->stream);
  }
  p->dual_gmres = (p->opt.flags & FETI_DUAL_GMRES) != 0;
  if (p->dual_gmres) {
    const int m = std::min(std::max(p->opt.max_it, 1), kDualRestart);
    p->dm = m;
    TRY(dalloc(p, p->d_dv, (size_t)(m + 1) * nl));
    TRY(dalloc(p, p->d_dz, (size_t)m * nl));
    TRY(dalloc(p, p->d_dw, nl));
    p->dg_H.assign((size_t)(m + 1) * m, 0.0);
    p->dg_g.assign(m + 1, 0.0);
    p->dg_c.assign(m, 0.0);
    p->dg_s.assign(m, 0.0);
    p->dg_y.assign(m, 0.0);
    p->dg_h.assign(m + 1, 0.0);
  }
  if (p->dual_gmres || refine) {   // cgs2: partial sums, then two coefficient vectors and a norm
    TRY(dalloc(p, p->d_gdots, (size_t)kGsMax * DOT_PARTS + 2 * kGsMax + 1));
    HIPCHK(hipHostMalloc((void**)&p->h_gdots, (2 * kGsMax + 1) * sizeof(double), hipHostMallocDefault));
  }
  if (refine) {   // flexible GMRES
    const int m = std::min(std::max(p->opt.ir_max, 1), kGmresRestart);
    p->gm = m;
    TRY(dalloc(p, p->d_gv, (size_t)(m + 1) * P.n_dof));
    TRY(dalloc(p, p->d_gz, (size_t)m * P.n_dof));
    TRY(dalloc(p, p->d_gw, (size_t)P.n_dof));
    p->gm_H.assign((size_t)(m + 1) * m, 0.0);
    p->gm_g.assign(m + 1, 0.0);
    p->gm_c.assign(m, 0.0);
    p->gm_s.assign(m, 0.0);
    p->gm_y.assign(m, 0.0);
    p->gm_h.assign(m + 1, 0.0);
  }
  PcgScratch& o = p->own;
  TRY(dalloc(p, o.dots, 2 * DOT_PARTS));
  o.hist_cap = std::max(1, p->opt.max_it);
  TRY(dalloc(p, o.hist, 2 * (size_t)o.hist_cap));
  TRY(dalloc(p, o.state, 1));
  TRY(dalloc(p, o.ticket, 4));
  HIPCHK(hipMemsetAsync(o.ticket, 0, 4 * sizeof(int), p->stream));
  TRY(dalloc(p, o.fpart, 2 * FUSE_BLOCKS));
  TRY(dalloc(p, o.apart, FUSE_BLOCKS));
  TRY(dalloc(p, p->d_qdense, (size_t)max_coarse * max_coarse));
  p->ldg = max_coarse;
  TRY(dalloc(p, o.gpart, (size_t)4 * max_coarse));
  p->sc = o;
  HIPCHK(hipHostMalloc((void**)&p->h_hist, 2 * (size_t)o.hist_cap * sizeof(double), hipHostMallocDefault));
  HIPCHK(hipHostMalloc((void**)&p->h_dots, 2 * DOT_PARTS * sizeof(double), hipHostMallocDefault));
  p->lz_d.resize(o.hist_cap);
  p->lz_e.resize(o.hist_cap);
  {
    int dev = -1;
    HIPCHK(hipGetDevice(&dev));
    p->noalloc_base = noalloc_scratch(dev);   // NULL: feti_solve_noalloc reports EDEVICE
  }
  TRY(dalloc(p, p->d_bco, (size_t)P.NB));
  TRY(dalloc(p, p->d_rco, (size_t)P.n_lam));
  for (auto& ev : p->ev) HIPCHK(hipEventCreate(&ev));
  HIPCHK(hipHostMalloc((void**)&p->h_state, 2 * sizeof(PcgState), hipHostMallocDefault));
  HIPCHK(hipStreamCreateWithFlags(&p->stream_c, hipStreamNonBlocking));
  HIPCHK(hipEventCreateWithFlags(&p->ev_cfork, hipEventDisableTiming));
  HIPCHK(hipEventCreateWithFlags(&p->ev_cjoin, hipEventDisableTiming));
  HIPCHK(hipEventCreateWithFlags(&p->ev_asm, hipEventDisableTiming));
  HIPCHK(hipEventCreateWithFlags(&p->ev_modes, hipEventDisableTiming));
  HIPCHK(hipEventCreateWithFlags(&p->ev_ffork, hipEventDisableTiming));
  HIPCHK(hipEventCreateWithFlags(&p->ev_fjoin, hipEventDisableTiming));
  HIPCHK(hipHostMalloc((void**)&p->h_nmodes, std::max(1, P.n_sub) * sizeof(int32_t), hipHostMallocDefault));
  HIPCHK(hipHostMalloc((void**)&p->h_sub, std::max<size_t>(1, P.sub.size()) * sizeof(SubInfo), hipHostMallocDefault));
  for (auto& ev : p->ev_rep) HIPCHK(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
  p->profile = (p->opt.flags & FETI_PROFILE) != 0;
  if (p->profile) {
    p->ev_gemv.resize(2);
    for (auto& ev : p->ev_gemv) HIPCHK(hipEventCreate(&ev));
    // no system-scope fence at these events: they bracket single launches
    p->ev_upd.resize(2 * (P.sched_interior.size() + P.sched_iface.size() + 2));
    for (auto& ev : p->ev_upd) HIPCHK(hipEventCreateWithFlags(&ev, hipEventDisableSystemFence));
  }
  p->autotune = (p->opt.flags & FETI_AUTOTUNE) != 0;
  if (p->autotune) {
    auto reg = [&](const HostPlan::Launch& L) {
      if (is_update_kind(L.kind) && L.count > 0 && L.wcount > 0) p->upd_first.push_back(L.first);
    };
    for (const auto& L : P.sched_interior) reg(L);
    reg(P.sched_schur);
    for (const auto& L : P.sched_iface) reg(L);
    std::sort(p->upd_first.begin(), p->upd_first.end());
    const size_t nl = p->upd_first.size();
    for (auto& tf : p->t_form) tf.assign(nl, 0.f);
    p->use_form.assign(nl, 0);
    p->ev_tune.resize(2 * nl);
    for (auto& ev : p->ev_tune) HIPCHK(hipEventCreateWithFlags(&ev, hipEventDisableSystemFence));
  }
  // algorithmic work: bytes of the packed symmetric interface inverses read by
  // one GEMV, and flops of the update launches counted on real (unpadded)
  // rows: tile updates (lower triangle only for diagonal tiles) and the rows
  // of the factor inverses fused into them
  {
    const double es = (double)elt(p);
    double bytes = 0.0, fl = 0.0;
    for (const auto& si : P.sub) bytes += 0.5 * si.n_if * (si.n_if + 1.0) * es;
    auto real = [&](const SubInfo& si, int t) -> double {
      if (t < si.nt_i) return std::min(TS, si.n_ii - t * TS);
      return std::min(TS, si.n_b - (t - si.nt_i) * TS);
    };
    auto add = [&](const HostPlan::Launch& L) {
      if (!is_update_kind(L.kind)) return;
      const int nupd = L.kind == K_UPDATE ? L.count : L.split;
      for (int k = 0; k < L.count; ++k) {
        const Task& t = P.tasks[L.first + k];
        const SubInfo& si = P.sub[t.sub];
        if (k < nupd) {
          double inner = 0.0;
          for (int q = t.k0; q < t.k1; ++q) inner += real(si, q);
          const double ri = real(si, t.i), rj = real(si, t.j);
          fl += (t.i == t.j ? ri * (ri + 1.0) : 2.0 * ri * rj) * inner;
        } else if (t.i != t.j) {
          // inverse row: sum_k L_ik W_kj, then L_ii^{-1} times it (tile indices
          // local to the interface block)
          const int off = si.nt_i;
          const double ri = real(si, off + t.i), rj = real(si, off + t.j);
          double inner = 0.0;
          for (int q = t.k0; q < t.i; ++q) inner += real(si, off + q);
          fl += 2.0 * ri * rj * inner + 2.0 * ri * ri * rj;
        }
      }
    };
    for (const auto& L : P.sched_interior) add(L);
    for (const auto& L : P.sched_iface) add(L);
    add(P.sched_schur);
    p->gemv_bytes = bytes;
    p->upd_flops = fl;
  }
  HIPCHK(hipStreamSynchronize(p->stream));
  return FETI_OK;
}

// ---------------------------------------------------------------------------
// Coarse matrix Q = G^T G, its Cholesky factor and explicit inverse (FP64),
// on stream st.  Needs the kernel bases and the coarse layout only, so it
// runs beside the batched local factorisation.  The host data it uploads
// (h_qsub, h_qt, h_big) live in the problem until the copies are done.
feti_status coarse_factor(feti_problem* p, hipStream_t st) {
  HostPlan& P = p->P;
  SubInfo& q = p->h_qsub;
  q = SubInfo{};
  q.n_ii = 0;
  q.n_b = p->n_coarse;
  q.n_if = p->n_coarse;
  q.nt_i = 0;
  q.nt_b = p->nq;
  q.nt = p->nq;
  q.floating = 0;
  HIPCHK(hipMemcpyAsync(p->d_qsub, &q, sizeof(SubInfo), hipMemcpyHostToDevice, st));
  std::vector<SubInfo> qs{q};
  std::vector<Task>& qt = p->h_qt;
  qt.clear();
  std::vector<HostPlan::Launch> qi, qf, qr;
  HostPlan::Launch qsch, qla, qx, qall;
  build_factor_schedule(qs, qt, qi, qsch, qf, qr, qla, qx, qall);
  p->q_xtiles = qx;
  if ((int)qt.size() > p->qtask_cap * (p->nq + 2)) {
    p->err = "coarse task list overflow";
    return FETI_EDEVICE;
  }
  HIPCHK(hipMemcpyAsync(p->d_qtasks, qt.data(), qt.size() * sizeof(Task), hipMemcpyHostToDevice, st));
  launch_init_arena<double>(p->d_qtasks + qall.first, qall.count, p->d_qsub, p->d_qarena, st);
  CoarseArgs c;
  c.n_pairs = (int)P.qp_s.size();
  c.qp_s = p->d_qp_s;
  c.qp_t = p->d_qp_t;
  c.qp_ptr = p->d_qp_ptr;
  c.qe_bs = p->d_qe_bs;
  c.qe_bt = p->d_qe_bt;
  c.qe_c = p->d_qe_c;
  c.subs = p->d_sub;
  c.rb = p->d_rb;
  c.q = p->d_qarena;
  asm_coarse(c, st);
  auto qd = [&](const HostPlan::Launch& L) {
    launch_dense<double>(L.kind, p->d_qtasks + L.first, L.count, p->d_qsub, p->d_qarena, p->d_qlinv, p->d_qW,
                         p->d_qX, p->d_err + 4, st, L.split, 0, L.ndiag);
  };
  HIPCHK(hipMemcpyAsync(p->d_err + 4, &p->h_big, sizeof(int), hipMemcpyHostToDevice, st));
  for (const auto& L : qf) qd(L);
  for (const auto& L : qr) qd(L);
  qd(qla);
  coarse_to_dense(p->n_coarse, p->n_coarse, p->d_qX, p->d_qdense, st);
  return FETI_OK;
}

feti_status do_factor(feti_problem* p, const double* U_dev) {
  HostPlan& P = p->P;
  hipStream_t st = p->stream;
  HIPCHK(hipEventRecord(p->ev[0], st));
  AsmArgs a;
  a.n_elems = P.n_elems;
  a.xyz = p->d_xyz;
  a.npe = P.npe;
  a.hex8 = p->d_hex8;
  a.elem_mat = p->d_elem_mat;
  a.mat = p->d_mat;
  a.fibers = p->d_fib;
  a.body = p->d_body;
  a.U = U_dev;
  a.Ke = p->d_Ke;
  a.fint = p->d_fint;
  // local factor flags: [0] first failing subdomain, [1] first element
  // inverted by U, [2] modified pivots allowed, [3] their count; [4..7] the
  // coarse factor's (never modified)
  const int big = 0x7fffffff;
  p->h_errinit[0] = big;
  p->h_errinit[1] = big;
  p->h_errinit[2] = p->allow_modified ? 1 : 0;
  p->h_errinit[3] = 0;
  HIPCHK(hipMemcpyAsync(p->d_err, p->h_errinit, 4 * sizeof(int), hipMemcpyHostToDevice, st));
  a.fbody = p->d_fbody;
  a.inverted = p->d_err + 1;
  // the arena fill does not need the element matrices: it runs on the coarse
  // stream while the elements are integrated.  The ELL values need no reset:
  // the gather writes every filled slot (the node pairs of the plan), and
  // every reader stops at, or skips, the empty ones.
  HIPCHK(hipEventRecord(p->ev_ffork, st));
  HIPCHK(hipStreamWaitEvent(p->stream_c, p->ev_ffork, 0));
  const auto& AT = P.sched_alltiles;
  if (P.mixed)
    launch_init_arena<float>(p->d_tasks + AT.first, AT.count, p->d_sub, (float*)p->d_arena, p->stream_c);
  else
    launch_init_arena<double>(p->d_tasks + AT.first, AT.count, p->d_sub, (double*)p->d_arena, p->stream_c);
  HIPCHK(hipEventRecord(p->ev_fjoin, p->stream_c));
  asm_elements(a, P.any_hgo, st);
  HIPCHK(hipStreamWaitEvent(st, p->ev_fjoin, 0));
  GatherArgs g;
  g.n_slots = (int64_t)P.ps_a.size();
  g.ps_a = p->d_ps_a;
  g.ps_b = p->d_ps_b;
  g.ps_nbr = p->d_ps_nbr;
  g.ps_c0 = p->d_ps_c0;
  g.ps_c1 = p->d_ps_c1;
  g.pc_e = p->d_pc_e;
  g.pc_ab = p->d_pc_ab;
  g.loc_sub = p->d_loc_sub;
  g.loc_pos = p->d_loc_pos;
  g.subs = p->d_sub;
  g.Ke = p->d_Ke;
  g.npe = P.npe;
  g.ell_val = p->d_ell_val;
  g.NF = P.NF;
  if (P.mixed) asm_gather<float>(g, (float*)p->d_arena, st);
  else asm_gather<double>(g, (double*)p->d_arena, st);
  ModesArgs m;
  m.n_sub = P.n_sub;
  m.subs = p->d_sub;
  m.loc_node = p->d_loc_node;
  m.loc_pos = p->d_loc_pos;
  m.fpos_lnode = p->d_fpos_lnode;
  m.fpos_comp = p->d_fpos_comp;
  m.xyz = p->d_xyz;
  m.U = U_dev;
  m.ell_col = p->d_ell_col;
  m.ell_val = p->d_ell_val;
  m.NF = P.NF;
  m.ellw = P.ellw;
  m.dmask = p->d_dmask;
  m.test_rotations = (P.any_hgo && U_dev && !(p->opt.flags & FETI_KERNEL6)) ? 1 : 0;
  m.kernel_tol = p->opt.kernel_tol;
  // the dual solve is of an approximate tangent (refined against the exact
  // one) with six-mode kernels, or with a kernel test looser than exact
  p->approx_tangent = P.any_hgo && U_dev && ((p->opt.flags & FETI_KERNEL6) || p->opt.kernel_tol > 1e-12);
  m.rfull = p->d_rfull;
  m.rb = p->d_rb;
  m.n_modes = p->d_nmodes;
  m.work = p->d_work;
  m.part = p->d_mpart;
  if (P.precond == FETI_PREC_LUMPED) lumped_fill(p->di, P.w_bb, p->d_bb_slot, p->d_ell_val, p->d_bb_val, st);
  HIPCHK(hipEventRecord(p->ev[1], st));
  // The rigid-body modes read only the assembled sparse rows, and the interior
  // steps and the Schur update do not need them: they run on the coarse
  // stream beside those steps, with the kernel dimensions copied back.
  HIPCHK(hipEventRecord(p->ev_asm, st));
  HIPCHK(hipStreamWaitEvent(p->stream_c, p->ev_asm, 0));
  asm_modes(m, p->stream_c);
  HIPCHK(hipMemcpyAsync(p->h_nmodes, p->d_nmodes, P.n_sub * sizeof(int32_t), hipMemcpyDeviceToHost, p->stream_c));
  HIPCHK(hipEventRecord(p->ev_modes, p->stream_c));
  // batched factorisation: interior steps and Schur update
  p->n_upd_recorded = 0;
  p->prof_upd_ms = 0.0;
  p->prof_upd_n = 0;
  p->prof_gemv_ms = 0.0;
  p->prof_gemv_n = 0;

  for (const auto& L : P.sched_interior) dense(p, L);
  dense(p, P.sched_schur);
  // coarse layout from the kernel dimensions (the host waits for the modes
  // while the GPU runs the steps above); the table is uploaded after the Schur
  // update in stream order, so no kernel before it sees it change
  HIPCHK(hipEventSynchronize(p->ev_modes));
  int off = 0;
  for (int s = 0; s < P.n_sub; ++s) {
    P.sub[s].n_modes = p->h_nmodes[s];
    P.sub[s].coarse_off = off;
    off += p->h_nmodes[s];
  }
  p->n_coarse = off;
  p->nq = (off + TS - 1) / TS;
  std::copy(P.sub.begin(), P.sub.end(), p->h_sub);
  HIPCHK(hipMemcpyAsync(p->d_sub, p->h_sub, P.sub.size() * sizeof(SubInfo), hipMemcpyHostToDevice, st));
  fill_bco(p->di, p->d_sub, p->d_bco, p->d_rco, st);
  // the modes (rb) are read by the regularisation below
  HIPCHK(hipStreamWaitEvent(st, p->ev_modes, 0));
  // the coarse problem on its own stream, beside the interface factorisation
  if (p->n_coarse > 0) {
    HIPCHK(hipEventRecord(p->ev_cfork, st));
    HIPCHK(hipStreamWaitEvent(p->stream_c, p->ev_cfork, 0));
    TRY(coarse_factor(p, p->stream_c));
    HIPCHK(hipEventRecord(p->ev_cjoin, p->stream_c));
  }
  const auto& XT = P.sched_xtiles;
  if (P.precond == FETI_PREC_DIRICHLET) {
    if (P.mixed)
      launch_copy_iface<float>(p->d_tasks + XT.first, XT.count, p->d_sub, (const float*)p->d_arena,
                               (float*)p->d_S, st);
    else
      launch_copy_iface<double>(p->d_tasks + XT.first, XT.count, p->d_sub, (const double*)p->d_arena,
                                (double*)p->d_S, st);
  }
  if (P.mixed) {
    launch_rho<float>(P.n_sub, p->d_sub, (const float*)p->d_arena, p->d_rho, st);
    launch_regularise<float>(p->d_tasks + XT.first, XT.count, p->d_sub, p->d_rb, p->d_rho, (float*)p->d_arena, st);
  } else {
    launch_rho<double>(P.n_sub, p->d_sub, (const double*)p->d_arena, p->d_rho, st);
    launch_regularise<double>(p->d_tasks + XT.first, XT.count, p->d_sub, p->d_rb, p->d_rho, (double*)p->d_arena,
                              st);
  }
  for (const auto& L : P.sched_iface) dense(p, L);
  for (const auto& L : P.sched_trtri) dense(p, L);
  dense(p, P.sched_lauum);
  {
    bool any_partial = false;
    for (const auto& si : P.sub) any_partial |= (si.floating == 1 && si.n_modes < 6);
    if (any_partial) {
      if (P.mixed)
        launch_woodbury<float>(P.n_sub, P.max_nt_b, p->d_tasks + XT.first, XT.count, p->d_sub, (float*)p->d_X,
                               p->d_rb, p->d_rho, p->d_work, p->d_wbm, st);
      else
        launch_woodbury<double>(P.n_sub, P.max_nt_b, p->d_tasks + XT.first, XT.count, p->d_sub,
                                (double*)p->d_X, p->d_rb, p->d_rho, p->d_work, p->d_wbm, st);
    }
  }
  if (p->n_coarse > 0) HIPCHK(hipStreamWaitEvent(st, p->ev_cjoin, 0));
  HIPCHK(hipEventRecord(p->ev[2], st));
  int errs[8] = {0x7fffffff, 0, 0, 0, 0x7fffffff, 0, 0, 0};
  HIPCHK(hipMemcpyAsync(errs, p->d_err, 8 * sizeof(int), hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  for (int k = 0; k < p->n_upd_recorded; ++k) {
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, p->ev_upd[2 * k], p->ev_upd[2 * k + 1]) == hipSuccess) {
      p->prof_upd_ms += ms;
      p->prof_upd_n++;
    } else {
      (void)hipGetLastError();
    }
  }
  autotune_step(p);
  if (errs[0] != 0x7fffffff) {
    p->err = std::string(p->allow_modified ? "non-finite" : "non-positive") + " pivot in the local factor of subdomain " +
             std::to_string(errs[0]);
    p->factored = false;
    return FETI_ENOTSPD;
  }
  p->modified_pivots = errs[3];
  if (errs[1] != 0x7fffffff) {
    p->err = "element " + std::to_string(errs[1]) + " is inverted by the displacement (det F <= 0)";
    p->factored = false;
    return FETI_EINVAL;
  }
  if (p->n_coarse > 0 && errs[4] != 0x7fffffff) {
    p->err = "coarse matrix G^T G is not positive definite";
    p->factored = false;
    return FETI_ENOTSPD;
  }
  p->factored = true;
  return FETI_OK;
}

// Dual solve for the local right-hand sides already in d_f and the Dirichlet
// data in d_dvals; writes the local displacements to d_u.  A correction solve
// (first = false) leaves the start event of the PCG phase where the first
// solve put it.
// Whether the stopping rule ||w|| <= rtol ||w_0|| is expected within n more
// PCG iterations of state h, at the faster of the mean reduction rate so far
// and that since the previous check (prev_it, prev_wn; prev_it = 0: none).
bool pcg_converges_within(const PcgState& h, int prev_it, double prev_wn, int n) {
  if (h.it <= 0 || !(h.w0 > 0.0) || !(h.wn > 0.0)) return false;
  const double ratio = h.wn / h.w0, target = h.rtol;
  if (ratio <= target) return true;
  double lrate = std::log(ratio) / h.it;   // log of the mean reduction per iteration
  if (prev_it > 0 && h.it > prev_it && prev_wn > 0.0)
    lrate = std::min(lrate, std::log(h.wn / prev_wn) / (h.it - prev_it));
  if (!(lrate < 0.0)) return false;
  return std::log(target / ratio) / lrate <= n;
}

feti_status dev_norm(feti_problem* p, const double* v, int64_t n, double* out);
feti_status cgs2(feti_problem* p, int64_t n, const double* V, int64_t ld, int k, double* w, double* h, double* nrm);

// Projected GMRES on the dual problem (FETI_DUAL_GMRES), for local operators
// that are not positive definite: P^T F lambda = P^T d on lambda_0 +
// range(P), right-preconditioned by P M^{-1} P (section 4.3 solves this
// system by CG; the paper notes that the FETI methods work for other systems
// with GMRES, section 3.2).  Starts from d_lam with d_r = d - F lambda;
// Arnoldi on w = P F z, z = P M^{-1} v, classical Gram-Schmidt with one
// reorthogonalisation, Givens rotations on the host, restarts every dm
// vectors; stops at ||P r|| <= target (rtol ||P r_0||, or the warm start's
// absolute target).  Leaves lambda in d_lam and d - F lambda in d_r.
feti_status dual_gmres(feti_problem* p, double rtol, int* iters_out, int* status_out, double* rel_out) {
  const int64_t n = p->P.n_lam;
  const int m = p->dm;
  PcgState* st = p->sc.state;   // initialised, never halted here
  auto V = [&](int j) { return p->d_dv + (size_t)j * n; };
  auto Z = [&](int j) { return p->d_dz + (size_t)j * n; };
  std::vector<double>& H = p->dg_H;
  std::vector<double>& g = p->dg_g;
  std::vector<double>& cs = p->dg_c;
  std::vector<double>& sn = p->dg_s;
  std::vector<double>& y = p->dg_y;
  std::vector<double>& hv = p->dg_h;
  project_fused(p, 0, 0, p->d_r, p->d_wv, nullptr, st, nullptr);
  double beta = 0.0;
  TRY(dev_norm(p, p->d_wv, n, &beta));
  const double beta0 = beta;
  const double target = p->dual_target >= 0.0 ? p->dual_target : rtol * beta0;
  int total = 0;
  while (beta > target && total < p->opt.max_it) {
    std::fill(H.begin(), H.end(), 0.0);
    std::fill(g.begin(), g.end(), 0.0);
    g[0] = beta;
    vec_axpby(n, 1.0 / beta, p->d_wv, 0.0, V(0), p->stream);
    double cur = beta;
    int k = 0;
    for (int j = 0; j < m && total < p->opt.max_it; ++j) {
      precondition(p, V(j), p->d_tv, st);
      project_fused(p, 0, 0, p->d_tv, Z(j), nullptr, st, nullptr);
      apply_F(p, Z(j), p->d_q, nullptr, 1.0, nullptr);
      project_fused(p, 0, 0, p->d_q, p->d_dw, nullptr, st, nullptr);
      double hn = 0.0;
      TRY(cgs2(p, n, V(0), n, j + 1, p->d_dw, hv.data(), &hn));
      for (int i = 0; i <= j; ++i) H[(size_t)j * (m + 1) + i] = hv[i];
      H[(size_t)j * (m + 1) + j + 1] = hn;
      if (hn > 0.0) vec_axpby(n, 1.0 / hn, p->d_dw, 0.0, V(j + 1), p->stream);
      double* col = &H[(size_t)j * (m + 1)];
      for (int i = 0; i < j; ++i) {
        const double t = cs[i] * col[i] + sn[i] * col[i + 1];
        col[i + 1] = -sn[i] * col[i] + cs[i] * col[i + 1];
        col[i] = t;
      }
      const double den = std::hypot(col[j], col[j + 1]);
      cs[j] = den > 0 ? col[j] / den : 1.0;
      sn[j] = den > 0 ? col[j + 1] / den : 0.0;
      col[j] = den;
      col[j + 1] = 0.0;
      g[j + 1] = -sn[j] * g[j];
      g[j] = cs[j] * g[j];
      cur = std::fabs(g[j + 1]);
      ++total;
      k = j + 1;
      if (cur <= target || hn == 0.0) break;
    }
    for (int i = k - 1; i >= 0; --i) {
      double acc = g[i];
      for (int l = i + 1; l < k; ++l) acc -= H[(size_t)l * (m + 1) + i] * y[l];
      const double d = H[(size_t)i * (m + 1) + i];
      y[i] = d != 0.0 ? acc / d : 0.0;
    }
    for (int i = 0; i < k; ++i) vec_axpby(n, y[i], Z(i), 1.0, p->d_lam, p->stream);
    // true residual r = d - F lambda and w = P r of the updated multipliers
    apply_F(p, p->d_lam, p->d_r, p->d_d, -1.0, nullptr);
    project_fused(p, 0, 0, p->d_r, p->d_wv, nullptr, st, nullptr);
    TRY(dev_norm(p, p->d_wv, n, &beta));
  }
  *iters_out = total;
  *status_out = beta <= target ? FETI_OK : FETI_ENOCONV;
  *rel_out = beta0 > 0 ? beta / beta0 : 0.0;
  return FETI_OK;
}

feti_status solve_core(feti_problem* p, feti_stats* stats, double rtol, bool first = true) {
  HostPlan& P = p->P;
  p->dual_target = -1.0;
  hipStream_t st = p->stream;
  const int64_t n = P.n_lam;
  if (first) HIPCHK(hipEventRecord(p->ev[3], st));
  // e = R^T f ; d = B K^+ f - b
  if (p->n_coarse) pcg_coarse_gt_full(P.n_sub, p->d_sub, p->d_rfull, p->d_f, p->d_e, st);
  int iters = 0, status = FETI_OK;
  double rel = 0.0, kappa = 1.0;
  if (n > 0) {
    kpinv_b(p, p->d_f, p->d_yb);
    vec_bvec(p->di, p->d_dvals, p->d_bv, st);
    pcg_scatter(p->di, 0, p->d_yb, p->d_bv, 1.0, p->d_d, nullptr, st);
    vec_axpby(n, -2.0, p->d_bv, 1.0, p->d_d, st);   // (b + B y) - 2 b = B y - b
    // lambda_0 = G Q^{-1} e
    if (p->n_coarse) {
      coarse_solve(p, p->d_e, p->d_calpha, nullptr);
      pcg_coarse_expand(p->di, p->d_sub, p->d_rb, p->d_calpha, p->d_vb, nullptr, st);
      pcg_scatter(p->di, 0, p->d_vb, nullptr, 1.0, p->d_lam, nullptr, st);
    } else {
      vec_fill(n, 0.0, p->d_lam, st);
    }
    // r = d - F lambda ; w = P r ; z = P M w ; s = z
    apply_F(p, p->d_lam, p->d_r, p->d_d, -1.0, nullptr);
    pcg_init_state(p->sc.state, rtol, 0.0, p->opt.max_it, p->sc.hist_cap, st);
    if (first && p->d_lamp && p->have_prev) {
      // warm start from the previous call's multipliers: lambda_0 += c P lambda_prev,
      // which keeps G^T lambda_0 = e, with c minimising the F-norm of the error
      // along that direction: c = (P lambda_prev . r) / (P lambda_prev . F P lambda_prev).
      // The stopping rule keeps the cold start's target: ||P r_k|| <= rtol ||P r_00||.
      project_fused(p, 0, 0, p->d_r, p->d_wv, nullptr, p->sc.state, nullptr);
      project_fused(p, 0, 0, p->d_lamp, p->d_tv, nullptr, p->sc.state, nullptr);
      apply_F(p, p->d_tv, p->d_q, nullptr, 1.0, nullptr);
      double a = 0.0, b = 0.0, w00 = 0.0;
      pcg_dot(n, p->d_tv, p->d_r, p->d_tv, p->d_q, p->sc.dots, nullptr, st);
      HIPCHK(hipMemcpyAsync(p->h_dots, p->sc.dots, 2 * DOT_PARTS * sizeof(double), hipMemcpyDeviceToHost, st));
      HIPCHK(hipStreamSynchronize(st));
      for (int k = 0; k < DOT_PARTS; ++k) {
        a += p->h_dots[2 * k];
        b += p->h_dots[2 * k + 1];
      }
      TRY(dev_norm(p, p->d_wv, n, &w00));
      const double c = b > 0.0 ? a / b : 0.0;
      p->warm_scale = c;
      if (c != 0.0) {
        vec_axpby(n, c, p->d_tv, 1.0, p->d_lam, st);
        vec_axpby(n, -c, p->d_q, 1.0, p->d_r, st);
      }
      pcg_init_state(p->sc.state, 0.0, rtol * w00, p->opt.max_it, p->sc.hist_cap, st);
      p->dual_target = rtol * w00;
    }
    if (p->dual_gmres) {
      TRY(dual_gmres(p, rtol, &iters, &status, &rel));
      p->dual_target = -1.0;
    } else {
      vec_fill(n, 0.0, p->d_s, st);   // s = z + 0 s in the first iteration
      project_fused(p, 0, 0, p->d_r, p->d_wv, nullptr, p->sc.state, nullptr);
      precondition(p, p->d_wv, p->d_tv, p->sc.state);
      project_fused(p, 2, 1, p->d_tv, p->d_zv, p->d_wv, p->sc.state, nullptr);
      // graph of graph_block iterations (feti_solve_noalloc launches the
      // iterations one by one instead: instantiating a graph may allocate)
      const int gb = std::max(1, p->opt.graph_block);
      if (p->use_graph && (!p->graph || p->graph_iters != gb)) {
        if (p->graph) {
          (void)hipGraphExecDestroy(p->graph);
          p->graph = nullptr;
        }
        hipGraph_t gr;
        HIPCHK(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
        for (int k = 0; k < gb; ++k) pcg_iteration(p);
        HIPCHK(hipStreamEndCapture(st, &gr));
        HIPCHK(hipGraphInstantiate(&p->graph, gr, nullptr, nullptr, 0));
        (void)hipGraphDestroy(gr);
        p->graph_iters = gb;
      }
      // Replays are pipelined: the host reads the state copied after one replay
      // while the next already runs, so the GPU does not wait for the host.  A
      // replay queued after convergence costs a block of iterations whose
      // kernels return at once, so no further replay is queued while the one in
      // flight is expected to reach the stopping rule (pcg_converges_within);
      // if it does not, the next replay starts after the host has seen it.
      // The state stops changing once the stopping rule is met.
      PcgState hs{};
      int rd = 0, wr = 0, queued = 0;   // ring of two state copies
      auto queue_state = [&]() -> hipError_t {
        hipError_t e = hipMemcpyAsync(&p->h_state[wr], p->sc.state, sizeof(PcgState), hipMemcpyDeviceToHost, st);
        if (e == hipSuccess) e = hipEventRecord(p->ev_rep[wr], st);
        wr ^= 1;
        ++queued;
        return e;
      };
      auto run_block = [&]() -> hipError_t {
        if (p->use_graph) return hipGraphLaunch(p->graph, st);
        for (int k = 0; k < gb; ++k) pcg_iteration(p);
        return hipGetLastError();
      };
      HIPCHK(queue_state());   // state after the initial residual
      HIPCHK(run_block());
      HIPCHK(queue_state());
      int prev_it = 0;
      double prev_wn = 0.0;
      for (;;) {
        HIPCHK(hipEventSynchronize(p->ev_rep[rd]));
        hs = p->h_state[rd];
        rd ^= 1;
        --queued;
        if (hs.done) break;
        if (queued == 0 || !pcg_converges_within(hs, prev_it, prev_wn, gb * queued)) {
          HIPCHK(run_block());
          HIPCHK(queue_state());
        }
        prev_it = hs.it;
        prev_wn = hs.wn;
      }
      HIPCHK(hipStreamSynchronize(st));
      iters = hs.it;
      status = hs.status;
      rel = hs.w0 > 0 ? hs.wn / hs.w0 : 0.0;
      if (stats && iters > 0) {
        const int m = std::min(iters, std::min(p->sc.hist_cap, p->own.hist_cap));
        HIPCHK(hipMemcpyAsync(p->h_hist, p->sc.hist, 2 * (size_t)m * sizeof(double), hipMemcpyDeviceToHost, st));
        HIPCHK(hipStreamSynchronize(st));
        kappa = lanczos_kappa(p->h_hist, m, p->lz_d, p->lz_e);
      }
    }
    if (first && p->d_lamp) {   // multipliers of this solve, for the next warm start
      vec_axpby(n, 1.0, p->d_lam, 0.0, p->d_lamp, st);
      p->have_prev = true;
    }
    // gamma = -Q^{-1} G^T r ; u = K^+(f - B^T lambda) + R gamma
    pcg_gather(p->di, 0, p->d_lam, p->d_xb, nullptr, st);
    if (P.mixed) kpinv_recover_t<float>(p, p->d_xb, p->d_u);
    else kpinv_recover_t<double>(p, p->d_xb, p->d_u);
    if (p->n_coarse) {
      pcg_gather(p->di, 0, p->d_r, p->d_xb, nullptr, st);
      pcg_coarse_gt(P.n_sub, p->d_sub, p->d_rb, p->d_xb, p->d_cg, nullptr, st);
      coarse_solve(p, p->d_cg, p->d_calpha, nullptr);
      vec_axpby(p->n_coarse, -1.0, p->d_calpha, 0.0, p->d_gamma, st);
      pcg_add_modes(P.NF, p->di.f_sub, p->d_sub, p->d_rfull, p->d_gamma, p->d_u, st);
    }
  } else {
    kpinv(p, p->d_f, p->d_u);
  }
  HIPCHK(hipEventRecord(p->ev[4], st));
  if (stats) {
    stats->kernel_gemv_launches = n > 0 ? iters + 1 : 0;
    stats->kernel_gemv_ms = p->prof_gemv_n ? p->prof_gemv_ms / p->prof_gemv_n : 0.0;
    stats->kernel_update_launches = p->prof_upd_n;
    stats->kernel_update_ms = p->prof_upd_n ? p->prof_upd_ms / p->prof_upd_n : 0.0;
    stats->gemv_bytes = p->gemv_bytes;
    stats->update_flops = p->upd_flops;
    stats->iters = iters;
    stats->converged = status == FETI_OK ? 1 : 0;
    stats->rel_res = rel;
    stats->kappa_est = kappa;
    stats->n_coarse = p->n_coarse;
    stats->n_lambda = n;
    stats->device_bytes = p->bytes;
    stats->autotune_wide = p->n_wide;
    stats->autotune_db = p->n_db;
    stats->modified_pivots = p->modified_pivots;
  }
  if (status == FETI_EBREAKDOWN) {
    p->err = "PCG breakdown (s.Fs <= 0)";
    return FETI_EBREAKDOWN;
  }
  if (status == FETI_ENOCONV) {
    p->err = "PCG reached max_it without convergence";
    return FETI_ENOCONV;
  }
  return FETI_OK;
}

// ||v||_2 of a device vector (deterministic partition, host finish).
feti_status dev_norm(feti_problem* p, const double* v, int64_t n, double* out) {
  pcg_dot(n, v, v, nullptr, nullptr, p->sc.dots, nullptr, p->stream);
  HIPCHK(hipMemcpyAsync(p->h_dots, p->sc.dots, 2 * DOT_PARTS * sizeof(double), hipMemcpyDeviceToHost, p->stream));
  HIPCHK(hipStreamSynchronize(p->stream));
  double s2 = 0.0;
  for (int k = 0; k < DOT_PARTS; ++k) s2 += p->h_dots[2 * k];
  *out = std::sqrt(s2);
  return FETI_OK;
}

// FETI_PROFILE: mean duration of the dual-operator GEMV (tile phase), from
// back-to-back launches on the problem's stream after the solve, on the last
// gathered interface vector (nothing reads the partial sums afterwards).
feti_status profile_gemv(feti_problem* p) {
  constexpr int kBurst = 20;
  if (!p->profile || p->P.n_lam == 0) return FETI_OK;
  const HostPlan::Launch& L = p->P.sched_xtiles;
  HIPCHK(hipEventRecord(p->ev_gemv[0], p->stream));
  for (int r = 0; r < kBurst; ++r) {
    if (p->P.mixed)
      pcg_symv_desc<float>(p->d_gdesc, L.count, (const float*)p->d_X, p->d_xb, p->d_part, p->di.NB, p->di.b_sub,
                           p->d_sub, nullptr, nullptr, p->stream, 1);
    else
      pcg_symv_desc<double>(p->d_gdesc, L.count, (const double*)p->d_X, p->d_xb, p->d_part, p->di.NB,
                            p->di.b_sub, p->d_sub, nullptr, nullptr, p->stream, 1);
  }
  HIPCHK(hipEventRecord(p->ev_gemv[1], p->stream));
  HIPCHK(hipEventSynchronize(p->ev_gemv[1]));
  float ms = 0.f;
  HIPCHK(hipEventElapsedTime(&ms, p->ev_gemv[0], p->ev_gemv[1]));
  p->prof_gemv_ms = ms;
  p->prof_gemv_n = kBurst;
  return FETI_OK;
}

// Classical Gram-Schmidt with one reorthogonalisation of w against the k
// basis vectors V_i = V + i ld (two passes of k dot products, one launch
// each, and w -= sum_i c_i V_i), then ||w||, all on the device with one
// synchronisation at the end: h[i] = the two passes' coefficients summed,
// *nrm = ||w||.  Every sum has a fixed order: deterministic.
feti_status cgs2(feti_problem* p, int64_t n, const double* V, int64_t ld, int k, double* w, double* h, double* nrm) {
  if (k > kGsMax) {   // cannot happen: both restart lengths are below kGsMax
    p->err = "internal: more Gram-Schmidt vectors than the buffers hold";
    return FETI_EINVAL;
  }
  double* part = p->d_gdots;
  double* c = p->d_gdots + (size_t)kGsMax * DOT_PARTS;
  for (int pass = 0; pass < 2; ++pass) {
    vec_multi_dot(n, V, ld, k, w, part, c + pass * kGsMax, p->stream);
    vec_multi_axpy(n, V, ld, k, c + pass * kGsMax, w, p->stream);
  }
  vec_multi_dot(n, w, 0, 1, w, part, c + 2 * kGsMax, p->stream);
  HIPCHK(hipMemcpyAsync(p->h_gdots, c, (2 * kGsMax + 1) * sizeof(double), hipMemcpyDeviceToHost, p->stream));
  HIPCHK(hipStreamSynchronize(p->stream));
  for (int i = 0; i < k; ++i) h[i] = p->h_gdots[i] + p->h_gdots[kGsMax + i];
  *nrm = std::sqrt(std::max(0.0, p->h_gdots[2 * kGsMax]));
  return FETI_OK;
}

// y = A x on the free DOFs of global vectors (Dirichlet DOFs of y are 0),
// with the FP64 sparse local stiffnesses: A = K, or K - tau d f_p / dU with
// the follower pressure's load stiffness (exact Newton step).  f0: local
// loads (y = assembled f0 - A x), or NULL (y = A x).
void apply_assembled(feti_problem* p, const double* x, const double* f0, double* y) {
  const HostPlan& P = p->P;
  hipStream_t st = p->stream;
  local_residual(P.NF, p->d_fpos_lnode, p->d_fpos_comp, p->d_loc_node, p->di.f_sub, p->d_sub, p->d_ell_col,
                 p->d_ell_val, P.ellw, p->d_dmask, x, p->d_ul, f0, p->d_t, st);
  vec_global(P.n_dof, p->d_uc_ptr, p->d_uc_idx, p->d_t, p->d_dmask, p->d_zero, y, 1, st);
  if (!f0) vec_axpby(P.n_dof, -1.0, y, 0.0, y, st);   // -(0 - K x)
  if (p->ls_on) {
    PressureArgs pa;
    pa.n_nodes = P.n_nodes;
    pa.xyz = p->d_xyz;
    pa.U = p->ls_U;
    pa.pface = p->d_pface;
    pa.nfn = P.nfn;
    pa.pf_ptr = p->d_pf_ptr;
    pa.pf_ent = p->d_pf_ent;
    pa.pressure = P.pressure;
    asm_pressure_dir(pa, x, p->d_dmask, p->d_out, st);
    // A x = K x - tau D x;  f0 - A x = (f0 - K x) + tau D x
    vec_axpby(P.n_dof, f0 ? p->ls_tau : -p->ls_tau, p->d_out, 1.0, y, st);
  }
}

// Solve for the local right-hand sides in d_f and the Dirichlet data in
// d_dvals; the global result goes to d_uglob (refined) or stays in d_u.
// One dual solve, unless the FETI solve is only an approximation of the
// assembled FP64 operator A (FP32 local factors; six-mode kernels of stressed
// tangents; or the exact Newton step, whose A includes the follower-load
// stiffness that the symmetric local tangents leave out).  Then the result
// is refined by flexible GMRES on the assembled system A x = b (free DOFs,
// FP64 sparse local stiffnesses), right-preconditioned by the FETI solve:
// each preconditioner application is a dual solve with zero Dirichlet data
// whose load is the Krylov vector split evenly over the subdomain copies of
// each node (a torn load would carry the full interface forces into the
// correction).  Classical Gram-Schmidt with one reorthogonalisation, Givens
// rotations on the host; restarted every kGmresRestart vectors; stops at
// ||b - A x|| <= ir_tol ||b|| or after ir_max preconditioner applications.
feti_status solve_refined(feti_problem* p, feti_stats* stats) {
  HostPlan& P = p->P;
  hipStream_t st = p->stream;
  feti_status s = solve_core(p, stats, p->opt.rtol);
  const bool refine = P.mixed || p->approx_tangent || p->ls_on;
  p->refined_out = false;
  if (refine && p->gm == 0) {   // cannot happen: refinable() covers every case above
    p->err = "internal: refinement buffers were not set up";
    return FETI_EINVAL;
  }
  if (!refine || (s != FETI_OK && s != FETI_ENOCONV)) {
    if ((s == FETI_OK || s == FETI_ENOCONV) && p->profile) {
      TRY(profile_gemv(p));
      // FP64 residual of the result, for comparison with the mixed path
      const int64_t nd = P.n_dof;
      double fnorm = 0.0, rnorm = 0.0;
      vec_global(nd, p->d_uc_ptr, p->d_uc_idx, p->d_u, p->d_dmask, p->d_dvals, p->d_uglob, 0, st);
      local_residual(P.NF, p->d_fpos_lnode, p->d_fpos_comp, p->d_loc_node, p->di.f_sub, p->d_sub, p->d_ell_col,
                     p->d_ell_val, P.ellw, p->d_dmask, p->d_uglob, p->d_ul, p->d_f, p->d_f0, st);
      vec_global(nd, p->d_uc_ptr, p->d_uc_idx, p->d_f0, p->d_dmask, p->d_zero, p->d_out, 1, st);
      TRY(dev_norm(p, p->d_out, nd, &rnorm));
      vec_global(nd, p->d_uc_ptr, p->d_uc_idx, p->d_f, p->d_dmask, p->d_zero, p->d_out, 1, st);
      TRY(dev_norm(p, p->d_out, nd, &fnorm));
      if (stats) {
        stats->kernel_gemv_ms = p->prof_gemv_n ? p->prof_gemv_ms / p->prof_gemv_n : 0.0;
        stats->res_primal = fnorm > 0 ? rnorm / fnorm : 0.0;
      }
    }
    return s;
  }
  int iters = stats ? stats->iters : 0;
  int launches = stats ? stats->kernel_gemv_launches : 0;
  const int64_t nd = P.n_dof;
  const int m = p->gm;
  auto V = [&](int j) { return p->d_gv + (size_t)j * nd; };
  auto Z = [&](int j) { return p->d_gz + (size_t)j * nd; };
  vec_axpby(P.NF, 1.0, p->d_f, 0.0, p->d_f0, st);
  vec_global(nd, p->d_uc_ptr, p->d_uc_idx, p->d_u, p->d_dmask, p->d_dvals, p->d_uglob, 0, st);
  double fnorm = 0.0, beta = 0.0;
  vec_global(nd, p->d_uc_ptr, p->d_uc_idx, p->d_f0, p->d_dmask, p->d_zero, p->d_out, 1, st);
  TRY(dev_norm(p, p->d_out, nd, &fnorm));
  apply_assembled(p, p->d_uglob, p->d_f0, p->d_gw);   // r0 = b - A x0
  TRY(dev_norm(p, p->d_gw, nd, &beta));
  const double target = p->opt.ir_tol * fnorm;
  HIPCHK(hipMemcpyAsync(p->d_dvals, p->d_zero, nd * sizeof(double), hipMemcpyDeviceToDevice, st));
  int sweeps = 0;
  std::vector<double>& H = p->gm_H;   // (m+1) x m, column-major
  std::vector<double>& g = p->gm_g;
  std::vector<double>& cs = p->gm_c;
  std::vector<double>& sn = p->gm_s;
  std::vector<double>& y = p->gm_y;
  std::vector<double>& hv = p->gm_h;
  // dual tolerance of a preconditioner application: the reduction still
  // needed, divided by the observed ratio amp of the primal reduction that a
  // dual reduction eta achieved (learnt after every application, start 10),
  // within [rtol, 1e-2].  On ill-conditioned problems a loose dual solve
  // gives a poor direction, and amp then keeps the inner solves tight.
  double amp = 10.0;
  bool stalled = false;
  while (beta > target && sweeps < p->opt.ir_max) {
    const double beta_start = beta;
    std::fill(H.begin(), H.end(), 0.0);
    std::fill(g.begin(), g.end(), 0.0);
    g[0] = beta;
    vec_axpby(nd, 1.0 / beta, p->d_gw, 0.0, V(0), st);
    double cur = beta;
    int k = 0;   // vectors in this cycle
    for (int j = 0; j < m && sweeps < p->opt.ir_max; ++j) {
      // preconditioner: a dual solve on the load V_j, to a relative dual
      // tolerance that follows the residual still to be removed
      const double eta = std::min(1e-2, std::max(p->opt.rtol, 0.5 * (target / cur) / amp));
      vec_distribute(P.NF, p->d_fpos_lnode, p->d_fpos_comp, p->d_loc_node, p->d_uc_ptr, p->d_dmask, V(j), p->d_f,
                     st);
      feti_stats cst{};
      s = solve_core(p, &cst, eta, false);
      if (s != FETI_OK && s != FETI_ENOCONV) return s;
      iters += cst.iters;
      launches += cst.kernel_gemv_launches;
      ++sweeps;
      vec_global(nd, p->d_uc_ptr, p->d_uc_idx, p->d_u, p->d_dmask, p->d_zero, Z(j), 0, st);
      // w = A z_j, orthogonalised against V_0..V_j (two passes)
      apply_assembled(p, Z(j), nullptr, p->d_gw);
      double hn = 0.0;
      TRY(cgs2(p, nd, V(0), nd, j + 1, p->d_gw, hv.data(), &hn));
      for (int i = 0; i <= j; ++i) H[(size_t)j * (m + 1) + i] = hv[i];
      H[(size_t)j * (m + 1) + j + 1] = hn;
      if (hn > 0.0) vec_axpby(nd, 1.0 / hn, p->d_gw, 0.0, V(j + 1), st);
      // Givens rotations of column j
      double* col = &H[(size_t)j * (m + 1)];
      for (int i = 0; i < j; ++i) {
        const double t = cs[i] * col[i] + sn[i] * col[i + 1];
        col[i + 1] = -sn[i] * col[i] + cs[i] * col[i + 1];
        col[i] = t;
      }
      const double den = std::hypot(col[j], col[j + 1]);
      cs[j] = den > 0 ? col[j] / den : 1.0;
      sn[j] = den > 0 ? col[j + 1] / den : 0.0;
      col[j] = den;
      col[j + 1] = 0.0;
      g[j + 1] = -sn[j] * g[j];
      g[j] = cs[j] * g[j];
      const double prev = cur;
      cur = std::fabs(g[j + 1]);
      if (prev > 0.0) amp = std::max(1.0, (cur / prev) / eta);
      k = j + 1;
      if (cur <= target || hn == 0.0) break;
    }
    // x += Z y with H(0:k, 0:k) y = g(0:k)
    for (int i = k - 1; i >= 0; --i) {
      double acc = g[i];
      for (int l = i + 1; l < k; ++l) acc -= H[(size_t)l * (m + 1) + i] * y[l];
      const double d = H[(size_t)i * (m + 1) + i];
      y[i] = d != 0.0 ? acc / d : 0.0;
    }
    for (int i = 0; i < k; ++i) vec_axpby(nd, y[i], Z(i), 1.0, p->d_uglob, st);
    // true residual of the updated iterate
    apply_assembled(p, p->d_uglob, p->d_f0, p->d_gw);
    TRY(dev_norm(p, p->d_gw, nd, &beta));
    if (!(beta < beta_start)) {
      // the cycle did not reduce the true residual (a preconditioner far
      // from A, whose Krylov basis lost its accuracy): keep the iterate the
      // cycle started from and stop
      for (int i = 0; i < k; ++i) vec_axpby(nd, -y[i], Z(i), 1.0, p->d_uglob, st);
      beta = beta_start;
      stalled = true;
      break;
    }
  }
  p->refined_out = true;
  TRY(profile_gemv(p));
  if (stats) {
    stats->iters = iters;
    stats->ir_sweeps = sweeps;
    stats->kernel_gemv_launches = launches;
    stats->kernel_gemv_ms = p->prof_gemv_n ? p->prof_gemv_ms / p->prof_gemv_n : 0.0;
    stats->res_primal = fnorm > 0 ? beta / fnorm : 0.0;
  }
  if (p->opt.ir_max > 0 && !(beta <= target)) {
    p->err = stalled ? "refinement stalled: a restart cycle did not reduce the residual"
                     : "refinement did not reach ir_tol within ir_max preconditioner applications";
    return FETI_ENOCONV;
  }
  return FETI_OK;
}

feti_status write_output(feti_problem* p, double* out, int sum_mode) {
  HostPlan& P = p->P;
  double* dst = (p->opt.flags & FETI_DEVICE_PTRS) ? out : p->d_out;
  if (p->refined_out)
    HIPCHK(hipMemcpyAsync(dst, p->d_uglob, P.n_dof * sizeof(double), hipMemcpyDeviceToDevice, p->stream));
  else
    vec_global(P.n_dof, p->d_uc_ptr, p->d_uc_idx, p->d_u, p->d_dmask, p->d_dvals, dst, sum_mode, p->stream);
  if (!(p->opt.flags & FETI_DEVICE_PTRS))
    HIPCHK(hipMemcpyAsync(out, p->d_out, P.n_dof * sizeof(double), hipMemcpyDeviceToHost, p->stream));
  HIPCHK(hipStreamSynchronize(p->stream));
  return FETI_OK;
}

float ev_ms(hipEvent_t a, hipEvent_t b) {
  float ms = 0.f;
  if (hipEventElapsedTime(&ms, a, b) != hipSuccess) {
    (void)hipGetLastError();
    return 0.f;
  }
  return ms;
}

feti_status load_U(feti_problem* p, const double* U, const double** U_dev) {
  *U_dev = nullptr;
  if (!U) return FETI_OK;
  if (p->opt.flags & FETI_DEVICE_PTRS) {
    *U_dev = U;
    return FETI_OK;
  }
  for (int64_t k = 0; k < p->P.n_dof; ++k)
    if (!std::isfinite(U[k])) {
      p->err = "non-finite displacement";
      return FETI_EINVAL;
    }
  HIPCHK(hipMemcpyAsync(p->d_U, U, p->P.n_dof * sizeof(double), hipMemcpyHostToDevice, p->stream));
  HIPCHK(hipStreamSynchronize(p->stream));
  *U_dev = p->d_U;
  return FETI_OK;
}

// Body of feti_solve and feti_solve_noalloc (defined after them).
feti_status solve_linear_call(feti_problem* p, double load_factor, double* u, feti_stats* stats);

}  // namespace

// ===========================================================================
extern "C" {

feti_status feti_setup(const feti_mesh* mesh, const feti_options* opts, feti_problem** out) {
  if (!out) {
    g_setup_error = "out is NULL";
    return FETI_EINVAL;
  }
  *out = nullptr;
  std::unique_ptr<feti_problem> p(new feti_problem());
  if (opts) p->opt = *opts;
  else {
    p->opt.variant = FETI_ALL_FLOATING;
    p->opt.precond = FETI_PREC_LUMPED;
    p->opt.precision = FETI_FP64;
  }
  if (p->opt.rtol <= 0) p->opt.rtol = 1e-8;
  if (p->opt.max_it <= 0) p->opt.max_it = 1000;
  if (p->opt.ir_tol <= 0) p->opt.ir_tol = 1e-10;
  if (p->opt.ir_max < 0) p->opt.ir_max = 6;
  if (p->opt.graph_block <= 0) p->opt.graph_block = 8;
  if (!(p->opt.kernel_tol > 0.0)) p->opt.kernel_tol = 1e-12;
  p->opt.graph_block = std::min(p->opt.graph_block, 64);   // also bounds the profiling event slots
  if (p->opt.variant != FETI_CLASSICAL && p->opt.variant != FETI_ALL_FLOATING) {
    g_setup_error = "bad variant";
    return FETI_EINVAL;
  }
  if (p->opt.precision != FETI_FP64 && p->opt.precision != FETI_MIXED) {
    g_setup_error = "bad precision";
    return FETI_EINVAL;
  }
  if ((p->opt.dev_alloc == nullptr) != (p->opt.dev_free == nullptr)) {
    g_setup_error = "dev_alloc and dev_free must be given together";
    return FETI_EINVAL;
  }
  p->da.fn = p->opt.dev_alloc;
  p->da.fr = p->opt.dev_free;
  p->da.ctx = p->opt.alloc_ctx;
  std::string e = build_plan(mesh, &p->opt, p->P);
  if (!e.empty()) {
    g_setup_error = e;
    return FETI_EINVAL;
  }
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || ndev <= 0) {
    (void)hipGetLastError();
    g_setup_error = "no HIP device available";
    return FETI_EDEVICE;
  }
  if (p->opt.hip_stream) {
    p->stream = (hipStream_t)p->opt.hip_stream;
  } else {
    if (hipStreamCreateWithFlags(&p->stream, hipStreamNonBlocking) != hipSuccess) {
      (void)hipGetLastError();
      g_setup_error = "hipStreamCreate failed";
      return FETI_EDEVICE;
    }
    p->own_stream = true;
  }
  feti_status s = setup_device(p.get());
  if (s != FETI_OK) {
    g_setup_error = p->err;
    feti_destroy(p.release());
    return s;
  }
  *out = p.release();
  return FETI_OK;
}

feti_status feti_footprint(const feti_problem* p, size_t* device_bytes) {
  if (!p || !device_bytes) return FETI_EINVAL;
  *device_bytes = p->bytes;
  return FETI_OK;
}

feti_status feti_factor(feti_problem* p, const double* U) {
  if (!p) return FETI_EINVAL;
  p->err.clear();
  const double* Ud = nullptr;
  TRY(load_U(p, U, &Ud));
  p->allow_modified = p->P.mixed;   // feti_solve refines the mixed path
  feti_status s = do_factor(p, Ud);
  p->factored_linear = (s == FETI_OK && U == nullptr);
  return s;
}

feti_status feti_solve(feti_problem* p, double load_factor, double* u, feti_stats* stats) {
  if (!p) return FETI_EINVAL;
  p->err.clear();
  return solve_linear_call(p, load_factor, u, stats);
}

feti_status feti_solve_noalloc(feti_problem* p, double load_factor, double* u, feti_stats* stats) {
  if (!p) return FETI_EINVAL;
  p->err.clear();
  if (!(p->opt.flags & FETI_DEVICE_PTRS)) {
    p->err = "feti_solve_noalloc needs FETI_DEVICE_PTRS (u on the device)";
    return FETI_EINVAL;
  }
  if (p->opt.max_it > kNoAllocMaxIt) {
    p->err = "max_it above " + std::to_string(kNoAllocMaxIt) + ", the iteration history the static scratch holds";
    return FETI_EINVAL;
  }
  if (p->P.n_sub > kMaxSub || !p->noalloc_base) {
    p->err = "static scratch array unavailable on this device";
    return FETI_EDEVICE;
  }
  // the dual iteration's scratch set from the static array; the ticket
  // counters must start at zero (a fill kernel, not a memset node)
  p->sc = noalloc_layout(p->noalloc_base, p->P.n_sub);
  p->sc.hist_cap = std::min(p->sc.hist_cap, p->own.hist_cap);
  vec_fill(2, 0.0, reinterpret_cast<double*>(p->sc.ticket), p->stream);
  p->use_graph = false;
  const feti_status s = solve_linear_call(p, load_factor, u, stats);
  p->sc = p->own;
  p->use_graph = true;
  return s;
}

}  // extern "C"

namespace {

feti_status solve_linear_call(feti_problem* p, double load_factor, double* u, feti_stats* stats) {
  p->ls_on = false;
  if (!u) {
    p->err = "u is NULL";
    return FETI_EINVAL;
  }
  if (!std::isfinite(load_factor)) {
    p->err = "non-finite load factor";
    return FETI_EINVAL;
  }
  if (!p->factored || !p->factored_linear) {
    p->err = "feti_solve needs a preceding feti_factor(p, NULL)";
    return FETI_ESTATE;
  }
  HostPlan& P = p->P;
  hipStream_t st = p->stream;
  HIPCHK(hipEventRecord(p->ev[5], st));
  vec_axpby(P.n_dof, load_factor, p->d_dirval, 0.0, p->d_dvals, st);
  const double* fn = nullptr;
  if (!P.pface.empty() && P.pressure != 0.0) {
    PressureArgs pa;
    pa.n_nodes = P.n_nodes;
    pa.xyz = p->d_xyz;
    pa.U = nullptr;
    pa.pface = p->d_pface;
    pa.nfn = P.nfn;
    pa.pf_ptr = p->d_pf_ptr;
    pa.pf_ent = p->d_pf_ent;
    pa.pressure = P.pressure;
    pa.fnodal = p->d_fnodal;
    asm_pressure(pa, st);
    fn = p->d_fnodal;
  }
  vec_fill(P.NF, 0.0, p->d_f, st);
  RhsArgs r;
  r.n_loc_nodes = P.n_loc_nodes;
  r.diag_slot = p->d_diag_slot;
  r.ps_c0 = p->d_ps_c0;
  r.ps_c1 = p->d_ps_c1;
  r.pc_e = p->d_pc_e;
  r.pc_ab = p->d_pc_ab;
  r.loc_sub = p->d_loc_sub;
  r.loc_pos = p->d_loc_pos;
  r.loc_ncopy = p->d_loc_ncopy;
  r.loc_node = p->d_loc_node;
  r.subs = p->d_sub;
  r.fbody = p->d_fbody;
  r.fint = p->d_fint;
  r.fnodal = fn;
  r.ell_col = p->d_ell_col;
  r.ell_val = p->d_ell_val;
  r.NF = P.NF;
  r.ellw = P.ellw;
  r.npe = P.npe;
  r.dvals = p->d_dvals;
  r.body_scale = load_factor;
  r.int_scale = 0.0;
  r.nodal_scale = load_factor;
  r.f = p->d_f;
  asm_rhs(r, st);
  feti_status s = solve_refined(p, stats);
  if (s != FETI_OK && s != FETI_ENOCONV) return s;
  feti_status s2 = write_output(p, u, 0);
  if (s2 != FETI_OK) return s2;
  if (stats) {
    stats->t_pcg = ev_ms(p->ev[3], p->ev[4]) * 1e-3;
    stats->t_total = ev_ms(p->ev[5], p->ev[4]) * 1e-3;
    stats->t_assemble = ev_ms(p->ev[0], p->ev[1]) * 1e-3;
    stats->t_factor = ev_ms(p->ev[1], p->ev[2]) * 1e-3;
  }
  return s;
}

}  // namespace

extern "C" {

feti_status feti_newton_step(feti_problem* p, const double* U_k, double tau, double* dU, double* res_norm,
                             feti_stats* stats) {
  if (!p) return FETI_EINVAL;
  p->err.clear();
  if (!dU || !std::isfinite(tau)) {
    p->err = "bad arguments";
    return FETI_EINVAL;
  }
  HostPlan& P = p->P;
  hipStream_t st = p->stream;
  const double* Ud = nullptr;
  TRY(load_U(p, U_k, &Ud));
  // a refined Newton step may factor with modified pivots
  p->allow_modified = P.mixed || (P.any_hgo && Ud && ((p->opt.flags & FETI_KERNEL6) || p->opt.kernel_tol > 1e-12)) ||
                      ((p->opt.flags & FETI_LOAD_STIFFNESS) && !P.pface.empty() && P.pressure != 0.0 && tau != 0.0);
  TRY(do_factor(p, Ud));
  p->factored_linear = (U_k == nullptr);
  HIPCHK(hipEventRecord(p->ev[5], st));
  vec_dirinc(P.n_dof, p->d_dmask, p->d_dirval, tau, Ud, p->d_dvals, st);
  const double* fn = nullptr;
  if (!P.pface.empty() && P.pressure != 0.0) {
    PressureArgs pa;
    pa.n_nodes = P.n_nodes;
    pa.xyz = p->d_xyz;
    pa.U = Ud;
    pa.pface = p->d_pface;
    pa.nfn = P.nfn;
    pa.pf_ptr = p->d_pf_ptr;
    pa.pf_ent = p->d_pf_ent;
    pa.pressure = P.pressure;
    pa.fnodal = p->d_fnodal;
    asm_pressure(pa, st);
    fn = p->d_fnodal;
  }
  RhsArgs r;
  r.n_loc_nodes = P.n_loc_nodes;
  r.diag_slot = p->d_diag_slot;
  r.ps_c0 = p->d_ps_c0;
  r.ps_c1 = p->d_ps_c1;
  r.pc_e = p->d_pc_e;
  r.pc_ab = p->d_pc_ab;
  r.loc_sub = p->d_loc_sub;
  r.loc_pos = p->d_loc_pos;
  r.loc_ncopy = p->d_loc_ncopy;
  r.loc_node = p->d_loc_node;
  r.subs = p->d_sub;
  r.fbody = p->d_fbody;
  r.fint = p->d_fint;
  r.fnodal = fn;
  r.ell_col = p->d_ell_col;
  r.ell_val = p->d_ell_val;
  r.NF = P.NF;
  r.ellw = P.ellw;
  r.npe = P.npe;
  r.body_scale = tau;
  r.int_scale = 1.0;
  r.nodal_scale = tau;
  // residual norm tau f_ext - f_int over free DOFs (no Dirichlet lifting)
  if (res_norm) {
    vec_fill(P.n_dof, 0.0, p->d_out, st);
    vec_fill(P.NF, 0.0, p->d_f, st);
    r.dvals = p->d_out;   // zeros: no lifting
    r.f = p->d_f;
    asm_rhs(r, st);
    vec_global(P.n_dof, p->d_uc_ptr, p->d_uc_idx, p->d_f, p->d_dmask, p->d_dvals, p->d_out, 1, st);
    TRY(dev_norm(p, p->d_out, P.n_dof, res_norm));
  }
  vec_fill(P.NF, 0.0, p->d_f, st);
  r.dvals = p->d_dvals;
  r.f = p->d_f;
  asm_rhs(r, st);
  p->ls_on = (p->opt.flags & FETI_LOAD_STIFFNESS) && !P.pface.empty() && P.pressure != 0.0 && tau != 0.0;
  p->ls_U = Ud;
  p->ls_tau = tau;
  feti_status s = solve_refined(p, stats);
  p->ls_on = false;
  if (s != FETI_OK && s != FETI_ENOCONV) return s;
  feti_status s2 = write_output(p, dU, 0);
  if (s2 != FETI_OK) return s2;
  if (stats) {
    stats->t_pcg = ev_ms(p->ev[3], p->ev[4]) * 1e-3;
    stats->t_assemble = ev_ms(p->ev[0], p->ev[1]) * 1e-3;
    stats->t_factor = ev_ms(p->ev[1], p->ev[2]) * 1e-3;
    stats->t_total = stats->t_assemble + stats->t_factor + ev_ms(p->ev[5], p->ev[4]) * 1e-3;
  }
  return s;
}

feti_status feti_set_tolerances(feti_problem* p, double rtol, double ir_tol) {
  if (!p) return FETI_EINVAL;
  p->err.clear();
  if (!(rtol > 0.0 && rtol < 1.0) || !(ir_tol > 0.0 && ir_tol < 1.0)) {
    p->err = "tolerances must lie in (0, 1)";
    return FETI_EINVAL;
  }
  p->opt.rtol = rtol;
  p->opt.ir_tol = ir_tol;
  return FETI_OK;
}

const char* feti_last_error(const feti_problem* p) {
  if (!p) return g_setup_error.c_str();
  return p->err.c_str();
}

void feti_destroy(feti_problem* p) {
  if (!p) return;
  if (p->stream) (void)hipStreamSynchronize(p->stream);
  if (p->graph) (void)hipGraphExecDestroy(p->graph);
  for (auto& ev : p->ev)
    if (ev) (void)hipEventDestroy(ev);
  for (auto& ev : p->ev_gemv)
    if (ev) (void)hipEventDestroy(ev);
  for (auto& ev : p->ev_upd)
    if (ev) (void)hipEventDestroy(ev);
  for (auto& ev : p->ev_tune)
    if (ev) (void)hipEventDestroy(ev);
  for (void* a : p->allocs) {
    if (p->da.fr) p->da.fr(a, p->da.ctx);
    else (void)hipFree(a);
  }
  for (auto& ev : p->ev_rep)
    if (ev) (void)hipEventDestroy(ev);
  if (p->h_state) (void)hipHostFree(p->h_state);
  if (p->h_hist) (void)hipHostFree(p->h_hist);
  if (p->h_dots) (void)hipHostFree(p->h_dots);
  if (p->h_gdots) (void)hipHostFree(p->h_gdots);
  if (p->stream_c) {
    (void)hipStreamSynchronize(p->stream_c);
    (void)hipStreamDestroy(p->stream_c);
  }
  if (p->ev_cfork) (void)hipEventDestroy(p->ev_cfork);
  if (p->ev_cjoin) (void)hipEventDestroy(p->ev_cjoin);
  if (p->ev_asm) (void)hipEventDestroy(p->ev_asm);
  if (p->ev_modes) (void)hipEventDestroy(p->ev_modes);
  if (p->ev_ffork) (void)hipEventDestroy(p->ev_ffork);
  if (p->ev_fjoin) (void)hipEventDestroy(p->ev_fjoin);
  if (p->h_nmodes) (void)hipHostFree(p->h_nmodes);
  if (p->h_sub) (void)hipHostFree(p->h_sub);
  if (p->own_stream && p->stream) (void)hipStreamDestroy(p->stream);
  delete p;
}

}  // extern "C"
