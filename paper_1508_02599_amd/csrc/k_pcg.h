// Device-side PCG state and launchers of the dual-iteration and assembly kernels.
#pragma once

#include <vector>

#include "feti_impl.h"

namespace feti {

constexpr int DOT_PARTS = 256;   // fixed partition of every dot product
constexpr int FUSE_BLOCKS = 2048;   // most row blocks of a fused per-multiplier kernel

// Scalars of the projected PCG, resident on the device so that iterations can
// be captured in a HIP graph and run without host synchronisation.
struct PcgState {
  double rho, alpha, beta, w0, wn, pq, rtol, atol;
  int32_t it, max_it, done, status, hist_cap, pad_;
};

// Scratch of the dual iteration: the device-resident CG state, the ticket
// counters of the last-block reductions (must start at zero), block partial
// sums of the dot products and of the coarse right-hand sides, and the
// (alpha, beta) history of the condition estimate (hist_cap iterations).
struct PcgScratch {
  PcgState* state = nullptr;
  int* ticket = nullptr;       // 4 counters
  double* fpart = nullptr;     // 2 * FUSE_BLOCKS
  double* apart = nullptr;     // FUSE_BLOCKS
  double* dots = nullptr;      // 2 * DOT_PARTS
  double* gpart = nullptr;     // 4 * 6 * n_sub
  double* hist = nullptr;      // 2 * hist_cap
  int hist_cap = 0;
};

// Static scratch array of feti_solve_noalloc: its size, the largest
// iteration history it holds, and its device address on `device` (looked up
// once per device with hipGetSymbolAddress; NULL on failure).
constexpr size_t kNoAllocScratchBytes = 512 * 1024;
constexpr int kNoAllocMaxIt = 8192;
void* noalloc_scratch(int device);
// Carves the scratch set out of the static array (base from noalloc_scratch).
PcgScratch noalloc_layout(void* base, int n_sub);

// Device index arrays used by the dual-space kernels.
struct DevIdx {
  int64_t NB = 0, NF = 0, n_lam = 0;
  const int32_t *g_ptr = nullptr, *g_row = nullptr, *b_sub = nullptr, *f_sub = nullptr;
  const double *g_coef = nullptr, *r_w = nullptr, *r_c0 = nullptr, *r_c1 = nullptr;
  const int64_t *r_b0 = nullptr, *r_b1 = nullptr, *r_gdof = nullptr, *b2full = nullptr;
  const int32_t *c_ptr = nullptr, *c_col = nullptr;   // copy coupling B^T B (CSR over b)
  const double *c_v0 = nullptr, *c_v1 = nullptr;      // B^T B, B^T diag(w) B
};

// --- dense factor kernels (k_dense.hip)
// form (update kinds): 0 64x64 tiles, 1 the wide task list (128x64), 2 double-buffered 64x64;
// ndiag: leading diagonal tasks of an update launch
template <typename T>
void launch_dense(int kind, const Task* tasks, int count, const SubInfo* subs, T* arena, T* linv, T* W, T* X,
                  int* err, hipStream_t st, int split = 0, int form = 0, int ndiag = 0);
template <typename T>
void launch_init_arena(const Task* tasks, int count, const SubInfo* subs, T* arena, hipStream_t st);
template <typename T>
void launch_copy_iface(const Task* tasks, int count, const SubInfo* subs, const T* arena, T* S, hipStream_t st);
template <typename T>
void launch_rho(int n_sub, const SubInfo* subs, const T* arena, double* rho, hipStream_t st);
template <typename T>
void launch_regularise(const Task* tasks, int count, const SubInfo* subs, const double* rb, const double* rho,
                       T* arena, hipStream_t st);

template <typename T>
void launch_woodbury(int n_sub, int max_nt_b, const Task* xtasks, int xcount, const SubInfo* subs, T* X,
                     const double* rb, const double* rho, double* Y, double* M, hipStream_t st);

// --- dual iteration kernels (k_pcg.hip)
void pcg_gather(const DevIdx& d, int weighted, const double* v, double* xb, const PcgState* st, hipStream_t s);
void pcg_scatter(const DevIdx& d, int weighted, const double* y, const double* base, double sgn, double* out,
                 const PcgState* st, hipStream_t s);
// Packed symmetric GEMV over the interface tiles of every subdomain: tile
// partial sums into part, then their ordered sum into yb (yb NULL: the tile
// phase only).
template <typename T>
void pcg_symv(const Task* tasks, int count, const SubInfo* subs, const T* M, const double* xb, double* part,
              int64_t NB, const int32_t* b_sub, double* yb, const PcgState* st, hipStream_t s, int iface_only);
// The same product over precomputed tile descriptors (gemv_descriptors), one
// vector load per tile instead of two dependent scalar loads, and 16-byte
// tile loads: the interface tiles of the dual operator and of the Dirichlet
// preconditioner.
void gemv_descriptors(const Task* tasks, int count, const SubInfo* subs, std::vector<int64_t>& out);
template <typename T>
void pcg_symv_desc(const int64_t* desc, int count, const T* M, const double* xb, double* part, int64_t NB,
                   const int32_t* b_sub, const SubInfo* subs, double* yb, const PcgState* st, hipStream_t s,
                   int iface_only);
void pcg_dot(int64_t n, const double* a, const double* b, const double* c, const double* d, double* part,
             const PcgState* st, hipStream_t s);
void pcg_coarse_gt(int n_sub, const SubInfo* subs, const double* rb, const double* xb, double* g,
                   const PcgState* st, hipStream_t s);
void pcg_coarse_gt_full(int n_sub, const SubInfo* subs, const double* rf, const double* xf, double* g,
                        hipStream_t s);
void pcg_coarse_expand(const DevIdx& d, const SubInfo* subs, const double* rb, const double* alpha, double* vb,
                       const PcgState* st, hipStream_t s);
void pcg_add_modes(int64_t NF, const int32_t* f_sub, const SubInfo* subs, const double* rf, const double* gamma,
                   double* u, hipStream_t s);
void pcg_lumped(const DevIdx& d, int w_bb, const int32_t* bb_col, const double* bb_val, const double* xb,
                double* yb, const PcgState* st, hipStream_t s);
void lumped_fill(const DevIdx& d, int w_bb, const int32_t* bb_slot, const double* ell_val, double* bb_val,
                 hipStream_t s);
void vec_bvec(const DevIdx& d, const double* dvals, double* out, hipStream_t s);
void vec_global(int64_t n_dof, const int32_t* uc_ptr, const int64_t* uc_idx, const double* ufull,
                const uint8_t* dmask, const double* dvals, double* out, int sum_mode, hipStream_t s);
void vec_dirinc(int64_t n_dof, const uint8_t* dmask, const double* dirval, double tau, const double* U,
                double* dvals, hipStream_t s);
void vec_axpby(int64_t n, double a, const double* x, double b, double* y, hipStream_t s);
// out[i] = V_i . w for the k vectors V_i = V + i ld, from the fixed partition
// of every dot product (part: k * DOT_PARTS partial sums of scratch), summed
// on the device in a fixed order; and y -= sum_i h_i V_i with the k
// coefficients h on the device.
void vec_multi_dot(int64_t n, const double* V, int64_t ld, int k, const double* w, double* part, double* out,
                   hipStream_t s);
void vec_multi_axpy(int64_t n, const double* V, int64_t ld, int k, const double* h, double* y, hipStream_t s);
void vec_fill(int64_t n, double v, double* y, hipStream_t s);
void pcg_init_state(PcgState* st, double rtol, double atol, int max_it, int hist_cap, hipStream_t s);
template <typename T>
void local_kp_tiles(int mode, int n_sub, int max_rows, const SubInfo* subs, const int32_t* env, const T* arena,
                    const double* x, const double* xb, const double* base, double* y, double* yb, hipStream_t s);
// Interior solves y = L_II^{-1} x (mode 0) or L_II^{-T} x (mode 3), tile by tile inside the envelope.
template <typename T>
void local_kp_band(int mode, int n_sub, int max_nt_i, const SubInfo* subs, const int32_t* env, const T* arena,
                   const T* linv, const double* x, double* y, hipStream_t s);
void vec_set_b2f(const DevIdx& d, const double* b, double* full, hipStream_t s);
// fused iteration kernels
void pcg_gather_s(const DevIdx& d, const double* z, const double* sv, double* xb, const PcgState* st,
                  hipStream_t s);
// Fused scatters that also form the coarse right-hand side of the next
// projection from the interface vector (coarse = 0: no coarse space).
void pcg_scatter_dot_alpha_gt(const DevIdx& d, int n_sub, int coarse, const SubInfo* subs, const double* rbv,
                              const double* yb, const double* z, double* sv, double* q, double* part,
                              PcgState* st, double* gpart, int ldg, hipStream_t s);
void pcg_scatter_w_gt(const DevIdx& d, int n_sub, int coarse, const SubInfo* subs, const double* rbv,
                      const double* y, double* out, const PcgState* st, double* gpart, int ldg, hipStream_t s);
void pcg_proj_gt(int n_sub, const SubInfo* subs, const DevIdx& d, const double* rbv, const double* x,
                 const double* q, int with_update, double* gpart, int ldg, const PcgState* st, hipStream_t s);
void pcg_coarse_dense(int nc, int ld, const double* Qi, const double* gpart, int ldg, double* a, const PcgState* st,
                      hipStream_t s);
void pcg_proj_apply(int mode, int init, const DevIdx& d, int coarse, const int2* rco, const double* rbv,
                    const double* ac, double* x, const double* q, const double* sv, double* lam, double* out,
                    const double* w, double* part, int* ticket, PcgState* st, double* hist, hipStream_t s,
                    const double* apart = nullptr);
void fill_bco(const DevIdx& d, const SubInfo* subs, int32_t* bco, int2* rco, hipStream_t s);
void coarse_to_dense(int nc, int ld, const double* tiles, double* D, hipStream_t s);
void local_residual(int64_t NF, const int32_t* fpos_lnode, const int8_t* fpos_comp, const int64_t* loc_node,
                    const int32_t* f_sub, const SubInfo* subs, const int32_t* ell_col, const double* ell_val,
                    int ellw, const uint8_t* dmask, const double* uglob, double* ul, const double* f, double* r,
                    hipStream_t s);
void vec_distribute(int64_t NF, const int32_t* fpos_lnode, const int8_t* fpos_comp, const int64_t* loc_node,
                    const int32_t* uc_ptr, const uint8_t* dmask, const double* rg, double* r, hipStream_t s);

// --- assembly kernels (k_assemble.hip)
struct AsmArgs {
  int64_t n_elems = 0;
  const double* xyz = nullptr;        // [n_nodes*3]
  int npe = 8;                        // nodes per element: 8 (Q1) or 27 (Q2)
  const int64_t* hex8 = nullptr;      // [n_elems*npe]
  const int32_t* elem_mat = nullptr;
  const double* mat = nullptr;        // [n_mat*7] kind,E,nu,c,k1,k2,kappa
  const double* fibers = nullptr;     // [n_elems*6] or null
  const double* body = nullptr;       // [n_elems*3] or null
  const double* U = nullptr;          // [n_nodes*3] or null
  double* Ke = nullptr;               // [n_elems*(3 npe)^2]  layout [a][b][i][j]
  double* fint = nullptr;             // [n_elems*3 npe]
  double* fbody = nullptr;            // [n_elems*3 npe]
  int* inverted = nullptr;            // smallest element with det F <= 0 at U (atomicMin), or NULL
};
void asm_elements(const AsmArgs& a, int any_hgo, hipStream_t s);

struct GatherArgs {
  int64_t n_slots = 0;
  const int32_t *ps_a = nullptr, *ps_b = nullptr, *ps_nbr = nullptr, *ps_c0 = nullptr, *ps_c1 = nullptr;
  const int32_t *pc_e = nullptr, *pc_ab = nullptr;
  const int32_t* loc_sub = nullptr;   // [n_loc_nodes] owning subdomain
  const int32_t* loc_pos = nullptr;   // [3*n_loc_nodes]
  const SubInfo* subs = nullptr;
  const double* Ke = nullptr;
  int npe = 8;                        // nodes per element of Ke
  double* ell_val = nullptr;          // [ellw][NF] slot-major
  int64_t NF = 0;
};
template <typename T>
void asm_gather(const GatherArgs& g, T* arena, hipStream_t s);

struct RhsArgs {
  int64_t n_loc_nodes = 0;
  const int32_t *diag_slot = nullptr, *ps_c0 = nullptr, *ps_c1 = nullptr, *pc_e = nullptr, *pc_ab = nullptr;
  const int32_t *loc_sub = nullptr, *loc_pos = nullptr, *loc_ncopy = nullptr;
  const int64_t* loc_node = nullptr;
  const SubInfo* subs = nullptr;
  const double *fbody = nullptr, *fint = nullptr, *fnodal = nullptr;   // fnodal [n_dof] or null
  const int32_t* ell_col = nullptr;   // [ellw][NF] slot-major
  const double* ell_val = nullptr;
  int64_t NF = 0;
  int ellw = ELLW_Q1;
  int npe = 8;                        // nodes per element of fbody / fint
  const double* dvals = nullptr;      // [n_dof] prescribed values / increments
  double body_scale = 1.0, int_scale = 0.0, nodal_scale = 0.0;
  double* f = nullptr;                // [NF]
};
void asm_rhs(const RhsArgs& r, hipStream_t s);

struct PressureArgs {
  int64_t n_nodes = 0;
  const double *xyz = nullptr, *U = nullptr;
  const int64_t* pface = nullptr;
  const int32_t *pf_ptr = nullptr, *pf_ent = nullptr;
  int nfn = 4;                        // nodes per face: 4 (bilinear) or 9 (biquadratic)
  double pressure = 0.0;
  double* fnodal = nullptr;           // [n_dof]
};
void asm_pressure(const PressureArgs& p, hipStream_t s);
// out = (d f_p / d x) z: the follower pressure's load stiffness applied to z
// (global node-major vectors; Dirichlet DOFs of out are 0).
void asm_pressure_dir(const PressureArgs& p, const double* z, const uint8_t* dmask, double* out, hipStream_t s);

constexpr int MODES_CH = 16;   // workgroups per subdomain of the rotation test's sweep
struct ModesArgs {
  int n_sub = 0;
  const SubInfo* subs = nullptr;
  const int64_t* loc_node = nullptr;
  const int32_t* loc_pos = nullptr;
  const int32_t* fpos_lnode = nullptr; // [NF] local-node index (incl. node_off) of a full position, -1 pad
  const int8_t* fpos_comp = nullptr;   // [NF]
  const double *xyz = nullptr, *U = nullptr;
  const int32_t* ell_col = nullptr;   // [ellw][NF] slot-major
  const double* ell_val = nullptr;
  int64_t NF = 0;
  int ellw = ELLW_Q1;
  const uint8_t* dmask = nullptr;      // [n_dof] Dirichlet DOFs (partially constrained subdomains)
  int test_rotations = 0;              // keep a rotation only if K annihilates it
  double kernel_tol = 1e-12;
  double* rfull = nullptr;             // [NF*6]
  double* rb = nullptr;                // [NB*6]
  int32_t* n_modes = nullptr;          // [n_sub] (output)
  double* work = nullptr;              // [NF*6] scratch
  double* part = nullptr;              // [n_sub*MODES_CH*13] partial sums of the rotation test
};
void asm_modes(const ModesArgs& m, hipStream_t s);

struct CoarseArgs {
  int n_pairs = 0;
  const int32_t *qp_s = nullptr, *qp_t = nullptr, *qp_ptr = nullptr;
  const int64_t *qe_bs = nullptr, *qe_bt = nullptr;
  const double* qe_c = nullptr;
  const SubInfo* subs = nullptr;
  const double* rb = nullptr;
  double* q = nullptr;                 // lower tiles of the coarse matrix
};
void asm_coarse(const CoarseArgs& c, hipStream_t s);

}  // namespace feti
