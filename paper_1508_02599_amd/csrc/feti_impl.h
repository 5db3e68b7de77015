// Internal declarations of libfeti: host plan (decomposition and index maps),
// device-side problem state, and the launchers of the HIP kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/feti.h"

namespace feti {

// Edge of the square tiles that every dense local matrix is stored in.
constexpr int TS = 64;
constexpr int TS2 = TS * TS;
// Width of the ELL rows of the sparse local stiffnesses: at most 27 neighbour
// nodes of a Q1 node, 125 of a Q2 node (a Q2 corner node), x 3 DOFs; the Q2
// width is rounded up to a multiple of 9 slots (whole slot groups).
constexpr int ELLW_Q1 = 81;
constexpr int ELLW_Q2 = 378;
// Maximum number of subdomains: the coarse vector (6 entries per subdomain)
// of one projection fits in 64 KiB of LDS.
constexpr int kMaxSub = 1365;

// Per-subdomain layout, copied to the device as a plain struct array.
// A subdomain's local DOFs are ordered interior first, constraint ("b") DOFs
// last; each class is padded to a multiple of TS with decoupled identity rows.
// Dense blocks are stored as lower-triangular arrays of column-major TSxTS tiles;
// tile (i, j), i >= j, sits at tile index i*(i+1)/2 + j.
struct SubInfo {
  int32_t n_nodes;      // local nodes
  int32_t n_ii, n_b;    // interior / constraint DOFs (without padding)
  int32_t nt_i, nt_b, nt;
  int32_t node_off;     // offset into local-node arrays
  int32_t floating;     // 0: no rigid-body kernel; 1: floating (all six rigid modes regularise,
                        // the inverse is corrected for those outside the kernel); 2: classical
                        // subdomain touching the Dirichlet boundary (kernel: the rigid modes that
                        // vanish on its Dirichlet DOFs, found on the device; only they regularise)
  int32_t n_modes;      // kernel dimension used (0..6)
  int32_t coarse_off;   // first coarse index of this subdomain
  int32_t n_if;         // interface DOFs (with multipliers): the first n_if of the trailing block
  int32_t env_off;      // offset of its tile envelope (first nonzero tile column of each tile row)
  int64_t tile_off;     // element offset into the factor arena
  int64_t linv_off;     // element offset into the diagonal-inverse arena
  int64_t x_off;        // element offset into the interface arenas (X, W, S)
  int64_t full_off;     // offset of the local vector in full-space vectors
  int64_t b_off;        // offset of the interface part in b-space vectors
  int64_t part_off;     // offset into interface GEMV partial sums
};

// One work item of a batched tile kernel.
struct Task {
  int32_t sub, i, j, k0, k1;
  int32_t n = 1;   // wide tile updates: output tiles (i, j) .. (i + n - 1, j)
};

struct HostPlan {
  // ---- problem copy
  int64_t n_nodes = 0, n_elems = 0, n_dof = 0;
  int32_t n_sub = 0;
  bool af = true;
  int precond = 1;
  bool mixed = false;
  bool any_hgo = false;
  std::vector<double> xyz;
  int npe = 8;                          // nodes per element: 8 (Q1) or 27 (Q2)
  int nfn = 4;                          // nodes per pressure face: 4 (Q1) or 9 (Q2)
  int ellw = ELLW_Q1;                   // ELL row width (ELLW_Q1 or ELLW_Q2)
  std::vector<int64_t> hex8;            // [n_elems][npe] element nodes
  std::vector<int32_t> elem_sub, elem_mat;
  std::vector<feti_material> mat;
  std::vector<double> fibers, body_force;
  std::vector<int64_t> pface;           // [n_pfaces][nfn]
  double pressure = 0.0;
  std::vector<uint8_t> dir_mask;        // [n_dof]
  std::vector<double> dir_val;          // [n_dof]
  std::vector<int64_t> dir_list;        // Dirichlet dofs, ascending

  // ---- subdomains
  std::vector<SubInfo> sub;
  std::vector<int32_t> env;             // tile envelopes of the local matrices, sub[s].env_off onwards
  int64_t n_loc_nodes = 0;              // total local nodes
  std::vector<int64_t> loc_node;        // [n_loc_nodes] global node
  std::vector<int32_t> loc_pos;         // [3*n_loc_nodes] position in local full space, -1 eliminated
  std::vector<int32_t> loc_ncopy;       // [n_loc_nodes] number of subdomain copies of the node
  std::vector<int32_t> loc_sub;         // [n_loc_nodes] owning subdomain
  std::vector<int32_t> fpos_lnode;      // [NF] local node of a full-space position (-1 padding)
  std::vector<int8_t> fpos_comp;        // [NF] component of a full-space position
  std::vector<int32_t> f_sub;           // [NF] subdomain of a full-space position
  int64_t NF = 0, NB = 0;               // full-space and b-space lengths
  int64_t n_tiles = 0, n_xtiles = 0, n_linv = 0, n_part = 0;

  // ---- assembly gather (node pairs inside a subdomain)
  std::vector<int32_t> ps_a, ps_b, ps_nbr, ps_c0, ps_c1;   // per pair slot (a,b: local-node index incl. node_off)
  std::vector<int32_t> pc_e;            // contribution element
  std::vector<int32_t> pc_ab;           // la | lb << 8
  std::vector<int32_t> diag_slot;       // [n_loc_nodes] slot of (a, a)
  std::vector<int32_t> ell_col;         // [ellw][NF] slot-major: >=0 local pos, -1 empty, <=-2 Dirichlet dof -(g+2);
                                        // the filled slots of every row form a prefix (kernels stop at the first -1)
  int32_t w_bb = 0;                     // width of the interface-interface block K_bb in slots
  std::vector<int32_t> bb_slot;         // [w_bb][NB] ELL slot of each K_bb entry (-1 none)
  std::vector<int32_t> bb_col;          // [w_bb][NB] b-space column

  // ---- multipliers
  int64_t n_lam = 0;
  std::vector<int64_t> r_b0, r_b1;      // b-space index of the two entries (-1 if none)
  std::vector<double> r_c0, r_c1, r_w;  // coefficients and weight of the row in B_D
  std::vector<int64_t> r_gdof;          // Dirichlet dof of an AF Dirichlet row, else -1
  std::vector<int32_t> g_ptr;           // [NB+1] multiplier rows touching each b entry
  std::vector<int32_t> g_row;
  std::vector<double> g_coef;
  std::vector<int32_t> c_ptr, c_col;    // copy coupling B^T B in CSR over b-space
  std::vector<double> c_v0, c_v1;       // values of B^T B and of B^T diag(w) B
  std::vector<int64_t> b2full;          // [NB]
  std::vector<int32_t> b_sub;           // [NB]

  // ---- recovery of global displacements
  std::vector<int32_t> uc_ptr;          // [n_dof+1]
  std::vector<int64_t> uc_idx;          // full-space index of each copy

  // ---- pressure faces: per global node, (face*nfn + face node) list
  std::vector<int32_t> pf_ptr, pf_ent;

  // ---- coarse problem: neighbour pairs (s >= t) and their shared rows
  std::vector<int32_t> qp_s, qp_t, qp_ptr;       // per pair, entries [qp_ptr[k], qp_ptr[k+1])
  std::vector<int64_t> qe_bs, qe_bt;
  std::vector<double> qe_c;                       // c_s * c_t

  // ---- factor schedule (task lists, launched in order on one stream)
  // split: for a fused update + inverse-row launch, the number of tasks before
  // the inverse rows.  ndiag: the leading diagonal tasks of an update launch
  // (last update term, factorisation and inverse of the column's diagonal
  // tiles).  wfirst/wcount/wsplit: the same launch with the tile updates
  // paired into 128x64 outputs (wcount = 0: no such form).
  struct Launch {
    int kind;
    int32_t first, count;
    int32_t split = 0;                      // update kinds: tasks before the rows of an inverse
    int32_t wfirst = 0, wcount = 0, wsplit = 0;   // the same launch in the wide form
    int32_t ndiag = 0;                      // update kinds: leading diagonal tasks
  };
  std::vector<Task> tasks;
  std::vector<Launch> sched_interior;   // stage 1
  Launch sched_schur{0, 0, 0};          // stage 2
  std::vector<Launch> sched_iface;      // stage 4
  std::vector<Launch> sched_trtri;      // stage 5
  Launch sched_lauum{0, 0, 0};          // stage 6
  Launch sched_xtiles{0, 0, 0};         // all interface lower tiles (sub, I, J)
  Launch sched_alltiles{0, 0, 0};       // factor tiles that are read (sub, i, j): inside the envelope, and the interface block
  int max_nt_i = 0, max_nt_b = 0;
};

enum LaunchKind { K_UPDATE = 0, K_DIAG = 1, K_TRSM = 2, K_TRTRI = 3, K_LAUUM = 4,
                  K_UPD_TRTRI = 5 };   // update tasks, then rows of the interface inverse
inline bool is_update_kind(int kind) { return kind == K_UPDATE || kind == K_UPD_TRTRI; }

// Builds the plan; returns an empty string on success, else an error message.
std::string build_plan(const feti_mesh* m, const feti_options* o, HostPlan& P);

// Appends the factor schedule of a batch of matrices described by `subs`
// (interior/interface tile counts) into P-like containers.
// env (optional): env[s][I] = first tile column holding a nonzero of matrix s
// in tile row I.  A Cholesky factor has no nonzero left of the first nonzero
// of its row in the matrix, so factor tiles left of env stay zero: the
// interior and Schur steps skip them and every product with them.
void build_factor_schedule(const std::vector<SubInfo>& subs, std::vector<Task>& tasks,
                           std::vector<HostPlan::Launch>& interior, HostPlan::Launch& schur,
                           std::vector<HostPlan::Launch>& iface, std::vector<HostPlan::Launch>& trtri,
                           HostPlan::Launch& lauum, HostPlan::Launch& xtiles,
                           HostPlan::Launch& alltiles,
                           const std::vector<std::vector<int32_t>>* env = nullptr);

}  // namespace feti
