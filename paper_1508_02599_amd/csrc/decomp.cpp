// Host side of feti_setup: validation, tearing of the mesh into subdomains,
// multiplier rows, their weights, interior-first DOF ordering, index
// maps for the device kernels and the tile schedule of the batched factor.
//
// Paper references: non-overlapping decomposition and reordering into interior
// and coupling DOFs (section 4, eqs. (decomposition), (skeleton), (reordered));
// jump operators B_i with entries in {0, +1, -1} (section 4.1), "fully
// redundant" gluing (Fig. 3); all-floating Dirichlet rows B_D,i with right-hand
// side b (section 4.2, eq. (jumpoperatorAF)); scaled rows B_D for the
// preconditioner (eq. (feti_preconditioner)).
#include <algorithm>
#include <array>
#include <functional>
#include <cmath>
#include <numeric>

#include "feti_impl.h"

namespace feti {

static int32_t ceil_tiles(int64_t n) { return (int32_t)((n + TS - 1) / TS); }

void build_factor_schedule(const std::vector<SubInfo>& subs, std::vector<Task>& tasks,
                           std::vector<HostPlan::Launch>& interior, HostPlan::Launch& schur,
                           std::vector<HostPlan::Launch>& iface, std::vector<HostPlan::Launch>& trtri,
                           HostPlan::Launch& lauum, HostPlan::Launch& xtiles, HostPlan::Launch& alltiles,
                           const std::vector<std::vector<int32_t>>* env) {
  const int ns = (int)subs.size();
  // first possibly nonzero factor tile column of tile row I (0: dense)
  auto E = [&](int s, int I) -> int { return env ? (*env)[s][I] : 0; };
  int max_i = 0, max_b = 0;
  for (const auto& s : subs) {
    max_i = std::max(max_i, s.nt_i);
    max_b = std::max(max_b, s.nt_b);
  }
  auto begin = [&](int kind) { return HostPlan::Launch{kind, (int32_t)tasks.size(), 0}; };
  auto finish = [&](HostPlan::Launch& L) { L.count = (int32_t)tasks.size() - L.first; };
  // block row ib of the inverse of the interface factor, for the subdomains
  // that have it: tasks (ib, jb), jb <= ib (the interface block is dense)
  auto inverse_row = [&](int ib) {
    for (int s = 0; s < ns; ++s)
      if (subs[s].nt_b > ib)
        for (int jb = 0; jb <= ib; ++jb) tasks.push_back({s, ib, jb, jb, ib});
  };
  // the wide form of an update launch: consecutive tasks of one subdomain and
  // column with adjacent rows become one two-tile task; the diagonal tasks
  // before them and the inverse-row tasks after them are kept unchanged
  auto widen = [&](HostPlan::Launch& L) {
    const int32_t nupd = L.kind == K_UPDATE ? L.count : L.split;
    std::vector<Task> w;
    for (int32_t k = 0; k < L.ndiag; ++k) w.push_back(tasks[L.first + k]);
    for (int32_t k = L.ndiag; k < nupd;) {
      Task a = tasks[L.first + k];
      if (k + 1 < nupd) {
        const Task& b = tasks[L.first + k + 1];
        if (b.sub == a.sub && b.j == a.j && b.k0 == a.k0 && b.k1 == a.k1 && b.i == a.i + 1) {
          a.n = 2;
          w.push_back(a);
          k += 2;
          continue;
        }
      }
      w.push_back(a);
      ++k;
    }
    const int32_t nw = (int32_t)w.size();
    for (int32_t k = nupd; k < L.count; ++k) w.push_back(tasks[L.first + k]);
    L.wfirst = (int32_t)tasks.size();
    L.wcount = (int32_t)w.size();
    L.wsplit = nw;
    tasks.insert(tasks.end(), w.begin(), w.end());
  };
  // update launch of a column step, with the previous block row of the
  // inverse appended (its inputs are final once that column step is done)
  auto fused = [&](HostPlan::Launch& L, int kind_fused, int row) {
    const int32_t nupd = (int32_t)tasks.size() - L.first;
    inverse_row(row);
    finish(L);
    if (L.count > nupd) {
      L.kind = kind_fused;
      L.split = nupd;
    }
    widen(L);
  };
  auto plain = [&](HostPlan::Launch& L) {
    finish(L);
    widen(L);
  };
  // stage 1: interior columns, left-looking (rows run over every tile row
  // below that is not left of its envelope).  Column step j > 0 is one update
  // launch and the panel solve.  The launch's first tasks take the diagonal
  // tiles: the last update term (k = j - 1, unless left of the envelope),
  // factorisation and inverse; the others update the tiles below (and
  // subtract the terms k < j of diagonal tile j + 1, so that the diagonal
  // tasks of the next step carry one term at most).  Update terms run from
  // the later envelope of the two tile rows; tasks left with none are dropped.
  for (int j = 0; j < max_i; ++j) {
    if (j == 0) {
      auto D = begin(K_DIAG);
      for (int s = 0; s < ns; ++s)
        if (subs[s].nt_i > 0) tasks.push_back({s, 0, 0, 0, 0});
      finish(D);
      interior.push_back(D);
    } else {
      auto L = begin(K_UPDATE);
      for (int s = 0; s < ns; ++s)
        if (subs[s].nt_i > j) tasks.push_back({s, j, j, std::max(j - 1, E(s, j)), j});
      L.ndiag = (int32_t)tasks.size() - L.first;
      for (int s = 0; s < ns; ++s)
        if (subs[s].nt_i > j) {
          for (int i = j + 1; i < subs[s].nt; ++i) {
            const int k0 = std::max(E(s, i), E(s, j));
            if (E(s, i) <= j && k0 < j) tasks.push_back({s, i, j, k0, j});
          }
          if (subs[s].nt_i > j + 1 && E(s, j + 1) < j) tasks.push_back({s, j + 1, j + 1, E(s, j + 1), j});
        }
      plain(L);
      interior.push_back(L);
    }
    auto T = begin(K_TRSM);
    for (int s = 0; s < ns; ++s)
      if (subs[s].nt_i > j)
        for (int i = j + 1; i < subs[s].nt; ++i)
          if (E(s, i) <= j) tasks.push_back({s, i, j, 0, 0});
    finish(T);
    interior.push_back(T);
  }
  // stage 2: Schur complement of the interior on every interface tile
  schur = begin(K_UPDATE);
  for (int s = 0; s < ns; ++s)
    if (subs[s].nt_i > 0)
      for (int J = subs[s].nt_i; J < subs[s].nt; ++J)
        for (int I = J; I < subs[s].nt; ++I) {
          const int k0 = std::max(E(s, I), E(s, J));
          if (k0 < subs[s].nt_i) tasks.push_back({s, I, J, k0, subs[s].nt_i});
        }
  plain(schur);
  // stage 4: interface columns (updates only over interface columns), each
  // update launch carrying the diagonal tasks of its column, as in stage 1,
  // and the previous block row of the interface inverse
  for (int jb = 0; jb < max_b; ++jb) {
    if (jb == 0) {
      auto D = begin(K_DIAG);
      for (int s = 0; s < ns; ++s)
        if (subs[s].nt_b > 0) tasks.push_back({s, subs[s].nt_i, subs[s].nt_i, 0, 0});
      finish(D);
      iface.push_back(D);
    } else {
      auto L = begin(K_UPDATE);
      for (int s = 0; s < ns; ++s)
        if (subs[s].nt_b > jb) {
          const int j = subs[s].nt_i + jb;
          tasks.push_back({s, j, j, j - 1, j});
        }
      L.ndiag = (int32_t)tasks.size() - L.first;
      for (int s = 0; s < ns; ++s)
        if (subs[s].nt_b > jb) {
          const int j = subs[s].nt_i + jb;
          for (int i = j + 1; i < subs[s].nt; ++i) tasks.push_back({s, i, j, subs[s].nt_i, j});
          if (subs[s].nt_b > jb + 1) tasks.push_back({s, j + 1, j + 1, subs[s].nt_i, j});
        }
      fused(L, K_UPD_TRTRI, jb - 1);
      iface.push_back(L);
    }
    auto T = begin(K_TRSM);
    for (int s = 0; s < ns; ++s)
      if (subs[s].nt_b > jb) {
        const int j = subs[s].nt_i + jb;
        for (int i = j + 1; i < subs[s].nt; ++i) tasks.push_back({s, i, j, 0, 0});
      }
    finish(T);
    iface.push_back(T);
  }
  // stage 5: the last block row of the interface inverse
  if (max_b > 0) {
    auto L = begin(K_TRTRI);
    inverse_row(max_b - 1);
    finish(L);
    trtri.push_back(L);
  }
  // stage 6: X = W^T W
  lauum = begin(K_LAUUM);
  for (int s = 0; s < ns; ++s)
    for (int I = 0; I < subs[s].nt_b; ++I)
      for (int J = 0; J <= I; ++J) tasks.push_back({s, I, J, I, subs[s].nt_b});
  finish(lauum);
  xtiles = begin(-1);
  for (int s = 0; s < ns; ++s)
    for (int I = 0; I < subs[s].nt_b; ++I)
      for (int J = 0; J <= I; ++J) tasks.push_back({s, I, J, 0, 0});
  finish(xtiles);
  // the tiles any step reads: inside the envelope, and the whole interface
  // block (dense after the Schur update)
  alltiles = begin(-1);
  for (int s = 0; s < ns; ++s)
    for (int i = 0; i < subs[s].nt; ++i)
      for (int j = 0; j <= i; ++j)
        if (E(s, i) <= j || j >= subs[s].nt_i) tasks.push_back({s, i, j, 0, 0});
  finish(alltiles);
}

static bool finite(double v) { return std::isfinite(v); }

std::string build_plan(const feti_mesh* m, const feti_options* o, HostPlan& P) {
  if (!m) return "mesh is NULL";
  if (m->n_nodes <= 0 || m->n_elems <= 0 || m->n_sub <= 0 || m->n_mat <= 0) return "empty mesh";
  // the coarse vector (6 per subdomain) of a projection is staged in 64 KiB of LDS
  if (m->n_sub > kMaxSub) return "more than " + std::to_string(kMaxSub) + " subdomains";
  if (!m->xyz || !m->hex8 || !m->elem_sub || !m->mat || !m->elem_mat) return "missing mesh array";
  if (m->n_dir < 0 || (m->n_dir > 0 && (!m->dir_dof || !m->dir_val))) return "bad Dirichlet arrays";
  if (m->n_pfaces < 0 || (m->n_pfaces > 0 && !m->pface)) return "bad pressure faces";
  if (m->n_nodes > (int64_t)1 << 30 || m->n_elems > (int64_t)1 << 30) return "mesh too large";
  if (m->order != 0 && m->order != 1 && m->order != 2) return "element order must be 1 (Q1) or 2 (Q2)";
  P.npe = m->order == 2 ? 27 : 8;
  P.nfn = m->order == 2 ? 9 : 4;
  P.ellw = m->order == 2 ? ELLW_Q2 : ELLW_Q1;
  P.af = !o || o->variant == FETI_ALL_FLOATING;
  P.precond = o ? (int)o->precond : (int)FETI_PREC_LUMPED;
  P.mixed = o && o->precision == FETI_MIXED;
  if (P.precond < 0 || P.precond > 2) return "bad preconditioner";
  P.n_nodes = m->n_nodes;
  P.n_elems = m->n_elems;
  P.n_dof = 3 * m->n_nodes;
  P.n_sub = m->n_sub;
  P.xyz.assign(m->xyz, m->xyz + 3 * m->n_nodes);
  for (double v : P.xyz)
    if (!finite(v)) return "non-finite coordinate";
  const int npe = P.npe;
  P.hex8.assign(m->hex8, m->hex8 + (int64_t)npe * m->n_elems);
  for (int64_t v : P.hex8)
    if (v < 0 || v >= m->n_nodes) return "element node id out of range";
  P.elem_sub.assign(m->elem_sub, m->elem_sub + m->n_elems);
  for (int32_t v : P.elem_sub)
    if (v < 0 || v >= m->n_sub) return "subdomain id out of range";
  P.elem_mat.assign(m->elem_mat, m->elem_mat + m->n_elems);
  P.mat.assign(m->mat, m->mat + m->n_mat);
  for (const auto& mt : P.mat) {
    if (mt.kind == 0) {
      if (!(mt.E > 0) || !(mt.nu > -1.0 && mt.nu < 0.5)) return "bad linear material";
    } else if (mt.kind == 1) {
      if (!(mt.c > 0) || !(mt.k1 >= 0) || !(mt.k2 > 0) || !(mt.kappa > 0)) return "bad HGO material";
    } else {
      return "unknown material kind";
    }
  }
  for (int32_t v : P.elem_mat) {
    if (v < 0 || v >= m->n_mat) return "material id out of range";
    if (P.mat[v].kind == 1) P.any_hgo = true;
  }
  if (P.any_hgo) {
    if (!m->elem_fibers) return "HGO material needs fibre directions";
    P.fibers.assign(m->elem_fibers, m->elem_fibers + 6 * m->n_elems);
    for (double v : P.fibers)
      if (!finite(v)) return "non-finite fibre";
  }
  if (m->body_force) {
    P.body_force.assign(m->body_force, m->body_force + 3 * m->n_elems);
    for (double v : P.body_force)
      if (!finite(v)) return "non-finite body force";
  }
  if (m->n_pfaces > 0) {
    P.pface.assign(m->pface, m->pface + (int64_t)P.nfn * m->n_pfaces);
    for (int64_t v : P.pface)
      if (v < 0 || v >= m->n_nodes) return "pressure face node out of range";
  }
  if (!finite(m->pressure)) return "non-finite pressure";
  P.pressure = m->pressure;
  P.dir_mask.assign(P.n_dof, 0);
  P.dir_val.assign(P.n_dof, 0.0);
  for (int64_t k = 0; k < m->n_dir; ++k) {
    const int64_t d = m->dir_dof[k];
    if (d < 0 || d >= P.n_dof) return "Dirichlet dof out of range";
    if (P.dir_mask[d]) return "duplicate Dirichlet dof";
    if (!finite(m->dir_val[k])) return "non-finite Dirichlet value";
    P.dir_mask[d] = 1;
    P.dir_val[d] = m->dir_val[k];
  }
  for (int64_t d = 0; d < P.n_dof; ++d)
    if (P.dir_mask[d]) P.dir_list.push_back(d);
  if (P.dir_list.empty()) return "no Dirichlet data: the problem is singular";

  const int ns = P.n_sub;
  // ---- elements per subdomain (ascending element id)
  std::vector<int64_t> se_ptr(ns + 1, 0), se_list(P.n_elems);
  for (int32_t s : P.elem_sub) se_ptr[s + 1]++;
  for (int s = 0; s < ns; ++s) {
    if (se_ptr[s + 1] == 0) return "empty subdomain " + std::to_string(s);
    se_ptr[s + 1] += se_ptr[s];
  }
  {
    std::vector<int64_t> fill(se_ptr.begin(), se_ptr.end() - 1);
    for (int64_t e = 0; e < P.n_elems; ++e) se_list[fill[P.elem_sub[e]]++] = e;
  }
  // ---- local nodes and connectivity check
  P.sub.assign(ns, SubInfo{});
  std::vector<int32_t> g2l(P.n_nodes, -1);
  std::vector<std::vector<int32_t>> elem_ln(ns);   // per sub: npe local node ids per element
  for (int s = 0; s < ns; ++s) {
    std::vector<int64_t> nodes;
    for (int64_t k = se_ptr[s]; k < se_ptr[s + 1]; ++k)
      for (int c = 0; c < npe; ++c) nodes.push_back(P.hex8[se_list[k] * npe + c]);
    std::sort(nodes.begin(), nodes.end());
    nodes.erase(std::unique(nodes.begin(), nodes.end()), nodes.end());
    SubInfo& si = P.sub[s];
    si.n_nodes = (int32_t)nodes.size();
    si.node_off = (int32_t)P.loc_node.size();
    for (size_t q = 0; q < nodes.size(); ++q) {
      g2l[nodes[q]] = (int32_t)q;
      P.loc_node.push_back(nodes[q]);
    }
    auto& el = elem_ln[s];
    const int64_t ne = se_ptr[s + 1] - se_ptr[s];
    el.resize(npe * ne);
    for (int64_t k = 0; k < ne; ++k)
      for (int c = 0; c < npe; ++c) el[npe * k + c] = g2l[P.hex8[se_list[se_ptr[s] + k] * npe + c]];
    // union-find over elements sharing a node
    std::vector<int32_t> parent(ne), owner(nodes.size(), -1);
    std::iota(parent.begin(), parent.end(), 0);
    std::function<int32_t(int32_t)> findp = [&](int32_t x) {
      while (parent[x] != x) x = parent[x] = parent[parent[x]];
      return x;
    };
    for (int64_t k = 0; k < ne; ++k)
      for (int c = 0; c < npe; ++c) {
        const int32_t ln = el[npe * k + c];
        if (owner[ln] < 0) owner[ln] = (int32_t)k;
        else parent[findp((int32_t)k)] = findp(owner[ln]);
      }
    for (int64_t k = 1; k < ne; ++k)
      if (findp((int32_t)k) != findp(0)) return "disconnected subdomain " + std::to_string(s);
    for (int64_t g : nodes) g2l[g] = -1;
  }
  P.n_loc_nodes = (int64_t)P.loc_node.size();
  // ---- node copies (ascending subdomain)
  std::vector<int32_t> nc_ptr(P.n_nodes + 1, 0), nc_loc;
  for (int s = 0; s < ns; ++s)
    for (int q = 0; q < P.sub[s].n_nodes; ++q) nc_ptr[P.loc_node[P.sub[s].node_off + q] + 1]++;
  for (int64_t n = 0; n < P.n_nodes; ++n) nc_ptr[n + 1] += nc_ptr[n];
  nc_loc.resize(nc_ptr[P.n_nodes]);
  {
    std::vector<int32_t> fill(nc_ptr.begin(), nc_ptr.end() - 1);
    for (int s = 0; s < ns; ++s)
      for (int q = 0; q < P.sub[s].n_nodes; ++q) {
        const int32_t ln = P.sub[s].node_off + q;
        nc_loc[fill[P.loc_node[ln]]++] = ln;
      }
  }
  P.loc_sub.assign(P.n_loc_nodes, 0);
  auto& loc_sub = P.loc_sub;
  for (int s = 0; s < ns; ++s)
    for (int q = 0; q < P.sub[s].n_nodes; ++q) loc_sub[P.sub[s].node_off + q] = s;
  P.loc_ncopy.resize(P.n_loc_nodes);
  for (int64_t ln = 0; ln < P.n_loc_nodes; ++ln) {
    const int64_t g = P.loc_node[ln];
    P.loc_ncopy[ln] = nc_ptr[g + 1] - nc_ptr[g];
  }
  // ---- multiplier rows (entries as local-dof ids 3*ln + comp)
  std::vector<int64_t> re0, re1;
  std::vector<uint8_t> is_b(3 * P.n_loc_nodes, 0);
  for (int64_t g = 0; g < P.n_dof; ++g) {
    const int64_t nd = g / 3;
    const int comp = (int)(g % 3);
    const int nc = nc_ptr[nd + 1] - nc_ptr[nd];
    const bool isdir = P.dir_mask[g];
    if (!P.af && isdir) continue;
    // Scaled rows of B_D (eq. (feti_preconditioner)): 1/multiplicity on the
    // gluing rows.  At a Dirichlet DOF of the all-floating variant the
    // boundary is a neighbour whose value is fixed: its row carries the whole
    // jump of each copy (weight 1) and the gluing rows between the copies
    // carry none, which keeps B B_D^T B = B (B_D^T B a projection).
    const bool afdir = P.af && isdir;
    const double w_glue = afdir ? 0.0 : 1.0 / nc;
    for (int a = 0; a < nc; ++a)
      for (int b = a + 1; b < nc; ++b) {
        re0.push_back(3 * (int64_t)nc_loc[nc_ptr[nd] + a] + comp);
        re1.push_back(3 * (int64_t)nc_loc[nc_ptr[nd] + b] + comp);
        P.r_c0.push_back(1.0);
        P.r_c1.push_back(-1.0);
        P.r_w.push_back(w_glue);
        P.r_gdof.push_back(-1);
      }
    if (P.af && isdir)
      for (int a = 0; a < nc; ++a) {
        re0.push_back(3 * (int64_t)nc_loc[nc_ptr[nd] + a] + comp);
        re1.push_back(-1);
        P.r_c0.push_back(1.0);
        P.r_c1.push_back(0.0);
        P.r_w.push_back(1.0);
        P.r_gdof.push_back(g);
      }
  }
  P.n_lam = (int64_t)re0.size();
  for (size_t r = 0; r < re0.size(); ++r) {
    is_b[re0[r]] = 1;
    if (re1[r] >= 0) is_b[re1[r]] = 1;
  }
  // ---- interior-first positions
  P.loc_pos.assign(3 * P.n_loc_nodes, -1);
  int64_t tile_off = 0, linv_off = 0, x_off = 0, full_off = 0, b_off = 0, part_off = 0;
  for (int s = 0; s < ns; ++s) {
    SubInfo& si = P.sub[s];
    int n_ii = 0, n_b = 0;
    bool has_dir = false;
    for (int q = 0; q < si.n_nodes; ++q)
      for (int c = 0; c < 3; ++c) {
        const int64_t ld = 3 * (int64_t)(si.node_off + q) + c;
        const int64_t g = 3 * P.loc_node[si.node_off + q] + c;
        if (P.dir_mask[g]) has_dir = true;
        if (!P.af && P.dir_mask[g]) continue;
        if (is_b[ld]) n_b++;
        else n_ii++;
      }
    // The interior block holds whole tiles only when that costs no interface
    // tile: the last n_ii mod 64 interior DOFs then join the trailing block,
    // behind the interface DOFs.  Eliminating fewer DOFs first gives another
    // generalised inverse of K_i; the projected dual iteration and the
    // displacements do not depend on that choice (they differ by terms in
    // range(G)).  The Dirichlet preconditioner needs the Schur complement on
    // exactly the interface DOFs and keeps the split as it is.
    int r_move = 0;
    if (P.precond != FETI_PREC_DIRICHLET) {
      const int r = n_ii % TS;
      if (r > 0 && ceil_tiles(n_b + r) == ceil_tiles(n_b)) r_move = r;
    }
    si.n_if = n_b;
    si.n_ii = n_ii - r_move;
    si.n_b = n_b + r_move;
    si.nt_i = ceil_tiles(si.n_ii);
    si.nt_b = ceil_tiles(si.n_b);
    si.nt = si.nt_i + si.nt_b;
    // A classical subdomain with Dirichlet DOFs has the partial kernel of the
    // rigid modes that vanish on them (none for a clamped face; rotations
    // about a clamped vertex or edge; modes free of a constrained component),
    // section 4.3.  Its dimension is found on the device (k_modes).
    si.floating = (P.af || !has_dir) ? 1 : 2;
    si.n_modes = si.floating == 1 ? 6 : 0;
    if (si.floating == 1 && n_b == 0) return "floating subdomain " + std::to_string(s) + " has no interface";
    int pi = 0, pb = si.nt_i * TS, px = si.nt_i * TS + si.n_if;
    for (int q = 0; q < si.n_nodes; ++q)
      for (int c = 0; c < 3; ++c) {
        const int64_t ld = 3 * (int64_t)(si.node_off + q) + c;
        const int64_t g = 3 * P.loc_node[si.node_off + q] + c;
        if (!P.af && P.dir_mask[g]) continue;
        P.loc_pos[ld] = is_b[ld] ? pb++ : (pi < si.n_ii ? pi++ : px++);
      }
    si.tile_off = tile_off;
    si.linv_off = linv_off;
    si.x_off = x_off;
    si.full_off = full_off;
    si.b_off = b_off;
    si.part_off = part_off;
    tile_off += (int64_t)si.nt * (si.nt + 1) / 2 * TS2;
    linv_off += (int64_t)si.nt * TS2;
    x_off += (int64_t)si.nt_b * (si.nt_b + 1) / 2 * TS2;
    full_off += (int64_t)si.nt * TS;
    b_off += (int64_t)si.nt_b * TS;
    part_off += (int64_t)si.nt_b * si.nt_b * TS;
    P.max_nt_i = std::max(P.max_nt_i, si.nt_i);
    P.max_nt_b = std::max(P.max_nt_b, si.nt_b);
  }
  P.n_tiles = tile_off;
  P.n_linv = linv_off;
  P.n_xtiles = x_off;
  P.NF = full_off;
  P.NB = b_off;
  P.n_part = part_off;
  if (P.NB >= ((int64_t)1 << 31) || P.n_lam >= ((int64_t)1 << 31)) return "problem too large";
  P.fpos_lnode.assign(P.NF, -1);
  P.fpos_comp.assign(P.NF, 0);
  P.f_sub.assign(P.NF, 0);
  for (int s = 0; s < ns; ++s) {
    const SubInfo& si = P.sub[s];
    for (int64_t k = 0; k < (int64_t)si.nt * TS; ++k) P.f_sub[si.full_off + k] = s;
    for (int q = 0; q < si.n_nodes; ++q)
      for (int c = 0; c < 3; ++c) {
        const int pos = P.loc_pos[3 * (int64_t)(si.node_off + q) + c];
        if (pos < 0) continue;
        P.fpos_lnode[si.full_off + pos] = si.node_off + q;
        P.fpos_comp[si.full_off + pos] = (int8_t)c;
      }
  }
  // ---- rows in b-space
  auto bidx = [&](int64_t ld) -> int64_t {
    const int s = loc_sub[ld / 3];
    const SubInfo& si = P.sub[s];
    return si.b_off + (P.loc_pos[ld] - (int64_t)si.nt_i * TS);
  };
  P.r_b0.resize(P.n_lam);
  P.r_b1.resize(P.n_lam);
  for (int64_t r = 0; r < P.n_lam; ++r) {
    P.r_b0[r] = bidx(re0[r]);
    P.r_b1[r] = re1[r] >= 0 ? bidx(re1[r]) : -1;
  }
  P.g_ptr.assign(P.NB + 1, 0);
  for (int64_t r = 0; r < P.n_lam; ++r) {
    P.g_ptr[P.r_b0[r] + 1]++;
    if (P.r_b1[r] >= 0) P.g_ptr[P.r_b1[r] + 1]++;
  }
  for (int64_t b = 0; b < P.NB; ++b) P.g_ptr[b + 1] += P.g_ptr[b];
  P.g_row.resize(P.g_ptr[P.NB]);
  P.g_coef.resize(P.g_ptr[P.NB]);
  {
    std::vector<int32_t> fill(P.g_ptr.begin(), P.g_ptr.end() - 1);
    for (int64_t r = 0; r < P.n_lam; ++r) {
      int32_t k = fill[P.r_b0[r]]++;
      P.g_row[k] = (int32_t)r;
      P.g_coef[k] = P.r_c0[r];
      if (P.r_b1[r] >= 0) {
        k = fill[P.r_b1[r]]++;
        P.g_row[k] = (int32_t)r;
        P.g_coef[k] = P.r_c1[r];
      }
    }
  }
  // ---- copy coupling C = B^T B and C~ = B^T diag(w) B: entry (b, b') sums
  // c_{r,b} c_{r,b'} (times w_r) over the rows r holding both, so that
  // B^T (B v) is one gather from v; columns ascending
  P.c_ptr.assign(P.NB + 1, 0);
  P.c_col.clear();
  P.c_v0.clear();
  P.c_v1.clear();
  {
    std::vector<std::pair<int64_t, std::pair<double, double>>> ent;
    for (int64_t b = 0; b < P.NB; ++b) {
      ent.clear();
      for (int32_t k = P.g_ptr[b]; k < P.g_ptr[b + 1]; ++k) {
        const int64_t r = P.g_row[k];
        const double c = P.g_coef[k], w = P.r_w[r];
        ent.push_back({P.r_b0[r], {c * P.r_c0[r], c * P.r_c0[r] * w}});
        if (P.r_b1[r] >= 0) ent.push_back({P.r_b1[r], {c * P.r_c1[r], c * P.r_c1[r] * w}});
      }
      std::sort(ent.begin(), ent.end(), [](const auto& x, const auto& y) { return x.first < y.first; });
      for (size_t i = 0; i < ent.size();) {
        size_t j = i;
        double v0 = 0.0, v1 = 0.0;
        for (; j < ent.size() && ent[j].first == ent[i].first; ++j) {
          v0 += ent[j].second.first;
          v1 += ent[j].second.second;
        }
        P.c_col.push_back((int32_t)ent[i].first);
        P.c_v0.push_back(v0);
        P.c_v1.push_back(v1);
        i = j;
      }
      P.c_ptr[b + 1] = (int32_t)P.c_col.size();
    }
  }
  P.b2full.resize(P.NB);
  P.b_sub.resize(P.NB);
  for (int s = 0; s < ns; ++s) {
    const SubInfo& si = P.sub[s];
    for (int64_t k = 0; k < (int64_t)si.nt_b * TS; ++k) {
      P.b2full[si.b_off + k] = si.full_off + (int64_t)si.nt_i * TS + k;
      P.b_sub[si.b_off + k] = s;
    }
  }
  // ---- node pairs and element contributions (per subdomain, fixed order)
  P.diag_slot.assign(P.n_loc_nodes, -1);
  P.ell_col.assign(P.NF * P.ellw, -1);
  const int max_nbr = P.ellw / 3;
  for (int s = 0; s < ns; ++s) {
    const SubInfo& si = P.sub[s];
    const auto& el = elem_ln[s];
    const int64_t ne = se_ptr[s + 1] - se_ptr[s];
    std::vector<int32_t> inc_ptr(si.n_nodes + 1, 0), inc(npe * ne);
    for (int64_t k = 0; k < ne; ++k)
      for (int c = 0; c < npe; ++c) inc_ptr[el[npe * k + c] + 1]++;
    for (int q = 0; q < si.n_nodes; ++q) inc_ptr[q + 1] += inc_ptr[q];
    {
      std::vector<int32_t> fill(inc_ptr.begin(), inc_ptr.end() - 1);
      for (int64_t k = 0; k < ne; ++k)
        for (int c = 0; c < npe; ++c) inc[fill[el[npe * k + c]]++] = (int32_t)(npe * k + c);
    }
    std::vector<std::array<int32_t, 4>> tup;   // (b, elem-local k, la, lb)
    for (int a = 0; a < si.n_nodes; ++a) {
      tup.clear();
      for (int t = inc_ptr[a]; t < inc_ptr[a + 1]; ++t) {
        const int32_t k = inc[t] / npe, la = inc[t] % npe;
        for (int lb = 0; lb < npe; ++lb) tup.push_back({el[npe * k + lb], k, la, lb});
      }
      std::sort(tup.begin(), tup.end());
      int nbr = -1, prev_b = -1;
      for (size_t t = 0; t < tup.size(); ++t) {
        if (tup[t][0] != prev_b) {
          if (nbr >= 0) P.ps_c1.push_back((int32_t)P.pc_e.size());
          ++nbr;
          if (nbr >= max_nbr)
            return "node with more than " + std::to_string(max_nbr) + " neighbours (not a hexahedral mesh)";
          prev_b = tup[t][0];
          P.ps_a.push_back(si.node_off + a);
          P.ps_b.push_back(si.node_off + tup[t][0]);
          P.ps_nbr.push_back(nbr);
          P.ps_c0.push_back((int32_t)P.pc_e.size());
          if (tup[t][0] == a) P.diag_slot[si.node_off + a] = (int32_t)P.ps_a.size() - 1;
          // ELL columns of the three rows of node a against node b
          for (int i = 0; i < 3; ++i) {
            const int row = P.loc_pos[3 * (int64_t)(si.node_off + a) + i];
            if (row < 0) continue;
            for (int j = 0; j < 3; ++j) {
              const int64_t ldb = 3 * (int64_t)(si.node_off + tup[t][0]) + j;
              const int col = P.loc_pos[ldb];
              const int64_t gb = 3 * P.loc_node[si.node_off + tup[t][0]] + j;
              P.ell_col[(int64_t)(nbr * 3 + j) * P.NF + si.full_off + row] = col >= 0 ? col : (int32_t)(-(gb + 2));
            }
          }
        }
        P.pc_e.push_back((int32_t)se_list[se_ptr[s] + tup[t][1]]);
        P.pc_ab.push_back(tup[t][2] | (tup[t][3] << 8));
      }
      if (nbr >= 0) P.ps_c1.push_back((int32_t)P.pc_e.size());
    }
  }
  // ---- interface-interface block of every local stiffness (lumped preconditioner)
  {
    std::vector<std::vector<std::pair<int32_t, int32_t>>> rows(P.NB);
    int32_t w = 0;
    for (int s = 0; s < ns; ++s) {
      const SubInfo& si = P.sub[s];
      const int bstart = si.nt_i * TS;
      for (int pb = 0; pb < si.n_if; ++pb) {
        const int64_t row = si.full_off + bstart + pb;
        auto& L = rows[si.b_off + pb];
        for (int k = 0; k < P.ellw; ++k) {
          const int c = P.ell_col[(int64_t)k * P.NF + row];
          if (c >= bstart && c < bstart + si.n_if) L.push_back({k, (int32_t)(si.b_off + c - bstart)});
        }
        w = std::max<int32_t>(w, (int32_t)L.size());
      }
    }
    P.w_bb = w;
    P.bb_slot.assign((size_t)w * P.NB, -1);
    P.bb_col.assign((size_t)w * P.NB, 0);
    for (int64_t b = 0; b < P.NB; ++b)
      for (size_t k = 0; k < rows[b].size(); ++k) {
        P.bb_slot[k * P.NB + b] = rows[b][k].first;
        P.bb_col[k * P.NB + b] = rows[b][k].second;
      }
  }
  // ---- copies of every global dof in the full local space
  P.uc_ptr.assign(P.n_dof + 1, 0);
  for (int64_t g = 0; g < P.n_dof; ++g) {
    const int64_t nd = g / 3;
    int cnt = 0;
    for (int k = nc_ptr[nd]; k < nc_ptr[nd + 1]; ++k)
      if (P.loc_pos[3 * (int64_t)nc_loc[k] + g % 3] >= 0) cnt++;
    P.uc_ptr[g + 1] = P.uc_ptr[g] + cnt;
  }
  P.uc_idx.resize(P.uc_ptr[P.n_dof]);
  for (int64_t g = 0; g < P.n_dof; ++g) {
    const int64_t nd = g / 3;
    int w = P.uc_ptr[g];
    for (int k = nc_ptr[nd]; k < nc_ptr[nd + 1]; ++k) {
      const int32_t ln = nc_loc[k];
      const int pos = P.loc_pos[3 * (int64_t)ln + g % 3];
      if (pos >= 0) P.uc_idx[w++] = P.sub[loc_sub[ln]].full_off + pos;
    }
  }
  // ---- pressure faces per node
  P.pf_ptr.assign(P.n_nodes + 1, 0);
  const int nfn = P.nfn;
  const int64_t nf = (int64_t)P.pface.size() / nfn;
  for (int64_t f = 0; f < nf; ++f)
    for (int c = 0; c < nfn; ++c) P.pf_ptr[P.pface[nfn * f + c] + 1]++;
  for (int64_t n = 0; n < P.n_nodes; ++n) P.pf_ptr[n + 1] += P.pf_ptr[n];
  P.pf_ent.resize(P.pf_ptr[P.n_nodes]);
  {
    std::vector<int32_t> fill(P.pf_ptr.begin(), P.pf_ptr.end() - 1);
    for (int64_t f = 0; f < nf; ++f)
      for (int c = 0; c < nfn; ++c) P.pf_ent[fill[P.pface[nfn * f + c]]++] = (int32_t)(nfn * f + c);
  }
  // ---- coarse pairs: (s >= t) with the rows they share; diagonal pairs use every entry
  {
    std::vector<std::array<int64_t, 4>> ent;   // (s, t, bs, bt) with coef in parallel array
    std::vector<double> cf;
    for (int64_t r = 0; r < P.n_lam; ++r) {
      const int s0 = P.b_sub[P.r_b0[r]];
      ent.push_back({s0, s0, P.r_b0[r], P.r_b0[r]});
      cf.push_back(P.r_c0[r] * P.r_c0[r]);
      if (P.r_b1[r] >= 0) {
        const int s1 = P.b_sub[P.r_b1[r]];
        ent.push_back({s1, s1, P.r_b1[r], P.r_b1[r]});
        cf.push_back(P.r_c1[r] * P.r_c1[r]);
        if (s1 >= s0) ent.push_back({s1, s0, P.r_b1[r], P.r_b0[r]});
        else ent.push_back({s0, s1, P.r_b0[r], P.r_b1[r]});
        cf.push_back(P.r_c0[r] * P.r_c1[r]);
      }
    }
    std::vector<size_t> ord(ent.size());
    std::iota(ord.begin(), ord.end(), 0);
    std::stable_sort(ord.begin(), ord.end(), [&](size_t x, size_t y) {
      return ent[x][0] != ent[y][0] ? ent[x][0] < ent[y][0] : ent[x][1] < ent[y][1];
    });
    for (size_t k = 0; k < ord.size(); ++k) {
      const auto& e = ent[ord[k]];
      if (k == 0 || e[0] != ent[ord[k - 1]][0] || e[1] != ent[ord[k - 1]][1]) {
        P.qp_s.push_back((int32_t)e[0]);
        P.qp_t.push_back((int32_t)e[1]);
        P.qp_ptr.push_back((int32_t)P.qe_bs.size());
      }
      P.qe_bs.push_back(e[2]);
      P.qe_bt.push_back(e[3]);
      P.qe_c.push_back(cf[ord[k]]);
    }
    P.qp_ptr.push_back((int32_t)P.qe_bs.size());
  }
  // tile envelope of every local stiffness (arena order): the first tile
  // column with an entry of the assembled sparse rows of each tile row
  std::vector<std::vector<int32_t>> env(ns);
  P.env.clear();
  for (int s = 0; s < ns; ++s) {
    SubInfo& si = P.sub[s];
    env[s].resize(si.nt);
    for (int I = 0; I < si.nt; ++I) env[s][I] = I;
    for (int r = 0; r < si.nt * TS; ++r)
      for (int k = 0; k < P.ellw; ++k) {
        const int c = P.ell_col[(int64_t)k * P.NF + si.full_off + r];
        if (c >= 0) env[s][r / TS] = std::min(env[s][r / TS], c / TS);
      }
    si.env_off = (int32_t)P.env.size();
    P.env.insert(P.env.end(), env[s].begin(), env[s].end());
  }
  build_factor_schedule(P.sub, P.tasks, P.sched_interior, P.sched_schur, P.sched_iface, P.sched_trtri,
                        P.sched_lauum, P.sched_xtiles, P.sched_alltiles, &env);
  return "";
}

}  // namespace feti
