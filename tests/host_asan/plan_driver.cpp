// Host-only driver of the plan builder (decomp.cpp), built with AddressSanitizer
// and UndefinedBehaviorSanitizer by tests/test_host_sanitizers.py.  It builds
// structured cube meshes in memory, runs build_plan for both variants and all
// preconditioners, checks the multiplier counts against their closed forms, and
// feeds malformed meshes that must be rejected with a message.
#include <cstdio>
#include <cstdlib>
#include <string>
#include <vector>

#include "feti_impl.h"

namespace {

struct Cube {
  std::vector<double> xyz;
  std::vector<int64_t> hex8;
  std::vector<int32_t> esub, emat;
  std::vector<int64_t> ddof;
  std::vector<double> dval, body;
  feti_material mat{0, 1.0, 0.3, 0, 0, 0, 0};
};

// n^3 elements of the unit cube in m^3 boxes; clamped on the whole boundary
// (partial = false), or on the quarter y, z <= 1/2 of x = 0 plus u_x = 0 on x = 1.
Cube cube(int n, int m, bool partial) {
  Cube c;
  const int nn = n + 1;
  for (int k = 0; k < nn; ++k)
    for (int j = 0; j < nn; ++j)
      for (int i = 0; i < nn; ++i) {
        c.xyz.push_back((double)i / n);
        c.xyz.push_back((double)j / n);
        c.xyz.push_back((double)k / n);
      }
  const int h = n / m;
  for (int ez = 0; ez < n; ++ez)
    for (int ey = 0; ey < n; ++ey)
      for (int ex = 0; ex < n; ++ex) {
        const int64_t b = ex + (int64_t)nn * (ey + (int64_t)nn * ez);
        const int64_t o[8] = {0, 1, nn, nn + 1, (int64_t)nn * nn, (int64_t)nn * nn + 1,
                              (int64_t)nn * nn + nn, (int64_t)nn * nn + nn + 1};
        for (int a = 0; a < 8; ++a) c.hex8.push_back(b + o[a]);
        c.esub.push_back(ex / h + m * (ey / h + m * (ez / h)));
        c.emat.push_back(0);
        c.body.insert(c.body.end(), {0.0, 0.0, -1.0});
      }
  for (int k = 0; k < nn; ++k)
    for (int j = 0; j < nn; ++j)
      for (int i = 0; i < nn; ++i) {
        const int64_t g = i + (int64_t)nn * (j + (int64_t)nn * k);
        const bool bnd = i == 0 || j == 0 || k == 0 || i == n || j == n || k == n;
        if (!partial && bnd) {
          for (int d = 0; d < 3; ++d) c.ddof.push_back(3 * g + d);
        } else if (partial && i == 0 && 2 * j <= n && 2 * k <= n) {
          for (int d = 0; d < 3; ++d) c.ddof.push_back(3 * g + d);
        } else if (partial && i == n) {
          c.ddof.push_back(3 * g);
        }
      }
  c.dval.assign(c.ddof.size(), 0.0);
  return c;
}

// The same node grid with n^3 27-node (Q2) elements, (2n+1)^3 nodes, clamped
// on the whole boundary, and 9-node pressure faces on x = 0.
Cube cube27(int n, int m, std::vector<int64_t>& pface) {
  Cube c;
  const int nn = 2 * n + 1;
  for (int k = 0; k < nn; ++k)
    for (int j = 0; j < nn; ++j)
      for (int i = 0; i < nn; ++i) {
        c.xyz.push_back((double)i / (2 * n));
        c.xyz.push_back((double)j / (2 * n));
        c.xyz.push_back((double)k / (2 * n));
      }
  const int h = n / m;
  auto id = [&](int i, int j, int k) { return i + (int64_t)nn * (j + (int64_t)nn * k); };
  for (int ez = 0; ez < n; ++ez)
    for (int ey = 0; ey < n; ++ey)
      for (int ex = 0; ex < n; ++ex) {
        for (int a = 0; a < 27; ++a) c.hex8.push_back(id(2 * ex + a % 3, 2 * ey + (a / 3) % 3, 2 * ez + a / 9));
        c.esub.push_back(ex / h + m * (ey / h + m * (ez / h)));
        c.emat.push_back(0);
        c.body.insert(c.body.end(), {0.0, 0.0, -1.0});
      }
  for (int k = 0; k < nn; ++k)
    for (int j = 0; j < nn; ++j)
      for (int i = 0; i < nn; ++i)
        if (i == 0 || j == 0 || k == 0 || i == nn - 1 || j == nn - 1 || k == nn - 1)
          for (int d = 0; d < 3; ++d) c.ddof.push_back(3 * id(i, j, k) + d);
  c.dval.assign(c.ddof.size(), 0.0);
  for (int ez = 0; ez < n; ++ez)
    for (int ey = 0; ey < n; ++ey)
      for (int a = 0; a < 9; ++a) pface.push_back(id(0, 2 * ey + a / 3, 2 * ez + a % 3));
  return c;
}

feti_mesh view(Cube& c, int m) {
  feti_mesh M{};
  M.n_nodes = (int64_t)c.xyz.size() / 3;
  M.xyz = c.xyz.data();
  M.n_elems = (int64_t)c.esub.size();
  M.hex8 = c.hex8.data();
  M.n_sub = m * m * m;
  M.elem_sub = c.esub.data();
  M.n_mat = 1;
  M.mat = &c.mat;
  M.elem_mat = c.emat.data();
  M.n_dir = (int64_t)c.ddof.size();
  M.dir_dof = c.ddof.data();
  M.dir_val = c.dval.data();
  M.body_force = c.body.data();
  return M;
}

int failures = 0;
void expect(bool ok, const std::string& what) {
  if (!ok) {
    std::printf("FAIL %s\n", what.c_str());
    ++failures;
  }
}

}  // namespace

int main() {
  // multiplier counts of the 8^3 cube in 2^3 boxes (fully redundant gluing,
  // all-floating Dirichlet rows per copy): 2556 all-floating, 732 classical
  for (int af = 0; af < 2; ++af)
    for (int pc = 0; pc < 3; ++pc) {
      Cube c = cube(8, 2, false);
      feti_mesh M = view(c, 2);
      feti_options o{};
      o.variant = af ? FETI_ALL_FLOATING : FETI_CLASSICAL;
      o.precond = (feti_precond)pc;
      feti::HostPlan P;
      const std::string e = feti::build_plan(&M, &o, P);
      expect(e.empty(), "cube8 plan: " + e);
      expect(P.n_lam == (af ? 2556 : 732), "cube8 multipliers " + std::to_string(P.n_lam));
      expect(P.n_sub == 8 && !P.tasks.empty(), "cube8 schedule");
      bool prefix = true;
      for (int64_t r = 0; r < P.NF; ++r) {
        bool empty = false;
        for (int k = 0; k < P.ellw; ++k) {
          const int cc = P.ell_col[(int64_t)k * P.NF + r];
          if (cc == -1) empty = true;
          else if (empty) prefix = false;
        }
      }
      expect(prefix, "cube8 ELL rows are not prefix-filled");
    }
  // Q2 elements on the node grid of the 8^3 Q1 cube: the same multipliers;
  // 9-node pressure faces
  for (int af = 0; af < 2; ++af) {
    std::vector<int64_t> pf;
    Cube c = cube27(4, 2, pf);
    feti_mesh M = view(c, 2);
    M.order = 2;
    M.n_pfaces = (int64_t)pf.size() / 9;
    M.pface = pf.data();
    M.pressure = 1.0;
    feti_options o{};
    o.variant = af ? FETI_ALL_FLOATING : FETI_CLASSICAL;
    o.precond = FETI_PREC_DIRICHLET;
    feti::HostPlan P;
    const std::string e = feti::build_plan(&M, &o, P);
    expect(e.empty(), "q2 cube plan: " + e);
    expect(P.n_lam == (af ? 2556 : 732), "q2 cube multipliers " + std::to_string(P.n_lam));
    expect(P.npe == 27 && P.nfn == 9 && P.ellw == feti::ELLW_Q2, "q2 element and face sizes");
    expect(P.pf_ptr.back() == (int32_t)pf.size(), "q2 pressure face entries");
    // the filled ELL slots of every row form a prefix (the kernels stop at
    // the first empty slot)
    bool prefix = true;
    for (int64_t r = 0; r < P.NF; ++r) {
      bool empty = false;
      for (int k = 0; k < P.ellw; ++k) {
        const int c = P.ell_col[(int64_t)k * P.NF + r];
        if (c == -1) empty = true;
        else if (empty) prefix = false;
      }
    }
    expect(prefix, "q2 ELL rows are not prefix-filled");
    M.order = 3;
    feti::HostPlan P2;
    expect(!feti::build_plan(&M, &o, P2).empty(), "element order 3 accepted");
  }
  // uneven boxes and partial Dirichlet data
  for (int af = 0; af < 2; ++af) {
    Cube c = cube(12, 3, true);
    feti_mesh M = view(c, 3);
    feti_options o{};
    o.variant = af ? FETI_ALL_FLOATING : FETI_CLASSICAL;
    o.precond = FETI_PREC_DIRICHLET;
    feti::HostPlan P;
    const std::string e = feti::build_plan(&M, &o, P);
    expect(e.empty(), "partial plan: " + e);
    int partial = 0;
    for (const auto& s : P.sub) partial += s.floating == 2;
    expect(af ? partial == 0 : partial > 0, "partially constrained subdomains " + std::to_string(partial));
  }
  // malformed meshes are rejected with a message
  {
    Cube c = cube(4, 2, false);
    feti_mesh M = view(c, 2);
    feti_options o{};
    o.variant = FETI_ALL_FLOATING;
    c.hex8[5] = 1 << 20;
    feti::HostPlan P;
    expect(!feti::build_plan(&M, &o, P).empty(), "node id out of range accepted");
    c = cube(4, 2, false);
    M = view(c, 2);
    c.esub[0] = 99;
    feti::HostPlan P2;
    expect(!feti::build_plan(&M, &o, P2).empty(), "subdomain id out of range accepted");
    c = cube(4, 2, false);
    M = view(c, 2);
    M.n_dir = 0;
    feti::HostPlan P3;
    expect(!feti::build_plan(&M, &o, P3).empty(), "singular problem accepted");
    feti::HostPlan P4;
    expect(!feti::build_plan(nullptr, &o, P4).empty(), "NULL mesh accepted");
  }
  std::printf("%s (%d failures)\n", failures ? "FAILED" : "OK", failures);
  return failures ? 1 : 0;
}
