"""Checks against values the paper prints (fixtures in tests/golden/, each
citing its table).  The paper's cube uses P1 and P2 tetrahedra and a
different mesh and material, so its numbers are matched where the method
fixes them: the second-order L2 convergence of linear elements (Table 2 eoc)
and the third-order convergence of quadratic ones (Table 3 eoc), the
ordering of the preconditioners' iteration counts, the monotone growth of
the counts with refinement, and the material data (Table 1)."""
import json
import os

import numpy as np

from oracle import feti_ref, monolithic
from workloads import cube_mesh, kelvin_displacement, tube_mesh
from workloads.meshes import MEDIA, MAT_HGO

HERE = os.path.dirname(os.path.abspath(__file__))


def _golden(name):
    with open(os.path.join(HERE, "golden", name)) as f:
        return json.load(f)


def test_table1_media_parameters():
    g = _golden("table1_hgo_parameters.json")
    assert (MEDIA["c"], MEDIA["k1"], MEDIA["k2"]) == (g["c_kPa"], g["k1_kPa"], g["k2"])
    m = tube_mesh(nr=2, nth=8, nz=2, sub=(1, 1, 1))
    media = m.mat[(m.mat[:, 0] == MAT_HGO) & (m.mat[:, 3] == g["c_kPa"])]
    assert media.shape[0] == 1
    assert tuple(media[0, 3:6]) == (g["c_kPa"], g["k1_kPa"], g["k2"])


def test_table2_convergence_order():
    """The oracle's L2 error against the Kelvin solution falls with the order the
    paper prints for its finest levels (1.99), within 0.1."""
    g = _golden("table2_linear_cube.json")
    paper_eoc = g["all_floating"]["eoc"][-1]
    E, nu = 1.0, 0.3
    from test_oracle_pins import _l2_error
    errs = []
    for n in (8, 16):
        m = cube_mesh(n, 1, E=E, nu=nu, body_force=None, dirichlet_fn=lambda x: kelvin_displacement(x, E, nu))
        errs.append(_l2_error(m, monolithic.solve_linear(m), lambda x: kelvin_displacement(x, E, nu)))
    eoc = np.log(errs[0] / errs[1]) / np.log(2.0)
    assert abs(eoc - paper_eoc) <= 0.1, (eoc, paper_eoc)
    # the paper's own errors: ratio 4 per level at the finest levels
    l2 = g["all_floating"]["l2_error"]
    assert abs(np.log(l2[-2] / l2[-1]) / np.log(2.0) - paper_eoc) < 0.01


def test_table2_preconditioner_ordering():
    """Table 2 orders the iteration counts Dirichlet < lumped < identity at every
    level and both variants, they grow with refinement, and all-floating needs
    fewer iterations at a smaller condition number than classical FETI; the
    CPU reference FETI reproduces all three on 2^3 subdomains at two
    refinements (condition numbers from its Lanczos estimate)."""
    g = _golden("table2_linear_cube.json")
    for v in ("all_floating", "classical"):
        t = g[v]
        for lev in range(5):
            assert t["dirichlet_it"][lev] < t["lumped_it"][lev] < t["identity_it"][lev]
        for key in ("identity_it", "lumped_it", "dirichlet_it"):
            assert all(a < b for a, b in zip(t[key], t[key][1:]))
    for variant in ("af", "classical"):
        its = {}
        for n in (4, 8):
            tp = feti_ref.linear_torn_problem(cube_mesh(n, 2), variant)
            its[n] = {pc: feti_ref.FetiRef(tp, pc).solve(rtol=1e-8)["iters"]
                      for pc in ("dirichlet", "lumped", "identity")}
            assert its[n]["dirichlet"] <= its[n]["lumped"] <= its[n]["identity"], (variant, n, its[n])
        assert its[8]["lumped"] >= its[4]["lumped"] and its[8]["identity"] >= its[4]["identity"], its
    # all-floating: fewer iterations at a smaller condition number for every
    # preconditioner and level (Table 2).  The reference FETI shows the same on
    # 4^3 subdomains (interior subdomains floating in both variants, as in the
    # paper's 8^3); on 2^3 every classical subdomain touches the Dirichlet
    # boundary and none floats, which is not the paper's setting.
    for lev in range(5):
        for pc in ("identity", "lumped", "dirichlet"):
            assert g["all_floating"][pc + "_kappa"][lev] < g["classical"][pc + "_kappa"][lev]
            assert g["all_floating"][pc + "_it"][lev] < g["classical"][pc + "_it"][lev]
    m = cube_mesh(8, 4)
    kappa = {}
    for variant in ("af", "classical"):
        tp = feti_ref.linear_torn_problem(m, variant)
        kappa[variant] = {pc: feti_ref.FetiRef(tp, pc).solve(rtol=1e-8)["kappa"]
                          for pc in ("identity", "lumped", "dirichlet")}
    for pc in ("identity", "lumped", "dirichlet"):
        assert kappa["af"][pc] < kappa["classical"][pc], (pc, kappa)


def test_quadratic_cube_convergence_order():
    """The paper's cube with quadratic elements converges with order 3 in L2
    (eoc 2.97-3.01 in Table 3); the oracle's Q2 hexahedra on the Kelvin
    solution fall with the paper's finest-level order within 0.1.  The
    fixture's eoc column is also checked against its own L2 errors."""
    g = _golden("table3_quadratic_cube.json")
    for v in ("all_floating", "classical"):
        l2, eoc = g[v]["l2_error"], g[v]["eoc"]
        for lev in range(1, 4):
            assert abs(np.log(l2[lev - 1] / l2[lev]) / np.log(2.0) - eoc[lev]) < 0.02, (v, lev)
    paper_eoc = g["all_floating"]["eoc"][-1]
    from test_oracle_q2 import _l2_error_q2
    E, nu = 1.0, 0.3
    errs = []
    for n in (4, 8):
        m = cube_mesh(n, 1, E=E, nu=nu, body_force=None, order=2,
                      dirichlet_fn=lambda x: kelvin_displacement(x, E, nu))
        errs.append(_l2_error_q2(m, monolithic.solve_linear(m), lambda x: kelvin_displacement(x, E, nu)))
    eoc = np.log(errs[0] / errs[1]) / np.log(2.0)
    assert abs(eoc - paper_eoc) <= 0.1, (eoc, paper_eoc)


def test_quadratic_cube_preconditioner_ordering():
    """With quadratic elements the paper's iteration counts keep the ordering
    Dirichlet < lumped < identity at every level and both variants (Table 3);
    the CPU reference FETI on a Q2 cube in 2^3 subdomains reproduces it."""
    g = _golden("table3_quadratic_cube.json")
    for v in ("all_floating", "classical"):
        t = g[v]
        for lev in range(4):
            assert t["dirichlet_it"][lev] < t["lumped_it"][lev] < t["identity_it"][lev]
    for variant in ("af", "classical"):
        tp = feti_ref.linear_torn_problem(cube_mesh(4, 2, order=2), variant)
        its = {pc: feti_ref.FetiRef(tp, pc).solve(rtol=1e-8)["iters"] for pc in ("dirichlet", "lumped", "identity")}
        assert its["dirichlet"] <= its["lumped"] <= its["identity"], (variant, its)
