"""Full-size workloads on the GPU, checked against the oracle.

Displacement parity uses oracle solutions computed once on the CPU by
tests/golden/make_fullsize_refs.py (the 40^3 uneven-box cube, whose boxes are
as large as those of the 64^3 workload, and the full 16x128x64 tube).  For
the 824k-DOF uneven-box cube the direct solve is out of reach, so the check
there is nodal equilibrium: at 300 sampled nodes the oracle
assembles the rows of the linear(ised) system from the elements and pressure
faces around each node and evaluates them at the GPU's displacements.  The
componentwise relative residual |r| / (sum of the magnitudes of the terms)
must be small; Dirichlet DOFs must carry their prescribed values exactly.
"""
import numpy as np
import pytest

from oracle import fem
from workloads import config_mesh

pytestmark = pytest.mark.gpu


def _problem(mesh, **kw):
    from paper_1508_02599_amd.feti import Problem
    return Problem(mesh, **kw)


def _sampled_residual(mesh, u, U=None, tau=1.0, n=300, seed=0):
    rng = np.random.default_rng(seed)
    nodes = rng.choice(mesh.n_nodes, n, replace=False)
    res, sc = fem.nodal_residual(mesh, nodes, u, U=U, tau=tau)
    return float((np.abs(res) / sc).max())


_MESH = {}


def _mesh(name):
    if name not in _MESH:
        _MESH[name] = config_mesh(name)
    return _MESH[name]


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_random_boxes_full_size(precision):
    """64^3 cube cut into 512 uneven boxes (630-5577 DOFs), all-floating,
    lumped preconditioner, every subdomain in one batch."""
    m = _mesh("random_boxes_64")
    kw = dict(rtol=1e-10) if precision == "fp64" else dict(rtol=1e-6, ir_tol=1e-10)
    with _problem(m, variant="af", precond="lumped", precision=precision, max_it=3000, **kw) as p:
        p.factor()
        u, st = p.solve()
        fp = p.footprint()
    rr = _sampled_residual(m, u)
    dir_err = float(np.abs(u[m.dir_dof] - m.dir_val).max())
    print(f"random boxes {precision}: subs={m.n_sub} dofs={m.n_dofs} it={st['iters']} "
          f"sweeps={st['ir_sweeps']} nodal res={rr:.2e} t_factor={st['t_factor']:.3f} "
          f"t_pcg={st['t_pcg']:.3f} device={fp / 2**30:.1f} GiB")
    assert st["converged"] == 1
    assert dir_err == 0.0
    assert rr <= 1e-8


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_tube_full_size_newton_step(precision):
    """Two-layer HGO tube, 16x128x64 Q1-P0 elements in 128 subdomains: the first
    Newton step of the first load step (tau = 0.1) from rest."""
    m = _mesh("tube_16x128x64")
    U = np.zeros(m.n_dofs)
    kw = dict(rtol=1e-10) if precision == "fp64" else dict(rtol=1e-6, ir_tol=1e-10, ir_max=10)
    with _problem(m, variant="af", precond="dirichlet", precision=precision, max_it=10000, **kw) as p:
        dU, rn, st = p.newton_step(U, 0.1)
    rr = _sampled_residual(m, dU, U=U.reshape(-1, 3), tau=0.1)
    print(f"tube full {precision}: dofs={m.n_dofs} it={st['iters']} sweeps={st['ir_sweeps']} "
          f"res0={rn:.4e} nodal res={rr:.2e} t_factor={st['t_factor']:.3f} t_pcg={st['t_pcg']:.3f}")
    assert st["converged"] == 1
    assert rr <= 1e-8


def test_tube_q2_full_size_exact_newton_step():
    """The same tube with 8x64x32 Q2-P0 elements (27-node hexahedra, the same
    424,320 DOFs and 128 subdomains): the exact Newton step (follower-load
    stiffness) of the first load step from rest, classical FETI with the
    Dirichlet preconditioner, against the oracle's element rows at sampled
    nodes."""
    m = _mesh("tube_q2_8x64x32")
    U = np.zeros(m.n_dofs)
    tau = 1.0 / 40.0
    with _problem(m, variant="classical", precond="dirichlet", rtol=1e-10, ir_tol=1e-11, ir_max=60,
                  max_it=10000, load_stiffness=True) as p:
        dU, rn, st = p.newton_step(U, tau)
    # the oracle's rows of the exact linearisation: K' dU - tau dfp/dU dU = r
    from oracle import fem
    rng = np.random.default_rng(0)
    nodes = np.sort(rng.choice(m.n_nodes, size=200, replace=False))
    res, scale = fem.nodal_residual(m, nodes, dU, U=U.reshape(-1, 3), tau=tau)
    D = fem.assemble_load_stiffness(m, U.reshape(-1, 3))
    corr = tau * (D @ dU).reshape(-1, 3)[nodes]
    dm = np.zeros(m.n_dofs, dtype=bool)
    dm[m.dir_dof] = True
    corr[dm.reshape(-1, 3)[nodes]] = 0.0
    rr = float(np.max(np.abs(res + corr) / np.maximum(scale, 1e-300)))
    print(f"tube q2 full: dofs={m.n_dofs} it={st['iters']} sweeps={st['ir_sweeps']} res0={rn:.4e} "
          f"nodal res={rr:.2e} t_factor={st['t_factor']:.3f} t_pcg={st['t_pcg']:.3f}")
    assert rr <= 1e-8


# ---------------------------------------------------------------- displacement parity at full size
def _reference(case, mesh, *extra):
    """Oracle displacements written by tests/golden/make_fullsize_refs.py for
    exactly this input (the key hashes the mesh, loads and state)."""
    import importlib.util
    import os
    here = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "make_fullsize_refs.py")
    spec = importlib.util.spec_from_file_location("make_fullsize_refs", here)
    mk = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mk)
    path = mk.path_for(case, mk.fullsize_key(mesh, *extra))
    if not os.path.exists(path):
        pytest.skip(f"no oracle reference {os.path.basename(path)} (run tests/golden/make_fullsize_refs.py)")
    return np.load(path), mk


def _errs(u, ref):
    l2 = float(np.linalg.norm(u - ref) / np.linalg.norm(ref))
    li = float(np.abs(u - ref).max() / np.abs(ref).max())
    return l2, li


@pytest.mark.parametrize("precision,rtol", [("fp64", 1e-11), ("fp64", 1e-8), ("mixed", 1e-8)])
def test_uneven_boxes_displacement_parity(precision, rtol):
    """40^3 cube in 5^3 uneven boxes of 450-5616 DOFs (the box sizes of the
    64^3 workload) against the oracle's sparse direct solution, in both the
    2-norm and element-wise: <= 1e-9 for FP64 at rtol 1e-11, <= 1e-8 for mixed
    after refinement; at the benchmark's rtol 1e-8 the FP64 error (about 2e-8
    in the 2-norm, 1e-7 element-wise) is reported and bounded by 1e-6."""
    m = _mesh("random_boxes_40")
    ref, _ = _reference("random_boxes_40", m)
    kw = dict(ir_tol=1e-10) if precision == "mixed" else {}
    with _problem(m, variant="af", precond="lumped", precision=precision, rtol=rtol, max_it=3000, **kw) as p:
        p.factor()
        u, st = p.solve()
    l2, li = _errs(u, ref)
    print(f"random_boxes_40 {precision} rtol {rtol:g}: it={st['iters']} sweeps={st['ir_sweeps']} "
          f"err l2={l2:.2e} max={li:.2e}")
    bar = 1e-6 if (precision == "fp64" and rtol > 1e-10) else (1e-9 if precision == "fp64" else 1e-8)
    assert max(l2, li) <= bar


@pytest.mark.parametrize("step", [0, 1])
def test_tube_full_size_step_displacement_parity(step):
    """The 16x128x64 tube (424k DOFs, 128 all-floating subdomains): the first
    Newton step from rest at load factor 1/40, and the step at
    U_1 = U_0 + dU_0 / 4 (a stressed state), against the oracle's sparse
    direct Newton steps (<= 1e-9).  At the stressed state the rotations of
    small stress-induced stiffness join the kernels (an approximate tangent,
    refined by flexible GMRES against the exact one) and the dual problem is
    solved by projected GMRES.  The refinement's target 1e-11 sits above the
    rounding floor of the assembled residual there (about 1.2e-12 of |b|)."""
    m = _mesh("tube_16x128x64")
    U = np.zeros(m.n_dofs)
    ref0, mk = _reference("tube_step0", m, U, np.array([1.0 / 40.0]))
    tau = mk.TUBE_TAU
    if step == 1:
        U = U + mk.STEP1_SCALE * ref0
        ref, _ = _reference("tube_step1", m, U, np.array([tau]))
    else:
        ref = ref0
    kw = dict(dual_gmres=True, kernel_tol=1e-6, ir_tol=1e-11, ir_max=60) if step == 1 else {}
    with _problem(m, variant="af", precond="dirichlet", rtol=1e-10, max_it=10000, **kw) as p:
        dU, rn, st = p.newton_step(U, tau)
    l2, li = _errs(dU, ref)
    print(f"tube full step {step}: it={st['iters']} sweeps={st['ir_sweeps']} err l2={l2:.2e} max={li:.2e} "
          f"t_factor={st['t_factor']:.3f} t_pcg={st['t_pcg']:.3f}")
    assert max(l2, li) <= 1e-9
