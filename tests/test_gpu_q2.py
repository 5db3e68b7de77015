"""Parity of the HIP FETI path on Q2 (27-node) hexahedra against the CPU
oracle, through the C ABI: linear cubes (both variants, every
preconditioner, FP64 and mixed precision), the exact reproduction of a
quadratic displacement field, and Newton steps of the Q2-P0 HGO tube (from
rest, from a stressed equilibrium, the exact step with the follower-load
stiffness in FP64 and mixed precision, and a converged load path at the
benchmark's settings).  Errors are max(relative 2-norm, element-wise max relative to
max|u_ref|), as in the Q1 parity tests."""
import numpy as np
import pytest

from oracle import fem, monolithic
from workloads import cube_mesh, tube_mesh

pytestmark = pytest.mark.gpu


def _problem(mesh, **kw):
    from paper_1508_02599_amd.feti import Problem
    return Problem(mesh, **kw)


def _rel(u, ref):
    l2 = float(np.linalg.norm(u - ref) / np.linalg.norm(ref))
    li = float(np.max(np.abs(u - ref)) / np.max(np.abs(ref)))
    return max(l2, li)


_REF = {}


def _cube(n_el, m):
    """Q2 cube of n_el^3 elements in m^3 subdomains with per-subdomain
    Poisson ratios (seeded) and its monolithic solution."""
    key = (n_el, m)
    if key not in _REF:
        nu = 0.25 + 0.1 * np.random.default_rng(0).random(m ** 3)
        mesh = cube_mesh(n_el, m, nu_per_sub=nu, order=2)
        _REF[key] = (mesh, monolithic.solve_linear(mesh))
    return _REF[key]


@pytest.mark.parametrize("variant", ["af", "classical"])
@pytest.mark.parametrize("precond", ["lumped", "dirichlet", "identity"])
def test_q2_cube_parity(variant, precond):
    """4^3 Q2 elements in 2^3 subdomains (375 DOFs each: six tiles, a ragged
    tail)."""
    m, ref = _cube(4, 2)
    with _problem(m, variant=variant, precond=precond, rtol=1e-11) as p:
        p.factor()
        u, st = p.solve()
    err = _rel(u, ref)
    print(f"q2 cube4 {variant} {precond}: it={st['iters']} err={err:.3e}")
    assert st["converged"] == 1
    assert err <= 1e-9


@pytest.mark.parametrize("variant,precond,precision", [("af", "dirichlet", "fp64"), ("classical", "lumped", "fp64"),
                                                       ("af", "dirichlet", "mixed")])
def test_q2_cube_many_tiles_parity(variant, precond, precision):
    """8^3 Q2 elements in 2^3 subdomains: 2,187 DOFs per subdomain (35 tiles,
    ragged tail of 11), 14,739 DOFs in all."""
    m, ref = _cube(8, 2)
    kw = dict(rtol=1e-11) if precision == "fp64" else dict(precision="mixed", rtol=1e-8, ir_tol=1e-12, ir_max=30)
    with _problem(m, variant=variant, precond=precond, **kw) as p:
        p.factor()
        u, st = p.solve()
    err = _rel(u, ref)
    print(f"q2 cube8 {variant} {precond} {precision}: it={st['iters']} err={err:.3e}")
    assert err <= (1e-9 if precision == "fp64" else 1e-8)


def test_q2_quadratic_field_exact_through_feti():
    """A quadratic displacement with the constant body force it needs is in
    the Q2 space: the FETI solution on boxes of unequal sizes equals it at
    every node (checked against the closed form, not the oracle)."""
    E, nu = 2.0, 0.3
    lam, mu = fem.lame(E, nu)
    rng = np.random.default_rng(4)
    Q = 0.05 * rng.standard_normal((3, 3, 3))
    Q = 0.5 * (Q + Q.transpose(0, 2, 1))
    div_grad = np.einsum("jji->i", 2.0 * Q)
    lap = 2.0 * np.einsum("ijj->i", Q)
    b = -(lam * div_grad + mu * (lap + div_grad))
    m = cube_mesh(4, 2, E=E, nu=nu, body_force=tuple(b), order=2)
    m.xyz = np.interp(m.xyz, [0.0, 0.25, 0.5, 0.75, 1.0], [0.0, 0.2, 0.55, 0.7, 1.0])
    ue = np.einsum("ijk,nj,nk->ni", Q, m.xyz, m.xyz)
    m.dir_val = ue[m.dir_dof // 3, m.dir_dof % 3]
    for variant in ("af", "classical"):
        with _problem(m, variant=variant, precond="dirichlet", rtol=1e-12) as p:
            p.factor()
            u, st = p.solve()
        err = _rel(u, ue.reshape(-1))
        print(f"q2 quadratic field {variant}: it={st['iters']} err={err:.3e}")
        assert err <= 1e-9


def _q2_tube():
    return tube_mesh(nr=1, nth=16, nz=4, sub=(1, 4, 2), order=2)


@pytest.mark.parametrize("variant", ["af", "classical"])
def test_q2_tube_newton_step_from_rest(variant):
    m = _q2_tube()
    U = np.zeros(m.n_dofs)
    dU_ref, rn_ref = monolithic.newton_increment(m, U, 0.05)
    with _problem(m, variant=variant, precond="dirichlet", rtol=1e-12) as p:
        dU, rn, st = p.newton_step(U, 0.05)
    err = _rel(dU, dU_ref)
    print(f"q2 tube newton {variant} from rest: it={st['iters']} err={err:.3e} res={rn:.6e}/{rn_ref:.6e}")
    assert abs(rn - rn_ref) <= 1e-10 * rn_ref
    assert err <= 1e-9


@pytest.mark.parametrize("variant", ["af", "classical"])
def test_q2_tube_exact_newton_steps(variant):
    """Exact Newton steps (follower-load stiffness, flexible GMRES on the
    assembled operator) of the Q2-P0 tube: from rest, and from the equilibrium
    of the first load step (tau = 1/40) to the second (tau = 2/40)."""
    m = _q2_tube()
    U1 = np.zeros(m.n_dofs)
    for _ in range(20):
        dU, rn = monolithic.newton_increment(m, U1, 1 / 40, load_stiffness=True)
        U1 = U1 + dU
        if rn < 1e-11:
            break
    for step, (U, tau) in enumerate([(np.zeros(m.n_dofs), 1 / 40), (U1, 2 / 40)]):
        dU_ref, rn_ref = monolithic.newton_increment(m, U, tau, load_stiffness=True)
        with _problem(m, variant=variant, precond="dirichlet", rtol=1e-8, ir_tol=1e-12, ir_max=60,
                      load_stiffness=True) as p:
            dU, rn, st = p.newton_step(U, tau)
        err = _rel(dU, dU_ref)
        print(f"q2 exact newton {variant} step {step}: it={st['iters']} gmres={st['ir_sweeps']} "
              f"coarse={st['n_coarse']} err={err:.3e}")
        assert abs(rn - rn_ref) <= 1e-9 * rn_ref
        assert err <= 1e-9


def test_q2_tube_exact_newton_mixed():
    """Mixed precision (FP32 local factors, FP64 refinement) on the exact
    Newton step of the Q2-P0 tube from rest: the oracle's step to 1e-8."""
    m = _q2_tube()
    U = np.zeros(m.n_dofs)
    dU_ref, rn_ref = monolithic.newton_increment(m, U, 1 / 40, load_stiffness=True)
    with _problem(m, variant="af", precond="dirichlet", precision="mixed", rtol=1e-8, ir_tol=1e-10, ir_max=60,
                  load_stiffness=True) as p:
        dU, rn, st = p.newton_step(U, 1 / 40)
    err = _rel(dU, dU_ref)
    print(f"q2 exact newton mixed: it={st['iters']} gmres={st['ir_sweeps']} err={err:.3e}")
    assert abs(rn - rn_ref) <= 1e-9 * rn_ref
    assert err <= 1e-8


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_q2_converged_load_path_parity(precision):
    """The Q2-P0 tube's load path at the benchmark's settings (classical,
    Dirichlet preconditioner, exact Newton steps, kernel tolerance 1e-6,
    projected dual GMRES, warm starts, inexact Newton forcing; mixed: FP32
    local factors, first dual solves to 1e-6) ends every load step at the
    equilibrium the oracle's Newton iteration finds."""
    import sys
    import torch
    from paper_1508_02599_amd.feti import Problem
    from paper_1508_02599_amd.loadpath import run_load_path
    m = tube_mesh(nr=1, nth=16, nz=4, sub=(1, 4, 4), order=2)   # end rings clamped, middle rings floating
    n_inc, n_steps = 160, 4
    ref, U = {}, np.zeros(m.n_dofs)
    for s in range(1, n_steps + 1):
        r0 = None
        for _ in range(30):
            dU, rn = monolithic.newton_increment(m, U, s / n_inc, load_stiffness=True)
            r0 = rn if r0 is None else r0
            if rn <= 1e-10 * r0:
                break
            U = U + dU
        ref[s] = U.copy()
    got = {}

    def record(tau, k, Uk):
        got[round(tau * n_inc, 9)] = Uk.double().cpu().numpy()

    rtol = 1e-10 if precision == "fp64" else 1e-6
    with Problem(m, variant="classical", precond="dirichlet", precision=precision, rtol=rtol, ir_tol=1e-3,
                 ir_max=60, max_it=3000, device_ptrs=True, load_stiffness=True, warm_start=True, dual_gmres=True,
                 kernel_tol=1e-6) as p:
        Ug = torch.zeros(m.n_dofs, dtype=torch.float64, device="cuda")
        r = run_load_path(p, Ug, n_inc, rtol=rtol, newton_tol=1e-9, tau_end=n_steps / n_inc, record=record,
                          log=sys.stdout)
    assert r["error"] is None and abs(r["tau_reached"] - n_steps / n_inc) < 1e-12, r["error"]
    errs = [_rel(got[float(s)], ref[s]) for s in range(1, n_steps + 1)]
    for s, err in zip(range(1, n_steps + 1), errs):
        print(f"q2 load step {s} {precision}: Newton steps {r['newton_per_load'][s - 1]}, error {err:.3e}")
    assert max(errs) <= 1e-8


@pytest.mark.parametrize("variant", ["classical", "af"])
def test_q2_partial_kernels_parity(variant):
    """Q2 cube of 4^3 elements in 2^3 boxes (the node grid of the 8^3 Q1 cube)
    clamped on a quarter face with a roller face: classical subdomains that
    touch the Dirichlet boundary at a vertex, along an edge or in one
    component keep their partial kernels (section 4.3), the same 17 coarse
    columns as on the Q1 cube; the displacements match the direct solve."""
    from workloads import partial_dirichlet_cube
    m = partial_dirichlet_cube(4, 2, order=2)
    ref = monolithic.solve_linear(m)
    with _problem(m, variant=variant, precond="dirichlet", rtol=1e-11) as p:
        p.factor()
        u, st = p.solve()
    err = _rel(u, ref)
    print(f"q2 partial kernels {variant}: it={st['iters']} coarse={st['n_coarse']} err={err:.3e}")
    assert st["n_coarse"] == (17 if variant == "classical" else 48)
    assert err <= 1e-9
