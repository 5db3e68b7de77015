"""Full-size workloads on the GPU, checked against the oracle's element
routines at sampled nodes.

The direct solve of the oracle is out of reach at these sizes (824k and 424k
DOFs), so the check is nodal equilibrium: at 300 sampled nodes the oracle
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
