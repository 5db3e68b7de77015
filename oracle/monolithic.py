"""The plain definition of what FETI computes: one global sparse FP64 solve.

Oracle module (test infrastructure only).  Section 4 of the paper states the
FETI systems (eqs. (classicalFetiLGS) and (AFFETI)) as exact reformulations of
the assembled system (eq. (reordered)), itself the Newton linearisation of
eq. (LGS).  The oracle therefore assembles the global tangent, eliminates the
Dirichlet degrees of freedom and solves with a sparse direct factorisation:
SciPy's SuperLU in symmetric mode with no pivoting, which for an SPD matrix is
a Cholesky-equivalent LDL^T factorisation.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse.linalg as spla

from . import fem


def sparse_lu_solve(A, b):
    """Direct solve of a general sparse system (partial pivoting)."""
    return spla.splu(A.tocsc()).solve(b)


def sparse_spd_solve(A, b):
    """Direct solve of a sparse SPD system (no pivoting, symmetric ordering)."""
    lu = spla.splu(A.tocsc(), permc_spec="MMD_AT_PLUS_A", diag_pivot_thresh=0.0,
                   options=dict(SymmetricMode=True))
    return lu.solve(b)


def solve_with_dirichlet(K, rhs, dir_dof, dir_inc, symmetric=True):
    """Solve K x = rhs on the free DOFs with x = dir_inc on ``dir_dof``
    (``symmetric``: K is SPD; otherwise a pivoted sparse LU)."""
    n = K.shape[0]
    x = np.zeros(n)
    x[dir_dof] = dir_inc
    free = np.ones(n, dtype=bool)
    free[dir_dof] = False
    fi = np.nonzero(free)[0]
    Kff = K[fi][:, fi]
    b = rhs[fi] - K[fi][:, dir_dof] @ x[dir_dof]
    x[fi] = sparse_spd_solve(Kff, b) if symmetric else sparse_lu_solve(Kff, b)
    return x


def solve_linear(mesh, load_factor=1.0):
    """Displacements of a linear problem: K u = lf f_ext, u = lf u_D on Gamma_D.

    Returns the global DOF vector [3*n_nodes].
    """
    K, _, f = fem.assemble(mesh, None, tau=load_factor)
    return solve_with_dirichlet(K, f, mesh.dir_dof, load_factor * mesh.dir_val)


def newton_increment(mesh, U, tau, load_stiffness=False):
    """One Newton increment (eqs. (LGS), (loadStepping)).

    K'(U) dU = tau f_ext(U) - f_int(U) on the free DOFs, dU = tau u_D - U on
    Gamma_D.  The follower pressure acts on the current geometry.  As in the
    paper its load stiffness is neglected by default; with ``load_stiffness``
    the exact linearisation (K'(U) - tau d f_p / dU) dU = tau f_ext - f_int is
    solved instead, the non-symmetric system the paper mentions (section 3.2,
    last paragraph).  Returns (dU, ||residual||_2 on free DOFs).
    """
    U = np.asarray(U, dtype=np.float64).reshape(-1)
    K, f_int, f_ext = fem.assemble(mesh, U.reshape(-1, 3), tau=tau)
    r = f_ext - f_int
    free = np.ones(mesh.n_dofs, dtype=bool)
    free[mesh.dir_dof] = False
    inc = tau * mesh.dir_val - U[mesh.dir_dof]
    if load_stiffness:
        K = (K - tau * fem.assemble_load_stiffness(mesh, U)).tocsr()
    dU = solve_with_dirichlet(K, r, mesh.dir_dof, inc, symmetric=not load_stiffness)
    return dU, float(np.linalg.norm(r[free]))


def residual_norm(mesh, U, tau):
    """(||tau f_ext(U) - f_int(U)||_2, ||tau f_ext(U)||_2) over the free DOFs."""
    U = np.asarray(U, dtype=np.float64).reshape(-1)
    _, f_int, f_ext = fem.assemble(mesh, U.reshape(-1, 3), tau=tau)
    free = np.ones(mesh.n_dofs, dtype=bool)
    free[mesh.dir_dof] = False
    return float(np.linalg.norm((f_ext - f_int)[free])), float(np.linalg.norm(f_ext[free]))
