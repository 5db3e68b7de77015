"""Error paths of the C ABI on the GPU: each condition is forced from the host
(an iteration cap, a call out of order, inverted elements), so every kernel
still runs to its normal end; the call returns the documented status.
"""
import ctypes as C

import numpy as np
import pytest

from workloads import config_mesh

pytestmark = pytest.mark.gpu


def _feti():
    from paper_1508_02599_amd import feti
    return feti


def test_enoconv_writes_u():
    """max_it = 1: FETI_ENOCONV, stats.converged = 0, and u is still written
    (finite, Dirichlet DOFs at their prescribed values)."""
    feti = _feti()
    m = config_mesh("cube8_s2")
    with feti.Problem(m, max_it=1, rtol=1e-12) as p:
        p.factor()
        u = np.full(m.n_dofs, np.nan)
        stats = feti.feti_stats()
        st = p.lib.feti_solve(p.h, 1.0, u.ctypes.data_as(C.c_void_p), C.byref(stats))
        assert st == feti.FETI_ENOCONV
        assert stats.converged == 0 and stats.iters == 1
        assert np.all(np.isfinite(u))
        assert np.all(u[m.dir_dof] == m.dir_val)
        assert "max_it" in p.lib.feti_last_error(p.h).decode()


def test_estate_solve_before_factor():
    feti = _feti()
    m = config_mesh("cube8_s2")
    with feti.Problem(m) as p:
        with pytest.raises(feti.FetiError) as ei:
            p.solve()
        assert ei.value.status == feti.FETI_ESTATE


@pytest.mark.parametrize("variant", ["af", "classical"])
def test_enotspd_names_the_subdomain(variant):
    """Subdomain 5 of the 2^3 cube with every element's corner order mirrored
    (negative Jacobian): its local stiffness is negative definite, the factor
    meets a negative pivot and the message names subdomain 5.  A solve after
    the failed factorisation reports FETI_ESTATE."""
    feti = _feti()
    m = config_mesh("cube8_s2")
    bad = m.hex8.copy()
    sel = m.elem_sub == 5
    bad[sel] = bad[sel][:, [1, 0, 3, 2, 5, 4, 7, 6]]
    m.hex8 = bad
    with feti.Problem(m, variant=variant, precond="dirichlet") as p:
        with pytest.raises(feti.FetiError) as ei:
            p.factor()
        assert ei.value.status == feti.FETI_ENOTSPD
        assert "subdomain 5" in str(ei.value)
        with pytest.raises(feti.FetiError) as ei:
            p.solve()
        assert ei.value.status == feti.FETI_ESTATE
