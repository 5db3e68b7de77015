"""feti_solve_noalloc (the solve whose dual-iteration scratch lives in the
library's static device array) against feti_solve, through the C ABI: two
calls in a row on different problems, the second one smaller, each equal to
feti_solve on the same factors, bit for bit (same kernels, same order)."""
import numpy as np
import pytest

from workloads import cube_mesh, config_mesh

pytestmark = pytest.mark.gpu


def _run(mesh, **kw):
    import torch
    from paper_1508_02599_amd.feti import Problem
    u_ref = torch.empty(mesh.n_dofs, dtype=torch.float64, device="cuda")
    u_na = torch.full((mesh.n_dofs,), float("nan"), dtype=torch.float64, device="cuda")
    with Problem(mesh, device_ptrs=True, **kw) as p:
        p.factor()
        _, st_ref = p.solve(out=u_ref)
        _, st_na = p.solve_noalloc(u_na)
        torch.cuda.synchronize()
        # the regular path still works after a call on the static array
        u_again = torch.empty_like(u_ref)
        p.solve(out=u_again)
        torch.cuda.synchronize()
    return u_ref.cpu().numpy(), u_na.cpu().numpy(), u_again.cpu().numpy(), st_ref, st_na


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_noalloc_matches_solve_twice_second_smaller(precision):
    from oracle import monolithic
    big = cube_mesh(16, 2, nu=0.28)
    small = config_mesh("cube8_s2")
    kw = dict(rtol=1e-10, precision=precision, variant="af", precond="lumped")
    for mesh in (big, small):
        u_ref, u_na, u_again, st_ref, st_na = _run(mesh, **kw)
        assert st_na["converged"] == 1 and st_na["iters"] == st_ref["iters"]
        assert np.array_equal(u_na, u_ref)
        assert np.array_equal(u_again, u_ref)
        ref = monolithic.solve_linear(mesh)
        err = max(np.linalg.norm(u_na - ref) / np.linalg.norm(ref),
                  np.abs(u_na - ref).max() / np.abs(ref).max())
        print(f"noalloc {precision} n_dofs={mesh.n_dofs}: it={st_na['iters']} err={err:.2e}")
        assert err <= (1e-9 if precision == "fp64" else 1e-8)


def test_noalloc_rejects_host_output_and_large_max_it():
    import torch
    from paper_1508_02599_amd.feti import Problem, FetiError, FETI_EINVAL
    m = config_mesh("cube8_s2")
    with Problem(m, device_ptrs=True, max_it=9000) as p:
        p.factor()
        u = torch.empty(m.n_dofs, dtype=torch.float64, device="cuda")
        with pytest.raises(FetiError) as ei:
            p.solve_noalloc(u)
        assert ei.value.status == FETI_EINVAL and "max_it" in str(ei.value)
    with Problem(m) as p:
        p.factor()
        import ctypes as C
        from paper_1508_02599_amd.feti import feti_stats
        st = p.lib.feti_solve_noalloc(p.h, 1.0, np.zeros(m.n_dofs).ctypes.data_as(C.c_void_p),
                                      C.byref(feti_stats()))
        assert st == FETI_EINVAL
