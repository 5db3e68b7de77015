"""Host logic of the load path (paper_1508_02599_amd.loadpath) on the CPU,
with a one-DOF nonlinear stand-in for the FETI problem: the equilibrium
tau f = g(U), g(U) = U + U^3, solved by exact Newton steps.  Checks the
inexact-Newton forcing terms, that every accepted load step ends at its
equilibrium, that a failing increment is halved and regrows after two
accepted steps, and the error once the increment falls below 1/64 of the
nominal one."""
import numpy as np
import pytest
import torch

from paper_1508_02599_amd.feti import FETI_ENOTSPD, FetiError
from paper_1508_02599_amd.loadpath import run_load_path

F = 3.0


def g(u):
    return u + u ** 3


class OneDof:
    """newton_step(U, tau): residual r = tau F - g(U) at U (returned as its
    norm) and the exact Newton increment r / g'(U) written to `out`.
    fail(U, tau) -> True raises ENOTSPD, as a failing local factor would."""

    def __init__(self, fail=None):
        self.fail = fail
        self.tolerances = []
        self.calls = 0

    def set_tolerances(self, rtol, eta):
        self.tolerances.append((rtol, eta))

    def newton_step(self, U, tau, out=None, allow_noconv=False):
        self.calls += 1
        u = float(U[0])
        if self.fail is not None and self.fail(u, tau):
            raise FetiError(FETI_ENOTSPD, "non-positive pivot in the local factor of subdomain 0")
        r = tau * F - g(u)
        out[0] = r / (1.0 + 3.0 * u * u)
        return out, abs(r), {"iters": 1, "ir_sweeps": 0, "modified_pivots": 0}


@pytest.fixture(autouse=True)
def _no_device_sync(monkeypatch):
    monkeypatch.setattr(torch.cuda, "synchronize", lambda *a, **k: None)


def _equilibrium(tau):
    """The real root of U^3 + U - tau F (g is strictly increasing)."""
    roots = np.roots([1.0, 0.0, 1.0, -tau * F])
    return float(roots[np.abs(roots.imag) < 1e-12].real[0])


def test_path_reaches_the_end_at_every_equilibrium():
    p = OneDof()
    U = torch.zeros(1, dtype=torch.float64)
    seen = {}

    def record(tau, k, Uk):
        seen.setdefault(round(tau, 12), []).append(float(Uk[0]))

    r = run_load_path(p, U, 10, newton_tol=1e-10, eta_max=1e-3, record=record, log=None)
    assert r["error"] is None and abs(r["tau_reached"] - 1.0) < 1e-12
    assert r["rejected_steps"] == 0 and r["cuts"] == 0
    assert r["taus"] == pytest.approx([0.1 * s for s in range(1, 11)])
    for tau in r["taus"]:
        its = seen[round(tau, 12)]
        assert abs(its[-1] - _equilibrium(tau)) < 1e-9    # the last iterate is the equilibrium
    assert abs(float(U[0]) - _equilibrium(1.0)) < 1e-9
    # Newton converges quadratically: a handful of steps per load step
    assert max(r["newton_per_load"]) <= 6
    # forcing terms: the first step of a load step gets eta_max, all within (0, eta_max]
    etas = [e for _, e in p.tolerances]
    assert etas[0] == 1e-3 and all(0.0 < e <= 1e-3 for e in etas)


def test_failing_increments_are_halved_and_regrow():
    """Above tau = 0.5 an increment larger than 0.03 beyond the state's own
    load fails; the nominal increment is 0.05, so it is halved to 0.025, and
    after two accepted steps doubled back (and halved again)."""
    p = OneDof(fail=lambda u, tau: tau > 0.5 and tau - g(u) / F > 0.03)
    U = torch.zeros(1, dtype=torch.float64)
    r = run_load_path(p, U, 20, newton_tol=1e-10, log=None)
    assert r["error"] is None and abs(r["tau_reached"] - 1.0) < 1e-12
    # each rejection fails at its first factorisation: no Newton step of a
    # rejected load step completes (rejected_steps counts those)
    assert r["cuts"] > 0 and r["rejected_steps"] == 0
    inc = np.diff([0.0] + r["taus"])
    assert np.all(inc <= 0.05 + 1e-12)
    assert np.all(inc[np.array(r["taus"]) > 0.5 + 0.05 + 1e-12] <= 0.025 + 1e-12)
    assert abs(float(U[0]) - _equilibrium(1.0)) < 1e-9


def test_increment_below_the_floor_is_an_error():
    p = OneDof(fail=lambda u, tau: tau > 0.5)
    U = torch.zeros(1, dtype=torch.float64)
    r = run_load_path(p, U, 10, newton_tol=1e-10, log=None)
    assert r["error"] is not None and "1/64" in r["error"]
    assert abs(r["tau_reached"] - 0.5) < 1e-12
    # the state stays at the last equilibrium
    assert abs(float(U[0]) - _equilibrium(0.5)) < 1e-9
