"""Admission logic of the serving loop, on the CPU with a stand-in problem.

The stand-in records the device bytes its live instances would hold, so the
tests can check what the server promises: every request is served (or
reported failed), admitted problems never hold more than the budget, idle
problems of other meshes are evicted when memory is needed, the number of
requests running at once never exceeds the worker count, and results come
back on the request that asked for them."""
import threading
import time

import numpy as np
import pytest

from paper_1508_02599_amd import serve


class _Mesh:
    """n_elem disjoint hexahedra in one subdomain: 8 n_elem nodes, which is
    all the server's footprint bound looks at."""

    def __init__(self, key, n_elem):
        self.key = key
        self.fp = 0
        self.n_sub = 1
        self.hex8 = np.arange(8 * n_elem, dtype=np.int64).reshape(n_elem, 8)
        self.elem_sub = np.zeros(n_elem, dtype=np.int32)


class _Ledger:
    def __init__(self):
        self.lock = threading.Lock()
        self.live = 0
        self.max_live = 0
        self.running = 0
        self.max_running = 0
        self.created = 0
        self.closed = 0


def _fake_problem_class(ledger):
    class FakeProblem:
        n_dof = 3

        def __init__(self, mesh, **opts):
            self.mesh = mesh
            with ledger.lock:
                ledger.live += mesh.fp
                ledger.max_live = max(ledger.max_live, ledger.live)
                ledger.created += 1

        def footprint(self):
            return self.mesh.fp

        def _work(self, value):
            with ledger.lock:
                ledger.running += 1
                ledger.max_running = max(ledger.max_running, ledger.running)
            time.sleep(0.005)
            with ledger.lock:
                ledger.running -= 1
            return np.full(self.n_dof, value)

        def factor(self):
            pass

        def solve(self, load_factor=1.0):
            return self._work(hash(self.mesh.key) % 97 + load_factor), {"iters": 1}

        def newton_step(self, U, tau):
            return self._work(-(hash(self.mesh.key) % 89) - tau), 0.0, {"iters": 2}

        def close(self):
            with ledger.lock:
                ledger.live -= self.mesh.fp
                ledger.closed += 1

    return FakeProblem


def _expected(key, kind, param):
    return (hash(key) % 97 + param) if kind == "solve" else (-(hash(key) % 89) - param)


def _stream(keys, n, seed=0):
    rng = np.random.default_rng(seed)
    out = []
    for k in range(n):
        key = keys[rng.integers(len(keys))]
        kind = "solve" if rng.random() < 0.5 else "newton"
        out.append({"t": 0.001 * k, "key": key, "kind": kind, "param": float(rng.integers(1, 9))})
    return out


def _serve(monkeypatch, sizes, budget_of, workers, stream, fp_of=None):
    """sizes: key -> elements.  A problem's footprint is 90% of the server's
    bound for its mesh (fp_of(key, bound) overrides); budget_of(bounds) gives
    the device-memory budget from the bounds."""
    ledger = _Ledger()
    monkeypatch.setattr(serve, "Problem", _fake_problem_class(ledger))
    meshes = {k: _Mesh(k, n) for k, n in sizes.items()}
    bounds = {k: serve.Server._estimate(_Probe(meshes), k) for k in sizes}
    for k, m in meshes.items():
        m.fp = fp_of(k, bounds[k]) if fp_of else int(0.9 * bounds[k])
    srv = serve.Server(lambda key: meshes[key], workers=workers, hbm_budget=budget_of(bounds))
    try:
        reqs = serve.run_stream(srv, stream)
        held = srv.held
    finally:
        srv.close()
    return reqs, ledger, held, budget_of(bounds)


class _Probe:
    """Just enough of a server for its footprint bound."""

    def __init__(self, meshes):
        self.meshes, self.est, self.options = meshes, {}, {}

    def mesh(self, key):
        return self.meshes[key]


SIZES = {("a", 1): 40, ("b", 2): 60, ("c", 3): 90}


@pytest.mark.parametrize("room,workers", [("roomy", 3), ("one_at_a_time", 3), ("one_at_a_time", 1)])
def test_every_request_served_within_budget(monkeypatch, room, workers):
    budget_of = (lambda b: 10 * sum(b.values())) if room == "roomy" else (lambda b: int(1.05 * max(b.values())))
    stream = _stream(list(SIZES), 40)
    reqs, ledger, held, budget = _serve(monkeypatch, SIZES, budget_of, workers, stream)
    assert all(r.error is None for r in reqs), [r.error for r in reqs if r.error]
    for r, s in zip(reqs, stream):
        assert r.key == s["key"]
        assert np.all(r.result == _expected(s["key"], s["kind"], s["param"]))
    assert ledger.max_live <= budget
    assert ledger.max_running <= workers
    assert ledger.live == 0 and ledger.created == ledger.closed   # close() released everything
    if room == "roomy":
        assert ledger.created <= len(SIZES) * workers   # idle problems are reused, none evicted
    else:
        assert ledger.created > len(SIZES)              # meshes alternate: idle problems were evicted
    assert held >= 0


def test_problem_larger_than_budget_is_reported(monkeypatch):
    """A mesh whose measured footprint exceeds the budget fails its requests
    with MemoryError; the other requests are still served."""
    sizes = {("small", 1): 40, ("huge", 2): 60}
    stream = [{"t": 0.0, "key": ("small", 1), "kind": "solve", "param": 1.0},
              {"t": 0.001, "key": ("huge", 2), "kind": "solve", "param": 2.0},
              {"t": 0.002, "key": ("small", 1), "kind": "newton", "param": 3.0}]
    # the huge mesh measures 10x its bound once set up
    reqs, ledger, _, _ = _serve(monkeypatch, sizes, lambda b: 2 * max(b.values()), 2, stream,
                                fp_of=lambda k, b: 10 * b if k[0] == "huge" else int(0.9 * b))
    assert reqs[1].error is not None and "MemoryError" in reqs[1].error
    assert reqs[0].error is None and reqs[2].error is None
    assert ledger.live == 0
