"""Pins of the CPU oracle against facts fixed by the paper and by mathematics.

Each test pins one part of the oracle so that a plausible mistake (a dropped
term, a wrong sign, a transposed index) fails at least one of them:
closed forms, invariants, special cases, brute force on tiny inputs and the
convergence order the paper reports.
"""
import numpy as np
import pytest

from oracle import fem, monolithic, feti_ref
from workloads import cube_mesh, kelvin_displacement, tube_mesh, config_mesh


def _affine_element(seed=0):
    rng = np.random.default_rng(seed)
    A = np.eye(3) + 0.3 * rng.standard_normal((3, 3))
    if np.linalg.det(A) < 0:
        A[:, 0] *= -1
    X = (fem.XI + 1.0) * 0.5 @ A.T + rng.standard_normal(3)
    return X, abs(np.linalg.det(A))


def _distorted_element(seed=1):
    rng = np.random.default_rng(seed)
    X = (fem.XI + 1.0) * 0.5 + 0.08 * rng.standard_normal((8, 3))
    return X


# ---------------------------------------------------------------- Q1 linear
def test_q1_rigid_modes_span_kernel():
    """K_e annihilates the six rigid motions and has rank 24 - 6 = 18."""
    X = _distorted_element()
    lam, mu = fem.lame(1.0, 0.3)
    K = fem.linear_stiffness(X[None], lam, mu)[0]
    R = feti_ref.rigid_modes(X)
    assert np.allclose(K, K.T, atol=1e-14)
    assert np.linalg.norm(K @ R) <= 1e-13 * np.linalg.norm(K) * np.linalg.norm(R)
    ev = np.linalg.eigvalsh(K)
    assert np.sum(ev < 1e-10 * ev[-1]) == 6
    assert ev[6] > 1e-6 * ev[-1]


def test_q1_uniform_strain_energy_closed_form():
    """For u = A x the energy u^T K u equals V (lam tr(eps)^2 + 2 mu eps:eps)."""
    X, vol = _affine_element()
    lam, mu = fem.lame(2.5, 0.27)
    K = fem.linear_stiffness(X[None], lam, mu)[0]
    rng = np.random.default_rng(3)
    A = rng.standard_normal((3, 3))
    u = (X @ A.T).reshape(-1)
    eps = 0.5 * (A + A.T)
    exact = vol * (lam * np.trace(eps) ** 2 + 2 * mu * np.sum(eps * eps))
    assert abs(u @ K @ u - exact) <= 1e-12 * abs(exact)


def test_body_force_total():
    """Nodal forces of a constant body force sum to b * volume."""
    X, vol = _affine_element(5)
    b = np.array([[0.3, -1.0, 2.0]])
    f = fem.body_force_vector(X[None], b)[0].reshape(8, 3)
    assert np.allclose(f.sum(axis=0), b[0] * vol, rtol=1e-13)


def _perturbed_cube(n, seed=0):
    m = cube_mesh(n, 1, body_force=None)
    rng = np.random.default_rng(seed)
    x = m.xyz.copy()
    inner = np.all((x > 1e-12) & (x < 1 - 1e-12), axis=1)
    x[inner] += 0.15 / n * rng.uniform(-1, 1, size=(inner.sum(), 3))
    m.xyz = x
    return m


def test_patch_test_monolithic():
    """Linear displacement data on a distorted mesh is reproduced at every node."""
    m = _perturbed_cube(4)
    rng = np.random.default_rng(7)
    A = 0.01 * rng.standard_normal((3, 3))
    c = 0.01 * rng.standard_normal(3)
    exact = m.xyz @ A.T + c
    m.dir_val = exact.reshape(-1)[m.dir_dof]
    u = monolithic.solve_linear(m)
    assert np.max(np.abs(u - exact.reshape(-1))) <= 1e-12 * np.max(np.abs(exact)) * 10


def _l2_error(mesh, u, exact_fn):
    """||u - u_h||_L2 with 3x3x3 Gauss quadrature per element."""
    g = np.sqrt(3.0 / 5.0)
    pts = [(-g, 5 / 9), (0.0, 8 / 9), (g, 5 / 9)]
    Xe = mesh.xyz[mesh.hex8]
    ue = u.reshape(-1, 3)[mesh.hex8]
    err2 = 0.0
    for a, wa in pts:
        for b, wb in pts:
            for c, wc in pts:
                N, dN = fem.shape_hex8([a, b, c])
                x = np.einsum("a,ead->ed", N, Xe)
                J = np.einsum("ead,ak->edk", Xe, dN)
                det = np.linalg.det(J)
                uh = np.einsum("a,ead->ed", N, ue)
                d = uh - exact_fn(x)
                err2 += np.sum(wa * wb * wc * det * np.sum(d * d, axis=1))
    return np.sqrt(err2)


def test_kelvin_second_order():
    """Kelvin's solution as Dirichlet data: the L2 error of Q1 falls with order 2
    (section 5.1, eqs. (fundSol), (L2Error), (L2Errora); Table 2 shows eoc ~ 2)."""
    E, nu = 1.0, 0.3
    errs = []
    for n in (4, 8, 16):
        m = cube_mesh(n, 1, E=E, nu=nu, body_force=None,
                      dirichlet_fn=lambda x: kelvin_displacement(x, E, nu))
        u = monolithic.solve_linear(m)
        errs.append(_l2_error(m, u, lambda x: kelvin_displacement(x, E, nu)))
    eoc = [np.log(errs[i] / errs[i + 1]) / np.log(2.0) for i in range(2)]
    assert 1.85 < eoc[0] < 2.2 and 1.9 < eoc[1] < 2.1, (errs, eoc)


def test_sparse_solve_matches_dense_cholesky():
    m = config_mesh("cube8_s2")
    K, _, f = fem.assemble(m)
    u = monolithic.solve_linear(m)
    free = np.setdiff1d(np.arange(m.n_dofs), m.dir_dof)
    import scipy.linalg as sla
    ud = sla.cho_solve(sla.cho_factor(K[free][:, free].toarray()), f[free])
    assert np.allclose(u[free], ud, rtol=1e-12, atol=1e-15 * np.abs(ud).max())
    r = K[free][:, free] @ u[free] - f[free]
    assert np.linalg.norm(r) <= 1e-13 * np.linalg.norm(f[free])


# ---------------------------------------------------------------- FETI reference
def _tiny_mesh():
    # 2x1x1 elements, split into two subdomains of one element each; partial
    # Dirichlet boundary (x = 0 face) so that classical FETI has a floating subdomain.
    m = cube_mesh(2, 1, body_force=(0.2, -0.5, 1.0))
    m.xyz = m.xyz * np.array([1.0, 0.5, 0.5])
    m.hex8 = m.hex8[:0]
    from workloads.meshes import _grid_hex, _grid_nodes
    m.xyz = _grid_nodes(2, 1, 1, 1.0, 0.5, 0.5)
    m.hex8, _ = _grid_hex(2, 1, 1)
    m.elem_sub = np.array([0, 1], dtype=np.int32)
    m.n_sub = 2
    m.elem_mat = np.zeros(2, dtype=np.int32)
    m.body_force = np.tile([0.2, -0.5, 1.0], (2, 1))
    left = np.nonzero(np.isclose(m.xyz[:, 0], 0.0))[0]
    m.dir_dof = (3 * left[:, None] + np.arange(3)).ravel()
    m.dir_val = 0.01 * np.arange(m.dir_dof.size, dtype=np.float64)
    return m


@pytest.mark.parametrize("variant", ["af", "classical"])
def test_feti_ref_matches_kkt_bruteforce(variant):
    """Subdomain displacements of the FETI reference equal those of the full
    saddle-point system (eqs. (classicalFetiLGS), (AFFETI)) solved densely."""
    m = _tiny_mesh()
    tp = feti_ref.linear_torn_problem(m, variant)
    sol = feti_ref.FetiRef(tp, "dirichlet").solve(rtol=1e-14)
    ub = feti_ref.kkt_bruteforce(tp)
    for i in range(2):
        assert np.allclose(sol["u_loc"][i], ub[i], rtol=1e-9, atol=1e-12)
    u_mono = monolithic.solve_linear(m)
    assert np.allclose(sol["u"], u_mono, rtol=1e-9, atol=1e-12)


@pytest.fixture(scope="module")
def cube8():
    m = config_mesh("cube8_s2")
    return m, monolithic.solve_linear(m)


@pytest.mark.parametrize("variant", ["af", "classical"])
def test_feti_ref_preconditioners_agree_with_monolithic(cube8, variant):
    m, u_ref = cube8
    tp = feti_ref.linear_torn_problem(m, variant)
    its = {}
    for pc in ("identity", "lumped", "dirichlet"):
        sol = feti_ref.FetiRef(tp, pc).solve(rtol=1e-12, track_invariants=True)
        err = np.linalg.norm(sol["u"] - u_ref) / np.linalg.norm(u_ref)
        assert err <= 1e-9, (pc, err)
        its[pc] = sol["iters"]
        if sol["n_coarse"]:
            assert max(sol["inv_err"]) <= 1e-10          # G^T lambda_k = e
    # Dirichlet <= lumped <= identity (Tables 2-7)
    assert its["dirichlet"] <= its["lumped"] <= its["identity"], its
    if variant == "af":
        assert tp.n_lam == 2556
    else:
        assert tp.n_lam == 732


@pytest.mark.parametrize("variant", ["af", "classical"])
def test_scaled_jump_operator_is_generalised_inverse(variant):
    """The scaled rows B_D of the preconditioner (eq. (feti_preconditioner))
    satisfy B B_D^T B = B, so that B_D^T B is a projection; checked on the dense
    B over all subdomain copies of a 3x3x3-subdomain cube, which has DOFs with
    1, 2, 4 and 8 copies, on and off the Dirichlet boundary."""
    m = cube_mesh(6, 3)
    tp = feti_ref.linear_torn_problem(m, variant)
    off = np.cumsum([0] + [sd["K"].shape[0] for sd in tp.subs])
    B = np.zeros((tp.n_lam, off[-1]))
    for r, row in enumerate(tp.rows):
        for (sub, ld, c) in row:
            B[r, off[sub] + ld] = c
    Pd = (tp.w[:, None] * B).T @ B
    assert np.abs(B @ Pd - B).max() <= 1e-14
    assert np.abs(Pd @ Pd - Pd).max() <= 1e-14
    assert tp.w.min() >= 0.0 and tp.w.max() <= 1.0


def test_feti_ref_constraint_residual(cube8):
    m, _ = cube8
    tp = feti_ref.linear_torn_problem(m, "af")
    sol = feti_ref.FetiRef(tp, "lumped").solve(rtol=1e-12)
    jump = -tp.b.copy()
    for i in range(m.n_sub):
        jump += tp.B(i) @ sol["u_loc"][i]
    assert np.linalg.norm(jump) <= 1e-9 * np.linalg.norm(sol["u"])


def test_floating_subdomain_kernel_dimension_six():
    m = config_mesh("cube8_s2")
    tp = feti_ref.linear_torn_problem(m, "af")
    K = tp.subs[0]["K"]
    R = feti_ref.rigid_modes(tp.subs[0]["x"])
    assert np.linalg.norm(K @ R) <= 1e-12 * np.linalg.norm(K) * np.linalg.norm(R)
    ev = np.linalg.eigvalsh(K)
    assert np.sum(ev < 1e-10 * ev[-1]) == 6


def test_projected_operator_symmetric_psd():
    """P^T F P is symmetric positive semi-definite (section 4.3 uses CG on it)."""
    m = cube_mesh(4, 2)
    tp = feti_ref.linear_torn_problem(m, "af")
    fr = feti_ref.FetiRef(tp, "lumped")
    n = tp.n_lam
    Fm = np.stack([fr.F(e) for e in np.eye(n)], axis=1)
    Gm = np.stack([fr.G(e) for e in np.eye(fr.n_coarse)], axis=1)
    P = np.eye(n) - Gm @ np.linalg.solve(Gm.T @ Gm, Gm.T)
    A = P.T @ Fm @ P
    assert np.allclose(A, A.T, atol=1e-12 * np.abs(A).max())
    ev = np.linalg.eigvalsh(0.5 * (A + A.T))
    assert ev.min() >= -1e-10 * ev.max()


def test_af_and_classical_same_displacement():
    m = cube_mesh(6, 3)
    u_ref = monolithic.solve_linear(m)
    for variant in ("af", "classical"):
        sol = feti_ref.FetiRef(feti_ref.linear_torn_problem(m, variant), "dirichlet").solve(rtol=1e-12)
        assert np.linalg.norm(sol["u"] - u_ref) <= 1e-9 * np.linalg.norm(u_ref)


@pytest.mark.slow
def test_dirichlet_condition_log_growth():
    """kappa of Dirichlet-preconditioned AF FETI grows like (1 + log(H/h))^2:
    kappa / (1+log(H/h))^2 stays within a factor 2.5 for H/h = 2, 4, 8."""
    ratios = []
    kap = {}
    for Hh in (2, 4, 8):
        m = cube_mesh(2 * Hh, 2)
        tp = feti_ref.linear_torn_problem(m, "af")
        sol = feti_ref.FetiRef(tp, "dirichlet").solve(rtol=1e-10)
        kap[Hh] = sol["kappa"]
        ratios.append(sol["kappa"] / (1 + np.log(Hh)) ** 2)
    assert max(ratios) / min(ratios) <= 2.5, (kap, ratios)
    assert kap[2] <= kap[4] <= kap[8]


# ---------------------------------------------------------------- HGO
HGO = dict(c=3.0, k1=2.3632, k2=0.8393)


def _rand_F(rng, scale=0.15):
    F = np.eye(3) + scale * rng.standard_normal((3, 3))
    if np.linalg.det(F) < 0:
        F[:, 0] *= -1
    return F


def _unit(v):
    return v / np.linalg.norm(v)


def test_hgo_stress_is_energy_derivative():
    """S_iso = 2 dPsi/dC (complex-step derivative of the written-out energy)."""
    rng = np.random.default_rng(0)
    for _ in range(5):
        F = _rand_F(rng, 0.2)
        C = F.T @ F
        a1, a2 = _unit(rng.standard_normal(3)), _unit(rng.standard_normal(3))
        S = fem.hgo_isochoric_stress(C[None], a1[None], a2[None], **HGO)[0]
        h = 1e-30
        Sfd = np.zeros((3, 3))
        for I in range(3):
            for J in range(3):
                dC = np.zeros((3, 3), dtype=complex)
                dC[I, J] += 0.5j * h
                dC[J, I] += 0.5j * h
                Sfd[I, J] = 2 * fem.hgo_isochoric_energy((C + dC)[None], a1[None], a2[None],
                                                         **HGO)[0].imag / h
        assert np.allclose(S, Sfd, rtol=1e-12, atol=1e-12)


def test_hgo_uniaxial_fibre_stress_hand_derived():
    """Isochoric uniaxial stretch along both fibre families: the Cauchy stress
    difference sigma_11 - sigma_22 = c (l^2 - 1/l) + 4 k1 (l^2-1) exp(k2 (l^2-1)^2) l^2."""
    c, k1, k2 = HGO["c"], HGO["k1"], HGO["k2"]
    e1 = np.array([1.0, 0.0, 0.0])
    for lam in (1.05, 1.2, 1.4):
        F = np.diag([lam, lam ** -0.5, lam ** -0.5])
        S = fem.hgo_isochoric_stress((F.T @ F)[None], e1[None], e1[None], c, k1, k2)[0]
        sig = F @ S @ F.T / np.linalg.det(F)
        E = lam ** 2 - 1
        exact = c * (lam ** 2 - 1 / lam) + 4 * k1 * E * np.exp(k2 * E * E) * lam ** 2
        assert abs((sig[0, 0] - sig[1, 1]) - exact) <= 1e-12 * abs(exact)
    # compression: fibres inactive, pure neo-Hooke
    lam = 0.9
    F = np.diag([lam, lam ** -0.5, lam ** -0.5])
    S = fem.hgo_isochoric_stress((F.T @ F)[None], e1[None], e1[None], c, k1, k2)[0]
    sig = F @ S @ F.T
    assert abs((sig[0, 0] - sig[1, 1]) - c * (lam ** 2 - 1 / lam)) <= 1e-12


def _hgo_elem(rng, scale=0.1):
    X = _distorted_element(4)
    U = scale * rng.standard_normal((8, 3))
    a1, a2 = _unit(rng.standard_normal(3)), _unit(rng.standard_normal(3))
    return X, U, a1, a2


def test_hgo_force_is_energy_gradient_and_tangent_is_force_gradient():
    rng = np.random.default_rng(11)
    X, U, a1, a2 = _hgo_elem(rng)
    kap = 50.0
    args = (a1[None], a2[None], HGO["c"], HGO["k1"], HGO["k2"], kap)
    f, _, _ = fem.hgo_element_force(X[None], U[None], *args)
    K, f2 = fem.hgo_element_tangent(X[None], U[None], *args)
    eps = 1e-6
    gfd = np.zeros(24)
    Kfd = np.zeros((24, 24))
    for k in range(24):
        dU = np.zeros(24)
        dU[k] = eps
        Ep = fem.hgo_element_energy(X[None], (U.reshape(-1) + dU).reshape(1, 8, 3), *args)[0]
        Em = fem.hgo_element_energy(X[None], (U.reshape(-1) - dU).reshape(1, 8, 3), *args)[0]
        gfd[k] = (Ep - Em) / (2 * eps)
        fp, _, _ = fem.hgo_element_force(X[None], (U.reshape(-1) + dU).reshape(1, 8, 3), *args)
        fm, _, _ = fem.hgo_element_force(X[None], (U.reshape(-1) - dU).reshape(1, 8, 3), *args)
        Kfd[:, k] = (fp[0] - fm[0]) / (2 * eps)
    assert np.allclose(f[0], gfd, rtol=1e-7, atol=1e-7 * np.abs(f).max())
    assert np.allclose(K[0], Kfd, rtol=1e-6, atol=1e-6 * np.abs(K).max())
    assert np.allclose(K[0], K[0].T, atol=1e-10 * np.abs(K).max())   # hyperelastic => symmetric
    assert np.allclose(f2[0], f[0].real)


def test_hgo_tangent_at_reference_is_mean_dilatation_elasticity():
    """At U = 0 the tangent is isotropic elasticity with mu = c, lambda = -2c/3,
    plus the condensed volumetric term (kappa / V_e) g g^T with g_a = int grad N_a."""
    X = _distorted_element(9)
    rng = np.random.default_rng(2)
    a1, a2 = _unit(rng.standard_normal(3)), _unit(rng.standard_normal(3))
    c, kap = 3.0, 300.0
    K, f = fem.hgo_element_tangent(X[None], np.zeros((1, 8, 3)), a1[None], a2[None], c,
                                   HGO["k1"], HGO["k2"], kap)
    Kdev = fem.linear_stiffness(X[None], -2.0 * c / 3.0, c)[0]
    g = np.zeros(24)
    V = 0.0
    for _, dN, det in fem.ref_gradients(X[None]):
        g += det[0] * dN[0].reshape(-1)
        V += det[0]
    assert np.allclose(K[0], Kdev + kap / V * np.outer(g, g), rtol=1e-10,
                       atol=1e-10 * np.abs(K).max())
    assert np.abs(f).max() < 1e-12


def test_hgo_objectivity_and_translations():
    """K(U)(W x) = W f_int(U) for skew W, x = X + U; translations are in ker K(U)."""
    rng = np.random.default_rng(5)
    X, U, a1, a2 = _hgo_elem(rng, 0.08)
    args = (a1[None], a2[None], HGO["c"], HGO["k1"], HGO["k2"], 100.0)
    K, f = fem.hgo_element_tangent(X[None], U[None], *args)
    w = rng.standard_normal(3)
    W = np.array([[0, -w[2], w[1]], [w[2], 0, -w[0]], [-w[1], w[0], 0]])
    x = X + U
    lhs = K[0] @ (x @ W.T).reshape(-1)
    rhs = (f[0].reshape(8, 3) @ W.T).reshape(-1)
    assert np.allclose(lhs, rhs, atol=1e-9 * np.abs(K).max())
    for k in range(3):
        t = np.zeros((8, 3))
        t[:, k] = 1.0
        assert np.abs(K[0] @ t.reshape(-1)).max() <= 1e-11 * np.abs(K).max()


def test_pressure_load_total_force():
    """The follower pressure on a closed flat face sums to -p * area * n."""
    xf = np.array([[[0, 0, 0], [2, 0, 0], [2, 3, 0], [0, 3, 0]]], dtype=np.float64)
    f = fem.pressure_face_load(xf, 1.5)
    assert np.allclose(f[0].sum(axis=0), [0, 0, -1.5 * 6.0])
    # a full closed tube surface integrates to zero net force
    m = tube_mesh(nr=1, nth=16, nz=2, sub=(1, 1, 1))
    fp = fem.pressure_face_load(m.xyz[m.pface], 1.0)
    tot = fp.sum(axis=(0, 1))
    assert abs(tot[0]) < 1e-12 and abs(tot[1]) < 1e-12


def test_newton_quadratic_with_dead_load():
    """Newton on the HGO tube with a dead body load converges quadratically."""
    m = tube_mesh(nr=2, nth=16, nz=4, sub=(1, 1, 1), pressure=0.0)
    m.body_force = np.tile([0.0, 0.0, 0.1], (m.n_elems, 1))
    U = np.zeros(m.n_dofs)
    res = []
    for _ in range(10):
        dU, rn = monolithic.newton_increment(m, U, 1.0)
        res.append(rn)
        U = U + dU
        if rn < 1e-12:
            break
    rates = [res[k + 1] / res[k] ** 2 for k in range(1, len(res) - 1) if res[k + 1] > 1e-11]
    assert res[-1] < 1e-10, res
    # the last contractions are quadratic: r_{k+1} <= C r_k^2
    assert len(rates) >= 2 and all(r < 50.0 for r in rates[-2:]), (res, rates)


def test_nodal_residual_matches_assembled_rows():
    """The sampled-node residual (elements and faces around the nodes only)
    equals the rows of the globally assembled system, linear and HGO with a
    follower pressure; it vanishes at the direct solution."""
    rng = np.random.default_rng(3)
    m = config_mesh("cube8_s2")
    u = monolithic.solve_linear(m)
    nodes = rng.choice(m.n_nodes, 40, replace=False)
    res, sc = fem.nodal_residual(m, nodes, u)
    assert (np.abs(res) / sc).max() < 1e-13
    w = rng.standard_normal(m.n_dofs)
    K, _, f = fem.assemble(m, None)
    r = (f - K @ w).reshape(-1, 3)[nodes]
    dm = np.zeros(m.n_dofs, bool)
    dm[m.dir_dof] = True
    r[dm.reshape(-1, 3)[nodes]] = 0.0
    res, _ = fem.nodal_residual(m, nodes, w)
    assert np.abs(res - r).max() <= 1e-13 * np.abs(r).max()
    # HGO tube with pressure, at a displaced state
    t = tube_mesh(nr=2, nth=8, nz=4, sub=(1, 2, 1), pressure=2.0)
    U = 1e-3 * rng.standard_normal(t.n_dofs)
    U[t.dir_dof] = 0.0
    du = rng.standard_normal(t.n_dofs)
    nodes = rng.choice(t.n_nodes, 30, replace=False)
    K, fint, fext = fem.assemble(t, U.reshape(-1, 3), tau=0.7)
    r = (fext - fint - K @ du).reshape(-1, 3)[nodes]
    dm = np.zeros(t.n_dofs, bool)
    dm[t.dir_dof] = True
    r[dm.reshape(-1, 3)[nodes]] = 0.0
    res, _ = fem.nodal_residual(t, nodes, du, U=U.reshape(-1, 3), tau=0.7)
    assert np.abs(res - r).max() <= 1e-12 * np.abs(r).max()


# ---------------------------------------------------------------- pins added for
# the condition estimate and the nodal splits of the loads
def _plain_cg(A, b, n_it):
    """Textbook CG (x0 = 0) returning its (alpha_k, beta_k)."""
    x = np.zeros_like(b)
    r = b.copy()
    p = r.copy()
    rr = r @ r
    al, be = [], []
    for _ in range(n_it):
        q = A @ p
        a = rr / (p @ q)
        x += a * p
        r -= a * q
        rr2 = r @ r
        al.append(a)
        be.append(rr2 / rr)
        p = r + be[-1] * p
        rr = rr2
    return al, be


def test_lanczos_kappa_exact_on_known_spectrum():
    """After n CG steps on an n x n SPD matrix the Lanczos tridiagonal built
    from (alpha, beta) has the matrix's own eigenvalues, so the estimate is
    exactly lambda_max / lambda_min."""
    rng = np.random.default_rng(4)
    lam = np.array([1.0, 1.7, 2.2, 3.0, 4.1, 5.5, 6.0, 7.3, 8.8, 9.5])
    Qm, _ = np.linalg.qr(rng.standard_normal((10, 10)))
    A = Qm @ np.diag(lam) @ Qm.T
    al, be = _plain_cg(A, rng.standard_normal(10), 10)
    assert abs(feti_ref.lanczos_kappa(al, be) - 9.5) <= 1e-9 * 9.5
    # fewer steps: Ritz values lie inside the spectrum (interlacing)
    al, be = _plain_cg(A, rng.standard_normal(10), 5)
    assert 1.0 <= feti_ref.lanczos_kappa(al, be) <= 9.5 * (1 + 1e-12)


@pytest.mark.parametrize("variant", ["af", "classical"])
def test_lanczos_kappa_matches_spectrum_of_preconditioned_operator(variant):
    """The FETI reference's condition estimate equals the ratio of the extreme
    nonzero eigenvalues of (P M P)(P F P), formed explicitly, for every
    preconditioner.  A random body force excites every eigen-direction, so the
    Lanczos values reach the extreme eigenvalues at a tight tolerance."""
    m = cube_mesh(4, 2)
    rng = np.random.default_rng(5)
    m.body_force = rng.standard_normal((m.n_elems, 3))
    tp = feti_ref.linear_torn_problem(m, variant)
    n = tp.n_lam
    for pc in ("lumped", "dirichlet", "identity"):
        fr = feti_ref.FetiRef(tp, pc)
        if pc == "lumped":
            Fm = np.stack([fr.F(e) for e in np.eye(n)], axis=1)
            P = np.eye(n)
            if fr.n_coarse:
                Gm = np.stack([fr.G(e) for e in np.eye(fr.n_coarse)], axis=1)
                P = P - Gm @ np.linalg.solve(Gm.T @ Gm, Gm.T)
        Mm = np.stack([fr.Mprec(e) for e in np.eye(n)], axis=1)
        ev = np.sort(np.abs(np.linalg.eigvals((P @ Mm @ P) @ (P @ Fm @ P)).real))
        nz = ev[ev > 1e-9 * ev[-1]]
        exact = nz[-1] / nz[0]
        est = fr.solve(rtol=1e-12)["kappa"]
        assert abs(est / exact - 1.0) <= 2e-3, (pc, est, exact)


def _gauss3():
    g = np.sqrt(3.0 / 5.0)
    return [(-g, 5.0 / 9.0), (0.0, 8.0 / 9.0), (g, 5.0 / 9.0)]


def test_body_force_nodal_split_on_distorted_element():
    """int N_a b dX on a distorted trilinear element: N_a det(dX/dxi) has degree
    3 in each reference coordinate, so a 3-point Gauss rule (written here
    independently of the element code) gives the exact nodal split."""
    X = _distorted_element(7) * np.array([1.3, 0.8, 1.1])
    b = np.array([0.4, -1.2, 0.7])
    ref = np.zeros((8, 3))
    for xa, wa in _gauss3():
        for xb, wb in _gauss3():
            for xc, wc in _gauss3():
                xi = np.array([xa, xb, xc])
                N = np.prod(1.0 + fem.XI * xi, axis=1) / 8.0
                dN = np.stack([fem.XI[:, k] / 8.0 * np.prod(np.delete(1.0 + fem.XI * xi, k, axis=1), axis=1)
                               for k in range(3)], axis=1)
                det = np.linalg.det(X.T @ dN)
                ref += wa * wb * wc * det * N[:, None] * b[None, :]
    f = fem.body_force_vector(X[None], b[None])[0].reshape(8, 3)
    assert np.abs(f - ref).max() <= 1e-14 * np.abs(ref).max() * 10
    # the split is not the naive equal share on a distorted element
    assert np.abs(f - f.sum(axis=0) / 8).max() > 1e-4 * np.abs(f).max()


def _curved_face(seed=3):
    rng = np.random.default_rng(seed)
    xf = np.array([[0, 0, 0], [1.2, 0, 0], [1.1, 0.9, 0], [0, 1.0, 0]], dtype=np.float64)
    xf[:, 2] = [0.0, 0.25, -0.15, 0.3]            # warped: the four corners are not coplanar
    return xf + 0.05 * rng.standard_normal((4, 3))


def test_pressure_nodal_split_on_warped_face():
    """f_a = -p int N_a (dx/deta1 x dx/deta2) deta on a warped bilinear face,
    against a 3x3 Gauss rule written here (the integrand has degree 2 in each
    variable, so both rules are exact); the corner order of the face is
    (-1,-1), (1,-1), (1,1), (-1,1)."""
    xf = _curved_face()
    p = 1.7
    eta = np.array([[-1, -1], [1, -1], [1, 1], [-1, 1]], dtype=np.float64)
    ref = np.zeros((4, 3))
    for s, ws in _gauss3():
        for t, wt in _gauss3():
            N = 0.25 * (1 + eta[:, 0] * s) * (1 + eta[:, 1] * t)
            dNs = 0.25 * eta[:, 0] * (1 + eta[:, 1] * t)
            dNt = 0.25 * eta[:, 1] * (1 + eta[:, 0] * s)
            n = np.cross(dNs @ xf, dNt @ xf)
            ref += -p * ws * wt * N[:, None] * n[None, :]
    f = fem.pressure_face_load(xf[None], p)[0]
    assert np.abs(f - ref).max() <= 1e-14 * np.abs(ref).max() * 10


def test_pressure_load_follows_the_geometry():
    """A follower load on the current surface rotates with a rigid rotation of
    the face, f(Q x) = Q f(x), and scales with the area, f(s x) = s^2 f(x); a
    translation leaves it unchanged."""
    xf = _curved_face(8)
    rng = np.random.default_rng(9)
    Q, _ = np.linalg.qr(rng.standard_normal((3, 3)))
    if np.linalg.det(Q) < 0:
        Q[:, 0] *= -1
    f = fem.pressure_face_load(xf[None], 0.9)[0]
    fq = fem.pressure_face_load((xf @ Q.T)[None], 0.9)[0]
    assert np.abs(fq - f @ Q.T).max() <= 1e-14 * np.abs(f).max() * 10
    fs = fem.pressure_face_load((2.5 * xf)[None], 0.9)[0]
    assert np.abs(fs - 6.25 * f).max() <= 1e-14 * np.abs(fs).max() * 10
    ft = fem.pressure_face_load((xf + np.array([3.0, -1.0, 2.0]))[None], 0.9)[0]
    assert np.abs(ft - f).max() <= 1e-14 * np.abs(f).max() * 100


# ---------------------------------------------------------------- follower-load stiffness
def test_pressure_load_stiffness_is_load_derivative():
    """The complex-step load stiffness equals central finite differences of
    the pressure load (a different differentiation), and follows from the
    load's invariances: translations do not change the load (D t = 0) and an
    infinitesimal rotation W rotates it (D (W x) = W f)."""
    xf = _curved_face(4)
    p = 1.3
    D = fem.pressure_load_stiffness(xf[None], p)[0]
    eps = 1e-6
    Dfd = np.zeros((12, 12))
    for c in range(12):
        dx = np.zeros(12)
        dx[c] = eps
        fp = fem.pressure_face_load((xf.reshape(-1) + dx).reshape(1, 4, 3), p)[0].reshape(-1)
        fm = fem.pressure_face_load((xf.reshape(-1) - dx).reshape(1, 4, 3), p)[0].reshape(-1)
        Dfd[:, c] = (fp - fm) / (2 * eps)
    assert np.abs(D - Dfd).max() <= 1e-8 * np.abs(D).max()
    for k in range(3):
        t = np.zeros((4, 3))
        t[:, k] = 1.0
        assert np.abs(D @ t.reshape(-1)).max() <= 1e-13 * np.abs(D).max()
    w = np.array([0.3, -0.7, 0.4])
    W = np.array([[0, -w[2], w[1]], [w[2], 0, -w[0]], [-w[1], w[0], 0]])
    f = fem.pressure_face_load(xf[None], p)[0]
    assert np.allclose(D @ (xf @ W.T).reshape(-1), (f @ W.T).reshape(-1), atol=1e-13 * np.abs(f).max())


def test_assembled_load_stiffness_symmetric_when_edges_clamped():
    """A pressure on a surface whose boundary does not move is conservative:
    the assembled load stiffness is symmetric on the free DOFs (tube with
    clamped ends), while a single face with free edges gives a non-symmetric
    one."""
    t = tube_mesh(nr=1, nth=12, nz=4, sub=(1, 1, 1), pressure=1.5)
    rng = np.random.default_rng(2)
    U = 0.05 * rng.standard_normal(t.n_dofs)
    U[t.dir_dof] = 0.0
    D = fem.assemble_load_stiffness(t, U).toarray()
    free = np.setdiff1d(np.arange(t.n_dofs), t.dir_dof)
    Dff = D[np.ix_(free, free)]
    assert np.abs(Dff - Dff.T).max() <= 1e-13 * np.abs(Dff).max()
    assert np.abs(D - D.T).max() > 1e-3 * np.abs(D).max()      # the clamped rows break it
    Df = fem.pressure_load_stiffness(_curved_face(5)[None], 1.5)[0]
    assert np.abs(Df - Df.T).max() > 1e-3 * np.abs(Df).max()


def test_exact_newton_quadratic_with_follower_load():
    """With the load stiffness the Newton step is the exact linearisation of
    the follower-pressure problem and converges quadratically; without it the
    contraction is only linear (the load stiffness the paper neglects)."""
    m = tube_mesh(nr=2, nth=16, nz=8, sub=(1, 1, 1))
    tau = 1.0 / 40.0

    def run(ls, n):
        U = np.zeros(m.n_dofs)
        res = []
        for _ in range(n):
            dU, rn = monolithic.newton_increment(m, U, tau, load_stiffness=ls)
            res.append(rn)
            U = U + dU
        res.append(monolithic.residual_norm(m, U, tau)[0])
        return np.array(res) / res[0]
    r = run(True, 6)
    assert r[-1] < 1e-10, r
    q = [r[k + 1] / r[k] ** 2 for k in range(len(r) - 1) if r[k + 1] > 2e-11 and r[k] < 0.1]
    assert len(q) >= 2 and max(q) < 1.0, (r, q)
    r0 = run(False, 7)
    assert r0[-1] > 1e-10 and r0[-1] / r0[-2] ** 2 > 100.0, r0


# ---------------------------------------------------------------- partial kernels (classical)
def test_classical_partial_kernels_match_monolithic():
    """Classical FETI on a cube whose Dirichlet data touch subdomains only
    partially (section 4.3): the subdomain at the clamped quarter face has no
    kernel, the two that touch it along an edge keep one rotation, the one
    that touches it at a vertex keeps three rotations, and the four whose
    face has only u_x fixed keep two translations and one rotation; the
    reference FETI then gives the monolithic solution for every
    preconditioner, and each kernel is annihilated by its K_i."""
    from workloads import partial_dirichlet_cube
    m = partial_dirichlet_cube(4, 2)
    u_ref = monolithic.solve_linear(m)
    tp = feti_ref.linear_torn_problem(m, "classical")
    dims = []
    for pc in ("lumped", "dirichlet"):
        fr = feti_ref.FetiRef(tp, pc)
        dims = [0 if lc["R"] is None else lc["R"].shape[1] for lc in fr.locals]
        for i, lc in enumerate(fr.locals):
            if lc["R"] is not None:
                K = tp.subs[i]["K"]
                assert np.linalg.norm(K @ lc["R"]) <= 1e-12 * np.linalg.norm(K) * np.linalg.norm(lc["R"])
        sol = fr.solve(rtol=1e-12)
        assert np.linalg.norm(sol["u"] - u_ref) <= 1e-9 * np.linalg.norm(u_ref), pc
    # subdomain id = ix + 2 iy + 4 iz
    assert dims == [0, 3, 1, 3, 1, 3, 3, 3], dims
