"""Pins of the oracle's Q2 (27-node hexahedron, P0 pressure) elements against
facts fixed by mathematics: interpolation properties, exactness of the
3-point Gauss rule, the exact reproduction of quadratic displacement fields,
rigid-body kernels, closed-form consistent nodal loads, energy and force
derivatives, objectivity, and the FETI oracle against the monolithic solve on
Q2 meshes.  The quadratic elements are those of section 3.2 (P2-P0 pairs) and
the Q2 tube of section 5.3's discretisations."""
import numpy as np
import pytest

from oracle import fem, monolithic, feti_ref
from workloads import cube_mesh, tube_mesh

HGO = dict(c=3.0, k1=2.3632, k2=0.8393)


def _curved_element(seed=0, amp=0.06):
    """A Q2 element whose 27 nodes are a unit cube's, moved by a smooth
    quadratic map plus small random offsets of the mid-side and centre nodes."""
    rng = np.random.default_rng(seed)
    X = 0.5 * (fem.XI27 + 1.0)
    X = X + 0.1 * X[:, [1, 2, 0]] ** 2
    mid = np.abs(fem.XI27).sum(axis=1) < 3
    X[mid] += amp * rng.standard_normal((mid.sum(), 3))
    return X


def _unit(v):
    return v / np.linalg.norm(v)


# ---------------------------------------------------------------- shapes
def test_shape_hex27_interpolation_properties():
    """N_a(xi_b) = delta_ab, sum N_a = 1, sum dN_a = 0, and exact
    reproduction of a triquadratic polynomial and its gradient."""
    for b in range(27):
        N, _ = fem.shape_hex27(fem.XI27[b])
        assert np.allclose(N, np.eye(27)[b], atol=1e-15)
    rng = np.random.default_rng(0)
    c = rng.standard_normal((3, 3, 3))

    def poly(x):
        return sum(c[i, j, k] * x[0] ** i * x[1] ** j * x[2] ** k
                   for i in range(3) for j in range(3) for k in range(3))

    def grad(x):
        g = np.zeros(3)
        for i in range(3):
            for j in range(3):
                for k in range(3):
                    g[0] += c[i, j, k] * i * x[0] ** max(i - 1, 0) * x[1] ** j * x[2] ** k
                    g[1] += c[i, j, k] * j * x[0] ** i * x[1] ** max(j - 1, 0) * x[2] ** k
                    g[2] += c[i, j, k] * k * x[0] ** i * x[1] ** j * x[2] ** max(k - 1, 0)
        return g

    vals = np.array([poly(x) for x in fem.XI27])
    for _ in range(5):
        x = rng.uniform(-1, 1, 3)
        N, dN = fem.shape_hex27(x)
        assert abs(N.sum() - 1.0) < 1e-14
        assert np.abs(dN.sum(axis=0)).max() < 1e-14
        assert abs(N @ vals - poly(x)) < 1e-12
        assert np.allclose(dN.T @ vals, grad(x), atol=1e-12)


def test_q2_gauss_rule_exact_to_degree_five():
    """The 27-point rule integrates x^i y^j z^k exactly for i, j, k <= 5 on an
    affine element (volume scaled by |det A|)."""
    rng = np.random.default_rng(1)
    A = np.diag([0.5, 1.5, 2.0])
    X = fem.XI27 @ A.T + rng.standard_normal(3)[None, :] * 0.0
    for (i, j, k) in [(0, 0, 0), (2, 4, 0), (5, 1, 3), (4, 4, 4), (5, 5, 5)]:
        s = 0.0
        for N, _, dV in fem.ref_gradients(X[None]):
            x = N @ X
            s += dV[0] * x[0] ** i * x[1] ** j * x[2] ** k

        def m1(p, h):   # int_{-h}^{h} t^p dt
            return 0.0 if p % 2 else 2.0 * h ** (p + 1) / (p + 1)

        exact = m1(i, 0.5) * m1(j, 1.5) * m1(k, 2.0)
        assert abs(s - exact) <= 1e-13 * max(1.0, abs(exact))


# ---------------------------------------------------------------- linear Q2
def test_q2_rigid_modes_span_kernel():
    """The curved Q2 element stiffness annihilates the six rigid motions and
    has rank 81 - 6 = 75."""
    X = _curved_element()
    lam, mu = fem.lame(1.0, 0.3)
    K = fem.linear_stiffness(X[None], lam, mu)[0]
    R = feti_ref.rigid_modes(X)
    assert K.shape == (81, 81)
    assert np.allclose(K, K.T, atol=1e-14 * np.abs(K).max())
    assert np.linalg.norm(K @ R) <= 1e-12 * np.linalg.norm(K) * np.linalg.norm(R)
    ev = np.linalg.eigvalsh(K)
    assert np.sum(ev < 1e-10 * ev[-1]) == 6
    assert ev[6] > 1e-6 * ev[-1]


def test_q2_reproduces_quadratic_solution_exactly():
    """Q2 patch test: for a quadratic displacement u the stress is linear and
    the body force b = -div sigma constant; with u on the boundary as Dirichlet
    data, the Q2 solution on a mesh of boxes of unequal sizes equals u at every
    node, mid-side and centre nodes included, to rounding."""
    E, nu = 2.0, 0.3
    lam, mu = fem.lame(E, nu)
    rng = np.random.default_rng(4)
    Q = 0.05 * rng.standard_normal((3, 3, 3))
    Q = 0.5 * (Q + Q.transpose(0, 2, 1))       # u_i = sum_jk Q_ijk x_j x_k, Q_ijk = Q_ikj

    def u_exact(x):
        return np.einsum("ijk,nj,nk->ni", Q, x, x)

    # grad u_ij = 2 Q_ijk x_k; div sigma_i = lam d_i(div u) + mu (lap u_i + d_i div u)
    div_grad = np.einsum("jji->i", 2.0 * Q)          # d_i (div u) = 2 Q_jji
    lap = 2.0 * np.einsum("ijj->i", Q)              # lap u_i = 2 Q_ijj
    b = -(lam * div_grad + mu * (lap + div_grad))
    knots, moved = [0.0, 1 / 3, 2 / 3, 1.0], [0.0, 0.2, 0.65, 1.0]
    m = cube_mesh(3, 1, E=E, nu=nu, body_force=tuple(b), order=2)
    # piecewise linear per axis, linear inside every element: boxes of
    # unequal sizes whose mid-side nodes stay at the midpoints
    m.xyz = np.interp(m.xyz, knots, moved)
    m.dir_val = u_exact(m.xyz[m.dir_dof // 3])[np.arange(m.dir_dof.size), m.dir_dof % 3]
    u = monolithic.solve_linear(m).reshape(-1, 3)
    assert np.abs(u).max() > 1e-3
    err = np.abs(u - u_exact(m.xyz)).max() / np.abs(u_exact(m.xyz)).max()
    assert err < 1e-11, err
    # a wrong body force (a dropped Lame term) breaks the exactness
    m.body_force = np.tile(-(mu * (lap + div_grad)), (m.n_elems, 1))
    u2 = monolithic.solve_linear(m).reshape(-1, 3)
    assert np.abs(u2 - u_exact(m.xyz)).max() / np.abs(u_exact(m.xyz)).max() > 1e-4


def test_q2_body_force_consistent_split():
    """On an affine element a constant body force gives the tensor product of
    Simpson's weights (1, 4, 1)/6 in each direction, times b * volume."""
    A = np.array([[1.0, 0.2, 0.0], [0.0, 2.0, 0.3], [0.1, 0.0, 0.5]])
    X = 0.5 * (fem.XI27 + 1.0) @ A.T
    b = np.array([[0.3, -1.0, 2.0]])
    f = fem.body_force_vector(X[None], b)[0].reshape(27, 3)
    w1 = np.array([1.0, 4.0, 1.0]) / 6.0
    w = np.array([w1[a % 3] * w1[(a // 3) % 3] * w1[a // 9] for a in range(27)])
    assert np.allclose(f, np.linalg.det(A) * w[:, None] * b, rtol=1e-13, atol=1e-15)


# ---------------------------------------------------------------- pressure Q2
def test_q2_pressure_consistent_split_flat_face():
    """Uniform pressure on a flat rectangle: the biquadratic face's consistent
    nodal loads are -p A n times (1, 4, 1)/6 x (1, 4, 1)/6."""
    s = 0.5 * (fem.XI27[:9, :2] + 1.0)              # the face z = -1 of the reference nodes
    xf = np.stack([2.0 * s[:, 0], 3.0 * s[:, 1], np.zeros(9)], axis=1)
    p = 1.5
    f = fem.pressure_face_load(xf[None], p)[0]
    w1 = np.array([1.0, 4.0, 1.0]) / 6.0
    w = np.array([w1[a % 3] * w1[a // 3] for a in range(9)])
    assert np.allclose(f, -p * 6.0 * w[:, None] * np.array([0.0, 0.0, 1.0])[None, :], atol=1e-14)


def test_q2_pressure_curved_face_matches_fine_quadrature():
    """On a curved, warped 9-node face the 3x3 rule equals an independent
    10x10 Gauss-Legendre quadrature of -p N_a (x_s x x_t) (the integrand is of
    degree 5 per direction, so both are exact)."""
    rng = np.random.default_rng(7)
    s = fem.XI27[:9, :2]
    xf = np.stack([s[:, 0] + 0.1 * s[:, 1] ** 2, s[:, 1], 0.3 * s[:, 0] ** 2 - 0.2 * s[:, 1] ** 2], axis=1)
    xf = xf + 0.05 * rng.standard_normal((9, 3))
    p = 0.7
    f = fem.pressure_face_load(xf[None], p)[0]
    pts, wts = np.polynomial.legendre.leggauss(10)
    ref = np.zeros((9, 3))

    def L(x):
        return np.array([0.5 * x * (x - 1), 1 - x * x, 0.5 * x * (x + 1)])

    def dL(x):
        return np.array([x - 0.5, -2 * x, x + 0.5])

    for u, wu in zip(pts, wts):
        for v, wv in zip(pts, wts):
            N = np.array([L(u)[a % 3] * L(v)[a // 3] for a in range(9)])
            Ns = np.array([dL(u)[a % 3] * L(v)[a // 3] for a in range(9)])
            Nt = np.array([L(u)[a % 3] * dL(v)[a // 3] for a in range(9)])
            n = np.cross(Ns @ xf, Nt @ xf)
            ref += -p * wu * wv * N[:, None] * n[None, :]
    assert np.allclose(f, ref, atol=1e-13 * np.abs(ref).max())


def test_q2_tube_pressure_closed_surface_and_axial_force():
    """The follower pressure on the Q2 tube's inner surface has no net
    transverse force; its radial resultant per unit length matches
    p * 2 r sin(pi/n) per polygon side summed (the Q2 face is a parabola
    through three points of the circle: net radial push > 0)."""
    m = tube_mesh(nr=1, nth=8, nz=2, sub=(1, 1, 1), order=2, pressure=1.0)
    fp = fem.pressure_face_load(m.xyz[m.pface], 1.0)
    tot = fp.sum(axis=(0, 1))
    assert np.abs(tot).max() < 1e-12
    # radial components push outward... no: the load is -p n with n towards the
    # axis, i.e. radially outwards on the inner wall
    x = m.xyz[m.pface]
    r = np.linalg.norm(x[:, :, :2], axis=2)
    radial = (fp[:, :, 0] * x[:, :, 0] + fp[:, :, 1] * x[:, :, 1]) / r
    assert radial.sum() > 0.0


def test_q2_pressure_load_stiffness_is_load_derivative():
    """Central differences of the 9-node face load equal the complex-step
    load stiffness."""
    rng = np.random.default_rng(3)
    s = fem.XI27[:9, :2]
    xf = np.stack([s[:, 0], s[:, 1], 0.2 * s[:, 0] * s[:, 1]], axis=1) + 0.03 * rng.standard_normal((9, 3))
    D = fem.pressure_load_stiffness(xf[None], 0.9)[0]
    eps = 1e-6
    Dfd = np.zeros((27, 27))
    for k in range(27):
        dx = np.zeros(27)
        dx[k] = eps
        fp = fem.pressure_face_load((xf.reshape(-1) + dx).reshape(1, 9, 3), 0.9)[0].reshape(-1)
        fm = fem.pressure_face_load((xf.reshape(-1) - dx).reshape(1, 9, 3), 0.9)[0].reshape(-1)
        Dfd[:, k] = (fp - fm) / (2 * eps)
    assert np.allclose(D, Dfd, atol=1e-8 * np.abs(D).max())


# ---------------------------------------------------------------- HGO Q2-P0
def _hgo_q2(seed, amp=0.05):
    rng = np.random.default_rng(seed)
    X = _curved_element(seed)
    U = amp * rng.standard_normal((27, 3))
    a1, a2 = _unit(rng.standard_normal(3)), _unit(rng.standard_normal(3))
    return X, U, a1, a2


def test_q2_hgo_force_is_energy_gradient_and_tangent_is_force_gradient():
    X, U, a1, a2 = _hgo_q2(11)
    args = (a1[None], a2[None], HGO["c"], HGO["k1"], HGO["k2"], 50.0)
    f, _, _ = fem.hgo_element_force(X[None], U[None], *args)
    K, f2 = fem.hgo_element_tangent(X[None], U[None], *args)
    eps = 1e-6
    gfd = np.zeros(81)
    cols = list(range(0, 81, 7))
    Kfd = np.zeros((81, len(cols)))
    for k in range(81):
        dU = np.zeros(81)
        dU[k] = eps
        Ep = fem.hgo_element_energy(X[None], (U.reshape(-1) + dU).reshape(1, 27, 3), *args)[0]
        Em = fem.hgo_element_energy(X[None], (U.reshape(-1) - dU).reshape(1, 27, 3), *args)[0]
        gfd[k] = (Ep - Em) / (2 * eps)
        if k in cols:
            fp, _, _ = fem.hgo_element_force(X[None], (U.reshape(-1) + dU).reshape(1, 27, 3), *args)
            fm, _, _ = fem.hgo_element_force(X[None], (U.reshape(-1) - dU).reshape(1, 27, 3), *args)
            Kfd[:, cols.index(k)] = (fp[0] - fm[0]) / (2 * eps)
    assert np.allclose(f[0], gfd, rtol=1e-7, atol=1e-7 * np.abs(f).max())
    assert np.allclose(K[0][:, cols], Kfd, rtol=1e-6, atol=1e-6 * np.abs(K).max())
    assert np.allclose(K[0], K[0].T, atol=1e-10 * np.abs(K).max())
    assert np.allclose(f2[0], f[0].real)


def test_q2_hgo_tangent_at_reference_is_mean_dilatation_elasticity():
    """At U = 0 the Q2-P0 tangent is isotropic elasticity with mu = c,
    lambda = -2c/3, plus (kappa / V_e) g g^T with g_a = int grad N_a."""
    X = _curved_element(9)
    rng = np.random.default_rng(2)
    a1, a2 = _unit(rng.standard_normal(3)), _unit(rng.standard_normal(3))
    c, kap = 3.0, 300.0
    K, f = fem.hgo_element_tangent(X[None], np.zeros((1, 27, 3)), a1[None], a2[None], c,
                                   HGO["k1"], HGO["k2"], kap)
    Kdev = fem.linear_stiffness(X[None], -2.0 * c / 3.0, c)[0]
    g = np.zeros(81)
    V = 0.0
    for _, dN, det in fem.ref_gradients(X[None]):
        g += det[0] * dN[0].reshape(-1)
        V += det[0]
    assert np.allclose(K[0], Kdev + kap / V * np.outer(g, g), rtol=1e-10, atol=1e-10 * np.abs(K).max())
    assert np.abs(f).max() < 1e-12


def test_q2_hgo_objectivity_and_translations():
    """K(U)(W x) = W f_int(U) for skew W, x = X + U; translations are in ker K(U)."""
    rng = np.random.default_rng(5)
    X, U, a1, a2 = _hgo_q2(5, 0.04)
    args = (a1[None], a2[None], HGO["c"], HGO["k1"], HGO["k2"], 100.0)
    K, f = fem.hgo_element_tangent(X[None], U[None], *args)
    w = rng.standard_normal(3)
    W = np.array([[0, -w[2], w[1]], [w[2], 0, -w[0]], [-w[1], w[0], 0]])
    x = X + U
    lhs = K[0] @ (x @ W.T).reshape(-1)
    rhs = (f[0].reshape(27, 3) @ W.T).reshape(-1)
    assert np.allclose(lhs, rhs, atol=1e-9 * np.abs(K).max())
    for k in range(3):
        t = np.zeros((27, 3))
        t[:, k] = 1.0
        assert np.abs(K[0] @ t.reshape(-1)).max() <= 1e-11 * np.abs(K).max()


# ---------------------------------------------------------------- FETI on Q2
@pytest.mark.parametrize("variant", ["af", "classical"])
def test_feti_ref_q2_cube_matches_monolithic(variant):
    """The FETI oracle on a Q2 cube in 2^3 subdomains equals the monolithic
    solve (both variants, Dirichlet preconditioner)."""
    m = cube_mesh(4, 2, order=2)
    u_ref = monolithic.solve_linear(m)
    tp = feti_ref.linear_torn_problem(m, variant)
    fr = feti_ref.FetiRef(tp, precond="dirichlet")
    u = fr.solve(rtol=1e-12)["u"]
    assert np.abs(u - u_ref).max() <= 1e-9 * np.abs(u_ref).max()


def test_feti_ref_q2_tube_newton_step_matches_monolithic():
    """One Newton step of the Q2-P0 HGO tube at a stressed state, FETI
    oracle (all-floating) against the monolithic Newton increment."""
    m = tube_mesh(nr=1, nth=8, nz=2, sub=(1, 2, 2), order=2)
    tau = 1 / 40
    dU0, _ = monolithic.newton_increment(m, np.zeros(m.n_dofs), tau)
    U = 0.5 * dU0
    dU_ref, _ = monolithic.newton_increment(m, U, tau)
    tp = feti_ref.newton_torn_problem(m, U, tau, "af")
    fr = feti_ref.FetiRef(tp, precond="dirichlet")
    dU = fr.solve(rtol=1e-12)["u"]
    assert np.abs(dU - dU_ref).max() <= 1e-8 * np.abs(dU_ref).max()


def _l2_error_q2(mesh, u, exact_fn, npts=5):
    """||u - u_h||_L2 of a Q2 mesh with an npts^3 Gauss-Legendre rule per
    element (written here, apart from the oracle's 3-point rule)."""
    pts, wts = np.polynomial.legendre.leggauss(npts)
    Xe = mesh.xyz[mesh.hex8]
    ue = u.reshape(-1, 3)[mesh.hex8]
    err2 = 0.0
    for a, wa in zip(pts, wts):
        for b, wb in zip(pts, wts):
            for c, wc in zip(pts, wts):
                N, dN = fem.shape_hex27([a, b, c])
                x = np.einsum("a,ead->ed", N, Xe)
                det = np.linalg.det(np.einsum("ead,ak->edk", Xe, dN))
                d = np.einsum("a,ead->ed", N, ue) - exact_fn(x)
                err2 += np.sum(wa * wb * wc * det * np.sum(d * d, axis=1))
    return np.sqrt(err2)


def test_q2_kelvin_third_order():
    """Kelvin's solution as Dirichlet data: the L2 error of the quadratic
    elements falls with order 3 (section 5.1, eqs. (fundSol), (L2Error); the
    paper's table of the linear cube with quadratic ansatz functions shows
    eoc 2.97-3.01)."""
    from workloads import kelvin_displacement
    E, nu = 1.0, 0.3
    errs = []
    for n in (2, 4, 8):
        m = cube_mesh(n, 1, E=E, nu=nu, body_force=None, order=2,
                      dirichlet_fn=lambda x: kelvin_displacement(x, E, nu))
        u = monolithic.solve_linear(m)
        errs.append(_l2_error_q2(m, u, lambda x: kelvin_displacement(x, E, nu)))
    eoc = [np.log(errs[i] / errs[i + 1]) / np.log(2.0) for i in range(2)]
    assert 2.6 < eoc[0] < 3.4 and 2.8 < eoc[1] < 3.2, (errs, eoc)


def test_q2_tube_recipe_geometry_and_face_orientation():
    """The Q2 tube's nodes lie on their cylinders (mid-side nodes included),
    it has the Q1 tube's element layers, media/adventitia split and fibres,
    and every 9-node pressure face has dx/ds x dx/dt pointing out of the wall
    (towards the axis) at its centre."""
    m2 = tube_mesh(nr=2, nth=16, nz=4, sub=(1, 4, 2), order=2)
    m1 = tube_mesh(nr=2, nth=16, nz=4, sub=(1, 4, 2))
    r = np.sqrt(m2.xyz[:, 0] ** 2 + m2.xyz[:, 1] ** 2)
    radii = 1.0 + 0.3 * np.arange(5) / 4
    assert np.abs(r[:, None] - radii[None, :]).min(axis=1).max() < 1e-14
    assert np.array_equal(m2.elem_mat, m1.elem_mat) and np.allclose(m2.fibers, m1.fibers)
    xf = m2.xyz[m2.pface]
    _, dLs = fem._lagrange3(0.0)
    Ls, _ = fem._lagrange3(0.0)
    ds = np.array([dLs[a % 3] * Ls[a // 3] for a in range(9)])
    dt = np.array([Ls[a % 3] * dLs[a // 3] for a in range(9)])
    n = np.cross(np.einsum("fad,a->fd", xf, ds), np.einsum("fad,a->fd", xf, dt))
    c = xf[:, 4]
    radial = n[:, 0] * c[:, 0] + n[:, 1] * c[:, 1]
    assert (radial < 0).all()
    assert np.allclose(np.sqrt(c[:, 0] ** 2 + c[:, 1] ** 2), 1.0)


def test_q2_workloads_share_the_q1_nodes():
    """tube_q2_8x64x32 has exactly the nodes (coordinates and numbering),
    Dirichlet DOFs and subdomain boxes of tube_16x128x64, and cube_q2_16_s4
    those of cube32_s4."""
    from workloads import config_mesh
    for q2, q1 in (("tube_q2_8x64x32", "tube_16x128x64"), ("cube_q2_16_s4", "cube32_s4")):
        a, b = config_mesh(q2), config_mesh(q1)
        assert a.order == 2 and b.order == 1
        assert np.array_equal(a.xyz, b.xyz)
        assert np.array_equal(a.dir_dof, b.dir_dof)
        assert a.n_sub == b.n_sub
        # the Q1 element whose first corner is a Q2 element's centre node lies
        # inside that Q2 element: both are in the same subdomain box
        centre = a.hex8[:, 13]
        q1_sub_at_centre = np.full(b.n_nodes, -1)
        np.put(q1_sub_at_centre, b.hex8[:, 0], b.elem_sub)
        assert np.array_equal(q1_sub_at_centre[centre], a.elem_sub)
