"""Structured hexahedral problems (Q1 or Q2) with a non-overlapping element
partition.

Conventions (shared by every consumer):
  * node ids are global, coordinates ``xyz[n_nodes, 3]`` (float64);
  * ``hex8[n_elems, npe]`` lists the nodes of each hexahedron in lexicographic
    order, x fastest.  Q1 (npe = 8): local corner ``a = i + 2 j + 4 k`` sits at
    reference coordinates ``(2i-1, 2j-1, 2k-1)``.  Q2 (npe = 27, the 27-node
    triquadratic element): local node ``a = i + 3 j + 9 k`` sits at
    ``(i-1, j-1, k-1)``;
  * ``elem_sub[e]`` is the subdomain of element ``e`` (the tearing of the
    domain into non-overlapping subdomains, paper section 4, eq. (decomposition));
  * a Dirichlet degree of freedom is ``3*node + component``;
  * ``body_force[e]`` is a constant force per unit reference volume;
  * ``pface[f]`` holds the nodes of a quadrilateral loaded by a follower
    pressure: Q1, four corners ordered so that the right-hand normal of
    (x1 - x0) x (x3 - x0) points out of the body; Q2, nine nodes, node
    ``i + 3 j`` at face coordinates ``(s, t) = (i-1, j-1)`` with
    dx/ds x dx/dt pointing out of the body.

Materials: ``mat`` is a float64 table with one row per material,
``[kind, E, nu, c, k1, k2, kappa]`` where kind 0 is isotropic linear elasticity
and kind 1 the Holzapfel-Gasser-Ogden model with a condensed P0 pressure.
"""
from __future__ import annotations

from dataclasses import dataclass, field
import numpy as np

MAT_LINEAR = 0
MAT_HGO = 1


@dataclass
class Mesh:
    xyz: np.ndarray                 # [n_nodes, 3] f64
    hex8: np.ndarray                # [n_elems, 8 or 27] i64 (Q1 or Q2)
    elem_sub: np.ndarray            # [n_elems] i32
    n_sub: int
    mat: np.ndarray                 # [n_mat, 7] f64 (kind, E, nu, c, k1, k2, kappa)
    elem_mat: np.ndarray            # [n_elems] i32
    dir_dof: np.ndarray             # [n_dir] i64
    dir_val: np.ndarray             # [n_dir] f64
    body_force: np.ndarray | None = None   # [n_elems, 3] f64
    fibers: np.ndarray | None = None       # [n_elems, 2, 3] f64 unit vectors
    pface: np.ndarray | None = None        # [n_pfaces, 4 or 9] i64
    pressure: float = 0.0
    name: str = ""
    meta: dict = field(default_factory=dict)

    @property
    def n_nodes(self) -> int:
        return int(self.xyz.shape[0])

    @property
    def n_elems(self) -> int:
        return int(self.hex8.shape[0])

    @property
    def n_dofs(self) -> int:
        return 3 * self.n_nodes

    @property
    def order(self) -> int:
        """Polynomial order of the elements: 1 (8 nodes) or 2 (27 nodes)."""
        return 1 if self.hex8.shape[1] == 8 else 2


def _grid_nodes(nx, ny, nz, lx=1.0, ly=1.0, lz=1.0):
    x = np.linspace(0.0, lx, nx + 1)
    y = np.linspace(0.0, ly, ny + 1)
    z = np.linspace(0.0, lz, nz + 1)
    Z, Y, X = np.meshgrid(z, y, x, indexing="ij")
    return np.stack([X.ravel(), Y.ravel(), Z.ravel()], axis=1)


def _grid_hex(nx, ny, nz):
    """Hexahedra of an (nx, ny, nz) element grid; element id = ex + nx*(ey + ny*ez)."""
    ez, ey, ex = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    ex, ey, ez = ex.ravel(), ey.ravel(), ez.ravel()
    sx, sy = nx + 1, (nx + 1) * (ny + 1)
    base = ex + sx * ey + sy * ez
    offs = np.array([0, 1, sx, sx + 1, sy, sy + 1, sy + sx, sy + sx + 1], dtype=np.int64)
    return (base[:, None] + offs[None, :]).astype(np.int64), np.stack([ex, ey, ez], axis=1)


def _grid_hex27(nx, ny, nz):
    """27-node hexahedra of an (nx, ny, nz) element grid on the node grid of
    (2nx+1, 2ny+1, 2nz+1) nodes; element id = ex + nx*(ey + ny*ez)."""
    ez, ey, ex = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    ex, ey, ez = ex.ravel(), ey.ravel(), ez.ravel()
    sx, sy = 2 * nx + 1, (2 * nx + 1) * (2 * ny + 1)
    base = 2 * ex + sx * 2 * ey + sy * 2 * ez
    offs = np.array([i + sx * j + sy * k for k in range(3) for j in range(3) for i in range(3)], dtype=np.int64)
    return (base[:, None] + offs[None, :]).astype(np.int64), np.stack([ex, ey, ez], axis=1)


def box_partition(cuts_x, cuts_y, cuts_z, elem_ijk):
    """Subdomain id of each element for axis-aligned slab cuts.

    ``cuts_*`` are increasing element indices including 0 and the element count.
    Subdomain id = bx + Bx*(by + By*bz) for box indices (bx, by, bz).
    """
    bx = np.searchsorted(np.asarray(cuts_x), elem_ijk[:, 0], side="right") - 1
    by = np.searchsorted(np.asarray(cuts_y), elem_ijk[:, 1], side="right") - 1
    bz = np.searchsorted(np.asarray(cuts_z), elem_ijk[:, 2], side="right") - 1
    Bx, By = len(cuts_x) - 1, len(cuts_y) - 1
    return (bx + Bx * (by + By * bz)).astype(np.int32)


def _boundary_nodes_cube(nx, ny, nz):
    ids = np.arange((nx + 1) * (ny + 1) * (nz + 1))
    i = ids % (nx + 1)
    j = (ids // (nx + 1)) % (ny + 1)
    k = ids // ((nx + 1) * (ny + 1))
    on = (i == 0) | (i == nx) | (j == 0) | (j == ny) | (k == 0) | (k == nz)
    return ids[on]


def cube_mesh(n_el: int, n_sub_axis: int, *, E=1.0, nu=0.3, nu_per_sub=None,
              body_force=(0.0, 0.0, -1.0), dirichlet="zero", dirichlet_fn=None,
              name="cube", order=1) -> Mesh:
    """Unit cube, ``n_el``^3 Q1 (order 1) or Q2 (order 2) elements, cut into
    ``n_sub_axis``^3 equal boxes.

    Subdomain order is s = ix + m*iy + m*m*iz.  ``nu_per_sub`` (length m^3)
    gives one Poisson ratio per subdomain; otherwise every element has ``nu``.
    Dirichlet data is imposed on all of the cube's surface: zero, or
    ``dirichlet_fn(xyz) -> [n, 3]`` evaluated at the boundary nodes.
    """
    assert n_el % n_sub_axis == 0 and order in (1, 2)
    xyz = _grid_nodes(order * n_el, order * n_el, order * n_el)
    hex8, ijk = _grid_hex(n_el, n_el, n_el) if order == 1 else _grid_hex27(n_el, n_el, n_el)
    h = n_el // n_sub_axis
    cuts = list(range(0, n_el + 1, h))
    elem_sub = box_partition(cuts, cuts, cuts, ijk)
    n_sub = n_sub_axis ** 3
    if nu_per_sub is not None:
        nu_per_sub = np.asarray(nu_per_sub, dtype=np.float64)
        assert nu_per_sub.shape == (n_sub,)
        mat = np.zeros((n_sub, 7))
        mat[:, 0] = MAT_LINEAR
        mat[:, 1] = E
        mat[:, 2] = nu_per_sub
        elem_mat = elem_sub.copy()
    else:
        mat = np.array([[MAT_LINEAR, E, nu, 0, 0, 0, 0]], dtype=np.float64)
        elem_mat = np.zeros(hex8.shape[0], dtype=np.int32)
    bnodes = _boundary_nodes_cube(order * n_el, order * n_el, order * n_el)
    dir_dof = (3 * bnodes[:, None] + np.arange(3)[None, :]).ravel().astype(np.int64)
    if dirichlet_fn is not None:
        dir_val = np.asarray(dirichlet_fn(xyz[bnodes]), dtype=np.float64).reshape(-1)
    else:
        dir_val = np.zeros(dir_dof.shape[0])
    bf = None
    if body_force is not None:
        bf = np.tile(np.asarray(body_force, dtype=np.float64), (hex8.shape[0], 1))
    return Mesh(xyz=xyz, hex8=hex8, elem_sub=elem_sub, n_sub=n_sub, mat=mat,
                elem_mat=elem_mat, dir_dof=dir_dof, dir_val=dir_val, body_force=bf,
                name=name, meta={"n_el": n_el, "n_sub_axis": n_sub_axis, "order": order})


def partial_dirichlet_cube(n_el=8, n_sub_axis=2, **kw) -> Mesh:
    """Unit cube in n_sub_axis^3 boxes whose Dirichlet data touch some
    subdomains only partially: u = 0 on the quarter y, z <= 0.5 of the face
    x = 0, and u_x = 0 (only that component) on the face x = 1.  With 2^3
    boxes, one subdomain holds the clamped quarter face, two touch it along an
    edge, one at a single vertex, and the four at x = 1 have one constrained
    component on a whole face."""
    m = cube_mesh(n_el, n_sub_axis, **kw)
    x = m.xyz
    tol = 1e-12
    clamp = np.nonzero((x[:, 0] < tol) & (x[:, 1] < 0.5 + tol) & (x[:, 2] < 0.5 + tol))[0]
    roller = np.nonzero(x[:, 0] > 1.0 - tol)[0]
    dofs = np.concatenate([(3 * clamp[:, None] + np.arange(3)[None, :]).ravel(), 3 * roller])
    m.dir_dof = np.sort(dofs).astype(np.int64)
    m.dir_val = np.zeros(m.dir_dof.size)
    m.name = "partial_dirichlet_cube"
    return m


def kelvin_displacement(x, E, nu, src=(1.5, 1.5, 1.5)):
    """Kelvin's fundamental solution of linear elastostatics (paper section 5.1,
    eq. (fundSol)): the displacement at ``x`` caused by a unit point force in
    direction 1 applied at ``src`` outside the domain."""
    d = np.asarray(x, dtype=np.float64) - np.asarray(src, dtype=np.float64)[None, :]
    r = np.sqrt((d * d).sum(axis=1))
    c = (1.0 + nu) / (8.0 * np.pi * E * (1.0 - nu))
    u = c * (d[:, 0:1] * d) / r[:, None] ** 3
    u[:, 0] += c * (3.0 - 4.0 * nu) / r
    return u


def random_box_cube(n_el=64, n_box_axis=8, seed=0, *, E=1.0, nu=0.3, lo=4, hi=12,
                    dof_lo=300, dof_hi=6000, n_modes=8) -> Mesh:
    """Unit cube of ``n_el``^3 Q1 elements cut by seeded axis-aligned planes.

    Per axis, ``n_box_axis`` slab widths are integers in [lo, hi] summing to
    ``n_el`` (rejection sampling from ``default_rng(seed)``); a draw is
    rejected if any box has a DOF count outside [dof_lo, dof_hi].  The body
    force is a random smooth field sum_k a_k sin(2 pi w_k.x + phi_k),
    evaluated at element centroids.
    """
    rng = np.random.default_rng(seed)

    def widths():
        while True:
            w = rng.integers(lo, hi + 1, size=n_box_axis)
            if w.sum() == n_el:
                return w

    while True:
        wx, wy, wz = widths(), widths(), widths()
        dofs = 3 * np.einsum("i,j,k->ijk", wx + 1, wy + 1, wz + 1)
        if dofs.min() >= dof_lo and dofs.max() <= dof_hi:
            break
    cx = np.concatenate([[0], np.cumsum(wx)])
    cy = np.concatenate([[0], np.cumsum(wy)])
    cz = np.concatenate([[0], np.cumsum(wz)])
    xyz = _grid_nodes(n_el, n_el, n_el)
    hex8, ijk = _grid_hex(n_el, n_el, n_el)
    elem_sub = box_partition(cx, cy, cz, ijk)
    bnodes = _boundary_nodes_cube(n_el, n_el, n_el)
    dir_dof = (3 * bnodes[:, None] + np.arange(3)[None, :]).ravel().astype(np.int64)
    a = rng.standard_normal((n_modes, 3))
    w = rng.integers(0, 4, size=(n_modes, 3)).astype(np.float64)
    phi = rng.uniform(0.0, 2.0 * np.pi, size=n_modes)
    cen = xyz[hex8].mean(axis=1)
    arg = 2.0 * np.pi * cen @ w.T + phi[None, :]
    bf = np.sin(arg) @ a
    mat = np.array([[MAT_LINEAR, E, nu, 0, 0, 0, 0]], dtype=np.float64)
    return Mesh(xyz=xyz, hex8=hex8, elem_sub=elem_sub, n_sub=n_box_axis ** 3, mat=mat,
                elem_mat=np.zeros(hex8.shape[0], dtype=np.int32), dir_dof=dir_dof,
                dir_val=np.zeros(dir_dof.shape[0]), body_force=bf, name="random_boxes",
                meta={"cuts": (cx, cy, cz), "seed": seed})


# Holzapfel-Gasser-Ogden parameters of the two arterial layers.  The media set
# is the paper's Table 1; the adventitia set and the layer thickness ratio are
# part of the synthetic tube workload.
MEDIA = dict(c=3.0, k1=2.3632, k2=0.8393, angle_deg=29.0)
MMHG = 0.133322          # kPa per mmHg: stresses and moduli are in kPa, as in Table 1
ADVENTITIA = dict(c=0.3, k1=0.562, k2=0.7112, angle_deg=62.0)


def tube_mesh(nr=16, nth=128, nz=64, sub=(1, 16, 8), r_in=1.0, r_out=1.3, length=4.0,
              r_layer=1.2, kappa_factor=1000.0, pressure=16.0 * 0.133322, order=1) -> Mesh:
    """Two-layer thick-walled tube, periodic in the circumferential direction,
    of nr x nth x nz Q1 (order 1) or Q2 (order 2) elements.

    Nodes sit at r_i = r_in + (r_out-r_in) i/(order nr), theta_j = 2 pi
    j/(order nth), z_k = length k/(order nz) (Q2: the mid-side nodes lie on the
    cylinders).  Element (er, et, ez) has id er + nr*(et + nth*ez).  Elements
    whose centroid radius (mean of the eight corners) is below ``r_layer`` are
    media, the others adventitia.  Fibre families are cos(a) e_theta +/- sin(a)
    e_z at that centroid.  Both ends (z=0 and z=length) are clamped.  The inner
    surface carries a follower pressure, in kPa like the material moduli
    (default 16 mmHg).  Subdomains are boxes of the (r, theta, z) element
    grid, id = br + Br*(bt + Bt*bz).
    """
    assert order in (1, 2)
    q = order
    nrn, nthn, nzn = q * nr + 1, q * nth, q * nz + 1
    ri = r_in + (r_out - r_in) * np.arange(nrn) / (q * nr)
    th = 2.0 * np.pi * np.arange(nthn) / (q * nth)
    zk = length * np.arange(nzn) / (q * nz)
    K, J, I = np.meshgrid(np.arange(nzn), np.arange(nthn), np.arange(nrn), indexing="ij")
    I, J, K = I.ravel(), J.ravel(), K.ravel()
    xyz = np.stack([ri[I] * np.cos(th[J]), ri[I] * np.sin(th[J]), zk[K]], axis=1)

    def nid(i, j, k):
        return i + nrn * ((j % nthn) + nthn * k)

    ez, et, er = np.meshgrid(np.arange(nz), np.arange(nth), np.arange(nr), indexing="ij")
    er, et, ez = er.ravel(), et.ravel(), ez.ravel()
    hex8 = np.stack([nid(q * er + di, q * et + dj, q * ez + dk)
                     for dk in range(q + 1) for dj in range(q + 1) for di in range(q + 1)],
                    axis=1).astype(np.int64)
    corners = hex8[:, [0, q, q * (q + 1), q * (q + 1) + q, q * (q + 1) ** 2, q * (q + 1) ** 2 + q,
                       q * (q + 1) ** 2 + q * (q + 1), (q + 1) ** 3 - 1]]
    ijk = np.stack([er, et, ez], axis=1)
    Br, Bt, Bz = sub
    assert nr % Br == 0 and nth % Bt == 0 and nz % Bz == 0
    elem_sub = box_partition(list(range(0, nr + 1, nr // Br)), list(range(0, nth + 1, nth // Bt)),
                             list(range(0, nz + 1, nz // Bz)), ijk)
    cen = xyz[corners].mean(axis=1)
    rc = np.sqrt(cen[:, 0] ** 2 + cen[:, 1] ** 2)
    media = rc < r_layer
    etheta = np.stack([-cen[:, 1] / rc, cen[:, 0] / rc, np.zeros_like(rc)], axis=1)
    ezv = np.zeros_like(etheta)
    ezv[:, 2] = 1.0
    ang = np.where(media, np.deg2rad(MEDIA["angle_deg"]), np.deg2rad(ADVENTITIA["angle_deg"]))
    a1 = np.cos(ang)[:, None] * etheta + np.sin(ang)[:, None] * ezv
    a2 = np.cos(ang)[:, None] * etheta - np.sin(ang)[:, None] * ezv
    fibers = np.stack([a1, a2], axis=1)
    mat = np.array([
        [MAT_HGO, 0, 0, MEDIA["c"], MEDIA["k1"], MEDIA["k2"], kappa_factor * MEDIA["c"]],
        [MAT_HGO, 0, 0, ADVENTITIA["c"], ADVENTITIA["k1"], ADVENTITIA["k2"],
         kappa_factor * ADVENTITIA["c"]],
    ], dtype=np.float64)
    elem_mat = np.where(media, 0, 1).astype(np.int32)
    ends = np.nonzero((K == 0) | (K == q * nz))[0]
    dir_dof = (3 * ends[:, None] + np.arange(3)[None, :]).ravel().astype(np.int64)
    # inner surface faces (radial index 0).  Q1: corners (j,k),(j,k+1),(j+1,k+1),
    # (j+1,k), so x1-x0 runs along +z and x3-x0 along +theta; Q2: node i + 3j at
    # z offset i and theta offset j, so s runs along +z and t along +theta.
    # Either way e_z x e_theta = -e_r points out of the body (towards the axis).
    jj, kk = np.meshgrid(np.arange(nth), np.arange(nz), indexing="ij")
    jj, kk = jj.ravel(), kk.ravel()
    if q == 1:
        pface = np.stack([nid(0, jj, kk), nid(0, jj, kk + 1), nid(0, jj + 1, kk + 1),
                          nid(0, jj + 1, kk)], axis=1).astype(np.int64)
    else:
        pface = np.stack([nid(0, 2 * jj + j, 2 * kk + i) for j in range(3) for i in range(3)],
                         axis=1).astype(np.int64)
    return Mesh(xyz=xyz, hex8=hex8, elem_sub=elem_sub, n_sub=Br * Bt * Bz, mat=mat,
                elem_mat=elem_mat, dir_dof=dir_dof, dir_val=np.zeros(dir_dof.shape[0]),
                body_force=None, fibers=fibers, pface=pface, pressure=float(pressure),
                name="tube", meta={"nr": nr, "nth": nth, "nz": nz, "sub": sub, "order": order})


def _cfg2_nu(seed: int, n_sub: int) -> np.ndarray:
    rng = np.random.default_rng(seed)
    return 0.25 + 0.1 * rng.random(n_sub)


# Named workloads.  "cube8_s2" is the small 2x2x2-subdomain cube; "cube32_s4"
# the 4x4x4-subdomain cube of 8^3-element boxes with per-subdomain Poisson ratios.
CONFIGS = {
    "cube8_s2": dict(kind="cube", n_el=8, n_sub_axis=2),
    "cube32_s4": dict(kind="cube", n_el=32, n_sub_axis=4, nu_seed=0),
    # the nodes and subdomains of cube32_s4 with 16^3 Q2 elements
    "cube_q2_16_s4": dict(kind="cube", n_el=16, n_sub_axis=4, nu_seed=0, order=2),
    "tube_16x128x64": dict(kind="tube", nr=16, nth=128, nz=64, sub=(1, 16, 8)),
    # the same tube with Q2-P0 elements of twice the size: the same nodes
    # (424,320 DOFs) and subdomains, 27-node elements
    "tube_q2_8x64x32": dict(kind="tube", nr=8, nth=64, nz=32, sub=(1, 16, 8), order=2),
    "random_boxes_64": dict(kind="random", n_el=64, n_box_axis=8, seed=0),
    # 40^3 cube in 5x5x5 uneven boxes of 450-5616 DOFs (seed 0): boxes as large
    # as those of random_boxes_64 on a mesh whose direct solve fits a test
    "random_boxes_40": dict(kind="random", n_el=40, n_box_axis=5, seed=0),
}


def config_mesh(name: str, **over) -> Mesh:
    """Build one of the named workloads; keyword overrides replace entries."""
    cfg = dict(CONFIGS[name])
    cfg.update(over)
    kind = cfg.pop("kind")
    if kind == "cube":
        seed = cfg.pop("nu_seed", None)
        m = cfg["n_sub_axis"]
        if seed is not None:
            cfg["nu_per_sub"] = _cfg2_nu(seed, m ** 3)
        return cube_mesh(name=name, **cfg)
    if kind == "tube":
        return tube_mesh(**cfg)
    if kind == "random":
        return random_box_cube(**cfg)
    raise KeyError(name)


# ---------------------------------------------------------------------------
# served request stream
# ---------------------------------------------------------------------------
TUBE_SUBS = {64: (1, 8, 8), 128: (1, 16, 8), 256: (1, 16, 16)}


def request_mesh(key):
    """Mesh of a served request: ("cube", k) = unit cube of (8k)^3 Q1 elements
    in k^3 boxes of 8^3 with nu per box from seed 0; ("tube", p) = the
    16x128x64 two-layer tube in p subdomains; ("tube_small", p) = a 2x16x8
    tube in 1 x p/2 x 2 subdomains (tests)."""
    kind, n = key
    if kind == "cube":
        return config_mesh("cube32_s4", n_el=8 * n, n_sub_axis=n)
    if kind == "tube":
        return tube_mesh(16, 128, 64, sub=TUBE_SUBS[n])
    if kind == "tube_small":
        return tube_mesh(2, 16, 8, sub=(1, n // 2, 2))
    raise KeyError(key)


def request_stream(n, rate, seed=0, cube_k=(2, 8), tube_subs=(64, 128, 256), tube_kind="tube", n_steps=10,
                   iterates=4):
    """n requests with Poisson arrivals of the given rate (per second): half
    cube linear solves with k^3 subdomains, k uniform in cube_k (inclusive),
    and a load factor uniform in [0.5, 2]; half tube Newton steps on one of
    tube_subs subdomain counts at a state (s, k) of the tube's converged load
    path: load step s uniform in 1..n_steps, Newton iterate k uniform in
    0..iterates-1.  Returns a list of dicts (arrival time in s, key, kind,
    parameter)."""
    rng = np.random.default_rng(seed)
    t = np.cumsum(rng.exponential(1.0 / rate, size=n))
    out = []
    for k in range(n):
        if rng.random() < 0.5:
            kk = int(rng.integers(cube_k[0], cube_k[1] + 1))
            out.append(dict(t=float(t[k]), key=("cube", kk), kind="solve",
                            param=float(rng.uniform(0.5, 2.0))))
        else:
            p = int(rng.choice(tube_subs))
            out.append(dict(t=float(t[k]), key=(tube_kind, p), kind="newton",
                            param=(int(rng.integers(1, n_steps + 1)), int(rng.integers(0, iterates)))))
    return out
