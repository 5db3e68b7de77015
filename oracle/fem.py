"""Q1 and Q2 hexahedral finite elements, written plainly in NumPy (FP64).

Oracle module (test infrastructure only).  Each function cites the passage of
the paper it follows.

* Isotropic linear elasticity: K_e = int B^T D B dX with Lame constants from
  (E, nu); used by the linear cube experiments (section 5.1).
* Holzapfel-Gasser-Ogden material (section 2, eqs. (decompositionStrain),
  (iso), (aniso_1), (aniso_2)): the strain energy is written out, the second
  Piola-Kirchhoff stress follows the additive split of eq. (additiveStress),
  and the volumetric part uses a pressure that is constant per element and
  condensed element-wise (section 3.2, static condensation, P0 pressure;
  the paper's Q1-P0 and Q2-P0 pairs).
* The element internal force is the weak form of eq. (WeakReference); the
  consistent tangent of eq. (Tangent) is obtained as the exact derivative of
  that internal force by complex-step differentiation, so no closed-form
  elasticity tensor is needed here (the paper leaves it to its references).
* Follower pressure on the current surface without load stiffness
  (section 3.2, last paragraph).

Elements: Q1 = 8-node trilinear hexahedron, local node a = i + 2j + 4k at
reference point (2i-1, 2j-1, 2k-1), 2x2x2 Gauss points; Q2 = 27-node
triquadratic hexahedron (section 3.2's quadratic elements), local node
a = i + 3j + 9k at (i-1, j-1, k-1), 3x3x3 Gauss points.  The element order is
read from the number of nodes per element (8 or 27).  Pressure faces: Q1
quadrilaterals of 4 corners (counter-clockwise, 2x2 Gauss points) and Q2
quadrilaterals of 9 nodes (node i + 3j at face point (i-1, j-1), 3x3 Gauss
points); both oriented so that dx/ds x dx/dt points out of the body.
"""
from __future__ import annotations

import numpy as np

# reference corner coordinates of local node a = i + 2j + 4k
XI = np.array([[2 * (a & 1) - 1, 2 * ((a >> 1) & 1) - 1, 2 * ((a >> 2) & 1) - 1]
               for a in range(8)], dtype=np.float64)
_G = 1.0 / np.sqrt(3.0)
GAUSS_PTS = XI * _G          # 8 points, unit weights

# Q2: reference nodes of local node a = i + 3j + 9k, and the 3-point Gauss rule
XI27 = np.array([[a % 3 - 1, (a // 3) % 3 - 1, a // 9 - 1] for a in range(27)], dtype=np.float64)
_G3 = np.sqrt(0.6)
_G3_PTS = np.array([-_G3, 0.0, _G3])
_G3_WTS = np.array([5.0, 8.0, 5.0]) / 9.0


def shape_hex8(xi):
    """Trilinear shape functions N_a and dN_a/dxi at one reference point."""
    xi = np.asarray(xi, dtype=np.float64)
    f = 1.0 + XI * xi[None, :]             # (8,3)
    N = 0.125 * f.prod(axis=1)
    dN = np.empty((8, 3))
    for k in range(3):
        others = [d for d in range(3) if d != k]
        dN[:, k] = 0.125 * XI[:, k] * f[:, others[0]] * f[:, others[1]]
    return N, dN


def _lagrange3(x):
    """1D quadratic Lagrange polynomials on the nodes -1, 0, 1 and their
    derivatives at x: ([L_-1, L_0, L_1], [L'_-1, L'_0, L'_1])."""
    return (np.array([0.5 * x * (x - 1.0), 1.0 - x * x, 0.5 * x * (x + 1.0)]),
            np.array([x - 0.5, -2.0 * x, x + 0.5]))


def shape_hex27(xi):
    """Triquadratic shape functions N_a and dN_a/dxi at one reference point:
    products of 1D quadratic Lagrange polynomials, node a = i + 3j + 9k."""
    xi = np.asarray(xi, dtype=np.float64)
    L = [_lagrange3(xi[d]) for d in range(3)]
    N = np.empty(27)
    dN = np.empty((27, 3))
    for a in range(27):
        ijk = (a % 3, (a // 3) % 3, a // 9)
        v = [L[d][0][ijk[d]] for d in range(3)]
        dv = [L[d][1][ijk[d]] for d in range(3)]
        N[a] = v[0] * v[1] * v[2]
        dN[a] = (dv[0] * v[1] * v[2], v[0] * dv[1] * v[2], v[0] * v[1] * dv[2])
    return N, dN


_SHAPES = [shape_hex8(g) for g in GAUSS_PTS]
_WEIGHTS = np.ones(8)
_SHAPES27 = []
_WEIGHTS27 = []
for _k in range(3):
    for _j in range(3):
        for _i in range(3):
            _SHAPES27.append(shape_hex27([_G3_PTS[_i], _G3_PTS[_j], _G3_PTS[_k]]))
            _WEIGHTS27.append(_G3_WTS[_i] * _G3_WTS[_j] * _G3_WTS[_k])


def ref_gradients(Xe):
    """For each Gauss point of elements Xe [ne, npe, 3] (npe = 8: Q1, 27: Q2):
    (N, dN/dX [ne,npe,3], dV [ne]) with dV = Gauss weight x det(dX/dxi), the
    quadrature weight of the point in the reference configuration."""
    npe = Xe.shape[1]
    shapes, weights = (_SHAPES, _WEIGHTS) if npe == 8 else (_SHAPES27, _WEIGHTS27)
    out = []
    for (N, dNxi), wq in zip(shapes, weights):
        Jm = np.einsum("ead,ak->edk", Xe, dNxi)           # dX_d/dxi_k
        det = np.linalg.det(Jm)
        inv = np.linalg.inv(Jm)                             # dxi_k/dX_d
        dNX = np.einsum("ak,ekd->ead", dNxi, inv)
        out.append((N, dNX, wq * det))
    return out


def lame(E, nu):
    E = np.asarray(E, dtype=np.float64)
    nu = np.asarray(nu, dtype=np.float64)
    lam = E * nu / ((1.0 + nu) * (1.0 - 2.0 * nu))
    mu = E / (2.0 * (1.0 + nu))
    return lam, mu


def linear_stiffness(Xe, lam, mu):
    """Element stiffness of isotropic linear elasticity, K_e[3a+i, 3b+j].

    The bilinear form is int (lam div v div w + 2 mu eps(v):eps(w)) dX, i.e.
    K_{ai,bj} = int lam dN_a/dX_i dN_b/dX_j + mu (dN_a/dX_j dN_b/dX_i
    + delta_ij grad N_a . grad N_b) dX.
    """
    ne, npe = Xe.shape[:2]
    lam = np.broadcast_to(np.asarray(lam, dtype=np.float64), (ne,))
    mu = np.broadcast_to(np.asarray(mu, dtype=np.float64), (ne,))
    K = np.zeros((ne, npe, 3, npe, 3))
    eye = np.eye(3)
    for _, dN, det in ref_gradients(Xe):
        w = det
        t1 = np.einsum("eai,ebj->eaibj", dN, dN)
        t2 = np.einsum("eaj,ebi->eaibj", dN, dN)
        dot = np.einsum("eak,ebk->eab", dN, dN)
        t3 = dot[:, :, None, :, None] * eye[None, None, :, None, :]
        K += w[:, None, None, None, None] * (lam[:, None, None, None, None] * t1
                                             + mu[:, None, None, None, None] * (t2 + t3))
    return K.reshape(ne, 3 * npe, 3 * npe)


def body_force_vector(Xe, b):
    """f_e[3a+i] = int N_a b_i dX for a force b [ne,3] per unit reference volume."""
    ne, npe = Xe.shape[:2]
    f = np.zeros((ne, npe, 3))
    for N, _, det in ref_gradients(Xe):
        f += det[:, None, None] * N[None, :, None] * b[:, None, :]
    return f.reshape(ne, 3 * npe)


# ---------------------------------------------------------------------------
# Holzapfel-Gasser-Ogden model
# ---------------------------------------------------------------------------

def _inv3(A):
    """Inverse and determinant of a stack of 3x3 matrices (real or complex)."""
    a, b, c = A[..., 0, 0], A[..., 0, 1], A[..., 0, 2]
    d, e, f = A[..., 1, 0], A[..., 1, 1], A[..., 1, 2]
    g, h, i = A[..., 2, 0], A[..., 2, 1], A[..., 2, 2]
    co00 = e * i - f * h
    co01 = -(d * i - f * g)
    co02 = d * h - e * g
    det = a * co00 + b * co01 + c * co02
    inv = np.empty_like(A)
    inv[..., 0, 0] = co00
    inv[..., 1, 0] = co01
    inv[..., 2, 0] = co02
    inv[..., 0, 1] = -(b * i - c * h)
    inv[..., 1, 1] = a * i - c * g
    inv[..., 2, 1] = -(a * h - b * g)
    inv[..., 0, 2] = b * f - c * e
    inv[..., 1, 2] = -(a * f - c * d)
    inv[..., 2, 2] = a * e - b * d
    inv /= det[..., None, None]
    return inv, det


def _fibre_terms(C, Jm23, a, k1, k2, active=None):
    """E = Ibar_4 - 1, the fibre stretch measure, and dPsi/dIbar_4 (zero unless E > 0).

    With a unit fibre a, Ibar_4 - 1 = J^{-2/3} a.(C - I)a + (J^{-2/3} - 1); this form
    is exactly zero at C = I, so the tension-only switch does not flip on rounding
    of |a|^2 in the reference state.
    """
    eye = np.eye(3)
    E = Jm23 * np.einsum("...i,...ij,...j->...", a, C - eye, a) + (Jm23 - 1.0)
    if active is None:
        active = np.real(E) > 0.0             # fibres carry tension only (section 2)
    dpsi = np.where(active, k1 * E * np.exp(k2 * E * E), 0.0)
    psi = np.where(active, k1 / (2.0 * k2) * (np.exp(k2 * E * E) - 1.0), 0.0)
    return E, dpsi, psi, active


def hgo_isochoric_energy(C, a1, a2, c, k1, k2):
    """Psi_iso + Psi_aniso(a1) + Psi_aniso(a2) of eqs. (iso), (aniso_1), (aniso_2)."""
    _, J2 = _inv3(C)
    Jm23 = J2 ** (-1.0 / 3.0)
    I1 = Jm23 * np.einsum("...ii->...", C)
    _, _, p4, _ = _fibre_terms(C, Jm23, a1, k1, k2)
    _, _, p6, _ = _fibre_terms(C, Jm23, a2, k1, k2)
    return 0.5 * c * (I1 - 3.0) + p4 + p6


def hgo_isochoric_stress(C, a1, a2, c, k1, k2, act=None, return_act=False):
    """S_iso = 2 dPsi_bar/dC for the HGO energy (isochoric part of eq. (additiveStress)).

    With Sbar = c I + 2 psi4' a1(x)a1 + 2 psi6' a2(x)a2 the chain rule through
    Cbar = J^{-2/3} C gives S_iso = J^{-2/3} (Sbar - (Sbar:C)/3 C^{-1}).
    Works for complex input (used for complex-step derivatives); ``act`` fixes
    the fibre activity (decided at the real base state) for such evaluations.
    """
    Cinv, J2 = _inv3(C)
    Jm23 = J2 ** (-1.0 / 3.0)
    _, d4, _, a4 = _fibre_terms(C, Jm23, a1, k1, k2, None if act is None else act[0])
    _, d6, _, a6 = _fibre_terms(C, Jm23, a2, k1, k2, None if act is None else act[1])
    eye = np.eye(3)
    Sbar = (np.asarray(c)[..., None, None] * eye + 2.0 * d4[..., None, None] * np.einsum("...i,...j->...ij", a1, a1)
            + 2.0 * d6[..., None, None] * np.einsum("...i,...j->...ij", a2, a2))
    tr = np.einsum("...ij,...ij->...", Sbar, C)
    S = Jm23[..., None, None] * (Sbar - (tr / 3.0)[..., None, None] * Cinv)
    return (S, (a4, a6)) if return_act else S


def _deformation(Xe, Ue):
    """Per Gauss point: (N, dN/dX, detJ0, F) with F = I + Grad U."""
    out = []
    eye = np.eye(3)
    for N, dNX, det0 in ref_gradients(Xe):
        F = eye[None] + np.einsum("eai,eaJ->eiJ", Ue, dNX)
        out.append((N, dNX, det0, F))
    return out


def hgo_element_energy(Xe, Ue, a1, a2, c, k1, k2, kappa):
    """Pi_e = int Psi_bar(C) dX + V_e kappa/2 (Jbar_e - 1)^2 with Jbar_e = v_e / V_e.

    The volumetric energy Psi_vol = kappa/2 (J-1)^2 is evaluated on the element
    mean dilatation, which is the element-wise condensation of a P0 pressure.
    """
    W = 0.0
    V = 0.0
    v = 0.0
    for _, _, det0, F in _deformation(Xe, Ue):
        C = np.einsum("...kI,...kJ->...IJ", F, F)
        W = W + det0 * hgo_isochoric_energy(C, a1, a2, c, k1, k2)
        _, J = _inv3(F)
        V = V + det0
        v = v + det0 * J
    Jbar = v / V
    return W + V * 0.5 * kappa * (Jbar - 1.0) ** 2


def hgo_element_force(Xe, Ue, a1, a2, c, k1, k2, kappa, acts=None, return_acts=False):
    """Internal force f_e[3a+i] = dPi_e/du_ai (eq. (WeakReference), left side).

    Isochoric part: int F S_iso Grad N_a dX.  Volumetric part: p_e g_a with
    p_e = kappa (Jbar_e - 1) and g_a = dv_e/du_a = int J F^{-T} Grad N_a dX.
    Returns (f [ne,3 npe], p_e [ne], Jbar [ne]) (and the fibre activity per
    Gauss point if ``return_acts``); ``acts`` imposes a previously decided
    activity.
    """
    ne, npe = Xe.shape[:2]
    dtype = np.result_type(Ue, np.float64)
    f = np.zeros((ne, npe, 3), dtype=dtype)
    g = np.zeros((ne, npe, 3), dtype=dtype)
    V = np.zeros(ne)
    v = np.zeros(ne, dtype=dtype)
    out_acts = []
    for q, (_, dNX, det0, F) in enumerate(_deformation(Xe, Ue)):
        C = np.einsum("ekI,ekJ->eIJ", F, F)
        S, act = hgo_isochoric_stress(C, a1, a2, c, k1, k2, None if acts is None else acts[q],
                                      return_act=True)
        out_acts.append(act)
        Finv, J = _inv3(F)
        P = np.einsum("eiI,eIJ->eiJ", F, S)
        f += det0[:, None, None] * np.einsum("eiJ,eaJ->eai", P, dNX)
        # J F^{-T} Grad N_a : (J F^{-T})_{iI} = J Finv_{Ii}
        g += (det0 * J)[:, None, None] * np.einsum("eIi,eaI->eai", Finv, dNX)
        V += det0
        v = v + det0 * J
    Jbar = v / V
    p = kappa * (Jbar - 1.0)
    f = f + p[:, None, None] * g
    if return_acts:
        return f.reshape(ne, 3 * npe), p, Jbar, out_acts
    return f.reshape(ne, 3 * npe), p, Jbar


def hgo_element_tangent(Xe, Ue, a1, a2, c, k1, k2, kappa, h=1e-30):
    """Consistent tangent K_e = d f_e / d u_e (eq. (Tangent) with the condensed
    pressure), computed exactly by complex-step differentiation of
    :func:`hgo_element_force`: column (b,j) is Im f(u + i h e_bj) / h.
    Returns (K [ne,3 npe,3 npe], f [ne,3 npe]).
    """
    ne, npe = Xe.shape[:2]
    f0, _, _, acts = hgo_element_force(Xe, Ue, a1, a2, c, k1, k2, kappa, return_acts=True)
    K = np.empty((ne, 3 * npe, 3 * npe))
    Uc = Ue.astype(np.complex128)
    for col in range(3 * npe):
        a, j = divmod(col, 3)
        Up = Uc.copy()
        Up[:, a, j] += 1j * h
        fc, _, _ = hgo_element_force(Xe, Up, a1, a2, c, k1, k2, kappa, acts=acts)
        K[:, :, col] = fc.imag / h
    return K, f0.real


def _face_rule(nfn):
    """Shape values and derivatives of the face element at its Gauss points:
    [(w, N [nfn], dN/ds [nfn], dN/dt [nfn])]; nfn = 4 (Q1, 2x2 points) or 9
    (Q2, 3x3 points)."""
    out = []
    if nfn == 4:
        eta = np.array([[-1, -1], [1, -1], [1, 1], [-1, 1]], dtype=np.float64)
        for g1 in (-_G, _G):
            for g2 in (-_G, _G):
                N = 0.25 * (1 + eta[:, 0] * g1) * (1 + eta[:, 1] * g2)
                d1 = 0.25 * eta[:, 0] * (1 + eta[:, 1] * g2)
                d2 = 0.25 * eta[:, 1] * (1 + eta[:, 0] * g1)
                out.append((1.0, N, d1, d2))
        return out
    for j in range(3):
        for i in range(3):
            Ls, dLs = _lagrange3(_G3_PTS[i])
            Lt, dLt = _lagrange3(_G3_PTS[j])
            N = np.array([Ls[a % 3] * Lt[a // 3] for a in range(9)])
            d1 = np.array([dLs[a % 3] * Lt[a // 3] for a in range(9)])
            d2 = np.array([Ls[a % 3] * dLt[a // 3] for a in range(9)])
            out.append((_G3_WTS[i] * _G3_WTS[j], N, d1, d2))
    return out


def pressure_face_load(xf, p):
    """Follower pressure load on quadrilateral faces in the current geometry.

    f_a = -p int N_a n da, with n da = (dx/ds x dx/dt) ds dt; the node order
    makes this normal point out of the body.  xf [nf,nfn,3] -> [nf,nfn,3]
    with nfn = 4 (Q1 faces) or 9 (Q2 faces).
    """
    f = np.zeros_like(xf)
    for w, N, d1, d2 in _face_rule(xf.shape[1]):
        t1 = np.einsum("fad,a->fd", xf, d1)
        t2 = np.einsum("fad,a->fd", xf, d2)
        n = np.cross(t1, t2)
        f += -p * w * N[None, :, None] * n[:, None, :]
    return f


def pressure_load_stiffness(xf, p, h=1e-30):
    """Derivative of the follower pressure load with respect to the current
    node positions, D[f, 3a+i, 3b+j] = d f_ai / d x_bj (xf [nf,nfn,3]).

    The paper drops this term from the tangent and notes that keeping it
    makes the system non-symmetric (section 3.2, last paragraph).  Computed
    exactly by complex-step differentiation of :func:`pressure_face_load`.
    """
    nf, nfn = xf.shape[:2]
    D = np.empty((nf, 3 * nfn, 3 * nfn))
    xc = np.asarray(xf, dtype=np.complex128)
    for col in range(3 * nfn):
        b, j = divmod(col, 3)
        xp = xc.copy()
        xp[:, b, j] += 1j * h
        D[:, :, col] = pressure_face_load(xp, p).reshape(nf, 3 * nfn).imag / h
    return D


# ---------------------------------------------------------------------------
# global assembly
# ---------------------------------------------------------------------------

def _elem_material(mesh):
    m = mesh.mat[mesh.elem_mat]
    return m


def element_matrices(mesh, U=None, chunk=4096, elems=None):
    """Element tangents and internal forces for every element of ``mesh``
    (or the elements listed in ``elems``).

    Linear material: K_e = int B^T D B and f_int = K_e u_e.  HGO: exact tangent
    and internal force at displacement U (global [n_nodes,3] or None = 0).
    """
    from workloads.meshes import MAT_HGO
    el = np.arange(mesh.n_elems) if elems is None else np.asarray(elems)
    ne = el.size
    hex8 = mesh.hex8[el]
    Xe = mesh.xyz[hex8]
    Ue = np.zeros_like(Xe) if U is None else np.asarray(U).reshape(-1, 3)[hex8]
    m = _elem_material(mesh)[el]
    nde = 3 * hex8.shape[1]
    Ke = np.empty((ne, nde, nde))
    fe = np.zeros((ne, nde))
    hgo = m[:, 0] == MAT_HGO
    lin = ~hgo
    if lin.any():
        idx = np.nonzero(lin)[0]
        lam, mu = lame(m[idx, 1], m[idx, 2])
        for s in range(0, idx.size, chunk):
            ii = idx[s:s + chunk]
            Ke[ii] = linear_stiffness(Xe[ii], lam[s:s + chunk], mu[s:s + chunk])
            fe[ii] = np.einsum("eij,ej->ei", Ke[ii], Ue[ii].reshape(-1, nde))
    if hgo.any():
        idx = np.nonzero(hgo)[0]
        for s in range(0, idx.size, chunk):
            ii = idx[s:s + chunk]
            mm = m[ii]
            a1 = mesh.fibers[el[ii], 0]
            a2 = mesh.fibers[el[ii], 1]
            K, f = hgo_element_tangent(Xe[ii], Ue[ii], a1, a2, mm[:, 3], mm[:, 4], mm[:, 5],
                                       mm[:, 6])
            Ke[ii] = K
            fe[ii] = f
    return Ke, fe


def assemble(mesh, U=None, tau=1.0):
    """Global tangent K (CSR), internal force f_int and external load tau*f_ext.

    f_ext = body force (dead load) + follower pressure on the geometry X + U.
    """
    import scipy.sparse as sp
    Ke, fe = element_matrices(mesh, U)
    nde = 3 * mesh.hex8.shape[1]
    dofs = (3 * mesh.hex8[:, :, None] + np.arange(3)[None, None, :]).reshape(-1, nde)
    rows = np.repeat(dofs, nde, axis=1).ravel()
    cols = np.tile(dofs, (1, nde)).ravel()
    n = mesh.n_dofs
    K = sp.coo_matrix((Ke.ravel(), (rows, cols)), shape=(n, n)).tocsr()
    K.sum_duplicates()
    f_int = np.bincount(dofs.ravel(), weights=fe.ravel(), minlength=n)
    f_ext = np.zeros(n)
    if mesh.body_force is not None:
        Xe = mesh.xyz[mesh.hex8]
        fb = body_force_vector(Xe, mesh.body_force)
        f_ext += np.bincount(dofs.ravel(), weights=fb.ravel(), minlength=n)
    if mesh.pface is not None and mesh.pressure != 0.0:
        x = mesh.xyz + (0.0 if U is None else np.asarray(U).reshape(-1, 3))
        fp = pressure_face_load(x[mesh.pface], mesh.pressure)
        pd = (3 * mesh.pface[:, :, None] + np.arange(3)[None, None, :]).ravel()
        f_ext += np.bincount(pd, weights=fp.ravel(), minlength=n)
    return K, f_int, tau * f_ext


def assemble_load_stiffness(mesh, U=None):
    """Global derivative of the follower pressure load f_p(X + U) with respect
    to U (CSR, n_dofs x n_dofs); zero without pressure faces."""
    import scipy.sparse as sp
    n = mesh.n_dofs
    if mesh.pface is None or mesh.pressure == 0.0:
        return sp.csr_matrix((n, n))
    x = mesh.xyz + (0.0 if U is None else np.asarray(U).reshape(-1, 3))
    D = pressure_load_stiffness(x[mesh.pface], mesh.pressure)
    ndf = 3 * mesh.pface.shape[1]
    dofs = (3 * mesh.pface[:, :, None] + np.arange(3)[None, None, :]).reshape(-1, ndf)
    rows = np.repeat(dofs, ndf, axis=1).ravel()
    cols = np.tile(dofs, (1, ndf)).ravel()
    A = sp.coo_matrix((D.ravel(), (rows, cols)), shape=(n, n)).tocsr()
    A.sum_duplicates()
    return A


def nodal_residual(mesh, nodes, u, U=None, tau=1.0):
    """Rows of the linear(ised) system at sampled nodes, from the elements and
    pressure faces around them only.

    The system is K'(U) u = tau f_ext(U) - f_int(U) (U = None: the linear
    problem K u = tau f_ext).  Returns (res, scale), both [len(nodes), 3]:
    res = tau f_ext - f_int - K' u on each DOF of the nodes, and scale = the
    sum of the magnitudes of the element and load terms of that row, so that
    |res| / scale is a componentwise relative residual.  Rows of Dirichlet
    DOFs are returned as 0 with scale 1.
    """
    nodes = np.asarray(nodes, dtype=np.int64)
    u = np.asarray(u, dtype=np.float64).reshape(-1, 3)
    elems = np.nonzero(np.isin(mesh.hex8, nodes).any(axis=1))[0]
    Ke, fe = element_matrices(mesh, U, elems=elems)
    hex8 = mesh.hex8[elems]
    npe = hex8.shape[1]
    ue = u[hex8].reshape(-1, 3 * npe)
    Ku = np.einsum("eij,ej->ei", Ke, ue)
    pos = {int(n): k for k, n in enumerate(nodes)}
    res = np.zeros((nodes.size, 3))
    scale = np.zeros((nodes.size, 3))
    loc = np.array([[pos.get(int(n), -1) for n in row] for row in hex8])
    fb = None
    if mesh.body_force is not None:
        fb = body_force_vector(mesh.xyz[hex8], mesh.body_force[elems])
    for e in range(elems.size):
        for a in range(npe):
            k = loc[e, a]
            if k < 0:
                continue
            sl = slice(3 * a, 3 * a + 3)
            res[k] -= Ku[e, sl] + (0.0 if U is None else fe[e, sl])
            scale[k] += np.abs(Ke[e, sl, :]) @ np.abs(ue[e]) + (0.0 if U is None else np.abs(fe[e, sl]))
            if fb is not None:
                res[k] += tau * fb[e, sl]
                scale[k] += np.abs(tau * fb[e, sl])
    if mesh.pface is not None and mesh.pressure != 0.0:
        faces = np.nonzero(np.isin(mesh.pface, nodes).any(axis=1))[0]
        if faces.size:
            x = mesh.xyz + (0.0 if U is None else np.asarray(U).reshape(-1, 3))
            fp = pressure_face_load(x[mesh.pface[faces]], mesh.pressure)
            for q, f in enumerate(faces):
                for a in range(mesh.pface.shape[1]):
                    k = pos.get(int(mesh.pface[f, a]), -1)
                    if k >= 0:
                        res[k] += tau * fp[q, a]
                        scale[k] += np.abs(tau * fp[q, a])
    dmask = np.zeros(mesh.n_dofs, dtype=bool)
    dmask[mesh.dir_dof] = True
    dm = dmask.reshape(-1, 3)[nodes]
    res[dm] = 0.0
    scale[dm] = 1.0
    return res, scale
