"""CPU reference of the classical and all-floating FETI algebra (FP64, dense).

Oracle module (test infrastructure only).  It follows section 4 of the paper:

* tearing of the assembled system (eq. (reordered)) into subdomain systems
  with Boolean jump operators B_i (section 4.1, eq. (jumpConstraints 1));
  "fully redundant" gluing: one multiplier for every pair of subdomain copies
  of an interface degree of freedom (Fig. 3);
* all-floating variant (section 4.2, eq. (jumpoperatorAF)): Dirichlet values
  are enforced by extra multiplier rows with right-hand side b, so that every
  subdomain is floating; the classical variant eliminates Dirichlet DOFs;
* local solutions through a generalised inverse and the rigid-body kernel
  (eq. (localSolutions)); the dual system (eq. (classicalFetiF)) with
  F = sum B_i K_i^+ B_i^T, G = [B_i R_i], d = sum B_i K_i^+ f_i - b, e_i = R_i^T f_i;
* the projection P = I - G (G^T G)^{-1} G^T (eq. (projection), read with G^T G
  as in the initial iterate), the projected system (eq. (dualProblem)) solved
  by preconditioned CG from lambda_0 = G (G^T G)^{-1} e, and the recovery of
  gamma and u_i (end of section 4.3);
* preconditioners of the form sum B_D,i Y_i B_D,i^T (eq. (feti_preconditioner))
  with scaled rows B_D: lumped (Y_i = K_i, eq. (LumpedVK)),
  Dirichlet (Y_i = Schur complement on the interface, eq. (DirichletVK)) and
  identity (section 4.4, last paragraph).

Readings where the paper is silent (stated in the design notes):
* generalised inverse: interior-first block elimination; the interface Schur
  complement S_i is regularised as S_i + rho Rb Rb^T with Rb an orthonormal
  basis of the kernel restricted to the interface and rho = mean(diag S_i);
* scaled jump rows B_D: a gluing row of a DOF with m subdomain copies has
  weight 1/m; at a Dirichlet DOF of the all-floating variant the Dirichlet
  rows have weight 1 and the gluing rows weight 0 (the fixed boundary value is
  the neighbour that takes the whole jump).  Both choices give
  B B_D^T B = B, the defining property of a scaled jump operator;
* stopping rule ||P r_k|| <= rtol ||P r_0||;
* kernel of a stressed tangent: the three translations, plus each rotation
  about the current positions that K_i annihilates to 1e-12 relative.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla

from . import fem


class TornProblem:
    """Subdomain matrices, loads and constraint rows of one linear system."""

    def __init__(self, mesh, Ke, fe, nodal_load, dir_dof, dir_inc, variant, U=None):
        assert variant in ("af", "classical")
        self.mesh = mesh
        self.variant = variant
        n_nodes = mesh.n_nodes
        ndof = 3 * n_nodes
        self.ndof = ndof
        dir_mask = np.zeros(ndof, dtype=bool)
        dir_mask[dir_dof] = True
        dir_value = np.zeros(ndof)
        dir_value[dir_dof] = dir_inc
        self.dir_mask, self.dir_value = dir_mask, dir_value
        p = mesh.n_sub
        # subdomain copies of every node
        copies = [[] for _ in range(n_nodes)]
        self.subs = []
        for i in range(p):
            el = np.nonzero(mesh.elem_sub == i)[0]
            nodes = np.unique(mesh.hex8[el])
            for nd in nodes:
                copies[nd].append(i)
            self.subs.append(dict(elems=el, nodes=nodes))
        self.copies = copies
        node_mult = np.array([len(c) for c in copies])
        # local systems
        x_cur = mesh.xyz + (0.0 if U is None else np.asarray(U).reshape(-1, 3))
        for i, sd in enumerate(self.subs):
            nodes = sd["nodes"]
            gd = (3 * nodes[:, None] + np.arange(3)[None, :]).ravel()
            loc = -np.ones(ndof, dtype=np.int64)
            loc[gd] = np.arange(gd.size)
            n = gd.size
            K = np.zeros((n, n))
            f = np.zeros(n)
            el = sd["elems"]
            edofs = loc[(3 * mesh.hex8[el][:, :, None] + np.arange(3)).reshape(-1, 3 * mesh.hex8.shape[1])]
            for e in range(el.size):
                ix = edofs[e]
                K[np.ix_(ix, ix)] += Ke[el[e]]
                f[ix] += fe[el[e]]
            # nodal loads are split evenly between the subdomain copies
            f += nodal_load[gd] / np.repeat(node_mult[nodes], 3)
            keep = np.ones(n, dtype=bool)
            if variant == "classical":
                dm = dir_mask[gd]
                if dm.any():
                    f = f - K[:, dm] @ dir_value[gd][dm]
                keep = ~dm
            sd["gdof_all"] = gd
            sd["gdof"] = gd[keep]
            sd["K"] = K[np.ix_(keep, keep)]
            sd["f"] = f[keep]
            sd["x"] = x_cur[nodes]
            sd["has_dir"] = bool(dir_mask[gd].any())
            sd["loc_of_gdof"] = {int(g): k for k, g in enumerate(gd[keep])}
        # constraint rows
        rows = []           # list of [(sub, local dof, coef), ...]
        bvals = []
        wts = []
        for g in range(ndof):
            nd = g // 3
            cs = copies[nd]
            isdir = dir_mask[g]
            if variant == "classical" and isdir:
                continue
            # weights of the scaled rows B_D (eq. (feti_preconditioner)): 1/m on
            # gluing rows of a DOF with m copies; at an all-floating Dirichlet
            # DOF the fixed boundary value is the neighbour that takes the whole
            # jump: weight 1 on its rows, 0 on the gluing rows of that DOF
            afdir = variant == "af" and isdir
            w_glue = 0.0 if afdir else 1.0 / len(cs)
            if len(cs) >= 2:
                for a in range(len(cs)):
                    for b in range(a + 1, len(cs)):
                        sa, sb = cs[a], cs[b]
                        rows.append([(sa, self.subs[sa]["loc_of_gdof"][g], 1.0),
                                     (sb, self.subs[sb]["loc_of_gdof"][g], -1.0)])
                        bvals.append(0.0)
                        wts.append(w_glue)
            if variant == "af" and isdir:
                for sa in cs:
                    rows.append([(sa, self.subs[sa]["loc_of_gdof"][g], 1.0)])
                    bvals.append(dir_value[g])
                    wts.append(1.0)
        self.rows = rows
        self.b = np.array(bvals)
        self.w = np.array(wts)
        self.n_lam = len(rows)
        # per-subdomain B_i as dense (n_lam x n_i) -- small problems only
        for i, sd in enumerate(self.subs):
            sd["Brows"] = []
        for r, row in enumerate(rows):
            for (s, ld, c) in row:
                self.subs[s]["Brows"].append((r, ld, c))

    def B(self, i):
        sd = self.subs[i]
        Bi = np.zeros((self.n_lam, sd["K"].shape[0]))
        for (r, ld, c) in sd["Brows"]:
            Bi[r, ld] += c
        return Bi


def rigid_modes(x):
    """Translations and infinitesimal rotations about the centroid at points x [n,3].

    Returns R [3n, 6] in node-major DOF order.
    """
    n = x.shape[0]
    xc = x - x.mean(axis=0)
    R = np.zeros((n, 3, 6))
    for k in range(3):
        R[:, k, k] = 1.0
    # rotation about x: (0, -z, y); about y: (z, 0, -x); about z: (-y, x, 0)
    R[:, 1, 3], R[:, 2, 3] = -xc[:, 2], xc[:, 1]
    R[:, 0, 4], R[:, 2, 4] = xc[:, 2], -xc[:, 0]
    R[:, 0, 5], R[:, 1, 5] = -xc[:, 1], xc[:, 0]
    return R.reshape(3 * n, 6)


def partial_kernel(x, dmask, tol=1e-10):
    """Rigid modes of the points x that vanish on the DOFs flagged in dmask
    (node-major), restricted to the other DOFs: the null space of the six
    modes' rows at the flagged DOFs (rotations scaled by the points' radius),
    by singular value decomposition.  Returns [n_free, k], k = 6 - rank."""
    R = rigid_modes(x)
    L = np.sqrt(np.mean(np.sum((x - x.mean(axis=0)) ** 2, axis=1)))
    Rs = R * np.array([1, 1, 1, 1 / L, 1 / L, 1 / L])
    RD = Rs[dmask]
    if RD.shape[0] == 0:
        N = np.eye(6)
    else:
        _, sv, Vt = np.linalg.svd(RD)
        sv = np.concatenate([sv, np.zeros(6 - sv.size)])
        N = Vt.T[:, sv <= tol * sv.max()]
    return Rs[~dmask] @ N


class FetiRef:
    """Classical / all-floating FETI solve of a :class:`TornProblem`."""

    def __init__(self, tp: TornProblem, precond="lumped", kernel_tol=1e-12):
        assert precond in ("lumped", "dirichlet", "identity")
        self.tp = tp
        self.precond = precond
        self.locals = []
        for i, sd in enumerate(tp.subs):
            K = sd["K"]
            n = K.shape[0]
            bset = sorted({ld for (_, ld, _) in sd["Brows"]})
            bmask = np.zeros(n, dtype=bool)
            bmask[bset] = True
            I = np.nonzero(~bmask)[0]
            Bd = np.nonzero(bmask)[0]
            R = None
            nK = np.linalg.norm(K)
            if tp.variant == "af" or not sd["has_dir"]:
                Rfull = rigid_modes(sd["x"])
                # keep translations; keep a rotation only if K annihilates it
                keep = [0, 1, 2]
                for k in range(3, 6):
                    r = Rfull[:, k]
                    if np.linalg.norm(K @ r) <= kernel_tol * nK * np.linalg.norm(r):
                        keep.append(k)
                R = Rfull[:, keep]
            else:
                # classical subdomain with Dirichlet DOFs: its kernel is the set of
                # rigid modes that vanish on them (section 4.3: a subdomain that
                # touches the Dirichlet boundary at a vertex or an edge keeps a
                # partial kernel), restricted to the free DOFs
                R = partial_kernel(sd["x"], tp.dir_mask[sd["gdof_all"]])
                R = np.stack([r for r in R.T
                              if np.linalg.norm(K @ r) <= kernel_tol * nK * np.linalg.norm(r)], axis=1) \
                    if R.shape[1] else R
                if R.shape[1] == 0:
                    R = None
            Kii = K[np.ix_(I, I)]
            Kib = K[np.ix_(I, Bd)]
            Kbb = K[np.ix_(Bd, Bd)]
            if I.size:
                cii = sla.cho_factor(Kii, lower=True)
                X = sla.cho_solve(cii, Kib)
                S = Kbb - Kib.T @ X
            else:
                cii, X, S = None, np.zeros((0, Bd.size)), Kbb.copy()
            S = 0.5 * (S + S.T)
            if R is not None:
                Qb, Rq = np.linalg.qr(R[Bd])
                T = np.linalg.inv(Rq)
                Rh = R @ T
                rho = float(np.mean(np.diag(S)))
                St = S + rho * (Rh[Bd] @ Rh[Bd].T)
            else:
                Rh = None
                St = S
            cS = sla.cho_factor(St, lower=True)
            self.locals.append(dict(I=I, Bd=Bd, cii=cii, X=X, S=S, cS=cS, Kbb=Kbb, R=Rh,
                                    floating=R is not None, n=n))
        self.coarse_cols = []
        for i, lc in enumerate(self.locals):
            if lc["floating"]:
                self.coarse_cols.append((i, lc["R"].shape[1]))
        self.n_coarse = sum(m for _, m in self.coarse_cols)

    # -- local operators ---------------------------------------------------
    def kpinv(self, i, g):
        """Generalised inverse K_i^+ g by the interior-first block formula."""
        lc = self.locals[i]
        I, Bd = lc["I"], lc["Bd"]
        out = np.zeros(lc["n"])
        gI, gb = g[I], g[Bd]
        yI = sla.cho_solve(lc["cii"], gI) if I.size else np.zeros(0)
        t = gb - (self.tp.subs[i]["K"][np.ix_(I, Bd)].T @ yI if I.size else 0.0)
        zb = sla.cho_solve(lc["cS"], t)
        out[Bd] = zb
        if I.size:
            out[I] = yI - lc["X"] @ zb
        return out

    def gather(self, i, lam, weighted=False):
        """B_i^T lam (local vector); rows scaled by their weight if ``weighted``."""
        sd = self.tp.subs[i]
        x = np.zeros(self.locals[i]["n"])
        for (r, ld, c) in sd["Brows"]:
            x[ld] += c * lam[r] * (self.tp.w[r] if weighted else 1.0)
        return x

    def scatter(self, i, y, out, weighted=False):
        sd = self.tp.subs[i]
        for (r, ld, c) in sd["Brows"]:
            out[r] += c * y[ld] * (self.tp.w[r] if weighted else 1.0)

    def F(self, lam):
        q = np.zeros(self.tp.n_lam)
        for i, lc in enumerate(self.locals):
            x = self.gather(i, lam)
            y = np.zeros(lc["n"])
            y[lc["Bd"]] = sla.cho_solve(lc["cS"], x[lc["Bd"]])
            self.scatter(i, y, q)
        return q

    def Gt(self, lam):
        out = []
        for i, m in self.coarse_cols:
            x = self.gather(i, lam)
            out.append(self.locals[i]["R"].T @ x)
        return np.concatenate(out) if out else np.zeros(0)

    def G(self, alpha):
        q = np.zeros(self.tp.n_lam)
        o = 0
        for i, m in self.coarse_cols:
            y = self.locals[i]["R"] @ alpha[o:o + m]
            self.scatter(i, y, q)
            o += m
        return q

    def Mprec(self, w):
        z = np.zeros(self.tp.n_lam)
        for i, lc in enumerate(self.locals):
            x = self.gather(i, w, weighted=True)
            y = np.zeros(lc["n"])
            xb = x[lc["Bd"]]
            if self.precond == "lumped":
                y[lc["Bd"]] = lc["Kbb"] @ xb
            elif self.precond == "dirichlet":
                y[lc["Bd"]] = lc["S"] @ xb
            else:
                y[lc["Bd"]] = xb
            self.scatter(i, y, z, weighted=True)
        return z

    # -- solve ----------------------------------------------------------------
    def solve(self, rtol=1e-8, max_it=2000, track_invariants=False):
        tp = self.tp
        nc = self.n_coarse
        if nc:
            Gm = np.stack([self.G(e) for e in np.eye(nc)], axis=1)
            Qm = Gm.T @ Gm
            cQ = sla.cho_factor(Qm, lower=True)
        e = np.concatenate([self.locals[i]["R"].T @ tp.subs[i]["f"] for i, _ in self.coarse_cols]) \
            if nc else np.zeros(0)

        def proj(v):
            if not nc:
                return v
            return v - self.G(sla.cho_solve(cQ, self.Gt(v)))

        d = -tp.b.copy()
        for i in range(len(self.locals)):
            self.scatter(i, self.kpinv(i, tp.subs[i]["f"]), d)
        lam = self.G(sla.cho_solve(cQ, e)) if nc else np.zeros(tp.n_lam)
        r = d - self.F(lam)
        w = proj(r)
        z = proj(self.Mprec(w))
        s = z.copy()
        rho = w @ z
        w0 = np.linalg.norm(w)
        alphas, betas, res = [], [], [w0]
        inv_err = []
        k = 0
        while np.linalg.norm(w) > rtol * w0 and k < max_it:
            q = self.F(s)
            sq = s @ q
            alpha = rho / sq
            lam = lam + alpha * s
            r = r - alpha * q
            w = proj(r)
            z = proj(self.Mprec(w))
            rho_new = w @ z
            beta = rho_new / rho
            rho = rho_new
            s = z + beta * s
            alphas.append(alpha)
            betas.append(beta)
            res.append(np.linalg.norm(w))
            if track_invariants and nc:
                inv_err.append(np.linalg.norm(self.Gt(lam) - e) / max(np.linalg.norm(e), 1e-300))
            k += 1
        gamma = -sla.cho_solve(cQ, self.Gt(r)) if nc else np.zeros(0)
        # local and global displacements
        u_loc = []
        gam = {}
        o = 0
        for i, m in self.coarse_cols:
            gam[i] = gamma[o:o + m]
            o += m
        for i, lc in enumerate(self.locals):
            g = tp.subs[i]["f"] - self.gather(i, lam)
            ui = self.kpinv(i, g)
            if i in gam:
                ui = ui + lc["R"] @ gam[i]
            u_loc.append(ui)
        u = np.zeros(tp.ndof)
        cnt = np.zeros(tp.ndof)
        for i, sd in enumerate(tp.subs):
            np.add.at(u, sd["gdof"], u_loc[i])
            np.add.at(cnt, sd["gdof"], 1.0)
        u = np.where(cnt > 0, u / np.maximum(cnt, 1), 0.0)
        u[tp.dir_mask] = tp.dir_value[tp.dir_mask]
        return dict(u=u, u_loc=u_loc, lam=lam, gamma=gamma, iters=k, res=np.array(res),
                    kappa=lanczos_kappa(alphas, betas), e=e, inv_err=inv_err,
                    n_lam=tp.n_lam, n_coarse=nc)


def lanczos_kappa(alphas, betas):
    """Condition estimate from the CG coefficients: the Lanczos tridiagonal has
    diagonal 1/alpha_k + beta_{k-1}/alpha_{k-1} and off-diagonal
    sqrt(beta_k)/alpha_k; the ratio of its extreme eigenvalues estimates kappa."""
    m = len(alphas)
    if m == 0:
        return 1.0
    T = np.zeros((m, m))
    for k in range(m):
        T[k, k] = 1.0 / alphas[k] + (betas[k - 1] / alphas[k - 1] if k > 0 else 0.0)
        if k + 1 < m:
            T[k, k + 1] = T[k + 1, k] = np.sqrt(betas[k]) / alphas[k]
    ev = np.linalg.eigvalsh(T)
    return float(ev[-1] / ev[0])


def linear_torn_problem(mesh, variant, load_factor=1.0):
    """Torn form of the linear elastic problem K u = lf f_ext, u = lf u_D."""
    Ke, _ = fem.element_matrices(mesh, None)
    fe = np.zeros((mesh.n_elems, 3 * mesh.hex8.shape[1]))
    if mesh.body_force is not None:
        fe = load_factor * fem.body_force_vector(mesh.xyz[mesh.hex8], mesh.body_force)
    return TornProblem(mesh, Ke, fe, np.zeros(mesh.n_dofs), mesh.dir_dof,
                       load_factor * mesh.dir_val, variant)


def newton_torn_problem(mesh, U, tau, variant):
    """Torn form of one Newton system K'(U) dU = tau f_ext(U) - f_int(U)."""
    U = np.asarray(U, dtype=np.float64).reshape(-1)
    Ke, fint_e = fem.element_matrices(mesh, U.reshape(-1, 3))
    fe = -fint_e
    if mesh.body_force is not None:
        fe = fe + tau * fem.body_force_vector(mesh.xyz[mesh.hex8], mesh.body_force)
    nodal = np.zeros(mesh.n_dofs)
    if mesh.pface is not None and mesh.pressure != 0.0:
        x = mesh.xyz + U.reshape(-1, 3)
        fp = fem.pressure_face_load(x[mesh.pface], mesh.pressure)
        pd = (3 * mesh.pface[:, :, None] + np.arange(3)).ravel()
        nodal = tau * np.bincount(pd, weights=fp.ravel(), minlength=mesh.n_dofs)
    inc = tau * mesh.dir_val - U[mesh.dir_dof]
    return TornProblem(mesh, Ke, fe, nodal, mesh.dir_dof, inc, variant, U=U)


def kkt_bruteforce(tp: TornProblem):
    """Solve the full saddle-point system (eqs. (classicalFetiLGS)/(AFFETI)) densely
    by least squares; returns the subdomain displacements (unique) as a list."""
    sizes = [sd["K"].shape[0] for sd in tp.subs]
    N = sum(sizes)
    offs = np.concatenate([[0], np.cumsum(sizes)])
    A = np.zeros((N + tp.n_lam, N + tp.n_lam))
    rhs = np.zeros(N + tp.n_lam)
    for i, sd in enumerate(tp.subs):
        o = offs[i]
        A[o:o + sizes[i], o:o + sizes[i]] = sd["K"]
        rhs[o:o + sizes[i]] = sd["f"]
        for (r, ld, c) in sd["Brows"]:
            A[N + r, o + ld] += c
            A[o + ld, N + r] += c
    rhs[N:] = tp.b
    sol = np.linalg.lstsq(A, rhs, rcond=1e-13)[0]
    return [sol[offs[i]:offs[i + 1]] for i in range(len(sizes))]
