"""The method's sweeps and iterations (FP64).

Test infrastructure: plain FP64 NumPy/SciPy.

Notation: U is a grid field (ny*nx, row-major) holding the unknowns on the
interior nodes and the Dirichlet value g elsewhere; family 0 (B) are the
beta-curves, family 1 (G) the gamma-curves; G_F gathers a grid field to the
interior nodes of family F (eq. (21)-(23)), P_F scatters line values back
(Sec. 6); M, K, C are the line matrices of eq. (17), (19); S = mu K + C + sigma M;
L = int f v dl.

One step of eq. (10), as the paper describes it on the curves (eq. (16),
(18)) with *values* of u_{j+1/2} handed from one family to the other through
the grid (the paper substitutes "the values from u_{j+1/2}" into the second
substep):
    beta substep   u = G_B U                       (values on the beta-curves)
                   (M + theta dt S) udot = L - S u            eq. (16)-(17)
                   v = u + dt udot ;   U_half = P_B v
    gamma substep  u = G_G U_half
                   (M + theta dt mu K) udot = - mu K u        eq. (18)-(19)
                   v = u + dt udot ;   U_next = P_G v
Algebraically v = (M + theta dt S)^{-1} [(M - (1-theta) dt S) u + dt L] on the
beta-curves and v = (M + theta dt mu K)^{-1} (M - (1-theta) dt mu K) u on the
gamma-curves; the sweeps below use that form.

Dirichlet data (the paper has u = 0 on Gamma; a nodal field g generalises it):
g at a point is its bilinear interpolant (eq. (22)); the curve ends, which lie
on Gamma, take g there; grid nodes not strictly inside Omega hold g, so that
the bilinear gather near Gamma reads it; a boundary point that brackets a grid
node in the scatter carries g.

Stationary problem (Sec. 2: eq. (1) is the t -> infinity limit of eq. (2)):
the steps are repeated with a fixed pseudo time step until they stop moving
the solution.  With Phi(U) the step above, the iterate U_{k+1} = Phi(U_k) has
residual  rel_k = |U_{k+1} - U_k|_2 / |Phi(0)|_2  over the interior nodes, and
the iteration stops at the first k with rel_k <= tol (returning U_{k+1}).
Phi is affine, Phi(U) = T U + c with c = Phi(0); its fixed point solves
(I - T) U = c (see oracle.dense).
"""
from __future__ import annotations

import numpy as np

from . import geometry as geo
from . import linefe as lfe
from . import transfer as tr


class Oracle:
    """All operators of one problem instance (a workloads.Problem)."""

    def __init__(self, prob, families=None, stabilize=False):
        """stabilize: exponentially fitted beta-lines (oracle.linefe)."""
        self.prob = prob
        self.grid = geo.Grid(prob.box, prob.nx, prob.ny)
        self.dom = geo.make_domain(prob.domain, prob.dom_params, prob.box)
        if prob.beta1 is None and prob.beta2 is None:  # beta from the stream function
            b1, b2 = geo.beta_from_psi(self.grid, prob.psi)
        else:
            b1, b2 = prob.beta1, prob.beta2
        self.flow = geo.Flow(self.grid, b1, b2)
        self.mask = geo.interior_mask(self.grid, self.dom)
        self.inner_idx = np.nonzero(self.mask.ravel())[0]
        self.fams = families if families is not None else geo.build_families(
            self.grid, self.dom, self.flow)
        self.mu = float(prob.mu)
        self.sigma = float(prob.sigma)
        self.G, self.P, self.inner, bnd = [], [], [], []
        for fam in self.fams:
            self.G.append(tr.gather_matrix(self.grid, fam))
            P, b = tr.scatter_matrix(self.grid, self.dom, fam, self.mask)
            self.P.append(P)
            bnd.append(b)
            self.inner.append(fam.interior())
        fb = self.fams[0]
        b1, b2 = self.flow.beta(fb.x, fb.y)
        self.bnorm = np.hypot(b1, b2)
        M, K, C = lfe.line_operators(fb, self.bnorm)
        self.MB, self.KB, self.CB = M, K, C
        if stabilize:
            K = lfe.fitted_stiffness(fb, self.bnorm, self.mu)
            self.KB = K
        self.SB = K.scale(self.mu) + C + M.scale(self.sigma)
        fG = self.fams[1]
        self.MG, self.KG, _ = lfe.line_operators(fG, None)
        self.fnode = self.grid.interp(prob.f, fb.x, fb.y)
        self.L = self.MB.apply(self.fnode)
        self.L[~self.inner[0]] = 0.0
        # Dirichlet data: nodal g, its values at the curve ends and the
        # boundary points' share of each scatter
        ny, nx = self.grid.ny, self.grid.nx
        self.g = np.zeros((ny, nx)) if getattr(prob, "g", None) is None else np.asarray(prob.g, float)
        self.bfield = np.where(self.mask, 0.0, self.g).ravel()
        self.gend, self.Pb = [], []
        for k, fam in enumerate(self.fams):
            ge = np.zeros(fam.n_nodes)
            ends = ~self.inner[k]
            ge[ends] = self.grid.interp(self.g, fam.x[ends], fam.y[ends])
            self.gend.append(ge)
            rows, coef, xb, yb = bnd[k]
            pb = np.zeros(nx * ny)
            np.add.at(pb, rows, coef * self.grid.interp(self.g, xb, yb))
            self.Pb.append(pb)

    # -- pieces ----------------------------------------------------------------
    def zero_field(self):
        """The grid field with zero on the interior nodes (g elsewhere)."""
        return self.bfield.copy()

    def with_boundary(self, U):
        """U with its non-interior nodes set to g."""
        out = np.array(U, float, copy=True)
        out[~self.mask.ravel()] = self.bfield[~self.mask.ravel()]
        return out

    def gather(self, fam, U):
        """Values on the curve nodes: eq. (22) inside, g at the ends."""
        u = self.G[fam] @ U
        ends = ~self.inner[fam]
        u[ends] = self.gend[fam][ends]
        return u

    def scatter(self, fam, v):
        """Grid field from curve values (Sec. 6); g outside the interior."""
        return self.P[fam] @ v + self.Pb[fam] + self.bfield

    def beta_substep(self, U, theta, dt, source=True, S=None, L=None):
        """S, L: the beta-curves' operator and load (default: the problem's)."""
        S = self.SB if S is None else S
        L = self.L if L is None else L
        u = self.gather(0, U)
        A = self.MB + S.scale(theta * dt)
        rhs = self.MB.apply(u) - (1.0 - theta) * dt * S.apply(u)
        if source:
            rhs = rhs + dt * L
        v = lfe.solve_lines(A, rhs, self.inner[0], self.gend[0])
        return self.scatter(0, v), v

    def gamma_substep(self, U, theta, dt):
        u = self.gather(1, U)
        A = self.MG + self.KG.scale(theta * dt * self.mu)
        rhs = self.MG.apply(u) - (1.0 - theta) * dt * self.mu * self.KG.apply(u)
        v = lfe.solve_lines(A, rhs, self.inner[1], self.gend[1])
        return self.scatter(1, v), v

    def step(self, U, theta, dt, source=True, S=None, L=None):
        """One step of eq. (10) with value transfer (see module docstring)."""
        Uh, _ = self.beta_substep(U, theta, dt, source, S, L)
        Un, _ = self.gamma_substep(Uh, theta, dt)
        return Un

    def norm(self, U):
        return float(np.linalg.norm(U[self.inner_idx]))

    # -- stationary iteration --------------------------------------------------
    def c_norm(self, theta, dt):
        return self.norm(self.step(self.zero_field(), theta, dt))

    def rel_residual(self, U, theta, dt):
        return self.norm(self.step(U, theta, dt) - U) / self.c_norm(theta, dt)

    def iterate(self, U0, theta, dt, max_iters, tol, history=False):
        """U_{k+1} = Phi(U_k) until rel_k <= tol; returns (U, iters, rel, hist)."""
        cn = self.c_norm(theta, dt)
        U = self.with_boundary(U0)
        hist = []
        rel = np.inf
        it = 0
        while it < max_iters:
            Un = self.step(U, theta, dt)
            rel = self.norm(Un - U) / cn
            U = Un
            it += 1
            hist.append(rel)
            if rel <= tol or not np.isfinite(rel):
                break
        return U, it, rel, (hist if history else None)

    # -- eq. (11) initial guess --------------------------------------------
    def s_guess(self):
        """u0 with s(u0, v) = <l, v> on the beta-curves, scattered to the grid."""
        v = lfe.solve_lines(self.SB, self.L, self.inner[0], self.gend[0])
        return self.scatter(0, v)

    # -- time marching -------------------------------------------------------
    def strang_step(self, U, theta, dt):
        """Symmetric splitting of eq. (10): beta substep over dt/2, gamma substep
        over dt, beta substep over dt/2 (each with the theta-scheme of eq. (7)
        and values handed on through the grid)."""
        Uh, _ = self.beta_substep(U, theta, dt / 2)
        Ug, _ = self.gamma_substep(Uh, theta, dt)
        Un, _ = self.beta_substep(Ug, theta, dt / 2)
        return Un

    def march(self, U0, theta, dt, steps, strang=False):
        U = self.with_boundary(U0)
        for _ in range(steps):
            U = self.strang_step(U, theta, dt) if strang else self.step(U, theta, dt)
        return U

    # -- implicit Euler steps iterated to convergence ---------------------------
    def step_operators(self, Un, dt):
        """One implicit Euler step of eq. (2) (eq. (7) with theta = 1),
        (u - u_n)/dt + A u = f, is the stationary problem A u + u/dt = f + u_n/dt:
        sigma + 1/dt in S and, on the beta-curves (which carry the reaction and
        the source), the load L + M (G_B u_n)/dt.  Returns (S, L)."""
        ub = self.gather(0, self.with_boundary(Un))
        S = self.SB + self.MB.scale(1.0 / dt)
        L = self.L + self.MB.apply(ub) / dt
        L[~self.inner[0]] = 0.0
        return S, L

    def implicit_step(self, Un, dt, tau, tol, max_inner, theta=1.0):
        """u_{n+1}: the stationary iteration (pseudo step tau, theta) on the step's
        problem from u_n, to rel <= tol; returns (U, inner iterations, rel)."""
        S, L = self.step_operators(Un, dt)
        cn = self.norm(self.step(self.zero_field(), theta, tau, S=S, L=L))
        U = self.with_boundary(Un)
        rel, it = np.inf, 0
        while it < max_inner:
            Un1 = self.step(U, theta, tau, S=S, L=L)
            rel = self.norm(Un1 - U) / cn
            U = Un1
            it += 1
            if rel <= tol or not np.isfinite(rel):
                break
        return U, it, rel

    def march_converged(self, U0, dt, steps, tau, tol, max_inner):
        """`steps` implicit Euler steps, each iterated to tol; returns (U, counts)."""
        U = self.with_boundary(U0)
        counts = []
        for _ in range(steps):
            U, it, _ = self.implicit_step(U, dt, tau, tol, max_inner)
            counts.append(it)
        return U, counts
