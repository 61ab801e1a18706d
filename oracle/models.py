"""Coefficients of the transport system (Sec. 1, eq:equations) for the oracle.

    d_t u_i + alpha_i(x)^T grad u_i = (i/eps) beta_i(x) u_i + sum_j gamma_ij(x) u_j

Each model exposes, vectorised over beams (``X`` is (N, m), ``comp`` is (N,)):

* ``alpha(X, comp)``        alpha_l(X)                       (N, m)
* ``jac_alpha(X, comp)``    J_ab = d alpha_a / d x_b          (N, m, m)
  (the paper writes grad_x alpha; the O(eps^-1/2) matching of Sec. 2.1
  makes it the Jacobian with this index order)
* ``beta``, ``grad_beta``, ``hess_beta``                      (N,), (N, m), (N, m, m)
* ``hess_P_alpha(X, comp, P)``  Hessian in x of P . alpha_l(x) at X   (N, m, m)
* ``gamma(X)``              gamma_ij(X), row i receives from column j (N, n, n) complex

Models:

* ``QCLE``    the two-level quantum-classical Liouville equation of Sec. 3.3
  (eq:QCLE, adiabatic quantities the adiabatic energies and d21 below eq:QCLE) with a nuclear mass, written as
  a linear four-component system for (u11, u22, u21, u12 := conj u21).
  Component order: 0 = u11 (upper surface E1, the '+' root), 1 = u22 (lower
  surface E2), 2 = u21, 3 = u12.  Diabatic potential
      V11 = A tanh(B q1) + Vb(r),  V22 = -A tanh(B q1) + Vb(r),
      V12 = C exp(-D q1^2),
      Vb(r) = sum_{k>=2} ( M w_k^2 q_k^2 / 2 + lam q1 q_k )  (d > 1 only).
  The adiabatic energies and d21 are taken from the adiabatic energies and d21 below eq:QCLE symbolically
  (SymPy) and differentiated symbolically in q1; the quadratic bath part is
  differentiated by hand.
* ``LinQuad`` alpha linear, beta quadratic, gamma constant: the class of
  Sec. 3.1 for which the Gaussian beam ansatz has no modelling error.  With
  alpha = 0 and constant beta it is the x-independent system whose exact
  solution is a matrix exponential (Sec. 2.2, eq:tilde_gamma).
* ``Paper32`` the two-component system with nonlinear coefficients of
  Sec. 3.2, eq:ex2, in the form d_t u + alpha.grad u = (i/eps) beta u
  + gamma u: the transport fields are minus the printed drifts,
  beta_1 = sin|x|^2, beta_2 = cos|x|^2, and gamma = |x|^2 [[-1, 5], [-5, -1/2]].
"""

import numpy as np
import sympy as sp


class QCLE:
    n_comp = 4
    # E_l = Vb + sigma_l * s, beta_l = bcoef_l * s, with s = (E1 - E2)/2
    sigma = np.array([1.0, -1.0, 0.0, 0.0])
    bcoef = np.array([0.0, 0.0, 2.0, -2.0])

    def __init__(self, A, B, C, D, mass, d=1, lam=0.0, bath_omega=()):
        self.A, self.B, self.C, self.D = float(A), float(B), float(C), float(D)
        self.mass = float(mass)
        self.d = int(d)
        self.m = 2 * self.d
        self.lam = float(lam)
        self.bath_omega = np.asarray(bath_omega, dtype=np.float64).reshape(-1)
        if self.d > 1 and self.bath_omega.size != self.d - 1:
            raise ValueError("need d-1 bath frequencies")
        q = sp.Symbol("q", real=True)
        a = self.A * sp.tanh(self.B * q)          # q1-dependent part of V11 (V22 = -a)
        V11, V22, V12 = a, -a, self.C * sp.exp(-self.D * q**2)
        # the adiabatic energies and d21 below eq:QCLE: E_{1,2} = (V11+V22)/2 +- sqrt((V11-V22)^2 + 4 V12^2)/2
        s = sp.sqrt((V11 - V22) ** 2 + 4 * V12**2) / 2
        d21 = ((V11 - V22) * sp.diff(V12, q) - V12 * sp.diff(V11 - V22, q)) / (
            (V11 - V22) ** 2 + 4 * V12**2)
        self._s = [sp.lambdify(q, sp.diff(s, q, k), "numpy") for k in range(4)]
        self._d21 = sp.lambdify(q, d21, "numpy")
        self._theta = sp.lambdify(q, sp.atan2(2 * V12, V11 - V22) / 2, "numpy")
        # bath Hessian (constant) and its gradient map
        Hb = np.zeros((self.d, self.d))
        if self.d > 1:
            Hb[0, 1:] = self.lam
            Hb[1:, 0] = self.lam
            Hb[np.arange(1, self.d), np.arange(1, self.d)] = self.mass * self.bath_omega**2
        self.Hb = Hb

    # --- adiabatic quantities ------------------------------------------------
    def s(self, q1, k=0):
        """k-th q1-derivative of s = (E1 - E2)/2."""
        return np.broadcast_to(np.asarray(self._s[k](q1), dtype=np.float64), np.shape(q1)).copy()

    def d21(self, q1):
        return np.asarray(self._d21(q1), dtype=np.float64) * np.ones_like(q1)

    def mixing_angle(self, q1):
        return np.asarray(self._theta(q1), dtype=np.float64) * np.ones_like(q1)

    def Vb(self, r):
        if self.d == 1:
            return np.zeros(r.shape[0])
        qk = r[:, 1:]
        return (0.5 * self.mass * self.bath_omega**2 * qk**2).sum(1) + self.lam * r[:, 0] * qk.sum(1)

    def energy(self, r, comp):
        return self.Vb(r) + self.sigma[comp] * self.s(r[:, 0])

    def grad_energy(self, r, comp):
        g = r @ self.Hb.T  # gradient of the quadratic bath part (Hb r)
        g[:, 0] += self.sigma[comp] * self.s(r[:, 0], 1)
        return g

    def hess_energy(self, r, comp):
        H = np.broadcast_to(self.Hb, (r.shape[0], self.d, self.d)).copy()
        H[:, 0, 0] += self.sigma[comp] * self.s(r[:, 0], 2)
        return H

    # --- coefficients of eq:equations --------------------------------------------
    def _split(self, X):
        return X[:, : self.d], X[:, self.d:]

    def alpha(self, X, comp):
        r, p = self._split(X)
        return np.concatenate([p / self.mass, -self.grad_energy(r, comp)], axis=1)

    def jac_alpha(self, X, comp):
        r, _ = self._split(X)
        n, d = X.shape[0], self.d
        J = np.zeros((n, 2 * d, 2 * d))
        J[:, :d, d:] = np.eye(d) / self.mass
        J[:, d:, :d] = -self.hess_energy(r, comp)
        return J

    def beta(self, X, comp):
        return self.bcoef[comp] * self.s(X[:, 0])

    def grad_beta(self, X, comp):
        g = np.zeros_like(X)
        g[:, 0] = self.bcoef[comp] * self.s(X[:, 0], 1)
        return g

    def hess_beta(self, X, comp):
        H = np.zeros((X.shape[0], self.m, self.m))
        H[:, 0, 0] = self.bcoef[comp] * self.s(X[:, 0], 2)
        return H

    def hess_P_alpha(self, X, comp, P):
        # P . alpha = P_r . p / M - P_p . grad E_l(r); only the r-r block of its
        # Hessian survives: -sum_c P_{p,c} d_c Hess E_l, and the third
        # derivatives of E_l come from s''' (Vb is quadratic).
        H = np.zeros((X.shape[0], self.m, self.m))
        H[:, 0, 0] = -P[:, self.d] * self.sigma[comp] * self.s(X[:, 0], 3)
        return H

    def kappa(self, X):
        """(p/M) . d21(r): the real coupling coefficient of eq:QCLE."""
        return X[:, self.d] / self.mass * self.d21(X[:, 0])

    def gamma(self, X):
        k = self.kappa(X)
        G = np.zeros((X.shape[0], 4, 4), dtype=np.complex128)
        G[:, 0, 2] = k
        G[:, 0, 3] = k
        G[:, 1, 2] = -k
        G[:, 1, 3] = -k
        G[:, 2, 0] = -k
        G[:, 3, 0] = -k
        G[:, 2, 1] = k
        G[:, 3, 1] = k
        return G


class LinQuad:
    """alpha_l = a_l + Jl x, beta_l = b0_l + b_l.x + x^T H_l x / 2, gamma constant."""

    def __init__(self, a, J, b0, b, H, gamma):
        self.a = np.asarray(a, dtype=np.float64)        # (n, m)
        self.J = np.asarray(J, dtype=np.float64)        # (n, m, m)
        self.b0 = np.asarray(b0, dtype=np.float64)      # (n,)
        self.b = np.asarray(b, dtype=np.float64)        # (n, m)
        self.H = np.asarray(H, dtype=np.float64)        # (n, m, m), symmetric
        self.G = np.asarray(gamma, dtype=np.complex128)  # (n, n)
        self.n_comp, self.m = self.a.shape

    @classmethod
    def xindep(cls, b0, gamma, m=2):
        b0 = np.asarray(b0, dtype=np.float64)
        n = b0.size
        return cls(np.zeros((n, m)), np.zeros((n, m, m)), b0, np.zeros((n, m)),
                   np.zeros((n, m, m)), gamma)

    def alpha(self, X, comp):
        return self.a[comp] + np.einsum("nab,nb->na", self.J[comp], X)

    def jac_alpha(self, X, comp):
        return self.J[comp].copy()

    def beta(self, X, comp):
        return (self.b0[comp] + np.einsum("na,na->n", self.b[comp], X)
                + 0.5 * np.einsum("na,nab,nb->n", X, self.H[comp], X))

    def grad_beta(self, X, comp):
        return self.b[comp] + np.einsum("nab,nb->na", self.H[comp], X)

    def hess_beta(self, X, comp):
        return self.H[comp].copy()

    def hess_P_alpha(self, X, comp, P):
        return np.zeros((X.shape[0], self.m, self.m))

    def gamma(self, X):
        return np.broadcast_to(self.G, (X.shape[0],) + self.G.shape).copy()


class Paper32:
    """Eq:ex2: alpha_1 = -(sin(x1 + x2), cos(x1 - x2)), alpha_2 = -(sin(x1 - x2), cos(x1 + x2)),
    beta_1 = sin(r^2), beta_2 = cos(r^2) with r^2 = x1^2 + x2^2,
    gamma = r^2 [[-1, 5], [-5, -1/2]] (row receives from column).  Derivatives by hand."""

    n_comp, m = 2, 2
    G_UNIT = np.array([[-1.0, 5.0], [-5.0, -0.5]])

    @staticmethod
    def _uv(X):
        return X[:, 0] + X[:, 1], X[:, 0] - X[:, 1]

    def alpha(self, X, comp):
        u, v = self._uv(X)
        a0 = np.stack([-np.sin(u), -np.cos(v)], 1)
        a1 = np.stack([-np.sin(v), -np.cos(u)], 1)
        return np.where((comp == 0)[:, None], a0, a1)

    def jac_alpha(self, X, comp):
        u, v = self._uv(X)
        cu, su, cv, sv = np.cos(u), np.sin(u), np.cos(v), np.sin(v)
        J0 = np.stack([np.stack([-cu, -cu], 1), np.stack([sv, -sv], 1)], 1)
        J1 = np.stack([np.stack([-cv, cv], 1), np.stack([su, su], 1)], 1)
        return np.where((comp == 0)[:, None, None], J0, J1)

    def beta(self, X, comp):
        r2 = (X ** 2).sum(1)
        return np.where(comp == 0, np.sin(r2), np.cos(r2))

    def grad_beta(self, X, comp):
        r2 = (X ** 2).sum(1)
        f = np.where(comp == 0, 2.0 * np.cos(r2), -2.0 * np.sin(r2))
        return f[:, None] * X

    def hess_beta(self, X, comp):
        r2 = (X ** 2).sum(1)
        f1 = np.where(comp == 0, 2.0 * np.cos(r2), -2.0 * np.sin(r2))      # coefficient of I
        f2 = np.where(comp == 0, -4.0 * np.sin(r2), -4.0 * np.cos(r2))     # coefficient of x x^T
        return f1[:, None, None] * np.eye(2)[None] + f2[:, None, None] * np.einsum("na,nb->nab", X, X)

    def hess_P_alpha(self, X, comp, P):
        u, v = self._uv(X)
        ones = np.array([[1.0, 1.0], [1.0, 1.0]])
        alt = np.array([[1.0, -1.0], [-1.0, 1.0]])
        # P.alpha_1 = -(P1 sin u + P2 cos v);  P.alpha_2 = -(P1 sin v + P2 cos u)
        h0 = (P[:, 0] * np.sin(u))[:, None, None] * ones + (P[:, 1] * np.cos(v))[:, None, None] * alt
        h1 = (P[:, 0] * np.sin(v))[:, None, None] * alt + (P[:, 1] * np.cos(u))[:, None, None] * ones
        return np.where((comp == 0)[:, None, None], h0, h1)

    def gamma(self, X):
        r2 = (X ** 2).sum(1)
        return r2[:, None, None] * self.G_UNIT[None].astype(np.complex128)
