"""Surface hopping Gaussian beam ensemble: beam ODEs, RK4, hopping (oracle).

Follows Cai & Lu Sec. 2.3-2.4.  Per beam the state is

    X, P in R^m; M, N real symmetric m x m; S real; A complex;
    logw = Re omega at the last hop; Lam = integral of the total out-rate since
    the last hop (so Re omega(t) = logw + Lam); phase = exp(i Im omega);
    E = -log(1 - Y), the threshold of the current waiting time;
    comp = l_t, the current component; nhop = number of hops so far.

Readings taken where the paper leaves a choice:

* time stepping: fixed intervals [t_n, t_n + dt]; classical RK4 (the
  workloads prescribe RK4); Kutta's third-order method as an option (Sec.
  2.4 integrates with "a third-order Runge-Kutta method", variant unnamed).
* step 3/4: the trial step covers the rest of the interval; the hop test
  exp(omega~ - omega(t+dt)) <= 1 - Y reads Lam' >= E with E = -log(1-Y).
* step 4 "interpolation of omega": linear in Lam over the trial step,
  theta = (E - Lam)/(Lam' - Lam); theta = 0 when E <= Lam already.
* step 5: the whole system is re-integrated over theta*h from the step's
  start (the trial result is reused when theta == 1), the hop is applied,
  and the beam finishes the same interval on its new component.  At most
  HOP_CAP hops per interval; after that the rest of the interval is
  integrated without a test (counted as overflow).
* the destination is the smallest j != l, in ascending order, with
  U * R < C_j, C_j the running sum of |gamma_jl| and R the full sum; the
  phase jump i arg gamma_jl multiplies the stored unit phase by
  gamma_jl/|gamma_jl|.
* a threshold tie is |Lam' - E| <= tau E; a destination tie is
  |U R - C_j| <= tau R for some j.  Both are counted per beam.  tau is
  1e-12 against an FP64 run and 1e-5 against a run whose trajectories are
  FP32 (hop times then move by about 1e-7 relative).
"""

import numpy as np

from . import philox

HOP_CAP = 16
TIE_REL = 1e-12
TIE_REL_MIXED = 1e-5


class Ensemble:
    """Beam ensemble in the oracle's own layout (full matrices, complex A)."""

    def __init__(self, n, m, n_comp):
        self.n, self.m, self.n_comp = n, m, n_comp
        self.X = np.zeros((n, m))
        self.P = np.zeros((n, m))
        self.M = np.zeros((n, m, m))
        self.N = np.zeros((n, m, m))
        self.S = np.zeros(n)
        self.A = np.zeros(n, dtype=np.complex128)
        self.logw = np.zeros(n)
        self.phase = np.ones(n, dtype=np.complex128)
        self.Lam = np.zeros(n)
        self.E = np.zeros(n)
        self.comp = np.zeros(n, dtype=np.int64)
        self.nhop = np.zeros(n, dtype=np.int64)
        self.gid = np.zeros(n, dtype=np.uint64)
        # diagnostics per beam
        self.thr_ties = np.zeros(n, dtype=np.int64)
        self.dest_ties = np.zeros(n, dtype=np.int64)
        self.cap_overflow = np.zeros(n, dtype=np.int64)
        self.zero_rate = np.zeros(n, dtype=np.int64)
        self.hop_log = [[] for _ in range(n)]   # (interval index, destination)
        self.interval = 0

    ODE_FIELDS = ("X", "P", "M", "N", "S", "A", "Lam")

    def ode(self, idx):
        return tuple(getattr(self, f)[idx].copy() for f in self.ODE_FIELDS)

    def set_ode(self, idx, y):
        for f, v in zip(self.ODE_FIELDS, y):
            getattr(self, f)[idx] = v

    def subset(self, idx):
        e = Ensemble(len(idx), self.m, self.n_comp)
        for f in ("X", "P", "M", "N", "S", "A", "logw", "phase", "Lam", "E", "comp",
                  "nhop", "gid", "thr_ties", "dest_ties", "cap_overflow", "zero_rate"):
            setattr(e, f, getattr(self, f)[idx].copy())
        e.hop_log = [list(self.hop_log[i]) for i in idx]
        e.interval = self.interval
        return e


def rhs(model, comp, y):
    """Right-hand side of the beam ODEs, Sec. 2.3 eq:shgb_odes, on component l = comp.

    dX/dt = alpha_l, dS/dt = beta_l, dP/dt = grad beta_l - J^T P,
    dA/dt = gamma_ll A, dM/dt = -M J - J^T M,
    dN/dt = Hess(P.alpha_l) - Hess beta_l - N J - J^T N,
    d Re(omega)/dt = sum_{j != l} |gamma_jl|   (the jump part is applied at hops).
    """
    X, P, M, N, S, A, Lam = y
    J = model.jac_alpha(X, comp)
    Jt = np.swapaxes(J, 1, 2)
    G = model.gamma(X)
    idx = np.arange(X.shape[0])
    out_rate = np.abs(G[idx, :, comp]).sum(1) - np.abs(G[idx, comp, comp])
    dX = model.alpha(X, comp)
    dS = model.beta(X, comp)
    dP = model.grad_beta(X, comp) - np.einsum("nab,nb->na", Jt, P)
    dA = G[idx, comp, comp] * A
    dM = -M @ J - Jt @ M
    dN = model.hess_P_alpha(X, comp, P) - model.hess_beta(X, comp) - N @ J - Jt @ N
    return (dX, dP, dM, dN, dS, dA, out_rate)


def _axpy(y, h, k):
    return tuple(a + _bcast(h, a) * b for a, b in zip(y, k))


def _bcast(h, a):
    h = np.asarray(h, dtype=np.float64)
    return h.reshape(h.shape + (1,) * (a.ndim - h.ndim)) if h.ndim else h


def rk4(model, comp, y, h):
    """One classical fourth-order Runge-Kutta step of size h (per beam) on component comp."""
    k1 = rhs(model, comp, y)
    k2 = rhs(model, comp, _axpy(y, 0.5 * h, k1))
    k3 = rhs(model, comp, _axpy(y, 0.5 * h, k2))
    k4 = rhs(model, comp, _axpy(y, h, k3))
    return tuple(a + _bcast(h / 6.0, a) * (b1 + 2.0 * b2 + 2.0 * b3 + b4)
                 for a, b1, b2, b3, b4 in zip(y, k1, k2, k3, k4))


def rk3(model, comp, y, h):
    """One step of Kutta's third-order Runge-Kutta method (Sec. 2.4 integrates the system with a
    third-order Runge-Kutta method without naming the variant): k1 = f(y), k2 = f(y + h k1 / 2),
    k3 = f(y - h k1 + 2 h k2), y + h (k1 + 4 k2 + k3) / 6."""
    k1 = rhs(model, comp, y)
    k2 = rhs(model, comp, _axpy(y, 0.5 * h, k1))
    k3 = rhs(model, comp, _axpy(_axpy(y, -h, k1), 2.0 * h, k2))
    return tuple(a + _bcast(h / 6.0, a) * (b1 + 4.0 * b2 + b3) for a, b1, b2, b3 in zip(y, k1, k2, k3))


STEPPERS = {"rk4": rk4, "rk3": rk3}


def threshold(Y):
    """Waiting-time threshold: the hop test exp(-Lam) <= 1 - Y, i.e. Lam >= -log(1 - Y)."""
    return -np.log(1.0 - Y)


def hop_event(model, ens, idx, seed, times=None, tie_rel=TIE_REL):
    """Apply a hop to each beam in idx at its current state (Sec. 2.4 step 5).

    Destination j != l drawn with probability |gamma_jl| / sum_k |gamma_kl|;
    omega += i arg gamma_jl (unit phase); Re omega accumulated into logw;
    a new waiting-time threshold is drawn.
    """
    idx = np.asarray(idx, dtype=np.int64)
    if idx.size == 0:
        return
    G = model.gamma(ens.X[idx])
    for t, b in enumerate(idx):
        l = int(ens.comp[b])
        w = philox.block(seed, int(ens.gid[b]), int(ens.nhop[b]) + 1, philox.TAG_HOP)
        U, Y = philox.u01(w[0]), philox.u01(w[1])
        # |gamma_jl| and gamma_jl/|gamma_jl| with CPython's complex abs (hypot), which is
        # exact for real gamma: the phase factor exp(i arg gamma) is then exactly +-1
        col = [complex(g) for g in G[t, :, l]]
        order = [j for j in range(model.n_comp) if j != l]
        R = 0.0
        for j in order:
            R = R + abs(col[j])
        dest = l
        if R > 0.0:
            C = 0.0
            last_pos = l
            for j in order:
                C = C + abs(col[j])
                if abs(col[j]) > 0.0:
                    last_pos = j
                if abs(U * R - C) <= tie_rel * R:
                    ens.dest_ties[b] += 1
            C = 0.0
            for j in order:
                C = C + abs(col[j])
                if U * R < C:
                    dest = j
                    break
            else:
                dest = last_pos
            ens.phase[b] = ens.phase[b] * (col[dest] / abs(col[dest]))
        else:
            ens.zero_rate[b] += 1
        ens.logw[b] += ens.Lam[b]
        ens.Lam[b] = 0.0
        ens.comp[b] = dest
        ens.nhop[b] += 1
        ens.E[b] = threshold(Y)
        ens.hop_log[b].append((ens.interval, dest, None if times is None else float(times[t])))


def advance_interval(model, ens, dt, seed, cap=HOP_CAP, tie_rel=TIE_REL, scheme="rk4"):
    """Advance every beam over one interval of length dt (Sec. 2.4 steps 3-5) with the
    Runge-Kutta scheme named by `scheme` ("rk4" classical, "rk3" Kutta's third order)."""
    step = STEPPERS[scheme]
    n = ens.n
    rem = np.full(n, float(dt))
    hops_here = np.zeros(n, dtype=np.int64)
    active = np.ones(n, dtype=bool)
    while active.any():
        ia = np.flatnonzero(active)
        y0 = ens.ode(ia)
        comp = ens.comp[ia]
        yt = step(model, comp, y0, rem[ia])
        L0, L1, E = y0[-1], yt[-1], ens.E[ia]
        capped = hops_here[ia] >= cap
        tie = (~capped) & (np.abs(L1 - E) <= tie_rel * E)
        ens.thr_ties[ia[tie]] += 1
        cross = (~capped) & (L1 >= E)
        ens.cap_overflow[ia[capped]] += 1
        # step 5 without a hop: the trial step is the step
        acc = ~cross
        ens.set_ode(ia[acc], tuple(v[acc] for v in yt))
        active[ia[acc]] = False
        if not cross.any():
            continue
        # step 4: hop time by linear interpolation of the integrated rate
        ic = ia[cross]
        L0c, L1c, Ec = L0[cross], L1[cross], E[cross]
        with np.errstate(divide="ignore", invalid="ignore"):
            theta = np.where(Ec <= L0c, 0.0, (Ec - L0c) / (L1c - L0c))
        ynew = tuple(v[cross] for v in y0)
        part = (theta > 0.0) & (theta < 1.0)
        if part.any():
            yp = step(model, comp[cross][part], tuple(v[part] for v in ynew),
                     theta[part] * rem[ic][part])
            ynew = tuple(_put(v, part, w) for v, w in zip(ynew, yp))
        full = theta >= 1.0
        if full.any():
            ynew = tuple(_put(v, full, w[cross][full]) for v, w in zip(ynew, yt))
        ens.set_ode(ic, ynew)
        # step 5 with a hop
        t_hop = ens.interval * dt + (dt - rem[ic]) + theta * rem[ic]
        hop_event(model, ens, ic, seed, t_hop, tie_rel)
        hops_here[ic] += 1
        rem[ic] = rem[ic] * (1.0 - theta)
        active[ic] = rem[ic] > 0.0
    ens.interval += 1


def _put(v, mask, w):
    v = v.copy()
    v[mask] = w
    return v


def advance(model, ens, nsteps, dt, seed, cap=HOP_CAP, tie_rel=TIE_REL, scheme="rk4"):
    for _ in range(int(nsteps)):
        advance_interval(model, ens, dt, seed, cap, tie_rel, scheme)
    return ens
