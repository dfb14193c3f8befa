"""Fixed-iteration Jacobi-preconditioned CG and one reconstructor time step
(Sec. 3.3, Algorithm 1 in open loop, with F = I).

Readings:
* The paper's preconditioner input J^{-1/2} (split form) and the textbook
  form z = J^{-1} r give the same iterates in exact arithmetic; the textbook
  form is used.
* Warm restart: initial guess c^(i), r_0 = (b^(i+1) - b^(i)) + r^(i); with
  cfg["augment"] = m > 0 the step runs the augmented PCG of augmented.py
  with the previous step's first m search directions (Sec. 3.3).
* r^(i) is the final recurrence residual of the previous step.
* A residual that vanishes exactly (a zero right-hand side) gives p = 0 and
  p^T M p = 0: the step then keeps the iterate (alpha = 0, and beta = 0 when
  the previous rho is 0), i.e. CG stops at the exact solution instead of
  dividing 0 by 0.
* Open loop, a^(i+1) = (1 - gain) a^(i) + gain * F W^{-1} c^(i+1), F = I when
  the reconstruction layers sit at the DM altitudes.
* Closed loop (cfg["loop"] == "closed"), with the two-step delay of
  Algorithm 1: the measurement of step i+1 was taken with the commands
  a^(i-1) on the mirrors, so the pseudo-open-loop slopes are
  s + Gamma a^(i-1), Gamma being the mirrors' slope response; with F = I the
  mirrors are the reconstruction layers and that response is A itself.  The
  control is a^(i+1) = a^(i) + gain (a~ - a^(i-1)).
"""

import numpy as np


def pcg(apply_M, x0, r0, Jdiag, iters, record=None):
    """Textbook PCG for a fixed number of iterations (no convergence test).
    Returns (x, r, history) with history the per-iteration (rho, pi); the
    search directions are appended to ``record`` when it is a list."""
    x = np.array(x0, dtype=np.float64, copy=True)
    r = np.array(r0, dtype=np.float64, copy=True)
    z = r / Jdiag
    p = z.copy()
    rho = r @ z
    hist = []
    for _ in range(iters):
        if record is not None:
            record.append(p.copy())
        q = apply_M(p)
        pi = p @ q
        a = rho / pi if pi > 0.0 else 0.0
        x += a * p
        r -= a * q
        z = r / Jdiag
        rho_new = r @ z
        hist.append((rho, pi))
        beta = rho_new / rho if rho != 0.0 else 0.0
        p = z + beta * p
        rho = rho_new
    return x, r, hist


def pcg_to_tolerance(apply_M, b, Jdiag, rtol=1e-12, max_iters=100000, x0=None):
    """PCG from x0 (default 0) until ||r|| <= rtol ||b|| (used as the exact
    MAP solution c* = M^{-1} b for convergence checks)."""
    x = np.zeros_like(b) if x0 is None else np.array(x0, dtype=np.float64, copy=True)
    r = b - apply_M(x) if x0 is not None else np.array(b, dtype=np.float64, copy=True)
    z = r / Jdiag
    p = z.copy()
    rho = r @ z
    nb = np.linalg.norm(b)
    it = 0
    while np.linalg.norm(r) > rtol * nb and it < max_iters:
        q = apply_M(p)
        a = rho / (p @ q)
        x += a * p
        r -= a * q
        z = r / Jdiag
        rho_new = r @ z
        p = z + (rho_new / rho) * p
        rho = rho_new
        it += 1
    return x, it


class State:
    """Algorithm 1's state between frames: c, b, r, a^(i-1), a^(i) and, for
    the augmented PCG, the previous step's search directions P and their
    images Q = M P (at most `keep` of each).

    Packed layout: [c | b | r | a_prev | a], then with keep > 0
    [P_0 .. P_{keep-1} | Q_0 .. Q_{keep-1} | count, 0, 0, 0], the directions
    past `count` zero."""

    def __init__(self, n_coeff, n_act, keep=0):
        self.c = np.zeros(n_coeff)
        self.b = np.zeros(n_coeff)
        self.r = np.zeros(n_coeff)
        self.a_prev = np.zeros(n_act)
        self.a = np.zeros(n_act)
        self.keep = keep
        self.P = []
        self.Q = []

    def pack(self):
        parts = [self.c, self.b, self.r, self.a_prev, self.a]
        if self.keep:
            n = len(self.c)
            pad = [np.zeros(n)] * (self.keep - len(self.P))
            parts += list(self.P) + pad + list(self.Q) + pad + [np.array([len(self.P), 0.0, 0.0, 0.0])]
        return np.concatenate(parts)

    @classmethod
    def unpack(cls, v, n_coeff, n_act, keep=0):
        st = cls(n_coeff, n_act, keep)
        v = np.asarray(v, dtype=np.float64)
        o = 0
        for name, n in (("c", n_coeff), ("b", n_coeff), ("r", n_coeff), ("a_prev", n_act), ("a", n_act)):
            setattr(st, name, v[o:o + n].copy())
            o += n
        if keep:
            count = int(v[o + 2 * keep * n_coeff])
            st.P = [v[o + k * n_coeff:o + (k + 1) * n_coeff].copy() for k in range(count)]
            o += keep * n_coeff
            st.Q = [v[o + k * n_coeff:o + (k + 1) * n_coeff].copy() for k in range(count)]
        return st


def frame(system, state, s, iters=None, gain=None, refresh=False):
    """One time step (open or closed loop, F = I); returns (new_state,
    layers phi = W^{-1} c).  refresh: start from the true residual
    b - M c^(i) instead of the recurrence (b - b^(i)) + r^(i) (the two agree
    in exact arithmetic when r^(i) is the previous step's residual)."""
    cfg = system.cfg
    iters = cfg["iters"] if iters is None else iters
    gain = cfg["gain"] if gain is None else gain
    closed = cfg.get("loop", "open") == "closed"
    if closed:  # pseudo-open-loop measurement (two-step delay)
        s = np.asarray(s, dtype=np.float64) + system.apply_A(state.a_prev)
    b = system.rhs(s)
    r0 = b - system.apply_M(state.c) if refresh else (b - state.b) + state.r
    J = system.preconditioner()
    keep = cfg.get("augment", 0)
    new = State(len(state.c), len(state.a), keep)
    if keep:  # augmented PCG with the previous step's directions (Sec. 3.3)
        from .augmented import aug_pcg
        x, r, new.P, new.Q, _ = aug_pcg(system.apply_M, state.c, r0, J, iters, state.P, state.Q, keep)
    else:
        x, r, _ = pcg(system.apply_M, state.c, r0, J, iters)
    phi = system.W_inv(x)
    new.c = x
    new.b = b
    new.r = r
    new.a_prev = state.a.copy()
    if closed:
        new.a = state.a + gain * (phi - state.a_prev)
    else:
        new.a = (1.0 - gain) * state.a + gain * phi
    return new, phi
