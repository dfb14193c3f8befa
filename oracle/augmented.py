"""Augmented (deflated) PCG reusing the previous time step's search
directions (Sec. 3.3, "Convergence improvements"; Algorithm 1, the augPCG
line with inputs P^(i), Q^(i) = M P^(i) and outputs P^(i+1), Q^(i+1)).

The paper specifies the method only by reference to another paper of its
authors.  The algorithm used here is the deflated conjugate gradient of
Saad, Yeung, Erhel and Guyomarc'h ("A deflated version of the conjugate
gradient algorithm", SIAM J. Sci. Comput. 21(5), 2000), with the Jacobi
preconditioner, augmentation space W = P^(i) (the columns are the previous
step's search directions) and A W = Q^(i):

* start:   G = W^T A W;  x_0 = x + W G^{-1} W^T r;  r_0 = r - A W G^{-1} W^T r
           (the warm-start residual of Algorithm 1 projected so that
           W^T r_0 = 0);
           z_0 = J^{-1} r_0;  p_0 = z_0 - W mu_0,  G mu_0 = (A W)^T z_0;
* step j:  alpha = r_j^T z_j / p_j^T A p_j;  x += alpha p_j;  r -= alpha A p_j;
           z = J^{-1} r;  beta = r_{j+1}^T z_{j+1} / r_j^T z_j;
           G mu = (A W)^T z_{j+1};  p_{j+1} = z_{j+1} + beta p_j - W mu.

Every residual stays orthogonal to W and every new direction A-conjugate
to it.  The step's own directions p_j and A p_j (its first `keep`) are the
next step's W and A W.

Readings:
* G is factored by Cholesky; a direction whose pivot is not positive
  (a zero direction, or one dependent on the others, e.g. after a step
  that met an exact solution) is dropped: its coefficient is 0 and its
  row and column are left out.
* With no previous directions (the first frame) the method is the plain
  PCG of solver.pcg, operation for operation.
* alpha = 0 when p^T A p <= 0 and beta = 0 after a zero rho, as in
  solver.pcg.
"""

import numpy as np


def factor(G):
    """Cholesky factor of the small SPD matrix G with dropped directions:
    returns (L, keep) with keep[k] False where the pivot of direction k was
    not positive (L's row and column k are then zero)."""
    m = G.shape[0]
    L = np.zeros((m, m))
    keep = np.zeros(m, dtype=bool)
    for k in range(m):
        d = G[k, k] - sum(L[k, i] * L[k, i] for i in range(k) if keep[i])
        if not (d > 0.0) or not np.isfinite(d):
            continue
        keep[k] = True
        L[k, k] = np.sqrt(d)
        for r in range(k + 1, m):
            L[r, k] = (G[r, k] - sum(L[r, i] * L[k, i] for i in range(k) if keep[i])) / L[k, k]
    return L, keep


def solve(L, keep, v):
    """G^{-1} v on the kept directions (0 on the dropped ones)."""
    m = len(v)
    y = np.zeros(m)
    for k in range(m):  # L y = v
        if keep[k]:
            y[k] = (v[k] - sum(L[k, i] * y[i] for i in range(k) if keep[i])) / L[k, k]
    x = np.zeros(m)
    for k in reversed(range(m)):  # L^T x = y
        if keep[k]:
            x[k] = (y[k] - sum(L[i, k] * x[i] for i in range(k + 1, m) if keep[i])) / L[k, k]
    return x


def aug_pcg(apply_M, x0, r0, Jdiag, iters, P, Q, keep_dirs, record=None):
    """Deflated PCG for a fixed number of iterations from the iterate x0 with
    residual r0 and the previous directions P (list of vectors) with
    Q = [M p for p in P].  Returns (x, r, P_new, Q_new, history); history
    holds the per-iteration (rho, pi); P_new / Q_new are the first
    keep_dirs directions of this run and their images under M; `record`, a
    list, receives (P^T r_j, Q^T p_j) after the start and every step."""
    x = np.array(x0, dtype=np.float64, copy=True)
    r = np.array(r0, dtype=np.float64, copy=True)
    m = len(P)
    W = np.stack(P, axis=1) if m else np.zeros((len(x), 0))
    AW = np.stack(Q, axis=1) if m else np.zeros((len(x), 0))
    if m:
        L, kept = factor(W.T @ AW)
        y = solve(L, kept, W.T @ r)
        x += W @ y
        r -= AW @ y
    z = r / Jdiag
    p = z - W @ solve(L, kept, AW.T @ z) if m else z.copy()
    rho = r @ z
    hist, P_new, Q_new = [], [], []
    for j in range(iters):
        if record is not None:
            record.append((W.T @ r, AW.T @ p))
        q = apply_M(p)
        if j < keep_dirs:
            P_new.append(p.copy())
            Q_new.append(q.copy())
        pi = p @ q
        a = rho / pi if pi > 0.0 else 0.0
        x += a * p
        r -= a * q
        z = r / Jdiag
        rho_new = r @ z
        hist.append((rho, pi))
        beta = rho_new / rho if rho != 0.0 else 0.0
        p = z + beta * p
        if m:
            p -= W @ solve(L, kept, AW.T @ z)
        rho = rho_new
    if record is not None:
        record.append((W.T @ r, AW.T @ p))
    return x, r, P_new, Q_new, hist
