"""The l1-penalised quantile-regression linear program, solved three independent ways.

Test infrastructure only.  Writing beta = b+ - b-, and the residual y - X1 beta =
u - v with b+, b-, u, v >= 0, the penalised QR problem (eq. vanilla_QR with the
weighted-l1 penalty) is the LP

    min  sum_j lam_j (b+_j + b-_j) + (tau/n) 1^T u + ((1-tau)/n) 1^T v
    s.t. X1 (b+ - b-) + u - v = y,   all variables >= 0,

the Koenker-Bassett form extended by the penalty (lam_0 = 0: free intercept).

* ``simplex_exact``: dense two-phase simplex with Bland's anti-cycling rule over
  ``fractions.Fraction`` (exact; tiny inputs only).
* ``vertex_enumeration``: brute force in beta-space.  P(beta) is convex and
  piecewise linear; its kinks lie on the hyperplanes x_i^T beta = y_i and
  beta_j = 0 (lam_j > 0).  A minimiser is attained at an intersection of p+1
  independent kink hyperplanes, so the minimum over all such intersections is
  the optimum (exact rationals; p+1 <= 4).
* ``highs``: scipy.optimize.linprog(method="highs") on the same LP in floats.

The LP dual is  max y^T theta  s.t.  (tau-1)/n <= theta_i <= tau/n,
|x_j^T theta| <= lam_j  (A^T theta <= c for A = [X1, -X1, I, -I]), the dual of the
Lagrangian eq. main_lagrangian; ``simplex_exact(..., duals=True)`` returns its
optimal theta as c_B^T B^-1 from the final tableau, ``highs_with_duals`` HiGHS's
equality marginals, and ``highs_face_range`` the range of chosen coefficients over
the optimal face (minimise and maximise beta_j subject to the objective staying at
the optimum): a library-side test of the uniqueness of the minimiser.
"""
from fractions import Fraction
from itertools import combinations

import numpy as np


def _F(x):
    return x if isinstance(x, Fraction) else Fraction(x)


def lp_data(X1, y, tau, lam):
    """Return (c, A, b) of the standard-form LP (lists of Fractions)."""
    n = len(y)
    p1 = len(X1[0])
    tau = _F(tau)
    c = [_F(l) for l in lam] + [_F(l) for l in lam] + [tau / n] * n + [(1 - tau) / n] * n
    A = []
    for i in range(n):
        row = [_F(X1[i][j]) for j in range(p1)] + [-_F(X1[i][j]) for j in range(p1)]
        row += [Fraction(1) if k == i else Fraction(0) for k in range(n)]
        row += [Fraction(-1) if k == i else Fraction(0) for k in range(n)]
        A.append(row)
    b = [_F(v) for v in y]
    return c, A, b


def _pivot(T, r, col):
    piv = T[r][col]
    T[r] = [v / piv for v in T[r]]
    for i in range(len(T)):
        if i != r and T[i][col] != 0:
            f = T[i][col]
            T[i] = [a - f * b for a, b in zip(T[i], T[r])]


def _simplex_phase(T, basis, cost, allowed):
    """Minimise cost^T x over the tableau T (rows [A | b]) with Bland's rule."""
    m = len(T)
    ncol = len(T[0]) - 1
    while True:
        # reduced costs d_j = c_j - c_B^T T[:, j]
        enter = None
        for j in range(ncol):
            if not allowed[j] or j in basis:
                continue
            d = cost[j] - sum(cost[basis[i]] * T[i][j] for i in range(m))
            if d < 0:
                enter = j
                break
        if enter is None:
            return
        best = None
        for i in range(m):
            a = T[i][enter]
            if a > 0:
                ratio = T[i][-1] / a
                if best is None or ratio < best[0] or (ratio == best[0] and basis[i] < basis[best[1]]):
                    best = (ratio, i)
        if best is None:
            raise RuntimeError("LP unbounded")
        _pivot(T, best[1], enter)
        basis[best[1]] = enter


def simplex_exact(c, A, b, duals=False):
    """Exact two-phase simplex.  Returns (optimal value, x) as Fractions, and with
    duals=True also the optimal dual y = c_B^T B^-1 of the equality rows (read from
    the artificial columns of the final tableau, which hold B^-1 of the sign-adjusted
    rows).  A holds an identity block here, so no row is ever redundant."""
    m, nv = len(A), len(c)
    T = []
    for i in range(m):
        sgn = -1 if b[i] < 0 else 1
        row = [sgn * a for a in A[i]] + [Fraction(1) if k == i else Fraction(0) for k in range(m)]
        T.append(row + [sgn * b[i]])
    basis = [nv + i for i in range(m)]
    cost1 = [Fraction(0)] * nv + [Fraction(1)] * m
    _simplex_phase(T, basis, cost1, [True] * (nv + m))
    if sum(T[i][-1] for i in range(m) if basis[i] >= nv) != 0:
        raise RuntimeError("LP infeasible")
    # drive zero-level artificials out of the basis (or drop redundant rows)
    keep = []
    for i in range(m):
        if basis[i] >= nv:
            col = next((j for j in range(nv) if T[i][j] != 0), None)
            if col is None:
                continue
            _pivot(T, i, col)
            basis[i] = col
        keep.append(i)
    if duals and len(keep) != m:
        raise RuntimeError("redundant equality rows: duals not defined by the tableau")
    T = [T[i] for i in keep]
    basis = [basis[i] for i in keep]
    cost2 = list(c) + [Fraction(0)] * m
    allowed = [True] * nv + [False] * m
    _simplex_phase(T, basis, cost2, allowed)
    x = [Fraction(0)] * nv
    for i, bi in enumerate(basis):
        if bi < nv:
            x[bi] = T[i][-1]
    val = sum(ci * xi for ci, xi in zip(c, x))
    if not duals:
        return val, x
    sgn = [-1 if bv < 0 else 1 for bv in b]
    y = [sgn[i] * sum(cost2[basis[r]] * T[r][nv + i] for r in range(len(T))) for i in range(m)]
    return val, x, y


def objective_exact(X1, y, beta, tau, lam):
    n = len(y)
    tau = _F(tau)
    tot = Fraction(0)
    for i in range(n):
        r = _F(y[i]) - sum(_F(X1[i][j]) * beta[j] for j in range(len(beta)))
        tot += (tau - (1 if r < 0 else 0)) * r
    return tot / n + sum(abs(_F(l) * bj) for l, bj in zip(lam, beta))


def _solve_exact(M, rhs):
    """Gauss-Jordan over Fractions; returns None if singular."""
    k = len(M)
    A = [list(M[i]) + [rhs[i]] for i in range(k)]
    for col in range(k):
        piv = next((r for r in range(col, k) if A[r][col] != 0), None)
        if piv is None:
            return None
        A[col], A[piv] = A[piv], A[col]
        pv = A[col][col]
        A[col] = [v / pv for v in A[col]]
        for r in range(k):
            if r != col and A[r][col] != 0:
                f = A[r][col]
                A[r] = [a - f * b for a, b in zip(A[r], A[col])]
    return [A[i][-1] for i in range(k)]


def vertex_enumeration(X1, y, tau, lam):
    """Minimum of P over all intersections of p+1 kink hyperplanes (exact)."""
    n = len(y)
    p1 = len(X1[0])
    planes = [([_F(v) for v in X1[i]], _F(y[i])) for i in range(n)]
    for j in range(1, p1):
        if _F(lam[j]) > 0:
            e = [Fraction(0)] * p1
            e[j] = Fraction(1)
            planes.append((e, Fraction(0)))
    best = None
    for sub in combinations(range(len(planes)), p1):
        sol = _solve_exact([planes[s][0] for s in sub], [planes[s][1] for s in sub])
        if sol is None:
            continue
        val = objective_exact(X1, y, sol, tau, lam)
        if best is None or val < best[0]:
            best = (val, sol)
    return best


def optimal_vertices(X1, y, tau, lam):
    """Every distinct kink-hyperplane intersection attaining the minimum (exact).  The
    minimiser set of the convex piecewise-linear P is a polyhedron whose vertices are
    among these points; one point means a unique minimiser (when that set is
    bounded, as it is whenever the design has full column rank)."""
    n = len(y)
    p1 = len(X1[0])
    planes = [([_F(v) for v in X1[i]], _F(y[i])) for i in range(n)]
    for j in range(1, p1):
        if _F(lam[j]) > 0:
            e = [Fraction(0)] * p1
            e[j] = Fraction(1)
            planes.append((e, Fraction(0)))
    best, pts = None, set()
    for sub in combinations(range(len(planes)), p1):
        sol = _solve_exact([planes[s][0] for s in sub], [planes[s][1] for s in sub])
        if sol is None:
            continue
        val = objective_exact(X1, y, sol, tau, lam)
        if best is None or val < best:
            best, pts = val, {tuple(sol)}
        elif val == best:
            pts.add(tuple(sol))
    return best, sorted(pts)


def highs(X1, y, tau, lam):
    """HiGHS (via scipy) on the same LP in floats.  Returns (value, beta)."""
    from scipy.optimize import linprog
    from scipy.sparse import csr_matrix, hstack, identity
    X1 = np.asarray(X1, dtype=np.float64)
    n, p1 = X1.shape
    lam = np.asarray(lam, dtype=np.float64)
    c = np.concatenate([lam, lam, np.full(n, tau / n), np.full(n, (1 - tau) / n)])
    Xs = csr_matrix(X1)
    A = hstack([Xs, -Xs, identity(n, format="csr"), -identity(n, format="csr")], format="csr")
    res = linprog(c, A_eq=A, b_eq=np.asarray(y, dtype=np.float64), bounds=(0, None),
                  method="highs", options={"primal_feasibility_tolerance": 1e-10,
                                           "dual_feasibility_tolerance": 1e-10})
    if res.status != 0:
        raise RuntimeError(res.message)
    x = res.x
    return float(res.fun), x[:p1] - x[p1:2 * p1]


def _highs_lp(X1, y, tau, lam):
    from scipy.sparse import csr_matrix, hstack, identity
    X1 = np.asarray(X1, dtype=np.float64)
    n, p1 = X1.shape
    lam = np.asarray(lam, dtype=np.float64)
    c = np.concatenate([lam, lam, np.full(n, tau / n), np.full(n, (1 - tau) / n)])
    Xs = csr_matrix(X1)
    A = hstack([Xs, -Xs, identity(n, format="csr"), -identity(n, format="csr")], format="csr")
    return c, A, np.asarray(y, dtype=np.float64), p1


_HIGHS_OPT = {"primal_feasibility_tolerance": 1e-10, "dual_feasibility_tolerance": 1e-10}


def highs_with_duals(X1, y, tau, lam):
    """HiGHS on the LP; returns (value, beta, theta) with theta the equality
    marginals, i.e. an optimal point of the dual above."""
    from scipy.optimize import linprog
    c, A, b, p1 = _highs_lp(X1, y, tau, lam)
    res = linprog(c, A_eq=A, b_eq=b, bounds=(0, None), method="highs", options=_HIGHS_OPT)
    if res.status != 0:
        raise RuntimeError(res.message)
    x = res.x
    return float(res.fun), x[:p1] - x[p1:2 * p1], np.asarray(res.eqlin.marginals, dtype=np.float64)


def highs_face_range(X1, y, tau, lam, value, cols, rel=1e-9):
    """For each j in cols: (min, max) of beta_j over {feasible, objective <= value (1 +
    rel) + rel}, the optimal face widened by rel.  A face of width ~0 in every
    coordinate means the minimiser is unique (up to the widening)."""
    from scipy.optimize import linprog
    c, A, b, p1 = _highs_lp(X1, y, tau, lam)
    bound = value * (1 + rel) + rel
    out = []
    for j in cols:
        e = np.zeros_like(c)
        e[j], e[p1 + j] = 1.0, -1.0
        lo = linprog(e, A_ub=c[None, :], b_ub=[bound], A_eq=A, b_eq=b, bounds=(0, None),
                     method="highs", options=_HIGHS_OPT)
        hi = linprog(-e, A_ub=c[None, :], b_ub=[bound], A_eq=A, b_eq=b, bounds=(0, None),
                     method="highs", options=_HIGHS_OPT)
        if lo.status != 0 or hi.status != 0:
            raise RuntimeError(lo.message if lo.status else hi.message)
        out.append((float(lo.fun), float(-hi.fun)))
    return out
