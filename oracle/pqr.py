"""Plain FP64 implementation of weighted-l1 PQR and of FS-QRPPA (Algorithm 1).

Test infrastructure only (see the package docstring).  Everything here is
written for a reader to check against the paper by eye: no blocking, fusion
or reordering beyond what the equations state.

Conventions
-----------
* ``X1`` is the n x (p+1) design WITH the intercept as column 0 (Sec. 1, the
  feature vector x_i = (1, x_i1, ..., x_ip)).
* ``lam`` is the (p+1)-vector of penalty weights with lam[0] = 0, so the
  intercept is never penalised (weighted-l1 penalty equation).
* A partition of the columns into G contiguous blocks (decomposition of X
  into X_1..X_G) is a list ``blocks`` of index arrays over 0..p.

Pins (see tests/test_oracle_*.py): prox maps against brute-force 1-D
minimisation; lambda_max and the intercept-only fit against the sample-quantile
closed form; the full solve against an exact rational simplex, vertex
enumeration and HiGHS; the certificates (FP64 and on the quantised dual point) by
weak duality, exact feasibility and agreement with each other; the step by the
non-increase of the H-norm successive difference.
"""
import math

import numpy as np


# ----------------------------------------------------------------------------
# Objective (eq. vanilla_QR with the weighted-l1 penalty)
# ----------------------------------------------------------------------------

def pinball(u, tau):
    """rho_tau(u) = (tau - 1{u < 0}) u, elementwise (Sec. 1)."""
    u = np.asarray(u, dtype=np.float64)
    return (tau - (u < 0).astype(np.float64)) * u


def _sum(a):
    a = np.asarray(a, dtype=np.float64).ravel()
    return math.fsum(a) if a.size <= 200_000 else float(np.sum(a))


def objective(X1, y, beta, tau, lam):
    """P(beta) = (1/n) sum_i rho_tau(y_i - x_i^T beta) + sum_{j>=1} lam_j |beta_j|."""
    n = X1.shape[0]
    r = y - X1 @ beta
    return _sum(pinball(r, tau)) / n + _sum(np.abs(lam * beta))


def penalty(beta, lam):
    return _sum(np.abs(lam * beta))


# ----------------------------------------------------------------------------
# Closed-form updates (eqs. beta_update and z_update)
# ----------------------------------------------------------------------------

def beta_prox(beta_g, v_g, lam_g, eta_g):
    """beta_update: (1/eta)[(eta b + v - lam)_+ - (-eta b - v - lam)_+], v = X_g^T theta."""
    a = eta_g * beta_g + v_g
    return (np.maximum(a - lam_g, 0.0) - np.maximum(-a - lam_g, 0.0)) / eta_g


def z_prox(z, theta, tau, n, mu):
    """z_update: (z + theta/mu - tau/(n mu))_+ - (-z - theta/mu - (1-tau)/(n mu))_+."""
    u = z + theta / mu
    return np.maximum(u - tau / (n * mu), 0.0) - np.maximum(-u - (1.0 - tau) / (n * mu), 0.0)


# ----------------------------------------------------------------------------
# Partition and step sizes (decomposition of X; M_g = eta_g I, eta_g > mu Lambda_max)
# ----------------------------------------------------------------------------

def partition(p, G, align=1, intercept_block=False):
    """Contiguous near-equal blocks over the p feature columns (the decomposition
    of X into X_1..X_G; the paper fixes only sum p_g = p + 1).  Feature boundaries
    b_g = align * floor(g * ceil(p/align) / G), b_G = p.  The intercept (column 0)
    is either the first column of the first block, or, with intercept_block, a
    block of its own placed first (G + 1 blocks in all).  Returns a list of index
    arrays over the full columns 0..p."""
    units = -(-p // align)
    if not 1 <= G <= units:
        raise ValueError("need 1 <= G <= ceil(p / align)")
    b = [min(p, align * ((g * units) // G)) for g in range(G)] + [p]
    blocks = [np.array([0])] if intercept_block else []
    for g in range(G):
        cols = np.arange(1 + b[g], 1 + b[g + 1])
        if g == 0 and not intercept_block:
            cols = np.concatenate([[0], cols])
        blocks.append(cols)
    return blocks


def block_lambda_max(Xg):
    """Largest eigenvalue of X_g^T X_g, computed as the top singular value squared."""
    if min(Xg.shape) <= 400:
        s = np.linalg.svd(Xg, compute_uv=False)
        return float(s[0] ** 2)
    from scipy.sparse.linalg import svds
    s = svds(Xg, k=1, return_singular_vectors=False, tol=1e-12, random_state=0)
    return float(s[0] ** 2)


def step_sizes(X1, blocks, mu, margin=0.01):
    """eta_g = (1 + margin) * mu * Lambda_max(X_g^T X_g) (text after eq. fsppa_update)."""
    return np.array([(1.0 + margin) * mu * block_lambda_max(X1[:, b]) for b in blocks])


def default_mu(y, G, scale=1.0):
    """Reading of the unstated augmentation parameter: mu = scale*sqrt(G+1)/(n sd(y))."""
    n = len(y)
    return scale * math.sqrt(G + 1.0) / (n * float(np.std(y)))


# ----------------------------------------------------------------------------
# Algorithm 1 (FS-QRPPA), one step and the loop
# ----------------------------------------------------------------------------

def fsqrppa_step(X1, y, tau, lam, blocks, mu, eta, beta, z, theta):
    """One pass of the while-loop body of Algorithm 1, in its order:
    parallel-for over blocks (beta_update), then z (z_update), then theta
    (third line of eq. fsppa_update).  Returns the new (beta, z, theta)."""
    n = X1.shape[0]
    G = len(blocks)
    beta_new = beta.copy()
    for g, cols in enumerate(blocks):
        v_g = X1[:, cols].T @ theta
        beta_new[cols] = beta_prox(beta[cols], v_g, lam[cols], eta[g])
    z_new = z_prox(z, theta, tau, n, mu)
    r_new = sum(X1[:, cols] @ beta_new[cols] for cols in blocks) + z_new - y
    r_old = sum(X1[:, cols] @ beta[cols] for cols in blocks) + z - y
    theta_new = theta - (mu / (G + 1.0)) * (2.0 * r_new - r_old)
    return beta_new, z_new, theta_new


def fsqrppa_step_cached(X1, y, tau, lam, blocks, mu, eta, beta, z, theta, r):
    """fsqrppa_step with r^k = X beta^k + z^k - y carried from the previous step (the
    third line of eq. fsppa_update needs r^k, which the previous step computed), so a
    step costs two products with X instead of three.  Returns (beta, z, theta, r)."""
    n = X1.shape[0]
    G = len(blocks)
    beta_new = beta.copy()
    for g, cols in enumerate(blocks):
        v_g = X1[:, cols].T @ theta
        beta_new[cols] = beta_prox(beta[cols], v_g, lam[cols], eta[g])
    z_new = z_prox(z, theta, tau, n, mu)
    r_new = X1 @ beta_new + z_new - y
    theta_new = theta - (mu / (G + 1.0)) * (2.0 * r_new - r)
    return beta_new, z_new, theta_new, r_new


def h_norm_sq(X1, blocks, mu, eta, d_beta, d_z, d_theta):
    """||dw||_H^2 with H = [[D, A^T], [A, ((G+1)/mu) I]], D = diag(eta_g I, mu I),
    A = [X, I]: the metric in which the iteration is a proximal point step
    (Theorem 1 names such an H; its form is derived from eq. fsppa_update)."""
    G = len(blocks)
    q = sum(eta[g] * float(d_beta[c] @ d_beta[c]) for g, c in enumerate(blocks))
    q += mu * float(d_z @ d_z)
    q += 2.0 * float(d_theta @ (X1 @ d_beta + d_z))
    q += ((G + 1.0) / mu) * float(d_theta @ d_theta)
    return q


def zero_start(y, p1):
    """beta = 0, z = y, theta = 0 (so the first residual Xbeta + z - y is 0)."""
    return np.zeros(p1), np.array(y, dtype=np.float64), np.zeros(len(y))


def fsqrppa(X1, y, tau, lam, blocks, mu, eta, start=None, max_iter=100_000,
            tol_gap=1e-10, check_every=10, record=False):
    """Iterate Algorithm 1 until the FP64 relative duality gap (dual_certificate)
    is at most tol_gap.  Returns dict(beta, z, theta, iters, rel_gap, history)."""
    n, p1 = X1.shape
    beta, z, theta = zero_start(y, p1) if start is None else (np.array(s, dtype=np.float64)
                                                              for s in start)
    hist = []
    cert = dual_certificate(X1, y, tau, lam, beta, theta)
    k = 0
    while k < max_iter:
        b1, z1, t1 = fsqrppa_step(X1, y, tau, lam, blocks, mu, eta, beta, z, theta)
        if record:
            hist.append(h_norm_sq(X1, blocks, mu, eta, b1 - beta, z1 - z, t1 - theta))
        beta, z, theta = b1, z1, t1
        k += 1
        if k % check_every == 0:
            cert = dual_certificate(X1, y, tau, lam, beta, theta)
            if cert["rel_gap"] <= tol_gap:
                break
    cert = dual_certificate(X1, y, tau, lam, beta, theta)
    return dict(beta=beta, z=z, theta=theta, iters=k, rel_gap=cert["rel_gap"],
                gap=cert["gap"], primal=cert["primal"], dual=cert["dual"], history=hist)


# ----------------------------------------------------------------------------
# lambda_max and the null fit (project reading; the paper does not define it)
# ----------------------------------------------------------------------------

def tau_quantile(y, tau):
    """q = y_(ceil(n tau)), the tau-quantile of the sample (inf{t : F_n(t) >= tau},
    the definition of the conditional quantile in the notation paragraph)."""
    ys = np.sort(np.asarray(y, dtype=np.float64))
    n = len(ys)
    k = max(1, math.ceil(n * tau - 1e-12))
    return float(ys[k - 1])


def quantile_minimizers(y, tau):
    """Closed form of argmin_c sum rho_tau(y_i - c): [y_(n tau), y_(n tau + 1)] if
    n tau is an integer, else {y_(ceil(n tau))}.  Returns (lo, hi)."""
    ys = np.sort(np.asarray(y, dtype=np.float64))
    n = len(ys)
    nt = n * tau
    if abs(nt - round(nt)) < 1e-12 and 1 <= round(nt) < n:
        k = int(round(nt))
        return float(ys[k - 1]), float(ys[k])
    k = math.ceil(nt)
    return float(ys[k - 1]), float(ys[k - 1])


def null_dual(y, tau):
    """psi with psi_i = tau (y_i > q), tau - 1 (y_i < q), and the common value on
    ties with q that makes sum psi = 0.  Returns (q, psi)."""
    y = np.asarray(y, dtype=np.float64)
    q = tau_quantile(y, tau)
    above, below, tie = y > q, y < q, y == q
    psi = np.where(above, tau, tau - 1.0)
    c = -(tau * above.sum() + (tau - 1.0) * below.sum()) / tie.sum()
    psi[tie] = c
    return q, psi


def lambda_max(X1, y, tau, weights=None):
    """Smallest lambda at which (q, 0, ..., 0) is optimal: max_{j>=1} |x_j^T psi| / (n w_j)
    over columns with w_j > 0 (follows from the KKT conditions of Prop. 1)."""
    n, p1 = X1.shape
    _, psi = null_dual(y, tau)
    s = np.abs(X1[:, 1:].T @ psi) / n
    w = np.ones(p1 - 1) if weights is None else np.asarray(weights, dtype=np.float64)[1:]
    pos = w > 0
    return float(np.max(s[pos] / w[pos])) if pos.any() else 0.0


# ----------------------------------------------------------------------------
# Dual certificate and KKT check (Lagrangian eq. main_lagrangian, Prop. 1)
# ----------------------------------------------------------------------------

def project_box_sum(theta, lo, hi, iters=200):
    """theta' = clip(theta - c, lo, hi) with c chosen by bisection so sum theta' = 0."""
    theta = np.asarray(theta, dtype=np.float64)
    a = float(np.min(theta)) - hi
    b = float(np.max(theta)) - lo
    for _ in range(iters):
        c = 0.5 * (a + b)
        s = _sum(np.clip(theta - c, lo, hi))
        if s > 0:
            a = c
        else:
            b = c
        if b - a <= 0:
            break
    return np.clip(theta - 0.5 * (a + b), lo, hi)


def dual_certificate(X1, y, tau, lam, beta, theta):
    """Weak-duality certificate.  The dual of the constrained form is
    max_theta y^T theta  s.t.  (tau-1)/n <= theta_i <= tau/n,  |x_j^T theta| <= lam_j
    (lam_0 = 0 forces sum theta = 0, and any other lam_j = 0 forces x_j^T theta = 0).
    theta is made feasible by a shift-and-clip projection; with unpenalized feature
    columns U it is then projected onto {sum theta = 0, X_U^T theta = 0} (least
    squares) and scaled toward 0, which lies inside the box, until the box holds;
    finally a scaling alpha in (0, 1] meets |x_j^T theta| <= lam_j.  The equality
    constraints hold to rounding.  gap = P(beta) - y^T theta~ >= 0."""
    n = X1.shape[0]
    lo, hi = (tau - 1.0) / n, tau / n
    tp = project_box_sum(theta, lo, hi)
    lj = lam[1:]
    U = np.nonzero(lj == 0)[0]
    if len(U):
        A = np.column_stack([np.ones(n), X1[:, 1 + U]])
        c, *_ = np.linalg.lstsq(A, tp, rcond=None)
        t1 = tp - A @ c
        s = 1.0
        for t in t1:
            if t > hi:
                s = min(s, hi / t)
            elif t < lo:
                s = min(s, lo / t)
        tp = s * t1
    v = X1[:, 1:].T @ tp
    alpha = 1.0
    for vj, l in zip(np.abs(v), lj):
        if l > 0 and vj > l:
            alpha = min(alpha, l / vj)
    tf = alpha * tp
    primal = objective(X1, y, beta, tau, lam)
    dual = _sum(y * tf)
    gap = primal - dual
    return dict(primal=primal, dual=dual, gap=gap, rel_gap=gap / max(abs(primal), 1e-300),
                theta_feasible=tf, alpha=alpha)


def quantize_dual_point(theta, tau, n, slices=4):
    """The exactly representable dual point of the batched reading: theta' (the
    shift-and-clip projection) truncated toward zero to theta_q = unit T, unit = c
    2^-(7 slices - 1) with c the power of two >= max(tau, 1 - tau)/n, the integer sum
    of T moved onto its largest entry (sum > 0) or smallest (sum < 0), first index on
    ties.  Returns (theta_q, T, unit, t_lo, t_hi), or None when that entry would
    leave the box."""
    lo, hi = (tau - 1.0) / n, tau / n
    tp = project_box_sum(theta, lo, hi)
    _, e = math.frexp(max(tau, 1.0 - tau) / n)
    unit = math.ldexp(1.0, e - (7 * slices - 1))
    t_lo, t_hi = math.ceil(lo / unit), math.floor(hi / unit)
    T = np.clip(np.trunc(tp / unit), t_lo, t_hi).astype(np.int64)
    s = int(T.sum())
    if s > 0:
        i = int(np.argmax(T))
        if T[i] - s < t_lo:
            return None
        T[i] -= s
    elif s < 0:
        i = int(np.argmin(T))
        if T[i] - s > t_hi:
            return None
        T[i] -= s
    return T.astype(np.float64) * unit, T, unit, t_lo, t_hi


def dual_value(y, t, max_ratio):
    """Dual objective of the feasible point alpha t, alpha = min(1, 1/max_ratio), where
    t is in the box with sum t = 0 and max_ratio = max_j |x_j^T t| / lam_j over the
    penalized columns (the last step of dual_certificate, for ratios computed
    elsewhere, e.g. column chunk by column chunk)."""
    alpha = 1.0 if max_ratio <= 1.0 else (0.0 if math.isinf(max_ratio) else 1.0 / max_ratio)
    return alpha * _sum(np.asarray(y, dtype=np.float64) * np.asarray(t, dtype=np.float64))


def quantized_dual_certificate(X1, y, tau, lam, beta, theta, slices=4):
    """Weak-duality certificate on an exactly representable dual point (Prop. 1 holds
    for any point of the dual feasible set; the batched form's reading).  theta' is
    the shift-and-clip projection of dual_certificate (positive weights only).  With
    unit = c 2^-(7 slices - 1), c the power of two >= max(tau, 1 - tau)/n, the point
    is theta_q = unit T with T = trunc(theta'/unit) (toward zero, so inside the box).
    The integer sum of T is moved onto its largest entry (sum > 0) or its smallest
    (sum < 0), the first index on ties, so that sum theta_q = 0 exactly; if that
    entry would leave the box the function returns None.  Then alpha = min(1, min_j
    lam_j / |x_j^T theta_q|) and the dual value is alpha y^T theta_q."""
    n = X1.shape[0]
    lam = np.asarray(lam, dtype=np.float64)
    if np.any(lam[1:] <= 0):
        raise ValueError("positive feature weights only")
    q = quantize_dual_point(theta, tau, n, slices)
    if q is None:
        return None
    tq, T, unit, t_lo, t_hi = q
    v = X1[:, 1:].T @ tq
    alpha = 1.0
    for vj, l in zip(np.abs(v), lam[1:]):
        if vj > l:
            alpha = min(alpha, l / vj)
    primal = objective(X1, y, beta, tau, lam)
    dual = alpha * _sum(y * tq)
    gap = primal - dual
    return dict(primal=primal, dual=dual, gap=gap, rel_gap=gap / max(abs(primal), 1e-300),
                T=T, unit=unit, alpha=alpha, t_lo=t_lo, t_hi=t_hi)


def kkt_violation(X1, y, tau, lam, beta, theta, zero_tol=0.0):
    """Largest violations of the optimality conditions (Prop. 1 with subgradients):
    theta_i = tau/n (r_i > 0), (tau-1)/n (r_i < 0), in between (r_i = 0); sum theta = 0;
    x_j^T theta = lam_j sign(beta_j) (beta_j != 0), |x_j^T theta| <= lam_j (beta_j = 0)."""
    n = X1.shape[0]
    r = y - X1 @ beta
    lo, hi = (tau - 1.0) / n, tau / n
    t_dual = np.where(r > zero_tol, np.abs(theta - hi),
                      np.where(r < -zero_tol, np.abs(theta - lo),
                               np.maximum(0.0, np.maximum(theta - hi, lo - theta))))
    v = X1.T @ theta
    nz = beta != 0
    stat = np.where(nz, np.abs(v - lam * np.sign(beta)), np.maximum(0.0, np.abs(v) - lam))
    return dict(dual_box=float(t_dual.max()), stationarity=float(stat.max()),
                intercept=float(abs(v[0])))


def coef_uniqueness(X1, tau, lam, theta, margin=1e-7, rank_tol=1e-9):
    """Is the minimiser unique?  theta must be an optimal dual point (the dual of the
    Lagrangian eq. main_lagrangian: box (tau-1)/n <= theta_i <= tau/n, |x_j^T theta|
    <= lam_j).  By complementary slackness (Prop. 1 with subgradients) every minimiser
    beta' has beta'_j = 0 wherever |x_j^T theta| < lam_j and a zero residual
    y_i = x_i^T beta' wherever theta_i lies strictly inside the box.  With J the
    columns that may be nonzero (the intercept, unpenalized columns and those with
    |x_j^T theta| >= lam_j (1 - margin)) and I the rows with theta_i at least
    margin (hi - lo) inside the box, the minimiser is unique when X1[I, J] has full
    column rank |J| (smallest singular value above rank_tol times the largest).  The
    margins make the test conservative against the rounding of theta."""
    X1 = np.asarray(X1, dtype=np.float64)
    theta = np.asarray(theta, dtype=np.float64)
    lam = np.asarray(lam, dtype=np.float64)
    n = X1.shape[0]
    lo, hi = (tau - 1.0) / n, tau / n
    v = X1.T @ theta
    J = np.nonzero((np.abs(v) >= lam * (1.0 - margin)) | (lam == 0))[0]
    J = np.union1d([0], J)
    w = margin * (hi - lo)
    I = np.nonzero((theta > lo + w) & (theta < hi - w))[0]
    if len(I) < len(J):
        return dict(unique=False, J=J, I=I, sigma_min=0.0)
    s = np.linalg.svd(X1[np.ix_(I, J)], compute_uv=False)
    smin = float(s[-1]) if len(s) else 0.0
    return dict(unique=bool(smin > rank_tol * max(1.0, float(s[0]))), J=J, I=I, sigma_min=smin)


# ----------------------------------------------------------------------------
# Screening (the Discussion's direction, Sec. 8): the sequential strong rule on the
# null-fit scores, made exact by the dual check on every column
# ----------------------------------------------------------------------------

def strong_rule(score, lam, lam_prev, w=None):
    """Columns kept by the sequential strong rule: |S_j| >= (2 lam - lam_prev) w_j, S_j
    the null-fit score x_j^T psi / n (feature columns only, 0-based)."""
    score = np.asarray(score, dtype=np.float64)
    w = np.ones_like(score) if w is None else np.asarray(w, dtype=np.float64)
    return np.nonzero(np.abs(score) >= (2.0 * lam - lam_prev) * w)[0]


def screened_solve(X1, y, tau, lam, A, solve, max_rounds=20):
    """Solve on the kept columns A (0-based feature indices), check every discarded
    column's dual value |x_j^T theta| <= lam_j at the restricted optimum (Prop. 1),
    add the violators and repeat.  `solve(X1r, y, tau, lamr)` returns (value, beta,
    theta) of the restricted problem.  Returns (value, beta, theta, rounds, added)."""
    p = X1.shape[1] - 1
    A = np.array(sorted(set(int(j) for j in A)), dtype=np.int64)
    added = 0
    for rounds in range(1, max_rounds + 1):
        cols = np.concatenate([[0], 1 + A])
        val, bA, th = solve(X1[:, cols], y, tau, lam[cols])
        v = np.abs(X1[:, 1:].T @ th)
        out = np.ones(p, dtype=bool)
        out[A] = False
        viol = np.nonzero(out & (v > lam[1:] * (1.0 + 1e-9)))[0]
        if len(viol) == 0:
            beta = np.zeros(p + 1)
            beta[cols] = bA
            return val, beta, th, rounds, added
        added += len(viol)
        A = np.union1d(A, viol)
    raise RuntimeError("screened_solve: violators remain after max_rounds")


# ----------------------------------------------------------------------------
# Standardisation (Sec. 7: standardised design, coefficients back-transformed)
# ----------------------------------------------------------------------------

def standardize(X):
    """x~_ij = (x_ij - m_j)/s_j with the population sd (divisor n).  Zero-variance
    columns get s_j = 0 and are returned as all-zero columns."""
    X = np.asarray(X, dtype=np.float64)
    n = X.shape[0]
    m = X.sum(axis=0) / n
    var = (X * X).sum(axis=0) / n - m * m
    s = np.sqrt(np.maximum(var, 0.0))
    Xt = np.zeros_like(X)
    ok = s > 0
    Xt[:, ok] = (X[:, ok] - m[ok]) / s[ok]
    return Xt, m, s


def with_intercept(X):
    X = np.asarray(X, dtype=np.float64)
    return np.hstack([np.ones((X.shape[0], 1)), X])


def back_transform(beta_std, m, s):
    """beta_j = beta~_j / s_j, beta_0 = beta~_0 - sum_j m_j beta~_j / s_j."""
    b = np.zeros_like(beta_std)
    ok = s > 0
    b[1:][ok] = beta_std[1:][ok] / s[ok]
    b[0] = beta_std[0] - float(np.dot(m[ok], b[1:][ok]))
    return b


# ----------------------------------------------------------------------------
# Folded-concave derivatives for the L-step LLA (eqs. scad, mcp; Algorithm 2)
# ----------------------------------------------------------------------------

def scad_deriv(b, lam, a=3.7):
    b = np.abs(np.asarray(b, dtype=np.float64))
    return np.where(b <= lam, lam, np.where(b < a * lam, (a * lam - b) / (a - 1.0), 0.0))


def mcp_deriv(b, lam, a=3.0):
    b = np.abs(np.asarray(b, dtype=np.float64))
    return np.where(b <= a * lam, lam - b / a, 0.0)


def lla(X1, y, tau, lam, blocks, mu, eta, L=1, penalty_kind="scad", a=None, start=None,
        **solve_kw):
    """Algorithm 2: a weighted-l1 FS-QRPPA solve at unit weights, then L reweighted
    solves with lam_j = p'_lam(|beta~_j|) (lam_0 stays 0), each warm-started from
    the previous (beta, z, theta)."""
    p1 = X1.shape[1]
    lam_vec = np.full(p1, float(lam))
    lam_vec[0] = 0.0
    res = fsqrppa(X1, y, tau, lam_vec, blocks, mu, eta, start=start, **solve_kw)
    for _ in range(L):
        d = scad_deriv if penalty_kind == "scad" else mcp_deriv
        kw = {} if a is None else {"a": a}
        w = d(res["beta"], lam, **kw)
        w[0] = 0.0
        res = fsqrppa(X1, y, tau, w, blocks, mu, eta,
                      start=(res["beta"], res["z"], res["theta"]), **solve_kw)
        res["lam"] = w
    return res
