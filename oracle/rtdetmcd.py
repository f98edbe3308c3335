"""Plain float64 RT-DetMCD oracle (test infrastructure; see package docstring).

Section and equation references are to arXiv 1910.05615.  Each function takes
the paper's steps in its order and notation; numpy/scipy routines (sort,
cumsum, Cholesky, triangular solve, eigh, chi-square quantiles) serve as single
steps.  Readings of points where the paper is silent or ambiguous are marked
"Reading:".
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional, Sequence

import numpy as np
from scipy import linalg as sla
from scipy import stats

# Paper constants.
CUTOFF_Q = 0.975          # chi-square quantile of the cutoff c_p (Sec. 2.1)
KAPPA_MAX = 1000.0        # condition threshold (Sec. 3.3 step 2, Sec. 3.4)
WRAP_B, WRAP_C, WRAP_Q1, WRAP_Q2 = 1.5, 4.0, 1.541, 0.862   # eq. (wrapping)
OMEGA = 4096              # default rows-per-dimension bound (eq. partitionsize)
MAX_CSTEPS = 100

# Start / chunk status codes (shared meaning with the library's public header,
# but defined here independently).
ST_CONVERGED = 0          # H_new == H_old reached
ST_NOTCONV = 1            # max_csteps reached
ST_ILLCOND = 2            # stopped because the next C-step was not taken (Sec. 3.4)
ST_DROP_REFINE = 3        # start dropped in refinement (Sec. 3.3 step 2)
ST_DROP_FIRST = 4         # start dropped: ill-conditioned before any C-step
ST_SINGULAR = 5           # start dropped: a subset covariance was singular
CHUNK_INVALID = 3         # both starts dropped: chunk excluded from aggregation


# --------------------------------------------------------------------------
# Distribution helpers (library routines serve as steps).
# --------------------------------------------------------------------------

def chi2_quantile(q: float, df: int) -> float:
    return float(stats.chi2.ppf(q, df))


def consistency_factor(alpha: float, p: int) -> float:
    """c(alpha) of the raw MCD scatter (Sec. 2.1, eq. mcdraw).

    The paper cites the factor without printing it.  Reading: the Gaussian
    consistency factor c(alpha) = alpha / F_{chi2_{p+2}}(chi2_{p,alpha}).
    Pinned against its closed forms at p = 1 and p = 2 in the tests.
    """
    if alpha >= 1.0:
        return 1.0
    return float(alpha / stats.chi2.cdf(stats.chi2.ppf(alpha, p), p + 2))


def n_blocks(n: int, p: int, omega: int = OMEGA) -> int:
    """Number of blocks q = max(floor(n / (p omega)), 1) (eq. partitionsize)."""
    return max(n // (p * omega), 1)


def subset_size(m: int, p: int, alpha: float) -> int:
    """h for a block of m rows.

    Reading: h = floor(alpha m) clamped into the range the MCD allows,
    [(m+p+1)/2] <= h < m (Sec. 2.1).
    """
    h = int(math.floor(alpha * m))
    lo = (m + p + 1) // 2
    return int(min(max(h, lo), m - 1))


# --------------------------------------------------------------------------
# Univariate MCD (Sec. 3.1).
# --------------------------------------------------------------------------

@dataclasses.dataclass
class UniMCD:
    mu_raw: float
    var_raw: float
    mu: float
    var: float
    start: int       # first sorted position of the optimal window
    n_kept: int


def unimcd(x: np.ndarray, cutoff_q: float = CUTOFF_Q) -> UniMCD:
    """Univariate reweighted MCD with coverage h~ = [n/2] + 1 (Sec. 3.1).

    Raw step: sort the data, slide a window of h~ consecutive order statistics
    and keep the window of smallest variance; its mean and standard deviation
    are the raw estimates.  Reading (the paper only names the estimator):
      * window variance uses the divisor h~ - 1; ties go to the lowest start;
      * the raw variance is multiplied by c(h~/n) for p = 1;
      * reweighting keeps (x - mu_raw)^2 <= chi2_{1,q} var_raw; the final
        location and variance are the mean and variance (divisor n_w - 1) of
        the kept values, the variance times c(q) for p = 1.
    The running window sums are prefix sums of the values centred at the
    middle order statistic; centring only conditions the sums.
    """
    x = np.asarray(x, dtype=np.float64).ravel()
    n = x.size
    hh = n // 2 + 1
    v = np.sort(x)
    c = v[n // 2]
    d = v - c
    P1 = np.concatenate(([0.0], np.cumsum(d)))
    P2 = np.concatenate(([0.0], np.cumsum(d * d)))
    j = np.arange(n - hh + 1)
    s1 = P1[j + hh] - P1[j]
    s2 = P2[j + hh] - P2[j]
    wvar = (s2 - s1 * s1 / hh) / (hh - 1)
    js = int(np.argmin(wvar))
    mu_raw = c + s1[js] / hh
    var_raw = float(wvar[js]) * consistency_factor(hh / n, 1)
    keep = (x - mu_raw) ** 2 <= chi2_quantile(cutoff_q, 1) * var_raw
    xk = x[keep]
    nk = int(xk.size)
    mu = float(np.mean(xk)) if nk > 0 else float("nan")
    var = float(np.var(xk, ddof=1)) * consistency_factor(cutoff_q, 1) if nk > 1 else 0.0
    return UniMCD(float(mu_raw), var_raw, mu, var, js, nk)


def medmad(x: np.ndarray):
    """Median and 1.4826 * MAD (the alternative standardisation of DetMCD, Sec. 2.2 step 1)."""
    x = np.asarray(x, dtype=np.float64).ravel()
    med = float(np.median(x))
    return med, 1.4826 * float(np.median(np.abs(x - med)))


# --------------------------------------------------------------------------
# Initial estimators (Sec. 3.2).
# --------------------------------------------------------------------------

def wrap(z: np.ndarray, b=WRAP_B, c=WRAP_C, q1=WRAP_Q1, q2=WRAP_Q2) -> np.ndarray:
    """Wrapping transform g (eq. wrapping)."""
    a = np.abs(z)
    mid = q1 * np.tanh(q2 * (c - a)) * np.sign(z)
    return np.where(a <= b, z, np.where(a <= c, mid, 0.0))


def init_wrap_cov(Z: np.ndarray) -> np.ndarray:
    """S~1: classical covariance (divisor m-1, centred at the column means) of g(Z)."""
    W = wrap(Z)
    return np.cov(W, rowvar=False, ddof=1).reshape(Z.shape[1], Z.shape[1])


def gsscm_cutoffs(r: np.ndarray):
    """Cutoffs A <= B of the linearly redescending weight (eq. LR).

    The paper defers the definition to a cited paper and only says A is about
    the median of the norms.  Reading: A = med(r); with s = r^(2/3)
    (Wilson-Hilferty), B = (med(s) + med|s - med(s)|)^(3/2), the back-transformed
    upper quartile of s.  Parity unpinned against the cited paper; pinned by
    the A, B -> infinity special case and by tests of the weight function.
    """
    A = float(np.median(r))
    s = r ** (2.0 / 3.0)
    ms = float(np.median(s))
    B = float((ms + float(np.median(np.abs(s - ms)))) ** 1.5)
    return A, B


def xi_lr(r: np.ndarray, A: float, B: float) -> np.ndarray:
    """Linearly redescending weight: 1 up to A, linear down to 0 at B.

    Reading for the degenerate case B <= A: the ramp is empty, weight 1 for
    r <= A and 0 beyond.
    """
    if B <= A:
        return np.where(r <= A, 1.0, 0.0)
    return np.where(r <= A, 1.0, np.where(r <= B, (B - r) / (B - A), 0.0))


def init_gsscm(Z: np.ndarray, A: Optional[float] = None,
               B: Optional[float] = None) -> np.ndarray:
    """S~2 = (1/m) sum_i xi^2(||z_i||) z_i z_i^T (eq. LR), z_i not centred."""
    m = Z.shape[0]
    r = np.sqrt(np.sum(Z * Z, axis=1))
    if A is None or B is None:
        A, B = gsscm_cutoffs(r)
    w = xi_lr(r, A, B) ** 2
    return (Z * w[:, None]).T @ Z / m


# --------------------------------------------------------------------------
# Refinement (Sec. 3.3).
# --------------------------------------------------------------------------

@dataclasses.dataclass
class Start:
    mu: Optional[np.ndarray]
    sigma: Optional[np.ndarray]
    ok: bool


def refine(S: np.ndarray, Z: np.ndarray, kappa_max: float = KAPPA_MAX) -> Start:
    """Refine an initial scatter S into a start (mu_k, Sigma_k) (Sec. 3.3 steps 1-4).

    Reading: Z~ = Sigma_k^{-1/2} Z is taken row-wise with the symmetric root
    V D~^{-1/2} V^T, the scores T = Z V use the uncentred Z, and a start whose
    score scale is zero is dropped like an ill-conditioned one.
    """
    p = S.shape[0]
    lam, V = np.linalg.eigh(0.5 * (S + S.T))
    lam = lam[::-1]
    V = V[:, ::-1]
    if not (lam[-1] > 0.0) or lam[0] / lam[-1] > kappa_max:
        return Start(None, None, False)
    T = Z @ V
    sig2 = np.array([unimcd(T[:, j]).var for j in range(p)])
    if not np.all(sig2 > 0.0):
        return Start(None, None, False)
    Sigma = (V * sig2) @ V.T
    Sinvh = (V / np.sqrt(sig2)) @ V.T
    Zt = Z @ Sinvh
    mut = np.array([unimcd(Zt[:, j]).mu for j in range(p)])
    mu = ((V * np.sqrt(sig2)) @ V.T) @ mut
    return Start(mu, 0.5 * (Sigma + Sigma.T), True)


# --------------------------------------------------------------------------
# C-steps (Sec. 2.1 eq. cstep1..cstep4b, Sec. 3.4, Sec. 3.5).
# --------------------------------------------------------------------------

def mahalanobis2(X: np.ndarray, mu: np.ndarray, L: np.ndarray) -> np.ndarray:
    """Squared distances ||L^{-1}(x_i - mu)||^2 by forward substitution (Sec. 3.4)."""
    Y = sla.solve_triangular(L, (X - mu).T, lower=True, check_finite=False)
    return np.sum(Y * Y, axis=0)


def mahalanobis2_inverse(X: np.ndarray, mu: np.ndarray, P: np.ndarray) -> np.ndarray:
    """Squared distances (x_i - mu)^T P (x_i - mu) with an explicit inverse P
    of the scatter: the distance computation that Sec. 3.4 replaces by the
    Cholesky form (the ID versus I rows of Table 1 in Sec. 5)."""
    R = X - mu
    return np.sum((R @ P) * R, axis=1)


def chol_or_none(S: np.ndarray):
    try:
        L = np.linalg.cholesky(S)
    except np.linalg.LinAlgError:
        return None
    if not np.all(np.isfinite(L)) or not np.all(np.diag(L) > 0):
        return None
    return L


def kappa1(S: np.ndarray, L: np.ndarray) -> float:
    """||S||_1 ||S^{-1}||_1 (eq. choleskymonitor).

    Reading: the exact 1-norm condition number, from S^{-1} = L^{-T} L^{-1};
    the paper's Higham estimator is a lower bound of it.
    """
    Li = sla.solve_triangular(L, np.eye(L.shape[0]), lower=True)
    Si = Li.T @ Li
    return float(np.max(np.sum(np.abs(S), axis=0)) * np.max(np.sum(np.abs(Si), axis=0)))


def select_h(d2: np.ndarray, h: int) -> np.ndarray:
    """Indices of the h smallest distances, ascending (Sec. 2.1 C-step steps 2-3).

    Reading: ties in the distance are broken by row index (stable sort).
    """
    order = np.argsort(d2, kind="stable")
    return np.sort(order[:h])


def h_gap(d2: np.ndarray, h: int) -> float:
    """Near-tie margin of a selection: d2_(h+1) - d2_(h), the gap between the
    largest distance kept and the smallest left out (0 for a tie across the
    threshold; the diagnostics of the h-subset decision).  NaN when every
    distance is kept."""
    if h >= len(d2):
        return math.nan
    s = np.sort(np.asarray(d2, dtype=np.float64))
    return float(s[h] - s[h - 1])


def subset_stats(X: np.ndarray, H: np.ndarray):
    """Mean and covariance (divisor h-1) of the rows in H (eq. cstep4a, cstep4b)."""
    Xh = X[H]
    mu = Xh.mean(axis=0)
    D = Xh - mu
    return mu, D.T @ D / (len(H) - 1)


def update_stats(X, H_old, H_new, mu_old, Lam_old):
    """Update-based C-step (Sec. 3.5): sequential mean / sscp update over swapped rows.

    Follows the paper's loop literally: for each row with delta_i != 0 the
    count, centre and sscp are updated in turn.  Rows are visited in index
    order, leaving rows first (any order gives the same result in exact
    arithmetic).  Returns (mu_new, Lambda_new) with Lambda = (h-1) Sigma.
    """
    old = np.zeros(X.shape[0], bool)
    old[H_old] = True
    new = np.zeros(X.shape[0], bool)
    new[H_new] = True
    delta = new.astype(int) - old.astype(int)
    h = len(H_old)
    mu = mu_old.copy()
    Lam = Lam_old.copy()
    order = list(np.nonzero(delta == -1)[0]) + list(np.nonzero(delta == 1)[0])
    for i in order:
        di = delta[i]
        h = h + di
        u = X[i] - mu
        mu = mu + (di / h) * u
        v = X[i] - mu
        Lam = Lam + di * np.outer(u, v)
    return mu, 0.5 * (Lam + Lam.T)


def smw_swap(x: np.ndarray, delta: int, h: int, mu: np.ndarray, Lam: np.ndarray,
             Lam_inv: np.ndarray, logdet_lam: float):
    """One case entering (delta = +1) or leaving (delta = -1) the subset, with
    the inverse and the determinant of the sscp matrix carried along (Sec. 3.5:
    the sequential update eq. propcstep1, muUpdate, propcstep2; the
    Sherman-Morrison-Woodbury identity eq. woodbury; the determinant identity
    eq. scaleddetUpdate).  Returns (h, mu, Lam, Lam_inv, logdet_lam), or None
    when Delta_i <= 0 (the updated sscp matrix would not be positive
    definite)."""
    h = h + delta
    u = x - mu
    mu = mu + (delta / h) * u
    v = x - mu
    a = Lam_inv @ u                       # Lam^{-1} u
    b = Lam_inv @ v                       # (v^T Lam^{-1})^T, Lam symmetric
    Delta = 1.0 + delta * float(v @ a)
    if not (Delta > 0.0):
        return None
    Lam_inv = Lam_inv - (delta / Delta) * np.outer(a, b)
    Lam = Lam + delta * np.outer(u, v)
    return h, mu, Lam, Lam_inv, logdet_lam + math.log(Delta)


@dataclasses.dataclass
class CStepResult:
    status: int
    H: Optional[np.ndarray]
    mu: Optional[np.ndarray]
    sigma: Optional[np.ndarray]      # subset covariance, divisor h-1, no c(alpha)
    logdet: float
    iters: int
    logdets: List[float]             # logdet of Sigma_old at each evaluated step
    smw_steps: int = 0               # steps taken by the single-swap update (mode "smw")
    hgap: float = math.nan           # h_gap of the last evaluated distances


def _with_gap(r: "CStepResult", gap: float) -> "CStepResult":
    r.hgap = gap
    return r


def csteps(X: np.ndarray, h: int, mu0: np.ndarray, sigma0: np.ndarray,
           max_steps: int = MAX_CSTEPS, kappa_max: float = KAPPA_MAX,
           kappa_scale: Optional[np.ndarray] = None, distance: str = "cholesky",
           mode: str = "full") -> CStepResult:
    """Iterate C-steps from (mu0, sigma0) until the h-subset repeats (Sec. 2.2 step 4).

    Each step: Cholesky of Sigma_old and its condition monitor (Sec. 3.4); if
    Sigma_old is not positive definite or kappa_1 >= kappa_max the step is not
    taken; otherwise distances, the h smallest, and the subset mean and
    covariance (full recomputation).
    Reading: a step refused on the first iteration drops the start; a refusal
    later keeps the last subset, except that a subset whose covariance is not
    positive definite drops the start (its determinant is zero and the
    distances are undefined).  Convergence is H_new == H_old; otherwise
    stop after max_steps steps (status ST_NOTCONV).

    ``kappa_scale``: the condition check is made in standardised units; when X
    is in raw units pass the column scales so that Sigma_old is divided by
    scale_j scale_k before the check.

    ``distance="inverse"``: distances by the explicit inverse of Sigma_old
    (mahalanobis2_inverse) instead of forward substitution (Sec. 3.4).

    ``mode="smw"``: a step whose new subset differs from the old one by one
    case out and one case in (sum |delta_i| = 2) updates the mean and sscp
    matrix case by case (leaving case first) and carries the inverse and the
    determinant of the sscp matrix by eq. (woodbury) and eq. (scaleddetUpdate)
    (smw_swap); the next step's distances then use that inverse and its
    condition check uses it too.  Other steps recompute in full.
    """
    p = len(mu0)
    mu, S = np.asarray(mu0, float), np.asarray(sigma0, float)
    H_prev = None
    logdets: List[float] = []
    gap = math.nan        # h_gap of the last evaluated distances
    smw = None            # (Sigma^{-1}, log det Sigma) after a single-swap update
    nsmw = 0
    for t in range(1, max_steps + 1):
        if smw is None:
            L = chol_or_none(S)
            if L is None:
                # Sigma_old is not positive definite: no step can be taken and the
                # subset (if any) has a singular covariance, so the start is dropped.
                return _with_gap(CStepResult(ST_DROP_FIRST if H_prev is None else ST_SINGULAR,
                                   None, None, None, math.nan, t - 1, logdets, nsmw), gap)
            Sk, Lk = S, L
            if kappa_scale is not None:
                Sk = S / np.outer(kappa_scale, kappa_scale)
                Lk = chol_or_none(Sk)
            kap = kappa1(Sk, Lk) if Lk is not None else math.inf
            ld = 2.0 * float(np.sum(np.log(np.diag(L))))
        else:
            Si, ld = smw
            Sk, Ski = S, Si
            if kappa_scale is not None:
                Sk = S / np.outer(kappa_scale, kappa_scale)
                Ski = Si * np.outer(kappa_scale, kappa_scale)
            kap = float(np.max(np.sum(np.abs(Sk), axis=0)) *
                        np.max(np.sum(np.abs(Ski), axis=0)))
        if not (kap < kappa_max):
            if H_prev is None:
                return _with_gap(CStepResult(ST_DROP_FIRST, None, None, None, math.nan, t - 1, logdets,
                                   nsmw), gap)
            return _with_gap(CStepResult(ST_ILLCOND, H_prev, mu, S, ld, t - 1, logdets, nsmw), gap)
        logdets.append(ld)
        if smw is not None:
            d2 = mahalanobis2_inverse(X, mu, smw[0])
        elif distance == "inverse":
            d2 = mahalanobis2_inverse(X, mu, np.linalg.inv(S))
        else:
            d2 = mahalanobis2(X, mu, L)
        H = select_h(d2, h)
        gap = h_gap(d2, h)
        if H_prev is not None and np.array_equal(H, H_prev):
            return _with_gap(CStepResult(ST_CONVERGED, H, mu, S, ld, t, logdets, nsmw), gap)
        smw_next = None
        if mode == "smw" and H_prev is not None:
            out_ = np.setdiff1d(H_prev, H)
            in_ = np.setdiff1d(H, H_prev)
            if len(out_) == 1 and len(in_) == 1:
                Lam = (h - 1) * S
                if smw is not None:
                    Lam_inv = smw[0] / (h - 1)
                else:
                    Li = sla.solve_triangular(L, np.eye(p), lower=True)
                    Lam_inv = (Li.T @ Li) / (h - 1)
                st = (h, mu, Lam, Lam_inv, ld + p * math.log(h - 1))
                for i, dlt in ((int(out_[0]), -1), (int(in_[0]), +1)):
                    st = smw_swap(X[i], dlt, st[0], st[1], st[2], st[3], st[4])
                    if st is None:
                        break
                if st is None:
                    return _with_gap(CStepResult(ST_SINGULAR, None, None, None, math.nan, t, logdets,
                                       nsmw), gap)
                _, mu, Lam, Lam_inv, ldl = st
                S = 0.5 * (Lam + Lam.T) / (h - 1)
                smw_next = ((h - 1) * Lam_inv, ldl - p * math.log(h - 1))
                nsmw += 1
        if smw_next is None:
            mu, S = subset_stats(X, H)
        smw = smw_next
        H_prev = H
    if smw is not None:
        return _with_gap(CStepResult(ST_NOTCONV, H_prev, mu, S, smw[1], max_steps, logdets, nsmw), gap)
    L = chol_or_none(S)
    if L is None:
        return _with_gap(CStepResult(ST_SINGULAR, None, None, None, math.nan, max_steps, logdets, nsmw), gap)
    return _with_gap(CStepResult(ST_NOTCONV, H_prev, mu, S, 2.0 * float(np.sum(np.log(np.diag(L)))),
                       max_steps, logdets, nsmw), gap)


# --------------------------------------------------------------------------
# Aggregation (Sec. 4 steps 5-7, 9).
# --------------------------------------------------------------------------

def kl_deviation(a, A, b, B) -> float:
    """KL[(a, A), (b, B)] (eq. KL); needs det(A B^{-1}) > 0."""
    p = len(a)
    Bi = np.linalg.inv(B)
    sign, ld = np.linalg.slogdet(A @ Bi)
    d = a - b
    return float(np.trace(A @ Bi) - p - (ld if sign > 0 else math.nan) + d @ Bi @ d)


def kl_rank_key(mu_med, S_med, mu_l, S_l) -> float:
    """KL'_l = tr(S_med S_l^-1) + log det S_l + (mu_med-mu_l)' S_l^-1 (mu_med-mu_l).

    Reading: S_med need not be positive definite (Sec. 4 step 5), so the
    l-independent term -p - log det S_med of eq. (KL) is dropped.  The order
    over l is the KL order whenever KL is defined.
    """
    Si = np.linalg.inv(S_l)
    _, ld = np.linalg.slogdet(S_l)
    d = mu_med - mu_l
    return float(np.trace(S_med @ Si) + ld + d @ Si @ d)


def pool_printed(mus: Sequence[np.ndarray], sigmas: Sequence[np.ndarray], m: int):
    """Single-pass pooling of Sec. 4 step 7 with the printed counts (each block m)."""
    mu = np.array(mus[0], float)
    Lam = (m - 1) * np.array(sigmas[0], float)
    n = m
    for mu_l, S_l in zip(mus[1:], sigmas[1:]):
        dmu = mu_l - mu
        Lam = Lam + (m - 1) * S_l + np.outer(dmu, dmu) * (n * m / (n + m))
        mu = (n * mu + m * mu_l) / (n + m)
        n = n + m
    return mu, Lam / (n - 1)


def pool_counts(mus, lams, counts):
    """Same pooling with per-block counts and sscp matrices (Sec. 4 step 9)."""
    mu = np.array(mus[0], float)
    Lam = np.array(lams[0], float)
    n = counts[0]
    for mu_l, L_l, m_l in zip(mus[1:], lams[1:], counts[1:]):
        if m_l == 0:
            continue
        dmu = mu_l - mu
        Lam = Lam + L_l + np.outer(dmu, dmu) * (n * m_l / (n + m_l))
        mu = (n * mu + m_l * mu_l) / (n + m_l)
        n = n + m_l
    return mu, Lam, n


def aggregate(mus, sigmas, m: int, pool: str = "printed", subsets=None, Zfit=None,
              alpha_factor: float = 1.0):
    """Entrywise median, KL ranking, keep ceil(q/2), pool (Sec. 4 steps 5-7).

    Reading of the median of an even count: the mean of the two middle values.
    Ties in KL' go to the lower block index.  Pooling order is the KL order.
    ``pool='union'`` pools the union of the kept h-subsets (the text of step 7)
    and multiplies by c(alpha) (``alpha_factor``).
    Returns (mu_raw, sigma_raw, kept block positions in KL order, KL' values).
    """
    q = len(mus)
    M = np.stack(mus)
    S = np.stack(sigmas)
    mu_med = np.median(M, axis=0)
    S_med = np.median(S, axis=0)
    keys = np.array([kl_rank_key(mu_med, S_med, M[l], S[l]) for l in range(q)])
    order = np.argsort(keys, kind="stable")
    keep = order[: (q + 1) // 2]
    if pool == "printed":
        mu, Sig = pool_printed([M[l] for l in keep], [S[l] for l in keep], m)
    elif pool == "union":
        U = np.concatenate([subsets[l] for l in keep])
        mu, Sig = subset_stats(Zfit, U)
        Sig = Sig * alpha_factor
    else:
        raise ValueError(pool)
    return mu, 0.5 * (Sig + Sig.T), keep, keys


# --------------------------------------------------------------------------
# Full fit (Sec. 4 steps 1-10; q = 1 is the serial version IDC).
# --------------------------------------------------------------------------

@dataclasses.dataclass
class Fit:
    mu: np.ndarray
    sigma: np.ndarray
    mu_raw: np.ndarray
    sigma_raw: np.ndarray
    logdet_raw: float
    logdet_rew: float
    dist: np.ndarray
    outlier: np.ndarray
    hsubset: np.ndarray          # q x h, ascending row indices of the dataset
    chunk_status: np.ndarray
    chunk_start: np.ndarray
    chunk_iters: np.ndarray
    loc: np.ndarray
    scale: np.ndarray
    q: int
    m: int
    h: int
    n_w: int
    rew_mask: np.ndarray         # n, 1 for the rows kept by the reweighting (Sec. 4 step 8)
    diag: dict


START_WARM = 2             # chunk_start of a block fitted from a warm start


def fit(X: np.ndarray, alpha: float = 0.75, h_sub: int = 0, n_chunks: int = 0,
        standardize: str = "unimcd", pool: str = "printed",
        rew_consistency: bool = False, max_csteps: int = MAX_CSTEPS,
        kappa_max: float = KAPPA_MAX, cutoff_q: float = CUTOFF_Q,
        omega: int = OMEGA, perm: Optional[np.ndarray] = None,
        distance: str = "cholesky", cstep_mode: str = "full",
        warm: Optional[tuple] = None) -> Fit:
    """RT-DetMCD fit of one dataset X (n x p), every step in float64.

    Reading of the partition (Sec. 4): contiguous blocks of m = floor(n/q)
    rows in the given order (``perm`` re-orders the rows first); the n - q m
    remainder rows are not fitted but are scored and flagged in step 10.

    ``distance="inverse"`` computes every distance of the fit (C-steps,
    reweighting, final) with the explicit inverse of the scatter instead of
    the Cholesky form of Sec. 3.4 (Table 1: version I against ID);
    ``cstep_mode="smw"`` takes single-swap C-steps by the inverse and
    determinant updates of Sec. 3.5 (csteps).

    ``warm=(mu, sigma)`` (units of X): the warm start of the last paragraph of
    Sec. 4.  Reading: a previous fit's reweighted estimate is the one start of
    every block's C-steps (step 3); the initial estimators and their
    refinement (steps 1-2) are skipped, the standardisation of this data and
    steps 4-10 are as usual (chunk_start = START_WARM).
    """
    X = np.asarray(X, dtype=np.float64)
    n, p = X.shape
    if n < 2 * p + 1 or p < 1:
        raise ValueError("need n > 2p")
    q = n_chunks if n_chunks > 0 else n_blocks(n, p, omega)
    m = n // q
    h = h_sub if h_sub > 0 else subset_size(m, p, alpha)
    if not (p < h < m):
        raise ValueError("need p < h < m")
    order = np.arange(n) if perm is None else np.asarray(perm)

    # Sec. 3.1 / Sec. 4 eq. (standardization): one global location and scale.
    loc = np.empty(p)
    scale = np.empty(p)
    for j in range(p):
        if standardize == "unimcd":
            u = unimcd(X[:, j], cutoff_q)
            loc[j], scale[j] = u.mu, math.sqrt(max(u.var, 0.0))
        else:
            loc[j], scale[j] = medmad(X[:, j])
    if not np.all(scale > 0):
        raise ValueError("a column has zero robust scale")
    Z = (X - loc) / scale

    c_alpha = consistency_factor(h / m, p)
    chi2 = chi2_quantile(cutoff_q, p)
    fits_mu, fits_sig, fits_ld, valid = [], [], [], []
    chunk_status = np.zeros(q, np.int32)
    chunk_start = np.full(q, -1, np.int32)
    chunk_iters = np.zeros(q, np.int32)
    hsub = np.full((q, h), -1, np.int64)
    starts_diag = []
    # O12 diagnostics of the chosen start of each block: log det of Sigma_old
    # at each evaluated C-step, and the selection gap of its last distances
    block_logdets = np.full((q, max_csteps), np.nan)
    block_hgap = np.full(q, np.nan)
    if warm is not None:
        mu_w = (np.asarray(warm[0], float) - loc) / scale
        S_w = np.asarray(warm[1], float) / np.outer(scale, scale)
        S_w = 0.5 * (S_w + S_w.T)
    for l in range(q):
        rows = order[l * m:(l + 1) * m]
        Zl = Z[rows]
        res = []
        if warm is not None:                                # step 3 from the warm start
            res.append(csteps(Zl, h, mu_w, S_w, max_csteps, kappa_max,
                              distance=distance, mode=cstep_mode))
        else:
            for S0 in (init_wrap_cov(Zl), init_gsscm(Zl)):  # Sec. 4 step 1
                st = refine(S0, Zl, kappa_max)              # step 2
                if not st.ok:
                    res.append(CStepResult(ST_DROP_REFINE, None, None, None, math.nan, 0, []))
                    continue
                res.append(csteps(Zl, h, st.mu, st.sigma, max_csteps, kappa_max,
                                  distance=distance, mode=cstep_mode))   # step 3
        starts_diag.append(res)
        ok = [k for k in range(len(res)) if res[k].H is not None]
        if not ok:
            chunk_status[l] = CHUNK_INVALID
            continue
        # step 4: smaller determinant; ties to the first start
        best = ok[0]
        for k in ok[1:]:
            if res[k].logdet < res[best].logdet:
                best = k
        r = res[best]
        chunk_status[l] = r.status
        chunk_start[l] = START_WARM if warm is not None else best
        chunk_iters[l] = r.iters
        block_logdets[l, :len(r.logdets)] = r.logdets
        block_hgap[l] = r.hgap
        hsub[l] = rows[r.H]
        fits_mu.append(r.mu)
        fits_sig.append(c_alpha * r.sigma)
        fits_ld.append(r.logdet)
        valid.append(l)
    if not valid:
        raise ValueError("no valid block")

    Zfit = Z[order[: q * m]]
    mu_raw, sig_raw, keep, keys = aggregate(
        fits_mu, fits_sig, m, pool, subsets=[hsub[l] for l in valid], Zfit=Z,
        alpha_factor=c_alpha)

    # Steps 8-9: reweighting over the fitted rows.
    def dist2(Zr, mu_, S_):
        if distance == "inverse":
            return mahalanobis2_inverse(Zr, mu_, np.linalg.inv(S_))
        return mahalanobis2(Zr, mu_, np.linalg.cholesky(S_))

    d2 = dist2(Zfit, mu_raw, sig_raw)
    W = d2 <= chi2
    n_w = int(W.sum())
    mu_rew, sig_rew = subset_stats(Zfit, np.nonzero(W)[0])
    if rew_consistency:
        sig_rew = sig_rew * consistency_factor(cutoff_q, p)
    # Step 10: final distances and flags for every row.
    d2all = dist2(Z, mu_rew, sig_rew)
    rew_mask = np.zeros(n, np.uint8)
    rew_mask[order[: q * m][W]] = 1

    D = np.diag(scale)
    logs = 2.0 * float(np.sum(np.log(scale)))
    return Fit(
        mu=loc + scale * mu_rew, sigma=D @ sig_rew @ D,
        mu_raw=loc + scale * mu_raw, sigma_raw=D @ sig_raw @ D,
        logdet_raw=float(np.linalg.slogdet(sig_raw)[1]) + logs,
        logdet_rew=float(np.linalg.slogdet(sig_rew)[1]) + logs,
        dist=np.sqrt(d2all), outlier=(d2all > chi2).astype(np.uint8),
        hsubset=hsub, chunk_status=chunk_status, chunk_start=chunk_start,
        chunk_iters=chunk_iters, loc=loc, scale=scale, q=q, m=m, h=h, n_w=n_w,
        rew_mask=rew_mask,
        diag=dict(starts=starts_diag, kl_keys=keys, keep=np.asarray(valid)[keep],
                  d2_final=d2all, d2_reweight=d2, valid=np.asarray(valid),
                  mu_raw_z=mu_raw, sigma_raw_z=sig_raw, mu_rew_z=mu_rew,
                  sigma_rew_z=sig_rew, c_alpha=c_alpha, chi2=chi2,
                  block_logdets=block_logdets, block_hgap=block_hgap,
                  cmargin=float(np.min(np.abs(d2all - chi2)))))
