"""Exact laws that pin the CPU oracle (test helpers; numpy/scipy only).

Nothing here calls the oracle or the GPU library.  The model propensities are
written out again, directly from the paper's tables and the benchmark model
definitions, so that a mistake in the oracle's factored propensity code shows
up as a disagreement.

* birth-death chains (Schloegl, Sec. IV A, is one): closed-form stationary law
  pi(x) ~ prod_{k<=x} lam+(k-1)/lam-(k), the asymptotic variance (IAF) of
  int f, and CME sensitivities by differentiating the closed form;
* general CTMCs on a truncated lattice: stationary law from pi Q = 0 (eq. Q);
* the embedded (jump) chain restricted to a metastable set W: its
  quasi-stationary distribution nu (left Perron vector, Sec. II A) and the
  law of X_n conditioned on N > n, which Fleming-Viot dephasing samples.
"""
from __future__ import annotations

import math

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla


# ----------------------------------------------------------------------------
# Model propensities, written from the model definitions
# ----------------------------------------------------------------------------

def schlogl_classic_rates(x, c=(3e-7, 1e-4, 1e-3, 3.5), A=1e5, B=2e5):
    """(lam1..lam4) of the classic Schloegl network at integer states x (array)."""
    x = np.asarray(x, dtype=np.float64)
    c1, c2, c3, c4 = c
    l1 = c1 / 2.0 * A * x * (x - 1)
    l2 = c2 / 6.0 * x * (x - 1) * (x - 2)
    l3 = c3 * B * np.ones_like(x)
    l4 = c4 * x
    return np.clip(np.stack([l1, l2, l3, l4]), 0.0, None)


def schlogl_paper_rates(x, c=(3.0, 0.6, 0.25, 2.95), V=25.0, a=1.0, b=2.0):
    """Table I: c1 a x(x-1)/V, c2 x(x-1)(x-2)/V^2, c3 b V, c4 x."""
    x = np.asarray(x, dtype=np.float64)
    c1, c2, c3, c4 = c
    l1 = c1 * a * x * (x - 1) / V
    l2 = c2 * x * (x - 1) * (x - 2) / V ** 2
    l3 = c3 * b * V * np.ones_like(x)
    l4 = c4 * x
    return np.clip(np.stack([l1, l2, l3, l4]), 0.0, None)


def toggle_rates(u, v, omega, c=(3.0, 3.0, 2.0, 2.0)):
    """Gardner toggle: Omega a1/(1+(v/Omega)^beta), u, Omega a2/(1+(u/Omega)^gamma), v."""
    u = np.asarray(u, dtype=np.float64)
    v = np.asarray(v, dtype=np.float64)
    a1, a2, be, ga = c
    l1 = omega * a1 / (1.0 + (v / omega) ** be)
    l2 = u
    l3 = omega * a2 / (1.0 + (u / omega) ** ga)
    l4 = v
    return np.stack([l1, l2, l3, l4])


TOGGLE_STOICH = ((1, 0), (-1, 0), (0, 1), (0, -1))


# ----------------------------------------------------------------------------
# Birth-death chains
# ----------------------------------------------------------------------------

def birth_death_pi(lp: np.ndarray, lm: np.ndarray) -> np.ndarray:
    """Stationary law on {0..N} of a birth-death chain with birth rates lp[x]
    and death rates lm[x] (lm[0] ignored): pi(x) ~ prod_{k=1}^x lp[k-1]/lm[k]."""
    N = len(lp) - 1
    logw = np.zeros(N + 1)
    for x in range(1, N + 1):
        logw[x] = logw[x - 1] + math.log(lp[x - 1]) - math.log(lm[x])
    logw -= logw.max()
    w = np.exp(logw)
    return w / w.sum()


def schlogl_classic_pi(N=1000, c=(3e-7, 1e-4, 1e-3, 3.5)):
    x = np.arange(N + 1)
    l = schlogl_classic_rates(x, c)
    return birth_death_pi(l[0] + l[2], l[1] + l[3])


def schlogl_paper_pi(N=400, c=(3.0, 0.6, 0.25, 2.95), V=25.0):
    x = np.arange(N + 1)
    l = schlogl_paper_rates(x, c, V)
    return birth_death_pi(l[0] + l[2], l[1] + l[3])


def birth_death_iaf(pi: np.ndarray, lp: np.ndarray, f: np.ndarray) -> float:
    """Asymptotic variance lim Var(int_0^T f)/T of a birth-death chain:
    2 sum_x G(x)^2 / (pi(x) lp(x)), G(x) = sum_{y<=x} pi(y)(f(y) - pi f).
    G is summed from the nearer tail (G(x) = -sum_{y>x}...) to avoid cancellation."""
    pf = float(np.dot(pi, f))
    d = pi * (f - pf)
    G_lo = np.cumsum(d)
    G_hi = -(np.cumsum(d[::-1])[::-1] - d)
    G = np.where(np.arange(len(pi)) < len(pi) // 2, G_lo, G_hi)
    m = pi[:-1] * lp[:-1] > 0
    return float(2.0 * np.sum(G[:-1][m] ** 2 / (pi[:-1][m] * lp[:-1][m])))


def schlogl_paper_mean(c, V=25.0, N=400):
    pi = schlogl_paper_pi(N, c, V)
    return float(np.dot(pi, np.arange(N + 1)))


def schlogl_paper_sensitivity(k: int, V=25.0, h=1e-6, N=400):
    """d E_pi[x] / d c_k by a central difference of the closed-form law."""
    c = np.array((3.0, 0.6, 0.25, 2.95))
    cp, cm = c.copy(), c.copy()
    cp[k] *= 1 + h
    cm[k] *= 1 - h
    return (schlogl_paper_mean(cp, V, N) - schlogl_paper_mean(cm, V, N)) / (2 * h * c[k])


def schlogl_rre_roots(c=(3.0, 0.6, 0.25, 2.95), a=1.0, b=2.0):
    """Roots of the RRE right-hand side c1 a x^2 - c2 x^3 + c3 b - c4 x (Sec. IV A)."""
    c1, c2, c3, c4 = c
    r = np.roots([-c2, c1 * a, -c4, c3 * b])
    return np.sort(r[np.abs(r.imag) < 1e-9].real)


# ----------------------------------------------------------------------------
# Truncated lattices
# ----------------------------------------------------------------------------

class Lattice:
    """States of a truncated 2-D lattice [0,N]^2 with reflecting truncation
    (transitions leaving the box are dropped)."""

    def __init__(self, N: int):
        self.N = N
        self.n = (N + 1) ** 2

    def idx(self, u, v):
        return u * (self.N + 1) + v

    def states(self):
        g = np.arange(self.N + 1)
        U, V = np.meshgrid(g, g, indexing="ij")
        return U.ravel(), V.ravel()


def toggle_generator(omega, N, c=(3.0, 3.0, 2.0, 2.0)):
    L = Lattice(N)
    U, V = L.states()
    lam = toggle_rates(U, V, omega, c)
    rows, cols, vals = [], [], []
    for j, (du, dv) in enumerate(TOGGLE_STOICH):
        u2, v2 = U + du, V + dv
        ok = (u2 >= 0) & (u2 <= N) & (v2 >= 0) & (v2 <= N) & (lam[j] > 0)
        src = L.idx(U[ok], V[ok])
        dst = L.idx(u2[ok], v2[ok])
        rows.append(src)
        cols.append(dst)
        vals.append(lam[j][ok])
    rows = np.concatenate(rows)
    cols = np.concatenate(cols)
    vals = np.concatenate(vals)
    Q = sp.coo_matrix((vals, (rows, cols)), shape=(L.n, L.n)).tocsr()
    out = np.asarray(Q.sum(axis=1)).ravel()
    Q = Q - sp.diags(out)
    return L, Q.tocsr()


def stationary_from_generator(Q: sp.csr_matrix) -> np.ndarray:
    """Solve pi Q = 0, sum pi = 1 by replacing one balance equation."""
    n = Q.shape[0]
    A = Q.T.tolil()
    A[0, :] = np.ones(n)
    b = np.zeros(n)
    b[0] = 1.0
    pi = spla.spsolve(A.tocsc(), b)
    pi = np.clip(pi, 0.0, None)
    return pi / pi.sum()


def toggle_pi(omega, N, c=(3.0, 3.0, 2.0, 2.0)):
    L, Q = toggle_generator(omega, N, c)
    return L, stationary_from_generator(Q).reshape(N + 1, N + 1)


def toggle_fim_exact(omega, N, c=(3.0, 3.0, 2.0, 2.0)):
    """E_pi[sum_j lam_j grad log lam_j grad log lam_j^T] w.r.t. (a1, a2, beta, gamma)."""
    L, pi = toggle_pi(omega, N, c)
    U, V = L.states()
    F = toggle_fim_integrand(U, V, omega, c)
    return np.einsum("s,sab->ab", pi.ravel(), F)


def toggle_fim_integrand(U, V, omega, c=(3.0, 3.0, 2.0, 2.0)):
    """Per-state FIM integrand of the toggle, (S, 4, 4)."""
    a1, a2, be, ga = c
    U = np.asarray(U, dtype=np.float64)
    V = np.asarray(V, dtype=np.float64)
    lam = toggle_rates(U, V, omega, c)
    yv, yu = V / omega, U / omega
    qv, qu = yv ** be, yu ** ga
    with np.errstate(divide="ignore", invalid="ignore"):
        dbeta = np.where(yv > 0, -qv * np.log(np.where(yv > 0, yv, 1.0)) / (1 + qv), 0.0)
        dgam = np.where(yu > 0, -qu * np.log(np.where(yu > 0, yu, 1.0)) / (1 + qu), 0.0)
    g1 = np.stack([1 / a1 * np.ones_like(U), 0 * U, dbeta, 0 * U], axis=1)
    g3 = np.stack([0 * U, 1 / a2 * np.ones_like(U), 0 * U, dgam], axis=1)
    return (lam[0][:, None, None] * g1[:, :, None] * g1[:, None, :]
            + lam[2][:, None, None] * g3[:, :, None] * g3[:, None, :])


# ----------------------------------------------------------------------------
# Embedded chain on a metastable set
# ----------------------------------------------------------------------------

def embedded_substochastic(L: Lattice, Q: sp.csr_matrix, in_W: np.ndarray):
    """Jump-chain transition matrix restricted to W (rows of W, columns of W)."""
    out = -Q.diagonal()
    P = sp.diags(1.0 / np.where(out > 0, out, 1.0)) @ (Q + sp.diags(out))
    Wi = np.flatnonzero(in_W)
    return P.tocsr()[Wi][:, Wi].tocsr(), Wi


def qsd_embedded(PW: sp.csr_matrix):
    """Left Perron vector nu (nu P_W = rho nu) and rho of the embedded chain on W."""
    vals, vecs = spla.eigs(PW.T.tocsc(), k=4, which="LR")
    i = int(np.argmax(vals.real))
    rho = float(vals[i].real)
    nu = np.abs(vecs[:, i].real)
    return nu / nu.sum(), rho


def conditioned_law(PW: sp.csr_matrix, start: int, n: int) -> np.ndarray:
    """Law of X_n given no exit from W by step n, starting at W-index start."""
    mu = np.zeros(PW.shape[0])
    mu[start] = 1.0
    PT = PW.T.tocsr()
    for _ in range(n):
        mu = PT @ mu
        mu /= mu.sum()
    return mu


def tv(p: np.ndarray, q: np.ndarray) -> float:
    return 0.5 * float(np.abs(np.asarray(p, dtype=float) - np.asarray(q, dtype=float)).sum())


# ----------------------------------------------------------------------------
# Genetic switch (Sec. IV B): xi in {0,1} active DNA, x1 mRNA, x2 protein
# ----------------------------------------------------------------------------

GS_STOICH = ((0, 1, 0), (0, -1, 0), (0, 0, 1), (0, 0, -1), (1, 0, 0), (-1, 0, 0))


def genetic_switch_rates(xi, x1, x2, c):
    """Table IV propensities and the switching rates F (inactive -> active)
    and G (active -> inactive) of Eq. (10); c = (a, b, gamma, k0min, k0max,
    k1min, k1max, D).  Channel order: transcription, mRNA decay, translation,
    protein decay, activation, deactivation."""
    a, b, g, k0n, k0x, k1n, k1x, D = c
    xi = np.asarray(xi, dtype=np.float64)
    x1 = np.asarray(x1, dtype=np.float64)
    x2 = np.asarray(x2, dtype=np.float64)
    h = x2 ** 2 / (x2 ** 2 + D ** 2)
    F = k0n + (k0x - k0n) * h
    G = k1x - (k1x - k1n) * h
    return np.stack([a * xi, g * x1, g * b * x1, x2, F * (1 - xi), G * xi])


def genetic_switch_grad(xi, x1, x2, c):
    """d lam_j / d c_k, shape (8, 6, S), differentiated by hand from
    genetic_switch_rates."""
    a, b, g, k0n, k0x, k1n, k1x, D = c
    xi = np.asarray(xi, dtype=np.float64)
    x1 = np.asarray(x1, dtype=np.float64)
    x2 = np.asarray(x2, dtype=np.float64)
    h = x2 ** 2 / (x2 ** 2 + D ** 2)
    dh = -2.0 * x2 ** 2 * D / (x2 ** 2 + D ** 2) ** 2
    d = np.zeros((8, 6, xi.size))
    d[0, 0] = xi
    d[1, 2] = g * x1
    d[2, 1] = x1
    d[2, 2] = b * x1
    d[3, 4] = (1 - h) * (1 - xi)
    d[4, 4] = h * (1 - xi)
    d[7, 4] = (k0x - k0n) * dh * (1 - xi)
    d[5, 5] = h * xi
    d[6, 5] = (1 - h) * xi
    d[7, 5] = -(k1x - k1n) * dh * xi
    return d


class SwitchLattice:
    """States (xi, x1, x2) in {0,1} x [0,N1] x [0,N2], numbered with x2
    slowest so that the generator is banded (bandwidth 2 (N1+1)); transitions
    leaving the box are dropped."""

    def __init__(self, N1: int, N2: int):
        self.N1, self.N2 = N1, N2
        self.n = 2 * (N1 + 1) * (N2 + 1)

    def idx(self, xi, x1, x2):
        return (np.asarray(x2) * 2 + xi) * (self.N1 + 1) + x1

    def states(self):
        x2, xi, x1 = np.meshgrid(np.arange(self.N2 + 1), np.arange(2), np.arange(self.N1 + 1),
                                 indexing="ij")
        return xi.ravel(), x1.ravel(), x2.ravel()


def genetic_switch_generator(c, N1: int, N2: int):
    L = SwitchLattice(N1, N2)
    xi, x1, x2 = L.states()
    lam = genetic_switch_rates(xi, x1, x2, c)
    rows, cols, vals = [], [], []
    for j, (ds, d1, d2) in enumerate(GS_STOICH):
        s2, m2, p2 = xi + ds, x1 + d1, x2 + d2
        ok = (s2 >= 0) & (s2 <= 1) & (m2 >= 0) & (m2 <= N1) & (p2 >= 0) & (p2 <= N2) & (lam[j] > 0)
        rows.append(L.idx(xi[ok], x1[ok], x2[ok]))
        cols.append(L.idx(s2[ok], m2[ok], p2[ok]))
        vals.append(lam[j][ok])
    Q = sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                      shape=(L.n, L.n)).tocsr()
    Q = Q - sp.diags(np.asarray(Q.sum(axis=1)).ravel())
    return L, Q.tocsr()


def _pin_solve(M: sp.csr_matrix, rhs: np.ndarray, k: int) -> np.ndarray:
    """Solve M z = rhs with equation k replaced by z_k = rhs_k (keeps the
    band; natural ordering)."""
    A = M.tolil()
    A[k, :] = 0.0
    A[k, k] = 1.0
    return spla.spsolve(A.tocsc(), rhs, permc_spec="NATURAL")


def genetic_switch_pi(c, N1: int, N2: int):
    """Stationary law on the truncated lattice: pi Q = 0 with pi pinned at a
    state of positive mass (inactive DNA, no mRNA, protein near the low
    equilibrium), then normalised."""
    L, Q = genetic_switch_generator(c, N1, N2)
    k = int(L.idx(0, 0, min(N2, max(1, int(round(25.0 * c[7] / 1000.0))))))
    e = np.zeros(L.n)
    e[k] = 1.0
    pi = np.clip(_pin_solve(Q.T.tocsr(), e, k), 0.0, None)
    return L, Q, pi / pi.sum()


def ctmc_iaf(L, Q: sp.csr_matrix, pi: np.ndarray, f: np.ndarray) -> float:
    """Asymptotic variance lim Var(int_0^T f)/T = 2 pi((f - pi f) g), where
    Q g = -(f - pi f) (Poisson equation; g is defined up to a constant,
    which drops out since pi(f - pi f) = 0)."""
    d = np.asarray(f, dtype=np.float64) - float(pi @ f)
    k = int(np.argmax(pi))
    rhs = -d.copy()
    rhs[k] = 0.0
    g = _pin_solve(Q, rhs, k)
    return float(2.0 * pi @ (d * g))


def genetic_switch_fim_integrand(xi, x1, x2, c):
    """Per-state path-space FIM integrand sum_j (d lam_j)(d lam_j)^T / lam_j, (S, 8, 8)."""
    lam = genetic_switch_rates(xi, x1, x2, c)
    d = genetic_switch_grad(xi, x1, x2, c)
    out = np.zeros((lam.shape[1], 8, 8))
    for j in range(6):
        l = lam[j]
        w = np.where(l > 0, 1.0 / np.where(l > 0, l, 1.0), 0.0)
        out += np.einsum("as,bs,s->sab", d[:, j], d[:, j], w)
    return out


# --------------------------------------------------------------------------
# Exact laws of the time-mode stopping rules of Alg. 1 (decorrelation and
# dephasing), on chains whose total rate a0 is the same in every state, so
# that the holding times are iid Exp(a0) and independent of the jump chain.
# --------------------------------------------------------------------------

def dephase_rounds_cdf(a0: float, t_p: float, R: int, n_max: int) -> np.ndarray:
    """P(N <= n), n = 0..n_max, for the number N of dephasing rounds when no
    replica ever leaves the set: replica r is done after the first round n_r
    at which its own elapsed time (a sum of n_r iid Exp(a0)) reaches t_p, and
    the step stops after the first round at which every replica is done, so
    N = max_r n_r with P(n_r <= n) = P(Poisson(a0 t_p) <= n - 1)."""
    from scipy import stats
    n = np.arange(n_max + 1)
    single = np.where(n >= 1, stats.poisson(a0 * t_p).cdf(n - 1), 0.0)
    return single ** R


def decorr_events_pmf(a0: float, p_flip: float, t_c: float, k_max: int) -> np.ndarray:
    """P(K = k), k = 0..k_max, for the number K of decorrelation events when
    every jump leaves the current set with probability p_flip, independently
    of the holding times (iid Exp(a0)).  Time in the current set grows by the
    holding time of each jump that stays in it and restarts at 0 on a jump
    that leaves it; the step ends at the first jump after which it is >= t_c.

    Renewal: an attempt starts with time 0 in a set.  With M the number of
    in-set jumps whose holding times first reach t_c (P(M = m) =
    P(Poisson(a0 t_c) = m - 1)), it succeeds after m jumps with probability
    P(M = m) q^m (q = 1 - p_flip), or fails at jump j (the first j - 1 stay,
    the j-th leaves) with probability P(M >= j) q^(j-1) p_flip.  K is the sum
    of the failed attempts' lengths and the successful one's:
    f = g + h * f (discrete convolution)."""
    from scipy import stats
    q = 1.0 - p_flip
    k = np.arange(k_max + 1)
    pois = stats.poisson(a0 * t_c)
    pm = np.where(k >= 1, pois.pmf(k - 1), 0.0)        # P(M = k)
    p_ge = np.where(k >= 1, pois.sf(k - 2), 0.0)       # P(M >= k) = P(Poisson >= k - 1)
    p_ge[1] = 1.0
    g = pm * q ** k
    h = np.where(k >= 1, p_ge * q ** np.maximum(k - 1, 0) * p_flip, 0.0)
    f = np.zeros(k_max + 1)
    for kk in range(1, k_max + 1):
        f[kk] = g[kk] + np.dot(h[1:kk], f[kk - 1:0:-1])
    return f


def toggle_well_law(omega, u_lo, u_hi, v_lo, v_hi, c=(3.0, 3.0, 2.0, 2.0)):
    """Stationary law of the toggle switch restricted to the box
    [u_lo, u_hi] x [v_lo, v_hi] (transitions leaving the box dropped).  For a
    box around one well, many standard deviations wide and far from the
    other well, this is the law of the process conditioned on that well, as
    long as the time horizon is far below the switching time.  Returns the
    (u_hi - u_lo + 1, v_hi - v_lo + 1) array."""
    gu = np.arange(u_lo, u_hi + 1)
    gv = np.arange(v_lo, v_hi + 1)
    U, V = np.meshgrid(gu, gv, indexing="ij")
    U, V = U.ravel(), V.ravel()
    nu, nv = len(gu), len(gv)
    lam = toggle_rates(U, V, omega, c)
    rows, cols, vals = [], [], []
    for j, (du, dv) in enumerate(TOGGLE_STOICH):
        u2, v2 = U + du, V + dv
        ok = (u2 >= u_lo) & (u2 <= u_hi) & (v2 >= v_lo) & (v2 <= v_hi) & (lam[j] > 0)
        rows.append((U[ok] - u_lo) * nv + (V[ok] - v_lo))
        cols.append((u2[ok] - u_lo) * nv + (v2[ok] - v_lo))
        vals.append(lam[j][ok])
    n = nu * nv
    Q = sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                      shape=(n, n)).tocsr()
    Q = Q - sp.diags(np.asarray(Q.sum(axis=1)).ravel())
    return stationary_from_generator(Q.tocsr()).reshape(nu, nv)
