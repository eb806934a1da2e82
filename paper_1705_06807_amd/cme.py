"""Host tool: stationary laws and their parameter sensitivities from the
chemical master equation (CME) on a truncated state space.

The paper compares its pathwise sensitivity bounds with sensitivities of
stationary expectations obtained from the CME itself (Sec. IV A, the "CME
approximation" row of Table III, with the Schloegl chain truncated to
[0, 149]).  This module computes them for any network of the library's
factored propensity form (workloads.Network):

* the generator Q(c) of the CME restricted to a box of states (transitions
  that would leave the box are dropped, i.e. a reflecting truncation);
* the stationary law pi(c): pi Q = 0, sum(pi) = 1 (one balance equation
  replaced by the normalisation, sparse LU);
* its exact derivative with respect to each parameter c_k: differentiating
  pi Q = 0 gives (d pi) Q = -pi (dQ/dc_k) with sum(d pi) = 0, one more solve
  with the same factorisation; dQ/dc_k comes from the propensities'
  derivatives, lambda_j d(log lambda_j)/dc_k, written out per factor kind;
* the sensitivity of a stationary expectation, d E_pi[f] / d c_k =
  sum_x f(x) d pi(x) / dc_k.

The box's states must form one closed communicating class under the
truncated dynamics (otherwise the stationary law is not unique and the
factorisation reports a singular matrix); a network with a conservation law
(the genetic switch's DNA pair) needs a box that holds only the states that
respect it, which this rectangular box cannot express.

It runs on the host with numpy and scipy (a sparse solve is not a GPU
workload here); it shares no code with the HIP library or the oracle.

Command line: ``python -m paper_1705_06807_amd.cme`` prints E_pi[x] and its
sensitivities for the paper's Schloegl setting on [0, 149].
"""
from __future__ import annotations

import dataclasses
from typing import Callable, Sequence

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from . import workloads as W


@dataclasses.dataclass
class Box:
    """Integer states lo[i] <= x_i <= hi[i], enumerated row-major (species 0 slowest)."""
    lo: Sequence[int]
    hi: Sequence[int]

    def states(self) -> np.ndarray:
        axes = [np.arange(a, b + 1) for a, b in zip(self.lo, self.hi)]
        grid = np.meshgrid(*axes, indexing="ij")
        return np.stack([g.ravel() for g in grid], axis=1)

    def index(self, x: np.ndarray) -> np.ndarray:
        """Row index of each state in x (n x s); -1 outside the box."""
        dims = np.array([b - a + 1 for a, b in zip(self.lo, self.hi)])
        off = x - np.asarray(self.lo)
        inside = np.all((off >= 0) & (off < dims), axis=1)
        strides = np.array([int(np.prod(dims[i + 1:])) for i in range(len(dims))])
        idx = off @ strides
        return np.where(inside, idx, -1)


def _factor(f: W.Factor, x: np.ndarray, c: np.ndarray):
    """phi(x) of one state factor and d(log phi)/dc (n x p) over states x."""
    n = x.shape[0]
    p = len(c)
    dlog = np.zeros((n, p))
    xs = x[:, f.species].astype(np.float64)
    if f.kind == W.FALLING:
        phi = np.ones(n)
        for i in range(f.order):
            phi = phi * np.clip(xs - i, 0.0, None)
        return phi, dlog
    if f.kind == W.HILL_REP:
        h = c[f.hill_param]
        y = xs / f.K
        with np.errstate(divide="ignore"):
            q = np.where(y > 0, y ** h, 0.0 if h > 0 else 1.0)
            ly = np.where(y > 0, np.log(np.where(y > 0, y, 1.0)), 0.0)
        phi = 1.0 / (1.0 + q)
        # d log phi / dh = -q ln(y) / (1 + q)
        dlog[:, f.hill_param] = -q * ly / (1.0 + q)
        return phi, dlog
    if f.kind == W.HILL_SWITCH:
        lo, hi, Kp = c[f.hill_param], c[f.param2], c[f.param3]
        y = xs / Kp
        q = y ** f.order
        s = q / (1.0 + q)
        phi = lo + (hi - lo) * s
        with np.errstate(divide="ignore", invalid="ignore"):
            inv = np.where(phi > 0, 1.0 / phi, 0.0)
        dlog[:, f.hill_param] += (1.0 - s) * inv
        dlog[:, f.param2] += s * inv
        # ds/dKp = -order s (1 - s) / Kp
        dlog[:, f.param3] += (hi - lo) * (-f.order * s * (1.0 - s) / Kp) * inv
        return phi, dlog
    raise ValueError("not a state factor")


def propensities(net: W.Network, c: Sequence[float], x: np.ndarray):
    """lambda (m x n) and d(log lambda)/dc (m x n x p) at the states x (n x s)."""
    c = np.asarray(c, dtype=np.float64)
    n = x.shape[0]
    m = net.n_reactions
    lam = np.zeros((m, n))
    dlog = np.zeros((m, n, len(c)))
    for j, r in enumerate(net.reactions):
        k = (c[r.rate_param] if r.rate_param >= 0 else 1.0) * r.kappa
        g = np.zeros((n, len(c)))
        if r.rate_param >= 0:
            g[:, r.rate_param] += 1.0 / c[r.rate_param]
        val = np.full(n, k)
        for f in r.factors:
            if f.kind == W.PARAM:
                val = val * c[f.hill_param]
                g[:, f.hill_param] += 1.0 / c[f.hill_param]
            else:
                phi, dl = _factor(f, x, c)
                val = val * phi
                g += dl
        lam[j] = val
        dlog[j] = g
    return lam, dlog


def generator(net: W.Network, c: Sequence[float], box: Box):
    """Q (n x n, CSR) of the CME on the box and dQ/dc_k for every k."""
    X = box.states()
    n = X.shape[0]
    lam, dlog = propensities(net, c, X)
    rows, cols, vals, dvals = [], [], [], []
    for j, r in enumerate(net.reactions):
        dst = box.index(X + np.asarray(r.stoich)[None, :])
        ok = (dst >= 0) & (lam[j] > 0)
        src = np.flatnonzero(ok)
        rows.append(src)
        cols.append(dst[ok])
        vals.append(lam[j][ok])
        dvals.append(lam[j][ok][:, None] * dlog[j][ok])
    rows = np.concatenate(rows)
    cols = np.concatenate(cols)
    vals = np.concatenate(vals)
    dvals = np.concatenate(dvals)

    def assemble(v):
        A = sp.coo_matrix((v, (rows, cols)), shape=(n, n)).tocsr()
        return (A - sp.diags(np.asarray(A.sum(axis=1)).ravel())).tocsr()

    Q = assemble(vals)
    dQ = [assemble(dvals[:, k]) for k in range(dvals.shape[1])]
    return X, Q, dQ


def stationary_and_sensitivity(net: W.Network, c: Sequence[float], box: Box):
    """(states, pi, dpi) with dpi[k] = d pi / d c_k, from the truncated CME."""
    X, Q, dQ = generator(net, c, box)
    n = X.shape[0]
    # pi Q = 0 with the first balance equation replaced by sum(pi) = 1
    A = Q.T.tolil()
    A[0, :] = np.ones(n)
    lu = spla.splu(A.tocsc())
    b = np.zeros(n)
    b[0] = 1.0
    pi = lu.solve(b)
    dpi = []
    for D in dQ:
        rhs = -(D.T @ pi)
        rhs[0] = 0.0  # sum(d pi) = 0
        dpi.append(lu.solve(rhs))
    return X, pi, np.array(dpi)


def expectation_sensitivity(net: W.Network, c: Sequence[float], box: Box,
                            f: Callable[[np.ndarray], np.ndarray]):
    """E_pi[f] and d E_pi[f] / d c (one entry per parameter)."""
    X, pi, dpi = stationary_and_sensitivity(net, c, box)
    fx = np.asarray(f(X), dtype=np.float64)
    return float(pi @ fx), dpi @ fx


def main(argv=None) -> int:
    import argparse
    ap = argparse.ArgumentParser(description="stationary mean and its CME sensitivities")
    ap.add_argument("--model", choices=("schlogl", "toggle"), default="schlogl")
    ap.add_argument("--V", type=float, default=25.0, help="Schloegl system size")
    ap.add_argument("--omega", type=float, default=4.0, help="toggle system size")
    ap.add_argument("--box", type=int, default=149, help="upper end of the box per species")
    args = ap.parse_args(argv)
    if args.model == "schlogl":
        net, c, box = W.schlogl_paper(args.V), W.SCHLOGL_PAPER_C, Box([0], [args.box])
    else:
        net, c, box = W.toggle(args.omega), (3.0, 3.0, 2.0, 2.0), Box([0, 0], [args.box] * 2)
    E, d = expectation_sensitivity(net, c, box, lambda X: X[:, 0])
    names = net.param_names or tuple("c%d" % (k + 1) for k in range(len(c)))
    print("E_pi[x0] = %.6g" % E)
    for k, v in enumerate(d):
        print("d/d%-6s % .6g" % (names[k], v))
    return 0


if __name__ == "__main__":
    raise SystemExit(main())
