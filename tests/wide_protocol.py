"""Host model of the protocol by which one ParRep instance is spread over
several workgroups (test infrastructure).

The device kernel for large replica counts splits the R replicas of one
instance into G contiguous groups, one per workgroup, that only meet at
chunk boundaries.  This module runs the same protocol on the host, group by
group, with the oracle's SSA event and Philox as its primitives, so that its
decisions can be checked against the oracle's serial Alg. 1 (Sec. II A)
before and beside the kernel:

* decorrelation: serial, one event at a time (every group runs it; one
  credits);
* dephasing: each group runs up to S rounds on its own, stopping at its
  first round with an exit; at the chunk's end the groups agree on the first
  exit round E and on the stopping round D (the largest of the groups' first
  rounds at which all their replicas have t^r >= t_p).  Groups that ran past
  min(D, E) replay the chunk from its saved start.  An exit round ends with
  the Fleming-Viot restart over all groups' survivors;
* parallel step: each group runs up to S rounds without crediting, stopping
  at its first exit, and keeps the exact fixed-point sum of its holding
  times per round.  The groups then agree on the first exit key, sum the
  round totals to find the first round that crosses the burn-in time or the
  horizon, and replay the chunk crediting whole rounds in parallel; the
  boundary or exit round is credited by an exact scan in key order.

The model's outputs must equal the oracle's: integers exactly, times up to
summation order.
"""
from __future__ import annotations

import math
from fractions import Fraction

import numpy as np

TAG_DECORR, TAG_DEPHASE, TAG_FV, TAG_PARALLEL = 1, 2, 3, 4
SAT = 1 << (52 + 64)
INF = float("inf")


def fx(d: float) -> int:
    """floor(d 2^64), saturating at 2^52 (+inf included)."""
    if not d < 2.0 ** 52:
        return SAT
    if not d > 0.0:
        return 0
    return math.floor(Fraction(d) * (1 << 64))


def fx_f64(v: int) -> float:
    return float(Fraction(v, 1 << 64))


class Model:
    def __init__(self, O, p, G: int, S2: int, S3: int):
        self.O, self.p, self.G, self.S2, self.S3 = O, p, G, S2, S3
        self.R = p.R
        self.n = p.net.n_species
        self.key = (p.seed, p.instance_id)
        # replica r belongs to group r // per (contiguous ranges, as in the kernel)
        self.per = -(-p.R // G)
        self.stoich = [tuple(r.stoich) for r in p.net.reactions]
        shape = tuple(hi - lo + 1 for lo, hi in zip(p.hist_lo, p.hist_hi))
        self.hist = np.zeros(shape)
        self.hist_w = np.zeros(shape)
        self.outside = 0.0
        self.outside_w = 0.0
        self.Tq = fx(p.T)
        self.tbq = fx(p.t_burn)
        self.C = 0
        self.ev_total = 0
        self.max_ev = p.max_events if p.max_events > 0 else 1 << 62
        self.counters = dict(ev_decorr=0, ev_dephase=0, ev_par_credited=0, ev_par_discarded=0,
                             cycles=0, s3_rounds=0, s2_rounds=0, status=0, fv_restarts=0,
                             end_phase=0, n_cycle_log=0)
        self.cycle_log = []
        self.x_final = None
        self.replays = 0

    # ---- primitives ------------------------------------------------------
    def region(self, x):
        d = sum(w * v for w, v in zip(self.p.region_w, x))
        return 1 if d >= self.p.region_theta else 0

    def event(self, x, step, rep, cycle, tag):
        ctr = (step & 0xFFFFFFFF, rep, cycle, (tag << 28) | ((step >> 32) & 0x0FFFFFFF))
        blk = self.O.philox(ctr, self.key)
        _, _, tau, J, _ = self.O.event(self.p.net, self.p.c, x, blk)
        post = tuple(x) if J < 0 else tuple(a + b for a, b in zip(x, self.stoich[J]))
        return tau, post

    def groups(self):
        for g in range(self.G):
            lo = g * self.per
            hi = min(self.R, lo + self.per)
            if lo < hi:
                yield range(lo, hi)

    def add_credit(self, x, full, w):
        idx = []
        for v, lo, hi in zip(x, self.p.hist_lo, self.p.hist_hi):
            if not lo <= v <= hi:
                self.outside += full
                self.outside_w += w
                return
            idx.append(v - lo)
        idx = tuple(idx)
        self.hist[idx] += full
        self.hist_w[idx] += w

    def credit_at(self, x, tau, start):
        """Credit the interval [start, start + tau) at x, cut at T; the
        interval's end."""
        E = start + fx(tau)
        full = tau
        hit = False
        if E >= self.Tq:
            hit, E = True, self.Tq
            full = fx_f64(E - start)
        if self.tbq >= E:
            w = 0.0
        elif start >= self.tbq:
            w = full
        else:
            w = fx_f64(E - self.tbq)
        self.add_credit(x, full, w)
        return E, hit

    # ---- the three steps -------------------------------------------------
    def decorrelate(self, x, W, cycle):
        steps = self.p.decorr_mode == 0
        n_c, t_c = int(self.p.decorr), self.p.decorr
        Nc, k, e = 0, 0, 0.0
        while not (Nc >= n_c if steps else e >= t_c):
            if self.ev_total + 1 > self.max_ev:
                return x, W, k, 9
            tau, post = self.event(x, k, 0, cycle, TAG_DECORR)
            k += 1
            self.ev_total += 1
            self.counters["ev_decorr"] += 1
            self.C, hit = self.credit_at(x, tau, self.C)
            if hit:
                self.x_final = tuple(x)
                return x, W, k, 1
            x = post
            if self.region(x) == W:
                Nc += 1
                e = e + tau
            else:
                W, Nc, e = self.region(x), 0, 0.0
        return x, W, k, 0

    def dephase(self, xt, W, cycle):
        p, R = self.p, self.R
        steps = p.dephase_mode == 0
        Y = [tuple(xt)] * R
        tr = [0.0] * R
        if (int(p.dephase) <= 0) if steps else (0.0 >= p.dephase):
            return Y, 0
        budget = max(0, (self.max_ev - self.ev_total) // R)
        n0 = 0
        done_at = {}  # group -> first round after which all its replicas are done (TIME)
        while True:
            if n0 >= budget:
                return None, n0
            end = min(n0 + self.S2, budget) - 1
            Y0, tr0 = list(Y), list(tr)
            exit_at = {}
            for gi, grp in enumerate(self.groups()):
                for n in range(n0, end + 1):
                    ex = False
                    for r in grp:
                        tau, post = self.event(Y[r], n, r, cycle, TAG_DEPHASE)
                        Y[r] = post
                        tr[r] = tr[r] + tau
                        ex = ex or self.region(post) != W
                    if not steps and gi not in done_at and all(tr[r] >= p.dephase for r in grp):
                        done_at[gi] = n
                    if ex:
                        exit_at[gi] = n
                        break
            E = min(exit_at.values()) if exit_at else None
            if steps:
                D = int(p.dephase) - 1
                D = D if D <= end else None
            else:
                ng = len(list(self.groups()))
                D = max(done_at.values()) if len(done_at) == ng else None
            if D is not None and (E is None or D < E):
                target, fv, stop = D, False, True
            elif E is not None:
                target, fv, stop = E, True, D == E
            else:
                n0 = end + 1
                continue
            # replay the chunk up to the target round
            Y, tr = list(Y0), list(tr0)
            for n in range(n0, target + 1):
                for r in range(R):
                    tau, post = self.event(Y[r], n, r, cycle, TAG_DEPHASE)
                    Y[r] = post
                    tr[r] = tr[r] + tau
            self.replays += 1
            # a done round found past the exit round no longer holds
            done_at = {g: d for g, d in done_at.items() if d <= target}
            if fv:
                surv = [r for r in range(R) if self.region(Y[r]) == W]
                post = list(Y)
                for r in range(R):
                    if self.region(post[r]) == W:
                        continue
                    self.counters["fv_restarts"] += 1
                    if surv:
                        ctr = (target & 0xFFFFFFFF, r, cycle,
                               (TAG_FV << 28) | ((target >> 32) & 0x0FFFFFFF))
                        blk = self.O.philox(ctr, self.key)
                        pick = (int(blk[0]) * len(surv)) >> 32
                        Y[r] = post[surv[pick]]
                    else:
                        Y[r] = tuple(xt)
            n0 = target + 1
            if stop:
                return Y, n0

    def parallel(self, Z, W, cycle):
        R = self.R
        budget = max(0, (self.max_ev - self.ev_total) // R)
        m0 = 0
        cred = disc = 0
        while True:
            if m0 >= budget:
                return None, m0, cred, disc, 0
            end = min(m0 + self.S3, budget) - 1
            # pass 1: exit detection and per-group exact round sums
            keys = []
            sums = {}
            for gi, grp in enumerate(self.groups()):
                Zg = {r: Z[r] for r in grp}
                for m in range(m0, end + 1):
                    s = 0
                    first = None
                    for r in grp:
                        tau, post = self.event(Zg[r], m, r, cycle, TAG_PARALLEL)
                        s = min(SAT, s + fx(tau))
                        if first is None and self.region(post) != W:
                            first = r
                        Zg[r] = post
                    sums[(gi, m)] = s
                    if first is not None:
                        keys.append(m * R + first)
                        break
            kstar = min(keys) if keys else None
            nstar = kstar // R if kstar is not None else None
            last_full = (nstar - 1) if nstar is not None else end
            # the first full round that crosses the burn-in time or the horizon
            C = self.C
            b = None
            for m in range(m0, last_full + 1):
                tot = min(SAT, sum(sums[(gi, m)] for gi in range(len(list(self.groups())))))
                Ce = C + tot
                if Ce >= self.Tq or (self.tbq > C and Ce > self.tbq):
                    b = m
                    break
                C = Ce
            # pass 2: replay, crediting
            for m in range(m0, (b if b is not None else last_full + 1)):
                win = self.C >= self.tbq
                tot = 0
                for r in range(R):
                    tau, post = self.event(Z[r], m, r, cycle, TAG_PARALLEL)
                    self.add_credit(Z[r], tau, tau if win else 0.0)
                    tot += fx(tau)
                    Z[r] = post
                self.C += tot
                cred += R
            rb = b if b is not None else nstar
            if rb is None:
                m0 = end + 1
                continue
            # the boundary or exit round: exact scan in key order
            K = (kstar % R) + 1 if (nstar is not None and rb == nstar) else R
            posts = []
            hit_r = None
            start = self.C
            for r in range(K):
                tau, post = self.event(Z[r], rb, r, cycle, TAG_PARALLEL)
                posts.append(post)
                start, hit = self.credit_at(Z[r], tau, start)
                if hit:
                    hit_r = r
                    break
            self.C = start
            credited = (hit_r + 1) if hit_r is not None else K
            cred += credited
            exited = nstar is not None and rb == nstar
            if hit_r is not None:
                disc += R - credited
                self.x_final = tuple(Z[hit_r])
                return "horizon", rb + 1, cred, disc, 0
            if exited:
                disc += R - credited
                return posts[K - 1], rb + 1, cred, disc, K
            for r in range(R):
                _, post = self.event(Z[r], rb, r, cycle, TAG_PARALLEL)
                Z[r] = post
            m0 = rb + 1

    def run(self):
        p = self.p
        x = tuple(p.x0)
        W = self.region(x)
        cycle = 0
        while True:
            x, W, k, stop = self.decorrelate(x, W, cycle)
            if stop:
                self.counters["end_phase"] = stop
                if stop == 9:
                    self.x_final = tuple(x)
                self.cycle_log.append((cycle, k, 0, 0, 0, stop) + tuple(self.x_final))
                break
            Y, n2 = self.dephase(x, W, cycle)
            if Y is None:
                self.counters["end_phase"] = 9
                self.x_final = tuple(x)
                self.ev_total += n2 * self.R
                self.counters["ev_dephase"] += n2 * self.R
                self.cycle_log.append((cycle, k, 0, 0, 0, 9) + tuple(x))
                break
            self.ev_total += n2 * self.R
            self.counters["ev_dephase"] += n2 * self.R
            self.counters["s2_rounds"] += n2
            out, n3, cred, disc, K = self.parallel(Y, W, cycle)
            self.ev_total += n3 * self.R
            self.counters["s3_rounds"] += n3
            self.counters["ev_par_credited"] += cred
            self.counters["ev_par_discarded"] += disc
            if out is None or out == "horizon":
                ph = 3 if out == "horizon" else 9
                if ph == 9:
                    self.x_final = tuple(x)
                self.counters["end_phase"] = ph
                self.cycle_log.append((cycle, k, n2, n3, 0, ph) + tuple(self.x_final))
                break
            self.counters["cycles"] += 1
            x = tuple(out)
            self.cycle_log.append((cycle, k, n2, n3, K, 3) + x)
            W = self.region(x)
            cycle += 1
        self.counters["status"] = 1 if self.counters["end_phase"] == 9 else 0
        self.counters["n_cycle_log"] = len(self.cycle_log)
        self.T_s = fx_f64(self.C)
        return self
