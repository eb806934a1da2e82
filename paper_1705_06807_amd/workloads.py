"""Seeded synthetic inputs: reaction networks, problems and batches.

This module only builds input data (stoichiometry, rate constants, regions,
thresholds, seeds).  It holds none of the method's arithmetic, so the CPU
oracle's tests and the HIP path's tests can both draw their inputs from it.

Networks are described in one factored form used throughout the project:

    lambda_j(x, c) = k_j * phi_j1(x) * phi_j2(x) * ...      (state factors, left to right)
    k_j = c[rate_param_j] * kappa_j * c[p_1] * ...           (PARAM factors, left to right)

with the factor kinds

* ``FALLING``     phi(x) = x_s (x_s - 1) ... (x_s - order + 1)   (mass action)
* ``HILL_REP``    phi(x) = 1 / (1 + (x_s / K) ** c[hill_param])   (repression)
* ``HILL_SWITCH`` phi(x) = c[lo] + (c[hi] - c[lo]) q / (1 + q), q = (x_s / c[Kp]) ** order,
  with lo = hill_param, hi = param2, Kp = param3   (switching rates, Eq. (10))
* ``PARAM``       a parameter c[hill_param] in the rate constant

Stoichiometry rows are net changes (products minus reactants), which is what
both model tables of the paper list (Sec. IV, Tables I and IV).
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional, Sequence

import numpy as np

FALLING = 0
HILL_REP = 1
HILL_SWITCH = 2
PARAM = 3

STEPS = 0
TIME = 1

MAX_SPECIES = 4
MAX_REACTIONS = 8
MAX_FACTORS = 2
MAX_PARAMS = 8


@dataclasses.dataclass(frozen=True)
class Factor:
    kind: int
    species: int
    order: int = 0          # FALLING: order; HILL_SWITCH: exponent
    K: float = 1.0          # HILL_REP only: x_s is divided by K
    hill_param: int = -1    # HILL_REP: exponent; HILL_SWITCH: value at 0; PARAM: the parameter
    param2: int = -1        # HILL_SWITCH: value as x_s -> infinity
    param3: int = -1        # HILL_SWITCH: scale


@dataclasses.dataclass(frozen=True)
class Reaction:
    rate_param: int
    kappa: float
    factors: Sequence[Factor]
    stoich: Sequence[int]


@dataclasses.dataclass(frozen=True)
class Network:
    name: str
    n_species: int
    n_params: int
    reactions: Sequence[Reaction]
    param_names: Sequence[str] = ()

    @property
    def n_reactions(self) -> int:
        return len(self.reactions)

    def stoich_matrix(self) -> np.ndarray:
        return np.array([list(r.stoich) for r in self.reactions], dtype=np.int32)


@dataclasses.dataclass
class Problem:
    """One ParRep solve: the paper's problem data (Sec. II A, Alg. 1) plus outputs."""
    net: Network
    c: Sequence[float]
    x0: Sequence[int]
    region_w: Sequence[int]
    region_theta: int
    R: int
    decorr_mode: int = TIME
    decorr: float = 1.0
    dephase_mode: int = TIME
    dephase: float = 1.0
    T: float = 200.0
    t_burn: float = 0.0
    hist_lo: Sequence[int] = (0,)
    hist_hi: Sequence[int] = (1000,)
    rer_eps: Optional[Sequence[float]] = None
    seed: int = 0
    instance_id: int = 0
    max_events: int = 0

    def nbins(self) -> int:
        n = 1
        for lo, hi in zip(self.hist_lo, self.hist_hi):
            n *= hi - lo + 1
        return n

    def replace(self, **kw) -> "Problem":
        return dataclasses.replace(self, **kw)


# --------------------------------------------------------------------------
# Networks
# --------------------------------------------------------------------------

def schlogl_classic(A: float = 1e5, B: float = 2e5) -> Network:
    """Schloegl model with binomial mass action and baths A, B folded into kappa.

    A+2X->3X: c1/2*A*x(x-1); 3X->A+2X: c2/6*x(x-1)(x-2); B->X: c3*B; X->B: c4*x.
    """
    return Network(
        name="schlogl_classic",
        n_species=1,
        n_params=4,
        param_names=("c1", "c2", "c3", "c4"),
        reactions=(
            Reaction(0, A / 2.0, (Factor(FALLING, 0, order=2),), (1,)),
            Reaction(1, 1.0 / 6.0, (Factor(FALLING, 0, order=3),), (-1,)),
            Reaction(2, B, (), (1,)),
            Reaction(3, 1.0, (Factor(FALLING, 0, order=1),), (-1,)),
        ),
    )


SCHLOGL_CLASSIC_C = (3e-7, 1e-4, 1e-3, 3.5)


def schlogl_paper(V: float = 25.0, a: float = 1.0, b: float = 2.0) -> Network:
    """Schloegl model in the paper's form (Sec. IV A, Table I) at system size V."""
    return Network(
        name="schlogl_paper",
        n_species=1,
        n_params=4,
        param_names=("c1", "c2", "c3", "c4"),
        reactions=(
            Reaction(0, a / V, (Factor(FALLING, 0, order=2),), (1,)),
            Reaction(1, 1.0 / (V * V), (Factor(FALLING, 0, order=3),), (-1,)),
            Reaction(2, b * V, (), (1,)),
            Reaction(3, 1.0, (Factor(FALLING, 0, order=1),), (-1,)),
        ),
    )


SCHLOGL_PAPER_C = (3.0, 0.6, 0.25, 2.95)


def toggle(omega: float) -> Network:
    """Two-gene toggle switch, parameters ordered (a1, a2, beta, gamma).

    0->U: Omega*a1/(1+(v/Omega)^beta); U->0: u; 0->V: Omega*a2/(1+(u/Omega)^gamma); V->0: v.
    """
    om = float(omega)
    return Network(
        name="toggle",
        n_species=2,
        n_params=4,
        param_names=("a1", "a2", "beta", "gamma"),
        reactions=(
            Reaction(0, om, (Factor(HILL_REP, 1, K=om, hill_param=2),), (1, 0)),
            Reaction(-1, 1.0, (Factor(FALLING, 0, order=1),), (-1, 0)),
            Reaction(1, om, (Factor(HILL_REP, 0, K=om, hill_param=3),), (0, 1)),
            Reaction(-1, 1.0, (Factor(FALLING, 1, order=1),), (0, -1)),
        ),
    )


TOGGLE_C = (3.0, 3.0, 2.0, 2.0)


def genetic_switch() -> Network:
    """Genetic switch with positive feedback (Sec. IV B, Table IV, Eq. (10)).

    Species (DNA_in, DNA_act, mRNA, protein); parameters ordered
    (a, b, gamma, k0_min, k0_max, k1_min, k1_max, D).  Reactions: mRNA
    production a*DNA_act, mRNA decay gamma*x1, protein production gamma*b*x1,
    protein decay x2, and the DNA switching reactions that Table IV leaves
    out: inactive -> active at F(x2) and active -> inactive at G(x2) with
    F = k0_min + (k0_max - k0_min) x2^2/(x2^2 + D^2),
    G = k1_max + (k1_min - k1_max) x2^2/(x2^2 + D^2).
    """
    sw = lambda lo, hi: Factor(HILL_SWITCH, 3, order=2, hill_param=lo, param2=hi, param3=7)
    return Network(
        name="genetic_switch",
        n_species=4,
        n_params=8,
        param_names=("a", "b", "gamma", "k0_min", "k0_max", "k1_min", "k1_max", "D"),
        reactions=(
            Reaction(0, 1.0, (Factor(FALLING, 1, order=1),), (0, 0, 1, 0)),
            Reaction(2, 1.0, (Factor(FALLING, 2, order=1),), (0, 0, -1, 0)),
            Reaction(2, 1.0, (Factor(FALLING, 2, order=1), Factor(PARAM, 0, hill_param=1)),
                     (0, 0, 0, 1)),
            Reaction(-1, 1.0, (Factor(FALLING, 3, order=1),), (0, 0, 0, -1)),
            Reaction(-1, 1.0, (sw(3, 4), Factor(FALLING, 0, order=1)), (-1, 1, 0, 0)),
            Reaction(-1, 1.0, (sw(6, 5), Factor(FALLING, 1, order=1)), (1, -1, 0, 0)),
        ),
    )


def genetic_switch_c(V: float = 2400.0) -> tuple:
    """Parameters of Sec. IV B at system size V = a b (2400 in the paper):
    b = 22.5, gamma = 50, a = V/b, k_min = V/(100 b), k_max = V/b,
    D = 1000 V/2400 (the rates and the feedback scale follow V, so smaller
    V gives the same structure with faster switching)."""
    b = 22.5
    return (V / b, b, 50.0, V / (100.0 * b), V / b, V / (100.0 * b), V / b, 1000.0 * V / 2400.0)


def genetic_switch_problem(seed: int = 0, instance_id: int = 0, V: float = 2400.0, R: int = 100,
                           n_c: float = 2e4, n_p: float = 2e4, T: float = 2e6,
                           mode: int = STEPS) -> Problem:
    """W+ = {x2 < 511.2865 V/2400} (the horizontal line through the saddle),
    start at the low stable point with inactive DNA, histogram box
    [0,1]^2 x [0, 24 V/2400] x [0, 4000 V/2400] (at V = 2400 the stationary
    law leaves about 3e-12 of its mass above 4000 proteins)."""
    f = V / 2400.0
    return Problem(
        net=genetic_switch(), c=genetic_switch_c(V), x0=(1, 0, 0, int(round(25.2628 * f))),
        region_w=(0, 0, 0, 1), region_theta=int(math.floor(511.2865 * f)) + 1,
        R=R, decorr_mode=mode, decorr=n_c, dephase_mode=mode, dephase=n_p,
        T=T, t_burn=T / 2.0, hist_lo=(0, 0, 0, 0),
        hist_hi=(1, 1, int(math.ceil(24 * f)), int(math.ceil(4000 * f))),
        rer_eps=(0.01,) * 8, seed=seed, instance_id=instance_id)


def pure_death(rate: float = 1.0) -> Network:
    """X -> 0 at rate c1*x: reaches the absorbing state x = 0 (a0 = 0)."""
    return Network(
        name="pure_death",
        n_species=1,
        n_params=1,
        param_names=("c1",),
        reactions=(Reaction(0, 1.0, (Factor(FALLING, 0, order=1),), (-1,)),),
    )


def birth_death(kb: float = 1.0) -> Network:
    """0 -> X at c1, X -> 0 at c2*x (Poisson stationary law)."""
    return Network(
        name="birth_death",
        n_species=1,
        n_params=2,
        param_names=("c1", "c2"),
        reactions=(
            Reaction(0, 1.0, (), (1,)),
            Reaction(1, 1.0, (Factor(FALLING, 0, order=1),), (-1,)),
        ),
    )


def self_loop() -> Network:
    """One channel that fires at the constant rate c1 and changes nothing:
    every holding time is Exp(c1) and the state never moves."""
    return Network(
        name="self_loop",
        n_species=1,
        n_params=1,
        param_names=("c1",),
        reactions=(Reaction(0, 1.0, (), (0,)),),
    )


def flip_chain() -> Network:
    """Two species with x + y = 1: a self-loop at rate c1, and y -> x, x -> y
    at rate c2 each (so a0 = c1 + c2 in both states).  With the sets
    {x >= 1} and {x < 1}, every jump leaves the current set with probability
    c2 / (c1 + c2), independently of the holding times."""
    return Network(
        name="flip_chain",
        n_species=2,
        n_params=2,
        param_names=("c1", "c2"),
        reactions=(
            Reaction(0, 1.0, (), (0, 0)),
            Reaction(1, 1.0, (Factor(FALLING, 1, order=1),), (1, -1)),
            Reaction(1, 1.0, (Factor(FALLING, 0, order=1),), (-1, 1)),
        ),
    )


def self_loop_problem(seed: int = 0, instance_id: int = 0, rate: float = 4.0, R: int = 16,
                      t_p: float = 2.5) -> Problem:
    """Dephasing-rule pin: constant a0 = rate and one set containing every
    state, so no replica ever leaves it (no Fleming-Viot restart)."""
    return Problem(
        net=self_loop(), c=(rate,), x0=(0,), region_w=(0,), region_theta=0, R=R,
        decorr_mode=TIME, decorr=0.0, dephase_mode=TIME, dephase=t_p, T=1e6, t_burn=0.0,
        hist_lo=(0,), hist_hi=(0,), rer_eps=None, seed=seed, instance_id=instance_id)


def flip_chain_problem(seed: int = 0, instance_id: int = 0, c1: float = 3.0, c2: float = 1.0,
                       t_c: float = 1.0, R: int = 1, T: float = 2e4) -> Problem:
    """Decorrelation-rule pin: the flip chain from (1, 0) with sets {x >= 1}
    and {x < 1}, TIME decorrelation t_c and no dephasing rounds."""
    return Problem(
        net=flip_chain(), c=(c1, c2), x0=(1, 0), region_w=(1, 0), region_theta=1, R=R,
        decorr_mode=TIME, decorr=t_c, dephase_mode=STEPS, dephase=0.0, T=T, t_burn=T / 2.0,
        hist_lo=(0, 0), hist_hi=(1, 1), rer_eps=None, seed=seed, instance_id=instance_id)


# --------------------------------------------------------------------------
# Problems at the benchmark configurations
# --------------------------------------------------------------------------

def c1_schlogl(seed: int = 0, instance_id: int = 0, R: int = 32, T: float = 200.0) -> Problem:
    """Classic Schloegl, x0 = 85, regions x < 250 / x >= 250, R = 32, t_c = t_p = 1.0."""
    return Problem(
        net=schlogl_classic(), c=SCHLOGL_CLASSIC_C, x0=(85,), region_w=(1,), region_theta=250,
        R=R, decorr_mode=TIME, decorr=1.0, dephase_mode=TIME, dephase=1.0,
        T=T, t_burn=T / 2.0, hist_lo=(0,), hist_hi=(1000,), rer_eps=(0.01,) * 4,
        seed=seed, instance_id=instance_id)


# Decorrelation and dephasing time of the toggle switch.  ParRep is exact
# only as these grow (Sec. II B): the replicas must reach the quasi-stationary
# law of the well before the parallel step.  With R = 1024 at Omega = 50 the
# pooled stationary histogram is within TV 0.01 of the exact law from about
# 10 time units on (0.0013 at 20); at 1 it is off by TV 0.79.
TOGGLE_T_CP = 20.0


def c2_toggle(seed: int = 0, instance_id: int = 0, omega: float = 50.0, R: int = 1024,
              T: float = 2e4, t_cp: float = TOGGLE_T_CP) -> Problem:
    """Toggle switch, x0 = (0,0), regions u > v / u <= v, histogram [0, 8*Omega]^2,
    decorrelation and dephasing time t_cp."""
    hi = int(round(8 * omega))
    return Problem(
        net=toggle(omega), c=TOGGLE_C, x0=(0, 0), region_w=(-1, 1), region_theta=0,
        R=R, decorr_mode=TIME, decorr=t_cp, dephase_mode=TIME, dephase=t_cp,
        T=T, t_burn=T / 2.0, hist_lo=(0, 0), hist_hi=(hi, hi), rer_eps=(0.01,) * 4,
        seed=seed, instance_id=instance_id)


def c4_toggle(seed: int = 0, instance_id: int = 0, R: int = 65536, T: float = 1e5,
              omega: float = 150.0, t_cp: float = TOGGLE_T_CP) -> Problem:
    """Large single run: the toggle switch at Omega = 150 (rarer transitions)
    with 65536 replicas and horizon 1e5, histogram [0, 1200]^2."""
    return c2_toggle(seed=seed, instance_id=instance_id, omega=omega, R=R, T=T, t_cp=t_cp)


def paper_schlogl_problem(seed: int = 0, instance_id: int = 0, R: int = 100, n_c: int = 5000,
                          n_p: int = 5000, T: float = 1e5, V: float = 25.0) -> Problem:
    """The paper's Schloegl run: STEPS thresholds, W+ = {x <= 25.96} (Sec. IV A)."""
    return Problem(
        net=schlogl_paper(V), c=SCHLOGL_PAPER_C, x0=(0,), region_w=(1,), region_theta=26,
        R=R, decorr_mode=STEPS, decorr=float(n_c), dephase_mode=STEPS, dephase=float(n_p),
        T=T, t_burn=T / 2.0, hist_lo=(0,), hist_hi=(149,), rer_eps=(0.01,) * 4,
        seed=seed, instance_id=instance_id)


def c3_batch(seed: int = 0, n_schlogl: int = 128, n_toggle: int = 128,
             r_lo: int = 64, r_hi: int = 4096, omega_lo: int = 25, omega_hi: int = 100,
             T_schlogl: float = 200.0, T_toggle: float = 2e4) -> List[Problem]:
    """Mixed batch: Schloegl with each c_k scaled by a log-uniform factor in [0.9, 1.1],
    toggle with Omega uniform on {omega_lo..omega_hi}; R log-uniform on [r_lo, r_hi]."""
    rng = np.random.default_rng(seed)
    out: List[Problem] = []
    for i in range(n_schlogl):
        f = np.exp(rng.uniform(math.log(0.9), math.log(1.1), size=4))
        R = int(round(math.exp(rng.uniform(math.log(r_lo), math.log(r_hi)))))
        c = tuple(float(a * b) for a, b in zip(SCHLOGL_CLASSIC_C, f))
        p = c1_schlogl(seed=0, instance_id=i, R=R, T=T_schlogl).replace(c=c)
        out.append(p)
    for i in range(n_toggle):
        om = int(rng.integers(omega_lo, omega_hi + 1))
        R = int(round(math.exp(rng.uniform(math.log(r_lo), math.log(r_hi)))))
        out.append(c2_toggle(seed=0, instance_id=n_schlogl + i, omega=float(om), R=R, T=T_toggle))
    return out


REQUEST_ID_STRIDE = 4096


def c5_requests(seed: int = 0, n: int = 64, rate: float = 10.0, r_lo: int = 256,
                r_hi: int = 16384, omega_lo: int = 25, omega_hi: int = 150,
                T_schlogl: float = 200.0, T_toggle: float = 2e4):
    """Poisson request stream: returns (arrival_times, problems); 50% Schloegl with
    perturbed c, 50% toggle.  Request i's runs take Philox instance ids
    i * REQUEST_ID_STRIDE + k, so requests never share a stream."""
    rng = np.random.default_rng(seed)
    gaps = rng.exponential(1.0 / rate, size=n)
    arrivals = np.cumsum(gaps) - gaps[0]
    probs: List[Problem] = []
    for i in range(n):
        R = int(round(math.exp(rng.uniform(math.log(r_lo), math.log(r_hi)))))
        if rng.uniform() < 0.5:
            f = np.exp(rng.uniform(math.log(0.9), math.log(1.1), size=4))
            c = tuple(float(a * b) for a, b in zip(SCHLOGL_CLASSIC_C, f))
            probs.append(c1_schlogl(seed=seed, instance_id=i * REQUEST_ID_STRIDE, R=R,
                                    T=T_schlogl).replace(c=c))
        else:
            om = int(rng.integers(omega_lo, omega_hi + 1))
            probs.append(c2_toggle(seed=seed, instance_id=i * REQUEST_ID_STRIDE, omega=float(om),
                                   R=R, T=T_toggle))
    return arrivals, probs
