"""PAI coefficients and the per-rotation table (oracle side).

Sources in the paper:
* rotation convention R_k(theta) = exp(-i h_k theta / 2) and
  theta_k = 2 c_k T / N for time-independent H (appendix "PAI & TE-PAI",
  eq. productFormula and the text after it);
* gate settings A = I, B = R_k(sign(theta) Delta), C = R_k(pi) (eq. settings);
* coefficients gamma_1..3(|theta|) (eq. gammas), probabilities
  p_l = |gamma_l| / ||gamma||_1 and the per-gate estimator (text after it);
* ||g||_1 = prod_{j,k} ||gamma(|theta_kj|)||_1 (eq. overhead-bound).

Reading taken where the paper assumes |theta| <= Delta: a rotation with
|theta_k| > Delta is split into m_k = ceil(|theta_k| / Delta) consecutive
identical rotations R_k(theta_k / m_k) (same generator, so their product is
exactly R_k(theta_k) and the Trotter circuit is unchanged).

Biased variant without pi rotations (appendix "Proof of Statement 3"): the
gate is approximated by A and B only, with gamma~ = (1 - lambda, lambda, 0),
lambda = |theta| / Delta; both are non-negative, ||gamma~||_1 = 1 exactly,
every sign is +1 and ||g||_1 = 1, at the price of a per-gate bias
|theta| (Delta - |theta|) / 2 R''(0) + O(Delta^3).

Each table row holds one (sub-)rotation of one Trotter step.  The sampler
takes the top 63 bits v = u >> 1 of a 64-bit uniform u and compares them with
two integer thresholds:
    v < t1 -> A,   t1 <= v < t2 -> B,   otherwise C,
where t1 = floor(p1 * 2^63) and t2 = floor((p1 + p2) * 2^63), both set to
2^63 when the probability mass reaches 1 (so a setting of probability 0 is
never drawn and one of probability 1 always is).
"""
from __future__ import annotations

import math
from dataclasses import dataclass
from typing import List, Tuple

TWO63 = float(2 ** 63)
T_ONE = 2 ** 63


def gammas(theta_abs: float, delta: float) -> Tuple[float, float, float]:
    """(gamma_1, gamma_2, gamma_3) at angle |theta| for PAI angle Delta (eq. gammas)."""
    t = theta_abs
    g1 = math.cos(t / 2.0) * math.sin(delta / 2.0 - t / 2.0) / math.sin(delta / 2.0)
    g2 = math.sin(t) / math.sin(delta)
    g3 = -math.sin(t / 2.0) * math.sin(delta / 2.0 - t / 2.0) / math.cos(delta / 2.0)
    return g1, g2, g3


def gammas_no_pi(theta_abs: float, delta: float) -> Tuple[float, float, float]:
    """(1 - lambda, lambda, 0) with lambda = |theta| / Delta (no-pi variant)."""
    lam = theta_abs / delta
    return 1.0 - lam, lam, 0.0


def to_threshold(p: float) -> int:
    """floor(p * 2^63) as an integer, with p >= 1 mapped to 2^63."""
    if p >= 1.0:
        return T_ONE
    if p <= 0.0:
        return 0
    return int(p * TWO63)          # exact: scaling by 2^63 does not round


@dataclass(frozen=True)
class Row:
    term: int          # index into Problem.terms
    theta: float       # signed sub-rotation angle theta_k / m_k
    gamma: Tuple[float, float, float]
    norm1: float       # ||gamma||_1
    p: Tuple[float, float, float]
    t1: int
    t2: int


@dataclass(frozen=True)
class Table:
    rows: Tuple[Row, ...]
    log_g1_step: float      # sum over rows of log ||gamma||_1 (one Trotter step)
    n_split_terms: int
    trotter_steps: int

    @property
    def l_eff(self) -> int:
        return len(self.rows)

    def log_g1(self, layers: int | None = None) -> float:
        """log ||g||_1 of the first ``layers`` Trotter steps (all by default)."""
        j = self.trotter_steps if layers is None else layers
        return j * self.log_g1_step


def theta_of(coeff: float, total_time: float, trotter_steps: int) -> float:
    return 2.0 * coeff * total_time / trotter_steps


def build_table(problem) -> Table:
    delta = problem.delta
    if not (0.0 < delta < math.pi):
        raise ValueError("Delta must lie in (0, pi)")
    rows: List[Row] = []
    n_split = 0
    for k, term in enumerate(problem.terms):
        theta = theta_of(term.coeff, problem.total_time, problem.trotter_steps)
        m = 1
        if abs(theta) > delta:
            m = int(math.ceil(abs(theta) / delta))
            n_split += 1
        sub = theta / m
        if getattr(problem, "trotter", False):
            # deterministic product formula (eq. Trotter-Suzuki): each rotation is
            # always present and exact; read as the one-setting table (0, 1, 0)
            g = (0.0, 1.0, 0.0)
            row = Row(term=k, theta=sub, gamma=g, norm1=1.0, p=g, t1=0, t2=T_ONE)
        elif getattr(problem, "no_pi", False):
            # probabilities are the coefficients themselves; C is never drawn
            g = gammas_no_pi(abs(sub), delta)
            row = Row(term=k, theta=sub, gamma=g, norm1=1.0, p=g,
                      t1=to_threshold(g[0]), t2=T_ONE)
        else:
            g = gammas(abs(sub), delta)
            nrm = abs(g[0]) + abs(g[1]) + abs(g[2])
            p = (abs(g[0]) / nrm, abs(g[1]) / nrm, abs(g[2]) / nrm)
            row = Row(term=k, theta=sub, gamma=g, norm1=nrm, p=p,
                      t1=to_threshold(p[0]), t2=to_threshold(p[0] + p[1]))
        rows.extend([row] * m)
    log_step = 0.0
    for r in rows:
        log_step += math.log(r.norm1)
    return Table(rows=tuple(rows), log_g1_step=log_step, n_split_terms=n_split,
                 trotter_steps=problem.trotter_steps)
