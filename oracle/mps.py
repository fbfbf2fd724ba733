"""Mixed-canonical MPS simulator (oracle side, complex128).

Executes the operation list produced by ``schedule.build_schedule`` on an
MPS with site tensors A[k] of shape (chi_left, 2, chi_right).  The method is
the one outlined in the paper's sec. "Resource model and cost metrics":
two-site gate on a mixed-canonical MPS, SVD re-factorisation, and truncation
to the chi largest singular values at each two-site update; LAPACK's SVD
(numpy.linalg.svd) does the factorisations.

Per-update bookkeeping (for the cost model C_circ ~ sum_m chi_m^3 of eq.
Wsample) records the bond dimensions of every update.

Near-ties at a cut made by the bond cap (the paper does not discuss them):
the singular vectors straddling a cut between sigma_{k-1} and sigma_k are
fixed by FP64 arithmetic only to an angle theta = min(1, eps / g), with g =
(sigma_{k-1} - sigma_k) / sigma_0 the gap and eps = u sqrt(R C) a backward
error of an SVD of the R x C matrix relative to sigma_0 (u = 2^-53; Wedin's
sin-theta theorem).  Turning the kept subspace by theta moves the normalised
truncated state by at most sqrt(2) theta sigma_{k-1} / |sigma_kept|, so two
SVDs that both meet that error bound give states within twice that, and an
observable of unit norm differs by at most
    B = 4 sqrt(2) theta sigma_{k-1} / |sigma_kept|.
A cut whose B exceeds 1e-10 (FP64 cannot fix its truncated state to the
1e-10 bar) counts as a tie.  B is local: a later cut amplifies a difference
that earlier rounding left, so the sensitivity of a whole trajectory is
measured instead by running it again with every factorised matrix perturbed
at the level of an SVD's backward error (``perturb``).
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import List

import numpy as np


@dataclass
class Stats:
    updates: int = 0
    shifts: int = 0
    locals: int = 0
    sum_chi3: float = 0.0          # sum over updates of chi_mid^3
    nominal_flops: float = 0.0     # see nominal_update_flops
    discarded: float = 0.0         # sum of discarded squared weights
    max_discarded: float = 0.0
    ties: int = 0
    min_gap: float = np.inf
    flags: int = 0                 # NONFINITE: a factorisation met a non-finite value


NONFINITE = 1
U_ROUND = 2.0 ** -53
TIE_BOUND = 1e-10


def cut_sensitivity(S: np.ndarray, k: int, rows: int, cols: int, eps=None) -> float:
    """Bound B on how far two SVDs may move a unit-norm observable through the
    cut between S[k-1] and S[k] (S descending; see the module docstring);
    eps is the SVDs' backward error relative to S[0], u sqrt(rows cols) for
    FP64 by default."""
    gap = (S[k - 1] - S[k]) / S[0]
    if eps is None:
        eps = U_ROUND * np.sqrt(float(rows) * float(cols))
    theta = 1.0 if gap <= eps else eps / gap
    return 4.0 * np.sqrt(2.0) * theta * S[k - 1] / np.linalg.norm(S[:k])


def svd_flops(m: int, n: int) -> float:
    """Nominal real flops of a complex SVD with thin U and V of an m x n matrix.

    Golub-Reinsch operation count 4 m^2 n + 8 m n^2 + 9 n^3 (m >= n) for real
    data (Golub & Van Loan, sec. 5.4.5), times 4 for complex arithmetic.
    """
    if m < n:
        m, n = n, m
    return 4.0 * (4.0 * m * m * n + 8.0 * m * n * n + 9.0 * n ** 3)


def nominal_update_flops(chi_l: int, chi_m: int, chi_r: int) -> float:
    """Contraction (2chi_l x chi_m) . (chi_m x 2chi_r) plus the SVD of the result."""
    return 8.0 * (2 * chi_l) * chi_m * (2 * chi_r) + svd_flops(2 * chi_l, 2 * chi_r)


class MPS:
    """``perturb = (seed, scale)``: before every factorisation add a random
    complex matrix of Frobenius norm scale * u * sqrt(R C) * |M|_F to the
    R x C matrix M (a backward error of that size; scale 1 for FP64 and
    2^29 for FP32 rounding), to measure how sensitive the trajectory is to
    rounding."""

    def __init__(self, bits: str, cutoff: float = 1e-12, perturb=None):
        self.n = len(bits)
        self.A: List[np.ndarray] = []
        for b in bits:
            t = np.zeros((1, 2, 1), dtype=complex)
            t[0, int(b), 0] = 1.0
            self.A.append(t)
        self.centre = 0
        self.cutoff = cutoff
        self.stats = Stats()
        self.perturb = None
        if perturb is not None:
            self.perturb = (np.random.default_rng(perturb[0]), float(perturb[1]))

    @classmethod
    def from_initial(cls, init, cutoff: float = 1e-12, perturb=None) -> "MPS":
        """A copy of a given mixed-canonical MPS (site order as given)."""
        m = cls("0" * len(init.tensors), cutoff, perturb)
        m.A = [np.array(a, dtype=complex, copy=True) for a in init.tensors]
        m.centre = init.centre
        return m

    # -- single-site ------------------------------------------------------
    def apply_local(self, site: int, U: np.ndarray):
        self.A[site] = np.einsum("st,atb->asb", U, self.A[site])
        self.stats.locals += 1

    def _svd(self, M: np.ndarray):
        """LAPACK's SVD; a matrix with a non-finite entry flags the sample and
        gives a rank-one NaN factorisation (its values become NaN)."""
        if not np.all(np.isfinite(M)):
            self.stats.flags |= NONFINITE
            m, n = M.shape
            return (np.full((m, 1), np.nan, dtype=complex), np.array([np.nan]),
                    np.full((1, n), np.nan, dtype=complex))
        if self.perturb is not None:
            rng, scale = self.perturb
            E = rng.standard_normal(M.shape) + 1j * rng.standard_normal(M.shape)
            size = scale * U_ROUND * np.sqrt(float(M.size)) * np.linalg.norm(M)
            M = M + E * (size / np.linalg.norm(E))
        return np.linalg.svd(M, full_matrices=False)

    def _keep(self, S: np.ndarray) -> int:
        if S.size == 0 or S[0] == 0.0:
            return 0
        return int(np.count_nonzero(S > self.cutoff * S[0]))

    def shift(self, c: int, d: int):
        """Move the centre from site c to c + d by an SVD of A[c] (reading 4)."""
        assert c == self.centre
        A = self.A[c]
        cl, _, cr = A.shape
        if d > 0:
            U, S, Vh = self._svd(A.reshape(cl * 2, cr))
            k = max(self._keep(S), 1)
            self.A[c] = U[:, :k].reshape(cl, 2, k)
            self.A[c + 1] = np.einsum("kb,bsc->ksc", S[:k, None] * Vh[:k], self.A[c + 1])
        else:
            U, S, Vh = self._svd(A.reshape(cl, 2 * cr))
            k = max(self._keep(S), 1)
            self.A[c] = Vh[:k].reshape(k, 2, cr)
            self.A[c - 1] = np.einsum("asb,bk->ask", self.A[c - 1], U[:, :k] * S[None, :k])
        self.centre = c + d
        self.stats.shifts += 1

    def truncate_to(self, chi: int):
        """Bring every bond to at most chi: the copy of a shared start for a
        sample whose cap is below the start's largest bond (the hybrid start
        of sec. "Implementation" leaves the cap of the shared state open).
        The centre moves to the first site by the exact shifts above, then
        sweeps to the last site; each step factorises the centre site as a
        (2 chi_l) x chi_r matrix, keeps k = min(chi, #{sigma > cutoff
        sigma_0}) singular values renormalised to unit norm, and moves the
        centre one site right.  With the rest of the chain right-canonical,
        step c is the optimal rank-k truncation, across the cut after site c,
        of the state that the earlier steps left.  Every step counts as a
        shift."""
        while self.centre > 0:
            self.shift(self.centre, -1)
        for c in range(self.n - 1):
            A = self.A[c]
            cl, _, cr = A.shape
            U, S, Vh = self._svd(A.reshape(cl * 2, cr))
            k = min(chi, max(self._keep(S), 1))
            Sk = S[:k] / np.linalg.norm(S[:k])
            self.A[c] = U[:, :k].reshape(cl, 2, k)
            self.A[c + 1] = np.einsum("kb,bsc->ksc", Sk[:, None] * Vh[:k], self.A[c + 1])
            self.centre = c + 1
            self.stats.shifts += 1

    # -- two-site ---------------------------------------------------------
    def update(self, i: int, G: np.ndarray, chi: int, right: bool):
        assert self.centre in (i, i + 1)
        A, B = self.A[i], self.A[i + 1]
        cl, cm, cr = A.shape[0], A.shape[2], B.shape[2]
        theta = np.einsum("asb,btc->astc", A, B)
        theta = np.einsum("uvst,astc->auvc", G.reshape(2, 2, 2, 2), theta)
        U, S, Vh = self._svd(theta.reshape(2 * cl, 2 * cr))
        r = max(self._keep(S), 1)
        k = min(chi, r)
        tot = float(np.sum(S * S))
        disc = float(np.sum(S[k:] ** 2)) / tot if tot > 0 else 0.0
        st = self.stats
        st.updates += 1
        st.sum_chi3 += float(cm) ** 3
        st.nominal_flops += nominal_update_flops(cl, cm, cr)
        st.discarded += disc
        st.max_discarded = max(st.max_discarded, disc)
        if k < r:
            # a cut made by the bond cap: the kept state is unique only when
            # sigma_{k-1} > sigma_k; record the gap and the cut's sensitivity
            gap = (S[k - 1] - S[k]) / S[0]
            st.min_gap = min(st.min_gap, gap)
            if cut_sensitivity(S, k, 2 * cl, 2 * cr) > TIE_BOUND:
                st.ties += 1
        Sk = S[:k] / np.linalg.norm(S[:k])
        if right:
            self.A[i] = U[:, :k].reshape(cl, 2, k)
            self.A[i + 1] = (Sk[:, None] * Vh[:k]).reshape(k, 2, cr)
            self.centre = i + 1
        else:
            self.A[i] = (U[:, :k] * Sk[None, :]).reshape(cl, 2, k)
            self.A[i + 1] = Vh[:k].reshape(k, 2, cr)
            self.centre = i

    def run(self, ops):
        for op in ops:
            kind = op[0]
            if kind == "local":
                self.apply_local(op[1], op[2])
            elif kind == "update":
                self.update(op[1], op[2], op[3], op[4])
            elif kind == "shift":
                self.shift(op[1], op[2])
            elif kind == "truncate":
                self.truncate_to(op[1])
            else:
                raise ValueError(kind)
        return self

    # -- read-out ---------------------------------------------------------
    def bonds(self) -> List[int]:
        return [1] + [a.shape[2] for a in self.A]

    def to_dense(self) -> np.ndarray:
        """State vector in site order (site 0 = most significant index)."""
        v = np.ones((1, 1), dtype=complex)
        for A in self.A:
            v = np.einsum("xa,asb->xsb", v, A).reshape(-1, A.shape[2])
        return v.reshape(-1)

    def expectation(self, ops_at_site) -> complex:
        """<psi| prod_k O_k |psi> / <psi|psi> with O_k = ops_at_site[k] (2x2 or None).

        Plain left-to-right transfer-matrix contraction over every site; it
        assumes no canonical form.
        """
        E = np.ones((1, 1), dtype=complex)
        N = np.ones((1, 1), dtype=complex)
        for k, A in enumerate(self.A):
            O = ops_at_site[k]
            AO = A if O is None else np.einsum("st,atb->asb", O, A)
            # the same triple sum, contracted pairwise (E with A^*, then with
            # AO) so that it costs chi^3 per site instead of chi^4
            E = np.einsum("xy,xsa,ysb->ab", E, A.conj(), AO, optimize=True)
            N = np.einsum("xy,xsa,ysb->ab", N, A.conj(), A, optimize=True)
        return complex(E[0, 0] / N[0, 0])
