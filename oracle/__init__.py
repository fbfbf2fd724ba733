"""CPU oracle for MPS TE-PAI (test infrastructure, not part of the product).

A plain, slow, float64/complex128 implementation of what the GPU path
computes, written from the paper:

* ``philox``      Philox4x32-10 counter-based generator (Salmon et al., SC'11).
* ``pai``         PAI coefficients gamma_l, selection probabilities, the
                  per-rotation table with sub-rotation splitting and
                  log ||g||_1 (appendix "PAI & TE-PAI", eqs. settings/gammas,
                  eq. overhead-bound).
* ``sampler``     TE-PAI circuit sampling (protocol steps 1-2, sec. "TE-PAI").
* ``schedule``    the MPS operation schedule of one sampled circuit (two-site
                  updates, fused runs or one update per gate, centre shifts,
                  SWAP routing of the wrap bond, truncation of a shared
                  start wider than the sample's cap).
* ``mps``         mixed-canonical MPS simulator with truncated SVD
                  (sec. "Resource model and cost metrics": bond-dimension and
                  truncation paragraphs), the near-tie bound of a cap cut and
                  a perturbed mode that measures a trajectory's rounding
                  sensitivity.
* ``trotter``     the deterministic product-formula circuit and the shared
                  Trotter state of the hybrid start (sec. "Implementation").
* ``dense``       dense state-vector references: exact circuit, Trotter,
                  exp(-iHT), and a dense replay of the MPS schedule that
                  performs each truncation as a Schmidt cut of the full state.
* ``estimator``   weights ||g||_1 sign(g_l), mean, standard error,
                  configuration variance (Statement 2 and its proof).
* ``enumerate``   exhaustive sum over all gate settings of tiny circuits
                  (Statement 1, unbiasedness).
* ``run``         the whole estimator for one Problem.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  It imports nothing from the GPU
package, and the GPU package imports nothing from here.
"""
