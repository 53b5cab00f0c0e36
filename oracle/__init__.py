"""CPU oracle for the QPT-assisted MPDO simulator (arXiv 2508.07610).

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
link this package: only the tests, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` use it.  It shares no code with the HIP
library; the one module both sides read is the input generator
``paper_2508_07610_amd.workloads`` (gate matrices, textbook Kraus sets,
synthetic process matrices, circuit programs), which contains none of the
simulator's arithmetic.

Everything here is plain NumPy in complex128, written from the paper:

* ``channels`` -- chi-matrix -> Choi-like matrix -> eigendecomposition ->
  Kraus operators, with weight pruning (Sec. III, Eqs. (12)-(16)).
* ``dense``    -- dense density-matrix simulator (n <= 12): Kraus channels
  (Eq. (1)), Pauli expectations, pure-state and Uhlmann fidelities (Eq. (23)).
* ``mpdo``     -- CPU matrix product density operator: site tensors
  T[l, p, n, r] (Eq. (5)), noisy gate nodes K_i = N_i K~ (Eq. (8)), inner
  (noise) truncation by SVD (Eqs. (9)-(11)), bond truncation by SVD, the
  canonicalise-then-truncate sweep (Sec. II.D), transfer-matrix observables
  (Eqs. (6)-(7)).
"""
