"""Plain complex128 CPU oracle for the structured-layer state-vector path.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and
the ``cpu_baseline`` leg of ``bench.py`` may import or run anything here; the
library path never does, and shares no code with it.

What it computes is the plain definition of a circuit: the state
U_G ... U_1 psi_0 obtained by applying the gates one at a time, in complex128
(numpy), with the (A, 2, B) slice update for single-qubit gates and a tensor
contraction for multi-qubit gates (paper, Section "Gate Operations" and
Appendix A, "The pure-MLX path").  The fused layers of the paper
("Hand-Tuned Metal Shaders", Section "Kernel Taxonomy" and "Semantics-
Preserving Fusion") are exact rewrites of such a stream, so this
one-gate-at-a-time result is what every fused path must reproduce.

Modules
  gates        gate matrices (qubit q = index bit n-1-q, MSB-first)
  statevec     apply gates / streams, probabilities, Pauli expectations
  metrics      normalised cancellation-free infidelity, L2, MAE, norm drift
  hamiltonian  dense Pauli-sum Hamiltonians and exact evolution (expm)
  gradients    parameter-shift and central finite-difference gradients
  closed       per-amplitude definitions used for sampled checks at sizes
               where a dense host state is too large (QFT, Walsh, index
               permutations)
  readout      marginal distributions and inverse-CDF shot sampling

Pins (see ``tests/test_oracle_pins.py``): dense brute force via Kronecker
products at <= 10 qubits, unitarity and norm preservation, the QFT closed form
and numpy.fft, the Walsh closed form and scipy.linalg.hadamard, GHZ and Bell
amplitudes, Grover success probability, the paper's Trotter-error table
(``tests/golden/trotter_error_n6.txt``), the p=1 QAOA closed form, XXZ
expectation closed forms, exact gradients of single-gate circuits, and for
the read-out a hand-worked sampling table, sample frequencies, product-state
and GHZ marginals and a per-index loop.
"""
