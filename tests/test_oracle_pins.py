"""Pins of the CPU oracle to things other than itself (CPU only).

Each test ties part of the oracle to a closed form, a printed value of the
paper, a library routine, an invariant or a brute-force construction, so that
a dropped term, a wrong sign, a swapped wire order or a transposed operand in
``oracle/`` fails at least one of them.
"""
import math
import os

import numpy as np
import pytest
import scipy.linalg

import workloads as W
from oracle import closed, gates as og, gradients, hamiltonian, metrics, statevec as sv

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# ---------------------------------------------------------------- brute force
def dense_gate(n, U, wires):
    """Full 2^n x 2^n matrix of a gate by explicit index bookkeeping:
    M[i, j] = U[sub(i), sub(j)] if i and j agree off the gate's wires."""
    N = 1 << n
    k = len(wires)
    idx = np.arange(N)
    sub = np.zeros(N, dtype=np.int64)
    for m, w in enumerate(wires):
        sub |= ((idx >> (n - 1 - w)) & 1) << (k - 1 - m)
    wmask = sum(1 << (n - 1 - w) for w in wires)
    rest = idx & ~wmask
    M = U[sub[:, None], sub[None, :]] * (rest[:, None] == rest[None, :])
    return M


def dense_run(n, stream, psi0, params=None):
    psi = np.array(psi0, dtype=np.complex128)
    for g in stream:
        psi = dense_gate(n, og.matrix(g, params), g.wires) @ psi
    return psi


ALL_KINDS = ("H", "X", "Y", "Z", "S", "SDG", "T", "TDG", "SX", "RX", "RY", "RZ", "P", "U",
             "CNOT", "CZ", "CPHASE", "SWAP", "RZZ", "RXX", "RYY", "CU")


@pytest.mark.parametrize("n,seed", [(1, 0), (2, 1), (3, 2), (5, 3), (8, 4)])
def test_bruteforce_random_streams(n, seed):
    kinds = ALL_KINDS if n >= 2 else ("H", "X", "Y", "Z", "S", "T", "SX", "RX", "RY", "RZ", "P", "U")
    stream = W.random_stream(n, 60, seed, kinds)
    psi0 = W.gaussian_state(n, seed)
    a = sv.run(psi0, n, stream)
    b = dense_run(n, stream, psi0)
    assert np.max(np.abs(a - b)) < 1e-12


def test_bruteforce_three_qubit_gates():
    rng = np.random.default_rng(7)
    n = 6
    U = W.random_unitary(8, rng)
    stream = [W.G("UNITARY", 4, 1, 2, mat=U), W.G("MCZ", 0, 3, 5), W.G("MCP", 5, 2, 1, theta=0.3),
              W.G("UNITARY", 0, 5, 3, mat=U)]
    psi0 = W.gaussian_state(n, 3)
    assert np.max(np.abs(sv.run(psi0, n, stream) - dense_run(n, stream, psi0))) < 1e-12


def test_wire_order_msb_first():
    # X on qubit 0 of |000> gives index 4 (qubit 0 = most significant bit)
    psi = sv.run(sv.basis(3, 0), 3, [W.G("X", 0)])
    assert psi[4] == 1.0
    # CNOT(control=2, target=0) on |001> (qubit 2 set) -> |101>
    psi = sv.run(sv.basis(3, 1), 3, [W.G("CNOT", 2, 0)])
    assert psi[5] == 1.0


@pytest.mark.parametrize("name", ALL_KINDS + ("MCZ", "MCP"))
def test_gate_unitarity(name):
    rng = np.random.default_rng(1)
    if name in ("U",):
        g = W.G(name, 0, mat=W.random_unitary(2, rng))
    elif name == "CU":
        g = W.G(name, 0, 1, mat=W.random_unitary(2, rng))
    elif name in ("MCZ", "MCP"):
        g = W.G(name, 0, 1, 2, theta=0.7)
    elif name in W.TWO_QUBIT:
        g = W.G(name, 0, 1, theta=1.234)
    else:
        g = W.G(name, 0, theta=1.234)
    U = og.matrix(g)
    assert np.allclose(U.conj().T @ U, np.eye(U.shape[0]), atol=1e-14)


def test_rotation_conventions():
    t = 0.37
    assert np.allclose(og.rx(t), scipy.linalg.expm(-0.5j * t * og.X))
    assert np.allclose(og.ry(t), scipy.linalg.expm(-0.5j * t * og.Y))
    assert np.allclose(og.rz(t), scipy.linalg.expm(-0.5j * t * og.Z))
    for P, name in ((og.X, "RXX"), (og.Y, "RYY"), (og.Z, "RZZ")):
        assert np.allclose(og.matrix(W.G(name, 0, 1, theta=t)),
                           scipy.linalg.expm(-0.5j * t * np.kron(P, P)))
    assert np.allclose(og.SX @ og.SX, og.X)
    assert np.allclose(og.S @ og.S, og.Z) and np.allclose(og.T @ og.T, og.S)


def test_norm_preserved_every_gate():
    n = 7
    psi = W.gaussian_state(n, 11)
    for g in W.random_stream(n, 80, 12):
        psi = sv.apply_gate(psi, n, g)
        assert abs(metrics.norm2(psi) - 1.0) < 1e-13


# ---------------------------------------------------------------- QFT
@pytest.mark.parametrize("n", [1, 2, 5, 8])
def test_qft_basis_closed_form(n):
    N = 1 << n
    rev = closed.bit_reverse(np.arange(N), n).astype(np.int64)
    for j in range(0, N, max(1, N // 16)):
        psi = sv.run(sv.basis(n, j), n, W.qft_stream(n))
        k = np.arange(N)
        expect = np.exp(2j * math.pi * j * k / N) / math.sqrt(N)
        got = psi[rev]  # amplitude of k sits at rev_n(k)
        assert np.max(np.abs(got - expect)) < 1e-13


def test_qft_matches_numpy_ifft():
    n = 10
    psi0 = W.gaussian_state(n, 5)
    psi = sv.run(psi0, n, W.qft_stream(n))
    N = 1 << n
    ref = np.fft.ifft(psi0) * math.sqrt(N)
    rev = closed.bit_reverse(np.arange(N), n).astype(np.int64)
    assert np.max(np.abs(psi[rev] - ref)) < 1e-13
    assert len(W.qft_stream(25)) == 325  # gate count of the paper's QFT stream


def test_qft_of_zero_is_uniform():
    n = 9
    psi = sv.run(sv.basis(n, 0), n, W.qft_stream(n))
    assert np.allclose(psi, 1 / math.sqrt(1 << n), atol=1e-14)


def test_qft_sparse_closed_matches_oracle():
    n = 9
    idx, c = W.sparse_state(n, 4, k=5)
    psi0 = np.zeros(1 << n, np.complex128)
    psi0[idx.astype(np.int64)] = c
    full = sv.run(psi0, n, W.qft_stream(n))
    ys = np.arange(1 << n, dtype=np.uint64)
    assert np.max(np.abs(closed.qft_sparse(n, idx, c, ys) - full)) < 1e-13


# ---------------------------------------------------------------- Walsh
@pytest.mark.parametrize("n", [1, 3, 6, 10])
def test_wht_hadamard_matrix(n):
    psi0 = W.gaussian_state(n, n)
    psi = sv.run(psi0, n, W.wht_stream(n))
    Hn = scipy.linalg.hadamard(1 << n) / math.sqrt(1 << n)
    assert np.max(np.abs(psi - Hn @ psi0)) < 1e-13


def test_wht_sparse_closed_and_involution():
    n = 8
    idx, c = W.sparse_state(n, 9, k=6)
    psi0 = np.zeros(1 << n, np.complex128)
    psi0[idx.astype(np.int64)] = c
    full = sv.run(psi0, n, W.wht_stream(n))
    ys = np.arange(1 << n, dtype=np.uint64)
    assert np.max(np.abs(closed.wht_sparse(n, idx, c, ys) - full)) < 1e-14
    back = sv.run(full, n, W.wht_stream(n))
    assert np.max(np.abs(back - psi0)) < 1e-14


@pytest.mark.parametrize("n", [1, 5, 9])
def test_qft_then_wht_product_form_matches_composition(n):
    # brute force: the two streams applied one gate at a time
    idx, c = W.sparse_state(n, 30 + n, k=min(5, 1 << n))
    psi0 = np.zeros(1 << n, np.complex128)
    psi0[idx.astype(np.int64)] = c
    full = sv.run(psi0, n, W.qft_stream(n) + W.wht_stream(n))
    ys = np.arange(1 << n, dtype=np.uint64)
    assert np.max(np.abs(closed.qft_wht_sparse(n, idx, c, ys) - full)) < 1e-13


def test_qft_then_wht_special_cases():
    n = 12
    ys = np.arange(1 << n, dtype=np.uint64)
    # |0>: the QFT gives the uniform state and the Walsh layer maps it back to |0>
    out = closed.qft_wht_sparse(n, np.array([0], np.uint64), np.array([1.0 + 0j]), ys)
    assert abs(out[0] - 1) < 1e-14 and np.max(np.abs(out[1:])) < 1e-14
    # |N/2>: QFT gives (-1)^k on amplitude k, stored at index rev(k), so the sign
    # follows bit 0 of k = the top bit of the index; its Walsh image is |N/2>
    top = 1 << (n - 1)
    out = closed.qft_wht_sparse(n, np.array([top], np.uint64), np.array([1.0 + 0j]), ys)
    assert abs(out[top] - 1) < 1e-13 and np.max(np.abs(np.delete(out, top))) < 1e-13


# ---------------------------------------------------------------- permutations
def int_replay_forward(n, stream, x):
    """Forward image g(x) of one basis index through the gates (python ints)."""
    for g in stream:
        bits = [n - 1 - w for w in g.wires]
        if g.name == "X":
            x ^= 1 << bits[0]
        elif g.name == "CNOT":
            if (x >> bits[0]) & 1:
                x ^= 1 << bits[1]
        elif g.name == "SWAP":
            a, b = (x >> bits[0]) & 1, (x >> bits[1]) & 1
            if a != b:
                x ^= (1 << bits[0]) | (1 << bits[1])
    return x


@pytest.mark.parametrize("n,seed", [(2, 1), (5, 2), (9, 3)])
def test_permutation_block(n, seed):
    stream = W.random_perm_block(n, 40, seed)
    tag = W.index_tag_state(n)
    out = sv.run(tag, n, stream)
    N = 1 << n
    # forward definition: amplitude of |x> moves to |g(x)>
    fwd = np.array([int_replay_forward(n, stream, x) for x in range(N)])
    assert sorted(fwd.tolist()) == list(range(N))
    expect = np.empty(N, np.complex128)
    expect[fwd] = tag
    assert np.array_equal(out, expect)
    src = closed.perm_source(n, stream, np.arange(N, dtype=np.uint64)).astype(np.int64)
    assert np.array_equal(out, tag[src])


def test_ghz_and_bell():
    for n in (2, 5, 11):
        psi = sv.run(sv.basis(n, 0), n, W.ghz_stream(n))
        expect = np.zeros(1 << n)
        expect[0] = expect[-1] = 1 / math.sqrt(2)
        assert np.max(np.abs(psi - expect)) < 1e-15
    bell = sv.run(sv.basis(2, 0), 2, [W.G("H", 0), W.G("CNOT", 0, 1)])
    assert np.allclose(bell, [1 / math.sqrt(2), 0, 0, 1 / math.sqrt(2)])


# ---------------------------------------------------------------- Grover
@pytest.mark.parametrize("n,k", [(4, 1), (6, 3), (8, 6), (8, 12)])
def test_grover_success_probability(n, k):
    marked = (0b1011 << (n - 4)) | 1
    psi = sv.run(sv.basis(n, 0), n, W.grover_stream(n, marked, k))
    th = math.asin(1 / math.sqrt(1 << n))
    assert abs(abs(psi[marked]) ** 2 - math.sin((2 * k + 1) * th) ** 2) < 1e-12


# ---------------------------------------------------------------- Trotter
def test_trotter_error_table_reproduced():
    rows = np.loadtxt(os.path.join(GOLDEN, "trotter_error_n6.txt"))
    n, J, h, t = 6, 1.0, 0.5, 1.0
    psi0 = sv.basis(n, 0)
    exact = hamiltonian.evolve(n, hamiltonian.tfim_terms(n, J, h), t, psi0)
    for r, L2p, maep, infp in rows:
        psi = sv.run(psi0, n, W.tfim_first_order_stream(n, J, h, t, int(r)))
        got = (metrics.l2(psi, exact), metrics.prob_mae(psi, exact),
               metrics.infidelity(psi, exact))
        for g, p in zip(got, (L2p, maep, infp)):
            # printed with three significant digits
            assert float(f"{g:.2e}") == pytest.approx(p, rel=1e-9), (r, got)


def test_second_order_trotter_scaling():
    n, J, h, T = 8, 1.0, 0.8, 0.5
    plus = sv.plus(n)
    exact = hamiltonian.evolve(n, hamiltonian.tfim_terms(n, J, h), T, plus)
    inf = []
    for steps in (5, 10, 20):
        s = W.tfim_strang_stream(n, J, h, T / steps, steps)
        psi = sv.run(sv.basis(n, 0), n, s)
        inf.append(metrics.infidelity(psi, exact))
    # infidelity ~ dt^4 for a second-order formula
    assert 12 < inf[0] / inf[1] < 20 and 12 < inf[1] / inf[2] < 20


def test_tfim_z_invariant():
    n = 8
    psi = sv.run(sv.basis(n, 0), n, W.tfim_strang_stream(n, 1.0, 0.8, 0.05, 6))
    assert np.max(np.abs(sv.expect_terms(psi, n, W.z_terms(n)))) < 1e-13
    assert np.max(np.abs(sv.expect_terms(psi, n, W.zz_chain_terms(n)))) > 1e-3


# ---------------------------------------------------------------- QAOA p=1
def qaoa_p1_edge(graph_adj, u, v, gamma, beta):
    """Closed form of <C_uv> for p=1 MaxCut QAOA (Wang, Hadfield, Jiang,
    Rieffel 2018), with d = degree - 1 and f = triangles through (u, v)."""
    du = len(graph_adj[u]) - 1
    dv = len(graph_adj[v]) - 1
    f = len((graph_adj[u] & graph_adj[v]))
    c, s = math.cos, math.sin
    return (0.5 + 0.25 * s(4 * beta) * s(gamma) * (c(gamma) ** du + c(gamma) ** dv)
            - 0.25 * s(2 * beta) ** 2 * c(gamma) ** (du + dv - 2 * f) * (1 - c(2 * gamma) ** f))


@pytest.mark.parametrize("n,seed", [(8, 1), (10, 2), (12, 3)])
def test_qaoa_p1_closed_form(n, seed):
    rng = np.random.default_rng(seed)
    edges = W.random_regular3_graph(n, rng)
    inst = W.QaoaInstance(n, edges, np.array([0.83]), np.array([0.41]))
    psi = sv.run(sv.basis(n, 0), n, W.qaoa_stream(inst))
    got = sv.expect(psi, n, W.maxcut_terms(edges))
    adj = {q: set() for q in range(n)}
    for u, v in edges:
        adj[u].add(v)
        adj[v].add(u)
    ref = sum(qaoa_p1_edge(adj, u, v, 0.83, 0.41) for u, v in edges)
    assert abs(got - ref) < 1e-12


# ---------------------------------------------------------------- expectations
def test_xxz_closed_forms():
    n = 7
    terms = W.xxz_terms(n, 0.5)
    assert sv.expect(sv.basis(n, 0), n, terms) == pytest.approx(0.5 * (n - 1), abs=1e-14)
    assert sv.expect(sv.plus(n), n, terms) == pytest.approx(n - 1, abs=1e-13)
    neel = int("01" * 4, 2) >> 1  # 0101010 for n = 7
    assert sv.expect(sv.basis(n, neel), n, terms) == pytest.approx(-0.5 * (n - 1), abs=1e-14)


def test_pauli_apply_matches_dense_matrix():
    n = 5
    rng = np.random.default_rng(3)
    psi = W.gaussian_state(n, 2)
    for _ in range(20):
        xm, zm = int(rng.integers(0, 32)), int(rng.integers(0, 32))
        a = sv.apply_pauli(psi, n, xm, zm)
        b = hamiltonian.pauli_matrix(n, xm, zm) @ psi
        assert np.max(np.abs(a - b)) < 1e-14


def test_ground_energy_two_site_heisenberg():
    # XX + YY + ZZ on two sites: singlet energy -3
    assert hamiltonian.ground_energy(2, W.xxz_terms(2, 1.0)) == pytest.approx(-3.0)


# ---------------------------------------------------------------- gradients
def test_single_gate_gradient():
    for th in (-2.0, 0.3, 1.7):
        st = [W.G("RY", 0, param=0)]
        g = gradients.parameter_shift(1, st, [th], [(1.0, 0, 1)])
        assert g[0] == pytest.approx(-math.sin(th), abs=1e-14)
        assert gradients.energy(1, st, [th], [(1.0, 0, 1)]) == pytest.approx(math.cos(th), abs=1e-15)


def test_parameter_shift_vs_fd_hea():
    n, L = 4, 2
    st = W.hea_stream(n, L)
    p = W.hea_params(n, L, 3)
    terms = W.xxz_terms(n, 0.5)
    ps = gradients.parameter_shift(n, st, p, terms)
    fd = gradients.finite_differences(n, st, p, terms)
    assert np.max(np.abs(ps - fd)) < 1e-8


def test_parameter_shift_scaled_shared_params():
    n = 4
    rng = np.random.default_rng(0)
    inst = W.QaoaInstance(n, [(0, 1), (1, 2), (2, 3), (3, 0)], np.array([0.0, 0.0]), np.array([0.0, 0.0]))
    st = W.qaoa_stream(inst, param_offset=0)
    p = rng.uniform(0, 3, size=4)
    terms = W.maxcut_terms(inst.edges)
    ps = gradients.parameter_shift(n, st, p, terms)
    fd = gradients.finite_differences(n, st, p, terms)
    assert np.max(np.abs(ps - fd)) < 1e-8


# ---------------------------------------------------------------- metrics
def test_infidelity_small_angle_exact():
    for t in (1e-3, 1e-8, 1e-13):
        a = np.array([1.0, 0.0], np.complex128)
        b = np.array([math.cos(t), math.sin(t)], np.complex128) * np.exp(0.7j)
        assert metrics.infidelity(a, b) == pytest.approx(math.sin(t) ** 2, rel=1e-6)
    psi = W.gaussian_state(6, 1)
    assert metrics.infidelity(psi, 3.0 * np.exp(1.1j) * psi) < 1e-30


def test_inverse_stream_returns_input():
    n = 6
    st = W.random_stream(n, 50, 8)
    psi0 = W.gaussian_state(n, 8)
    back = sv.run(sv.run(psi0, n, st), n, sv.inverse_stream(st))
    assert metrics.infidelity(back, psi0) < 1e-28


# ---------------------------------------------------------------- weighted diagonal families
@pytest.mark.parametrize("t,j", [(5, 0), (5, 19), (7, 100), (8, 255)])
def test_qpe_exact_phase_gives_one_basis_state(t, j):
    # theta = 2 pi j / 2^t: the counting register ends in |j>, target in |1>
    n = t + 1
    psi = sv.run(sv.basis(n, 0), n, W.qpe_ladder_stream(t, 2 * math.pi * j / 2 ** t))
    assert abs(abs(psi[(j << 1) | 1]) ** 2 - 1) < 1e-12


def test_qpe_large_angle_ladder_equals_small_angle_ladder():
    # theta 2^p with theta 2^p = 2 pi j / 2^t + 2 pi m: the same state although
    # the ladder's angles reach ~1e7 rad (exercises the phase reduction)
    t, j, p = 6, 11, 20
    theta = (2 * math.pi * j / 2 ** t + 2 * math.pi * 3) / 2 ** p
    n = t + 1
    big = sv.run(sv.basis(n, 0), n, W.qpe_ladder_stream(t, theta, first_power=p))
    assert abs(abs(big[(j << 1) | 1]) ** 2 - 1) < 1e-9


def test_long_range_ising_zz_layer_is_exact_diagonal_evolution():
    # one step with h = 0: exp(+i dt sum J(r) Z_i Z_j) exactly (all terms commute)
    n, j0, alpha, dt = 6, 1.0, 1.5, 0.07
    stream = W.long_range_ising_stream(n, j0, alpha, 0.0, dt, 1)
    psi0 = W.gaussian_state(n, 8)
    got = sv.run(psi0, n, stream)
    terms = []
    for i in range(n):
        for k in range(i + 1, n):
            terms.append((-j0 / (k - i) ** alpha, 0, (1 << i) | (1 << k)))
    ref = hamiltonian.evolve(n, terms, dt, psi0)
    assert np.max(np.abs(got - ref)) < 1e-13


# ---------------------------------------------------------------- read-out
def test_sampling_hand_worked_table():
    """Three qubits, mass 1/4 at indices 0, 2, 3, 4 (exact in binary): the
    inverse CDF skips zero-mass indices and moves on at each quarter."""
    from oracle import readout
    psi = np.array([0.5, 0, 0.5j, -0.5, 0.5, 0, 0, 0], dtype=np.complex128)
    u = [0.0, 0.1, 0.25, 0.49, 0.5, 0.74, 0.75, 0.999]
    assert list(readout.inverse_cdf_sample(psi, u)) == [0, 0, 2, 2, 3, 3, 4, 4]
    # an unnormalised state draws the same indices (mass 4 in all)
    assert list(readout.inverse_cdf_sample(2.0 * psi, u)) == [0, 0, 2, 2, 3, 3, 4, 4]


def test_sampling_frequencies_match_probabilities():
    from oracle import readout
    n = 4
    psi = W.gaussian_state(n, 5)
    p = np.abs(psi) ** 2 / np.sum(np.abs(psi) ** 2)
    u = np.random.default_rng(9).random(200_000)
    freq = np.bincount(readout.inverse_cdf_sample(psi, u).astype(np.int64), minlength=1 << n) / u.size
    sigma = np.sqrt(p * (1 - p) / u.size)
    assert np.all(np.abs(freq - p) <= 5 * sigma + 1e-12)


def test_marginal_product_state_and_ghz():
    from oracle import readout
    rng = np.random.default_rng(4)
    n = 5
    singles = [rng.normal(size=2) + 1j * rng.normal(size=2) for _ in range(n)]
    singles = [v / np.linalg.norm(v) for v in singles]
    psi = singles[0]
    for v in singles[1:]:
        psi = np.kron(psi, v)                      # qubit 0 most significant
    p1 = [np.abs(v) ** 2 for v in singles]
    assert np.allclose(readout.marginal(psi, n, [1, 3]), np.kron(p1[1], p1[3]), atol=1e-15)
    assert np.allclose(readout.marginal(psi, n, [4, 0, 2]), np.kron(np.kron(p1[0], p1[2]), p1[4]), atol=1e-15)
    assert np.allclose(readout.marginal(psi, n, list(range(n))), np.abs(psi) ** 2, atol=1e-15)
    assert readout.marginal(psi, n, []).shape == (1,)
    ghz = sv.run(sv.basis(n, 0), n, W.ghz_stream(n))
    for pair in ([0, 1], [2, 4], [1, 3]):
        assert np.allclose(readout.marginal(ghz, n, pair), [0.5, 0, 0, 0.5], atol=1e-15)


def test_marginal_per_index_loop():
    from oracle import readout
    n = 6
    psi = W.gaussian_state(n, 12)
    qubits = [4, 1]
    ref = np.zeros(4)
    for i in range(1 << n):
        b = (((i >> (n - 1 - 1)) & 1) << 1) | ((i >> (n - 1 - 4)) & 1)
        ref[b] += abs(psi[i]) ** 2
    assert np.allclose(readout.marginal(psi, n, qubits), ref, rtol=1e-14)


# ---------------------------------------------------------------- XXZ chain and ladder
def ladder_terms(rungs, J, delta):
    out = []
    for a, b in W.ladder_bonds(rungs):
        out += [W.pauli(J, {a: "X", b: "X"}), W.pauli(J, {a: "Y", b: "Y"}), W.pauli(J * delta, {a: "Z", b: "Z"})]
    return out


def test_single_bond_triple_is_exact_xxz_evolution():
    # XX, YY and ZZ on one pair commute: one Trotter step of one bond is exact
    J, delta, dt = 0.7, 0.4, 0.3
    psi0 = W.gaussian_state(2, 3)
    ref = hamiltonian.evolve(2, W.xxz_terms(2, delta, J), dt, psi0)
    assert np.max(np.abs(sv.run(psi0, 2, W.heisenberg_stream(2, J, delta, dt, 1)) - ref)) < 1e-13
    assert np.max(np.abs(sv.run(psi0, 2, W.ladder_stream(1, J, delta, dt, 1)) - ref)) < 1e-13


def test_heisenberg_random_field_first_order_convergence():
    n, J, delta, T = 6, 1.0, 1.0, 0.5
    h = W.random_fields(n, 1.0, 3)
    terms = W.xxz_terms(n, delta, J) + [(float(h[q]), 0, 1 << q) for q in range(n)]
    psi0 = sv.basis(n, W.neel_index(n))
    exact = hamiltonian.evolve(n, terms, T, psi0)
    err = [np.linalg.norm(sv.run(psi0, n, W.heisenberg_stream(n, J, delta, T / r, r, h)) - exact)
           for r in (10, 20, 40)]
    # first-order product formula: the error halves when the step halves
    assert 1.8 < err[0] / err[1] < 2.2 and 1.8 < err[1] / err[2] < 2.2


def test_ladder_conserves_magnetisation_and_converges():
    rungs, J, delta, T = 3, 1.0, 0.5, 0.4
    n = 2 * rungs
    psi0 = sv.basis(n, W.neel_index(n))
    exact = hamiltonian.evolve(n, ladder_terms(rungs, J, delta), T, psi0)
    err = []
    for r in (8, 16, 32):
        psi = sv.run(psi0, n, W.ladder_stream(rungs, J, delta, T / r, r))
        # each bond factor exp(-i dt (XX + YY + delta ZZ)) commutes with sum Z
        assert abs(sum(sv.expect_terms(psi, n, W.z_terms(n)))) < 1e-12
        err.append(np.linalg.norm(psi - exact))
    assert 1.8 < err[0] / err[1] < 2.2 and 1.8 < err[1] / err[2] < 2.2


@pytest.mark.parametrize("n", [3, 6])
def test_decomposed_qft_equals_qft(n):
    psi0 = W.gaussian_state(n, 4)
    assert np.max(np.abs(sv.run(psi0, n, W.decomposed_qft_stream(n)) - sv.run(psi0, n, W.qft_stream(n)))) < 1e-13
