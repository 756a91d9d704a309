"""Adjoint-method gradients on the GPU against the oracle's parameter-shift
gradients (tolerances: complex64 1e-5, complex128 1e-11 on every component)
and against the oracle's central finite differences (h = 1e-5: complex64
1e-5, complex128 1e-8, the finite-difference error bar)."""
import math

import numpy as np
import pytest

import workloads as W
from oracle import gradients, metrics, statevec as sv

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def qs():
    import torch
    assert torch.cuda.is_available()
    import paper_2609_19147_amd as q
    return q


def test_single_rotation_closed_form(qs):
    n = 4
    for th in (-2.1, 0.4, 1.3):
        plan = qs.Plan(n, [W.G("RY", 0, param=0)], n_params=1, params=[th])
        st = qs.State(n, "c128")
        e, g = qs.adjoint_grad(st, plan, [W.pauli(1.0, {0: "Z"})])
        assert abs(e - math.cos(th)) < 1e-14
        assert abs(g[0] + math.sin(th)) < 1e-14


@pytest.mark.parametrize("dtype,tol", [("c64", 1e-5), ("c128", 1e-11)])
def test_hea_xxz_gradients_match_parameter_shift(qs, dtype, tol):
    n, layers = 12, 4
    stream = W.hea_stream(n, layers)
    params = W.hea_params(n, layers, 24)
    terms = W.xxz_terms(n, 0.5)
    plan = qs.Plan(n, stream, n_params=len(params), params=params)
    st = qs.State(n, dtype)
    e, g = qs.adjoint_grad(st, plan, terms)
    e_ref = gradients.energy(n, stream, params, terms)
    g_ref = gradients.parameter_shift(n, stream, params, terms)
    assert abs(e - e_ref) < tol
    assert np.max(np.abs(g - g_ref)) < tol, np.max(np.abs(g - g_ref))
    # the state is left at psi_L
    ref = sv.run(sv.basis(n, 0), n, stream, params)
    assert metrics.infidelity(st.download(), ref) < (1e-10 if dtype == "c64" else 1e-24)


@pytest.fixture(scope="module")
def hea12_reference():
    """The 24-qubit adjoint configuration's ansatz at 12 qubits (8 layers of
    RY, RZ on every qubit and the CNOT ladder, 192 parameters U[-pi, pi],
    seed 24, XXZ with Jz = 0.5): the oracle's energy, parameter-shift and
    central finite-difference gradients (385 + 384 circuits)."""
    n, layers = 12, 8
    stream = W.hea_stream(n, layers)
    params = W.hea_params(n, layers, 24)
    terms = W.xxz_terms(n, 0.5)
    e = gradients.energy(n, stream, params, terms)
    ps = gradients.parameter_shift(n, stream, params, terms)
    fd = gradients.finite_differences(n, stream, params, terms, h=1e-5)
    return n, stream, params, terms, e, ps, fd


@pytest.mark.parametrize("dtype,tol_ps,tol_fd", [("c64", 1e-5, 1e-5), ("c128", 1e-11, 1e-8)])
def test_config_ansatz_at_12_qubits_against_parameter_shift_and_finite_differences(
        qs, hea12_reference, dtype, tol_ps, tol_fd):
    n, stream, params, terms, e_ref, ps, fd = hea12_reference
    assert np.max(np.abs(ps - fd)) < 1e-8  # the two oracle gradients agree first
    for tile_bits in (0, 9):
        plan = qs.Plan(n, stream, n_params=len(params), params=params, max_tile_bits=tile_bits)
        st = qs.State(n, dtype)
        e, g = qs.adjoint_grad(st, plan, terms)
        assert abs(e - e_ref) < tol_ps
        assert np.max(np.abs(g - ps)) < tol_ps, np.max(np.abs(g - ps))
        assert np.max(np.abs(g - fd)) < tol_fd, np.max(np.abs(g - fd))


def test_small_tiles_and_rx_windows(qs):
    n, layers = 9, 3
    stream = []
    for l in range(layers):
        stream += [W.G("RX", q, param=2 * (l * n + q)) for q in range(n)]
        stream += [W.G("RZ", q, param=2 * (l * n + q) + 1) for q in range(n)]
        stream += [W.G("CNOT", q, (q + 3) % n) for q in range(n)]
    params = np.random.default_rng(1).uniform(-3, 3, size=2 * n * layers)
    terms = W.xxz_terms(n, 0.5) + W.z_terms(n)
    plan = qs.Plan(n, stream, n_params=len(params), params=params, max_tile_bits=5)
    e, g = qs.adjoint_grad(qs.State(n, "c128"), plan, terms)
    g_ref = gradients.parameter_shift(n, stream, params, terms)
    assert np.max(np.abs(g - g_ref)) < 1e-11


def test_unsupported_parameter_placement_is_rejected_before_any_work(qs):
    inst = W.qaoa_instances(1, 2, depth=1, n_choices=(8,))[0]
    plan = qs.Plan(8, W.qaoa_stream(inst, param_offset=0), n_params=2, params=[0.3, 0.2])
    st = qs.State(8, "c64")
    before = st.download()
    with pytest.raises(qs.QsError) as e:
        qs.adjoint_grad(st, plan, W.maxcut_terms(inst.edges))
    assert e.value.code == -4
    assert np.array_equal(st.download(), before)


def test_torch_autograd_function(qs):
    import torch
    n, layers = 8, 2
    stream = W.hea_stream(n, layers)
    terms = W.xxz_terms(n, 0.5)
    plan = qs.Plan(n, stream, n_params=2 * n * layers)
    params = torch.tensor(W.hea_params(n, layers, 5), dtype=torch.float64, requires_grad=True)
    E = qs.energy_function().apply(params, plan, terms, "c128")
    E.backward()
    g_ref = gradients.parameter_shift(n, stream, params.detach().numpy(), terms)
    assert abs(E.item() - gradients.energy(n, stream, params.detach().numpy(), terms)) < 1e-12
    assert np.max(np.abs(params.grad.numpy() - g_ref)) < 1e-11
    # parameters of any shape (the gradient takes it); the state is reused by
    # later calls, which start from |0...0> again; no gradient under no_grad
    shaped = params.detach().reshape(layers, n, 2).clone().requires_grad_(True)
    for _ in range(2):
        E2 = qs.energy_function().apply(shaped, plan, terms, "c128")
        E2.backward()
        assert E2.item() == E.item()
        assert shaped.grad.shape == shaped.shape
        assert np.max(np.abs(shaped.grad.numpy().ravel() - g_ref)) < 1e-11
        shaped.grad = None
    with torch.no_grad():
        E3 = qs.energy_function().apply(shaped, plan, terms, "c128")
    assert abs(E3.item() - E.item()) < 1e-13 and not E3.requires_grad


def test_inverse_plan_on_device(qs):
    n = 18
    stream = W.random_stream(n, 120, 9) + W.qft_stream(n) + W.random_perm_block(n, 30, 2)
    psi0 = W.gaussian_state(n, 3)
    st = qs.State(n, "c128", init=None)
    st.upload(psi0)
    plan = qs.Plan(n, stream)
    qs.apply(st, plan)
    qs.apply(st, plan.inverse())
    assert metrics.infidelity(st.download(), psi0) < 1e-24


@pytest.mark.parametrize("dtype,tol,tile_bits", [("c64", 1e-5, 13), ("c64", 1e-5, 11), ("c128", 1e-11, 12),
                                                 ("c128", 1e-11, 9)])
def test_tiled_cross_densities_on_partial_bit_sets(qs, dtype, tol, tile_bits):
    """Parametrised rotations on uneven subsets of the wires, so that a tile
    pass asks for 1 .. 13 bits' cross densities (whole register chunks, part
    chunks and spare bits), at 14 qubits against parameter shift."""
    n = 14
    rng = np.random.default_rng(5)
    subsets = [list(range(13)), [0, 5, 13], [2, 3, 4, 6, 7, 8, 9, 10, 11], [12], [1, 13, 7, 4, 9]]
    stream, k = [], 0
    for sub in subsets:
        for q in range(n):
            if q in sub:
                stream.append(W.G("RY" if k % 2 == 0 else "RX", q, param=k))
                k += 1
            else:
                stream.append(W.G("RZ", q, theta=float(rng.uniform(-1, 1))))
        stream += [W.G("CNOT", q, q + 1) for q in range(0, n - 1, 2)]
        stream += [W.G("CNOT", q, q + 1) for q in range(1, n - 1, 2)]
    params = rng.uniform(-3, 3, size=k)
    terms = W.xxz_terms(n, 0.5) + W.z_terms(n)
    plan = qs.Plan(n, stream, n_params=k, params=params, max_tile_bits=tile_bits)
    assert "tile" in [L["kind"] for L in plan.describe()["layers"]]
    e, g = qs.adjoint_grad(qs.State(n, dtype), plan, terms)
    assert abs(e - gradients.energy(n, stream, params, terms)) < tol
    g_ref = gradients.parameter_shift(n, stream, params, terms)
    assert np.max(np.abs(g - g_ref)) < tol, np.max(np.abs(g - g_ref))


def test_work_states_are_reused_across_calls_and_plans(qs):
    """The adjoint's work states stay with the state: repeated calls give the
    same bits, and a second plan (other structure, other parameter count) on
    the same state still matches parameter shift."""
    n = 10
    st = qs.State(n, "c64")
    s1 = W.hea_stream(n, 2)
    p1 = W.hea_params(n, 2, 3)
    plan1 = qs.Plan(n, s1, n_params=len(p1), params=p1)
    terms = W.xxz_terms(n, 0.5)
    e_a, g_a = qs.adjoint_grad(st, plan1, terms)
    st.set_basis(0)
    e_b, g_b = qs.adjoint_grad(st, plan1, terms)
    assert e_a == e_b and np.array_equal(g_a, g_b)
    s2 = ([W.G("RX", q, param=q) for q in range(n)] + [W.G("CNOT", q, (q + 3) % n) for q in range(n)]
          + [W.G("RY", q, param=n + q) for q in range(n - 1)])
    p2 = np.linspace(-1.0, 1.2, 2 * n - 1)
    plan2 = qs.Plan(n, s2, n_params=len(p2), params=p2)
    st.set_basis(3)
    e2, g2 = qs.adjoint_grad(st, plan2, W.z_terms(n))
    psi0 = sv.basis(n, 3)
    assert abs(e2 - gradients.energy(n, s2, p2, W.z_terms(n), psi0=psi0)) < 1e-5
    g_ref = gradients.parameter_shift(n, s2, p2, W.z_terms(n), psi0=psi0)
    assert np.max(np.abs(g2 - g_ref)) < 1e-5


@pytest.mark.parametrize("dtype,tol", [("c64", 1e-5), ("c128", 1e-11)])
def test_mixed_pauli_strings(qs, dtype, tol):
    """Observables beyond XXZ: random X/Y/Z strings of length 1-5 (some
    sharing an X mask, some with equal coefficients and Z masks that overlap
    or repeat), every term shape of the grouped H psi against the oracle's
    energy and parameter-shift gradients."""
    n, layers = 8, 2
    stream = W.hea_stream(n, layers)
    params = W.hea_params(n, layers, 7)
    rng = np.random.default_rng(11)
    terms = []
    for _ in range(40):
        k = int(rng.integers(1, 6))
        qubits = rng.choice(n, size=k, replace=False)
        ops = {int(q): "XYZ"[int(rng.integers(0, 3))] for q in qubits}
        terms.append(W.pauli(float(rng.choice([0.5, -0.25, rng.normal()])), ops))
    # repeated and same-coefficient diagonal terms (merged counts must stay disjoint)
    terms += [W.pauli(0.5, {1: "Z", 2: "Z"}), W.pauli(0.5, {1: "Z", 2: "Z"}), W.pauli(0.5, {2: "Z", 3: "Z"}),
              W.pauli(0.5, {4: "Z"}), W.pauli(0.5, {4: "Z"}), W.pauli(0.5, {5: "Z"}), W.pauli(1.5, {})]
    plan = qs.Plan(n, stream, n_params=len(params), params=params)
    e, g = qs.adjoint_grad(qs.State(n, dtype), plan, terms)
    assert abs(e - gradients.energy(n, stream, params, terms)) < tol
    g_ref = gradients.parameter_shift(n, stream, params, terms)
    assert np.max(np.abs(g - g_ref)) < tol, np.max(np.abs(g - g_ref))
