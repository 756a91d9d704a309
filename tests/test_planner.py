"""Planner semantics on the CPU: plans built through the C ABI, interpreted
in numpy from their description, compared with the one-gate-at-a-time oracle.
Permutation layers are compared bit-exactly on index-tag states."""
import math

import numpy as np
import pytest

import workloads as W
from oracle import metrics, statevec as sv
from tests.plan_interp import run_plan

qs = pytest.importorskip("paper_2609_19147_amd")


def plan_of(n, stream, n_params=0, params=None, **kw):
    p = qs.Plan(n, stream, n_params=n_params, **kw)
    if params is not None:
        p.set_params(params)
    return p


def check_plan(n, stream, psi0=None, params=None, n_params=0, tol=1e-12, **kw):
    p = plan_of(n, stream, n_params, params, **kw)
    d = p.describe()
    psi0 = W.gaussian_state(n, 17) if psi0 is None else psi0
    got = run_plan(d, psi0, stream, params)
    ref = sv.run(psi0, n, stream, params)
    assert np.max(np.abs(got - ref)) < tol, d["layers"][:3]
    return d


def kinds(d):
    return [L["kind"] for L in d["layers"]]


@pytest.mark.parametrize("n", [4, 6, 9, 12])
def test_qft_stream_fuses_to_tile_passes(n):
    d = check_plan(n, W.qft_stream(n))
    assert set(kinds(d)) == {"tile"}
    ops = [op for L in d["layers"] for op in L["ops"]]
    assert [op["kind"] for op in ops] == [2] * n          # one QFT stage op per qubit
    assert [op["bit"] for op in ops] == list(range(n - 1, -1, -1))


@pytest.mark.parametrize("n", [5, 13, 16])
def test_qft_pass_structure_and_semantics(n):
    d = check_plan(n, W.qft_stream(n), tol=1e-11)
    assert len(d["layers"]) == (1 if n <= 13 else 2)


def test_pass_counts_at_30_qubits():
    # structure only (no state at this size): QFT and Walsh take 3 tile passes,
    # a 200-gate random permutation block is one gather
    for stream, want in ((W.qft_stream(30), ["tile"] * 3), (W.wht_stream(30), ["tile"] * 3),
                         (W.random_perm_block(30, 200, 31), ["gf2"])):
        assert kinds(qs.Plan(30, stream).describe()) == want
    # the Walsh butterflies on high bits commute with the remaining (lower) QFT
    # stages, so the composed circuit still needs only three tile passes
    both = W.qft_stream(30) + W.wht_stream(30) + W.random_perm_block(30, 200, 31)
    assert kinds(qs.Plan(30, both).describe()) == ["tile"] * 3 + ["gf2"]


@pytest.mark.parametrize("n", [4, 7, 10])
def test_walsh_layer(n):
    d = check_plan(n, W.wht_stream(n))
    assert set(kinds(d)) == {"tile"}
    assert all(op["kind"] == 1 for L in d["layers"] for op in L["ops"])


@pytest.mark.parametrize("n,seed", [(4, 1), (8, 2), (11, 3)])
def test_permutation_block_bit_exact(n, seed):
    stream = W.random_perm_block(n, 60, seed)
    d = qs.Plan(n, stream).describe()
    assert kinds(d) == ["gf2"]
    tag = W.index_tag_state(n)
    assert np.array_equal(run_plan(d, tag, stream), sv.run(tag, n, stream))


def test_ghz_chain_is_one_gather():
    n = 10
    st = W.ghz_stream(n)
    d = check_plan(n, st, psi0=sv.basis(n, 0))
    assert kinds(d) == ["tile", "gf2"]


def test_tfim_strang_fuses_diagonals_into_passes():
    n = 10
    st = W.tfim_strang_stream(n, 1.0, 0.8, 0.05, 6)
    d = check_plan(n, st, psi0=sv.basis(n, 0), tol=1e-12)
    assert set(kinds(d)) == {"tile"}
    # n <= tile bits: the evolution needs one pass per four fused diagonal layers
    assert len(d["layers"]) == 2
    d25 = qs.Plan(25, W.tfim_strang_stream(25, 1.0, 0.8, 0.05, 40)).describe()
    assert set(kinds(d25)) == {"tile"}
    # 25 qubits need three bit groups: the first window takes three passes and
    # every later step two (the diagonal rides inside a pass)
    assert len(d25["layers"]) <= 2 * 40 + 3


@pytest.mark.parametrize("n,seed", [(4, 0), (5, 1), (6, 2), (7, 3), (8, 4), (9, 5)])
def test_random_mixed_streams(n, seed):
    st = W.random_stream(n, 120, seed)
    check_plan(n, st, tol=1e-12)


def test_random_mixed_streams_small_tiles():
    n = 9
    st = W.random_stream(n, 150, 7)
    # 5-bit tiles force several groups and high tiles at n = 9
    check_plan(n, st, tol=1e-12, max_tile_bits=5)
    check_plan(10, W.qft_stream(10) + W.tfim_strang_stream(10, 1, 0.8, 0.1, 3), tol=1e-12, max_tile_bits=6)


def test_xx_yy_runs():
    n = 7
    st = ([W.G("H", q) for q in range(n)] + [W.G("RXX", q, q + 1, theta=0.3 + 0.1 * q) for q in range(n - 1)]
          + [W.G("RYY", q, (q + 2) % n, theta=-0.7) for q in range(n)] + [W.G("RX", 2, theta=0.2)])
    check_plan(n, st, tol=1e-12)


def test_parametrised_qaoa_and_hea():
    rng = np.random.default_rng(3)
    inst = W.qaoa_instances(1, 5, depth=3, n_choices=(8,))[0]
    st = W.qaoa_stream(inst, param_offset=0)
    params = rng.uniform(0, math.pi, size=6)
    check_plan(8, st, psi0=sv.basis(8, 0), params=params, n_params=6)
    st = W.hea_stream(6, 3)
    params = W.hea_params(6, 3, 1)
    check_plan(6, st, psi0=sv.basis(6, 0), params=params, n_params=len(params))


def test_identity_windows_vanish_but_small_rotations_survive():
    n = 5
    d = qs.Plan(n, [W.G("H", 1), W.G("H", 1), W.G("X", 2), W.G("X", 2)]).describe()
    assert d["layers"] == []
    # RZ(1e-6) is a real rotation: it must not be dropped as identity
    st = [W.G("RZ", 3, theta=1e-6)]
    d = check_plan(n, st, tol=1e-15)
    assert d["layers"] != []
    psi0 = W.gaussian_state(n, 1)
    got = run_plan(d, psi0, st)
    assert np.max(np.abs(got - psi0)) > 1e-8


def test_window_collapsing_to_x_becomes_a_bit_flip():
    n = 6
    st = [W.G("H", 2), W.G("H", 2), W.G("X", 2), W.G("Y", 4), W.G("Z", 4)]  # Z Y = -i X... not X
    d = qs.Plan(n, st[:3]).describe()
    assert kinds(d) == ["gf2"] and d["layers"][0]["cprime"] == 1 << (n - 1 - 2)
    check_plan(n, st, tol=1e-14)


def test_multi_controlled_and_dense_gates():
    n = 6
    rng = np.random.default_rng(2)
    U = W.random_unitary(8, rng)
    st = [W.G("H", q) for q in range(n)] + [W.G("MCZ", 0, 2, 5), W.G("MCP", 1, 3, 4, 5, theta=0.4),
                                              W.G("UNITARY", 4, 0, 2, mat=U), W.G("CU", 3, 1, mat=W.random_unitary(2, rng))]
    check_plan(n, st, tol=1e-12)


@pytest.mark.parametrize("k", [4, 5, 6])
def test_unitary_blocks_become_dense_layers(k):
    n = 11
    st = W.dense_block_stream(n, 3, k, 40 + k) + W.random_stream(n, 30, k) + W.dense_block_stream(n, 2, k, 50 + k)
    check_plan(n, st, tol=1e-12)                       # whichever plan the cost model keeps
    d = check_plan(n, st, tol=1e-12, window_k=-1)      # structured plan: one dense layer per block
    dense = [L for L in d["layers"] if L["kind"] == "dense"]
    assert len(dense) == 5
    for L in dense:
        assert L["bits"] == sorted(L["bits"]) and len(L["bits"]) == k
    # the plain path keeps them as per-gate layers, a small cap or a small state disables them
    assert "dense" not in kinds(plan_of(n, st, mode="plain").describe())
    assert "dense" not in kinds(plan_of(n, st, dense_k_max=k - 1, window_k=-1).describe())
    assert "dense" not in kinds(plan_of(k + 3, W.dense_block_stream(k + 3, 1, k, 1)).describe())


def test_dense_inverse_plan():
    n = 10
    st = W.dense_block_stream(n, 4, 5, 8) + W.qft_stream(n)
    p = plan_of(n, st)
    psi0 = W.gaussian_state(n, 2)
    fwd = run_plan(p.describe(), psi0, st)
    back = run_plan(p.inverse().describe(), fwd, st)
    assert np.max(np.abs(back - psi0)) < 1e-12


def test_grover_plan():
    n = 8
    st = W.grover_stream(n, 0b10110011, 3)
    check_plan(n, st, psi0=sv.basis(n, 0), tol=1e-12)


def test_plain_mode_is_one_layer_per_gate():
    n = 6
    st = W.random_stream(n, 40, 4)
    d = check_plan(n, st, mode="plain")
    assert kinds(d) == ["plain"] * len([g for g in st])


@pytest.mark.parametrize("bad", [
    [W.G("CNOT", 1, 1)],
    [W.G("H", 7)],
    [W.G("RX", -1, theta=0.1)],
    [W.G("RY", 0, param=3)],
    [W.G("H", 0, param=0)],
])
def test_invalid_streams_are_rejected(bad):
    with pytest.raises(qs.QsError) as e:
        qs.Plan(5, bad, n_params=1)
    assert e.value.code == -1


def test_params_must_be_bound_and_sized():
    p = qs.Plan(3, [W.G("RX", 0, param=0)], n_params=1)
    with pytest.raises(qs.QsError):
        p.set_params([0.1, 0.2])
    with pytest.raises(qs.QsError):
        p.set_params([float("nan")])


@pytest.mark.parametrize("tile_bits", [5, 6, 9, 13])
def test_twiddle_squaring_stays_inside_a_round(tile_bits):
    # a QFT stage may reuse the squared twiddle of the stage one bit above
    # only when that stage is computed freshly in the same round
    n = 18
    st = W.qft_stream(n) + W.wht_stream(n) + W.tfim_strang_stream(n, 1, 0.8, 0.05, 1, h_layer=False)
    d = qs.Plan(n, st, max_tile_bits=tile_bits).describe()
    for L in d["layers"]:
        if L["kind"] != "tile":
            continue
        for R in L["rounds"]:
            ops = L["ops"][R["ops"][0]:R["ops"][1]]
            for k, op in enumerate(ops):
                if op["square"]:
                    prev = [o for o in ops[:k] if o["kind"] == 2]
                    assert R["type"] in (1, 2), R
                    assert prev and prev[-1]["bit"] == op["bit"] + 1 and prev[-1]["base"] == op["base"]


@pytest.mark.parametrize("case", ["qft", "mixed", "tfim", "hea", "perm", "xxyy"])
def test_inverse_plan_undoes_the_plan(case):
    n = 9
    params = None
    n_params = 0
    if case == "qft":
        st = W.qft_stream(n) + W.wht_stream(n)
    elif case == "mixed":
        st = W.random_stream(n, 150, 21)
    elif case == "tfim":
        st = W.tfim_strang_stream(n, 1, 0.8, 0.1, 3)
    elif case == "hea":
        st = W.hea_stream(n, 3)
        params = W.hea_params(n, 3, 2)
        n_params = len(params)
    elif case == "perm":
        st = W.random_perm_block(n, 50, 4) + W.wht_stream(n)
    else:
        st = ([W.G("RXX", q, q + 1, theta=0.3) for q in range(n - 1)]
              + [W.G("RYY", q, q + 2, theta=0.2) for q in range(n - 2)] + W.random_stream(n, 20, 3))
    for tb in (5, 13):
        p = plan_of(n, st, n_params, params, max_tile_bits=tb)
        inv = p.inverse()
        psi0 = W.gaussian_state(n, 5)
        fwd = run_plan(p.describe(), psi0, st, params)
        np.testing.assert_allclose(fwd, sv.run(psi0, n, st, params), atol=1e-12)
        back = run_plan(inv.describe(), fwd, st, params)
        assert np.max(np.abs(back - psi0)) < 1e-12


@pytest.mark.parametrize("case", ["lr_ising", "qpe_big"])
def test_weighted_diagonal_families(case):
    if case == "lr_ising":
        n = 10
        st = W.long_range_ising_stream(n, 1.0, 1.5, 0.8, 0.05, 2)
        d = check_plan(n, st, tol=1e-12)
        groups = [len(dd["lut_groups"]) for L in d["layers"] for dd in L.get("diags", [L.get("diag")]) if dd]
        assert max(groups) == n - 1  # one group per bond distance
    else:
        t = 9
        st = W.qpe_ladder_stream(t, 0.4, first_power=23 - (t - 1))  # angles up to 0.4 * 2^23
        check_plan(t + 1, st, psi0=sv.basis(t + 1, 0), tol=1e-12)


@pytest.mark.parametrize("offset", [1, 3])
def test_qft_and_inverse_qft_on_an_upper_register(offset):
    # the register's wires are 0..t-1 of an (t + offset)-qubit state: its lowest
    # state bit is `offset`, so every stage's twiddle reads bits [offset, p)
    t = 8
    n = t + offset
    fwd = W.qft_stream(t)
    inv = [W.G("CPHASE", *g.wires, theta=-g.theta) if g.name == "CPHASE" else g for g in reversed(fwd)]
    for stream, kind in ((fwd, 2), (inv, 4)):
        d = check_plan(n, stream, tol=1e-12)
        ops = [o for L in d["layers"] for o in L.get("ops", [])]
        stages = [o for o in ops if o["kind"] == kind]
        assert len(stages) >= t - 1 and all(o["base"] == offset for o in stages)
        assert "diag" not in kinds(d)


@pytest.mark.parametrize("degree", [1, 2, 3, 5, 8])
@pytest.mark.parametrize("tile_bits", [6, 13])
def test_approximate_qft(degree, tile_bits):
    # stage p of an approximate QFT reads the bits [p - degree, p), so
    # consecutive stages have different bases: a round may not square one
    # stage's group twiddle into the next
    n = 12
    d = check_plan(n, W.qft_register_stream(range(n), degree), tol=1e-12, max_tile_bits=tile_bits)
    stages = [o for L in d["layers"] for o in L.get("ops", []) if o["kind"] == 2]
    if degree > 1:
        assert len(stages) >= n - 1
        assert any(o["base"] > 0 for o in stages)


@pytest.mark.parametrize("split", [4, 6, 8])
def test_qfts_on_adjacent_registers(split):
    # a QFT on the upper qubits (bits [n - split, n)), then one on the lower
    # qubits, then the lower register's QFT again before the upper one's:
    # stages on neighbouring bits with different bases share rounds
    n = 12
    hi = W.qft_register_stream(range(split))
    lo = W.qft_register_stream(range(split, n))
    for stream in (hi + lo, lo + hi, lo + hi + W.qft_stream(n)):
        check_plan(n, stream, tol=1e-12)
        check_plan(n, stream, tol=1e-12, max_tile_bits=7)


# ---------------------------------------------------------------- dense-window fusion
@pytest.mark.parametrize("rungs", [4, 5, 7])
def test_ladder_fuses_to_dense_windows(rungs):
    """The two-leg ladder interleaves XX, YY and ZZ per bond, so no same-family
    run forms; dense windows take it in fewer passes, exactly."""
    n = 2 * rungs
    stream = W.ladder_stream(rungs, 1.0, 0.5, 0.05, 2)
    d = check_plan(n, stream, tol=1e-12)
    assert d["windows"] > 0 and "dense" in kinds(d)
    assert all(len(L["bits"]) <= 5 for L in d["layers"] if L["kind"] == "dense")
    d0 = qs.Plan(n, stream, window_k=-1).describe()
    assert d0["windows"] == 0 and len(d["layers"]) < len(d0["layers"])
    # the windows cover every gate exactly once
    assert sum(L["window"] for L in d["layers"] if L["kind"] == "dense") + sum(
        1 for L in d["layers"] if L["kind"] == "plain") <= len(stream)


@pytest.mark.parametrize("n,k", [(9, 4), (10, 5), (12, 6)])
def test_decomposed_qft_window_plans(n, k):
    stream = W.decomposed_qft_stream(n)
    d = check_plan(n, stream, tol=1e-11, window_k=k)
    assert all(len(L["bits"]) <= k for L in d["layers"] if L["kind"] == "dense")
    d0 = qs.Plan(n, stream, window_k=-1).describe()
    assert len(d["layers"]) <= len(d0["layers"])


def test_window_fusion_on_random_decomposed_streams():
    for seed in range(6):
        n = 8 + seed % 3
        stream = W.random_stream(n, 120, 40 + seed, kinds=("H", "RX", "RZ", "CNOT", "CZ", "SWAP", "RXX", "CU", "T"))
        check_plan(n, stream, tol=1e-11)
        check_plan(n, stream, tol=1e-11, window_k=4)
        check_plan(n, stream, tol=1e-11, window_k=6)


def test_structured_streams_keep_structured_plans():
    cases = [(20, W.qft_stream(20)), (16, W.tfim_strang_stream(16, 1.0, 0.8, 0.05, 3)),
             (12, W.qaoa_stream(W.qaoa_instances(1, 5, depth=2, n_choices=(12,))[0])),
             (14, W.heisenberg_stream(14, 1.0, 0.5, 0.05, 2, W.random_fields(14, 1.0, 2))),
             (30, W.qft_stream(30) + W.wht_stream(30) + W.random_perm_block(30, 200, 31))]
    for n, stream in cases:
        assert qs.Plan(n, stream).describe()["windows"] == 0, n


def test_window_fusion_leaves_parametrised_gates():
    n = 9
    stream = W.ladder_stream(4, 1.0, 0.5, 0.05, 1)[:30]
    stream[7] = W.G("RZZ", 0, 1, theta=0.1, param=0)
    stream[20] = W.G("RX", 5, theta=0.0, param=1)
    stream += [W.G("H", q) for q in range(n)]
    p = plan_of(n, stream, n_params=2)
    for params in ([0.3, -1.1], [2.0, 0.25]):
        p.set_params(params)
        got = run_plan(p.describe(), W.gaussian_state(n, 3), stream, params)
        ref = sv.run(W.gaussian_state(n, 3), n, stream, params)
        assert np.max(np.abs(got - ref)) < 1e-12


def test_window_inverse_plan_returns_input():
    rungs = 5
    n = 2 * rungs
    stream = W.ladder_stream(rungs, 1.0, 0.5, 0.05, 1)
    p = qs.Plan(n, stream)
    psi0 = W.gaussian_state(n, 9)
    fwd = run_plan(p.describe(), psi0, stream)
    back = run_plan(p.inverse().describe(), fwd, stream)
    assert p.describe()["windows"] > 0
    assert np.max(np.abs(back - psi0)) < 1e-12


def test_window_option_validation():
    for bad in (3, 7, -2):
        with pytest.raises(Exception):
            qs.Plan(10, W.ladder_stream(5, 1.0, 0.5, 0.05, 1), window_k=bad)
    # fewer than 8 qubits: no window (a dense block needs 4 other bits)
    assert qs.Plan(6, W.ladder_stream(3, 1.0, 0.5, 0.05, 1)).describe()["windows"] == 0


@pytest.mark.parametrize("n", [9, 14, 20])
def test_trivial_qft_stage_and_hadamard_cancel(n):
    """The QFT's last stage (on the register's lowest bit: no twiddle bits)
    is a plain butterfly; the Walsh layer's H on the same bit cancels it."""
    stream = W.qft_stream(n) + W.wht_stream(n)
    d = check_plan(n, stream, tol=1e-11)
    ops = [op for L in d["layers"] if L["kind"] == "tile" for op in L["ops"]]
    assert len(ops) == 2 * n - 2
    assert all(op["bit"] != 0 for op in ops)
    # an H on another bit in between does not block it; a gate on bit 0 does
    blocked = W.qft_stream(n) + [W.G("T", n - 1)] + W.wht_stream(n)
    d2 = check_plan(n, blocked, tol=1e-11)
    assert sum(1 for L in d2["layers"] if L["kind"] == "tile" for op in L["ops"]) > 2 * n - 2


def test_mixed_streams_choose_windows_per_chunk():
    """A structured transform, a decomposed ladder and a structured transform
    again: the ladder's chunks take dense windows, the transforms keep their
    tile passes, and the whole plan is exact and shorter than the structured one."""
    n = 12
    stream = W.qft_stream(n) + W.ladder_stream(6, 1.0, 0.5, 0.05, 2) + W.wht_stream(n) + W.qft_stream(n)
    d = check_plan(n, stream, tol=1e-11)
    assert d["windows"] > 0
    k = kinds(d)
    assert "dense" in k and "tile" in k
    d0 = qs.Plan(n, stream, window_k=-1).describe()
    assert len(d["layers"]) < len(d0["layers"])
    # the structured head stays a tile pass: no window swallows the transform
    assert k[0] == "tile"


@pytest.mark.parametrize("balance", [0, -1])
@pytest.mark.parametrize("dl", [0, -1, 2, 4])
def test_diagonal_pass_geometry_and_balance_options(balance, dl):
    # every combination of the two knobs is the same operator
    n = 14
    st = W.tfim_strang_stream(n, 1.0, 0.8, 0.05, 4)
    d = check_plan(n, st, psi0=sv.basis(n, 0), tol=1e-11, max_tile_bits=8, diag_low_bits=dl,
                   balance_passes=balance)
    assert set(kinds(d)) == {"tile"}
    if dl > 0:
        for L in d["layers"]:
            if L["diags"] and L["h"] > 0:
                assert L["L"] <= dl


def test_balance_moves_ops_after_the_diagonal_to_the_next_pass():
    # structure at 25 qubits: with balancing the diagonal-carrying passes hand
    # trailing rotations on low bits to the following contiguous pass; the pass
    # count and the total op count are unchanged
    st = W.tfim_strang_stream(25, 1.0, 0.8, 0.05, 10)
    on = qs.Plan(25, st, diag_low_bits=-1).describe()["layers"]
    off = qs.Plan(25, st, diag_low_bits=-1, balance_passes=-1).describe()["layers"]
    assert len(on) == len(off)
    assert sum(len(L["ops"]) for L in on) == sum(len(L["ops"]) for L in off)
    moved = 0
    for a, b in zip(on, off):
        if a["diags"]:
            assert len(a["ops"]) <= len(b["ops"])
            moved += len(b["ops"]) - len(a["ops"])
    assert moved > 0
    # and the semantics at a size the interpreter runs
    n = 12
    st12 = W.tfim_strang_stream(n, 1.0, 0.7, 0.1, 5)
    d_on = check_plan(n, st12, psi0=sv.basis(n, 0), tol=1e-11, max_tile_bits=7, diag_low_bits=-1)
    d_off = check_plan(n, st12, psi0=sv.basis(n, 0), tol=1e-11, max_tile_bits=7, diag_low_bits=-1,
                       balance_passes=-1)
    assert [len(L["ops"]) for L in d_on["layers"]] != [len(L["ops"]) for L in d_off["layers"]]


def test_balance_keeps_qaoa_layers_exact():
    # a random 3-regular MaxCut instance, angles bound as parameters
    inst = W.qaoa_instances(1, 5, depth=3, n_choices=(12,))[0]
    n = inst.n
    stream = W.qaoa_stream(inst, param_offset=0, h_layer=True)
    params = np.empty(6)
    params[0::2], params[1::2] = inst.gammas, inst.betas
    for tb in (5, 7):
        for bal in (0, -1):
            check_plan(n, stream, params=params, n_params=6, tol=1e-11, max_tile_bits=tb, balance_passes=bal)


def test_option_ranges():
    st = W.tfim_strang_stream(6, 1.0, 0.8, 0.05, 1)
    for kw in ({"diag_low_bits": 1}, {"diag_low_bits": 9}, {"diag_low_bits": -2}, {"balance_passes": 1},
               {"balance_passes": -2}):
        with pytest.raises(qs.QsError):
            qs.Plan(6, st, **kw)
