"""Whole-plan HIP graphs (qs_apply_graph) against eager application: the same
kernels in the same order, so replays must match the eager result bit for
bit.  Each graph is replayed several times with eager work and host
synchronisations in between, across parameter updates and for plans whose
gathers flip the state between its two buffers."""
import numpy as np
import pytest

import workloads as W
from oracle import metrics, statevec as sv

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def qs():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    import paper_2609_19147_amd as q
    q._lib.lib()
    return q


def pair(qs, n, dtype, seed):
    psi0 = W.gaussian_state(n, seed).astype(np.complex64 if dtype == "c64" else np.complex128)
    a = qs.State(n, dtype, init=None)
    b = qs.State(n, dtype, init=None)
    a.upload(psi0)
    b.upload(psi0)
    return a, b, psi0


@pytest.mark.parametrize("dtype", ["c64", "c128"])
@pytest.mark.parametrize("case", ["tfim", "qft_perm", "odd_gathers", "dense_windows", "diag_only"])
def test_graph_replays_match_eager(qs, case, dtype):
    n = 14
    streams = {
        "tfim": W.tfim_strang_stream(n, 1.0, 0.8, 0.05, 6),
        "qft_perm": W.qft_stream(n) + W.random_perm_block(n, 30, 4),
        "odd_gathers": W.random_perm_block(n, 20, 1) + W.wht_stream(n) + W.random_perm_block(n, 20, 2)
                       + [W.G("RX", 3, theta=0.2)] + W.random_perm_block(n, 20, 3),
        "dense_windows": W.ladder_stream(n // 2, 1.0, 0.5, 0.05, 2),
        "diag_only": W.long_range_ising_stream(n, 1.0, 1.5, 0.0, 0.05, 1),
    }
    plan = qs.Plan(n, streams[case])
    a, b, psi0 = pair(qs, n, dtype, 3)
    for rep in range(4):
        qs.apply_graph(a, plan)
        qs.apply(b, plan)
        if rep == 1:
            qs.norm2(a)  # eager work on the same stream between replays
        assert np.array_equal(a.download(), b.download()), rep
    ref = psi0.astype(np.complex128)
    for _ in range(4):
        ref = sv.run(ref, n, streams[case])
    assert metrics.infidelity(a.download().astype(np.complex128), ref) <= (1e-9 if dtype == "c64" else 1e-22)


def test_graph_follows_parameter_updates(qs):
    n = 12
    stream = W.hea_stream(n, 2)
    plan = qs.Plan(n, stream, n_params=4 * n)
    a, b, _ = pair(qs, n, "c64", 5)
    for seed in range(3):
        params = W.hea_params(n, 2, seed)
        plan.set_params(params)
        for _ in range(2):
            qs.apply_graph(a, plan)
            qs.apply(b, plan)
            assert np.array_equal(a.download(), b.download()), seed


def test_graph_falls_back_for_host_staged_gates(qs):
    n = 9
    rng = np.random.default_rng(2)
    stream = [W.G("UNITARY", 0, 4, 7, mat=W.random_unitary(8, rng))] + W.qft_stream(n)
    plan = qs.Plan(n, stream, window_k=-1)
    assert any(L["kind"] == "plain" for L in plan.describe()["layers"])
    a, b, _ = pair(qs, n, "c128", 6)
    qs.apply_graph(a, plan)
    qs.apply(b, plan)
    assert np.array_equal(a.download(), b.download())


def test_parameter_updates_are_ordered_after_enqueued_work(qs):
    # set_params uploads the new tables on the library's upload stream after
    # the work already enqueued on any stream that reads them: an apply that
    # is still running keeps its parameters, applies after the update see the
    # new ones, with no device-wide synchronisation in between
    import torch
    n = 20
    stream = W.hea_stream(n, 6)
    plan = qs.Plan(n, stream, n_params=12 * n)
    s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
    a = qs.State(n, "c64", stream=s1)
    b = qs.State(n, "c64", stream=s2)
    p0, p1 = W.hea_params(n, 6, 1), W.hea_params(n, 6, 2)
    plan.set_params(p0)
    qs.apply(a, plan)          # warm: tables on the device
    a.sync()
    ref_a = sv.run(sv.run(sv.basis(n, 0), n, stream, p0), n, stream, p0)
    ref_b = sv.run(sv.basis(n, 0), n, stream, p1)
    for _ in range(3):
        a.set_basis(0)
        b.set_basis(0)
        plan.set_params(p0)
        qs.apply(a, plan)      # enqueued on s1, reads the p0 tables
        qs.apply_graph(a, plan)
        plan.set_params(p1)    # no host wait for s1
        qs.apply(b, plan)      # s2, after the p1 upload
        a.sync()
        b.sync()
        assert metrics.infidelity(a.download().astype(np.complex128), ref_a) < 1e-9
        assert metrics.infidelity(b.download().astype(np.complex128), ref_b) < 1e-9
