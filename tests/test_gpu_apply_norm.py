"""Apply-and-norm: the norm summed by the last layer's kernel (tile pass or
GF(2) gather) against a separate FP64 reduction of the same final state, and
the final state against the plain apply (the epilogue only reads what is
stored).  Plans ending in other layers fall back to the separate reduction."""
import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def qs():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    import paper_2609_19147_amd as q
    q._lib.lib()
    return q


@pytest.fixture(autouse=True)
def _free_device_memory():
    yield
    import gc

    import torch
    gc.collect()
    torch.cuda.empty_cache()


def streams(n):
    return {
        "tile_last": W.qft_stream(n),
        "gf2_last": W.wht_stream(n) + W.random_perm_block(n, 40, 3),
        "tile_with_diag_last": W.tfim_strang_stream(n, 1.0, 0.8, 0.05, 2),
        "diag_last": W.wht_stream(n) + [W.G("RZZ", q, q + 1, theta=0.3) for q in range(n - 1)],
        "dense_last": W.dense_block_stream(n, 2, 5, 8),
    }


@pytest.mark.parametrize("dtype", ["c64", "c128"])
@pytest.mark.parametrize("n", [9, 16, 21])
@pytest.mark.parametrize("case", ["tile_last", "gf2_last", "tile_with_diag_last", "diag_last", "dense_last"])
def test_fused_norm_matches_reduction(qs, n, case, dtype):
    stream = streams(n)[case]
    plan = qs.Plan(n, stream)
    psi0 = (1.3 * W.gaussian_state(n, n)).astype(np.complex64 if dtype == "c64" else np.complex128)
    a = qs.State(n, dtype, init=None)
    a.upload(psi0)
    b = qs.State(n, dtype, init=None)
    b.upload(psi0)
    got = qs.apply_norm2(a, plan)
    qs.apply(b, plan)
    ref = qs.norm2(b)
    assert np.array_equal(a.download(), b.download())
    assert abs(got - ref) <= 1e-13 * ref, (got, ref)
    host = float(np.sum(np.abs(b.download().astype(np.complex128)) ** 2))
    assert abs(got - host) <= 1e-12 * host


def test_fused_norm_30q_benchmark_circuit(qs):
    from bench import STATE_SEED, circuit
    n = 30
    plan = qs.Plan(n, circuit(n))
    assert plan.describe()["layers"][-1]["kind"] == "gf2"
    st = qs.State(n, "c64", init=None)
    W.gaussian_state_torch(n, STATE_SEED, "c64", out=st.tensor())
    got = qs.apply_norm2(st, plan)
    ref = qs.norm2(st)
    assert abs(got - ref) <= 1e-12 * ref
    # repeatable bit for bit
    got2 = qs.apply_norm2(st, plan)
    assert abs(got2 - qs.norm2(st)) <= 1e-12 * got2
