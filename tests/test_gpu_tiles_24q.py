"""Tile passes at 24 qubits, tiles of 2^10 .. 2^13 amplitudes (thousands of
cosets per pass, every round pattern): each structured plan is checked
against the plain one-kernel-per-gate apply of the same stream on the same
input (infidelity <= 1e-10 in complex64, 1e-24 in complex128), and the norm summed by the last
pass against a separate reduction.  The oracle parity of the same round
patterns at small sizes is in the parity tests."""
import pytest

import workloads as W

pytestmark = pytest.mark.gpu

N = 24


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
    one_qubit = ("H", "X", "Y", "S", "T", "SX", "RX", "RY", "U")
    return {
        "qft_walsh": W.qft_stream(n) + W.wht_stream(n),
        "inverse_qft": [W.G("CPHASE", *g.wires, theta=-g.theta) if g.name == "CPHASE" else g
                        for g in reversed(W.qft_stream(n))],
        "rx_layers": [W.G("RX", q, theta=0.1 + 0.02 * q) for q in range(n)] * 2,
        "ry_layers": [W.G("RY", q, theta=0.3 - 0.01 * q) for q in range(n)],
        "one_qubit_windows": W.random_stream(n, 160, 8, kinds=one_qubit),
        "mixed": W.random_stream(n, 120, 9),
    }


INF = {"c64": 1e-10, "c128": 1e-24}


@pytest.mark.parametrize("dtype", ["c64", "c128"])
@pytest.mark.parametrize("tile_bits", [10, 11, 12, 13])
@pytest.mark.parametrize("name", ["qft_walsh", "inverse_qft", "rx_layers", "ry_layers", "one_qubit_windows", "mixed"])
def test_tile_passes_match_plain_apply(qs, dtype, tile_bits, name):
    stream = streams(N)[name]
    fused = qs.Plan(N, stream, max_tile_bits=tile_bits, window_k=-1)
    kinds = [L["kind"] for L in fused.describe()["layers"]]
    assert "tile" in kinds
    plain = qs.Plan(N, stream, mode="plain")
    a = qs.State(N, dtype, init=None)
    W.gaussian_state_torch(N, 21, dtype, out=a.tensor())
    b = qs.State(N, dtype, init=None)
    b.copy_from(a)
    print(f"tiles 24q: {name} {dtype} tile_bits={tile_bits} layers={len(kinds)}", flush=True)
    nf = qs.apply_norm2(a, fused)
    qs.apply(b, plain)
    assert qs.infidelity(a, b) <= INF[dtype]
    assert abs(nf - qs.norm2(a)) <= 1e-9 * max(1.0, nf)
    # a second application starts from a state the first one wrote in place
    qs.apply(a, fused)
    qs.apply(b, plain)
    assert qs.infidelity(a, b) <= INF[dtype]
