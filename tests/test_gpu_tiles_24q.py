"""Tile passes at 24 qubits, tiles of 2^10 .. 2^13 amplitudes (thousands of
cosets per pass, every round pattern): each structured plan is checked
against the plain one-kernel-per-gate apply of the same stream on the same
input (infidelity <= 1e-10 in complex64, 1e-24 in complex128), and the norm summed by the last
pass against a separate reduction; four of the streams also against a stored
run of the oracle at 24 qubits (sampled amplitudes and the norm).  The oracle
parity of the same round patterns at small sizes is in the parity tests."""
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


@pytest.mark.parametrize("dtype", ["c64", "c128"])
@pytest.mark.parametrize("tile_bits", [11, 13])
@pytest.mark.parametrize("name", ["qft_walsh", "inverse_qft", "one_qubit_windows", "mixed"])
def test_tile_passes_against_stored_oracle_run(qs, dtype, tile_bits, name):
    """The fused tile passes at 24 qubits against the oracle's one-gate-at-a-
    time complex128 run of the same stream from the same seeded input
    (tests/golden/tiles24_streams.json, written by make_tiles24.py): 256
    sampled amplitudes and the norm."""
    import json
    import os

    import numpy as np
    import torch

    with open(os.path.join(os.path.dirname(__file__), "golden", "tiles24_streams.json")) as fh:
        gold = json.load(fh)
    rec = gold["streams"][name]
    stream = streams(N)[name]
    assert len(stream) == rec["gates"]
    plan = qs.Plan(N, stream, max_tile_bits=tile_bits, window_k=-1)
    assert "tile" in [L["kind"] for L in plan.describe()["layers"]]
    st = qs.State(N, dtype, init=None)
    st.upload(W.gaussian_state(N, 21).astype(np.complex64 if dtype == "c64" else np.complex128))
    print(f"tiles 24q vs oracle: {name} {dtype} tile_bits={tile_bits}", flush=True)
    nf = qs.apply_norm2(st, plan)
    idx = torch.tensor(gold["indices"], dtype=torch.long, device="cuda")
    got = st.tensor()[idx].cpu().numpy().astype(np.complex128)
    ref = np.array([complex(a, b) for a, b in rec["amps"]])
    amp = 2.0 ** (-N / 2)
    # complex64: float32 rounding over a few hundred gates, relative to the typical amplitude
    tol = (2e-5 if dtype == "c64" else 1e-12) * amp
    assert np.max(np.abs(got - ref)) <= tol, np.max(np.abs(got - ref)) / amp
    assert abs(nf - rec["norm2"]) <= (1e-6 if dtype == "c64" else 1e-13)
