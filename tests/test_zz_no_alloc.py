"""The allocation-free sampling entry point (qs_sample_noalloc, static device
scratch) against qs_sample on the same states and uniform numbers: the drawn
indices must be equal, bit for bit, on consecutive calls of different sizes."""
import ctypes as C

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


def noalloc(qs, st, u):
    """Direct C-ABI call of qs_sample_noalloc; returns (status, indices)."""
    uu = np.ascontiguousarray(u, dtype=np.float64)
    out = np.full(uu.size, np.iinfo(np.uint64).max, dtype=np.uint64)
    rc = qs._lib.lib().qs_sample_noalloc(st.h, uu.ctypes.data_as(C.POINTER(C.c_double)), uu.size,
                                         out.ctypes.data_as(C.POINTER(C.c_uint64)))
    return rc, out


def state(qs, n, dtype, seed, zero_blocks=False):
    psi = W.gaussian_state(n, seed)
    if zero_blocks:  # runs without mass: draws must skip them
        psi[: len(psi) // 3] = 0.0
        psi[len(psi) // 2: len(psi) // 2 + 4096] = 0.0
        psi /= np.linalg.norm(psi)
    st = qs.State(n, dtype, init=None)
    st.upload(psi.astype(np.complex64 if dtype == "c64" else np.complex128))
    return st


def test_noalloc_sampling_equals_sample_on_consecutive_calls(qs):
    # the second call is smaller (fewer qubits, fewer draws) and reuses the
    # scratch the first one filled; the first state is then sampled again
    cases = [(22, "c64", 20000, 1, True), (12, "c128", 300, 2, False), (7, "c64", 64, 3, False)]
    states = [state(qs, n, dt, seed, zb) for n, dt, _, seed, zb in cases]
    for (n, dt, count, seed, _), st in list(zip(cases, states)) + [(cases[0], states[0])]:
        u = np.random.default_rng(100 + seed).random(count)
        u[:3] = (0.0, 0.5, np.nextafter(1.0, 0.0))
        rc, got = noalloc(qs, st, u)
        assert rc == 0, qs._lib.lib().qs_last_error()
        ref = qs.sample(st, u)
        assert np.array_equal(got, ref), (n, dt, count, int(np.sum(got != ref)))
        assert np.all(got < (1 << n))


def test_noalloc_limits_are_errors_before_any_work(qs):
    big = qs.State(27, "c64", init="zero")
    rc, out = noalloc(qs, big, np.array([0.5]))
    assert rc == qs._lib.QS_EINVAL and b"26 qubits" in qs._lib.lib().qs_last_error()
    assert out[0] == np.iinfo(np.uint64).max
    del big
    st = state(qs, 10, "c64", 4)
    rc, out = noalloc(qs, st, np.full(65537, 0.25))
    assert rc == qs._lib.QS_EINVAL and b"65536" in qs._lib.lib().qs_last_error()
    rc, out = noalloc(qs, st, np.array([0.25, 1.0]))
    assert rc == qs._lib.QS_EINVAL
    # the largest allowed request still works
    rc, out = noalloc(qs, st, np.linspace(0.0, 0.999, 65536))
    assert rc == 0 and np.array_equal(out, qs.sample(st, np.linspace(0.0, 0.999, 65536)))
