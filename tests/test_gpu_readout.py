"""Read-out: inverse-CDF shot sampling and marginal distributions on the
device against the oracle (``oracle/readout.py``).

Sampling is a decision taken from floating-point sums, so both sides read
the same amplitudes (the seeded input rounded to the state's dtype) and
compare indices exactly; a differing index is accepted only when u ||psi||^2
lies within 1e-12 ||psi||^2 of the cumulative-mass boundary that separates
the two answers (the device sums in a blocked order, the oracle in index
order), and it must still carry mass.  Marginals are FP64 sums and match to
1e-12 relative.  Where the state itself comes from a circuit on the device,
its cumulative masses and marginals can differ from the exact ones by at most
sum |p - p'| <= ||psi - psi'|| (||psi|| + ||psi'||), i.e. 2e-5 at the complex64
state bar (relative L2 error 1e-5) and 2e-12 at the complex128 bar.  At 30
qubits: a sparse state (the oracle samples its
nonzero entries exactly), a product state whose cumulative mass below any
index has a closed form, and GHZ.
"""
import math

import numpy as np
import pytest

import workloads as W
from oracle import readout

pytestmark = pytest.mark.gpu

N30 = 30


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


def uniforms(seed, count):
    u = np.random.default_rng(seed).random(count)
    return np.concatenate([u, [0.0, np.nextafter(1.0, 0.0), 0.5]])


def upload(qs, psi, dtype):
    nd = np.complex64 if dtype == "c64" else np.complex128
    held = psi.astype(nd)
    n = int(round(math.log2(psi.size)))
    st = qs.State(n, dtype, init=None)
    st.upload(held)
    return st, held.astype(np.complex128)


def check_samples(got, psi, u):
    ref = readout.inverse_cdf_sample(psi, u)
    C = readout.cumulative_mass(psi)
    T = C[-1]
    p = np.abs(psi) ** 2
    bad = np.nonzero(got != ref)[0]
    assert bad.size <= max(2, u.size // 100), bad.size
    for j in bad:
        d = int(got[j])
        t = u[j] * T
        lo = C[d - 1] if d > 0 else 0.0
        assert p[d] > 0.0, (j, d)
        assert lo - 1e-12 * T <= t <= C[d] + 1e-12 * T, (j, d, int(ref[j]))


@pytest.mark.parametrize("dtype", ["c64", "c128"])
@pytest.mark.parametrize("n", [1, 3, 5, 6, 7, 13, 14, 15, 19])
def test_sample_matches_oracle(qs, n, dtype):
    psi = W.gaussian_state(n, 40 + n)
    st, held = upload(qs, psi, dtype)
    u = uniforms(n, 4096)
    got = qs.sample(st, u)
    assert got.dtype == np.uint64 and got.shape == u.shape
    check_samples(got, held, u)


@pytest.mark.parametrize("dtype", ["c64", "c128"])
def test_sample_zero_mass_regions_and_unnormalised(qs, dtype):
    """Whole 2^14-amplitude blocks and 64-amplitude sub-blocks without mass,
    isolated zeros, and a state of norm 9: zero-mass indices are never drawn."""
    n = 17
    psi = 3.0 * W.gaussian_state(n, 2)
    psi[: 3 << 14] = 0              # three empty blocks in front
    psi[5 << 14: 7 << 14] = 0       # two empty blocks in the middle
    psi[-(1 << 14):] = 0            # the last block empty
    psi[(8 << 14) + 64: (8 << 14) + 640] = 0
    psi[(9 << 14)::3] = 0
    st, held = upload(qs, psi, dtype)
    u = uniforms(7, 8192)
    got = qs.sample(st, u)
    assert np.all(np.abs(held[got.astype(np.int64)]) > 0)
    check_samples(got, held, u)


@pytest.mark.parametrize("dtype", ["c64", "c128"])
def test_sample_basis_state_and_empty_request(qs, dtype):
    n = 16
    st = qs.State(n, dtype)
    st.set_basis(12345)
    assert np.all(qs.sample(st, uniforms(3, 1000)) == 12345)
    assert qs.sample(st, []).size == 0


def test_sample_rejects_bad_input(qs):
    st = qs.State(6, "c64")
    with pytest.raises(Exception):
        qs.sample(st, [0.5, 1.0])
    with pytest.raises(Exception):
        qs.sample(st, [-0.1])
    with pytest.raises(Exception):
        qs.sample(st, [float("nan")])
    z = qs.State(6, "c64", init=None)
    z.tensor().zero_()
    with pytest.raises(Exception):
        qs.sample(z, [0.5])


@pytest.mark.parametrize("dtype", ["c64", "c128"])
@pytest.mark.parametrize("n,qubits", [(1, [0]), (5, [0, 4]), (8, [3]), (12, [11, 0, 5]),
                                      (15, list(range(15))), (16, [2, 3, 7, 9, 14]),
                                      (18, [0, 1, 2, 3, 4, 5, 6, 7, 8, 9, 10, 11, 12, 13, 14, 17]),
                                      (9, [])])
def test_marginal_matches_oracle(qs, n, qubits, dtype):
    psi = 1.7 * W.gaussian_state(n, 60 + n)
    st, held = upload(qs, psi, dtype)
    got = qs.marginal(st, qubits)
    ref = readout.marginal(held, n, qubits)
    assert got.shape == ref.shape
    assert np.allclose(got, ref, rtol=1e-12, atol=1e-15 * float(np.sum(ref))), np.max(np.abs(got - ref))


def test_marginal_rejects_bad_input(qs):
    st = qs.State(20, "c64")
    with pytest.raises(Exception):
        qs.marginal(st, list(range(17)))
    with pytest.raises(Exception):
        qs.marginal(st, [20])


# ---------------------------------------------------------------- 30 qubits
@pytest.mark.parametrize("dtype", ["c64", "c128"])
def test_sample_sparse_30q(qs, dtype):
    """Eight nonzero amplitudes among 2^30: the inverse CDF over the whole
    state equals the inverse CDF over the nonzero entries in index order."""
    import torch
    idx, c = W.sparse_state(N30, 21, 8)
    nd = np.complex64 if dtype == "c64" else np.complex128
    c = c.astype(nd).astype(np.complex128)
    order = np.argsort(idx)
    idx, c = idx[order], c[order]
    st = qs.State(N30, dtype, init=None, lazy_scratch=True)
    t = st.tensor()
    t.zero_()
    t[torch.as_tensor(idx.astype(np.int64), device="cuda")] = torch.as_tensor(c.astype(nd), device="cuda")
    u = uniforms(5, 20000)
    got = qs.sample(st, u)
    pos = np.searchsorted(idx, got)
    assert np.all(idx[np.minimum(pos, idx.size - 1)] == got)
    check_samples(pos.astype(np.uint64), c, u)
    # marginal over the top four qubits: the nonzero entries binned by their top bits
    m = qs.marginal(st, [0, 1, 2, 3])
    ref = np.zeros(16)
    np.add.at(ref, (idx >> np.uint64(N30 - 4)).astype(np.int64), np.abs(c) ** 2)
    assert np.allclose(m, ref, rtol=1e-12, atol=1e-15)


def product_cdf(theta, d):
    """For RY(theta_q) on each qubit of |0...0>: the mass of all indices
    below d and the mass of d itself (qubit 0 the most significant bit)."""
    n = len(theta)
    p1 = np.sin(np.asarray(theta) / 2) ** 2
    below, pref = 0.0, 1.0
    for q in range(n):
        bit = (int(d) >> (n - 1 - q)) & 1
        if bit:
            below += pref * (1.0 - p1[q])
            pref *= p1[q]
        else:
            pref *= 1.0 - p1[q]
    return below, pref


@pytest.mark.parametrize("dtype", ["c64", "c128"])
def test_sample_and_marginal_product_state_30q(qs, dtype):
    rng = np.random.default_rng(8)
    theta = rng.uniform(0.2, math.pi - 0.2, size=N30)
    st = qs.State(N30, dtype)
    qs.apply(st, qs.Plan(N30, [W.G("RY", q, theta=float(theta[q])) for q in range(N30)]))
    u = uniforms(9, 4000)
    got = qs.sample(st, u)
    tol = 2e-5 if dtype == "c64" else 2e-12
    for j in range(u.size):
        lo, pd = product_cdf(theta, got[j])
        assert pd > 0
        assert lo - tol <= u[j] <= lo + pd + tol, (j, int(got[j]))
    p1 = np.sin(theta / 2) ** 2
    for qubits in ([0], [29], [3, 17], [0, 5, 10, 15, 20, 25, 29], list(range(4, 20))):
        ref = np.ones(1)
        for q in qubits:
            ref = np.kron(ref, [1 - p1[q], p1[q]])
        got_m = qs.marginal(st, qubits)
        assert np.max(np.abs(got_m - ref)) <= tol, np.max(np.abs(got_m - ref))


def test_sample_ghz_30q(qs):
    st = qs.State(N30, "c64")
    qs.apply(st, qs.Plan(N30, W.ghz_stream(N30)))
    u = uniforms(4, 2000)
    got = qs.sample(st, u)
    away = np.abs(u - 0.5) > 2e-5
    assert np.all(got[away & (u < 0.5)] == 0)
    assert np.all(got[away & (u > 0.5)] == (1 << N30) - 1)
    m = qs.marginal(st, [0, 29])
    assert np.allclose(m, [0.5, 0, 0, 0.5], atol=2e-5)
