"""MI355X structured-layer state-vector library: Python binding of libqs.

States live in device memory owned by PyTorch (complex64 / complex128
tensors); every gate, layer, reduction and gradient runs in the library's HIP
kernels.  This module only marshals arguments.

    import paper_2609_19147_amd as qs
    st = qs.State(25)                 # complex64, |0...0>
    plan = qs.Plan(25, gates)         # fused layer plan (host only)
    qs.apply(st, plan)
    e = qs.expect(st, terms)
"""
from __future__ import annotations

import ctypes as C
import json
import weakref
from typing import List, Optional, Sequence

import numpy as np

from . import _lib
from ._lib import QsError, QsGate, QsPauli, QsPlanOpts, check, lib
from . import qasm  # noqa: E402  (OpenQASM 2.0 import; host only)

__all__ = ["State", "StateView", "Batch", "Plan", "apply", "apply_graph", "apply_norm2", "apply_gates", "expect", "norm2", "overlap", "infidelity",
           "amplitudes", "qasm", "to_c_gates", "to_c_terms", "profile", "QsError", "version", "adjoint_grad",
           "energy_function"]


def version() -> str:
    return lib().qs_version().decode()


def memory_info():
    """(bytes held in library-allocated amplitude buffers, QS_MAX_BYTES cap or 0)."""
    held, cap = C.c_size_t(), C.c_size_t()
    check(lib().qs_memory_info(C.byref(held), C.byref(cap)))
    return held.value, cap.value


# ------------------------------------------------------------------ marshalling
class CGates:
    """A C array of qs_gate plus the matrix buffers it points into."""

    def __init__(self, gates):
        self.n = len(gates)
        self.arr = (QsGate * max(1, self.n))()
        self._keep = []
        for i, g in enumerate(gates):
            cg = self.arr[i]
            cg.kind = _lib.KIND[g.name]
            cg.param = int(g.param)
            cg.theta = float(g.theta)
            cg.scale = float(g.scale)
            if g.name in ("MCZ", "MCP"):
                cg.nw = 0
                cg.mask = sum(1 << int(w) for w in g.wires)
            else:
                cg.nw = len(g.wires)
                for j, w in enumerate(g.wires):
                    cg.wires[j] = int(w)
            if g.mat is not None:
                m = np.asarray(g.mat, dtype=np.complex128).ravel()
                buf = (C.c_double * (2 * m.size))(*np.stack([m.real, m.imag], axis=1).ravel())
                self._keep.append(buf)
                cg.mat = C.cast(buf, C.POINTER(C.c_double))


def to_c_gates(gates) -> CGates:
    return CGates(list(gates))


def to_c_terms(terms):
    arr = (QsPauli * max(1, len(terms)))()
    for i, (c, xm, zm) in enumerate(terms):
        arr[i].coeff = float(c)
        arr[i].x_mask = int(xm)
        arr[i].z_mask = int(zm)
    return arr


def _dbl(v):
    v = np.ascontiguousarray(np.asarray(v, dtype=np.float64))
    return v, v.ctypes.data_as(C.POINTER(C.c_double))


# ------------------------------------------------------------------ states
class State:
    """A 2^n amplitude state on the current HIP device.

    Memory is two torch tensors (the state and the permutation ping-pong
    buffer) borrowed by the library; ``tensor()`` returns the current one.
    """

    def __init__(self, n: int, dtype: str = "c64", init: Optional[str] = "zero", stream=None,
                 lazy_scratch: bool = False):
        import torch
        self.n = int(n)
        self.dtype = dtype
        tdt = torch.complex64 if dtype == "c64" else torch.complex128
        self._bufs = [torch.empty(1 << self.n, dtype=tdt, device="cuda")]
        if not lazy_scratch:
            self._bufs.append(torch.empty(1 << self.n, dtype=tdt, device="cuda"))
        if stream is None:
            stream = torch.cuda.current_stream()
        self._stream = stream
        h = C.c_void_p()
        nbytes = self._bufs[0].numel() * self._bufs[0].element_size()
        check(lib().qs_alloc(self.n, _lib.QS_C64 if dtype == "c64" else _lib.QS_C128,
                             C.c_void_p(self._bufs[0].data_ptr()),
                             C.c_void_p(self._bufs[1].data_ptr()) if len(self._bufs) > 1 else None,
                             nbytes, C.c_void_p(stream.cuda_stream), C.byref(h)))
        self.h = h
        if init == "zero":
            self.set_basis(0)
        elif init == "plus":
            self.set_uniform()

    def __del__(self):
        h = getattr(self, "h", None)
        L = getattr(_lib, "_lib", None) if _lib is not None else None
        if h is not None and h.value and L is not None:
            L.qs_free(h)
            self.h = None

    # -- initialisation
    def set_basis(self, index: int) -> "State":
        check(lib().qs_set_basis(self.h, C.c_uint64(int(index))))
        return self

    def set_uniform(self) -> "State":
        check(lib().qs_set_uniform(self.h))
        return self

    def upload(self, host: np.ndarray) -> "State":
        nd = np.complex64 if self.dtype == "c64" else np.complex128
        a = np.ascontiguousarray(np.asarray(host, dtype=nd))
        if a.size != (1 << self.n):
            raise ValueError("host state must have 2^n amplitudes")
        check(lib().qs_upload(self.h, a.ctypes.data_as(C.c_void_p), a.nbytes))
        return self

    def download(self) -> np.ndarray:
        nd = np.complex64 if self.dtype == "c64" else np.complex128
        a = np.empty(1 << self.n, dtype=nd)
        check(lib().qs_download(self.h, a.ctypes.data_as(C.c_void_p), a.nbytes))
        return a

    def copy_from(self, other: "State") -> "State":
        check(lib().qs_copy(self.h, other.h))
        return self

    def tensor(self):
        """The torch tensor currently holding the amplitudes."""
        cur = C.c_void_p()
        check(lib().qs_state_buffers(self.h, C.byref(cur), None))
        for b in self._bufs:
            if b.data_ptr() == cur.value:
                return b
        raise RuntimeError("current buffer is not a torch tensor of this state")

    def sync(self) -> None:
        check(lib().qs_sync(self.h))


class StateView:
    """A state owned by a Batch (no torch tensor; read it with download())."""

    def __init__(self, handle, n, dtype, owner):
        self.h = handle
        self.n = n
        self.dtype = dtype
        self._owner = owner

    download = State.download
    upload = State.upload


class Batch:
    """Many circuits in one device arena, run as one recorded HIP graph."""

    def __init__(self, plans, init: str = "plus", dtype: str = "c64", stream=None):
        import torch
        self.plans = list(plans)
        self.n = [p.n for p in self.plans]
        self.dtype = dtype
        nq = (C.c_int * len(self.plans))(*self.n)
        ph = (C.c_void_p * len(self.plans))(*[p.h.value for p in self.plans])
        if stream is None:
            stream = torch.cuda.current_stream()
        self._stream = stream
        h = C.c_void_p()
        check(lib().qs_batch_create(len(self.plans), nq, ph, 1 if init == "plus" else 0,
                                    _lib.QS_C64 if dtype == "c64" else _lib.QS_C128,
                                    C.c_void_p(stream.cuda_stream), C.byref(h)))
        self.h = h

    def __del__(self):
        h = getattr(self, "h", None)
        L = getattr(_lib, "_lib", None) if _lib is not None else None
        if h is not None and h.value and L is not None:
            L.qs_batch_free(h)
            self.h = None

    def refresh(self) -> None:
        check(lib().qs_batch_refresh(self.h))

    def run(self) -> None:
        check(lib().qs_batch_run(self.h))

    def _expect(self, fn, observables) -> np.ndarray:
        arrs = [to_c_terms(o) for o in observables]
        ptrs = (C.POINTER(QsPauli) * len(arrs))(*[C.cast(a, C.POINTER(QsPauli)) for a in arrs])
        cnt = (C.c_size_t * len(arrs))(*[len(o) for o in observables])
        out = np.zeros(len(arrs))
        check(fn(self.h, ptrs, cnt, out.ctypes.data_as(C.POINTER(C.c_double))))
        return out

    def expect_diag(self, observables) -> np.ndarray:
        """Per-instance expectation of Z-type Pauli sums (one batched reduction)."""
        return self._expect(lib().qs_batch_expect_diag, observables)

    def expect(self, observables) -> np.ndarray:
        """Per-instance expectation of any Pauli sums (X / Y terms per instance)."""
        return self._expect(lib().qs_batch_expect, observables)

    def set_observables(self, observables) -> None:
        """Store Z-type Pauli sums (one per instance) on the device once."""
        arrs = [to_c_terms(o) for o in observables]
        ptrs = (C.POINTER(QsPauli) * len(arrs))(*[C.cast(a, C.POINTER(QsPauli)) for a in arrs])
        cnt = (C.c_size_t * len(arrs))(*[len(o) for o in observables])
        check(lib().qs_batch_set_observables(self.h, ptrs, cnt))

    def expect_stored(self) -> np.ndarray:
        """Per-instance expectation of the stored observables (one batched reduction)."""
        out = np.zeros(len(self.n))
        check(lib().qs_batch_expect_stored(self.h, out.ctypes.data_as(C.POINTER(C.c_double))))
        return out

    def state(self, i: int) -> StateView:
        v = C.c_void_p()
        check(lib().qs_batch_state(self.h, i, C.byref(v)))
        return StateView(v, self.n[i], self.dtype, self)


# ------------------------------------------------------------------ plans
class Plan:
    """A fused (or plain) layer plan of a gate stream, built on the host."""

    def __init__(self, n: int, gates, n_params: int = 0, mode: str = "fused", max_tile_bits: int = 0,
                 params=None, dense_k_max: int = 0, window_k: int = 0, low_bits: int = 0,
                 coset_order: int = 0, diag_low_bits: int = 0, balance_passes: int = 0):
        self.n = int(n)
        self.gates = list(gates)
        self.n_params = int(n_params)
        cg = CGates(self.gates)
        opts = QsPlanOpts(_lib.QS_FUSED if mode == "fused" else _lib.QS_PLAIN, int(max_tile_bits),
                          int(dense_k_max), int(window_k), int(low_bits), int(coset_order),
                          int(diag_low_bits), int(balance_passes))
        h = C.c_void_p()
        check(lib().qs_plan_create(self.n, cg.arr, cg.n, self.n_params, C.byref(opts), C.byref(h)))
        self.h = h
        if params is not None:
            self.set_params(params)

    def __del__(self):
        h = getattr(self, "h", None)
        L = getattr(_lib, "_lib", None) if _lib is not None else None
        if h is not None and h.value and L is not None:
            L.qs_plan_free(h)
            self.h = None

    def set_params(self, params) -> "Plan":
        v, p = _dbl(params)
        check(lib().qs_plan_set_params(self.h, p, v.size))
        return self

    def num_layers(self) -> int:
        out = C.c_size_t()
        check(lib().qs_plan_num_layers(self.h, C.byref(out)))
        return out.value

    def inverse(self) -> "Plan":
        """Plan of the inverse circuit (shares the current parameter values)."""
        h = C.c_void_p()
        check(lib().qs_plan_inverse(self.h, C.byref(h)))
        q = Plan.__new__(Plan)
        q.n, q.gates, q.n_params, q.h = self.n, self.gates, self.n_params, h
        return q

    def describe(self) -> dict:
        need = C.c_size_t()
        check(lib().qs_plan_describe(self.h, None, 0, C.byref(need)))
        buf = C.create_string_buffer(need.value)
        check(lib().qs_plan_describe(self.h, buf, need.value, C.byref(need)))
        return json.loads(buf.value.decode())


# ------------------------------------------------------------------ operations
def apply(state: State, plan: Plan, first: int = 0, count: int = -1) -> None:
    cnt = C.c_size_t(-1 & ((1 << 64) - 1)) if count < 0 else C.c_size_t(count)
    check(lib().qs_apply_layer(state.h, plan.h, first, cnt))


def apply_gates(state: State, gates, params=None) -> None:
    cg = CGates(list(gates))
    if params is None:
        check(lib().qs_apply_gates(state.h, cg.arr, cg.n, None, 0))
    else:
        v, p = _dbl(params)
        check(lib().qs_apply_gates(state.h, cg.arr, cg.n, p, v.size))


def expect(state: State, terms, per_term: bool = False):
    arr = to_c_terms(terms)
    out = np.zeros(len(terms))
    tot = C.c_double()
    check(lib().qs_expect(state.h, arr, len(terms), out.ctypes.data_as(C.POINTER(C.c_double)), C.byref(tot)))
    return (tot.value, out) if per_term else tot.value


def apply_graph(state: State, plan: Plan) -> None:
    """Apply the whole plan as one recorded HIP graph (recorded on first use
    for this state, plan and parameter values; replayed afterwards)."""
    check(lib().qs_apply_graph(state.h, plan.h))


def apply_norm2(state: State, plan: Plan) -> float:
    """Apply the whole plan and return ||psi||^2 of the result (FP64); the last
    layer's kernel accumulates it when it is a tile pass or a gather."""
    out = C.c_double()
    check(lib().qs_apply_norm2(state.h, plan.h, C.byref(out)))
    return out.value


def norm2(state: State) -> float:
    out = C.c_double()
    check(lib().qs_norm2(state.h, C.byref(out)))
    return out.value


def overlap(a: State, b: State) -> complex:
    out = (C.c_double * 2)()
    check(lib().qs_overlap(a.h, b.h, out))
    return complex(out[0], out[1])


def infidelity(a: State, b: State) -> float:
    out = C.c_double()
    check(lib().qs_infidelity(a.h, b.h, C.byref(out)))
    return out.value


def amplitudes(state: State, idx) -> np.ndarray:
    idx = np.ascontiguousarray(np.asarray(idx, dtype=np.uint64))
    nd = np.complex64 if state.dtype == "c64" else np.complex128
    out = np.empty(idx.size, dtype=nd)
    check(lib().qs_amplitudes(state.h, idx.ctypes.data_as(C.POINTER(C.c_uint64)), idx.size,
                              out.ctypes.data_as(C.c_void_p)))
    return out


def sample(state: State, u) -> np.ndarray:
    """Indices drawn from |psi_i|^2 / ||psi||^2 for the uniform numbers u in [0, 1)
    (one draw each; the library takes the first index whose cumulative mass
    exceeds u ||psi||^2)."""
    uu = np.ascontiguousarray(np.asarray(u, dtype=np.float64).ravel())
    out = np.empty(uu.size, dtype=np.uint64)
    if uu.size:
        check(lib().qs_sample(state.h, uu.ctypes.data_as(C.POINTER(C.c_double)), uu.size,
                              out.ctypes.data_as(C.POINTER(C.c_uint64))))
    return out


def sample_noalloc(state: State, u) -> np.ndarray:
    """As sample(), through the allocation-free entry point (static device
    scratch; at most 26 qubits and 65536 draws per call)."""
    uu = np.ascontiguousarray(np.asarray(u, dtype=np.float64).ravel())
    out = np.empty(uu.size, dtype=np.uint64)
    if uu.size:
        check(lib().qs_sample_noalloc(state.h, uu.ctypes.data_as(C.POINTER(C.c_double)), uu.size,
                                      out.ctypes.data_as(C.POINTER(C.c_uint64))))
    return out


def marginal(state: State, qubits) -> np.ndarray:
    """Unnormalised marginal over the given qubits (at most 16): 2^k FP64 sums,
    the lowest-numbered qubit most significant in the bin index."""
    mask = 0
    for q in qubits:
        mask |= 1 << int(q)
    k = bin(mask).count("1")
    out = np.zeros(1 << k)
    check(lib().qs_marginal(state.h, C.c_uint64(mask), out.ctypes.data_as(C.POINTER(C.c_double))))
    return out


def adjoint_grad(state: State, plan: Plan, terms):
    """Energy <psi_L|H|psi_L> and its gradient w.r.t. the plan's parameters by
    the adjoint method; ``state`` holds psi_0 on entry and psi_L on return."""
    arr = to_c_terms(terms)
    e = C.c_double()
    g = np.zeros(plan.n_params)
    check(lib().qs_adjoint_grad(state.h, plan.h, arr, len(terms), C.byref(e),
                                g.ctypes.data_as(C.POINTER(C.c_double)), plan.n_params))
    return e.value, g


# One state per (plan, dtype) for energy_function: made on the first forward
# and reset to |0...0> on every later one, so that repeated evaluations (an
# optimisation loop) allocate no device memory; it lives as long as the plan.
_energy_states = weakref.WeakKeyDictionary()


def _energy_state(plan: Plan, dtype: str) -> State:
    per = _energy_states.get(plan)
    if per is None:
        per = _energy_states[plan] = {}
    st = per.get(dtype)
    if st is None:
        st = per[dtype] = State(plan.n, dtype, init=None)
    return st.set_basis(0)


def energy_function():
    """torch.autograd.Function computing E(params) = <psi(params)|H|psi(params)>
    from |0...0> with the adjoint backward of the library.  The gradient is
    computed in the forward call only when ``params`` requires one; it has the
    shape of ``params``."""
    import torch

    class QsEnergy(torch.autograd.Function):
        @staticmethod
        def forward(ctx, params, plan, terms, dtype="c64"):
            p = params.detach().to("cpu", torch.float64).numpy().ravel()
            plan.set_params(p)
            st = _energy_state(plan, dtype)
            if ctx.needs_input_grad[0]:
                e, g = adjoint_grad(st, plan, terms)
                ctx.grad = torch.as_tensor(g.reshape(params.shape), dtype=params.dtype, device=params.device)
            else:
                apply(st, plan)
                e = expect(st, terms)
                ctx.grad = None
            return torch.tensor(e, dtype=params.dtype, device=params.device)

        @staticmethod
        def backward(ctx, grad_out):
            return grad_out * ctx.grad, None, None, None

    return QsEnergy


class profile:
    """Context manager: per-kernel HIP-event timings of the library's launches."""

    def __enter__(self):
        check(lib().qs_profile_reset())
        check(lib().qs_profile_enable(1))
        self.report: List[dict] = []
        return self

    def __exit__(self, *exc):
        check(lib().qs_profile_enable(0))
        need = C.c_size_t()
        check(lib().qs_profile_report(None, 0, C.byref(need)))
        buf = C.create_string_buffer(need.value)
        check(lib().qs_profile_report(buf, need.value, C.byref(need)))
        self.report = json.loads(buf.value.decode())
        return False
