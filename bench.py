"""Benchmark of the structured-layer state-vector path on one MI355X.

Workload (one step): a 30-qubit seeded Gaussian complex64 state, resident in
HBM, goes through the composed circuit QFT (465 gates) -> Walsh-Hadamard
layer (30 H) -> 200-gate random X/CNOT/SWAP block, planned by the fusion
planner (three tile passes and one GF(2) gather), followed by the FP64 norm
of the result.  The reported value is the achieved effective state-vector
bandwidth: passes used x 2 S per step (S = 8 * 2^30 bytes) divided by the
step time.  The library sums the norm inside the gather as it writes the
state (qs_apply_norm2), so the norm moves no bytes of its own; the figure
that counts it as a separate S-byte read is reported beside it.

The JSON line also carries the roofline of the dominant kernel (the tile
pass: HIP-event durations measured inside the timed region on the stream
the library launches on), the gate-stream-equivalent bandwidth, and the
CPU oracle timed on a bounded 23-qubit sample of the same circuit.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import workloads as W  # noqa: E402

HBM_PEAK_GBS = 8000.0
N_QUBITS = 30
STATE_SEED, BLOCK_SEED = 30, 31


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def t95(n):
    """Two-sided 95% Student-t quantile for n samples (n - 1 degrees of freedom)."""
    from scipy.stats import t as student_t
    return float(student_t.ppf(0.975, n - 1)) if n > 1 else float("nan")


def summary(xs, scale=1e3, nd=4):
    """Mean and t-based 95% half-width of repeated timings (seconds -> ms)."""
    a = np.asarray(xs, dtype=np.float64) * scale
    ci = t95(a.size) * a.std(ddof=1) / math.sqrt(a.size) if a.size > 1 else None
    return {"mean": round(float(a.mean()), nd), "ci95": None if ci is None else round(float(ci), nd),
            "n": int(a.size)}


def paired(arms, reps=10, warmup=2, ref=None):
    """Timing protocol: every arm runs `warmup` times, then `reps` repeats in
    which the arms run round-robin (interleaved, so drift hits all arms
    alike).  Each arm callable must return only once its device work is done.
    Returns per-arm {mean, ci95, n} in ms and, against the reference arm (the
    first unless named), the per-repeat paired ratios t_arm / t_ref as
    {mean, ci95}."""
    names = list(arms)
    ref = ref or names[0]
    for _ in range(warmup):
        for k in names:
            arms[k]()
    times = {k: [] for k in names}
    for _ in range(reps):
        for k in names:
            t0 = time.perf_counter()
            arms[k]()
            times[k].append(time.perf_counter() - t0)
    out = {k: summary(v) for k, v in times.items()}
    for k in names:
        if k != ref:
            r = np.asarray(times[k]) / np.asarray(times[ref])
            out[k]["ratio_vs_" + ref] = summary(r, scale=1.0, nd=3)
    return out


def speedup(T, arm, ref):
    """Paired speedup of ref over arm: mean of t_arm / t_ref with its 95% half-width."""
    r = T[arm]["ratio_vs_" + ref]
    return {"mean": round(r["mean"], 2), "ci95": r["ci95"]}


def circuit(n):
    return W.qft_stream(n) + W.wht_stream(n) + W.random_perm_block(n, 200, BLOCK_SEED)


def kernel_source_hash(kernel: str) -> str:
    files = {"tile_pass": ["k_tile.hip", "dev.h", "layout.h", "kernels.h"],
             "gf2_gather": ["k_stream.hip", "dev.h", "layout.h", "kernels.h"]}[kernel]
    h = hashlib.sha256()
    for f in files:
        with open(os.path.join(ROOT, "paper_2609_19147_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(kernel: str):
    """HBM bytes per launch from the committed rocprofv3 counter summary, or
    None when the kernel source changed since the counters were taken."""
    path = os.path.join(ROOT, "profiles", f"{kernel}_30q_counters.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        d = json.load(fh)
    if d.get("source_hash") != kernel_source_hash(kernel):
        return None
    return d.get("hbm_bytes_per_launch")


def streaming_ceiling(n=N_QUBITS, timeout=240):
    """The device's achievable streaming rates from the library's standalone
    probe (built beside libqs.so): hipMemcpyAsync, streaming copies, read- and
    write-only streams, and the tile passes' access patterns with and without
    butterfly rounds, per geometry and coset order (2 S per pass)."""
    import subprocess
    exe = os.path.join(ROOT, "paper_2609_19147_amd", "ceiling_probe")
    if not os.path.exists(exe):
        return {"error": "ceiling_probe not built"}
    r = subprocess.run([exe, str(n)], capture_output=True, text=True, timeout=timeout)
    rows = [json.loads(line) for line in r.stdout.splitlines() if line.startswith("{")]
    out = {"n_qubits": n, "returncode": r.returncode,
           "probes": {d["probe"]: {"ms": d["best_ms"], "GBs": d["GBs"]} for d in rows if "probe" in d}}
    copies = [v["GBs"] for k, v in out["probes"].items() if k.startswith("copy")]
    if copies:
        out["best_copy_GBs"] = max(copies)
        out["best_copy_frac"] = round(max(copies) / HBM_PEAK_GBS, 4)
    return out


def _pool_init():
    from threadpoolctl import threadpool_limits
    threadpool_limits(1)


def _qaoa_oracle(args):
    """One QAOA instance on the oracle: its expected cut (for the process pool)."""
    from oracle import statevec as sv
    n, edges, gammas, betas = args
    inst = W.QaoaInstance(n, edges, np.asarray(gammas), np.asarray(betas))
    psi = sv.run(sv.plus(n), n, W.qaoa_stream(inst, h_layer=False))
    return sv.expect(psi, n, W.maxcut_terms(edges))


def oracle_timings():
    """The oracle on the host cores beside the GPU arms, on bounded samples:
    the 12-qubit QFT stream; a seeded subset of the 512-instance QAOA batch
    (the first 16 instances of 16 qubits and 2 of 18) on one core and over
    all available cores with a process pool (workers started and warmed
    before the timing); and the 12-qubit, 8-layer ansatz's
    parameter-shift and central finite-difference gradients (385 + 384
    energy evaluations of 280 gates).  BLAS threads pinned to one."""
    import multiprocessing as mp
    from threadpoolctl import threadpool_limits
    from oracle import gradients, statevec as sv
    cores = len(os.sched_getaffinity(0))
    out = {"cores_available": cores}
    with threadpool_limits(1):
        psi = W.gaussian_state(12, 12)
        stream = W.qft_stream(12)
        t0 = time.perf_counter()
        for _ in range(5):
            sv.run(psi, 12, stream)
        out["qft_12q"] = {"gates": len(stream), "ms": round(1e3 * (time.perf_counter() - t0) / 5, 2), "cores": 1}
        insts = W.qaoa_instances(512, 512, depth=4)
        sub = [i for i in insts if i.n == 16][:16] + [i for i in insts if i.n == 18][:2]
        args = [(i.n, i.edges, i.gammas.tolist(), i.betas.tolist()) for i in sub]
        t0 = time.perf_counter()
        for a in args:
            _qaoa_oracle(a)
        t1 = time.perf_counter() - t0
        out["qaoa_subset_1_core"] = {"instances": len(sub), "n_qubits": "16 x 16, 2 x 18", "s": round(t1, 2),
                                     "instances_per_s": round(len(sub) / t1, 3), "cores": 1}
    ctx = mp.get_context("spawn")
    workers = min(cores, len(args))
    with ctx.Pool(workers, initializer=_pool_init) as pool:
        pool.map(_qaoa_oracle, args[:workers])  # workers started and imports done
        t0 = time.perf_counter()
        pool.map(_qaoa_oracle, args, chunksize=1)
        t2 = time.perf_counter() - t0
    out["qaoa_subset_all_cores"] = {"instances": len(sub), "s": round(t2, 2), "instances_per_s": round(len(sub) / t2, 3),
                                    "cores": workers, "pool": "spawn, one BLAS thread per worker"}
    with threadpool_limits(1):
        n, layers = 12, 8
        hs = W.hea_stream(n, layers)
        prm = W.hea_params(n, layers, 24)
        terms = W.xxz_terms(n, 0.5)
        t0 = time.perf_counter()
        gradients.parameter_shift(n, hs, prm, terms)
        tps = time.perf_counter() - t0
        t0 = time.perf_counter()
        gradients.finite_differences(n, hs, prm, terms, h=1e-5)
        tfd = time.perf_counter() - t0
    out["adjoint_config_12q"] = {"params": len(prm), "gates": len(hs), "param_shift_s": round(tps, 2),
                                 "finite_differences_s": round(tfd, 2), "cores": 1}
    return out


def cpu_baseline(n=23, time_budget=25.0):
    """The oracle (one gate at a time, complex128 numpy) on a bounded sample:
    the same circuit at 23 qubits, single-threaded."""
    try:
        from threadpoolctl import threadpool_limits
    except ImportError:  # pragma: no cover
        threadpool_limits = None
    from oracle import statevec as sv
    stream = circuit(n)
    psi = W.gaussian_state(n, STATE_SEED)
    ctx = threadpool_limits(1) if threadpool_limits else None
    t0 = time.perf_counter()
    done = 0
    for g in stream:
        psi = sv.apply_gate(psi, n, g)
        done += 1
        if time.perf_counter() - t0 > time_budget:
            break
    float(np.vdot(psi, psi).real)  # the norm reduction
    dt = time.perf_counter() - t0
    if ctx is not None:
        ctx.__exit__(None, None, None)
    frac = done / len(stream)
    S = 16 * (1 << n)  # the oracle's complex128 state
    # same accounting as the GPU value: 4 fused-layer passes of 2 S each,
    # prorated when the time budget cut the sample short
    gbs = frac * (4 * 2 * S) / dt / 1e9
    return {"value": round(gbs, 3), "unit": "GB/s", "cores": 1, "kind": "oracle",
            "sample": f"{done}/{len(stream)} gates of the same circuit at {n} qubits "
                      f"(complex128 numpy, one gate at a time), {dt:.1f} s"}


def qaoa_tile_bits(n):
    """Two equal tile groups per QAOA instance: 2^((n+4)/2) amplitudes per tile."""
    return max(6, min(14, (n + 4) // 2))


def qaoa_plan(qs, inst, depth, opts):
    prm = np.empty(2 * depth)
    prm[0::2] = inst.gammas
    prm[1::2] = inst.betas
    return qs.Plan(inst.n, W.qaoa_stream(inst, param_offset=0, h_layer=False), n_params=2 * depth, params=prm,
                   **opts)


def qaoa_tuned_options(qs, insts, depth):
    """Plan options per qubit count (tile limit x low bits of the diagonal
    passes), tuned on a batch of 16 instances of that size and cached by the
    tuner: a later process on the same device reads the cache and runs
    nothing."""
    from paper_2609_19147_amd.tune import TileTuner, option_grid
    tuner = TileTuner()
    out = {}
    for n in sorted({i.n for i in insts}):
        sample = [i for i in insts if i.n == n][:16]
        built = {}

        def run(opts, sample=sample, built=built):
            key = tuple(sorted(opts.items()))
            if key not in built:
                built[key] = qs.Batch([qaoa_plan(qs, i, depth, opts) for i in sample], init="plus")
            built[key].run()

        tiles = range(max(8, qaoa_tile_bits(n) - 3), min(14, n - 2) + 1)
        out[n] = tuner.best_options(f"qaoa-maxcut-p{depth}-batched", n, "c64", run,
                                    option_grid(max_tile_bits=tiles, diag_low_bits=(0, -1)))
        del built
    return out


def bench_batched_qaoa(qs, torch, count=512, depth=4, seed=512, reps=10):
    """512 MaxCut QAOA instances (n uniform over 16..24 even, 3-regular graphs,
    p = 4, angles U[0, pi)) as one recorded graph launch + one batched FP64
    expectation, against the per-instance fused and plain per-gate paths
    (plain-mode plans built beforehand); the three arms interleaved in every
    repeat."""
    insts = W.qaoa_instances(count, seed, depth=depth)
    options = qaoa_tuned_options(qs, insts, depth)
    plans = [qaoa_plan(qs, inst, depth, options[inst.n]) for inst in insts]
    plain = [qs.Plan(inst.n, W.qaoa_stream(inst, h_layer=False), mode="plain") for inst in insts]
    obs = [W.maxcut_terms(inst.edges) for inst in insts]
    t0 = time.perf_counter()
    B = qs.Batch(plans, init="plus")
    t_record = time.perf_counter() - t0
    # the cost observables go to the device once (an optimisation loop re-runs
    # the batch with new angles and reads the same observables every time)
    B.set_observables(obs)
    pool = {n: qs.State(n, "c64", init=None, lazy_scratch=True) for n in sorted({i.n for i in insts})}
    res = {}

    def batched():
        B.run()
        res["batched"] = B.expect_stored()

    def per_instance(name, which):
        out = np.empty(count)
        for k, inst in enumerate(insts):
            st = pool[inst.n]
            st.set_uniform()
            qs.apply(st, which[k])
            out[k] = qs.expect(st, obs[k])
        res[name] = out

    T = paired({"batched": batched, "fused_per_instance": lambda: per_instance("fused", plans),
                "plain_per_instance": lambda: per_instance("plain", plain)}, reps=reps)
    # the same step with the observables passed (and converted) on every call
    t0 = time.perf_counter()
    B.run()
    c_percall = B.expect_diag(obs)
    t_percall = time.perf_counter() - t0
    assert np.array_equal(c_percall, res["batched"])
    norms = B.expect_diag([[(1.0, 0, 0)]] * count)
    del B, pool
    torch.cuda.empty_cache()
    ms = {k: T[k]["mean"] * 1e-3 for k in ("batched", "fused_per_instance", "plain_per_instance")}
    return {"instances": count, "n_qubits": "16-24 even", "depth": depth,
            "protocol": f"2 warmups, {reps} repeats, arms interleaved; mean and t-based 95% half-width",
            "instances_per_s": round(count / ms["batched"], 1),
            "plain_instances_per_s": round(count / ms["plain_per_instance"], 1),
            "fused_per_instance_instances_per_s": round(count / ms["fused_per_instance"], 1),
            "speedup_vs_plain": speedup(T, "plain_per_instance", "batched"),
            "speedup_vs_fused_per_instance": speedup(T, "fused_per_instance", "batched"),
            "ms": {k: {kk: vv for kk, vv in T[k].items() if not kk.startswith("ratio")}
                   for k in ("batched", "fused_per_instance", "plain_per_instance")},
            "ms_batch_observables_per_call": round(1e3 * t_percall, 2),
            "ms_record_graph": round(1e3 * t_record, 1),
            "max_abs_diff_vs_plain": float(np.max(np.abs(res["batched"] - res["plain"]))),
            "max_abs_diff_vs_fused": float(np.max(np.abs(res["batched"] - res["fused"]))),
            "max_norm_drift_batched": float(np.max(np.abs(norms - 1.0))),
            "mean_cut": round(float(np.mean(res["batched"])), 4),
            "options_by_n": {str(k): v for k, v in sorted(options.items())}}


def bench_adjoint(qs, torch, n=24, layers=8, seed=24, ps_sample=8, reps=10):
    """24-qubit hardware-efficient ansatz (384 parameters), XXZ energy: one
    adjoint forward + backward against GPU parameter shift (769 circuits; the
    fused and plain per-circuit paths are timed on a sample of shifted
    circuits, plain-mode plans built beforehand), arms interleaved."""
    from paper_2609_19147_amd.tune import TileTuner
    stream = W.hea_stream(n, layers)
    params = W.hea_params(n, layers, seed)
    terms = W.xxz_terms(n, 0.5)
    st = qs.State(n, "c64")
    # tile limit of the plan: measured once per device (untimed), like the
    # batched section's
    plans = {}

    def run(tb):
        if tb not in plans:
            plans[tb] = qs.Plan(n, stream, n_params=len(params), params=params, max_tile_bits=tb)
        st.set_basis(0)
        qs.adjoint_grad(st, plans[tb], terms)
    tile_bits = TileTuner().best(f"adjoint-hea{layers}-xxz", n, "c64", run, (11, 12, 13))
    plan = plans.get(tile_bits) or qs.Plan(n, stream, n_params=len(params), params=params, max_tile_bits=tile_bits)
    n_circ = 2 * len(params) + 1
    rng = np.random.default_rng(seed)
    idx = rng.choice(len(params), size=ps_sample // 2, replace=False)
    shifted = []
    for j in idx:
        for sgn in (1, -1):
            p2 = params.copy()
            p2[j] += sgn * 0.5 * math.pi
            shifted.append((int(j), sgn, p2))
    fused_ps = [qs.Plan(n, stream, n_params=len(params), params=p2, max_tile_bits=tile_bits) for _, _, p2 in shifted]
    plain_ps = [qs.Plan(n, stream, n_params=len(params), params=p2, mode="plain") for _, _, p2 in shifted]
    out = {}

    def adjoint():
        st.set_basis(0)
        out["adj"] = qs.adjoint_grad(st, plan, terms)

    def ps(name, which):
        vals = []
        for pl in which:
            st.set_basis(0)
            qs.apply(st, pl)
            vals.append(qs.expect(st, terms))
        out[name] = vals

    T = paired({"adjoint": adjoint, "param_shift_fused": lambda: ps("fused", fused_ps),
                "param_shift_plain": lambda: ps("plain", plain_ps)}, reps=reps)
    e, g = out["adj"]
    t_adj = T["adjoint"]["mean"] * 1e-3
    per_fused = T["param_shift_fused"]["mean"] * 1e-3 / len(shifted)
    per_plain = T["param_shift_plain"]["mean"] * 1e-3 / len(shifted)
    diff = max(abs(g[j] - 0.5 * (out["fused"][2 * k] - out["fused"][2 * k + 1])) for k, j in enumerate(idx))
    diff_plain = max(abs(g[j] - 0.5 * (out["plain"][2 * k] - out["plain"][2 * k + 1])) for k, j in enumerate(idx))
    return {"n_qubits": n, "params": len(params), "terms": len(terms), "energy": e,
            "protocol": f"2 warmups, {reps} repeats, arms interleaved; mean and t-based 95% half-width",
            "max_tile_bits": tile_bits, "ms_adjoint": T["adjoint"],
            "equiv_circuits_per_s": round(n_circ / t_adj, 1),
            "plain_circuits_per_s": round(1.0 / per_plain, 2),
            "fused_circuits_per_s": round(1.0 / per_fused, 2),
            "speedup_vs_plain_param_shift": round(n_circ * per_plain / t_adj, 1),
            "speedup_vs_fused_param_shift": round(n_circ * per_fused / t_adj, 1),
            "max_abs_diff_vs_param_shift_sample": float(diff),
            "max_abs_diff_vs_plain_param_shift_sample": float(diff_plain),
            "param_shift_sample": f"{len(shifted)} shifted circuits ({len(idx)} parameters) on each path, "
                                  f"scaled to {n_circ} circuits"}


def bench_precision(qs, torch, n=N_QUBITS, reps=10):
    """The composed 30-qubit circuit in complex128 on the GPU beside complex64
    from the same input (the complex128 Gaussian state rounded once): time and
    effective GB/s of each, the complex64 result's infidelity against the
    complex128 one, and its norm drift (FP64 reductions)."""
    from paper_2609_19147_amd.tune import TileTuner
    stream = circuit(n)
    plans = {13: qs.Plan(n, stream)}
    s128 = qs.State(n, "c128", init=None)
    W.gaussian_state_torch(n, STATE_SEED, "c128", out=s128.tensor())
    s64 = qs.State(n, "c64", init=None)
    src = qs.State(n, "c128", init=None, lazy_scratch=True)
    src.copy_from(s128)

    # complex128 tiles of 2^13 amplitudes fill a CU's LDS (one workgroup per
    # CU): the tile limit for complex128 is measured (untimed), as elsewhere
    def run128(tb):
        if tb not in plans:
            plans[tb] = qs.Plan(n, stream, max_tile_bits=tb)
        qs.apply(s128, plans[tb])
    tb128 = TileTuner().best("composed-circuit", n, "c128", run128, (11, 12, 13))
    out = {"max_tile_bits_c64": 13, "max_tile_bits_c128": tb128,
           "protocol": f"2 warmups, {reps} repeats, arms interleaved; the copy of the input is outside the timing"}
    cases = {"c64": (s64, 8, plans[13]), "c128": (s128, 16, plans[tb128])}
    times = {k: [] for k in cases}
    for r in range(reps + 2):
        for name, (st, amp, plan) in cases.items():
            st.copy_from(src)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            qs.apply(st, plan)
            st.sync()
            if r >= 2:
                times[name].append(time.perf_counter() - t0)
    for name, (st, amp, plan) in cases.items():
        t = float(np.mean(times[name]))
        out[f"ms_{name}"] = summary(times[name], nd=3)
        out[f"passes_{name}"] = plan.num_layers()
        out[f"GBs_{name}"] = round(plan.num_layers() * 2 * amp * (1 << n) / t / 1e9, 1)
    with qs.profile() as prof:
        for _ in range(3):
            s128.copy_from(src)
            qs.apply(s128, plans[tb128])
        torch.cuda.synchronize()
    tp = {r_["kernel"]: r_ for r_ in prof.report}.get("tile_pass")
    if tp:
        avg = tp["total_ms"] / tp["launches"]
        out["tile_pass_c128"] = {"avg_ms": round(avg, 4), "GBs": round(2 * 16 * (1 << n) / avg / 1e6, 1)}
    del src
    torch.cuda.empty_cache()
    out["infidelity_c64_vs_c128"] = qs.infidelity(s64, s128)
    out["norm2_drift_c64"] = abs(qs.norm2(s64) - 1.0)
    out["norm2_drift_c128"] = abs(qs.norm2(s128) - 1.0)
    return out


def bench_tfim(qs, torch, n=25, steps=40, reps=10):
    """25-qubit open-chain TFIM, J = 1, h = 0.8, dt = 0.05, 40 Strang steps
    after an H layer, complex64: fused plan against the plain per-gate plan
    (built beforehand), arms interleaved."""
    stream = W.tfim_strang_stream(n, 1.0, 0.8, 0.05, steps)
    plan = qs.Plan(n, stream)
    plain = qs.Plan(n, stream, mode="plain")
    st = qs.State(n, "c64")

    def arm(pl):
        st.set_basis(0)
        qs.apply(st, pl)
        st.sync()

    T = paired({"fused": lambda: arm(plan), "plain": lambda: arm(plain)}, reps=reps)
    arm(plan)
    z = qs.expect(st, W.z_terms(n), per_term=True)[1]
    return {"n_qubits": n, "gates": len(stream), "layers": plan.num_layers(),
            "ms_fused": T["fused"], "ms_plain": {k: v for k, v in T["plain"].items() if k != "ratio_vs_fused"},
            "speedup_vs_plain": speedup(T, "plain", "fused"),
            "max_abs_Z": float(np.max(np.abs(z)))}


MFMA_F32_PEAK_TFLOPS = 157.3


def layer_streams(n):
    """One structured layer of each kind at n qubits (fixed angles, seeded graph)."""
    rng = np.random.default_rng(7)
    graph = W.random_regular3_graph(n, rng)
    return {
        "diag_zz_chain": [W.G("RZZ", q, q + 1, theta=-0.1) for q in range(n - 1)],
        "diag_qaoa_cut": [W.G("RZZ", u, v, theta=-0.7) for u, v in graph],
        "gf2_block": W.random_perm_block(n, 200, BLOCK_SEED),
        "rx_layer": [W.G("RX", q, theta=0.1 + 0.01 * q) for q in range(n)],
        "qft": W.qft_stream(n),
        "walsh": W.wht_stream(n),
        "xx_layer": [W.G("RXX", q, q + 1, theta=0.3) for q in range(n - 1)],
    }


def bench_layers(qs, torch, n=30, reps=10):
    """Each structured layer alone on the resident 30-qubit state: its plan's
    layers, time per application (2 warmups, 10 repeats, mean and t-based 95%
    half-width) and the per-pass effective bandwidth (passes x 2 S / t), plus
    every kernel's average from the library's HIP events."""
    S = 8 * (1 << n)
    st = qs.State(n, "c64", init=None)
    W.gaussian_state_torch(n, STATE_SEED, "c64", out=st.tensor())
    out = {}
    for name, stream in layer_streams(n).items():
        plan = qs.Plan(n, stream)
        kinds = [L["kind"] for L in plan.describe()["layers"]]
        for _ in range(2):
            qs.apply(st, plan)
        torch.cuda.synchronize()
        ts = []
        with qs.profile() as prof:
            for _ in range(reps):
                t0 = time.perf_counter()
                qs.apply(st, plan)
                torch.cuda.synchronize()
                ts.append(time.perf_counter() - t0)
        t = float(np.mean(ts))
        kern = {r["kernel"]: {"launches": r["launches"] // reps,
                              "GBs": round(2 * S * r["launches"] / r["total_ms"] / 1e6, 1)} for r in prof.report}
        out[name] = {"gates": len(stream), "layers": kinds, "ms": summary(ts, nd=3),
                     "GBs_per_pass": round(len(kinds) * 2 * S / t / 1e9, 1),
                     "frac_per_pass": round(len(kinds) * 2 * S / t / 1e9 / HBM_PEAK_GBS, 4), "kernels": kern}
    del st
    torch.cuda.empty_cache()
    return out


MFMA_F64_PEAK_TFLOPS = 78.6


def bench_dense(qs, torch, n=30, blocks=20, seed=6, reps=3):
    """Dense k-qubit blocks on the matrix cores at 30 qubits, complex64 (FP32
    MFMA) and complex128 (FP64 MFMA): 20 UNITARY gates on seeded random wire
    sets per k = 4, 5, 6, each one dense layer.  Reports the per-block kernel
    time (HIP events, 3 x 20 launches), achieved HBM GB/s (2 S per block),
    TFLOP/s (8 2^k flop per amplitude) against the dtype's matrix-core peak,
    and one block on the plain per-gate k-qubit kernel for comparison."""
    out = {}
    for dt, amp, peak in (("c64", 8, MFMA_F32_PEAK_TFLOPS), ("c128", 16, MFMA_F64_PEAK_TFLOPS)):
        S = amp * (1 << n)
        st = qs.State(n, dt, init=None, lazy_scratch=True)
        W.gaussian_state_torch(n, STATE_SEED, dt, out=st.tensor())
        for k in (4, 5, 6):
            stream = W.dense_block_stream(n, blocks, k, seed + k)
            plan = qs.Plan(n, stream)
            qs.apply(st, plan)
            torch.cuda.synchronize()
            with qs.profile() as prof:
                for _ in range(reps):
                    qs.apply(st, plan)
                torch.cuda.synchronize()
            kern = {r["kernel"]: r for r in prof.report}[f"dense_k{k}"]
            avg = kern["total_ms"] / kern["launches"] * 1e-3
            flop = 8 * (1 << k) * (1 << n)
            one = qs.Plan(n, stream[:1], mode="plain")
            qs.apply(st, one)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            qs.apply(st, one)
            st.sync()
            t_plain = time.perf_counter() - t0
            key = f"k{k}" if dt == "c64" else f"k{k}_c128"
            out[key] = {"ms_per_block": round(1e3 * avg, 4), "GBs": round(2 * S / avg / 1e9, 1),
                        "hbm_frac": round(2 * S / avg / 1e9 / HBM_PEAK_GBS, 4),
                        "TFLOPs": round(flop / avg / 1e12, 2),
                        "mfma_frac": round(flop / avg / 1e12 / peak, 4), "mfma_peak_TFLOPs": peak,
                        "plain_ms_per_block": round(1e3 * t_plain, 2),
                        "speedup_vs_plain": round(t_plain / avg, 1)}
        out[f"norm_after_{dt}"] = qs.norm2(st)
        del st
        torch.cuda.empty_cache()
    return out


def bench_families(qs, torch, n=25, reps=10):
    """Weighted diagonal families at 25 qubits (complex64), fused plan against
    the plain per-gate plan (built beforehand), arms interleaved: 5
    first-order steps of the long-range Ising chain (300 bonds in 24 distance
    groups, J(r) = 1 / r^1.5, h = 0.8, dt = 0.05) and phase estimation of
    P(0.4) with 24 counting qubits (ladder angles up to 0.4 2^23 rad)."""
    S = 8 * (1 << n)
    out = {}
    cases = {"long_range_ising_5_steps": W.long_range_ising_stream(n, 1.0, 1.5, 0.8, 0.05, 5),
             "qpe_ladder_24_counting": W.qpe_ladder_stream(n - 1, 0.4)}
    st = qs.State(n, "c64")
    for name, stream in cases.items():
        plan = qs.Plan(n, stream)
        plain = qs.Plan(n, stream, mode="plain")
        kinds = [L["kind"] for L in plan.describe()["layers"]]

        def arm(pl):
            st.set_basis(0)
            qs.apply(st, pl)
            st.sync()

        T = paired({"fused": lambda: arm(plan), "plain": lambda: arm(plain)}, reps=reps)
        with qs.profile() as prof:
            for _ in range(3):
                arm(plan)
        kern = {r["kernel"]: {"launches": r["launches"] // 3,
                              "GBs": round(2 * S * r["launches"] / r["total_ms"] / 1e6, 1)}
                for r in prof.report if r["kernel"] not in ("fill_basis",)}
        t = T["fused"]["mean"] * 1e-3
        out[name] = {"gates": len(stream), "layers": len(kinds), "ms_fused": T["fused"],
                     "ms_plain": {k: v for k, v in T["plain"].items() if k != "ratio_vs_fused"},
                     "speedup_vs_plain": speedup(T, "plain", "fused"),
                     "GBs_per_pass": round(len(kinds) * 2 * S / t / 1e9, 1), "kernels": kern}
    del st
    torch.cuda.empty_cache()
    return out


def bench_xxz(qs, torch, reps=10):
    """Pauli-pair Trotter families, complex64, from the Neel state: the XXZ
    chain (delta = 0.5) and the Heisenberg chain with random fields
    h ~ U[-1, 1] at 25 qubits, 10 first-order steps, dt = 0.05 (conjugated XX /
    YY layers); the two-leg Heisenberg ladder at 24 qubits (12 rungs), 5 steps
    (families interleaved per bond: dense windows); and a 25-qubit QFT written
    out as phase gates and CNOTs (dense windows).  Fused plan against the
    structured plan without windows and the plain per-gate plan, arms
    interleaved."""
    cases = {
        "xxz_chain_25q_10_steps": (25, W.heisenberg_stream(25, 1.0, 0.5, 0.05, 10)),
        "heisenberg_random_field_25q_10_steps": (25, W.heisenberg_stream(25, 1.0, 1.0, 0.05, 10,
                                                                         W.random_fields(25, 1.0, 25))),
        "ladder_24q_5_steps": (24, W.ladder_stream(12, 1.0, 1.0, 0.05, 5)),
        "decomposed_qft_25q": (25, W.decomposed_qft_stream(25)),
    }
    out = {}
    for name, (n, stream) in cases.items():
        st = qs.State(n, "c64")
        init = W.neel_index(n)

        def arm(pl):
            st.set_basis(init)
            qs.apply(st, pl)
            st.sync()

        plan = qs.Plan(n, stream)
        d = plan.describe()
        kinds = [L["kind"] for L in d["layers"]]
        arms = {"fused": lambda: arm(plan)}
        if d["windows"]:
            structured = qs.Plan(n, stream, window_k=-1)
            arms["structured"] = lambda: arm(structured)
        plain = qs.Plan(n, stream, mode="plain")
        arms["plain"] = lambda: arm(plain)
        T = paired(arms, reps=reps)
        arm(plan)
        z = qs.expect(st, W.z_terms(n))
        rec = {"n_qubits": n, "gates": len(stream), "layers": len(kinds), "windows": d["windows"],
               "dense_layers": kinds.count("dense"), "ms_fused": T["fused"], "sum_Z": z}
        if d["windows"]:
            rec["layers_structured"] = structured.num_layers()
            rec["ms_structured"] = {k: v for k, v in T["structured"].items() if k != "ratio_vs_fused"}
            rec["speedup_vs_structured"] = speedup(T, "structured", "fused")
        rec["ms_plain"] = {k: v for k, v in T["plain"].items() if k != "ratio_vs_fused"}
        rec["speedup_vs_plain"] = speedup(T, "plain", "fused")
        out[name] = rec
        del st
        torch.cuda.empty_cache()
    return out


def bench_graphs(qs, torch, steps=40, reps=20):
    """Launch cost at small sizes: the 40-step Strang TFIM applied eagerly (one
    launch per layer) and as one recorded HIP graph, complex64, for the fused
    plan (tens of layers, each long enough to hide its launch) and for the
    plain per-gate plan (2985 short layers at these sizes)."""
    out = {}
    for n in (10, 14, 18):
        for mode in ("fused", "plain"):
            plan = qs.Plan(n, W.tfim_strang_stream(n, 1.0, 0.8, 0.05, steps), mode=mode)
            st = qs.State(n, "c64")
            res = {"layers": plan.num_layers()}

            def arm(fn):
                fn(st, plan)
                torch.cuda.synchronize()

            T = paired({"eager": lambda: arm(qs.apply), "graph": lambda: arm(qs.apply_graph)}, reps=reps)
            res["ms_eager"] = T["eager"]
            res["ms_graph"] = {k: v for k, v in T["graph"].items() if k != "ratio_vs_eager"}
            r = T["graph"]["ratio_vs_eager"]
            res["speedup_graph_vs_eager"] = round(1.0 / r["mean"], 2)
            out[f"tfim_{n}q_{mode}"] = res
            del st
    torch.cuda.empty_cache()
    return out


def manifest(qs, torch):
    """Run manifest: library, runtime and device identification, seeds."""
    import platform
    p = torch.cuda.get_device_properties(0)
    rev = None
    head = os.path.join(ROOT, ".git", "HEAD")
    if os.path.exists(head):
        ref = open(head).read().strip()
        if ref.startswith("ref: "):
            f = os.path.join(ROOT, ".git", ref[5:])
            rev = open(f).read().strip() if os.path.exists(f) else None
        else:
            rev = ref
    return {"library": qs.version(), "git_rev": rev, "torch": torch.__version__, "hip": torch.version.hip,
            "device": p.name, "arch": getattr(p, "gcnArchName", None), "compute_units": p.multi_processor_count,
            "device_memory_GiB": round(p.total_memory / 2 ** 30, 1), "host": platform.node(),
            "host_cpus": len(os.sched_getaffinity(0)), "state_seed": STATE_SEED, "block_seed": BLOCK_SEED,
            "timing": "HIP events on the library stream + host wall clock around K steps, synchronised"}


def profile_run(qs, torch, name):
    """One warm application of a section's fused path alone (no plain or
    per-instance arms): what rocprofv3 counter runs attach to."""
    if name == "tfim25":
        n = 25
        plan = qs.Plan(n, W.tfim_strang_stream(n, 1.0, 0.8, 0.05, 40))
        st = qs.State(n, "c64")

        def run():
            st.set_basis(0)
            qs.apply(st, plan)
    elif name == "batched_qaoa":
        # plan options from the tuner's cache (a bench.py --only batched_qaoa
        # run in the same environment fills it; otherwise the tuning runs here)
        depth = 4
        insts = W.qaoa_instances(512, 512, depth=depth)
        options = qaoa_tuned_options(qs, insts, depth)
        B = qs.Batch([qaoa_plan(qs, i, depth, options[i.n]) for i in insts], init="plus")

        def run():
            B.run()
    elif name == "adjoint":
        # the C5 gradient with the tuner's tile limit (cached by a preceding
        # bench.py --only adjoint run in the same environment)
        from paper_2609_19147_amd.tune import TileTuner
        n, layers = 24, 8
        stream = W.hea_stream(n, layers)
        params = W.hea_params(n, layers, 24)
        terms = W.xxz_terms(n, 0.5)
        st = qs.State(n, "c64")
        plans = {}

        def make(tb):
            if tb not in plans:
                plans[tb] = qs.Plan(n, stream, n_params=len(params), params=params, max_tile_bits=tb)
            return plans[tb]

        def tune_run(tb):
            st.set_basis(0)
            qs.adjoint_grad(st, make(tb), terms)
        plan = make(TileTuner().best(f"adjoint-hea{layers}-xxz", n, "c64", tune_run, (11, 12, 13)))

        def run():
            st.set_basis(0)
            qs.adjoint_grad(st, plan, terms)
    else:
        raise SystemExit(f"no profile run for {name}")
    run()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    run()
    torch.cuda.synchronize()
    return {"profile_run": name, "ms": round(1e3 * (time.perf_counter() - t0), 3)}


SECTIONS = {
    "batched_qaoa": lambda qs, torch: bench_batched_qaoa(qs, torch),
    "adjoint": lambda qs, torch: bench_adjoint(qs, torch),
    "tfim25": lambda qs, torch: bench_tfim(qs, torch),
    "precision_30q": lambda qs, torch: bench_precision(qs, torch),
    "dense_blocks": lambda qs, torch: bench_dense(qs, torch),
    "layers_30q": lambda qs, torch: bench_layers(qs, torch),
    "diag_families_25q": lambda qs, torch: bench_families(qs, torch),
    "xxz_families": lambda qs, torch: bench_xxz(qs, torch),
    "graphs_small_n": lambda qs, torch: bench_graphs(qs, torch),
}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--n", type=int, default=N_QUBITS)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extra", action="store_true", help="skip the batched, adjoint and TFIM sections")
    ap.add_argument("--no-ceiling", action="store_true", help="skip the standalone streaming-ceiling probe")
    ap.add_argument("--probe-copy", action="store_true",
                    help="also run one plain device copy of the state (2 S bytes) as a counter calibration")
    ap.add_argument("--only", choices=sorted(SECTIONS),
                    help="run one extra section alone and print its JSON (a profiling aid; not the benchmark line)")
    ap.add_argument("--profile-run", choices=["tfim25", "batched_qaoa", "adjoint"],
                    help="one warm application of a section's fused path, for counter runs (not the benchmark line)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark measures one GPU only; sharding over several GPUs is "
                                   "described in the design notes, not run", "n_gpus": args.gpus}))
        sys.exit(2)

    import torch
    import paper_2609_19147_amd as qs

    if args.only:
        print(json.dumps({args.only: SECTIONS[args.only](qs, torch)}))
        return
    if args.profile_run:
        print(json.dumps(profile_run(qs, torch, args.profile_run)))
        return

    n = args.n
    S = 8 * (1 << n)
    stream = circuit(n)
    t_plan = time.perf_counter()
    plan = qs.Plan(n, stream)
    t_plan = time.perf_counter() - t_plan
    desc = plan.describe()
    kinds = [L["kind"] for L in desc["layers"]]
    n_pass = len(kinds)

    st = qs.State(n, "c64", init=None)
    W.gaussian_state_torch(n, STATE_SEED, "c64", out=st.tensor())
    torch.cuda.synchronize()

    if args.probe_copy:
        other = qs.State(n, "c64", init=None, lazy_scratch=True)
        other.copy_from(st)
        torch.cuda.synchronize()
        del other

    def step():
        # the circuit, then the FP64 norm of its result (summed by the last
        # layer's kernel as it writes the state)
        return qs.apply_norm2(st, plan)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    with qs.profile() as prof:
        evs = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps + 1)]
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        evs[0].record()
        for k in range(args.steps):
            nrm = step()
            evs[k + 1].record()
        torch.cuda.synchronize()
        t1 = time.perf_counter()
    wall = t1 - t0
    # per-step device times: mean and the t-based 95% confidence half-width
    per_step = np.array([evs[k].elapsed_time(evs[k + 1]) for k in range(args.steps)])
    ci95 = None
    if args.steps > 1:
        from scipy.stats import t as student_t
        ci95 = float(student_t.ppf(0.975, args.steps - 1) * per_step.std(ddof=1) / math.sqrt(args.steps))
    ms_step = 1e3 * wall / args.steps
    # effective bandwidth: passes used x 2S per step (the norm is summed by
    # the last pass as it writes, so it moves no bytes of its own)
    alg_bytes = n_pass * 2 * S
    value = alg_bytes / (wall / args.steps) / 1e9
    # the same step counted as if the norm were a separate S-byte read
    norm_inclusive = (alg_bytes + S) / (wall / args.steps) / 1e9

    # the achievable streaming ceiling: the library's own device copy of the
    # same state (2 S bytes per launch), timed with HIP events like the step
    other = qs.State(n, "c64", init=None, lazy_scratch=True)
    other.copy_from(st)
    torch.cuda.synchronize()
    with qs.profile() as cprof:
        for _ in range(3):
            other.copy_from(st)
        torch.cuda.synchronize()
    del other
    torch.cuda.empty_cache()
    cp = {r["kernel"]: r for r in cprof.report}.get("copy")
    copy_gbs = 2 * S / (cp["total_ms"] / cp["launches"] * 1e-3) / 1e9 if cp else None

    kern = {r["kernel"]: r for r in prof.report}
    ceiling = None
    if not args.no_ceiling:
        log("streaming ceiling probe")
        ceiling = streaming_ceiling(n)
        if ceiling.get("best_copy_GBs") and (copy_gbs is None or ceiling["best_copy_GBs"] > copy_gbs):
            copy_gbs = ceiling["best_copy_GBs"]
    tp = kern.get("tile_pass")
    roof = None
    if tp:
        avg_ms = tp["total_ms"] / tp["launches"]
        achieved = 2 * S / (avg_ms * 1e-3) / 1e9
        traffic = measured_traffic("tile_pass")
        roof = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                "kernel": "tile_pass", "avg_ms": round(avg_ms, 4), "algorithmic_bytes_per_launch": 2 * S,
                "copy_ceiling_GBs": round(copy_gbs, 1) if copy_gbs else None,
                "frac_of_copy": round(achieved / copy_gbs, 4) if copy_gbs else None,
                "copy_ceiling_source": "best of the library's copy and the streaming-ceiling probe's copies"}
    kernels = {k: {"launches": v["launches"], "avg_ms": round(v["total_ms"] / v["launches"], 4)}
               for k, v in kern.items()}
    gf = kern.get("gf2_gather")
    if gf:
        kernels["gf2_gather"]["achieved_GBs"] = round(2 * S / (gf["total_ms"] / gf["launches"] * 1e-3) / 1e9, 1)
        if copy_gbs:
            kernels["gf2_gather"]["frac_of_copy"] = round(kernels["gf2_gather"]["achieved_GBs"] / copy_gbs, 4)

    out = {
        "metric": "effective state-vector HBM GB/s at 30q; circuits/s batched & adjoint vs plain",
        "value": round(value, 1),
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 3),
        "ms_per_step_events": {"mean": round(float(per_step.mean()), 4),
                               "ci95": round(ci95, 4) if ci95 is not None else None, "steps": args.steps},
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "c64",
        "data": "synthetic",
        "config": {"workload": f"{n}-qubit QFT ({n + n * (n - 1) // 2} gates) + Walsh-Hadamard ({n} H) + "
                               f"200-gate random X/CNOT/SWAP block, seeded Gaussian complex64 state, "
                               f"then FP64 norm", "n_qubits": n, "layers": kinds,
                   "gates": len(stream), "state_seed": STATE_SEED, "block_seed": BLOCK_SEED},
        "gate_stream_equiv_GBs": round(len(stream) * 2 * S / (wall / args.steps) / 1e9, 1),
        "norm_inclusive_equiv_GBs": round(norm_inclusive, 1),
        "norm_after": nrm,
        "hbm_bytes_per_step": n_pass * 2 * S,
        "plan_ms": round(1e3 * t_plan, 2),
        "roofline": roof,
        "kernels": kernels,
        "streaming_ceiling": ceiling,
        "manifest": manifest(qs, torch),
    }
    if not args.no_extra:
        del st
        torch.cuda.empty_cache()
        log("batched QAOA: 512 instances")
        out["batched_qaoa"] = bench_batched_qaoa(qs, torch)
        log("adjoint gradient: 24-qubit HEA")
        out["adjoint"] = bench_adjoint(qs, torch)
        log("TFIM: 25 qubits, 40 Strang steps")
        out["tfim25"] = bench_tfim(qs, torch)
        log("precision: the 30-qubit circuit in complex64 and complex128")
        out["precision_30q"] = bench_precision(qs, torch)
        log("dense k-qubit blocks: 30 qubits, k = 4, 5, 6")
        out["dense_blocks"] = bench_dense(qs, torch)
        log("single layers: 30 qubits")
        out["layers_30q"] = bench_layers(qs, torch)
        if copy_gbs:
            for v in out["layers_30q"].values():
                if isinstance(v, dict) and "GBs_per_pass" in v:
                    v["frac_of_copy"] = round(v["GBs_per_pass"] / copy_gbs, 4)
        log("weighted diagonal families: 25 qubits")
        out["diag_families_25q"] = bench_families(qs, torch)
        log("Pauli-pair Trotter families and decomposed streams: 24-25 qubits")
        out["xxz_families"] = bench_xxz(qs, torch)
        log("whole-plan graphs against eager launches: TFIM at 10-18 qubits")
        out["graphs_small_n"] = bench_graphs(qs, torch)
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle)")
        out["cpu_baseline"] = cpu_baseline()
        if not args.no_extra:
            log("oracle timings: 12-qubit QFT, QAOA subset (1 core, all cores), 12-qubit ansatz gradients")
            out["oracle_timings"] = oracle_timings()
    print(json.dumps(out))


if __name__ == "__main__":
    main()
