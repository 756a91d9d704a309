"""Write tests/golden/qaoa_p4_22q_24q.json from the CPU oracle (one gate at a time).

Workload: the batched MaxCut QAOA configuration (512 instances, seed 512,
qubit counts 16-24 even, random 3-regular graphs, depth p = 4, angles
U[0, pi)).  The first two instances with 22 qubits and the first two with 24
qubits are evolved from |+>^n through the four cost and mixer layers
(RZZ(-gamma) per edge, then RX(2 beta) per qubit) in complex128.  Stored per
instance: its position in the 512-instance list, the expected cut <C>, the
norm, and the amplitudes at 256 seeded random indices.  Takes about five
minutes on one core; only ``oracle/`` and ``workloads`` are used.

    python tests/golden/make_qaoa_p4.py
"""
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import workloads as W  # noqa: E402
from oracle import metrics, statevec as sv  # noqa: E402

COUNT, SEED, DEPTH = 512, 512, 4
PER_N = {22: 2, 24: 2}
SAMPLE_SEED, N_SAMPLES = 4096, 256


def main(out=os.path.join(HERE, "qaoa_p4_22q_24q.json")):
    insts = W.qaoa_instances(COUNT, SEED, depth=DEPTH)
    chosen = []
    for n, k in PER_N.items():
        chosen += [i for i, inst in enumerate(insts) if inst.n == n][:k]
    recs = []
    for pos in chosen:
        inst = insts[pos]
        t0 = time.time()
        psi = sv.plus(inst.n)
        stream = W.qaoa_stream(inst, h_layer=False)
        for g in stream:
            psi = sv.apply_gate(psi, inst.n, g)
        rng = np.random.default_rng(SAMPLE_SEED + pos)
        idx = np.sort(rng.choice(1 << inst.n, size=N_SAMPLES, replace=False))
        recs.append({
            "position": pos, "n": inst.n, "edges": [list(e) for e in inst.edges],
            "gammas": inst.gammas.tolist(), "betas": inst.betas.tolist(), "gates": len(stream),
            "cut": sv.expect(psi, inst.n, W.maxcut_terms(inst.edges)),
            "norm2": metrics.norm2(psi),
            "sample_idx": idx.tolist(),
            "sample_re": psi[idx].real.tolist(),
            "sample_im": psi[idx].imag.tolist(),
            "oracle_seconds": round(time.time() - t0, 1),
        })
        print(f"instance {pos}: n = {inst.n}, <C> = {recs[-1]['cut']:.12f}, "
              f"{recs[-1]['oracle_seconds']} s", flush=True)
    rec = {"workload": {"instances": COUNT, "seed": SEED, "depth": DEPTH, "start": "|+>^n",
                        "layer": "RZZ(-gamma) on every edge, then RX(2 beta) on every qubit"},
           "sample_seed": SAMPLE_SEED, "instances": recs}
    with open(out, "w") as fh:
        json.dump(rec, fh)
    print("wrote", out)


if __name__ == "__main__":
    main()
