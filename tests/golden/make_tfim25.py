"""Write tests/golden/tfim25_strang.json from the CPU oracle (one gate at a time).

Workload: 25-qubit open-chain TFIM, J = 1, h = 0.8, dt = 0.05, 40 second-order
(Strang) steps after an H layer on |0...0> (2985 gates).  Stores the
observables <Z_i>, <X_i>, <Z_i Z_{i+1}>, the norm, and the amplitudes at 4096
seeded random indices.  Takes about 40 minutes on one core; only ``oracle/``
and ``workloads`` are used.

    python tests/golden/make_tfim25.py
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

N, J, H, DT, STEPS = 25, 1.0, 0.8, 0.05, 40
SAMPLE_SEED, N_SAMPLES = 2025, 4096


def main(out=os.path.join(HERE, "tfim25_strang.json")):
    stream = W.tfim_strang_stream(N, J, H, DT, STEPS)
    psi = sv.basis(N, 0)
    t0 = time.time()
    for k, g in enumerate(stream):
        psi = sv.apply_gate(psi, N, g)
        if k % 200 == 0:
            print(f"gate {k}/{len(stream)}  {time.time() - t0:.0f} s", flush=True)
    rng = np.random.default_rng(SAMPLE_SEED)
    idx = np.sort(rng.choice(1 << N, size=N_SAMPLES, replace=False))
    rec = {
        "workload": {"n": N, "J": J, "h": H, "dt": DT, "steps": STEPS, "gates": len(stream),
                     "start": "|0...0> then H on every qubit", "order": "RX(h dt) RZZ(-2 J dt) RX(h dt)"},
        "norm2": metrics.norm2(psi),
        "z": sv.expect_terms(psi, N, W.z_terms(N)).tolist(),
        "x": sv.expect_terms(psi, N, W.x_terms(N)).tolist(),
        "zz": sv.expect_terms(psi, N, W.zz_chain_terms(N)).tolist(),
        "sample_seed": SAMPLE_SEED,
        "sample_idx": idx.tolist(),
        "sample_re": psi[idx].real.tolist(),
        "sample_im": psi[idx].imag.tolist(),
        "oracle_seconds": round(time.time() - t0, 1),
    }
    with open(out, "w") as fh:
        json.dump(rec, fh)
    print("wrote", out)


if __name__ == "__main__":
    main()
