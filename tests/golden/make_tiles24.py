"""Write tests/golden/tiles24_streams.json from the CPU oracle (one gate at a time).

Workload: four of the 24-qubit tile-pass streams of tests/test_gpu_tiles_24q.py
(the QFT followed by the Walsh layer, the inverse QFT, a random stream of
single-qubit gates, and a random mixed stream), each applied in complex128 to
the seeded Gaussian state gaussian_state(24, 21).  Stored per stream: the gate
count, the norm and the amplitudes at 256 seeded random indices.  Takes a
few minutes on one core; only ``oracle/``, ``workloads`` and the test module's
stream definitions are used.

    python tests/golden/make_tiles24.py
"""
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))
sys.path.insert(0, os.path.dirname(HERE))

import workloads as W  # noqa: E402
from oracle import metrics, statevec as sv  # noqa: E402
from test_gpu_tiles_24q import streams  # noqa: E402

N, STATE_SEED = 24, 21
NAMES = ("qft_walsh", "inverse_qft", "one_qubit_windows", "mixed")
SAMPLE_SEED, N_SAMPLES = 2424, 256


def main(out=os.path.join(HERE, "tiles24_streams.json")):
    psi0 = W.gaussian_state(N, STATE_SEED)
    idx = np.sort(np.random.default_rng(SAMPLE_SEED).choice(1 << N, size=N_SAMPLES, replace=False))
    recs = {}
    all_streams = streams(N)
    for name in NAMES:
        t0 = time.time()
        psi = sv.run(psi0.copy(), N, all_streams[name])
        recs[name] = {"gates": len(all_streams[name]), "norm2": float(metrics.norm2(psi)),
                      "amps": [[float(psi[i].real), float(psi[i].imag)] for i in idx]}
        print(f"{name}: {len(all_streams[name])} gates, {time.time() - t0:.1f} s", flush=True)
    doc = {"n": N, "state": f"gaussian_state({N}, {STATE_SEED})", "indices": [int(i) for i in idx],
           "source": "oracle/statevec.py, one gate at a time in complex128", "streams": recs}
    with open(out, "w") as fh:
        json.dump(doc, fh)


if __name__ == "__main__":
    main()
