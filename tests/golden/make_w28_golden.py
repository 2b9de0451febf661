"""Write the expected values of the 28-qubit, batch-1 ring workload.

Calls only the CPU oracle (complex128 forward, float64 adjoint) on the seeded
inputs of `inputs.workload("w28_b1_ring")` with upstream gradient g = 1 (loss
= sum_i <Z_i>), and stores <Z_i>, the weight gradients and the input
gradients, plus a few amplitudes, in w28_b1_ring.json next to this script.
Needs about 12 GiB of host memory and tens of minutes of CPU time.

    python tests/golden/make_w28_golden.py
"""
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

from oracle import oracle  # noqa: E402
from paper_2404_09213_amd import inputs  # noqa: E402

AMP_INDICES = [0, 1, 2, 12345, 1 << 20, (1 << 27) + 777, (1 << 28) - 1]


def main():
    c, batch, seed = inputs.workload("w28_b1_ring")
    w, x = inputs.draw_angles(c, batch, seed)
    g = np.ones((batch, c.n_qubits))
    t = time.time()
    gw, gx, st = oracle.adjoint(c.n_qubits, c.gates, w.astype(np.float64), x.astype(np.float64),
                                batch, g, want_state=True)
    E = oracle.expval(c.n_qubits, st)
    out = {
        "workload": "w28_b1_ring", "seed": seed, "grad_out": "ones",
        "source": "oracle/qsv_oracle.c via oracle.oracle.adjoint (complex128 / float64)",
        "expval": E[0].tolist(),
        "grad_weights": gw.tolist(),
        "grad_inputs": gx[0].tolist(),
        "amp_indices": AMP_INDICES,
        "amps_re": [float(st[0, i].real) for i in AMP_INDICES],
        "amps_im": [float(st[0, i].imag) for i in AMP_INDICES],
        "oracle_seconds": round(time.time() - t, 1),
    }
    with open(os.path.join(HERE, "w28_b1_ring.json"), "w") as f:
        json.dump(out, f, indent=1)
    print("wrote", os.path.join(HERE, "w28_b1_ring.json"), out["oracle_seconds"], "s")


if __name__ == "__main__":
    main()
