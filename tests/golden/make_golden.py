"""Writes the golden fixtures of tests/golden from the CPU oracle only.

integer_ring_n3.json: a 2x2x2 ring with ranks (2, 1, 1) and small integer
slices.  X(i1,i2,i3) = Trace(G1(i1) G2(i2) G3(i3)) (tensor-ring format,
Section 1) reduces to G2(i2) * (G3(i3) . G1(i1)) for these ranks; the
``hand_entries`` were worked out by hand from that formula:
  X(0,0,0) =  3 * (1*1 + 1*2)      =  9
  X(1,1,1) = -2 * (2*0 + (-1)*(-1)) = -2
  X(0,1,1) = -2 * (2*1 + (-1)*2)   =  0
  X(1,0,0) =  3 * (1*0 + 1*(-1))   = -3
The stored tensor and block gradient come from the oracle.
"""
import json
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import tr  # noqa: E402


def main():
    c1 = np.zeros((2, 2, 1)); c1[:, 0, 0] = [1, 2]; c1[:, 1, 0] = [0, -1]
    c2 = np.zeros((1, 2, 1)); c2[0, 0, 0] = 3; c2[0, 1, 0] = -2
    c3 = np.zeros((1, 2, 2)); c3[0, 0, :] = [1, 1]; c3[0, 1, :] = [2, -1]
    cores = [c1, c2, c3]
    X = tr.full_tensor(cores)
    G = tr.full_gradient(cores, np.zeros_like(X), 1)
    out = {
        "citation": "tensor-ring format (Section 1); eq:gradient (Section 3)",
        "cores": [c.tolist() for c in cores],
        "X": X.tolist(),
        "hand_entries": [
            {"index": [0, 0, 0], "value": 9.0},
            {"index": [1, 1, 1], "value": -2.0},
            {"index": [0, 1, 1], "value": 0.0},
            {"index": [1, 0, 0], "value": -3.0},
        ],
        "grad_mode2_at_zero_X": G.tolist(),
    }
    with open(os.path.join(HERE, "integer_ring_n3.json"), "w") as fh:
        json.dump(out, fh, indent=1)


if __name__ == "__main__":
    main()
