"""Write the full-size expected values used by the GPU parity tests.

Calls only the oracle: explicit trajectory matrix, S = X X^T, Jacobi
eigen-decomposition (the paper's statement of the SVD step).  Stores the
leading singular values and the leading left vectors of each workload.

    python tests/golden/make_golden.py [2] [3] [4]
"""
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle                                   # noqa: E402
from paper_1309_5050_amd import workloads as W  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))
NVEC = {2: 6, 3: 4, 4: 4}          # leading U columns kept (gap-stable groups)


def main(which):
    for i in which:
        w = W.config(i)
        t0 = time.time()
        if w["kind"] == "mssa":
            s, U, V = oracle.decompose_mssa(w["x"], w["window"], method="gram", nvec=0)
        else:
            sh, s, U, V = oracle.decompose(w["x"], w["mask"], w["wmask"], w["window"],
                                           method="gram", nvec=0)
        r = w["r"]
        np.savez(os.path.join(HERE, f"config{i}_full.npz"), sigma=s[:r + 10],
                 U=U[:, :NVEC[i]], fro2=np.sum(s ** 2))
        print(f"config {i}: {time.time() - t0:.0f} s, sigma[:8] = {s[:8]}", flush=True)


if __name__ == "__main__":
    main([int(a) for a in sys.argv[1:]] or [4, 3, 2])
