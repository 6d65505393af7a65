"""Write stored oracle outputs used by the GPU parity tests.

Calls only oracle/ and cqm_workloads/ (no GPU code).  Run from the repository
root:  python tests/golden/make_golden.py
Outputs: tests/golden/sphere1280_N64_T4.npz with the density q (N+1, M), the
forward-transformed data ghat and the frequency-domain solutions xhat.
"""
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import cqm_workloads as W  # noqa: E402
import oracle as O  # noqa: E402


def main():
    wl = W.C2
    V, T = wl.mesh()
    t = time.time()
    r = O.solve(V, T, wl.N, wl.T, return_all=True)
    print(f"{wl.name}: oracle {time.time() - t:.1f}s, im_ratio {r['im_ratio']:.2e}")
    np.savez_compressed(os.path.join(HERE, f"{wl.name}.npz"), q=r["q"], ghat=r["ghat"],
                        xhat=r["xhat"], static=r["static"])


if __name__ == "__main__":
    main()
