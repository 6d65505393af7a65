"""Write stored oracle outputs used by the GPU parity tests.

Calls only oracle/ and cqm_workloads/ (no GPU code).  Run from the repository
root:
    python tests/golden/make_golden.py            # sphere1280_N64_T4
    python tests/golden/make_golden.py --c3 -j 7  # sphere5120_N128_T6
    python tests/golden/make_golden.py --h2m4     # sphere1280_N16_T2_h2m4
    python tests/golden/make_golden.py --h2order  # two_spheres640_N16_T2_h2
    python tests/golden/make_golden.py --h2rows   # sphere5120_N128_T6_h2rows
    python tests/golden/make_golden.py --h2march  # two_spheres640_N16_T2_h2march
Outputs tests/golden/<workload>.npz with the density q (N+1, M) and the
frequency-domain solutions xhat (distinct frequencies); the 1280-triangle file
also holds the forward-transformed data ghat and the static near-field values.
The h2m4 file holds the oracle's compressed operator (Algorithm 3: leaf size
32, eta = 1, Chebyshev order m = 4, MACA tolerances 1e-6 and 1e-10, near
blocks formed on demand) applied to a seeded input, with its block counts
and ranks.  The h2 file of two 320-triangle spheres six radii apart holds the
same for Chebyshev orders m = 4 .. 8 (leaf size 16, eta = 1, tolerance 1e-10,
near blocks from the dense tensor) and the plain product: the two spheres' clusters form admissible
blocks of 320 x 320, stored as Tucker cores for m <= 6 and expanded for m >= 7.
The h2rows file holds rows of the 5120-triangle workload's compressed
operator (leaf size 32, eta = 1, m = 4, MACA tolerances 1e-6 and 1e-10: the
configured setting) applied to a seeded input: the triangles of four leaf
clusters, with only the blocks of their block rows compressed (entries on
demand).  The h2march file holds the oracle's compressed time-marching
solution (weights from the transformed fibres) of the two spheres, N = 16,
T = 2, leaf size 16, eta = 1, tolerance 1e-10, m = 4 and 6 (the 320 x 320
blocks are Tucker cores), with the plain marching solution.

The 5120-triangle file is the same all-at-once oracle solve: its frequencies
are independent (one dense assembly and LU each), so they are spread over
worker processes, each running oracle.assemble_V and an LU solve for its
frequencies; the transforms and near-field values are the oracle's own.
"""
import argparse
import multiprocessing as mp
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))


def _c2():
    import numpy as np
    import cqm_workloads as W
    import oracle as O
    wl = W.C2
    V, T = wl.mesh()
    t = time.time()
    r = O.solve(V, T, wl.N, wl.T, return_all=True)
    print(f"{wl.name}: oracle {time.time() - t:.1f}s, im_ratio {r['im_ratio']:.2e}")
    np.savez_compressed(os.path.join(HERE, f"{wl.name}.npz"), q=r["q"], ghat=r["ghat"],
                        xhat=r["xhat"], static=r["static"])


_G = {}


def _init(V, T, pairs, static):
    _G.update(V=V, T=T, pairs=pairs, static=static)


def _one(args):
    import scipy.linalg as sla
    import oracle as O
    l, s, g = args
    A = O.assemble_V(_G["V"], _G["T"], s, 5, _G["pairs"], _G["static"])
    return l, sla.lu_solve(sla.lu_factor(A, overwrite_a=True), g)


def _c3(workers):
    import numpy as np
    import cqm_workloads as W
    import oracle as O
    wl = W.C3
    V, T = wl.mesh()
    t = time.time()
    s, rho, dt = O.frequencies(wl.N, wl.T)
    F = wl.N + 1
    H = O.num_frequencies_half(F)
    w = wl.wave
    b = O.rhs(V, T, wl.N, wl.T, w.direction, w.sigma, w.t0, w.amplitude)
    ghat = O.forward_dft(b, rho, H)
    pairs = O.near_pairs(T)
    static = O.near_static(V, T, pairs, 5)
    xhat = np.empty((H, len(T)), dtype=np.complex128)
    ctx = mp.get_context("fork")
    with ctx.Pool(workers, initializer=_init, initargs=(V, T, pairs, static)) as pool:
        for l, x in pool.imap_unordered(_one, [(l, s[l], ghat[l]) for l in range(H)]):
            xhat[l] = x
            print(f"  frequency {l} done at {time.time() - t:.0f}s", flush=True)
    q, im_ratio = O.inverse_dft(xhat, rho, F, conjugate_fill=True)
    print(f"{wl.name}: oracle {time.time() - t:.1f}s, im_ratio {im_ratio:.2e}")
    np.savez_compressed(os.path.join(HERE, f"{wl.name}.npz"), q=q, xhat=xhat)


def _h2m4():
    import numpy as np
    import cqm_workloads as W
    import oracle as O
    V, T = W.icosphere(3)
    N, Tend = 16, 2.0
    s, _, _ = O.frequencies(N, Tend)
    x = W.random_complex((len(s), len(T)), seed=31)
    out = {"x": x}
    for tag, eps in (("e6", 1e-6), ("e10", 1e-10)):
        t = time.time()
        op = O.build_compressed(V, T, s, 32, 1.0, 4, eps)
        out[f"y_{tag}"] = O.compressed_matvec(op, x)
        out[f"ranks_{tag}"] = np.asarray([b["rank"] for b in op["blocks"]])
        out[f"kinds_{tag}"] = np.asarray([b["kind"] == "far" for b in op["blocks"]])
        print(f"eps {eps}: {len(op['far'])} far / {len(op['near'])} near blocks, "
              f"{time.time() - t:.0f}s", flush=True)
    np.savez_compressed(os.path.join(HERE, "sphere1280_N16_T2_h2m4.npz"), **out)


def _h2rows():
    import numpy as np
    import cqm_workloads as W
    import oracle as O
    wl = W.C3
    V, T = wl.mesh()
    s, _, _ = O.frequencies(wl.N, wl.T)
    cl = O.compress.cluster_tree(V, T, 32)
    leaves = [c for c in cl if not c["sons"]]
    pick = [leaves[k * len(leaves) // 4]["idx"] for k in range(4)]
    rows = np.sort(np.concatenate(pick))
    x = W.random_complex((len(s), len(T)), seed=33)  # regenerated by the test from the seed
    out = {"rows": rows, "seed": np.asarray(33)}
    for tag, eps in (("e6", 1e-6), ("e10", 1e-10)):
        t = time.time()
        op = O.build_compressed(V, T, s, 32, 1.0, 4, eps, rows=rows)
        out[f"y_{tag}"] = O.compressed_matvec(op, x)[:, rows]
        out[f"nblocks_{tag}"] = np.asarray(len(op["blocks"]))
        print(f"eps {eps}: {len(op['blocks'])} blocks for {len(rows)} rows, {time.time() - t:.0f}s",
              flush=True)
    np.savez_compressed(os.path.join(HERE, "sphere5120_N128_T6_h2rows.npz"), **out)


def _h2march():
    import numpy as np
    import cqm_workloads as W
    import oracle as O
    V, T = W.two_spheres(2)
    N, Tend = 16, 2.0
    out = {}
    for m in (4, 6):
        t = time.time()
        out[f"q_m{m}"] = O.solve_marching_compressed(V, T, N, Tend, 16, 1.0, m, 1e-10)
        print(f"compressed marching m {m}: {time.time() - t:.0f}s", flush=True)
    out["q_plain"] = O.solve_marching(V, T, N, Tend)
    np.savez_compressed(os.path.join(HERE, "two_spheres640_N16_T2_h2march.npz"), **out)


ORDERS = (4, 5, 6, 7, 8)


def _h2order():
    import numpy as np
    import cqm_workloads as W
    import oracle as O
    V, T = W.two_spheres(2)
    N, Tend = 16, 2.0
    s, _, _ = O.frequencies(N, Tend)
    x = W.random_complex((len(s), len(T)), seed=32)
    t = time.time()
    dense = O.dense_tensor(V, T, s)
    print(f"dense tensor {time.time() - t:.0f}s", flush=True)
    out = {"x": x, "y_plain": np.einsum("ijl,lj->li", dense, x)}
    for m in ORDERS:
        t = time.time()
        op = O.build_compressed(V, T, s, 16, 1.0, m, 1e-10, dense=dense)
        out[f"y_m{m}"] = O.compressed_matvec(op, x)
        out[f"ranks_m{m}"] = np.asarray([b["rank"] for b in op["blocks"]])
        out[f"kinds_m{m}"] = np.asarray([b["kind"] == "far" for b in op["blocks"]])
        print(f"m {m}: {len(op['far'])} far / {len(op['near'])} near blocks, "
              f"{time.time() - t:.0f}s", flush=True)
    np.savez_compressed(os.path.join(HERE, "two_spheres640_N16_T2_h2.npz"), **out)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--c3", action="store_true", help="the 5120-triangle workload")
    ap.add_argument("-j", type=int, default=4, help="worker processes (--c3)")
    ap.add_argument("--h2m4", action="store_true", help="compressed operator, m = 4")
    ap.add_argument("--h2order", action="store_true",
                    help="compressed operator of two spheres, m = 4 .. 8")
    ap.add_argument("--h2rows", action="store_true",
                    help="sampled rows of the 5120-triangle compressed operator")
    ap.add_argument("--h2march", action="store_true",
                    help="compressed marching of two spheres, m = 4 and 6")
    a = ap.parse_args()
    if a.h2march:
        _h2march()
    elif a.h2rows:
        _h2rows()
    elif a.h2order:
        _h2order()
    elif a.h2m4:
        _h2m4()
    elif a.c3:
        for k in ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS"):
            os.environ[k] = "1"
        _c3(a.j)
    else:
        _c2()


if __name__ == "__main__":
    main()
