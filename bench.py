#!/usr/bin/env python
"""Benchmark: time-domain CQM-BEM solves per second on one MI355X.

A step is one complete solve of the hot path on a synthetic workload: near
field (Duffy static part + per-frequency remainder), operator evaluation for
all frequency systems, right-hand side, forward scaled DFT, batched GMRES with
FP64 refinement, inverse scaled DFT -- everything from the mesh to the
time-domain density, with inputs already resident on the device.

Prints ONE JSON line.  Default workload: unit-sphere icosphere with 1280
triangles, N = 64 steps on T = 4 (33 frequency systems), Gaussian plane wave.
"""
import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import cqm_workloads as W  # noqa: E402

PEAK_FP32_TFLOPS = 157.3
PEAK_FP64_TFLOPS = 78.6
PEAK_HBM_GBS = 8000.0
# Algorithmic flops of one point-pair-frequency kernel value
# exp(-s r)/(4 pi r) accumulated with a real weight: three transcendental
# evaluations (exp, sin, cos; one flop each), three multiplies (sigma r,
# omega r, weight) and two fused multiply-adds (4 flops).
FLOPS_PER_UNIT = 10
# Kernel-value ceilings from the chip's unit counts: 256 CUs x 64 lanes x
# 2.4 GHz = 3.93e13 lane-cycles/s, divided by the lane-cycles one kernel
# value costs.  FP32: 3 transcendentals at quarter rate plus ~6 full-rate
# ops = ~18 lane-cycles.  FP64 (no hardware transcendentals; FP64 FMA is
# full rate): VALU instructions per value counted in the ISA of the inner
# loop, 32 for the dense assembly (table-driven exp and sincos on arguments
# pre-scaled to table steps, index arithmetic, accumulation; 356 per 11
# frequencies) and 36 for the FP64 matrix-free apply (the same math, which
# also multiplies by x and accumulates per target; 328 per 9 frequencies).
# Expressed in TFLOP/s with the 10-flop convention above.
LANE_CYCLES_PER_S = 256 * 64 * 2.4e9
ALU_PEAK_TFLOPS = {"far32": LANE_CYCLES_PER_S / 18 * FLOPS_PER_UNIT / 1e12,
                   "far64": LANE_CYCLES_PER_S / 36 * FLOPS_PER_UNIT / 1e12,
                   "assemble": LANE_CYCLES_PER_S / 32 * FLOPS_PER_UNIT / 1e12}

WORKLOADS = {"C1": W.C1, "C2": W.C2, "C3": W.C3}
KCLS = ["far32", "far64", "assemble", "gemv32", "gemv64", "near", "arnoldi", "other"]


def area_of(V, T):
    P = V[T]
    return 0.5 * np.linalg.norm(np.cross(P[:, 1] - P[:, 0], P[:, 2] - P[:, 0]), axis=1)


def rel_err(q, ref, area):
    return float(np.sqrt(np.sum(area * (q - ref) ** 2) / np.sum(area * ref ** 2)))


def run_variant(C, Problem, ctx, wl, mode, form, steps, warmup, torch, profile=0):
    V, T = wl.mesh()
    p = Problem(ctx, V, T, wl.N, wl.T, mode=mode, form=form, profile=profile)
    p.set_plane_wave(wl.wave.direction, wl.wave.sigma, wl.wave.t0, wl.wave.amplitude)
    out = torch.empty((wl.N + 1, len(T)), dtype=torch.float64, device="cuda")
    for _ in range(warmup):
        p.solve(out)
    torch.cuda.synchronize()
    lat, diags = [], []
    t0 = time.perf_counter()
    for _ in range(steps):
        s0 = time.perf_counter()
        _, rc, d = p.solve(out)
        lat.append(time.perf_counter() - s0)
        if rc != C.CQM_OK:
            raise RuntimeError(f"solve did not converge (rc={rc})")
        diags.append(d.as_dict())
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    q = out.cpu().numpy()
    p.close()
    return dict(elapsed=el, lat=lat, diags=diags, q=q, V=V, T=T,
                workspace=p.workspace_bytes)


def summarise_kernels(diags):
    ms = np.zeros(len(KCLS))
    calls = np.zeros(len(KCLS), dtype=int)
    for d in diags:
        ms += np.asarray(d["kernel_ms"])
        calls += np.asarray(d["kernel_calls"])
    return ms, calls


def roofline(diags):
    """Dominant kernel class over the timed steps and where it stands against
    its roofline.  Durations are the HIP-event times of every launch in the
    timed steps (recorded on the solve stream); the algorithmic work is what
    the kernels counted themselves: kernel values for the evaluation kernels
    (x FLOPS_PER_UNIT), bytes for the bandwidth-bound products and the
    Arnoldi step."""
    ms, calls = summarise_kernels(diags)
    work = np.zeros(len(KCLS))
    for d in diags:
        work += np.asarray(d["kernel_work"])
    k = int(np.argmax(ms))
    name = KCLS[k]
    n = max(int(calls[k]), 1)
    avg_ms = ms[k] / n
    out = {"kernel": name, "avg_launch_ms": avg_ms, "launches": int(calls[k]),
           "share_of_kernel_time": float(ms[k] / ms.sum()),
           "work_per_launch": work[k] / n}
    if name in ("far32", "far64", "assemble"):
        ach = work[k] / n * FLOPS_PER_UNIT / (avg_ms * 1e-3) / 1e12
        peak = ALU_PEAK_TFLOPS[name]
        vendor = PEAK_FP32_TFLOPS if name == "far32" else PEAK_FP64_TFLOPS
        return out | {"bound": "alu", "achieved": ach, "peak": peak, "unit": "TFLOP/s",
                      "frac": ach / peak, "traffic": traffic_per_launch(name),
                      "work_unit": "kernel values", "flops_per_unit": FLOPS_PER_UNIT,
                      "frac_of_vendor_peak": ach / vendor}
    if name in ("gemv32", "gemv64", "arnoldi"):
        ach = work[k] / n / (avg_ms * 1e-3) / 1e9
        return out | {"bound": "hbm", "achieved": ach, "peak": PEAK_HBM_GBS, "unit": "GB/s",
                      "frac": ach / PEAK_HBM_GBS, "traffic": traffic_per_launch(name),
                      "work_unit": "bytes"}
    return out | {"bound": "hbm", "achieved": None, "peak": PEAK_HBM_GBS, "unit": "GB/s",
                  "frac": None, "traffic": None}


def traffic_per_launch(cls):
    """HBM bytes per launch of the class's kernel from the committed counter
    summary (FETCH_SIZE + WRITE_SIZE, scaled by the plain-copy calibration),
    or None when the summary is missing or the kernel source changed since."""
    import hashlib
    path = os.path.join(ROOT, "profiles", f"traffic_{cls}_sphere1280_N64.txt")
    if not os.path.exists(path):
        return None
    kv = {}
    for line in open(path):
        if ":" in line and not line.startswith(" "):
            key, _, val = line.partition(":")
            kv[key.strip()] = val.strip()
    try:
        src = os.path.join(ROOT, kv["source"])
        if hashlib.sha256(open(src, "rb").read()).hexdigest()[:16] != kv["source_sha256_16"]:
            return None
        return float(kv["hbm_bytes_per_launch"])
    except (KeyError, OSError, ValueError):
        return None


def cpu_baseline(wl, sample_freqs=2):
    """The oracle on the host: near field, right-hand side, both DFTs, and the
    dense assembly + LU of `sample_freqs` of the frequency systems; the
    per-frequency part is scaled to all systems of one solve."""
    import scipy.linalg as sla

    import oracle as O
    V, T = wl.mesh()
    F = wl.N + 1
    H = O.num_frequencies_half(F)
    t0 = time.perf_counter()
    s, rho, dt = O.frequencies(wl.N, wl.T)
    b = O.rhs(V, T, wl.N, wl.T)
    ghat = O.forward_dft(b, rho, H)
    pairs = O.near_pairs(T)
    static = O.near_static(V, T, pairs, 5)
    t_fixed = time.perf_counter() - t0
    t1 = time.perf_counter()
    xh = np.zeros((H, len(T)), dtype=complex)
    for l in range(sample_freqs):
        A = O.assemble_V(V, T, s[l], pairs=pairs, static=static)
        xh[l] = sla.lu_solve(sla.lu_factor(A), ghat[l])
    t_freq = (time.perf_counter() - t1) / sample_freqs
    t2 = time.perf_counter()
    O.inverse_dft(xh, rho, F)
    t_fixed += time.perf_counter() - t2
    t_solve = t_fixed + H * t_freq
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    return {"value": 1.0 / t_solve, "unit": "solves/s", "cores": threads, "kind": "oracle",
            "sample": f"{sample_freqs} of {H} frequency systems (dense assembly + LU) plus the "
                      f"near field, right-hand side and both DFTs; per-frequency time scaled "
                      f"x{H}", "seconds_per_solve": t_solve}


def run_compressed(C, torch, ctx):
    """The paper's compressed form (H2 in space x MACA across frequencies,
    cluster leaves 32, eta 1, Chebyshev m = 4, eps 1e-6, full band) on the
    5120-triangle sphere, N = 128, T = 6, against the stored dense form (FP64
    refined to 1e-15, itself within 1e-8 of the oracle at the sizes the oracle
    reaches) and the matrix-free plain form."""
    from paper_2006_05186_amd.solver import Problem
    wl = W.C3
    V, T = wl.mesh()
    area = area_of(V, T)
    res = {}
    ref = None
    # eta = 0.125: at this size no block is admissible, so every block is
    # compressed across frequencies only (MACA) and the time-domain error is
    # set by eps instead of the m = 4 spatial interpolation
    for name, mode, form, eta in (("dense_mixed", C.CQM_MIXED_PLAIN, C.CQM_FORM_DENSE, None),
                                  ("compressed_mixed", C.CQM_MIXED_H2ACA, C.CQM_FORM_DENSE, None),
                                  ("compressed_mixed_eta0.125", C.CQM_MIXED_H2ACA, C.CQM_FORM_DENSE, 0.125),
                                  ("matrix_free_mixed", C.CQM_MIXED_PLAIN, C.CQM_FORM_MATRIX_FREE, None)):
        kw = {} if eta is None else {"eta": eta}
        p = Problem(ctx, V, T, wl.N, wl.T, mode=mode, form=form, **kw)
        p.set_plane_wave()
        p.solve()  # warm-up
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        q, rc, d = p.solve()
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        qn = q.cpu().numpy()
        r = {"seconds_per_solve": el, "rc": rc, "iters": d.total_iters, "cycles": d.cycles,
             "t_setup_ms": d.t_setup_ms, "operator_GB": d.operator_bytes / 1e9}
        if mode == C.CQM_MIXED_H2ACA:
            r |= {"max_rank": d.max_rank, "mean_rank": d.mean_rank, "far_blocks": d.n_far_blocks,
                  "near_blocks": d.n_near_blocks}
        if ref is None:
            ref = qn
        else:
            r["error_vs_dense"] = rel_err(qn, ref, area)
            num = np.sqrt(np.sum(area[None, :] * (qn - ref) ** 2, axis=1))
            den = np.sqrt(np.sum(area[None, :] * ref ** 2, axis=1))
            r["max_step_error_vs_dense"] = float(np.max(num / np.maximum(den, 1e-300)))
        res[name] = r
        p.close()
    res["compressed_speedup_vs_dense"] = (res["dense_mixed"]["seconds_per_solve"] /
                                          res["compressed_mixed"]["seconds_per_solve"])
    res["compressed_speedup_vs_matrix_free"] = (res["matrix_free_mixed"]["seconds_per_solve"] /
                                                res["compressed_mixed"]["seconds_per_solve"])
    return {"workload": wl.name} | res


def run_batch48(C, torch, ctx):
    """Uneven batch: 48 seeded problems (spheres/ellipsoids of 80..5120
    triangles, N in {16,32,64,128}, random direction and pulse width) solved
    by one cqm_solve_batch call; dense stored operators up to 1280 triangles,
    matrix-free products for 5120."""
    from paper_2006_05186_amd.solver import Problem, solve_batch
    mix = W.problem_mix(48)
    probs = []
    for w in mix:
        V, T = w.mesh()
        form = C.CQM_FORM_DENSE if len(T) <= 1280 else C.CQM_FORM_MATRIX_FREE
        p = Problem(ctx, V, T, w.N, w.T, mode=C.CQM_MIXED_PLAIN, form=form)
        p.set_plane_wave(w.wave.direction, w.wave.sigma, w.wave.t0)
        probs.append(p)
    solve_batch(probs)  # warm-up (kernels, descriptor buffers)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    res, rc = solve_batch(probs)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    iters = sum(d.total_iters for _, d in res)
    for p in probs:
        p.close()
    return {"problems": len(mix), "makespan_s": el, "solves_per_s": len(mix) / el, "rc": rc,
            "triangles": sorted({w.M for w in mix}), "steps": sorted({w.N for w in mix}),
            "total_arnoldi_steps": iters}


def run_serving(C, torch, ctx, rate, duration):
    """Poisson stream of solve requests on the 5120-triangle sphere (N = 128,
    T = 6, random direction and pulse per request) served by the continuous-
    batching loop with the operator cache (dense mixed form)."""
    from paper_2006_05186_amd.solver import Server
    wl = W.C3
    V, T = wl.mesh()
    arrivals = W.poisson_arrivals(rate, duration)
    rng = np.random.default_rng(W.DEFAULT_SEED + 1)
    srv = Server(ctx, 96 << 30, max_active=16, mode=C.CQM_MIXED_PLAIN, form=C.CQM_FORM_DENSE)
    # the first request builds the cached operator; it is timed like the rest
    tickets = []
    t0 = time.perf_counter()
    for a in arrivals:
        now = time.perf_counter() - t0
        if a > now:
            time.sleep(a - now)
        sigma = float(rng.uniform(0.2, 0.4))
        tickets.append(srv.submit(V, T, wl.N, wl.T, W.random_direction(rng), sigma, 1.0 + 2 * sigma))
    lat, rcs = {}, []
    while len(lat) < len(tickets):
        for t in tickets:
            if t not in lat:
                done, rc, _, d, l = srv.poll(t)
                if done:
                    lat[t] = l
                    rcs.append(rc)
        time.sleep(0.001)
    el = time.perf_counter() - t0
    st = srv.stats()
    srv.close()
    L = np.asarray(list(lat.values()))
    return {"workload": wl.name, "rate_per_s": rate, "duration_s": duration, "requests": len(tickets),
            "solves_per_s": len(tickets) / el, "p50_ms": float(np.percentile(L, 50)),
            "p99_ms": float(np.percentile(L, 99)), "max_ms": float(L.max()),
            "all_ok": all(r == C.CQM_OK for r in rcs), "peak_active": st["peak_active"],
            "operators_built": st["operators_built"], "cache_hits": st["operator_cache_hits"]}


def run_serving_mix(C, torch, ctx, rate, duration, large_frac=0.2):
    """Poisson stream mixing sphere5120_N128_T6 requests with a fraction of
    sphere20480_N256_T6 ones.  The large lane is on: requests whose stored
    dense operator would exceed a quarter of the budget (the 20480-triangle
    ones) are solved in the compressed form on a second stream; the others in
    the dense mixed form.  Operators cached; latency per class."""
    from paper_2006_05186_amd.solver import Server
    small, large = W.C3, W.C5_LARGE
    meshes = {small.name: small.mesh(), large.name: large.mesh()}
    arrivals = W.poisson_arrivals(rate, duration)
    rng = np.random.default_rng(W.DEFAULT_SEED + 2)
    kinds = [large if rng.uniform() < large_frac else small for _ in arrivals]
    srv = Server(ctx, 200 << 30, max_active=16, mode=C.CQM_MIXED_PLAIN, form=C.CQM_FORM_DENSE,
                 large_lane=1)
    tickets = []
    t0 = time.perf_counter()
    for a, wl in zip(arrivals, kinds):
        now = time.perf_counter() - t0
        if a > now:
            time.sleep(a - now)
        V, T = meshes[wl.name]
        sigma = float(rng.uniform(0.2, 0.4))
        tickets.append((srv.submit(V, T, wl.N, wl.T, W.random_direction(rng), sigma, 1.0 + 2 * sigma),
                        wl.name))
    lat, rcs = {}, []
    while len(lat) < len(tickets):
        for t, name in tickets:
            if t not in lat:
                done, rc, _, d, l = srv.poll(t)
                if done:
                    lat[t] = (l, name)
                    rcs.append(rc)
        time.sleep(0.005)
    el = time.perf_counter() - t0
    st = srv.stats()
    srv.close()
    out = {"rate_per_s": rate, "duration_s": duration, "requests": len(tickets),
           "large_fraction": large_frac, "makespan_s": el, "solves_per_s": len(tickets) / el,
           "all_ok": all(r == C.CQM_OK for r in rcs), "lane_completed": st["lane_completed"],
           "operators_built": st["operators_built"], "cache_hits": st["operator_cache_hits"]}
    for name in (small.name, large.name):
        L = np.asarray([l for l, n in lat.values() if n == name])
        if len(L):
            out[name] = {"count": int(len(L)), "p50_ms": float(np.percentile(L, 50)),
                         "p99_ms": float(np.percentile(L, 99)), "max_ms": float(L.max())}
    L = np.asarray([l for l, _ in lat.values()])
    out |= {"p50_ms": float(np.percentile(L, 50)), "p99_ms": float(np.percentile(L, 99))}
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=30)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="C2", choices=sorted(WORKLOADS))
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-variants", action="store_true")
    ap.add_argument("--serve-rate", type=float, default=10.0)
    ap.add_argument("--serve-seconds", type=float, default=6.0)
    ap.add_argument("--serve-mix", type=float, default=0.0, metavar="RATE",
                    help="only run the mixed serving stream (5120- and 20% 20480-triangle "
                         "requests) at RATE requests/s for --serve-seconds and exit")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain 1 GiB device-to-device copy three times (the reference "
                         "kernel for scaling HBM traffic counters) and exit")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); sharding across GPUs "
              f"is not built", file=sys.stderr)
        sys.exit(2)
    import torch

    from paper_2006_05186_amd import cqm as C
    from paper_2006_05186_amd.solver import Problem

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    if args.copy_calibration:
        n = 1 << 30
        src = torch.ones(n, dtype=torch.uint8, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes": n, "copies": 3}), flush=True)
        return
    wl = WORKLOADS[args.workload]
    ctx = C.cqm_ctx_create(0)
    if args.serve_mix > 0:
        mix = run_serving_mix(C, torch, ctx, args.serve_mix, args.serve_seconds)
        C.cqm_ctx_destroy(ctx)
        print(json.dumps({"serving_mix": mix}), flush=True)
        return
    main_mode, main_form = C.CQM_MIXED_PLAIN, C.CQM_FORM_DENSE
    r = run_variant(C, Problem, ctx, wl, main_mode, main_form, args.steps, args.warmup, torch)
    K = args.steps
    value = K / r["elapsed"]
    lat_ms = np.asarray(r["lat"]) * 1e3
    d0 = r["diags"][-1]
    # Kernel durations come from HIP events recorded around every launch on
    # the solve stream; the event records cost about a tenth of a step, so
    # they run in a second pass of the same workload right after the timed
    # steps rather than inside them.
    KP = min(K, 10)
    rp = run_variant(C, Problem, ctx, wl, main_mode, main_form, KP, 1, torch, profile=1)
    rl = roofline(rp["diags"])
    out = {
        "metric": "time-domain CQM-BEM solves/s + p50/p99 latency; kernel entries/s vs VALU peak",
        "value": value, "unit": "solves/s", "n_gpus": 1, "steps": K, "warmup": args.warmup,
        "ms_per_step": 1e3 * r["elapsed"] / K, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32+f64", "data": "synthetic",
        "config": {"workload": wl.name, "triangles": len(r["T"]), "N": wl.N, "T": wl.T,
                   "frequency_systems": wl.N // 2 + 1, "mode": "mixed", "form": "dense",
                   "pulse": {"direction": wl.wave.direction, "sigma": wl.wave.sigma,
                             "t0": wl.wave.t0}},
        "latency_ms": {"p50": float(np.percentile(lat_ms, 50)),
                       "p99": float(np.percentile(lat_ms, 99))},
        "roofline": {k: rl[k] for k in ("bound", "achieved", "peak", "unit", "frac", "traffic")},
        "dominant_kernel": {k: v for k, v in rl.items()
                            if k not in ("bound", "achieved", "peak", "unit", "frac", "traffic")}
        | {"profiled_steps": KP, "profiled_ms_per_step": 1e3 * rp["elapsed"] / KP},
        "solver": {"total_iters": d0["total_iters"], "max_iters": d0["max_iters"],
                   "cycles": d0["cycles"], "max_rel_residual": d0["max_rel_residual"],
                   "t_setup_ms": d0["t_setup_ms"], "t_solve_ms": d0["t_solve_ms"],
                   "workspace_GB": r["workspace"] / 1e9},
        "kernel_ms_per_step": dict(zip(KCLS, (summarise_kernels(rp["diags"])[0] / KP).round(4).tolist())),
    }
    golden = os.path.join(ROOT, "tests", "golden", f"{wl.name}.npz")
    if os.path.exists(golden):
        ref = np.load(golden)["q"]
        out["error_vs_oracle"] = rel_err(r["q"], ref, area_of(r["V"], r["T"]))
    if not args.no_variants:
        var = {}
        for name, mode, form, steps in (("fp64_dense", C.CQM_FP64_PLAIN, C.CQM_FORM_DENSE, 10),
                                        ("mixed_matrix_free", C.CQM_MIXED_PLAIN, C.CQM_FORM_MATRIX_FREE, 5),
                                        ("fp64_matrix_free", C.CQM_FP64_PLAIN, C.CQM_FORM_MATRIX_FREE, 3)):
            rv = run_variant(C, Problem, ctx, wl, mode, form, steps, 1, torch, profile=1)
            ms, calls = summarise_kernels(rv["diags"])
            v = {"solves_per_s": steps / rv["elapsed"]}
            for kn in ("far32", "far64"):
                k = KCLS.index(kn)
                if calls[k]:
                    v[f"{kn}_avg_ms"] = ms[k] / calls[k]
            if os.path.exists(golden):
                v["error_vs_oracle"] = rel_err(rv["q"], ref, area_of(rv["V"], rv["T"]))
            var[name] = v
        # kernel evaluation rate of the matrix-free FP32 far product (all
        # frequency systems active): one cqm_apply_V probe, timed by events
        V, T = wl.mesh()
        p = Problem(ctx, V, T, wl.N, wl.T, mode=C.CQM_MIXED_PLAIN, form=C.CQM_FORM_MATRIX_FREE)
        H = wl.N // 2 + 1
        x = torch.as_tensor(W.random_complex((H, len(T)), seed=3), device="cuda").to(torch.complex64)
        for _ in range(2):
            p.apply(x, 0, 32)
        torch.cuda.synchronize()
        st = torch.cuda.current_stream()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        reps = 10
        e0.record(st)
        for _ in range(reps):
            p.apply(x, 0, 32)
        e1.record(st)
        torch.cuda.synchronize()
        t_apply = e0.elapsed_time(e1) / reps * 1e-3
        u = C.cqm_operator_stats(p.handle).far_units
        var["far32_apply_probe"] = {"ms": t_apply * 1e3, "units_per_s": u / t_apply,
                                    "entries_per_s": u / 36 / t_apply,
                                    "tflops": u * FLOPS_PER_UNIT / t_apply / 1e12,
                                    "frac_fp32_peak": u * FLOPS_PER_UNIT / t_apply / 1e12 / PEAK_FP32_TFLOPS,
                                    "frac_transcendental_ceiling": u / t_apply / (LANE_CYCLES_PER_S / 18)}
        p.close()
        out["variants"] = var
    if not args.no_variants:
        out["compressed"] = run_compressed(C, torch, ctx)
        out["batch48"] = run_batch48(C, torch, ctx)
        out["serving"] = run_serving(C, torch, ctx, rate=args.serve_rate, duration=args.serve_seconds)
    C.cqm_ctx_destroy(ctx)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(wl)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
