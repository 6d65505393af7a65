#!/usr/bin/env python
"""Benchmark: time-domain CQM-BEM solves per second on one MI355X.

A step is one complete solve of the hot path on a synthetic workload: near
field (Duffy static part + per-frequency remainder), operator evaluation for
all frequency systems, right-hand side, forward scaled DFT, batched GMRES with
FP64 refinement, inverse scaled DFT -- everything from the mesh to the
time-domain density, with inputs already resident on the device.

Prints ONE JSON line.  Default workload: unit-sphere icosphere with 5120
triangles, N = 128 steps on T = 6 (65 distinct frequency systems), Gaussian
plane wave, solved in the mixed stored form; its error is measured against
the stored oracle solution of the same workload.
"""
import argparse
import gc
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import cqm_workloads as W  # noqa: E402

# MI355X published peaks: FP32 vector 157.3 TFLOP/s (packed FMA; 78.6 without
# packed instructions, which this build does not emit), FP64 vector 78.6,
# HBM3E 8 TB/s.
PEAK_FP32_TFLOPS = 157.3
PEAK_FP32_UNPACKED_TFLOPS = 78.6
PEAK_FP64_TFLOPS = 78.6
PEAK_HBM_GBS = 8000.0
# Algorithmic flops of one point-pair-frequency kernel value
# exp(-s r)/(4 pi r) accumulated with a real weight: three transcendental
# evaluations (exp, sin, cos; one flop each), three multiplies (sigma r,
# omega r, weight) and two fused multiply-adds (4 flops).
FLOPS_PER_UNIT = 10
# Instruction-count ceilings (reported beside the vendor-peak fraction, not
# as the roofline's peak): 256 CUs x 64 lanes x 2.4 GHz = 3.93e13
# lane-cycles/s, divided by the lane-cycles one kernel value costs.  FP32:
# 3 transcendentals (v_exp_f32, v_sin_f32, v_cos_f32) plus ~6 full-rate ops;
# the transcendentals measure half the FP32 FMA rate on gfx950
# (profiles/alu_rates_gfx950.txt: 29.5 vs 58.1 lane-ops per CU per cycle),
# so 3 x 2.18 + 6 x 1.10 = 13.2 lane-cycles.  FP64 (no hardware
# transcendentals): VALU instructions per value counted in the ISA of the
# inner loop, 32 for the dense assembly (table-driven exp and sincos on
# arguments pre-scaled to table steps, index arithmetic, accumulation; 356
# per 11 frequencies) and 36 for the FP64 matrix-free apply (the same math,
# which also multiplies by x and accumulates per target; 328 per 9
# frequencies).  Expressed in TFLOP/s with the 10-flop convention above.
LANE_CYCLES_PER_S = 256 * 64 * 2.4e9
ALU_PEAK_TFLOPS = {"far32": LANE_CYCLES_PER_S / 13.2 * FLOPS_PER_UNIT / 1e12,
                   "far64": LANE_CYCLES_PER_S / 36 * FLOPS_PER_UNIT / 1e12,
                   "assemble": LANE_CYCLES_PER_S / 32 * FLOPS_PER_UNIT / 1e12}

VENDOR_PEAK_TFLOPS = {"far32": PEAK_FP32_TFLOPS, "far64": PEAK_FP64_TFLOPS,
                      "assemble": PEAK_FP64_TFLOPS}

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


def roofline(diags, tag, cls=None):
    """Dominant kernel class (or class `cls`) over the timed steps and where
    it stands against its roofline.  Durations are the HIP-event times of every launch in the
    timed steps (recorded on the solve stream); the algorithmic work is what
    the kernels counted themselves: kernel values for the evaluation kernels
    (x FLOPS_PER_UNIT), bytes for the bandwidth-bound products and the
    Arnoldi step."""
    ms, calls = summarise_kernels(diags)
    work = np.zeros(len(KCLS))
    for d in diags:
        work += np.asarray(d["kernel_work"])
    k = int(np.argmax(ms)) if cls is None else KCLS.index(cls)
    name = KCLS[k]
    n = max(int(calls[k]), 1)
    avg_ms = ms[k] / n
    out = {"kernel": name, "avg_launch_ms": avg_ms, "launches": int(calls[k]),
           "share_of_kernel_time": float(ms[k] / ms.sum()),
           "work_per_launch": work[k] / n}
    if not (avg_ms > 0 and work[k] > 0):
        return out | {"bound": None, "achieved": None, "peak": None, "unit": None,
                      "frac": None, "traffic": None}
    if name in ("far32", "far64", "assemble"):
        ach = work[k] / n * FLOPS_PER_UNIT / (avg_ms * 1e-3) / 1e12
        peak = VENDOR_PEAK_TFLOPS[name]
        isa = ALU_PEAK_TFLOPS[name]
        return out | {"bound": "alu", "achieved": ach, "peak": peak, "unit": "TFLOP/s",
                      "frac": ach / peak, "traffic": traffic_per_launch(name, tag),
                      "work_unit": "kernel values", "flops_per_unit": FLOPS_PER_UNIT,
                      "isa_count_ceiling_tflops": isa, "frac_of_isa_count_ceiling": ach / isa}
    if name in ("gemv32", "gemv64", "arnoldi"):
        ach = work[k] / n / (avg_ms * 1e-3) / 1e9
        return out | {"bound": "hbm", "achieved": ach, "peak": PEAK_HBM_GBS, "unit": "GB/s",
                      "frac": ach / PEAK_HBM_GBS, "traffic": traffic_per_launch(name, tag),
                      "work_unit": "bytes"}
    return out | {"bound": "hbm", "achieved": None, "peak": PEAK_HBM_GBS, "unit": "GB/s",
                  "frac": None, "traffic": None}


def traffic_per_launch(cls, tag):
    """HBM bytes per launch of the class's kernel from the committed counter
    summary profiles/traffic_<cls>_<tag>.txt (FETCH_SIZE + WRITE_SIZE, scaled
    by the plain-copy calibration), or None when the summary is missing or the
    kernel source changed since."""
    import hashlib
    path = os.path.join(ROOT, "profiles", f"traffic_{cls}_{tag}.txt")
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


def golden_q(wl):
    path = os.path.join(ROOT, "tests", "golden", f"{wl.name}.npz")
    return np.load(path)["q"] if os.path.exists(path) else None


def errors(q, ref, area):
    """Area-weighted relative error over all steps and the largest per-step one."""
    num = np.sqrt(np.sum(area[None, :] * (q - ref) ** 2, axis=1))
    den = np.sqrt(np.sum(area[None, :] * ref ** 2, axis=1))
    return rel_err(q, ref, area), float(np.max(num / np.maximum(den, 1e-300)))


def blas_threads():
    try:
        from threadpoolctl import threadpool_info
        n = [d["num_threads"] for d in threadpool_info() if d.get("user_api") == "blas"]
        if n:
            return int(max(n))
    except Exception:
        pass
    return int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))


def cpu_baseline(wl, sample_rows=128):
    """The oracle on the host, timed on a bounded sample of one solve of `wl`:
    the frequency-independent parts run whole (right-hand side, forward
    transform, near-field pairs and static integrals, inverse transform); of
    the per-frequency part (dense assembly of V(s_l), LU, solve) the assembly
    of `sample_rows` rows of V(s_0) is timed and scaled to all rows, and one
    LU factorisation + solve of an M x M complex matrix is timed (its cost
    does not depend on the values); the two are scaled to all distinct
    frequencies."""
    import scipy.linalg as sla

    import oracle as O
    V, T = wl.mesh()
    M = len(T)
    F = wl.N + 1
    H = O.num_frequencies_half(F)
    w = wl.wave
    t0 = time.perf_counter()
    s, rho, dt = O.frequencies(wl.N, wl.T)
    b = O.rhs(V, T, wl.N, wl.T, w.direction, w.sigma, w.t0, w.amplitude)
    ghat = O.forward_dft(b, rho, H)
    pairs = O.near_pairs(T)
    static = O.near_static(V, T, pairs, 5)
    O.inverse_dft(np.zeros((H, M), dtype=complex), rho, F)
    t_fixed = time.perf_counter() - t0
    rows = np.linspace(0, M - 1, min(sample_rows, M)).astype(int)
    t1 = time.perf_counter()
    A_rows = O.assemble_V(V, T, s[0], pairs=pairs, static=static, rows=rows)
    t_asm = (time.perf_counter() - t1) * M / len(rows)
    rng = np.random.default_rng(0)
    A = rng.standard_normal((M, M)) + 1j * rng.standard_normal((M, M)) + M * np.eye(M)
    A[rows] = A_rows
    t2 = time.perf_counter()
    sla.lu_solve(sla.lu_factor(A, overwrite_a=True), ghat[0])
    t_lu = time.perf_counter() - t2
    t_solve = t_fixed + H * (t_asm + t_lu)
    return {"value": 1.0 / t_solve, "unit": "solves/s", "cores": blas_threads(), "kind": "oracle",
            "sample": f"{wl.name}: right-hand side, forward/inverse transforms and the near field "
                      f"whole ({t_fixed:.1f} s); assembly of {len(rows)} of {M} rows of V(s_0) "
                      f"scaled x{M / len(rows):.0f} ({t_asm:.1f} s per frequency) and one "
                      f"{M} x {M} complex LU + solve ({t_lu:.1f} s), both scaled to the {H} "
                      f"distinct frequencies; elementwise assembly single-threaded, LU on the "
                      f"BLAS threads", "seconds_per_solve": t_solve}


def run_compressed(C, torch, ctx, only=None):
    """The paper's compressed form (H2 in space x MACA across frequencies,
    cluster leaves 32, eta 1, Chebyshev m = 4, eps 1e-6, full band; and
    m = 6, eta = 0.25) on the
    5120-triangle sphere, N = 128, T = 6, against the stored oracle solution
    of the same workload, beside the stored dense and matrix-free plain forms.
    "compressed_mixed" refines with residuals of the plain operator (the
    default: the plain method's answer, the compressed operator carrying the
    inner iterations); the "_approx" variants refine with the compressed
    operator itself, so its approximation error stays in the answer."""
    from paper_2006_05186_amd.solver import Problem
    wl = W.C3
    V, T = wl.mesh()
    area = area_of(V, T)
    ref = golden_q(wl)
    res = {}
    # m = 6, eta = 0.25: the cheapest setting of the order sweep whose own
    # approximation error is below 1e-5 at this size
    H2 = C.CQM_MIXED_H2ACA
    m6 = {"cheb_m": 6, "eta": 0.25}
    for name, mode, form, kw in (("dense_mixed", C.CQM_MIXED_PLAIN, C.CQM_FORM_DENSE, {}),
                                 ("compressed_mixed", H2, C.CQM_FORM_DENSE, {}),
                                 ("compressed_mixed_approx", H2, C.CQM_FORM_DENSE,
                                  {"refine_plain": 0}),
                                 ("compressed_mixed_m6_eta0.25", H2, C.CQM_FORM_DENSE, m6),
                                 ("compressed_mixed_approx_m6_eta0.25", H2, C.CQM_FORM_DENSE,
                                  {"refine_plain": 0} | m6),
                                 ("matrix_free_mixed", C.CQM_MIXED_PLAIN, C.CQM_FORM_MATRIX_FREE, {})):
        if only and name not in only:
            continue
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
        if ref is not None:
            r["error_vs_oracle"], r["max_step_error_vs_oracle"] = errors(qn, ref, area)
        res[name] = r
        p.close()
    if only is None:
        res["compressed_speedup_vs_dense"] = (res["dense_mixed"]["seconds_per_solve"] /
                                              res["compressed_mixed"]["seconds_per_solve"])
        res["compressed_speedup_vs_matrix_free"] = (res["matrix_free_mixed"]["seconds_per_solve"] /
                                                    res["compressed_mixed"]["seconds_per_solve"])
        a = res["compressed_mixed_approx_m6_eta0.25"]["seconds_per_solve"]
        res["approx_m6_eta0.25_speedup_vs_dense"] = res["dense_mixed"]["seconds_per_solve"] / a
        res["approx_m6_eta0.25_speedup_vs_matrix_free"] = res["matrix_free_mixed"]["seconds_per_solve"] / a
    return {"workload": wl.name} | res


ORDER_SWEEP = ((1.0, (4, 5, 6)), (0.5, (4, 5, 6)), (0.25, (5, 6, 7)))


def run_orders(C, torch, ctx, sweep=ORDER_SWEEP):
    """The compressed approximation itself (refined with the compressed
    operator, as the paper solves) on the 5120-triangle sphere, N = 128, T = 6
    for admissibility parameters eta and Chebyshev orders m (Section 4.2's
    trade: the interpolation error falls with m and with eta), against the
    stored oracle solution: error, ranks, storage, set-up and solve time."""
    from paper_2006_05186_amd.solver import Problem
    wl = W.C3
    V, T = wl.mesh()
    area = area_of(V, T)
    ref = golden_q(wl)
    res = {"workload": wl.name, "eps_aca": 1e-6, "n_min": 32}
    for eta, orders in sweep:
        for m in orders:
            p = Problem(ctx, V, T, wl.N, wl.T, mode=C.CQM_MIXED_H2ACA, form=C.CQM_FORM_DENSE,
                        cheb_m=m, eta=eta, refine_plain=0)
            p.set_plane_wave()
            t0 = time.perf_counter()
            p.solve()  # includes the set-up (MACA of every block)
            torch.cuda.synchronize()
            first = time.perf_counter() - t0
            t0 = time.perf_counter()
            q, rc, d = p.solve()
            torch.cuda.synchronize()
            el = time.perf_counter() - t0
            r = {"m": m, "eta": eta, "rc": rc, "seconds_per_solve": el,
                 "first_solve_s": first, "t_setup_ms": d.t_setup_ms,
                 "operator_GB": d.operator_bytes / 1e9, "max_rank": d.max_rank,
                 "mean_rank": d.mean_rank, "far_blocks": d.n_far_blocks,
                 "near_blocks": d.n_near_blocks, "iters": d.total_iters}
            if ref is not None:
                r["error_vs_oracle"], r["max_step_error_vs_oracle"] = errors(q.cpu().numpy(), ref, area)
            res[f"m{m}_eta{eta:g}"] = r
            print(f"orders: m={m} eta={eta} done ({el:.2f} s, error "
                  f"{r.get('error_vs_oracle', float('nan')):.2e})", file=sys.stderr, flush=True)
            p.close()
            del q
            gc.collect()
            torch.cuda.empty_cache()
    return res


def run_batch48(C, torch, ctx, sample=4):
    """Uneven batch: 48 seeded problems (spheres/ellipsoids of 80..5120
    triangles, N in {16,32,64,128}, random direction and pulse width) solved
    by one cqm_solve_batch call, every problem in the stored form (about
    130 GB of operators, assembled by one work-queue launch).  The first
    `sample` problems of at most 320 triangles are compared with the
    oracle."""
    import oracle as O
    from paper_2006_05186_amd.solver import Problem, solve_batch
    mix = W.problem_mix(48)
    probs = []
    for w in mix:
        V, T = w.mesh()
        p = Problem(ctx, V, T, w.N, w.T, mode=C.CQM_MIXED_PLAIN, form=C.CQM_FORM_DENSE)
        p.set_plane_wave(w.wave.direction, w.wave.sigma, w.wave.t0)
        probs.append(p)
    solve_batch(probs)  # warm-up (kernels, descriptor buffers)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    res, rc = solve_batch(probs)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    iters = sum(d.total_iters for _, d in res)
    checked = []
    for k, w in enumerate(mix):
        if len(checked) >= sample:
            break
        if w.M > 320:
            continue
        V, T = w.mesh()
        ref = O.solve(V, T, w.N, w.T, direction=w.wave.direction, sigma=w.wave.sigma,
                      t0=w.wave.t0, amplitude=w.wave.amplitude)
        e, emax = errors(res[k][0].cpu().numpy(), ref, area_of(V, T))
        checked.append({"problem": w.name, "error_vs_oracle": e, "max_step_error_vs_oracle": emax})
    for p in probs:
        p.close()
    return {"problems": len(mix), "makespan_s": el, "solves_per_s": len(mix) / el, "rc": rc,
            "triangles": sorted({w.M for w in mix}), "steps": sorted({w.N for w in mix}),
            "total_arnoldi_steps": iters, "sampled_errors": checked,
            "max_sampled_error_vs_oracle": max(c["error_vs_oracle"] for c in checked)}


def run_serving(C, torch, ctx, rate, duration, large_frac=0.2, check_every=8):
    """Poisson stream of solve requests (seeded): sphere5120_N128_T6 requests
    and, with probability `large_frac`, sphere20480_N256_T6 ones, each with a
    random direction and pulse width, served by the continuous-batching loop
    with the operator cache; the large lane (second stream) solves requests
    whose stored dense operator would exceed a quarter of the budget -- the
    20480-triangle ones -- in the compressed form, refined with residuals of
    the plain operator, on half of the compute units.  Every `check_every`-th
    5120-triangle request carries the stored oracle workload's pulse and is
    compared with the oracle's solution."""
    from paper_2006_05186_amd.solver import Server
    # the server takes its arena with one device allocation: hand back what
    # torch's caching allocator still holds from earlier records
    gc.collect()
    torch.cuda.empty_cache()
    small, large = W.C3, W.C5_LARGE
    meshes = {small.name: small.mesh(), large.name: large.mesh()}
    ref = golden_q(small)
    area = area_of(*meshes[small.name])
    arrivals = W.poisson_arrivals(rate, duration)
    rng = np.random.default_rng(W.DEFAULT_SEED + 2)
    kinds = [large if rng.uniform() < large_frac else small for _ in arrivals]
    srv = Server(ctx, 200 << 30, max_active=16, mode=C.CQM_MIXED_PLAIN, form=C.CQM_FORM_DENSE,
                 large_lane=int(large_frac > 0))
    tickets = []
    nsmall = 0
    t0 = time.perf_counter()
    for a, wl in zip(arrivals, kinds):
        now = time.perf_counter() - t0
        if a > now:
            time.sleep(a - now)
        V, T = meshes[wl.name]
        checked = False
        if wl is small:
            checked = ref is not None and nsmall % check_every == 0
            nsmall += 1
        if checked:
            w = small.wave
            d, sigma, t0w = w.direction, w.sigma, w.t0
        else:
            d = W.random_direction(rng)
            sigma = float(rng.uniform(0.2, 0.4))
            t0w = 1.0 + 2 * sigma
        tickets.append((srv.submit(V, T, wl.N, wl.T, d, sigma, t0w), wl.name, checked))
    lat, rcs, errs, large_res = {}, [], [], []
    while len(lat) < len(tickets):
        for t, name, checked in tickets:
            if t not in lat:
                done, rc, q, dg, l = srv.poll(t)
                if done:
                    lat[t] = (l, name)
                    rcs.append(rc)
                    if name == large.name and done == 1:
                        large_res.append(dg.max_rel_residual)
                    if name == large.name or len(lat) == len(tickets):
                        print(f"served {len(lat)}/{len(tickets)} ({name}: {l:.0f} ms)",
                              file=sys.stderr, flush=True)
                    if checked and done == 1:
                        errs.append(errors(q, ref, area)[0])
        time.sleep(0.002)
    el = time.perf_counter() - t0
    st = srv.stats()
    srv.close()
    out = {"rate_per_s": rate, "duration_s": duration, "requests": len(tickets),
           "large_fraction": large_frac, "makespan_s": el, "solves_per_s": len(tickets) / el,
           "all_ok": all(r == C.CQM_OK for r in rcs), "lane_completed": st["lane_completed"],
           "operators_built": st["operators_built"], "cache_hits": st["operator_cache_hits"],
           "peak_active": st["peak_active"], "checked_requests": len(errs),
           "max_error_vs_oracle_checked": max(errs) if errs else None,
           # large requests are refined with residuals of the plain operator
           # (refine_plain): their largest final residual against it
           "large_max_plain_rel_residual": max(large_res) if large_res else None}
    for name in (small.name, large.name):
        L = np.asarray([l for l, n in lat.values() if n == name])
        if len(L):
            out[name] = {"count": int(len(L)), "p50_ms": float(np.percentile(L, 50)),
                         "p99_ms": float(np.percentile(L, 99)), "max_ms": float(L.max())}
    L = np.asarray([l for l, _ in lat.values()])
    out |= {"p50_ms": float(np.percentile(L, 50)), "p99_ms": float(np.percentile(L, 99))}
    return out


def tag_of(wl):
    return f"sphere{wl.M}_N{wl.N}"


def run_hypersingular(C, torch, ctx, wl, reps=5):
    """The hypersingular product D(s_l) x_l on the piecewise-linear space
    (cqm_apply_D, FP64) over every frequency of the band, timed by events
    after the once-per-mesh static parts; the far rate counts the 6 x 6
    point pairs of every ordered far pair of triangles per frequency."""
    from paper_2006_05186_amd.solver import Problem
    V, T = wl.mesh()
    p = Problem(ctx, V, T, wl.N, wl.T, formulation=C.CQM_FORMULATION_DIRECT)
    H = wl.N // 2 + 1
    x = torch.as_tensor(W.random_complex((H, len(V)), seed=5), device="cuda")
    st = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(st)
    p.apply_D(x)
    e1.record(st)
    torch.cuda.synchronize()
    t_first = e0.elapsed_time(e1) * 1e-3
    e0.record(st)
    for _ in range(reps):
        p.apply_D(x)
    e1.record(st)
    torch.cuda.synchronize()
    t_apply = e0.elapsed_time(e1) / reps * 1e-3
    p.close()
    # ordered pairs of triangles sharing a vertex (the near field)
    by_vertex = {}
    for i, tri in enumerate(T):
        for v in tri:
            by_vertex.setdefault(int(v), set()).add(i)
    near = sum(len(set().union(*(by_vertex[int(v)] for v in tri))) for tri in T)
    far_pairs = len(T) * len(T) - near
    return {"workload": wl.name, "vertices": len(V), "frequencies": H, "ms": t_apply * 1e3,
            "first_call_ms": t_first * 1e3, "far_point_pairs_per_s": far_pairs * 36 * H / t_apply,
            "near_pairs": near}


def far32_probe(C, torch, ctx, wl):
    """Kernel evaluation rate of the matrix-free FP32 far product (all
    distinct frequency systems active, no cut-off): cqm_apply_V timed by
    events."""
    from paper_2006_05186_amd.solver import Problem
    V, T = wl.mesh()
    # no cut-off: every far point-pair-frequency value is evaluated, so the
    # count of values per product is exactly far_units
    p = Problem(ctx, V, T, wl.N, wl.T, mode=C.CQM_MIXED_PLAIN, form=C.CQM_FORM_MATRIX_FREE,
                cutoff_inner=0.0, cutoff_outer=0.0)
    H = wl.N // 2 + 1
    x = torch.as_tensor(W.random_complex((H, len(T)), seed=3), device="cuda").to(torch.complex64)
    for _ in range(2):
        p.apply(x, 0, 32)
    torch.cuda.synchronize()
    st = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    reps = 5
    e0.record(st)
    for _ in range(reps):
        p.apply(x, 0, 32)
    e1.record(st)
    torch.cuda.synchronize()
    t_apply = e0.elapsed_time(e1) / reps * 1e-3
    u = C.cqm_operator_stats(p.handle).far_units
    p.close()
    tf = u * FLOPS_PER_UNIT / t_apply / 1e12
    return {"workload": wl.name, "ms": t_apply * 1e3, "units_per_s": u / t_apply,
            "entries_per_s": u / 36 / t_apply, "tflops": tf,
            "frac_fp32_peak": tf / PEAK_FP32_TFLOPS,
            "frac_fp32_unpacked_peak": tf / PEAK_FP32_UNPACKED_TFLOPS,
            "frac_of_measured_issue_ceiling": tf / ALU_PEAK_TFLOPS["far32"]}


def h2_apply_probe(C, torch, ctx, wl, reps=5):
    """The compressed operator of `wl` (m = 4, leaf size 32, eta = 1, eps
    1e-6, mixed) built once (MACA) and applied `reps` times in each
    precision to all frequencies, timed by events: the compressed kernels
    without a whole solve around them (for counter profiles)."""
    from paper_2006_05186_amd.solver import Problem
    V, T = wl.mesh()
    p = Problem(ctx, V, T, wl.N, wl.T, mode=C.CQM_MIXED_H2ACA)
    F = wl.N + 1
    x = torch.as_tensor(W.random_complex((F, len(T)), seed=5), device="cuda")
    p.apply(x, 0, 64)  # builds the operator
    torch.cuda.synchronize()
    st = torch.cuda.current_stream()
    out = {"workload": wl.name}
    for prec in (32, 64):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(st)
        for _ in range(reps):
            p.apply(x, 0, prec)
        e1.record(st)
        torch.cuda.synchronize()
        out[f"apply{prec}_ms"] = e0.elapsed_time(e1) / reps
    d = C.cqm_operator_stats(p.handle)
    out |= {"max_rank": d.max_rank, "mean_rank": d.mean_rank, "far_blocks": d.n_far_blocks,
            "near_blocks": d.n_near_blocks, "operator_GB": d.operator_bytes / 1e9}
    p.close()
    return out


def run_marching(C, torch, ctx, wl, steps=3, compressed=False, warmup=True):
    """The paper's time-marching solve (weights of eq. dft from the stored
    FP64 operator, history sums, conjugate gradients on What_0) of `wl`,
    against the stored all-at-once oracle solution (they agree to order
    rho^(N+1)).  compressed: the weights of the compressed operator instead
    (eq. fastdft: transformed MACA fibres; m = 4, eta = 1, eps 1e-6, FP32
    slices), whose approximation error stays in the answer."""
    from paper_2006_05186_amd.solver import Problem
    V, T = wl.mesh()
    mode = C.CQM_MIXED_H2ACA if compressed else C.CQM_FP64_PLAIN
    p = Problem(ctx, V, T, wl.N, wl.T, mode=mode, marching=1)
    p.set_plane_wave()
    if warmup:
        p.solve_marching()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        q, rc, d = p.solve_marching()
    torch.cuda.synchronize()
    el = (time.perf_counter() - t0) / steps
    out = {"workload": wl.name, "weights": "compressed" if compressed else "stored",
           "seconds_per_solve": el, "rc": rc, "cg_iterations": d.total_iters,
           "max_cg_per_step": d.max_iters, "t_setup_ms": d.t_setup_ms, "t_steps_ms": d.t_solve_ms,
           "weights_GB": d.operator_bytes / 1e9}
    ref = golden_q(wl)
    if ref is not None:
        out["error_vs_oracle_all_at_once"], out["max_step_error"] = errors(
            q.cpu().numpy(), ref, area_of(V, T))
    p.close()
    return out


def marching_compressed(C, torch, ctx, wl):
    """run_marching with the compressed weights; a step whose CG misses its
    tolerance is reported, not raised."""
    try:
        return run_marching(C, torch, ctx, wl, steps=1, compressed=True, warmup=False)
    except C.CqmError as e:
        return {"workload": wl.name, "weights": "compressed", "rc": e.code, "error": str(e)}


def tensor_error(C, torch, ctx, V, T, N, Tend, n_min, eta, m, eps):
    """Section 7.1's relative error e = ||V - V~||_F / ||V||_F of the
    compressed tensor over all (i, j, k), k = 0..N, formed exactly from the
    products of both operators with every unit vector (FP64; the plain
    operator without cut-off, its conjugate frequencies by reflection), with
    the compressed operator's ranks and storage.  Returns a dict."""
    from paper_2006_05186_amd.solver import Problem
    M, F = len(T), N + 1
    H = F // 2 + 1
    pd = Problem(ctx, V, T, N, Tend, mode=C.CQM_FP64_PLAIN, form=C.CQM_FORM_DENSE,
                 cutoff_inner=0.0, cutoff_outer=0.0)
    pc = Problem(ctx, V, T, N, Tend, mode=C.CQM_FP64_H2ACA, n_min=n_min, eta=eta, cheb_m=m,
                 eps_aca=eps)
    x = torch.zeros((F, M), dtype=torch.complex128, device="cuda")
    num = torch.zeros((), dtype=torch.float64, device="cuda")
    den = torch.zeros((), dtype=torch.float64, device="cuda")
    t0 = time.perf_counter()
    for j in range(M):
        x[:, j] = 1.0
        yh = pd.apply(x[:H], 0, 64)
        yd = torch.cat([yh, torch.conj(torch.flip(yh[1:F - H + 1], [0]))])
        yc = pc.apply(x, 0, 64)
        num += torch.sum(torch.abs(yc - yd) ** 2)
        den += torch.sum(torch.abs(yd) ** 2)
        x[:, j] = 0.0
    torch.cuda.synchronize()
    st = C.cqm_operator_stats(pc.handle)
    out = {"m": m, "eps": eps, "eta": eta, "e": float(torch.sqrt(num / den)),
           "max_rank": st.max_rank, "mean_rank": st.mean_rank, "far_blocks": st.n_far_blocks,
           "near_blocks": st.n_near_blocks, "bytes": st.operator_bytes,
           "storage_vs_dense": st.operator_bytes / (16.0 * M * M * F),
           "storage_vs_plain_h2": st.operator_bytes / max(st.h2_plain_bytes, 1),
           "seconds": time.perf_counter() - t0}
    pd.close()
    pc.close()
    return out


def run_study(C, torch, ctx):
    """The tensor-approximation study of Section 7.1 at reduced size: the
    unit-sphere polyhedron with 1280 triangles, N = 64 steps with
    dt / h = 0.83 (T = 8, the paper's Courant number), leaf size 32, the
    paper's eta = 2 and the configured eta = 1; e, ranks and storage against
    eps for m = 2, 3, 4, and along eps = 10^-m."""
    V, T = W.icosphere(3)
    N, Tend = 64, 8.0
    rows = []
    for eta in (2.0, 1.0):
        for m in (2, 3, 4):
            for k in range(2, 9):
                rows.append(tensor_error(C, torch, ctx, V, T, N, Tend, 32, eta, m, 10.0 ** -k))
                print(f"study eta={eta} m={m} eps=1e-{k}: e={rows[-1]['e']:.3e}", file=sys.stderr,
                      flush=True)
    return {"mesh_triangles": len(T), "N": N, "T": Tend, "n_min": 32, "rows": rows}


def alu_probe(blocks=256 * 16, iters=4096):
    """Lane-op rates of single VALU instructions (probes/alu_rate.hip), as
    operations per second and per compute unit per cycle (256 CUs, 2.4 GHz)."""
    import ctypes
    L = ctypes.CDLL(os.path.join(ROOT, "paper_2006_05186_amd", "lib", "libcqm_probe.so"))
    rates = (ctypes.c_double * 6)()
    rc = L.cqm_probe_alu_rates(0, blocks, iters, rates)
    if rc != 0:
        raise RuntimeError("ALU probe failed")
    names = ["v_exp_f32", "v_sin_f32", "v_cos_f32", "v_rsq_f32", "v_fma_f32", "v_fma_f64"]
    out = {"blocks": blocks, "threads": 256, "iters": iters, "chains": 8}
    for n, r in zip(names, rates):
        out[n] = {"lane_ops_per_s": r, "lane_ops_per_cu_cycle": r / (256 * 2.4e9)}
    return {"alu_probe": out}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=30)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="C3", choices=sorted(WORKLOADS))
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-variants", action="store_true")
    ap.add_argument("--serve-rate", type=float, default=1.0)
    ap.add_argument("--serve-seconds", type=float, default=30.0)
    ap.add_argument("--serve-large", type=float, default=0.2,
                    help="fraction of 20480-triangle requests in the serving stream")
    ap.add_argument("--serve-only", action="store_true",
                    help="only run the serving stream and print its record")
    ap.add_argument("--alu-probe", action="store_true",
                    help="only measure the lane-op rates of v_exp_f32, v_sin_f32, v_cos_f32, "
                         "v_rsq_f32 and FP32/FP64 FMA (lib/libcqm_probe.so) and exit")
    ap.add_argument("--part", choices=["far32", "compressed", "h2apply", "marching", "study",
                                       "batch48", "orders", "hypersingular"],
                    help="only run one piece on the workload (for counter profiles) and print "
                         "its record")
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
    if args.alu_probe:
        print(json.dumps(alu_probe()), flush=True)
        return
    wl = WORKLOADS[args.workload]
    ctx = C.cqm_ctx_create(0)
    if args.part:
        if args.part == "far32":
            rec = far32_probe(C, torch, ctx, wl)
        elif args.part == "h2apply":
            rec = h2_apply_probe(C, torch, ctx, wl)
        elif args.part == "batch48":
            rec = run_batch48(C, torch, ctx)
        elif args.part == "study":
            rec = run_study(C, torch, ctx)
        elif args.part == "orders":
            rec = run_orders(C, torch, ctx)
        elif args.part == "compressed":
            rec = run_compressed(C, torch, ctx)
        elif args.part == "hypersingular":
            rec = run_hypersingular(C, torch, ctx, wl)
        else:
            rec = [run_marching(C, torch, ctx, wl), marching_compressed(C, torch, ctx, wl)]
        C.cqm_ctx_destroy(ctx)
        print(json.dumps({args.part: rec}), flush=True)
        return
    if args.serve_only:
        rec = run_serving(C, torch, ctx, args.serve_rate, args.serve_seconds, args.serve_large)
        C.cqm_ctx_destroy(ctx)
        print(json.dumps({"serving": rec}), flush=True)
        return
    main_mode, main_form = C.CQM_MIXED_PLAIN, C.CQM_FORM_DENSE
    r = run_variant(C, Problem, ctx, wl, main_mode, main_form, args.steps, args.warmup, torch)
    K = args.steps
    value = K / r["elapsed"]
    lat_ms = np.asarray(r["lat"]) * 1e3
    d0 = r["diags"][-1]
    area = area_of(r["V"], r["T"])
    # Kernel durations come from HIP events recorded around every launch on
    # the solve stream; the event records cost part of a step, so they run
    # in a second pass of the same workload right after the timed steps
    # rather than inside them.
    KP = min(K, 10)
    rp = run_variant(C, Problem, ctx, wl, main_mode, main_form, KP, 1, torch, profile=1)
    rl = roofline(rp["diags"], tag_of(wl))
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
        # every class with GPU time against its own roofline
        "rooflines": {c: {k: v for k, v in roofline(rp["diags"], tag_of(wl), c).items()
                          if k not in ("kernel", "share_of_kernel_time")}
                      for c in ("assemble", "gemv32", "gemv64", "arnoldi")},
    }
    ref = golden_q(wl)
    if ref is not None:
        out["error_vs_oracle"], out["max_step_error_vs_oracle"] = errors(r["q"], ref, area)
    print(f"headline {wl.name}: {value:.2f} solves/s", file=sys.stderr, flush=True)
    if not args.no_variants:
        var = {}
        for name, mode, form, steps in (("fp64_dense", C.CQM_FP64_PLAIN, C.CQM_FORM_DENSE, 5),
                                        ("mixed_matrix_free", C.CQM_MIXED_PLAIN, C.CQM_FORM_MATRIX_FREE, 2),
                                        ("fp64_matrix_free", C.CQM_FP64_PLAIN, C.CQM_FORM_MATRIX_FREE, 1)):
            rv = run_variant(C, Problem, ctx, wl, mode, form, steps, 1, torch, profile=1)
            ms, calls = summarise_kernels(rv["diags"])
            v = {"solves_per_s": steps / rv["elapsed"]}
            for kn in ("far32", "far64", "assemble"):
                k = KCLS.index(kn)
                if calls[k]:
                    v[f"{kn}_avg_ms"] = ms[k] / calls[k]
            if ref is not None:
                v["error_vs_oracle"], v["max_step_error_vs_oracle"] = errors(rv["q"], ref, area)
            var[name] = v
            print(f"variant {name} done", file=sys.stderr, flush=True)
        var["far32_apply_probe"] = far32_probe(C, torch, ctx, wl)
        out["variants"] = var
        # the smaller plain configuration (1280 triangles, N = 64) as a sub-record
        c2 = W.C2
        r2 = run_variant(C, Problem, ctx, c2, main_mode, main_form, 30, 3, torch)
        rec2 = {"workload": c2.name, "solves_per_s": 30 / r2["elapsed"],
                "p50_ms": float(np.percentile(np.asarray(r2["lat"]) * 1e3, 50)),
                "p99_ms": float(np.percentile(np.asarray(r2["lat"]) * 1e3, 99))}
        ref2 = golden_q(c2)
        if ref2 is not None:
            rec2["error_vs_oracle"], rec2["max_step_error_vs_oracle"] = errors(
                r2["q"], ref2, area_of(r2["V"], r2["T"]))
        out["C2"] = rec2
        out["marching"] = [run_marching(C, torch, ctx, W.C2), run_marching(C, torch, ctx, wl, steps=1),
                           marching_compressed(C, torch, ctx, wl)]
        print("marching done", file=sys.stderr, flush=True)
        out["compressed"] = run_compressed(C, torch, ctx)
        print("compressed done", file=sys.stderr, flush=True)
        out["compressed_orders"] = run_orders(C, torch, ctx)
        out["hypersingular"] = run_hypersingular(C, torch, ctx, wl)
        out["batch48"] = run_batch48(C, torch, ctx)
        print("batch48 done", file=sys.stderr, flush=True)
        out["serving"] = run_serving(C, torch, ctx, args.serve_rate, args.serve_seconds,
                                     args.serve_large)
        print("serving done", file=sys.stderr, flush=True)
        # the 5120-triangle requests alone at 20 per second (C5's rate): the
        # continuously batched requests share one cached operator
        out["serving_5120_20per_s"] = run_serving(C, torch, ctx, 20.0, 10.0, large_frac=0.0)
        print("serving at 20/s done", file=sys.stderr, flush=True)
    C.cqm_ctx_destroy(ctx)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(wl)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
