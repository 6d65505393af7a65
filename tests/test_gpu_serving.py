"""Serving loop: requests that arrive while others run are admitted at cycle
boundaries; each result equals the same request solved alone; HBM-budget
admission queues or rejects; operators are shared through the cache."""
import sys
import time

import numpy as np
import pytest

import cqm_workloads as W
import oracle as O

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_2006_05186_amd import cqm as C  # noqa: E402
from paper_2006_05186_amd.solver import Problem, Server  # noqa: E402


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ctx():
    c = C.cqm_ctx_create(0)
    yield c
    C.cqm_ctx_destroy(c)


def requests(n, seed):
    """Requests on two meshes (so operators are shared) with random pulses."""
    rng = np.random.default_rng(seed)
    meshes = [(W.icosphere(2), 16, 2.0), (W.ellipsoid(1, (1.3, 0.8, 1.0)), 12, 2.0)]
    out = []
    for k in range(n):
        (V, T), N, Tend = meshes[k % 2]
        d = W.random_direction(rng)
        sigma = float(rng.uniform(0.2, 0.4))
        out.append((V, T, N, Tend, d, sigma, 1.0 + 2 * sigma))
    return out


def wait_all(srv, tickets, timeout=120.0):
    res = {}
    t0 = time.time()
    while len(res) < len(tickets):
        assert time.time() - t0 < timeout, "serving loop did not finish"
        for t in tickets:
            if t not in res:
                done, rc, q, d, lat = srv.poll(t)
                if done:
                    res[t] = (done, rc, q, d, lat)
        time.sleep(0.002)
    return res


def test_results_equal_alone_while_streaming(ctx):
    reqs = requests(8, seed=5)
    srv = Server(ctx, 2 << 30, max_active=4, mode=C.CQM_MIXED_PLAIN, form=C.CQM_FORM_DENSE)
    tickets = []
    for k, (V, T, N, Tend, d, sigma, t0) in enumerate(reqs):
        tickets.append(srv.submit(V, T, N, Tend, d, sigma, t0))
        time.sleep(0.003 * (k % 3))  # arrivals while others are on the GPU
    res = wait_all(srv, tickets)
    st = srv.stats()
    say(f"stats {st}")
    assert st["completed"] == 8 and st["operators_built"] == 2 and st["operator_cache_hits"] == 6
    assert st["peak_active"] >= 2
    for t, (V, T, N, Tend, d, sigma, t0) in zip(tickets, reqs):
        done, rc, q, diag, lat = res[t]
        assert done == 1 and rc == C.CQM_OK
        p = Problem(ctx, V, T, N, Tend, mode=C.CQM_MIXED_PLAIN, form=C.CQM_FORM_DENSE)
        p.set_plane_wave(d, sigma, t0)
        qa, rca, _ = p.solve()
        _, _, area = O.triangle_quadrature(V, T)
        e = O.rel_error(q, qa.cpu().numpy(), area)
        ref = O.solve(V, T, N, Tend, direction=d, sigma=sigma, t0=t0)
        e_or = O.rel_error(q, ref, area)
        say(f"  ticket {t}: latency {lat:.1f} ms, vs alone {e:.1e}, vs oracle {e_or:.1e}")
        assert e < 1e-12 and e_or < 1e-8
        p.close()
    srv.close()


def test_admission_by_budget_and_rejection(ctx):
    (V, T), N = W.icosphere(2), 16
    p = Problem(ctx, V, T, N, 2.0, mode=C.CQM_MIXED_PLAIN, form=C.CQM_FORM_DENSE)
    op_bytes = p.workspace_bytes
    p.close()
    # room for the operator (with its own state) and about one more request
    # state: requests must queue.  The dense mixed operator keeps the upper
    # triangle of 64 x 64 tiles of each of the Fsys slices, 24 B per entry.
    nt = (len(T) + 63) // 64
    state = op_bytes - (N // 2 + 1) * (nt * (nt + 1) // 2) * 64 * 64 * 24
    srv = Server(ctx, int(op_bytes + 1.5 * state), max_active=8, mode=C.CQM_MIXED_PLAIN,
                 form=C.CQM_FORM_DENSE)
    ts = [srv.submit(V, T, N, 2.0) for _ in range(4)]
    res = wait_all(srv, ts)
    st = srv.stats()
    say(f"budget stats {st}")
    assert all(r[0] == 1 and r[1] == C.CQM_OK for r in res.values())
    assert st["peak_active"] < 4 and st["peak_arena_bytes"] <= st["arena_bytes"]
    # a request that can never fit is rejected, later ones still run
    V3, T3 = W.icosphere(3)
    big = srv.submit(V3, T3, 32, 2.0)
    small = srv.submit(V, T, N, 2.0)
    res = wait_all(srv, [big, small])
    assert res[big][0] == -1 and res[big][1] == C.CQM_ENOMEM
    assert res[small][0] == 1
    srv.close()


def test_large_lane_compressed_beside_plain(ctx):
    """With the large lane on, a request whose stored dense operator exceeds
    the limit is solved in the compressed form on its own stream while the
    others keep streaming on the first lane; every result equals the same
    request solved alone in its form, and the large one (refined with the
    plain operator) equals the plain stored-form solution."""
    small = requests(4, seed=13)
    (VL, TL), NL, TLend = W.icosphere(3), 8, 2.0  # 1280 triangles: over the limit below
    nt = (len(TL) + 63) // 64
    limit = (NL // 2 + 1) * (nt * (nt + 1) // 2) * 64 * 64 * 24 - 1
    srv = Server(ctx, 24 << 30, max_active=8, mode=C.CQM_MIXED_PLAIN, form=C.CQM_FORM_DENSE,
                 large_lane=1, large_bytes=limit)
    say(f"large lane: limit {limit / 1e6:.1f} MB")
    tl = srv.submit(VL, TL, NL, TLend, (0.0, 0.6, 0.8), 0.3, 1.6)
    ts = [srv.submit(V, T, N, Tend, d, s, t0) for (V, T, N, Tend, d, s, t0) in small]
    res = wait_all(srv, [tl] + ts, timeout=300.0)
    st = srv.stats()
    say(f"  stats {st}")
    assert st["lane_completed"] == [4, 1]
    srv.close()
    assert res[tl][0] == 1 and res[tl][1] == C.CQM_OK
    p = Problem(ctx, VL, TL, NL, TLend, mode=C.CQM_MIXED_H2ACA)
    p.set_plane_wave((0.0, 0.6, 0.8), 0.3, 1.6)
    qa = p.solve()[0].cpu().numpy()
    p.close()
    _, _, area = O.triangle_quadrature(VL, TL)
    e = O.rel_error(res[tl][2], qa, area)
    p = Problem(ctx, VL, TL, NL, TLend, mode=C.CQM_FP64_PLAIN, form=C.CQM_FORM_DENSE)
    p.set_plane_wave((0.0, 0.6, 0.8), 0.3, 1.6)
    qp = p.solve()[0].cpu().numpy()
    p.close()
    e_plain = O.rel_error(res[tl][2], qp, area)
    say(f"  large request vs compressed alone {e:.1e}, vs plain stored form {e_plain:.1e}")
    assert e < 1e-12 and e_plain < 1e-7
    for t, (V, T, N, Tend, d, s, t0) in zip(ts, small):
        p = Problem(ctx, V, T, N, Tend, mode=C.CQM_MIXED_PLAIN, form=C.CQM_FORM_DENSE)
        p.set_plane_wave(d, s, t0)
        qa = p.solve()[0].cpu().numpy()
        p.close()
        _, _, area = O.triangle_quadrature(V, T)
        assert res[t][0] == 1 and O.rel_error(res[t][2], qa, area) < 1e-12


def test_serving_is_deterministic(ctx):
    reqs = requests(4, seed=9)
    outs = []
    for _ in range(2):
        srv = Server(ctx, 1 << 30, max_active=4, mode=C.CQM_MIXED_PLAIN, form=C.CQM_FORM_DENSE)
        ts = [srv.submit(V, T, N, Tend, d, s, t0) for (V, T, N, Tend, d, s, t0) in reqs]
        res = wait_all(srv, ts)
        outs.append([res[t][2] for t in ts])
        srv.close()
    for a, b in zip(*outs):
        assert np.array_equal(a, b)



def test_failed_lane_releases_and_refuses(ctx):
    # lane 0 is stopped from the host after one restart cycle (the
    # fail_after_cycles hook), as after a device error: its requests are
    # rejected with CQM_EDEVICE, their arena regions are given back, later
    # submits to it are refused at once, the other lane keeps serving, and
    # drain/destroy return instead of waiting forever
    say("serving: failed lane")
    srv = Server(ctx, 256 << 20, max_active=4, cache_operators=0, large_lane=1,
                 large_bytes=4 << 20, fail_after_cycles=1, mode=C.CQM_MIXED_PLAIN)
    Vs, Ts = W.icosphere(1)   # 80 triangles, N = 8: lane 0
    Vb, Tb = W.icosphere(2)   # 320 triangles, N = 16: above 4 MB dense, lane 1
    rng = np.random.default_rng(11)
    tickets = [srv.submit(Vs, Ts, 8, 2.0, W.random_direction(rng), 0.3, 1.6) for _ in range(3)]
    res = wait_all(srv, tickets, timeout=60.0)
    assert all(r[0] == -1 and r[1] == C.CQM_EDEVICE for r in res.values())
    with pytest.raises(C.CqmError) as e:
        srv.submit(Vs, Ts, 8, 2.0, (1.0, 0.0, 0.0), 0.3, 1.6)
    assert e.value.code == C.CQM_EDEVICE
    t = srv.submit(Vb, Tb, 16, 2.0, (0.0, 1.0, 0.0), 0.3, 1.6)
    done, rc, q, d, lat = wait_all(srv, [t], timeout=60.0)[t]
    assert done == 1 and rc == C.CQM_OK and np.all(np.isfinite(q))
    with pytest.raises(C.CqmError) as e:
        srv.drain()
    assert e.value.code == C.CQM_EDEVICE
    st = srv.stats()
    assert st["rejected"] == 3 and st["completed"] == 1 and st["active"] == 0
    assert st["arena_used"] == 0, st
    srv.close()
