"""The device serving pool: each request's result is the same alone and in a mix of uneven
lattice sizes (bitwise), matches the single-simulation path and the oracle, admission respects
the HBM budget, slots are reused while others run, and an unstable request is retired without
disturbing the others."""
import numpy as np
import pytest

from paper_1705_10045_amd import inputs as I
from paper_1705_10045_amd import lbm, serve
from parity import describe, rel_errors, run_oracle

pytestmark = pytest.mark.gpu

GIB = 1 << 30


def _req(i, edge, steps, kind="droplet", Tr=0.8):
    return dict(id=i, edge=edge, Tr=Tr, kind=kind, steps=steps, seed=I.SEED + 1 + i, noise=0.01)


def _run_pool(reqs, budget=2 * GIB, slots=16, spr=10, arrivals=None):
    with lbm.Pool(budget, max_slots=slots, steps_per_run=spr) as pool:
        ex = serve.PoolExecutor(pool)
        arr = np.zeros(len(reqs)) if arrivals is None else arrivals
        return serve.serve(reqs, arr, ex, keep_results=True)


def test_result_same_alone_and_in_mix():
    target = _req(0, 32, 57, "droplet", 0.78)
    others = [_req(1, 48, 33, "slab", 0.9), _req(2, 64, 80, "droplet", 0.72),
              _req(3, 32, 21, "slab", 0.85), _req(4, 48, 64, "droplet", 0.93)]
    alone = _run_pool([target])["results"][0]
    mix = _run_pool(others[:2] + [target] + others[2:])
    assert mix["completed"] == 5
    in_mix = mix["results"][2]
    for k in alone:
        assert np.array_equal(alone[k], in_mix[k]), k


def test_pool_matches_single_simulation_and_oracle():
    req = _req(5, 32, 40, "slab", 0.8)
    res = _run_pool([req])["results"][0]
    f = I.request_fields(req)
    with lbm.Sim(19, f["params"], f["rho0"], f["u0"], f["T0"], storage_bytes=4) as s:
        s.step(req["steps"])
        single = s.moments()
    for k in res:
        assert np.array_equal(res[k], single[k]), k
    o, _ = run_oracle(f, req["steps"])
    errs = rel_errors(res, o)
    describe("pool vs oracle", errs)
    assert max(errs.values()) < 1e-5


def test_pool_mixes_tau_values():
    """One batched launch serves requests with tau = 1 and tau != 1 (the collision decides per
    request whether to re-read N_k); each result equals its single simulation bit for bit."""
    reqs = [(_req(11, 32, 30, "droplet", 0.8), 0.8), (_req(12, 48, 30, "slab", 0.85), 1.0)]
    with lbm.Pool(2 * GIB, max_slots=4, steps_per_run=10) as pool:
        tickets = []
        for req, tau in reqs:
            f = I.request_fields(req, I.physics(tau=tau))
            tickets.append(pool.submit(f["params"], f["rho0"], f["u0"], f["T0"], req["steps"]))
        for _ in range(3):
            pool.run()
        results = [pool.collect(t)[0] for t in tickets]
    for (req, tau), res in zip(reqs, results):
        f = I.request_fields(req, I.physics(tau=tau))
        with lbm.Sim(19, f["params"], f["rho0"], f["u0"], f["T0"], storage_bytes=4) as s:
            s.step(req["steps"])
            single = s.moments()
        for k in res:
            assert np.array_equal(res[k], single[k]), (tau, k)


def test_admission_respects_budget_and_reuses_slots():
    params = I.physics()
    f32 = I.request_fields(_req(6, 32, 30))
    f64 = I.request_fields(_req(7, 64, 30))
    one32 = 2 * 2 * 19 * 32 ** 3 * 4
    with lbm.Pool(3 * one32 + (1 << 20), max_slots=8, steps_per_run=10) as pool:
        t = [pool.submit(params, f32["rho0"], f32["u0"], f32["T0"], 30) for _ in range(4)]
        assert t[3] is None and all(x is not None for x in t[:3])      # budget binds
        assert pool.submit(params, f64["rho0"], f64["u0"], f64["T0"], 30) is None
        st = pool.stats()
        assert st["bytes_in_use"] <= st["budget"] and st["active"] == 3
        for _ in range(3):
            pool.run()
        assert all(pool.poll(x)[0] for x in t[:3])
        for x in t[:3]:
            pool.collect(x)
        assert pool.stats()["bytes_in_use"] == 0
        again = pool.submit(params, f32["rho0"], f32["u0"], f32["T0"], 30)
        assert again is not None


def test_unstable_request_is_isolated():
    good = _req(8, 32, 30, "droplet", 0.8)
    shape = (24, 24, 24)
    bad_rho = I.two_phase(I.sphere_mask(shape, 5), 2.3, 0.02)
    with lbm.Pool(2 * GIB, max_slots=4, steps_per_run=10) as pool:
        fg = I.request_fields(good)
        tg = pool.submit(fg["params"], fg["rho0"], fg["u0"], fg["T0"], good["steps"])
        tb = pool.submit(I.physics(tau=0.501), bad_rho, I.uniform_velocity(shape, (0.3, 0, 0)),
                         np.full(shape, 0.6), 200)
        for _ in range(20):
            pool.run()
            if pool.poll(tg)[0] and pool.poll(tb)[0]:
                break
        assert pool.poll(tb) == (True, lbm.LBM_EUNSTABLE)
        assert pool.poll(tg) == (True, lbm.LBM_OK)
        res, st = pool.collect(tg)
        assert st == lbm.LBM_OK
        _, stb = pool.collect(tb)
        assert stb == lbm.LBM_EUNSTABLE
    alone = _run_pool([good])["results"][0]
    for k in res:
        assert np.array_equal(res[k], alone[k])


def test_continuous_arrivals_complete():
    reqs = I.serving_requests(24, steps_range=(20, 120), edges=(32, 48, 64))
    arr = serve.poisson_arrivals(len(reqs), rate=200.0)
    rep = _run_pool(reqs, budget=GIB, slots=8, spr=10, arrivals=arr)
    assert rep["completed"] == 24 and rep["failed"] == 0
    assert rep["peak_in_flight"] <= 8
    print("serving: p50 %.3fs p99 %.3fs %.0f MLUPS" % (rep["p50_s"], rep["p99_s"],
                                                       rep["aggregate_mlups"]), flush=True)


def test_admissions_and_collections_overlap_replay_in_flight():
    """With lbm_pool_run_async a replay stays in flight while requests are admitted (upload and
    initial state on the pool's second stream) and finished ones are collected.  Each result must
    still equal its single simulation bit for bit, whichever replay it joined."""
    reqs = [_req(20 + i, e, s, k, t) for i, (e, s, k, t) in enumerate(
        [(32, 35, "droplet", 0.8), (48, 23, "slab", 0.85), (32, 61, "slab", 0.75),
         (64, 17, "droplet", 0.9), (48, 44, "droplet", 0.82), (32, 12, "slab", 0.88)])]
    results = {}
    with lbm.Pool(2 * GIB, max_slots=3, steps_per_run=5) as pool:
        waiting = list(reqs)
        inflight = {}
        replays = 0
        while waiting or inflight:
            # admit one request per replay at most, so admissions land while a replay runs
            if waiting and pool.stats()["free_slots"] > 0:
                r = waiting.pop(0)
                f = I.request_fields(r)
                t = pool.submit(f["params"], f["rho0"], f["u0"], f["T0"], r["steps"])
                assert t is not None
                inflight[t] = r
            pool.run_async()
            replays += 1
            assert replays < 200
            for t in list(inflight):
                done, st = pool.poll(t)
                if done:
                    res, st = pool.collect(t)
                    assert st == lbm.LBM_OK
                    results[inflight.pop(t)["id"]] = res
        pool.run()   # nothing active: returns at once
    assert len(results) == len(reqs)
    for r in reqs:
        f = I.request_fields(r)
        with lbm.Sim(19, f["params"], f["rho0"], f["u0"], f["T0"], storage_bytes=4) as s:
            s.step(r["steps"])
            single = s.moments()
        for k in single:
            assert np.array_equal(results[r["id"]][k], single[k]), (r["id"], k)


def test_per_request_totals():
    """lbm_pool_totals: a finished request's totals at admission and at its end, as the single
    simulation's lbm_reduce gives them (the pool's state equals the single simulation's bit for
    bit, so they agree to the order of the FP64 sums), mass conserved over the run; a ticket
    that is still running is refused."""
    reqs = [_req(21, 32, 45, "droplet", 0.8), _req(22, 48, 30, "slab", 0.85)]
    with lbm.Pool(2 * GIB, max_slots=4, steps_per_run=10) as pool:
        tickets = []
        for req in reqs:
            f = I.request_fields(req)
            tickets.append(pool.submit(f["params"], f["rho0"], f["u0"], f["T0"], req["steps"]))
        pool.run()
        with pytest.raises(lbm.LbmError) as e:
            pool.totals(tickets[0])
        assert e.value.status == lbm.LBM_EBUSY
        for _ in range(4):
            pool.run()
        totals = [pool.totals(t) for t in tickets]
        for t in tickets:
            pool.collect(t)
    for req, (t0, t1) in zip(reqs, totals):
        f = I.request_fields(req)
        with lbm.Sim(19, f["params"], f["rho0"], f["u0"], f["T0"], storage_bytes=4) as s:
            r0 = s.reduce()
            s.step(req["steps"])
            r1 = s.reduce()
        mass = r0[0]
        assert np.abs(t0 - r0).max() <= 1e-12 * mass
        assert np.abs(t1 - r1).max() <= 1e-12 * mass
        assert abs(t1[0] - t0[0]) < 2e-8 * mass


def test_pool_serves_walls_and_gravity_beside_periodic_requests():
    """Pool-boiling requests (walls normal to z with held wall temperatures, gravity), at tau = 1
    and tau != 1, run in the pool beside a periodic droplet: the periodic request goes through
    the periodic launch and the others through the one with walls, and each result equals its
    single simulation bit for bit."""
    cases = [I.request_fields(_req(31, 32, 30, "droplet", 0.8)),
             I.pool_boiling_3d(shape=(40, 32, 32), gravity=1e-4),
             I.pool_boiling_3d(shape=(24, 20, 48), gravity=1e-4, params=I.physics(tau=0.8))]
    steps = [30, 40, 25]
    with lbm.Pool(2 * GIB, max_slots=4, steps_per_run=10) as pool:
        tickets = [pool.submit(c["params"], c["rho0"], c["u0"], c["T0"], n)
                   for c, n in zip(cases, steps)]
        for _ in range(4):
            pool.run()
        results = []
        for t in tickets:
            fields, st = pool.collect(t)
            assert st == lbm.LBM_OK
            results.append(fields)
    for c, n, res in zip(cases, steps, results):
        with lbm.Sim(19, c["params"], c["rho0"], c["u0"], c["T0"], storage_bytes=4) as s:
            s.step(n)
            single = s.moments()
        for k in res:
            assert np.array_equal(res[k], single[k]), (c["rho0"].shape, k)


def test_pool_serves_mrt_requests():
    """MRT requests (periodic, and with walls and gravity) beside a BGK one: each kind runs in
    its own launch of the batched step, and each result equals its single simulation bit for
    bit."""
    rates = dict(collision=lbm.LBM_COLLISION_MRT, s_e=1.19, s_eps=1.4, s_q=1.2, s_m=1.98)
    mrt = I.request_fields(_req(41, 32, 30, "droplet", 0.8), I.physics(tau=0.8))
    mrt["params"] = dict(mrt["params"], **rates)
    mrt_walls = I.pool_boiling_3d(shape=(24, 20, 40), gravity=1e-4, params=I.physics(tau=0.7))
    mrt_walls["params"] = dict(mrt_walls["params"], **rates)
    cases = [I.request_fields(_req(42, 48, 20, "slab", 0.85)), mrt, mrt_walls]
    steps = [20, 30, 25]
    with lbm.Pool(2 * GIB, max_slots=4, steps_per_run=10) as pool:
        tickets = [pool.submit(c["params"], c["rho0"], c["u0"], c["T0"], n)
                   for c, n in zip(cases, steps)]
        for _ in range(3):
            pool.run()
        results = []
        for t in tickets:
            fields, st = pool.collect(t)
            assert st == lbm.LBM_OK
            results.append(fields)
    for c, n, res in zip(cases, steps, results):
        with lbm.Sim(19, c["params"], c["rho0"], c["u0"], c["T0"], storage_bytes=4) as s:
            s.step(n)
            single = s.moments()
        for k in res:
            assert np.array_equal(res[k], single[k]), (c["rho0"].shape, k)
