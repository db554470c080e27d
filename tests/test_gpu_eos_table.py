"""The tabulated equation of state on the GPU (lbm_params.eos = LBM_EOS_TABLE; section 3 names
tabulated EOS of real fluids) against the oracle with the same table, element by element: the
reduced van der Waals EOS sampled on a 2048 x 501 grid (rho~ 0.01-2.6, T~ 0.5-1.0) with its
Maxwell band per row.  Real-fluid tables are not in this container (parity unpinned for them)."""
import numpy as np
import pytest

from eos_tables import vdw_table
from paper_1705_10045_amd import inputs as I
from paper_1705_10045_amd import lbm
from parity import compare, describe, run_gpu

pytestmark = pytest.mark.gpu

TOL = {4: 1e-5, 8: 1e-11}


def with_table(case, table=None):
    case = dict(case)
    case["params"] = dict(case["params"], eos_table=table or vdw_table())
    return case


@pytest.mark.parametrize("storage", [4, 8])
def test_droplet_with_table_against_oracle(storage):
    case = with_table(I.droplet_3d(shape=(28, 36, 40), radius=8.0))
    print("table EOS: D3Q19 droplet 40x36x28 %dB, 100 steps" % storage, flush=True)
    errs, *_ = compare(case, 100, storage)
    describe("table EOS droplet %dB" % storage, errs)
    assert max(errs.values()) < TOL[storage]


@pytest.mark.parametrize("storage", [4, 8])
def test_pool_boiling_with_table_against_oracle(storage):
    """Walls, held wall temperatures, gravity and the table together."""
    case = with_table(I.pool_boiling_3d(shape=(24, 20, 30), gravity=1e-4))
    print("table EOS: pool boiling 30x20x24 %dB, 100 steps" % storage, flush=True)
    errs, *_ = compare(case, 100, storage)
    describe("table EOS pool boiling %dB" % storage, errs)
    assert max(errs.values()) < TOL[storage]


@pytest.mark.parametrize("storage", [4, 8])
def test_d2q9_slab_with_table_against_oracle(storage):
    case = with_table(I.slab_2d(n=64, width=20, params=I.physics(tau=0.9)))
    print("table EOS: D2Q9 slab 64^2 tau 0.9 %dB, 100 steps" % storage, flush=True)
    errs, *_ = compare(case, 100, storage)
    describe("table EOS D2Q9 slab %dB" % storage, errs)
    assert max(errs.values()) < TOL[storage]


def test_table_of_vdw_follows_the_analytic_path_on_the_gpu():
    """The same droplet with the tabulated and the analytic van der Waals EOS on the GPU (FP64):
    they differ by the interpolation only, as in the oracle (1.1e-9 there after 40 steps)."""
    case = I.droplet_3d(shape=(20, 22, 24), radius=6.0, velocity=(0.03, 0.0, 0.0))
    a, _ = run_gpu(case, 40, 8)
    b, _ = run_gpu(with_table(case), 40, 8)
    for k in ("rho", "E", "T"):
        assert np.abs(a[k] - b[k]).max() / np.abs(a[k]).max() < 1e-8, k


@pytest.mark.parametrize("tau", [1.0, 0.8])
def test_table_launch_variants_are_bitwise_identical(tau):
    case = with_table(I.droplet_3d(shape=(21, 30, 45), radius=6.0, params=I.physics(tau=tau)))
    ref = None
    with lbm.Sim(case["Q"], case["params"], case["rho0"], case["u0"], case["T0"],
                 storage_bytes=4) as s:
        ck = s.checkpoint()
        for v in range(8):
            s.set_launch(v, 0)
            s.restore(ck)
            s.step(12)
            m = s.moments()
            if ref is None:
                ref = m
            for k in m:
                assert np.array_equal(m[k], ref[k]), (v, k)


def test_leaving_the_table_is_unstable():
    """A density outside the table's grid lies outside the EOS domain: an initial field there is
    refused (the droplet's vapour, 0.24, below a grid starting at 0.3), and a node that the flow
    carries below the grid (a diverging jet in vapour at 0.32; the oracle leaves the grid at
    step 2) is reported as LBM_EUNSTABLE."""
    table = vdw_table(rho_range=(0.3, 2.6))
    case = with_table(I.droplet_3d(shape=(16, 16, 16), radius=5.0), table)
    with pytest.raises(lbm.LbmError) as e:
        lbm.Sim(case["Q"], case["params"], case["rho0"], case["u0"], case["T0"])
    assert e.value.status == lbm.LBM_EINVAL and "outside the EOS table" in str(e.value)
    # inside at init, then a node is pushed below the grid by the flow
    rho = np.full((16, 16, 16), 0.32)
    u = np.zeros((3, 16, 16, 16))
    u[0, :, :, :8] = 0.2
    u[0, :, :, 8:] = -0.2
    p = dict(I.physics(), eos_table=table)
    with lbm.Sim(19, p, rho, u, np.full((16, 16, 16), 0.8)) as s:
        with pytest.raises(lbm.LbmError) as e:
            s.step(50)
        assert e.value.status == lbm.LBM_EUNSTABLE


def _single(case, steps):
    with lbm.Sim(19, case["params"], case["rho0"], case["u0"], case["T0"], storage_bytes=4) as s:
        s.step(steps)
        return s.moments()


def test_pool_runs_table_requests_beside_the_others():
    """The serving pool takes tabulated-EOS requests (BGK at tau = 1 and 0.8, MRT, walls and
    gravity) in their own batched launches beside a van der Waals request in the same replays:
    each result equals its single simulation's bit for bit.  The request keeps its own copy of
    the table: the caller's arrays are overwritten after submission."""
    def own():
        t = vdw_table()
        return dict(t, p=t["p"].copy(), coex=t["coex"].copy())

    mrt = dict(collision=lbm.LBM_COLLISION_MRT, s_e=1.19, s_eps=1.4, s_q=1.2, s_m=1.98)
    cases = [
        I.droplet_3d(shape=(16, 16, 16), radius=4.0),
        with_table(I.droplet_3d(shape=(16, 20, 24), radius=5.0, velocity=(0.03, 0.0, 0.0)), own()),
        with_table(I.droplet_3d(shape=(18, 16, 20), radius=5.0, params=I.physics(tau=0.8)), own()),
        with_table(I.pool_boiling_3d(shape=(20, 16, 24), gravity=1e-4), own()),
    ]
    cases[2]["params"] = dict(cases[2]["params"], **mrt)
    steps = 10
    singles = [_single(c, steps) for c in cases]
    with lbm.Pool(1 << 29, max_slots=8, steps_per_run=5) as pool:
        tickets = []
        for c in cases:
            tickets.append(pool.submit(c["params"], c["rho0"], c["u0"], c["T0"], steps))
            tab = c["params"].get("eos_table")
            if tab is not None:
                tab["p"][...] = np.nan
                tab["coex"][...] = np.nan
        print("pool: 1 vdW + 3 table requests, %d steps" % steps, flush=True)
        pool.run()
        pool.run()
        for i, (t, ref) in enumerate(zip(tickets, singles)):
            res, st = pool.collect(t)
            assert st == lbm.LBM_OK, i
            for k in res:
                assert np.array_equal(res[k], ref[k]), (i, k)


def test_pool_reports_a_table_request_leaving_the_grid():
    """The diverging jet in vapour at rho~ = 0.32 with a table starting at 0.3 (the single
    simulation's case above) leaves the grid in the pool too: collect returns LBM_EUNSTABLE for
    it, and a van der Waals request in the same replays finishes normally."""
    table = vdw_table(rho_range=(0.3, 2.6))
    rho = np.full((16, 16, 16), 0.32)
    u = np.zeros((3, 16, 16, 16))
    u[0, :, :, :8] = 0.2
    u[0, :, :, 8:] = -0.2
    ok = I.droplet_3d(shape=(16, 16, 16), radius=4.0)
    with lbm.Pool(1 << 28, max_slots=4, steps_per_run=10) as pool:
        bad = pool.submit(dict(I.physics(), eos_table=table), rho, u, np.full((16, 16, 16), 0.8), 50)
        good = pool.submit(ok["params"], ok["rho0"], ok["u0"], ok["T0"], 50)
        print("pool: table request leaving the grid beside a vdW request", flush=True)
        for _ in range(5):
            pool.run()
        _, st = pool.collect(bad)
        assert st == lbm.LBM_EUNSTABLE
        res, st = pool.collect(good)
        assert st == lbm.LBM_OK
    assert np.array_equal(res["rho"], _single(ok, 50)["rho"])

def test_pool_budget_counts_the_table_copy():
    """A table request's footprint is its two population buffers plus its copy of the table
    (rounded up to the arena's 256-byte alignment): a budget one alignment unit short of that
    declines it (LBM_EBUSY, nothing allocated) and still admits the same box with the van der
    Waals EOS."""
    table = vdw_table()
    nT, nrho = table["p"].shape
    table_bytes = -(-8 * (nrho * nT + 2 * nT) // 256) * 256
    plain = I.droplet_3d(shape=(16, 16, 16), radius=4.0)
    tab = with_table(plain, table)
    with lbm.Pool(1 << 28, max_slots=4, steps_per_run=5) as pool:
        a = pool.submit(plain["params"], plain["rho0"], plain["u0"], plain["T0"], 5)
        state = pool.stats()["bytes_in_use"]
        b = pool.submit(tab["params"], tab["rho0"], tab["u0"], tab["T0"], 5)
        assert pool.stats()["bytes_in_use"] == 2 * state + table_bytes
        pool.run()
        for t in (a, b):
            assert pool.collect(t)[1] == lbm.LBM_OK
        assert pool.stats()["bytes_in_use"] == 0
    with lbm.Pool(state + table_bytes - 256, max_slots=4, steps_per_run=5) as pool:
        assert pool.submit(tab["params"], tab["rho0"], tab["u0"], tab["T0"], 5) is None
        assert pool.stats()["bytes_in_use"] == 0
        assert pool.submit(plain["params"], plain["rho0"], plain["u0"], plain["T0"], 5) is not None
