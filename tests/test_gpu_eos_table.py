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
        for v in range(7):
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


def test_pool_refuses_table():
    table = vdw_table()
    f = I.request_fields(dict(id=0, edge=32, Tr=0.8, kind="droplet", steps=10, seed=I.SEED + 1,
                              noise=0.01))
    with lbm.Pool(1 << 30, max_slots=2, steps_per_run=5) as pool:
        with pytest.raises(lbm.LbmError) as e:
            pool.submit(dict(f["params"], eos_table=table), f["rho0"], f["u0"], f["T0"], 10)
        assert e.value.status == lbm.LBM_EINVAL
