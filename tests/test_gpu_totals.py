"""lbm_step_reduce: the totals of the state (mass, momentum, internal energy; the stored
post-collision populations of eq:edm summed in FP64) formed inside the last step, against the
plain step followed by the separate reduction on a twin simulation.

The fields must be bitwise those of the plain step.  The totals sum the same stored values in
another order: each node's sum of FP32 values is exact in FP64, so the two differ only by the
rounding of the sums over nodes, ~1e-16 relative per addition; the bound below is 1e-12 of the
total mass for mass and momentum (momenta can be ~0) and 1e-12 of the energy."""
import numpy as np
import pytest

from eos_tables import vdw_table
from paper_1705_10045_amd import inputs as I
from paper_1705_10045_amd import lbm

pytestmark = pytest.mark.gpu


def _twins(case, storage, steps, variant=None, chunk=0):
    args = (case["Q"], case["params"], case["rho0"], case["u0"], case["T0"])
    with lbm.Sim(*args, storage_bytes=storage) as a, lbm.Sim(*args, storage_bytes=storage) as b:
        if variant is not None:
            a.set_launch(variant, chunk)
            b.set_launch(variant, chunk)
        ta = a.step_reduce(steps)
        b.step(steps)
        tb = b.reduce()
        assert lbm.lbm_step_count(a._h) == lbm.lbm_step_count(b._h) == steps
        ma, mb = a.moments(), b.moments()
        # the state after the fused step is the plain step's, so its own reduction agrees bitwise
        ra = a.reduce()
    for k in ("rho", "u_star", "E", "T"):
        assert np.array_equal(ma[k], mb[k]), k
    assert np.array_equal(ra, tb)
    return ta, tb


def _check_totals(ta, tb):
    mass = abs(tb[0])
    assert np.abs(ta[:4] - tb[:4]).max() <= 1e-12 * mass, (ta, tb)
    assert abs(ta[4] - tb[4]) <= 1e-12 * abs(tb[4]), (ta, tb)


CASES = {
    "droplet": lambda: I.droplet_3d(shape=(28, 36, 40), radius=8.0, velocity=(0.03, 0.01, 0.0)),
    "droplet_tau": lambda: I.droplet_3d(shape=(28, 36, 40), radius=8.0, params=I.physics(tau=0.8)),
    "pool_boiling": lambda: I.pool_boiling_3d(shape=(24, 20, 30), gravity=1e-4),
    "slab_d2q9": lambda: I.slab_2d(n=96, width=30, params=I.physics(tau=0.9)),
}


@pytest.mark.parametrize("storage", [4, 8])
@pytest.mark.parametrize("name", sorted(CASES))
def test_fused_totals_match_the_separate_reduction(name, storage):
    case = CASES[name]()
    print("step_reduce: %s %dB, 30 steps" % (name, storage), flush=True)
    ta, tb = _twins(case, storage, 30)
    _check_totals(ta, tb)


@pytest.mark.parametrize("storage", [4, 8])
def test_fused_totals_with_mrt_and_the_table(storage):
    case = I.droplet_3d(shape=(20, 22, 24), radius=6.0, params=I.physics(tau=0.8))
    case["params"] = dict(case["params"], collision=lbm.LBM_COLLISION_MRT, s_e=1.19, s_eps=1.4,
                          s_q=1.2, s_m=1.98, eos_table=vdw_table())
    print("step_reduce: MRT + table EOS %dB" % storage, flush=True)
    ta, tb = _twins(case, storage, 20)
    _check_totals(ta, tb)


@pytest.mark.parametrize("variant", [5, 7, 3])
def test_fused_totals_global_addressing_and_fallback(variant):
    """Variants 5 and 7 (global addressing on 32 x 16 and 64 x 8 tiles, the forms of states of
    4 GB and more) have the fused form; variant 3 has none and runs the step and then the
    separate reduction."""
    case = CASES["droplet"]()
    ta, tb = _twins(case, 4, 12, variant=variant)
    _check_totals(ta, tb)


@pytest.mark.parametrize("variant", [0, 2])
def test_fused_totals_d2q9_tile_shapes(variant):
    """D2Q9 FP32 on 32 x 8 tiles (the default) and 64 x 8 tiles, both with the fused form."""
    case = I.slab_2d(n=768, width=240)
    ta, tb = _twins(case, 4, 10, variant=variant)
    _check_totals(ta, tb)


def test_fused_totals_at_128_in_bench_launch():
    case = I.droplet_3d(n=128, radius=24.0, Tr=0.8, noise=0.005, velocity=(0.05, 0.0, 0.0))
    print("step_reduce: droplet 128^3 4B, 10 steps", flush=True)
    ta, tb = _twins(case, 4, 10)
    _check_totals(ta, tb)


def test_fused_totals_track_conservation_over_calls():
    """Totals every 25 steps through the fused step: the same trajectory as the plain step, and
    mass conserved to FP32 rounding of the stored values."""
    case = CASES["droplet"]()
    args = (case["Q"], case["params"], case["rho0"], case["u0"], case["T0"])
    with lbm.Sim(*args, storage_bytes=4) as a, lbm.Sim(*args, storage_bytes=4) as b:
        m0 = a.reduce()[0]
        for _ in range(4):
            ta = a.step_reduce(25)
            b.step(25)
            _check_totals(ta, b.reduce())
            assert abs(ta[0] - m0) < 2e-8 * m0


def test_step_reduce_rejects_bad_arguments():
    case = CASES["droplet"]()
    with lbm.Sim(case["Q"], case["params"], case["rho0"], case["u0"], case["T0"], storage_bytes=4) as s:
        with pytest.raises(lbm.LbmError):
            s.step_reduce(0)
        assert lbm.lbm_step_count(s._h) == 0
