"""Long runs of the three single-box workloads on the GPU path.

  - D2Q9 slab 128^2, FP64 storage, 1000 steps: element-wise parity with the FP64 oracle (the
    drift of rounding differences over a long run stays far below the 1e-11 bar);
  - D3Q19 droplet 128^3 moving at u = 0.05 for 2000 steps, 100 nodes: Galilean invariance
    against the same droplet at rest, shifted by 100 nodes (to within the model's own error:
    the moving drop runs a quarter of a node ahead);
  - D3Q19 spinodal 256^3, 5000 steps in FP32 and in FP64 storage: the decomposition is chaotic,
    so the two storages are compared through the statistics of the phases (liquid fraction,
    phase-mean temperatures), not node by node.  This long run starts at T~ = 0.8: from the
    benchmark's T~ = 0.75 the pressure work cools the vapour to T~ ~ 0.43 and a node leaves the
    equation of state's domain after about 700 steps, in the FP64 oracle (32^3) as on the GPU
    (64^3 to 256^3, both storages), while the pseudoforces alone keep it stable.
"""
import numpy as np
import pytest

from paper_1705_10045_amd import inputs as I
from paper_1705_10045_amd import lbm

from parity import compare, describe

pytestmark = pytest.mark.gpu


def test_d2q9_slab_fp64_1000_steps_against_oracle():
    errs, g, o, gt, ot = compare(I.slab_2d(), 1000, 8)
    describe("D2Q9 slab 128^2 8B, 1000 steps", errs)
    assert max(errs.values()) < 1e-11
    assert abs(gt[0] - ot[0]) < 1e-13 * ot[0]


def _moments_after(case, steps, storage=4, fields=("rho", "T")):
    with lbm.Sim(case["Q"], case["params"], case["rho0"], case["u0"], case["T0"],
                 storage_bytes=storage) as s:
        s.step(steps)
        m = s.moments()
        return {k: np.array(m[k], copy=True) for k in fields}


def _centroid_x(rho, threshold):
    """Circular mean of the x index over the liquid nodes of a periodic box."""
    n = rho.shape[2]
    xs = np.nonzero(rho > threshold)[2]
    return (np.angle(np.exp(2j * np.pi * xs / n).mean()) * n / (2 * np.pi)) % n


def test_droplet_128_moves_100_nodes_like_the_resting_one():
    steps, u = 2000, 0.05
    move = _moments_after(I.droplet_3d(velocity=(u, 0.0, 0.0)), steps)
    rest = _moments_after(I.droplet_3d(velocity=(0.0, 0.0, 0.0)), steps)
    shifted = {k: np.roll(v, int(round(u * steps)), axis=2) for k, v in rest.items()}
    rv, rl = I.coexistence(0.8)
    mid = 0.5 * (rv + rl)
    lag = (_centroid_x(move["rho"], mid) - _centroid_x(shifted["rho"], mid) + 64) % 128 - 64
    drho = np.abs(move["rho"] - shifted["rho"]).max() / (rl - rv)
    dT = np.abs(move["T"] - shifted["T"]).max()
    liq_move = (move["rho"] > mid).sum()
    liq_rest = (rest["rho"] > mid).sum()
    print("droplet 128^3 after %d steps at u = %.2f: centroid %.3f nodes from the shifted "
          "resting drop, max|drho|/(rho_l - rho_v) %.3e, max|dT| %.3e, liquid nodes %d vs %d"
          % (steps, u, lag, drho, dT, liq_move, liq_rest), flush=True)
    # measured: 0.26 nodes ahead (the model's own Galilean error, as for the 2D drop of Fig. 7),
    # 5.9% of the density jump at the interface that this offset moves, dT 1.9e-3
    assert abs(lag) < 0.4
    assert drho < 0.1
    assert dT < 5e-3
    assert abs(liq_move - liq_rest) < 0.005 * liq_rest


def test_spinodal_256_5000_steps_fp32_and_fp64_agree_statistically():
    case = I.spinodal_3d(Tr=0.8)
    stats = {}
    for storage in (4, 8):
        m = _moments_after(case, 5000, storage)
        rho, T = m["rho"], m["T"]
        rv, rl = I.coexistence(0.8)
        mid = 0.5 * (rv + rl)
        liq = rho > mid
        stats[storage] = (liq.mean(), T[liq].mean(), T[~liq].mean(), rho[liq].mean(),
                          rho[~liq].mean())
        del m, rho, T, liq
        print("spinodal 256^3 %dB, 5000 steps: liquid fraction %.4f, T_liq %.4f, T_vap %.4f, "
              "rho_liq %.4f, rho_vap %.4f" % ((storage,) + stats[storage]), flush=True)
    a, b = stats[4], stats[8]
    assert abs(a[0] - b[0]) < 2e-3
    for x, y in zip(a[1:], b[1:]):
        assert abs(x - y) < 2e-3


def test_pool_boiling_128_2000_steps_heats_from_the_bottom():
    """The 128^3 pool-boiling workload for 2000 steps: it stays inside the equation of state's
    domain, conserves mass to FP32 rounding, and takes in heat.  The hot bottom wall faces the
    liquid, whose conductance rho c_v chi is about eight times that of the vapour under the cold
    top wall, so the total energy grows and the plane next to the bottom ends between the
    liquid's initial and the wall's temperature."""
    case = I.pool_boiling_3d(n=128)
    p = case["params"]
    with lbm.Sim(case["Q"], p, case["rho0"], case["u0"], case["T0"]) as s:
        t0 = s.reduce()
        s.step(2000)
        t1 = s.reduce()
        m = s.moments()
    T_bottom_plane = m["T"][0].mean()
    print("pool boiling 128^3, 2000 steps: mass %.3e rel, energy %.6g -> %.6g, bottom plane "
          "T %.4f, T range [%.4f, %.4f]" % ((t1[0] - t0[0]) / t0[0], t0[4], t1[4], T_bottom_plane,
                                           m["T"].min(), m["T"].max()), flush=True)
    assert abs(t1[0] - t0[0]) < 1e-7 * t0[0]
    assert t1[4] > t0[4]
    assert 0.8 * p["T_c"] < T_bottom_plane < p["T_bottom"]
    assert np.isfinite(m["T"]).all()


# The 256^3 spinodal at its listed T~ = 0.75 with c_v = 8 p_c (gamma = 4/3).  With c_v = 4 p_c
# the pressure work cools the vapour out of the EOS domain within about 700 steps, in the oracle
# (32^3) as on the GPU; the paper does not fix c_v, and with twice the heat capacity the same
# work cools half as much: the oracle runs 5000 steps of this state at 32^3 and 64^3.
CV_T075 = 8.0 * I.P_C


def test_spinodal_256_at_t075_5000_steps_fp32_and_fp64_agree_statistically():
    case = I.spinodal_3d(Tr=0.75, params=I.physics(c_v=CV_T075))
    stats = {}
    for storage in (4, 8):
        print("spinodal 256^3 T~ 0.75 c_v 8 p_c %dB, 5000 steps" % storage, flush=True)
        m = _moments_after(case, 5000, storage)
        rho, T = m["rho"], m["T"]
        rv, rl = I.coexistence(0.75)
        mid = 0.5 * (rv + rl)
        liq = rho > mid
        stats[storage] = (liq.mean(), T[liq].mean(), T[~liq].mean(), rho[liq].mean(),
                          rho[~liq].mean())
        assert np.isfinite(T).all() and np.isfinite(rho).all()
        del m, rho, T, liq
        print("spinodal 256^3 T~ 0.75 %dB, 5000 steps: liquid fraction %.4f, T_liq %.4f, "
              "T_vap %.4f, rho_liq %.4f, rho_vap %.4f" % ((storage,) + stats[storage]), flush=True)
    a, b = stats[4], stats[8]
    assert abs(a[0] - b[0]) < 2e-3
    for x, y in zip(a[1:], b[1:]):
        assert abs(x - y) < 2e-3
    # the pressure work cools the vapour below the liquid (sections 6.2-6.3)
    assert a[2] < a[1]
