"""The C-ABI library: it loads without a GPU, exports every entry point declared in
include/*.h, and its host-only pieces (lattice tables, Maxwell table, parameter and field
validation) behave as documented.  No kernel is launched here."""
import ctypes
import glob
import os
import re

import numpy as np
import pytest

from paper_1705_10045_amd import inputs as I
from paper_1705_10045_amd import lbm

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_functions():
    names = set()
    for h in glob.glob(os.path.join(ROOT, "include", "*.h")):
        text = open(h).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        for m in re.finditer(r"\b(lbm_[a-z_]+)\s*\(", text):
            names.add(m.group(1))
    return names


def test_library_exports_every_declared_symbol():
    L = lbm.lib()
    declared = _declared_functions()
    assert len(declared) >= 20
    missing = [n for n in sorted(declared) if not hasattr(L, n)]
    assert not missing, missing
    bound = {name for name, _, _ in lbm._SIGNATURES}
    assert declared == bound


@pytest.mark.parametrize("Q", [9, 19])
def test_library_lattice_matches_identities(Q):
    """The library's velocity set satisfies the same isotropy identities the oracle's does."""
    c, w, G, alpha, D = lbm.lbm_lattice_info(Q)
    cf = c[:, :D].astype(float)
    assert w.sum() == pytest.approx(1.0, abs=1e-15)
    assert np.allclose(np.einsum("k,ka,kb->ab", w, cf, cf), np.eye(D) / 3, atol=1e-15)
    assert np.allclose(np.einsum("k,ka,kb->ab", G, cf, cf), 2 * alpha * np.eye(D))
    m4 = np.einsum("k,ka,kb,kc,kd->abcd", w, cf, cf, cf, cf)
    I3 = np.eye(D)
    iso = (np.einsum("ab,cd->abcd", I3, I3) + np.einsum("ac,bd->abcd", I3, I3)
           + np.einsum("ad,bc->abcd", I3, I3)) / 9
    assert np.allclose(m4, iso, atol=1e-15)
    assert len({tuple(v) for v in c}) == Q and (c[0] == 0).all()


def test_library_maxwell_table_matches_oracle(orc):
    for Tr in (0.4, 0.55, 0.7, 0.75, 0.8, 0.8123, 0.9, 0.97, 0.995, 0.999):
        rv, rl = lbm.lbm_coexistence(Tr)
        ov, ol, _ = orc.maxwell(Tr)
        assert rv == pytest.approx(ov, rel=1e-11, abs=1e-12)
        assert rl == pytest.approx(ol, rel=1e-11, abs=1e-12)
    with pytest.raises(lbm.LbmError):
        lbm.lbm_coexistence(0.3)


def _case():
    d = I.droplet_3d(shape=(8, 9, 10), radius=2.5)
    return d["params"], d["rho0"], d["u0"], d["T0"]


@pytest.mark.parametrize("bad", [dict(tau=0.5), dict(tau_E=0.45), dict(chi=0.2), dict(p_c=-1.0),
                                 dict(c_v=0.0)])
def test_init_rejects_bad_parameters_before_touching_a_device(bad):
    phys, rho, u, T = _case()
    p = lbm.make_params(19, rho.shape, dict(phys, **bad))
    with pytest.raises(lbm.LbmError) as e:
        lbm.lbm_init(p, rho, u, T)
    assert e.value.status == lbm.LBM_EINVAL
    assert lbm.lbm_last_error()


def test_init_rejects_bad_fields():
    phys, rho, u, T = _case()
    p = lbm.make_params(19, rho.shape, phys)
    for r, t in ((np.where(rho > 1, 3.2, rho), T), (rho, -T), (rho * np.nan, T)):
        with pytest.raises(lbm.LbmError):
            lbm.lbm_init(p, r, u, t)
    # Phi^2 = rho/3 - p <= 0: a dense cold liquid with a large critical pressure
    p2 = lbm.make_params(19, rho.shape, dict(phys, p_c=0.5))
    with pytest.raises(lbm.LbmError) as e:
        lbm.lbm_init(p2, np.full(rho.shape, 0.5), u, np.full(rho.shape, 2.0))
    assert "Phi" in str(e.value) or "stability" in str(e.value)
    # lattice / shape mismatch
    p3 = lbm.make_params(9, rho.shape, phys)
    with pytest.raises(lbm.LbmError):
        lbm.lbm_init(p3, rho, u, T)


def test_stability_criterion_enforced():
    """Section 3: (dp/drho)_T <= (h/dt)^2 + theta.  A liquid with p_c large enough to break it
    is rejected at init."""
    phys, rho, u, T = _case()
    p = lbm.make_params(19, rho.shape, dict(phys, p_c=0.2, c_v=0.8))
    with pytest.raises(lbm.LbmError) as e:
        lbm.lbm_init(p, np.full(rho.shape, 2.3), u, np.full(rho.shape, 0.6))
    assert "stability" in str(e.value)


def test_footprint():
    phys, rho, u, T = _case()
    p = lbm.make_params(19, (128, 128, 128), phys)
    fp = lbm.lbm_footprint_bytes(p)
    assert fp >= 2 * 2 * 19 * 128 ** 3 * 4
    assert fp < 2 * 2 * 19 * 128 ** 3 * 4 * 1.01


def test_init_rejects_a_population_plane_over_4gb():
    """The step addresses nodes within one population plane with 32-bit byte offsets: a box whose
    plane exceeds 4 GB (far beyond what fits in HBM anyway) is refused before any field is read."""
    phys, rho, u, T = _case()
    p = lbm.make_params(19, (1024, 1024, 1024), phys, storage_bytes=4)
    h = ctypes.c_void_p()
    st = lbm.lib().lbm_init(ctypes.byref(p), None, None, None, None, ctypes.byref(h))
    assert st == lbm.LBM_EINVAL
    assert "4 GB" in lbm.lbm_last_error()
    assert not h.value


@pytest.mark.parametrize("change, message", [
    (dict(walls=2), "walls must be 0"),
    (dict(walls=1, wall_heat=1, T_bottom=0.8, chi=0.15), "1/(2d + 1)"),
    (dict(walls=1, wall_heat=2, T_top=-1.0), "held wall temperature"),
    (dict(gravity=(0.0, float("nan"), 0.0)), "gravity must be finite"),
    (dict(collision=2), "collision must be"),
    (dict(collision=1, s_e=2.0), "MRT rates"),
    (dict(collision=1, s_q=0.0), "MRT rates"),
])
def test_init_rejects_bad_walls_body_force_and_collision(change, message):
    """Wall, body-force and collision parameters are validated before any field is read or any
    device is touched: walls other than 0/1, chi too large next to a held wall (its face is half
    a cell away), a non-positive held wall temperature, a non-finite gravity, an unknown
    collision, an MRT rate outside (0, 2)."""
    phys, rho, u, T = _case()
    phys = dict(phys, **change)
    p = lbm.make_params(19, (8, 6, 5), phys, storage_bytes=4)
    h = ctypes.c_void_p()
    st = lbm.lib().lbm_init(ctypes.byref(p), None, None, None, None, ctypes.byref(h))
    assert st == lbm.LBM_EINVAL
    assert message in lbm.lbm_last_error()
    assert not h.value


def test_init_rejects_walls_on_d2q9():
    phys, rho, u, T = _case()
    p = lbm.make_params(9, (1, 6, 5), dict(phys, walls=1), storage_bytes=4)
    h = ctypes.c_void_p()
    st = lbm.lib().lbm_init(ctypes.byref(p), None, None, None, None, ctypes.byref(h))
    assert st == lbm.LBM_EINVAL
    assert "walls need D3Q19" in lbm.lbm_last_error()


def _rounds_cost(nz, cols, target=256):
    """Rounds of `target` resident workgroups times (chunk + 4) planes for every chunk count:
    the launch plan must take a chunk of least cost (fewest chunks among equals)."""
    best = None
    for nc in range(1, max(nz // 4, 1) + 1):
        c = -(-nz // nc)
        chunks = -(-nz // c)
        cost = -(-cols * chunks // target) * (c + 4)
        if best is None or cost < best[0]:
            best = (cost, c)
    return best[1]


@pytest.mark.parametrize("shape,expect", [
    ((512, 512, 512), (64, 8, 512, 512)),
    ((128, 128, 128), (32, 16, 16, 256)),
    ((256, 256, 256), (32, 16, 128, 256)),
    ((288, 288, 288), (32, 16, 96, 486)),
    ((320, 320, 320), (64, 8, 64, 1000)),
    ((300, 300, 300), (64, 8, 75, 760)),
    ((1024, 320, 96), (32, 16, 256, 240)),
])
def test_launch_plan_of_d3q19_boxes(shape, expect):
    """The host-only launch plan (no device): 32 x 16 tiles, or 64 x 8 for FP32 states of 4 GB
    and more (288^3 is 3.6 GB) unless 64-wide tiles leave more x columns idle (nx = 96), and
    the z chunk that minimises the rounds of 256 resident workgroups times the chunk plus its 4
    halo planes."""
    plan = lbm.lbm_launch_plan(19, shape, I.physics(), 4)
    assert (plan["tile_x"], plan["tile_y"], plan["chunk"], plan["workgroups"]) == expect
    cols = -(-shape[2] // plan["tile_x"]) * -(-shape[1] // plan["tile_y"])
    assert plan["chunk"] == _rounds_cost(shape[0], cols)


def test_launch_plan_of_d2q9_and_fp64():
    d2 = lbm.lbm_launch_plan(9, (1, 1000, 1000), I.physics(), 4)
    assert (d2["tile_x"], d2["tile_y"], d2["chunk"], d2["workgroups"]) == (32, 8, 1, 32 * 125)
    d64 = lbm.lbm_launch_plan(19, (256, 256, 256), I.physics(), 8)
    assert (d64["tile_x"], d64["tile_y"]) == (32, 8)
    assert d64["workgroups"] == 8 * 32 * (-(-256 // d64["chunk"]))
    with pytest.raises(lbm.LbmError):
        lbm.lbm_launch_plan(9, (2, 8, 8), I.physics(), 4)     # D2Q9 needs nz = 1
