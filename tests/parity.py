"""Shared helpers of the GPU parity tests: run the HIP library and the FP64 oracle on the same
seeded inputs and compare fields element by element."""
import numpy as np

import oracle
from paper_1705_10045_amd import lbm

FIELDS = ("rho", "u_star", "E", "T")
# Velocities are compared relative to max(|u*|_inf, U_FLOOR): a fluid at rest has no scale of
# its own, and the spurious currents of the interfaces are ~1e-3.
U_FLOOR = 0.01


class Errors(dict):
    """Relative max-norm error per field (the tolerance applies to these values).
    `u_star_unfloored` is the u* error relative to max|u*| itself, without the floor: reported
    beside the floored value, because for a fluid nearly at rest it is several times larger."""
    u_star_unfloored = float("nan")


def rel_errors(gpu, ref):
    out = Errors()
    for k in FIELDS:
        a, b = gpu[k], ref[k]
        scale = np.abs(b).max()
        if k == "u_star":
            out.u_star_unfloored = float(np.abs(a - b).max() / scale) if scale > 0 else 0.0
            scale = max(scale, U_FLOOR)
        out[k] = float(np.abs(a - b).max() / scale)
    return out


def run_gpu(case, steps, storage_bytes):
    with lbm.Sim(case["Q"], case["params"], case["rho0"], case["u0"], case["T0"],
                 storage_bytes=storage_bytes) as s:
        if steps:
            s.step(steps)
        return s.moments(), s.reduce()


def run_oracle(case, steps):
    s = oracle.Sim(case["Q"], case["params"], case["rho0"], case["u0"], case["T0"])
    if steps:
        s.step(steps)
    m = s.moments()
    tot = s.totals()
    s.close()
    return m, tot


def compare(case, steps, storage_bytes):
    """(relative errors per field, gpu moments, oracle moments, gpu totals, oracle totals)."""
    g, gt = run_gpu(case, steps, storage_bytes)
    o, ot = run_oracle(case, steps)
    return rel_errors(g, o), g, o, gt, ot


def describe(name, errs):
    msg = "%s: " % name + " ".join("%s %.2e" % (k, v) for k, v in errs.items())
    raw = getattr(errs, "u_star_unfloored", None)
    if raw is not None and raw == raw:
        msg += " (u_star unfloored %.2e)" % raw
    print(msg, flush=True)
    return msg
