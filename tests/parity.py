"""Shared helpers of the GPU parity tests: run the HIP library and the FP64 oracle on the same
seeded inputs and compare fields element by element."""
import numpy as np

import oracle
from paper_1705_10045_amd import lbm

FIELDS = ("rho", "u_star", "E", "T")
# Velocities are compared relative to max(|u*|_inf, U_FLOOR): a fluid at rest has no scale of
# its own, and the spurious currents of the interfaces are ~1e-3.
U_FLOOR = 0.01


def rel_errors(gpu, ref):
    out = {}
    for k in FIELDS:
        a, b = gpu[k], ref[k]
        scale = np.abs(b).max()
        if k == "u_star":
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
    print(msg, flush=True)
    return msg
