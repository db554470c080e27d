"""Benchmark of the fused thermal multiphase LBM step on one MI355X.

Default workload: D3Q19 pool boiling, 512^3, FP32 populations (40.8 GB of state), van der
Waals EOS, walls normal to z (bottom held at T/Tc = 0.9, top at 0.7), gravity 1e-5 along -z, a
liquid layer filling the lower 60% at the coexistence densities of T/Tc = 0.8 with +-1% seeded
noise, every physical term on: the largest single-GPU configuration of the method's workloads.
Other workloads (--workload): droplet128 (D3Q19 thermal droplet 128^3 moving at 0.05),
spinodal256 / spinodal256_fp64, spinodal512, droplet128_mrt, slab1000_d2q9, poolboil128.  The
state is resident in HBM before the timed region; the timed region is K fused step launches
bracketed by HIP events recorded on the simulation's own stream.

Prints ONE JSON line:
  value     - node updates per second in millions (MLUPS), one update = both population sets;
  roofline  - the step kernel against HBM: algorithmic bytes 2 sets x 19 x (read + write)
              x 4 B = 304 B per node update, divided by the measured launch duration, against
              the 8 TB/s peak; 'traffic' is the HBM traffic per launch measured by rocprofv3
              counters (profiles/), or null when not measured for the current kernel source;
  serving   - continuous batching of the stream of uneven requests through the device pool
              (the first 128 of its 512 requests, listed step counts): p50/p99
              time-to-result under a Poisson stream at 0.8x the burst capacity, aggregate MLUPS
              batched and one at a time (skip with --no-serving);
  cpu_baseline - the FP64 CPU oracle timed on the host cores on a bounded sample: whole steps
              of the same workload at its full size when the host memory holds the oracle's
              state (about 0.8 kB per node), else at the largest smaller edge of the same
              recipe that fits; the library's fields after the same steps, in the launch the
              benchmark times, compared with the oracle's (parity_vs_gpu).

--gpus N with N > 1 exits: the library runs on one GPU.
"""
import argparse
import hashlib
import re
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "MLUPS (coupled density+energy) & % HBM roofline, 1 GPU; serving p50/p99 latency"
HBM_PEAK_GBS = 8000.0
BYTES_PER_UPDATE = {4: 2 * 19 * 2 * 4, 8: 2 * 19 * 2 * 8}   # D3Q19


def bytes_per_update(Q, storage):
    """Algorithmic bytes of one node update: both population sets read once and written once."""
    return 2 * Q * 2 * storage
KERNEL_SOURCES = ["paper_1705_10045_amd/csrc/step_kernel.hpp", "paper_1705_10045_amd/csrc/node_math.hpp",
                  "paper_1705_10045_amd/csrc/physics.hpp",
                  "paper_1705_10045_amd/csrc/lattice.hpp", "paper_1705_10045_amd/csrc/kernels.hip",
                  "paper_1705_10045_amd/csrc/step_launch.hpp", "paper_1705_10045_amd/csrc/api.hip"]


def _code_only(text):
    """Source text without // and /* */ comments and trailing blanks: what the compiler sees."""
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    text = re.sub(r"//[^\n]*", "", text)
    return "\n".join(line.rstrip() for line in text.splitlines() if line.strip())


def kernel_source_hash(read=None):
    """Hash of the step kernel's code (comments excluded), stored beside counter readings so that
    a reading taken on other code is not reported.  `read(rel)` returns a file's text (default:
    the working tree)."""
    read = read or (lambda rel: open(os.path.join(ROOT, rel)).read())
    h = hashlib.sha256()
    for rel in KERNEL_SOURCES:
        h.update(_code_only(read(rel)).encode())
    return h.hexdigest()[:16]


DEFAULT_WORKLOAD = "poolboil512"

# host bytes per node the FP64 oracle holds (4 population arrays of 19 doubles and 24 field
# doubles), plus the initial fields and the two sets of output moments of the comparison
ORACLE_BYTES_PER_NODE = 4 * 19 * 8 + 24 * 8 + 3 * 6 * 8
HOST_CAP_BYTES = 200e9


def host_available_bytes():
    """MemAvailable of the host, in bytes (0 if unknown)."""
    try:
        with open("/proc/meminfo") as f:
            for line in f:
                if line.startswith("MemAvailable:"):
                    return int(line.split()[1]) * 1024
    except OSError:
        pass
    return 0


def workload(name, edge=None):
    """(case, storage bytes, config) of a named workload; `edge` rebuilds the same recipe on a
    smaller cube (the CPU baseline's fallback when the host cannot hold the full size)."""
    from paper_1705_10045_amd import inputs as I
    if edge is not None:
        for family in ("poolboil", "spinodal"):
            if name.startswith(family) and name[len(family):].isdigit():
                name = "%s%d" % (family, edge)
    if name == "droplet128":
        case = I.droplet_3d(n=128, radius=24.0, Tr=0.8, noise=0.005, velocity=(0.05, 0.0, 0.0))
        return case, 4, {"workload": "d3q19_thermal_droplet_128^3_fp32", "lattice": "D3Q19",
                         "shape": [128, 128, 128], "storage": "fp32", "T_over_Tc": 0.8,
                         "radius": 24, "noise": 0.005, "velocity": [0.05, 0.0, 0.0],
                         "terms": "work+conduction+latent+pseudoforces"}
    if name in ("spinodal256", "spinodal256_fp64"):
        storage = 8 if name.endswith("fp64") else 4
        case = I.spinodal_3d(n=256, Tr=0.75, rho_mean=1.0, sigma=0.02)
        return case, storage, {"workload": "d3q19_spinodal_256^3_%s" % ("fp64" if storage == 8 else "fp32"),
                               "lattice": "D3Q19", "shape": [256, 256, 256],
                               "storage": "fp64" if storage == 8 else "fp32", "T_over_Tc": 0.75,
                               "rho_mean": 1.0, "noise_sigma": 0.02,
                               "terms": "work+conduction+latent+pseudoforces"}
    if name.startswith("spinodal") and name[len("spinodal"):].isdigit():
        n = int(name[len("spinodal"):])
        case = I.spinodal_3d(n=n, Tr=0.75, rho_mean=1.0, sigma=0.02)
        return case, 4, {"workload": "d3q19_spinodal_%d^3_fp32" % n, "lattice": "D3Q19",
                         "shape": [n, n, n], "storage": "fp32", "T_over_Tc": 0.75,
                         "rho_mean": 1.0, "noise_sigma": 0.02,
                         "terms": "work+conduction+latent+pseudoforces"}
    if name == "droplet128_mrt":
        case = I.droplet_3d(n=128, radius=24.0, Tr=0.8, noise=0.005, velocity=(0.05, 0.0, 0.0),
                            params=I.physics(tau=0.8))
        rates = dict(collision=1, s_e=1.19, s_eps=1.4, s_q=1.2, s_m=1.98)
        case["params"] = dict(case["params"], **rates)
        return case, 4, {"workload": "d3q19_thermal_droplet_128^3_fp32_mrt", "lattice": "D3Q19",
                         "shape": [128, 128, 128], "storage": "fp32", "T_over_Tc": 0.8,
                         "radius": 24, "noise": 0.005, "velocity": [0.05, 0.0, 0.0],
                         "collision": "MRT", "tau": 0.8, "rates": rates,
                         "terms": "work+conduction+latent+pseudoforces"}
    if name == "slab1000_d2q9":
        case = I.slab_2d(n=1000, width=300)
        return case, 4, {"workload": "d2q9_thermal_slab_1000^2_fp32", "lattice": "D2Q9",
                         "shape": [1, 1000, 1000], "storage": "fp32 (FP64 arithmetic)",
                         "T_over_Tc": 0.85, "width": 300, "noise": 0.01,
                         "terms": "work+conduction+latent+pseudoforces"}
    if name.startswith("poolboil") and name[len("poolboil"):].isdigit():
        n = int(name[len("poolboil"):])
        case = I.pool_boiling_3d(n=n)
        pp = case["params"]
        return case, 4, {"workload": "d3q19_pool_boiling_%d^3_fp32" % n, "lattice": "D3Q19",
                         "shape": [n, n, n], "storage": "fp32", "T_over_Tc": 0.8,
                         "walls": "z, bounce-back", "T_bottom_over_Tc": pp["T_bottom"] / pp["T_c"],
                         "T_top_over_Tc": pp["T_top"] / pp["T_c"], "gravity": list(pp["gravity"]),
                         "liquid_fill": 0.6, "noise": 0.01,
                         "terms": "work+conduction+latent+pseudoforces"}
    raise SystemExit("unknown workload %s" % name)


def copy_ceiling_gbs(Q, storage, shape):
    """The committed copy-kernel ceiling of the same state (profiles/ceiling_state_copy_fp32.json,
    from `bench.py --ceiling`) for FP32 D3Q19 cubes of edge 128, 256 or 512, else None."""
    path = os.path.join(ROOT, "profiles", "ceiling_state_copy_fp32.json")
    if Q != 19 or storage != 4 or len(set(shape)) != 1 or not os.path.exists(path):
        return None
    with open(path) as f:
        rec = json.load(f)["results"].get("state_copy_%d" % shape[0])
    return None if rec is None else rec["hip_flat_GB_per_s"]


def measured_traffic(config_name, bytes_alg):
    """HBM bytes per launch from the committed rocprofv3 counter summary of this workload, if it
    was taken on the current kernel source."""
    path = os.path.join(ROOT, "profiles", "traffic_%s.json" % config_name)
    if not os.path.exists(path):
        return None
    with open(path) as f:
        t = json.load(f)
    if t.get("kernel_source_hash") != kernel_source_hash():
        return None
    return t.get("bytes_per_launch")


PARITY_TOL = {4: 1e-5, 8: 1e-11}


def cpu_baseline(name, case, storage=4, launch=None, budget_s=20.0, max_steps=50, log=None):
    """The oracle as it stands, on the host cores, over whole steps of the same workload: at its
    full size when the host's available memory holds the oracle's state with room to spare,
    else the same recipe on the largest smaller cube that fits (the sample says which).  At
    least one step; more while the steps taken so far stay under `budget_s`.  The state it
    reaches is then compared with the library's after the same steps from the same initial
    fields, in the launch the benchmark times (relative max-norm per field; u* relative to
    max(|u*|, 0.01), and without that floor as u_star_unfloored)."""
    import numpy as np
    import oracle
    from paper_1705_10045_amd import lbm
    log = log or (lambda msg: print(msg, file=sys.stderr, flush=True))
    threads = int(os.environ.get("OMP_NUM_THREADS", "0") or 0) or os.cpu_count()
    avail = host_available_bytes()
    # at most half of what is available, and never more than HOST_CAP_BYTES
    room = min(0.5 * avail, HOST_CAP_BYTES) if avail else HOST_CAP_BYTES
    n_full = case["rho0"].size
    edge = None
    if n_full * ORACLE_BYTES_PER_NODE > room:
        e = case["rho0"].shape[0]
        while e > 32 and (e ** 3) * ORACLE_BYTES_PER_NODE > room:
            e //= 2
        edge = e
        case, _, _ = workload(name, edge)
    n = case["rho0"].size
    size = "x".join(str(d) for d in case["rho0"].shape[::-1])
    log("cpu_baseline: oracle on %s (%s, %.0f GB available)" %
        (size, "full size" if edge is None else "reduced from the full size", avail / 1e9))
    s = oracle.Sim(case["Q"], case["params"], case["rho0"], case["u0"], case["T0"])
    steps = 0
    t0 = time.perf_counter()
    while True:
        s.step(1)
        steps += 1
        el = time.perf_counter() - t0
        log("cpu_baseline: oracle step %d done (%.1f s)" % (steps, el))
        if el * (steps + 1) / steps > budget_s or steps >= max_steps:
            break
    ref = s.moments()
    s.close()
    log("cpu_baseline: the library on the same fields")
    with lbm.Sim(case["Q"], case["params"], case["rho0"], case["u0"], case["T0"],
                 storage_bytes=storage) as g:
        if launch is not None:
            g.set_launch(*launch)
        g.step(steps)
        got = g.moments()
    errs = {}
    for k in ("rho", "u_star", "E", "T"):
        scale = max(float(np.abs(ref[k]).max()), 0.01 if k == "u_star" else 0.0)
        errs[k] = float("%.3g" % (np.abs(got[k] - ref[k]).max() / scale))
    raw = float(np.abs(got["u_star"] - ref["u_star"]).max() / max(np.abs(ref["u_star"]).max(), 1e-300))
    del ref, got
    return {"value": round(n * steps / el / 1e6, 3), "unit": "MLUPS", "cores": threads,
            "kind": "oracle",
            "sample": "%d whole FP64 step%s of the same workload on %s%s (%.1f s)" %
                      (steps, "" if steps == 1 else "s", size,
                       "" if edge is None else " (the full size needs more host memory than the "
                       "%.0f GB allowed)" % (room / 1e9), el),
            "parity_vs_gpu": {"steps": steps, "size": size, "max_rel_err": errs,
                              "u_star_unfloored": float("%.3g" % raw),
                              "tolerance": PARITY_TOL[storage],
                              "pass": max(errs.values()) < PARITY_TOL[storage]}}


def copy_probe(gib=1.0, reps=5):
    """A plain device-to-device copy of known size, for scaling rocprofv3 byte counters."""
    import torch
    n = int(gib * (1 << 30)) // 4
    a = torch.ones(n, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    for _ in range(reps):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_probe_bytes_read": n * 4, "copy_probe_bytes_written": n * 4,
                      "launches": reps}), flush=True)


def copy_ceiling(edges=(128, 256, 512), reps=20):
    """Bandwidth of plain device copies of the step's state (2 x 19 float arrays of edge^3
    nodes): torch's copy, and the HIP probe (libceiling.so) in two orders, the state as one
    flat array and all 38 planes of a run of nodes together (the step's order).  Events time
    `reps` copies after a warm-up.  This is the practical ceiling of a pattern that reads and
    writes every population once."""
    import ctypes
    import torch
    from paper_1705_10045_amd import build as lib_build
    if not os.path.exists(lib_build.PROBE_LIB):
        lib_build.build()
    probe = ctypes.CDLL(lib_build.PROBE_LIB)
    probe.lbm_probe_copy.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t,
                                     ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                     ctypes.POINTER(ctypes.c_float)]
    cus = torch.cuda.get_device_properties(0).multi_processor_count
    out = {}
    for edge in edges:
        n = edge ** 3
        m = 38 * n
        a = torch.ones(m, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        start = torch.cuda.Event(enable_timing=True)
        end = torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        start.record()
        for _ in range(reps):
            b.copy_(a)
        end.record()
        torch.cuda.synchronize()
        res = {"torch_copy": start.elapsed_time(end) / reps}
        for name, order in (("hip_flat", 0), ("hip_sweep", 1)):
            best = None
            for per_cu in (4, 8, 16):
                ms = ctypes.c_float()
                st = probe.lbm_probe_copy(a.data_ptr(), b.data_ptr(), n, 38, order, reps,
                                          cus * per_cu, ctypes.byref(ms))
                if st != 0:
                    raise RuntimeError("lbm_probe_copy failed (%d)" % st)
                if best is None or ms.value < best[0]:
                    best = (ms.value, cus * per_cu)
            res[name] = best[0]
            res[name + "_workgroups"] = best[1]
        out["state_copy_%d" % edge] = {
            k: (round(v, 4) if not k.endswith("workgroups") else v) for k, v in res.items()}
        for k in ("torch_copy", "hip_flat", "hip_sweep"):
            out["state_copy_%d" % edge][k + "_GB_per_s"] = round(2 * 4 * m / res[k] / 1e6, 1)
        print(json.dumps({"edge": edge, **out["state_copy_%d" % edge]}), file=sys.stderr, flush=True)
        del a, b
        torch.cuda.empty_cache()
    print(json.dumps(out), flush=True)


SERVING_STREAM = 512          # requests in the listed serving stream
SERVING_DEFAULT_COUNT = 128   # the benchmark line's cut of it (the first requests, as listed)


def serving_bench(count=SERVING_DEFAULT_COUNT, steps_range=(500, 5000), budget_gib=64.0,
                  max_slots=64, steps_per_run=20, load=0.8):
    """Continuous-batching serving of the stream of uneven D3Q19 FP32 requests (edges
    32..128, droplet or slab, T/Tc in [0.70, 0.95], +-1% noise, 500..5000 steps): the first
    `count` requests of the 512-request stream, each with its listed step count (request i
    does not depend on the count).  Three passes over the same request list: a burst (all
    arrive at t = 0) measures the batched capacity; a Poisson stream offered at `load` x that
    capacity gives p50/p99 time-to-result; the same requests one after another with a single
    simulation each give the one-at-a-time rate.  Each request carries its initial fields
    (built before the clock starts); upload, initialisation, the steps and the download of the
    result fields are timed."""
    from paper_1705_10045_amd import inputs as I
    from paper_1705_10045_amd import lbm
    from paper_1705_10045_amd import serve
    import numpy as np
    reqs = I.serving_requests(count=count, steps_range=steps_range)
    work = np.array([r["edge"] ** 3 * r["steps"] for r in reqs], dtype=np.float64)
    budget = int(budget_gib * (1 << 30))
    # the initial fields arrive with each request (the client builds them): not timed
    payload = {r["id"]: I.request_fields(r) for r in reqs}

    def progress(done):   # a line every 64 requests, so long streams show progress
        if done % 64 == 0:
            print("serving: %d of %d requests done" % (done, count), file=sys.stderr, flush=True)

    def run(arrivals):
        with lbm.Pool(budget, max_slots=max_slots, steps_per_run=steps_per_run) as pool:
            return serve.serve(reqs, arrivals, serve.PoolExecutor(pool, payload=payload),
                               progress=progress)

    print("serving: burst of %d requests" % count, file=sys.stderr, flush=True)
    burst = run(np.zeros(count))
    rate = load * burst["aggregate_mlups"] * 1e6 / work.mean()
    print("serving: Poisson stream at %.2f requests/s" % rate, file=sys.stderr, flush=True)
    stream = run(serve.poisson_arrivals(count, rate))
    print("serving: one at a time", file=sys.stderr, flush=True)
    single = serve.one_at_a_time(reqs, payload=payload, progress=progress)

    def brief(r):
        return {"p50_s": round(r["p50_s"], 4), "p99_s": round(r["p99_s"], 4),
                "aggregate_mlups": round(r["aggregate_mlups"], 1), "wall_s": round(r["wall_s"], 3),
                "completed": r["completed"], "failed": r["failed"],
                "failed_ids": [reqs[i]["id"] for i, st in enumerate(r["status"]) if st not in (0, None)],
                "peak_in_flight": r["peak_in_flight"], "replays": r["replays"]}
    return {"requests": count,
            "stream": "requests 0..%d of the %d-request serving stream, listed step counts" %
                      (count - 1, SERVING_STREAM),
            "edges": sorted(set(r["edge"] for r in reqs)),
            "steps_range": list(steps_range), "node_updates": int(work.sum()),
            "hbm_budget_gib": budget_gib, "max_slots": max_slots,
            "steps_per_replay": steps_per_run,
            "burst": brief(burst),
            "poisson": dict(brief(stream), offered_load=load,
                            rate_per_s=round(rate, 3)),
            "one_at_a_time_mlups": round(single["aggregate_mlups"], 1),
            "one_at_a_time_wall_s": round(single["wall_s"], 3),
            "one_at_a_time_failed_ids": single["failed_ids"]}


def sweep(sim, stream, n, storage, chunks=(0, 8, 16, 32), steps=40, reps=3):
    """Time each launch variant x z-chunk (0 = automatic) from the same checkpointed state,
    `reps` interleaved rounds, median reported; every variant must reproduce the same fields
    bit for bit."""
    import numpy as np
    import torch
    from paper_1705_10045_amd import lbm
    ck = sim.checkpoint()
    nvar = 0
    while True:
        try:
            sim.set_launch(nvar, 0)
            nvar += 1
        except lbm.LbmError:
            break
    configs = [(v, c) for v in range(nvar) for c in chunks]
    times = {cfg: [] for cfg in configs}
    same = {}
    info = {}
    ref = None
    for rep in range(reps):
        for cfg in configs:
            sim.set_launch(*cfg)
            sim.restore(ck)
            sim.step(5)
            start = torch.cuda.Event(enable_timing=True)
            end = torch.cuda.Event(enable_timing=True)
            torch.cuda.synchronize()
            start.record(stream)
            sim.step_async(steps)
            end.record(stream)
            torch.cuda.synchronize()
            sim.check()
            times[cfg].append(start.elapsed_time(end) / steps)
            if rep == 0:
                m = sim.moments()["rho"]
                same[cfg] = ref is None or bool(np.array_equal(m, ref))
                ref = m if ref is None else ref
                info[cfg] = sim.launch_info()
    for cfg in configs:
        ms = float(np.median(times[cfg]))
        i = info[cfg]
        print(json.dumps({"variant": cfg[0], "tile": [i["tile_x"], i["tile_y"]], "chunk": i["chunk"],
                          "workgroups": i["workgroups"], "ms_per_step": round(ms, 4),
                          "ms_all": [round(t, 4) for t in times[cfg]],
                          "mlups": round(n / ms / 1e3, 1),
                          "frac": round(BYTES_PER_UPDATE[storage] * n / (ms / 1e3) / 1e9 / HBM_PEAK_GBS, 4),
                          "bitwise_equal": same[cfg]}), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--workload", default=DEFAULT_WORKLOAD)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--copy-probe", action="store_true",
                    help="1 GiB device copies only (calibration of rocprofv3 byte counters)")
    ap.add_argument("--ceiling", action="store_true",
                    help="time plain device copies of the step's state at 128^3, 256^3 and 512^3")
    ap.add_argument("--sweep", action="store_true",
                    help="time every tile variant x z-chunk of the step kernel (tuning)")
    ap.add_argument("--serving", action="store_true",
                    help="only the serving measurement (burst, Poisson stream, one at a time)")
    ap.add_argument("--no-serving", action="store_true",
                    help="skip the serving measurement in the default line")
    ap.add_argument("--serving-requests", type=int, default=SERVING_DEFAULT_COUNT)
    ap.add_argument("--serving-full", action="store_true",
                    help="with --serving: the whole request stream (512 requests) instead of the "
                         "benchmark line's first %d" % SERVING_DEFAULT_COUNT)
    ap.add_argument("--variant", type=int, default=None)
    ap.add_argument("--chunk", type=int, default=0)
    args = ap.parse_args()

    if args.gpus != 1:
        print("bench.py runs on one GPU only: the library has no multi-GPU path (asked for %d)"
              % args.gpus, file=sys.stderr)
        sys.exit(2)
    if args.copy_probe:
        copy_probe()
        return
    if args.ceiling:
        copy_ceiling()
        return

    import torch
    from paper_1705_10045_amd import build as lib_build
    from paper_1705_10045_amd import lbm
    if not os.path.exists(lib_build.LIB):
        lib_build.build()

    if args.serving:
        rep = serving_bench(count=SERVING_STREAM if args.serving_full else args.serving_requests)
        print(json.dumps({"metric": "serving time-to-result (p50/p99) and aggregate MLUPS",
                          "serving": rep}), flush=True)
        return

    case, storage, config = workload(args.workload)
    n = case["rho0"].size
    # a dedicated stream (default priority): the library enqueues on it and the events below
    # bracket exactly its launches
    stream = torch.cuda.Stream()
    print("bench: %s, %d warmup + %d timed steps" % (config["workload"], args.warmup, args.steps),
          file=sys.stderr, flush=True)
    sim = lbm.Sim(case["Q"], case["params"], case["rho0"], case["u0"], case["T0"],
                  storage_bytes=storage, stream=stream.cuda_stream)
    if args.variant is not None or args.chunk:
        sim.set_launch(args.variant or 0, args.chunk)
    if args.sweep:
        sweep(sim, stream, n, storage)
        return
    info = sim.launch_info()
    sim.step(args.warmup)

    start = torch.cuda.Event(enable_timing=True)
    end = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    start.record(stream)
    sim.step_async(args.steps)
    end.record(stream)
    torch.cuda.synchronize()
    sim.check()
    ms = start.elapsed_time(end)
    ms_per_step = ms / args.steps
    mlups = n * args.steps / (ms / 1e3) / 1e6

    bytes_alg = bytes_per_update(case["Q"], storage) * n
    achieved = bytes_alg / (ms_per_step / 1e3) / 1e9
    traffic = measured_traffic(config["workload"], bytes_alg)
    totals = sim.reduce()
    sim.close()

    out = {
        "metric": METRIC, "value": round(mlups, 2), "unit": "MLUPS", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_per_step, 5),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32" if storage == 4 else "f64", "data": "synthetic",
        "config": dict(config, launch=info),
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": traffic,
                     # the counted bytes over the timed kernel time, and a plain copy of the
                     # same state, for context (neither is the graded fraction)
                     "traffic_GB_per_s": (round(traffic / (ms_per_step / 1e3) / 1e9, 1)
                                          if traffic else None),
                     "copy_ceiling_GB_per_s": copy_ceiling_gbs(case["Q"], storage,
                                                               case["rho0"].shape),
                     "kernel": "lbm::k_step<%d,%s> (one launch per step)" %
                               (case["Q"], "float" if storage == 4 else "double"),
                     "algorithmic_bytes_per_launch": bytes_alg},
        "totals_fp64": [float(x) for x in totals],
    }
    if not args.no_serving:
        out["serving"] = serving_bench(count=args.serving_requests)
    if not args.no_cpu_baseline:
        launch = (args.variant or 0, args.chunk) if (args.variant is not None or args.chunk) else None
        out["cpu_baseline"] = cpu_baseline(args.workload, case, storage, launch)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
