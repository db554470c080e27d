"""The benchmark on a host without a GPU: multi-GPU requests are refused with a message (this
build has one GPU path) before anything touches a device, and the kernel-code hash that ties
stored counter readings to the code they were taken on ignores comments but not code."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_bench_refuses_more_than_one_gpu():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def test_kernel_hash_ignores_comments_but_not_code():
    sys.path.insert(0, ROOT)
    import bench
    text = {rel: open(os.path.join(ROOT, rel)).read() for rel in bench.KERNEL_SOURCES}
    first = bench.KERNEL_SOURCES[0]
    h0 = bench.kernel_source_hash(lambda rel: text[rel])
    assert h0 == bench.kernel_source_hash()

    commented = dict(text)
    commented[first] = "// a note\n/* a block\n   comment */\n" + text[first].replace(
        "\n", "   // trailing remark\n", 3)
    assert bench.kernel_source_hash(lambda rel: commented[rel]) == h0

    changed = dict(text)
    changed[first] = text[first].replace("#pragma once", "#pragma once\nconstexpr int kProbe = 1;", 1)
    assert changed[first] != text[first]
    assert bench.kernel_source_hash(lambda rel: changed[rel]) != h0


def test_algorithmic_bytes_and_workload_table():
    """Bytes per node update are both population sets read once and written once (304 B for
    D3Q19 FP32, 608 B FP64, 144 B for D2Q9 FP32), and every named workload builds its seeded
    input with the lattice, storage and shape its config states."""
    sys.path.insert(0, ROOT)
    import bench
    assert bench.bytes_per_update(19, 4) == 304
    assert bench.bytes_per_update(19, 8) == 608
    assert bench.bytes_per_update(9, 4) == 144
    for name, Q, storage, shape in (("droplet128", 19, 4, (128, 128, 128)),
                                    ("droplet128_mrt", 19, 4, (128, 128, 128)),
                                    ("spinodal256", 19, 4, (256, 256, 256)),
                                    ("spinodal256_fp64", 19, 8, (256, 256, 256)),
                                    ("poolboil128", 19, 4, (128, 128, 128)),
                                    ("slab1000_d2q9", 9, 4, (1, 1000, 1000))):
        case, st, config = bench.workload(name)
        assert case["Q"] == Q and st == storage, name
        assert case["rho0"].shape == shape, name
        assert list(config["shape"]) == list(shape[::-1]) or list(config["shape"]) == list(shape)
        assert config["workload"]
    case, _, config = bench.workload("droplet128_mrt")
    assert case["params"]["collision"] == 1 and config["collision"] == "MRT"
