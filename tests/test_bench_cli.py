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
