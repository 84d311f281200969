"""The oracle built with the compiler's address and undefined-behaviour
sanitizers (gcc, CPU only) runs its entry points on small seeded networks
without a report, with the same results on one and four threads."""
import os
import shutil
import struct
import subprocess

import numpy as np
import pytest

from paper_2306_07212_amd import workloads as wl

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def write_nets(path, nets):
    with open(path, "wb") as f:
        f.write(struct.pack("<i", len(nets)))
        for n in nets:
            L = len(n.widths) - 1
            f.write(struct.pack("<i", L))
            f.write(struct.pack(f"<{L + 1}i", *n.widths))
            for W, b in zip(n.W, n.b):
                f.write(np.ascontiguousarray(W, "<f8").tobytes())
                f.write(np.ascontiguousarray(b, "<f8").tobytes())


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc not available")
def test_oracle_under_address_and_undefined_behaviour_sanitizers(tmp_path):
    exe = str(tmp_path / "oracle_sanitized")
    cmd = ["gcc", "-O1", "-g", "-std=c11", "-ffp-contract=off", "-fopenmp", "-fno-omit-frame-pointer",
           "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined",
           os.path.join(ROOT, "oracle", "pcx_oracle.c"), os.path.join(ROOT, "oracle", "sanitize_main.c"),
           "-o", exe, "-lm"]
    subprocess.check_call(cmd)
    nets = [wl.plain_small(), wl.he_mlp([3, 8, 8, 1], 5), wl.he_mlp([1, 6, 5, 1], 41),
            wl.he_mlp([2, 12, 12, 12, 1], 42), wl.he_mlp([4, 5, 5, 1], 43)]
    write_nets(tmp_path / "nets.bin", nets)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1")
    p = subprocess.run([exe, str(tmp_path / "nets.bin")], capture_output=True, text=True, env=env, timeout=600)
    print(p.stdout[-2000:])
    assert p.returncode == 0, p.stderr[-4000:]
    assert "runtime error" not in p.stderr and "AddressSanitizer" not in p.stderr, p.stderr[-4000:]
    assert p.stdout.count("case") == 5 * len(nets)
