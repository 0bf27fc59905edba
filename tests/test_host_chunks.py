"""Host logic of the automatic chunk of the wave kernels (no GPU needed).

The launcher cuts each column of tiles into chunks and runs them in rounds
of resident waves; the chosen chunk must (nearly) minimise
rounds * (chunk + warm-up) over every admissible chunk length, never go
below the minimum unless the axis is shorter, and pick the expected lengths
on the benchmark shapes.  The helper is compiled (its host side runs)
from the library's own header and checked against a brute force over every chunk
length.
"""
import math
import os
import shutil
import subprocess

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

SRC = r"""
#include <stdio.h>
#include <stdlib.h>
#include "lope_internal.h"
int main(int argc, char** argv) {
    for (int i = 1; i + 4 < argc; i += 5)
        printf("%d\n", lope::balanced_chunk(atoll(argv[i]), atoi(argv[i + 1]), atoll(argv[i + 2]),
                                            atoi(argv[i + 3]), atoi(argv[i + 4])));
    return 0;
}
"""


@pytest.fixture(scope="module")
def chooser(tmp_path_factory):
    if not os.path.exists(HIPCC):
        pytest.skip("hipcc not available")
    d = tmp_path_factory.mktemp("chunks")
    src = d / "chunks.hip"
    src.write_text(SRC)
    exe = d / "chunks"
    cmd = [HIPCC, "--offload-arch=gfx950", "-std=c++17", "-O1",
           "-I" + os.path.join(ROOT, "include"), "-I" + os.path.join(ROOT, "paper_1502_03504_amd", "csrc"),
           str(src), "-o", str(exe)]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-2000:]

    def run(cases):
        args = [str(v) for c in cases for v in c]
        out = subprocess.run([str(exe)] + args, capture_output=True, text=True, check=True).stdout.split()
        return [int(v) for v in out]
    yield run
    shutil.rmtree(d, ignore_errors=True)


def _cost(ncols, nz, slots, warm, chunk):
    return math.ceil(ncols * math.ceil(nz / chunk) / slots) * (chunk + warm)


def _best(ncols, nz, slots, warm, mn):
    lens = [c for c in range(1, nz + 1) if c >= mn or c == nz]
    return min(_cost(ncols, nz, slots, warm, c) for c in lens)


def test_benchmark_shapes(chooser):
    # 512^3 heat, wave bricks 56 x 8 outputs (640 columns), two waves per SIMD on 1024 SIMDs
    # 8192^2 box-9, 52-column strips (158), seven waves per SIMD
    got = chooser([(640, 512, 2048, 10, 8), (158, 8192, 7168, 14, 12)])
    assert got == [171, 183]


def test_near_optimal_and_admissible(chooser):
    rng = np.random.default_rng(7)
    cases = [(1, 1, 2048, 10, 8), (3, 19, 2048, 10, 8), (2, 1 << 20, 7168, 14, 12), (5000, 64, 2048, 10, 8),
             (1, 7, 2048, 10, 8), (640, 512, 4096, 10, 8)]
    for _ in range(40):
        cases.append((int(rng.integers(1, 3000)), int(rng.integers(1, 5000)), int(rng.choice([1024, 2048, 7168])),
                      int(rng.integers(2, 20)), int(rng.integers(1, 16))))
    got = chooser(cases)
    for (ncols, nz, slots, warm, mn), c in zip(cases, got):
        assert 1 <= c <= nz, (ncols, nz, c)
        assert c >= mn or c == nz, (ncols, nz, mn, c)
        best = _best(ncols, nz, slots, warm, mn)
        assert _cost(ncols, nz, slots, warm, c) <= 1.05 * best + 1, (ncols, nz, slots, warm, mn, c, best)
