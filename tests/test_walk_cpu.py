"""CPU test of the tile walk of the persistent gather kernels: the walk function is taken
from the kernels' header as written, built with g++ (ASan + UBSan) and run over many frame
widths, heights and strip widths; every walk position must be a distinct tile of the frame,
since the kernels compute pixel coordinates from it."""
import os
import shutil
import subprocess
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "paper_2301_11376_amd", "csrc", "ssvb_internal.h")

DRIVER = r"""
#include <stdint.h>
#include <stdio.h>
#include <vector>
constexpr int kXcds = 8;
struct FrameArgs { int32_t tiles_x, tiles_y, strip; };
%s
int main() {
    long configs = 0, bad = 0;
    for (int tx = 1; tx <= 1100; ++tx)
        for (int ty : {1, 2, 5, 67, 135})
            for (int s0 : {1, 2, 3, 4, 8}) {
                FrameArgs A{tx, ty, s0 < tx ? s0 : tx};
                std::vector<char> seen((size_t)tx * ty, 0);
                for (uint32_t o = 0; o < (uint32_t)(tx * ty); ++o) {
                    int x = -1, y = -1;
                    walk_tile(A, o, x, y);
                    if (x < 0 || x >= tx || y < 0 || y >= ty || seen[(size_t)y * tx + x]++) {
                        if (++bad < 5) printf("bad: %%d x %%d tiles, strip %%d, position %%u -> (%%d, %%d)\n",
                                              tx, ty, A.strip, o, x, y);
                    }
                }
                ++configs;
            }
    printf("%%ld configurations, %%ld bad\n", configs, bad);
    return bad != 0;
}
"""


def walk_source():
    text = open(HEADER).read()
    i = text.index("SSVB_HD void walk_tile(")
    j = text.index("\n}\n", i) + 3
    return text[i:j].replace("SSVB_HD", "static inline")


@pytest.mark.skipif(shutil.which("g++") is None, reason="needs g++")
def test_walk_visits_every_tile_once():
    with tempfile.TemporaryDirectory() as d:
        src, exe = os.path.join(d, "walk.cpp"), os.path.join(d, "walk")
        with open(src, "w") as fh:
            fh.write(DRIVER % walk_source())
        subprocess.run(["g++", "-std=c++17", "-O2", "-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
                        src, "-o", exe], check=True, capture_output=True, text=True)
        res = subprocess.run([exe], capture_output=True, text=True, timeout=300)
        assert res.returncode == 0, res.stdout + res.stderr
        assert " 0 bad" in res.stdout
