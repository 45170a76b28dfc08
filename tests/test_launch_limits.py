"""Host check of the launch-size arithmetic (csrc/launch_limits.h), compiled
with g++: every batch a launcher forms stays within the dispatch limit of
2^32 - 1 work-items per grid dimension, and the batches cover all lines of
sight."""
import os
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1810_06250_amd", "csrc")

PROG = r"""
#include <cstdio>
#include "launch_limits.h"
int main() {
    const int64_t lim = 0xffffffffLL;
    int bad = 0;
    // simple one-thread-per-item and one-wave-per-item launchers
    const int64_t cases[][2] = {{1, 256}, {4, 256}, {64, 256}, {256, 256}, {8, 512}};
    for (auto& c : cases) {
        const int64_t per = c[0], bs = c[1];
        const int64_t n = max_items(per, bs);
        if ((n / per) * bs > lim) ++bad;              // one batch fits
        if (((n / per) + 1) * bs <= lim) ++bad;       // and is the largest that does
    }
    // tiled transforms: nlos x tiles_n workgroups of 256 threads, LOS tiles of 64
    const int64_t tiles[] = {1, 2, 16, 32, 8192};
    const int64_t nlos_list[] = {1, 4194304, (int64_t)1 << 33};
    for (int64_t tn : tiles)
        for (int64_t nlos : nlos_list) {
            const int64_t per = max_los_tiled(tn, 64, 256);
            int64_t covered = 0;
            for (int64_t l0 = 0; l0 < nlos; l0 += per) {
                const int64_t n = nlos - l0 < per ? nlos - l0 : per;
                const int64_t blocks = ((n + 63) / 64) * tn;     // at 64 LOS per tile
                if (blocks * 256 > lim) ++bad;
                covered += n;
            }
            if (covered != nlos) ++bad;
        }
    std::printf("%d\n", bad);
    return bad != 0;
}
"""


def test_launch_batches_stay_within_the_grid_limit(tmp_path):
    src = tmp_path / "lim.cpp"
    src.write_text(PROG)
    exe = tmp_path / "lim"
    subprocess.run(["g++", "-std=c++17", "-O1", "-I", CSRC, "-o", str(exe), str(src)], check=True)
    r = subprocess.run([str(exe)], capture_output=True, text=True)
    assert r.returncode == 0, r.stdout + r.stderr
