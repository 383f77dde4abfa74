"""The LDS layout of a staged chunk of transactions, built on the host with
g++ from the library's own header (no GPU): every sub-array of the image is
aligned for the LDS operations the kernels issue on it (64-bit loads of xh,
32-bit atomics on the bucket words), the arrays do not overlap, and the
image ends inside the dynamic LDS the launch reserves.  Odd lead offsets and
odd entry counts are the cases a misaligned u16 array would break."""
import os
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1210_0461_amd", "csrc")

PROG = r"""
#include <cstdio>
#include "crop_layout.hpp"
using namespace crop;
int main() {
    long bad = 0, n = 0;
    for (uint32_t lead = 0; lead < 9000; lead += (lead < 80 ? 1 : 97)) {
        for (uint32_t m = 0; m < 20000; m += (m < 300 ? 1 : 131)) {
            const TxLayout t = tx_layout(lead, m);
            const size_t sm = 4 * tx_lds_words(lead, m);
            ++n;
            bool ok = tx_layout_ok(lead, m, sm);
            ok = ok && (4 * t.xh) % 8 == 0 && t.xh >= lead;      // 8-byte xh
            ok = ok && (4 * t.w) % 4 == 0 && (4 * t.perm) % 4 == 0;
            ok = ok && (4 * t.bucket) % 4 == 0;                   // word atomics
            ok = ok && 4 * t.w >= 4 * t.xh + 8 * (size_t)m;       // xh fits
            ok = ok && 4 * t.perm >= 4 * t.w + 2 * (size_t)m;     // w fits
            ok = ok && 4 * t.bucket >= 4 * t.perm + 2 * (size_t)m;
            ok = ok && 4 * t.end <= sm && t.end == t.bucket + 64;
            ok = ok && !tx_layout_ok(lead, m, sm - 4);            // tight bound
            if (!ok) { if (bad < 5) printf("bad lead=%u m=%u\n", lead, m); ++bad; }
        }
    }
    printf("%ld %ld\n", n, bad);
    return bad ? 1 : 0;
}
"""


def test_chunk_layout_alignment_and_bounds(tmp_path):
    src = tmp_path / "layout.cpp"
    exe = tmp_path / "layout"
    src.write_text(PROG)
    subprocess.run(["g++", "-std=c++17", "-O1", "-I", CSRC, str(src), "-o", str(exe)],
                   check=True)
    out = subprocess.run([str(exe)], capture_output=True, text=True)
    assert out.returncode == 0, out.stdout
    n, bad = map(int, out.stdout.split()[-2:])
    assert n > 10000 and bad == 0
