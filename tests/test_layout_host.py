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


PROG_SB = r"""
#include <cstdio>
#include "crop_layout.hpp"
using namespace crop;
int main() {
    long bad = 0, n = 0;
    const uint32_t nbs[] = {1, 2, 3, 63, 64, 65, 1000, 1024, 3072, 4097, 8191, 8192};
    const uint32_t terms[] = {16, 1024, 16384, 24576, 65532};
    for (uint32_t NB : nbs)
        for (uint32_t T : terms)
            for (uint32_t kb = 4; kb <= 8; kb += 4)
                for (uint32_t rows = 1; rows < 3000; rows += (rows < 40 ? 1 : 211))
                    for (uint32_t items = 0; items < 9000; items += (items < 40 ? 1 : 377)) {
                        const SbLayout t = sb_layout(NB, rows, items, T, kb);
                        const size_t sm = 4 * (size_t)t.end;
                        ++n;
                        bool ok = sb_layout_ok(NB, rows, items, T, kb, sm);
                        ok = ok && t.ro >= t.hist + NB + 2;               // hist: NB + 2 words
                        ok = ok && t.tp >= t.ro + rows + 1;               // ro, tp: rows + 1
                        ok = ok && t.xh >= t.tp + rows + 1 && (4 * t.xh) % 8 == 0;
                        ok = ok && t.keys >= t.xh + 2 * items && (4 * t.keys) % 16 == 0;
                        ok = ok && (size_t)t.end >= t.keys + (size_t)T * kb / 4;
                        ok = ok && !sb_layout_ok(NB, rows, items, T, kb, sm - 4);  // tight bound
                        if (!ok) { if (bad < 5) printf("bad NB=%u T=%u kb=%u rows=%u items=%u\n", NB, T, kb, rows, items); ++bad; }
                    }
    // refused: too many bins or terms, a key width other than 4 or 8
    if (sb_layout_ok(8193, 10, 10, 1024, 4, 1u << 30)) ++bad;
    if (sb_layout_ok(64, 10, 10, 65536, 4, 1u << 30)) ++bad;
    if (sb_layout_ok(64, 10, 10, 1024, 2, 1u << 30)) ++bad;
    if (sb_layout_ok(64, 10, 10, 1022, 4, 1u << 30)) ++bad;  // not whole 16-byte groups
    printf("%ld %ld\n", n, bad);
    return bad ? 1 : 0;
}
"""


def test_region_route_layout_alignment_and_bounds(tmp_path):
    """The LDS image of a region-route sub-batch (bin counters, row offsets
    and term prefixes, staged items, sorted keys): arrays in order without
    overlap, the staged items 8-byte aligned and the sorted keys 16-byte
    aligned (they leave LDS in 16-byte loads), the image inside the dynamic
    allocation, and the 16-bit limits refused."""
    src = tmp_path / "sb_layout.cpp"
    exe = tmp_path / "sb_layout"
    src.write_text(PROG_SB)
    subprocess.run(["g++", "-std=c++17", "-O1", "-I", CSRC, str(src), "-o", str(exe)],
                   check=True)
    out = subprocess.run([str(exe)], capture_output=True, text=True)
    assert out.returncode == 0, out.stdout
    n, bad = map(int, out.stdout.split()[-2:])
    assert n > 10000 and bad == 0


PROG_WIN = r"""
#include <cstdio>
#include "crop_layout.hpp"
using namespace crop;
int main() {
    long bad = 0, n = 0;
    for (uint32_t lead = 0; lead < 8200; lead += (lead < 40 ? 1 : 389))
        for (uint32_t rows = 1; rows <= 512; rows += (rows < 20 ? 1 : 61))
            for (uint32_t kb = 2; kb <= 5; ++kb)
                for (uint32_t m = 0; m < 12000; m += (m < 40 ? 1 : 523)) {
                    const WinLayout t = win_layout(lead, rows, kb, m);
                    const size_t sm = 4 * t.end;
                    ++n;
                    bool ok = win_layout_ok(lead, rows, kb, m, sm);
                    ok = ok && t.hist >= lead;                                  // after the bin words
                    ok = ok && t.yh >= t.hist + ((size_t)rows << kb) + 1;       // bucket words
                    ok = ok && (4 * t.yh) % 8 == 0;                             // uint2 entries
                    ok = ok && 4 * t.row >= 4 * t.yh + 8 * (size_t)m;
                    ok = ok && 4 * t.rin >= 4 * t.row + 2 * (size_t)m;          // u16 rows, sorted
                    ok = ok && 4 * t.end >= 4 * t.rin + 2 * (size_t)m;          // u16 rows, input order
                    ok = ok && !win_layout_ok(lead, rows, kb, m, sm - 4);       // tight bound
                    if (!ok) { if (bad < 5) printf("bad lead=%u rows=%u kb=%u m=%u\n", lead, rows, kb, m); ++bad; }
                }
    if (win_layout_ok(0, 65536, 2, 10, 1u << 30)) ++bad;   // rows beyond 16 bits
    if (win_layout_ok(0, 10, 2, 65536, 1u << 30)) ++bad;   // entries beyond 16 bits
    printf("%ld %ld\n", n, bad);
    return bad ? 1 : 0;
}
"""


def test_window_layout_alignment_and_bounds(tmp_path):
    """The LDS image of a chunk staged for windowed enumeration (bin words,
    (row, bucket) words, (item, h_b) entries, sorted and input-order rows):
    arrays in order without overlap, entries 8-byte aligned, the image inside
    the dynamic allocation, and the 16-bit limits refused."""
    src = tmp_path / "win_layout.cpp"
    exe = tmp_path / "win_layout"
    src.write_text(PROG_WIN)
    subprocess.run(["g++", "-std=c++17", "-O1", "-I", CSRC, str(src), "-o", str(exe)],
                   check=True)
    out = subprocess.run([str(exe)], capture_output=True, text=True)
    assert out.returncode == 0, out.stdout
    n, bad = map(int, out.stdout.split()[-2:])
    assert n > 10000 and bad == 0
