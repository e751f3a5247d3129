"""The work dealing of the free-surface class passes, on the host (no GPU).

A class-pass wave numbers its work items (item k of lane l, k major) from 16
ballots and hands item i to lane i mod 64 in round i / 64; the lane finds
the item's k from the prefix counts of the ballots and its source lane as
the n-th set bit of ballot k (`nth_set_bit` in csrc/freesurf.hpp).  The
function is compiled here from the kernel source with the host compiler and
checked against a plain enumeration, and the dealing itself (a model of
`for_items`) is checked to hand every item to exactly one lane.
"""
import os
import random
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "paper_0912_4230_amd", "csrc", "freesurf.hpp")


def _function_source():
    s = open(SRC).read()
    m = re.search(r"__host__ __device__ inline int nth_set_bit\(uint64_t v, uint32_t n\)\n\{.*?\n\}\n", s, re.S)
    assert m, "nth_set_bit not found"
    return m.group(0).replace("__host__ __device__ ", "")


def test_nth_set_bit_against_enumeration(tmp_path):
    prog = tmp_path / "t.cpp"
    prog.write_text("#include <cstdint>\n#include <cstdio>\n#include <random>\n" + _function_source() + r"""
int main() {
    std::mt19937_64 g(7);
    long bad = 0, n = 0;
    const uint64_t edge[] = {1ull, 1ull << 63, ~0ull, 0x8000000000000001ull, 0x5555555555555555ull};
    for (int it = 0; it < 100005; ++it) {
        uint64_t v = it < 5 ? edge[it] : g();
        if (it % 3 == 0) v &= g();
        if (it % 7 == 0) v >>= g() % 64;
        if (!v) continue;
        int c = 0;
        for (int p = 0; p < 64; ++p)
            if ((v >> p) & 1) { bad += nth_set_bit(v, c) != p; ++c; ++n; }
    }
    std::printf("%ld %ld\n", n, bad);
    return bad != 0;
}
""")
    exe = tmp_path / "t"
    subprocess.run(["g++", "-O2", "-std=c++17", "-o", str(exe), str(prog)], check=True)
    out = subprocess.run([str(exe)], capture_output=True, text=True)
    n, bad = map(int, out.stdout.split())
    assert out.returncode == 0 and bad == 0 and n > 1_000_000


def _nth(v, n):
    pos, w = 0, 32
    while w >= 1:
        c = bin((v >> pos) & ((1 << w) - 1)).count("1")
        if n >= c:
            n -= c
            pos += w
        w //= 2
    return pos


@pytest.mark.parametrize("density", [0.0, 0.01, 0.1, 0.5, 1.0])
def test_dealing_hands_every_item_to_one_lane(density):
    rng = random.Random(int(density * 1000) + 3)
    for _ in range(200):
        masks = [sum(1 << k for k in range(16) if rng.random() < density) for _ in range(64)]
        ballots = [sum(1 << l for l in range(64) if (masks[l] >> k) & 1) for k in range(16)]
        start = [0]
        for b in ballots:
            start.append(start[-1] + bin(b).count("1"))
        total, dealt = start[16], []
        for r in range(0, total, 64):
            for lane in range(64):
                i = r + lane
                if i >= total:
                    continue
                k, bits, n = 0, ballots[0], i
                for kk in range(1, 16):
                    if i >= start[kk]:
                        k, bits, n = kk, ballots[kk], i - start[kk]
                dealt.append((_nth(bits, n), k))
        want = sorted((l, k) for l in range(64) for k in range(16) if (masks[l] >> k) & 1)
        assert sorted(dealt) == want and len(set(dealt)) == len(dealt)
