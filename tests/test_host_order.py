"""Host logic of the node ordering: the Hilbert-curve key used to order the
nodes of a batched context is a bijection of the 2^b x 2^b x 2^b cells onto
[0, 8^b) whose consecutive values are face-adjacent cells (a continuous,
space-filling curve).  The function is compiled from the library source
with the host compiler."""
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "paper_2510_12011_amd", "csrc", "mdx_order.hip")

PROG = r"""
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <vector>
#include <algorithm>
%s
int main() {
    for (int bits = 1; bits <= 5; ++bits) {
        const int n = 1 << bits;
        std::vector<std::pair<uint64_t, int>> k;
        for (int x = 0; x < n; ++x)
            for (int y = 0; y < n; ++y)
                for (int z = 0; z < n; ++z) k.push_back({hilbert_key(x, y, z, bits), (x * n + y) * n + z});
        std::sort(k.begin(), k.end());
        int bad = 0;
        for (size_t i = 0; i < k.size(); ++i) bad += k[i].first != i;
        for (size_t i = 1; i < k.size(); ++i) {
            const int a = k[i - 1].second, b = k[i].second;
            const int d = std::abs(a / (n * n) - b / (n * n)) + std::abs(a / n %% n - b / n %% n) +
                          std::abs(a %% n - b %% n);
            bad += d != 1;
        }
        printf("%%d %%d\n", bits, bad);
    }
}
"""


def test_hilbert_key_is_a_unit_step_bijection(tmp_path):
    src = open(SRC).read()
    m = re.search(r"uint64_t hilbert_key\(.*?\n}\n", src, re.S)
    assert m, "hilbert_key not found"
    cpp = tmp_path / "t.cpp"
    cpp.write_text(PROG % m.group(0))
    exe = tmp_path / "t"
    r = subprocess.run(["g++", "-O2", "-o", str(exe), str(cpp)], capture_output=True, text=True)
    if r.returncode != 0:
        pytest.fail(r.stderr)
    out = subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout.split()
    pairs = list(zip(out[::2], out[1::2]))
    assert len(pairs) == 5
    assert all(bad == "0" for _, bad in pairs), pairs
