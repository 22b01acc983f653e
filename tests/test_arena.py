"""The served form's arena allocator (csrc/pt_arena.h, plain C++) against a
first-fit model written here: random alloc/release sequences must return the
same offsets, keep allocations disjoint and inside the arena, and coalesce
every free neighbour, so that releasing everything leaves one free range."""
import os
import random
import subprocess
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2512_03825_amd", "csrc")

DRIVER = r"""
#include "pt_arena.h"
#include <cstdio>
int main() {
  size_t size, align;
  if (scanf("%zu %zu", &size, &align) != 2) return 2;
  ptmi::Arena a(size, align);
  char op;
  size_t x, y;
  while (scanf(" %c", &op) == 1) {
    if (op == 'a') {
      scanf("%zu", &x);
      size_t off = 0;
      bool ok = a.alloc(x, &off);
      printf("%d %zu\n", ok ? 1 : 0, ok ? off : 0);
    } else if (op == 'r') {
      scanf("%zu %zu", &x, &y);
      printf("%d\n", a.release(x, y) ? 1 : 0);
    } else if (op == 's') {
      printf("%zu %zu %zu %zu\n", a.used(), a.peak(), a.largest_free(), a.free_ranges());
    }
  }
  return 0;
}
"""


@pytest.fixture(scope="module")
def driver():
    d = tempfile.mkdtemp()
    src = os.path.join(d, "arena_driver.cpp")
    exe = os.path.join(d, "arena_driver")
    open(src, "w").write(DRIVER)
    subprocess.run(["g++", "-std=c++17", "-O1", "-Wall", "-I", CSRC, src, "-o", exe], check=True)
    return exe


class Model:
    """First fit over a sorted list of free (offset, length) ranges."""

    def __init__(self, size, align):
        self.align = align
        self.size = size - size % align
        self.free = [(0, self.size)] if self.size else []
        self.used = self.peak = 0

    def rnd(self, n):
        return -(-n // self.align) * self.align

    def alloc(self, n):
        n = self.rnd(n)
        if n == 0 or n > self.size:
            return None
        for i, (o, l) in enumerate(self.free):
            if l >= n:
                self.free[i:i + 1] = [(o + n, l - n)] if l > n else []
                self.used += n
                self.peak = max(self.peak, self.used)
                return o
        return None

    def release(self, off, n):
        n = self.rnd(n)
        self.free.append((off, n))
        self.free.sort()
        merged = []
        for o, l in self.free:
            if merged and merged[-1][0] + merged[-1][1] == o:
                merged[-1] = (merged[-1][0], merged[-1][1] + l)
            else:
                merged.append((o, l))
        self.free = merged
        self.used -= n


def run(driver, size, align, ops):
    text = "%d %d\n" % (size, align) + "\n".join(ops) + "\n"
    out = subprocess.run([driver], input=text, capture_output=True, text=True, check=True).stdout
    return out.split("\n")


@pytest.mark.parametrize("seed", [0, 1, 2, 3])
def test_random_sequences_match_first_fit(driver, seed):
    rng = random.Random(seed)
    size, align = 1 << 20, 256
    model = Model(size, align)
    live = []
    ops, expect = [], []
    for _ in range(2000):
        if live and rng.random() < 0.45:
            off, n = live.pop(rng.randrange(len(live)))
            ops.append("r %d %d" % (off, n))
            model.release(off, n)
            expect.append(("r", True))
        else:
            n = rng.choice([1, 255, 256, 257, 4096, 30000, 70000, 200000])
            off = model.alloc(n)
            ops.append("a %d" % n)
            expect.append(("a", off))
            if off is not None:
                live.append((off, n))
        if rng.random() < 0.05:
            ops.append("s")
            expect.append(("s", (model.used, model.peak,
                                 max([l for _, l in model.free], default=0), len(model.free))))
    # release everything: one free range of the whole arena remains
    for off, n in live:
        ops.append("r %d %d" % (off, n))
        model.release(off, n)
        expect.append(("r", True))
    ops.append("s")
    expect.append(("s", (0, model.peak, size, 1)))
    lines = run(driver, size, align, ops)
    for (kind, want), line in zip(expect, lines):
        f = line.split()
        if kind == "a":
            ok, off = int(f[0]), int(f[1])
            assert (off if ok else None) == want
        elif kind == "r":
            assert f == ["1"]
        else:
            assert tuple(int(v) for v in f) == want
    assert model.free == [(0, size)]


def test_allocations_are_disjoint_and_inside(driver):
    rng = random.Random(7)
    size, align = 3 * 4096 + 100, 64
    ops = ["a %d" % rng.choice([1, 64, 100, 1000, 5000]) for _ in range(40)]
    lines = run(driver, size, align, ops)
    got = []
    for op, line in zip(ops, lines):
        ok, off = map(int, line.split())
        if ok:
            n = -(-int(op.split()[1]) // align) * align
            assert off % align == 0 and off + n <= size - size % align
            got.append((off, off + n))
    got.sort()
    assert all(a[1] <= b[0] for a, b in zip(got, got[1:]))


def test_bad_releases_are_refused(driver):
    lines = run(driver, 4096, 256, ["a 512", "r 0 512", "r 0 512", "r 256 256", "r 4096 256",
                                    "r 100 256", "a 4097", "a 0", "s"])
    assert lines[0] == "1 0"
    assert lines[1:6] == ["1", "0", "0", "0", "0"]  # double free, free space, past the end, unaligned
    assert lines[6] == "0 0" and lines[7] == "0 0"  # larger than the arena, empty
    assert lines[8] == "0 512 4096 1"
