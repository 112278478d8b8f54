"""The serving arena's ring allocator (csrc/ring_alloc.hpp), compiled on the
host with g++ into a small driver and checked under random allocate /
release sequences: every live allocation lies inside the arena, aligned, and
overlaps no other; space comes back once everything older is released; an
allocation that fits after a full drain always succeeds."""
import os
import random
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER_DIR = os.path.join(ROOT, "paper_1303_4312_amd", "csrc")

DRIVER = r"""
#include <stdio.h>
#include "ring_alloc.hpp"
int main(int argc, char** argv) {
  unsigned long long size = strtoull(argv[1], 0, 10);
  cm::RingAlloc ring(size);
  char op;
  unsigned long long id, bytes;
  while (scanf(" %c", &op) == 1) {
    if (op == 'a') {
      if (scanf("%llu %llu", &id, &bytes) != 2) return 2;
      const long long off = (long long)ring.alloc(bytes, id);
      printf("%lld %llu\n", off, (unsigned long long)ring.used());
    } else if (op == 'r') {
      if (scanf("%llu", &id) != 1) return 2;
      const int ok = ring.release(id) ? 1 : 0;
      printf("%d %llu\n", ok, (unsigned long long)ring.used());
    }
  }
  return 0;
}
"""


@pytest.fixture(scope="module")
def driver(tmp_path_factory):
    d = tmp_path_factory.mktemp("ring")
    src = d / "driver.cpp"
    src.write_text(DRIVER.replace("#include <stdio.h>", "#include <stdio.h>\n#include <stdlib.h>"))
    exe = d / "driver"
    subprocess.run(["g++", "-O1", "-std=c++17", "-I", HEADER_DIR, str(src), "-o", str(exe)],
                   check=True)
    return str(exe)


def run(driver, size, ops):
    text = "\n".join(f"a {i} {b}" if op == "a" else f"r {i}" for op, i, b in ops) + "\n"
    out = subprocess.run([driver, str(size)], input=text, capture_output=True, text=True,
                         check=True).stdout.split("\n")
    return [tuple(int(x) for x in line.split()) for line in out if line.strip()]


def test_fifo_and_wrap(driver):
    size = 256 * 10
    ops = [("a", 1, 1000), ("a", 2, 1000), ("a", 3, 600),   # 1024 + 1024 fit, 768 does not
           ("r", 1, 0), ("a", 4, 600),                       # wraps to 0 once 1 is gone
           ("r", 3, 0),                                      # never allocated: no-op
           ("a", 5, 0),                                      # empty: always at 0
           ("r", 2, 0), ("r", 4, 0), ("a", 6, 2560), ("a", 7, 1)]
    res = run(driver, size, ops)
    assert res[0] == (0, 1024) and res[1] == (1024, 2048)
    assert res[2][0] == -1
    assert res[3] == (1, 1024) and res[4] == (0, 1792)
    assert res[5][0] == 0
    assert res[6][0] == 0 and res[6][1] == 1792
    assert res[7] == (1, 768) and res[8] == (1, 0)
    assert res[9] == (0, 2560)      # whole arena after a full drain
    assert res[10][0] == -1


@pytest.mark.parametrize("seed", range(6))
def test_random_sequences(driver, seed):
    rng = random.Random(seed)
    size = 256 * rng.randint(8, 400)
    ops, live, next_id = [], [], 1
    for _ in range(3000):
        if live and (rng.random() < 0.45 or len(live) > 50):
            ops.append(("r", live.pop(rng.randrange(len(live))), 0))
        else:
            b = rng.choice([0, 1, 255, 256, 257, rng.randint(1, size // 3), rng.randint(1, size)])
            ops.append(("a", next_id, b))
            live.append(next_id)
            next_id += 1
    res = run(driver, size, ops)
    spans = {}
    order = []  # live allocation ids in allocation order
    for (op, i, b), (r0, used) in zip(ops, res):
        if op == "a":
            if r0 < 0:
                assert b > 0
                continue
            if b == 0:
                assert r0 == 0
                continue
            length = -(-b // 256) * 256
            assert r0 % 256 == 0 and 0 <= r0 and r0 + length <= size
            for lo, hi in spans.values():
                assert r0 + length <= lo or hi <= r0, "overlap"
            spans[i] = (r0, r0 + length)
            order.append(i)
        else:
            assert r0 == (1 if i in spans else 0)
            spans.pop(i, None)
        assert used == sum(hi - lo for lo, hi in spans.values())
    # with nothing live, the whole arena is one free range again
    drain = [("r", i, 0) for i in list(spans)] + [("a", 10 ** 9, size)]
    assert run(driver, size, ops + drain)[-1][0] == 0
