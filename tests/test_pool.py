"""The request server's HBM-budget allocator (host code, CPU only), compiled
with g++ into a small driver and compared with a plain first-fit model over a
list of free ranges: the same offsets for every request, the same bytes in
use and peak, free neighbours merged back into a single range, and the
allocator's index of free lengths equal to its free ranges after every run."""
import os
import random
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)


class FirstFitModel:
    """First fit: sizes round up to 256; the lowest free offset that holds the
    request; a release merges with adjacent free ranges."""

    def __init__(self, size):
        size &= ~255
        self.free = [[0, size]] if size else []
        self.used = self.peak = 0

    def alloc(self, b):
        b = (b + 255) & ~255
        for r in self.free:
            if r[1] >= b:
                off = r[0]
                r[0] += b
                r[1] -= b
                self.used += b
                self.peak = max(self.peak, self.used)
                self.free = [x for x in self.free if x[1] > 0]
                return off
        return -1

    def release(self, off, b):
        b = (b + 255) & ~255
        self.used -= b
        self.free.append([off, b])
        self.free.sort()
        merged = []
        for r in self.free:
            if merged and merged[-1][0] + merged[-1][1] == r[0]:
                merged[-1][1] += r[1]
            else:
                merged.append(r)
        self.free = merged


@pytest.fixture(scope="module")
def driver(tmp_path_factory):
    if shutil.which("g++") is None:
        pytest.skip("g++ is not installed")
    exe = str(tmp_path_factory.mktemp("pool") / "pool_driver")
    subprocess.run(["g++", "-O1", "-g", "-std=c++17", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
                    "-I", os.path.join(ROOT, "paper_1903_00227_amd", "csrc"), os.path.join(HERE, "pool_driver.cpp"),
                    "-o", exe], check=True, capture_output=True, text=True)
    return exe


def run(exe, size, ops):
    text = f"{size}\n" + "".join(f"a {o[1]}\n" if o[0] == "a" else f"r {o[1]} {o[2]}\n" for o in ops)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=1:verify_asan_link_order=0")
    r = subprocess.run([exe], input=text, capture_output=True, text=True, env=env, timeout=120)
    assert r.returncode == 0, r.stderr[-2000:]
    lines = r.stdout.split("\n")
    nalloc = sum(1 for o in ops if o[0] == "a")
    offs = [int(x) for x in lines[:nalloc]]
    used, peak, ranges, sz, index_ok = (int(x) for x in lines[nalloc].split())
    assert index_ok == 1  # the length index matches the free ranges
    return offs, used, peak, ranges, sz


def test_hand_cases(driver):
    # fill, free the middle, refill it exactly; ranges merge back to one
    ops = [("a", 300), ("a", 256), ("a", 1000)]
    offs, used, peak, ranges, sz = run(driver, 4096, ops)
    assert offs == [0, 512, 768] and used == 512 + 256 + 1024 and ranges == 1 and sz == 4096
    ops = [("a", 256), ("a", 256), ("a", 256), ("r", 256, 256), ("a", 200), ("r", 0, 256), ("r", 256, 1),
           ("r", 512, 256)]
    offs, used, peak, ranges, sz = run(driver, 1024, ops)
    assert offs == [0, 256, 512, 256] and used == 0 and peak == 768 and ranges == 1
    # too large, and a region smaller than one unit
    assert run(driver, 1024, [("a", 1025)])[0] == [-1]
    assert run(driver, 255, [("a", 1)])[0] == [-1]


@pytest.mark.parametrize("seed", range(4))
def test_random_sequences_match_first_fit(driver, seed):
    rng = random.Random(seed)
    size = rng.choice([1 << 16, 1 << 20, (1 << 20) + 200])
    m = FirstFitModel(size)
    live, ops, offs = [], [], []
    for _ in range(3000):
        if live and rng.random() < 0.45:
            off, b = live.pop(rng.randrange(len(live)))
            ops.append(("r", off, b))
            m.release(off, b)
        else:
            b = rng.choice([1, 255, 256, 257, 1000, 4096, rng.randrange(1, 1 << 14)])
            ops.append(("a", b))
            off = m.alloc(b)  # where it lands, so later releases name the right offset
            offs.append(off)
            if off >= 0:
                live.append((off, b))
    got = run(driver, size, ops)
    assert got[0] == offs
    assert got[1:4] == (m.used, m.peak, len(m.free))
