"""Pins of the oracle's random-number generators (CPU only).

Philox4x32-10 is checked against the published known-answer vectors and, as a
second independent implementation, against rocRAND's host-callable block
function.  SplitMix64 is checked against its reference sequence.
"""
import os
import shutil
import subprocess

import numpy as np
import pytest

import oracle as O

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _rows(name):
    with open(os.path.join(GOLDEN, name)) as f:
        return [l.split() for l in f if l.strip() and not l.startswith("#")]


def test_philox_known_answers():
    for r in _rows("philox4x32_10_kat.txt"):
        v = [int(x, 16) for x in r]
        assert O.philox4x32_10(v[0:4], v[4:6]) == tuple(v[6:10])


def test_splitmix64_reference_sequence():
    for state, out in _rows("splitmix64_seed0.txt"):
        assert O.splitmix64(int(state, 16)) == int(out, 16)


@pytest.mark.skipif(shutil.which("hipcc") is None, reason="hipcc not available")
def test_philox_matches_rocrand_host(tmp_path):
    exe = tmp_path / "rp"
    src = os.path.join(GOLDEN, "rocrand_philox_probe.cpp")
    subprocess.check_call(["hipcc", "-O1", "-I/opt/rocm/include", src, "-o", str(exe)],
                          stdout=subprocess.DEVNULL, stderr=subprocess.DEVNULL)
    g = np.random.Generator(np.random.PCG64(123))
    cases = g.integers(0, 2 ** 32, size=(200, 6), dtype=np.uint64)
    # include the structured counters the renderer uses (pixel, sample, bounce, block)
    cases[:4, :4] = [[0, 0, 0, 0], [4095, 1, 3, 1], [262143, 0, 12, 0], [1, 2, 0, 1]]
    inp = "\n".join(" ".join("%x" % int(v) for v in row) for row in cases) + "\n"
    out = subprocess.run([str(exe)], input=inp, capture_output=True, text=True, check=True)
    got = [tuple(int(x, 16) for x in l.split()) for l in out.stdout.strip().splitlines()]
    assert len(got) == len(cases)
    for row, ref in zip(cases, got):
        assert O.philox4x32_10([int(v) for v in row[:4]], [int(v) for v in row[4:]]) == ref


def test_stream_keys_distinct():
    keys = {O.stream_key(s, it, tag) for s in range(4) for it in range(50) for tag in range(1, 9)}
    assert len(keys) == 4 * 50 * 8
