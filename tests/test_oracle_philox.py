"""Pin the oracle's Philox4x32-10 against an independent library implementation.

The library reference is PyTorch's header-only ``at::philox_engine``
(tests/helpers/philox_library_pin.cpp), compiled here with g++.  A dropped
round, a swapped multiplier or a wrong key bump changes every output word.
"""
import os
import subprocess

import numpy as np
import pytest

HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.fixture(scope="module")
def library_philox(tmp_path_factory):
    import torch
    inc = os.path.join(os.path.dirname(torch.__file__), "include")
    exe = str(tmp_path_factory.mktemp("philox") / "philox_pin")
    subprocess.check_call(["g++", "-O1", "-std=c++17", "-I" + inc,
                           os.path.join(HERE, "helpers", "philox_library_pin.cpp"), "-o", exe])

    def run(rows):
        text = "\n".join(" ".join(str(int(v)) for v in r) for r in rows) + "\n"
        out = subprocess.run([exe], input=text, capture_output=True, text=True, check=True).stdout
        return np.array([[int(t) for t in ln.split()] for ln in out.strip().splitlines()],
                        dtype=np.uint64).astype(np.uint32)
    return run


def test_philox_matches_library(orc, library_philox):
    rng = np.random.default_rng(11)
    rows = [[0, 0, 0, 0, 0, 0], [2**32 - 1] * 6, [1, 0, 0, 0, 0, 0], [0, 0, 0, 0, 1, 0],
            [0, 0, 0, 0, 0, 1], [5, 7, 3, 0x80000003, 20260609, 0]]
    rows += rng.integers(0, 2**32, size=(2000, 6), dtype=np.uint64).tolist()
    ref = library_philox(rows)
    got = np.array([orc.philox4x32_10(r[:4], r[4:]) for r in rows], dtype=np.uint32)
    assert got.shape == ref.shape
    mism = np.nonzero((got != ref).any(axis=1))[0]
    assert mism.size == 0, f"first mismatch at row {mism[:5]}: {got[mism[0]]} vs {ref[mism[0]]}"


def test_philox_output_bits_are_balanced(orc):
    # Sanity on the counter layout used for moves: consecutive bead counters
    # give independent-looking words (each output bit set ~half the time).
    words = np.array([orc.philox4x32_10([i, 3, 17, 0], [20260609, 0]) for i in range(4096)],
                     dtype=np.uint32)
    bits = np.unpackbits(words.view(np.uint8)).reshape(-1, 8).mean()
    assert abs(bits - 0.5) < 0.01
