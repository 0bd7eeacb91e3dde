"""Oracle pin: Philox4x32-10 against an independent library implementation.

The oracle's Philox is written from the published round function (Salmon et
al., SC'11).  It is pinned here to rocRAND's host-callable Philox4x32-10
engine: a small program built from tests/pins/ calls the library's engine
with (seed, subsequence, offset) and prints the blocks.  rocRAND's engine uses
key = seed and counter = (offset/4 as 64 bits, subsequence as 64 bits), which
is the oracle's counter layout (particle index, segment id, draw).
"""
import os
import shutil
import subprocess

import numpy as np
import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
PIN_SRC = os.path.join(HERE, "pins", "rocrand_philox_blocks.cpp")


@pytest.fixture(scope="module")
def rocrand_pin(tmp_path_factory):
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not available to build the rocRAND pin")
    exe = str(tmp_path_factory.mktemp("pin") / "rocrand_philox_blocks")
    subprocess.run([hipcc, "-O1", "-x", "hip", "--offload-arch=gfx950", PIN_SRC, "-o", exe],
                   check=True, capture_output=True)

    def blocks(seed, subseq, first, count):
        out = subprocess.run([exe, str(seed), str(subseq), str(first), str(count)],
                             check=True, capture_output=True, text=True).stdout
        return np.array([[int(w) for w in line.split()] for line in out.strip().splitlines()],
                        dtype=np.uint32)
    return blocks


CASES = [
    # seed, segment id, draw, first particle index, count
    (0, 0, 0, 0, 64),
    (1, 0, 0, 12345, 32),
    (2, 0, 0, (1 << 32) - 8, 16),          # particle index crossing 2^32
    (4, 12287, 0, 0, 16),                   # batched segment id
    (0x0123456789ABCDEF, 7, 3, 99, 16),     # 64-bit seed, later draw
    ((1 << 64) - 1, (1 << 32) - 1, (1 << 32) - 1, (1 << 40) + 5, 8),
]


@pytest.mark.parametrize("seed,seg,draw,first,count", CASES)
def test_philox_matches_rocrand(orc, rocrand_pin, seed, seg, draw, first, count):
    got = orc.philox_blocks(count, seed, counter_offset=first, seg=seg, draw=draw)
    ref = rocrand_pin(seed, (draw << 32) | seg, first, count)
    np.testing.assert_array_equal(got, ref)


def test_philox_bits_balanced(orc):
    """Each of the 128 output bits is set about half the time (binomial 6 sigma)."""
    n = 1 << 16
    r = orc.philox_blocks(n, 12345)
    bits = np.unpackbits(r.view(np.uint8), axis=1)
    frac = bits.mean(axis=0)
    assert np.all(np.abs(frac - 0.5) < 6 * 0.5 / np.sqrt(n))
