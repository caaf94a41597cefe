"""Pin of the oracle's Philox4x32-10 against an independent implementation.

The generator is a reading (the paper only asks for a seeded generator,
Sec. 2.1); its definition is Salmon et al., SC'11.  rocRAND ships its own
Philox4x32-10 engine as header source; ``tests/golden/philox_rocrand_host.cpp``
builds it for the host and the oracle must reproduce its words exactly, at
counters that exercise every word, the carry-free high words and the tag
values the sketches use (0xFFFFFFFF, 0xFFFFFFFE).
"""

import os
import shutil
import subprocess

import numpy as np
import pytest

from oracle.philox import philox4x32

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "golden", "philox_rocrand_host.cpp")


def _hipcc():
    for cand in (shutil.which("hipcc"), "/opt/rocm/bin/hipcc"):
        if cand and os.path.exists(cand):
            return cand
    return None


@pytest.fixture(scope="module")
def rocrand_host(tmp_path_factory):
    hipcc = _hipcc()
    if hipcc is None or not os.path.exists("/opt/rocm/include/rocrand/rocrand_philox4x32_10.h"):
        pytest.skip("hipcc / rocRAND headers not available")
    exe = str(tmp_path_factory.mktemp("philox") / "philox_ref")
    subprocess.run([hipcc, "-O1", "--offload-arch=gfx950", SRC, "-o", exe], check=True,
                   stdout=subprocess.PIPE, stderr=subprocess.PIPE)
    return exe


def _cases():
    g = np.random.Generator(np.random.PCG64(7))
    rows = [
        (0, 0, 0, 0, 0, 0),
        (0xFFFFFFFF, 0xFFFFFFFF, 0xFFFFFFFF, 0xFFFFFFFF, 0xFFFFFFFF, 0xFFFFFFFF),
        (42, 0, 0, 0, 0, 0),
        (42, 0, 5, 0xFFFFFFFF, 1, 0),          # SRHT sign word layout
        (42, 0, 17, 0xFFFFFFFE, 0, 3),         # SRHT row draw layout
        (42, 0, 1234, 77, 2, 9),               # Gaussian entry layout
    ]
    for _ in range(40):
        rows.append(tuple(int(v) for v in g.integers(0, 2 ** 32, size=6, dtype=np.uint64)))
    return rows


def test_philox_matches_rocrand_engine(rocrand_host):
    cases = _cases()
    text = "\n".join(" ".join(str(v) for v in c) for c in cases) + "\n"
    out = subprocess.run([rocrand_host], input=text.encode(), check=True,
                         stdout=subprocess.PIPE).stdout.decode().split("\n")
    ref = np.array([[int(v) for v in line.split()] for line in out if line.strip()], dtype=np.uint64)
    key = np.array([[c[0], c[1]] for c in cases], dtype=np.uint64)
    ctr = np.array([[c[2], c[3], c[4], c[5]] for c in cases], dtype=np.uint64)
    got = philox4x32(ctr, key).astype(np.uint64)
    assert ref.shape == got.shape
    bad = np.nonzero((ref != got).any(axis=1))[0]
    assert bad.size == 0, "mismatch at cases %s" % bad[:5]


def test_philox_is_a_bijection_for_fixed_key():
    # Each round is invertible, so distinct counters give distinct outputs.
    ctr = np.zeros((1 << 16, 4), dtype=np.uint64)
    ctr[:, 0] = np.arange(1 << 16)
    out = philox4x32(ctr, (42, 0))
    packed = {tuple(r) for r in out.tolist()}
    assert len(packed) == 1 << 16


def test_philox_bits_are_balanced():
    ctr = np.zeros((1 << 15, 4), dtype=np.uint64)
    ctr[:, 0] = np.arange(1 << 15)
    ctr[:, 1] = 3
    words = philox4x32(ctr, (42, 0)).reshape(-1)
    bits = np.unpackbits(words.view(np.uint8))
    frac = bits.mean()
    # 2**22 bits: the mean of fair bits has sd 2.4e-4
    assert abs(frac - 0.5) < 2e-3
