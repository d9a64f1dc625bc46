"""The numpy reference of the synthetic-noise stream (tests/philox_ref.py),
pinned by the published known-answer vectors of Philox4x32-10 (Random123's
test vectors: zero counter and key, all-ones counter and key, and the pi
digits) and by the moments of its normals."""
import numpy as np

from philox_ref import normals, philox4x32_10

KAT = [
    ((0, 0, 0, 0), (0, 0), (0x6627E8D5, 0xE169C58D, 0xBC57AC4C, 0x9B00DBD8)),
    ((0xFFFFFFFF,) * 4, (0xFFFFFFFF, 0xFFFFFFFF), (0x408F276D, 0x41C83B0E, 0xA20BC7C6, 0x6D5451FD)),
    ((0x243F6A88, 0x85A308D3, 0x13198A2E, 0x03707344), (0xA4093822, 0x299F31D0),
     (0xD16CFE09, 0x94FDCCEB, 0x5001E420, 0x24126EA1)),
]


def test_philox_known_answers():
    for ctr, key, expect in KAT:
        out = philox4x32_10(np.array([ctr], dtype=np.uint64), key)[0]
        assert [int(v) for v in out] == list(expect)


def test_normals_moments():
    z = normals(1 << 20, 1806)
    assert abs(z.mean()) < 5e-3
    assert abs(z.std() - 1.0) < 5e-3
    # fourth moment of a standard normal is 3
    assert abs(np.mean(z ** 4) - 3.0) < 0.05
    # a different seed gives a different stream
    assert not np.allclose(z[:100], normals(100, 1807))
