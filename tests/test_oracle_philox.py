"""Pins for the oracle's Philox4x32-10 (SC'11, section 4.2)."""
import numpy as np

from oracle import philox

# Known-answer vectors published with the Random123 reference implementation
# of Philox4x32-10: (counter, key) -> output words.
KAT = [
    ((0, 0, 0, 0), (0, 0), (0x6627E8D5, 0xE169C58D, 0xBC57AC4C, 0x9B00DBD8)),
    ((0xFFFFFFFF,) * 4, (0xFFFFFFFF, 0xFFFFFFFF), (0x408F276D, 0x41C83B0E, 0xA20BC7C6, 0x6D5451FD)),
    ((0x243F6A88, 0x85A308D3, 0x13198A2E, 0x03707344), (0xA4093822, 0x299F31D0),
     (0xD16CFE09, 0x94FDCCEB, 0x5001E420, 0x24126EA1)),
]


def test_known_answers():
    for ctr, key, want in KAT:
        got = philox.philox4x32(*ctr, *key)
        assert tuple(int(x) for x in got) == want


def test_vectorised_equals_scalar():
    c0 = np.arange(100, dtype=np.uint64)
    w = philox.philox4x32(c0, 7, 3, 1, 123, 456)
    for i in (0, 17, 99):
        s = philox.philox4x32(i, 7, 3, 1, 123, 456)
        assert all(int(a[i]) == int(b) for a, b in zip(w, s))


def test_uniform_range_and_resolution():
    assert philox.to_unit_double(0, 0) == 0.0
    top = philox.to_unit_double(0xFFFFFFFF, 0xFFFFFFFF)
    assert top == 1.0 - 2.0 ** -53
    u = philox.uniform(99, np.arange(200000, dtype=np.uint64), 0, 0, 0)
    assert u.min() >= 0.0 and u.max() < 1.0
    assert abs(u.mean() - 0.5) < 0.003
    assert abs((u < 0.25).mean() - 0.25) < 0.003


def test_streams_and_keys_differ():
    a = philox.uniform(1, np.arange(1000, dtype=np.uint64), 0, 0, philox.STREAM_SITE)
    b = philox.uniform(1, np.arange(1000, dtype=np.uint64), 0, 0, philox.STREAM_ACCEPT)
    c = philox.uniform(2, np.arange(1000, dtype=np.uint64), 0, 0, philox.STREAM_SITE)
    assert not np.array_equal(a, b) and not np.array_equal(a, c)
    assert philox.key_of((5 << 32) | 9) == (9, 5)
