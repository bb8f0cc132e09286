"""The numpy Philox used to check the renderer's noise, against the published
known-answer vectors of Philox4x32-10."""
import numpy as np

from philox_ref import philox4x32_10


def _run(ctr, key):
    out = philox4x32_10(*[np.array([v], np.uint32) for v in ctr], *key)
    return [int(v[0]) for v in out]


def test_known_answers():
    assert _run((0, 0, 0, 0), (0, 0)) == [0x6627E8D5, 0xE169C58D, 0xBC57AC4C, 0x9B00DBD8]
    f = 0xFFFFFFFF
    assert _run((f, f, f, f), (f, f)) == [0x408F276D, 0x41C83B0E, 0xA20BC7C6, 0x6D5451FD]
    assert _run((0x243F6A88, 0x85A308D3, 0x13198A2E, 0x03707344), (0xA4093822, 0x299F31D0)) == \
        [0xD16CFE09, 0x94FDCCEB, 0x5001E420, 0x24126EA1]
