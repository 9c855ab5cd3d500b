"""Counter-based Gaussian blocks (Philox4x32-10) drawn by the serving loop from a seed.

Pinned by the generator's published known-answer vectors (Salmon et al., SC 2011,
Random123 distribution) and by the C ABI's generator agreeing with the
independent NumPy one in workloads/.
"""

import numpy as np
import pytest

import workloads as W


@pytest.mark.parametrize("ctr,key,expect", [
    ((0, 0, 0, 0), (0, 0), (0x6627E8D5, 0xE169C58D, 0xBC57AC4C, 0x9B00DBD8)),
    ((0xFFFFFFFF,) * 4, (0xFFFFFFFF,) * 2, (0x408F276D, 0x41C83B0E, 0xA20BC7C6, 0x6D5451FD)),
    ((0x243F6A88, 0x85A308D3, 0x13198A2E, 0x03707344), (0xA4093822, 0x299F31D0),
     (0xD16CFE09, 0x94FDCCEB, 0x5001E420, 0x24126EA1)),
])
def test_philox_known_answers(ctr, key, expect):
    out = W.philox4x32_10(np.array([ctr], dtype=np.uint32), key)[0]
    assert tuple(int(v) for v in out) == expect


def test_omega_block_is_standard_complex_gaussian():
    z = W.omega_philox(2024, 1, 3, 500, 40).ravel()
    assert abs(z.mean()) < 0.02
    assert abs(np.mean(np.abs(z) ** 2) - 1.0) < 0.02
    assert abs(np.mean(z.real ** 2) - 0.5) < 0.02 and abs(np.mean(z * z)) < 0.02


def test_omega_blocks_differ_by_level_box_and_seed():
    a = W.omega_philox(7, 1, 0, 30, 5)
    for other in (W.omega_philox(7, 2, 0, 30, 5), W.omega_philox(7, 1, 1, 30, 5), W.omega_philox(8, 1, 0, 30, 5)):
        assert not np.allclose(a, other)


def test_library_generator_matches_numpy_generator():
    import paper_2512_12538_amd as hh

    for seed, level, box, m_in, s in [(0, 1, 0, 17, 5), (2 ** 40 + 12345, 3, 11, 133, 26), (99, 2, 7, 1, 1)]:
        lib = hh.hh_omega_philox(seed, level, box, m_in, s)
        ref = W.omega_philox(seed, level, box, m_in, s)
        assert np.max(np.abs(lib - ref)) < 1e-14
