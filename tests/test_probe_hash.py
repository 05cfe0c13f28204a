"""The probe hash's seed shift (CPU): under the counter hash of the C ABI, probe 64 q + j of a
seed is probe j of seed + q * gamma (gamma = 0x9E3779B97F4A7C15, SplitMix64's increment), as
long as a row has fewer than 2^16 probe words.  The gradient runs wide probe blocks in passes of
a multiple of 64 probes and relies on this identity; checked here with the oracle's own
implementation of the hash."""
from __future__ import annotations

import numpy as np
import pytest

GAMMA = 0x9E3779B97F4A7C15


@pytest.mark.parametrize("seed", [0, 12, 2**64 - 5])
@pytest.mark.parametrize("q", [1, 2, 63])
def test_probe_block_shift_is_a_seed_shift(oracle_lib, seed, q):
    d = 300
    shifted = (seed + q * GAMMA) % 2**64
    for j in (0, 1, 17, 63):
        assert np.array_equal(oracle_lib.probe(seed, 64 * q + j, d), oracle_lib.probe(shifted, j, d))
    # and not for a shift that is not a whole word
    assert not np.array_equal(oracle_lib.probe(seed, 64 * q + 5, d), oracle_lib.probe(shifted, 4, d))
