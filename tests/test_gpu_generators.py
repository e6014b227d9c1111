"""The device generators behind the random decisions against the published
known-answer vectors (tests/golden/philox4x32_10_kat.json) and against the
oracle's independent implementation on many counters."""
import json
import os

import numpy as np
import pytest

from paper_2106_03058_amd import agp

pytestmark = pytest.mark.gpu

_GOLD = os.path.join(os.path.dirname(__file__), "golden", "philox4x32_10_kat.json")


def _kat():
    with open(_GOLD) as f:
        return json.load(f)


def test_device_philox_known_answers():
    v = _kat()["vectors"]
    ctr = [[int(h, 16) for h in e["ctr"]] for e in v]
    key = [[int(h, 16) for h in e["key"]] for e in v]
    out = agp.device_philox4x32_10(ctr, key)
    assert out.tolist() == [[int(h, 16) for h in e["out"]] for e in v]


def test_device_splitmix64_known_answer():
    v = _kat()["splitmix64"]["vectors"]
    out = agp.device_splitmix64([int(e["in"], 16) for e in v])
    assert out.tolist() == [int(e["out"], 16) for e in v]


def test_device_generators_equal_oracle(orc):
    rng = np.random.default_rng(11)
    ctr = rng.integers(0, 2**32, size=(2000, 4), dtype=np.uint64).astype(np.uint32)
    key = rng.integers(0, 2**32, size=(2000, 2), dtype=np.uint64).astype(np.uint32)
    got = agp.device_philox4x32_10(ctr, key)
    for i in range(0, 2000, 97):
        assert got[i].tolist() == orc.philox(ctr[i], key[i]).tolist()
    ids = rng.integers(0, 2**63, size=500, dtype=np.int64).astype(np.uint64)
    sm = agp.device_splitmix64(ids)
    assert [int(v) for v in sm] == [orc.splitmix64(int(v)) for v in ids]


def test_device_generators_reject_bad_arguments():
    with pytest.raises(ValueError):
        agp.device_philox4x32_10(np.zeros((2, 4)), np.zeros((1, 2)))
    assert agp.lib().agp_device_splitmix64(-1, None, None) == agp.AGP_EINVAL
