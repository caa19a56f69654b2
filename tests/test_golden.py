"""The oracle still reproduces the stored fixture written by
``tests/golden/make_golden.py`` (oracle + generators only)."""
import json
import os

from tests.golden import make_golden


def test_oracle_matches_stored_fixture(oracle_lib):
    with open(make_golden.OUT) as f:
        stored = json.load(f)
    now = json.loads(json.dumps(make_golden.compute(), sort_keys=True))
    assert now == stored
