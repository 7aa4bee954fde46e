"""The stored expected results under tests/golden/ are the oracle's answers
(written by tests/golden/make_golden.py): recomputing them must give the same
numbers, so any change to the oracle's arithmetic shows up here."""
import json
import os
import sys

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
sys.path.insert(0, GOLDEN)

import make_golden  # noqa: E402


def test_golden_fixtures_equal_a_fresh_oracle_run():
    fresh = make_golden.fixtures()
    for name, fx in fresh.items():
        with open(os.path.join(GOLDEN, name + ".json")) as fh:
            assert json.load(fh) == json.loads(json.dumps(fx)), name
