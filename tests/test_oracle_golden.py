"""The oracle still reproduces its stored snapshot (tests/golden/oracle_small.json)."""
import json
import os

import pytest

from tests.golden.make_golden import snapshot


def test_oracle_matches_golden_snapshot():
    path = os.path.join(os.path.dirname(__file__), "golden", "oracle_small.json")
    ref = json.load(open(path))
    cur = snapshot()
    assert cur["delta"] == pytest.approx(ref["delta"], rel=1e-12)
    for case in ("u0", "u_true"):
        for k, v in ref[case].items():
            assert cur[case][k] == pytest.approx(v, rel=1e-10, abs=1e-12), (case, k)
