"""The oracle still reproduces its stored small-case results."""
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.join(HERE, "golden"))


def test_oracle_matches_golden():
    import make_golden
    with open(os.path.join(HERE, "golden", "oracle_small.json")) as f:
        stored = json.load(f)["cases"]
    assert make_golden.compute() == stored
