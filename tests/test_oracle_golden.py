"""The oracle reproduces its stored small-workload outputs bit for bit."""
import json
from pathlib import Path

from tests.golden.make_golden import record

GOLDEN = Path(__file__).resolve().parent / "golden" / "small_oracle.json"


def test_small_workload_golden():
    assert record("small") == json.loads(GOLDEN.read_text())
