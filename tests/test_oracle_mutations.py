"""Each planted oracle mistake (tests/oracle_mutations.py) fails at least
one of the oracle's pins (tests/test_oracle_pins.py), and the unmutated
oracle passes them all.  The pins run in a child pytest process per
mutation, with the mutated oracle installed before collection."""
import os
import subprocess
import sys

import pytest

from oracle_mutations import MUTATIONS, mutated_source

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)


def run_pins(mutation):
    env = dict(os.environ)
    env.pop("QOC_ORACLE_MUTATION", None)
    if mutation:
        env["QOC_ORACLE_MUTATION"] = mutation
    cmd = [sys.executable, "-m", "pytest", os.path.join(HERE, "test_oracle_pins.py"), "-x",
           "-q", "-p", "no:cacheprovider", "-m", "not gpu"]
    return subprocess.run(cmd, cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)


def test_unmutated_oracle_passes_pins():
    r = run_pins(None)
    assert r.returncode == 0, r.stdout[-2000:]


@pytest.mark.parametrize("name", sorted(MUTATIONS))
def test_mutation_fails_a_pin(name):
    mutated_source(name)  # the fragment still exists exactly once
    r = run_pins(name)
    assert r.returncode == 1, f"mutation {name} survived every pin:\n{r.stdout[-2000:]}"
