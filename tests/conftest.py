import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    # a planted oracle mistake (tests/oracle_mutations.py), for the mutation
    # tests' child processes only
    mutation = os.environ.get("QOC_ORACLE_MUTATION")
    if mutation:
        sys.path.insert(0, os.path.dirname(os.path.abspath(__file__)))
        import oracle_mutations
        oracle_mutations.install(mutation)
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: oracle work of more than a few seconds")
