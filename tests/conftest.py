import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: large CPU-only case")


@pytest.fixture(scope="session")
def oracle_mod():
    import oracle
    oracle._load()
    return oracle


@pytest.fixture
def bench_ctx():
    """Make contexts in the launch configuration bench.py times: the
    autotuned shapes of this GPU for the given workload ("single" or
    "batch"), the library defaults when none are stored."""
    made = []

    def make(workload="single"):
        import paper_2103_15217_amd as et
        from paper_2103_15217_amd import autotune
        ctx = et.Context()
        autotune.apply(ctx, workload)
        made.append(ctx)
        return ctx

    yield make
    for ctx in made:
        ctx.close()
