import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: longer CPU test")


@pytest.fixture(scope="session")
def cyl_workload():
    """The 32768-cylinder workload at t = 0 and its brute-force pair list
    (generated once per test session: random sequential placement takes a
    few tens of seconds)."""
    from oracle import beads as obeads
    from synth import configs, state
    cfg = configs.config5()
    print(f"[tests] generating {cfg.name}", flush=True)
    st = state.initial_state(cfg)
    pairs = obeads.pairs_within(st["x"], cfg.box, cfg.r_list)
    return cfg, st, pairs
