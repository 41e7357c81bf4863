import functools
import os
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (runs through the HIP library)")
    config.addinivalue_line("markers", "slow: larger CPU cases")


def oracle_truth_forward(spec, x0, steps):
    """Truth trajectory for observation synthesis, computed by the oracle."""
    from oracle import model
    return model.forward_at(model.Grid.of(spec), x0, steps)


@functools.lru_cache(maxsize=None)
def _problem(name, key=()):
    import synth
    cfg = synth.CONFIGS[name] if isinstance(name, str) else None
    kw = dict(key)
    return synth.make_problem(cfg if cfg is not None else name, oracle_truth_forward, **kw)


def problem(name, **kw):
    """Cached synthetic problem whose observations come from the oracle truth run."""
    return _problem(name, tuple(sorted(kw.items())))


def custom_problem(cfg, **kw):
    import synth
    return synth.make_problem(cfg, oracle_truth_forward, **kw)


@pytest.fixture
def rng():
    return np.random.default_rng(20220513)
