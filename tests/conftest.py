import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")


def gpu_available() -> bool:
    try:
        import torch
        return torch.cuda.is_available()
    except Exception:
        return False


@pytest.fixture(scope="session")
def oracle():
    import oracle as o
    o.build()
    return o


class _Tuning:
    """Library tuning overrides for one test (bb_set_tuning); every setting is
    restored to automatic when the test ends."""

    def set(self, name, value):
        from paper_2107_05395_amd.solver import set_tuning
        set_tuning(name, None if value is None else int(value))

    def reset(self):
        from paper_2107_05395_amd.solver import TUNING_NAMES, set_tuning
        for n in TUNING_NAMES:
            set_tuning(n, None)


@pytest.fixture
def tuning():
    t = _Tuning()
    yield t
    t.reset()
