import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (HIP device)")
    config.addinivalue_line("markers", "slow: long CPU-only oracle checks")


@pytest.fixture(scope="session")
def gpu_lib():
    """The HIP library through its Python binding (GPU tests only)."""
    from paper_1810_03698_amd import pbmp
    lib = pbmp.load()
    return lib


@pytest.fixture
def say(capsys):
    """Print a progress line past pytest's output capture, so that a long
    test reports each finished step as it happens."""
    def _say(*args):
        with capsys.disabled():
            print(*args, flush=True)
    return _say


@pytest.fixture(scope="module")
def say_module(request):
    """`say` for module-scoped fixtures (no capsys there): writes to the
    terminal reporter, which pytest does not capture."""
    tr = request.config.pluginmanager.get_plugin("terminalreporter")

    def _say(*args):
        line = " ".join(str(a) for a in args)
        if tr is not None:
            tr.write_line(line)
        else:
            print(line, flush=True)
    return _say
