import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) and the built HIP library")
    config.addinivalue_line("markers", "slow: longer CPU test")


@pytest.fixture(scope="session")
def repo_root():
    return ROOT


@pytest.fixture(scope="session")
def host_check():
    """Run the sanitized host-check program (built once per session): the
    library's host sources under AddressSanitizer and UndefinedBehaviorSanitizer.
    Returns run(mode) -> (exit status, combined output)."""
    import shutil
    import subprocess

    if shutil.which("hipcc") is None and not os.path.exists("/opt/rocm/bin/hipcc"):
        pytest.skip("hipcc is needed to build the sanitized host check")
    from paper_1909_04573_amd import build

    exe = build.build_host_check()
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1", UBSAN_OPTIONS="print_stacktrace=1")

    def run(mode):
        r = subprocess.run([exe, mode], capture_output=True, text=True, timeout=300, env=env)
        return r.returncode, r.stdout + r.stderr

    return run


def pytest_collection_modifyitems(config, items):
    try:
        import torch

        has_gpu = torch.cuda.is_available()
    except Exception:  # pragma: no cover
        has_gpu = False
    if has_gpu:
        return
    skip = pytest.mark.skip(reason="needs a GPU")
    for it in items:
        if "gpu" in it.keywords:
            it.add_marker(skip)
