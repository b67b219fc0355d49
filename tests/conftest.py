import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: long-running statistical test")


def pytest_sessionstart(session):
    # tuned kernel choices cached by earlier runs (ess_autotune) must not
    # change what a test's contexts launch: one empty cache per session
    import tempfile
    os.environ["ESS_TUNE_CACHE"] = os.path.join(tempfile.mkdtemp(prefix="ess_tune_"), "tune.json")
