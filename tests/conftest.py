import os
import sys
import tempfile

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

# the library's set-up tuning cache: one fresh file per test session, so that
# tests neither read nor write the user's cache
os.environ.setdefault("ETH_TUNE_CACHE", os.path.join(tempfile.mkdtemp(prefix="eth_tune_"), "tune.txt"))


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: longer CPU oracle checks")
