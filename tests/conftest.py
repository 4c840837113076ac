import os
import runpy
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

# Build the HIP library and the oracle only when nothing is built yet.
_LIB = os.path.join(ROOT, "paper_2203_02530_amd", "libspmv.so")
if not os.path.exists(_LIB):
    runpy.run_path(os.path.join(ROOT, "paper_2203_02530_amd", "build.py"))["build"]()


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU")
    config.addinivalue_line("markers", "slow: full-size case (minutes on CPU)")
