import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")



_config = None


def pytest_sessionstart(session):
    global _config
    _config = session.config


def pytest_runtest_logstart(nodeid, location):
    # a timestamped line before every test names the case if a run stalls
    import time
    tr = _config.pluginmanager.get_plugin("terminalreporter") if _config else None
    if tr is not None:
        tr.write_line(f"[{time.strftime('%H:%M:%S')}] start {nodeid}", flush=True)
