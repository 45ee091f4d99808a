import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: CPU test that takes tens of seconds")


def pytest_runtest_teardown(item, nextitem):
    """After a GPU test module's last test, return torch's cached device
    memory (the full-size tests hold tens of GB each)."""
    if item.get_closest_marker("gpu") is None:
        return
    if nextitem is not None and nextitem.module is item.module:
        return
    torch = sys.modules.get("torch")
    if torch is not None and torch.cuda.is_available():
        import gc
        gc.collect()
        torch.cuda.empty_cache()
