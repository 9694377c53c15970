import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: CPU test that takes more than a few seconds")


@pytest.fixture(scope="session")
def water8():
    import synth
    return synth.make_workload("water8")


@pytest.fixture(scope="session")
def golden_theta():
    """Hand-derived Theta cases of tests/golden/theta_identity_rows.txt."""
    import importlib.util
    spec = importlib.util.spec_from_file_location("golden_load", os.path.join(ROOT, "tests", "golden", "load.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod.theta_identity_rows()


@pytest.fixture(scope="session")
def full_kmeans_ref():
    """get(name) -> (workload dict, oracle K-means with the workload's round
    count from its seeds and the oracle's weight), computed once per session
    (tens of seconds of host time for the 64-water and SiO2 grids)."""
    import time

    import oracle
    import synth

    cache = {}

    def get(name):
        if name not in cache:
            d = synth.make_workload(name)
            wl = d["wl"]
            t0 = time.time()
            w = oracle.weight(d["phi"], None if wl.aliased else d["psi"])
            km = oracle.kmeans(wl.n, w, d["c0"], wl.kmeans_iters)
            print(f"[oracle] {name}: {km['iters']} K-means rounds in {time.time() - t0:.1f} s, "
                  f"{km['near_ties']} near ties", flush=True)
            cache[name] = (d, km)
        return cache[name]

    return get
