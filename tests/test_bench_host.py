"""Host-side logic of bench.py (no GPU): the one-GPU guard, the workload
table, the heat-bath workloads' field generation at a small size, and the
counter-traffic lookup."""
import subprocess
import sys
import os

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, 'bench.py'), '--gpus', '2'], capture_output=True, text=True)
    assert r.returncode == 2
    assert 'one GPU' in r.stderr


def test_workloads_are_well_formed():
    for name, w in bench.WORKLOADS.items():
        assert len(w['dims']) == 4 and len(w['block']) == 4, name
        # SAP colouring needs an even number of blocks in every direction
        assert all((d // b) % 2 == 0 and d % b == 0 for d, b in zip(w['dims'], w['block'])), name
        assert ('eps' in w) != ('gauge' in w), name
        assert bench.gauge_desc(w)


@pytest.mark.parametrize('name', ['hb16', 'hb32'])
def test_heatbath_workload_field_on_the_host(name):
    w = dict(bench.WORKLOADS[name])
    w['gauge'] = (w['gauge'][0], w['gauge'][1], 2)
    U = bench.gauge_numpy(w, (4, 4, 4, 4))
    assert U.shape == (4, 4, 4, 4, 4, 3, 3)
    assert np.abs(U @ np.conj(np.swapaxes(U, -1, -2)) - np.eye(3)).max() < 1e-12



def test_counter_traffic_lookup():
    # a class without counters, or with counters taken on other sources, has none
    assert bench.counter_traffic('no_such_class', 1.0) is None
    assert bench.counter_traffic('coarse_mv', 1.0) is None or bench.counter_traffic('coarse_mv', 1.0) > 0
