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


def _write_counter_csv(path, rows):
    os.makedirs(path, exist_ok=True)
    with open(os.path.join(path, 'x_counter_collection.csv'), 'w') as f:
        f.write('Correlation_Id,Dispatch_Id,Kernel_Name,Counter_Name,Counter_Value\n')
        for d, k, v in rows:
            f.write('%d,%d,"%s",C,%r\n' % (d, d, k, v))


def test_counter_summary_calibrates_and_divides_by_units(tmp_path):
    """The counter summary scales by the 1 GiB calibration copies, keeps only
    the dispatches after them, and divides by the measured pass's units."""
    import json
    V = 1024
    units = dict(V=V, workload=[8, 8, 4, 4], classes={c: dict(units=0.0, bytes=0.0) for c in bench.CLASSES})
    units['classes']['sap_half'] = dict(units=12.0, bytes=5e6)  # 12 RHS-launches of a half-sweep
    units['classes']['dslash64'] = dict(units=2.0, bytes=3e6)
    uj = tmp_path / 'units.json'
    uj.write_text(json.dumps(units))
    copy = '__amd_rocclr_copyBuffer'
    # fetch counter reads half the bytes (factor 2), write counter all of them (factor 1)
    fetch = [(1, 'void wc::k_sap_dom<512>(wc::Geo)', 999.0)] + [(2 + i, copy, 524288.0) for i in range(3)] + \
            [(5, 'void wc::k_sap_dom<512>(wc::Geo)', 100.0), (6, 'void wc::k_dslash_lds<double, double2>(wc::Geo)', 50.0),
             (7, copy, 10.0)]
    write = [(1, 'void wc::k_sap_dom<512>(wc::Geo)', 999.0)] + [(2 + i, copy, 1048576.0) for i in range(3)] + \
            [(5, 'void wc::k_sap_dom<512>(wc::Geo)', 30.0), (6, 'void wc::k_dslash_lds<double, double2>(wc::Geo)', 10.0),
             (7, copy, 10.0)]
    _write_counter_csv(str(tmp_path / 'f'), fetch)
    _write_counter_csv(str(tmp_path / 'w'), write)
    out = bench.summarize_counters(str(tmp_path / 'f'), str(tmp_path / 'w'), str(uj), str(tmp_path / 'o.json'))
    k = out['kernels']
    assert k['sap_half']['dispatches'] == 1
    assert k['sap_half']['fetch_bytes'] == pytest.approx(100 * 1024 * 2.0)
    assert k['sap_half']['write_bytes'] == pytest.approx(30 * 1024 * 1.0)
    assert k['sap_half']['fetch_per_unit'] == pytest.approx(100 * 1024 * 2.0 / (12 * V / 2))
    assert k['dslash64']['write_per_unit'] == pytest.approx(10 * 1024 / (2 * V))
    assert k['coarse_mv']['dispatches'] == 0
