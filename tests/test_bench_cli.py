"""CPU checks of bench.py's command line: it runs on one GPU only, and the
committed HBM-traffic record is read back for its kernel."""
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    line = json.loads(r.stdout.strip().splitlines()[-1])
    assert line["n_gpus"] == 2 and "one GPU" in line["error"]


def test_traffic_record_is_readable():
    sys.path.insert(0, ROOT)
    import bench

    rec = json.load(open(os.path.join(ROOT, "profiles", "traffic.json")))
    assert "landau_3d3v/f32" in rec
    t = bench.read_traffic("landau_3d3v/f32")
    # None only when the sweep source changed after the counters were taken
    assert t is None or t > 0


def test_alloc_f_falls_back_to_torch():
    """Where the driver cannot provide contiguous memory, bench.py places f
    in an ordinary torch allocation and says so."""
    sys.path.insert(0, ROOT)
    import torch

    import bench

    class _Err(Exception):
        pass

    class _Refusing:
        SlmppError = _Err

        class DeviceBuffer:
            def __init__(self, nbytes, contiguous=True):
                raise _Err("no contiguous memory")

    buf, t, placement = bench.alloc_f(_Refusing, torch, (3, 5), torch.float64, torch.device("cpu"))
    assert buf is None and placement == "default"
    assert t.shape == (3, 5) and t.dtype == torch.float64
