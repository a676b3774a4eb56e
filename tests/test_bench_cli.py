"""Host-side behaviour of bench.py and the Python binding that needs no GPU."""

import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_bench_refuses_more_than_one_gpu():
    p = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert p.returncode == 2
    assert "one GPU" in p.stderr


def test_band_kind_is_checked_before_any_device_call():
    from paper_2305_04711_amd import cpm
    with pytest.raises(ValueError):
        cpm.Band(cpm.sphere(), [], 16, band="narrow")


def test_batch_needs_one_coefficient_pair_per_band():
    # ctypes would zero-fill a short coefficient list; the binding refuses it
    # before it touches the library or the bands
    from paper_2305_04711_amd import cpm
    for bands, m, n, nrhs in (([object(), object()], [1.0], [-1.0, -1.0], 1),
                              ([object(), object()], [1.0, 1.0], [-1.0], 1),
                              ([], [], [], 1),
                              ([object()], [1.0], [-1.0], 0)):
        with pytest.raises(ValueError):
            cpm.Batch(bands, m, n, nrhs)
