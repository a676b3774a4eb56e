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


def test_counter_hash_ignores_comments_but_not_code():
    # the counters bench.py reports as `traffic` stay valid across comment
    # edits and are dropped when the code itself changes
    sys.path.insert(0, ROOT)
    import bench
    src = 'int f(int a) { // one\n  /* two\n three */ return a + 1; }\nconst char* s = "x//y";\n'
    same = 'int f(int a) {\n  return a + 1;   // other words\n}\nconst char* s = "x//y";'
    other = 'int f(int a) { return a + 2; }\nconst char* s = "x//y";'
    assert bench._code(src) == bench._code(same)
    assert bench._code(src) != bench._code(other)
    assert '"x//y"' in bench._code(src)
