"""Host-side checks of the C-ABI library (no GPU needed): it loads, exports
every symbol the headers declare, and rejects bad arguments with the
documented status before touching the device."""
import ctypes
import glob
import os
import re

import numpy as np
import pytest

import synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    names = set()
    for h in glob.glob(os.path.join(ROOT, "include", "*.h")):
        text = open(h).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        names.update(re.findall(r"\b(dp_[a-z_0-9]+)\s*\(", text))
    return names


def test_library_exports_declared_symbols():
    from paper_2201_01446_amd import _lib
    names = declared_symbols()
    assert {"dp_build_nlist", "dp_tabulate", "dp_compute"} <= names
    for n in sorted(names):
        assert hasattr(_lib.lib, n), n


def test_python_binding_names_match_header():
    from paper_2201_01446_amd import _lib
    assert set(_lib._SIG) | {"dp_last_error"} == declared_symbols()


def test_bad_arguments_are_rejected():
    from paper_2201_01446_amd import _lib
    cfg = synth.copper_model_config()
    p = synth.model_params(cfg)
    P = __import__("paper_2201_01446_amd")
    with pytest.raises(P.DPError) as e:
        P.Model(dict(cfg, sel=0), p)
    assert e.value.status == -5
    with pytest.raises(P.DPError) as e:
        P.Model(cfg, p[:-1])
    assert e.value.status == -1 and "parameter count" in str(e.value)
    with pytest.raises(P.DPError) as e:
        P.Model(dict(cfg, rcut_smth=9.0), p)
    assert e.value.status == -1
    bad = p.copy()
    bad[7] = np.nan
    with pytest.raises(P.DPError):
        P.Model(cfg, bad)
    h = ctypes.c_void_p()
    assert _lib.lib.dp_model_create(None, None, 0, ctypes.byref(h)) == -1
    assert b"NULL" in _lib.lib.dp_last_error()
    assert _lib.lib.dp_tabulate(None, 0.7, 0.01, 1.5, 0.1, None) == -1
    assert _lib.lib.dp_compute(None, None, 0, None, None, None, 0, 0, None, None, None, None, None) == -1
    assert _lib.lib.dp_model_destroy(None) == 0
    assert _lib.lib.dp_nlist_destroy(None) == 0
    assert _lib.lib.dp_nlist_check(None) == -1
    n = ctypes.c_int()
    assert _lib.lib.dp_nlist_export(None, ctypes.byref(n), ctypes.byref(n), None, None, None, None, None,
                                    None) == -1
    assert _lib.lib.dp_tanh_table_download(None, None, None) == -1
    assert _lib.lib.dp_nve_run(None, None, 0, None, None, None, None, None, 1.0, 1, 1, 2.0, 0, 0, None,
                               None) == -1


def test_status_codes_named():
    """Every status the header declares has its name in the binding."""
    from paper_2201_01446_amd import _lib
    text = open(os.path.join(ROOT, "include", "dp.h")).read()
    codes = {int(v): k for k, v in re.findall(r"\b(DP_[A-Z_]+)\s*=\s*(-?\d+)", text) if k.startswith(("DP_OK", "DP_ERR"))}
    assert codes == {k: v for k, v in _lib.STATUS.items()}
    assert codes[-8] == "DP_ERR_SKIN" and codes[-7] == "DP_ERR_NONFINITE"


def test_bench_refuses_more_than_one_gpu():
    """The benchmark runs on one GPU; --gpus 2 exits with a message and status 2."""
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    p = subprocess.run([sys.executable, os.path.join(root, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert p.returncode == 2
    assert "one GPU" in p.stderr
