"""ctypes binding of libdp.so (include/dp.h): argument marshalling only.

Every step of the force computation runs in the library's HIP kernels; this
module converts torch tensors to device pointers and numpy arrays to host
pointers, and turns error codes into exceptions.  It raises at import time
when the library has not been built: there is no fallback.
"""
import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libdp.so")

DP_OK = 0
STATUS = {0: "DP_OK", -1: "DP_ERR_ARG", -2: "DP_ERR_HIP", -3: "DP_ERR_OOM", -4: "DP_ERR_CAPACITY",
          -5: "DP_ERR_UNSUPPORTED", -6: "DP_ERR_STATE", -7: "DP_ERR_NONFINITE", -8: "DP_ERR_SKIN"}
FP64, FP32, MIXED_BF16 = 0, 1, 2
COMPRESSED, PLAIN, TAB_UNFUSED, FUSED_PADDED, FUSED = 0, 1, 2, 3, 4


class DPError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


class ModelConfig(ctypes.Structure):
    _fields_ = [("ntypes", ctypes.c_int), ("rcut", ctypes.c_double), ("rcut_smth", ctypes.c_double),
                ("sel", ctypes.c_int), ("emb", ctypes.c_int * 3), ("m_lt", ctypes.c_int),
                ("fit", ctypes.c_int * 3), ("desc_scale", ctypes.c_double), ("switch_kind", ctypes.c_int),
                ("sel_t", ctypes.c_int * 4)]


if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is missing: build it with `python paper_2201_01446_amd/build.py`")

lib = ctypes.CDLL(LIB_PATH)
_vp, _i, _d, _sz = ctypes.c_void_p, ctypes.c_int, ctypes.c_double, ctypes.c_size_t
_pvp = ctypes.POINTER(ctypes.c_void_p)
_pi = ctypes.POINTER(ctypes.c_int)
_SIG = {
    "dp_model_create": [ctypes.POINTER(ModelConfig), _vp, _sz, _pvp],
    "dp_model_destroy": [_vp],
    "dp_tabulate": [_vp, _d, _d, _d, _d, _vp],
    "dp_fitting_tanh": [_vp, _i, _vp],
    "dp_table_download": [_vp, _vp, _pi],
    "dp_tanh_table_download": [_vp, _vp, _pi],
    "dp_build_nlist": [_vp, _i, _vp, _vp, _vp, _d, _pvp, _vp],
    "dp_nlist_destroy": [_vp],
    "dp_compute": [_vp, _vp, _i, _vp, _vp, _vp, _i, _i, _vp, _vp, _vp, _vp, _vp],
    "dp_compute_noalloc": [_vp, _vp, _i, _vp, _vp, _vp, _i, _i, _vp, _vp, _vp, _vp, _vp],
    "dp_descriptor": [_vp, _vp, _i, _vp, _vp, _i, _i, _vp, _vp, _vp, _vp, _vp],
    "dp_energy_forward": [_vp, _vp, _i, _vp, _i, _i, _vp, _vp, _vp],
    "dp_energy_backward": [_vp, _vp, _i, _vp, _i, _i, _vp, _vp, _vp],
    "dp_nlist_stats": [_vp, _pi, _pi, _pi, _pi],
    "dp_nlist_check": [_vp],
    "dp_nlist_export": [_vp, _pi, _pi, _vp, _vp, _vp, _vp, _vp, _vp],
    "dp_nve_run": [_vp, _pvp, _i, _vp, _vp, _vp, _vp, _vp, _d, _i, _i, _d, _i, _i, _vp, _vp],
    "dp_nve_continue": [_vp, _vp, _i, _vp, _vp, _vp, _d, _i, _i, _i, _i, _vp, _vp],
    "dp_batch_create": [_vp, _i, _i, _d, _pvp],
    "dp_batch_destroy": [_vp],
    "dp_batch_compute": [_vp, _vp, _i, _vp, _vp, _i, _vp, _vp, _vp, _vp, _vp],
    "dp_batch_stats": [_vp, _pi, _pi, _pi, _pi],
    "dp_footprint_bytes": [_vp, _i, ctypes.POINTER(_sz)],
    "dp_timers_enable": [_i],
    "dp_timers_read": [_i, _vp, _vp, _vp, _pi],
}
for _name, _args in _SIG.items():
    f = getattr(lib, _name)
    f.argtypes = _args
    f.restype = ctypes.c_int
lib.dp_last_error.argtypes = []
lib.dp_last_error.restype = ctypes.c_char_p


def check(status):
    if status != DP_OK:
        raise DPError(status, lib.dp_last_error().decode())
    return status


def timers_enable(on=True):
    check(lib.dp_timers_enable(1 if on else 0))


def timers_read(max_names=64):
    """{kernel name: (total ms, launches)} since the last read."""
    names = ctypes.create_string_buffer(32 * max_names)
    ms = (ctypes.c_double * max_names)()
    cnt = (ctypes.c_int * max_names)()
    n = ctypes.c_int()
    check(lib.dp_timers_read(max_names, names, ms, cnt, ctypes.byref(n)))
    out = {}
    for k in range(n.value):
        nm = names.raw[32 * k:32 * k + 32].split(b"\0")[0].decode()
        out[nm] = (ms[k], cnt[k])
    return out
