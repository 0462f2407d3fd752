"""Python front end of libdp: handles and calls with torch tensors.

Device arrays are torch CUDA (HIP) tensors; their data pointers are handed to
the library together with the current torch stream.  Boxes are host arrays.
"""
import ctypes

import numpy as np
import torch

from ._lib import (COMPRESSED, FP32, FP64, FUSED, FUSED_PADDED, MIXED_BF16, PLAIN, TAB_UNFUSED, DPError,  # noqa: F401
                   ModelConfig, check, lib)


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t):
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError("device tensor expected")
    if not t.is_contiguous():
        raise ValueError("contiguous tensor expected")
    return ctypes.c_void_p(t.data_ptr())


def _box(box):
    if box is None:
        return None, None
    b = np.ascontiguousarray(np.asarray(box, dtype=np.float64).reshape(9))
    return b, b.ctypes.data_as(ctypes.c_void_p)


def _f64(t, shape):
    if t.dtype != torch.float64 or tuple(t.shape) != shape:
        raise ValueError(f"float64 tensor of shape {shape} expected, got {t.dtype} {tuple(t.shape)}")
    return t


class Model:
    """A model (config + FP64 parameters) resident on the current device."""

    def __init__(self, cfg, params):
        c = ModelConfig()
        c.ntypes = cfg.get("ntypes", 1)
        for t, v in enumerate(cfg.get("sel_t", ())):
            c.sel_t[t] = v
        c.rcut, c.rcut_smth, c.sel = cfg["rcut"], cfg["rcut_smth"], cfg["sel"]
        c.emb[:] = list(cfg["emb"])
        c.m_lt = cfg["m_lt"]
        c.fit[:] = list(cfg["fit"])
        c.desc_scale = cfg["desc_scale"]
        c.switch_kind = cfg.get("switch_kind", 0)
        p = np.ascontiguousarray(params, dtype=np.float64)
        h = ctypes.c_void_p()
        check(lib.dp_model_create(ctypes.byref(c), p.ctypes.data_as(ctypes.c_void_p), p.size, ctypes.byref(h)))
        self.h = h
        self.cfg = dict(cfg)

    def tabulate(self, s_max=0.7, stride=0.01, tail_max=1.5, tail_stride=0.1):
        check(lib.dp_tabulate(self.h, s_max, stride, tail_max, tail_stride, _stream()))
        self.table_args = (s_max, stride, tail_max, tail_stride)
        return self

    def fitting_tanh(self, tabulated=True):
        """The fitting net's tanh in every precision: the second-order table
        (True) or the native function (False)."""
        check(lib.dp_fitting_tanh(self.h, 1 if tabulated else 0, _stream()))
        return self

    def tanh_table(self):
        """FP64 coefficients [1024, 4] of the tabulated tanh (a0, a1, a2, 0 per
        interval of width 1/128 on [0, 8))."""
        n = ctypes.c_int()
        check(lib.dp_tanh_table_download(self.h, None, ctypes.byref(n)))
        out = np.zeros((n.value, 4))
        check(lib.dp_tanh_table_download(self.h, out.ctypes.data_as(ctypes.c_void_p), ctypes.byref(n)))
        return out

    def table(self):
        """FP64 coefficients [ntypes * n_int, M, 6] (the types' tables back to back)."""
        n = ctypes.c_int()
        check(lib.dp_table_download(self.h, None, ctypes.byref(n)))
        out = np.zeros((max(1, self.cfg.get("ntypes", 1)) * n.value, self.cfg["emb"][2], 6))
        check(lib.dp_table_download(self.h, out.ctypes.data_as(ctypes.c_void_p), ctypes.byref(n)))
        return out

    def __del__(self):
        if getattr(self, "h", None):
            lib.dp_model_destroy(self.h)
            self.h = None


class NeighborList:
    """A neighbor list with skin for one configuration; owns its scratch.
    types: int32 device tensor of per-atom types (None: all type 0)."""

    def __init__(self, model, coords, box=None, skin=2.0, types=None):
        self.h = ctypes.c_void_p()
        self.model = model
        self.build(coords, box, skin, types)

    def build(self, coords, box=None, skin=2.0, types=None):
        n = coords.shape[0]
        _f64(coords, (n, 3))
        b, bp = _box(box)
        if types is not None and (types.dtype != torch.int32 or tuple(types.shape) != (n,)):
            raise ValueError("types must be an int32 tensor with one entry per atom")
        self.box, self.skin, self.natoms = b, skin, n
        check(lib.dp_build_nlist(self.model.h, n, _ptr(coords), _ptr(types), bp, skin, ctypes.byref(self.h),
                                 _stream()))
        return self

    def check(self):
        """Raises DPError for what the evaluations since the last build flagged
        (DP_ERR_NONFINITE, DP_ERR_SKIN) or a capacity overflow of the build."""
        check(lib.dp_nlist_check(self.h))
        return self

    def stats(self):
        v = [ctypes.c_int() for _ in range(4)]
        check(lib.dp_nlist_stats(self.h, *[ctypes.byref(x) for x in v]))
        return dict(max_nei=v[0].value, sel_overflow=v[1].value, table_oob=v[2].value, cap_overflow=v[3].value)

    def export(self):
        """The candidate arrays (device tensors): cnt [N], and nei, shift
        (three packed int8), dist (FP32) and rev (int16) [N, cap]."""
        n, c = ctypes.c_int(), ctypes.c_int()
        check(lib.dp_nlist_export(self.h, ctypes.byref(n), ctypes.byref(c), None, None, None, None, None, None))
        N, C = n.value, c.value
        dev = torch.device("cuda", torch.cuda.current_device())
        out = dict(cnt=torch.empty(N, dtype=torch.int32, device=dev),
                   nei=torch.empty(N, C, dtype=torch.int32, device=dev),
                   shift=torch.empty(N, C, dtype=torch.int32, device=dev),
                   dist=torch.empty(N, C, dtype=torch.float32, device=dev),
                   rev=torch.empty(N, C, dtype=torch.int16, device=dev))
        check(lib.dp_nlist_export(self.h, ctypes.byref(n), ctypes.byref(c), _ptr(out["cnt"]), _ptr(out["nei"]),
                                  _ptr(out["shift"]), _ptr(out["dist"]), _ptr(out["rev"]), _stream()))
        return out

    def __del__(self):
        if getattr(self, "h", None):
            lib.dp_nlist_destroy(self.h)
            self.h = None


def compute(model, nlist, coords, mode=COMPRESSED, precision=FP64, forces=True, virial=True,
            atom_energy=False, out=None, noalloc=False):
    """Energy (1), forces (N,3), virial (3,3), per-atom energies (N) as float64 tensors.
    noalloc: run dp_compute_noalloc (the library's static scratch instead of
    the list's; pass `out` tensors to keep torch from allocating as well)."""
    n = coords.shape[0]
    _f64(coords, (n, 3))
    dev = coords.device
    o = out if out is not None else {}
    E = o.get("E") if o.get("E") is not None else torch.empty(1, dtype=torch.float64, device=dev)
    F = (o.get("F") if o.get("F") is not None else torch.empty((n, 3), dtype=torch.float64, device=dev)) \
        if forces else None
    W = (o.get("W") if o.get("W") is not None else torch.empty((3, 3), dtype=torch.float64, device=dev)) \
        if virial else None
    Ea = (o.get("e_atom") if o.get("e_atom") is not None else torch.empty(n, dtype=torch.float64, device=dev)) \
        if atom_energy else None
    _, bp = _box(nlist.box.reshape(3, 3) if nlist.box is not None else None)
    fn = lib.dp_compute_noalloc if noalloc else lib.dp_compute
    check(fn(model.h, nlist.h, n, _ptr(coords), None, bp, mode, precision, _ptr(E), _ptr(F), _ptr(W), _ptr(Ea),
             _stream()))
    res = dict(E=E, F=F, W=W, e_atom=Ea)
    if out is not None:
        out.update({k: v for k, v in res.items() if v is not None})
    return res


def descriptor(model, nlist, coords, mode=COMPRESSED, precision=FP64):
    """Per-atom neighbor count, interval-run count (compressed mode; zeros
    in plain mode), T (N,4,M) and D (N, M<*M) as float64 tensors."""
    n = coords.shape[0]
    M, Ml = model.cfg["emb"][2], model.cfg["m_lt"]
    dev = coords.device
    nn = torch.empty(n, dtype=torch.int32, device=dev)
    ns = torch.zeros(n, dtype=torch.int32, device=dev)
    T = torch.empty((n, 4, M), dtype=torch.float64, device=dev)
    D = torch.empty((n, Ml * M), dtype=torch.float64, device=dev)
    check(lib.dp_descriptor(model.h, nlist.h, n, _ptr(coords), None, mode, precision, _ptr(nn), _ptr(ns), _ptr(T),
                            _ptr(D), _stream()))
    return dict(nnei=nn, nseg=ns, T=T, D=D)


def nve_run(model, nlist, x, v, box, mass, dt, nsteps, rebuild_every=10, skin=2.0, mode=COMPRESSED,
            precision=FP64, thermo=True, types=None):
    """Velocity-Verlet NVE in place on x, v (float64 device tensors).  mass:
    one number per type (a single number for a one-type model); types: int32
    device tensor (None: all type 0).
    Returns the thermo tensor (nsteps+1, 2): potential and kinetic energy."""
    n = x.shape[0]
    _f64(x, (n, 3))
    _f64(v, (n, 3))
    th = torch.empty((nsteps + 1, 2), dtype=torch.float64, device=x.device) if thermo else None
    _, bp = _box(box)
    m = np.ascontiguousarray(np.atleast_1d(np.asarray(mass, dtype=np.float64)))
    if m.size != max(1, model.cfg.get("ntypes", 1)):
        raise ValueError("one mass per type expected")
    check(lib.dp_nve_run(model.h, ctypes.byref(nlist.h), n, _ptr(x), _ptr(v), _ptr(types), bp,
                         m.ctypes.data_as(ctypes.c_void_p), dt, nsteps, rebuild_every, skin, mode, precision,
                         _ptr(th), _stream()))
    nlist.box = None if box is None else np.asarray(box, dtype=np.float64).reshape(9)
    nlist.natoms = n
    return th


def nve_continue(model, nlist, x, v, mass, dt, nsteps, rebuild_every=10, mode=COMPRESSED, precision=FP64,
                 thermo=True):
    """Continues the trajectory of the last nve_run / nve_continue on nlist
    (same x tensor, mode and precision): no build and no first evaluation at
    the start.  Returns the thermo tensor (nsteps+1, 2)."""
    n = x.shape[0]
    _f64(x, (n, 3))
    _f64(v, (n, 3))
    th = torch.empty((nsteps + 1, 2), dtype=torch.float64, device=x.device) if thermo else None
    m = np.ascontiguousarray(np.atleast_1d(np.asarray(mass, dtype=np.float64)))
    if m.size != max(1, model.cfg.get("ntypes", 1)):
        raise ValueError("one mass per type expected")
    check(lib.dp_nve_continue(model.h, nlist.h, n, _ptr(x), _ptr(v), m.ctypes.data_as(ctypes.c_void_p), dt, nsteps,
                              rebuild_every, mode, precision, _ptr(th), _stream()))
    return th
