"""FP64 CPU oracle for the Deep Potential force step (test infrastructure).

Only the tests, the smoke check and the benchmark's CPU-baseline leg use this
package.  The GPU library never imports it.  The arithmetic lives in
``dp_oracle.c`` (plain C, FP64, OpenMP over atoms); this module only marshals
numpy arrays through ctypes.

Parity pins for each function are in ``tests/test_oracle_*.py``.
"""
import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "dp_oracle.c")
_LIB = os.path.join(_HERE, "liborc.so")


def build(force=True):
    """Compile ``liborc.so`` with gcc (plain -O2, no fast-math)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        cmd = ["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-Wall", "-o", _LIB + ".tmp", _SRC, "-lm"]
        subprocess.check_call(cmd)
        os.replace(_LIB + ".tmp", _LIB)
    return _LIB


class Config(ctypes.Structure):
    _fields_ = [
        ("rcut", ctypes.c_double),
        ("rcut_smth", ctypes.c_double),
        ("sel", ctypes.c_int),
        ("d1", ctypes.c_int),
        ("d2", ctypes.c_int),
        ("d3", ctypes.c_int),
        ("m_lt", ctypes.c_int),
        ("f1", ctypes.c_int),
        ("f2", ctypes.c_int),
        ("f3", ctypes.c_int),
        ("desc_scale", ctypes.c_double),
        ("switch_kind", ctypes.c_int),
        ("tanh_table", ctypes.c_int),
        ("ntypes", ctypes.c_int),
        ("sel_t", ctypes.c_int * 4),
    ]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=False)
        L = ctypes.CDLL(_LIB)
        P = ctypes.POINTER
        d, i, l = ctypes.c_double, ctypes.c_int, ctypes.c_long
        pd, pi, pl = P(d), P(i), P(l)
        pc = P(Config)
        L.orc_param_count.argtypes = [pc]
        L.orc_param_count.restype = l
        L.orc_switch.argtypes = [pc, d, pd, pd]
        L.orc_tanh_table.argtypes = [d]
        L.orc_tanh_table.restype = d
        L.orc_embed.argtypes = [pc, pd, i, d, pd, pd, pd]
        L.orc_hermite.argtypes = [d, d, d, d, d, d, d, pd]
        L.orc_table_intervals.argtypes = [d, d, d, d]
        L.orc_table_intervals.restype = i
        L.orc_tabulate.argtypes = [pc, pd, i, d, d, d, d, pd]
        L.orc_tabulate.restype = i
        L.orc_table_eval.argtypes = [pc, i, i, d, d, d, d, pd, d, pd, pd]
        L.orc_neighbors.argtypes = [pc, i, pd, pd, i, i, pi, pi, pd]
        L.orc_neighbors.restype = i
        L.orc_evaluate.argtypes = [pc, pd, i, pd, pd, pi, i, pi, i, i, d, d, d, d, pd,
                                   pd, pd, pd, pi, pd, pd, pl]
        L.orc_evaluate.restype = l
        L.orc_num_threads.restype = i
        _lib = L
    return _lib


def _dp(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double)) if a is not None else None


def _ip(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_int)) if a is not None else None


def make_config(cfg):
    """cfg: mapping with rcut, rcut_smth, sel, emb (3), m_lt, fit (3), desc_scale, switch_kind and,
    optionally, tanh_table (1: the fitting net's tanh from the second-order table) and, for
    several atom types, ntypes and sel_t (neighbors kept per neighbor type; sel = their sum)."""
    c = Config()
    c.rcut = cfg["rcut"]
    c.rcut_smth = cfg["rcut_smth"]
    c.sel = cfg["sel"]
    c.d1, c.d2, c.d3 = cfg["emb"]
    c.m_lt = cfg["m_lt"]
    c.f1, c.f2, c.f3 = cfg["fit"]
    c.desc_scale = cfg["desc_scale"]
    c.switch_kind = cfg.get("switch_kind", 0)
    c.tanh_table = cfg.get("tanh_table", 0)
    c.ntypes = cfg.get("ntypes", 1)
    for t, v in enumerate(cfg.get("sel_t", ())):
        c.sel_t[t] = v
    return c


def ntypes(cfg):
    return max(1, cfg.get("ntypes", 1))


def param_count(cfg):
    return int(lib().orc_param_count(ctypes.byref(make_config(cfg))))


def switch(cfg, r):
    """Gate w(r) and dw/dr (Eq. 1)."""
    c = make_config(cfg)
    w, dw = ctypes.c_double(), ctypes.c_double()
    lib().orc_switch(ctypes.byref(c), float(r), ctypes.byref(w), ctypes.byref(dw))
    return w.value, dw.value


def embed(cfg, params, s, ntype=0):
    """G(s), G'(s), G''(s) of the embedding net of neighbor type ntype (Eqs. 3-5)."""
    c = make_config(cfg)
    p = np.ascontiguousarray(params, dtype=np.float64)
    M = cfg["emb"][2]
    G, dG, ddG = (np.zeros(M) for _ in range(3))
    lib().orc_embed(ctypes.byref(c), _dp(p), int(ntype), float(s), _dp(G), _dp(dG), _dp(ddG))
    return G, dG, ddG


def hermite(y0, d0, dd0, y1, d1, dd1, h):
    """Quintic coefficients in t matching value/1st/2nd derivative at t=0 and t=h."""
    a = np.zeros(6)
    lib().orc_hermite(y0, d0, dd0, y1, d1, dd1, h, _dp(a))
    return a


class Table:
    """Tabulated embedding nets (Sec. 3.2), one per neighbor type, back to
    back: coef[type * n + theta, eta, xi] (n intervals per type)."""

    def __init__(self, cfg, params, s_max, h, tail_max, h_tail):
        c = make_config(cfg)
        n = lib().orc_table_intervals(s_max, h, tail_max, h_tail)
        M = cfg["emb"][2]
        T = ntypes(cfg)
        self.coef = np.zeros((T * n, M, 6))
        p = np.ascontiguousarray(params, dtype=np.float64)
        for t in range(T):
            part = np.zeros((n, M, 6))
            lib().orc_tabulate(ctypes.byref(c), _dp(p), t, s_max, h, tail_max, h_tail, _dp(part))
            self.coef[t * n:(t + 1) * n] = part
        self.n_int = n
        self.n_fine = int(round(s_max / h))
        self.n_tail = n - self.n_fine
        self.h, self.s_max, self.h_tail, self.tail_max = h, s_max, h_tail, tail_max
        self.cfg = cfg

    def eval(self, s, ntype=0):
        c = make_config(self.cfg)
        M = self.cfg["emb"][2]
        G, dG = np.zeros(M), np.zeros(M)
        part = np.ascontiguousarray(self.coef[ntype * self.n_int:(ntype + 1) * self.n_int])
        lib().orc_table_eval(ctypes.byref(c), self.n_fine, self.n_tail, self.h, self.s_max,
                             self.h_tail, self.tail_max, _dp(part), float(s), _dp(G), _dp(dG))
        return G, dG


def neighbors(cfg, coords, box, i, cap=4096):
    """Sorted neighbor set of atom i: (j, image shift, r), all within rcut."""
    c = make_config(cfg)
    x = np.ascontiguousarray(coords, dtype=np.float64).reshape(-1, 3)
    b = None if box is None else np.ascontiguousarray(box, dtype=np.float64).reshape(9)
    j = np.zeros(cap, dtype=np.int32)
    img = np.zeros((cap, 3), dtype=np.int32)
    r = np.zeros(cap)
    n = lib().orc_neighbors(ctypes.byref(c), x.shape[0], _dp(x), _dp(b), int(i), cap, _ip(j), _ip(img), _dp(r))
    m = min(n, cap)
    return j[:m], img[:m], r[:m], n


def evaluate(cfg, params, coords, box, table=None, centers=None, forces=True, desc=False, types=None):
    """Energy, per-atom energy, forces and virial.

    centers: optional index array; then e_atom is per listed center and the
    force holds only those centers' contributions.  types: per-atom type
    (None: all type 0).
    Returns a dict with E, e_atom, F, W (3x3), nnei, dropped, table_oob and,
    when desc is set, T (n,4,M) and D (n, M<*M).
    """
    c = make_config(cfg)
    x = np.ascontiguousarray(coords, dtype=np.float64).reshape(-1, 3)
    N = x.shape[0]
    b = None if box is None else np.ascontiguousarray(box, dtype=np.float64).reshape(9)
    cen = None if centers is None else np.ascontiguousarray(centers, dtype=np.int32)
    typ = None if types is None else np.ascontiguousarray(types, dtype=np.int32)
    if typ is not None and (typ.shape != (N,) or typ.min() < 0 or typ.max() >= ntypes(cfg)):
        raise ValueError("types must hold one type in [0, ntypes) per atom")
    nc = N if cen is None else cen.shape[0]
    M, Ml = cfg["emb"][2], cfg["m_lt"]
    p = np.ascontiguousarray(params, dtype=np.float64)
    e_atom = np.zeros(nc)
    F = np.zeros((N, 3)) if forces else None
    W = np.zeros(9) if forces else None
    nnei = np.zeros(nc, dtype=np.int32)
    T = np.zeros((nc, 4, M)) if desc else None
    D = np.zeros((nc, Ml * M)) if desc else None
    oob = ctypes.c_long(0)
    if table is None:
        tab = (0, 0, 1.0, 0.0, 1.0, 0.0, None)
    else:
        tab = (table.n_fine, table.n_tail, table.h, table.s_max, table.h_tail, table.tail_max, _dp(table.coef))
    dropped = lib().orc_evaluate(ctypes.byref(c), _dp(p), N, _dp(x), _dp(b), _ip(typ), nc, _ip(cen), *tab,
                                 _dp(e_atom), _dp(F), _dp(W), _ip(nnei), _dp(T), _dp(D), ctypes.byref(oob))
    if dropped < 0:
        raise MemoryError("oracle allocation failed")
    out = dict(E=float(np.sum(e_atom)) if cen is None else None, e_atom=e_atom, nnei=nnei,
               dropped=int(dropped), table_oob=int(oob.value))
    if forces:
        out["F"] = F
        out["W"] = W.reshape(3, 3)
    if desc:
        out["T"], out["D"] = T, D
    return out


def num_threads():
    return int(lib().orc_num_threads())


# Units: eV, A, fs, amu.  1 eV/(A amu) = 9.64853321e-3 A/fs^2;
# 1 amu A^2/fs^2 = 103.642691 eV.
ACC_UNIT = 9.64853321e-3
KE_UNIT = 103.642691


def velocity_verlet(cfg, params, x, v, box, mass, dt, nsteps, table=None, types=None):
    """Plain velocity-Verlet NVE (the MD protocol of the paper's
    physical-systems section): half kick, drift, force, half kick.  mass is
    one number or one per atom.  Returns (x, v, rows) with rows[t] = (PE, KE)
    after step t (t = 0 is the start)."""
    x = np.array(x, dtype=np.float64)
    v = np.array(v, dtype=np.float64)
    mass = np.asarray(mass, dtype=np.float64)
    if mass.ndim == 1:
        mass = mass[:, None]
    out = evaluate(cfg, params, x, box, table=table, types=types)
    F = out["F"]
    rows = [(out["E"], 0.5 * KE_UNIT * float(np.sum(mass * v * v)))]
    for _ in range(nsteps):
        v = v + 0.5 * dt * ACC_UNIT * F / mass
        x = x + dt * v
        out = evaluate(cfg, params, x, box, table=table, types=types)
        F = out["F"]
        v = v + 0.5 * dt * ACC_UNIT * F / mass
        rows.append((out["E"], 0.5 * KE_UNIT * float(np.sum(mass * v * v))))
    return x, v, np.array(rows)


def tanh_table(x):
    """The oracle's tabulated tanh (second order, [0, 8], odd, 1 beyond 8)."""
    f = lib().orc_tanh_table
    return np.array([f(float(v)) for v in np.ravel(x)]).reshape(np.shape(x))
