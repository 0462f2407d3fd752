"""Seeded synthetic inputs shared by the oracle tests and the GPU path.

This module holds no arithmetic of the method: it only draws lattices,
displacements, weights, velocities and request streams with numpy's PCG64,
so that both sides of a parity test see the same numbers.

The copper workload follows the paper's physical-systems section: perfect
FCC copper with lattice constant 3.634 A, cut-off 8 A, embedding widths
32/64/128, fitting widths 240/240/240, velocities drawn at 330 K.  The paper
used trained models; none exist here, so weights are seeded random normals
N(0, 1/fan_in) (hidden biases N(0, 1), output bias 0).
"""
import math

import numpy as np

A_CU = 3.634        # FCC lattice constant of copper, A
M_CU = 63.546       # atomic mass of copper, amu

# Seeds (one per workload so that inputs are reproducible one by one).
SEED_WEIGHTS = 0
SEED_CFG = {1: 11, 2: 12, 3: 13, 4: 14}
SEED_SERVING = 15
SEED_VELOCITY = 16


def copper_model_config(sel=192):
    """The copper model: rcut 8, rcut_smth 2, sel, embedding 32-64-128, M<=16,
    fitting 240-240-240, contraction scaled by 1/sel."""
    return dict(rcut=8.0, rcut_smth=2.0, sel=sel, emb=(32, 64, 128), m_lt=16,
                fit=(240, 240, 240), desc_scale=1.0 / sel, switch_kind=0)


def param_layout(cfg):
    """(name, shape) of every block of the flat FP64 parameter vector, in file
    order: one embedding net per neighbor type, then one fitting net per
    center type.  Matrices are row-major [fan_in][fan_out].  With several
    types the names carry the type ("W0_1" is W0 of the net of type 1)."""
    d1, d2, d3 = cfg["emb"]
    f1, f2, f3 = cfg["fit"]
    nD = cfg["m_lt"] * d3
    T = max(1, cfg.get("ntypes", 1))
    emb = [("W0", (1, d1)), ("b0", (d1,)), ("W1", (d1, d2)), ("b1", (d2,)),
           ("W2", (d2, d3)), ("b2", (d3,))]
    fit = [("V1", (nD, f1)), ("c1", (f1,)), ("V2", (f1, f2)), ("c2", (f2,)),
           ("V3", (f2, f3)), ("c3", (f3,)), ("w4", (f3,)), ("b4", (1,))]
    if T == 1:
        return emb + fit
    return ([(f"{n}_{t}", sh) for t in range(T) for n, sh in emb] +
            [(f"{n}_{t}", sh) for t in range(T) for n, sh in fit])


def model_params(cfg, seed=SEED_WEIGHTS):
    """Flat FP64 parameters: weights N(0, 1/fan_in), hidden biases N(0, 1),
    output bias 0."""
    rng = np.random.Generator(np.random.PCG64(seed))
    out = []
    for name, shape in param_layout(cfg):
        base = name.split("_")[0]
        if base == "b4":
            out.append(np.zeros(1))
        elif len(shape) == 2:
            out.append(rng.standard_normal(shape).ravel() / math.sqrt(shape[0]))
        elif base == "w4":
            out.append(rng.standard_normal(shape) / math.sqrt(shape[0]))
        else:
            out.append(rng.standard_normal(shape))
    return np.concatenate(out).astype(np.float64)


def split_params(cfg, flat):
    """Dict of named views into the flat vector (for tests that plant values)."""
    out, k = {}, 0
    for name, shape in param_layout(cfg):
        n = int(np.prod(shape))
        out[name] = flat[k:k + n].reshape(shape)
        k += n
    assert k == flat.shape[0]
    return out


def fcc(n1, n2=None, n3=None, a=A_CU):
    """Perfect FCC lattice of n1 x n2 x n3 cubic cells: (coords[N,3], box[3,3])."""
    n2 = n1 if n2 is None else n2
    n3 = n1 if n3 is None else n3
    basis = np.array([[0, 0, 0], [0, .5, .5], [.5, 0, .5], [.5, .5, 0]])
    g = np.stack(np.meshgrid(np.arange(n1), np.arange(n2), np.arange(n3), indexing="ij"), -1).reshape(-1, 1, 3)
    x = ((g + basis[None]) * a).reshape(-1, 3)
    box = np.diag([n1 * a, n2 * a, n3 * a]).astype(np.float64)
    return np.ascontiguousarray(x, dtype=np.float64), box


def perturb(coords, sigma, seed):
    """Gaussian displacements N(0, sigma^2) per component."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return coords + sigma * rng.standard_normal(coords.shape)


def copper(ncell, sigma, seed):
    x, box = fcc(ncell)
    return perturb(x, sigma, seed), box


# Boltzmann constant in eV/K; 1 amu*A^2/fs^2 in eV.
KB_EV = 8.617333262e-5
MVV_TO_EV = 103.642691


def maxwell_boltzmann(natoms, temperature, mass=M_CU, seed=SEED_VELOCITY):
    """Velocities (A/fs) at the given temperature with zero net momentum."""
    rng = np.random.Generator(np.random.PCG64(seed))
    sd = math.sqrt(KB_EV * temperature / (mass * MVV_TO_EV))
    v = sd * rng.standard_normal((natoms, 3))
    v -= v.mean(axis=0, keepdims=True)
    return v


def serving_request(rng, n_target):
    """One request: a periodic FCC-derived cell with about n_target atoms.

    The most cubic (n1, n2, n3) with 4 n1 n2 n3 >= n_target is built, the
    excess atoms plus a vacancy fraction U[0, 0.05] of n_target are removed at
    random, and
    every atom is displaced by N(0, sigma^2) with sigma ~ U[0.02, 0.15]."""
    best = None
    ncell = math.ceil(n_target / 4)
    for n1 in range(2, 40):
        for n2 in range(n1, 40):
            n3 = max(n2, math.ceil(ncell / (n1 * n2)))
            if 4 * n1 * n2 * n3 < n_target:
                continue
            key = (n3 - n1, 4 * n1 * n2 * n3)
            if best is None or key < best[0]:
                best = (key, (n1, n2, n3))
    n1, n2, n3 = best[1]
    x, box = fcc(n1, n2, n3)
    vac = rng.uniform(0.0, 0.05)
    keep = max(1, int(round(n_target * (1.0 - vac))))
    idx = np.sort(rng.permutation(x.shape[0])[:keep])
    sigma = rng.uniform(0.02, 0.15)
    x = x[idx] + sigma * rng.standard_normal((keep, 3))
    return np.ascontiguousarray(x), box, sigma


def serving_stream(nreq, nmin=32, nmax=20000, seed=SEED_SERVING):
    """nreq requests with atom counts log-uniform in [nmin, nmax]."""
    rng = np.random.Generator(np.random.PCG64(seed))
    sizes = np.exp(rng.uniform(math.log(nmin), math.log(nmax), nreq)).astype(int)
    return [serving_request(rng, int(n)) for n in sizes]


# ------------------------------------------------------------------ water
# The paper's water system: two types (O, H), cut-off 6 A, 0.5 fs steps, the
# configuration made by replicating an equilibrated 192-atom box.  No
# equilibrated box exists here: the stand-in places 64 rigid-geometry
# molecules (O-H 0.9572 A, H-O-H 104.52 deg) in a cubic box at 0.997 g/cm^3,
# oxygens on a jittered 4x4x4 grid, orientations uniformly random with
# rejection of any intermolecular pair closer than 1.45 A, then replicates it.

M_O, M_H = 15.999, 1.008      # amu
R_OH, ANGLE_HOH = 0.9572, 104.52
WATER_DENSITY = 0.997         # g/cm^3
SEED_WATER = 21


def water_model_config(sel_t=(46, 92)):
    """The water model: two types (0 = O, 1 = H), rcut 6, rcut_smth 0.5,
    per-type neighbor limits sel_t (46 O + 92 H = 138, the paper's largest
    neighbor count for water), embedding 32-64-128, fitting 240-240-240,
    contraction scaled by 1/138."""
    sel = int(sum(sel_t))
    return dict(rcut=6.0, rcut_smth=0.5, sel=sel, sel_t=tuple(sel_t), ntypes=2, emb=(32, 64, 128),
                m_lt=16, fit=(240, 240, 240), desc_scale=1.0 / sel, switch_kind=0)


def _water_box_edge(nmol):
    grams = nmol * (M_O + 2 * M_H) * 1.66053906660e-24
    return (grams / WATER_DENSITY * 1e24) ** (1.0 / 3.0)


def water_cell(seed=SEED_WATER, nmol_edge=4, min_dist=1.45):
    """One cell of nmol_edge^3 molecules: (coords[N,3], types[N], box[3,3]),
    atoms ordered O, H, H per molecule."""
    rng = np.random.Generator(np.random.PCG64(seed))
    nmol = nmol_edge ** 3
    L = _water_box_edge(nmol)
    a = L / nmol_edge
    half = math.radians(ANGLE_HOH) / 2.0
    placed = []
    for ix in range(nmol_edge):
        for iy in range(nmol_edge):
            for iz in range(nmol_edge):
                for _ in range(1000):
                    o = (np.array([ix, iy, iz]) + 0.5) * a + 0.25 * rng.standard_normal(3)
                    # random orthonormal frame: the molecule's bisector and plane
                    q = rng.standard_normal(4)
                    q /= np.linalg.norm(q)
                    w, x, y, z = q
                    Rm = np.array([[1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)],
                                   [2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)],
                                   [2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)]])
                    h1 = o + R_OH * Rm @ np.array([math.sin(half), 0.0, math.cos(half)])
                    h2 = o + R_OH * Rm @ np.array([-math.sin(half), 0.0, math.cos(half)])
                    mol = np.stack([o, h1, h2])
                    ok = True
                    for other in placed:
                        dd = mol[:, None, :] - other[None, :, :]
                        dd -= L * np.round(dd / L)
                        if np.min(np.sqrt(np.sum(dd * dd, -1))) < min_dist:
                            ok = False
                            break
                    if ok:
                        placed.append(mol)
                        break
                else:
                    raise RuntimeError("water placement failed")
    x = np.concatenate(placed)
    types = np.tile(np.array([0, 1, 1], dtype=np.int32), nmol)
    return np.ascontiguousarray(x), types, np.diag([L, L, L]).astype(np.float64)


def replicate(x, types, box, n1, n2=None, n3=None):
    """The cell repeated n1 x n2 x n3 times (orthorhombic box)."""
    n2 = n1 if n2 is None else n2
    n3 = n1 if n3 is None else n3
    L = np.diag(box)
    shifts = np.stack(np.meshgrid(np.arange(n1), np.arange(n2), np.arange(n3), indexing="ij"), -1).reshape(-1, 3)
    xr = (x[None, :, :] + (shifts * L)[:, None, :]).reshape(-1, 3)
    tr = np.tile(types, shifts.shape[0])
    return (np.ascontiguousarray(xr), np.ascontiguousarray(tr, dtype=np.int32),
            np.diag(L * np.array([n1, n2, n3])).astype(np.float64))


def water(nrep, sigma=0.0, seed=SEED_WATER):
    """The 192-atom cell replicated nrep^3 times, then every atom displaced
    by N(0, sigma^2) (seed + 1) so that replicas differ."""
    x, t, box = water_cell(seed)
    x, t, box = replicate(x, t, box, nrep)
    if sigma > 0:
        x = perturb(x, sigma, seed + 1)
    return x, t, box


def water_masses(types):
    return np.where(np.asarray(types) == 0, M_O, M_H).astype(np.float64)
