"""GPU path against the FP64 oracle, element by element, through the C-ABI.

Tolerances:
  FP64   E_i and F within 1e-10 of the scale of the oracle's values (the two
         sides differ only in summation order and the table's evaluation
         scheme);
  FP32   |dE|/N <= 1e-5 eV/atom and RMSE_F <= 1e-3 eV/A (the paper's RMSE
         definitions, Sec. 3.2), and, because random weights give small
         forces, RMSE_F <= 1e-4 of the oracle's force RMS;
  BF16   fitting-net GEMMs on BF16 MFMA with hi/lo split operands:
         |dE|/N <= 1e-5 eV/atom, RMSE_F <= 1e-3 eV/A and <= 1e-3 of the force
         RMS, max |dE_i| <= 1e-4 eV.
Integer results (neighbor counts) must match exactly.
"""
import math

import numpy as np
import pytest

import oracle
import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

S_MAX, H, TAIL, H_TAIL = 0.7, 0.01, 1.5, 0.1


@pytest.fixture(scope="module")
def P():
    import paper_2201_01446_amd as P
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return P


@pytest.fixture(scope="module")
def model(P, cu_cfg, cu_params):
    m = P.Model(cu_cfg, cu_params).tabulate(S_MAX, H, TAIL, H_TAIL)
    torch.cuda.synchronize()
    return m


@pytest.fixture(scope="module")
def otab(cu_cfg, cu_params):
    return oracle.Table(cu_cfg, cu_params, S_MAX, H, TAIL, H_TAIL)


def dev(x):
    return torch.tensor(np.ascontiguousarray(x), dtype=torch.float64, device="cuda")


def run(P, model, x, box, precision, mode=0):
    nl = P.NeighborList(model, dev(x), box, skin=2.0)
    out = P.compute(model, nl, dev(x), mode=mode, precision=precision, atom_energy=True)
    torch.cuda.synchronize()
    return {k: (v.cpu().numpy() if v is not None else None) for k, v in out.items()}, nl


def rmse(a, b):
    return float(np.sqrt(np.mean((np.asarray(a) - np.asarray(b)) ** 2)))


def check_against(ref, got, precision, n):
    Fs = max(float(np.sqrt(np.mean(ref["F"] ** 2))), 1e-30)
    dE = abs(float(got["E"][0]) - ref["E"]) / n
    eF = rmse(got["F"], ref["F"])
    eEi = float(np.max(np.abs(got["e_atom"] - ref["e_atom"])))
    eW = float(np.max(np.abs(got["W"] - ref["W"])))
    Ws = max(float(np.max(np.abs(ref["W"]))), 1e-30)
    info = f"prec={precision} dE/N={dE:.3g} maxdEi={eEi:.3g} RMSE_F={eF:.3g} (F_rms {Fs:.3g}) dW={eW:.3g}"
    print(info)
    if precision == 0:
        Es = max(float(np.max(np.abs(ref["e_atom"]))), 1.0)
        assert eEi <= 1e-10 * Es, info
        assert float(np.max(np.abs(got["F"] - ref["F"]))) <= 1e-10 * float(np.max(np.abs(ref["F"]))), info
        assert eW <= 1e-10 * Ws, info
    elif precision == 1:
        assert dE <= 1e-5 and eF <= 1e-3, info
        assert eF <= 1e-4 * Fs, info
        assert eEi <= 1e-5, info
        assert eW <= 1e-4 * Ws, info
    else:
        assert dE <= 1e-5 and eF <= 1e-3, info
        assert eF <= 1e-3 * Fs, info
        assert eEi <= 1e-4, info


# ------------------------------------------------------------------ table

def test_table_matches_oracle(model, otab):
    """Coefficients of the device table (Hermite basis expansion) against the
    oracle's (residual form), compared as contributions a_k h^k."""
    t = model.table()
    assert t.shape == otab.coef.shape
    w = np.where(np.arange(t.shape[0]) < otab.n_fine, H, H_TAIL)[:, None, None]
    scale = w ** np.arange(6)[None, None, :]
    ymax = np.max(np.abs(otab.coef[:, :, 0]))
    np.testing.assert_allclose(t * scale, otab.coef * scale, rtol=0, atol=1e-12 * ymax)


# ------------------------------------------------------- descriptor, counts

@pytest.mark.parametrize("ncell,sigma,seed", [(5, 0.05, 11), (2, 0.1, 3), (3, 0.15, 7)])
def test_descriptor_and_counts(P, model, cu_cfg, cu_params, otab, ncell, sigma, seed):
    x, box = synth.copper(ncell, sigma, seed)
    ref = oracle.evaluate(cu_cfg, cu_params, x, box, table=otab, forces=False, desc=True)
    nl = P.NeighborList(model, dev(x), box)
    for prec, tol in ((0, 1e-12), (1, 2e-6)):
        d = P.descriptor(model, nl, dev(x), precision=prec)
        torch.cuda.synchronize()
        np.testing.assert_array_equal(d["nnei"].cpu().numpy(), ref["nnei"])
        T, D = d["T"].cpu().numpy(), d["D"].cpu().numpy()
        np.testing.assert_allclose(T, ref["T"], rtol=0, atol=tol * np.max(np.abs(ref["T"])))
        np.testing.assert_allclose(D, ref["D"], rtol=0, atol=tol * np.max(np.abs(ref["D"])))


# ------------------------------------------------------- energy and forces

@pytest.mark.parametrize("precision", [0, 1, 2])
def test_cu500_vs_tabulated_oracle(P, model, cu_cfg, cu_params, otab, precision):
    """500-atom copper (5x5x5 cells, sigma 0.05): E_i, F, W."""
    x, box = synth.copper(5, 0.05, synth.SEED_CFG[1])
    ref = oracle.evaluate(cu_cfg, cu_params, x, box, table=otab)
    got, _ = run(P, model, x, box, precision)
    check_against(ref, got, precision, len(x))


def test_cu500_fp64_vs_untabulated_oracle(P, model, cu_cfg, cu_params):
    """Compressed FP64 against the net itself: only the table error remains
    (stride 0.01), far below the FP32 gates."""
    x, box = synth.copper(5, 0.05, synth.SEED_CFG[1])
    ref = oracle.evaluate(cu_cfg, cu_params, x, box)
    got, _ = run(P, model, x, box, 0)
    assert abs(got["E"][0] - ref["E"]) / len(x) < 1e-10
    assert rmse(got["F"], ref["F"]) < 1e-10


@pytest.mark.parametrize("width", [8, 100, 256])
@pytest.mark.parametrize("precision", [0, 1, 2])
def test_fitting_widths(P, width, precision):
    """Fitting nets narrower than the 256-column padding, and one at it: the
    products run over the net's width (partial weight chunks and half K
    stages at 8 and 100), with the padding's zero weights never read."""
    cfg = dict(synth.copper_model_config(), fit=(width, width, width))
    p = synth.model_params(cfg)
    m = P.Model(cfg, p).tabulate(S_MAX, H, TAIL, H_TAIL)
    tab = oracle.Table(cfg, p, S_MAX, H, TAIL, H_TAIL)
    x, box = synth.copper(3, 0.1, 61)
    ref = oracle.evaluate(cfg, p, x, box, table=tab)
    got, _ = run(P, m, x, box, precision)
    check_against(ref, got, precision, len(x))


@pytest.mark.parametrize("ncell", [2, 3])
@pytest.mark.parametrize("precision", [0, 1])
def test_small_periodic_cells(P, model, cu_cfg, cu_params, otab, ncell, precision):
    """Cells smaller than the cut-off sphere: every atom sees many periodic
    images of each other atom and of itself."""
    x, box = synth.copper(ncell, 0.1, 40 + ncell)
    ref = oracle.evaluate(cu_cfg, cu_params, x, box, table=otab)
    got, _ = run(P, model, x, box, precision)
    check_against(ref, got, precision, len(x))


def test_ragged_request_cell(P, model, cu_cfg, cu_params, otab):
    """An uneven serving-style cell (vacancies, odd atom count)."""
    rng = np.random.Generator(np.random.PCG64(5))
    x, box, _ = synth.serving_request(rng, 97)
    ref = oracle.evaluate(cu_cfg, cu_params, x, box, table=otab)
    got, _ = run(P, model, x, box, 0)
    check_against(ref, got, 0, len(x))


def test_open_clusters(P, model, cu_cfg, cu_params, otab):
    """Open boundary: a single atom (no neighbors), a dimer, a small cluster."""
    for x in (np.array([[0.3, 0.2, 0.1]]),
              np.array([[0.0, 0.0, 0.0], [1.7, 1.9, 0.4]]),
              synth.copper(2, 0.1, 9)[0]):
        ref = oracle.evaluate(cu_cfg, cu_params, x, None, table=otab)
        got, _ = run(P, model, x, None, 0)
        assert np.max(np.abs(got["e_atom"] - ref["e_atom"])) <= 1e-12 * max(1, np.max(np.abs(ref["e_atom"])))
        assert np.max(np.abs(got["F"] - ref["F"])) <= 1e-12 + 1e-10 * np.max(np.abs(ref["F"]))


@pytest.mark.parametrize("sel", [150, 179])
def test_sel_overflow_keeps_nearest(P, cu_params, sel):
    """More neighbors than sel: the sel nearest are kept, as in the oracle.
    sel = 150 cuts every atom's list; sel = 179 cuts about half of them, so
    the force gather takes both of its paths (kept pairs only, and every
    candidate within rcut) in one launch."""
    cfg = synth.copper_model_config(sel=sel)
    p = synth.model_params(cfg)
    m = P.Model(cfg, p).tabulate(S_MAX, H, TAIL, H_TAIL)
    tab = oracle.Table(cfg, p, S_MAX, H, TAIL, H_TAIL)
    x, box = synth.copper(3, 0.1, 17)
    ref = oracle.evaluate(cfg, p, x, box, table=tab)
    assert ref["dropped"] > 0
    n_over = int(np.sum(ref["nnei"] > sel))
    if sel == 179:
        assert 0 < n_over < len(x)
    for precision in (0, 1):
        got, nl = run(P, m, x, box, precision)
        check_against(ref, got, precision, len(x))
        st = nl.stats()
        assert st["sel_overflow"] == n_over
        assert st["max_nei"] == int(np.max(ref["nnei"]))


@pytest.mark.parametrize("precision", [0, 1])
def test_sel_cut_inside_self_image_tie(P, precision):
    """32-atom cell (edge 7.268 A, below rcut): every atom has 134 neighbors
    closer than the edge and its six own images exactly at it.  sel = 137
    cuts inside that six-fold tie, so which three images are kept decides
    E_i; both sides keep the first three in the order (r, j, image shift x,
    y, z), i.e. the images (-1,0,0), (0,-1,0), (0,0,-1)."""
    x, box = synth.copper(2, 0.05, 13)
    L = box[0, 0]
    cfg = synth.copper_model_config(sel=137)
    p = synth.model_params(cfg)
    for i in range(len(x)):
        _, img, r, _ = oracle.neighbors(cfg, x, box, i)
        assert int(np.sum(r < L)) == 134 and int(np.sum(r == L)) == 6
        np.testing.assert_array_equal(img[134:137], [[-1, 0, 0], [0, -1, 0], [0, 0, -1]])
    m = P.Model(cfg, p).tabulate(S_MAX, H, TAIL, H_TAIL)
    tab = oracle.Table(cfg, p, S_MAX, H, TAIL, H_TAIL)
    ref = oracle.evaluate(cfg, p, x, box, table=tab)
    assert ref["dropped"] == 3 * len(x) + int(np.sum(ref["nnei"] - 140))
    print(f"self-image tie: n={len(x)} precision={precision}", flush=True)
    got, nl = run(P, m, x, box, precision)
    check_against(ref, got, precision, len(x))
    assert nl.stats()["sel_overflow"] == len(x)


def table_overrun_cases():
    """(name, coordinates, box, table parameters): an open cluster with one
    pair at 0.6 A (s = 1.67, past the default table end 1.5), and a 108-atom
    periodic cell (sigma 0.1) with a table ending at s = 0.4 (r = 2.5 A),
    inside the spread of the nearest-neighbor shell."""
    xc = np.array([[0.0, 0.0, 0.0], [0.6, 0.05, -0.02], [2.3, 0.4, 0.1], [-1.1, 2.2, 0.3], [0.4, -0.3, 2.5]])
    x3, box3 = synth.copper(3, 0.1, 17)
    return [("open_close_pair", xc, None, (S_MAX, H, TAIL, H_TAIL)),
            ("periodic_short_table", x3, box3, (0.3, 0.01, 0.4, 0.05))]


@pytest.mark.parametrize("case", [0, 1])
@pytest.mark.parametrize("precision", [0, 1])
def test_table_overrun_clamp(P, cu_cfg, cu_params, case, precision):
    """s past the table end: s is clamped to the end (G constant, G' = 0)
    and each look-up counted.  E_i, F, W against the oracle's tabulated mode,
    and the overrun count against the oracle's."""
    name, x, box, targs = table_overrun_cases()[case]
    m = P.Model(cu_cfg, cu_params).tabulate(*targs)
    tab = oracle.Table(cu_cfg, cu_params, *targs)
    ref = oracle.evaluate(cu_cfg, cu_params, x, box, table=tab)
    assert ref["table_oob"] > 0
    print(f"table overrun: case={name} n={len(x)} precision={precision} oracle oob={ref['table_oob']}", flush=True)
    nl = P.NeighborList(m, dev(x), box, skin=2.0)
    out = P.compute(m, nl, dev(x), precision=precision, atom_energy=True)
    torch.cuda.synchronize()
    got = {k: (v.cpu().numpy() if v is not None else None) for k, v in out.items()}
    check_against(ref, got, precision, len(x))
    oob = nl.stats()["table_oob"]
    if precision == 0:
        assert oob == ref["table_oob"]
    else:   # FP32 s can round across the table end for a pair within ~1e-7 of it
        assert abs(oob - ref["table_oob"]) <= 2


def test_forces_are_minus_gradient_of_gpu_energy(P, model):
    """Central differences of the GPU's own FP64 energy (h = 1e-4 A)."""
    x, box = synth.copper(2, 0.1, 33)
    got, _ = run(P, model, x, box, 0)
    h = 1e-4
    for i, c in ((0, 0), (5, 1), (17, 2)):
        xp, xm = x.copy(), x.copy()
        xp[i, c] += h
        xm[i, c] -= h
        Ep = run(P, model, xp, box, 0)[0]["E"][0]
        Em = run(P, model, xm, box, 0)[0]["E"][0]
        fd = -(Ep - Em) / (2 * h)
        assert abs(got["F"][i, c] - fd) <= 2e-9 + 1e-5 * abs(fd)


# -------------------------------------------------------------------- NVE

def test_nve_matches_oracle_verlet(P, cu_cfg):
    """Velocity Verlet on the GPU against the oracle's, with the output
    weights scaled so forces are of copper's size; the list is rebuilt every
    5 steps on the GPU and never by the oracle (which searches anew)."""
    p = synth.model_params(cu_cfg)
    synth.split_params(cu_cfg, p)["w4"][:] *= 2000.0
    m = P.Model(cu_cfg, p).tabulate(S_MAX, H, TAIL, H_TAIL)
    tab = oracle.Table(cu_cfg, p, S_MAX, H, TAIL, H_TAIL)
    x0, box = synth.copper(2, 0.05, 3)
    v0 = synth.maxwell_boltzmann(len(x0), 330.0, seed=4)
    xo, vo, rows = oracle.velocity_verlet(cu_cfg, p, x0, v0, box, synth.M_CU, 1.0, 20, table=tab)
    x, v = dev(x0), dev(v0)
    nl = P.NeighborList(m, x, box)
    th = P.nve_run(m, nl, x, v, box, synth.M_CU, 1.0, 20, rebuild_every=5, precision=0)
    torch.cuda.synchronize()
    np.testing.assert_allclose(x.cpu().numpy(), xo, rtol=0, atol=1e-10)
    np.testing.assert_allclose(v.cpu().numpy(), vo, rtol=0, atol=1e-12)
    np.testing.assert_allclose(th.cpu().numpy(), rows, rtol=1e-10, atol=1e-10)


# --------------------------------------------------- full size, sampled

def sampled_reference(cfg, params, tab, x, box, e_idx, f_idx):
    """Oracle E_i at e_idx, and the full force on each atom of f_idx from the
    energies of every atom within rcut of it (and its own)."""
    e = oracle.evaluate(cfg, params, x, box, table=tab, centers=e_idx, forces=False)["e_atom"]
    F = np.zeros((len(f_idx), 3))
    for n, k in enumerate(f_idx):
        j, _, _, _ = oracle.neighbors(cfg, x, box, int(k))
        cen = np.unique(np.concatenate([[k], j])).astype(np.int32)
        F[n] = oracle.evaluate(cfg, params, x, box, table=tab, centers=cen)["F"][k]
    return e, F


@pytest.mark.parametrize("precision", [0, 1])
def test_cu108k_sampled(P, model, cu_cfg, cu_params, otab, precision):
    """108,000-atom copper (30^3 cells): sampled per-atom energies and forces."""
    x, box = synth.copper(30, 0.05, synth.SEED_CFG[2])
    got, nl = run(P, model, x, box, precision)
    rng = np.random.default_rng(2)
    e_idx = rng.choice(len(x), 64, replace=False)
    f_idx = rng.choice(len(x), 8, replace=False)
    e_ref, F_ref = sampled_reference(cu_cfg, cu_params, otab, x, box, e_idx, f_idx)
    dEi = np.max(np.abs(got["e_atom"][e_idx] - e_ref))
    dF = np.max(np.abs(got["F"][f_idx] - F_ref))
    Fs = np.max(np.abs(F_ref))
    print(f"108k prec={precision} max dE_i={dEi:.3g} max dF={dF:.3g} (|F| {Fs:.3g})")
    if precision == 0:
        assert dEi <= 1e-10 and dF <= 1e-10 * Fs
    else:
        assert dEi <= 1e-5 and dF <= 1e-4 * Fs
    assert abs(float(np.sum(got["F"][:, 0]))) < 1e-8 * math.sqrt(len(x))
    st = nl.stats()
    assert st["table_oob"] == 0 and st["cap_overflow"] == 0


@pytest.fixture(scope="module")
def cu1m(cu_cfg, cu_params, otab):
    """1,048,576-atom copper (64^3 cells, sigma 0.08 A) and oracle values at
    4,096 random atoms (E_i) and 512 random atoms (forces), from cut-outs."""
    from sampling import LocalSampler
    x, box = synth.copper(64, 0.08, synth.SEED_CFG[3])
    s = LocalSampler(cu_cfg, cu_params, otab, x, box)
    rng = np.random.default_rng(3)
    e_idx = rng.choice(len(x), 4096, replace=False)
    f_idx = rng.choice(len(x), 512, replace=False)
    e_ref = np.array([s.energy(int(k)) for k in e_idx])
    F_ref = np.array([s.force(int(k)) for k in f_idx])
    return x, box, e_idx, f_idx, e_ref, F_ref


@pytest.mark.parametrize("precision", [2, 1])
def test_cu1m_mixed_sampled(P, model, cu1m, precision):
    """1M atoms in mixed BF16 and in FP32: sampled per-atom energies and
    forces against the FP64 oracle."""
    x, box, e_idx, f_idx, e_ref, F_ref = cu1m
    got, nl = run(P, model, x, box, precision)
    dEi = np.max(np.abs(got["e_atom"][e_idx] - e_ref))
    eF = np.sqrt(np.mean((got["F"][f_idx] - F_ref) ** 2))
    Fs = np.sqrt(np.mean(F_ref ** 2))
    print(f"1M prec={precision} max dE_i={dEi:.3g} RMSE_F={eF:.3g} (F_rms {Fs:.3g})")
    assert dEi <= (1e-4 if precision == 2 else 1e-5)
    assert eF <= 1e-3 and eF <= (1e-3 if precision == 2 else 1e-4) * Fs
    st = nl.stats()
    assert st["table_oob"] == 0 and st["cap_overflow"] == 0


@pytest.mark.parametrize("precision", [0, 1, 2])
def test_forces_deterministic(P, model, precision):
    """Forces are gathered per atom in a fixed order (no atomics): two runs
    give bitwise-identical results in every precision."""
    x, box = synth.copper(6, 0.1, 71)
    a, _ = run(P, model, x, box, precision)
    b, _ = run(P, model, x, box, precision)
    np.testing.assert_array_equal(a["F"], b["F"])
    np.testing.assert_array_equal(a["W"], b["W"])
    assert a["E"][0] == b["E"][0]


@pytest.mark.parametrize("move", ["small", "large"])
@pytest.mark.parametrize("precision", [0, 1])
def test_moved_atoms_against_list_of_build(P, model, otab, cu_cfg, cu_params, precision, move):
    """A list built at x, evaluated at moved positions.  Small moves (largest
    0.1-0.2 A, under a quarter of the 2 A skin per pair) take the early end of
    the candidate scan; the large case moves atom a toward an atom b that
    was 8.55-8.7 A away at build (past rcut + skin/4) to 7.9 A, inside rcut,
    so the scan must reach past the prefix to find the pair."""
    x, box = synth.copper(6, 0.05, 11)
    n, Lb = len(x), box[0, 0]
    xm = x + np.random.Generator(np.random.PCG64(5)).normal(0.0, 0.03, x.shape)
    if move == "large":
        xm = x.copy()
        d = x[None, :64, :] - x[:, None, :]
        d -= Lb * np.round(d / Lb)
        r = np.linalg.norm(d, axis=2)
        ib, ia = np.argwhere((r > 8.55) & (r < 8.7))[0]
        u = x[ib] - x[ia]
        u -= Lb * np.round(u / Lb)
        xm[ia] += (np.linalg.norm(u) - 7.9) * u / np.linalg.norm(u)   # 0.65-0.8 A, to 7.9 A from b
        v = xm[ib] - xm[ia]
        assert np.linalg.norm(v - Lb * np.round(v / Lb)) < cu_cfg["rcut"]
    print(f"moved atoms: n={n} precision={precision} move={move}", flush=True)
    nl = P.NeighborList(model, dev(x), box, skin=2.0)
    xd = dev(xm)
    out = P.compute(model, nl, xd, precision=precision, atom_energy=True)
    nn = P.descriptor(model, nl, xd, precision=precision)["nnei"]
    torch.cuda.synchronize()
    got = {k: v.cpu().numpy() for k, v in out.items()}
    ref = oracle.evaluate(cu_cfg, cu_params, xm, box, table=otab)
    np.testing.assert_array_equal(nn.cpu().numpy(), ref["nnei"])
    check_against(ref, got, precision, n)
