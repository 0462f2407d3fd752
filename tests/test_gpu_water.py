"""The two-type (water-like O/H) system on the GPU against the FP64 oracle.

The water model: rcut 6 A, per-type neighbor limits 46 O + 92 H, one
embedding table per neighbor type, one fitting net per center type; the
coordinates are the synthetic stand-in for the paper's replicated 192-atom
box (see synth.water).  Tolerances as for copper (test_gpu_parity): FP64
within 1e-10 of the oracle's scale; FP32 |dE|/N <= 1e-5 eV/atom, RMSE_F
<= 1e-3 eV/A and <= 1e-4 of the force RMS; mixed BF16 |dE|/N <= 1e-5,
RMSE_F <= 1e-3 of the force RMS.  Neighbor counts must match exactly.
"""
import numpy as np
import pytest

import oracle
import synth
from sampling import LocalSampler

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TAB = (0.7, 0.01, 1.5, 0.1)


@pytest.fixture(scope="module")
def P():
    import paper_2201_01446_amd as P
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return P


@pytest.fixture(scope="module")
def w_cfg():
    return synth.water_model_config()


@pytest.fixture(scope="module")
def w_params(w_cfg):
    return synth.model_params(w_cfg)


@pytest.fixture(scope="module")
def model(P, w_cfg, w_params):
    m = P.Model(w_cfg, w_params).tabulate(*TAB)
    torch.cuda.synchronize()
    return m


@pytest.fixture(scope="module")
def otab(w_cfg, w_params):
    return oracle.Table(w_cfg, w_params, *TAB)


def dev(a, dtype=torch.float64):
    return torch.tensor(np.ascontiguousarray(a), dtype=dtype, device="cuda")


def run(P, model, x, t, box, precision, mode=0):
    nl = P.NeighborList(model, dev(x), box, skin=2.0, types=dev(t, torch.int32))
    out = P.compute(model, nl, dev(x), mode=mode, precision=precision, atom_energy=True)
    torch.cuda.synchronize()
    return {k: (v.cpu().numpy() if v is not None else None) for k, v in out.items()}, nl


def shuffled(x, t, seed):
    perm = np.random.Generator(np.random.PCG64(seed)).permutation(len(x))
    return x[perm], t[perm]


def check(ref, got, precision, n):
    Fs = max(float(np.sqrt(np.mean(ref["F"] ** 2))), 1e-30)
    dE = abs(float(got["E"][0]) - ref["E"]) / n
    eF = float(np.sqrt(np.mean((got["F"] - ref["F"]) ** 2)))
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
        assert dE <= 1e-5 and eF <= 1e-3 and eF <= 1e-4 * Fs, info
        assert eEi <= 1e-5, info
    else:
        assert dE <= 1e-5 and eF <= 1e-3 * Fs, info
        assert eEi <= 1e-4, info


@pytest.mark.parametrize("order", ["molecules", "shuffled"])
@pytest.mark.parametrize("precision", [0, 1, 2])
def test_water_parity(P, model, otab, w_cfg, w_params, precision, order):
    """1536 atoms (the 192-atom cell 2 x 2 x 2), several tiles of each type's
    rows and a ragged tail; 'shuffled' interleaves the types at random."""
    x, t, box = synth.water(2, sigma=0.05)
    if order == "shuffled":
        x, t = shuffled(x, t, 3)
    print(f"water parity: n={len(x)} precision={precision} order={order}", flush=True)
    got, nl = run(P, model, x, t, box, precision)
    ref = oracle.evaluate(w_cfg, w_params, x, box, table=otab, types=t)
    check(ref, got, precision, len(x))
    st = nl.stats()
    assert st["sel_overflow"] == 0 and st["table_oob"] == 0
    assert st["max_nei"] == int(ref["nnei"].max())


def test_water_descriptor_fp64(P, model, otab, w_cfg, w_params):
    x, t, box = synth.water(1, sigma=0.05)
    x, t = shuffled(x, t, 4)
    nl = P.NeighborList(model, dev(x), box, skin=2.0, types=dev(t, torch.int32))
    d = P.descriptor(model, nl, dev(x), precision=0)
    ref = oracle.evaluate(w_cfg, w_params, x, box, table=otab, types=t, forces=False, desc=True)
    np.testing.assert_array_equal(d["nnei"].cpu().numpy(), ref["nnei"])
    T, D = d["T"].cpu().numpy(), d["D"].cpu().numpy()
    assert np.max(np.abs(T - ref["T"])) <= 1e-12 * np.max(np.abs(ref["T"]))
    assert np.max(np.abs(D - ref["D"])) <= 1e-12 * np.max(np.abs(ref["D"]))
    # interval runs never mix types: at least one per type present
    assert int(d["nseg"].min()) >= 2


@pytest.mark.parametrize("mode", [3, 4])
def test_water_per_neighbor_modes(P, model, otab, w_cfg, w_params, mode):
    x, t, box = synth.water(1, sigma=0.05)
    got, _ = run(P, model, x, t, box, 0, mode=mode)
    ref = oracle.evaluate(w_cfg, w_params, x, box, table=otab, types=t)
    check(ref, got, 0, len(x))


@pytest.mark.parametrize("precision", [0, 1])
def test_water_per_type_truncation(P, w_cfg, w_params, precision):
    """Limits below the counts (20 O, 40 H): of each type the nearest are kept."""
    cfg = dict(w_cfg, sel_t=(20, 40), sel=60)
    m = P.Model(cfg, w_params).tabulate(*TAB)
    tab = oracle.Table(cfg, w_params, *TAB)
    x, t, box = synth.water(1, sigma=0.05)
    x, t = shuffled(x, t, 5)
    got, nl = run(P, m, x, t, box, precision)
    ref = oracle.evaluate(cfg, w_params, x, box, table=tab, types=t)
    assert ref["dropped"] > 0
    check(ref, got, precision, len(x))
    assert nl.stats()["sel_overflow"] == len(x)


def test_water_nve_matches_oracle(P, model, otab, w_cfg, w_params):
    """Ten velocity-Verlet steps of 0.5 fs with the O and H masses."""
    x, t, box = synth.water(1, sigma=0.02)
    m = synth.water_masses(t)
    rng = np.random.Generator(np.random.PCG64(8))
    v = rng.standard_normal(x.shape) * np.sqrt(synth.KB_EV * 330.0 / (m[:, None] * synth.MVV_TO_EV))
    xd, vd = dev(x), dev(v)
    nl = P.NeighborList(model, xd, box, skin=2.0, types=dev(t, torch.int32))
    th = P.nve_run(model, nl, xd, vd, box, [synth.M_O, synth.M_H], 0.5, 10, rebuild_every=5, precision=0,
                   types=dev(t, torch.int32)).cpu().numpy()
    xo, vo, rows = oracle.velocity_verlet(w_cfg, w_params, x, v, box, m, 0.5, 10, table=otab, types=t)
    np.testing.assert_allclose(xd.cpu().numpy(), xo, rtol=0, atol=1e-10)
    np.testing.assert_allclose(vd.cpu().numpy(), vo, rtol=0, atol=1e-12)
    np.testing.assert_allclose(th, rows, rtol=1e-10, atol=1e-12)


def test_water_large_sampled(P, model, otab, w_cfg, w_params):
    """98,304 atoms (8 x 8 x 8 cells, shuffled), FP32 and mixed BF16 in the
    launch configuration the benchmark uses; the oracle on cut-outs at 192
    sampled energies and 48 sampled forces."""
    x, t, box = synth.water(8, sigma=0.05)
    x, t = shuffled(x, t, 6)
    n = len(x)
    rng = np.random.Generator(np.random.PCG64(7))
    e_idx = rng.choice(n, 192, replace=False)
    f_idx = rng.choice(n, 48, replace=False)
    s = LocalSampler(w_cfg, w_params, otab, x, box, types=t)
    e_ref = np.array([s.energy(k) for k in e_idx])
    f_ref = np.array([s.force(k) for k in f_idx])
    for precision in (1, 2):
        print(f"water large sampled: n={n} precision={precision}", flush=True)
        got, nl = run(P, model, x, t, box, precision)
        dE = np.abs(got["e_atom"][e_idx] - e_ref)
        dF = got["F"][f_idx] - f_ref
        Fs = float(np.sqrt(np.mean(f_ref ** 2)))
        eF = float(np.sqrt(np.mean(dF ** 2)))
        print(f"  max dE_i {dE.max():.3g}  RMSE_F {eF:.3g} (F_rms {Fs:.3g})")
        assert dE.max() <= (1e-5 if precision == 1 else 1e-4)
        assert eF <= (1e-4 if precision == 1 else 1e-3) * Fs
        assert nl.stats()["sel_overflow"] == 0


def test_water_errors(P, model, w_cfg, w_params):
    x, t, box = synth.water(1)
    xd = dev(x)
    bad = t.copy()
    bad[5] = 2
    with pytest.raises(P.DPError, match="DP_ERR_ARG"):
        P.NeighborList(model, xd, box, skin=2.0, types=dev(bad, torch.int32))
    nl = P.NeighborList(model, xd, box, skin=2.0, types=dev(t, torch.int32))
    for mode in (1, 2):
        with pytest.raises(P.DPError, match="DP_ERR_UNSUPPORTED"):
            P.compute(model, nl, xd, mode=mode, precision=0)
    from paper_2201_01446_amd import serve
    with pytest.raises(P.DPError, match="DP_ERR_UNSUPPORTED"):
        serve.Batch(model, 1000, 4, 2.0)
    with pytest.raises(P.DPError, match="DP_ERR_ARG"):
        P.Model(dict(w_cfg, sel=100), w_params)          # sel != sum of sel_t
    with pytest.raises(ValueError):
        P.nve_run(model, nl, xd, dev(np.zeros_like(x)), box, synth.M_O, 0.5, 1, types=dev(t, torch.int32))


@pytest.mark.parametrize("precision", [0, 1])
def test_water_autograd_matches_compute(P, model, otab, w_cfg, w_params, precision):
    """The autograd function on the two-type system: E and dE/dx equal the
    one-call step's E and -F (the same kernels, split at the fitting net),
    and, in FP64, the oracle's."""
    from paper_2201_01446_amd.autograd import DPEnergy
    x, t, box = synth.water(1, sigma=0.05)
    x, t = shuffled(x, t, 9)
    xd = dev(x).requires_grad_(True)
    nl = P.NeighborList(model, xd.detach(), box, skin=2.0, types=dev(t, torch.int32))
    E = DPEnergy.apply(xd, model, nl, precision, P.COMPRESSED)
    (g,) = torch.autograd.grad(E.sum(), xd)
    one = P.compute(model, nl, xd.detach(), precision=precision)
    torch.cuda.synchronize()
    assert float(E.item()) == float(one["E"].item())
    np.testing.assert_array_equal(g.cpu().numpy(), -one["F"].cpu().numpy())
    if precision == 0:
        ref = oracle.evaluate(w_cfg, w_params, x, box, table=otab, types=t)
        assert abs(float(E.item()) - ref["E"]) <= 1e-10 * abs(ref["E"])
        np.testing.assert_allclose(-g.cpu().numpy(), ref["F"], rtol=0, atol=1e-10 * np.max(np.abs(ref["F"])))


@pytest.mark.parametrize("move", ["small", "large"])
@pytest.mark.parametrize("precision", [0, 1])
def test_water_moved_atoms_against_list_of_build(P, model, otab, w_cfg, w_params, precision, move):
    """A two-type list built at x and evaluated at moved positions: small
    moves keep every atom within skin/8 (each type run scanned up to its
    prefix within rcut + skin/4 = 6.5 A); the large case moves atom a from
    6.55-6.7 A of atom b to 5.9 A, inside rcut, so the full runs are read."""
    x, t, box = synth.water(2, sigma=0.05)
    n, Lb = len(x), box[0, 0]
    xm = x + np.random.Generator(np.random.PCG64(12)).normal(0.0, 0.03, x.shape)
    if move == "large":
        xm = x.copy()
        d = x[None, :64, :] - x[:, None, :]
        d -= Lb * np.round(d / Lb)
        r = np.linalg.norm(d, axis=2)
        ib, ia = np.argwhere((r > 6.55) & (r < 6.7))[0]
        u = x[ib] - x[ia]
        u -= Lb * np.round(u / Lb)
        xm[ia] += (np.linalg.norm(u) - 5.9) * u / np.linalg.norm(u)
    print(f"water moved atoms: n={n} precision={precision} move={move}", flush=True)
    nl = P.NeighborList(model, dev(x), box, skin=2.0, types=dev(t, torch.int32))
    xd = dev(xm)
    out = P.compute(model, nl, xd, precision=precision, atom_energy=True)
    nn = P.descriptor(model, nl, xd, precision=precision)["nnei"]
    torch.cuda.synchronize()
    got = {k: v.cpu().numpy() for k, v in out.items()}
    ref = oracle.evaluate(w_cfg, w_params, xm, box, table=otab, types=t)
    np.testing.assert_array_equal(nn.cpu().numpy(), ref["nnei"])
    check(ref, got, precision, n)
