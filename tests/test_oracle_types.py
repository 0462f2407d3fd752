"""Pins of the oracle's several-type model (the two-type water system).

Readings pinned here (the paper names the water system's two species but
not how they enter the model): the embedding net is chosen by the neighbor's
type, the fitting net by the center's type, and of each neighbor type only
the sel_t nearest neighbors are kept.  Each test below fails for a plausible
mistake in that bookkeeping: nets picked by the wrong atom, parameter blocks
at the wrong offset, truncation over all types at once instead of per type,
a dropped or doubled term in the gradient.
"""
import numpy as np
import pytest

import synth


@pytest.fixture(scope="module")
def w_cfg():
    return synth.water_model_config()


@pytest.fixture(scope="module")
def w_params(w_cfg):
    return synth.model_params(w_cfg)


@pytest.fixture(scope="module")
def small_cell():
    # 8 molecules in a 6.2 A box: the 6 A sphere then spans several images
    x, t, box = synth.water_cell(nmol_edge=2)
    return synth.perturb(x, 0.03, 5), t, box


def _one_type_cfg(w_cfg):
    c = dict(w_cfg)
    c.pop("sel_t")
    c["ntypes"] = 1
    return c


def _block(cfg, params, prefix_set, t):
    """Flat slices of the parameter blocks of type t whose base names are in prefix_set."""
    out, k = [], 0
    for name, shape in synth.param_layout(cfg):
        n = int(np.prod(shape))
        base, tt = name.rsplit("_", 1)
        if base in prefix_set and int(tt) == t:
            out.append(slice(k, k + n))
        k += n
    return out


EMB = {"W0", "b0", "W1", "b1", "W2", "b2"}
FIT = {"V1", "c1", "V2", "c2", "V3", "c3", "w4", "b4"}


def test_param_count_two_types(orc, w_cfg):
    one = orc.param_count(_one_type_cfg(w_cfg))
    assert orc.param_count(w_cfg) == 2 * one
    assert sum(int(np.prod(s)) for _, s in synth.param_layout(w_cfg)) == 2 * one


def test_identical_nets_collapse_to_one_type(orc, w_cfg, w_params, small_cell):
    """Two types whose embedding nets and fitting nets are copies of each
    other, with per-type limits above every count, are the one-type model
    with sel = sum of the limits (same contraction scale)."""
    x, t, box = small_cell
    one = _one_type_cfg(w_cfg)
    p1 = synth.model_params(one, seed=3)
    ne = sum(int(np.prod(s)) for n, s in synth.param_layout(one) if n in EMB)
    emb, fit = p1[:ne], p1[ne:]
    p2 = np.concatenate([emb, emb, fit, fit])
    a = orc.evaluate(w_cfg, p2, x, box, types=t)
    b = orc.evaluate(one, p1, x, box)
    assert a["dropped"] == 0 and b["dropped"] == 0
    assert a["E"] == pytest.approx(b["E"], rel=1e-12)
    np.testing.assert_allclose(a["F"], b["F"], rtol=1e-10, atol=1e-12)
    np.testing.assert_allclose(a["W"], b["W"], rtol=1e-10, atol=1e-12)


def _cluster(center_type, nbr_types, seed):
    rng = np.random.Generator(np.random.PCG64(seed))
    n = len(nbr_types)
    v = rng.standard_normal((n, 3))
    v /= np.linalg.norm(v, axis=1, keepdims=True)
    r = np.linspace(1.1, 4.5, n)
    x = np.vstack([np.zeros(3), v * r[:, None]])
    return x, np.array([center_type] + list(nbr_types), dtype=np.int32)


@pytest.mark.parametrize("center", [0, 1])
def test_embedding_by_neighbor_type_fitting_by_center_type(orc, w_cfg, w_params, center):
    """A center whose neighbors are all of the other type: its energy moves
    with the other type's embedding net and its own fitting net only."""
    other = 1 - center
    x, t = _cluster(center, [other] * 6, seed=7 + center)
    base = orc.evaluate(w_cfg, w_params, x, None, types=t, centers=[0], forces=False)["e_atom"][0]
    rng = np.random.Generator(np.random.PCG64(1))

    def moved(prefixes, ty):
        p = w_params.copy()
        for s in _block(w_cfg, p, prefixes, ty):
            p[s] += 0.05 * rng.standard_normal(s.stop - s.start)
        return orc.evaluate(w_cfg, p, x, None, types=t, centers=[0], forces=False)["e_atom"][0]

    assert moved(EMB, center) == base          # own type's embedding: unused
    assert moved(FIT, other) == base           # other type's fitting net: unused
    assert abs(moved(EMB, other) - base) > 1e-6
    assert abs(moved(FIT, center) - base) > 1e-6


def test_truncation_is_per_neighbor_type(orc, w_cfg, w_params):
    """sel_t = (2, 1) keeps the two nearest type-0 and the nearest type-1
    neighbor; the center's energy equals that of the cluster holding only
    those three neighbors."""
    x = np.array([[0, 0, 0],
                  [1.5, 0, 0], [0, 2.0, 0], [0, 0, 2.5],          # type 0 at 1.5, 2.0, 2.5
                  [-1.2, 0, 0], [0, -1.7, 0], [0, 0, -2.2]],      # type 1 at 1.2, 1.7, 2.2
                 dtype=np.float64)
    t = np.array([0, 0, 0, 0, 1, 1, 1], dtype=np.int32)
    cfg = dict(w_cfg, sel_t=(2, 1), sel=3, desc_scale=1.0 / 138)
    full = orc.evaluate(cfg, w_params, x, None, types=t, centers=[0])
    keep = [0, 1, 2, 4]
    red = orc.evaluate(w_cfg, w_params, x[keep], None, types=t[keep], centers=[0])
    assert full["nnei"][0] == 6 and full["dropped"] == 3
    assert full["e_atom"][0] == pytest.approx(red["e_atom"][0], rel=1e-14)
    # the center's gradient lands on the kept neighbors only
    np.testing.assert_allclose(full["F"][keep], red["F"], rtol=1e-13, atol=1e-15)
    assert np.all(full["F"][[3, 5, 6]] == 0.0)


def test_forces_are_minus_energy_gradient(orc, w_cfg, w_params, small_cell):
    x, t, box = small_cell
    ref = orc.evaluate(w_cfg, w_params, x, box, types=t)
    h = 1e-5
    for i, a in [(0, 0), (1, 2), (2, 1), (9, 0), (13, 2)]:   # O and H atoms
        xp, xm = x.copy(), x.copy()
        xp[i, a] += h
        xm[i, a] -= h
        ep = orc.evaluate(w_cfg, w_params, xp, box, types=t, forces=False)["E"]
        em = orc.evaluate(w_cfg, w_params, xm, box, types=t, forces=False)["E"]
        fd = -(ep - em) / (2 * h)
        assert ref["F"][i, a] == pytest.approx(fd, rel=1e-6, abs=1e-7), (i, a)


def test_virial_is_minus_strain_derivative(orc, w_cfg, w_params, small_cell):
    """W = -dE/d(eps) for the homogeneous strain x -> x (1 + eps), box with it."""
    x, t, box = small_cell
    ref = orc.evaluate(w_cfg, w_params, x, box, types=t)
    h = 1e-6
    for a in range(3):
        S = np.eye(3)
        S[a, a] += h
        ep = orc.evaluate(w_cfg, w_params, x @ S, box @ S, types=t, forces=False)["E"]
        S[a, a] -= 2 * h
        em = orc.evaluate(w_cfg, w_params, x @ S, box @ S, types=t, forces=False)["E"]
        assert ref["W"][a, a] == pytest.approx(-(ep - em) / (2 * h), rel=1e-5, abs=1e-6)


def test_invariances_with_types(orc, w_cfg, w_params):
    x, t, box = synth.water_cell(nmol_edge=2)
    x = synth.perturb(x, 0.05, 9)
    cl = x[:18] - x[:18].mean(0)         # an open cluster of six molecules
    tc = t[:18]
    a = orc.evaluate(w_cfg, w_params, cl, None, types=tc)
    # rotation
    q = np.linalg.qr(np.random.Generator(np.random.PCG64(2)).standard_normal((3, 3)))[0]
    b = orc.evaluate(w_cfg, w_params, cl @ q.T, None, types=tc)
    assert b["E"] == pytest.approx(a["E"], rel=1e-13)
    np.testing.assert_allclose(b["F"], a["F"] @ q.T, atol=1e-13)
    # permutation of the atoms, types carried along
    perm = np.random.Generator(np.random.PCG64(3)).permutation(18)
    c = orc.evaluate(w_cfg, w_params, cl[perm], None, types=tc[perm])
    assert c["E"] == pytest.approx(a["E"], rel=1e-13)
    np.testing.assert_allclose(c["F"], a["F"][perm], atol=1e-13)
    # relabelling the types together with their parameter blocks
    one = _one_type_cfg(w_cfg)
    ne = sum(int(np.prod(s)) for n, s in synth.param_layout(one) if n in EMB)
    nf = orc.param_count(one) - ne
    e0, e1 = w_params[:ne], w_params[ne:2 * ne]
    f0, f1 = w_params[2 * ne:2 * ne + nf], w_params[2 * ne + nf:]
    swapped = np.concatenate([e1, e0, f1, f0])
    cfg_s = dict(w_cfg, sel_t=tuple(reversed(w_cfg["sel_t"])))
    d = orc.evaluate(cfg_s, swapped, cl, None, types=1 - tc)
    assert d["E"] == pytest.approx(a["E"], rel=1e-13)
    # net force and torque vanish on an open cluster
    np.testing.assert_allclose(a["F"].sum(0), 0.0, atol=1e-13)
    np.testing.assert_allclose(np.cross(cl, a["F"]).sum(0), 0.0, atol=1e-12)


def test_tables_per_type_match_their_nets(orc, w_cfg, w_params):
    tab = orc.Table(w_cfg, w_params, 0.7, 0.01, 1.5, 0.1)
    assert tab.coef.shape == (2 * 78, 128, 6)
    for ty in (0, 1):
        # fine intervals (h = 0.01), then a tail interval (h = 0.1, error ~ h^6)
        for s, tg, td in ((0.0, 1e-9, 1e-7), (0.123, 1e-9, 1e-7), (0.55, 1e-9, 1e-7),
                          (0.69, 1e-9, 1e-7), (1.04, 1e-6, 1e-5)):
            G, dG = tab.eval(s, ntype=ty)
            Gn, dGn, _ = orc.embed(w_cfg, w_params, s, ntype=ty)
            np.testing.assert_allclose(G, Gn, atol=tg)
            np.testing.assert_allclose(dG, dGn, atol=td)
    # the two types' tables differ (separate nets)
    assert np.max(np.abs(tab.coef[:78] - tab.coef[78:])) > 1e-3


def test_tabulated_water_energy_close_to_net(orc, w_cfg, w_params, small_cell):
    x, t, box = small_cell
    tab = orc.Table(w_cfg, w_params, 0.7, 0.01, 1.5, 0.1)
    a = orc.evaluate(w_cfg, w_params, x, box, types=t)
    b = orc.evaluate(w_cfg, w_params, x, box, types=t, table=tab)
    assert b["table_oob"] == 0
    n = x.shape[0]
    assert abs(a["E"] - b["E"]) / n < 1e-8
    assert np.max(np.abs(a["F"] - b["F"])) < 1e-6


def test_nve_conserves_energy_two_masses(orc, w_cfg, w_params, small_cell):
    """Velocity Verlet with the O and H masses at 0.5 fs: total energy
    drifts by far less than the kinetic energy moves."""
    x, t, box = small_cell
    m = synth.water_masses(t)
    rng = np.random.Generator(np.random.PCG64(4))
    v = rng.standard_normal(x.shape) * np.sqrt(synth.KB_EV * 330.0 / (m[:, None] * synth.MVV_TO_EV))
    v -= (m[:, None] * v).sum(0) / m.sum()
    _, _, rows = orc.velocity_verlet(w_cfg, w_params, x, v, box, m, 0.5, 20, types=t)
    tot = rows[:, 0] + rows[:, 1]
    ke_swing = np.ptp(rows[:, 1])
    assert ke_swing > 0
    assert np.ptp(tot) < 0.05 * ke_swing, (np.ptp(tot), ke_swing)
