"""Pins of the FP64 oracle against facts that do not come from the oracle.

Each test names what fixes the expected value: a closed form, a textbook
function or library routine in a special case, an exact invariance of the
model (Sec. 2.1: translational, rotational and permutational symmetry), the
definition F = -grad E (central finite differences), crystallography (FCC
neighbor shells), or brute force on tiny inputs.
"""
import itertools
import json
import math
import os

import numpy as np
import pytest

import synth

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def small_cfg(**kw):
    """A narrow model (same structure) so that brute-force tests stay fast."""
    cfg = dict(rcut=6.0, rcut_smth=1.0, sel=64, emb=(4, 8, 16), m_lt=4, fit=(12, 12, 12),
               desc_scale=1.0 / 64, switch_kind=0)
    cfg.update(kw)
    return cfg


def random_rotation(rng):
    q, r = np.linalg.qr(rng.standard_normal((3, 3)))
    q = q * np.sign(np.diag(r))
    if np.linalg.det(q) < 0:
        q[:, 0] = -q[:, 0]
    return q


# ------------------------------------------------------------------ gate

@pytest.mark.parametrize("kind", [0, 1])
def test_gate_endpoints_and_derivative(orc, kind):
    cfg = small_cfg(switch_kind=kind)
    rs, rc = cfg["rcut_smth"], cfg["rcut"]
    assert orc.switch(cfg, rs - 1e-3) == (1.0, 0.0)
    assert orc.switch(cfg, rs)[0] == pytest.approx(1.0, abs=1e-15)
    assert orc.switch(cfg, rc) == (0.0, 0.0)
    assert orc.switch(cfg, rc - 1e-9)[0] < 1e-12
    # value at the midpoint: 1/2 for both gates (symmetric about u = 1/2)
    assert orc.switch(cfg, 0.5 * (rs + rc))[0] == pytest.approx(0.5, abs=1e-15)
    # derivative against central differences
    h = 1e-6
    for r in np.linspace(rs + 0.01, rc - 0.01, 17):
        fd = (orc.switch(cfg, r + h)[0] - orc.switch(cfg, r - h)[0]) / (2 * h)
        assert orc.switch(cfg, r)[1] == pytest.approx(fd, abs=1e-8)


def test_quintic_gate_is_c2(orc):
    """The quintic gate has zero first and second derivative at both ends."""
    cfg = small_cfg()
    rs, rc = cfg["rcut_smth"], cfg["rcut"]
    h = 1e-4
    for r0 in (rs, rc):
        d1 = orc.switch(cfg, r0)[1]
        assert abs(d1) < 1e-12
        # second derivative from the first by one-sided differences inside
        side = 1 if r0 == rs else -1
        d2 = (orc.switch(cfg, r0 + side * h)[1] - d1) / (side * h)
        assert abs(d2) < 1e-2  # O(h) for a function with w'' = 0 at the end


def test_quintic_gate_closed_form(orc):
    """w(u) = 1 - 10u^3 + 15u^4 - 6u^5 at a few u (reference from numpy's
    polynomial evaluation of the smoothstep polynomial)."""
    cfg = small_cfg()
    rs, rc = cfg["rcut_smth"], cfg["rcut"]
    poly = np.polynomial.Polynomial([1, 0, 0, -10, 15, -6])
    for u in (0.1, 0.3, 0.77):
        assert orc.switch(cfg, rs + u * (rc - rs))[0] == pytest.approx(poly(u), rel=1e-13)


# ------------------------------------------------------- embedding net

def test_embed_derivatives_fd(orc, cu_cfg, cu_params):
    """Forward-mode G', G'' against central differences of G."""
    h = 1e-4
    for s in (0.0, 0.05, 0.23, 0.41, 1.2):
        G, dG, ddG = orc.embed(cu_cfg, cu_params, s)
        Gp, dGp, _ = orc.embed(cu_cfg, cu_params, s + h)
        Gm, dGm, _ = orc.embed(cu_cfg, cu_params, s - h)
        np.testing.assert_allclose(dG, (Gp - Gm) / (2 * h), atol=1e-7)
        np.testing.assert_allclose(ddG, (dGp - dGm) / (2 * h), atol=1e-7)
        np.testing.assert_allclose(ddG, (Gp - 2 * G + Gm) / h**2, atol=1e-5)


def test_embed_structure_special_weights(orc, cu_cfg):
    """With W1 = W2 = 0, layer k adds tanh(b_k) to [x, x]: G reduces to
    tanh(s W0 + b0) of column (eta mod d1) plus tanh(b1) of column
    (eta mod d2) plus tanh(b2) (Eqs. 4-5 with the concatenation shortcut)."""
    rng = np.random.default_rng(3)
    p = synth.model_params(cu_cfg, seed=5)
    q = synth.split_params(cu_cfg, p)
    q["W1"][:] = 0.0
    q["W2"][:] = 0.0
    d1, d2, d3 = cu_cfg["emb"]
    for s in rng.uniform(0, 0.6, 4):
        G, dG, _ = orc.embed(cu_cfg, p, s)
        eta = np.arange(d3)
        want = (np.tanh(s * q["W0"][0, eta % d1] + q["b0"][eta % d1])
                + np.tanh(q["b1"][eta % d2]) + np.tanh(q["b2"]))
        np.testing.assert_allclose(G, want, rtol=1e-14, atol=1e-14)
        dwant = q["W0"][0, eta % d1] / np.cosh(s * q["W0"][0, eta % d1] + q["b0"][eta % d1]) ** 2
        np.testing.assert_allclose(dG, dwant, rtol=1e-12, atol=1e-14)


# --------------------------------------------------------- tabulation

def test_hermite_reproduces_planted_quintic(orc):
    """A quintic is its own Hermite interpolant: the coefficients of
    P(x0 + t) in t (numpy's polynomial composition) come back exactly."""
    rng = np.random.default_rng(0)
    for _ in range(20):
        c = rng.standard_normal(6)
        x0, h = rng.uniform(0, 1), rng.choice([0.1, 0.01, 0.001])
        P = np.polynomial.Polynomial(c)
        shifted = P(np.polynomial.Polynomial([x0, 1.0]))     # P(x0 + t)
        want = np.zeros(6)
        want[:len(shifted.coef)] = shifted.coef
        dP, ddP = P.deriv(1), P.deriv(2)
        a = orc.hermite(P(x0), dP(x0), ddP(x0), P(x0 + h), dP(x0 + h), ddP(x0 + h), h)
        scale = np.abs(want) * np.array([1, h, h**2, h**3, h**4, h**5])
        err = np.abs(a - want) * np.array([1, h, h**2, h**3, h**4, h**5])
        assert np.all(err <= 1e-12 * max(1.0, scale.max())), (a, want)


def test_table_matches_net_at_nodes_and_is_c2(orc, cu_cfg, cu_params):
    """Value and first derivative equal the net's at every node, from both
    neighbouring intervals (the interpolation conditions of Sec. 3.2)."""
    tab = orc.Table(cu_cfg, cu_params, 0.7, 0.01, 1.5, 0.1)
    assert tab.coef.shape == (78, 128, 6)
    for theta in (0, 7, 33, 69, 70, 74, 77):
        if theta < 70:
            lo, w = theta * 0.01, 0.01
        else:
            lo, w = 0.7 + (theta - 70) * 0.1, 0.1
        a = tab.coef[theta]
        for x, t in ((lo, 0.0), (lo + w, w)):
            G, dG, ddG = orc.embed(cu_cfg, cu_params, x)
            v = sum(a[:, k] * t**k for k in range(6))
            d = sum(k * a[:, k] * t**(k - 1) for k in range(1, 6))
            dd = sum(k * (k - 1) * a[:, k] * t**(k - 2) for k in range(2, 6))
            np.testing.assert_allclose(v, G, atol=1e-13)
            np.testing.assert_allclose(d, dG, atol=1e-10)
            np.testing.assert_allclose(dd, ddG, atol=1e-7)


def _table_error(orc, cfg, params, h):
    tab = orc.Table(cfg, params, 0.6, h, 0.6, h)
    worst = 0.0
    for s in np.linspace(0.0005, 0.5995, 1201):
        G = orc.embed(cfg, params, s)[0]
        worst = max(worst, np.max(np.abs(tab.eval(s)[0] - G)))
    return worst


def test_table_error_order_six(orc, cu_cfg, cu_params):
    """Quintic Hermite interpolation is sixth order: the error bound is
    h^6 max|g^(6)| / 46080, so halving h divides the error by about 64."""
    e1 = _table_error(orc, cu_cfg, cu_params, 0.1)
    e2 = _table_error(orc, cu_cfg, cu_params, 0.05)
    e3 = _table_error(orc, cu_cfg, cu_params, 0.025)
    assert 30 < e1 / e2 < 100, (e1, e2)
    assert 30 < e2 / e3 < 100, (e2, e3)


def test_table_error_within_remainder_bound(orc, cu_cfg, cu_params):
    """|f - g| <= h^6 max|g^(6)| / 46080 on each interval, with g^(6)
    bounded by a tenth-order finite difference stencil of the net's second
    derivative (a generous bound: the stencil's own error is added)."""
    h = 0.05
    tab = orc.Table(cu_cfg, cu_params, 0.6, h, 0.6, h)
    # g^(6) = (g'')^(4); fourth difference of the analytic g'' with step k
    k = 2e-3
    worst_g6 = 0.0
    for s in np.linspace(0.0, 0.6, 121):
        vals = [orc.embed(cu_cfg, cu_params, s + (m - 2) * k)[2] for m in range(5)]
        g6 = (vals[0] - 4 * vals[1] + 6 * vals[2] - 4 * vals[3] + vals[4]) / k**4
        worst_g6 = max(worst_g6, np.max(np.abs(g6)))
    bound = h**6 * worst_g6 / 46080.0 * 1.5
    err = 0.0
    for s in np.linspace(0.0, 0.5999, 600):
        err = max(err, np.max(np.abs(tab.eval(s)[0] - orc.embed(cu_cfg, cu_params, s)[0])))
    assert err <= bound, (err, bound)


def test_table_beyond_end_is_clamped(orc, cu_cfg, cu_params):
    tab = orc.Table(cu_cfg, cu_params, 0.7, 0.01, 1.5, 0.1)
    G_end, _ = tab.eval(1.5)
    G_far, dG_far = tab.eval(3.0)
    np.testing.assert_allclose(G_far, G_end, atol=1e-12)
    np.testing.assert_allclose(G_far, orc.embed(cu_cfg, cu_params, 1.5)[0], atol=1e-9)
    assert np.all(dG_far == 0.0)


# ---------------------------------------------------------- neighbors

def _shell_counts_by_enumeration(max_m):
    counts = {}
    r = int(math.isqrt(2 * max_m)) + 1
    for n in itertools.product(range(-r, r + 1), repeat=3):
        if sum(n) % 2 or n == (0, 0, 0):
            continue
        q = n[0] ** 2 + n[1] ** 2 + n[2] ** 2
        if q % 2 == 0 and q // 2 <= max_m:
            counts[q // 2] = counts.get(q // 2, 0) + 1
    return counts


@pytest.mark.parametrize("ncell", [2, 3, 5])
def test_fcc_neighbor_shells(orc, cu_cfg, ncell):
    """Perfect FCC: 176 neighbors within 8 A in the nine shells of the
    golden file, for cells smaller and larger than the cut-off sphere
    (the 2x2x2 cell needs several periodic images of every atom)."""
    gold = json.load(open(os.path.join(GOLD, "fcc_shells.json")))
    want = {s["m"]: s["count"] for s in gold["shells"]}
    assert want == _shell_counts_by_enumeration(9)
    x, box = synth.fcc(ncell)
    for i in (0, 1, len(x) - 1):
        j, img, r, n = orc.neighbors(cu_cfg, x, box, i)
        assert n == gold["total_within_rcut"]
        m = np.rint(2 * (r / gold["a"]) ** 2).astype(int)
        np.testing.assert_allclose(r, gold["a"] * np.sqrt(m / 2.0), rtol=1e-12)
        got = {int(k): int(v) for k, v in zip(*np.unique(m, return_counts=True))}
        assert got == want
        assert np.all(np.diff(r) >= 0)


def test_neighbors_brute_force_tiny_cell(orc):
    """Random tiny periodic cell against a direct enumeration of images."""
    cfg = small_cfg(rcut=4.0, rcut_smth=0.5)
    rng = np.random.default_rng(7)
    box = np.diag([3.1, 4.3, 5.2])
    x = rng.uniform(0, 1, (5, 3)) * np.diag(box)
    for i in range(5):
        j, img, r, n = orc.neighbors(cfg, x, box, i)
        want = []
        for jj in range(5):
            for sh in itertools.product(range(-3, 4), repeat=3):
                if jj == i and sh == (0, 0, 0):
                    continue
                d = (x[jj] - x[i]) + np.array(sh) * np.diag(box)
                rr = math.sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2])
                if rr < cfg["rcut"]:
                    want.append((rr, jj, sh))
        want.sort()
        assert n == len(want)
        np.testing.assert_allclose(r, [w[0] for w in want], rtol=1e-14)
        assert list(j) == [w[1] for w in want]
        assert [tuple(v) for v in img] == [w[2] for w in want]


def test_sel_truncation_keeps_nearest(orc):
    """With more neighbors than sel, the sel nearest are kept (the rest are
    counted as dropped).  T is additive over neighbors, so T of an atom must
    equal the sum of the T's of the dimers it forms with its sel nearest
    neighbors (each dimer pinned by the closed form above)."""
    cfg = synth.copper_model_config(sel=150)
    p = synth.model_params(cfg)
    x, box = synth.copper(3, 0.1, 17)
    r = orc.evaluate(cfg, p, x, box, forces=False, desc=True)
    assert r["dropped"] == int(np.sum(np.maximum(r["nnei"] - 150, 0))) > 0
    i = 5
    j, img, rr, n = orc.neighbors(cfg, x, box, i)
    assert n > 150
    L = np.diag(box)
    T = np.zeros_like(r["T"][i])
    for jj, sh in zip(j[:150], img[:150]):
        d = (x[jj] - x[i]) + sh * L
        dimer = orc.evaluate(cfg, p, np.array([[0.0, 0.0, 0.0], d]), None, forces=False, desc=True)
        T += dimer["T"][0]
    np.testing.assert_allclose(r["T"][i], T, rtol=1e-11, atol=1e-15)
    r2 = orc.evaluate(cfg, p, x + 0.37, box, forces=False)
    assert r2["E"] == pytest.approx(r["E"], rel=1e-12)


# ------------------------------------------------------- descriptor

def test_dimer_closed_form(orc, cu_cfg, cu_params):
    """One neighbor at distance r: T_k = sig s u_k G(s) with u = (1, r_hat),
    so D_ab = 2 sig^2 s^2 G_a G_b (Eq. 2 with |u|^2 = 2)."""
    r = 3.1
    d = np.array([0.6, -1.1, 0.0])
    d[2] = math.sqrt(r * r - d[0] ** 2 - d[1] ** 2)
    x = np.array([[1.0, 2.0, 3.0], [1.0, 2.0, 3.0] + d])
    out = orc.evaluate(cu_cfg, cu_params, x, None, desc=True)
    w, _ = orc.switch(cu_cfg, r)
    s = w / r
    G = orc.embed(cu_cfg, cu_params, s)[0]
    sig, Ml = cu_cfg["desc_scale"], cu_cfg["m_lt"]
    u = np.concatenate([[1.0], d / r])
    np.testing.assert_allclose(out["T"][0], sig * s * np.outer(u, G), rtol=1e-13, atol=1e-16)
    np.testing.assert_allclose(out["D"][0].reshape(Ml, -1), 2 * sig**2 * s**2 * np.outer(G[:Ml], G),
                               rtol=1e-12, atol=1e-18)
    # the two atoms see mirror images: same descriptor, same energy
    np.testing.assert_allclose(out["D"][1], out["D"][0], rtol=1e-13)
    assert out["e_atom"][0] == pytest.approx(out["e_atom"][1], rel=1e-14)
    # Newton's third law
    np.testing.assert_allclose(out["F"][0], -out["F"][1], rtol=1e-12, atol=1e-18)


def test_fitting_net_special_weights(orc, cu_cfg):
    """With V2 = V3 = 0 and c2 = c3 = 0 the shortcuts pass y1 through:
    E_i = tanh(D V1 + c1) . w4 + b4; and an isolated atom has D = 0, so
    E_i = tanh(c1) . w4 + b4 and no force."""
    p = synth.model_params(cu_cfg, seed=9)
    q = synth.split_params(cu_cfg, p)
    q["V2"][:] = 0.0
    q["V3"][:] = 0.0
    q["c2"][:] = 0.0
    q["c3"][:] = 0.0
    q["b4"][:] = 0.3
    x, box = synth.copper(2, 0.1, 4)
    out = orc.evaluate(cu_cfg, p, x, box, desc=True)
    want = np.tanh(out["D"] @ q["V1"] + q["c1"]) @ q["w4"] + 0.3
    np.testing.assert_allclose(out["e_atom"], want, rtol=1e-13)
    iso = orc.evaluate(cu_cfg, p, np.zeros((1, 3)), None, desc=True)
    assert np.all(iso["D"] == 0.0)
    assert iso["e_atom"][0] == pytest.approx(np.tanh(q["c1"]) @ q["w4"] + 0.3, rel=1e-14)
    assert np.all(iso["F"] == 0.0)


# -------------------------------------------------------- symmetries

@pytest.fixture(scope="module")
def cell108():
    return synth.copper(3, 0.1, 21)


def test_translation_invariance(orc, cu_cfg, cu_params, cell108):
    x, box = cell108
    a = orc.evaluate(cu_cfg, cu_params, x, box)
    b = orc.evaluate(cu_cfg, cu_params, x + np.array([0.37, -5.1, 12.9]), box)
    assert b["E"] == pytest.approx(a["E"], rel=1e-13)
    np.testing.assert_allclose(b["F"], a["F"], atol=1e-15)


def test_permutation_invariance(orc, cu_cfg, cu_params, cell108):
    x, box = cell108
    perm = np.random.default_rng(1).permutation(len(x))
    a = orc.evaluate(cu_cfg, cu_params, x, box)
    b = orc.evaluate(cu_cfg, cu_params, x[perm], box)
    assert b["E"] == pytest.approx(a["E"], rel=1e-13)
    np.testing.assert_allclose(b["F"], a["F"][perm], atol=1e-15)
    np.testing.assert_allclose(b["e_atom"], a["e_atom"][perm], rtol=1e-13)


def test_rotation_invariance_open_cluster(orc, cu_cfg, cu_params):
    """Open cluster: E unchanged and F rotates under a random rotation."""
    rng = np.random.default_rng(2)
    x = synth.copper(2, 0.15, 5)[0]
    Q = random_rotation(rng)
    a = orc.evaluate(cu_cfg, cu_params, x, None)
    b = orc.evaluate(cu_cfg, cu_params, x @ Q.T, None)
    assert b["E"] == pytest.approx(a["E"], rel=1e-13)
    np.testing.assert_allclose(b["F"], a["F"] @ Q.T, atol=1e-14)
    # torque-free and momentum-free
    np.testing.assert_allclose(a["F"].sum(0), 0.0, atol=1e-14)
    np.testing.assert_allclose(np.cross(x, a["F"]).sum(0), 0.0, atol=1e-13)
    # virial of an open cluster equals sum_k x_k (x) F_k
    np.testing.assert_allclose(a["W"], x.T @ a["F"], atol=1e-13)


def test_axis_permutation_periodic(orc, cu_cfg, cu_params, cell108):
    """A cubic periodic cell is invariant under relabelling the axes."""
    x, box = cell108
    a = orc.evaluate(cu_cfg, cu_params, x, box)
    for perm in ((1, 0, 2), (2, 0, 1)):
        b = orc.evaluate(cu_cfg, cu_params, x[:, perm], box)
        assert b["E"] == pytest.approx(a["E"], rel=1e-13)
        np.testing.assert_allclose(b["F"], a["F"][:, perm], atol=1e-15)
    # mirror x -> L - x
    L = box[0, 0]
    xm = x.copy()
    xm[:, 0] = L - xm[:, 0]
    b = orc.evaluate(cu_cfg, cu_params, xm, box)
    assert b["E"] == pytest.approx(a["E"], rel=1e-13)
    np.testing.assert_allclose(b["F"][:, 0], -a["F"][:, 0], atol=1e-15)


def test_extensivity_tiling(orc, cu_cfg, cu_params):
    """E of a 2x2x2 tiling of a 32-atom cell is 8 E(cell), forces tile.
    The small cell reaches its neighbors through many periodic images; the
    tiled cell through fewer, so this pins the image handling."""
    x, box = synth.copper(2, 0.1, 8)
    L = box[0, 0]
    tiles = [x + L * np.array(t) for t in itertools.product(range(2), repeat=3)]
    X = np.concatenate(tiles)
    a = orc.evaluate(cu_cfg, cu_params, x, box)
    b = orc.evaluate(cu_cfg, cu_params, X, 2 * box)
    assert b["E"] == pytest.approx(8 * a["E"], rel=1e-13)
    np.testing.assert_allclose(b["F"], np.tile(a["F"], (8, 1)), atol=1e-15)
    np.testing.assert_allclose(b["W"], 8 * a["W"], rtol=1e-11, atol=1e-15)


def test_perfect_fcc_has_zero_force(orc, cu_cfg, cu_params):
    """Every atom of a perfect FCC crystal is an inversion centre."""
    x, box = synth.fcc(3)
    a = orc.evaluate(cu_cfg, cu_params, x, box)
    assert np.max(np.abs(a["F"])) < 1e-15
    np.testing.assert_allclose(a["e_atom"], a["e_atom"][0], rtol=1e-13)
    W = a["W"]
    np.testing.assert_allclose(W, W[0, 0] * np.eye(3), atol=1e-12 * abs(W[0, 0]))


# --------------------------------------------------------- gradients

@pytest.mark.parametrize("ncell", [2, 3])
def test_forces_central_differences(orc, cu_cfg, cu_params, ncell):
    """F = -dE/dx by central differences with h = 1e-4 A in FP64."""
    x, box = synth.copper(ncell, 0.1, 30 + ncell)
    a = orc.evaluate(cu_cfg, cu_params, x, box)
    h = 1e-4
    rng = np.random.default_rng(ncell)
    for i in rng.choice(len(x), 4, replace=False):
        for c in range(3):
            xp, xm = x.copy(), x.copy()
            xp[i, c] += h
            xm[i, c] -= h
            Ep = orc.evaluate(cu_cfg, cu_params, xp, box, forces=False)["E"]
            Em = orc.evaluate(cu_cfg, cu_params, xm, box, forces=False)["E"]
            fd = -(Ep - Em) / (2 * h)
            assert a["F"][i, c] == pytest.approx(fd, abs=2e-9 + 1e-5 * abs(fd))
    np.testing.assert_allclose(a["F"].sum(0), 0.0, atol=1e-15)


def test_virial_strain_derivative(orc, cu_cfg, cu_params):
    """W = -dE/d(eps) under a homogeneous strain of box and positions;
    W is symmetric."""
    x, box = synth.copper(2, 0.1, 41)
    a = orc.evaluate(cu_cfg, cu_params, x, box)
    W = a["W"]
    np.testing.assert_allclose(W, W.T, atol=1e-12)
    h = 1e-5
    for (p, q) in ((0, 0), (1, 1), (2, 2)):
        eps = np.zeros((3, 3))
        eps[p, q] = h
        Ep = orc.evaluate(cu_cfg, cu_params, x @ (np.eye(3) + eps).T, box @ (np.eye(3) + eps).T, forces=False)["E"]
        Em = orc.evaluate(cu_cfg, cu_params, x @ (np.eye(3) - eps).T, box @ (np.eye(3) - eps).T, forces=False)["E"]
        fd = -(Ep - Em) / (2 * h)
        assert W[p, q] == pytest.approx(fd, rel=1e-6, abs=1e-9)


def test_tabulated_oracle_close_to_net(orc, cu_cfg, cu_params):
    """The tabulated model approaches the net as the stride shrinks
    (Sec. 3.2: the error vanishes with the interval size)."""
    x, box = synth.copper(3, 0.05, 11)
    ref = orc.evaluate(cu_cfg, cu_params, x, box)
    errs = []
    for h in (0.1, 0.01):
        tab = orc.Table(cu_cfg, cu_params, 0.7, h, 1.5, 0.1)
        t = orc.evaluate(cu_cfg, cu_params, x, box, table=tab)
        assert t["table_oob"] == 0
        rmse_e = abs(t["E"] - ref["E"]) / len(x)
        rmse_f = np.sqrt(np.mean((t["F"] - ref["F"]) ** 2))
        errs.append((rmse_e, rmse_f))
    assert errs[1][0] < errs[0][0] and errs[1][1] < errs[0][1]
    assert errs[1][0] < 1e-10 and errs[1][1] < 1e-10


def test_flop_model_of_the_paper():
    """Sec. 3.2: tabulated/original embedding FLOPs = 56/(1 + 10 d1); at
    d1 = 32 this saves 82 percent (ideal speed-up 5.6-5.7)."""
    gold = json.load(open(os.path.join(GOLD, "paper_numbers.json")))
    d1 = gold["d1"]
    orig = 512 * d1 + 10 * 512 * d1 ** 2
    tab = 56 * 512 * d1
    assert int(100 * (1 - tab / orig)) == gold["flops_saved_percent"]   # 82.6 printed as 82
    assert abs(orig / tab - gold["ideal_speedup"]) < 0.2
    # d1 + 10 d1^2 is the multiply-add count of the 1-32-64-128 net
    e = gold["embedding_widths"]
    assert e[0] + e[0] * e[1] + e[1] * e[2] == d1 + 10 * d1 ** 2
    g = gold["G_memory_example"]
    assert round(g["N_a"] * g["N_m"] * g["M"] * g["bytes_per"] / 1e9, 1) == g["GB"]


def test_nve_energy_error_scales_with_dt_squared(orc, cu_cfg):
    """Velocity Verlet conserves energy to O(dt^2): halving dt divides the
    largest total-energy deviation by about 4.  The output weights are scaled
    up so that forces reach the size of real copper forces (0.1 eV/A)."""
    import synth
    p = synth.model_params(cu_cfg)
    synth.split_params(cu_cfg, p)["w4"][:] *= 2000.0
    x, box = synth.copper(2, 0.05, 3)
    v = synth.maxwell_boltzmann(len(x), 330.0, seed=4)
    dev = []
    for dt, n in ((1.0, 40), (0.5, 80)):
        _, _, rows = orc.velocity_verlet(cu_cfg, p, x, v, box, synth.M_CU, dt, n)
        et = rows.sum(1)
        dev.append(np.max(np.abs(et - et[0])))
        # no secular drift: the end point is not the worst point by far
        assert abs(et[-1] - et[0]) <= dev[-1]
    assert 3.5 < dev[0] / dev[1] < 4.5, dev
    assert dev[0] < 1e-3 * rows[0, 1]


# ---------------------------------------------------------- tabulated tanh

def test_tanh_table_error_bound(orc):
    """Second-order table on [0, 8): value and slope at the left node, value
    at the right node.  Its error is f'''(xi)/6 t^2 (t - h), at most
    (4/27)(h^3/6) max|tanh'''| = (4/27)(h^3/6) 2 inside the range; beyond 8
    it is 1 - tanh(x) (the saturation the paper states); odd exactly."""
    h = 1.0 / 128.0
    x = np.linspace(0.0, 8.0, 256001)[:-1]
    e = np.abs(orc.tanh_table(x) - np.tanh(x))
    bound = 4.0 / 27.0 * h ** 3 / 6.0 * 2.0
    assert e.max() <= 1.001 * bound
    assert e.max() > 0.5 * bound          # the bound is attained near 0, where |tanh'''| = 2
    nodes = np.arange(0, 1024) * h
    np.testing.assert_allclose(orc.tanh_table(nodes), np.tanh(nodes), rtol=0, atol=3e-16)   # libm vs numpy: 1 ulp
    right = nodes[1:] - 1e-13             # value at the right node is matched too
    assert np.max(np.abs(orc.tanh_table(right) - np.tanh(right))) < 1e-12
    big = np.array([8.0, 9.5, 40.0])
    assert np.all(orc.tanh_table(big) == 1.0)
    assert abs(orc.tanh_table(np.array([8.0]))[0] - np.tanh(8.0)) == pytest.approx(1 - np.tanh(8.0), rel=1e-9)
    xs = np.linspace(-10, 10, 2001)
    np.testing.assert_array_equal(orc.tanh_table(-xs), -orc.tanh_table(xs))


def test_tanh_table_in_fitting_net(orc, cu_cfg, cu_params):
    """The option switches only the fitting net's tanh: a dimer (where the
    embedding is untouched) changes by the table's error times the fitting
    net's sensitivity, and the forces stay -dE/dx by central differences."""
    import synth
    cfg = dict(cu_cfg, tanh_table=1)
    x, box = synth.copper(2, 0.1, 5)
    a = orc.evaluate(cu_cfg, cu_params, x, box)
    b = orc.evaluate(cfg, cu_params, x, box)
    dE = abs(a["E"] - b["E"]) / len(x)
    assert 0 < dE < 1e-5
    hstep = 1e-5
    for (i, c) in ((0, 0), (7, 2)):
        xp, xm = x.copy(), x.copy()
        xp[i, c] += hstep
        xm[i, c] -= hstep
        fd = (orc.evaluate(cfg, cu_params, xp, box)["E"] - orc.evaluate(cfg, cu_params, xm, box)["E"]) / (2 * hstep)
        # the backward takes 1 - y^2 of the tabulated y, not the table's own slope: agreement to the table error
        assert abs(-b["F"][i, c] - fd) <= 1e-6 * np.max(np.abs(b["F"])) + 1e-9
