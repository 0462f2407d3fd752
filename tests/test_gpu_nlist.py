"""The neighbor list with skin (paper Sec. 2.1, L_Rc(i) with the 2 A buffer of
the MD protocol) against brute force, entry by entry, through
dp_nlist_export.

For every atom the list must hold exactly the (j, image n) pairs within
rcut + skin (compared as sets with the oracle's brute-force search over all
atoms and images, cut-off rcut + skin, for sampled atoms), each stored
distance must be |x_j - x_i + n L| rounded to FP32 (within one FP32 ulp: the
device measures from the wrapped positions), rows are sorted by that
distance (with several types: grouped by neighbor type, type 0 first, and
sorted within each type), and the reverse slot of every pair must point at
(i, -n) in j's row.  Exact integer results; the counts must equal the
oracle's for every sampled atom.
"""
import numpy as np
import pytest

import oracle
import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

SKIN = 2.0


@pytest.fixture(scope="module")
def P():
    import paper_2201_01446_amd as P
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return P


def dev(a, dtype=torch.float64):
    return torch.tensor(np.ascontiguousarray(a), dtype=dtype, device="cuda")


def unpack(sh):
    """Packed image shifts -> [..., 3] int (three int8 in the low 24 bits)."""
    sh = sh.astype(np.int64)
    return np.stack([((sh >> (8 * a)) & 0xFF).astype(np.uint8).view(np.int8) for a in range(3)], -1).astype(np.int64)


def check_list(P, cfg, params, x, box, types=None, sample=None, seed=0, skin=SKIN):
    m = P.Model(cfg, params)
    t = None if types is None else dev(types, torch.int32)
    nl = P.NeighborList(m, dev(x), box, skin=skin, types=t)
    e = {k: v.cpu().numpy() for k, v in nl.export().items()}
    assert nl.stats()["cap_overflow"] == 0
    cnt, nei, dist, rev = e["cnt"], e["nei"], e["dist"], e["rev"].astype(np.int64)
    n, C = nei.shape
    assert n == len(x) and np.all(cnt >= 0) and np.all(cnt <= C)
    L = np.diag(box)
    valid = np.arange(C)[None, :] < cnt[:, None]
    ii = np.nonzero(valid)[0]
    jj, dd, rr = nei[valid].astype(np.int64), dist[valid], rev[valid]
    ss = unpack(e["shift"][valid])
    assert np.all((jj >= 0) & (jj < n))

    # distances: those of (j, n) from the caller's coordinates, in FP32
    r = np.sqrt(np.sum((x[jj] - x[ii] + ss * L) ** 2, axis=1))
    assert np.all(np.abs(dd.astype(np.float64) - r) <= np.spacing(r.astype(np.float32)))
    assert np.all(r < cfg["rcut"] + skin)

    # order: ascending distance within each row (within each type's run)
    same_row = ii[1:] == ii[:-1]
    if types is None:
        assert np.all(dd[1:][same_row] >= dd[:-1][same_row])
    else:
        tj = types[jj]
        assert np.all(tj[1:][same_row] >= tj[:-1][same_row])
        same_run = same_row & (tj[1:] == tj[:-1])
        assert np.all(dd[1:][same_run] >= dd[:-1][same_run])

    # no pair twice
    key = (ii * n + jj) * 4096 + ((ss[:, 0] + 8) * 256 + (ss[:, 1] + 8) * 16 + (ss[:, 2] + 8))
    assert len(np.unique(key)) == len(key)

    # reverse slots: (i, -n) at rev in j's row; -1 only where the two sides'
    # distances straddle rcut + skin
    miss = rr < 0
    assert np.all(np.abs(r[miss] - (cfg["rcut"] + skin)) < 1e-5)
    ok = ~miss
    assert np.all(rr[ok] < cnt[jj[ok]])
    assert np.array_equal(nei[jj[ok], rr[ok]], ii[ok])
    assert np.array_equal(unpack(e["shift"][jj[ok], rr[ok]]), -ss[ok])

    # the sets against brute force
    cfg_b = dict(cfg, rcut=cfg["rcut"] + skin)
    atoms = np.arange(n) if sample is None else np.random.Generator(np.random.PCG64(seed)).choice(n, sample,
                                                                                                   replace=False)
    for i in atoms:
        oj, on, _, ocnt = oracle.neighbors(cfg_b, x, box, int(i))
        assert cnt[i] == ocnt, f"atom {i}: {cnt[i]} candidates, brute force {ocnt}"
        got = set(zip(nei[i, :cnt[i]].tolist(), map(tuple, unpack(e["shift"][i, :cnt[i]]).tolist())))
        assert got == set(zip(oj.tolist(), map(tuple, on.tolist()))), f"atom {i}"
    return cnt


@pytest.mark.parametrize("ncell,sigma,seed", [(5, 0.05, 21), (3, 0.1, 5), (2, 0.1, 8)])
def test_copper_lists_small_cells(P, cu_cfg, cu_params, ncell, sigma, seed):
    """Boxes of 2-5 FCC cells (7.3-18.2 A edges, below 2 (rcut + skin)): many
    images of every atom, and of the atom itself, in each list."""
    x, box = synth.copper(ncell, sigma, seed)
    check_list(P, cu_cfg, cu_params, x, box)


def test_copper_lists_wide_skin(P, cu_cfg, cu_params):
    """A 4 A skin: about 610 candidates per atom, so the rows take the sort
    for more than 512 keys."""
    x, box = synth.copper(5, 0.05, 23)
    cnt = check_list(P, cu_cfg, cu_params, x, box, skin=4.0)
    assert cnt.min() > 512


def test_copper_list_108k_sampled(P, cu_cfg, cu_params):
    """The MD workload's box: 30^3 FCC cells (108,000 atoms), sigma 0.08 A;
    every entry checked for distance, order and reverse slot, and 24
    sampled atoms' sets against brute force."""
    x, box = synth.copper(30, 0.08, synth.SEED_CFG[1])
    cnt = check_list(P, cu_cfg, cu_params, x, box, sample=24, seed=3)
    assert 330 < cnt.mean() < 380


@pytest.mark.parametrize("nrep", [1, 2])
def test_water_lists_grouped_by_type(P, nrep):
    """Two types (rcut 6 A): rows grouped by neighbor type, sorted within.
    One cell (12.4 A edge, below 2 (rcut + skin)) holds several images of
    some atoms in a list; two cells at most one."""
    cfg = synth.water_model_config()
    p = synth.model_params(cfg)
    x, t, box = synth.water(nrep, sigma=0.02)
    check_list(P, cfg, p, x, box, types=t, sample=64, seed=4)


def test_list_after_rebuild_at_moved_positions(P, cu_cfg, cu_params):
    """A list rebuilt in place at displaced positions (as the MD loop does)
    is the list of the new positions."""
    x, box = synth.copper(5, 0.05, 31)
    m = P.Model(cu_cfg, cu_params)
    nl = P.NeighborList(m, dev(x), box, skin=SKIN)
    x2 = synth.perturb(x, 0.3, 32)
    nl.build(dev(x2), box, skin=SKIN)
    e = nl.export()
    cnt = e["cnt"].cpu().numpy()
    cfg_b = dict(cu_cfg, rcut=cu_cfg["rcut"] + SKIN)
    for i in range(0, len(x2), 25):
        assert cnt[i] == oracle.neighbors(cfg_b, x2, box, i)[3]
    check_list(P, cu_cfg, cu_params, x2, box, sample=50, seed=5)
