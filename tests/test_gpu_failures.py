"""Failure handling of the force step on the GPU, through the C-ABI: each
condition the library detects on the device ends in its documented status,
and the kernels themselves run to completion (no input here makes a kernel
fault: a far-moved atom only loses candidates, a NaN position fails every
distance test, an overflowing energy is an ordinary inf).

  DP_ERR_SKIN       an atom moved skin/2 or more since the build
  DP_ERR_NONFINITE  a non-finite coordinate (after the build) or energy
  DP_ERR_ARG        a non-finite coordinate at the build; a model whose rcut
                    reaches past the list's rcut + skin
  capacity retry    a crowded cell and a candidate list past its capacity are
                    grown and built again, and the result equals the oracle's
"""
import numpy as np
import pytest

import oracle
import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TAB = (0.7, 0.01, 1.5, 0.1)


@pytest.fixture(scope="module")
def P():
    import paper_2201_01446_amd as P
    assert torch.cuda.is_available()
    return P


@pytest.fixture(scope="module")
def model(P, cu_cfg, cu_params):
    return P.Model(cu_cfg, cu_params).tabulate(*TAB)


def dev(x):
    return torch.tensor(np.ascontiguousarray(x), dtype=torch.float64, device="cuda")


def status_of(fn):
    import paper_2201_01446_amd as P
    try:
        fn()
    except P.DPError as e:
        return e.status
    return 0


@pytest.mark.parametrize("move,expect", [(0.9, 0), (1.1, -8)])
def test_skin_flag_on_compute(P, model, move, expect):
    """One atom moved by 0.9 A (under skin/2 = 1 A) or 1.1 A (over it) after
    the build: the evaluation completes either way, and only the second is
    reported by dp_nlist_check."""
    x, box = synth.copper(4, 0.05, 3)
    nl = P.NeighborList(model, dev(x), box, skin=2.0)
    xm = x.copy()
    xm[5] += move * np.array([0.6, 0.8, 0.0])
    print(f"skin flag: move={move} A", flush=True)
    out = P.compute(model, nl, dev(xm), precision=P.FP64)
    torch.cuda.synchronize()
    assert np.isfinite(out["E"].item())
    assert status_of(nl.check) == expect
    nl.build(dev(xm), box, 2.0)    # a rebuild clears the flag
    assert status_of(nl.check) == 0


def test_skin_flag_stops_nve(P, model):
    """An MD run whose atoms move ~0.3 A per step (velocities far above any
    temperature) with rebuilds every 10 steps: the check at the first rebuild
    stops it with DP_ERR_SKIN."""
    x, box = synth.copper(4, 0.05, 3)
    v = synth.maxwell_boltzmann(len(x), 330.0, seed=4)
    v *= 0.3 / np.sqrt(np.mean(np.sum(v * v, axis=1)))
    xd, vd = dev(x), dev(v)
    nl = P.NeighborList(model, xd, box, skin=2.0)
    print("skin flag: nve", flush=True)
    st = status_of(lambda: P.nve_run(model, nl, xd, vd, box, synth.M_CU, 1.0, 20, rebuild_every=10,
                                     precision=P.FP64))
    assert st == -8


def test_nonfinite_coordinate(P, model):
    """A NaN coordinate: DP_ERR_ARG at the build; after a build, the
    evaluation completes and dp_nlist_check reports DP_ERR_NONFINITE."""
    x, box = synth.copper(3, 0.05, 5)
    bad = x.copy()
    bad[7, 1] = np.nan
    print("nonfinite coordinate", flush=True)
    assert status_of(lambda: P.NeighborList(model, dev(bad), box)) == -1
    nl = P.NeighborList(model, dev(x), box)
    P.compute(model, nl, dev(bad), precision=P.FP32)
    torch.cuda.synchronize()
    assert status_of(nl.check) == -7


def test_nonfinite_energy(P, cu_cfg, cu_params):
    """Output bias 1e308: every E_i is finite, their sum is not.  The FP64
    evaluation completes and dp_nlist_check reports DP_ERR_NONFINITE; an MD
    run over the same model stops with it."""
    p = cu_params.copy()
    synth.split_params(cu_cfg, p)["b4"][:] = 1e308
    m = P.Model(cu_cfg, p).tabulate(*TAB)
    x, box = synth.copper(2, 0.05, 5)
    nl = P.NeighborList(m, dev(x), box)
    print("nonfinite energy", flush=True)
    out = P.compute(m, nl, dev(x), precision=P.FP64, atom_energy=True)
    torch.cuda.synchronize()
    assert np.all(np.isfinite(out["e_atom"].cpu().numpy())) and not np.isfinite(out["E"].item())
    assert status_of(nl.check) == -7
    xd, vd = dev(x), dev(np.zeros_like(x))
    assert status_of(lambda: P.nve_run(m, nl, xd, vd, box, synth.M_CU, 1.0, 2, precision=P.FP64)) == -7


def test_model_cutoff_beyond_list(P, cu_cfg, cu_params):
    """A list built for rcut 8 A + skin 2 A serves a model of rcut 9.5 A
    (within its reach: correct, the early end of the scan switched off) but
    not one of rcut 10.5 A (DP_ERR_ARG)."""
    x, box = synth.copper(5, 0.05, 11)
    m8 = P.Model(cu_cfg, cu_params).tabulate(*TAB)
    nl = P.NeighborList(m8, dev(x), box, skin=2.0)
    cfg95 = dict(cu_cfg, rcut=9.5)
    p95 = synth.model_params(cfg95)
    m95 = P.Model(cfg95, p95).tabulate(*TAB)
    print("model cut-off beyond list", flush=True)
    out = P.compute(m95, nl, dev(x), precision=P.FP64, atom_energy=True)
    torch.cuda.synchronize()
    ref = oracle.evaluate(cfg95, p95, x, box, table=oracle.Table(cfg95, p95, *TAB))
    Es = max(1.0, float(np.max(np.abs(ref["e_atom"]))))
    assert np.max(np.abs(out["e_atom"].cpu().numpy() - ref["e_atom"])) <= 1e-10 * Es
    assert np.max(np.abs(out["F"].cpu().numpy() - ref["F"])) <= 1e-10 * np.max(np.abs(ref["F"]))
    cfg105 = dict(cu_cfg, rcut=10.5)
    m105 = P.Model(cfg105, synth.model_params(cfg105)).tabulate(*TAB)
    assert status_of(lambda: P.compute(m105, nl, dev(x), precision=P.FP64)) == -1


def crowded_cell():
    """216 atoms in a 30 A box: 150 in a ball of radius 4.5 A (pairs at least
    0.85 A apart) around the center of one cell of the 6^3 grid, the rest on
    a 5 A lattice away from it.  The cell holds 48 atoms against a capacity
    of 16, and the ball's atoms have up to 158 candidates against 128."""
    rng = np.random.Generator(np.random.PCG64(23))
    g = np.stack(np.meshgrid(*[np.arange(6) * 5.0 + 2.5] * 3, indexing="ij"), -1).reshape(-1, 3)
    c = np.array([17.5, 17.5, 17.5])
    lat = g[np.linalg.norm(g - c, axis=1) > 6.0][:66]
    ball = []
    while len(ball) < 150:
        p = c + rng.uniform(-4.5, 4.5, 3)
        if np.linalg.norm(p - c) <= 4.5 and all(np.linalg.norm(p - q) >= 0.85 for q in ball):
            ball.append(p)
    return np.concatenate([lat, np.array(ball)]), np.diag([30.0] * 3)


@pytest.mark.parametrize("driver", ["build", "nve"])
def test_capacity_retry(P, model, cu_cfg, cu_params, driver):
    """The crowded cell overflows both the cell and the candidate capacity of
    the first build; the list grows both and builds again.  The energy,
    forces and neighbor counts then equal the oracle's (FP64), through
    dp_build_nlist and through the first build of an MD run (0 steps)."""
    x, box = crowded_cell()
    ref = oracle.evaluate(cu_cfg, cu_params, x, box, table=oracle.Table(cu_cfg, cu_params, *TAB))
    print(f"capacity retry: {driver}", flush=True)
    xd = dev(x)
    if driver == "build":
        nl = P.NeighborList(model, xd, box, skin=2.0)
    else:
        # a list first built for the uncrowded 6^3 lattice (capacities 16 and 128)
        g = np.stack(np.meshgrid(*[np.arange(6) * 5.0 + 2.5] * 3, indexing="ij"), -1).reshape(-1, 3)
        nl = P.NeighborList(model, dev(g), box, skin=2.0)
        th = P.nve_run(model, nl, xd, dev(np.zeros_like(x)), box, synth.M_CU, 1.0, 0, precision=P.FP64)
        torch.cuda.synchronize()
        assert abs(th[0, 0].item() - ref["E"]) <= 1e-10 * abs(ref["E"])
    out = P.compute(model, nl, xd, precision=P.FP64, atom_energy=True)
    nn = P.descriptor(model, nl, xd, precision=P.FP64)["nnei"]
    torch.cuda.synchronize()
    np.testing.assert_array_equal(nn.cpu().numpy(), ref["nnei"])
    Es = max(1.0, float(np.max(np.abs(ref["e_atom"]))))
    assert np.max(np.abs(out["e_atom"].cpu().numpy() - ref["e_atom"])) <= 1e-10 * Es
    assert np.max(np.abs(out["F"].cpu().numpy() - ref["F"])) <= 1e-10 * np.max(np.abs(ref["F"]))
    assert nl.stats()["cap_overflow"] == 0
    nl.check()
