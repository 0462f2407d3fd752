"""The rungs of the optimization ladder (plain; tabulated but unfused;
fused per neighbor over padded rows; fused per neighbor over real
neighbors; fused per table-interval run) compute the same model: each
tabulated rung equals the oracle's tabulated mode, at sel = 192 and at the
paper's padding regime sel = 512."""
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


def gpu_eval(P, model, x, box, mode, precision):
    xd = torch.tensor(x, dtype=torch.float64, device="cuda")
    nl = P.NeighborList(model, xd, box, skin=2.0)
    out = P.compute(model, nl, xd, mode=mode, precision=precision, atom_energy=True)
    torch.cuda.synchronize()
    return {k: v.cpu().numpy() for k, v in out.items() if v is not None}


def check(got, ref, precision, n):
    if precision == 0:
        assert abs(got["E"][0] - ref["E"]) <= 1e-10 * abs(ref["E"])
        assert np.max(np.abs(got["F"] - ref["F"])) <= 1e-10 * np.max(np.abs(ref["F"]))
        assert np.max(np.abs(got["W"] - ref["W"])) <= 1e-10 * np.max(np.abs(ref["W"]))
    else:
        Fs = np.sqrt(np.mean(ref["F"] ** 2))
        assert abs(got["E"][0] - ref["E"]) / n <= 1e-5
        assert np.sqrt(np.mean((got["F"] - ref["F"]) ** 2)) <= min(1e-3, 1e-4 * Fs)
        assert np.max(np.abs(got["e_atom"] - ref["e_atom"])) <= 1e-5


@pytest.mark.parametrize("precision", [0, 1])
@pytest.mark.parametrize("mode", [2, 3, 4])
def test_rungs_sel192(P, cu_cfg, cu_params, mode, precision):
    model = P.Model(cu_cfg, cu_params).tabulate(*TAB)
    x, box = synth.copper(5, 0.05, synth.SEED_CFG[1])
    ref = oracle.evaluate(cu_cfg, cu_params, x, box, table=oracle.Table(cu_cfg, cu_params, *TAB))
    got = gpu_eval(P, model, x, box, mode, precision)
    check(got, ref, precision, len(x))


@pytest.mark.parametrize("mode", [0, 1, 2, 3, 4])
def test_rungs_sel512(P, mode):
    """sel = 512 (most rows are padding: ~178 real neighbors): every rung in
    FP64 against the oracle (untabulated for the plain rung)."""
    cfg = synth.copper_model_config(sel=512)
    params = synth.model_params(cfg)
    model = P.Model(cfg, params).tabulate(*TAB)
    x, box = synth.copper(3, 0.1, 91)
    table = None if mode == 1 else oracle.Table(cfg, params, *TAB)
    ref = oracle.evaluate(cfg, params, x, box, table=table)
    got = gpu_eval(P, model, x, box, mode, 0)
    check(got, ref, 0, len(x))
