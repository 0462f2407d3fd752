"""Table stride sweep (h = 0.1, 0.01, 0.001 on [0, 0.7), tail stride 0.1 to
1.5): at every stride the GPU's compressed FP64 path equals the oracle's
tabulated mode, and the table's error against the untabulated network
shrinks with h as the quintic interpolation predicts (sixth order, down to
rounding)."""
import numpy as np
import pytest

import oracle
import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

STRIDES = (0.1, 0.01, 0.001)
_err = {}


@pytest.fixture(scope="module")
def P():
    import paper_2201_01446_amd as P
    assert torch.cuda.is_available()
    return P


@pytest.fixture(scope="module")
def cell(cu_cfg, cu_params):
    x, box = synth.copper(5, 0.05, synth.SEED_CFG[1])
    return x, box, oracle.evaluate(cu_cfg, cu_params, x, box)


def gpu_eval(P, model, x, box, precision):
    xd = torch.tensor(x, dtype=torch.float64, device="cuda")
    nl = P.NeighborList(model, xd, box, skin=2.0)
    out = P.compute(model, nl, xd, precision=precision)
    torch.cuda.synchronize()
    return {k: v.cpu().numpy() for k, v in out.items() if v is not None}


@pytest.mark.parametrize("h", STRIDES)
def test_stride_gpu_vs_oracle(P, cu_cfg, cu_params, cell, h):
    x, box, ref = cell
    m = P.Model(cu_cfg, cu_params).tabulate(0.7, h, 1.5, 0.1)
    tab = oracle.Table(cu_cfg, cu_params, 0.7, h, 1.5, 0.1)
    rtab = oracle.evaluate(cu_cfg, cu_params, x, box, table=tab)
    got = gpu_eval(P, m, x, box, P.FP64)
    assert abs(got["E"][0] - rtab["E"]) <= 1e-10 * abs(rtab["E"])
    assert np.max(np.abs(got["F"] - rtab["F"])) <= 1e-10 * np.max(np.abs(rtab["F"]))
    assert np.max(np.abs(got["W"] - rtab["W"])) <= 1e-10 * np.max(np.abs(rtab["W"]))
    n = len(x)
    eE = abs(got["E"][0] - ref["E"]) / n
    eF = float(np.sqrt(np.mean((got["F"] - ref["F"]) ** 2)))
    _err[h] = (eE, eF)
    # FP32 at this stride within the FP32 bounds of the table it uses
    g32 = gpu_eval(P, m, x, box, P.FP32)
    assert abs(g32["E"][0] - rtab["E"]) / n <= 1e-5
    assert np.sqrt(np.mean((g32["F"] - rtab["F"]) ** 2)) <= 1e-4 * np.sqrt(np.mean(rtab["F"] ** 2))
    print(f"h={h}: {tab.coef.shape[0]} intervals, vs untabulated net dE/N {eE:.3g} eV, RMSE_F {eF:.3g} eV/A")


def test_stride_error_order():
    """Ten times finer stride, ~1e6 times smaller table error, until the
    FP64 rounding floor of the energy sum."""
    if len(_err) < 3:
        pytest.skip("needs the three stride runs")
    floor_e, floor_f = 1e-14, 1e-16
    (e1, f1), (e2, f2), (e3, f3) = (_err[h] for h in STRIDES)
    assert e1 > 1e3 * max(e2, floor_e) or e2 <= floor_e
    assert f1 > 1e3 * max(f2, floor_f) or f2 <= floor_f
    assert e3 <= max(10 * e2, floor_e) and f3 <= max(10 * f2, floor_f)
