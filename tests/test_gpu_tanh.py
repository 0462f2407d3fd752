"""Tabulated tanh in the fitting net (FP32 and mixed modes): the GPU equals
the oracle's tabulated-tanh mode within the mode's bounds, FP64 keeps the
native tanh, and switching back restores the native results."""
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


def gpu_eval(P, model, x, box, precision):
    xd = torch.tensor(x, dtype=torch.float64, device="cuda")
    nl = P.NeighborList(model, xd, box, skin=2.0)
    out = P.compute(model, nl, xd, precision=precision)
    torch.cuda.synchronize()
    return {k: v.cpu().numpy() for k, v in out.items() if v is not None}


def test_tanh_table_vs_oracle(P, cu_cfg, cu_params):
    x, box = synth.copper(5, 0.05, synth.SEED_CFG[1])
    tab = oracle.Table(cu_cfg, cu_params, *TAB)
    ref_t = oracle.evaluate(dict(cu_cfg, tanh_table=1), cu_params, x, box, table=tab)
    ref_n = oracle.evaluate(cu_cfg, cu_params, x, box, table=tab)
    m = P.Model(cu_cfg, cu_params).tabulate(*TAB).fitting_tanh(True)
    n = len(x)
    Fs = np.sqrt(np.mean(ref_t["F"] ** 2))
    for prec, tol_f in ((P.FP32, 1e-4), (P.MIXED_BF16, 1e-3)):
        g = gpu_eval(P, m, x, box, prec)
        dE = abs(g["E"][0] - ref_t["E"]) / n
        eF = np.sqrt(np.mean((g["F"] - ref_t["F"]) ** 2))
        print(f"tanh table prec {prec}: dE/N {dE:.3g} RMSE_F {eF:.3g}; table effect "
              f"{abs(ref_t['E'] - ref_n['E']) / n:.3g} eV/atom")
        assert dE <= 1e-5 and eF <= min(1e-3, tol_f * Fs)
    g64 = gpu_eval(P, m, x, box, P.FP64)      # FP64 keeps tanh
    assert abs(g64["E"][0] - ref_n["E"]) <= 1e-10 * abs(ref_n["E"])
    m.fitting_tanh(False)
    g32 = gpu_eval(P, m, x, box, P.FP32)
    assert abs(g32["E"][0] - ref_n["E"]) / n <= 1e-5
    assert np.sqrt(np.mean((g32["F"] - ref_n["F"]) ** 2)) <= 1e-4 * Fs
