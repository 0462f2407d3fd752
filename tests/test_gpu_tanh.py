"""Tabulated tanh in the fitting net (the second-order table of Sec. 3.5).

Each check here fails when the device ignores the table: the table itself
is compared with the oracle's construction at every node and mid-interval
(to 1e-14, while the table and tanh differ by up to 2.4e-8 inside the range),
and the FP64 force step with the table on is held to the oracle's
tabulated-tanh mode at the FP64 bounds, which the native-tanh results miss by
a wide margin (asserted, so the test shows that it discriminates).  The FP32
and mixed modes are held to the oracle's tabulated mode within their own
bounds, and switching the table off restores the native results."""
import numpy as np
import pytest

import oracle
import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TAB = (0.7, 0.01, 1.5, 0.1)
H = 1.0 / 128.0


@pytest.fixture(scope="module")
def P():
    import paper_2201_01446_amd as P
    assert torch.cuda.is_available()
    return P


def gpu_eval(P, model, x, box, precision):
    xd = torch.tensor(x, dtype=torch.float64, device="cuda")
    nl = P.NeighborList(model, xd, box, skin=2.0)
    out = P.compute(model, nl, xd, precision=precision, atom_energy=True)
    torch.cuda.synchronize()
    return {k: v.cpu().numpy() for k, v in out.items() if v is not None}


def fp64_misfit(got, ref):
    """Largest error of E_i, F and W, each over the FP64 bound of the parity
    tests (1e-10 of the scale of the oracle's values): <= 1 passes."""
    Es = max(float(np.max(np.abs(ref["e_atom"]))), 1.0)
    Fs = float(np.max(np.abs(ref["F"])))
    Ws = float(np.max(np.abs(ref["W"])))
    return max(float(np.max(np.abs(got["e_atom"] - ref["e_atom"]))) / (1e-10 * Es),
               float(np.max(np.abs(got["F"] - ref["F"]))) / (1e-10 * Fs),
               float(np.max(np.abs(got["W"] - ref["W"]))) / (1e-10 * Ws))


def test_tanh_table_coefficients(P, cu_cfg, cu_params):
    """The device's FP64 table against the oracle's tabulated tanh at every
    node and every mid-interval of [0, 8)."""
    m = P.Model(cu_cfg, cu_params).fitting_tanh(True)
    a = m.tanh_table()
    assert a.shape == (1024, 4) and np.all(a[:, 3] == 0.0)
    x0 = np.arange(1024) * H
    t = 0.5 * H
    y_mid = a[:, 0] + t * (a[:, 1] + t * a[:, 2])
    ref_node = oracle.tanh_table(x0)
    ref_mid = oracle.tanh_table(x0 + t)
    err = max(float(np.max(np.abs(a[:, 0] - ref_node))), float(np.max(np.abs(y_mid - ref_mid))))
    gap = float(np.max(np.abs(ref_mid - np.tanh(x0 + t))))   # the table's own error
    print(f"tanh table: max error vs oracle {err:.3g}; table vs tanh at mid-intervals {gap:.3g}")
    assert err <= 1e-14
    assert gap >= 1e-8   # a device tanh in place of the table would fail the bound above
    # the slope at each node is tanh's: a1 = 1 - a0^2
    np.testing.assert_allclose(a[:, 1], 1.0 - a[:, 0] ** 2, rtol=0, atol=1e-15)


def test_tanh_table_fp64_discriminates(P, cu_cfg, cu_params):
    """FP64, 500-atom copper: with the table on the GPU equals the oracle's
    tabulated-tanh mode at the FP64 bounds, and misses the native-tanh oracle
    by more than 10 times those bounds (with the table off it is the other
    way round)."""
    x, box = synth.copper(5, 0.05, synth.SEED_CFG[1])
    tab = oracle.Table(cu_cfg, cu_params, *TAB)
    ref_t = oracle.evaluate(dict(cu_cfg, tanh_table=1), cu_params, x, box, table=tab)
    ref_n = oracle.evaluate(cu_cfg, cu_params, x, box, table=tab)
    m = P.Model(cu_cfg, cu_params).tabulate(*TAB).fitting_tanh(True)
    g = gpu_eval(P, m, x, box, P.FP64)
    on_t, on_n = fp64_misfit(g, ref_t), fp64_misfit(g, ref_n)
    m.fitting_tanh(False)
    g = gpu_eval(P, m, x, box, P.FP64)
    off_t, off_n = fp64_misfit(g, ref_t), fp64_misfit(g, ref_n)
    print(f"FP64 misfit / bound: table on: vs tabulated {on_t:.3g}, vs native {on_n:.3g}; "
          f"table off: vs tabulated {off_t:.3g}, vs native {off_n:.3g}")
    assert on_t <= 1.0 and on_n >= 10.0
    assert off_n <= 1.0 and off_t >= 10.0


def test_tanh_table_fp32_mixed_vs_oracle(P, cu_cfg, cu_params):
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
    m.fitting_tanh(False)
    g32 = gpu_eval(P, m, x, box, P.FP32)
    assert abs(g32["E"][0] - ref_n["E"]) / n <= 1e-5
    assert np.sqrt(np.mean((g32["F"] - ref_n["F"]) ** 2)) <= 1e-4 * Fs
