"""The cut-out oracle evaluation used for large cells equals the oracle on
the whole periodic cell."""
import numpy as np

import oracle
import synth
from sampling import LocalSampler


def test_cutouts_match_whole_cell(cu_cfg, cu_params):
    x, box = synth.copper(10, 0.1, 77)            # L = 36.3 A > 4 rcut + 1
    tab = oracle.Table(cu_cfg, cu_params, 0.7, 0.01, 1.5, 0.1)
    ref = oracle.evaluate(cu_cfg, cu_params, x, box, table=tab)
    s = LocalSampler(cu_cfg, cu_params, tab, x, box)
    for k in (0, 1234, 3999):
        assert abs(s.energy(k) - ref["e_atom"][k]) <= 1e-12 * abs(ref["e_atom"][k])
        np.testing.assert_allclose(s.force(k), ref["F"][k], rtol=0, atol=1e-12 * np.max(np.abs(ref["F"])))


def test_cutouts_match_whole_cell_two_types():
    cfg = synth.water_model_config()
    params = synth.model_params(cfg)
    x, t, box = synth.water(3, sigma=0.05)        # L = 37.3 A > 4 rcut + 1
    tab = oracle.Table(cfg, params, 0.7, 0.01, 1.5, 0.1)
    ref = oracle.evaluate(cfg, params, x, box, table=tab, types=t)
    s = LocalSampler(cfg, params, tab, x, box, types=t)
    for k in (0, 1, 2000, 5183):
        assert abs(s.energy(k) - ref["e_atom"][k]) <= 1e-12 * abs(ref["e_atom"][k])
        np.testing.assert_allclose(s.force(k), ref["F"][k], rtol=0, atol=1e-12 * np.max(np.abs(ref["F"])))
