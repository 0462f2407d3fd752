"""dp_compute_noalloc (the entry point for callers that cannot allocate)
against dp_compute, through the C-ABI.

Both run the same kernels on the same rows in the same order; only the
scratch differs (the library's static device array against the list's own),
so every result must be bit-identical, which is tighter than the oracle
tolerances of the parity tests.  Two calls in a row, the second with fewer
atoms, so the second call's scratch layout overlaps what the first left
behind.  Sizes past the static scratch and the plain modes are refused
before anything is enqueued.
"""
import ctypes

import numpy as np
import pytest

import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def P():
    import paper_2201_01446_amd as P
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return P


def dev(a, dtype=torch.float64):
    return torch.tensor(np.ascontiguousarray(a), dtype=dtype, device="cuda")


def vp(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def call(P, fn, model, nl, x, box, precision, mode=0):
    """One evaluation through the C-ABI into fresh outputs (NaN-filled, so
    an output the call did not write shows up)."""
    from paper_2201_01446_amd import _lib
    n = x.shape[0]
    out = dict(E=torch.full((1,), np.nan, dtype=torch.float64, device="cuda"),
               F=torch.full((n, 3), np.nan, dtype=torch.float64, device="cuda"),
               W=torch.full((3, 3), np.nan, dtype=torch.float64, device="cuda"),
               e_atom=torch.full((n,), np.nan, dtype=torch.float64, device="cuda"))
    b = None if box is None else np.ascontiguousarray(np.asarray(box, dtype=np.float64).reshape(9))
    bp = None if b is None else b.ctypes.data_as(ctypes.c_void_p)
    st = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    status = fn(model.h, nl.h, n, vp(x), None, bp, mode, precision, vp(out["E"]), vp(out["F"]), vp(out["W"]),
                vp(out["e_atom"]), st)
    torch.cuda.synchronize()
    if status != 0:
        raise P.DPError(status, _lib.lib.dp_last_error().decode())
    return {k: v.cpu().numpy() for k, v in out.items()}


def same(a, b, what):
    for k in ("E", "F", "W", "e_atom"):
        assert np.all(np.isfinite(a[k])), (what, k)
        assert np.array_equal(a[k], b[k]), (what, k, float(np.max(np.abs(a[k] - b[k]))))


@pytest.mark.parametrize("precision", [0, 1, 2])
def test_noalloc_equals_compute_copper(P, cu_cfg, cu_params, precision):
    from paper_2201_01446_amd import _lib
    model = P.Model(cu_cfg, cu_params).tabulate(0.7, 0.01, 1.5, 0.1)
    # a larger call, then a smaller one over what the first left in the scratch
    for ncell, seed in ((5, 11), (3, 12)):
        x, box = synth.copper(ncell, 0.05, seed)
        print(f"noalloc copper: {len(x)} atoms, precision {precision}", flush=True)
        xd = dev(x)
        nl = P.NeighborList(model, xd, box)
        ref = call(P, _lib.lib.dp_compute, model, nl, xd, box, precision)
        got = call(P, _lib.lib.dp_compute_noalloc, model, nl, xd, box, precision)
        same(got, ref, (len(x), precision))
        # and again after dp_compute has run on the list's own scratch
        again = call(P, _lib.lib.dp_compute_noalloc, model, nl, xd, box, precision)
        same(again, ref, (len(x), precision, "repeat"))


@pytest.mark.parametrize("mode", [3, 4])
def test_noalloc_per_neighbor_modes(P, cu_cfg, cu_params, mode):
    from paper_2201_01446_amd import _lib
    model = P.Model(cu_cfg, cu_params).tabulate(0.7, 0.01, 1.5, 0.1)
    x, box = synth.copper(3, 0.05, 13)
    print(f"noalloc mode {mode}: {len(x)} atoms", flush=True)
    xd = dev(x)
    nl = P.NeighborList(model, xd, box)
    same(call(P, _lib.lib.dp_compute_noalloc, model, nl, xd, box, 0, mode),
         call(P, _lib.lib.dp_compute, model, nl, xd, box, 0, mode), ("mode", mode))


def test_noalloc_two_types(P):
    """Rows grouped by center type (each group padded to a GEMM tile)."""
    from paper_2201_01446_amd import _lib
    cfg = synth.water_model_config()
    params = synth.model_params(cfg)
    model = P.Model(cfg, params).tabulate(0.7, 0.01, 1.5, 0.1)
    # 1,536 atoms fit the scratch in FP32 (not in FP64); then 192 atoms
    for nrep, precision in ((2, 1), (1, 0), (1, 1)):
        x, t, box = synth.water(nrep, 0.05)
        print(f"noalloc water: {len(x)} atoms, precision {precision}", flush=True)
        xd = dev(x)
        nl = P.NeighborList(model, xd, box, types=dev(t, torch.int32))
        same(call(P, _lib.lib.dp_compute_noalloc, model, nl, xd, box, precision),
             call(P, _lib.lib.dp_compute, model, nl, xd, box, precision), ("water", len(x), precision))


def test_noalloc_refusals(P, cu_cfg, cu_params):
    """Too large for the static scratch, or a plain mode: refused with the
    documented status, and a following call still works."""
    from paper_2201_01446_amd import _lib
    model = P.Model(cu_cfg, cu_params).tabulate(0.7, 0.01, 1.5, 0.1)
    x, box = synth.copper(8, 0.05, 14)   # 2,048 atoms: more than the 96 MiB scratch holds in FP64
    print(f"noalloc refusals: {len(x)} atoms", flush=True)
    xd = dev(x)
    nl = P.NeighborList(model, xd, box)
    with pytest.raises(P.DPError) as e:
        call(P, _lib.lib.dp_compute_noalloc, model, nl, xd, box, 0)
    assert e.value.status == -4 and "scratch" in str(e.value)
    xs, boxs = synth.copper(3, 0.05, 14)
    xsd = dev(xs)
    nls = P.NeighborList(model, xsd, boxs)
    with pytest.raises(P.DPError) as e:
        call(P, _lib.lib.dp_compute_noalloc, model, nls, xsd, boxs, 0, mode=1)
    assert e.value.status == -5
    same(call(P, _lib.lib.dp_compute_noalloc, model, nls, xsd, boxs, 0),
         call(P, _lib.lib.dp_compute, model, nls, xsd, boxs, 0), "after refusals")
