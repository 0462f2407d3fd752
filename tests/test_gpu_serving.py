"""Batched evaluation of many independent cells (the serving path) through
the C-ABI: each request's result inside a mixed batch equals its result
alone and the oracle's; the continuous-batching server returns the same
results under closed-loop and Poisson arrivals."""
import numpy as np
import pytest

import oracle
import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

S_MAX, H, TAIL, H_TAIL = 0.7, 0.01, 1.5, 0.1


@pytest.fixture(scope="module")
def P():
    import paper_2201_01446_amd as P
    assert torch.cuda.is_available()
    return P


@pytest.fixture(scope="module")
def model(P, cu_cfg, cu_params):
    m = P.Model(cu_cfg, cu_params).tabulate(S_MAX, H, TAIL, H_TAIL)
    torch.cuda.synchronize()
    return m


@pytest.fixture(scope="module")
def table(cu_cfg, cu_params):
    return oracle.Table(cu_cfg, cu_params, S_MAX, H, TAIL, H_TAIL)


def mixed_requests(seed, sizes, open_cluster=True):
    """Periodic cells of the given sizes plus, optionally, an open 55-atom
    cluster (a displaced FCC fragment far from the origin)."""
    rng = np.random.default_rng(seed)
    reqs = [synth.serving_request(rng, n)[:2] for n in sizes]
    if open_cluster:
        xc, _ = synth.copper(3, 0.1, seed)
        reqs.insert(1, (np.ascontiguousarray(xc[:55] + 30.0), None))
    return reqs


def run_batch(P, model, reqs, precision, batch=None):
    from paper_2201_01446_amd.serve import Batch
    if batch is None:
        batch = Batch(model, sum(len(x) for x, _ in reqs) + 64, 64)
    X = torch.tensor(np.concatenate([x for x, _ in reqs]), dtype=torch.float64, device="cuda")
    out = batch.compute([(len(x), box) for x, box in reqs], X, precision)
    torch.cuda.synchronize()
    E, F, W = (out[k].cpu().numpy() for k in ("E", "F", "W"))
    res, off = [], 0
    for k, (x, _) in enumerate(reqs):
        res.append(dict(E=E[k], F=F[off:off + len(x)], W=W[k]))
        off += len(x)
    return res, batch


def test_batch_fp64_vs_oracle_and_alone(P, model, cu_cfg, cu_params, table):
    """FP64: every request of a mixed batch (32..1500 atoms, one open
    cluster) equals the tabulated oracle and its own result computed alone."""
    reqs = mixed_requests(21, [32, 300, 1500, 90, 700])
    mix, batch = run_batch(P, model, reqs, P.FP64)
    for k, (x, box) in enumerate(reqs):
        ref = oracle.evaluate(cu_cfg, cu_params, x, box, table=table)
        r = mix[k]
        Fs, Ws = np.max(np.abs(ref["F"])), np.max(np.abs(ref["W"]))
        print(f"req {k} ({len(x)} atoms, {'open' if box is None else 'periodic'}): "
              f"dE/N {abs(r['E'] - ref['E']) / len(x):.3g} max dF {np.max(np.abs(r['F'] - ref['F'])):.3g}")
        assert abs(r["E"] - ref["E"]) <= 1e-10 * abs(ref["E"])
        assert np.max(np.abs(r["F"] - ref["F"])) <= 1e-10 * Fs
        assert np.max(np.abs(r["W"] - ref["W"])) <= 1e-10 * Ws
        # every sum over a request runs in an order fixed by the request itself
        # (forces are gathered, not scattered): alone and in the mix agree exactly
        alone, _ = run_batch(P, model, [(x, box)], P.FP64, batch=batch)
        assert alone[0]["E"] == r["E"]
        np.testing.assert_array_equal(alone[0]["F"], r["F"])
        np.testing.assert_array_equal(alone[0]["W"], r["W"])
    st = batch.stats()
    assert st["sel_overflow"] == 0 and st["cap_overflow"] == 0


@pytest.mark.parametrize("prec,tol_e,tol_f", [(1, 1e-5, 1e-4), (2, 1e-5, 1e-3)])
def test_batch_reduced_precision_vs_oracle(P, model, cu_cfg, cu_params, table, prec, tol_e, tol_f):
    """FP32 and mixed BF16: the bounds of the single-cell tests, per request."""
    reqs = mixed_requests(22, [40, 500, 2500])
    mix, _ = run_batch(P, model, reqs, prec)
    for k, (x, box) in enumerate(reqs):
        ref = oracle.evaluate(cu_cfg, cu_params, x, box, table=table)
        Fs = np.sqrt(np.mean(ref["F"] ** 2))
        eF = np.sqrt(np.mean((mix[k]["F"] - ref["F"]) ** 2))
        dE = abs(mix[k]["E"] - ref["E"]) / len(x)
        print(f"prec {prec} req {k} ({len(x)}): dE/N {dE:.3g} RMSE_F {eF:.3g} (F_rms {Fs:.3g})")
        assert dE <= tol_e
        assert eF <= 1e-3 and eF <= tol_f * Fs


def test_batch_large_request_sampled(P, model, cu_cfg, cu_params, table):
    """A 20,000-atom request beside small ones: E_i and forces at sampled
    atoms against the oracle (FP32)."""
    reqs = mixed_requests(23, [20000, 64], open_cluster=False)
    X = torch.tensor(np.concatenate([x for x, _ in reqs]), dtype=torch.float64, device="cuda")
    from paper_2201_01446_amd.serve import Batch
    b = Batch(model, len(X), 8)
    out = b.compute([(len(x), box) for x, box in reqs], X, P.FP32)
    torch.cuda.synchronize()
    F = out["F"].cpu().numpy()
    x, box = reqs[0]
    rng = np.random.default_rng(7)
    for k in rng.choice(len(x), 3, replace=False):
        j, _, _, _ = oracle.neighbors(cu_cfg, x, box, int(k))
        cen = np.unique(np.concatenate([[k], j])).astype(np.int32)
        Fk = oracle.evaluate(cu_cfg, cu_params, x, box, table=table, centers=cen)["F"][k]
        assert np.max(np.abs(F[k] - Fk)) <= 1e-4 * np.max(np.abs(Fk)) + 1e-9
    # the second request starts right after the first: its rows are its own
    ref = oracle.evaluate(cu_cfg, cu_params, reqs[1][0], reqs[1][1], table=table)
    assert np.sqrt(np.mean((F[len(x):] - ref["F"]) ** 2)) <= 1e-4 * np.sqrt(np.mean(ref["F"] ** 2))


def test_batch_argument_errors(P, model):
    """Host-side checks: capacity and layout errors are reported, not run."""
    from paper_2201_01446_amd._lib import DPError
    from paper_2201_01446_amd.serve import Batch
    b = Batch(model, 200, 2)
    reqs = mixed_requests(24, [100, 100, 100], open_cluster=False)
    X = torch.zeros((sum(len(x) for x, _ in reqs), 3), dtype=torch.float64, device="cuda")
    with pytest.raises(DPError, match="CAPACITY"):
        b.compute([(len(x), box) for x, box in reqs], X, P.FP32)     # 3 requests > 2
    big = mixed_requests(25, [300], open_cluster=False)
    Xb = torch.zeros((len(big[0][0]), 3), dtype=torch.float64, device="cuda")
    with pytest.raises(DPError, match="CAPACITY"):
        b.compute([(len(x), box) for x, box in big], Xb, P.FP32)      # more atoms than max_atoms
    thin = np.eye(3).reshape(9) * np.array([4.0, 1, 1, 1, 30.0, 1, 1, 1, 30.0])
    with pytest.raises(DPError, match="UNSUPPORTED"):
        b.compute([(10, thin.reshape(3, 3))], X, P.FP32)              # box edge < (rc + skin) / 2


def test_server_closed_loop_and_poisson(P, model):
    """The server's results equal each request computed alone, bit for bit
    (FP32), with several batches in flight."""
    from paper_2201_01446_amd.serve import Server, poisson_arrivals
    reqs = [r[:2] for r in synth.serving_stream(24, 32, 3000, seed=synth.SEED_SERVING)]
    srv = Server(model, P.FP32, slots=3, hbm_budget=3 * 400 << 20)
    assert srv.slot_atoms >= 3000
    res, st = srv.run(reqs)
    print("closed loop:", st)
    assert st["batches"] >= 3
    for k in range(len(reqs)):
        alone, _ = run_batch(P, model, [reqs[k]], P.FP32)
        r, a = res[k], alone[0]
        assert r["E"] == a["E"]
        np.testing.assert_array_equal(r["F"], a["F"])
        np.testing.assert_array_equal(r["W"], a["W"])
    rate = 0.7 * len(reqs) / st["wall_s"]
    res2, st2 = srv.run(reqs, poisson_arrivals(len(reqs), rate, seed=3))
    print("poisson:", st2)
    for k in range(len(reqs)):
        assert res2[k]["E"] == res[k]["E"]
        np.testing.assert_array_equal(res2[k]["F"], res[k]["F"])
    assert st2["p99_ms"] >= st2["p50_ms"] > 0
    # a cap on the atoms per batch: smaller batches (a request above the cap
    # alone), the same results
    sizes = [len(x) for x, _ in reqs]
    res3, st3 = srv.run(reqs, max_batch_atoms=2000)
    print("capped:", st3)
    assert st3["batches"] > st["batches"]
    assert st3["mean_batch_atoms"] <= max(2000, max(sizes))
    for k in range(len(reqs)):
        assert res3[k]["E"] == res[k]["E"]
        np.testing.assert_array_equal(res3[k]["F"], res[k]["F"])


def test_server_rejects_oversize_request_alone(P, model):
    """A request larger than every slot is answered with an error of its own;
    the requests around it are served, with the results they have alone, and
    the latency split (wait for a slot + service) adds up."""
    from paper_2201_01446_amd.serve import Server
    reqs = [r[:2] for r in synth.serving_stream(8, 32, 1500, seed=synth.SEED_SERVING + 7)]
    srv = Server(model, P.FP32, slots=2, hbm_budget=2 * 200 << 20)
    big = synth.copper(10, 0.05, 5)   # 4,000 atoms
    assert srv.slot_atoms < 4000 and max(x.shape[0] for x, _ in reqs) <= srv.slot_atoms
    reqs.insert(3, big)
    res, st = srv.run(reqs)
    print("with an oversize request:", st)
    assert st["rejected"] == 1 and "exceed" in res[3]["error"]
    assert st["atoms"] == sum(x.shape[0] for x, _ in reqs) - 4000
    for k in (0, 4, len(reqs) - 1):
        alone, _ = run_batch(P, model, [reqs[k]], P.FP32)
        assert res[k]["E"] == alone[0]["E"]
        np.testing.assert_array_equal(res[k]["F"], alone[0]["F"])
    assert abs(st["mean_wait_ms"] + st["mean_service_ms"] - st["mean_ms"]) <= 1e-6 * st["mean_ms"]
    assert st["tail_wait_ms"] >= 0 and st["tail_service_ms"] > 0
