"""Benchmark of the compressed Deep Potential MD step on one MI355X.

Workload: 108,000-atom FCC copper (30x30x30 cells, a = 3.634 A, Gaussian
displacements sigma = 0.05 A), seeded random weights of the copper model
(embedding 32-64-128, fitting 240-240-240, rcut 8 A, sel 192), velocity
Verlet NVE at dt = 1 fs, neighbor list (2 A skin) rebuilt every 10 steps.
One step = half kick + drift (+ rebuild) + energy/forces/virial + half kick.

    python bench.py [--gpus 1] [--steps 100] [--warmup 10]

Prints one JSON line: atom-steps/s of the FP64 compressed path (value: the
paper's arithmetic), the FP32 and mixed-precision paths and the plain
(untabulated) path beside it, per-kernel times from HIP events recorded on
the launch stream, the roofline of each path's dominant kernel, the
1,048,576-atom mixed-precision run and the 500,000-atom autograd step, and
the FP64 CPU oracle on the host cores: its rate (the CPU baseline) and its
values at sampled atoms of every timed run's final configuration (the
accuracy gate: force RMSE and energy error per atom).
"""
import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK = {  # MI355X published peaks, TFLOP/s (dense)
    ("alu", "f32"): 157.3, ("alu", "f64"): 78.6,
    ("mfma", "f32"): 157.3, ("mfma", "f64"): 78.6, ("mfma", "bf16"): 2500.0,
}
HBM_PEAK_GBS = 8000.0
COUNTERS = os.path.join(ROOT, "profiles", "hbm_counters.json")


def _kernel_sources_digest():
    """Digest of every kernel source (csrc/*.hip, csrc/*.h, in name order)."""
    import glob
    import hashlib
    h = hashlib.sha256()
    for f in sorted(glob.glob(os.path.join(ROOT, "paper_2201_01446_amd", "csrc", "*.hip")) +
                    glob.glob(os.path.join(ROOT, "paper_2201_01446_amd", "csrc", "*.h"))):
        with open(f, "rb") as fh:
            h.update(os.path.basename(f).encode())
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(kernel, dt):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 counter
    summary (FETCH_SIZE and WRITE_SIZE, each scaled by the same counter's
    reading for an elementwise kernel of known size), or None when there is
    none or the kernel sources changed after it was taken."""
    try:
        with open(COUNTERS) as fh:
            rec = json.load(fh)
    except (OSError, ValueError):
        return None
    k = rec.get("kernels", {}).get(f"{kernel}_{dt}")
    if k is None or rec.get("sources_digest") != _kernel_sources_digest():
        return None
    return round(k["fetch_kib"] * rec["fetch_scale"] * 1024 + k["write_kib"] * rec["write_scale"] * 1024)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--ncell", type=int, default=30)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle leg (baseline and accuracy gate)")
    ap.add_argument("--no-reduced", action="store_true", help="FP64 only (no FP32 and mixed legs)")
    ap.add_argument("--cpu-samples", type=int, default=512,
                    help="oracle energies sampled per FP64 run (forces: one eighth; other runs half of each)")
    ap.add_argument("--no-big", action="store_true", help="skip the 1,048,576-atom mixed-precision run")
    ap.add_argument("--big-ncell", type=int, default=64)
    ap.add_argument("--big-steps", type=int, default=50)
    ap.add_argument("--no-autograd", action="store_true", help="skip the 500,000-atom autograd timing")
    ap.add_argument("--grad-ncell", type=int, default=50)
    ap.add_argument("--grad-iters", type=int, default=10)
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--plain-steps", type=int, default=10)
    ap.add_argument("--serve-requests", type=int, default=4096)
    ap.add_argument("--no-serve", action="store_true")
    ap.add_argument("--no-strides", action="store_true", help="skip the table-stride sweep")
    ap.add_argument("--no-ablation", action="store_true", help="skip the optimization ladder")
    ap.add_argument("--no-tanh", action="store_true", help="skip the tabulated-tanh comparison")
    ap.add_argument("--no-water", action="store_true", help="skip the two-type water system")
    ap.add_argument("--water-rep", type=int, default=8, help="replicas per edge of the 192-atom water cell")
    ap.add_argument("--water-only", action="store_true",
                    help="run only the water section (--steps timed steps) and print it (for profiling)")
    ap.add_argument("--ablation-steps", type=int, default=10)
    ap.add_argument("--rebuild-every", type=int, default=10,
                    help="neighbor-list rebuild cadence in steps (the workload's is 10)")
    ap.add_argument("--stride-steps", type=int, default=20)
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="first run one elementwise negation over this many MiB (reads and writes it once): "
                         "the calibration of HBM byte counters")
    return ap.parse_args()


# neighbor-list rebuild cadence (the paper updates its list with a 2 A buffer
# every 50 steps; here every 10: the interval-run kernels are fastest on a
# freshly sorted list, and 10 to 20 steps balance that against the rebuild)
REBUILD = 10


def run_nve(P, model, x0, v0, box, steps, warmup, precision, mode=0, keep=False, types=None, mass=63.546, dt=1.0):
    rebuild = REBUILD
    import torch
    x = torch.tensor(x0, dtype=torch.float64, device="cuda")
    v = torch.tensor(v0, dtype=torch.float64, device="cuda")
    td = None if types is None else torch.tensor(types, dtype=torch.int32, device="cuda")
    nl = P.NeighborList(model, x, box, skin=2.0, types=td)
    if warmup:
        P.nve_run(model, nl, x, v, box, mass, dt, warmup, rebuild_every=rebuild, precision=precision, mode=mode, types=td)
    torch.cuda.synchronize()
    from paper_2201_01446_amd import _lib
    _lib.timers_read()
    _lib.timers_enable(True)
    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    wall0 = time.perf_counter()
    t0.record()
    if warmup:   # the timed steps continue the warm-up's trajectory (no set-up build and evaluation)
        th = P.nve_continue(model, nl, x, v, mass, dt, steps, rebuild_every=rebuild, precision=precision, mode=mode)
    else:
        th = P.nve_run(model, nl, x, v, box, mass, dt, steps, rebuild_every=rebuild, precision=precision, mode=mode,
                       types=td)
    t1.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - wall0
    _lib.timers_enable(False)
    kern = _lib.timers_read()
    ms = t0.elapsed_time(t1)
    out = dict(ms=ms, wall=wall, thermo=th.cpu().numpy(), kernels=kern)
    if keep:   # the list owns the scratch (tens of GB for the plain path): kept only on request
        out.update(x=x, nl=nl)
    return out


def kernel_work(N, sum_nei, sum_seg, rs, d_in_emb):
    """Algorithmic work per launch of each kernel (FMA = 2 FLOP) and its
    bound: the fitting GEMMs count the model's 240 columns (not the padded
    256) and one pass of K (not the BF16 hi/lo split's three); the embedding
    kernels count the interval-moment form they execute: forward 24 moments
    per neighbor, 24 per (segment, column), and D 16 x 128 x 4 where it forms
    D (d_in_emb: the mixed mode; in FP32 and FP64 the first fitting layer
    forms D from T, VALU work beside its MFMA product that is not counted);
    backward dE/dT 2 x 16 x 128 x 4, 24 per (segment, column), 40 per
    neighbor."""
    fit_in = N * 2.0 * 240 * 2048          # 2048 -> 240 (and its transpose)
    fit_hid = N * 2.0 * 240 * 240          # 240 -> 240
    return {
        "emb_fwd": (2.0 * (24 * sum_nei + 24 * 128 * sum_seg + (8192 * N if d_in_emb else 0)), "alu"),
        "emb_bwd": (2.0 * (16384 * N + 24 * 128 * sum_seg + 40 * sum_nei), "alu"),
        "fit_fwd1": (fit_in, "mfma"), "fit_bwd1": (fit_in, "mfma"),
        "fit_fwd2": (fit_hid, "mfma"), "fit_fwd3": (fit_hid, "mfma"),
        "fit_bwd3": (fit_hid, "mfma"), "fit_bwd2": (fit_hid, "mfma"),
        # the fused tail: the two 240 -> 240 layers and their two input-gradient products
        "fit_tail": (4 * fit_hid, "mfma"),
        "dT": (N * 3072.0 * rs, "hbm"),      # read dD (2048) and T (512), write dT (512)
    }


def roofline(res, steps, work, dt_alu, dt_mfma, counter_tag):
    """Per-kernel average launch time (HIP events on the launch stream),
    work, bound and fraction of the published peak; the dominant kernel (the
    largest time per step) is the roofline of the line.  VALU-bound rows also
    give the fraction of the unpacked FP32 rate (78.6 TFLOP/s), the most this
    build can issue (it compiles without packed FP32)."""
    table = {}
    for name, (tot_ms, cnt) in res["kernels"].items():
        avg = tot_ms / max(cnt, 1)
        row = dict(avg_ms=round(avg, 4), launches_per_step=round(cnt / steps, 3))
        if name in work:
            w, bound = work[name]
            if bound == "hbm":
                ach, peak, unit = w / (avg * 1e-3) / 1e9, HBM_PEAK_GBS, "GB/s"
            else:
                dt = dt_alu if bound == "alu" else dt_mfma
                ach, peak, unit = w / (avg * 1e-3) / 1e12, PEAK[(bound, dt)], "TFLOP/s"
            row.update(bound=bound, achieved=round(ach, 3), peak=peak, unit=unit, frac=round(ach / peak, 4))
            if bound == "alu" and dt_alu == "f32":
                row["frac_of_unpacked_78.6"] = round(ach / 78.6, 4)
        table[name] = row
    dom = max((n for n in table if "frac" in table[n]),
              key=lambda n: table[n]["avg_ms"] * table[n]["launches_per_step"])
    t = table[dom]
    roof = dict(bound=t["bound"], achieved=t["achieved"], peak=t["peak"], unit=t["unit"], frac=t["frac"],
                traffic=measured_traffic(dom, counter_tag), kernel=dom, per_launch_work=work[dom][0],
                avg_ms=t["avg_ms"])
    return roof, table


def final_state(P, model, res, precision):
    """E_i and forces of the run's final configuration (one more evaluation,
    outside the timed region), as host arrays for the accuracy gate."""
    import torch
    out = P.compute(model, res["nl"], res["x"], precision=precision, atom_energy=True)
    torch.cuda.synchronize()
    return dict(x=res["x"].cpu().numpy(), e_atom=out["e_atom"].cpu().numpy(), F=out["F"].cpu().numpy())


def main():
    args = parse()
    global REBUILD
    REBUILD = args.rebuild_every
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); the per-GPU share is the "
              "108,000-atom kernel measured at --gpus 1.", file=sys.stderr)
        sys.exit(2)
    import gc
    import torch

    import paper_2201_01446_amd as P
    import synth

    if args.water_only:
        print(json.dumps({"water": water(P, args.water_rep, args.steps, args.warmup)}))
        return
    if args.copy_probe_mib:
        a = torch.ones(args.copy_probe_mib << 18, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        torch.neg(a, out=b)
        torch.cuda.synchronize()
        del a, b
    cfg = synth.copper_model_config()
    params = synth.model_params(cfg)
    model = P.Model(cfg, params).tabulate(0.7, 0.01, 1.5, 0.1)
    x0, box = synth.copper(args.ncell, 0.05, synth.SEED_CFG[2])
    v0 = synth.maxwell_boltzmann(len(x0), 330.0)
    N = len(x0)
    K, W = args.steps, args.warmup

    # the headline: FP64, the paper's arithmetic; then FP32 and mixed beside it
    legs = [("fp64", P.FP64, "f64", "f64", 8)]
    if not args.no_reduced:
        legs += [("fp32", P.FP32, "f32", "f32", 4), ("mixed_bf16", P.MIXED_BF16, "f32", "bf16", 4)]
    runs, finals = {}, {}
    for name, prec, _, _, _ in legs:
        r = run_nve(P, model, x0, v0, box, K, W, prec, keep=True)
        finals[name] = final_state(P, model, r, prec)
        if name == "fp64":
            # neighbor statistics of the final configuration (for the work counts)
            d = P.descriptor(model, r["nl"], r["x"], precision=P.FP64)
            sum_nei = int(d["nnei"].sum().item())
            sum_seg = int(d["nseg"].sum().item())
            del d
        r.pop("nl")
        r.pop("x")
        runs[name] = r
        gc.collect()
    # the plain (untabulated, padded, materialised) path: same MD protocol,
    # fewer steps (it is the denominator of the speed-up)
    Kp = max(1, min(K, args.plain_steps))
    plain = {}
    if not args.no_plain:
        for name, prec in (("plain_fp64", P.FP64), ("plain_fp32", P.FP32)):
            if name == "plain_fp32" and args.no_reduced:
                continue
            plain[name] = run_nve(P, model, x0, v0, box, Kp, 1, prec, mode=P.PLAIN)
            gc.collect()

    summary = {}
    for name, prec, dt_alu, dt_mfma, rs in legs:
        r = runs[name]
        roof, per = roofline(r, K, kernel_work(N, sum_nei, sum_seg, rs, name == "mixed_bf16"), dt_alu, dt_mfma,
                             {"fp64": "f64", "fp32": "f32", "mixed_bf16": "bf16"}[name])
        th = r["thermo"]
        etot = th[:, 0] + th[:, 1]
        v = N * K / (r["ms"] * 1e-3)
        summary[name] = {"value": round(v, 1), "ms_per_step": round(r["ms"] / K, 4),
                         "ns_per_day": round(v / N * 86400 * 1e-6, 3), "roofline": roof, "kernels": per,
                         "energy_drift_eV_per_atom": float((etot[-1] - etot[0]) / N)}
    for name, r in plain.items():
        vp = N * Kp / (r["ms"] * 1e-3)
        comp = summary.get(name.replace("plain_", ""), {}).get("value")
        summary[name] = {"value": round(vp, 1), "ms_per_step": round(r["ms"] / Kp, 4), "steps": Kp,
                         "kernels": {k: round(t[0] / max(t[1], 1), 4) for k, t in r["kernels"].items()},
                         "speedup_compressed_vs_plain": round(comp / vp, 3) if comp else None}
        tag = "f64" if name.endswith("64") else "f32"
        tr = plain_traffic(r["kernels"], tag, Kp)
        if tr:
            summary[name]["roofline"] = tr
        sb = plain_step_bytes(tag)
        if sb:
            # the whole step against HBM: how slack this denominator is, and
            # the compressed path's advantage over a plain path at its bound
            bound_ms = sb / (HBM_PEAK_GBS * 1e9) * 1e3
            summary[name]["step_hbm_bytes"] = sb
            summary[name]["step_hbm_bound_ms"] = round(bound_ms, 3)
            summary[name]["frac_of_step_hbm_bound"] = round(bound_ms / (r["ms"] / Kp), 4)
            if comp:
                summary[name]["speedup_at_plain_hbm_bound"] = round(bound_ms / (N / comp * 1e3), 3)
    del runs, plain
    gc.collect()

    big = None if args.no_big else config_1m(P, model, args.big_ncell, args.big_steps)
    grad = None if args.no_autograd else config_autograd(P, model, args.grad_ncell, args.grad_iters)
    gc.collect()

    head = summary["fp64"]
    out = {
        "metric": "atom-steps/s on 1 GPU, compressed DP MD step (FP64), force RMSE <= 1e-3 eV/A",
        "value": head["value"],
        "unit": "atom-steps/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": W,
        "ms_per_step": head["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic: seeded FCC Cu + Gaussian displacements, seeded random weights",
        "config": {"workload": f"Cu FCC {args.ncell}^3 cells ({N} atoms), sigma 0.05 A, 330 K, NVE dt 1 fs, "
                               f"nlist skin 2 A rebuilt every {REBUILD} steps, compressed (stride 0.01, tail 0.1)",
                   "natoms": N, "precision": "fp64", "mode": "compressed"},
        "ns_per_day": head["ns_per_day"],
        "roofline": head["roofline"],
        "kernels_fp64": head["kernels"],
        "energy_drift_fp64_eV_per_atom": head["energy_drift_eV_per_atom"],
        "mean_neighbors": sum_nei / N,
        "mean_interval_segments": sum_seg / N,
    }
    for name in ("fp32", "mixed_bf16", "plain_fp64", "plain_fp32"):
        if name in summary:
            out[name] = summary[name]
    if big is not None:
        out["config_1m_mixed"] = {k: v for k, v in big.items() if k not in ("final", "box")}
    if grad is not None:
        out["config_autograd_500k"] = {k: v for k, v in grad.items() if k not in ("final", "box")}
    if not args.no_tanh:
        out["tanh_table"] = tanh_compare(P, cfg, params, x0, v0, box, min(K, 50))
    if not args.no_ablation:
        out["ablation"] = ablation(P, x0, v0, box, args.ablation_steps)
    if not args.no_strides:
        out["stride_sweep"] = stride_sweep(P, cfg, params, x0, v0, box, args.stride_steps)
    if not args.no_serve:
        out["serving"] = serving(P, model, args.serve_requests)
    if not args.no_water:
        out["water"] = water(P, args.water_rep, min(K, 50), W)
    if not args.no_cpu:
        # the oracle leg: its timing is the CPU baseline, and its values at
        # sampled atoms of each timed run's final configuration are the
        # accuracy gate of that run
        cases = {name: (finals[name], box) for name in finals}
        if big is not None:
            cases["config_1m_mixed"] = (big["final"], big["box"])
        if grad is not None:
            cases["config_autograd_500k"] = (grad["final"], grad["box"])
        cpu, gate = oracle_leg(cfg, params, cases, args.cpu_samples)
        out["cpu_baseline"] = cpu
        out["accuracy"] = gate
        for name, g in gate.items():
            tgt = out if name == "fp64" else out.get(name)
            if isinstance(tgt, dict):
                tgt["accuracy_gate_pass"] = g["pass"]
    print(json.dumps(out))


def plain_step_bytes(tag):
    """The plain path's HBM bytes per step from the committed counters (None
    when there are none for these sources)."""
    try:
        with open(COUNTERS) as fh:
            rec = json.load(fh)
    except (OSError, ValueError):
        return None
    if rec.get("sources_digest") != _kernel_sources_digest():
        return None
    return rec.get("plain_step_bytes", {}).get(tag)


def plain_traffic(kern, tag, steps):
    """HBM roofline of the plain path's dominant kernel from the committed
    counters (None when there are none for these sources)."""
    best = max(kern.items(), key=lambda kv: kv[1][0], default=None)
    if best is None:
        return None
    name, (tot, cnt) = best
    b = measured_traffic(name, tag)
    if b is None:
        return None
    avg = tot / max(cnt, 1)
    ach = b / (avg * 1e-3) / 1e9
    return dict(bound="hbm", achieved=round(ach, 1), peak=HBM_PEAK_GBS, unit="GB/s",
                frac=round(ach / HBM_PEAK_GBS, 4), traffic=b, kernel=name, avg_ms=round(avg, 4),
                launches_per_step=round(cnt / steps, 3))


def config_1m(P, model, ncell, steps):
    """The large mixed-precision run: 4 ncell^3 atoms of copper (64^3 cells:
    1,048,576 atoms), sigma 0.08 A, 330 K, 50 NVE steps in the mixed mode
    (FP32 table and contraction, BF16 fitting GEMMs, FP64 reductions and
    integration)."""
    import gc
    import synth
    x0, box = synth.copper(ncell, 0.08, synth.SEED_CFG[3])
    v0 = synth.maxwell_boltzmann(len(x0), 330.0, seed=synth.SEED_VELOCITY + 1)
    N = len(x0)
    r = run_nve(P, model, x0, v0, box, steps, 2, P.MIXED_BF16, keep=True)
    fin = final_state(P, model, r, P.MIXED_BF16)
    st = r["nl"].stats()
    th = r["thermo"]
    etot = th[:, 0] + th[:, 1]
    v = N * steps / (r["ms"] * 1e-3)
    out = {"workload": f"Cu FCC {ncell}^3 cells ({N} atoms), sigma 0.08 A, 330 K, NVE dt 1 fs, nlist skin 2 A "
                       "rebuilt every 10 steps, mixed precision (BF16 fitting GEMMs)",
           "natoms": N, "steps": steps, "value": round(v, 1), "unit": "atom-steps/s",
           "ms_per_step": round(r["ms"] / steps, 4), "ns_per_day": round(v / N * 86400 * 1e-6, 3),
           "energy_drift_eV_per_atom": float((etot[-1] - etot[0]) / N), "table_oob": st["table_oob"],
           "sel_overflow": st["sel_overflow"],
           "kernels": {k: round(t[0] / max(t[1], 1), 4) for k, t in r["kernels"].items()},
           "final": fin, "box": box}
    del r
    gc.collect()
    return out


def config_autograd(P, model, ncell, iters):
    """Differentiation at scale: 4 ncell^3 atoms of copper (50^3 cells:
    500,000 atoms), sigma 0.1 A, FP32; one iteration = DPEnergy forward
    (energy, activations kept) + backward (forces through the hand-written
    adjoint, G recomputed), timed over `iters` iterations."""
    import torch
    import synth
    from paper_2201_01446_amd.autograd import DPEnergy
    x0, box = synth.copper(ncell, 0.1, synth.SEED_CFG[4])
    N = len(x0)
    x = torch.tensor(x0, dtype=torch.float64, device="cuda")
    nl = P.NeighborList(model, x, box, skin=2.0)
    xg = x.clone().requires_grad_(True)

    def step():
        E = DPEnergy.apply(xg, model, nl, P.FP32, P.COMPRESSED)
        (g,) = torch.autograd.grad(E.sum(), xg)
        return E, g

    step()
    torch.cuda.synchronize()
    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)
    t0.record()
    for _ in range(iters):
        E, g = step()
    t1.record()
    torch.cuda.synchronize()
    ms = t0.elapsed_time(t1) / iters
    e_atom = P.compute(model, nl, x, precision=P.FP32, atom_energy=True)["e_atom"]
    fin = dict(x=x0, e_atom=e_atom.cpu().numpy(), F=-g.detach().cpu().numpy())
    v = N / (ms * 1e-3)
    return {"workload": f"Cu FCC {ncell}^3 cells ({N} atoms), sigma 0.1 A, FP32, DPEnergy forward + backward "
                        "(forces by the hand-written adjoint, G recomputed)",
            "natoms": N, "iterations": iters, "ms_per_iteration": round(ms, 4), "value": round(v, 1),
            "unit": "atom-evaluations/s (energy + gradient)", "final": fin, "box": box}


def oracle_leg(cfg, params, cases, nsamp):
    """The FP64 oracle on the host cores, untabulated and as it stands.  For
    every timed run, at random atoms of its final configuration: E_i (from
    the atoms within rcut) and the force (from the energies of every atom
    within rcut of it, on a cut-out of radius 2 rcut + 0.5 A: the same
    definition on the same neighborhoods).  Returns the CPU baseline (the
    rate of the force cut-outs: atom energies with their gradients per
    second) and per run the gate: RMSE_F over the sampled force components,
    |mean dE_i| (the estimate of |dE|/N), max |dE_i|."""
    import importlib.util
    import oracle
    spec = importlib.util.spec_from_file_location("dp_sampling", os.path.join(ROOT, "tests", "sampling.py"))
    smp = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(smp)
    gate = {}
    centers = 0
    t_force = 0.0
    nf_total = 0
    for name, (fin, box) in cases.items():
        ne, nf = (nsamp, nsamp // 8) if name == "fp64" else (nsamp // 2, nsamp // 16)
        s = smp.LocalSampler(cfg, params, None, fin["x"], box)
        rng = np.random.default_rng(7)
        e_idx = rng.choice(len(fin["x"]), ne, replace=False)
        f_idx = rng.choice(len(fin["x"]), max(1, nf), replace=False)
        e_ref = np.array([s.energy(int(k)) for k in e_idx])
        t = time.perf_counter()
        F_ref = []
        for k in f_idx:
            idx, _, r = s._cut(int(k), s.radius)
            centers += int(np.sum(r < cfg["rcut"]))
            F_ref.append(s.force(int(k)))
        t_force += time.perf_counter() - t
        nf_total += len(f_idx)
        F_ref = np.array(F_ref)
        dE = fin["e_atom"][e_idx] - e_ref
        rmse_F = float(np.sqrt(np.mean((fin["F"][f_idx] - F_ref) ** 2)))
        F_rms = float(np.sqrt(np.mean(F_ref ** 2)))
        gate[name] = {"sampled_energies": int(ne), "sampled_forces": int(len(f_idx)),
                      "rmse_F": rmse_F, "rmse_F_rel": rmse_F / max(F_rms, 1e-300), "F_rms_oracle": F_rms,
                      "dE_per_atom": float(abs(np.mean(dE))), "max_abs_dE_i": float(np.max(np.abs(dE))),
                      "pass": bool(rmse_F <= 1e-3 and abs(np.mean(dE)) <= 1e-5)}
    cpu = {"value": round(centers / t_force, 2), "unit": "atom-steps/s", "cores": oracle.num_threads(),
           "kind": "oracle",
           "sample": f"{nf_total} force cut-outs at random atoms of the final configurations of the timed runs "
                     f"({centers} atom energies with gradients, untabulated FP64 oracle, {t_force:.1f} s)"}
    return cpu, gate


def water(P, nrep, steps, warmup):
    """The two-type system (the paper's water: O and H, rcut 6 A, NVE at
    0.5 fs): the synthetic 192-atom cell replicated nrep^3 times, in the
    three precisions."""
    import synth
    cfg = synth.water_model_config()
    params = synth.model_params(cfg)
    model = P.Model(cfg, params).tabulate(0.7, 0.01, 1.5, 0.1)
    x0, t, box = synth.water(nrep, sigma=0.05)
    m = synth.water_masses(t)
    rng = np.random.Generator(np.random.PCG64(synth.SEED_VELOCITY))
    v0 = rng.standard_normal(x0.shape) * np.sqrt(synth.KB_EV * 330.0 / (m[:, None] * synth.MVV_TO_EV))
    v0 -= (m[:, None] * v0).sum(0) / m.sum()
    N = len(x0)
    out = {"workload": f"water-like O/H, 192-atom cell x {nrep}^3 ({N} atoms), NVE dt 0.5 fs, sel 46 O + 92 H, "
                       "nlist skin 2 A rebuilt every 10 steps, compressed (stride 0.01, tail 0.1)",
           "natoms": N, "steps": steps}
    for name, prec in (("fp32", P.FP32), ("fp64", P.FP64), ("mixed_bf16", P.MIXED_BF16)):
        res = run_nve(P, model, x0, v0, box, steps, warmup, prec, types=t, mass=[synth.M_O, synth.M_H], dt=0.5,
                      keep=(name == "fp32"))
        v = N * steps / (res["ms"] * 1e-3)
        th = res["thermo"]
        etot = th[:, 0] + th[:, 1]
        out[name] = {"value": round(v, 1), "unit": "atom-steps/s", "ms_per_step": round(res["ms"] / steps, 4),
                     "ns_per_day": round(v / N * 86400 * 0.5e-6, 3),
                     "energy_drift_eV_per_atom": float((etot[-1] - etot[0]) / N),
                     "kernels": {k: round(vv[0] / max(vv[1], 1), 4) for k, vv in res["kernels"].items()}}
        if name == "fp32":
            # look-ups past the table end over the run: the random-weight
            # model has no repulsive core, so atoms in near free flight can
            # pass closer than the table reaches (s > 1.5, r < 0.67 A), where
            # G is clamped and the energy is no longer conserved
            out[name]["table_oob_lookups"] = res["nl"].stats()["table_oob"]
            d = P.descriptor(model, res["nl"], res["x"], precision=P.FP32)
            out["mean_neighbors"] = float(d["nnei"].double().mean().item())
            out["mean_interval_segments"] = float(d["nseg"].double().mean().item())
            del res
    return out


def tanh_compare(P, cfg, params, x0, v0, box, steps):
    """The fitting net's tanh from the second-order table against the native
    tanh, FP32: MD speed, fitting-GEMM times, and the change of one
    evaluation of the start configuration."""
    import torch
    N = len(x0)
    out = {}
    x = torch.tensor(x0, dtype=torch.float64, device="cuda")
    res = {}
    for tab in (False, True):
        m = P.Model(cfg, params).tabulate(0.7, 0.01, 1.5, 0.1).fitting_tanh(tab)
        nl = P.NeighborList(m, x, box, skin=2.0)
        res[tab] = P.compute(m, nl, x, precision=P.FP32)
        r = run_nve(P, m, x0, v0, box, steps, 2, P.FP32)
        out["table" if tab else "native"] = {
            "atom_steps_per_s": round(N * steps / (r["ms"] * 1e-3), 1), "ms_per_step": round(r["ms"] / steps, 4),
            "fitting_forward_ms": round(sum(v[0] / max(v[1], 1) for k, v in r["kernels"].items()
                                            if k.startswith("fit_fwd")), 4)}
        del nl, m
    a, b = res[False], res[True]
    out["dE_per_atom"] = abs(float(a["E"][0] - b["E"][0])) / N
    out["rmse_F_change"] = float(torch.sqrt(torch.mean((a["F"] - b["F"]) ** 2)))
    return out


def ablation(P, x0, v0, box, steps):
    """The optimization ladder, FP32, same MD protocol: the plain network;
    the tabulated G materialised; fused per neighbor over all sel rows;
    fused per neighbor over the real neighbors only; fused per table-interval
    run (the default).  At sel = 192 (the copper model) and sel = 512 (the
    padding regime of the paper's ablation), with weights drawn for each."""
    import gc
    import torch
    import synth
    rungs = (("plain", P.PLAIN), ("tabulated_unfused", P.TAB_UNFUSED), ("fused_padded", P.FUSED_PADDED),
             ("fused", P.FUSED), ("fused_interval_runs", P.COMPRESSED))
    out = {}
    N = len(x0)
    for sel in (192, 512):
        cfg = synth.copper_model_config(sel=sel)
        m = P.Model(cfg, synth.model_params(cfg)).tabulate(0.7, 0.01, 1.5, 0.1)
        rows = {}
        for name, mode in rungs:
            r = run_nve(P, m, x0, v0, box, steps, 1, P.FP32, mode=mode)
            emb = sum(v[0] / steps for k, v in r["kernels"].items()
                      if k.startswith(("emb", "plain", "tab_", "dT", "force_gather")))
            rows[name] = {"atom_steps_per_s": round(N * steps / (r["ms"] * 1e-3), 1),
                          "ms_per_step": round(r["ms"] / steps, 4), "embedding_ms_per_step": round(emb, 4)}
            del r
            gc.collect()
            torch.cuda.synchronize()
        base = rows["plain"]["ms_per_step"]
        for v in rows.values():
            v["speedup_vs_plain"] = round(base / v["ms_per_step"], 3)
        out[f"sel{sel}"] = rows
        del m
        gc.collect()
    return out


def stride_sweep(P, cfg, params, x0, v0, box, steps):
    """The table stride h of the fine range [0, 0.7) (tail 0.1 to 1.5): table
    size, segments per atom, FP32 MD speed, and the error of one evaluation
    of the start configuration against the untabulated network (the plain
    FP64 path of the same library, which the tests hold to the oracle at
    1e-10)."""
    import torch
    x = torch.tensor(x0, dtype=torch.float64, device="cuda")
    ref_model = P.Model(cfg, params).tabulate(0.7, 0.01, 1.5, 0.1)
    nl = P.NeighborList(ref_model, x, box, skin=2.0)
    ref = P.compute(ref_model, nl, x, mode=P.PLAIN, precision=P.FP64)
    Fr = ref["F"]
    Frms = float(torch.sqrt(torch.mean(Fr * Fr)))
    N = x.shape[0]
    rows = []
    for h in (0.1, 0.01, 0.001):
        m = P.Model(cfg, params).tabulate(0.7, h, 1.5, 0.1)
        nint = int(round(0.7 / h)) + 8
        row = {"stride": h, "intervals": nint, "table_bytes_fp32": nint * 128 * 6 * 4,
               "table_bytes_fp64": nint * 128 * 6 * 8}
        for prec, tag in ((P.FP64, "fp64"), (P.FP32, "fp32")):
            o = P.compute(m, nl, x, precision=prec)
            dE = abs(float(o["E"][0] - ref["E"][0])) / N
            eF = float(torch.sqrt(torch.mean((o["F"] - Fr) ** 2)))
            row[f"{tag}_dE_per_atom"] = dE
            row[f"{tag}_rmse_F"] = eF
            row[f"{tag}_rmse_F_rel"] = eF / Frms
        d = P.descriptor(m, nl, x, precision=P.FP32)
        row["mean_segments"] = float(d["nseg"].float().mean())
        r = run_nve(P, m, x0, v0, box, steps, 2, P.FP32)
        row["fp32_atom_steps_per_s"] = round(N * steps / (r["ms"] * 1e-3), 1)
        row["fp32_ms_per_step"] = round(r["ms"] / steps, 4)
        row["kernels_ms"] = {k: round(v[0] / max(v[1], 1), 4) for k, v in r["kernels"].items()
                             if k in ("emb_fwd", "emb_bwd")}
        rows.append(row)
        del m
    return rows


SERVE_BATCH_ATOMS = 20000   # the Poisson (latency) phase's cap on atoms per batch


def serving(P, model, nreq):
    """Continuous batching of nreq evaluation requests (periodic FCC-derived
    Cu cells, atom counts log-uniform in [32, 20000], sigma U[0.02, 0.15] A,
    0-5 % vacancies), FP32.  A closed loop (all requests at t = 0) gives the
    saturated throughput; Poisson arrivals at 70 % of the saturated
    throughput of the latency mode (batches of at most SERVE_BATCH_ATOMS
    atoms) give the latency percentiles (arrival to results on the host)."""
    import synth
    from paper_2201_01446_amd.serve import Server, poisson_arrivals
    t = time.perf_counter()
    reqs = [r[:2] for r in synth.serving_stream(nreq)]
    gen_s = time.perf_counter() - t
    srv = Server(model, P.FP32, slots=3, hbm_budget=24 << 30)
    srv.run(reqs[:64])                          # warm-up
    _, closed = srv.run(reqs)                   # throughput: full slots
    # latency mode: at most SERVE_BATCH_ATOMS atoms per batch, so that a burst
    # of arrivals becomes several shorter batches rather than a few full slots
    # that share the GPU and return late; Poisson arrivals at 70 % of this
    # mode's own saturated throughput
    _, capped = srv.run(reqs, max_batch_atoms=SERVE_BATCH_ATOMS)
    rate = 0.7 * nreq / capped["wall_s"]
    _, pois = srv.run(reqs, poisson_arrivals(nreq, rate, seed=synth.SEED_SERVING + 1), max_batch_atoms=SERVE_BATCH_ATOMS)
    keep = ("atoms_per_s", "p50_ms", "p99_ms", "mean_ms", "mean_wait_ms", "mean_service_ms", "tail_wait_ms",
            "tail_service_ms", "tail_mean_atoms", "mean_atoms", "batches", "mean_batch_atoms", "wall_s")
    return {"requests": nreq, "rejected": closed["rejected"], "atoms": closed["atoms"], "slots": closed["slots"],
            "slot_atoms": closed["slot_atoms"], "precision": "fp32",
            "closed_loop": {k: round(closed[k], 4) for k in keep},
            "poisson": dict({k: round(pois[k], 4) for k in keep}, rate_req_per_s=round(rate, 2),
                            max_batch_atoms=SERVE_BATCH_ATOMS,
                            saturated_atoms_per_s=round(capped["atoms_per_s"], 1)),
            "request_generation_s": round(gen_s, 2)}


if __name__ == "__main__":
    main()
