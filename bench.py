#!/usr/bin/env python3
"""Throughput of the per-candidate MoM evaluation on one MI355X.

Workload (default): two metal layers of 20 x 20 half-millimetre pixels in a
lossy dielectric (eps_r 3.5, tan d 0.002), three ports, 13 vias, parent size
M = 2371, 101 frequencies over 1-8 GHz; one step evaluates all 800
single-flip candidates of the seeded Bernoulli(0.5) map at every frequency
(gather, dense LU, S, FoM, argmin).  Inputs are synthetic and resident in HBM
before timing starts; the parent fill is pre-computation and not timed.

Prints one JSON line (stdout).  Progress goes to stderr.
"""

from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_TFLOPS = {"fp64": 78.6, "mixed32": 157.3}


def log(msg):
    print(f"[bench {time.strftime('%H:%M:%S')}] {msg}", file=sys.stderr, flush=True)


def lu_flops(N, P):
    """Algorithmic work of one (candidate, frequency) item: complex LU of the
    N x N system plus forward and back substitution for P right-hand sides."""
    N = np.asarray(N, dtype=np.float64)
    return (8.0 / 3.0) * N ** 3 + 8.0 * P * N ** 2


KERNEL_OF = {"fp64": "k_eval_plain", "mixed32": "k_eval_mixed"}


def measured_traffic(workload, kernel, items):
    """HBM bytes per launch of `kernel` from the committed counter summary
    (FETCH_SIZE + WRITE_SIZE, copy-calibrated), or None when there is none for
    this workload or the kernel sources changed since it was taken."""
    import hashlib

    path = os.path.join(ROOT, "profiles", f"k_eval_{workload}_traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        rec = json.load(fh)
    h = hashlib.sha256()
    for f in rec["source_files"]:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    k = rec["kernels"].get(kernel)
    if h.hexdigest() != rec["source_sha256"] or k is None or rec["items_per_launch"] != items:
        return None
    return k["hbm_bytes_per_launch"]


def cpu_baseline(spec, gpu_S, sample_c, seconds):
    """Time the oracle (as it stands) on a bounded sample of the same
    workload: its own parent fill at one frequency (not timed), then Eq. 5
    gather, LAPACK solve, S and the per-frequency FoM terms for a set of
    candidates, repeated until `seconds` of work; scaled to evaluations/s over
    all frequencies.  Also returns the sampled max |dS| against the GPU."""
    from oracle import efie, fom as ofom, geometry, network, search

    try:
        from threadpoolctl import threadpool_info

        cores = max([d.get("num_threads", 1) for d in threadpool_info()] or [1])
    except Exception:  # pragma: no cover
        cores = os.cpu_count()
    f_idx = int(np.argmin(np.abs(spec.freqs - 5.5e9)))
    f = spec.freqs[f_idx]
    st = geometry.build_structure(spec)
    log(f"cpu baseline: oracle fill at {f / 1e9:.2f} GHz (M = {st.M})")
    t = time.time()
    Z = efie.fill(st, f)
    log(f"cpu baseline: oracle fill took {time.time() - t:.1f} s")
    base = spec.base_map()
    off, cells = spec.flips()
    maps = search.candidate_maps(base, off, cells)
    pl = search.port_lengths(st)
    dS = 0.0
    done = 0
    t0 = time.perf_counter()
    while True:
        for c in sample_c:
            sel = st.active(maps[c])
            rows = network.port_positions(sel, st.port_bf)
            S = network.s_parameters(network.reduce_matrix(Z, sel), rows, pl, spec.z0)
            ofom.rewards(S)
            if done < len(sample_c):
                dS = max(dS, float(np.abs(S - gpu_S[c, f_idx]).max()))
            done += 1
        el = time.perf_counter() - t0
        if el >= seconds:
            break
    per_item = el / done
    value = 1.0 / (per_item * spec.n_freq)
    sample = (f"{len(sample_c)} candidates x 1 frequency ({f / 1e9:.2f} GHz), {done} solves in {el:.1f} s, "
              f"scaled x{spec.n_freq} frequencies per evaluation")
    return {"value": value, "unit": "evals/s", "cores": int(cores), "kind": "oracle", "sample": sample}, dS


def lowrank_leg(args, pxd, spec, pb, Z, base, off, cells, results):
    """The same batch through the low-rank flip evaluation (FP64, from the
    cached inverse of the base map), host buffers in and out."""
    C = len(off) - 1
    ev = pxd.Evaluator(device=0, precision=pxd.PREC_FP64)
    ev.load_parent(Z, spec.freqs)
    ev.load_problem(pb, spec.z0)
    ev.set_fom_paper()
    Nc, idx = ev.expand(base, off, cells)
    NB, idx_b = ev.expand(base, np.zeros(2, np.int32), np.zeros(0, np.int32))
    bset = set(idx_b[0].tolist())
    added = np.array([len(set(idx[c].tolist()) - bset) for c in range(C)])
    t0 = time.perf_counter()
    S, fom, st, am = ev.evaluate_flips_lowrank(base, off, cells)
    first_ms = (time.perf_counter() - t0) * 1e3
    s_first = ev.stats()
    log(f"[lowrank] first call {first_ms:.1f} ms (base inverse {s_first['ms_base_inverse']:.1f} ms, "
        f"N_B = {NB[0]}, {s_first['fallbacks']} dense items)")
    t0 = time.perf_counter()
    k_ms = []
    for i in range(args.steps):
        S, fom, st, am = ev.evaluate_flips_lowrank(base, off, cells)
        k_ms.append(ev.stats()["ms_solve"])
        log(f"[lowrank] step {i + 1}/{args.steps}: kernel {k_ms[-1]:.2f} ms")
    ms = (time.perf_counter() - t0) * 1e3 / args.steps
    stats = ev.stats()
    ev.close()
    # algorithmic bytes of the low-rank kernel: one pass over G (N_B^2 complex128)
    # per four added functions, per (candidate, frequency)
    passes = float(np.sum((added + 3) // 4)) * spec.n_freq
    g_bytes = passes * float(NB[0]) ** 2 * 16
    k = float(np.mean(k_ms))
    out = {
        "value": C / (ms / 1e3), "unit": "evals/s", "ms_per_step": ms, "kernel_ms": k,
        "first_call_ms": first_ms, "ms_base_inverse": s_first["ms_base_inverse"],
        "base_reused": int(stats["base_reused"]), "dense_fallback_items": int(stats["fallbacks"]),
        "status_errors": int(np.count_nonzero(st != 0)),
        "io": "host buffers (PCIe copies of flips and S inside the timed step)",
        "g_stream": {"bytes_per_launch": g_bytes, "achieved_GBps": g_bytes / (k / 1e3) / 1e9,
                     "basis": "N_B^2 x 16 B per pass, ceil(added / 4) passes per (candidate, frequency)"},
        "traffic": measured_traffic(spec.name, "k_lowrank", C * spec.n_freq),
    }
    if "fp64" in results:
        f64 = results["fp64"]
        sc = f64["sample_c"]
        out["max_dS_vs_fp64_plain"] = float(np.abs(S[sc] - f64["S_sample"]).max())
        out["argmin_equal_fp64_plain"] = bool(am == f64["am"])
        out["fom_rel_dev_vs_fp64_plain"] = float(np.max(np.abs(fom - f64["fom"]) / f64["fom"]))
        out["speedup_vs_fp64_plain"] = out["value"] / f64["value"]
    return out


def surrogate_leg(args, pxd, spec, pb, torch):
    """Ranking by the CNN surrogate at its working size: a 3 x 24 x 24 map
    (channels 32-64, hidden 256, BF16 products) scored on the workload's 101
    frequencies with its FoM table; every single flip and every pair of
    cells, then the top 32.  Random-init weights (throughput only)."""
    dev = torch.device("cuda:0")
    ev = pxd.Evaluator(device=0)
    ev.load_problem(pb, spec.z0)
    ev.load_parent_problem(pb, spec.freqs)
    ev.set_fom_paper()
    L, ny, nx = 3, 24, 24
    n = L * ny * nx
    sur = pxd.Surrogate(L, ny, nx, spec.freqs, spec.freqs[0], spec.freqs[-1], precision=pxd.SUR_BF16,
                        max_batch=2048)
    sur.init_params(17)
    iu, ju = np.triu_indices(n, 1)
    C = n + len(iu)
    off = np.concatenate([np.arange(n + 1), n + 2 * np.arange(1, len(iu) + 1)]).astype(np.int32)
    cells = np.concatenate([np.arange(n), np.stack([iu, ju], 1).ravel()]).astype(np.int32)
    base = (np.arange(n) % 2).astype(np.uint8)
    t_base, t_off, t_cells = (torch.from_numpy(a).to(dev) for a in (base, off, cells))
    fp = torch.empty(C, dtype=torch.float64, device=dev)
    top = torch.empty(32, dtype=torch.int32, device=dev)
    stream = torch.cuda.current_stream()
    sur.rank(ev, t_base, t_off, t_cells, 32, fp, top, stream)  # warm-up
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    sur.rank(ev, t_base, t_off, t_cells, 32, fp, top, stream)
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    ok = bool(torch.isfinite(fp).all().item()) and int(top.min().item()) >= 0
    log(f"[surrogate] ranked {C:,} candidates (3x24x24 map, 101 frequencies) in {ms:.0f} ms, top-32 valid {ok}")
    # trunk work per map: four 3x3 convolutions; head: two products per (map, frequency)
    ch = (3, 32, 32, 64, 64)
    px = (ny * nx, ny * nx, ny * nx // 4, ny * nx // 4)
    trunk = sum(2 * 9 * ch[i] * ch[i + 1] * px[i] for i in range(4))
    feat = 64 * (ny // 4) * (nx // 4)
    flops = C * (trunk + 2 * feat * 256 + len(spec.freqs) * 2 * 256 * 9)
    sur.close()
    ev.close()
    return {"value": C / (ms / 1e3), "unit": "maps/s", "ms": ms, "candidates": C,
            "workload": "every single flip and cell pair of a 3x24x24 map, 101 frequencies, top 32",
            "precision": "bf16 products, fp32 accumulation", "weights": "random init (throughput only)",
            "flops_per_call": flops, "achieved_TFLOPs": flops / (ms / 1e3) / 1e12, "peak_TFLOPs": 2500.0,
            "top_valid": ok}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="batched20")
    ap.add_argument("--precision", default="both", choices=sorted(PEAK_TFLOPS) + ["both"])
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-lowrank", action="store_true", help="skip the low-rank flip evaluation leg")
    ap.add_argument("--no-surrogate", action="store_true", help="skip the surrogate ranking leg")
    ap.add_argument("--fill-threads", type=int, default=16)
    ap.add_argument("--copy-calibration", action="store_true",
                    help="first copy 1 GiB device to device, a reference kernel of known traffic for "
                         "byte counters (FETCH_SIZE / WRITE_SIZE)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py: this build runs on one GPU; --gpus must be 1 (the path shards by frequency "
              "across GPUs by design, but no multi-GPU run is part of this build)", file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_2412_17617_amd import pxd
    from synth import get_spec

    if args.copy_calibration:
        src = torch.ones(2 ** 27, dtype=torch.float64, device="cuda:0")
        torch.cuda.synchronize()
        dst = src.clone()  # reads 1 GiB, writes 1 GiB
        torch.cuda.synchronize()
        del src, dst
        log("copy calibration: 1 GiB device-to-device copy done")

    spec = get_spec(args.workload)
    freqs = spec.freqs
    log(f"workload {spec.name}: {spec.n_layers} layers {spec.nx}x{spec.ny}, {spec.n_freq} frequencies")
    pb = pxd.Problem.from_spec(spec)
    t = time.time()
    Z = pb.fill(freqs, n_threads=args.fill_threads)
    host_fill_s = time.time() - t
    log(f"parent fill (host, {args.fill_threads} threads): M = {pb.M}, {host_fill_s:.1f} s")
    dev = torch.device("cuda:0")
    Zd = torch.empty((spec.n_freq, pb.M, pb.M), dtype=torch.complex128, device=dev)
    torch.cuda.synchronize()
    t = time.time()
    pb.fill_device(freqs, Zd)
    torch.cuda.synchronize()
    gpu_fill_s = time.time() - t
    chk = list(range(0, spec.n_freq, max(1, spec.n_freq // 4)))
    fill_dev = float(max(np.abs(Zd[f].cpu().numpy() - Z[f]).max() / np.abs(Z[f]).max() for f in chk))
    del Zd
    log(f"parent fill (GPU): {gpu_fill_s * 1e3:.0f} ms, max |dZ| / max |Z| vs host fill {fill_dev:.1e}")
    parent_fill = {"gpu_s": gpu_fill_s, "host_s": host_fill_s, "host_threads": args.fill_threads,
                   "speedup": host_fill_s / gpu_fill_s, "max_rel_dZ_vs_host": fill_dev,
                   "frequencies": spec.n_freq, "M": pb.M}
    base = spec.base_map()
    off, cells = spec.flips()
    C = len(off) - 1
    P = len(spec.ports)
    t_base = torch.from_numpy(base).to(dev)
    t_off = torch.from_numpy(off).to(dev)
    t_cells = torch.from_numpy(cells).to(dev)
    stream = torch.cuda.current_stream()
    modes = ["fp64", "mixed32"] if args.precision == "both" else [args.precision]
    results = {}
    for mode in modes:
        prec = pxd.PREC_FP64 if mode == "fp64" else pxd.PREC_MIXED32
        # full-width register sub-panel; workgroups per CU and item order autotuned
        ev = pxd.Evaluator(device=0, precision=prec, half_subpanel=1)
        ev.load_parent(Z, freqs)
        ev.load_problem(pb, spec.z0)
        ev.set_fom_paper()
        n_tune = min(C, 96)
        tune = ev.autotune(base, off[:n_tune + 1], cells[:off[n_tune]], n_reps=1)
        log(f"[{mode}] autotuned on {n_tune} candidates: " +
            ", ".join(f"wg/CU {t['wg_per_cu']} order {t['schedule']} {t['ms']:.0f} ms" for t in tune))
        S_out = torch.empty((C, spec.n_freq, P, P, 2), dtype=torch.float64, device=dev)
        fom_out = torch.empty(C, dtype=torch.float64, device=dev)
        st_out = torch.empty(C, dtype=torch.int32, device=dev)
        am_out = torch.empty(1, dtype=torch.int32, device=dev)
        N, _ = ev.expand(base, off, cells)
        flops_per_launch = float(lu_flops(N, P).sum() * spec.n_freq)
        log(f"[{mode}] candidates {C}, active size {N.min()}..{N.max()}, {flops_per_launch / 1e12:.1f} TFLOP per step")

        def step():
            ev.evaluate_flips_device(stream, t_base, t_off, t_cells, S_out, fom_out, st_out, am_out)

        for i in range(args.warmup):
            step()
            torch.cuda.synchronize()
            log(f"[{mode}] warmup {i + 1}/{args.warmup}")
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        kernel_ms, stats = [], []
        e0.record(stream)
        for i in range(args.steps):
            step()
            stats.append(ev.stats())
            kernel_ms.append(stats[-1]["ms_solve"])
            log(f"[{mode}] step {i + 1}/{args.steps}: evaluator kernel {kernel_ms[-1]:.1f} ms, "
                f"fallback {stats[-1]['ms_fallback']:.1f} ms ({stats[-1]['fallbacks']} items), "
                f"refinement steps {stats[-1]['ir_iterations']}")
        e1.record(stream)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / args.steps
        k_ms = float(np.mean(kernel_ms))
        if mode == "mixed32":  # refinement: residual and correction solve, 16 P N^2 per step
            flops_per_launch += 16.0 * P * float(np.mean(N.astype(np.float64) ** 2)) * stats[-1]["ir_iterations"]
        achieved = flops_per_launch / (k_ms / 1e3) / 1e12
        results[mode] = {
            "value": C / (ms / 1e3), "ms_per_step": ms, "kernel_ms": k_ms, "achieved": achieved,
            "peak": PEAK_TFLOPS[mode], "N": N, "fallbacks": int(stats[-1]["fallbacks"]),
            "ir_steps": int(stats[-1]["ir_iterations"]), "status_nonzero": int(np.count_nonzero(
                (st_out.cpu().numpy() != 0) & (st_out.cpu().numpy() != 1))),
            "fom": fom_out.cpu().numpy(), "am": int(am_out.cpu().numpy()[0]),
            "tuned": {"wg_per_cu": tune[0]["wg_per_cu"], "schedule": tune[0]["schedule"], "half_subpanel": 1,
                      "tried": [(t["wg_per_cu"], t["schedule"], round(t["ms"], 1)) for t in tune],
                      "batch": f"first {n_tune} candidates"},
            "S_sample": None,
        }
        sample_c = list(range(0, C, max(1, C // 16)))[:16]
        results[mode]["sample_c"] = sample_c
        results[mode]["S_sample"] = torch.view_as_complex(S_out[sample_c].contiguous()).cpu().numpy()
        ev.close()
        del S_out
    lowrank = None if args.no_lowrank else lowrank_leg(args, pxd, spec, pb, Z, base, off, cells, results)
    surrogate = None if args.no_surrogate else surrogate_leg(args, pxd, spec, pb, torch)
    del Z
    chosen = "mixed32" if "mixed32" in results else modes[0]
    r = results[chosen]
    N = r["N"]
    out = {
        "metric": "pixel-map evals/sec (all freqs, S+FoM) vs FP64 plain, at max |dS|<=1e-4",
        "value": r["value"],
        "unit": "evals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": r["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if chosen == "fp64" else "f32+f64",
        "data": "synthetic",
        "config": {
            "workload": f"{spec.name}: {spec.n_layers} layers {spec.nx}x{spec.ny} pixels, M={pb.M}, "
                        f"{spec.n_freq} freqs {spec.f_lo / 1e9:g}-{spec.f_hi / 1e9:g} GHz, {C} single flips",
            "precision": chosen,
            "candidates": C,
            "frequencies": spec.n_freq,
            "active_size": [int(N.min()), int(N.max())],
            "status_errors": r["status_nonzero"],
            "fallback_items": r["fallbacks"],
            "refinement_steps": r["ir_steps"],
            "launch": r["tuned"],
        },
        "roofline": {
            "bound": "mfma",
            "achieved": r["achieved"],
            "peak": r["peak"],
            "unit": "TFLOP/s",
            "frac": r["achieved"] / r["peak"],
            "traffic": None,
            "kernel": KERNEL_OF[chosen],
            "kernel_ms": r["kernel_ms"],
        },
    }
    traffic = measured_traffic(spec.name, KERNEL_OF[chosen], C * spec.n_freq)
    if traffic is not None:
        out["roofline"]["traffic"] = traffic
        out["roofline"]["traffic_unit"] = "bytes/launch"
        out["roofline"]["traffic_TBps"] = traffic / (r["kernel_ms"] / 1e3) / 1e12
    if "fp64" in results and chosen != "fp64":
        f64 = results["fp64"]
        out["fp64_plain"] = {"value": f64["value"], "ms_per_step": f64["ms_per_step"], "kernel_ms": f64["kernel_ms"],
                             "roofline_frac": f64["achieved"] / f64["peak"], "achieved_tflops": f64["achieved"],
                             "traffic": measured_traffic(spec.name, KERNEL_OF["fp64"], C * spec.n_freq)}
        out["speedup_vs_fp64_plain"] = r["value"] / f64["value"]
        out["config"]["max_dS_vs_fp64_plain"] = float(np.abs(r["S_sample"] - f64["S_sample"]).max())
        out["config"]["argmin_equal_fp64_plain"] = bool(r["am"] == f64["am"])
        out["config"]["fom_rel_dev_vs_fp64_plain"] = float(np.max(np.abs(r["fom"] - f64["fom"]) / f64["fom"]))
    out["parent_fill"] = parent_fill
    if lowrank is not None:
        out["lowrank"] = lowrank
    if surrogate is not None:
        out["surrogate"] = surrogate
    if not args.no_cpu_baseline:
        sample_c = r["sample_c"]
        S_full = np.zeros((C,) + r["S_sample"].shape[1:], np.complex128)
        S_full[sample_c] = r["S_sample"]
        cb, dS = cpu_baseline(spec, S_full, sample_c, args.cpu_seconds)
        out["cpu_baseline"] = cb
        out["config"]["max_dS_vs_oracle_sample"] = dS
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
