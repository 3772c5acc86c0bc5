#!/usr/bin/env python3
"""Throughput of the per-candidate MoM evaluation on one MI355X.

Headline workload (default, the largest one-GPU configuration): three metal
layers of 32 x 32 pixels of 0.3 mm (Table I's 0.4866 mm stack, eps_r 3.66,
tan d 0.004), three ports, parent size M = 9,036, 201 frequencies over
0.5-10 GHz.  One step is one search step of the depth-two tree search on the
seeded Bernoulli(0.5) map: the CNN surrogate ranks all 9,024 pair flips within
3 x 3 neighbourhoods, and the best 32 are evaluated exactly at every frequency
(gather of Z_A, dense LU, S, FoM, argmin).  The chosen form (complex64 LU +
FP64 iterative refinement) is timed beside the FP64 plain path on the same
candidates.  Inputs are synthetic and resident in HBM before timing starts;
the parent fill (the paper's pre-computation phase) is not timed.

Further legs (each its own context): the 24 x 24 x 3 stack (64 single flips,
101 frequencies; FP64, complex64 and split-BF16 update forms), the 20 x 20 x 2
stack with vias (all 800 single flips, 101 frequencies; path autotuned), the
surrogate ranking at its working size and the low-rank flip evaluation.

Prints one JSON line (stdout).  Progress goes to stderr.
"""

from __future__ import annotations

import argparse
import concurrent.futures
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# dense MFMA peaks of the data type each form's trailing update issues
PEAK_TFLOPS = {"fp64": 78.6, "mixed32": 157.3, "bf16x3": 2500.0}
HBM_PEAK_GBPS = 8000.0
PREC = {"fp64": 0, "mixed32": 1, "bf16": 2, "bf16x3": 4}


def log(msg):
    print(f"[bench {time.strftime('%H:%M:%S')}] {msg}", file=sys.stderr, flush=True)


def lu_flops(N, P):
    """Algorithmic work of one (candidate, frequency) item: complex LU of the
    N x N system plus forward and back substitution for P right-hand sides."""
    N = np.asarray(N, dtype=np.float64)
    return (8.0 / 3.0) * N ** 3 + 8.0 * P * N ** 2


def kernel_name(path, mode):
    if path == "tiled":
        return {"fp64": "k_tl_update<double>", "mixed32": "k_tl_update<float>",
                "bf16x3": "k_tl_update_bf16x3"}[mode]
    return "k_eval_plain" if mode == "fp64" else "k_eval_mixed"


def binding_roof(form, gflop_per_launch, gbyte_per_launch):
    """The roof that binds one trailing-update launch: the larger of its
    compute floor (the MFMA flops it issues at the dense peak of their type;
    split-BF16 issues three BF16 products per real product: hi hi, hi lo,
    lo hi) and its memory floor (its algorithmic bytes at the HBM peak).
    Returns (bound, compute floor us, memory floor us, products issued per
    real product)."""
    issued = 3.0 if form == "bf16x3" else 1.0
    compute_us = issued * gflop_per_launch / PEAK_TFLOPS[form] * 1e3
    memory_us = gbyte_per_launch / HBM_PEAK_GBPS * 1e6
    return ("hbm" if memory_us > compute_us else "mfma"), compute_us, memory_us, issued


def measured_traffic(workload, kernel, items):
    """HBM bytes per launch of `kernel` from the committed counter summary
    (FETCH_SIZE + WRITE_SIZE, copy-calibrated), or None when there is none for
    this workload or the kernel sources changed since it was taken."""
    path = os.path.join(ROOT, "profiles", f"traffic_{workload}.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        rec = json.load(fh)
    h = hashlib.sha256()
    for f in rec["source_files"]:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    k = rec["kernels"].get(kernel)
    if h.hexdigest() != rec["source_sha256"] or k is None or rec["items_per_step"] != items:
        return None
    return k


# ---------------------------------------------------------------- CPU baseline (oracle)

def oracle_prepare(jobs):
    """Untimed part of the CPU baseline, run in a background thread while the
    GPU legs run: the oracle's own fill for each sampled system (the paper's
    pre-computation phase).  jobs: (label, spec, maps, f_index, subset)."""
    from oracle import efie, geometry, network

    out = []
    for label, spec, maps, fi, subset in jobs:
        t = time.time()
        st = geometry.build_structure(spec)
        if subset:  # the union of the sampled candidates' active sets only
            union = np.zeros(st.M, bool)
            for m in maps:
                union |= st.active(m)
            idx = network.support(union)
        else:
            idx = np.arange(st.M)
        Z = efie.fill(st, spec.freqs[fi], bf_subset=idx)
        out.append((label, spec, st, maps, fi, idx, Z))
        log(f"cpu baseline: oracle fill for {label} ({len(idx)} functions) took {time.time() - t:.0f} s")
    return out


def oracle_time(prepared, seconds, threads=None):
    """Time the oracle's per-candidate work (Eq. 5 gather, LAPACK solve, S by
    Eqs. 6-7, Eq. 9 terms) on each prepared sample for about `seconds`,
    scaled to evaluations/s over all the workload's frequencies."""
    from threadpoolctl import threadpool_info, threadpool_limits

    from oracle import fom as ofom
    from oracle import network, search

    res = {}
    with threadpool_limits(limits=threads):
        cores = max([d.get("num_threads", 1) for d in threadpool_info()] or [1])
        for label, spec, st, maps, fi, idx, Z in prepared:
            pos = -np.ones(st.M, np.int64)
            pos[idx] = np.arange(len(idx))
            pl = search.port_lengths(st)
            done, t0, c0 = 0, time.perf_counter(), time.process_time()
            while True:
                for m in maps:
                    sel = st.active(m)
                    rows = pos[network.support(sel)]
                    Za = Z[np.ix_(rows, rows)]
                    S = network.s_parameters(Za, network.port_positions(sel, st.port_bf), pl, spec.z0)
                    ofom.rewards(S)
                    done += 1
                el = time.perf_counter() - t0
                if el >= seconds / len(prepared):
                    break
            busy = (time.process_time() - c0) / el  # CPU seconds per second: the cores actually kept busy
            res[label] = {"value": 1.0 / (el / done * spec.n_freq), "unit": "evals/s",
                          "cores": max(1, int(round(busy))), "blas_threads": int(cores),
                          "cores_busy": round(busy, 2), "kind": "oracle",
                          "sample": f"{len(maps)} candidates x 1 frequency ({spec.freqs[fi] / 1e9:.3f} GHz), "
                                    f"{done} solves in {el:.1f} s, scaled x{spec.n_freq} frequencies per evaluation"}
    return res


# ---------------------------------------------------------------- GPU legs

def _events(torch, stream):
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    return e0, e1


def headline_leg(args, pxd, torch, spec, modes):
    """Surrogate-prefiltered search step of the 32 x 32 x 3 workload."""
    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream()
    pb = pxd.Problem.from_spec(spec)
    freqs = spec.freqs
    base = spec.base_map()
    off, cells = spec.flips()
    C_all, k = len(off) - 1, args.top_k
    P = len(spec.ports)
    pairs = cells.reshape(C_all, 2)
    t_base, t_off, t_cells = (torch.from_numpy(a).to(dev) for a in (base, off, cells))
    sub_off = torch.from_numpy(np.arange(0, 2 * k + 1, 2, dtype=np.int32)).to(dev)
    sub_cells = torch.zeros(2 * k, dtype=torch.int32, device=dev)
    fp = torch.empty(C_all, dtype=torch.float64, device=dev)
    top = torch.empty(k, dtype=torch.int32, device=dev)
    sur = pxd.Surrogate(spec.n_layers, spec.ny, spec.nx, freqs, freqs[0], freqs[-1], precision=pxd.SUR_BF16,
                        max_batch=2048)
    sur.init_params(17)
    out = {"candidates_ranked": C_all, "top_k": k}
    for mode in modes:
        ev = pxd.Evaluator(device=0, precision=PREC[mode], ir_max_iter=args.ir_max)
        ev.load_problem(pb, spec.z0)
        torch.cuda.synchronize()
        t = time.time()
        ev.load_parent_problem(pb, freqs)
        fill_s = time.time() - t
        ev.set_fom_paper()
        log(f"[headline {mode}] parent filled on the GPU: M = {pb.M}, {len(freqs)} frequencies, "
            f"{len(freqs) * pb.M * pb.M * 16 / 1e9:.0f} GB complex128, {fill_s:.1f} s")
        S_out = torch.empty((k, len(freqs), P, P, 2), dtype=torch.float64, device=dev)
        fom_out = torch.empty(k, dtype=torch.float64, device=dev)
        st_out = torch.empty(k, dtype=torch.int32, device=dev)
        am_out = torch.empty(1, dtype=torch.int32, device=dev)
        rank_ms = []

        def step():
            r0, r1 = _events(torch, stream)
            r0.record(stream)
            sur.rank(ev, t_base, t_off, t_cells, k, fp, top, stream)
            r1.record(stream)
            sel = top.cpu().numpy()  # the surrogate's best k (synchronises)
            rank_ms.append(r0.elapsed_time(r1))
            sub_cells.copy_(torch.from_numpy(np.ascontiguousarray(pairs[sel].reshape(-1))))
            ev.evaluate_flips_device(stream, t_base, sub_off, sub_cells, S_out, fom_out, st_out, am_out)
            return sel

        n_warm, n_steps = (args.warmup, args.steps) if mode == modes[-1] else (args.warmup, 1)
        ev.set_profiling(True)
        for i in range(n_warm):
            step()
            torch.cuda.synchronize()
            log(f"[headline {mode}] warmup {i + 1}/{n_warm}")
        torch.cuda.synchronize()
        rank_ms.clear()
        stats = []
        e0, e1 = _events(torch, stream)
        e0.record(stream)
        for i in range(n_steps):
            sel = step()
            stats.append(ev.stats())
            s = stats[-1]
            log(f"[headline {mode}] step {i + 1}/{n_steps}: solve {s['ms_solve']:.0f} ms, fallback "
                f"{s['ms_fallback']:.0f} ms ({s['fallbacks']} items), refinement steps {s['ir_iterations']}, "
                f"trailing updates {s['ms_update']:.0f} ms in {s['update_launches']} launches "
                f"({s['update_gflop'] / max(s['ms_update'], 1e-9):.1f} TFLOP/s)")
        e1.record(stream)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / n_steps
        sub_o = np.arange(0, 2 * k + 1, 2, dtype=np.int32)
        N, _ = ev.expand(base, sub_o, pairs[sel].reshape(-1).astype(np.int32))
        s = stats[-1]
        flops = float(lu_flops(N, P).sum() * len(freqs))
        if mode != "fp64":
            flops += 16.0 * P * float(np.mean(N.astype(np.float64) ** 2)) * s["ir_iterations"]
        upd_ms = float(np.mean([x["ms_update"] for x in stats]))
        upd_gflop = float(np.mean([x["update_gflop"] for x in stats]))
        upd_gbyte = float(np.mean([x["update_gbyte"] for x in stats]))
        upd_n = int(stats[-1]["update_launches"])
        out[mode] = {
            "value": k / (ms / 1e3), "ms_per_step": ms, "steps": n_steps, "warmup": n_warm,
            "solve_ms": float(np.mean([x["ms_solve"] for x in stats])),
            "fallback_ms": float(np.mean([x["ms_fallback"] for x in stats])),
            "rank_ms": float(np.mean(rank_ms)), "fill_s": fill_s,
            "fallbacks": int(s["fallbacks"]), "ir_steps": int(s["ir_iterations"]), "N": N,
            "lu_tflops_step": flops / (ms / 1e3) / 1e12,
            "update": {"kernel": kernel_name("tiled", mode), "launches_per_step": upd_n,
                       "ms_per_step": upd_ms, "gflop_per_step": upd_gflop, "gbyte_per_step": upd_gbyte,
                       "achieved_tflops": upd_gflop / upd_ms, "achieved_GBps": upd_gbyte / upd_ms * 1e3,
                       "avg_launch_us": 1e3 * upd_ms / max(upd_n, 1),
                       "gflop_per_launch": upd_gflop / max(upd_n, 1), "gbyte_per_launch": upd_gbyte / max(upd_n, 1)},
            "status_errors": int(np.count_nonzero(st_out.cpu().numpy() < 0)),
            "fom": fom_out.cpu().numpy(), "am": int(am_out.cpu().numpy()[0]), "sel": sel,
            "S": torch.view_as_complex(S_out.contiguous()).cpu().numpy(),
        }
        ev.close()
        del S_out
        torch.cuda.empty_cache()
    sur.close()
    return out


def graph_rate(args, torch, ev, stream, inputs, n_max, eager, n_cand, label, mode):
    """The same step captured once into a HIP graph (expand, order, evaluator,
    FP64 re-solve, FoM, argmin; bound = the batch's largest active size) and
    replayed: replays between HIP events on the capture's launch stream.
    Every replay's S is checked against the eager step's."""
    dev = torch.device("cuda:0")
    P = eager["S"].shape[-1]
    S_g = torch.empty((n_cand, eager["S"].shape[1], P, P, 2), dtype=torch.float64, device=dev)
    F_g = torch.empty(n_cand, dtype=torch.float64, device=dev)
    st_g = torch.empty(n_cand, dtype=torch.int32, device=dev)
    am_g = torch.empty(1, dtype=torch.int32, device=dev)
    g = ev.graph(*inputs, n_max, S_g, F_g, st_g, am_g)
    dS = 0.0
    g.launch(stream)  # warm-up replay
    torch.cuda.synchronize()
    dS = max(dS, float(np.abs(torch.view_as_complex(S_g.contiguous()).cpu().numpy() - eager["S"]).max()))
    e0, e1 = _events(torch, stream)
    e0.record(stream)
    for _ in range(args.leg_steps):
        g.launch(stream)
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / args.leg_steps
    dS = max(dS, float(np.abs(torch.view_as_complex(S_g.contiguous()).cpu().numpy() - eager["S"]).max()))
    am = int(am_g.cpu().numpy()[0])
    g.close()
    log(f"[{label} {mode}] graph replay: {n_cand / (ms / 1e3):.1f} evals/s ({ms:.0f} ms per replay), "
        f"max |dS| vs eager {dS:.1e}")
    return {"value": n_cand / (ms / 1e3), "ms_per_step": ms, "replays": args.leg_steps, "bound": n_max,
            "max_dS_vs_eager": dS, "argmin_equal_eager": am == eager["am"]}


def batch_leg(args, pxd, torch, spec, n_cand, modes, label, tune=False, graph=False, lu_path=0):
    """Single-flip candidates of a workload at every frequency, device
    buffers, one evaluator call per step (and, with `graph`, the same step as
    replays of a captured HIP graph)."""
    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream()
    pb = pxd.Problem.from_spec(spec)
    base = spec.base_map()
    off, cells = spec.flips()
    off, cells = off[:n_cand + 1], cells[:off[n_cand]]
    P = len(spec.ports)
    t_base, t_off, t_cells = (torch.from_numpy(a).to(dev) for a in (base, off, cells))
    out = {"candidates": n_cand, "frequencies": spec.n_freq}
    for mode in modes:
        ev = pxd.Evaluator(device=0, precision=PREC[mode], ir_max_iter=args.ir_max, half_subpanel=1, lu_path=lu_path)
        ev.load_problem(pb, spec.z0)
        ev.load_parent_problem(pb, spec.freqs)
        ev.set_fom_paper()
        tuned = None
        if tune:
            nt = min(n_cand, 96)
            rep = ev.autotune(base, off[:nt + 1], cells[:off[nt]], n_reps=1)
            tuned = [(r["lu_path"], r["tile_kb"], r["wg_per_cu"], r["schedule"], round(r["ms"], 1)) for r in rep]
            log(f"[{label} {mode}] autotuned on {nt} candidates: {tuned[:4]}")
        S_out = torch.empty((n_cand, spec.n_freq, P, P, 2), dtype=torch.float64, device=dev)
        fom_out = torch.empty(n_cand, dtype=torch.float64, device=dev)
        st_out = torch.empty(n_cand, dtype=torch.int32, device=dev)
        am_out = torch.empty(1, dtype=torch.int32, device=dev)

        def step():
            ev.evaluate_flips_device(stream, t_base, t_off, t_cells, S_out, fom_out, st_out, am_out)

        step()
        torch.cuda.synchronize()
        e0, e1 = _events(torch, stream)
        e0.record(stream)
        stats = []
        for i in range(args.leg_steps):
            step()
            stats.append(ev.stats())
        e1.record(stream)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / args.leg_steps
        s = stats[-1]
        N, _ = ev.expand(base, off, cells)
        flops = float(lu_flops(N, P).sum() * spec.n_freq)
        out[mode] = {"value": n_cand / (ms / 1e3), "ms_per_step": ms, "solve_ms": s["ms_solve"],
                     "fallback_ms": s["ms_fallback"], "fallbacks": int(s["fallbacks"]),
                     "ir_steps": int(s["ir_iterations"]), "active_size": [int(N.min()), int(N.max())],
                     "lu_tflops_step": flops / (ms / 1e3) / 1e12, "tuned": tuned,
                     "status_errors": int(np.count_nonzero(st_out.cpu().numpy() < 0)),
                     "fom": fom_out.cpu().numpy(), "am": int(am_out.cpu().numpy()[0]),
                     "S": torch.view_as_complex(S_out.contiguous()).cpu().numpy()}
        log(f"[{label} {mode}] {out[mode]['value']:.1f} evals/s ({ms:.0f} ms per step, N {N.min()}-{N.max()}, "
            f"{s['fallbacks']} to FP64, {s['ir_iterations']} refinement steps)")
        if graph and int(N.max()) <= 2048:
            try:
                out[mode]["graph"] = graph_rate(args, torch, ev, stream, (t_base, t_off, t_cells), int(N.max()),
                                                out[mode], n_cand, label, mode)
            except pxd.PxdError as e:
                log(f"[{label} {mode}] graph not timed: {e}")
                out[mode]["graph"] = {"error": str(e)}
        ev.close()
        del S_out
        torch.cuda.empty_cache()
    ref = out.get("fp64")
    for mode in modes:
        if mode != "fp64" and ref is not None:
            r = out[mode]
            r["max_dS_vs_fp64_plain"] = float(np.abs(r["S"] - ref["S"]).max())
            r["argmin_equal_fp64_plain"] = bool(r["am"] == ref["am"])
            r["speedup_vs_fp64_plain"] = r["value"] / ref["value"]
    for mode in modes:
        for key in ("S", "fom"):
            out[mode].pop(key, None)
    return out


def search_leg(args, pxd, torch):
    """The surrogate-pruned search at its working size against exhaustive
    steepest descent over every single flip, from the same start map, on the
    24 x 24 x 3 stack (101 frequencies); exact solves in the complex64 +
    FP64 refinement form.
    1. Exhaustive descent: every step solves all 1,728 single flips.  Its
       first step's exact S (1,728 maps x 101 frequencies, about 175,000
       (map, frequency) solves) is the surrogate's training set (10 % held
       out), encoded on the device.
    2. Training: BF16 products, AdamW, batches of 64; held-out loss and the
       rank correlation of predicted and exact FoM on the held-out maps.
    3. Pruned descent: each step the surrogate ranks all 1,728 singles and
       1,492,128 pairs, its top 32 are solved exactly and the best strict
       improvement is accepted; when none improves every single flip is
       solved exactly (fallback); every exact solve fine-tunes the network.
    Reported: FoM, wall time and exact solves after each step of both."""
    from paper_2412_17617_amd.tree_search import descent
    from synth import get_spec

    dev = torch.device("cuda:0")
    spec = get_spec("stress24")
    pb = pxd.Problem.from_spec(spec)
    ev = pxd.Evaluator(device=0, precision=pxd.PREC_MIXED32, ir_max_iter=args.ir_max, lu_path=pxd.PATH_TILED)
    ev.load_problem(pb, spec.z0)
    ev.load_parent_problem(pb, spec.freqs)
    ev.set_fom_paper()
    n = spec.n_cells
    s_off, s_cells = np.arange(n + 1, dtype=np.int32), np.arange(n, dtype=np.int32)
    start = spec.base_map()
    entries = ((0, 0), (1, 0), (2, 0), (2, 1))
    sur = pxd.Surrogate(spec.n_layers, spec.ny, spec.nx, spec.freqs, spec.freqs[0], spec.freqs[-1],
                        entries=entries, precision=pxd.SUR_BF16, max_batch=2048)
    sur.init_params(4)
    first = {}

    def keep_first(maps, S):
        if not first:
            first["maps"], first["S"] = maps, S
        log(f"[search24] exhaustive: {len(maps)} moves solved exactly ({time.time() - t0:.0f} s)")

    t0 = time.time()
    ex = descent(ev, start, s_off, s_cells, args.search_steps, learn=keep_first)
    t_ex = time.time() - t0
    log(f"[search24] exhaustive: FoM {ex.start_fom:.4g} -> {ex.fom:.4g} in "
        f"{len(ex.trace)} steps, {ex.exact_solves} exact solves, {t_ex:.0f} s")
    # training set: the first exhaustive step's exact solves
    maps, S = first["maps"], first["S"]
    t_S = torch.from_numpy(np.ascontiguousarray(np.stack([S.real, S.imag], -1))).to(dev)
    tgt = torch.empty((len(maps), spec.n_freq, 3 * len(entries)), dtype=torch.float32, device=dev)
    sur.encode_device(t_S, tgt)
    del t_S
    t_maps = torch.from_numpy(maps).to(dev)
    perm = np.random.default_rng(4).permutation(len(maps))
    n_held = len(maps) // 10
    held, train = perm[:n_held], perm[n_held:]
    loss = torch.zeros(1, dtype=torch.float32, device=dev)

    def held_loss():
        hi = torch.from_numpy(held).to(dev)
        sur.gradient(t_maps[hi[:512]], tgt[hi[:512]], None, loss)
        return float(loss.item())

    def fit(idx, steps, lr, seed):
        rng = np.random.default_rng(seed)
        for st in range(steps):
            b = torch.from_numpy(rng.choice(idx, 64, replace=len(idx) < 64)).to(dev)
            sur.train_step(t_maps[b], tgt[b], lr=lr, weight_decay=1e-4)

    loss0 = held_loss()
    t1 = time.time()
    fit(train, args.search_train_steps, 2e-3, 5)
    torch.cuda.synchronize()
    t_train = time.time() - t1
    loss1 = held_loss()
    # ranking quality on the held-out single flips of the start map
    cand = maps ^ start[None, :]
    h_cells = np.array([int(np.nonzero(cand[i])[0][0]) for i in held], np.int32)
    fp = torch.empty(len(held), dtype=torch.float64, device=dev)
    sur.rank(ev, torch.from_numpy(start).to(dev), torch.from_numpy(np.arange(len(held) + 1, dtype=np.int32)).to(dev),
             torch.from_numpy(h_cells).to(dev), 0, fp, None)
    _, F_exact, _, _ = ev.evaluate_flips(start, np.arange(len(held) + 1, dtype=np.int32), h_cells, want_S=False)
    ra = np.argsort(np.argsort(fp.cpu().numpy()))
    rb = np.argsort(np.argsort(F_exact))
    spearman = float(np.corrcoef(ra, rb)[0, 1])
    log(f"[search24] surrogate trained on {len(train)} maps x {spec.n_freq} frequencies in {t_train:.1f} s: "
        f"held-out loss {loss0:.3g} -> {loss1:.3g}, rank correlation {spearman:.3f}")
    # pruned descent: singles and pairs ranked, top 32 exact, singles as fallback
    iu, ju = np.triu_indices(n, 1)
    a_off = np.concatenate([s_off, n + 2 * np.arange(1, len(iu) + 1)]).astype(np.int32)
    a_cells = np.concatenate([s_cells, np.stack([iu, ju], 1).ravel()]).astype(np.int32)
    t_aoff, t_acells = torch.from_numpy(a_off).to(dev), torch.from_numpy(a_cells).to(dev)
    fp_all = torch.empty(len(a_off) - 1, dtype=torch.float64, device=dev)
    top = torch.empty(32, dtype=torch.int32, device=dev)

    def ranker(m, o, c):
        sur.rank(ev, torch.from_numpy(m).to(dev), t_aoff, t_acells, 32, fp_all, top)
        torch.cuda.synchronize()
        return top.cpu().numpy()

    seen_m, seen_t = [t_maps[torch.from_numpy(train).to(dev)]], [tgt[torch.from_numpy(train).to(dev)]]

    def learn(new_maps, S_new):
        log(f"[search24] pruned: {len(new_maps)} moves solved exactly ({time.time() - t2:.0f} s)")
        tS = torch.from_numpy(np.ascontiguousarray(np.stack([S_new.real, S_new.imag], -1))).to(dev)
        tt = torch.empty((len(new_maps), spec.n_freq, 3 * len(entries)), dtype=torch.float32, device=dev)
        sur.encode_device(tS, tt)
        seen_m.append(torch.from_numpy(new_maps).to(dev))
        seen_t.append(tt)
        allm, allt = torch.cat(seen_m), torch.cat(seen_t)
        rng = np.random.default_rng(len(allm))
        for _ in range(args.search_finetune_steps):  # half of each batch from the newest solves
            b_new = torch.from_numpy(rng.integers(len(allm) - len(new_maps), len(allm), 32)).to(dev)
            b_old = torch.from_numpy(rng.integers(0, len(allm), 32)).to(dev)
            b = torch.cat([b_new, b_old])
            sur.train_step(allm[b], allt[b], lr=5e-4, weight_decay=1e-4)

    t2 = time.time()
    pr = descent(ev, start, a_off, a_cells, args.search_steps, ranker=ranker, top_k=32, fallback=(s_off, s_cells),
                 learn=learn)
    t_pr = time.time() - t2
    log(f"[search24] pruned: FoM {pr.fom:.4g} in {len(pr.trace)} steps ({[t[3] for t in pr.trace]}), "
        f"{pr.exact_solves} exact solves, {t_pr:.0f} s (+ {t_train:.0f} s training)")
    sur.close()
    ev.close()
    torch.cuda.empty_cache()

    def traj(r):
        return [{"s": round(t[0], 2), "exact_solves": int(t[1]), "fom": float(t[2]), "step": t[3]} for t in r.trace]

    return {"workload": "24x24x3 stack, 101 frequencies; start = the workload's Bernoulli(0.5) map",
            "exact_form": "complex64 LU + FP64 refinement (tiled, lock step)",
            "start_fom": ex.start_fom,
            "exhaustive": {"moves": int(n), "final_fom": ex.fom, "exact_solves": ex.exact_solves, "seconds": t_ex,
                           "trajectory": traj(ex)},
            "surrogate": {"train_maps": int(len(train)), "held_out_maps": int(n_held), "frequencies": spec.n_freq,
                          "train_steps": args.search_train_steps, "batch": 64, "train_seconds": t_train,
                          "held_out_loss_before": loss0, "held_out_loss_after": loss1,
                          "held_out_rank_correlation": spearman},
            "pruned": {"ranked_moves": int(len(a_off) - 1), "verified": 32, "final_fom": pr.fom,
                       "exact_solves": pr.exact_solves, "seconds": t_pr, "trajectory": traj(pr)}}


def lowrank_leg(args, pxd, spec):
    """All single flips of the 20 x 20 x 2 map through the low-rank flip
    evaluation (FP64, from the cached inverse of the base map), host buffers."""
    pb = pxd.Problem.from_spec(spec)
    base = spec.base_map()
    off, cells = spec.flips()
    C = len(off) - 1
    ev = pxd.Evaluator(device=0, precision=pxd.PREC_FP64)
    ev.load_problem(pb, spec.z0)
    ev.load_parent_problem(pb, spec.freqs)
    ev.set_fom_paper()
    t0 = time.perf_counter()
    ev.evaluate_flips_lowrank(base, off, cells, want_S=False)
    first_ms = (time.perf_counter() - t0) * 1e3
    s_first = ev.stats()
    t0 = time.perf_counter()
    k_ms = []
    for i in range(args.leg_steps):
        ev.evaluate_flips_lowrank(base, off, cells, want_S=False)
        k_ms.append(ev.stats()["ms_solve"])
    ms = (time.perf_counter() - t0) * 1e3 / args.leg_steps
    st = ev.stats()
    ev.close()
    log(f"[lowrank] {C / (ms / 1e3):.0f} evals/s ({ms:.1f} ms per step, kernel {np.mean(k_ms):.1f} ms, base inverse "
        f"{s_first['ms_base_inverse']:.0f} ms once)")
    return {"value": C / (ms / 1e3), "unit": "evals/s", "ms_per_step": ms, "kernel_ms": float(np.mean(k_ms)),
            "first_call_ms": first_ms, "ms_base_inverse": s_first["ms_base_inverse"],
            "base_reused": int(st["base_reused"]), "dense_fallback_items": int(st["fallbacks"]),
            "io": "host buffers (flips up, FoM down inside the timed step)"}


def surrogate_leg(args, pxd, spec, torch):
    """Ranking by the CNN surrogate at its working size: a 3 x 24 x 24 map
    (channels 32-64, hidden 256, BF16 products) scored on 101 frequencies with
    the context's FoM table; every single flip and every pair of cells, then
    the top 32.  Random-init weights (throughput only)."""
    dev = torch.device("cuda:0")
    pb = pxd.Problem.from_spec(spec)
    ev = pxd.Evaluator(device=0)
    ev.load_problem(pb, spec.z0)
    ev.load_parent_problem(pb, spec.freqs)
    ev.set_fom_paper()
    L, ny, nx = spec.n_layers, spec.ny, spec.nx
    n = L * ny * nx
    sur = pxd.Surrogate(L, ny, nx, spec.freqs, spec.freqs[0], spec.freqs[-1], precision=pxd.SUR_BF16, max_batch=2048)
    sur.init_params(17)
    path = {pxd.SUR_INFER_FUSED: "fused", pxd.SUR_INFER_GENERIC: "generic"}[sur.inference]
    iu, ju = np.triu_indices(n, 1)
    C = n + len(iu)
    off = np.concatenate([np.arange(n + 1), n + 2 * np.arange(1, len(iu) + 1)]).astype(np.int32)
    cells = np.concatenate([np.arange(n), np.stack([iu, ju], 1).ravel()]).astype(np.int32)
    base = spec.base_map()
    t_base, t_off, t_cells = (torch.from_numpy(a).to(dev) for a in (base, off, cells))
    fp = torch.empty(C, dtype=torch.float64, device=dev)
    top = torch.empty(32, dtype=torch.int32, device=dev)
    stream = torch.cuda.current_stream()
    sur.rank(ev, t_base, t_off, t_cells, 32, fp, top, stream)
    torch.cuda.synchronize()
    e0, e1 = _events(torch, stream)
    e0.record(stream)
    sur.rank(ev, t_base, t_off, t_cells, 32, fp, top, stream)
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    fp_h, top_h = fp.cpu().numpy(), top.cpu().numpy()  # checked on the host: no other kernels in a profile
    ok = bool(np.isfinite(fp_h).all()) and int(top_h.min()) >= 0
    generic = None
    if sur.inference == pxd.SUR_INFER_FUSED:
        # the same ranking through the training path's products, for comparison
        gen = pxd.Surrogate(L, ny, nx, spec.freqs, spec.freqs[0], spec.freqs[-1], precision=pxd.SUR_BF16,
                            max_batch=2048, inference=pxd.SUR_INFER_GENERIC)
        gen.init_params(17)
        fp_g = torch.empty_like(fp)
        top_g = torch.empty_like(top)
        gen.rank(ev, t_base, t_off, t_cells, 32, fp_g, top_g, stream)
        e0.record(stream)
        gen.rank(ev, t_base, t_off, t_cells, 32, fp_g, top_g, stream)
        e1.record(stream)
        torch.cuda.synchronize()
        fp_gh = fp_g.cpu().numpy()
        dev_rel = float(np.max(np.abs(fp_h - fp_gh) / np.abs(fp_gh)))
        same_top = int(np.intersect1d(top_h, top_g.cpu().numpy()).size)
        generic = {"ms": e0.elapsed_time(e1), "max_rel_fom_dev": dev_rel, "top32_overlap": same_top}
        gen.close()
    ch = (L, 32, 32, 64, 64)
    px = (ny * nx, ny * nx, ny * nx // 4, ny * nx // 4)
    trunk = sum(2 * 9 * ch[i] * ch[i + 1] * px[i] for i in range(4))
    feat = 64 * (ny // 4) * (nx // 4)
    flops = C * (trunk + 2 * feat * 256 + spec.n_freq * 2 * 256 * 9)
    sur.close()
    ev.close()
    log(f"[surrogate] ranked {C:,} candidates in {ms:.0f} ms ({flops / (ms / 1e3) / 1e12:.1f} TFLOP/s, {path}"
        + (f"; generic products {generic['ms']:.0f} ms)" if generic else ")"))
    return {"value": C / (ms / 1e3), "unit": "maps/s", "ms": ms, "candidates": C,
            "workload": f"every single flip and cell pair of a {L}x{ny}x{nx} map, {spec.n_freq} frequencies, top 32",
            "precision": "bf16 products, fp32 accumulation", "weights": "random init (throughput only)",
            "flops_per_call": flops, "achieved_TFLOPs": flops / (ms / 1e3) / 1e12, "peak_TFLOPs": 2500.0,
            "top_valid": ok, "inference": path, "generic_products": generic}


def run_legs(args, pxd, torch, legs):
    """The extra legs named in `legs`, each an object of the JSON line."""
    from synth import get_spec

    extra = {}
    if "stress24" in legs:
        extra["stress24"] = batch_leg(args, pxd, torch, get_spec("stress24"), 64, ["fp64", "mixed32", "bf16x3"],
                                      "stress24", lu_path=pxd.PATH_TILED)
    if "batched20" in legs:
        extra["batched20"] = batch_leg(args, pxd, torch, get_spec("batched20"), 800, ["fp64", "mixed32", "bf16x3"],
                                       "batched20", tune=True, graph=True)
    if "surrogate" in legs:
        extra["surrogate"] = surrogate_leg(args, pxd, get_spec("stress24"), torch)
    if "search24" in legs:
        extra["search24"] = search_leg(args, pxd, torch)
    if "lowrank" in legs:
        extra["lowrank"] = lowrank_leg(args, pxd, get_spec("batched20"))
    return extra


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="ceiling32")
    ap.add_argument("--top-k", type=int, default=32)
    ap.add_argument("--forms", default="mixed32,bf16x3",
                    help="mixed-precision forms timed beside FP64 plain on the headline step (the last one gets the "
                         "full step count)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="first copy 1 GiB device to device: a reference kernel of known traffic for the byte "
                         "counters (FETCH_SIZE / WRITE_SIZE)")
    ap.add_argument("--ir-max", type=int, default=10)
    ap.add_argument("--leg-steps", type=int, default=1)
    ap.add_argument("--search-steps", type=int, default=4, help="search24 leg: descent steps per method")
    ap.add_argument("--search-train-steps", type=int, default=1500, help="search24 leg: initial training steps")
    ap.add_argument("--search-finetune-steps", type=int, default=40, help="search24 leg: steps per new solve batch")
    ap.add_argument("--no-headline", action="store_true",
                    help="run only the extra legs (no CPU baseline) and print their objects: a profiling aid, "
                         "not the benchmark line")
    ap.add_argument("--legs", default="stress24,batched20,surrogate,lowrank",
                    help="comma list of extra legs (stress24, batched20, surrogate, lowrank; search24, the "
                         "surrogate-pruned against exhaustive search, about 8 minutes, is not in the default) or 'none'")
    ap.add_argument("--cpu-seconds", type=float, default=20.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py: this build runs on one GPU; --gpus must be 1 (the path shards by frequency "
              "across GPUs by design, but no multi-GPU run is part of this build)", file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_2412_17617_amd import pxd
    from synth import get_spec

    legs = [] if args.legs == "none" else [x for x in args.legs.split(",") if x]
    if args.copy_calibration:
        src = torch.ones(2 ** 27, dtype=torch.float64, device="cuda:0")
        torch.cuda.synchronize()
        dst = src.clone()  # reads 1 GiB, writes 1 GiB
        torch.cuda.synchronize()
        del src, dst
        log("copy calibration: 1 GiB device-to-device copy done")
    spec = get_spec(args.workload)
    if args.no_headline:
        print(json.dumps(run_legs(args, pxd, torch, legs)), flush=True)
        return
    log(f"workload {spec.name}: {spec.n_layers} layers {spec.nx}x{spec.ny}, {spec.n_freq} frequencies")

    # the CPU baseline's oracle fills (untimed) run beside the GPU legs
    pool = concurrent.futures.ThreadPoolExecutor(1)
    prep = None
    if not args.no_cpu_baseline:
        from oracle import search

        jobs = []
        base = spec.base_map()
        off, cells = spec.flips()
        jobs.append(("headline", spec, search.candidate_maps(base, off[:2], cells[:off[1]]),
                     int(np.argmin(np.abs(spec.freqs - 5.5e9))), True))
        for name, nc in (("stress24", 2), ("batched20", 8)):
            s2 = get_spec(name)
            b2 = s2.base_map()
            o2, c2 = s2.flips()
            jobs.append((name, s2, search.candidate_maps(b2, o2[:nc + 1], c2[:o2[nc]]),
                         int(np.argmin(np.abs(s2.freqs - 5.5e9))), name != "batched20"))
        prep = pool.submit(oracle_prepare, jobs)

    modes = ["fp64"] + [m for m in args.forms.split(",") if m]
    head = headline_leg(args, pxd, torch, spec, modes)
    extra = run_legs(args, pxd, torch, legs)

    f64 = head["fp64"]
    forms = {}
    for mode in modes:
        r = head[mode]
        u = r["update"]
        peak = PEAK_TFLOPS[mode]
        forms[mode] = {
            "value": r["value"], "ms_per_step": r["ms_per_step"], "steps": r["steps"], "warmup": r["warmup"],
            "fallback_items": r["fallbacks"], "refinement_steps": r["ir_steps"], "status_errors": r["status_errors"],
            "lu_tflops_whole_step": r["lu_tflops_step"],
            "step_breakdown_ms": {"solve": r["solve_ms"], "fp64_fallback": r["fallback_ms"],
                                  "trailing_updates": u["ms_per_step"], "surrogate_rank": r["rank_ms"]},
            "update_kernel": {"kernel": u["kernel"], "achieved_TFLOPs": u["achieved_tflops"], "peak_TFLOPs": peak,
                              "frac": u["achieved_tflops"] / peak, "achieved_GBps": u["achieved_GBps"],
                              "hbm_frac": u["achieved_GBps"] / 8000.0, "launches_per_step": u["launches_per_step"],
                              "avg_launch_us": u["avg_launch_us"]},
        }
        if mode != "fp64":
            forms[mode].update({
                "max_dS_vs_fp64_plain": float(np.abs(r["S"] - f64["S"]).max()),
                "argmin_equal_fp64_plain": bool(r["am"] == f64["am"]),
                "fom_rel_dev_vs_fp64_plain": float(np.max(np.abs(r["fom"] - f64["fom"]) / f64["fom"])),
                "same_candidates_as_fp64_plain": bool(np.array_equal(r["sel"], f64["sel"])),
                "speedup_vs_fp64_plain": r["value"] / f64["value"]})
    # the chosen form: the fastest one that meets the metric's bar against FP64 plain
    valid = [m for m in modes if m != "fp64" and forms[m]["max_dS_vs_fp64_plain"] <= 1e-4
             and forms[m]["argmin_equal_fp64_plain"] and forms[m]["status_errors"] == 0]
    chosen = max(valid, key=lambda m: forms[m]["value"]) if valid else "fp64"
    r = head[chosen]
    N = r["N"]
    upd = r["update"]
    out = {
        "metric": "pixel-map evals/sec (all freqs, S+FoM) vs FP64 plain, at max |dS|<=1e-4",
        "value": r["value"],
        "unit": "evals/s",
        "n_gpus": 1,
        "steps": r["steps"],
        "warmup": r["warmup"],
        "ms_per_step": r["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"fp64": "f64", "mixed32": "f32+f64", "bf16x3": "bf16+f32+f64"}[chosen],
        "data": "synthetic",
        "config": {
            "workload": f"{spec.name}: {spec.n_layers} layers {spec.nx}x{spec.ny} pixels, M={pb_M(pxd, spec)}, "
                        f"{spec.n_freq} freqs {spec.f_lo / 1e9:g}-{spec.f_hi / 1e9:g} GHz; one search step: "
                        f"surrogate ranks {head['candidates_ranked']} 3x3 pair flips, top {head['top_k']} "
                        f"evaluated exactly",
            "form": chosen,
            "precision": {"fp64": "complex128 LU (FP64 plain)",
                          "mixed32": "complex64 LU + FP64 refinement (FP64 fallback)",
                          "bf16x3": "complex64 LU with split-BF16 trailing updates + FP64 refinement "
                                    "(FP64 fallback)"}[chosen],
            "candidates_per_step": head["top_k"],
            "frequencies": spec.n_freq,
            "active_size": [int(N.min()), int(N.max())],
            "lu_path": "tiled",
            "status_errors": r["status_errors"],
            "fallback_items": r["fallbacks"],
            "refinement_steps": r["ir_steps"],
            "surrogate_rank_ms": r["rank_ms"],
            "surrogate_weights": "random init (the prefilter's throughput, not its ranking quality)",
        },
        "roofline": {
            "bound": "mfma",
            "achieved": upd["achieved_tflops"],
            "peak": PEAK_TFLOPS[chosen],
            "unit": "TFLOP/s",
            "frac": upd["achieved_tflops"] / PEAK_TFLOPS[chosen],
            "traffic": None,
            "kernel": upd["kernel"],
            "launches_per_step": upd["launches_per_step"],
            "avg_launch_us": upd["avg_launch_us"],
            "gflop_per_launch": upd["gflop_per_launch"],
            "algorithmic_GBps": upd["achieved_GBps"],
            "basis": "algorithmic 8 kb (N - Kend)(ncols - Kend) flops per item and block column, summed over the "
                     "step's trailing-update launches, / their summed duration (HIP event pair around each launch "
                     "on the evaluation stream); peak of the MFMA data type the kernel issues",
        },
        "forms": forms,
        "speedup_vs_fp64_plain": r["value"] / f64["value"],
        "parent_fill_gpu_s": r["fill_s"],
    }
    if chosen != "fp64":
        for key in ("max_dS_vs_fp64_plain", "argmin_equal_fp64_plain", "fom_rel_dev_vs_fp64_plain",
                    "same_candidates_as_fp64_plain"):
            out["config"][key] = forms[chosen][key]
    bound, floor_compute_us, floor_memory_us, issued = binding_roof(chosen, upd["gflop_per_launch"],
                                                                    upd["gbyte_per_launch"])
    ro = out["roofline"]
    ro.update({"compute_floor_us": floor_compute_us, "memory_floor_us": floor_memory_us,
               "mfma_issued_TFLOPs": issued * upd["achieved_tflops"],
               "mfma_issued_frac": issued * upd["achieved_tflops"] / PEAK_TFLOPS[chosen],
               "hbm_frac_algorithmic": upd["achieved_GBps"] / HBM_PEAK_GBPS})
    if bound == "hbm":
        ro.update({"bound": "hbm", "achieved": upd["achieved_GBps"], "peak": HBM_PEAK_GBPS, "unit": "GB/s",
                   "frac": upd["achieved_GBps"] / HBM_PEAK_GBPS})
        ro["basis"] = ("algorithmic bytes: the element size times (2 m n + kb m + kb n) per item and block column "
                       "(C read and written once, L21 and U12 read once; m = N - Kend rows, n = trailing columns), "
                       "summed over the "
                       "step's trailing-update launches, / their summed duration (HIP event pair around each launch "
                       "on the evaluation stream); HBM-bound because these bytes at 8 TB/s take longer than the "
                       "issued MFMA flops at their dense peak")
    tr = measured_traffic(spec.name, upd["kernel"], head["top_k"] * spec.n_freq)
    if tr is not None:
        out["roofline"]["traffic"] = tr["hbm_bytes_per_launch"]
        out["roofline"]["traffic_unit"] = "bytes/launch (average)"
    out.update(extra)
    if prep is not None:
        prepared = prep.result()
        cb = oracle_time(prepared, args.cpu_seconds)
        cb1 = oracle_time(prepared[:1], args.cpu_seconds / 3, threads=1)
        import platform

        model = "unknown"
        try:
            with open("/proc/cpuinfo") as fh:
                for line in fh:
                    if line.startswith("model name"):
                        model = line.split(":", 1)[1].strip()
                        break
        except OSError:
            pass
        out["cpu_baseline"] = dict(cb["headline"])
        affinity = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else None
        out["cpu_baseline"].update({"nproc": os.cpu_count(), "affinity_cpus": affinity, "cpu_model": model,
                                    "machine": platform.machine(),
                                    "one_thread": cb1["headline"],
                                    "other_workloads": {k: v for k, v in cb.items() if k != "headline"}})
    pool.shutdown()
    print(json.dumps(out), flush=True)


def pb_M(pxd, spec):
    return pxd.Problem.from_spec(spec).M


if __name__ == "__main__":
    main()
