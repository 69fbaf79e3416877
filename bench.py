"""Benchmark: H^2 factorization + refined solve on one MI355X.

A step is one pass of the hot path over the resident H^2 matrix of the
headline workload (64^3 cube grid, N = 262144, leaf 64, eta = 1, eps = 1e-4):
the level-by-level factorization followed by one right-hand side solved and
iteratively refined to a relative residual of 1e-8 against the H^2 matrix.
Construction of the H^2 representation is setup (untimed), as in the paper.
Both arithmetic forms run on the same matrix: FP64, and the mixed form
(complex FP32 Schur updates and projections, FP64 elsewhere), each refined to
the same residual.

Prints one JSON line.  `value` = unknowns per second of whole steps of the
faster form (N * steps / timed seconds); both forms' rates, factor times per
level, warm solve medians (1 RHS refined, 1 RHS plain, 64 RHS plain), the
Schur flush roofline, every kernel family's roofline, a 32^3 leg, the
64-problem batching leg and the CPU oracle's rate on the small workload are
reported beside it.
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

PEAK_FP64_TFLOPS = 78.6   # MI355X dense FP64 (matrix and vector)
PEAK_FP32_TFLOPS = 157.3  # MI355X dense FP32 (matrix)
PEAK_HBM_GBS = 8000.0


def cpu_baseline() -> dict:
    """The oracle on the small cube workload itself (16^3, N = 4096, leaf 32, eta 1,
    eps 1e-6): factor + 1 RHS refined to 1e-8, construction excluded (timed apart), once
    with every host thread the BLAS may use and once limited to one thread (the paper's
    timings are single-core)."""
    from threadpoolctl import threadpool_info, threadpool_limits
    from oracle import h2_oracle as O
    from paper_1703_06155_amd import inputs as I

    pr = I.config(0)
    t0 = time.perf_counter()
    H = O.construct(pr.points, pr.k, pr.h, pr.chi, pr.leaf, pr.eta, pr.eps)
    construct_s = time.perf_counter() - t0

    def run():
        t0 = time.perf_counter()
        Fz = O.factor(H)
        t1 = time.perf_counter()
        _, hist = O.refine(Fz, pr.rhs[:, 0], tol=1e-8, max_iter=10)
        t2 = time.perf_counter()
        return t1 - t0, t2 - t1, hist

    threads = max([i.get("num_threads", 1) for i in threadpool_info()] + [1])
    f_all, s_all, hist = run()
    with threadpool_limits(limits=1):
        f_one, s_one, _ = run()
    sample = (f"the oracle on the 16^3 cube workload (N={pr.n}, leaf 32, eta 1, eps 1e-6): factor + 1 RHS "
              f"refined to {hist[-1]:.1e}; construction ({construct_s:.1f} s) excluded; os.cpu_count() = "
              f"{os.cpu_count()}, BLAS threads = {threads}")
    print(f"# cpu baseline done ({f_all + s_all:.1f} s all threads, {f_one + s_one:.1f} s one thread)",
          file=sys.stderr, flush=True)
    return {"value": pr.n / (f_all + s_all), "unit": "unknowns/s", "cores": int(threads), "kind": "oracle",
            "sample": sample, "factor_s": f_all, "solve_refined_s": s_all, "construct_s": construct_s,
            "os_cpu_count": os.cpu_count(),
            "single_thread": {"value": pr.n / (f_one + s_one), "unit": "unknowns/s", "cores": 1,
                              "factor_s": f_one, "solve_refined_s": s_one}}


# HBM bytes per Schur flush (flush kernel + partial-tile reduction), keyed by
# (cube side, form), from rocprofv3 FETCH_SIZE and WRITE_SIZE counters scaled by a
# 1 GiB copy (the summaries under profiles/); valid only for that workload, its fixed
# execution settings (CUBE64_SETTINGS) and the kernel sources hashed here.
SCHUR_TRAFFIC = {(64, "mixed"): {"sources_sha256": "583c2b91efba2d15f0094b054d3bf31082d88c5557bfbe1fa44f12786e4d14f0",
                                   "bytes_per_launch": 12904049067},
                 (64, "fp64"): {"sources_sha256": "583c2b91efba2d15f0094b054d3bf31082d88c5557bfbe1fa44f12786e4d14f0",
                                  "bytes_per_launch": 13125095600}}


def kernel_sources_sha256() -> str:
    """Hash of the Schur flush kernel's source: the tile engine header and the
    kernel's own section of the kernel file."""
    import hashlib
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_1703_06155_amd", "csrc")
    with open(os.path.join(csrc, "h2_device.hpp"), "rb") as fh:
        h.update(fh.read())
    with open(os.path.join(csrc, "h2_kernels.hip"), "rb") as fh:
        src = fh.read()
    a, b = src.index(b"struct SchurTerm"), src.index(b"void launch_schur(")
    h.update(src[a:b])
    return h.hexdigest()


LATENCY_BOUND = ("step0_basis", "partial_lu")


def kernel_rooflines(led: dict, solve1_ms: float = None, matvec_ms: float = None, mixed: bool = False) -> dict:
    """Roofline position of every kernel family of one FP64 factorization (HIP-event
    intervals of a factorization run with kernel timing on, algorithmic flops and bytes
    of the library's ledger), of the 1-RHS forward + backward sweeps (bytes of the
    factors they read) and of one H^2 matvec.  Both fractions are given; `bound` names
    the roof the kernel's intensity points to, or "latency" for the per-cluster
    eigen-solver and LU kernels, which are bound by dependent steps."""
    ridge = PEAK_FP64_TFLOPS * 1e12 / (PEAK_HBM_GBS * 1e9)
    out = {}
    from paper_1703_06155_amd import KERNEL_FAMILIES
    for fam in KERNEL_FAMILIES:
        ms, flops, nbytes = led[fam]
        if ms <= 0:
            continue
        tf = flops / (ms * 1e-3) / 1e12
        gbs = nbytes / (ms * 1e-3) / 1e9
        inten = flops / nbytes if nbytes > 0 else float("inf")
        bound = "latency" if fam in LATENCY_BOUND else ("mfma" if inten >= ridge else "hbm")
        out[fam] = {"ms": float(ms), "gflop": flops / 1e9, "gbytes": nbytes / 1e9, "bound": bound,
                    "tflops": tf, "mfma_frac": tf / PEAK_FP64_TFLOPS, "gbs": gbs, "hbm_frac": gbs / PEAK_HBM_GBS}
        if mixed:
            # complex FP32 terms where the routing allows, FP64 elsewhere: both peaks bound the rate
            # (the ledger's bytes are those of the FP64 form)
            out[fam]["mfma_frac_fp32_peak"] = tf / PEAK_FP32_TFLOPS
    if solve1_ms is None:
        return out
    for fam, ms, nbytes in (("sweeps_1rhs", solve1_ms, led["sweep_bytes_per_rhs"]),
                            ("matvec_1rhs", matvec_ms, led["matvec_bytes"])):
        gbs = nbytes / (ms * 1e-3) / 1e9
        out[fam] = {"ms": ms, "gbytes": nbytes / 1e9, "bound": "hbm", "gbs": gbs, "hbm_frac": gbs / PEAK_HBM_GBS}
    return out


def schur_roofline(flops: float, nbytes: float, ms: float, launches: int, grid: int, form: str = "fp64",
                   fixed_settings: bool = True) -> dict:
    """Roofline of the Schur flush (the FP64 flush kernel plus the kernel that adds
    the partial tiles of split target blocks) from the algorithmic ledger and the
    flush durations the library measured with HIP events on its stream; one
    "launch" is one flush of a colour's pending updates."""
    per_launch_s = ms * 1e-3 / max(launches, 1)
    ridge = PEAK_FP64_TFLOPS * 1e12 / (PEAK_HBM_GBS * 1e9)  # flop / byte
    intensity = flops / nbytes if nbytes > 0 else float("inf")
    traffic = None
    rec = SCHUR_TRAFFIC.get((grid, form))
    if rec and fixed_settings and rec["sources_sha256"] == kernel_sources_sha256():
        traffic = rec["bytes_per_launch"]
    if intensity >= ridge:
        achieved = flops / max(launches, 1) / per_launch_s / 1e12 if ms > 0 else 0.0
        out = {"bound": "mfma", "achieved": achieved, "peak": PEAK_FP64_TFLOPS, "unit": "TFLOP/s"}
    else:
        achieved = nbytes / max(launches, 1) / per_launch_s / 1e9 if ms > 0 else 0.0
        out = {"bound": "hbm", "achieved": achieved, "peak": PEAK_HBM_GBS, "unit": "GB/s"}
    kernel = "k_schur_fp64 + k_schur_reduce" if form == "fp64" else "k_schur_mixed / k_schur_fp64 (per level) + k_schur_reduce"
    out.update({"frac": out["achieved"] / out["peak"], "traffic": traffic, "kernel": kernel,
                "launches": launches, "flops_per_launch": flops / max(launches, 1),
                "bytes_per_launch_algorithmic": nbytes / max(launches, 1), "intensity_flop_per_byte": intensity,
                "avg_launch_ms": ms / max(launches, 1)})
    return out


COPY_BYTES = 1 << 30      # one direction of the calibration copy


def copy_calibration(torch):
    """A plain 1 GiB device-to-device copy, 5 times: FETCH_SIZE / WRITE_SIZE of
    its kernel divided by 1 GiB is the factor that turns the counters of any
    other kernel into bytes."""
    src = torch.ones(COPY_BYTES // 8, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(5):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes": COPY_BYTES, "launches": 5}), flush=True)


def batch_leg(torch, h2, I, chunk: int) -> dict:
    """Independent box problems (sides U{12..32} cells, leaf 48, eps 1e-4, 16 plane-wave
    right-hand sides each): factor + 16-RHS solve refined to 1e-8, one problem at a time
    in FP64 versus batched (h2_factor_batch_mode / h2_solve_batch_mode): fused launches
    across problems (factorization and sweeps) in FP64 and in the mixed form, and one
    stream per problem (graph-replayed sweeps) in FP64, in chunks of `chunk` problems
    whose handles are released after their solve.  Every run reports the largest final
    residual over the problems."""
    probs = I.batch_problems(count=64, nrhs=16)
    n_total = sum(pr.n for pr in probs)

    def run(mode, precision: str) -> tuple:
        batched = mode is not None
        elapsed, worst, iters = 0.0, 0.0, 0
        for c0 in range(0, len(probs), chunk):
            part = probs[c0:c0 + chunk]
            hs = [h2.H2(pr.points, pr.k, pr.h, pr.chi, pr.leaf, pr.eta, pr.eps, precision=precision)
                  for pr in part]
            rhs = [torch.from_numpy(pr.rhs.copy()).cuda() for pr in part]
            for G in hs:
                G.set_sweep_graph(mode == "streams")
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            if batched:
                h2.factor_batch(hs, mode=mode)
                _, infos = h2.solve_batch(hs, rhs, tol=1e-8, max_iter=20, info=True, mode=mode)
            else:
                infos = []
                for G, b in zip(hs, rhs):
                    G.factor()
                    infos.append(G.solve(b, tol=1e-8, max_iter=20, info=True)[1])
            torch.cuda.synchronize()
            elapsed += time.perf_counter() - t0
            worst = max([worst] + [i["rel_residual"] for i in infos])
            iters = max([iters] + [i["iterations"] for i in infos])
            for G in hs:
                G.close()
            # the handles' memory went back to PyTorch's cache: hand it to the device before the
            # next chunk allocates buffers of other sizes (untimed)
            del hs, rhs
            torch.cuda.empty_cache()
        return elapsed, worst, iters

    t_seq, r_seq, it_seq = run(None, "fp64")
    t_bat, r_bat, it_bat = run("fused", "fp64")
    t_str, r_str, it_str = run("streams", "fp64")
    t_mix, r_mix, it_mix = run("fused", "mixed")
    return {"workload": "64 box problems, sides U{12..32}, leaf 48, eps 1e-4, 16 RHS each, refined to 1e-8",
            "unknowns": n_total, "chunk": chunk, "sequential_s": t_seq, "batched_s": t_bat,
            "sequential_unknowns_per_s": n_total / t_seq, "batched_unknowns_per_s": n_total / t_bat,
            "speedup": t_seq / t_bat,
            "batched_streams_s": t_str, "batched_streams_unknowns_per_s": n_total / t_str,
            "batched_mixed_s": t_mix, "batched_mixed_unknowns_per_s": n_total / t_mix,
            "mixed_batched_vs_fp64_sequential": t_seq / t_mix, "mixed_batched_vs_fp64_batched": t_bat / t_mix,
            "max_rel_residual": {"fp64_sequential": r_seq, "fp64_batched": r_bat, "fp64_streams": r_str,
                                 "mixed_batched": r_mix},
            "max_refine_iterations": {"fp64_sequential": it_seq, "fp64_batched": it_bat, "fp64_streams": it_str,
                                      "mixed_batched": it_mix}}


def median_ms(torch, fn, reps: int = 5) -> float:
    """Median wall time (ms) of `reps` warm calls, each bracketed by device synchronisation."""
    fn()
    torch.cuda.synchronize()
    ts = []
    for _ in range(reps):
        t0 = time.perf_counter()
        fn()
        torch.cuda.synchronize()
        ts.append(1000.0 * (time.perf_counter() - t0))
    return float(np.median(ts))


# Execution settings of the 64^3 workload per form: the stop level, the Schur flush
# split threshold of every factored level and, in the mixed form, each level's flush
# mode, as h2_tune chose them in one measured run (stop level first, then one
# factorization per candidate).  Fixed here so that
# every run, and the profiles under profiles/, use the same launches; --tune measures
# them again at setup instead.
UNLIMITED = 2 ** 63 - 1
CUBE64_SETTINGS = {"fp64": {"stop_level": 7,
                            "split_below": {7: 8192, 8: 2048, 9: 0, 10: UNLIMITED, 11: UNLIMITED, 12: 32768}},
                   "mixed": {"stop_level": 7,
                             "split_below": {7: 32768, 8: 32768, 9: 0, 10: 8192, 11: 8192, 12: 0},
                             "mixed_flush": {7: 0, 8: 1, 9: 0, 10: 0, 11: 0, 12: 1}}}


def apply_settings(G, settings: dict) -> dict:
    G.set_stop_level(settings["stop_level"])
    for lev, v in settings["split_below"].items():
        G.set_schur_split(int(v), int(lev))
    for lev, v in settings.get("mixed_flush", {}).items():
        G.set_mixed_flush(int(v), int(lev))
    for lev, v in settings.get("schur_chunk", {}).items():
        G.set_schur_chunk(int(v), int(lev))
    return dict(settings, source="fixed (h2_tune)")


def form_leg(torch, G, pr, precision: str, steps: int, warmup: int, b, B64, tag: str, setup=None) -> dict:
    """One arithmetic form on the resident H^2 matrix: `warmup` untimed and `steps` timed
    steps (factor + 1 RHS refined to 1e-8), then warm solve and matvec medians and one
    more factorization with every kernel family timed (untimed, for the roofline).
    `setup(G)` (untimed) fixes or tunes the execution settings and returns them."""
    G.set_precision(precision)
    t0 = time.perf_counter()
    settings = setup(G) if setup else None
    setup_s = time.perf_counter() - t0
    if settings is not None:
        print(f"# {tag} {precision} settings {settings} ({setup_s:.1f} s)", file=sys.stderr, flush=True)

    def step():
        G.factor()
        return G.solve(b, tol=1e-8, max_iter=20, info=True)

    for w in range(warmup):
        step()
        print(f"# {tag} {precision} warmup {w} done", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    timings, levels, infos = [], [], []
    for k in range(steps):
        _, info = step()
        infos.append(info)
        timings.append(G.timing(ledger=False))
        levels.append(G.level_timing())
        print(f"# {tag} {precision} step {k} done", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    total = time.perf_counter() - t0
    ledger = G.timing()[6:]
    info = infos[-1]
    solve_ref_ms = median_ms(torch, lambda: G.solve(b, tol=1e-8, max_iter=20))
    solve1_ms = median_ms(torch, lambda: G.solve(b))
    solve64_ms = median_ms(torch, lambda: G.solve(B64))
    matvec_ms = median_ms(torch, lambda: G.matvec(b))
    stats = G.stats()
    G.set_kernel_timing(True)
    G.factor()
    kled = G.kernel_ledger()
    kern = kernel_rooflines(kled, solve1_ms, matvec_ms, mixed=(precision == "mixed"))
    G.set_kernel_timing(False)
    print(f"# {tag} {precision} solves and kernel timing done", file=sys.stderr, flush=True)
    tm = np.median(np.array(timings), axis=0)
    lv = np.median(np.array(levels), axis=0)
    out = {"precision": precision, "steps": steps, "warmup": warmup, "total_s": total,
           "unknowns_per_s": pr.n * steps / total, "ms_per_step": 1000.0 * total / steps,
           "factor_ms": float(tm[0]), "factor_unknowns_per_s": pr.n / (tm[0] * 1e-3),
           "factor_phase_ms": {"steps0_2": tm[1], "lu_panels": tm[2], "schur": tm[3], "merge": tm[4],
                               "final_lu": tm[5]},
           "factor_tflops": ledger[2] / (tm[0] * 1e-3) / 1e12,
           "level_ms": [{"level": int(r[0]), "clusters": int(r[1]), "sum_n": int(r[2]), "max_n": int(r[3]),
                         "sum_kt": int(r[6]), "eliminated": int(r[9]), "ms": float(ms)}
                        for r, ms in zip(stats, lv)],
           "refine_iterations": info["iterations"], "rel_residual": info["rel_residual"],
           "rel_residual_first": info["rel_residual_first"],
           "solve_ms_refined_1e-8": solve_ref_ms, "solve_ms_1rhs": solve1_ms, "solve_ms_64rhs": solve64_ms,
           "matvec_ms_1rhs": matvec_ms, "kernel_roofline": kern,
           "schur_fp32_flop_frac": kled["schur_fp32_flop_frac"],
           "settings": settings, "settings_s": setup_s,
           "_ledger": ledger, "_schur_ms": float(tm[3])}
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--grid", type=int, default=64)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-batch", action="store_true", help="skip the 64-problem batching leg")
    ap.add_argument("--no-cube32", action="store_true", help="skip the 32^3 leg")
    ap.add_argument("--forms", default="fp64,mixed")
    ap.add_argument("--stop-level", type=int, default=0,
                    help="last factored level of the headline workload (0: the fixed settings, or --tune)")
    ap.add_argument("--tune", action="store_true",
                    help="choose the stop level and Schur split thresholds by h2_tune at setup")
    ap.add_argument("--batch-chunk", type=int, default=16)
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain device copy of known size (for scaling HBM counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: the library has no multi-GPU path (use --gpus 1)", file=sys.stderr)
        sys.exit(2)
    import torch
    if args.copy_calibration:
        copy_calibration(torch)
        return

    import paper_1703_06155_amd as h2
    from paper_1703_06155_amd import inputs as I

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    # the batching leg first, on a device no other handle has touched yet
    batch = None
    if not args.no_batch:
        batch = batch_leg(torch, h2, I, args.batch_chunk)
        torch.cuda.empty_cache()
        print("# batch leg done", file=sys.stderr, flush=True)
    g = args.grid
    pr = I.make_problem(f"cube{g}", (g, g, g), 64, 1e-4)
    t0 = time.perf_counter()
    G = h2.H2(pr.points, pr.k, pr.h, pr.chi, pr.leaf, pr.eta, pr.eps)
    torch.cuda.synchronize()
    build_s = time.perf_counter() - t0
    print(f"# build {g}^3 {build_s:.2f} s (setup, untimed)", file=sys.stderr, flush=True)
    # setup, untimed, per form: the stop level (Sec. III-C early stop) and the per-level
    # Schur split thresholds: fixed for 64^3 (chosen by h2_tune), measured otherwise
    if args.stop_level:
        def setup(G, form):
            G.set_stop_level(args.stop_level)
            return {"stop_level": args.stop_level, "source": "--stop-level"}
    elif args.tune or g not in (64,):
        def setup(G, form):
            return dict(G.tune(max_final=16384), source="h2_tune at setup")
    else:
        def setup(G, form):
            return apply_settings(G, CUBE64_SETTINGS[form])
    b = torch.from_numpy(pr.rhs[:, 0].copy()).cuda()
    B64 = torch.from_numpy(I.plane_waves(pr.points, I.directions(64, 3))).cuda()
    forms = [f for f in args.forms.split(",") if f]
    legs = {f: form_leg(torch, G, pr, f, args.steps, args.warmup, b, B64, f"{g}^3", lambda G_, f=f: setup(G_, f))
            for f in forms}
    head = max(legs.values(), key=lambda d: d["unknowns_per_s"])
    hf = head["precision"]
    schur_flops, schur_launches, factor_flops, schur_bytes = head["_ledger"]
    roof = schur_roofline(schur_flops, schur_bytes, head["_schur_ms"], int(schur_launches), g, hf,
                          fixed_settings=(head["settings"] or {}).get("source") == "fixed (h2_tune)")
    for d in legs.values():
        d.pop("_ledger")
        d.pop("_schur_ms")
    G.close()
    del G
    torch.cuda.empty_cache()
    out = {
        "metric": "H² factor unknowns/s + solve ms at rel. residual 1e-8, mixed/batched vs FP64",
        "value": head["unknowns_per_s"],
        "unit": "unknowns/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": head["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "c128" if hf == "fp64" else "c128+c64",
        "data": "synthetic",
        "config": {"workload": f"VIE cube grid {g}^3 (N={pr.n}), leaf 64, eta 1, eps 1e-4, "
                               f"factor + 1 RHS refined to 1e-8; value = the faster form ({hf})",
                   "N": pr.n, "leaf": 64, "eta": 1.0, "eps": 1e-4, "precision": hf, "build_s": build_s,
                   "stop_level": head["settings"]["stop_level"], "settings": head["settings"]},
        "factor_ms": head["factor_ms"],
        "factor_unknowns_per_s": head["factor_unknowns_per_s"],
        "solve_ms_refined_1e-8": head["solve_ms_refined_1e-8"],
        "solve_ms_1rhs": head["solve_ms_1rhs"],
        "solve_ms_64rhs": head["solve_ms_64rhs"],
        "refine_iterations": head["refine_iterations"],
        "rel_residual": head["rel_residual"],
        "forms": legs,
        "roofline": roof,
    }
    if "fp64" in legs and "mixed" in legs:
        out["mixed_vs_fp64"] = {"step": legs["mixed"]["unknowns_per_s"] / legs["fp64"]["unknowns_per_s"],
                                "factor": legs["fp64"]["factor_ms"] / legs["mixed"]["factor_ms"],
                                "solve_refined": legs["fp64"]["solve_ms_refined_1e-8"]
                                / legs["mixed"]["solve_ms_refined_1e-8"]}
    if not args.no_cube32 and g != 32:
        p32 = I.make_problem("cube32", (32, 32, 32), 64, 1e-4)
        G32 = h2.H2(p32.points, p32.k, p32.h, p32.chi, p32.leaf, p32.eta, p32.eps)
        b32 = torch.from_numpy(p32.rhs[:, 0].copy()).cuda()
        B32 = torch.from_numpy(I.plane_waves(p32.points, I.directions(64, 3))).cuda()
        leg32 = form_leg(torch, G32, p32, "fp64", max(args.steps, 3), 1, b32, B32, "32^3",
                         lambda G_: dict(G_.tune(max_final=16384), source="h2_tune at setup"))
        leg32.pop("_ledger")
        leg32.pop("_schur_ms")
        leg32.pop("kernel_roofline")
        leg32["workload"] = "VIE cube grid 32^3 (N=32768), leaf 64, eta 1, eps 1e-4, FP64, factor + 1 RHS refined"
        leg32["stop_level"] = leg32["settings"]["stop_level"]
        out["cube32"] = leg32
        G32.close()
        del G32
        torch.cuda.empty_cache()
    if batch is not None:
        out["batch"] = batch
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
