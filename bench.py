"""Benchmark: H^2 factorization + refined solve on one MI355X.

A step is one pass of the hot path over the resident H^2 matrix of the
headline workload (32^3 cube grid, N = 32768, leaf 64, eta = 1, eps = 1e-4):
the level-by-level factorization followed by one right-hand side solved and
iteratively refined to a relative residual of 1e-8 against the H^2 matrix.
Construction of the H^2 representation is setup (untimed), as in the paper.

Prints one JSON line.  `value` = unknowns per second of whole steps
(N * steps / timed seconds); the factorization rate alone, the solve times
(1 RHS refined, 1 RHS plain, 64 RHS plain), the Schur kernel's roofline and
the CPU oracle's rate on a bounded sample are reported beside it.
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


def cpu_baseline(budget_s: float = 30.0) -> dict:
    """The oracle on a 16^3 sub-cube of the same generator (leaf 64, eps 1e-4)."""
    from threadpoolctl import threadpool_info
    from oracle import h2_oracle as O
    from paper_1703_06155_amd import inputs as I

    pr = I.make_problem("cpu_sample", (16, 16, 16), 64, 1e-4)
    H = O.construct(pr.points, pr.k, pr.h, pr.chi, pr.leaf, pr.eta, pr.eps)
    t0 = time.perf_counter()
    Fz = O.factor(H)
    x, hist = O.refine(Fz, pr.rhs[:, 0], tol=1e-8, max_iter=10)
    dt = time.perf_counter() - t0
    threads = max([i.get("num_threads", 1) for i in threadpool_info()] + [1])
    return {"value": pr.n / dt, "unit": "unknowns/s", "cores": int(threads), "kind": "oracle",
            "sample": f"16^3 sub-cube of the same generator (N={pr.n}, leaf 64, eta 1, eps 1e-4): "
                      f"factor + 1 RHS refined to {hist[-1]:.1e} in {dt:.1f} s; construction excluded"}


# HBM bytes per FP64 Schur flush (flush kernel + partial-tile reduction) on the
# default workload, from rocprofv3 FETCH_SIZE and WRITE_SIZE counters scaled by a
# 1 GiB copy (profiles/k_schur_cube32_fp64.md); valid only for that 32^3 workload
# and the kernel sources hashed here.
SCHUR_TRAFFIC = {"sources_sha256": "8d0ef45760b189416cd8b410a670676237a85e2c082123f289136bebc7a94a34",
                 "bytes_per_launch": 952878868, "grid": 32}


def kernel_sources_sha256() -> str:
    """Hash of the Schur flush kernel's source: the tile engine header, the
    kernel interface header and the kernel's own section of the kernel file."""
    import hashlib
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_1703_06155_amd", "csrc")
    for f in ("h2_device.hpp", "h2_kernels.hpp"):
        with open(os.path.join(csrc, f), "rb") as fh:
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


def schur_roofline(flops: float, nbytes: float, ms: float, launches: int, grid: int) -> dict:
    """Roofline of the Schur flush (the FP64 flush kernel plus the kernel that adds
    the partial tiles of split target blocks) from the algorithmic ledger and the
    flush durations the library measured with HIP events on its stream; one
    "launch" is one flush of a colour's pending updates."""
    per_launch_s = ms * 1e-3 / max(launches, 1)
    ridge = PEAK_FP64_TFLOPS * 1e12 / (PEAK_HBM_GBS * 1e9)  # flop / byte
    intensity = flops / nbytes if nbytes > 0 else float("inf")
    traffic = None
    if (grid == SCHUR_TRAFFIC["grid"] and SCHUR_TRAFFIC["sources_sha256"]
            and SCHUR_TRAFFIC["sources_sha256"] == kernel_sources_sha256()):
        traffic = SCHUR_TRAFFIC["bytes_per_launch"]
    if intensity >= ridge:
        achieved = flops / max(launches, 1) / per_launch_s / 1e12 if ms > 0 else 0.0
        out = {"bound": "mfma", "achieved": achieved, "peak": PEAK_FP64_TFLOPS, "unit": "TFLOP/s"}
    else:
        achieved = nbytes / max(launches, 1) / per_launch_s / 1e9 if ms > 0 else 0.0
        out = {"bound": "hbm", "achieved": achieved, "peak": PEAK_HBM_GBS, "unit": "GB/s"}
    out.update({"frac": out["achieved"] / out["peak"], "traffic": traffic, "kernel": "k_schur_fp64 + k_schur_reduce",
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
    in FP64 versus batched (h2_factor_batch / h2_solve_batch, graph-replayed sweeps) in
    FP64 and in the mixed form, in chunks of `chunk` problems whose handles are released
    after their solve.  Every run reports the largest final residual over the problems."""
    probs = I.batch_problems(count=64, nrhs=16)
    n_total = sum(pr.n for pr in probs)

    def run(batched: bool, precision: str) -> tuple:
        elapsed, worst, iters = 0.0, 0.0, 0
        for c0 in range(0, len(probs), chunk):
            part = probs[c0:c0 + chunk]
            hs = [h2.H2(pr.points, pr.k, pr.h, pr.chi, pr.leaf, pr.eta, pr.eps, precision=precision)
                  for pr in part]
            rhs = [torch.from_numpy(pr.rhs.copy()).cuda() for pr in part]
            for G in hs:
                G.set_sweep_graph(batched)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            if batched:
                h2.factor_batch(hs)
                _, infos = h2.solve_batch(hs, rhs, tol=1e-8, max_iter=20, info=True)
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
        return elapsed, worst, iters

    t_seq, r_seq, it_seq = run(False, "fp64")
    t_bat, r_bat, it_bat = run(True, "fp64")
    t_mix, r_mix, it_mix = run(True, "mixed")
    return {"workload": "64 box problems, sides U{12..32}, leaf 48, eps 1e-4, 16 RHS each, refined to 1e-8",
            "unknowns": n_total, "chunk": chunk, "sequential_s": t_seq, "batched_s": t_bat,
            "sequential_unknowns_per_s": n_total / t_seq, "batched_unknowns_per_s": n_total / t_bat,
            "speedup": t_seq / t_bat,
            "batched_mixed_s": t_mix, "batched_mixed_unknowns_per_s": n_total / t_mix,
            "mixed_batched_vs_fp64_sequential": t_seq / t_mix, "mixed_batched_vs_fp64_batched": t_bat / t_mix,
            "max_rel_residual": {"fp64_sequential": r_seq, "fp64_batched": r_bat, "mixed_batched": r_mix},
            "max_refine_iterations": {"fp64_sequential": it_seq, "fp64_batched": it_bat, "mixed_batched": it_mix}}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--grid", type=int, default=32)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-batch", action="store_true", help="skip the 64-problem batching leg")
    ap.add_argument("--batch-chunk", type=int, default=16)
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain device copy of known size (for scaling HBM counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: this build has no multi-GPU path (use --gpus 1)", file=sys.stderr)
        sys.exit(2)
    import torch
    if args.copy_calibration:
        copy_calibration(torch)
        return

    import paper_1703_06155_amd as h2
    from paper_1703_06155_amd import inputs as I

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    g = args.grid
    pr = I.make_problem(f"cube{g}", (g, g, g), 64, 1e-4)
    t0 = time.perf_counter()
    G = h2.H2(pr.points, pr.k, pr.h, pr.chi, pr.leaf, pr.eta, pr.eps)
    torch.cuda.synchronize()
    build_s = time.perf_counter() - t0
    print(f"# build {build_s:.2f} s (setup, untimed)", file=sys.stderr, flush=True)
    b = torch.from_numpy(pr.rhs[:, 0].copy()).cuda()
    B64 = torch.from_numpy(I.plane_waves(pr.points, I.directions(64, 3))).cuda()

    def step():
        G.factor()
        return G.solve(b, tol=1e-8, max_iter=20, info=True)

    for w in range(args.warmup):
        step()
        print(f"# warmup {w} done", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    infos = []
    fac_ms = []
    timings = []
    for k in range(args.steps):
        x, info = step()
        infos.append(info)
        tm = G.timing(ledger=False)
        timings.append(tm)
        fac_ms.append(tm[0])
    torch.cuda.synchronize()
    total = time.perf_counter() - t0
    ledger = G.timing()[6:]  # algorithmic ledger of the last factorization (same ranks every step)
    ms_per_step = 1000.0 * total / args.steps
    # solve-only timings (factor resident)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    x, info = G.solve(b, tol=1e-8, max_iter=20, info=True)
    torch.cuda.synchronize()
    solve_ref_ms = 1000.0 * (time.perf_counter() - t1)
    t1 = time.perf_counter()
    G.solve(b)
    torch.cuda.synchronize()
    solve1_ms = 1000.0 * (time.perf_counter() - t1)
    t1 = time.perf_counter()
    G.solve(B64)
    torch.cuda.synchronize()
    solve64_ms = 1000.0 * (time.perf_counter() - t1)
    stats = G.stats()
    # per-kernel roofline: one more FP64 factorization (untimed) with events around every kernel family
    for _ in range(2):
        G.matvec(b)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    G.matvec(b)
    torch.cuda.synchronize()
    matvec_ms = 1000.0 * (time.perf_counter() - t1)
    G.set_kernel_timing(True)
    G.factor()
    kern = kernel_rooflines(G.kernel_ledger(), solve1_ms, matvec_ms)
    G.set_kernel_timing(False)
    # mixed form: complex FP32 Schur updates and projections, FP64 refinement to the same residual
    G.set_precision("mixed")
    step()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    mixed_fac = []
    for k in range(args.steps):
        xm, info_m = step()
        mixed_fac.append(G.timing(ledger=False))
    torch.cuda.synchronize()
    mixed_total = time.perf_counter() - t1
    tm_mixed = np.mean(np.array(mixed_fac), axis=0)
    G.set_kernel_timing(True)
    G.factor()
    kern_mixed = kernel_rooflines(G.kernel_ledger(), mixed=True)
    G.set_kernel_timing(False)
    tm = np.mean(np.array(timings), axis=0)
    schur_flops, schur_launches, factor_flops, schur_bytes = ledger
    schur_ms = tm[3]
    roof = schur_roofline(schur_flops, schur_bytes, schur_ms, int(schur_launches), g)
    out = {
        "metric": "H² factor unknowns/s + solve ms at rel. residual 1e-8, mixed/batched vs FP64",
        "value": pr.n * args.steps / total,
        "unit": "unknowns/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "c128",
        "data": "synthetic",
        "config": {"workload": f"VIE cube grid {g}^3 (N={pr.n}), leaf 64, eta 1, eps 1e-4, FP64 form, "
                               f"factor + 1 RHS refined to 1e-8", "N": pr.n, "leaf": 64, "eta": 1.0,
                   "eps": 1e-4, "precision": "fp64"},
        "factor_ms": float(np.mean(fac_ms)),
        "factor_unknowns_per_s": pr.n / (np.mean(fac_ms) * 1e-3),
        "solve_ms_refined_1e-8": solve_ref_ms,
        "refine_iterations": info["iterations"],
        "rel_residual": info["rel_residual"],
        "rel_residual_first": info["rel_residual_first"],
        "mixed": {"unknowns_per_s": pr.n * args.steps / mixed_total, "ms_per_step": 1000.0 * mixed_total / args.steps,
                  "factor_ms": float(tm_mixed[0]), "refine_iterations": info_m["iterations"],
                  "rel_residual": info_m["rel_residual"], "rel_residual_first": info_m["rel_residual_first"],
                  "factor_phase_ms": {"steps0_2": tm_mixed[1], "lu_panels": tm_mixed[2], "schur": tm_mixed[3],
                                      "merge": tm_mixed[4], "final_lu": tm_mixed[5]},
                  "kernel_roofline": kern_mixed},
        "solve_ms_1rhs": solve1_ms,
        "solve_ms_64rhs": solve64_ms,
        "factor_phase_ms": {"steps0_2": tm[1], "lu_panels": tm[2], "schur": tm[3], "merge": tm[4],
                            "final_lu": tm[5]},
        "factor_tflops": factor_flops / (tm[0] * 1e-3) / 1e12,
        "levels": stats.tolist(),
        "roofline": roof,
        "kernel_roofline": kern,
    }
    if not args.no_batch:
        G.close()
        out["batch"] = batch_leg(torch, h2, I, args.batch_chunk)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
