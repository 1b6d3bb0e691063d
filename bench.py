"""Benchmark: pair energy+gradient evaluations per second inside the on-device
L-BFGS minimizer on the 50,000-atom compacted chain (FP32 pair terms, FP64
accumulation), plus the roofline of the pair kernel and the CPU oracle's rate.

One step = one L-BFGS iteration (m = 10) of the whole path: direction from
the stored pairs, LS_PAR with its trial points, each trial an energy+gradient
evaluation (bonded terms, all-pairs kernel, finalize), and the accept pass.
The system, its parameters and the start point are resident in HBM before the
timed region; W warm-up iterations run first, then exactly K timed ones.

Prints one JSON line.  `python bench.py` runs the default single-GPU case.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

FLOPS_PER_PAIR = 38            # algorithmic flops of one pair (energy + gradient)
# Published MI355X vector peaks (TFLOP/s): FP32 157.3 (two FP32 operations per
# lane and cycle, i.e. packed FP32) and FP64 78.6.  This build issues no packed
# FP32, so its FP32 ceiling is the scalar issue rate, 256 CU x 4 SIMD x 16
# lanes x 2 flop (FMA) x 2.4 GHz = 78.6 TFLOP/s, reported beside the peak.
PEAK_FP32_TFLOPS = 157.3
PEAK_FP64_TFLOPS = 78.6
SCALAR_ISSUE_TFLOPS = 256 * 4 * 16 * 2 * 2.4e9 / 1e12


# the pair kernel and the host code that lays out its chunk tables (both decide its traffic)
PAIR_SOURCES = ["paper_1810_03358_amd/csrc/ff_pair.hip", "paper_1810_03358_amd/csrc/ff_internal.h",
                "paper_1810_03358_amd/csrc/ff_api.hip"]


def measured_traffic(workload: str, precision: str):
    """HBM bytes per pair-kernel launch from the committed FETCH_SIZE /
    WRITE_SIZE summary (copy-kernel calibrated), or None when there is no
    summary for this workload or the kernel sources changed since it was
    taken."""
    import hashlib
    if precision != "fp32":
        return None
    path = os.path.join(ROOT, "profiles", f"k_pair32_{workload}_hbm_traffic.txt")
    if not os.path.exists(path):
        return None
    fields = {}
    for line in open(path):
        if ":" in line:
            k, v = line.split(":", 1)
            fields[k.strip()] = v.strip()
    h = hashlib.sha256()
    for f in PAIR_SOURCES:
        h.update(open(os.path.join(ROOT, f), "rb").read())
    if fields.get("source_sha256 (ff_pair.hip + ff_internal.h + ff_api.hip at measurement)") != h.hexdigest():
        return None
    return float(fields["traffic_bytes_per_launch"])


def non_excluded_pairs(n: int) -> int:
    # chain topology: 1-2 and 1-3 pairs excluded
    return n * (n - 1) // 2 - max(0, n - 1) - max(0, n - 2)


def cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(system, x0, seconds: float = 15.0):
    """The FP64 CPU oracle, timed on a bounded sample of the same workload:
    full energy+gradient evaluations at the start point on all the oracle's
    threads, repeated until about `seconds` of CPU time (at least one); then
    one thread on a sample of gradient rows (each row is the same O(N) loop a
    full evaluation runs N times), scaled to a full evaluation."""
    import numpy as np
    import oracle
    sysc = oracle.System(system)
    n = 0
    t0 = time.perf_counter()
    while True:
        oracle.energy_grad(sysc, x0)
        n += 1
        dt = time.perf_counter() - t0
        if dt >= seconds or n >= 50:
            break
    threads = oracle.num_threads()
    natoms = system["n_atoms"]
    oracle.set_num_threads(1)
    rows, dt1 = 64, 0.0
    try:
        while True:
            atoms = np.linspace(0, natoms - 1, min(rows, natoms)).astype(np.int32)
            t1 = time.perf_counter()
            oracle.atom_gradients(sysc, x0, atoms)
            dt1 = time.perf_counter() - t1
            if dt1 >= seconds / 5 or len(atoms) == natoms:
                break
            rows *= 4
    finally:
        oracle.set_num_threads(threads)
    one_core = len(atoms) / (dt1 * natoms)
    return {"value": n / dt, "unit": "evals/s", "cores": threads, "kind": "oracle",
            "sample": f"{n} full FP64 energy+gradient evaluation(s) of the {natoms}-atom start point "
                      f"({dt:.1f} s)",
            "cpu_model": cpu_model(), "host_cpus": os.cpu_count(),
            "one_core": {"value": one_core, "unit": "evals/s", "cores": 1,
                         "sample": f"{len(atoms)} of {natoms} gradient rows on one thread ({dt1:.1f} s), "
                                   f"scaled to a full evaluation"}}


def batch_bench(args):
    """The many-systems workload: 256 independent chains with sizes log-uniform
    in [200, 4000] atoms (seeds 100..355), minimized together by L-BFGS (m = 10)
    in one ff_minimize call to |grad E|_inf < 1e-3 or --batch-iters iterations
    (default 60,000).  Reports the wall time per system from the start points
    resident in HBM to the certified results.

    The tiling is the library's default for batches (128-atom I-blocks with
    two atoms per lane, chunks of 4 j-tiles in both kernels), which ran
    faster per evaluation than what the autotuner picks from timings at the
    start points; --batch-autotune
    tunes the FP64 kernel's configuration and chunk length (runs to 1e-3
    spend about nine in ten evaluations in FP64) and, in FP32 mode, the FP32
    kernel's chunk length for the same configuration."""
    import numpy as np
    import torch
    import paper_1810_03358_amd as ff
    from synth import batch_sizes, chain_system

    dev = torch.device("cuda:0")
    sizes = batch_sizes()
    systems = [chain_system(n, 100 + b) for b, n in enumerate(sizes)]
    x0 = torch.tensor(np.concatenate([s["x"] for s in systems]), dtype=torch.float64, device=dev).contiguous()
    stream = torch.cuda.Stream(device=dev)
    with torch.cuda.stream(stream):
        tiling, tune_ms = None, None
        if args.batch_autotune:
            (cfg, chunk64), tune_ms = ff.autotune(systems, x0, "fp64", reps=3, stream=stream)
            chunk = chunk64
            if args.precision == "fp32":
                (cfg32, chunk32), _ = ff.autotune(systems, x0, "fp32", reps=3, stream=stream)
                if cfg32 == cfg:
                    chunk = chunk32
            tiling = (cfg, chunk, chunk64)
        ctx = ff.Context(systems, m_max=10, device=dev, stream=stream, tiling=tiling)
        tiling = ctx.tiling
        x = x0.clone()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        res = ctx.minimize(x, "lbfgs", m=10, tol=1e-3, max_iter=args.batch_iters, precision=args.precision,
                           stream=stream)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
    evals = sum(r["evals"] for r in res)
    iters = np.array([r["iters"] for r in res])
    conv = sum(r["term"] == ff.FF_CONVERGED for r in res)
    pairs = sum(non_excluded_pairs(n) for n in sizes)
    out = {
        "metric": "time to |grad E|_inf<1e-3 per system (batch)",
        "value": wall / len(systems),
        "unit": "s/system",
        "n_gpus": 1,
        "higher_is_better": False,
        "dtype": "f32" if args.precision == "fp32" else "f64",
        "data": "synthetic",
        "config": {"workload": "batch256", "systems": len(systems), "atoms": int(sum(sizes)),
                   "sizes": "log-uniform [200, 4000], seeds 100-355", "pairs_per_eval_all_systems": pairs,
                   "method": f"L-BFGS m=10, LS_PAR, tol 1e-3, max_iter {args.batch_iters}",
                   "tiling": list(tiling)},
        "wall_s": wall,
        "converged": int(conv),
        "iters_median": float(np.median(iters)), "iters_max": int(iters.max()),
        "evals_total": int(evals), "evals_fp64_total": int(sum(r["evals_fp64"] for r in res)),
        "system_evals_per_s": evals / wall,
        "tiling_source": "autotuned" if args.batch_autotune else "library default",
        "autotune_ms_per_fp64_batch_eval": tune_ms,
    }
    print(json.dumps(out), flush=True)
    ctx.close()


def oracle_solve(system, method: str, max_iter: int, threads: int | None = None):
    """The FP64 oracle minimizing the same system with the same method and
    stopping rule, timed on the host (all the oracle's threads, or `threads`)."""
    import oracle
    sysc = oracle.System(system)
    code = {"gd": oracle.GD, "fgm": oracle.FGM, "cg": oracle.CG, "lbfgs": oracle.LBFGS}[method]
    p = oracle.MinParams(method=code, m=10, tol=1e-3, max_iter=max_iter)
    keep = oracle.num_threads()
    if threads:
        oracle.set_num_threads(threads)
    state = {"evals": 0, "last": time.perf_counter()}

    def fg(v):
        state["evals"] += 1
        now = time.perf_counter()
        if now - state["last"] >= 10.0:
            state["last"] = now
            print(f"oracle {method}: {state['evals']} evaluations, {now - t0:.0f} s", file=sys.stderr, flush=True)
        return oracle.energy_grad(sysc, v.reshape(-1, 3))

    try:
        t0 = time.perf_counter()
        r = oracle.minimize(fg, system["x"].ravel(), p)
        wall = time.perf_counter() - t0
        used = oracle.num_threads()
    finally:
        oracle.set_num_threads(keep)
    term = {oracle.CONVERGED: "converged", oracle.MAX_ITER: "max_iter", oracle.LS_FAILED: "ls_failed",
            oracle.NONFINITE_START: "nonfinite_start"}.get(r.term, str(r.term))
    return {"time_s": wall, "cores": used, "term": term, "iters": r.iters, "evals": r.evals, "energy": r.f,
            "grad_inf": float(abs(r.g).max()), "x": r.x}


def solve_bench(args):
    """One named chain minimized from its start to |grad E|_inf < 1e-3 (or
    --solve-iters iterations) in one ff_minimize call by --method (m = 10;
    LS_PAR, FGM: LS_H), start point resident in HBM; reports the wall time and
    the end point, certified by an FP64 evaluation after the timed region.
    --oracle also runs the FP64 oracle on the host with the same method and
    stopping rule (all threads, and one thread with --oracle-one-core) and
    compares the two end points."""
    import numpy as np
    import torch
    import paper_1810_03358_amd as ff
    from synth import config_system

    dev = torch.device("cuda:0")
    s = config_system(args.workload)
    stream = torch.cuda.Stream(device=dev)
    with torch.cuda.stream(stream):
        ctx = ff.Context(s, m_max=10, device=dev, stream=stream)
        x = torch.tensor(s["x"], dtype=torch.float64, device=dev).contiguous()
        torch.cuda.synchronize()
        # one minimization, run as resumed calls of 5000 iterations so that
        # progress is printed (a resumed call continues the same iterate
        # exactly); the end point is evaluated in FP64 after the timed region
        t0 = time.perf_counter()
        iters = evals = evals64 = 0
        while True:
            r = ctx.minimize(x, args.method, m=10, tol=1e-3, max_iter=min(5000, args.solve_iters - iters),
                             precision=args.precision, resume=iters > 0, certify=False, stream=stream)
            iters += r["iters"]
            evals, evals64 = r["evals"], r["evals_fp64"]
            print(f"solve: {iters} iterations, {r['term_name']}, E {r['energy']:.9e}, |g|_inf {r['grad_inf']:.3e}, "
                  f"{evals} evaluations ({evals64} FP64), {time.perf_counter() - t0:.1f} s", file=sys.stderr,
                  flush=True)
            if r["term"] != ff.FF_MAX_ITER or iters >= args.solve_iters:
                break
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        e, g = ctx.energy_grad(x, "fp64", stream=stream)
        torch.cuda.synchronize()
        r = dict(r, iters=iters, evals=evals, evals_fp64=evals64, energy=float(e.cpu()[0]),
                 grad_inf=float(g.abs().max().cpu()))
        x_gpu = x.cpu().numpy()
    ls = "LS_H" if args.method == "fgm" else "LS_PAR"
    out = {
        "metric": "time to |grad E|_inf<1e-3 (one system)", "value": wall, "unit": "s", "n_gpus": 1,
        "higher_is_better": False, "vs_baseline": None, "dtype": "f32" if args.precision == "fp32" else "f64",
        "data": "synthetic",
        "config": {"workload": args.workload, "atoms": s["n_atoms"], "seed": s["seed"],
                   "method": f"{args.method} m=10, {ls}, tol 1e-3, max_iter {args.solve_iters}"},
        "term": r["term_name"], "iters": r["iters"], "evals": r["evals"], "evals_fp64": r["evals_fp64"],
        "energy": r["energy"], "grad_inf": r["grad_inf"], "evals_per_s": r["evals"] / wall,
    }
    if args.oracle:
        runs = [oracle_solve(s, args.method, args.solve_iters)]
        if args.oracle_one_core:
            runs.append(oracle_solve(s, args.method, args.solve_iters, threads=1))
        o = runs[0]
        rmsd = float(np.sqrt(((x_gpu - o["x"].reshape(-1, 3)) ** 2).sum(1).mean()))
        out["cpu_baseline"] = {"value": o["time_s"], "unit": "s", "cores": o["cores"], "kind": "oracle",
                               "sample": "the whole solve: same system, method and stopping rule, FP64",
                               "cpu_model": cpu_model(), "host_cpus": os.cpu_count()}
        if len(runs) > 1:
            out["cpu_baseline"]["one_core"] = {"value": runs[1]["time_s"], "unit": "s", "cores": 1}
        out["oracle"] = {k: v for k, v in o.items() if k != "x"}
        out["vs_oracle"] = {"energy_rel_diff": abs(r["energy"] - o["energy"]) / abs(o["energy"]),
                            "rmsd_per_atom_A": rmsd, "same_term": r["term_name"] == o["term"],
                            "time_ratio_oracle_over_gpu": o["time_s"] / wall}
    print(json.dumps(out), flush=True)
    ctx.close()


def learned_bench(args):
    """The learned warm start against plain L-BFGS: held-out 10,000-atom
    chains (seed 300000 + k; compacted start for even k, extended for odd k),
    each minimized alone to |grad E|_inf < 1e-3 (FP32 pair sums) from its
    stored start (plain) and from the learned start (features, network, a
    race of the start and two displaced candidates over 200-1000 iterations,
    then L-BFGS from the winner), and, as controls, with the race's restart
    but no network and with the network's displacements in random
    directions.  Per-system times include everything after the start point
    is resident in HBM; the network was trained beforehand by
    paper_1810_03358_amd.train_warmstart on other chains."""
    import numpy as np
    import torch
    import paper_1810_03358_amd as ff
    from paper_1810_03358_amd import learn as L
    from paper_1810_03358_amd.train_warmstart import DEFAULT_WEIGHTS
    from synth import chain_system

    dev = torch.device("cuda:0")
    path = args.weights or DEFAULT_WEIGHTS
    net = L.Net.load(path, device=dev)
    ks = range(args.test_offset, args.test_offset + args.test_chains)
    systems = [chain_system(args.test_atoms, 300_000 + k, compact=k % 2 == 0) for k in ks]
    rows = L.evaluate(net, systems, lambda s: ff.Context(s, device=dev), max_iter=args.learned_iters,
                      probe_iters=args.probe_iters, control=not args.no_control,
                      random_control=args.random_control, device=dev,
                      log=lambda m: print(m, file=sys.stderr, flush=True))
    pt = np.array([r["plain_time"] for r in rows])
    lt = np.array([r["learned_time"] for r in rows])
    both = np.array([r["plain_term"] == "converged" and r["learned_term"] == "converged" for r in rows])
    pe = np.array([r["plain_energy"] for r in rows])
    le = np.array([r["learned_energy"] for r in rows])
    out = {
        "metric": "time to |grad E|_inf<1e-3 per system, plain vs learned",
        "value": float(lt.mean()),
        "unit": "s/system",
        "n_gpus": 1,
        "higher_is_better": False,
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"learned{args.test_chains}x{args.test_atoms}",
                   "test_chains": args.test_chains, "first_chain": args.test_offset, "atoms": args.test_atoms,
                   "starts": "even k compacted, odd k extended, seeds 300000+k",
                   "method": f"L-BFGS m=10, LS_PAR, FP32 pair sums, tol 1e-3, max_iter {args.learned_iters}",
                   "warm_start": "16-NN + centroid features, 3-layer BF16 MLP, race of x0, x0+0.5d, x0+d "
                                 "over " + (f"{args.probe_iters}" if args.probe_iters else "min(1000, max(200, n/10))")
                                 + " iterations", "weights": os.path.relpath(path, ROOT)},
        "plain_s_per_system": float(pt.mean()),
        "learned_over_plain": float(lt.sum() / pt.sum()),
        "median_time_ratio": float(np.median(lt / pt)),
        "converged_plain": int(sum(r["plain_term"] == "converged" for r in rows)),
        "converged_learned": int(sum(r["learned_term"] == "converged" for r in rows)),
        "both_converged_time_ratio": float(lt[both].sum() / pt[both].sum()) if both.any() else None,
        "learned_energy_lower": int(np.sum(le < pe)),
        "energy_equal_1e-4": int(np.sum(np.abs(le - pe) <= 1e-4 * np.abs(pe))),
        "mean_rel_energy_change": float(np.mean((le - pe) / np.abs(pe))),
        "race_winner_counts": {str(k): int(sum(r["scale_taken"] == k for r in rows)) for k in (0.0, 0.5, 1.0)},
    }
    if args.random_control:
        rt = np.array([r["random_time"] for r in rows])
        out["random_direction_control_s_per_system"] = float(rt.mean())
        out["learned_over_random_control"] = float(lt.sum() / rt.sum())
    if not args.no_control:
        ct = np.array([r["control_time"] for r in rows])
        out["restart_control_s_per_system"] = float(ct.mean())
        out["learned_over_restart_control"] = float(lt.sum() / ct.sum())
    out["systems"] = [{k: (round(v, 6) if isinstance(v, float) else
                           [float(f"{e:.6e}") for e in v] if k == "probe_energies" else v) for k, v in r.items()}
                      for r in rows]
    print(json.dumps(out), flush=True)


def spread_bench(args):
    """How far apart correct runs end: 32 chains of 2,000 atoms (the learned
    test recipe: seed 300000 + k, compacted start for even k, extended for
    odd k), minimized together by L-BFGS (m = 10) to |grad E|_inf < 1e-3 in
    FP64 and in FP32 mode, five times each: under four tilings (four
    summation orders of the same sums) and from the start moved by 1e-12 A
    (seeded normal).  Reports, per pair of runs, the relative difference of
    the final energies and the ratio of the iteration counts: the scale of a
    rounding-level change of the path, against which a criterion such as
    "equal final energy within 1e-4" can be judged."""
    import numpy as np
    import torch
    import paper_1810_03358_amd as ff
    from synth import chain_system

    k_sys = 32
    systems = [chain_system(2000, 300_000 + k, compact=k % 2 == 0) for k in range(k_sys)]
    x0 = np.concatenate([s["x"] for s in systems])
    moved = x0 + 1e-12 * np.random.default_rng(5).standard_normal(x0.shape)
    variants = [((0, 4), x0, "tiling (0, 4)"), ((0, 1), x0, "tiling (0, 1)"), ((1, 1), x0, "tiling (1, 1)"),
                ((5, 1), x0, "tiling (5, 1)"), ((0, 4), moved, "tiling (0, 4), start moved 1e-12 A")]
    out = {"metric": "spread of final energies under rounding-level path changes", "unit": "relative",
           "n_gpus": 1, "data": "synthetic",
           "config": {"workload": "spread32x2000", "systems": k_sys, "atoms": 2000,
                      "starts": "even k compacted, odd k extended, seeds 300000+k",
                      "method": f"L-BFGS m=10, LS_PAR, tol 1e-3, max_iter {args.learned_iters}"},
           "modes": {}}
    for mode in ("fp64", "fp32"):
        E, iters, conv = [], [], []
        for tiling, start, label in variants:
            ctx = ff.Context(systems, m_max=10, device=torch.device("cuda:0"), tiling=tiling)
            x = torch.tensor(start, dtype=torch.float64, device="cuda:0").contiguous()
            res = ctx.minimize(x, "lbfgs", m=10, tol=1e-3, max_iter=args.learned_iters, precision=mode)
            ctx.close()
            E.append([r["energy"] for r in res])
            iters.append([r["iters"] for r in res])
            conv.append(sum(r["term"] == ff.FF_CONVERGED for r in res))
            print(f"{mode} {label}: {conv[-1]} of {k_sys} converged, median {np.median(iters[-1]):.0f} iterations",
                  file=sys.stderr, flush=True)
        E, iters = np.array(E), np.array(iters, dtype=float)
        pairs = []
        for a in range(len(variants)):
            for b in range(a + 1, len(variants)):
                d = np.abs(E[b] - E[a]) / np.abs(E[a])
                pairs.extend(d.tolist())
        pairs = np.array(pairs)
        spread = (E.max(0) - E.min(0)) / np.abs(np.median(E, 0))
        ratio = iters.max(0) / iters.min(0)
        out["modes"][mode] = {
            "runs": [v[2] for v in variants], "converged_per_run": conv,
            "median_iters_per_run": np.median(iters, 1).tolist(),
            "pairwise_rel_energy_difference_median": float(np.median(pairs)),
            "pairwise_within_1e-4": f"{int((pairs < 1e-4).sum())} of {len(pairs)}",
            "per_system_rel_spread_median": float(np.median(spread)),
            "per_system_rel_spread_min": float(spread.min()),
            "per_system_max_over_min_iterations_median": float(np.median(ratio)),
            "per_system_max_over_min_iterations_max": float(ratio.max())}
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--workload", default="chain50k",
                    choices=["chain512", "chain10k", "chain50k", "batch256", "learned", "spread"])
    ap.add_argument("--precision", default="fp32", choices=["fp32", "fp64"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--batch-iters", type=int, default=60_000, help="batch256: iteration limit per system")
    ap.add_argument("--batch-autotune", action="store_true",
                    help="batch256: autotune the tiling instead of the library default")
    ap.add_argument("--solve", action="store_true",
                    help="chain512/10k/50k: minimize to |grad E|_inf < 1e-3 and report the time instead")
    ap.add_argument("--solve-iters", type=int, default=100_000, help="--solve: iteration limit")
    ap.add_argument("--method", default="lbfgs", choices=["lbfgs", "gd", "fgm", "cg"], help="--solve: method")
    ap.add_argument("--oracle", action="store_true", help="--solve: also run the FP64 oracle on the host")
    ap.add_argument("--oracle-one-core", action="store_true", help="--solve --oracle: and on one thread")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--test-chains", type=int, default=8, help="learned: held-out chains")
    ap.add_argument("--test-offset", type=int, default=0, help="learned: index of the first held-out chain")
    ap.add_argument("--test-atoms", type=int, default=10_000, help="learned: atoms per held-out chain")
    ap.add_argument("--learned-iters", type=int, default=60_000, help="learned, spread: iteration limit per run")
    ap.add_argument("--weights", default=None, help="learned: network file (default: the shipped one)")
    ap.add_argument("--no-control", action="store_true", help="learned: skip the restart-only control")
    ap.add_argument("--probe-iters", type=int, default=None,
                    help="learned: length of the race (default: by system size, 200 to 1000)")
    ap.add_argument("--random-control", action="store_true",
                    help="learned: add the race with the displacements in random directions")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="run a plain 256 MiB device copy first (reference for HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU: every system here is minimized on a single device "
              "(the path shards by independent systems across GPUs); run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    if args.workload == "batch256":
        batch_bench(args)
        return
    if args.workload == "learned":
        learned_bench(args)
        return
    if args.workload == "spread":
        spread_bench(args)
        return
    if args.solve:
        solve_bench(args)
        return

    import torch
    import paper_1810_03358_amd as ff
    from synth import config_system

    dev = torch.device("cuda:0")
    s = config_system(args.workload)
    n = s["n_atoms"]
    pairs = non_excluded_pairs(n)
    stream = torch.cuda.Stream(device=dev)      # default priority
    if args.copy_calibration:
        # a kernel of known traffic: reads and writes exactly 256 MiB
        src = torch.ones(64 << 20, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    with torch.cuda.stream(stream):
        ctx = ff.Context(s, m_max=10, device=dev, stream=stream)
        x = torch.tensor(s["x"], dtype=torch.float64, device=dev).contiguous()
        x_start = x.clone()
        torch.cuda.synchronize()

        # warm-up: W iterations from the start point
        rw = ctx.minimize(x, "lbfgs", m=10, max_iter=args.warmup, precision=args.precision,
                          certify=False, stream=stream)
        torch.cuda.synchronize()
        # timed: exactly K more iterations, continuing the same minimization
        t0 = time.perf_counter()
        rt = ctx.minimize(x, "lbfgs", m=10, max_iter=args.steps, precision=args.precision,
                          certify=False, resume=True, stream=stream)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        evals = rt["evals"] - rw["evals"]
        iters = rt["iters"]
        wall = t1 - t0

        # pair kernel alone at the current point (HIP events on this stream)
        reps = 20 if n >= 10_000 else 200
        ms_pair = ctx.time_pair(x, args.precision, reps=reps, stream=stream)
        # back-to-back ff_energy_grad throughput at the start point
        e, g = ctx.energy_grad(x_start, args.precision, stream=stream)
        torch.cuda.synchronize()
        ev0 = time.perf_counter()
        nrep = 20 if n >= 10_000 else 500
        for _ in range(nrep):
            ctx.energy_grad(x_start, args.precision, out_e=e, out_g=g, stream=stream)
        torch.cuda.synchronize()
        direct_rate = nrep / (time.perf_counter() - ev0)

    achieved = FLOPS_PER_PAIR * pairs / (ms_pair * 1e-3) / 1e12
    out = {
        "metric": "pair energy+grad evals/s",
        "value": evals / wall,
        "unit": "evals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": wall * 1e3 / max(iters, 1),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if args.precision == "fp32" else "f64",
        "data": "synthetic",
        "config": {
            "workload": args.workload, "atoms": n, "seed": s["seed"], "pairs": pairs,
            "step": "one L-BFGS iteration (m=10, LS_PAR) on device",
            "precision": "fp32 pair terms, fp64 accumulation and optimizer" if args.precision == "fp32"
            else "fp64", "parallelism": "single GPU",
        },
        "iters_timed": iters,
        "evals_timed": evals,
        "term": rt["term_name"],
        "energy_after": rt["energy"],
        "direct_energy_grad_evals_per_s": direct_rate,
        "roofline": {
            "kernel": "k_pair32" if args.precision == "fp32" else "k_pair64",
            "bound": "alu",
            "achieved": achieved,
            "peak": PEAK_FP32_TFLOPS if args.precision == "fp32" else PEAK_FP64_TFLOPS,
            "unit": "TFLOP/s",
            "frac": achieved / (PEAK_FP32_TFLOPS if args.precision == "fp32" else PEAK_FP64_TFLOPS),
            "traffic": measured_traffic(args.workload, args.precision),
            "traffic_unit": "bytes per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, copy-calibrated)",
            "kernel_ms": ms_pair,
            "flops_per_pair": FLOPS_PER_PAIR,
        },
    }
    if args.precision == "fp32":
        out["roofline"]["scalar_issue_peak"] = SCALAR_ISSUE_TFLOPS
        out["roofline"]["frac_of_scalar_issue_peak"] = achieved / SCALAR_ISSUE_TFLOPS
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(s, s["x"], args.cpu_seconds)
    print(json.dumps(out), flush=True)
    ctx.close()


if __name__ == "__main__":
    main()
