"""Benchmark of the OFM hot path on one MI355X.

One step = the whole path over one synthetic system with the potential
already resident in HBM: fragment setup (boxes, pair list, V per box),
batched fragment eigensolve + whole-system H|phi>, grouped pair matrix
elements, and the thresholded generalised eigenproblem.

Prints ONE JSON line.  `value` is fragment eigenstates delivered per second
by the whole job (sum_j s_j x steps / time of the timed steps).  By default
two steps are in flight (two contexts on two HIP streams, one host thread
each; every step runs the whole path and must return the serial step's
eigenvalues), so the global solve's latency-bound launches overlap the other
step's bandwidth-bound fragment stage; `serial_ms_per_step` is the same
workload one step at a time (--inflight 1 makes it the value).  The
per-stage rates (fragment eigenstates/s of the eigensolver stage, H,S
elements/s of the element stage), the roofline of the dominant kernel (the
fragment-Hamiltonian stencil of the Chebyshev filter) come from the serial
profiled steps; the CPU oracle's rate on a bounded sample rides along.

  python bench.py [--gpus 1] [--steps K] [--warmup W] [--config alkane]
                  [--precision fp64|mixed] [--inflight 2|1] [--no-cpu-baseline]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import threading
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0        # MI355X HBM3E, GB/s
FP64_PEAK_TFS = 78.6         # MI355X FP64 (vector and matrix), TFLOP/s
# LDS: 128 B per clock per CU, 256 CUs, 2.4 GHz
LDS_PEAK_GBS = 128 * 256 * 2.4
LDS_BYTES_PER_POINT_STEP = 11 * 4   # on-chip filter, FP32
STENCIL_KERNELS = {
    "stencil": "k_apply_h (one Chebyshev filter step of H_j per launch)",
    "multistep": "k_apply_hm (two or three Chebyshev filter steps of H_j "
                 "per launch)",
    "sweep": "filter sweep replayed as one graph: k_apply_hm on the boxes "
             "whose plane fits it, k_apply_h on the others",
}


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=4)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--config", default="alkane")
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--precision", default="fp64", choices=["fp64", "mixed"])
    ap.add_argument("--window", type=float, default=0.3,
                    help="energy window above the lowest OFM eigenvalue (Ha)")
    ap.add_argument("--tol", type=float, default=0.0,
                    help="eigensolver residual bound (0: the form's default)")
    ap.add_argument("--degree", type=int, default=0,
                    help="Chebyshev filter degree, FP64 runs (0: default)")
    ap.add_argument("--degree-mixed", type=int, default=0,
                    help="Chebyshev filter degree, mixed runs (0: default)")
    ap.add_argument("--no-mixed", action="store_true",
                    help="skip the mixed-form comparison runs")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--inflight", type=int, default=2, choices=[1, 2],
                    help="steps in flight during the timed throughput run "
                         "(2: two contexts on two streams; 1: serial)")
    ap.add_argument("--cpu-sample", type=int, default=64,
                    help="fragments in the oracle's timed sample")
    ap.add_argument("--calibrate-copy-gib", type=float, default=0.0,
                    help="run a device copy of this size first (counter "
                         "calibration for rocprofv3 --pmc runs)")
    return ap.parse_args()


def measured_traffic(stem):
    """HBM traffic per launch from the committed rocprofv3 counter summary
    profiles/<stem>.md, if the stencil sources have not changed since the
    counters were taken (else None)."""
    path = os.path.join(ROOT, "profiles", f"{stem}.md")
    try:
        line = [l for l in open(path) if l.startswith("traffic: ")][-1]
        rec = json.loads(line[len("traffic: "):])
        sha = stencil_source_sha1()
    except (OSError, IndexError, ValueError):
        return None
    return rec["bytes_per_launch"] if rec.get("stencil_src_sha1") == sha else None


def stencil_source_sha1():
    """SHA-1 over the stencil kernel's sources (stencil.hip, kdev.h)."""
    import hashlib
    h = hashlib.sha1()
    for name in ("stencil.hip", "kdev.h"):
        with open(os.path.join(ROOT, "paper_1011_4764_amd", "csrc", name),
                  "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def cpu_baseline(system, n_sample, seed):
    """The CPU oracle, as it stands, on a seeded sample of fragments of the
    same workload: their eigenpairs, whole-system H|phi> and the pair blocks
    among them.  Rate in fragment eigenstates/s."""
    import numpy as np

    import oracle as O
    rng = np.random.default_rng(seed + 1234)
    nf = system.n_frag
    pick = sorted(rng.choice(nf, size=min(n_sample, nf), replace=False).tolist())
    V = system.potential()
    t0 = time.perf_counter()
    r = O.run(V, system.grid.h, system.frag_lo, system.frag_dims,
              system.frag_states, fragments=pick, solve=False)
    t = time.perf_counter() - t0
    n_states = int(sum(int(system.frag_states[j]) for j in pick))
    try:
        import threadpoolctl
        info = threadpoolctl.threadpool_info()
        cores = max([i.get("num_threads", 1) for i in info] + [1])
    except Exception:
        cores = os.cpu_count() or 1
    return {"value": n_states / t, "unit": "fragment eigenstates/s",
            "cores": int(cores), "kind": "oracle",
            "sample": (f"{len(pick)} of {nf} fragments (seeded), their "
                       f"eigenpairs + whole-system H|phi> + {len(r.pairs)} "
                       f"pair blocks among them; {t:.1f} s")}


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on exactly one GPU (asked for {args.gpus}); the "
              "multi-GPU sharding of this path is a design note, not a "
              "measured configuration", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch

    import paper_1011_4764_amd as P
    from ofm_inputs import make_system

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    log("generating", args.config, "seed", args.seed)
    system = make_system(args.config, seed=args.seed)
    V = system.potential()
    g = system.grid
    n_states = system.n_basis
    log(f"grid {g.nx}x{g.ny}x{g.nz}, {system.n_frag} fragments, "
        f"{n_states} states")

    if args.calibrate_copy_gib > 0:
        n = int(args.calibrate_copy_gib * (1 << 30) // 4)
        a = torch.ones(n, dtype=torch.float32, device=dev)
        b = torch.empty_like(a)
        torch.mul(a, 1.0, out=b)   # one elementwise kernel: reads a, writes b
        torch.cuda.synchronize()
        log(f"copy calibration: elementwise kernel, {n * 4} bytes read, "
            f"{n * 4} bytes written")
        del a, b

    stream = torch.cuda.current_stream(dev)
    V_dev = torch.from_numpy(np.ascontiguousarray(V)).to(dev)
    torch.cuda.synchronize()

    def run_form(precision, tol, steps, warmup, profile, inflight=1):
        """Serial timed steps (stage times, kernel statistics), then, with
        inflight = 2, the same number of steps with two in flight: two
        contexts on two HIP streams, one host thread each, every step the
        whole path on its own (the global solve's latency-bound launches of
        one step overlap the bandwidth-bound fragment stage of the other)."""
        prec = P.OFM_FP64 if precision == "fp64" else P.OFM_MIXED_BF16X3
        ctx = P.ofm_create(0, stream.cuda_stream, prec)
        last = {}

        def step(cx, out):
            f = P.ofm_build_fragments(cx, (g.nx, g.ny, g.nz), g.h, V_dev,
                                      system.frag_lo, system.frag_dims,
                                      system.frag_states, origin=g.origin)
            deg = args.degree if precision == "fp64" else args.degree_mixed
            st, eps, it, cv = P.ofm_solve_fragments(cx, f, tol=tol,
                                                    degree=deg)
            m = P.ofm_matrix_elements(cx, f)
            gs = P.ofm_solve_global(cx, m, 1e-6)
            E = gs["E"]
            out.update(status=st, iters=it, conv=cv, n_pairs=f.n_pairs,
                       n_values=m.n_values, E=E, n_kept=gs["n_kept"],
                       stages=cx.stage_times())
            m.close()
            f.close()

        for w in range(warmup):
            t = time.perf_counter()
            step(ctx, last)
            log(f"{precision} tol {tol or 'default'} warmup {w}: "
                f"{time.perf_counter() - t:.3f} s, status {last['status']}, "
                f"iters max {int(last['iters'].max())}")
        ctx.reset_stats()
        ctx.set_profiling(profile)
        stage_sum = {"solve_ms": 0.0, "elements_ms": 0.0, "global_ms": 0.0}
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for k in range(steps):
            step(ctx, last)
            for key in stage_sum:
                stage_sum[key] += last["stages"][key]
            log(f"{precision} step {k} done")
        torch.cuda.synchronize()
        elapsed = time.perf_counter() - t0
        ctx.set_profiling(False)
        res = {"ms_step_serial": 1000.0 * elapsed / steps, "last": last}
        for key in stage_sum:
            res[key] = stage_sum[key] / steps
        for fam in ("stencil", "multistep", "sweep", "elements", "gram",
                    "filter", "tridiag"):
            res[fam] = ctx.kernel_stats(fam)
        res["ms_step"] = res["ms_step_serial"]
        if inflight == 2:
            stream2 = torch.cuda.Stream(dev)   # default priority
            ctx2 = P.ofm_create(0, stream2.cuda_stream, prec)
            other = {}
            for w in range(warmup):
                step(ctx2, other)
            outs = [dict() for _ in range(steps)]
            errors = []

            def worker(cx, first):
                try:
                    for k in range(first, steps, 2):
                        step(cx, outs[k])
                        log(f"{precision} in-flight step {k} done")
                except Exception as e:   # reported after the join
                    errors.append(e)

            torch.cuda.synchronize()
            t0 = time.perf_counter()
            th = [threading.Thread(target=worker, args=(cx, i))
                  for i, cx in enumerate((ctx, ctx2))]
            for x in th:
                x.start()
            for x in th:
                x.join()
            torch.cuda.synchronize()
            elapsed = time.perf_counter() - t0
            ctx2.close()
            if errors:
                raise errors[0]
            # every in-flight step delivers the serial step's eigenvalues
            for o in outs:
                if not np.array_equal(o["E"], last["E"]):
                    raise RuntimeError("an in-flight step differs from the "
                                       "serial one")
            res["ms_step"] = 1000.0 * elapsed / steps
        ctx.close()
        return res

    main_form = run_form(args.precision, args.tol, args.steps, args.warmup,
                         True, args.inflight)
    last = main_form["last"]
    ms_step = main_form["ms_step"]
    el, gr, td = main_form["elements"], main_form["gram"], main_form["tridiag"]
    # the dominant stencil kernel: two filter steps per launch where every
    # plane fits one workgroup, else one step per launch
    fam = max(("stencil", "multistep", "sweep"), key=lambda k: main_form[k]["ms"])
    st = main_form[fam]
    kname = STENCIL_KERNELS[fam]
    avg_ms = st["ms"] / max(st["launches"], 1)
    bytes_launch = st["bytes"] / max(st["launches"], 1)
    achieved = bytes_launch / (avg_ms * 1e-3) / 1e9 if avg_ms > 0 else 0.0
    solve_ms = main_form["solve_ms"]
    elem_ms = main_form["elements_ms"]
    glob_ms = main_form["global_ms"]
    n_elem = 2 * last["n_values"]
    E = last["E"]
    window = E[E <= E[0] + args.window]
    out = {
        "metric": "fragment eigenstates/s + H,S elements/s; mixed vs FP64 at 1e-5 Ha",
        "value": n_states / (ms_step * 1e-3),
        "unit": "fragment eigenstates/s (whole step)",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": ms_step, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None,
        "steps_in_flight": args.inflight,
        "serial_ms_per_step": main_form["ms_step_serial"],
        "dtype": "f64" if args.precision == "fp64" else "f32+bf16x3",
        "data": "synthetic",
        "config": {"workload": f"{args.config} seed {args.seed}: "
                               f"{len(system.atoms)} atoms, grid "
                               f"{g.nx}x{g.ny}x{g.nz} (h={g.h}), "
                               f"{system.n_frag} fragments, "
                               f"{n_states} states, {last['n_pairs']} pairs",
                   "precision": args.precision},
        "stages": {
            "fragment_eigenstates_per_s": n_states / (solve_ms * 1e-3),
            "solve_ms": solve_ms,
            "hs_elements_per_s": n_elem / (elem_ms * 1e-3),
            "elements_ms": elem_ms,
            "global_ms": glob_ms,
            "outer_iterations_max": int(last["iters"].max()),
            "outer_iterations_mean": float(last["iters"].mean()),
            "all_converged": bool(last["conv"].all()),
            "window_Ha": [float(window[0]), float(window[-1])],
            "window_eigenvalues": int(len(window)),
            "basis_kept": int(last["n_kept"]),
        },
        "roofline": {
            "kernel": kname,
            "bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS,
            "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
            "traffic": measured_traffic(
                f"{fam}_{args.config}_{args.precision}"),
            "traffic_unit": "bytes per launch (rocprofv3 FETCH_SIZE + "
                            "WRITE_SIZE, copy-calibrated)",
            "launches": st["launches"], "avg_launch_ms": avg_ms,
            "alg_bytes_per_launch": bytes_launch,
        },
        "other_kernels": {
            "gram": {"launches": gr["launches"],
                     "avg_ms": gr["ms"] / max(gr["launches"], 1),
                     "GBps": (gr["bytes"] / gr["ms"] / 1e6) if gr["ms"] else 0,
                     "TFLOPs": (gr["flops"] / gr["ms"] / 1e9) if gr["ms"] else 0},
            "tridiag": {"kernel": "k_mvt / k_mv + k_fin (Householder "
                                  "tridiagonal reduction of the global solve)",
                        "reductions": td["launches"],
                        "avg_ms": td["ms"] / max(td["launches"], 1),
                        "alg_bytes": td["bytes"] / max(td["launches"], 1),
                        "GBps": (td["bytes"] / td["ms"] / 1e6) if td["ms"] else 0,
                        "frac_hbm": ((td["bytes"] / td["ms"] / 1e6) / HBM_PEAK_GBS)
                                    if td["ms"] else 0},
            "elements": {"launches": el["launches"],
                         "avg_ms": el["ms"] / max(el["launches"], 1),
                         "GBps": (el["bytes"] / el["ms"] / 1e6) if el["ms"] else 0,
                         "TFLOPs": (el["flops"] / el["ms"] / 1e9) if el["ms"] else 0,
                         "frac_fp64_peak": ((el["flops"] / el["ms"] / 1e9)
                                            / FP64_PEAK_TFS) if el["ms"] else 0},
        },
    }
    if args.precision == "fp64" and not args.no_mixed:
        # the same workload in the mixed form, and FP64 stopped at the mixed
        # tolerance (equal accuracy); window eigenvalues compared to FP64's
        mx = run_form("mixed", 0.0, args.steps, args.warmup, True,
                      args.inflight)
        eq = run_form("fp64", 2e-5, args.steps, args.warmup, False)
        Em = mx["last"]["E"]
        nw = len(window)
        dE = float(np.abs(Em[:nw] - window).max())
        out["mixed"] = {
            "value": n_states / (mx["ms_step"] * 1e-3),
            "ms_per_step": mx["ms_step"],
            "serial_ms_per_step": mx["ms_step_serial"],
            "fragment_eigenstates_per_s": n_states / (mx["solve_ms"] * 1e-3),
            "hs_elements_per_s": 2 * mx["last"]["n_values"] / (mx["elements_ms"] * 1e-3),
            "solve_ms": mx["solve_ms"], "elements_ms": mx["elements_ms"],
            "global_ms": mx["global_ms"],
            "outer_iterations_max": int(mx["last"]["iters"].max()),
            "all_converged": bool(mx["last"]["conv"].all()),
            "window_Ha": [float(x) for x in Em[:nw]],
            "basis_kept": int(mx["last"]["n_kept"]),
            "window_max_abs_dE_vs_fp64_Ha": dE,
            "within_1e-5_Ha": bool(dE <= 1e-5),
            "fragment_stage_speedup_vs_fp64_own_tol": solve_ms / mx["solve_ms"],
            "fragment_stage_speedup_vs_fp64_equal_tol": eq["solve_ms"] / mx["solve_ms"],
            "whole_step_speedup_vs_fp64": ms_step / mx["ms_step"],
            "fp64_at_2e-5_solve_ms": eq["solve_ms"],
        }
        ms2 = mx["multistep"]
        if ms2["launches"]:
            a_ms = ms2["ms"] / ms2["launches"]
            ach = ms2["bytes"] / ms2["launches"] / (a_ms * 1e-3) / 1e9
            out["mixed"]["multistep_roofline"] = {
                "kernel": "k_apply_hm<float>", "bound": "hbm", "achieved": ach,
                "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": ach / HBM_PEAK_GBS, "avg_launch_ms": a_ms,
                "launches": ms2["launches"]}
        ms_ = mx["stencil"]
        if ms_["launches"]:
            a_ms = ms_["ms"] / ms_["launches"]
            ach = ms_["bytes"] / ms_["launches"] / (a_ms * 1e-3) / 1e9
            out["mixed"]["stencil_roofline"] = {
                "kernel": "k_apply_h<float>", "bound": "hbm", "achieved": ach,
                "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": ach / HBM_PEAK_GBS, "avg_launch_ms": a_ms,
                "launches": ms_["launches"]}
        mf = mx["filter"]
        if mf["launches"]:
            # on-chip filter: per point and step 9 LDS reads and 2 LDS
            # accesses of the column swap (4 B each); 32 flops per point-step
            a_ms = mf["ms"] / mf["launches"]
            psteps = mf["flops"] / 32.0 / mf["launches"]
            lds = psteps * LDS_BYTES_PER_POINT_STEP / (a_ms * 1e-3) / 1e9
            out["mixed"]["filter_roofline"] = {
                "kernel": "k_filter_resident (whole Chebyshev filter, vector "
                          "in LDS)",
                "bound": "lds", "achieved": lds, "peak": LDS_PEAK_GBS,
                "unit": "GB/s", "frac": lds / LDS_PEAK_GBS,
                "avg_launch_ms": a_ms, "launches": mf["launches"],
                "point_steps_per_s": psteps / (a_ms * 1e-3),
                "hbm_alg_bytes_per_launch": mf["bytes"] / mf["launches"],
                "hbm_traffic": measured_traffic(f"filter_{args.config}_mixed"),
                "hbm_GBps": mf["bytes"] / mf["launches"] / (a_ms * 1e-3) / 1e9}
        me = mx["elements"]
        if me["ms"]:
            out["mixed"]["elements_TFLOPs_useful"] = me["flops"] / me["ms"] / 1e9
    if not args.no_cpu_baseline:
        log("timing the CPU oracle on a sample")
        out["cpu_baseline"] = cpu_baseline(system, args.cpu_sample, args.seed)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
