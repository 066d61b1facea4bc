"""Benchmark: central eigenvalues per second of the DACP path on one MI355X.

A step is one dacp_central_eigs call (bound + window, filter, evolution,
projection, subspace diagonalisation, acceptance) on the chaotic Ising chain
H = sum Z_i Z_{i+1} + 1.05 sum X_i + 0.5 sum Z_i.  Default workload: L = 20
(D = 2^20), N = 5000 central eigenvalues.  Prints one JSON line.
"""
import argparse
import json
import math
import os
import sys
import time

T_PROCESS_START = time.perf_counter()

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "central eigenvalues/sec at L=20 (err≤1e-10) + filter HBM GB/s, plain vs tuned"
WORKLOADS = {
    "chain_L20_N5000": dict(L=20, N=5000, b=64),
    "chain_L16_N1000": dict(L=16, N=1000, b=64),
    "chain_L14_N500": dict(L=14, N=500, b=16),
    "chain_L10_N100": dict(L=10, N=100, b=4),
}
HBM_PEAK_GBPS = 8000.0
# HBM bytes per evolution launch measured with the FETCH_SIZE and WRITE_SIZE counters (each scaled by
# its reading on a 256 MiB device copy), for the kernel build and launch shape named by the key:
# (workload, kernel pair, column group).  Reported as roofline.traffic only for that configuration.
EVOLUTION_KERNELS = "k_rec_lo/k_rec_hi v5"
# key: (workload, kernel build, group, threads, fused tile, high-tile rows knob, XCD tile order knob)
MEASURED_TRAFFIC = {("chain_L20_N5000", EVOLUTION_KERNELS, 8, 1024, 8192, 0, 2): 279.67e6}
# Filter chain: counted bytes per order of one 8-column group (low + high kernel), FP32 and FP64 orders;
# key: (workload, kernel build, FP32 filter group, FP64 filter group).
FILTER_TRAFFIC_PER_ORDER = {("chain_L20_N5000", EVOLUTION_KERNELS, 8, 8): {"fp32": 306.3e6, "fp64": 628.0e6}}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1)
    ap.add_argument("--warmup", type=int, default=0)
    ap.add_argument("--workload", default="chain_L20_N5000",
                    choices=sorted(WORKLOADS) + ["glass_batch96_N200", "glass_L18_N3000_learned", "stage_sweep_L15",
                                                          "scaling_paper_models"])
    ap.add_argument("--mode", default="tuned", choices=["plain", "tuned"])
    ap.add_argument("--kfac", type=float, default=None)
    ap.add_argument("--seed", type=int, default=None, help="start-block seed (default: the library's)")
    ap.add_argument("--window-ratio", type=float, default=None)
    ap.add_argument("--basis-ratio", type=float, default=None)
    ap.add_argument("--tail", type=float, default=None, help="FP64 tail fraction of the filter (tuned mode)")
    ap.add_argument("--group", type=int, default=0)
    ap.add_argument("--block", type=int, default=0, help="start-block width b (default: the workload's)")
    ap.add_argument("--max-retries", type=int, default=None, help="wider-window retries (default: the library's)")
    ap.add_argument("--moments", action="store_true",
                    help="moment mode (App. C product identity): S and P from moments, no stored basis")
    ap.add_argument("--moment-mode", type=int, default=None, choices=[0, 1, 2],
                    help="opts.moment_mode: 0 S = V^T V and P = V^T (H V) of the stored basis, 1 moment mode, "
                         "2 stored basis with S and P from the anchor panels' moments (default: the mode's)")
    ap.add_argument("--eigvecs", action="store_true",
                    help="time dacp_central_eigpairs (eigenvalues and unit eigenvectors) instead of dacp_central_eigs")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample-s", type=float, default=12.0,
                    help="seconds of oracle applies timed for the CPU baseline (at least one apply)")
    ap.add_argument("--budget-s", type=float, default=480.0,
                    help="wall-time budget of the whole run from process start, seconds: at most one warm-up "
                         "call, then as many timed calls as fit (up to --steps), one plain FP64 call and the CPU "
                         "baseline; the JSON line reports the number of calls actually timed")
    ap.add_argument("--no-plain", action="store_true", help="skip the plain FP64 comparison call (tuned mode)")
    ap.add_argument("--batched-only", action="store_true",
                    help="glass_batch96_N200: only the autotuned batched calls (no learned window, default "
                         "options or per-realisation loop), so that the last call of a kernel trace is the "
                         "timed one")
    ap.add_argument("--profile-gemm", action="store_true",
                    help="run only the Gram product C = V^T V (V of 2^20 x 4096, FP64 MFMA) three times and "
                         "print one JSON line (for MFMA counter runs)")
    ap.add_argument("--profile-project", type=int, default=0, metavar="M",
                    help="run only the projection S = V^T V, P = V^T (H V) of the L = 20 chain on a seeded V of "
                         "2^20 x M columns, twice, and print one JSON line (for MFMA counter runs at the "
                         "benchmark's basis size)")
    ap.add_argument("--profile-kernels", action="store_true",
                    help="run only a device copy of known size and a short evolution at the workload's shape "
                         "(for hardware-counter runs), print one JSON line and exit")
    return ap.parse_args()


def opts_for(args, wl):
    from paper_2011_02107_amd import binding as B

    if args.mode == "plain":
        o = B.default_opts(b=wl["b"], kfac=18.0, window_ratio=2.2, precision=B.DACP_F64, group=args.group)
    else:
        # basis 1.2 N_w: at 1.1 - 1.15 a cluster of near-degenerate levels somewhere in the core can
        # stay unresolved (residuals ~5e-7) on some start blocks and force a retry with a wider window.
        # Window 2.4 N: at L = 20 the quadratic residual bound's core ends near |theta| = 0.44 a
        # (4851 values with a 2.2 N window, 5234 with 2.4 N, 5469 with 2.5 N, all 5625 candidates
        # with 2.6 N), so 2.4 N is the narrowest window that holds N = 5000 on the first attempt
        # (63.8 s; a retry with the 1.5x window would take about 80 s more)
        # S and P from the anchor panels' moments (moment_mode 2): the same core as V^T V and V^T (H V)
        # at L = 20 (5234 values at the 2.4 N window, rank 10962), 0.6 s against 8.4 s for the products
        o = B.default_opts(b=wl["b"], kfac=12.0, window_ratio=2.4, basis_ratio=1.2, precision=B.DACP_F32,
                           fp64_tail_frac=0.3, group=args.group, moment_mode=2)
    if args.block:
        o.b = args.block
    if args.max_retries is not None:
        o.max_retries = args.max_retries
    if args.seed is not None:
        o.seed = args.seed
    if args.kfac:
        o.kfac = args.kfac
    if args.window_ratio:
        o.window_ratio = args.window_ratio
    if args.basis_ratio:
        o.basis_ratio = args.basis_ratio
    if args.tail is not None:
        o.fp64_tail_frac = args.tail
    if args.moments:
        o.moment_mode = 1
    if args.moment_mode is not None:
        o.moment_mode = args.moment_mode
    return o


def progress(msg):
    print(f"# {msg}", file=sys.stderr, flush=True)


def host_info():
    """Host cores, CPU model and memory of the machine the benchmark runs on."""
    model = ""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    mem_gb = None
    try:
        with open("/proc/meminfo") as f:
            for line in f:
                if line.startswith("MemTotal"):
                    mem_gb = round(int(line.split()[1]) / 2**20, 1)
                    break
    except OSError:
        pass
    try:
        usable = len(os.sched_getaffinity(0))
    except AttributeError:
        usable = os.cpu_count()
    return {"nproc": os.cpu_count(), "usable_cpus": usable, "cpu_model": model, "mem_gb": mem_gb}


def cpu_baseline(wl, rep, sample_s, threads):
    """The oracle's matrix-free apply (numpy, FP64) on the workload's L x b block, spread over
    `threads` host threads by column slices (numpy releases the interpreter lock inside its array
    operations), repeated for about `sample_s` seconds and scaled to the run's total apply count
    (2K filter applies + the evolution steps).  Projection and the subspace solve are
    not counted, so the CPU figure is optimistic."""
    from concurrent.futures import ThreadPoolExecutor

    import numpy as np

    from oracle import hamiltonian
    from paper_2011_02107_amd import inputs

    L, b = wl["L"], rep["b"]
    terms = inputs.ising_chain(L)
    X = np.random.default_rng(0).standard_normal((1 << L, b))
    threads = max(1, min(threads, b))
    bounds = [(b * t // threads, b * (t + 1) // threads) for t in range(threads)]

    def one(c):
        c0, c1 = c
        return hamiltonian.apply_h(L, terms, X[:, c0:c1])

    n = 0
    with ThreadPoolExecutor(max_workers=threads) as ex:
        t0 = time.perf_counter()
        while True:
            parts = list(ex.map(one, bounds))
            n += 1
            if time.perf_counter() - t0 >= sample_s or n >= 64:
                break
        dt = (time.perf_counter() - t0) / n
    del parts
    # evol_steps counts the steps of one column group; every group takes as many, so the evolution
    # is evol_steps applies of the whole b-column block, as one oracle apply here
    applies = 2 * rep["K"] + rep["evol_steps"]
    total_s = applies * dt
    return {
        "value": wl["N"] / total_s,
        "unit": "eigenvalues/s",
        "cores": threads,
        "kind": "oracle",
        "sample": f"{n} oracle matrix-free applies (numpy FP64, L={L}, b={b} split over {threads} threads by "
        f"columns) at {dt:.3f} s each, scaled to the run's {applies} applies of all b columns "
        f"(2K filter + evolution steps); projection and subspace solve excluded",
        "host": host_info(),
    }


def profile_kernels(args):
    """A 256 MiB device copy (read and write byte counts known exactly) followed by 64 steps of the
    evolution recurrence on one column group at the workload's L, with the same kernels and tiles
    as a full step.  Used to scale the FETCH_SIZE / WRITE_SIZE counters to algorithmic bytes."""
    import numpy as np
    import torch

    from paper_2011_02107_amd import binding as B
    from paper_2011_02107_amd import inputs

    wl = WORKLOADS[args.workload]
    L = wl["L"]
    D = 1 << L
    ctx = B.Context(0)
    ham = B.dacp_build_hamiltonian(ctx, L, inputs.ising_chain(L))
    src = torch.ones(32 << 20, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    g = args.group or 8
    eb = 1.01 * (1.723 * L)  # above the chain norm 1.723 L - 0.73; checked by the evolution norm guard
    psi = torch.ones((D, g), dtype=torch.float64, device="cuda") / math.sqrt(D)
    n = 1
    V = torch.zeros((D, g * (2 * n + 1)), dtype=torch.float64, device="cuda")
    a_r = math.pi / 64.0  # k_1 = 64 evolution steps
    B.dacp_basis(ctx, ham, psi, V, eb, a_r * eb, n, group=g)
    torch.cuda.synchronize()
    # the filter chain on one group: 24 FP32 orders, then 8 FP64 orders (fused low/high kernels)
    fout = torch.empty((D, g), dtype=torch.float64, device="cuda")
    B.dacp_filter(ctx, ham, fout, eb, 0.05 * eb, 32, start=psi, precision=B.DACP_F32, fp64_tail=8)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes_each_way": src.numel() * 8, "evolution_steps": 64, "group": g, "L": L,
                      "algorithmic_bytes_per_step": 3 * D * g * 8, "e_bound": eb,
                      "filter_orders": {"fp32": 24, "fp64": 8}}), flush=True)


def profile_gemm(args):
    """The Gram product of the projection, C = V^T V, at D = 2^20 rows and m = 4096 columns (a full
    square, 2 D m^2 = 3.5e13 flops per call), three calls through the C ABI.  Used for the MFMA
    counters (SQ_INSTS_VALU_MFMA_MOPS_F64 x 512 = flops, SQ_VALU_MFMA_BUSY_CYCLES)."""
    import torch

    from paper_2011_02107_amd import binding as B

    ctx = B.Context(0)
    D, m = 1 << 20, 4096
    g = torch.Generator(device="cuda").manual_seed(3)
    V = torch.randn(D, m, dtype=torch.float64, device="cuda", generator=g)
    C = torch.empty(m, m, dtype=torch.float64, device="cuda")
    rates = []
    for _ in range(3):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        B.dacp_gemm(ctx, 1, 0, V, V, C)
        torch.cuda.synchronize()
        rates.append(2.0 * D * m * m / (time.perf_counter() - t0) / 1e12)
    print(json.dumps({"gemm": "C = V^T V", "D": D, "m": m, "flops_per_call": 2 * D * m * m,
                      "tflops": rates, "peak_tflops": 78.6}), flush=True)


def profile_project(args):
    """The projection of the benchmark (Sec. II.C, Eq. (9)) at its real shape: S = V^T V and
    P = V^T (H V) of the L = 20 chain for a seeded Gaussian V of D = 2^20 rows and m columns, two
    calls of dacp_project.  S and P are upper-triangle products of D m (m + 1) flops each."""
    import torch

    from paper_2011_02107_amd import binding as B
    from paper_2011_02107_amd import inputs

    ctx = B.Context(0)
    L, m = 20, args.profile_project
    D = 1 << L
    ham = B.dacp_build_hamiltonian(ctx, L, inputs.ising_chain(L))
    g = torch.Generator(device="cuda").manual_seed(5)
    V = torch.empty(D, m, dtype=torch.float64, device="cuda")
    for c0 in range(0, m, 1024):  # fill in slabs: one randn of the whole block would double the peak
        c1 = min(m, c0 + 1024)
        V[:, c0:c1] = torch.randn(D, c1 - c0, dtype=torch.float64, device="cuda", generator=g)
    torch.cuda.empty_cache()  # hand the slab back: the library allocates H V beside V when it fits
    S = torch.empty(m, m, dtype=torch.float64, device="cuda")
    P = torch.empty(m, m, dtype=torch.float64, device="cuda")
    times = []
    for _ in range(2):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        B.dacp_project(ctx, ham, V, S, P)
        torch.cuda.synchronize()
        times.append(time.perf_counter() - t0)
    print(json.dumps({"projection": "S = V^T V, P = V^T (H V)", "L": L, "D": D, "m": m,
                      "flops_per_product": D * m * (m + 1), "s_per_call": times, "peak_tflops": 78.6}), flush=True)


def train_window_model(ctx, Ls=(10, 11, 12, 13, 14), per_L=48, seed0=5000):
    """The learned window's network trained by the library's kernels on Lanczos / KPM labels of
    spin-glass shards with disorder seeds disjoint from the benchmark's (untimed set-up)."""
    import numpy as np

    from paper_2011_02107_amd import binding as B
    from paper_2011_02107_amd import inputs

    hams, feats = [], []
    for L in Ls:
        for s_ in range(per_L):
            h = B.dacp_build_hamiltonian(ctx, L, inputs.spin_glass(L, seed0 + 131 * L + s_))
            hams.append(h)
            feats.append(B.dacp_window_features(ctx, h))
    labels = B.dacp_window_labels(ctx, hams)
    net = B.Mlp(ctx, seed=0)
    loss = B.dacp_mlp_train(ctx, net, np.array(feats), labels, epochs=400, batch=64, lr=2e-3, seed=0)
    for h in hams:
        h.close()
    return net, {"realisations": len(feats), "final_loss": loss}


def batch96(args):
    """96 spin-glass shards (32 each at L = 12, 13, 14, disorder seeds 0..95), N = 200 each:
    dacp_central_eigs_batched (one persistent launch per stage) with the Lanczos / KPM windows and
    with the learned windows, against a per-realisation loop of plain FP64 dacp_central_eigs (timed
    on the first 12 realisations, scaled to 96)."""
    import numpy as np
    import torch

    from paper_2011_02107_amd import binding as B
    from paper_2011_02107_amd import inputs

    ctx = B.Context(0)
    sets = inputs.batched_spin_glass_set()
    hams = [B.dacp_build_hamiltonian(ctx, L, t) for (L, _, t) in sets]
    N = 200
    # b = 16 start columns: with 8, close pairs of levels are left unresolved more often and more
    # realisations need the retry round (autotuned schedule: 0.63 s per call against 0.76 s).
    # S and P from the anchor panels' moments (moment_mode 2): 0.50 s per call against 0.63 s with
    # the explicit products
    opts = B.default_opts(b=16, precision=B.DACP_F32, fp64_tail_frac=0.3, moment_mode=2)
    if args.moment_mode is not None:
        opts.moment_mode = args.moment_mode
    if args.block:
        opts.b = args.block
    if args.kfac:
        opts.kfac = args.kfac
    if args.basis_ratio:
        opts.basis_ratio = args.basis_ratio
    if not args.batched_only:
        t0 = time.perf_counter()
        net, train = train_window_model(ctx)
        train["s"] = time.perf_counter() - t0
    B.dacp_central_eigs_batched(ctx, hams[:3], N, opts)  # load the kernels
    for _ in range(args.warmup):  # untimed full calls: the device block cache then holds the call's buffers
        B.dacp_central_eigs_batched(ctx, hams, N, opts)

    def timed(model, o):
        times, last = [], None
        for _ in range(max(1, args.steps)):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            last = B.dacp_central_eigs_batched(ctx, hams, N, o, model=model, bound_margin=0.05)
            torch.cuda.synchronize()
            times.append(time.perf_counter() - t0)
        return float(np.median(times)), last

    # one-time schedule autotune (window, basis and filter order) on the whole set, retry rounds
    # included, not part of the timed calls
    t0 = time.perf_counter()
    tuned, t_sample = B.dacp_autotune_batched(ctx, hams, N, opts, sample_every=1)
    tuning_s = time.perf_counter() - t0
    B.dacp_central_eigs_batched(ctx, hams, N, tuned)  # the tuned shapes' buffers into the block cache
    options = {"kfac": tuned.kfac, "basis_ratio": tuned.basis_ratio, "window_ratio": tuned.window_ratio,
               "b": tuned.b, "moment_mode": tuned.moment_mode, "autotuned": True, "tuning_s": tuning_s,
               "tuning_sample_call_s": t_sample}
    if args.batched_only:
        dt, (eigs, errs, n_out, reps, st) = timed(None, tuned)
        options["retried"] = int(sum(r["retries"] > 0 for r in reps))
        print(json.dumps({
            "metric": "central eigenvalues/s, 96 spin-glass realisations L=12/13/14, N=200 each (batched)",
            "value": int(n_out.sum()) / dt, "unit": "eigenvalues/s", "s_per_call": dt,
            "all_reached_N": bool(np.all(n_out == N)), "shared_launch_ms": reps[0]["t_evol_ms"],
            "steps": max(1, args.steps), "warmup": args.warmup, "options": options,
            "dtype": "f32-filter+f64", "data": "synthetic"}), flush=True)
        return
    dt0, (eigs0, _, n_out0, reps0, _) = timed(None, opts)
    dt, (eigs, errs, n_out, reps, st) = timed(None, tuned)
    dtl, (eigl, errl, n_outl, repl, stl) = timed(net, opts)
    t0 = time.perf_counter()
    for h in hams[:12]:
        B.dacp_central_eigs(ctx, h, N, B.default_opts(b=8))
    loop = (time.perf_counter() - t0) / 12 * len(hams)
    options["retried"] = int(sum(r["retries"] > 0 for r in reps))
    print(json.dumps({
        "metric": "central eigenvalues/s, 96 spin-glass realisations L=12/13/14, N=200 each (batched)",
        "value": int(n_out.sum()) / dt, "unit": "eigenvalues/s", "realisations_per_s": len(hams) / dt,
        "s_per_call": dt, "all_reached_N": bool(np.all(n_out == N)),
        "shared_launch_ms": reps[0]["t_evol_ms"], "bounds_ms": reps[0]["t_bound_ms"],
        "learned": {"value": int(n_outl.sum()) / dtl, "s_per_call": dtl, "all_reached_N": bool(np.all(n_outl == N)),
                    "bounds_ms": float(np.median([r["t_bound_ms"] for r in repl])),
                    "fallbacks": int(sum(r["model_fallback"] for r in repl)),
                    "max_abs_diff_to_lanczos_kpm": float(np.abs(eigl - eigs).max()),
                    "speedup_vs_loop": loop / dtl, "training": train},
        "per_realisation_loop_fp64": {"value": N * len(hams) / loop, "s": loop, "timed": "first 12, scaled"},
        "speedup_vs_loop": loop / dt, "steps": max(1, args.steps), "warmup": args.warmup,
        "options": options,
        "default_options": {"value": int(n_out0.sum()) / dt0, "s_per_call": dt0, "kfac": opts.kfac,
                            "basis_ratio": opts.basis_ratio, "window_ratio": opts.window_ratio,
                            "retried": int(sum(r["retries"] > 0 for r in reps0)),
                            "max_abs_diff_to_tuned": float(np.abs(eigs0 - eigs).max())},
        "dtype": "f32-filter+f64", "data": "synthetic"}), flush=True)


def glass18_learned(args):
    """Spin-glass shard L = 18 (disorder seed 0), N = 3000: bound and window from the learned
    network (trained on Lanczos/KPM labels of 448 realisations, L = 10..16, seeds 1000+) against the
    Lanczos/KPM estimators; reports times, fallback and whether the predicted window held N."""
    import numpy as np

    from paper_2011_02107_amd import binding as B
    from paper_2011_02107_amd import inputs

    ctx = B.Context(0)
    t0 = time.perf_counter()
    hams, feats = [], []
    for L in (10, 11, 12, 13, 14, 15, 16):
        for s_ in range(80 if L <= 14 else 24):
            h = B.dacp_build_hamiltonian(ctx, L, inputs.spin_glass(L, 1000 + 131 * L + s_))
            hams.append(h)
            feats.append(B.dacp_window_features(ctx, h))
    labels = B.dacp_window_labels(ctx, hams)
    t_labels = time.perf_counter() - t0
    net = B.Mlp(ctx, seed=0)
    t0 = time.perf_counter()
    loss = B.dacp_mlp_train(ctx, net, np.array(feats), labels, epochs=400, batch=64, lr=2e-3, seed=0)
    t_train = time.perf_counter() - t0
    for h in hams:
        h.close()
    L, N = 18, 3000
    ham = B.dacp_build_hamiltonian(ctx, L, inputs.spin_glass(L, 0))
    opts = B.default_opts(b=64)
    truth = B.dacp_window_labels(ctx, [ham])[0]
    pred = B.dacp_mlp_predict(ctx, net, B.dacp_window_features(ctx, ham)[None, :])[0]
    t0 = time.perf_counter()
    e1, _, r1, _ = B.dacp_central_eigs_learned(ctx, ham, net, N, bound_margin=0.08, opts=opts)
    t_learned = time.perf_counter() - t0
    t0 = time.perf_counter()
    e2, _, r2, _ = B.dacp_central_eigs(ctx, ham, N, opts)
    t_plain = time.perf_counter() - t0
    print(json.dumps({
        "metric": "spin glass L=18 N=3000: learned window vs Lanczos/KPM", "unit": "s",
        "learned_s": t_learned, "lanczos_kpm_s": t_plain,
        "learned_bound_stage_ms": r1["t_bound_ms"], "lanczos_kpm_bound_stage_ms": r2["t_bound_ms"],
        "fallback": r1["model_fallback"], "window_held_N": int(r1["model_fallback"] == 0 and r1["retries"] == 0),
        "m_learned": r1["m"], "m_lanczos_kpm": r2["m"],
        "label_true": truth.tolist(), "label_pred": pred.tolist(),
        "max_abs_diff_between_paths": float(np.abs(np.sort(e1) - np.sort(e2)).max()),
        "train": {"realisations": len(feats), "label_s": t_labels, "train_s": t_train, "final_loss": loss},
        "data": "synthetic"}), flush=True)


def stage_sweep_L15(args):
    """Stage times against the number of central eigenvalues R at L = 15 (the timing analysis of
    Sec. IV: filter time ~ 1/R, evolution time ~ R^0, subspace diagonalisation ~ R^3), for the
    chaotic chain and a spin-glass shard, plain FP64 options, b = 16.  Each row is one call after an
    untimed warm-up call; the slopes are least-squares fits of log T against log R."""
    import numpy as np

    from paper_2011_02107_amd import binding as B
    from paper_2011_02107_amd import inputs

    ctx = B.Context(0)
    L = 15
    Rs = (30, 100, 300, 1000, 3000)
    out = {"metric": "stage times vs number of eigenvalues R (L=15, plain FP64, b=16)", "L": L, "models": {}}
    for name, terms in (("chain", inputs.ising_chain(L)), ("glass", inputs.spin_glass(L, 0))):
        ham = B.dacp_build_hamiltonian(ctx, L, terms)
        o = B.default_opts(b=16, kfac=18.0, window_ratio=2.2, precision=B.DACP_F64)
        B.dacp_central_eigs(ctx, ham, 300, o, raise_on_window=False)  # warm-up
        rows = []
        for R in Rs:
            eigs, errs, rep, st = B.dacp_central_eigs(ctx, ham, R, o, raise_on_window=False)
            rows.append({"R": R, "status": st, "K": rep["K"], "m": rep["m"], "evol_steps": rep["evol_steps"],
                         "t_filter_ms": rep["t_filter_ms"], "t_evol_ms": rep["t_evol_ms"],
                         "t_project_ms": rep["t_project_ms"], "t_gep_ms": rep["t_gep_ms"],
                         "t_accept_ms": rep["t_accept_ms"], "t_total_ms": rep["t_total_ms"]})
            print(f"# {name} R={R}: status {st}, total {rep['t_total_ms']:.1f} ms", file=sys.stderr, flush=True)
        ok = [r for r in rows if r["status"] == 0]
        slopes = {}
        if len(ok) >= 3:
            lr = np.log([r["R"] for r in ok])
            for key in ("t_filter_ms", "t_evol_ms", "t_gep_ms", "evol_steps"):
                slopes[key] = float(np.polyfit(lr, np.log([max(r[key], 1e-9) for r in ok]), 1)[0])
        out["models"][name] = {"rows": rows, "loglog_slopes": slopes}
    print(json.dumps(out), flush=True)


def scaling_paper_models(args):
    """Time against system size for the paper's two models with its distributions (Sec. III: the
    random transverse-field chain and the all-to-all spin-glass shard, J ~ U[-10/sqrt(L), 10/sqrt(L)],
    Gamma ~ U[0, 1]), N = 5000 central values, L = 15 .. 18, tuned options (S and P as explicit
    products unless --moment-mode says otherwise) with the evolution autotuned per shape (untimed,
    as in the headline).  alpha is the
    least-squares slope of log T against L (T = T0 exp(alpha L), the paper's scaling constant),
    for the filter + evolution time and for the whole call."""
    import numpy as np

    from paper_2011_02107_amd import binding as B
    from paper_2011_02107_amd import inputs

    ctx = B.Context(0)
    N = 5000
    Ls = (15, 16, 17, 18)
    small = B.dacp_build_hamiltonian(ctx, 8, inputs.ising_chain(8))
    B.dacp_central_eigs(ctx, small, 20, B.default_opts(b=4), raise_on_window=False)  # load the kernels
    small.close()
    out = {"metric": "time vs L, N=5000, paper models (tuned options)", "N": N,
           "moment_mode": args.moment_mode or 0, "models": {}}
    for name, build in (("ising", inputs.paper_tfim), ("glass", inputs.paper_sgs)):
        rows = []
        for L in Ls:
            ham = B.dacp_build_hamiltonian(ctx, L, build(L, 0))
            t0 = time.perf_counter()
            g, us = B.dacp_autotune(ctx, ham, b=64, steps=64)  # as in the headline's tuned mode, untimed
            t_tune = time.perf_counter() - t0
            # tuned options with the 2.2 N window (wider first windows do not help here: at L = 15,
            # N = 5000 is 15 % of the spectrum and a 2.6 N window, retried at 3.9 N, falls short)
            o = B.default_opts(b=64, kfac=12.0, window_ratio=2.2, basis_ratio=1.2, precision=B.DACP_F32,
                               fp64_tail_frac=0.3, moment_mode=args.moment_mode or 0)
            eigs, errs, rep, st = B.dacp_central_eigs(ctx, ham, N, o, raise_on_window=False)
            rows.append({"L": L, "status": st, "accepted": len(eigs), "retries": rep["retries"], "K": rep["K"], "m": rep["m"],
                         "evol_steps": rep["evol_steps"], "t_filter_ms": rep["t_filter_ms"],
                         "t_evol_ms": rep["t_evol_ms"], "t_project_ms": rep["t_project_ms"],
                         "t_gep_ms": rep["t_gep_ms"], "t_total_ms": rep["t_total_ms"],
                         "autotune": {"group": g, "rec_threads": ctx.tune_get("rec_threads"),
                                      "rec_tile": ctx.tune_get("rec_tile"), "rec_hi_w": ctx.tune_get("rec_hi_w"),
                                      "us_per_column_step": us, "s": t_tune}})
            ham.close()
            print(f"# {name} L={L}: status {st}, total {rep['t_total_ms']:.0f} ms, evolution {rep['t_evol_ms']:.0f} ms",
                  file=sys.stderr, flush=True)
        ok = [r for r in rows if r["status"] == 0]
        fit = {}
        if len(ok) >= 2:
            Lv = [r["L"] for r in ok]
            fit["alpha_filter_plus_evolution"] = float(np.polyfit(Lv, np.log([r["t_filter_ms"] + r["t_evol_ms"]
                                                                              for r in ok]), 1)[0])
            fit["alpha_total"] = float(np.polyfit(Lv, np.log([r["t_total_ms"] for r in ok]), 1)[0])
        out["models"][name] = {"rows": rows, **fit}
    print(json.dumps(out), flush=True)


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the multi-GPU form (start columns "
              "sharded across GPUs, V panels passed around a ring for S and P) is not built", file=sys.stderr)
        sys.exit(2)
    if args.profile_kernels:
        return profile_kernels(args)
    if args.profile_gemm:
        return profile_gemm(args)
    if args.profile_project:
        return profile_project(args)
    if args.workload == "glass_batch96_N200":
        return batch96(args)
    if args.workload == "glass_L18_N3000_learned":
        return glass18_learned(args)
    if args.workload == "stage_sweep_L15":
        return stage_sweep_L15(args)
    if args.workload == "scaling_paper_models":
        return scaling_paper_models(args)
    import numpy as np
    import torch

    from paper_2011_02107_amd import binding as B
    from paper_2011_02107_amd import inputs

    wl = WORKLOADS[args.workload]
    L, N = wl["L"], wl["N"]
    terms = inputs.ising_chain(L)
    ctx = B.Context(0)
    ham = B.dacp_build_hamiltonian(ctx, L, terms)
    opts = opts_for(args, wl)
    tuned = None
    if args.mode == "tuned" and not args.group:
        # one-time autotune of the evolution kernels at this shape (not part of the timed steps)
        t0 = time.perf_counter()
        g, us = B.dacp_autotune(ctx, ham, b=wl["b"], steps=64)
        tuned = {"group": g, "us_per_column_step": us, "s": time.perf_counter() - t0}
    # load every kernel once on a tiny problem (not a timed step)
    small = B.dacp_build_hamiltonian(ctx, 8, inputs.ising_chain(8))
    B.dacp_central_eigs(ctx, small, 20, B.default_opts(b=4), raise_on_window=False)
    small.close()
    vecs = torch.empty((1 << L, N), dtype=torch.float64, device="cuda:0") if args.eigvecs else None

    def call():
        if vecs is not None:
            return B.dacp_central_eigpairs(ctx, ham, N, vecs, opts)
        return B.dacp_central_eigs(ctx, ham, N, opts)

    def elapsed():
        return time.perf_counter() - T_PROCESS_START

    # Wall budget.  One call at L = 20 takes about a minute, so `--steps` and `--warmup` are caps:
    # at most one untimed warm-up call, then timed calls while the next one still fits, keeping
    # room for the plain FP64 call (about 1.4 tuned calls) and the CPU baseline.
    t_call = None
    for i in range(min(args.warmup, 1)):
        progress(f"warm-up call {i + 1} at {elapsed():.0f} s")
        t0 = time.perf_counter()
        call()
        t_call = time.perf_counter() - t0
        progress(f"warm-up call done: {t_call:.1f} s")
    want_plain = args.mode == "tuned" and not args.no_plain
    cpu_s = 0.0 if args.no_cpu_baseline else args.cpu_sample_s + 15.0

    def reserve(tc):
        return (1.5 * tc if want_plain else 0.0) + cpu_s + 10.0

    torch.cuda.synchronize()
    t0 = time.perf_counter()
    reps = []
    n_ok = 0
    while len(reps) < max(1, args.steps):
        eigs, errs, rep, st = call()
        reps.append(rep)
        n_ok += len(eigs)
        tc = (time.perf_counter() - t0) / len(reps)
        progress(f"timed call {len(reps)}: {len(eigs)} values, {tc:.1f} s per call so far, elapsed {elapsed():.0f} s")
        if elapsed() + tc + reserve(tc) > args.budget_s:
            break
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    steps_timed = len(reps)
    t_call = dt / steps_timed
    rep = reps[-1]
    D = 1 << L
    g = rep["evol_group"]
    # one evolution step of a column group reads T_k and T_{k-1} and writes T_{k+1}:
    # 3 D g 8 algorithmic bytes per step (one step = the low-bit and the high-bit pass at L >= 15)
    bytes_per_launch = 3.0 * D * g * 8
    evol_launch_ms = rep["evol_kernel_ms"] / max(1, rep["evol_launches"])
    achieved = bytes_per_launch / (evol_launch_ms * 1e-3) / 1e9
    # filter: per order 5 D b s algorithmic bytes (w round trip included); s = 4 for the FP32 orders
    # and 8 for the FP64 tail (all orders FP64 in plain mode)
    K = rep["K"]
    k64 = min(K, math.ceil(opts.fp64_tail_frac * K)) if opts.precision == B.DACP_F32 else K
    filter_bytes = 5.0 * D * rep["b"] * (4 * (K - k64) + 8 * k64)
    filter_gbps = filter_bytes / (rep["t_filter_ms"] * 1e-3) / 1e9
    out = {
        "metric": METRIC,
        "value": n_ok / dt,
        "unit": "eigenvalues/s",
        "n_gpus": 1,
        "steps": steps_timed,
        "warmup": min(args.warmup, 1),
        "ms_per_step": dt * 1e3 / steps_timed,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if opts.precision == B.DACP_F64 else "f32-filter+f64",
        "data": "synthetic",
        "config": {
            "workload": args.workload,
            "hamiltonian": "sum Z_i Z_i+1 + 1.05 sum X_i + 0.5 sum Z_i, open chain",
            "L": L,
            "N": N,
            "mode": args.mode,
            "eigenvectors": bool(args.eigvecs),
            "moment_mode": int(opts.moment_mode),
            "b": rep["b"],
            "group": g,
            "K": rep["K"],
            "m": rep["m"],
            "rank": rep["rank"],
            "retries": rep["retries"],
            "evol_steps": rep["evol_steps"],
            "acceptance": "block quadratic residual bound on the Rayleigh quotients of the Ritz vectors <= 1e-10 ||H|| (no oracle at this size)",
            "autotune": tuned,
            "evolution_kernel_config": {k: ctx.tune_get(k) for k in ("group", "rec_threads", "rec_tile", "rec_hi_w",
                                                                     "rec_xcd")},
        },
        "roofline": {
            "bound": "hbm",
            "kernel": "k_rec_lo / k_rec_hi (fused evolution recurrence, FP64)",
            "achieved": achieved,
            "peak": HBM_PEAK_GBPS,
            "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBPS,
            "traffic": MEASURED_TRAFFIC.get((args.workload, EVOLUTION_KERNELS, g, ctx.tune_get("rec_threads"),
                                             ctx.tune_get("rec_tile"), ctx.tune_get("rec_hi_w"),
                                             ctx.tune_get("rec_xcd"))),
            "avg_launch_ms": evol_launch_ms,
            "bytes_per_launch": bytes_per_launch,
        },
        "stages_ms": {k: rep[k] for k in ("t_bound_ms", "t_filter_ms", "t_evol_ms", "t_project_ms", "t_gep_ms",
                                          "t_accept_ms", "t_total_ms")},
        "filter_algorithmic_GBps": filter_gbps,
    }
    # counted filter bytes per order (FETCH_SIZE + WRITE_SIZE, fused chain, 8-column groups at L = 20)
    fb = FILTER_TRAFFIC_PER_ORDER.get((args.workload, EVOLUTION_KERNELS, ctx.tune_get("filter_group_f32"),
                                       ctx.tune_get("filter_group_f64")))
    if fb is not None:
        groups = rep["b"] // 8
        counted = groups * (fb["fp32"] * (K - k64) + fb["fp64"] * k64)
        out["filter_counted"] = {"bytes": counted, "GBps": counted / (rep["t_filter_ms"] * 1e-3) / 1e9,
                                 "bytes_per_order_per_group": fb}
    out["budget"] = {"requested_steps": args.steps, "requested_warmup": args.warmup, "budget_s": args.budget_s}
    if want_plain:
        if elapsed() + 1.5 * t_call + cpu_s < args.budget_s:
            progress(f"plain FP64 call at {elapsed():.0f} s")
            plain_args = argparse.Namespace(**{**vars(args), "mode": "plain"})
            popts = opts_for(plain_args, wl)
            t0 = time.perf_counter()
            pe, _, prep, pst = B.dacp_central_eigs(ctx, ham, N, popts)
            tp = time.perf_counter() - t0
            out["plain"] = {
                "value": len(pe) / tp, "unit": "eigenvalues/s", "s": tp, "dtype": "f64",
                "options": "FP64 filter, kfac 18, window 2.2, basis 1.5, no autotune of the options",
                "K": prep["K"], "m": prep["m"], "rank": prep["rank"], "retries": prep["retries"],
                "evol_steps": prep["evol_steps"],
                "stages_ms": {k: prep[k] for k in ("t_bound_ms", "t_filter_ms", "t_evol_ms", "t_project_ms",
                                                   "t_gep_ms", "t_accept_ms", "t_total_ms")},
                "tuned_over_plain": (n_ok / dt) / (len(pe) / tp),
                "max_abs_diff_to_tuned": float(np.abs(np.sort(pe) - np.sort(eigs)).max()),
            }
            progress(f"plain call done: {tp:.1f} s")
        else:
            out["plain"] = {"skipped": f"no room in the {args.budget_s:.0f} s budget"}
    if not args.no_cpu_baseline:
        progress(f"CPU baseline at {elapsed():.0f} s")
        out["cpu_baseline"] = cpu_baseline(wl, rep, args.cpu_sample_s, min(16, host_info()["usable_cpus"] or 1))
    out["wall_s"] = elapsed()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
