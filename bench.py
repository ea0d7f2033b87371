"""Benchmark: time-to-eps and coordinate updates/s of LGCD on one MI355X.

A step is one complete solve of the paper-shaped workload (P=7, K=25, W=200,
T=150,000, Bernoulli(0.007) x N(0, 10^2) activations, noise sigma 0.1,
lambda = 0.1 lambda_max, eps = 1e-6, float descent with double-precision
stop test) with X already resident in HBM: beta init, lambda_max, the coloured
descent phases and the final double-precision check, through the C ABI.

Prints one JSON line.  value = coordinate updates per second over the timed
steps (whole job); ms_per_step = time-to-eps of one solve.

Three more workloads are measured beside it (skip with --no-long /
--no-batched / --no-served):
  * long: one signal of T = 5,000,000 (P=7 K=25 W=200), time-to-eps;
  * batched: 256 signals, T uniform in [10,000, 500,000], shared dictionary
    P=7 K=25 W=64, Bernoulli(0.005) activations, solved in one batched call,
    against the same signals solved one call per signal on the same GPU;
  * served: a Poisson stream of encode requests (lengths log-uniform in
    [2,000, 2,000,000], P=7 K=25 W=200) through dicod_submit / dicod_poll at
    0.5 and 0.8 of the measured saturation rate: p50/p99 latency and
    updates/s, against the same requests solved one at a time.
"""
import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

PEAK_HBM_GBS = 8000.0
KERNEL_SRC = os.path.join(ROOT, "paper_1705_10087_amd", "csrc", "kernels.hip")
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "lgcd_phase_paper_shaped_traffic.json")


def algorithmic_bytes_per_update(K, W, elem=4):
    """S slice read + window of g read + written: 3 * K * (2W - 1) elements."""
    return 3 * elem * K * (2 * W - 1)


def kernel_sha():
    return hashlib.sha256(open(KERNEL_SRC, "rb").read()).hexdigest()[:16]


def measured_traffic():
    """HBM bytes per LGCD launch from the committed rocprofv3 counter runs, or
    None when they are missing or were taken on a different kernel source."""
    try:
        rec = json.load(open(TRAFFIC_FILE))
    except (OSError, ValueError):
        return None
    if rec.get("kernel_src_sha") != kernel_sha():
        return None
    return rec.get("hbm_bytes_per_launch")


def cpu_baseline(X, D, lam, eps, M, cap, colors):
    import oracle
    t0 = time.perf_counter()
    Z, st, _ = oracle.lgcd(X.astype(np.float64), D.astype(np.float64), lam, eps, M, cap=cap,
                           colors=colors)
    dt = time.perf_counter() - t0
    return {"value": st["n_updates"] / dt, "unit": "coord updates/s", "cores": 1,
            "kind": "oracle", "time_to_eps_s": dt, "n_updates": int(st["n_updates"]),
            "sample": f"one full solve of the same workload by the FP64 C oracle, same "
                      f"schedule ({colors} colours, M={M}, update cap {cap}), single thread"}


def effective_cap(cap, W):
    """The library's update cap: cap > 0 as given, 0 = none, -1 = max(4, round(2 sqrt(W)))."""
    return cap if cap >= 0 else max(4, int(math.floor(2.0 * math.sqrt(W) + 0.5)))


def ms_per_step_of(stats, wall, steps):
    return 1e3 * wall / steps


def s_last(stats):
    return stats[-1]


def adjacent_pairs(tr, W):
    """Updates of one phase in adjacent segments: pairs, and pairs closer than
    W (interfering, Sec. 3)."""
    by = {}
    for p, m, t in zip(tr["phase"], tr["seg"], tr["t0"]):
        by.setdefault((int(p), int(m)), []).append(int(t))
    n_adj = n_int = 0
    for (p, m), us in by.items():
        vs = by.get((p, m + 1))
        if not vs:
            continue
        vs = np.asarray(vs)
        for u in us:
            n_adj += vs.size
            n_int += int(np.count_nonzero(np.abs(u - vs) < W))
    return n_adj, n_int


def _gen_signal(job):
    import synth
    P, K, W, T, rho, sigma, seed, D = job
    return synth.generate_fast(P, K, W, int(T), rho, sigma, seed, D)


def gen_signals(P, K, W, lengths, rho, sigma, seed0, D, workers=8):
    """Seeded signals of the given lengths with a shared dictionary, generated
    in a process pool (before the GPU is initialised)."""
    import concurrent.futures as cf
    import multiprocessing as mp
    jobs = [(P, K, W, T, rho, sigma, seed0 + i, D) for i, T in enumerate(lengths)]
    with cf.ProcessPoolExecutor(max_workers=workers, mp_context=mp.get_context("fork")) as ex:
        return list(ex.map(_gen_signal, jobs, chunksize=4))


def batched_bench(d, torch, D, Ts, Xs, cap, colors):
    """One batched call over all signals vs one call per signal."""
    K, P, W = D.shape
    n = len(Ts)
    Ls = [int(T) - W + 1 for T in Ts]
    x_off = np.concatenate([[0], np.cumsum([P * int(T) for T in Ts])[:-1]]).astype(np.int64)
    z_off = np.concatenate([[0], np.cumsum([K * L for L in Ls])[:-1]]).astype(np.int64)
    dev = torch.device("cuda:0")
    Xd = torch.from_numpy(np.concatenate([X.ravel() for X in Xs])).to(dev)
    nz = int(sum(K * L for L in Ls))
    Zb = torch.empty(nz, dtype=torch.float64, device=dev)
    Zs = torch.empty(nz, dtype=torch.float64, device=dev)
    lam = np.full(n, -0.1)
    with d.Context(update_cap=cap, colors=colors) as c:
        c.set_dictionary(D)
        c.solve_batch_device(Xd, Ts, x_off, lam, 1e-6, None, Zb, z_off)   # warm-up
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        sts = c.solve_batch_device(Xd, Ts, x_off, lam, 1e-6, None, Zb, z_off)
        torch.cuda.synchronize()
        t_batch = time.perf_counter() - t0
        upd_b = sum(s["n_updates"] for s in sts)
        t0 = time.perf_counter()
        upd_s = 0
        for i in range(n):
            Xi = Xd[x_off[i]:x_off[i] + P * int(Ts[i])].view(P, int(Ts[i]))
            Zi = Zs[z_off[i]:z_off[i] + K * Ls[i]].view(K, Ls[i])
            _, st, _ = c.solve_device(Xi, -0.1, 1e-6, 0, Zi)
            upd_s += st["n_updates"]
        torch.cuda.synchronize()
        t_seq = time.perf_counter() - t0
    same = bool(torch.equal(Zb, Zs))
    return {"workload": f"{n} signals, T uniform in [10000, 500000], P={P} K={K} W={W}, "
                        "rho=0.005, sigma=0.1, lambda=0.1*lambda_max per signal, eps=1e-6",
            "total_samples": int(sum(int(T) for T in Ts)), "coefficients": nz,
            "batched": {"time_to_eps_s": t_batch, "updates": int(upd_b),
                        "updates_per_s": upd_b / t_batch,
                        "converged": int(sum(s["converged"] for s in sts))},
            "per_signal": {"time_to_eps_s": t_seq, "updates": int(upd_s),
                           "updates_per_s": upd_s / t_seq},
            "speedup": t_seq / t_batch, "batched_equals_per_signal": same}


def long_bench(d, torch, D, X, cap, colors, steps=2):
    """Long single signal (T = 5,000,000): time-to-eps on the device."""
    K, P, W = D.shape
    dev = torch.device("cuda:0")
    Xd = torch.from_numpy(X).to(dev)
    Zd = torch.empty((K, X.shape[1] - W + 1), dtype=torch.float64, device=dev)
    with d.Context(update_cap=cap, colors=colors) as c:
        c.set_dictionary(D)
        c.solve_device(Xd, -0.1, 1e-6, 0, Zd)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            _, st, _ = c.solve_device(Xd, -0.1, 1e-6, 0, Zd)
        torch.cuda.synchronize()
        t = (time.perf_counter() - t0) / steps
    return {"workload": f"single signal P={P} K={K} W={W} T={X.shape[1]}, rho=0.007, "
                        "sigma=0.1, lambda=0.1*lambda_max, eps=1e-6",
            "precision": "FP32 descent, FP64 beta init and stop test",
            "time_to_eps_s": t, "updates": st["n_updates"], "updates_per_s": st["n_updates"] / t,
            "n_seg": st["n_seg"], "n_phases": st["n_phases"], "t_init_ms": st["t_init_ms"],
            "t_cd_ms": st["t_cd_ms"], "t_verify_ms": st["t_verify_ms"],
            "round_updates": st["round_updates"], "round_ms": st["round_ms"],
            "converged": st["converged"]}


def served_bench(d, torch, D, pool_T, pool_X, n_req, cap, colors, seed):
    """Poisson stream through dicod_submit / dicod_poll vs requests solved alone."""
    import threading
    import synth
    K, P, W = D.shape
    Lmax = max(int(T) for T in pool_T) - W + 1
    out_buf = torch.empty(K * Lmax, dtype=torch.float64, pin_memory=True).numpy()
    npool = len(pool_X)
    res = {"workload": f"requests drawn from {npool} signals with T log-uniform in [2000, "
                       f"2000000], P={P} K={K} W={W}, rho=0.007, sigma=0.1, "
                       "lambda=0.1*lambda_max, eps=1e-6",
           "requests": n_req}

    def run_stream(c, rate):
        """Submits n_req requests (closed batch if rate is None) and polls
        them; returns (makespan s, client latencies ms, server latencies ms,
        updates)."""
        arrivals = (np.zeros(n_req) if rate is None else
                    synth.poisson_arrivals(n_req, rate, seed + int(rate or 0)))
        t_sub = [0.0] * n_req
        ids = [None] * n_req
        done = {}
        start = time.perf_counter()

        def submitter():
            for i in range(n_req):
                dt = start + arrivals[i] - time.perf_counter()
                if dt > 0:
                    time.sleep(dt)
                t_sub[i] = time.perf_counter()
                ids[i] = c.submit(pool_X[i % npool], -0.1, 1e-6)

        th = threading.Thread(target=submitter)
        th.start()
        lat_c, lat_s, upd = [], [], 0
        while len(done) < n_req:
            for i in range(n_req):
                if i in done or ids[i] is None:
                    continue
                ok, _, st = c.poll(ids[i], int(pool_T[i % npool]), out_buf)
                if ok:
                    done[i] = time.perf_counter()
                    lat_c.append(1e3 * (done[i] - t_sub[i]))
                    lat_s.append(st["t_latency_ms"])
                    upd += st["n_updates"]
            time.sleep(5e-5)
        th.join()
        return max(done.values()) - start, np.array(lat_c), np.array(lat_s), upd

    with d.Context(update_cap=cap, colors=colors) as c:
        c.set_dictionary(D)
        # alone: every distinct request solved by itself
        alone, upd_alone = [], 0
        for i in range(min(n_req, npool)):
            t0 = time.perf_counter()
            _, st = c.solve(pool_X[i], -0.1, 1e-6)
            alone.append(1e3 * (time.perf_counter() - t0))
            upd_alone += st["n_updates"]
        alone = np.array(alone)
        res["alone"] = {"p50_ms": float(np.percentile(alone, 50)),
                        "p99_ms": float(np.percentile(alone, 99)),
                        "requests_per_s": 1e3 / alone.mean(),
                        "updates_per_s": upd_alone / (alone.sum() / 1e3)}
        run_stream(c, None)  # warm-up of the serving path
        mk, lc, ls, upd = run_stream(c, None)
        sat = n_req / mk
        res["saturation"] = {"requests_per_s": sat, "updates_per_s": upd / mk,
                             "makespan_s": mk}
        for frac in (0.5, 0.8):
            mk, lc, ls, upd = run_stream(c, frac * sat)
            res[f"rate_{frac}"] = {"rate_per_s": frac * sat,
                                   "p50_ms": float(np.percentile(lc, 50)),
                                   "p99_ms": float(np.percentile(lc, 99)),
                                   "server_p50_ms": float(np.percentile(ls, 50)),
                                   "server_p99_ms": float(np.percentile(ls, 99)),
                                   "updates_per_s": upd / mk}
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--cap", type=int, default=-1,
                    help="updates per segment per phase (-1: the library's automatic cap)")
    ap.add_argument("--n-seg", type=int, default=0, help="0 = library default")
    ap.add_argument("--colors", type=int, default=3, help="phase classes of the schedule")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-sweep", action="store_true")
    ap.add_argument("--copy-calib", type=int, default=0, metavar="MIB",
                    help="first run one plain device copy of MIB MiB (counter calibration)")
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--no-served", action="store_true")
    ap.add_argument("--no-long", action="store_true")
    ap.add_argument("--batch-signals", type=int, default=256)
    ap.add_argument("--served-requests", type=int, default=200)
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on exactly one GPU; --gpus "
                                   f"{args.gpus} is not supported (multi-GPU sharding is "
                                   "a design only)"}))
        sys.exit(2)

    import torch
    import synth
    import paper_1705_10087_amd as d

    # inputs of the batched and served workloads, drawn before the GPU starts
    batch_data = served_data = long_data = None
    if not args.no_batched:
        a = synth.BATCH_ATOM
        Db = synth.dictionary(np.random.Generator(np.random.PCG64(args.seed + 11)),
                              a["K"], a["P"], a["W"]).astype(np.float32)
        Tb = synth.batch_lengths(args.batch_signals, 10_000, 500_000, args.seed + 12)
        Xb = gen_signals(a["P"], a["K"], a["W"], Tb, a["rho"], a["sigma_noise"],
                         args.seed + 1000, Db)
        batch_data = (Db, Tb, Xb)
        print(f"[bench] batched inputs: {len(Tb)} signals, {int(Tb.sum())} samples",
              file=sys.stderr, flush=True)
    if not args.no_long:
        w = synth.LONG
        Dl = synth.dictionary(np.random.Generator(np.random.PCG64(args.seed + 31)),
                              w.K, w.P, w.W).astype(np.float32)
        long_data = (Dl, synth.generate_fast(w.P, w.K, w.W, w.T, w.rho, w.sigma_noise,
                                             args.seed + 32, Dl))
        print(f"[bench] long input: T={w.T}", file=sys.stderr, flush=True)
    if not args.no_served:
        Ds = synth.dictionary(np.random.Generator(np.random.PCG64(args.seed + 21)),
                              25, 7, 200).astype(np.float32)
        Ts = synth.served_lengths(min(64, args.served_requests), 2_000, 2_000_000,
                                  args.seed + 22)
        Xs = gen_signals(7, 25, 200, Ts, 0.007, 0.1, args.seed + 5000, Ds)
        served_data = (Ds, Ts, Xs)
        print(f"[bench] served inputs: {len(Ts)} signals, {int(Ts.sum())} samples",
              file=sys.stderr, flush=True)

    w = synth.PAPER
    X, D, _ = synth.workload(w, args.seed)
    K, P, W = D.shape
    T = X.shape[1]
    L = T - W + 1
    dev = torch.device("cuda:0")
    Xd = torch.from_numpy(X).to(dev)
    Zd = torch.empty((K, L), dtype=torch.float64, device=dev)
    stream = torch.cuda.current_stream(dev).cuda_stream
    if args.copy_calib > 0:
        # a plain copy of known size: its FETCH_SIZE / WRITE_SIZE readings
        # convert the counters of the LGCD kernels into bytes
        n = args.copy_calib * (1 << 20) // 4
        a = torch.ones(n, dtype=torch.float32, device=dev)
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        b.copy_(a)
        torch.cuda.synchronize()
        del a, b
    print(f"[bench] workload {w.name}; steps={args.steps} warmup={args.warmup}",
          file=sys.stderr, flush=True)

    with d.Context(update_cap=args.cap, colors=args.colors) as c:
        c.set_dictionary(D)
        for i in range(args.warmup):
            _, st, _ = c.solve_device(Xd, -w.lam_rel, w.eps, args.n_seg, Zd, stream)
        torch.cuda.synchronize()
        stats = []
        t0 = time.perf_counter()
        for i in range(args.steps):
            _, st, _ = c.solve_device(Xd, -w.lam_rel, w.eps, args.n_seg, Zd, stream)
            stats.append(st)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        print(f"[bench] timed {args.steps} solves in {wall:.3f} s", file=sys.stderr, flush=True)

    with d.Context(update_cap=args.cap, timing=1, colors=args.colors) as c:
        c.set_dictionary(D)
        _, tst, _ = c.solve_device(Xd, -w.lam_rel, w.eps, args.n_seg, Zd, stream)
        torch.cuda.synchronize()

    n_upd = sum(s["n_updates"] for s in stats)
    ms_per_step = 1e3 * wall / args.steps
    bpu = algorithmic_bytes_per_update(K, W)
    # dominant kernel: the float LDS-state phase kernel of the first round
    # (the double finish round, if any, runs the HBM-state kernel)
    assert tst["round_state"][0] == 0, "first round expected on the float LDS-state kernel"
    launches = tst["round_launches"][0]
    kern_ms = tst["round_kernel_ms"][0]
    upd0 = tst["round_updates"][0]
    achieved = (upd0 * bpu / launches) / (kern_ms / launches * 1e-3) / 1e9
    traffic = measured_traffic()
    s0 = stats[-1]
    out = {
        "metric": "time-to-eps (s) & coord updates/s on 1 MI355X; p50/p99 solve latency "
                  "(served)",
        "value": n_upd / wall,
        "unit": "coord updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "time_to_eps_s": ms_per_step / 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": w.name, "P": P, "K": K, "W": W, "T": T, "rho": w.rho,
                   "sigma_noise": w.sigma_noise, "lambda": "0.1*lambda_max",
                   "eps": w.eps, "n_seg": s0["n_seg"], "seg_len": s0["seg_len"],
                   "update_cap": effective_cap(args.cap, w.W),
                   "precision": "FP32 descent, FP64 stop test",
                   "schedule": f"{args.colors}-colour phases", "seed": args.seed},
        "solve": {"n_updates": s0["n_updates"], "n_phases": s0["n_phases"],
                  "n_phase_launches": s0["n_phase_launches"], "n_refresh": s0["n_refresh"],
                  "nnz": s0["nnz"], "objective": s0["objective"], "max_dz": s0["max_dz"],
                  "converged": s0["converged"], "t_init_ms": s0["t_init_ms"],
                  "t_cd_ms": s0["t_cd_ms"], "t_verify_ms": s0["t_verify_ms"],
                  "round_updates": s0["round_updates"], "round_phases": s0["round_phases"],
                  "round_ms": s0["round_ms"],
                  "polished_fp64": s0["polished_fp64"]},
        "roofline": {"kernel": "k_lgcd_phase<float> (LDS state)", "bound": "hbm",
                     "achieved": achieved, "peak": PEAK_HBM_GBS, "unit": "GB/s",
                     "frac": achieved / PEAK_HBM_GBS, "traffic": traffic,
                     "bytes_per_update": bpu,
                     "updates_per_launch": upd0 / launches,
                     "avg_launch_us": 1e3 * kern_ms / launches,
                     "launches": launches, "kernel_ms": kern_ms},
    }
    if tst["round_launches"][1] > 0:
        l1, k1, u1 = tst["round_launches"][1], tst["round_kernel_ms"][1], tst["round_updates"][1]
        out["finish_round"] = {"state": "double, HBM" if tst["round_state"][1] & 2
                               else "double, LDS", "launches": l1, "kernel_ms": k1,
                               "updates": u1, "avg_launch_us": 1e3 * k1 / l1}
    # the same solve under each precision policy (time-to-eps, 5 solves each)
    variants = {}
    for name, prec in (("FP64", d.DICOD_PREC_FP64), ("FP32", d.DICOD_PREC_FP32),
                       ("MIXED", d.DICOD_PREC_MIXED)):
        with d.Context(update_cap=args.cap, colors=args.colors, precision=prec) as c:
            c.set_dictionary(D)
            c.solve_device(Xd, -w.lam_rel, w.eps, args.n_seg, Zd, stream)
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            for _ in range(5):
                _, st, _ = c.solve_device(Xd, -w.lam_rel, w.eps, args.n_seg, Zd, stream)
            torch.cuda.synchronize()
            variants[name] = {"time_to_eps_ms": 1e3 * (time.perf_counter() - t1) / 5,
                              "n_updates": st["n_updates"], "t_init_ms": st["t_init_ms"],
                              "round_updates": st["round_updates"][:3],
                              "objective": st["objective"]}
    out["precision_variants"] = variants
    # Algorithm 2 in lockstep (DICOD schedule) against the coloured schedule:
    # time-to-eps, and the interference rate from a traced solve
    sched = {"coloured": {"time_to_eps_ms": ms_per_step_of(stats, wall, args.steps),
                          "n_updates": s_last(stats)["n_updates"],
                          "n_phases": s_last(stats)["n_phases"]}}
    with d.Context(schedule=d.DICOD_SCHED_DICOD, update_cap=1) as c:
        c.set_dictionary(D)
        c.solve_device(Xd, -w.lam_rel, w.eps, args.n_seg, Zd, stream)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        for _ in range(5):
            _, st, _ = c.solve_device(Xd, -w.lam_rel, w.eps, args.n_seg, Zd, stream)
        torch.cuda.synchronize()
        t_dicod = 1e3 * (time.perf_counter() - t1) / 5
    with d.Context(schedule=d.DICOD_SCHED_DICOD, update_cap=1, trace_capacity=400_000) as c:
        c.set_dictionary(D)
        _, stt, _ = c.solve_device(Xd, -w.lam_rel, w.eps, args.n_seg, Zd, stream)
        torch.cuda.synchronize()
        tr = c.trace()
    first = tr[tr["phase"] < stt["round_phases"][0]]   # first (float) round
    n_adj, n_int = adjacent_pairs(first, W)
    Lm = (T - W + 1) / stt["n_seg"]
    sched["dicod_lockstep"] = {
        "time_to_eps_ms": t_dicod, "n_updates": st["n_updates"], "n_phases": st["n_phases"],
        "update_cap": 1, "n_seg": stt["n_seg"],
        "first_round": {"adjacent_concurrent_pairs": n_adj, "interfering_pairs": n_int,
                        "interference_rate": n_int / max(n_adj, 1),
                        "model_paper_(MW/T)^2": min(1.0, (W / Lm) ** 2),
                        "model_uniform_W^2/(2 L_M^2)": min(1.0, W * W / (2 * Lm * Lm))}}
    out["schedules"] = sched
    if not args.no_sweep:
        sweep = []
        with d.Context(update_cap=args.cap, colors=args.colors) as c:
            c.set_dictionary(D)
            for M in (8, 16, 32, 64, 128, 256, 374, 512, 749):
                try:
                    t1 = time.perf_counter()
                    _, st, _ = c.solve_device(Xd, -w.lam_rel, w.eps, M, Zd, stream)
                    torch.cuda.synchronize()
                    sweep.append({"n_seg": M, "time_to_eps_s": time.perf_counter() - t1,
                                  "n_updates": st["n_updates"], "n_phases": st["n_phases"]})
                except d.DicodError as e:
                    sweep.append({"n_seg": M, "error": str(e)[:120]})
        out["segment_sweep"] = sweep
    if long_data is not None:
        out["long"] = long_bench(d, torch, *long_data, args.cap, args.colors)
        print(f"[bench] long done", file=sys.stderr, flush=True)
    if batch_data is not None:
        out["batched"] = batched_bench(d, torch, *batch_data, args.cap, args.colors)
        print(f"[bench] batched done", file=sys.stderr, flush=True)
    if served_data is not None:
        out["served"] = served_bench(d, torch, *served_data, args.served_requests, args.cap,
                                     args.colors, args.seed)
        print(f"[bench] served done", file=sys.stderr, flush=True)
    if not args.no_cpu_baseline:
        lam = s0["lambda"]
        out["cpu_baseline"] = cpu_baseline(X, D, lam, w.eps, s0["n_seg"], effective_cap(args.cap, w.W),
                                           args.colors)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
