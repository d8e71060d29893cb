"""Benchmark of the fused three-lattice MCLBM step on one MI355X.

One "step" is one pass of the whole hot path over the cavity: streaming with
the walls, moments, properties, lagged gradients, six slip forces plus
buoyancy, BGK collision of the fluid, particle and temperature lattices
(one fused kernel launch).  Prints one JSON line.

  python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload NAME]
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

HBM_PEAK_GBPS = 8000.0          # MI355X HBM3E
LLC_BYTES = 256 << 20           # MI355X last-level cache (MALL)
BYTES_PER_LUP_FP32 = 232        # 27 populations read + written (4 B), lag field read + written (8 B)
BYTES_PER_LUP_16 = 124          # the same with 2-byte populations
STORAGE = {"fp32": (0, BYTES_PER_LUP_FP32, "fp32"), "fp16": (1, BYTES_PER_LUP_16, "fp16 (scaled)"),
           "bf16": (2, BYTES_PER_LUP_16, "bf16")}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50000)
    ap.add_argument("--warmup", type=int, default=2000)
    ap.add_argument("--workload", default="cavity512_ra1e5")
    ap.add_argument("--cpu-seconds", type=float, default=15.0,
                    help="approximate CPU time budget of the oracle baseline sample")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--traffic", default=os.path.join(ROOT, "profiles", "traffic.json"),
                    help="HBM bytes per launch measured by rocprofv3 counters")
    ap.add_argument("--batch", type=int, default=256,
                    help="cavities in the batched-sweep measurement (0 skips it)")
    ap.add_argument("--no-warm-start", action="store_true",
                    help="skip the time-to-steady comparison of cold and learned warm starts")
    ap.add_argument("--no-secondary", action="store_true",
                    help="skip the 2048^2 (larger than the last-level cache) measurement")
    ap.add_argument("--storage", choices=("fp32", "fp16", "bf16"), default="fp32",
                    help="population storage of the timed workload")
    ap.add_argument("--steps-per-launch", type=int, choices=(0, 1, 2), default=0,
                    help="1: one step per launch (k_step); 2: an even and an odd step per "
                         "launch (k_step2); 0: the library's choice for the workload")
    ap.add_argument("--gemm-only", action="store_true",
                    help="time only the warm-start network's BF16 GEMM at 4096^3 and print its line")
    ap.add_argument("--small-batches-only", action="store_true",
                    help="time only the batches of many small cavities (tiles against one workgroup per "
                         "cavity) and print their line")
    ap.add_argument("--copy-only", action="store_true",
                    help="time plain device copies (this library's streaming copy kernel and torch's "
                         "copy_) of 16, 30.4 (the bytes each way of one 512^2 step), 61 and 1024 MB "
                         "and print their line")
    ap.add_argument("--pmc-summary", nargs=2, metavar=("FETCH_DIR", "WRITE_DIR"),
                    help="summarise two rocprofv3 --pmc runs (FETCH_SIZE, WRITE_SIZE) of this "
                         "bench into the traffic file and exit")
    return ap.parse_args()


def copy_bandwidth(torch, mc, nbytes=1 << 30, reps=20):
    src = torch.empty(nbytes // 4, dtype=torch.float32, device="cuda").fill_(1.0)
    dst = torch.empty_like(src)
    s = torch.cuda.current_stream()
    for _ in range(3):
        mc.copy_kernel(dst, src, s)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(s)
    for _ in range(reps):
        mc.copy_kernel(dst, src, s)
    e1.record(s)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    del src, dst
    return 2.0 * nbytes / (ms * 1e-3) / 1e9


def time_steps(torch, cav, n):
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(cav.stream)
    cav.step(n)
    e1.record(cav.stream)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / n


def _counter_rows(d):
    import csv
    import glob
    rows = []
    for f in glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True):
        rows += list(csv.DictReader(open(f)))
    return rows


def pmc_summary(fetch_dir, write_dir, workload, out_path, storage="fp32"):
    """Bytes per launch of the step kernels from FETCH_SIZE / WRITE_SIZE
    (KiB per dispatch), each scaled by what the same counter reads for the
    1 GiB copy kernel this bench runs (known to move 1 GiB each way)."""
    res = {}
    for name, d in (("FETCH_SIZE", fetch_dir), ("WRITE_SIZE", write_dir)):
        per = {}
        for r in _counter_rows(d):
            if r["Counter_Name"] != name:
                continue
            k = r["Kernel_Name"]
            key = "copy" if k.startswith("k_copy") else ("step_even" if "k_step<false" in k else
                                                         "step_odd" if "k_step<true" in k else
                                                         "step_pair" if "k_step2<" in k else None)
            if key:
                per.setdefault(key, []).append(float(r["Counter_Value"]))
        scale = (1 << 20) / (sum(per["copy"]) / len(per["copy"]))  # KiB of 1 GiB / counted
        res[name] = {"scale": scale, **{k: sum(v) / len(v) * 1024 * scale for k, v in per.items() if k != "copy"}}
    # the kernels the run launched: pairs of steps (k_step2) or single steps
    spl = 2 if "step_pair" in res["FETCH_SIZE"] else 1
    kinds = ("step_pair",) if spl == 2 else ("step_even", "step_odd")
    per_launch = {k: res["FETCH_SIZE"][k] + res["WRITE_SIZE"][k] for k in kinds}
    out = {"workload": workload, "storage": storage, "steps_per_launch": spl, "kernel_hash": kernel_hash(),
           "bytes_per_launch": sum(per_launch.values()) / len(kinds),
           "fetch_bytes": {k: res["FETCH_SIZE"][k] for k in kinds},
           "write_bytes": {k: res["WRITE_SIZE"][k] for k in kinds},
           "fetch_scale": res["FETCH_SIZE"]["scale"], "write_scale": res["WRITE_SIZE"]["scale"]}
    json.dump(out, open(out_path, "w"), indent=1)
    print(json.dumps(out, indent=1))


def copy_measure(torch, mc):
    """Microseconds and GB/s (bytes read plus written) of plain device copies
    of several sizes: the library's streaming copy kernel and torch's copy_.
    30.4 MB each way is what one 512^2 FP32 step reads and writes, so these
    copies are the rate a step of that size could reach if it did nothing
    but move its bytes."""
    s = torch.cuda.current_stream()
    out = []
    for mb in (16.0, 30.4, 61.0, 1024.0):
        n = int(mb * (1 << 20)) // 16 * 4
        src = torch.empty(n, dtype=torch.float32, device="cuda").fill_(1.0)
        dst = torch.empty_like(src)
        reps = 2000 if mb < 100 else 100
        row = {"mb_each_way": mb}
        for name, fn in (("copy_kernel", lambda: mc.copy_kernel(dst, src, s)), ("torch_copy", lambda: dst.copy_(src))):
            for _ in range(20):
                fn()
            torch.cuda.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(s)
            for _ in range(reps):
                fn()
            e1.record(s)
            torch.cuda.synchronize()
            us = e0.elapsed_time(e1) * 1e3 / reps
            row[name] = {"us": round(us, 2), "GBps": round(2 * n * 4 / us / 1e3, 1)}
        out.append(row)
        del src, dst
        torch.cuda.empty_cache()
    return out


def batch_measure(torch, mc, inputs, n, steps=64):
    """Uneven-cavity parameter sweep: n cavities with sides from
    {64, 128, 256, 384, 512}, Ra log-uniform in [1e3, 1e6], phi in [0, 5 %],
    d_p in [10, 100] nm (automatic tau_f), two steps per launch for every
    cavity with band heights from the autotuner, replayed from a captured
    graph; beside it the same sweep with one step per launch (tile shapes
    from the autotuner)."""
    def run(spl):
        cfgs = inputs.sweep_parameters(3, n)
        for c in cfgs:
            c["tau_f"] = -1.0
            c["steps_per_launch"] = spl
        xis = [inputs.phi_perturbation(c["seed"], c["nx"], c["ny"]) for c in cfgs]
        b = mc.Batch(cfgs, xis=xis)
        shapes = b.autotune(steps=8)
        nodes = sum(c["nx"] * c["ny"] for c in cfgs)
        b.step(32)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record(b.stream)
        b.step(steps)
        e1.record(b.stream)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / steps
        gbs = BYTES_PER_LUP_FP32 / spl * nodes / (ms * 1e-3) / 1e9
        out = {"workload": f"sweep of {n} uneven cavities (seed 3)", "nodes": nodes, "steps": steps,
               "steps_per_launch": spl, "ms_per_step": round(ms, 5),
               "MLUPS": round(nodes / (ms * 1e-3) / 1e6, 1), "achieved_GBps": round(gbs, 1),
               "frac": round(gbs / HBM_PEAK_GBPS, 4),
               "tile_shapes": sorted({f"{c['nx']}: {bx}x{by}" for c, (bx, by) in zip(cfgs, shapes)})}
        b.close()
        del b
        torch.cuda.empty_cache()
        return out

    out = run(2)
    out["one_step_per_launch"] = run(1)
    return out


def small_batch_measure(torch, mc, inputs, steps=512):
    """Batches of many small cavities (Ra log-uniform in [1e3, 1e5], phi in
    [0, 5 %], d_p in [20, 100] nm, automatic tau_f): microseconds per step of
    the whole batch over the tiles (one launch per step, replayed from a
    captured graph) and with one workgroup per cavity (up to 256 steps per
    launch), and the schedule the library picks by default."""
    import numpy as np
    out = []
    for n, side in ((16, 64), (128, 32), (256, 32), (256, 64)):
        rng = np.random.default_rng(17)
        cfgs = [dict(nx=side, ny=side, Ra=float(10 ** rng.uniform(3, 5)), phi0=float(rng.uniform(0, 0.05)),
                     dp_nm=float(rng.uniform(20, 100)), tau_f=-1.0) for _ in range(n)]
        xis = [inputs.phi_perturbation(40 + k, side, side) for k in range(n)]
        b = mc.Batch(cfgs, xis=xis)
        row = {"workload": f"{n} x {side}^2", "default": "per_cavity" if b.per_cavity else "tiles"}
        for name, on in (("tiles_us_per_step", False), ("per_cavity_us_per_step", True)):
            b.per_cavity = on
            b.step(64)
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            torch.cuda.synchronize()
            e0.record(b.stream)
            b.step(steps)
            e1.record(b.stream)
            torch.cuda.synchronize()
            row[name] = round(e0.elapsed_time(e1) * 1e3 / steps, 2)
        out.append(row)
        b.close()
        del b
        torch.cuda.empty_cache()
    return out


def gemm_measure(torch, mc, n=4096, reps=20):
    """The warm-start network's GEMM (mclbm_nn_gemm: FP32 operands rounded to
    BF16, MFMA with FP32 accumulation) on an n^3 product, B as K x N and as
    N x K, against the dense BF16 peak of 2.5 PFLOP/s; torch's BF16 matmul
    (hipBLASLt, BF16 operands) on the same shape for context."""
    import ctypes
    g = torch.Generator(device="cuda").manual_seed(0)
    A = torch.randn(n, n, device="cuda", generator=g)
    B = torch.randn(n, n, device="cuda", generator=g)
    C = torch.empty(n, n, device="cuda")
    s = torch.cuda.current_stream()
    out = {"shape": f"{n}^3", "peak_tflops": 2500.0}
    for tb, name in ((0, "b_k_by_n"), (1, "b_n_by_k")):
        def run():
            rc = mc.lib().mclbm_nn_gemm(0, tb, n, n, n, 1.0, ctypes.c_void_p(A.data_ptr()), n, 0, 0,
                                        ctypes.c_void_p(B.data_ptr()), n, 0, 0, 0.0,
                                        ctypes.c_void_p(C.data_ptr()), n, 0, 0, 1, 1,
                                        ctypes.c_void_p(s.cuda_stream))
            if rc != 0:
                raise RuntimeError(mc.lib().mclbm_last_error())
        run()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(s)
        for _ in range(reps):
            run()
        e1.record(s)
        torch.cuda.synchronize()
        us = e0.elapsed_time(e1) / reps * 1e3
        tf = 2.0 * n ** 3 / (us * 1e-6) / 1e12
        out[name] = {"us": round(us, 1), "tflops": round(tf, 1), "frac": round(tf / 2500.0, 4)}
    Ab, Bb = A.bfloat16(), B.bfloat16()
    for _ in range(3):
        torch.matmul(Ab, Bb)
    torch.cuda.synchronize()
    e0.record(s)
    for _ in range(reps):
        torch.matmul(Ab, Bb)
    e1.record(s)
    torch.cuda.synchronize()
    out["torch_bf16_matmul_tflops"] = round(2.0 * n ** 3 / (e0.elapsed_time(e1) / reps * 1e-3) / 1e12, 1)
    return out


def warm_start_measure():
    """Time to a steady hot-wall Nu on 16 held-out 64^2 cavities, four ways:
    plain (each cavity alone, one after another, FP32, cold start), batched
    cold, batched warm (a surrogate trained on 128 steady states of 32^2
    cavities predicts the fields, up-sampled and loaded), and batched warm
    with the transient in FP16 storage, finished in FP32.  Every run stops
    where the solver's own criterion is met (change of u and theta over 500
    steps below 1e-6; batched cavities drop out there).  Nu_inf is the final
    Nu of a cold batch run for 1e6 steps without drop-out; a run has settled
    from the first record after which its Nu stays within 1e-3 of Nu_inf.
    Wall times are measured: to the settled record of every cavity (plain:
    summed, since the cavities run one after another; batched: the last one)
    and to the criterion of every cavity."""
    import numpy as np
    import torch
    from paper_1511_04552_amd import inputs, surrogate as sg

    def cases(seed, n, side):
        return [dict(c, tau_f=-1.0) for c in inputs.sweep_parameters(seed, n, sides=(side,))]

    t0 = time.perf_counter()
    train = cases(9001, 128, 32)
    F, _, ok = sg.generate_dataset(train, chunk=2000, tol=1e-6, max_steps=800_000)
    torch.cuda.synchronize()
    t_data = time.perf_counter() - t0
    print(f"# warm start: {int(ok.sum())} training states in {t_data:.1f} s", file=sys.stderr, flush=True)
    ws = sg.WarmStart(S=32, C=32, m=8, L=4, Q=64, B=16, seed=0)
    t0 = time.perf_counter()
    ws.fit([c for c, o in zip(train, ok) if o], F[ok], epochs=150, lr=3e-3, weights=(1, 1, 4, 1, 1))
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t0
    test = cases(9002, 16, 64)
    ref = sg.run_to_steady(test, None, chunk=500, tol=1e-6, max_steps=1_000_000, drop=False)
    nu_inf = ref["nu"]
    print(f"# warm start: reference runs {ref['seconds']:.1f} s", file=sys.stderr, flush=True)
    cold = sg.run_to_steady(test, None, chunk=500, tol=1e-6, max_steps=1_000_000, drop=True)
    warm = sg.run_to_steady(test, ws, chunk=500, tol=1e-6, max_steps=1_000_000, drop=True)
    # the reduced-precision leg: FP16 storage for the transient, each cavity
    # moved to FP32 (mclbm_copy_state) once its change over 500 steps is
    # below 1e-3 (FP16 storage levels off at ~6e-4, its Nu ~3e-3 from Nu_inf)
    mixed = sg.run_mixed(test, ws, storage=1, switch_tol=1e-3, chunk=500, tol=1e-6, max_steps=1_000_000)
    plain = sg.run_plain(test, chunk=500, tol=1e-6, max_steps=1_000_000)
    print(f"# warm start: plain runs {sum(p['seconds'] for p in plain):.1f} s", file=sys.stderr, flush=True)

    def batched(run):
        st = sg.settle_steps(run["times"], run["nu_hist"], nu_inf)
        at = {int(t): w for t, w in zip(run["times"], run["walls"])}
        settle = max(at[int(s)] for s in st) + run["t_load"]
        own = run["seconds"] + run["t_load"]
        return st, settle, own

    sc, cold_settle, cold_own = batched(cold)
    sw, warm_settle, warm_own = batched(warm)
    sm, mixed_settle, mixed_own = batched(mixed)
    plain_settle, plain_own, sp = 0.0, 0.0, []
    for k, p in enumerate(plain):
        rec = p["records"]
        s_k = sg.settle_steps(rec[:, 0], rec[:, 2:3], nu_inf[k:k + 1])[0]
        sp.append(s_k)
        plain_settle += float(rec[rec[:, 0] == s_k, 1][0])
        plain_own += p["seconds"]
    sp = np.array(sp)
    final = lambda run: np.abs(run["nu"] - nu_inf) / np.abs(nu_inf)
    return {"workload": "16 held-out 64^2 cavities (Ra 1e3-1e6, phi0 0-0.05, d_p 10-100 nm) warm-started "
                        "from an FNO trained on 128 steady states of 32^2",
            "criterion": "wall time until the hot-wall Nu stays within 1e-3 of Nu_inf (settle), and until "
                         "the solver's own criterion (change of u, theta over 500 steps < 1e-6)",
            "nu_inf": "final Nu of a cold batched FP32 run of 1e6 steps without drop-out",
            "settle_steps_sum": {"plain": int(sp.sum()), "cold": int(sc.sum()), "warm": int(sw.sum())},
            "settle_ratio": round(float(sc.sum() / max(sw.sum(), 1)), 2),
            "settle_ratio_median": round(float(np.median(sc / np.maximum(sw, 1))), 2),
            "own_criterion_steps_sum": {"plain": int(sum(p["steps"] for p in plain)),
                                        "cold": int(cold["steps"].sum()), "warm": int(warm["steps"].sum())},
            "own_criterion_met": {"plain": int(sum(p["steps"] > 0 for p in plain)),
                                  "cold": int(cold["converged"].sum()), "warm": int(warm["converged"].sum())},
            "final_nu_rel_err_max": {"plain": float(max(abs(p["records"][-1, 2] - nu_inf[k]) / abs(nu_inf[k])
                                                        for k, p in enumerate(plain))),
                                     "cold": float(final(cold).max()), "warm": float(final(warm).max())},
            "seconds_to_settle": {"plain": round(plain_settle, 3), "cold_batched": round(cold_settle, 3),
                                  "warm_batched": round(warm_settle, 3),
                                  "warm_batched_fp16_transient": round(mixed_settle, 3)},
            "seconds_to_own_criterion": {"plain": round(plain_own, 3), "cold_batched": round(cold_own, 3),
                                         "warm_batched": round(warm_own, 3),
                                         "warm_batched_fp16_transient": round(mixed_own, 3)},
            "fp16_transient": {"switch_tol": 1e-3, "switched": int((mixed["switched"] > 0).sum()),
                               "own_criterion_met": int(mixed["converged"].sum()),
                               "final_nu_rel_err_max": float(final(mixed).max()),
                               "settle_steps_sum": int(sm.sum())},
            "plain_over_warm_batched": round(plain_settle / warm_settle, 1),
            "plain_over_warm_batched_own_criterion": round(plain_own / warm_own, 1),
            "gain_from_batching": round(plain_settle / cold_settle, 2),
            "gain_from_warm_start": round(cold_settle / warm_settle, 2),
            "gain_from_warm_start_own_criterion": round(cold_own / warm_own, 2),
            "seconds_load": round(warm["t_load"], 3),
            "seconds_training_data": round(t_data, 1), "seconds_training": round(t_train, 1)}


def cpu_baseline(w, xi, seconds):
    """The FP64 oracle as it stands, on this host's cores, on a bounded
    sample of the same workload (same cavity, first steps)."""
    import oracle
    cfg = {k: v for k, v in w.items() if k != "seed"}
    o = oracle.Oracle(xi=xi, **cfg)
    nodes = cfg["nx"] * cfg["ny"]
    o.step(2)
    t0 = time.perf_counter()
    o.step(5)
    per_step = (time.perf_counter() - t0) / 5
    steps = max(2, min(int(seconds / max(per_step, 1e-9)), 100000))
    t0 = time.perf_counter()
    o.step(steps)
    dt = time.perf_counter() - t0
    return {"value": nodes * steps / dt / 1e6, "unit": "MLUPS", "cores": oracle.max_threads(),
            "kind": "oracle",
            "sample": f"{cfg['nx']}x{cfg['ny']} cavity, {steps} steps after 7 warm-up steps, FP64, "
                      f"{dt:.1f} s"}


def main():
    a = parse()
    if a.pmc_summary:
        pmc_summary(a.pmc_summary[0], a.pmc_summary[1], a.workload, a.traffic, a.storage)
        return
    if a.gpus != 1:
        print(f"bench.py runs on exactly one GPU (asked for {a.gpus}); the multi-GPU "
              "decomposition is a design only in this build.", file=sys.stderr)
        sys.exit(2)
    import torch
    import paper_1511_04552_amd as mc
    from paper_1511_04552_amd import inputs

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    if a.gemm_only:
        print(json.dumps({"gemm_bf16": gemm_measure(torch, mc)}), flush=True)
        return
    if a.copy_only:
        print(json.dumps({"copies": copy_measure(torch, mc)}), flush=True)
        return
    if a.small_batches_only:
        from paper_1511_04552_amd import inputs
        print(json.dumps({"small_batches": small_batch_measure(torch, mc, inputs)}), flush=True)
        return
    w = inputs.WORKLOADS[a.workload]
    cfg = {k: v for k, v in w.items() if k != "seed"}
    nx, ny = cfg["nx"], cfg["ny"]
    xi = inputs.phi_perturbation(w["seed"], nx, ny)
    print(f"# workload {a.workload}: {nx}x{ny}, warmup {a.warmup}, steps {a.steps}", file=sys.stderr, flush=True)
    st_code, bytes_lup, st_name = STORAGE[a.storage]
    spl = a.steps_per_launch
    if spl == 0:
        two = (mc.device_bytes(storage=st_code, **cfg) >
               mc.device_bytes(storage=st_code, steps_per_launch=1, **cfg))
        spl = 2 if two else 1
    if spl == 2 and (a.steps % 2 or a.warmup % 2):
        print("with two steps per launch, --steps and --warmup must be even", file=sys.stderr)
        sys.exit(2)
    cav = mc.Cavity(xi=xi, storage=st_code, steps_per_launch=spl, **cfg)
    nbytes_dev = cav.nbytes
    stream = cav.stream
    cav.step(a.warmup)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    e0.record(stream)
    cav.step(a.steps)
    e1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms_total = e0.elapsed_time(e1)
    ms_step = ms_total / a.steps
    nodes = nx * ny
    mlups = nodes * a.steps / (ms_total * 1e-3) / 1e6
    nu_hot, nu_cold, _ = cav.nusselt()
    print(f"# timed {a.steps} steps: {ms_total:.2f} ms (wall {wall*1e3:.1f} ms), Nu hot {nu_hot:.5f}",
          file=sys.stderr, flush=True)
    # the two reductions, per synchronous call (launch, FP64 reduction, copy of
    # the result to the host), outside the timed steps
    red = {}
    for name, fn in (("nusselt", cav.nusselt), ("residual", cav.residual)):
        fn()
        t0 = time.perf_counter()
        for _ in range(200):
            fn()
        red[name + "_call_us"] = round((time.perf_counter() - t0) / 200 * 1e6, 1)

    # one launch moves the algorithmic bytes once: one step (k_step) or two
    # steps (k_step2, which reads and writes the populations once per pair)
    bytes_launch = bytes_lup * nodes
    achieved = bytes_launch / (spl * ms_step * 1e-3) / 1e9
    traffic = None
    if os.path.exists(a.traffic):
        try:
            t = json.load(open(a.traffic))
            if (t.get("workload") == a.workload and t.get("kernel_hash") == kernel_hash()
                    and t.get("storage", "fp32") == a.storage and t.get("steps_per_launch", 1) == spl):
                traffic = t.get("bytes_per_launch")
        except Exception:
            traffic = None
    copy_gbps = copy_bandwidth(torch, mc)
    secondary = None
    streaming = None
    above_2gib = None
    if not a.no_secondary:
        del cav
        torch.cuda.empty_cache()

        def measure(name, steps, steps_per_launch=0):
            w2 = inputs.WORKLOADS[name]
            cfg2 = {k: v for k, v in w2.items() if k != "seed"}
            if steps_per_launch == 0:  # the library's choice for this cavity
                two = mc.device_bytes(**cfg2) > mc.device_bytes(steps_per_launch=1, **cfg2)
                steps_per_launch = 2 if two else 1
            cav2 = mc.Cavity(xi=inputs.phi_perturbation(w2["seed"], cfg2["nx"], cfg2["ny"]),
                             steps_per_launch=steps_per_launch, **cfg2)
            cav2.step(20)
            ms2 = time_steps(torch, cav2, steps)
            n2 = cfg2["nx"] * cfg2["ny"]
            # two steps per launch read and write the populations once per
            # two steps: half the algorithmic bytes per lattice update
            bpl = BYTES_PER_LUP_FP32 / steps_per_launch
            gbs2 = bpl * n2 / (ms2 * 1e-3) / 1e9
            del cav2
            torch.cuda.empty_cache()
            return {"workload": name, "nx": cfg2["nx"], "ny": cfg2["ny"], "steps": steps,
                    "steps_per_launch": steps_per_launch, "bytes_per_lup": bpl,
                    "ms_per_step": round(ms2, 5), "MLUPS": round(n2 / (ms2 * 1e-3) / 1e6, 1),
                    "achieved_GBps": round(gbs2, 1), "frac": round(gbs2 / HBM_PEAK_GBPS, 4),
                    "frac_of_copy": round(gbs2 / copy_gbps, 4)}

        # the default schedule of these sizes is two steps per launch
        # (k_step2); one step per launch (k_step) is timed beside it
        secondary = measure("cavity2048_ra1e6", 200)   # 450 MB: partly served by the 256 MB cache
        secondary["one_step_per_launch"] = measure("cavity2048_ra1e6", 200, steps_per_launch=1)
        streaming = measure("cavity4096_ra1e6", 50)    # 1.8 GB: streams from HBM
        streaming["one_step_per_launch"] = measure("cavity4096_ra1e6", 50, steps_per_launch=1)
        # 2.29 GB of populations: 64-bit element offsets in both schedules
        above_2gib = measure("cavity4608_ra1e6", 40)
        above_2gib["one_step_per_launch"] = measure("cavity4608_ra1e6", 40, steps_per_launch=1)
    batched = None
    if a.batch > 0 and not a.no_secondary:
        batched = batch_measure(torch, mc, inputs, a.batch)
    warm = None
    if not a.no_warm_start and not a.no_secondary:
        warm = warm_start_measure()
    small = None if a.no_secondary else small_batch_measure(torch, mc, inputs)
    gemm = None if a.no_secondary else gemm_measure(torch, mc)
    # a working set inside the 256 MB last-level cache (MALL) is served from
    # it, not from HBM: the fraction is then an effective rate, and the
    # HBM-bound figure is the hbm_streaming line
    resident = nbytes_dev <= LLC_BYTES
    roof = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBPS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBPS, 4), "traffic": traffic,
            "cache_resident": resident, "working_set_bytes": nbytes_dev,
            "note": ("working set fits the 256 MB last-level cache: effective bandwidth, not HBM; "
                     "see hbm_streaming for the HBM-bound rate") if resident else "streams from HBM",
            "kernel": ("k_step (even and odd A-A parities)" if spl == 1 else
                       "k_step2 (an even and an odd step per launch)"),
            "algorithmic_bytes_per_launch": bytes_launch, "copy_kernel_gbps": round(copy_gbps, 1)}
    out = {
        "metric": "MLUPS (3 lattices)", "value": round(mlups, 1), "unit": "MLUPS",
        "n_gpus": 1, "steps": a.steps, "warmup": a.warmup, "ms_per_step": round(ms_step, 6),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic (seeded uniform suspension at rest, +-1e-6 phi perturbation)",
        "config": {"workload": a.workload, "nx": nx, "ny": ny, "Ra": cfg["Ra"], "Pr": cfg["Pr"],
                   "phi0": cfg["phi0"], "dp_nm": cfg["dp_nm"], "tau_f": cfg["tau_f"],
                   "forces": "drag+brownian+thermophoresis+saffman+magnus/rotation+gravity+buoyancy",
                   "storage": f"{st_name} shifted SoA, " + ("A-A in place" if spl == 1 else
                                                             "two copies, two steps per launch"),
                   "parallelism": "single GPU"},
        "roofline": roof,
        "nu_hot": nu_hot,
        "reductions": red,
        "larger_than_llc": secondary,
        "hbm_streaming": streaming,
        "above_2gib": above_2gib,
        "batched_sweep": batched,
        "small_batches": small,
        "time_to_steady": warm,
        "gemm_bf16": gemm,
    }
    if not a.no_cpu_baseline:
        print("# cpu baseline (FP64 oracle) ...", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(w, xi, a.cpu_seconds)
    print(json.dumps(out), flush=True)


def code_text(text: str) -> bytes:
    """Source text without line comments and blank lines."""
    import re
    lines = (re.sub(r"//.*", "", ln).rstrip() for ln in text.splitlines())
    return "\n".join(ln for ln in lines if ln).encode()


def kernel_hash() -> str:
    """Hash of the step kernels' device code (the device header and the text
    from step_node to k_step2), which the measured traffic belongs to; line
    comments and blank lines are left out, so a change of wording keeps the
    measurement."""
    import hashlib
    code = code_text
    h = hashlib.sha256()
    h.update(code(open(os.path.join(ROOT, "paper_1511_04552_amd/csrc/lbm_device.h")).read()))
    src = open(os.path.join(ROOT, "paper_1511_04552_amd/csrc/mclbm.hip")).read()
    a = src.index("// One node of one time step")
    b = src.index("// Batched sweep:")
    h.update(code(src[a:b]))
    return h.hexdigest()[:16]


if __name__ == "__main__":
    main()
