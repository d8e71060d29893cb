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


def warm_start_measure():
    """Time to a steady hot-wall Nu (within 1e-3 of Nu_inf), cold start vs
    the learned warm start: a surrogate trained on 128 steady states of 32^2
    cavities predicts 16 held-out 64^2 cavities (up-sampled); both starts run
    one fixed horizon as a batch, Nu_inf is the cold start's final Nu.  The
    plain reference runs the cavities one at a time from a cold start."""
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
    cold = sg.run_to_steady(test, None, chunk=500, tol=1e-6, max_steps=1_000_000, drop=False)
    print(f"# warm start: cold runs {cold['seconds']:.1f} s", file=sys.stderr, flush=True)
    warm = sg.run_to_steady(test, ws, chunk=500, tol=1e-6, max_steps=1_000_000, drop=False)
    sc = sg.settle_steps(cold["times"], cold["nu_hist"], cold["nu"])
    sw = sg.settle_steps(warm["times"], warm["nu_hist"], cold["nu"])
    both = cold["converged"] & warm["converged"]
    per_step = cold["seconds"] / cold["times"][-1]
    # the plain way: one cavity at a time, FP32, cold start, each run until
    # its Nu has settled, at the measured step time of a single cavity
    from paper_1511_04552_amd import Cavity
    one = Cavity(**sg._cavity_kw(test[0]))
    one.step(200)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(one.stream)
    one.step(4000)
    e1.record(one.stream)
    torch.cuda.synchronize()
    single_step = e0.elapsed_time(e1) * 1e-3 / 4000
    del one
    plain = float(sc.sum() * single_step)
    warm_s = float(sw.max() * per_step + warm["t_load"])
    return {"workload": "16 held-out 64^2 cavities (Ra 1e3-1e6, phi0 0-0.05, d_p 10-100 nm) warm-started "
                        "from an FNO trained on 128 steady states of 32^2",
            "criterion": "steps until Nu stays within 1e-3 of Nu_inf", "horizon_steps": 1_000_000,
            "cold_settle_steps_sum": int(sc.sum()), "warm_settle_steps_sum": int(sw.sum()),
            "settle_ratio": round(float(sc.sum() / max(sw.sum(), 1)), 2),
            "settle_ratio_median": round(float(np.median(sc / np.maximum(sw, 1))), 2),
            "own_criterion_ratio": round(float(cold["steps"][both].sum() / max(warm["steps"][both].sum(), 1)), 2),
            "final_nu_rel_diff_max": float(np.max(np.abs(warm["nu"] - cold["nu"]) / np.abs(cold["nu"]))),
            "seconds_to_settle_cold": round(float(sc.max() * per_step), 3),
            "seconds_to_settle_warm": round(warm_s, 3),
            "seconds_to_settle_plain": round(plain, 3),
            "plain_over_warm_batched": round(plain / warm_s, 1),
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
    batched = None
    if a.batch > 0 and not a.no_secondary:
        batched = batch_measure(torch, mc, inputs, a.batch)
    warm = None
    if not a.no_warm_start and not a.no_secondary:
        warm = warm_start_measure()
    roof = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBPS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBPS, 4), "traffic": traffic,
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
        "batched_sweep": batched,
        "time_to_steady": warm,
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
