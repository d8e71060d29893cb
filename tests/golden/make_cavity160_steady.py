"""Write the FP64 oracle's approach to steady state of the paper's own
lattice, the reference for the GPU's long-horizon parity there.

The workload is the paper's grid and case (Section 2.d, Fig 3a): 160 x 160,
Ra 1e6, Pr 8.923, 4 % alumina in water, d_p 33 nm, every slip force of
Table 1 on, tau_f chosen automatically (free-fall velocity at most 0.1 c_s;
with tau_f 0.8 the flow reorganises after ~4e5 steps), seeded +-1e-6 phi
perturbation.  The oracle runs
until the relative change of the mixture velocity and of theta over 1000
steps is below ``--tol`` (or for ``--max-steps``), recording the Nusselt
numbers (Section 2.d, Fig 3a) and that change every ``--every`` steps, and
then each moment's scale over the whole field and the nine moments (Eqs
29-32) at a 10 x 10 set of nodes (including the wall columns and rows).

Only the oracle is called.  ``--checkpoint`` lets an interrupted run resume.

    python tests/golden/make_cavity160_steady.py --checkpoint /tmp/c160.ckpt
"""
import argparse
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
from paper_1511_04552_amd import inputs  # noqa: E402

OUT = os.path.join(HERE, "cavity160_paper_steady.txt")
CFG = dict(nx=160, ny=160, Ra=1e6, Pr=8.923, phi0=0.04, dp_nm=33.0, tau_f=-1.0)
SEED = 6
SAMPLE = (0, 1, 10, 40, 79, 80, 120, 150, 158, 159)
FIELDS = oracle.FIELDS[:9]


def main() -> int:
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--tol", type=float, default=1e-8)
    ap.add_argument("--max-steps", type=int, default=1500000)
    ap.add_argument("--every", type=int, default=100000)
    ap.add_argument("--out", default=OUT)
    ap.add_argument("--checkpoint", default=None)
    ap.add_argument("--rewrite", action="store_true",
                    help="rewrite --out from --checkpoint (the state of its last record) and the records "
                         "already in --out, without stepping")
    args = ap.parse_args()
    if args.every < 1000 or args.max_steps % args.every:
        ap.error("--every must be >= 1000 and divide --max-steps")

    xi = inputs.phi_perturbation(SEED, CFG["nx"], CFG["ny"])
    o = oracle.Oracle(xi=xi, **CFG)
    rows = []
    part = args.out + ".partial"
    if args.checkpoint and os.path.exists(args.checkpoint) and os.path.exists(part):
        o.restore(args.checkpoint)
        with open(part) as f:
            rows = [ln for ln in f if not ln.startswith("#")]
        print(f"resumed at step {o.time} with {len(rows)} records", flush=True)

    if args.rewrite:
        o.restore(args.checkpoint)
        with open(args.out) as f:
            rows = []
            for ln in f:
                if ln.startswith("# moments") or ln.startswith("# scales"):
                    break
                if not ln.startswith("#"):
                    rows.append(ln)
        if int(rows[-1].split()[0]) != o.time:
            ap.error("the checkpoint is not at the last record")
        args.max_steps = o.time
    t0 = time.time()
    ru = rt = float("inf")
    if rows:
        ru, rt = (float(v) for v in rows[-1].split()[4:6])
    while o.time < args.max_steps and max(ru, rt) >= args.tol:
        nxt = (o.time // args.every + 1) * args.every
        o.step(nxt - 1000 - o.time)
        o.residual()
        o.step(1000)
        ru, rt = o.residual()
        nh, nc, nk = o.nusselt()
        rows.append(f"{o.time} {nh:.15e} {nc:.15e} {nk:.15e} {ru:.6e} {rt:.6e}\n")
        print(f"step {o.time}: Nu hot {nh:.10f} res u {ru:.3e} theta {rt:.3e} ({time.time() - t0:.0f} s)",
              flush=True)
        if args.checkpoint:
            o.checkpoint(args.checkpoint)
            with open(part, "w") as f:
                f.writelines(rows)

    m = o.moments(FIELDS)
    d = o.derived()
    lines = [
        "# FP64 oracle, 160 x 160 cavity (the paper's lattice), Ra 1e6, Pr 8.923, phi0 0.04 alumina/water,\n",
        "# d_p 33 nm, all six slip forces of Table 1 plus buoyancy, tau_f automatic (%.17g), seed 6 for the\n" % d["tau_f"],
        "# +-1e-6 phi\n",
        "# perturbation.  Records: step, hot-wall Nusselt number (Section 2.d, Fig 3a), cold-wall and\n",
        "# conductivity-weighted values, L2-relative change of u_ns and theta over the 1000 steps before.\n",
        "# Then, for the state of the last record, each moment's mean, largest deviation from the mean\n",
        "# and largest magnitude over the whole field, and the nine moments (Eqs 29-32) at nodes x, y\n",
        "# in %s.\n" % (SAMPLE,),
        "# Written by tests/golden/make_cavity160_steady.py (oracle only).\n",
        "# columns: step nu_hot nu_cold nu_hot_k res_u res_theta\n",
    ]
    lines += rows
    lines.append("# scales: field mean max_abs_deviation max_abs\n")
    for name in FIELDS:
        v = m[name]
        lines.append(f"scale {name} {v.mean():.17e} {np.abs(v - v.mean()).max():.17e} {np.abs(v).max():.17e}\n")
    lines.append("# moments: field x y value\n")
    for name in FIELDS:
        for y in SAMPLE:
            for x in SAMPLE:
                lines.append(f"{name} {x} {y} {m[name][y, x]:.17e}\n")
    with open(args.out, "w") as f:
        f.writelines(lines)
    if os.path.exists(part):
        os.remove(part)
    print("wrote", args.out, "at step", o.time, flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
