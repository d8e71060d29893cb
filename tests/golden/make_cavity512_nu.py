"""Write the FP64 oracle's long-horizon Nusselt numbers of the 512^2 workload.

The workload is the benchmarked cavity: 512 x 512, Ra 1e5, Pr 6.2, tau_f 0.8,
3 % alumina in water, d_p 50 nm, every slip force of Table 1 on, seeded
+-1e-6 phi perturbation.  The output is the average hot-wall Nusselt number
(Section 2.d, Fig 3a, with the second-order one-sided wall gradient) and its
cold-wall and conductivity-weighted companions, every ``--every`` steps up to
``--steps``, with the relative change of the mixture velocity and of theta
over the last 1000 steps before each record.

Only the oracle is called.  A run takes about 40 minutes on 8 host cores at
1e5 steps; ``--checkpoint`` lets an interrupted run resume.

    python tests/golden/make_cavity512_nu.py --steps 100000 --every 10000
"""
import argparse
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
from paper_1511_04552_amd import inputs  # noqa: E402

OUT = os.path.join(HERE, "cavity512_ra1e5_nu.txt")
WORKLOAD = "cavity512_ra1e5"


def main() -> int:
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--steps", type=int, default=100000)
    ap.add_argument("--every", type=int, default=10000)
    ap.add_argument("--out", default=OUT)
    ap.add_argument("--checkpoint", default=None,
                    help="oracle checkpoint file: resumed from if present, rewritten at every record")
    args = ap.parse_args()
    if args.every < 1000 or args.steps % args.every:
        ap.error("--every must be >= 1000 and divide --steps")

    w = inputs.WORKLOADS[WORKLOAD]
    cfg = {k: v for k, v in w.items() if k != "seed"}
    xi = inputs.phi_perturbation(w["seed"], cfg["nx"], cfg["ny"])
    o = oracle.Oracle(xi=xi, **cfg)
    rows = []
    if args.checkpoint and os.path.exists(args.checkpoint) and os.path.exists(args.out + ".partial"):
        o.restore(args.checkpoint)
        with open(args.out + ".partial") as f:
            rows = [ln for ln in f if not ln.startswith("#")]
        print(f"resumed at step {o.time} with {len(rows)} records", flush=True)

    t0 = time.time()
    while o.time < args.steps:
        nxt = (o.time // args.every + 1) * args.every
        o.step(nxt - 1000 - o.time)
        o.residual()                      # snapshot 1000 steps before the record
        o.step(1000)
        ru, rt = o.residual()
        nh, nc, nk = o.nusselt()
        rows.append(f"{o.time} {nh:.15e} {nc:.15e} {nk:.15e} {ru:.6e} {rt:.6e}\n")
        print(f"step {o.time}: Nu hot {nh:.10f} cold {nc:.10f} k {nk:.10f} "
              f"res u {ru:.3e} theta {rt:.3e}  ({time.time() - t0:.0f} s)", flush=True)
        if args.checkpoint:
            o.checkpoint(args.checkpoint)
            with open(args.out + ".partial", "w") as f:
                f.writelines(rows)

    header = [
        "# FP64 oracle, 512 x 512 cavity, Ra 1e5, Pr 6.2, tau_f 0.8, phi0 0.03 alumina/water,\n",
        "# d_p 50 nm, all six slip forces of Table 1 plus buoyancy, seed 2 for the +-1e-6 phi\n",
        "# perturbation (SplitMix64, row-major).  Average hot-wall Nusselt number of Section 2.d\n",
        "# (Fig 3a) from the second-order one-sided wall gradient, its cold-wall mirror and the\n",
        "# conductivity-weighted hot-wall value; res_u / res_theta are the L2-relative changes of\n",
        "# the mixture velocity (Eq 32) and of theta over the 1000 steps before the record.\n",
        "# Written by tests/golden/make_cavity512_nu.py (oracle only).\n",
        "# columns: step nu_hot nu_cold nu_hot_k res_u res_theta\n",
    ]
    with open(args.out, "w") as f:
        f.writelines(header + rows)
    if os.path.exists(args.out + ".partial"):
        os.remove(args.out + ".partial")
    print("wrote", args.out, flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
