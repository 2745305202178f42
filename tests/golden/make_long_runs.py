"""Write the reference results of the long-run parity tests (oracle only).

Each case is one of the seeded workloads of workloads.py at a reduced grid
size, run by the CPU oracle (oracle/cdbm.py) for the full length of the
configuration it stands for; the final rho, u_x, u_y and T go to
tests/golden/long_runs.npz.  Nothing here calls the HIP path.

    python tests/golden/make_long_runs.py            # every case, in parallel
    python tests/golden/make_long_runs.py --only tg  # one case

Cases (name: workload, steps):
  headline_128_g1.2 / _g1.4 / _g1.667: the throughput workload (Lax tube
      extruded in y with the oblique density wave) on 128 x 128 cells of the
      same size, at each of its three specific-heat ratios, 2000 steps;
  ensemble_14, ensemble_34: grids 14 and 34 of the 96-grid ensemble (128 x 128,
      gamma 1.61 / 1.20, tau 5.2e-4 / 3.9e-5), each with its own gamma and
      tau, 1000 steps;
  tg_64: the Taylor-Green vortex on [0, 2 pi)^2 with 64 x 64 cells,
      10000 steps (t = 1).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time
from concurrent.futures import ProcessPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
OUT = os.path.join(HERE, "long_runs.npz")


def cases():
    sys.path.insert(0, ROOT)
    import workloads as W
    out = {}
    for g in W.HEADLINE_GAMMAS:
        out[f"headline_128_g{g:.4g}"] = W.lax_acoustic_2d(128, seed=0, steps=2000, gamma=g)
    ens = W.batched_ensemble()
    for k in (14, 34):
        out[f"ensemble_{k}"] = ens[k]
    out["tg_64"] = W.taylor_green_2pi(n=64)
    return out


def run_case(name):
    sys.path.insert(0, ROOT)
    import torch
    torch.set_num_threads(1)
    from oracle import cdbm as C
    run = cases()[name]
    t0 = time.time()
    p = C.Params.from_run(run)
    f = C.initial_distribution(run.rho, run.ux, run.uy, run.T, p)
    f = C.run(f, p, run.steps)
    fields = [a.numpy() for a in C.fields(f, p)]
    desc = {"name": run.name, "nx": run.nx, "ny": run.ny, "steps": run.steps,
            "gamma": run.gamma, "tau": run.tau, "dt": run.dt, "seconds": time.time() - t0}
    print(f"{name}: {run.steps} steps in {desc['seconds']:.0f} s", flush=True)
    return name, fields, desc


def main():
    import numpy as np
    ap = argparse.ArgumentParser()
    ap.add_argument("--only", default=None, help="substring of the case names to run")
    ap.add_argument("--jobs", type=int, default=6)
    args = ap.parse_args()
    names = [n for n in cases() if args.only is None or args.only in n]
    old = {}
    if os.path.exists(OUT):
        with np.load(OUT) as z:
            old = {k: z[k] for k in z.files}
    meta = json.loads(str(old.pop("meta"))) if "meta" in old else {}
    with ProcessPoolExecutor(max_workers=min(args.jobs, len(names))) as ex:
        for name, fields, desc in ex.map(run_case, names):
            for q, a in zip(("rho", "ux", "uy", "T"), fields):
                old[f"{name}.{q}"] = a
            meta[name] = desc
    np.savez_compressed(OUT, meta=np.array(json.dumps(meta, sort_keys=True)), **old)
    print(f"wrote {OUT}")


if __name__ == "__main__":
    main()
