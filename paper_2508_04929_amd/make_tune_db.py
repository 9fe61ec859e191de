"""Regenerate the tuning database (tune_mi355x.txt) on the GPU: run the
library's autotuner (cs_autotune) on the benchmark workloads and record its
choices, one line per problem signature.

    python -m paper_2508_04929_amd.make_tune_db [output path]

Runs on one MI355X; the autotuner times each candidate (tile, halo,
budget) on the real problem, reps timed calls each.
"""
from __future__ import annotations

import os
import sys


def main(out: str, reps: int = 3) -> None:
    if os.path.exists(out):
        os.remove(out)
    os.environ["CS_AUTOTUNE_CACHE"] = out   # fresh database, written by the library
    import numpy as np
    import torch

    from . import binding, inputs

    lib = binding.library()
    dev = torch.device("cuda", 0)
    t = lambda x: torch.from_numpy(np.ascontiguousarray(x, dtype=np.float32)).to(dev)

    def problem(g, v, loss_only=False):
        ctf = binding.Ctf(t(v.defocus_u), t(v.defocus_v), t(v.astig), t(v.phase), v.voltage_kv,
                          v.cs_mm, v.amp_contrast, v.bfactor)
        Y = torch.zeros(v.b, v.D, v.D, device=dev)   # the observed values do not change the work
        return lib.make_problem(t(g.means), t(g.log_scales), t(g.quats), t(g.amps), t(v.rot),
                                t(v.shift), v.D, v.pixel, Y, ctf=ctf, reduction="mean",
                                want_grads=not loss_only)

    g, v, _gt, _rn = inputs.c4()
    probs = [problem(g, v)]
    g, v, _gt, _rn = inputs.c2()
    probs.append(problem(g, v))
    g, v, _gt = inputs.c1()
    probs.append(problem(g, v, loss_only=True))
    for g, v, _gt, _rn in inputs.c3():
        probs.append(problem(g, v))
    for pr in probs:
        lib.autotune([pr], reps=reps)
        print(f"D={pr.D} N={pr.means.shape[0]} B={pr.rot.shape[0]}: tile {pr.options.tile} "
              f"halo {pr.options.halo} budget {pr.options.budget} lane order {pr.options.lane_order}", flush=True)


if __name__ == "__main__":
    main(sys.argv[1] if len(sys.argv) > 1 else
         os.path.join(os.path.dirname(os.path.abspath(__file__)), "tune_mi355x.txt"))
