#!/usr/bin/env python
"""Benchmark of one training step of the splat renderer on one MI355X.

Workload (the configuration the headline metric is quoted on): a mixture of
N = 200,000 Gaussians (isotropic, s = 2.112 A, A = 1/(2N), means uniform in a
ball of radius 75 A), 64 particle images of 256 x 256 pixels at 1.1 A,
Haar-random poses, defocus U(0.5, 2.5) um, observed images rendered from an
independent ground-truth mixture plus white noise at SNR -20 dB.

One step = render with CTF + squared-error loss + adjoint + Adam on all
11 N parameters, every stage in the HIP library.  Inputs are resident in
HBM before the timed region.  Prints one JSON line.
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

METRIC = ("particle images/sec fwd+bwd (N=200k, D=256) and % roofline; "
          "pose-proposal speedup")
Q_CUT = 27.631021115928547  # 2 ln 1e6, the library default

# Nominal per-pair budget of the splat (one exp2 plus FMA-class ops) priced
# at chip rates: 256 CUs at 2.4 GHz, transcendental at a quarter of the
# 64-lane FP32 rate, FMA-class ops at the packed-FP32 rate.  Reported as a
# separately labelled ratio; the kernels evaluate no exp per pixel, so this
# is a budget, not a ceiling.
EXP_RATE = 256 * 16 * 2.4e9          # exp2 per second
FMA_RATE = 256 * 128 * 2.4e9         # FP32 lane-ops per second (packed)
PAIR_OPS = {"k_splat_fwd": 8, "k_splat_bwd": 20}
# VALU issue ceiling: the published FP32 vector rate, 157.3 TFLOP/s = 256 CUs
# x 128 lanes x 2 (FMA) x 2.4 GHz, i.e. two wave64 VALU instructions per CU
# per cycle (the splat kernels are measured above one per CU per cycle, so
# one is not a ceiling); a transcendental takes four issue slots.
VALU_INSTR_RATE = 256 * 2 * 2.4e9    # wave64 VALU instructions per second
TRANS_SLOTS = 4
# LDS: 128 bytes per CU per cycle
LDS_CYCLE_RATE = 256 * 2.4e9         # LDS cycles per second, all CUs


def _source_digest(kernel: str) -> str:
    """sha1 of the sources that define the splat kernels (counter validity)."""
    import hashlib
    h = hashlib.sha1()
    for f in ("k_splat.hip", "cs_internal.hpp"):
        with open(os.path.join(ROOT, "paper_2508_04929_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def _profile_record(name: str, tag: str):
    """The `tag` JSON line of a committed rocprofv3 summary under profiles/,
    or None when missing or taken on other splat sources."""
    path = os.path.join(ROOT, "profiles", name)
    if not os.path.exists(path):
        return None
    rec = None
    with open(path) as fh:
        for line in fh:
            if line.startswith(tag + ": "):
                rec = json.loads(line[len(tag) + 2:])
    if not rec or rec.get("source_sha1") != _source_digest(""):
        return None
    return rec


def measured_traffic(kernel: str, launches_per_step: int = 1):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 counter
    summary (FETCH_SIZE + WRITE_SIZE scaled by a copy kernel of known size),
    or None when the summary is missing or the kernel source has changed
    since the counters were taken."""
    rec = _profile_record("splat_hbm_traffic_c4.md", "traffic-json")
    k = (rec or {}).get("kernels", {}).get(kernel)
    return None if k is None else float(k["bytes_per_launch"])


def issue_ceiling(kernel: str, profile: str = "splat_issue_counters_c4.md"):
    """Hardware ceilings of a splat kernel from its committed instruction
    counters (SQ_INSTS_VALU, SQ_INSTS_VALU_TRANS_F32, SQ_LDS_IDX_ACTIVE per
    launch, the launch's algorithmic pairs): pairs per second at the VALU
    issue ceiling, and the LDS busy cycles per pair; None when missing or
    stale."""
    rec = _profile_record(profile, "issue-json")
    k = (rec or {}).get("kernels", {}).get(kernel)
    if k is None:
        return None
    slots = k["valu_insts"] + (TRANS_SLOTS - 1) * k["trans_insts"]
    out = {"valu_insts_per_pair": k["valu_insts"] / k["pairs"],
           "valu_issue_slots_per_pair": slots / k["pairs"],
           "pairs_per_s_at_issue_ceiling": VALU_INSTR_RATE * k["pairs"] / slots}
    if k.get("lds_idx_active"):
        out["lds_cycles_per_pair"] = k["lds_idx_active"] / k["pairs"]
        out["pairs_per_s_at_lds_ceiling"] = LDS_CYCLE_RATE * k["pairs"] / k["lds_idx_active"]
    return out


def pair_peak(kernel: str) -> float:
    """Pairs per second at 100% of the nominal per-pair budget."""
    return 1.0 / (1.0 / EXP_RATE + PAIR_OPS[kernel] / FMA_RATE)


# --------------------------------------------------------------- CPU oracle

_W = {}


def _oracle_init(workload, barrier):
    """Pool worker set-up: the workload's seeded inputs, built once per worker."""
    import numpy as np
    from paper_2508_04929_amd import inputs
    if workload == "c1":
        g, v, _gt = inputs.c1()
    elif workload == "c2":
        g, v, _gt, _rn = inputs.c2()
    else:
        g, v, _gt, _rn = inputs.c4()
    _W.update(g=g, v=v, workload=workload, rng=np.random.default_rng(1234))
    _W["barrier"] = barrier


def _oracle_ready(_):
    _W["barrier"].wait()


def _oracle_task(b):
    """One image of the workload through the FP64 oracle: forward + CTF + loss
    (c1: forward and loss only), else also the analytic gradient."""
    import numpy as np
    from oracle import objective
    g, v = _W["g"], _W["v"]
    vs = v.subset([b])
    Y = _W["rng"].standard_normal((1, v.D, v.D)) * 1e-4   # the values do not change the work
    if _W["workload"] == "c1":
        objective.forward(g, vs, Y, q_cut=Q_CUT)
    else:
        objective.loss_and_grad(g, vs, Y, q_cut=Q_CUT)


def cpu_baseline(n_images: int, workload: str = "c4"):
    """The FP64 oracle on n_images images of a workload, one image per task in
    a process pool over the host's cores; throughput = images / pool wall
    time (inputs built in every worker before the clock starts)."""
    import multiprocessing as mp
    cores = min(len(os.sched_getaffinity(0)), 16, n_images)
    ctx = mp.get_context("spawn")
    barrier = ctx.Barrier(cores)
    with ctx.Pool(cores, initializer=_oracle_init, initargs=(workload, barrier)) as pool:
        pool.map(_oracle_ready, range(cores), chunksize=1)
        t0 = time.perf_counter()
        pool.map(_oracle_task, range(n_images), chunksize=1)
        wall = time.perf_counter() - t0
    what = {"c1": "N=1,000, D=64, forward + CTF + loss",
            "c2": "N=20,000, D=128, forward + CTF + loss + analytic gradient",
            "c4": "N=200,000, D=256, forward + CTF + loss + analytic gradient"}[workload]
    return {"value": n_images / wall, "unit": "images/s", "cores": cores, "kind": "oracle",
            "sample": (f"{n_images} images of the workload ({what}), FP64 numpy oracle with "
                       f"the same q_cut as the GPU, one image per task on {cores} worker "
                       f"processes; {wall:.1f} s pool wall time")}


# ------------------------------------------------------------------- GPU

def run(args):
    import numpy as np
    import torch

    from paper_2508_04929_amd import binding, inputs

    lib = binding.library()
    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    g, v, gt, rn = inputs.c4(b=args.batch)
    N, B, D, p = g.n, v.b, v.D, v.pixel

    t = lambda x: torch.from_numpy(np.ascontiguousarray(x, dtype=np.float32)).to(dev)
    # parameters and gradients as one flat buffer each: [means | log_scales | quats | amps]
    flat = torch.cat([t(g.means).reshape(-1), t(g.log_scales).reshape(-1),
                      t(g.quats).reshape(-1), t(g.amps).reshape(-1)]).contiguous()
    sizes = [3 * N, 3 * N, 4 * N, N]
    shapes = [(N, 3), (N, 3), (N, 4), (N,)]

    def views_of(buf):
        out, o = [], 0
        for s, sh in zip(sizes, shapes):
            out.append(buf[o:o + s].view(*sh))
            o += s
        return out

    params = views_of(flat)
    gflat = torch.zeros_like(flat)
    gviews = views_of(gflat)
    grads = dict(zip(("means", "log_scales", "quats", "amps"), gviews))
    m = torch.zeros_like(flat)
    vv = torch.zeros_like(flat)
    rot, shift = t(v.rot), t(v.shift)
    ctf = binding.Ctf(t(v.defocus_u), t(v.defocus_v), t(v.astig), t(v.phase),
                      v.voltage_kv, v.cs_mm, v.amp_contrast, v.bfactor)
    # observed images: ground-truth render + white noise at -20 dB
    Xgt = lib.render(t(gt.means), t(gt.log_scales), t(gt.quats), t(gt.amps), rot, shift, D, p,
                     ctf=ctf)
    gen = torch.Generator(device=dev).manual_seed(4)
    sd = torch.sqrt(Xgt.double().var() / 10 ** (-20 / 10)).float()
    Y = (Xgt + sd * torch.randn(Xgt.shape, device=dev, generator=gen)).contiguous()
    del Xgt
    loss = torch.empty(B + 1, device=dev)
    pairs = lib.pair_count(*params, rot, shift, D, p)
    torch.cuda.synchronize()
    pairs_step = int(pairs.sum().item())

    step_no = [0]

    # launch options (tile, halo, budget) from the library's autotuner on this
    # step's own problem; results do not depend on them
    pr = lib.make_problem(*params, rot, shift, D, p, Y, ctf=ctf, reduction="mean")
    lib.autotune([pr], reps=3)
    tuned = pr.options
    del pr
    graph_opt = binding.Options(tile=tuned.tile, halo=tuned.halo, budget=tuned.budget, graph=1,
                                lane_order=tuned.lane_order)

    def step(graph=False):
        lib.loss_and_grad(*params, rot, shift, D, p, Y, ctf=ctf, reduction="mean",
                          grads=grads, loss=loss, options=graph_opt if graph else tuned)
        step_no[0] += 1
        lib.adam_step(flat, gflat, m, vv, step_no[0], lr=1e-3)

    if args.calib_copy_mib > 0:
        # a plain device copy of known size, for scaling the HBM byte counters
        nel = args.calib_copy_mib * (1 << 20) // 4
        src = torch.ones(nel, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    # timed steps run without per-kernel events (optionally as graph replays);
    # per-kernel times come from a separate pass with HIP events around every
    # kernel
    for _ in range(args.warmup):
        step(graph=args.graph)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step(graph=args.graph)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    lib.set_timing(dev, True)
    timing_steps = max(3, min(args.steps, 10))
    for _ in range(timing_steps):
        step(graph=False)
    torch.cuda.synchronize()
    stages = {}
    for name in binding.STAGES:
        ms, n = lib.stage_time(dev, name)
        if n:
            stages[name] = {"ms_total": ms, "launches": n, "ms_per_launch": ms / n}
    lib.set_timing(dev, False)
    final_loss = float(loss[-1].item())

    # the same step with the gradients w.r.t. the 64 views' rotations and
    # shifts as well (joint pose refinement): step time, and the pose-gradient
    # kernels' HIP-event times against the bytes they must read
    grads_pose = dict(grads, rot=torch.empty(B, 3, 3, device=dev), shift=torch.empty(B, 2, device=dev))

    def step_pose():
        lib.loss_and_grad(*params, rot, shift, D, p, Y, ctf=ctf, reduction="mean",
                          grads=grads_pose, loss=loss, options=tuned)
        step_no[0] += 1
        lib.adam_step(flat, gflat, m, vv, step_no[0], lr=1e-3)

    for _ in range(2):
        step_pose()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    for _ in range(args.steps):
        step_pose()
    torch.cuda.synchronize()
    ms_pose = 1e3 * (time.perf_counter() - t1) / args.steps
    lib.set_timing(dev, True)
    for _ in range(timing_steps):
        step_pose()
    torch.cuda.synchronize()
    pg = {}
    for name in ("k_pose_grad_part", "k_pose_grad_sum"):
        ms, n = lib.stage_time(dev, name)
        if n:
            pg[name] = ms / n
    lib.set_timing(dev, False)
    # per launch: six pixel moments and the visibility key per (image, Gaussian),
    # the Gaussian records, 8 partial sums per (image, block of 1,024 Gaussians)
    pg_bytes = B * N * (24 + 4) + N * 48 + B * ((N + 1023) // 1024) * 32
    pose_grad = {
        "ms_per_step": ms_pose, "ms_per_step_without": None,
        "ms_per_launch": pg,
        "roofline": ({"bound": "hbm", "kernel": "k_pose_grad_part",
                      "achieved": pg_bytes / (pg["k_pose_grad_part"] * 1e-3) / 1e9,
                      "peak": 8000.0, "unit": "GB/s",
                      "frac": pg_bytes / (pg["k_pose_grad_part"] * 1e-3) / 8e12,
                      "bytes_per_launch": pg_bytes}
                     if "k_pose_grad_part" in pg else None)}

    ms_step = 1e3 * elapsed / args.steps
    value = B * args.steps / elapsed
    dom = max(("k_splat_fwd", "k_splat_bwd"), key=lambda k: stages.get(k, {}).get("ms_total", 0))
    d = stages[dom]
    achieved = pairs_step / (d["ms_per_launch"] * 1e-3)     # pairs per second

    def ceilings(kernel, ach):
        """(peak pairs/s, ceiling record): the lower of the VALU issue and LDS
        ceilings from the committed counters, None without them."""
        c = issue_ceiling(kernel)
        if c is None:
            return None, None
        peaks = {"valu_issue": c["pairs_per_s_at_issue_ceiling"]}
        if "pairs_per_s_at_lds_ceiling" in c:
            peaks["lds"] = c["pairs_per_s_at_lds_ceiling"]
        limit = min(peaks, key=peaks.get)
        c["binding"] = limit
        c["frac_of_valu_issue"] = ach / peaks["valu_issue"]
        if "lds" in peaks:
            c["frac_of_lds"] = ach / peaks["lds"]
        return peaks[limit], c

    peak, ceil_rec = ceilings(dom, achieved)
    nominal = pair_peak(dom)
    roof = {"bound": "alu", "kernel": dom, "achieved": achieved / 1e9,
            "peak": None if peak is None else peak / 1e9, "unit": "Gpair/s",
            "frac": None if peak is None else achieved / peak,
            "traffic": measured_traffic(dom), "pairs_per_launch": pairs_step,
            "ms_per_launch": d["ms_per_launch"], "ceiling": ceil_rec,
            "nominal_budget": {"peak": nominal / 1e9, "frac": achieved / nominal,
                               "note": "1 exp2 + FMA-class ops per pair at datasheet rates; "
                                       "a budget, not a ceiling"}}
    other = "k_splat_bwd" if dom == "k_splat_fwd" else "k_splat_fwd"
    if other in stages:
        o = stages[other]
        ach_o = pairs_step / (o["ms_per_launch"] * 1e-3)
        peak_o, ceil_o = ceilings(other, ach_o)
        roof["other_splat"] = {"kernel": other, "achieved": ach_o / 1e9,
                               "peak": None if peak_o is None else peak_o / 1e9,
                               "frac": None if peak_o is None else ach_o / peak_o,
                               "ceiling": ceil_o, "ms_per_launch": o["ms_per_launch"],
                               "traffic": measured_traffic(other),
                               "nominal_budget": {"peak": pair_peak(other) / 1e9,
                                                  "frac": ach_o / pair_peak(other)}}
    step_roof_s = pairs_step * (1 / pair_peak("k_splat_fwd") + 1 / pair_peak("k_splat_bwd"))

    # Whole-step roofline: T_roof = sum over the step's kernels of the time
    # at the bound that limits each, T_roof / T_measured.  The splat kernels
    # at their hardware ceilings (the lower of VALU issue and LDS, from the
    # committed counters); every other kernel at its HBM bytes per launch
    # (FETCH_SIZE + WRITE_SIZE, committed counters) over the 8 TB/s peak,
    # times its launches per step.  None when a summary is missing or stale.
    def step_roofline(rates=None):
        """With rates (the chip-rate probes of this GPU), every term at the
        measured rate instead: VALU issue slots at the FP32 probe's wave64
        instructions per second, LDS busy cycles at its clock, HBM bytes at
        the copy probe's rate."""
        terms, unpriced = {}, []
        for name, st in stages.items():
            per_step = st["launches"] / timing_steps
            if name in ("k_splat_fwd", "k_splat_bwd"):
                c = issue_ceiling(name)
                if c is None:
                    return None
                if rates is None:
                    t = c["valu_issue_slots_per_pair"] / VALU_INSTR_RATE
                    if "lds_cycles_per_pair" in c:
                        t = max(t, c["lds_cycles_per_pair"] / LDS_CYCLE_RATE)
                else:
                    t = c["valu_issue_slots_per_pair"] / rates["fma"]["wave_instr_per_s"]
                    if "lds_cycles_per_pair" in c:
                        t = max(t, c["lds_cycles_per_pair"]
                                / (256 * rates["fma"]["clock_ghz"] * 1e9))
                terms[name] = per_step * pairs_step * t * 1e3
            else:
                bts = measured_traffic(name)
                if bts is None:
                    unpriced.append(name)  # left out: T_roof only shrinks
                    continue
                bw = 8e12 if rates is None else rates["copy"]["gb_per_s"] * 1e9
                terms[name] = per_step * bts / bw * 1e3
        t_roof = sum(terms.values())
        return {"t_roof_ms": t_roof, "t_measured_ms": ms_step, "frac": t_roof / ms_step,
                "terms_ms": terms, "unpriced": unpriced,
                "note": ("splat kernels at their VALU-issue / LDS ceilings (counters), other "
                         "kernels at measured HBM bytes / 8 TB/s; measured step from wall time"
                         if rates is None else
                         "as above, at the rates the chip-rate probes measured on this GPU "
                         "(FP32 VALU issue and its clock, simple-copy bandwidth); the FP32 "
                         "probe's all-FMA load runs at a lower clock than the splat kernels, "
                         "so their terms here can exceed their measured times")}
    result = {
        "metric": METRIC, "value": value, "unit": "images/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_step,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": ("training step: N=200,000 Gaussians, 64 images D=256, "
                                "p=1.1 A, CTF, squared-error loss, adjoint, Adam on 11N "
                                "parameters"),
                   "N": N, "batch": B, "D": D, "pixel_A": p, "q_cut": Q_CUT,
                   "pairs_per_step": pairs_step, "pairs_per_image": pairs_step / B,
                   "launch_options": {"tile": tuned.tile, "halo": tuned.halo,
                                      "budget": tuned.budget, "lane_order": tuned.lane_order,
                                      "source": "cs_autotune"},
                   "final_loss": final_loss},
        "roofline": roof,
        "step_fraction_of_splat_roofline": step_roof_s / (ms_step * 1e-3),
        "step_roofline": step_roofline(),
        "step_roofline_at_measured_rates": (step_roofline(getattr(args, "rates", None))
                                            if getattr(args, "rates", None) else None),
        "stages_ms_per_step": {k: s["ms_total"] / timing_steps for k, s in stages.items()},
        "graph_replay": bool(args.graph),
        "pose_gradients": pose_grad,
    }
    pose_grad["ms_per_step_without"] = ms_step
    return result


def run_small(workload: str, steps: int = 20, warmup: int = 3, cpu_images: int = 16):
    """The other two single-mixture workloads:
    c2: N=20,000 anisotropic Gaussians, 256 images of 128^2 at 1.5 A with
        shifts, CTF, observed = ground-truth render + noise at -20 dB;
        forward + loss + adjoint + Adam per step;
    c1: N=1,000 isotropic Gaussians, 16 images of 64^2 at 3 A, CTF; forward +
        squared-error loss only.
    Images/s with inputs resident, the splat kernels' pairs/s (against the
    ceilings of a committed counter summary of this workload when there is
    one) and the FP64 oracle on cpu_images images."""
    import numpy as np
    import torch

    from paper_2508_04929_amd import binding, inputs

    lib = binding.library()
    dev = torch.device("cuda", 0)
    t = lambda x: torch.from_numpy(np.ascontiguousarray(x, dtype=np.float32)).to(dev)
    if workload == "c1":
        g, v, gt = inputs.c1()
    else:
        g, v, gt, _rn = inputs.c2()
    N, B, D, p = g.n, v.b, v.D, v.pixel
    prm = [t(g.means), t(g.log_scales), t(g.quats), t(g.amps)]
    rot, shift = t(v.rot), t(v.shift)
    ctf = binding.Ctf(t(v.defocus_u), t(v.defocus_v), t(v.astig), t(v.phase),
                      v.voltage_kv, v.cs_mm, v.amp_contrast, v.bfactor)
    X = lib.render(t(gt.means), t(gt.log_scales), t(gt.quats), t(gt.amps), rot, shift, D, p, ctf=ctf)
    if workload == "c2":
        gen = torch.Generator(device=dev).manual_seed(4)
        sd = torch.sqrt(X.double().var() / 10 ** (-20 / 10)).float()
        Y = (X + sd * torch.randn(X.shape, device=dev, generator=gen)).contiguous()
    else:
        Y = X
    pairs = int(lib.pair_count(*prm, rot, shift, D, p).sum().item())
    flat = torch.cat([x.reshape(-1) for x in prm]).contiguous()
    sizes = [3 * N, 3 * N, 4 * N, N]
    views = lambda buf: [buf[o:o + n].view(*x.shape) for o, n, x in
                         zip(np.cumsum([0] + sizes[:-1]), sizes, prm)]
    params = views(flat)
    gflat = torch.zeros_like(flat)
    grads = dict(zip(("means", "log_scales", "quats", "amps"), views(gflat)))
    m, vv = torch.zeros_like(flat), torch.zeros_like(flat)
    loss = torch.empty(B + 1, device=dev)
    k = [0]
    pr = lib.make_problem(*params, rot, shift, D, p, Y, ctf=ctf, reduction="mean",
                          want_grads=workload != "c1")
    lib.autotune([pr], reps=3)
    tuned = pr.options
    del pr

    def step():
        if workload == "c1":
            lib.loss_and_grad(*params, rot, shift, D, p, Y, ctf=ctf, reduction="mean",
                              want_grads=False, loss=loss, options=tuned)
        else:
            lib.loss_and_grad(*params, rot, shift, D, p, Y, ctf=ctf, reduction="mean",
                              grads=grads, loss=loss, options=tuned)
            k[0] += 1
            lib.adam_step(flat, gflat, m, vv, k[0], lr=1e-3)

    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        step()
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / steps
    lib.set_timing(dev, True)
    for _ in range(3):
        step()
    torch.cuda.synchronize()
    stages = {}
    for name in binding.STAGES:
        ms, n = lib.stage_time(dev, name)
        if n:
            stages[name] = ms / n
    lib.set_timing(dev, False)
    splat = {}
    for kern in ("k_splat_fwd", "k_splat_bwd"):
        if kern not in stages:
            continue
        ach = pairs / (stages[kern] * 1e-3)
        c = issue_ceiling(kern, f"splat_issue_counters_{workload}.md")
        rec = {"ms_per_launch": stages[kern], "pairs_per_s": ach,
               "nominal_budget_frac": ach / pair_peak(kern), "ceiling": c}
        if c is not None:
            peaks = {"valu_issue": c["pairs_per_s_at_issue_ceiling"]}
            if "pairs_per_s_at_lds_ceiling" in c:
                peaks["lds"] = c["pairs_per_s_at_lds_ceiling"]
            lim = min(peaks, key=peaks.get)
            rec.update(bound=lim, frac=ach / peaks[lim])
        splat[kern] = rec
    out = {"workload": ("N=20,000 anisotropic Gaussians, 256 images D=128, p=1.5 A, shifts, CTF, "
                        "-20 dB; forward + loss + adjoint + Adam" if workload == "c2" else
                        "N=1,000 isotropic Gaussians, 16 images D=64, p=3 A, CTF; forward + "
                        "squared-error loss"),
           "images_per_s": B / dt, "ms_per_step": dt * 1e3, "pairs_per_step": pairs,
           "launch_options": [tuned.tile, tuned.halo, tuned.budget, tuned.lane_order],
           "splat": splat, "stages_ms_per_step": stages}
    if cpu_images > 0:
        out["cpu_baseline"] = cpu_baseline(min(cpu_images, B), workload)
    return out


def run_volume(reps: int = 5):
    """The reconstruction read out as a volume and compared (Sec. 3 overview,
    Sec. 4 Eq. 10): voxelise the N = 200,000 training mixture and its ground
    truth at D = 256 (1.1 A voxels), FSC between them."""
    import numpy as np
    import torch

    from paper_2508_04929_amd import binding, inputs

    lib = binding.library()
    dev = torch.device("cuda", 0)
    t = lambda x: torch.from_numpy(np.ascontiguousarray(x, dtype=np.float32)).to(dev)
    g, v, gt, rn = inputs.c4(b=1)
    D, p = 256, 1.1
    ma = [t(g.means), t(g.log_scales), t(g.quats), t(g.amps)]
    mb = [t(gt.means), t(gt.log_scales), t(gt.quats), t(gt.amps)]
    Va, Vb = lib.voxelize(*ma, D, p), lib.voxelize(*mb, D, p)
    curve = lib.fsc(Va, Vb)
    torch.cuda.synchronize()

    def timed_ms(fn):
        ts = []
        for _ in range(reps):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            fn()
            e1.record()
            torch.cuda.synchronize()
            ts.append(e0.elapsed_time(e1))
        return float(np.median(ts))

    ms_vox = timed_ms(lambda: lib.voxelize(*mb, D, p, out=Vb))
    ms_fsc = timed_ms(lambda: lib.fsc(Va, Vb, out=curve))
    return {"workload": ("voxelise the N=200,000 ground-truth mixture at D=256, 1.1 A "
                         "(q <= 2 ln 1e6); FSC of the training start vs the ground truth"),
            "voxelize_ms": ms_vox, "voxels_per_s": D ** 3 / (ms_vox * 1e-3),
            "gaussians_per_s": gt.n / (ms_vox * 1e-3),
            "fsc_ms": ms_fsc,
            "fsc_bytes_min": 2 * D ** 3 * 4,
            "resolution_A": lib.resolution(curve, D, p)[0]}


def run_trainer(steps: int = 1024, sizes=((256, 2048), (256, 10000), (256, 30000))):
    """The paper-faithful loop of Alg. 1 at batch size 1 (Sec. 4.1): box
    units, the paper's initialisation, Adam per particle.  Particles: a
    domain mixture (20,000 Gaussians, 3 A widths) at Haar-random poses with
    CTF (1.1 A pixels) and white noise at 0 dB, translations up to 2 px
    (centred by FourierShift before training).  Per size: one warm-up pass,
    then `steps` timed steps with the loss path replayed as a HIP graph,
    and the same steps launched eagerly."""
    import numpy as np
    import torch

    from paper_2508_04929_amd import binding, inputs, trainer

    lib = binding.library()
    dev = torch.device("cuda", 0)
    t = lambda x: torch.from_numpy(np.ascontiguousarray(x, dtype=np.float32)).to(dev)
    out = []
    for D, N in sizes:
        rng = np.random.default_rng(7)
        p_a = 1.1
        L = D * p_a
        gt = inputs.mixture_domains(rng, 20000, radius=0.2 * L, scale_mu=np.log(3.0))
        amps = np.asarray(gt.amps, np.float64)
        g = [t(np.asarray(gt.means, np.float64) / L), t(np.asarray(gt.log_scales, np.float64) - np.log(L)),
             t(gt.quats), t(0.5 * amps / amps.sum())]
        v = inputs.views(rng, steps, D, 1.0 / D)
        rot, shift = t(v.rot), t(rng.uniform(-2, 2, size=(steps, 2)) / D)
        ctf = binding.Ctf(t(v.defocus_u), t(v.defocus_v), t(v.astig), t(v.phase), v.voltage_kv,
                          v.cs_mm, v.amp_contrast, v.bfactor, pixel_a=p_a)
        images = lib.render(*g, rot, shift, D, 1.0 / D, ctf=ctf)
        lib.add_noise(images, 0.0, seed=11)
        data = trainer.Trainer.centre(lib, trainer.Dataset(images=images, rot=rot, shift=shift, ctf=ctf))
        res = {"D": D, "N": N, "steps": steps}
        for graph in (True, False):
            tr = trainer.Trainer(lib, t(rng.standard_normal((N, 3))), graph=graph)
            tr.epoch(data, rng.permutation(steps), 1e-3)          # warm-up pass
            torch.cuda.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            tr.epoch(data, rng.permutation(steps), 1e-3)
            e1.record()
            torch.cuda.synchronize()
            ms = e0.elapsed_time(e1)
            key = "graph" if graph else "eager"
            res[f"{key}_images_per_s"] = steps / (ms * 1e-3)
            res[f"{key}_ms_per_step"] = ms / steps
        out.append(res)
        print(f"[bench] trainer D={D} N={N}: {res['graph_images_per_s']:.0f} img/s graphed, "
              f"{res['eager_images_per_s']:.0f} eager", file=sys.stderr, flush=True)
    return {"workload": ("batch-1 Adam training of Alg. 1 (box units, paper initialisation, "
                         "softplus activations, CTF, 0 dB noise, FourierShift-centred particles)"),
            "sizes": out}


def run_reconstruction(n: int = 10000, m: int = 10000, D: int = 128, p_a: float = 1.5,
                       snr_db: float = -10.0, epochs: int = 5, gamma: float = 0.1):
    """End to end with the settings of Sec. 4.1: N = 10,000 Gaussians from the
    paper's initialisation, batch-1 Adam (lr 1e-3, x gamma per epoch) for 5
    epochs over M synthetic particles (a 20,000-Gaussian domain mixture at
    Haar poses, CTF, white noise at snr_db, translations up to 2 px removed
    by FourierShift), then the FSC of the voxelised result against the
    voxelised ground truth (D^3 grid of the box)."""
    import numpy as np
    import torch

    from paper_2508_04929_amd import binding, inputs, trainer

    lib = binding.library()
    dev = torch.device("cuda", 0)
    t = lambda x: torch.from_numpy(np.ascontiguousarray(x, dtype=np.float32)).to(dev)
    rng = np.random.default_rng(21)
    L = D * p_a
    gt = inputs.mixture_domains(rng, 20000, radius=0.2 * L, scale_mu=np.log(2.0))
    amps = np.asarray(gt.amps, np.float64)
    g = [t(np.asarray(gt.means, np.float64) / L), t(np.asarray(gt.log_scales, np.float64) - np.log(L)),
         t(gt.quats), t(0.5 * amps / amps.sum())]
    v = inputs.views(rng, m, D, 1.0 / D)
    rot, shift = t(v.rot), t(rng.uniform(-2, 2, size=(m, 2)) / D)
    ctf = binding.Ctf(t(v.defocus_u), t(v.defocus_v), t(v.astig), t(v.phase), v.voltage_kv,
                      v.cs_mm, v.amp_contrast, v.bfactor, pixel_a=p_a)
    images = lib.render(*g, rot, shift, D, 1.0 / D, ctf=ctf)
    lib.add_noise(images, snr_db, seed=22)
    Vgt = lib.voxelize(*g, D, 1.0 / D)
    tr = trainer.Trainer(lib, t(rng.standard_normal((n, 3))))
    res0 = lib.resolution(lib.fsc(tr.voxelize(D), Vgt), D, p_a)[0]
    data = trainer.Dataset(images=images, rot=rot, shift=shift, ctf=ctf)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    losses = tr.fit(data, epochs=epochs, lr=1e-3, gamma=gamma, seed=23, record_loss=True)
    torch.cuda.synchronize()
    secs = time.perf_counter() - t0
    curve_d = lib.fsc(tr.voxelize(D), Vgt)
    curve = curve_d.cpu().numpy()
    floor, _, _ = lib.loss_and_grad(*g, rot, shift, D, 1.0 / D, images, ctf=ctf, want_grads=False)
    lo = losses.cpu().numpy()
    return {"workload": (f"N={n} Gaussians, paper initialisation, batch-1 Adam lr 1e-3 x {gamma}/epoch, "
                         f"{epochs} epochs over {m} particles D={D} p={p_a} A (CTF, {snr_db:g} dB, "
                         "translations); ground truth a 20,000-Gaussian domain mixture"),
            "seconds": secs, "images_per_s": epochs * m / secs,
            "loss_first_epoch": float(lo[:m].mean()), "loss_last_epoch": float(lo[-m:].mean()),
            "loss_ground_truth": float(floor[-1]) / m,
            "fsc_resolution_A_initial": res0,
            "fsc_resolution_A": lib.resolution(curve_d, D, p_a)[0],
            "fsc_curve": [round(float(x), 4) for x in curve]}


def run_densify(n: int = 200000, reps: int = 20):
    """SplitGaussian of every Gaussian with the Adam moments (Alg. 1
    densification): N = 200,000 -> 400,000.  Algorithmic bytes: read the
    parameters and both moments (3 x 11 N floats), write them for 2N."""
    import numpy as np
    import torch

    from paper_2508_04929_amd import binding

    lib = binding.library()
    gen = torch.Generator(device="cuda").manual_seed(5)
    p = torch.randn(11 * n, device="cuda", generator=gen)
    m = torch.randn(11 * n, device="cuda", generator=gen)
    v = torch.rand(11 * n, device="cuda", generator=gen)
    out = lib.split_gaussians(p, m, v)   # the outputs, reused by the timed calls
    torch.cuda.synchronize()
    ts = []
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        lib.split_gaussians(p, m, v, out=out)
        e1.record()
        torch.cuda.synchronize()
        ts.append(e0.elapsed_time(e1))
    ms = float(np.median(ts))
    nbytes = 3 * 11 * n * 4 * 3
    return {"workload": f"split N={n} Gaussians (parameters and Adam moments) into {2 * n}",
            "ms": ms, "bytes": nbytes, "GB_per_s": nbytes / (ms * 1e-3) / 1e9,
            "frac_of_hbm_peak": nbytes / (ms * 1e-3) / 8e12,
            "note": "median over calls into preallocated outputs (no allocation timed)"}


def run_batched(reps: int = 10, autotune: bool = True):
    """Uneven batching: 8 mixtures (N = 5k ... 150k) x 128 images, D in
    {128, 192, 256}, fwd + adjoint of all problems in one persistent launch
    per pass (replayed graph), against the same problems as 8 calls."""
    import numpy as np
    import torch

    from paper_2508_04929_amd import binding, inputs

    lib = binding.library()
    dev = torch.device("cuda", 0)
    t = lambda x: torch.from_numpy(np.ascontiguousarray(x, dtype=np.float32)).to(dev)
    probs, n_img, pairs = [], 0, 0
    for g, v, gt, rn in inputs.c3():
        rot, shift = t(v.rot), t(v.shift)
        ctf = binding.Ctf(t(v.defocus_u), t(v.defocus_v), t(v.astig), t(v.phase),
                          v.voltage_kv, v.cs_mm, v.amp_contrast, v.bfactor)
        X = lib.render(t(gt.means), t(gt.log_scales), t(gt.quats), t(gt.amps), rot, shift, v.D,
                       v.pixel, ctf=ctf)
        sd = torch.sqrt(X.double().var() / 10 ** (-20 / 10)).float()
        gen = torch.Generator(device=dev).manual_seed(3)
        Y = (X + sd * torch.randn(X.shape, device=dev, generator=gen)).contiguous()
        prm = [t(g.means), t(g.log_scales), t(g.quats), t(g.amps)]
        probs.append(lib.make_problem(*prm, rot, shift, v.D, v.pixel, Y, ctf=ctf,
                                      reduction="mean"))
        pairs += int(lib.pair_count(*prm, rot, shift, v.D, v.pixel).sum().item())
        n_img += v.b
    if autotune:
        lib.autotune(probs, reps=2)

    def batched():
        lib.loss_and_grad_multi(probs, use_graph=True)

    def separate():
        for pr in probs:
            lib.loss_and_grad(pr.means, pr.log_scales, pr.quats, pr.amps, pr.rot, pr.shift, pr.D,
                              pr.pixel, pr.observed, ctf=pr.ctf, options=pr.options,
                              reduction="mean", grads=pr.grads, loss=pr.loss)

    # per-kernel HIP-event times of one eager batched call (the splat kernels
    # run one launch per canvas size over all problems)
    lib.set_timing(dev, True)
    lib.loss_and_grad_multi(probs, use_graph=False)
    torch.cuda.synchronize()
    stages = {}
    for name in binding.STAGES:
        ms, n = lib.stage_time(dev, name)
        if n:
            stages[name] = {"ms": ms, "launches": n}
    lib.set_timing(dev, False)
    splat = {}
    for kern in ("k_splat_fwd", "k_splat_bwd"):
        if kern not in stages:
            continue
        ach = pairs / (stages[kern]["ms"] * 1e-3)
        c = issue_ceiling(kern, "splat_issue_counters_c3.md")
        rec = {"ms": stages[kern]["ms"], "launches": stages[kern]["launches"], "pairs_per_s": ach,
               "nominal_budget_frac": ach / pair_peak(kern), "ceiling": c}
        if c is not None:
            peaks = {"valu_issue": c["pairs_per_s_at_issue_ceiling"]}
            if "pairs_per_s_at_lds_ceiling" in c:
                peaks["lds"] = c["pairs_per_s_at_lds_ceiling"]
            lim = min(peaks, key=peaks.get)
            rec.update(bound=lim, frac=ach / peaks[lim])
        splat[kern] = rec
    out = {"splat": splat, "stages_ms": {k: v["ms"] for k, v in stages.items()}}
    for name, fn in (("batched", batched), ("separate", separate)):
        fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            fn()
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / reps
        out[name] = {"ms": dt * 1e3, "images_per_s": n_img / dt, "pairs_per_s": pairs / dt}
    out["workload"] = ("uneven batching: 8 mixtures, N = 5k...150k, 128 images each at D in "
                       "{128,192,256}, CTF, fwd + adjoint, autotuned tile/halo/budget")
    out["images"] = n_img
    out["pairs"] = pairs
    out["options"] = [[pr.options.tile, pr.options.halo, pr.options.budget, pr.options.lane_order]
                      for pr in probs]
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--batch", type=int, default=64)
    ap.add_argument("--calib-copy-mib", type=int, default=0,
                    help="run one device copy of this many MiB before warm-up (counter calibration)")
    ap.add_argument("--cpu-images", type=int, default=16,
                    help="images of the workload timed through the CPU oracle (0 = skip)")
    ap.add_argument("--graph", action="store_true",
                    help="replay the library's captured graph of the loss-and-gradient call "
                         "in the timed steps (measured equal to eager calls)")
    ap.add_argument("--no-pose", dest="pose", action="store_false",
                    help="skip the learned-pose experiment (network trained on 200k renders, "
                         "then learned proposal + refinement vs grid search; about a minute)")
    ap.add_argument("--no-trainer", dest="trainer", action="store_false",
                    help="skip the batch-1 training-loop measurement")
    ap.add_argument("--no-volume", dest="volume", action="store_false",
                    help="skip the voxelisation / FSC measurement")
    ap.add_argument("--no-batched", dest="batched", action="store_false",
                    help="skip the uneven-batching measurement (8 mixtures in one launch)")
    ap.add_argument("--no-pose-sweep", dest="pose_sweep", action="store_false",
                    help="skip the extra refinement configurations of the pose leg")
    ap.add_argument("--no-small", dest="small", action="store_false",
                    help="skip the N=20,000 (256 x 128^2) and N=1,000 (16 x 64^2) workloads")
    ap.add_argument("--no-probe", dest="probe", action="store_false",
                    help="skip the chip-rate probes (VALU, exp, LDS, BF16 MFMA, copy; ~0.2 s)")
    ap.add_argument("--only-small", action="store_true",
                    help="run only the N=20,000 and N=1,000 workloads (counter profiling)")
    ap.add_argument("--pose-train", type=int, default=200000)
    ap.add_argument("--pose-epochs", type=int, default=12)
    ap.add_argument("--pose-test", type=int, default=8192)
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "the benchmark runs on one GPU; --gpus must be 1 "
                          "(multi-GPU data parallelism is a design, not implemented)"}))
        sys.exit(2)
    if args.only_small:
        print(json.dumps({k: run_small(k, args.steps, args.warmup, args.cpu_images)
                          for k in ("c2", "c1")}))
        return
    cpu = None
    if args.cpu_images > 0 and int(os.environ.get("RANK", "0")) == 0:
        cpu = cpu_baseline(args.cpu_images)
        print(f"[bench] cpu oracle: {cpu['value']:.4f} images/s on {cpu['cores']} cores",
              file=sys.stderr, flush=True)
    args.rates = None
    if args.probe:
        # the chip's rates measured on this GPU, beside the published peaks
        # the rooflines use (FP32 VALU issue, v_exp_f32, LDS, BF16 MFMA, copy)
        from paper_2508_04929_amd import probe
        args.rates = probe.measure()
    res = run(args)
    res["cpu_baseline"] = cpu
    if args.rates:
        res["measured_rates"] = r = args.rates
        print(f"[bench] measured: VALU {r['fma']['per_cu_per_cycle']:.2f} wave64 instr/CU/cycle "
              f"at {r['fma']['clock_ghz']:.2f} GHz, LDS {r['lds']['bytes_per_cu_per_cycle']:.0f} "
              f"B/CU/cycle, BF16 MFMA {r['mfma']['tflops_bf16']:.0f} TFLOP/s, copy "
              f"{r['copy']['gb_per_s']:.0f} GB/s", file=sys.stderr, flush=True)
    if args.small:
        for k in ("c2", "c1"):
            res[k] = run_small(k, cpu_images=args.cpu_images)
            print(f"[bench] {k}: {res[k]['images_per_s']:.0f} images/s", file=sys.stderr,
                  flush=True)
    if args.trainer:
        res["trainer"] = run_trainer()
        res["densify"] = run_densify()
        res["reconstruction"] = run_reconstruction()
        r = res["reconstruction"]
        print(f"[bench] reconstruction: {r['seconds']:.1f} s, FSC resolution "
              f"{r['fsc_resolution_A_initial']:.1f} -> {r['fsc_resolution_A']:.1f} A", file=sys.stderr,
              flush=True)
    if args.volume:
        res["volume"] = run_volume()
        print(f"[bench] volume: voxelise {res['volume']['voxelize_ms']:.2f} ms, "
              f"FSC {res['volume']['fsc_ms']:.2f} ms", file=sys.stderr, flush=True)
    if args.batched:
        res["batched"] = run_batched()
        print(f"[bench] batched: {res['batched']['batched']['images_per_s']:.0f} images/s "
              f"(separate calls {res['batched']['separate']['images_per_s']:.0f})",
              file=sys.stderr, flush=True)
    if args.pose:
        from paper_2508_04929_amd import binding, pose
        log = lambda m: print(f"[pose] {m}", file=sys.stderr, flush=True)
        # the default refinement (coarse 6 directions x 2 angles, fine 4 x 2) and,
        # with the same network, two configurations with more candidates
        r = pose.run_c5(binding.library(), n_train=args.pose_train, epochs=args.pose_epochs,
                        n_test=args.pose_test, log=log,
                        stage_sweep=(((0, 5, 3), (1, 5, 3)), ((0, 5, 2), (1, 5, 3)))
                        if args.pose_sweep else ())
        res["pose"] = {
            "workload": ("learned pose proposal: N=20,000 mixture, D=128, p=1.5 A, SNR -20 dB, "
                         "CTF; network trained on %d renders x %d epochs; %d held-out particles; "
                         "grid search = 4,608 rotations x 25 shifts; each path timed in batches "
                         "of 2,048 / 4,096 / 8,192 particles, reported at its fastest" % (r["n_train"],
                                                                      r["training"]["epochs"],
                                                                      r["n_test"])),
            "speedup_vs_grid_search": r["speedup_vs_grid_search"],
            "reaches_grid_search_error": r["reaches_grid_search_error"],
            "speedup_same_batch": r.get("speedup_same_batch"),
            "learned_fallback": r.get("learned_fallback"),
            "grid_search": r["grid_search"], "learned": r["learned"],
            "untrained": r["untrained"], "training": r["training"],
            "literal_grid_search_images_per_s": r.get("literal_grid_search_images_per_s"),
            "speedup_vs_literal_grid_search": r.get("speedup_vs_literal_grid_search"),
            "stage_sweep": r.get("stage_sweep"),
            "bank_build_s": r["bank_build_s"], "bank_sizes": r["bank_sizes"]}
    print(json.dumps(res))


if __name__ == "__main__":
    main()
