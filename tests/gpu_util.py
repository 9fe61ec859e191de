"""Helpers shared by the GPU tests: host arrays -> device tensors, error norms."""
import numpy as np
import torch

from paper_2508_04929_amd import binding


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(x, dtype=np.float32)).cuda()


def host(t):
    return t.detach().cpu().numpy().astype(np.float64)


def mixture_args(g):
    return dict(means=dev(g.means), log_scales=dev(g.log_scales), quats=dev(g.quats),
                amps=dev(g.amps))


def view_args(v):
    return dict(rot=dev(v.rot), shift=dev(v.shift), D=v.D, pixel=v.pixel)


def ctf_arg(v):
    return binding.Ctf(defocus_u=dev(v.defocus_u), defocus_v=dev(v.defocus_v),
                       astig=dev(v.astig), phase=dev(v.phase), voltage_kv=v.voltage_kv,
                       cs_mm=v.cs_mm, amp_contrast=v.amp_contrast, bfactor=v.bfactor,
                       pixel_a=v.pixel_a)


def normwise(got, ref):
    """max |got - ref| / max |ref| (per-image or per-group normwise error)."""
    got = np.asarray(got, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    den = np.abs(ref).max()
    return float(np.abs(got - ref).max() / den) if den > 0 else float(np.abs(got).max())


def per_image_normwise(got, ref):
    return max(normwise(got[b], ref[b]) for b in range(ref.shape[0]))


def announce(msg):
    print(f"[gpu-test] {msg}", flush=True)


def headline_options(lib, m, rot, shift, D, pixel, observed, ctf):
    """Launch options of the headline step as the bench chooses them: the
    library's autotuner on the step's own problem (mean reduction)."""
    pr = lib.make_problem(m["means"], m["log_scales"], m["quats"], m["amps"], rot, shift, D, pixel,
                          observed, ctf=ctf, reduction="mean")
    lib.autotune([pr], reps=3)
    return pr.options
