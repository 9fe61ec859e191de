"""Chip-rate probes: the FP32 VALU issue rate, v_exp_f32, conflict-free LDS
reads, BF16 MFMA (16x16x32) and a device-memory copy, measured on this GPU
by the kernels of ``probe/probe.hip`` (``libcsprobe.so``, built by
``build.build``).  The benchmark reports them beside the rooflines, whose
peaks are the published figures; nothing in the renderer uses them."""
from __future__ import annotations

import ctypes
import os

import numpy as np
import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libcsprobe.so")
N_CU = 256

# per pass of each probe's loop and per wave
PER_PASS = {"fma": 32, "exp": 32, "lds": 32, "mfma": 16}
ITERS = {"fma": 20000, "exp": 5000, "lds": 2000, "mfma": 5000}


def load(path: str = LIB_PATH) -> ctypes.CDLL:
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is missing: build it with __graft_entry__.build()")
    lib = ctypes.CDLL(path)
    for name in ("csp_fma", "csp_exp", "csp_lds", "csp_mfma"):
        f = getattr(lib, name)
        f.restype = ctypes.c_double
        f.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int, ctypes.c_int]
    lib.csp_copy.restype = ctypes.c_double
    lib.csp_copy.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64, ctypes.c_int]
    lib.csp_wall_clock_khz.restype = ctypes.c_int
    lib.csp_wall_clock_khz.argtypes = [ctypes.c_int]
    return lib


def measure(device: int = 0, blocks: int = 8 * N_CU, copy_mib: int = 1024) -> dict:
    """Rates of this GPU: each probe is launched once to warm up and once
    timed with HIP events; the shader clock comes from per-block stamps of
    the shader and constant clocks around the timed loop."""
    lib = load()
    torch.cuda.synchronize(device)
    dev = torch.device("cuda", device)
    out = torch.empty(blocks * 256, device=dev, dtype=torch.float32)
    clk = torch.zeros(blocks * 4, device=dev, dtype=torch.int64)
    khz = lib.csp_wall_clock_khz(device)
    waves = blocks * 4
    res = {"blocks": blocks, "waves": waves, "wall_clock_khz": khz}
    for name, iters in ITERS.items():
        fn = getattr(lib, f"csp_{name}")
        if fn(out.data_ptr(), clk.data_ptr(), blocks, max(1, iters // 10)) < 0:
            raise RuntimeError(f"probe {name} failed")
        ms = fn(out.data_ptr(), clk.data_ptr(), blocks, iters)
        if ms <= 0:
            raise RuntimeError(f"probe {name} failed")
        st = clk.view(blocks, 4).cpu().numpy().astype(np.float64)
        ghz = float(np.median((st[:, 1] - st[:, 0]) / ((st[:, 3] - st[:, 2]) / (khz * 1e3)) / 1e9))
        ops = PER_PASS[name] * iters * waves / (ms * 1e-3)  # wave instructions per second
        res[name] = {"ms": ms, "wave_instr_per_s": ops, "clock_ghz": ghz,
                     "per_cu_per_cycle": ops / (N_CU * ghz * 1e9)}
    res["fma"]["tflops_fp32"] = res["fma"]["wave_instr_per_s"] * 64 * 2 / 1e12
    res["exp"]["exp_per_s"] = res["exp"]["wave_instr_per_s"] * 64
    res["lds"]["bytes_per_cu_per_cycle"] = res["lds"]["per_cu_per_cycle"] * 64 * 16
    res["mfma"]["tflops_bf16"] = res["mfma"]["wave_instr_per_s"] * 2 * 16 * 16 * 32 / 1e12
    n4 = copy_mib * (1 << 20) // 16
    src = torch.empty(n4 * 4, device=dev, dtype=torch.float32).fill_(1.0)
    dst = torch.empty_like(src)
    times = []
    for _ in range(6):
        ms = lib.csp_copy(src.data_ptr(), dst.data_ptr(), n4, 65536)
        if ms <= 0:
            raise RuntimeError("probe copy failed")
        times.append(ms)
    ms = float(np.median(times[1:]))
    res["copy"] = {"mib": copy_mib, "ms": ms, "gb_per_s": 2 * n4 * 16 / (ms * 1e-3) / 1e9}
    del src, dst
    torch.cuda.synchronize(device)
    return res
