"""Debug-check mode (CS_ERR_NONFINITE) through the C-ABI.

The non-finite values are planted from the host in the inputs (or forced
into the outputs by an amplitude that overflows FP32 in the splat); every
kernel still runs to completion, the call then reports the status.
"""
import numpy as np
import pytest
import torch

from paper_2508_04929_amd import binding, inputs

from gpu_util import announce, ctf_arg, dev, mixture_args, view_args

pytestmark = pytest.mark.gpu


def _case(seed=0):
    rng = np.random.default_rng(seed)
    g = inputs.mixture_anisotropic(rng, 300, 15.0)
    v = inputs.views(rng, 3, 48, 1.5)
    Y = (1e-3 * rng.standard_normal((3, 48, 48))).astype(np.float32)
    return g, v, Y


def test_nonfinite_inputs_and_outputs_are_reported(gpu_lib):
    g, v, Y = _case()
    announce("debug checks: clean call, NaN input, infinite output")
    D = torch.device("cuda", 0)
    m, va = mixture_args(g), view_args(v)
    try:
        gpu_lib.set_debug_checks(D, True)
        gpu_lib.loss_and_grad(**m, **va, observed=dev(Y), ctf=ctf_arg(v))   # clean: no error
        gpu_lib.render(**m, **va, ctf=ctf_arg(v))
        bad = dict(m)
        bad["means"] = m["means"].clone()
        bad["means"][7, 1] = float("nan")
        with pytest.raises(binding.NonFiniteError, match="input"):
            gpu_lib.loss_and_grad(**bad, **va, observed=dev(Y), ctf=ctf_arg(v))
        with pytest.raises(binding.NonFiniteError, match="input"):
            gpu_lib.render(**bad, **va)
        Yb = dev(Y)
        Yb[1, 3, 4] = float("inf")
        with pytest.raises(binding.NonFiniteError, match="input"):
            gpu_lib.loss_and_grad(**m, **va, observed=Yb, ctf=ctf_arg(v))
        with pytest.raises(binding.NonFiniteError, match="input"):
            gpu_lib.render_backward(**m, **va, d_images=Yb)
        # finite inputs, an overflowing output: with amplitudes of 1e30 the
        # images are about 1e29 and the squared error exceeds the FP32 range
        huge = dict(m)
        huge["amps"] = torch.full_like(m["amps"], 1e30)
        with pytest.raises(binding.NonFiniteError, match="output"):
            gpu_lib.loss_and_grad(**huge, **va, observed=dev(Y), ctf=ctf_arg(v))
        # batched call
        probs = [gpu_lib.make_problem(**m, **va, observed=dev(Y), ctf=ctf_arg(v)),
                 gpu_lib.make_problem(**bad, **va, observed=dev(Y), ctf=ctf_arg(v))]
        with pytest.raises(binding.NonFiniteError):
            gpu_lib.loss_and_grad_multi(probs, use_graph=False)
    finally:
        gpu_lib.set_debug_checks(D, False)
    # without debug checks the same call returns normally (no scan, no status)
    gpu_lib.loss_and_grad(**bad, **va, observed=dev(Y), ctf=ctf_arg(v))
    torch.cuda.synchronize()
