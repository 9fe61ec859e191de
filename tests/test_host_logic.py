"""Host-side library logic that runs without a GPU.

`cs_pose_grid` is plain host code (HEALPix pixel centres and the view
rotations): it is checked here against the independent oracle grid, and the
argument checks of the entry points that fail before touching a device.
"""
import ctypes
import os

import numpy as np
import pytest

from oracle import pose as o_pose

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_2508_04929_amd", "libcryosplat.so")
pytestmark = pytest.mark.skipif(not os.path.exists(LIB), reason="libcryosplat.so not built")


@pytest.fixture(scope="module")
def lib():
    from paper_2508_04929_amd import binding
    return binding.Library(binding.load_library())


@pytest.mark.parametrize("nside,n_psi", [(1, 1), (1, 8), (2, 12), (4, 24), (8, 48)])
def test_pose_grid_matches_oracle(lib, nside, n_psi):
    got = lib.pose_grid(nside, n_psi)
    assert got.shape == (12 * nside * nside * n_psi, 3, 3)
    np.testing.assert_allclose(got, o_pose.grid(nside, n_psi), atol=2e-6)


def test_pose_grid_count_query_and_bad_arguments(lib):
    n = ctypes.c_int64()
    assert lib.lib.cs_pose_grid(4, 24, None, ctypes.byref(n)) == 0 and n.value == 4608
    for bad in ((0, 24), (4, 0), (2000, 1), (1, 5000)):
        assert lib.lib.cs_pose_grid(bad[0], bad[1], None, ctypes.byref(n)) == -1
    assert lib.lib.cs_pose_grid(1, 1, None, None) == -1


def test_null_context_arguments_are_rejected(lib):
    L = lib.lib
    assert L.cs_render(None, None, None, None, None, None, None) == -1
    assert L.cs_adam_step(None, None, None, None, None, 0, 1, 1e-3, 0.9, 0.999, 1e-8, None) == -1
    assert L.cs_cnn_forward(None, None, 1, None, None, None, None) == -1
    assert L.cs_pose_batch_load(None, None, None, 1, None, None, None) == -1
    assert L.cs_cnn_forward_std(None, None, 1, None, None, None, None) == -1
    assert L.cs_pose_grid_search(None, None, None, 1, 2, None, None, None, None, None) == -1
    assert L.cs_cnn_param_count(None) == -1 and L.cs_pose_bank_size(None) == -1
    assert L.cs_voxelize(None, None, 8, 1.0, 0.0, None, None) == -1
    assert L.cs_fsc(None, None, None, 8, None, None) == -1
    assert L.cs_fourier_shift(None, None, None, 1, 8, 1.0, 1.0, None, None) == -1
    assert L.cs_init_attributes(None, None, 1, None, None) == -1
    assert L.cs_train_sequential(None, None, None, None, 1, 1, 1, None, None, None, 0, None, 0, 0,
                                 1e-3, 0.9, 0.999, 1e-8, None, None) == -1
    assert L.cs_split_gaussians(None, None, None, None, 1, 1, 1, None, None, None, None) == -1


def test_flat_parameter_methods_reject_bad_lengths(lib):
    """The binding checks the flat layout (11 values per Gaussian) before any
    device call."""
    import torch
    bad = torch.zeros(12)
    with pytest.raises(ValueError):
        lib.split_gaussians(bad)
    with pytest.raises(ValueError):
        lib.train_sequential(bad, bad.clone(), bad.clone(), torch.zeros(1, 8, 8),
                             torch.eye(3)[None], 1 / 8, [0], 0, 1e-3)


def test_status_codes_map_to_exceptions():
    """The binding's error mapping, forced from the host with a stand-in
    library object: CS_ERR_NONFINITE raises NonFiniteError (a CryoSplatError),
    other negative codes CryoSplatError with the context's message."""
    from paper_2508_04929_amd import binding

    class Fake:
        def cs_last_error(self, ctx):
            return b"debug checks: NaN or infinity in an input array"

    L = binding.Library(Fake())
    L._check(None, 0, "ok call")
    with pytest.raises(binding.NonFiniteError, match="input array"):
        L._check(None, binding.CS_ERR_NONFINITE, "cs_render")
    with pytest.raises(binding.CryoSplatError) as e:
        L._check(None, binding.CS_ERR_INVALID_ARG, "cs_render")
    assert not isinstance(e.value, binding.NonFiniteError)
    # the header's enum carries the same value
    src = open(os.path.join(ROOT, "include", "cryosplat.h")).read()
    assert "CS_ERR_NONFINITE = -5" in src


def test_debug_check_switch_rejects_null_context(lib):
    assert lib.lib.cs_set_debug_checks(None, 1) == -1
