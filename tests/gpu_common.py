"""Helpers shared by the GPU parity tests (not collected as tests)."""

import numpy as np
import pytest
import torch

import synth
from oracle.solve import fixed_point, residual_momentum
from oracle.system import assemble

requires_gpu = pytest.mark.skipif(not torch.cuda.is_available(), reason="needs an MI355X")

DEV = "cuda:0"


def announce(*args):
    print("[gpu-case]", *args, flush=True)


def np_(t):
    return t.detach().cpu().numpy()


def oracle_for(w):
    mask = np.ones(tuple(reversed(w.dims)), np.uint8) if w.mask is None else np_(w.mask)
    sys_ = assemble(mask, w.spacing)
    return sys_


def rel_maxabs(got, ref):
    return float(np.abs(got - ref).max() / np.sqrt(np.mean(ref**2)))


def fp64_cases():
    """Grids whose fixed point FP64 can resolve to 1e-11 of RMS(P): the
    attainable agreement is about machine epsilon times the conditioning of
    the fixed-point operator, which grows with the side length."""
    return [
        ("2d_aniso_masked_45x37", lambda: synth.random_small(41, 2, (45, 37), mask_frac=0.1)),
        ("2d_iso_64x64", lambda: synth.random_small(12, 2, (64, 64), anisotropic=False, mask_frac=0.0)),
        ("3d_aniso_masked_24x17x13", lambda: synth.random_small(42, 3, (24, 17, 13), mask_frac=0.1)),
        ("3d_iso_masked_70x21x9", lambda: synth.random_small(43, 3, (70, 21, 9), anisotropic=False,
                                                             mask_frac=0.1)),
        ("3d_iso_unmasked_32x20x12", lambda: synth.random_small(45, 3, (32, 20, 12), anisotropic=False,
                                                                mask_frac=0.0)),
    ]


def fp32_cases():
    """Larger ragged grids: several strips along x, several march segments,
    masks and anisotropic spacing."""
    return [
        ("2d_aniso_masked_197x131", lambda: synth.random_small(11, 2, (197, 131), mask_frac=0.1)),
        ("3d_aniso_masked_70x37x29", lambda: synth.random_small(13, 3, (70, 37, 29), mask_frac=0.1)),
        ("3d_iso_masked_33x65x17", lambda: synth.random_small(14, 3, (33, 65, 17), anisotropic=False,
                                                              mask_frac=0.1)),
        ("3d_aniso_unmasked_48x24x20", lambda: synth.random_small(15, 3, (48, 24, 20), mask_frac=0.0)),
        ("2d_aniso_unmasked_132x90", lambda: synth.random_small(16, 2, (132, 90), mask_frac=0.0)),
    ]


def small_cases():
    return fp64_cases() + fp32_cases()
