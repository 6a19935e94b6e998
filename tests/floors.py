"""Bars of the reduced-precision network kernels against the FP64 oracle.

A BF16 (or E4M3) kernel cannot match FP64 exactly.  How far it may deviate is
measured on the CPU by the FP64 network oracle with the factors of each product
rounded as the kernels round them (oracle.ndf_net.Operands), which isolates the
error that rounding alone causes.  A GPU result must stay within FLOOR_FACTOR
times that emulated error (relative L2 per output vector or gradient tensor,
plus FLOOR_SLACK where the floor is near zero) and its largest element error
within MAX_FACTOR times the emulation's largest.  On the MI355X the kernels'
relative errors come out at 0.99-1.01 times the emulated ones (230 comparisons:
forward, adjoint per tensor, BF16 and FP8 inference, positions, hash grids) and
their largest element errors at 0.94-1.34 times.
"""
import sys

import numpy as np

from oracle import ndf_net as nn

FLOOR_FACTOR = 1.25  # GPU relative L2 error against the emulated rounding floor
FLOOR_SLACK = 1e-3   # absolute slack on relative errors whose floor is near zero
MAX_FACTOR = 2.0     # largest element error against the emulation's largest

TRAIN_OPS = nn.Operands()                    # training kernels: bf16 operands
BF16_OPS = nn.bf16_inference_operands()      # inference: also bf16 latents


def fp8_ops(net):
    """Inference with layers 2-5 in E4M3 (static activation scales from the
    network's own calibration): the one-reference FP8 field."""
    return nn.fp8_inference_operands(net)


def fp8_decoder_ops(net):
    """BF16 encoder, decoder layers 4-5 in E4M3: FP8 fields of several references,
    decoded from the cached query latents."""
    return nn.fp8_decoder_operands(net)


def _log(*a):
    print(*a, file=sys.stderr, flush=True)


def check_floor(got, want, emul, what):
    """The GPU result `got` against the FP64 oracle `want`, held to the error that
    the oracle with the kernels' operand rounding (`emul`) shows."""
    got = np.asarray(got, dtype=np.float64)
    rms = np.sqrt(np.mean(want ** 2))
    nw = np.linalg.norm(want)
    rel = np.linalg.norm(got - want) / nw
    floor = np.linalg.norm(emul - want) / nw
    mx = np.max(np.abs(got - want))
    mx_e = np.max(np.abs(emul - want))
    _log(f"{what}: rms={rms:.3g} relL2={rel:.2e} floor={floor:.2e} "
         f"ratio={rel / max(floor, 1e-30):.2f} max|d|={mx:.3g} emulated max={mx_e:.3g}")
    assert rel <= FLOOR_FACTOR * floor + FLOOR_SLACK, what
    assert mx <= MAX_FACTOR * mx_e + FLOOR_SLACK * rms, what


def check_grad_floor(lay, g, g_o, g_e, what):
    """Every parameter tensor of the GPU gradient g against the FP64 gradient g_o,
    held to the emulated gradient g_e's error (flat vectors in the library layout)."""
    for name_t, _shape in lay.tensors():
        a = lay.view(g, name_t).ravel()
        b = lay.view(g_o, name_t).ravel()
        nb = np.linalg.norm(b)
        if nb == 0:
            assert np.all(a == 0), name_t
            continue
        rel = np.linalg.norm(a - b) / nb
        floor = np.linalg.norm(lay.view(g_e, name_t).ravel() - b) / nb
        _log(f"{what} {name_t}: relL2 {rel:.2e} floor {floor:.2e} "
             f"ratio {rel / max(floor, 1e-30):.2f}")
        assert rel <= FLOOR_FACTOR * floor + 2 * FLOOR_SLACK, (what, name_t)
