"""Test-side helpers: device transfer, column sampling, and an emulation of the
low-precision operand formats (IEEE single, bfloat16, OCP E4M3 with one E8M0
power-of-two scale per 32 elements along the reduction dimension), written
from the format definitions, independently of the HIP kernels.  Used to check
each tier's GEMM path exactly up to its FP32 accumulation."""
from __future__ import annotations

import numpy as np

DEV = "cuda:0"
U64 = 2.0 ** -53
U32 = 2.0 ** -24


def to_dev(A, dtype=None):
    import torch
    dtype = dtype or torch.float64
    return torch.tensor(np.ascontiguousarray(A), dtype=dtype, device=DEV)


def to_np(T):
    return T.detach().to("cpu").double().numpy()


def sample_cols(n, k, seed=0):
    rng = np.random.default_rng(seed)
    cols = sorted(set([0, n - 1] + list(rng.choice(n, size=min(k, n), replace=False))))
    return cols


# ---------------------------------------------------------------- formats
def round_f32(x):
    return np.asarray(x, dtype=np.float64).astype(np.float32).astype(np.float64)


def round_bf16(x):
    """Round-to-nearest-even of float32 values to bfloat16 (as float64)."""
    b = np.asarray(x, dtype=np.float32).view(np.uint32).astype(np.uint64)
    b = ((b + 0x7FFF + ((b >> 16) & 1)) >> 16) << 16
    return b.astype(np.uint32).view(np.float32).astype(np.float64)


def round_e4m3(x):
    """Round-to-nearest-even onto the OCP E4M3 grid: 3 fraction bits, minimum
    normal exponent -6, subnormal spacing 2^-9, largest finite 448."""
    x = np.asarray(x, dtype=np.float64)
    ax = np.abs(x)
    e = np.floor(np.log2(np.where(ax > 0, ax, 1.0)))
    e = np.maximum(e, -6.0)
    ulp = np.exp2(e - 3)
    q = np.round(x / ulp) * ulp
    return np.clip(q, -448.0, 448.0)


def mx_e4m3(M, axis):
    """E4M3 with a power-of-two scale per 32 consecutive elements along `axis`.
    Scale exponent: frexp exponent of the block's max |x| minus 8 (so the scaled
    block max lies in [128, 256)); zero blocks use scale 1."""
    M = np.asarray(M, dtype=np.float64)
    X = np.moveaxis(M, axis, -1)
    n = X.shape[-1]
    pad = (-n) % 32
    Xp = np.concatenate([X, np.zeros(X.shape[:-1] + (pad,))], axis=-1)
    blocks = Xp.reshape(X.shape[:-1] + (-1, 32))
    amax = np.max(np.abs(blocks.astype(np.float32)), axis=-1).astype(np.float64)
    _, ex = np.frexp(amax)
    sexp = np.clip(ex - 8, -127, 127)
    sexp = np.where(amax > 0, sexp, 0)
    scale = np.exp2(sexp)[..., None]
    q = round_e4m3(blocks / scale) * scale
    q = q.reshape(Xp.shape)[..., :n]
    return np.moveaxis(q, -1, axis)


def quantize_operand(M, tier, side):
    """The operand as the tier's GEMM sees it.  `side` is 'A' (left operand:
    blocks run along each row) or 'B' (right operand: along each column).
    Values first pass through float32, as in the kernels."""
    if tier == 0:
        return np.asarray(M, dtype=np.float64)
    M32 = round_f32(M)
    if tier == 1:
        return M32
    if tier == 2:
        return round_bf16(M32)
    return mx_e4m3(M32, axis=1 if side == "A" else 0)


def relerr_cols(P, ref_hi, ref_lo):
    D = (np.asarray(P) - ref_hi) - ref_lo
    return float(np.max(np.sum(np.abs(D), axis=0)) / np.max(np.sum(np.abs(ref_hi), axis=0)))
