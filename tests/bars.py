"""Residual bars for solves whose basis is stored below FP64.

The solver stops when its Krylov-Schur residual estimate is below
tol * |theta|.  That estimate assumes the Krylov relation A V = V T + Q B
holds exactly, while a basis stored in FP32 (or BF16) carries it only to the
storage rounding: each stored column moves by up to u_s of its norm, which
moves A v by up to u_s ||A||.  So the explicit FP64 residual of a returned
pair can exceed tol * |theta| by about 2 u_s ||A|| (the expansion block and
the orthogonalised block are each rounded once), with ||A|| = |lambda_1|,
the largest eigenvalue in magnitude, for a symmetric matrix.
"""
import numpy as np
import torch

UNIT_ROUNDOFF = {torch.float64: 2.0 ** -53, torch.float32: 2.0 ** -24, torch.bfloat16: 2.0 ** -8}


def resid_bar(tol, evals, dtype, lam1=None):
    """Per-pair bar on ||A x - theta x|| / (|theta| ||x||) for storage `dtype`.

    lam1: |lambda_1| (defaults to the largest returned |theta|).
    """
    th = np.abs(np.asarray(evals, dtype=np.float64))
    a = th.max() if lam1 is None else float(lam1)
    return tol + 2.0 * UNIT_ROUNDOFF[dtype] * a / th
