"""The canonical FP32 squared distance the GPU kernels decide argmins with (oracle).

TEST INFRASTRUCTURE ONLY.  The paper does not fix a precision.  The kernels
define one FP32 distance as canonical and guarantee that every argmin they
return (centroid assignment, PQ code) is the argmin of this distance over the
candidate set, lowest index on equal values:

    acc = 0;  for i = 0 .. d-1:  t = x_i - c_i;  acc = acc + t * t

with every operation rounded to float32 (round to nearest even) and no fused
multiply-add.  This module evaluates that definition with NumPy float32
arithmetic, which rounds each elementwise operation exactly once, so integer
decisions of the oracle and the kernels can be compared bit for bit.

Pinned by: exact agreement with the float64 distance on dyadic inputs where
every float32 operation is exact, and a rounding bound against float64 on
random inputs (tests/test_oracle_lloyd.py).
"""
from __future__ import annotations

import numpy as np


def pairwise(X: np.ndarray, C: np.ndarray) -> np.ndarray:
    """float32[n, k]: canonical distance of every row of X to every row of C."""
    X = np.ascontiguousarray(X, dtype=np.float32)
    C = np.ascontiguousarray(C, dtype=np.float32)
    acc = np.zeros((X.shape[0], C.shape[0]), dtype=np.float32)
    for i in range(X.shape[1]):
        t = X[:, i, None] - C[None, :, i]
        acc += t * t
    return acc


def rowwise(X: np.ndarray, C: np.ndarray) -> np.ndarray:
    """float32[n]: canonical distance of row r of X to row r of C."""
    X = np.ascontiguousarray(X, dtype=np.float32)
    C = np.ascontiguousarray(C, dtype=np.float32)
    acc = np.zeros(X.shape[0], dtype=np.float32)
    for i in range(X.shape[1]):
        t = X[:, i] - C[:, i]
        acc += t * t
    return acc


def sqnorm(X: np.ndarray) -> np.ndarray:
    """float32[n]: canonical sum of squares of each row (sequential, unfused)."""
    X = np.ascontiguousarray(X, dtype=np.float32)
    acc = np.zeros(X.shape[0], dtype=np.float32)
    for i in range(X.shape[1]):
        acc += X[:, i] * X[:, i]
    return acc
