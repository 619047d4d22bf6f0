"""Algorithmic work of the stepping kernel (bytes and flops that one field evaluation must move
or compute at minimum), used to turn measured kernel times into roofline fractions.

Per mesh group with N nodes, nnz pattern entries, R instances, p bytes per real:
  demag operator S         p N^2                         (read once per evaluation; p N (N+1) / 2
                                                          when only its upper triangle is read;
                                                          p = 2 for the FP16 tiles)
  CSR pattern + values     nnz (8 + 7 p)                 (col twice, K and D in phase A, DT in C)
  node constants           N (12 + 2 p)                  (rowptr, layer, partner, V, aif)
  per-instance vectors     R N p * 35.5                  (stage input twice, yex, b, u, the
                                                          previous stage slopes on average,
                                                          m, the new slope and next input)
Flops per evaluation: 2 N^2 R (demag) + nnz R 14 (SpMVs) + N R ~90 (pointwise field + LLG).
"""
from __future__ import annotations

MI355X_HBM_GBS = 8000.0          # published HBM3E bandwidth
MI355X_FP32_TFLOPS = 157.3
MI355X_FP64_TFLOPS = 78.6
MI355X_BF16_TFLOPS = 2500.0


def eval_bytes(N: int, nnz: int, R: int, p: int, symmetric: bool = False, ps: int | None = None) -> float:
    """ps: bytes per stored entry of S when it differs from p (FP16 tiles: 2)."""
    ps = p if ps is None else ps
    s_bytes = ps * N * (N + 1) / 2 if symmetric else ps * N * N
    return s_bytes + nnz * (8 + 7 * p) + N * (12 + 2 * p) + R * N * p * 35.5


def eval_flops(N: int, nnz: int, R: int) -> float:
    return 2.0 * N * N * R + 14.0 * nnz * R + 90.0 * N * R
