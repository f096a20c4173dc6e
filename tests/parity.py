"""Comparison helpers of the GPU parity tests (host only, no method arithmetic).

Every comparison states two bars: the relative L1 error over the compared
cells (paper §4.1's e1 norm made relative) and a per-element bound,
max |got - ref| <= cell_bar * max |ref|, so that a wrong value confined to a
few cells (one tile on the wrong path, one node in the wrong cell) cannot
hide inside an aggregate norm.
"""
import numpy as np

# Per-element bars (relative to max |ref|) beside each precision's rel-L1 bar.
# FP64: rounding of a few dozen operations amplified by at most the 20x cell
# size ratio of the workloads, ~1e-14; the bar leaves three orders of margin
# below any wrong term (>= 1e-8 for the smallest perturbations tested).
CELL_F64 = 1e-11
# FP32 forward, one to five steps: the stencil's FP32 weights and sums give
# a few units of 2^-24 per step, up to 20x more in a cell 20x smaller than its
# source cell; 2e-5 bounds that (the tests print the measured maxima).
CELL_F32 = 2e-5
# FP32 adjoints: the transposed stencil sums the FP32 weights of every node
# that reads a cell (about 2p + 2 of them) into each gradient entry, whose
# inputs are N(0, 1) draws, so single entries cancel more than the forward's
# cell values do: 1e-4 of max |ref| (the rel-L1 bar is 1e-5).
CELL_F32_ADJ = 1e-4


def rel_l1(a, b, w=None):
    a = np.asarray(a, dtype=np.float64).reshape(-1)
    b = np.asarray(b, dtype=np.float64).reshape(-1)
    if w is None:
        return float(np.sum(np.abs(a - b)) / np.sum(np.abs(b)))
    w = np.asarray(w, dtype=np.float64).reshape(-1)
    return float(np.sum(np.abs(a - b) * w) / np.sum(np.abs(b) * w))


def max_cell(a, b):
    """max |a - b| / max |b|."""
    a = np.asarray(a, dtype=np.float64).reshape(-1)
    b = np.asarray(b, dtype=np.float64).reshape(-1)
    return float(np.max(np.abs(a - b)) / np.max(np.abs(b)))


def assert_parity(got, ref, rel_bar, cell_bar, what=""):
    """Both bars; returns (rel-L1, per-cell) for printing."""
    e1, ec = rel_l1(got, ref), max_cell(got, ref)
    assert e1 <= rel_bar, f"{what}: rel-L1 {e1:.3e} > {rel_bar:.1e}"
    assert ec <= cell_bar, f"{what}: max cell error {ec:.3e} of max|ref| > {cell_bar:.1e}"
    return e1, ec
