"""Failure paths of dyson_iterate, forced from the host so that every kernel
still exits normally: a sweep limit that is too small, a NaN planted in S by
the caller, and a hopping so large that the Dyson series diverges."""
import numpy as np
import pytest

from paper_1309_5994_amd import workloads as W
from helpers import gpu_inputs

pytestmark = pytest.mark.gpu


def _B():
    from paper_1309_5994_amd import scdyson as B
    return B


def test_not_converged_reports_stats(device):
    B = _B()
    wl = W.config(1)
    prob, V, U, J = gpu_inputs(wl, device)
    S = B.sigma_build(prob, V, U)
    with pytest.raises(B.ScdError) as ei:
        B.dyson_iterate(prob, S, J, list(range(16)), max_iter=2)
    assert ei.value.code == B.SCD_ENOTCONV
    assert ei.value.stats["sweeps_max"] == 2 and ei.value.stats["final_err"] > 1e-12


def test_nan_in_sigma_is_detected(device):
    B = _B()
    wl = W.config(1)
    prob, V, U, J = gpu_inputs(wl, device)
    S = B.sigma_build(prob, V, U)
    S[5, 3, 7] = complex(float("nan"), 0.0)
    with pytest.raises(B.ScdError) as ei:
        B.dyson_iterate(prob, S, J, list(range(16)), max_iter=50)
    assert ei.value.code == B.SCD_ENAN


def test_divergent_hopping_is_detected(device):
    import torch
    B = _B()
    wl = W.config(1)
    prob, V, U, J = gpu_inputs(wl, device)
    S = B.sigma_build(prob, V, U)
    J_big = torch.full_like(J, 3.0)
    with pytest.raises(B.ScdError) as ei:
        B.dyson_iterate(prob, S, J_big, list(range(16)), max_iter=200)
    assert ei.value.code in (B.SCD_EDIVERGED, B.SCD_ENAN)
