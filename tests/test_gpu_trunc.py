"""GPU parity of the far-block truncation (dyson_iterate_trunc) through the
C-ABI: the columns of each source solved on the sites within a lattice
distance of it, against the oracle's restricted dense solve (1e-12 relative);
a radius covering the lattice reproduces dyson_iterate bit for bit."""
import numpy as np
import pytest

import oracle as O
from paper_1309_5994_amd import workloads as W
from helpers import oracle_setup, rel_maxnorm, gpu_inputs

pytestmark = pytest.mark.gpu


def _np(t):
    return t.detach().cpu().numpy()


@pytest.mark.parametrize("wl", [W.custom(4, 5, 7, 5, J0=0.1, seed=4),
                                W.custom(4, 4, 6, 4, J0=0.12, periodic=True, seed=6)],
                         ids=["4x5", "periodic4x4"])
@pytest.mark.parametrize("radius", [0, 1, 2, 4])
def test_truncated_columns_match_oracle(wl, radius, device):
    from paper_1309_5994_amd import scdyson as B
    c, S_ref = oracle_setup(wl)
    D = O.hopping_operator_dense(wl.Lx, wl.Ly, wl.periodic, wl.J, c)
    sources = list(range(wl.n_r))[::-1]
    ref = O.dyson_columns_truncated(S_ref, D, wl.Lx, wl.Ly, wl.periodic, sources, radius)
    prob, V, U, J = gpu_inputs(wl, device)
    S = B.sigma_build(prob, V, U)
    r = B.dyson_iterate_trunc(prob, S, J, sources, radius, block_sites=7, tol=1e-14,
                              max_iter=400, want_cols=True)
    assert rel_maxnorm(_np(r["G_cols"]), ref) <= 1e-12
    got = _np(r["G_cols"])
    for s, j in enumerate(sources):
        far = [i for i in range(wl.n_r) if O.lattice_distance(i, j, wl.Lx, wl.Ly, wl.periodic) > radius]
        if far:
            assert np.abs(got[far][:, :, s * c.n_t:(s + 1) * c.n_t]).max() == 0.0


def test_full_radius_is_bitwise_the_untruncated_solve(device):
    from paper_1309_5994_amd import scdyson as B
    import torch
    wl = W.custom(4, 4, 8, 6, J0=0.1, seed=21)
    prob, V, U, J = gpu_inputs(wl, device)
    S = B.sigma_build(prob, V, U)
    src = list(range(16))
    a = B.dyson_iterate(prob, S, J, src, block_sites=7, tol=1e-13, want_cols=True)
    b = B.dyson_iterate_trunc(prob, S, J, src, wl.Lx + wl.Ly, block_sites=7, tol=1e-13,
                              want_cols=True)
    assert torch.equal(a["G_cols"], b["G_cols"])
