"""Shared test helpers: oracle references and GPU runs of the same seeded inputs."""
import numpy as np

import oracle as O
from paper_1309_5994_amd import workloads as W


def oracle_setup(wl):
    c = O.make_contour(wl.n_real, wl.n_imag, wl.dt, wl.beta, wl.t_min)
    eps = O.site_levels(wl.V, wl.U, wl.mu)
    S = np.stack([O.atomic_gf(e, wl.U, c) for e in eps])
    return c, S


def oracle_dense(wl):
    c, S = oracle_setup(wl)
    D = O.hopping_operator_dense(wl.Lx, wl.Ly, wl.periodic, wl.J, c)
    G = O.dyson_dense(S, D)
    return c, S, G


def dense_columns(G, n_r, n_t, sources):
    """[N_r, N_t, n_src * N_t] column layout of the library from a dense G."""
    cols = np.concatenate([G[:, j * n_t:(j + 1) * n_t] for j in sources], axis=1)
    return cols.reshape(n_r, n_t, len(sources) * n_t)


def rel_maxnorm(a, b):
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


def gpu_inputs(wl, device):
    import torch
    from paper_1309_5994_amd import scdyson as B
    prob = B.problem_from_workload(wl)
    V = torch.tensor(wl.V, dtype=torch.float64, device=device)
    U = torch.tensor(wl.U, dtype=torch.float64, device=device)
    J = torch.tensor(wl.J, dtype=torch.float64, device=device)
    return prob, V, U, J
