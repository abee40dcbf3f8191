"""Write the oracle's expected values for the full-size workloads.

Calls only ``oracle/`` (and the seeded input generator).  For each workload it
solves G = (I - S D)^-1 S exactly for the seeded sample of source sites by
block-tridiagonal elimination in lattice rows, and stores, per source:
occupancy n(t) and kinetic energy e_kin(t) on the forward grid, 1024 seeded
entries of the local block G(j, j), and 2048 seeded entries of the source's
columns (target site, row time, column time).  For the 12x12 workload it also stores n(t) and
e_kin(t) for every site (all columns solved).

    python tests/golden/make_golden.py 2 3 4 5      # writes tests/golden/cfg<k>.npz
"""
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle as O                                    # noqa: E402
from paper_1309_5994_amd import workloads as W        # noqa: E402

N_SAMPLES = 2048
N_LOCAL = 1024


def solve_sources(wl, c, S, sources):
    return O.dyson_columns_blocktri(S, wl.Lx, wl.Ly, wl.J, c, sources)


def summarise(wl, c, cols, sources, rng):
    n_t = c.n_t
    nbr = O.neighbours(wl.Lx, wl.Ly, wl.periodic)
    out = {}
    G_loc = np.stack([cols[j, :, s * n_t:(s + 1) * n_t] for s, j in enumerate(sources)])
    G_nn = np.zeros((len(sources), 4, n_t, n_t), dtype=complex)
    for s, j in enumerate(sources):
        for d in range(4):
            k = nbr[j, d]
            if k >= 0:
                G_nn[s, d] = cols[k, :, s * n_t:(s + 1) * n_t]
    out["n"] = O.occupancy(G_loc, c)
    out["ekin"] = O.kinetic_energy(G_nn, nbr[np.asarray(sources)], wl.J, c)
    la = rng.integers(0, n_t, size=(len(sources), N_LOCAL))
    lb = rng.integers(0, n_t, size=(len(sources), N_LOCAL))
    lv = np.stack([G_loc[s][la[s], lb[s]] for s in range(len(sources))])
    out["loc_a"], out["loc_b"], out["loc_re"], out["loc_im"] = la, lb, lv.real, lv.imag
    tgt = rng.integers(0, wl.n_r, size=(len(sources), N_SAMPLES))
    ra = rng.integers(0, n_t, size=(len(sources), N_SAMPLES))
    rb = rng.integers(0, n_t, size=(len(sources), N_SAMPLES))
    vals = np.zeros((len(sources), N_SAMPLES), dtype=complex)
    for s in range(len(sources)):
        vals[s] = cols[tgt[s], ra[s], s * n_t + rb[s]]
    out["sample_site"], out["sample_a"], out["sample_b"] = tgt, ra, rb
    out["sample_re"], out["sample_im"] = vals.real, vals.imag
    out["G_absmax"] = np.array([np.abs(cols).max()])
    return out


def make(k):
    wl = W.config(k)
    c = O.make_contour(wl.n_real, wl.n_imag, wl.dt, wl.beta, wl.t_min)
    eps = O.site_levels(wl.V, wl.U, wl.mu)
    S = np.stack([O.atomic_gf(e, wl.U, c) for e in eps])
    sources = W.sample_sources(wl)
    rng = np.random.default_rng(100 + k)
    t0 = time.time()
    cols = solve_sources(wl, c, S, sources)
    res = summarise(wl, c, cols, sources, rng)
    res["sources"] = np.asarray(sources, dtype=np.int64)
    print(f"cfg{k}: sampled sources solved in {time.time() - t0:.1f} s", flush=True)
    del cols
    if k == 4:
        t0 = time.time()
        n_all = np.zeros((wl.n_r, wl.n_real))
        e_all = np.zeros((wl.n_r, wl.n_real))
        nbr = O.neighbours(wl.Lx, wl.Ly, wl.periodic)
        chunk = 24
        for start in range(0, wl.n_r, chunk):
            src = list(range(start, min(wl.n_r, start + chunk)))
            cols = solve_sources(wl, c, S, src)
            n_t = c.n_t
            G_loc = np.stack([cols[j, :, s * n_t:(s + 1) * n_t] for s, j in enumerate(src)])
            G_nn = np.zeros((len(src), 4, n_t, n_t), dtype=complex)
            for s, j in enumerate(src):
                for d in range(4):
                    kk = nbr[j, d]
                    if kk >= 0:
                        G_nn[s, d] = cols[kk, :, s * n_t:(s + 1) * n_t]
            n_all[src] = O.occupancy(G_loc, c)
            e_all[src] = O.kinetic_energy(G_nn, nbr[src], wl.J, c)
        res["n_all"], res["ekin_all"] = n_all, e_all
        print(f"cfg{k}: all sites in {time.time() - t0:.1f} s", flush=True)
    np.savez_compressed(os.path.join(HERE, f"cfg{k}.npz"), **res)


if __name__ == "__main__":
    for arg in sys.argv[1:]:
        make(int(arg))
