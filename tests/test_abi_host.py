"""Host-side checks of the C-ABI library that need no GPU: it loads, it exports
every function include/scdyson.h declares, and argument validation rejects bad
input before any HIP call (so these run on a machine without a GPU)."""
import ctypes

import numpy as np
import pytest

from paper_1309_5994_amd import scdyson as B


def test_library_exports_every_declared_function():
    L = B.lib()
    names = B.header_functions()
    assert {"sigma_build", "dyson_iterate", "local_observables", "scd_workspace_bytes",
            "scd_last_error"} <= set(names)
    for name in names:
        assert hasattr(L, name), name


def test_workspace_bytes_layout():
    p = B.problem(4, 4, 20, 10, 0.1, 5.0)
    n = B.workspace_bytes(p, 16, 16)
    # S operand (64x64 padded) + one 16 x 64 x 800 iterate (16 sources x 50 contour
    # columns, padded to the 32-column tile; red-black sweeps update it in place)
    assert n >= 16 * 64 * 64 * 16 + 16 * 64 * 800 * 16
    assert B.workspace_bytes(p, 16, 4) < n
    # A periodic lattice with an odd extent is not bipartite: Jacobi needs two iterates.
    q = B.problem(3, 4, 20, 10, 0.1, 5.0, periodic=True)
    assert B.workspace_bytes(q, 12, 12) >= 12 * 64 * 64 * 16 + 2 * 12 * 64 * 608 * 16
    # FP32 refinement: + complex64 operand, residual and correction
    assert B.workspace_bytes(p, 16, 16, 1) >= n + 16 * 64 * 64 * 8 + 2 * 16 * 64 * 800 * 8
    # BF16x3 refinement: four bf16 planes of the operand (hi/lo of Re and Im, K
    # padded to 64) instead of the complex64 one
    assert B.workspace_bytes(p, 16, 16, 2) >= n + 16 * 4 * 64 * 64 * 2 + 2 * 16 * 64 * 800 * 8


@pytest.mark.parametrize("kw,msg", [
    (dict(Lx=0), "lattice extent"),
    (dict(periodic=1, Lx=2), "periodic"),
    (dict(n_real=0), "n_real"),
    (dict(n_real=200), "contour"),
    (dict(dt=0.0), "dt"),
    (dict(beta=-1.0), "beta"),
])
def test_problem_validation(kw, msg):
    base = dict(Lx=4, Ly=4, periodic=0, n_real=20, n_imag=10, dt=0.1, beta=5.0, mu=0.0, t_min=0.0)
    base.update(kw)
    p = B.Problem(**base)
    out = ctypes.c_size_t(0)
    rc = B.lib().scd_workspace_bytes(ctypes.byref(p), 1, 1, 0, ctypes.byref(out))
    assert rc == B.SCD_EINVAL
    assert msg in B.last_error()


def test_dyson_iterate_rejects_bad_arguments_before_launch():
    L = B.lib()
    p = B.problem(3, 3, 5, 4, 0.1, 2.0)
    src = np.array([0, 9], dtype=np.int32)          # 9 is outside the 3x3 lattice
    fake = ctypes.c_void_p(0x1000)                   # never dereferenced: validation fails first
    st = B.Stats()
    rc = L.dyson_iterate(ctypes.byref(p), fake, fake, src.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                         2, 2, 0, 1e-12, 10, None, fake, None, fake, ctypes.c_size_t(1 << 40),
                         ctypes.byref(st), None)
    assert rc == B.SCD_EINVAL and "src[1]" in B.last_error()
    assert st.status == B.SCD_EINVAL
    rc = L.dyson_iterate(ctypes.byref(p), fake, fake, src.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                         1, 1, 0, 1e-12, 10, None, fake, None, fake, ctypes.c_size_t(16),
                         ctypes.byref(st), None)
    assert rc == B.SCD_ENOMEM
    rc = L.dyson_iterate(ctypes.byref(p), fake, fake, src.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                         1, 1, 7, 1e-12, 10, None, fake, None, fake, ctypes.c_size_t(1 << 40),
                         ctypes.byref(st), None)
    assert rc == B.SCD_EINVAL and "precision" in B.last_error()
    rc = L.dyson_iterate(ctypes.byref(p), fake, fake, src.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                         1, 1, 0, 0.0, 10, None, fake, None, fake, ctypes.c_size_t(1 << 40),
                         ctypes.byref(st), None)
    assert rc == B.SCD_EINVAL and "tol" in B.last_error()
    rc = L.dyson_iterate(ctypes.byref(p), fake, fake, src.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                         0, 1, 0, 1e-12, 10, None, fake, None, fake, ctypes.c_size_t(1 << 40),
                         ctypes.byref(st), None)
    assert rc == B.SCD_EINVAL and "n_src" in B.last_error()      # an empty source list


def test_sigma_build_and_observables_reject_nulls():
    L = B.lib()
    p = B.problem(2, 2, 3, 2, 0.1, 1.0)
    assert L.sigma_build(ctypes.byref(p), None, None, None, None) == B.SCD_EINVAL
    assert L.local_observables(ctypes.byref(p), None, None, None, 1, None, None, None) == B.SCD_EINVAL
    assert L.sigma_build(None, None, None, None, None) == B.SCD_EINVAL


def test_gmres_workspace_and_validation():
    p = B.problem(4, 4, 20, 10, 0.1, 5.0)
    # St + iterate + restart + 1 basis vectors (16 x 64 x 800 complex128 each)
    it = 16 * 64 * 800 * 16
    n = B.gmres_workspace_bytes(p, 16, 16, 4)
    assert n >= 16 * 64 * 64 * 16 + 6 * it
    assert B.gmres_workspace_bytes(p, 16, 16, 8) - n >= 4 * it
    out = ctypes.c_size_t(0)
    for bad in (0, 17):
        assert B.lib().scd_gmres_workspace_bytes(ctypes.byref(p), 16, 16, bad,
                                                 ctypes.byref(out)) == B.SCD_EINVAL
        assert "restart" in B.last_error()
    L = B.lib()
    src = np.array([0, 3], dtype=np.int32)
    fake = ctypes.c_void_p(0x1000)                   # never dereferenced
    st = B.Stats()
    args = lambda restart, tol, ws_bytes: (
        ctypes.byref(p), fake, fake, src.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), 2, 2,
        restart, tol, 10, None, fake, None, fake, ctypes.c_size_t(ws_bytes), ctypes.byref(st), None)
    assert L.dyson_gmres(*args(0, 1e-12, 1 << 40)) == B.SCD_EINVAL and "restart" in B.last_error()
    assert L.dyson_gmres(*args(4, -1.0, 1 << 40)) == B.SCD_EINVAL and "tol" in B.last_error()
    assert L.dyson_gmres(*args(4, 1e-12, 64)) == B.SCD_ENOMEM
    assert st.status == B.SCD_ENOMEM


def test_sym_workspace_counts_orbit_representatives():
    # 16x16 lattice, all sources: C4v orbits of 8 (4 on the diagonals) -> 36 representatives
    p = B.problem(16, 16, 64, 16, 0.1, 10.0)
    every = list(range(256))
    full = B.workspace_bytes(p, 256, 256)
    red = B.sym_workspace_bytes(p, every, 256)
    assert red < full / 6
    assert red >= B.workspace_bytes(p, 36, 36)
    assert red < B.workspace_bytes(p, 37, 37)
    # 3x5 (C2v): orbits of 4, 2 on the middle row/column, 1 at the centre -> 6
    q = B.problem(3, 5, 10, 4, 0.1, 2.0)
    assert B.workspace_bytes(q, 6, 6) <= B.sym_workspace_bytes(q, list(range(15)), 15) \
        < B.workspace_bytes(q, 7, 7)


def test_extrapolation_matches_the_oracle_and_validates():
    import oracle as O
    rng = np.random.default_rng(11)
    vals = rng.standard_normal((3, 7))
    for dts in ([0.1, 0.05, 0.025], [0.2, 0.1]):
        got = B.extrapolate_dt(dts, vals[:len(dts)])
        ref = O.extrapolate_dt(dts, vals[:len(dts)])
        assert np.abs(got - ref).max() <= 1e-14 * max(1.0, np.abs(ref).max())
    with pytest.raises(B.ScdError):
        B.extrapolate_dt([0.1, 0.1], vals[:2])
    with pytest.raises(B.ScdError):
        B.extrapolate_dt([0.1], vals[:1])
