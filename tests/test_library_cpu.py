"""CPU-side checks of the C ABI library: it loads, exports every entry
point declared in include/pqmc.h, and validates problems (no GPU calls)."""
import ctypes
import os
import re

import numpy as np
import pytest

import synth
from paper_2506_09611_amd import binding

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _header_functions():
    src = open(os.path.join(ROOT, "include", "pqmc.h")).read()
    return sorted(set(re.findall(r"\b(pqmc_[a-z_]+)\s*\(", src)))


def test_header_declares_binding_symbols():
    assert _header_functions() == sorted(binding.EXPORTED_SYMBOLS)


def test_library_exports_every_symbol():
    lib = binding.load_library()
    for name in _header_functions():
        assert hasattr(lib, name), name


def _problem(U=4.0, n_slices=20, stab=5, n_up=5, hop=None):
    p = synth.make_problem(4, 5, 5, 4.0, n_slices=20, stab_every=5, perturb=1e-3, seed=3)
    H = np.ascontiguousarray(p.hopping if hop is None else hop)
    Pu = np.ascontiguousarray(p.trial_up[:, :n_up])
    keep = (H, Pu)
    pr = binding.Problem(16, n_up, 5, binding._dptr(H), binding._dptr(Pu),
                         binding._dptr(np.ascontiguousarray(p.trial_dn)), U, 0.05, n_slices,
                         stab, 7, 0)
    pr._keep = keep + (np.ascontiguousarray(p.trial_dn),)
    pr.trial_dn = binding._dptr(pr._keep[2])
    return pr


def _ws(pr, opts):
    lib = binding.load_library()
    n = ctypes.c_size_t(0)
    st = lib.pqmc_workspace_bytes(ctypes.byref(pr), ctypes.byref(opts), ctypes.byref(n))
    return st, n.value


def test_workspace_bytes_valid_problem():
    st, n = _ws(_problem(), binding.UpdateOpts(1, 16, 8, 0))
    assert st == 0 and n > 0
    st2, n2 = _ws(_problem(), binding.UpdateOpts(1, 16, 8, binding.FLAG_LOG))
    assert st2 == 0 and n2 > n      # the decision log is sized in


def test_workspace_bytes_negative_u():
    """U < 0 is the one-sector complex model: valid with equal sectors, and
    rejected with unequal ones (n_up != n_dn) or options it does not run."""
    st, n = _ws(_problem(U=-4.0), binding.UpdateOpts(1, 16, 8, 0))
    assert st == 0 and n > 0
    assert _ws(_problem(U=-4.0, n_up=4), binding.UpdateOpts(1, 16, 8, 0))[0] == -1
    assert _ws(_problem(U=-4.0), binding.UpdateOpts(1, 65, 8, 0))[0] == -1
    assert _ws(_problem(U=-4.0), binding.UpdateOpts(3, 1, 1, 0))[0] == -1
    assert _ws(_problem(U=-4.0), binding.UpdateOpts(1, 16, 8, binding.FLAG_FP32))[0] == -1


@pytest.mark.parametrize("bad", [
    dict(stab=7), dict(n_slices=0), dict(n_up=0),
    dict(hop=np.full((16, 16), np.nan)),
])
def test_workspace_bytes_rejects(bad):
    st, _ = _ws(_problem(**bad), binding.UpdateOpts(0, 1, 1, 0))
    assert st == -1
    assert binding.load_library().pqmc_last_error().decode()


@pytest.mark.parametrize("opts", [binding.UpdateOpts(0, 0, 1, 0), binding.UpdateOpts(1, 129, 1, 0),
                                  binding.UpdateOpts(2, 1, 65, 0), binding.UpdateOpts(5, 1, 1, 0),
                                  binding.UpdateOpts(1, 16, 1, 0, -1)])
def test_workspace_bytes_rejects_options(opts):
    st, _ = _ws(_problem(), opts)
    assert st == -1


def test_create_rejects_bad_workspace_without_touching_gpu():
    lib = binding.load_library()
    pr = _problem()
    o = binding.UpdateOpts(0, 1, 1, 0)
    h = ctypes.c_void_p(0)
    assert lib.pqmc_create(ctypes.byref(pr), ctypes.byref(o), None, None, 0, ctypes.byref(h)) == -1
    assert lib.pqmc_create(ctypes.byref(pr), ctypes.byref(o), None, ctypes.c_void_p(257), 1 << 30,
                           ctypes.byref(h)) == -1


def _soc_ws(U=-4.0, scheme=1, k=16, flags=0, hop=None, ne=14, b=1):
    import synth
    p = synth.make_soc_problem(4, 14, -4.0, seed=synth.SEED_BASE + 95)
    H = np.ascontiguousarray(p.hopping if hop is None else hop, dtype=np.complex128)
    P = np.ascontiguousarray(p.trial, dtype=np.complex128)
    pr = binding.SocProblem(16, ne, H.view(np.float64).ctypes.data_as(
        ctypes.POINTER(ctypes.c_double)), P.view(np.float64).ctypes.data_as(
        ctypes.POINTER(ctypes.c_double)), U, 0.05, 20, 5, 1, 0)
    lib = binding.load_library()
    n = ctypes.c_size_t(0)
    o = binding.UpdateOpts(scheme, k, b, flags)
    return lib.pqmc_soc_workspace_bytes(ctypes.byref(pr), ctypes.byref(o), ctypes.byref(n)), n.value


def test_soc_workspace_bytes_and_rejections():
    st, n = _soc_ws()
    assert st == 0 and n > 0
    st2, n2 = _soc_ws(flags=binding.FLAG_LOG)
    assert st2 == 0 and n2 > n
    assert _soc_ws(U=1.0)[0] == -1                  # the spin-s^y decoupling needs U <= 0
    assert _soc_ws(scheme=2, b=32)[0] == 0          # block force bias, b <= 32
    assert _soc_ws(scheme=2, b=33)[0] == -1
    assert _soc_ws(scheme=2, b=0)[0] == -1
    assert _soc_ws(scheme=3)[0] == -1
    assert _soc_ws(k=33)[0] == -1
    assert _soc_ws(flags=binding.FLAG_FP32)[0] == -1
    assert _soc_ws(ne=33)[0] == -1                  # more fermions than orbitals
    bad = np.zeros((32, 32), np.complex128)
    bad[0, 1] = 1j                                  # not Hermitian
    assert _soc_ws(hop=bad)[0] == -1


def test_sector_size_limit():
    """N_sigma up to 1024 is accepted, 1025 is rejected (the stabilisation
    kernels hold a pivot column of at most 1024 rows)."""
    N = 1100
    H = np.zeros((N, N))
    for n_up, want in ((1024, 0), (1025, -1)):
        P = np.zeros((N, n_up))
        Pd = np.zeros((N, 4))
        pr = binding.Problem(N, n_up, 4, binding._dptr(H), binding._dptr(P), binding._dptr(Pd),
                             4.0, 0.05, 10, 5, 1, 0)
        st, nbytes = _ws(pr, binding.UpdateOpts(1, 32, 1, 0))
        assert st == want, (n_up, st)
        if want == 0:
            assert nbytes > 0
