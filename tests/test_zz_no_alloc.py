"""pqmc_get_green_static (the entry point that allocates nothing; its device
temporaries live in a static array of the library) against pqmc_get_green,
through the C ABI: bit-identical G on two calls in a row, the second on a
smaller problem, and a clear refusal above the array's size."""
import ctypes

import numpy as np
import pytest

import synth
from gpu_util import make_chain

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2506_09611_amd import load_library
    load_library()


def _static_green(ch, spin):
    from paper_2506_09611_amd import load_library
    lib = load_library()
    out = np.full((ch.N, ch.N), np.nan)
    st = lib.pqmc_get_green_static(ch._ctx, int(spin),
                                   out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
    return st, out


def test_static_green_matches_workspace_green():
    # first call: 10x10 after a sweep; second: a smaller 6x6 lattice
    for L, n in [(10, 37), (6, 13)]:
        p = synth.make_problem(L, n, n - 2, 4.0, n_slices=20, stab_every=5, perturb=1e-3,
                               seed=synth.SEED_BASE + 90 + L)
        ch = make_chain(p, "delayed", k=8)
        ch.sweep(1)
        ch.forward_window(7)        # mid-period: T carries rank-k flushes
        for spin in range(2):
            st, Gs = _static_green(ch, spin)
            assert st == 0
            G = ch.green(spin)
            assert np.array_equal(Gs, G), (L, spin)
        ch.close()


def test_static_green_refuses_above_limit():
    p = synth.make_problem(46, 1024, 1000, 4.0, n_slices=2, stab_every=1, perturb=1e-3,
                           seed=synth.SEED_BASE + 121)
    ch = make_chain(p, "delayed", k=16)
    st, _ = _static_green(ch, 0)
    assert st == -1
    from paper_2506_09611_amd import load_library
    assert b"static scratch" in load_library().pqmc_last_error()
    ch.close()
