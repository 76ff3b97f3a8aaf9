"""The slice propagation B_l = e^{H_I(x_l)} e^{-dtau H0} (Eq. (9)) applied two
ways: the Taylor series of the sparse H0 (the default for lattice models) and
the dense K = e^{-dtau H0} (PQMC_FLAG_DENSE_PROP, and the fallback for a dense
H0).  Both are the same operator to rounding: the chains must take the same
decisions and reach the same G to 1e-12, the oracle's to 1e-10, and not be
bitwise equal (so that the two paths really ran)."""
import dataclasses

import numpy as np
import pytest

import synth
from oracle.pqmc import Walker
from gpu_util import make_chain, compare_decisions, green_rel_err, rel_err

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2506_09611_amd import load_library
    load_library()


def _both(p, scheme, sweeps=1, window=None, **kw):
    w = Walker(p, scheme, **kw)
    sp = make_chain(p, scheme, **kw)
    de = make_chain(p, scheme, dense_prop=True, **kw)
    for sw in range(sweeps):
        if window is None:
            w.sweep()
            sp.sweep(1)
            de.sweep(1)
        else:
            w.forward_window(window)
            sp.forward_window(window)
            de.forward_window(window)
        for ch in (sp, de):
            meta, margin = ch.decisions()
            compare_decisions(meta, margin, w.log, sw, p.n_slices)
            assert np.array_equal(ch.fields(), w.fields)
            assert green_rel_err(ch, w) < 1e-10
        d = max(rel_err(sp.green(s), de.green(s)) for s in range(2))
        print(f"{scheme} L={p.L} sweep {sw}: sparse vs dense G {d:.2e}", flush=True)
        assert d < 1e-12
    assert not all(np.array_equal(sp.green(s), de.green(s)) for s in range(2))
    sp.close()
    de.close()


@pytest.mark.parametrize("scheme,kw", [("local", {}), ("delayed", {"k": 4}), ("block", {"b": 4})])
def test_sparse_and_dense_propagation_4x4(scheme, kw):
    p = synth.make_problem(4, 5, 5, 4.0, n_slices=20, stab_every=5, perturb=1e-3,
                           seed=synth.SEED_BASE + 101)
    _both(p, scheme, sweeps=2, **kw)


@pytest.mark.timeout(600)
def test_sparse_and_dense_propagation_c2_sweep():
    """16x16, N_sigma = 121, M = 400: one whole delayed sweep each way."""
    _both(synth.workload("c2"), "delayed", k=16)


@pytest.mark.timeout(300)
def test_sparse_and_dense_propagation_c3_window():
    """40x40, N_sigma = 800 (R = 4 rows per thread): a 12-slice window that
    crosses a stabilisation."""
    _both(synth.workload("c3", n_slices=20, stab_every=10), "delayed", window=12, k=32)


def test_dense_hopping_falls_back_to_gemm():
    """A hopping matrix with every entry nonzero (N = 16: above the eight
    nonzeros per row of the sparse path) runs on the dense K, against the
    oracle over two sweeps."""
    p = synth.make_problem(4, 5, 5, 4.0, n_slices=20, stab_every=5, perturb=1e-3,
                           seed=synth.SEED_BASE + 102)
    rng = np.random.default_rng(7)
    E = rng.uniform(-0.05, 0.05, size=(16, 16))
    H = p.hopping + (E + E.T) / 2
    e, V = np.linalg.eigh(H)
    q = dataclasses.replace(p, hopping=H, trial_up=np.ascontiguousarray(V[:, :5]),
                            trial_dn=np.ascontiguousarray(V[:, :5]))
    assert e[5] - e[4] > 1e-6
    w = Walker(q, "delayed", k=4)
    ch = make_chain(q, "delayed", k=4)
    de = make_chain(q, "delayed", k=4, dense_prop=True)
    for sw in range(2):
        w.sweep()
        ch.sweep(1)
        de.sweep(1)
        meta, margin = ch.decisions()
        compare_decisions(meta, margin, w.log, sw, q.n_slices)
        assert green_rel_err(ch, w) < 1e-10
    # the same path either way: bitwise equal
    for s in range(2):
        assert np.array_equal(ch.green(s), de.green(s))
    ch.close()
    de.close()


def test_triangular_hopping_eight_wide_rows():
    """Nearest and next-nearest neighbours (eight nonzeros per row: the wide
    ELL form) on 6x6, against the oracle."""
    p = synth.make_problem(6, 13, 13, 4.0, n_slices=20, stab_every=5, perturb=1e-3,
                           seed=synth.SEED_BASE + 103)
    L = 6
    H = p.hopping.copy()
    for y in range(L):
        for x in range(L):
            i = x + L * y
            for dx, dy in ((1, 1), (1, -1)):
                j = (x + dx) % L + L * ((y + dy) % L)
                H[i, j] = H[j, i] = 0.3
    assert max(np.count_nonzero(H[i]) for i in range(36)) == 8
    e, V = np.linalg.eigh(H)
    assert e[13] - e[12] > 1e-6
    q = dataclasses.replace(p, hopping=H, trial_up=np.ascontiguousarray(V[:, :13]),
                            trial_dn=np.ascontiguousarray(V[:, :13]))
    _both(q, "delayed", sweeps=1, k=6)


def _soc_both(p, scheme, k, sweeps=1):
    """SOC walkers with the Taylor propagation of the sparse complex H0 and with
    the dense K: the oracle's decisions and G for both, the two G equal to
    1e-12 and not bitwise equal."""
    from oracle.soc import SocWalker
    from paper_2506_09611_amd import SocChain, Scheme
    sc = {"local": Scheme.LOCAL, "delayed": Scheme.DELAYED, "block": Scheme.BLOCK_FB}[scheme]
    chains = [SocChain(p.hopping, p.trial, p.U, p.dtau, p.n_slices, p.stab_every, p.seed,
                       p.walker_id, scheme=sc, k=k, log=True, dense_prop=d)
              for d in (False, True)]
    w = SocWalker(p, scheme, k=k, b=k)
    for sw in range(sweeps):
        w.sweep()
        for ch in chains:
            ch.sweep(1)
            meta, margin = ch.decisions()
            compare_decisions(meta, margin, w.log, sw, p.n_slices)
            assert np.array_equal(ch.fields(), w.fields)
            G, Gr = ch.green(), w.green()
            assert np.max(np.abs(G - Gr)) / max(1.0, np.max(np.abs(Gr))) < 1e-10
        Gs, Gd = chains[0].green(), chains[1].green()
        d = np.max(np.abs(Gs - Gd)) / max(1.0, np.max(np.abs(Gd)))
        print(f"soc {scheme} L={p.L} sweep {sw}: sparse vs dense G {d:.2e}", flush=True)
        assert d < 1e-12
    assert not np.array_equal(chains[0].green(), chains[1].green())
    for ch in chains:
        ch.close()


@pytest.mark.parametrize("scheme,k", [("local", 1), ("delayed", 8), ("block", 4)])
def test_soc_sparse_and_dense_propagation_4x4(scheme, k):
    """Rashba hopping (eight nonzeros per row of the 2N x 2N H0: four same-spin
    and four spin-flip neighbours) on 4x4, two sweeps."""
    p = synth.make_soc_problem(4, 14, -4.0, lam=0.5, dtau=0.05, n_slices=20, stab_every=5,
                               perturb=1e-3, seed=synth.SEED_BASE + 106)
    _soc_both(p, scheme, k, sweeps=2)


@pytest.mark.timeout(300)
def test_soc_sparse_and_dense_propagation_16x16():
    """2N = 512, N_e = 256 (R = 1 row a thread, eight entries): one sweep."""
    p = synth.make_soc_problem(16, 256, -4.0, lam=0.5, dtau=0.05, n_slices=10, stab_every=5,
                               perturb=1e-3, seed=synth.SEED_BASE + 107)
    _soc_both(p, "delayed", 32)


def test_negative_u_sparse_and_dense_propagation():
    """The U < 0 one-sector model (real H0 embedded in complex) through the
    spin-decoupled calls, both propagation forms against the oracle."""
    p = synth.make_problem(6, 13, 13, -4.0, n_slices=20, stab_every=5, perturb=1e-3,
                           seed=synth.SEED_BASE + 108)
    _both(p, "delayed", sweeps=2, k=4)
