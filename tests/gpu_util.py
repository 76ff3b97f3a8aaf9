"""Helpers shared by the GPU parity tests (not collected by pytest)."""
import numpy as np

from oracle.pqmc import Walker

LOW = 1e-12


def make_chain(p, scheme, k=1, b=1, log=True, timing=False, **extra):
    from paper_2506_09611_amd import Chain, Scheme
    sc = {"local": Scheme.LOCAL, "delayed": Scheme.DELAYED, "block": Scheme.BLOCK_FB}[scheme]
    return Chain(p.hopping, p.trial_up, p.trial_dn, p.U, p.dtau, p.n_slices, p.stab_every,
                 p.seed, p.walker_id, scheme=sc, k=k, b=b, log=log, timing=timing, **extra)


def compare_decisions(meta, margin, ref_log, sweep, M, low=LOW, margin_tol=1e-9):
    """Decisions of one GPU call vs the oracle's entries of that sweep.
    Exact equality up to the first decision with |margin| < low on either side;
    margins agree to margin_tol (relative above 1).  Returns
    (n_compared, n_low_margin)."""
    ref = [e for e in ref_log if e[0] == sweep]
    assert len(ref) == len(meta), (len(ref), len(meta))
    n = 0
    for (code, site, acc), mg, e in zip(meta, margin, ref):
        assert int(code) == e[1] * M + e[2], (n, code, e)
        assert int(site) == e[3], (n, site, e)
        if abs(mg) < low or abs(e[5]) < low:
            return n, 1
        assert bool(acc) == e[4], f"decision {n} differs: gpu {acc} margin {mg:.3e}, oracle {e}"
        if np.isinf(mg) or np.isinf(e[5]):
            assert mg == e[5], (n, mg, e[5])
        else:
            assert abs(mg - e[5]) < margin_tol * max(1.0, abs(e[5])), (n, mg, e[5])
        n += 1
    return n, 0


def green_rel_err(chain, walker):
    err = 0.0
    for s in range(2):
        G, Gr = chain.green(s), walker.green(s)
        err = max(err, np.max(np.abs(G - Gr)) / np.max(np.abs(Gr)))
    return err
