"""Helpers shared by the GPU parity tests (not collected by pytest)."""
import numpy as np

from oracle.pqmc import Walker

LOW = 1e-12


def make_chain(p, scheme, k=1, b=1, log=True, timing=False, **extra):
    from paper_2506_09611_amd import Chain, Scheme
    sc = {"local": Scheme.LOCAL, "delayed": Scheme.DELAYED, "block": Scheme.BLOCK_FB,
          "local_g": Scheme.LOCAL_G}[scheme]
    return Chain(p.hopping, p.trial_up, p.trial_dn, p.U, p.dtau, p.n_slices, p.stab_every,
                 p.seed, p.walker_id, scheme=sc, k=k, b=b, log=log, timing=timing, **extra)


def compare_decisions(meta, margin, ref_log, sweep, M, low=LOW, margin_tol=1e-9,
                      allow_low=False):
    """Decisions of one GPU call vs the oracle's entries of that sweep.

    Every decision must agree exactly (accept flag, slice, site) and margins
    to margin_tol (relative above 1).  A decision with |margin| < low on
    either side may legitimately differ; it fails the comparison unless
    allow_low is set, in which case the comparison stops there.  Returns
    (n_compared, n_low_margin); without allow_low, n_compared is always the
    whole call."""
    ref = [e for e in ref_log if e[0] == sweep]
    assert len(ref) == len(meta), (len(ref), len(meta))
    assert len(ref) > 0, "no decisions to compare"
    n = 0
    for (code, site, acc), mg, e in zip(meta, margin, ref):
        assert int(code) == e[1] * M + e[2], (n, code, e)
        assert int(site) == e[3], (n, site, e)
        if abs(mg) < low or abs(e[5]) < low:
            assert allow_low, f"low-margin decision {n} of {len(ref)}: gpu {mg:.3e}, oracle {e}"
            return n, 1
        assert bool(acc) == e[4], f"decision {n} differs: gpu {acc} margin {mg:.3e}, oracle {e}"
        if np.isinf(mg) or np.isinf(e[5]):
            assert mg == e[5], (n, mg, e[5])
        else:
            assert abs(mg - e[5]) < margin_tol * max(1.0, abs(e[5])), (n, mg, e[5])
        n += 1
    assert n == len(ref)
    return n, 0


def rel_err(G, Gr):
    """max|G - Gr| / max|Gr|, absolute where Gr vanishes; always finite."""
    scale = float(np.max(np.abs(Gr))) if Gr.size else 0.0
    err = float(np.max(np.abs(G - Gr))) / (scale if scale > 0.0 else 1.0)
    assert np.isfinite(err), "non-finite Green's function difference"
    return err


def green_rel_err(chain, walker):
    return max(rel_err(chain.green(s), walker.green(s)) for s in range(2))
