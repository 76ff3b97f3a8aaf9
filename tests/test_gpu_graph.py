"""Graph-captured sweeps (PQMC_FLAG_GRAPH) against sweeps launched one by one.

A captured sweep replays the same launches with the Philox sweep counter
read from device memory, so every decision, field and Green's function entry
must be bit for bit that of the ordinary sweep; the graph must be captured
again when a walker's options or fields change, and walker 0 must still take
the oracle's decisions.
"""
import dataclasses

import numpy as np
import pytest

import synth
from oracle.pqmc import Walker
from gpu_util import make_chain, compare_decisions, green_rel_err

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2506_09611_amd import load_library
    load_library()


def _pair(probs, scheme, kw, **extra):
    """The same walkers twice, each set on a stream of its own; the first set
    sweeps through captured graphs."""
    import torch
    from paper_2506_09611_amd import Scheme
    sa, sb = torch.cuda.Stream(), torch.cuda.Stream()
    ga = [make_chain(q, scheme, stream=sa, **kw, **extra) for q in probs]
    gb = [make_chain(q, scheme, stream=sb, **kw, **extra) for q in probs]
    sc = {"delayed": Scheme.DELAYED, "block": Scheme.BLOCK_FB}[scheme]
    for ch in ga:
        ch.set_opts(sc, graph=True, **kw)
    return ga, gb


def _same(ga, gb, label):
    for i, (a, b) in enumerate(zip(ga, gb)):
        ma, xa = a.decisions()
        mb, xb = b.decisions()
        assert np.array_equal(ma, mb), f"{label} walker {i}: decisions"
        assert np.array_equal(xa, xb), f"{label} walker {i}: margins"
        assert np.array_equal(a.fields(), b.fields()), f"{label} walker {i}: fields"
        for s in range(2):
            assert np.array_equal(a.green(s), b.green(s)), f"{label} walker {i}: G_{s}"


@pytest.mark.parametrize("scheme,kw", [("delayed", {"k": 4}), ("block", {"b": 4})])
def test_graph_sweeps_equal_launched_sweeps(scheme, kw):
    """Three walkers of three sizes (4x4, 6x6, 8x8, one batch): graph sweeps
    one at a time and two per call, bitwise against launched sweeps; walker 0
    against the oracle."""
    from paper_2506_09611_amd import batch_sweep
    probs = [synth.make_problem(L, n, n, 4.0, n_slices=20, stab_every=5, perturb=1e-3,
                                seed=synth.SEED_BASE + 91)
             for L, n in [(4, 5), (6, 13), (8, 25)]]
    probs = [dataclasses.replace(q, walker_id=i) for i, q in enumerate(probs)]
    ga, gb = _pair(probs, scheme, kw)
    ref = Walker(probs[0], scheme, **kw)
    for sw in range(3):
        batch_sweep(ga, 1)
        batch_sweep(gb, 1)
        ref.sweep()
        _same(ga, gb, f"{scheme} sweep {sw}")
        meta, margin = ga[0].decisions()
        n, _ = compare_decisions(meta, margin, ref.log, sw, probs[0].n_slices)
        assert green_rel_err(ga[0], ref) < 1e-10
        print(f"{scheme} sweep {sw}: {n} oracle decisions equal", flush=True)
    # two sweeps in one call: the log holds the last one
    batch_sweep(ga, 2)
    batch_sweep(gb, 1)
    batch_sweep(gb, 1)
    _same(ga, gb, f"{scheme} two-sweep call")
    for ch in ga + gb:
        ch.close()


def test_graph_recaptured_after_changes():
    """New options (k) and new fields on one walker: the next graph sweep must
    follow them, bitwise with launched sweeps given the same changes."""
    from paper_2506_09611_amd import Scheme, batch_sweep
    p = synth.make_problem(6, 13, 13, 4.0, n_slices=20, stab_every=5, perturb=1e-3,
                           seed=synth.SEED_BASE + 92)
    probs = [dataclasses.replace(p, walker_id=i) for i in range(2)]
    ga, gb = _pair(probs, "delayed", {"k": 4}, k_max=8)
    batch_sweep(ga, 1)
    batch_sweep(gb, 1)
    _same(ga, gb, "before changes")
    for chs, graph in [(ga, True), (gb, False)]:
        for ch in chs:
            ch.set_opts(Scheme.DELAYED, k=8, graph=graph)
    batch_sweep(ga, 1)
    batch_sweep(gb, 1)
    _same(ga, gb, "after k = 8")
    rng = np.random.default_rng(5)
    X = (2 * rng.integers(0, 2, size=(p.n_slices, p.n_sites)) - 1).astype(np.int8)
    ga[1].set_fields(X)
    gb[1].set_fields(X)
    batch_sweep(ga, 1)
    batch_sweep(gb, 1)
    _same(ga, gb, "after new fields")
    for ch in ga + gb:
        ch.close()


@pytest.mark.timeout(300)
def test_graph_fp32_form_mixed_batch():
    """The precision form (float32 panels and tiles, k = 32) on a batch of a
    24x24 and a 12x12 walker over a whole sweep."""
    from paper_2506_09611_amd import batch_sweep
    a = synth.make_problem(24, 288, 288, 6.0, n_slices=40, stab_every=10, perturb=1e-3,
                           seed=synth.SEED_BASE + 4)
    b = synth.make_problem(12, 72, 72, 6.0, n_slices=40, stab_every=10, perturb=1e-3,
                           seed=synth.SEED_BASE + 5)
    probs = [dataclasses.replace(a, walker_id=0), dataclasses.replace(b, walker_id=1)]
    ga, gb = _pair(probs, "delayed", {"k": 32}, fp32=True)
    for _ in range(2):
        batch_sweep(ga, 1)
        batch_sweep(gb, 1)
        _same(ga, gb, "fp32 mixed batch")
    for ch in ga + gb:
        ch.close()


def test_graph_multi_stream_captures_concurrently():
    """Six batches on six streams captured at once by the multi-stream sweep's
    threads (their captures overlap each other's copies and launches), two
    sweeps, bitwise against the same walkers launched."""
    import torch
    from paper_2506_09611_amd import Scheme, multi_sweep
    probs = []
    for i in range(12):
        L, n = [(4, 5), (6, 13)][i % 2]
        q = synth.make_problem(L, n, n, 4.0, n_slices=20, stab_every=5, perturb=1e-3,
                               seed=synth.SEED_BASE + 93)
        probs.append(dataclasses.replace(q, walker_id=i))
    sa = [torch.cuda.Stream() for _ in range(6)]
    sb = [torch.cuda.Stream() for _ in range(6)]
    ga = [make_chain(q, "delayed", k=4, stream=sa[i // 2]) for i, q in enumerate(probs)]
    gb = [make_chain(q, "delayed", k=4, stream=sb[i // 2]) for i, q in enumerate(probs)]
    for ch in ga:
        ch.set_opts(Scheme.DELAYED, k=4, graph=True)
    for sw in range(2):
        multi_sweep(ga, 1)
        multi_sweep(gb, 1)
        _same(ga, gb, f"multi-stream sweep {sw}")
    for ch in ga + gb:
        ch.close()
