"""Delay-rank autotuner: selection and cache on the CPU, a tuning run on the GPU."""
import json

import numpy as np
import pytest

import synth
from paper_2506_09611_amd.autotune import choose, shape_key, tune_delay


def test_choose_fastest_ties_to_smaller_k():
    assert choose({8: 3.0, 16: 1.0, 32: 2.0}) == 16
    assert choose({32: 1.0, 16: 1.0}) == 16
    with pytest.raises(ValueError):
        choose({})


def test_cache_hit_needs_no_device(tmp_path):
    p = synth.make_problem(4, 5, 5, 4.0, n_slices=20, stab_every=5)
    path = tmp_path / "tune.json"
    key = shape_key(16, 5, 5, 4.0, 2, False)
    path.write_text(json.dumps({key: {
        "k": 8, "times": {"8": 1e-4, "16": 2e-4}, "tile_chunks": 4,
        "chunk_candidates": [2, 4], "chunk_times": {"2": 1e-4, "4": 0.9e-4}}}))
    r = tune_delay(p.hopping, p.trial_up, p.trial_dn, p.U, p.dtau, p.stab_every,
                   candidates=(8, 16), walkers=2, cache=str(path), chunk_candidates=(2, 4))
    assert r.cached and r.k == 8 and r.tile_chunks == 4
    assert r.update_s_per_slice == {8: 1e-4, 16: 2e-4}
    assert r.chunk_s_per_slice == {2: 1e-4, 4: 0.9e-4}


def test_cache_entry_for_other_candidates_is_not_a_hit(tmp_path):
    """A cached entry tuned over other chunk candidates must be retuned (here
    that needs a device, which the CPU suite does not have)."""
    pytest.importorskip("torch")
    import torch
    if torch.cuda.is_available():
        pytest.skip("checks the CPU path")
    p = synth.make_problem(4, 5, 5, 4.0, n_slices=20, stab_every=5)
    path = tmp_path / "tune.json"
    key = shape_key(16, 5, 5, 4.0, 2, False)
    path.write_text(json.dumps({key: {"k": 8, "times": {"8": 1e-4, "16": 2e-4}}}))
    with pytest.raises(Exception):
        tune_delay(p.hopping, p.trial_up, p.trial_dn, p.U, p.dtau, p.stab_every,
                   candidates=(8, 16), walkers=2, cache=str(path), chunk_candidates=(2, 4))


@pytest.mark.gpu
def test_tune_on_device(tmp_path):
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    p = synth.make_problem(10, 50, 50, 4.0, n_slices=20, stab_every=5, perturb=1e-3,
                           seed=synth.SEED_BASE + 70)
    path = str(tmp_path / "tune.json")
    r = tune_delay(p.hopping, p.trial_up, p.trial_dn, p.U, p.dtau, p.stab_every,
                   candidates=(8, 16, 32, 128), walkers=2, cache=path)
    print("tuned", r, flush=True)
    assert not r.cached and r.k in (8, 16, 32, 100)    # 128 is clipped to N = 100
    assert set(r.update_s_per_slice) == {8, 16, 32, 100}
    assert all(t > 0 for t in r.update_s_per_slice.values())
    if r.k <= 64:   # the chunk stage (fused path) at the chosen k
        assert set(r.chunk_s_per_slice) == {1, 2, 4, 64} and r.tile_chunks in (1, 2, 4, 64)
        assert all(t > 0 for t in r.chunk_s_per_slice.values())
    again = tune_delay(p.hopping, p.trial_up, p.trial_dn, p.U, p.dtau, p.stab_every,
                       candidates=(8, 16, 32, 128), walkers=2, cache=path)
    assert again.cached and again.k == r.k and again.tile_chunks == r.tile_chunks
