"""The sweep autotuner and the sweep variants: every variant gives the
oracle's cost and gradient, and the tuned configuration does too."""
import sys

import numpy as np
import pytest

import workloads
from test_gpu_parity import check, compare

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.mark.parametrize("d,S,variant", [(100, 2, 1), (100, 2, 2), (12, 4, 1), (12, 4, 3),
                                         (40, 3, 3), (100, 2, 5),
                                         (260, 18, 5)])  # ragged row tile, two state tiles
def test_sweep_variants_match_oracle(d, S, variant):
    rng = np.random.default_rng(23 + d)
    p = workloads.random_problem(rng, d=d, M=2, N=70, S=S, dt=0.25, scale=1.5)
    from paper_1612_04929_amd import qoc
    import oracle
    ref = oracle.cost_grad(p)
    say(f"[tune] d={d} S={S} variant {variant}")
    h = qoc.Problem(p, precision="fp32", checkpoint_every=8)
    h.set_sweep(-1, variant)
    out = h.cost_grad(p.u)
    h.close()
    dF = abs((1 - out["C_fid"]) - ref["F"])
    rel = np.linalg.norm(out["grad"] - ref["grad"]) / np.linalg.norm(ref["grad"])
    say(f"[tune] variant {variant}: dF={dF:.2e} grad_rel={rel:.2e}")
    assert dF <= 1e-6 and rel <= 1e-4


def test_mfma_sweeps_fp64_match_oracle():
    """Sweep variant 5 (per-step launches, products on the FP64 MFMA) in
    FP64 chains, with the level penalty (block-local penalty costates)."""
    rng = np.random.default_rng(31)
    p = workloads.random_problem(rng, d=100, M=2, N=60, S=3, dt=0.25, scale=1.5)
    from paper_1612_04929_amd import qoc
    import oracle
    ref = oracle.cost_grad(p)
    h = qoc.Problem(p, precision="fp64", checkpoint_every=8)
    h.set_sweep(-1, 5)
    out = h.cost_grad(p.u)
    h.close()
    dF = abs((1 - out["C_fid"]) - ref["F"])
    rel = np.linalg.norm(out["grad"] - ref["grad"]) / np.linalg.norm(ref["grad"])
    say(f"[tune] fp64 variant 5: dF={dF:.2e} grad_rel={rel:.2e}")
    assert dF <= 1e-11 and rel <= 1e-9
    assert np.max(np.abs(out["c"] - ref["c"])) <= 1e-11


def test_tuned_configuration_matches_oracle():
    from paper_1612_04929_amd import tune
    rng = np.random.default_rng(29)
    p = workloads.random_problem(rng, d=90, M=2, N=120, S=3, dt=0.25, scale=1.5)
    cfg = tune.tune(p, precision="fp32", reps=1)
    say(f"[tune] chose L={cfg['checkpoint_every']} sweeps={cfg['sweep']} in {cfg['seconds']:.2f} s")
    assert cfg["checkpoint_every"] in [r["L"] for r in cfg["table"]]
    out, ref, e = compare("tuned", p, checkpoint_every=cfg["checkpoint_every"])
    check(p, e)


@pytest.mark.parametrize("d,pm", [(100, 64), (40, 64), (70, 32), (20, 64)])
def test_padding_multiple_matches_oracle(d, pm):
    # zero padding to a multiple of 32 / 64 (64 x 64 tiles) is exact
    rng = np.random.default_rng(31 + d)
    p = workloads.random_problem(rng, d=d, M=3, N=40, S=2, dt=0.2, scale=1.5)
    out, ref, e = compare(f"pad{pm}_d{d}", p, pad_multiple=pm)
    check(p, e)
    assert out["d_pad"] == (d + pm - 1) // pm * pm


def test_tile_tuner_picks_a_candidate_and_caches(tmp_path, monkeypatch):
    from paper_1612_04929_amd import tune
    monkeypatch.setenv("QOC_TUNE_CACHE", str(tmp_path / "tiles.json"))
    monkeypatch.setattr(tune, "_TILE_CACHE", None)
    rng = np.random.default_rng(37)
    p = workloads.random_problem(rng, d=100, M=2, N=300, S=2, dt=0.2)
    say("[tune] tiles d=100")
    r = tune.tune_tiles(p, steps=128)
    say(f"[tune] tiles: {r}")
    assert r["pad_multiple"] in tune.pad_candidates(100) and not r["cached"]
    assert set(r["ms"]) == {"16", "64"}
    r2 = tune.tune_tiles(p, steps=128)
    assert r2["cached"] and r2["pad_multiple"] == r["pad_multiple"]
    assert (tmp_path / "tiles.json").exists()
    assert tune.pad_candidates(64) == [16] and tune.pad_candidates(20) == [16]
