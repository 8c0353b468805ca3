"""End to end on the GPU, at small sizes: the batched horn ensemble, the
per-shape runs, surrogate training, inference on candidates, the fallback
set and the LBM judge, through the same entry point as the full study."""
import json
import math
import sys

import pytest

pytestmark = pytest.mark.gpu


def say(*a):
    print("[gpu-test]", *a, file=sys.stderr, flush=True)


def test_study_pipeline_small(tmp_path):
    from paper_1705_01801_amd import surrogate_study
    out = tmp_path / "study.json"
    say("study: 16 horns x 6000 steps, 2 per shape, 400 Adam steps, 2000 candidates")
    surrogate_study.main(["--train", "16", "--steps", "6000", "--plain", "2", "--judge", "4",
                          "--fallback-sample", "4", "--candidates", "2000", "--train-steps", "400",
                          "--hidden", "64", "--out", str(out)])
    rep = json.loads(out.read_text())
    assert rep["batched"]["horns"] == 16 and rep["batched"]["spectra_per_s"] > 0
    # per-shape and batched runs use the same tile body: identical spectra
    assert rep["plain"]["max_rel_diff_vs_batched"] == 0.0
    assert rep["training"]["widths"] == [3, 64, 64, 64, 10]
    assert all(math.isfinite(v) for v in rep["training"]["final_losses"])
    inf = rep["inference"]
    assert inf["candidates"] == 2000 and 0.0 <= inf["fallback_fraction"] <= 1.0
    if inf["fallback"] < inf["candidates"]:
        assert rep["judge"]["sampled"] > 0 and math.isfinite(rep["judge"]["rel_err_median"])
    if inf["fallback"] > 0:
        assert rep["fallback_sample"]["seconds_per_spectrum"] > 0
    assert rep["end_to_end"]["spectra_per_s"] > 0
