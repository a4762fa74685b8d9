"""The size-class autotuner on the GPU (needs an MI355X)."""
import os

import numpy as np
import pytest

from paper_2503_01276_amd import workloads as W

from gpu_util import gpu_forward, say

pytestmark = pytest.mark.gpu


def test_autotune_times_instantiated_shapes_and_the_tuned_plan_agrees():
    from paper_2503_01276_amd import autotune, mch

    cfg = W.PRESETS["t3"]  # level cell widths 32, 16, 8
    k, l = W.medium("t3")
    widths = [cfg.n_cell // cfg.eta ** n for n in range(cfg.levels)]
    saved = {nc: os.environ.get(f"MCH_RPT_{nc}") for nc in widths}
    try:
        default = mch.Plan(cfg)
        default_rows = list(default.rows_per_thread)
        default.close()
        table = autotune.tune(cfg, k, l, reps=2)
        say(f"[gpu] autotune t3: {table}")
        for n, nc in enumerate(widths):
            assert table[nc]["best"] in table[nc]["ms"]
            assert all(t > 0 for t in table[nc]["ms"].values())
            assert default_rows[n] in table[nc]["ms"]  # the static choice is one of the candidates
        _, A0, *_ = gpu_forward(cfg, k, l)
        autotune.apply(table)
        tuned = mch.Plan(cfg)
        assert tuned.rows_per_thread == [table[nc]["best"] for nc in widths]
        tuned.close()
        _, A1, *_ = gpu_forward(cfg, k, l)
        err = np.abs(A1 - A0).max() / np.abs(A0).max()
        say(f"[gpu] autotune t3: tuned vs default plan A_eff rel diff {err:.2e}")
        assert err <= 1e-9, err
    finally:
        for nc, v in saved.items():
            if v is None:
                os.environ.pop(f"MCH_RPT_{nc}", None)
            else:
                os.environ[f"MCH_RPT_{nc}"] = v
