"""The size-class autotuner on the GPU (needs an MI355X)."""
import os

import numpy as np
import pytest

from paper_2503_01276_amd import workloads as W

from gpu_util import gpu_forward, say

pytestmark = pytest.mark.gpu


def test_autotune_times_every_knob_and_the_tuned_plan_agrees():
    from paper_2503_01276_amd import autotune, mch

    cfg = W.PRESETS["t3"]  # level cell widths 32, 16, 8
    k, l = W.medium("t3")
    widths = [cfg.n_cell // cfg.eta ** n for n in range(cfg.levels)]
    keys = [f"MCH_RPT_{nc}" for nc in widths] + [f"MCH_PREC_{nc}" for nc in widths] + ["MCH_SPLIT"]
    saved = {key: os.environ.get(key) for key in keys}
    try:
        default = mch.Plan(cfg)
        default_rows, default_prec = list(default.rows_per_thread), list(default.band_precond)
        default.close()
        assert default_prec == [False, False, False]  # band correction by default on 64^2 cells only
        table = autotune.tune(cfg, k, l, reps=2)
        say(f"[gpu] autotune t3: {table}")
        for n, nc in enumerate(widths):
            rows, prec = table["rows"][nc], table["prec"][nc]
            assert rows["best"] in rows["ms"] and all(t > 0 for t in rows["ms"].values())
            assert default_rows[n] in rows["ms"]  # the static choice is one of the candidates
            assert prec["best"] in prec["ms"] and 0 in prec["ms"]
        assert set(table["split"]["ms"]) == {0, 1}
        _, A0, *_ = gpu_forward(cfg, k, l)
        autotune.apply(table)
        tuned = mch.Plan(cfg)
        assert tuned.rows_per_thread == [table["rows"][nc]["best"] for nc in widths]
        assert tuned.band_subbands == [table["prec"][nc]["best"] for nc in widths]
        tuned.close()
        _, A1, *_ = gpu_forward(cfg, k, l)
        err = np.abs(A1 - A0).max() / np.abs(A0).max()
        say(f"[gpu] autotune t3: tuned vs default plan A_eff rel diff {err:.2e}")
        assert err <= 1e-9, err
    finally:
        for key, v in saved.items():
            if v is None:
                os.environ.pop(key, None)
            else:
                os.environ[key] = v
