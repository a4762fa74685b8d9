"""Host-side parts of the size-class autotuner (no GPU)."""
import os

import pytest

from paper_2503_01276_amd import autotune
from paper_2503_01276_amd import workloads as W


def test_apply_sets_the_overrides_the_library_reads():
    saved = {nc: os.environ.get(f"MCH_RPT_{nc}") for nc in (64, 32)}
    try:
        autotune.apply({64: {"best": 8, "ms": {8: 1.0}}, "32": {"best": 4, "ms": {4: 1.0}}})
        assert os.environ["MCH_RPT_64"] == "8" and os.environ["MCH_RPT_32"] == "4"
    finally:
        for nc, v in saved.items():
            if v is None:
                os.environ.pop(f"MCH_RPT_{nc}", None)
            else:
                os.environ[f"MCH_RPT_{nc}"] = v


def test_three_dimensional_configs_are_refused_before_any_device_use():
    cfg = W.PRESETS["t3d"]
    with pytest.raises(ValueError):
        autotune.tune(cfg, None, None)
