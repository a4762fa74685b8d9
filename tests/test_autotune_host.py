"""Host-side parts of the size-class autotuner (no GPU)."""
import os

from paper_2503_01276_amd import autotune


def test_apply_sets_the_overrides_the_library_reads():
    keys = ["MCH_RPT_64", "MCH_RPT_32", "MCH_PREC_64", "MCH_PREC_32", "MCH_SPLIT"]
    saved = {k: os.environ.get(k) for k in keys}
    try:
        autotune.apply({"rows": {64: {"best": 8, "ms": {8: 1.0}}, "32": {"best": 4, "ms": {4: 1.0}}},
                        "prec": {64: {"best": 1, "ms": {1: 1.0, 0: 2.0}}, "32": {"best": 0, "ms": {0: 1.0}}},
                        "split": {"best": 0, "ms": {0: 1.0, 1: 1.5}}})
        assert os.environ["MCH_RPT_64"] == "8" and os.environ["MCH_RPT_32"] == "4"
        assert os.environ["MCH_PREC_64"] == "1" and os.environ["MCH_PREC_32"] == "0"
        assert os.environ["MCH_SPLIT"] == "0"
    finally:
        for k, v in saved.items():
            if v is None:
                os.environ.pop(k, None)
            else:
                os.environ[k] = v
