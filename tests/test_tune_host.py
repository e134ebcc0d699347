"""The autotuner's host side (no GPU): argument checks, the cache file read
at configuration, and the report of its decisions."""
import pytest

from paper_2304_05460_amd import afn


def test_invalid_modes_rejected():
    for mode, idx in ((-1, 0), (3, 0), (0, -1)):
        with pytest.raises(afn.AFNError) as e:
            afn.tune_config(mode, idx)
        assert e.value.status == afn.AFN_EINVAL


def test_cache_file_is_read_and_reported(tmp_path):
    f = tmp_path / "tune.txt"
    f.write_text("gemm_splits|m4000_K200000_R64_f64|gfx950/256cu 2\nkmv_tile|d8_n200000_f32_k0|gfx950/256cu 0\n")
    afn.tune_config(afn.AFN_TUNE_ON, 0, str(f))
    rep = afn.tune_report()
    assert "gemm_splits|m4000_K200000_R64_f64|gfx950/256cu 2" in rep
    assert "kmv_tile|d8_n200000_f32_k0|gfx950/256cu 0" in rep
    afn.tune_config(afn.AFN_TUNE_OFF)
