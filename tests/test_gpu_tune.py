"""The launch-shape autotuner and every configuration it can choose: each
forced configuration matches the oracle (the FFT path at its own bound), and
the tuner keeps the fastest of the ones it timed."""
import numpy as np
import pytest

from paper_1510_01815_amd import inputs as I
from parity import assert_maps_close
from test_gpu_eval import oracle_maps, rows_for

pytestmark = pytest.mark.gpu

GRIDS = {
    "c1_32x32x64": I.Grid(32, 32, 64, 30.0, psf_fwhm=2.5, lsf_sigma=30.0),
    "wide_80x70x24": I.Grid(80, 70, 24, 30.0, psf_fwhm=3.0, lsf_sigma=30.0),
    "u2_30x26x32": I.Grid(30, 26, 32, 30.0, psf_fwhm=3.0, lsf_sigma=30.0, u=2),
}


@pytest.mark.parametrize("name", sorted(GRIDS))
def test_every_configuration_matches_oracle(O, gbk, name):
    grid = GRIDS[name]
    rows = rows_for(grid, 4, 13)
    ref = oracle_maps(O, grid, rows)
    m = gbk.Model.from_grid(grid)
    tried = 0
    for conv, tx, ty in gbk.TUNE_CANDIDATES:
        try:
            m.set_conv_config(conv, tx, ty)
        except gbk.GkError:
            continue  # does not fit this grid
        tried += 1
        out = m.evaluate(rows).cpu().numpy()
        for b in range(len(rows)):
            assert_maps_close(out[b], ref[b], f"{name} {conv} {tx}x{ty} row {b}",
                              bright_frac=1e-8 if conv == "fft" else 1e-12)
    assert tried >= 3


def test_autotune_keeps_fastest(O, gbk):
    grid = GRIDS["wide_80x70x24"]
    m = gbk.Model.from_grid(grid)
    r = m.autotune(64)
    print("tune", r)
    assert r["n_candidates"] == len(r["ms"]) >= 3
    assert r["ms_best"] == min(r["ms"].values())
    key = (r["conv"], *r["tile"])
    assert r["ms"][key] == r["ms_best"]
    rows = rows_for(grid, 3, 14)
    out = m.evaluate(rows).cpu().numpy()
    ref = oracle_maps(O, grid, rows)
    for b in range(3):
        assert_maps_close(out[b], ref[b], f"tuned row {b}",
                          bright_frac=1e-8 if r["conv"] == "fft" else 1e-12)


def test_forced_path_restricts_tuning(gbk):
    m = gbk.Model.from_grid(GRIDS["c1_32x32x64"], conv="direct")
    r = m.autotune(16)
    assert r["conv"] == "direct" and ("fft", 0, 0) not in r["ms"]
    with pytest.raises(gbk.GkError):
        m.set_conv_config("direct", 64, 64)  # 4096 data pixels: more than a block makes
