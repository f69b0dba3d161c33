"""HIP-graph replay of the evaluation launch chain: every replay equals the
eager launch bit for bit, with the rows changed in place and other eager
work and synchronisations between replays; a new observation drops the
recorded chains; the fitters give identical results in both modes."""
import numpy as np
import pytest

from paper_1510_01815_amd import inputs as I
from test_gpu_eval import make_obs, rows_for

pytestmark = pytest.mark.gpu

GRID = I.Grid(32, 32, 64, 30.0, psf_fwhm=2.5, lsf_sigma=30.0)


def test_graph_replays_equal_eager(O, gbk):
    import torch
    rows = rows_for(GRID, 24, 3)
    obs = make_obs(O, GRID, rows[0], 5, random_mask=0.1)
    g = gbk.Model.from_grid(GRID)
    e = gbk.Model.from_grid(GRID)
    e.set_launch_mode("eager")
    for m in (g, e):
        m.set_obs(obs)
    s = torch.cuda.Stream()
    dev_rows = torch.tensor(rows, device="cuda")
    out = torch.empty(24, dtype=torch.float64, device="cuda")
    nv = torch.empty(24, dtype=torch.int64, device="cuda")
    maps = torch.empty((24, 3, 32, 32), dtype=torch.float32, device="cuda")
    rng = np.random.default_rng(8)
    for it in range(6):
        # new values in the same device rows
        fresh = rows_for(GRID, 24, 100 + it)
        with torch.cuda.stream(s):
            dev_rows.copy_(torch.tensor(fresh, device="cuda"))
            g.chi2(dev_rows, out=out, n_valid=nv, stream=s)
            g.evaluate(dev_rows, out=maps, stream=s)
        s.synchronize()
        ref, ref_nv = e.chi2(torch.tensor(fresh, device="cuda"), stream=s)
        ref_maps = e.evaluate(torch.tensor(fresh, device="cuda"), stream=s)
        s.synchronize()
        assert torch.equal(out, ref) and torch.equal(nv, ref_nv), it
        assert torch.equal(maps, ref_maps), it
        # unrelated eager work between replays
        _ = e.chi2(rows_for(GRID, 5, 200 + it))
        torch.cuda.synchronize()
    assert g.graph_launches() >= 8  # calls 2..6 of both entry points replay
    assert e.graph_launches() == 0
    # a new observation drops the recorded chains; results follow it
    obs2 = make_obs(O, GRID, rows[3], 6, random_mask=0.2, W=0.3)
    g.set_obs(obs2)
    e.set_obs(obs2)
    for it in range(3):
        with torch.cuda.stream(s):
            g.chi2(dev_rows, out=out, n_valid=nv, stream=s)
        s.synchronize()
        ref, ref_nv = e.chi2(dev_rows.clone(), stream=s)
        s.synchronize()
        assert torch.equal(out, ref) and torch.equal(nv, ref_nv)


def test_fitters_identical_in_graph_and_eager_modes(O, gbk):
    truth = I.c1_truth()
    obs = make_obs(O, I.c1_grid(), truth, 11)
    res = {}
    for mode in ("graph", "eager"):
        m = gbk.Model.from_grid(I.c1_grid())
        m.set_launch_mode(mode)
        m.set_obs(obs)
        start = I.c1_start(I.rng_for(1, 0, 2))
        free = [1, 1, 1, 1, 1, 1, 1, 1, 1, 0, 0, 0]
        lm = m.fit_lm(start, free)
        lo = truth - np.array([2, 2, 20, 20, 20, 60, 2, 20, 2, 0, 0, 0.0])
        hi = truth + np.array([2, 2, 20, 20, 20, 60, 2, 20, 2, 0, 0, 0.0])
        ns = m.fit_nested(lo, hi, [1, 1, 0, 1, 1, 1, 0, 1, 0, 0, 0, 0], truth, n_live=100, seed=3)
        res[mode] = (lm, ns, m.graph_launches())
    lg, ng, cg = res["graph"]
    le, ne, ce = res["eager"]
    assert cg > 0 and ce == 0
    np.testing.assert_array_equal(lg["p"], le["p"])
    assert lg["chi2"] == le["chi2"] and lg["iterations"] == le["iterations"]
    assert ng["logz"] == ne["logz"]
    np.testing.assert_array_equal(ng["median"], ne["median"])
