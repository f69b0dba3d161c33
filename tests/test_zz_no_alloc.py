"""gk_chi2_batch_noalloc (the allocation-free chi-square) against
gk_chi2_batch, through the C ABI: the same kernels on the library's fixed
scratch array, so chi-square and n_valid must agree bit for bit.  Two calls in
a row on each model, the second with fewer rows; the 128 x 128 x 48 workload's
400-row batch needs two passes through the array."""
import numpy as np
import pytest

from paper_1510_01815_amd import inputs as I
from parity import oracle_desc

pytestmark = pytest.mark.gpu


def _observed_model(O, gbk, grid, truth, seed, conv="auto"):
    d = oracle_desc(O, grid.as_dict())
    obs = I.make_observation(O.evaluate(d, truth), 5.0, I.rng_for(900, seed, 1))
    m = gbk.Model.from_grid(grid, device=0, conv=conv)
    m.set_obs(obs)
    return m


def _compare(gbk, m, rows_np):
    import torch
    rows = torch.tensor(rows_np, device="cuda:0")
    B = rows.shape[0]
    ref, ref_n = m.chi2(rows)
    out = torch.full((B,), -1.0, dtype=torch.float64, device="cuda:0")
    nv = torch.full((B,), -1, dtype=torch.int64, device="cuda:0")
    m.chi2_noalloc(rows, out, nv)
    torch.cuda.synchronize()
    a, b = out.cpu().numpy(), ref.cpu().numpy()
    assert np.array_equal(a.view(np.int64), b.view(np.int64)), (a[:4], b[:4])
    assert np.array_equal(nv.cpu().numpy(), ref_n.cpu().numpy())
    return a


def _c2_rows(n, seed):
    rows = I.c2_draw(I.rng_for(2, seed, 11), n)
    rows[3, I.INC] = 95.0  # an out-of-domain row: chi2 = +inf on both paths
    return rows


def test_noalloc_matches_chi2_batch_c2(O, gbk):
    grid = I.c2_grid()
    truth = I.c2_draw(I.rng_for(2, 0, 10), 1)[0]
    m = _observed_model(O, gbk, grid, truth, 0)
    a = _compare(gbk, m, _c2_rows(400, 1))       # two passes through the array
    assert np.isinf(a[3]) and np.isfinite(np.delete(a, 3)).all()
    _compare(gbk, m, _c2_rows(37, 2))            # then a smaller batch
    m.close()


def test_noalloc_matches_chi2_batch_small_and_fft(O, gbk):
    grid = I.c1_grid()
    m = _observed_model(O, gbk, grid, I.c1_truth(), 1)
    rows = np.stack([I.c1_start(I.rng_for(1, 0, 20 + k)) for k in range(19)])
    _compare(gbk, m, rows)
    _compare(gbk, m, rows[:5])
    m.close()
    # the FFT path also carves the x-pass planes out of the array
    grid = I.Grid(24, 20, 32, 30.0, psf_fwhm=4.0, lsf_sigma=30.0)
    m = _observed_model(O, gbk, grid, np.array([12, 10, 30, 50, 0, 150, 3, 40, 5, 1, 1, 1.0]),
                        2, conv="fft")
    assert m.conv_path() == "fft"
    rows = I.c1_box_draw(I.rng_for(900, 3, 0), 64, 20, 4.0)
    _compare(gbk, m, rows)
    _compare(gbk, m, rows[:9])
    m.close()


def test_noalloc_refusals(gbk):
    import torch
    m = gbk.Model.from_grid(I.c1_grid(), device=0)
    out = torch.empty(2, dtype=torch.float64, device="cuda:0")
    rows = torch.tensor(np.stack([I.c1_truth()] * 2), device="cuda:0")
    with pytest.raises(gbk.GkError) as e:            # no observation
        m.chi2_noalloc(rows, out)
    assert e.value.status == gbk.GK_ESTATE
    with pytest.raises(gbk.GkError) as e:            # rows in host memory
        m.chi2_noalloc(np.stack([I.c1_truth()] * 2), out)
    assert e.value.status == gbk.GK_EINVAL
    m.close()
    # one row of a 2400 x 2400 image needs more than the array holds
    big = gbk.Model(2400, 2400, 1, 30.0, device=0)
    with pytest.raises(gbk.GkError) as e:
        big.chi2_noalloc(rows, out)
    assert e.value.status == gbk.GK_EINVAL and "scratch" in str(e.value)
    big.close()
