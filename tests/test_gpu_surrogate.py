"""The surrogate network on the GPU against the FP64 reference network and
the oracle: BF16 GEMM in every operand layout, forward maps, loss gradients,
training, surrogate chi-square, and screened nested sampling against the
plain sampler (same posterior, fewer plain evaluations)."""
import math

import numpy as np
import pytest

from oracle import mlp_ref as R
from paper_1510_01815_amd import inputs as I
from parity import oracle_desc

pytestmark = pytest.mark.gpu


def bf16_round(a):
    import torch
    return torch.as_tensor(np.asarray(a, dtype=np.float32)).to(torch.bfloat16).to(torch.float32).numpy()


@pytest.mark.parametrize("ta,tb", [(0, 0), (0, 1), (1, 1), (1, 0)])
@pytest.mark.parametrize("M,N,K", [(200, 150, 96), (1, 1, 32), (128, 128, 32), (257, 129, 1024),
                                   (64, 4096, 64)])
def test_gemm_bf16_all_layouts(gbk, ta, tb, M, N, K):
    """C = A(m,k) B(n,k) against an FP64 product of the same BF16 values,
    with padded row strides and ragged M, N (several tiles plus a tail)."""
    import torch
    g = torch.Generator().manual_seed(M * 7 + N * 3 + K + 11 * ta + 5 * tb)
    pad = lambda n: (n + 7) // 8 * 8 + 8  # row strides: multiples of 8, padded
    a_shape = (K, pad(M)) if ta else (M, pad(K))
    b_shape = (K, pad(N)) if tb else (N, pad(K))
    Af = torch.randn(a_shape, generator=g).to(torch.bfloat16)
    Bf = torch.randn(b_shape, generator=g).to(torch.bfloat16)
    A = Af[:, :M] if ta else Af[:, :K]
    B = Bf[:, :N] if tb else Bf[:, :K]
    # device views keep the padded row stride
    Ad = Af.cuda()[:, : (M if ta else K)]
    Bd = Bf.cuda()[:, : (N if tb else K)]
    C = gbk.gemm_bf16(Ad, Bd, trans_a=bool(ta), trans_b=bool(tb), M=M, N=N, K=K)
    torch.cuda.synchronize()
    a64 = A.to(torch.float64).numpy()
    b64 = B.to(torch.float64).numpy()
    am = a64.T if ta else a64          # [M][K]
    bn = b64.T if tb else b64          # [N][K]
    ref = am @ bn.T
    got = C.cpu().numpy().astype(np.float64)
    scale = np.sqrt(K) * 1.0
    err = np.max(np.abs(got - ref))
    assert err <= 1e-5 * scale * max(1.0, np.max(np.abs(ref)) / scale), err


def test_gemm_rejects_bad_shapes(gbk):
    import torch
    A = torch.zeros((64, 40), dtype=torch.bfloat16, device="cuda")
    with pytest.raises(gbk.GkError):
        gbk.gemm_bf16(A, A, M=64, N=64, K=40)  # K not a multiple of 32


def small_setup(O, hidden=64, layers=2, batch=32, seed=3):
    grid = I.Grid(16, 16, 32, 30.0, psf_fwhm=2.0, lsf_sigma=30.0)
    lo = np.array([6.4, 6.4, 0.0, 5.0, -50.0, 50.0, 1.0, 20.0, 2.0, 0.5, 1.0, 1.0])
    hi = np.array([9.6, 9.6, 360.0, 85.0, 50.0, 300.0, 4.0, 100.0, 6.0, 2.0, 1.0, 1.0])
    return grid, lo, hi, dict(hidden=hidden, layers=layers, batch=batch, seed=seed)


def draw_rows(rng, lo, hi, n):
    return lo + rng.random((n, 12)) * (hi - lo)


def unpack(w, sizes):
    Ws, bs, o = [], [], 0
    for a, b in zip(sizes[:-1], sizes[1:]):
        Ws.append(w[o:o + a * b].reshape(b, a).astype(np.float64))
        o += a * b
        bs.append(w[o:o + b].astype(np.float64))
        o += b
    assert o == w.size
    return Ws, bs


def targets(O, d, rows):
    ts, ms = [], []
    for p in rows:
        m0, m1, m2 = O.evaluate(d, p)
        use = (m0 >= 0.01 * np.nanmax(m0)) & np.isfinite(m1) & np.isfinite(m2)
        ts.append(np.concatenate([np.where(use, m1 / 300.0, 0).ravel(), np.where(use, m2 / 100.0, 0).ravel()]))
        ms.append(np.concatenate([use.ravel(), use.ravel()]).astype(np.float64))
    return np.array(ts), np.array(ms)


def test_forward_and_gradients_match_fp64_reference(O, gbk):
    """Predicted maps and the loss gradient of every layer against the FP64
    network of the reference (same BF16-representable weights and inputs),
    with targets and mask from the oracle's maps; the bound is BF16's (2^-8)."""
    grid, lo, hi, opts = small_setup(O)
    m = gbk.Model.from_grid(grid)
    S = gbk.Surrogate(m, lo, hi, **opts)
    sizes = [32, opts["hidden"], opts["hidden"], 2 * 16 * 16]
    rng = np.random.default_rng(21)
    w = np.zeros(S.weight_count(), dtype=np.float32)
    Ws, bs = [], []
    for a, b in zip(sizes[:-1], sizes[1:]):
        Ws.append(bf16_round(rng.normal(0, 1.5 / math.sqrt(a), (b, a))))
        bs.append(rng.normal(0, 0.1, b).astype(np.float32))
    o = 0
    for W, b in zip(Ws, bs):
        w[o:o + W.size] = W.ravel()
        o += W.size
        w[o:o + b.size] = b
        o += b.size
    S.set_weights(w)
    np.testing.assert_array_equal(S.get_weights(), w)
    Ws, bs = unpack(w, sizes)
    rows = draw_rows(rng, lo, hi, 64)
    x = bf16_round(R.encode(rows, lo, hi)).astype(np.float64)
    y_ref, _ = R.forward(x, Ws, bs)
    y = S.predict(rows).cpu().numpy().reshape(64, -1).astype(np.float64)
    y_ref_kms = y_ref * np.repeat([300.0, 100.0], 256)
    err = np.abs(y - y_ref_kms)
    scale = np.abs(y_ref_kms).max()
    assert err.max() <= 2e-2 * scale, (err.max(), scale)
    # gradients
    d = oracle_desc(O, grid.as_dict())
    t, mask = targets(O, d, rows)
    loss_ref, gW, gb = R.loss_and_grads(x, t, mask, Ws, bs)
    loss, g = S.gradients(rows)
    assert abs(loss - loss_ref) <= 2e-2 * loss_ref, (loss, loss_ref)
    gW_gpu, gb_gpu = unpack(g, sizes)
    for l in range(len(Ws)):
        rel_w = np.linalg.norm(gW_gpu[l] - gW[l]) / np.linalg.norm(gW[l])
        rel_b = np.linalg.norm(gb_gpu[l] - gb[l]) / np.linalg.norm(gb[l])
        print(f"layer {l}: grad W rel {rel_w:.3g}, grad b rel {rel_b:.3g}")
        assert rel_w <= 5e-2 and rel_b <= 5e-2, (l, rel_w, rel_b)
    # the padded input columns see zero inputs, so their gradient is zero
    assert np.all(gW_gpu[0][:, 11:] == 0.0)
    S.close()


def test_training_reduces_loss(O, gbk):
    grid, lo, hi, opts = small_setup(O, hidden=128, layers=2, batch=64, seed=5)
    m = gbk.Model.from_grid(grid)
    S = gbk.Surrogate(m, lo, hi, lr=2e-3, lr_final=2e-4, **opts)
    losses = S.train(600)
    print("loss first", losses[:5], "last", losses[-5:])
    assert np.all(np.isfinite(losses))
    assert losses[-50:].mean() < 0.15 * losses[:10].mean()
    # a second call continues from the trained weights
    more = S.train(50)
    assert more.mean() < 0.3 * losses[:10].mean()
    S.close()


def test_surrogate_chi2_matches_oracle_chi2_of_predicted_maps(O, gbk):
    """Surrogate chi2 = eq. 11 (oracle) evaluated on the predicted maps; rows
    outside the parameter domain give +inf."""
    grid, lo, hi, opts = small_setup(O, seed=9)
    m = gbk.Model.from_grid(grid)
    d = oracle_desc(O, grid.as_dict())
    truth = np.array([8.0, 8.2, 40.0, 50.0, 0.0, 180.0, 2.5, 40.0, 3.0, 1.0, 1.0, 1.0])
    obs = I.make_observation(O.evaluate(d, truth), 5.0, I.rng_for(70, 0, 0), W=0.7)
    m.set_obs(obs)
    S = gbk.Surrogate(m, lo, hi, **opts)
    S.train(20)
    rows = draw_rows(np.random.default_rng(2), lo, hi, 50)
    rows[7, 3] = 95.0  # inclination outside (0, 90)
    maps = S.predict(rows).cpu().numpy().astype(np.float64)
    c = S.chi2(m, rows).cpu().numpy()
    for b in range(50):
        if b == 7:
            assert c[b] == np.inf
            continue
        ref, n = O.chi2(maps[b, 0], maps[b, 1], obs.vel, obs.sig, obs.evel, obs.esig, obs.mask, 0.7)
        assert abs(c[b] - ref) <= 1e-9 * ref, (b, c[b], ref)
    # a new observation (another mask) and further training: the restricted
    # output layer follows both
    obs2 = I.make_observation(O.evaluate(d, rows[3]), 3.0, I.rng_for(70, 1, 0), random_mask=0.3, W=1.0)
    m.set_obs(obs2)
    S.train(5)
    maps = S.predict(rows).cpu().numpy().astype(np.float64)
    c = S.chi2(m, rows).cpu().numpy()
    for b in (0, 1, 2, 20, 49):
        ref, n = O.chi2(maps[b, 0], maps[b, 1], obs2.vel, obs2.sig, obs2.evel, obs2.esig, obs2.mask, 1.0)
        assert abs(c[b] - ref) <= 1e-9 * ref, (b, c[b], ref)
    # all pixels masked: chi2 = 0 for rows in the domain
    obs2.mask[:] = 0
    m.set_obs(obs2)
    c = S.chi2(m, rows).cpu().numpy()
    assert c[7] == np.inf and np.all(c[np.arange(50) != 7] == 0.0)
    S.close()


def ns_problem(O, gbk):
    grid = I.Grid(24, 24, 40, 25.0, psf_fwhm=2.5, lsf_sigma=25.0)
    d = oracle_desc(O, grid.as_dict())
    truth = np.array([12.3, 11.6, 40.0, 50.0, 4.0, 180.0, 3.0, 35.0, 5.0, 1.0, 1.0, 1.0])
    obs = I.make_observation(O.evaluate(d, truth), 5.0, I.rng_for(60, 0, 0), W=1.0)
    m = gbk.Model.from_grid(grid)
    m.set_obs(obs)
    lo = np.array([10, 9, 0, 20, -30, 60, 0.5, 5, 5.0, 0.5, 1, 1], dtype=float)
    hi = np.array([14, 14, 90, 80, 30, 350, 8.0, 80, 5.0, 2.0, 1, 1], dtype=float)
    free = [1, 1, 1, 1, 1, 1, 1, 1, 0, 1, 0, 0]
    return m, truth, lo, hi, free


@pytest.fixture(scope="module")
def trained(O, gbk):
    m, truth, lo, hi, free = ns_problem(O, gbk)
    S = gbk.Surrogate(m, lo, hi, hidden=256, layers=3, batch=256, lr=2e-3, lr_final=1e-5, seed=7)
    losses = S.train(3000)
    print("surrogate loss", losses[:3], losses[-3:])
    return m, truth, lo, hi, free, S


def test_screened_nested_sampling_with_full_audit_equals_plain(gbk, trained):
    """audit = 1 evaluates every candidate plainly, so the run must equal the
    plain sampler bit for bit; the audit counts what the screen would have
    discarded."""
    m, truth, lo, hi, free, S = trained
    plain = m.fit_nested(lo, hi, free, truth, n_live=200, seed=11)
    full = S.fit_nested(m, lo, hi, free, truth, margin=25.0, audit=1.0, n_live=200, seed=11)
    assert full["logz"] == plain["logz"] and full["n_iter"] == plain["n_iter"]
    np.testing.assert_array_equal(full["median"], plain["median"])
    assert full["n_evals"] == plain["n_evals"]
    assert full["n_screened"] == plain["n_evals"]  # every candidate, the first live points too
    assert full["n_rejected"] == 0
    print("screen would discard", full["n_audited"], "of", full["n_screened"],
          "wrongly:", full["n_audit_miss"])
    assert full["n_audited"] > 0.5 * full["n_screened"]


def test_screened_nested_sampling_matches_plain_with_fewer_evaluations(gbk, trained):
    """What the trained network gains: the screened sampler reaches the plain
    sampler's posterior medians (within 0.1 sigma) with far fewer plain
    evaluations."""
    m, truth, lo, hi, free, S = trained
    plain = m.fit_nested(lo, hi, free, truth, n_live=200, seed=11)
    scr = S.fit_nested(m, lo, hi, free, truth, margin=25.0, audit=0.02, n_live=200, seed=11)
    print("plain evals", plain["n_evals"], "screened plain evals", scr["n_evals"],
          "screened", scr["n_screened"], "rejected", scr["n_rejected"],
          "audited", scr["n_audited"], "misses", scr["n_audit_miss"])
    print("logz plain", plain["logz"], "screened", scr["logz"])
    assert scr["status"] == 0
    for k in range(12):
        if free[k]:
            assert abs(scr["median"][k] - plain["median"][k]) <= 0.1 * plain["sd"][k], k
    assert abs(scr["logz"] - plain["logz"]) < 3 * plain["logz_err"]
    assert scr["n_evals"] < 0.5 * plain["n_evals"]


def test_screened_nested_sampling_skips_unprofitable_rounds(gbk, trained):
    """With the screen priced above a plain evaluation (screen_cost 2) a round
    is screened only every 8th time: far fewer candidates reach the network,
    and the posterior still matches the plain sampler's."""
    m, truth, lo, hi, free, S = trained
    plain = m.fit_nested(lo, hi, free, truth, n_live=200, seed=11)
    always = S.fit_nested(m, lo, hi, free, truth, margin=25.0, audit=0.02, n_live=200, seed=11)
    rare = S.fit_nested(m, lo, hi, free, truth, margin=25.0, audit=0.02, n_live=200, seed=11,
                        screen_cost=2.0)
    total = rare["n_evals"] + rare["n_rejected"]  # every candidate of the run
    print("screened", rare["n_screened"], "of", total, "(always:", always["n_screened"], ")")
    assert rare["status"] == 0
    assert 0 < rare["n_screened"] < 0.3 * total
    assert always["n_screened"] == always["n_evals"] + always["n_rejected"]
    for k in range(12):
        if free[k]:
            assert abs(rare["median"][k] - plain["median"][k]) <= 0.1 * plain["sd"][k], k
    assert abs(rare["logz"] - plain["logz"]) < 3 * plain["logz_err"]


def test_surrogate_save_and_load_round_trip(O, gbk, tmp_path):
    """A saved surrogate loads with the same weights and predicts the same maps;
    another instrument, a foreign file and a missing file are refused."""
    grid, lo, hi, opts = small_setup(O)
    m = gbk.Model.from_grid(grid)
    S = gbk.Surrogate(m, lo, hi, **opts)
    S.train(20)
    path = str(tmp_path / "net.gks")
    S.save(path)
    T = gbk.Surrogate.load(m, path)
    np.testing.assert_array_equal(S.get_weights(), T.get_weights())
    rows = draw_rows(np.random.default_rng(5), lo, hi, 64)
    np.testing.assert_array_equal(S.predict(rows).cpu().numpy(), T.predict(rows).cpu().numpy())
    other = gbk.Model.from_grid(I.Grid(16, 16, 32, 25.0, psf_fwhm=2.0, lsf_sigma=30.0))
    with pytest.raises(gbk.GkError):
        gbk.Surrogate.load(other, path)                               # other channel width
    bad = tmp_path / "bad.gks"
    bad.write_bytes(b"GKSURR01" + bytes(16))
    with pytest.raises(gbk.GkError):
        gbk.Surrogate.load(m, str(bad))                               # truncated
    with pytest.raises(gbk.GkError):
        gbk.Surrogate.load(m, str(tmp_path / "missing.gks"))
    T.close()
    S.close()


def test_surrogate_rejects_bad_arguments(O, gbk):
    grid, lo, hi, opts = small_setup(O)
    m = gbk.Model.from_grid(grid)
    with pytest.raises(gbk.GkError):
        gbk.Surrogate(m, lo, hi, hidden=48, layers=2, batch=32)   # width not a multiple of 32
    bad = hi.copy()
    bad[3] = 95.0
    with pytest.raises(gbk.GkError):
        gbk.Surrogate(m, lo, bad, **opts)                          # box leaves the domain
    odd = gbk.Model.from_grid(I.Grid(15, 15, 32, 30.0, psf_fwhm=2.0, lsf_sigma=30.0))
    with pytest.raises(gbk.GkError):
        gbk.Surrogate(odd, lo, hi, **opts)                         # nx ny not a multiple of 16
    S = gbk.Surrogate(m, lo, hi, **opts)
    other = gbk.Model.from_grid(I.Grid(16, 16, 40, 30.0, psf_fwhm=2.0, lsf_sigma=30.0))
    with pytest.raises(gbk.GkError):
        S.chi2(other, np.tile(lo, (2, 1)))                          # instrument differs / no obs
    S.close()
