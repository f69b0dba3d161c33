"""Host logic of the library's nested sampler and random generator (no GPU):
the sampler runs on a Python likelihood through gk_nested_sample."""
import math

import numpy as np
import pytest


def philox_ref(ctr, key):
    """Philox4x32-10 from its published definition (Salmon et al. 2011):
    10 rounds of two 32x32->64 multiplications with a Weyl-sequence key bump."""
    M0, M1, W0, W1 = 0xD2511F53, 0xCD9E8D57, 0x9E3779B9, 0xBB67AE85
    c = list(ctr)
    k0, k1 = key
    for r in range(10):
        if r:
            k0 = (k0 + W0) & 0xFFFFFFFF
            k1 = (k1 + W1) & 0xFFFFFFFF
        p0, p1 = M0 * c[0], M1 * c[2]
        c = [((p1 >> 32) ^ c[1] ^ k0) & 0xFFFFFFFF, p1 & 0xFFFFFFFF,
             ((p0 >> 32) ^ c[3] ^ k1) & 0xFFFFFFFF, p0 & 0xFFFFFFFF]
    return c


def test_philox_known_answer_and_reference():
    from paper_1510_01815_amd import gbk
    # published known-answer vector: zero counter, zero key
    assert gbk.philox4x32([0, 0, 0, 0], [0, 0]) == [0x6627E8D5, 0xE169C58D, 0xBC57AC4C, 0x9B00DBD8]
    rng = np.random.default_rng(0)
    for _ in range(50):
        ctr = [int(v) for v in rng.integers(0, 2**32, 4)]
        key = [int(v) for v in rng.integers(0, 2**32, 2)]
        assert gbk.philox4x32(ctr, key) == philox_ref(ctr, key)


def gauss_loglike(mu, sig):
    def f(th):
        return -0.5 * np.sum(((th[:, : len(mu)] - mu) / sig) ** 2, axis=1)
    return f


@pytest.mark.parametrize("batch", [100, 400])
def test_ns_gaussian_evidence_and_moments(batch):
    """3-D Gaussian likelihood in a wide box: log Z = sum log(sigma sqrt(2 pi)
    / width); posterior mean mu, sd sigma, 16/50/84% at mu -/+ sigma.  A 4th
    parameter absent from the likelihood keeps its uniform prior."""
    from paper_1510_01815_amd import gbk
    mu = np.array([1.0, -2.0, 0.5])
    sig = np.array([0.5, 1.0, 0.2])
    lo = np.array([-6.0, -10.0, -2.0, 0.0])
    hi = np.array([6.0, 8.0, 3.0, 4.0])
    r = gbk.nested_sample(gauss_loglike(mu, sig), lo, hi, n_live=400, batch=batch, seed=7)
    logz_true = float(np.sum(np.log(sig * math.sqrt(2 * math.pi) / (hi[:3] - lo[:3]))))
    print(r["logz"], r["logz_err"], logz_true, r["n_iter"], r["n_evals"], r["n_launches"])
    assert r["status"] == 0
    assert abs(r["logz"] - logz_true) < 3 * r["logz_err"] + 0.1
    np.testing.assert_allclose(r["mean"][:3], mu, atol=0.1 * sig.max())
    np.testing.assert_allclose(r["sd"][:3], sig, rtol=0.1)
    assert np.all(np.abs(r["median"][:3] - mu) <= 0.12 * sig)
    assert np.all(np.abs(r["q16"][:3] - (mu - sig)) <= 0.15 * sig)
    assert np.all(np.abs(r["q84"][:3] - (mu + sig)) <= 0.15 * sig)
    # flat direction: marginal = prior U[0, 4]
    assert abs(r["mean"][3] - 2.0) < 0.15 and abs(r["sd"][3] - 4 / math.sqrt(12)) < 0.1
    assert abs(r["max_logl"]) < 0.5


def test_ns_reproducible_and_samples():
    from paper_1510_01815_amd import gbk
    f = gauss_loglike(np.array([0.3]), np.array([0.1]))
    a = gbk.nested_sample(f, [-1.0], [1.0], want_samples=100000, n_live=100, seed=3)
    b = gbk.nested_sample(f, [-1.0], [1.0], want_samples=100000, n_live=100, seed=3)
    c = gbk.nested_sample(f, [-1.0], [1.0], n_live=100, seed=4)
    assert a["logz"] == b["logz"] and (a["samples"] == b["samples"]).all()
    assert a["logz"] != c["logz"]
    w = a["samples"][:, -1]
    assert abs(w.sum() - 1.0) < 1e-9 and len(w) == a["n_iter"] + 100
    assert abs(np.sum(w * a["samples"][:, 0]) - a["mean"][0]) < 1e-12


def test_ns_callback_failure_is_an_error():
    from paper_1510_01815_amd import gbk

    def bad(th):
        raise RuntimeError("boom")
    with pytest.raises(gbk.GkError):
        gbk.nested_sample(bad, [0.0], [1.0], n_live=10)


def test_ns_two_modes_split_bound():
    """Two separated Gaussian modes of equal mass: the evidence is analytic,
    each mode carries half the posterior, and the multi-ellipsoid bound needs
    far fewer evaluations than one ellipsoid."""
    from paper_1510_01815_amd import gbk

    def f(th):
        a = np.sum((th - np.array([-3.0, 0.0])) ** 2, axis=1)
        b = np.sum((th - np.array([3.0, 0.0])) ** 2, axis=1)
        return np.logaddexp(-a / 0.18, -b / 0.18)  # sigma = 0.3
    lo, hi = np.array([-6.0, -6.0]), np.array([6.0, 6.0])
    true = math.log(2 * 2 * math.pi * 0.09 / 144)
    multi = gbk.nested_sample(f, lo, hi, want_samples=100000, n_live=400, seed=3)
    single = gbk.nested_sample(f, lo, hi, n_live=400, seed=3, max_ell=1)
    for r in (multi, single):
        assert abs(r["logz"] - true) < 3 * r["logz_err"] + 0.1
    w, x = multi["samples"][:, -1], multi["samples"][:, 0]
    assert abs(w[x < 0].sum() - 0.5) < 0.1
    assert multi["n_evals"] < 0.6 * single["n_evals"]


def test_ns_curved_posterior():
    """Banana likelihood exp(-x^2/2 - (y - x^2)^2 / (2 0.1^2)): Z, the
    moments of x ~ N(0, 1) and of y = x^2 + N(0, 0.01) (mean 1, variance
    2.01) are analytic; the split bound follows the curve with several times
    fewer evaluations."""
    from paper_1510_01815_amd import gbk

    def f(th):
        x, y = th[:, 0], th[:, 1]
        return -x ** 2 / 2 - (y - x ** 2) ** 2 / 0.02
    lo, hi = np.array([-5.0, -2.0]), np.array([5.0, 28.0])
    true = math.log(2 * math.pi * 0.1 / 300)
    multi = gbk.nested_sample(f, lo, hi, n_live=400, seed=5)
    single = gbk.nested_sample(f, lo, hi, n_live=400, seed=5, max_ell=1)
    for r in (multi, single):
        assert abs(r["logz"] - true) < 3 * r["logz_err"] + 0.1
        assert abs(r["mean"][0]) < 0.1 and abs(r["sd"][0] - 1.0) < 0.1
        assert abs(r["mean"][1] - 1.0) < 0.15 and abs(r["sd"][1] - math.sqrt(2.01)) < 0.15
    assert multi["n_evals"] < 0.4 * single["n_evals"]


def test_ns_adaptive_batch_keeps_the_statistics():
    """Where the bound fits poorly (one ellipsoid on the curved likelihood) a
    batch that grows with falling acceptance needs far fewer rounds, and the
    evidence and posterior moments stay within their errors."""
    from paper_1510_01815_amd import gbk

    def f(th):
        x, y = th[:, 0], th[:, 1]
        return -x ** 2 / 2 - (y - x ** 2) ** 2 / 0.02
    lo, hi = np.array([-5.0, -2.0]), np.array([5.0, 28.0])
    true = math.log(2 * math.pi * 0.1 / 300)
    fixed = gbk.nested_sample(f, lo, hi, n_live=400, seed=5, max_ell=1)
    grow = gbk.nested_sample(f, lo, hi, n_live=400, seed=5, max_ell=1, batch_max=6400)
    assert grow["n_launches"] < 0.5 * fixed["n_launches"]
    for r in (fixed, grow):
        assert abs(r["logz"] - true) < 3 * r["logz_err"] + 0.1
        assert abs(r["mean"][0]) < 0.1 and abs(r["sd"][0] - 1.0) < 0.1
        assert abs(r["mean"][1] - 1.0) < 0.15 and abs(r["sd"][1] - math.sqrt(2.01)) < 0.15
    with pytest.raises(gbk.GkError):
        gbk.nested_sample(f, lo, hi, n_live=400, batch=400, batch_max=100)


def test_ns_accept_target_sets_the_round_size():
    """A larger acceptance target per round (adaptive batch) takes fewer
    rounds; evidence and moments stay within their errors; a negative target
    is rejected."""
    from paper_1510_01815_amd import gbk

    def f(th):
        x, y = th[:, 0], th[:, 1]
        return -x ** 2 / 2 - (y - x ** 2) ** 2 / 0.02
    lo, hi = np.array([-5.0, -2.0]), np.array([5.0, 28.0])
    true = math.log(2 * math.pi * 0.1 / 300)
    small = gbk.nested_sample(f, lo, hi, n_live=400, seed=7, batch=100, batch_max=6400)
    large = gbk.nested_sample(f, lo, hi, n_live=400, seed=7, batch=100, batch_max=6400,
                              accept_target=100)
    assert large["n_launches"] < 0.7 * small["n_launches"]
    for r in (small, large):
        assert abs(r["logz"] - true) < 3 * r["logz_err"] + 0.1
        assert abs(r["mean"][0]) < 0.1 and abs(r["sd"][0] - 1.0) < 0.1
        assert abs(r["mean"][1] - 1.0) < 0.15 and abs(r["sd"][1] - math.sqrt(2.01)) < 0.15
    with pytest.raises(gbk.GkError):
        gbk.nested_sample(f, lo, hi, n_live=400, accept_target=-1)
    for bad in ({"screen_cost": -1.0}, {"screen_rows": -1}, {"screen_cost": float("nan")}):
        with pytest.raises(gbk.GkError):
            gbk.nested_sample(f, lo, hi, n_live=400, **bad)


def mixture_loglike(ws, mus, sig):
    """log of sum_k w_k N(theta; mu_k, sig^2 I) (normalised densities)."""
    mus = np.asarray(mus)
    d = mus.shape[1]

    def f(th):
        x = th[:, :d]
        terms = [math.log(w) - 0.5 * np.sum(((x - m) / sig) ** 2, axis=1)
                 - d * math.log(sig * math.sqrt(2 * math.pi)) for w, m in zip(ws, mus)]
        return np.logaddexp.reduce(np.stack(terms), axis=0)
    return f


@pytest.mark.parametrize("batch", [200, 800])
def test_ns_mode_separation_two_gaussians(batch):
    """Two well separated normal components of weights 0.3 and 0.7 in a box of
    volume V: with mode separation the sampler finds two modes whose local
    evidences are w_k / V (closed form: each component integrates to its
    weight, its mass outside the box is < 1e-20), with means at the
    component centres and sd sigma; the total evidence is 1 / V.  Without
    mode separation the run still gets the total evidence, as one mode."""
    from paper_1510_01815_amd import gbk
    ws, sig = (0.3, 0.7), 0.5
    mus = [[-3.0, -3.0, 0.0], [3.0, 2.0, 1.0]]
    lo, hi = np.full(3, -8.0), np.full(3, 8.0)
    logV = 3 * math.log(16.0)
    f = mixture_loglike(ws, mus, sig)
    r = gbk.nested_sample(f, lo, hi, n_live=400, batch=batch, seed=3, separate_modes=1)
    print("logz", r["logz"], "+-", r["logz_err"], "closed form", -logV, "modes", len(r["modes"]))
    assert r["status"] == 0
    assert abs(r["logz"] + logV) < 3 * r["logz_err"] + 0.05
    assert len(r["modes"]) == 2
    found = sorted(r["modes"], key=lambda m: m["mean"][0])
    for md, w, mu in zip(found, ws, mus):
        print("  mode logz", md["logz"], "+-", md["logz_err"], "closed form", math.log(w) - logV,
              "mean", md["mean"], "sd", md["sd"], "live", md["n_live"])
        assert abs(md["logz"] - (math.log(w) - logV)) < 3 * md["logz_err"] + 0.1
        np.testing.assert_allclose(md["mean"], mu, atol=0.1 * sig)
        np.testing.assert_allclose(md["sd"], sig, rtol=0.12)
        assert abs(md["median"][0] - mu[0]) < 0.12 * sig
    assert sum(m["n_live"] for m in found) == 400
    one = gbk.nested_sample(f, lo, hi, n_live=400, batch=batch, seed=3)
    assert len(one["modes"]) == 1
    assert abs(one["logz"] + logV) < 3 * one["logz_err"] + 0.05
    assert one["modes"][0]["logz"] == one["logz"]


def test_ns_mode_separation_leaves_a_single_mode_alone():
    """A single (correlated) Gaussian: mode separation finds one mode and the
    same evidence and moments as the closed form."""
    from paper_1510_01815_amd import gbk
    mu = np.array([1.0, -1.0, 0.5])
    sig = np.array([0.5, 1.0, 0.3])
    lo, hi = np.full(3, -6.0), np.full(3, 6.0)
    r = gbk.nested_sample(gauss_loglike(mu, sig), lo, hi, n_live=400, seed=9, separate_modes=1)
    logz_true = float(np.sum(np.log(sig * math.sqrt(2 * math.pi) / (hi - lo))))
    assert len(r["modes"]) == 1
    assert abs(r["logz"] - logz_true) < 3 * r["logz_err"] + 0.1
    np.testing.assert_allclose(r["mean"], mu, atol=0.1 * sig.max())


def test_ns_wall_time_cap():
    """max_wall_s stops a run at a round boundary once the time is spent: the
    call reports the cap (GK_ENOTCONV) with results from the points so far."""
    import time
    from paper_1510_01815_amd import gbk

    def slow(th):
        time.sleep(0.01)
        return gauss_loglike(np.zeros(3), np.full(3, 0.01))(th)
    lo, hi = np.full(3, -1.0), np.full(3, 1.0)
    t0 = time.perf_counter()
    r = gbk.nested_sample(slow, lo, hi, n_live=100, seed=2, max_wall_s=0.3)
    dt = time.perf_counter() - t0
    assert r["status"] == gbk.GK_ENOTCONV
    assert dt < 2.0 and r["n_iter"] > 0 and np.isfinite(r["logz"])
