// gbk_ns.hip -- batched single-ellipsoid nested sampling (Sec. 2.3.2) and the
// Philox4x32-10 counter-based generator it draws from.
//
// The driver is generic over a batch log-likelihood; gk_fit_nested plugs in
// the model's chi-square (one launch per round), gk_fit_nested_screened the
// surrogate screen in front of it, gk_nested_sample a host callback.  The
// algorithm is written out in gbk.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cfloat>
#include <cmath>
#include <cstring>
#include <functional>
#include <numeric>
#include <vector>

#include "gbk_model.h"
#include "gbk_rng.h"
#include "gbk_surrogate.h"

using namespace gbk;

namespace {

double logaddexp(double a, double b)
{
    if (a == -INFINITY) return b;
    if (b == -INFINITY) return a;
    const double m = std::max(a, b);
    return m + std::log1p(std::exp(-std::fabs(a - b)));
}

// Lower Cholesky factor of a d x d SPD matrix in place; false if not SPD.
bool cholesky(std::vector<double> &M, int d)
{
    for (int i = 0; i < d; ++i)
        for (int j = 0; j <= i; ++j) {
            double s = M[i * d + j];
            for (int k = 0; k < j; ++k) s -= M[i * d + k] * M[j * d + k];
            if (i == j) {
                if (!(s > 0.0)) return false;
                M[i * d + i] = std::sqrt(s);
            } else {
                M[i * d + j] = s / M[j * d + j];
            }
        }
    for (int i = 0; i < d; ++i)
        for (int j = i + 1; j < d; ++j) M[i * d + j] = 0.0;
    return true;
}

// Volume of the unit d-ball.
double ball_volume(int d) { return std::pow(M_PI, 0.5 * d) / std::tgamma(0.5 * d + 1.0); }

// Batch log-likelihood of n unit-cube points; floor is the lowest live
// log-likelihood when the batch was drawn (candidates at or below it cannot
// be accepted in this round).
using BatchLogL = std::function<gk_status(const std::vector<double> &u, int n, double floor,
                                          std::vector<double> &logl)>;

struct Point {
    std::vector<double> u;
    double logl;
};

// Runs the sampler in the unit cube [0,1]^d; eval maps unit-cube points to
// log-likelihoods.  Fills the posterior in unit-cube coordinates through
// `post` (u, normalised weight) and the evidence fields of res.
gk_status ns_run(int d, const BatchLogL &eval, const gk_ns_opts &o, gk_ns_result *res,
                 std::vector<std::pair<std::vector<double>, double>> &post, bool &capped)
{
    const int N = o.n_live, B = o.batch;
    Rng rng(o.seed, 0x6e73u);
    std::vector<Point> live(N);
    std::vector<double> ub((size_t)std::max(N, B) * d), lb;
    for (int i = 0; i < N; ++i)
        for (int k = 0; k < d; ++k) ub[(size_t)i * d + k] = rng.uniform();
    GK_TRY(eval(ub, N, -DBL_MAX, lb));
    int64_t n_evals = N, n_launch = 1;
    for (int i = 0; i < N; ++i) {
        live[i].u.assign(ub.begin() + (size_t)i * d, ub.begin() + (size_t)(i + 1) * d);
        live[i].logl = std::isfinite(lb[i]) ? lb[i] : -DBL_MAX;
    }
    std::vector<Point> dead;
    std::vector<double> dead_logwt;
    double logz = -INFINITY, max_logl = -INFINITY;
    std::vector<double> best;
    for (auto &p : live)
        if (p.logl > max_logl) {
            max_logl = p.logl;
            best = p.u;
        }
    // min-heap of (logl, index): the lowest live point, ties to the lowest index
    std::vector<std::pair<double, int>> heap(N);
    for (int i = 0; i < N; ++i) heap[i] = {live[i].logl, i};
    std::make_heap(heap.begin(), heap.end(), std::greater<>());
    const double log_shrink = std::log1p(-std::exp(-1.0 / N));  // log(1 - e^{-1/N})
    int64_t k = 0;
    bool done = false;
    capped = false;
    std::vector<double> mu(d), C((size_t)d * d), L((size_t)d * d), z(d);
    while (!done) {
        // bounding ellipsoid of the live points (unit-cube coordinates)
        std::fill(mu.begin(), mu.end(), 0.0);
        for (auto &p : live)
            for (int a = 0; a < d; ++a) mu[a] += p.u[a] / N;
        std::fill(C.begin(), C.end(), 0.0);
        for (auto &p : live)
            for (int a = 0; a < d; ++a)
                for (int b = 0; b < d; ++b) C[a * d + b] += (p.u[a] - mu[a]) * (p.u[b] - mu[b]) / N;
        for (int a = 0; a < d; ++a) C[a * d + a] += 1e-12;
        L = C;
        bool ell = cholesky(L, d);
        double kmax = 0.0;
        if (ell) {
            for (auto &p : live) {  // Mahalanobis radius^2: solve L y = u - mu
                double m2 = 0.0;
                for (int a = 0; a < d; ++a) {
                    double s = p.u[a] - mu[a];
                    for (int b = 0; b < a; ++b) s -= L[a * d + b] * z[b];
                    z[a] = s / L[a * d + a];
                    m2 += z[a] * z[a];
                }
                kmax = std::max(kmax, m2);
            }
            const double scale2 = kmax * std::pow(o.enlarge, 2.0 / d);
            double logdet = 0.0;
            for (int a = 0; a < d; ++a) logdet += std::log(L[a * d + a]);
            const double logvol = std::log(ball_volume(d)) + 0.5 * d * std::log(scale2) + logdet;
            if (logvol >= 0.0) ell = false;  // the ellipsoid is larger than the box
            for (double &v : L) v *= std::sqrt(scale2);
        }
        // candidates inside the ellipsoid and the unit cube
        for (int c = 0; c < B; ++c) {
            double *u = &ub[(size_t)c * d];
            for (int tries = 0;; ++tries) {
                if (!ell || tries > 100000) {
                    for (int a = 0; a < d; ++a) u[a] = rng.uniform();
                    break;
                }
                double nrm = 0.0;
                for (int a = 0; a < d; ++a) {
                    z[a] = rng.normal();
                    nrm += z[a] * z[a];
                }
                const double rad = std::pow(rng.uniform(), 1.0 / d) / std::sqrt(nrm);
                bool inside = true;
                for (int a = 0; a < d; ++a) {
                    double s = mu[a];
                    for (int b = 0; b <= a; ++b) s += L[a * d + b] * z[b] * rad;
                    u[a] = s;
                    inside = inside && s > 0.0 && s < 1.0;
                }
                if (inside) break;
            }
        }
        GK_TRY(eval(ub, B, heap.front().first, lb));
        n_evals += B;
        ++n_launch;
        for (int c = 0; c < B && !done; ++c) {
            const double lc = std::isfinite(lb[c]) ? lb[c] : -DBL_MAX;
            const int imin = heap.front().second;
            if (!(lc > live[imin].logl)) continue;
            std::pop_heap(heap.begin(), heap.end(), std::greater<>());
            heap.back() = {lc, imin};
            std::push_heap(heap.begin(), heap.end(), std::greater<>());
            ++k;
            const double logwt = live[imin].logl + (-(double)(k - 1) / N + log_shrink);
            logz = logaddexp(logz, logwt);
            dead.push_back(live[imin]);
            dead_logwt.push_back(logwt);
            live[imin].u.assign(ub.begin() + (size_t)c * d, ub.begin() + (size_t)(c + 1) * d);
            live[imin].logl = lc;
            if (lc > max_logl) {
                max_logl = lc;
                best = live[imin].u;
            }
            // the retired point is the lowest, so the live maximum is the running one
            if (logaddexp(logz, max_logl - (double)k / N) - logz < o.tol) done = true;
            if (k >= o.max_iter) {
                done = true;
                capped = true;
            }
        }
    }
    // final live points with weight X_k / N
    for (auto &p : live) {
        const double logwt = p.logl - (double)k / N - std::log((double)N);
        logz = logaddexp(logz, logwt);
        dead.push_back(p);
        dead_logwt.push_back(logwt);
    }
    double H = 0.0;
    post.clear();
    post.reserve(dead.size());
    for (size_t i = 0; i < dead.size(); ++i) {
        const double pw = std::exp(dead_logwt[i] - logz);
        if (pw > 0.0 && dead[i].logl > -DBL_MAX) H += pw * (dead[i].logl - logz);
        post.emplace_back(dead[i].u, pw);
    }
    res->logz = logz;
    res->info_h = H;
    res->logz_err = std::sqrt(std::max(H, 0.0) / N);
    res->max_logl = max_logl;
    res->n_iter = k;
    res->n_evals = n_evals;
    res->n_launches = n_launch;
    for (int a = 0; a < d; ++a) res->best[a] = best.empty() ? 0.0 : best[a];
    return GK_OK;
}

// Weighted mean, sd and quantiles of coordinate a of the posterior.
void posterior_stats(const std::vector<std::pair<std::vector<double>, double>> &post, int a,
                     double scale, double offset, gk_ns_result *res, int slot)
{
    std::vector<std::pair<double, double>> v;
    v.reserve(post.size());
    double m = 0.0, w = 0.0;
    for (auto &p : post) {
        const double x = offset + scale * p.first[a];
        v.emplace_back(x, p.second);
        m += p.second * x;
        w += p.second;
    }
    m /= w;
    double var = 0.0;
    for (auto &x : v) var += x.second * (x.first - m) * (x.first - m);
    res->mean[slot] = m;
    res->sd[slot] = std::sqrt(var / w);
    std::sort(v.begin(), v.end());
    auto quant = [&](double q) {
        double c = 0.0;
        for (size_t i = 0; i < v.size(); ++i) {
            const double nc = c + v[i].second / w;
            if (nc >= q) {
                if (i == 0 || v[i].second == 0.0) return v[i].first;
                const double t = (q - c) / (nc - c);  // interpolate inside the step
                return v[i - 1].first + t * (v[i].first - v[i - 1].first);
            }
            c = nc;
        }
        return v.back().first;
    };
    res->q16[slot] = quant(0.16);
    res->median[slot] = quant(0.5);
    res->q84[slot] = quant(0.84);
}

gk_status check_opts(const gk_ns_opts &o)
{
    if (o.n_live < 2 || o.batch < 1 || o.max_iter < 1 || !(o.enlarge >= 1.0) || !(o.tol > 0.0))
        return fail(GK_EINVAL, "invalid nested-sampling options");
    return GK_OK;
}

}  // namespace

extern "C" gk_status gk_philox4x32(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    if (!ctr || !key || !out) return fail(GK_EINVAL, "NULL argument");
    philox4x32_10(ctr, key, out);
    return GK_OK;
}

extern "C" gk_status gk_ns_default_opts(gk_ns_opts *o)
{
    if (!o) return fail(GK_EINVAL, "opts is NULL");
    o->n_live = 400;
    o->batch = 400;
    o->max_iter = 1000000;
    o->enlarge = 1.25;
    o->tol = 0.5;
    o->seed = 1;
    return GK_OK;
}

extern "C" gk_status gk_nested_sample(int32_t dim, const double *lo, const double *hi,
                                      gk_loglike_fn fn, void *user, const gk_ns_opts *o_in,
                                      gk_ns_result *res, double *samples, int64_t cap,
                                      int64_t *n_samples)
{
    if (dim < 1 || dim > GK_NP || !lo || !hi || !fn || !res)
        return fail(GK_EINVAL, "invalid arguments");
    gk_ns_opts o;
    gk_ns_default_opts(&o);
    if (o_in) o = *o_in;
    GK_TRY(check_opts(o));
    for (int a = 0; a < dim; ++a)
        if (!(hi[a] > lo[a])) return fail(GK_EINVAL, "empty prior range in dimension %d", a);
    std::vector<double> theta;
    BatchLogL eval = [&](const std::vector<double> &u, int n, double, std::vector<double> &logl) -> gk_status {
        theta.resize((size_t)n * dim);
        for (int i = 0; i < n; ++i)
            for (int a = 0; a < dim; ++a)
                theta[(size_t)i * dim + a] = lo[a] + u[(size_t)i * dim + a] * (hi[a] - lo[a]);
        logl.resize(n);
        if (fn(theta.data(), n, dim, logl.data(), user) != 0)
            return fail(GK_EINVAL, "likelihood callback failed");
        return GK_OK;
    };
    std::memset(res, 0, sizeof *res);
    std::vector<std::pair<std::vector<double>, double>> post;
    bool capped = false;
    GK_TRY(ns_run(dim, eval, o, res, post, capped));
    for (int a = 0; a < dim; ++a) {
        res->best[a] = lo[a] + res->best[a] * (hi[a] - lo[a]);
        posterior_stats(post, a, hi[a] - lo[a], lo[a], res, a);
    }
    if (samples && n_samples) {
        const int64_t n = std::min<int64_t>(cap, (int64_t)post.size());
        for (int64_t i = 0; i < n; ++i) {
            for (int a = 0; a < dim; ++a)
                samples[i * (GK_NP + 1) + a] = lo[a] + post[i].first[a] * (hi[a] - lo[a]);
            samples[i * (GK_NP + 1) + GK_NP] = post[i].second;
        }
        *n_samples = n;
    }
    return capped ? GK_ENOTCONV : GK_OK;
}

// Workspace of gk_fit_nested lives in the fitter workspace of the model.
namespace gbk {
gk_status fit_reserve_rows(gk_model *m, int rows, double **h_params, double **d_params,
                           double **d_chi2, double **h_chi2, hipStream_t *stream);
}

namespace {

// Plain (s == NULL) or surrogate-screened nested sampling of a model.
gk_status fit_nested(gk_model *m, gk_surrogate *sur, const double *lo, const double *hi,
                     const uint8_t *free_mask, const double *fixed, const gk_ns_opts *o_in,
                     double margin, double audit, gk_ns_result *res, double *samples, int64_t cap,
                     int64_t *n_samples)
{
    if (!m || !lo || !hi || !free_mask || !fixed || !res) return fail(GK_EINVAL, "NULL argument");
    if (!m->has_obs) return fail(GK_ESTATE, "no observation set");
    gk_ns_opts o;
    gk_ns_default_opts(&o);
    if (o_in) o = *o_in;
    GK_TRY(check_opts(o));
    if (sur) {
        if (!(margin >= 0.0) || !(audit >= 0.0 && audit <= 1.0))
            return fail(GK_EINVAL, "margin must be >= 0 and audit in [0, 1]");
        if (!surrogate_matches(sur, m)) return fail(GK_EINVAL, "model instrument differs from the surrogate's");
        if (surrogate_device(sur) != m->device) return fail(GK_EINVAL, "model and surrogate on different devices");
    }
    std::vector<int> fr;
    for (int k = 0; k < NPAR; ++k) {
        if (!free_mask[k]) continue;
        if (!(hi[k] > lo[k])) return fail(GK_EINVAL, "empty prior range in slot %d", k);
        fr.push_back(k);
    }
    const int d = (int)fr.size();
    if (d == 0) return fail(GK_EINVAL, "no free parameter");
    DeviceGuard g(m->device);
    HIP_TRY(g.err);
    double *h_params, *d_params, *d_chi2, *h_chi2;
    hipStream_t stream;
    const int rows = std::max(o.n_live, o.batch);
    // chi2 rows, then (screened) surrogate chi2 rows
    GK_TRY(fit_reserve_rows(m, 2 * rows, &h_params, &d_params, &d_chi2, &h_chi2, &stream));
    double *d_chi2s = d_chi2 + rows, *h_chi2s = h_chi2 + rows;
    std::memset(res, 0, sizeof *res);
    auto fill_rows = [&](const std::vector<double> &u, const std::vector<int> &idx) {
        for (size_t i = 0; i < idx.size(); ++i) {
            double *row = h_params + i * NPAR;
            std::memcpy(row, fixed, sizeof(double) * NPAR);
            for (int a = 0; a < d; ++a)
                row[fr[a]] = lo[fr[a]] + u[(size_t)idx[i] * d + a] * (hi[fr[a]] - lo[fr[a]]);
        }
    };
    // plain chi2 of the rows in h_params [0, n) into h_chi2
    auto plain = [&](int n) -> gk_status {
        if (n == 0) return GK_OK;
        HIP_TRY(hipMemcpyAsync(d_params, h_params, sizeof(double) * NPAR * n, hipMemcpyHostToDevice,
                               stream));
        GK_TRY(run_batch(m, d_params, n, nullptr, nullptr, d_chi2, nullptr, stream));
        HIP_TRY(hipMemcpyAsync(h_chi2, d_chi2, sizeof(double) * n, hipMemcpyDeviceToHost, stream));
        HIP_TRY(hipStreamSynchronize(stream));
        return GK_OK;
    };
    std::vector<int> all, keep;
    int64_t n_plain = 0;
    Rng audit_rng(o.seed, 0x617564u);
    std::vector<double> recent;  // surrogate-minus-plain chi2 of the latest plain evaluations
    size_t recent_pos = 0;
    double shift = 0.0;
    BatchLogL eval = [&](const std::vector<double> &u, int n, double floor,
                         std::vector<double> &logl) -> gk_status {
        logl.assign(n, -INFINITY);
        all.resize(n);
        std::iota(all.begin(), all.end(), 0);
        keep.clear();
        if (!sur) {
            fill_rows(u, all);
            GK_TRY(plain(n));
            n_plain += n;
            for (int i = 0; i < n; ++i) logl[i] = -0.5 * h_chi2[i];
            return GK_OK;
        }
        // surrogate chi2 of every candidate
        fill_rows(u, all);
        HIP_TRY(hipMemcpyAsync(d_params, h_params, sizeof(double) * NPAR * n, hipMemcpyHostToDevice,
                               stream));
        GK_TRY(surrogate_chi2(sur, m, d_params, n, d_chi2s, stream));
        HIP_TRY(hipMemcpyAsync(h_chi2s, d_chi2s, sizeof(double) * n, hipMemcpyDeviceToHost, stream));
        HIP_TRY(hipStreamSynchronize(stream));
        const double chi2_floor = floor > -DBL_MAX ? -2.0 * floor : INFINITY;
        const double cut = chi2_floor + shift + margin;
        std::vector<char> audited(n, 0);
        for (int i = 0; i < n; ++i) {
            const double a = audit_rng.uniform();  // one draw per candidate, used or not
            if (!(h_chi2s[i] > cut)) {
                keep.push_back(i);
            } else if (a < audit) {
                keep.push_back(i);
                audited[i] = 1;
            }
        }
        res->n_screened += n;
        res->n_rejected += n - (int64_t)keep.size();
        fill_rows(u, keep);
        GK_TRY(plain((int)keep.size()));
        n_plain += (int64_t)keep.size();
        const size_t window = (size_t)std::max(o.n_live, o.batch);
        for (size_t j = 0; j < keep.size(); ++j) {
            const int i = keep[j];
            const double c = h_chi2[j];
            logl[i] = -0.5 * c;
            if (audited[i]) {
                res->n_audited += 1;
                res->n_audit_miss += c < chi2_floor;
            }
            const double delta = h_chi2s[i] - c;
            if (std::isfinite(delta)) {
                if (recent.size() < window) {
                    recent.push_back(delta);
                } else {
                    recent[recent_pos] = delta;
                    recent_pos = (recent_pos + 1) % window;
                }
            }
        }
        shift = 0.0;
        for (double v : recent) shift = std::max(shift, v);
        return GK_OK;
    };
    std::vector<std::pair<std::vector<double>, double>> post;
    bool capped = false;
    GK_TRY(ns_run(d, eval, o, res, post, capped));
    res->n_evals = n_plain;  // plain evaluations only
    double best_u[GK_NP];
    std::memcpy(best_u, res->best, sizeof best_u);
    for (int k = 0; k < NPAR; ++k) {
        res->best[k] = res->mean[k] = res->median[k] = res->q16[k] = res->q84[k] = fixed[k];
        res->sd[k] = 0.0;
    }
    for (int a = 0; a < d; ++a) {
        const int k = fr[a];
        res->best[k] = lo[k] + best_u[a] * (hi[k] - lo[k]);
        posterior_stats(post, a, hi[k] - lo[k], lo[k], res, k);
    }
    if (samples && n_samples) {
        const int64_t n = std::min<int64_t>(cap, (int64_t)post.size());
        for (int64_t i = 0; i < n; ++i) {
            double *row = samples + i * (GK_NP + 1);
            std::memcpy(row, fixed, sizeof(double) * NPAR);
            for (int a = 0; a < d; ++a)
                row[fr[a]] = lo[fr[a]] + post[i].first[a] * (hi[fr[a]] - lo[fr[a]]);
            row[GK_NP] = post[i].second;
        }
        *n_samples = n;
    }
    return capped ? GK_ENOTCONV : GK_OK;
}

}  // namespace

extern "C" gk_status gk_fit_nested(gk_model *m, const double *lo, const double *hi,
                                   const uint8_t *free_mask, const double *fixed,
                                   const gk_ns_opts *o_in, gk_ns_result *res, double *samples,
                                   int64_t cap, int64_t *n_samples)
{
    return fit_nested(m, nullptr, lo, hi, free_mask, fixed, o_in, 0.0, 0.0, res, samples, cap,
                      n_samples);
}

extern "C" gk_status gk_fit_nested_screened(gk_model *m, gk_surrogate *s, const double *lo,
                                            const double *hi, const uint8_t *free_mask,
                                            const double *fixed, const gk_ns_opts *o_in,
                                            double margin, double audit, gk_ns_result *res,
                                            double *samples, int64_t cap, int64_t *n_samples)
{
    if (!s) return fail(GK_EINVAL, "surrogate is NULL");
    return fit_nested(m, s, lo, hi, free_mask, fixed, o_in, margin, audit, res, samples, cap,
                      n_samples);
}
