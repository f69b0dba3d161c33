// gbk_ns.hip -- batched nested sampling with an ellipsoidal bound (Sec. 2.3.2) and the
// Philox4x32-10 counter-based generator it draws from.
//
// The driver is generic over a batch log-likelihood; gk_fit_nested plugs in
// the model's chi-square (one launch per round), gk_fit_nested_screened the
// surrogate screen in front of it, gk_nested_sample a host callback.  The
// algorithm is written out in gbk.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cfloat>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <functional>
#include <mutex>
#include <new>
#include <numeric>
#include <thread>
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

// Sampling region of a round: the union of up to kMaxEll ellipsoids
// x = mu_e + L_e z, |z| <= 1 (L_e lower triangular, row-major d x d), drawn
// from in proportion to their volumes (cum = cumulative volume fractions),
// or the whole unit cube when n_ell is 0.
constexpr int kMaxEll = 8;
constexpr int kMeansPoints = 256;  // points of the 2-means iterations of a split
struct Bound {
    int n_ell;
    int d;
    double cum[kMaxEll];
    double mu[kMaxEll][GK_NP];
    double L[kMaxEll][GK_NP * GK_NP];
    double inv_diag[kMaxEll][GK_NP];
};

// Enclosing ellipsoid of the points idx[0..n) of U [.][d]: covariance of the
// points scaled to enclose them all, volume enlarged by `enlarge` and raised
// to at least exp(min_logvol).  False if the covariance is not positive
// definite.
bool fit_ellipsoid(const double *U, const int *idx, int n, int d, double enlarge,
                   double min_logvol, double *mu, double *L, double *inv_diag, double &logvol)
{
    double C[GK_NP * GK_NP] = {}, z[GK_NP];
    for (int a = 0; a < d; ++a) mu[a] = 0.0;
    for (int i = 0; i < n; ++i)
        for (int a = 0; a < d; ++a) mu[a] += U[(size_t)idx[i] * d + a];
    for (int a = 0; a < d; ++a) mu[a] /= n;
    for (int i = 0; i < n; ++i) {
        const double *u = &U[(size_t)idx[i] * d];
        for (int a = 0; a < d; ++a) z[a] = u[a] - mu[a];
        for (int a = 0; a < d; ++a)
            for (int b = 0; b <= a; ++b) C[a * d + b] += z[a] * z[b];
    }
    for (int a = 0; a < d; ++a)
        for (int b = 0; b <= a; ++b) C[b * d + a] = C[a * d + b] = C[a * d + b] / n;
    for (int a = 0; a < d; ++a) C[a * d + a] += 1e-12;
    std::vector<double> M(C, C + d * d);
    if (!cholesky(M, d)) return false;
    double invd[GK_NP], kmax = 0.0;
    for (int a = 0; a < d; ++a) invd[a] = 1.0 / M[a * d + a];
    for (int i = 0; i < n; ++i) {  // Mahalanobis radius^2: solve M y = u - mu
        const double *u = &U[(size_t)idx[i] * d];
        double m2 = 0.0;
        for (int a = 0; a < d; ++a) {
            double s = u[a] - mu[a];
            for (int b = 0; b < a; ++b) s -= M[a * d + b] * z[b];
            z[a] = s * invd[a];
            m2 += z[a] * z[a];
        }
        kmax = std::max(kmax, m2);
    }
    double logdet = 0.0;
    for (int a = 0; a < d; ++a) logdet += std::log(M[a * d + a]);
    double scale2 = kmax * std::pow(enlarge, 2.0 / d);
    logvol = std::log(ball_volume(d)) + 0.5 * d * std::log(scale2) + logdet;
    if (logvol < min_logvol) {  // expand to the expected prior volume of its points
        scale2 *= std::exp(2.0 * (min_logvol - logvol) / d);
        logvol = min_logvol;
    }
    const double sc = std::sqrt(scale2);
    for (int k = 0; k < d * d; ++k) L[k] = M[k] * sc;
    for (int a = 0; a < d; ++a) inv_diag[a] = 1.0 / L[a * d + a];
    return true;
}

// Region of the live points U [N][d] at prior volume exp(logX): one
// enclosing ellipsoid, split recursively in two (2-means in unit-cube
// coordinates) while the two children's volumes sum to less than half the
// parent's and each child keeps at least 2 (d + 1) points, up to max_ell
// ellipsoids (MultiNest's decomposition, simplified).  An ellipsoid is never
// smaller than the prior volume its points stand for, n_e X / N.
void build_bound(const double *U, int N, int d, double enlarge, double logX, int max_ell, Bound &bnd)
{
    bnd.d = d;
    bnd.n_ell = 0;
    struct Node {
        std::vector<int> idx;
        double mu[GK_NP], L[GK_NP * GK_NP], invd[GK_NP], logvol;
    };
    auto min_vol = [&](int n) { return logX + std::log((double)n / N); };
    std::vector<Node> done, todo(1);
    todo[0].idx.resize(N);
    std::iota(todo[0].idx.begin(), todo[0].idx.end(), 0);
    if (!fit_ellipsoid(U, todo[0].idx.data(), N, d, enlarge, min_vol(N), todo[0].mu, todo[0].L,
                       todo[0].invd, todo[0].logvol))
        return;  // degenerate: the whole cube
    std::vector<double> w;
    while (!todo.empty()) {
        Node nd = std::move(todo.back());
        todo.pop_back();
        const int n = (int)nd.idx.size();
        bool split = false;
        if (max_ell > 1 && (int)(done.size() + todo.size()) + 2 <= max_ell && n >= 4 * (d + 1)) {
            // the node's points relative to its centre (unit-cube coordinates, where
            // every parameter is scaled by its prior range)
            w.assign((size_t)n * d, 0.0);
            for (int i = 0; i < n; ++i)
                for (int a = 0; a < d; ++a)
                    w[(size_t)i * d + a] = U[(size_t)nd.idx[i] * d + a] - nd.mu[a];
            auto dist2 = [&](const double *x, const double *c) {
                double s = 0.0;
                for (int a = 0; a < d; ++a) s += (x[a] - c[a]) * (x[a] - c[a]);
                return s;
            };
            // 2-means: start from the point farthest from the centre and the one farthest from it
            double c0[GK_NP], c1[GK_NP], zero[GK_NP] = {};
            int f0 = 0, f1 = 0;
            for (int i = 1; i < n; ++i)
                if (dist2(&w[(size_t)i * d], zero) > dist2(&w[(size_t)f0 * d], zero)) f0 = i;
            for (int i = 1; i < n; ++i)
                if (dist2(&w[(size_t)i * d], &w[(size_t)f0 * d]) > dist2(&w[(size_t)f1 * d], &w[(size_t)f0 * d])) f1 = i;
            std::copy_n(&w[(size_t)f0 * d], d, c0);
            std::copy_n(&w[(size_t)f1 * d], d, c1);
            // Lloyd iterations on an evenly strided subset of at most
            // kMeansPoints points, then every point goes to its nearer centre
            const int stride = (n + kMeansPoints - 1) / kMeansPoints, ns = (n + stride - 1) / stride;
            std::vector<char> lab(ns, 0);
            for (int it = 0; it < 20; ++it) {
                bool changed = false;
                double s0[GK_NP] = {}, s1[GK_NP] = {};
                int n0 = 0, n1 = 0;
                for (int i = 0; i < ns; ++i) {
                    const double *y = &w[(size_t)i * stride * d];
                    const char l = dist2(y, c1) < dist2(y, c0) ? 1 : 0;
                    changed = changed || l != lab[i];
                    lab[i] = l;
                    double *acc = l ? s1 : s0;
                    for (int a = 0; a < d; ++a) acc[a] += y[a];
                    (l ? n1 : n0) += 1;
                }
                if (n0 == 0 || n1 == 0) break;
                for (int a = 0; a < d; ++a) {
                    c0[a] = s0[a] / n0;
                    c1[a] = s1[a] / n1;
                }
                if (!changed && it > 0) break;
            }
            Node ch[2];
            for (int i = 0; i < n; ++i) {
                const double *y = &w[(size_t)i * d];
                ch[dist2(y, c1) < dist2(y, c0) ? 1 : 0].idx.push_back(nd.idx[i]);
            }
            const int n0 = (int)ch[0].idx.size(), n1 = (int)ch[1].idx.size();
            if (n0 >= 2 * (d + 1) && n1 >= 2 * (d + 1) &&
                fit_ellipsoid(U, ch[0].idx.data(), n0, d, enlarge, min_vol(n0), ch[0].mu, ch[0].L,
                              ch[0].invd, ch[0].logvol) &&
                fit_ellipsoid(U, ch[1].idx.data(), n1, d, enlarge, min_vol(n1), ch[1].mu, ch[1].L,
                              ch[1].invd, ch[1].logvol) &&
                logaddexp(ch[0].logvol, ch[1].logvol) < nd.logvol + std::log(0.5)) {
                todo.push_back(std::move(ch[0]));
                todo.push_back(std::move(ch[1]));
                split = true;
            }
        }
        if (!split) done.push_back(std::move(nd));
    }
    double logtot = -INFINITY;
    for (auto &e : done) logtot = logaddexp(logtot, e.logvol);
    if (logtot >= 0.0) return;  // the union is larger than the box: the whole cube
    bnd.n_ell = (int)done.size();
    double c = 0.0;
    for (int e = 0; e < bnd.n_ell; ++e) {
        c += std::exp(done[e].logvol - logtot);
        bnd.cum[e] = c;
        std::copy_n(done[e].mu, d, bnd.mu[e]);
        std::copy_n(done[e].L, d * d, bnd.L[e]);
        std::copy_n(done[e].invd, d, bnd.inv_diag[e]);
    }
    bnd.cum[bnd.n_ell - 1] = 1.0;
}

// Draws n candidates from bnd (NULL: the first live points, uniform in the
// cube), evaluates them and returns their unit-cube coordinates u [n][d] and
// log-likelihoods; floor is the lowest live log-likelihood when the round
// starts (candidates at or below it cannot be accepted in this round).
using DrawEval = std::function<gk_status(const Bound *bnd, int n, int64_t round, double floor,
                                         double *u, double *logl)>;

// True if x lies in ellipsoid e of bnd.
__host__ __device__ inline bool in_ellipsoid(const Bound &bnd, int e, const double *x)
{
    const int d = bnd.d;
    double y[GK_NP], m2 = 0.0;
    for (int a = 0; a < d; ++a) {
        double t = x[a] - bnd.mu[e][a];
        for (int b = 0; b < a; ++b) t -= bnd.L[e][a * d + b] * y[b];
        y[a] = t * bnd.inv_diag[e][a];
        m2 += y[a] * y[a];
    }
    return m2 <= 1.0;
}

// Candidates from bnd with a sequential Philox stream (host side): pick an
// ellipsoid by volume, a direction from d normals and a radius U^(1/d);
// reject outside the cube, and keep a point lying in q ellipsoids with
// probability 1/q (uniform over the union).  After 10^5 rejections, uniform
// in the cube.
void draw_host(const Bound *bnd, int n, int d, Rng &rng, double *ub)
{
    double z[GK_NP];
    for (int c = 0; c < n; ++c) {
        double *u = ub + (size_t)c * d;
        for (int tries = 0;; ++tries) {
            if (!bnd || bnd->n_ell == 0 || tries > 100000) {
                for (int a = 0; a < d; ++a) u[a] = rng.uniform();
                break;
            }
            int e = 0;
            if (bnd->n_ell > 1) {
                const double pick = rng.uniform();
                while (e < bnd->n_ell - 1 && bnd->cum[e] < pick) ++e;
            }
            double nrm = 0.0;
            for (int a = 0; a < d; ++a) {
                z[a] = rng.normal();
                nrm += z[a] * z[a];
            }
            const double rad = std::pow(rng.uniform(), 1.0 / d) / std::sqrt(nrm);
            bool inside = true;
            for (int a = 0; a < d; ++a) {
                double s = bnd->mu[e][a];
                for (int b = 0; b <= a; ++b) s += bnd->L[e][a * d + b] * z[b] * rad;
                u[a] = s;
                inside = inside && s > 0.0 && s < 1.0;
            }
            if (!inside) continue;
            if (bnd->n_ell > 1) {
                int q = 1;
                for (int f = 0; f < bnd->n_ell; ++f) q += f != e && in_ellipsoid(*bnd, f, u);
                if (q > 1 && !(rng.uniform() * q < 1.0)) continue;
            }
            break;
        }
    }
}

// One host thread that runs a job (the next bound) while the caller's thread
// draws and evaluates a round.
class Worker {
  public:
    Worker() : th_([this] { loop(); }) {}
    ~Worker()
    {
        {
            std::lock_guard<std::mutex> l(mu_);
            quit_ = true;
        }
        cv_.notify_all();
        th_.join();
    }
    void submit(std::function<void()> job)
    {
        {
            std::lock_guard<std::mutex> l(mu_);
            job_ = std::move(job);
            pending_ = true;
        }
        cv_.notify_all();
    }
    void wait()
    {
        std::unique_lock<std::mutex> l(mu_);
        cv_.wait(l, [&] { return !pending_; });
    }

  private:
    void loop()
    {
        std::unique_lock<std::mutex> l(mu_);
        for (;;) {
            cv_.wait(l, [&] { return (pending_ && job_) || quit_; });
            if (quit_) return;
            std::function<void()> job = std::move(job_);
            job_ = nullptr;
            l.unlock();
            job();
            l.lock();
            pending_ = false;
            cv_.notify_all();
        }
    }
    std::mutex mu_;
    std::condition_variable cv_;
    std::function<void()> job_;
    bool pending_ = false, quit_ = false;
    std::thread th_;
};

// Runs the sampler in the unit cube [0,1]^d.  Fills the evidence fields of
// res, best[] in unit-cube coordinates, and the posterior samples post_u
// [M][d] with normalised weights post_w [M].
gk_status ns_run(int d, const DrawEval &draw_eval, const gk_ns_opts &o, gk_ns_result *res,
                 std::vector<double> &post_u, std::vector<double> &post_w, bool &capped)
{
    const int N = o.n_live, Bmax = std::max(o.batch, o.batch_max);
    std::vector<double> live_u((size_t)N * d), live_l(N);
    std::vector<double> ub((size_t)std::max(N, Bmax) * d), lb(std::max(N, Bmax));
    int B = o.batch;
    double acc_prev = -1.0, cand_prev = 0.0;  // acceptances and candidates of the last round
    GK_TRY(draw_eval(nullptr, N, 0, -DBL_MAX, live_u.data(), lb.data()));
    int64_t n_evals = N, n_launch = 1;
    for (int i = 0; i < N; ++i) live_l[i] = std::isfinite(lb[i]) ? lb[i] : -DBL_MAX;
    std::vector<double> dead_u, dead_l, dead_logwt;
    double logz = -INFINITY, max_logl = -INFINITY;
    std::vector<double> best(d, 0.0);
    for (int i = 0; i < N; ++i)
        if (live_l[i] > max_logl) {
            max_logl = live_l[i];
            std::copy_n(&live_u[(size_t)i * d], d, best.begin());
        }
    // min-heap of (logl, index): the lowest live point, ties to the lowest index
    std::vector<std::pair<double, int>> heap(N);
    for (int i = 0; i < N; ++i) heap[i] = {live_l[i], i};
    std::make_heap(heap.begin(), heap.end(), std::greater<>());
    const double log_shrink = std::log1p(-std::exp(-1.0 / N));  // log(1 - e^{-1/N})
    int64_t k = 0;
    bool done = false;
    capped = false;
    // The bound is rebuilt after every N/20 retired points.  The first one is
    // built before the first round; later ones are built on a worker thread
    // from the live points at the start of a round, while that round is drawn
    // and evaluated, and are used from the next round on.  A bound one round
    // old still contains the current, smaller constrained region, so it stays
    // valid, only less tight.
    const int64_t rebuild = std::max(1, N / 20);
    Bound bnd{}, next{};
    build_bound(live_u.data(), N, d, o.enlarge, 0.0, o.max_ell, bnd);
    int64_t k_built = 0;
    Worker worker;
    while (!done) {
        const bool building = k - k_built >= rebuild;
        bool build_failed = false;
        if (building) {
            const double logX = -(double)k / N;
            worker.submit([&, logX] {
                try {
                    build_bound(live_u.data(), N, d, o.enlarge, logX, o.max_ell, next);
                } catch (const std::bad_alloc &) {
                    build_failed = true;
                }
            });
        }
        const gk_status st = draw_eval(&bnd, B, n_launch, heap.front().first, ub.data(), lb.data());
        if (building) {  // the live points change below: the build must be over
            worker.wait();
            bnd = next;
            k_built = k;
        }
        GK_TRY(st);
        if (build_failed) return fail(GK_ENOMEM, "out of host memory building the bound");
        n_evals += B;
        ++n_launch;
        const int64_t k_round = k;
        for (int c = 0; c < B && !done; ++c) {
            const double lc = std::isfinite(lb[c]) ? lb[c] : -DBL_MAX;
            const int imin = heap.front().second;
            if (!(lc > live_l[imin])) continue;
            std::pop_heap(heap.begin(), heap.end(), std::greater<>());
            heap.back() = {lc, imin};
            std::push_heap(heap.begin(), heap.end(), std::greater<>());
            ++k;
            const double logwt = live_l[imin] + (-(double)(k - 1) / N + log_shrink);
            logz = logaddexp(logz, logwt);
            dead_u.insert(dead_u.end(), &live_u[(size_t)imin * d], &live_u[(size_t)imin * d] + d);
            dead_l.push_back(live_l[imin]);
            dead_logwt.push_back(logwt);
            std::copy_n(&ub[(size_t)c * d], d, &live_u[(size_t)imin * d]);
            live_l[imin] = lc;
            if (lc > max_logl) {
                max_logl = lc;
                std::copy_n(&ub[(size_t)c * d], d, best.begin());
            }
            // the retired point is the lowest, so the live maximum is the running one
            if (logaddexp(logz, max_logl - (double)k / N) - logz < o.tol) done = true;
            if (k >= o.max_iter) {
                done = true;
                capped = true;
            }
        }
        if (Bmax > o.batch) {  // next batch from the acceptance rate of the last two rounds
            const double acc = (double)(k - k_round), cand = B;
            const double rate = acc_prev < 0.0 ? acc / cand : (acc + acc_prev) / (cand + cand_prev);
            acc_prev = acc;
            cand_prev = cand;
            const int target = o.accept_target > 0 ? o.accept_target : std::max(1, N / 10);
            const double want = rate > 0.0 ? std::ceil(target / rate) : (double)Bmax;
            B = (int)std::min<double>(Bmax, std::max<double>(o.batch, want));
        }
    }
    // final live points with weight X_k / N
    for (int i = 0; i < N; ++i) {
        const double logwt = live_l[i] - (double)k / N - std::log((double)N);
        logz = logaddexp(logz, logwt);
        dead_u.insert(dead_u.end(), &live_u[(size_t)i * d], &live_u[(size_t)i * d] + d);
        dead_l.push_back(live_l[i]);
        dead_logwt.push_back(logwt);
    }
    double H = 0.0;
    post_u.swap(dead_u);
    post_w.resize(dead_l.size());
    for (size_t i = 0; i < dead_l.size(); ++i) {
        const double pw = std::exp(dead_logwt[i] - logz);
        if (pw > 0.0 && dead_l[i] > -DBL_MAX) H += pw * (dead_l[i] - logz);
        post_w[i] = pw;
    }
    res->logz = logz;
    res->info_h = H;
    res->logz_err = std::sqrt(std::max(H, 0.0) / N);
    res->max_logl = max_logl;
    res->n_iter = k;
    res->n_evals = n_evals;
    res->n_launches = n_launch;
    for (int a = 0; a < d; ++a) res->best[a] = best[a];
    return GK_OK;
}

// Weighted mean, sd and quantiles of coordinate a of the posterior.
void posterior_stats(const std::vector<double> &pu, const std::vector<double> &pw, int d, int a,
                     double scale, double offset, gk_ns_result *res, int slot)
{
    std::vector<std::pair<double, double>> v;
    v.reserve(pw.size());
    double m = 0.0, w = 0.0;
    for (size_t i = 0; i < pw.size(); ++i) {
        const double x = offset + scale * pu[i * d + a];
        v.emplace_back(x, pw[i]);
        m += pw[i] * x;
        w += pw[i];
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
    if (o.n_live < 2 || o.batch < 1 || o.max_iter < 1 || !(o.enlarge >= 1.0) || !(o.tol > 0.0) ||
        o.max_ell < 1 || o.max_ell > kMaxEll || (o.batch_max != 0 && o.batch_max < o.batch) ||
        o.accept_target < 0 || !(o.screen_cost >= 0.0) || o.screen_rows < 0)
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
    o->max_ell = 8;
    o->batch_max = 0;
    o->accept_target = 0;
    o->screen_cost = 0.0;
    o->screen_rows = 0;
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
    Rng rng(o.seed, 0x6e73u);
    DrawEval eval = [&](const Bound *bnd, int n, int64_t, double, double *u,
                        double *logl) -> gk_status {
        draw_host(bnd, n, dim, rng, u);
        theta.resize((size_t)n * dim);
        for (int i = 0; i < n; ++i)
            for (int a = 0; a < dim; ++a)
                theta[(size_t)i * dim + a] = lo[a] + u[(size_t)i * dim + a] * (hi[a] - lo[a]);
        if (fn(theta.data(), n, dim, logl, user) != 0)
            return fail(GK_EINVAL, "likelihood callback failed");
        return GK_OK;
    };
    std::memset(res, 0, sizeof *res);
    std::vector<double> pu, pw;
    bool capped = false;
    GK_TRY(ns_run(dim, eval, o, res, pu, pw, capped));
    for (int a = 0; a < dim; ++a) {
        res->best[a] = lo[a] + res->best[a] * (hi[a] - lo[a]);
        posterior_stats(pu, pw, dim, a, hi[a] - lo[a], lo[a], res, a);
    }
    if (samples && n_samples) {
        const int64_t n = std::min<int64_t>(cap, (int64_t)pw.size());
        for (int64_t i = 0; i < n; ++i) {
            for (int a = 0; a < dim; ++a)
                samples[i * (GK_NP + 1) + a] = lo[a] + pu[i * dim + a] * (hi[a] - lo[a]);
            samples[i * (GK_NP + 1) + GK_NP] = pw[i];
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

// ---------------------------------------------------------------------------
// Device-side candidates of the model fits: Philox4x32-10 streams keyed by
// the seed (high word xor a tag), one per (candidate, round, trial); normals
// by Box-Muller (both outputs).  Same rule as draw_host: ellipsoid by volume,
// direction from d normals, radius U^(1/d), rejected outside the cube and
// kept with probability 1/q where q ellipsoids overlap.
// ---------------------------------------------------------------------------
struct DrawArgs {
    const Bound *bnd;  // device copy of the round's region
    int d, n, round_valid;
    uint64_t round;
    uint32_t key0, key1;
    int fr[GK_NP];
    double lo[GK_NP], span[GK_NP], fixed[GK_NP];
    double *u;     // [n][d]
    double *rows;  // [n][GK_NP]
};

struct DevStream {
    uint32_t ctr[4], key[2], buf[4];
    int left;
    __device__ uint32_t u32()
    {
        if (!left) {
            philox4x32_10(ctr, key, buf);
            ++ctr[3];
            left = 4;
        }
        return buf[4 - left--];
    }
    __device__ double uniform()
    {
        const uint64_t a = u32(), b = u32();
        return ((double)((a << 21) ^ (b >> 11)) + 0.5) * 0x1.0p-53;
    }
    __device__ float uniformf()  // 24 random bits, never 0 or 1
    {
        return ((float)(u32() >> 8) + 0.5f) * 0x1.0p-24f;
    }
};

// One wave per candidate: the 64 lanes make independent trials (lane l of
// attempt t uses counter (c, r, l + 256 t, block)) and the lowest lane whose
// trial is accepted supplies the candidate -- the first success of trials
// taken in lane order, so the candidate is uniform over the region.  After
// 156 attempts (~10^4 trials) lane 0 draws uniformly in the cube.
__global__ __launch_bounds__(256) void k_ns_draw(DrawArgs g)
{
    const int c = blockIdx.x * 4 + (threadIdx.x >> 6), lane = threadIdx.x & 63;
    if (c >= g.n) return;  // whole waves
    const int d = g.d;
    double x[GK_NP], z[GK_NP];
    bool drawn = false;
    int attempt = 0;
    auto stream = [&](int t) {
        DevStream rs;
        rs.ctr[0] = (uint32_t)c;
        rs.ctr[1] = (uint32_t)g.round;
        rs.ctr[2] = (uint32_t)(lane + 256 * t);
        rs.ctr[3] = 0u;
        rs.key[0] = g.key0;
        rs.key[1] = g.key1;
        rs.left = 0;
        return rs;
    };
    if (g.round_valid && g.bnd->n_ell > 0) {
        const Bound &bnd = *g.bnd;
        for (; attempt < 156; ++attempt) {
            DevStream rs = stream(attempt);
            int e = 0;
            if (bnd.n_ell > 1) {
                const double pick = rs.uniform();
                while (e < bnd.n_ell - 1 && bnd.cum[e] < pick) ++e;
            }
            // direction and radius in FP32 (only their distribution matters;
            // the point itself is formed in FP64)
            float nrm = 0.0f;
            for (int a = 0; a < d; a += 2) {
                const float r = sqrtf(-2.0f * logf(rs.uniformf()));
                float sn, cs;
                sincosf(6.28318531f * rs.uniformf(), &sn, &cs);
                z[a] = r * cs;
                if (a + 1 < d) z[a + 1] = r * sn;
            }
            for (int a = 0; a < d; ++a) nrm += (float)(z[a] * z[a]);
            const double rad = (double)(exp2f(log2f(rs.uniformf()) / (float)d) / sqrtf(nrm));
            bool ok = true;
            for (int a = 0; a < d; ++a) {
                double v = bnd.mu[e][a];
                for (int b = 0; b <= a; ++b) v += bnd.L[e][a * d + b] * z[b] * rad;
                x[a] = v;
                ok = ok && v > 0.0 && v < 1.0;
            }
            if (ok && bnd.n_ell > 1) {
                int q = 1;
                for (int f = 0; f < bnd.n_ell; ++f) q += f != e && in_ellipsoid(bnd, f, x);
                ok = q == 1 || rs.uniform() * q < 1.0;
            }
            const unsigned long long hits = __ballot(ok);
            if (hits) {  // uniform over the wave
                drawn = lane == __ffsll((long long)hits) - 1;
                if (!drawn) return;
                break;
            }
        }
    }
    if (!drawn) {
        if (lane != 0) return;
        DevStream rs = stream(attempt);
        for (int a = 0; a < d; ++a) x[a] = rs.uniform();
    }
    double *row = g.rows + (size_t)c * GK_NP;
    for (int k = 0; k < GK_NP; ++k) row[k] = g.fixed[k];
    for (int a = 0; a < d; ++a) {
        g.u[(size_t)c * d + a] = x[a];
        row[g.fr[a]] = g.lo[g.fr[a]] + x[a] * g.span[g.fr[a]];
    }
}

// dst[i] = src[idx[i]] (parameter rows)
__global__ void k_gather_rows(const double *__restrict__ src, const int *__restrict__ idx, int n,
                              double *__restrict__ dst)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n * GK_NP) return;
    const int r = i / GK_NP, k = i - r * GK_NP;
    dst[i] = src[(size_t)idx[r] * GK_NP + k];
}

// Device buffers of one fit, freed on scope exit.
struct NsBuffers {
    double *d_u = nullptr, *d_rows2 = nullptr, *h_u = nullptr;
    int *d_idx = nullptr, *h_idx = nullptr;
    Bound *d_bnd = nullptr, *h_bnd = nullptr;
    ~NsBuffers()
    {
        (void)hipFree(d_bnd);
        if (h_bnd) (void)hipHostFree(h_bnd);
        (void)hipFree(d_u);
        (void)hipFree(d_rows2);
        (void)hipFree(d_idx);
        if (h_u) (void)hipHostFree(h_u);
        if (h_idx) (void)hipHostFree(h_idx);
    }
};

// Plain (sur == NULL) or surrogate-screened nested sampling of a model.
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
    DrawArgs g{};
    int d = 0;
    for (int k = 0; k < NPAR; ++k) {
        g.fixed[k] = fixed[k];
        g.lo[k] = lo[k];
        g.span[k] = hi[k] - lo[k];
        if (!free_mask[k]) continue;
        if (!(hi[k] > lo[k])) return fail(GK_EINVAL, "empty prior range in slot %d", k);
        g.fr[d++] = k;
    }
    if (d == 0) return fail(GK_EINVAL, "no free parameter");
    g.key0 = (uint32_t)o.seed;
    g.key1 = (uint32_t)(o.seed >> 32) ^ 0x6e736477u;
    DeviceGuard dg(m->device);
    HIP_TRY(dg.err);
    using clock = std::chrono::steady_clock;
    const auto t_start = clock::now();
    double t_wait = 0.0;
    auto wait = [&](hipStream_t st) -> hipError_t {
        const auto t0 = clock::now();
        const hipError_t e = hipStreamSynchronize(st);
        t_wait += std::chrono::duration<double>(clock::now() - t0).count();
        return e;
    };
    double *h_params, *d_params, *d_chi2, *h_chi2;
    hipStream_t stream;
    const int rows = std::max({o.n_live, o.batch, o.batch_max});
    // chi2 rows, then (screened) surrogate chi2 rows
    GK_TRY(fit_reserve_rows(m, 2 * rows, &h_params, &d_params, &d_chi2, &h_chi2, &stream));
    double *d_chi2s = d_chi2 + rows, *h_chi2s = h_chi2 + rows;
    NsBuffers nb;
    HIP_TRY(hipMalloc((void **)&nb.d_u, sizeof(double) * rows * d));
    HIP_TRY(hipMalloc((void **)&nb.d_bnd, sizeof(Bound)));
    HIP_TRY(hipHostMalloc((void **)&nb.h_bnd, sizeof(Bound), 0));
    HIP_TRY(hipHostMalloc((void **)&nb.h_u, sizeof(double) * rows * d, 0));
    if (sur) {
        HIP_TRY(hipMalloc((void **)&nb.d_rows2, sizeof(double) * rows * NPAR));
        HIP_TRY(hipMalloc((void **)&nb.d_idx, sizeof(int) * rows));
        HIP_TRY(hipHostMalloc((void **)&nb.h_idx, sizeof(int) * rows, 0));
    }
    std::memset(res, 0, sizeof *res);
    int64_t n_plain = 0;
    const uint32_t audit_key[2] = {(uint32_t)o.seed, (uint32_t)(o.seed >> 32) ^ 0x61756474u};
    std::vector<double> recent;  // surrogate-minus-plain chi2 of the latest plain evaluations
    size_t recent_pos = 0;
    double shift = 0.0;
    std::vector<int> keep;
    std::vector<char> audited;
    double pass_frac = 0.0;  // of the last screened round
    int since_screen = 8;    // rounds since the last screened one (the first is screened)
    DrawEval eval = [&](const Bound *bnd, int n, int64_t round, double floor, double *u,
                        double *logl) -> gk_status {
        g.n = n;
        g.d = d;
        g.round = (uint64_t)round;
        g.round_valid = bnd != nullptr;
        if (bnd) {
            // the pinned copy is free: every earlier round ended with a stream synchronisation
            std::memcpy(nb.h_bnd, bnd, sizeof(Bound));
            HIP_TRY(hipMemcpyAsync(nb.d_bnd, nb.h_bnd, sizeof(Bound), hipMemcpyHostToDevice, stream));
        }
        g.bnd = nb.d_bnd;
        g.u = nb.d_u;
        g.rows = d_params;
        hipLaunchKernelGGL(k_ns_draw, dim3((n + 3) / 4), dim3(256), 0, stream, g);
        HIP_TRY(hipGetLastError());
        HIP_TRY(hipMemcpyAsync(nb.h_u, nb.d_u, sizeof(double) * n * d, hipMemcpyDeviceToHost, stream));
        for (int i = 0; i < n; ++i) logl[i] = -INFINITY;
        // screen this round only where the plain evaluations it saves (at the
        // last screened round's pass fraction) outweigh its own cost
        const bool adaptive = o.screen_cost > 0.0 || o.screen_rows > 0;
        const bool screen = sur && (!adaptive || since_screen >= 8 ||
                                    (1.0 - pass_frac) * n > o.screen_cost * n + o.screen_rows);
        if (!screen) {
            ++since_screen;
            GK_TRY(run_batch(m, d_params, n, nullptr, nullptr, d_chi2, nullptr, stream));
            HIP_TRY(hipMemcpyAsync(h_chi2, d_chi2, sizeof(double) * n, hipMemcpyDeviceToHost, stream));
            HIP_TRY(wait(stream));
            std::memcpy(u, nb.h_u, sizeof(double) * n * d);
            n_plain += n;
            for (int i = 0; i < n; ++i) logl[i] = -0.5 * h_chi2[i];
            return GK_OK;
        }
        // surrogate chi2 of every candidate, then the plain chi2 of the survivors
        GK_TRY(surrogate_chi2(sur, m, d_params, n, d_chi2s, stream));
        HIP_TRY(hipMemcpyAsync(h_chi2s, d_chi2s, sizeof(double) * n, hipMemcpyDeviceToHost, stream));
        HIP_TRY(wait(stream));
        std::memcpy(u, nb.h_u, sizeof(double) * n * d);
        const double chi2_floor = floor > -DBL_MAX ? -2.0 * floor : INFINITY;
        const double cut = chi2_floor + shift + margin;
        keep.clear();
        audited.assign(n, 0);
        // the audit draw of candidate i is 32-bit word i % 4 of the Philox block
        // (i / 4, round) under the fit's audit key, made only for candidates
        // the screen discards
        uint32_t blk[4];
        int blk_id = -1;
        for (int i = 0; i < n; ++i) {
            if (!(h_chi2s[i] > cut)) {
                keep.push_back(i);
                continue;
            }
            if (!(audit > 0.0)) continue;
            if (i / 4 != blk_id) {
                blk_id = i / 4;
                const uint32_t ctr[4] = {(uint32_t)blk_id, (uint32_t)round, 0x617564u, 0u};
                philox4x32_10(ctr, audit_key, blk);
            }
            if (((double)blk[i % 4] + 0.5) * 0x1.0p-32 < audit) {
                keep.push_back(i);
                audited[i] = 1;
            }
        }
        res->n_screened += n;
        res->n_rejected += n - (int64_t)keep.size();
        const int nk = (int)keep.size();
        pass_frac = (double)nk / n;
        since_screen = 0;
        if (nk > 0) {
            std::memcpy(nb.h_idx, keep.data(), sizeof(int) * nk);
            HIP_TRY(hipMemcpyAsync(nb.d_idx, nb.h_idx, sizeof(int) * nk, hipMemcpyHostToDevice, stream));
            hipLaunchKernelGGL(k_gather_rows, dim3((nk * NPAR + 255) / 256), dim3(256), 0, stream,
                               d_params, nb.d_idx, nk, nb.d_rows2);
            HIP_TRY(hipGetLastError());
            GK_TRY(run_batch(m, nb.d_rows2, nk, nullptr, nullptr, d_chi2, nullptr, stream));
            HIP_TRY(hipMemcpyAsync(h_chi2, d_chi2, sizeof(double) * nk, hipMemcpyDeviceToHost, stream));
            HIP_TRY(wait(stream));
        }
        n_plain += nk;
        const size_t window = (size_t)std::max(o.n_live, o.batch);  // recent plain evaluations
        for (int j = 0; j < nk; ++j) {
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
    std::vector<double> pu, pw;
    bool capped = false;
    GK_TRY(ns_run(d, eval, o, res, pu, pw, capped));
    res->n_evals = n_plain;  // plain evaluations only
    res->t_wall_s = std::chrono::duration<double>(clock::now() - t_start).count();
    res->t_wait_s = t_wait;
    double best_u[GK_NP];
    std::memcpy(best_u, res->best, sizeof best_u);
    for (int k = 0; k < NPAR; ++k) {
        res->best[k] = res->mean[k] = res->median[k] = res->q16[k] = res->q84[k] = fixed[k];
        res->sd[k] = 0.0;
    }
    for (int a = 0; a < d; ++a) {
        const int k = g.fr[a];
        res->best[k] = lo[k] + best_u[a] * (hi[k] - lo[k]);
        posterior_stats(pu, pw, d, a, hi[k] - lo[k], lo[k], res, k);
    }
    if (samples && n_samples) {
        const int64_t n = std::min<int64_t>(cap, (int64_t)pw.size());
        for (int64_t i = 0; i < n; ++i) {
            double *row = samples + i * (GK_NP + 1);
            std::memcpy(row, fixed, sizeof(double) * NPAR);
            for (int a = 0; a < d; ++a)
                row[g.fr[a]] = lo[g.fr[a]] + pu[i * d + a] * (hi[g.fr[a]] - lo[g.fr[a]]);
            row[GK_NP] = pw[i];
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
