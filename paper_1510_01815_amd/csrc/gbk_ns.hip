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
// x = mu_e + L_e z, |z| <= 1 (L_e lower triangular, row-major d x d), each
// belonging to one mode, drawn from in proportion to their volumes (cum =
// cumulative volume fractions over the ellipsoids of unfinished modes), or
// the whole unit cube when n_ell is 0.
constexpr int kMaxEll = 16;
constexpr int kMaxModes = GK_NS_MAX_MODES;
constexpr int kMeansPoints = 256;  // points of the 2-means iterations of a split
struct Bound {
    int n_ell;
    int d;
    double cum[kMaxEll];
    double logvol[kMaxEll];
    int mode[kMaxEll];
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

// One ellipsoid of a decomposition and the live points it was fitted to.
struct Ell {
    std::vector<int> idx;
    double mu[GK_NP], L[GK_NP * GK_NP], invd[GK_NP], logvol;
};

// Decomposition of the points `pts` of one mode (prior volume exp(logX),
// n_ref live points): one enclosing ellipsoid, split recursively in two
// (2-means in unit-cube coordinates) while the two children's volumes sum
// to less than half the parent's and each child keeps at least 2 (d + 1)
// points, up to max_ell ellipsoids (MultiNest's decomposition, simplified).
// An ellipsoid is never smaller than the prior volume its points stand for,
// n_e X / n_ref.  False if the first ellipsoid is degenerate.
bool decompose(const double *U, const std::vector<int> &pts, int d, double enlarge, double logX,
               int n_ref, int max_ell, std::vector<Ell> &done)
{
    done.clear();
    auto min_vol = [&](int n) { return logX + std::log((double)n / n_ref); };
    std::vector<Ell> todo(1);
    todo[0].idx = pts;
    const int N = (int)pts.size();
    if (!fit_ellipsoid(U, todo[0].idx.data(), N, d, enlarge, min_vol(N), todo[0].mu, todo[0].L,
                       todo[0].invd, todo[0].logvol))
        return false;
    std::vector<double> w;
    while (!todo.empty()) {
        Ell nd = std::move(todo.back());
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
            Ell ch[2];
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
    return true;
}

// delta^T (Sa / (1 - s) + Sb / s)^-1 delta for the covariances Sa, Sb (d x d)
double overlap_q(const double *Sa, const double *Sb, const double *delta, int d, double s)
{
    std::vector<double> M((size_t)d * d);
    for (int k = 0; k < d * d; ++k) M[k] = Sa[k] / (1.0 - s) + Sb[k] / s;
    if (!cholesky(M, d)) return INFINITY;
    double y[GK_NP], q = 0.0;
    for (int a = 0; a < d; ++a) {
        double t = delta[a];
        for (int b = 0; b < a; ++b) t -= M[a * d + b] * y[b];
        y[a] = t / M[a * d + a];
        q += y[a] * y[a];
    }
    return q;
}

// True if the ellipsoids x = mu_a + L_a z and x = mu_b + L_b z (|z| <= 1)
// intersect.  With S = L L^T, they are disjoint exactly when
// K(s) = 1 - delta^T (S_a / (1 - s) + S_b / s)^-1 delta is negative for some s
// in (0, 1), delta = mu_b - mu_a (Gilitschenski & Hanebeck 2012); K is convex
// in s, so a golden-section search finds its minimum.
bool ellipsoids_overlap(const double *mua, const double *La, const double *mub, const double *Lb, int d)
{
    double Sa[GK_NP * GK_NP] = {}, Sb[GK_NP * GK_NP] = {}, delta[GK_NP];
    for (int a = 0; a < d; ++a) {
        delta[a] = mub[a] - mua[a];
        for (int b = 0; b < d; ++b)
            for (int k = 0; k <= std::min(a, b); ++k) {
                Sa[a * d + b] += La[a * d + k] * La[b * d + k];
                Sb[a * d + b] += Lb[a * d + k] * Lb[b * d + k];
            }
    }
    const double g = 0.5 * (std::sqrt(5.0) - 1.0);
    double lo = 1e-9, hi = 1.0 - 1e-9;
    double x1 = hi - g * (hi - lo), x2 = lo + g * (hi - lo);
    double f1 = 1.0 - overlap_q(Sa, Sb, delta, d, x1), f2 = 1.0 - overlap_q(Sa, Sb, delta, d, x2);
    for (int it = 0; it < 80; ++it) {
        if (f1 < 0.0 || f2 < 0.0) return false;
        if (f1 < f2) {
            hi = x2;
            x2 = x1;
            f2 = f1;
            x1 = hi - g * (hi - lo);
            f1 = 1.0 - overlap_q(Sa, Sb, delta, d, x1);
        } else {
            lo = x1;
            x1 = x2;
            f1 = f2;
            x2 = lo + g * (hi - lo);
            f2 = 1.0 - overlap_q(Sa, Sb, delta, d, x2);
        }
    }
    return f1 >= 0.0 && f2 >= 0.0;
}

// Per-mode state of the sampler.  A mode's live points evolve as a nested
// sampling run of their own: its prior volume starts at exp(logX0) and
// shrinks by exp(-1/n) with each point it retires.
struct Mode {
    int n = 0;                  // live points
    double logX0 = 0.0;         // log prior volume when the mode was created
    int64_t j = 0;              // points retired since
    double logz_own = -INFINITY;  // evidence of its own retired (and, at the end, live) points
    double logz_inh = -INFINITY;  // share of its ancestors' evidence (by live points at each split)
    double lmax = -DBL_MAX;     // highest live log-likelihood
    bool split = false;         // replaced by child modes
    bool finished = false;      // remaining evidence negligible: no more candidates
    double logX() const { return logX0 - (double)j / n; }
};

// A split of mode `parent` into modes parent's children (live point indices).
struct ModeSplit {
    int parent;
    std::vector<std::vector<int>> children;
};

// The region built from the live points at the start of a round: the bound
// and the mode splits its decomposition found.
struct Region {
    Bound bnd;
    std::vector<ModeSplit> splits;
};

// Builds the region of the live points U [N][d] (live_mode [N]) for the
// modes' current volumes.  Every unsplit, unfinished mode is decomposed on
// its own points; with `separate`, a mode whose ellipsoids fall into groups
// that do not intersect is split into one mode per group (at most kMaxModes
// modes in all; MultiNest's mode separation, simplified).  Ellipsoids per
// mode: max_ell, fewer when several modes share the kMaxEll ellipsoids.  A
// single mode whose ellipsoids outgrow the unit cube gets the whole cube.
void build_region(const double *U, const int *live_mode, int N, int d, const std::vector<Mode> &modes,
                  double enlarge, int max_ell, bool separate, Region &out)
{
    Bound &bnd = out.bnd;
    bnd.d = d;
    bnd.n_ell = 0;
    out.splits.clear();
    std::vector<int> act;
    for (int m = 0; m < (int)modes.size(); ++m)
        if (!modes[m].split && !modes[m].finished) act.push_back(m);
    if (act.empty()) return;
    const int per_mode = std::max(1, std::min(max_ell, kMaxEll / (int)act.size()));
    int n_modes = (int)modes.size();
    std::vector<std::vector<int>> pts(modes.size());
    for (int i = 0; i < N; ++i) pts[live_mode[i]].push_back(i);
    std::vector<Ell> ells;
    std::vector<int> ell_mode;
    for (int m : act) {
        std::vector<Ell> e;
        if (!decompose(U, pts[m], d, enlarge, modes[m].logX(), modes[m].n, per_mode, e)) {
            if (act.size() == 1) return;  // degenerate single mode: the whole cube
            // keep a ball of the mode's expected volume around its points
            Ell b;
            b.idx = pts[m];
            double r2 = 0.0;
            for (int a = 0; a < d; ++a) {
                b.mu[a] = 0.0;
                for (int i : pts[m]) b.mu[a] += U[(size_t)i * d + a];
                b.mu[a] /= pts[m].size();
            }
            for (int i : pts[m]) {
                double s = 0.0;
                for (int a = 0; a < d; ++a) s += (U[(size_t)i * d + a] - b.mu[a]) * (U[(size_t)i * d + a] - b.mu[a]);
                r2 = std::max(r2, s);
            }
            const double rad = std::max(std::sqrt(r2) * std::pow(enlarge, 1.0 / d),
                                        std::exp((modes[m].logX() - std::log(ball_volume(d))) / d));
            std::fill(b.L, b.L + d * d, 0.0);
            for (int a = 0; a < d; ++a) {
                b.L[a * d + a] = rad;
                b.invd[a] = 1.0 / rad;
            }
            b.logvol = std::log(ball_volume(d)) + d * std::log(rad);
            e.assign(1, std::move(b));
        }
        // groups of intersecting ellipsoids (connected components)
        const int ne = (int)e.size();
        std::vector<int> comp(ne);
        std::iota(comp.begin(), comp.end(), 0);
        std::function<int(int)> root = [&](int x) { return comp[x] == x ? x : comp[x] = root(comp[x]); };
        if (separate && ne > 1)
            for (int a = 0; a < ne; ++a)
                for (int b = a + 1; b < ne; ++b)
                    if (root(a) != root(b) && ellipsoids_overlap(e[a].mu, e[a].L, e[b].mu, e[b].L, d))
                        comp[root(a)] = root(b);
        std::vector<int> roots;
        for (int a = 0; a < ne; ++a)
            if (std::find(roots.begin(), roots.end(), root(a)) == roots.end()) roots.push_back(root(a));
        const bool do_split = separate && roots.size() > 1 &&
                              n_modes + (int)roots.size() <= kMaxModes;
        ModeSplit sp{m, {}};
        for (int a = 0; a < ne; ++a) {
            int label = m;
            if (do_split) {
                const int g = (int)(std::find(roots.begin(), roots.end(), root(a)) - roots.begin());
                label = n_modes + g;
                if ((int)sp.children.size() <= g) sp.children.resize(g + 1);
                sp.children[g].insert(sp.children[g].end(), e[a].idx.begin(), e[a].idx.end());
            }
            ells.push_back(std::move(e[a]));
            ell_mode.push_back(label);
        }
        if (do_split) {
            n_modes += (int)roots.size();
            out.splits.push_back(std::move(sp));
        }
    }
    double logtot = -INFINITY;
    for (auto &e : ells) logtot = logaddexp(logtot, e.logvol);
    if (act.size() == 1 && out.splits.empty() && logtot >= 0.0) return;  // the whole cube
    if ((int)ells.size() > kMaxEll) return;  // cannot happen: per_mode * modes <= kMaxEll
    bnd.n_ell = (int)ells.size();
    for (int e = 0; e < bnd.n_ell; ++e) {
        bnd.logvol[e] = ells[e].logvol;
        bnd.mode[e] = ell_mode[e];
        std::copy_n(ells[e].mu, d, bnd.mu[e]);
        std::copy_n(ells[e].L, d * d, bnd.L[e]);
        std::copy_n(ells[e].invd, d, bnd.inv_diag[e]);
    }
}

// Cumulative draw weights of bnd's ellipsoids by volume, over the modes that
// are not finished; false if none is left.
bool set_draw_weights(Bound &bnd, const std::vector<Mode> &modes)
{
    double logtot = -INFINITY;
    for (int e = 0; e < bnd.n_ell; ++e)
        if (!modes[bnd.mode[e]].finished) logtot = logaddexp(logtot, bnd.logvol[e]);
    if (logtot == -INFINITY) return false;
    double c = 0.0;
    int last = 0;
    for (int e = 0; e < bnd.n_ell; ++e) {
        if (!modes[bnd.mode[e]].finished) {
            c += std::exp(bnd.logvol[e] - logtot);
            last = e;
        }
        bnd.cum[e] = c;
    }
    for (int e = last; e < bnd.n_ell; ++e) bnd.cum[e] = 1.0;
    return true;
}

// Draws n candidates from bnd (NULL: the first live points, uniform in the
// cube), evaluates them and returns their unit-cube coordinates u [n][d],
// log-likelihoods, and the mode of the ellipsoid each was drawn from (-1 for
// a draw from the whole cube); floor is the lowest live log-likelihood when
// the round starts (candidates at or below it cannot be accepted in this
// round).
using DrawEval = std::function<gk_status(const Bound *bnd, int n, int64_t round, double floor,
                                         double *u, double *logl, int *mode)>;

// Mahalanobis radius^2 of x in ellipsoid e of bnd (<= 1 inside).
__host__ __device__ inline double ellipsoid_m2(const Bound &bnd, int e, const double *x)
{
    const int d = bnd.d;
    double y[GK_NP], m2 = 0.0;
    for (int a = 0; a < d; ++a) {
        double t = x[a] - bnd.mu[e][a];
        for (int b = 0; b < a; ++b) t -= bnd.L[e][a * d + b] * y[b];
        y[a] = t * bnd.inv_diag[e][a];
        m2 += y[a] * y[a];
    }
    return m2;
}

// True if x lies in ellipsoid e of bnd.
__host__ __device__ inline bool in_ellipsoid(const Bound &bnd, int e, const double *x)
{
    return ellipsoid_m2(bnd, e, x) <= 1.0;
}

// Candidates from bnd with a sequential Philox stream (host side): pick an
// ellipsoid by volume, a direction from d normals and a radius U^(1/d);
// reject outside the cube, and keep a point lying in q ellipsoids of the
// picked one's mode with probability 1/q (uniform over that mode's union).
// After 10^5 rejections, uniform in the cube.
void draw_host(const Bound *bnd, int n, int d, Rng &rng, double *ub, int *mode)
{
    double z[GK_NP];
    for (int c = 0; c < n; ++c) {
        double *u = ub + (size_t)c * d;
        mode[c] = -1;
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
                for (int f = 0; f < bnd->n_ell; ++f)
                    q += f != e && bnd->mode[f] == bnd->mode[e] && in_ellipsoid(*bnd, f, u);
                if (q > 1 && !(rng.uniform() * q < 1.0)) continue;
            }
            mode[c] = bnd->mode[e];
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
// res, best[] in unit-cube coordinates, the posterior samples post_u [M][d]
// with normalised weights post_w [M] and their modes post_mode [M], and the
// final modes (split ones included, with n = 0 live points after the split).
// Screened sampling: the surrogate's error bound (`shift`) is the largest
// surrogate-minus-plain chi2 among the latest plain evaluations whose plain
// chi2 lay within kShiftBand margins of the floor, once kShiftMinNear of them
// exist (before that, among all the latest plain evaluations).
constexpr double kShiftBand = 4.0;
constexpr size_t kShiftMinNear = 64;

gk_status ns_run(int d, const DrawEval &draw_eval, const gk_ns_opts &o, gk_ns_result *res,
                 std::vector<double> &post_u, std::vector<double> &post_w,
                 std::vector<int> &post_mode, std::vector<Mode> &modes, bool &capped)
{
    const int N = o.n_live, Bmax = std::max(o.batch, o.batch_max);
    const bool separate = o.separate_modes != 0;
    const auto t_start = std::chrono::steady_clock::now();
    std::vector<double> live_u((size_t)N * d), live_l(N);
    std::vector<int> live_mode(N, 0);
    std::vector<double> ub((size_t)std::max(N, Bmax) * d), lb(std::max(N, Bmax));
    std::vector<int> mb(std::max(N, Bmax));
    int B = o.batch;
    double acc_prev = -1.0, cand_prev = 0.0;  // acceptances and candidates of the last round
    GK_TRY(draw_eval(nullptr, N, 0, -DBL_MAX, live_u.data(), lb.data(), mb.data()));
    int64_t n_evals = N, n_launch = 1;
    for (int i = 0; i < N; ++i) live_l[i] = std::isfinite(lb[i]) ? lb[i] : -DBL_MAX;
    std::vector<double> dead_u, dead_l, dead_logwt;
    std::vector<int> dead_mode;
    double logz = -INFINITY, max_logl = -INFINITY;
    std::vector<double> best(d, 0.0);
    for (int i = 0; i < N; ++i)
        if (live_l[i] > max_logl) {
            max_logl = live_l[i];
            std::copy_n(&live_u[(size_t)i * d], d, best.begin());
        }
    modes.assign(1, Mode{});
    modes[0].n = N;
    modes[0].lmax = max_logl;
    // per mode, a min-heap of (logl, index): its lowest live point, ties to the lowest index
    std::vector<std::vector<std::pair<double, int>>> heaps(1);
    auto make_heaps = [&] {
        heaps.assign(modes.size(), {});
        for (int i = 0; i < N; ++i) heaps[live_mode[i]].push_back({live_l[i], i});
        for (auto &h : heaps) std::make_heap(h.begin(), h.end(), std::greater<>());
    };
    make_heaps();
    std::vector<double> log_shrink(1, std::log1p(-std::exp(-1.0 / N)));  // log(1 - e^{-1/n})
    int64_t k = 0;
    bool done = false;
    capped = false;
    auto lowest_live = [&] {
        double f = DBL_MAX;
        for (size_t m = 0; m < modes.size(); ++m)
            if (!heaps[m].empty()) f = std::min(f, heaps[m].front().first);
        return f;
    };
    // A mode is finished when its remaining evidence, at most L_max X, is
    // below (e^tol - 1) Z / (number of modes), so that the sum over modes
    // meets the stopping rule log(Z + sum L_max X) - log Z < tol.
    auto check_finished = [&] {
        int leaves = 0;
        for (auto &md : modes) leaves += !md.split;
        bool all = true;
        for (auto &md : modes) {
            if (md.split || md.finished) continue;
            if (logaddexp(logz, std::log((double)leaves) + md.lmax + md.logX()) - logz < o.tol)
                md.finished = true;
            else
                all = false;
        }
        return all;
    };
    // The region is rebuilt after every N/20 retired points.  The first one is
    // built before the first round; later ones are built on a worker thread
    // from the live points at the start of a round, while that round is drawn
    // and evaluated, and are used from the next round on.  A region one round
    // old still contains the current, smaller constrained region, so it stays
    // valid, only less tight.  Mode splits it finds take effect when it is
    // installed: the split mode's live points and this round's candidates
    // drawn from it pass to the child modes.
    const int64_t rebuild = std::max(1, N / 20);
    Region cur{}, next{};
    auto install = [&](Region &r, int ncand) {
        for (const ModeSplit &sp : r.splits) {
            // (modes grows below: copy what the children need from the parent)
            const Mode par = modes[sp.parent];
            const double logz_par = logaddexp(par.logz_inh, par.logz_own);
            const int first = (int)modes.size();
            for (const auto &ch : sp.children) {
                Mode c;
                c.n = (int)ch.size();
                c.logX0 = par.logX() + std::log((double)c.n / par.n);
                c.logz_inh = logz_par + std::log((double)c.n / par.n);
                for (int i : ch) {
                    live_mode[i] = (int)modes.size();
                    c.lmax = std::max(c.lmax, live_l[i]);
                }
                modes.push_back(c);
                log_shrink.push_back(std::log1p(-std::exp(-1.0 / c.n)));
            }
            modes[sp.parent].split = true;
            // this round's candidates from the split mode: the child whose
            // ellipsoid holds them, else the one whose ellipsoid is nearest
            for (int c = 0; c < ncand; ++c) {
                if (mb[c] != sp.parent) continue;
                double best_m2 = INFINITY;
                int to = first;
                for (int e = 0; e < r.bnd.n_ell; ++e) {
                    if (r.bnd.mode[e] < first || r.bnd.mode[e] >= (int)modes.size()) continue;
                    const double m2 = ellipsoid_m2(r.bnd, e, &ub[(size_t)c * d]);
                    if (m2 < best_m2) {
                        best_m2 = m2;
                        to = r.bnd.mode[e];
                    }
                }
                mb[c] = to;
            }
        }
        if (!r.splits.empty()) make_heaps();
        cur = r;
    };
    build_region(live_u.data(), live_mode.data(), N, d, modes, o.enlarge, o.max_ell, separate, next);
    install(next, 0);
    int64_t k_built = 0;
    Worker worker;
    Bound draw{};
    while (!done) {
        const bool building = k - k_built >= rebuild;
        bool build_failed = false;
        if (building) {
            worker.submit([&] {
                try {
                    build_region(live_u.data(), live_mode.data(), N, d, modes, o.enlarge, o.max_ell,
                                 separate, next);
                } catch (const std::bad_alloc &) {
                    build_failed = true;
                }
            });
        }
        draw = cur.bnd;
        const bool any = draw.n_ell == 0 || set_draw_weights(draw, modes);
        gk_status st = GK_OK;
        if (any) st = draw_eval(&draw, B, n_launch, lowest_live(), ub.data(), lb.data(), mb.data());
        if (building) {  // the live points change below: the build must be over
            worker.wait();
            if (!build_failed) install(next, any ? B : 0);
            k_built = k;
        }
        GK_TRY(st);
        if (build_failed) return fail(GK_ENOMEM, "out of host memory building the bound");
        if (!any) break;  // every mode finished
        n_evals += B;
        ++n_launch;
        const int64_t k_round = k;
        for (int c = 0; c < B && !done; ++c) {
            const double lc = std::isfinite(lb[c]) ? lb[c] : -DBL_MAX;
            int m = mb[c];
            if (modes.size() == 1) {
                m = 0;
            } else if (m < 0 || m >= (int)modes.size() || modes[m].split) {
                // a draw from the whole cube: the mode whose live point is nearest
                double bd = INFINITY;
                m = 0;
                for (int i = 0; i < N; ++i) {
                    double s = 0.0;
                    for (int a = 0; a < d; ++a) {
                        const double t = ub[(size_t)c * d + a] - live_u[(size_t)i * d + a];
                        s += t * t;
                    }
                    if (s < bd) {
                        bd = s;
                        m = live_mode[i];
                    }
                }
            }
            auto &hp = heaps[m];
            const int imin = hp.front().second;
            if (!(lc > live_l[imin])) continue;
            std::pop_heap(hp.begin(), hp.end(), std::greater<>());
            hp.back() = {lc, imin};
            std::push_heap(hp.begin(), hp.end(), std::greater<>());
            ++k;
            Mode &md = modes[m];
            const double logwt = live_l[imin] + md.logX() + log_shrink[m];
            md.j += 1;
            md.logz_own = logaddexp(md.logz_own, logwt);
            logz = logaddexp(logz, logwt);
            dead_u.insert(dead_u.end(), &live_u[(size_t)imin * d], &live_u[(size_t)imin * d] + d);
            dead_l.push_back(live_l[imin]);
            dead_logwt.push_back(logwt);
            dead_mode.push_back(m);
            std::copy_n(&ub[(size_t)c * d], d, &live_u[(size_t)imin * d]);
            live_l[imin] = lc;
            md.lmax = std::max(md.lmax, lc);
            if (lc > max_logl) {
                max_logl = lc;
                std::copy_n(&ub[(size_t)c * d], d, best.begin());
            }
            if (check_finished()) done = true;
            if (k >= o.max_iter) {
                done = true;
                capped = true;
            }
        }
        if (!done && o.max_wall_s > 0.0 &&
            std::chrono::duration<double>(std::chrono::steady_clock::now() - t_start).count() >
                o.max_wall_s) {
            done = true;
            capped = true;
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
    // final live points of each mode with weight X_m / n_m
    for (int i = 0; i < N; ++i) {
        Mode &md = modes[live_mode[i]];
        const double logwt = live_l[i] + md.logX() - std::log((double)md.n);
        md.logz_own = logaddexp(md.logz_own, logwt);
        logz = logaddexp(logz, logwt);
        dead_u.insert(dead_u.end(), &live_u[(size_t)i * d], &live_u[(size_t)i * d] + d);
        dead_l.push_back(live_l[i]);
        dead_logwt.push_back(logwt);
        dead_mode.push_back(live_mode[i]);
    }
    double H = 0.0;
    post_u.swap(dead_u);
    post_mode.swap(dead_mode);
    post_w.resize(dead_l.size());
    for (size_t i = 0; i < dead_l.size(); ++i) {
        const double pw = std::exp(dead_logwt[i] - logz);
        if (pw > 0.0 && dead_l[i] > -DBL_MAX) H += pw * (dead_l[i] - logz);
        post_w[i] = pw;
    }
    // per-mode information over the mode's own points, normalised by their evidence
    std::vector<double> Hm(modes.size(), 0.0);
    for (size_t i = 0; i < dead_l.size(); ++i) {
        const Mode &md = modes[post_mode[i]];
        const double pw = std::exp(dead_logwt[i] - md.logz_own);
        if (pw > 0.0 && dead_l[i] > -DBL_MAX) Hm[post_mode[i]] += pw * (dead_l[i] - md.logz_own);
    }
    res->logz = logz;
    res->info_h = H;
    res->logz_err = std::sqrt(std::max(H, 0.0) / N);
    res->max_logl = max_logl;
    res->n_iter = k;
    res->n_evals = n_evals;
    res->n_launches = n_launch;
    for (int a = 0; a < d; ++a) res->best[a] = best[a];
    int nm = 0;
    for (size_t m = 0; m < modes.size() && nm < kMaxModes; ++m) {
        if (modes[m].split) continue;
        gk_ns_mode &r = res->modes[nm++];
        r.logz = logaddexp(modes[m].logz_inh, modes[m].logz_own);
        r.info_h = Hm[m];
        r.logz_err = std::sqrt(std::max(Hm[m], 0.0) / modes[m].n);
        r.n_live = modes[m].n;
    }
    res->n_modes = nm;
    return GK_OK;
}

// Posterior summaries of one parameter: mean, sd and the 16/50/84% quantiles.
struct StatOut {
    double *mean, *sd, *q16, *median, *q84;
};

// Weighted mean, sd and quantiles of coordinate a of the posterior points
// whose mode is `mode` (every point for mode < 0), x = offset + scale u;
// writes element `slot` of each output.
void posterior_stats(const std::vector<double> &pu, const std::vector<double> &pw,
                     const std::vector<int> &pmode, int mode, int d, int a, double scale,
                     double offset, const StatOut &out, int slot)
{
    std::vector<std::pair<double, double>> v;
    v.reserve(pw.size());
    double m = 0.0, w = 0.0;
    for (size_t i = 0; i < pw.size(); ++i) {
        if (mode >= 0 && pmode[i] != mode) continue;
        const double x = offset + scale * pu[i * d + a];
        v.emplace_back(x, pw[i]);
        m += pw[i] * x;
        w += pw[i];
    }
    if (v.empty() || !(w > 0.0)) {
        out.mean[slot] = out.sd[slot] = out.q16[slot] = out.median[slot] = out.q84[slot] = NAN;
        return;
    }
    m /= w;
    double var = 0.0;
    for (auto &x : v) var += x.second * (x.first - m) * (x.first - m);
    out.mean[slot] = m;
    out.sd[slot] = std::sqrt(var / w);
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
    out.q16[slot] = quant(0.16);
    out.median[slot] = quant(0.5);
    out.q84[slot] = quant(0.84);
}

// The whole posterior's summaries of coordinate a into res, and each final
// mode's (in the order of res->modes) into res->modes[].
void all_stats(const std::vector<double> &pu, const std::vector<double> &pw,
               const std::vector<int> &pmode, const std::vector<Mode> &modes, int d, int a,
               double scale, double offset, gk_ns_result *res, int slot)
{
    posterior_stats(pu, pw, pmode, -1, d, a, scale, offset,
                    StatOut{res->mean, res->sd, res->q16, res->median, res->q84}, slot);
    int k = 0;
    for (int m = 0; m < (int)modes.size() && k < res->n_modes; ++m) {
        if (modes[m].split) continue;
        gk_ns_mode &r = res->modes[k++];
        posterior_stats(pu, pw, pmode, m, d, a, scale, offset,
                        StatOut{r.mean, r.sd, r.q16, r.median, r.q84}, slot);
    }
}

// Posterior points of each final mode (weights above zero).
void mode_counts(const std::vector<double> &pw, const std::vector<int> &pmode,
                 const std::vector<Mode> &modes, gk_ns_result *res)
{
    int k = 0;
    for (int m = 0; m < (int)modes.size() && k < res->n_modes; ++m) {
        if (modes[m].split) continue;
        int64_t c = 0;
        for (size_t i = 0; i < pw.size(); ++i) c += pmode[i] == m && pw[i] > 0.0;
        res->modes[k++].n_samples = c;
    }
}

gk_status check_opts(const gk_ns_opts &o)
{
    if (o.n_live < 2 || o.batch < 1 || o.max_iter < 1 || !(o.enlarge >= 1.0) || !(o.tol > 0.0) ||
        o.max_ell < 1 || o.max_ell > kMaxEll || (o.batch_max != 0 && o.batch_max < o.batch) ||
        o.accept_target < 0 || !(o.screen_cost >= 0.0) || o.screen_rows < 0 ||
        (o.separate_modes != 0 && o.separate_modes != 1) || !(o.max_wall_s >= 0.0))
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
    o->separate_modes = 0;
    o->max_wall_s = 0.0;
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
    DrawEval eval = [&](const Bound *bnd, int n, int64_t, double, double *u, double *logl,
                        int *mode) -> gk_status {
        draw_host(bnd, n, dim, rng, u, mode);
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
    std::vector<int> pm;
    std::vector<Mode> modes;
    bool capped = false;
    GK_TRY(ns_run(dim, eval, o, res, pu, pw, pm, modes, capped));
    for (int a = 0; a < dim; ++a) {
        res->best[a] = lo[a] + res->best[a] * (hi[a] - lo[a]);
        all_stats(pu, pw, pm, modes, dim, a, hi[a] - lo[a], lo[a], res, a);
    }
    mode_counts(pw, pm, modes, res);
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
// kept with probability 1/q where q ellipsoids of its mode overlap.
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
    int *mode;     // [n]: mode of the ellipsoid drawn from, -1 for the whole cube
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
// taken in lane order, so the candidate is uniform over its mode's part of
// the region, and the mode is picked in proportion to that part's volume.
// After 156 attempts (~10^4 trials) lane 0 draws uniformly in the cube.
__global__ __launch_bounds__(256) void k_ns_draw(DrawArgs g)
{
    const int c = blockIdx.x * 4 + (threadIdx.x >> 6), lane = threadIdx.x & 63;
    if (c >= g.n) return;  // whole waves
    const int d = g.d;
    double x[GK_NP], z[GK_NP];
    bool drawn = false;
    int attempt = 0, mode = -1;
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
                for (int f = 0; f < bnd.n_ell; ++f)
                    q += f != e && bnd.mode[f] == bnd.mode[e] && in_ellipsoid(bnd, f, x);
                ok = q == 1 || rs.uniform() * q < 1.0;
            }
            const unsigned long long hits = __ballot(ok);
            if (hits) {  // uniform over the wave
                drawn = lane == __ffsll((long long)hits) - 1;
                if (!drawn) return;
                mode = bnd.mode[e];
                break;
            }
        }
    }
    if (!drawn) {
        if (lane != 0) return;
        DevStream rs = stream(attempt);
        for (int a = 0; a < d; ++a) x[a] = rs.uniform();
    }
    g.mode[c] = mode;
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
// A round's candidates (unit-cube coordinates, modes), plain chi-squares and
// surrogate chi-squares go straight to pinned, device-mapped, coherent host
// buffers: the draw kernel and the chi-square reductions write them there, and
// no copy is queued behind the round's launches (h_*: host addresses, dv_*:
// the device's).
struct NsBuffers {
    double *d_rows2 = nullptr, *h_u = nullptr, *h_chi2 = nullptr, *h_chi2s = nullptr;
    double *dv_u = nullptr, *dv_chi2 = nullptr, *dv_chi2s = nullptr;
    int *d_idx = nullptr, *h_idx = nullptr, *h_mode = nullptr, *dv_mode = nullptr;
    Bound *d_bnd = nullptr, *h_bnd = nullptr;
    ~NsBuffers()
    {
        (void)hipFree(d_bnd);
        if (h_bnd) (void)hipHostFree(h_bnd);
        (void)hipFree(d_rows2);
        (void)hipFree(d_idx);
        if (h_u) (void)hipHostFree(h_u);
        if (h_chi2) (void)hipHostFree(h_chi2);
        if (h_chi2s) (void)hipHostFree(h_chi2s);
        if (h_idx) (void)hipHostFree(h_idx);
        if (h_mode) (void)hipHostFree(h_mode);
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
    GK_TRY(fit_reserve_rows(m, rows, &h_params, &d_params, &d_chi2, &h_chi2, &stream));
    NsBuffers nb;
    HIP_TRY(hipMalloc((void **)&nb.d_bnd, sizeof(Bound)));
    HIP_TRY(hipHostMalloc((void **)&nb.h_bnd, sizeof(Bound), 0));
    const unsigned mapped = hipHostMallocMapped | hipHostMallocCoherent;
    HIP_TRY(hipHostMalloc((void **)&nb.h_u, sizeof(double) * rows * d, mapped));
    HIP_TRY(hipHostMalloc((void **)&nb.h_mode, sizeof(int) * rows, mapped));
    HIP_TRY(hipHostMalloc((void **)&nb.h_chi2, sizeof(double) * rows, mapped));
    HIP_TRY(hipHostGetDevicePointer((void **)&nb.dv_u, nb.h_u, 0));
    HIP_TRY(hipHostGetDevicePointer((void **)&nb.dv_mode, nb.h_mode, 0));
    HIP_TRY(hipHostGetDevicePointer((void **)&nb.dv_chi2, nb.h_chi2, 0));
    if (sur) {
        HIP_TRY(hipHostMalloc((void **)&nb.h_chi2s, sizeof(double) * rows, mapped));
        HIP_TRY(hipHostGetDevicePointer((void **)&nb.dv_chi2s, nb.h_chi2s, 0));
    }
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
    // the same for the latest plain evaluations within kShiftBand of the floor
    // (the acceptable candidates' errors are what the screen must bound)
    std::vector<double> near;
    size_t near_pos = 0;
    const size_t near_window = (size_t)4 * std::max({o.n_live, o.batch, o.batch_max});
    const double band = kShiftBand * std::max(margin, 1.0);
    double shift = 0.0;
    std::vector<int> keep;
    std::vector<char> audited;
    double pass_frac = 0.0;  // of the last screened round
    int since_screen = 8;    // rounds since the last screened one (the first is screened)
    DrawEval eval = [&](const Bound *bnd, int n, int64_t round, double floor, double *u,
                        double *logl, int *mode) -> gk_status {
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
        g.u = nb.dv_u;
        g.rows = d_params;
        g.mode = nb.dv_mode;
        hipLaunchKernelGGL(k_ns_draw, dim3((n + 3) / 4), dim3(256), 0, stream, g);
        HIP_TRY(hipGetLastError());
        for (int i = 0; i < n; ++i) logl[i] = -INFINITY;
        // screen this round only where the plain evaluations it saves (at the
        // last screened round's pass fraction) outweigh its own cost
        const bool adaptive = o.screen_cost > 0.0 || o.screen_rows > 0;
        const bool screen = sur && (!adaptive || since_screen >= 8 ||
                                    (1.0 - pass_frac) * n > o.screen_cost * n + o.screen_rows);
        if (!screen) {
            ++since_screen;
            GK_TRY(run_batch(m, d_params, n, nullptr, nullptr, nb.dv_chi2, nullptr, stream, true));
            HIP_TRY(wait(stream));
            std::memcpy(u, nb.h_u, sizeof(double) * n * d);
            std::memcpy(mode, nb.h_mode, sizeof(int) * n);
            n_plain += n;
            for (int i = 0; i < n; ++i) logl[i] = -0.5 * nb.h_chi2[i];
            return GK_OK;
        }
        // surrogate chi2 of every candidate, then the plain chi2 of the survivors
        GK_TRY(surrogate_chi2(sur, m, d_params, n, nb.dv_chi2s, stream));
        HIP_TRY(wait(stream));
        std::memcpy(u, nb.h_u, sizeof(double) * n * d);
        std::memcpy(mode, nb.h_mode, sizeof(int) * n);
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
            if (!(nb.h_chi2s[i] > cut)) {
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
            GK_TRY(run_batch(m, nb.d_rows2, nk, nullptr, nullptr, nb.dv_chi2, nullptr, stream, true));
            HIP_TRY(wait(stream));
        }
        n_plain += nk;
        const size_t window = (size_t)std::max(o.n_live, o.batch);  // recent plain evaluations
        for (int j = 0; j < nk; ++j) {
            const int i = keep[j];
            const double c = nb.h_chi2[j];
            logl[i] = -0.5 * c;
            if (audited[i]) {
                res->n_audited += 1;
                res->n_audit_miss += c < chi2_floor;
            }
            const double delta = nb.h_chi2s[i] - c;
            if (std::isfinite(delta)) {
                if (recent.size() < window) {
                    recent.push_back(delta);
                } else {
                    recent[recent_pos] = delta;
                    recent_pos = (recent_pos + 1) % window;
                }
                if (c < chi2_floor + band) {
                    if (near.size() < near_window) {
                        near.push_back(delta);
                    } else {
                        near[near_pos] = delta;
                        near_pos = (near_pos + 1) % near_window;
                    }
                }
            }
        }
        shift = 0.0;
        for (double v : near.size() >= kShiftMinNear ? near : recent) shift = std::max(shift, v);
        return GK_OK;
    };
    std::vector<double> pu, pw;
    std::vector<int> pm;
    std::vector<Mode> modes;
    bool capped = false;
    GK_TRY(ns_run(d, eval, o, res, pu, pw, pm, modes, capped));
    res->n_evals = n_plain;  // plain evaluations only
    res->t_wall_s = std::chrono::duration<double>(clock::now() - t_start).count();
    res->t_wait_s = t_wait;
    double best_u[GK_NP];
    std::memcpy(best_u, res->best, sizeof best_u);
    for (int k = 0; k < NPAR; ++k) {
        res->best[k] = res->mean[k] = res->median[k] = res->q16[k] = res->q84[k] = fixed[k];
        res->sd[k] = 0.0;
        for (int j = 0; j < res->n_modes; ++j) {
            gk_ns_mode &r = res->modes[j];
            r.mean[k] = r.median[k] = r.q16[k] = r.q84[k] = fixed[k];
            r.sd[k] = 0.0;
        }
    }
    for (int a = 0; a < d; ++a) {
        const int k = g.fr[a];
        res->best[k] = lo[k] + best_u[a] * (hi[k] - lo[k]);
        all_stats(pu, pw, pm, modes, d, a, hi[k] - lo[k], lo[k], res, k);
    }
    mode_counts(pw, pm, modes, res);
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
