// gbk_fit.hip -- optimisers that drive the batched evaluation (Sec. 2.3).
//
// Levenberg-Marquardt (Sec. 2.3.1): each iteration is one batched launch of
// the trial point and its finite-difference Jacobian rows (gk_residual_batch
// machinery), then one FP64 kernel forming J^T J, J^T r and chi2, then a
// Cholesky solve on the host.  The step rule is written out in gbk.h.
#include <hip/hip_runtime.h>

#include <cfloat>
#include <cmath>
#include <cstring>
#include <new>
#include <vector>

#include "gbk_model.h"

using namespace gbk;

namespace gbk {

// Per-model workspace of the fitters: a stream of their own (default
// priority), parameter rows (pinned host + device), residual rows and the
// normal-equation results.
struct FitWork {
    hipStream_t stream = nullptr;
    int rows_cap = 0, resid_cap = 0;
    double *h_params = nullptr, *d_params = nullptr;  // [rows_cap][NPAR]
    double *d_chi2 = nullptr, *h_chi2 = nullptr;      // [rows_cap]
    double *d_resid = nullptr;                        // [resid_cap][2][npix]
    double *d_norm = nullptr, *h_norm = nullptr;
    // normal equations: chunk partials, and {goff[2], scale[NPAR]} staged per evaluation
    double *d_part = nullptr;
    char *d_aux = nullptr, *h_aux = nullptr;
};

void fit_release(FitWork *w)
{
    if (!w) return;
    if (w->stream) (void)hipStreamSynchronize(w->stream);
    (void)hipHostFree(w->h_params);
    (void)hipFree(w->d_params);
    (void)hipFree(w->d_chi2);
    (void)hipHostFree(w->h_chi2);
    (void)hipFree(w->d_resid);
    (void)hipFree(w->d_norm);
    (void)hipHostFree(w->h_norm);
    (void)hipFree(w->d_part);
    (void)hipFree(w->d_aux);
    (void)hipHostFree(w->h_aux);
    if (w->stream) (void)hipStreamDestroy(w->stream);
    delete w;
}

template <int NF>
__global__ __launch_bounds__(256) void k_lm_normal_chunks(const double *__restrict__ R,
                                                          const int64_t *__restrict__ goff,
                                                          const int64_t *__restrict__ nused,
                                                          const double *__restrict__ scale,
                                                          int nchunk, double *__restrict__ partial)
{
    constexpr int NP = NF * (NF + 1) / 2, NB = NP + NF + 1;
    const int g = blockIdx.y, ch = blockIdx.x, tid = threadIdx.x;
    const int64_t base = goff[g];
    const int64_t stride = (goff[g + 1] - base) / (1 + 2 * NF);
    const int64_t n = nused ? nused[g] : stride;
    const double *R0 = R + base;
    double s[NF], acc[NB];
#pragma unroll
    for (int a = 0; a < NF; ++a) s[a] = scale[(size_t)g * NPAR + a];
#pragma unroll
    for (int k = 0; k < NB; ++k) acc[k] = 0.0;
    const int clen = lm_chunk_len(n);
    const int64_t i0 = (int64_t)ch * clen;
    for (int q = 0; q < clen / 256; ++q) {
        const int64_t i = i0 + q * 256 + tid;
        if (i >= n) break;
        const double r0 = R0[i];
        double j[NF];
#pragma unroll
        for (int a = 0; a < NF; ++a)
            j[a] = (R0[(size_t)(1 + 2 * a) * stride + i] - R0[(size_t)(2 + 2 * a) * stride + i]) * s[a];
        int k = 0;
#pragma unroll
        for (int a = 0; a < NF; ++a)
#pragma unroll
            for (int b = a; b < NF; ++b) acc[k++] += j[a] * j[b];
#pragma unroll
        for (int a = 0; a < NF; ++a) acc[NP + a] += j[a] * r0;
        acc[NB - 1] += r0 * r0;
    }
    __shared__ double ws[4][NB];
    const int wave = tid >> 6, lane = tid & 63;
#pragma unroll
    for (int k = 0; k < NB; ++k) {
        double v = acc[k];
        for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
        if (lane == 0) ws[wave][k] = v;
    }
    __syncthreads();
    if (tid < NB)
        partial[((size_t)g * nchunk + ch) * NB + tid] = ((ws[0][tid] + ws[1][tid]) + ws[2][tid]) + ws[3][tid];
}

// One workgroup per (fit, output) for fits whose rows form one chunk.
__global__ __launch_bounds__(256) void k_lm_normal_rows(const double *__restrict__ R,
                                                        const int64_t *__restrict__ goff,
                                                        const int64_t *__restrict__ nused,
                                                        const double *__restrict__ scale, int nf,
                                                        double *__restrict__ out)
{
    const int k = blockIdx.x, g = blockIdx.y, tid = threadIdx.x;
    const int np = nf * (nf + 1) / 2, nblk = np + nf + 1;
    const int64_t base = goff[g];
    const int64_t stride = (goff[g + 1] - base) / (1 + 2 * nf);
    const int64_t n = nused ? nused[g] : stride;
    const double *R0 = R + base;
    const double *s = scale + (size_t)g * NPAR;
    double acc = 0.0;
    if (k < np) {
        int a = 0, r = k;
        while (r >= nf - a) {  // pair index k -> (a, b), a <= b, in row order
            r -= nf - a;
            ++a;
        }
        const int b = a + r;
        const double *pa = R0 + (size_t)(1 + 2 * a) * stride, *ma = R0 + (size_t)(2 + 2 * a) * stride;
        const double *pb = R0 + (size_t)(1 + 2 * b) * stride, *mb = R0 + (size_t)(2 + 2 * b) * stride;
        for (int64_t i = tid; i < n; i += 256) acc += ((pa[i] - ma[i]) * s[a]) * ((pb[i] - mb[i]) * s[b]);
    } else if (k < np + nf) {
        const int a = k - np;
        const double *pa = R0 + (size_t)(1 + 2 * a) * stride, *ma = R0 + (size_t)(2 + 2 * a) * stride;
        for (int64_t i = tid; i < n; i += 256) acc += ((pa[i] - ma[i]) * s[a]) * R0[i];
    } else {
        for (int64_t i = tid; i < n; i += 256) acc += R0[i] * R0[i];
    }
    for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o, 64);
    __shared__ double ws[4];
    if ((tid & 63) == 0) ws[tid >> 6] = acc;
    __syncthreads();
    if (tid == 0) out[(size_t)g * nblk + k] = 0.0 + (((ws[0] + ws[1]) + ws[2]) + ws[3]);
}

__global__ __launch_bounds__(128) void k_lm_normal_finish(const double *__restrict__ partial,
                                                          const int64_t *__restrict__ goff,
                                                          const int64_t *__restrict__ nused,
                                                          int rows, int nchunk, int nblk,
                                                          double *__restrict__ out)
{
    const int g = blockIdx.x, k = threadIdx.x;
    if (k >= nblk) return;
    const int nc = lm_normal_chunks(nused ? nused[g] : (goff[g + 1] - goff[g]) / rows);
    const double *p = partial + (size_t)g * nchunk * nblk + k;
    double s = 0.0;
    for (int c = 0; c < nc; ++c) s += p[(size_t)c * nblk];
    out[(size_t)g * nblk + k] = s;
}

template <int NF>
void launch_lm_chunks(const double *R, const int64_t *goff, const int64_t *nused,
                      const double *scale, int ng, int nchunk, double *partial, hipStream_t s)
{
    hipLaunchKernelGGL(k_lm_normal_chunks<NF>, dim3(nchunk, ng), dim3(256), 0, s, R, goff, nused,
                       scale, nchunk, partial);
}

hipError_t launch_lm_normal(const double *R, const int64_t *goff, const int64_t *nused,
                            const double *scale, int ng, int nf, int nchunk, double *partial,
                            double *out, hipStream_t s)
{
    using Fn = void (*)(const double *, const int64_t *, const int64_t *, const double *, int, int,
                        double *, hipStream_t);
    static const Fn table[NPAR] = {launch_lm_chunks<1>, launch_lm_chunks<2>, launch_lm_chunks<3>,
                                   launch_lm_chunks<4>, launch_lm_chunks<5>, launch_lm_chunks<6>,
                                   launch_lm_chunks<7>, launch_lm_chunks<8>, launch_lm_chunks<9>,
                                   launch_lm_chunks<10>, launch_lm_chunks<11>, launch_lm_chunks<12>};
    if (nf < 1 || nf > NPAR || ng < 1 || ng > 65535 || nchunk < 1)
        return hipErrorInvalidValue;
    const int nblk = nf * (nf + 1) / 2 + nf + 1;
    if (nchunk == 1) {
        hipLaunchKernelGGL(k_lm_normal_rows, dim3(nblk, ng), dim3(256), 0, s, R, goff, nused, scale,
                           nf, out);
        return hipGetLastError();
    }
    table[nf - 1](R, goff, nused, scale, ng, nchunk, partial, s);
    hipLaunchKernelGGL(k_lm_normal_finish, dim3(ng), dim3(128), 0, s, partial, goff, nused,
                       1 + 2 * nf, nchunk, nblk, out);
    return hipGetLastError();
}

}  // namespace gbk

namespace {

constexpr int kMaxFree = NPAR;
constexpr int kMaxPairs = kMaxFree * (kMaxFree + 1) / 2;
constexpr int kNormSlots = kMaxPairs + kMaxFree + 1;
constexpr size_t kAuxBytes = 4 * sizeof(int64_t) + NPAR * sizeof(double);  // goff[2], nused, pad, scale

// Grows the fitter workspace to `rows` parameter rows (and `resid_rows`
// residual rows when > 0).
gk_status fit_reserve(gk_model *m, int rows, int resid_rows)
{
    if (!m->fit) {
        m->fit = new (std::nothrow) FitWork();
        if (!m->fit) return fail(GK_ENOMEM, "host allocation failed");
        HIP_TRY(hipStreamCreate(&m->fit->stream));
        HIP_TRY(hipMalloc((void **)&m->fit->d_norm, sizeof(double) * kNormSlots));
        HIP_TRY(hipHostMalloc((void **)&m->fit->h_norm, sizeof(double) * kNormSlots, 0));
        const int nchunk = lm_normal_chunks((int64_t)2 * m->d.nx * m->d.ny);
        HIP_TRY(hipMalloc((void **)&m->fit->d_part, sizeof(double) * kNormSlots * nchunk));
        HIP_TRY(hipMalloc((void **)&m->fit->d_aux, kAuxBytes));
        HIP_TRY(hipHostMalloc((void **)&m->fit->h_aux, kAuxBytes, 0));
    }
    FitWork *w = m->fit;
    if (rows > w->rows_cap) {
        HIP_TRY(hipStreamSynchronize(w->stream));
        (void)hipHostFree(w->h_params);
        (void)hipFree(w->d_params);
        (void)hipFree(w->d_chi2);
        (void)hipHostFree(w->h_chi2);
        w->h_params = w->d_params = w->d_chi2 = w->h_chi2 = nullptr;
        w->rows_cap = 0;
        HIP_TRY(hipHostMalloc((void **)&w->h_params, sizeof(double) * NPAR * rows, 0));
        HIP_TRY(dev_alloc(&w->d_params, (size_t)rows * NPAR));
        HIP_TRY(dev_alloc(&w->d_chi2, (size_t)rows));
        HIP_TRY(hipHostMalloc((void **)&w->h_chi2, sizeof(double) * rows, 0));
        w->rows_cap = rows;
    }
    if (resid_rows > w->resid_cap) {
        HIP_TRY(hipStreamSynchronize(w->stream));
        (void)hipFree(w->d_resid);
        w->d_resid = nullptr;
        w->resid_cap = 0;
        const size_t npix = (size_t)m->d.nx * m->d.ny;
        HIP_TRY(dev_alloc(&w->d_resid, (size_t)resid_rows * 2 * npix));
        w->resid_cap = resid_rows;
    }
    return GK_OK;
}

// Row indices and scales of the Jacobian columns of the normal equations.
struct LMIdx {
    int nf, npairs;
    int ip[kMaxFree], im[kMaxFree];
    double s[kMaxFree];
    unsigned char pa[kMaxPairs], pb[kMaxPairs];
};

// Solves M x = b for symmetric positive definite M (n <= 12) by Cholesky;
// false if M is not positive definite.
bool cholesky_solve(std::vector<double> M, int n, const double *b, double *x)
{
    for (int i = 0; i < n; ++i)
        for (int j = 0; j <= i; ++j) {
            double s = M[i * n + j];
            for (int k = 0; k < j; ++k) s -= M[i * n + k] * M[j * n + k];
            if (i == j) {
                if (!(s > 0.0)) return false;
                M[i * n + i] = std::sqrt(s);
            } else {
                M[i * n + j] = s / M[j * n + j];
            }
        }
    std::vector<double> y(n);
    for (int i = 0; i < n; ++i) {
        double s = b[i];
        for (int k = 0; k < i; ++k) s -= M[i * n + k] * y[k];
        y[i] = s / M[i * n + i];
    }
    for (int i = n - 1; i >= 0; --i) {
        double s = y[i];
        for (int k = i + 1; k < n; ++k) s -= M[k * n + i] * x[k];
        x[i] = s / M[i * n + i];
    }
    return true;
}

// Normal equations of one point: chi2, A (nf x nf), g (nf).
struct LMSys {
    double chi2 = INFINITY;
    std::vector<double> A, g;
    bool finite = false;
};

// Domain-safe bounds: every finite-difference row stays inside the model's domain.
void domain_bounds(int rc, double *lo, double *hi)
{
    const double tiny = 1e-6;
    lo[P_INC] = std::max(lo[P_INC], 1e-3);
    hi[P_INC] = std::min(hi[P_INC], 90.0 - 1e-3);
    for (int k : {P_SIG, P_R0, P_RT, P_I0}) lo[k] = std::max(lo[k], tiny);
    if (rc == RC_EPINAT) {
        lo[P_G] = std::max(lo[P_G], tiny);
        lo[P_A] = std::max(lo[P_A], 0.0);
    }
}

}  // namespace

extern "C" gk_status gk_lm_default_opts(gk_lm_opts *o)
{
    if (!o) return fail(GK_EINVAL, "opts is NULL");
    o->max_iter = 200;
    o->reserved = 0;
    o->fd_step = 0.1;
    o->lambda0 = 1e-3;
    o->ftol = 1e-10;
    o->xtol = 1e-10;
    return GK_OK;
}

extern "C" gk_status gk_fit_lm(gk_model *m, double *p_io, const uint8_t *free_mask,
                               const double *lo_in, const double *hi_in, const gk_lm_opts *o_in,
                               gk_lm_result *res)
{
    if (!m || !p_io || !free_mask || !res) return fail(GK_EINVAL, "NULL argument");
    if (!m->has_obs) return fail(GK_ESTATE, "no observation set");
    gk_lm_opts o;
    gk_lm_default_opts(&o);
    if (o_in) o = *o_in;
    if (o.max_iter < 1 || !(o.fd_step > 0.0) || !(o.lambda0 > 0.0) || o.reserved != 0)
        return fail(GK_EINVAL, "invalid LM options");
    double lo[NPAR], hi[NPAR], p[NPAR];
    for (int k = 0; k < NPAR; ++k) {
        lo[k] = lo_in ? lo_in[k] : -DBL_MAX;
        hi[k] = hi_in ? hi_in[k] : DBL_MAX;
        if (!(lo[k] <= hi[k])) return fail(GK_EINVAL, "lo > hi in slot %d", k);
    }
    domain_bounds(m->d.rc, lo, hi);
    for (int k = 0; k < NPAR; ++k) p[k] = std::min(std::max(p_io[k], lo[k]), hi[k]);
    if (!row_valid(p, m->d.rc)) return fail(GK_EINVAL, "start point outside the model domain");
    std::vector<int> fr;
    for (int k = 0; k < NPAR; ++k)
        if (free_mask[k] && hi[k] > lo[k]) fr.push_back(k);
    const int nf = (int)fr.size(), rows = 1 + 2 * nf;
    DeviceGuard g(m->device);
    HIP_TRY(g.err);
    GK_TRY(fit_reserve(m, rows, rows));
    FitWork *w = m->fit;
    const size_t npix = (size_t)m->d.nx * m->d.ny;
    const int n = (int)(2 * npix);
    int64_t n_evals = 0;

    LMIdx ix{};
    ix.nf = nf;
    ix.npairs = nf * (nf + 1) / 2;
    for (int a = 0, k = 0; a < nf; ++a)
        for (int b = a; b < nf; ++b, ++k) {
            ix.pa[k] = (unsigned char)a;
            ix.pb[k] = (unsigned char)b;
        }
    const int nblk = ix.npairs + nf + 1;

    // residual rows of pc and its Jacobian rows -> chi2, A, g
    auto evaluate = [&](const double *pc, LMSys &sys) -> gk_status {
        double *hp = w->h_params;
        std::memcpy(hp, pc, sizeof(double) * NPAR);
        for (int a = 0; a < nf; ++a) {
            const int k = fr[a];
            double *rp = hp + (size_t)(1 + 2 * a) * NPAR, *rm = rp + NPAR;
            std::memcpy(rp, pc, sizeof(double) * NPAR);
            std::memcpy(rm, pc, sizeof(double) * NPAR);
            rp[k] = std::min(pc[k] + o.fd_step, hi[k]);
            rm[k] = std::max(pc[k] - o.fd_step, lo[k]);
            ix.ip[a] = 1 + 2 * a;
            ix.im[a] = 2 + 2 * a;
            ix.s[a] = 1.0 / (rp[k] - rm[k]);
        }
        HIP_TRY(hipMemcpyAsync(w->d_params, hp, sizeof(double) * NPAR * rows, hipMemcpyHostToDevice,
                               w->stream));
        GK_TRY(run_batch(m, w->d_params, rows, nullptr, w->d_resid, nullptr, nullptr, w->stream));
        // without a weighted dispersion term the second map of each row is 0
        const int64_t used = m->obs_sig ? n : n / 2;
        int64_t *goff = (int64_t *)w->h_aux;
        goff[0] = 0;
        goff[1] = (int64_t)rows * n;
        goff[2] = used;
        goff[3] = 0;
        std::memcpy(w->h_aux + 4 * sizeof(int64_t), ix.s, sizeof(double) * nf);
        HIP_TRY(hipMemcpyAsync(w->d_aux, w->h_aux, kAuxBytes, hipMemcpyHostToDevice, w->stream));
        HIP_TRY(launch_lm_normal(w->d_resid, (const int64_t *)w->d_aux,
                                 (const int64_t *)w->d_aux + 2,
                                 (const double *)(w->d_aux + 4 * sizeof(int64_t)), 1, nf,
                                 lm_normal_chunks(used), w->d_part, w->d_norm, w->stream));
        HIP_TRY(hipMemcpyAsync(w->h_norm, w->d_norm, sizeof(double) * nblk, hipMemcpyDeviceToHost,
                               w->stream));
        HIP_TRY(hipStreamSynchronize(w->stream));
        n_evals += rows;
        sys.A.assign((size_t)nf * nf, 0.0);
        sys.g.assign(nf, 0.0);
        bool fin = true;
        for (int k = 0; k < ix.npairs; ++k) {
            const double v = w->h_norm[k];
            sys.A[ix.pa[k] * nf + ix.pb[k]] = sys.A[ix.pb[k] * nf + ix.pa[k]] = v;
            fin = fin && std::isfinite(v);
        }
        for (int a = 0; a < nf; ++a) {
            sys.g[a] = w->h_norm[ix.npairs + a];
            fin = fin && std::isfinite(sys.g[a]);
        }
        sys.chi2 = w->h_norm[nblk - 1];
        if (!std::isfinite(sys.chi2)) sys.chi2 = INFINITY;
        sys.finite = fin && std::isfinite(sys.chi2);
        return GK_OK;
    };

    LMSys cur, trial;
    GK_TRY(evaluate(p, cur));
    if (!cur.finite) return fail(GK_EINVAL, "non-finite residuals at the start point");
    double lam = o.lambda0;
    int it = 0, reason = GK_LM_MAXITER;
    std::vector<double> d(nf), pt(NPAR);
    while (it < o.max_iter) {
        ++it;
        // active slots: non-zero Jacobian column
        std::vector<int> act;
        for (int a = 0; a < nf; ++a)
            if (cur.A[a * nf + a] > 0.0) act.push_back(a);
        std::fill(d.begin(), d.end(), 0.0);
        const int na = (int)act.size();
        if (na) {
            std::vector<double> M((size_t)na * na), rhs(na), x(na);
            for (int i = 0; i < na; ++i) {
                for (int j = 0; j < na; ++j) M[i * na + j] = cur.A[act[i] * nf + act[j]];
                M[i * na + i] *= 1.0 + lam;
                rhs[i] = -cur.g[act[i]];
            }
            if (cholesky_solve(M, na, rhs.data(), x.data()))
                for (int i = 0; i < na; ++i) d[act[i]] = x[i];
        }
        std::memcpy(pt.data(), p, sizeof p);
        for (int a = 0; a < nf; ++a) {
            const int k = fr[a];
            pt[k] = std::min(std::max(p[k] + d[a], lo[k]), hi[k]);
        }
        GK_TRY(evaluate(pt.data(), trial));
        if (trial.finite && trial.chi2 < cur.chi2) {
            double step = 0.0;
            for (int a = 0; a < nf; ++a) {
                const int k = fr[a];
                step = std::max(step, std::fabs(pt[k] - p[k]) / (std::fabs(p[k]) + 1e-10));
            }
            const double dec = cur.chi2 > 0.0 ? (cur.chi2 - trial.chi2) / cur.chi2 : 0.0;
            std::memcpy(p, pt.data(), sizeof p);
            std::swap(cur, trial);
            lam /= 10.0;
            if (cur.chi2 == 0.0 || dec <= o.ftol) {
                reason = GK_LM_FTOL;
                break;
            }
            if (step <= o.xtol) {
                reason = GK_LM_XTOL;
                break;
            }
        } else {
            lam *= 10.0;
            if (lam > 1e10) {
                reason = GK_LM_LAMBDA;
                break;
            }
        }
    }
    // errors: sqrt(diag(A^-1)) over the active slots
    std::memset(res->errors, 0, sizeof res->errors);
    {
        std::vector<int> act;
        for (int a = 0; a < nf; ++a)
            if (cur.A[a * nf + a] > 0.0) act.push_back(a);
        const int na = (int)act.size();
        std::vector<double> M((size_t)na * na), e(na), col(na);
        for (int i = 0; i < na; ++i)
            for (int j = 0; j < na; ++j) M[i * na + j] = cur.A[act[i] * nf + act[j]];
        for (int i = 0; i < na; ++i) {
            std::fill(e.begin(), e.end(), 0.0);
            e[i] = 1.0;
            if (cholesky_solve(M, na, e.data(), col.data()))
                res->errors[fr[act[i]]] = std::sqrt(std::max(col[i], 0.0));
        }
    }
    std::memcpy(p_io, p, sizeof p);
    res->chi2 = cur.chi2;
    res->n_valid = m->nvalid;
    res->iterations = it;
    res->reason = reason;
    res->n_evals = n_evals;
    return reason == GK_LM_MAXITER ? GK_ENOTCONV : GK_OK;
}

namespace gbk {

// Parameter-row and chi-square buffers of the fitter workspace (for the
// nested sampler and the grid search).
gk_status fit_reserve_rows(gk_model *m, int rows, double **h_params, double **d_params,
                           double **d_chi2, double **h_chi2, hipStream_t *stream)
{
    GK_TRY(fit_reserve(m, rows, 0));
    *h_params = m->fit->h_params;
    *d_params = m->fit->d_params;
    *d_chi2 = m->fit->d_chi2;
    *h_chi2 = m->fit->h_chi2;
    *stream = m->fit->stream;
    return GK_OK;
}

}  // namespace gbk
