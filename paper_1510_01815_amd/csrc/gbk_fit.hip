// gbk_fit.hip -- optimisers that drive the batched evaluation (Sec. 2.3).
//
// Levenberg-Marquardt (Sec. 2.3.1): each iteration is one batched launch of
// the trial point and its finite-difference Jacobian rows (gk_residual_batch
// machinery), then one FP64 kernel forming J^T J, J^T r and chi2, then one
// thread applying the step rule (accept or reject, damping, stopping tests,
// Cholesky solve of the next step) to a state kept in device memory, so
// iterations chain on the device; a HIP graph holds eight of them and the
// host reads the state between replays.  The step rule is written out in
// gbk.h.  The survey LM (gbk_survey.hip) applies the same rule on the host.
#include <hip/hip_runtime.h>

#include <cfloat>
#include <cmath>
#include <array>
#include <cstring>
#include <new>
#include <utility>
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
    // device-resident Levenberg-Marquardt: its state, and a graph of kLMGraphIters
    // iterations recorded for the key below
    void *d_lm = nullptr, *h_lm = nullptr;
    hipGraph_t lm_graph = nullptr;
    hipGraphExec_t lm_exec = nullptr;
    struct LMKey {
        int nf = -1;
        uint64_t gen = 0;
        const void *params = nullptr, *resid = nullptr;
        bool operator==(const LMKey &o) const
        {
            return nf == o.nf && gen == o.gen && params == o.params && resid == o.resid;
        }
    } lm_key;
    void drop_lm_graph()
    {
        if (lm_exec) (void)hipGraphExecDestroy(lm_exec);
        if (lm_graph) (void)hipGraphDestroy(lm_graph);
        lm_exec = nullptr;
        lm_graph = nullptr;
        lm_key = LMKey{};
    }
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
    w->drop_lm_graph();
    (void)hipFree(w->d_lm);
    (void)hipHostFree(w->h_lm);
    if (w->stream) (void)hipStreamDestroy(w->stream);
    delete w;
}

// The value that v += __shfl_xor(v, o, 64) for o = 32, 16, ..., 1 leaves in
// every lane of the wave, bit for bit, with cheaper exchanges: a permlane32
// swap, a swizzle and four DPP moves per 32-bit half instead of six LDS
// permutes.  The swap hands each lane the pair (v[l mod 32], v[l mod 32 + 32])
// in some order, and IEEE addition commutes.  After the steps over 32, 16 and
// 8 lanes a lane's value depends only on its index mod 8, so the steps over 4,
// 2 and 1 lanes may rotate the 16 lanes of a row instead of exchanging them.
template <int CTRL> __device__ __forceinline__ double dpp_f64(double v)
{
    const uint64_t u = __builtin_bit_cast(uint64_t, v);
    const uint32_t lo = __builtin_amdgcn_mov_dpp((int)(uint32_t)u, CTRL, 0xF, 0xF, false);
    const uint32_t hi = __builtin_amdgcn_mov_dpp((int)(uint32_t)(u >> 32), CTRL, 0xF, 0xF, false);
    return __builtin_bit_cast(double, (uint64_t)lo | ((uint64_t)hi << 32));
}

__device__ __forceinline__ double wave_butterfly_sum(double v)
{
    {
        const uint64_t u = __builtin_bit_cast(uint64_t, v);
        const auto lo = __builtin_amdgcn_permlane32_swap((uint32_t)u, (uint32_t)u, false, false);
        const auto hi = __builtin_amdgcn_permlane32_swap((uint32_t)(u >> 32), (uint32_t)(u >> 32),
                                                         false, false);
        const double a = __builtin_bit_cast(double, (uint64_t)lo[0] | ((uint64_t)hi[0] << 32));
        const double b = __builtin_bit_cast(double, (uint64_t)lo[1] | ((uint64_t)hi[1] << 32));
        v = a + b;  // xor 32
    }
    {
        const uint64_t u = __builtin_bit_cast(uint64_t, v);
        constexpr int kSwap16 = 0x401F;  // bitmask mode: and 0x1F, xor 0x10
        const uint32_t lo = __builtin_amdgcn_ds_swizzle((int)(uint32_t)u, kSwap16);
        const uint32_t hi = __builtin_amdgcn_ds_swizzle((int)(uint32_t)(u >> 32), kSwap16);
        v = v + __builtin_bit_cast(double, (uint64_t)lo | ((uint64_t)hi << 32));  // xor 16
    }
    v = v + dpp_f64<0x128>(v);  // row_ror 8: xor 8
    v = v + dpp_f64<0x124>(v);  // row_ror 4
    v = v + dpp_f64<0x122>(v);  // row_ror 2
    v = v + dpp_f64<0x121>(v);  // row_ror 1
    return v;
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
    // butterfly over the lanes
#pragma unroll
    for (int k = 0; k < NB; ++k) acc[k] = wave_butterfly_sum(acc[k]);
    if (lane == 0)
#pragma unroll
        for (int k = 0; k < NB; ++k) ws[wave][k] = acc[k];
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

// State of one Levenberg-Marquardt fit on the device (gk_fit_lm): the step
// rule of the header, applied once per evaluated trial by k_lm_update, so that
// iterations follow each other on the device without the host.
struct LMDev {
    double p[NPAR], pt[NPAR], lo[NPAR], hi[NPAR];  // point, trial, box
    double A[kMaxFree * kMaxFree], g[kMaxFree];     // normal equations at p
    double chi2, lam, fd_step, ftol, xtol;
    int fr[kMaxFree];
    int nf, max_iter, it, reason, done, started;
    long long n_evals;
};
constexpr int kLMBadStart = -1;   // LMDev::reason: the start point's residuals are not finite
constexpr int kLMGraphIters = 8;  // iterations recorded per graph replay

// Rows of the trial point pt and its central-difference Jacobian rows, and
// the columns' scales 1 / (p+ - p-) (the header's rule).  After the fit has
// ended the rows are made invalid, so the evaluation kernels skip them.
__device__ void lm_rows(const LMDev *__restrict__ st, double *__restrict__ rows,
                        double *__restrict__ scale, int t)
{
    const int nf = st->nf;
    if (t < 1 + 2 * nf) {
        double *r = rows + (size_t)t * NPAR;
        for (int k = 0; k < NPAR; ++k) r[k] = st->pt[k];
        if (t > 0) {
            const int a = (t - 1) >> 1, k = st->fr[a];
            r[k] = (t & 1) ? fmin(st->pt[k] + st->fd_step, st->hi[k])
                           : fmax(st->pt[k] - st->fd_step, st->lo[k]);
        }
        if (st->done) r[P_INC] = NAN;
    }
    if (t < nf) {
        const int k = st->fr[t];
        scale[t] = 1.0 / (fmin(st->pt[k] + st->fd_step, st->hi[k]) -
                          fmax(st->pt[k] - st->fd_step, st->lo[k]));
    }
}

__global__ void k_lm_rows(const LMDev *__restrict__ st, double *__restrict__ rows,
                          double *__restrict__ scale)
{
    lm_rows(st, rows, scale, threadIdx.x);
}

#pragma clang fp contract(off)
// Work arrays of the step rule, kept in LDS by the kernels that run it (one
// thread's private arrays would live in scratch memory, where each dependent
// access of the serial solve waits on memory).
struct LMWork {
    double A[kMaxFree * kMaxFree], g[kMaxFree], M[kMaxFree * kMaxFree];
    double rhs[kMaxFree], x[kMaxFree], y[kMaxFree], d[kMaxFree];
    int act[kMaxFree];
};

// Cholesky solve of M x = b (n <= kMaxFree), as cholesky_solve on the host.
__device__ bool lm_chol(double *M, int n, const double *b, double *x, double *y)
{
    for (int i = 0; i < n; ++i)
        for (int j = 0; j <= i; ++j) {
            double v = M[i * n + j];
            for (int k = 0; k < j; ++k) v -= M[i * n + k] * M[j * n + k];
            if (i == j) {
                if (!(v > 0.0)) return false;
                M[i * n + i] = sqrt(v);
            } else {
                M[i * n + j] = v / M[j * n + j];
            }
        }
    for (int i = 0; i < n; ++i) {
        double v = b[i];
        for (int k = 0; k < i; ++k) v -= M[i * n + k] * y[k];
        y[i] = v / M[i * n + i];
    }
    for (int i = n - 1; i >= 0; --i) {
        double v = y[i];
        for (int k = i + 1; k < n; ++k) v -= M[k * n + i] * x[k];
        x[i] = v / M[i * n + i];
    }
    return true;
}

// One step of the rule: take the trial's normal equations `norm` (pairs a <= b
// in row order, then J^T r, then chi2), accept or reject the trial, test the
// stopping rules, and form the next trial point (one thread).
__device__ void lm_rule(LMDev *__restrict__ st, const double *__restrict__ norm, LMWork *__restrict__ w)
{
    if (st->done) return;
    const int nf = st->nf, npairs = nf * (nf + 1) / 2;
    st->n_evals += 1 + 2 * nf;
    double *A = w->A, *g = w->g;
    bool fin = true;
    for (int a = 0, k = 0; a < nf; ++a)
        for (int b = a; b < nf; ++b, ++k) {
            const double v = norm[k];
            A[a * nf + b] = A[b * nf + a] = v;
            fin = fin && isfinite(v);
        }
    for (int a = 0; a < nf; ++a) {
        g[a] = norm[npairs + a];
        fin = fin && isfinite(g[a]);
    }
    double chi2 = norm[npairs + nf];
    if (!isfinite(chi2)) chi2 = INFINITY;
    fin = fin && isfinite(chi2);
    bool take = false;
    if (!st->started) {
        st->started = 1;
        if (!fin) {
            st->done = 1;
            st->reason = kLMBadStart;
            return;
        }
        take = true;
    } else if (fin && chi2 < st->chi2) {
        double step = 0.0;
        for (int a = 0; a < nf; ++a) {
            const int k = st->fr[a];
            step = fmax(step, fabs(st->pt[k] - st->p[k]) / (fabs(st->p[k]) + 1e-10));
        }
        const double dec = st->chi2 > 0.0 ? (st->chi2 - chi2) / st->chi2 : 0.0;
        take = true;
        st->lam /= 10.0;
        if (chi2 == 0.0 || dec <= st->ftol) {
            st->reason = GK_LM_FTOL;
            st->done = 1;
        } else if (step <= st->xtol) {
            st->reason = GK_LM_XTOL;
            st->done = 1;
        }
    } else {
        st->lam *= 10.0;
        if (st->lam > 1e10) {
            st->reason = GK_LM_LAMBDA;
            st->done = 1;
        }
    }
    if (take) {
        for (int k = 0; k < NPAR; ++k) st->p[k] = st->pt[k];
        for (int k = 0; k < nf * nf; ++k) st->A[k] = A[k];
        for (int a = 0; a < nf; ++a) st->g[a] = g[a];
        st->chi2 = chi2;
    }
    if (st->done) return;
    if (st->it >= st->max_iter) {
        st->reason = GK_LM_MAXITER;
        st->done = 1;
        return;
    }
    st->it += 1;
    // (A + lam diag A) d = -g over the slots with a non-zero Jacobian column
    int *act = w->act, na = 0;
    for (int a = 0; a < nf; ++a)
        if (st->A[a * nf + a] > 0.0) act[na++] = a;
    double *d = w->d;
    for (int a = 0; a < nf; ++a) d[a] = 0.0;
    if (na) {
        double *M = w->M, *rhs = w->rhs, *x = w->x;
        for (int i = 0; i < na; ++i) {
            for (int j = 0; j < na; ++j) M[i * na + j] = st->A[act[i] * nf + act[j]];
            M[i * na + i] *= 1.0 + st->lam;
            rhs[i] = -st->g[act[i]];
        }
        if (lm_chol(M, na, rhs, x, w->y))
            for (int i = 0; i < na; ++i) d[act[i]] = x[i];
    }
    for (int k = 0; k < NPAR; ++k) st->pt[k] = st->p[k];
    for (int a = 0; a < nf; ++a) {
        const int k = st->fr[a];
        st->pt[k] = fmin(fmax(st->p[k] + d[a], st->lo[k]), st->hi[k]);
    }
}

// lm_rule for a compile-time number of free slots, with the damped system in
// registers: every index is static, so the serial solve keeps its operands in
// registers instead of waiting on memory.  A slot whose Jacobian column is
// zero gets an identity row and a zero right-hand side instead of being
// dropped from the system; the terms this adds are exact zeros, so the other
// slots' steps are those of the compressed solve bit for bit.
template <int NF>
__device__ void lm_rule_t(LMDev *__restrict__ st, const double *__restrict__ norm)
{
    constexpr int NPr = NF * (NF + 1) / 2;
    if (st->done) return;
    st->n_evals += 1 + 2 * NF;
    bool fin = true;
#pragma unroll
    for (int k = 0; k < NPr + NF; ++k) fin = fin && isfinite(norm[k]);
    double chi2 = norm[NPr + NF];
    if (!isfinite(chi2)) chi2 = INFINITY;
    fin = fin && isfinite(chi2);
    bool take = false;
    if (!st->started) {
        st->started = 1;
        if (!fin) {
            st->done = 1;
            st->reason = kLMBadStart;
            return;
        }
        take = true;
    } else if (fin && chi2 < st->chi2) {
        double step = 0.0;
#pragma unroll
        for (int a = 0; a < NF; ++a) {
            const int k = st->fr[a];
            step = fmax(step, fabs(st->pt[k] - st->p[k]) / (fabs(st->p[k]) + 1e-10));
        }
        const double dec = st->chi2 > 0.0 ? (st->chi2 - chi2) / st->chi2 : 0.0;
        take = true;
        st->lam /= 10.0;
        if (chi2 == 0.0 || dec <= st->ftol) {
            st->reason = GK_LM_FTOL;
            st->done = 1;
        } else if (step <= st->xtol) {
            st->reason = GK_LM_XTOL;
            st->done = 1;
        }
    } else {
        st->lam *= 10.0;
        if (st->lam > 1e10) {
            st->reason = GK_LM_LAMBDA;
            st->done = 1;
        }
    }
    if (take) {
        for (int k = 0; k < NPAR; ++k) st->p[k] = st->pt[k];
#pragma unroll
        for (int a = 0, k = 0; a < NF; ++a)
#pragma unroll
            for (int b = a; b < NF; ++b, ++k) st->A[a * NF + b] = st->A[b * NF + a] = norm[k];
#pragma unroll
        for (int a = 0; a < NF; ++a) st->g[a] = norm[NPr + a];
        st->chi2 = chi2;
    }
    if (st->done) return;
    if (st->it >= st->max_iter) {
        st->reason = GK_LM_MAXITER;
        st->done = 1;
        return;
    }
    st->it += 1;
    // (A + lam diag A) d = -g; lower triangle L(i, j) at i (i + 1) / 2 + j
    double L[NPr], y[NF], x[NF];
    bool act[NF];
    const double damp = 1.0 + st->lam;
#pragma unroll
    for (int i = 0; i < NF; ++i) act[i] = st->A[i * NF + i] > 0.0;
#pragma unroll
    for (int i = 0; i < NF; ++i)
#pragma unroll
        for (int j = 0; j <= i; ++j) {
            double v = (act[i] && act[j]) ? st->A[i * NF + j] : (i == j ? 1.0 : 0.0);
            if (i == j && act[i]) v *= damp;
            L[i * (i + 1) / 2 + j] = v;
        }
    bool ok = true;
#pragma unroll
    for (int i = 0; i < NF; ++i)
#pragma unroll
        for (int j = 0; j <= i; ++j) {
            double v = L[i * (i + 1) / 2 + j];
#pragma unroll
            for (int k = 0; k < j; ++k) v -= L[i * (i + 1) / 2 + k] * L[j * (j + 1) / 2 + k];
            if (i == j) {
                ok = ok && v > 0.0;
                L[i * (i + 1) / 2 + i] = sqrt(v);
            } else {
                L[i * (i + 1) / 2 + j] = v / L[j * (j + 1) / 2 + j];
            }
        }
#pragma unroll
    for (int i = 0; i < NF; ++i) {
        double v = act[i] ? -st->g[i] : 0.0;
#pragma unroll
        for (int k = 0; k < i; ++k) v -= L[i * (i + 1) / 2 + k] * y[k];
        y[i] = v / L[i * (i + 1) / 2 + i];
    }
#pragma unroll
    for (int i = NF - 1; i >= 0; --i) {
        double v = y[i];
#pragma unroll
        for (int k = i + 1; k < NF; ++k) v -= L[k * (k + 1) / 2 + i] * x[k];
        x[i] = v / L[i * (i + 1) / 2 + i];
    }
    for (int k = 0; k < NPAR; ++k) st->pt[k] = st->p[k];
#pragma unroll
    for (int a = 0; a < NF; ++a) {
        const int k = st->fr[a];
        const double d = ok && act[a] ? x[a] : 0.0;
        st->pt[k] = fmin(fmax(st->p[k] + d, st->lo[k]), st->hi[k]);
    }
}

// Copies of the fit state between global memory and LDS (all threads of the block).
__device__ void lm_copy(LMDev *__restrict__ dst, const LMDev *__restrict__ src)
{
    static_assert(sizeof(LMDev) % 4 == 0, "state copied as 32-bit words");
    const uint32_t *s = reinterpret_cast<const uint32_t *>(src);
    uint32_t *d = reinterpret_cast<uint32_t *>(dst);
    for (int i = threadIdx.x; i < (int)(sizeof(LMDev) / 4); i += blockDim.x) d[i] = s[i];
}

// The fit state in the registers of a block of BS threads (word t + BS q of
// the state in thread t), so that its fetch can be issued early and its store
// to LDS made later.
constexpr int kLMWords = (int)(sizeof(LMDev) / 4);
template <int BS> struct LMRegs {
    uint32_t w[(kLMWords + BS - 1) / BS];
};
template <int BS> __device__ __forceinline__ LMRegs<BS> lm_fetch(const LMDev *__restrict__ src)
{
    const uint32_t *s = reinterpret_cast<const uint32_t *>(src);
    LMRegs<BS> r;
#pragma unroll
    for (int q = 0; q < (kLMWords + BS - 1) / BS; ++q) {
        const int i = threadIdx.x + BS * q;
        r.w[q] = i < kLMWords ? s[i] : 0u;
    }
    return r;
}
template <int BS>
__device__ __forceinline__ void lm_put(LMDev *__restrict__ dst, const LMRegs<BS> &r)
{
    uint32_t *d = reinterpret_cast<uint32_t *>(dst);
#pragma unroll
    for (int q = 0; q < (kLMWords + BS - 1) / BS; ++q) {
        const int i = threadIdx.x + BS * q;
        if (i < kLMWords) d[i] = r.w[q];
    }
}

// Cross-workgroup staging of k_lm_step: the four waves' sums and the count of
// waves that have stored theirs (zero between launches: the last wave of a
// launch resets it).
struct LMRed {
    double ws[4][kNormSlots];
    unsigned int arrived, pad;
};

__global__ void k_lm_update(LMDev *__restrict__ st, const double *__restrict__ norm)
{
    __shared__ LMDev ls;
    __shared__ LMWork lw;
    lm_copy(&ls, st);
    __syncthreads();
    if (threadIdx.x == 0) lm_rule(&ls, norm, &lw);
    __syncthreads();
    lm_copy(st, &ls);
}
#pragma clang fp contract(on)

// One fused step of the Levenberg-Marquardt iteration for residual rows of a
// single chunk (n <= 16384 weighted entries): the trial's normal equations in
// the summation order of k_lm_normal_rows (thread t of 256 sums entries t,
// t + 256, ... in order, then the lanes of each wave by butterfly and the four
// waves in order, so the sums are the same bit for bit), the step rule, and
// the next trial's rows and column scales.  The four waves of that order run
// as four workgroups of 64 threads on four CUs, each fetching a quarter of the
// residual rows; a wave's lane sums go through LDS and are added in the
// butterfly's pairing order (lanes l and l + 32, then l and l + 16, ...,
// which is the value the exchanges leave in lane 0); the last workgroup to
// store its sums adds the four in order and runs the step rule and the rows.
// first: only the rows (the start of a fit; one workgroup), and the arrival
// count set to zero.
template <int NF>
__global__ __launch_bounds__(64) void k_lm_step(LMDev *__restrict__ st,
                                                const double *__restrict__ R, int64_t stride,
                                                int64_t n, double *__restrict__ rows,
                                                double *__restrict__ scale, int first,
                                                LMRed *__restrict__ red)
{
    constexpr int NP = NF * (NF + 1) / 2, NB = NP + NF + 1, SP = 65;
    __shared__ double tr[NB * SP];  // lane sums [output][lane], then the sums
    __shared__ LMDev ls;
    __shared__ int last;
    const int wave = blockIdx.x, lane = threadIdx.x, tid = 64 * wave + lane;
    const LMRegs<64> sreg = lm_fetch<64>(st);  // in flight with the residual rows
    if (first) {
        lm_put<64>(&ls, sreg);
        if (lane == 0) red->arrived = 0u;
        __syncthreads();
        lm_rows(&ls, rows, scale, lane);
        return;
    }
    double sc[NF], acc[NB];
#pragma unroll
    for (int a = 0; a < NF; ++a) sc[a] = scale[a];
#pragma unroll
    for (int k = 0; k < NB; ++k) acc[k] = 0.0;
    // entries t, t + 256, ... in order, U of them loaded before their sums
    // (the whole of a thread's entries for n <= 256 U: one wait for memory)
    constexpr int U = NF <= 6 ? 12 : NF <= 9 ? 8 : 4;
    for (int64_t i0 = tid; i0 < n; i0 += 256 * U) {
        double r0[U], j[U][NF];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int64_t i = i0 + 256 * u < n ? i0 + 256 * u : i0;
            r0[u] = R[i];
#pragma unroll
            for (int a = 0; a < NF; ++a)
                j[u][a] = (R[(size_t)(1 + 2 * a) * stride + i] - R[(size_t)(2 + 2 * a) * stride + i]) * sc[a];
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            if (i0 + 256 * u >= n) break;
            int k = 0;
#pragma unroll
            for (int a = 0; a < NF; ++a)
#pragma unroll
                for (int b = a; b < NF; ++b) acc[k++] += j[u][a] * j[u][b];
#pragma unroll
            for (int a = 0; a < NF; ++a) acc[NP + a] += j[u][a] * r0[u];
            acc[NB - 1] += r0[u] * r0[u];
        }
    }
#pragma unroll
    for (int k = 0; k < NB; ++k) tr[k * SP + lane] = acc[k];
    __syncthreads();
    for (int k = lane; k < NB; k += 64) {
        const double *v = tr + k * SP;
        double t[32];
#pragma unroll
        for (int i = 0; i < 32; ++i) t[i] = v[i] + v[i + 32];
#pragma unroll
        for (int h = 16; h > 0; h >>= 1)
#pragma unroll
            for (int i = 0; i < h; ++i) t[i] = t[i] + t[i + h];
        red->ws[wave][k] = t[0];
    }
    __threadfence();
    __syncthreads();
    if (lane == 0) last = atomicAdd(&red->arrived, 1u) == 3u;
    __syncthreads();
    if (!last) return;
    __threadfence();
    lm_put<64>(&ls, sreg);
    double *norm = tr;
    for (int k = lane; k < NB; k += 64)
        norm[k] = 0.0 + (((red->ws[0][k] + red->ws[1][k]) + red->ws[2][k]) + red->ws[3][k]);
    if (lane == 0) red->arrived = 0u;
    __syncthreads();
    if (lane == 0) lm_rule_t<NF>(&ls, norm);
    __syncthreads();
    lm_copy(st, &ls);
    lm_rows(&ls, rows, scale, lane);
}

template <int NF>
void launch_lm_step(LMDev *st, const double *R, int64_t stride, int64_t n, double *rows,
                    double *scale, int first, LMRed *red, hipStream_t s)
{
    hipLaunchKernelGGL(k_lm_step<NF>, dim3(first ? 1 : 4), dim3(64), 0, s, st, R, stride, n, rows,
                       scale, first, red);
}
using LMStepFn = void (*)(LMDev *, const double *, int64_t, int64_t, double *, double *, int,
                          LMRed *, hipStream_t);
template <int... F> constexpr auto make_lm_step_table(std::integer_sequence<int, F...>)
{
    return std::array<LMStepFn, sizeof...(F)>{&launch_lm_step<F + 1>...};
}
const auto kLMStepTable = make_lm_step_table(std::make_integer_sequence<int, kMaxFree>{});

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
        HIP_TRY(hipMalloc(&m->fit->d_lm, sizeof(LMDev) + sizeof(LMRed)));
        HIP_TRY(hipMemset((char *)m->fit->d_lm + sizeof(LMDev), 0, sizeof(LMRed)));
        HIP_TRY(hipHostMalloc(&m->fit->h_lm, sizeof(LMDev), 0));
    }
    FitWork *w = m->fit;
    if (rows > w->rows_cap) {
        HIP_TRY(hipStreamSynchronize(w->stream));
        w->drop_lm_graph();
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
        w->drop_lm_graph();
        (void)hipFree(w->d_resid);
        w->d_resid = nullptr;
        w->resid_cap = 0;
        const size_t npix = (size_t)m->d.nx * m->d.ny;
        HIP_TRY(dev_alloc(&w->d_resid, (size_t)resid_rows * 2 * npix));
        w->resid_cap = resid_rows;
    }
    return GK_OK;
}

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

    // normal-equation layout of one fit: rows * n residuals, of which the
    // first `used` per row carry weight (no dispersion term: the first map only)
    const int64_t used = m->obs_sig ? n : n / 2;
    {
        int64_t *goff = (int64_t *)w->h_aux;
        goff[0] = 0;
        goff[1] = (int64_t)rows * n;
        goff[2] = used;
        goff[3] = 0;
        LMDev &st = *(LMDev *)w->h_lm;
        std::memset(&st, 0, sizeof st);
        std::memcpy(st.p, p, sizeof p);
        std::memcpy(st.pt, p, sizeof p);
        std::memcpy(st.lo, lo, sizeof lo);
        std::memcpy(st.hi, hi, sizeof hi);
        for (int a = 0; a < nf; ++a) st.fr[a] = fr[a];
        st.nf = nf;
        st.max_iter = o.max_iter;
        st.lam = o.lambda0;
        st.fd_step = o.fd_step;
        st.ftol = o.ftol;
        st.xtol = o.xtol;
        st.chi2 = INFINITY;
    }
    HIP_TRY(hipMemcpyAsync(w->d_aux, w->h_aux, kAuxBytes, hipMemcpyHostToDevice, w->stream));
    HIP_TRY(hipMemcpyAsync(w->d_lm, w->h_lm, sizeof(LMDev), hipMemcpyHostToDevice, w->stream));
    HIP_TRY(m->reserve(std::min(rows, m->chunk_rows())));
    LMDev *d_st = (LMDev *)w->d_lm;
    LMRed *d_red = (LMRed *)((char *)w->d_lm + sizeof(LMDev));
    double *d_scale = (double *)(w->d_aux + 4 * sizeof(int64_t));
    // Small u = 1 models whose residual rows form one chunk take two launches
    // per iteration: every row's whole evaluation in one workgroup
    // (k_eval_small), then the normal equations, the step rule and the next
    // rows in one workgroup (k_lm_step); the results are those of the general
    // chain below bit for bit.
    PsfArgs pa = psf_args(m, true);
    pa.resid = w->d_resid;
    const bool fused = nf >= 1 && used <= 16384 && !m->prof_flags &&
                       eval_small_ok(pa, m->d.upsample, m->use_fft, kMaxLds);
    if (fused) {
        kLMStepTable[nf - 1](d_st, w->d_resid, n, used, w->d_params, d_scale, 1, d_red,
                             w->stream);
        HIP_TRY(hipGetLastError());
    }
    // one iteration: trial rows -> residuals -> J^T J, J^T r, chi2 -> step rule
    auto iteration = [&]() -> gk_status {
        if (fused) {
            HIP_TRY(launch_eval_small(w->d_params, m->d_wz, m->NZE, m->d.rc, m->dvf, m->vf0,
                                      m->inv_dvf, m->zedge_lo, m->zedge_hi, pa, rows, w->stream));
            kLMStepTable[nf - 1](d_st, w->d_resid, n, used, w->d_params, d_scale, 0, d_red,
                                 w->stream);
            HIP_TRY(hipGetLastError());
            return GK_OK;
        }
        hipLaunchKernelGGL(k_lm_rows, dim3(1), dim3(64), 0, w->stream, d_st, w->d_params, d_scale);
        HIP_TRY(hipGetLastError());
        GK_TRY(enqueue_device_rows(m, w->d_params, rows, nullptr, w->d_resid, nullptr, nullptr,
                                   w->stream));
        HIP_TRY(launch_lm_normal(w->d_resid, (const int64_t *)w->d_aux,
                                 (const int64_t *)w->d_aux + 2, d_scale, 1, nf,
                                 lm_normal_chunks(used), w->d_part, w->d_norm, w->stream));
        hipLaunchKernelGGL(k_lm_update, dim3(1), dim3(64), 0, w->stream, d_st, w->d_norm);
        HIP_TRY(hipGetLastError());
        return GK_OK;
    };
    // replays of kLMGraphIters recorded iterations (eager launches under the
    // profiling hooks or in eager launch mode), the state read after each
    const bool graph = m->launch_mode == GK_LAUNCH_GRAPH && !m->prof_flags;
    const FitWork::LMKey key{nf, m->gen, w->d_params, w->d_resid};
    if (graph && !(w->lm_exec && w->lm_key == key)) {
        w->drop_lm_graph();
        HIP_TRY(hipStreamBeginCapture(w->stream, hipStreamCaptureModeRelaxed));
        gk_status cst = GK_OK;
        for (int i = 0; i < kLMGraphIters && cst == GK_OK; ++i) cst = iteration();
        hipGraph_t gr = nullptr;
        const hipError_t ec = hipStreamEndCapture(w->stream, &gr);
        if (cst < 0 || ec != hipSuccess) {
            if (gr) (void)hipGraphDestroy(gr);
            if (cst < 0) return cst;
            HIP_TRY(ec);
        }
        hipGraphExec_t ex = nullptr;
        const hipError_t ei = hipGraphInstantiateWithFlags(&ex, gr, 0);
        if (ei != hipSuccess) {
            (void)hipGraphDestroy(gr);
            HIP_TRY(ei);
        }
        w->lm_graph = gr;
        w->lm_exec = ex;
        w->lm_key = key;
    }
    LMDev &hs = *(LMDev *)w->h_lm;
    for (;;) {
        if (graph) {
            HIP_TRY(hipGraphLaunch(w->lm_exec, w->stream));
        } else {
            for (int i = 0; i < kLMGraphIters; ++i) GK_TRY(iteration());
        }
        HIP_TRY(hipMemcpyAsync(&hs, d_st, sizeof(LMDev), hipMemcpyDeviceToHost, w->stream));
        HIP_TRY(hipStreamSynchronize(w->stream));
        if (hs.done) break;
    }
    if (hs.reason == kLMBadStart) return fail(GK_EINVAL, "non-finite residuals at the start point");
    std::memcpy(p, hs.p, sizeof p);
    LMSys cur;
    cur.chi2 = hs.chi2;
    cur.A.assign(hs.A, hs.A + (size_t)nf * nf);
    const int it = hs.it, reason = hs.reason;
    const int64_t n_evals = hs.n_evals;
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
