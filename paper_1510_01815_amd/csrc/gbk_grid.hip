// gbk_grid.hip -- nested-grid brute-force search (Sec. 2.3.3): nodes are
// generated on the device, evaluated in batched chi-square launches, and
// reduced to the least-chi2 node (lowest linear index on ties) on the device.
#include <hip/hip_runtime.h>

#include <cfloat>
#include <cmath>
#include <cstring>
#include <vector>

#include "gbk_model.h"

using namespace gbk;

namespace gbk {
gk_status fit_reserve_rows(gk_model *m, int rows, double **h_params, double **d_params,
                           double **d_chi2, double **h_chi2, hipStream_t *stream);
}

namespace {

struct GridSpec {
    int d;
    int n[NPAR];  // nodes along free slot a
    int slot[NPAR];
    double lo[NPAR], step[NPAR];
    double fixed[NPAR];
};

// Rows of nodes [first, first + count): digit a of the node index (mixed
// radix n_a, first free slot most significant) selects lo_a + digit * step_a.
__global__ void k_grid_rows(GridSpec g, int64_t first, int count, double *__restrict__ rows)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= count) return;
    double *r = rows + (size_t)i * NPAR;
    for (int k = 0; k < NPAR; ++k) r[k] = g.fixed[k];
    int64_t L = first + i;
    for (int a = g.d - 1; a >= 0; --a) {
        const int digit = (int)(L % g.n[a]);
        L /= g.n[a];
        r[g.slot[a]] = g.lo[a] + digit * g.step[a];
    }
}

// (min chi2, lowest index) of chi2[0..count) offset by `first`; one block of
// 256 threads, fixed-order reduction; NaN counts as +inf.
__global__ __launch_bounds__(256) void k_argmin(const double *__restrict__ chi2, int count,
                                                int64_t first, double *__restrict__ out_val,
                                                int64_t *__restrict__ out_idx)
{
    double best = INFINITY;
    int64_t bi = INT64_MAX;
    for (int i = threadIdx.x; i < count; i += 256) {
        const double v = chi2[i] == chi2[i] ? chi2[i] : INFINITY;
        if (v < best) {  // strictly less: the first (lowest) index wins within a thread
            best = v;
            bi = first + i;
        }
    }
    __shared__ double sv[256];
    __shared__ int64_t si[256];
    sv[threadIdx.x] = best;
    si[threadIdx.x] = bi;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (threadIdx.x < s) {
            const double a = sv[threadIdx.x], b = sv[threadIdx.x + s];
            const int64_t ia = si[threadIdx.x], ib = si[threadIdx.x + s];
            if (b < a || (b == a && ib < ia)) {
                sv[threadIdx.x] = b;
                si[threadIdx.x] = ib;
            }
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        *out_val = sv[0];
        *out_idx = si[0];
    }
}

}  // namespace

extern "C" gk_status gk_fit_grid_nd(gk_model *m, const double *lo0, const double *hi0,
                                    const uint8_t *free_mask, const double *fixed,
                                    const int32_t *n_per_slot, int32_t max_levels,
                                    const double *accuracy, gk_grid_result *res)
{
    if (!m || !lo0 || !hi0 || !free_mask || !fixed || !n_per_slot || !res)
        return fail(GK_EINVAL, "NULL argument");
    if (!m->has_obs) return fail(GK_ESTATE, "no observation set");
    if (max_levels < 1) return fail(GK_EINVAL, "need max_levels >= 1");
    GridSpec g{};
    double lo[NPAR], hi[NPAR];
    double total = 1.0;
    for (int k = 0; k < NPAR; ++k) {
        g.fixed[k] = fixed[k];
        if (!free_mask[k]) continue;
        if (!(hi0[k] > lo0[k])) return fail(GK_EINVAL, "empty range in slot %d", k);
        if (n_per_slot[k] < 2) return fail(GK_EINVAL, "slot %d: need at least 2 nodes", k);
        g.n[g.d] = n_per_slot[k];
        total *= n_per_slot[k];
        g.slot[g.d++] = k;
        lo[k] = lo0[k];
        hi[k] = hi0[k];
    }
    if (g.d == 0) return fail(GK_EINVAL, "no free parameter");
    if (total > 2147483648.0) return fail(GK_EINVAL, "too many nodes per level");
    const int64_t nodes = (int64_t)llround(total);
    DeviceGuard guard(m->device);
    HIP_TRY(guard.err);
    const int chunk = (int)std::min<int64_t>(nodes, std::min(m->chunk_rows(), 1 << 20));
    double *h_params, *d_params, *d_chi2, *h_chi2;
    hipStream_t stream;
    GK_TRY(fit_reserve_rows(m, chunk, &h_params, &d_params, &d_chi2, &h_chi2, &stream));
    const int nchunks = (int)((nodes + chunk - 1) / chunk);
    double *d_val = nullptr;
    int64_t *d_idx = nullptr;
    HIP_TRY(hipMalloc((void **)&d_val, sizeof(double) * nchunks));
    HIP_TRY(hipMalloc((void **)&d_idx, sizeof(int64_t) * nchunks));
    std::vector<double> h_val(nchunks);
    std::vector<int64_t> h_idx(nchunks);
    int64_t n_evals = 0;
    int level = 0;
    double best_val = INFINITY;
    int64_t best_idx = 0;
    gk_status st = GK_OK;
    for (; level < max_levels; ++level) {
        for (int a = 0; a < g.d; ++a) {
            const int k = g.slot[a];
            g.lo[a] = lo[k];
            g.step[a] = (hi[k] - lo[k]) / (g.n[a] - 1);
        }
        for (int c = 0; c < nchunks && st == GK_OK; ++c) {
            const int64_t first = (int64_t)c * chunk;
            const int cnt = (int)std::min<int64_t>(chunk, nodes - first);
            hipLaunchKernelGGL(k_grid_rows, dim3((cnt + 255) / 256), dim3(256), 0, stream, g, first,
                               cnt, d_params);
            if (hipGetLastError() != hipSuccess) st = fail(GK_EDEVICE, "grid row kernel failed");
            if (st == GK_OK) st = run_batch(m, d_params, cnt, nullptr, nullptr, d_chi2, nullptr, stream);
            if (st == GK_OK) {
                hipLaunchKernelGGL(k_argmin, dim3(1), dim3(256), 0, stream, d_chi2, cnt, first,
                                   d_val + c, d_idx + c);
                if (hipGetLastError() != hipSuccess) st = fail(GK_EDEVICE, "argmin kernel failed");
            }
            n_evals += cnt;
        }
        if (st == GK_OK && (hipMemcpyAsync(h_val.data(), d_val, sizeof(double) * nchunks,
                                           hipMemcpyDeviceToHost, stream) != hipSuccess ||
                            hipMemcpyAsync(h_idx.data(), d_idx, sizeof(int64_t) * nchunks,
                                           hipMemcpyDeviceToHost, stream) != hipSuccess ||
                            hipStreamSynchronize(stream) != hipSuccess))
            st = fail(GK_EDEVICE, "argmin copy failed");
        if (st != GK_OK) break;
        best_val = INFINITY;
        best_idx = INT64_MAX;
        for (int c = 0; c < nchunks; ++c)  // chunks in index order: ties keep the lowest index
            if (h_val[c] < best_val || (h_val[c] == best_val && h_idx[c] < best_idx)) {
                best_val = h_val[c];
                best_idx = h_idx[c];
            }
        // best node and the next box
        int64_t L = best_idx;
        bool fine = accuracy != nullptr;
        for (int a = g.d - 1; a >= 0; --a) {
            const int k = g.slot[a];
            const int digit = (int)(L % g.n[a]);
            L /= g.n[a];
            const double x = g.lo[a] + digit * g.step[a];
            res->best[k] = x;
            res->spacing[k] = g.step[a];
            if (accuracy) fine = fine && g.step[a] < accuracy[k];
            lo[k] = std::max(x - g.step[a], lo0[k]);
            hi[k] = std::min(x + g.step[a], hi0[k]);
        }
        if (fine) {
            ++level;
            break;
        }
    }
    (void)hipFree(d_val);
    (void)hipFree(d_idx);
    if (st != GK_OK) return st;
    for (int k = 0; k < NPAR; ++k)
        if (!free_mask[k]) {
            res->best[k] = fixed[k];
            res->spacing[k] = 0.0;
        }
    res->chi2 = best_val;
    res->best_index = best_idx;
    res->levels = std::min(level, max_levels);
    res->reserved = 0;
    res->n_evals = n_evals;
    return GK_OK;
}

extern "C" gk_status gk_fit_grid(gk_model *m, const double *lo0, const double *hi0,
                                 const uint8_t *free_mask, const double *fixed, int32_t n,
                                 int32_t max_levels, const double *accuracy, gk_grid_result *res)
{
    if (n < 2) return fail(GK_EINVAL, "need n_per_dim >= 2");
    int32_t ns[NPAR];
    for (int k = 0; k < NPAR; ++k) ns[k] = n;
    return gk_fit_grid_nd(m, lo0, hi0, free_mask, fixed, ns, max_levels, accuracy, res);
}
