// gbk_linefit.hip -- Gaussian line fitting of every spectrum of a cube, the
// alternative to moment maps named in Bekiaris et al. 2016, Sec. 2.2.5, which
// the paper ran with mpfit on the CPU and left to a GPU Levenberg-Marquardt as
// future work (Sec. 5.2, Sec. 6).
//
// k_line_fit: one lane per spectrum, the whole fit in registers (the spectrum
// in LDS, up to 64 channels).  The cube is channel-major ([nz][nspec]), so at
// every channel the lanes of a wave read consecutive spectra (coalesced).  Per spectrum: start from the moments of
// the spectrum clipped at zero, then damped Gauss-Newton on
// A exp(-(v - mu)^2 / (2 s^2)) with the analytic Jacobian; each trial is one
// pass over the channels forming chi2, J^T J (6) and J^T r (3) at the trial
// point, used if the trial is accepted.  FP64 throughout.
#include <hip/hip_runtime.h>

#include <cmath>

#include "gbk_model.h"

using namespace gbk;

namespace {

struct LineArgs {
    const float *cube;
    int nz;
    int64_t nspec;
    double v0, dv, crpix;
    int max_iter;
    double lam0, ftol, xtol;
    float *maps;
    int32_t *status, *iters;
};

struct Sys {
    double chi2, m[6], g[3];  // m: (00, 01, 02, 11, 12, 22)
};

// Spectra of at most kLdsChannels channels are copied once into LDS (the
// workgroup's 256 spectra as [channel][lane], conflict-free); longer ones are
// read from the cube at every pass.  Both visit the channels in the same order
// with the same arithmetic, so they give identical fits.
constexpr int kLdsChannels = 64;

// Calls f(k, D_k) for the lane's channels in order.
template <bool LDS, class F>
__device__ __forceinline__ void for_channels(const LineArgs &a, const float *spec, const float *lds,
                                             F f)
{
    if constexpr (LDS) {
        for (int k = 0; k < a.nz; ++k) f(k, (double)lds[k * 256]);
    } else {
        for (int k = 0; k < a.nz; ++k) f(k, (double)spec[(size_t)k * a.nspec]);
    }
}

template <bool LDS>
__device__ inline void line_system(const LineArgs &a, const float *spec, const float *lds, double A,
                                   double mu, double s, Sys &y)
{
    double c = 0.0, m0 = 0.0, m1 = 0.0, m2 = 0.0, m3 = 0.0, m4 = 0.0, m5 = 0.0;
    double g0 = 0.0, g1 = 0.0, g2 = 0.0;
    const double is = 1.0 / s;
    for_channels<LDS>(a, spec, lds, [&](int k, double d) {
        const double v = a.v0 + (k - a.crpix) * a.dv;
        const double t = (v - mu) * is;
        const double e = exp(-0.5 * t * t);
        const double r = A * e - d;
        const double j0 = e, j1 = A * e * t * is, j2 = j1 * t;
        c += r * r;
        m0 += j0 * j0;
        m1 += j0 * j1;
        m2 += j0 * j2;
        m3 += j1 * j1;
        m4 += j1 * j2;
        m5 += j2 * j2;
        g0 += j0 * r;
        g1 += j1 * r;
        g2 += j2 * r;
    });
    y.chi2 = c;
    y.m[0] = m0; y.m[1] = m1; y.m[2] = m2; y.m[3] = m3; y.m[4] = m4; y.m[5] = m5;
    y.g[0] = g0; y.g[1] = g1; y.g[2] = g2;
}

// (M + lam diag M) d = -g by Cholesky; false if not positive definite
__device__ inline bool solve3(const double *m, const double *g, double lam, double *d)
{
    const double a00 = m[0] * (1.0 + lam), a11 = m[3] * (1.0 + lam), a22 = m[5] * (1.0 + lam);
    if (!(a00 > 0.0)) return false;
    const double l00 = sqrt(a00);
    const double l10 = m[1] / l00, l20 = m[2] / l00;
    const double s11 = a11 - l10 * l10;
    if (!(s11 > 0.0)) return false;
    const double l11 = sqrt(s11);
    const double l21 = (m[4] - l20 * l10) / l11;
    const double s22 = a22 - l20 * l20 - l21 * l21;
    if (!(s22 > 0.0)) return false;
    const double l22 = sqrt(s22);
    const double y0 = -g[0] / l00;
    const double y1 = (-g[1] - l10 * y0) / l11;
    const double y2 = (-g[2] - l20 * y0 - l21 * y1) / l22;
    d[2] = y2 / l22;
    d[1] = (y1 - l21 * d[2]) / l11;
    d[0] = (y0 - l10 * d[1] - l20 * d[2]) / l00;
    return true;
}

template <bool LDS>
__global__ __launch_bounds__(256) void k_line_fit(LineArgs a)
{
    extern __shared__ float lds_all[];
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= a.nspec) return;  // no barrier below: each lane reads only its own column
    const float *spec = a.cube + p;
    const int64_t ns = a.nspec;
    float *lds = lds_all + threadIdx.x;
    if constexpr (LDS) {
        for (int k = 0; k < a.nz; ++k) lds[k * 256] = spec[(size_t)k * a.nspec];
    }
    // start: moments of the spectrum clipped at zero
    double s0 = 0.0, s1 = 0.0;
    for_channels<LDS>(a, spec, lds, [&](int k, double d) {
        const double v = a.v0 + (k - a.crpix) * a.dv;
        d = fmax(d, 0.0);
        s0 += d;
        s1 += d * v;
    });
    int status = 0, it = 0;
    double A = 0.0, mu = __builtin_nan(""), s = __builtin_nan("");
    if (s0 > 0.0) {
        const double m = s1 / s0;
        double s2 = 0.0;
        for_channels<LDS>(a, spec, lds, [&](int k, double d) {
            const double v = a.v0 + (k - a.crpix) * a.dv;
            d = fmax(d, 0.0);
            s2 += d * (v - m) * (v - m);
        });
        const double var = s2 / s0;
        if (var > 0.0) {
            const double vfirst = a.v0 - a.crpix * a.dv, vlast = a.v0 + (a.nz - 1 - a.crpix) * a.dv;
            const double lo[3] = {0.0, fmin(vfirst, vlast), 0.25 * a.dv};
            const double hi[3] = {__builtin_inf(), fmax(vfirst, vlast), a.nz * a.dv};
            const double w = sqrt(var);
            double q[3] = {s0 * a.dv / (w * 2.5066282746310002), m, w};  // sqrt(2 pi)
            for (int i = 0; i < 3; ++i) q[i] = fmin(fmax(q[i], lo[i]), hi[i]);
            Sys cur, tri;
            line_system<LDS>(a, spec, lds, q[0], q[1], q[2], cur);
            double lam = a.lam0;
            status = 3;
            while (it < a.max_iter) {
                ++it;
                double dlt[3] = {0.0, 0.0, 0.0};
                if (!solve3(cur.m, cur.g, lam, dlt)) dlt[0] = dlt[1] = dlt[2] = 0.0;
                double qt[3];
                for (int i = 0; i < 3; ++i) qt[i] = fmin(fmax(q[i] + dlt[i], lo[i]), hi[i]);
                line_system<LDS>(a, spec, lds, qt[0], qt[1], qt[2], tri);
                if (tri.chi2 < cur.chi2) {
                    double step = 0.0;
                    for (int i = 0; i < 3; ++i) step = fmax(step, fabs(qt[i] - q[i]) / (fabs(q[i]) + 1e-10));
                    const double dec = (cur.chi2 - tri.chi2) / cur.chi2;
                    for (int i = 0; i < 3; ++i) q[i] = qt[i];
                    cur = tri;
                    lam /= 10.0;
                    if (cur.chi2 == 0.0 || dec <= a.ftol || step <= a.xtol) {
                        status = 1;
                        break;
                    }
                } else {
                    lam *= 10.0;
                    if (lam > 1e10) {
                        status = 2;
                        break;
                    }
                }
            }
            A = q[0];
            mu = q[1];
            s = q[2];
        }
    }
    a.maps[p] = status ? (float)(A * s * 2.5066282746310002) : 0.0f;
    a.maps[ns + p] = (float)mu;
    a.maps[2 * ns + p] = (float)s;
    if (a.status) a.status[p] = status;
    if (a.iters) a.iters[p] = it;
}

}  // namespace

extern "C" gk_status gk_line_default_opts(gk_line_opts *o)
{
    if (!o) return fail(GK_EINVAL, "opts is NULL");
    o->max_iter = 100;
    o->reserved = 0;
    o->lambda0 = 1e-3;
    o->ftol = 1e-12;
    o->xtol = 1e-12;
    return GK_OK;
}

extern "C" gk_status gk_fit_lines(const float *cube, int32_t nz, int64_t nspec, double v0_kms,
                                  double dv_kms, double crpix, const gk_line_opts *o_in,
                                  float *maps, int32_t *status, int32_t *iterations, void *stream)
{
    if (nspec < 0 || nz < 1) return fail(GK_EINVAL, "need nz >= 1 and nspec >= 0");
    if (nspec == 0) return GK_OK;
    if (!cube || !maps) return fail(GK_EINVAL, "cube and maps must not be NULL");
    if (!(dv_kms > 0.0) || !std::isfinite(dv_kms) || !std::isfinite(v0_kms) || !std::isfinite(crpix))
        return fail(GK_EINVAL, "channel grid must be finite with dv > 0");
    if ((double)nz * (double)nspec >= 9.0e18 / 4) return fail(GK_EINVAL, "cube too large");
    gk_line_opts o;
    gk_line_default_opts(&o);
    if (o_in) o = *o_in;
    if (o.max_iter < 1 || o.reserved != 0 || !(o.lambda0 > 0.0) || !(o.ftol >= 0.0) || !(o.xtol >= 0.0))
        return fail(GK_EINVAL, "invalid line-fit options");
    for (const void *ptr : {(const void *)cube, (const void *)maps, (const void *)status,
                            (const void *)iterations})
        if (ptr && pointer_kind(ptr) != PTR_DEVICE) return fail(GK_EINVAL, "arrays must be device memory");
    LineArgs a{};
    a.cube = cube;
    a.nz = nz;
    a.nspec = nspec;
    a.v0 = v0_kms;
    a.dv = dv_kms;
    a.crpix = crpix;
    a.max_iter = o.max_iter;
    a.lam0 = o.lambda0;
    a.ftol = o.ftol;
    a.xtol = o.xtol;
    a.maps = maps;
    a.status = status;
    a.iters = iterations;
    const int64_t blocks = (nspec + 255) / 256;
    if (blocks > 0x7fffffff) return fail(GK_EINVAL, "too many spectra");
    if (nz <= kLdsChannels)
        launch(k_line_fit<true>, dim3((unsigned)blocks), dim3(256), sizeof(float) * 256 * nz,
               (hipStream_t)stream, a);
    else
        launch(k_line_fit<false>, dim3((unsigned)blocks), dim3(256), 0, (hipStream_t)stream, a);
    HIP_TRY(hipGetLastError());
    return GK_OK;
}
