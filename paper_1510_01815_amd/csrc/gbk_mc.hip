// gbk_mc.hip -- Monte-Carlo parameter errors (Bekiaris et al. 2016, Sec. 4.2
// and Sec. 4.3): simulated observations built on the device from a best fit,
// refitted all at once by the survey Levenberg-Marquardt.
//
// Shuffle (Sec. 4.2): the best fit's residual field is re-dealt over the
// unmasked pixels by a permutation per simulation and added to the best-fit
// field.  Perturb (Sec. 4.3): every unmasked pixel of the observed maps moves
// by its measurement error times a standard normal draw.  The permutations
// and the normal draws are inputs.  Each simulation is a model of its own
// (same instrument, its own observation); a group of them forms a survey, so
// one launch chain per LM iteration evaluates every simulation's trial point
// and Jacobian rows.
#include <hip/hip_runtime.h>

#include <cfloat>
#include <cmath>
#include <cstring>
#include <vector>

#include "gbk_model.h"

using namespace gbk;

namespace {

// Residuals of the LM workspace per group (1 + 2 n_free rows of 2 maps each).
constexpr size_t kMcResidBudget = (size_t)4 << 30;

// V_sim(p) = V_best(p) + R(q), q = valid[perm[k]] for p = valid[k], with
// V_best(p) = vo(p) + rv(p) / iev(p) and R(q) = -rv(q) / iev(q) from the best
// fit's residuals rv = (V_best - vo) iev; the dispersion map likewise when the
// observation has that term.  Masked pixels keep their values.
__global__ void k_mc_shuffle(const int *__restrict__ valid, const int *__restrict__ perm, int nvalid,
                             const float *__restrict__ vo, const float *__restrict__ so,
                             const double *__restrict__ iev, const double *__restrict__ ies,
                             const double *__restrict__ rv, const double *__restrict__ rs, int sig,
                             float *__restrict__ vo_out, float *__restrict__ so_out)
{
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= nvalid) return;
    const int p = valid[k], q = valid[perm[k]];
    vo_out[p] = (float)(((double)vo[p] + rv[p] / iev[p]) - rv[q] / iev[q]);
    if (sig) so_out[p] = (float)(((double)so[p] + rs[p] / ies[p]) - rs[q] / ies[q]);
}

// V_sim(p) = vo(p) + E_v(p) n_v(p), E_v = 1 / iev; sigma likewise with
// E_s = sqrt(W) / ies when the observation has that term.
__global__ void k_mc_perturb(const int *__restrict__ valid, int nvalid, int npix,
                             const float *__restrict__ noise, const float *__restrict__ vo,
                             const float *__restrict__ so, const double *__restrict__ iev,
                             const double *__restrict__ ies, int sig, double sqrt_w,
                             float *__restrict__ vo_out, float *__restrict__ so_out)
{
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= nvalid) return;
    const int p = valid[k];
    vo_out[p] = (float)((double)vo[p] + (double)noise[p] / iev[p]);
    if (sig) so_out[p] = (float)((double)so[p] + (double)noise[npix + p] * (sqrt_w / ies[p]));
}

struct DevMem {
    void *p = nullptr;
    ~DevMem() { (void)hipFree(p); }
    template <class T> T *as() const { return (T *)p; }
};

// Clones the parent's instrument and observation (the velocity and
// dispersion maps to be overwritten by the caller).
gk_status clone_model(const gk_model *m, gk_model **out)
{
    GK_TRY(gk_create_model(&m->d, m->device, out));
    gk_model *c = *out;
    const size_t n = (size_t)m->d.nx * m->d.ny;
    HIP_TRY(dev_alloc(&c->d_vo, n));
    HIP_TRY(dev_alloc(&c->d_so, n));
    HIP_TRY(dev_alloc(&c->d_iev, n));
    HIP_TRY(dev_alloc(&c->d_ies, n));
    HIP_TRY(dev_alloc(&c->d_mask, n));
    HIP_TRY(hipMemcpy(c->d_vo, m->d_vo, n * sizeof(float), hipMemcpyDeviceToDevice));
    HIP_TRY(hipMemcpy(c->d_so, m->d_so, n * sizeof(float), hipMemcpyDeviceToDevice));
    HIP_TRY(hipMemcpy(c->d_iev, m->d_iev, n * sizeof(double), hipMemcpyDeviceToDevice));
    HIP_TRY(hipMemcpy(c->d_ies, m->d_ies, n * sizeof(double), hipMemcpyDeviceToDevice));
    HIP_TRY(hipMemcpy(c->d_mask, m->d_mask, n, hipMemcpyDeviceToDevice));
    c->nvalid = m->nvalid;
    c->obs_sig = m->obs_sig;
    c->obs_W = m->obs_W;
    c->has_obs = true;
    return GK_OK;
}

struct Clones {
    std::vector<gk_model *> v;
    gk_survey *s = nullptr;
    ~Clones()
    {
        if (s) (void)gk_destroy_survey(s);
        for (gk_model *m : v) (void)gk_destroy_model(m);
    }
};

}  // namespace

extern "C" gk_status gk_mc_errors(gk_model *m, const double *best, const uint8_t *free_mask,
                                  const double *lo, const double *hi, const gk_lm_opts *opts,
                                  int32_t mode, int32_t n_sim, const int32_t *perm,
                                  const float *noise, double *fits, double *sd, int32_t *n_capped)
{
    if (!m || !best || !free_mask || !fits || !sd) return fail(GK_EINVAL, "NULL argument");
    if (!m->has_obs) return fail(GK_ESTATE, "no observation set");
    if (n_sim < 2) return fail(GK_EINVAL, "n_sim must be >= 2");
    if (mode != GK_MC_SHUFFLE && mode != GK_MC_PERTURB) return fail(GK_EINVAL, "unknown mode %d", mode);
    if (mode == GK_MC_SHUFFLE && !perm) return fail(GK_EINVAL, "shuffle needs the permutations");
    if (mode == GK_MC_PERTURB && !noise) return fail(GK_EINVAL, "perturb needs the normal draws");
    if (!m->vfield && m->use_fft)
        return fail(GK_EINVAL, "Monte-Carlo refits take direct-path models (surveys refuse the FFT path)");
    if (!row_valid(best, m->d.rc)) return fail(GK_EINVAL, "best row outside the model domain");
    const int nv = (int)m->nvalid;
    if (nv < 1) return fail(GK_EINVAL, "the observation has no unmasked pixel");
    if (mode == GK_MC_SHUFFLE) {
        std::vector<char> seen(nv);
        for (int s = 0; s < n_sim; ++s) {
            std::fill(seen.begin(), seen.end(), 0);
            const int32_t *ps = perm + (size_t)s * nv;
            for (int k = 0; k < nv; ++k) {
                if (ps[k] < 0 || ps[k] >= nv || seen[ps[k]])
                    return fail(GK_EINVAL, "simulation %d: not a permutation of 0..%d", s, nv - 1);
                seen[ps[k]] = 1;
            }
        }
    }
    int nf = 0;
    for (int k = 0; k < NPAR; ++k) nf += free_mask[k] != 0;
    if (nf == 0) return fail(GK_EINVAL, "no free parameter");
    DeviceGuard g(m->device);
    HIP_TRY(g.err);
    const int npix = m->d.nx * m->d.ny;

    // unmasked pixels in row-major order
    std::vector<uint8_t> mask(npix);
    HIP_TRY(hipDeviceSynchronize());
    HIP_TRY(hipMemcpy(mask.data(), m->d_mask, npix, hipMemcpyDeviceToHost));
    std::vector<int> valid;
    valid.reserve(nv);
    for (int p = 0; p < npix; ++p)
        if (mask[p]) valid.push_back(p);
    if ((int)valid.size() != nv) return fail(GK_EDEVICE, "mask and valid count disagree");
    DevMem d_valid, d_res, d_perm, d_noise;
    HIP_TRY(hipMalloc(&d_valid.p, sizeof(int) * nv));
    HIP_TRY(hipMemcpy(d_valid.p, valid.data(), sizeof(int) * nv, hipMemcpyHostToDevice));
    if (mode == GK_MC_SHUFFLE) {
        // residuals of the best fit, FP64 (the same path the fitter uses)
        HIP_TRY(hipMalloc(&d_res.p, sizeof(double) * 2 * (size_t)npix));
        GK_TRY(run_batch(m, best, 1, nullptr, d_res.as<double>(), nullptr, nullptr, nullptr));
        HIP_TRY(hipDeviceSynchronize());
    }

    // simulations per group: the survey LM keeps every row's residual maps
    const size_t per_sim = (size_t)(1 + 2 * nf) * 2 * npix * sizeof(double);
    const int G = (int)std::max<size_t>(1, std::min<size_t>(n_sim, kMcResidBudget / per_sim));
    std::vector<double> p_io((size_t)G * NPAR), lo_g, hi_g;
    if (lo) lo_g.resize((size_t)G * NPAR);
    if (hi) hi_g.resize((size_t)G * NPAR);
    for (int i = 0; i < G; ++i) {
        if (lo) std::memcpy(&lo_g[(size_t)i * NPAR], lo, sizeof(double) * NPAR);
        if (hi) std::memcpy(&hi_g[(size_t)i * NPAR], hi, sizeof(double) * NPAR);
    }
    std::vector<gk_lm_result> res(G);
    int capped = 0;
    // one set of clones and one survey serve every group (the last, shorter
    // group gets a survey of the first clones)
    Clones cl;
    for (int i = 0; i < G; ++i) {
        gk_model *c = nullptr;
        const gk_status st = clone_model(m, &c);
        if (c) cl.v.push_back(c);
        GK_TRY(st);
    }
    GK_TRY(gk_create_survey(cl.v.data(), G, &cl.s));
    if (mode == GK_MC_SHUFFLE) HIP_TRY(hipMalloc(&d_perm.p, sizeof(int32_t) * (size_t)G * nv));
    else HIP_TRY(hipMalloc(&d_noise.p, sizeof(float) * (size_t)G * 2 * npix));
    const int sig = m->obs_sig ? 1 : 0;
    for (int s0 = 0; s0 < n_sim; s0 += G) {
        const int ng = std::min(G, n_sim - s0);
        if (mode == GK_MC_SHUFFLE)
            HIP_TRY(hipMemcpy(d_perm.p, perm + (size_t)s0 * nv, sizeof(int32_t) * (size_t)ng * nv,
                              hipMemcpyHostToDevice));
        else
            HIP_TRY(hipMemcpy(d_noise.p, noise + (size_t)s0 * 2 * npix,
                              sizeof(float) * (size_t)ng * 2 * npix, hipMemcpyHostToDevice));
        for (int i = 0; i < ng; ++i) {
            gk_model *c = cl.v[i];
            if (mode == GK_MC_SHUFFLE)
                hipLaunchKernelGGL(k_mc_shuffle, dim3((nv + 255) / 256), dim3(256), 0, nullptr,
                                   d_valid.as<int>(), d_perm.as<int>() + (size_t)i * nv, nv,
                                   m->d_vo, m->d_so, m->d_iev, m->d_ies, d_res.as<double>(),
                                   d_res.as<double>() + npix, sig, c->d_vo, c->d_so);
            else
                hipLaunchKernelGGL(k_mc_perturb, dim3((nv + 255) / 256), dim3(256), 0, nullptr,
                                   d_valid.as<int>(), nv, npix,
                                   d_noise.as<float>() + (size_t)i * 2 * npix, m->d_vo, m->d_so,
                                   m->d_iev, m->d_ies, sig, std::sqrt(m->obs_W), c->d_vo,
                                   c->d_so);
            HIP_TRY(hipGetLastError());
        }
        HIP_TRY(hipDeviceSynchronize());
        Clones tail;  // holds only the shorter group's survey
        if (ng < G) GK_TRY(gk_create_survey(cl.v.data(), ng, &tail.s));
        for (int i = 0; i < ng; ++i) std::memcpy(&p_io[(size_t)i * NPAR], best, sizeof(double) * NPAR);
        const gk_status st = gk_fit_lm_survey(ng < G ? tail.s : cl.s, p_io.data(), free_mask,
                                              lo ? lo_g.data() : nullptr, hi ? hi_g.data() : nullptr,
                                              opts, res.data());
        if (st < 0 && st != GK_ENOTCONV) return st;
        for (int i = 0; i < ng; ++i) {
            std::memcpy(fits + (size_t)(s0 + i) * NPAR, &p_io[(size_t)i * NPAR], sizeof(double) * NPAR);
            capped += res[i].reason == GK_LM_MAXITER;
        }
    }
    // sample standard deviation over the simulations (two-pass)
    for (int k = 0; k < NPAR; ++k) {
        if (!free_mask[k]) {
            sd[k] = 0.0;
            continue;
        }
        double mean = 0.0;
        for (int s = 0; s < n_sim; ++s) mean += fits[(size_t)s * NPAR + k];
        mean /= n_sim;
        double ss = 0.0;
        for (int s = 0; s < n_sim; ++s) {
            const double d = fits[(size_t)s * NPAR + k] - mean;
            ss += d * d;
        }
        sd[k] = std::sqrt(ss / (n_sim - 1));
    }
    if (n_capped) *n_capped = capped;
    return GK_OK;
}
