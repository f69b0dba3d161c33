// gbk_tune.hip -- the launch-shape autotuner: times the spatial-convolution
// configurations a model can run (the FFT path and direct data tiles) on a
// synthetic batch and keeps the fastest.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "gbk_model.h"

using namespace gbk;

namespace {

struct Candidate {
    bool fft;
    int tx, ty;
};

// fixed order; the result's ms[] follows it
constexpr Candidate kCandidates[] = {
    {true, 0, 0},   {false, 32, 32}, {false, 64, 32}, {false, 32, 16}, {false, 16, 16},
    {false, 32, 8}, {false, 16, 8},  {false, 8, 8},   {false, 64, 16},
};
constexpr int kNumCandidates = sizeof(kCandidates) / sizeof(kCandidates[0]);
static_assert(kNumCandidates <= 16, "gk_tune_result holds 16 timings");

// Rows of a moderately inclined disc centred in the window, its line inside
// the band, with a small deterministic spread between rows.
std::vector<double> tune_rows(const gk_model *m, int B)
{
    const gk_model_desc &d = m->d;
    const double band = 0.5 * d.nz * d.dv_kms, size = std::min(d.nx, d.ny);
    std::vector<double> p((size_t)B * NPAR);
    for (int b = 0; b < B; ++b) {
        const double f = (double)b / std::max(1, B - 1);
        double *r = p.data() + (size_t)b * NPAR;
        r[P_XO] = 0.5 * (d.nx - 1) + 0.1 * f;
        r[P_YO] = 0.5 * (d.ny - 1) - 0.1 * f;
        r[P_PA] = 30.0 + 300.0 * f;
        r[P_INC] = 30.0 + 30.0 * f;
        r[P_VSYS] = m->vref;
        r[P_VT] = 0.4 * band;
        r[P_RT] = std::max(0.5, 0.1 * size);
        r[P_SIG] = std::max(2.0 * d.dv_kms, 10.0);
        r[P_R0] = std::max(1.0, 0.2 * size);
        r[P_I0] = 1.0;
        r[P_A] = 1.0;
        r[P_G] = 1.0;
    }
    return p;
}

}  // namespace

extern "C" gk_status gk_set_conv_config(gk_model *m, int32_t conv_mode, int32_t tile_x, int32_t tile_y)
{
    if (!m) return fail(GK_EINVAL, "model is NULL");
    if (m->vfield) return fail(GK_EINVAL, "a velocity-field model has no convolution");
    if (conv_mode != GK_CONV_DIRECT && conv_mode != GK_CONV_FFT)
        return fail(GK_EINVAL, "conv_mode must be GK_CONV_DIRECT or GK_CONV_FFT");
    if (m->prof_flags) return fail(GK_ESTATE, "profiling is on");
    DeviceGuard g(m->device);
    HIP_TRY(g.err);
    if (!set_conv_config(m, conv_mode == GK_CONV_FFT, tile_x, tile_y))
        return fail(GK_EINVAL, "configuration does not fit this model");
    return GK_OK;
}

extern "C" gk_status gk_autotune(gk_model *m, int32_t B, gk_tune_result *res)
{
    if (!m || !res) return fail(GK_EINVAL, "NULL argument");
    if (m->vfield) return fail(GK_EINVAL, "a velocity-field model has no convolution to tune");
    if (B < 1 || B > 65535) return fail(GK_EINVAL, "batch must be in 1..65535");
    if (m->prof_flags) return fail(GK_ESTATE, "profiling is on");
    DeviceGuard g(m->device);
    HIP_TRY(g.err);
    std::memset(res, 0, sizeof *res);
    // keep the current configuration to restore it on failure
    const bool fft0 = m->use_fft;
    const int tx0 = m->TXd, ty0 = m->TYd;
    hipStream_t s = nullptr;
    double *d_rows = nullptr, *d_chi2 = nullptr;
    float *d_maps = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    auto cleanup = [&] {
        if (s) (void)hipStreamSynchronize(s);
        (void)hipFree(d_rows);
        (void)hipFree(d_chi2);
        (void)hipFree(d_maps);
        if (e0) (void)hipEventDestroy(e0);
        if (e1) (void)hipEventDestroy(e1);
        if (s) (void)hipStreamDestroy(s);
    };
    auto run = [&]() -> gk_status {
        HIP_TRY(hipStreamCreateWithFlags(&s, hipStreamNonBlocking));
        HIP_TRY(hipEventCreate(&e0));
        HIP_TRY(hipEventCreate(&e1));
        const std::vector<double> rows = tune_rows(m, B);
        HIP_TRY(hipMalloc((void **)&d_rows, rows.size() * sizeof(double)));
        HIP_TRY(hipMemcpy(d_rows, rows.data(), rows.size() * sizeof(double), hipMemcpyHostToDevice));
        if (m->has_obs) HIP_TRY(hipMalloc((void **)&d_chi2, (size_t)B * sizeof(double)));
        else HIP_TRY(hipMalloc((void **)&d_maps, (size_t)B * 3 * m->d.nx * m->d.ny * sizeof(float)));
        const int saved_mode = m->launch_mode;
        m->launch_mode = GK_LAUNCH_EAGER;
        double best = INFINITY;
        int best_k = -1;
        for (int k = 0; k < kNumCandidates; ++k) {
            const Candidate &c = kCandidates[k];
            res->ms[k] = -1.0;
            const bool allowed = m->d.conv_mode == GK_CONV_AUTO ||
                                 (m->d.conv_mode == GK_CONV_FFT) == c.fft;
            if (!allowed || !set_conv_config(m, c.fft, c.tx, c.ty)) continue;
            auto once = [&]() {
                return run_batch(m, d_rows, B, d_maps, nullptr, d_chi2, nullptr, s);
            };
            gk_status st = once();  // warm-up (allocates the scratch)
            if (st < 0) {
                m->launch_mode = saved_mode;
                return st;
            }
            float ms_min = INFINITY;
            for (int rep = 0; rep < 3; ++rep) {
                HIP_TRY(hipEventRecord(e0, s));
                GK_TRY(once());
                HIP_TRY(hipEventRecord(e1, s));
                HIP_TRY(hipEventSynchronize(e1));
                float ms = 0.f;
                HIP_TRY(hipEventElapsedTime(&ms, e0, e1));
                ms_min = std::min(ms_min, ms);
            }
            res->ms[k] = ms_min;
            ++res->n_candidates;
            if (ms_min < best) {
                best = ms_min;
                best_k = k;
            }
        }
        m->launch_mode = saved_mode;
        if (best_k < 0) return fail(GK_EINVAL, "no configuration fits this model");
        const Candidate &c = kCandidates[best_k];
        if (!set_conv_config(m, c.fft, c.tx, c.ty)) return fail(GK_EINVAL, "configuration lost");
        res->conv_mode = c.fft ? GK_CONV_FFT : GK_CONV_DIRECT;
        res->tile_x = c.fft ? 0 : c.tx;
        res->tile_y = c.fft ? 0 : c.ty;
        res->ms_best = best;
        return GK_OK;
    };
    const gk_status st = run();
    cleanup();
    if (st < 0) (void)set_conv_config(m, fft0, tx0, ty0);
    return st;
}
