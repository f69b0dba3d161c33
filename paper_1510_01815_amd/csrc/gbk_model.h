// gbk_model.h -- private: the model object behind the opaque gk_model handle,
// error helpers and the batch runner shared by the evaluation entry points
// and the fitters.
#pragma once
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <string>
#include <utility>
#include <vector>

#include "gbk.h"
#include "gbk_internal.h"

namespace gbk {

// Sets the thread's last-error message and returns `st`.
gk_status fail(gk_status st, const char *fmt, ...);

#define HIP_TRY(expr)                                                                        \
    do {                                                                                     \
        hipError_t e_ = (expr);                                                              \
        if (e_ != hipSuccess)                                                                \
            return ::gbk::fail(e_ == hipErrorOutOfMemory ? GK_ENOMEM : GK_EDEVICE,           \
                               "%s: %s (%s:%d)", #expr, hipGetErrorString(e_), __FILE__,     \
                               __LINE__);                                                    \
    } while (0)

#define GK_TRY(expr)                                                                         \
    do {                                                                                     \
        gk_status s_ = (expr);                                                               \
        if (s_ < 0) return s_;                                                               \
    } while (0)

// Restores the caller's current device on scope exit.
struct DeviceGuard {
    int prev = -1;
    hipError_t err = hipSuccess;
    explicit DeviceGuard(int dev)
    {
        if (hipGetDevice(&prev) != hipSuccess) prev = -1;
        err = hipSetDevice(dev);
    }
    ~DeviceGuard()
    {
        if (prev >= 0) (void)hipSetDevice(prev);
    }
};

// Scratch budget for the T_j planes of one chunk of rows.
constexpr size_t kScratchBudget = size_t(1) << 30;
constexpr size_t kMaxLds = 64 * 1024;

enum PtrKind { PTR_HOST, PTR_DEVICE, PTR_BAD };
PtrKind pointer_kind(const void *p);
bool row_valid(const double *p, int rc);

template <class T> hipError_t dev_alloc(T **p, size_t n)
{
    return hipMalloc((void **)p, std::max<size_t>(n, 1) * sizeof(T));
}

struct FitWork;
void fit_release(FitWork *w);

}  // namespace gbk

struct gk_model {
    // see gbk_api.hip for the meaning of each field
    gk_model_desc d{};
    int device = 0;
    int hp = 0, hl = 0, NX = 0, NY = 0, NZ = 0, EX = 0, EY = 0, NZE = 0;
    double vf0 = 0, dvf = 0, inv_dvf = 0, vref = 0;
    // Fine channel positions between which the spectral weight W0 is at least
    // 2^-5 of its largest value.  A line centred outside them (in the LSF
    // taper at a band edge, or beyond the band) can have most of its weighted
    // flux in channels below the 2^-40 support cut, so its sums run over the
    // whole band.
    float zedge_lo = 0.0f, zedge_hi = 0.0f;
    int TXd = 0, TYd = 0, ntx = 0, nty = 0, ntiles = 0;
    // velocity-field strategy (Sec. 2.2.1): no cube, ntiles = pixel tiles of k_vfield
    bool vfield = false;
    size_t lds_bytes = 0;
    double *d_kp = nullptr, *d_wz = nullptr;
    // FFT path of the spatial convolution (gbk_fft.hip)
    bool use_fft = false, fft_ok = false;
    gbk::FftArgs fft{};  // sizes, twiddles and spectra; T/U set per chunk
    double2 *d_twx = nullptr, *d_twy = nullptr;
    double *d_kbx = nullptr, *d_kby = nullptr, *d_U = nullptr;
    // observation
    bool has_obs = false;
    bool obs_sig = false;  // the observation's dispersion weight W > 0
    double obs_W = 0.0;    // that weight
    int64_t nvalid = 0;
    float *d_vo = nullptr, *d_so = nullptr;
    double *d_iev = nullptr, *d_ies = nullptr;
    uint8_t *d_mask = nullptr;
    // scratch, sized for `cap` rows
    int cap = 0;
    double *d_params = nullptr, *d_consts = nullptr, *d_T = nullptr, *d_partial = nullptr;
    // pinned staging of host-given rows; ev_staged marks when its last copy is done
    double *h_params = nullptr;
    hipEvent_t ev_staged = nullptr;
    // measurement hooks (gk_set_profiling)
    int prof_flags = 0;
    std::vector<std::vector<std::pair<int, std::pair<hipEvent_t, hipEvent_t>>>> prof_events;
    unsigned long long *d_count = nullptr;
    int64_t prof_rows = 0;
    // fitter workspace (gbk_fit.hip), created on first use
    gbk::FitWork *fit = nullptr;
    // HIP graphs of repeated launch chains (run_batch); gen changes whenever a
    // pointer or size baked into a recorded chain may have changed
    struct GraphKey {
        const void *params, *maps, *resid, *chi2, *nvalid;
        hipStream_t stream;
        int B;
        uint64_t gen;
        bool operator==(const GraphKey &o) const
        {
            return params == o.params && maps == o.maps && resid == o.resid && chi2 == o.chi2 &&
                   nvalid == o.nvalid && stream == o.stream && B == o.B && gen == o.gen;
        }
    };
    struct GraphEntry {
        GraphKey key;
        hipGraph_t graph;
        hipGraphExec_t exec;
    };
    int launch_mode = GK_LAUNCH_GRAPH;
    uint64_t gen = 0;
    std::vector<GraphEntry> graphs;  // at most kMaxGraphs, oldest first
    std::vector<GraphKey> seen;      // keys met once, not yet recorded
    int64_t graph_launches = 0;

    void drop_graphs()
    {
        if (!graphs.empty()) (void)hipDeviceSynchronize();  // a replay may still run
        for (auto &g : graphs) {
            (void)hipGraphExecDestroy(g.exec);
            (void)hipGraphDestroy(g.graph);
        }
        graphs.clear();
        seen.clear();
        ++gen;
    }

    int chunk_rows() const
    {
        if (vfield) return 65535;  // per-row scratch: constants and tile partials only
        size_t per = (size_t)3 * EX * EY * sizeof(double);
        if (use_fft) per += (size_t)3 * EY * NX * sizeof(double);
        size_t n = std::max<size_t>(1, gbk::kScratchBudget / per);
        return (int)std::min<size_t>(n, 65535);
    }

    size_t count_slots() const
    {
        return (size_t)chunk_rows() * ((EX + 15) / 16) * ((EY + 15) / 16) * 4;
    }

    hipError_t reserve(int rows)
    {
        if (rows <= cap) return hipSuccess;
        drop_graphs();
        (void)hipFree(d_params);
        (void)hipFree(d_consts);
        (void)hipFree(d_T);
        (void)hipFree(d_partial);
        (void)hipFree(d_U);
        if (h_params) {
            if (ev_staged) (void)hipEventSynchronize(ev_staged);
            (void)hipHostFree(h_params);
        }
        d_params = d_consts = d_T = d_partial = h_params = d_U = nullptr;
        cap = 0;
        hipError_t e;
        if (!ev_staged && (e = hipEventCreateWithFlags(&ev_staged, hipEventDisableTiming)) != hipSuccess)
            return e;
        if ((e = hipHostMalloc((void **)&h_params, sizeof(double) * gbk::NPAR * rows, 0)) != hipSuccess)
            return e;
        if ((e = gbk::dev_alloc(&d_params, (size_t)rows * gbk::NPAR)) != hipSuccess) return e;
        if ((e = gbk::dev_alloc(&d_consts, (size_t)rows * gbk::NCONST)) != hipSuccess) return e;
        if (!vfield && (e = gbk::dev_alloc(&d_T, (size_t)rows * 3 * EX * EY)) != hipSuccess)
            return e;
        if ((e = gbk::dev_alloc(&d_partial, (size_t)rows * ntiles)) != hipSuccess) return e;
        if (use_fft && (e = gbk::dev_alloc(&d_U, (size_t)rows * 3 * EY * NX)) != hipSuccess) return e;
        cap = rows;
        return hipSuccess;
    }

    // frees the row scratch (sizes depend on the convolution configuration)
    void drop_scratch()
    {
        drop_graphs();
        (void)hipDeviceSynchronize();
        (void)hipFree(d_params);
        (void)hipFree(d_consts);
        (void)hipFree(d_T);
        (void)hipFree(d_partial);
        (void)hipFree(d_U);
        (void)hipFree(d_count);
        if (h_params) (void)hipHostFree(h_params);
        d_params = d_consts = d_T = d_partial = h_params = d_U = nullptr;
        d_count = nullptr;
        cap = 0;
    }

    void release()
    {
        (void)hipFree(d_kp);
        (void)hipFree(d_wz);
        (void)hipFree(d_vo);
        (void)hipFree(d_so);
        (void)hipFree(d_iev);
        (void)hipFree(d_ies);
        (void)hipFree(d_mask);
        (void)hipFree(d_params);
        (void)hipFree(d_consts);
        (void)hipFree(d_T);
        (void)hipFree(d_partial);
        (void)hipFree(d_U);
        (void)hipFree(d_twx);
        (void)hipFree(d_twy);
        (void)hipFree(d_kbx);
        (void)hipFree(d_kby);
        drop_graphs();
        gbk::fit_release(fit);
        fit = nullptr;
        if (h_params) (void)hipHostFree(h_params);
        if (ev_staged) (void)hipEventDestroy(ev_staged);
        (void)hipFree(d_count);
        for (auto &call : prof_events)
            for (auto &k : call) {
                (void)hipEventDestroy(k.second.first);
                (void)hipEventDestroy(k.second.second);
            }
    }
};

namespace gbk {

// Evaluates B rows (host or device) on `stream`: any of maps [B][3][ny][nx]
// float, resid [B][2][ny][nx] double, chi2 [B] / nvalid [B] (device; with
// mapped_chi2, chi2 may also be the device address of pinned, device-mapped
// host memory, which the chi-square reduction then writes directly).
gk_status run_batch(gk_model *m, const double *params, int32_t B, float *maps, double *resid,
                    double *chi2, int64_t *nvalid, void *stream, bool mapped_chi2 = false);

// The launch chain of B rows in device memory on stream s, using the model's
// row scratch (already reserved for min(B, chunk_rows()) rows when the caller
// records a graph), outside the model's own graph replay.
gk_status enqueue_device_rows(gk_model *m, const double *d_params, int32_t B, float *maps,
                              double *resid, double *chi2, int64_t *nvalid, hipStream_t s);

// PSF/moment-pass arguments of a model (row pointers and outputs unset); the
// observation's pointers when with_obs.
PsfArgs psf_args(const gk_model *m, bool with_obs);

// Data tile of a model inside a survey: the model's own, except that the
// 64 x 32 register-blocked tile (which the survey kernels do not run) becomes
// the 32 x 32 one, or a generic tile where that does not apply.
struct SurveyTile {
    int TXd, TYd, ntx, nty, ntiles;
    size_t lds_bytes;
};
void survey_tile(const gk_model *m, SurveyTile *t);

// Switches the spatial convolution to the FFT path or to direct data tiles of
// tx x ty; false (nothing changed) if the configuration does not fit.  Frees
// the row scratch.
bool set_conv_config(gk_model *m, bool fft, int tx, int ty);

}  // namespace gbk
