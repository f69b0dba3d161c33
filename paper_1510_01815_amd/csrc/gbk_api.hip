// gbk_api.hip -- host runtime and C ABI of libgbk.so (declared in gbk.h).
//
// Owns the per-model device state: PSF taps, the three per-channel moment
// weight tables W_j (LSF + spectral down-sampling + moment weights, see
// gbk_kernels.hip), the observation, and growable scratch for the per-row
// constants, the T_j planes and the chi-square tile partials.  Batches larger
// than the scratch budget are processed in chunks on the caller's stream.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "gbk_model.h"

using namespace gbk;

thread_local std::string g_err;

// The allocation-free entry point's row scratch (see noalloc_scratch).
static __device__ __align__(256) unsigned char scratch[GK_NOALLOC_SCRATCH_BYTES];

namespace gbk {

gk_status fail(gk_status st, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return st;
}




static double fwhm_to_sigma(double f) { return f / (2.0 * std::sqrt(2.0 * std::log(2.0))); }

// Unit-sum Gaussian taps at integer offsets -h..h, h = ceil(R sigma); a zero
// width gives the single tap 1 (eq. 9, one axis).
static std::vector<double> gaussian_taps(double sigma, double R)
{
    if (!(sigma > 0.0)) return {1.0};
    int h = (int)std::ceil(R * sigma);
    std::vector<double> t(2 * h + 1);
    double s = 0.0;
    for (int k = -h; k <= h; ++k) s += (t[k + h] = std::exp(-0.5 * (double)k * k / (sigma * sigma)));
    for (double &v : t) v /= s;
    return t;
}


PtrKind pointer_kind(const void *p)
{
    hipPointerAttribute_t at;
    std::memset(&at, 0, sizeof at);
    hipError_t e = hipPointerGetAttributes(&at, p);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return PTR_HOST;  // unregistered host memory
    }
    switch (at.type) {
    case hipMemoryTypeDevice:
    case hipMemoryTypeManaged:
        return PTR_DEVICE;
    case hipMemoryTypeHost:
    case hipMemoryTypeUnregistered:
        return PTR_HOST;
    default:
        return PTR_BAD;
    }
}

bool row_valid(const double *p, int rc)
{
    for (int k = 0; k < NPAR; ++k)
        if (!std::isfinite(p[k])) return false;
    if (!(p[P_INC] > 0.0 && p[P_INC] < 90.0)) return false;
    if (!(p[P_SIG] > 0.0 && p[P_R0] > 0.0 && p[P_RT] > 0.0 && p[P_I0] > 0.0)) return false;
    if (rc == RC_EPINAT && !(p[P_G] > 0.0 && p[P_A] >= 0.0)) return false;
    return true;
}


}  // namespace gbk


namespace {

size_t psf_lds_bytes(int TXd, int TYd, int u, int hp)
{
    size_t TX = (size_t)u * TXd, TY = (size_t)u * TYd, LX = TX + 2 * hp, LY = TY + 2 * hp;
    return sizeof(double) * (LY * LX + LY * TX + (size_t)(2 * hp + 1));
}

// LDS of the register-blocked u = 1 kernels (padded rows): the 32 x 32 tile
// keeps the y-pass rows of one plane, the 64 x 32 tile one plane of T plus its
// x-pass rows
size_t psf_u1_lds_bytes(int TX, int hp)
{
    if (TX == 32) return yx_lds_bytes(hp);
    const size_t LY = 32 + 2 * hp;
    return sizeof(double) * (LY * pad_stride(TX + 2 * hp) + LY * pad_stride(TX));
}

// The 32 x 32 register-blocked kernel addresses a T plane with 32-bit byte
// offsets.
bool fast_plane_ok(const gk_model *m)
{
    return sizeof(double) * (size_t)m->EX * (size_t)m->EY < ((size_t)1 << 31);
}

// Picks the data-pixel tile of the PSF/moment kernel.  u = 1 with an image
// of at least 16 x 16 takes the register-blocked 32 x 32 kernel; otherwise
// the tile is as large as the thread budget and the LDS limit allow, and no
// wider than the image.
void choose_tile(gk_model *m)
{
    // the register-blocked kernel takes ragged 32 x 32 tiles (loads beyond the
    // window are zero, outputs beyond it skipped); below 16 pixels a side most
    // of such a tile would be idle, and the generic tile fits the image
    if (m->d.upsample == 1 && m->d.nx >= 16 && m->d.ny >= 16 && m->hp <= kMaxFastHalo &&
        fast_plane_ok(m)) {
        const int tx = 32;
        if (psf_u1_lds_bytes(tx, m->hp) <= kMaxLds) {
            m->TXd = tx;
            m->TYd = 32;
            m->ntx = (m->d.nx + tx - 1) / tx;
            m->nty = (m->d.ny + 31) / 32;
            m->ntiles = m->ntx * m->nty;
            m->lds_bytes = psf_u1_lds_bytes(tx, m->hp);
            return;
        }
    }
    int tx = 32, ty = 16;
    while (tx > 1 && tx >= 2 * m->d.nx) tx /= 2;
    while (ty > 1 && ty >= 2 * m->d.ny) ty /= 2;
    while (psf_lds_bytes(tx, ty, m->d.upsample, m->hp) > kMaxLds && (tx > 1 || ty > 1)) {
        if (tx >= ty && tx > 1) tx /= 2;
        else ty /= 2;
    }
    m->TXd = tx;
    m->TYd = ty;
    m->ntx = (m->d.nx + tx - 1) / tx;
    m->nty = (m->d.ny + ty - 1) / ty;
    m->ntiles = m->ntx * m->nty;
    m->lds_bytes = psf_lds_bytes(tx, ty, m->d.upsample, m->hp);
}

// log2 of the smallest power of two >= n
int ceil_log2(int n)
{
    int l = 0;
    while ((1 << l) < n) ++l;
    return l;
}

int bit_reverse(int i, int bits)
{
    int r = 0;
    for (int k = 0; k < bits; ++k) r = (r << 1) | ((i >> k) & 1);
    return r;
}

// Sizes, twiddles and PSF spectra of the FFT path; false if a line or a
// column block does not fit the LDS budget.
bool setup_fft(gk_model *m, const std::vector<double> &kp, std::vector<double2> &twx,
               std::vector<double2> &twy, std::vector<double> &kbx, std::vector<double> &kby)
{
    FftArgs &f = m->fft;
    f.EX = m->EX;
    f.EY = m->EY;
    f.NXF = m->NX;
    f.hp = m->hp;
    f.logPX = std::max(1, ceil_log2(m->EX));
    f.logPY = std::max(1, ceil_log2(m->EY));
    f.PX = 1 << f.logPX;
    f.PY = 1 << f.logPY;
    f.NLX = std::max<int>(1, (int)(32768 / (sizeof(double2) * f.PX)));
    if (fft_x_lds_bytes(f) > kMaxLds) return false;
    f.DC = 0;
    for (int dc = 8; dc >= 1; dc /= 2) {
        f.DC = dc;
        if (fft_y_lds_bytes(f, m->d.upsample) <= kMaxLds) break;
        f.DC = 0;
    }
    if (f.DC == 0) return false;
    f.ncb = (m->d.nx + f.DC - 1) / f.DC;
    // tw[k] = exp(-2 pi i k / P); spectrum of the circularly placed taps,
    // real because they are symmetric, scaled by 1/P, in bit-reversed order
    auto make = [&](int P, int logP, std::vector<double2> &tw, std::vector<double> &kb) {
        tw.resize(P / 2);
        for (int k = 0; k < P / 2; ++k) {
            const double a = 2.0 * M_PI * k / P;
            tw[k] = double2{std::cos(a), -std::sin(a)};
        }
        const int h = (int)kp.size() / 2;
        std::vector<double> spec(P);
        for (int q = 0; q < P; ++q) {
            double s = 0.0;
            for (int t = -h; t <= h; ++t) {
                const long r = (((long)q * t) % P + P) % P;  // exact phase index
                s += kp[t + h] * std::cos(2.0 * M_PI * (double)r / P);
            }
            spec[q] = s / P;
        }
        kb.resize(P);
        for (int i = 0; i < P; ++i) kb[i] = spec[bit_reverse(i, logP)];
    };
    make(f.PX, f.logPX, twx, kbx);
    make(f.PY, f.logPY, twy, kby);
    return true;
}

}  // namespace

namespace {

// Row scratch of one chunk: per-row constants, T planes, chi-square tile
// partials and (FFT path) the x-pass planes, each sized for `chunk` rows.
struct RowScratch {
    double *consts = nullptr, *T = nullptr, *partial = nullptr, *U = nullptr;
    int chunk = 0;
};

// Enqueues the launch chain of B rows (every chunk) on s.  With sc == NULL
// the model's own scratch is grown to one chunk and the profiling hooks
// apply; otherwise the chain runs in *sc (device rows only, no hooks).
gk_status enqueue_batch(gk_model *m, const double *params, PtrKind pk, int32_t B, float *maps,
                        double *resid, double *chi2, int64_t *nvalid, hipStream_t s,
                        const RowScratch *sc = nullptr)
{
    RowScratch own;
    if (!sc) {
        own.chunk = std::min<int>(B, m->chunk_rows());
        HIP_TRY(m->reserve(own.chunk));
        own.consts = m->d_consts;
        own.T = m->d_T;
        own.partial = m->d_partial;
        own.U = m->d_U;
        sc = &own;
    } else if (pk != PTR_DEVICE) {
        return fail(GK_EINVAL, "rows must be device memory here");
    }
    const int chunk = sc->chunk;
    const bool hooks = sc == &own;
    const bool timing = hooks && (m->prof_flags & GK_PROF_TIMING);
    unsigned long long *counter =
        (hooks && (m->prof_flags & GK_PROF_COUNT)) ? m->d_count : nullptr;
    if (timing) m->prof_events.emplace_back();
    // launches stage `k` through `fn`; when timing, its launches carry a
    // start and a stop event (the stage's first dispatch starts, its last ends)
    auto timed = [&](int k, auto fn) -> hipError_t {
        hipEvent_t e0 = nullptr, e1 = nullptr;
        if (timing) {
            // device-scope timestamps: no system-memory fence around the dispatch
            hipError_t e = hipEventCreateWithFlags(&e0, hipEventDisableSystemFence);
            if (e != hipSuccess) return e;
            e = hipEventCreateWithFlags(&e1, hipEventDisableSystemFence);
            if (e != hipSuccess) {
                (void)hipEventDestroy(e0);
                return e;
            }
            launch_events() = {e0, e1};
        }
        hipError_t e = fn();
        if (timing) {
            launch_events() = {};
            m->prof_events.back().push_back({k, {e0, e1}});
        }
        return e;
    };
    if (hooks && m->prof_flags) m->prof_rows += B;
    const size_t npix = (size_t)m->d.nx * m->d.ny;
    for (int b0 = 0; b0 < B; b0 += chunk) {
        const int nb = std::min(chunk, B - b0);
        const double *prow = params + (size_t)b0 * NPAR;
        if (pk == PTR_HOST) {
            // the staging buffer is reused: wait for its previous copy only
            HIP_TRY(hipEventSynchronize(m->ev_staged));
            std::memcpy(m->h_params, prow, sizeof(double) * NPAR * nb);
            HIP_TRY(hipMemcpyAsync(m->d_params, m->h_params, sizeof(double) * NPAR * nb,
                                   hipMemcpyHostToDevice, s));
            HIP_TRY(hipEventRecord(m->ev_staged, s));
            prow = m->d_params;
        }
        if (m->vfield) {
            // Sec. 2.2.1: constants at u = 1 with no halo, then eq. 8 and the
            // chi-square terms per pixel (the channel width only enters
            // constants this path does not read)
            HIP_TRY(timed(0, [&] {
                return launch_prep(prow, nb, m->d.rc, 1.0, 0, 1, 0.0, 1.0, sc->consts, s);
            }));
            VfArgs v{};
            v.params = prow;
            v.consts = sc->consts;
            v.rc = m->d.rc;
            v.nx = m->d.nx;
            v.ny = m->d.ny;
            v.B = nb;
            v.ntiles = m->ntiles;
            v.rows_per_block = vfield_rows_per_block(m->ntiles, nb);
            v.use_sig = m->obs_sig;
            if (resid || chi2) {
                v.mask = m->d_mask;
                v.vo = m->d_vo;
                v.so = m->d_so;
                v.iev = m->d_iev;
                v.ies = m->d_ies;
            }
            v.maps = maps ? maps + (size_t)b0 * 3 * npix : nullptr;
            v.resid = resid ? resid + (size_t)b0 * 2 * npix : nullptr;
            v.partial = chi2 ? sc->partial : nullptr;
            HIP_TRY(timed(1, [&] { return launch_vfield(v, s); }));
            if (chi2)
                HIP_TRY(timed(3, [&] {
                    return launch_reduce_chi2(sc->partial, m->ntiles, sc->consts, m->nvalid,
                                              chi2 + b0, nvalid ? nvalid + b0 : nullptr, nb, s);
                }));
            continue;
        }
        HIP_TRY(timed(0, [&] {
            return launch_prep(prow, nb, m->d.rc, m->dvf, m->hp, m->d.upsample, m->vf0, m->inv_dvf,
                               sc->consts, s);
        }));
        HIP_TRY(timed(1, [&] {
            return launch_line_sums(sc->consts, m->d_wz, m->NZE, m->EX, m->EY, m->hp,
                                    m->d.upsample, m->d.rc, m->vf0, m->inv_dvf, m->zedge_lo,
                                    m->zedge_hi, sc->T, counter, nb, s);
        }));
        PsfArgs a = psf_args(m, resid || chi2);
        a.T = sc->T;
        a.consts = sc->consts;
        a.maps = maps ? maps + (size_t)b0 * 3 * npix : nullptr;
        a.resid = resid ? resid + (size_t)b0 * 2 * npix : nullptr;
        a.partial = chi2 ? sc->partial : nullptr;
        if (m->use_fft) {
            FftArgs f = m->fft;
            f.T = sc->T;
            f.U = sc->U;
            HIP_TRY(timed(2, [&] {
                hipError_t e = launch_fft_x(f, nb, s);
                return e == hipSuccess ? launch_fft_y_moments(f, a, nb, s) : e;
            }));
        } else {
            HIP_TRY(timed(2, [&] { return launch_psf_moments(a, nb, m->lds_bytes, s); }));
        }
        if (chi2)
            HIP_TRY(timed(3, [&] {
                return launch_reduce_chi2(sc->partial, m->ntiles, sc->consts, m->nvalid,
                                          chi2 + b0, nvalid ? nvalid + b0 : nullptr, nb, s);
            }));
    }
    return GK_OK;
}

constexpr size_t kMaxGraphs = 8;

// Row scratch of gk_chi2_batch_noalloc: one fixed array per GPU, loaded with
// the library's code object and held until the process ends.  Host code never
// passes the array's name to a kernel (on the host it is only a stand-in
// symbol): its device address, looked up once per device with that device
// current, is kept in scratch_addr.
constexpr int kMaxDevices = 64;
std::mutex scratch_mu;
unsigned char *scratch_addr[kMaxDevices] = {};

// Per-row scratch carved from the fixed array: for `rows` rows, the row
// constants, the T_j planes, the chi-square tile partials and (FFT path) the
// x-pass planes, each region 256-byte aligned.
struct NoAllocLayout {
    int rows = 0;
    size_t row_bytes = 0;
    size_t off_consts = 0, off_T = 0, off_partial = 0, off_U = 0;
    bool T = false, U = false;
};

size_t align256(size_t n) { return (n + 255) & ~size_t(255); }

NoAllocLayout noalloc_layout(const gk_model *m)
{
    NoAllocLayout L;
    L.T = !m->vfield;
    L.U = !m->vfield && m->use_fft;
    const size_t c = gbk::NCONST * sizeof(double);
    const size_t t = L.T ? (size_t)3 * m->EX * m->EY * sizeof(double) : 0;
    const size_t p = (size_t)m->ntiles * sizeof(double);
    const size_t u = L.U ? (size_t)3 * m->EY * m->NX * sizeof(double) : 0;
    L.row_bytes = c + t + p + u;
    const size_t cap = (size_t)GK_NOALLOC_SCRATCH_BYTES;
    // four regions lose at most 255 bytes each to alignment
    size_t rows = cap > 4 * 256 ? (cap - 4 * 256) / L.row_bytes : 0;
    rows = std::min<size_t>(rows, 65535);
    L.rows = (int)rows;
    L.off_consts = 0;
    L.off_T = align256(L.off_consts + rows * c);
    L.off_partial = align256(L.off_T + rows * t);
    L.off_U = align256(L.off_partial + rows * p);
    return L;
}

// Device address of `scratch` on `dev` (the current device).
hipError_t noalloc_scratch(int dev, unsigned char **out)
{
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(scratch_mu);
    if (!scratch_addr[dev]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        scratch_addr[dev] = static_cast<unsigned char *>(p);
    }
    *out = scratch_addr[dev];
    return hipSuccess;
}

}  // namespace

// PSF/moment-pass arguments of a model (row pointers and outputs unset); the
// observation's pointers when with_obs.
PsfArgs gbk::psf_args(const gk_model *m, bool with_obs)
{
    PsfArgs a{};
    a.kp = m->d_kp;
    a.hp = m->hp;
    a.u = m->d.upsample;
    a.nx = m->d.nx;
    a.ny = m->d.ny;
    a.EX = m->EX;
    a.EY = m->EY;
    a.TXd = m->TXd;
    a.TYd = m->TYd;
    a.ntx = m->ntx;
    a.ntiles = m->ntiles;
    a.dv = m->d.dv_kms;
    a.vref = m->vref;
    if (with_obs) {
        a.mask = m->d_mask;
        a.vo = m->d_vo;
        a.so = m->d_so;
        a.iev = m->d_iev;
        a.ies = m->d_ies;
    }
    return a;
}

// The launch chain of B device rows on s, with the model's scratch and no
// graph bookkeeping (the caller may be recording a graph of its own).
gk_status gbk::enqueue_device_rows(gk_model *m, const double *d_params, int32_t B, float *maps,
                                   double *resid, double *chi2, int64_t *nvalid, hipStream_t s)
{
    if (B <= 0) return GK_OK;
    return enqueue_batch(m, d_params, PTR_DEVICE, B, maps, resid, chi2, nvalid, s);
}


gk_status gbk::run_batch(gk_model *m, const double *params, int32_t B, float *maps,
                          double *resid, double *chi2, int64_t *nvalid, void *stream,
                          bool mapped_chi2)
{
    if (!m) return fail(GK_EINVAL, "model is NULL");
    if (B < 0) return fail(GK_EINVAL, "negative batch size %d", B);
    if (B == 0) return GK_OK;
    if (!params) return fail(GK_EINVAL, "params is NULL");
    if ((resid || chi2) && !m->has_obs) return fail(GK_ESTATE, "no observation set");
    DeviceGuard g(m->device);
    HIP_TRY(g.err);
    hipStream_t s = (hipStream_t)stream;

    for (const void *out : {(const void *)maps, (const void *)resid, (const void *)chi2,
                            (const void *)nvalid}) {
        if (out && pointer_kind(out) != PTR_DEVICE && !(mapped_chi2 && out == chi2))
            return fail(GK_EINVAL, "output arrays must be device memory");
    }
    PtrKind pk = pointer_kind(params);
    if (pk == PTR_BAD) return fail(GK_EINVAL, "params pointer of unknown kind");
    int n_bad = 0;
    if (pk == PTR_HOST)
        for (int b = 0; b < B; ++b) n_bad += !row_valid(params + (size_t)b * NPAR, m->d.rc);

    const bool graphable = m->launch_mode == GK_LAUNCH_GRAPH && pk == PTR_DEVICE &&
                           !m->prof_flags && s != nullptr;
    if (!graphable) {
        GK_TRY(enqueue_batch(m, params, pk, B, maps, resid, chi2, nvalid, s));
        return n_bad ? GK_PARTIAL : GK_OK;
    }
    // scratch first, so that recording allocates nothing
    HIP_TRY(m->reserve(std::min<int>(B, m->chunk_rows())));
    const gk_model::GraphKey key{params, maps, resid, chi2, nvalid, s, B, m->gen};
    for (auto &g : m->graphs)
        if (g.key == key) {
            HIP_TRY(hipGraphLaunch(g.exec, s));
            ++m->graph_launches;
            return GK_OK;
        }
    auto it = std::find(m->seen.begin(), m->seen.end(), key);
    if (it == m->seen.end()) {  // first sighting: run eagerly, remember the key
        if (m->seen.size() >= 2 * kMaxGraphs) m->seen.erase(m->seen.begin());
        m->seen.push_back(key);
        GK_TRY(enqueue_batch(m, params, pk, B, maps, resid, chi2, nvalid, s));
        return GK_OK;
    }
    m->seen.erase(it);
    // second sighting: record the chain, then launch the graph
    HIP_TRY(hipStreamBeginCapture(s, hipStreamCaptureModeRelaxed));
    const gk_status st = enqueue_batch(m, params, pk, B, maps, resid, chi2, nvalid, s);
    hipGraph_t graph = nullptr;
    const hipError_t ec = hipStreamEndCapture(s, &graph);
    if (st < 0 || ec != hipSuccess) {
        if (graph) (void)hipGraphDestroy(graph);
        if (st < 0) return st;
        HIP_TRY(ec);
    }
    hipGraphExec_t exec = nullptr;
    const hipError_t ei = hipGraphInstantiateWithFlags(&exec, graph, 0);
    if (ei != hipSuccess) {
        (void)hipGraphDestroy(graph);
        HIP_TRY(ei);
    }
    if (m->graphs.size() >= kMaxGraphs) {
        (void)hipGraphExecDestroy(m->graphs.front().exec);
        (void)hipGraphDestroy(m->graphs.front().graph);
        m->graphs.erase(m->graphs.begin());
    }
    m->graphs.push_back({key, graph, exec});
    HIP_TRY(hipGraphLaunch(exec, s));
    ++m->graph_launches;
    return GK_OK;
}


extern "C" {

const char *gk_last_error(void) { return g_err.c_str(); }

gk_status gk_set_launch_mode(gk_model *m, int32_t mode)
{
    if (!m) return fail(GK_EINVAL, "model is NULL");
    if (mode != GK_LAUNCH_EAGER && mode != GK_LAUNCH_GRAPH)
        return fail(GK_EINVAL, "unknown launch mode %d", mode);
    DeviceGuard g(m->device);
    HIP_TRY(g.err);
    HIP_TRY(hipDeviceSynchronize());  // recorded graphs may still run
    m->drop_graphs();
    m->launch_mode = mode;
    return GK_OK;
}

gk_status gk_graph_launches(const gk_model *m, int64_t *count)
{
    if (!m || !count) return fail(GK_EINVAL, "NULL argument");
    *count = m->graph_launches;
    return GK_OK;
}

gk_status gk_model_conv_path(const gk_model *m, int32_t *conv_mode)
{
    if (!m || !conv_mode) return fail(GK_EINVAL, "NULL argument");
    if (m->vfield) return fail(GK_EINVAL, "a velocity-field model has no convolution");
    *conv_mode = m->use_fft ? GK_CONV_FFT : GK_CONV_DIRECT;
    return GK_OK;
}

// The velocity-field strategy (Sec. 2.2.1): the data grid only, no kernel
// tables, no convolution path.
static gk_status create_vfield_model(const gk_model_desc &d, int device, gk_model **out)
{
    if (d.nx < 1 || d.ny < 1) return fail(GK_EINVAL, "grid sizes must be >= 1");
    if ((double)d.nx * d.ny >= 2.0e9) return fail(GK_EINVAL, "velocity field too large");
    if (d.upsample != 1) return fail(GK_EINVAL, "the velocity-field strategy needs upsample = 1");
    if (d.psf_fwhm_pix != 0.0 || d.lsf_sigma_kms != 0.0)
        return fail(GK_EINVAL, "the velocity-field strategy has no PSF or LSF (both must be 0)");
    if (d.rc < GK_RC_ARCTAN || d.rc > GK_RC_BOISSIER) return fail(GK_EINVAL, "unknown rotation curve");
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev)
        return fail(GK_EINVAL, "no HIP device %d", device);
    gk_model *m = new (std::nothrow) gk_model();
    if (!m) return fail(GK_ENOMEM, "host allocation failed");
    m->d = d;
    m->device = device;
    m->vfield = true;
    m->NX = m->EX = d.nx;
    m->NY = m->EY = d.ny;
    m->NZ = m->NZE = 1;
    m->ntiles = (int)(((int64_t)d.nx * d.ny + kVfTile - 1) / kVfTile);
    *out = m;
    return GK_OK;
}

gk_status gk_create_model(const gk_model_desc *desc, int device, gk_model **out)
{
    if (!desc || !out) return fail(GK_EINVAL, "desc and out must not be NULL");
    *out = nullptr;
    const gk_model_desc &d = *desc;
    if (d.strategy == GK_STRATEGY_VFIELD) return create_vfield_model(d, device, out);
    if (d.strategy != GK_STRATEGY_CUBE) return fail(GK_EINVAL, "unknown strategy %d", d.strategy);
    if (d.nx < 1 || d.ny < 1 || d.nz < 1) return fail(GK_EINVAL, "grid sizes must be >= 1");
    if (d.upsample < 1 || d.upsample > 8) return fail(GK_EINVAL, "upsample must be in 1..8");
    if (!(d.dv_kms > 0.0) || !std::isfinite(d.dv_kms)) return fail(GK_EINVAL, "dv must be > 0");
    if (!std::isfinite(d.v0_kms) || !std::isfinite(d.crpix))
        return fail(GK_EINVAL, "v0 and crpix must be finite");
    if (!(d.psf_fwhm_pix >= 0.0) || !std::isfinite(d.psf_fwhm_pix) || !(d.lsf_sigma_kms >= 0.0) ||
        !std::isfinite(d.lsf_sigma_kms))
        return fail(GK_EINVAL, "PSF FWHM and LSF sigma must be finite and >= 0");
    if (!(d.kernel_radius_sigma > 0.0) || d.kernel_radius_sigma > 16.0)
        return fail(GK_EINVAL, "kernel radius must be in (0, 16]");
    if (d.rc < GK_RC_ARCTAN || d.rc > GK_RC_BOISSIER) return fail(GK_EINVAL, "unknown rotation curve");
    if (d.conv_mode < GK_CONV_AUTO || d.conv_mode > GK_CONV_FFT)
        return fail(GK_EINVAL, "unknown convolution mode %d", d.conv_mode);
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev)
        return fail(GK_EINVAL, "no HIP device %d", device);

    gk_model *m = new (std::nothrow) gk_model();
    if (!m) return fail(GK_ENOMEM, "host allocation failed");
    m->d = d;
    m->device = device;
    const int u = d.upsample;
    const double sp = d.psf_fwhm_pix > 0 ? u * fwhm_to_sigma(d.psf_fwhm_pix) : 0.0;
    const double sl = d.lsf_sigma_kms > 0 ? u * d.lsf_sigma_kms / d.dv_kms : 0.0;
    std::vector<double> kp = gaussian_taps(sp, d.kernel_radius_sigma);
    std::vector<double> kl = gaussian_taps(sl, d.kernel_radius_sigma);
    m->hp = (int)(kp.size() / 2);
    m->hl = (int)(kl.size() / 2);
    m->NX = u * d.nx;
    m->NY = u * d.ny;
    m->NZ = u * d.nz;
    m->EX = m->NX + 2 * m->hp;
    m->EY = m->NY + 2 * m->hp;
    m->NZE = m->NZ + 2 * m->hl;
    // the kernels address a T plane (FP64 per fine spaxel with halo) with
    // 32-bit byte offsets
    if ((double)m->EX * m->EY * sizeof(double) >= 2147483648.0) {
        delete m;
        return fail(GK_EINVAL, "model grid too large (%d x %d fine spaxels with halo)", m->EX, m->EY);
    }
    // the line-sum kernel packs a wave's channel range into two 16-bit fields
    // holding values up to NZE + 1
    if (m->NZE > kMaxFineChannels) {
        const int nze = m->NZE;
        delete m;
        return fail(GK_EINVAL, "%d fine channels with the LSF halo (nz u + 2 h_lsf); at most %d",
                    nze, kMaxFineChannels);
    }
    m->dvf = d.dv_kms / u;
    m->inv_dvf = u / d.dv_kms;
    m->vf0 = d.v0_kms + ((0 - m->hl + 0.5) / u - 0.5 - d.crpix) * d.dv_kms;
    // reference velocity of the moment sums: the centre of the data band
    m->vref = d.v0_kms + (0.5 * (d.nz - 1) - d.crpix) * d.dv_kms;

    // W_j(z') = (1/u) sum_{m in [0, NZ)} vrel(m/u)^j K_z[m + 2 hl - z']
    std::vector<double> wz((size_t)4 * m->NZE, 0.0);  // [NZE][4] = {W0, W1, W2, 0}
    for (int zp = 0; zp < m->NZE; ++zp) {
        double w0 = 0, w1 = 0, w2 = 0;
        for (int t = 0; t <= 2 * m->hl; ++t) {
            int mm = zp + t - 2 * m->hl;  // fine window channel reached by tap t
            if (mm < 0 || mm >= m->NZ) continue;
            double vr = (mm / u - 0.5 * (d.nz - 1)) * d.dv_kms;
            double k = kl[t];
            w0 += k;
            w1 += k * vr;
            w2 += k * vr * vr;
        }
        wz[4 * (size_t)zp + 0] = w0 / u;
        wz[4 * (size_t)zp + 1] = w1 / u;
        wz[4 * (size_t)zp + 2] = w2 / u;
    }
    {
        double wmax = 0.0;
        for (int zp = 0; zp < m->NZE; ++zp) wmax = std::max(wmax, wz[4 * (size_t)zp]);
        int lo = m->NZE - 1, hi = 0;
        for (int zp = 0; zp < m->NZE; ++zp)
            if (wz[4 * (size_t)zp] >= std::ldexp(wmax, -5)) {
                lo = std::min(lo, zp);
                hi = std::max(hi, zp);
            }
        m->zedge_lo = (float)lo;
        m->zedge_hi = (float)hi;
    }
    choose_tile(m);
    const bool direct_ok = m->lds_bytes <= kMaxLds;
    std::vector<double2> twx, twy;
    std::vector<double> kbx, kby;
    m->fft_ok = setup_fft(m, kp, twx, twy, kbx, kby);
    if (d.conv_mode == GK_CONV_DIRECT && !direct_ok) {
        delete m;
        return fail(GK_EINVAL, "PSF too wide for the direct convolution path");
    }
    if (d.conv_mode == GK_CONV_FFT && !m->fft_ok) {
        delete m;
        return fail(GK_EINVAL, "model grid too large for the FFT convolution path");
    }
    if (!direct_ok && !m->fft_ok) {
        delete m;
        return fail(GK_EINVAL, "model grid too large for both convolution paths");
    }
    m->use_fft = d.conv_mode == GK_CONV_FFT ||
                 (d.conv_mode == GK_CONV_AUTO && m->fft_ok && (!direct_ok || m->hp > kMaxFastHalo));
    if (m->use_fft) m->ntiles = m->fft.ncb;  // chi-square partials per row

    DeviceGuard g(device);
    hipError_t e = g.err;
    if (e == hipSuccess) e = dev_alloc(&m->d_kp, kp.size());
    if (e == hipSuccess) e = dev_alloc(&m->d_wz, wz.size());
    if (e == hipSuccess)
        e = hipMemcpy(m->d_kp, kp.data(), kp.size() * sizeof(double), hipMemcpyHostToDevice);
    if (e == hipSuccess)
        e = hipMemcpy(m->d_wz, wz.data(), wz.size() * sizeof(double), hipMemcpyHostToDevice);
    if (m->fft_ok) {
        auto up = [&](auto **dst, const auto &v) {
            if (e == hipSuccess) e = dev_alloc(dst, v.size());
            if (e == hipSuccess)
                e = hipMemcpy(*dst, v.data(), v.size() * sizeof(v[0]), hipMemcpyHostToDevice);
        };
        up(&m->d_twx, twx);
        up(&m->d_twy, twy);
        up(&m->d_kbx, kbx);
        up(&m->d_kby, kby);
        m->fft.twx = m->d_twx;
        m->fft.twy = m->d_twy;
        m->fft.kbx = m->d_kbx;
        m->fft.kby = m->d_kby;
    }
    if (e != hipSuccess) {
        m->release();
        delete m;
        return fail(e == hipErrorOutOfMemory ? GK_ENOMEM : GK_EDEVICE, "create_model: %s",
                    hipGetErrorString(e));
    }
    *out = m;
    return GK_OK;
}

gk_status gk_destroy_model(gk_model *m)
{
    if (!m) return GK_OK;
    {
        DeviceGuard g(m->device);
        (void)hipDeviceSynchronize();
        m->release();
    }
    delete m;
    return GK_OK;
}

gk_status gk_set_profiling(gk_model *m, int flags)
{
    if (!m) return fail(GK_EINVAL, "model is NULL");
    if (flags & ~(GK_PROF_TIMING | GK_PROF_COUNT)) return fail(GK_EINVAL, "unknown profiling flag");
    DeviceGuard g(m->device);
    HIP_TRY(g.err);
    if ((flags & GK_PROF_COUNT) && !m->d_count && !m->vfield) {
        // one counter per (row, wave) of the largest chunk
        const size_t n = m->count_slots();
        HIP_TRY(hipMalloc((void **)&m->d_count, n * sizeof(unsigned long long)));
        HIP_TRY(hipMemset(m->d_count, 0, n * sizeof(unsigned long long)));
    }
    m->prof_flags = flags;
    return GK_OK;
}

gk_status gk_read_profile(gk_model *m, gk_profile_stats *out)
{
    if (!m || !out) return fail(GK_EINVAL, "NULL argument");
    DeviceGuard g(m->device);
    HIP_TRY(g.err);
    std::memset(out, 0, sizeof *out);
    hipError_t err = hipSuccess;
    for (auto &call : m->prof_events)
        for (auto &k : call) {
            float ms = 0.0f;
            hipError_t e = hipEventSynchronize(k.second.second);
            if (e == hipSuccess) e = hipEventElapsedTime(&ms, k.second.first, k.second.second);
            if (e == hipSuccess) {
                out->kernel_ms[k.first] += ms;
                out->launches[k.first] += 1;
            } else if (err == hipSuccess) {
                err = e;
            }
            (void)hipEventDestroy(k.second.first);
            (void)hipEventDestroy(k.second.second);
        }
    m->prof_events.clear();
    if (m->d_count) {
        const size_t n = m->count_slots();
        std::vector<unsigned long long> c(n);
        HIP_TRY(hipDeviceSynchronize());
        HIP_TRY(hipMemcpy(c.data(), m->d_count, n * sizeof(unsigned long long),
                          hipMemcpyDeviceToHost));
        HIP_TRY(hipMemset(m->d_count, 0, n * sizeof(unsigned long long)));
        unsigned long long tot = 0;
        for (unsigned long long v : c) tot += v;
        out->support_voxels = (int64_t)tot;
    }
    out->rows = m->prof_rows;
    m->prof_rows = 0;
    HIP_TRY(err);
    return GK_OK;
}

gk_status gk_model_dims(const gk_model *m, int32_t dims[5])
{
    if (!m || !dims) return fail(GK_EINVAL, "NULL argument");
    dims[0] = m->EX;
    dims[1] = m->EY;
    dims[2] = m->NZE;
    dims[3] = m->hp;
    dims[4] = m->hl;
    return GK_OK;
}

gk_status gk_set_observation(gk_model *m, const float *vel, const float *sig, const float *evel,
                             const float *esig, const uint8_t *mask, double W)
{
    if (!m || !vel || !evel || !mask) return fail(GK_EINVAL, "NULL observation array");
    if (!(W >= 0.0) || !std::isfinite(W)) return fail(GK_EINVAL, "W must be finite and >= 0");
    if (W > 0.0 && (!sig || !esig)) return fail(GK_EINVAL, "dispersion maps needed when W > 0");
    const size_t n = (size_t)m->d.nx * m->d.ny;
    std::vector<float> vo(n), so(n, 0.0f);
    std::vector<double> iev(n, 0.0), ies(n, 0.0);
    std::vector<uint8_t> mk(n);
    int64_t nv = 0;
    const double sw = std::sqrt(W);
    for (size_t i = 0; i < n; ++i) {
        mk[i] = mask[i] ? 1 : 0;
        vo[i] = vel[i];
        if (sig) so[i] = sig[i];
        if (!mk[i]) continue;
        if (!std::isfinite(vel[i]) || !std::isfinite(evel[i]) || !(evel[i] > 0.0f))
            return fail(GK_EINVAL, "pixel %zu: velocity or its error invalid", i);
        iev[i] = 1.0 / (double)evel[i];
        if (W > 0.0) {
            if (!std::isfinite(sig[i]) || !std::isfinite(esig[i]) || !(esig[i] > 0.0f))
                return fail(GK_EINVAL, "pixel %zu: dispersion or its error invalid", i);
            ies[i] = sw / (double)esig[i];
        }
        ++nv;
    }
    DeviceGuard g(m->device);
    HIP_TRY(g.err);
    if (!m->d_vo) {
        HIP_TRY(dev_alloc(&m->d_vo, n));
        HIP_TRY(dev_alloc(&m->d_so, n));
        HIP_TRY(dev_alloc(&m->d_iev, n));
        HIP_TRY(dev_alloc(&m->d_ies, n));
        HIP_TRY(dev_alloc(&m->d_mask, n));
    }
    HIP_TRY(hipDeviceSynchronize());  // no pending kernel may still read the old observation
    HIP_TRY(hipMemcpy(m->d_vo, vo.data(), n * sizeof(float), hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(m->d_so, so.data(), n * sizeof(float), hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(m->d_iev, iev.data(), n * sizeof(double), hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(m->d_ies, ies.data(), n * sizeof(double), hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(m->d_mask, mk.data(), n, hipMemcpyHostToDevice));
    m->nvalid = nv;
    m->obs_sig = W > 0.0;
    m->obs_W = W;
    m->has_obs = true;
    m->drop_graphs();  // recorded chains hold the observation's pointers and count
    return GK_OK;
}

gk_status gk_observation_count(const gk_model *m, int64_t *n_valid)
{
    if (!m || !n_valid) return fail(GK_EINVAL, "NULL argument");
    if (!m->has_obs) return fail(GK_ESTATE, "no observation set");
    *n_valid = m->nvalid;
    return GK_OK;
}

gk_status gk_evaluate_batch(gk_model *m, const double *params, int32_t B, float *maps,
                            void *stream)
{
    if (!maps && B > 0) return fail(GK_EINVAL, "maps is NULL");
    return run_batch(m, params, B, maps, nullptr, nullptr, nullptr, stream);
}

gk_status gk_chi2_batch(gk_model *m, const double *params, int32_t B, double *chi2,
                        int64_t *n_valid, void *stream)
{
    if (!chi2 && B > 0) return fail(GK_EINVAL, "chi2 is NULL");
    return run_batch(m, params, B, nullptr, nullptr, chi2, n_valid, stream);
}

gk_status gk_residual_batch(gk_model *m, const double *params, int32_t B, double *resid,
                            void *stream)
{
    if (!resid && B > 0) return fail(GK_EINVAL, "resid is NULL");
    return run_batch(m, params, B, nullptr, resid, nullptr, nullptr, stream);
}

gk_status gk_chi2_batch_noalloc(gk_model *m, const double *params, int32_t B, double *chi2,
                                int64_t *n_valid, void *stream)
{
    if (!m) return fail(GK_EINVAL, "model is NULL");
    if (B < 0) return fail(GK_EINVAL, "negative batch size %d", B);
    if (B == 0) return GK_OK;
    if (!params || !chi2) return fail(GK_EINVAL, "params or chi2 is NULL");
    DeviceGuard g(m->device);
    HIP_TRY(g.err);
    if (pointer_kind(params) != PTR_DEVICE) return fail(GK_EINVAL, "rows must be device memory");
    if (pointer_kind(chi2) != PTR_DEVICE || (n_valid && pointer_kind(n_valid) != PTR_DEVICE))
        return fail(GK_EINVAL, "output arrays must be device memory");
    const NoAllocLayout lay = noalloc_layout(m);
    if (lay.rows < 1)
        return fail(GK_EINVAL,
                    "one row of this model needs %zu bytes of scratch; the allocation-free "
                    "array holds %zu",
                    lay.row_bytes, (size_t)GK_NOALLOC_SCRATCH_BYTES);
    if (!m->has_obs) return fail(GK_ESTATE, "no observation set");
    unsigned char *base = nullptr;
    HIP_TRY(noalloc_scratch(m->device, &base));
    RowScratch sc;
    sc.chunk = std::min(lay.rows, (int)B);
    sc.consts = reinterpret_cast<double *>(base + lay.off_consts);
    sc.T = lay.T ? reinterpret_cast<double *>(base + lay.off_T) : nullptr;
    sc.partial = reinterpret_cast<double *>(base + lay.off_partial);
    sc.U = lay.U ? reinterpret_cast<double *>(base + lay.off_U) : nullptr;
    return enqueue_batch(m, params, PTR_DEVICE, B, nullptr, nullptr, chi2, n_valid,
                         (hipStream_t)stream, &sc);
}

}  // extern "C"

bool gbk::set_conv_config(gk_model *m, bool fft, int tx, int ty)
{
    if (fft) {
        if (!m->fft_ok) return false;
        m->use_fft = true;
        m->ntiles = m->fft.ncb;
    } else {
        const int u = m->d.upsample;
        const bool fast = u == 1 && ty == 32 && (tx == 32 || tx == 64) && m->hp <= kMaxFastHalo;
        size_t lds;
        if (fast) {
            if (m->d.nx < tx / 2 || m->d.ny < 16) return false;
            if (tx == 32 && !fast_plane_ok(m)) return false;
            lds = psf_u1_lds_bytes(tx, m->hp);
        } else {
            if (tx < 1 || ty < 1 || tx * ty > 256 * kMaxPixPerThread) return false;
            if (u == 1 && ty == 32 && (tx == 32 || tx == 64)) return false;  // the fast kernel's shapes
            lds = psf_lds_bytes(tx, ty, u, m->hp);
        }
        if (lds > kMaxLds) return false;
        m->use_fft = false;
        m->TXd = tx;
        m->TYd = ty;
        m->ntx = (m->d.nx + tx - 1) / tx;
        m->nty = (m->d.ny + ty - 1) / ty;
        m->ntiles = m->ntx * m->nty;
        m->lds_bytes = lds;
    }
    m->drop_scratch();
    return true;
}

void gbk::survey_tile(const gk_model *m, SurveyTile *t)
{
    t->TXd = m->TXd;
    t->TYd = m->TYd;
    t->ntx = m->ntx;
    t->nty = m->nty;
    t->ntiles = m->ntiles;
    t->lds_bytes = m->lds_bytes;
    if (m->use_fft || m->TXd * m->TYd <= 256 * kMaxPixPerThread) return;
    // the 64 x 32 register-blocked tile: the survey kernels take 32 x 32
    // register-blocked tiles or generic tiles of at most 1024 pixels
    if (fast_plane_ok(m) && psf_u1_lds_bytes(32, m->hp) <= kMaxLds) {
        t->TXd = t->TYd = 32;
        t->lds_bytes = psf_u1_lds_bytes(32, m->hp);
    } else {
        int tx = 32, ty = 16;
        while (psf_lds_bytes(tx, ty, m->d.upsample, m->hp) > kMaxLds && (tx > 1 || ty > 1)) {
            if (tx >= ty && tx > 1) tx /= 2;
            else ty /= 2;
        }
        t->TXd = tx;
        t->TYd = ty;
        t->lds_bytes = psf_lds_bytes(tx, ty, m->d.upsample, m->hp);
    }
    t->ntx = (m->d.nx + t->TXd - 1) / t->TXd;
    t->nty = (m->d.ny + t->TYd - 1) / t->TYd;
    t->ntiles = t->ntx * t->nty;
}
