// gbk_survey.hip -- ragged batches over many models (galaxies of uneven cube
// sizes) in one launch chain, and Levenberg-Marquardt over a whole survey.
//
// A batch is a list of (model, parameter row).  The host builds per-row
// arrays -- model index, offsets of the row's T planes, residuals and chi2
// partials, prefix sums of the line-sum tiles -- and groups the rows by PSF
// kernel variant (register-blocked kernel per PSF half-width, generic kernel
// otherwise).  Kernels find their (row, tile) by binary search over the tile
// prefix sums, so one launch covers every row of a chunk whatever its shape.
#include <hip/hip_runtime.h>

#include <cfloat>
#include <cmath>
#include <cstring>
#include <map>
#include <new>
#include <vector>

#include "gbk_model.h"

using namespace gbk;

// Growable device or pinned-host array.
template <class T, bool PINNED> struct Buf {
    T *p = nullptr;
    size_t cap = 0;
    gk_status need(size_t n)
    {
        if (n <= cap) return GK_OK;
        const size_t c = std::max(n, cap + cap / 2);
        if (p) HIP_TRY(hipDeviceSynchronize());  // queued kernels may still use the old array
        free();
        if (PINNED) HIP_TRY(hipHostMalloc((void **)&p, c * sizeof(T), 0));
        else HIP_TRY(hipMalloc((void **)&p, c * sizeof(T)));
        cap = c;
        return GK_OK;
    }
    void free()
    {
        if (p) (void)(PINNED ? hipHostFree(p) : hipFree(p));
        p = nullptr;
        cap = 0;
    }
};
template <class T> using DBuf = Buf<T, false>;
template <class T> using HBuf = Buf<T, true>;

struct gk_survey {
    std::vector<gk_model *> models;
    int device = 0;
    hipStream_t fit_stream = nullptr;
    hipEvent_t ev_staged = nullptr;  // the last copy out of the pinned staging buffers
    DBuf<ModelDev> md;
    std::vector<ModelDev> h_md;
    // evaluation scratch
    DBuf<double> params, consts, T, partial;
    DBuf<char> idx;
    HBuf<char> h_idx;
    HBuf<double> h_params;
    // LM workspace
    DBuf<double> resid, norm, scale, npart;
    // nested-grid workspace
    DBuf<double> grid_rows, grid_chi2, grid_spec, grid_val;
    DBuf<int64_t> grid_idx;
    DBuf<int64_t> goff;
    HBuf<double> h_norm, h_scale;
    HBuf<int64_t> h_goff;

    void release()
    {
        if (ev_staged) (void)hipEventSynchronize(ev_staged);
        if (fit_stream) (void)hipStreamSynchronize(fit_stream);
        md.free(); params.free(); consts.free(); T.free(); partial.free(); idx.free();
        h_idx.free(); h_params.free(); resid.free(); norm.free(); scale.free(); goff.free();
        npart.free();
        grid_rows.free(); grid_chi2.free(); grid_spec.free(); grid_val.free(); grid_idx.free();
        h_norm.free(); h_scale.free(); h_goff.free();
        if (ev_staged) (void)hipEventDestroy(ev_staged);
        if (fit_stream) (void)hipStreamDestroy(fit_stream);
    }
};

namespace {

// Refreshes the device copies of the model descriptors (observations may change).
gk_status refresh_models(gk_survey *s, hipStream_t st)
{
    const int n = (int)s->models.size();
    s->h_md.resize(n);
    for (int i = 0; i < n; ++i) {
        gk_model *m = s->models[i];
        ModelDev &d = s->h_md[i];
        std::memset(&d, 0, sizeof d);
        PsfArgs &a = d.psf;
        a.kp = m->d_kp;
        a.hp = m->hp;
        a.u = m->d.upsample;
        a.nx = m->d.nx;
        a.ny = m->d.ny;
        a.EX = m->EX;
        a.EY = m->EY;
        SurveyTile tile;
        survey_tile(m, &tile);
        a.TXd = tile.TXd;
        a.TYd = tile.TYd;
        a.ntx = tile.ntx;
        a.ntiles = tile.ntiles;
        a.dv = m->d.dv_kms;
        a.vref = m->vref;
        if (m->has_obs) {
            a.mask = m->d_mask;
            a.vo = m->d_vo;
            a.so = m->d_so;
            a.iev = m->d_iev;
            a.ies = m->d_ies;
        }
        d.wz = m->d_wz;
        d.NZE = m->NZE;
        d.EX = m->EX;
        d.EY = m->EY;
        d.hp = m->hp;
        d.u = m->d.upsample;
        d.rc = m->d.rc;
        d.dvf = m->dvf;
        d.inv_dvf = m->inv_dvf;
        d.vf0 = m->vf0;
        d.zedge_lo = m->zedge_lo;
        d.zedge_hi = m->zedge_hi;
        d.nvalid = m->nvalid;
        d.fast_hp = (m->d.upsample == 1 && tile.TXd == 32 && tile.TYd == 32 &&
                     m->hp <= kMaxFastHalo) ? m->hp : -1;
        d.lds_bytes = (int)tile.lds_bytes;
        d.vfield = m->vfield ? 1 : 0;
        d.use_sig = m->obs_sig ? 1 : 0;
        if (m->vfield) {  // constants at u = 1 without halo (Sec. 2.2.1)
            d.hp = 0;
            d.u = 1;
            d.dvf = 1.0;
            d.fast_hp = -1;
        }
    }
    GK_TRY(s->md.need(n));
    HIP_TRY(hipMemcpyAsync(s->md.p, s->h_md.data(), sizeof(ModelDev) * n, hipMemcpyHostToDevice, st));
    HIP_TRY(hipStreamSynchronize(st));
    return GK_OK;
}

// Velocity-field surveys (every model of the survey uses that strategy): per
// row the constants, then one workgroup per (row, pixel tile), then the
// fixed-order sum of the tile partials.  No T planes, so chunks are bounded
// only by the 65,535 rows of a launch.
gk_status survey_batch_vfield(gk_survey *s, const int32_t *midx, const double *d_params, int B,
                              double *chi2, double *resid, const int64_t *resid_off, hipStream_t st)
{
    for (int b0 = 0; b0 < B; b0 += 65535) {
        const int nb = std::min(B - b0, 65535);
        std::vector<int> rmodel(nb), lsb(nb + 1);
        std::vector<int64_t> poff(nb), roff(nb);
        int64_t pt = 0;
        lsb[0] = 0;
        int rc = s->h_md[midx[b0]].rc;
        for (int i = 0; i < nb; ++i) {
            const ModelDev &m = s->h_md[midx[b0 + i]];
            rmodel[i] = midx[b0 + i];
            if (m.rc != rc) rc = -1;
            if ((int64_t)lsb[i] + m.psf.ntiles > INT32_MAX) return fail(GK_EINVAL, "batch too large");
            lsb[i + 1] = lsb[i] + m.psf.ntiles;
            poff[i] = pt;
            pt += m.psf.ntiles;
            roff[i] = resid_off ? resid_off[b0 + i] : 0;
        }
        // staging: ints [rmodel | lsb], then int64 [poff | roff]
        const size_t bytes = (size_t)(2 * nb + 1) * sizeof(int) + 8 + (size_t)2 * nb * sizeof(int64_t);
        HIP_TRY(hipEventSynchronize(s->ev_staged));
        GK_TRY(s->h_idx.need(bytes));
        GK_TRY(s->idx.need(bytes));
        char *h = s->h_idx.p;
        size_t o = 0;
        auto put = [&](const void *src, size_t n) { std::memcpy(h + o, src, n); o += n; };
        const size_t o_rm = o; put(rmodel.data(), nb * sizeof(int));
        const size_t o_ls = o; put(lsb.data(), (nb + 1) * sizeof(int));
        o = (o + 7) & ~(size_t)7;
        const size_t o_po = o; put(poff.data(), nb * sizeof(int64_t));
        const size_t o_ro = o; put(roff.data(), nb * sizeof(int64_t));
        GK_TRY(s->consts.need((size_t)nb * NCONST));
        GK_TRY(s->partial.need((size_t)pt));
        HIP_TRY(hipMemcpyAsync(s->idx.p, h, o, hipMemcpyHostToDevice, st));
        HIP_TRY(hipEventRecord(s->ev_staged, st));
        const char *d = s->idx.p;
        RowMap rm{};
        rm.row_model = (const int *)(d + o_rm);
        rm.ls_base = (const int *)(d + o_ls);
        rm.part_off = (const int64_t *)(d + o_po);
        rm.resid_off = resid ? (const int64_t *)(d + o_ro) : nullptr;
        rm.B = nb;
        const double *prow = d_params + (size_t)b0 * NPAR;
        HIP_TRY(launch_prep_multi(prow, nb, rm.row_model, s->md.p, s->consts.p, st));
        HIP_TRY(launch_vfield_multi(s->md.p, rm, lsb[nb], rc, prow, s->consts.p, resid,
                                    chi2 ? s->partial.p : nullptr, st));
        if (chi2)
            HIP_TRY(launch_reduce_multi(s->partial.p, s->md.p, rm, s->consts.p, chi2 + b0, nb, st));
    }
    return GK_OK;
}

// Evaluates rows [0, B) (device params) of models midx[] into chi2 and/or
// ragged residuals (resid_off per row, host array, NULL = no residuals).
gk_status survey_batch(gk_survey *s, const int32_t *midx, const double *d_params, int B,
                       double *chi2, double *resid, const int64_t *resid_off, hipStream_t st)
{
    const int nm = (int)s->models.size();
    for (int b = 0; b < B; ++b)
        if (midx[b] < 0 || midx[b] >= nm) return fail(GK_EINVAL, "row %d: model index %d", b, midx[b]);
    if (s->models[0]->vfield) return survey_batch_vfield(s, midx, d_params, B, chi2, resid, resid_off, st);
    // chunk so that the T planes fit the scratch budget
    int b0 = 0;
    while (b0 < B) {
        size_t tsum = 0;
        int b1 = b0;
        while (b1 < B && b1 - b0 < 65535) {
            const ModelDev &m = s->h_md[midx[b1]];
            const size_t t = (size_t)3 * m.EX * m.EY;
            if (b1 > b0 && (tsum + t) * sizeof(double) > kScratchBudget) break;
            tsum += t;
            ++b1;
        }
        const int nb = b1 - b0;
        // per-row arrays: model, T offset, line-sum tile base, partial offset, resid offset
        std::vector<int> rmodel(nb), lsb(nb + 1);
        std::vector<int64_t> toff(nb), poff(nb), roff(nb);
        int64_t t = 0, pt = 0;
        lsb[0] = 0;
        std::map<int, std::vector<int>> buckets;
        for (int i = 0; i < nb; ++i) {
            const ModelDev &m = s->h_md[midx[b0 + i]];
            rmodel[i] = midx[b0 + i];
            toff[i] = t;
            t += (int64_t)3 * m.EX * m.EY;
            lsb[i + 1] = lsb[i] + ((m.EX + 15) / 16) * ((m.EY + 15) / 16);
            poff[i] = pt;
            pt += m.psf.ntiles;
            roff[i] = resid_off ? resid_off[b0 + i] : 0;
            buckets[m.fast_hp].push_back(i);
        }
        // bucket arrays: rows and tile prefix sums, concatenated
        std::vector<int> brows, bbase;
        struct Bk { int fast_hp, row0, base0, n, nblocks; size_t lds; };
        std::vector<Bk> bks;
        for (auto &kv : buckets) {
            Bk k{kv.first, (int)brows.size(), (int)bbase.size(), (int)kv.second.size(), 0, 0};
            int acc = 0;
            for (int i : kv.second) {
                brows.push_back(i);
                bbase.push_back(acc);
                const ModelDev &m = s->h_md[rmodel[i]];
                acc += m.psf.ntiles;
                k.lds = std::max(k.lds, (size_t)m.lds_bytes);
            }
            bbase.push_back(acc);
            k.nblocks = acc;
            bks.push_back(k);
        }
        // staging: ints [rmodel | lsb | brows | bbase], then int64 [toff | poff | roff]
        const size_t n_int = (size_t)nb + (nb + 1) + brows.size() + bbase.size();
        const size_t bytes = n_int * sizeof(int) + 8 + (size_t)3 * nb * sizeof(int64_t);
        HIP_TRY(hipEventSynchronize(s->ev_staged));
        GK_TRY(s->h_idx.need(bytes));
        GK_TRY(s->idx.need(bytes));
        char *h = s->h_idx.p;
        size_t o = 0;
        auto put = [&](const void *src, size_t n) { std::memcpy(h + o, src, n); o += n; };
        const size_t o_rm = o; put(rmodel.data(), nb * sizeof(int));
        const size_t o_ls = o; put(lsb.data(), (nb + 1) * sizeof(int));
        const size_t o_br = o; put(brows.data(), brows.size() * sizeof(int));
        const size_t o_bb = o; put(bbase.data(), bbase.size() * sizeof(int));
        o = (o + 7) & ~(size_t)7;
        const size_t o_to = o; put(toff.data(), nb * sizeof(int64_t));
        const size_t o_po = o; put(poff.data(), nb * sizeof(int64_t));
        const size_t o_ro = o; put(roff.data(), nb * sizeof(int64_t));
        // scratch (grown before the copy: growing frees, which waits for the device)
        GK_TRY(s->consts.need((size_t)nb * NCONST));
        GK_TRY(s->T.need((size_t)t));
        GK_TRY(s->partial.need((size_t)pt));
        HIP_TRY(hipMemcpyAsync(s->idx.p, h, o, hipMemcpyHostToDevice, st));
        HIP_TRY(hipEventRecord(s->ev_staged, st));
        const char *d = s->idx.p;
        RowMap rm;
        rm.row_model = (const int *)(d + o_rm);
        rm.ls_base = (const int *)(d + o_ls);
        rm.T_off = (const int64_t *)(d + o_to);
        rm.part_off = (const int64_t *)(d + o_po);
        rm.resid_off = resid ? (const int64_t *)(d + o_ro) : nullptr;
        rm.B = nb;
        const double *prow = d_params + (size_t)b0 * NPAR;
        HIP_TRY(launch_prep_multi(prow, nb, rm.row_model, s->md.p, s->consts.p, st));
        HIP_TRY(launch_line_sums_multi(s->consts.p, s->md.p, rm, lsb[nb], s->T.p, st));
        for (const Bk &k : bks) {
            BucketMap bm;
            bm.rows = (const int *)(d + o_br) + k.row0;
            bm.tile_base = (const int *)(d + o_bb) + k.base0;
            bm.n = k.n;
            HIP_TRY(launch_psf_multi(k.fast_hp, s->md.p, rm, bm, k.nblocks, s->T.p, s->consts.p,
                                     resid, chi2 ? s->partial.p : nullptr, k.lds, st));
        }
        if (chi2)
            HIP_TRY(launch_reduce_multi(s->partial.p, s->md.p, rm, s->consts.p, chi2 + b0, nb, st));
        b0 = b1;
    }
    return GK_OK;
}

// Shape shared by the grids of a survey level: free slots, nodes per slot
// (mixed radix, first free slot most significant) and nodes per galaxy.
struct GridShape {
    int d;
    int n[NPAR];
    int slot[NPAR];
    int64_t nodes;
};

// Rows [first, first + count) of a level: row F = j nodes + L is node L of
// the level's j-th galaxy, whose box is spec[j] = {lo_a [NPAR], step_a [NPAR],
// fixed [NPAR]} (lo and step per free slot a).
__global__ void k_grid_rows_multi(GridShape g, const double *__restrict__ spec, int64_t first,
                                  int count, double *__restrict__ rows)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= count) return;
    const int64_t F = first + i;
    const int64_t j = F / g.nodes;
    int64_t L = F - j * g.nodes;
    const double *sp = spec + (size_t)j * 3 * NPAR;
    double *r = rows + (size_t)i * NPAR;
    for (int k = 0; k < NPAR; ++k) r[k] = sp[2 * NPAR + k];
    for (int a = g.d - 1; a >= 0; --a) {
        const int digit = (int)(L % g.n[a]);
        L /= g.n[a];
        r[g.slot[a]] = sp[a] + digit * sp[NPAR + a];
    }
}

// One block per galaxy j0 + blockIdx.x whose nodes meet the rows
// [first, first + count): the least chi2 of those rows (NaN as +inf; lowest
// node index on ties) merged into best_val/best_idx[j].  The chunks of a level
// run in index order, so keeping the stored node on ties keeps the lowest.
__global__ __launch_bounds__(256) void k_argmin_seg(const double *__restrict__ chi2, int64_t first,
                                                    int count, int64_t nodes, int j0,
                                                    double *__restrict__ best_val,
                                                    int64_t *__restrict__ best_idx)
{
    const int j = j0 + blockIdx.x;
    const int64_t a = std::max<int64_t>(first, (int64_t)j * nodes);
    const int64_t b = std::min<int64_t>(first + count, (int64_t)(j + 1) * nodes);
    double best = INFINITY;
    int64_t bi = INT64_MAX;
    for (int64_t F = a + threadIdx.x; F < b; F += 256) {
        const double c = chi2[F - first];
        const double v = c == c ? c : INFINITY;
        if (v < best) {
            best = v;
            bi = F - (int64_t)j * nodes;
        }
    }
    __shared__ double sv[256];
    __shared__ int64_t si[256];
    sv[threadIdx.x] = best;
    si[threadIdx.x] = bi;
    __syncthreads();
    for (int st = 128; st > 0; st >>= 1) {
        if (threadIdx.x < st) {
            const double x = sv[threadIdx.x], y = sv[threadIdx.x + st];
            const int64_t ix = si[threadIdx.x], iy = si[threadIdx.x + st];
            if (y < x || (y == x && iy < ix)) {
                sv[threadIdx.x] = y;
                si[threadIdx.x] = iy;
            }
        }
        __syncthreads();
    }
    if (threadIdx.x == 0 && (sv[0] < best_val[j] || (sv[0] == best_val[j] && si[0] < best_idx[j]))) {
        best_val[j] = sv[0];
        best_idx[j] = si[0];
    }
}

__global__ void k_grid_best_init(int n, double *__restrict__ v, int64_t *__restrict__ idx)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    v[i] = INFINITY;
    idx[i] = INT64_MAX;
}

// Index of the normal-equation pairs (a <= b) in output order.
struct NormIdx {
    int nf, npairs, nblk;
    unsigned char pa[NPAR * (NPAR + 1) / 2], pb[NPAR * (NPAR + 1) / 2];
};

bool chol_solve(std::vector<double> M, int n, const double *b, double *x)
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

}  // namespace

extern "C" gk_status gk_create_survey(gk_model *const *models, int32_t n, gk_survey **out)
{
    if (!models || n < 1 || !out) return fail(GK_EINVAL, "invalid arguments");
    *out = nullptr;
    for (int i = 0; i < n; ++i) {
        if (!models[i]) return fail(GK_EINVAL, "model %d is NULL", i);
        if (models[i]->vfield != models[0]->vfield)
            return fail(GK_EINVAL, "model %d: all models of a survey must use one strategy", i);
        if (models[i]->use_fft)
            return fail(GK_EINVAL, "model %d uses the FFT convolution path; surveys take direct-path models", i);
        if (models[i]->device != models[0]->device)
            return fail(GK_EINVAL, "all models of a survey must be on one device");
    }
    gk_survey *s = new (std::nothrow) gk_survey();
    if (!s) return fail(GK_ENOMEM, "host allocation failed");
    s->models.assign(models, models + n);
    s->device = models[0]->device;
    DeviceGuard g(s->device);
    hipError_t e = g.err;
    if (e == hipSuccess) e = hipEventCreateWithFlags(&s->ev_staged, hipEventDisableTiming);
    if (e == hipSuccess) e = hipStreamCreate(&s->fit_stream);
    if (e != hipSuccess) {
        s->release();
        delete s;
        return fail(GK_EDEVICE, "create_survey: %s", hipGetErrorString(e));
    }
    *out = s;
    return GK_OK;
}

extern "C" gk_status gk_destroy_survey(gk_survey *s)
{
    if (!s) return GK_OK;
    {
        DeviceGuard g(s->device);
        s->release();
    }
    delete s;
    return GK_OK;
}

extern "C" gk_status gk_survey_chi2(gk_survey *s, const int32_t *model_idx, const double *params,
                                    int32_t B, double *chi2, void *stream)
{
    if (!s || B < 0) return fail(GK_EINVAL, "invalid arguments");
    if (B == 0) return GK_OK;
    if (!model_idx || !params || !chi2) return fail(GK_EINVAL, "NULL argument");
    for (gk_model *m : s->models)
        if (!m->has_obs) return fail(GK_ESTATE, "a model of the survey has no observation");
    DeviceGuard g(s->device);
    HIP_TRY(g.err);
    hipStream_t st = (hipStream_t)stream;
    if (pointer_kind(chi2) != PTR_DEVICE) return fail(GK_EINVAL, "chi2 must be device memory");
    GK_TRY(refresh_models(s, st));
    const double *dp = params;
    if (pointer_kind(params) != PTR_DEVICE) {
        HIP_TRY(hipStreamSynchronize(st));
        HIP_TRY(hipEventSynchronize(s->ev_staged));
        GK_TRY(s->h_params.need((size_t)B * NPAR));
        GK_TRY(s->params.need((size_t)B * NPAR));
        std::memcpy(s->h_params.p, params, sizeof(double) * NPAR * B);
        HIP_TRY(hipMemcpyAsync(s->params.p, s->h_params.p, sizeof(double) * NPAR * B,
                               hipMemcpyHostToDevice, st));
        dp = s->params.p;
    }
    return survey_batch(s, model_idx, dp, B, chi2, nullptr, nullptr, st);
}

extern "C" gk_status gk_fit_lm_survey(gk_survey *s, double *p_io, const uint8_t *free_mask,
                                      const double *lo_in, const double *hi_in,
                                      const gk_lm_opts *o_in, gk_lm_result *res)
{
    if (!s || !p_io || !free_mask || !res) return fail(GK_EINVAL, "NULL argument");
    for (gk_model *m : s->models)
        if (!m->has_obs) return fail(GK_ESTATE, "a model of the survey has no observation");
    gk_lm_opts o;
    gk_lm_default_opts(&o);
    if (o_in) o = *o_in;
    if (o.max_iter < 1 || !(o.fd_step > 0.0) || !(o.lambda0 > 0.0) || o.reserved != 0)
        return fail(GK_EINVAL, "invalid LM options");
    const int G = (int)s->models.size();
    std::vector<int> fr;
    for (int k = 0; k < NPAR; ++k)
        if (free_mask[k]) fr.push_back(k);
    const int nf = (int)fr.size(), rows = 1 + 2 * nf;
    DeviceGuard guard(s->device);
    HIP_TRY(guard.err);
    hipStream_t st = s->fit_stream;
    GK_TRY(refresh_models(s, st));
    // per-galaxy state
    std::vector<double> lo((size_t)G * NPAR), hi((size_t)G * NPAR), p((size_t)G * NPAR);
    for (int g = 0; g < G; ++g)
        for (int k = 0; k < NPAR; ++k) {
            double l = lo_in ? lo_in[(size_t)g * NPAR + k] : -DBL_MAX;
            double h = hi_in ? hi_in[(size_t)g * NPAR + k] : DBL_MAX;
            if (!(l <= h)) return fail(GK_EINVAL, "galaxy %d slot %d: lo > hi", g, k);
            lo[(size_t)g * NPAR + k] = l;
            hi[(size_t)g * NPAR + k] = h;
        }
    for (int g = 0; g < G; ++g) {
        double *L = &lo[(size_t)g * NPAR], *H = &hi[(size_t)g * NPAR];
        L[P_INC] = std::max(L[P_INC], 1e-3);
        H[P_INC] = std::min(H[P_INC], 90.0 - 1e-3);
        for (int k : {P_SIG, P_R0, P_RT, P_I0}) L[k] = std::max(L[k], 1e-6);
        if (s->models[g]->d.rc == RC_EPINAT) {
            L[P_G] = std::max(L[P_G], 1e-6);
            L[P_A] = std::max(L[P_A], 0.0);
        }
        for (int k = 0; k < NPAR; ++k)
            p[(size_t)g * NPAR + k] = std::min(std::max(p_io[(size_t)g * NPAR + k], L[k]), H[k]);
        if (!row_valid(&p[(size_t)g * NPAR], s->models[g]->d.rc))
            return fail(GK_EINVAL, "galaxy %d: start point outside the model domain", g);
    }
    NormIdx ix{};
    ix.nf = nf;
    ix.npairs = nf * (nf + 1) / 2;
    ix.nblk = ix.npairs + nf + 1;
    for (int a = 0, k = 0; a < nf; ++a)
        for (int b = a; b < nf; ++b, ++k) {
            ix.pa[k] = (unsigned char)a;
            ix.pb[k] = (unsigned char)b;
        }
    struct Sys { double chi2; std::vector<double> A, g; bool finite; };
    std::vector<Sys> cur(G), tri(G);
    std::vector<double> lam(G, o.lambda0);
    std::vector<int> iters(G, 0), reason(G, 0);
    std::vector<char> done(G, 0);
    std::vector<double> pt((size_t)G * NPAR);
    int64_t n_evals = 0;

    // evaluates the points q (one per listed galaxy) with their Jacobian rows
    auto evaluate = [&](const std::vector<int> &gal, const std::vector<double> &q,
                        std::vector<Sys> &out) -> gk_status {
        const int ng = (int)gal.size();
        const int B = ng * rows;
        std::vector<int32_t> midx(B);
        std::vector<int64_t> roff(B), goff(ng + 1);
        int max_chunks = 1;
        HIP_TRY(hipStreamSynchronize(st));  // the staging buffers are free again
        GK_TRY(s->h_params.need((size_t)B * NPAR));
        GK_TRY(s->params.need((size_t)B * NPAR));
        GK_TRY(s->h_scale.need((size_t)ng * NPAR));
        GK_TRY(s->scale.need((size_t)ng * NPAR));
        // [goff (ng + 1) | used entries per row (ng)]
        GK_TRY(s->h_goff.need((size_t)2 * ng + 1));
        GK_TRY(s->goff.need((size_t)2 * ng + 1));
        std::vector<int64_t> nused(ng);
        GK_TRY(s->norm.need((size_t)ng * ix.nblk));
        GK_TRY(s->h_norm.need((size_t)ng * ix.nblk));
        int64_t r = 0;
        for (int i = 0; i < ng; ++i) {
            const int g = gal[i];
            const size_t n2 = (size_t)2 * s->models[g]->d.nx * s->models[g]->d.ny;
            // without a weighted dispersion term the second map of each row is 0
            // (and velocity-field rows leave it unwritten)
            nused[i] = s->models[g]->obs_sig ? (int64_t)n2 : (int64_t)n2 / 2;
            max_chunks = std::max(max_chunks, lm_normal_chunks(nused[i]));
            goff[i] = r;
            const double *qg = &q[(size_t)g * NPAR];
            double *row = s->h_params.p + (size_t)i * rows * NPAR;
            std::memcpy(row, qg, sizeof(double) * NPAR);
            for (int a = 0; a < nf; ++a) {
                const int k = fr[a];
                double *rp = row + (size_t)(1 + 2 * a) * NPAR, *rm = rp + NPAR;
                std::memcpy(rp, qg, sizeof(double) * NPAR);
                std::memcpy(rm, qg, sizeof(double) * NPAR);
                rp[k] = std::min(qg[k] + o.fd_step, hi[(size_t)g * NPAR + k]);
                rm[k] = std::max(qg[k] - o.fd_step, lo[(size_t)g * NPAR + k]);
                s->h_scale.p[(size_t)i * NPAR + a] = rp[k] > rm[k] ? 1.0 / (rp[k] - rm[k]) : 0.0;
            }
            for (int j = 0; j < rows; ++j) {
                midx[(size_t)i * rows + j] = g;
                roff[(size_t)i * rows + j] = r + (int64_t)j * n2;
            }
            r += (int64_t)rows * n2;
        }
        goff[ng] = r;
        GK_TRY(s->resid.need((size_t)r));
        const int nchunk = max_chunks;
        GK_TRY(s->npart.need((size_t)ng * nchunk * ix.nblk));
        std::memcpy(s->h_goff.p, goff.data(), sizeof(int64_t) * (ng + 1));
        std::memcpy(s->h_goff.p + ng + 1, nused.data(), sizeof(int64_t) * ng);
        HIP_TRY(hipMemcpyAsync(s->params.p, s->h_params.p, sizeof(double) * NPAR * B,
                               hipMemcpyHostToDevice, st));
        HIP_TRY(hipMemcpyAsync(s->scale.p, s->h_scale.p, sizeof(double) * NPAR * ng,
                               hipMemcpyHostToDevice, st));
        HIP_TRY(hipMemcpyAsync(s->goff.p, s->h_goff.p, sizeof(int64_t) * (2 * ng + 1),
                               hipMemcpyHostToDevice, st));
        GK_TRY(survey_batch(s, midx.data(), s->params.p, B, nullptr, s->resid.p, roff.data(), st));
        HIP_TRY(launch_lm_normal(s->resid.p, s->goff.p, s->goff.p + ng + 1, s->scale.p, ng, nf,
                                 nchunk, s->npart.p,
                                 s->norm.p, st));
        HIP_TRY(hipMemcpyAsync(s->h_norm.p, s->norm.p, sizeof(double) * ng * ix.nblk,
                               hipMemcpyDeviceToHost, st));
        HIP_TRY(hipStreamSynchronize(st));
        n_evals += B;
        for (int i = 0; i < ng; ++i) {
            Sys &y = out[gal[i]];
            const double *v = s->h_norm.p + (size_t)i * ix.nblk;
            y.A.assign((size_t)nf * nf, 0.0);
            y.g.assign(nf, 0.0);
            bool fin = true;
            for (int k = 0; k < ix.npairs; ++k) {
                y.A[ix.pa[k] * nf + ix.pb[k]] = y.A[ix.pb[k] * nf + ix.pa[k]] = v[k];
                fin = fin && std::isfinite(v[k]);
            }
            for (int a = 0; a < nf; ++a) {
                y.g[a] = v[ix.npairs + a];
                fin = fin && std::isfinite(y.g[a]);
            }
            y.chi2 = std::isfinite(v[ix.nblk - 1]) ? v[ix.nblk - 1] : INFINITY;
            y.finite = fin && std::isfinite(y.chi2);
        }
        return GK_OK;
    };

    std::vector<int> active(G);
    for (int g = 0; g < G; ++g) active[g] = g;
    GK_TRY(evaluate(active, p, cur));
    for (int g = 0; g < G; ++g)
        if (!cur[g].finite) {
            done[g] = 1;
            reason[g] = GK_LM_LAMBDA;
        }
    std::vector<double> d(nf);
    while (true) {
        active.clear();
        for (int g = 0; g < G; ++g)
            if (!done[g]) active.push_back(g);
        if (active.empty()) break;
        for (int g : active) {  // trial points
            ++iters[g];
            std::vector<int> act;
            for (int a = 0; a < nf; ++a)
                if (cur[g].A[a * nf + a] > 0.0) act.push_back(a);
            std::fill(d.begin(), d.end(), 0.0);
            const int na = (int)act.size();
            if (na) {
                std::vector<double> M((size_t)na * na), rhs(na), x(na);
                for (int i = 0; i < na; ++i) {
                    for (int j = 0; j < na; ++j) M[i * na + j] = cur[g].A[act[i] * nf + act[j]];
                    M[i * na + i] *= 1.0 + lam[g];
                    rhs[i] = -cur[g].g[act[i]];
                }
                if (chol_solve(M, na, rhs.data(), x.data()))
                    for (int i = 0; i < na; ++i) d[act[i]] = x[i];
            }
            double *q = &pt[(size_t)g * NPAR];
            std::memcpy(q, &p[(size_t)g * NPAR], sizeof(double) * NPAR);
            for (int a = 0; a < nf; ++a) {
                const int k = fr[a];
                q[k] = std::min(std::max(p[(size_t)g * NPAR + k] + d[a], lo[(size_t)g * NPAR + k]),
                                hi[(size_t)g * NPAR + k]);
            }
        }
        GK_TRY(evaluate(active, pt, tri));
        for (int g : active) {
            double *pg = &p[(size_t)g * NPAR], *qg = &pt[(size_t)g * NPAR];
            if (tri[g].finite && tri[g].chi2 < cur[g].chi2) {
                double step = 0.0;
                for (int k : fr) step = std::max(step, std::fabs(qg[k] - pg[k]) / (std::fabs(pg[k]) + 1e-10));
                const double dec = cur[g].chi2 > 0.0 ? (cur[g].chi2 - tri[g].chi2) / cur[g].chi2 : 0.0;
                std::memcpy(pg, qg, sizeof(double) * NPAR);
                std::swap(cur[g], tri[g]);
                lam[g] /= 10.0;
                if (cur[g].chi2 == 0.0 || dec <= o.ftol) { done[g] = 1; reason[g] = GK_LM_FTOL; }
                else if (step <= o.xtol) { done[g] = 1; reason[g] = GK_LM_XTOL; }
            } else {
                lam[g] *= 10.0;
                if (lam[g] > 1e10) { done[g] = 1; reason[g] = GK_LM_LAMBDA; }
            }
            if (!done[g] && iters[g] >= o.max_iter) { done[g] = 1; reason[g] = GK_LM_MAXITER; }
        }
    }
    bool capped = false;
    for (int g = 0; g < G; ++g) {
        gk_lm_result &r = res[g];
        std::memset(&r, 0, sizeof r);
        std::vector<int> act;
        for (int a = 0; a < nf; ++a)
            if (cur[g].A.size() && cur[g].A[a * nf + a] > 0.0) act.push_back(a);
        const int na = (int)act.size();
        std::vector<double> M((size_t)na * na), e(na), col(na);
        for (int i = 0; i < na; ++i)
            for (int j = 0; j < na; ++j) M[i * na + j] = cur[g].A[act[i] * nf + act[j]];
        for (int i = 0; i < na; ++i) {
            std::fill(e.begin(), e.end(), 0.0);
            e[i] = 1.0;
            if (chol_solve(M, na, e.data(), col.data())) r.errors[fr[act[i]]] = std::sqrt(std::max(col[i], 0.0));
        }
        std::memcpy(&p_io[(size_t)g * NPAR], &p[(size_t)g * NPAR], sizeof(double) * NPAR);
        r.chi2 = cur[g].chi2;
        r.n_valid = s->models[g]->nvalid;
        r.iterations = iters[g];
        r.reason = reason[g];
        r.n_evals = (int64_t)(iters[g] + 1) * rows;
        capped = capped || reason[g] == GK_LM_MAXITER;
    }
    (void)n_evals;
    return capped ? GK_ENOTCONV : GK_OK;
}

extern "C" gk_status gk_fit_grid_survey(gk_survey *s, const double *lo0, const double *hi0,
                                        const uint8_t *free_mask, const double *fixed,
                                        const int32_t *n_per_slot, int32_t max_levels,
                                        const double *accuracy, gk_grid_result *res)
{
    if (!s || !lo0 || !hi0 || !free_mask || !fixed || !n_per_slot || !res)
        return fail(GK_EINVAL, "NULL argument");
    if (max_levels < 1) return fail(GK_EINVAL, "need max_levels >= 1");
    for (gk_model *m : s->models)
        if (!m->has_obs) return fail(GK_ESTATE, "a model of the survey has no observation");
    const int G = (int)s->models.size();
    GridShape shape{};
    double total = 1.0;
    for (int k = 0; k < NPAR; ++k) {
        if (!free_mask[k]) continue;
        if (n_per_slot[k] < 2) return fail(GK_EINVAL, "slot %d: need at least 2 nodes", k);
        shape.n[shape.d] = n_per_slot[k];
        shape.slot[shape.d++] = k;
        total *= n_per_slot[k];
    }
    if (shape.d == 0) return fail(GK_EINVAL, "no free parameter");
    if (total > 2147483648.0) return fail(GK_EINVAL, "too many nodes per level");
    shape.nodes = (int64_t)llround(total);
    std::vector<double> lo((size_t)G * NPAR), hi((size_t)G * NPAR);
    for (int g = 0; g < G; ++g)
        for (int k = 0; k < NPAR; ++k) {
            const size_t o = (size_t)g * NPAR + k;
            lo[o] = lo0[o];
            hi[o] = hi0[o];
            if (free_mask[k] && !(hi[o] > lo[o]))
                return fail(GK_EINVAL, "galaxy %d slot %d: empty range", g, k);
        }
    DeviceGuard guard(s->device);
    HIP_TRY(guard.err);
    hipStream_t st = s->fit_stream;
    GK_TRY(refresh_models(s, st));
    std::memset(res, 0, sizeof(gk_grid_result) * G);
    std::vector<int> active(G);
    for (int g = 0; g < G; ++g) active[g] = g;
    std::vector<int> levels(G, 0);
    const int64_t kChunk = 1 << 20;
    std::vector<double> spec, h_val;
    std::vector<int64_t> h_idx;
    std::vector<int32_t> midx;
    for (int level = 0; level < max_levels && !active.empty(); ++level) {
        const int na = (int)active.size();
        spec.assign((size_t)na * 3 * NPAR, 0.0);
        for (int j = 0; j < na; ++j) {
            const size_t o = (size_t)active[j] * NPAR;
            double *sp = &spec[(size_t)j * 3 * NPAR];
            for (int a = 0; a < shape.d; ++a) {
                const int k = shape.slot[a];
                sp[a] = lo[o + k];
                sp[NPAR + a] = (hi[o + k] - lo[o + k]) / (shape.n[a] - 1);
            }
            for (int k = 0; k < NPAR; ++k) sp[2 * NPAR + k] = fixed[o + k];
        }
        const int64_t rows = (int64_t)na * shape.nodes;
        const int chunk = (int)std::min<int64_t>(rows, kChunk);
        GK_TRY(s->grid_spec.need(spec.size()));
        GK_TRY(s->grid_rows.need((size_t)chunk * NPAR));
        GK_TRY(s->grid_chi2.need((size_t)chunk));
        GK_TRY(s->grid_val.need((size_t)na));
        GK_TRY(s->grid_idx.need((size_t)na));
        HIP_TRY(hipMemcpyAsync(s->grid_spec.p, spec.data(), sizeof(double) * spec.size(),
                               hipMemcpyHostToDevice, st));
        hipLaunchKernelGGL(k_grid_best_init, dim3((na + 255) / 256), dim3(256), 0, st, na,
                           s->grid_val.p, s->grid_idx.p);
        HIP_TRY(hipGetLastError());
        for (int64_t first = 0; first < rows; first += chunk) {
            const int cnt = (int)std::min<int64_t>(chunk, rows - first);
            hipLaunchKernelGGL(k_grid_rows_multi, dim3((cnt + 255) / 256), dim3(256), 0, st, shape,
                               s->grid_spec.p, first, cnt, s->grid_rows.p);
            HIP_TRY(hipGetLastError());
            midx.resize(cnt);
            for (int i = 0; i < cnt; ++i) midx[i] = active[(first + i) / shape.nodes];
            GK_TRY(survey_batch(s, midx.data(), s->grid_rows.p, cnt, s->grid_chi2.p, nullptr,
                                nullptr, st));
            const int j0 = (int)(first / shape.nodes), j1 = (int)((first + cnt - 1) / shape.nodes);
            hipLaunchKernelGGL(k_argmin_seg, dim3(j1 - j0 + 1), dim3(256), 0, st, s->grid_chi2.p,
                               first, cnt, shape.nodes, j0, s->grid_val.p, s->grid_idx.p);
            HIP_TRY(hipGetLastError());
        }
        h_val.resize(na);
        h_idx.resize(na);
        HIP_TRY(hipMemcpyAsync(h_val.data(), s->grid_val.p, sizeof(double) * na,
                               hipMemcpyDeviceToHost, st));
        HIP_TRY(hipMemcpyAsync(h_idx.data(), s->grid_idx.p, sizeof(int64_t) * na,
                               hipMemcpyDeviceToHost, st));
        HIP_TRY(hipStreamSynchronize(st));
        std::vector<int> next;
        for (int j = 0; j < na; ++j) {
            const int g = active[j];
            const size_t o = (size_t)g * NPAR;
            gk_grid_result &r = res[g];
            const double *sp = &spec[(size_t)j * 3 * NPAR];
            int64_t L = h_idx[j] == INT64_MAX ? 0 : h_idx[j];
            bool fine = accuracy != nullptr;
            for (int a = shape.d - 1; a >= 0; --a) {
                const int k = shape.slot[a];
                const int digit = (int)(L % shape.n[a]);
                L /= shape.n[a];
                const double x = sp[a] + digit * sp[NPAR + a];
                r.best[k] = x;
                r.spacing[k] = sp[NPAR + a];
                if (accuracy) fine = fine && sp[NPAR + a] < accuracy[k];
                lo[o + k] = std::max(x - sp[NPAR + a], lo0[o + k]);
                hi[o + k] = std::min(x + sp[NPAR + a], hi0[o + k]);
            }
            r.chi2 = h_val[j];
            r.best_index = h_idx[j];
            r.n_evals += shape.nodes;
            levels[g] = level + 1;
            if (!fine) next.push_back(g);
        }
        active.swap(next);
    }
    for (int g = 0; g < G; ++g) {
        for (int k = 0; k < NPAR; ++k)
            if (!free_mask[k]) {
                res[g].best[k] = fixed[(size_t)g * NPAR + k];
                res[g].spacing[k] = 0.0;
            }
        res[g].levels = levels[g];
        res[g].reserved = 0;
    }
    return GK_OK;
}
