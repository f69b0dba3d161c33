/*
 * gk_oracle.c -- plain, slow, FP64 CPU reference of one likelihood evaluation
 * of the thin-disc intensity-cube model of Bekiaris et al. (2016), "Kinematic
 * modelling of disc galaxies using graphics processing units".
 *
 * TEST INFRASTRUCTURE ONLY.  This library exists so that tests, the smoke
 * check and the CPU-baseline leg of the benchmark can check the GPU path
 * against an independent computation.  The product path never links, loads
 * or calls it.  It shares no code, header, table or constant generator with
 * the GPU library; its declarations live in this file and in oracle.py.
 *
 * Everything is double precision and follows the paper's steps in order,
 * literally: build the model cube (Sec. 2.1 eqs. 1-8, Sec. 2.2.2), convolve it
 * with the separable PSF/LSF kernel of eq. 9 (Sec. 2.2.3, done as three 1-D
 * passes z, x, y), average down by the upsampling factor (Sec. 2.2.4), take
 * the zeroth/first/second moments of every spectrum (Sec. 2.2.5) and form the
 * masked chi-square of eq. 11 (Sec. 2.2.6).  The velocity-field strategy
 * (Sec. 2.2.1) evaluates eq. 8 per data pixel and goes straight to eq. 11.
 * No blocking, fusion or reordering.  The fitters at the end (Levenberg-Marquardt, Sec. 2.3.1; nested
 * grids, Sec. 2.3.3) call the evaluation exactly as written here.
 *
 * Readings of points the paper leaves open (all listed in the design doc):
 *  - data pixel (i,j) is centred at (x,y) = (i,j); at upsampling u, fine
 *    pixel m sits at x = (m + 1/2)/u - 1/2 (fine pixels tile the data pixel);
 *  - data channel k has velocity v0 + (k - crpix) dv; fine channel m has
 *    velocity v0 + ((m + 1/2)/u - 1/2 - crpix) dv;
 *  - line profile = I(r) times a unit-area Gaussian of width sigma_model,
 *    point-sampled at channel centres; I(r) = I0 exp(-min(r/r0, 60));
 *  - r = 0 gives cos(theta) = 0;
 *  - PSF sigma = FWHM / (2 sqrt(2 ln 2)) data pixels, LSF sigma in channels =
 *    sigma_kms / dv, both times u on the fine grid; taps at integer offsets
 *    -h..h with h = ceil(R sigma), normalised to unit discrete sum; a zero
 *    width gives the single tap 1;
 *  - the model is evaluated on the fine data window plus a halo of h fine
 *    pixels (channels) on every side, and each convolution pass is "valid",
 *    so every output voxel sees real model values (consistent with the
 *    N_DATA + N_PSF - 1 extent of eq. 10);
 *  - a fine spaxel's line is kept only if it rises above 2^-40 of its peak
 *    (|v - vlos| <= sigma sqrt(80 ln 2)) at some channel of the fine model
 *    band (data channels plus the spectral halo); otherwise the spaxel has no
 *    flux.  Where it is kept, the whole sampled Gaussian is used.  This
 *    integer decision is taken in single precision (line_reaches_band);
 *  - m0 = dv * sum C; m1 = sum C v / sum C; m2 = sqrt(sum C (v - m1)^2 / sum C)
 *    (two-pass); a spectrum with sum C == 0 gets m0 = 0, m1 = Vsys, m2 = 0;
 *  - chi2 = sum over mask != 0 of (m1 - vo)^2/Ev^2 + W (m2 - so)^2/Es^2.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* parameter slots, in the order of the model description (Sec. 2.1.5):
 * centre x, centre y, position angle [deg], inclination [deg], systemic
 * velocity, rotation-curve velocity scale, turn-over radius, intrinsic
 * dispersion, disc scale length, central surface brightness, Epinat outer
 * slope a, Epinat inner slope g. */
enum { P_XO, P_YO, P_PA, P_INC, P_VSYS, P_VT, P_RT, P_SIG, P_R0, P_I0, P_A, P_G, P_N };

enum { RC_ARCTAN = 0, RC_EPINAT = 1, RC_BOISSIER = 2 };

typedef struct {
    int32_t nx, ny, nz, u;  /* data grid, upsampling factor */
    double dv, v0, crpix;   /* channel width, reference velocity, reference channel */
    double psf_fwhm;        /* data pixels, 0 = no PSF */
    double lsf_sigma;       /* km/s, 0 = no LSF */
    double R;               /* kernel truncation radius in sigmas */
    int32_t rc;             /* rotation-curve family */
    int32_t pad_;
} go_desc;

#define GO_PI 3.14159265358979323846

/* ---- kernel taps (eq. 9, one axis) ------------------------------------ */

/* Writes 2h+1 normalised Gaussian taps for standard deviation `sigma`
 * (in grid units) into taps[0..2h] (tap index j = offset + h) and returns h,
 * or -1 if more than `cap` taps would be needed. */
int go_kernel_taps(double sigma, double R, double *taps, int cap)
{
    if (!(sigma > 0.0)) {
        if (cap < 1) return -1;
        taps[0] = 1.0;
        return 0;
    }
    int h = (int)ceil(R * sigma);
    if (2 * h + 1 > cap) return -1;
    double s = 0.0;
    for (int k = -h; k <= h; ++k) {
        double t = exp(-(double)k * (double)k / (2.0 * sigma * sigma));
        taps[k + h] = t;
        s += t;
    }
    for (int k = 0; k < 2 * h + 1; ++k) taps[k] /= s;
    return h;
}

static double fwhm_to_sigma(double fwhm) { return fwhm / (2.0 * sqrt(2.0 * log(2.0))); }

/* Fine-grid PSF and LSF standard deviations. */
static double psf_sigma_fine(const go_desc *d) { return d->psf_fwhm > 0 ? d->u * fwhm_to_sigma(d->psf_fwhm) : 0.0; }
static double lsf_sigma_fine(const go_desc *d) { return d->lsf_sigma > 0 ? d->u * d->lsf_sigma / d->dv : 0.0; }

static int halo_of(double sigma, double R) { return sigma > 0.0 ? (int)ceil(R * sigma) : 0; }

/* dims[0..4] = fine halo-extended cube size (nxe, nye, nze) and the spatial
 * and spectral halos (hp, hl). */
int go_cube_dims(const go_desc *d, int32_t *dims)
{
    int hp = halo_of(psf_sigma_fine(d), d->R);
    int hl = halo_of(lsf_sigma_fine(d), d->R);
    dims[0] = d->u * d->nx + 2 * hp;
    dims[1] = d->u * d->ny + 2 * hp;
    dims[2] = d->u * d->nz + 2 * hl;
    dims[3] = hp;
    dims[4] = hl;
    return 0;
}

/* ---- parameter domain --------------------------------------------------- */

/* 1 if the parameter vector lies in the model's domain. */
int go_params_valid(const go_desc *d, const double *p)
{
    for (int k = 0; k < P_N; ++k)
        if (!isfinite(p[k])) return 0;
    if (!(p[P_INC] > 0.0 && p[P_INC] < 90.0)) return 0;
    if (!(p[P_SIG] > 0.0)) return 0;
    if (!(p[P_R0] > 0.0)) return 0;
    if (!(p[P_RT] > 0.0)) return 0;
    if (!(p[P_I0] > 0.0)) return 0;
    if (d->rc == RC_EPINAT && !(p[P_G] > 0.0 && p[P_A] >= 0.0)) return 0;
    return 1;
}

/* ---- the model (Sec. 2.1) ----------------------------------------------- */

/* Rotation curve: arctan (eq. 6), Epinat (eq. 7), or Vt (1 - exp(-r/rt)). */
double go_vrot(int rc, double r, const double *p)
{
    double vt = p[P_VT], rt = p[P_RT];
    switch (rc) {
    case RC_ARCTAN:
        return (2.0 / GO_PI) * vt * atan(r / rt);
    case RC_EPINAT: {
        double q = r / rt;
        return vt * pow(q, p[P_G]) / (1.0 + pow(q, p[P_A]));
    }
    case RC_BOISSIER:
        return vt * (1.0 - exp(-r / rt));
    }
    return NAN;
}

/* Line-of-sight velocity (eq. 8) and surface brightness (eq. 5) at sky
 * position (x, y), through the disc geometry of eqs. 1-4. */
void go_sky_point(int rc, const double *p, double x, double y, double *vlos, double *inten)
{
    double pa = p[P_PA] * GO_PI / 180.0;
    double inc = p[P_INC] * GO_PI / 180.0;
    double dx = x - p[P_XO], dy = y - p[P_YO];
    double xe = -dx * sin(pa) + dy * cos(pa);                 /* eq. 1 */
    double ye = -dx * cos(pa) - dy * sin(pa);                 /* eq. 2 */
    double r = sqrt(xe * xe + (ye / cos(inc)) * (ye / cos(inc))); /* eq. 3 */
    double costh = r > 0.0 ? xe / r : 0.0;                    /* eq. 4 */
    *vlos = p[P_VSYS] + go_vrot(rc, r, p) * sin(inc) * costh; /* eq. 8 */
    double rr = r / p[P_R0];
    if (rr > 60.0) rr = 60.0;
    *inten = p[P_I0] * exp(-rr);                              /* eq. 5 */
}

/* 1 if a line of centre vlos and width sig (km/s) rises above 2^-40 of its
 * peak, i.e. |v - vlos| <= sig sqrt(80 ln 2), at some channel of the fine model
 * band, whose channel zz (0 <= zz < nze) has velocity v_first + zz dvf.  The
 * answer is an integer decision, taken in single precision: the nearest
 * channels inside the window are ceil(c - s) and floor(c + s), with the line
 * centre c and half-width s in channel units rounded to float. */
int go_line_reaches_band(double vlos, double sig, double v_first, double dvf, int nze)
{
    float c = (float)((vlos - v_first) / dvf);
    float s = (float)(sig / dvf * sqrt(80.0 * log(2.0)));
    float lo = ceilf(c - s), hi = floorf(c + s);
    if (lo < 0.0f) lo = 0.0f;
    if (hi > (float)(nze - 1)) hi = (float)(nze - 1);
    return lo <= hi;
}

/* Model cube on the fine grid plus halo: cube[z][y][x], size nze*nye*nxe
 * (go_cube_dims).  Returns 0, or -1 for parameters outside the domain. */
int go_model_cube(const go_desc *d, const double *p, double *cube)
{
    int32_t dims[5];
    go_cube_dims(d, dims);
    int nxe = dims[0], nye = dims[1], nze = dims[2], hp = dims[3], hl = dims[4];
    if (!go_params_valid(d, p)) return -1;
    double u = d->u, sig = p[P_SIG];
    double norm = 1.0 / (sqrt(2.0 * GO_PI) * sig);
    for (int yy = 0; yy < nye; ++yy) {
        double y = ((yy - hp) + 0.5) / u - 0.5;
        for (int xx = 0; xx < nxe; ++xx) {
            double x = ((xx - hp) + 0.5) / u - 0.5;
            double vlos, inten;
            go_sky_point(d->rc, p, x, y, &vlos, &inten);
            double v_first = d->v0 + (((0 - hl) + 0.5) / u - 0.5 - d->crpix) * d->dv;
            if (!go_line_reaches_band(vlos, sig, v_first, d->dv / u, nze)) inten = 0.0;
            for (int zz = 0; zz < nze; ++zz) {
                double v = d->v0 + (((zz - hl) + 0.5) / u - 0.5 - d->crpix) * d->dv;
                double t = (v - vlos) / sig;
                cube[((size_t)zz * nye + yy) * nxe + xx] = inten * norm * exp(-0.5 * t * t);
            }
        }
    }
    return 0;
}

/* ---- convolution (eq. 9 as three 1-D passes, Sec. 2.2.3) ---------------- */

/* "Valid" separable convolution: in[nze][nye][nxe] -> out[nze-2hz][nye-2hy][nxe-2hx],
 * out[z][y][x] = sum_{a,b,c} kz[a] ky[b] kx[c] in[z+hz-a'][y+hy-b'][x+hx-c']
 * with a' = a - hz etc.  Done as a z pass, then an x pass, then a y pass. */
int go_convolve3(const double *in, int nze, int nye, int nxe,
                 const double *kz, int hz, const double *ky, int hy,
                 const double *kx, int hx, double *out)
{
    int oz = nze - 2 * hz, oy = nye - 2 * hy, ox = nxe - 2 * hx;
    if (oz <= 0 || oy <= 0 || ox <= 0) return -1;
    double *t1 = (double *)malloc(sizeof(double) * (size_t)oz * nye * nxe);
    double *t2 = (double *)malloc(sizeof(double) * (size_t)oz * nye * ox);
    if (!t1 || !t2) { free(t1); free(t2); return -2; }
    /* z pass */
    for (int z = 0; z < oz; ++z)
        for (int y = 0; y < nye; ++y)
            for (int x = 0; x < nxe; ++x) {
                double s = 0.0;
                for (int k = -hz; k <= hz; ++k)
                    s += kz[k + hz] * in[((size_t)(z + hz - k) * nye + y) * nxe + x];
                t1[((size_t)z * nye + y) * nxe + x] = s;
            }
    /* x pass */
    for (int z = 0; z < oz; ++z)
        for (int y = 0; y < nye; ++y)
            for (int x = 0; x < ox; ++x) {
                double s = 0.0;
                for (int k = -hx; k <= hx; ++k)
                    s += kx[k + hx] * t1[((size_t)z * nye + y) * nxe + (x + hx - k)];
                t2[((size_t)z * nye + y) * ox + x] = s;
            }
    /* y pass */
    for (int z = 0; z < oz; ++z)
        for (int y = 0; y < oy; ++y)
            for (int x = 0; x < ox; ++x) {
                double s = 0.0;
                for (int k = -hy; k <= hy; ++k)
                    s += ky[k + hy] * t2[((size_t)z * nye + (y + hy - k)) * ox + x];
                out[((size_t)z * oy + y) * ox + x] = s;
            }
    free(t1);
    free(t2);
    return 0;
}

/* ---- down-sampling (Sec. 2.2.4) ----------------------------------------- */

/* Mean of every u x u x u block: in[u*nz][u*ny][u*nx] -> out[nz][ny][nx]. */
int go_downsample(const double *in, int nz, int ny, int nx, int u, double *out)
{
    int NY = u * ny, NX = u * nx;
    double inv = 1.0 / ((double)u * u * u);
    for (int z = 0; z < nz; ++z)
        for (int y = 0; y < ny; ++y)
            for (int x = 0; x < nx; ++x) {
                double s = 0.0;
                for (int a = 0; a < u; ++a)
                    for (int b = 0; b < u; ++b)
                        for (int c = 0; c < u; ++c)
                            s += in[((size_t)(z * u + a) * NY + (y * u + b)) * NX + (x * u + c)];
                out[((size_t)z * ny + y) * nx + x] = s * inv;
            }
    return 0;
}

/* ---- moments (Sec. 2.2.5) ----------------------------------------------- */

/* cube[nz][ny][nx] with channel velocities vel[nz] -> maps m0, m1, m2 [ny][nx]. */
int go_moments(const double *cube, int nz, int ny, int nx, const double *vel,
               double dv, double vsys, double *m0, double *m1, double *m2)
{
    for (int y = 0; y < ny; ++y)
        for (int x = 0; x < nx; ++x) {
            size_t i = (size_t)y * nx + x;
            double s0 = 0.0, s1 = 0.0;
            for (int z = 0; z < nz; ++z) {
                double c = cube[(size_t)z * ny * nx + i];
                s0 += c;
                s1 += c * vel[z];
            }
            if (s0 > 0.0) {
                double mean = s1 / s0, s2 = 0.0;
                for (int z = 0; z < nz; ++z) {
                    double c = cube[(size_t)z * ny * nx + i];
                    s2 += c * (vel[z] - mean) * (vel[z] - mean);
                }
                m0[i] = dv * s0;
                m1[i] = mean;
                m2[i] = sqrt(s2 / s0);
            } else {
                m0[i] = 0.0;
                m1[i] = vsys;
                m2[i] = 0.0;
            }
        }
    return 0;
}

/* ---- one evaluation ------------------------------------------------------ */

/* Full pipeline: params -> maps[3][ny][nx] (m0, m1, m2).  Returns 0, -1 for
 * out-of-domain parameters (maps filled with NaN), -2 on allocation failure. */
int go_evaluate(const go_desc *d, const double *p, double *maps)
{
    size_t npix = (size_t)d->nx * d->ny;
    if (!go_params_valid(d, p)) {
        for (size_t i = 0; i < 3 * npix; ++i) maps[i] = NAN;
        return -1;
    }
    int32_t dims[5];
    go_cube_dims(d, dims);
    int nxe = dims[0], nye = dims[1], nze = dims[2], hp = dims[3], hl = dims[4];
    int u = d->u, NX = u * d->nx, NY = u * d->ny, NZ = u * d->nz;
    double *kp = (double *)malloc(sizeof(double) * (2 * hp + 1));
    double *kl = (double *)malloc(sizeof(double) * (2 * hl + 1));
    double *cube = (double *)malloc(sizeof(double) * (size_t)nxe * nye * nze);
    double *conv = (double *)malloc(sizeof(double) * (size_t)NX * NY * NZ);
    double *down = (double *)malloc(sizeof(double) * npix * d->nz);
    double *vel = (double *)malloc(sizeof(double) * d->nz);
    int rc = 0;
    if (!kp || !kl || !cube || !conv || !down || !vel) { rc = -2; goto done; }
    go_kernel_taps(psf_sigma_fine(d), d->R, kp, 2 * hp + 1);
    go_kernel_taps(lsf_sigma_fine(d), d->R, kl, 2 * hl + 1);
    go_model_cube(d, p, cube);
    if (go_convolve3(cube, nze, nye, nxe, kl, hl, kp, hp, kp, hp, conv) != 0) { rc = -2; goto done; }
    go_downsample(conv, d->nz, d->ny, d->nx, u, down);
    for (int k = 0; k < d->nz; ++k) vel[k] = d->v0 + (k - d->crpix) * d->dv;
    go_moments(down, d->nz, d->ny, d->nx, vel, d->dv, p[P_VSYS], maps, maps + npix, maps + 2 * npix);
done:
    free(kp); free(kl); free(cube); free(conv); free(down); free(vel);
    return rc;
}

/* ---- goodness of fit (eq. 11) ------------------------------------------- */

/* Masked chi-square over n pixels.  The dispersion term is skipped when W == 0. */
int go_chi2(int n, const double *m1, const double *m2, const double *vo, const double *so,
            const double *ev, const double *es, const uint8_t *mask, double W,
            double *chi2, int64_t *nvalid)
{
    double c = 0.0;
    int64_t nv = 0;
    for (int i = 0; i < n; ++i) {
        if (!mask[i]) continue;
        double rv = (m1[i] - vo[i]) / ev[i];
        c += rv * rv;
        if (W != 0.0) {
            double rs = (m2[i] - so[i]) / es[i];
            c += W * rs * rs;
        }
        ++nv;
    }
    *chi2 = c;
    if (nvalid) *nvalid = nv;
    return 0;
}

/* Evaluate then chi2 against an observation; chi2 = +inf for an out-of-domain row. */
int go_eval_chi2(const go_desc *d, const double *p, const double *vo, const double *so,
                 const double *ev, const double *es, const uint8_t *mask, double W,
                 double *chi2, int64_t *nvalid)
{
    size_t npix = (size_t)d->nx * d->ny;
    double *maps = (double *)malloc(sizeof(double) * 3 * npix);
    if (!maps) return -2;
    int rc = go_evaluate(d, p, maps);
    if (rc == -1) {
        *chi2 = INFINITY;
        if (nvalid) *nvalid = 0;
        free(maps);
        return -1;
    }
    if (rc == 0)
        go_chi2((int)npix, maps + npix, maps + 2 * npix, vo, so, ev, es, mask, W, chi2, nvalid);
    free(maps);
    return rc;
}

/* ---- velocity-field modelling strategy (Sec. 2.2.1) --------------------- */

/* The second strategy: the kinematic model evaluated straight on the data
 * grid, one value per pixel centre (x, y) = (i, j), with no cube, no PSF or
 * LSF, no down-sampling and no moments; the residual step (eq. 11) follows.
 * maps[3][ny][nx] = surface brightness (eq. 5), line-of-sight velocity
 * (eq. 8) and the intrinsic dispersion sigma, which is the model's
 * dispersion map when no beam smearing acts.  Only nx and ny of the
 * descriptor (and its rotation curve) are used.  Out-of-domain parameters
 * give NaN maps and -1. */
int go_vfield(const go_desc *d, const double *p, double *maps)
{
    size_t npix = (size_t)d->nx * d->ny;
    if (!go_params_valid(d, p)) {
        for (size_t i = 0; i < 3 * npix; ++i) maps[i] = NAN;
        return -1;
    }
    for (int y = 0; y < d->ny; ++y)
        for (int x = 0; x < d->nx; ++x) {
            size_t i = (size_t)y * d->nx + x;
            double vlos, inten;
            go_sky_point(d->rc, p, (double)x, (double)y, &vlos, &inten);
            maps[i] = inten;
            maps[npix + i] = vlos;
            maps[2 * npix + i] = p[P_SIG];
        }
    return 0;
}

/* Velocity field then chi2 (eq. 11; the dispersion term only when W != 0);
 * chi2 = +inf for an out-of-domain row. */
int go_vfield_chi2(const go_desc *d, const double *p, const double *vo, const double *so,
                   const double *ev, const double *es, const uint8_t *mask, double W,
                   double *chi2, int64_t *nvalid)
{
    size_t npix = (size_t)d->nx * d->ny;
    double *maps = (double *)malloc(sizeof(double) * 3 * npix);
    if (!maps) return -2;
    int rc = go_vfield(d, p, maps);
    if (rc == -1) {
        *chi2 = INFINITY;
        if (nvalid) *nvalid = 0;
    } else {
        go_chi2((int)npix, maps + npix, maps + 2 * npix, vo, so, ev, es, mask, W, chi2, nvalid);
    }
    free(maps);
    return rc;
}
