// gbk_vfield.hip -- the velocity-field modelling strategy (Bekiaris et al.
// 2016, Sec. 2.2.1): the kinematic model of eq. 8 evaluated directly at
// every data pixel, followed by the masked residuals and chi-square terms of
// eq. 11 (Sec. 2.2.6).  There is no cube, no PSF or LSF, no down-sampling and
// no moment step.
//
// k_vfield: one block = one tile of kVfTile consecutive pixels (a thread
// takes kVfPixPerThread of them, 256 apart, so consecutive lanes read and
// write consecutive pixels) for a group of rows.  The tile's observation
// (mask, velocity, dispersion and their inverse errors) is loaded once into
// registers and reused for every row of the group; each row's constants come
// from k_prep.  Per pixel and row: disc geometry (eqs. 1-4) from the affine
// coefficients of k_prep, rotation curve (eq. 6, eq. 7 or the exponential
// rise), eq. 8, then the chi-square terms.  Everything is FP64; the maps are
// stored as FP32.  Per row, the waves' chi-square sums go to LDS and are added
// in wave order at the end, so the tile partial has a fixed summation order.
// The row's tile partials are summed by k_reduce_chi2.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "gbk_internal.h"

namespace gbk {

namespace {

constexpr double kTwoOverPi = 0.63661977236758134308;

// 1/sqrt(r2) in FP64 (r2 >= 0; ~1e15 at r2 = 0): the FP32 estimate refined
// by one Newton step (relative error ~1e-14)
__device__ inline double rsqrt_refined(double r2)
{
    const double y0 = (double)__builtin_amdgcn_rsqf(fmaxf((float)r2, 1e-30f));
    return y0 * fma(-0.5 * r2 * y0, y0, 1.5);
}

// Rotation-curve shape V_rot(r) / V_t at q = r / r_t (r2 = r^2 tells r = 0),
// FP64: arctan (eq. 6), Epinat (eq. 7; 0 at r = 0, where a = 0 would give
// 0 * -inf), exponential rise.
template <int RC> __device__ inline double rc_shape(double qr, double r2, const double *c)
{
    if (RC == RC_ARCTAN) return kTwoOverPi * atan(qr);
    if (RC == RC_EPINAT) {
        const double lq = log2(qr);
        return r2 > 0.0 ? exp2(c[C_G] * lq) / (1.0 + exp2(c[C_A] * lq)) : 0.0;
    }
    return -expm1(-qr);
}

__device__ inline double rc_shape_rt(int rc, double qr, double r2, const double *c)
{
    switch (rc) {
    case RC_ARCTAN: return rc_shape<RC_ARCTAN>(qr, r2, c);
    case RC_EPINAT: return rc_shape<RC_EPINAT>(qr, r2, c);
    default: return rc_shape<RC_BOISSIER>(qr, r2, c);
    }
}

// eqs. 1-4 and 8 at pixel (fx, fy) of a row with constants c: returns the
// line-of-sight velocity and the deprojected radius r.  x_e and y_e / cos(i)
// are affine in the pixel indices; cos(theta) = x_e / r, 0 at the centre.
template <int RC> __device__ inline double vf_velocity(const double *c, double fx, double fy,
                                                       int rc, double &r)
{
    const double xe = fma(fx, c[C_XEX], fma(fy, c[C_XEY], c[C_XE0]));
    const double ye = fma(fx, c[C_YEX], fma(fy, c[C_YEY], c[C_YE0]));
    const double r2 = fma(xe, xe, ye * ye);
    const double yr = rsqrt_refined(r2);  // 1/r
    r = r2 * yr;
    const double qr = r * c[C_IRT];
    double shape;
    if constexpr (RC >= 0) shape = rc_shape<RC>(qr, r2, c);
    else shape = rc_shape_rt(rc, qr, r2, c);
    return c[C_VSYS] + c[C_VTSINI] * shape * (r2 > 0.0 ? xe * yr : 0.0);
}

template <int RC, bool MAPS, bool RESID, bool SIG>
__global__ __launch_bounds__(256) void k_vfield(VfArgs a)
{
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const int npix = a.nx * a.ny;
    const int tile = blockIdx.x;
    const int r0 = blockIdx.y * a.rows_per_block;
    const int r1 = min(r0 + a.rows_per_block, a.B);

    // the tile's pixels and their observation, once for all rows
    double fx[kVfPixPerThread], fy[kVfPixPerThread], vo[kVfPixPerThread], iev[kVfPixPerThread];
    double so[kVfPixPerThread], ies[kVfPixPerThread];
    bool in[kVfPixPerThread], use[kVfPixPerThread];
#pragma unroll
    for (int q = 0; q < kVfPixPerThread; ++q) {
        const int p = tile * kVfTile + q * 256 + tid;
        in[q] = p < npix;
        const int pc = in[q] ? p : 0;
        const int y = pc / a.nx;
        fx[q] = (double)(pc - y * a.nx);
        fy[q] = (double)y;
        use[q] = a.mask && in[q] && a.mask[pc] != 0;
        vo[q] = use[q] ? (double)a.vo[pc] : 0.0;
        iev[q] = use[q] ? a.iev[pc] : 0.0;
        so[q] = SIG && use[q] ? (double)a.so[pc] : 0.0;
        ies[q] = SIG && use[q] ? a.ies[pc] : 0.0;
    }

    __shared__ double wsum[kVfMaxRowsPerBlock][4];
    for (int b = r0; b < r1; ++b) {
        const double *c = a.consts + (size_t)b * NCONST;  // uniform: scalar loads
        const bool valid = c[C_VALID] != 0.0;
        const double *prow = a.params + (size_t)b * NPAR;
        const double sig = prow[P_SIG];
        double acc = 0.0;
#pragma unroll
        for (int q = 0; q < kVfPixPerThread; ++q) {
            if (!in[q]) continue;
            const size_t p = (size_t)tile * kVfTile + q * 256 + tid;
            double inten = __builtin_nan(""), v = __builtin_nan(""), s = __builtin_nan("");
            double rv = __builtin_nan(""), rs = __builtin_nan("");
            if (valid) {
                double r;
                v = vf_velocity<RC>(c, fx[q], fy[q], RC, r);
                s = sig;
                if (MAPS) inten = prow[P_I0] * exp(-fmin(r * c[C_IR0], 60.0));  // eq. 5
                rv = use[q] ? (v - vo[q]) * iev[q] : 0.0;
                rs = use[q] ? (s - so[q]) * ies[q] : 0.0;
                if (use[q]) acc += chi2_term(rv, rs);
            }
            if (MAPS) {
                float *mb = a.maps + (size_t)b * 3 * npix;
                mb[p] = (float)inten;
                mb[npix + p] = (float)v;
                mb[2 * (size_t)npix + p] = (float)s;
            }
            if (RESID) {
                double *rb = a.resid + (size_t)b * 2 * npix;
                rb[p] = valid ? rv : __builtin_nan("");
                rb[npix + p] = valid ? rs : __builtin_nan("");
            }
        }
        if (a.partial) {
            for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o, 64);
            if (lane == 0) wsum[b - r0][wave] = acc;
        }
    }
    if (a.partial) {
        __syncthreads();
        const int b = r0 + tid;
        if (b < r1) {
            const double *w = wsum[tid];
            a.partial[(size_t)b * a.ntiles + tile] = ((w[0] + w[1]) + w[2]) + w[3];
        }
    }
}

// Row-model lookup of a ragged launch: the largest k with base[k] <= x
__device__ inline int vf_find_row(const int *__restrict__ base, int n, int x)
{
    int lo = 0, hi = n;
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (base[mid] <= x) lo = mid;
        else hi = mid;
    }
    return lo;
}

// One (row, tile) per workgroup over rows of different velocity-field models
// (each with its own grid and observation); chi-square terms and residuals
// only, the same per-pixel arithmetic and summation order as k_vfield.  RC is
// the rotation curve when every row's model shares it, -1 to read it per row.
template <int RC>
__global__ __launch_bounds__(256) void k_vfield_multi(const ModelDev *__restrict__ md, RowMap rm,
                                                      const double *__restrict__ params,
                                                      const double *__restrict__ consts,
                                                      double *__restrict__ resid,
                                                      double *__restrict__ partial)
{
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const int b = vf_find_row(rm.ls_base, rm.B, blockIdx.x);
    const ModelDev &m = md[rm.row_model[b]];
    const PsfArgs &a = m.psf;
    const int tile = blockIdx.x - rm.ls_base[b];
    const int npix = a.nx * a.ny;
    const double *c = consts + (size_t)b * NCONST;
    const bool valid = c[C_VALID] != 0.0;
    const bool sig_term = m.use_sig != 0;
    double acc = 0.0;
#pragma unroll
    for (int q = 0; q < kVfPixPerThread; ++q) {
        const int p = tile * kVfTile + q * 256 + tid;
        if (p >= npix) continue;
        const int y = p / a.nx;
        const bool use = a.mask && a.mask[p] != 0;
        double rv = __builtin_nan(""), rs = __builtin_nan("");
        if (valid) {
            double r;
            const double v = vf_velocity<RC>(c, (double)(p - y * a.nx), (double)y, m.rc, r);
            const double s = params[(size_t)b * NPAR + P_SIG];
            rv = use ? (v - (double)a.vo[p]) * a.iev[p] : 0.0;
            rs = use && sig_term ? (s - (double)a.so[p]) * a.ies[p] : 0.0;
            if (use) acc += chi2_term(rv, rs);
        }
        if (resid) {  // the fitters do not read the dispersion map unless it is weighted
            double *rb = resid + rm.resid_off[b];
            rb[p] = valid ? rv : __builtin_nan("");
            if (sig_term) rb[npix + p] = valid ? rs : __builtin_nan("");
        }
    }
    if (partial) {
        for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o, 64);
        __shared__ double ws[4];
        if (lane == 0) ws[wave] = acc;
        __syncthreads();
        if (tid == 0) partial[rm.part_off[b] + tile] = ((ws[0] + ws[1]) + ws[2]) + ws[3];
    }
}

template <int RC, bool MAPS, bool RESID, bool SIG>
void launch_vf(const VfArgs &a, dim3 grid, hipStream_t s)
{
    launch(k_vfield<RC, MAPS, RESID, SIG>, grid, dim3(256), 0, s, a);
}

template <int RC, bool MAPS, bool RESID>
void launch_vf_sig(const VfArgs &a, dim3 grid, hipStream_t s)
{
    if (a.use_sig) launch_vf<RC, MAPS, RESID, true>(a, grid, s);
    else launch_vf<RC, MAPS, RESID, false>(a, grid, s);
}

template <int RC> void launch_vf_rc(const VfArgs &a, dim3 grid, hipStream_t s)
{
    const bool maps = a.maps != nullptr, resid = a.resid != nullptr;
    if (maps && resid) launch_vf_sig<RC, true, true>(a, grid, s);
    else if (maps) launch_vf_sig<RC, true, false>(a, grid, s);
    else if (resid) launch_vf_sig<RC, false, true>(a, grid, s);
    else launch_vf_sig<RC, false, false>(a, grid, s);
}

}  // namespace

int vfield_rows_per_block(int ntiles, int B)
{
    // enough blocks to give every CU several (2048 ~ 8 per CU), and within
    // that as many rows per block as possible to reuse the tile's observation
    const long target = 2048;
    long r = ((long)ntiles * B) / target;
    r = r < 1 ? 1 : (r > kVfMaxRowsPerBlock ? kVfMaxRowsPerBlock : r);
    return (int)r;
}

hipError_t launch_vfield_multi(const ModelDev *md, const RowMap &rm, int nblocks, int rc,
                               const double *params, const double *consts, double *resid,
                               double *partial, hipStream_t s)
{
    if (nblocks <= 0) return hipSuccess;
    const dim3 g(nblocks), b(256);
    switch (rc) {
    case RC_ARCTAN: launch(k_vfield_multi<RC_ARCTAN>, g, b, 0, s, md, rm, params, consts, resid, partial); break;
    case RC_EPINAT: launch(k_vfield_multi<RC_EPINAT>, g, b, 0, s, md, rm, params, consts, resid, partial); break;
    case RC_BOISSIER: launch(k_vfield_multi<RC_BOISSIER>, g, b, 0, s, md, rm, params, consts, resid, partial); break;
    default: launch(k_vfield_multi<-1>, g, b, 0, s, md, rm, params, consts, resid, partial); break;
    }
    return hipGetLastError();
}

hipError_t launch_vfield(const VfArgs &a, hipStream_t s)
{
    if (a.B <= 0) return hipSuccess;
    if (a.rows_per_block < 1 || a.rows_per_block > kVfMaxRowsPerBlock) return hipErrorInvalidValue;
    if (a.ntiles != (a.nx * a.ny + kVfTile - 1) / kVfTile) return hipErrorInvalidValue;
    const dim3 grid(a.ntiles, (a.B + a.rows_per_block - 1) / a.rows_per_block);
    if (grid.y > 65535) return hipErrorInvalidValue;
    switch (a.rc) {
    case RC_ARCTAN: launch_vf_rc<RC_ARCTAN>(a, grid, s); break;
    case RC_EPINAT: launch_vf_rc<RC_EPINAT>(a, grid, s); break;
    case RC_BOISSIER: launch_vf_rc<RC_BOISSIER>(a, grid, s); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace gbk
