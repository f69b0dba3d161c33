// gbk_kernels.hip -- gfx950 kernels of one likelihood evaluation of the
// thin-disc intensity-cube model (Bekiaris et al. 2016, Sec. 2.1-2.2).
//
// The moment sums of Sec. 2.2.5 are linear in the convolved, down-sampled
// cube, and the convolution of eq. 9 is separable.  So for moment order j
// (j = 0, 1, 2)
//
//   S_j(pixel) = sum_k vrel_k^j D[k](pixel)
//              = (1/u^2) sum_{fine block} (K_xy * T_j)(fine pixel),
//   T_j(y', x') = sum_z' c[z'][y'][x'] W_j(z'),
//   W_j(z')    = (1/u) sum_{fine channel m in the window} vrel_{m/u}^j K_z[m - z'],
//
// where c is the halo-extended fine model cube, D the down-sampled convolved
// cube (Sec. 2.2.4), vrel the data-channel velocity minus a reference
// velocity, K_z the LSF taps and K_xy the PSF.  The LSF pass, the spectral
// half of the down-sampling and the moment weighting therefore fold into three
// per-channel weight tables W_j built once per model, each fine spaxel's line
// profile reduces to three sums T_j, and only the 2-D PSF pass is left, on
// three maps.  Exact arithmetic gives the same maps as the literal
// cube -> z, x, y passes -> block mean -> moments chain; in floating point
// the difference is rounding only.
//
// Precision: the line profile exp() is evaluated in FP32 from an FP64
// argument; T_j, the PSF passes, the moment sums and chi-square are FP64.
//
// Kernels, in launch order:
//   k_prep         per evaluation: validate the row, per-row constants
//   k_line_sums    per fine spaxel of the halo-extended grid: geometry
//                  (eqs. 1-4), rotation curve (eqs. 6-7), velocity (eq. 8),
//                  brightness (eq. 5), then T_j over the channels; the weight
//                  table wz is [NZE][4] = {W0, W1, W2, 0} per fine channel
//   k_psf_moments  per (evaluation, tile): PSF x and y passes on T_j (LDS
//                  staged, or y first from HBM for 32 x 32 tiles at u = 1),
//                  u x u block sum, moments, masked chi-square terms (eq. 11)
//   k_reduce_chi2  per evaluation: fixed-order sum of the tile partials
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <array>
#include <utility>

#include "gbk_internal.h"

namespace gbk {

constexpr double kLog2e = 1.4426950408889634074;
constexpr double kInvSqrt2Pi = 0.39894228040143267794;
constexpr double kPi = 3.14159265358979323846;

// ---------------------------------------------------------------------------
// k_prep: per-row constants (FP64) -- slot layout in gbk_internal.h
// ---------------------------------------------------------------------------
__device__ inline double pack_f32x2(float lo, float hi)
{
    return __builtin_bit_cast(double, make_float2(lo, hi));
}

__device__ void prep_row(const double *__restrict__ p, double *__restrict__ c, int rc, double dvf,
                         int hp, int u, double vf0, double inv_dvf)
{
    bool ok = true;
    for (int k = 0; k < NPAR; ++k) ok = ok && isfinite(p[k]);
    ok = ok && p[P_INC] > 0.0 && p[P_INC] < 90.0 && p[P_SIG] > 0.0 && p[P_R0] > 0.0 &&
         p[P_RT] > 0.0 && p[P_I0] > 0.0;
    if (rc == RC_EPINAT) ok = ok && p[P_G] > 0.0 && p[P_A] >= 0.0;
    if (!ok) {
        for (int k = 0; k < NCONST; ++k) c[k] = 0.0;
        c[C_VALID] = 0.0;
        return;
    }
    double pa = p[P_PA] * (kPi / 180.0), inc = p[P_INC] * (kPi / 180.0);
    double sig = p[P_SIG];
    double kappa = kLog2e * dvf * dvf / (2.0 * sig * sig);
    c[C_XO] = p[P_XO];
    c[C_YO] = p[P_YO];
    c[C_SPA] = sin(pa);
    c[C_CPA] = cos(pa);
    c[C_SECI] = 1.0 / cos(inc);
    c[C_SINI] = sin(inc);
    c[C_VSYS] = p[P_VSYS];
    c[C_VT] = p[P_VT];
    c[C_IRT] = 1.0 / p[P_RT];
    c[C_IR0] = 1.0 / p[P_R0];
    c[C_LOG2AMP] = log2(p[P_I0] * kInvSqrt2Pi / sig);
    c[C_KAPPA] = kappa;
    c[C_A] = p[P_A];
    c[C_G] = p[P_G];
    c[C_VALID] = 1.0;
    c[C_ZSPAN] = sqrt(kZSpanLog2 / kappa);
    c[C_SQK] = sqrt(kappa);
    c[C_Q] = exp2(-2.0 * kappa);
    c[C_VTSINI] = p[P_VT] * sin(inc);
    c[C_F32A] = pack_f32x2((float)c[C_IRT], (float)(c[C_VTSINI] * inv_dvf));
    c[C_F32B] = pack_f32x2((float)c[C_ZSPAN], 0.0f);
    c[C_ZC0] = (p[P_VSYS] - vf0) * inv_dvf;
    c[C_IR0L] = kLog2e * c[C_IR0];
    // fine pixel (gx, gy) of the halo-extended grid sits at x = gx/u + base
    const double invu = 1.0 / u, base = (0.5 - hp) * invu - 0.5;
    const double sp = c[C_SPA], cp = c[C_CPA], se = c[C_SECI];
    const double bx = base - p[P_XO], by = base - p[P_YO];
    c[C_XEX] = -invu * sp;                       // x_e = -dx sin PA + dy cos PA   (eq. 1)
    c[C_XEY] = invu * cp;
    c[C_XE0] = -bx * sp + by * cp;
    c[C_YEX] = -invu * cp * se;                  // y_e / cos i, eqs. 2-3
    c[C_YEY] = -invu * sp * se;
    c[C_YE0] = (-bx * cp - by * sp) * se;
}

__global__ void k_prep(const double *__restrict__ params, int B, int rc, double dvf, int hp,
                       int u, double vf0, double inv_dvf, double *__restrict__ consts)
{
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b < B)
        prep_row(params + (size_t)b * NPAR, consts + (size_t)b * NCONST, rc, dvf, hp, u, vf0,
                 inv_dvf);
}

// Row -> model lookup of the ragged multi-model launches: the largest k with
// base[k] <= x, base[0] = 0 <= x < base[n] (uniform across the block).
__device__ inline int find_row(const int *__restrict__ base, int n, int x)
{
    int lo = 0, hi = n;
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (base[mid] <= x) lo = mid;
        else hi = mid;
    }
    return lo;
}

__global__ void k_prep_multi(const double *__restrict__ params, int B,
                             const int *__restrict__ row_model, const ModelDev *__restrict__ md,
                             double *__restrict__ consts)
{
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= B) return;
    const ModelDev &m = md[row_model[b]];
    prep_row(params + (size_t)b * NPAR, consts + (size_t)b * NCONST, m.rc, m.dvf, m.hp, m.u,
             m.vf0, m.inv_dvf);
}

// ---------------------------------------------------------------------------
// Wave-wide (wave64) minimum of two small non-negative integers at once:
// a and b (< 65536) are packed into one register and reduced with packed
// 16-bit minima, DPP within each row of 16 lanes, then the four row results
// through scalar registers.  The results are uniform.
// ---------------------------------------------------------------------------
__device__ inline void wave_min2(int a, int b, int &amin, int &bmin)
{
    typedef unsigned short u16x2 __attribute__((ext_vector_type(2)));
    auto pmin = [](unsigned x, unsigned y) {
        u16x2 r = __builtin_elementwise_min(__builtin_bit_cast(u16x2, x),
                                            __builtin_bit_cast(u16x2, y));
        return __builtin_bit_cast(unsigned, r);
    };
    unsigned v = (unsigned)a | ((unsigned)b << 16);
    // every lane of every row is written, so no old value is needed
    v = pmin(v, __builtin_amdgcn_mov_dpp(v, 0xB1, 0xF, 0xF, false));   // quad_perm 1,0,3,2
    v = pmin(v, __builtin_amdgcn_mov_dpp(v, 0x4E, 0xF, 0xF, false));   // quad_perm 2,3,0,1
    v = pmin(v, __builtin_amdgcn_mov_dpp(v, 0x124, 0xF, 0xF, false));  // row_ror 4
    v = pmin(v, __builtin_amdgcn_mov_dpp(v, 0x128, 0xF, 0xF, false));  // row_ror 8
    const unsigned r0 = __builtin_amdgcn_readlane(v, 0), r1 = __builtin_amdgcn_readlane(v, 16);
    const unsigned r2 = __builtin_amdgcn_readlane(v, 32), r3 = __builtin_amdgcn_readlane(v, 48);
    const unsigned lo = min(min(r0 & 0xffff, r1 & 0xffff), min(r2 & 0xffff, r3 & 0xffff));
    const unsigned hi = min(min(r0 >> 16, r1 >> 16), min(r2 >> 16, r3 >> 16));
    amin = (int)lo;
    bmin = (int)hi;
}

// Word 3 of a raw buffer descriptor on gfx9-family chips (32-bit data format;
// no swizzle, no index stride).
constexpr int kBufferDword3 = 0x00020000;
// the 64-bit payload type of the raw buffer load/store builtins
typedef unsigned int u32x2v __attribute__((__vector_size__(2 * sizeof(unsigned int))));

// 2^x for x in roughly [-1070, 1000] in FP64 with FP32 relative accuracy:
// x = n + f, f in [0, 1), 2^x = ldexp(2^f, n).
__device__ inline double exp2_wide(double x)
{
    const double n = floor(x);
    return ldexp((double)__builtin_amdgcn_exp2f((float)(x - n)), (int)n);
}

// 2^x in FP64 to ~1e-11 relative for x in roughly [-1070, 1000]: x = n + f
// with n the nearest integer and |f| <= 1/2, 2^f by its Taylor series
// sum_k (f ln 2)^k / k! to degree 9 (remainder below 1.1e-11 for |f ln 2| <=
// 0.347), then scaled by 2^n.  Used for the ratio of the channel recurrences,
// whose rounding would otherwise grow linearly along a long channel range.
__device__ inline double exp2_precise(double x)
{
    const double n = rint(x), f = x - n;
    // (ln 2)^k / k!, k = 9 .. 1
    double p = 1.0178086009239696e-07;
    p = fma(p, f, 1.3215486790144305e-06);
    p = fma(p, f, 1.5252733804059838e-05);
    p = fma(p, f, 0.00015403530393381606);
    p = fma(p, f, 0.0013333558146428441);
    p = fma(p, f, 0.009618129107628477);
    p = fma(p, f, 0.055504108664821576);
    p = fma(p, f, 0.2402265069591007);
    p = fma(p, f, 0.6931471805599453);
    p = fma(p, f, 1.0);
    return ldexp(p, (int)n);
}

// ---------------------------------------------------------------------------
// k_line_sums: T_j for every fine spaxel of the halo-extended grid.
// grid = (ceil(EX/16), ceil(EY/16), B); a block covers 16 x 16 spaxels and
// each wave an 8 x 8 square of them, so the union of the lanes' line
// supports (the wave's channel loop) stays close to each lane's own support.
// T layout [B][3][EY][EX] (x fastest).
//
// Along the channel loop the brightness-weighted line profile
// A 2^(-e^2), e = (z - zc) sqrt(kappa), is carried by the exact ratio
// recurrence g <- g r, r <- r q with q = 2^(-2 kappa), started at the wave's
// first channel.  The start values come from FP32 exp2 scaled into FP64;
// their rounding multiplies a spaxel's whole line by a constant (or tilts it
// by ~1e-6 over its width), which the moment ratios do not see at the stated
// tolerances.  When some lane would start below 2^-1020 (a steep velocity
// gradient across the wave's square), the wave evaluates exp2 per channel.
// ---------------------------------------------------------------------------
// One 16 x 16 tile (tile_x, tile_y) of one row: c = the row's constants,
// T = the row's three planes (in global memory, or in LDS when T_IN_LDS),
// count = this block's 4 support-count slots (measurement only, may be NULL).
template <bool T_IN_LDS = false>
__device__ __forceinline__ void line_sums_tile(const double *__restrict__ c,
                                               const double *__restrict__ wz, int NZE, int EX,
                                               int EY, int hp, int u, int rc, double vf0,
                                               double inv_dvf, float zedge_lo, float zedge_hi,
                                               double *__restrict__ T, int tile_x, int tile_y,
                                               unsigned long long *__restrict__ count)
{
    if (c[C_VALID] == 0.0) return;  // uniform over the block
    // a group of four waves covers the tile (workgroups of 256 threads hold
    // one group, k_eval_small's four)
    const int wave = (threadIdx.x >> 6) & 3, lane = threadIdx.x & 63;
    const int gx = (tile_x << 4) + ((wave & 1) << 3) + (lane & 7);
    const int gy = (tile_y << 4) + ((wave >> 1) << 3) + (lane >> 3);
    const bool in = gx < EX && gy < EY;

    // disc geometry, eqs. 1-4: x_e and y_e / cos(i) are affine in the fine
    // pixel indices (coefficients from k_prep).  The radius is FP64: the
    // brightness exponent r/r0 reaches 60, where FP32 rounding of r would move
    // I(r) by ~1e-5.  It is r2 * rsqrt(r2), the FP32 rsqrt refined by one
    // Newton step in FP64 (relative error ~1e-14).
    const double fx = (double)gx, fy = (double)gy;
    const double xe = fma(fx, c[C_XEX], fma(fy, c[C_XEY], c[C_XE0]));
    const double ye = fma(fx, c[C_YEX], fma(fy, c[C_YEY], c[C_YE0]));
    const double r2 = fma(xe, xe, ye * ye);
    // y0 ~ 1/r (FP32), t = r2 y0 ~ r, one Newton step: r = t (1 + e/2), e = 1 - r2 y0^2
    const double y0 = (double)__builtin_amdgcn_rsqf(fmaxf((float)r2, 1e-30f));
    const double t = r2 * y0, e = fma(-t, y0, 1.0);
    const double rd = fma(0.5 * t, e, t);
    const float r = (float)rd;

    // rotation curve (eqs. 6-7 or exponential rise) and eq. 8.  The bounded
    // curves (arctan, exponential rise: |V_rot| <= V_t) run in FP32, and the
    // product is added to Vsys in FP64.  The Epinat curve rises without bound
    // when g > a (Sec. 2.1.3), where FP32 would leave ~3e-7 of a velocity of
    // thousands of km/s in the line centre, and a line centred outside the
    // band then changes its in-band wing by ~1e-5; that curve runs in FP64.
    // line centre zc in fine halo-channel units: eq. 8 divided by the fine
    // channel width, with the line centre at zero rotation (C_ZC0) in FP64
    double zc;
    if (rc == RC_EPINAT) {
        // shape 0 at r = 0, where a = 0 would give exp2(0 * -inf) = NaN
        const double yr = y0 * fma(0.5, e, 1.0);  // 1/r
        const double lq = log2(rd * c[C_IRT]);
        const double shape = r2 > 0.0 ? exp2(c[C_G] * lq) / (1.0 + exp2(c[C_A] * lq)) : 0.0;
        const double vlos = c[C_VSYS] + c[C_VTSINI] * shape * (r2 > 0.0 ? xe * yr : 0.0);
        zc = (vlos - vf0) * inv_dvf;
    } else {
        const float2 fa = __builtin_bit_cast(float2, c[C_F32A]);
        const float costh = r > 0.0f ? (float)xe * __builtin_amdgcn_rcpf(r) : 0.0f;
        const float q = r * fa.x;
        float shape;
        if (rc == RC_ARCTAN) {
            shape = (float)(2.0 / kPi) * atanf(q);
        } else {
            // 1 - e^-q; absolute error ~1e-7, i.e. ~1e-5 km/s on the velocity
            shape = 1.0f - __builtin_amdgcn_exp2f(-q * (float)kLog2e);
        }
        zc = c[C_ZC0] + (double)(fa.y * shape * costh);
    }

    // its significant range
    const float zcf = (float)zc, span = __builtin_bit_cast(float2, c[C_F32B]).x;
    // clamp in floating point first so that the integer conversion cannot overflow;
    // an empty range is lo = NZE, hi = -1 (packed below as NZE - hi = NZE + 1)
    const int lo_in = (int)__builtin_amdgcn_fmed3f(ceilf(zcf - span), 0.0f, (float)NZE);
    const int hi_in = (int)__builtin_amdgcn_fmed3f(floorf(zcf + span), -1.0f, (float)(NZE - 1));
    const int lo0 = in ? lo_in : NZE, hi0 = in ? hi_in : -1;
    // a line centred where the spectral weight tapers off (or beyond the band)
    // sums over the whole band: the channels it would drop can carry more
    // weighted flux than the ones it keeps
    const bool edge = lo0 <= hi0 && (zcf < zedge_lo || zcf > zedge_hi);
    const int lo = edge ? 0 : lo0, hi = edge ? NZE - 1 : hi0;
    int zlo, nhi;
    wave_min2(lo, NZE - hi, zlo, nhi);
    const int zhi = NZE - nhi;
    if (count) {  // measurement only: voxels inside each lane's own support
        int n = max(hi0 - lo0 + 1, 0);
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) n += __shfl_xor(n, o, 64);
        // one slot per (block, wave): launches on a stream are ordered, so += is race-free
        if (lane == 0) count[wave] += n;
    }

    // log2 of the brightness factor: I(r) / (sqrt(2 pi) sigma), eq. 5 with the
    // exp(-60) floor
    const double lamp = c[C_LOG2AMP] - fmin(rd * c[C_IR0L], 60.0 * kLog2e);
    const double sqk = c[C_SQK];
    const double4 *w = reinterpret_cast<const double4 *>(wz);
    const double e0 = ((double)zlo - zc) * sqk;
    double t0 = 0.0, t1 = 0.0, t2 = 0.0;
    // a line below 2^-40 of its peak at every channel of the band has no flux
    // (the wave's channel range may still be run for the other lanes): its
    // lane sums g = 0
    const bool empty = lo > hi;
    if (__builtin_expect(!__any(in && e0 * e0 - lamp > 1020.0), 1)) {
        double g = empty ? 0.0 : exp2_wide(lamp - e0 * e0);
        // the ratio's rounding grows linearly along the range: beyond 48
        // channels it is formed to ~1e-11 instead of FP32's ~6e-8
        const double ra = -(2.0 * e0 + sqk) * sqk;
        double rt = zhi - zlo >= 48 ? exp2_precise(ra) : exp2_wide(ra);
        const double qq = c[C_Q];
        auto step = [&](const double4 &wk) {
            t0 = fma(g, wk.x, t0);
            t1 = fma(g, wk.y, t1);
            t2 = fma(g, wk.z, t2);
            g *= rt;
            rt *= qq;
        };
        // the next channel's weights are requested one step ahead, which
        // lets the scalar loads of two channels merge into one
        if (zlo <= zhi) {
            double4 wk = w[zlo];
#pragma unroll 2
            for (int z = zlo; z <= zhi; ++z) {
                const double4 wn = w[z < zhi ? z + 1 : z];
                step(wk);
                wk = wn;
            }
        }
    } else {
        double e = e0;
#pragma unroll 2
        for (int z = zlo; z <= zhi; ++z) {
            const double g = (double)__builtin_amdgcn_exp2f(-(float)(e * e));
            const double4 wk = w[z];
            t0 = fma(g, wk.x, t0);
            t1 = fma(g, wk.y, t1);
            t2 = fma(g, wk.z, t2);
            e += sqk;
        }
        const double amp = empty ? 0.0 : exp2_wide(lamp);
        t0 *= amp;
        t1 *= amp;
        t2 *= amp;
    }
    if (in && T_IN_LDS) {
        const int plane = EX * EY, off = gy * EX + gx;
        T[off] = t0;
        T[plane + off] = t1;
        T[2 * plane + off] = t2;
    } else if (in) {
        // buffer stores: one 32-bit byte offset from each plane's uniform base
        // (a model's plane is under 2^31 bytes)
        const size_t plane = (size_t)EX * EY;
        const int pb = (int)(sizeof(double) * plane);
        const uint32_t off = (uint32_t)(gy * EX + gx) * (uint32_t)sizeof(double);
        __builtin_amdgcn_raw_buffer_store_b64(
            __builtin_bit_cast(u32x2v, t0), __builtin_amdgcn_make_buffer_rsrc(T, 0, pb, kBufferDword3), off, 0, 0);
        __builtin_amdgcn_raw_buffer_store_b64(
            __builtin_bit_cast(u32x2v, t1), __builtin_amdgcn_make_buffer_rsrc(T + plane, 0, pb, kBufferDword3), off, 0, 0);
        __builtin_amdgcn_raw_buffer_store_b64(
            __builtin_bit_cast(u32x2v, t2), __builtin_amdgcn_make_buffer_rsrc(T + 2 * plane, 0, pb, kBufferDword3), off, 0, 0);
    }
}

__global__ __launch_bounds__(256) void k_line_sums(const double *__restrict__ consts,
                                                   const double *__restrict__ wz, int NZE, int EX,
                                                   int EY, int hp, int u, int rc, double vf0,
                                                   double inv_dvf, float zedge_lo, float zedge_hi,
                                                   double *__restrict__ T,
                                                   unsigned long long *__restrict__ support_count)
{
    const int b = blockIdx.z;
    unsigned long long *cnt = nullptr;
    if (support_count)
        cnt = support_count + (((size_t)b * gridDim.y + blockIdx.y) * gridDim.x + blockIdx.x) * 4;
    line_sums_tile(consts + (size_t)b * NCONST, wz, NZE, EX, EY, hp, u, rc, vf0, inv_dvf, zedge_lo,
                   zedge_hi, T + (size_t)b * 3 * EX * EY, blockIdx.x, blockIdx.y, cnt);
}

// Ragged rows of several models: block -> (row, tile) through the tile prefix
// sums of the rows.
__global__ __launch_bounds__(256) void k_line_sums_multi(const double *__restrict__ consts,
                                                         const ModelDev *__restrict__ md,
                                                         RowMap rm, double *__restrict__ T)
{
    const int b = find_row(rm.ls_base, rm.B, blockIdx.x);
    const ModelDev &m = md[rm.row_model[b]];
    const int t = blockIdx.x - rm.ls_base[b], tiles_x = (m.EX + 15) >> 4;
    line_sums_tile(consts + (size_t)b * NCONST, m.wz, m.NZE, m.EX, m.EY, m.hp, m.u, m.rc,
                   m.vf0, m.inv_dvf, m.zedge_lo, m.zedge_hi, T + rm.T_off[b], t % tiles_x,
                   t / tiles_x, nullptr);
}

// ---------------------------------------------------------------------------
// k_psf_moments: per (tile, evaluation).  Dynamic LDS:
//   sT [LY][LX]  one T_j plane of the tile plus PSF halo
//   sX [LY][TX]  after the x pass
//   sK [2hp+1]   PSF taps
// ---------------------------------------------------------------------------
__device__ __forceinline__ void psf_generic_tile(const PsfArgs &a, const RowPtrs &r)
{
    extern __shared__ double lds[];
    const int tile = r.tile, tid = threadIdx.x;
    const int tx0 = (tile % a.ntx) * a.TXd, ty0 = (tile / a.ntx) * a.TYd;
    const int u = a.u, hp = a.hp, K = 2 * hp + 1;
    const int TX = u * a.TXd, TY = u * a.TYd, LX = TX + 2 * hp, LY = TY + 2 * hp;
    double *sT = lds, *sX = lds + LY * LX, *sK = sX + LY * TX;
    const double *cb = r.c;
    const bool valid = cb[C_VALID] != 0.0;
    const int npx = a.TXd * a.TYd;

    for (int k = tid; k < K; k += 256) sK[k] = a.kp[k];

    double S[3][kMaxPixPerThread];
#pragma unroll
    for (int j = 0; j < 3; ++j)
#pragma unroll
        for (int q = 0; q < kMaxPixPerThread; ++q) S[j][q] = 0.0;

    if (valid) {
        const size_t plane = (size_t)a.EX * a.EY;
        const int gx0 = u * tx0, gy0 = u * ty0;
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            const double *Tj = r.T + (size_t)j * plane;
            __syncthreads();
            for (int i = tid; i < LY * LX; i += 256) {
                const int ly = i / LX, lx = i - ly * LX;
                const int gy = gy0 + ly, gx = gx0 + lx;
                sT[i] = (gy < a.EY && gx < a.EX) ? Tj[(size_t)gy * a.EX + gx] : 0.0;
            }
            __syncthreads();
            // x pass: sX[ly][X] = sum_k K[k] sT[ly][X + 2hp - k]
            for (int i = tid; i < LY * TX; i += 256) {
                const int ly = i / TX, X = i - ly * TX;
                const double *row = sT + ly * LX + X + 2 * hp;
                double s = 0.0;
                for (int k = 0; k < K; ++k) s = fma(sK[k], row[-k], s);
                sX[i] = s;
            }
            __syncthreads();
            // y pass and u x u block sum, one data pixel per (thread, q)
#pragma unroll
            for (int q = 0; q < kMaxPixPerThread; ++q) {
                const int pix = tid + 256 * q;
                if (pix < npx) {
                    const int xd = pix % a.TXd, yd = pix / a.TXd;
                    double s = 0.0;
                    for (int ay = 0; ay < u; ++ay)
                        for (int ax = 0; ax < u; ++ax) {
                            const int Y = yd * u + ay, X = xd * u + ax;
                            const double *col = sX + (Y + 2 * hp) * TX + X;
                            for (int k = 0; k < K; ++k) s = fma(sK[k], col[-k * TX], s);
                        }
                    S[j][q] = s;
                }
            }
        }
    }

    // moments (Sec. 2.2.5) and chi-square terms (eq. 11)
    double acc = 0.0;
    const double inv_uu = 1.0 / ((double)u * u);
#pragma unroll
    for (int q = 0; q < kMaxPixPerThread; ++q) {
        const int pix = tid + 256 * q;
        if (pix >= npx) continue;
        const int xd = tx0 + pix % a.TXd, yd = ty0 + pix / a.TXd;
        if (xd >= a.nx || yd >= a.ny) continue;
        const size_t p = (size_t)yd * a.nx + xd;
        double m0, m1, m2;
        if (!valid) {
            m0 = m1 = m2 = __builtin_nan("");
        } else {
            moment_maps(S[0][q] * inv_uu, S[1][q] * inv_uu, S[2][q] * inv_uu, a.dv, a.vref,
                        cb[C_VSYS], m0, m1, m2);
        }
        const size_t npix = (size_t)a.nx * a.ny;
        if (r.maps) {
            float *mb = r.maps;
            mb[p] = (float)m0;
            mb[npix + p] = (float)m1;
            mb[2 * npix + p] = (float)m2;
        }
        if (a.mask) {
            const bool use = a.mask[p] != 0;
            const double rv = use ? (m1 - (double)a.vo[p]) * a.iev[p] : 0.0;
            const double rs = use ? (m2 - (double)a.so[p]) * a.ies[p] : 0.0;
            if (use) acc += chi2_term(rv, rs);
            if (r.resid) {
                double *rb = r.resid;
                rb[p] = valid ? rv : __builtin_nan("");
                rb[npix + p] = valid ? rs : __builtin_nan("");
            }
        }
    }
    if (r.partial) {
        // fixed-order block reduction: wave butterfly, then waves in order
        for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o, 64);
        __shared__ double wsum[4];
        __syncthreads();
        if ((tid & 63) == 0) wsum[tid >> 6] = acc;
        __syncthreads();
        if (tid == 0)
            *r.partial = ((wsum[0] + wsum[1]) + wsum[2]) + wsum[3];
    }
}

// ---------------------------------------------------------------------------
// psf_u1_tile<HP, TX>: the u = 1 case with TX x 32 data-pixel tiles (used for
// TX = 64; 32 x 32 tiles take psf_yx_tile below) and a compile-time PSF
// half-width HP (0..kMaxFastHalo).
// Each plane j: T tile + halo -> LDS (sT), x pass -> sX, y pass -> registers.
// Both passes are register-blocked along the pass direction (a thread makes
// 4 or RPT consecutive outputs from one window of LDS values) with the taps
// in scalar registers.  Row strides of sT and sX are = 1 (mod 4) doubles so
// that the lanes of a wave spread over all LDS banks.  Thread t owns column
// t % TX and RPT = TX * 32 / 256 consecutive rows.
// ---------------------------------------------------------------------------
template <int HP, int N>
__device__ inline void window(const double *src, int stride, const double *kp, double *out)
{
    constexpr int K = 2 * HP + 1;
    double v[K + N - 1];
#pragma unroll
    for (int w = 0; w < K + N - 1; ++w) v[w] = src[w * stride];
#pragma unroll
    for (int o = 0; o < N; ++o) {
        double acc = 0.0;
        // output o = sum_k K[k] v[o + 2HP - k]
#pragma unroll
        for (int k = 0; k < K; ++k) acc = fma(kp[k], v[o + 2 * HP - k], acc);
        out[o] = acc;
    }
}


template <int HP, int TX>
__device__ __forceinline__ void psf_u1_tile(const PsfArgs &a, const RowPtrs &r)
{
    extern __shared__ double lds[];
    constexpr int TY = 32, K = 2 * HP + 1;
    constexpr int LX = TX + 2 * HP, LY = TY + 2 * HP;
    constexpr int ST = pad_stride(LX), SX = pad_stride(TX);
    constexpr int RPT = TX * TY / 256;       // rows per thread in the y pass
    constexpr int TPR = TX / 4;              // x-pass tasks per row
    const int tile = r.tile, tid = threadIdx.x;
    const int tx0 = (tile % a.ntx) * TX, ty0 = (tile / a.ntx) * TY;
    double *sT = lds, *sX = lds + LY * ST;
    const double *cb = r.c;
    const bool valid = cb[C_VALID] != 0.0;
    double kp[K];
#pragma unroll
    for (int k = 0; k < K; ++k) kp[k] = a.kp[k];
    const int col = tid % TX, row0 = (tid / TX) * RPT;

    double S[3][RPT];
#pragma unroll
    for (int j = 0; j < 3; ++j)
#pragma unroll
        for (int q = 0; q < RPT; ++q) S[j][q] = 0.0;

    if (valid) {
        const size_t plane = (size_t)a.EX * a.EY;
        // tile + halo, LY x LX values: element i of thread t is flat index
        // t + 256 i; the next plane is fetched into registers while the
        // current one is convolved
        constexpr int NLD = (LY * LX + 255) / 256;
        int goff[NLD];
        bool gok[NLD];
#pragma unroll
        for (int i = 0; i < NLD; ++i) {
            const int f = tid + 256 * i, ly = f / LX, lx = f - ly * LX;
            const int gy = ty0 + ly, gx = tx0 + lx;
            gok[i] = f < LY * LX && gy < a.EY && gx < a.EX;
            goff[i] = gok[i] ? gy * a.EX + gx : 0;
        }
        const double *Tb = r.T;
        double pre[NLD];
#pragma unroll
        for (int i = 0; i < NLD; ++i) pre[i] = gok[i] ? Tb[goff[i]] : 0.0;
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            if (j) __syncthreads();
#pragma unroll
            for (int i = 0; i < NLD; ++i) {
                const int f = tid + 256 * i, ly = f / LX, lx = f - ly * LX;
                if (f < LY * LX) sT[ly * ST + lx] = pre[i];
            }
            if (j < 2) {
                const double *Tn = Tb + (size_t)(j + 1) * plane;
#pragma unroll
                for (int i = 0; i < NLD; ++i) pre[i] = gok[i] ? Tn[goff[i]] : 0.0;
            }
            __syncthreads();
            for (int task = tid; task < LY * TPR; task += 256) {
                const int ly = task / TPR, x0 = (task % TPR) * 4;
                double o4[4];
                window<HP, 4>(sT + ly * ST + x0, 1, kp, o4);
                double *dst = sX + ly * SX + x0;
#pragma unroll
                for (int o = 0; o < 4; ++o) dst[o] = o4[o];
            }
            __syncthreads();
            window<HP, RPT>(sX + row0 * SX + col, SX, kp, S[j]);
        }
    }

    double acc = 0.0;
    const size_t npix = (size_t)a.nx * a.ny;
#pragma unroll
    for (int q = 0; q < RPT; ++q) {
        const int xd = tx0 + col, yd = ty0 + row0 + q;
        if (xd >= a.nx || yd >= a.ny) continue;
        const size_t p = (size_t)yd * a.nx + xd;
        double m0, m1, m2;
        if (!valid)
            m0 = m1 = m2 = __builtin_nan("");
        else
            moment_maps(S[0][q], S[1][q], S[2][q], a.dv, a.vref, cb[C_VSYS], m0, m1, m2);
        if (r.maps) {
            float *mb = r.maps;
            mb[p] = (float)m0;
            mb[npix + p] = (float)m1;
            mb[2 * npix + p] = (float)m2;
        }
        if (a.mask) {
            const bool use = a.mask[p] != 0;
            const double rv = use ? (m1 - (double)a.vo[p]) * a.iev[p] : 0.0;
            const double rs = use ? (m2 - (double)a.so[p]) * a.ies[p] : 0.0;
            if (use) acc += chi2_term(rv, rs);
            if (r.resid) {
                double *rb = r.resid;
                rb[p] = valid ? rv : __builtin_nan("");
                rb[npix + p] = valid ? rs : __builtin_nan("");
            }
        }
    }
    if (r.partial) {
        for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o, 64);
        __shared__ double wsum[4];
        __syncthreads();
        if ((tid & 63) == 0) wsum[tid >> 6] = acc;
        __syncthreads();
        if (tid == 0)
            *r.partial = ((wsum[0] + wsum[1]) + wsum[2]) + wsum[3];
    }
}

// Observation of the four pixels xd0 .. xd0 + 3 of row yd (nx = 0 mod 4 and
// a mask present; otherwise nothing is read and the epilogue reads the
// observation per pixel).
struct ObsQuad {
    uint32_t mk;  // the four mask bytes, unpacked where they are used
    float4 vo, so;
    double2 ev0, ev1, es0, es1;
};

__device__ __forceinline__ ObsQuad load_obs_quad(const PsfArgs &a, int yd, int xd0)
{
    ObsQuad q{};
    if (a.mask && (a.nx & 3) == 0 && yd < a.ny && xd0 < a.nx) {
        const size_t p0 = (size_t)yd * a.nx + xd0;
        q.mk = *reinterpret_cast<const uint32_t *>(a.mask + p0);
        q.vo = *reinterpret_cast<const float4 *>(a.vo + p0);
        q.so = *reinterpret_cast<const float4 *>(a.so + p0);
        q.ev0 = *reinterpret_cast<const double2 *>(a.iev + p0);
        q.ev1 = *reinterpret_cast<const double2 *>(a.iev + p0 + 2);
        q.es0 = *reinterpret_cast<const double2 *>(a.ies + p0);
        q.es1 = *reinterpret_cast<const double2 *>(a.ies + p0 + 2);
    }
    return q;
}

// Moments, maps, residuals and the tile's chi-square partial of the 32 x 32
// u = 1 kernels: thread tid holds the sums S of the pixels xd0 .. xd0 + 3 of
// data row yd; ob is their observation (load_obs_quad).  With nx = 0 (mod 4)
// the pixels are inside the image and 16-byte aligned, and the outputs are
// written as vectors.
__device__ __forceinline__ void yx_epilogue(const PsfArgs &a, const RowPtrs &r,
                                            const double (&S)[3][4], bool valid, int yd, int xd0,
                                            int tid, const ObsQuad &ob)
{
    const int wave = tid >> 6, lane = tid & 63;
    const double *cb = r.c;
    double acc = 0.0;
    const size_t npix = (size_t)a.nx * a.ny;
    if (yd < a.ny && xd0 < a.nx) {
        double m0[4], m1[4], m2[4];
#pragma unroll
        for (int o = 0; o < 4; ++o) {
            if (!valid)
                m0[o] = m1[o] = m2[o] = __builtin_nan("");
            else
                moment_maps(S[0][o], S[1][o], S[2][o], a.dv, a.vref, cb[C_VSYS], m0[o], m1[o],
                            m2[o]);
        }
        const size_t p0 = (size_t)yd * a.nx + xd0;
        double rv[4], rs[4];
        if ((a.nx & 3) == 0) {
            if (r.maps) {
                float *mb = r.maps + p0;
                *reinterpret_cast<float4 *>(mb) =
                    make_float4((float)m0[0], (float)m0[1], (float)m0[2], (float)m0[3]);
                *reinterpret_cast<float4 *>(mb + npix) =
                    make_float4((float)m1[0], (float)m1[1], (float)m1[2], (float)m1[3]);
                *reinterpret_cast<float4 *>(mb + 2 * npix) =
                    make_float4((float)m2[0], (float)m2[1], (float)m2[2], (float)m2[3]);
            }
            if (a.mask) {
                const uchar4 mk = __builtin_bit_cast(uchar4, ob.mk);
                const float4 vo = ob.vo, so = ob.so;
                const double2 ev0 = ob.ev0, ev1 = ob.ev1, es0 = ob.es0, es1 = ob.es1;
                const bool use[4] = {mk.x != 0, mk.y != 0, mk.z != 0, mk.w != 0};
                const float vof[4] = {vo.x, vo.y, vo.z, vo.w}, sof[4] = {so.x, so.y, so.z, so.w};
                const double iev[4] = {ev0.x, ev0.y, ev1.x, ev1.y};
                const double ies[4] = {es0.x, es0.y, es1.x, es1.y};
#pragma unroll
                for (int o = 0; o < 4; ++o) {
                    rv[o] = use[o] ? (m1[o] - (double)vof[o]) * iev[o] : 0.0;
                    rs[o] = use[o] ? (m2[o] - (double)sof[o]) * ies[o] : 0.0;
                    if (use[o]) acc += chi2_term(rv[o], rs[o]);
                }
                if (r.resid) {
                    double *rb = r.resid + p0;
                    if (!valid)
#pragma unroll
                        for (int o = 0; o < 4; ++o) rv[o] = rs[o] = __builtin_nan("");
                    *reinterpret_cast<double2 *>(rb) = make_double2(rv[0], rv[1]);
                    *reinterpret_cast<double2 *>(rb + 2) = make_double2(rv[2], rv[3]);
                    *reinterpret_cast<double2 *>(rb + npix) = make_double2(rs[0], rs[1]);
                    *reinterpret_cast<double2 *>(rb + npix + 2) = make_double2(rs[2], rs[3]);
                }
            }
        } else {
#pragma unroll
            for (int o = 0; o < 4; ++o) {
                if (xd0 + o >= a.nx) break;
                const size_t p = p0 + o;
                if (r.maps) {
                    float *mb = r.maps;
                    mb[p] = (float)m0[o];
                    mb[npix + p] = (float)m1[o];
                    mb[2 * npix + p] = (float)m2[o];
                }
                if (a.mask) {
                    const bool use = a.mask[p] != 0;
                    rv[o] = use ? (m1[o] - (double)a.vo[p]) * a.iev[p] : 0.0;
                    rs[o] = use ? (m2[o] - (double)a.so[p]) * a.ies[p] : 0.0;
                    if (use) acc += chi2_term(rv[o], rs[o]);
                    if (r.resid) {
                        double *rb = r.resid;
                        rb[p] = valid ? rv[o] : __builtin_nan("");
                        rb[npix + p] = valid ? rs[o] : __builtin_nan("");
                    }
                }
            }
        }
    }
    if (r.partial) {
        for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o, 64);
        __shared__ double wsum[4];
        if (lane == 0) wsum[wave] = acc;
        __syncthreads();
        if (tid == 0)
            *r.partial = ((wsum[0] + wsum[1]) + wsum[2]) + wsum[3];
    }
}

// ---------------------------------------------------------------------------
// psf_yx_tile<HP>: the u = 1 case with 32 x 32 data-pixel tiles, y pass first.
// Wave w owns output rows 8w..8w+7 of the tile and lane l the T column
// tx0 + l (l < 32 + 2 HP <= 64).  Each lane loads its column's 8 + 2 HP
// values straight from global memory (a wave reads contiguous row segments)
// and makes the 8 y-pass outputs in registers; the y-pass rows go to LDS once
// per plane, and the x pass reads them back register-blocked (a lane makes 4
// consecutive outputs of one row from a window of 4 + 2 HP values).  The LDS
// rows a wave reads in the x pass are the rows it wrote itself, so the passes
// and the planes (which reuse the rows) are ordered by wave-level fences only,
// and the waves of a tile run independently until the chi-square sum.
// Row stride of sY = 1 (mod 4) doubles, which spreads the x-pass lanes of a
// wave (8 rows x 8 windows) over all LDS banks.
// ---------------------------------------------------------------------------

// Orders a wave's LDS accesses before and after this point (the hardware runs
// one wave's LDS instructions in order; this keeps the compiler from moving
// them across).
__device__ __forceinline__ void wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

template <int HP>
__device__ __forceinline__ void psf_yx_tile(const PsfArgs &a, const RowPtrs &r)
{
    extern __shared__ double lds[];
    constexpr int TT = 32, K = 2 * HP + 1, LX = TT + 2 * HP;
    constexpr int RW = 8, NW = RW + 2 * HP;  // y-pass outputs and window per lane
    constexpr int SY = pad_stride(LX);
    static_assert(LX <= 64, "one lane per T column");
    const int tile = r.tile, tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const int tx0 = (tile % a.ntx) * TT, ty0 = (tile / a.ntx) * TT;
    const double *cb = r.c;
    const bool valid = cb[C_VALID] != 0.0;
    double kp[K];
#pragma unroll
    for (int k = 0; k < K; ++k) kp[k] = a.kp[k];
    // x pass: lane -> row ry of the tile (inside this wave's 8 rows) and
    // columns x0 .. x0 + 3
    const int ry = tid >> 3, x0 = (tid & 7) * 4;

    double S[3][4];
#pragma unroll
    for (int j = 0; j < 3; ++j)
#pragma unroll
        for (int o = 0; o < 4; ++o) S[j][o] = 0.0;

    if (valid) {
        // Loads go through one buffer descriptor per plane whose range is the
        // plane: a row beyond EY reads 0 from the hardware's range check, and a
        // lane beyond the tile's columns or EX gets an offset beyond every
        // plane (the host keeps a plane under 2^31 bytes for this kernel).
        const uint32_t plane_bytes = (uint32_t)(sizeof(double) * a.EX * a.EY);
        const int gx = tx0 + lane, gy0 = ty0 + RW * wave;
        const bool colok = lane < LX && gx < a.EX;
        const uint32_t off0 = colok ? (uint32_t)(sizeof(double) * ((size_t)gy0 * a.EX + gx))
                                    : 0x80000000u;
        const uint32_t step = colok ? (uint32_t)(sizeof(double) * a.EX) : 0u;
        auto load_plane = [&](int j, double *dst) {
            const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(
                (void *)(r.T + (size_t)j * a.EX * a.EY), 0, (int)plane_bytes, kBufferDword3);
#pragma unroll
            for (int w = 0; w < NW; ++w)
                dst[w] = __builtin_bit_cast(
                    double, __builtin_amdgcn_raw_buffer_load_b64(rs, off0 + (uint32_t)w * step, 0, 0));
        };
        double *sw = lds + (size_t)RW * wave * SY;  // this wave's rows
        double v[NW], vn[NW];
        load_plane(0, v);
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            if (j < 2) load_plane(j + 1, vn);
            double y[RW];
#pragma unroll
            for (int o = 0; o < RW; ++o) {
                double acc = 0.0;
                // output o = sum_k K[k] v[o + 2HP - k]
#pragma unroll
                for (int k = 0; k < K; ++k) acc = fma(kp[k], v[o + 2 * HP - k], acc);
                y[o] = acc;
            }
            // the x pass of the previous plane has read these rows
            wave_sync();
            if (lane < LX) {
                double *dst = sw + lane;
#pragma unroll
                for (int o = 0; o < RW; ++o) dst[o * SY] = y[o];
            }
            wave_sync();
            window<HP, 4>(lds + (size_t)ry * SY + x0, 1, kp, S[j]);
            if (j < 2) {
#pragma unroll
                for (int w = 0; w < NW; ++w) v[w] = vn[w];
            }
        }
    }

    // moments and chi-square terms of the lane's 4 pixels (xd0 .. xd0 + 3, yd)
    const int yd = ty0 + ry, xd0 = tx0 + x0;
    yx_epilogue(a, r, S, valid, yd, xd0, tid, load_obs_quad(a, yd, xd0));
}

// Row pointers of a single-model launch, grid (ntiles, B).  Workgroups go to
// the 8 XCDs round-robin by linear id; the ids are remapped so that all tiles
// of one row run on one XCD and the halo each tile shares with its
// neighbours is re-read from that XCD's L2 rather than from HBM: id L goes to
// XCD L % 8, which takes rows b = L % 8 (mod 8) tile by tile (rows beyond the
// last full group of 8 keep the plain order).
__device__ __forceinline__ RowPtrs single_row(const PsfArgs &a)
{
    const int ntiles = gridDim.x, L = blockIdx.x + blockIdx.y * ntiles;
    const int full = gridDim.y >> 3, base = 8 * ntiles * full;
    int b, tile;
    if (L < base) {
        const int s = L >> 3;
        b = (L & 7) + 8 * (s / ntiles);
        tile = s % ntiles;
    } else {
        const int rest = L - base;
        b = 8 * full + rest / ntiles;
        tile = rest % ntiles;
    }
    const size_t npix = (size_t)a.nx * a.ny;
    RowPtrs r;
    r.T = a.T + (size_t)b * 3 * a.EX * a.EY;
    r.c = a.consts + (size_t)b * NCONST;
    r.maps = a.maps ? a.maps + (size_t)b * 3 * npix : nullptr;
    r.resid = a.resid ? a.resid + (size_t)b * 2 * npix : nullptr;
    r.partial = a.partial ? a.partial + (size_t)b * a.ntiles + tile : nullptr;
    r.tile = tile;
    return r;
}

__global__ __launch_bounds__(256) void k_psf_moments(PsfArgs a) { psf_generic_tile(a, single_row(a)); }

template <int HP, int TX>
__global__ __launch_bounds__(256) void k_psf_moments_u1(PsfArgs a)
{
    if constexpr (TX == 32)
        psf_yx_tile<HP>(a, single_row(a));
    else
        psf_u1_tile<HP, TX>(a, single_row(a));
}

// ---------------------------------------------------------------------------
// k_eval_small: the whole evaluation of one row of a small u = 1 model in one
// workgroup of 1024 threads, for latency-bound callers (the Levenberg-Marquardt
// iteration evaluates 1 + 2 n_free rows at a time): the row's constants (one
// thread, into LDS), the line sums, the PSF passes, moments and residuals, in
// one launch.  The T planes stay in LDS
// ([3][EY][EX]); each plane's y pass goes to LDS ([ny][EX]) and its x pass to
// registers (pixel tid + 1024 q, q < kSmallPix); then moments, maps and the
// residuals of eq. 11.  The passes take the taps in the order of
// psf_yx_tile (y first, each output an FMA chain from k = 0 to 2 HP), so the
// maps and residuals equal, bit for bit, those of the 32 x 32 register-blocked
// path.
// ---------------------------------------------------------------------------
constexpr int kSmallPix = 2;  // pixels per thread: nx * ny <= 2048

__global__ __launch_bounds__(1024) void k_eval_small(const double *__restrict__ params,
                                                     const double *__restrict__ wz, int NZE,
                                                     int rc, double dvf, double vf0,
                                                     double inv_dvf, float zedge_lo,
                                                     float zedge_hi, PsfArgs a)
{
    extern __shared__ double lds[];
    __shared__ double c[NCONST];  // the row's constants (k_prep's)
    const int b = blockIdx.x, tid = threadIdx.x, hp = a.hp, K = 2 * a.hp + 1;
    const int EX = a.EX, EY = a.EY, nx = a.nx, ny = a.ny, npix = nx * ny;
    if (tid == 0) prep_row(params + (size_t)b * NPAR, c, rc, dvf, hp, 1, vf0, inv_dvf);
    __syncthreads();
    const bool valid = c[C_VALID] != 0.0;
    double *T = lds, *Y = lds + (size_t)3 * EX * EY;
    if (valid) {  // uniform: line sums of the 16 x 16 tiles, four at a time
        const int ntx = (EX + 15) >> 4, nt = ntx * ((EY + 15) >> 4);
        for (int t = tid >> 8; t < nt; t += 4)
            line_sums_tile<true>(c, wz, NZE, EX, EY, hp, 1, rc, vf0, inv_dvf, zedge_lo, zedge_hi, T,
                           t % ntx, t / ntx, nullptr);
    }
    __syncthreads();
    double S[3][kSmallPix];
#pragma unroll
    for (int j = 0; j < 3; ++j) {
#pragma unroll
        for (int q = 0; q < kSmallPix; ++q) S[j][q] = 0.0;
        if (!valid) continue;
        const double *Tj = T + (size_t)j * EX * EY;
        for (int e = tid; e < ny * EX; e += 1024) {
            const int y = e / EX, x = e - y * EX;
            const double *col = Tj + (size_t)(y + 2 * hp) * EX + x;
            double acc = 0.0;
            for (int k = 0; k < K; ++k) acc = fma(a.kp[k], col[-(ptrdiff_t)k * EX], acc);
            Y[e] = acc;
        }
        __syncthreads();
#pragma unroll
        for (int q = 0; q < kSmallPix; ++q) {
            const int p = tid + 1024 * q;
            if (p >= npix) continue;
            const int y = p / nx, x = p - y * nx;
            const double *row = Y + (size_t)y * EX + x + 2 * hp;
            double acc = 0.0;
            for (int k = 0; k < K; ++k) acc = fma(a.kp[k], row[-k], acc);
            S[j][q] = acc;
        }
        __syncthreads();
    }
    float *maps = a.maps ? a.maps + (size_t)b * 3 * npix : nullptr;
    double *resid = a.resid ? a.resid + (size_t)b * 2 * npix : nullptr;
#pragma unroll
    for (int q = 0; q < kSmallPix; ++q) {
        const int p = tid + 1024 * q;
        if (p >= npix) continue;
        double m0, m1, m2;
        if (!valid)
            m0 = m1 = m2 = __builtin_nan("");
        else
            moment_maps(S[0][q], S[1][q], S[2][q], a.dv, a.vref, c[C_VSYS], m0, m1, m2);
        if (maps) {
            maps[p] = (float)m0;
            maps[npix + p] = (float)m1;
            maps[2 * npix + p] = (float)m2;
        }
        if (resid && a.mask) {
            const bool use = a.mask[p] != 0;
            const double rv = use ? (m1 - (double)a.vo[p]) * a.iev[p] : 0.0;
            const double rs = use ? (m2 - (double)a.so[p]) * a.ies[p] : 0.0;
            resid[p] = valid ? rv : __builtin_nan("");
            resid[npix + p] = valid ? rs : __builtin_nan("");
        }
    }
}

size_t eval_small_lds_bytes(int EX, int EY, int ny)
{
    return sizeof(double) * ((size_t)3 * EX * EY + (size_t)ny * EX);
}

bool eval_small_ok(const PsfArgs &a, int u, bool fft, size_t max_lds)
{
    return !fft && u == 1 && a.TXd == 32 && a.TYd == 32 && a.hp <= kMaxFastHalo &&
           (int64_t)a.nx * a.ny <= 1024 * kSmallPix &&
           eval_small_lds_bytes(a.EX, a.EY, a.ny) <= max_lds;
}

hipError_t launch_eval_small(const double *params, const double *wz, int NZE, int rc, double dvf,
                             double vf0, double inv_dvf, float zedge_lo, float zedge_hi,
                             const PsfArgs &a, int B, hipStream_t s)
{
    hipLaunchKernelGGL(k_eval_small, dim3(B), dim3(1024), eval_small_lds_bytes(a.EX, a.EY, a.ny),
                       s, params, wz, NZE, rc, dvf, vf0, inv_dvf, zedge_lo, zedge_hi, a);
    return hipGetLastError();
}

// Row pointers of a ragged multi-model launch over one bucket of rows.
__device__ __forceinline__ RowPtrs multi_row(const ModelDev *md, const RowMap &rm,
                                             const BucketMap &bk, const double *T,
                                             const double *consts, double *resid,
                                             double *partial, PsfArgs &a)
{
    const int i = find_row(bk.tile_base, bk.n, blockIdx.x);
    const int b = bk.rows[i];
    a = md[rm.row_model[b]].psf;
    RowPtrs r;
    r.tile = blockIdx.x - bk.tile_base[i];
    r.T = T + rm.T_off[b];
    r.c = consts + (size_t)b * NCONST;
    r.maps = nullptr;
    r.resid = resid ? resid + rm.resid_off[b] : nullptr;
    r.partial = partial ? partial + rm.part_off[b] + r.tile : nullptr;
    return r;
}

__global__ __launch_bounds__(256) void k_psf_generic_multi(const ModelDev *md, RowMap rm,
                                                           BucketMap bk, const double *T,
                                                           const double *consts, double *resid,
                                                           double *partial)
{
    PsfArgs a;
    const RowPtrs r = multi_row(md, rm, bk, T, consts, resid, partial, a);
    psf_generic_tile(a, r);
}

template <int HP>
__global__ __launch_bounds__(256) void k_psf_u1_multi(const ModelDev *md, RowMap rm, BucketMap bk,
                                                      const double *T, const double *consts,
                                                      double *resid, double *partial)
{
    PsfArgs a;
    const RowPtrs r = multi_row(md, rm, bk, T, consts, resid, partial, a);
    psf_yx_tile<HP>(a, r);
}

template <int HP, int TX> void launch_u1(const PsfArgs &a, dim3 grid, size_t lds, hipStream_t s)
{
    launch(k_psf_moments_u1<HP, TX>, grid, dim3(256), lds, s, a);
}

using LaunchFn = void (*)(const PsfArgs &, dim3, size_t, hipStream_t);
template <int TX, int... H> constexpr auto make_u1_table(std::integer_sequence<int, H...>)
{
    return std::array<LaunchFn, sizeof...(H)>{&launch_u1<H, TX>...};
}
static const auto kU1Table32 = make_u1_table<32>(std::make_integer_sequence<int, kMaxFastHalo + 1>{});
static const auto kU1Table64 = make_u1_table<64>(std::make_integer_sequence<int, kMaxFastHalo + 1>{});

// ---------------------------------------------------------------------------
// k_reduce_chi2: one wave per evaluation, fixed order
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(64) void k_reduce_chi2(const double *__restrict__ partial, int ntiles,
                                                    const double *__restrict__ consts,
                                                    int64_t nvalid_obs, double *__restrict__ chi2,
                                                    int64_t *__restrict__ nvalid)
{
    const int b = blockIdx.x, lane = threadIdx.x;
    double s = 0.0;
    for (int t = lane; t < ntiles; t += 64) s += partial[(size_t)b * ntiles + t];
    for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o, 64);
    if (lane == 0) {
        const bool valid = consts[(size_t)b * NCONST + C_VALID] != 0.0;
        chi2[b] = valid ? s : __builtin_inf();
        if (nvalid) nvalid[b] = valid ? nvalid_obs : 0;
    }
}

__global__ __launch_bounds__(64) void k_reduce_chi2_multi(const double *__restrict__ partial,
                                                          const ModelDev *__restrict__ md,
                                                          RowMap rm,
                                                          const double *__restrict__ consts,
                                                          double *__restrict__ chi2)
{
    const int b = blockIdx.x, lane = threadIdx.x;
    const ModelDev &m = md[rm.row_model[b]];
    const int ntiles = m.psf.ntiles;
    const double *pp = partial + rm.part_off[b];
    double s = 0.0;
    for (int t = lane; t < ntiles; t += 64) s += pp[t];
    for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o, 64);
    if (lane == 0) chi2[b] = consts[(size_t)b * NCONST + C_VALID] != 0.0 ? s : __builtin_inf();
}

// ---------------------------------------------------------------------------
// launch wrappers
// ---------------------------------------------------------------------------
template <int HP> void launch_u1_multi(const ModelDev *md, const RowMap &rm, const BucketMap &bk,
                                       int nblocks, const double *T, const double *consts,
                                       double *resid, double *partial, size_t lds, hipStream_t s)
{
    hipLaunchKernelGGL(k_psf_u1_multi<HP>, dim3(nblocks), dim3(256), lds, s, md, rm, bk, T, consts,
                       resid, partial);
}
using MultiFn = void (*)(const ModelDev *, const RowMap &, const BucketMap &, int, const double *,
                         const double *, double *, double *, size_t, hipStream_t);
template <int... H> constexpr auto make_multi_table(std::integer_sequence<int, H...>)
{
    return std::array<MultiFn, sizeof...(H)>{&launch_u1_multi<H>...};
}
static const auto kU1MultiTable = make_multi_table(std::make_integer_sequence<int, kMaxFastHalo + 1>{});

hipError_t launch_prep_multi(const double *params, int B, const int *row_model, const ModelDev *md,
                             double *consts, hipStream_t s)
{
    hipLaunchKernelGGL(k_prep_multi, dim3((B + 63) / 64), dim3(64), 0, s, params, B, row_model, md,
                       consts);
    return hipGetLastError();
}

hipError_t launch_line_sums_multi(const double *consts, const ModelDev *md, const RowMap &rm,
                                  int nblocks, double *T, hipStream_t s)
{
    hipLaunchKernelGGL(k_line_sums_multi, dim3(nblocks), dim3(256), 0, s, consts, md, rm, T);
    return hipGetLastError();
}

hipError_t launch_psf_multi(int fast_hp, const ModelDev *md, const RowMap &rm, const BucketMap &bk,
                            int nblocks, const double *T, const double *consts, double *resid,
                            double *partial, size_t lds, hipStream_t s)
{
    if (fast_hp >= 0)
        kU1MultiTable[fast_hp](md, rm, bk, nblocks, T, consts, resid, partial, lds, s);
    else
        hipLaunchKernelGGL(k_psf_generic_multi, dim3(nblocks), dim3(256), lds, s, md, rm, bk, T,
                           consts, resid, partial);
    return hipGetLastError();
}

hipError_t launch_reduce_multi(const double *partial, const ModelDev *md, const RowMap &rm,
                               const double *consts, double *chi2, int B, hipStream_t s)
{
    hipLaunchKernelGGL(k_reduce_chi2_multi, dim3(B), dim3(64), 0, s, partial, md, rm, consts, chi2);
    return hipGetLastError();
}
hipError_t launch_prep(const double *params, int B, int rc, double dvf, int hp, int u,
                       double vf0, double inv_dvf, double *consts, hipStream_t s)
{
    launch(k_prep, dim3((B + 63) / 64), dim3(64), 0, s, params, B, rc, dvf, hp, u, vf0, inv_dvf,
           consts);
    return hipGetLastError();
}

hipError_t launch_line_sums(const double *consts, const double *wz, int NZE, int EX, int EY,
                            int hp, int u, int rc, double vf0, double inv_dvf, float zedge_lo,
                            float zedge_hi, double *T, unsigned long long *support_count, int B,
                            hipStream_t s)
{
    dim3 grid((EX + 15) / 16, (EY + 15) / 16, B);
    launch(k_line_sums, grid, dim3(256), 0, s, consts, wz, NZE, EX, EY, hp, u, rc, vf0, inv_dvf,
           zedge_lo, zedge_hi, T, support_count);
    return hipGetLastError();
}

hipError_t launch_psf_moments(const PsfArgs &a, int B, size_t lds_bytes, hipStream_t s)
{
    dim3 grid(a.ntiles, B);
    if (a.u == 1 && a.TXd == 64 && a.TYd == 32 && a.hp <= kMaxFastHalo)
        kU1Table64[a.hp](a, grid, lds_bytes, s);
    else if (a.u == 1 && a.TXd == 32 && a.TYd == 32 && a.hp <= kMaxFastHalo)
        kU1Table32[a.hp](a, grid, lds_bytes, s);
    else
        launch(k_psf_moments, grid, dim3(256), lds_bytes, s, a);
    return hipGetLastError();
}

hipError_t launch_reduce_chi2(const double *partial, int ntiles, const double *consts,
                              int64_t nvalid_obs, double *chi2, int64_t *nvalid, int B,
                              hipStream_t s)
{
    launch(k_reduce_chi2, dim3(B), dim3(64), 0, s, partial, ntiles, consts, nvalid_obs,
                       chi2, nvalid);
    return hipGetLastError();
}

}  // namespace gbk
