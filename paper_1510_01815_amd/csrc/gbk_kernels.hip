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
//   k_psf_moments  per (evaluation, tile): PSF x then y pass on T_j in LDS,
//                  u x u block sum, moments, masked chi-square terms (eq. 11)
//   k_reduce_chi2  per evaluation: fixed-order sum of the tile partials
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "gbk_internal.h"

namespace gbk {

constexpr double kLog2e = 1.4426950408889634074;
constexpr double kInvSqrt2Pi = 0.39894228040143267794;
constexpr double kPi = 3.14159265358979323846;

// ---------------------------------------------------------------------------
// k_prep: per-row constants (FP64) -- slot layout in gbk_internal.h
// ---------------------------------------------------------------------------
__global__ void k_prep(const double *__restrict__ params, int B, int rc, double dvf,
                       double *__restrict__ consts)
{
    int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= B) return;
    const double *p = params + (size_t)b * NPAR;
    double *c = consts + (size_t)b * NCONST;
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
    c[C_AMP] = p[P_I0] * kInvSqrt2Pi / sig;
    c[C_KAPPA] = kappa;
    c[C_A] = p[P_A];
    c[C_G] = p[P_G];
    c[C_VALID] = 1.0;
    c[C_ZSPAN] = sqrt(kZSpanLog2 / kappa);
    c[C_SQK] = sqrt(kappa);
}

// ---------------------------------------------------------------------------
// wave-wide integer min / max (wave64, butterfly over all 64 lanes)
// ---------------------------------------------------------------------------
__device__ inline int wave_min(int v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = min(v, __shfl_xor(v, o, 64));
    return v;
}
__device__ inline int wave_max(int v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = max(v, __shfl_xor(v, o, 64));
    return v;
}

// ---------------------------------------------------------------------------
// k_line_sums: T_j for every fine spaxel of the halo-extended grid.
// grid = (ceil(EX*EY / 256), B); T layout [B][3][EY][EX] (x fastest).
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_line_sums(const double *__restrict__ consts,
                                                   const double *__restrict__ wz, int NZE, int EX,
                                                   int EY, int hp, int u, int rc, double vf0,
                                                   double inv_dvf, double *__restrict__ T,
                                                   unsigned long long *__restrict__ support_count)
{
    const int b = blockIdx.y;
    const double *c = consts + (size_t)b * NCONST;
    if (c[C_VALID] == 0.0) return;  // uniform over the block
    const int idx = blockIdx.x * 256 + threadIdx.x;
    const bool in = idx < EX * EY;
    const int xx = in ? idx % EX : 0, yy = in ? idx / EX : 0;
    const double invu = 1.0 / u;
    const double x = ((xx - hp) + 0.5) * invu - 0.5;
    const double y = ((yy - hp) + 0.5) * invu - 0.5;

    // disc geometry, eqs. 1-4
    const double dx = x - c[C_XO], dy = y - c[C_YO];
    const double xe = -dx * c[C_SPA] + dy * c[C_CPA];
    const double ye = (-dx * c[C_CPA] - dy * c[C_SPA]) * c[C_SECI];
    const double r = sqrt(xe * xe + ye * ye);
    const double costh = r > 0.0 ? xe / r : 0.0;

    // rotation curve (eqs. 6-7 or exponential rise), FP32 transcendental
    const float q = (float)(r * c[C_IRT]);
    float shape;
    if (rc == RC_ARCTAN) {
        shape = (float)(2.0 / kPi) * atanf(q);
    } else if (rc == RC_EPINAT) {
        shape = q > 0.0f ? powf(q, (float)c[C_G]) / (1.0f + powf(q, (float)c[C_A])) : 0.0f;
    } else {
        shape = -expm1f(-q);
    }
    const double vlos = c[C_VSYS] + c[C_VT] * (double)shape * c[C_SINI] * costh;  // eq. 8

    // surface brightness (eq. 5) with the exp(-60) floor, times 1/(sqrt(2 pi) sigma)
    const float rr = fminf((float)(r * c[C_IR0]), 60.0f);
    const double amp = c[C_AMP] * (double)expf(-rr);

    // line centre in fine halo-channel units, its significant range
    const double zc = (vlos - vf0) * inv_dvf;
    const double span = c[C_ZSPAN];
    // clamp in floating point first so that the integer conversion cannot overflow
    int lo = in ? (int)fmin(fmax(ceil(zc - span), 0.0), (double)NZE) : NZE;
    int hi = in ? (int)fmax(fmin(floor(zc + span), (double)(NZE - 1)), -1.0) : -1;
    const int zlo = __builtin_amdgcn_readfirstlane(wave_min(lo));
    const int zhi = __builtin_amdgcn_readfirstlane(wave_max(hi));
    if (support_count) {  // measurement only: voxels inside each lane's own support
        int n = max(hi - lo + 1, 0);
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) n += __shfl_xor(n, o, 64);
        if ((threadIdx.x & 63) == 0) atomicAdd(support_count, (unsigned long long)n);
    }

    // e = (z - zc) sqrt(kappa), so the profile is 2^(-e^2); the weights of a
    // channel are one 32-byte record {W0, W1, W2, 0} read with a scalar load
    const double sqk = c[C_SQK];
    const double4 *w = reinterpret_cast<const double4 *>(wz);
    double e = ((double)zlo - zc) * sqk;
    double t0 = 0.0, t1 = 0.0, t2 = 0.0;
#pragma unroll 2
    for (int z = zlo; z <= zhi; ++z) {
        const double g = (double)__builtin_amdgcn_exp2f(-(float)(e * e));
        const double4 wk = w[z];
        t0 = fma(g, wk.x, t0);
        t1 = fma(g, wk.y, t1);
        t2 = fma(g, wk.z, t2);
        e += sqk;
    }
    if (in) {
        const size_t plane = (size_t)EX * EY;
        double *Tb = T + (size_t)b * 3 * plane + idx;
        Tb[0] = t0 * amp;
        Tb[plane] = t1 * amp;
        Tb[2 * plane] = t2 * amp;
    }
}

// ---------------------------------------------------------------------------
// k_psf_moments: per (tile, evaluation).  Dynamic LDS:
//   sT [LY][LX]  one T_j plane of the tile plus PSF halo
//   sX [LY][TX]  after the x pass
//   sK [2hp+1]   PSF taps
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_psf_moments(PsfArgs a)
{
    extern __shared__ double lds[];
    const int b = blockIdx.y, tile = blockIdx.x, tid = threadIdx.x;
    const int tx0 = (tile % a.ntx) * a.TXd, ty0 = (tile / a.ntx) * a.TYd;
    const int u = a.u, hp = a.hp, K = 2 * hp + 1;
    const int TX = u * a.TXd, TY = u * a.TYd, LX = TX + 2 * hp, LY = TY + 2 * hp;
    double *sT = lds, *sX = lds + LY * LX, *sK = sX + LY * TX;
    const double *cb = a.consts + (size_t)b * NCONST;
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
            const double *Tj = a.T + ((size_t)b * 3 + j) * plane;
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
            const double s0 = S[0][q] * inv_uu, s1 = S[1][q] * inv_uu, s2 = S[2][q] * inv_uu;
            if (s0 > 0.0) {
                const double mr = s1 / s0;
                m0 = a.dv * s0;
                m1 = a.vref + mr;
                m2 = sqrt(fmax(s2 / s0 - mr * mr, 0.0));
            } else {
                m0 = 0.0;
                m1 = cb[C_VSYS];
                m2 = 0.0;
            }
        }
        const size_t npix = (size_t)a.nx * a.ny;
        if (a.maps) {
            float *mb = a.maps + (size_t)b * 3 * npix;
            mb[p] = (float)m0;
            mb[npix + p] = (float)m1;
            mb[2 * npix + p] = (float)m2;
        }
        if (a.mask) {
            const bool use = a.mask[p] != 0;
            const double rv = use ? (m1 - (double)a.vo[p]) * a.iev[p] : 0.0;
            const double rs = use ? (m2 - (double)a.so[p]) * a.ies[p] : 0.0;
            if (use) acc += rv * rv + rs * rs;
            if (a.resid) {
                double *rb = a.resid + (size_t)b * 2 * npix;
                rb[p] = valid ? rv : __builtin_nan("");
                rb[npix + p] = valid ? rs : __builtin_nan("");
            }
        }
    }
    if (a.partial) {
        // fixed-order block reduction: wave butterfly, then waves in order
        for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o, 64);
        __shared__ double wsum[4];
        __syncthreads();
        if ((tid & 63) == 0) wsum[tid >> 6] = acc;
        __syncthreads();
        if (tid == 0)
            a.partial[(size_t)b * a.ntiles + tile] = ((wsum[0] + wsum[1]) + wsum[2]) + wsum[3];
    }
}

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

// ---------------------------------------------------------------------------
// launch wrappers
// ---------------------------------------------------------------------------
hipError_t launch_prep(const double *params, int B, int rc, double dvf, double *consts,
                       hipStream_t s)
{
    hipLaunchKernelGGL(k_prep, dim3((B + 63) / 64), dim3(64), 0, s, params, B, rc, dvf, consts);
    return hipGetLastError();
}

hipError_t launch_line_sums(const double *consts, const double *wz, int NZE, int EX, int EY,
                            int hp, int u, int rc, double vf0, double inv_dvf, double *T,
                            unsigned long long *support_count, int B, hipStream_t s)
{
    dim3 grid((EX * EY + 255) / 256, B);
    hipLaunchKernelGGL(k_line_sums, grid, dim3(256), 0, s, consts, wz, NZE, EX, EY, hp, u, rc, vf0,
                       inv_dvf, T, support_count);
    return hipGetLastError();
}

hipError_t launch_psf_moments(const PsfArgs &a, int B, size_t lds_bytes, hipStream_t s)
{
    dim3 grid(a.ntiles, B);
    hipLaunchKernelGGL(k_psf_moments, grid, dim3(256), lds_bytes, s, a);
    return hipGetLastError();
}

hipError_t launch_reduce_chi2(const double *partial, int ntiles, const double *consts,
                              int64_t nvalid_obs, double *chi2, int64_t *nvalid, int B,
                              hipStream_t s)
{
    hipLaunchKernelGGL(k_reduce_chi2, dim3(B), dim3(64), 0, s, partial, ntiles, consts, nvalid_obs,
                       chi2, nvalid);
    return hipGetLastError();
}

}  // namespace gbk
