// gbk_fft.hip -- FFT path of the spatial PSF convolution (eq. 9 with the
// FFT extent of eq. 10) for PSFs too wide for the direct passes.
//
// The moment planes T_j (see gbk_kernels.hip) are convolved with the
// separable PSF one axis at a time.  A line of length E (the window plus its
// halo) is zero-padded to P = 2^ceil(log2 E); the circular convolution of
// length P then equals the "valid" linear convolution on the outputs h..E-1-h
// (no wrapped term reaches them because P >= E).  Two real lines share one
// complex FFT (the PSF spectrum is real, so their results stay in the real
// and imaginary parts).  Transform: decimation in frequency (natural in,
// bit-reversed out), product with the spectrum stored in bit-reversed order,
// decimation in time back (bit-reversed in, natural out); all in FP64 in LDS.
// The y pass also forms the u x u block sums, the moments (Sec. 2.2.5) and
// the chi-square terms (eq. 11) with the same formulas as the direct path.
#include <hip/hip_runtime.h>

#include "gbk_internal.h"

namespace gbk {

namespace {

__device__ inline double2 cmul(double2 a, double2 b)
{
    return double2{a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}

// Copies the twiddles (P/2) and the spectrum (P) of a line length into LDS
// (tw_s, kb_s); the caller synchronises before use.
__device__ inline void stage_tables(int P, const double2 *__restrict__ tw, const double *__restrict__ kbr,
                                    double2 *tw_s, double *kb_s)
{
    for (int i = threadIdx.x; i < P / 2; i += blockDim.x) tw_s[i] = tw[i];
    for (int i = threadIdx.x; i < P; i += blockDim.x) kb_s[i] = kbr[i];
}

// In-place convolution of NL complex lines of length P = 2^logP in LDS, with
// the twiddles and the spectrum also in LDS.
__device__ void fft_convolve(double2 *x, int NL, int P, int logP, const double2 *tw,
                             const double *kbr)
{
    const int hP = P >> 1, nb = NL * hP;
    for (int len = P, stride = 1; len >= 2; len >>= 1, stride <<= 1) {
        const int half = len >> 1;
        for (int t = threadIdx.x; t < nb; t += blockDim.x) {
            const int line = t >> (logP - 1), k = t & (hP - 1);
            const int j = k & (half - 1), b = 2 * (k - j);
            double2 *xl = x + line * P;
            const double2 u = xl[b + j], v = xl[b + j + half];
            xl[b + j] = double2{u.x + v.x, u.y + v.y};
            xl[b + j + half] = cmul(double2{u.x - v.x, u.y - v.y}, tw[j * stride]);
        }
        __syncthreads();
    }
    for (int i = threadIdx.x; i < NL * P; i += blockDim.x) {
        const double k = kbr[i & (P - 1)];
        x[i].x *= k;
        x[i].y *= k;
    }
    __syncthreads();
    for (int len = 2, stride = hP; len <= P; len <<= 1, stride >>= 1) {
        const int half = len >> 1;
        for (int t = threadIdx.x; t < nb; t += blockDim.x) {
            const int line = t >> (logP - 1), k = t & (hP - 1);
            const int j = k & (half - 1), b = 2 * (k - j);
            double2 *xl = x + line * P;
            const double2 w = tw[j * stride];
            const double2 u = xl[b + j], v = cmul(xl[b + j + half], double2{w.x, -w.y});
            xl[b + j] = double2{u.x + v.x, u.y + v.y};
            xl[b + j + half] = double2{u.x - v.x, u.y - v.y};
        }
        __syncthreads();
    }
}

// grid (ceil(ceil(3 EY / 2) / NLX), B): complex line q holds the real lines
// 2q and 2q + 1 of the row's 3 EY lines (line l = plane l / EY, row l % EY)
__global__ __launch_bounds__(256) void k_fft_x(FftArgs f)
{
    extern __shared__ double2 sx[];
    double2 *tw_s = sx + (size_t)f.NLX * f.PX;
    double *kb_s = reinterpret_cast<double *>(tw_s + f.PX / 2);
    stage_tables(f.PX, f.twx, f.kbx, tw_s, kb_s);
    const int b = blockIdx.y, nreal = 3 * f.EY;
    const int q0 = blockIdx.x * f.NLX;
    const int NL = min(f.NLX, (nreal + 1) / 2 - q0);
    const double *T = f.T + (size_t)b * nreal * f.EX;
    double *U = f.U + (size_t)b * nreal * f.NXF;
    for (int i = threadIdx.x; i < NL * f.PX; i += blockDim.x) {
        const int ql = i >> f.logPX, x = i & (f.PX - 1);
        const int l0 = 2 * (q0 + ql), l1 = l0 + 1;
        double re = 0.0, im = 0.0;
        if (x < f.EX) {
            re = T[(size_t)l0 * f.EX + x];
            if (l1 < nreal) im = T[(size_t)l1 * f.EX + x];
        }
        sx[i] = double2{re, im};
    }
    __syncthreads();
    fft_convolve(sx, NL, f.PX, f.logPX, tw_s, kb_s);
    for (int i = threadIdx.x; i < NL * f.NXF; i += blockDim.x) {
        const int ql = i / f.NXF, X = i - ql * f.NXF;
        const int l0 = 2 * (q0 + ql), l1 = l0 + 1;
        const double2 v = sx[ql * f.PX + X + f.hp];
        U[(size_t)l0 * f.NXF + X] = v.x;
        if (l1 < nreal) U[(size_t)l1 * f.NXF + X] = v.y;
    }
}

// grid (ncb, B): block c takes data columns [c DC, c DC + DC), i.e. CW = u DC
// fine columns of the three planes (3 CW real columns, paired into complex
// lines of length PY), convolves them along y, then makes the data pixels.
__global__ __launch_bounds__(256) void k_fft_y_moments(FftArgs f, PsfArgs a)
{
    extern __shared__ double2 sy[];
    const int b = blockIdx.y, cb = blockIdx.x, u = a.u;
    const int CW = u * f.DC, nreal = 3 * CW, nlc = (nreal + 1) / 2;
    double2 *tw_s = sy + (size_t)nlc * f.PY;
    double *kb_s = reinterpret_cast<double *>(tw_s + f.PY / 2);
    stage_tables(f.PY, f.twy, f.kby, tw_s, kb_s);
    const int xd0 = cb * f.DC, X0 = xd0 * u;
    const double *U = f.U + (size_t)b * 3 * f.EY * f.NXF;
    const double *cbp = a.consts + (size_t)b * NCONST;
    const bool valid = cbp[C_VALID] != 0.0;
    double *sr = reinterpret_cast<double *>(sy);
    // real column L (plane L / CW, fine column X0 + L % CW) -> complex line L / 2, part L % 2
    for (int i = threadIdx.x; i < 2 * nlc * f.PY; i += blockDim.x) {
        const int y = i / (2 * nlc), L = i - y * (2 * nlc);
        double v = 0.0;
        if (L < nreal && y < f.EY) {
            const int j = L / CW, X = X0 + (L - j * CW);
            if (X < f.NXF) v = U[((size_t)j * f.EY + y) * f.NXF + X];
        }
        sr[2 * ((L >> 1) * f.PY + y) + (L & 1)] = v;
    }
    __syncthreads();
    fft_convolve(sy, nlc, f.PY, f.logPY, tw_s, kb_s);

    double acc = 0.0;
    const double inv_uu = 1.0 / ((double)u * u);
    const size_t npix = (size_t)a.nx * a.ny;
    for (int pix = threadIdx.x; pix < f.DC * a.ny; pix += blockDim.x) {
        const int xl = pix % f.DC, yd = pix / f.DC, xd = xd0 + xl;
        if (xd >= a.nx) continue;
        double S[3];
        for (int j = 0; j < 3; ++j) {
            double s = 0.0;
            for (int ay = 0; ay < u; ++ay)
                for (int ax = 0; ax < u; ++ax) {
                    const int L = j * CW + xl * u + ax, Y = yd * u + ay + f.hp;
                    s += sr[2 * ((L >> 1) * f.PY + Y) + (L & 1)];
                }
            S[j] = s;
        }
        const size_t p = (size_t)yd * a.nx + xd;
        double m0, m1, m2;
        if (!valid) {
            m0 = m1 = m2 = __builtin_nan("");
        } else {
            moment_maps(S[0] * inv_uu, S[1] * inv_uu, S[2] * inv_uu, a.dv, a.vref, cbp[C_VSYS], m0,
                        m1, m2);
        }
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
            if (use) acc += chi2_term(rv, rs);
            if (a.resid) {
                double *rb = a.resid + (size_t)b * 2 * npix;
                rb[p] = valid ? rv : __builtin_nan("");
                rb[npix + p] = valid ? rs : __builtin_nan("");
            }
        }
    }
    if (a.partial) {
        for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o, 64);
        __shared__ double wsum[4];
        if ((threadIdx.x & 63) == 0) wsum[threadIdx.x >> 6] = acc;
        __syncthreads();
        if (threadIdx.x == 0)
            a.partial[(size_t)b * f.ncb + cb] = ((wsum[0] + wsum[1]) + wsum[2]) + wsum[3];
    }
}

}  // namespace

// lines, then P/2 twiddles and P spectrum values
size_t fft_x_lds_bytes(const FftArgs &f)
{
    return sizeof(double2) * ((size_t)f.NLX * f.PX + f.PX / 2) + sizeof(double) * f.PX;
}

size_t fft_y_lds_bytes(const FftArgs &f, int u)
{
    return sizeof(double2) * ((size_t)((3 * u * f.DC + 1) / 2) * f.PY + f.PY / 2) +
           sizeof(double) * f.PY;
}

hipError_t launch_fft_x(const FftArgs &f, int B, hipStream_t s)
{
    const int nlc = (3 * f.EY + 1) / 2;
    dim3 grid((nlc + f.NLX - 1) / f.NLX, B);
    launch(k_fft_x, grid, dim3(256), fft_x_lds_bytes(f), s, f);
    return hipGetLastError();
}

hipError_t launch_fft_y_moments(const FftArgs &f, const PsfArgs &a, int B, hipStream_t s)
{
    dim3 grid(f.ncb, B);
    launch(k_fft_y_moments, grid, dim3(256), fft_y_lds_bytes(f, a.u), s, f, a);
    return hipGetLastError();
}

}  // namespace gbk
