// gbk_internal.h -- private declarations shared by the kernels and the
// runtime of libgbk.so (not part of the C ABI).
#pragma once
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace gbk {

// Timing of the launches made through launch(): while events are set, each
// launch carries them itself (the start event takes the time its dispatch
// begins, the stop event the time it ends), so no marker packets sit between
// the kernels of a timed chain.  A launch consumes the start event; the stop
// event stays set, so the last launch of a multi-kernel stage ends it.
struct LaunchEvents {
    hipEvent_t start = nullptr, stop = nullptr;
};
inline LaunchEvents &launch_events()
{
    static thread_local LaunchEvents ev;
    return ev;
}

template <typename F, typename... A>
inline void launch(F kernel, dim3 grid, dim3 block, size_t lds, hipStream_t s, A... args)
{
    LaunchEvents &ev = launch_events();
    if (ev.start || ev.stop) {
        hipExtLaunchKernelGGL(kernel, grid, block, (uint32_t)lds, s, ev.start, ev.stop, 0u, args...);
        ev.start = nullptr;
    } else {
        hipLaunchKernelGGL(kernel, grid, block, lds, s, args...);
    }
}

// parameter slots of a row (same order as the public enum)
enum { P_XO = 0, P_YO, P_PA, P_INC, P_VSYS, P_VT, P_RT, P_SIG, P_R0, P_I0, P_A, P_G, NPAR };
enum { RC_ARCTAN = 0, RC_EPINAT = 1, RC_BOISSIER = 2 };

// per-row constants written by k_prep (FP64)
enum {
    C_XO = 0, C_YO, C_SPA, C_CPA, C_SECI, C_SINI, C_VSYS, C_VT, C_IRT, C_IR0, C_LOG2AMP, C_KAPPA,
    C_A, C_G, C_VALID, C_ZSPAN, C_SQK, C_Q, C_VTSINI, C_XEX, C_XEY, C_XE0, C_YEX, C_YEY, C_YE0,
    // for the line-sum kernel: two FP32 values packed in one slot each (read
    // straight from scalar registers), the line centre at zero projected
    // rotation in fine halo channels, and the brightness exponent's factor
    C_F32A,  // {1 / r_t, V_t sin i / fine channel width}
    C_F32B,  // {channel span of the 2^-40 support, 0}
    C_ZC0,   // (Vsys - v(first fine halo channel)) / fine channel width
    C_IR0L,  // log2(e) / r0
    NCONST
};

// A fine channel further than sqrt(kZSpanLog2 / kappa) from the line centre
// carries less than 2^-kZSpanLog2 of the line peak and is skipped: the mass
// dropped is below 1e-12 of the line, far under what the moment maps resolve.
constexpr double kZSpanLog2 = 40.0;

// data pixels handled by one thread of k_psf_moments (tile <= 256 * this)
constexpr int kMaxPixPerThread = 4;

// largest PSF half-width (fine pixels) of the register-blocked u = 1 kernel
constexpr int kMaxFastHalo = 16;
// LDS row stride (doubles) of the register-blocked kernels: n rounded up to
// 1 (mod 4), which spreads the lanes of a register-blocked pass over all banks
constexpr int pad_stride(int n) { return n + ((1 - n) % 4 + 4) % 4; }
// dynamic LDS (bytes) of the 32 x 32 u = 1 kernel at PSF half-width hp: the
// y-pass rows of one plane
constexpr size_t yx_lds_bytes(int hp) { return sizeof(double) * 32 * (size_t)pad_stride(32 + 2 * hp); }
// Fine channels with the LSF halo (NZE) a model may have: the line-sum kernel
// packs a wave's channel range into two 16-bit fields of values up to NZE + 1.
constexpr int kMaxFineChannels = 65534;

// One pixel's chi-square term of eq. 11 from its weighted residuals,
// rounded as fma(rv, rv, rs^2) in every kernel: the compiler's own
// contraction of rv^2 + rs^2 can differ between inlined copies, and paths
// that share a tile order must agree bit for bit.
__device__ inline double chi2_term(double rv, double rs) { return __builtin_fma(rv, rv, rs * rs); }

// Moment maps of one pixel (Sec. 2.2.5) from its sums s0 = sum C, s1 =
// sum C vrel, s2 = sum C vrel^2 (vrel: channel velocity minus vref):
// m0 = dv s0, m1 = vref + s1/s0, m2 = sqrt(max(s2/s0 - (s1/s0)^2, 0)); a pixel
// without flux gives (0, vsys, 0).  1/s0 and the square root come from the
// hardware reciprocal and reciprocal square root, each refined by one Newton
// step (relative error ~1e-16); a variance below 2^-1000 gives m2 = 0.
__device__ inline void moment_maps(double s0, double s1, double s2, double dv, double vref,
                                   double vsys, double &m0, double &m1, double &m2)
{
    if (s0 > 0.0) {
        double inv = __builtin_amdgcn_rcp(s0);
        inv = fma(inv, fma(-s0, inv, 1.0), inv);
        const double mr = s1 * inv;
        m0 = dv * s0;
        m1 = vref + mr;
        const double var = s2 * inv - mr * mr;
        const double r = __builtin_amdgcn_rsq(var);
        double sd = var * r;
        sd = fma(fma(-sd, sd, var), 0.5 * r, sd);
        m2 = var > 0x1p-1000 ? sd : 0.0;
    } else {
        m0 = 0.0;
        m1 = vsys;
        m2 = 0.0;
    }
}

struct PsfArgs {
    const double *T;       // [B][3][EY][EX]
    const double *consts;  // [B][NCONST]
    const double *kp;      // PSF taps, 2hp+1
    int hp, u, nx, ny, EX, EY;
    int TXd, TYd, ntx, ntiles;
    double dv, vref;
    // observation (mask == nullptr: no observation, no chi2 or residuals)
    const uint8_t *mask;
    const float *vo, *so;
    const double *iev, *ies;
    // outputs (nullable)
    float *maps;      // [B][3][ny][nx]
    double *resid;    // [B][2][ny][nx]
    double *partial;  // [B][ntiles]
};

// Per-row pointers of one (row, tile) of the PSF/moment pass.
struct RowPtrs {
    const double *T;   // the row's three T planes
    const double *c;   // the row's constants
    float *maps;       // [3][ny][nx] of the row, or NULL
    double *resid;     // [2][ny][nx] of the row, or NULL
    double *partial;   // this tile's chi2 partial, or NULL
    int tile;
};

// Device-resident description of one model for ragged multi-model launches.
struct ModelDev {
    PsfArgs psf;            // per-model fields of the PSF/moment pass (row pointers unused)
    const double *wz;       // channel weight table [NZE][4]
    int NZE, EX, EY, hp, u, rc;
    double dvf, inv_dvf, vf0;
    float zedge_lo, zedge_hi;  // see gk_model::zedge_lo
    int64_t nvalid;         // unmasked pixels of the observation
    int fast_hp;            // >= 0: register-blocked u = 1 kernel with this half-width; -1: generic
    int lds_bytes;          // dynamic LDS of its PSF/moment kernel
    int vfield;             // velocity-field strategy: psf.ntiles = k_vfield tiles, no T planes
    int use_sig;            // its observation has a dispersion term
};

// Ragged rows of a multi-model launch (device arrays).
struct RowMap {
    const int *row_model;    // [B] model index of each row
    const int64_t *T_off;    // [B] offset of the row's T planes (doubles)
    const int *ls_base;      // [B + 1] prefix sum of line-sum tiles
    const int64_t *part_off; // [B] offset of the row's chi2 partials
    const int64_t *resid_off;// [B] offset of the row's residual maps, or NULL
    int B;
};

// Rows of one PSF-kernel bucket (same kernel variant) and their tile prefix sums.
struct BucketMap {
    const int *rows;       // [n] row indices
    const int *tile_base;  // [n + 1]
    int n;
};

hipError_t launch_prep_multi(const double *params, int B, const int *row_model, const ModelDev *md,
                             double *consts, hipStream_t s);
hipError_t launch_line_sums_multi(const double *consts, const ModelDev *md, const RowMap &rm,
                                  int nblocks, double *T, hipStream_t s);
hipError_t launch_psf_multi(int fast_hp, const ModelDev *md, const RowMap &rm, const BucketMap &bk,
                            int nblocks, const double *T, const double *consts, double *resid,
                            double *partial, size_t lds, hipStream_t s);
hipError_t launch_reduce_multi(const double *partial, const ModelDev *md, const RowMap &rm,
                               const double *consts, double *chi2, int B, hipStream_t s);

hipError_t launch_prep(const double *params, int B, int rc, double dvf, int hp, int u,
                       double vf0, double inv_dvf, double *consts, hipStream_t s);
hipError_t launch_line_sums(const double *consts, const double *wz, int NZE, int EX, int EY,
                            int hp, int u, int rc, double vf0, double inv_dvf, float zedge_lo,
                            float zedge_hi, double *T, unsigned long long *support_count, int B,
                            hipStream_t s);
hipError_t launch_psf_moments(const PsfArgs &a, int B, size_t lds_bytes, hipStream_t s);
// One workgroup per parameter row of a small u = 1 model (32 x 32 data
// tiles, T planes in LDS): constants, line sums, PSF passes, moments, maps and
// residuals in one launch, equal to k_prep -> k_line_sums -> the 32 x 32 PSF
// pass; a.consts and a.partial are not used.
size_t eval_small_lds_bytes(int EX, int EY, int ny);
bool eval_small_ok(const PsfArgs &a, int u, bool fft, size_t max_lds);
hipError_t launch_eval_small(const double *params, const double *wz, int NZE, int rc, double dvf,
                             double vf0, double inv_dvf, float zedge_lo, float zedge_hi,
                             const PsfArgs &a, int B, hipStream_t s);

// FFT path of the spatial convolution (gbk_fft.hip): k_fft_x convolves every
// line of the T planes along x into U [B][3][EY][NXF]; k_fft_y_moments
// convolves columns of U along y and forms block sums, moments and chi2
// partials [B][ncb] (one per block of DC data columns).
struct FftArgs {
    const double *T;      // [B][3][EY][EX]
    double *U;            // [B][3][EY][NXF]
    int EX, EY, NXF, hp;
    int PX, PY, logPX, logPY;
    int NLX;              // complex lines per k_fft_x block
    int DC, ncb;          // data columns per k_fft_y_moments block, number of such blocks
    const double2 *twx, *twy;  // exp(-2 pi i k / P), k < P / 2
    const double *kbx, *kby;   // PSF spectra / P, bit-reversed order
};
size_t fft_x_lds_bytes(const FftArgs &f);
size_t fft_y_lds_bytes(const FftArgs &f, int u);
hipError_t launch_fft_x(const FftArgs &f, int B, hipStream_t s);
hipError_t launch_fft_y_moments(const FftArgs &f, const PsfArgs &a, int B, hipStream_t s);
hipError_t launch_reduce_chi2(const double *partial, int ntiles, const double *consts,
                              int64_t nvalid_obs, double *chi2, int64_t *nvalid, int B,
                              hipStream_t s);

// Normal equations of Levenberg-Marquardt over ng fits at once (gbk_fit.hip).
// Fit g's residual rows start at goff[g] (device), all of one stride
// (goff[g+1] - goff[g]) / (1 + 2 nf), of which the first n_g = nused[g] entries
// enter the sums (nused NULL: the whole stride; the fitters leave out the
// dispersion half when the observation does not weigh it): row 0 is the point's residual vector,
// rows 1 + 2a and 2 + 2a its plus and minus rows for free slot a, and
// J_a = (R[1 + 2a] - R[2 + 2a]) scale[g * NPAR + a] (device).  out [ng][nblk],
// nblk = nf (nf + 1) / 2 + nf + 1: (J^T J)[a][b] for a <= b in row order,
// then J^T r, then r.r.  Rows of up to 16384 entries form one chunk, longer
// ones chunks of 4096.  When every fit of a launch has one chunk, one
// workgroup per (fit, output) sums its products over the whole rows; otherwise
// a first pass reads every residual row once, one workgroup per (fit, chunk)
// forming all outputs, into partials [ng][nchunk][nblk], and a second pass
// adds each fit's chunk partials in chunk order.  In both, thread t sums
// entries t, t + 256, ... of a chunk in order, then the lanes by butterfly and
// the four waves in order, so a fit's sums depend on its row length only, not
// on the variant or on which fits share the launch.
__host__ __device__ inline int lm_chunk_len(int64_t n)
{
    return n <= 16384 ? (int)(((n + 255) / 256) * 256 < 256 ? 256 : ((n + 255) / 256) * 256) : 4096;
}
__host__ __device__ inline int lm_normal_chunks(int64_t n)
{
    const int c = lm_chunk_len(n);
    return (int)((n + c - 1) / c);
}
hipError_t launch_lm_normal(const double *R, const int64_t *goff, const int64_t *nused,
                            const double *scale, int ng, int nf, int nchunk, double *partial,
                            double *out, hipStream_t s);

// Velocity-field strategy (gbk_vfield.hip): eq. 8 per data pixel and the
// chi-square terms of eq. 11, no cube.  A block covers kVfTile consecutive
// pixels (kVfPixPerThread per thread) for up to kVfMaxRowsPerBlock rows.
constexpr int kVfPixPerThread = 4;
constexpr int kVfTile = 256 * kVfPixPerThread;
constexpr int kVfMaxRowsPerBlock = 64;
struct VfArgs {
    const double *params;  // [B][NPAR] (device)
    const double *consts;  // [B][NCONST] from k_prep with u = 1, hp = 0
    int rc, nx, ny, B;
    int ntiles;            // ceil(nx * ny / kVfTile)
    int rows_per_block;    // 1..kVfMaxRowsPerBlock
    bool use_sig;          // the observation has a dispersion term (W > 0)
    // observation (mask == nullptr: none)
    const uint8_t *mask;
    const float *vo, *so;
    const double *iev, *ies;
    // outputs (nullable)
    float *maps;      // [B][3][ny][nx]: brightness, velocity, dispersion
    double *resid;    // [B][2][ny][nx]
    double *partial;  // [B][ntiles]
};
int vfield_rows_per_block(int ntiles, int B);
hipError_t launch_vfield(const VfArgs &a, hipStream_t s);
// Ragged rows of velocity-field models (one row per workgroup): rm.ls_base
// holds the prefix sums of the rows' tiles; chi2 partials at rm.part_off,
// residuals at rm.resid_off (if resid != NULL; the dispersion map only for
// models whose observation weighs it, the fitters' use).  rc: the rotation
// curve shared by every row's model, -1 if they differ.
hipError_t launch_vfield_multi(const ModelDev *md, const RowMap &rm, int nblocks, int rc,
                               const double *params, const double *consts, double *resid,
                               double *partial, hipStream_t s);

}  // namespace gbk
