// gbk_mlp.hip -- learned surrogate of the velocity and dispersion maps: a
// multilayer perceptron with BF16 weights and activations, FP32 accumulation
// on the matrix cores, FP32 master weights and Adam, trained on maps that the
// plain evaluation (Sec. 2.2) streams into it.  It is not part of the paper:
// the nested sampler (Sec. 2.3.2) uses it to screen candidates.
//
//   x = encode(p)      slots x0 y0 PA i Vsys Vt rt sigma r0 I0: each mapped
//                      from its box to [-1, 1] (0 where the box is a point),
//                      PA as (cos PA, sin PA); zero padding to 32 inputs
//   h_l = gelu(h_{l-1} W_l^T + b_l)   l = 1..L, gelu(z) = z Phi(z) (erf form)
//   y = h_L W_o^T + b_o                velocity map / 300, dispersion map / 100
//   loss = sum mask (y - t)^2 / sum mask, mask: truth flux >= 1% of its peak
//
// GEMM: C[M][N] = sum_k A(m, k) B(n, k) on the 16x16x32 BF16 MFMA, each wave
// owning a grid of 16 x 16 products.  Operands are staged through LDS as
// [row][k], so each operand may be stored k-contiguous or k-strided: the
// forward product and the two backward products (data and weight gradients)
// need all of those patterns.  k-contiguous operands (the forward product)
// take a pipelined kernel with two LDS stages and 128 x 128 or 256 x 256
// tiles; the others, and narrow products, a register-staged one.
#include <hip/hip_runtime.h>

#include <cfloat>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <vector>

#include "gbk_model.h"
#include "gbk_rng.h"
#include "gbk_surrogate.h"

using namespace gbk;

typedef __bf16 bf16;
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

namespace {

constexpr int kInPad = 32;
constexpr float kVelScale = 300.0f, kSigScale = 100.0f;
constexpr int kRedBlocks = 256;
// LDS rows of a stage are padded by 16 bytes (8 bf16) beyond its K depth

// Word 3 of a raw buffer descriptor on gfx9-family chips (32-bit data format;
// no swizzle, no index stride), and a byte offset past every range used here.
constexpr int kBufferDword3 = 0x00020000;
constexpr uint32_t kOutOfRange = 0x80000000u;

enum Epi {
    EPI_F32 = 0,    // C (f32) = acc + bias
    EPI_GELU = 1,   // Z (f32, if not NULL) = acc + bias, H (bf16) = gelu(acc + bias)
    EPI_DGELU = 2,  // H (bf16) = acc * gelu'(Z)
    EPI_CHI2 = 3,   // per-row partial chi2 of (acc + bias) scaled to maps against an observation
};

// observation terms of the fused chi2 epilogue: column n < npix is the velocity
// map at pixel n, n >= npix the dispersion map at pixel n - npix (mask NULL:
// every pixel counts)
struct ObsArgs {
    const uint8_t *mask;
    const float *vo, *so;
    const double *iev, *ies;
    int npix;
    double *partial;  // [M][nparts]
    int nparts;
};

struct GemmArgs {
    const bf16 *A, *B;
    int lda, ldb;       // row strides in elements
    int M, N, K;        // K % 32 == 0
    const float *bias;  // [N] or NULL
    float *C;           // EPI_F32 output
    float *Z;           // EPI_GELU pre-activation out, EPI_DGELU pre-activation in
    bf16 *H;            // bf16 output
    int ldc;
    ObsArgs obs;
};

__device__ inline float gelu(float z) { return 0.5f * z * (1.0f + erff(z * 0.70710678118654752f)); }
__device__ inline float gelu_grad(float z)
{
    return 0.5f * (1.0f + erff(z * 0.70710678118654752f)) +
           z * expf(-0.5f * z * z) * 0.39894228040143268f;
}

// Global -> registers for one stage: the R x BK block (rows r0.., k0..) of
// X(row, k), X(row, k) = X[row * ldx + k] (TR false) or X[k * ldx + row] (TR
// true), as uint4 chunks of 8 bf16 dealt over NT threads; out-of-range
// elements are zero.
template <int R, int BK, bool TR, int NT = 256>
__device__ inline void load_stage(const uint16_t *__restrict__ X, int ldx, int rows, int K, int r0,
                                  int k0, uint4 (&reg)[R * BK / (8 * NT)], int tid)
{
#pragma unroll
    for (int i = 0; i < R * BK / (8 * NT); ++i) {
        const int c = tid + i * NT;
        if (!TR) {  // chunk = 8 consecutive k of one row
            const int row = c / (BK / 8), kc = (c % (BK / 8)) * 8;
            const bool ok = r0 + row < rows && k0 + kc < K;
            reg[i] = ok ? *reinterpret_cast<const uint4 *>(X + (size_t)(r0 + row) * ldx + k0 + kc)
                        : uint4{0u, 0u, 0u, 0u};
        } else {  // chunk = 8 consecutive rows of one k
            const int kk = c / (R / 8), rc = (c % (R / 8)) * 8;
            const uint16_t *src = X + (size_t)(k0 + kk) * ldx + r0 + rc;
            if (k0 + kk >= K) {
                reg[i] = uint4{0u, 0u, 0u, 0u};
            } else if (r0 + rc + 8 <= rows) {
                reg[i] = *reinterpret_cast<const uint4 *>(src);
            } else {
                uint16_t v[8];
#pragma unroll
                for (int j = 0; j < 8; ++j) v[j] = (r0 + rc + j < rows) ? src[j] : (uint16_t)0;
                reg[i] = *reinterpret_cast<const uint4 *>(v);
            }
        }
    }
}

// registers -> LDS S[row][k] (row stride BK + 8)
template <int R, int BK, bool TR, int NT = 256>
__device__ inline void store_stage(const uint4 (&reg)[R * BK / (8 * NT)], uint16_t *__restrict__ S, int tid)
{
    constexpr int LDK = BK + 8;
#pragma unroll
    for (int i = 0; i < R * BK / (8 * NT); ++i) {
        const int c = tid + i * NT;
        if (!TR) {
            const int row = c / (BK / 8), kc = (c % (BK / 8)) * 8;
            *reinterpret_cast<uint4 *>(S + row * LDK + kc) = reg[i];
        } else {
            const int kk = c / (R / 8), rc = (c % (R / 8)) * 8;
            const uint16_t *v = reinterpret_cast<const uint16_t *>(&reg[i]);
#pragma unroll
            for (int j = 0; j < 8; ++j) S[(rc + j) * LDK + kk] = v[j];
        }
    }
}

// Epilogue of one wave's TM x TN grid of 16 x 16 products whose first row is
// mw and first column nw.  Lane: row m = mw + 16 i + lane % 16, columns
// n = nw + 16 j + 4 (lane / 16) + r.  part: the wave's chi-square partial
// column (EPI_CHI2).
template <int TM, int TN, int EPI>
__device__ __forceinline__ void gemm_epilogue(const GemmArgs &g, const f32x4 (&acc)[TM][TN], int mw, int nw,
                                              int lane, int part)
{
    double row_chi2[TM];
#pragma unroll
    for (int i = 0; i < TM; ++i) row_chi2[i] = 0.0;
#pragma unroll
    for (int i = 0; i < TM; ++i) {
        const int m = mw + i * 16 + (lane & 15);
#pragma unroll
        for (int j = 0; j < TN; ++j) {
            const int nb = nw + j * 16 + 4 * (lane >> 4);
            if (m >= g.M || nb >= g.N) continue;
            float v[4];
#pragma unroll
            for (int r = 0; r < 4; ++r) v[r] = acc[i][j][r];
            const size_t o = (size_t)m * g.ldc + nb;
            const bool full = nb + 4 <= g.N && (g.ldc & 3) == 0;
            if (EPI == EPI_F32 || EPI == EPI_GELU || EPI == EPI_CHI2) {
                if (g.bias)
#pragma unroll
                    for (int r = 0; r < 4; ++r) v[r] += (nb + r < g.N) ? g.bias[nb + r] : 0.0f;
            }
            if (EPI == EPI_F32) {
                if (full) {
                    *reinterpret_cast<float4 *>(g.C + o) = float4{v[0], v[1], v[2], v[3]};
                } else {
                    for (int r = 0; r < 4 && nb + r < g.N; ++r) g.C[o + r] = v[r];
                }
            } else if (EPI == EPI_GELU || EPI == EPI_DGELU) {
                uint16_t hb[4];
                if (EPI == EPI_GELU) {
                    if (g.Z) {
                        if (full) {
                            *reinterpret_cast<float4 *>(g.Z + o) = float4{v[0], v[1], v[2], v[3]};
                        } else {
                            for (int r = 0; r < 4 && nb + r < g.N; ++r) g.Z[o + r] = v[r];
                        }
                    }
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        const bf16 h = (bf16)gelu(v[r]);
                        hb[r] = *reinterpret_cast<const uint16_t *>(&h);
                    }
                } else {
                    float z[4];
                    if (full) {
                        const float4 zz = *reinterpret_cast<const float4 *>(g.Z + o);
                        z[0] = zz.x, z[1] = zz.y, z[2] = zz.z, z[3] = zz.w;
                    } else {
                        for (int r = 0; r < 4; ++r) z[r] = (nb + r < g.N) ? g.Z[o + r] : 0.0f;
                    }
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        const bf16 h = (bf16)(v[r] * gelu_grad(z[r]));
                        hb[r] = *reinterpret_cast<const uint16_t *>(&h);
                    }
                }
                uint16_t *H = reinterpret_cast<uint16_t *>(g.H);
                if (full) {
                    *reinterpret_cast<uint2 *>(H + o) = *reinterpret_cast<const uint2 *>(hb);
                } else {
                    for (int r = 0; r < 4 && nb + r < g.N; ++r) H[o + r] = hb[r];
                }
            } else {  // EPI_CHI2: the maps as gk_surrogate_predict returns them (FP32 scaling)
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int n = nb + r;
                    if (n >= g.N) continue;
                    const bool vel = n < g.obs.npix;
                    const int p = vel ? n : n - g.obs.npix;
                    if (g.obs.mask && !g.obs.mask[p]) continue;
                    const float y = v[r] * (vel ? kVelScale : kSigScale);
                    const double d = ((double)y - (vel ? g.obs.vo[p] : g.obs.so[p])) *
                                     (vel ? g.obs.iev[p] : g.obs.ies[p]);
                    row_chi2[i] += d * d;
                }
            }
        }
    }
    if (EPI == EPI_CHI2) {
        // lanes l, l ^ 16, l ^ 32, l ^ 48 hold the same row: sum them, then one
        // partial per (row, block column, wave column), no atomics
#pragma unroll
        for (int i = 0; i < TM; ++i) {
            double c = row_chi2[i];
            c += __shfl_xor(c, 16, 64);
            c += __shfl_xor(c, 32, 64);
            const int m = mw + i * 16 + (lane & 15);
            if (lane < 16 && m < g.M) g.obs.partial[(size_t)m * g.obs.nparts + part] = c;
        }
    }
}

// C[M][N] = sum_k A(m, k) B(n, k) on BM x BN tiles, 4 waves of (BM/2) x (BN/2).
// The MFMA takes the B fragment as its row operand, so a lane's four results
// are four consecutive columns n of one row m (vector stores in the epilogue).
template <int BM, int BN, int BK, bool TA, bool TB, int EPI>
__global__ __launch_bounds__(256) void k_gemm(GemmArgs g)
{
    constexpr int WM = BM / 2, WN = BN / 2, TM = WM / 16, TN = WN / 16, LDK = BK + 8;
    __shared__ __attribute__((aligned(16))) uint16_t As[BM * LDK];
    __shared__ __attribute__((aligned(16))) uint16_t Bs[BN * LDK];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm = wave & 1, wn = wave >> 1;
    const int m0 = blockIdx.y * BM, n0 = blockIdx.x * BN;
    const uint16_t *A = reinterpret_cast<const uint16_t *>(g.A);
    const uint16_t *B = reinterpret_cast<const uint16_t *>(g.B);
    f32x4 acc[TM][TN];
#pragma unroll
    for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int j = 0; j < TN; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};

    // two register sets: stage s + 2 is loaded while stage s is multiplied
    constexpr int RA = BM * BK / 2048, RB = BN * BK / 2048;
    uint4 ra0[RA], rb0[RB], ra1[RA], rb1[RB];
    auto load = [&](int k0, uint4(&ra)[RA], uint4(&rb)[RB]) {
        if (k0 < g.K) {
            load_stage<BM, BK, TA>(A, g.lda, g.M, g.K, m0, k0, ra, tid);
            load_stage<BN, BK, TB>(B, g.ldb, g.N, g.K, n0, k0, rb, tid);
        }
    };
    auto multiply = [&]() {
#pragma unroll
        for (int kk = 0; kk < BK; kk += 32) {
            bf16x8 af[TM], bfr[TN];
#pragma unroll
            for (int i = 0; i < TM; ++i)
                af[i] = *reinterpret_cast<const bf16x8 *>(
                    As + (wm * WM + i * 16 + (lane & 15)) * LDK + kk + (lane >> 4) * 8);
#pragma unroll
            for (int j = 0; j < TN; ++j)
                bfr[j] = *reinterpret_cast<const bf16x8 *>(
                    Bs + (wn * WN + j * 16 + (lane & 15)) * LDK + kk + (lane >> 4) * 8);
#pragma unroll
            for (int i = 0; i < TM; ++i)
#pragma unroll
                for (int j = 0; j < TN; ++j)
                    acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(bfr[j], af[i], acc[i][j], 0, 0, 0);
        }
    };
    load(0, ra0, rb0);
    load(BK, ra1, rb1);
    for (int k0 = 0; k0 < g.K; k0 += 2 * BK) {
        store_stage<BM, BK, TA>(ra0, As, tid);
        store_stage<BN, BK, TB>(rb0, Bs, tid);
        __syncthreads();
        load(k0 + 2 * BK, ra0, rb0);
        multiply();
        __syncthreads();
        if (k0 + BK < g.K) {  // uniform
            store_stage<BM, BK, TA>(ra1, As, tid);
            store_stage<BN, BK, TB>(rb1, Bs, tid);
            __syncthreads();
            load(k0 + 3 * BK, ra1, rb1);
            multiply();
            __syncthreads();
        }
    }

    gemm_epilogue<TM, TN, EPI>(g, acc, m0 + wm * WM, n0 + wn * WN, lane, blockIdx.x * 2 + wn);
}

// C[M][N] = sum_k A(m, k) B(n, k) for k-contiguous operands of products with
// at least two 128 x 128 tiles per compute unit: BM x BN tiles, 2 x NWN waves
// of (BM / 2) x (BN / NWN); 256 x 256 tiles (8 waves of 128 x 64) for f32
// products of at least four such tiles per compute unit, where a wave reads
// 3/4 of the LDS bytes per product that a 64 x 64 wave does, else 128 x 128
// (4 waves of 64 x 64).  Two LDS stages (131,072 or 65,536 bytes)
// take one barrier per 64-deep K stage: stage s is multiplied from one buffer
// while stage s + 1 goes from registers into the other, after the first half
// of stage s's products.  Stage s + 1 was fetched into its register set during
// stage s - 1 and stage s + 2 is fetched into the other set during stage s.
// LDS rows are 64 k (128 bytes, unpadded) with the 16-byte chunk c of row r
// stored at c ^ f(r), f(r) = (r & 7) ^ ((r >> 3) & 1): the 16 rows that 16
// lanes read at one chunk then fall in 16 distinct 16-byte bank groups (and
// any 8 consecutive of them in 8), and a row's 8 chunks stay in one 128-byte
// line for the stores.
template <int BM, int BN, int NWN, int EPI>
__global__ __launch_bounds__(128 * NWN, NWN == 2 ? 2 : 1) void k_gemm_db(GemmArgs g)
{
    constexpr int BK = 64, NT = 128 * NWN, WM = BM / 2, WN = BN / NWN, RS = NT / 8;
    constexpr int TM = WM / 16, TN = WN / 16;
    static_assert(RS % 16 == 0 && BM % RS == 0 && BN % RS == 0, "tile rows per store pass");
    __shared__ __attribute__((aligned(16))) uint16_t S[2][(BM + BN) * BK];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm = wave & 1, wn = wave >> 1;
    // Workgroups reach the 8 XCDs in turn (workgroup b on XCD b % 8).  With
    // 128 x 128 tiles, XCD x takes the x-th eighth of the tiles in row-major
    // order, so the row and column panels that its L2 serves are those of a
    // compact block of tiles, not of every eighth column.  256 x 256 tiles
    // keep the launch order (every eighth column: 4 row panels by 8 column
    // panels in flight per XCD, against 1 by 32 for the eighth in row order).
    int bx = blockIdx.x, by = blockIdx.y;
    if (NWN == 2) {
        const int T = gridDim.x * gridDim.y, b = blockIdx.y * gridDim.x + blockIdx.x;
        const int q = T >> 3, r = T & 7, x = b & 7;
        const int t = x * q + min(x, r) + (b >> 3);
        bx = t % gridDim.x;
        by = t / gridDim.x;
    }
    const int m0 = by * BM, n0 = bx * BN;
    f32x4 acc[TM][TN];
#pragma unroll
    for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int j = 0; j < TN; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};

    constexpr int RA = BM / RS, RB = BN / RS;
    uint4 ra0[RA], rb0[RB], ra1[RA], rb1[RB];
    // The thread's chunks: rows (tid >> 3) + RS i, k = 8 (tid & 7) of the
    // stage.  Fetched by range-checked buffer loads with no branch, so that
    // the compiler can wait for the older of two register sets alone: rows
    // at or past M (N) lie past the descriptor's range (M lda elements) and
    // read as zero, and k past K gets an offset past that range.
    const int sr = tid >> 3;
    const __amdgpu_buffer_rsrc_t rsA =
        __builtin_amdgcn_make_buffer_rsrc((void *)g.A, 0, (int)((size_t)g.M * g.lda * 2), kBufferDword3);
    const __amdgpu_buffer_rsrc_t rsB =
        __builtin_amdgcn_make_buffer_rsrc((void *)g.B, 0, (int)((size_t)g.N * g.ldb * 2), kBufferDword3);
    const uint32_t oA = (uint32_t)(m0 + sr) * (uint32_t)g.lda * 2u + 16u * (tid & 7);
    const uint32_t oB = (uint32_t)(n0 + sr) * (uint32_t)g.ldb * 2u + 16u * (tid & 7);
    auto load = [&](int k0, uint4(&ra)[RA], uint4(&rb)[RB]) {
        const bool kin = k0 + 8 * (tid & 7) < g.K;
#pragma unroll
        for (int i = 0; i < RA; ++i)
            ra[i] = __builtin_bit_cast(uint4, __builtin_amdgcn_raw_buffer_load_b128(
                                                  rsA, kin ? oA + (uint32_t)(RS * i * g.lda + k0) * 2u : kOutOfRange, 0, 0));
#pragma unroll
        for (int i = 0; i < RB; ++i)
            rb[i] = __builtin_bit_cast(uint4, __builtin_amdgcn_raw_buffer_load_b128(
                                                  rsB, kin ? oB + (uint32_t)(RS * i * g.ldb + k0) * 2u : kOutOfRange, 0, 0));
    };
    // the thread's stores: a row's f depends on row & 15 only, the same for every i
    const int st_off = sr * BK + 8 * ((tid & 7) ^ (sr & 7) ^ ((sr >> 3) & 1));
    auto store = [&](const uint4(&ra)[RA], const uint4(&rb)[RB], int buf) {
        uint16_t *As = S[buf], *Bs = S[buf] + BM * BK;
#pragma unroll
        for (int i = 0; i < RA; ++i) *reinterpret_cast<uint4 *>(As + st_off + i * RS * BK) = ra[i];
#pragma unroll
        for (int i = 0; i < RB; ++i) *reinterpret_cast<uint4 *>(Bs + st_off + i * RS * BK) = rb[i];
    };
    // the lane's reads: row lane & 15 of each 16-row tile, chunk kk / 8 + lane / 16
    const int lr = lane & 15, gq = (lane >> 4) ^ (lr & 7) ^ ((lr >> 3) & 1);
    const int ld_off0 = lr * BK + 8 * gq, ld_off1 = lr * BK + (8 * gq ^ 32);
    auto multiply = [&](int buf, int half) {
        const uint16_t *As = S[buf] + (half ? ld_off1 : ld_off0);
        const uint16_t *Bs = S[buf] + BM * BK + (half ? ld_off1 : ld_off0);
        bf16x8 af[TM], bfr[TN];
#pragma unroll
        for (int i = 0; i < TM; ++i)
            af[i] = *reinterpret_cast<const bf16x8 *>(As + (wm * WM + i * 16) * BK);
#pragma unroll
        for (int j = 0; j < TN; ++j)
            bfr[j] = *reinterpret_cast<const bf16x8 *>(Bs + (wn * WN + j * 16) * BK);
#pragma unroll
        for (int i = 0; i < TM; ++i)
#pragma unroll
            for (int j = 0; j < TN; ++j)
                acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(bfr[j], af[i], acc[i][j], 0, 0, 0);
    };
    // Stage s: fetched into register set s & 1 during stage s - 2, stored
    // into LDS buffer s & 1 during stage s - 1, multiplied in stage s.  Fetches
    // and stores of stages past K are not skipped (they read nothing and fill
    // a buffer that is not read again): with no branch around them the
    // compiler's wait for the older register set leaves the newer in flight.
    load(0, ra0, rb0);
    load(BK, ra1, rb1);
    store(ra0, rb0, 0);
    load(2 * BK, ra0, rb0);
    __syncthreads();
    for (int k0 = 0; k0 < g.K; k0 += 2 * BK) {
        multiply(0, 0);
        store(ra1, rb1, 1);
        load(k0 + 3 * BK, ra1, rb1);
        multiply(0, 1);
        __syncthreads();
        if (k0 + BK >= g.K) break;  // uniform
        multiply(1, 0);
        store(ra0, rb0, 0);
        load(k0 + 4 * BK, ra0, rb0);
        multiply(1, 1);
        __syncthreads();
    }
    gemm_epilogue<TM, TN, EPI>(g, acc, m0 + wm * WM, n0 + wn * WN, lane, bx * NWN + wn);
}

// uniform draws of parameter rows in the box: slot s = lo_s + u (hi_s - lo_s)
// rounded once, u from Philox4x32-10 with counter (row, step, step >> 32, block)
// and the seed as key
__global__ void k_draw(uint64_t seed, uint64_t step, int B, const double *__restrict__ lo,
                       const double *__restrict__ hi, double *__restrict__ p)
{
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= B) return;
    const uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32) ^ 0x73757272u};
    uint32_t r[12];
    for (int j = 0; j < 3; ++j) {
        const uint32_t c[4] = {(uint32_t)b, (uint32_t)step, (uint32_t)(step >> 32), (uint32_t)j};
        philox4x32_10(c, key, r + 4 * j);
    }
    for (int s = 0; s < NPAR; ++s) {
        const double u = ((double)r[s] + 0.5) * 0x1.0p-32;
        // one rounding: fma(u, hi - lo, lo)
        p[(size_t)b * NPAR + s] = hi[s] > lo[s] ? fma(u, hi[s] - lo[s], lo[s]) : lo[s];
    }
}

__global__ void k_encode(const double *__restrict__ p, int B, const double *__restrict__ lo,
                         const double *__restrict__ hi, bf16 *__restrict__ x)
{
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= B) return;
    const double *r = p + (size_t)b * NPAR;
    bf16 *o = x + (size_t)b * kInPad;
    int col = 0;
    for (int s = 0; s <= P_I0; ++s) {
        if (s == P_PA) {
            const double a = r[s] * (M_PI / 180.0);
            o[col++] = (bf16)(float)cos(a);
            o[col++] = (bf16)(float)sin(a);
        } else {
            const double w = hi[s] - lo[s];
            o[col++] = (bf16)(float)(w > 0.0 ? 2.0 * (r[s] - lo[s]) / w - 1.0 : 0.0);
        }
    }
    for (; col < kInPad; ++col) o[col] = (bf16)0.0f;
}

// Targets and mask of one row per block from maps [B][3][npix]; cnt[b] = ones in the mask.
__global__ __launch_bounds__(256) void k_targets(const float *__restrict__ maps, int npix,
                                                 float *__restrict__ t, float *__restrict__ mask,
                                                 unsigned *__restrict__ cnt)
{
    const int b = blockIdx.x;
    const float *m = maps + (size_t)b * 3 * npix;
    float mx = 0.0f;
    for (int i = threadIdx.x; i < npix; i += 256) mx = fmaxf(mx, m[i]);  // NaN rows stay 0
    for (int o = 32; o > 0; o >>= 1) mx = fmaxf(mx, __shfl_xor(mx, o, 64));
    __shared__ float ws[4];
    __shared__ unsigned wc[4];
    if ((threadIdx.x & 63) == 0) ws[threadIdx.x >> 6] = mx;
    __syncthreads();
    mx = fmaxf(fmaxf(ws[0], ws[1]), fmaxf(ws[2], ws[3]));
    float *tb = t + (size_t)b * 2 * npix;
    float *mb = mask + (size_t)b * 2 * npix;
    unsigned c = 0;
    for (int i = threadIdx.x; i < npix; i += 256) {
        const float v = m[npix + i], s = m[2 * npix + i];
        const bool use = mx > 0.0f && m[i] >= 0.01f * mx && isfinite(v) && isfinite(s);
        tb[i] = use ? v / kVelScale : 0.0f;
        tb[npix + i] = use ? s / kSigScale : 0.0f;
        mb[i] = mb[npix + i] = use ? 1.0f : 0.0f;
        c += use ? 2u : 0u;
    }
    for (int o = 32; o > 0; o >>= 1) c += __shfl_xor(c, o, 64);
    if ((threadIdx.x & 63) == 0) wc[threadIdx.x >> 6] = c;
    __syncthreads();
    if (threadIdx.x == 0) cnt[b] = wc[0] + wc[1] + wc[2] + wc[3];
}

// dY = 2 mask (y - t) / count (bf16), count = sum of cnt[0..B); per-block sums of
// mask (y - t)^2 into partial[]
__global__ __launch_bounds__(256) void k_mse_grad(const float *__restrict__ y,
                                                  const float *__restrict__ t,
                                                  const float *__restrict__ mask, size_t n,
                                                  const unsigned *__restrict__ cnt, int B,
                                                  bf16 *__restrict__ dy, double *__restrict__ partial)
{
    __shared__ unsigned long long wt[4];
    __shared__ double ws[4];
    unsigned long long c = 0;
    for (int b = threadIdx.x; b < B; b += 256) c += cnt[b];
    for (int o = 32; o > 0; o >>= 1) c += __shfl_xor(c, o, 64);
    if ((threadIdx.x & 63) == 0) wt[threadIdx.x >> 6] = c;
    __syncthreads();
    const unsigned long long total = wt[0] + wt[1] + wt[2] + wt[3];
    const float scale = 2.0f / (float)(total > 0 ? total : 1);
    double acc = 0.0;
    for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (size_t)gridDim.x * 256) {
        const float r = (y[i] - t[i]) * mask[i];
        acc += (double)r * r;
        dy[i] = (bf16)(scale * r);
    }
    for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o, 64);
    if ((threadIdx.x & 63) == 0) ws[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) partial[blockIdx.x] = ((ws[0] + ws[1]) + ws[2]) + ws[3];
}

// loss = sum(partial) / count, in a fixed order
__global__ __launch_bounds__(256) void k_loss_finish(const double *__restrict__ partial, int np,
                                                     const unsigned *__restrict__ cnt, int B,
                                                     float *__restrict__ loss)
{
    __shared__ double ws[256];
    __shared__ unsigned long long wc[256];
    double a = 0.0;
    unsigned long long c = 0;
    for (int i = threadIdx.x; i < np; i += 256) a += partial[i];
    for (int b = threadIdx.x; b < B; b += 256) c += cnt[b];
    ws[threadIdx.x] = a;
    wc[threadIdx.x] = c;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (threadIdx.x < s) {
            ws[threadIdx.x] += ws[threadIdx.x + s];
            wc[threadIdx.x] += wc[threadIdx.x + s];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) *loss = (float)(ws[0] / (double)(wc[0] > 0 ? wc[0] : 1));
}

// db[n] = sum_m d[m][n] in two fixed-order passes: grid (ceil(N/256), kColChunks)
// sums chunk c of the rows into part[c][n]; k_colsum_finish adds the chunks.
constexpr int kColChunks = 32;
__global__ void k_colsum(const bf16 *__restrict__ d, int M, int N, float *__restrict__ part)
{
    const int n = blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= N) return;
    const int rows = (M + kColChunks - 1) / kColChunks, m0 = blockIdx.y * rows;
    const int m1 = min(M, m0 + rows);
    float s = 0.0f;
    for (int m = m0; m < m1; ++m) s += (float)d[(size_t)m * N + n];
    part[(size_t)blockIdx.y * N + n] = s;
}

__global__ void k_colsum_finish(const float *__restrict__ part, int N, float *__restrict__ db)
{
    const int n = blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= N) return;
    float s = 0.0f;
    for (int c = 0; c < kColChunks; ++c) s += part[(size_t)c * N + n];
    db[n] = s;
}

__global__ void k_adam(float *__restrict__ w, const float *__restrict__ g, float *__restrict__ m,
                       float *__restrict__ v, bf16 *__restrict__ wb, size_t n, float lr, float c1,
                       float c2)
{
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float gi = g[i];
    const float mi = 0.9f * m[i] + 0.1f * gi, vi = 0.999f * v[i] + 0.001f * gi * gi;
    m[i] = mi;
    v[i] = vi;
    const float wi = w[i] - lr * (mi * c1) / (sqrtf(vi * c2) + 1e-8f);
    w[i] = wi;
    if (wb) wb[i] = (bf16)wi;
}

__global__ void k_to_bf16(const float *__restrict__ a, bf16 *__restrict__ b, size_t n)
{
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) b[i] = (bf16)a[i];
}

// chi2[m] = sum of the row's epilogue partials in a fixed order (one wave
// per row: lane sums, then a butterfly); +INF for rows outside the domain
__global__ __launch_bounds__(256) void k_chi2_finish(const double *__restrict__ partial, int nparts,
                                                     int M, const double *__restrict__ params,
                                                     int rc, double *__restrict__ chi2)
{
    const int m = blockIdx.x * 4 + (threadIdx.x >> 6), lane = threadIdx.x & 63;
    if (m >= M) return;  // wave-uniform
    double c = 0.0;
    for (int j = lane; j < nparts; j += 64) c += partial[(size_t)m * nparts + j];
    for (int o = 32; o > 0; o >>= 1) c += __shfl_xor(c, o, 64);
    if (lane == 0) {
        const double *p = params + (size_t)m * NPAR;
        bool ok = true;
        for (int k = 0; k < NPAR; ++k) ok = ok && isfinite(p[k]);
        ok = ok && p[P_INC] > 0.0 && p[P_INC] < 90.0 && p[P_SIG] > 0.0 && p[P_R0] > 0.0 &&
             p[P_RT] > 0.0 && (rc != RC_EPINAT || p[P_G] > 0.0);
        chi2[m] = ok ? c : __builtin_inf();
    }
}

__global__ void k_scale_maps(const float *__restrict__ y, int npix, size_t n, float *__restrict__ maps)
{
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const size_t r = i % (2 * (size_t)npix);
    maps[i] = y[i] * (r < (size_t)npix ? kVelScale : kSigScale);
}

// Rows of the compact output layer: row j < nv is velocity pixel idx[j], row
// nv + j dispersion pixel idx[j]; one block per row.
__global__ void k_compact_rows(const bf16 *__restrict__ W, const float *__restrict__ bias, int hidden,
                               int npix, const int *__restrict__ idx, int nv, bf16 *__restrict__ Wc,
                               float *__restrict__ bc)
{
    const int j = blockIdx.x;
    const int src = j < nv ? idx[j] : npix + idx[j - nv];
    for (int k = threadIdx.x; k < hidden; k += blockDim.x)
        Wc[(size_t)j * hidden + k] = W[(size_t)src * hidden + k];
    if (threadIdx.x == 0) bc[j] = bias[src];
}

__global__ void k_compact_obs(const float *__restrict__ vo, const float *__restrict__ so,
                              const double *__restrict__ iev, const double *__restrict__ ies,
                              const int *__restrict__ idx, int nv, float *__restrict__ cvo,
                              float *__restrict__ cso, double *__restrict__ ciev,
                              double *__restrict__ cies)
{
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= nv) return;
    const int p = idx[j];
    cvo[j] = vo[p];
    cso[j] = so[p];
    ciev[j] = iev[p];
    cies[j] = ies[p];
}

bool aligned16(const void *p) { return ((uintptr_t)p & 15u) == 0; }  // NULL passes

// Tile edge for an M x N product: 128 (K stages of 64) when that still gives
// two tiles per compute unit, else 64 (K stages of 128: more, smaller tiles
// for the narrow layers, with as many products per stage).
int gemm_tile(int M, int N)
{
    const long t = (long)((M + 127) / 128) * ((N + 127) / 128);
    return t >= 512 ? 128 : 64;
}

// k_gemm_db for k-contiguous operands when every operand offset of a tile,
// rows past the end included, stays below 2^31 bytes; its 256 x 256 tiles
// when they give at least four per compute unit
bool buffer_offsets_fit(int M, int N, int lda, int ldb)
{
    return ((double)M + 256) * lda * 2 < 2147483648.0 && ((double)N + 256) * ldb * 2 < 2147483648.0;
}
bool wide_tiles(int M, int N) { return (long)((M + 255) / 256) * ((N + 255) / 256) >= 1024; }

template <bool TA, bool TB, int EPI> gk_status gemm(const GemmArgs &g, hipStream_t s)
{
    if (g.M <= 0 || g.N <= 0 || g.K <= 0 || g.K % 32 || g.lda % 8 || g.ldb % 8 ||
        !aligned16(g.A) || !aligned16(g.B) || !aligned16(g.C) || !aligned16(g.Z) || !aligned16(g.H))
        return fail(GK_EINVAL, "GEMM shape %dx%dx%d (lda %d, ldb %d) or alignment not supported",
                    g.M, g.N, g.K, g.lda, g.ldb);
    if ((TA ? g.lda < g.M : g.lda < g.K) || (TB ? g.ldb < g.N : g.ldb < g.K) ||
        (EPI != EPI_CHI2 && g.ldc < g.N))
        return fail(GK_EINVAL, "GEMM leading dimension too small");
    const int T = gemm_tile(g.M, g.N);
    const int gy = (g.M + T - 1) / T;
    if (gy > 65535) return fail(GK_EINVAL, "GEMM M = %d too large", g.M);
    dim3 grid((g.N + T - 1) / T, gy);
    if (EPI == EPI_CHI2 && g.obs.nparts != 2 * (int)grid.x)
        return fail(GK_EINVAL, "chi2 partial count mismatch");
    if constexpr (!TA && !TB && EPI != EPI_DGELU) {
        if (T == 128 && buffer_offsets_fit(g.M, g.N, g.lda, g.ldb)) {
            bool wide = false;
            if constexpr (EPI == EPI_F32) {
                if ((wide = wide_tiles(g.M, g.N)))
                    hipLaunchKernelGGL((k_gemm_db<256, 256, 4, EPI>),
                                       dim3((g.N + 255) / 256, (g.M + 255) / 256), dim3(512), 0, s, g);
            }
            if (!wide) hipLaunchKernelGGL((k_gemm_db<128, 128, 2, EPI>), grid, dim3(256), 0, s, g);
            HIP_TRY(hipGetLastError());
            return GK_OK;
        }
    }
    if (T == 128)
        hipLaunchKernelGGL((k_gemm<128, 128, 64, TA, TB, EPI>), grid, dim3(256), 0, s, g);
    else
        hipLaunchKernelGGL((k_gemm<64, 64, 128, TA, TB, EPI>), grid, dim3(256), 0, s, g);
    HIP_TRY(hipGetLastError());
    return GK_OK;
}

unsigned blocks(size_t n, unsigned t = 256) { return (unsigned)((n + t - 1) / t); }

}  // namespace

// ---------------------------------------------------------------------------
// surrogate object
// ---------------------------------------------------------------------------
struct gk_surrogate {
    gk_model *model = nullptr;  // the instrument whose plain evaluation trains the network
    int device = 0;
    uint64_t wver = 0;          // bumped whenever the weights change
    // output layer restricted to the unmasked pixels of one observation (the
    // chi2 needs no other outputs): rows of W_o and b_o for the velocity, then
    // the dispersion, of each unmasked pixel, and that pixel's observation
    const gk_model *c_model = nullptr;
    uint64_t c_gen = 0, c_wver = 0;
    int c_nv = -1;
    bf16 *c_W = nullptr;
    float *c_b = nullptr, *c_vo = nullptr, *c_so = nullptr;
    double *c_iev = nullptr, *c_ies = nullptr;
    int *c_idx = nullptr;
    gk_surrogate_opts o{};
    int npix = 0, nout = 0, layers = 0;
    double lo[NPAR]{}, hi[NPAR]{};
    double *d_lo = nullptr, *d_hi = nullptr;
    int64_t step = 0;  // Adam steps taken
    hipStream_t stream = nullptr;
    // layer l = 0..layers (the last is the output layer): W_l [out][in], b_l [out]
    std::vector<int> fin, fout;
    std::vector<float *> W, b, gW, gb, mW, vW, mb, vb;
    std::vector<bf16 *> Wb;
    // per-row buffers: the inference set (X, H, d_params, h_params, d_cpart)
    // for cap rows, the training and full-output set (Z, dH, Y, T, Mask, dY,
    // maps, cnt, d_partial, d_colpart) for tcap rows
    int cap = 0, tcap = 0;
    bf16 *X = nullptr, *dY = nullptr;
    std::vector<bf16 *> H, dH;
    std::vector<float *> Z;
    float *Y = nullptr, *T = nullptr, *Mask = nullptr, *maps = nullptr, *d_loss = nullptr;
    unsigned *cnt = nullptr;
    double *d_params = nullptr, *h_params = nullptr, *d_partial = nullptr;
    double *d_cpart = nullptr;  // [cap][2 ceil(nout / 64)] chi2 partials of the output layer
    float *d_colpart = nullptr;  // [kColChunks][max(hidden, nout)] bias-gradient partials
    hipEvent_t ev_staged = nullptr;  // recorded after the last copy out of h_params
    int loss_cap = 0;

    size_t weight_count() const
    {
        size_t n = 0;
        for (int l = 0; l <= layers; ++l) n += (size_t)fout[l] * fin[l] + fout[l];
        return n;
    }
    void free_infer()
    {
        auto F = [](void *p) { if (p) (void)hipFree(p); };
        F(X);
        for (bf16 *p : H) F(p);
        H.clear();
        F(d_params);
        F(d_cpart);
        if (h_params) {
            if (ev_staged) (void)hipEventSynchronize(ev_staged);
            (void)hipHostFree(h_params);
        }
        X = nullptr;
        d_params = h_params = d_cpart = nullptr;
        cap = 0;
    }
    void free_full()
    {
        auto F = [](void *p) { if (p) (void)hipFree(p); };
        F(dY);
        for (bf16 *p : dH) F(p);
        for (float *p : Z) F(p);
        dH.clear();
        Z.clear();
        F(Y);
        F(T);
        F(Mask);
        F(maps);
        F(cnt);
        F(d_partial);
        F(d_colpart);
        dY = nullptr;
        Y = T = Mask = maps = nullptr;
        cnt = nullptr;
        d_partial = nullptr;
        d_colpart = nullptr;
        tcap = 0;
    }
    void free_rows()
    {
        free_infer();
        free_full();
    }
    void free_compact()
    {
        for (void *p : {(void *)c_W, (void *)c_b, (void *)c_vo, (void *)c_so, (void *)c_iev,
                        (void *)c_ies, (void *)c_idx})
            if (p) (void)hipFree(p);
        c_W = nullptr;
        c_b = c_vo = c_so = nullptr;
        c_iev = c_ies = nullptr;
        c_idx = nullptr;
        c_model = nullptr;
        c_nv = -1;
    }
    void release()
    {
        if (stream) (void)hipStreamSynchronize(stream);
        free_rows();
        for (auto *v : {&W, &b, &gW, &gb, &mW, &vW, &mb, &vb})
            for (float *p : *v) (void)hipFree(p);
        for (bf16 *p : Wb) (void)hipFree(p);
        (void)hipFree(d_lo);
        (void)hipFree(d_hi);
        (void)hipFree(d_loss);
        free_compact();
        if (ev_staged) (void)hipEventDestroy(ev_staged);
        if (stream) (void)hipStreamDestroy(stream);
    }
};

namespace {

// Buffers for `rows` rows: the inference set always, the training and
// full-output set when `full`.  Capacities grow at least twofold, so a
// sampler whose batches grow round by round reallocates a few times only.
gk_status reserve_rows(gk_surrogate *s, int rows, bool full)
{
    auto grown = [](int need, int have) {
        return (std::max(need, 2 * have) + 31) / 32 * 32;
    };
    const size_t hid = (size_t)s->o.hidden, no = (size_t)s->nout;
    if (rows > s->cap) {
        HIP_TRY(hipStreamSynchronize(s->stream));
        const int rc = grown(rows, s->cap);
        s->free_infer();
        const size_t R = (size_t)rc;
        HIP_TRY(hipMalloc((void **)&s->X, R * kInPad * sizeof(bf16)));
        for (int l = 0; l < s->layers; ++l) {
            bf16 *h;
            HIP_TRY(hipMalloc((void **)&h, R * hid * sizeof(bf16)));
            s->H.push_back(h);
        }
        HIP_TRY(hipMalloc((void **)&s->d_params, R * NPAR * sizeof(double)));
        HIP_TRY(hipHostMalloc((void **)&s->h_params, R * NPAR * sizeof(double), 0));
        HIP_TRY(hipMalloc((void **)&s->d_cpart, R * 2 * ((no + 63) / 64) * sizeof(double)));
        s->cap = rc;
    }
    if (full && rows > s->tcap) {
        HIP_TRY(hipStreamSynchronize(s->stream));
        const int rt = grown(rows, s->tcap);
        s->free_full();
        const size_t R = (size_t)rt;
        for (int l = 0; l < s->layers; ++l) {
            bf16 *dh;
            float *z;
            HIP_TRY(hipMalloc((void **)&dh, R * hid * sizeof(bf16)));
            s->dH.push_back(dh);
            HIP_TRY(hipMalloc((void **)&z, R * hid * sizeof(float)));
            s->Z.push_back(z);
        }
        HIP_TRY(hipMalloc((void **)&s->Y, R * no * sizeof(float)));
        HIP_TRY(hipMalloc((void **)&s->T, R * no * sizeof(float)));
        HIP_TRY(hipMalloc((void **)&s->Mask, R * no * sizeof(float)));
        HIP_TRY(hipMalloc((void **)&s->dY, R * no * sizeof(bf16)));
        HIP_TRY(hipMalloc((void **)&s->maps, R * 3 * s->npix * sizeof(float)));
        HIP_TRY(hipMalloc((void **)&s->cnt, R * sizeof(unsigned)));
        HIP_TRY(hipMalloc((void **)&s->d_partial, kRedBlocks * sizeof(double)));
        HIP_TRY(hipMalloc((void **)&s->d_colpart, (size_t)kColChunks * std::max(hid, no) * sizeof(float)));
        s->tcap = rt;
    }
    return GK_OK;
}

// hidden layers of M rows whose inputs are in s->X; keeps pre-activations if `keep`
gk_status hidden_layers(gk_surrogate *s, int M, bool keep, hipStream_t st)
{
    const bf16 *h = s->X;
    int in = kInPad;
    for (int l = 0; l < s->layers; ++l) {
        GemmArgs g{h, s->Wb[l], in, in, M, s->o.hidden, in, s->b[l], nullptr,
                   keep ? s->Z[l] : nullptr, s->H[l], s->o.hidden};
        GK_TRY((gemm<false, false, EPI_GELU>(g, st)));
        h = s->H[l];
        in = s->o.hidden;
    }
    return GK_OK;
}

// output layer into s->Y (scaled maps)
gk_status output_layer(gk_surrogate *s, int M, hipStream_t st)
{
    const int L = s->layers, in = s->o.hidden;
    GemmArgs g{s->H[L - 1], s->Wb[L], in, in, M, s->nout, in, s->b[L], s->Y, nullptr, nullptr, s->nout};
    return gemm<false, false, EPI_F32>(g, st);
}

gk_status forward(gk_surrogate *s, int M, bool keep, hipStream_t st)
{
    GK_TRY(hidden_layers(s, M, keep, st));
    return output_layer(s, M, st);
}

// targets from the plain evaluation of the rows in s->d_params, loss gradient,
// backward pass into gW/gb; the loss goes to *loss_dev
gk_status loss_and_grads(gk_surrogate *s, int M, float *loss_dev, hipStream_t st)
{
    GK_TRY(run_batch(s->model, s->d_params, M, s->maps, nullptr, nullptr, nullptr, st));
    hipLaunchKernelGGL(k_targets, dim3(M), dim3(256), 0, st, s->maps, s->npix, s->T, s->Mask, s->cnt);
    hipLaunchKernelGGL(k_encode, dim3(blocks(M, 64)), dim3(64), 0, st, s->d_params, M, s->d_lo,
                       s->d_hi, s->X);
    HIP_TRY(hipGetLastError());
    GK_TRY(forward(s, M, true, st));
    const size_t n = (size_t)M * s->nout;
    hipLaunchKernelGGL(k_mse_grad, dim3(kRedBlocks), dim3(256), 0, st, s->Y, s->T, s->Mask, n,
                       s->cnt, M, s->dY, s->d_partial);
    hipLaunchKernelGGL(k_loss_finish, dim3(1), dim3(256), 0, st, s->d_partial, kRedBlocks, s->cnt,
                       M, loss_dev);
    HIP_TRY(hipGetLastError());
    // backward: layer l has input h_{l-1} (X for l = 0) and output gradient d_l
    const int L = s->layers, hid = s->o.hidden;
    const bf16 *d = s->dY;
    for (int l = L; l >= 0; --l) {
        const int in = s->fin[l], out = s->fout[l];
        const bf16 *hin = l ? s->H[l - 1] : s->X;
        // gW_l[o][i] = sum_b d[b][o] hin[b][i]
        GemmArgs gw{d, hin, out, in, out, in, M, nullptr, s->gW[l], nullptr, nullptr, in};
        GK_TRY((gemm<true, true, EPI_F32>(gw, st)));
        hipLaunchKernelGGL(k_colsum, dim3(blocks(out), kColChunks), dim3(256), 0, st, d, M, out,
                           s->d_colpart);
        hipLaunchKernelGGL(k_colsum_finish, dim3(blocks(out)), dim3(256), 0, st, s->d_colpart, out,
                           s->gb[l]);
        HIP_TRY(hipGetLastError());
        if (l == 0) break;
        // d_{l-1}[b][i] = (sum_o d[b][o] W_l[o][i]) gelu'(Z_{l-1}[b][i])
        GemmArgs gd{d, s->Wb[l], out, in, M, in, out, nullptr, nullptr, s->Z[l - 1], s->dH[l - 1], hid};
        GK_TRY((gemm<false, true, EPI_DGELU>(gd, st)));
        d = s->dH[l - 1];
    }
    return GK_OK;
}

gk_status adam(gk_surrogate *s, double lr, hipStream_t st)
{
    s->step += 1;
    s->wver += 1;
    const double t = (double)s->step;
    const float c1 = (float)(1.0 / (1.0 - std::pow(0.9, t)));
    const float c2 = (float)(1.0 / (1.0 - std::pow(0.999, t)));
    for (int l = 0; l <= s->layers; ++l) {
        const size_t nw = (size_t)s->fout[l] * s->fin[l], nb = (size_t)s->fout[l];
        hipLaunchKernelGGL(k_adam, dim3(blocks(nw)), dim3(256), 0, st, s->W[l], s->gW[l], s->mW[l],
                           s->vW[l], s->Wb[l], nw, (float)lr, c1, c2);
        hipLaunchKernelGGL(k_adam, dim3(blocks(nb)), dim3(256), 0, st, s->b[l], s->gb[l], s->mb[l],
                           s->vb[l], (bf16 *)nullptr, nb, (float)lr, c1, c2);
    }
    HIP_TRY(hipGetLastError());
    return GK_OK;
}

// rows (host or device) -> s->d_params (on st); `full`: the caller needs the
// training and full-output buffers too
gk_status stage_params(gk_surrogate *s, const double *params, int B, bool full, hipStream_t st)
{
    const PtrKind pk = pointer_kind(params);
    if (pk == PTR_BAD) return fail(GK_EINVAL, "params pointer of unknown kind");
    GK_TRY(reserve_rows(s, B, full));
    if (pk == PTR_DEVICE) {
        HIP_TRY(hipMemcpyAsync(s->d_params, params, sizeof(double) * NPAR * B,
                               hipMemcpyDeviceToDevice, st));
    } else {
        HIP_TRY(hipEventSynchronize(s->ev_staged));  // the pinned rows may still feed a copy
        std::memcpy(s->h_params, params, sizeof(double) * NPAR * B);
        HIP_TRY(hipMemcpyAsync(s->d_params, s->h_params, sizeof(double) * NPAR * B,
                               hipMemcpyHostToDevice, st));
        HIP_TRY(hipEventRecord(s->ev_staged, st));
    }
    return GK_OK;
}

// inference chunk: rows per pass through the network (large passes keep
// the narrow hidden-layer products busy on every compute unit)
int infer_chunk(const gk_surrogate *s) { return std::max(s->o.batch, 8192); }

gk_status encode_rows(gk_surrogate *s, int B, hipStream_t st)
{
    hipLaunchKernelGGL(k_encode, dim3(blocks(B, 64)), dim3(64), 0, st, s->d_params, B, s->d_lo,
                       s->d_hi, s->X);
    HIP_TRY(hipGetLastError());
    return GK_OK;
}

// surrogate chi2 of the B rows in s->d_params against m's observation: the
// output layer reduces its own residuals, so the maps never reach memory
// The compact output layer for m's current observation and the current weights.
gk_status compact_output(gk_surrogate *s, gk_model *m, hipStream_t st)
{
    if (s->c_model == m && s->c_gen == m->gen && s->c_wver == s->wver && s->c_nv >= 0)
        return GK_OK;
    std::vector<uint8_t> mask(s->npix);
    HIP_TRY(hipStreamSynchronize(st));
    HIP_TRY(hipMemcpy(mask.data(), m->d_mask, s->npix, hipMemcpyDeviceToHost));
    std::vector<int> idx;
    for (int p = 0; p < s->npix; ++p)
        if (mask[p]) idx.push_back(p);
    s->free_compact();
    const int nv = (int)idx.size(), hid = s->o.hidden;
    if (nv > 0) {
        HIP_TRY(hipMalloc((void **)&s->c_W, (size_t)2 * nv * hid * sizeof(bf16)));
        HIP_TRY(hipMalloc((void **)&s->c_b, (size_t)2 * nv * sizeof(float)));
        HIP_TRY(hipMalloc((void **)&s->c_vo, (size_t)nv * sizeof(float)));
        HIP_TRY(hipMalloc((void **)&s->c_so, (size_t)nv * sizeof(float)));
        HIP_TRY(hipMalloc((void **)&s->c_iev, (size_t)nv * sizeof(double)));
        HIP_TRY(hipMalloc((void **)&s->c_ies, (size_t)nv * sizeof(double)));
        HIP_TRY(hipMalloc((void **)&s->c_idx, (size_t)nv * sizeof(int)));
        HIP_TRY(hipMemcpy(s->c_idx, idx.data(), (size_t)nv * sizeof(int), hipMemcpyHostToDevice));
        const int L = s->layers;
        hipLaunchKernelGGL(k_compact_rows, dim3(2 * nv), dim3(256), 0, st, s->Wb[L], s->b[L], hid,
                           s->npix, s->c_idx, nv, s->c_W, s->c_b);
        hipLaunchKernelGGL(k_compact_obs, dim3(blocks(nv)), dim3(256), 0, st, m->d_vo, m->d_so,
                           m->d_iev, m->d_ies, s->c_idx, nv, s->c_vo, s->c_so, s->c_iev, s->c_ies);
        HIP_TRY(hipGetLastError());
    }
    s->c_nv = nv;
    s->c_model = m;
    s->c_gen = m->gen;
    s->c_wver = s->wver;
    return GK_OK;
}

// surrogate chi2 of the B rows in s->d_params against m's observation: the
// output layer, restricted to the unmasked pixels, reduces its own
// residuals, so the maps never reach memory
gk_status infer_chi2(gk_surrogate *s, gk_model *m, int B, double *chi2, hipStream_t st)
{
    GK_TRY(compact_output(s, m, st));
    GK_TRY(encode_rows(s, B, st));
    GK_TRY(hidden_layers(s, B, false, st));
    const int L = s->layers, in = s->o.hidden, nc = 2 * s->c_nv;
    int nparts = 0;
    if (nc > 0) {
        const int T = gemm_tile(B, nc);
        nparts = 2 * ((nc + T - 1) / T);
        ObsArgs ob{nullptr, s->c_vo, s->c_so, s->c_iev, s->c_ies, s->c_nv, s->d_cpart, nparts};
        GemmArgs g{s->H[L - 1], s->c_W, in, in, B, nc, in, s->c_b, nullptr, nullptr, nullptr, 0, ob};
        GK_TRY((gemm<false, false, EPI_CHI2>(g, st)));
    }
    hipLaunchKernelGGL(k_chi2_finish, dim3((B + 3) / 4), dim3(256), 0, st, s->d_cpart, nparts, B,
                       s->d_params, m->d.rc, chi2);
    HIP_TRY(hipGetLastError());
    return GK_OK;
}

}  // namespace

// ---------------------------------------------------------------------------
// internal entry used by the screened sampler
// ---------------------------------------------------------------------------
gk_status gbk::surrogate_chi2(gk_surrogate *s, gk_model *obs, const double *d_params, int B,
                              double *d_chi2, hipStream_t st)
{
    for (int r0 = 0; r0 < B; r0 += infer_chunk(s)) {
        const int n = std::min(infer_chunk(s), B - r0);
        GK_TRY(stage_params(s, d_params + (size_t)r0 * NPAR, n, false, st));
        GK_TRY(infer_chi2(s, obs, n, d_chi2 + r0, st));
    }
    return GK_OK;
}

bool gbk::surrogate_matches(const gk_surrogate *s, const gk_model *m)
{
    const gk_model_desc &a = s->model->d, &b = m->d;
    return a.nx == b.nx && a.ny == b.ny && a.nz == b.nz && a.upsample == b.upsample &&
           a.dv_kms == b.dv_kms && a.v0_kms == b.v0_kms && a.crpix == b.crpix &&
           a.psf_fwhm_pix == b.psf_fwhm_pix && a.lsf_sigma_kms == b.lsf_sigma_kms &&
           a.kernel_radius_sigma == b.kernel_radius_sigma && a.rc == b.rc;
}

int gbk::surrogate_device(const gk_surrogate *s) { return s->device; }

// ---------------------------------------------------------------------------
// C ABI
// ---------------------------------------------------------------------------
extern "C" {

gk_status gk_surrogate_default_opts(gk_surrogate_opts *o)
{
    if (!o) return fail(GK_EINVAL, "opts is NULL");
    std::memset(o, 0, sizeof *o);
    o->hidden = 1024;
    o->layers = 4;
    o->batch = 512;
    o->lr = 1e-3;
    o->lr_final = 1e-5;
    o->seed = 1;
    return GK_OK;
}

gk_status gk_surrogate_create(gk_model *m, const double *lo, const double *hi,
                              const gk_surrogate_opts *o_in, gk_surrogate **out)
{
    if (!m || !lo || !hi || !out) return fail(GK_EINVAL, "NULL argument");
    *out = nullptr;
    if (m->vfield) return fail(GK_EINVAL, "the surrogate learns cube-strategy maps");
    gk_surrogate_opts o;
    gk_surrogate_default_opts(&o);
    if (o_in) o = *o_in;
    if (o.hidden < 32 || o.hidden % 32 || o.hidden > 8192 || o.layers < 1 || o.layers > 16 ||
        o.batch < 32 || o.batch % 32 || o.batch > 65536 || !(o.lr > 0.0) || !(o.lr_final > 0.0))
        return fail(GK_EINVAL, "invalid surrogate options (hidden and batch multiples of 32)");
    for (int k = 0; k < NPAR; ++k)
        if (!(hi[k] >= lo[k]) || !std::isfinite(lo[k]) || !std::isfinite(hi[k]))
            return fail(GK_EINVAL, "invalid box in slot %d", k);
    if (m->d.rc == RC_EPINAT && (hi[P_A] > lo[P_A] || hi[P_G] > lo[P_G]))
        return fail(GK_EINVAL, "the surrogate does not take the Epinat shape slots as inputs");
    if (m->d.upsample != 1) return fail(GK_EINVAL, "the surrogate needs upsample = 1");
    if ((m->d.nx * m->d.ny) % 16)
        return fail(GK_EINVAL, "the surrogate needs nx * ny to be a multiple of 16");
    if (!(lo[P_INC] > 0.0 && hi[P_INC] < 90.0 && lo[P_SIG] > 0.0 && lo[P_R0] > 0.0 && lo[P_RT] > 0.0))
        return fail(GK_EINVAL, "the box leaves the parameter domain");
    auto *s = new (std::nothrow) gk_surrogate;
    if (!s) return fail(GK_ENOMEM, "out of host memory");
    s->model = m;
    s->device = m->device;
    s->o = o;
    s->npix = m->d.nx * m->d.ny;
    s->nout = 2 * s->npix;
    s->layers = o.layers;
    std::memcpy(s->lo, lo, sizeof s->lo);
    std::memcpy(s->hi, hi, sizeof s->hi);
    DeviceGuard g(m->device);
    auto fail_free = [&](gk_status st) {
        s->release();
        delete s;
        return st;
    };
    if (g.err != hipSuccess) return fail_free(fail(GK_EDEVICE, "hipSetDevice failed"));
    auto init = [&]() -> gk_status {
        HIP_TRY(hipStreamCreateWithFlags(&s->stream, hipStreamNonBlocking));
        HIP_TRY(hipEventCreateWithFlags(&s->ev_staged, hipEventDisableTiming));
        HIP_TRY(hipMalloc((void **)&s->d_lo, sizeof s->lo));
        HIP_TRY(hipMalloc((void **)&s->d_hi, sizeof s->hi));
        HIP_TRY(hipMemcpy(s->d_lo, s->lo, sizeof s->lo, hipMemcpyHostToDevice));
        HIP_TRY(hipMemcpy(s->d_hi, s->hi, sizeof s->hi, hipMemcpyHostToDevice));
        for (int l = 0; l <= s->layers; ++l) {
            s->fin.push_back(l ? o.hidden : kInPad);
            s->fout.push_back(l < s->layers ? o.hidden : s->nout);
        }
        // He initialisation for the GELU layers, 1/sqrt(fan-in) for the output
        // layer, zero biases; weights drawn from Philox normals
        Rng rng(o.seed, 0x6d6c70u);
        for (int l = 0; l <= s->layers; ++l) {
            const size_t nw = (size_t)s->fout[l] * s->fin[l], nb = (size_t)s->fout[l];
            const int fan = l ? s->fin[l] : 11;
            const double sd = (l < s->layers ? std::sqrt(2.0) : 1.0) / std::sqrt((double)fan);
            std::vector<float> w(nw, 0.0f);
            for (size_t r = 0; r < (size_t)s->fout[l]; ++r)
                for (int c = 0; c < s->fin[l]; ++c)
                    w[r * s->fin[l] + c] = (l == 0 && c >= 11) ? 0.0f : (float)(sd * rng.normal());
            float *p;
            bf16 *pb;
            for (auto *v : {&s->W, &s->gW, &s->mW, &s->vW}) {
                HIP_TRY(hipMalloc((void **)&p, nw * sizeof(float)));
                HIP_TRY(hipMemset(p, 0, nw * sizeof(float)));
                v->push_back(p);
            }
            for (auto *v : {&s->b, &s->gb, &s->mb, &s->vb}) {
                HIP_TRY(hipMalloc((void **)&p, nb * sizeof(float)));
                HIP_TRY(hipMemset(p, 0, nb * sizeof(float)));
                v->push_back(p);
            }
            HIP_TRY(hipMalloc((void **)&pb, nw * sizeof(bf16)));
            s->Wb.push_back(pb);
            HIP_TRY(hipMemcpy(s->W[l], w.data(), nw * sizeof(float), hipMemcpyHostToDevice));
            hipLaunchKernelGGL(k_to_bf16, dim3(blocks(nw)), dim3(256), 0, s->stream, s->W[l], pb, nw);
            HIP_TRY(hipGetLastError());
        }
        GK_TRY(reserve_rows(s, o.batch, true));
        HIP_TRY(hipStreamSynchronize(s->stream));
        return GK_OK;
    };
    const gk_status st = init();
    if (st < 0) return fail_free(st);
    *out = s;
    return GK_OK;
}

gk_status gk_surrogate_destroy(gk_surrogate *s)
{
    if (!s) return GK_OK;
    DeviceGuard g(s->device);
    s->release();
    delete s;
    return GK_OK;
}

int64_t gk_surrogate_weight_count(const gk_surrogate *s) { return s ? (int64_t)s->weight_count() : -1; }

gk_status gk_surrogate_get_weights(gk_surrogate *s, float *w, int64_t n)
{
    if (!s || !w) return fail(GK_EINVAL, "NULL argument");
    if (n != (int64_t)s->weight_count()) return fail(GK_EINVAL, "weight count mismatch");
    DeviceGuard g(s->device);
    HIP_TRY(g.err);
    HIP_TRY(hipStreamSynchronize(s->stream));
    for (int l = 0; l <= s->layers; ++l) {
        const size_t nw = (size_t)s->fout[l] * s->fin[l], nb = (size_t)s->fout[l];
        HIP_TRY(hipMemcpy(w, s->W[l], nw * sizeof(float), hipMemcpyDeviceToHost));
        HIP_TRY(hipMemcpy(w + nw, s->b[l], nb * sizeof(float), hipMemcpyDeviceToHost));
        w += nw + nb;
    }
    return GK_OK;
}

gk_status gk_surrogate_set_weights(gk_surrogate *s, const float *w, int64_t n)
{
    if (!s || !w) return fail(GK_EINVAL, "NULL argument");
    if (n != (int64_t)s->weight_count()) return fail(GK_EINVAL, "weight count mismatch");
    DeviceGuard g(s->device);
    HIP_TRY(g.err);
    HIP_TRY(hipStreamSynchronize(s->stream));
    for (int l = 0; l <= s->layers; ++l) {
        const size_t nw = (size_t)s->fout[l] * s->fin[l], nb = (size_t)s->fout[l];
        HIP_TRY(hipMemcpy(s->W[l], w, nw * sizeof(float), hipMemcpyHostToDevice));
        HIP_TRY(hipMemcpy(s->b[l], w + nw, nb * sizeof(float), hipMemcpyHostToDevice));
        hipLaunchKernelGGL(k_to_bf16, dim3(blocks(nw)), dim3(256), 0, s->stream, s->W[l], s->Wb[l], nw);
        HIP_TRY(hipGetLastError());
        w += nw + nb;
    }
    // a fresh optimiser state goes with new weights
    for (int l = 0; l <= s->layers; ++l) {
        const size_t nw = (size_t)s->fout[l] * s->fin[l], nb = (size_t)s->fout[l];
        HIP_TRY(hipMemsetAsync(s->mW[l], 0, nw * sizeof(float), s->stream));
        HIP_TRY(hipMemsetAsync(s->vW[l], 0, nw * sizeof(float), s->stream));
        HIP_TRY(hipMemsetAsync(s->mb[l], 0, nb * sizeof(float), s->stream));
        HIP_TRY(hipMemsetAsync(s->vb[l], 0, nb * sizeof(float), s->stream));
    }
    s->step = 0;
    s->wver += 1;
    HIP_TRY(hipStreamSynchronize(s->stream));
    return GK_OK;
}

gk_status gk_surrogate_train(gk_surrogate *s, int64_t steps, float *losses)
{
    if (!s) return fail(GK_EINVAL, "surrogate is NULL");
    if (steps < 0) return fail(GK_EINVAL, "negative step count");
    if (steps == 0) return GK_OK;
    DeviceGuard g(s->device);
    HIP_TRY(g.err);
    hipStream_t st = s->stream;
    GK_TRY(reserve_rows(s, s->o.batch, true));
    const int64_t chunk = 4096;  // losses are gathered per chunk of steps
    if (s->loss_cap < chunk) {
        HIP_TRY(hipStreamSynchronize(st));
        if (s->d_loss) (void)hipFree(s->d_loss);
        s->d_loss = nullptr;
        s->loss_cap = 0;
        HIP_TRY(hipMalloc((void **)&s->d_loss, chunk * sizeof(float)));
        s->loss_cap = (int)chunk;
    }
    const int B = s->o.batch;
    for (int64_t t0 = 0; t0 < steps; t0 += chunk) {
        const int64_t n = std::min<int64_t>(chunk, steps - t0);
        for (int64_t t = t0; t < t0 + n; ++t) {
            // cosine decay from lr to lr_final over the steps of this call
            const double f = steps > 1 ? (double)t / (double)(steps - 1) : 0.0;
            const double lr = s->o.lr_final + 0.5 * (s->o.lr - s->o.lr_final) * (1.0 + std::cos(M_PI * f));
            hipLaunchKernelGGL(k_draw, dim3(blocks(B, 64)), dim3(64), 0, st, s->o.seed,
                               (uint64_t)s->step, B, s->d_lo, s->d_hi, s->d_params);
            HIP_TRY(hipGetLastError());
            GK_TRY(loss_and_grads(s, B, s->d_loss + (t - t0), st));
            GK_TRY(adam(s, lr, st));
        }
        if (losses)
            HIP_TRY(hipMemcpyAsync(losses + t0, s->d_loss, n * sizeof(float), hipMemcpyDeviceToHost, st));
        HIP_TRY(hipStreamSynchronize(st));
    }
    return GK_OK;
}

namespace {

constexpr char kSurrogateTag[8] = {'G', 'K', 'S', 'U', 'R', 'R', '0', '1'};

// The instrument fields a saved surrogate depends on, in file order (no
// padding: six doubles, then six 32-bit integers, the last always 0).
struct SavedInstrument {
    double dv, v0, crpix, psf, lsf, R;
    int32_t nx, ny, nz, upsample, rc, zero;
};
static_assert(sizeof(SavedInstrument) == 72, "unpadded layout");

SavedInstrument instrument_of(const gk_model_desc &d)
{
    return {d.dv_kms, d.v0_kms, d.crpix, d.psf_fwhm_pix, d.lsf_sigma_kms, d.kernel_radius_sigma,
            d.nx, d.ny, d.nz, d.upsample, d.rc, 0};
}

bool same_instrument(const SavedInstrument &a, const SavedInstrument &b)
{
    return a.dv == b.dv && a.v0 == b.v0 && a.crpix == b.crpix && a.psf == b.psf && a.lsf == b.lsf &&
           a.R == b.R && a.nx == b.nx && a.ny == b.ny && a.nz == b.nz && a.upsample == b.upsample &&
           a.rc == b.rc;
}

struct File {
    FILE *f = nullptr;
    ~File()
    {
        if (f) std::fclose(f);
    }
};

}  // namespace

gk_status gk_surrogate_save(gk_surrogate *s, const char *path)
{
    if (!s || !path) return fail(GK_EINVAL, "NULL argument");
    std::vector<float> w(s->weight_count());
    GK_TRY(gk_surrogate_get_weights(s, w.data(), (int64_t)w.size()));
    File f;
    f.f = std::fopen(path, "wb");
    if (!f.f) return fail(GK_EINVAL, "cannot open %s for writing", path);
    const SavedInstrument ins = instrument_of(s->model->d);
    const int32_t ints[3] = {s->o.hidden, s->o.layers, s->o.batch};
    const double lrs[2] = {s->o.lr, s->o.lr_final};
    const int64_t n = (int64_t)w.size();
    bool ok = std::fwrite(kSurrogateTag, 1, 8, f.f) == 8;
    ok = ok && std::fwrite(ints, sizeof ints, 1, f.f) == 1;
    ok = ok && std::fwrite(lrs, sizeof lrs, 1, f.f) == 1;
    ok = ok && std::fwrite(&s->o.seed, sizeof s->o.seed, 1, f.f) == 1;
    ok = ok && std::fwrite(s->lo, sizeof s->lo, 1, f.f) == 1;
    ok = ok && std::fwrite(s->hi, sizeof s->hi, 1, f.f) == 1;
    ok = ok && std::fwrite(&ins, sizeof ins, 1, f.f) == 1;
    ok = ok && std::fwrite(&n, sizeof n, 1, f.f) == 1;
    ok = ok && std::fwrite(w.data(), sizeof(float), w.size(), f.f) == w.size();
    ok = std::fclose(f.f) == 0 && ok;
    f.f = nullptr;
    if (!ok) return fail(GK_EINVAL, "writing %s failed", path);
    return GK_OK;
}

gk_status gk_surrogate_load(gk_model *m, const char *path, gk_surrogate **out)
{
    if (!m || !path || !out) return fail(GK_EINVAL, "NULL argument");
    *out = nullptr;
    File f;
    f.f = std::fopen(path, "rb");
    if (!f.f) return fail(GK_EINVAL, "cannot open %s", path);
    char tag[8];
    int32_t ints[3];
    double lrs[2], lo[NPAR], hi[NPAR];
    uint64_t seed;
    SavedInstrument ins;
    int64_t n = 0;
    bool ok = std::fread(tag, 1, 8, f.f) == 8 && std::memcmp(tag, kSurrogateTag, 8) == 0;
    ok = ok && std::fread(ints, sizeof ints, 1, f.f) == 1;
    ok = ok && std::fread(lrs, sizeof lrs, 1, f.f) == 1;
    ok = ok && std::fread(&seed, sizeof seed, 1, f.f) == 1;
    ok = ok && std::fread(lo, sizeof lo, 1, f.f) == 1;
    ok = ok && std::fread(hi, sizeof hi, 1, f.f) == 1;
    ok = ok && std::fread(&ins, sizeof ins, 1, f.f) == 1;
    ok = ok && std::fread(&n, sizeof n, 1, f.f) == 1;
    if (!ok) return fail(GK_EINVAL, "%s is not a saved surrogate or is truncated", path);
    const SavedInstrument mine = instrument_of(m->d);
    if (!same_instrument(ins, mine))
        return fail(GK_EINVAL, "%s was saved for another instrument", path);
    gk_surrogate_opts o;
    gk_surrogate_default_opts(&o);
    o.hidden = ints[0];
    o.layers = ints[1];
    o.batch = ints[2];
    o.lr = lrs[0];
    o.lr_final = lrs[1];
    o.seed = seed;
    gk_surrogate *s = nullptr;
    GK_TRY(gk_surrogate_create(m, lo, hi, &o, &s));
    std::vector<float> w;
    gk_status st = GK_OK;
    if (n != gk_surrogate_weight_count(s)) {
        st = fail(GK_EINVAL, "%s holds %lld weights, the network has %lld", path, (long long)n,
                  (long long)gk_surrogate_weight_count(s));
    } else {
        w.resize((size_t)n);
        if (std::fread(w.data(), sizeof(float), w.size(), f.f) != w.size())
            st = fail(GK_EINVAL, "%s is truncated", path);
        else
            st = gk_surrogate_set_weights(s, w.data(), n);
    }
    if (st != GK_OK) {
        gk_surrogate_destroy(s);
        return st;
    }
    *out = s;
    return GK_OK;
}

gk_status gk_surrogate_gradients(gk_surrogate *s, const double *params, int32_t B, float *grads,
                                 double *loss)
{
    if (!s || !params || !grads) return fail(GK_EINVAL, "NULL argument");
    if (B <= 0 || B > 65536) return fail(GK_EINVAL, "invalid batch size %d", B);
    if (B % 32) return fail(GK_EINVAL, "gradient batches must be a multiple of 32 rows");
    DeviceGuard g(s->device);
    HIP_TRY(g.err);
    hipStream_t st = s->stream;
    GK_TRY(stage_params(s, params, B, true, st));
    if (!s->d_loss) {
        HIP_TRY(hipMalloc((void **)&s->d_loss, 4096 * sizeof(float)));
        s->loss_cap = 4096;
    }
    GK_TRY(loss_and_grads(s, B, s->d_loss, st));
    HIP_TRY(hipStreamSynchronize(st));
    float lf;
    HIP_TRY(hipMemcpy(&lf, s->d_loss, sizeof lf, hipMemcpyDeviceToHost));
    if (loss) *loss = lf;
    for (int l = 0; l <= s->layers; ++l) {
        const size_t nw = (size_t)s->fout[l] * s->fin[l], nb = (size_t)s->fout[l];
        HIP_TRY(hipMemcpy(grads, s->gW[l], nw * sizeof(float), hipMemcpyDeviceToHost));
        HIP_TRY(hipMemcpy(grads + nw, s->gb[l], nb * sizeof(float), hipMemcpyDeviceToHost));
        grads += nw + nb;
    }
    return GK_OK;
}

gk_status gk_surrogate_step(gk_surrogate *s, const double *params, int32_t B, double lr,
                            double *loss)
{
    if (!s || !params) return fail(GK_EINVAL, "NULL argument");
    if (B <= 0 || B > 65536) return fail(GK_EINVAL, "invalid batch size %d", B);
    if (B % 32) return fail(GK_EINVAL, "training batches must be a multiple of 32 rows");
    if (!(lr > 0.0) || !std::isfinite(lr)) return fail(GK_EINVAL, "step size must be finite and > 0");
    DeviceGuard g(s->device);
    HIP_TRY(g.err);
    hipStream_t st = s->stream;
    GK_TRY(stage_params(s, params, B, true, st));
    if (!s->d_loss) {
        HIP_TRY(hipMalloc((void **)&s->d_loss, 4096 * sizeof(float)));
        s->loss_cap = 4096;
    }
    GK_TRY(loss_and_grads(s, B, s->d_loss, st));
    GK_TRY(adam(s, lr, st));
    HIP_TRY(hipStreamSynchronize(st));
    float lf;
    HIP_TRY(hipMemcpy(&lf, s->d_loss, sizeof lf, hipMemcpyDeviceToHost));
    if (loss) *loss = lf;
    return GK_OK;
}

gk_status gk_surrogate_predict(gk_surrogate *s, const double *params, int32_t B, float *maps,
                               void *stream)
{
    if (!s) return fail(GK_EINVAL, "surrogate is NULL");
    if (B < 0) return fail(GK_EINVAL, "negative batch size");
    if (B == 0) return GK_OK;
    if (!params || !maps) return fail(GK_EINVAL, "NULL argument");
    if (pointer_kind(maps) != PTR_DEVICE) return fail(GK_EINVAL, "maps must be device memory");
    DeviceGuard g(s->device);
    HIP_TRY(g.err);
    hipStream_t st = (hipStream_t)stream;
    for (int r0 = 0; r0 < B; r0 += infer_chunk(s)) {
        const int n = std::min(infer_chunk(s), B - r0);
        GK_TRY(stage_params(s, params + (size_t)r0 * NPAR, n, true, st));
        GK_TRY(encode_rows(s, n, st));
        GK_TRY(forward(s, n, false, st));
        const size_t ne = (size_t)n * s->nout;
        hipLaunchKernelGGL(k_scale_maps, dim3(blocks(ne)), dim3(256), 0, st, s->Y, s->npix, ne,
                           maps + (size_t)r0 * s->nout);
        HIP_TRY(hipGetLastError());
    }
    return GK_OK;
}

gk_status gk_surrogate_chi2(gk_surrogate *s, gk_model *m, const double *params, int32_t B,
                            double *chi2, void *stream)
{
    if (!s || !m) return fail(GK_EINVAL, "NULL argument");
    if (B < 0) return fail(GK_EINVAL, "negative batch size");
    if (B == 0) return GK_OK;
    if (!params || !chi2) return fail(GK_EINVAL, "NULL argument");
    if (!m->has_obs) return fail(GK_ESTATE, "no observation set");
    if (!surrogate_matches(s, m)) return fail(GK_EINVAL, "model instrument differs from the surrogate's");
    if (m->device != s->device) return fail(GK_EINVAL, "model and surrogate on different devices");
    if (pointer_kind(chi2) != PTR_DEVICE) return fail(GK_EINVAL, "chi2 must be device memory");
    DeviceGuard g(s->device);
    HIP_TRY(g.err);
    hipStream_t st = (hipStream_t)stream;
    for (int r0 = 0; r0 < B; r0 += infer_chunk(s)) {
        const int n = std::min(infer_chunk(s), B - r0);
        GK_TRY(stage_params(s, params + (size_t)r0 * NPAR, n, false, st));
        GK_TRY(infer_chi2(s, m, n, chi2 + r0, st));
    }
    return GK_OK;
}

gk_status gk_gemm_bf16(int32_t trans_a, int32_t trans_b, int32_t M, int32_t N, int32_t K,
                       const uint16_t *A, int32_t lda, const uint16_t *B, int32_t ldb, float *C,
                       int32_t ldc, void *stream)
{
    if (!A || !B || !C) return fail(GK_EINVAL, "NULL argument");
    for (const void *p : {(const void *)A, (const void *)B, (const void *)C})
        if (pointer_kind(p) != PTR_DEVICE) return fail(GK_EINVAL, "GEMM operands must be device memory");
    GemmArgs g{reinterpret_cast<const bf16 *>(A), reinterpret_cast<const bf16 *>(B), lda, ldb, M, N, K,
               nullptr, C, nullptr, nullptr, ldc};
    hipStream_t s = (hipStream_t)stream;
    if (!trans_a && !trans_b) return gemm<false, false, EPI_F32>(g, s);
    if (!trans_a && trans_b) return gemm<false, true, EPI_F32>(g, s);
    if (trans_a && trans_b) return gemm<true, true, EPI_F32>(g, s);
    return gemm<true, false, EPI_F32>(g, s);
}

}  // extern "C"
