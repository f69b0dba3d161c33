// gbk_rng.h -- private: Philox4x32-10 counter-based generator (the block
// function for host and device code, a sequential stream for host code).
#pragma once
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>

namespace gbk {

// ---- Philox4x32-10 (Salmon, Moraes, Dror & Shaw 2011) ----------------------
constexpr uint32_t kPhiloxM0 = 0xD2511F53u, kPhiloxM1 = 0xCD9E8D57u;
constexpr uint32_t kPhiloxW0 = 0x9E3779B9u, kPhiloxW1 = 0xBB67AE85u;

__host__ __device__ inline void philox4x32_10(const uint32_t in[4], const uint32_t key_in[2], uint32_t out[4])
{
    uint32_t c0 = in[0], c1 = in[1], c2 = in[2], c3 = in[3];
    uint32_t k0 = key_in[0], k1 = key_in[1];
    for (int r = 0; r < 10; ++r) {
        if (r) {
            k0 += kPhiloxW0;
            k1 += kPhiloxW1;
        }
        const uint64_t p0 = (uint64_t)kPhiloxM0 * c0, p1 = (uint64_t)kPhiloxM1 * c2;
        const uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        const uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        const uint32_t n0 = hi1 ^ c1 ^ k0, n2 = hi0 ^ c3 ^ k1;
        c0 = n0;
        c1 = lo1;
        c2 = n2;
        c3 = lo0;
    }
    out[0] = c0;
    out[1] = c1;
    out[2] = c2;
    out[3] = c3;
}

// Sequential uniforms in (0, 1) from Philox blocks: counter = (n, n >> 32, stream, 0).
struct Rng {
    uint32_t key[2];
    uint32_t stream;
    uint64_t n = 0;
    uint32_t buf[4];
    int left = 0;
    Rng(uint64_t seed, uint32_t s) : stream(s)
    {
        key[0] = (uint32_t)seed;
        key[1] = (uint32_t)(seed >> 32);
    }
    uint32_t u32()
    {
        if (!left) {
            const uint32_t c[4] = {(uint32_t)n, (uint32_t)(n >> 32), stream, 0u};
            philox4x32_10(c, key, buf);
            ++n;
            left = 4;
        }
        return buf[4 - left--];
    }
    double uniform()  // 53 random bits, never 0 or 1
    {
        const uint64_t a = u32(), b = u32();
        return ((double)((a << 21) ^ (b >> 11)) + 0.5) * 0x1.0p-53;
    }
    double normal()  // Box-Muller
    {
        const double u1 = uniform(), u2 = uniform();
        return std::sqrt(-2.0 * std::log(u1)) * std::cos(6.283185307179586 * u2);
    }
};

}  // namespace gbk
