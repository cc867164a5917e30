// Philox4x32-10 counter-based generator (Salmon, Moraes, Dror, Shaw,
// "Parallel random numbers: as easy as 1, 2, 3", SC 2011), for device and host.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

namespace htri {

struct U4 {
    uint32_t x, y, z, w;
};

__host__ __device__ __forceinline__ void mulhilo32(uint32_t a, uint32_t b, uint32_t &hi, uint32_t &lo) {
    uint64_t p = (uint64_t)a * (uint64_t)b;
    hi = (uint32_t)(p >> 32);
    lo = (uint32_t)p;
}

__host__ __device__ __forceinline__ U4 philox4x32_10(U4 c, uint32_t k0, uint32_t k1) {
#pragma unroll
    for (int r = 0; r < 10; r++) {
        if (r) {
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        uint32_t hi0, lo0, hi1, lo1;
        mulhilo32(0xD2511F53u, c.x, hi0, lo0);
        mulhilo32(0xCD9E8D57u, c.z, hi1, lo1);
        c = U4{hi1 ^ c.y ^ k0, lo1, hi0 ^ c.w ^ k1, lo0};
    }
    return c;
}

// 64-bit uniform word number t of stream `stream` under key `seed`
__host__ __device__ __forceinline__ uint64_t philox_u64(uint64_t seed, uint32_t stream, uint64_t t) {
    U4 o = philox4x32_10(U4{(uint32_t)t, (uint32_t)(t >> 32), stream, 0u}, (uint32_t)seed,
                         (uint32_t)(seed >> 32));
    return ((uint64_t)o.y << 32) | o.x;
}

__host__ __device__ __forceinline__ uint64_t mulhi64(uint64_t a, uint64_t b) {
    return (uint64_t)(((unsigned __int128)a * b) >> 64);
}

// uniform integer in [0, n): floor(u * n / 2^64)
__host__ __device__ __forceinline__ uint64_t philox_index(uint64_t seed, uint32_t stream, uint64_t t, uint64_t n) {
    return mulhi64(philox_u64(seed, stream, t), n);
}

// uniform double in [0, 1): top 53 bits
__host__ __device__ __forceinline__ double philox_unit(uint64_t seed, uint32_t stream, uint64_t t) {
    return (double)(philox_u64(seed, stream, t) >> 11) * (1.0 / 9007199254740992.0);
}

}  // namespace htri
