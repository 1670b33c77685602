// fp61.hpp -- arithmetic in F_p, p = 2^61 - 1 (Sec. 6.1), for device and host.
//
// Values are kept canonical (0 <= x < p) in uint64_t.  A product is built
// from the 64 x 64 -> 128-bit multiply (low word and mulhi) and reduced
// with 2^61 = 1 (mod p): x = q 2^61 + r  ==  q + r.  Sums of up to eight
// canonical values fit in 64 bits (8 (p - 1) < 2^64), which the reductions
// use to fold lazily.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace fp {

typedef uint64_t u64;
typedef uint32_t u32;

constexpr u64 P = (1ull << 61) - 1;

__host__ __device__ __forceinline__ u64 add(u64 a, u64 b) {
    u64 s = a + b;
    return s >= P ? s - P : s;
}

__host__ __device__ __forceinline__ u64 sub(u64 a, u64 b) {
    return a >= b ? a - b : a + P - b;
}

// Fold a value below 2^64 into [0, p].  Callers that need a canonical
// result apply canon() afterwards.
__host__ __device__ __forceinline__ u64 fold64(u64 x) { return (x & P) + (x >> 61); }

__host__ __device__ __forceinline__ u64 canon(u64 x) { return x >= P ? x - P : x; }

__host__ __device__ __forceinline__ u64 mul(u64 a, u64 b) {
    unsigned __int128 x = (unsigned __int128)a * b;  // < 2^122
    u64 lo = (u64)x, hi = (u64)(x >> 64);
    u64 s = (lo & P) + ((lo >> 61) | (hi << 3));     // r + q < 2^62 - 1
    s = (s & P) + (s >> 61);                          // <= p
    return canon(s);
}

// Lazy reduction: a sum of up to 64 products of canonical values (each
// below 2^122) is accumulated exactly in 128 bits and reduced once.
typedef unsigned __int128 u128;

__host__ __device__ __forceinline__ u128 wide(u64 a, u64 b) { return (u128)a * b; }

__host__ __device__ __forceinline__ u64 red128(u128 x) {
    const u64 lo = (u64)x, hi = (u64)(x >> 64);
    // x = hi 2^64 + lo and 2^64 = 8 (mod p); hi 8 = (hi >> 58) 2^61 + ((hi << 3) & p)
    u64 s = (lo & P) + (lo >> 61) + ((hi << 3) & P) + (hi >> 58);  // < 2^63
    s = (s & P) + (s >> 61);                                          // <= p + 3
    return canon(s);
}

// eq(bit, r) = r if bit else 1 - r
__host__ __device__ __forceinline__ u64 eqbit(u32 bit, u64 r) { return bit ? r : sub(1, r); }

// eq(x, y) = x y + (1 - x)(1 - y) = 2 x y + 1 - x - y: one product, the
// rest added unreduced (2 p + 1 - x - y > 0) and reduced once.
__host__ __device__ __forceinline__ u64 eq(u64 x, u64 y) {
    return red128((wide(x, y) << 1) + (2 * P + 1 - x - y));
}

__host__ __device__ __forceinline__ u64 pow(u64 a, u64 e) {
    u64 r = 1;
    while (e) {
        if (e & 1) r = mul(r, a);
        a = mul(a, a);
        e >>= 1;
    }
    return r;
}

__host__ __device__ __forceinline__ u64 inv(u64 a) { return pow(a, P - 2); }

// ---------------------------------------------------------------------------
// SplitMix64 (Steele, Lea, Flood, OOPSLA 2014): the verifier's coin stream.
// state_0 = (seed << 8) | purpose; each draw adds gamma and mixes.
constexpr u64 SM_GAMMA = 0x9E3779B97F4A7C15ull;

__host__ __device__ __forceinline__ u64 sm_mix(u64 z) {
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

__host__ __device__ __forceinline__ u64 sm_state(u64 seed, u64 purpose) {
    return (seed << 8) | purpose;
}

// One field challenge: the low 61 bits of the next output, redrawn if they
// are all ones (2^61 - 1 = p is not a field element).
__host__ __device__ __forceinline__ u64 sm_field(u64 &state) {
    for (;;) {
        state += SM_GAMMA;
        u64 x = sm_mix(state) & P;
        if (x != P) return x;
    }
}

enum { PURPOSE_GKR = 2, PURPOSE_F2SC = 4 };

}  // namespace fp
