// wide.h -- arithmetic of the 32-bit field path: uint32 residues, p prime,
// 2 <= p < 2^32 (the uint32 coefficient version of Sec. 2).
//
// Model (exact integers throughout):
//  * a product of two residues needs 64 bits; it is reduced by Barrett with
//    mu = floor((2^64 - 1) / p): q = umul64hi(x, mu) lies in
//    [floor(x/p) - 2, floor(x/p)] for every x < 2^64, so two conditional
//    subtractions finish;
//  * a multiply-accumulate keeps a 64-bit sum of raw products: when adding a
//    product wraps the sum past 2^64 (the new sum is below the product),
//    c64 = 2^64 mod p is added back.  The wrapped sum is below the product,
//    at most (p - 1)^2 < 2^64 - 2^33, so adding c64 < 2^32 cannot wrap again;
//  * int8 limbs for the matrix cores: a residue x is centred to
//    r = x (x <= 2139062143) or x - p, so r lies in [-2155905152, 2139062143]
//    = 127 * (1 + 2^8 + 2^16 + 2^24) down to -128 * (same), and written as
//    four balanced signed bytes r = l0 + 2^8 l1 + 2^16 l2 + 2^24 l3
//    (l_i in [-128, 127]).  A product sum over K terms is then
//    sum_{d=0..6} 2^{8d} D_d with D_d = sum_{i+j=d} sum_k a_i b_j: at most four
//    limb products per diagonal, each |a_i b_j| <= 2^14, so
//    |D_d| <= 4 * 2^14 * K < 2^31 for K <= kWideKChunk = 32704 terms.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace flw {

constexpr uint32_t kWideKChunk = 32704;       // multiple of 64, 4 * 2^14 * K < 2^31
constexpr int64_t kWideWindow = 2139062143;   // 127 * (1 + 2^8 + 2^16 + 2^24)

struct Mod64 {
    uint32_t p;
    uint64_t mu;   // floor((2^64 - 1) / p)
    uint64_t c64;  // 2^64 mod p
    uint32_t c32;  // 2^32 mod p
    uint32_t c57;  // 2^57 mod p
};

inline Mod64 make_mod64(uint32_t p) {
    Mod64 m;
    m.p = p;
    m.mu = ~(uint64_t)0 / p;
    m.c64 = (~(uint64_t)0 % p + 1) % p;
    m.c32 = (uint32_t)(((uint64_t)1 << 32) % p);
    m.c57 = (uint32_t)(((uint64_t)1 << 57) % p);
    return m;
}

__device__ __forceinline__ uint32_t reduce64(uint64_t x, const Mod64 &m) {
    const uint64_t q = __umul64hi(x, m.mu);
    uint64_t r = x - q * m.p;
    r = r >= m.p ? r - m.p : r;
    r = r >= m.p ? r - m.p : r;
    return (uint32_t)r;
}

__device__ __forceinline__ uint32_t mulw(uint32_t a, uint32_t b, const Mod64 &m) {
    return reduce64((uint64_t)a * b, m);
}

// a + b and a - b mod p for residues, without leaving 32 bits (p < 2^32)
__device__ __forceinline__ uint32_t addw(uint32_t a, uint32_t b, uint32_t p) {
    const uint32_t nb = p - b;
    return a >= nb ? a - nb : a + b;
}
__device__ __forceinline__ uint32_t subw(uint32_t a, uint32_t b, uint32_t p) {
    return a >= b ? a - b : a + (p - b);
}

// acc += a b (64-bit sum of raw products, wrap folded back with c64)
__device__ __forceinline__ void macw(uint64_t &acc, uint32_t a, uint32_t b, const Mod64 &m) {
    const uint64_t prod = (uint64_t)a * b;
    acc += prod;
    if (acc < prod) acc += m.c64;
}

// Inverse by Fermat's little theorem (x != 0, p prime).
__device__ inline uint32_t invw(uint32_t x, const Mod64 &m) {
    uint32_t r = 1 % m.p, b = x, e = m.p - 2;
    while (e) {
        if (e & 1) r = mulw(r, b, m);
        b = mulw(b, b, m);
        e >>= 1;
    }
    return r;
}

// Residue -> four balanced signed limbs (see the header comment).
__device__ __forceinline__ void split_limbs4(uint32_t x, uint32_t p, int (&l)[4]) {
    int64_t r = (int64_t)x <= kWideWindow ? (int64_t)x : (int64_t)x - (int64_t)p;
#pragma unroll
    for (int i = 0; i < 3; i++) {
        const int64_t h = (r + 128) >> 8;  // arithmetic shift: floor
        l[i] = (int)(r - (h << 8));
        r = h;
    }
    l[3] = (int)r;
}

// The residue of S = sum_d 2^{8d} D_d from the seven int32 diagonal sums:
// S = S_lo + 2^32 S_hi with S_lo = D0 + 2^8 D1 + 2^16 D2 + 2^24 D3 (|S_lo| <
// 2^31 (1 + 2^8 + 2^16 + 2^24) < 2^56) and S_hi = D4 + 2^8 D5 + 2^16 D6
// (|S_hi| < 2^48), both exact in 64 bits; each is shifted by 2^57 into
// [0, 2^58), reduced, and the residue of 2^57 taken off.
__device__ __forceinline__ uint32_t combine7(int d0, int d1, int d2, int d3, int d4, int d5, int d6,
                                             const Mod64 &m) {
    const int64_t lo = (int64_t)d0 + (int64_t)d1 * 256 + (int64_t)d2 * 65536 + (int64_t)d3 * 16777216;
    const int64_t hi = (int64_t)d4 + (int64_t)d5 * 256 + (int64_t)d6 * 65536;
    const int64_t bias = (int64_t)1 << 57;
    const uint32_t rl = subw(reduce64((uint64_t)(lo + bias), m), m.c57, m.p);
    const uint32_t rh = subw(reduce64((uint64_t)(hi + bias), m), m.c57, m.p);
    return addw(rl, mulw(rh, m.c32, m), m.p);
}

}  // namespace flw
