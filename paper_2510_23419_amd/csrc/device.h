// device.h — device-side building blocks of the p-bit sweep for gfx950.
//
// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11) keyed by the anneal seed,
// and the integer heat-bath decision of the p-bit law m = sgn(tanh(beta I) - u)
// (paper Sec. 1.2.1, Eq. 2) through a per-sweep uint32 minority-threshold row.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace pbit {

// Philox4x32-10 block function.  The key words are wave-uniform in every
// caller, so the key schedule runs on the scalar unit; each round is two
// 32x32->64 products (v_mad_u64_u32) and two three-way XORs.
struct Block4 {
    uint32_t w[4];
};

__device__ __forceinline__ Block4 philox(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                         uint32_t k0, uint32_t k1)
{
#pragma unroll
    for (int round = 0; round < 10; ++round) {
        const uint64_t p = (uint64_t)c0 * 0xD2511F53u;
        const uint64_t q = (uint64_t)c2 * 0xCD9E8D57u;
        // three-input XORs as single v_bitop3_b32 (truth table 0x96 = a ^ b ^ c)
        const uint32_t n0 = __builtin_amdgcn_bitop3_b32((uint32_t)(q >> 32), c1, k0, 0x96);
        const uint32_t n2 = __builtin_amdgcn_bitop3_b32((uint32_t)(p >> 32), c3, k1, 0x96);
        c1 = (uint32_t)q;
        c3 = (uint32_t)p;
        c0 = n0;
        c2 = n2;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    Block4 b;
    b.w[0] = c0; b.w[1] = c1; b.w[2] = c2; b.w[3] = c3;
    return b;
}

// Counter domains.
constexpr uint32_t kDomainSweep = 0;
constexpr uint32_t kDomainInit = 1;

// Heat-bath decision for field I, minority threshold T = Tm(beta, |I|) and
// uniform word w: -s if x < T else s, with s = sign(I) (+1 at I = 0) and
// x = ~w for I >= 0, w for I < 0.
__device__ __forceinline__ int8_t decide(int32_t I, uint32_t T, uint32_t w)
{
    const bool pos = I >= 0;
    const uint32_t x = pos ? ~w : w;
    const bool minority = x < T;
    return (pos != minority) ? (int8_t)1 : (int8_t)-1;
}

// v_writelane_b32: lane `lane` of `old` takes the wave-uniform `val` (the
// compiler's intrinsic, bound by name: hip exposes no builtin for it).
__device__ int lane_write(int val, int lane, int old) __asm("llvm.amdgcn.writelane.i32");

// q = n / d and r = n % d for 0 <= n < 2^22 and 1 <= d < 2^10 from a float
// reciprocal: the estimate is within one of the quotient and is corrected.
__device__ __forceinline__ int div_small(int n, int d, float inv, int &r)
{
    int q = (int)((float)n * inv);
    int rr = n - q * d;
    if (rr < 0) {
        q -= 1;
        rr += d;
    } else if (rr >= d) {
        q += 1;
        rr -= d;
    }
    r = rr;
    return q;
}

// A load from global memory through a pointer the compiler cannot place (one read
// out of a job descriptor, say): issued as a global load, counted by vmcnt alone.
// Through a generic pointer it would be a flat load, which also counts against
// lgkmcnt, so that every wait for an LDS read would wait for it as well.
template <typename T>
__device__ __forceinline__ T load_global(const void *p)
{
    return *(const __attribute__((address_space(1))) T *)p;
}

typedef int v4i_t __attribute__((ext_vector_type(4)));

// Spin bits widened for the int8 MFMA: the K bytes that lane half g of a 32x32x32
// fragment holds (dword j byte i = K position 16 g + 4 j + i) from a word w of
// 32 spin bits (set = -1): byte i of dword j holds bit 8 i + 4 g + j of w as the
// value 0 or 2^j.  Couplings stored in that site order and scaled by 2^(3 - j)
// make every product 8 J b.
__device__ __forceinline__ v4i_t widen_bits(uint32_t w, int g)
{
    const uint32_t x = w >> (4 * g);
    v4i_t a;
    a[0] = (int)(x & 0x01010101u);
    a[1] = (int)(x & 0x02020202u);
    a[2] = (int)(x & 0x04040404u);
    a[3] = (int)(x & 0x08080808u);
    return a;
}

// Initial spin from a domain-1 word.
__device__ __forceinline__ int8_t init_spin(uint32_t w)
{
    return w < 0x80000000u ? (int8_t)1 : (int8_t)-1;
}

}  // namespace pbit
