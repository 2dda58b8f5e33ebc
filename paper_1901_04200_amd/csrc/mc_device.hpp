// Device building blocks shared by the Monte Carlo kernels: the counter-based
// random stream and wavefront reductions.  gfx950 (CDNA4), wave64.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace mcaad {

constexpr int kWave = 64;
constexpr int kBlock = 256;          // 4 waves per workgroup
constexpr int kWavesPerBlock = kBlock / kWave;

// a ^ b ^ k in one VALU instruction (k uniform, in a scalar register):
// gfx950's three-input bitwise op with truth table 0x96 (odd parity), which
// is symmetric in its operands.  (gfx9 has no v_xor3_b32.)
__device__ __forceinline__ uint32_t xor3_vvs(uint32_t a, uint32_t b, uint32_t k)
{
    uint32_t r;
    asm("v_bitop3_b32 %0, %1, %2, %3 bitop3:0x96" : "=v"(r) : "v"(a), "v"(b), "s"(k));
    return r;
}

// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11): ten rounds of two
// 32x32->64 multiplies on the even words, the high halves xor-ed with the odd
// words and the round key, the key bumped by the Weyl constants after every
// round.  The key is uniform across the wavefront, so its schedule lives in
// scalar registers.  With counter (call, path, inst, 0) only the path word
// differs per lane, so the first rounds are partly uniform and are left to
// the compiler's scalar/vector split; from the fourth round on every word
// differs per lane and each new word is one v_mad_u64_u32 half plus one
// three-way xor.
__device__ __forceinline__ void philox4x32_10(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                              uint32_t k0, uint32_t k1, uint32_t out[4])
{
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)c0;
        const uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)c2;
        uint32_t n0, n2;
        if (r >= 3) {
            n0 = xor3_vvs((uint32_t)(p1 >> 32), c1, k0);
            n2 = xor3_vvs((uint32_t)(p0 >> 32), c3, k1);
        } else {
            n0 = (uint32_t)(p1 >> 32) ^ c1 ^ k0;
            n2 = (uint32_t)(p0 >> 32) ^ c3 ^ k1;
        }
        c1 = (uint32_t)p1;
        c3 = (uint32_t)p0;
        c0 = n0;
        c2 = n2;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    out[0] = c0;
    out[1] = c1;
    out[2] = c2;
    out[3] = c3;
}

// Uniform in (0,1): ((w >> 9) + 0.5) * 2^-23, exact in FP32 and FP64.
__device__ __forceinline__ float uniform_f32(uint32_t w)
{
    return ((float)(w >> 9) + 0.5f) * 0x1p-23f;
}

__device__ __forceinline__ double uniform_f64(uint32_t w)
{
    return ((double)(w >> 9) + 0.5) * 0x1p-23;
}

// Box-Muller on one pair: rho = sqrt(-2 ln u0), (rho cos 2pi u1, rho sin 2pi u1).
// FP32 uses the hardware transcendentals: v_log_f32 (log2), v_sqrt_f32 and
// v_sin/v_cos_f32, whose argument is in revolutions, so 2 pi u1 needs no
// multiply and no range reduction.
__device__ __forceinline__ void box_muller(float u0, float u1, float &z0, float &z1)
{
    const float m2ln2 = -1.3862943611198906f;   // -2 ln 2
    const float rho = __builtin_amdgcn_sqrtf(m2ln2 * __builtin_amdgcn_logf(u0));
    z0 = rho * __builtin_amdgcn_cosf(u1);
    z1 = rho * __builtin_amdgcn_sinf(u1);
}

__device__ __forceinline__ void box_muller(double u0, double u1, double &z0, double &z1)
{
    const double rho = sqrt(-2.0 * log(u0));
    double s, c;
    sincospi(2.0 * u1, &s, &c);
    z0 = rho * c;
    z1 = rho * s;
}

// Four normals of one Philox call (counter (call, path, inst, 0)).
template <typename R>
__device__ __forceinline__ void normals4(uint32_t call, uint32_t path, uint32_t inst, uint32_t k0, uint32_t k1,
                                         R z[4])
{
    uint32_t w[4];
    philox4x32_10(call, path, inst, 0u, k0, k1, w);
    if constexpr (sizeof(R) == 4) {
        box_muller(uniform_f32(w[0]), uniform_f32(w[1]), z[0], z[1]);
        box_muller(uniform_f32(w[2]), uniform_f32(w[3]), z[2], z[3]);
    } else {
        box_muller(uniform_f64(w[0]), uniform_f64(w[1]), z[0], z[1]);
        box_muller(uniform_f64(w[2]), uniform_f64(w[3]), z[2], z[3]);
    }
}

// Butterfly sum over the 64 lanes of a wavefront; every lane receives the
// total.  The pairing order is fixed, so the FP64 result is deterministic.
__device__ __forceinline__ double wave_sum(double v)
{
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, kWave);
    return v;
}

}  // namespace mcaad
