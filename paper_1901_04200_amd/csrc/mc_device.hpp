// Device building blocks shared by the Monte Carlo kernels: the counter-based
// random stream and wavefront reductions.  gfx950 (CDNA4), wave64.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace mcaad {

constexpr int kWave = 64;
constexpr int kBlock = 256;          // 4 waves per workgroup
constexpr int kWavesPerBlock = kBlock / kWave;

// Read element i of a table that no kernel writes while the reading kernel
// runs (instrument tables, seeds): through the constant address space, so a
// uniform index becomes a scalar load even when the table's pointer was itself
// loaded from memory (batched instances), where the compiler cannot prove it.
template <typename T>
__device__ __forceinline__ T ldc(const T *p, int i)
{
    return ((const __attribute__((address_space(4))) T *)p)[i];
}

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
// FP32: one v_alignbit_b32 builds the float 1 + (w >> 9) 2^-23 (exponent bits
// 0x7F above the 23 high bits of w), and subtracting 1 - 2^-24 is exact
// (Sterbenz), so the value is the same as the textbook formula's.
__device__ __forceinline__ float uniform_f32(uint32_t w)
{
    return __uint_as_float(__builtin_amdgcn_alignbit(0x7Fu, w, 9u)) - 0x1.fffffep-1f;
}

__device__ __forceinline__ double uniform_f64(uint32_t w)
{
    return ((double)(w >> 9) + 0.5) * 0x1p-23;
}

// Box-Muller on one pair, scaled by sqrt(h): rho = sqrt(-2 h ln u0),
// (rho cos 2pi u1, rho sin 2pi u1).  bm is the constant under the root:
// -2 ln(2) h in FP32, which multiplies v_log_f32 (log2), and -2 h in FP64.
// FP32 uses the hardware transcendentals: v_log_f32, v_sqrt_f32 and
// v_sin/v_cos_f32, whose argument is in revolutions, so 2 pi u1 needs no
// multiply and no range reduction.
template <typename R>
__device__ __forceinline__ R box_muller_scale(double h)
{
    if constexpr (sizeof(R) == 4) return (float)(-2.0 * 0.69314718055994530942 * h);
    else return -2.0 * h;
}

__device__ __forceinline__ void box_muller(float u0, float u1, float bm, float &z0, float &z1)
{
    const float rho = __builtin_amdgcn_sqrtf(bm * __builtin_amdgcn_logf(u0));
    z0 = rho * __builtin_amdgcn_cosf(u1);
    z1 = rho * __builtin_amdgcn_sinf(u1);
}

__device__ __forceinline__ void box_muller(double u0, double u1, double bm, double &z0, double &z1)
{
    const double rho = sqrt(bm * log(u0));
    double s, c;
    sincospi(2.0 * u1, &s, &c);
    z0 = rho * c;
    z1 = rho * s;
}

// Four normals of one Philox call (counter (call, path, inst, 0)), each
// scaled by sqrt(h) for bm = box_muller_scale(h).
template <typename R>
__device__ __forceinline__ void normals4(uint32_t call, uint32_t path, uint32_t inst, uint32_t k0, uint32_t k1, R bm,
                                         R z[4])
{
    uint32_t w[4];
    philox4x32_10(call, path, inst, 0u, k0, k1, w);
    if constexpr (sizeof(R) == 4) {
        box_muller(uniform_f32(w[0]), uniform_f32(w[1]), bm, z[0], z[1]);
        box_muller(uniform_f32(w[2]), uniform_f32(w[3]), bm, z[2], z[3]);
    } else {
        box_muller(uniform_f64(w[0]), uniform_f64(w[1]), bm, z[0], z[1]);
        box_muller(uniform_f64(w[2]), uniform_f64(w[3]), bm, z[2], z[3]);
    }
}

// ---------------------------------------------------------------------------
// Wavefront sums of FP64 values, with no LDS traffic: the two halves of the
// wave and the row pairs (rows = 16 lanes) are exchanged with gfx950's
// v_permlane32_swap / v_permlane16_swap, the steps inside a row with DPP
// moves.  A double moves as two 32-bit halves.
//
// Every sum follows one fixed tree: lane l with l+32, then rows 2r with
// 2r+1, then lane i of a row with lane 15-i, then i with 7-i inside each
// half row, then quad partners 2 apart, then 1 apart.  Each step adds two
// operands that are exchanged between partner lanes, so partners compute the
// same sum (FP64 addition commutes) and the result is deterministic and
// identical in every lane that holds it.
// ---------------------------------------------------------------------------
namespace lanes {

__device__ __forceinline__ uint32_t lo32(double v) { return (uint32_t)__builtin_bit_cast(uint64_t, v); }
__device__ __forceinline__ uint32_t hi32(double v) { return (uint32_t)(__builtin_bit_cast(uint64_t, v) >> 32); }
__device__ __forceinline__ double join(uint32_t lo, uint32_t hi)
{
    return __builtin_bit_cast(double, ((uint64_t)hi << 32) | lo);
}

constexpr int kQuadXor1 = 0xB1;        // quad_perm [1,0,3,2]
constexpr int kQuadXor2 = 0x4E;        // quad_perm [2,3,0,1]
constexpr int kRowHalfMirror = 0x141;  // lane i of each 8 reads lane 7-i
constexpr int kRowMirror = 0x140;      // lane i of each 16 reads lane 15-i

template <int CTRL>
__device__ __forceinline__ double dpp(double v)
{
    return join(__builtin_amdgcn_update_dpp(0u, lo32(v), CTRL, 0xF, 0xF, false),
                __builtin_amdgcn_update_dpp(0u, hi32(v), CTRL, 0xF, 0xF, false));
}

// v_permlane32_swap(a, b) exchanges lanes 32..63 of a with lanes 0..31 of b:
// afterwards a = (a's lanes 0..31, b's lanes 0..31) and b = (a's lanes
// 32..63, b's lanes 32..63), so a + b is, in lanes 0..31, the sum of a over
// lanes l and l+32, and in lanes 32..63 the sum of b over lanes l-32 and l.
__device__ __forceinline__ double fold32(double a, double b)
{
    const auto L = __builtin_amdgcn_permlane32_swap(lo32(a), lo32(b), false, false);
    const auto H = __builtin_amdgcn_permlane32_swap(hi32(a), hi32(b), false, false);
    return join(L[0], H[0]) + join(L[1], H[1]);
}

// v_permlane16_swap(a, b) exchanges the odd rows of a with the even rows of
// b: afterwards each row pair of a holds a's even row then b's even row, and
// of b a's odd row then b's odd row, so a + b is, in even rows, the sum of a
// over the row pair, and in odd rows the sum of b over the row pair.
__device__ __forceinline__ double fold16(double a, double b)
{
    const auto L = __builtin_amdgcn_permlane16_swap(lo32(a), lo32(b), false, false);
    const auto H = __builtin_amdgcn_permlane16_swap(hi32(a), hi32(b), false, false);
    return join(L[0], H[0]) + join(L[1], H[1]);
}

// the steps inside a row; the caller has already folded halves and row pairs
__device__ __forceinline__ double row_tail(double v)
{
    v += dpp<kRowHalfMirror>(v);
    v += dpp<kQuadXor2>(v);
    v += dpp<kQuadXor1>(v);
    return v;
}

}  // namespace lanes

// Sum over the 64 lanes; every lane receives the total.  Must be called with
// all 64 lanes active.
__device__ __forceinline__ double wave_sum(double v)
{
    v = lanes::fold32(v, v);
    v = lanes::fold16(v, v);
    v += lanes::dpp<lanes::kRowMirror>(v);
    return lanes::row_tail(v);
}

// Eight sums at once: a[j] summed over the 64 lanes for j = 0..7, at the
// cost of about ten single-value steps instead of 48.  The total of a[j] is
// returned in the eight lanes 8j..8j+7 (j = lane / 8); it is bitwise the
// value wave_sum(a[j]) gives.  Must be called with all 64 lanes active.
__device__ __forceinline__ double wave_sum8(const double a[8])
{
    const int lane = (int)(threadIdx.x & (kWave - 1));
    double b[4], c[2];
#pragma unroll
    for (int i = 0; i < 4; ++i) b[i] = lanes::fold32(a[i], a[i + 4]);        // lanes 0..31: a[i]; 32..63: a[i+4]
#pragma unroll
    for (int i = 0; i < 2; ++i) c[i] = lanes::fold16(b[i], b[i + 2]);        // even rows: b[i]; odd rows: b[i+2]
    const bool up = lane & 8;                                                 // lanes 8..15 of a row keep c[1]
    const double keep = up ? c[1] : c[0];
    const double send = up ? c[0] : c[1];
    return lanes::row_tail(keep + lanes::dpp<lanes::kRowMirror>(send));
}

// Node-adjoint slices: `rows` rows of kBlock FP32 values in LDS, one column
// per lane (slices[q * kBlock + tid]).  Adds the sum over the workgroup's
// lanes of row q to dst[q] (FP64) and clears the slices.  Wave w takes rows
// w, w + 4, ...: each lane loads four neighbouring columns of the row (one
// 16-byte read in FP32, two in FP64: the wave covers the whole row), adds them
// in the slices' precision, and the
// wave sums the 64 lane values in FP64 along wave_sum's fixed tree, so the
// sums are deterministic.  A rolled loop keeps the register footprint small
// where this is inlined into a register-heavy sweep.  Called by all threads of
// the workgroup (uniform control flow); slices must be 16-byte aligned.
template <typename T>
__device__ __forceinline__ void flush_slices(T *slices, int rows, double *dst)
{
    const int tid = threadIdx.x;
    const int lane = tid & (kWave - 1);
    const int wave = tid / kWave;
    __syncthreads();
#pragma unroll 1
    for (int q = wave; q < rows; q += kWavesPerBlock) {
        T *cell = slices + q * kBlock + 4 * lane;
        double t;
        if constexpr (sizeof(T) == 4) {
            const float4 v = *reinterpret_cast<float4 *>(cell);
            *reinterpret_cast<float4 *>(cell) = make_float4(0.f, 0.f, 0.f, 0.f);
            t = (double)((v.x + v.y) + (v.z + v.w));
        } else {
            const double2 v0 = reinterpret_cast<double2 *>(cell)[0], v1 = reinterpret_cast<double2 *>(cell)[1];
            reinterpret_cast<double2 *>(cell)[0] = make_double2(0.0, 0.0);
            reinterpret_cast<double2 *>(cell)[1] = make_double2(0.0, 0.0);
            t = (v0.x + v0.y) + (v1.x + v1.y);
        }
        t = wave_sum(t);
        if (lane == 0) dst[q] += t;
    }
    __syncthreads();
}

// Wave totals of the discounted call payoffs disc[k] max(S - strike[k], 0),
// k in [kb, ke) (the instruments maturing at one date), eight instruments per
// wave_sum8; lanes with active == false add 0.  Total k goes to out[k], or is
// added to it when `add` (a lane's later paths).
__device__ __forceinline__ void payoff_sums(const double *__restrict__ strike, const double *__restrict__ disc,
                                            double S, bool active, int lane, int kb, int ke, double *out,
                                            bool add = false)
{
    for (int k0 = kb; k0 < ke; k0 += 8) {
        double a[8];
#pragma unroll
        for (int i = 0; i < 8; ++i) {
            const int k = k0 + i < ke ? k0 + i : ke - 1;   // stays inside the table
            a[i] = active && k0 + i < ke ? ldc(disc, k) * fmax(S - ldc(strike, k), 0.0) : 0.0;
        }
        const double y = wave_sum8(a);
        const int k = k0 + (lane >> 3);
        if ((lane & 7) == 0 && k < ke) out[k] = add ? out[k] + y : y;
    }
}

}  // namespace mcaad
