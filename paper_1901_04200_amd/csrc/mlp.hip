// Learned surrogate of the calibration map theta -> E y on gfx950: forward
// pass with input tangents (the network's Jacobian), price + gradient loss,
// double backpropagation and Adam.  Matrix products run on bf16 MFMA
// (v_mfma_f32_32x32x16_bf16) with FP32 accumulation; everything elementwise
// is FP32; the loss is summed in FP64 in a fixed order.  C ABI declared in
// include/mcaad_surrogate.h.
//
// Row layout of every activation matrix: R = (n_in + 1) * Bp rows, row
// t * Bp + b holds the primal values of sample b (t = 0) or its tangent
// along input t - 1 (t >= 1); columns are the layer's units.  One product
// with the layer's weights therefore advances the primal pass and all n_in
// tangent passes together.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <string>
#include <vector>

#include "../../include/mcaad_surrogate.h"

namespace {

typedef __attribute__((ext_vector_type(8))) __bf16 bf16x8;
typedef __attribute__((ext_vector_type(16))) float f32x16;

constexpr int kThreads = 256;
constexpr int BM = 128, BN = 64, BK = 32, LDK = BK + 8;   // LDS row stride 80 bytes
constexpr int LDT = 64;                                   // transposed operands: 128-byte rows

// LDS element index of (row, k) for an operand staged with k contiguous (KC)
// or transposed on the way in (k < BK; a k-aligned group of 8 stays contiguous).
template <bool KC>
__device__ __forceinline__ int lds_idx(int row, int k)
{
    if constexpr (KC) return row * LDK + k;
    else return row * LDT + ((k + 8 * ((row + (row >> 3)) & 7)) & (LDT - 1));
}
constexpr int kOutPad = 64;                               // output units padded to one N tile
constexpr int kMaxSplits = 64;

// FP32 -> bf16 with round-to-nearest-even (finite inputs).
__device__ __forceinline__ uint16_t f2bf(float f)
{
    uint32_t u = __float_as_uint(f);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

__device__ __forceinline__ float sigm(float z) { return 1.0f / (1.0f + __expf(-z)); }

// ---------------------------------------------------------------------------
// C[z] (M x N, FP32) = sum over split z of A(m,k) B(k,n), bf16 operands.
//   A(m,k) = A_KC ? A[m*lda + k] : A[k*lda + m]
//   B(k,n) = B_KC ? B[n*ldb + k] : B[k*ldb + n]
// Tiles 128 x 64 x 32; wave w owns rows 32w..32w+31 and both 32-column
// blocks.  Operands are staged in LDS with k contiguous, so every MFMA
// operand is one 16-byte LDS read (8 bf16 along k for one row / column).
// An operand stored with k contiguous keeps its rows (stride LDK); one stored
// with k as the slow index is transposed element by element on its way into
// LDS, into 128-byte rows whose eight 16-byte groups are rotated by
// (row + row / 8) mod 8: the 16 rows that one such store instruction writes
// (8 apart) and the 16 rows that an operand read touches then spread over
// the LDS banks instead of meeting in one.
// Two LDS buffers and two register sets: the global loads of the next two
// k-tiles are in flight while the current tile's MFMAs run; the next one is
// written to the other buffer after them, one barrier per k-tile.  The k
// order of the accumulation is the plain one, so results do not depend on
// the pipelining.
// Requires M % 128 == 0, N % 64 == 0, K % 32 == 0, k_split % 32 == 0.
// ---------------------------------------------------------------------------
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));   // 16 bytes
constexpr int kAChunks = BM * BK / 8 / kThreads;   // 16-byte A pieces per thread and k-tile (2)
static_assert(BN * BK / 8 == kThreads, "one 16-byte B piece per thread and k-tile");

template <bool A_KC>
__device__ __forceinline__ void gemm_load_a(const uint16_t *__restrict__ A, int lda, int m0, int k0, u32x4 *ra)
{
#pragma unroll
    for (int i = 0; i < kAChunks; ++i) {
        const int c = threadIdx.x + i * kThreads;
        if constexpr (A_KC) {
            const int r = c / (BK / 8), kc = c % (BK / 8);
            ra[i] = *(const u32x4 *)(A + (int64_t)(m0 + r) * lda + k0 + kc * 8);
        } else {
            const int kr = c / (BM / 8), mc = c % (BM / 8);
            ra[i] = *(const u32x4 *)(A + (int64_t)(k0 + kr) * lda + m0 + mc * 8);
        }
    }
}

template <bool A_KC>
__device__ __forceinline__ void gemm_store_a(uint16_t *sA, const u32x4 *ra)
{
#pragma unroll
    for (int i = 0; i < kAChunks; ++i) {
        const int c = threadIdx.x + i * kThreads;
        if constexpr (A_KC) {
            const int r = c / (BK / 8), kc = c % (BK / 8);
            *(u32x4 *)(sA + r * LDK + kc * 8) = ra[i];
        } else {
            const int kr = c / (BM / 8), mc = c % (BM / 8);
            const uint16_t *e = (const uint16_t *)&ra[i];
#pragma unroll
            for (int q = 0; q < 8; ++q) sA[lds_idx<false>(mc * 8 + q, kr)] = e[q];
        }
    }
}

template <bool B_KC>
__device__ __forceinline__ u32x4 gemm_load_b(const uint16_t *__restrict__ B, int ldb, int n0, int k0)
{
    const int c = threadIdx.x;
    if constexpr (B_KC) {
        const int r = c / (BK / 8), kc = c % (BK / 8);
        return *(const u32x4 *)(B + (int64_t)(n0 + r) * ldb + k0 + kc * 8);
    } else {
        const int kr = c / (BN / 8), nc = c % (BN / 8);
        return *(const u32x4 *)(B + (int64_t)(k0 + kr) * ldb + n0 + nc * 8);
    }
}

template <bool B_KC>
__device__ __forceinline__ void gemm_store_b(uint16_t *sB, u32x4 rb)
{
    const int c = threadIdx.x;
    if constexpr (B_KC) {
        const int r = c / (BK / 8), kc = c % (BK / 8);
        *(u32x4 *)(sB + r * LDK + kc * 8) = rb;
    } else {
        const int kr = c / (BN / 8), nc = c % (BN / 8);
        const uint16_t *e = (const uint16_t *)&rb;
#pragma unroll
        for (int q = 0; q < 8; ++q) sB[lds_idx<false>(nc * 8 + q, kr)] = e[q];
    }
}

template <bool A_KC, bool B_KC>
__global__ __launch_bounds__(kThreads) void k_gemm(const uint16_t *__restrict__ A, int lda,
                                                   const uint16_t *__restrict__ B, int ldb, float *__restrict__ C,
                                                   int ldc, int64_t split_stride, int K, int k_split)
{
    __shared__ __attribute__((aligned(16))) uint16_t sA[2][BM * (A_KC ? LDK : LDT)];
    __shared__ __attribute__((aligned(16))) uint16_t sB[2][BN * (B_KC ? LDK : LDT)];
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    // Tile of this workgroup.  Workgroups go to the 8 XCDs (each with its own
    // L2) in turn by linear id, so the logical tiles are dealt out in 8
    // contiguous runs, N-tile fastest: an XCD takes all column tiles of its
    // row tiles and whole k-splits, and the A and B panels they share are read
    // from memory once per XCD instead of once per workgroup.
    const int nM = gridDim.x, nN = gridDim.y;
    const int total = nM * nN * gridDim.z;
    const int lin = blockIdx.x + nM * (blockIdx.y + nN * blockIdx.z);
    const int lid = total % 8 == 0 ? (lin % 8) * (total / 8) + lin / 8 : lin;
    const int tn = lid % nN, tm = (lid / nN) % nM, tz = lid / (nN * nM);
    const int m0 = tm * BM;
    const int n0 = tn * BN;
    const int kbeg = tz * k_split;
    const int kend = min(K, kbeg + k_split);
    f32x16 acc0, acc1;
#pragma unroll
    for (int i = 0; i < 16; ++i) {
        acc0[i] = 0.f;
        acc1[i] = 0.f;
    }
    // k-tile t (k = kbeg + t BK) is multiplied from LDS buffer t % 2 while
    // the global loads of tiles t + 1 and t + 2 are in flight in the two
    // register sets (set (t + 1) % 2 holds tile t + 1); after tile t's MFMAs
    // tile t + 1 goes to the other LDS buffer (last read before the previous
    // barrier) and tile t + 3 is requested into the set just emptied.
    const int nt = kbeg < kend ? (kend - kbeg + BK - 1) / BK : 0;
    u32x4 ra0[kAChunks], rb0, ra1[kAChunks], rb1;
    auto mma = [&](const uint16_t *a_s, const uint16_t *b_s) {
#pragma unroll
        for (int kk = 0; kk < BK; kk += 16) {
            const int ko = kk + 8 * (lane >> 5);
            const bf16x8 a = *(const bf16x8 *)(a_s + lds_idx<A_KC>(wave * 32 + (lane & 31), ko));
            const bf16x8 b0 = *(const bf16x8 *)(b_s + lds_idx<B_KC>(lane & 31, ko));
            const bf16x8 b1 = *(const bf16x8 *)(b_s + lds_idx<B_KC>(32 + (lane & 31), ko));
            acc0 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b0, acc0, 0, 0, 0);
            acc1 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b1, acc1, 0, 0, 0);
        }
    };
    if (nt > 0) {
        gemm_load_a<A_KC>(A, lda, m0, kbeg, ra0);
        rb0 = gemm_load_b<B_KC>(B, ldb, n0, kbeg);
        gemm_store_a<A_KC>(sA[0], ra0);
        gemm_store_b<B_KC>(sB[0], rb0);
    }
    if (nt > 1) {
        gemm_load_a<A_KC>(A, lda, m0, kbeg + BK, ra1);
        rb1 = gemm_load_b<B_KC>(B, ldb, n0, kbeg + BK);
    }
    if (nt > 2) {
        gemm_load_a<A_KC>(A, lda, m0, kbeg + 2 * BK, ra0);
        rb0 = gemm_load_b<B_KC>(B, ldb, n0, kbeg + 2 * BK);
    }
    __syncthreads();
    for (int t = 0; t < nt; t += 2) {
        // even tile t: LDS buffer 0; set 1 holds tile t + 1, set 0 tile t + 2
        mma(sA[0], sB[0]);
        if (t + 1 < nt) {
            gemm_store_a<A_KC>(sA[1], ra1);
            gemm_store_b<B_KC>(sB[1], rb1);
        }
        if (t + 3 < nt) {
            gemm_load_a<A_KC>(A, lda, m0, kbeg + (t + 3) * BK, ra1);
            rb1 = gemm_load_b<B_KC>(B, ldb, n0, kbeg + (t + 3) * BK);
        }
        __syncthreads();
        if (t + 1 >= nt) break;
        // odd tile t + 1: LDS buffer 1; set 0 holds tile t + 2, set 1 tile t + 3
        mma(sA[1], sB[1]);
        if (t + 2 < nt) {
            gemm_store_a<A_KC>(sA[0], ra0);
            gemm_store_b<B_KC>(sB[0], rb0);
        }
        if (t + 4 < nt) {
            gemm_load_a<A_KC>(A, lda, m0, kbeg + (t + 4) * BK, ra0);
            rb0 = gemm_load_b<B_KC>(B, ldb, n0, kbeg + (t + 4) * BK);
        }
        __syncthreads();
    }
    float *Cz = C + (int64_t)tz * split_stride;
    const int col = n0 + (lane & 31);
#pragma unroll
    for (int i = 0; i < 16; ++i) {
        const int row = m0 + wave * 32 + (i >> 2) * 8 + (lane >> 5) * 4 + (i & 3);
        Cz[(int64_t)row * ldc + col] = acc0[i];
        Cz[(int64_t)row * ldc + col + 32] = acc1[i];
    }
}

// out[i*ldo + j] = sum_z part[z][i][j], j < ncols: eight threads per output,
// thread q adding splits q, q + 8, ... in order (all its loads in flight
// together), then the eight sums in a fixed tree; 32 outputs per workgroup.
__global__ __launch_bounds__(kThreads) void k_split_reduce(const float *__restrict__ part, int S, int M, int N,
                                                           float *__restrict__ out, int ldo, int ncols)
{
    __shared__ float sh[kThreads];
    const int q = threadIdx.x & 7;
    const int64_t o = (int64_t)blockIdx.x * (kThreads / 8) + (threadIdx.x >> 3);
    const bool live = o < (int64_t)M * ncols;
    const int i = live ? (int)(o / ncols) : 0, j = live ? (int)(o % ncols) : 0;
    float s = 0.f;
    if (live) {
#pragma unroll 8
        for (int z = q; z < S; z += 8) s += part[(int64_t)z * M * N + (int64_t)i * N + j];
    }
    sh[threadIdx.x] = s;
    __syncthreads();
    if (q == 0 && live) {
        const float *v = sh + threadIdx.x;
        out[(int64_t)i * ldo + j] = ((v[0] + v[1]) + (v[2] + v[3])) + ((v[4] + v[5]) + (v[6] + v[7]));
    }
}

// ---------------------------------------------------------------------------
// Row-block products fused with the elementwise work around them (the
// training step and large-batch inference, n_in + 1 <= kRowsMaxNR).
//
// A workgroup of NR = n_in + 1 waves takes 32 samples (b0 .. b0 + 31) and 64
// output columns (n0 .. n0 + 63) of Z = A W^T across all NR row blocks of the
// activation layout: wave t computes rows t Bp + b0 .. t Bp + b0 + 31, so the
// primal values that a tangent row's elementwise work needs are produced in
// the same workgroup and meet in LDS.  Operand staging, k order and MFMA
// (v_mfma_f32_32x32x16_bf16, FP32 accumulation from zero) are k_gemm's, so the
// pre-activations are those k_gemm gives.  Epilogues:
//   kEpiStore   Z (FP32 [NR Bp][ldz]) as k_gemm (inference output layer)
//   kEpiActFwd  hidden layer: z = acc + bias, activations SiLU(z) and
//               SiLU'(z) u (bf16, the next product's operand), the primal
//               pre-activations z (FP32) and the tangent pre-activations u
//               (bf16) for the backward pass
//   kEpiActBwd  adjoint of a hidden layer's activation from the next layer's
//               input adjoint (double backprop):
//                 zbar = hbar SiLU'(z) + sum_t tbar_t u_t SiLU''(z),
//                 ubar_t = tbar_t SiLU'(z)
//               written as bf16 operands, plus the column partials of zbar
//               (the layer's bias gradient)
//   kEpiL1Bwd   the same for layer 1 (u_t = row t of W1), reduced at once to
//               the workgroup's column partials of W1bar[t][j] =
//               sum_b (x_bt zbar_bj + ubar_t,bj) and b1bar[j] = sum_b zbar_bj
// Column partials over the workgroup's 32 samples go to part[blk][...]
// (blk = b0 / 32), summed over workgroups by k_chunk_reduce in a fixed order.
// ---------------------------------------------------------------------------
constexpr int kRowsMaxNR = 8;
enum { kEpiStore = 0, kEpiActFwd = 1, kEpiActBwd = 3, kEpiL1Bwd = 4 };

struct RowsArgs {
    const uint16_t *A;      // [NR Bp][K] bf16, k contiguous
    const uint16_t *W;      // [N][K] bf16, k contiguous
    int Bp, K, N;           // samples per row block, k extent, output columns (multiple of 64)
    float *Z;               // kEpiStore: [NR Bp][N]
    const float *bias;      // kEpiActFwd: [N]
    uint16_t *Aout;         // kEpiActFwd: [NR Bp][N]
    float *Zp;              // kEpiActFwd: [Bp][N]
    uint16_t *U;            // kEpiActFwd: [(NR - 1) Bp][N]
    const float *Zp_in;     // kEpiActBwd, kEpiL1Bwd: [Bp][N] this layer's primal pre-activations
    const uint16_t *U_in;   // kEpiActBwd: [(NR - 1) Bp][N]
    const float *W1;        // kEpiL1Bwd: [NR - 1][N] (FP32)
    const float *X;         // kEpiL1Bwd: [Bp][NR - 1] normalised inputs
    uint16_t *Zbar;         // kEpiActBwd: [NR Bp][N]
    float *part;            // column partials [Bp / 32][ncols]
};

__device__ __forceinline__ float bf2f(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

// Sum of v over the 32 rows of this wave's tile for column (lane & 31) (one
// accumulator of the 32x32 MFMA: the lane holds 16 of the column's rows, its
// partner lane ^ 32 the other 16); every lane gets its column's total.
__device__ __forceinline__ float tile_colsum(const float *v)
{
    float s = 0.f;
#pragma unroll
    for (int i = 0; i < 16; ++i) s += v[i];
    return s + __shfl_xor(s, 32);
}

template <int NR, int EPI>
__global__ __launch_bounds__(NR * 64) void k_rows(RowsArgs a)
{
    constexpr int NT = NR * 64;
    constexpr int kBC = (256 + NT - 1) / NT;   // 16-byte B pieces per thread and k-tile
    // operand tiles during the products; the epilogue's exchange area afterwards
    constexpr int kOpBytes = 2 * (2 * NR * 32 * LDK + 2 * BN * LDK);
    constexpr int kEpBytes = (NR + 1) * 32 * 64 * 4;
    __shared__ __attribute__((aligned(16))) unsigned char smem[kOpBytes > kEpBytes ? kOpBytes : kEpBytes];
    uint16_t(*sA)[NR * 32 * LDK] = reinterpret_cast<uint16_t(*)[NR * 32 * LDK]>(smem);
    uint16_t(*sB)[BN * LDK] = reinterpret_cast<uint16_t(*)[BN * LDK]>(smem + 2 * 2 * NR * 32 * LDK);
    float *sE = reinterpret_cast<float *>(smem);
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = tid >> 6;               // the row block this wave computes
    const int b0 = blockIdx.x * 32, n0 = blockIdx.y * BN;
    const int Bp = a.Bp, K = a.K, N = a.N;
    f32x16 acc0, acc1;
#pragma unroll
    for (int i = 0; i < 16; ++i) {
        acc0[i] = 0.f;
        acc1[i] = 0.f;
    }
    // A pieces: c = tid + i NT (i = 0, 1) of the NR * 32 rows x 4 pieces
    auto load_a = [&](int k0, u32x4 *ra) {
#pragma unroll
        for (int i = 0; i < 2; ++i) {
            const int c = tid + i * NT;
            const int r = c >> 2, kc = c & 3;
            const int64_t grow = (int64_t)(r >> 5) * Bp + b0 + (r & 31);
            ra[i] = *(const u32x4 *)(a.A + grow * K + k0 + kc * 8);
        }
    };
    auto store_a = [&](uint16_t *s, const u32x4 *ra) {
#pragma unroll
        for (int i = 0; i < 2; ++i) {
            const int c = tid + i * NT;
            *(u32x4 *)(s + (c >> 2) * LDK + (c & 3) * 8) = ra[i];
        }
    };
    auto load_b = [&](int k0, u32x4 *rb) {
#pragma unroll
        for (int i = 0; i < kBC; ++i) {
            const int c = tid + i * NT;
            if (c < 256) rb[i] = *(const u32x4 *)(a.W + (int64_t)(n0 + (c >> 2)) * K + k0 + (c & 3) * 8);
        }
    };
    auto store_b = [&](uint16_t *s, const u32x4 *rb) {
#pragma unroll
        for (int i = 0; i < kBC; ++i) {
            const int c = tid + i * NT;
            if (c < 256) *(u32x4 *)(s + (c >> 2) * LDK + (c & 3) * 8) = rb[i];
        }
    };
    auto mma = [&](const uint16_t *a_s, const uint16_t *b_s) {
#pragma unroll
        for (int kk = 0; kk < BK; kk += 16) {
            const int ko = kk + 8 * (lane >> 5);
            const bf16x8 av = *(const bf16x8 *)(a_s + (wave * 32 + (lane & 31)) * LDK + ko);
            const bf16x8 bv0 = *(const bf16x8 *)(b_s + (lane & 31) * LDK + ko);
            const bf16x8 bv1 = *(const bf16x8 *)(b_s + (32 + (lane & 31)) * LDK + ko);
            acc0 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(av, bv0, acc0, 0, 0, 0);
            acc1 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(av, bv1, acc1, 0, 0, 0);
        }
    };
    // the epilogue's primal pre-activations (wave 0; layer 1: the W1 values
    // the other waves need), requested before the products so that their
    // latency hides behind them
    const int c0 = lane & 31;
    auto rr = [&](int i) { return (i >> 2) * 8 + (lane >> 5) * 4 + (i & 3); };
    float pre[32];
    if constexpr (EPI == kEpiActBwd || EPI == kEpiL1Bwd) {
#pragma unroll
        for (int i = 0; i < 16; ++i) {
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                const int64_t col = n0 + c0 + 32 * h;
                if (wave == 0) pre[2 * i + h] = a.Zp_in[(int64_t)(b0 + rr(i)) * N + col];
                else if constexpr (EPI == kEpiL1Bwd) pre[2 * i + h] = a.W1[(int64_t)(wave - 1) * N + col];
            }
        }
    }
    // the k-tiles as in k_gemm: tile t multiplied from buffer t % 2 while the
    // global loads of tiles t + 1 and t + 2 are in flight in two register sets
    const int nt = K / BK;
    u32x4 ra0[2], ra1[2], rb0[kBC], rb1[kBC];
    load_a(0, ra0);
    load_b(0, rb0);
    store_a(sA[0], ra0);
    store_b(sB[0], rb0);
    if (nt > 1) {
        load_a(BK, ra1);
        load_b(BK, rb1);
    }
    if (nt > 2) {
        load_a(2 * BK, ra0);
        load_b(2 * BK, rb0);
    }
    __syncthreads();
    for (int t = 0; t < nt; t += 2) {
        mma(sA[0], sB[0]);
        if (t + 1 < nt) {
            store_a(sA[1], ra1);
            store_b(sB[1], rb1);
        }
        if (t + 3 < nt) {
            load_a((t + 3) * BK, ra1);
            load_b((t + 3) * BK, rb1);
        }
        __syncthreads();
        if (t + 1 >= nt) break;
        mma(sA[1], sB[1]);
        if (t + 2 < nt) {
            store_a(sA[0], ra0);
            store_b(sB[0], rb0);
        }
        if (t + 4 < nt) {
            load_a((t + 4) * BK, ra0);
            load_b((t + 4) * BK, rb0);
        }
        __syncthreads();
    }

    // epilogue: element i of acc0 / acc1 is (row rr(i), column c0 / c0 + 32) of the wave's tile
    const int64_t rbase = (int64_t)wave * Bp + b0;   // first global row of this wave's tile
    const int blk = blockIdx.x;
    if constexpr (EPI == kEpiStore) {
#pragma unroll
        for (int i = 0; i < 16; ++i) {
            float *z = a.Z + (rbase + rr(i)) * N + n0 + c0;
            z[0] = acc0[i];
            z[32] = acc1[i];
        }
    } else if constexpr (EPI == kEpiActFwd) {
        float *d1s = sE;   // [32][64] SiLU'(z) of the primal rows
        if (wave == 0) {
            const float bi0 = a.bias[n0 + c0], bi1 = a.bias[n0 + c0 + 32];
#pragma unroll
            for (int i = 0; i < 16; ++i) {
                const int r = rr(i);
#pragma unroll
                for (int h = 0; h < 2; ++h) {
                    const float z = (h ? acc1[i] : acc0[i]) + (h ? bi1 : bi0);
                    const float sg = sigm(z);
                    const float d1 = sg * (1.f + z * (1.f - sg));
                    const int64_t o = (int64_t)(b0 + r) * N + n0 + c0 + 32 * h;
                    a.Aout[o] = f2bf(z * sg);
                    a.Zp[o] = z;
                    d1s[r * 64 + c0 + 32 * h] = d1;
                }
            }
        }
        __syncthreads();
        if (wave > 0) {
#pragma unroll
            for (int i = 0; i < 16; ++i) {
                const int r = rr(i);
#pragma unroll
                for (int h = 0; h < 2; ++h) {
                    const float u = h ? acc1[i] : acc0[i];
                    const int64_t col = n0 + c0 + 32 * h;
                    a.Aout[(rbase + r) * N + col] = f2bf(d1s[r * 64 + c0 + 32 * h] * u);
                    a.U[((int64_t)(wave - 1) * Bp + b0 + r) * N + col] = f2bf(u);
                }
            }
        }
    } else {   // kEpiActBwd, kEpiL1Bwd
        float *d1s = sE, *d2s = sE + 32 * 64, *tus = sE + 2 * 32 * 64;   // tus: [NR - 1][32][64]
        if (wave == 0) {
#pragma unroll
            for (int i = 0; i < 16; ++i) {
                const int r = rr(i);
#pragma unroll
                for (int h = 0; h < 2; ++h) {
                    const float z = pre[2 * i + h];
                    const float sg = sigm(z);
                    d1s[r * 64 + c0 + 32 * h] = sg * (1.f + z * (1.f - sg));
                    d2s[r * 64 + c0 + 32 * h] = sg * (1.f - sg) * (2.f + z * (1.f - 2.f * sg));
                }
            }
        }
        __syncthreads();
        float ub0[16], ub1[16];
        if (wave > 0) {
            const int tt = wave - 1;
#pragma unroll
            for (int i = 0; i < 16; ++i) {
                const int r = rr(i);
#pragma unroll
                for (int h = 0; h < 2; ++h) {
                    const int e = r * 64 + c0 + 32 * h;
                    const float tb = h ? acc1[i] : acc0[i];
                    float u;
                    if constexpr (EPI == kEpiL1Bwd) u = pre[2 * i + h];
                    else u = bf2f(a.U_in[((int64_t)tt * Bp + b0 + r) * N + n0 + c0 + 32 * h]);
                    const float ub = tb * d1s[e];
                    if constexpr (EPI == kEpiActBwd) a.Zbar[(rbase + r) * N + n0 + c0 + 32 * h] = f2bf(ub);
                    if (h) ub1[i] = ub;
                    else ub0[i] = ub;
                    tus[tt * 32 * 64 + e] = tb * u;
                }
            }
        }
        __syncthreads();
        if (wave == 0) {
            float zb0[16], zb1[16];
#pragma unroll
            for (int i = 0; i < 16; ++i) {
                const int r = rr(i);
#pragma unroll
                for (int h = 0; h < 2; ++h) {
                    const int e = r * 64 + c0 + 32 * h;
                    float zb = (h ? acc1[i] : acc0[i]) * d1s[e];
                    for (int tt = 0; tt < NR - 1; ++tt) zb += tus[tt * 32 * 64 + e] * d2s[e];
                    if constexpr (EPI == kEpiActBwd) a.Zbar[(rbase + r) * N + n0 + c0 + 32 * h] = f2bf(zb);
                    if (h) zb1[i] = zb;
                    else zb0[i] = zb;
                }
            }
            if constexpr (EPI == kEpiActBwd) {
                const float s0 = tile_colsum(zb0), s1 = tile_colsum(zb1);
                if (lane < 32) {
                    a.part[(int64_t)blk * N + n0 + c0] = s0;
                    a.part[(int64_t)blk * N + n0 + c0 + 32] = s1;
                }
            } else {
                // row NR - 1 of the partials: b1bar; rows t < NR - 1: sum_b x_bt zbar_b
                const int nin = NR - 1;
                const int64_t prow = (int64_t)blk * NR * N;
                const float s0 = tile_colsum(zb0), s1 = tile_colsum(zb1);
                if (lane < 32) {
                    a.part[prow + (int64_t)nin * N + n0 + c0] = s0;
                    a.part[prow + (int64_t)nin * N + n0 + c0 + 32] = s1;
                }
                for (int tt = 0; tt < nin; ++tt) {
                    float x0[16], x1[16];
#pragma unroll
                    for (int i = 0; i < 16; ++i) {
                        const float x = a.X[(int64_t)(b0 + rr(i)) * nin + tt];
                        x0[i] = x * zb0[i];
                        x1[i] = x * zb1[i];
                    }
                    const float q0 = tile_colsum(x0), q1 = tile_colsum(x1);
                    if (lane < 32) {   // the tangent waves add their sum_b ubar below
                        tus[tt * 64 + c0] = q0;
                        tus[tt * 64 + c0 + 32] = q1;
                    }
                }
            }
        }
        if constexpr (EPI == kEpiL1Bwd) {
            __syncthreads();
            if (wave > 0) {
                const int tt = wave - 1;
                const float s0 = tile_colsum(ub0), s1 = tile_colsum(ub1);
                if (lane < 32) {
                    const int64_t prow = (int64_t)blk * NR * N + (int64_t)tt * N;
                    a.part[prow + n0 + c0] = tus[tt * 64 + c0] + s0;
                    a.part[prow + n0 + c0 + 32] = tus[tt * 64 + c0 + 32] + s1;
                }
            }
        }
    }
}

// ---------------------------------------------------------------------------
// elementwise kernels
// ---------------------------------------------------------------------------
// Layer 1 (n_in -> H) from the raw parameters: x = (theta[row b] - shift)
// scale (row b is rows[b], or b when rows is null; x = 0 for padding rows
// b >= B), z = x W1 + b1; the tangent pre-activations are the rows of W1 (the
// input tangents are unit vectors).  The threads of unit 0 keep x for the
// backward pass.
__global__ void k_l1_fwd(const float *__restrict__ th, const int32_t *__restrict__ rows, int B,
                         const float *__restrict__ shift, const float *__restrict__ scale,
                         const float *__restrict__ W1, const float *__restrict__ b1, int Bp, int nin, int H,
                         float *__restrict__ X, float *__restrict__ Z, uint16_t *__restrict__ A)
{
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= Bp * H) return;
    const int b = idx / H, j = idx % H;
    const int64_t r = rows ? (int64_t)rows[b] : b;
    float z = b1[j];
    for (int k = 0; k < nin; ++k) {
        const float x = b < B ? (th[r * nin + k] - shift[k]) * scale[k] : 0.f;
        if (j == 0) X[b * nin + k] = x;
        z += x * W1[k * H + j];
    }
    const float s = sigm(z);
    const float d1 = s * (1.f + z * (1.f - s));
    Z[(int64_t)b * H + j] = z;
    A[(int64_t)b * H + j] = f2bf(z * s);
    // tangent rows: only their bf16 activations are stored; the pre-activations
    // are the rows of W1, which the backward pass reads there
    for (int t = 0; t < nin; ++t) {
        const int64_t rr = (int64_t)(t + 1) * Bp + b;
        A[rr * H + j] = f2bf(d1 * W1[t * H + j]);
    }
}

// Hidden layers 2, 3: add the bias to the primal rows, SiLU, tangents.
__global__ void k_act_fwd(float *__restrict__ Z, const float *__restrict__ bias, int Bp, int nin, int H,
                          uint16_t *__restrict__ A)
{
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= Bp * H) return;
    const int b = idx / H, j = idx % H;
    const float z = Z[(int64_t)b * H + j] + bias[j];
    const float s = sigm(z);
    const float d1 = s * (1.f + z * (1.f - s));
    Z[(int64_t)b * H + j] = z;
    A[(int64_t)b * H + j] = f2bf(z * s);
    for (int t = 0; t < nin; ++t) {
        const int64_t r = (int64_t)(t + 1) * Bp + b;
        A[r * H + j] = f2bf(d1 * Z[r * H + j]);
    }
}

// Output layer: prices and price Jacobian in physical units.
__global__ void k_out_fwd(const float *__restrict__ Z4, const float *__restrict__ b4, int B, int Bp, int nin,
                          int nout, const float *__restrict__ in_scale, const float *__restrict__ out_shift,
                          const float *__restrict__ out_scale, float *__restrict__ Y, float *__restrict__ J)
{
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= B * nout) return;
    const int b = idx / nout, i = idx % nout;
    Y[idx] = (Z4[(int64_t)b * kOutPad + i] + b4[i]) * out_scale[i] + out_shift[i];
    for (int t = 0; t < nin; ++t)
        J[(int64_t)idx * nin + t] = Z4[((int64_t)(t + 1) * Bp + b) * kOutPad + i] * out_scale[i] * in_scale[t];
}

// Differential loss, its adjoint G4 (bf16, network units) and FP64 block partials.
__global__ __launch_bounds__(kThreads) void k_loss(const float *__restrict__ Z4, const float *__restrict__ b4,
                                                   const float *__restrict__ Ylab, const float *__restrict__ Jlab,
                                                   const float *__restrict__ jw, const int32_t *__restrict__ rows,
                                                   int B, int nin, int nout, float w,
                                                   const float *__restrict__ in_scale,
                                                   const float *__restrict__ out_shift,
                                                   const float *__restrict__ out_scale, uint16_t *__restrict__ G4,
                                                   float *__restrict__ dYP, double *__restrict__ partial)
{
    __shared__ double sh[kThreads];
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    double acc = 0.0;
    if (idx < B * kOutPad) {
        const int b = idx / kOutPad, i = idx % kOutPad;
        const int64_t d = rows ? (int64_t)rows[b] : b;   // the sample's data row
        if (i < nout) {
            const float cy = 2.f / (float)(B * nout);
            const float cj = 2.f * w / (float)(B * nout * nin);
            const float z = Z4[(int64_t)b * kOutPad + i] + b4[i];
            const float zl = (Ylab[d * nout + i] - out_shift[i]) / out_scale[i];
            const float dz = z - zl;
            G4[(int64_t)b * kOutPad + i] = f2bf(cy * dz);
            dYP[(int64_t)b * kOutPad + i] = cy * dz;
            acc = (double)dz * dz / (double)(B * nout);
            const float cb = jw ? jw[d] : 1.f;
            for (int t = 0; t < nin; ++t) {
                const int64_t r = (int64_t)(t + 1) * B + b;
                if (cb == 0.f) {
                    G4[r * kOutPad + i] = 0;
                    continue;
                }
                const float jl = Jlab[(d * nout + i) * nin + t] / (out_scale[i] * in_scale[t]);
                const float dj = Z4[r * kOutPad + i] - jl;
                G4[r * kOutPad + i] = f2bf(cj * cb * dj);
                acc += (double)w * cb * dj * dj / (double)(B * nout * nin);
            }
        } else {
            G4[(int64_t)b * kOutPad + i] = 0;
            dYP[(int64_t)b * kOutPad + i] = 0.f;
            for (int t = 0; t < nin; ++t) G4[((int64_t)(t + 1) * B + b) * kOutPad + i] = 0;
        }
    }
    sh[threadIdx.x] = acc;
    __syncthreads();
    for (int s = kThreads / 2; s > 0; s >>= 1) {
        if (threadIdx.x < s) sh[threadIdx.x] += sh[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) partial[blockIdx.x] = sh[0];
}

// out[0] = sum of the n block partials: thread t adds p[t], p[t + 256], ... in
// order, then a fixed tree over the threads (one workgroup of kThreads).
__global__ __launch_bounds__(kThreads) void k_sum_partials(const double *__restrict__ p, int n,
                                                           double *__restrict__ out)
{
    __shared__ double sh[kThreads];
    double s = 0.0;
    for (int i = threadIdx.x; i < n; i += kThreads) s += p[i];
    sh[threadIdx.x] = s;
    __syncthreads();
    for (int h = kThreads / 2; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h) sh[threadIdx.x] += sh[threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[0] = sh[0];
}

// Adjoint through a hidden layer's activation (double backprop):
//   primal:  zbar   = hbar s'(z) + sum_t tbar_t u_t s''(z)
//   tangent: ubar_t = tbar_t s'(z)
__global__ void k_act_bwd(const float *__restrict__ Hbar, const float *__restrict__ Z, int B, int nin, int H,
                          uint16_t *__restrict__ Zbar, float *__restrict__ ZbarP)
{
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= B * H) return;
    const int b = idx / H, j = idx % H;
    const float z = Z[(int64_t)b * H + j];
    const float s = sigm(z);
    const float d1 = s * (1.f + z * (1.f - s));
    const float d2 = s * (1.f - s) * (2.f + z * (1.f - 2.f * s));
    float zb = Hbar[(int64_t)b * H + j] * d1;
    for (int t = 0; t < nin; ++t) {
        const int64_t r = (int64_t)(t + 1) * B + b;
        const float tb = Hbar[r * H + j];
        zb += tb * Z[r * H + j] * d2;
        Zbar[r * H + j] = f2bf(tb * d1);
    }
    Zbar[(int64_t)b * H + j] = f2bf(zb);
    ZbarP[(int64_t)b * H + j] = zb;
}

// Column sums over the rows of a batch, in two deterministic stages: block
// x sums rows x*kChunk .. x*kChunk + kChunk - 1 of column j in order into
// part[x][j], then k_chunk_reduce adds the chunks in a fixed order.
constexpr int kChunk = 32;   // rows per chunk; batches are multiples of 128

__global__ void k_colsum_part(const float *__restrict__ X, int ld, int ncols, float *__restrict__ part)
{
    const int j = blockIdx.y * blockDim.x + threadIdx.x;
    if (j >= ncols) return;
    const int64_t b0 = (int64_t)blockIdx.x * kChunk;
    float s = 0.f;
#pragma unroll 8
    for (int b = 0; b < kChunk; ++b) s += X[(b0 + b) * ld + j];
    part[(int64_t)blockIdx.x * ncols + j] = s;
}

// out[o] = sum over z < S of part[z * n + o], o < n: eight threads per output,
// thread q adding chunks q, q + 8, q + 16, ... in order, then the eight sums
// in a fixed tree; 32 outputs per workgroup.
__global__ __launch_bounds__(kThreads) void k_chunk_reduce(const float *__restrict__ part, int S, int n,
                                                           float *__restrict__ out)
{
    __shared__ float sh[kThreads];
    const int q = threadIdx.x & 7;
    const int o = blockIdx.x * (kThreads / 8) + (threadIdx.x >> 3);
    float s = 0.f;
    if (o < n) {
#pragma unroll 8
        for (int z = q; z < S; z += 8) s += part[(int64_t)z * n + o];
    }
    sh[threadIdx.x] = s;
    __syncthreads();
    if (q == 0 && o < n) {
        const float *v = sh + threadIdx.x;
        out[o] = ((v[0] + v[1]) + (v[2] + v[3])) + ((v[4] + v[5]) + (v[6] + v[7]));
    }
}

// Layer-1 gradients: W1bar[t][j] = sum_b x_bt zbar_bj + sum_b ubar_t,bj, b1bar[j] = sum_b zbar_bj,
// chunk by chunk (kChunkL1 rows; the per-row work is heavier, so more, smaller
// chunks) as k_colsum_part: part[x][t][j] for t <= nin (row nin: b1bar).
constexpr int kMaxIn = 16;
constexpr int kChunkL1 = 8;

template <int NI>   // n_in
__global__ void k_l1_bwd_part(const float *__restrict__ Hbar, const float *__restrict__ Z,
                              const float *__restrict__ W1, const float *__restrict__ X, int B, int H,
                              float *__restrict__ part)
{
    const int j = blockIdx.y * blockDim.x + threadIdx.x;
    if (j >= H) return;
    const int b0 = blockIdx.x * kChunkL1;
    float acc[NI + 1];
#pragma unroll
    for (int t = 0; t <= NI; ++t) acc[t] = 0.f;
    for (int b = b0; b < b0 + kChunkL1; ++b) {
        // the row's primal and tangent values, requested together
        const float z = Z[(int64_t)b * H + j];
        const float hb0 = Hbar[(int64_t)b * H + j];
        float hb[NI], zt[NI], xb[NI];
#pragma unroll
        for (int q = 0; q < NI; ++q) {
            const int64_t r = (int64_t)(q + 1) * B + b;
            hb[q] = Hbar[r * H + j];
            zt[q] = W1[q * H + j];   // the tangent pre-activations of layer 1
            xb[q] = X[b * NI + q];
        }
        const float s = sigm(z);
        const float d1 = s * (1.f + z * (1.f - s));
        const float d2 = s * (1.f - s) * (2.f + z * (1.f - 2.f * s));
        float zb = hb0 * d1;
#pragma unroll
        for (int q = 0; q < NI; ++q) zb += hb[q] * zt[q] * d2;
#pragma unroll
        for (int t = 0; t < NI; ++t) acc[t] += xb[t] * zb + hb[t] * d1;
        acc[NI] += zb;
    }
    float *pz = part + (int64_t)blockIdx.x * (NI + 1) * H;
#pragma unroll
    for (int t = 0; t <= NI; ++t) pz[(int64_t)t * H + j] = acc[t];
}

// bf16 copies of the product weights (layers 2..4): W [in x out] at offset
// off of the parameters goes to WT [out_pad x in] and Wb [in x out_pad].
struct WeightCopies {
    int64_t off[3];
    int in[3], out[3], out_pad[3];
    uint16_t *WT[3], *Wb[3];
};

// Adam with the learning rate and step count read on the device, each
// updated product weight written to its bf16 copies at once; the workgroup
// that finishes last (a counter of finished workgroups, reset by it) advances
// the step count, after every workgroup has read it.  A grid of at most
// kAdamGroups workgroups strides over the parameters, so that few workgroups
// meet at the counter.
constexpr int kAdamGroups = 128;
__global__ __launch_bounds__(kThreads) void k_adam_dev(float *__restrict__ p, const float *__restrict__ g,
                                                       float *__restrict__ m, float *__restrict__ v, int64_t n,
                                                       const float *__restrict__ lr_p, float b1, float b2, float eps,
                                                       int32_t *__restrict__ t_p, unsigned *__restrict__ done,
                                                       WeightCopies wc)
{
    __shared__ bool last;
    const float t = (float)t_p[0], lr = lr_p[0];
    const float bc1 = 1.f - powf(b1, t), bc2 = 1.f - powf(b2, t);
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const float gi = g[i];
        const float mi = b1 * m[i] + (1.f - b1) * gi;
        const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
        m[i] = mi;
        v[i] = vi;
        const float pi = p[i] - lr * (mi / bc1) / (sqrtf(vi / bc2) + eps);
        p[i] = pi;
#pragma unroll
        for (int l = 0; l < 3; ++l) {
            const int64_t q64 = i - wc.off[l];
            if (q64 >= 0 && q64 < (int64_t)wc.in[l] * wc.out[l]) {
                const unsigned q = (unsigned)q64, out = (unsigned)wc.out[l];   // < 2^20: 32-bit division
                const unsigned ii = q / out, o = q - ii * out;
                const uint16_t h = f2bf(pi);
                wc.WT[l][o * (unsigned)wc.in[l] + ii] = h;
                wc.Wb[l][ii * (unsigned)wc.out_pad[l] + o] = h;
            }
        }
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        __threadfence();
        last = atomicAdd(done, 1u) == gridDim.x - 1;
    }
    __syncthreads();
    if (last && threadIdx.x == 0) {
        t_p[0] += 1;
        *done = 0u;
    }
}

__global__ void k_adam(float *__restrict__ p, const float *__restrict__ g, float *__restrict__ m,
                       float *__restrict__ v, int64_t n, float lr, float b1, float b2, float eps, float bc1, float bc2)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.f - b1) * gi;
    const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    p[i] -= lr * (mi / bc1) / (sqrtf(vi / bc2) + eps);
}

// bf16 copies of W [in x out]: WT [out_pad x in] (forward operand, k = in
// contiguous) and Wb [in x out_pad] (backward operand, k = out contiguous).
__global__ void k_refresh(const float *__restrict__ W, int in, int out, int out_pad, uint16_t *__restrict__ WT,
                          uint16_t *__restrict__ Wb)
{
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= in * out_pad) return;
    const int i = idx / out_pad, o = idx % out_pad;
    const uint16_t h = o < out ? f2bf(W[i * out + o]) : (uint16_t)0;
    WT[(int64_t)o * in + i] = h;
    Wb[(int64_t)i * out_pad + o] = h;
}

// Surrogate calibration functional per sample: r = y - C, G = 1/2 sum r^2,
// grad_j = sum_i J_ij r_i (FP64; one workgroup per sample, fixed-order sums).
__global__ __launch_bounds__(kThreads) void k_calib_grad(const float *__restrict__ Y, const float *__restrict__ J,
                                                         const double *__restrict__ C, int nout, int nin,
                                                         double *__restrict__ G, double *__restrict__ grad)
{
    __shared__ double r[kOutPad];
    const int b = blockIdx.x;
    const int t = threadIdx.x;
    if (t < nout) r[t] = (double)Y[(int64_t)b * nout + t] - C[t];
    __syncthreads();
    if (t == 0) {
        double s = 0.0;
        for (int i = 0; i < nout; ++i) s += 0.5 * r[i] * r[i];
        G[b] = s;
    }
    if (t < nin) {
        double s = 0.0;
        for (int i = 0; i < nout; ++i) s += (double)J[((int64_t)b * nout + i) * nin + t] * r[i];
        grad[(int64_t)b * nin + t] = s;
    }
}

// ---------------------------------------------------------------------------
// Small batches: one workgroup per sample runs the whole evaluation (the four
// layers with the sample's primal row and n_in tangent rows, the outputs in
// price units and, given targets, the calibration functional), so that a
// calibration iteration on one parameter vector is one launch instead of
// nine.  The layer products are the batched path's: the same MFMA
// (v_mfma_f32_32x32x16_bf16) on the same bf16 operands, accumulated over k in
// the same order from zero, and each product row depends on its own operand
// row only, so a sample's pre-activations do not depend on the batch it came
// in; the elementwise work is that of the batched kernels.  NR = n_in + 1
// operand rows in LDS (bf16, row stride H + 8), padded to the MFMA's 32 rows
// with a row of zeros.
// ---------------------------------------------------------------------------
constexpr int kSmallMaxB = 64;       // batches up to this size take the one-launch path
constexpr int kSmallMaxRows = 9;     // n_in <= 8
constexpr int kSmallThreads = 512;   // 8 waves: one 32-column tile each at H = 256
constexpr int kSmallSteps = 16;      // k-steps whose B operands are loaded at once
constexpr int kSmallUnits = 2;       // hidden units per thread (n_hidden <= 1024)

// B operands (16 bytes per lane and k-step) of the first kSmallSteps k-steps
// of this wave's first tile of z = act WT^T (N columns, K = k extent); issued
// early so that their latency overlaps the work before the product.
__device__ __forceinline__ void small_prefetch(const uint16_t *__restrict__ WT, int N, int K, bf16x8 *bv)
{
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int n0 = wave * 32;
    if (n0 >= N) return;
    const uint16_t *brow = WT + (int64_t)(n0 + (lane & 31)) * K + 8 * (lane >> 5);
    const int steps = min(kSmallSteps, K / 16);
#pragma unroll
    for (int q = 0; q < kSmallSteps; ++q)
        if (q < steps) bv[q] = *(const bf16x8 *)(brow + 16 * q);
}

// z[row][n] (row < NR, n < N) = sum_k act[row][k] WT[n][k] over k < K, N a
// multiple of 32: wave w takes the 32-column tiles w, w + 8, ...  act: LDS
// bf16 rows of stride lda, row NR all zeros.  bv holds small_prefetch's
// operands for this product.
template <int NR>
__device__ __forceinline__ void small_product(const uint16_t *act, int lda, const uint16_t *__restrict__ WT, int N,
                                              int K, float *z, int ldz, bf16x8 *bv)
{
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int r = lane & 31, kofs = 8 * (lane >> 5);
    const uint16_t *arow = act + (r < NR ? r : NR) * lda + kofs;
    bool loaded = true;
    for (int n0 = wave * 32; n0 < N; n0 += (kSmallThreads / 64) * 32) {
        const uint16_t *brow = WT + (int64_t)(n0 + r) * K + kofs;
        f32x16 acc;
#pragma unroll
        for (int i = 0; i < 16; ++i) acc[i] = 0.f;
        for (int k0 = 0; k0 < K; k0 += 16 * kSmallSteps) {
            const int steps = min(kSmallSteps, (K - k0) / 16);
            if (!loaded) {
#pragma unroll
                for (int q = 0; q < kSmallSteps; ++q)
                    if (q < steps) bv[q] = *(const bf16x8 *)(brow + k0 + 16 * q);
            }
            loaded = false;
#pragma unroll
            for (int q = 0; q < kSmallSteps; ++q)
                if (q < steps) {
                    const bf16x8 a = *(const bf16x8 *)(arow + k0 + 16 * q);
                    acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, bv[q], acc, 0, 0, 0);
                }
        }
#pragma unroll
        for (int i = 0; i < 16; ++i) {
            const int row = (i >> 2) * 8 + (lane >> 5) * 4 + (i & 3);
            if (row < NR) z[row * ldz + n0 + r] = acc[i];
        }
    }
}

// Bias, SiLU and tangents of a hidden layer, as k_act_fwd: act[0] = SiLU(z0 +
// bias), act[q] = SiLU'(z0 + bias) z[q]; bias[u] is that of this thread's
// unit t + u kSmallThreads.
template <int NR>
__device__ __forceinline__ void small_activate(const float *z, const float *bias, int H, uint16_t *act, int lda)
{
#pragma unroll
    for (int u = 0; u < kSmallUnits; ++u) {
        const int j = threadIdx.x + u * kSmallThreads;
        if (j >= H) break;
        const float zz = z[j] + bias[u];
        const float s = sigm(zz);
        const float d1 = s * (1.f + zz * (1.f - s));
        act[j] = f2bf(zz * s);
        for (int q = 1; q < NR; ++q) act[q * lda + j] = f2bf(d1 * z[q * H + j]);
    }
}

template <int NR>
__global__ __launch_bounds__(kSmallThreads) void k_small_eval(
    const float *__restrict__ th, int H, int nout, const float *__restrict__ in_shift,
    const float *__restrict__ in_scale, const float *__restrict__ W1, const float *__restrict__ b1,
    const uint16_t *__restrict__ WT2, const float *__restrict__ b2, const uint16_t *__restrict__ WT3,
    const float *__restrict__ b3, const uint16_t *__restrict__ WT4, const float *__restrict__ b4,
    const float *__restrict__ out_shift, const float *__restrict__ out_scale, const double *__restrict__ C,
    float *__restrict__ Y, float *__restrict__ J, double *__restrict__ G, double *__restrict__ grad)
{
    constexpr int nin = NR - 1;
    extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
    const int lda = H + 8;
    uint16_t *act = (uint16_t *)smem;                          // [NR + 1][lda] bf16
    float *z = (float *)(smem + (size_t)(NR + 1) * lda * 2);   // [NR][H] FP32
    __shared__ float xs[nin];
    __shared__ float ys[kOutPad];
    __shared__ float js[kOutPad * nin];
    __shared__ double r[kOutPad];
    __shared__ float o_b[kOutPad], o_scale[kOutPad], o_shift[kOutPad], i_scale[nin];
    __shared__ double cs[kOutPad];
    const int b = blockIdx.x, t = threadIdx.x;
    // everything the sample needs from memory but the output layer's weights
    // and later batches of wider layers, requested at once
    bf16x8 bv2[kSmallSteps], bv3[kSmallSteps];
    small_prefetch(WT2, H, H, bv2);
    small_prefetch(WT3, H, H, bv3);
    float w1[kSmallUnits][NR], bias2[kSmallUnits], bias3[kSmallUnits];
#pragma unroll
    for (int u = 0; u < kSmallUnits; ++u) {
        const int j = t + u * kSmallThreads;
        if (j < H) {
            w1[u][0] = b1[j];
#pragma unroll
            for (int k = 0; k < nin; ++k) w1[u][k + 1] = W1[k * H + j];
            bias2[u] = b2[j];
            bias3[u] = b3[j];
        }
    }
    if (t < nin) {
        xs[t] = (th[b * nin + t] - in_shift[t]) * in_scale[t];
        i_scale[t] = in_scale[t];
    }
    if (t < nout) {
        o_b[t] = b4[t];
        o_scale[t] = out_scale[t];
        o_shift[t] = out_shift[t];
        if (C) cs[t] = C[t];
    }
    for (int i = t; i < H; i += kSmallThreads) act[NR * lda + i] = 0;
    __syncthreads();
    // layer 1 (n_in -> H), as k_l1_fwd: the tangent pre-activations are the rows of W1
#pragma unroll
    for (int u = 0; u < kSmallUnits; ++u) {
        const int j = t + u * kSmallThreads;
        if (j >= H) break;
        float zz = w1[u][0];
        for (int k = 0; k < nin; ++k) zz += xs[k] * w1[u][k + 1];
        const float s = sigm(zz);
        const float d1 = s * (1.f + zz * (1.f - s));
        act[j] = f2bf(zz * s);
#pragma unroll
        for (int q = 1; q < NR; ++q) act[q * lda + j] = f2bf(d1 * w1[u][q]);
    }
    __syncthreads();
    // hidden layers 2, 3
    small_product<NR>(act, lda, WT2, H, H, z, H, bv2);
    bf16x8 *bv4 = bv2;   // free again: the output layer's first operands
    small_prefetch(WT4, kOutPad, H, bv4);
    __syncthreads();
    small_activate<NR>(z, bias2, H, act, lda);
    __syncthreads();
    small_product<NR>(act, lda, WT3, H, H, z, H, bv3);
    __syncthreads();
    small_activate<NR>(z, bias3, H, act, lda);
    __syncthreads();
    // output layer (units padded to kOutPad; WT4's padding rows are zero), as k_out_fwd
    small_product<NR>(act, lda, WT4, kOutPad, H, z, kOutPad, bv4);
    __syncthreads();
    for (int q = t; q < NR * nout; q += kSmallThreads) {
        const int row = q / nout, o = q % nout;
        const float v = z[row * kOutPad + o];
        if (row == 0) ys[o] = (v + o_b[o]) * o_scale[o] + o_shift[o];
        else js[o * nin + row - 1] = v * o_scale[o] * i_scale[row - 1];
    }
    __syncthreads();
    for (int q = t; q < nout * (nin + 1); q += kSmallThreads) {
        if (q < nout) Y[(int64_t)b * nout + q] = ys[q];
        else J[(int64_t)b * nout * nin + (q - nout)] = js[q - nout];
    }
    if (!C) return;   // uniform: inference only
    // the calibration functional, as k_calib_grad
    if (t < nout) r[t] = (double)ys[t] - cs[t];
    __syncthreads();
    if (t == 0) {
        double sacc = 0.0;
        for (int i = 0; i < nout; ++i) sacc += 0.5 * r[i] * r[i];
        G[b] = sacc;
    }
    if (t < nin) {
        double sacc = 0.0;
        for (int i = 0; i < nout; ++i) sacc += (double)js[i * nin + t] * r[i];
        grad[(int64_t)b * nin + t] = sacc;
    }
}

__global__ void k_fill(float *p, int64_t n, float v)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

inline unsigned nb(int64_t n) { return (unsigned)((n + kThreads - 1) / kThreads); }

}  // namespace

// ---------------------------------------------------------------------------
// context and C ABI
// ---------------------------------------------------------------------------
struct mlp_ctx {
    int nin = 0, H = 0, nout = 0, Bmax = 0;
    int64_t np = 0;
    int64_t off[8] = {0};
    float *p = nullptr, *m = nullptr, *v = nullptr;
    uint16_t *WT[4] = {nullptr}, *Wb[4] = {nullptr};   // layers 2..4 used
    float *in_shift = nullptr, *in_scale = nullptr, *out_shift = nullptr, *out_scale = nullptr;
    float *Z[5] = {nullptr};      // Z[1..3]: R x H, Z[4]: R x kOutPad
    uint16_t *A[4] = {nullptr};   // A[1..3]: R x H
    uint16_t *G4 = nullptr;       // R x kOutPad
    float *Hbar = nullptr;        // R x H
    uint16_t *Zbar = nullptr;     // R x H
    uint16_t *Zbar2 = nullptr;    // R x H (fused path: the layer below's adjoints)
    uint16_t *U[4] = {nullptr};   // U[2..3]: n_in Bmax x H tangent pre-activations (bf16, fused path)
    float *ZbarP = nullptr;       // Bmax x H
    float *Xn = nullptr;          // Bmax x nin
    float *split = nullptr;       // kMaxSplits x H x H, or row-chunk partials of the column sums
    double *lossp = nullptr;
    unsigned *done = nullptr;     // finished-workgroup counter of k_adam_dev (zero between launches)
    // fused path: the weight and bias gradients of the layers above the one the
    // backward sweep is in run on a second stream (they are off its critical
    // path), with buffers of their own
    float *gsplit = nullptr;      // kMaxSplits x H x H: that stream's split-K and column-sum partials
    float *rpart[2] = {nullptr};  // (Bmax / 32) x H: column partials of the hidden layers' bias adjoints
    hipStream_t side = nullptr;   // default priority, non-blocking
    hipEvent_t ev[4] = {nullptr};
    std::vector<void *> allocs;
    std::string err;
};

static thread_local std::string g_mlp_err;

static int mfail(mlp_ctx *c, int code, const std::string &m)
{
    if (c) c->err = m;
    g_mlp_err = m;
    return code;
}

template <int NI>
static void launch_l1_bwd_t(dim3 grid, hipStream_t st, const float *Hbar, const float *Z, const float *W1,
                            const float *X, int B, int H, float *part)
{
    hipLaunchKernelGGL((k_l1_bwd_part<NI>), grid, dim3(kThreads), 0, st, Hbar, Z, W1, X, B, H, part);
}

// Layer-1 gradient partials for n_in = nin (1..16).
static void launch_l1_bwd(int nin, dim3 grid, hipStream_t st, const float *Hbar, const float *Z, const float *W1,
                          const float *X, int B, int H, float *part)
{
    typedef void (*fn)(dim3, hipStream_t, const float *, const float *, const float *, const float *, int, int,
                       float *);
    static const fn tab[kMaxIn] = {launch_l1_bwd_t<1>,  launch_l1_bwd_t<2>,  launch_l1_bwd_t<3>,  launch_l1_bwd_t<4>,
                                   launch_l1_bwd_t<5>,  launch_l1_bwd_t<6>,  launch_l1_bwd_t<7>,  launch_l1_bwd_t<8>,
                                   launch_l1_bwd_t<9>,  launch_l1_bwd_t<10>, launch_l1_bwd_t<11>, launch_l1_bwd_t<12>,
                                   launch_l1_bwd_t<13>, launch_l1_bwd_t<14>, launch_l1_bwd_t<15>, launch_l1_bwd_t<16>};
    tab[nin - 1](grid, st, Hbar, Z, W1, X, B, H, part);
}

static hipError_t launch_gemm(bool akc, bool bkc, const uint16_t *A, int lda, const uint16_t *B, int ldb, float *C,
                              int ldc, int M, int N, int K, int splits, hipStream_t st)
{
    const int ks = ((K + splits - 1) / splits + BK - 1) / BK * BK;
    const dim3 grid(M / BM, N / BN, splits);
    const int64_t ss = (int64_t)M * N;
    if (akc && bkc)
        hipLaunchKernelGGL((k_gemm<true, true>), grid, dim3(kThreads), 0, st, A, lda, B, ldb, C, ldc, ss, K, ks);
    else if (!akc && !bkc)
        hipLaunchKernelGGL((k_gemm<false, false>), grid, dim3(kThreads), 0, st, A, lda, B, ldb, C, ldc, ss, K, ks);
    else if (akc)
        hipLaunchKernelGGL((k_gemm<true, false>), grid, dim3(kThreads), 0, st, A, lda, B, ldb, C, ldc, ss, K, ks);
    else
        hipLaunchKernelGGL((k_gemm<false, true>), grid, dim3(kThreads), 0, st, A, lda, B, ldb, C, ldc, ss, K, ks);
    return hipGetLastError();
}

// out[j] = sum over the B rows of X (leading dimension ld) of column j < ncols,
// through c->split (nchunk x ncols partials), deterministic order.
static void colsum(float *part, const float *X, int B, int ld, int ncols, float *out, hipStream_t st)
{
    const int nchunk = B / kChunk;
    hipLaunchKernelGGL(k_colsum_part, dim3(nchunk, (ncols + kThreads - 1) / kThreads), dim3(kThreads), 0, st, X, ld,
                       ncols, part);
    hipLaunchKernelGGL(k_chunk_reduce, dim3((ncols + kThreads / 8 - 1) / (kThreads / 8)), dim3(kThreads), 0, st,
                       part, nchunk, ncols, out);
}

extern "C" int mlp_destroy(mlp_ctx *c)
{
    if (!c) return 0;
    (void)hipDeviceSynchronize();
    for (hipEvent_t ev : c->ev)
        if (ev) (void)hipEventDestroy(ev);
    if (c->side) (void)hipStreamDestroy(c->side);
    for (void *p : c->allocs) (void)hipFree(p);
    delete c;
    return 0;
}

extern "C" int mlp_create(int32_t n_in, int32_t n_hidden, int32_t n_out, int32_t max_batch, mlp_ctx **out)
{
    if (!out) return mfail(nullptr, -1, "null output pointer");
    *out = nullptr;
    if (n_in < 1 || n_in > 16) return mfail(nullptr, -1, "n_in must be in 1..16");
    if (n_hidden < 128 || n_hidden > 1024 || n_hidden % 128)
        return mfail(nullptr, -1, "n_hidden must be a multiple of 128 in 128..1024");
    if (n_out < 1 || n_out > kOutPad) return mfail(nullptr, -1, "n_out must be in 1..64");
    if (max_batch < 1 || max_batch > 65536) return mfail(nullptr, -1, "max_batch must be in 1..65536");
    mlp_ctx *c = new mlp_ctx();
    c->nin = n_in;
    c->H = n_hidden;
    c->nout = n_out;
    c->Bmax = (max_batch + 127) / 128 * 128;
    const int H = n_hidden;
    const int64_t sizes[8] = {(int64_t)n_in * H, H, (int64_t)H * H, H, (int64_t)H * H, H, (int64_t)H * n_out, n_out};
    int64_t o = 0;
    for (int i = 0; i < 8; ++i) {
        c->off[i] = o;
        o += sizes[i];
    }
    c->np = o;
    const int64_t R = (int64_t)(n_in + 1) * c->Bmax;
    hipError_t e = hipSuccess;
    auto A = [&](void **p, int64_t bytes) {
        if (e != hipSuccess) return;
        e = hipMalloc(p, (size_t)(bytes > 0 ? bytes : 16));
        if (e == hipSuccess) c->allocs.push_back(*p);
    };
    A((void **)&c->p, 4 * c->np);
    A((void **)&c->m, 4 * c->np);
    A((void **)&c->v, 4 * c->np);
    for (int l = 2; l <= 4; ++l) {
        const int64_t opad = l == 4 ? kOutPad : H;
        A((void **)&c->WT[l - 1], 2 * opad * H);
        A((void **)&c->Wb[l - 1], 2 * opad * H);
    }
    A((void **)&c->in_shift, 4 * 16);
    A((void **)&c->in_scale, 4 * 16);
    A((void **)&c->out_shift, 4 * kOutPad);
    A((void **)&c->out_scale, 4 * kOutPad);
    for (int l = 1; l <= 3; ++l) {
        A((void **)&c->Z[l], 4 * R * H);
        A((void **)&c->A[l], 2 * R * H);
    }
    A((void **)&c->Z[4], 4 * R * kOutPad);
    A((void **)&c->G4, 2 * R * kOutPad);
    A((void **)&c->Hbar, 4 * R * H);
    A((void **)&c->Zbar, 2 * R * H);
    A((void **)&c->Zbar2, 2 * R * H);
    for (int l = 2; l <= 3; ++l) A((void **)&c->U[l], 2 * (int64_t)n_in * c->Bmax * H);
    A((void **)&c->ZbarP, 4 * (int64_t)c->Bmax * H);
    A((void **)&c->Xn, 4 * (int64_t)c->Bmax * n_in);
    // split-K GEMM partials, or the row-chunk partials of the column sums (at most
    // (Bmax / kChunkL1) x (n_in + 1) x H floats)
    A((void **)&c->split, 4 * std::max((int64_t)kMaxSplits * H * H, (int64_t)(c->Bmax / kChunkL1) * (n_in + 1) * H));
    A((void **)&c->lossp, 8 * (int64_t)((c->Bmax * kOutPad + kThreads - 1) / kThreads));
    A((void **)&c->done, 256);
    A((void **)&c->gsplit, 4 * std::max((int64_t)kMaxSplits * H * H, (int64_t)(c->Bmax / kChunk) * kOutPad));
    for (int i = 0; i < 2; ++i) A((void **)&c->rpart[i], 4 * (int64_t)(c->Bmax / 32) * H);
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&c->side, hipStreamNonBlocking);
    for (int i = 0; i < 4 && e == hipSuccess; ++i) e = hipEventCreateWithFlags(&c->ev[i], hipEventDisableTiming);
    if (e != hipSuccess) {
        mlp_destroy(c);
        return mfail(nullptr, -2, std::string("allocation failed: ") + hipGetErrorString(e));
    }
    hipLaunchKernelGGL(k_fill, dim3(nb(c->np)), dim3(kThreads), 0, 0, c->p, c->np, 0.f);
    hipLaunchKernelGGL(k_fill, dim3(1), dim3(kThreads), 0, 0, (float *)c->done, (int64_t)64, 0.f);
    hipLaunchKernelGGL(k_fill, dim3(nb(c->np)), dim3(kThreads), 0, 0, c->m, c->np, 0.f);
    hipLaunchKernelGGL(k_fill, dim3(nb(c->np)), dim3(kThreads), 0, 0, c->v, c->np, 0.f);
    hipLaunchKernelGGL(k_fill, dim3(1), dim3(kThreads), 0, 0, c->in_shift, (int64_t)16, 0.f);
    hipLaunchKernelGGL(k_fill, dim3(1), dim3(kThreads), 0, 0, c->in_scale, (int64_t)16, 1.f);
    hipLaunchKernelGGL(k_fill, dim3(1), dim3(kThreads), 0, 0, c->out_shift, (int64_t)kOutPad, 0.f);
    hipLaunchKernelGGL(k_fill, dim3(1), dim3(kThreads), 0, 0, c->out_scale, (int64_t)kOutPad, 1.f);
    for (int l = 2; l <= 4; ++l) {
        const int opad = l == 4 ? kOutPad : H;
        const int outd = l == 4 ? n_out : H;
        hipLaunchKernelGGL(k_refresh, dim3(nb((int64_t)H * opad)), dim3(kThreads), 0, 0, c->p + c->off[2 * (l - 1)],
                           H, outd, opad, c->WT[l - 1], c->Wb[l - 1]);
    }
    e = hipDeviceSynchronize();
    if (e != hipSuccess) {
        mlp_destroy(c);
        return mfail(nullptr, -3, std::string("initialisation failed: ") + hipGetErrorString(e));
    }
    *out = c;
    return 0;
}

extern "C" int64_t mlp_num_params(const mlp_ctx *c) { return c ? c->np : -1; }

static hipError_t refresh_all(mlp_ctx *c, hipStream_t st)
{
    for (int l = 2; l <= 4; ++l) {
        const int opad = l == 4 ? kOutPad : c->H;
        const int outd = l == 4 ? c->nout : c->H;
        hipLaunchKernelGGL(k_refresh, dim3(nb((int64_t)c->H * opad)), dim3(kThreads), 0, st, c->p + c->off[2 * (l - 1)],
                           c->H, outd, opad, c->WT[l - 1], c->Wb[l - 1]);
    }
    return hipGetLastError();
}

extern "C" int mlp_set_params(mlp_ctx *c, const float *d_params, void *stream)
{
    if (!c || !d_params) return mfail(c, -1, "null argument");
    hipStream_t st = (hipStream_t)stream;
    hipError_t e = hipMemcpyAsync(c->p, d_params, 4 * c->np, hipMemcpyDeviceToDevice, st);
    if (e == hipSuccess) {
        hipLaunchKernelGGL(k_fill, dim3(nb(c->np)), dim3(kThreads), 0, st, c->m, c->np, 0.f);
        hipLaunchKernelGGL(k_fill, dim3(nb(c->np)), dim3(kThreads), 0, st, c->v, c->np, 0.f);
        e = refresh_all(c, st);
    }
    return e == hipSuccess ? 0 : mfail(c, -3, hipGetErrorString(e));
}

extern "C" int mlp_get_params(const mlp_ctx *c, float *d_params, void *stream)
{
    if (!c || !d_params) return mfail(nullptr, -1, "null argument");
    hipError_t e = hipMemcpyAsync(d_params, c->p, 4 * c->np, hipMemcpyDeviceToDevice, (hipStream_t)stream);
    return e == hipSuccess ? 0 : mfail(nullptr, -3, hipGetErrorString(e));
}

extern "C" int mlp_set_scaling(mlp_ctx *c, const float *d_in_shift, const float *d_in_scale, const float *d_out_shift,
                               const float *d_out_scale, void *stream)
{
    if (!c || !d_in_shift || !d_in_scale || !d_out_shift || !d_out_scale) return mfail(c, -1, "null argument");
    hipStream_t st = (hipStream_t)stream;
    hipError_t e = hipMemcpyAsync(c->in_shift, d_in_shift, 4 * c->nin, hipMemcpyDeviceToDevice, st);
    if (e == hipSuccess) e = hipMemcpyAsync(c->in_scale, d_in_scale, 4 * c->nin, hipMemcpyDeviceToDevice, st);
    if (e == hipSuccess) e = hipMemcpyAsync(c->out_shift, d_out_shift, 4 * c->nout, hipMemcpyDeviceToDevice, st);
    if (e == hipSuccess) e = hipMemcpyAsync(c->out_scale, d_out_scale, 4 * c->nout, hipMemcpyDeviceToDevice, st);
    return e == hipSuccess ? 0 : mfail(c, -3, hipGetErrorString(e));
}

// Whether the training step and large-batch inference take the fused
// row-block kernels (one wave per row block).
static bool fused_path(const mlp_ctx *c) { return c->nin + 1 <= kRowsMaxNR; }

template <int NR>
static void launch_rows_nr(int epi, const RowsArgs &a, hipStream_t st)
{
    const dim3 grid((unsigned)(a.Bp / 32), (unsigned)(a.N / BN)), block(NR * 64);
    switch (epi) {
    case kEpiStore: hipLaunchKernelGGL((k_rows<NR, kEpiStore>), grid, block, 0, st, a); break;
    case kEpiActFwd: hipLaunchKernelGGL((k_rows<NR, kEpiActFwd>), grid, block, 0, st, a); break;
    case kEpiActBwd: hipLaunchKernelGGL((k_rows<NR, kEpiActBwd>), grid, block, 0, st, a); break;
    default: hipLaunchKernelGGL((k_rows<NR, kEpiL1Bwd>), grid, block, 0, st, a); break;
    }
}

static hipError_t launch_rows(int NR, int epi, const RowsArgs &a, hipStream_t st)
{
    switch (NR) {
    case 2: launch_rows_nr<2>(epi, a, st); break;
    case 3: launch_rows_nr<3>(epi, a, st); break;
    case 4: launch_rows_nr<4>(epi, a, st); break;
    case 5: launch_rows_nr<5>(epi, a, st); break;
    case 6: launch_rows_nr<6>(epi, a, st); break;
    case 7: launch_rows_nr<7>(epi, a, st); break;
    case 8: launch_rows_nr<8>(epi, a, st); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

// Fused forward over B samples (theta rows `rows`, padded to Bp): layer 1,
// then the two hidden layers' products with their activations; with
// store_out the output layer's pre-activations go to c->Z[4].
static hipError_t forward_fused(mlp_ctx *c, const float *th, const int32_t *rows, int B, int Bp, bool store_out,
                                hipStream_t st)
{
    const int H = c->H, nin = c->nin, NR = nin + 1;
    const float *p = c->p;
    hipLaunchKernelGGL(k_l1_fwd, dim3(nb((int64_t)Bp * H)), dim3(kThreads), 0, st, th, rows, B, c->in_shift,
                       c->in_scale, p + c->off[0], p + c->off[1], Bp, nin, H, c->Xn, c->Z[1], c->A[1]);
    hipError_t e = hipGetLastError();
    for (int l = 2; l <= 3 && e == hipSuccess; ++l) {
        RowsArgs a{};
        a.A = c->A[l - 1];
        a.W = c->WT[l - 1];
        a.Bp = Bp;
        a.K = H;
        a.N = H;
        a.bias = p + c->off[2 * l - 1];
        a.Aout = c->A[l];
        a.Zp = c->Z[l];
        a.U = c->U[l];
        e = launch_rows(NR, kEpiActFwd, a, st);
    }
    if (e == hipSuccess && store_out) {
        RowsArgs a{};
        a.A = c->A[3];
        a.W = c->WT[3];
        a.Bp = Bp;
        a.K = H;
        a.N = kOutPad;
        a.Z = c->Z[4];
        e = launch_rows(NR, kEpiStore, a, st);
    }
    return e;
}

// Forward over B samples (theta rows `rows`, padded to Bp).
static hipError_t forward_core(mlp_ctx *c, const float *th, const int32_t *rows, int B, int Bp, hipStream_t st)
{
    if (fused_path(c)) return forward_fused(c, th, rows, B, Bp, true, st);
    const int H = c->H, nin = c->nin;
    const int R = (nin + 1) * Bp;
    const float *p = c->p;
    hipLaunchKernelGGL(k_l1_fwd, dim3(nb((int64_t)Bp * H)), dim3(kThreads), 0, st, th, rows, B, c->in_shift,
                       c->in_scale, p + c->off[0], p + c->off[1], Bp, nin, H, c->Xn, c->Z[1], c->A[1]);
    hipError_t e = hipGetLastError();
    for (int l = 2; l <= 3 && e == hipSuccess; ++l) {
        e = launch_gemm(true, true, c->A[l - 1], H, c->WT[l - 1], H, c->Z[l], H, R, H, H, 1, st);
        if (e != hipSuccess) break;
        hipLaunchKernelGGL(k_act_fwd, dim3(nb((int64_t)Bp * H)), dim3(kThreads), 0, st, c->Z[l], p + c->off[2 * l - 1],
                           Bp, nin, H, c->A[l]);
        e = hipGetLastError();
    }
    if (e == hipSuccess) e = launch_gemm(true, true, c->A[3], H, c->WT[3], H, c->Z[4], kOutPad, R, kOutPad, H, 1, st);
    return e;
}

// Dynamic LDS of k_small_eval: NR + 1 bf16 operand rows of stride H + 8 and
// NR FP32 rows of pre-activations.
static size_t small_lds(int NR, int H) { return (size_t)(NR + 1) * (H + 8) * 2 + (size_t)NR * H * 4; }

// Whether a batch of B samples takes the one-launch path (k_small_eval).
static bool small_path(const mlp_ctx *c, int B)
{
    return B <= kSmallMaxB && c->nin + 1 <= kSmallMaxRows && c->H <= kSmallUnits * kSmallThreads &&
           small_lds(c->nin + 1, c->H) <= 60 * 1024;
}

template <int NR>
static void launch_small_t(const mlp_ctx *c, const float *th, int B, const double *C, float *Y, float *J, double *G,
                           double *grad, hipStream_t st)
{
    const size_t lds = small_lds(NR, c->H);
    const float *p = c->p;
    hipLaunchKernelGGL((k_small_eval<NR>), dim3((unsigned)B), dim3(kSmallThreads), lds, st, th, c->H, c->nout,
                       c->in_shift, c->in_scale, p + c->off[0], p + c->off[1], c->WT[1], p + c->off[3], c->WT[2],
                       p + c->off[5], c->WT[3], p + c->off[7], c->out_shift, c->out_scale, C, Y, J, G, grad);
}

static hipError_t launch_small(const mlp_ctx *c, const float *th, int B, const double *C, float *Y, float *J,
                               double *G, double *grad, hipStream_t st)
{
    switch (c->nin + 1) {
    case 2: launch_small_t<2>(c, th, B, C, Y, J, G, grad, st); break;
    case 3: launch_small_t<3>(c, th, B, C, Y, J, G, grad, st); break;
    case 4: launch_small_t<4>(c, th, B, C, Y, J, G, grad, st); break;
    case 5: launch_small_t<5>(c, th, B, C, Y, J, G, grad, st); break;
    case 6: launch_small_t<6>(c, th, B, C, Y, J, G, grad, st); break;
    case 7: launch_small_t<7>(c, th, B, C, Y, J, G, grad, st); break;
    case 8: launch_small_t<8>(c, th, B, C, Y, J, G, grad, st); break;
    case 9: launch_small_t<9>(c, th, B, C, Y, J, G, grad, st); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

extern "C" int mlp_forward(mlp_ctx *c, const float *d_theta, int32_t B, float *d_Y, float *d_J, void *stream)
{
    if (!c || !d_theta || !d_Y || !d_J) return mfail(c, -1, "null argument");
    if (B < 1 || B > c->Bmax) return mfail(c, -1, "batch outside 1..max_batch");
    hipStream_t st = (hipStream_t)stream;
    if (small_path(c, B)) {
        const hipError_t e = launch_small(c, d_theta, B, nullptr, d_Y, d_J, nullptr, nullptr, st);
        return e == hipSuccess ? 0 : mfail(c, -3, hipGetErrorString(e));
    }
    const int Bp = (B + 127) / 128 * 128;
    hipError_t e = forward_core(c, d_theta, nullptr, B, Bp, st);
    if (e == hipSuccess) {
        hipLaunchKernelGGL(k_out_fwd, dim3(nb((int64_t)B * c->nout)), dim3(kThreads), 0, st, c->Z[4],
                           c->p + c->off[7], B, Bp, c->nin, c->nout, c->in_scale, c->out_shift, c->out_scale, d_Y, d_J);
        e = hipGetLastError();
    }
    return e == hipSuccess ? 0 : mfail(c, -3, hipGetErrorString(e));
}

// The training step on the fused kernels: forward, the loss with the output
// layer's adjoint, then per layer the weight gradient (split-K product, fixed-
// order reduction), the bias gradient (workgroup column partials, fixed-order
// reduction) and the next layer's input adjoint fused with the activation
// adjoint; layer 1's gradients from the last product's epilogue.
// The backward sweep (layer adjoints, top down) runs on st; the weight and
// bias gradients of each layer, which nothing later in the sweep reads, run
// on c->side as soon as their layer's adjoints exist: fork at events ev[0..2],
// join at ev[3] before returning, so that all work is complete in st's order.
// Every buffer one stream writes while the other may read it is its own, and
// each gradient is reduced by the same kernels in the same order as on one
// stream, so the results do not depend on how the two overlap.
static hipError_t loss_grad_fused(mlp_ctx *c, const float *th, const float *Ylab, const float *Jlab, const float *jw,
                                  const int32_t *idx, int B, float w, double *loss, float *g, hipStream_t st)
{
    const int H = c->H, nin = c->nin, NR = nin + 1, R = NR * B;
    const int nwg = B / 32;   // workgroups (32 samples each) along the batch
    hipStream_t sd = c->side;
    hipError_t e = forward_fused(c, th, idx, B, B, false, st);
    if (e == hipSuccess) e = launch_gemm(true, true, c->A[3], H, c->WT[3], H, c->Z[4], kOutPad, R, kOutPad, H, 1, st);
    if (e != hipSuccess) return e;
    // the loss and the output layer's adjoint (elementwise over the R x 64 outputs)
    const unsigned nlb = nb((int64_t)B * kOutPad);
    hipLaunchKernelGGL(k_loss, dim3(nlb), dim3(kThreads), 0, st, c->Z[4], c->p + c->off[7], Ylab, Jlab, jw, idx, B, nin,
                       c->nout, w, c->in_scale, c->out_shift, c->out_scale, c->G4, c->ZbarP, c->lossp);
    const int S = std::min(kMaxSplits, std::max(1, R / 512));
    // side: the loss, b4bar and W4bar = A3^T G4
    if ((e = hipEventRecord(c->ev[0], st)) != hipSuccess || (e = hipStreamWaitEvent(sd, c->ev[0], 0)) != hipSuccess)
        return e;
    hipLaunchKernelGGL(k_sum_partials, dim3(1), dim3(kThreads), 0, sd, c->lossp, (int)nlb, loss);
    colsum(c->gsplit, c->ZbarP, B, kOutPad, c->nout, g + c->off[7], sd);
    e = launch_gemm(false, false, c->A[3], H, c->G4, kOutPad, c->gsplit, kOutPad, H, kOutPad, R, S, sd);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_split_reduce, dim3(nb((int64_t)H * c->nout * 8)), dim3(kThreads), 0, sd, c->gsplit, S, H,
                       kOutPad, g + c->off[6], c->nout, c->nout);
    // hidden layers 3 and 2: H_l bar = (adjoint above) W_{l+1}^T with layer l's
    // activation adjoint in the epilogue (st); then b_l bar and W_l bar (side)
    const uint16_t *adj = c->G4;   // the adjoint of the layer above's input
    int kadj = kOutPad;
    uint16_t *zb[2] = {c->Zbar, c->Zbar2};
    for (int l = 3; l >= 2 && e == hipSuccess; --l) {
        RowsArgs b{};
        b.A = adj;
        b.W = c->Wb[l];
        b.Bp = B;
        b.K = kadj;
        b.N = H;
        b.Zp_in = c->Z[l];
        b.U_in = c->U[l];
        b.Zbar = zb[l & 1];
        b.part = c->rpart[l & 1];
        e = launch_rows(NR, kEpiActBwd, b, st);
        if (e != hipSuccess) break;
        if ((e = hipEventRecord(c->ev[4 - l], st)) != hipSuccess ||
            (e = hipStreamWaitEvent(sd, c->ev[4 - l], 0)) != hipSuccess)
            break;
        hipLaunchKernelGGL(k_chunk_reduce, dim3((H + kThreads / 8 - 1) / (kThreads / 8)), dim3(kThreads), 0, sd,
                           c->rpart[l & 1], nwg, H, g + c->off[2 * l - 1]);
        e = launch_gemm(false, false, c->A[l - 1], H, zb[l & 1], H, c->gsplit, H, H, H, R, S, sd);
        if (e != hipSuccess) break;
        hipLaunchKernelGGL(k_split_reduce, dim3(nb((int64_t)H * H * 8)), dim3(kThreads), 0, sd, c->gsplit, S, H, H,
                           g + c->off[2 * l - 2], H, H);
        adj = zb[l & 1];
        kadj = H;
    }
    if (e != hipSuccess) return e;
    // layer 1: H1bar = Zbar W2^T, reduced in the epilogue to column partials of W1bar and b1bar
    RowsArgs d{};
    d.A = adj;
    d.W = c->Wb[1];
    d.Bp = B;
    d.K = H;
    d.N = H;
    d.Zp_in = c->Z[1];
    d.W1 = c->p + c->off[0];
    d.X = c->Xn;
    d.part = c->split;
    e = launch_rows(NR, kEpiL1Bwd, d, st);
    if (e != hipSuccess) return e;
    const int nout1 = NR * H;   // W1bar (nin rows) and b1bar are contiguous in the gradient
    hipLaunchKernelGGL(k_chunk_reduce, dim3((nout1 + kThreads / 8 - 1) / (kThreads / 8)), dim3(kThreads), 0, st,
                       c->split, nwg, nout1, g + c->off[0]);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if ((e = hipEventRecord(c->ev[3], sd)) != hipSuccess) return e;
    return hipStreamWaitEvent(st, c->ev[3], 0);
}

extern "C" int mlp_loss_grad(mlp_ctx *c, const float *d_theta, const float *d_Ylab, const float *d_Jlab,
                             const float *d_jw, const int32_t *d_idx, int32_t B, float w, double *d_loss, float *d_grad,
                             void *stream)
{
    if (!c || !d_theta || !d_Ylab || !d_Jlab || !d_loss || !d_grad) return mfail(c, -1, "null argument");
    if (B < 128 || B > c->Bmax || B % 128)
        return mfail(c, -1, "training batch must be a multiple of 128 up to max_batch");
    hipStream_t st = (hipStream_t)stream;
    const int H = c->H, nin = c->nin, R = (nin + 1) * B;
    float *g = d_grad;
    hipError_t e = hipSuccess;
    if (fused_path(c)) {
        e = loss_grad_fused(c, d_theta, d_Ylab, d_Jlab, d_jw, d_idx, B, w, d_loss, g, st);
        return e == hipSuccess ? 0 : mfail(c, -3, hipGetErrorString(e));
    }
    e = forward_core(c, d_theta, d_idx, B, B, st);
    if (e != hipSuccess) return mfail(c, -3, hipGetErrorString(e));
    // loss and the output-layer adjoint
    const unsigned nlb = nb((int64_t)B * kOutPad);
    hipLaunchKernelGGL(k_loss, dim3(nlb), dim3(kThreads), 0, st, c->Z[4], c->p + c->off[7], d_Ylab, d_Jlab, d_jw,
                       d_idx, B, nin, c->nout, w, c->in_scale, c->out_shift, c->out_scale, c->G4, c->ZbarP, c->lossp);
    hipLaunchKernelGGL(k_sum_partials, dim3(1), dim3(kThreads), 0, st, c->lossp, (int)nlb, d_loss);
    colsum(c->split, c->ZbarP, B, kOutPad, c->nout, g + c->off[7], st);
    // output layer: W4bar = A3^T G4 (split over rows), H3bar = G4 W4^T
    const int S = std::min(kMaxSplits, std::max(1, R / 512));
    e = launch_gemm(false, false, c->A[3], H, c->G4, kOutPad, c->split, kOutPad, H, kOutPad, R, S, st);
    if (e == hipSuccess) {
        hipLaunchKernelGGL(k_split_reduce, dim3(nb((int64_t)H * c->nout * 8)), dim3(kThreads), 0, st, c->split, S, H,
                           kOutPad, g + c->off[6], c->nout, c->nout);
        e = launch_gemm(true, true, c->G4, kOutPad, c->Wb[3], kOutPad, c->Hbar, H, R, H, kOutPad, 1, st);
    }
    // hidden layers 3 and 2
    for (int l = 3; l >= 2 && e == hipSuccess; --l) {
        hipLaunchKernelGGL(k_act_bwd, dim3(nb((int64_t)B * H)), dim3(kThreads), 0, st, c->Hbar, c->Z[l], B, nin, H,
                           c->Zbar, c->ZbarP);
        colsum(c->split, c->ZbarP, B, H, H, g + c->off[2 * l - 1], st);
        e = launch_gemm(false, false, c->A[l - 1], H, c->Zbar, H, c->split, H, H, H, R, S, st);
        if (e != hipSuccess) break;
        hipLaunchKernelGGL(k_split_reduce, dim3(nb((int64_t)H * H * 8)), dim3(kThreads), 0, st, c->split, S, H, H,
                           g + c->off[2 * l - 2], H, H);
        e = launch_gemm(true, true, c->Zbar, H, c->Wb[l - 1], H, c->Hbar, H, R, H, H, 1, st);
    }
    if (e == hipSuccess) {
        // W1bar (nin rows) and b1bar are contiguous in the gradient: one (nin + 1) x H reduction
        const int nchunk = B / kChunkL1;
        launch_l1_bwd(nin, dim3(nchunk, (H + kThreads - 1) / kThreads), st, c->Hbar, c->Z[1], c->p + c->off[0], c->Xn,
                      B, H, c->split);
        const int nout1 = (nin + 1) * H;
        hipLaunchKernelGGL(k_chunk_reduce, dim3((nout1 + kThreads / 8 - 1) / (kThreads / 8)), dim3(kThreads), 0, st,
                           c->split, nchunk, nout1, g + c->off[0]);
        e = hipGetLastError();
    }
    return e == hipSuccess ? 0 : mfail(c, -3, hipGetErrorString(e));
}

extern "C" int mlp_adam_step(mlp_ctx *c, const float *d_grad, float lr, float beta1, float beta2, float eps, int32_t t,
                             void *stream)
{
    if (!c || !d_grad) return mfail(c, -1, "null argument");
    if (t < 1) return mfail(c, -1, "Adam step count starts at 1");
    hipStream_t st = (hipStream_t)stream;
    const float bc1 = 1.f - std::pow(beta1, (float)t), bc2 = 1.f - std::pow(beta2, (float)t);
    hipLaunchKernelGGL(k_adam, dim3(nb(c->np)), dim3(kThreads), 0, st, c->p, d_grad, c->m, c->v, c->np, lr, beta1,
                       beta2, eps, bc1, bc2);
    hipError_t e = hipGetLastError();
    if (e == hipSuccess) e = refresh_all(c, st);
    return e == hipSuccess ? 0 : mfail(c, -3, hipGetErrorString(e));
}

extern "C" int mlp_adam_step_dev(mlp_ctx *c, const float *d_grad, const float *d_lr, float beta1, float beta2,
                                 float eps, int32_t *d_t, void *stream)
{
    if (!c || !d_grad || !d_lr || !d_t) return mfail(c, -1, "null argument");
    hipStream_t st = (hipStream_t)stream;
    WeightCopies wc{};
    for (int l = 2; l <= 4; ++l) {
        const int k = l - 2;
        wc.off[k] = c->off[2 * (l - 1)];
        wc.in[k] = c->H;
        wc.out[k] = l == 4 ? c->nout : c->H;
        wc.out_pad[k] = l == 4 ? kOutPad : c->H;
        wc.WT[k] = c->WT[l - 1];
        wc.Wb[k] = c->Wb[l - 1];
    }
    hipLaunchKernelGGL(k_adam_dev, dim3(std::min<unsigned>(nb(c->np), kAdamGroups)), dim3(kThreads), 0, st, c->p,
                       d_grad, c->m, c->v, c->np, d_lr, beta1, beta2, eps, d_t, c->done, wc);
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? 0 : mfail(c, -3, hipGetErrorString(e));
}

extern "C" int mlp_calibration_gradient(mlp_ctx *c, const float *d_theta, int32_t B, const double *d_C, float *d_Y,
                                        float *d_J, double *d_G, double *d_grad, void *stream)
{
    if (c && d_theta && d_Y && d_J && d_C && d_G && d_grad && B >= 1 && B <= c->Bmax && small_path(c, B)) {
        const hipError_t e = launch_small(c, d_theta, B, d_C, d_Y, d_J, d_G, d_grad, (hipStream_t)stream);
        return e == hipSuccess ? 0 : mfail(c, -3, hipGetErrorString(e));
    }
    int rc = mlp_forward(c, d_theta, B, d_Y, d_J, stream);
    if (rc) return rc;
    if (!d_C || !d_G || !d_grad) return mfail(c, -1, "null argument");
    hipLaunchKernelGGL(k_calib_grad, dim3((unsigned)B), dim3(kThreads), 0, (hipStream_t)stream, d_Y, d_J, d_C, c->nout,
                       c->nin, d_G, d_grad);
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? 0 : mfail(c, -3, hipGetErrorString(e));
}

extern "C" const char *mlp_last_error(const mlp_ctx *c) { return c ? c->err.c_str() : g_mlp_err.c_str(); }
