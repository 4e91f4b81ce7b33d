// BF16 MLP kernels of the learned angular sampler (gfx950).
//
// Network: in = [trajectory features (nf), point inputs (np)] -> 256 -> 256 -> 256 -> 1,
// SiLU activations, BF16 weights and activations, FP32 accumulation, Adam on FP32
// master weights.  The dense layers are matrix products on the MFMA units
// (v_mfma_f32_32x32x16_bf16); the 3-input point layer of inference, the output
// layer, the loss, the reductions and Adam are vector kernels.
//
// Layouts: activations [point][feature] row-major; weights [out][in] row-major;
// a transposed copy [in][out] of the 256 x 256 weights serves the backward
// data products.  BF16 values are stored as uint16 (round to nearest even).
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>

#include "mlp_internal.h"

namespace radmlp {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float floatx16 __attribute__((ext_vector_type(16)));

__device__ __forceinline__ uint16_t f2bf(float f)
{
    uint32_t u = __float_as_uint(f);
    if ((u & 0x7fffffffu) > 0x7f800000u) return 0x7fc0;   // NaN
    u += 0x7fffu + ((u >> 16) & 1u);                       // round to nearest even
    return (uint16_t)(u >> 16);
}

__device__ __forceinline__ float bf2f(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

__device__ __forceinline__ float sigmoidf_(float z) { return 1.0f / (1.0f + __expf(-z)); }
__device__ __forceinline__ float silu(float z) { return z * sigmoidf_(z); }
// silu'(z) = s (1 + z (1 - s)) with s = sigmoid(z)
__device__ __forceinline__ float dsilu_s(float z, float s) { return s * (1.0f + z * (1.0f - s)); }

// ---------------------------------------------------------------- GEMM
// MFMA operand layout (v_mfma_f32_32x32x16_bf16): lane l holds A[l % 32][8 (l / 32) + j]
// and B[l % 32][8 (l / 32) + j], j = 0..7, for C[m][n] = sum_k A[m][k] B[n][k]; result
// register i of lane l is C[8 (i / 4) + 4 (l / 32) + i % 4][l % 32].
//
// Two product shapes cover the network:
// * gemm_rows_kernel: C[Bp][256] = A[Bp][K] W^T (W [256][K], both K contiguous; the
//   layers' forward products and the backward data products).  A block computes 64
//   rows x all 256 columns; K runs in slices of 32 staged through LDS (double buffered,
//   one barrier per slice), so that each A and W element is fetched once per block and
//   shared by the block's four waves; each wave computes 32 x 128 (4 MFMA tiles).  Three
//   blocks fit a CU (at most 168 VGPRs, 53 kB of LDS), so that the blocks' load phases and
//   their store-heavy epilogues overlap.
//   The epilogue applies the layer (bias + SiLU, or times SiLU' of the layer below),
//   stores the results row-major and in the k8 layout below, and, in the backward form,
//   the block's column sums of dz (bias gradients) in a fixed order.
// * gemm_k8_kernel: C[256][N] = sum over the batch of dz[k][m] h[k][n] (weight
//   gradients, K = the batch).  Both operands are read in the k8 layout
//   [Bp / 8][width][8] (8 consecutive batch rows of one unit in 16 bytes), in which an
//   MFMA operand is one coalesced 16-byte load per lane, so no transpose is needed;
//   split-K slices write FP32 partials summed in a fixed order afterwards.
typedef uint16_t bf16x8u __attribute__((ext_vector_type(8)));

template <int EPI, int K>
__global__ __launch_bounds__(256, 3) void gemm_rows_kernel(RowsArgs g)
{
    constexpr int KS = 32;                // K slice
    constexpr int LD = KS + 8;            // LDS row stride (elements): 80 bytes
    constexpr int NS = K / KS;
    // one LDS region: the K loop's A and W stages, reused by the epilogue
    constexpr int kStageA = kRowTile * LD, kStageB = kWidth * LD;
    __shared__ __attribute__((aligned(16))) uint16_t smem[2 * kStageA + 2 * kStageB];
    uint16_t (*sA)[kStageA] = reinterpret_cast<uint16_t (*)[kStageA]>(smem);
    uint16_t (*sB)[kStageB] = reinterpret_cast<uint16_t (*)[kStageB]>(smem + 2 * kStageA);
    __shared__ float sCol[2][kWidth];
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const int wm = wave & 1, wn = wave >> 1;
    const int r = lane & 31, hs = lane >> 5;
    const int64_t row0 = (int64_t)blockIdx.x * kRowTile;
    // global -> register staging of one slice: A 64 x 32 (one chunk of 8 per thread),
    // W 256 x 32 (4 chunks per thread)
    uint4 ra0, rb0, rb1, rb2, rb3;
    const int srr = tid >> 2, skc = (tid & 3) * 8;   // this thread's row (and row + 64 q) and k chunk
    auto load = [&](int s) __attribute__((always_inline)) {
        const uint16_t *a = g.A + (row0 + srr) * K + s * KS + skc;
        const uint16_t *w = g.W + (int64_t)srr * K + s * KS + skc;
        ra0 = *reinterpret_cast<const uint4 *>(a);
        rb0 = *reinterpret_cast<const uint4 *>(w);
        rb1 = *reinterpret_cast<const uint4 *>(w + 64 * K);
        rb2 = *reinterpret_cast<const uint4 *>(w + 128 * K);
        rb3 = *reinterpret_cast<const uint4 *>(w + 192 * K);
    };
    auto store = [&](int buf) __attribute__((always_inline)) {
        uint16_t *w = &sB[buf][srr * LD + skc];
        *reinterpret_cast<uint4 *>(&sA[buf][srr * LD + skc]) = ra0;
        *reinterpret_cast<uint4 *>(w) = rb0;
        *reinterpret_cast<uint4 *>(w + 64 * LD) = rb1;
        *reinterpret_cast<uint4 *>(w + 128 * LD) = rb2;
        *reinterpret_cast<uint4 *>(w + 192 * LD) = rb3;
    };
    floatx16 acc[4];
#pragma unroll
    for (int b = 0; b < 4; ++b) acc[b] = floatx16{};
    load(0);
    store(0);
    __syncthreads();
#pragma unroll 1
    for (int s = 0; s < NS; ++s) {
        const int buf = s & 1;
        if (s + 1 < NS) load(s + 1);
#pragma unroll
        for (int ks = 0; ks < KS / 16; ++ks) {
            const bf16x8 av = *reinterpret_cast<const bf16x8 *>(&sA[buf][(wm * 32 + r) * LD + ks * 16 + 8 * hs]);
            bf16x8 bv[4];
#pragma unroll
            for (int b = 0; b < 4; ++b)
                bv[b] = *reinterpret_cast<const bf16x8 *>(&sB[buf][(wn * 128 + b * 32 + r) * LD + ks * 16 + 8 * hs]);
#pragma unroll
            for (int b = 0; b < 4; ++b) acc[b] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(av, bv[b], acc[b], 0, 0, 0);
        }
        if (s + 1 < NS) store(buf ^ 1);
        __syncthreads();
    }
    // ---- epilogue, one 32 x 32 tile at a time.  A lane holds 4 consecutive rows of one
    // column (the MFMA result layout); the row-major outputs go through a per-wave LDS
    // stage (the K loop's buffers, free after its last barrier) so that every global store
    // is 16 contiguous bytes per lane; the k8 layout takes the 4 rows directly.
    // The wave's 32 x 128 results go through a per-wave LDS stage (the K loop's buffers,
    // free after its last barrier), so that stored row segments are whole 128-byte lines or
    // longer (16 bytes per lane); the k8 copy is written directly (4 consecutive rows of a
    // column are 8 contiguous bytes).  Forward: h and silu'(z) of two 32 x 32 tiles per
    // round (storing the two outputs in separate rounds of whole rows measured slower).
    // Backward: the block's silu' rows are first staged in LDS with 16-byte loads and read
    // into registers; then dz of the wave's 32 x 128 in one round of 256-byte rows.
    const int64_t trow = row0 + wm * 32;        // first row of the wave's tiles
    auto store_k8 = [&](int col, int rt, const uint16_t (&hv)[4]) __attribute__((always_inline)) {
        const int64_t rb = trow + rt;
        const int64_t k8 = ((rb >> 3) * kWidth + col) * 8 + (rb & 7);
        uint2 pk;
        pk.x = (uint32_t)hv[0] | ((uint32_t)hv[1] << 16);
        pk.y = (uint32_t)hv[2] | ((uint32_t)hv[3] << 16);
        *reinterpret_cast<uint2 *>(g.out_k8 + k8) = pk;
    };
    float csum[4] = {0.0f, 0.0f, 0.0f, 0.0f};   // backward: this lane's column sums of dz
    if constexpr (EPI == kEpiFwd) {
        constexpr int HLD = 64 + 8;              // stage row stride (bf16), 16-byte aligned
        uint16_t *hst = smem + wave * (2 * 32 * HLD);
        uint16_t *dst = hst + 32 * HLD;
        static_assert(4 * 2 * 32 * HLD <= 2 * kStageA + 2 * kStageB, "epilogue stage fits");
#pragma unroll
        for (int bp = 0; bp < 2; ++bp) {
#pragma unroll
            for (int bt = 0; bt < 2; ++bt) {
                const int b = 2 * bp + bt;
                const int col = wn * 128 + b * 32 + r;
                const float bias = g.bias[col];
#pragma unroll
                for (int q = 0; q < 4; ++q) {    // rows 8 q + 4 hs + (0..3) of the tile
                    const int rt = 8 * q + 4 * hs;
                    uint16_t hv[4];
#pragma unroll
                    for (int j = 0; j < 4; ++j) {
                        const float z = acc[b][4 * q + j] + bias;
                        const float sg = sigmoidf_(z);
                        hv[j] = f2bf(z * sg);
                        hst[(rt + j) * HLD + bt * 32 + r] = hv[j];
                        dst[(rt + j) * HLD + bt * 32 + r] = f2bf(dsilu_s(z, sg));
                    }
                    if (g.out_k8) store_k8(col, rt, hv);
                }
            }
            __builtin_amdgcn_wave_barrier();     // the wave's stage writes before its reads
            const int c0 = wn * 128 + bp * 64;
#pragma unroll
            for (int k = 0; k < 4; ++k) {        // 32 rows x 8 chunks of 16 bytes
                const int c = lane + 64 * k, rr = c >> 3, cc = c & 7;
                *reinterpret_cast<uint4 *>(g.out_h + (trow + rr) * kWidth + c0 + cc * 8) =
                    *reinterpret_cast<const uint4 *>(&hst[rr * HLD + cc * 8]);
                if (g.out_ds)
                    *reinterpret_cast<uint4 *>(g.out_ds + (trow + rr) * kWidth + c0 + cc * 8) =
                        *reinterpret_cast<const uint4 *>(&dst[rr * HLD + cc * 8]);
            }
            __builtin_amdgcn_wave_barrier();     // reads done before the next round's writes
        }
    } else {
        // rows padded to 264 elements: the two row halves a wave reads fall in disjoint banks
        constexpr int DLD = kWidth + 8;
        uint16_t *sds = smem;
        static_assert(kRowTile * DLD <= 2 * kStageA + 2 * kStageB, "silu' stage fits");
#pragma unroll
        for (int k = 0; k < kRowTile * kWidth / 8 / 256; ++k) {
            const int c = tid + 256 * k, rr = c >> 5, cc = c & 31;
            *reinterpret_cast<uint4 *>(&sds[rr * DLD + cc * 8]) =
                *reinterpret_cast<const uint4 *>(g.dsin + (row0 + rr) * kWidth + cc * 8);
        }
        __syncthreads();
        float dsin[4][16];
#pragma unroll
        for (int b = 0; b < 4; ++b)
#pragma unroll
            for (int i = 0; i < 16; ++i)
                dsin[b][i] = bf2f(sds[(wm * 32 + 8 * (i >> 2) + 4 * hs + (i & 3)) * DLD + wn * 128 + b * 32 + r]);
        __syncthreads();                         // every wave has its values: the stage may overwrite
        constexpr int HLD = 128 + 8;             // stage row stride (bf16), 16-byte aligned
        uint16_t *stg = smem + wave * 32 * HLD;
        static_assert(4 * 32 * HLD <= 2 * kStageA + 2 * kStageB, "epilogue stage fits");
#pragma unroll
        for (int b = 0; b < 4; ++b) {
            const int col = wn * 128 + b * 32 + r;
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int rt = 8 * q + 4 * hs;
                uint16_t hv[4];
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    const float out = acc[b][4 * q + j] * dsin[b][4 * q + j];
                    csum[b] += out;
                    hv[j] = f2bf(out);
                    stg[(rt + j) * HLD + b * 32 + r] = hv[j];
                }
                if (g.out_k8) store_k8(col, rt, hv);
            }
        }
        __builtin_amdgcn_wave_barrier();        // the wave's stage writes before its reads
#pragma unroll
        for (int k = 0; k < 8; ++k) {           // 32 rows x 16 chunks of 16 bytes
            const int c = lane + 64 * k, rr = c >> 4, cc = c & 15;
            *reinterpret_cast<uint4 *>(g.out_h + (trow + rr) * kWidth + wn * 128 + cc * 8) =
                *reinterpret_cast<const uint4 *>(&stg[rr * HLD + cc * 8]);
        }
    }
    if constexpr (EPI == kEpiBwd) {
        // column sums over the block's 64 rows in a fixed order: the two row halves of a
        // tile (lanes l and l ^ 32), then the two row-halves of the block (waves wm = 0, 1)
        // through LDS
#pragma unroll
        for (int b = 0; b < 4; ++b) csum[b] += __shfl_xor(csum[b], 32, 64);
        if (hs == 0)
#pragma unroll
            for (int b = 0; b < 4; ++b) sCol[wm][wn * 128 + b * 32 + r] = csum[b];
        __syncthreads();
        g.col_part[(int64_t)blockIdx.x * kWidth + tid] = sCol[0][tid] + sCol[1][tid];
    }
}

// Weight gradients from the k8 layouts: C[m][n] = sum_k A8[k / 8][m][k % 8] B8[k / 8][n][k % 8]
// over the batch slice [z kslice, (z + 1) kslice); WM x WN tiles of 64 x 64, each computed by
// two waves over alternate 16-row steps of the slice (operands loaded four steps ahead of
// their products), their sums added in a fixed order through LDS.  One-dimensional grid of
// T = 256 / (64 WM) x N / (64 WN) blocks per slice: when the slices come in multiples of 8,
// the T blocks of a slice are given ids congruent mod 8, which puts them on one XCD (blocks
// are dealt to the 8 XCDs round-robin), so that the slice's operands are fetched from HBM
// once into that XCD's L2 and shared by the T blocks.
template <int WM, int WN>
__global__ __launch_bounds__(512) void gemm_k8_kernel(K8Args g)
{
    constexpr int NT = WM * WN;
    constexpr int BM = kWidth / (64 * WM);       // blocks along m
    __shared__ float sRed[NT][64 * 64];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int tile = wave % NT, par = wave / NT;
    const int wm = tile % WM, wn = tile / WM;
    const int r = lane & 31, hs = lane >> 5;
    const int T = BM * (g.N / (64 * WN));
    const int L = blockIdx.x;
    int z, t;
    if (T > 1 && g.splits % 8 == 0) {
        z = L % 8 + 8 * (L / (8 * T));
        t = (L / 8) % T;
    } else {
        z = L / T;
        t = L % T;
    }
    const int m0 = (t % BM) * (64 * WM) + wm * 64, n0 = (t / BM) * (64 * WN) + wn * 64;
    const int64_t kb = (int64_t)z * g.kslice;
    floatx16 acc[2][2];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) acc[a][b] = floatx16{};
    const bf16x8u *A = reinterpret_cast<const bf16x8u *>(g.A8);
    const bf16x8u *B = reinterpret_cast<const bf16x8u *>(g.B8);
    const int steps = (int)(g.kslice / 32);       // pairs of 16-row steps
    auto load = [&](int st, bf16x8 (&av)[2], bf16x8 (&bv)[2]) __attribute__((always_inline)) {
        const int64_t kg = ((kb + 32 * (int64_t)st + 16 * par) >> 3) + hs;
#pragma unroll
        for (int a = 0; a < 2; ++a) av[a] = __builtin_bit_cast(bf16x8, A[kg * g.M + m0 + a * 32 + r]);
#pragma unroll
        for (int b = 0; b < 2; ++b) bv[b] = __builtin_bit_cast(bf16x8, B[kg * g.N + n0 + b * 32 + r]);
    };
    // PD steps of operands in flight: a ring of PD register sets, the loop unrolled by PD
    // so that each set keeps its registers (the products wait on HBM latency otherwise:
    // 33.1 us with two steps ahead, 25.3 us with four, 25.6 us with eight, for the
    // 256 x 256 product)
    constexpr int PD = 4;
    bf16x8 av[PD][2], bv[PD][2];
#pragma unroll
    for (int i = 0; i < PD; ++i)
        if (i < steps) load(i, av[i], bv[i]);
    for (int st = 0; st < steps; st += PD) {
#pragma unroll
        for (int i = 0; i < PD; ++i) {
            if (st + i < steps) {
#pragma unroll
                for (int a = 0; a < 2; ++a)
#pragma unroll
                    for (int b = 0; b < 2; ++b)
                        acc[a][b] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(av[i][a], bv[i][b], acc[a][b], 0, 0, 0);
                if (st + i + PD < steps) load(st + i + PD, av[i], bv[i]);
            }
        }
    }
    if (par == 1) {
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
            for (int b = 0; b < 2; ++b)
#pragma unroll
                for (int i = 0; i < 16; ++i) sRed[tile][((a * 2 + b) * 16 + i) * 64 + lane] = acc[a][b][i];
    }
    __syncthreads();
    if (par == 1) return;
    float *out = g.part + (int64_t)z * g.M * g.N;
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b)
#pragma unroll
            for (int i = 0; i < 16; ++i) {
                const int row = m0 + a * 32 + 8 * (i >> 2) + 4 * hs + (i & 3);
                out[(int64_t)row * g.N + n0 + b * 32 + r] = acc[a][b][i] + sRed[tile][((a * 2 + b) * 16 + i) * 64 + lane];
            }
}

// ---------------------------------------------------------------- reductions
// The gradient's reductions, one launch at the end of the backward pass (none of the
// step's other kernels reads them).  Tasks, by block range:
// * W tasks: out[r][c] = sum over the split-K slices s of part[s][r][src_cols r + c]
//   (r < 256, c < n_cols), four columns per thread where the widths allow, the slices in
//   order;
// * column-sum tasks: out[c] = sum over rows m of x[m][c] (c < N; columns from `split` on
//   go to out2), 4 columns per block, 64 row lanes per column each summing rows j, j + 64,
//   ... in order, then a fixed tree over the lanes.
__global__ __launch_bounds__(256) void finish_grad_kernel(FinishArgs f)
{
    __shared__ float red[256];
    int b = blockIdx.x;
    for (int t = 0; t < kFinishW; ++t) {
        const FinishW &w = f.w[t];
        if (b >= w.blocks) {
            b -= w.blocks;
            continue;
        }
        const int64_t len = (int64_t)kWidth * w.src_cols;
        const int64_t i = (int64_t)b * 256 + threadIdx.x;
        if (w.n_cols % 4 == 0) {
            const int q = w.n_cols / 4;
            if (i >= (int64_t)kWidth * q) return;
            const int64_t r = i / q, c = 4 * (i % q);
            float4 acc = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
#pragma unroll 8
            for (int s = 0; s < w.slices; ++s) {
                const float4 v = *reinterpret_cast<const float4 *>(w.part + s * len + r * w.src_cols + c);
                acc.x += v.x;
                acc.y += v.y;
                acc.z += v.z;
                acc.w += v.w;
            }
            float *o = w.out + r * w.n_cols + c;
            o[0] = acc.x;
            o[1] = acc.y;
            o[2] = acc.z;
            o[3] = acc.w;
        } else {
            if (i >= (int64_t)kWidth * w.n_cols) return;
            const int64_t r = i / w.n_cols, c = i % w.n_cols;
            float acc = 0.0f;
#pragma unroll 8
            for (int s = 0; s < w.slices; ++s) acc += w.part[s * len + r * w.src_cols + c];
            w.out[r * w.n_cols + c] = acc;
        }
        return;
    }
    for (int t = 0; t < kFinishC; ++t) {
        const FinishC &c = f.c[t];
        if (b >= c.blocks) {
            b -= c.blocks;
            continue;
        }
        const int col = 4 * b + (threadIdx.x & 3), j = threadIdx.x >> 2;
        float acc = 0.0f;
        if (col < c.N)
            for (int m = j; m < c.M; m += 64) acc += c.x[(int64_t)m * c.ld + col];
        red[threadIdx.x] = acc;
        __syncthreads();
        for (int h = 32; h >= 1; h >>= 1) {
            if (j < h) red[threadIdx.x] += red[threadIdx.x + 4 * h];
            __syncthreads();
        }
        if (j == 0 && col < c.N) {
            if (col < c.split) c.out[col] = red[threadIdx.x];
            else c.out2[col - c.split] = red[threadIdx.x];
        }
        return;
    }
}

// ---------------------------------------------------------------- input / output layers
// in1[m][c] = bf16(feat[traj[m]][c]) for c < nf, bf16(x[m][c - nf]) for c < nf + np, else 0;
// also in the k8 layout in1_k8[m / 8][c][m % 8] when it is not null.
__global__ __launch_bounds__(256) void assemble_in1(const float *__restrict__ feat, int nf, const int *__restrict__ traj,
                                                    const float *__restrict__ x, int np, int B, int Bp,
                                                    uint16_t *__restrict__ in1, uint16_t *__restrict__ in1_k8)
{
    // one thread per (group of 8 rows, column): 8 row-major entries (a wave writes 128
    // contiguous bytes per row) and one 16-byte chunk of the k8 layout
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (int64_t)(Bp / 8) * kIn1) return;
    const int grp = (int)(i / kIn1), c = (int)(i % kIn1);
    uint16_t h[8];
#pragma unroll
    for (int p = 0; p < 8; ++p) {
        const int m = 8 * grp + p;
        float v = 0.0f;
        if (m < B) {
            if (c < nf) v = feat[(size_t)traj[m] * nf + c];
            else if (c < nf + np) v = x[(size_t)m * np + (c - nf)];
        }
        h[p] = f2bf(v);
        in1[(int64_t)m * kIn1 + c] = h[p];
    }
    if (in1_k8) {
        uint4 pk;
        pk.x = (uint32_t)h[0] | ((uint32_t)h[1] << 16);
        pk.y = (uint32_t)h[2] | ((uint32_t)h[3] << 16);
        pk.z = (uint32_t)h[4] | ((uint32_t)h[5] << 16);
        pk.w = (uint32_t)h[6] | ((uint32_t)h[7] << 16);
        *reinterpret_cast<uint4 *>(in1_k8 + i * 8) = pk;
    }
}

// Inference, trajectory part of layer 1 folded into a bias:
// cb[t][o] = b1[o] + sum_{f < nf} W1[o][f] bf16(feat[t][f]).
__global__ __launch_bounds__(256) void fold_bias(const uint16_t *__restrict__ W1p, const float *__restrict__ b1,
                                                 const float *__restrict__ feat, int nf, int n_traj,
                                                 float *__restrict__ cb)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n_traj * kWidth) return;
    const int t = i / kWidth, o = i % kWidth;
    float acc = 0.0f;
    for (int f = 0; f < nf; ++f) acc += bf2f(W1p[o * kIn1 + f]) * bf2f(f2bf(feat[(size_t)t * nf + f]));
    cb[i] = acc + b1[o];
}

// Inference layer 1 on the point inputs: h1[m][o] = silu(cb[traj[m]][o] + sum_j W1[o][nf+j] bf16(x[m][j])).
__global__ __launch_bounds__(256) void layer1_points(const uint16_t *__restrict__ W1p, const float *__restrict__ cb,
                                                     int nf, const int *__restrict__ traj,
                                                     const float *__restrict__ x, int np, int B, int Bp,
                                                     uint16_t *__restrict__ h1)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (int64_t)Bp * kWidth) return;
    const int m = (int)(i / kWidth), o = (int)(i % kWidth);
    float z = 0.0f;
    if (m < B) {
        z = cb[(size_t)traj[m] * kWidth + o];
        for (int j = 0; j < np; ++j) z += bf2f(W1p[o * kIn1 + nf + j]) * bf2f(f2bf(x[(size_t)m * np + j]));
    }
    h1[i] = f2bf(silu(z));
}

// Output layer: y[m] = b4 + sum_i W4[i] h3[m][i], one wave per point (inference).
__global__ __launch_bounds__(256) void output_layer(const uint16_t *__restrict__ h3, const uint16_t *__restrict__ W4b,
                                                    const float *__restrict__ b4, int B, int Bp,
                                                    float *__restrict__ y)
{
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int m = blockIdx.x * 4 + wave;
    if (m >= Bp) return;
    if (m >= B) {
        if (lane == 0) y[m] = 0.0f;
        return;
    }
    float acc = 0.0f;
    for (int i = lane; i < kWidth; i += 64) acc += bf2f(W4b[i]) * bf2f(h3[(size_t)m * kWidth + i]);
    for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off, 64);
    if (lane == 0) y[m] = acc + b4[0];
}

// Output layer of a training step, 64 points per block (16 per wave, lane j owning units
// j + 64 q): y = b4 + W4 . h3, d = y - target, dy = 2 d / B, and the start of the backward
// pass dz3 = dy W4 silu'(z3) (silu'(z3) as the forward epilogue stored it, in BF16), stored
// in BF16 row-major and in the k8 layout (8 points at a time, one 16-byte store per unit).  The block's sums, in a fixed order, go to
// part[block][0 .. 513): the b3 gradient (sum of dz3, FP32), the W4 gradient (sum of
// dy h3), the b4 gradient (sum of dy), then the sum of d^2.  Rows B..Bp-1 are padding:
// every output there is zero.
constexpr int kOutPoints = 64;
constexpr int kOutPart = 2 * kWidth + 2;
static_assert(kOutPoints == kOutPointsHost && kOutPart == kOutPartHost, "output partials");
static_assert(kRowBlock % kOutPoints == 0, "row blocks hold whole output blocks");

__global__ __launch_bounds__(256) void output_grad_kernel(const uint16_t *__restrict__ h3,
                                                          const uint16_t *__restrict__ W4b,
                                                          const float *__restrict__ b4, int B,
                                                          const float *__restrict__ target,
                                                          const uint16_t *__restrict__ ds3,
                                                          uint16_t *__restrict__ dzb, uint16_t *__restrict__ dz_k8,
                                                          float *__restrict__ part)
{
    __shared__ float sP[4][kOutPart];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    float w4[4], sb3[4] = {0.0f, 0.0f, 0.0f, 0.0f}, sw4[4] = {0.0f, 0.0f, 0.0f, 0.0f};
    float sdy = 0.0f, ssq = 0.0f;
#pragma unroll
    for (int q = 0; q < 4; ++q) w4[q] = bf2f(W4b[lane + 64 * q]);
    const float inv = 2.0f / (float)B;
    for (int grp = 0; grp < 2; ++grp) {
        const int64_t mg = (int64_t)blockIdx.x * kOutPoints + wave * 16 + grp * 8;   // multiple of 8
        // all loads of the 8 points first, then their 8 reductions side by side
        float hq[8][4], zq[8][4], acc[8];
#pragma unroll
        for (int p = 0; p < 8; ++p)
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int64_t o = (mg + p) * kWidth + lane + 64 * q;
                hq[p][q] = bf2f(h3[o]);
                zq[p][q] = bf2f(ds3[o]);
            }
#pragma unroll
        for (int p = 0; p < 8; ++p) {
            acc[p] = 0.0f;
#pragma unroll
            for (int q = 0; q < 4; ++q) acc[p] += w4[q] * hq[p][q];
        }
#pragma unroll
        for (int off = 32; off > 0; off >>= 1)
#pragma unroll
            for (int p = 0; p < 8; ++p) acc[p] += __shfl_xor(acc[p], off, 64);
        uint16_t hv[4][8];
#pragma unroll
        for (int p = 0; p < 8; ++p) {
            const int64_t m = mg + p;
            const bool real = m < B;
            const float d = real ? acc[p] + b4[0] - target[m] : 0.0f;
            const float gdy = inv * d;
            sdy += gdy;
            ssq += d * d;
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int64_t o = m * kWidth + lane + 64 * q;
                const float dz = real ? gdy * w4[q] * zq[p][q] : 0.0f;
                sb3[q] += dz;
                sw4[q] += gdy * hq[p][q];
                hv[q][p] = f2bf(dz);
                dzb[o] = hv[q][p];
            }
        }
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            uint4 pk;
            pk.x = (uint32_t)hv[q][0] | ((uint32_t)hv[q][1] << 16);
            pk.y = (uint32_t)hv[q][2] | ((uint32_t)hv[q][3] << 16);
            pk.z = (uint32_t)hv[q][4] | ((uint32_t)hv[q][5] << 16);
            pk.w = (uint32_t)hv[q][6] | ((uint32_t)hv[q][7] << 16);
            *reinterpret_cast<uint4 *>(dz_k8 + ((mg >> 3) * kWidth + lane + 64 * q) * 8) = pk;
        }
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        sP[wave][lane + 64 * q] = sb3[q];
        sP[wave][kWidth + lane + 64 * q] = sw4[q];
    }
    if (lane == 0) {
        sP[wave][2 * kWidth] = sdy;
        sP[wave][2 * kWidth + 1] = ssq;
    }
    __syncthreads();
    for (int i = threadIdx.x; i < kOutPart; i += 256)
        part[(int64_t)blockIdx.x * kOutPart + i] = ((sP[0][i] + sP[1][i]) + sP[2][i]) + sP[3][i];
}

// ---------------------------------------------------------------- Adam and working copies
__global__ __launch_bounds__(256) void adam_kernel(float *__restrict__ p, float *__restrict__ m1,
                                                   float *__restrict__ m2, const float *__restrict__ g, int64_t n,
                                                   float lr, float b1, float b2, float eps, float c1, float c2)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float gi = g[i];
    const float a = b1 * m1[i] + (1.0f - b1) * gi;
    const float v = b2 * m2[i] + (1.0f - b2) * gi * gi;
    m1[i] = a;
    m2[i] = v;
    p[i] -= lr * (a / c1) / (sqrtf(v / c2) + eps);
}

// Column order of W3 for the fused inference kernel: within every group of 16
// columns, position q = 8 h + j (h = 0, 1; j = 0..7) holds column 8 (j / 4) + 4 h + j % 4
// of the group.  That is the order in which a lane of infer_fused_kernel holds the
// layer-2 outputs (the MFMA result layout), so they serve as the next product's
// operand without a transpose.
__host__ __device__ inline int w3_fused_column(int q)
{
    const int g = q & ~15, h = (q >> 3) & 1, j = q & 7;
    return g + 8 * (j >> 2) + 4 * h + (j & 3);
}

// BF16 working copies of the FP32 masters: W1 padded to kIn1 columns, W2, W3 and
// their transposes, W3 in the fused kernel's column order, W4.
__global__ __launch_bounds__(256) void refresh_bf16(const float *__restrict__ p, MlpLayout L,
                                                    uint16_t *__restrict__ W1p, uint16_t *__restrict__ W2,
                                                    uint16_t *__restrict__ W2T, uint16_t *__restrict__ W3,
                                                    uint16_t *__restrict__ W3T, uint16_t *__restrict__ W3P,
                                                    uint16_t *__restrict__ W4)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t sq = (int64_t)kWidth * kWidth;
    if (i < (int64_t)kWidth * kIn1) {
        const int o = (int)(i / kIn1), c = (int)(i % kIn1);
        W1p[i] = c < L.n_in ? f2bf(p[L.w1 + (int64_t)o * L.n_in + c]) : (uint16_t)0;
    }
    if (i < sq) {
        const int o = (int)(i / kWidth), c = (int)(i % kWidth);
        W2[i] = f2bf(p[L.w2 + i]);
        W3[i] = f2bf(p[L.w3 + i]);
        W2T[(int64_t)c * kWidth + o] = f2bf(p[L.w2 + i]);
        W3T[(int64_t)c * kWidth + o] = f2bf(p[L.w3 + i]);
        W3P[i] = f2bf(p[L.w3 + (int64_t)o * kWidth + w3_fused_column(c)]);
    }
    if (i < kWidth) W4[i] = f2bf(p[L.w4 + i]);
}

// ---------------------------------------------------------------- fused inference
// y = W4 silu(W3 silu(W2 silu(cb[traj] + W1x x) + b2) + b3) + b4 for 32 points per wave
// without storing activations: a persistent grid, one block per CU, W2 (BF16) resident
// in LDS (rows padded to 264 elements, so that the 32 rows an MFMA operand read touches
// fall in distinct banks).  Products are computed transposed, C^T = W h^T (output units
// as MFMA rows, points as columns): a lane then holds one point's values, the layer-1
// activations are formed directly in the operand layout, and the layer-2 results in
// the MFMA result layout are the layer-3 operand once W3's columns are permuted
// (w3_fused_column).  BF16 rounding points as in the unfused path.
constexpr int kFusedRow = kWidth + 8;
constexpr int kFusedMaxPoint = 8;
constexpr int kFusedWaves = 8;                     // 2 per SIMD: one block per CU holds the LDS
constexpr int kFusedThreads = 64 * kFusedWaves;

struct FusedArgs {
    const uint16_t *W1p, *W2, *W3P, *W4;
    const float *cb, *b2, *b3, *b4;
    const int *traj;    // per-point trajectory, or null for the grid form
    const float *x;     // [B][np], or the point table [n_pts][np] of the grid form
    int nf, np;
    int64_t B;          // points (grid form: n_traj * n_pts, point m = (m / n_pts, m % n_pts))
    int64_t n_pts;
    float *y;
};

// Round to BF16 (nearest even; the gfx950 conversion instruction) and pack 8 values.
__device__ __forceinline__ bf16x8 pack_bf16x8(const float v[8])
{
    bf16x8 r;
#pragma unroll
    for (int k = 0; k < 8; ++k) r[k] = (__bf16)v[k];
    return r;
}

__device__ __forceinline__ float round_bf16(float v) { return (float)(__bf16)v; }

// SiLU with the hardware reciprocal (1 ulp) instead of an IEEE division.
__device__ __forceinline__ float silu_fast(float z) { return z * __builtin_amdgcn_rcpf(1.0f + __expf(-z)); }

template <int NPMAX>
__global__ __launch_bounds__(kFusedThreads, 1) void infer_fused_kernel(FusedArgs a)
{
    __shared__ __attribute__((aligned(16))) uint16_t sW2[kWidth * kFusedRow];
    __shared__ float sW1[kWidth * kFusedMaxPoint];
    __shared__ float sb2[kWidth], sb3[kWidth], sW4[kWidth];
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    for (int i = tid; i < kWidth * (kWidth / 8); i += kFusedThreads) {
        const int r = i / (kWidth / 8), c8 = i % (kWidth / 8);
        *reinterpret_cast<uint4 *>(&sW2[r * kFusedRow + c8 * 8]) =
            *reinterpret_cast<const uint4 *>(&a.W2[r * kWidth + c8 * 8]);
    }
    // point weights of layer 1, zero beyond n_point so that every unit runs NPMAX products
    for (int i = tid; i < kWidth * kFusedMaxPoint; i += kFusedThreads) {
        const int u = i / kFusedMaxPoint, q = i % kFusedMaxPoint;
        sW1[i] = q < a.np ? bf2f(a.W1p[u * kIn1 + a.nf + q]) : 0.0f;
    }
    for (int i = tid; i < kWidth; i += kFusedThreads) {
        sb2[i] = a.b2[i];
        sb3[i] = a.b3[i];
        sW4[i] = bf2f(a.W4[i]);
    }
    __syncthreads();
    const int r = lane & 31, hs = lane >> 5;
    const int64_t n_tiles = (a.B + 31) / 32;
    for (int64_t tile = (int64_t)blockIdx.x * kFusedWaves + wave; tile < n_tiles;
         tile += (int64_t)gridDim.x * kFusedWaves) {
        const int64_t pt = tile * 32 + r;
        const int64_t pc = pt < a.B ? pt : a.B - 1;      // padding lanes recompute the last point
        int64_t t, xi;
        if (a.traj) {
            t = a.traj[pc];
            xi = pc;
        } else {
            t = pc / a.n_pts;
            xi = pc - t * a.n_pts;
        }
        const float *cbt = a.cb + (size_t)t * kWidth;
        float xv[kFusedMaxPoint];
#pragma unroll
        for (int j = 0; j < kFusedMaxPoint; ++j) xv[j] = j < a.np ? round_bf16(a.x[(size_t)xi * a.np + j]) : 0.0f;
        // layer 1: units ks*16 + 8 hs + j of this lane's point, in operand layout
        bf16x8 h1[kWidth / 16];
#pragma unroll
        for (int ks = 0; ks < kWidth / 16; ++ks) {
            // one group of 8 units at a time (hoisting all 128 bias loads exhausts registers)
            __builtin_amdgcn_sched_barrier(0);
            float v[8];
#pragma unroll
            for (int j = 0; j < 8; ++j) {
                const int u = ks * 16 + 8 * hs + j;
                float z = cbt[u];
#pragma unroll
                for (int q = 0; q < NPMAX; ++q) z += sW1[u * kFusedMaxPoint + q] * xv[q];
                v[j] = silu_fast(z);
            }
            h1[ks] = pack_bf16x8(v);
        }
        // layer 2: C2^T tile mt = W2[mt*32 .. +32][:] h1^T; result register i is unit
        // mt*32 + 8 (i/4) + 4 hs + i%4 of this lane's point
        bf16x8 h2[kWidth / 16];
#pragma unroll
        for (int mt = 0; mt < kWidth / 32; ++mt) {
            // one output tile at a time: keeps the operand reads of later tiles from being
            // hoisted (which would exhaust the registers)
            __builtin_amdgcn_sched_barrier(0);
            floatx16 acc = {};
#pragma unroll
            for (int ks = 0; ks < kWidth / 16; ++ks) {
                const bf16x8 w = *reinterpret_cast<const bf16x8 *>(&sW2[(mt * 32 + r) * kFusedRow + ks * 16 + 8 * hs]);
                acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(w, h1[ks], acc, 0, 0, 0);
            }
#pragma unroll
            for (int s2 = 0; s2 < 2; ++s2) {
                float v[8];
#pragma unroll
                for (int j = 0; j < 8; ++j) {
                    const int i = 8 * s2 + j;
                    const int u = mt * 32 + 8 * (i >> 2) + 4 * hs + (i & 3);
                    v[j] = silu_fast(acc[i] + sb2[u]);
                }
                h2[2 * mt + s2] = pack_bf16x8(v);
            }
        }
        // layer 3 with W3's columns in the same order, then the output dot product; the W3
        // operands come from L2 (the second wave on each SIMD covers their latency)
        __builtin_amdgcn_sched_barrier(0);
        // this lane's W3 row base, re-derived every tile: the empty asm keeps the compiler
        // from hoisting the 128 operand addresses out of the tile loop (which would hold
        // them in registers for the whole kernel)
        const __attribute__((address_space(1))) uint16_t *w3base =
            (const __attribute__((address_space(1))) uint16_t *)(a.W3P + (size_t)r * kWidth + 8 * hs);
        asm volatile("" : "+v"(w3base));
        float ys = 0.0f;
#pragma unroll
        for (int mt = 0; mt < kWidth / 32; ++mt) {
            __builtin_amdgcn_sched_barrier(0);
            const __attribute__((address_space(1))) uint16_t *w3 = w3base + (size_t)mt * 32 * kWidth;
            floatx16 acc = {};
#pragma unroll
            for (int ks = 0; ks < kWidth / 16; ++ks)
                acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(
                    *reinterpret_cast<const __attribute__((address_space(1))) bf16x8 *>(w3 + ks * 16), h2[ks], acc, 0,
                    0, 0);
#pragma unroll
            for (int i = 0; i < 16; ++i) {
                const int u = mt * 32 + 8 * (i >> 2) + 4 * hs + (i & 3);
                ys += sW4[u] * round_bf16(silu_fast(acc[i] + sb3[u]));
            }
        }
        ys += __shfl_xor(ys, 32, 64);
        if (hs == 0 && pt < a.B) a.y[pt] = ys + a.b4[0];
    }
}

// ---------------------------------------------------------------- launchers
hipError_t launch_rows(int epi, const RowsArgs &g, hipStream_t st)
{
    if (g.M % kRowTile || (g.K != kIn1 && g.K != kWidth) || (epi != kEpiFwd && epi != kEpiBwd))
        return hipErrorInvalidValue;
    const dim3 grid((unsigned)(g.M / kRowTile));
    if (epi == kEpiFwd) {
        if (g.K == kIn1) hipLaunchKernelGGL((gemm_rows_kernel<kEpiFwd, kIn1>), grid, dim3(256), 0, st, g);
        else hipLaunchKernelGGL((gemm_rows_kernel<kEpiFwd, kWidth>), grid, dim3(256), 0, st, g);
    } else {
        if (g.K == kIn1) hipLaunchKernelGGL((gemm_rows_kernel<kEpiBwd, kIn1>), grid, dim3(256), 0, st, g);
        else hipLaunchKernelGGL((gemm_rows_kernel<kEpiBwd, kWidth>), grid, dim3(256), 0, st, g);
    }
    return hipGetLastError();
}

hipError_t launch_k8(const K8Args &g, int splits, hipStream_t st)
{
    if (g.M != kWidth || (g.N != kWidth && g.N != kIn1) || g.kslice < 32 || g.kslice % 32 || splits < 1)
        return hipErrorInvalidValue;
    K8Args a = g;
    a.splits = splits;
    if (g.N == kWidth)
        hipLaunchKernelGGL((gemm_k8_kernel<2, 2>), dim3(4u * (unsigned)splits), dim3(512), 0, st, a);
    else
        hipLaunchKernelGGL((gemm_k8_kernel<4, 1>), dim3((unsigned)splits), dim3(512), 0, st, a);
    return hipGetLastError();
}

hipError_t launch_finish_grad(FinishArgs f, hipStream_t st)
{
    int blocks = 0;
    for (FinishW &w : f.w) {
        if (w.slices < 1 || w.n_cols < 1 || w.n_cols > w.src_cols) return hipErrorInvalidValue;
        const bool v4 = w.n_cols % 4 == 0 && w.src_cols % 4 == 0 &&
                        ((uintptr_t)w.part % 16) == 0;
        if (w.n_cols % 4 == 0 && !v4) return hipErrorInvalidValue;
        const int64_t items = (int64_t)kWidth * (w.n_cols % 4 == 0 ? w.n_cols / 4 : w.n_cols);
        w.blocks = (int)((items + 255) / 256);
        blocks += w.blocks;
    }
    for (FinishC &c : f.c) {
        if (c.M < 1 || c.N < 1 || c.split < 0 || c.split > c.N || (c.split < c.N && !c.out2))
            return hipErrorInvalidValue;
        c.blocks = (c.N + 3) / 4;
        blocks += c.blocks;
    }
    hipLaunchKernelGGL(finish_grad_kernel, dim3((unsigned)blocks), dim3(256), 0, st, f);
    return hipGetLastError();
}

hipError_t launch_assemble_in1(const float *feat, int nf, const int *traj, const float *x, int np, int B, int Bp,
                               uint16_t *in1, uint16_t *in1_k8, hipStream_t st)
{
    if (Bp % 8) return hipErrorInvalidValue;
    const int64_t n = (int64_t)(Bp / 8) * kIn1;
    hipLaunchKernelGGL(assemble_in1, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, feat, nf, traj, x, np,
                       B, Bp, in1, in1_k8);
    return hipGetLastError();
}

hipError_t launch_fold_bias(const uint16_t *W1p, const float *b1, const float *feat, int nf, int n_traj, float *cb,
                            hipStream_t st)
{
    const int n = n_traj * kWidth;
    hipLaunchKernelGGL(fold_bias, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, W1p, b1, feat, nf, n_traj, cb);
    return hipGetLastError();
}

hipError_t launch_layer1_points(const uint16_t *W1p, const float *cb, int nf, const int *traj, const float *x, int np,
                                int B, int Bp, uint16_t *h1, hipStream_t st)
{
    const int64_t n = (int64_t)Bp * kWidth;
    hipLaunchKernelGGL(layer1_points, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, W1p, cb, nf, traj, x, np,
                       B, Bp, h1);
    return hipGetLastError();
}

hipError_t launch_output(const uint16_t *h3, const uint16_t *W4b, const float *b4, int B, int Bp, float *y,
                         hipStream_t st)
{
    hipLaunchKernelGGL(output_layer, dim3((unsigned)((Bp + 3) / 4)), dim3(256), 0, st, h3, W4b, b4, B, Bp, y);
    return hipGetLastError();
}

hipError_t launch_output_grad(const uint16_t *h3, const uint16_t *W4b, const float *b4, int B, int Bp,
                              const float *target, const uint16_t *ds3, uint16_t *dzb, uint16_t *dz_k8, float *part,
                              hipStream_t st)
{
    if (Bp % kOutPoints) return hipErrorInvalidValue;
    hipLaunchKernelGGL(output_grad_kernel, dim3((unsigned)(Bp / kOutPoints)), dim3(256), 0, st, h3, W4b, b4, B, target,
                       ds3, dzb, dz_k8, part);
    return hipGetLastError();
}

hipError_t launch_adam(float *p, float *m1, float *m2, const float *g, int64_t n, float lr, float b1, float b2,
                       float eps, float c1, float c2, hipStream_t st)
{
    hipLaunchKernelGGL(adam_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, p, m1, m2, g, n, lr, b1, b2,
                       eps, c1, c2);
    return hipGetLastError();
}

hipError_t launch_refresh(const float *p, const MlpLayout &L, uint16_t *W1p, uint16_t *W2, uint16_t *W2T,
                          uint16_t *W3, uint16_t *W3T, uint16_t *W3P, uint16_t *W4, hipStream_t st)
{
    const int64_t n = (int64_t)kWidth * kWidth;
    hipLaunchKernelGGL(refresh_bf16, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, p, L, W1p, W2, W2T, W3,
                       W3T, W3P, W4);
    return hipGetLastError();
}

hipError_t launch_infer_fused(const uint16_t *W1p, const uint16_t *W2, const uint16_t *W3P, const uint16_t *W4,
                              const float *cb, const float *b2, const float *b3, const float *b4, const int *traj,
                              const float *x, int nf, int np, int64_t B, int64_t n_pts, float *y, int n_cu,
                              hipStream_t st)
{
    if (np > kFusedMaxPoint || np < 1 || B < 1 || (!traj && n_pts < 1)) return hipErrorInvalidValue;
    FusedArgs a{W1p, W2, W3P, W4, cb, b2, b3, b4, traj, x, nf, np, B, n_pts, y};
    const int64_t tiles = (B + 31) / 32;
    const int blocks = (int)std::max<int64_t>(1, std::min<int64_t>(n_cu, (tiles + kFusedWaves - 1) / kFusedWaves));
    if (np <= 4)
        hipLaunchKernelGGL(infer_fused_kernel<4>, dim3((unsigned)blocks), dim3(kFusedThreads), 0, st, a);
    else
        hipLaunchKernelGGL(infer_fused_kernel<kFusedMaxPoint>, dim3((unsigned)blocks), dim3(kFusedThreads), 0, st, a);
    return hipGetLastError();
}

}  // namespace radmlp
