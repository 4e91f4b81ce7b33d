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
__device__ __forceinline__ float dsilu(float z)
{
    const float s = sigmoidf_(z);
    return s * (1.0f + z * (1.0f - s));
}

// ---------------------------------------------------------------- GEMM
// C[m][n] = sum_k A[m][k] B[n][k]; A, B BF16 with K contiguous (lda, ldb in
// elements, multiples of 8, 16-byte aligned rows); M, N multiples of 64; the K
// range of blockIdx.z is [z kslice, (z+1) kslice), a multiple of 16.
// Block = 4 waves in a 2 x 2 arrangement of 32 x 32 MFMA tiles.
// MFMA operand layout (32x32x16 bf16): lane l holds A[l % 32][8 (l / 32) + j] and
// B[l % 32][8 (l / 32) + j], j = 0..7; result register i of lane l is
// C[8 (i / 4) + 4 (l / 32) + i % 4][l % 32].
template <int EPI>
__global__ __launch_bounds__(256) void gemm_nt_kernel(GemmArgs g)
{
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int m0 = blockIdx.x * 64 + (wave & 1) * 32;
    const int n0 = blockIdx.y * 64 + (wave >> 1) * 32;
    const int kb = blockIdx.z * g.kslice;
    const int ke = min(g.K, kb + g.kslice);
    const int r = lane & 31, kh = (lane >> 5) * 8;
    const uint16_t *Ap = g.A + (size_t)(m0 + r) * g.lda + kh;
    const uint16_t *Bp = g.B + (size_t)(n0 + r) * g.ldb + kh;
    floatx16 acc = {};
    for (int k = kb; k < ke; k += 16) {
        const bf16x8 av = *reinterpret_cast<const bf16x8 *>(Ap + k);
        const bf16x8 bv = *reinterpret_cast<const bf16x8 *>(Bp + k);
        acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(av, bv, acc, 0, 0, 0);
    }
    const int col = n0 + r;
#pragma unroll
    for (int i = 0; i < 16; ++i) {
        const int row = m0 + 8 * (i >> 2) + 4 * (lane >> 5) + (i & 3);
        const size_t o = (size_t)row * g.N + col;
        const float v = acc[i];
        if constexpr (EPI == kEpiFwd) {            // z = acc + b; h = silu(z)
            const float z = v + g.bias[col];
            if (g.out_z) g.out_z[o] = z;
            g.out_h[(size_t)row * g.ldh + col] = f2bf(silu(z));
        } else if constexpr (EPI == kEpiBwd) {     // dz = acc * silu'(z_prev)
            const float dz = v * dsilu(g.zin[o]);
            g.out_z[o] = dz;
            g.out_h[(size_t)row * g.ldh + col] = f2bf(dz);
        } else {                                   // split-K partial
            g.out_z[(size_t)blockIdx.z * g.M * g.N + o] = v;
        }
    }
}

// out[n][m] = in[m][n] (BF16), 32 x 32 tiles through LDS; M, N multiples of 32.
__global__ __launch_bounds__(256) void transpose_bf16_kernel(const uint16_t *__restrict__ in, int M, int N,
                                                             uint16_t *__restrict__ out)
{
    __shared__ uint16_t t[32][33];
    const int bx = blockIdx.x * 32, by = blockIdx.y * 32;   // bx over N, by over M
    const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;  // 32 x 8
    for (int j = ty; j < 32; j += 8) t[j][tx] = in[(size_t)(by + j) * N + bx + tx];
    __syncthreads();
    for (int j = ty; j < 32; j += 8) out[(size_t)(bx + j) * M + by + tx] = t[tx][j];
}

// ---------------------------------------------------------------- reductions
// Column sums, out[n] = sum over rows m of w[m] X[m][n] (w null -> 1), X FP32 (xf) or BF16
// (xb), in two passes of one kernel: pass 1 over `slices` row slices writes part[s][n],
// pass 2 sums the slices.  A block of 256 threads takes nb columns x (256 / nb) row lanes:
// lane j of a column sums rows m0 + j, m0 + j + lanes, ... of its slice in order, then
// the lanes are added in a fixed LDS tree, so the result is deterministic.
__global__ __launch_bounds__(256) void colsum_kernel(const float *__restrict__ xf, const uint16_t *__restrict__ xb,
                                                     const float *__restrict__ w, int M, int N, int nb,
                                                     int rows_per, float *__restrict__ out)
{
    __shared__ float red[256];
    const int lanes = 256 / nb;
    const int c = threadIdx.x % nb, j = threadIdx.x / nb;
    const int n = blockIdx.x * nb + c;   // < N: the grid has N / nb blocks along x
    const int s = blockIdx.y;
    const int m0 = s * rows_per, m1 = min(M, m0 + rows_per);
    float acc = 0.0f;
    for (int m = m0 + j; m < m1; m += lanes) {
        const float v = xf ? xf[(size_t)m * N + n] : bf2f(xb[(size_t)m * N + n]);
        acc += w ? w[m] * v : v;
    }
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int h = lanes / 2; h >= 1; h >>= 1) {
        if (j < h) red[threadIdx.x] += red[threadIdx.x + h * nb];
        __syncthreads();
    }
    if (j == 0) out[(size_t)s * N + n] = red[c];
}

__global__ __launch_bounds__(256) void sum_slices(const float *__restrict__ part, int slices, int64_t len,
                                                  float *__restrict__ out, int64_t out_stride, int n_cols,
                                                  int src_cols)
{
    // out row r, column c (c < n_cols) = sum_s part[s][r * src_cols + c]
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t rows = len / src_cols;
    if (i >= rows * n_cols) return;
    const int64_t r = i / n_cols, c = i % n_cols;
    float acc = 0.0f;
    for (int s = 0; s < slices; ++s) acc += part[(size_t)s * len + r * src_cols + c];
    out[r * out_stride + c] = acc;
}

// ---------------------------------------------------------------- input / output layers
// in1[m][c] = bf16(feat[traj[m]][c]) for c < nf, bf16(x[m][c - nf]) for c < nf + np, else 0.
__global__ __launch_bounds__(256) void assemble_in1(const float *__restrict__ feat, int nf, const int *__restrict__ traj,
                                                    const float *__restrict__ x, int np, int B, int Bp,
                                                    uint16_t *__restrict__ in1)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (int64_t)Bp * kIn1) return;
    const int m = (int)(i / kIn1), c = (int)(i % kIn1);
    float v = 0.0f;
    if (m < B) {
        if (c < nf) v = feat[(size_t)traj[m] * nf + c];
        else if (c < nf + np) v = x[(size_t)m * np + (c - nf)];
    }
    in1[i] = f2bf(v);
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

// Output layer: y[m] = b4 + sum_i W4[i] h3[m][i], one wave per point.  Training
// (target != null): also dy[m] = 2 (y - t)/B, loss part, and the start of the
// backward pass dz3[m][i] = dy W4[i] silu'(z3[m][i]) (FP32 and BF16).
// Rows B..Bp-1 are padding: every output there is zero.
__global__ __launch_bounds__(256) void output_layer(const uint16_t *__restrict__ h3, const uint16_t *__restrict__ W4b,
                                                    const float *__restrict__ b4, int B, int Bp,
                                                    const float *__restrict__ target, const float *__restrict__ z3,
                                                    float *__restrict__ y, float *__restrict__ dy,
                                                    float *__restrict__ sqerr, float *__restrict__ dz3,
                                                    uint16_t *__restrict__ dz3b)
{
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int m = blockIdx.x * 4 + wave;
    if (m >= Bp) return;
    if (m >= B) {
        if (lane == 0) {
            y[m] = 0.0f;
            if (target) {
                dy[m] = 0.0f;
                sqerr[m] = 0.0f;
            }
        }
        if (target)
            for (int i = lane; i < kWidth; i += 64) {
                dz3[(size_t)m * kWidth + i] = 0.0f;
                dz3b[(size_t)m * kWidth + i] = 0;
            }
        return;
    }
    float acc = 0.0f;
    for (int i = lane; i < kWidth; i += 64) acc += bf2f(W4b[i]) * bf2f(h3[(size_t)m * kWidth + i]);
    for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off, 64);
    const float ym = acc + b4[0];
    if (lane == 0) y[m] = ym;
    if (!target) return;
    const float d = ym - target[m];
    const float g = 2.0f * d / (float)B;
    if (lane == 0) {
        dy[m] = g;
        sqerr[m] = d * d;
    }
    for (int i = lane; i < kWidth; i += 64) {
        const size_t o = (size_t)m * kWidth + i;
        const float v = g * bf2f(W4b[i]) * dsilu(z3[o]);
        dz3[o] = v;
        dz3b[o] = f2bf(v);
    }
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
hipError_t launch_gemm(int epi, const GemmArgs &g, int splits, hipStream_t st)
{
    const dim3 grid((unsigned)(g.M / 64), (unsigned)(g.N / 64), (unsigned)splits);
    switch (epi) {
    case kEpiFwd: hipLaunchKernelGGL(gemm_nt_kernel<kEpiFwd>, grid, dim3(256), 0, st, g); break;
    case kEpiBwd: hipLaunchKernelGGL(gemm_nt_kernel<kEpiBwd>, grid, dim3(256), 0, st, g); break;
    default: hipLaunchKernelGGL(gemm_nt_kernel<kEpiPartial>, grid, dim3(256), 0, st, g); break;
    }
    return hipGetLastError();
}

hipError_t launch_transpose(const uint16_t *in, int M, int N, uint16_t *out, hipStream_t st)
{
    hipLaunchKernelGGL(transpose_bf16_kernel, dim3((unsigned)(N / 32), (unsigned)(M / 32)), dim3(256), 0, st,
                       in, M, N, out);
    return hipGetLastError();
}

hipError_t launch_colsum(const float *xf, const uint16_t *xb, const float *w, int M, int N, float *part,
                         int slices, float *out, hipStream_t st)
{
    // columns per block: N itself up to 64 (a power of two), else 64 (then pass 2 takes 16)
    auto cols = [](int n, int most) { return n <= most ? n : most; };
    const int nb1 = cols(N, 64), nb2 = cols(N, 16);
    if (M < 1 || N < 1 || slices < 1 || 256 % nb1 != 0 || N % nb1 != 0 || 256 % nb2 != 0 || N % nb2 != 0)
        return hipErrorInvalidValue;
    const int rows_per = (M + slices - 1) / slices;
    hipLaunchKernelGGL(colsum_kernel, dim3((unsigned)(N / nb1), (unsigned)slices), dim3(256), 0, st, xf, xb, w, M,
                       N, nb1, rows_per, part);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(colsum_kernel, dim3((unsigned)(N / nb2), 1u), dim3(256), 0, st, part, nullptr, nullptr,
                       slices, N, nb2, slices, out);
    return hipGetLastError();
}

hipError_t launch_sum_slices(const float *part, int slices, int rows, int src_cols, int n_cols, float *out,
                             int64_t out_stride, hipStream_t st)
{
    const int64_t items = (int64_t)rows * n_cols;
    hipLaunchKernelGGL(sum_slices, dim3((unsigned)((items + 255) / 256)), dim3(256), 0, st, part, slices,
                       (int64_t)rows * src_cols, out, out_stride, n_cols, src_cols);
    return hipGetLastError();
}

hipError_t launch_assemble_in1(const float *feat, int nf, const int *traj, const float *x, int np, int B, int Bp,
                               uint16_t *in1, hipStream_t st)
{
    const int64_t n = (int64_t)Bp * kIn1;
    hipLaunchKernelGGL(assemble_in1, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, feat, nf, traj, x, np,
                       B, Bp, in1);
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

hipError_t launch_output(const uint16_t *h3, const uint16_t *W4b, const float *b4, int B, int Bp,
                         const float *target, const float *z3, float *y, float *dy, float *sqerr, float *dz3,
                         uint16_t *dz3b, hipStream_t st)
{
    hipLaunchKernelGGL(output_layer, dim3((unsigned)((Bp + 3) / 4)), dim3(256), 0, st, h3, W4b, b4, B, Bp, target,
                       z3, y, dy, sqerr, dz3, dz3b);
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
