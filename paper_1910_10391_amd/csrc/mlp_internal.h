// Internal data structures of the BF16 MLP kernels (learned angular sampler).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace radmlp {

constexpr int kWidth = 256;   // hidden width
constexpr int kIn1 = 64;      // layer-1 inputs padded to one MFMA-friendly width

enum { kEpiFwd = 0, kEpiBwd = 1 };

constexpr int kRowBlock = 128;   // batches are padded to a multiple of this many rows
constexpr int kRowTile = 64;     // rows per block of the row products

// C[M][256] = A[M][K] W^T (A, W BF16, K = 64 or 256 contiguous) with an epilogue:
// forward: z = C + bias, h = bf16(silu(z)) and, in training, ds = bf16(silu'(z)) (the
// factor the backward pass needs, computed here from the FP32 z); backward: dz = C dsin
// (dsin the ds of the layer below), h = bf16(dz) and the per-block column sums of dz
// (col_part [M / 64][256]).  h goes row-major to out_h and, if out_k8 is given, to the k8
// layout [M / 8][256][8].
struct RowsArgs {
    const uint16_t *A, *W;
    int M, K;
    const float *bias;    // forward
    const uint16_t *dsin; // backward: silu' of the layer below (BF16), [M][256]
    uint16_t *out_ds;     // forward, training: silu'(z) (BF16) [M][256] (or null)
    uint16_t *out_h;      // [M][256]
    uint16_t *out_k8;     // [M / 8][256][8] or null
    float *col_part;      // backward: [M / 64][256]
};

// Weight gradients, C[M][N] = sum over the batch of A8[k/8][m][k%8] B8[k/8][n][k%8] (k8
// layouts), split over the batch: part[s][M][N] for slices of kslice rows.
struct K8Args {
    const uint16_t *A8, *B8;
    int M, N;
    int64_t kslice;
    float *part;
    int splits;      // slices of the batch (set by launch_k8)
};

// Offsets of the parameter vector: W1 [256][n_in], b1, W2 [256][256], b2, W3, b3, W4 [256], b4.
struct MlpLayout {
    int n_feat, n_point, n_in;
    int64_t w1, b1, w2, b2, w3, b3, w4, b4, total;
};

hipError_t launch_rows(int epi, const RowsArgs &g, hipStream_t st);
hipError_t launch_k8(const K8Args &g, int splits, hipStream_t st);
// The gradient's final reductions in one launch, each in a fixed order:
// W tasks: out[r][c] = sum_s part[s][r][c] over the split-K slices (part [slices][256]
// [src_cols], out [256][n_cols], n_cols <= src_cols); column-sum tasks: the sums over rows
// of x [M][ld] (first N columns), columns c < split to out[c], the rest to out2[c - split].
constexpr int kFinishW = 3, kFinishC = 3;
struct FinishW {
    const float *part;
    int slices, src_cols, n_cols;
    float *out;
    int blocks;      // set by launch_finish_grad
};
struct FinishC {
    const float *x;
    int64_t ld;
    int M, N, split;
    float *out, *out2;
    int blocks;      // set by launch_finish_grad
};
struct FinishArgs {
    FinishW w[kFinishW];
    FinishC c[kFinishC];
};
hipError_t launch_finish_grad(FinishArgs f, hipStream_t st);
hipError_t launch_assemble_in1(const float *feat, int nf, const int *traj, const float *x, int np, int B, int Bp,
                               uint16_t *in1, uint16_t *in1_k8, hipStream_t st);
hipError_t launch_fold_bias(const uint16_t *W1p, const float *b1, const float *feat, int nf, int n_traj, float *cb,
                            hipStream_t st);
hipError_t launch_layer1_points(const uint16_t *W1p, const float *cb, int nf, const int *traj, const float *x, int np,
                                int B, int Bp, uint16_t *h1, hipStream_t st);
hipError_t launch_output(const uint16_t *h3, const uint16_t *W4b, const float *b4, int B, int Bp, float *y,
                         hipStream_t st);
// training: y, dz3 (BF16 row-major and k8) and per-block partial sums [Bp / 64][514]:
// b3 gradient, W4 gradient, b4 gradient, sum of squared errors
constexpr int kOutPointsHost = 64;
constexpr int kOutPartHost = 2 * kWidth + 2;
hipError_t launch_output_grad(const uint16_t *h3, const uint16_t *W4b, const float *b4, int B, int Bp,
                              const float *target, const uint16_t *ds3, uint16_t *dzb, uint16_t *dz_k8, float *part,
                              hipStream_t st);
hipError_t launch_adam(float *p, float *m1, float *m2, const float *g, int64_t n, float lr, float b1, float b2,
                       float eps, float c1, float c2, hipStream_t st);
hipError_t launch_refresh(const float *p, const MlpLayout &L, uint16_t *W1p, uint16_t *W2, uint16_t *W2T,
                          uint16_t *W3, uint16_t *W3T, uint16_t *W3P, uint16_t *W4, hipStream_t st);
// Fused inference (n_point <= 8): y for B points, cb from fold_bias; one block per CU.
// traj null: grid form, point m is (trajectory m / n_pts, point m % n_pts of x).
constexpr int kFusedMaxPointHost = 8;
hipError_t launch_infer_fused(const uint16_t *W1p, const uint16_t *W2, const uint16_t *W3P, const uint16_t *W4,
                              const float *cb, const float *b2, const float *b3, const float *b4, const int *traj,
                              const float *x, int nf, int np, int64_t B, int64_t n_pts, float *y, int n_cu,
                              hipStream_t st);

}  // namespace radmlp
