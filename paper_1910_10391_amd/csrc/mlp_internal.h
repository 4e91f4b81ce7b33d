// Internal data structures of the BF16 MLP kernels (learned angular sampler).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace radmlp {

constexpr int kWidth = 256;   // hidden width
constexpr int kIn1 = 64;      // layer-1 inputs padded to one MFMA-friendly width

enum { kEpiFwd = 0, kEpiBwd = 1, kEpiPartial = 2 };

// C[m][n] = sum_k A[m][k] B[n][k] with an epilogue (see gemm_nt_kernel).
struct GemmArgs {
    const uint16_t *A, *B;
    int M, N, K, lda, ldb, kslice;
    const float *bias;    // kEpiFwd
    const float *zin;     // kEpiBwd: pre-activation of the layer below, [M][N]
    float *out_z;         // FP32 output [M][N] (or [splits][M][N] partials)
    uint16_t *out_h;      // BF16 output, row stride ldh
    int ldh;
};

// Offsets of the parameter vector: W1 [256][n_in], b1, W2 [256][256], b2, W3, b3, W4 [256], b4.
struct MlpLayout {
    int n_feat, n_point, n_in;
    int64_t w1, b1, w2, b2, w3, b3, w4, b4, total;
};

hipError_t launch_gemm(int epi, const GemmArgs &g, int splits, hipStream_t st);
hipError_t launch_transpose(const uint16_t *in, int M, int N, uint16_t *out, hipStream_t st);
hipError_t launch_colsum(const float *xf, const uint16_t *xb, const float *w, int M, int N, float *part,
                         int slices, float *out, hipStream_t st);
hipError_t launch_sum_slices(const float *part, int slices, int rows, int src_cols, int n_cols, float *out,
                             int64_t out_stride, hipStream_t st);
hipError_t launch_assemble_in1(const float *feat, int nf, const int *traj, const float *x, int np, int B, int Bp,
                               uint16_t *in1, hipStream_t st);
hipError_t launch_fold_bias(const uint16_t *W1p, const float *b1, const float *feat, int nf, int n_traj, float *cb,
                            hipStream_t st);
hipError_t launch_layer1_points(const uint16_t *W1p, const float *cb, int nf, const int *traj, const float *x, int np,
                                int B, int Bp, uint16_t *h1, hipStream_t st);
hipError_t launch_output(const uint16_t *h3, const uint16_t *W4b, const float *b4, int B, int Bp,
                         const float *target, const float *z3, float *y, float *dy, float *sqerr, float *dz3,
                         uint16_t *dz3b, hipStream_t st);
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
