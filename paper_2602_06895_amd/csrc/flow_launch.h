// Host-side launchers of the coupling-flow kernels (defined in flow_kernels.hip).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace msx {

constexpr int kFlowMaxBins = 32;   // spline bins per coordinate
constexpr int kFlowMaxHalf = 32;   // transformed coordinates per layer (dims / 2)

// Element type of the MLP operands on the matrix cores.
enum FlowType : int { FT_BF16 = 0, FT_F32 = 1 };

// Epilogue of a GEMM tile.
enum GemmEpi : int {
    EPI_PARTIAL = 0,    // out_f32[z][m][n] = acc (split-K partial sums)
    EPI_BIAS_RELU = 1,  // out_t[m][n] = T(max(acc + bias[n], 0))
    EPI_BIAS_F32 = 2,   // out_f32[m][n] = acc + bias[n]
    EPI_RELU_MASK = 3,  // out_t[m][n] = T(mask[m][n] > 0 ? acc : 0)
    EPI_F32 = 4         // out_f32[m][n] = acc
};

// C[M][N] (+ epilogue) = sum_k A(m, k) B(k, n) with A(m, k) = A[m a_m + k a_k]
// and B(k, n) = B[k b_k + n b_n] (one of the two strides of each operand is
// 1).  `splits` > 1 divides K into that many chunks (EPI_PARTIAL only).
struct GemmArgs {
    int type;  // FlowType of A, B, out_t and mask
    int M, N, K;
    const void* A;
    int64_t a_m, a_k;
    const void* B;
    int64_t b_k, b_n;
    int splits;
    int epi;
    void* out;
    int64_t ldc;
    const float* bias;
    const void* mask;
    int64_t ldm;
};
hipError_t launch_gemm(const GemmArgs& g, hipStream_t s);

// One whole coupling layer in one kernel (BF16 operands, hidden width 128,
// up to 16 bins): conditioner on the matrix cores and spline (forward, or
// inverse when `inverse`), z updated in place, logdet accumulated.
// params_t / params: the layer's block of the BF16 operand copy (16-byte
// aligned) / of the FP32 parameters (biases), with the offsets off[0..7]
// (W1 b1 W2 b2 W3 b3 W4 b4) in both.  save_x0 [n][nh] BF16, save_h [3][n][128]
// BF16 and save_theta [n][nh (3K + 1)] FP32, when all three are set, receive
// the conditioning inputs, hidden activations and spline parameters.
hipError_t launch_flow_layer(bool inverse, float* z, int64_t n, const void* params_t, const float* params,
                             const int64_t* off, int nh, const int32_t* trans_host, const int32_t* cond_host, int K,
                             float* logdet, void* save_x0, void* save_h, float* save_theta, hipStream_t s);
constexpr int kFusedHidden = 128;
constexpr int kFusedMaxBins = 16;

// out[m][n] = sum_z part[z][m][n] in z order (out has leading dimension ldo).
hipError_t launch_reduce_partials(const float* part, int splits, int M, int N, float* out, int64_t ldo,
                                  hipStream_t s);

// Column sums of an [R][N] matrix of type `type` (bias gradients), written to
// out[N]; `part` holds at least nchunk * N floats.
hipError_t launch_colsum(int type, const void* X, int64_t R, int N, int64_t ldx, float* part, int nchunk, float* out,
                         hipStream_t s);

// X0[b][i] = T(z[cond[i]][b]) for the conditioning coordinates of a layer.
hipError_t launch_gather(int type, const float* z, int64_t n, int n_cond, const int32_t* cond_host, void* x0,
                         hipStream_t s);

// Spline of every transformed coordinate of one layer, one thread per
// (event, coordinate).
//   forward: z[t_j] <- S(z[t_j]), logdet += sum_j log S'
//   inverse: z[t_j] <- S^-1(z[t_j]), logdet += sum_j log (S^-1)'
// ld_part: scratch of n_half x n floats (the per-coordinate terms).
hipError_t launch_spline(bool inverse, float* z, int64_t n, const float* theta, int64_t ldt, int n_half,
                         const int32_t* trans_host, int K, float* logdet, float* ld_part, hipStream_t s);

// Reverse mode through one inverse spline layer.  y: layer input (its
// transformed coordinates, before inversion), adj: adjoint of the layer output
// on entry, of the layer input on exit (transformed coordinates; conditioning
// coordinates are left for launch_scatter_add), G[b] = dLoss/dlogq_b.  Writes
// dtheta (type `type`, leading dimension ldt).
hipError_t launch_spline_backward(int type, const float* y, float* adj, int64_t n, const float* theta, int64_t ldt,
                                  int n_half, const int32_t* trans_host, int K, const float* G, void* dtheta,
                                  hipStream_t s);

// adj[cond[i]][b] += dx0[b][i]
hipError_t launch_scatter_add(float* adj, const float* dx0, int64_t n, int n_cond, const int32_t* cond_host,
                              hipStream_t s);

// G[b] = -F_b exp(-logq_b - logq_old_b) / n with F_b = wfj_b^2, and the loss
// sum_b F_b exp(...) / n into loss[0] (deterministic two-pass sum; `part`
// holds 1024 doubles).  log_loss: G is then divided by the loss (dlogL/dlogq).
hipError_t launch_flow_loss(int64_t n, const double* wfj, const float* logq, const float* logq_old, float* G,
                            double* part, double* loss, bool log_loss, hipStream_t s);

// Adam step on P parameters (bias corrections folded into lr_t, eps_t by the
// caller), then the operand copy of the parameters in `type`.  The copy pads
// each layer block of `per` parameters to `per_t` (a multiple of 8).
hipError_t launch_adam(int64_t P, float* params, const float* grad, float* m, float* v, float b1, float b2,
                       float lr_t, float eps_t, int type, void* params_t, int64_t per, int64_t per_t, hipStream_t s);
hipError_t launch_cast(int64_t P, const float* params, int type, void* params_t, int64_t per, int64_t per_t,
                       hipStream_t s);

// u[k][i] = 24-bit Philox uniforms in (0, 1) (same counters as the FP64
// generator: key (seed, sid), counter (e0 + i, k / 4, 0, 0)).
hipError_t launch_uniform_f32(uint64_t seed, uint64_t sid, uint64_t e0, int64_t n, int d, float* u, hipStream_t s);

// y_d[k][i] = y[k][i] (FP32 -> FP64 for the mapping chain)
hipError_t launch_widen(int64_t count, const float* y, double* y_d, hipStream_t s);

// w[i] = wfj[i] * exp(logdet[i]); logq[i] = -logdet[i]
hipError_t launch_flow_weight(int64_t n, const double* wfj, const float* logdet, double* w, float* logq,
                              hipStream_t s);

}  // namespace msx
