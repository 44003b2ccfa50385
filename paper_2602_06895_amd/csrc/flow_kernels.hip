// Kernels of the rational-quadratic spline coupling flow on gfx950: the MLP
// conditioner as GEMMs on the matrix cores (BF16 operands with FP32
// accumulation, or FP32 operands), the spline forward / inverse / reverse-mode
// passes in FP32 (one thread per event), the variance loss and Adam.
//
// The spline is the monotone rational-quadratic transformation of Durkan et
// al. (2019) that the paper uses for its neural importance sampler (section
// 2.3, adaptive sampling); its single-bin case is the RQF of the FastRambo
// mapping (section 2.2.9).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>

#include "chain.h"
#include "device_util.h"
#include "flow_launch.h"

namespace msx {

namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float floatx4 __attribute__((ext_vector_type(4)));

// ---------------------------------------------------------------------------
// GEMM on the matrix cores: 64 x 128 output tile per 256-thread workgroup,
// 64-deep K steps through LDS; wave w owns rows 32 (w / 2).., columns
// 64 (w % 2).. as 2 x 4 tiles of 16 x 16.
//   BF16: v_mfma_f32_16x16x32_bf16, lane l holds A[l % 16][8 (l / 16) + 0..7]
//         and B[8 (l / 16) + 0..7][l % 16];
//   FP32: v_mfma_f32_16x16x4_f32,  lane l holds A[l % 16][l / 16], B[l / 16][l % 16];
//   both: lane l receives D[4 (l / 16) + 0..3][l % 16].
// ---------------------------------------------------------------------------
constexpr int BM = 64, BN = 128, BK = 64, GT = 256;

template <class T>
struct Lds;
template <>
struct Lds<__bf16> {
    static constexpr int LDK = BK + 8;  // 144-byte rows keep 16-byte operand reads aligned
};
template <>
struct Lds<float> {
    static constexpr int LDK = BK + 1;  // odd stride: column reads spread over the banks
};

template <class T>
__device__ __forceinline__ T to_t(float v) {
    return (T)v;
}

// Eight consecutive elements from global memory: one or two 16-byte loads
// when the run is in bounds and aligned, element by element otherwise.
template <class T>
__device__ __forceinline__ void load8(const T* __restrict__ src, int valid, T (&v)[8]) {
    if (valid == 8 && (((uintptr_t)src) & 15) == 0) {
        constexpr int W = (int)(8 * sizeof(T) / 16);  // 16-byte words: 1 (BF16) or 2 (FP32)
        uint4 q[W];
#pragma unroll
        for (int i = 0; i < W; ++i) q[i] = ((const uint4*)src)[i];
        __builtin_memcpy(v, q, sizeof v);
        return;
    }
#pragma unroll
    for (int i = 0; i < 8; ++i) v[i] = i < valid ? src[i] : to_t<T>(0.0f);
}

// One ROWS x BK tile of P (rows r0.., k k0..) into S[r][k]; zero outside
// rows < R and k < kend.  Runs of 8 elements along the unit stride.
template <class T, int ROWS>
__device__ __forceinline__ void load_tile(const T* __restrict__ P, int64_t s_r, int64_t s_k, int R, int r0, int k0,
                                          int kend, T (*S)[Lds<T>::LDK], int tid) {
    constexpr int RUNS = ROWS * BK / 8 / GT;
    T v[8];
    if (s_r == 1 && s_k != 1) {
        // runs of 8 consecutive rows at one k, consecutive lanes at
        // consecutive k: each of the 8 transposing LDS stores of a wave then
        // covers all banks (lanes 8 rows apart would hit the same bank with
        // a 16-byte-multiple row pitch)
#pragma unroll
        for (int t = 0; t < RUNS; ++t) {
            const int q = tid + GT * t;
            const int kk = q % BK, rb = (q / BK) * 8;
            const int k = k0 + kk;
            const int valid = k < kend ? max(0, min(8, R - (r0 + rb))) : 0;
            load8<T>(P + (int64_t)(r0 + rb) + (int64_t)k * s_k, valid, v);
#pragma unroll
            for (int i = 0; i < 8; ++i) S[rb + i][kk] = v[i];
        }
    } else {
        // runs of 8 consecutive k of one row
#pragma unroll
        for (int t = 0; t < RUNS; ++t) {
            const int q = tid + GT * t;
            const int rr = q / (BK / 8), kb = (q % (BK / 8)) * 8;
            const int r = r0 + rr;
            if (s_k == 1) {
                const int valid = r < R ? max(0, min(8, kend - (k0 + kb))) : 0;
                load8<T>(P + (int64_t)r * s_r + (k0 + kb), valid, v);
            } else {
#pragma unroll
                for (int i = 0; i < 8; ++i) {
                    const int k = k0 + kb + i;
                    v[i] = (r < R && k < kend) ? P[(int64_t)r * s_r + (int64_t)k * s_k] : to_t<T>(0.0f);
                }
            }
#pragma unroll
            for (int i = 0; i < 8; ++i) S[rr][kb + i] = v[i];
        }
    }
}

__device__ __forceinline__ void mma(const __bf16 (*As)[Lds<__bf16>::LDK], const __bf16 (*Bs)[Lds<__bf16>::LDK], int wm,
                                    int wn, int lane, floatx4 (&acc)[2][4]) {
#pragma unroll
    for (int ks = 0; ks < BK / 32; ++ks) {
        bf16x8 a[2], b[4];
#pragma unroll
        for (int i = 0; i < 2; ++i) a[i] = *(const bf16x8*)&As[wm + i * 16 + (lane & 15)][32 * ks + 8 * (lane >> 4)];
#pragma unroll
        for (int j = 0; j < 4; ++j) b[j] = *(const bf16x8*)&Bs[wn + j * 16 + (lane & 15)][32 * ks + 8 * (lane >> 4)];
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
            for (int j = 0; j < 4; ++j)
                acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[i], b[j], acc[i][j], 0, 0, 0);
    }
}

__device__ __forceinline__ void mma(const float (*As)[Lds<float>::LDK], const float (*Bs)[Lds<float>::LDK], int wm,
                                    int wn, int lane, floatx4 (&acc)[2][4]) {
#pragma unroll
    for (int ks = 0; ks < BK / 4; ++ks) {
        float a[2], b[4];
#pragma unroll
        for (int i = 0; i < 2; ++i) a[i] = As[wm + i * 16 + (lane & 15)][4 * ks + (lane >> 4)];
#pragma unroll
        for (int j = 0; j < 4; ++j) b[j] = Bs[wn + j * 16 + (lane & 15)][4 * ks + (lane >> 4)];
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
            for (int j = 0; j < 4; ++j) acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[i], b[j], acc[i][j], 0, 0, 0);
    }
}

template <class T>
__global__ __launch_bounds__(GT) void k_gemm(GemmArgs g, int kchunk) {
    constexpr int LDK = Lds<T>::LDK;
    __shared__ __attribute__((aligned(16))) T As[BM][LDK];
    __shared__ __attribute__((aligned(16))) T Bs[BN][LDK];
    const T* __restrict__ A = (const T*)g.A;
    const T* __restrict__ B = (const T*)g.B;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int m0 = blockIdx.x * BM, n0 = blockIdx.y * BN;
    const int kbeg = blockIdx.z * kchunk;
    const int kend = min(g.K, kbeg + kchunk);
    const int wm = (wave >> 1) * 32, wn = (wave & 1) * 64;
    floatx4 acc[2][4];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = floatx4{0.0f, 0.0f, 0.0f, 0.0f};
    for (int k0 = kbeg; k0 < kend; k0 += BK) {
        load_tile<T, BM>(A, g.a_m, g.a_k, g.M, m0, k0, kend, As, tid);
        load_tile<T, BN>(B, g.b_n, g.b_k, g.N, n0, k0, kend, Bs, tid);
        __syncthreads();
        mma(As, Bs, wm, wn, lane, acc);
        __syncthreads();
    }
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j)
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int r = m0 + wm + i * 16 + 4 * (lane >> 4) + e;
                const int c = n0 + wn + j * 16 + (lane & 15);
                if (r >= g.M || c >= g.N) continue;
                const float v = acc[i][j][e];
                switch (g.epi) {
                    case EPI_PARTIAL:
                        ((float*)g.out)[((int64_t)blockIdx.z * g.M + r) * g.N + c] = v;
                        break;
                    case EPI_BIAS_RELU:
                        ((T*)g.out)[(int64_t)r * g.ldc + c] = to_t<T>(fmaxf(v + g.bias[c], 0.0f));
                        break;
                    case EPI_BIAS_F32:
                        ((float*)g.out)[(int64_t)r * g.ldc + c] = v + g.bias[c];
                        break;
                    case EPI_RELU_MASK: {
                        const float h = (float)((const T*)g.mask)[(int64_t)r * g.ldm + c];
                        ((T*)g.out)[(int64_t)r * g.ldc + c] = to_t<T>(h > 0.0f ? v : 0.0f);
                        break;
                    }
                    default:
                        ((float*)g.out)[(int64_t)r * g.ldc + c] = v;
                        break;
                }
            }
}

// out[i] = sum over z of part[z][i], i < M N.  A workgroup takes 64
// consecutive i; its four waves sum the partials z = w, w + 4, w + 8, ...
// with four independent accumulators each, then the 16 sums of every i are
// added in a fixed order (deterministic for a given split count).
__global__ __launch_bounds__(256) void k_reduce_partials(const float* __restrict__ part, int splits, int M, int N,
                                                         float* __restrict__ out, int64_t ldo) {
    __shared__ float red[4][64];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int64_t MN = (int64_t)M * N;
    const int64_t i = (int64_t)blockIdx.x * 64 + lane;
    float a0 = 0.0f, a1 = 0.0f, a2 = 0.0f, a3 = 0.0f;
    if (i < MN) {
        int z = w;
        for (; z + 12 < splits; z += 16) {
            a0 += part[(int64_t)z * MN + i];
            a1 += part[(int64_t)(z + 4) * MN + i];
            a2 += part[(int64_t)(z + 8) * MN + i];
            a3 += part[(int64_t)(z + 12) * MN + i];
        }
        for (; z < splits; z += 4) a0 += part[(int64_t)z * MN + i];
    }
    red[w][lane] = (a0 + a1) + (a2 + a3);
    __syncthreads();
    if (w == 0 && i < MN) {
        const float sum = (red[0][lane] + red[1][lane]) + (red[2][lane] + red[3][lane]);
        const int64_t r = i / N, c = i % N;
        out[r * ldo + c] = sum;
    }
}

// Column sums of X [R][N] in row chunks: part[chunk][c].  Threads take
// columns; four independent accumulators over rows r, r + 1, r + 2, r + 3.
template <class T>
__global__ __launch_bounds__(256) void k_colsum(const T* __restrict__ X, int64_t R, int N, int64_t ldx, int64_t chunk,
                                                float* __restrict__ part) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= N) return;
    const int64_t r0 = (int64_t)blockIdx.y * chunk, r1 = min(R, r0 + chunk);
    float s0 = 0.0f, s1 = 0.0f, s2 = 0.0f, s3 = 0.0f;
    int64_t r = r0;
    for (; r + 3 < r1; r += 4) {
        s0 += (float)X[r * ldx + c];
        s1 += (float)X[(r + 1) * ldx + c];
        s2 += (float)X[(r + 2) * ldx + c];
        s3 += (float)X[(r + 3) * ldx + c];
    }
    for (; r < r1; ++r) s0 += (float)X[r * ldx + c];
    part[(int64_t)blockIdx.y * N + c] = (s0 + s1) + (s2 + s3);
}

// Column sums for BF16 X with N and ldx multiples of 8: 16 threads cover 128
// columns of one row with 16-byte loads, the workgroup's 16 row groups take
// rows r0 + g, r0 + g + 16, ...; the 16 partial sums of a column are added
// in a fixed order through LDS.  grid.x: column blocks of 128, grid.y: row
// chunks.
__global__ __launch_bounds__(256) void k_colsum8(const __bf16* __restrict__ X, int64_t R, int N, int64_t ldx,
                                                 int64_t chunk, float* __restrict__ part) {
    __shared__ float red[16][129];
    const int g = threadIdx.x >> 4, cl = (threadIdx.x & 15) * 8;
    const int c0 = blockIdx.x * 128 + cl;
    const int64_t r0 = (int64_t)blockIdx.y * chunk, r1 = min(R, r0 + chunk);
    float acc[8];
#pragma unroll
    for (int i = 0; i < 8; ++i) acc[i] = 0.0f;
    if (c0 < N) {
        for (int64_t r = r0 + g; r < r1; r += 16) {
            const uint4 q = *(const uint4*)(X + r * ldx + c0);
            __bf16 v[8];
            __builtin_memcpy(v, &q, sizeof v);
#pragma unroll
            for (int i = 0; i < 8; ++i) acc[i] += (float)v[i];
        }
    }
#pragma unroll
    for (int i = 0; i < 8; ++i) red[g][cl + i] = acc[i];
    __syncthreads();
    if (threadIdx.x < 128) {
        const int c = blockIdx.x * 128 + threadIdx.x;
        float sum = 0.0f;
#pragma unroll
        for (int k = 0; k < 16; ++k) sum += red[k][threadIdx.x];
        if (c < N) part[(int64_t)blockIdx.y * N + c] = sum;
    }
}

// ---------------------------------------------------------------------------
// Layer plumbing
// ---------------------------------------------------------------------------
struct Idx {
    int32_t v[kFlowMaxHalf];
};

template <class T>
__global__ __launch_bounds__(256) void k_gather(const float* __restrict__ z, int64_t n, int nc, Idx cond,
                                                T* __restrict__ x0) {
    const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= n) return;
    for (int i = 0; i < nc; ++i) x0[b * nc + i] = to_t<T>(z[(int64_t)cond.v[i] * n + b]);
}

__global__ __launch_bounds__(256) void k_scatter_add(float* __restrict__ adj, const float* __restrict__ dx0, int64_t n,
                                                     int nc, Idx cond) {
    const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= n) return;
    for (int i = 0; i < nc; ++i) adj[(int64_t)cond.v[i] * n + b] += dx0[b * nc + i];
}

// ---------------------------------------------------------------------------
// Spline: bin of a value from the 3K + 1 unconstrained parameters.
// Widths / heights: kMin + (1 - K kMin) softmax; knot slopes: kMin +
// softplus(theta + s0) with s0 = log(e^(1 - kMin) - 1) (theta = 0 -> slope 1);
// knots are cumulative sums with the last one exactly 1.
// ---------------------------------------------------------------------------
constexpr float kMinW = 1e-3f, kMinH = 1e-3f, kMinD = 1e-3f;

// softplus(x) = max(x, 0) + log(1 + e^-|x|) through the hardware's exp2 and
// log2 (a few instructions instead of log1pf(expf(x))): absolute error about
// 1e-7, against knot slopes of at least kMinD
__device__ __forceinline__ float softplus_f(float x) {
    return x > 20.0f ? x : fmaxf(x, 0.0f) + __logf(1.0f + __expf(-fabsf(x)));
}
__device__ __forceinline__ float sigmoid_f(float x) {
    return 1.0f / (1.0f + expf(-x));
}
__device__ __forceinline__ float slope_shift() {
    return logf(expm1f(1.0f - kMinD));
}

struct Bin {
    int k;
    float x0, w, y0, h, d0, d1;
    float pw, ph;  // softmax mass of the widths / heights below bin k
};

// BY_Y: locate v among the y knots (inverse) instead of the x knots.
template <bool BY_Y>
__device__ __forceinline__ Bin spline_bin(const float* __restrict__ th, int K, float v, float& mw, float& sw,
                                          float& mh, float& sh) {
    mw = -INFINITY;
    mh = -INFINITY;
    for (int i = 0; i < K; ++i) {
        mw = fmaxf(mw, th[i]);
        mh = fmaxf(mh, th[K + i]);
    }
    sw = 0.0f;
    sh = 0.0f;
    for (int i = 0; i < K; ++i) {
        sw += expf(th[i] - mw);
        sh += expf(th[K + i] - mh);
    }
    const float cw = (1.0f - K * kMinW) / sw, ch = (1.0f - K * kMinH) / sh;
    Bin b{};
    float cx = 0.0f, cy = 0.0f, pw = 0.0f, ph = 0.0f;
    for (int i = 0; i < K; ++i) {
        const float ew = expf(th[i] - mw), eh = expf(th[K + i] - mh);
        const float xl = cx, yl = cy;
        cx = (i == K - 1) ? 1.0f : cx + (kMinW + cw * ew);
        cy = (i == K - 1) ? 1.0f : cy + (kMinH + ch * eh);
        const bool take = (i == 0) || (v >= (BY_Y ? yl : xl));
        if (take) {
            b.k = i;
            b.x0 = xl;
            b.w = cx - xl;
            b.y0 = yl;
            b.h = cy - yl;
            b.pw = pw;
            b.ph = ph;
        }
        pw += ew / sw;
        ph += eh / sh;
    }
    const float s0 = slope_shift();
    b.d0 = kMinD + softplus_f(th[2 * K + b.k] + s0);
    b.d1 = kMinD + softplus_f(th[2 * K + b.k + 1] + s0);
    return b;
}

// spline_bin for a bin count known at compile time: the exponentials are
// evaluated once, with the hardware's exp2 (their sums are normalised, so its
// ulp-level error cancels to first order), and kept in registers.
template <bool BY_Y, int KS>
__device__ __forceinline__ Bin spline_bin_k(const float* __restrict__ th, float v, float (&ew)[KS], float (&eh)[KS],
                                            float& sw, float& sh) {
    float mw = th[0], mh = th[KS];
#pragma unroll
    for (int i = 1; i < KS; ++i) {
        mw = fmaxf(mw, th[i]);
        mh = fmaxf(mh, th[KS + i]);
    }
    sw = 0.0f;
    sh = 0.0f;
#pragma unroll
    for (int i = 0; i < KS; ++i) {
        ew[i] = __expf(th[i] - mw);
        eh[i] = __expf(th[KS + i] - mh);
        sw += ew[i];
        sh += eh[i];
    }
    const float cw = (1.0f - KS * kMinW) / sw, ch = (1.0f - KS * kMinH) / sh;
    Bin b{};
    float cx = 0.0f, cy = 0.0f, pw = 0.0f, ph = 0.0f;
#pragma unroll
    for (int i = 0; i < KS; ++i) {
        const float xl = cx, yl = cy;
        cx = (i == KS - 1) ? 1.0f : cx + (kMinW + cw * ew[i]);
        cy = (i == KS - 1) ? 1.0f : cy + (kMinH + ch * eh[i]);
        const bool take = (i == 0) || (v >= (BY_Y ? yl : xl));
        if (take) {
            b.k = i;
            b.x0 = xl;
            b.w = cx - xl;
            b.y0 = yl;
            b.h = cy - yl;
            b.pw = pw;
            b.ph = ph;
        }
        pw += ew[i] / sw;
        ph += eh[i] / sh;
    }
    const float s0 = slope_shift();
    b.d0 = kMinD + softplus_f(th[2 * KS + b.k] + s0);
    b.d1 = kMinD + softplus_f(th[2 * KS + b.k + 1] + s0);
    return b;
}
template <bool BY_Y, int KS>
__device__ __forceinline__ Bin spline_bin_k(const float* __restrict__ th, float v) {
    float ew[KS], eh[KS], sw, sh;
    return spline_bin_k<BY_Y, KS>(th, v, ew, eh, sw, sh);
}

__device__ __forceinline__ float spline_slope(const Bin& b, float xi) {
    const float s = b.h / b.w;
    const float om = xi * (1.0f - xi);
    const float den = s + (b.d1 + b.d0 - 2.0f * s) * om;
    return s * s * (b.d1 * xi * xi + 2.0f * s * om + b.d0 * (1.0f - xi) * (1.0f - xi)) / (den * den);
}

// The spline kernels take one wave of kSplineT events per workgroup and walk
// the transformed coordinates; for each, the events' 3K + 1 parameters (a
// strided slab of theta) are staged through LDS with coalesced loads (odd row
// length: conflict-free reads).
constexpr int kSplineT = 64;

__device__ __forceinline__ void load_slab(const float* __restrict__ theta, int64_t ldt, int64_t e0, int rows, int j,
                                          int P, float* __restrict__ slab) {
    const int total = rows * P;
    for (int i = threadIdx.x; i < total; i += kSplineT) {
        const int r = i / P, c = i - r * P;
        slab[i] = theta[(e0 + r) * ldt + (int64_t)j * P + c];
    }
}

// One transformed coordinate j = blockIdx.y of kSplineT events per block (the
// coordinates are independent, so the grid carries nh times more waves);
// its log |dy/dx| (or log |dx/dy|) goes to ldp[j][e] and k_ld_add sums them.
template <bool INV>
__global__ __launch_bounds__(kSplineT) void k_spline(float* __restrict__ z, int64_t n, const float* __restrict__ theta,
                                                     int64_t ldt, Idx trans, int K, float* __restrict__ ldp) {
    extern __shared__ float slab[];
    const int64_t e0 = (int64_t)blockIdx.x * kSplineT;
    const int rows = (int)min<int64_t>(kSplineT, n - e0);
    const int P = 3 * K + 1;
    const int64_t e = e0 + threadIdx.x;
    const bool active = threadIdx.x < rows;
    const int j = blockIdx.y;
    {
        load_slab(theta, ldt, e0, rows, j, P, slab);
        __syncthreads();
        if (active) {
            const float* th = slab + threadIdx.x * P;
            float* zp = z + (int64_t)trans.v[j] * n + e;
            const float v = *zp;
            Bin b;
            if (K == 16) {
                b = spline_bin_k<INV, 16>(th, v);
            } else {
                float mw, sw, mh, sh;
                b = spline_bin<INV>(th, K, v, mw, sw, mh, sh);
            }
            const float s = b.h / b.w;
            const float kap = b.d1 + b.d0 - 2.0f * s;
            float xi, out;
            if (!INV) {
                xi = (v - b.x0) / b.w;
                const float om = xi * (1.0f - xi);
                out = b.y0 + b.h * (s * xi * xi + b.d0 * om) / (s + kap * om);
            } else {
                const float dy = v - b.y0;
                const float qa = b.h * (s - b.d0) + dy * kap;
                const float qb = b.h * b.d0 - dy * kap;
                const float qc = -s * dy;
                const float disc = fmaxf(qb * qb - 4.0f * qa * qc, 0.0f);
                xi = 2.0f * qc / (-qb - sqrtf(disc));
                out = b.x0 + xi * b.w;
            }
            const float g = spline_slope(b, xi);
            ldp[(int64_t)j * n + e] = INV ? -logf(g) : logf(g);
            *zp = out;
        }
    }
}

// logdet[e] += sum over j of ldp[j][e], j in order.
__global__ __launch_bounds__(256) void k_ld_add(const float* __restrict__ ldp, int64_t n, int nh,
                                                float* __restrict__ logdet) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n) return;
    float ld = 0.0f;
    for (int j = 0; j < nh; ++j) ld += ldp[(int64_t)j * n + e];
    logdet[e] += ld;
}

// Forward-mode dual numbers with 7 tangents: (y, x0, w, y0, h, d0, d1).
struct D7 {
    float v;
    float g[7];
};
__device__ __forceinline__ D7 dconst(float v) {
    D7 r;
    r.v = v;
#pragma unroll
    for (int i = 0; i < 7; ++i) r.g[i] = 0.0f;
    return r;
}
__device__ __forceinline__ D7 dvar(float v, int i) {
    D7 r = dconst(v);
    r.g[i] = 1.0f;
    return r;
}
__device__ __forceinline__ D7 operator+(const D7& a, const D7& b) {
    D7 r;
    r.v = a.v + b.v;
#pragma unroll
    for (int i = 0; i < 7; ++i) r.g[i] = a.g[i] + b.g[i];
    return r;
}
__device__ __forceinline__ D7 operator-(const D7& a, const D7& b) {
    D7 r;
    r.v = a.v - b.v;
#pragma unroll
    for (int i = 0; i < 7; ++i) r.g[i] = a.g[i] - b.g[i];
    return r;
}
__device__ __forceinline__ D7 operator*(const D7& a, const D7& b) {
    D7 r;
    r.v = a.v * b.v;
#pragma unroll
    for (int i = 0; i < 7; ++i) r.g[i] = a.g[i] * b.v + a.v * b.g[i];
    return r;
}
__device__ __forceinline__ D7 operator*(float a, const D7& b) {
    D7 r;
    r.v = a * b.v;
#pragma unroll
    for (int i = 0; i < 7; ++i) r.g[i] = a * b.g[i];
    return r;
}
__device__ __forceinline__ D7 operator/(const D7& a, const D7& b) {
    D7 r;
    const float ib = 1.0f / b.v;
    r.v = a.v * ib;
#pragma unroll
    for (int i = 0; i < 7; ++i) r.g[i] = (a.g[i] - r.v * b.g[i]) * ib;
    return r;
}
__device__ __forceinline__ D7 dsqrt(const D7& a) {
    D7 r;
    r.v = sqrtf(a.v);
    const float c = 0.5f / r.v;
#pragma unroll
    for (int i = 0; i < 7; ++i) r.g[i] = a.g[i] * c;
    return r;
}
__device__ __forceinline__ D7 dlog(const D7& a) {
    D7 r;
    r.v = logf(a.v);
    const float c = 1.0f / a.v;
#pragma unroll
    for (int i = 0; i < 7; ++i) r.g[i] = a.g[i] * c;
    return r;
}

// Reverse mode through the inverse spline of one layer (see flow_launch.h).
// The parameter slab comes in through LDS and the parameter gradients go out
// through a second LDS slab with coalesced stores.
// Reverse mode of the inverse spline of one (event, coordinate): gradient
// of G ld + adj x with respect to y (into adj) and the layer's 3K + 1
// unconstrained parameters (into dth).  KS > 0: the bin count is KS and the
// bin exponentials are computed once (the same values as the general path).
// th and dth may be the same row: each element is read before it is written.
template <int KS>
__device__ __forceinline__ void spline_backward_one(const float* th, int K, float v, float ge, float& ax, float* dth) {
    constexpr int KX = KS > 0 ? KS : 1;
    float ewk[KX], ehk[KX];
    float mw = 0.0f, sw, mh = 0.0f, sh;
    Bin bn;
    if (KS > 0) {
        bn = spline_bin_k<true, KX>(th, v, ewk, ehk, sw, sh);
    } else {
        bn = spline_bin<true>(th, K, v, mw, sw, mh, sh);
    }
    auto pw_of = [&](int i) -> float { return KS > 0 ? ewk[i] / sw : expf(th[i] - mw) / sw; };
    auto ph_of = [&](int i) -> float { return KS > 0 ? ehk[i] / sh : expf(th[K + i] - mh) / sh; };
    // x = S^-1(y) and ld = log (S^-1)'(y) = -log S'(x) as duals
    const D7 Y = dvar(v, 0), X0 = dvar(bn.x0, 1), W = dvar(bn.w, 2), Y0 = dvar(bn.y0, 3), H = dvar(bn.h, 4),
             Dd0 = dvar(bn.d0, 5), Dd1 = dvar(bn.d1, 6);
    const D7 s = H / W;
    const D7 dy = Y - Y0;
    const D7 kap = Dd1 + Dd0 - 2.0f * s;
    const D7 qa = H * (s - Dd0) + dy * kap;
    const D7 qb = H * Dd0 - dy * kap;
    const D7 qc = dconst(0.0f) - s * dy;
    D7 disc = qb * qb - 4.0f * (qa * qc);
    disc.v = fmaxf(disc.v, 1e-30f);
    const D7 xi = (2.0f * qc) / (dconst(0.0f) - qb - dsqrt(disc));
    const D7 X = X0 + xi * W;
    const D7 om = xi * (dconst(1.0f) - xi);
    const D7 den = s + kap * om;
    const D7 omx = dconst(1.0f) - xi;
    const D7 num = s * s * (Dd1 * xi * xi + 2.0f * (s * om) + Dd0 * omx * omx);
    const D7 ld = 2.0f * dlog(den) - dlog(num);
    float gp[7];
#pragma unroll
    for (int i = 0; i < 7; ++i) gp[i] = ax * X.g[i] + ge * ld.g[i];
    ax = gp[0];
    // to the unconstrained parameters: softmax of widths / heights, softplus of slopes
    const float Cw = 1.0f - K * kMinW, Ch = 1.0f - K * kMinH;
    float pwk = 0.0f, phk = 0.0f;
    if (KS > 0) {
#pragma unroll
        for (int i = 0; i < KX; ++i)
            if (i == bn.k) {
                pwk = pw_of(i);
                phk = ph_of(i);
            }
    } else {
        pwk = pw_of(bn.k);
        phk = ph_of(bn.k);
    }
    const float sumw = gp[1] * bn.pw + gp[2] * pwk;
    const float sumh = gp[3] * bn.ph + gp[4] * phk;
#pragma unroll
    for (int i = 0; i < (KS > 0 ? KS : K); ++i) {
        const float pwi = pw_of(i), phi = ph_of(i);
        const float dwi = (i < bn.k ? gp[1] : 0.0f) + (i == bn.k ? gp[2] : 0.0f);
        const float dhi = (i < bn.k ? gp[3] : 0.0f) + (i == bn.k ? gp[4] : 0.0f);
        dth[i] = Cw * pwi * (dwi - sumw);
        dth[K + i] = Ch * phi * (dhi - sumh);
    }
    const float s0 = slope_shift();
#pragma unroll
    for (int i = 0; i <= (KS > 0 ? KS : K); ++i) {
        const float dd = (i == bn.k ? gp[5] : 0.0f) + (i == bn.k + 1 ? gp[6] : 0.0f);
        dth[2 * K + i] = dd * sigmoid_f(th[2 * K + i] + s0);
    }
}

template <class T>
__global__ __launch_bounds__(kSplineT) void k_spline_backward(const float* __restrict__ y, float* __restrict__ adj,
                                                              int64_t n, const float* __restrict__ theta, int64_t ldt,
                                                              Idx trans, int K, const float* __restrict__ G,
                                                              T* __restrict__ dtheta) {
    extern __shared__ float slab[];
    const int P = 3 * K + 1;
    // d theta overwrites theta in the thread's own row: every parameter is
    // read before the element of the same index is written
    float* dslab = slab;
    const int64_t e0 = (int64_t)blockIdx.x * kSplineT;
    const int rows = (int)min<int64_t>(kSplineT, n - e0);
    const int64_t e = e0 + threadIdx.x;
    const bool active = threadIdx.x < rows;
    const int j = blockIdx.y;  // one transformed coordinate per block row of the grid
    load_slab(theta, ldt, e0, rows, j, P, slab);
    __syncthreads();
    if (active) {
        const int64_t zi = (int64_t)trans.v[j] * n + e;
        float ax = adj[zi];
        if (K == 16)
            spline_backward_one<16>(slab + threadIdx.x * P, K, y[zi], G[e], ax, dslab + threadIdx.x * P);
        else
            spline_backward_one<0>(slab + threadIdx.x * P, K, y[zi], G[e], ax, dslab + threadIdx.x * P);
        adj[zi] = ax;
    }
    __syncthreads();
    const int total = rows * P;
    for (int i = threadIdx.x; i < total; i += kSplineT) {
        const int r = i / P, c = i - r * P;
        dtheta[(e0 + r) * ldt + (int64_t)j * P + c] = to_t<T>(dslab[i]);
    }
}

// ---------------------------------------------------------------------------
// Loss, optimiser, conversions
// ---------------------------------------------------------------------------
constexpr int kLossBlocks = 1024;

__global__ __launch_bounds__(256) void k_flow_loss(int64_t n, const double* __restrict__ wfj,
                                                   const float* __restrict__ logq, const float* __restrict__ lqo,
                                                   float* __restrict__ G, double* __restrict__ part) {
    __shared__ double red[4];
    double acc = 0.0;
    const double inv_n = 1.0 / (double)n;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x) {
        const double f = wfj[e];
        const double t = f * f * exp(-(double)logq[e] - (double)lqo[e]);
        acc += t;
        G[e] = (float)(-t * inv_n);
    }
    const double s = wave_sum(acc);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) part[blockIdx.x] = ((red[0] + red[1]) + red[2]) + red[3];
}

__global__ __launch_bounds__(256) void k_loss_final(const double* __restrict__ part, int nb, double inv_n,
                                                    double* __restrict__ loss) {
    __shared__ double red[4];
    double a = 0.0;
    for (int i = threadIdx.x; i < nb; i += blockDim.x) a += part[i];
    const double s = wave_sum(a);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) loss[0] = (((red[0] + red[1]) + red[2]) + red[3]) * inv_n;
}

// G[e] /= loss: the gradient of log L instead of L
__global__ __launch_bounds__(256) void k_scale_by_loss(int64_t n, const double* __restrict__ loss,
                                                       float* __restrict__ G) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) G[i] = (float)((double)G[i] / loss[0]);
}

// The operand copy pads every layer block to a multiple of 8 elements
// (16-byte aligned fragments): master element i = layer * per + j sits at
// layer * per_t + j.
__device__ __forceinline__ int64_t padded_index(int64_t i, int64_t per, int64_t per_t) {
    const int64_t l = i / per;
    return l * per_t + (i - l * per);
}

template <class T>
__global__ __launch_bounds__(256) void k_adam(int64_t P, float* __restrict__ p, const float* __restrict__ g,
                                              float* __restrict__ m, float* __restrict__ v, float b1, float b2,
                                              float lr_t, float eps_t, T* __restrict__ pt, int64_t per,
                                              int64_t per_t) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= P) return;
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.0f - b1) * gi;
    const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    const float q = p[i] - lr_t * mi / (sqrtf(vi) + eps_t);
    p[i] = q;
    pt[padded_index(i, per, per_t)] = to_t<T>(q);
}

template <class T>
__global__ __launch_bounds__(256) void k_cast(int64_t P, const float* __restrict__ p, T* __restrict__ pt, int64_t per,
                                              int64_t per_t) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < P) pt[padded_index(i, per, per_t)] = to_t<T>(p[i]);
}

__global__ __launch_bounds__(256) void k_uniform_f32(uint64_t seed, uint64_t sid, uint64_t e0, int64_t n, int d,
                                                     float* __restrict__ u) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const uint64_t e = e0 + (uint64_t)i;
    for (int g = 0; g < (d + 3) / 4; ++g) {
        uint64_t c0 = e, c1 = (uint64_t)g, c2 = 0, c3 = 0;
        philox4x64_10(c0, c1, c2, c3, seed, sid);
        const uint64_t wv[4] = {c0, c1, c2, c3};
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int k = 4 * g + j;
            if (k < d) u[(int64_t)k * n + i] = ((float)(wv[j] >> 40) + 0.5f) * 0x1.0p-24f;
        }
    }
}

__global__ __launch_bounds__(256) void k_widen(int64_t count, const float* __restrict__ y, double* __restrict__ yd) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= count) return;
    // keep the mapped point inside the open unit cube
    yd[i] = (double)fminf(fmaxf(y[i], 0x1.0p-26f), 1.0f - 0x1.0p-24f);
}

__global__ __launch_bounds__(256) void k_flow_weight(int64_t n, const double* __restrict__ wfj,
                                                     const float* __restrict__ logdet, double* __restrict__ w,
                                                     float* __restrict__ logq) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float ld = logdet[i];
    w[i] = wfj[i] * exp((double)ld);
    if (logq) logq[i] = -ld;
}

// ---------------------------------------------------------------------------
// Fused forward coupling layer (BF16 conditioner of hidden width 128).  Each
// wave takes 64 events.  Their conditioning coordinates are gathered straight
// into MFMA operand fragments; the hidden layers run on the matrix cores with
// the weight fragments read from L2 (about 2 KB per event and layer) and the
// activations passed through a per-wave LDS tile, which also turns the MFMA
// output layout (4 rows of one column per lane) into the operand layout (8 k
// of one row per lane).  The last layer produces the 3K + 1 spline
// parameters of one transformed coordinate at a time into LDS, where each of
// the 64 lanes evaluates the spline of its own event.  Per event only z and
// the log-determinant touch HBM.
// ---------------------------------------------------------------------------
constexpr int kFH = 128;                 // hidden width of the fused path
constexpr int kFW = 2;                   // waves per workgroup
constexpr int kFRow = kFH + 8;           // LDS row of an activation tile (bf16)
constexpr int kFStage = 64 * kFRow;      // bf16 elements per wave (>= 64 x 49 floats)

struct FusedW {
    const __bf16* w1;  // [128][nh]
    const __bf16* w2;  // [128][128]
    const __bf16* w3;  // [128][128]
    const __bf16* w4;  // [n_out][128]
    const float* b1;
    const float* b2;
    const float* b3;
    const float* b4;
};

// acc (16 events x 16 columns per tile t) + bias, ReLU, BF16 -> activation tile
__device__ __forceinline__ void hidden_epilogue(const floatx4 (&acc)[4], const float* __restrict__ b, int c, int lane,
                                                __bf16* __restrict__ st) {
    const int r16 = lane & 15, kq = lane >> 4;
    const float bias = b[16 * c + r16];
#pragma unroll
    for (int t = 0; t < 4; ++t)
#pragma unroll
        for (int e = 0; e < 4; ++e)
            st[(16 * t + 4 * kq + e) * kFRow + 16 * c + r16] = (__bf16)fmaxf(acc[t][e] + bias, 0.0f);
}

// 128 -> 128 layer from the activation tile in LDS back into it
__device__ __forceinline__ void hidden_layer(const __bf16* __restrict__ Wl, const float* __restrict__ bl, int lane,
                                             __bf16* __restrict__ st) {
    const int r16 = lane & 15, kq = lane >> 4;
    bf16x8 a[4][4];
#pragma unroll
    for (int t = 0; t < 4; ++t)
#pragma unroll
        for (int s4 = 0; s4 < 4; ++s4) a[t][s4] = *(const bf16x8*)&st[(16 * t + r16) * kFRow + 32 * s4 + 8 * kq];
    __syncthreads();  // the tile is overwritten below
    // weight fragments of the next column tile are in flight while this
    // tile's MFMAs run
    bf16x8 bn[4];
#pragma unroll
    for (int s4 = 0; s4 < 4; ++s4) bn[s4] = *(const bf16x8*)&Wl[r16 * kFH + 32 * s4 + 8 * kq];
#pragma unroll 2
    for (int c = 0; c < kFH / 16; ++c) {
        bf16x8 b[4];
#pragma unroll
        for (int s4 = 0; s4 < 4; ++s4) b[s4] = bn[s4];
        if (c + 1 < kFH / 16) {
#pragma unroll
            for (int s4 = 0; s4 < 4; ++s4)
                bn[s4] = *(const bf16x8*)&Wl[(16 * (c + 1) + r16) * kFH + 32 * s4 + 8 * kq];
        }
        floatx4 acc[4];
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            acc[t] = floatx4{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
            for (int s4 = 0; s4 < 4; ++s4) acc[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[t][s4], b[s4], acc[t], 0, 0, 0);
        }
        hidden_epilogue(acc, bl, c, lane, st);
    }
    __syncthreads();
}

// What the reverse pass of training reads, written by the fused inverse
// layer when the pointers are set: the BF16 conditioning inputs x0 [n][nh],
// the hidden activations h [3][n][128] and the spline parameters theta
// [n][n_out] (FP32), the same values the unfused path stores.
struct FusedSave {
    __bf16* x0;
    __bf16* h;
    float* theta;
};

// Copy a wave's 64 x 128 activation tile to h[e0 ..][128] (16-byte stores).
__device__ __forceinline__ void save_tile(const __bf16* __restrict__ st, __bf16* __restrict__ h, int64_t e0,
                                          int64_t n, int lane) {
#pragma unroll
    for (int it = 0; it < 16; ++it) {
        const int idx = it * 64 + lane;        // 16-byte chunk: row idx / 16, column block idx % 16
        const int r = idx >> 4, cb = (idx & 15) * 8;
        if (e0 + r < n) *(uint4*)&h[(e0 + r) * kFH + cb] = *(const uint4*)&st[r * kFRow + cb];
    }
}

template <bool INV, bool SAVE>
__global__ __launch_bounds__(64 * kFW) void k_flow_layer(float* __restrict__ z, int64_t n, FusedW fw, int nh,
                                                         Idx trans, Idx cond, int K, float* __restrict__ logdet,
                                                         FusedSave sv) {
    extern __shared__ __attribute__((aligned(16))) unsigned char fsm[];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int r16 = lane & 15, kq = lane >> 4;
    __bf16* st = (__bf16*)fsm + (size_t)wave * kFStage;
    float* th = (float*)st;
    const int64_t e0 = ((int64_t)blockIdx.x * kFW + wave) * 64;
    const int P = 3 * K + 1;
    const int n_out = nh * P;

    // layer 1: A fragments = BF16 conditioning coordinates (k = 8 kq + i < nh)
    bf16x8 a1[4];
#pragma unroll
    for (int i = 0; i < 8; ++i) {
        const int k = 8 * kq + i;
        const int ci = kq == 0 ? cond.v[i] : (kq == 1 ? cond.v[8 + i] : (kq == 2 ? cond.v[16 + i] : cond.v[24 + i]));
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            const int64_t e = e0 + 16 * t + r16;
            a1[t][i] = (__bf16)((k < nh && e < n) ? z[(int64_t)ci * n + e] : 0.0f);
            if (SAVE && k < nh && e < n) sv.x0[e * nh + k] = a1[t][i];
        }
    }
#pragma unroll 2
    for (int c = 0; c < kFH / 16; ++c) {
        bf16x8 b;
#pragma unroll
        for (int i = 0; i < 8; ++i) {
            const int k = 8 * kq + i;
            b[i] = k < nh ? fw.w1[(16 * c + r16) * nh + k] : (__bf16)0.0f;
        }
        floatx4 acc[4];
#pragma unroll
        for (int t = 0; t < 4; ++t)
            acc[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a1[t], b, floatx4{0.0f, 0.0f, 0.0f, 0.0f}, 0, 0, 0);
        hidden_epilogue(acc, fw.b1, c, lane, st);
    }
    __syncthreads();
    if (SAVE) save_tile(st, sv.h, e0, n, lane);
    hidden_layer(fw.w2, fw.b2, lane, st);
    if (SAVE) save_tile(st, sv.h + n * kFH, e0, n, lane);
    hidden_layer(fw.w3, fw.b3, lane, st);
    if (SAVE) save_tile(st, sv.h + 2 * n * kFH, e0, n, lane);

    // last layer, one transformed coordinate at a time, then its spline
    bf16x8 a3[4][4];
#pragma unroll
    for (int t = 0; t < 4; ++t)
#pragma unroll
        for (int s4 = 0; s4 < 4; ++s4) a3[t][s4] = *(const bf16x8*)&st[(16 * t + r16) * kFRow + 32 * s4 + 8 * kq];
    __syncthreads();
    const int64_t e = e0 + lane;
    const bool active = e < n;
    float ld = 0.0f;
    for (int j = 0; j < nh; ++j) {
#pragma unroll 2
        for (int c = 0; c < (P + 15) / 16; ++c) {
            const int q = 16 * c + r16;          // parameter within the coordinate
            const int row = j * P + q;           // row of W4 / column of theta
            const bool ok = q < P && row < n_out;
            bf16x8 b[4];
#pragma unroll
            for (int s4 = 0; s4 < 4; ++s4) {
                if (ok) {
                    b[s4] = *(const bf16x8*)&fw.w4[(int64_t)row * kFH + 32 * s4 + 8 * kq];
                } else {
#pragma unroll
                    for (int i = 0; i < 8; ++i) b[s4][i] = (__bf16)0.0f;
                }
            }
            const float bias = ok ? fw.b4[row] : 0.0f;
#pragma unroll
            for (int t = 0; t < 4; ++t) {
                floatx4 acc = floatx4{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
                for (int s4 = 0; s4 < 4; ++s4) acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a3[t][s4], b[s4], acc, 0, 0, 0);
                if (ok) {
#pragma unroll
                    for (int x = 0; x < 4; ++x) {
                        const int r = 16 * t + 4 * kq + x;
                        th[r * P + q] = acc[x] + bias;
                        if (SAVE && e0 + r < n) sv.theta[(e0 + r) * n_out + row] = acc[x] + bias;
                    }
                }
            }
        }
        __syncthreads();
        if (active) {
            float* zp = z + (int64_t)trans.v[j] * n + e;
            const float v = *zp;
            Bin bn;
            if (K == 16) {
                bn = spline_bin_k<INV, 16>(th + lane * P, v);
            } else {
                float mw, sw, mh, sh;
                bn = spline_bin<INV>(th + lane * P, K, v, mw, sw, mh, sh);
            }
            const float sl = bn.h / bn.w;
            const float kap = bn.d1 + bn.d0 - 2.0f * sl;
            if (!INV) {
                const float xi = (v - bn.x0) / bn.w;
                const float om = xi * (1.0f - xi);
                *zp = bn.y0 + bn.h * (sl * xi * xi + bn.d0 * om) / (sl + kap * om);
                ld += logf(spline_slope(bn, xi));
            } else {
                // the same root as the unfused inverse spline
                const float dy = v - bn.y0;
                const float qa = bn.h * (sl - bn.d0) + dy * kap;
                const float qb = bn.h * bn.d0 - dy * kap;
                const float qc = -sl * dy;
                const float disc = fmaxf(qb * qb - 4.0f * qa * qc, 0.0f);
                const float xi = 2.0f * qc / (-qb - sqrtf(disc));
                *zp = bn.x0 + xi * bn.w;
                ld += -logf(spline_slope(bn, xi));
            }
        }
        __syncthreads();
    }
    if (active) logdet[e] += ld;
}

unsigned blocks(int64_t n) {
    return (unsigned)std::max<int64_t>(1, (n + 255) / 256);
}

Idx make_idx(const int32_t* h, int count) {
    Idx r{};
    for (int i = 0; i < count && i < kFlowMaxHalf; ++i) r.v[i] = h[i];
    return r;
}

}  // namespace

// ---------------------------------------------------------------------------
// Launchers
// ---------------------------------------------------------------------------
hipError_t launch_gemm(const GemmArgs& g, hipStream_t s) {
    if (g.M <= 0 || g.N <= 0) return hipSuccess;
    const int splits = std::max(1, g.splits);
    int kchunk = (g.K + splits - 1) / splits;
    kchunk = ((kchunk + BK - 1) / BK) * BK;
    dim3 grid((unsigned)((g.M + BM - 1) / BM), (unsigned)((g.N + BN - 1) / BN), (unsigned)splits);
    if (g.type == FT_BF16)
        k_gemm<__bf16><<<grid, GT, 0, s>>>(g, kchunk);
    else
        k_gemm<float><<<grid, GT, 0, s>>>(g, kchunk);
    return hipGetLastError();
}

hipError_t launch_flow_layer(bool inverse, float* z, int64_t n, const void* params_t, const float* params,
                             const int64_t* off, int nh, const int32_t* trans_host, const int32_t* cond_host, int K,
                             float* logdet, void* save_x0, void* save_h, float* save_theta, hipStream_t s) {
    if (n == 0) return hipSuccess;
    FusedW fw;
    const __bf16* W = (const __bf16*)params_t;
    fw.w1 = W + off[0];
    fw.b1 = params + off[1];
    fw.w2 = W + off[2];
    fw.b2 = params + off[3];
    fw.w3 = W + off[4];
    fw.b3 = params + off[5];
    fw.w4 = W + off[6];
    fw.b4 = params + off[7];
    const unsigned nb = (unsigned)((n + 64 * kFW - 1) / (64 * kFW));
    const size_t lds = sizeof(__bf16) * kFStage * kFW;
    FusedSave sv{(__bf16*)save_x0, (__bf16*)save_h, save_theta};
    const bool save = save_x0 && save_h && save_theta;
    const Idx ti = make_idx(trans_host, nh), ci = make_idx(cond_host, nh);
    if (inverse && save)
        k_flow_layer<true, true><<<nb, 64 * kFW, lds, s>>>(z, n, fw, nh, ti, ci, K, logdet, sv);
    else if (inverse)
        k_flow_layer<true, false><<<nb, 64 * kFW, lds, s>>>(z, n, fw, nh, ti, ci, K, logdet, sv);
    else if (save)
        k_flow_layer<false, true><<<nb, 64 * kFW, lds, s>>>(z, n, fw, nh, ti, ci, K, logdet, sv);
    else
        k_flow_layer<false, false><<<nb, 64 * kFW, lds, s>>>(z, n, fw, nh, ti, ci, K, logdet, sv);
    return hipGetLastError();
}

hipError_t launch_reduce_partials(const float* part, int splits, int M, int N, float* out, int64_t ldo,
                                  hipStream_t s) {
    const int64_t MN = (int64_t)M * N;
    if (MN == 0) return hipSuccess;
    k_reduce_partials<<<(unsigned)((MN + 63) / 64), 256, 0, s>>>(part, splits, M, N, out, ldo);
    return hipGetLastError();
}

hipError_t launch_colsum(int type, const void* X, int64_t R, int N, int64_t ldx, float* part, int nchunk, float* out,
                         hipStream_t s) {
    const int64_t chunk = (R + nchunk - 1) / nchunk;
    dim3 grid((unsigned)((N + 255) / 256), (unsigned)nchunk);
    if (type == FT_BF16 && N % 8 == 0 && ldx % 8 == 0 && ((uintptr_t)X & 15) == 0)
        k_colsum8<<<dim3((unsigned)((N + 127) / 128), (unsigned)nchunk), 256, 0, s>>>((const __bf16*)X, R, N, ldx,
                                                                                      chunk, part);
    else if (type == FT_BF16)
        k_colsum<__bf16><<<grid, 256, 0, s>>>((const __bf16*)X, R, N, ldx, chunk, part);
    else
        k_colsum<float><<<grid, 256, 0, s>>>((const float*)X, R, N, ldx, chunk, part);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    return launch_reduce_partials(part, nchunk, 1, N, out, N, s);
}

hipError_t launch_gather(int type, const float* z, int64_t n, int n_cond, const int32_t* cond_host, void* x0,
                         hipStream_t s) {
    if (n == 0) return hipSuccess;
    Idx c = make_idx(cond_host, n_cond);
    if (type == FT_BF16)
        k_gather<__bf16><<<blocks(n), 256, 0, s>>>(z, n, n_cond, c, (__bf16*)x0);
    else
        k_gather<float><<<blocks(n), 256, 0, s>>>(z, n, n_cond, c, (float*)x0);
    return hipGetLastError();
}

hipError_t launch_spline(bool inverse, float* z, int64_t n, const float* theta, int64_t ldt, int n_half,
                         const int32_t* trans_host, int K, float* logdet, float* ld_part, hipStream_t s) {
    if (n == 0) return hipSuccess;
    Idx t = make_idx(trans_host, n_half);
    const dim3 grid((unsigned)((n + kSplineT - 1) / kSplineT), (unsigned)n_half);
    const size_t lds = sizeof(float) * kSplineT * (3 * K + 1);
    if (inverse)
        k_spline<true><<<grid, kSplineT, lds, s>>>(z, n, theta, ldt, t, K, ld_part);
    else
        k_spline<false><<<grid, kSplineT, lds, s>>>(z, n, theta, ldt, t, K, ld_part);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    k_ld_add<<<blocks(n), 256, 0, s>>>(ld_part, n, n_half, logdet);
    return hipGetLastError();
}

hipError_t launch_spline_backward(int type, const float* y, float* adj, int64_t n, const float* theta, int64_t ldt,
                                  int n_half, const int32_t* trans_host, int K, const float* G, void* dtheta,
                                  hipStream_t s) {
    if (n == 0) return hipSuccess;
    Idx t = make_idx(trans_host, n_half);
    const dim3 nb((unsigned)((n + kSplineT - 1) / kSplineT), (unsigned)n_half);
    const size_t lds = sizeof(float) * kSplineT * (3 * K + 1);
    if (type == FT_BF16)
        k_spline_backward<__bf16><<<nb, kSplineT, lds, s>>>(y, adj, n, theta, ldt, t, K, G, (__bf16*)dtheta);
    else
        k_spline_backward<float><<<nb, kSplineT, lds, s>>>(y, adj, n, theta, ldt, t, K, G, (float*)dtheta);
    return hipGetLastError();
}

hipError_t launch_scatter_add(float* adj, const float* dx0, int64_t n, int n_cond, const int32_t* cond_host,
                              hipStream_t s) {
    if (n == 0) return hipSuccess;
    k_scatter_add<<<blocks(n), 256, 0, s>>>(adj, dx0, n, n_cond, make_idx(cond_host, n_cond));
    return hipGetLastError();
}

hipError_t launch_flow_loss(int64_t n, const double* wfj, const float* logq, const float* logq_old, float* G,
                            double* part, double* loss, bool log_loss, hipStream_t s) {
    if (n == 0) return hipSuccess;
    k_flow_loss<<<kLossBlocks, 256, 0, s>>>(n, wfj, logq, logq_old, G, part);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    k_loss_final<<<1, 256, 0, s>>>(part, kLossBlocks, 1.0 / (double)n, loss);
    e = hipGetLastError();
    if (e != hipSuccess || !log_loss) return e;
    k_scale_by_loss<<<blocks(n), 256, 0, s>>>(n, loss, G);
    return hipGetLastError();
}

hipError_t launch_adam(int64_t P, float* params, const float* grad, float* m, float* v, float b1, float b2,
                       float lr_t, float eps_t, int type, void* params_t, int64_t per, int64_t per_t, hipStream_t s) {
    if (type == FT_BF16)
        k_adam<__bf16><<<blocks(P), 256, 0, s>>>(P, params, grad, m, v, b1, b2, lr_t, eps_t, (__bf16*)params_t, per,
                                                  per_t);
    else
        k_adam<float><<<blocks(P), 256, 0, s>>>(P, params, grad, m, v, b1, b2, lr_t, eps_t, (float*)params_t, per,
                                                 per_t);
    return hipGetLastError();
}

hipError_t launch_cast(int64_t P, const float* params, int type, void* params_t, int64_t per, int64_t per_t,
                       hipStream_t s) {
    if (type == FT_BF16)
        k_cast<__bf16><<<blocks(P), 256, 0, s>>>(P, params, (__bf16*)params_t, per, per_t);
    else
        k_cast<float><<<blocks(P), 256, 0, s>>>(P, params, (float*)params_t, per, per_t);
    return hipGetLastError();
}

hipError_t launch_uniform_f32(uint64_t seed, uint64_t sid, uint64_t e0, int64_t n, int d, float* u, hipStream_t s) {
    if (n == 0) return hipSuccess;
    k_uniform_f32<<<blocks(n), 256, 0, s>>>(seed, sid, e0, n, d, u);
    return hipGetLastError();
}

hipError_t launch_widen(int64_t count, const float* y, double* y_d, hipStream_t s) {
    if (count == 0) return hipSuccess;
    k_widen<<<blocks(count), 256, 0, s>>>(count, y, y_d);
    return hipGetLastError();
}

hipError_t launch_flow_weight(int64_t n, const double* wfj, const float* logdet, double* w, float* logq,
                              hipStream_t s) {
    if (n == 0) return hipSuccess;
    k_flow_weight<<<blocks(n), 256, 0, s>>>(n, wfj, logdet, w, logq);
    return hipGetLastError();
}

}  // namespace msx
